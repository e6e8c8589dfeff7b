"""GPU parity of the TRANSLATED kernel (ROM code translated to HIP at run time) against the oracle."""
import numpy as np
import pytest

from paper_2606_22447_amd import inputs as I
from tests.test_gpu_hard import gpu_run, oracle_env, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("G,tpb", [(16, 256), (4, 64), (32, 256)])
def test_translated_c1_slice_every_byte_across_calls(G, tpb):
    w = I.config_c1(num_envs=96, steps=12)
    say("translated c1 slice", G, tpb)
    ram, fr, done, vb = gpu_run(w, "translated", G, tpb, splits=(5, 6))
    say("translation", vb.translation)
    assert vb.translation["positions"] > 100
    for b in range(w.num_envs):
        ref = oracle_env(w, b)
        assert (ram[b] == ref["ram"]).all(), b
        assert (fr[b] == ref["frames"]).all(), b
    regs = vb.regs().cpu().numpy()
    for b in (0, 17, 95):
        r = oracle_env(w, b)["regs"]
        assert regs[b, :8].tolist() == [r[k] for k in ("A", "X", "Y", "S", "P", "PCL", "PCH", "bank")]


def test_translated_heterogeneous_roms_with_episode_resets():
    # 2K / 4K / F8 images that read SWCHA, INPT4 and INTIM; short episodes force in-run resets
    roms = [I.generate_rom(100 + i, sz, reads_inputs=True, timer_vblank=True)
            for i, sz in enumerate([2048, 4096, 8192, 8192, 2048, 4096])]
    B, S = 70, 10
    env_rom = (np.arange(B) * 7 % len(roms)).astype(np.int32)
    eps = (1 + (np.arange(B)[:, None] * 3 + np.arange(5)[None, :]) % 4).astype(np.uint32)
    w = I.Workload("hetero_test", roms, env_rom, I.initial_ram(9, B), I.action_stream(9, B, S), S, 4,
                   episode_steps=eps, seed=4242)
    say("translated hetero")
    ram, fr, done, vb = gpu_run(w, "translated", 4, 256, splits=(3,))
    say("translation", vb.translation)
    for b in range(B):
        ref = oracle_env(w, b)
        assert (done[b] == ref["done"]).all(), b
        assert (ram[b] == ref["ram"]).all(), b
        assert (fr[b] == ref["frames"]).all(), b


@pytest.mark.parametrize("prog", ["tia_pushes", "playfield_modes"])
@pytest.mark.parametrize("G,tpb", [(16, 256), (32, 64), (64, 256)])
def test_translated_hand_assembled_tia_programs(prog, G, tpb):
    # JSR pushes onto CTRLPF and COLUBK (two pixel-register writes at one clock, at
    # every pixel alignment), and CTRLPF cycled through reflected and score modes:
    # drawn by rows shared over the env's lanes
    from tests import test_translated_cpu as T
    w = {"tia_pushes": T.tia_pushes_workload, "playfield_modes": T.playfield_modes_workload}[prog](B=40, S=4)
    say("translated", prog, G, tpb)
    ram, fr, _, vb = gpu_run(w, "translated", G, tpb)
    for b in range(w.num_envs):
        ref = oracle_env(w, b)
        assert (ram[b] == ref["ram"]).all() and (fr[b] == ref["frames"]).all(), b


def test_translated_jam():
    from tests import asm as A
    img = A.program(lambda b: (b.ins("LDA", "imm", 0x2A), b.ins("STA", "zp", A.COLUBK), b.ins("INC", "zp", 0x80),
                               b.byte(0x02)))
    w = I.Workload("jam", [I.Rom(0, 4096, 1, img)], np.zeros(5, np.int32), I.initial_ram(5, 5), None, 3, 2,
                   seed=99)
    ram, fr, _, vb = gpu_run(w, "translated", 4, 64)
    for b in range(5):
        ref = oracle_env(w, b)
        assert (ram[b] == ref["ram"]).all() and (fr[b] == ref["frames"]).all()
    assert (vb.regs().cpu().numpy()[:, 8] & 1).all()  # jammed


@pytest.mark.parametrize("max_positions", [8, 48])
def test_translated_small_budget_mixes_blocks_and_interpreter(max_positions):
    # most of the code is not translated: waves move between blocks and the interpreter all the time
    w = I.config_c1(num_envs=64, steps=8)
    import torch
    from paper_2606_22447_amd.vcs import VcsBatch
    say("translated budget", max_positions)
    vb = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed, kernel="translated", lanes_per_env=16,
                  block_threads=256, max_positions=max_positions)
    assert vb.translation["positions"] <= max_positions and vb.translation["truncated"]
    vb.reset(ram0=w.ram0)
    ram, fr, _ = vb.step(actions=w.actions, frames="all")
    torch.cuda.synchronize()
    ram, fr = ram.cpu().numpy(), fr.cpu().numpy()
    for b in range(w.num_envs):
        ref = oracle_env(w, b)
        assert (ram[b] == ref["ram"]).all(), b
        assert (fr[b] == ref["frames"]).all(), b


def test_translated_frames_last_and_none_modes():
    w = I.config_c1(num_envs=8, steps=5)
    ram_all, fr_all, _, _ = gpu_run(w, "translated", 16, 256, frames="all")
    ram_last, fr_last, _, _ = gpu_run(w, "translated", 16, 256, frames="last")
    ram_none, fr_none, _, _ = gpu_run(w, "translated", 16, 256, frames="none")
    assert (ram_all == ram_last).all() and (ram_all == ram_none).all()
    assert (fr_last == fr_all[:, -1]).all() and fr_none is None
