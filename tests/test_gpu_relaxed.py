"""FULL relaxed mode on the GPU (vcs_step_relaxed, through the C ABI) against
the oracle over an (alpha, T) sweep on synthetic 2K/4K/F8 ROMs: the first
diverging instruction N_div and the failed casts of every env, and every RAM
and frame byte of the (possibly diverged) runs."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import inputs as I
from tests.test_relaxed_cpu import SWEEP, relaxed_roms

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("G,tpb", [(1, 64), (4, 256), (64, 256)])
def test_relaxed_sweep_matches_oracle(G, tpb):
    from paper_2606_22447_amd.vcs import VcsBatch
    roms = relaxed_roms()
    per, S, F = 8, 2, 1
    env_rom = np.repeat(np.arange(len(roms)), per).astype(np.int32)
    B = env_rom.size
    ram0 = I.initial_ram(70, B)
    acts = I.action_stream(71, B, S)
    for alpha, T in SWEEP:
        say("relaxed", G, tpb, "alpha", alpha, "T", T)
        vb = VcsBatch(roms, env_rom, frame_skip=F, kernel="grouped", lanes_per_env=G, block_threads=tpb)
        vb.reset(ram0=ram0)
        ram, fr, rx = vb.step_relaxed(alpha, T, actions=acts, frames="all")
        ram, fr, rx = ram.cpu().numpy(), fr.cpu().numpy(), rx.cpu().numpy()
        for b in range(B):
            rom = roms[int(env_rom[b])]
            ref = O.run_relaxed(rom.image, rom.mapper, ram0[b], acts[b], S, F, alpha, T)
            assert (int(rx[b, 0]), int(rx[b, 1])) == (ref["ndiv"], ref["fails"]), (b, alpha, T, rx[b])
            assert (ram[b] == ref["ram"]).all() and (fr[b] == ref["frames"]).all(), (b, alpha, T)


def test_relaxed_opcode_sweep_and_exact_point():
    """Every opcode form relaxed; and at alpha = 6, T = 0.14 the relaxed kernel equals
    the hard kernel on a full-size slice of the batched workload."""
    import torch
    from paper_2606_22447_amd.vcs import VcsBatch
    w = I.config_sweep(envs_per_rom=4, steps=2, frame_skip=1, episodes=False)
    for alpha, T in ((6.0, 0.14), (3.0, 0.25)):
        say("relaxed sweep workload", alpha, T)
        vb = VcsBatch(w.roms, w.env_rom, frame_skip=1, kernel="grouped", lanes_per_env=4, block_threads=256)
        vb.reset(ram0=w.ram0)
        ram, fr, rx = vb.step_relaxed(alpha, T, actions=w.actions, frames="all")
        ram, fr, rx = ram.cpu().numpy(), fr.cpu().numpy(), rx.cpu().numpy()
        for b in range(w.num_envs):
            rom = w.roms[int(w.env_rom[b])]
            ref = O.run_relaxed(rom.image, rom.mapper, w.ram0[b], w.actions[b], w.steps, 1, alpha, T)
            assert (int(rx[b, 0]), int(rx[b, 1])) == (ref["ndiv"], ref["fails"]), (b, alpha, T)
            assert (ram[b] == ref["ram"]).all() and (fr[b] == ref["frames"]).all(), (b, alpha, T)
    w = I.config_c1(num_envs=512, steps=3)
    say("relaxed exact point vs hard, 512 envs")
    a = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, kernel="grouped", lanes_per_env=16, block_threads=256)
    h = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, kernel="grouped", lanes_per_env=16, block_threads=256)
    a.reset(ram0=w.ram0)
    h.reset(ram0=w.ram0)
    ram_a, fr_a, rx = a.step_relaxed(6.0, 0.14, actions=w.actions, frames="all")
    ram_h, fr_h, _ = h.step(actions=w.actions, frames="all")
    torch.cuda.synchronize()
    assert (rx[:, 0] == -1).all() and (rx[:, 1] == 0).all()
    assert torch.equal(ram_a, ram_h) and torch.equal(fr_a, fr_h) and torch.equal(a.hash(), h.hash())


def test_relaxed_rejects_bad_parameters():
    from paper_2606_22447_amd import binding as Bd
    from paper_2606_22447_amd.vcs import VcsBatch
    w = I.config_c1(num_envs=4, steps=1)
    vb = VcsBatch(w.roms, w.env_rom, frame_skip=1, kernel="grouped")
    vb.reset(ram0=w.ram0)
    for alpha, T in ((0.0, 0.1), (6.0, 0.0), (float("nan"), 0.1), (6.0, float("inf"))):
        with pytest.raises(Bd.VcsError):
            vb.step_relaxed(alpha, T, actions=w.actions)
