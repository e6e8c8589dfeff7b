"""Further cartridge formats on the GPU, through the C ABI, byte for byte
against the oracle: F6, F6SC, F8SC and E0 on the LDS-staged kernels in several
launch shapes, all formats (also F4, F4SC) on the plain kernel, with in-run
resets reseeding RAM and Superchip RAM; the boot sequence with the console
RESET switch; soft gradients and FULL relaxed runs on F6 and E0 images; and
the configurations the kernels refuse."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import inputs as I
from tests.test_gpu_hard import gpu_run, oracle_env

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


_REF = {}


def _refs(w, key):
    if key not in _REF:
        _REF[key] = [oracle_env(w, b) for b in range(w.num_envs)]
    return _REF[key]


def _check(w, refs, ram, fr, done, vb, what):
    regs = vb.regs().cpu().numpy()
    for b in range(w.num_envs):
        ref, name = refs[b], I.MAPPER_NAMES[w.roms[int(w.env_rom[b])].mapper]
        assert (ram[b] == ref["ram"]).all(), (what, b, name)
        assert (fr[b] == ref["frames"]).all(), (what, b, name)
        assert (done[b] == ref["done"]).all(), (what, b, name)
        r = ref["regs"]
        assert regs[b].tolist() == [r[k] for k in O.REG_NAMES[:16]], (what, b, name)


@pytest.mark.parametrize("G,tpb", [(4, 256), (16, 256), (64, 1024), (1, 64)])
def test_lds_formats_every_byte(G, tpb):
    w = I.config_mappers(envs_per_rom=8, steps=4, frame_skip=2, lds_only=True)
    say("mappers grouped", G, tpb)
    ram, fr, done, vb = gpu_run(w, "grouped", G, tpb, splits=(2,))
    _check(w, _refs(w, "lds"), ram, fr, done, vb, f"grouped {G}/{tpb}")


def test_all_formats_on_the_plain_kernel():
    w = I.config_mappers(envs_per_rom=8, steps=4, frame_skip=2)
    say("mappers plain")
    ram, fr, done, vb = gpu_run(w, "plain", 1, 256, splits=(3,))
    _check(w, _refs(w, "all"), ram, fr, done, vb, "plain")


def test_boot_sequence_with_the_reset_switch():
    """60 NOOP + 4 RESET frames and 0..30 random NOOP frames (per env) at frame-skip 1, on a
    program that stores SWCHB to RAM every frame, and on the mapper images."""
    from paper_2606_22447_amd.vcs import VcsBatch
    roms = [I.generate_mapper_rom(s, m) for m, s in I.MAPPER_ROMS[:4]] + [I.generate_rom(104, 2048,
                                                                                          reads_inputs=True)]
    B = 20
    env_rom = (np.arange(B) % len(roms)).astype(np.int32)
    acts, extra = I.boot_actions(B, seed=8)
    for b in range(B):  # each env's random NOOPs, then joystick actions
        acts[b, 64 + extra[b]:] = I.action_stream(9, 1, acts.shape[1])[0][64 + extra[b]:]
    ram0 = I.initial_ram(8, B)
    vb = VcsBatch(roms, env_rom, frame_skip=1, seed=8, kernel="grouped", lanes_per_env=4, block_threads=256)
    vb.reset(ram0=ram0)
    ram, fr, _ = vb.step(actions=acts, frames="last")
    ram, fr = ram.cpu().numpy(), fr.cpu().numpy()
    for b in range(B):
        rom = roms[int(env_rom[b])]
        ref = O.run_env(rom.image, rom.mapper, ram0[b], acts[b], acts.shape[1], 1, seed=8, env_index=b,
                        frames="last")
        assert (ram[b] == ref["ram"]).all() and (fr[b] == ref["frames"][0]).all(), b


def test_soft_gradients_on_f6_and_e0():
    from tests.test_gpu_soft import Problem, assert_grad_close, run_gpu
    roms = [I.generate_mapper_rom(1, I.MAPPER_F6), I.generate_mapper_rom(4, I.MAPPER_E0)]
    B, S = 8, 2
    env_rom = (np.arange(B) % 2).astype(np.int32)
    w = I.Workload("soft_mappers", roms, env_rom, I.initial_ram(31, B), I.action_stream(31, B, S), S, 1, seed=31)
    p = Problem(w, 1.0)
    say("soft mappers")
    ram, frame, _, _, g = run_gpu(p, K=512)
    for b in range(B):
        assert (ram[b] == p.hard[b]["ram"]).all() and (frame[b] == p.hard[b]["frames"][0]).all(), b
    for gi, ri, name in zip(g, p.oracle_grads(), ("rom_logits", "ram_tape", "action_logits")):
        assert_grad_close(gi, ri, name)


def test_relaxed_on_f6_and_e0():
    from paper_2606_22447_amd.vcs import VcsBatch
    roms = [I.generate_mapper_rom(1, I.MAPPER_F6), I.generate_mapper_rom(4, I.MAPPER_E0)]
    B, S = 8, 2
    env_rom = (np.arange(B) % 2).astype(np.int32)
    ram0, acts = I.initial_ram(32, B), I.action_stream(32, B, S)
    for alpha, T in ((6.0, 0.14), (4.0, 0.14), (2.0, 0.3)):
        vb = VcsBatch(roms, env_rom, frame_skip=1, kernel="grouped", lanes_per_env=4, block_threads=256)
        vb.reset(ram0=ram0)
        ram, fr, rx = vb.step_relaxed(alpha, T, actions=acts, frames="all")
        ram, fr, rx = ram.cpu().numpy(), fr.cpu().numpy(), rx.cpu().numpy()
        for b in range(B):
            rom = roms[int(env_rom[b])]
            ref = O.run_relaxed(rom.image, rom.mapper, ram0[b], acts[b], S, 1, alpha, T)
            assert (int(rx[b, 0]), int(rx[b, 1])) == (ref["ndiv"], ref["fails"]), (b, alpha, T)
            assert (ram[b] == ref["ram"]).all() and (fr[b] == ref["frames"]).all(), (b, alpha, T)


def test_refused_configurations():
    import torch
    from paper_2606_22447_amd import binding as Bd
    from paper_2606_22447_amd.vcs import SoftVcs, VcsBatch
    f4 = I.generate_mapper_rom(5, I.MAPPER_F4)
    f6sc = I.generate_mapper_rom(2, I.MAPPER_F6SC)
    f6 = I.generate_mapper_rom(1, I.MAPPER_F6)
    with pytest.raises(Bd.VcsError):  # a 32 KB image does not fit the LDS-staged kernels
        VcsBatch([f4], [0], kernel="grouped")
    with pytest.raises(Bd.VcsError):  # 256 envs' RAM and Superchip RAM beside a 16 KB image
        VcsBatch([f6sc], [0], kernel="grouped", lanes_per_env=1, block_threads=256)
    with pytest.raises(Bd.VcsError):  # the translator takes 2K, 4K and F8
        VcsBatch([f6], [0], kernel="translated")
    sim = SoftVcs([f6sc], [0, 0], frame_skip=1)
    w = I.Workload("sc", [f6sc], np.zeros(2, np.int32), I.initial_ram(1, 2), I.action_stream(1, 2, 1), 1, 1)
    lv = I.soft_leaves(w)
    with pytest.raises(Bd.VcsError):  # no Superchip RAM in the soft graph
        sim.forward(torch.from_numpy(lv.rom_logits).cuda(), torch.from_numpy(lv.ram_tape).cuda(),
                    torch.from_numpy(lv.action_logits).cuda(), 1.0)
