"""GPU parity of the TIA objects (players, missiles, ball, motion, collisions)
and of the position sampler, through the C ABI, against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import inputs as I
from tests import asm as A
from tests.test_gpu_hard import gpu_run, oracle_env, say
from tests.test_objects_cpu import PROGRAMS, _hand_bodies, oracle_objects

pytestmark = pytest.mark.gpu

SHAPES = [("plain", 1, 256), ("grouped", 1, 64), ("grouped", 4, 256), ("grouped", 16, 256), ("grouped", 64, 1024),
          ("translated", 16, 256), ("translated", 4, 64)]


def _objects_of(vb):
    return vb.objects().cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("kernel,G,tpb", SHAPES)
def test_sprite_workload_every_byte(kernel, G, tpb):
    w = I.config_objects(envs_per_rom=6, steps=5, n_roms=8, frame_skip=2)
    say("objects", kernel, G, tpb, w.num_envs)
    ram, fr, done, vb = gpu_run(w, kernel, G, tpb, splits=(2,))
    objs = _objects_of(vb)
    for b in range(w.num_envs):
        ref = oracle_env(w, b)
        assert (ram[b] == ref["ram"]).all(), (kernel, b)
        assert (fr[b] == ref["frames"]).all(), (kernel, b, np.argwhere(fr[b] != ref["frames"])[:4])
        rom = w.roms[int(w.env_rom[b])]
        _, _, o = oracle_objects(rom.image, rom.mapper, w.ram0[b], w.actions[b], w.steps, w.frame_skip)
        assert (objs[b] == o).all(), (kernel, b, objs[b].tolist(), o.tolist())


@pytest.mark.parametrize("kernel,G,tpb", [("grouped", 4, 64), ("plain", 1, 64), ("translated", 16, 256)])
def test_hand_programs(kernel, G, tpb):
    images = [A.program(f) for f in PROGRAMS.values()] + _hand_bodies()
    roms = [I.Rom(i, 4096, 1, img) for i, img in enumerate(images)]
    B = 2 * len(roms)
    env_rom = (np.arange(B) % len(roms)).astype(np.int32)
    w = I.Workload("hand_objects", roms, env_rom, np.zeros((B, 128), np.uint8), None, 2, 1)
    say("hand objects", kernel, G, tpb)
    ram, fr, _, vb = gpu_run(w, kernel, G, tpb)
    objs = _objects_of(vb)
    for b in range(B):
        f, r, o = oracle_objects(roms[int(env_rom[b])].image, 1, np.zeros(128, np.uint8), None, 2, 1)
        assert (fr[b, -1] == f).all() and (ram[b, -1] == r).all(), (kernel, b)
        assert (objs[b] == o).all(), (kernel, b)


def test_soft_tangents_and_gradients():
    import torch
    from paper_2606_22447_amd.vcs import SoftVcs
    from tests.test_gpu_soft import Problem, assert_grad_close
    w = I.config_objects(envs_per_rom=4, steps=3, n_roms=4, frame_skip=1)
    p = Problem(w, 1.0)
    B = w.num_envs
    # a dense dL/dframe (the sprite kernels have no colour immediates for Problem's target to perturb)
    p.grad_frame = (np.random.default_rng(4).standard_normal((B, 210, 160)) * 1e-3).astype(np.float32)
    say("objects soft", B)
    sim = SoftVcs(w.roms, w.env_rom, frame_skip=1, ckpt_interval=1024)
    dev = sim.device
    L, T, Aa = (torch.from_numpy(x).to(dev) for x in (p.logits, p.tape, p.act))
    dpos = torch.empty((B, 5, 210, 160), dtype=torch.float32, device=dev)
    ram, frame, res, _, _ = sim.forward(L, T, Aa, p.tau, 6.0, frame_dpos=dpos)
    g = sim.backward(res, L, T, Aa, p.tau, 6.0, torch.from_numpy(p.grad_frame).to(dev), check_overflow=True)
    torch.cuda.synchronize()
    frame, dpos = frame.cpu().numpy(), dpos.cpu().numpy()
    for b in range(B):
        r = int(w.env_rom[b])
        o, n = p.offs[r], w.roms[r].size
        ref = O.soft_env(p.dec_rom[0][o:o + n], p.dec_rom[1][o:o + n], w.roms[r].mapper, p.hard_ram0[b],
                         p.dec_tape[1].reshape(B, 128)[b], p.hard_act[b], p.dec_act[1].reshape(B, -1)[b],
                         p.dec_act[2].reshape(B, -1)[b], w.steps, 1, grad_frame=p.grad_frame[b].astype(np.float64))
        assert (frame[b] == ref["frame"]).all(), b
        assert (dpos[b] == ref["frame_dpos"]).all(), (b, np.argwhere(dpos[b] != ref["frame_dpos"])[:4])
        g_pos = (dpos[b].astype(np.float64) * p.grad_frame[b][None].astype(np.float64)).reshape(5, -1).sum(1)
        np.testing.assert_allclose(g_pos, ref["g_pos"], rtol=1e-9, atol=1e-12)
    assert np.abs(dpos).sum() > 0
    refs = p.oracle_grads()
    assert np.abs(refs[0]).max() > 0  # object pixels route gradient to their colour sources
    for gi, ri, name in zip((x.cpu().numpy() for x in g), refs, ("rom_logits", "ram_tape", "action_logits")):
        assert_grad_close(gi, ri, name)


def test_relaxed_on_sprite_roms():
    from paper_2606_22447_amd.vcs import VcsBatch
    w = I.config_objects(envs_per_rom=2, steps=2, n_roms=4, frame_skip=1)
    say("objects relaxed")
    vb = VcsBatch(w.roms, w.env_rom, frame_skip=1, seed=w.seed, kernel="grouped", lanes_per_env=4, block_threads=64)
    vb.reset(ram0=w.ram0)
    ram, fr, rel = vb.step_relaxed(6.0, 0.14, actions=w.actions, frames="all")
    ram, fr, rel = ram.cpu().numpy(), fr.cpu().numpy(), rel.cpu().numpy()
    for b in range(w.num_envs):
        rom = w.roms[int(w.env_rom[b])]
        ref = O.run_relaxed(rom.image, rom.mapper, w.ram0[b], w.actions[b], w.steps, 1, 6.0, 0.14)
        assert (ram[b] == ref["ram"]).all() and (fr[b] == ref["frames"]).all(), b
        assert rel[b].tolist() == [ref["ndiv"], ref["fails"]], b


def test_collision_latches_reach_ram_and_differ_across_envs():
    # the overscan copies CXM0P..CXPPMM into $86-$8D: the joystick moves P0, so
    # the envs' latches differ; the GPU's match the oracle's (checked above) and
    # are not all zero
    w = I.config_objects(envs_per_rom=8, steps=4, n_roms=2, frame_skip=2)
    ram, _, _, _ = gpu_run(w, "grouped", 4, 256, frames="none")
    cx = ram[:, -1, I.OBJ_CX - 0x80:I.OBJ_CX - 0x80 + 8]
    assert cx.any() and len({bytes(r) for r in cx}) > 1
    for b in range(w.num_envs):
        assert (ram[b] == oracle_env(w, b, frames="none")["ram"]).all(), b


def test_address_surrogate_gradients():
    """The backward with the address surrogate on (Eq. s-read at temperature 1):
    indexed ROM reads (the sprite kernels' colour tables) pass gradient to Y."""
    import torch
    from paper_2606_22447_amd.vcs import SoftVcs
    from tests.test_gpu_soft import Problem, assert_grad_close
    w = I.config_objects(envs_per_rom=4, steps=2, n_roms=8, frame_skip=1)
    p = Problem(w, 1.0)
    B, S = w.num_envs, w.steps
    p.grad_frame = (np.random.default_rng(6).standard_normal((B, 210, 160)) * 1e-3).astype(np.float32)
    say("objects address surrogate", B)
    sim = SoftVcs(w.roms, w.env_rom, frame_skip=1, ckpt_interval=512)
    dev = sim.device
    L, T, Aa = (torch.from_numpy(x).to(dev) for x in (p.logits, p.tape, p.act))
    _, _, res, _, _ = sim.forward(L, T, Aa, p.tau, 6.0)
    g = [x.cpu().numpy() for x in sim.backward(res, L, T, Aa, p.tau, 6.0, torch.from_numpy(p.grad_frame).to(dev),
                                               check_overflow=True, read_T=1.0)]
    g_rom = np.zeros(p.logits.shape[0])
    g0 = np.zeros((B, 128))
    gsw = np.zeros((B, S))
    gin = np.zeros((B, S))
    for b in range(B):
        r = int(w.env_rom[b])
        o, n = p.offs[r], w.roms[r].size
        ref = O.soft_env(p.dec_rom[0][o:o + n], p.dec_rom[1][o:o + n], w.roms[r].mapper, p.hard_ram0[b],
                         p.dec_tape[1].reshape(B, 128)[b], p.hard_act[b], p.dec_act[1].reshape(B, S)[b],
                         p.dec_act[2].reshape(B, S)[b], S, 1, grad_frame=p.grad_frame[b].astype(np.float64),
                         read_T=1.0)
        g_rom[o:o + n] += ref["g_rom"]
        g0[b] = ref["g_ram0"]
        gsw[b], gin[b] = ref["g_swcha"], ref["g_inpt4"]
    refs = (O.epilogue_rom(p.logits, p.tau, g_rom), O.epilogue_tape(g0).reshape(B, 128, 256),
            O.epilogue_action(p.act, p.tau, gsw.reshape(-1), gin.reshape(-1)).reshape(B, S, 18))
    for gi, ri, name in zip(g, refs, ("rom_logits", "ram_tape", "action_logits")):
        assert_grad_close(gi, ri, name)
    # and the surrogate changed the ROM gradient against the plain STE one
    assert np.abs(refs[0] - p.oracle_grads()[0]).max() > 0
