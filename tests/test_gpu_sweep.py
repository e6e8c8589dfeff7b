"""GPU parity on the opcode-sweep workload: every one of the 189 opcode bytes in
every addressing form (indexed accesses with and without page crossings,
read-modify-write on RAM, TIA and RIOT registers, all timer intervals, TIMINT,
bank switches on every kind of data access, code in RAM), for every kernel and
launch shape, hard and soft, byte for byte / within the gradient tolerance
against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import inputs as I
from tests.test_gpu_hard import KERNELS, gpu_run, oracle_env, say
from tests.test_gpu_soft import assert_grad_close

pytestmark = pytest.mark.gpu

_REF = {}


def sweep_workload(objects=True):
    return I.config_sweep(envs_per_rom=32, steps=4, frame_skip=2, episodes=True, objects=objects)


def reference(w, objects=True):
    if objects not in _REF:
        _REF[objects] = [oracle_env(w, b) for b in range(w.num_envs)]
    return _REF[objects]


SHAPES = KERNELS + [("translated", 4, 256), ("translated", 32, 256), ("translated", 64, 64)]


# objects=False: images kept off the object registers run wholly in the hard
# step's first pass (the translated code, or the interpreter without the object
# paths); the full images mostly in its second pass (the interpreter with them)
@pytest.mark.parametrize("objects", [True, False], ids=["full", "no_objects"])
@pytest.mark.parametrize("kernel,G,tpb", SHAPES)
def test_sweep_every_byte(kernel, G, tpb, objects):
    w = sweep_workload(objects)
    say("sweep", kernel, G, tpb, "envs", w.num_envs, "objects", objects)
    refs = reference(w, objects)
    ram, fr, done, vb = gpu_run(w, kernel, G, tpb, splits=(1,))
    regs = vb.regs().cpu().numpy()
    for b in range(w.num_envs):
        ref = refs[b]
        assert (ram[b] == ref["ram"]).all(), (b, int(w.env_rom[b]))
        assert (fr[b] == ref["frames"]).all(), (b, int(w.env_rom[b]))
        assert (done[b] == ref["done"]).all(), b
        r = ref["regs"]
        assert regs[b].tolist() == [r[k] for k in O.REG_NAMES[:16]], (b, regs[b].tolist())


def test_sweep_soft_forward_and_gradients():
    """Soft forward = hard on the sweep images, and the surrogate gradients of a
    random dL/dframe and dL/dRAM_out against the FP64 oracle, K = 512."""
    import torch
    from paper_2606_22447_amd.vcs import SoftVcs
    w = I.config_sweep(envs_per_rom=8, steps=2, frame_skip=1, episodes=False)
    B, S, tau = w.num_envs, w.steps, 1.0
    lv = I.soft_leaves(w, 13)
    offs = w.rom_offsets()
    dr = O.decode_logits(lv.rom_logits, tau)
    dt = O.decode_tape(lv.ram_tape)
    da = O.decode_actions(lv.action_logits, tau)
    hard_act = da[0].reshape(B, S)
    ram0 = dt[0].reshape(B, 128)
    rng = np.random.default_rng(5)
    gf = (rng.standard_normal((B, 210, 160)) * 1e-3).astype(np.float32)
    gr = (rng.standard_normal((B, S, 128)) * 1e-2).astype(np.float32)
    g_rom = np.zeros(lv.rom_logits.shape[0])
    g0 = np.zeros((B, 128))
    gsw, gin = np.zeros((B, S)), np.zeros((B, S))
    ref_ram, ref_fr = [], []
    for b in range(B):
        r = int(w.env_rom[b])
        o, n = offs[r], w.roms[r].size
        res = O.soft_env(dr[0][o:o + n], dr[1][o:o + n], w.roms[r].mapper, ram0[b], dt[1].reshape(B, 128)[b],
                         hard_act[b], da[1].reshape(B, S)[b], da[2].reshape(B, S)[b], S, 1, mode="ste",
                         grad_frame=gf[b].astype(np.float64), grad_ram=gr[b].astype(np.float64))
        g_rom[o:o + n] += res["g_rom"]
        g0[b] = res["g_ram0"]
        gsw[b], gin[b] = res["g_swcha"], res["g_inpt4"]
        ref_ram.append(res["ram"])
        ref_fr.append(res["frame"])
    ref = (O.epilogue_rom(lv.rom_logits, tau, g_rom), O.epilogue_tape(g0).reshape(B, 128, 256),
           O.epilogue_action(lv.action_logits, tau, gsw.reshape(-1), gin.reshape(-1)).reshape(B, S, 18))
    for G in (64, 16):
        say("sweep soft, lanes per env", G)
        sim = SoftVcs(w.roms, w.env_rom, frame_skip=1, ckpt_interval=512, lanes_per_env=G, block_threads=256)
        L = torch.from_numpy(lv.rom_logits).cuda()
        T = torch.from_numpy(lv.ram_tape).cuda()
        A = torch.from_numpy(lv.action_logits).cuda()
        ram, frame, residual, _, _ = sim.forward(L, T, A, tau, 6.0)
        g = sim.backward(residual, L, T, A, tau, 6.0, torch.from_numpy(gf).cuda(), torch.from_numpy(gr).cuda(),
                         check_overflow=True)
        torch.cuda.synchronize()
        ram, frame = ram.cpu().numpy(), frame.cpu().numpy()
        for b in range(B):
            assert (ram[b] == ref_ram[b]).all() and (frame[b] == ref_fr[b]).all(), b
        for gi, ri, name in zip([x.cpu().numpy() for x in g], ref, ("rom_logits", "ram_tape", "action_logits")):
            assert_grad_close(gi, ri, name)
