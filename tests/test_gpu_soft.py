"""GPU parity of the SOFT-STE path: forward = hard = oracle (Theorem "Exact
forward equivalence") and surrogate gradients vs the oracle's FP64 reference."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import inputs as I

pytestmark = pytest.mark.gpu

N_PIX = 210 * 160


def say(*a):
    print(*a, flush=True)


def lum(c):
    return (np.asarray(c).astype(np.int64) >> 1) & 7


class Problem:
    """A soft workload with its loss gradient dL/dframe computed from the oracle."""

    def __init__(self, w: I.Workload, tau: float, seed: int = 7):
        self.w, self.tau = w, tau
        lv = I.soft_leaves(w, seed)
        self.logits, self.tape, self.act = lv.rom_logits, lv.ram_tape, lv.action_logits
        offs = w.rom_offsets()
        self.offs = offs
        self.dec_rom = O.decode_logits(self.logits, tau)      # hard, ev, m, z
        self.dec_tape = O.decode_tape(self.tape)              # hard, ev
        self.dec_act = O.decode_actions(self.act, tau)        # hard, E sw, E in
        B, S = w.num_envs, w.steps
        self.hard_act = self.dec_act[0].reshape(B, S)
        self.hard_ram0 = self.dec_tape[0].reshape(B, 128)
        self.target = np.zeros((B, 210, 160), np.uint8)
        self.hard = []
        for b in range(B):
            r = int(w.env_rom[b])
            img = self.dec_rom[0][offs[r]:offs[r] + w.roms[r].size]
            self.hard.append(O.run_env(img, w.roms[r].mapper, self.hard_ram0[b], self.hard_act[b], S, w.frame_skip,
                                       frames="last"))
            pert = lv.perturbed_roms[r]
            self.target[b] = O.run_env(pert, w.roms[r].mapper, self.hard_ram0[b], self.hard_act[b], S,
                                       w.frame_skip, frames="last")["frames"][0]
        fr = np.stack([h["frames"][0] for h in self.hard])
        d = lum(fr) - lum(self.target)
        self.grad_frame = ((2.0 * d / N_PIX) * 0.5).astype(np.float32)
        self.loss = float((d.astype(np.float64) ** 2).mean(axis=(1, 2)).sum())

    def oracle_grads(self):
        if getattr(self, "_grads", None) is None:
            self._grads = self._oracle_grads()
        return self._grads

    def _oracle_grads(self):
        w, B, S = self.w, self.w.num_envs, self.w.steps
        g_rom = np.zeros(self.logits.shape[0])
        g0 = np.zeros((B, 128))
        gsw = np.zeros((B, S))
        gin = np.zeros((B, S))
        for b in range(B):
            r = int(w.env_rom[b])
            o, n = self.offs[r], w.roms[r].size
            res = O.soft_env(self.dec_rom[0][o:o + n], self.dec_rom[1][o:o + n], w.roms[r].mapper,
                             self.hard_ram0[b], self.dec_tape[1].reshape(B, 128)[b], self.hard_act[b],
                             self.dec_act[1].reshape(B, S)[b], self.dec_act[2].reshape(B, S)[b], S, w.frame_skip,
                             mode="ste", grad_frame=self.grad_frame[b].astype(np.float64))
            g_rom[o:o + n] += res["g_rom"]
            g0[b] = res["g_ram0"]
            gsw[b], gin[b] = res["g_swcha"], res["g_inpt4"]
        return (O.epilogue_rom(self.logits, self.tau, g_rom), O.epilogue_tape(g0).reshape(B, 128, 256),
                O.epilogue_action(self.act, self.tau, gsw.reshape(-1), gin.reshape(-1)).reshape(B, S, 18))


def run_gpu(p: Problem, alpha=6.0, K=1024, G=0, tpb=0, grad_ram=None, tape=0):
    import torch
    from paper_2606_22447_amd.vcs import SoftVcs
    w = p.w
    sim = SoftVcs(w.roms, w.env_rom, frame_skip=w.frame_skip, ckpt_interval=K, lanes_per_env=G, block_threads=tpb,
                  tape_records=tape)
    dev = sim.device
    L = torch.from_numpy(p.logits).to(dev)
    T = torch.from_numpy(p.tape).to(dev)
    Aa = torch.from_numpy(p.act).to(dev)
    ram, frame, residual, dec, st = sim.forward(L, T, Aa, p.tau, alpha, want_decode=True)
    gf = torch.from_numpy(p.grad_frame).to(dev)
    gr = None if grad_ram is None else torch.from_numpy(grad_ram.astype(np.float32)).to(dev)
    g = sim.backward(residual, L, T, Aa, p.tau, alpha, gf, gr, check_overflow=True)
    torch.cuda.synchronize()
    return (ram.cpu().numpy(), frame.cpu().numpy(), dec.cpu().numpy(), sim, [x.cpu().numpy() for x in g])


def assert_grad_close(g, ref, name):
    m = np.abs(ref).max()
    if m == 0:  # no path from this leaf to the loss: structural zeros everywhere
        assert (g == 0).all(), (name, np.abs(g).max())
        return
    err = np.abs(g.astype(np.float64) - ref)
    assert err.max() <= 1e-4 * m, (name, err.max(), m)
    big = np.abs(ref) >= 1e-3 * m
    rel = err[big] / np.abs(ref[big])
    assert rel.max() <= 1e-4, (name, rel.max())
    zero = ref == 0
    assert (g[zero] == 0).all(), (name, np.abs(g[zero]).max())


@pytest.fixture(scope="module", params=[1.0, 0.1])
def c3(request):
    w = I.config_c3()  # the small soft workload at its size: 256 envs, 2 frames
    assert w.num_envs == 256
    return Problem(w, request.param)


def test_theorem1_soft_forward_equals_hard(c3):
    p = c3
    for alpha in (2.0, 6.0, 20.0):
        say("theorem1 tau", p.tau, "alpha", alpha)
        ram, frame, dec, sim, _ = run_gpu(p, alpha=alpha)
        for b in range(p.w.num_envs):
            assert (ram[b] == p.hard[b]["ram"].astype(np.float32)).all(), b
            assert (frame[b] == p.hard[b]["frames"][0].astype(np.float32)).all(), b


def test_decode_statistics(c3):
    p = c3
    _, _, dec, sim, _ = run_gpu(p)
    total = p.logits.shape[0]
    rom = dec[: total * 3].reshape(total, 3)
    assert np.allclose(rom[:, 0], p.dec_rom[1], rtol=1e-5, atol=1e-4)
    assert np.allclose(rom[:, 1], p.dec_rom[2], rtol=1e-6)
    assert np.allclose(rom[:, 2], p.dec_rom[3], rtol=1e-5)
    B, S = p.w.num_envs, p.w.steps
    tape = dec[total * 3: total * 3 + B * 128]
    assert np.allclose(tape, p.dec_tape[1], rtol=1e-6)
    act = dec[total * 3 + B * 128:].reshape(B * S, 2)
    assert np.allclose(act[:, 0], p.dec_act[1], rtol=1e-5) and np.allclose(act[:, 1], p.dec_act[2], rtol=1e-5,
                                                                              atol=1e-4)


def test_gradients_match_fp64_oracle(c3):
    p = c3
    say("grads tau", p.tau)
    ref = p.oracle_grads()
    _, _, _, _, g = run_gpu(p)
    for gi, ri, name in zip(g, ref, ("rom_logits", "ram_tape", "action_logits")):
        if name == "action_logits" and np.abs(ri).max() == 0:
            assert (gi == 0).all()  # this ROM reads no inputs: structural zeros
            continue
        assert_grad_close(gi, ri, name)


def test_gradients_invariant_to_alpha_and_checkpoint_interval(c3):
    p = c3
    base = run_gpu(p, alpha=6.0, K=1024)[4]
    for alpha, K in ((2.0, 1024), (20.0, 1024), (6.0, 256), (6.0, 4096)):
        say("invariance alpha", alpha, "K", K)
        g = run_gpu(p, alpha=alpha, K=K)[4]
        for a, b in zip(g, base):
            assert (a == b).all()


def test_hetero_roms_with_inputs_and_ram_out_gradient():
    roms = [I.generate_rom(100 + i, sz, reads_inputs=True, timer_vblank=True)
            for i, sz in enumerate([2048, 8192, 4096])]
    B, S = 12, 3
    env_rom = (np.arange(B) % 3).astype(np.int32)
    w = I.Workload("soft_hetero", roms, env_rom, I.initial_ram(21, B), I.action_stream(21, B, S), S, 1, seed=21)
    p = Problem(w, 1.0)
    rng = np.random.default_rng(3)
    grad_ram = rng.standard_normal((B, S, 128)) * 1e-2
    say("hetero soft with ram-out grad")
    g = run_gpu(p, K=256, grad_ram=grad_ram)[4]
    # oracle with the same dL/dRAM_out
    g_rom = np.zeros(p.logits.shape[0])
    g0 = np.zeros((B, 128))
    gsw, gin = np.zeros((B, S)), np.zeros((B, S))
    for b in range(B):
        r = int(env_rom[b])
        o, n = p.offs[r], roms[r].size
        res = O.soft_env(p.dec_rom[0][o:o + n], p.dec_rom[1][o:o + n], roms[r].mapper, p.hard_ram0[b],
                         p.dec_tape[1].reshape(B, 128)[b], p.hard_act[b], p.dec_act[1].reshape(B, S)[b],
                         p.dec_act[2].reshape(B, S)[b], S, 1, mode="ste",
                         grad_frame=p.grad_frame[b].astype(np.float64),
                         grad_ram=grad_ram[b].astype(np.float32).astype(np.float64))
        g_rom[o:o + n] += res["g_rom"]
        g0[b] = res["g_ram0"]
        gsw[b], gin[b] = res["g_swcha"], res["g_inpt4"]
    ref = (O.epilogue_rom(p.logits, 1.0, g_rom), O.epilogue_tape(g0).reshape(B, 128, 256),
           O.epilogue_action(p.act, 1.0, gsw.reshape(-1), gin.reshape(-1)).reshape(B, S, 18))
    for gi, ri, name in zip(g, ref, ("rom_logits", "ram_tape", "action_logits")):
        if np.abs(ri).max() == 0:
            assert (gi == 0).all(), name
            continue
        assert_grad_close(gi, ri, name)


@pytest.mark.parametrize("G,tpb,K,tape", [(64, 256, 512, -1), (16, 256, 1024, -1), (4, 64, 256, -1),
                                           (64, 1024, 512, 3000)])
def test_forward_tape_gives_the_recompute_gradients(G, tpb, K, tape):
    """The soft forward that keeps its tape (every segment before the final frame,
    or a 3000-record tape that runs out): the backward sweeps those segments
    without recomputing them, with gradients bit-identical to the recomputing
    backward's, and within the tolerance of the FP64 oracle."""
    roms = [I.generate_rom(100 + i, sz, reads_inputs=True, timer_vblank=True)
            for i, sz in enumerate([2048, 8192, 4096])]
    B, S = 24, 4
    env_rom = (np.arange(B) % 3).astype(np.int32)
    w = I.Workload("soft_tape", roms, env_rom, I.initial_ram(23, B), I.action_stream(23, B, S), S, 2, seed=23)
    p = Problem(w, 1.0)
    grad_ram = np.random.default_rng(8).standard_normal((B, S, 128)) * 1e-2
    say("forward tape G", G, "tpb", tpb, "K", K, "tape", tape)
    r0 = run_gpu(p, K=K, G=G, tpb=tpb, grad_ram=grad_ram)
    r1 = run_gpu(p, K=K, G=G, tpb=tpb, grad_ram=grad_ram, tape=tape)
    assert (r0[0] == r1[0]).all() and (r0[1] == r1[1]).all()
    for a, b, name in zip(r0[4], r1[4], ("rom_logits", "ram_tape", "action_logits")):
        assert np.array_equal(a, b), (name, np.abs(a - b).max())
    if tape < 0:  # one env against the oracle (the rest follow from the identity above)
        r, b = int(env_rom[1]), 1
        o, n = p.offs[r], roms[r].size
        res = O.soft_env(p.dec_rom[0][o:o + n], p.dec_rom[1][o:o + n], roms[r].mapper, p.hard_ram0[b],
                         p.dec_tape[1].reshape(B, 128)[b], p.hard_act[b], p.dec_act[1].reshape(B, S)[b],
                         p.dec_act[2].reshape(B, S)[b], S, 2, mode="ste",
                         grad_frame=p.grad_frame[b].astype(np.float64),
                         grad_ram=grad_ram[b].astype(np.float32).astype(np.float64))
        g0 = r1[4][1].reshape(B, 128, 256)[b]
        assert_grad_close(g0, O.epilogue_tape(res["g_ram0"][None]).reshape(128, 256), "ram_tape env 1")


def test_autograd_function_end_to_end(c3):
    import torch
    from paper_2606_22447_amd.vcs import SoftVcs, soft_rollout, ste_luminance
    p = c3
    w = p.w
    sim = SoftVcs(w.roms, w.env_rom, frame_skip=w.frame_skip)
    L = torch.from_numpy(p.logits).cuda().requires_grad_()
    T = torch.from_numpy(p.tape).cuda().requires_grad_()
    Aa = torch.from_numpy(p.act).cuda().requires_grad_()
    ram, frame = soft_rollout(sim, L, T, Aa, p.tau)
    tgt = torch.from_numpy(p.target).cuda().float()
    loss = ((ste_luminance(frame) - ste_luminance(tgt).detach()) ** 2).mean(dim=(1, 2)).sum()
    loss.backward()
    assert abs(loss.item() - p.loss) <= 1e-6 * max(1.0, p.loss)
    ref = p.oracle_grads()
    assert_grad_close(L.grad.cpu().numpy(), ref[0], "rom_logits")
    assert_grad_close(T.grad.cpu().numpy(), ref[1], "ram_tape")


def test_soft_forward_continues_a_hard_state():
    """The env step state + action -> next state taken softly: hard steps first
    (the interpreting kernel), then the soft forward from the state they left,
    on input-reading 2K/4K/F8 ROMs.  Forward = the oracle's hard rollout of all
    steps; gradients = the oracle's, with the state a constant (no tape
    gradient); the same through the autograd function."""
    import torch
    from paper_2606_22447_amd.vcs import SoftVcs, VcsBatch, soft_rollout
    roms = [I.generate_rom(100 + i, sz, reads_inputs=True, timer_vblank=True)
            for i, sz in enumerate([2048, 8192, 4096])]
    B, PRE, S, tau = 12, 3, 2, 1.0
    env_rom = (np.arange(B) % 3).astype(np.int32)
    ram0 = I.initial_ram(22, B)
    pre_act = I.action_stream(23, B, PRE)
    w = I.Workload("soft_from_state", roms, env_rom, ram0, I.action_stream(24, B, S), S, 1, seed=22)
    lv = I.soft_leaves(w, 9)
    offs = w.rom_offsets()
    dr = O.decode_logits(lv.rom_logits, tau)
    da = O.decode_actions(lv.action_logits, tau)
    hard_act = da[0].reshape(B, S)
    rng = np.random.default_rng(4)
    gf = (rng.standard_normal((B, 210, 160)) * 1e-3).astype(np.float32)
    gr = (rng.standard_normal((B, S, 128)) * 1e-2).astype(np.float32)
    # the hard steps run on the decoded ROM bytes: the soft steps continue the same machine
    imgs = [(dr[0][offs[r]:offs[r] + roms[r].size], roms[r].mapper) for r in range(3)]
    say("soft from state: hard pre-steps", PRE)
    vb = VcsBatch(imgs, env_rom, frame_skip=1, kernel="grouped")
    vb.reset(ram0=ram0)
    vb.step(actions=pre_act, frames="none")
    g_rom = np.zeros(lv.rom_logits.shape[0])
    gsw, gin = np.zeros((B, S)), np.zeros((B, S))
    refs = []
    for b in range(B):
        r = int(env_rom[b])
        o, n = offs[r], roms[r].size
        res = O.soft_env(dr[0][o:o + n], dr[1][o:o + n], roms[r].mapper, ram0[b], ram0[b].astype(np.float64),
                         hard_act[b], da[1].reshape(B, S)[b], da[2].reshape(B, S)[b], S, 1, mode="ste",
                         grad_frame=gf[b].astype(np.float64), grad_ram=gr[b].astype(np.float64),
                         pre_actions=pre_act[b])
        assert (res["g_ram0"] == 0).all()
        full = O.run_env(dr[0][o:o + n], roms[r].mapper, ram0[b], np.concatenate([pre_act[b], hard_act[b]]),
                         PRE + S, 1, frames="last")
        assert (res["ram"] == full["ram"][PRE:]).all() and (res["frame"] == full["frames"][0]).all()
        g_rom[o:o + n] += res["g_rom"]
        gsw[b], gin[b] = res["g_swcha"], res["g_inpt4"]
        refs.append(res)
    ref_rom = O.epilogue_rom(lv.rom_logits, tau, g_rom)
    ref_act = O.epilogue_action(lv.action_logits, tau, gsw.reshape(-1), gin.reshape(-1)).reshape(B, S, 18)
    for G in (64, 4):
        say("soft from state, lanes per env", G)
        sim = SoftVcs(roms, env_rom, frame_skip=1, ckpt_interval=512, lanes_per_env=G, block_threads=256)
        L = torch.from_numpy(lv.rom_logits).cuda()
        A = torch.from_numpy(lv.action_logits).cuda()
        state = vb.state.clone()
        ram, frame, residual, _, st = sim.forward(L, None, A, tau, 6.0, want_state=True, state_in=state)
        g = sim.backward(residual, L, None, A, tau, 6.0, torch.from_numpy(gf).cuda(), torch.from_numpy(gr).cuda(),
                         check_overflow=True)
        torch.cuda.synchronize()
        ram, frame = ram.cpu().numpy(), frame.cpu().numpy()
        for b in range(B):
            assert (ram[b] == refs[b]["ram"]).all() and (frame[b] == refs[b]["frame"]).all(), b
        assert g[1] is None
        assert_grad_close(g[0].cpu().numpy(), ref_rom, "rom_logits")
        assert_grad_close(g[2].cpu().numpy(), ref_act, "action_logits")
        # the soft call's final state is the hard machine's after PRE + S steps
        vh = VcsBatch(imgs, env_rom, frame_skip=1, kernel="grouped")
        vh.reset(ram0=ram0)
        vh.step(actions=np.concatenate([pre_act, hard_act], axis=1), frames="none")
        assert torch.equal(vh.regs(), _regs_of(vh, st)) and torch.equal(vh.hash(), _hash_of(vh, st))
    # autograd: the tape gets no gradient, the ROM and action logits get the oracle's
    Lg = torch.from_numpy(lv.rom_logits).cuda().requires_grad_()
    Ag = torch.from_numpy(lv.action_logits).cuda().requires_grad_()
    ram, frame = soft_rollout(sim, Lg, None, Ag, tau, 6.0, state_in=vb.state.clone())
    ((frame * torch.from_numpy(gf).cuda()).sum() + (ram * torch.from_numpy(gr).cuda()).sum()).backward()
    assert_grad_close(Lg.grad.cpu().numpy(), ref_rom, "rom_logits (autograd)")
    assert_grad_close(Ag.grad.cpu().numpy(), ref_act, "action_logits (autograd)")


def _regs_of(vb, state):
    saved = vb.state
    vb.state = state
    try:
        return vb.regs()
    finally:
        vb.state = saved


def _hash_of(vb, state):
    saved = vb.state
    vb.state = state
    try:
        return vb.hash()
    finally:
        vb.state = saved


def test_soft_api_refuses_wrong_leaves():
    """Leaves of the wrong dtype, shape, device or layout are refused before any launch."""
    import torch
    from paper_2606_22447_amd import binding as Bd
    from paper_2606_22447_amd.vcs import SoftVcs
    w = I.config_c3(num_envs=2)
    lv = I.soft_leaves(w)
    sim = SoftVcs(w.roms, w.env_rom, frame_skip=1)
    L = torch.from_numpy(lv.rom_logits).cuda()
    T = torch.from_numpy(lv.ram_tape).cuda()
    A = torch.from_numpy(lv.action_logits).cuda()
    for bad in (L.double(), L[:-1], L.cpu(), L.t().contiguous().t()):
        with pytest.raises(Bd.VcsError):
            sim.forward(bad, T, A, 1.0)
    with pytest.raises(Bd.VcsError):
        sim.forward(L, T[:, :64], A, 1.0)
    with pytest.raises(Bd.VcsError):
        sim.forward(L, None, A, 1.0)  # no tape and no starting state
    _, _, res, _, _ = sim.forward(L, T, A, 1.0)
    with pytest.raises(Bd.VcsError):
        sim.backward(res, L, T, A, 1.0, 6.0, torch.zeros((2, 210, 161), device="cuda"))
