"""Full-size parity in the benchmark's launch configurations.

Protocol: every env step of the full-size hard workloads is fingerprinted on the
GPU (vcs_hash: FNV-1a 64 of registers, RAM and frame); the oracle runs a sample
of >= 256 envs (>= 4 per ROM for the heterogeneous workload) and the same
fingerprints, computed from its outputs with numpy, must match step by step.
Final states are compared byte for byte for every env (or a 1024-env sample of
the 16384-env workload), and all steps byte for byte for a few envs.  The soft
workload's gradients are checked for every env of 8 of its ROMs."""
import multiprocessing as mp
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import inputs as I
from tests.fnv import fnv1a64

pytestmark = pytest.mark.gpu

# (kernel, lanes per env, threads per workgroup): the shapes the autotuner picks for the batched workload
SHAPES = [("translated", 16, 256), ("translated", 32, 256), ("grouped", 16, 256), ("grouped", 4, 64)]


def say(*a):
    print(*a, flush=True)


def _pool():
    return mp.get_context("fork").Pool(max(1, min(16, os.cpu_count() or 1)))


# --------------------------------------------------------------------------- oracle workers
_W = {}


def _oracle_env(args):
    name, b, mode = args
    w = _W[name]
    rom = w.roms[int(w.env_rom[b])]
    ep = None if w.episode_steps is None else w.episode_steps[b]
    r = O.run_env(rom.image, rom.mapper, w.ram0[b], w.actions[b], w.steps, w.frame_skip, ep_steps=ep, seed=w.seed,
                  env_index=b, frames="all" if mode == "steps" else "none", step_state=mode == "steps")
    if mode == "steps":  # per-step fingerprints of (registers, RAM, frame)
        msgs = np.concatenate([r["step_state"], r["frames"].reshape(w.steps, -1)], axis=1)
        return b, fnv1a64(msgs), None
    regs = np.array([r["regs"][k] for k in O.REG_NAMES[:16]], np.uint8)
    return b, regs, r["ram"][-1]


def oracle_runs(name, w, envs, mode):
    _W[name] = w
    with _pool() as pool:
        return pool.map(_oracle_env, [(name, int(b), mode) for b in envs], chunksize=4)


# --------------------------------------------------------------------------- GPU side
def gpu_step_hashes(w, kernel, G, tpb):
    """Run the whole workload one env step per call; fingerprint every env after every step."""
    import torch
    from paper_2606_22447_amd.vcs import VcsBatch
    vb = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed, kernel=kernel, lanes_per_env=G,
                  block_threads=tpb)
    vb.reset(ram0=w.ram0)
    B, S = w.num_envs, w.steps
    acts = torch.from_numpy(np.ascontiguousarray(w.actions)).cuda()
    eps = None if w.episode_steps is None else torch.from_numpy(w.episode_steps.view(np.int32)).cuda()
    ram_out = torch.empty((B, 1, 128), dtype=torch.uint8, device="cuda")
    frame = torch.empty((B, 210, 160), dtype=torch.uint8, device="cuda")
    done = torch.empty((B, 1), dtype=torch.uint8, device="cuda")
    hashes = torch.empty((S, B), dtype=torch.int64, device="cuda")
    for s in range(S):
        vb.step(acts[:, s:s + 1], frames="last", episode_steps=eps, ram_out=ram_out, frame_out=frame, done=done)
        hashes[s] = vb.hash(frame)
    regs = vb.regs()
    torch.cuda.synchronize()
    return hashes.cpu().numpy().view(np.uint64), regs.cpu().numpy(), ram_out[:, 0].cpu().numpy(), vb


def check_workload(w, sample, final_envs, shapes):
    say(w.name, "oracle: per-step fingerprints of", len(sample), "envs")
    per_step = {b: (h, r) for b, h, r in oracle_runs(w.name, w, sample, "steps")}
    say(w.name, "oracle: final states of", len(final_envs), "envs")
    final = {b: (regs, ram) for b, regs, ram in oracle_runs(w.name, w, final_envs, "final")}
    for kernel, G, tpb in shapes:
        say(w.name, "gpu", kernel, G, tpb)
        h, regs, ram_last, _ = gpu_step_hashes(w, kernel, G, tpb)
        for b in sample:
            bad = np.nonzero(h[:, b] != per_step[b][0])[0]
            assert bad.size == 0, (w.name, kernel, G, tpb, "env", b, "first differing step", int(bad[0]))
        for b in final_envs:
            assert (regs[b] == final[b][0]).all(), (w.name, kernel, G, tpb, "final registers of env", b)
            assert (ram_last[b] == final[b][1]).all(), (w.name, kernel, G, tpb, "final RAM of env", b)


def test_batched_hard_full_size_every_step_fingerprinted():
    w = I.config_c1()  # 4096 envs x 500 env steps, frame-skip 4
    sample = list(range(0, w.num_envs, 16))  # 256 envs
    check_workload(w, sample, list(range(w.num_envs)), SHAPES)


def test_heterogeneous_full_size_every_step_fingerprinted():
    w = I.config_c2()  # 16384 envs over 64 ROMs (2K / 4K / F8), in-run episode resets
    by_rom = [np.nonzero(w.env_rom == r)[0] for r in range(len(w.roms))]
    sample = sorted(int(e) for envs in by_rom for e in envs[:4])       # 4 per ROM = 256
    final_envs = sorted(int(e) for envs in by_rom for e in envs[:16])  # 16 per ROM = 1024
    cum = np.cumsum(w.episode_steps[sample], axis=1)
    assert (cum[:, 0] < w.steps).sum() >= 64  # many sampled envs cross an episode end
    check_workload(w, sample, final_envs, [("grouped", 4, 256), ("translated", 4, 256)])


@pytest.mark.parametrize("kernel,G,tpb", [("translated", 16, 256), ("translated", 32, 256), ("grouped", 16, 256)])
def test_batched_hard_full_size_bytes_of_sampled_envs(kernel, G, tpb):
    """Every RAM byte, frame byte and done flag of a few envs, in bench.py's call pattern (50 steps/call)."""
    import torch
    from paper_2606_22447_amd.vcs import VcsBatch
    w = I.config_c1()
    sample = [0, 1, 777, 2048, 4095]
    vb = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed, kernel=kernel, lanes_per_env=G,
                  block_threads=tpb)
    vb.reset(ram0=w.ram0)
    idx = torch.tensor(sample, device="cuda")
    rams, frs = [], []
    for s0 in range(0, w.steps, 50):
        acts = torch.from_numpy(np.ascontiguousarray(w.actions[:, s0:s0 + 50])).cuda()
        ram, fr, _ = vb.step(acts, frames="all")
        rams.append(ram[idx].cpu().numpy())
        frs.append(fr[idx].cpu().numpy())
    ram, fr = np.concatenate(rams, 1), np.concatenate(frs, 1)
    for i, b in enumerate(sample):
        ref = O.run_env(w.roms[0].image, w.roms[0].mapper, w.ram0[b], w.actions[b], w.steps, w.frame_skip)
        assert (ref["ram"] == ram[i]).all(), b
        assert (ref["frames"] == fr[i]).all(), b


# --------------------------------------------------------------------------- soft
_S = {}


def _soft_env(args):
    r, i = args
    d = _S["data"]
    dec_rom, hr0, ev0, ha, es, ei, w = d["dec_rom"][r], d["hr0"], d["ev0"], d["ha"], d["es"], d["ei"], d["w"]
    b = d["envs"][r][i]
    mapper = w.roms[r].mapper
    tgt = O.run_env(d["pert"][r], mapper, hr0[b], ha[b], w.steps, 1, frames="last")["frames"][0]
    hard = O.run_env(dec_rom[0], mapper, hr0[b], ha[b], w.steps, 1, frames="last")["frames"][0]
    dl = ((hard.astype(np.int64) >> 1) & 7) - ((tgt.astype(np.int64) >> 1) & 7)
    gf = ((2.0 * dl / 33600) * 0.5).astype(np.float32)
    res = O.soft_env(dec_rom[0], dec_rom[1], mapper, hr0[b], ev0[b], ha[b], es[b], ei[b], w.steps, 1, mode="ste",
                     grad_frame=gf.astype(np.float64))
    return r, b, gf, res["g_rom"], res["g_ram0"], res["g_swcha"], res["g_inpt4"], res["ram"], res["frame"]


def test_soft_scale_gradients_of_eight_roms():
    import torch
    from paper_2606_22447_amd.vcs import SoftVcs, VcsBatch
    from tests.test_gpu_soft import assert_grad_close
    w = I.config_c4()  # 4096 envs over 64 ROMs, 60 frames
    lv = I.soft_leaves(w)
    tau = 1.0
    B, S = w.num_envs, w.steps
    offs = w.rom_offsets()
    roms = [0, 9, 21, 30, 42, 51, 60, 63]  # 2K, 4K and F8 images
    hr0, ev0 = O.decode_tape(lv.ram_tape.reshape(-1, 256))
    ha, es, ei = O.decode_actions(lv.action_logits.reshape(-1, 18), tau)
    _S["data"] = {
        "w": w, "pert": lv.perturbed_roms, "hr0": hr0.reshape(B, 128), "ev0": ev0.reshape(B, 128),
        "ha": ha.reshape(B, S), "es": es.reshape(B, S), "ei": ei.reshape(B, S),
        "dec_rom": {r: O.decode_logits(lv.rom_logits[offs[r]:offs[r] + w.roms[r].size], tau) for r in roms},
        "envs": {r: np.nonzero(w.env_rom == r)[0] for r in roms}}
    jobs = [(r, i) for r in roms for i in range(len(_S["data"]["envs"][r]))]
    say("soft oracle:", len(jobs), "envs of ROMs", roms)
    with _pool() as pool:
        out = pool.map(_soft_env, jobs, chunksize=2)
    grad_frame = np.zeros((B, 210, 160), np.float32)
    g_rom = {r: np.zeros(w.roms[r].size) for r in roms}
    g0 = np.zeros((B, 128))
    gsw, gin = np.zeros((B, S)), np.zeros((B, S))
    ref_fwd = {}
    for r, b, gf, gr, g_0, g_s, g_i, ram_o, fr_o in out:
        grad_frame[b] = gf
        g_rom[r] += gr
        g0[b], gsw[b], gin[b] = g_0, g_s, g_i
        ref_fwd[b] = (ram_o, fr_o)
    say("soft gpu fwd+bwd at full size")
    sim = SoftVcs(w.roms, w.env_rom, frame_skip=1, ckpt_interval=1024, lanes_per_env=64)
    L = torch.from_numpy(lv.rom_logits).cuda()
    T = torch.from_numpy(lv.ram_tape).cuda()
    A = torch.from_numpy(lv.action_logits).cuda()
    ram_s, frame_s, residual, _, _ = sim.forward(L, T, A, tau, 6.0)
    g = sim.backward(residual, L, T, A, tau, 6.0, torch.from_numpy(grad_frame).cuda(), check_overflow=True)
    torch.cuda.synchronize()
    got_rom, got_tape, got_act = (x.cpu().numpy() for x in g)
    # forward outputs: every env's RAM after every step and final frame equal the hard kernel's on the
    # decoded leaves (Theorem "Exact forward equivalence"), and the oracle's for the envs of the 8 ROMs
    say("soft forward vs hard kernel, every env")
    dec_all = O.decode_logits(lv.rom_logits, tau)[0]
    imgs = [(dec_all[offs[r]:offs[r] + w.roms[r].size], w.roms[r].mapper) for r in range(len(w.roms))]
    vh = VcsBatch(imgs, w.env_rom, frame_skip=1, kernel="grouped", lanes_per_env=64)
    vh.reset(ram0=_S["data"]["hr0"])
    ram_h, frame_h, _ = vh.step(actions=_S["data"]["ha"], frames="last", want_done=False)
    assert torch.equal(ram_s, ram_h.float()) and torch.equal(frame_s, frame_h.float())
    ram_s, frame_s = ram_s.cpu().numpy(), frame_s.cpu().numpy()
    for b, (ram_o, fr_o) in ref_fwd.items():
        assert (ram_s[b] == ram_o).all() and (frame_s[b] == fr_o).all(), b
    for r in roms:
        o, n = offs[r], w.roms[r].size
        assert_grad_close(got_rom[o:o + n], O.epilogue_rom(lv.rom_logits[o:o + n], tau, g_rom[r]), f"rom {r}")
        envs = _S["data"]["envs"][r]
        assert_grad_close(got_tape[envs], O.epilogue_tape(g0[envs].reshape(-1)).reshape(len(envs), 128, 256),
                          f"ram_tape of rom {r}")
        ref_act = O.epilogue_action(lv.action_logits[envs].reshape(-1, 18), tau, gsw[envs].reshape(-1),
                                    gin[envs].reshape(-1)).reshape(len(envs), S, 18)
        assert_grad_close(got_act[envs], ref_act, f"action_logits of rom {r}")
    # every other env got a zero frame gradient: its leaves' gradients are exactly zero
    others = np.nonzero(~np.isin(w.env_rom, roms))[0][:256]
    assert (got_tape[others] == 0).all() and (got_act[others] == 0).all()
