#!/usr/bin/env python3
"""Throughput of batched Atari VCS emulation on one MI355X; prints one JSON line.

Timed step = one vcs_step_hard call of --chunk env steps for all envs of the
batched hard-forward workload (4096 envs of one seed-generated 4 KB ROM,
frame-skip 4, uniform joystick actions, RAM + frame written for every step);
--steps calls cover the 2000-frame run.  The same run also measures the plain
one-env-per-thread kernel, the heterogeneous persistent workload (64 ROMs x
256 envs with in-run episode resets), the soft forward+backward at scale and
the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/sec (hard fwd; soft fwd+bwd) at B envs, bit-exact vs oracle"
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # int32 lane-ops/s: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
OPS_PER_INSTRUCTION = 12                       # algorithmic integer ops of one emulated 6507 instruction
OPS_PER_PIXEL = 1                              # one store per returned pixel
OPS_PER_SWEEP = 6                              # reverse-sweep ops of one emulated instruction (soft backward)


PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "vcs_tr_step_c1_hbm_traffic.md")
HBM_PEAK_GBPS = 8000.0                         # MI355X HBM3E
SIMDS, CLOCK_HZ = 1024, 2.4e9                  # 256 CUs x 4 SIMDs; a wave64 VALU instruction takes 4 cycles
KERNEL_SOURCES = ["vcs_core.hpp", "vcs_paths.hpp", "vcs_internal.hpp", "vcs_kernels.hpp", "vcs_kernels.hip",
                  "vcs_device.hpp", "vcs_jit.hpp", "vcs_jit.cpp", "vcs_step_kernels.hpp", "vcs_step_hard.hip",
                  "vcs_step_soft.hip", "vcs_step_soft_obj.hip", "vcs_step_soft_tape.hip",
                  "vcs_step_soft_tape_obj.hip", "vcs_step_relaxed.hip", "vcs_step_hard_obj.hip"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_digest() -> str:
    """SHA-256 of the step kernel's sources and build flags (identifies the measured kernel)."""
    import hashlib
    from paper_2606_22447_amd import build as B
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(B.CSRC, f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(f for f in B.FLAGS if not os.path.isabs(f)).encode())  # flags without local paths
    return h.hexdigest()[:16]


def profile_figures(name: str):
    """The machine-readable figures (``key: value`` lines) of a committed rocprofv3
    summary under profiles/, or None when the kernel has changed since they were taken."""
    try:
        with open(os.path.join(PROFILES, name)) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    kv = {}
    for line in lines:
        k, sep, v = line.partition(": ")
        if sep and k.strip() == k and k.replace("_", "").isalnum() and " " not in v.strip():
            kv[k] = v.strip()
    if kv.get("kernel_digest") != kernel_digest():
        return None
    out = {"_file": "profiles/" + name}
    for k, v in kv.items():
        try:
            out[k] = float(v) if k != "kernel_digest" else v
        except ValueError:
            out[k] = v
    return out


def counter_fractions(fig, prefix: str, launch_s: float):
    """VALU-issue fraction of a kernel from committed counters (instructions per launch,
    scaled to this run's launch time): SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x clock x t),
    and the measured lane utilisation."""
    if not fig or f"{prefix}_sq_insts_valu_per_launch" not in fig or not launch_s:
        return None
    valu = fig[f"{prefix}_sq_insts_valu_per_launch"]
    issue = valu * 4.0 / (SIMDS * CLOCK_HZ * launch_s)
    out = {"source": "rocprofv3 SQ counters, " + fig.get("_file", ""), "sq_insts_valu_per_launch": valu,
           "valu_issue_frac": issue}
    for k in ("sq_insts_salu", "sq_insts_lds", "sq_insts_branch", "sq_insts_mfma", "sq_waves"):
        if f"{prefix}_{k}_per_launch" in fig:
            out[f"{k}_per_launch"] = fig[f"{prefix}_{k}_per_launch"]
    for k in ("valu_busy_pct", "valu_utilization_pct"):
        if f"{prefix}_{k}" in fig:
            out[k] = fig[f"{prefix}_{k}"]
    if "valu_utilization_pct" in out:
        out["valu_lane_op_frac"] = issue * out["valu_utilization_pct"] / 100.0
    return out


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None
    when the kernel has changed since those counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.split(":", 1) for line in fh.read().splitlines() if line.startswith("- ") is False
                      and ":" in line and line.split(":", 1)[0].strip().isidentifier())
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_digest") != kernel_digest():
        return None
    try:
        return int(kv["fetch_bytes_per_launch"]) + int(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed calls")
    ap.add_argument("--warmup", type=int, default=2, help="untimed calls")
    ap.add_argument("--chunk", type=int, default=50, help="env steps per call")
    ap.add_argument("--envs", type=int, default=4096)
    ap.add_argument("--kernel", default="translated", help="step kernel of the hard leg: translated, grouped, plain")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--tpb", type=int, default=0)
    ap.add_argument("--legs", default="hard,grouped,plain,hetero,objects,soft,cpu",
                    help="comma list of: hard, grouped, plain, hetero, objects, soft, cpu")
    ap.add_argument("--soft-k", default="256,1024,4096,1024t",
                    help="checkpoint intervals K of the soft leg; a trailing t: the forward also keeps its tape")
    ap.add_argument("--soft-passes", type=int, default=2)
    ap.add_argument("--soft-warmup", type=int, default=1)
    ap.add_argument("--soft-lanes", type=int, default=0, help="lanes per env of the soft forward (0 = auto)")
    ap.add_argument("--hetero-lanes", type=int, default=0, help="lanes per env of the heterogeneous leg (0 = auto)")
    ap.add_argument("--hetero-tpb", type=int, default=256)
    ap.add_argument("--hetero-kernel", default="grouped", help="step kernel of the heterogeneous leg")
    ap.add_argument("--hetero-calls", type=int, default=4, help="timed calls of 25 env steps")
    ap.add_argument("--hetero-warmup", type=int, default=1)
    ap.add_argument("--objects-lanes", type=int, default=0, help="lanes per env of the sprite leg (0 = auto)")
    ap.add_argument("--objects-tpb", type=int, default=256)
    ap.add_argument("--objects-calls", type=int, default=4, help="timed calls of 25 env steps")
    ap.add_argument("--cpu-soft-envs", type=int, default=256,
                    help="envs of the small soft workload in the single-core FP64 fwd+bwd oracle sample")
    ap.add_argument("--copy-probe", action="store_true", help="also run a plain device copy of known size")
    ap.add_argument("--no-graph", action="store_true",
                    help="time direct vcs_step_hard calls instead of replays of a captured HIP graph")
    return ap.parse_args()


def timed_calls(fn, warmup, steps):
    import torch
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record()
        fn(warmup + i)
        ev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) for a, b in ev]) / 1e3
    return wall, per


def instructions_per_step(w, envs=2, steps=4, stride=1):
    """Oracle-counted 6507 instructions per env step of this workload (sample of
    `envs` envs, every `stride`-th, over their first `steps` steps)."""
    from oracle import oracle as O
    tot = 0
    for b in range(0, envs * stride, stride):
        rom = w.roms[int(w.env_rom[b])]
        r = O.run_env(rom.image, rom.mapper, w.ram0[b], w.actions_or_noop()[b, :steps], steps, w.frame_skip,
                      frames="none")
        tot += r["instructions"]
    return tot / (envs * steps)


def hard_leg(args, kernel, lanes, tpb, w, check=True):
    import torch
    from paper_2606_22447_amd.vcs import VcsBatch
    B, C = w.num_envs, args.chunk
    vb = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed, kernel=kernel, lanes_per_env=lanes,
                  block_threads=tpb)
    vb.reset(ram0=w.ram0)
    ncalls = args.warmup + args.steps
    acts = [torch.from_numpy(np.ascontiguousarray(w.actions[:, i * C:(i + 1) * C])).cuda() for i in range(ncalls)]
    eps = None if w.episode_steps is None else torch.from_numpy(w.episode_steps.view(np.int32)).cuda()
    first = {}
    if getattr(args, "no_graph", False):
        ram_out = torch.empty((B, C, 128), dtype=torch.uint8, device="cuda")
        frame_out = torch.empty((B, C, 210, 160), dtype=torch.uint8, device="cuda")
        done = torch.empty((B, C), dtype=torch.uint8, device="cuda")

        def run(i):
            vb.step(acts[i], frames="all", episode_steps=eps, ram_out=ram_out, frame_out=frame_out, done=done)
    else:
        # one captured call of C env steps, replayed with the next actions copied into its input buffer
        act_buf = acts[0].clone()
        graph, ram_out, frame_out, done = vb.capture(act_buf, frames="all", episode_steps=eps)

        def run(i):
            act_buf.copy_(acts[i])
            graph.replay()

    def call(i):
        run(i)
        if i == 0 and check:
            torch.cuda.synchronize()
            first["ram"] = ram_out[:2].cpu().numpy()
            first["frames"] = frame_out[:2].cpu().numpy()

    wall, per = timed_calls(call, args.warmup, args.steps)
    parity = None
    if check:
        from oracle import oracle as O
        parity = "ok"
        for b in range(2):
            rom = w.roms[int(w.env_rom[b])]
            ep = None if w.episode_steps is None else w.episode_steps[b]
            ref = O.run_env(rom.image, rom.mapper, w.ram0[b], w.actions[b, :C], C, w.frame_skip, ep_steps=ep,
                            seed=w.seed, env_index=b)
            if not ((ref["ram"] == first["ram"][b]).all() and (ref["frames"] == first["frames"][b]).all()):
                parity = f"MISMATCH env {b}"
    info = vb.info()
    steps_done = B * C * args.steps
    return {"env_steps_per_s": steps_done / per.sum(), "wall_env_steps_per_s": steps_done / wall,
            "ms_per_call": float(per.mean() * 1e3), "ms_per_call_std": float(per.std() * 1e3),
            "env_steps": steps_done, "parity_sample": parity, "launch": info, "translation": vb.translation,
            "timing": "HIP events around direct calls" if getattr(args, "no_graph", False)
            else "HIP events around replays of a captured HIP graph (action refill + replay)"}


def soft_leg(args):
    import torch
    from paper_2606_22447_amd import binding as Bd
    from paper_2606_22447_amd import inputs as I
    from paper_2606_22447_amd.vcs import SoftVcs, VcsBatch, soft_rollout, ste_luminance
    w = I.config_c4()
    B, S = w.num_envs, w.steps
    log("soft: generating leaves")
    lv = I.soft_leaves(w)
    # target frames: hard run of the perturbed ROMs on the same hard inputs (setup, untimed)
    pert = [(img, r.mapper) for img, r in zip(lv.perturbed_roms, w.roms)]
    tb = VcsBatch(pert, w.env_rom, frame_skip=1)
    tb.reset(ram0=w.ram0)
    act_hard = torch.from_numpy(w.actions).cuda()
    _, target, _ = tb.step(act_hard, frames="last", want_done=False)
    lum_t = ((target.to(torch.int32) >> 1) & 7).float()
    L = torch.from_numpy(lv.rom_logits).cuda().requires_grad_()
    T = torch.from_numpy(lv.ram_tape).cuda().requires_grad_()
    A = torch.from_numpy(lv.action_logits).cuda().requires_grad_()
    out = {"workload": "c4_soft_scale: 64 ROMs (21x2K, 22x4K, 21xF8) x 64 envs = 4096 envs, 60 frames, "
                       "frame-skip 1, FP32 ROM logits/RAM tape/action logits, tau 1.0, alpha 6",
           "env_steps_per_pass": B * S, "by_ckpt_interval": {}}
    lanes = args.soft_lanes
    if lanes == 0:  # autotune the soft forward's lanes per env on a short trial of this workload
        from paper_2606_22447_amd import autotune
        tuned = autotune.tune_soft(w.roms, w.env_rom, L.detach(), T.detach(), A.detach(), 1.0, 6.0,
                                   trial_steps=6, ckpt=(1024,))
        lanes = tuned["lanes_per_env"]
        out["autotune"] = {"lanes_per_env": lanes,
                           "trials": [(r["lanes_per_env"], round(r["env_steps_per_s"])) for r in tuned["table"]]}
        log("soft autotune", out["autotune"])
    out["lanes_per_env"] = lanes
    for key in args.soft_k.split(","):
        K, tape = int(key.rstrip("t")), key.endswith("t")
        sim = SoftVcs(w.roms, w.env_rom, frame_skip=1, ckpt_interval=K, lanes_per_env=lanes,
                      tape_records=-1 if tape else 0)
        marks = []

        def one(_i):
            L.grad = T.grad = A.grad = None
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
            ram, frame = soft_rollout(sim, L, T, A, 1.0, 6.0)
            loss = ((ste_luminance(frame) - lum_t) ** 2).mean(dim=(1, 2)).sum()
            ev[1].record()
            loss.backward()
            ev[2].record()
            marks.append(ev)

        torch.cuda.reset_peak_memory_stats()
        wall, per = timed_calls(one, args.soft_warmup, args.soft_passes)
        sim.raise_if_overflowed()
        timed = marks[args.soft_warmup:]
        fwd_s = float(np.mean([a.elapsed_time(b) for a, b, _ in timed])) / 1e3
        bwd_s = float(np.mean([b.elapsed_time(c) for _, b, c in timed])) / 1e3
        res_b = Bd.size_query("vcs_residual_bytes", sim.h, S)
        ws_b = Bd.size_query("vcs_workspace_bytes", sim.h, Bd.VCS_OP_SOFT_BWD, S)
        out["by_ckpt_interval"][key] = {
            "forward_tape": tape,
            "env_steps_per_s": B * S / per.mean(), "ms_per_pass": float(per.mean() * 1e3),
            "ms_forward": fwd_s * 1e3, "ms_backward": bwd_s * 1e3,
            "residual_bytes_per_env": res_b / B, "bwd_workspace_bytes_per_env": ws_b / B,
            "peak_mem_bytes_per_env": torch.cuda.max_memory_allocated() / B}
        del sim
    best = max(out["by_ckpt_interval"].items(), key=lambda kv: kv[1]["env_steps_per_s"])
    out["best_ckpt_interval"] = best[0]
    out["env_steps_per_s"] = best[1]["env_steps_per_s"]
    out["instructions_per_env_step"] = instructions_per_step(w, envs=8, steps=6, stride=B // 8)
    out["instructions_per_s"] = out["env_steps_per_s"] * out["instructions_per_env_step"]
    # roofline of the pass: forward (12 ops per instruction) and reverse sweep (6: record read, class
    # decode, two adjoint multiply-adds, two adjoint moves), plus the returned frame drawn in the
    # forward and its pixel gradients summed in the backward; recomputing checkpoint segments is
    # re-execution, not algorithmic work
    ops = out["instructions_per_env_step"] * (OPS_PER_INSTRUCTION + OPS_PER_SWEEP) + 2 * 33600 / S
    achieved = out["env_steps_per_s"] * ops / 1e12
    fig = profile_figures("soft_c4_sq_counters.md")
    bk = best[1]
    out["roofline"] = {
        "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
        "frac": achieved / VALU_PEAK_TOPS, "ops_per_env_step": ops,
        "ops_model": f"{OPS_PER_INSTRUCTION + OPS_PER_SWEEP} integer ops per emulated instruction "
                     "(forward 12, sweep 6; recomputation not counted) + 2 per returned pixel",
        "kernel": ("k_step<soft> keeping its tape (dominant) and k_soft_bwd sweeping it" if bk.get("forward_tape")
                   else "k_soft_bwd (dominant: recompute and sweep) and k_step<soft>"),
        "k_soft_bwd": counter_fractions(fig, "k_soft_bwd", bk["ms_backward"] / 1e3),
        "k_step_soft": counter_fractions(fig, "k_step_soft", bk["ms_forward"] / 1e3),
        "timing": "HIP events on the current stream around the forward (autograd forward + loss) and the "
                  "backward (loss backward + vcs_step_soft_bwd) of each timed pass"}
    return out


def _cpu_worker(args):
    from oracle import oracle as O
    from paper_2606_22447_amd import inputs as I
    envs, steps = args
    w = I.config_c1(num_envs=max(envs) + 1, steps=steps)
    t0 = time.perf_counter()
    instr = 0
    for b in envs:
        r = O.run_env(w.roms[0].image, w.roms[0].mapper, w.ram0[b], w.actions[b], steps, w.frame_skip)
        instr += r["instructions"]
    return time.perf_counter() - t0, len(envs) * steps, instr


def _cpu_soft_worker(args):
    """Single-core FP64 soft forward + backward of the oracle on envs of the small soft workload
    (leaf decode, then per env the soft rollout with its reverse sweep), `reps` times."""
    from oracle import oracle as O
    from paper_2606_22447_amd import inputs as I
    n_envs, tau, reps = args
    w = I.config_c3()
    lv = I.soft_leaves(w)
    B, S = w.num_envs, w.steps
    gf = np.full((210, 160), 1e-4)
    t0 = time.perf_counter()
    for _ in range(reps):
        dr = O.decode_logits(lv.rom_logits, tau)
        hr0, ev0 = O.decode_tape(lv.ram_tape[:n_envs].reshape(-1, 256))
        ha, es, ei = O.decode_actions(lv.action_logits[:n_envs].reshape(-1, 18), tau)
        for b in range(n_envs):
            O.soft_env(dr[0], dr[1], w.roms[0].mapper, hr0.reshape(-1, 128)[b], ev0.reshape(-1, 128)[b],
                       ha.reshape(-1, S)[b], es.reshape(-1, S)[b], ei.reshape(-1, S)[b], S, 1, mode="ste",
                       grad_frame=gf)
    return time.perf_counter() - t0, reps * n_envs * S


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(envs_per_proc=4, steps=500, soft_envs=16):
    import multiprocessing as mp
    from oracle import build as obuild
    obuild.build(force=False)
    nproc = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = nproc
    # one process per usable core, at most 16 (the share of one GPU's host cores on the GPU machines)
    cores = max(1, min(usable, 16))
    jobs = [list(range(i * envs_per_proc, (i + 1) * envs_per_proc)) for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(j, steps) for j in jobs])
    wall = time.perf_counter() - t0
    n = sum(r[1] for r in res)
    cpu_s = sum(r[0] for r in res)
    soft_reps = 10
    with mp.get_context("fork").Pool(1) as pool:  # the soft oracle on one core
        soft_s, soft_n = pool.map(_cpu_soft_worker, [(soft_envs, 1.0, soft_reps)])[0]
    return {"value": n / wall, "unit": "env-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"batched hard-forward workload, {cores} processes x {envs_per_proc} envs x {steps} env steps "
                      f"(frame-skip 4, every frame rendered and stored), {cpu_s:.1f} s of CPU work",
            "nproc": nproc, "usable_cores": usable, "process_cap": 16, "cpu_model": cpu_model(),
            "single_core_env_steps_per_s": n / cpu_s, "instructions_per_s": sum(r[2] for r in res) / wall,
            "soft_fp64_fwd_bwd_single_core": {
                "env_steps_per_s": soft_n / soft_s, "seconds": soft_s,
                "sample": f"small soft workload (1 ROM, frame-skip 1): {soft_envs} envs x 2 env steps, FP64 "
                          f"SOFT-STE forward + reverse sweep + leaf decode, tau 1.0, one process, {soft_reps} "
                          "repetitions"}}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: every env is independent and this build measures one MI355X; "
              "multi-GPU sharding is described in DESIGN.md but not run", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2606_22447_amd import binding
    binding.lib()  # fails loudly if the HIP library is not built
    from paper_2606_22447_amd import inputs as I

    legs = set(args.legs.split(","))
    total_steps = args.chunk * (args.warmup + args.steps)
    w1 = I.config_c1(num_envs=args.envs, steps=total_steps)
    log(f"c1: {args.envs} envs x {total_steps} env steps")
    ips = instructions_per_step(w1)
    result = {}
    tuned = {}
    if "hard" in legs:
        lanes, tpb = args.lanes, args.tpb
        if lanes == 0 and args.kernel in ("grouped", "translated"):  # autotune the launch shape on this workload
            from paper_2606_22447_amd import autotune
            t = autotune.tune_hard(w1.roms, w1.env_rom, frame_skip=w1.frame_skip, seed=w1.seed, ram0=w1.ram0,
                                   actions=w1.actions, trial_steps=2, kernel=args.kernel)
            lanes, tpb = t["lanes_per_env"], t["block_threads"]
            tuned["hard"] = [(r["lanes_per_env"], r["block_threads"], round(r["env_steps_per_s"])) for r in t["table"]]
            log("hard autotune", tuned["hard"])
        result["hard"] = hard_leg(args, args.kernel, lanes, tpb, w1)
        log("hard", result["hard"])
    if "grouped" in legs:  # the interpreting kernel on the same workload
        ga = argparse.Namespace(**vars(args))
        ga.steps, ga.warmup = max(1, min(args.steps, 3)), 1
        result["grouped"] = hard_leg(ga, "grouped", 16, 256, w1, check=False)
        log("grouped", result["grouped"])
    if "plain" in legs:
        pa = argparse.Namespace(**vars(args))
        pa.steps, pa.warmup = max(1, min(args.steps, 3)), 1
        result["plain"] = hard_leg(pa, "plain", 1, 256, w1, check=False)
        log("plain", result["plain"])
    if "hetero" in legs:
        ha = argparse.Namespace(**vars(args))
        ha.chunk, ha.steps, ha.warmup = 25, args.hetero_calls, args.hetero_warmup
        w2 = I.config_c2(steps=25 * (args.hetero_calls + args.hetero_warmup))
        # the interpreting kernel: these ROMs read the joystick, so envs of a wave diverge and the
        # translated code (which needs every lane of a wave at one block) mostly falls back to it
        hl, ht = args.hetero_lanes, args.hetero_tpb
        if hl == 0:
            from paper_2606_22447_amd import autotune
            t = autotune.tune_hard(w2.roms, w2.env_rom, frame_skip=w2.frame_skip, seed=w2.seed, ram0=w2.ram0,
                                   actions=w2.actions, trial_steps=2)
            tuned["hetero"] = [(r["lanes_per_env"], r["block_threads"], round(r["env_steps_per_s"]))
                               for r in t["table"]]
            log("hetero autotune", tuned["hetero"])
            hl, ht = t["lanes_per_env"], t["block_threads"]
        result["hetero"] = hard_leg(ha, args.hetero_kernel, hl, ht, w2)
        result["hetero"]["instructions_per_env_step"] = instructions_per_step(w2, envs=8, steps=4,
                                                                              stride=w2.num_envs // 8)
        result["hetero"]["workload"] = ("c2_hetero_persistent: 64 ROMs (21x2K, 22x4K, 21xF8, reading SWCHA/INPT4/"
                                        "INTIM) x 256 envs = 16384 envs, frame-skip 4, geometric episodes "
                                        "(mean 1500 frames) with in-run resets")
        log("hetero", result["hetero"])
    if "objects" in legs:
        oa = argparse.Namespace(**vars(args))
        oa.chunk, oa.steps, oa.warmup = 25, args.objects_calls, 1
        w5 = I.config_objects(envs_per_rom=256, steps=25 * (args.objects_calls + 1), n_roms=16)
        ol, ot = args.objects_lanes, args.objects_tpb
        if ol == 0:
            from paper_2606_22447_amd import autotune
            t = autotune.tune_hard(w5.roms, w5.env_rom, frame_skip=w5.frame_skip, seed=w5.seed, ram0=w5.ram0,
                                   actions=w5.actions, trial_steps=2)
            tuned["objects"] = [(r["lanes_per_env"], r["block_threads"], round(r["env_steps_per_s"]))
                                for r in t["table"]]
            log("objects autotune", tuned["objects"])
            ol, ot = t["lanes_per_env"], t["block_threads"]
        result["objects"] = hard_leg(oa, "grouped", ol, ot, w5)
        result["objects"]["instructions_per_env_step"] = instructions_per_step(w5, envs=8, steps=4,
                                                                               stride=w5.num_envs // 8)
        result["objects"]["workload"] = ("objects: 16 seed-generated sprite kernels (4x2K, 12x4K: players, "
                                         "missiles, ball, HMOVE, collisions read every frame, P0 moved by the "
                                         "joystick) x 256 envs = 4096 envs, frame-skip 4, RAM and frame every step")
        log("objects", result["objects"])
    if "soft" in legs:
        result["soft"] = soft_leg(args)
        log("soft", result["soft"])
    if args.copy_probe:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    cpu = cpu_leg(soft_envs=args.cpu_soft_envs) if "cpu" in legs else None

    h = result.get("hard")
    value = h["env_steps_per_s"] if h else None
    ops_per_step = ips * OPS_PER_INSTRUCTION + 33600 * OPS_PER_PIXEL
    timed_steps = args.chunk * args.steps
    line = {
        "metric": METRIC, "value": value, "unit": "env-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": h["ms_per_call"] if h else None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"c1_batched_hard: {args.envs} envs of one seed-generated 4 KB ROM, uniform actions "
                               "over the 18 ALE actions, frame-skip 4, RAM (128 B) and frame (210x160 u8) written "
                               f"for every env step; each timed call = {args.chunk} env steps, {args.steps} timed "
                               f"calls = {timed_steps} env steps ({4 * timed_steps} frames) per env after "
                               f"{args.chunk * args.warmup} warm-up env steps",
                   "envs": args.envs, "env_steps_per_call": args.chunk, "frame_skip": 4,
                   "launch": h["launch"] if h else None},
    }
    if h:
        launch_s = h["ms_per_call"] / 1e3
        achieved = h["env_steps_per_s"] * ops_per_step / 1e12
        alg_bytes = args.envs * args.chunk * (33600 + 128 + 1 + 1)
        kname = {"translated": "vcs_tr_step", "grouped": "k_step_grouped", "plain": "k_step_plain"}[args.kernel]
        line["roofline"] = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                            "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(),
                            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                            "algorithmic_bytes_per_launch": alg_bytes,
                            "ops_per_env_step": ops_per_step, "instructions_per_env_step": ips,
                            "ops_model": f"{OPS_PER_INSTRUCTION} integer ops per emulated 6507 instruction (opcode "
                                         "fetch, operand fetch, decode, address, bus decode, access, ALU, N/Z, C/V, "
                                         "PC, cycles, loop test) + 1 store per returned pixel: an algorithmic model",
                            "kernel": {"translated": "vcs_tr_step (translated)", "grouped": "k_step (grouped)",
                                       "plain": "k_step (plain)"}[args.kernel],
                            "valu_issue": counter_fractions(profile_figures(f"{kname}_c1_sq_counters.md"), kname,
                                                            launch_s),
                            "hbm": {"achieved_GBps": alg_bytes / launch_s / 1e9, "peak_GBps": HBM_PEAK_GBPS,
                                    "frac": alg_bytes / launch_s / 1e9 / HBM_PEAK_GBPS,
                                    "note": "algorithmic bytes (frames, RAM, done, actions) per launch / launch time"}}
        line["instructions_per_s"] = h["env_steps_per_s"] * ips
        line["frames_per_s"] = h["env_steps_per_s"] * 4
        line["parity_sample"] = h["parity_sample"]
        line["timing"] = h["timing"]
        line["ms_per_step_std"] = h["ms_per_call_std"]
    if "plain" in result and h:
        line["plain_kernel"] = {"env_steps_per_s": result["plain"]["env_steps_per_s"],
                                "speedup_of_hard_leg": h["env_steps_per_s"] / result["plain"]["env_steps_per_s"]}
    if "grouped" in result and h:
        line["grouped_kernel"] = {"env_steps_per_s": result["grouped"]["env_steps_per_s"],
                                  "speedup_of_hard_leg": h["env_steps_per_s"] / result["grouped"]["env_steps_per_s"]}
    if h and h.get("translation"):
        line["translation"] = h["translation"]
    if "hetero" in result:
        r2 = result["hetero"]
        line["hetero"] = {k: r2[k] for k in ("env_steps_per_s", "ms_per_call", "parity_sample", "workload", "launch",
                                             "instructions_per_env_step")}
        ips2 = r2["instructions_per_env_step"]
        ops2 = ips2 * OPS_PER_INSTRUCTION + 33600 * OPS_PER_PIXEL
        ach2 = r2["env_steps_per_s"] * ops2 / 1e12
        line["hetero"]["instructions_per_s"] = r2["env_steps_per_s"] * ips2
        line["hetero"]["roofline"] = {
            "bound": "alu", "achieved": ach2, "peak": VALU_PEAK_TOPS, "unit": "Tops/s", "frac": ach2 / VALU_PEAK_TOPS,
            "ops_per_env_step": ops2, "kernel": "k_step (grouped, heterogeneous)",
            "valu_issue": counter_fractions(profile_figures("k_step_c2_hetero_sq_counters.md"), "k_step_hetero",
                                            r2["ms_per_call"] / 1e3)}
    if "objects" in result:
        r5 = result["objects"]
        line["objects"] = {k: r5[k] for k in ("env_steps_per_s", "ms_per_call", "parity_sample", "workload", "launch",
                                              "instructions_per_env_step")}
        ips5 = r5["instructions_per_env_step"]
        ops5 = ips5 * OPS_PER_INSTRUCTION + 33600 * OPS_PER_PIXEL
        ach5 = r5["env_steps_per_s"] * ops5 / 1e12
        line["objects"]["instructions_per_s"] = r5["env_steps_per_s"] * ips5
        line["objects"]["roofline"] = {
            "bound": "alu", "achieved": ach5, "peak": VALU_PEAK_TOPS, "unit": "Tops/s", "frac": ach5 / VALU_PEAK_TOPS,
            "ops_per_env_step": ops5, "kernel": "k_step (grouped, sprite workload)",
            "valu_issue": counter_fractions(profile_figures("k_step_objects_sq_counters.md"), "k_step_objects",
                                            r5["ms_per_call"] / 1e3)}
    if tuned:
        line["autotune"] = {k: {"trials (lanes_per_env, block_threads, env_steps_per_s)": v}
                            for k, v in tuned.items()}
    if "soft" in result:
        line["soft_fwd_bwd"] = result["soft"]
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
