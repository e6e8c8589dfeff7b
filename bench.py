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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "vcs_tr_step_c1_hbm_traffic.md")
KERNEL_SOURCES = ["vcs_core.hpp", "vcs_paths.hpp", "vcs_internal.hpp", "vcs_kernels.hpp", "vcs_kernels.hip",
                  "vcs_device.hpp", "vcs_jit.hpp", "vcs_jit.cpp"]


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
    ap.add_argument("--legs", default="hard,grouped,plain,hetero,soft,cpu",
                    help="comma list of: hard, plain, hetero, soft, cpu")
    ap.add_argument("--soft-k", default="256,1024,4096")
    ap.add_argument("--soft-passes", type=int, default=2)
    ap.add_argument("--soft-lanes", type=int, default=0, help="lanes per env of the soft forward (0 = auto)")
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


def instructions_per_step(w, envs=2, steps=4):
    """Oracle-counted 6507 instructions per env step of this workload (sample)."""
    from oracle import oracle as O
    tot = 0
    for b in range(envs):
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
    for K in [int(k) for k in args.soft_k.split(",")]:
        sim = SoftVcs(w.roms, w.env_rom, frame_skip=1, ckpt_interval=K, lanes_per_env=lanes)

        def one(_i):
            L.grad = T.grad = A.grad = None
            ram, frame = soft_rollout(sim, L, T, A, 1.0, 6.0)
            loss = ((ste_luminance(frame) - lum_t) ** 2).mean(dim=(1, 2)).sum()
            loss.backward()

        torch.cuda.reset_peak_memory_stats()
        wall, per = timed_calls(one, 1, args.soft_passes)
        res_b = Bd.size_query("vcs_residual_bytes", sim.h, S)
        ws_b = Bd.size_query("vcs_workspace_bytes", sim.h, Bd.VCS_OP_SOFT_BWD, S)
        out["by_ckpt_interval"][str(K)] = {
            "env_steps_per_s": B * S / per.mean(), "ms_per_pass": float(per.mean() * 1e3),
            "residual_bytes_per_env": res_b / B, "bwd_workspace_bytes_per_env": ws_b / B,
            "peak_mem_bytes_per_env": torch.cuda.max_memory_allocated() / B}
        del sim
    best = max(out["by_ckpt_interval"].items(), key=lambda kv: kv[1]["env_steps_per_s"])
    out["best_ckpt_interval"] = int(best[0])
    out["env_steps_per_s"] = best[1]["env_steps_per_s"]
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


def cpu_leg(envs_per_proc=4, steps=500):
    import multiprocessing as mp
    from oracle import build as obuild
    obuild.build(force=False)
    cores = min(os.cpu_count() or 1, 16)
    jobs = [list(range(i * envs_per_proc, (i + 1) * envs_per_proc)) for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(j, steps) for j in jobs])
    wall = time.perf_counter() - t0
    n = sum(r[1] for r in res)
    cpu_s = sum(r[0] for r in res)
    return {"value": n / wall, "unit": "env-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"batched hard-forward workload, {cores} processes x {envs_per_proc} envs x {steps} env steps "
                      f"(frame-skip 4, every frame rendered and stored), {cpu_s:.1f} s of CPU work",
            "single_core_env_steps_per_s": n / cpu_s, "instructions_per_s": sum(r[2] for r in res) / wall}


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
        ha.chunk, ha.steps, ha.warmup = 25, 4, 1
        w2 = I.config_c2(steps=25 * 5)
        from paper_2606_22447_amd import autotune
        # the interpreting kernel: these ROMs read the joystick, so envs of a wave diverge and the
        # translated code (which needs every lane of a wave at one block) mostly falls back to it
        t = autotune.tune_hard(w2.roms, w2.env_rom, frame_skip=w2.frame_skip, seed=w2.seed, ram0=w2.ram0,
                               actions=w2.actions, trial_steps=2)
        tuned["hetero"] = [(r["lanes_per_env"], r["block_threads"], round(r["env_steps_per_s"])) for r in t["table"]]
        log("hetero autotune", tuned["hetero"])
        result["hetero"] = hard_leg(ha, "grouped", t["lanes_per_env"], t["block_threads"], w2)
        result["hetero"]["workload"] = ("c2_hetero_persistent: 64 ROMs (21x2K, 22x4K, 21xF8, reading SWCHA/INPT4/"
                                        "INTIM) x 256 envs = 16384 envs, frame-skip 4, geometric episodes "
                                        "(mean 1500 frames) with in-run resets")
        log("hetero", result["hetero"])
    if "soft" in legs:
        result["soft"] = soft_leg(args)
        log("soft", result["soft"])
    if args.copy_probe:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    cpu = cpu_leg() if "cpu" in legs else None

    h = result.get("hard")
    value = h["env_steps_per_s"] if h else None
    ops_per_step = ips * OPS_PER_INSTRUCTION + 33600 * OPS_PER_PIXEL
    line = {
        "metric": METRIC, "value": value, "unit": "env-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": h["ms_per_call"] if h else None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "c1_batched_hard: 4096 envs of one seed-generated 4 KB ROM, uniform actions over "
                               "the 18 ALE actions, frame-skip 4, 2000 frames = 500 env steps, RAM (128 B) and "
                               "frame (210x160 u8) written for every env step",
                   "envs": args.envs, "env_steps_per_call": args.chunk, "frame_skip": 4,
                   "launch": h["launch"] if h else None},
    }
    if h:
        achieved = h["env_steps_per_s"] * ops_per_step / 1e12
        line["roofline"] = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                            "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(),
                            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                            "algorithmic_bytes_per_launch": args.envs * args.chunk * (33600 + 128 + 1 + 1),
                            "ops_per_env_step": ops_per_step, "instructions_per_env_step": ips,
                            "kernel": {"translated": "vcs_tr_step (translated)", "grouped": "k_step (grouped)",
                                       "plain": "k_step (plain)"}[args.kernel]}
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
        line["hetero"] = {k: result["hetero"][k] for k in ("env_steps_per_s", "ms_per_call", "parity_sample",
                                                           "workload", "launch")}
    if tuned:
        line["autotune"] = {k: {"trials (lanes_per_env, block_threads, env_steps_per_s)": v}
                            for k, v in tuned.items()}
    if "soft" in result:
        line["soft_fwd_bwd"] = result["soft"]
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
