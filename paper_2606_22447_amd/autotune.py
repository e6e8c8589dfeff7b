"""Launch-shape and checkpoint-interval autotuner.

The step kernels are latency-bound: every env is a serial chain of emulated
instructions, so throughput depends on how envs share wavefronts.  Lockstep
envs (one ROM, same control flow) gain from sharing a wave (one instruction
stream serves several envs), while envs whose control flow diverges (inputs,
different RAM) serialise inside a shared wave and gain from one env per wave.
The best lanes-per-env therefore depends on the workload, and is measured: each
candidate runs a short trial of the caller's own workload on the GPU, timed
with events on the current stream, and the fastest is kept.

For the soft path the checkpoint interval K trades residual memory
(cycles / K checkpoints per env) against recompute work in the backward; it is
tuned the same way on a forward+backward trial.
"""
from __future__ import annotations

import time

import numpy as np

LANES = (1, 4, 16, 64)
THREADS = (64, 256)
CKPT = (256, 1024, 4096)


def hard_candidates(num_envs: int):
    """(lanes_per_env, block_threads) pairs worth trying for `num_envs` envs.

    Shapes that leave most SIMDs (1024 on MI355X) without a wave, or that put
    many more waves than SIMDs on the chip, are skipped: the former waste the
    chip and the latter only compete for the same vector ALUs.
    """
    out = []
    for g in LANES:
        waves = num_envs * g / 64.0
        if waves < 16 or waves > 1024 * 8:
            continue
        for t in THREADS + ((1024,) if g == 64 else ()):  # one env per wave: 16 envs share a workgroup
            if t >= g:
                out.append((g, t))
    return out or [(1, 64)]


def _time(fn, reps: int) -> float:
    import torch
    fn()  # warm-up (first launch, workspace allocation)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def translated_candidates(num_envs: int):
    """Launch shapes tried for the TRANSLATED kernel (each one is a compilation):
    lane groups of 4, 16 and 32 (two envs per wave: twice the waves of 16 to
    hide latency), the shapes that keep one or a few waves per SIMD."""
    out = [(g, t) for g, t in hard_candidates(num_envs) if g in (4, 16) and t <= 256]
    if 1024 <= num_envs * 32 / 64.0 <= 1024 * 8:
        out += [(32, 64), (32, 256)]
    return out or [(1, 64)]


def tune_hard(roms, env_rom, frame_skip: int = 4, seed: int = 0, ram0=None, actions=None, trial_steps: int = 2,
              reps: int = 2, candidates=None, verbose: bool = False, kernel: str = "grouped") -> dict:
    """Time `trial_steps` env steps of the given workload for each launch shape.

    Returns {"lanes_per_env", "block_threads", "env_steps_per_s", "table"}; the
    table lists every candidate with its measured rate.
    """
    import torch
    from .vcs import VcsBatch
    env_rom = np.asarray(env_rom, np.int32)
    B = env_rom.size
    cands = candidates or (translated_candidates(B) if kernel == "translated" else hard_candidates(B))
    act = None
    if actions is not None:
        act = torch.as_tensor(np.ascontiguousarray(np.asarray(actions)[:, :trial_steps]), dtype=torch.uint8).cuda()
    table = []
    for g, t in cands:
        vb = VcsBatch(roms, env_rom, frame_skip=frame_skip, seed=seed, kernel=kernel, lanes_per_env=g,
                      block_threads=t)
        vb.reset(ram0=ram0)
        sec = _time(lambda: vb.step(actions=act, steps=None if act is not None else trial_steps, frames="last"),
                    reps)
        rate = B * trial_steps / sec
        table.append({"lanes_per_env": g, "block_threads": t, "env_steps_per_s": rate})
        if verbose:
            print(f"  tune_hard G={g:2d} tpb={t:3d}: {rate:,.0f} env-steps/s", flush=True)
        del vb
    best = max(table, key=lambda r: r["env_steps_per_s"])
    return {**best, "table": table}


def tune_soft(roms, env_rom, rom_logits, ram_tape, action_logits, tau: float = 1.0, alpha: float = 6.0,
              frame_skip: int = 1, trial_steps: int = 8, lanes=None, ckpt=CKPT, reps: int = 1,
              verbose: bool = False) -> dict:
    """Time a forward+backward over the first `trial_steps` steps for each
    (lanes_per_env, K); returns the fastest with the table."""
    import torch
    from .vcs import SoftVcs
    env_rom = np.asarray(env_rom, np.int32)
    B = env_rom.size
    lanes = lanes or tuple(g for g, _ in hard_candidates(B) if g in (4, 16, 64))
    lanes = tuple(sorted(set(lanes)))
    A = action_logits[:, :trial_steps].contiguous()
    table = []
    for g in lanes:
        for k in ckpt:
            sim = SoftVcs(roms, env_rom, frame_skip=frame_skip, ckpt_interval=k, lanes_per_env=g)
            gf = torch.zeros((B, 210, 160), dtype=torch.float32, device=rom_logits.device)
            gf[:, 100, 80] = 1.0

            def run():
                _, _, res, _, _ = sim.forward(rom_logits, ram_tape, A, tau, alpha)
                sim.backward(res, rom_logits, ram_tape, A, tau, alpha, gf)

            sec = _time(run, reps)
            rate = B * trial_steps / sec
            table.append({"lanes_per_env": g, "ckpt_interval": k, "env_steps_per_s": rate,
                          "residual_bytes_per_env": sim.residual_bytes(trial_steps) / B})
            if verbose:
                print(f"  tune_soft G={g:2d} K={k:5d}: {rate:,.0f} env-steps/s", flush=True)
            del sim
    best = max(table, key=lambda r: r["env_steps_per_s"])
    return {**best, "table": table}


def wall(fn):
    t0 = time.perf_counter()
    out = fn()
    return out, time.perf_counter() - t0
