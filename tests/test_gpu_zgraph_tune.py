"""HIP-graph capture of a multi-step hard call, and the autotuner, on the GPU."""
import numpy as np
import pytest

from paper_2606_22447_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("kernel", ["grouped", "translated"])
def test_graph_replays_match_eager_steps(kernel):
    import torch
    from paper_2606_22447_amd.vcs import VcsBatch
    w = I.config_c1(num_envs=64, steps=12)
    chunk = 3
    eager = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed, kernel=kernel)
    graphed = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed, kernel=kernel)
    eager.reset(ram0=w.ram0)
    graphed.reset(ram0=w.ram0)
    act = torch.empty((w.num_envs, chunk), dtype=torch.uint8, device="cuda")
    act.copy_(torch.from_numpy(np.ascontiguousarray(w.actions[:, :chunk])))
    torch.cuda.synchronize()
    g, ram_g, fr_g, dn_g = graphed.capture(act, frames="last")
    say("captured; replaying")
    for k in range(w.steps // chunk):
        a_k = torch.from_numpy(np.ascontiguousarray(w.actions[:, k * chunk:(k + 1) * chunk])).cuda()
        act.copy_(a_k)
        g.replay()
        torch.cuda.synchronize()
        ram_e, fr_e, dn_e = eager.step(actions=a_k, frames="last")  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(ram_g, ram_e), k
        assert torch.equal(fr_g, fr_e), k
        assert torch.equal(dn_g, dn_e), k
    # and the eager twin agrees with the oracle at the end
    from oracle import oracle as O
    ref = O.run_env(w.roms[0].image, w.roms[0].mapper, w.ram0[5], w.actions[5], w.steps, w.frame_skip,
                    frames="last")
    assert (ram_g[5, -1].cpu().numpy() == ref["ram"][-1]).all()
    assert (fr_g[5].cpu().numpy() == ref["frames"][0]).all()


def test_autotuner_picks_a_measured_shape_and_it_is_exact():
    from paper_2606_22447_amd import autotune
    from paper_2606_22447_amd.vcs import VcsBatch
    w = I.config_c1(num_envs=512, steps=2)
    res = autotune.tune_hard(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed, ram0=w.ram0,
                             actions=w.actions, trial_steps=1, reps=1)
    say("tuned", {k: v for k, v in res.items() if k != "table"})
    shapes = {(r["lanes_per_env"], r["block_threads"]) for r in res["table"]}
    assert (res["lanes_per_env"], res["block_threads"]) in shapes
    assert all(r["env_steps_per_s"] > 0 for r in res["table"])
    # the chosen shape computes the same bytes as any other
    import torch
    outs = []
    for g, t in [(res["lanes_per_env"], res["block_threads"]), (1, 64)]:
        vb = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed, kernel="grouped",
                      lanes_per_env=g, block_threads=t)
        vb.reset(ram0=w.ram0)
        ram, fr, _ = vb.step(actions=w.actions, frames="last")
        torch.cuda.synchronize()
        outs.append((ram.cpu().numpy(), fr.cpu().numpy()))
    assert (outs[0][0] == outs[1][0]).all() and (outs[0][1] == outs[1][1]).all()


def test_graph_keeps_what_it_reads_alive():
    """A graph captured with host (numpy) episode lengths keeps its device copy,
    the workspace and the batch alive: eager steps of another length on the same
    batch between replays, and fresh allocations that would reuse freed memory,
    change nothing."""
    import gc
    import torch
    from paper_2606_22447_amd.vcs import VcsBatch
    w = I.config_c2(envs_per_rom=4, steps=20, n_roms=4)
    eps = np.minimum(w.episode_steps, 3 + np.arange(w.episode_steps.size).reshape(w.episode_steps.shape) % 4)
    chunk, other = 3, 2
    eager = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed, kernel="grouped")
    graphed = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed, kernel="grouped")
    eager.reset(ram0=w.ram0)
    graphed.reset(ram0=w.ram0)
    act = torch.from_numpy(np.ascontiguousarray(w.actions[:, :chunk])).cuda()
    g, ram_g, fr_g, dn_g = graphed.capture(act, frames="last", episode_steps=eps.copy())
    gc.collect()
    col = 0
    for k in range(3):
        say("replay", k)
        a_k = torch.from_numpy(np.ascontiguousarray(w.actions[:, col:col + chunk])).cuda()
        act.copy_(a_k)
        g.replay()
        ram_e, fr_e, dn_e = eager.step(actions=a_k, frames="last", episode_steps=eps)
        torch.cuda.synchronize()
        assert torch.equal(ram_g, ram_e) and torch.equal(fr_g, fr_e) and torch.equal(dn_g, dn_e), k
        col += chunk
        # eager steps of another length on the graphed batch, then allocations over freed memory
        a_o = np.ascontiguousarray(w.actions[:, col:col + other])
        graphed.step(actions=a_o, frames="none", episode_steps=eps)
        eager.step(actions=a_o, frames="none", episode_steps=eps)
        junk = [torch.full((1 << 20,), 0xA5, dtype=torch.uint8, device="cuda") for _ in range(8)]
        torch.cuda.synchronize()
        del junk
        col += other
    assert torch.equal(graphed.hash(), eager.hash())
