"""Full-size parity in the benchmark's launch configuration, on outputs the
oracle can compute one env (or one ROM) at a time."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def run_sampled(w, sample, chunk):
    """Run the whole workload on the GPU in chunks; keep RAM/frames/done of `sample`."""
    import torch
    from paper_2606_22447_amd.vcs import VcsBatch
    vb = VcsBatch(w.roms, w.env_rom, frame_skip=w.frame_skip, seed=w.seed)
    vb.reset(ram0=w.ram0)
    B, S = w.num_envs, w.steps
    ram_out = torch.empty((B, chunk, 128), dtype=torch.uint8, device="cuda")
    frame_out = torch.empty((B, chunk, 210, 160), dtype=torch.uint8, device="cuda")
    done = torch.empty((B, chunk), dtype=torch.uint8, device="cuda")
    eps = None if w.episode_steps is None else torch.from_numpy(w.episode_steps.view(np.int32)).cuda()
    idx = torch.tensor(sample, device="cuda")
    rams, frs, dns = [], [], []
    for s0 in range(0, S, chunk):
        acts = torch.from_numpy(np.ascontiguousarray(w.actions[:, s0:s0 + chunk])).cuda()
        vb.step(acts, frames="all", episode_steps=eps, ram_out=ram_out, frame_out=frame_out, done=done)
        rams.append(ram_out[idx].cpu().numpy())
        frs.append(frame_out[idx].cpu().numpy())
        dns.append(done[idx].cpu().numpy())
    torch.cuda.synchronize()
    return np.concatenate(rams, 1), np.concatenate(frs, 1), np.concatenate(dns, 1), vb


def check_envs(w, sample, ram, fr, dn):
    for i, b in enumerate(sample):
        rom = w.roms[int(w.env_rom[b])]
        ep = None if w.episode_steps is None else w.episode_steps[b]
        ref = O.run_env(rom.image, rom.mapper, w.ram0[b], w.actions[b], w.steps, w.frame_skip, ep_steps=ep,
                        seed=w.seed, env_index=b)
        assert (ref["done"] == dn[i]).all(), b
        assert (ref["ram"] == ram[i]).all(), b
        assert (ref["frames"] == fr[i]).all(), b


def test_c1_full_size_sampled_envs():
    w = I.config_c1()
    sample = [0, 1, 777, 2048, 4095]
    say("c1 full: 4096 envs x 500 steps")
    ram, fr, dn, vb = run_sampled(w, sample, 50)
    check_envs(w, sample, ram, fr, dn)


def test_c2_full_size_sampled_envs():
    w = I.config_c2()
    # envs on 2K, 4K and F8 ROMs, and envs whose episodes end inside the run
    mappers = np.array([w.roms[int(r)].mapper for r in w.env_rom])
    cum = np.cumsum(w.episode_steps, axis=1)
    resets = (cum[:, 0] < w.steps)
    sample = []
    for m in (0, 1, 2):
        cand = np.nonzero((mappers == m) & resets)[0]
        sample += [int(cand[0]), int(cand[len(cand) // 2])]
    say("c2 full: 16384 envs x 500 steps, sample", sample)
    ram, fr, dn, vb = run_sampled(w, sample, 25)
    check_envs(w, sample, ram, fr, dn)
    assert dn.sum() >= len(sample)  # every sampled env crossed an episode end


def test_c4_full_size_gradients_of_one_rom():
    import torch
    from paper_2606_22447_amd.vcs import SoftVcs
    w = I.config_c4()
    lv = I.soft_leaves(w)
    tau = 1.0
    B, S = w.num_envs, w.steps
    offs = w.rom_offsets()
    r = 1  # a sampled ROM: every env that runs it enters its gradient
    envs = np.nonzero(w.env_rom == r)[0]
    o, n = offs[r], w.roms[r].size
    dec_rom = O.decode_logits(lv.rom_logits[o:o + n], tau)
    hard_ram0, ev0 = O.decode_tape(lv.ram_tape[envs].reshape(-1, 256))
    hard_ram0, ev0 = hard_ram0.reshape(-1, 128), ev0.reshape(-1, 128)
    ha, es, ei = O.decode_actions(lv.action_logits[envs].reshape(-1, 18), tau)
    ha, es, ei = ha.reshape(-1, S), es.reshape(-1, S), ei.reshape(-1, S)
    grad_frame = np.zeros((B, 210, 160), np.float32)
    g_rom = np.zeros(n)
    g0 = np.zeros((len(envs), 128))
    gsw, gin = np.zeros((len(envs), S)), np.zeros((len(envs), S))
    say("c4 oracle: ROM", r, "envs", len(envs))
    for i, b in enumerate(envs):
        tgt = O.run_env(lv.perturbed_roms[r], w.roms[r].mapper, hard_ram0[i], ha[i], S, 1, frames="last")["frames"][0]
        hard = O.run_env(dec_rom[0], w.roms[r].mapper, hard_ram0[i], ha[i], S, 1, frames="last")["frames"][0]
        d = ((hard.astype(np.int64) >> 1) & 7) - ((tgt.astype(np.int64) >> 1) & 7)
        grad_frame[b] = (2.0 * d / 33600) * 0.5
        res = O.soft_env(dec_rom[0], dec_rom[1], w.roms[r].mapper, hard_ram0[i], ev0[i], ha[i], es[i], ei[i], S, 1,
                         mode="ste", grad_frame=grad_frame[b].astype(np.float64))
        g_rom += res["g_rom"]
        g0[i], gsw[i], gin[i] = res["g_ram0"], res["g_swcha"], res["g_inpt4"]
    ref_rom = O.epilogue_rom(lv.rom_logits[o:o + n], tau, g_rom)
    ref_tape = O.epilogue_tape(g0.reshape(-1)).reshape(len(envs), 128, 256)
    ref_act = O.epilogue_action(lv.action_logits[envs].reshape(-1, 18), tau, gsw.reshape(-1),
                                gin.reshape(-1)).reshape(len(envs), S, 18)
    say("c4 gpu fwd+bwd at full size")
    sim = SoftVcs(w.roms, w.env_rom, frame_skip=1, ckpt_interval=1024)
    L = torch.from_numpy(lv.rom_logits).cuda()
    T = torch.from_numpy(lv.ram_tape).cuda()
    Aa = torch.from_numpy(lv.action_logits).cuda()
    _, _, residual, _, _ = sim.forward(L, T, Aa, tau, 6.0)
    g = sim.backward(residual, L, T, Aa, tau, 6.0, torch.from_numpy(grad_frame).cuda(), check_overflow=True)
    torch.cuda.synchronize()
    got_rom = g[0][o:o + n].cpu().numpy()
    got_tape = g[1][torch.from_numpy(envs).cuda()].cpu().numpy()
    got_act = g[2][torch.from_numpy(envs).cuda()].cpu().numpy()
    from tests.test_gpu_soft import assert_grad_close
    assert_grad_close(got_rom, ref_rom, "rom_logits")
    assert_grad_close(got_tape, ref_tape, "ram_tape")
    if np.abs(ref_act).max() > 0:
        assert_grad_close(got_act, ref_act, "action_logits")
    else:
        assert (got_act == 0).all()
    # every other env got a zero frame gradient: their leaves' gradients are exactly zero
    others = np.nonzero(w.env_rom != r)[0][:64]
    assert (g[1][torch.from_numpy(others).cuda()] == 0).all().item()
