"""Torch-facing wrappers of libvcs: device buffers, streams and autograd.

PyTorch provides device memory and the current HIP stream; every step of the
emulation, the soft decode, the surrogate backward and its epilogue runs in the
library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import binding as Bd

_FRAMES = {"none": Bd.VCS_FRAMES_NONE, "last": Bd.VCS_FRAMES_LAST, "all": Bd.VCS_FRAMES_ALL}
_KERNELS = {"auto": Bd.VCS_KERNEL_AUTO, "plain": Bd.VCS_KERNEL_PLAIN, "grouped": Bd.VCS_KERNEL_GROUPED,
            "translated": Bd.VCS_KERNEL_TRANSLATED}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _rom_arrays(roms):
    imgs, maps = [], []
    for r in roms:
        if hasattr(r, "image"):
            imgs.append(np.asarray(r.image, np.uint8))
            maps.append(int(r.mapper))
        else:
            img, mp = r
            imgs.append(np.asarray(img, np.uint8))
            maps.append(int(mp))
    return imgs, maps


class _Ctx:
    def __init__(self, roms, env_rom, frame_skip, ystart, seed, ckpt_interval, kernel, lanes_per_env,
                 block_threads, device, max_positions=0, tape_records=0):
        imgs, maps = _rom_arrays(roms)
        self.env_rom = np.asarray(env_rom, np.int32)
        self.B = int(self.env_rom.size)
        self.F = int(frame_skip)
        self.rom_sizes = [int(i.size) for i in imgs]
        self.h = Bd.create(self.rom_sizes, maps, self.env_rom, frame_skip, ystart, seed, ckpt_interval,
                           _KERNELS[kernel] if isinstance(kernel, str) else int(kernel), lanes_per_env,
                           block_threads, tape_records)
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:  # "cuda" = the current device
            self.device = torch.device("cuda", torch.cuda.current_device())
        host_rom = np.concatenate(imgs)
        self.rom = torch.from_numpy(host_rom).to(self.device)
        self._ws = {}
        self.translation = None
        if (_KERNELS[kernel] if isinstance(kernel, str) else int(kernel)) == Bd.VCS_KERNEL_TRANSLATED:
            with torch.cuda.device(self.device):
                self.translation = Bd.translate(self.h, host_rom, max_positions=max_positions)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and Bd._lib is not None:
            Bd.lib().vcs_destroy(h)
            self.h = None

    def info(self):
        return Bd.launch_info(self.h)

    def workspace(self, op: int, steps: int) -> torch.Tensor:
        """The context's workspace for op, grown when a call needs more.  A
        workspace that a captured graph uses is also held by that graph, so
        replacing it here never frees memory a graph reads."""
        n = Bd.size_query("vcs_workspace_bytes", self.h, op, steps)
        w = self._ws.get(op)
        if w is None or w.numel() < n:
            w = torch.empty(n, dtype=torch.uint8, device=self.device)
            self._ws[op] = w
        return w


class VcsBatch(_Ctx):
    """B independent consoles in HARD mode (bit-exact machine)."""

    def __init__(self, roms, env_rom, frame_skip: int = 4, ystart: int = 34, seed: int = 0,
                 kernel="auto", lanes_per_env: int = 0, block_threads: int = 0, device="cuda",
                 max_positions: int = 0):
        """kernel: "auto" / "grouped" (interpreter), "plain", or "translated" (the images'
        code translated to HIP at construction; max_positions bounds the translation,
        0 = the library default)."""
        super().__init__(roms, env_rom, frame_skip, ystart, seed, 0, kernel, lanes_per_env, block_threads,
                         device, max_positions)
        n = Bd.size_query("vcs_state_bytes", self.h)
        self.state = torch.zeros(n, dtype=torch.uint8, device=self.device)

    def reset(self, ram0=None, mask=None):
        self._was_reset = True
        r0 = None if ram0 is None else torch.as_tensor(np.asarray(ram0, np.uint8) if not torch.is_tensor(ram0)
                                                       else ram0, device=self.device).contiguous()
        mk = None if mask is None else torch.as_tensor(mask, dtype=torch.uint8, device=self.device).contiguous()
        Bd.check(Bd.lib().vcs_reset(self.h, Bd.ptr(self.state), Bd.ptr(mk), Bd.ptr(r0), _stream()), "vcs_reset")

    def step(self, actions=None, steps: int | None = None, frames: str = "all", episode_steps=None,
             ram_out=None, frame_out=None, done=None, want_done: bool = True):
        """Run `steps` env steps in place.  Returns (ram_out [B,S,128] u8, frames, done [B,S] u8)."""
        B = self.B
        act = None
        if actions is not None:
            act = actions if torch.is_tensor(actions) else torch.from_numpy(np.asarray(actions, np.uint8))
            act = act.to(self.device, torch.uint8).contiguous()
            steps = act.shape[1]
        assert steps is not None and steps >= 1
        if ram_out is None:
            ram_out = torch.empty((B, steps, 128), dtype=torch.uint8, device=self.device)
        mode = _FRAMES[frames]
        if frame_out is None and mode != Bd.VCS_FRAMES_NONE:
            shape = (B, steps, 210, 160) if mode == Bd.VCS_FRAMES_ALL else (B, 210, 160)
            frame_out = torch.empty(shape, dtype=torch.uint8, device=self.device)
        if done is None and want_done:
            done = torch.empty((B, steps), dtype=torch.uint8, device=self.device)
        eps, ne = None, 0
        if episode_steps is not None:
            eps = episode_steps if torch.is_tensor(episode_steps) else torch.from_numpy(
                np.ascontiguousarray(episode_steps, np.uint32).view(np.int32))
            eps = eps.to(self.device).contiguous()
            ne = eps.shape[1]
        work = self.workspace(Bd.VCS_OP_HARD, steps)
        rc = Bd.lib().vcs_step_hard(self.h, Bd.ptr(self.rom), Bd.ptr(self.state), Bd.ptr(act), steps,
                                    Bd.ptr(ram_out), mode, Bd.ptr(frame_out), Bd.ptr(done), Bd.ptr(eps), ne,
                                    Bd.ptr(work), _stream())
        Bd.check(rc, "vcs_step_hard")
        return ram_out, frame_out, done

    def step_relaxed(self, alpha: float, T: float, actions=None, steps: int | None = None, frames: str = "all"):
        """FULL relaxed env steps (every ROM/RAM read and branch relaxed and cast, no
        straight-through correction), in place.  Returns (ram_out [B,S,128] u8, frames,
        relax [B,2] int64 = (first diverging instruction or -1, casts that differed))."""
        B = self.B
        act = None
        if actions is not None:
            act = actions if torch.is_tensor(actions) else torch.from_numpy(np.asarray(actions, np.uint8))
            act = act.to(self.device, torch.uint8).contiguous()
            steps = act.shape[1]
        assert steps is not None and steps >= 1
        ram_out = torch.empty((B, steps, 128), dtype=torch.uint8, device=self.device)
        mode = _FRAMES[frames]
        frame_out = None
        if mode != Bd.VCS_FRAMES_NONE:
            shape = (B, steps, 210, 160) if mode == Bd.VCS_FRAMES_ALL else (B, 210, 160)
            frame_out = torch.empty(shape, dtype=torch.uint8, device=self.device)
        relax = torch.empty((B, 2), dtype=torch.int64, device=self.device)
        work = self.workspace(Bd.VCS_OP_HARD, steps)
        rc = Bd.lib().vcs_step_relaxed(self.h, Bd.ptr(self.rom), Bd.ptr(self.state), Bd.ptr(act), steps,
                                       Bd.ptr(ram_out), mode, Bd.ptr(frame_out), float(alpha), float(T),
                                       Bd.ptr(relax), Bd.ptr(work), _stream())
        Bd.check(rc, "vcs_step_relaxed")
        return ram_out, frame_out, relax

    def capture(self, actions: torch.Tensor, frames: str = "last", episode_steps=None):
        """Record one step call of ``actions.shape[1]`` env steps as a HIP graph.

        Returns (graph, ram_out, frame_out, done).  Each ``graph.replay()`` runs
        those steps again from the current state, reading the device tensor
        ``actions`` (refill it in place between replays) and writing the returned
        output tensors.  The call's stream work is one host-to-device copy of the
        launch tables and one kernel, so the graph holds no memset node.  The
        graph holds references to everything it reads or writes (this batch and
        its context, the workspace, the episode lengths, the actions and the
        outputs), so none of it is freed while the graph exists.
        """
        assert getattr(self, "_was_reset", False), "reset() the batch before capturing its steps"
        assert torch.is_tensor(actions) and actions.is_cuda and actions.dtype == torch.uint8
        assert actions.is_contiguous() and actions.shape[0] == self.B
        B, S = self.B, actions.shape[1]
        mode = _FRAMES[frames]
        ram_out = torch.empty((B, S, 128), dtype=torch.uint8, device=self.device)
        frame_out = None
        if mode != Bd.VCS_FRAMES_NONE:
            shape = (B, S, 210, 160) if mode == Bd.VCS_FRAMES_ALL else (B, 210, 160)
            frame_out = torch.empty(shape, dtype=torch.uint8, device=self.device)
        done = torch.empty((B, S), dtype=torch.uint8, device=self.device)
        eps = None
        if episode_steps is not None:
            eps = episode_steps if torch.is_tensor(episode_steps) else torch.from_numpy(
                np.ascontiguousarray(episode_steps, np.uint32).view(np.int32))
            eps = eps.to(self.device).contiguous()
        work = self.workspace(Bd.VCS_OP_HARD, S)  # allocated before capture
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.step(actions=actions, frames=frames, episode_steps=eps, ram_out=ram_out, frame_out=frame_out,
                      done=done)
        graph._vcs_keep_alive = (self, work, eps, actions, self.state, self.rom, ram_out, frame_out, done)
        return graph, ram_out, frame_out, done

    def hash(self, frame: torch.Tensor | None = None, step: int | None = None) -> torch.Tensor:
        """FNV-1a 64 fingerprint per env of (registers, RAM[, frame]) as int64 [B].

        ``frame`` is a [B, 210, 160] or [B, S, 210, 160] uint8 tensor (then ``step``
        picks one step's frame)."""
        fp, stride = None, 0
        if frame is not None:
            assert frame.dtype == torch.uint8 and frame.is_contiguous() and frame.shape[0] == self.B
            stride = frame[0].numel()
            fp = frame if frame.dim() == 3 else frame[:, step]
        out = torch.empty(self.B, dtype=torch.int64, device=self.device)
        rc = Bd.lib().vcs_hash(self.h, Bd.ptr(self.state), Bd.ptr(fp), C.c_int64(stride), Bd.ptr(out), _stream())
        Bd.check(rc, "vcs_hash")
        return out

    def regs(self) -> torch.Tensor:
        out = torch.empty((self.B, 16), dtype=torch.uint8, device=self.device)
        Bd.check(Bd.lib().vcs_read_regs(self.h, Bd.ptr(self.state), Bd.ptr(out), _stream()), "vcs_read_regs")
        return out

    def objects(self) -> torch.Tensor:
        """uint8 [B][32]: the TIA object registers and collision latches (vcs_read_objects layout)."""
        out = torch.empty((self.B, 32), dtype=torch.uint8, device=self.device)
        Bd.check(Bd.lib().vcs_read_objects(self.h, Bd.ptr(self.state), Bd.ptr(out), _stream()), "vcs_read_objects")
        return out


class SoftVcs(_Ctx):
    """B consoles in SOFT-STE mode: differentiable w.r.t. ROM logits, RAM tape and action logits.

    strict=True checks the backward's tape-overflow flag after every backward
    (a host synchronisation); otherwise the flags are summed on the device and
    raise_if_overflowed() checks them.  The tape is sized so that no segment
    can fill it (every instruction takes at least two cycles), so the flag is a
    safety net.

    tape_records: the forward keeps its tape in the residual for the backward
    (0: none, every checkpoint segment is recomputed; n > 0: up to n 16-byte
    records per env; -1: room for every segment before the final frame), which
    then sweeps those segments without recomputing them: memory for time."""

    def __init__(self, roms, env_rom, frame_skip: int = 1, ystart: int = 34, ckpt_interval: int = 1024,
                 lanes_per_env: int = 0, block_threads: int = 0, device="cuda", strict: bool = False,
                 tape_records: int = 0):
        super().__init__(roms, env_rom, frame_skip, ystart, 0, ckpt_interval, "grouped", lanes_per_env,
                         block_threads, device, tape_records=tape_records)
        self.strict = strict
        self._overflow = torch.zeros(1, dtype=torch.int32, device=self.device)

    def residual_bytes(self, steps: int) -> int:
        return Bd.size_query("vcs_residual_bytes", self.h, steps)

    def decode_split(self, dec: torch.Tensor, steps: int):
        total = sum(self.rom_sizes)
        rom = dec[: total * 3].view(total, 3)
        tape = dec[total * 3: total * 3 + self.B * 128].view(self.B, 128)
        act = dec[total * 3 + self.B * 128:].view(self.B, steps, 2)
        return rom, tape, act

    def _check(self, t, shape, name, dtype=torch.float32):
        """The kernels read exactly this layout: refuse anything else before launching."""
        if not torch.is_tensor(t) or t.dtype != dtype or t.device != self.device or not t.is_contiguous() \
                or tuple(t.shape) != tuple(shape):
            got = (tuple(t.shape), t.dtype, str(t.device), t.is_contiguous()) if torch.is_tensor(t) else type(t)
            raise Bd.VcsError(f"{name}: expected a contiguous {dtype} tensor of shape {tuple(shape)} on "
                              f"{self.device}, got {got}")

    def _check_leaves(self, rom_logits, ram_tape, action_logits, state_in=None):
        B = self.B
        S = action_logits.shape[1] if torch.is_tensor(action_logits) and action_logits.dim() == 3 else -1
        self._check(rom_logits, (sum(self.rom_sizes), 256), "rom_logits")
        if ram_tape is not None or state_in is None:
            self._check(ram_tape, (B, 128, 256), "ram_tape")
        self._check(action_logits, (B, S, 18), "action_logits")
        if S < 1:
            raise Bd.VcsError("action_logits: need at least one step")
        if state_in is not None:
            self._check(state_in, (B * Bd.STATE_BYTES,), "state_in", torch.uint8)
        return S

    def forward(self, rom_logits, ram_tape, action_logits, tau: float, alpha: float = 6.0,
                want_decode: bool = False, want_state: bool = False, state_in=None, frame_dpos=None):
        """Soft forward of S = action_logits.shape[1] env steps, from power-on with the
        tape's RAM or (state_in: a [B * 256] uint8 state, e.g. VcsBatch.state after hard
        steps) from that state, whose registers and RAM are then constants (ram_tape may
        be None).  frame_dpos: a float32 [B][5][210][160] tensor to receive the position
        sampler's tangents of the final frame (P0, P1, M0, M1, BL), or None.  Returns
        (ram_out, frame, residual, decode stats or None, state or None)."""
        S = self._check_leaves(rom_logits, ram_tape, action_logits, state_in)
        B, dev = self.B, self.device
        ram_out = torch.empty((B, S, 128), dtype=torch.float32, device=dev)
        frame = torch.empty((B, 210, 160), dtype=torch.float32, device=dev)
        residual = torch.empty(Bd.size_query("vcs_residual_bytes", self.h, S), dtype=torch.uint8, device=dev)
        dec = None
        if want_decode:
            dec = torch.empty(Bd.size_query("vcs_decode_bytes", self.h, S) // 4, dtype=torch.float32, device=dev)
        st = torch.empty(B * Bd.STATE_BYTES, dtype=torch.uint8, device=dev) if want_state else None
        if frame_dpos is not None:
            self._check(frame_dpos, (B, 5, 210, 160), "frame_dpos")
        work = self.workspace(Bd.VCS_OP_SOFT_FWD, S)
        rc = Bd.lib().vcs_step_soft_fwd(self.h, Bd.ptr(state_in), Bd.ptr(rom_logits), Bd.ptr(ram_tape),
                                        Bd.ptr(action_logits), float(tau), float(alpha), S, Bd.ptr(ram_out),
                                        Bd.ptr(frame), Bd.ptr(frame_dpos), Bd.ptr(dec), Bd.ptr(st),
                                        Bd.ptr(residual), Bd.ptr(work), _stream())
        Bd.check(rc, "vcs_step_soft_fwd")
        return ram_out, frame, residual, dec, st

    def backward(self, residual, rom_logits, ram_tape, action_logits, tau: float, alpha: float, grad_frame,
                 grad_ram_out=None, check_overflow: bool = False, read_T: float = 0.0):
        """Surrogate gradients (rom_logits, ram_tape, action_logits) of the forward whose
        residual is given; the RAM-tape gradient is None when ram_tape is None (a forward
        from a given state, where it would be zero).  read_T > 0 adds the address
        surrogate (indexed reads pass gradient to their index register, Eq. s-read at
        that temperature)."""
        S = action_logits.shape[1] if torch.is_tensor(action_logits) and action_logits.dim() == 3 else -1
        self._check(rom_logits, (sum(self.rom_sizes), 256), "rom_logits")
        if ram_tape is not None:
            self._check(ram_tape, (self.B, 128, 256), "ram_tape")
        self._check(action_logits, (self.B, S, 18), "action_logits")
        self._check(residual, (Bd.size_query("vcs_residual_bytes", self.h, S),), "residual", torch.uint8)
        self._check(grad_frame, (self.B, 210, 160), "grad_frame")
        if grad_ram_out is not None:
            self._check(grad_ram_out, (self.B, S, 128), "grad_ram_out")
        g_rom = torch.empty_like(rom_logits)
        g_tape = None if ram_tape is None else torch.empty_like(ram_tape)
        g_act = torch.empty_like(action_logits)
        work = self.workspace(Bd.VCS_OP_SOFT_BWD, S)
        rc = Bd.lib().vcs_step_soft_bwd(self.h, Bd.ptr(residual), Bd.ptr(rom_logits), Bd.ptr(ram_tape),
                                        Bd.ptr(action_logits), float(tau), float(alpha), float(read_T), S,
                                        Bd.ptr(grad_frame),
                                        Bd.ptr(grad_ram_out), Bd.ptr(g_rom), Bd.ptr(g_tape), Bd.ptr(g_act),
                                        Bd.ptr(work), _stream())
        Bd.check(rc, "vcs_step_soft_bwd")
        off = Bd.size_query("vcs_bwd_overflow_offset", self.h, S)
        self._overflow += work[off:off + 4].view(torch.int32)  # on the stream, no host sync
        if check_overflow or self.strict:
            self.raise_if_overflowed()
        return g_rom, g_tape, g_act

    def raise_if_overflowed(self):
        """Synchronise and raise if any backward since the last check overflowed its tape."""
        n = int(self._overflow.item())
        self._overflow.zero_()
        if n:
            raise Bd.VcsError("soft backward tape overflow: those gradients are invalid")


class VcsSoftFunction(torch.autograd.Function):
    """(rom_logits, ram_tape, action_logits) -> (ram_out [B,S,128], final frame [B,210,160]).

    Forward values equal the hard machine's; the backward is the hand-written
    surrogate adjoint (recompute from hard-state checkpoints, reverse sweep)."""

    @staticmethod
    def forward(ctx, rom_logits, ram_tape, action_logits, sim: SoftVcs, tau: float, alpha: float, state_in=None,
                read_T: float = 0.0):
        rom_logits = rom_logits.contiguous()
        ram_tape = None if ram_tape is None else ram_tape.contiguous()
        action_logits = action_logits.contiguous()
        ram_out, frame, residual, _, _ = sim.forward(rom_logits, ram_tape, action_logits, tau, alpha,
                                                     state_in=state_in)
        ctx.save_for_backward(rom_logits, ram_tape, action_logits, residual)
        ctx.sim, ctx.tau, ctx.alpha, ctx.read_T = sim, tau, alpha, read_T
        return ram_out, frame

    @staticmethod
    def backward(ctx, g_ram, g_frame):
        rom_logits, ram_tape, action_logits, residual = ctx.saved_tensors
        sim = ctx.sim
        if g_frame is None:
            g_frame = torch.zeros((sim.B, 210, 160), dtype=torch.float32, device=sim.device)
        g_rom, g_tape, g_act = sim.backward(residual, rom_logits, ram_tape, action_logits, ctx.tau, ctx.alpha,
                                            g_frame.float().contiguous(),
                                            None if g_ram is None else g_ram.float().contiguous(),
                                            read_T=ctx.read_T)
        return g_rom, g_tape, g_act, None, None, None, None, None


def soft_rollout(sim: SoftVcs, rom_logits, ram_tape, action_logits, tau: float, alpha: float = 6.0, state_in=None,
                 read_T: float = 0.0):
    """Differentiable rollout (ram_out, final frame); from power-on with the tape's RAM, or
    from state_in (then ram_tape may be None and gets no gradient).  read_T > 0: the
    backward adds the address surrogate."""
    return VcsSoftFunction.apply(rom_logits, ram_tape, action_logits, sim, tau, alpha, state_in, read_T)


def ste_luminance(frame: torch.Tensor) -> torch.Tensor:
    """Luminance (c >> 1) & 7 of palette indices, with d lum / d c = 1/2 (straight-through)."""
    hard = ((frame.detach().to(torch.int32) >> 1) & 7).to(frame.dtype)
    soft = frame * 0.5
    return soft + (hard - soft).detach()
