"""ctypes wrapper of the reference emulator.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg use it; the product library never does.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

SCREEN = (210, 160)
# cartridge formats (the oracle's numbering, shared with the library's C ABI)
MAPPER_2K, MAPPER_4K, MAPPER_F8, MAPPER_F6, MAPPER_F4, MAPPER_F8SC, MAPPER_F6SC, MAPPER_F4SC, MAPPER_E0 = range(9)
MAPPER_SIZE = {MAPPER_2K: 2048, MAPPER_4K: 4096, MAPPER_F8: 8192, MAPPER_F6: 16384, MAPPER_F4: 32768,
               MAPPER_F8SC: 8192, MAPPER_F6SC: 16384, MAPPER_F4SC: 32768, MAPPER_E0: 8192}
ACTION_RESET = 18  # the console RESET switch held, joystick idle

REG_NAMES = ["A", "X", "Y", "S", "P", "PCL", "PCH", "bank", "jammed", "INTIM", "TIMINT", "VBLANK",
             "COLUP0", "COLUP1", "COLUPF", "COLUBK", "CTRLPF", "PF0", "PF1", "PF2", "VSYNC", "cycle",
             "instructions", "episode", "ep_step"]
# vcs_read_objects layout (32 values): object columns, graphics, enables, shape and
# delay registers, motion registers, collision latches
OBJECT_NAMES = ["posP0", "posP1", "posM0", "posM1", "posBL", "GRP0", "GRP1", "GRP0old", "GRP1old", "ENAM0",
                "ENAM1", "ENABL", "ENABLold", "NUSIZ0", "NUSIZ1", "REFP0", "REFP1", "VDELP0", "VDELP1", "VDELBL",
                "RESMP0", "RESMP1", "HMP0", "HMP1", "HMM0", "HMM1", "HMBL", "CXlo", "CXhi", "pad0", "pad1", "pad2"]

u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        src = os.path.join(os.path.dirname(path), "vcs_oracle.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        L = C.CDLL(path)
        vp = C.c_void_p
        L.orc_new.restype = vp
        L.orc_free.argtypes = [vp]
        L.orc_power_on.argtypes = [vp, u8p, C.c_int, C.c_int, u8p, C.c_int]
        L.orc_power_on.restype = C.c_int
        L.orc_step_instruction.argtypes = [vp]
        L.orc_step_instruction.restype = C.c_int
        L.orc_run_cycles.argtypes = [vp, C.c_int64]
        L.orc_set_action.argtypes = [vp, C.c_int]
        L.orc_set_draw_frame.argtypes = [vp, C.c_int64]
        L.orc_env_step.argtypes = [vp, C.c_int, C.c_int, C.c_int64, C.c_int]
        L.orc_get_regs.argtypes = [vp, i64p]
        L.orc_ram.argtypes = [vp]
        L.orc_ram.restype = C.POINTER(C.c_uint8)
        L.orc_frame.argtypes = [vp]
        L.orc_frame.restype = C.POINTER(C.c_uint8)
        L.orc_poke_ram.argtypes = [vp, C.c_int, C.c_int]
        L.orc_op_stats.argtypes = [vp, u64p]
        L.orc_set_relax.argtypes = [vp, C.c_int, C.c_double, C.c_double]
        L.orc_relax_ndiv.argtypes = [vp]
        L.orc_relax_ndiv.restype = C.c_int64
        L.orc_relax_fails.argtypes = [vp]
        L.orc_relax_fails.restype = C.c_uint64
        L.orc_relax_last_dev.argtypes = [vp, f64p]
        L.orc_dispatch_deviation.argtypes = [vp, f64p, C.c_double] + [C.POINTER(C.c_double)] * 3
        L.orc_intim_at.argtypes = [vp, C.c_int64]
        L.orc_timint_at.argtypes = [vp, C.c_int64]
        L.orc_opcode_info.argtypes = [C.c_int] + [C.POINTER(C.c_int)] * 4
        L.orc_alu.argtypes = [C.c_int] * 4 + [C.POINTER(C.c_int)] * 2
        L.orc_splitmix_ram.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, u8p]
        L.orc_splitmix_sc_ram.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, u8p]
        L.orc_set_sc_ram.argtypes = [vp, u8p]
        L.orc_sc_ram.argtypes = [vp]
        L.orc_sc_ram.restype = C.POINTER(C.c_uint8)
        L.orc_splitmix_next.argtypes = [C.POINTER(C.c_uint64)]
        L.orc_splitmix_next.restype = C.c_uint64
        L.orc_gate.argtypes = [C.c_double, C.c_double]
        L.orc_gate.restype = C.c_double
        L.orc_gate_grad.argtypes = [C.c_double, C.c_double]
        L.orc_gate_grad.restype = C.c_double
        L.orc_run_env.argtypes = [u8p, C.c_int, C.c_int, u8p, vp, C.c_int, C.c_int, C.c_int, vp, C.c_int,
                                  C.c_uint64, C.c_int64, u8p, vp, C.c_int, vp, vp, vp, vp]
        L.orc_run_env.restype = C.c_int
        L.orc_decode_logit_rows.argtypes = [f32p, C.c_int64, C.c_int, C.c_double, u8p, f64p, f64p, f64p]
        L.orc_decode_tape_rows.argtypes = [f32p, C.c_int64, u8p, f64p]
        L.orc_decode_action_rows.argtypes = [f32p, C.c_int64, C.c_double, u8p, f64p, f64p]
        L.orc_epilogue_rom.argtypes = [f32p, C.c_int64, C.c_double, f64p, f64p]
        L.orc_epilogue_tape.argtypes = [C.c_int64, f64p, f64p]
        L.orc_epilogue_action.argtypes = [f32p, C.c_int64, C.c_double, f64p, f64p, f64p]
        L.orc_soft_env.argtypes = [u8p, f64p, C.c_int, C.c_int, u8p, f64p, u8p, f64p, f64p, C.c_int, C.c_int,
                                   C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, f64p, f64p, f64p, f64p, vp]
        L.orc_soft_env.restype = C.c_int
        L.orc_soft_env_from.argtypes = [u8p, f64p, C.c_int, C.c_int, u8p, f64p, C.c_int, vp, u8p, f64p, f64p,
                                        C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, vp, vp, vp, vp, vp, vp,
                                        f64p, f64p, f64p, f64p, f64p, vp, vp]
        L.orc_get_objects.argtypes = [vp, i64p]
        L.orc_soft_env_from.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------------
# Single machine (unit tests)
# --------------------------------------------------------------------------

class Machine:
    def __init__(self, rom: np.ndarray, mapper: int, ram0=None, ystart: int = 34):
        self.L = lib()
        self.h = self.L.orc_new()
        self.rom = np.ascontiguousarray(rom, dtype=np.uint8)
        r = np.zeros(128, np.uint8) if ram0 is None else np.ascontiguousarray(ram0, dtype=np.uint8)
        rc = self.L.orc_power_on(self.h, self.rom, self.rom.size, mapper, r, ystart)
        if rc:
            raise ValueError("bad ROM size / mapper / ystart")

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_free(self.h)
            self.h = None

    def step(self) -> int:
        return self.L.orc_step_instruction(self.h)

    def run_cycles(self, budget: int):
        self.L.orc_run_cycles(self.h, budget)

    def set_action(self, a: int):
        self.L.orc_set_action(self.h, a)

    def set_draw_frame(self, f: int):
        self.L.orc_set_draw_frame(self.h, f)

    def env_step(self, action: int, frame_skip: int, step_index: int, store_frame: bool = True):
        self.L.orc_env_step(self.h, action, frame_skip, step_index, int(store_frame))

    def set_sc_ram(self, v):
        self.L.orc_set_sc_ram(self.h, np.ascontiguousarray(v, dtype=np.uint8))

    def sc_ram(self) -> np.ndarray:
        return np.ctypeslib.as_array(self.L.orc_sc_ram(self.h), shape=(128,)).copy()

    def regs(self) -> dict:
        out = np.zeros(25, np.int64)
        self.L.orc_get_regs(self.h, out)
        return dict(zip(REG_NAMES, out.tolist()))

    def ram(self) -> np.ndarray:
        return np.ctypeslib.as_array(self.L.orc_ram(self.h), shape=(128,)).copy()

    def objects(self) -> dict:
        """Object registers now (collisions latched up to the current cycle)."""
        out = np.zeros(32, np.int64)
        self.L.orc_get_objects(self.h, out)
        return dict(zip(OBJECT_NAMES, out.tolist()))

    def frame(self) -> np.ndarray:
        return np.ctypeslib.as_array(self.L.orc_frame(self.h), shape=(210 * 160,)).copy().reshape(SCREEN)

    def poke(self, cell: int, v: int):
        self.L.orc_poke_ram(self.h, cell, v)

    def op_stats(self):
        """(executions, page-crossing executions, taken branches) per opcode byte since power-on."""
        out = np.zeros(768, np.uint64)
        self.L.orc_op_stats(self.h, out)
        return out[:256], out[256:512], out[512:]

    def set_relax(self, alpha: float, T: float, on: bool = True, track: bool = False):
        """FULL relaxed mode: sigmoid branches and distance-softmax reads cast to integers
        (track: also record each instruction's float64 pre-cast deviations)."""
        self.L.orc_set_relax(self.h, int(on) | (2 if track else 0), float(alpha), float(T))

    def relax_ndiv(self) -> int:
        return int(self.L.orc_relax_ndiv(self.h))

    def relax_fails(self) -> int:
        return int(self.L.orc_relax_fails(self.h))

    def relax_last_dev(self):
        """(summed read deviation, number of relaxed reads, branch deviation) of the last
        instruction, float64 before the casts."""
        out = np.zeros(3)
        self.L.orc_relax_last_dev(self.h, out)
        return float(out[0]), int(out[1]), float(out[2])

    def dispatch_deviation(self, logits: np.ndarray, T: float):
        """(dev, spread, w_star) of the relaxed dispatch of the next instruction."""
        d, sp, ws = C.c_double(), C.c_double(), C.c_double()
        self.L.orc_dispatch_deviation(self.h, np.ascontiguousarray(logits, np.float64), float(T), C.byref(d),
                                      C.byref(sp), C.byref(ws))
        return d.value, sp.value, ws.value

    def intim_at(self, t: int) -> int:
        return self.L.orc_intim_at(self.h, t)

    def timint_at(self, t: int) -> int:
        return self.L.orc_timint_at(self.h, t)


def opcode_info(op: int):
    a, b, c, d = (C.c_int() for _ in range(4))
    ok = lib().orc_opcode_info(op, C.byref(a), C.byref(b), C.byref(c), C.byref(d))
    return bool(ok), a.value, b.value, c.value, d.value


def alu(op: str, a: int, v: int, p: int):
    r, po = C.c_int(), C.c_int()
    lib().orc_alu(0 if op == "ADC" else 1, a, v, p, C.byref(r), C.byref(po))
    return r.value, po.value


def splitmix_ram(seed: int, env: int, episode: int) -> np.ndarray:
    out = np.zeros(128, np.uint8)
    lib().orc_splitmix_ram(seed, env, episode, out)
    return out


def splitmix_sc_ram(seed: int, env: int, episode: int) -> np.ndarray:
    """Seeded Superchip RAM of (seed, env, episode)."""
    out = np.zeros(128, np.uint8)
    lib().orc_splitmix_sc_ram(seed, env, episode, out)
    return out


def splitmix_next(state: int):
    s = C.c_uint64(state)
    v = lib().orc_splitmix_next(C.byref(s))
    return v, s.value


def gate(z: float, alpha: float) -> float:
    return lib().orc_gate(z, alpha)


def gate_grad(z: float, alpha: float) -> float:
    return lib().orc_gate_grad(z, alpha)


def action_ports(a: int):
    L = lib()
    L.orc_action_swcha.argtypes = [C.c_int]
    L.orc_action_inpt4.argtypes = [C.c_int]
    return L.orc_action_swcha(a), L.orc_action_inpt4(a)


# --------------------------------------------------------------------------
# Whole-env rollouts
# --------------------------------------------------------------------------

def run_env(rom: np.ndarray, mapper: int, ram0: np.ndarray, actions, steps: int, frame_skip: int,
            ystart: int = 34, ep_steps=None, seed: int = 0, env_index: int = 0, frames: str = "all",
            step_state: bool = False):
    """Hard rollout of one env from power-on.  Returns a dict of numpy arrays
    (with step_state: "step_state" [steps][144] = after each step, the 16 register
    bytes A X Y S P PCL PCH bank jammed INTIM TIMINT VBLANK COLUP0 COLUP1 COLUPF
    COLUBK, then the 128 RAM bytes)."""
    L = lib()
    rom = np.ascontiguousarray(rom, dtype=np.uint8)
    ram0 = np.ascontiguousarray(ram0, dtype=np.uint8)
    act = None if actions is None else np.ascontiguousarray(actions, dtype=np.uint8)
    eps = None if ep_steps is None else np.ascontiguousarray(ep_steps, dtype=np.uint32)
    ram_out = np.zeros((steps, 128), np.uint8)
    mode = {"none": 0, "last": 1, "all": 2}[frames]
    nfr = steps if mode == 2 else (1 if mode == 1 else 0)
    frame_out = np.zeros((max(nfr, 1), 210, 160), np.uint8)
    done = np.zeros(steps, np.uint8)
    regs = np.zeros(25, np.int64)
    instr = np.zeros(1, np.uint64)
    st = np.zeros((steps, 144), np.uint8) if step_state else None
    rc = L.orc_run_env(rom, rom.size, mapper, ram0, _ptr(act), steps, frame_skip, ystart, _ptr(eps),
                       0 if eps is None else eps.size, seed, env_index, ram_out, _ptr(frame_out), mode,
                       _ptr(done), _ptr(regs), _ptr(instr), _ptr(st))
    if rc:
        raise ValueError("oracle rejected the configuration")
    out = {"ram": ram_out, "frames": frame_out[:nfr], "done": done,
           "regs": dict(zip(REG_NAMES, regs.tolist())), "instructions": int(instr[0])}
    if step_state:
        out["step_state"] = st
    return out


def op_stats(rom: np.ndarray, mapper: int, ram0: np.ndarray, actions, steps: int, frame_skip: int):
    """Hard rollout of one env from power-on (no resets); returns the opcode
    statistics of Machine.op_stats."""
    m = Machine(rom, mapper, ram0)
    for s in range(steps):
        m.env_step(0 if actions is None else int(actions[s]), frame_skip, s, store_frame=False)
    return m.op_stats()


def run_relaxed(rom: np.ndarray, mapper: int, ram0: np.ndarray, actions, steps: int, frame_skip: int,
                alpha: float, T: float, frames: str = "all"):
    """FULL relaxed rollout of one env from power-on (no episodes): RAM [S][128]
    and frames after each step, the first diverging instruction (-1: none) and the
    number of casts that differed."""
    m = Machine(rom, mapper, ram0)
    m.set_relax(alpha, T)
    ram = np.zeros((steps, 128), np.uint8)
    fr = np.zeros((steps if frames == "all" else 1, 210, 160), np.uint8)
    for s in range(steps):
        store = frames == "all" or (frames == "last" and s == steps - 1)
        m.env_step(0 if actions is None else int(actions[s]), frame_skip, s, store_frame=store)
        ram[s] = m.ram()
        if store:
            fr[s if frames == "all" else 0] = m.frame()
    return {"ram": ram, "frames": fr, "ndiv": m.relax_ndiv(), "fails": m.relax_fails(),
            "regs": m.regs()}


def decode_logits(rows: np.ndarray, tau: float):
    rows = np.ascontiguousarray(rows, dtype=np.float32)
    n, k = rows.shape
    hard = np.zeros(n, np.uint8)
    ev, mx, z = (np.zeros(n) for _ in range(3))
    lib().orc_decode_logit_rows(rows, n, k, tau, hard, ev, mx, z)
    return hard, ev, mx, z


def decode_tape(rows: np.ndarray):
    rows = np.ascontiguousarray(rows, dtype=np.float32).reshape(-1, 256)
    n = rows.shape[0]
    hard = np.zeros(n, np.uint8)
    ev = np.zeros(n)
    lib().orc_decode_tape_rows(rows, n, hard, ev)
    return hard, ev


def decode_actions(rows: np.ndarray, tau: float):
    rows = np.ascontiguousarray(rows, dtype=np.float32).reshape(-1, 18)
    n = rows.shape[0]
    hard = np.zeros(n, np.uint8)
    es, ei = np.zeros(n), np.zeros(n)
    lib().orc_decode_action_rows(rows, n, tau, hard, es, ei)
    return hard, es, ei


def epilogue_rom(logits: np.ndarray, tau: float, g: np.ndarray) -> np.ndarray:
    logits = np.ascontiguousarray(logits, dtype=np.float32)
    out = np.zeros(logits.shape, np.float64)
    lib().orc_epilogue_rom(logits, logits.shape[0], tau, np.ascontiguousarray(g, np.float64), out)
    return out


def epilogue_tape(g0: np.ndarray) -> np.ndarray:
    g0 = np.ascontiguousarray(g0, np.float64).reshape(-1)
    out = np.zeros((g0.size, 256))
    lib().orc_epilogue_tape(g0.size, g0, out)
    return out


def epilogue_action(logits: np.ndarray, tau: float, g_swcha: np.ndarray, g_inpt4: np.ndarray) -> np.ndarray:
    logits = np.ascontiguousarray(logits, dtype=np.float32).reshape(-1, 18)
    out = np.zeros(logits.shape)
    lib().orc_epilogue_action(logits, logits.shape[0], tau, np.ascontiguousarray(g_swcha, np.float64).reshape(-1),
                              np.ascontiguousarray(g_inpt4, np.float64).reshape(-1), out)
    return out


def soft_env(rom_hard, rom_ev, mapper, ram0_hard, ram0_ev, act_hard, swcha_ev, inpt4_ev, steps, frame_skip,
             mode: str = "ste", grad_frame=None, grad_ram=None, ystart: int = 34, pre_actions=None,
             read_T: float = 0.0):
    """SOFT-STE (or SMOOTH) rollout of one env with its reverse sweep: from
    power-on, or (pre_actions given) after len(pre_actions) hard env steps from
    power-on, whose state the soft steps continue (its RAM is then a constant:
    g_ram0 = 0).  read_T > 0 turns on the address surrogate: indexed reads of ROM
    or RAM bytes also pass gradient to their index register through Eq. s-read
    at temperature read_T.

    Returns hard outputs, smooth outputs, the leaf gradients g_rom (per ROM
    byte), g_ram0, g_swcha, g_inpt4, and g_pos, the position sampler's
    derivative for the columns of P0, P1, M0, M1, BL, with its per-pixel
    tangents frame_dpos [5][210][160] (all float64)."""
    L = lib()
    rom_hard = np.ascontiguousarray(rom_hard, np.uint8)
    rom_ev = np.ascontiguousarray(rom_ev, np.float64)
    gf = None if grad_frame is None else np.ascontiguousarray(grad_frame, np.float64).reshape(-1)
    gr = None if grad_ram is None else np.ascontiguousarray(grad_ram, np.float64).reshape(-1)
    ram_out = np.zeros((steps, 128), np.uint8)
    frame_out = np.zeros((210, 160), np.uint8)
    ram_sm = np.zeros((steps, 128))
    frame_sm = np.zeros((210, 160))
    g_rom = np.zeros(rom_hard.size)
    g_ram0 = np.zeros(128)
    g_sw = np.zeros(steps)
    g_in = np.zeros(steps)
    g_pos = np.zeros(5)
    dpos = np.zeros((5, 210, 160))
    nn = np.zeros(1, np.int64)
    pre = None if pre_actions is None else np.ascontiguousarray(pre_actions, np.uint8)
    rc = L.orc_soft_env_from(rom_hard, rom_ev, rom_hard.size, mapper, np.ascontiguousarray(ram0_hard, np.uint8),
                             np.ascontiguousarray(ram0_ev, np.float64), 0 if pre is None else pre.size, _ptr(pre),
                             np.ascontiguousarray(act_hard, np.uint8),
                             np.ascontiguousarray(swcha_ev, np.float64), np.ascontiguousarray(inpt4_ev, np.float64),
                             steps, frame_skip, ystart, 1 if mode == "smooth" else 0, float(read_T), _ptr(gf),
                             _ptr(gr),
                             _ptr(ram_out), _ptr(frame_out), _ptr(ram_sm), _ptr(frame_sm), g_rom, g_ram0, g_sw, g_in,
                             g_pos, _ptr(dpos), _ptr(nn))
    if rc:
        raise ValueError("oracle rejected the configuration")
    return {"ram": ram_out, "frame": frame_out, "ram_smooth": ram_sm, "frame_smooth": frame_sm,
            "g_rom": g_rom, "g_ram0": g_ram0, "g_swcha": g_sw, "g_inpt4": g_in, "g_pos": g_pos, "frame_dpos": dpos,
            "nodes": int(nn[0])}
