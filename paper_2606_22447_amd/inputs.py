"""Seeded synthetic workloads for the batched Atari VCS emulator.

This module produces *data only*: cartridge images built by a small 6502
assembler, initial RAM bytes, joystick action streams, episode lengths and the
soft-mode leaf tensors (ROM logits, RAM tape, action logits).  It executes no
6502 code and contains none of the emulator's arithmetic; the reference
emulator under ``oracle/`` and the GPU library both consume its outputs as plain
arrays.

The real cartridges the paper measures on (Pong for throughput, 64 ALE titles
for conformance) are copyrighted and absent; seed-generated programs with the
same sizes (2K, 4K and F8 bank-switched 8K), the same NTSC frame structure
(3 VSYNC + 37 VBLANK + 192 kernel + 30 overscan lines of 76 CPU cycles) and the
same kinds of work (playfield/background colour writes raced against the beam,
RAM counters, decimal-mode arithmetic, subroutines, input and timer reads)
stand in for them.

Randomness is SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used in counter mode:
``value(key, i) = mix64(key + (i + 1) * GOLDEN)``; Gaussian noise is Box-Muller
in float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15

# --------------------------------------------------------------------------
# SplitMix64
# --------------------------------------------------------------------------


def mix64(z: int) -> int:
    """SplitMix64 output function (variant 13 finaliser)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def stream_key(seed: int, *ids: int) -> int:
    """Derive an independent stream key from a seed and integer ids."""
    k = seed & M64
    for i in ids:
        k = mix64((k + ((int(i) + 1) * GOLDEN)) & M64)
    return k


def u64_stream(key: int, n: int, start: int = 0) -> np.ndarray:
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + idx * np.uint64(GOLDEN)
    return mix64_np(z)


def byte_stream(key: int, n: int) -> np.ndarray:
    words = u64_stream(key, (n + 7) // 8)
    return words.view(np.uint8)[:n].copy()  # little-endian bytes of each word


def unit_stream(key: int, n: int) -> np.ndarray:
    """Uniform float64 in [0, 1) from the top 53 bits."""
    return (u64_stream(key, n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def int_stream(key: int, n: int, hi: int) -> np.ndarray:
    """Uniform integers in [0, hi) (53-bit float scaling; bias < 2^-40)."""
    return np.floor(unit_stream(key, n) * hi).astype(np.int64)


def normal_stream(key: int, n: int) -> np.ndarray:
    """Standard normal float64 via Box-Muller (one output per uniform pair)."""
    u = unit_stream(key, 2 * n)
    u1 = 1.0 - u[0::2]  # (0, 1]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


class Rng:
    """Sequential SplitMix64 for the program generator's decisions."""

    def __init__(self, seed: int):
        self.state = seed & M64

    def next(self) -> int:
        self.state = (self.state + GOLDEN) & M64
        return mix64(self.state)

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi]."""
        return lo + (self.next() >> 11) * (hi - lo + 1) // (1 << 53)

    def random(self) -> float:
        return (self.next() >> 11) * (1.0 / (1 << 53))

    def choice(self, seq):
        return seq[self.randint(0, len(seq) - 1)]

    def weighted(self, items):
        tot = sum(w for _, w in items)
        r = self.random() * tot
        for it, w in items:
            r -= w
            if r < 0:
                return it
        return items[-1][0]


# --------------------------------------------------------------------------
# Minimal 6502 assembler (encoding only)
# --------------------------------------------------------------------------

# (mnemonic, addressing mode) -> opcode byte, from the public MOS 6502 opcode
# matrix.  The last group are the undocumented forms the paper's opcode set
# includes (LAX, SAX, the NOP family and the $EB alias of SBC #imm).
_OPC_ROWS = """
ADC imm 69 zp 65 zpx 75 abs 6D abx 7D aby 79 izx 61 izy 71
AND imm 29 zp 25 zpx 35 abs 2D abx 3D aby 39 izx 21 izy 31
ASL acc 0A zp 06 zpx 16 abs 0E abx 1E
BCC rel 90
BCS rel B0
BEQ rel F0
BMI rel 30
BNE rel D0
BPL rel 10
BVC rel 50
BVS rel 70
BIT zp 24 abs 2C
BRK imp 00
CLC imp 18
CLD imp D8
CLI imp 58
CLV imp B8
CMP imm C9 zp C5 zpx D5 abs CD abx DD aby D9 izx C1 izy D1
CPX imm E0 zp E4 abs EC
CPY imm C0 zp C4 abs CC
DEC zp C6 zpx D6 abs CE abx DE
DEX imp CA
DEY imp 88
EOR imm 49 zp 45 zpx 55 abs 4D abx 5D aby 59 izx 41 izy 51
INC zp E6 zpx F6 abs EE abx FE
INX imp E8
INY imp C8
JMP abs 4C ind 6C
JSR abs 20
LDA imm A9 zp A5 zpx B5 abs AD abx BD aby B9 izx A1 izy B1
LDX imm A2 zp A6 zpy B6 abs AE aby BE
LDY imm A0 zp A4 zpx B4 abs AC abx BC
LSR acc 4A zp 46 zpx 56 abs 4E abx 5E
NOP imp EA
ORA imm 09 zp 05 zpx 15 abs 0D abx 1D aby 19 izx 01 izy 11
PHA imp 48
PHP imp 08
PLA imp 68
PLP imp 28
ROL acc 2A zp 26 zpx 36 abs 2E abx 3E
ROR acc 6A zp 66 zpx 76 abs 6E abx 7E
RTI imp 40
RTS imp 60
SBC imm E9 zp E5 zpx F5 abs ED abx FD aby F9 izx E1 izy F1
SEC imp 38
SED imp F8
SEI imp 78
STA zp 85 zpx 95 abs 8D abx 9D aby 99 izx 81 izy 91
STX zp 86 zpy 96 abs 8E
STY zp 84 zpx 94 abs 8C
TAX imp AA
TAY imp A8
TSX imp BA
TXA imp 8A
TXS imp 9A
TYA imp 98
LAX zp A7 zpy B7 abs AF aby BF izx A3 izy B3
SAX zp 87 zpy 97 abs 8F izx 83
USBC imm EB
"""

OPCODES: dict[tuple[str, str], int] = {}
for _row in _OPC_ROWS.strip().splitlines():
    _f = _row.split()
    for _i in range(1, len(_f), 2):
        OPCODES[(_f[0], _f[_i])] = int(_f[_i + 1], 16)

# Undocumented NOPs by mode (opcode bytes).
NOP_IMP = [0x1A, 0x3A, 0x5A, 0x7A, 0xDA, 0xFA]
NOP_IMM = [0x80, 0x82, 0x89, 0xC2, 0xE2]
NOP_ZP = [0x04, 0x44, 0x64]
NOP_ZPX = [0x14, 0x34, 0x54, 0x74, 0xD4, 0xF4]
NOP_ABS = [0x0C]
NOP_ABX = [0x1C, 0x3C, 0x5C, 0x7C, 0xDC, 0xFC]

_MODE_LEN = {"imp": 1, "acc": 1, "imm": 2, "zp": 2, "zpx": 2, "zpy": 2, "rel": 2,
             "izx": 2, "izy": 2, "abs": 3, "abx": 3, "aby": 3, "ind": 3}

# Conservative cycle estimates used only to keep each scan line's code inside
# its 76-cycle budget (upper bounds: page-crossing and taken-branch penalties
# included).  Exact timing is the emulator's business, not the generator's.
_RMW = {"ASL", "LSR", "ROL", "ROR", "INC", "DEC"}
_STORE = {"STA", "STX", "STY", "SAX"}


def est_cycles(mn: str, mode: str) -> int:
    if mode in ("imp", "acc"):
        return {"PHA": 3, "PHP": 3, "PLA": 4, "PLP": 4, "RTS": 6, "RTI": 6,
                "BRK": 7}.get(mn, 2)
    if mode == "rel":
        return 4
    if mn == "JSR":
        return 6
    if mn == "JMP":
        return 3 if mode == "abs" else 5
    if mn in _RMW:
        return {"zp": 5, "zpx": 6, "abs": 6, "abx": 7}[mode]
    base = {"imm": 2, "zp": 3, "zpx": 4, "zpy": 4, "abs": 4, "abx": 5, "aby": 5,
            "izx": 6, "izy": 6}[mode]
    return base


# TIA / RIOT register addresses used by the generated programs.
VSYNC, VBLANK, WSYNC = 0x00, 0x01, 0x02
COLUP0, COLUP1, COLUPF, COLUBK, CTRLPF = 0x06, 0x07, 0x08, 0x09, 0x0A
PF0, PF1, PF2 = 0x0D, 0x0E, 0x0F
INPT4 = 0x0C
SWCHA, INTIM, TIM64T = 0x280, 0x284, 0x296


class Bank:
    """One 4 KB (or 2 KB) code window assembled at CPU base address ``base``."""

    def __init__(self, size: int, base: int, fill: bytes):
        self.size = size
        self.base = base
        self.img = bytearray(fill)
        self.pos = 0
        self.labels: dict[str, int] = {}
        self.fix: list[tuple[int, str, str]] = []
        self.used = bytearray(size)

    # -- placement
    def at(self, off: int):
        self.pos = off

    def addr(self) -> int:
        return self.base + self.pos

    def label(self, name: str):
        assert name not in self.labels, name
        self.labels[name] = self.addr()

    def byte(self, *bs: int):
        for b in bs:
            assert 0 <= self.pos < self.size, "bank overflow"
            assert not self.used[self.pos], f"overlap at {self.pos:#x}"
            self.img[self.pos] = b & 0xFF
            self.used[self.pos] = 1
            self.pos += 1

    def ins(self, mn: str, mode: str = "imp", arg=None) -> int:
        """Emit one instruction; returns the bank offset of its first operand byte."""
        op = OPCODES[(mn, mode)]
        self.byte(op)
        operand_at = self.pos
        n = _MODE_LEN[mode] - 1
        if n == 0:
            return operand_at
        if isinstance(arg, str):
            self.fix.append((self.pos, mode, arg))
            self.byte(*([0] * n))
        else:
            v = int(arg)
            if n == 1:
                self.byte(v & 0xFF)
            else:
                self.byte(v & 0xFF, (v >> 8) & 0xFF)
        return operand_at

    def raw(self, opcode: int, *operand: int):
        self.byte(opcode, *operand)

    def link(self, extern: dict[str, int] | None = None):
        for pos, mode, name in self.fix:
            tgt = self.labels.get(name)
            if tgt is None and extern is not None:
                tgt = extern[name]
            assert tgt is not None, name
            if mode == "rel":
                d = tgt - (self.base + pos + 1)
                assert -128 <= d <= 127, f"branch out of range to {name}"
                self.img[pos] = d & 0xFF
            elif _MODE_LEN[mode] == 2:
                self.img[pos] = tgt & 0xFF
            else:
                self.img[pos] = tgt & 0xFF
                self.img[pos + 1] = (tgt >> 8) & 0xFF


# --------------------------------------------------------------------------
# Synthetic program generator
# --------------------------------------------------------------------------

MAPPER_2K, MAPPER_4K, MAPPER_F8 = 0, 1, 2
MAPPER_OF_SIZE = {2048: MAPPER_2K, 4096: MAPPER_4K, 8192: MAPPER_F8}

LINE_BODY_BUDGET = 56  # cycles of per-line work before STA WSYNC


@dataclass
class Rom:
    seed: int
    size: int
    mapper: int
    image: np.ndarray                      # uint8 [size]
    colour_imm: list[int] = field(default_factory=list)  # image offsets of LDA #imm feeding only COLUBK/COLUPF
    reads_inputs: bool = False


class _Gen:
    def __init__(self, seed: int, size: int, reads_inputs: bool, timer_vblank: bool):
        self.r = Rng(stream_key(seed, 0x524F4D))
        self.seed = seed
        self.size = size
        self.mapper = MAPPER_OF_SIZE[size]
        self.inputs = reads_inputs
        self.timer = timer_vblank
        self.bank_size = 2048 if size == 2048 else 4096
        base = 0xF800 if size == 2048 else 0xF000
        nb = 2 if size == 8192 else 1
        fill = byte_stream(stream_key(seed, 0x46494C), size)
        self.banks = [Bank(self.bank_size, base, bytes(fill[i * self.bank_size:(i + 1) * self.bank_size]))
                      for i in range(nb)]
        self.colour_imm: list[tuple[int, int]] = []  # (bank, offset)
        self.n_label = 0
        # RAM plan: variables in $80-$DF, pointers at $E0-$E3, stack from $FF down.
        self.vars = sorted({0x80 + self.r.randint(0, 0x5F) for _ in range(24)})
        self.colour_vars = self.vars[: max(4, len(self.vars) // 3)]

    def lab(self, stem: str) -> str:
        self.n_label += 1
        return f"{stem}_{self.n_label}"

    def var(self) -> int:
        return self.r.choice(self.vars)

    def colour(self) -> int:
        return self.r.randint(0, 127) * 2

    # -- snippets: each returns (estimated cycles); emits into bank b
    def snip_kernel(self, b: Bank, bi: int, tables: dict) -> int:
        r = self.r
        kind = r.weighted([
            ("bk_imm", 10), ("pf_imm", 8), ("col_imm", 10), ("pf_tab", 8), ("col_tab", 6),
            ("col_ram", 8), ("tya_eor", 4), ("incdec", 6), ("adc", 3), ("sbc", 3), ("dec_adc", 3),
            ("logic", 3), ("shift", 3), ("eor_col", 3), ("branch", 6), ("bit_branch", 3),
            ("illegal", 4), ("indexed", 3), ("indirect", 3 if "ptr" in tables else 0),
            ("stack", 2), ("ctrlpf", 3), ("score_col", 2), ("cmp_branch", 2),
        ])
        c = 0
        if kind == "bk_imm" or kind == "col_imm":
            reg = COLUBK if kind == "bk_imm" else COLUPF
            off = b.ins("LDA", "imm", self.colour())
            self.colour_imm.append((bi, off))
            b.ins("STA", "zp", reg)
            c = 5
        elif kind == "pf_imm":
            b.ins("LDA", "imm", r.randint(0, 255))
            b.ins("STA", "zp", r.choice([PF0, PF1, PF2]))
            c = 5
        elif kind == "pf_tab":
            b.ins("LDA", "aby", tables["pf"])
            b.ins("STA", "zp", r.choice([PF0, PF1, PF2]))
            c = 7
        elif kind == "col_tab":
            b.ins("LDA", "aby", tables["col"])
            b.ins("STA", "zp", r.choice([COLUPF, COLUBK]))
            c = 7
        elif kind == "col_ram":
            b.ins("LDA", "zp", r.choice(self.colour_vars))
            b.ins("STA", "zp", r.choice([COLUPF, COLUBK]))
            c = 6
        elif kind == "tya_eor":
            b.ins("TYA")
            b.ins("EOR", "zp", self.var())
            b.ins("STA", "zp", COLUPF)
            c = 8
        elif kind == "incdec":
            b.ins(r.choice(["INC", "DEC"]), "zp", self.var())
            c = 5
        elif kind == "adc":
            v = self.var()
            b.ins("LDA", "zp", v)
            b.ins("CLC")
            b.ins("ADC", "imm", r.randint(0, 255))
            b.ins("STA", "zp", v)
            c = 10
        elif kind == "sbc":
            v = self.var()
            b.ins("SEC")
            b.ins("LDA", "zp", v)
            b.ins("SBC", "zp", self.var())
            b.ins("STA", "zp", v)
            c = 10
        elif kind == "dec_adc":
            v = self.var()
            b.ins("SED")
            b.ins(r.choice(["CLC", "SEC"]))
            b.ins("LDA", "zp", v)
            if r.random() < 0.5:
                b.ins("ADC", "imm", r.randint(0, 255))
            else:
                b.ins("SBC", "zp", self.var())
            b.ins("STA", "zp", v)
            b.ins("CLD")
            c = 15
        elif kind == "logic":
            v = self.var()
            b.ins("LDA", "zp", v)
            b.ins("AND", "imm", r.randint(0, 255))
            b.ins("ORA", "zp", self.var())
            b.ins("STA", "zp", v)
            c = 11
        elif kind == "shift":
            # right shifts only in per-line code: under the straight-through
            # rule a left shift doubles the gradient, and a variable shifted on
            # every one of 192 lines would grow its gradient like 2**192
            b.ins(r.choice(["LSR", "ROR"]), "zp", self.var())
            c = 5
        elif kind == "eor_col":
            b.ins("LDA", "zp", self.var())
            b.ins("EOR", "imm", r.randint(0, 255))
            b.ins("STA", "zp", COLUPF)
            c = 8
        elif kind == "branch":
            skip = self.lab("sk")
            b.ins("LDA", "zp", self.var())
            b.ins("AND", "imm", 1 << r.randint(0, 7))
            b.ins(r.choice(["BEQ", "BNE"]), "rel", skip)
            off = b.ins("LDA", "imm", self.colour())
            self.colour_imm.append((bi, off))
            b.ins("STA", "zp", COLUPF)
            b.label(skip)
            c = 15
        elif kind == "bit_branch":
            skip = self.lab("bb")
            b.ins("BIT", "zp", self.var())
            b.ins(r.choice(["BMI", "BPL", "BVC", "BVS"]), "rel", skip)
            b.ins("INC", "zp", self.var())
            b.label(skip)
            c = 12
        elif kind == "cmp_branch":
            skip = self.lab("cb")
            b.ins("LDA", "zp", self.var())
            b.ins("CMP", "imm", r.randint(0, 255))
            b.ins(r.choice(["BCC", "BCS"]), "rel", skip)
            b.ins("DEC", "zp", self.var())
            b.label(skip)
            c = 14
        elif kind == "illegal":
            sub = r.randint(0, 4)
            if sub == 0:
                b.ins("LAX", "zp", self.var())
                b.ins("STX", "zp", COLUPF)
                c = 6
            elif sub == 1:
                b.ins("LDX", "imm", r.randint(0, 255))
                b.ins("SAX", "zp", self.var())
                c = 5
            elif sub == 2:
                b.raw(r.choice(NOP_IMP))
                b.raw(r.choice(NOP_IMM), r.randint(0, 255))
                c = 4
            elif sub == 3:
                b.raw(r.choice(NOP_ZP), self.var())
                b.raw(r.choice(NOP_ZPX), self.var())
                c = 7
            else:
                b.ins("LDA", "zp", self.var())
                b.ins("USBC", "imm", r.randint(0, 255))
                b.ins("STA", "zp", self.var())
                c = 8
        elif kind == "indexed":
            b.ins("LDX", "imm", r.randint(0, 15))
            b.ins("LDA", "zpx", r.choice(self.colour_vars))
            b.ins("STA", "zp", r.choice([COLUBK, COLUPF]))
            c = 9
        elif kind == "indirect":
            b.ins("LDA", "izy", 0xE0)
            b.ins("STA", "zp", r.choice([PF1, PF2]))
            c = 9
        elif kind == "stack":
            b.ins("PHA")
            b.ins("LDA", "zp", self.var())
            b.ins("PLA")
            c = 10
        elif kind == "ctrlpf":
            b.ins("LDA", "imm", r.choice([0x00, 0x01, 0x02, 0x03, 0x05]))
            b.ins("STA", "zp", CTRLPF)
            c = 5
        elif kind == "score_col":
            b.ins("LDA", "imm", self.colour())
            b.ins("STA", "zp", r.choice([COLUP0, COLUP1]))
            c = 5
        return c

    def snip_logic(self, b: Bank, bi: int, budget: int) -> int:
        """Frame-logic work (VBLANK / overscan); no WSYNC inside."""
        r = self.r
        used = 0
        while True:
            kinds = [("incdec", 6), ("adc", 4), ("dec_adc", 3), ("logic", 3), ("shift", 3),
                     ("lax", 1), ("nop", 1), ("colvar", 3)]
            if self.inputs:
                kinds += [("swcha", 4), ("inpt4", 4), ("intim", 2)]
            kind = r.weighted(kinds)
            cost = {"incdec": 5, "adc": 10, "dec_adc": 15, "logic": 11, "shift": 5, "lax": 6,
                    "nop": 5, "colvar": 10, "swcha": 12, "inpt4": 12, "intim": 7}[kind]
            if used + cost > budget:
                return used
            used += cost
            if kind == "incdec":
                b.ins(r.choice(["INC", "DEC"]), "zp", self.var())
            elif kind == "adc":
                v = self.var()
                b.ins("LDA", "zp", v)
                b.ins(r.choice(["CLC", "SEC"]))
                b.ins(r.choice(["ADC", "SBC"]), "imm", r.randint(0, 255))
                b.ins("STA", "zp", v)
            elif kind == "dec_adc":
                v = self.var()
                b.ins("SED")
                b.ins("CLC")
                b.ins("LDA", "zp", v)
                b.ins(r.choice(["ADC", "SBC"]), "imm", r.randint(0, 255))
                b.ins("STA", "zp", v)
                b.ins("CLD")
            elif kind == "logic":
                v = self.var()
                b.ins("LDA", "zp", v)
                b.ins(r.choice(["AND", "ORA", "EOR"]), "zp", self.var())
                b.ins(r.choice(["AND", "ORA", "EOR"]), "imm", r.randint(0, 255))
                b.ins("STA", "zp", v)
            elif kind == "shift":
                b.ins(r.choice(["LSR", "ROR"]), "zp", self.var())
            elif kind == "lax":
                b.ins("LAX", "zp", self.var())
                b.ins("STA", "zp", self.var())
            elif kind == "nop":
                b.raw(r.choice(NOP_IMP))
                b.raw(r.choice(NOP_ZP), self.var())
            elif kind == "colvar":
                v = r.choice(self.colour_vars)
                b.ins("LDA", "zp", v)
                b.ins("CLC")
                b.ins("ADC", "imm", 2 * r.randint(1, 8))
                b.ins("STA", "zp", v)
            elif kind == "swcha":
                v = r.choice(self.colour_vars)
                b.ins("LDA", "abs", SWCHA)
                b.ins("AND", "imm", 0xF0)
                b.ins("EOR", "zp", v)
                b.ins("STA", "zp", v)
            elif kind == "inpt4":
                skip = self.lab("f")
                b.ins("LDA", "zp", INPT4)
                b.ins("BMI", "rel", skip)
                b.ins("INC", "zp", r.choice(self.colour_vars))
                b.label(skip)
            elif kind == "intim":
                b.ins("LDA", "abs", INTIM)
                b.ins("STA", "zp", self.var())

    def build(self) -> Rom:
        r = self.r
        nb = len(self.banks)
        bs = self.bank_size
        kb = self.banks[0]         # bank holding the kernel, overscan and tables
        mb = self.banks[-1]        # bank holding the reset target, VSYNC and VBLANK
        self._pending_subs = []
        # page-aligned data tables near the top of the kernel bank
        tables = {}
        tab_bytes = byte_stream(stream_key(self.seed, 0x544142), 512)
        tbl_pf_off = bs - 0x300 if bs == 4096 else bs - 0x200
        kb.at(tbl_pf_off)
        tables["pf"] = kb.addr()
        for i in range(256):
            kb.byte(int(tab_bytes[i]))
        if bs == 4096:
            kb.at(bs - 0x200)
            tables["col"] = kb.addr()
            for i in range(256):
                kb.byte(int(tab_bytes[256 + i]) & 0xFE)
        else:
            tables["col"] = tables["pf"]
        if r.random() < 0.6:
            tables["ptr"] = tables["pf"]

        # fixed offsets near the top of every bank
        t_to0 = bs - 0x40          # main bank: LDA $1FF8 ; kernel bank at +3: JMP KERNEL
        t_to1 = bs - 0x30          # kernel bank: LDA $1FF9 ; main bank at +3: JMP FRAME
        reset_off = bs - 0x20
        frame_addr = mb.base       # FRAME is assembled at offset 0 of the main bank

        # identical reset stubs in every bank, so the power-on bank is unobservable
        for b in self.banks:
            b.at(reset_off)
            b.label("RESET")
            b.ins("SEI")
            b.ins("CLD")
            b.ins("LDX", "imm", 0xFF)
            b.ins("TXS")
            if nb == 2:
                b.ins("LDA", "abs", 0x1FF9)
            b.ins("JMP", "abs", frame_addr)

        # ---- main bank: VSYNC + VBLANK
        b = mb
        bi = nb - 1
        b.at(0)
        b.label("FRAME")
        assert b.addr() == frame_addr
        b.ins("LDA", "imm", 0x02)
        b.ins("STA", "zp", VBLANK)
        b.ins("STA", "zp", VSYNC)
        for _ in range(3):
            b.ins("STA", "zp", WSYNC)
        b.ins("LDA", "imm", 0x00)
        b.ins("STA", "zp", VSYNC)
        for reg in (COLUP0, COLUP1):  # score-mode colours
            b.ins("LDA", "imm", self.colour())
            b.ins("STA", "zp", reg)
        if "ptr" in tables:
            b.ins("LDA", "imm", tables["ptr"] & 0xFF)
            b.ins("STA", "zp", 0xE0)
            b.ins("LDA", "imm", tables["ptr"] >> 8)
            b.ins("STA", "zp", 0xE1)
        if self.timer:
            # INTIM reaches 0 after (44 - 1) * 64 + 64 cycles ~ 36.2 lines
            b.ins("LDA", "imm", 44)
            b.ins("STA", "abs", TIM64T)
            for _ in range(r.randint(6, 14)):
                self.snip_logic(b, bi, 60)
            self._extras(b, bi)
            w = self.lab("w")
            b.label(w)
            b.ins("LDA", "abs", INTIM)
            b.ins("BNE", "rel", w)
        else:
            # line 0: the setup above; line 1: subroutine/BRK/indirect extras;
            # then frame-logic lines, then a WSYNC loop for the rest of VBLANK
            nlog = r.randint(3, 7)
            for i in range(nlog):
                if i == 1:
                    self._extras(b, bi)
                elif i > 1:
                    self.snip_logic(b, bi, 55)
                b.ins("STA", "zp", WSYNC)
            b.ins("LDX", "imm", 37 - nlog - 1)
            lp = self.lab("vbl")
            b.label(lp)
            b.ins("STA", "zp", WSYNC)
            b.ins("DEX")
            b.ins("BNE", "rel", lp)
        # the last VBLANK line is ended by the STA WSYNC at KERNEL
        if nb == 2:
            b.ins("JMP", "abs", b.base + t_to0)
            main_end = b.pos
            b.at(t_to0)
            b.ins("LDA", "abs", 0x1FF8)
            kb.at(t_to0 + 3)
            kb.ins("JMP", "abs", "KERNEL")
            kb.at(t_to1)
            kb.ins("LDA", "abs", 0x1FF9)
            b.at(t_to1 + 3)
            b.ins("JMP", "abs", frame_addr)
            k = kb
            k.at(0)
        else:
            main_end = None
            k = b
        kbi = 0
        k.label("KERNEL")
        k.ins("STA", "zp", WSYNC)
        k.ins("LDA", "imm", 0x00)
        k.ins("STA", "zp", VBLANK)
        # ---- kernel: bands of identical line bodies, 192 lines in total
        nbands = r.randint(2, 5)
        cuts = sorted({r.randint(8, 184) for _ in range(nbands - 1)})
        edges = [0] + cuts + [192]
        lines = [e1 - e0 for e0, e1 in zip(edges, edges[1:]) if e1 > e0]
        for n in lines:
            k.ins("LDY", "imm", n)
            lp = self.lab("band")
            k.label(lp)
            used = 0
            while True:
                save = (k.pos, len(k.fix), len(self.colour_imm), self.n_label, dict(k.labels),
                        bytes(k.used), bytes(k.img))
                c = self.snip_kernel(k, kbi, tables)
                if used + c > LINE_BODY_BUDGET:
                    pos, nf, nc, nl, labs, usedb, imgb = save
                    k.pos = pos
                    del k.fix[nf:]
                    del self.colour_imm[nc:]
                    self.n_label = nl
                    k.labels = labs
                    k.used = bytearray(usedb)
                    k.img = bytearray(imgb)
                    break
                used += c
                if used > LINE_BODY_BUDGET - 5:
                    break
            k.ins("STA", "zp", WSYNC)
            k.ins("DEY")
            k.ins("BNE", "rel", lp)
        # ---- overscan: 30 lines
        k.ins("LDA", "imm", 0x02)
        k.ins("STA", "zp", VBLANK)
        self.snip_logic(k, kbi, 50)
        k.ins("STA", "zp", WSYNC)
        k.ins("LDX", "imm", 29)
        lp = self.lab("os")
        k.label(lp)
        k.ins("STA", "zp", WSYNC)
        k.ins("DEX")
        k.ins("BNE", "rel", lp)
        if nb == 2:
            k.ins("JMP", "abs", k.base + t_to1)
        else:
            k.ins("JMP", "abs", frame_addr)
        # ---- subroutines and the BRK handler after the code of their bank
        ends = {kbi: k.pos}
        if main_end is not None:
            ends[nb - 1] = main_end
        for bank_i, name, body in self._pending_subs:
            bb = self.banks[bank_i]
            bb.at(ends[bank_i])
            bb.label(name)
            body(bb)
            ends[bank_i] = bb.pos
        # ---- vectors (reset at $FFFC, IRQ/BRK at $FFFE)
        for bb in self.banks:
            bb.at(bs - 4)
            rs = bb.labels["RESET"]
            bb.byte(rs & 0xFF, rs >> 8)
            brk = bb.labels.get("BRKH", rs)
            bb.byte(brk & 0xFF, brk >> 8)
        for bb in self.banks:
            bb.link()
        img = np.frombuffer(b"".join(bytes(bb.img) for bb in self.banks), dtype=np.uint8).copy()
        assert img.size == self.size
        offs = [bi2 * bs + off for bi2, off in self.colour_imm]
        return Rom(seed=self.seed, size=self.size, mapper=self.mapper, image=img,
                   colour_imm=offs, reads_inputs=self.inputs)

    def _extras(self, b: Bank, bi: int):
        """Occasional subroutine call, BRK/RTI round trip and indirect jump."""
        r = self.r
        if r.random() < 0.8:
            name = self.lab("sub")
            v = self.var()
            inc = r.choice(["INC", "DEC"])
            acc = self.vars[0]

            def body(bb, v=v, inc=inc, acc=acc):
                bb.ins(inc, "zp", v)
                bb.ins("LDA", "zp", v)
                bb.ins("ROL", "acc")
                bb.ins("EOR", "zp", acc)
                bb.ins("STA", "zp", acc)
                bb.ins("RTS")
            b.ins("JSR", "abs", name)
            self._pending_subs.append((bi, name, body))
        if r.random() < 0.4 and "BRKH" not in b.labels:
            v = self.var()

            def brk_body(bb, v=v):
                bb.ins("INC", "zp", v)
                bb.ins("RTI")
            b.ins("BRK")
            b.byte(0xEA)  # padding byte skipped by the pushed return address
            self._pending_subs.append((bi, "BRKH", brk_body))
        if r.random() < 0.4:
            tgt = self.lab("ij")
            lo_at = b.ins("LDA", "imm", 0)
            b.ins("STA", "zp", 0xE2)
            hi_at = b.ins("LDA", "imm", 0)
            b.ins("STA", "zp", 0xE3)
            b.ins("JMP", "ind", 0x00E2)
            b.label(tgt)
            t = b.labels[tgt]
            b.img[lo_at] = t & 0xFF
            b.img[hi_at] = t >> 8


def generate_rom(seed: int, size: int = 4096, *, reads_inputs: bool = False,
                 timer_vblank: bool = False) -> Rom:
    """Assemble one synthetic cartridge (2048, 4096 or 8192 bytes)."""
    assert size in (2048, 4096, 8192)
    return _Gen(seed, size, reads_inputs, timer_vblank).build()


def perturb_rom(rom: Rom, seed: int, n: int = 8) -> np.ndarray:
    """Copy of the image with ``n`` seeded colour immediates replaced by new even bytes.

    Only immediates of ``LDA #imm`` that feed a ``STA COLUBK`` / ``STA COLUPF``
    are touched, so control flow is unchanged and only colours differ.
    """
    img = rom.image.copy()
    cand = list(rom.colour_imm)
    r = Rng(stream_key(seed, 0x505254, rom.seed))
    chosen = []
    while cand and len(chosen) < n:
        chosen.append(cand.pop(r.randint(0, len(cand) - 1)))
    for off in chosen:
        old = int(img[off])
        new = old
        while new == old:
            new = r.randint(0, 127) * 2
        img[off] = new
    return img


# --------------------------------------------------------------------------
# Per-env data
# --------------------------------------------------------------------------

N_ACTIONS = 18


def initial_ram(seed: int, num_envs: int) -> np.ndarray:
    """Uniform random power-on RAM, uint8 [B][128]."""
    return byte_stream(stream_key(seed, 0x52414D), num_envs * 128).reshape(num_envs, 128)


def action_stream(seed: int, num_envs: int, steps: int) -> np.ndarray:
    """Uniform joystick actions over the 18 ALE actions, uint8 [B][S]."""
    return int_stream(stream_key(seed, 0x414354), num_envs * steps, N_ACTIONS).astype(np.uint8).reshape(num_envs, steps)


def episode_steps(seed: int, num_envs: int, total_steps: int, frame_skip: int,
                  mean_frames: float = 1500.0) -> np.ndarray:
    """Episode lengths in env-steps, uint32 [B][E].

    Frames per episode are Geometric(p = 1/mean_frames) on {1, 2, ...}
    (inverse-CDF sampling); an episode ends after ceil(L / frame_skip) steps.
    Enough episodes are drawn for every env to cover ``total_steps``.
    """
    p = 1.0 / mean_frames
    lp = math.log1p(-p)
    cols = []
    covered = np.zeros(num_envs, dtype=np.int64)
    e = 0
    while (covered < total_steps).any() or e == 0:
        u = unit_stream(stream_key(seed, 0x455049, e), num_envs)
        frames = np.maximum(1, np.ceil(np.log1p(-u) / lp)).astype(np.int64)
        st = (frames + frame_skip - 1) // frame_skip
        cols.append(st)
        covered += st
        e += 1
    return np.stack(cols, axis=1).astype(np.uint32)


# --------------------------------------------------------------------------
# Soft-mode leaves
# --------------------------------------------------------------------------


def rom_logits(image: np.ndarray, seed: int, sigma: float = 0.1) -> np.ndarray:
    """float32 [size][256]: one-hot of the ROM bytes plus N(0, sigma^2) noise."""
    n = image.size
    noise = normal_stream(stream_key(seed, 0x4C4F47), n * 256).reshape(n, 256) * sigma
    out = noise
    out[np.arange(n), image.astype(np.int64)] += 1.0
    return out.astype(np.float32)


def ram_tape(ram0: np.ndarray) -> np.ndarray:
    """float32 [B][128][256]: one-hot content rows of the initial RAM bytes."""
    b = ram0.shape[0]
    t = np.zeros((b, 128, 256), dtype=np.float32)
    t[np.arange(b)[:, None], np.arange(128)[None, :], ram0.astype(np.int64)] = 1.0
    return t


def action_logits(actions: np.ndarray, seed: int, sigma: float = 0.1) -> np.ndarray:
    """float32 [B][S][18]: one-hot of the hard actions plus N(0, sigma^2) noise."""
    b, s = actions.shape
    noise = normal_stream(stream_key(seed, 0x414C47), b * s * N_ACTIONS).reshape(b, s, N_ACTIONS) * sigma
    noise[np.arange(b)[:, None], np.arange(s)[None, :], actions.astype(np.int64)] += 1.0
    return noise.astype(np.float32)


# --------------------------------------------------------------------------
# Workload configurations
# --------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    roms: list[Rom]
    env_rom: np.ndarray          # int32 [B]
    ram0: np.ndarray             # uint8 [B][128]
    actions: np.ndarray | None   # uint8 [B][S] or None (no input: NOOP)
    steps: int
    frame_skip: int
    episode_steps: np.ndarray | None = None  # uint32 [B][E]
    seed: int = 0

    @property
    def num_envs(self) -> int:
        return int(self.env_rom.size)

    def rom_concat(self) -> np.ndarray:
        return np.concatenate([r.image for r in self.roms])

    def rom_offsets(self) -> np.ndarray:
        return np.cumsum([0] + [r.size for r in self.roms])[:-1].astype(np.int64)

    def actions_or_noop(self) -> np.ndarray:
        if self.actions is not None:
            return self.actions
        return np.zeros((self.num_envs, self.steps), dtype=np.uint8)


def config_c0() -> Workload:
    """1 instance, one 4 KB ROM, 60 frames at frame-skip 1, no input."""
    rom = generate_rom(0, 4096)
    return Workload("c0_single_4k_60f", [rom], np.zeros(1, np.int32), initial_ram(0, 1),
                    None, steps=60, frame_skip=1, seed=0)


def config_c1(num_envs: int = 4096, steps: int = 500) -> Workload:
    """4096 instances of one 4 KB ROM, uniform actions, frame-skip 4, 2000 frames."""
    rom = generate_rom(1, 4096)
    return Workload("c1_batched_4k", [rom], np.zeros(num_envs, np.int32), initial_ram(1, num_envs),
                    action_stream(1, num_envs, steps), steps=steps, frame_skip=4, seed=1)


def c2_roms(n_roms: int = 64) -> list[Rom]:
    sizes = [2048] * 21 + [4096] * 22 + [8192] * 21
    sizes = sizes[:n_roms] if n_roms <= 64 else sizes * (n_roms // 64 + 1)
    order = np.argsort(unit_stream(stream_key(2, 0x4D4958), len(sizes)), kind="stable")
    sizes = [sizes[i] for i in order][:n_roms]
    return [generate_rom(100 + i, sizes[i], reads_inputs=True, timer_vblank=True)
            for i in range(n_roms)]


def config_c2(envs_per_rom: int = 256, steps: int = 500, n_roms: int = 64) -> Workload:
    """64 mixed ROMs x 256 envs, geometric episode lengths with in-run resets."""
    roms = c2_roms(n_roms)
    b = n_roms * envs_per_rom
    env_rom = np.repeat(np.arange(n_roms, dtype=np.int32), envs_per_rom)
    perm = np.argsort(unit_stream(stream_key(2, 0x50524D), b), kind="stable")
    env_rom = env_rom[perm].astype(np.int32)
    return Workload("c2_hetero_persistent", roms, env_rom, initial_ram(2, b),
                    action_stream(2, b, steps), steps=steps, frame_skip=4,
                    episode_steps=episode_steps(2, b, steps, 4), seed=2)


def config_c3(num_envs: int = 256) -> Workload:
    """Soft small: 256 envs of the C1 ROM, 2 frames at frame-skip 1."""
    rom = generate_rom(1, 4096)
    return Workload("c3_soft_small", [rom], np.zeros(num_envs, np.int32), initial_ram(3, num_envs),
                    action_stream(3, num_envs, 2), steps=2, frame_skip=1, seed=3)


def config_c4(envs_per_rom: int = 64, steps: int = 60, n_roms: int = 64) -> Workload:
    """Soft at scale: the heterogeneous ROM mix x 64 envs, 60 frames, no resets."""
    roms = c2_roms(n_roms)
    b = n_roms * envs_per_rom
    env_rom = np.repeat(np.arange(n_roms, dtype=np.int32), envs_per_rom)
    return Workload("c4_soft_scale", roms, env_rom, initial_ram(4, b),
                    action_stream(4, b, steps), steps=steps, frame_skip=1, seed=4)


@dataclass
class SoftLeaves:
    rom_logits: np.ndarray       # float32 [sum sizes][256]
    ram_tape: np.ndarray         # float32 [B][128][256]
    action_logits: np.ndarray    # float32 [B][S][18]
    perturbed_roms: list[np.ndarray]


def soft_leaves(w: Workload, seed: int | None = None) -> SoftLeaves:
    s = w.seed if seed is None else seed
    logits = np.concatenate([rom_logits(r.image, stream_key(s, 0x4C, i)) for i, r in enumerate(w.roms)])
    return SoftLeaves(rom_logits=logits, ram_tape=ram_tape(w.ram0),
                      action_logits=action_logits(w.actions_or_noop(), s),
                      perturbed_roms=[perturb_rom(r, s) for r in w.roms])


CONFIGS = {"c0": config_c0, "c1": config_c1, "c2": config_c2, "c3": config_c3, "c4": config_c4}


# --------------------------------------------------------------------------
# Opcode-sweep programs: every byte of the instruction set, every addressing
# form, page crossings, read-modify-write on RAM / TIA / RIOT, every timer
# interval, code in RAM.  A parity workload, not a performance one.
# --------------------------------------------------------------------------

def instruction_set() -> dict[int, tuple[str, str]]:
    """opcode byte -> (mnemonic, mode) for the 189 bytes of the paper's set."""
    ops = {op: mm for mm, op in OPCODES.items()}
    for lst, mode in ((NOP_IMP, "imp"), (NOP_IMM, "imm"), (NOP_ZP, "zp"), (NOP_ZPX, "zpx"), (NOP_ABS, "abs"),
                      (NOP_ABX, "abx")):
        for op in lst:
            ops[op] = ("NOP", mode)
    return ops


# RIOT registers (13-bit addresses; A2 = timer, A0 = TIMINT on reads, A4 = timer write)
TIM1T, TIM8T, T1024T, TIMINT = 0x294, 0x295, 0x297, 0x285


class _SweepGen:
    """One seeded opcode-sweep program.

    RAM plan: $80-$9F chain variables (the initial RAM, rewritten by the
    results), $A0-$A7 four pointers, $A8-$C7 a window for indexed writes,
    $C8-$CF flag accumulators, $D0-$D7 code written at run time, $D8-$FF the
    stack.  Values loaded from the variables steer the index registers, so
    envs with different RAM take different addresses, page crossings and
    branch directions; results are folded back into the variables, so an
    error anywhere reaches the RAM and the frame."""

    VAR0, NVAR, PTR, WIN, ACC, RAMCODE = 0x80, 32, 0xA0, 0xA8, 0xC8, 0xD0

    def __init__(self, seed: int, size: int, soft_safe: bool, objects: bool = True):
        self.r = Rng(stream_key(seed, 0x535750))
        self.seed, self.size, self.soft_safe = seed, size, soft_safe
        # objects=False: no access reaches a register only the TIA's objects use
        # (no collision reads, no object-register writes); the same random draws
        self.objects = objects
        self.bank_size = 2048 if size == 2048 else 4096
        self.base = 0xF800 if size == 2048 else 0xF000
        self.n_label = 0

    # ---- helpers
    def lab(self, stem: str) -> str:
        self.n_label += 1
        return f"{stem}_{self.n_label}"

    def var(self) -> int:
        return self.VAR0 + self.r.randint(0, self.NVAR - 1)

    def acc(self) -> int:
        return self.ACC + self.r.randint(0, 7)

    def idx_reg(self, b: Bank, reg: str, lo: int, span: int):
        """Load X or Y with lo + (a variable & (span-1)): per-env values in [lo, lo+span)."""
        b.ins("LDA", "zp", self.var())
        b.ins("AND", "imm", span - 1)
        if lo:
            b.ins("ORA", "imm", lo) if (lo & (span - 1)) == 0 else b.ins("ADC", "imm", lo)
        b.ins("TAX" if reg == "X" else "TAY")

    def setup_flags(self, b: Bank, decimal_ok: bool = True):
        r = self.r
        b.ins(r.choice(["CLC", "SEC"]))
        if decimal_ok and r.random() < 0.3:
            b.ins("SED")
        else:
            b.ins("CLD")

    def fold_flags(self, b: Bank):
        """Fold the status byte into an accumulator cell (no decimal adds: EOR)."""
        if self.r.random() < 0.5:
            return
        a = self.acc()
        b.ins("PHP")
        b.ins("PLA")
        b.ins("EOR", "zp", a)
        b.ins("STA", "zp", a)

    def save_a(self, b: Bank):
        b.ins("STA", "zp", self.var())

    def set_ptr(self, b: Bank, k: int, addr: int):
        b.ins("LDA", "imm", addr & 0xFF)
        b.ins("STA", "zp", self.PTR + 2 * k)
        b.ins("LDA", "imm", (addr >> 8) & 0xFF)
        b.ins("STA", "zp", self.PTR + 2 * k + 1)

    def op(self, b: Bank, opc: int, operand: int | None, mode: str):
        n = _MODE_LEN[mode] - 1
        if n == 0:
            b.raw(opc)
        elif n == 1:
            b.raw(opc, operand & 0xFF)
        else:
            b.raw(opc, operand & 0xFF, (operand >> 8) & 0xFF)

    # ---- operands by access kind: (address or operand, needs index setup)
    def read_target_zp(self) -> int:
        r = self.r
        k = r.weighted([("var", 7), ("tia", 2), ("win", 1)])
        if k == "var":
            return self.var()
        if k == "win":
            return self.WIN + r.randint(0, 31)
        cx = (0x00, 0x07) if self.objects else (0x08, 0x0F)
        return r.choice([INPT4, 0x0D, 0x3C, 0x2D, cx[0], cx[1], 0x1C])  # INPT4/5, mirrors, collisions

    def wraps_to_tia(self, base: int, span: int) -> bool:
        """objects=False: base + [0, span) past $FFFF wraps onto page 0, the TIA's
        collision latches among it."""
        return not self.objects and base + span - 1 > 0xFFFF

    def rmw_safe(self, a: int, rmw: bool) -> int:
        """objects=False: a read-modify-write of a TIA address also reads its read
        register, a collision latch for registers 0-7: use COLUPF/COLUBK instead."""
        if self.objects or not rmw or (a & 0x1080) or (a & 0xF) >= 8:
            return a
        return 0x08 | (a & 1)

    def write_target_zp(self) -> int:
        r = self.r
        k = r.weighted([("var", 5), ("win", 2), ("tia", 3)])
        if k == "var":
            return self.var()
        if k == "win":
            return self.WIN + r.randint(0, 31)
        return r.choice([COLUBK, COLUPF, COLUP0, COLUP1, PF0, PF1, PF2, CTRLPF, WSYNC, 0x49, 0x48, 0x03,
                         0x1F if self.objects else 0x2D])

    def read_target_abs(self, tables) -> int:
        r = self.r
        k = r.weighted([("ram", 3), ("mirror", 1), ("tia", 1), ("riot", 3), ("rom", 3)])
        if k == "ram":
            return self.var()
        if k == "mirror":
            return 0x100 | self.var()           # the stack page mirrors RAM
        if k == "tia":
            return r.choice([0x000C, 0x010C, 0x003D, 0x0105 if self.objects else 0x010D,
                             0x0040 if self.objects else 0x0048])
        if k == "riot":
            return r.choice([SWCHA, 0x281, 0x282, 0x283, INTIM, TIMINT, 0x286, 0x287, 0x2A4, 0x285])
        return tables[r.randint(0, len(tables) - 1)] + r.randint(0, 255)

    def write_target_abs(self) -> int:
        r = self.r
        k = r.weighted([("ram", 3), ("mirror", 1), ("tia", 3), ("riot", 2), ("rom", 1)])
        if k == "ram":
            return self.var()
        if k == "mirror":
            return 0x100 | (self.WIN + r.randint(0, 31))
        if k == "tia":
            return r.choice([0x0009, 0x0008, 0x0108, 0x004E, 0x000D, 0x000F, 0x0002,
                             0x0006 if self.objects else 0x000A])
        if k == "riot":
            return r.choice([TIM1T, TIM8T, TIM64T, T1024T, 0x29C, 0x29F, 0x280, 0x281])
        return self.base + r.randint(0, 0x7FF)  # cartridge: no effect

    # ---- one instruction of the set, with its operand set up and its result folded
    def emit(self, b: Bank, opc: int, mn: str, mode: str, tables, cross: bool | None = None):
        """cross (indexed forms): True = an address range some envs cross a page
        in, False = one no env crosses in, None = either."""
        r = self.r
        load = mn in ("LDA", "LDX", "LDY", "LAX", "ADC", "SBC", "AND", "ORA", "EOR", "CMP", "CPX", "CPY", "BIT",
                      "USBC") or (mn == "NOP" and mode != "imp")
        store = mn in ("STA", "STX", "STY", "SAX")
        rmw = mn in ("ASL", "LSR", "ROL", "ROR", "INC", "DEC")
        if mode == "rel":
            return self.emit_branch(b, opc, mn)
        if mode in ("imp", "acc") or mn in ("JMP", "JSR"):
            return self.emit_implied(b, opc, mn, mode)
        # registers the instruction reads besides the operand
        if mn in ("ADC", "SBC", "USBC"):
            self.setup_flags(b)
        elif mn in ("ROL", "ROR"):
            self.setup_flags(b, decimal_ok=False)
        # the address
        operand = 0
        if mode == "imm":
            operand = r.randint(0, 255)
        elif mode == "zp":
            operand = self.rmw_safe(self.write_target_zp(), rmw) if (store or rmw) else self.read_target_zp()
        elif mode in ("zpx", "zpy"):
            reg = "X" if mode == "zpx" else "Y"
            if r.random() < 0.35:  # wraps inside page 0, onto TIA registers $00-$0F (reads: collisions, INPT4)
                if self.objects:
                    self.idx_reg(b, reg, 0x10, 16)
                else:  # $08-$0F: reads INPT0-5; writes COLUPF/COLUBK
                    self.idx_reg(b, reg, 0x18, 2 if (store or rmw) else 8)
                operand = 0xF0
            else:
                self.idx_reg(b, reg, 0, 32)
                operand = (self.WIN if (store or rmw) else self.VAR0)
        elif mode == "abs":
            operand = self.rmw_safe(self.write_target_abs(), rmw) if (store or rmw) else self.read_target_abs(tables)
        elif mode in ("abx", "aby"):
            reg = "X" if mode == "abx" else "Y"
            kinds = [("ram", 3 if cross is not True else 0), ("cross_tia", 2 if cross is not False else 0),
                     ("rom", 3 if not (store or rmw) and cross is not False else 0),
                     ("riot", 1 if not rmw and cross is not True else 0)]
            kind = r.weighted(kinds)
            if kind == "ram":      # $A8 + [0, 32): no crossing
                self.idx_reg(b, reg, 0, 32)
                operand = self.WIN if (store or rmw) else self.VAR0
            elif kind == "cross_tia":
                # $F8 + [0, 16): some envs cross into $0100-$0107 (TIA mirror).  Between
                # snippets the stack is empty (S = $FF), so $F8-$FF hold nothing live.
                if self.objects:
                    self.idx_reg(b, reg, 0, 16)
                    operand = 0x00F8
                else:  # stores cross onto VSYNC/VBLANK only; loads and RMW stay in $F8-$FF
                    self.idx_reg(b, reg, 0, 8)
                    operand = 0x00FA if store else 0x00F8
            elif kind == "rom":    # a table near a page end: some envs cross
                if self.wraps_to_tia(tables[0] + 0xF0, 64):  # $FFF8 + [$10, $18): $0008-$000F
                    self.idx_reg(b, reg, 0x10, 8)
                    r.randint(0xE0, 0xF0)
                    operand = 0xFFF8
                else:
                    self.idx_reg(b, reg, 0, 64)
                    operand = tables[0] + r.randint(0xE0, 0xF0)
            else:                  # RIOT registers $0280-$0287 (ports, INTIM, TIMINT) or timer writes
                self.idx_reg(b, reg, 0, 8)
                operand = 0x0290 if store else 0x0280
        elif mode in ("izx", "izy"):
            targets = [self.var(), self.read_target_abs(tables) if not (store or rmw)
                       else self.rmw_safe(self.write_target_abs(), rmw),
                       self.WIN + r.randint(0, 8), r.choice([INTIM, COLUBK, COLUPF, SWCHA])]
            if mode == "izx":
                for k in range(4):
                    self.set_ptr(b, k, targets[k])
                b.ins("LDA", "zp", self.var())
                b.ins("AND", "imm", 3)
                b.ins("ASL", "acc")
                b.ins("TAX")
                operand = self.PTR
            else:
                k = r.randint(0, 3)
                kind = r.weighted([("rom", 3 if not store and cross is not False else 0),
                                   ("win", 2 if cross is not True else 0), ("cross", 1 if cross is not False else 0)])
                if kind == "rom":
                    base = tables[0] + r.randint(0xE0, 0xF0)
                    if self.wraps_to_tia(base, 64):  # $FFF8 + [$10, $18): $0008-$000F
                        self.set_ptr(b, k, 0xFFF8)
                        self.idx_reg(b, "Y", 0x10, 8)
                    else:
                        self.set_ptr(b, k, base)
                        self.idx_reg(b, "Y", 0, 64)
                elif kind == "win":
                    self.set_ptr(b, k, self.WIN)
                    self.idx_reg(b, "Y", 0, 32)
                elif self.objects:  # $F8 + Y: some envs cross into the TIA mirror $0100-$0107
                    self.set_ptr(b, k, 0x00F8)
                    self.idx_reg(b, "Y", 0, 16)
                else:
                    self.set_ptr(b, k, 0x00FA if store else 0x00F8)
                    self.idx_reg(b, "Y", 0, 8)
                operand = self.PTR + 2 * k
        # the accumulator / X operand of the instruction
        if mn in ("STX", "CPX"):
            if mode in ("abx", "zpx", "izx"):
                pass
            elif mode in ("zpy", "aby", "izy"):
                b.ins("LDX", "zp", self.var())
            else:
                b.ins("LDX", "zp", self.var())
        elif mn in ("STY", "CPY"):
            if mode not in ("zpy", "aby", "izy", "zpx", "abx", "izx"):
                b.ins("LDY", "zp", self.var())
        if mn not in ("LDA", "LAX", "LDX", "LDY") and not (rmw and mode == "acc"):
            b.ins("LDA", "zp", self.var())
        if mn == "SAX" and mode in ("zp", "abs"):
            b.ins("LDX", "zp", self.var())
        self.op(b, opc, operand, mode)
        # fold the results back
        if mn in ("LDA", "LAX", "ADC", "SBC", "USBC", "AND", "ORA", "EOR"):
            self.save_a(b)
        if mn in ("LDX", "LAX"):
            b.ins("STX", "zp", self.var())
        if mn == "LDY":
            b.ins("STY", "zp", self.var())
        if mn in ("ADC", "SBC", "USBC"):
            b.ins("CLD")
        if not store:
            self.fold_flags(b)

    def branch_cond(self, b: Bank, mn: str):
        """Flags for branch mn from a variable: taken for some envs, not for others."""
        r = self.r
        flag = {"BPL": "N", "BMI": "N", "BVC": "V", "BVS": "V", "BCC": "C", "BCS": "C", "BNE": "Z", "BEQ": "Z"}[mn]
        v = self.var()
        if flag == "N":
            b.ins("LDA", "zp", v)
        elif flag == "Z":
            b.ins("LDA", "zp", v)
            b.ins("AND", "imm", 1 << r.randint(0, 7))
        elif flag == "C":
            b.ins("LDA", "zp", v)
            b.ins("CMP", "imm", r.randint(0, 255))
        else:
            b.ins("BIT", "zp", v)

    def emit_branch(self, b: Bank, opc: int, mn: str):
        r = self.r
        self.branch_cond(b, mn)
        skip = self.lab("br")
        b.raw(opc, 0)
        b.fix.append((b.pos - 1, "rel", skip))
        b.ins("INC", "zp", self.var())
        b.label(skip)

    def page_end(self, b: Bank):
        """Near a page end, a branch across it: forward (a data-dependent
        condition; the taken path lands in the next page) or backward (a count
        loop whose head lies in the previous page)."""
        r = self.r
        if (b.pos & 0xFF) < 0xE0 or (b.pos & 0xFF) > 0xF5:
            return
        if r.random() < 0.8:
            mn = ["BPL", "BMI", "BVC", "BVS", "BCC", "BCS", "BNE", "BEQ"][self.n_cross % 8]
            self.n_cross += 1
            self.branch_cond(b, mn)
            while (b.pos & 0xFF) != 0xFC:
                b.byte(0xEA)
            b.ins(mn, "rel", 0)
            b.img[b.pos - 1] = 0x02  # over the next two bytes, into the next page
            b.ins("INC", "zp", self.var())
        else:
            b.ins("LDA", "zp", self.var())
            b.ins("AND", "imm", 7)
            b.ins("TAX")
            b.ins("INX")
            while (b.pos & 0xFF) != 0xFE:
                b.byte(0xEA)
            b.ins("DEX")  # the loop head, last byte of the page
            b.ins("NOP")
            b.ins("BNE", "rel", 0)
            b.img[b.pos - 1] = (-4) & 0xFF  # back to the DEX, across the page boundary
            b.ins("STX", "zp", self.var())

    def emit_implied(self, b: Bank, opc: int, mn: str, mode: str):
        r = self.r
        if mn in ("ASL", "LSR", "ROL", "ROR"):  # accumulator forms
            b.ins("LDA", "zp", self.var())
            if mn in ("ROL", "ROR"):
                self.setup_flags(b, decimal_ok=False)
            b.raw(opc)
            self.save_a(b)
            self.fold_flags(b)
        elif mn in ("TAX", "TAY"):
            b.ins("LDA", "zp", self.var())
            b.raw(opc)
            b.ins("STX" if mn == "TAX" else "STY", "zp", self.var())
            self.fold_flags(b)
        elif mn in ("TXA", "TYA"):
            b.ins("LDX" if mn == "TXA" else "LDY", "zp", self.var())
            b.raw(opc)
            self.save_a(b)
            self.fold_flags(b)
        elif mn in ("INX", "DEX", "INY", "DEY"):
            reg = "X" if mn in ("INX", "DEX") else "Y"
            b.ins("LDX" if reg == "X" else "LDY", "zp", self.var())
            b.raw(opc)
            b.ins("STX" if reg == "X" else "STY", "zp", self.var())
            self.fold_flags(b)
        elif mn in ("CLC", "SEC", "CLD", "SED", "CLI", "SEI", "CLV", "NOP"):
            if mn == "CLV":  # set V first: BIT of a byte with bit 6 set
                b.ins("BIT", "abs", 0x0282 if r.random() < 0.5 else SWCHA)
            b.raw(opc)
            self.fold_flags(b)
            if mn == "SED":
                b.ins("CLD")
        elif mn == "TSX":
            b.raw(opc)
            b.ins("STX", "zp", self.var())
        elif mn == "TXS":
            # move the stack into $F0-$FF, push and pull there, then onto the TIA
            # colour registers ($06-$09: pushes draw), and back
            b.ins("TSX")
            b.ins("STX", "zp", self.ACC + 7)
            b.ins("LDA", "zp", self.var())
            b.ins("ORA", "imm", 0xF0)
            b.ins("TAX")
            b.raw(opc)
            b.ins("LDA", "zp", self.var())
            b.ins("PHA")
            b.ins("PLA")
            b.ins("LDX", "imm", r.choice([0x07, 0x08, 0x09]))
            b.raw(opc)
            b.ins("LDA", "zp", self.var())
            b.ins("PHA")
            b.ins("PHP")
            b.ins("LDX", "zp", self.ACC + 7)
            b.raw(opc)
        elif mn == "PHA":
            b.ins("LDA", "zp", self.var())
            b.raw(opc)
            b.ins("LDA", "zp", self.var())
            b.ins("PLA")
            self.save_a(b)
        elif mn == "PLA":
            b.ins("LDA", "zp", self.var())
            b.ins("PHA")
            b.ins("LDA", "imm", r.randint(0, 255))
            b.raw(opc)
            self.save_a(b)
            self.fold_flags(b)
        elif mn == "PHP":
            b.ins("LDA", "zp", self.var())  # N, Z from a variable
            b.raw(opc)
            b.ins("PLA")
            self.save_a(b)
        elif mn == "PLP":
            b.ins("LDA", "zp", self.var())
            b.ins("PHA")
            b.raw(opc)            # any flags, D and I included
            self.fold_flags(b)
            b.ins("CLD")
        elif mn == "JMP" and mode == "abs":
            t = self.lab("jmp")
            b.raw(opc, 0, 0)
            b.fix.append((b.pos - 2, "abs", t))
            b.ins("INC", "zp", self.var())  # skipped
            b.label(t)
        elif mn == "JMP":  # (ind): through a RAM pointer, and through the table's page-wrapping pair
            t1, t2 = self.lab("ji"), self.lab("jw")
            b.ins("LDA", "imm", 0)
            lo_at = b.pos - 1
            b.ins("STA", "zp", self.PTR + 6)
            b.ins("LDA", "imm", 0)
            hi_at = b.pos - 1
            b.ins("STA", "zp", self.PTR + 7)
            b.raw(opc, self.PTR + 6, 0x00)
            b.ins("INC", "zp", self.var())  # skipped
            b.label(t1)
            self._late.append((lo_at, hi_at, t1))
            if self.wrap_page is not None:
                b.raw(opc, 0xFF, (self.wrap_page >> 8) & 0xFF)  # JMP ($xxFF): high byte from $xx00
                b.ins("INC", "zp", self.var())  # skipped
                b.label(t2)
                self.wrap_target = t2
        elif mn == "JSR":
            b.raw(opc, 0, 0)
            b.fix.append((b.pos - 2, "abs", "SUB"))
            self.fold_flags(b)
            # and a call of code written into RAM: LDA #v ; RTS
            b.ins("LDA", "imm", 0xA9)
            b.ins("STA", "zp", self.RAMCODE)
            b.ins("LDA", "zp", self.var())
            b.ins("STA", "zp", self.RAMCODE + 1)
            b.ins("LDA", "imm", 0x60)
            b.ins("STA", "zp", self.RAMCODE + 2)
            b.raw(opc, self.RAMCODE, 0x00)
            self.save_a(b)
        elif mn == "RTS":  # a computed jump: push target - 1, return
            t = self.lab("rts")
            b.ins("LDA", "imm", 0)
            hi_at = b.pos - 1
            b.ins("PHA")
            b.ins("LDA", "imm", 0)
            lo_at = b.pos - 1
            b.ins("PHA")
            b.raw(opc)
            b.ins("INC", "zp", self.var())  # skipped
            b.label(t)
            self._late.append((lo_at, hi_at, t, -1))
        elif mn == "RTI":  # a pushed frame: PCH, PCL, P
            t = self.lab("rti")
            b.ins("LDA", "imm", 0)
            hi_at = b.pos - 1
            b.ins("PHA")
            b.ins("LDA", "imm", 0)
            lo_at = b.pos - 1
            b.ins("PHA")
            b.ins("LDA", "zp", self.var())
            b.ins("AND", "imm", 0xF7)  # D clear
            b.ins("PHA")
            b.raw(opc)
            b.ins("INC", "zp", self.var())  # skipped
            b.label(t)
            self._late.append((lo_at, hi_at, t))
            self.fold_flags(b)
        elif mn == "BRK":
            b.ins("LDA", "zp", self.var())
            b.raw(opc)
            b.byte(0xEA)  # skipped by the pushed return address
            self.fold_flags(b)
        else:
            raise AssertionError((mn, mode))

    def build(self, ops: list[int]) -> Rom:
        r = self.r
        bs, base = self.bank_size, self.base
        nb = 2 if self.size == 8192 else 1
        fill = byte_stream(stream_key(self.seed, 0x535746), self.size)
        banks = [Bank(bs, base, bytes(fill[i * bs:(i + 1) * bs])) for i in range(nb)]
        # data tables at the top of each bank (different bytes per bank): a full
        # page, then (4K banks) 192 bytes below the vectors.  Indexed reads near
        # a table's end cross into the next page, or past $FFFF into page 0.
        tab0 = bs - (0x100 if bs == 2048 else 0x200)
        tab_len = [0xC0] if bs == 2048 else [0x100, 0xC0]
        tables = [base + tab0 + 256 * i for i in range(len(tab_len))]
        self.wrap_page = tables[0] if bs == 4096 else None
        for bi, b in enumerate(banks):
            tb = byte_stream(stream_key(self.seed, 0x544142, bi), sum(tab_len))
            b.at(tab0)
            for v in tb[:tab_len[0]]:
                b.byte(int(v))
            if len(tab_len) > 1:
                b.at(tab0 + 0x100)
                for v in tb[tab_len[0]:]:
                    b.byte(int(v))
        info = instruction_set()
        # the same code in every bank: a bank switch keeps the flow, the tables differ
        img_code = None
        for bi, b in enumerate(banks):
            self.r = Rng(stream_key(self.seed, 0x535750))  # identical decisions per bank
            self._late = []
            self.wrap_target = None
            self.n_cross = self.seed
            self.n_label = 0
            b.at(0)
            b.label("START")
            b.ins("SEI")
            b.ins("CLD")
            b.ins("LDX", "imm", 0xFF)
            b.ins("TXS")
            b.label("MAIN")
            order = list(ops)
            for i in range(len(order) - 1, 0, -1):  # seeded shuffle
                j = self.r.randint(0, i)
                order[i], order[j] = order[j], order[i]
            for k, opc in enumerate(order):
                mn, mode = info[opc]
                if mode in ("abx", "aby", "izy"):  # with and without page crossings
                    self.emit(b, opc, mn, mode, tables, cross=False)
                    self.emit(b, opc, mn, mode, tables, cross=True)
                else:
                    self.emit(b, opc, mn, mode, tables)
                self.page_end(b)
                if k % 16 == 15:  # a line boundary now and then
                    b.ins("STA", "zp", WSYNC)
                if nb == 2 and k % 40 == 20:  # bank switches on data accesses of every kind
                    self.emit_hotspot(b)
            # every timer interval, INTIM and TIMINT read back
            for reg in (TIM1T, TIM8T, TIM64T, T1024T):
                b.ins("LDA", "zp", self.var())
                b.ins("AND", "imm", 0x3F)
                b.ins("STA", "abs", reg)
                for _ in range(self.r.randint(0, 3)):
                    b.ins("NOP")
                b.ins("LDA", "abs", INTIM)
                self.save_a(b)
                b.ins("BIT", "abs", TIMINT)
                self.fold_flags(b)
            b.ins("LDA", "zp", self.var())
            b.ins("STA", "zp", COLUBK)
            b.ins("JMP", "abs", "MAIN")
            # subroutine and BRK handler
            b.label("SUB")
            b.ins("LDA", "zp", self.var())
            b.ins("EOR", "imm", self.r.randint(0, 255))
            b.ins("STA", "zp", self.var())
            b.ins("RTS")
            b.label("BRKH")
            b.ins("TSX")
            b.ins("LDA", "abx", 0x0101)   # the pushed status byte, through the stack page
            b.ins("EOR", "zp", self.ACC)
            b.ins("STA", "zp", self.ACC)
            b.ins("INC", "zp", self.var())
            b.ins("RTI")
            assert b.pos <= tab0, "sweep program overflows its bank"
            code_end = b.pos
            b.link()
            for item in self._late:
                lo_at, hi_at, t = item[:3]
                a = b.labels[t] + (item[3] if len(item) > 3 else 0)
                b.img[lo_at] = a & 0xFF
                b.img[hi_at] = (a >> 8) & 0xFF
            if self.wrap_target is not None:  # JMP ($xxFF) pair: low byte at $xxFF, high at $xx00
                a = b.labels[self.wrap_target]
                b.img[tab0 + 0xFF] = a & 0xFF
                b.img[tab0] = (a >> 8) & 0xFF
            # vectors: reset at $FFFC, IRQ/BRK at $FFFE
            b.at(bs - 4)
            st, brk = b.labels["START"], b.labels["BRKH"]
            b.byte(st & 0xFF, st >> 8, brk & 0xFF, brk >> 8)
            code = bytes(b.img[:code_end])
            assert img_code is None or img_code == code
            img_code = code
        img = np.frombuffer(b"".join(bytes(bb.img) for bb in banks), dtype=np.uint8).copy()
        return Rom(seed=self.seed, size=self.size, mapper=MAPPER_OF_SIZE[self.size], image=img, reads_inputs=True)

    def emit_hotspot(self, b: Bank):
        r = self.r
        kind = r.choice(["lda", "sta", "bit", "abx", "izy", "inc"])
        hs = 0x1FF8 + r.randint(0, 1)
        if kind == "lda":
            b.ins("LDA", "abs", hs)
            self.save_a(b)
        elif kind == "sta":
            b.ins("STA", "abs", hs | 0xE000)
        elif kind == "bit":
            b.ins("BIT", "abs", hs)
        elif kind == "abx":
            b.ins("LDA", "zp", self.var())
            b.ins("AND", "imm", 1)
            b.ins("TAX")
            b.ins("LDA", "abx", 0xFFF8)
            self.save_a(b)
        elif kind == "izy":
            self.set_ptr(b, 1, 0x1FF8)
            b.ins("LDA", "zp", self.var())
            b.ins("AND", "imm", 1)
            b.ins("TAY")
            b.ins("LDA", "izy", self.PTR + 2)
            self.save_a(b)
        else:
            b.ins("INC", "abs", hs)


def generate_sweep_rom(seed: int, size: int = 4096, *, soft_safe: bool = False, objects: bool = True) -> Rom:
    """A seeded program that executes every byte of the 189-opcode set (a 2K
    image holds a seeded 80 of them), in every addressing form, with indexed
    accesses that cross pages for some envs and not for others, read-modify-
    write on RAM, TIA and RIOT registers, all four timer intervals, TIMINT
    reads, the JMP ($xxFF) page wrap, BRK/RTI, computed RTS/RTI jumps, code run
    from RAM, pushes onto TIA registers and, for F8 images, bank switches on
    every kind of data access (the code is the same in both banks, the data
    tables differ).  objects=False keeps every access off the registers only the
    TIA's objects use (collision reads, object-register writes)."""
    assert size in (2048, 4096, 8192)
    g = _SweepGen(seed, size, soft_safe, objects)
    ops = sorted(instruction_set())
    if size == 2048:
        sel = Rng(stream_key(seed, 0x32304B))
        for i in range(len(ops) - 1, 0, -1):  # a seeded choice of 80 of them
            j = sel.randint(0, i)
            ops[i], ops[j] = ops[j], ops[i]
        ops = sorted(ops[:80])
    return g.build(ops)


SWEEP_ROMS = ((4, 4096), (1, 4096), (0, 8192), (7, 8192), (1, 2048), (7, 2048))


def config_sweep(envs_per_rom: int = 8, steps: int = 4, frame_skip: int = 2, episodes: bool = True,
                 objects: bool = True) -> Workload:
    """Parity workload over the opcode-sweep family: 4K, F8 and 2K sweep images,
    random RAM and joystick inputs, short geometric-free episodes (1-3 steps)
    for every other env so that in-run resets land mid-sweep.  objects=False:
    the images that stay off the object registers (see generate_sweep_rom)."""
    roms = [generate_sweep_rom(s, sz, objects=objects) for s, sz in SWEEP_ROMS]
    b = len(roms) * envs_per_rom
    env_rom = np.repeat(np.arange(len(roms), dtype=np.int32), envs_per_rom)
    eps = None
    if episodes:
        lens = 1 + int_stream(stream_key(5, 0x455053), b * 8, 3).reshape(b, 8)
        lens[::2] = 1 << 20  # every other env: one long episode
        eps = lens.astype(np.uint32)
    return Workload("sweep", roms, env_rom, initial_ram(5, b), action_stream(5, b, steps), steps=steps,
                    frame_skip=frame_skip, episode_steps=eps, seed=5)


# --------------------------------------------------------------------------
# Further cartridge formats: F6, F4, the Superchip variants and E0
# --------------------------------------------------------------------------

(MAPPER_F6, MAPPER_F4, MAPPER_F8SC, MAPPER_F6SC, MAPPER_F4SC, MAPPER_E0) = range(3, 9)
MAPPER_NAMES = {MAPPER_2K: "2K", MAPPER_4K: "4K", MAPPER_F8: "F8", MAPPER_F6: "F6", MAPPER_F4: "F4",
                MAPPER_F8SC: "F8SC", MAPPER_F6SC: "F6SC", MAPPER_F4SC: "F4SC", MAPPER_E0: "E0"}
_BANKS = {MAPPER_F8: 2, MAPPER_F6: 4, MAPPER_F4: 8, MAPPER_F8SC: 2, MAPPER_F6SC: 4, MAPPER_F4SC: 8}
_HOT_LO = {2: 0x1FF8, 4: 0x1FF6, 8: 0x1FF4}
_SC = (MAPPER_F8SC, MAPPER_F6SC, MAPPER_F4SC)
ACTION_RESET = 18


def _band_line(b: Bank, r: Rng, var, sc: bool, table: int | None, colour_imm: list, img_base: int):
    """One kernel line's body (<= ~40 cycles) before its STA WSYNC; the image offsets of
    colour immediates are added to colour_imm (img_base: the bank's offset in the image)."""
    for _ in range(r.randint(2, 4)):
        k = r.randint(0, 6 if sc else 4)
        if k == 0:
            colour_imm.append(img_base + b.ins("LDA", "imm", r.randint(0, 127) * 2))
            b.ins("STA", "zp", COLUBK)
        elif k == 1:
            b.ins("LDA", "zp", var())
            b.ins("STA", "zp", COLUPF)
        elif k == 2:
            b.ins("INC", "zp", var())
        elif k == 3:
            b.ins("LDA", "zp", var())
            b.ins("AND", "imm", 0xF0)
            b.ins("STA", "zp", PF1 if r.random() < 0.5 else PF2)
        elif k == 4:
            if table is not None:
                b.ins("LDA", "abs", table + r.randint(0, 255))
            else:
                b.ins("LDA", "imm", r.randint(0, 255))
            b.ins("STA", "zp", PF0 if r.random() < 0.5 else COLUBK)
        elif k == 5:  # Superchip RAM read port -> a colour
            b.ins("LDA", "abs", 0x1080 + r.randint(0, 127))
            b.ins("STA", "zp", COLUPF)
        else:  # a RAM counter into the Superchip write port
            b.ins("LDA", "zp", var())
            b.ins("STA", "abs", 0x1000 + r.randint(0, 127))


def generate_mapper_rom(seed: int, mapper: int) -> Rom:
    """A synthetic cartridge of a bank-switched format whose frames walk all of
    its banks (F8/F6/F4 and the Superchip variants: the kernel's bands run in
    banks 0..N-2, each hopping to the next through its hotspot; VSYNC, VBLANK and
    overscan in bank N-1) or slices (E0: the fixed last quarter maps each band's
    slice into a quarter of the window and calls it).  Superchip images move RAM
    counters through their 128-byte RAM into colours.  262 lines per frame."""
    r = Rng(stream_key(seed, 0x4D4150, mapper))
    sc = mapper in _SC
    nvar = [0]
    colour_imm: list[int] = []

    def var():  # RAM counters $80..$9F
        nvar[0] = (nvar[0] + 1) % 32
        return 0x80 + r.randint(0, 31)

    def vsync_vblank(b: Bank):
        b.ins("LDA", "imm", 0x02)
        b.ins("STA", "zp", VBLANK)
        b.ins("STA", "zp", VSYNC)
        for _ in range(3):
            b.ins("STA", "zp", WSYNC)
        b.ins("LDA", "imm", 0x00)
        b.ins("STA", "zp", VSYNC)
        b.ins("LDA", "imm", 44)            # ~37 lines of VBLANK on the timer
        b.ins("STA", "abs", TIM64T)
        for _ in range(r.randint(2, 5)):
            b.ins("INC", "zp", var())
        w = f"w{b.pos}"
        b.label(w)
        b.ins("LDA", "abs", INTIM)
        b.ins("BNE", "rel", w)
        b.ins("STA", "zp", WSYNC)
        b.ins("LDA", "imm", 0x00)
        b.ins("STA", "zp", VBLANK)

    def overscan(b: Bank):
        b.ins("LDA", "imm", 0x02)
        b.ins("STA", "zp", VBLANK)
        b.ins("LDX", "imm", 30)
        lp = f"os{b.pos}"
        b.label(lp)
        b.ins("STA", "zp", WSYNC)
        b.ins("DEX")
        b.ins("BNE", "rel", lp)

    def band(b: Bank, lines: int, table, img_base: int):
        b.ins("LDY", "imm", lines)
        lp = f"band{b.pos}"
        b.label(lp)
        _band_line(b, r, var, sc, table, colour_imm, img_base)
        b.ins("STA", "zp", WSYNC)
        b.ins("DEY")
        b.ins("BNE", "rel", lp)

    if mapper == MAPPER_E0:
        # slices 0..6 hold band subroutines assembled for the quarter they are mapped to;
        # slice 7 (the fixed last quarter, $1C00-$1FFF seen at $FC00) holds the frame
        nb = 7
        cuts = sorted(r.randint(8, 184) for _ in range(nb - 1))
        lines = [e1 - e0 for e0, e1 in zip([0] + cuts, cuts + [192])]
        slices = []
        order = list(range(nb))
        for i in range(nb - 1, 0, -1):
            j = r.randint(0, i)
            order[i], order[j] = order[j], order[i]
        plan = []  # (slice, quarter, lines)
        for i, s in enumerate(order):
            plan.append((s, i % 3, lines[i]))
        blobs = {}
        for s, q, n in plan:
            b = Bank(1024, 0xF000 + 0x400 * q, bytes([0xEA]) * 1024)
            b.at(0)
            if n > 0:
                band(b, n, 0xF000 + 0x400 * q + 0x300, 1024 * s)
            b.ins("RTS")
            b.at(0x300)
            for i in range(256):  # a data table read by the band
                b.byte(r.randint(0, 255))
            b.link()
            blobs[s] = bytes(b.img)
        m = Bank(1024, 0xFC00, bytes([0xEA]) * 1024)
        m.at(0x000)
        m.label("FRAME")
        vsync_vblank(m)
        for s, q, n in plan:
            m.ins("LDA", "abs", 0x1FE0 + 8 * q + s)   # quarter q <- slice s
            m.ins("JSR", "abs", 0xF000 + 0x400 * q)
        overscan(m)
        m.ins("JMP", "abs", "FRAME")
        m.at(0x3E0)
        m.label("RESET")
        m.ins("SEI")
        m.ins("CLD")
        m.ins("LDX", "imm", 0xFF)
        m.ins("TXS")
        m.ins("JMP", "abs", "FRAME")
        m.at(0x3FC)
        rs = m.labels["RESET"]
        m.byte(rs & 0xFF, rs >> 8, rs & 0xFF, rs >> 8)
        m.link()
        img = b"".join(blobs.get(s, bytes([0xEA]) * 1024) for s in range(7)) + bytes(m.img)
        return Rom(seed=seed, size=8192, mapper=mapper, image=np.frombuffer(img, np.uint8).copy(),
                   colour_imm=colour_imm)

    n = _BANKS[mapper]
    hot = _HOT_LO[n]
    main = n - 1
    banks = [Bank(4096, 0xF000, bytes([0xEA]) * 4096) for _ in range(n)]
    for i, b in enumerate(banks):
        b.at(0)
        for _ in range(256):  # the Superchip RAM window holds no code or data; others: a table
            b.byte(0xFF if sc else r.randint(0, 255))
        # identical reset stubs: any power-on bank reaches FRAME in the main bank
        b.at(0xFE0)
        b.ins("SEI")
        b.ins("CLD")
        b.ins("LDX", "imm", 0xFF)
        b.ins("TXS")
        b.ins("LDA", "abs", hot + main)
        b.ins("JMP", "abs", 0xF100)
        b.at(0xFFC)
        b.byte(0xE0, 0xFF, 0xE0, 0xFF)
        # the hop at $F800 selects the next bank, which continues at its own $F803:
        # its band at $F200, or the main bank's overscan at $F300
        b.at(0x800)
        b.ins("LDA", "abs", hot + (i + 1) % n)
        b.ins("JMP", "abs", 0xF200 if i != main else 0xF300)
    nbands = n - 1
    cuts = sorted(r.randint(8, 184) for _ in range(nbands - 1))
    lines = [e1 - e0 for e0, e1 in zip([0] + cuts, cuts + [192])]
    for i in range(nbands):  # band i in bank i at $F200, then the hop
        b = banks[i]
        b.at(0x200)
        if lines[i] > 0:
            band(b, lines[i], 0xFA00, 4096 * i)
        b.ins("JMP", "abs", 0xF800)
        b.at(0xA00)
        for _ in range(256):
            b.byte(r.randint(0, 255))
    m = banks[main]
    m.at(0x100)
    vsync_vblank(m)
    m.ins("JMP", "abs", 0xF800)      # -> bank 0's band
    m.at(0x300)                      # the last band's hop lands here (bank N-1 at $F803 -> $F300)
    overscan(m)
    m.ins("JMP", "abs", 0xF100)
    for b in banks:
        b.link()
    img = b"".join(bytes(b.img) for b in banks)
    return Rom(seed=seed, size=4096 * n, mapper=mapper, image=np.frombuffer(img, np.uint8).copy(),
               colour_imm=colour_imm)


MAPPER_ROMS = ((MAPPER_F6, 1), (MAPPER_F6SC, 2), (MAPPER_F8SC, 3), (MAPPER_E0, 4), (MAPPER_F4, 5), (MAPPER_F4SC, 6))


def config_mappers(envs_per_rom: int = 8, steps: int = 3, frame_skip: int = 2, lds_only: bool = False,
                   episodes: bool = True) -> Workload:
    """Parity workload over the further cartridge formats (F6, F6SC, F8SC, E0 and,
    unless lds_only, F4 and F4SC, which only the plain kernel holds), random RAM and
    joystick inputs, short episodes for every other env (in-run resets reseed RAM
    and Superchip RAM)."""
    sel = [(m, s) for m, s in MAPPER_ROMS if not (lds_only and m in (MAPPER_F4, MAPPER_F4SC))]
    roms = [generate_mapper_rom(s, m) for m, s in sel]
    b = len(roms) * envs_per_rom
    env_rom = np.repeat(np.arange(len(roms), dtype=np.int32), envs_per_rom)
    eps = None
    if episodes:
        lens = 1 + int_stream(stream_key(6, 0x455053), b * 8, 2).reshape(b, 8)
        lens[::2] = 1 << 20
        eps = lens.astype(np.uint32)
    return Workload("mappers", roms, env_rom, initial_ram(6, b), action_stream(6, b, steps), steps=steps,
                    frame_skip=frame_skip, episode_steps=eps, seed=6)


def boot_actions(num_envs: int, seed: int, noops: int = 60, resets: int = 4, max_random_noops: int = 30):
    """The boot sequence of Table s-params as per-frame actions [B][n]: `noops` NOOP
    frames, `resets` frames with the console RESET switch held, then 0..max random
    NOOP frames per env (Mnih-style episode-start randomisation), padded with NOOPs
    to one length; returns (actions, the random counts)."""
    extra = int_stream(stream_key(seed, 0x424F4F), num_envs, max_random_noops + 1)
    n = noops + resets + max_random_noops
    a = np.zeros((num_envs, n), np.uint8)
    a[:, noops:noops + resets] = ACTION_RESET
    return a, extra.astype(np.int64)


# --------------------------------------------------------------------------
# Sprite workloads: game-like kernels that use the TIA's movable objects
# --------------------------------------------------------------------------

NUSIZ0, NUSIZ1, REFP0, REFP1 = 0x04, 0x05, 0x0B, 0x0C
RESP0, RESP1, RESM0, RESM1, RESBL = 0x10, 0x11, 0x12, 0x13, 0x14
GRP0, GRP1, ENAM0, ENAM1, ENABL = 0x1B, 0x1C, 0x1D, 0x1E, 0x1F
HMP0, HMP1, HMM0, HMM1, HMBL = 0x20, 0x21, 0x22, 0x23, 0x24
VDELP0, VDELP1, VDELBL, RESMP0, RESMP1 = 0x25, 0x26, 0x27, 0x28, 0x29
HMOVE, HMCLR, CXCLR = 0x2A, 0x2B, 0x2C
OBJ_X = 0x80          # RAM: columns of P0, P1, M0, M1, BL ($80-$84)
OBJ_HITS = 0x85       # RAM: P0-P1 hit counter
OBJ_CX = 0x86         # RAM: the eight collision registers copied each frame ($86-$8D)


def generate_object_rom(seed: int, size: int = 4096) -> Rom:
    """A seed-generated sprite kernel (2K or 4K image), laid out like a game frame:
    VSYNC, a vertical blank that moves P0 with the joystick (REFP0 follows the
    direction), positions all five objects from RAM with the divide-by-15 strobe
    loop and fine motion (HMxx, HMOVE), then 192 lines that load GRP0/GRP1, the
    missile and ball enables and PF1 from page-aligned tables, and an overscan
    that copies the collision latches into RAM, counts P0-P1 hits and clears
    them.  NUSIZ, vertical delay, CTRLPF (reflection, score, priority, ball
    width), RESMP and the colours are drawn from the seed."""
    assert size in (2048, 4096)
    r = Rng(stream_key(seed, 0x4F424A))
    base = 0xF000 if size == 4096 else 0xF800
    b = Bank(size, base, bytes([0xEA]) * size)
    # tables: 5 pages at the top (graphics 0, graphics 1, enables, playfield, colours)
    tab = {}
    npages = 5 if size == 4096 else 3
    tb = byte_stream(stream_key(seed, 0x544F42), 256 * npages)
    for i, name in enumerate(["gfx0", "gfx1", "en", "pf", "col"][:npages]):
        off = size - 0x100 * (npages + 1) + 0x100 * i
        b.at(off)
        tab[name] = b.addr()
        for y in range(256):
            v = int(tb[256 * i + y])
            if name.startswith("gfx"):
                band = (y // 16) % 4  # sprites in bands of lines, blank between
                v = v if band in (1, 2) else 0
            elif name == "en":
                v = v & 0x2A  # bits 1, 3, 5: missile 0, missile 1, ball after shifts
            elif name == "pf":
                v = v & 0x81
            elif name == "col":
                v = v & 0xFE
            b.byte(v)
    if npages == 3:
        tab["pf"] = tab["en"]
        tab["col"] = tab["gfx0"]
    b.at(0)
    b.label("RESET")
    b.ins("SEI")
    b.ins("CLD")
    b.ins("LDX", "imm", 0xFF)
    b.ins("TXS")
    # static set-up from the seed
    settings = [(NUSIZ0, r.randint(0, 7) | (r.randint(0, 3) << 4)), (NUSIZ1, r.randint(0, 7) | (r.randint(0, 3) << 4)),
                (CTRLPF, r.randint(0, 7) | (r.randint(0, 3) << 4)), (VDELP0, r.randint(0, 1)),
                (VDELP1, r.randint(0, 1)), (VDELBL, r.randint(0, 1)), (REFP1, 8 * r.randint(0, 1)),
                (COLUP0, (r.randint(1, 127) * 2) & 0xFE), (COLUP1, (r.randint(1, 127) * 2) & 0xFE),
                (COLUPF, (r.randint(1, 127) * 2) & 0xFE), (COLUBK, (r.randint(0, 127) * 2) & 0xFE)]
    for reg, v in settings:
        b.ins("LDA", "imm", v)
        b.ins("STA", "zp", reg)
    b.label("FRAME")
    b.ins("LDA", "imm", 0x02)
    b.ins("STA", "zp", VBLANK)
    b.ins("STA", "zp", VSYNC)
    for _ in range(3):
        b.ins("STA", "zp", WSYNC)
    b.ins("LDA", "imm", 0x00)
    b.ins("STA", "zp", VSYNC)
    # line 1: the joystick moves P0 (right: +1, left: -1, reflected while moving left)
    b.ins("LDA", "abs", SWCHA)
    b.ins("BMI", "rel", "NR")
    b.ins("INC", "zp", OBJ_X)
    b.ins("LDA", "imm", 0x00)
    b.ins("STA", "zp", REFP0)
    b.label("NR")
    b.ins("LDA", "abs", SWCHA)
    b.ins("AND", "imm", 0x40)
    b.ins("BNE", "rel", "NL")
    b.ins("DEC", "zp", OBJ_X)
    b.ins("LDA", "imm", 0x08)
    b.ins("STA", "zp", REFP0)
    b.label("NL")
    b.ins("STA", "zp", WSYNC)
    # line 2: every object column kept in 0..151 (a wrapped one restarts at 8)
    for k in range(5):
        b.ins("LDA", "zp", OBJ_X + k)
        b.ins("CMP", "imm", 152)
        b.ins("BCC", "rel", f"C{k}")
        b.ins("LDA", "imm", 8)
        b.ins("STA", "zp", OBJ_X + k)
        b.label(f"C{k}")
    b.ins("STA", "zp", WSYNC)
    # lines 3-7: coarse strobe by the divide-by-15 loop, fine motion into HMxx
    used = 3
    for k, (hmr, resr) in enumerate(((HMP0, RESP0), (HMP1, RESP1), (HMM0, RESM0), (HMM1, RESM1), (HMBL, RESBL))):
        b.ins("STA", "zp", WSYNC)
        b.ins("LDA", "zp", OBJ_X + k)
        b.ins("SEC")
        b.label(f"D{k}")
        b.ins("SBC", "imm", 15)
        b.ins("BCS", "rel", f"D{k}")
        b.ins("EOR", "imm", 7)
        for _ in range(4):
            b.ins("ASL", "acc")
        b.ins("STA", "zp", hmr)
        b.ins("STA", "zp", resr)
        used += 1
    b.ins("STA", "zp", WSYNC)
    b.ins("STA", "zp", HMOVE)   # in horizontal blank: columns 0..7 of this line go black
    used += 1
    if r.random() < 0.5:        # lock missile 1 to player 1's centre for a line
        b.ins("LDA", "imm", 0x02)
        b.ins("STA", "zp", RESMP1)
        b.ins("STA", "zp", WSYNC)
        b.ins("LDA", "imm", 0x00)
        b.ins("STA", "zp", RESMP1)
        used += 1
    b.ins("STA", "zp", WSYNC)
    b.ins("STA", "zp", HMCLR)
    used += 1
    b.ins("LDX", "imm", 37 - used)
    b.label("VB")
    b.ins("STA", "zp", WSYNC)
    b.ins("DEX")
    b.ins("BNE", "rel", "VB")
    # kernel: 192 lines from the tables
    b.ins("STA", "zp", WSYNC)
    b.ins("LDA", "imm", 0x00)
    b.ins("STA", "zp", VBLANK)
    b.ins("LDY", "imm", 191)
    b.label("KL")
    b.ins("STA", "zp", WSYNC)
    b.ins("LDA", "aby", tab["gfx0"])
    b.ins("STA", "zp", GRP0)
    b.ins("LDA", "aby", tab["gfx1"])
    b.ins("STA", "zp", GRP1)
    b.ins("LDA", "aby", tab["en"])
    b.ins("STA", "zp", ENAM0)
    b.ins("LSR", "acc")
    b.ins("LSR", "acc")
    b.ins("STA", "zp", ENAM1)
    b.ins("LSR", "acc")
    b.ins("LSR", "acc")
    b.ins("STA", "zp", ENABL)
    b.ins("LDA", "aby", tab["pf"])
    b.ins("STA", "zp", PF1)
    if r.random() < 0.5:
        b.ins("LDA", "aby", tab["col"])
        b.ins("STA", "zp", COLUP1)
    b.ins("DEY")
    b.ins("BNE", "rel", "KL")
    # overscan: collisions into RAM, the P0-P1 hit count, clear
    b.ins("STA", "zp", WSYNC)
    b.ins("LDA", "imm", 0x02)
    b.ins("STA", "zp", VBLANK)
    b.ins("LDA", "imm", 0x00)
    b.ins("STA", "zp", GRP0)
    b.ins("STA", "zp", GRP1)
    for k in range(8):
        b.ins("LDA", "zp", k)
        b.ins("STA", "zp", OBJ_CX + k)
    b.ins("BIT", "zp", 0x07)      # CXPPMM bit 7: P0-P1
    b.ins("BPL", "rel", "NH")
    b.ins("INC", "zp", OBJ_HITS)
    b.label("NH")
    b.ins("STA", "zp", CXCLR)
    b.ins("LDX", "imm", 29)
    b.label("OS")
    b.ins("STA", "zp", WSYNC)
    b.ins("DEX")
    b.ins("BNE", "rel", "OS")
    b.ins("JMP", "abs", "FRAME")
    b.at(size - 4)
    b.byte(base & 0xFF, base >> 8, base & 0xFF, base >> 8)
    b.link()
    img = np.frombuffer(bytes(b.img), dtype=np.uint8).copy()
    return Rom(seed, size, MAPPER_OF_SIZE[size], img, reads_inputs=True)


def config_objects(envs_per_rom: int = 256, steps: int = 200, n_roms: int = 16, frame_skip: int = 4) -> Workload:
    """Sprite workload: seed-generated object kernels (2K and 4K) x envs_per_rom,
    random joystick actions (they move player 0), RAM and frames every step."""
    roms = [generate_object_rom(7000 + i, 4096 if i % 4 else 2048) for i in range(n_roms)]
    b = n_roms * envs_per_rom
    env_rom = np.repeat(np.arange(n_roms, dtype=np.int32), envs_per_rom)
    return Workload("objects", roms, env_rom, initial_ram(5, b), action_stream(5, b, steps), steps=steps,
                    frame_skip=frame_skip, seed=5)
