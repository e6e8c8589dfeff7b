"""Pins of the oracle that do not rest on its own tables or formulas.

1. Cycle counts of all 189 opcode bytes of the paper's set (151 documented,
   the $EB alias of SBC #imm and 37 undocumented NOP/LAX/SAX forms; Sec.
   "Building Two Differentiable VCS Ports"), measured by running each byte
   alone on the oracle, with page-crossing and not-crossing variants of every
   indexed form and taken / not-taken / page-crossing variants of every
   branch, against the NMOS 6502 data-sheet timings restated below.
2. Every surrogate rule of the soft backward (the stored-switch reading of Sec.
   "Hard and Soft Execution" with the straight-through estimator of Eq. ste),
   each on a hand-assembled program whose gradient is derived by hand from
   the rule, in STE mode (coefficients at hard values) and in SMOOTH mode
   (coefficients at the smooth values, and the smooth forward value itself).
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import asm as A

MAP_4K = 1

# ---------------------------------------------------------------------------
# NMOS 6502 data-sheet timings: "mnemonic  opcode:mode:cycles ...", where a
# trailing "+" marks an indexed read that takes one more cycle when the index
# carries into the high byte of the address.  Branches are listed at 2 cycles
# (+1 when taken, +1 more when the target lies in another page).
# ---------------------------------------------------------------------------
DATASHEET = """
ADC 69:imm:2 65:zp:3 75:zpx:4 6D:abs:4 7D:abx:4+ 79:aby:4+ 61:izx:6 71:izy:5+
AND 29:imm:2 25:zp:3 35:zpx:4 2D:abs:4 3D:abx:4+ 39:aby:4+ 21:izx:6 31:izy:5+
ASL 0A:acc:2 06:zp:5 16:zpx:6 0E:abs:6 1E:abx:7
BIT 24:zp:3 2C:abs:4
BPL 10:rel:2
BMI 30:rel:2
BVC 50:rel:2
BVS 70:rel:2
BCC 90:rel:2
BCS B0:rel:2
BNE D0:rel:2
BEQ F0:rel:2
BRK 00:imp:7
CMP C9:imm:2 C5:zp:3 D5:zpx:4 CD:abs:4 DD:abx:4+ D9:aby:4+ C1:izx:6 D1:izy:5+
CPX E0:imm:2 E4:zp:3 EC:abs:4
CPY C0:imm:2 C4:zp:3 CC:abs:4
DEC C6:zp:5 D6:zpx:6 CE:abs:6 DE:abx:7
EOR 49:imm:2 45:zp:3 55:zpx:4 4D:abs:4 5D:abx:4+ 59:aby:4+ 41:izx:6 51:izy:5+
CLC 18:imp:2
SEC 38:imp:2
CLI 58:imp:2
SEI 78:imp:2
CLV B8:imp:2
CLD D8:imp:2
SED F8:imp:2
INC E6:zp:5 F6:zpx:6 EE:abs:6 FE:abx:7
JMP 4C:abs:3 6C:ind:5
JSR 20:abs:6
LDA A9:imm:2 A5:zp:3 B5:zpx:4 AD:abs:4 BD:abx:4+ B9:aby:4+ A1:izx:6 B1:izy:5+
LDX A2:imm:2 A6:zp:3 B6:zpy:4 AE:abs:4 BE:aby:4+
LDY A0:imm:2 A4:zp:3 B4:zpx:4 AC:abs:4 BC:abx:4+
LSR 4A:acc:2 46:zp:5 56:zpx:6 4E:abs:6 5E:abx:7
NOP EA:imp:2
ORA 09:imm:2 05:zp:3 15:zpx:4 0D:abs:4 1D:abx:4+ 19:aby:4+ 01:izx:6 11:izy:5+
TAX AA:imp:2
TXA 8A:imp:2
DEX CA:imp:2
INX E8:imp:2
TAY A8:imp:2
TYA 98:imp:2
DEY 88:imp:2
INY C8:imp:2
ROL 2A:acc:2 26:zp:5 36:zpx:6 2E:abs:6 3E:abx:7
ROR 6A:acc:2 66:zp:5 76:zpx:6 6E:abs:6 7E:abx:7
RTI 40:imp:6
RTS 60:imp:6
SBC E9:imm:2 E5:zp:3 F5:zpx:4 ED:abs:4 FD:abx:4+ F9:aby:4+ E1:izx:6 F1:izy:5+
STA 85:zp:3 95:zpx:4 8D:abs:4 9D:abx:5 99:aby:5 81:izx:6 91:izy:6
TXS 9A:imp:2
TSX BA:imp:2
PHA 48:imp:3
PLA 68:imp:4
PHP 08:imp:3
PLP 28:imp:4
STX 86:zp:3 96:zpy:4 8E:abs:4
STY 84:zp:3 94:zpx:4 8C:abs:4
USBC EB:imm:2
LAX A7:zp:3 B7:zpy:4 AF:abs:4 BF:aby:4+ A3:izx:6 B3:izy:5+
SAX 87:zp:3 97:zpy:4 8F:abs:4 83:izx:6
NOP 1A:imp:2 3A:imp:2 5A:imp:2 7A:imp:2 DA:imp:2 FA:imp:2
NOP 80:imm:2 82:imm:2 89:imm:2 C2:imm:2 E2:imm:2
NOP 04:zp:3 44:zp:3 64:zp:3
NOP 14:zpx:4 34:zpx:4 54:zpx:4 74:zpx:4 D4:zpx:4 F4:zpx:4
NOP 0C:abs:4
NOP 1C:abx:4+ 3C:abx:4+ 5C:abx:4+ 7C:abx:4+ DC:abx:4+ FC:abx:4+
"""


def datasheet():
    rows = {}
    for line in DATASHEET.strip().splitlines():
        mn, *cells = line.split()
        for c in cells:
            op, mode, cyc = c.split(":")
            plus = cyc.endswith("+")
            rows[int(op, 16)] = (mn, mode, int(cyc.rstrip("+")), plus)
    return rows


# Index registers during a measurement: X = $10, Y = $20.  Zero-page pointers:
# ($82) = $F0F0 (+Y crosses into $F1xx), ($84) = $F000 (+Y stays), ($86,X) =
# ($96) = $F000.  Absolute indexed bases: $F0F8 (+X or +Y crosses), $F000.
def _ram0():
    r = np.zeros(128, np.uint8)
    r[0x02:0x04] = [0xF0, 0xF0]
    r[0x04:0x06] = [0x00, 0xF0]
    r[0x16:0x18] = [0x00, 0xF0]
    return r


def _measure(setup, target, org=0xF000, extra=None):
    """Cycles of the instruction `target` (raw bytes) run after the `setup`
    instructions, assembled from CPU address org; extra(img) patches the image."""
    img = A.raw_image(4096, {})
    off = org - 0xF000
    code = []
    for ins in setup:
        code += list(ins)
    code += list(target)
    img[off:off + len(code)] = code
    img[0xFFC:0xFFE] = [org & 0xFF, org >> 8]
    if extra:
        extra(img)
    m = O.Machine(img, MAP_4K, _ram0())
    for _ in setup:
        assert m.step() == 0
    c0 = m.regs()["cycle"]
    m.step()
    return m.regs()["cycle"] - c0


LDX10, LDY20 = (0xA2, 0x10), (0xA0, 0x20)
# flag setups that make each branch taken / not taken
_BRANCH_FLAGS = {
    0x10: ([(0xA9, 0x00)], [(0xA9, 0x80)]),                        # BPL: N clear / set
    0x30: ([(0xA9, 0x80)], [(0xA9, 0x00)]),                        # BMI
    0x50: ([(0xB8,)], [(0x18,), (0xA9, 0x7F), (0x69, 0x01)]),      # BVC: CLV / 7F + 1 overflows
    0x70: ([(0x18,), (0xA9, 0x7F), (0x69, 0x01)], [(0xB8,)]),      # BVS
    0x90: ([(0x18,)], [(0x38,)]),                                  # BCC
    0xB0: ([(0x38,)], [(0x18,)]),                                  # BCS
    0xD0: ([(0xA9, 0x01)], [(0xA9, 0x00)]),                        # BNE
    0xF0: ([(0xA9, 0x00)], [(0xA9, 0x01)]),                        # BEQ
}


def _cases(op, mode, cyc, plus):
    """(setup, target, org, extra, expected cycles) variants for one opcode."""
    idx = [LDX10, LDY20]
    if mode in ("imp", "acc"):
        if op == 0x40:  # RTI after a BRK whose handler is the RTI
            def vec(img):
                img[0xFFE:0x1000] = [0x10, 0xF0]
                img[0x10] = 0x40
            return [([(0x00, 0x00)], (), 0xF000, vec, cyc)]
        if op == 0x60:  # RTS after a JSR to it
            def sub(img):
                img[0x10] = 0x60
            return [([(0x20, 0x10, 0xF0)], (), 0xF000, sub, cyc)]
        if op in (0x68, 0x28):  # pulls after a push
            return [([(0x48,)], (op,), 0xF000, None, cyc)]
        if op == 0x00:
            def vec(img):
                img[0xFFE:0x1000] = [0x10, 0xF0]
            return [([], (op, 0x00), 0xF000, vec, cyc)]
        return [(idx, (op,), 0xF000, None, cyc)]
    if mode == "imm":
        return [(idx, (op, 0x00), 0xF000, None, cyc)]
    if mode in ("zp", "zpx", "zpy"):
        return [(idx, (op, 0x90), 0xF000, None, cyc)]
    if mode == "abs":
        if op in (0x4C, 0x20):
            return [(idx, (op, 0x40, 0xF0), 0xF000, None, cyc)]
        return [(idx, (op, 0x90, 0x00), 0xF000, None, cyc)]
    if mode in ("abx", "aby"):
        return [(idx, (op, 0xF8, 0xF0), 0xF000, None, cyc + (1 if plus else 0)),
                (idx, (op, 0x00, 0xF0), 0xF000, None, cyc)]
    if mode == "izx":
        return [(idx, (op, 0x86), 0xF000, None, cyc)]
    if mode == "izy":
        return [(idx, (op, 0x82), 0xF000, None, cyc + (1 if plus else 0)),
                (idx, (op, 0x84), 0xF000, None, cyc)]
    if mode == "ind":
        def ptr(img):
            img[0x800:0x802] = [0x40, 0xF0]
        return [(idx, (op, 0x00, 0xF8), 0xF000, ptr, cyc)]
    if mode == "rel":
        taken, not_taken = _BRANCH_FLAGS[op]
        n_t = sum(len(i) for i in taken)
        return [(not_taken, (op, 0x02), 0xF000, None, cyc),
                (taken, (op, 0x02), 0xF000, None, cyc + 1),
                # the branch starts at $F0F0: its next instruction is at $F0F2 and the
                # target $F0F2 + $20 lies in page $F1
                (taken, (op, 0x20), 0xF0F0 - n_t, None, cyc + 2),
                # backwards from page $F1 into page $F0
                (taken, (op, 0xF0), 0xF100 - n_t, None, cyc + 2)]
    raise AssertionError(mode)


def test_datasheet_is_the_papers_opcode_set():
    rows = datasheet()
    assert len(rows) == 189
    assert sum(1 for mn, *_ in rows.values() if mn not in ("LAX", "SAX", "USBC")) - 27 == 151
    implemented = {op for op in range(256) if O.opcode_info(op)[0]}
    assert implemented == set(rows)


def test_every_opcode_cycle_count_measured():
    rows = datasheet()
    measured = 0
    for op, (mn, mode, cyc, plus) in sorted(rows.items()):
        for setup, target, org, extra, want in _cases(op, mode, cyc, plus):
            if not target:  # RTS / RTI: the measured instruction is the one the setup reaches
                got = _measure(setup, (), org, extra)
            else:
                got = _measure(setup, target, org, extra)
            assert got == want, (hex(op), mn, mode, target, got, want)
            measured += 1
    assert measured >= 189 + 2 * 8 * 3  # every byte, plus the indexed and branch variants


def test_store_and_rmw_indexed_forms_pay_no_separate_crossing_cycle():
    rows = datasheet()
    for op, (mn, mode, cyc, plus) in rows.items():
        if mode in ("abx", "aby") and not plus:
            assert mn in ("STA", "ASL", "LSR", "ROL", "ROR", "INC", "DEC")
            assert _measure([LDX10, LDY20], (op, 0xF8, 0xF0)) == cyc


# ---------------------------------------------------------------------------
# Surrogate rules, each pinned by a hand-derived gradient.  The program's
# result goes to a RAM cell whose output gradient is set, so the leaf
# gradients are the rule's coefficients themselves.
# ---------------------------------------------------------------------------

def _soft(body, ram0, ram_ev=None, grad_cells=None, mode="ste", rom_ev_patch=None):
    rom = A.program(lambda b: (body(b), b.byte(A.JAM_OPCODE)))
    rom_ev = rom.astype(np.float64)
    if rom_ev_patch:
        for off, v in rom_ev_patch.items():
            rom_ev[off] = v
    ram0 = np.asarray(ram0, np.uint8)
    ev0 = ram0.astype(np.float64) if ram_ev is None else np.asarray(ram_ev, np.float64)
    gr = np.zeros((1, 128))
    for cell, w in (grad_cells or {}).items():
        gr[0, cell] = w
    act = np.zeros(1, np.uint8)
    sw = np.array([float(O.action_ports(0)[0])])
    ip = np.array([float(O.action_ports(0)[1])])
    r = O.soft_env(rom, rom_ev, MAP_4K, ram0, ev0, act, sw, ip, 1, 1, mode=mode, grad_ram=gr)
    return r, rom


def _ram(vals):
    r = np.zeros(128, np.uint8)
    for k, v in vals.items():
        r[k] = v
    return r


MODES = ["ste", "smooth"]


@pytest.mark.parametrize("mode", MODES)
def test_sbc_binary_minus_one(mode):
    # LDA $80 ; SEC ; SBC $81 ; STA $82:  r = A - M (no borrow), dr/dA = 1, dr/dM = -1
    ram0 = _ram({0: 0x53, 1: 0x21})
    ev = ram0.astype(float)
    if mode == "smooth":
        ev[0] += 0.25
        ev[1] -= 0.5
    r, _ = _soft(lambda b: (b.ins("LDA", "zp", 0x80), b.ins("SEC"), b.ins("SBC", "zp", 0x81),
                            b.ins("STA", "zp", 0x82)), ram0, ev, {2: 1.0}, mode)
    assert r["ram"][0, 2] == 0x32
    assert r["g_ram0"][0] == 1.0 and r["g_ram0"][1] == -1.0
    # smooth forward value: hard + (a_s - a) - (m_s - m)
    assert r["ram_smooth"][0, 2] == pytest.approx(0x32 + (ev[0] - 0x53) - (ev[1] - 0x21), abs=1e-12)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("opcode", [0xE9, 0xEB])  # SBC #imm and its $EB alias
def test_sbc_decimal_immediate_minus_one(mode, opcode):
    # SED ; LDA $80 ; SEC ; SBC #$17 ; STA $82 ; CLD  -> $52 - $17 = $35 in BCD,
    # with the decimal correction switch held: dr/dA = 1, dr/d(imm) = -1
    def body(b):
        b.ins("SED")
        b.ins("LDA", "zp", 0x80)
        b.ins("SEC")
        b.raw(opcode, 0x17)
        b.ins("STA", "zp", 0x82)
        b.ins("CLD")
    ram0 = _ram({0: 0x52})
    ev = ram0.astype(float) + (0.125 if mode == "smooth" else 0.0)
    r, rom = _soft(body, ram0, ev, {2: 1.0}, mode, rom_ev_patch={5: 0x17 - 0.375} if mode == "smooth" else None)
    assert rom[5] == 0x17 and r["ram"][0, 2] == 0x35
    assert r["g_ram0"][0] == 1.0 and r["g_rom"][5] == -1.0
    assert np.count_nonzero(r["g_rom"]) == 1
    if mode == "smooth":
        assert r["ram_smooth"][0, 2] == pytest.approx(0x35 + 0.125 + 0.375, abs=1e-12)


@pytest.mark.parametrize("mode", MODES)
def test_adc_decimal_plus_one(mode):
    # SED ; CLC ; LDA $80 ; ADC $81 ; STA $82:  $38 + $29 = $67 (BCD)
    def body(b):
        b.ins("SED")
        b.ins("CLC")
        b.ins("LDA", "zp", 0x80)
        b.ins("ADC", "zp", 0x81)
        b.ins("STA", "zp", 0x82)
    ram0 = _ram({0: 0x38, 1: 0x29})
    r, _ = _soft(body, ram0, ram0.astype(float) + (0.5 if mode == "smooth" else 0), {2: 2.0}, mode)
    assert r["ram"][0, 2] == 0x67
    assert r["g_ram0"][0] == 2.0 and r["g_ram0"][1] == 2.0


SHIFTS = [  # (mnemonic, accumulator coefficient, result for 0xB5 with carry in 1)
    ("ASL", 2.0, (0xB5 << 1) & 0xFF),
    ("ROL", 2.0, ((0xB5 << 1) | 1) & 0xFF),
    ("LSR", 0.5, 0xB5 >> 1),
    ("ROR", 0.5, (0xB5 >> 1) | 0x80),
]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("mn,k,want", SHIFTS)
def test_shift_rules_accumulator(mode, mn, k, want):
    # SEC ; LDA $80 ; <op> A ; STA $82
    ram0 = _ram({0: 0xB5})
    ev = ram0.astype(float) + (0.75 if mode == "smooth" else 0.0)
    r, _ = _soft(lambda b: (b.ins("SEC"), b.ins("LDA", "zp", 0x80), b.ins(mn, "acc"), b.ins("STA", "zp", 0x82)),
                 ram0, ev, {2: 1.0}, mode)
    assert r["ram"][0, 2] == want
    assert r["g_ram0"][0] == k
    assert r["ram_smooth"][0, 2] == pytest.approx(want + k * (ev[0] - 0xB5), abs=1e-12)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("mn,k,want", SHIFTS)
@pytest.mark.parametrize("addr_mode", ["zp", "zpx", "abs", "abx"])
def test_shift_rules_in_memory(mode, mn, k, want, addr_mode):
    # SEC ; LDX #1 ; <op> mem  with mem = RAM cell 1 ($81): RAM_out[1] = op(RAM0[1])
    ram0 = _ram({1: 0xB5})
    ev = ram0.astype(float) + (0.75 if mode == "smooth" else 0.0)
    operand = {"zp": 0x81, "zpx": 0x80, "abs": 0x0081, "abx": 0x0080}[addr_mode]
    r, _ = _soft(lambda b: (b.ins("SEC"), b.ins("LDX", "imm", 1), b.ins(mn, addr_mode, operand)),
                 ram0, ev, {1: 1.0}, mode)
    assert r["ram"][0, 1] == want
    assert r["g_ram0"][1] == k
    assert np.count_nonzero(r["g_ram0"]) == 1


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("mn,k", [("INC", 1), ("DEC", -1)])
def test_inc_dec_memory_unit_coefficient(mode, mn, k):
    ram0 = _ram({5: 0x00 if mn == "DEC" else 0xFF})  # both wrap: the wrap switch is held
    ev = ram0.astype(float) + (0.3 if mode == "smooth" else 0.0)
    r, _ = _soft(lambda b: b.ins(mn, "zp", 0x85), ram0, ev, {5: 3.0}, mode)
    assert r["ram"][0, 5] == (int(ram0[5]) + k) & 0xFF
    assert r["g_ram0"][5] == 3.0
    assert r["ram_smooth"][0, 5] == pytest.approx(r["ram"][0, 5] + 0.3 * (mode == "smooth"), abs=1e-12)


REGISTER_CHAINS = [  # (load, op, store, result of 0x41)
    (("LDX", "zp"), "INX", ("STX", "zp"), 0x42),
    (("LDX", "zp"), "DEX", ("STX", "zp"), 0x40),
    (("LDY", "zp"), "INY", ("STY", "zp"), 0x42),
    (("LDY", "zp"), "DEY", ("STY", "zp"), 0x40),
    (("LDA", "zp"), "TAX", ("STX", "zp"), 0x41),
    (("LDA", "zp"), "TAY", ("STY", "zp"), 0x41),
    (("LDX", "zp"), "TXA", ("STA", "zp"), 0x41),
    (("LDY", "zp"), "TYA", ("STA", "zp"), 0x41),
]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("load,op,store,want", REGISTER_CHAINS)
def test_register_increments_and_transfers_unit_coefficient(mode, load, op, store, want):
    ram0 = _ram({0: 0x41})
    ev = ram0.astype(float) + (0.2 if mode == "smooth" else 0.0)
    r, _ = _soft(lambda b: (b.ins(*load, 0x80), b.ins(op), b.ins(*store, 0x82)), ram0, ev, {2: 1.5}, mode)
    assert r["ram"][0, 2] == want
    assert r["g_ram0"][0] == 1.5 and np.count_nonzero(r["g_ram0"]) == 1
    assert r["ram_smooth"][0, 2] == pytest.approx(want + 0.2 * (mode == "smooth"), abs=1e-12)


@pytest.mark.parametrize("mode", MODES)
def test_transfer_overwrites_the_destination_adjoint(mode):
    # LDX $81 ; LDA $80 ; TAX ; STX $82: X's first value (RAM0[1]) is overwritten by TAX
    ram0 = _ram({0: 0x11, 1: 0x22})
    r, _ = _soft(lambda b: (b.ins("LDX", "zp", 0x81), b.ins("LDA", "zp", 0x80), b.ins("TAX"),
                            b.ins("STX", "zp", 0x82)), ram0, None, {2: 1.0}, mode)
    assert r["g_ram0"][0] == 1.0 and r["g_ram0"][1] == 0.0


@pytest.mark.parametrize("mode", MODES)
def test_pha_pla_through_the_stack(mode):
    # LDA $80 ; PHA ; LDA #$00 ; PLA ; STA $82:  the value goes to $01FD (RAM cell
    # $7D through the stack mirror) and back; the immediate it displaced in A and the
    # RAM cell the push overwrote get structural zeros
    ram0 = _ram({0: 0x9C, 0x7D: 0x33})
    ev = ram0.astype(float) + (0.4 if mode == "smooth" else 0.0)
    r, rom = _soft(lambda b: (b.ins("LDA", "zp", 0x80), b.ins("PHA"), b.ins("LDA", "imm", 0x00), b.ins("PLA"),
                              b.ins("STA", "zp", 0x82)), ram0, ev, {2: 1.0, 0x7D: 0.5}, mode)
    assert r["ram"][0, 2] == 0x9C and r["ram"][0, 0x7D] == 0x9C
    assert r["g_ram0"][0] == 1.5  # through PLA->STA (1.0) and through the stack cell's own output (0.5)
    assert r["g_ram0"][0x7D] == 0.0
    assert np.count_nonzero(r["g_rom"]) == 0


@pytest.mark.parametrize("mode", MODES)
def test_lax_feeds_a_and_x(mode):
    # LAX $80 ; STA $82 ; STX $83:  dL/dRAM0[0] = w2 + w3
    ram0 = _ram({0: 0x6E})
    r, _ = _soft(lambda b: (b.ins("LAX", "zp", 0x80), b.ins("STA", "zp", 0x82), b.ins("STX", "zp", 0x83)),
                 ram0, ram0.astype(float) + (0.1 if mode == "smooth" else 0.0), {2: 2.0, 3: 5.0}, mode)
    assert r["ram"][0, 2] == 0x6E and r["ram"][0, 3] == 0x6E
    assert r["g_ram0"][0] == 7.0


LOGIC = [  # (mnemonic, hard op, d/dA at (a, m), d/dM at (a, m))
    ("AND", lambda a, m: a & m, lambda a, m: m / 255.0, lambda a, m: a / 255.0),
    ("ORA", lambda a, m: a | m, lambda a, m: (255.0 - m) / 255.0, lambda a, m: (255.0 - a) / 255.0),
    ("EOR", lambda a, m: a ^ m, lambda a, m: (255.0 - 2 * m) / 255.0, lambda a, m: (255.0 - 2 * a) / 255.0),
]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("mn,op,da,dm", LOGIC)
def test_logic_rules_bit_uniform_multilinear(mode, mn, op, da, dm):
    # LDA $80 ; <op> $81 ; STA $82.  The extensions: A&M ~ AM/255, A|M ~ A+M-AM/255,
    # A^M ~ A+M-2AM/255; STE takes the partials at the hard bytes, SMOOTH at the
    # smooth values, and the SMOOTH forward value is hard + ext(smooth) - ext(hard).
    a, m = 0xB6, 0x5B
    ram0 = _ram({0: a, 1: m})
    ev = ram0.astype(float)
    if mode == "smooth":
        ev[0] += 0.3
        ev[1] -= 0.6
    r, _ = _soft(lambda b: (b.ins("LDA", "zp", 0x80), b.ins(mn, "zp", 0x81), b.ins("STA", "zp", 0x82)),
                 ram0, ev, {2: 1.0}, mode)
    assert r["ram"][0, 2] == op(a, m)
    pa, pm = (a, m) if mode == "ste" else (ev[0], ev[1])
    assert r["g_ram0"][0] == pytest.approx(da(pa, pm), rel=1e-14)
    assert r["g_ram0"][1] == pytest.approx(dm(pa, pm), rel=1e-14)
    ext = {"AND": lambda x, y: x * y / 255.0, "ORA": lambda x, y: x + y - x * y / 255.0,
           "EOR": lambda x, y: x + y - 2 * x * y / 255.0}[mn]
    if mode == "smooth":
        assert r["ram_smooth"][0, 2] == pytest.approx(op(a, m) + ext(ev[0], ev[1]) - ext(a, m), abs=1e-12)


@pytest.mark.parametrize("mode", MODES)
def test_logic_rules_exact_at_identity_and_complement(mode):
    # ORA #$00 is the identity (d/dA = 1), EOR #$FF the complement (d/dA = -1),
    # AND #$FF the identity (d/dA = 1): the extension is exact there
    for mn, imm, k in (("ORA", 0x00, 1.0), ("EOR", 0xFF, -1.0), ("AND", 0xFF, 1.0)):
        ram0 = _ram({0: 0x3C})
        r, rom = _soft(lambda b: (b.ins("LDA", "zp", 0x80), b.ins(mn, "imm", imm), b.ins("STA", "zp", 0x82)),
                       ram0, None, {2: 1.0}, mode)
        assert r["g_ram0"][0] == k, mn


@pytest.mark.parametrize("mode", MODES)
def test_sax_rule(mode):
    # LDA $80 ; LDX $81 ; SAX $82:  mem = A & X, d/dA = X/255, d/dX = A/255
    a, x = 0xE7, 0x3D
    ram0 = _ram({0: a, 1: x})
    ev = ram0.astype(float)
    if mode == "smooth":
        ev[0] -= 0.2
        ev[1] += 0.9
    r, _ = _soft(lambda b: (b.ins("LDA", "zp", 0x80), b.ins("LDX", "zp", 0x81), b.ins("SAX", "zp", 0x82)),
                 ram0, ev, {2: 1.0}, mode)
    assert r["ram"][0, 2] == a & x
    pa, px = (a, x) if mode == "ste" else (ev[0], ev[1])
    assert r["g_ram0"][0] == pytest.approx(px / 255.0, rel=1e-14)
    assert r["g_ram0"][1] == pytest.approx(pa / 255.0, rel=1e-14)


@pytest.mark.parametrize("mode", MODES)
def test_compare_flags_and_addresses_carry_no_gradient(mode):
    # CMP/CPX/CPY/BIT results and flags are not content: a value that only feeds a
    # compare and a branch reaches nothing; an index register that only forms an
    # address reaches nothing either (LDX $81 ; LDA $90,X ; STA $82)
    def body(b):
        b.ins("LDA", "zp", 0x80)
        b.ins("CMP", "zp", 0x83)
        b.ins("BIT", "zp", 0x84)
        b.ins("LDX", "zp", 0x81)
        b.ins("CPX", "imm", 0x01)
        b.ins("LDA", "zpx", 0x90)
        b.ins("STA", "zp", 0x82)
    ram0 = _ram({0: 0x10, 1: 0x02, 3: 0x10, 4: 0xC0, 0x12: 0x77})
    r, _ = _soft(body, ram0, None, {2: 1.0}, mode)
    assert r["ram"][0, 2] == 0x77
    assert r["g_ram0"][0x12] == 1.0
    assert np.count_nonzero(r["g_ram0"]) == 1
