"""Pins of the reference emulator's HARD mode against things other than itself.

Each test checks the oracle against an independent source: the arithmetic
definition of an operation, the documented MOS 6502 cycle counts, a
hand-assembled program whose final state is derived by hand, a tick-by-tick
model of the RIOT timer, or the published SplitMix64 output.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import inputs as I
from tests import asm as A

MAP_2K, MAP_4K, MAP_F8 = 0, 1, 2


def s8(v):
    return v - 256 if v >= 128 else v


# --------------------------------------------------------------------------
# opcode set (Sec. "Building Two Differentiable VCS Ports": 151 documented +
# the USBC alias + 37 illegal NOP/LAX/SAX bytes = 189)
# --------------------------------------------------------------------------

def test_opcode_set_is_the_papers_189_bytes():
    impl = [op for op in range(256) if O.opcode_info(op)[0]]
    assert len(impl) == 189
    illegal_nop = {0x1A, 0x3A, 0x5A, 0x7A, 0xDA, 0xFA, 0x80, 0x82, 0x89, 0xC2, 0xE2, 0x04, 0x44, 0x64,
                   0x14, 0x34, 0x54, 0x74, 0xD4, 0xF4, 0x0C, 0x1C, 0x3C, 0x5C, 0x7C, 0xDC, 0xFC}
    lax = {0xA7, 0xB7, 0xAF, 0xBF, 0xA3, 0xB3}
    sax = {0x87, 0x97, 0x8F, 0x83}
    assert len(illegal_nop | lax | sax) == 37
    documented = {v for (mn, mode), v in I.OPCODES.items() if mn not in ("LAX", "SAX", "USBC")}
    assert len(documented) == 151
    assert set(impl) == documented | illegal_nop | lax | sax | {0xEB}


# --------------------------------------------------------------------------
# ADC / SBC against their arithmetic definitions
# --------------------------------------------------------------------------

def test_adc_sbc_binary_bruteforce_vs_definition():
    for c in (0, 1):
        for a in range(256):
            for m in range(256):
                r, p = O.alu("ADC", a, m, 0x20 | c)
                u = a + m + c
                s = s8(a) + s8(m) + c
                assert r == u % 256
                assert (p & 1) == (u >= 256)
                assert bool(p & 0x40) == (not -128 <= s <= 127)
                assert bool(p & 0x80) == (r >= 128) and bool(p & 0x02) == (r == 0)
                r, p = O.alu("SBC", a, m, 0x20 | c)
                d = a - m - (1 - c)
                sd = s8(a) - s8(m) - (1 - c)
                assert r == d % 256
                assert (p & 1) == (d >= 0)
                assert bool(p & 0x40) == (not -128 <= sd <= 127)
                assert bool(p & 0x80) == (r >= 128) and bool(p & 0x02) == (r == 0)


def bcd(n):
    return (n // 10) * 16 + n % 10


def test_decimal_valid_bcd_bruteforce_vs_decimal_arithmetic():
    for c in (0, 1):
        for x in range(100):
            for y in range(100):
                r, p = O.alu("ADC", bcd(x), bcd(y), 0x28 | c)
                assert r == bcd((x + y + c) % 100)
                assert (p & 1) == (x + y + c >= 100)
                r, p = O.alu("SBC", bcd(x), bcd(y), 0x28 | c)
                assert r == bcd((x - y - (1 - c)) % 100)
                assert (p & 1) == (x - y - (1 - c) >= 0)


def test_decimal_worked_examples():
    assert O.alu("ADC", 0x19, 0x28, 0x28)[0] == 0x47
    r, p = O.alu("SBC", 0x50, 0x01, 0x29)
    assert r == 0x49 and p & 1
    r, p = O.alu("ADC", 0x99, 0x01, 0x28)
    assert r == 0x00 and p & 1
    # NMOS: Z follows the binary sum ($9A != 0) even though the BCD result is 0
    assert not (p & 0x02)
    # SBC flags follow binary subtraction
    r, p = O.alu("SBC", 0x00, 0x01, 0x29)
    assert r == 0x99 and not (p & 1) and (p & 0x80)


# --------------------------------------------------------------------------
# documented cycle counts, measured instruction by instruction
# --------------------------------------------------------------------------

def _deltas(rom, n, ram0=None):
    m = O.Machine(rom, MAP_4K, ram0)
    out = []
    for _ in range(n):
        c0 = m.regs()["cycle"]
        m.step()
        out.append(m.regs()["cycle"] - c0)
    return out, m


def test_cycle_counts_per_addressing_mode():
    ram0 = np.zeros(128, np.uint8)
    ram0[0x02:0x04] = [0xF0, 0xF0]   # ($82) -> $F0F0: +$20 crosses into $F1xx
    ram0[0x04:0x06] = [0x00, 0xF0]   # ($84) -> $F000: no crossing
    ram0[0x16:0x18] = [0x00, 0xF0]   # ($86,X) with X=$10 reads ($96)

    def body(b):
        b.ins("LDA", "imm", 1)          # 2
        b.ins("LDA", "zp", 0x80)        # 3
        b.ins("LDX", "imm", 0x10)       # 2
        b.ins("LDA", "zpx", 0x80)       # 4
        b.ins("LDA", "abx", 0xF0F8)     # 4 + 1 (page crossed)
        b.ins("LDA", "abx", 0xF000)     # 4
        b.ins("STA", "abx", 0xF0F8)     # 5 (stores never pay the penalty separately)
        b.ins("LDY", "imm", 0x20)       # 2
        b.ins("LDA", "izy", 0x82)       # 5 + 1
        b.ins("LDA", "izy", 0x84)       # 5
        b.ins("LDA", "izx", 0x86)       # 6
        b.ins("STA", "izy", 0x84)       # 6
        b.ins("INC", "zp", 0x90)        # 5
        b.ins("INC", "zpx", 0x90)       # 6
        b.ins("INC", "abx", 0xF000)     # 7
        b.ins("ASL", "acc")             # 2
        b.ins("PHA")                    # 3
        b.ins("PLA")                    # 4
        b.ins("PHP")                    # 3
        b.ins("PLP")                    # 4
        b.ins("BIT", "zp", 0x80)        # 3
        b.ins("CPX", "abs", 0xF000)     # 4
        b.ins("LAX", "aby", 0xF0F8)     # 4 + 1 (Y=$20)
        b.ins("SAX", "zpy", 0x90)       # 4
        b.raw(0x1C, 0x00, 0xF0)         # NOP abs,X: 4
        b.raw(0x14, 0x90)               # NOP zp,X: 4
        b.raw(0x04, 0x90)               # NOP zp: 3
        b.ins("JSR", "abs", "SUB")      # 6
        b.ins("JMP", "ind", 0xF800)     # 5
        b.label("SUB")
        b.ins("RTS")                    # 6
    rom = A.program(body)
    rom[0x800:0x802] = [0x10, 0xF8]     # pointer at $F800 -> $F810
    rom[0x810] = 0x18                   # CLC at $F810
    expected = [2, 3, 2, 4, 5, 4, 5, 2, 6, 5, 6, 6, 5, 6, 7, 2, 3, 4, 3, 4, 3, 4, 5, 4, 4, 4, 3, 6, 6, 5, 2]
    # JSR (6) -> SUB's RTS (6) -> back at the JMP (5) -> CLC (2)
    got, _ = _deltas(rom, len(expected), ram0)
    assert got == expected, list(zip(got, expected))


def test_branch_cycles_and_loop_total():
    # LDX #10 / DEX / BNE back = 2 + 10*2 + 9*3 + 2 = 51 cycles
    def body(b):
        b.ins("LDX", "imm", 10)
        b.label("L")
        b.ins("DEX")
        b.ins("BNE", "rel", "L")
        b.byte(A.JAM_OPCODE)
    m = O.Machine(A.program(body), MAP_4K)
    while not m.step():
        pass
    assert m.regs()["cycle"] == 51
    assert m.regs()["X"] == 0


def test_branch_page_cross_costs_two_extra():
    img = A.raw_image(4096, {0x0F0: [0xA9, 0x00, 0xF0, 0x20]})  # $F0F0: LDA #0 ; BEQ +$20 -> $F114
    img[0xFFC:0x1000] = [0xF0, 0xF0, 0, 0]
    m = O.Machine(img, MAP_4K)
    m.step()
    c0 = m.regs()["cycle"]
    m.step()
    r = m.regs()
    assert r["cycle"] - c0 == 4 and (r["PCH"] << 8 | r["PCL"]) == 0xF114


def test_wsync_resumes_at_next_line():
    for nops in range(0, 40, 3):
        def body(b, nops=nops):
            for _ in range(nops):
                b.ins("NOP")
            b.ins("STA", "zp", A.WSYNC)
            b.byte(A.JAM_OPCODE)
        m = O.Machine(A.program(body), MAP_4K)
        for _ in range(nops + 1):
            m.step()
        end = 2 * nops + 3
        assert m.regs()["cycle"] == (end + 75) // 76 * 76


# --------------------------------------------------------------------------
# hand-assembled programs with hand-derived final states
# --------------------------------------------------------------------------

def run_to_jam(rom, mapper=MAP_4K, ram0=None, limit=10000):
    m = O.Machine(rom, mapper, ram0)
    for _ in range(limit):
        if m.step():
            break
    return m


def test_arithmetic_chain_and_stack_bytes():
    def body(b):
        b.ins("LDX", "imm", 0xFF)
        b.ins("TXS")
        b.ins("LDA", "imm", 0x37)
        b.ins("CLC")
        b.ins("ADC", "imm", 0x4B)        # 0x82, V=1, N=1
        b.ins("STA", "zp", 0x80)
        b.ins("SEC")
        b.ins("SBC", "imm", 0x03)        # 0x7F, V=1
        b.ins("STA", "zp", 0x81)
        b.ins("ASL", "zp", 0x80)         # 0x04, C=1
        b.ins("ROR", "zp", 0x81)         # 0xBF, C=1
        b.ins("LDA", "imm", 0xF0)
        b.ins("AND", "imm", 0x3C)        # 0x30
        b.ins("ORA", "imm", 0x01)        # 0x31
        b.ins("EOR", "imm", 0xFF)        # 0xCE
        b.ins("STA", "zp", 0x82)
        b.ins("JSR", "abs", "SUB")
        b.byte(A.JAM_OPCODE)
        b.label("SUB")
        b.ins("PHA")
        b.ins("LDA", "imm", 0x11)
        b.ins("STA", "zp", 0x83)
        b.ins("PLA")
        b.byte(A.JAM_OPCODE)
    m = run_to_jam(A.program(body))
    ram = m.ram()
    assert ram[0x00] == 0x04 and ram[0x01] == 0xBF and ram[0x02] == 0xCE and ram[0x03] == 0x11
    # the JSR sits at $F01D (29 bytes of code before it); it pushes the return
    # address - 1 = $F01F at $01FF, $01FE, which the 13-bit decode maps to RAM $7F, $7E
    ret = 0xF01D + 2
    assert ram[0x7F] == ret >> 8 and ram[0x7E] == ret & 0xFF
    assert ram[0x7D] == 0xCE  # PHA inside the subroutine
    r = m.regs()
    assert r["A"] == 0xCE and r["S"] == 0xFD


def test_jmp_indirect_page_wrap():
    img = np.full(4096, A.JAM_OPCODE, np.uint8)
    img[0:3] = [0x6C, 0xFF, 0xF0]   # JMP ($F0FF)
    img[0x0FF] = 0x34               # low byte at $F0FF
    img[0x100] = 0x12               # would be the high byte without the page-wrap bug
    img[0xFFC:0x1000] = [0x00, 0xF0, 0, 0]
    m = O.Machine(img, MAP_4K)
    m.step()
    r = m.regs()
    # the high byte comes from $F000, which holds the opcode $6C itself
    assert (r["PCH"] << 8 | r["PCL"]) == 0x6C34


def test_brk_rti_round_trip():
    def body(b):
        b.ins("LDX", "imm", 0xFF)
        b.ins("TXS")
        b.ins("SED")
        b.ins("BRK")
        b.byte(0xEA)
        b.ins("STA", "zp", 0x81)
        b.byte(A.JAM_OPCODE)

    def handler(b):
        b.ins("LDA", "imm", 0x5A)
        b.ins("STA", "zp", 0x80)
        b.ins("RTI")
    rom = A.program(body, brk_handler=handler)
    m = run_to_jam(rom)
    ram = m.ram()
    assert ram[0x00] == 0x5A and ram[0x01] == 0x5A
    # pushes: PC+2 ($F006 after BRK at $F004) then P|$30 with I, D and N
    # (N from LDX #$FF) set
    assert ram[0x7F] == 0xF0 and ram[0x7E] == 0x06
    assert ram[0x7D] == (0x24 | 0x80 | 0x08 | 0x30)
    assert m.regs()["P"] & 0x08 and not (m.regs()["P"] & 0x10)


def test_zero_page_index_wraps_and_stack_maps_to_ram():
    def body(b):
        b.ins("LDX", "imm", 0x90)
        b.ins("LDA", "imm", 0x77)
        b.ins("STA", "zpx", 0xF5)       # $F5 + $90 wraps to $85 -> RAM[5]
        b.ins("LDX", "imm", 0x81)
        b.ins("TXS")
        b.ins("LDA", "imm", 0x66)
        b.ins("PHA")                    # $0181 -> RAM[1]
        b.byte(A.JAM_OPCODE)
    ram = run_to_jam(A.program(body)).ram()
    assert ram[5] == 0x77 and ram[1] == 0x66


def test_illegal_lax_sax_usbc():
    def body(b):
        b.ins("LAX", "zp", 0x80)        # A = X = RAM[0] = $C3
        b.ins("LDA", "imm", 0x5F)
        b.ins("SAX", "zp", 0x81)        # $5F & $C3 = $43
        b.ins("SEC")
        b.ins("USBC", "imm", 0x10)      # $5F - $10 = $4F
        b.ins("STA", "zp", 0x82)
        b.byte(A.JAM_OPCODE)
    ram0 = np.zeros(128, np.uint8)
    ram0[0] = 0xC3
    m = run_to_jam(A.program(body), ram0=ram0)
    assert m.ram()[1] == 0x43 and m.ram()[2] == 0x4F and m.regs()["X"] == 0xC3


def test_f8_bank_switch_and_hotspot_read_returns_new_bank():
    img = np.full(8192, A.JAM_OPCODE, np.uint8)
    b0, b1 = 0, 4096
    # start bank 1: reset -> $F000 in bank 1: LDA $1FF8 (switch to bank 0)
    img[b1 + 0x000:b1 + 0x003] = [0xAD, 0xF8, 0x1F]
    # continues at $F003 in bank 0: STA $80 ; LDA #$11 ; STA $81 ; LDA $1FF9
    img[b0 + 0x003:b0 + 0x00C] = [0x85, 0x80, 0xA9, 0x11, 0x85, 0x81, 0xAD, 0xF9, 0x1F]
    # continues at $F00C in bank 1: STA $82 ; JAM
    img[b1 + 0x00C:b1 + 0x00E] = [0x85, 0x82]
    img[b0 + 0xFF8] = 0x5A   # read by LDA $1FF8 after switching to bank 0
    img[b1 + 0xFF8] = 0xA5
    img[b0 + 0xFF9] = 0x3C
    img[b1 + 0xFF9] = 0xC3   # read by LDA $1FF9 after switching to bank 1
    for b in (b0, b1):
        img[b + 0xFFC:b + 0x1000] = [0x00, 0xF0, 0x00, 0xF0]
    m = run_to_jam(img, MAP_F8)
    ram = m.ram()
    assert ram[0] == 0x5A and ram[1] == 0x11 and ram[2] == 0xC3
    assert m.regs()["bank"] == 1


def test_2k_mirrors_on_a11():
    img = A.raw_image(2048, {0x000: [0xAD, 0x10, 0xF8, 0x85, 0x80, 0xAD, 0x10, 0xF0, 0x85, 0x81],
                             0x010: [0x99]})
    img[0x7FC:0x800] = [0x00, 0xF8, 0, 0]
    ram = run_to_jam(img, MAP_2K).ram()
    assert ram[0] == 0x99 and ram[1] == 0x99


def test_unimplemented_opcode_jams_and_cycles_still_elapse():
    img = A.raw_image(4096, {0x000: [0xEA, 0x02]})
    img[0xFFC:0x1000] = [0x00, 0xF0, 0, 0]
    m = O.Machine(img, MAP_4K)
    m.env_step(0, 1, 0)
    r = m.regs()
    assert r["jammed"] == 1 and r["cycle"] == 19912 and r["instructions"] == 1


# --------------------------------------------------------------------------
# TIA: write latency, playfield layout, score mode, VBLANK
# --------------------------------------------------------------------------

def _line40_program(nops, colour=0x44, reg=A.COLUBK):
    def body(b):
        b.ins("LDX", "imm", 40)
        b.label("W")
        b.ins("STA", "zp", A.WSYNC)
        b.ins("DEX")
        b.ins("BNE", "rel", "W")
        for _ in range(nops):
            b.ins("NOP")
        b.ins("LDA", "imm", colour)
        b.ins("STA", "zp", reg)
        b.byte(A.JAM_OPCODE)
    return A.program(body)


def test_colubk_write_boundary_pixel():
    # After the 40th WSYNC the CPU is at cycle 0 of line 40: DEX (2) + BNE not
    # taken (2) + k NOPs (2k) + LDA # (2), then STA's write lands in cycle
    # n = 8 + 2k of the line and shows from colour clock 3n + 3, i.e. x = 6k - 41.
    for k in (7, 10, 15, 20, 30, 34):
        m = O.Machine(_line40_program(k), MAP_4K)
        m.set_draw_frame(0)
        m.run_cycles(19912)
        f = m.frame()
        row = f[40 - 34]
        x0 = max(0, min(160, 6 * k - 41))
        assert (row[:x0] == 0).all() and (row[x0:] == 0x44).all(), (k, x0, row)
        assert (f[41 - 34] == 0x44).all() and (f[39 - 34] == 0).all()


def test_pixel_is_colour_and_0xfe_and_vblank_blanks():
    m = O.Machine(_line40_program(30, colour=0x45), MAP_4K)
    m.set_draw_frame(0)
    m.run_cycles(19912)
    assert m.frame()[100, 50] == 0x44

    def body(b):
        b.ins("LDA", "imm", 0x3E)
        b.ins("STA", "zp", A.COLUBK)
        b.ins("LDA", "imm", 0x02)
        b.ins("STA", "zp", A.VBLANK)
        b.byte(A.JAM_OPCODE)
    m = O.Machine(A.program(body), MAP_4K)
    m.set_draw_frame(0)
    m.run_cycles(19912)
    assert (m.frame() == 0).all()


def _pf_program(pf0, pf1, pf2, ctrlpf, c0=0x10, c1=0x20, cpf=0x30, cbk=0x40):
    def body(b):
        for v, r in ((pf0, A.PF0), (pf1, A.PF1), (pf2, A.PF2), (ctrlpf, A.CTRLPF), (c0, A.COLUP0),
                     (c1, A.COLUP1), (cpf, A.COLUPF), (cbk, A.COLUBK)):
            b.ins("LDA", "imm", v)
            b.ins("STA", "zp", r)
        b.byte(A.JAM_OPCODE)
    return A.program(body)


@pytest.mark.parametrize("ctrlpf", [0x00, 0x01, 0x02, 0x03])
def test_playfield_layout(ctrlpf):
    # Documented layout: 20 bits per half line, 4 colour clocks each, in the
    # order PF0 bits 4..7, PF1 bits 7..0, PF2 bits 0..7; the right half repeats
    # or (CTRLPF bit 0) mirrors it; score mode (bit 1) paints the left half
    # with COLUP0 and the right half with COLUP1.
    pf0, pf1, pf2 = 0xA0, 0x96, 0x3C
    order = [(pf0 >> b) & 1 for b in (4, 5, 6, 7)] + [(pf1 >> b) & 1 for b in range(7, -1, -1)] + \
            [(pf2 >> b) & 1 for b in range(8)]
    right = order[::-1] if ctrlpf & 1 else order
    bits = np.repeat(np.array(order + right), 4)
    pfcol = np.where(np.arange(160) < 80, 0x10, 0x20) if ctrlpf & 2 else np.full(160, 0x30)
    expect = np.where(bits == 1, pfcol, 0x40)
    m = O.Machine(_pf_program(pf0, pf1, pf2, ctrlpf), MAP_4K)
    m.set_draw_frame(0)
    m.run_cycles(19912)
    f = m.frame()
    assert (f[50] == expect).all() and (f[209] == expect).all()


# --------------------------------------------------------------------------
# RIOT: timer against a tick-by-tick counter model; inputs
# --------------------------------------------------------------------------

def timer_tick_model(write_cycle, value, interval, t):
    """Count down tick by tick: one decrement right after the write, then one
    every `interval` cycles; after passing zero it wraps to 255 and decrements
    every cycle."""
    cnt, fast = value, False
    for cyc in range(write_cycle + 1, t + 1):
        k = cyc - write_cycle - 1
        if fast:
            cnt = (cnt - 1) & 255
        elif k % interval == 0:
            if cnt == 0:
                cnt, fast = 255, True
            else:
                cnt -= 1
    return cnt, fast


@pytest.mark.parametrize("reg,interval", [(A.TIM1T, 1), (A.TIM8T, 8), (A.TIM64T, 64), (A.T1024T, 1024)])
def test_intim_matches_tick_model(reg, interval):
    v = 5 if interval == 1024 else 43

    def body(b):
        b.ins("LDA", "imm", v)
        b.ins("STA", "abs", reg)        # write lands in cycle 2 + 3 = 5
        b.byte(A.JAM_OPCODE)
    m = O.Machine(A.program(body), MAP_4K)
    m.step()
    m.step()
    w = 5
    for t in list(range(6, 6 + 3 * interval)) + [w + 1 + v * interval + d for d in (-2, -1, 0, 1, 2, 300)]:
        cnt, fast = timer_tick_model(w, v, interval, t)
        assert m.intim_at(t) == cnt, (t, m.intim_at(t), cnt)
        assert bool(m.timint_at(t) & 0x80) == fast


def test_intim_read_clears_flag_and_inputs():
    def body(b):
        b.ins("LDA", "imm", 2)
        b.ins("STA", "abs", A.TIM1T)    # write in cycle 5 -> underflow at 5+1+2 = 8
        b.ins("NOP")                    # cycles 6-7
        b.ins("NOP")                    # 8-9
        b.ins("LDA", "abs", A.TIMINT)   # read in cycle 13: flag set
        b.ins("STA", "zp", 0x80)
        b.ins("LDA", "abs", A.INTIM)    # read in cycle 20: 255 - (20 - 8) = 243, clears flag
        b.ins("STA", "zp", 0x81)
        b.ins("LDA", "abs", A.TIMINT)
        b.ins("STA", "zp", 0x82)
        b.ins("LDA", "abs", A.SWCHA)
        b.ins("STA", "zp", 0x83)
        b.ins("LDA", "zp", A.INPT4)
        b.ins("STA", "zp", 0x84)
        b.ins("LDA", "abs", A.SWCHB)
        b.ins("STA", "zp", 0x85)
        b.byte(A.JAM_OPCODE)
    m = O.Machine(A.program(body), MAP_4K)
    m.set_action(17)  # DOWNLEFTFIRE
    for _ in range(20):
        if m.step():
            break
    ram = m.ram()
    assert ram[0] == 0x80 and ram[1] == 243 and ram[2] == 0x00
    assert ram[3] == 0xFF & ~0x40 & ~0x20 and ram[4] == 0x00 and ram[5] == 0x0B


def test_action_ports_follow_ale_order():
    names = ["NOOP", "FIRE", "UP", "RIGHT", "LEFT", "DOWN", "UPRIGHT", "UPLEFT", "DOWNRIGHT", "DOWNLEFT",
             "UPFIRE", "RIGHTFIRE", "LEFTFIRE", "DOWNFIRE", "UPRIGHTFIRE", "UPLEFTFIRE", "DOWNRIGHTFIRE",
             "DOWNLEFTFIRE"]
    bit = {"RIGHT": 0x80, "LEFT": 0x40, "DOWN": 0x20, "UP": 0x10}
    for a, n in enumerate(names):
        sw = 0xFF
        for d, b in bit.items():
            if d in n:
                sw &= ~b
        assert O.action_ports(a) == (sw, 0x00 if "FIRE" in n else 0x80)


# --------------------------------------------------------------------------
# SplitMix64 (published outputs) and the in-run reset RAM
# --------------------------------------------------------------------------

def test_splitmix64_published_outputs():
    v1, s = O.splitmix_next(0)
    v2, s = O.splitmix_next(s)
    v3, s = O.splitmix_next(s)
    assert (v1, v2, v3) == (0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F)


def test_reset_ram_matches_generator_streams():
    for env, ep in ((0, 1), (5, 3), (4095, 17)):
        expect = I.byte_stream(I.stream_key(1234, env, ep), 128)
        assert (O.splitmix_ram(1234, env, ep) == expect).all()


# --------------------------------------------------------------------------
# whole-frame properties of the generated workloads
# --------------------------------------------------------------------------

def test_generated_roms_keep_262_line_frames_and_run_clean():
    for seed, size, inp in ((0, 4096, False), (1, 4096, False), (100, 2048, True), (101, 8192, True),
                            (102, 4096, True)):
        rom = I.generate_rom(seed, size, reads_inputs=inp, timer_vblank=inp)
        r = O.run_env(rom.image, rom.mapper, I.initial_ram(seed, 1)[0], np.arange(8, dtype=np.uint8) % 18, 8, 1)
        assert r["regs"]["jammed"] == 0
        f = r["frames"]
        # the picture is stable in position: every frame has the same blank rows
        blank = [(fr == 0).all(axis=1) for fr in f]
        assert all((b == blank[-1]).all() for b in blank[2:])
        assert len(np.unique(f[-1])) > 3


def test_episode_resets_restart_from_power_on():
    rom = I.generate_rom(100, 2048, reads_inputs=True, timer_vblank=True)
    ram0 = I.initial_ram(9, 1)[0]
    acts = np.zeros(10, np.uint8)
    eps = np.array([3, 4, 100], np.uint32)
    r = O.run_env(rom.image, rom.mapper, ram0, acts, 10, 4, ep_steps=eps, seed=77, env_index=5)
    assert r["done"].tolist() == [0, 0, 1, 0, 0, 0, 1, 0, 0, 0]
    # step 3 (first of episode 1) equals step 0 of a fresh run from the SplitMix64 RAM
    fresh = O.run_env(rom.image, rom.mapper, O.splitmix_ram(77, 5, 1), acts, 4, 4)
    assert (r["ram"][3:7] == fresh["ram"][:4]).all() and (r["frames"][3:7] == fresh["frames"][:4]).all()
    assert r["regs"]["episode"] == 2 and r["regs"]["ep_step"] == 3
