"""Pins of the oracle's TIA objects (players, missiles, ball, motion, collisions)
and of the position sampler.

Every expected column below is worked out by hand from the documented timing:
after STA WSYNC the CPU starts at cycle 0 of the next line, a NOP takes 2 cycles
and a zero-page STA writes in its third cycle, so "n NOPs then STA" writes in
cycle 2n + 2 of the line and takes effect at colour clock 3(2n + 3) = 6n + 9;
clock 68 is the first visible column.  The programs finish their writes before
the visible window starts (line 34) and then jam, so every visible row shows the
final state; row 100 is checked.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import asm as A

ROW = 100


def run(body):
    rom = A.program(body)
    m = O.Machine(rom, 1)
    m.env_step(0, 1, 0, True)
    return m.frame(), m, rom


def lit(row, colour):
    return [int(x) for x in np.nonzero(row == colour)[0]]


def strobe(b, reg, nops):
    """STA WSYNC, nops x NOP, STA reg."""
    b.ins("STA", "zp", A.WSYNC)
    for _ in range(nops):
        b.ins("NOP")
    b.ins("STA", "zp", reg)


def setreg(b, reg, v):
    b.ins("LDA", "imm", v)
    b.ins("STA", "zp", reg)


def player_program(grp, nusiz=0, nops=10, refp=0, col=0x44):
    def body(b):
        setreg(b, A.COLUP0, col)
        setreg(b, A.NUSIZ0, nusiz)
        setreg(b, A.REFP0, refp)
        setreg(b, A.GRP0, grp)
        strobe(b, A.RESP0, nops)
        b.byte(A.JAM_OPCODE)
    return body


@pytest.mark.parametrize("nops,pos,cols", [
    (10, 6, list(range(6, 14))),                          # clock 69: column 1, the player 5 columns later
    (0, 3, list(range(3, 11))),                           # clock 9: horizontal blank, column 3
    (11, 12, list(range(12, 20))),                        # clock 75: column 7 + 5
    (35, 156, list(range(0, 4)) + list(range(156, 160))),  # clock 219: column 151 + 5 = 156, wraps to 0..3
])
def test_player_strobe_column(nops, pos, cols):
    f, m, _ = run(player_program(0xFF, nops=nops))
    assert lit(f[ROW], 0x44) == cols
    assert (f[ROW][[c for c in range(160) if c not in cols]] == 0).all()
    assert m.objects()["posP0"] == pos


@pytest.mark.parametrize("nusiz,grp,refp,cols", [
    (0, 0x80, 0, [6]),
    (0, 0x80, 8, [13]),                               # reflected: bit 7 drawn last
    (0, 0x01, 8, [6]),
    (1, 0xFF, 0, list(range(6, 14)) + list(range(22, 30))),
    (2, 0xFF, 0, list(range(6, 14)) + list(range(38, 46))),
    (3, 0x81, 0, [6, 13, 22, 29, 38, 45]),
    (4, 0xC0, 0, [6, 7, 70, 71]),
    (5, 0x01, 0, [20, 21]),                           # double width: bit 0 covers columns 14..15 of the copy
    (6, 0x01, 0, [13, 45, 77]),
    (7, 0x80, 0, [6, 7, 8, 9]),                       # quad width: bit 7 covers 4 columns
    (7, 0x41, 0, [10, 11, 12, 13, 34, 35, 36, 37]),
])
def test_player_copies_sizes_and_reflection(nusiz, grp, refp, cols):
    f, _, _ = run(player_program(grp, nusiz=nusiz, refp=refp))
    assert lit(f[ROW], 0x44) == cols


def test_missile_and_ball_columns_and_widths():
    def body(b):
        setreg(b, A.COLUP0, 0x44)
        setreg(b, A.COLUPF, 0x88)
        setreg(b, A.NUSIZ0, 0x20)   # missile 4 wide, one copy
        setreg(b, A.ENAM0, 0x02)
        setreg(b, A.CTRLPF, 0x30)   # ball 8 wide
        setreg(b, A.ENABL, 0x02)
        strobe(b, A.RESM0, 10)      # clock 69: column 1 + 4 = 5
        strobe(b, A.RESBL, 12)      # clock 81: column 13 + 4 = 17
        b.byte(A.JAM_OPCODE)
    f, m, _ = run(body)
    assert lit(f[ROW], 0x44) == [5, 6, 7, 8]
    assert lit(f[ROW], 0x88) == list(range(17, 25))
    o = m.objects()
    assert (o["posM0"], o["posBL"]) == (5, 17)


def test_missile_copies_follow_the_player_mode():
    def body(b):
        setreg(b, A.COLUP1, 0x66)
        setreg(b, A.NUSIZ1, 0x13)   # three close copies, missile 2 wide
        setreg(b, A.ENAM1, 0x02)
        strobe(b, A.RESM1, 10)      # column 5
        b.byte(A.JAM_OPCODE)
    f, _, _ = run(body)
    assert lit(f[ROW], 0x66) == [5, 6, 21, 22, 37, 38]


@pytest.mark.parametrize("hm,cols", [
    (0x30, list(range(3, 11))),                       # +3: three columns left
    (0xD0, list(range(9, 17))),                       # -3: three columns right
    (0x70, [0, 1, 2, 3, 4, 5, 6, 159]),               # +7 from 6 wraps to 159
    (0x80, list(range(14, 22))),                      # -8: eight right
])
def test_hmove_moves_by_the_signed_motion_nibble(hm, cols):
    def body(b):
        setreg(b, A.COLUP0, 0x44)
        setreg(b, A.GRP0, 0xFF)
        strobe(b, A.RESP0, 10)      # column 6
        setreg(b, A.HMP0, hm)
        b.ins("STA", "zp", A.WSYNC)
        b.ins("STA", "zp", A.HMOVE)
        b.byte(A.JAM_OPCODE)
    f, m, _ = run(body)
    assert lit(f[ROW], 0x44) == cols
    assert m.objects()["HMP0"] == hm


def test_hmclr_clears_motion_and_a_second_hmove_moves_again():
    def body(b):
        setreg(b, A.COLUP0, 0x44)
        setreg(b, A.GRP0, 0x80)
        strobe(b, A.RESP0, 10)      # column 6
        setreg(b, A.HMP0, 0x20)     # +2
        b.ins("STA", "zp", A.WSYNC)
        b.ins("STA", "zp", A.HMOVE)  # 4
        b.ins("STA", "zp", A.WSYNC)
        b.ins("STA", "zp", A.HMOVE)  # 2
        b.ins("STA", "zp", A.HMCLR)
        b.ins("STA", "zp", A.WSYNC)
        b.ins("STA", "zp", A.HMOVE)  # stays 2
        b.byte(A.JAM_OPCODE)
    f, m, _ = run(body)
    assert lit(f[ROW], 0x44) == [2]
    assert m.objects()["HMP0"] == 0


def test_hmove_in_horizontal_blank_blanks_eight_columns_of_its_line():
    # 100 x WSYNC reaches line 100; DEX + BNE (not taken) then STA HMOVE writes
    # in cycle 6 (clock 21, horizontal blank): row 66 = line 100 - 34.
    def body(b):
        setreg(b, A.COLUBK, 0x0E)
        b.ins("LDX", "imm", 100)
        b.label("W")
        b.ins("STA", "zp", A.WSYNC)
        b.ins("DEX")
        b.ins("BNE", "rel", "W")
        b.ins("STA", "zp", A.HMOVE)
        b.byte(A.JAM_OPCODE)
    f, _, _ = run(body)
    assert (f[66, :8] == 0).all() and (f[66, 8:] == 0x0E).all()
    f2 = np.delete(f, 66, axis=0)
    assert (f2 == 0x0E).all()


def test_vertical_delay_of_players_and_ball():
    def body(gp1_write, vdel):
        def b_(b):
            setreg(b, A.COLUP0, 0x44)
            setreg(b, A.COLUPF, 0x88)
            setreg(b, A.VDELP0, vdel)
            setreg(b, A.VDELBL, vdel)
            setreg(b, A.ENABL, 0x02)
            setreg(b, A.GRP0, 0xFF)
            if gp1_write:
                setreg(b, A.GRP1, 0x00)  # copies GRP0 and ENABL into their old registers
            strobe(b, A.RESP0, 10)
            strobe(b, A.RESBL, 12)
            b.byte(A.JAM_OPCODE)
        return b_
    f, _, _ = run(body(False, 1))
    assert lit(f[ROW], 0x44) == [] and lit(f[ROW], 0x88) == []       # old registers still 0
    f, m, _ = run(body(True, 1))
    assert lit(f[ROW], 0x44) == list(range(6, 14)) and lit(f[ROW], 0x88) == [17]
    o = m.objects()
    assert (o["GRP0"], o["GRP0old"], o["ENABL"], o["ENABLold"]) == (0xFF, 0xFF, 2, 2)
    f, _, _ = run(body(False, 0))
    assert lit(f[ROW], 0x44) == list(range(6, 14)) and lit(f[ROW], 0x88) == [17]


def test_resmp_hides_the_missile_and_centres_it_on_release():
    def body(b):
        setreg(b, A.COLUP0, 0x44)
        setreg(b, A.ENAM0, 0x02)
        strobe(b, A.RESP0, 10)      # player column 6 (GRP0 = 0: not drawn)
        setreg(b, A.RESMP0, 0x02)
        setreg(b, A.RESMP0, 0x00)   # missile to 6 + 4
        b.byte(A.JAM_OPCODE)
    f, m, _ = run(body)
    assert lit(f[ROW], 0x44) == [10]

    def held(b):
        setreg(b, A.COLUP0, 0x44)
        setreg(b, A.ENAM0, 0x02)
        setreg(b, A.RESMP0, 0x02)
        b.byte(A.JAM_OPCODE)
    f, _, _ = run(held)
    assert lit(f[ROW], 0x44) == []


@pytest.mark.parametrize("ctrlpf,c67", [(0x00, 0x44), (0x04, 0x88)])
def test_priority_of_players_and_playfield(ctrlpf, c67):
    def body(b):
        setreg(b, A.COLUP0, 0x44)
        setreg(b, A.COLUPF, 0x88)
        setreg(b, A.CTRLPF, ctrlpf)
        setreg(b, A.PF0, 0x30)      # playfield columns 0..7 and 80..87
        setreg(b, A.GRP0, 0xFF)
        strobe(b, A.RESP0, 10)      # player columns 6..13
        b.byte(A.JAM_OPCODE)
    f, _, _ = run(body)
    row = f[ROW]
    assert (row[0:6] == 0x88).all() and row[6] == c67 and row[7] == c67
    assert (row[8:14] == 0x44).all() and (row[80:88] == 0x88).all()


def test_player0_over_player1_and_missile0_colour():
    def body(b):
        setreg(b, A.COLUP0, 0x44)
        setreg(b, A.COLUP1, 0x66)
        setreg(b, A.GRP0, 0xFF)
        setreg(b, A.GRP1, 0xFF)
        setreg(b, A.ENAM0, 0x02)    # missile 0 at its power-on column 0
        strobe(b, A.RESP0, 10)      # 6..13
        strobe(b, A.RESP1, 11)      # 12..19
        b.ins("STA", "zp", A.WSYNC)
        b.ins("STA", "zp", A.CXCLR)  # forget the lines drawn before the strobes
        b.byte(A.JAM_OPCODE)
    f, m, _ = run(body)
    assert lit(f[ROW], 0x44) == [0] + list(range(6, 14))
    assert lit(f[ROW], 0x66) == list(range(14, 20))
    o = m.objects()
    assert o["CXhi"] == 0x40     # pair 14 (P0-P1) latched; M0-M1 (pair 15) not
    assert o["CXlo"] == 0


def test_collision_read_clear_and_relatch():
    # P0 (6..13) and the playfield (0..7) overlap at columns 6, 7.  After two
    # WSYNCs a whole line has been drawn: LDA CXP0FB reads bit 7 in cycle 2;
    # STA CXCLR takes effect at clock 27 (blank), LDA CXP0FB in cycle 11 sees
    # clocks < 36: clear; the next line latches it again.
    def body(b):
        setreg(b, A.GRP0, 0xFF)
        setreg(b, A.PF0, 0x30)
        strobe(b, A.RESP0, 10)
        b.ins("STA", "zp", A.WSYNC)
        b.ins("STA", "zp", A.WSYNC)
        b.ins("LDA", "zp", A.CXP0FB)
        b.ins("STA", "zp", 0x80)
        b.ins("STA", "zp", A.CXCLR)
        b.ins("LDA", "zp", A.CXP0FB)
        b.ins("STA", "zp", 0x81)
        b.ins("STA", "zp", A.WSYNC)
        b.ins("LDA", "zp", A.CXP0FB)
        b.ins("STA", "zp", 0x82)
        b.ins("LDA", "zp", A.CXPPMM)  # no P0-P1 overlap: P1 has no graphics
        b.ins("STA", "zp", 0x83)
        b.byte(A.JAM_OPCODE)
    _, m, _ = run(body)
    assert m.ram()[:4].tolist() == [0x80, 0x00, 0x80, 0x00]


def test_collision_pairs_latch_exactly_the_overlaps():
    def body(b):
        setreg(b, A.GRP0, 0xFF)
        setreg(b, A.GRP1, 0xFF)
        setreg(b, A.ENAM0, 0x02)
        setreg(b, A.ENAM1, 0x02)
        setreg(b, A.ENABL, 0x02)
        setreg(b, A.PF0, 0x30)
        b.ins("STA", "zp", A.WSYNC)
        for _ in range(10):
            b.ins("NOP")
        b.ins("STA", "zp", A.RESP0)   # clock 69: column 6
        b.ins("STA", "zp", A.RESP1)   # clock 78: column 10 + 5 = 15: 15..22
        b.ins("STA", "zp", A.RESM0)   # clock 87: column 19 + 4 = 23
        b.ins("STA", "zp", A.WSYNC)
        b.ins("STA", "zp", A.CXCLR)   # forget the lines drawn before the strobes
        b.byte(A.JAM_OPCODE)
    _, m, _ = run(body)
    o = m.objects()
    assert (o["posP0"], o["posP1"], o["posM0"]) == (6, 15, 23)
    # P0 6..13, P1 15..22, M0 23, M1 and BL at column 0, playfield 0..7 and 80..87:
    # P0-PF (6, 7), M1-PF and BL-PF (0), M1-BL (0); nothing else
    cx = o["CXlo"] | o["CXhi"] << 8
    want = (1 << 4) | (1 << 10) | (1 << 11) | (1 << 12)
    assert cx == want


def test_sampler_derivative_of_a_ball_and_a_player():
    # ball at 17..24 in COLUPF = $46 on a black background; dL/dpixel = column
    # index.  Moving it right by one turns column 17 black and column 25 on:
    # per row 17 * (0 - 70) + 25 * 70 = 8 * 70, over 210 rows = 117,600.
    def ball(b):
        setreg(b, A.COLUPF, 0x46)
        setreg(b, A.CTRLPF, 0x30)
        setreg(b, A.ENABL, 0x02)
        strobe(b, A.RESBL, 12)
        b.byte(A.JAM_OPCODE)
    # player GRP0 = $81 at 6: columns 6 and 13 in $44 = 68; moving right:
    # -68 at 6 and 13, +68 at 7 and 14: per row 68 * 2, over 210 rows = 28,560
    def player(b):
        setreg(b, A.COLUP0, 0x44)
        setreg(b, A.GRP0, 0x81)
        strobe(b, A.RESP0, 10)
        b.byte(A.JAM_OPCODE)
    gf = np.tile(np.arange(160, dtype=np.float64), (210, 1))
    for body, obj, want in ((ball, 4, 117600.0), (player, 0, 28560.0)):
        rom = A.program(body)
        act = np.zeros(1, np.uint8)
        sw, ip = O.action_ports(0)
        r = O.soft_env(rom, rom.astype(np.float64), 1, np.zeros(128, np.uint8), np.zeros(128), act,
                       np.array([sw], np.float64), np.array([ip], np.float64), 1, 1, grad_frame=gf)
        others = [k for k in range(5) if k != obj]
        assert r["g_pos"][obj] == pytest.approx(want, rel=1e-12)
        assert (r["g_pos"][others] == 0).all()
        # uniform dL/dpixel: a shift moves colour mass without changing it
        r1 = O.soft_env(rom, rom.astype(np.float64), 1, np.zeros(128, np.uint8), np.zeros(128), act,
                        np.array([sw], np.float64), np.array([ip], np.float64), 1, 1,
                        grad_frame=np.ones((210, 160)))
        assert abs(r1["g_pos"][obj]) < 1e-9


def test_object_pixels_route_their_gradient_to_the_colour_register():
    # P0 ($81 at 6) shows 2 pixels per row in COLUP0 from LDA #$44 (operand byte 1):
    # with dL/dpixel = 1 that byte's gradient is 2 * 210 = 420; COLUBK was never
    # written (power-on constant), so no other ROM byte gets any.
    def body(b):
        setreg(b, A.COLUP0, 0x44)
        setreg(b, A.GRP0, 0x81)
        strobe(b, A.RESP0, 10)
        b.byte(A.JAM_OPCODE)
    rom = A.program(body)
    sw, ip = O.action_ports(0)
    r = O.soft_env(rom, rom.astype(np.float64), 1, np.zeros(128, np.uint8), np.zeros(128), np.zeros(1, np.uint8),
                   np.array([sw], np.float64), np.array([ip], np.float64), 1, 1, grad_frame=np.ones((210, 160)))
    assert r["g_rom"][1] == pytest.approx(420.0, rel=1e-12)
    assert np.count_nonzero(r["g_rom"]) == 1
