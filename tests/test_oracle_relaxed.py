"""Pins of the oracle's FULL relaxed mode (Table s-modes): the sigmoid branch
of Eq. s-branch and the distance-softmax read of Eq. s-read without the
straight-through correction, each cast to an integer; the relaxed dispatch of
Eq. s-select for the one-step bound.

Independent checks: the thresholds the paper prints for its cast-margin model
(Sec. "Forward Bit-Exactness Under Full Relaxation", paragraph "Choosing alpha
and T"), the behaviour of hand-assembled branches and reads on either side of
them, the program independence of the operating point alpha = 6, T = 0.14 on
generated ROMs, monotonicity of the first divergence in alpha, and the terms of
Theorem "Temperature-limit bound" against deviations measured by running the
relaxed reads, branches and all 256 dispatch candidates.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import inputs as I
from tests import asm as A


def test_thresholds_printed_in_the_paper():
    # a branch rounds to its target while |delta| < (1 + e^alpha) / 2
    assert math.log(2 * 127 - 1) == pytest.approx(5.5334, abs=1e-4)        # alpha >= ln(253) ~ 5.5
    assert 0.5 * (1 + math.exp(6)) == pytest.approx(202.21, abs=1e-2)       # tau_b(6) > the largest offset
    # a read is pulled by at most 255 (1 - w0) ~ 510 e^{-1/T} < 1/2 once T <= 1/ln(4*255)
    assert 1 / math.log(4 * 255) == pytest.approx(0.144351, abs=1e-6)       # T* ~ 0.144
    assert 510 * math.exp(-1 / 0.14) == pytest.approx(0.4032, abs=1e-4)     # worst-case pull at T = 0.14
    # one max-amplitude neighbour at T = 0.2: 255 w_1 with w_k ~ e^{-|k|/T}
    z = 1 + 2 * sum(math.exp(-k / 0.2) for k in range(1, 200))
    assert 255 * math.exp(-1 / 0.2) / z == pytest.approx(1.695, abs=1e-3)   # "~1.7 > 1/2"


def _branch_program(delta: int, taken: bool):
    """LDX #$FF / TXS, then a branch of offset delta (taken or not) in a loop of NOPs;
    the branch is the instruction with index 3."""
    def body(b):
        b.ins("LDX", "imm", 0xFF)
        b.ins("TXS")
        b.label("LOOP")
        b.ins("SEC" if taken else "CLC")
        if delta >= 0:
            b.ins("BCS", "rel", 0)
            b.img[b.pos - 1] = delta
            for _ in range(delta):
                b.byte(0xEA)
            b.ins("JMP", "abs", "LOOP")
        else:  # a backward branch: its target is NOP padding before the branch, ending in JMP LOOP
            b.ins("JMP", "abs", "BR")
            for _ in range(-delta - 5):
                b.byte(0xEA)
            b.ins("JMP", "abs", "LOOP")
            b.label("BR")
            b.ins("BCS", "rel", 0)
            b.img[b.pos - 1] = delta & 0xFF
            b.ins("JMP", "abs", "LOOP")
    return A.program(body, fill=0xEA)


@pytest.mark.parametrize("delta,alpha_star", [(127, math.log(253)), (-128, math.log(255))])
def test_branch_casts_exactly_above_the_threshold(delta, alpha_star):
    """The rounded relaxed counter reaches the target iff |delta| < (1 + e^alpha) / 2,
    i.e. alpha > ln(2|delta| - 1); the same bound holds for the untaken branch."""
    ram0 = np.zeros(128, np.uint8)
    for taken in (True, False):
        if delta < 0 and not taken:
            continue
        img = _branch_program(delta, taken)
        for alpha, exact in ((alpha_star - 0.005, False), (alpha_star + 0.005, True), (6.0, True), (20.0, True)):
            m = O.Machine(img, 1, ram0)
            m.set_relax(alpha, 0.02)
            for _ in range(12):
                m.step()
            nd = m.relax_ndiv()
            if exact:
                assert nd == -1, (delta, taken, alpha, nd)
            else:
                idx = 3 if delta > 0 else 4
                assert nd == idx, (delta, taken, alpha, nd)


def _read_program(cell: int):
    # LDA zp, then a loop: the step's ROM fetches ($A5, $C0 next to $4C) stay exact up to T ~ 0.17
    def body(b):
        b.ins("LDA", "zp", 0x80 + cell)
        b.label("L")
        b.ins("JMP", "abs", "L")
    return A.program(body, fill=0xEA)


def _read(ram, cell, T):
    m = O.Machine(_read_program(cell), 1, ram)
    m.set_relax(20.0, T)
    m.step()
    return m.regs()["A"], m.relax_ndiv()


def test_read_casts_and_the_temperature_threshold():
    # every other cell at 255, the read cell at 0: the worst-case pull
    ram = np.full(128, 255, np.uint8)
    ram[64] = 0
    assert _read(ram, 64, 0.14) == (0, -1)
    assert _read(ram, 64, 0.1443) == (0, -1)
    assert _read(ram, 64, 0.1445) == (1, 0)
    assert _read(ram, 64, 0.16) == (1, 0)   # pulled by 255 (1 - w0) = 0.98
    # one max-amplitude neighbour pulls by 255 w_1: 0.49 at T = 0.160, 0.53 at T = 0.162
    ram = np.zeros(128, np.uint8)
    ram[65] = 255
    assert _read(ram, 64, 0.160) == (0, -1)
    assert _read(ram, 64, 0.162) == (1, 0)
    assert _read(ram, 64, 0.14) == (0, -1)
    # the array's edge cell has neighbours on one side only: 255 S/(1 + S), S = sum_k e^{-k/T}
    ram = np.full(128, 255, np.uint8)
    ram[127] = 0
    for T, want in ((0.14, 0), (0.16, 0), (0.163, 1)):
        m = O.Machine(A.program(lambda b: (b.ins("LDX", "imm", 0x7F), b.ins("LDA", "zpx", 0x80), b.label("L"),
                                           b.ins("JMP", "abs", "L")), fill=0xEA), 1, ram)
        m.set_relax(20.0, T)
        m.step()
        m.step()
        assert (m.regs()["A"], m.relax_ndiv()) == (want, -1 if want == 0 else 1), T


@pytest.mark.parametrize("seed,size,inputs", [(1, 4096, False), (101, 2048, True), (103, 8192, True),
                                              (104, 4096, True)])
def test_operating_point_is_exact_on_generated_roms(seed, size, inputs):
    """alpha = 6, T = 0.14 is bit-exact whatever the program (the bounds depend only
    on the instruction set and the byte range); T = 0.2 is not."""
    rom = I.generate_rom(seed, size, reads_inputs=inputs, timer_vblank=inputs)
    ram0 = I.initial_ram(seed, 1)[0]
    acts = I.action_stream(seed, 1, 3)[0]
    hard = O.run_env(rom.image, rom.mapper, ram0, acts, 3, 2)
    for alpha, T in ((6.0, 0.14), (6.0, 0.10), (20.0, 0.12)):
        r = O.run_relaxed(rom.image, rom.mapper, ram0, acts, 3, 2, alpha, T)
        assert r["ndiv"] == -1 and r["fails"] == 0
        assert (r["ram"] == hard["ram"]).all() and (r["frames"] == hard["frames"]).all()
    assert O.run_relaxed(rom.image, rom.mapper, ram0, acts, 3, 2, 6.0, 0.2)["ndiv"] >= 0


def test_first_divergence_grows_with_alpha():
    """Every cast that fails at alpha also fails at a smaller alpha, and the runs agree
    up to their first failure, so N_div is non-decreasing in alpha."""
    for seed in (1, 2, 5):
        rom = I.generate_rom(seed, 4096)
        ram0 = I.initial_ram(seed, 1)[0]
        prev = -1
        for alpha in (0.5, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0):
            nd = O.run_relaxed(rom.image, rom.mapper, ram0, None, 2, 1, alpha, 0.14)["ndiv"]
            n = math.inf if nd < 0 else nd
            assert n >= prev, (seed, alpha, nd, prev)
            prev = n


def test_one_step_deviation_obeys_the_temperature_limit_bound():
    """Theorem "Temperature-limit bound", term by term, on states of a generated ROM:
    the float64 pre-cast deviation of the step's reads is at most rho * 255 * (1 - w0)
    <= rho * 510 e^{-1/T} / (1 - e^{-1/T}); the branch's at most 256 e^{-alpha}; and the
    relaxed dispatch over all 256 handlers deviates from the winner's output by at most
    (K - 1) e^{-Delta/T} times the handlers' spread, with w* >= 1 - (K - 1) e^{-Delta/T}."""
    rom = I.generate_rom(104, 4096, reads_inputs=True, timer_vblank=True)
    ram0 = I.initial_ram(104, 1)[0]
    rng = np.random.default_rng(0)
    # settings inside the exact region: the trajectory is the hard one, the pre-cast deviations are not 0
    for alpha, T in ((6.0, 0.14), (5.6, 0.12), (20.0, 0.08)):
        m = O.Machine(rom.image, rom.mapper, ram0)
        m.set_relax(alpha, T, track=True)
        e = math.exp(-1 / T)
        reads = branches = 0
        for i in range(600):
            m.step()
            dr, nr, db = m.relax_last_dev()
            assert dr <= nr * 510 * e / (1 - e) + 1e-9, (i, dr, nr)
            assert db <= 256 * math.exp(-alpha) + 1e-9, (i, db)
            reads += nr
            branches += db > 0
        assert reads > 900 and branches > 10 and m.relax_ndiv() == -1
    # dispatch: logits = scaled one-hot of the opcode byte + N(0, 0.1^2)
    m = O.Machine(rom.image, rom.mapper, ram0)
    for i in range(40):
        m.step()
        if i % 8:
            continue
        pc = m.regs()["PCL"] | (m.regs()["PCH"] << 8)
        op = int(rom.image[pc & 0xFFF])
        for gap, T in ((1.0, 0.05), (3.0, 0.3), (1.0, 0.5)):
            lg = rng.normal(0, 0.1, 256)
            lg[op] += gap
            delta = lg[op] - np.max(np.delete(lg, op))
            dev, spread, ws = m.dispatch_deviation(lg, T)
            bound = 255 * math.exp(-delta / T)
            assert 1 - ws <= bound * (1 + 1e-12)
            assert dev <= bound * spread * (1 + 1e-9) + 1e-12, (i, gap, T, dev, bound, spread)
    # and the deviations vanish as T -> 0, alpha -> infinity
    devs = []
    for alpha, T in ((6.0, 0.14), (8.0, 0.1), (12.0, 0.06)):
        m = O.Machine(rom.image, rom.mapper, ram0)
        m.set_relax(alpha, T, track=True)
        tot_r = tot_b = 0.0
        for _ in range(600):
            m.step()
            dr, _, db = m.relax_last_dev()
            tot_r += dr
            tot_b += db
        devs.append((tot_r, tot_b))
    assert devs[0][0] > devs[1][0] > devs[2][0] > 0 and devs[0][1] > devs[1][1] > devs[2][1] > 0
