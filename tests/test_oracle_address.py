"""Pins of the oracle's address surrogate (the leaky distance-softmax read of
Eq. s-read taken in the backward): an indexed read passes gradient to its index
register with the slope of the relaxed read at the hard address.

Independent checks: the closed form of that slope on a linear table (the
mean distance of the discrete Laplace window), zero on a symmetric table,
central finite differences of Eq. s-read evaluated directly, the T -> 0 limit,
and the structural zero with the surrogate off."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import asm as A

N_PIX = 210 * 160
TABLE = 0xF800  # a page of the 4K image: offset 0x800


def program(index_reg="X", mode="aby", idx=5, table=None):
    """LD? #idx ; LDA TABLE,? ; STA COLUBK ; jam.  The operand byte of the index
    load is image offset 1, the table at offset 0x800."""
    def body(b):
        if index_reg == "X":
            b.ins("LDX", "imm", idx)
            b.ins("LDA", "abx", TABLE)
        else:
            b.ins("LDY", "imm", idx)
            b.ins("LDA", mode, TABLE if mode == "aby" else 0x80)
        b.ins("STA", "zp", A.COLUBK)
        b.byte(A.JAM_OPCODE)
    img = A.program(body)
    if table is not None:
        img[0x800:0x800 + len(table)] = table
    return img


def soft(img, read_T, ram0=None, grad=None):
    ram0 = np.zeros(128, np.uint8) if ram0 is None else ram0
    sw, ip = O.action_ports(0)
    gf = np.ones((210, 160)) if grad is None else grad
    return O.soft_env(img, img.astype(np.float64), 1, ram0, ram0.astype(np.float64), np.zeros(1, np.uint8),
                      np.array([sw], np.float64), np.array([ip], np.float64), 1, 1, grad_frame=gf, read_T=read_T)


def laplace_mean_distance(T, K=8):
    """E|k| under weights exp(-|k|/T), k = -K..K."""
    e = [math.exp(-k / T) for k in range(1, K + 1)]
    return 2 * sum(k * x for k, x in zip(range(1, K + 1), e)) / (1 + 2 * sum(e))


@pytest.mark.parametrize("T", [1.0, 0.5, 2.0])
@pytest.mark.parametrize("reg", ["X", "Y"])
def test_linear_table_closed_form(T, reg):
    # TABLE[j] = 2j: the read value's slope in the address is 2 E|k| / T; every
    # visible pixel is COLUBK, so dL/dvalue = 33,600 and the index immediate
    # (offset 1) gets 33,600 * slope
    ramp = (2 * np.arange(64)).astype(np.uint8)
    r = soft(program(reg, table=ramp, idx=20), T)
    assert r["frame"][0, 0] == 40
    assert r["g_rom"][0x800 + 20] == pytest.approx(N_PIX, rel=1e-12)   # the content path
    assert r["g_rom"][1] == pytest.approx(N_PIX * 2 * laplace_mean_distance(T) / T, rel=1e-10)


def test_symmetric_table_has_zero_slope():
    t = np.zeros(64, np.uint8)
    for k in range(9):
        t[20 + k] = t[20 - k] = 10 + 7 * k
    r = soft(program("X", table=t, idx=20), 1.0)
    assert abs(r["g_rom"][1]) < 1e-9 * N_PIX  # zero up to rounding of the weighted sum
    assert r["g_rom"][0x800 + 20] == pytest.approx(N_PIX)


def eq_s_read(M, x, T, K=8):
    """Eq. s-read at a continuous address x: softmax(-|j - x| / T) blend of M over |j - round(x)| <= K."""
    c = int(round(x))
    j = np.arange(max(0, c - K), min(len(M), c + K + 1))
    w = np.exp(-np.abs(j - x) / T)
    return float((w * M[j]).sum() / w.sum())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_slope_matches_central_differences_of_eq_s_read(seed):
    rng = np.random.default_rng(seed)
    tab = rng.integers(0, 256, 64).astype(np.uint8)
    T, a, h = 0.5, 30, 1e-4
    M = tab.astype(float)
    d = lambda h: (eq_s_read(M, a + h, T) - eq_s_read(M, a - h, T)) / (2 * h)  # noqa: E731
    fd = 2 * d(h / 2) - d(h)  # Richardson: the |x - a| kink of the normaliser leaves an O(h) term in d(h)
    r = soft(program("X", table=tab, idx=a), T)
    assert r["g_rom"][1] / N_PIX == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_ram_indexed_read_and_pointer_form():
    # LDA ($80),Y with the pointer at $80/$81 -> TABLE and Y = 20: the window
    # (offsets 12..28 of the table) lies on the ramp
    ramp = (3 * np.arange(64)).astype(np.uint8)
    ram0 = np.zeros(128, np.uint8)
    ram0[0], ram0[1] = TABLE & 0xFF, TABLE >> 8
    img = program("Y", mode="izy", table=ramp, idx=20)
    r = soft(img, 1.0, ram0=ram0)
    assert r["frame"][0, 0] == 60
    assert r["g_rom"][1] == pytest.approx(N_PIX * 3 * laplace_mean_distance(1.0), rel=1e-10)

    # zero-page indexed into RAM: LDX #4 ; LDA $90,X with RAM $90.. a ramp of step 5
    def body(b):
        b.ins("LDX", "imm", 4)
        b.ins("LDA", "zpx", 0x90)
        b.ins("STA", "zp", A.COLUBK)
        b.byte(A.JAM_OPCODE)
    img = A.program(body)
    ram0 = ((5 * np.arange(128)) % 256).astype(np.uint8)  # linear over the cells the window reaches
    r = soft(img, 1.0, ram0=ram0)
    assert r["g_rom"][1] == pytest.approx(N_PIX * 5 * laplace_mean_distance(1.0), rel=1e-10)
    assert r["g_ram0"][0x14] == pytest.approx(N_PIX, rel=1e-12)  # the content path into the RAM cell


def test_cold_limit_and_off_switch():
    ramp = (2 * np.arange(64)).astype(np.uint8)
    img = program("X", table=ramp, idx=20)
    assert abs(soft(img, 0.04)["g_rom"][1]) < 1e-6 * N_PIX    # degenerate gradient as T -> 0
    assert soft(img, 0.0)["g_rom"][1] == 0.0                    # surrogate off: addresses carry none
