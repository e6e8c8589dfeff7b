"""Hand-assembled test programs (uses the input generator's encoder only)."""
import numpy as np

from paper_2606_22447_amd import inputs as I

VSYNC, VBLANK, WSYNC = 0x00, 0x01, 0x02
COLUP0, COLUP1, COLUPF, COLUBK, CTRLPF = 0x06, 0x07, 0x08, 0x09, 0x0A
PF0, PF1, PF2 = 0x0D, 0x0E, 0x0F
INPT4, SWCHA, SWCHB, INTIM, TIMINT = 0x0C, 0x280, 0x282, 0x284, 0x285
TIM1T, TIM8T, TIM64T, T1024T = 0x294, 0x295, 0x296, 0x297
JAM_OPCODE = 0x02
# TIA object registers (writes) and collision latches (reads)
NUSIZ0, NUSIZ1, REFP0, REFP1 = 0x04, 0x05, 0x0B, 0x0C
RESP0, RESP1, RESM0, RESM1, RESBL = 0x10, 0x11, 0x12, 0x13, 0x14
GRP0, GRP1, ENAM0, ENAM1, ENABL = 0x1B, 0x1C, 0x1D, 0x1E, 0x1F
HMP0, HMP1, HMM0, HMM1, HMBL = 0x20, 0x21, 0x22, 0x23, 0x24
VDELP0, VDELP1, VDELBL, RESMP0, RESMP1 = 0x25, 0x26, 0x27, 0x28, 0x29
HMOVE, HMCLR, CXCLR = 0x2A, 0x2B, 0x2C
CXM0P, CXM1P, CXP0FB, CXP1FB, CXM0FB, CXM1FB, CXBLPF, CXPPMM = range(8)


def program(body, size: int = 4096, fill: int = JAM_OPCODE, brk_handler=None) -> np.ndarray:
    """Assemble ``body(bank)`` at the start of a 4K (or 2K) image, reset vector -> start."""
    base = 0xF000 if size == 4096 else 0xF800
    b = I.Bank(size, base, bytes([fill]) * size)
    b.at(0)
    b.label("START")
    body(b)
    if brk_handler is not None:
        b.label("BRKH")
        brk_handler(b)
    b.at(size - 4)
    brk = b.labels.get("BRKH", base)
    b.byte(base & 0xFF, base >> 8, brk & 0xFF, brk >> 8)
    b.link()
    return np.frombuffer(bytes(b.img), dtype=np.uint8).copy()


def raw_image(size: int, writes: dict, fill: int = JAM_OPCODE) -> np.ndarray:
    img = np.full(size, fill, np.uint8)
    for off, bs in writes.items():
        img[off:off + len(bs)] = bs
    return img
