"""Pins of the oracle's further cartridge formats and console switch (the
paper's ports implement F8, F6, F4, their Superchip variants and E0; Sec.
"Building Two Differentiable VCS Ports"; the boot sequence of Table s-params
holds the console RESET switch).  Hand-assembled images whose final RAM and
bank registers follow from the documented hotspot maps by hand:

F8 $1FF8-9, F6 $1FF6-9, F4 $1FF4-B select a 4 KB bank on a data access (read
or write); E0 $1FE0-7 / $1FE8-F / $1FF0-7 select the 1 KB slice of the first
three quarters of the window (the last quarter is slice 7); Superchip RAM is
written at $1000-$107F and read at $1080-$10FF; SWCHB bit 0 is low while RESET
is held.  Behaviour of real cartridges is parity unpinned (no hardware or
reference emulator here)."""
import numpy as np
import pytest

from oracle import oracle as O

JAM = 0x02
RESET_VEC = [0x00, 0xF0]  # $F000


def run_to_jam(img, mapper, ram0=None, limit=2000, sc=None, action=None):
    m = O.Machine(img, mapper, ram0)
    if sc is not None:
        m.set_sc_ram(sc)
    if action is not None:
        m.set_action(action)
    for _ in range(limit):
        if m.step():
            break
    return m


def banked(nbanks, code_by_bank, vec_bank=None):
    """A 4K-banked image: code_by_bank[b] = {offset: bytes}; every bank's reset vector -> $F000."""
    img = np.full(4096 * nbanks, JAM, np.uint8)
    for b, writes in code_by_bank.items():
        for off, bs in writes.items():
            img[4096 * b + off:4096 * b + off + len(bs)] = bs
    for b in range(nbanks):
        img[4096 * b + 0xFFC:4096 * b + 0xFFE] = RESET_VEC
    return img


@pytest.mark.parametrize("mapper,nbanks,first", [(O.MAPPER_F6, 4, 0x1FF6), (O.MAPPER_F4, 8, 0x1FF4)])
def test_bank_switch_walks_every_bank(mapper, nbanks, first):
    """Starting in bank 0, the code at $F000+7k of bank k stores k*16+1 to RAM $80+k,
    then reads the hotspot of bank k+1 (execution continues at $F000+7(k+1) of bank k+1)."""
    code = {}
    for k in range(nbanks):
        c = {}
        pos = 7 * k
        nxt = first + (k + 1) % nbanks
        prog = [0xA9, (16 * k + 1) & 0xFF, 0x85, 0x80 + k]            # LDA #v ; STA $80+k
        if k + 1 < nbanks:
            prog += [0xAD, nxt & 0xFF, nxt >> 8]                      # LDA hotspot of bank k+1 (abs)
        c[pos] = prog
        c[0xFF0] = [0x40 + k]                                         # a marker byte at $FFF0 of every bank
        code[k] = c
    img = banked(nbanks, code)
    m = run_to_jam(img, mapper)
    ram = m.ram()
    for k in range(nbanks):
        assert ram[k] == (16 * k + 1) & 0xFF, (k, ram[:nbanks])
    assert m.regs()["bank"] == nbanks - 1


def test_hotspot_write_switches_and_reads_see_the_new_bank():
    """F4: STA $1FF6 (a write access) selects bank 2; LDA $FFF0 then reads bank 2's marker."""
    img = banked(8, {0: {0x000: [0x8D, 0xF6, 0x1F]},                  # STA $1FF6 -> bank 2
                     2: {0x003: [0xAD, 0xF0, 0xFF, 0x85, 0x80],       # LDA $FFF0 ; STA $80
                         0xFF0: [0x77]}})
    m = run_to_jam(img, O.MAPPER_F4)
    assert m.ram()[0] == 0x77 and m.regs()["bank"] == 2


def test_power_on_banks():
    """F8/F8SC start in bank 1, F6/F4 and their Superchip variants in bank 0."""
    for mapper, nb, bank in ((O.MAPPER_F8, 2, 1), (O.MAPPER_F8SC, 2, 1), (O.MAPPER_F6, 4, 0),
                             (O.MAPPER_F6SC, 4, 0), (O.MAPPER_F4, 8, 0), (O.MAPPER_F4SC, 8, 0)):
        img = banked(nb, {})
        assert O.Machine(img, mapper).regs()["bank"] == bank, mapper


def test_superchip_ram_write_and_read_ports():
    """F8SC: STA $1005 writes SC cell 5, LDA $1085 reads it back; a read of the write
    port returns the ROM byte; SC reads see the seeded contents."""
    sc0 = np.arange(128, dtype=np.uint8) ^ 0x5A
    code = {1: {0x100: [0xA9, 0x3D, 0x8D, 0x05, 0x10,     # LDA #$3D ; STA $1005
                        0xAD, 0x85, 0x10, 0x85, 0x80,     # LDA $1085 ; STA $80
                        0xAD, 0x86, 0x10, 0x85, 0x81,     # LDA $1086 ; STA $81 (seeded cell 6)
                        0xAD, 0x07, 0x10, 0x85, 0x82],    # LDA $1007 ; STA $82 (write port: ROM byte)
                0x007: [0xC4]}}
    img = banked(2, code)
    img[4096 + 0xFFC:4096 + 0xFFE] = [0x00, 0xF1]  # bank 1 resets to $F100
    m = run_to_jam(img, O.MAPPER_F8SC, sc=sc0)
    ram = m.ram()
    assert ram[0] == 0x3D and ram[1] == sc0[6] and ram[2] == 0xC4
    assert m.sc_ram()[5] == 0x3D
    # without Superchip RAM the same image reads ROM at $1085
    img[4096 + 0x085] = 0x99
    m = run_to_jam(img, O.MAPPER_F8)
    assert m.ram()[0] == 0x99


def test_e0_slices():
    """E0: code runs in the fixed last quarter (slice 7, $1C00-$1FFF); LDA $1FE3 maps
    slice 3 at $1000, LDA $1FEA slice 2 at $1400, STA $1FF5 slice 5 at $1800; power-on
    maps slices 4, 5, 6."""
    img = np.full(8192, JAM, np.uint8)
    for sl in range(8):
        img[1024 * sl + 0x000] = 0x10 + sl      # first byte of every slice
    code = [0xAD, 0x00, 0x10, 0x85, 0x80,       # LDA $1000 (power-on: slice 4) ; STA $80
            0xAD, 0xE3, 0x1F,                   # LDA $1FE3: segment 0 <- slice 3
            0xAD, 0x00, 0x10, 0x85, 0x81,       # LDA $1000 ; STA $81
            0xAD, 0xEA, 0x1F,                   # LDA $1FEA: segment 1 <- slice 2
            0xAD, 0x00, 0x14, 0x85, 0x82,       # LDA $1400 ; STA $82
            0x8D, 0xF5, 0x1F,                   # STA $1FF5: segment 2 <- slice 5
            0xAD, 0x00, 0x18, 0x85, 0x83,       # LDA $1800 ; STA $83
            0xAD, 0x00, 0x1C, 0x85, 0x84]       # LDA $1C00 (slice 7) ; STA $84
    base = 7 * 1024 + 0x100                     # $1D00 in the fixed slice
    img[base:base + len(code)] = code
    img[7 * 1024 + 0x3FC:7 * 1024 + 0x3FE] = [0x00, 0xFD]  # reset vector -> $FD00
    m = run_to_jam(img, O.MAPPER_E0)
    assert list(m.ram()[:5]) == [0x14, 0x13, 0x12, 0x15, 0x17]


def test_console_reset_switch_reads_in_swchb():
    """LDA SWCHB reads $0B normally and $0A while the RESET switch is held."""
    img = banked(1, {0: {0x000: [0xAD, 0x82, 0x02, 0x85, 0x80]}})
    assert run_to_jam(img, O.MAPPER_4K).ram()[0] == 0x0B
    assert run_to_jam(img, O.MAPPER_4K, action=O.ACTION_RESET).ram()[0] == 0x0A
    assert run_to_jam(img, O.MAPPER_4K, action=3).ram()[0] == 0x0B  # joystick RIGHT: switches untouched


def test_superchip_ram_is_seeded_per_env_and_episode():
    """run_env starts each episode's Superchip RAM from its own SplitMix64 stream."""
    a, b = O.splitmix_sc_ram(7, 0, 0), O.splitmix_sc_ram(7, 1, 0)
    assert not (a == b).all() and not (a == O.splitmix_ram(7, 0, 0)).all()
    assert (O.splitmix_sc_ram(7, 0, 0) == a).all()


def test_sizes_are_checked():
    for mapper, size in O.MAPPER_SIZE.items():
        O.Machine(np.full(size, JAM, np.uint8), mapper)
        with pytest.raises(ValueError):
            O.Machine(np.full(size * 2, JAM, np.uint8), mapper)
