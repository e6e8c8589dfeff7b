/*
 * Reference emulator ("the oracle") for the batched Atari VCS hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded CPU
 * implementation of what the GPU library computes.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg load it.  It shares no code,
 * header, table or constant with the GPU library; both sides consume the same
 * seeded input arrays and nothing else.
 *
 * What it follows (the paper is "A Differentiable Atari VCS"):
 *  - the machine: a 6507 CPU running a cartridge ROM, a TIA that turns register
 *    writes into pixels colour clock by colour clock, and a RIOT holding 128 B of
 *    RAM, an interval timer and the input ports (Sec. "Why the Atari VCS Is Good
 *    Ground Truth"; Sec. "Building Two Differentiable VCS Ports" for the opcode
 *    set of 151 documented + USBC + 37 illegal bytes and the 2K/4K/F8 mappers);
 *  - HARD mode: integer dispatch, integer ALU, flags as bits (Sec. "Hard and Soft
 *    Execution");
 *  - SOFT-STE mode: memory reads as one-hot dot products (Eq. peek / s-peek),
 *    discrete choices in saturated softmax form (Eq. select / s-select), branches
 *    through the sigmoid gate (Eq. branch / s-branch), all joined by the
 *    straight-through estimator (Eq. ste / s-ste); forward = hard (Theorem
 *    "Exact forward equivalence"), backward = the surrogate of the chosen
 *    relaxation (Corollary following Theorem "Temperature-limit bound"), with the
 *    "stored switch" rule routing every gradient to the selected value.
 *
 * Where the paper defers to its reference emulator (absent here), the readings
 * below are fixed once and used everywhere:
 *  R1 frames are cycle-framed: frame f covers CPU cycles [f*19912,(f+1)*19912);
 *     beam line / colour clock are (cycle mod 19912) / 76 and 3*(cycle mod 76).
 *     An env step of F frames ends at the first instruction boundary at or after
 *     its budget; the overshoot carries into the next step.
 *  R2 visible window: lines [ystart, ystart+210), colour clocks 68..227.
 *  R3 pixel = palette index = owning colour register & 0xFE; 0 while VBLANK bit 1.
 *  R4 a TIA write in CPU cycle n takes effect at colour clock 3n+3.
 *  R5 loads and stores access memory on an instruction's last cycle; a
 *     read-modify-write reads 3 cycles and writes 1 cycle before its end (the
 *     dummy write in between has no side effect); pushes of JSR/BRK/PHA/PHP take
 *     effect on the last cycle in push order.  F8 hotspots fire on data accesses
 *     (not on opcode/operand fetches); a hotspot read returns the byte of the
 *     newly selected bank.
 *  R6 WSYNC: the CPU resumes at cycle 0 of the line after the write cycle.
 *  R7 undriven TIA read bits read 0; INPT4 bit 7 = fire not pressed; INPT5 = 0x80.
 *  R8 SWCHA = 0xFF with P0 right/left/down/up (bits 7/6/5/4) cleared when held;
 *     SWCHB = 0x0B; the 18 actions in the standard ALE order.
 *  R9 RIOT timer: a write of V to TIM1T/TIM8T/TIM64T/T1024T (interval I) at
 *     cycle c gives, for t > c and k = t - c - 1, INTIM = V-1-floor(k/I) while
 *     k < V*I and (255 - (k - V*I)) & 255 afterwards; TIMINT bit 7 is set from
 *     the underflow (k = V*I) until an INTIM read; power-on is V=0, I=1024, flag
 *     clear.
 *  R10 the 67 opcode bytes outside the paper's set JAM the CPU: it stops, cycles
 *     still elapse and the TIA keeps drawing.
 *  R11 decimal ADC/SBC: NMOS sequences of B. Clark's "Decimal Mode" tutorial
 *     (Appendix A): ADC takes N and V from the signed intermediate after the
 *     low-nibble fix, Z from the binary sum and C from the adjusted sum; SBC
 *     takes all flags from the binary subtraction.
 *  R12 JMP ($xxFF) wraps within the page; zero-page indexing wraps; BRK pushes
 *     PC+2 and P|0x30; the stack page maps through the 13-bit decode.
 *
 * The TIA's movable objects (Sec. "Hard and Soft Execution": object priority,
 * sprite bits and the strobe-timed sprite column; Sec. "Discussion": sub-cycle
 * object rendering), read from the documented TIA as follows:
 *  R15 objects P0, P1, M0, M1, BL each have a column pos in [0, 160), the
 *      visible column of its first pixel, 0 at power-on.  A strobe (RESP0/1,
 *      RESM0/1, RESBL) whose effect clock (R4) lies at clock h of its line sets
 *      pos = (h - 68 + 5) mod 160 for a player and (h - 68 + 4) mod 160 for a
 *      missile or the ball, or 3 / 2 when h < 68 (horizontal blank).
 *  R16 shapes: NUSIZ bits 0-2 give a player's copies at column offsets
 *      {0} {0,16} {0,32} {0,16,32} {0,64} {0} {0,32,64} {0} and its pixel width
 *      1, except 2 (mode 5) and 4 (mode 7); the graphics byte shows bit 7 first,
 *      bit 0 first when REFP bit 3 is set.  A missile has its player's copies,
 *      width 2^(NUSIZ bits 4-5), and shows while ENAM bit 1 is set and RESMP bit
 *      1 is clear; clearing RESMP moves it to its player's column + 4 * width.
 *      The ball is one copy of width 2^(CTRLPF bits 4-5), shown while ENABL bit
 *      1 is set.  Vertical delay: a GRP0 write copies GRP1 into GRP1's old
 *      register; a GRP1 write copies GRP0 and ENABL into their old registers;
 *      VDELP0/1 and VDELBL bit 0 select the old register for display.
 *  R17 HMOVE moves every object left by its motion register's signed high
 *      nibble (pos - m mod 160); HMCLR zeroes the five motion registers.  An
 *      HMOVE whose effect clock lies in horizontal blank blanks columns 0..7 of
 *      its line: black, and no collisions there.
 *  R18 priority: with CTRLPF bit 2 clear, P0/M0 (COLUP0) over P1/M1 (COLUP1)
 *      over the playfield and ball over the background; with it set, the
 *      playfield and ball come first.  Score mode colours the playfield's left
 *      half COLUP0 and right half COLUP1; the ball is always COLUPF.
 *  R19 collisions latch wherever two objects, or an object and the
 *      playfield, show at one visible column of any line (VBLANK does not mask
 *      them); CXCLR clears them; a read in cycle t sees the clocks before
 *      3t + 3.  Register r = 0..7 (CXM0P, CXM1P, CXP0FB, CXP1FB, CXM0FB, CXM1FB,
 *      CXBLPF, CXPPMM) reads pair 2r in bit 7 and pair 2r+1 in bit 6, pairs
 *      M0-P1, M0-P0, M1-P0, M1-P1, P0-PF, P0-BL, P1-PF, P1-BL, M0-PF, M0-BL,
 *      M1-PF, M1-BL, BL-PF, (none), P0-P1, M0-M1.
 *  R20 position sampler (soft): the derivative of the returned frame with
 *      respect to an object's column is that of a triangular (bilinear)
 *      sampler at zero sub-pixel offset taken from the right: at every visible
 *      pixel, the colour with the object drawn one column further right minus
 *      the colour drawn; blanked pixels contribute nothing.  A shift moves the
 *      object in every span of the frame.
 *  R21 address surrogate (soft, off unless a read temperature T > 0 is given):
 *      the leaky variant's distance-softmax read (Eq. s-read) taken in the
 *      backward, so that an indexed read of a ROM or RAM byte passes gradient to
 *      its index register (X for zp,X and abs,X; Y for zp,Y, abs,Y and (zp),Y);
 *      the slope is Eq. s-read's at the hard address (see address_node).  The
 *      paper's other leaky pieces, gradients through branch gates and flags into
 *      data, need the untaken path's outcome, which a single hard trajectory
 *      does not have: they are not built.
 *
 * Soft surrogate (reverse sweep) rules, in the paper's "stored switch" reading:
 *  leaves: ROM byte = STE(sum_k k softmax(L_a/tau)_k, argmax_k L_a); RAM0 cell =
 *  STE(sum_k k P0[c,k], argmax_k P0[c,k]); a port read during step s =
 *  STE(E_softmax(l_s/tau)[port(a)], port(argmax l_s)).  Moves d=1; ADC/SBC d=1
 *  and +/-1; INC/DEC d=1; ASL/ROL d=2, LSR/ROR d=1/2; AND/ORA/EOR/SAX use the
 *  bit-uniform multilinear extension (A&B ~ AB/255, A|B ~ A+B-AB/255,
 *  A^B ~ A+B-2AB/255); flags, compares, PC, S, addresses (unless R21),
 *  opcodes and timer values carry no gradient; a pixel's adjoint goes to the colour register that
 *  owned it.  STE evaluates coefficients at hard values; SMOOTH re-runs the same
 *  trajectory with real-valued leaves and evaluates them at the smooth values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "vcs_oracle.h"

/* ------------------------------------------------------------------------ */
/* Frame geometry (NTSC)                                                    */
/* ------------------------------------------------------------------------ */
enum {
    CYCLES_PER_LINE = 76,
    LINES_PER_FRAME = 262,
    CYCLES_PER_FRAME = CYCLES_PER_LINE * LINES_PER_FRAME, /* 19912 */
    CLOCKS_PER_LINE = 228,
    CLOCKS_PER_FRAME = CLOCKS_PER_LINE * LINES_PER_FRAME, /* 59736 */
    HBLANK_CLOCKS = 68,
    SCREEN_W = 160,
    SCREEN_H = 210
};

/* ------------------------------------------------------------------------ */
/* Opcode table: the paper's 189 bytes                                       */
/* ------------------------------------------------------------------------ */
enum Mode { IMP, ACC, IMM, ZP, ZPX, ZPY, ABS, ABX, ABY, IZX, IZY, IND, REL };
enum Op {
    JAM = 0, ADC, AND, ASL, BCC, BCS, BEQ, BIT, BMI, BNE, BPL, BRK, BVC, BVS, CLC, CLD, CLI, CLV,
    CMP, CPX, CPY, DEC, DEX, DEY, EOR, INC, INX, INY, JMP, JSR, LDA, LDX, LDY, LSR, NOP, ORA,
    PHA, PHP, PLA, PLP, ROL, ROR, RTI, RTS, SBC, SEC, SED, SEI, STA, STX, STY, TAX, TAY, TSX,
    TXA, TXS, TYA, LAX, SAX
};
static const int MODE_LEN[] = {1, 1, 2, 2, 2, 2, 3, 3, 3, 2, 2, 3, 2};

typedef struct { uint8_t code, op, mode, cycles, page_penalty; } OpRow;

/* Documented NMOS 6502 cycle counts; page_penalty = +1 cycle when the indexed
 * read crosses a page. */
static const OpRow OP_ROWS[] = {
    {0x69, ADC, IMM, 2, 0}, {0x65, ADC, ZP, 3, 0}, {0x75, ADC, ZPX, 4, 0}, {0x6D, ADC, ABS, 4, 0},
    {0x7D, ADC, ABX, 4, 1}, {0x79, ADC, ABY, 4, 1}, {0x61, ADC, IZX, 6, 0}, {0x71, ADC, IZY, 5, 1},
    {0x29, AND, IMM, 2, 0}, {0x25, AND, ZP, 3, 0}, {0x35, AND, ZPX, 4, 0}, {0x2D, AND, ABS, 4, 0},
    {0x3D, AND, ABX, 4, 1}, {0x39, AND, ABY, 4, 1}, {0x21, AND, IZX, 6, 0}, {0x31, AND, IZY, 5, 1},
    {0x0A, ASL, ACC, 2, 0}, {0x06, ASL, ZP, 5, 0}, {0x16, ASL, ZPX, 6, 0}, {0x0E, ASL, ABS, 6, 0},
    {0x1E, ASL, ABX, 7, 0},
    {0x90, BCC, REL, 2, 0}, {0xB0, BCS, REL, 2, 0}, {0xF0, BEQ, REL, 2, 0}, {0x30, BMI, REL, 2, 0},
    {0xD0, BNE, REL, 2, 0}, {0x10, BPL, REL, 2, 0}, {0x50, BVC, REL, 2, 0}, {0x70, BVS, REL, 2, 0},
    {0x24, BIT, ZP, 3, 0}, {0x2C, BIT, ABS, 4, 0},
    {0x00, BRK, IMP, 7, 0},
    {0x18, CLC, IMP, 2, 0}, {0xD8, CLD, IMP, 2, 0}, {0x58, CLI, IMP, 2, 0}, {0xB8, CLV, IMP, 2, 0},
    {0xC9, CMP, IMM, 2, 0}, {0xC5, CMP, ZP, 3, 0}, {0xD5, CMP, ZPX, 4, 0}, {0xCD, CMP, ABS, 4, 0},
    {0xDD, CMP, ABX, 4, 1}, {0xD9, CMP, ABY, 4, 1}, {0xC1, CMP, IZX, 6, 0}, {0xD1, CMP, IZY, 5, 1},
    {0xE0, CPX, IMM, 2, 0}, {0xE4, CPX, ZP, 3, 0}, {0xEC, CPX, ABS, 4, 0},
    {0xC0, CPY, IMM, 2, 0}, {0xC4, CPY, ZP, 3, 0}, {0xCC, CPY, ABS, 4, 0},
    {0xC6, DEC, ZP, 5, 0}, {0xD6, DEC, ZPX, 6, 0}, {0xCE, DEC, ABS, 6, 0}, {0xDE, DEC, ABX, 7, 0},
    {0xCA, DEX, IMP, 2, 0}, {0x88, DEY, IMP, 2, 0},
    {0x49, EOR, IMM, 2, 0}, {0x45, EOR, ZP, 3, 0}, {0x55, EOR, ZPX, 4, 0}, {0x4D, EOR, ABS, 4, 0},
    {0x5D, EOR, ABX, 4, 1}, {0x59, EOR, ABY, 4, 1}, {0x41, EOR, IZX, 6, 0}, {0x51, EOR, IZY, 5, 1},
    {0xE6, INC, ZP, 5, 0}, {0xF6, INC, ZPX, 6, 0}, {0xEE, INC, ABS, 6, 0}, {0xFE, INC, ABX, 7, 0},
    {0xE8, INX, IMP, 2, 0}, {0xC8, INY, IMP, 2, 0},
    {0x4C, JMP, ABS, 3, 0}, {0x6C, JMP, IND, 5, 0},
    {0x20, JSR, ABS, 6, 0},
    {0xA9, LDA, IMM, 2, 0}, {0xA5, LDA, ZP, 3, 0}, {0xB5, LDA, ZPX, 4, 0}, {0xAD, LDA, ABS, 4, 0},
    {0xBD, LDA, ABX, 4, 1}, {0xB9, LDA, ABY, 4, 1}, {0xA1, LDA, IZX, 6, 0}, {0xB1, LDA, IZY, 5, 1},
    {0xA2, LDX, IMM, 2, 0}, {0xA6, LDX, ZP, 3, 0}, {0xB6, LDX, ZPY, 4, 0}, {0xAE, LDX, ABS, 4, 0},
    {0xBE, LDX, ABY, 4, 1},
    {0xA0, LDY, IMM, 2, 0}, {0xA4, LDY, ZP, 3, 0}, {0xB4, LDY, ZPX, 4, 0}, {0xAC, LDY, ABS, 4, 0},
    {0xBC, LDY, ABX, 4, 1},
    {0x4A, LSR, ACC, 2, 0}, {0x46, LSR, ZP, 5, 0}, {0x56, LSR, ZPX, 6, 0}, {0x4E, LSR, ABS, 6, 0},
    {0x5E, LSR, ABX, 7, 0},
    {0xEA, NOP, IMP, 2, 0},
    {0x09, ORA, IMM, 2, 0}, {0x05, ORA, ZP, 3, 0}, {0x15, ORA, ZPX, 4, 0}, {0x0D, ORA, ABS, 4, 0},
    {0x1D, ORA, ABX, 4, 1}, {0x19, ORA, ABY, 4, 1}, {0x01, ORA, IZX, 6, 0}, {0x11, ORA, IZY, 5, 1},
    {0x48, PHA, IMP, 3, 0}, {0x08, PHP, IMP, 3, 0}, {0x68, PLA, IMP, 4, 0}, {0x28, PLP, IMP, 4, 0},
    {0x2A, ROL, ACC, 2, 0}, {0x26, ROL, ZP, 5, 0}, {0x36, ROL, ZPX, 6, 0}, {0x2E, ROL, ABS, 6, 0},
    {0x3E, ROL, ABX, 7, 0},
    {0x6A, ROR, ACC, 2, 0}, {0x66, ROR, ZP, 5, 0}, {0x76, ROR, ZPX, 6, 0}, {0x6E, ROR, ABS, 6, 0},
    {0x7E, ROR, ABX, 7, 0},
    {0x40, RTI, IMP, 6, 0}, {0x60, RTS, IMP, 6, 0},
    {0xE9, SBC, IMM, 2, 0}, {0xE5, SBC, ZP, 3, 0}, {0xF5, SBC, ZPX, 4, 0}, {0xED, SBC, ABS, 4, 0},
    {0xFD, SBC, ABX, 4, 1}, {0xF9, SBC, ABY, 4, 1}, {0xE1, SBC, IZX, 6, 0}, {0xF1, SBC, IZY, 5, 1},
    {0x38, SEC, IMP, 2, 0}, {0xF8, SED, IMP, 2, 0}, {0x78, SEI, IMP, 2, 0},
    {0x85, STA, ZP, 3, 0}, {0x95, STA, ZPX, 4, 0}, {0x8D, STA, ABS, 4, 0}, {0x9D, STA, ABX, 5, 0},
    {0x99, STA, ABY, 5, 0}, {0x81, STA, IZX, 6, 0}, {0x91, STA, IZY, 6, 0},
    {0x86, STX, ZP, 3, 0}, {0x96, STX, ZPY, 4, 0}, {0x8E, STX, ABS, 4, 0},
    {0x84, STY, ZP, 3, 0}, {0x94, STY, ZPX, 4, 0}, {0x8C, STY, ABS, 4, 0},
    {0xAA, TAX, IMP, 2, 0}, {0xA8, TAY, IMP, 2, 0}, {0xBA, TSX, IMP, 2, 0}, {0x8A, TXA, IMP, 2, 0},
    {0x9A, TXS, IMP, 2, 0}, {0x98, TYA, IMP, 2, 0},
    /* undocumented forms in the paper's set */
    {0xEB, SBC, IMM, 2, 0}, /* USBC */
    {0xA7, LAX, ZP, 3, 0}, {0xB7, LAX, ZPY, 4, 0}, {0xAF, LAX, ABS, 4, 0}, {0xBF, LAX, ABY, 4, 1},
    {0xA3, LAX, IZX, 6, 0}, {0xB3, LAX, IZY, 5, 1},
    {0x87, SAX, ZP, 3, 0}, {0x97, SAX, ZPY, 4, 0}, {0x8F, SAX, ABS, 4, 0}, {0x83, SAX, IZX, 6, 0},
    {0x1A, NOP, IMP, 2, 0}, {0x3A, NOP, IMP, 2, 0}, {0x5A, NOP, IMP, 2, 0}, {0x7A, NOP, IMP, 2, 0},
    {0xDA, NOP, IMP, 2, 0}, {0xFA, NOP, IMP, 2, 0},
    {0x80, NOP, IMM, 2, 0}, {0x82, NOP, IMM, 2, 0}, {0x89, NOP, IMM, 2, 0}, {0xC2, NOP, IMM, 2, 0},
    {0xE2, NOP, IMM, 2, 0},
    {0x04, NOP, ZP, 3, 0}, {0x44, NOP, ZP, 3, 0}, {0x64, NOP, ZP, 3, 0},
    {0x14, NOP, ZPX, 4, 0}, {0x34, NOP, ZPX, 4, 0}, {0x54, NOP, ZPX, 4, 0}, {0x74, NOP, ZPX, 4, 0},
    {0xD4, NOP, ZPX, 4, 0}, {0xF4, NOP, ZPX, 4, 0},
    {0x0C, NOP, ABS, 4, 0},
    {0x1C, NOP, ABX, 4, 1}, {0x3C, NOP, ABX, 4, 1}, {0x5C, NOP, ABX, 4, 1}, {0x7C, NOP, ABX, 4, 1},
    {0xDC, NOP, ABX, 4, 1}, {0xFC, NOP, ABX, 4, 1},
};

static OpRow OPS[256];
static int OPS_READY = 0;

static void ops_init(void) {
    if (OPS_READY) return;
    for (int i = 0; i < 256; i++) {
        OPS[i].code = (uint8_t)i;
        OPS[i].op = JAM;
        OPS[i].mode = IMP;
        OPS[i].cycles = 0;
        OPS[i].page_penalty = 0;
    }
    for (size_t i = 0; i < sizeof(OP_ROWS) / sizeof(OP_ROWS[0]); i++) OPS[OP_ROWS[i].code] = OP_ROWS[i];
    OPS_READY = 1;
}

int orc_opcode_info(int opcode, int *op, int *mode, int *cycles, int *page_penalty) {
    ops_init();
    OpRow r = OPS[opcode & 0xFF];
    *op = r.op;
    *mode = r.mode;
    *cycles = r.cycles;
    *page_penalty = r.page_penalty;
    return r.op != JAM;
}

/* ------------------------------------------------------------------------ */
/* Status flags                                                             */
/* ------------------------------------------------------------------------ */
enum { FC = 0x01, FZ = 0x02, FI = 0x04, FD = 0x08, FB = 0x10, FU = 0x20, FV = 0x40, FN = 0x80 };

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood 2014), counter mode                       */
/* ------------------------------------------------------------------------ */
static const uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;

static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void orc_splitmix_ram(uint64_t seed, uint64_t env, uint64_t episode, uint8_t *out) {
    uint64_t key = mix64(seed + (env + 1) * GOLDEN);
    key = mix64(key + (episode + 1) * GOLDEN);
    for (int i = 0; i < 128; i++) {
        uint64_t w = mix64(key + (uint64_t)(i / 8 + 1) * GOLDEN);
        out[i] = (uint8_t)(w >> (8 * (i % 8)));
    }
}

uint64_t orc_splitmix_next(uint64_t *state) {
    *state += GOLDEN;
    return mix64(*state);
}

/* ------------------------------------------------------------------------ */
/* Joystick actions (standard ALE enumeration)                               */
/* ------------------------------------------------------------------------ */
/* up, down, left, right, fire for actions 0..17:
 * NOOP FIRE UP RIGHT LEFT DOWN UPRIGHT UPLEFT DOWNRIGHT DOWNLEFT
 * UPFIRE RIGHTFIRE LEFTFIRE DOWNFIRE UPRIGHTFIRE UPLEFTFIRE DOWNRIGHTFIRE DOWNLEFTFIRE */
static const uint8_t ACTION_DIRS[18][5] = {
    {0, 0, 0, 0, 0}, {0, 0, 0, 0, 1}, {1, 0, 0, 0, 0}, {0, 0, 0, 1, 0}, {0, 0, 1, 0, 0},
    {0, 1, 0, 0, 0}, {1, 0, 0, 1, 0}, {1, 0, 1, 0, 0}, {0, 1, 0, 1, 0}, {0, 1, 1, 0, 0},
    {1, 0, 0, 0, 1}, {0, 0, 0, 1, 1}, {0, 0, 1, 0, 1}, {0, 1, 0, 0, 1}, {1, 0, 0, 1, 1},
    {1, 0, 1, 0, 1}, {0, 1, 0, 1, 1}, {0, 1, 1, 0, 1},
};

int orc_action_swcha(int action) {
    const uint8_t *d = ACTION_DIRS[action];
    int v = 0xFF;
    if (d[3]) v &= ~0x80; /* right */
    if (d[2]) v &= ~0x40; /* left */
    if (d[1]) v &= ~0x20; /* down */
    if (d[0]) v &= ~0x10; /* up */
    return v;
}

int orc_action_inpt4(int action) { return ACTION_DIRS[action][4] ? 0x00 : 0x80; }

/* ------------------------------------------------------------------------ */
/* Soft value graph (used only by soft runs)                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t p0, p1;   /* parent nodes (-1: none) */
    double ste0, ste1; /* coefficients at hard values */
    double sm0, sm1;   /* coefficients at smooth values */
    double vs;         /* smooth value */
    int32_t vh;        /* hard value */
} Node;

typedef struct Graph {
    Node *n;
    int64_t len, cap;
    int32_t slot_a, slot_x, slot_y, slot_ram[128], slot_col[4];
    /* leaves */
    int rom_size;
    const uint8_t *rom_hard;
    const double *rom_ev;
    int32_t *rom_leaf;      /* [rom_size], -2 = not yet created */
    int32_t ram0_leaf[128];
    int steps;
    int32_t *swcha_leaf, *inpt4_leaf; /* [steps] */
    const double *swcha_ev, *inpt4_ev;
    const uint8_t *act_hard;
    int32_t *pixel_node;    /* [210*160] */
    int32_t *ramout_node;   /* [steps*128] */
    int32_t *pos_delta;     /* [5][210*160]: colour with the object one column right minus the colour (R20) */
    double read_T;          /* R21: the read temperature of the address surrogate (0: off) */
} Graph;

static int32_t g_new(Graph *g, int32_t p0, double s0, double m0, int32_t p1, double s1, double m1,
                     double vs, int vh) {
    if (g->len == g->cap) {
        g->cap = g->cap ? g->cap * 2 : 4096;
        g->n = (Node *)realloc(g->n, (size_t)g->cap * sizeof(Node));
    }
    Node *x = &g->n[g->len];
    x->p0 = p0;
    x->p1 = p1;
    x->ste0 = s0;
    x->ste1 = s1;
    x->sm0 = m0;
    x->sm1 = m1;
    x->vs = vs;
    x->vh = vh;
    return (int32_t)g->len++;
}

/* smooth value of a slot whose hard value is h */
static double g_sv(const Graph *g, int32_t id, int h) { return id < 0 ? (double)h : g->n[id].vs; }

/* result = hard + sum_i k_i (smooth_i - hard_i) for constant coefficients (moves,
 * ADC/SBC, INC/DEC, shifts): STE and SMOOTH coefficients coincide. */
static int32_t g_affine(Graph *g, int32_t pa, double ka, int ha, int32_t pb, double kb, int hb, int vh) {
    if (pa < 0 && pb < 0) return -1;
    double vs = vh + ka * (g_sv(g, pa, ha) - ha) + kb * (g_sv(g, pb, hb) - hb);
    return g_new(g, pa, ka, ka, pb, kb, kb, vs, vh);
}

enum { LOGIC_AND, LOGIC_ORA, LOGIC_EOR };

/* bit-uniform multilinear extension of a bitwise op on bytes */
static double logic_ext(int kind, double a, double b) {
    switch (kind) {
        case LOGIC_AND: return a * b / 255.0;
        case LOGIC_ORA: return a + b - a * b / 255.0;
        default: return a + b - 2.0 * a * b / 255.0;
    }
}
/* partial derivative of the extension w.r.t. its first argument, other = b */
static double logic_d(int kind, double b) {
    switch (kind) {
        case LOGIC_AND: return b / 255.0;
        case LOGIC_ORA: return (255.0 - b) / 255.0;
        default: return (255.0 - 2.0 * b) / 255.0;
    }
}

static int32_t g_logic(Graph *g, int kind, int32_t pa, int ha, int32_t pb, int hb, int vh) {
    if (pa < 0 && pb < 0) return -1;
    double as = g_sv(g, pa, ha), bs = g_sv(g, pb, hb);
    double vs = vh + logic_ext(kind, as, bs) - logic_ext(kind, ha, hb);
    return g_new(g, pa, logic_d(kind, hb), logic_d(kind, bs), pb, logic_d(kind, ha), logic_d(kind, as), vs, vh);
}

/* ------------------------------------------------------------------------ */
/* FULL relaxed mode (Table s-modes): the sigmoid branch of Eq. s-branch and  */
/* the distance-softmax read of Eq. s-read WITHOUT the straight-through      */
/* correction, each result cast back to an integer (Sec. "Forward            */
/* Bit-Exactness Under Full Relaxation").  Dispatch stays saturated in the    */
/* rollouts: the cast-margin model of that section has branch and read casts  */
/* only; the relaxed dispatch of Eq. s-select is evaluated by the one-step    */
/* deviation function below (Theorem "Temperature-limit bound").             */
/* Precision: float32 as the paper's soft mode; weights e^{-|k|/T} are       */
/* formed in double and stored as float; reads blend the neighbours          */
/* |k| <= RELAX_WINDOW inside the memory array (ROM image or the 128 RAM      */
/* cells), normalised over those; casts round to nearest, ties to even.      */
/* ------------------------------------------------------------------------ */
enum { RELAX_WINDOW = 8 };
typedef struct {
    int on;
    float u[RELAX_WINDOW + 1];   /* u[k] = e^{-k/T} (u[0] = 1) */
    float g_taken, g_not;        /* sigma(alpha), sigma(-alpha): the gate for z = +1 / -1 */
    int64_t ndiv;                /* first instruction whose cast differed from the exact value (-1: none) */
    uint64_t fails;              /* casts that differed */
    double T, alpha;
    /* the last instruction's pre-cast deviations in float64, each read blended over
     * its whole memory array (Theorem "Temperature-limit bound"): the sum over its
     * reads, their number, and the branch's */
    double dev_read, dev_branch;
    int nread, track;
} Relax;

/* ------------------------------------------------------------------------ */
/* Machine                                                                  */
/* ------------------------------------------------------------------------ */
enum { OBJ_P0, OBJ_P1, OBJ_M0, OBJ_M1, OBJ_BL, NOBJ };
struct Orc {
    /* cartridge */
    uint8_t rom[32768];
    int rom_size, mapper, bank;
    int slice[4];         /* E0: the 1 KB slice mapped at each quarter of the cartridge window */
    uint8_t sc_ram[128];  /* Superchip RAM (F8SC, F6SC, F4SC) */
    /* 6507 */
    uint8_t a, x, y, s, p;
    uint16_t pc;
    int jammed;
    /* RIOT */
    uint8_t ram[128];
    int64_t tim_write; /* c: cycle of the last TIMnT write */
    int tim_value;     /* V */
    int tim_interval;  /* I */
    int64_t tim_read;  /* cycle of the last INTIM read */
    uint8_t swcha, inpt4, swchb;
    /* TIA */
    uint8_t vsync, vblank, colup0, colup1, colupf, colubk, ctrlpf, pf0, pf1, pf2;
    int wsync;
    /* TIA objects (R15-R19), indexed P0, P1, M0, M1, BL */
    int pos[NOBJ];
    uint8_t grp_new[2], grp_old[2], enabl_new, enabl_old, enam[2], nusiz[2], refp[2], vdelp[2], vdelbl, resmp[2];
    uint8_t hm[NOBJ];
    uint16_t cx;          /* collision latches, bit k = pair k of R19 */
    int64_t cx_done;      /* colour clocks since power-on whose collisions are latched */
    int64_t hmove_line;   /* line since power-on whose columns 0..7 an HMOVE blanked (-1: none) */
    /* time */
    int64_t cycle;      /* CPU cycles since power-on */
    int64_t drawn;      /* colour clocks since power-on already rendered */
    int64_t draw_frame; /* frame whose visible pixels are stored (-1: none) */
    int ystart;
    uint8_t frame[SCREEN_H * SCREEN_W];
    uint64_t instructions;
    /* executions per opcode byte; of them, indexed accesses that crossed a page
     * (or taken branches that crossed one), and taken branches */
    uint64_t op_count[256], op_cross[256], op_taken[256];
    /* soft */
    Graph *g;
    int step;
    /* FULL relaxed mode (kept across power-on) */
    Relax rx;
    int rx_active;     /* an instruction is executing: its reads and branch are relaxed */
};

Orc *orc_new(void) {
    ops_init();
    Orc *m = (Orc *)calloc(1, sizeof(Orc));
    return m;
}

void orc_free(Orc *m) { free(m); }

/* Cartridge formats beyond 2K/4K (Sec. "Building Two Differentiable VCS Ports":
 * F8, F6, F4, their Superchip variants, E0).  F8/F6/F4 switch the whole 4 KB
 * window among 2/4/8 banks on a data access to one of their hotspots
 * ($1FF8-9, $1FF6-9, $1FF4-B); E0 maps 1 KB slices into the window's
 * first three quarters on accesses to $1FE0-7, $1FE8-F, $1FF0-7 (the last
 * quarter is slice 7).  Superchip carts add 128 bytes of RAM written through
 * $1000-$107F and read through $1080-$10FF. */
static int mapper_banks(int mapper) {
    switch (mapper) {
        case ORC_MAPPER_F8: case ORC_MAPPER_F8SC: return 2;
        case ORC_MAPPER_F6: case ORC_MAPPER_F6SC: return 4;
        case ORC_MAPPER_F4: case ORC_MAPPER_F4SC: return 8;
        default: return 1;
    }
}
static int mapper_size(int mapper) {
    switch (mapper) {
        case ORC_MAPPER_2K: return 2048;
        case ORC_MAPPER_4K: return 4096;
        case ORC_MAPPER_E0: return 8192;
        default: return 4096 * mapper_banks(mapper);
    }
}
static int mapper_sc(int mapper) {
    return mapper == ORC_MAPPER_F8SC || mapper == ORC_MAPPER_F6SC || mapper == ORC_MAPPER_F4SC;
}

static int cart_offset(const Orc *m, uint16_t addr) {
    switch (m->mapper) {
        case ORC_MAPPER_2K: return addr & 0x7FF;
        case ORC_MAPPER_4K: return addr & 0xFFF;
        case ORC_MAPPER_E0: return m->slice[(addr >> 10) & 3] * 1024 + (addr & 0x3FF);
        default: return m->bank * 4096 + (addr & 0xFFF);
    }
}

/* ---- TIA ---------------------------------------------------------------- */

static int playfield_bit(const Orc *m, int x) {
    int i = x < 80 ? x / 4 : (x - 80) / 4; /* 20 playfield bits per half line */
    if (x >= 80 && (m->ctrlpf & 0x01)) i = 19 - i; /* reflected right half */
    if (i < 4) return (m->pf0 >> (4 + i)) & 1;
    if (i < 12) return (m->pf1 >> (11 - i)) & 1;
    return (m->pf2 >> (i - 12)) & 1;
}

/* ---- objects (R15-R19) ---- */
enum { OCC_P0 = 1, OCC_P1 = 2, OCC_M0 = 4, OCC_M1 = 8, OCC_BL = 16, OCC_PF = 32 };

/* column offsets of the copies of NUSIZ modes 0..7 (-1: no further copy) */
static const int COPIES[8][3] = {{0, -1, -1}, {0, 16, -1}, {0, 32, -1}, {0, 16, 32},
                                 {0, 64, -1}, {0, -1, -1}, {0, 32, 64}, {0, -1, -1}};

/* columns from an object's first pixel to column x, going right with wrap-around */
static int columns_from(int pos, int x) { return ((x - pos) % SCREEN_W + SCREEN_W) % SCREEN_W; }

static int player_pixel(const Orc *m, int i, int x) {
    const int mode = m->nusiz[i] & 7, scale = mode == 5 ? 2 : mode == 7 ? 4 : 1;
    const int gfx = (m->vdelp[i] & 1) ? m->grp_old[i] : m->grp_new[i];
    const int d = columns_from(m->pos[OBJ_P0 + i], x);
    for (int k = 0; k < 3 && COPIES[mode][k] >= 0; k++) {
        const int e = d - COPIES[mode][k];
        if (e >= 0 && e < 8 * scale) {
            const int b = e / scale; /* graphics bit, counted from the first pixel */
            return (m->refp[i] & 0x08) ? (gfx >> b) & 1 : (gfx >> (7 - b)) & 1;
        }
    }
    return 0;
}

static int missile_shown(const Orc *m, int i) { return (m->enam[i] & 2) && !(m->resmp[i] & 2); }

static int missile_pixel(const Orc *m, int i, int x) {
    if (!missile_shown(m, i)) return 0;
    const int mode = m->nusiz[i] & 7, width = 1 << ((m->nusiz[i] >> 4) & 3);
    const int d = columns_from(m->pos[OBJ_M0 + i], x);
    for (int k = 0; k < 3 && COPIES[mode][k] >= 0; k++) {
        const int e = d - COPIES[mode][k];
        if (e >= 0 && e < width) return 1;
    }
    return 0;
}

static int ball_shown(const Orc *m) { return (((m->vdelbl & 1) ? m->enabl_old : m->enabl_new) & 2) != 0; }

static int ball_pixel(const Orc *m, int x) {
    return ball_shown(m) && columns_from(m->pos[OBJ_BL], x) < (1 << ((m->ctrlpf >> 4) & 3));
}

/* does any object show a pixel anywhere on the line (else nothing can collide) */
static int objects_shown(const Orc *m) {
    for (int i = 0; i < 2; i++)
        if (((m->vdelp[i] & 1) ? m->grp_old[i] : m->grp_new[i]) || missile_shown(m, i)) return 1;
    return ball_shown(m);
}

/* which objects and the playfield show at column x (OCC_* bits) */
static int occupancy(const Orc *m, int x) {
    return player_pixel(m, 0, x) * OCC_P0 | player_pixel(m, 1, x) * OCC_P1 | missile_pixel(m, 0, x) * OCC_M0 |
           missile_pixel(m, 1, x) * OCC_M1 | ball_pixel(m, x) * OCC_BL | playfield_bit(m, x) * OCC_PF;
}

/* which colour register owns pixel x given its occupancy (R18): 0 COLUP0,
 * 1 COLUP1, 2 COLUPF, 3 COLUBK */
static int pixel_owner(const Orc *m, int x, int occ) {
    const int field = (occ & OCC_PF) ? ((m->ctrlpf & 0x02) ? (x < 80 ? 0 : 1) : 2) : (occ & OCC_BL) ? 2 : -1;
    const int p0 = (occ & (OCC_P0 | OCC_M0)) != 0, p1 = (occ & (OCC_P1 | OCC_M1)) != 0;
    if ((m->ctrlpf & 0x04) && field >= 0) return field;
    if (p0) return 0;
    if (p1) return 1;
    if (field >= 0) return field;
    return 3;
}

/* the two occupancy bits of collision latch k (R19); pair 13 is unused */
static const int CX_PAIRS[16][2] = {
    {OCC_M0, OCC_P1}, {OCC_M0, OCC_P0}, {OCC_M1, OCC_P0}, {OCC_M1, OCC_P1}, {OCC_P0, OCC_PF}, {OCC_P0, OCC_BL},
    {OCC_P1, OCC_PF}, {OCC_P1, OCC_BL}, {OCC_M0, OCC_PF}, {OCC_M0, OCC_BL}, {OCC_M1, OCC_PF}, {OCC_M1, OCC_BL},
    {OCC_BL, OCC_PF}, {0, 0},           {OCC_P0, OCC_P1}, {OCC_M0, OCC_M1}};

/* Latch the collisions of colour clocks [cx_done, until) with the current state. */
static void tia_collide_until(Orc *m, int64_t until) {
    if (until <= m->cx_done) return;
    if (objects_shown(m)) {
        int occ[SCREEN_W];
        for (int x = 0; x < SCREEN_W; x++) occ[x] = occupancy(m, x);
        for (int64_t cc = m->cx_done; cc < until; cc++) {
            const int h = (int)(cc % CLOCKS_PER_LINE);
            if (h < HBLANK_CLOCKS) continue;
            const int x = h - HBLANK_CLOCKS;
            if (x < 8 && cc / CLOCKS_PER_LINE == m->hmove_line) continue; /* HMOVE blank */
            for (int k = 0; k < 16; k++)
                if (CX_PAIRS[k][0] && (occ[x] & CX_PAIRS[k][0]) && (occ[x] & CX_PAIRS[k][1])) m->cx |= 1u << k;
        }
    }
    m->cx_done = until;
}

static uint8_t colour_reg(const Orc *m, int owner) {
    switch (owner) {
        case 0: return m->colup0;
        case 1: return m->colup1;
        case 2: return m->colupf;
        default: return m->colubk;
    }
}

/* Render colour clocks [drawn, until) with the current register values.  Only
 * the visible window of the frame being stored is materialised; clocks outside
 * it produce no stored pixel. */
static void tia_draw_until(Orc *m, int64_t until) {
    if (m->draw_frame >= 0) {
        int64_t vis0 = m->draw_frame * CLOCKS_PER_FRAME + (int64_t)m->ystart * CLOCKS_PER_LINE;
        int64_t vis1 = vis0 + (int64_t)SCREEN_H * CLOCKS_PER_LINE;
        int64_t from = m->drawn > vis0 ? m->drawn : vis0;
        int64_t to = until < vis1 ? until : vis1;
        for (int64_t cc = from; cc < to; cc++) {
            int64_t rel = cc - vis0;
            int y = (int)(rel / CLOCKS_PER_LINE);
            int h = (int)(rel % CLOCKS_PER_LINE);
            if (h < HBLANK_CLOCKS) continue;
            int x = h - HBLANK_CLOCKS;
            int idx = y * SCREEN_W + x;
            if ((m->vblank & 0x02) || (x < 8 && cc / CLOCKS_PER_LINE == m->hmove_line)) {
                m->frame[idx] = 0;
                if (m->g) {
                    m->g->pixel_node[idx] = -1;
                    for (int o = 0; o < NOBJ; o++) m->g->pos_delta[o * SCREEN_H * SCREEN_W + idx] = 0;
                }
            } else {
                const int owner = pixel_owner(m, x, occupancy(m, x));
                const int c = colour_reg(m, owner) & 0xFE;
                m->frame[idx] = (uint8_t)c;
                if (m->g) {
                    m->g->pixel_node[idx] = m->g->slot_col[owner];
                    for (int o = 0; o < NOBJ; o++) { /* R20: the object one column further right */
                        const int saved = m->pos[o];
                        m->pos[o] = (saved + 1) % SCREEN_W;
                        const int c1 = colour_reg(m, pixel_owner(m, x, occupancy(m, x))) & 0xFE;
                        m->pos[o] = saved;
                        m->g->pos_delta[o * SCREEN_H * SCREEN_W + idx] = c1 - c;
                    }
                }
            }
        }
    }
    if (until > m->drawn) m->drawn = until;
}

/* Column of an object strobed at colour clock cc (R15): players start 5
 * columns after the strobe, missiles and the ball 4. */
static int strobe_column(int64_t cc, int lag) {
    const int h = (int)(cc % CLOCKS_PER_LINE);
    return h < HBLANK_CLOCKS ? lag - 2 : (h - HBLANK_CLOCKS + lag) % SCREEN_W;
}

static void tia_write(Orc *m, int reg, uint8_t v, int64_t w) {
    const int64_t cc = 3 * (w + 1); /* R4 */
    tia_draw_until(m, cc);
    tia_collide_until(m, cc);
    switch (reg & 0x3F) {
        case 0x04: m->nusiz[0] = v; break;
        case 0x05: m->nusiz[1] = v; break;
        case 0x0B: m->refp[0] = v; break;
        case 0x0C: m->refp[1] = v; break;
        case 0x10: m->pos[OBJ_P0] = strobe_column(cc, 5); break;
        case 0x11: m->pos[OBJ_P1] = strobe_column(cc, 5); break;
        case 0x12: m->pos[OBJ_M0] = strobe_column(cc, 4); break;
        case 0x13: m->pos[OBJ_M1] = strobe_column(cc, 4); break;
        case 0x14: m->pos[OBJ_BL] = strobe_column(cc, 4); break;
        case 0x1B: /* GRP0; GRP1's old register takes GRP1 */
            m->grp_new[0] = v;
            m->grp_old[1] = m->grp_new[1];
            break;
        case 0x1C: /* GRP1; GRP0's and ENABL's old registers take theirs */
            m->grp_new[1] = v;
            m->grp_old[0] = m->grp_new[0];
            m->enabl_old = m->enabl_new;
            break;
        case 0x1D: m->enam[0] = v; break;
        case 0x1E: m->enam[1] = v; break;
        case 0x1F: m->enabl_new = v; break;
        case 0x20: case 0x21: case 0x22: case 0x23: case 0x24: m->hm[(reg & 0x3F) - 0x20] = v; break;
        case 0x25: m->vdelp[0] = v; break;
        case 0x26: m->vdelp[1] = v; break;
        case 0x27: m->vdelbl = v; break;
        case 0x28: case 0x29: { /* RESMP: released, the missile moves to its player's centre */
            const int i = (reg & 0x3F) - 0x28, mode = m->nusiz[i] & 7;
            const int half = 4 * (mode == 5 ? 2 : mode == 7 ? 4 : 1);
            if ((m->resmp[i] & 2) && !(v & 2)) m->pos[OBJ_M0 + i] = (m->pos[OBJ_P0 + i] + half) % SCREEN_W;
            m->resmp[i] = v;
            break;
        }
        case 0x2A: /* HMOVE (R17) */
            for (int o = 0; o < NOBJ; o++) {
                const int mv = (int8_t)m->hm[o] >> 4;
                m->pos[o] = ((m->pos[o] - mv) % SCREEN_W + SCREEN_W) % SCREEN_W;
            }
            if (cc % CLOCKS_PER_LINE < HBLANK_CLOCKS) m->hmove_line = cc / CLOCKS_PER_LINE;
            break;
        case 0x2B: memset(m->hm, 0, sizeof m->hm); break;
        case 0x2C: m->cx = 0; break;
        case 0x00: m->vsync = v; break;
        case 0x01: m->vblank = v; break;
        case 0x02: m->wsync = 1; break;
        case 0x06: m->colup0 = v; break;
        case 0x07: m->colup1 = v; break;
        case 0x08: m->colupf = v; break;
        case 0x09: m->colubk = v; break;
        case 0x0A: m->ctrlpf = v; break;
        case 0x0D: m->pf0 = v; break;
        case 0x0E: m->pf1 = v; break;
        case 0x0F: m->pf2 = v; break;
        default: break; /* audio, RSYNC and the unused addresses */
    }
}

/* TIA read in cycle t (R7, R19) */
static uint8_t tia_read(Orc *m, int reg, int64_t t) {
    const int r = reg & 0x0F;
    if (r < 8) {
        tia_collide_until(m, 3 * t + 3);
        return (uint8_t)((((m->cx >> (2 * r)) & 1) << 7) | (((m->cx >> (2 * r + 1)) & 1) << 6));
    }
    switch (r) {
        case 0x0C: return m->inpt4;
        case 0x0D: return 0x80;
        default: return 0x00; /* paddles and undriven bits */
    }
}

/* ---- RIOT ---------------------------------------------------------------- */

static uint8_t intim_at(const Orc *m, int64_t t) {
    int64_t k = t - m->tim_write - 1;
    int64_t vi = (int64_t)m->tim_value * m->tim_interval;
    if (k < vi) return (uint8_t)(m->tim_value - 1 - k / m->tim_interval);
    return (uint8_t)((255 - (k - vi)) & 255);
}

static int timint_at(const Orc *m, int64_t t) {
    int64_t under = m->tim_write + 1 + (int64_t)m->tim_value * m->tim_interval;
    return (t >= under && m->tim_read < under) ? 0x80 : 0x00;
}

static uint8_t riot_read(Orc *m, uint16_t addr, int64_t t, int side_effects) {
    if (!(addr & 0x04)) {
        switch (addr & 0x03) {
            case 0: return m->swcha;
            case 2: return m->swchb; /* SWCHB: colour, difficulty B; RESET (bit 0) low while held */
            default: return 0x00; /* data-direction registers: all inputs */
        }
    }
    if (!(addr & 0x01)) {
        uint8_t v = intim_at(m, t);
        if (side_effects) m->tim_read = t;
        return v;
    }
    return (uint8_t)timint_at(m, t);
}

static void riot_write(Orc *m, uint16_t addr, uint8_t v, int64_t w) {
    if ((addr & 0x14) == 0x14) {
        static const int interval[4] = {1, 8, 64, 1024};
        m->tim_write = w;
        m->tim_value = v;
        m->tim_interval = interval[addr & 0x03];
    }
    /* port data / direction and edge-detect control: no visible effect here */
}

/* ---- bus ------------------------------------------------------------------ */

static void relax_note(Orc *m) {
    if (m->rx.ndiv < 0) m->rx.ndiv = (int64_t)m->instructions;
    m->rx.fails++;
}

/* Eq. s-read on the memory array r[0..n) at index a, cast to a byte. */
static uint8_t relaxed_read(Orc *m, const uint8_t *r, int n, int a) {
    if (m->rx.track) { /* float64 deviation of the read over the whole array, before the cast */
        double num = 0.0, den = 0.0;
        for (int i = 0; i < n; i++) {
            const double w = exp(-fabs((double)(i - a)) / m->rx.T);
            num += w * (double)r[i];
            den += w;
        }
        m->rx.dev_read += fabs(num / den - (double)r[a]);
        m->rx.nread++;
    }
    const float ra = (float)r[a];
    float num = 0.0f, den = 1.0f;
    for (int k = 1; k <= RELAX_WINDOW; k++) {
        const float u = m->rx.u[k];
        if (a + k < n) {
            num = num + u * ((float)r[a + k] - ra);
            den = den + u;
        }
        if (a - k >= 0) {
            num = num + u * ((float)r[a - k] - ra);
            den = den + u;
        }
    }
    const int v = (int)rintf(ra + num / den);
    if (v != r[a]) relax_note(m);
    return (uint8_t)v;
}

static uint8_t rom_value(Orc *m, int off) {
    return (m->rx.on && m->rx_active) ? relaxed_read(m, m->rom, m->rom_size, off) : m->rom[off];
}

static uint8_t ram_value(Orc *m, int cell) {
    return (m->rx.on && m->rx_active) ? relaxed_read(m, m->ram, 128, cell) : m->ram[cell];
}

/* Fetch-type read: no side effects (opcode/operand fetches, pointers, NOP reads). */
static uint8_t bus_peek(Orc *m, uint16_t addr, int64_t t) {
    addr &= 0x1FFF;
    if (mapper_sc(m->mapper) && (addr & 0x1F80) == 0x1080) return m->sc_ram[addr & 0x7F];
    if (addr & 0x1000) return rom_value(m, cart_offset(m, addr));
    if (!(addr & 0x80)) return tia_read(m, addr, t);
    if (!(addr & 0x200)) return ram_value(m, addr & 0x7F);
    return riot_read(m, addr, t, 0);
}

static void hotspot(Orc *m, uint16_t addr) {
    if (m->mapper == ORC_MAPPER_E0) {
        if (addr >= 0x1FE0 && addr <= 0x1FF7) m->slice[(addr - 0x1FE0) >> 3] = addr & 7;
        return;
    }
    const int n = mapper_banks(m->mapper);
    if (n > 1) { /* F8: $1FF8-9, F6: $1FF6-9, F4: $1FF4-B */
        const int first = n == 2 ? 0x1FF8 : n == 4 ? 0x1FF6 : 0x1FF4;
        if (addr >= first && addr < first + n) m->bank = addr - first;
    }
}

/* Data read at cycle t (R5). */
static uint8_t bus_read(Orc *m, uint16_t addr, int64_t t) {
    addr &= 0x1FFF;
    if (mapper_sc(m->mapper) && (addr & 0x1F80) == 0x1080) return m->sc_ram[addr & 0x7F];
    if (addr & 0x1000) {
        hotspot(m, addr);
        return rom_value(m, cart_offset(m, addr));
    }
    if (!(addr & 0x80)) return tia_read(m, addr, t);
    if (!(addr & 0x200)) return ram_value(m, addr & 0x7F);
    return riot_read(m, addr, t, 1);
}

/* A write to a TIA register shows from colour clock 3w+3 (R4): render the
 * pixels before that clock with the current registers and their current
 * content nodes before anything about the write is applied. */
static void draw_before_write(Orc *m, uint16_t addr, int64_t w) {
    addr &= 0x1FFF;
    if (!(addr & 0x1000) && !(addr & 0x80)) tia_draw_until(m, 3 * (w + 1));
}

/* Data write at cycle w (R5). */
static void bus_write(Orc *m, uint16_t addr, uint8_t v, int64_t w) {
    addr &= 0x1FFF;
    if (mapper_sc(m->mapper) && (addr & 0x1F80) == 0x1000) {
        m->sc_ram[addr & 0x7F] = v;
        return;
    }
    if (addr & 0x1000) {
        hotspot(m, addr);
        return;
    }
    if (!(addr & 0x80)) {
        tia_write(m, addr, v, w);
        return;
    }
    if (!(addr & 0x200)) {
        m->ram[addr & 0x7F] = v;
        return;
    }
    riot_write(m, addr, v, w);
}

/* ---- soft: content nodes of a data read / slot of a data write ------------ */

static int32_t rom_leaf(Orc *m, int off) {
    Graph *g = m->g;
    if (g->rom_leaf[off] == -2)
        g->rom_leaf[off] = g_new(g, -1, 0, 0, -1, 0, 0, g->rom_ev[off], g->rom_hard[off]);
    return g->rom_leaf[off];
}

/* Node holding the content of a data read at addr (after its side effects). */
static int32_t read_node(Orc *m, uint16_t addr) {
    Graph *g = m->g;
    addr &= 0x1FFF;
    if (addr & 0x1000) return rom_leaf(m, cart_offset(m, addr));
    if (!(addr & 0x80)) return (addr & 0x0F) == 0x0C ? g->inpt4_leaf[m->step] : -1;
    if (!(addr & 0x200)) return g->slot_ram[addr & 0x7F];
    if (!(addr & 0x04) && (addr & 0x03) == 0) return g->swcha_leaf[m->step];
    return -1; /* SWCHB, direction registers, timer: constants */
}

/* R21 (the leaky address surrogate): with a read temperature T > 0, an indexed
 * read of a ROM or RAM byte (zp,X  zp,Y  abs,X  abs,Y  (zp),Y) also depends on
 * its index register through Eq. s-read: the value at address a is the
 * distance-softmax blend of the array's bytes j with weights exp(-|j-a|/T)
 * (|j - a| <= 8, inside the ROM image or the 128 RAM cells), and its slope at the
 * hard address, taken symmetrically (the j = a term, whose kink has equal and
 * opposite one-sided slopes, contributes nothing), with the coefficients at
 * hard values (R[a] for the blend), is
 *   kappa = (1/T) sum_j w_j sign(j - a) (R[j] - R[a]),  w = the normalised weights.
 * A new node carries v + kappa (index - its hard value). */
static double read_slope(const uint8_t *r, int n, int a, double T) {
    double z = 0.0, acc = 0.0;
    for (int j = a - RELAX_WINDOW; j <= a + RELAX_WINDOW; j++) {
        if (j < 0 || j >= n) continue;
        const double w = exp(-fabs((double)(j - a)) / T);
        z += w;
        acc += w * (double)((j > a) - (j < a)) * ((double)r[j] - (double)r[a]);
    }
    return acc / (z * T);
}

static int32_t address_node(Orc *m, int32_t node, uint16_t ea, int mode, int v) {
    Graph *g = m->g;
    if (!(g->read_T > 0.0)) return node;
    int32_t idx_slot;
    int idx_hard;
    if (mode == ZPX || mode == ABX) {
        idx_slot = g->slot_x;
        idx_hard = m->x;
    } else if (mode == ZPY || mode == ABY || mode == IZY) {
        idx_slot = g->slot_y;
        idx_hard = m->y;
    } else {
        return node;
    }
    const uint16_t addr = ea & 0x1FFF;
    double kappa;
    if (addr & 0x1000) kappa = read_slope(m->rom, m->rom_size, cart_offset(m, addr), g->read_T);
    else if ((addr & 0x80) && !(addr & 0x200)) kappa = read_slope(m->ram, 128, addr & 0x7F, g->read_T);
    else return node; /* TIA and RIOT registers: no array to blend over */
    return g_affine(g, node, 1.0, v, idx_slot, kappa, idx_hard, v);
}

/* Slot overwritten by a data write at addr (NULL: a sink with no content). */
static int32_t *write_slot(Orc *m, uint16_t addr) {
    Graph *g = m->g;
    addr &= 0x1FFF;
    if (addr & 0x1000) return NULL;
    if (!(addr & 0x80)) {
        switch (addr & 0x3F) {
            case 0x06: return &g->slot_col[0];
            case 0x07: return &g->slot_col[1];
            case 0x08: return &g->slot_col[2];
            case 0x09: return &g->slot_col[3];
            default: return NULL;
        }
    }
    if (!(addr & 0x200)) return &g->slot_ram[addr & 0x7F];
    return NULL;
}

/* ---- flags ---------------------------------------------------------------- */

static void set_flag(Orc *m, int f, int on) {
    if (on) m->p |= f;
    else m->p &= (uint8_t)~f;
}

static void set_nz(Orc *m, uint8_t v) {
    set_flag(m, FZ, v == 0);
    set_flag(m, FN, v & 0x80);
}

/* ---- ALU (R11) ------------------------------------------------------------ */

static uint8_t alu_adc(Orc *m, uint8_t a, uint8_t v) {
    int c = m->p & FC;
    if (m->p & FD) {
        int lo = (a & 0x0F) + (v & 0x0F) + c;
        if (lo >= 0x0A) lo = ((lo + 0x06) & 0x0F) + 0x10;
        int sum = (a & 0xF0) + (v & 0xF0) + lo;
        int ssum = (int)(int8_t)(a & 0xF0) + (int)(int8_t)(v & 0xF0) + lo;
        set_flag(m, FZ, ((a + v + c) & 0xFF) == 0);
        set_flag(m, FN, ssum & 0x80);
        set_flag(m, FV, ssum < -128 || ssum > 127);
        if (sum >= 0xA0) sum += 0x60;
        set_flag(m, FC, sum >= 0x100);
        return (uint8_t)sum;
    }
    int sum = a + v + c;
    set_flag(m, FV, (~(a ^ v) & (a ^ sum) & 0x80) != 0);
    set_flag(m, FC, sum > 0xFF);
    set_nz(m, (uint8_t)sum);
    return (uint8_t)sum;
}

static uint8_t alu_sbc(Orc *m, uint8_t a, uint8_t v) {
    int c = m->p & FC;
    int diff = a - v - (1 - c);
    uint8_t bin = (uint8_t)diff;
    set_flag(m, FV, ((a ^ v) & (a ^ bin) & 0x80) != 0);
    set_flag(m, FC, diff >= 0);
    set_nz(m, bin);
    if (!(m->p & FD)) return bin;
    int lo = (a & 0x0F) - (v & 0x0F) + c - 1;
    if (lo < 0) lo = ((lo - 0x06) & 0x0F) - 0x10;
    int res = (a & 0xF0) - (v & 0xF0) + lo;
    if (res < 0) res -= 0x60;
    return (uint8_t)res;
}

void orc_alu(int op, int a, int v, int p_in, int *result, int *p_out) {
    Orc m;
    memset(&m, 0, sizeof m);
    m.p = (uint8_t)p_in;
    *result = op == 0 ? alu_adc(&m, (uint8_t)a, (uint8_t)v) : alu_sbc(&m, (uint8_t)a, (uint8_t)v);
    *p_out = m.p;
}

/* ---- stack ---------------------------------------------------------------- */

static void push(Orc *m, uint8_t v, int64_t w, int32_t node) {
    uint16_t addr = (uint16_t)(0x100 | m->s);
    draw_before_write(m, addr, w);
    if (m->g) {
        int32_t *sl = write_slot(m, addr);
        if (sl) *sl = node;
    }
    bus_write(m, addr, v, w);
    m->s--;
}

static uint8_t pull(Orc *m, int64_t t, int32_t *node) {
    m->s++;
    uint16_t addr = (uint16_t)(0x100 | m->s);
    uint8_t v = bus_read(m, addr, t);
    if (m->g && node) *node = read_node(m, addr);
    return v;
}

/* ------------------------------------------------------------------------ */
/* Power-on                                                                 */
/* ------------------------------------------------------------------------ */
int orc_power_on(Orc *m, const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0, int ystart) {
    ops_init();
    Graph *g = m->g;
    Relax rx = m->rx;
    memset(m, 0, sizeof *m);
    m->g = g;
    m->rx = rx;
    if (ystart < 0 || ystart + SCREEN_H > LINES_PER_FRAME) return -1;
    if (mapper < 0 || mapper >= ORC_MAPPER_COUNT || rom_size != mapper_size(mapper)) return -1;
    memcpy(m->rom, rom, (size_t)rom_size);
    m->rom_size = rom_size;
    m->mapper = mapper;
    /* power-on banks: F8 (and F8SC) bank 1, F6/F4 bank 0, E0 slices 4, 5, 6 (7 fixed) */
    m->bank = (mapper == ORC_MAPPER_F8 || mapper == ORC_MAPPER_F8SC) ? 1 : 0;
    m->slice[0] = 4;
    m->slice[1] = 5;
    m->slice[2] = 6;
    m->slice[3] = 7;
    memcpy(m->ram, ram0, 128);
    m->a = m->x = m->y = 0;
    m->s = 0xFD;
    m->p = FI | FU;
    m->tim_write = -1;
    m->tim_value = 0;
    m->tim_interval = 1024;
    m->tim_read = 0;
    m->swcha = 0xFF;
    m->inpt4 = 0x80;
    m->swchb = 0x0B;
    m->ystart = ystart;
    m->draw_frame = -1;
    m->hmove_line = -1;
    uint16_t lo = bus_peek(m, 0x1FFC, 0), hi = bus_peek(m, 0x1FFD, 0);
    m->pc = (uint16_t)(lo | (hi << 8));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One instruction                                                          */
/* ------------------------------------------------------------------------ */

static int branch_taken(const Orc *m, int op) {
    switch (op) {
        case BPL: return !(m->p & FN);
        case BMI: return (m->p & FN) != 0;
        case BVC: return !(m->p & FV);
        case BVS: return (m->p & FV) != 0;
        case BCC: return !(m->p & FC);
        case BCS: return (m->p & FC) != 0;
        case BNE: return !(m->p & FZ);
        default: return (m->p & FZ) != 0; /* BEQ */
    }
}

/* The branch gate of Eq. (branch): z = s(2f - 1), g = sigma(alpha z).  Flags are
 * exact bits on the executed path, so |z| = 1. */
double orc_gate(double z, double alpha) { return 1.0 / (1.0 + exp(-alpha * z)); }
double orc_gate_grad(double z, double alpha) {
    double g = orc_gate(z, alpha);
    return alpha * g * (1.0 - g);
}

/* Execute one instruction starting at m->cycle.  Returns 0, or 1 when the CPU
 * is (or becomes) jammed. */
int orc_step_instruction(Orc *m) {
    if (m->jammed) return 1;
    Graph *g = m->g;
    const int64_t t0 = m->cycle;
    const uint16_t pc = m->pc;
    m->rx_active = 1;
    m->rx.dev_read = m->rx.dev_branch = 0.0;
    m->rx.nread = 0;
    const uint8_t opc = bus_peek(m, pc, t0);
    const OpRow info = OPS[opc];
    if (info.op == JAM) {
        m->jammed = 1;
        m->rx_active = 0;
        return 1;
    }
    const uint16_t a1 = (uint16_t)(pc + 1);
    const uint8_t lo = bus_peek(m, a1, t0), hi = bus_peek(m, (uint16_t)(pc + 2), t0);
    m->pc = (uint16_t)(pc + MODE_LEN[info.mode]);

    /* effective address */
    uint16_t ea = 0;
    int crossed = 0;
    switch (info.mode) {
        case ZP: ea = lo; break;
        case ZPX: ea = (uint8_t)(lo + m->x); break;
        case ZPY: ea = (uint8_t)(lo + m->y); break;
        case ABS: ea = (uint16_t)(lo | (hi << 8)); break;
        case ABX: {
            uint16_t base = (uint16_t)(lo | (hi << 8));
            ea = (uint16_t)(base + m->x);
            crossed = (base & 0xFF00) != (ea & 0xFF00);
            break;
        }
        case ABY: {
            uint16_t base = (uint16_t)(lo | (hi << 8));
            ea = (uint16_t)(base + m->y);
            crossed = (base & 0xFF00) != (ea & 0xFF00);
            break;
        }
        case IZX: {
            uint8_t zp = (uint8_t)(lo + m->x);
            ea = (uint16_t)(bus_peek(m, zp, t0) | (bus_peek(m, (uint8_t)(zp + 1), t0) << 8));
            break;
        }
        case IZY: {
            uint16_t base = (uint16_t)(bus_peek(m, lo, t0) | (bus_peek(m, (uint8_t)(lo + 1), t0) << 8));
            ea = (uint16_t)(base + m->y);
            crossed = (base & 0xFF00) != (ea & 0xFF00);
            break;
        }
        case IND: {
            uint16_t ptr = (uint16_t)(lo | (hi << 8));
            uint16_t ptr_hi = (uint16_t)((ptr & 0xFF00) | ((ptr + 1) & 0x00FF)); /* R12 page wrap */
            ea = (uint16_t)(bus_peek(m, ptr, t0) | (bus_peek(m, ptr_hi, t0) << 8));
            break;
        }
        case IMM: ea = a1; break;
        default: break;
    }
    int n = info.cycles + (info.page_penalty && crossed);
    const int op = info.op;

    /* operand value for reading instructions, accessed on the last cycle (R5) */
#define LOAD_OPERAND(v, node)                                                   \
    do {                                                                        \
        if (info.mode == IMM) {                                                 \
            v = lo;                                                             \
            if (g) node = read_node(m, a1);                                     \
        } else {                                                                \
            v = bus_read(m, ea, t0 + n - 1);                                    \
            if (g) node = address_node(m, read_node(m, ea), ea, info.mode, v);  \
        }                                                                       \
    } while (0)

    uint8_t v = 0;
    int32_t vn = -1;
    switch (op) {
        case LDA:
            LOAD_OPERAND(v, vn);
            m->a = v;
            set_nz(m, v);
            if (g) g->slot_a = vn;
            break;
        case LDX:
            LOAD_OPERAND(v, vn);
            m->x = v;
            set_nz(m, v);
            if (g) g->slot_x = vn;
            break;
        case LDY:
            LOAD_OPERAND(v, vn);
            m->y = v;
            set_nz(m, v);
            if (g) g->slot_y = vn;
            break;
        case LAX:
            LOAD_OPERAND(v, vn);
            m->a = m->x = v;
            set_nz(m, v);
            if (g) g->slot_a = g->slot_x = vn;
            break;
        case STA:
        case STX:
        case STY:
        case SAX: {
            uint8_t val;
            int32_t node = -1;
            if (op == STA) {
                val = m->a;
                if (g) node = g->slot_a;
            } else if (op == STX) {
                val = m->x;
                if (g) node = g->slot_x;
            } else if (op == STY) {
                val = m->y;
                if (g) node = g->slot_y;
            } else {
                val = m->a & m->x;
                if (g) node = g_logic(g, LOGIC_AND, g->slot_a, m->a, g->slot_x, m->x, val);
            }
            draw_before_write(m, ea, t0 + n - 1);
            if (g) {
                int32_t *sl = write_slot(m, ea);
                if (sl) *sl = node;
            }
            bus_write(m, ea, val, t0 + n - 1);
            break;
        }
        case ADC:
        case SBC: {
            LOAD_OPERAND(v, vn);
            uint8_t a_old = m->a;
            m->a = op == ADC ? alu_adc(m, a_old, v) : alu_sbc(m, a_old, v);
            if (g) g->slot_a = g_affine(g, g->slot_a, 1.0, a_old, vn, op == ADC ? 1.0 : -1.0, v, m->a);
            break;
        }
        case AND:
        case ORA:
        case EOR: {
            LOAD_OPERAND(v, vn);
            uint8_t a_old = m->a;
            m->a = op == AND ? (a_old & v) : op == ORA ? (a_old | v) : (a_old ^ v);
            set_nz(m, m->a);
            if (g) {
                int kind = op == AND ? LOGIC_AND : op == ORA ? LOGIC_ORA : LOGIC_EOR;
                g->slot_a = g_logic(g, kind, g->slot_a, a_old, vn, v, m->a);
            }
            break;
        }
        case CMP:
        case CPX:
        case CPY: {
            LOAD_OPERAND(v, vn);
            uint8_t r = op == CMP ? m->a : op == CPX ? m->x : m->y;
            set_flag(m, FC, r >= v);
            set_nz(m, (uint8_t)(r - v));
            break;
        }
        case BIT:
            LOAD_OPERAND(v, vn);
            set_flag(m, FZ, (m->a & v) == 0);
            set_flag(m, FN, v & 0x80);
            set_flag(m, FV, v & 0x40);
            break;
        case ASL:
        case LSR:
        case ROL:
        case ROR:
        case INC:
        case DEC: {
            int32_t in_node = -1;
            if (info.mode == ACC) {
                v = m->a;
                if (g) in_node = g->slot_a;
            } else {
                v = bus_read(m, ea, t0 + n - 3);
                if (g) in_node = read_node(m, ea);
            }
            uint8_t r;
            double k = 1.0;
            int c = m->p & FC;
            switch (op) {
                case ASL: set_flag(m, FC, v & 0x80); r = (uint8_t)(v << 1); k = 2.0; break;
                case LSR: set_flag(m, FC, v & 0x01); r = (uint8_t)(v >> 1); k = 0.5; break;
                case ROL: set_flag(m, FC, v & 0x80); r = (uint8_t)((v << 1) | c); k = 2.0; break;
                case ROR: set_flag(m, FC, v & 0x01); r = (uint8_t)((v >> 1) | (c << 7)); k = 0.5; break;
                case INC: r = (uint8_t)(v + 1); break;
                default: r = (uint8_t)(v - 1); break;
            }
            set_nz(m, r);
            int32_t out_node = -1;
            if (g) out_node = g_affine(g, in_node, k, v, -1, 0.0, 0, r);
            if (info.mode == ACC) {
                m->a = r;
                if (g) g->slot_a = out_node;
            } else {
                draw_before_write(m, ea, t0 + n - 1);
                if (g) {
                    int32_t *sl = write_slot(m, ea);
                    if (sl) *sl = out_node;
                }
                bus_write(m, ea, r, t0 + n - 1);
            }
            break;
        }
        case INX:
        case INY:
        case DEX:
        case DEY: {
            uint8_t *reg = (op == INX || op == DEX) ? &m->x : &m->y;
            int32_t *sl = g ? ((op == INX || op == DEX) ? &g->slot_x : &g->slot_y) : NULL;
            uint8_t old = *reg;
            *reg = (uint8_t)(op == INX || op == INY ? old + 1 : old - 1);
            set_nz(m, *reg);
            if (g) *sl = g_affine(g, *sl, 1.0, old, -1, 0.0, 0, *reg);
            break;
        }
        case TAX:
            m->x = m->a;
            set_nz(m, m->x);
            if (g) g->slot_x = g->slot_a;
            break;
        case TAY:
            m->y = m->a;
            set_nz(m, m->y);
            if (g) g->slot_y = g->slot_a;
            break;
        case TXA:
            m->a = m->x;
            set_nz(m, m->a);
            if (g) g->slot_a = g->slot_x;
            break;
        case TYA:
            m->a = m->y;
            set_nz(m, m->a);
            if (g) g->slot_a = g->slot_y;
            break;
        case TSX:
            m->x = m->s;
            set_nz(m, m->x);
            if (g) g->slot_x = -1; /* the stack pointer is not content */
            break;
        case TXS: m->s = m->x; break;
        case PHA: push(m, m->a, t0 + n - 1, g ? g->slot_a : -1); break;
        case PHP: push(m, (uint8_t)(m->p | FB | FU), t0 + n - 1, -1); break;
        case PLA: {
            int32_t node = -1;
            m->a = pull(m, t0 + n - 1, &node);
            set_nz(m, m->a);
            if (g) g->slot_a = node;
            break;
        }
        case PLP: m->p = (uint8_t)((pull(m, t0 + n - 1, NULL) & ~FB) | FU); break;
        case JMP: m->pc = ea; break;
        case JSR: {
            uint16_t ret = (uint16_t)(m->pc - 1);
            push(m, (uint8_t)(ret >> 8), t0 + n - 1, -1);
            push(m, (uint8_t)ret, t0 + n - 1, -1);
            m->pc = ea;
            break;
        }
        case RTS: {
            uint16_t l = pull(m, t0 + n - 1, NULL);
            uint16_t h = pull(m, t0 + n - 1, NULL);
            m->pc = (uint16_t)(((h << 8) | l) + 1);
            break;
        }
        case BRK: {
            uint16_t ret = (uint16_t)(pc + 2);
            push(m, (uint8_t)(ret >> 8), t0 + n - 1, -1);
            push(m, (uint8_t)ret, t0 + n - 1, -1);
            push(m, (uint8_t)(m->p | FB | FU), t0 + n - 1, -1);
            m->p |= FI;
            uint16_t l = bus_peek(m, 0x1FFE, t0), h = bus_peek(m, 0x1FFF, t0);
            m->pc = (uint16_t)(l | (h << 8));
            break;
        }
        case RTI: {
            m->p = (uint8_t)((pull(m, t0 + n - 1, NULL) & ~FB) | FU);
            uint16_t l = pull(m, t0 + n - 1, NULL);
            uint16_t h = pull(m, t0 + n - 1, NULL);
            m->pc = (uint16_t)((h << 8) | l);
            break;
        }
        case CLC: set_flag(m, FC, 0); break;
        case SEC: set_flag(m, FC, 1); break;
        case CLD: set_flag(m, FD, 0); break;
        case SED: set_flag(m, FD, 1); break;
        case CLI: set_flag(m, FI, 0); break;
        case SEI: set_flag(m, FI, 1); break;
        case CLV: set_flag(m, FV, 0); break;
        case NOP: break; /* operand reads of the NOP family have no side effects */
        case BPL:
        case BMI:
        case BVC:
        case BVS:
        case BCC:
        case BCS:
        case BNE:
        case BEQ: {
            const int taken = branch_taken(m, op);
            if (m->rx.on) {
                /* Eq. s-branch without STE: the flag is crisp, so z = +1 (taken) or -1 and
                 * pc = round(pc_fallthrough + sigma(alpha z) * delta); the cycle penalties
                 * follow the flag and the page of the pc reached */
                const double gd = 1.0 / (1.0 + exp(-m->rx.alpha * (taken ? 1.0 : -1.0)));
                m->rx.dev_branch = fabs(gd * (double)(int8_t)lo - (taken ? (double)(int8_t)lo : 0.0));
                const float gz = taken ? m->rx.g_taken : m->rx.g_not;
                const uint16_t cast = (uint16_t)(int)rintf((float)m->pc + gz * (float)(int8_t)lo);
                const uint16_t hard = taken ? (uint16_t)(m->pc + (int8_t)lo) : m->pc;
                if (cast != hard) relax_note(m);
                if (taken) {
                    crossed = (cast & 0xFF00) != (m->pc & 0xFF00);
                    n += 1 + crossed;
                    m->op_taken[opc]++;
                }
                m->pc = cast;
            } else if (taken) {
                uint16_t target = (uint16_t)(m->pc + (int8_t)lo);
                crossed = (target & 0xFF00) != (m->pc & 0xFF00);
                n += 1 + crossed;
                m->pc = target;
                m->op_taken[opc]++;
            }
            break;
        }
        default: break;
    }
#undef LOAD_OPERAND
    m->rx_active = 0;
    m->cycle = t0 + n;
    if (m->wsync) { /* R6 */
        m->wsync = 0;
        int64_t r = m->cycle % CYCLES_PER_LINE;
        if (r) m->cycle += CYCLES_PER_LINE - r;
    }
    m->instructions++;
    m->op_count[opc]++;
    if (crossed) m->op_cross[opc]++;
    return 0;
}

/* Run instructions until the first instruction boundary at or after `budget`
 * (a jammed CPU just lets the cycles elapse). */
static void run_until(Orc *m, int64_t budget) {
    while (m->cycle < budget) {
        if (m->jammed || orc_step_instruction(m)) {
            m->cycle = budget;
            break;
        }
    }
    tia_draw_until(m, 3 * m->cycle);
    tia_collide_until(m, 3 * m->cycle);
}

/* Actions 0..17: the joystick; ORC_ACTION_RESET: the console's RESET switch held
 * with the joystick idle (the boot sequence's RESET frames). */
void orc_set_action(Orc *m, int action) {
    const int joy = action == ORC_ACTION_RESET ? 0 : action;
    m->swcha = (uint8_t)orc_action_swcha(joy);
    m->inpt4 = (uint8_t)orc_action_inpt4(joy);
    m->swchb = action == ORC_ACTION_RESET ? 0x0A : 0x0B;
}

/* Superchip RAM contents (for the formats that have it). */
void orc_set_sc_ram(Orc *m, const uint8_t *v) { memcpy(m->sc_ram, v, 128); }
const uint8_t *orc_sc_ram(const Orc *m) { return m->sc_ram; }

/* Seeded Superchip RAM of (seed, env, episode): its own SplitMix64 stream, the
 * RAM stream's with the seed offset by ORC_SC_SEED (the paper pins this RAM's
 * contents deterministically; Sec. Discussion). */
void orc_splitmix_sc_ram(uint64_t seed, uint64_t env, uint64_t episode, uint8_t *out) {
    orc_splitmix_ram(seed ^ ORC_SC_SEED, env, episode, out);
}

/* One env step of `frame_skip` frames; `step_index` counts steps since power-on
 * so that the budget is aligned to the frame grid (R1). */
void orc_env_step(Orc *m, int action, int frame_skip, int64_t step_index, int store_frame) {
    orc_set_action(m, action);
    int64_t first = step_index * frame_skip;
    m->draw_frame = store_frame ? first + frame_skip - 1 : -1;
    run_until(m, (first + frame_skip) * (int64_t)CYCLES_PER_FRAME);
}

void orc_run_cycles(Orc *m, int64_t budget) { run_until(m, budget); }

void orc_set_draw_frame(Orc *m, int64_t frame) { m->draw_frame = frame; }

/* A, X, Y, S, P, PCL, PCH, bank, jammed, INTIM(now), TIMINT(now), VBLANK,
 * COLUP0, COLUP1, COLUPF, COLUBK, CTRLPF, PF0, PF1, PF2, VSYNC */
void orc_get_regs(const Orc *m, int64_t *out) {
    out[0] = m->a;
    out[1] = m->x;
    out[2] = m->y;
    out[3] = m->s;
    out[4] = m->p;
    out[5] = m->pc & 0xFF;
    out[6] = m->pc >> 8;
    out[7] = m->bank;
    out[8] = m->jammed;
    out[9] = intim_at(m, m->cycle);
    out[10] = timint_at(m, m->cycle);
    out[11] = m->vblank;
    out[12] = m->colup0;
    out[13] = m->colup1;
    out[14] = m->colupf;
    out[15] = m->colubk;
    out[16] = m->ctrlpf;
    out[17] = m->pf0;
    out[18] = m->pf1;
    out[19] = m->pf2;
    out[20] = m->vsync;
    out[21] = m->cycle;
    out[22] = (int64_t)m->instructions;
}

/* Object registers (R15-R19) now: columns of P0, P1, M0, M1, BL; GRP0, GRP1;
 * their old registers; ENAM0, ENAM1, ENABL, its old register; NUSIZ0, NUSIZ1,
 * REFP0, REFP1, VDELP0, VDELP1, VDELBL, RESMP0, RESMP1; HMP0, HMP1, HMM0,
 * HMM1, HMBL; the collision latches (low byte, high byte); 0, 0, 0. */
void orc_get_objects(Orc *m, int64_t *out) {
    tia_collide_until(m, 3 * m->cycle);
    int n = 0;
    for (int o = 0; o < NOBJ; o++) out[n++] = m->pos[o];
    out[n++] = m->grp_new[0];
    out[n++] = m->grp_new[1];
    out[n++] = m->grp_old[0];
    out[n++] = m->grp_old[1];
    out[n++] = m->enam[0];
    out[n++] = m->enam[1];
    out[n++] = m->enabl_new;
    out[n++] = m->enabl_old;
    out[n++] = m->nusiz[0];
    out[n++] = m->nusiz[1];
    out[n++] = m->refp[0];
    out[n++] = m->refp[1];
    out[n++] = m->vdelp[0];
    out[n++] = m->vdelp[1];
    out[n++] = m->vdelbl;
    out[n++] = m->resmp[0];
    out[n++] = m->resmp[1];
    for (int o = 0; o < NOBJ; o++) out[n++] = m->hm[o];
    out[n++] = m->cx & 0xFF;
    out[n++] = m->cx >> 8;
    while (n < 32) out[n++] = 0;
}

/* FULL relaxed mode on (bit 0 of on; bit 1: also record the float64 pre-cast
 * deviations) at (alpha, T), or off; resets the divergence record. */
void orc_set_relax(Orc *m, int on, double alpha, double T) {
    m->rx.on = on & 1;
    m->rx.track = (on >> 1) & 1;
    m->rx.u[0] = 1.0f;
    for (int k = 1; k <= RELAX_WINDOW; k++) m->rx.u[k] = (float)exp(-(double)k / T);
    m->rx.g_taken = (float)(1.0 / (1.0 + exp(-alpha)));
    m->rx.g_not = (float)(1.0 / (1.0 + exp(alpha)));
    m->rx.ndiv = -1;
    m->rx.fails = 0;
    m->rx.T = T;
    m->rx.alpha = alpha;
}

/* The last instruction's float64 pre-cast deviations: out[0] = summed read
 * deviation, out[1] = number of relaxed reads, out[2] = branch deviation. */
void orc_relax_last_dev(const Orc *m, double *out) {
    out[0] = m->rx.dev_read;
    out[1] = m->rx.nread;
    out[2] = m->rx.dev_branch;
}

/* State vector of Theorem "Temperature-limit bound" (registers, RAM, RIOT, TIA,
 * frame buffer, time); returns its length. */
static int state_vector(const Orc *m, double *v) {
    int n = 0;
    v[n++] = m->a; v[n++] = m->x; v[n++] = m->y; v[n++] = m->s; v[n++] = m->p; v[n++] = m->pc;
    v[n++] = m->bank; v[n++] = m->jammed; v[n++] = (double)m->cycle;
    v[n++] = (double)m->tim_write; v[n++] = m->tim_value; v[n++] = m->tim_interval; v[n++] = (double)m->tim_read;
    v[n++] = m->vsync; v[n++] = m->vblank; v[n++] = m->colup0; v[n++] = m->colup1; v[n++] = m->colupf;
    v[n++] = m->colubk; v[n++] = m->ctrlpf; v[n++] = m->pf0; v[n++] = m->pf1; v[n++] = m->pf2;
    for (int i = 0; i < 128; i++) v[n++] = m->ram[i];
    for (int i = 0; i < SCREEN_H * SCREEN_W; i++) v[n++] = m->frame[i];
    return n;
}

/* Relaxed dispatch of Eq. s-select for the instruction at the machine's pc:
 * every handler k = 0..255 runs (hard) from the current state on a copy whose
 * opcode byte is k, giving the state vector V_k; with w = softmax(logits/T),
 * dev = max_i |sum_k w_k V_k[i] - V_k*[i]| for the argmax k*, spread =
 * max_k max_i |V_k[i] - V_k*[i]| and w_star = w_k*.  The machine is not
 * changed. */
void orc_dispatch_deviation(const Orc *m, const double *logits, double T, double *dev, double *spread,
                            double *w_star) {
    enum { NV = 23 + 128 + SCREEN_H * SCREEN_W };
    double *V = (double *)malloc(sizeof(double) * 256 * NV);
    Orc *c = (Orc *)malloc(sizeof(Orc));
    const int off = cart_offset(m, m->pc);
    int best = 0;
    for (int k = 0; k < 256; k++) {
        *c = *m;
        c->g = NULL;
        c->rx.on = 0;
        if (m->pc & 0x1000) c->rom[off] = (uint8_t)k;
        orc_step_instruction(c);
        state_vector(c, V + (size_t)k * NV);
        if (logits[k] > logits[best]) best = k;
    }
    double w[256], z = 0.0;
    for (int k = 0; k < 256; k++) z += (w[k] = exp((logits[k] - logits[best]) / T));
    for (int k = 0; k < 256; k++) w[k] /= z;
    double d = 0.0, sp = 0.0;
    const double *vs = V + (size_t)best * NV;
    for (int i = 0; i < NV; i++) {
        double acc = 0.0;
        for (int k = 0; k < 256; k++) {
            acc += w[k] * V[(size_t)k * NV + i];
            const double e = fabs(V[(size_t)k * NV + i] - vs[i]);
            if (e > sp) sp = e;
        }
        if (fabs(acc - vs[i]) > d) d = fabs(acc - vs[i]);
    }
    *dev = d;
    *spread = sp;
    *w_star = w[best];
    free(V);
    free(c);
}

/* First instruction (counted from power-on) whose cast differed from the exact
 * value, or -1; and the number of such casts. */
int64_t orc_relax_ndiv(const Orc *m) { return m->rx.ndiv; }
uint64_t orc_relax_fails(const Orc *m) { return m->rx.fails; }

/* Opcode statistics since power-on: out[0..255] executions per opcode byte,
 * out[256..511] of them with a page crossing (indexed address or taken branch),
 * out[512..767] taken branches. */
void orc_op_stats(const Orc *m, uint64_t *out) {
    for (int i = 0; i < 256; i++) {
        out[i] = m->op_count[i];
        out[256 + i] = m->op_cross[i];
        out[512 + i] = m->op_taken[i];
    }
}

const uint8_t *orc_ram(const Orc *m) { return m->ram; }
const uint8_t *orc_frame(const Orc *m) { return m->frame; }
void orc_poke_ram(Orc *m, int cell, int v) { m->ram[cell & 0x7F] = (uint8_t)v; }
int orc_intim_at(const Orc *m, int64_t t) { return intim_at(m, t); }
int orc_timint_at(const Orc *m, int64_t t) { return timint_at(m, t); }

/* ------------------------------------------------------------------------ */
/* Whole-env hard rollout                                                   */
/* ------------------------------------------------------------------------ */
int orc_run_env(const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0, const uint8_t *actions,
                int steps, int frame_skip, int ystart, const uint32_t *ep_steps, int n_episodes, uint64_t seed,
                int64_t env_index, uint8_t *ram_out, uint8_t *frame_out, int frames_mode, uint8_t *done_out,
                int64_t *final_regs, uint64_t *instructions, uint8_t *step_state) {
    Orc *m = orc_new();
    if (orc_power_on(m, rom, rom_size, mapper, ram0, ystart)) {
        orc_free(m);
        return -1;
    }
    uint8_t sc[128];
    orc_splitmix_sc_ram(seed, (uint64_t)env_index, 0, sc);
    orc_set_sc_ram(m, sc);
    int64_t ep = 0, ep_step = 0;
    uint64_t total_instr = 0;
    for (int s = 0; s < steps; s++) {
        int store = frames_mode == 2 || (frames_mode == 1 && s == steps - 1);
        orc_env_step(m, actions ? actions[s] : 0, frame_skip, ep_step, store);
        ep_step++;
        memcpy(ram_out + (size_t)s * 128, m->ram, 128);
        if (store && frame_out)
            memcpy(frame_out + (size_t)(frames_mode == 2 ? s : 0) * SCREEN_H * SCREEN_W, m->frame,
                   SCREEN_H * SCREEN_W);
        int done = 0;
        if (ep_steps && ep < n_episodes && ep_step >= (int64_t)ep_steps[ep]) done = 1;
        if (done_out) done_out[s] = (uint8_t)done;
        if (done) { /* in-run reset (power-on with SplitMix64 RAM for the next episode) */
            total_instr += m->instructions;
            ep++;
            uint8_t r[128];
            orc_splitmix_ram(seed, (uint64_t)env_index, (uint64_t)ep, r);
            orc_power_on(m, rom, rom_size, mapper, r, ystart);
            orc_splitmix_sc_ram(seed, (uint64_t)env_index, (uint64_t)ep, sc);
            orc_set_sc_ram(m, sc);
            ep_step = 0;
        }
        if (step_state) { /* machine state after the step: the 16 inspection bytes, then RAM */
            int64_t rg[25];
            orc_get_regs(m, rg);
            for (int i = 0; i < 16; i++) step_state[(size_t)s * 144 + i] = (uint8_t)rg[i];
            memcpy(step_state + (size_t)s * 144 + 16, m->ram, 128);
        }
    }
    total_instr += m->instructions;
    if (final_regs) {
        orc_get_regs(m, final_regs);
        final_regs[23] = ep;
        final_regs[24] = ep_step;
    }
    if (instructions) *instructions = total_instr;
    orc_free(m);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Soft decode (Eq. select with V = 0..255, and the RAM tape)                 */
/* ------------------------------------------------------------------------ */

/* Rows of K logits: hard = argmax (lowest index on ties), w = softmax(row/tau),
 * ev = sum_k k w_k, plus the softmax max and normaliser. */
void orc_decode_logit_rows(const float *rows, int64_t n, int k, double tau, uint8_t *hard, double *ev, double *mx,
                           double *z) {
    for (int64_t r = 0; r < n; r++) {
        const float *L = rows + r * k;
        int best = 0;
        for (int j = 1; j < k; j++)
            if (L[j] > L[best]) best = j;
        double m = L[best], s = 0.0, e = 0.0;
        for (int j = 0; j < k; j++) s += exp(((double)L[j] - m) / tau);
        for (int j = 0; j < k; j++) e += j * exp(((double)L[j] - m) / tau) / s;
        hard[r] = (uint8_t)best;
        ev[r] = e;
        if (mx) mx[r] = m;
        if (z) z[r] = s;
    }
}

/* RAM tape rows (content, not logits): hard = argmax, ev = sum_k k P[k]. */
void orc_decode_tape_rows(const float *rows, int64_t n, uint8_t *hard, double *ev) {
    for (int64_t r = 0; r < n; r++) {
        const float *P = rows + r * 256;
        int best = 0;
        double e = 0.0;
        for (int j = 0; j < 256; j++) {
            if (P[j] > P[best]) best = j;
            e += j * (double)P[j];
        }
        hard[r] = (uint8_t)best;
        ev[r] = e;
    }
}

/* Action rows: hard action = argmax l, and the expected port values
 * E_w[SWCHA], E_w[INPT4] under w = softmax(l/tau). */
void orc_decode_action_rows(const float *rows, int64_t n, double tau, uint8_t *hard, double *e_swcha,
                            double *e_inpt4) {
    for (int64_t r = 0; r < n; r++) {
        const float *L = rows + r * 18;
        int best = 0;
        for (int j = 1; j < 18; j++)
            if (L[j] > L[best]) best = j;
        double m = L[best], s = 0.0, es = 0.0, ei = 0.0;
        for (int j = 0; j < 18; j++) s += exp(((double)L[j] - m) / tau);
        for (int j = 0; j < 18; j++) {
            double w = exp(((double)L[j] - m) / tau) / s;
            es += w * orc_action_swcha(j);
            ei += w * orc_action_inpt4(j);
        }
        hard[r] = (uint8_t)best;
        e_swcha[r] = es;
        e_inpt4[r] = ei;
    }
}

/* Vector-Jacobian product through a softmax at temperature tau:
 * given dL/dv for a value v = sum_j val_j w_j, w = softmax(L/tau), return
 * dL/dL_k = sum_j gv * val_j * dw_j/dL_k with dw_j/dL_k = w_j (delta_jk - w_k)/tau
 * (the full Jacobian, written out). */
static void softmax_vjp(const float *L, int k, double tau, const double *val, double gv, double *out) {
    double m = L[0];
    for (int j = 1; j < k; j++)
        if (L[j] > m) m = L[j];
    double *w = (double *)malloc(sizeof(double) * (size_t)k);
    double s = 0.0;
    for (int j = 0; j < k; j++) s += (w[j] = exp(((double)L[j] - m) / tau));
    for (int j = 0; j < k; j++) w[j] /= s;
    for (int kk = 0; kk < k; kk++) {
        double acc = 0.0;
        for (int j = 0; j < k; j++) acc += gv * val[j] * w[j] * ((j == kk ? 1.0 : 0.0) - w[kk]) / tau;
        out[kk] = acc;
    }
    free(w);
}

/* dL/dlogits for ROM rows from dL/d(byte value) g[a]. */
void orc_epilogue_rom(const float *logits, int64_t n, double tau, const double *g, double *out) {
    double val[256];
    for (int j = 0; j < 256; j++) val[j] = j;
    for (int64_t r = 0; r < n; r++) softmax_vjp(logits + r * 256, 256, tau, val, g[r], out + r * 256);
}

/* dL/dP0[c,k] = k * g0[c] (ev0 = sum_k k P0[c,k] is linear in the tape). */
void orc_epilogue_tape(int64_t n, const double *g0, double *out) {
    for (int64_t r = 0; r < n; r++)
        for (int k = 0; k < 256; k++) out[r * 256 + k] = k * g0[r];
}

/* dL/dl for action rows from dL/dSWCHA and dL/dINPT4 of the step. */
void orc_epilogue_action(const float *logits, int64_t n, double tau, const double *g_swcha, const double *g_inpt4,
                         double *out) {
    double vs[18], vi[18], a[18], b[18];
    for (int j = 0; j < 18; j++) {
        vs[j] = orc_action_swcha(j);
        vi[j] = orc_action_inpt4(j);
    }
    for (int64_t r = 0; r < n; r++) {
        softmax_vjp(logits + r * 18, 18, tau, vs, g_swcha[r], a);
        softmax_vjp(logits + r * 18, 18, tau, vi, g_inpt4[r], b);
        for (int j = 0; j < 18; j++) out[r * 18 + j] = a[j] + b[j];
    }
}

/* ------------------------------------------------------------------------ */
/* Soft rollout of one env (SOFT-STE forward = hard; surrogate backward)      */
/* ------------------------------------------------------------------------ */
/* The soft rollout may start mid-episode: the machine first takes pre_steps
 * HARD env steps from power-on (actions pre_actions, no graph), and the soft
 * steps continue from that state (the paper's env step, state + action -> next
 * state).  The registers and RAM of that state are then constants of the
 * graph (no RAM0 leaves: g_ram0 is 0) and the soft steps' frames keep their
 * place on the frame grid. */
int orc_soft_env_from(const uint8_t *rom_hard, const double *rom_ev, int rom_size, int mapper,
                      const uint8_t *ram0_hard, const double *ram0_ev, int pre_steps, const uint8_t *pre_actions,
                      const uint8_t *act_hard, const double *swcha_ev, const double *inpt4_ev, int steps,
                      int frame_skip, int ystart, int mode, double read_T, const double *grad_frame,
                      const double *grad_ram, uint8_t *ram_out, uint8_t *frame_out, double *ram_smooth,
                      double *frame_smooth, double *g_rom, double *g_ram0, double *g_swcha, double *g_inpt4,
                      double *g_pos, double *frame_dpos, int64_t *n_nodes) {
    /* the soft value graph has no content nodes for Superchip RAM: those formats run hard only */
    if (mapper < 0 || mapper >= ORC_MAPPER_COUNT || mapper_sc(mapper)) return -1;
    Graph *g = (Graph *)calloc(1, sizeof(Graph));
    g->rom_size = rom_size;
    g->read_T = read_T;
    g->rom_hard = rom_hard;
    g->rom_ev = rom_ev;
    g->rom_leaf = (int32_t *)malloc(sizeof(int32_t) * (size_t)rom_size);
    for (int i = 0; i < rom_size; i++) g->rom_leaf[i] = -2;
    g->steps = steps;
    g->swcha_leaf = (int32_t *)malloc(sizeof(int32_t) * (size_t)steps);
    g->inpt4_leaf = (int32_t *)malloc(sizeof(int32_t) * (size_t)steps);
    g->swcha_ev = swcha_ev;
    g->inpt4_ev = inpt4_ev;
    g->act_hard = act_hard;
    g->pixel_node = (int32_t *)malloc(sizeof(int32_t) * SCREEN_H * SCREEN_W);
    for (int i = 0; i < SCREEN_H * SCREEN_W; i++) g->pixel_node[i] = -1;
    g->pos_delta = (int32_t *)calloc((size_t)NOBJ * SCREEN_H * SCREEN_W, sizeof(int32_t));
    g->ramout_node = (int32_t *)malloc(sizeof(int32_t) * (size_t)steps * 128);
    g->slot_a = g->slot_x = g->slot_y = -1; /* power-on registers are constants */
    for (int i = 0; i < 4; i++) g->slot_col[i] = -1;
    for (int c = 0; c < 128; c++)
        g->slot_ram[c] = g->ram0_leaf[c] =
            pre_steps > 0 ? -1 : g_new(g, -1, 0, 0, -1, 0, 0, ram0_ev[c], ram0_hard[c]);
    for (int s = 0; s < steps; s++) {
        g->swcha_leaf[s] = g_new(g, -1, 0, 0, -1, 0, 0, swcha_ev[s], orc_action_swcha(act_hard[s]));
        g->inpt4_leaf[s] = g_new(g, -1, 0, 0, -1, 0, 0, inpt4_ev[s], orc_action_inpt4(act_hard[s]));
    }

    Orc *m = orc_new();
    if (orc_power_on(m, rom_hard, rom_size, mapper, ram0_hard, ystart)) {
        orc_free(m);
        return -1;
    }
    for (int s = 0; s < pre_steps; s++) orc_env_step(m, pre_actions ? pre_actions[s] : 0, frame_skip, s, 0);
    m->g = g;
    for (int s = 0; s < steps; s++) {
        m->step = s;
        orc_env_step(m, act_hard[s], frame_skip, pre_steps + s, s == steps - 1);
        for (int c = 0; c < 128; c++) {
            g->ramout_node[s * 128 + c] = g->slot_ram[c];
            if (ram_out) ram_out[s * 128 + c] = m->ram[c];
            if (ram_smooth) ram_smooth[s * 128 + c] = g_sv(g, g->slot_ram[c], m->ram[c]);
        }
    }
    for (int i = 0; i < SCREEN_H * SCREEN_W; i++) {
        if (frame_out) frame_out[i] = m->frame[i];
        int32_t id = g->pixel_node[i];
        if (frame_smooth) frame_smooth[i] = m->frame[i] + (id >= 0 ? g->n[id].vs - g->n[id].vh : 0.0);
    }

    /* reverse sweep over the recorded graph */
    double *adj = (double *)calloc((size_t)g->len, sizeof(double));
    if (grad_frame)
        for (int i = 0; i < SCREEN_H * SCREEN_W; i++)
            if (g->pixel_node[i] >= 0) adj[g->pixel_node[i]] += grad_frame[i];
    if (grad_ram)
        for (int64_t i = 0; i < (int64_t)steps * 128; i++)
            if (g->ramout_node[i] >= 0) adj[g->ramout_node[i]] += grad_ram[i];
    for (int64_t i = g->len - 1; i >= 0; i--) {
        const Node *x = &g->n[i];
        if (adj[i] == 0.0) continue;
        if (x->p0 >= 0) adj[x->p0] += (mode ? x->sm0 : x->ste0) * adj[i];
        if (x->p1 >= 0) adj[x->p1] += (mode ? x->sm1 : x->ste1) * adj[i];
    }
    for (int a = 0; a < rom_size; a++)
        if (g->rom_leaf[a] >= 0) g_rom[a] += adj[g->rom_leaf[a]];
    for (int c = 0; c < 128; c++) g_ram0[c] = g->ram0_leaf[c] >= 0 ? adj[g->ram0_leaf[c]] : 0.0;
    for (int s = 0; s < steps; s++) {
        g_swcha[s] = adj[g->swcha_leaf[s]];
        g_inpt4[s] = adj[g->inpt4_leaf[s]];
    }
    if (frame_dpos) /* R20: the sampler's tangent images of the final frame */
        for (int i = 0; i < NOBJ * SCREEN_H * SCREEN_W; i++) frame_dpos[i] = (double)g->pos_delta[i];
    if (g_pos) /* R20: the sampler's derivative for each object's column */
        for (int o = 0; o < NOBJ; o++) {
            double acc = 0.0;
            if (grad_frame)
                for (int i = 0; i < SCREEN_H * SCREEN_W; i++)
                    acc += grad_frame[i] * (double)g->pos_delta[o * SCREEN_H * SCREEN_W + i];
            g_pos[o] = acc;
        }
    if (n_nodes) *n_nodes = g->len;

    free(adj);
    orc_free(m);
    free(g->n);
    free(g->rom_leaf);
    free(g->swcha_leaf);
    free(g->inpt4_leaf);
    free(g->pixel_node);
    free(g->pos_delta);
    free(g->ramout_node);
    free(g);
    return 0;
}

int orc_soft_env(const uint8_t *rom_hard, const double *rom_ev, int rom_size, int mapper, const uint8_t *ram0_hard,
                 const double *ram0_ev, const uint8_t *act_hard, const double *swcha_ev, const double *inpt4_ev,
                 int steps, int frame_skip, int ystart, int mode, const double *grad_frame, const double *grad_ram,
                 uint8_t *ram_out, uint8_t *frame_out, double *ram_smooth, double *frame_smooth, double *g_rom,
                 double *g_ram0, double *g_swcha, double *g_inpt4, int64_t *n_nodes) {
    return orc_soft_env_from(rom_hard, rom_ev, rom_size, mapper, ram0_hard, ram0_ev, 0, NULL, act_hard, swcha_ev,
                             inpt4_ev, steps, frame_skip, ystart, mode, 0.0, grad_frame, grad_ram, ram_out,
                             frame_out, ram_smooth, frame_smooth, g_rom, g_ram0, g_swcha, g_inpt4, NULL, NULL,
                             n_nodes);
}
