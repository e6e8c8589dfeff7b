// Per-env machine core of libvcs: 6507 CPU, TIA subset and RIOT, written for
// one env per lane (or per lane group).  Used by the hard-step, soft-forward
// and soft-backward kernels; memory placement and side outputs (pixels,
// checkpoints, tape records) come in through the Mem and Hook policies.
//
// Machine semantics (paper: "A Differentiable Atari VCS", Sec. "Why the Atari
// VCS Is Good Ground Truth", Sec. "Building Two Differentiable VCS Ports"):
//  - 13-bit bus: A12 set = cartridge; else A7 clear = TIA; else A9 clear = RAM
//    (128 B, mirrored through the stack page); else RIOT ports/timer.
//  - 2K images mirror on A11; F8 images switch 4 KB banks on data accesses to
//    $1FF8/$1FF9 (a hotspot read returns the newly selected bank's byte).
//  - Loads and stores access memory in an instruction's last cycle; a
//    read-modify-write reads three cycles before its end; all pushes of an
//    instruction take effect in its last cycle.
//  - A TIA write in CPU cycle n shows from colour clock 3n+3; WSYNC resumes the
//    CPU at cycle 0 of the next line; a pixel is the owning colour register &
//    0xFE (0 while VBLANK bit 1 is set).
//  - TIA objects (players, missiles, ball): see the object model below.
//  - RIOT timer: after writing V with interval 2^shift at cycle w the timer
//    underflows at u = w + 1 + V*2^shift; before u INTIM = -1 - floor((t-u)/I),
//    from u on INTIM = (255 - (t - u)) mod 256; TIMINT bit 7 is set from u
//    until an INTIM read.
//  - The 67 opcode bytes outside the paper's set of 189 jam the CPU.
#pragma once

#include "vcs_internal.hpp"

namespace vcs {

// ---------------------------------------------------------------------------
// Opcode decode, derived from the regular aaabbbcc structure of the 6502
// opcode matrix and the documented per-addressing-mode timing rules.
// ---------------------------------------------------------------------------
enum Cls : uint32_t {
    C_JAM = 0, C_LDA, C_LDX, C_LDY, C_LAX, C_STA, C_STX, C_STY, C_SAX,
    C_ADC, C_SBC, C_AND, C_ORA, C_EOR, C_CMP, C_CPX, C_CPY, C_BIT,
    C_ASL, C_LSR, C_ROL, C_ROR, C_INC, C_DEC,
    C_INX, C_INY, C_DEX, C_DEY, C_TAX, C_TAY, C_TXA, C_TYA, C_TSX, C_TXS,
    C_PHA, C_PHP, C_PLA, C_PLP, C_JMP, C_JSR, C_RTS, C_RTI, C_BRK,
    C_BRANCH, C_FLAG, C_NOP
};
enum Mode : uint32_t { M_IMP, M_ACC, M_IMM, M_ZP, M_ZPX, M_ZPY, M_ABS, M_ABX, M_ABY, M_IZX, M_IZY, M_IND, M_REL };

constexpr uint32_t kFlagC = 0x01, kFlagZ = 0x02, kFlagI = 0x04, kFlagD = 0x08, kFlagB = 0x10, kFlagU = 0x20,
                   kFlagV = 0x40, kFlagN = 0x80;

constexpr uint32_t mode_len(uint32_t m) {
    return (m == M_IMP || m == M_ACC) ? 1u : (m == M_ABS || m == M_ABX || m == M_ABY || m == M_IND) ? 3u : 2u;
}

// entry = class | mode << 6 | cycles << 10 | page penalty << 13 | length << 14 | aux << 16 | set << 24
constexpr uint32_t enc(uint32_t cls, uint32_t m, uint32_t cyc, uint32_t pen, uint32_t aux = 0, uint32_t set = 0) {
    return cls | (m << 6) | (cyc << 10) | (pen << 13) | (mode_len(m) << 14) | (aux << 16) | (set << 24);
}
// read instructions: +1 cycle when an indexed read crosses a page
constexpr uint32_t rd_timing(uint32_t cls, uint32_t m) {
    return m == M_IMM ? enc(cls, m, 2, 0) : m == M_ZP ? enc(cls, m, 3, 0)
         : (m == M_ZPX || m == M_ZPY) ? enc(cls, m, 4, 0) : m == M_ABS ? enc(cls, m, 4, 0)
         : (m == M_ABX || m == M_ABY) ? enc(cls, m, 4, 1) : m == M_IZX ? enc(cls, m, 6, 0) : enc(cls, m, 5, 1);
}
// write instructions: indexed forms always take the extra cycle
constexpr uint32_t wr_timing(uint32_t cls, uint32_t m) {
    return m == M_ZP ? enc(cls, m, 3, 0) : (m == M_ZPX || m == M_ZPY) ? enc(cls, m, 4, 0)
         : m == M_ABS ? enc(cls, m, 4, 0) : (m == M_ABX || m == M_ABY) ? enc(cls, m, 5, 0) : enc(cls, m, 6, 0);
}
// read-modify-write instructions
constexpr uint32_t rmw_timing(uint32_t cls, uint32_t m) {
    return m == M_ACC ? enc(cls, m, 2, 0) : m == M_ZP ? enc(cls, m, 5, 0)
         : (m == M_ZPX || m == M_ABS) ? enc(cls, m, 6, 0) : enc(cls, m, 7, 0);
}

constexpr uint32_t decode_op(uint32_t op) {
    const uint32_t aaa = op >> 5, bbb = (op >> 2) & 7u, cc = op & 3u;
    const uint32_t g1_mode[8] = {M_IZX, M_ZP, M_IMM, M_ABS, M_IZY, M_ZPX, M_ABY, M_ABX};
    if (cc == 1) {  // ORA AND EOR ADC STA LDA CMP SBC
        const uint32_t cls[8] = {C_ORA, C_AND, C_EOR, C_ADC, C_STA, C_LDA, C_CMP, C_SBC};
        if (aaa == 4) return bbb == 2 ? rd_timing(C_NOP, M_IMM) : wr_timing(C_STA, g1_mode[bbb]);
        return rd_timing(cls[aaa], g1_mode[bbb]);
    }
    if (cc == 2) {  // shifts, STX/LDX, DEC/INC and their implied column
        if (bbb == 4) return 0;
        if (aaa <= 3) {
            const uint32_t cls[4] = {C_ASL, C_ROL, C_LSR, C_ROR};
            switch (bbb) {
                case 1: return rmw_timing(cls[aaa], M_ZP);
                case 2: return rmw_timing(cls[aaa], M_ACC);
                case 3: return rmw_timing(cls[aaa], M_ABS);
                case 5: return rmw_timing(cls[aaa], M_ZPX);
                case 6: return enc(C_NOP, M_IMP, 2, 0);
                case 7: return rmw_timing(cls[aaa], M_ABX);
                default: return 0;
            }
        }
        if (aaa == 4) {
            switch (bbb) {
                case 0: return rd_timing(C_NOP, M_IMM);
                case 1: return wr_timing(C_STX, M_ZP);
                case 2: return enc(C_TXA, M_IMP, 2, 0);
                case 3: return wr_timing(C_STX, M_ABS);
                case 5: return wr_timing(C_STX, M_ZPY);
                case 6: return enc(C_TXS, M_IMP, 2, 0);
                default: return 0;
            }
        }
        if (aaa == 5) {
            switch (bbb) {
                case 0: return rd_timing(C_LDX, M_IMM);
                case 1: return rd_timing(C_LDX, M_ZP);
                case 2: return enc(C_TAX, M_IMP, 2, 0);
                case 3: return rd_timing(C_LDX, M_ABS);
                case 5: return rd_timing(C_LDX, M_ZPY);
                case 6: return enc(C_TSX, M_IMP, 2, 0);
                case 7: return rd_timing(C_LDX, M_ABY);
                default: return 0;
            }
        }
        const uint32_t cls = aaa == 6 ? C_DEC : C_INC;
        switch (bbb) {
            case 0: return rd_timing(C_NOP, M_IMM);
            case 1: return rmw_timing(cls, M_ZP);
            case 2: return enc(aaa == 6 ? C_DEX : C_NOP, M_IMP, 2, 0);
            case 3: return rmw_timing(cls, M_ABS);
            case 5: return rmw_timing(cls, M_ZPX);
            case 6: return enc(C_NOP, M_IMP, 2, 0);
            case 7: return rmw_timing(cls, M_ABX);
            default: return 0;
        }
    }
    if (cc == 0) {
        if (bbb == 4) {  // Bxx: flag N, V, C, Z by aaa>>1; branch when set if aaa is odd
            const uint32_t flag[4] = {kFlagN, kFlagV, kFlagC, kFlagZ};
            return enc(C_BRANCH, M_REL, 2, 0, flag[aaa >> 1], aaa & 1u);
        }
        if (bbb == 6) {  // CLC SEC CLI SEI TYA CLV CLD SED
            if (aaa == 4) return enc(C_TYA, M_IMP, 2, 0);
            const uint32_t flag[8] = {kFlagC, kFlagC, kFlagI, kFlagI, 0, kFlagV, kFlagD, kFlagD};
            return enc(C_FLAG, M_IMP, 2, 0, flag[aaa], (aaa & 1u) && aaa != 5);
        }
        if (bbb == 2) {  // PHP PLP PHA PLA DEY TAY INY INX
            const uint32_t cls[8] = {C_PHP, C_PLP, C_PHA, C_PLA, C_DEY, C_TAY, C_INY, C_INX};
            const uint32_t cyc[8] = {3, 4, 3, 4, 2, 2, 2, 2};
            return enc(cls[aaa], M_IMP, cyc[aaa], 0);
        }
        if (bbb == 0) {
            switch (aaa) {
                case 0: return enc(C_BRK, M_IMP, 7, 0);
                case 1: return enc(C_JSR, M_ABS, 6, 0);
                case 2: return enc(C_RTI, M_IMP, 6, 0);
                case 3: return enc(C_RTS, M_IMP, 6, 0);
                case 4: return rd_timing(C_NOP, M_IMM);
                case 5: return rd_timing(C_LDY, M_IMM);
                case 6: return rd_timing(C_CPY, M_IMM);
                default: return rd_timing(C_CPX, M_IMM);
            }
        }
        if (bbb == 1) {
            switch (aaa) {
                case 1: return rd_timing(C_BIT, M_ZP);
                case 4: return wr_timing(C_STY, M_ZP);
                case 5: return rd_timing(C_LDY, M_ZP);
                case 6: return rd_timing(C_CPY, M_ZP);
                case 7: return rd_timing(C_CPX, M_ZP);
                default: return rd_timing(C_NOP, M_ZP);
            }
        }
        if (bbb == 3) {
            switch (aaa) {
                case 0: return rd_timing(C_NOP, M_ABS);
                case 1: return rd_timing(C_BIT, M_ABS);
                case 2: return enc(C_JMP, M_ABS, 3, 0);
                case 3: return enc(C_JMP, M_IND, 5, 0);
                case 4: return wr_timing(C_STY, M_ABS);
                case 5: return rd_timing(C_LDY, M_ABS);
                case 6: return rd_timing(C_CPY, M_ABS);
                default: return rd_timing(C_CPX, M_ABS);
            }
        }
        if (bbb == 5) return aaa == 4 ? wr_timing(C_STY, M_ZPX) : aaa == 5 ? rd_timing(C_LDY, M_ZPX)
                                                                           : rd_timing(C_NOP, M_ZPX);
        /* bbb == 7 */
        return aaa == 4 ? 0u : aaa == 5 ? rd_timing(C_LDY, M_ABX) : rd_timing(C_NOP, M_ABX);
    }
    // cc == 3: only USBC ($EB), SAX and LAX belong to the set
    if (op == 0xEB) return rd_timing(C_SBC, M_IMM);
    if (aaa == 4) {
        switch (bbb) {
            case 0: return wr_timing(C_SAX, M_IZX);
            case 1: return wr_timing(C_SAX, M_ZP);
            case 3: return wr_timing(C_SAX, M_ABS);
            case 5: return wr_timing(C_SAX, M_ZPY);
            default: return 0;
        }
    }
    if (aaa == 5) {
        switch (bbb) {
            case 0: return rd_timing(C_LAX, M_IZX);
            case 1: return rd_timing(C_LAX, M_ZP);
            case 3: return rd_timing(C_LAX, M_ABS);
            case 4: return rd_timing(C_LAX, M_IZY);
            case 5: return rd_timing(C_LAX, M_ZPY);
            case 7: return rd_timing(C_LAX, M_ABY);
            default: return 0;
        }
    }
    return 0;
}

struct DecodeTable {
    uint32_t e[256];
};
constexpr DecodeTable make_decode_table() {
    DecodeTable t{};
    for (uint32_t i = 0; i < 256; ++i) t.e[i] = decode_op(i);
    return t;
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014) in counter form, for in-run reset RAM
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
// Word i (0..15) of the reset RAM of (seed, env, episode): 8 little-endian bytes.
__host__ __device__ __forceinline__ uint64_t reset_ram_word(uint64_t seed, uint64_t env, uint64_t episode, uint32_t i) {
    uint64_t k = sm64_mix(seed + (env + 1) * kGolden);
    k = sm64_mix(k + (episode + 1) * kGolden);
    return sm64_mix(k + (uint64_t)(i + 1) * kGolden);
}

// ---------------------------------------------------------------------------
// Playfield geometry: 40 groups of 4 pixels per line, one playfield bit each.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t rev8(uint32_t v) {
    v = ((v & 0xF0u) >> 4) | ((v & 0x0Fu) << 4);
    v = ((v & 0xCCu) >> 2) | ((v & 0x33u) << 2);
    return ((v & 0xAAu) >> 1) | ((v & 0x55u) << 1);
}
// 20-bit mask, bit i = playfield bit of half-line position i (PF0 b4..b7, PF1 b7..b0, PF2 b0..b7)
__host__ __device__ __forceinline__ uint32_t pf_mask20(uint32_t pf) {
    return ((pf >> 4) & 0xFu) | (rev8((pf >> 8) & 0xFFu) << 4) | (((pf >> 16) & 0xFFu) << 12);
}
// Owning colour register of 4-pixel group g (0..39): 0 COLUP0, 1 COLUP1, 2 COLUPF, 3 COLUBK.
__host__ __device__ __forceinline__ uint32_t group_owner(uint32_t g, uint32_t mask20, uint32_t ctrlpf) {
    const uint32_t i = g < 20 ? g : ((ctrlpf & 1u) ? 39u - g : g - 20u);
    if (!((mask20 >> i) & 1u)) return 3u;
    return (ctrlpf & 2u) ? (g < 20 ? 0u : 1u) : 2u;
}

// Visit the 4-pixel groups of frame-relative colour clocks [from, to) that fall in
// the visible window; lane `sub` of a group of G lanes takes every G-th group of
// each line.  f(y, g, xa, xb) gets the row, the group and the covered pixels [xa, xb).
template <class F>
__host__ __device__ __forceinline__ void for_each_group(int32_t from, int32_t to, int32_t ystart, uint32_t sub,
                                                        uint32_t G, F &&f) {
    const int32_t vis0 = ystart * kClocksPerLine, vis1 = vis0 + kScreenH * kClocksPerLine;
    if (from < vis0) from = vis0;
    if (to > vis1) to = vis1;
    while (from < to) {
        const int32_t rel = from - vis0;
        const int32_t y = rel / kClocksPerLine;
        const int32_t h = rel - y * kClocksPerLine;
        const int32_t line0 = from - h;
        const int32_t seg_end = to < line0 + kClocksPerLine ? to : line0 + kClocksPerLine;
        const int32_t x0 = h > kHBlank ? h - kHBlank : 0;
        const int32_t x1 = seg_end - line0 - kHBlank;
        if (x1 > x0) {
            const int32_t g1 = (x1 + 3) >> 2;
            for (int32_t g = (x0 >> 2) + (int32_t)sub; g < g1; g += (int32_t)G) {
                const int32_t xa = x0 > 4 * g ? x0 : 4 * g;
                const int32_t xb = x1 < 4 * g + 4 ? x1 : 4 * g + 4;
                f(y, g, xa, xb);
            }
        }
        from = seg_end;
    }
}

// ---------------------------------------------------------------------------
// TIA objects (Sec. "Hard and Soft Execution": object priority, sprite bits and
// the strobe-timed sprite column), as the documented TIA has them:
//  - P0, P1, M0, M1 and BL each sit at a column (its first pixel), 0 at
//    power-on.  A strobe (RESP0/1, RESM0/1, RESBL) taking effect at clock h of
//    its line puts a player at column h - 68 + 5 and a missile or the ball at
//    h - 68 + 4 (mod 160), or at 3 / 2 when h lies in horizontal blank.
//  - NUSIZ bits 0-2: a player's copies at column offsets {0} {0,16} {0,32}
//    {0,16,32} {0,64} {0} {0,32,64} {0}, its pixel width 1, 2 (mode 5) or 4
//    (mode 7); the graphics byte shows bit 7 first, bit 0 first when REFP bit 3
//    is set.  A missile has its player's copies, width 2^(NUSIZ bits 4-5), and
//    shows while ENAM bit 1 is set and RESMP bit 1 clear; releasing RESMP moves
//    it to its player's column + 4 * pixel width.  The ball is one copy, width
//    2^(CTRLPF bits 4-5), shown while ENABL bit 1 is set.  A GRP0 write copies
//    GRP1 to GRP1's old register; a GRP1 write copies GRP0 and ENABL to theirs;
//    VDELP0/1 and VDELBL bit 0 display the old registers.
//  - HMOVE moves each object left by the signed high nibble of its motion
//    register; HMCLR zeroes them.  An HMOVE taking effect in horizontal blank
//    blacks out columns 0..7 of its line (no collisions there either).
//  - Priority: P0/M0 (COLUP0) over P1/M1 (COLUP1) over playfield and ball over
//    the background; CTRLPF bit 2 puts playfield and ball first.  Score mode
//    colours the playfield only; the ball is COLUPF.
//  - Collisions latch wherever two objects, or an object and the playfield,
//    show at one visible column (VBLANK does not mask them); CXCLR clears; a read
//    in cycle t sees clocks before 3t + 3.  Register r reads pair 2r in bit 7 and
//    2r + 1 in bit 6: M0-P1, M0-P0, M1-P0, M1-P1, P0-PF, P0-BL, P1-PF, P1-BL,
//    M0-PF, M0-BL, M1-PF, M1-BL, BL-PF, -, P0-P1, M0-M1.
// Rows of 160 columns are five 32-bit words (column x = bit x & 31 of word
// x >> 5), so a row of a span is built once and read a 4-pixel nibble at a time.
// ---------------------------------------------------------------------------
constexpr uint32_t kObRefp0 = 1u << 16, kObRefp1 = 1u << 17, kObVdelp0 = 1u << 18, kObVdelp1 = 1u << 19,
                   kObVdelbl = 1u << 20, kObEnam0 = 1u << 21, kObEnam1 = 1u << 22, kObEnabl = 1u << 23,
                   kObEnablOld = 1u << 24, kObResmp0 = 1u << 25, kObResmp1 = 1u << 26;
struct Objs {
    uint32_t pos;  // columns: P0 | P1 << 8 | M0 << 16 | M1 << 24
    uint32_t gfx;  // GRP0 | GRP1 << 8 | GRP0 old << 16 | GRP1 old << 24
    uint32_t ctl;  // NUSIZ0 | NUSIZ1 << 8 | kOb* flags
    uint32_t bl;   // ball column | (frame-relative line of the last HMOVE blank + 1) << 8 (0: none)
};
// The TIA registers the pixel pipeline reads: colours, playfield + CTRLPF,
// VBLANK | VSYNC << 8, objects.
struct Tia {
    uint32_t col, pf, vb;
    Objs ob;
};
enum ObjRow : uint32_t { R_P0 = 0, R_P1, R_M0, R_M1, R_BL, R_PF, kRows };

__host__ __device__ __forceinline__ uint32_t shown_gfx(const Objs &o, uint32_t i) {
    const bool vdel = (o.ctl & (i ? kObVdelp1 : kObVdelp0)) != 0u;
    return (o.gfx >> (8u * i + (vdel ? 16u : 0u))) & 0xFFu;
}
__host__ __device__ __forceinline__ bool missile_on(const Objs &o, uint32_t i) {
    return (o.ctl & (i ? kObEnam1 : kObEnam0)) && !(o.ctl & (i ? kObResmp1 : kObResmp0));
}
__host__ __device__ __forceinline__ bool ball_on(const Objs &o) {
    return (o.ctl & ((o.ctl & kObVdelbl) ? kObEnablOld : kObEnabl)) != 0u;
}
// does any object show a pixel (else nothing but the playfield is drawn and nothing collides)
__host__ __device__ __forceinline__ bool objs_shown(const Objs &o) {
    return (shown_gfx(o, 0) | shown_gfx(o, 1)) != 0u || missile_on(o, 0) || missile_on(o, 1) || ball_on(o);
}
// NUSIZ mode m's copies as a set over column offsets 16 j, j = 0..4
__host__ __device__ __forceinline__ uint32_t copy_set(uint32_t m) {
    constexpr uint64_t kSets = 1ull | 3ull << 5 | 5ull << 10 | 7ull << 15 | 17ull << 20 | 1ull << 25 | 21ull << 30 |
                               1ull << 35;
    return (uint32_t)(kSets >> (5u * (m & 7u))) & 31u;
}
// log2 of a player's pixel width in NUSIZ mode m
__host__ __device__ __forceinline__ uint32_t player_shift(uint32_t m) {
    m &= 7u;
    return m == 5u ? 1u : m == 7u ? 2u : 0u;
}
__host__ __device__ __forceinline__ uint32_t wrap160(uint32_t c) { return c >= 160u ? c - 160u : c; }
// column of an object strobed at frame-relative colour clock cc (lag 5: players, 4: missiles and ball)
__host__ __device__ __forceinline__ uint32_t strobe_column(int32_t cc, uint32_t lag) {
    const uint32_t h = (uint32_t)(cc % kClocksPerLine);
    return h < (uint32_t)kHBlank ? lag - 2u : wrap160(h - (uint32_t)kHBlank + lag);
}

struct Row160 {
    uint32_t w[5];
};
__host__ __device__ __forceinline__ uint32_t row_word(const Row160 &r, uint32_t k) {
    uint32_t v = r.w[0];
#pragma unroll
    for (uint32_t i = 1; i < 5; ++i) v = k == i ? r.w[i] : v;
    return v;
}
// OR a pattern of up to 32 columns (bit e = column c + e, wrapping at 160) into r
__host__ __device__ __forceinline__ void row_place(Row160 &r, uint32_t pat, uint32_t c) {
    const uint32_t k = c >> 5, s = c & 31u;
    const uint32_t lo = pat << s, hi = s ? pat >> (32u - s) : 0u;
    const uint32_t k1 = k == 4u ? 0u : k + 1u;
#pragma unroll
    for (uint32_t i = 0; i < 5; ++i) r.w[i] |= (i == k ? lo : 0u) | (i == k1 ? hi : 0u);
}
// the same row one column further right (column 159 goes to 0)
__host__ __device__ __forceinline__ Row160 row_shift1(const Row160 &r) {
    Row160 o;
#pragma unroll
    for (uint32_t i = 0; i < 5; ++i) o.w[i] = (r.w[i] << 1) | (r.w[i == 0 ? 4 : i - 1] >> 31);
    return o;
}
// each bit of an 8-bit pattern repeated over 2^sh columns
__host__ __device__ __forceinline__ uint32_t widen(uint32_t p, uint32_t sh) {
    const uint32_t one = (1u << (1u << sh)) - 1u;
    uint32_t r = 0;
#pragma unroll
    for (uint32_t b = 0; b < 8; ++b) r |= ((p >> b) & 1u) ? one << (b << sh) : 0u;
    return r;
}
// 8 bits -> 32: bit i fills nibble i
__host__ __device__ __forceinline__ uint32_t spread4(uint32_t v) {
    v &= 0xFFu;
    v = (v | (v << 12)) & 0x000F000Fu;
    v = (v | (v << 6)) & 0x03030303u;
    v = (v | (v << 3)) & 0x11111111u;
    return v * 15u;
}
__host__ __device__ __forceinline__ void player_row(Row160 &r, const Objs &o, uint32_t i) {
    const uint32_t m = (o.ctl >> (8u * i)) & 7u;
    const uint32_t g = shown_gfx(o, i);
    const uint32_t p8 = (o.ctl & (i ? kObRefp1 : kObRefp0)) ? g : rev8(g);  // bit e = the e-th pixel
    const uint32_t pat = widen(p8, player_shift(m));
    const uint32_t c = (o.pos >> (8u * i)) & 0xFFu, set = copy_set(m);
#pragma unroll
    for (uint32_t j = 0; j < 5; ++j)
        if ((set >> j) & 1u) row_place(r, pat, wrap160(c + 16u * j));
}
__host__ __device__ __forceinline__ void missile_row(Row160 &r, const Objs &o, uint32_t i) {
    if (!missile_on(o, i)) return;
    const uint32_t nus = (o.ctl >> (8u * i)) & 0xFFu;
    const uint32_t pat = (1u << (1u << ((nus >> 4) & 3u))) - 1u;
    const uint32_t c = (o.pos >> (16u + 8u * i)) & 0xFFu, set = copy_set(nus & 7u);
#pragma unroll
    for (uint32_t j = 0; j < 5; ++j)
        if ((set >> j) & 1u) row_place(r, pat, wrap160(c + 16u * j));
}
__host__ __device__ __forceinline__ void playfield_row(Row160 &r, uint32_t pf) {
    const uint32_t m20 = pf_mask20(pf);
    const uint32_t right = ((pf >> 24) & 1u) ? (__builtin_bitreverse32(m20) >> 12) : m20;
    const uint64_t g40 = (uint64_t)m20 | ((uint64_t)right << 20);
#pragma unroll
    for (uint32_t k = 0; k < 5; ++k) r.w[k] = spread4((uint32_t)(g40 >> (8u * k)));
}
// rows of the five objects and the playfield for a TIA state
__host__ __device__ __forceinline__ void object_rows(Row160 (&r)[kRows], const Tia &t) {
#pragma unroll
    for (uint32_t o = 0; o < kRows; ++o)
#pragma unroll
        for (uint32_t i = 0; i < 5; ++i) r[o].w[i] = 0u;
    player_row(r[R_P0], t.ob, 0);
    player_row(r[R_P1], t.ob, 1);
    missile_row(r[R_M0], t.ob, 0);
    missile_row(r[R_M1], t.ob, 1);
    if (ball_on(t.ob)) row_place(r[R_BL], (1u << (1u << ((t.pf >> 28) & 3u))) - 1u, t.ob.bl & 0xFFu);
    playfield_row(r[R_PF], t.pf);
}
// owning colour register (0 COLUP0, 1 COLUP1, 2 COLUPF, 3 COLUBK) of column x
// whose occupancy has bit o set for each row o that shows there
__host__ __device__ __forceinline__ uint32_t owner_of(uint32_t occ, uint32_t x, uint32_t ctrl) {
    const bool pfb = (occ >> R_PF) & 1u, field = ((occ >> R_BL) & 3u) != 0u;
    const bool p0 = ((occ >> R_P0) | (occ >> R_M0)) & 1u, p1 = ((occ >> R_P1) | (occ >> R_M1)) & 1u;
    const uint32_t fo = (pfb && (ctrl & 2u)) ? (x < 80u ? 0u : 1u) : 2u;
    if (ctrl & 4u) return field ? fo : p0 ? 0u : p1 ? 1u : 3u;
    return p0 ? 0u : p1 ? 1u : field ? fo : 3u;
}
// occupancy nibbles of 4-pixel group g: bit j of nib[o] = row o at column 4g + j
__host__ __device__ __forceinline__ void group_occupancy(const Row160 (&r)[kRows], uint32_t g, uint32_t (&nib)[kRows]) {
    const uint32_t k = g >> 3, sh = 4u * (g & 7u);
#pragma unroll
    for (uint32_t o = 0; o < kRows; ++o) nib[o] = (row_word(r[o], k) >> sh) & 15u;
}
__host__ __device__ __forceinline__ uint32_t pixel_owner(const uint32_t (&nib)[kRows], uint32_t j, uint32_t x,
                                                        uint32_t ctrl) {
    uint32_t occ = 0;
#pragma unroll
    for (uint32_t o = 0; o < kRows; ++o) occ |= ((nib[o] >> j) & 1u) << o;
    return owner_of(occ, x, ctrl);
}
// the four colours of group g (column 4g in the low byte) with objects shown
__host__ __device__ __forceinline__ uint32_t group_colours(const Row160 (&r)[kRows], const Tia &t, uint32_t g) {
    uint32_t nib[kRows];
    group_occupancy(r, g, nib);
    uint32_t out = 0;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
        out |= ((t.col >> (8u * pixel_owner(nib, j, 4u * g + j, t.pf >> 24))) & 0xFEu) << (8u * j);
    return out;
}
// frame-relative line whose columns 0..7 an HMOVE blanked (-1: none)
__host__ __device__ __forceinline__ int32_t hmove_line(const Objs &o) { return (int32_t)(o.bl >> 8) - 1; }

// Latch into cx the collisions of frame-relative colour clocks [from, to) (0 <= from < to)
// drawn with state t.
__host__ __device__ inline __attribute__((noinline)) uint32_t collide_span(const Tia t, int32_t from, int32_t to) {
    uint32_t cx = 0;
    Row160 cov;
#pragma unroll
    for (uint32_t i = 0; i < 5; ++i) cov.w[i] = 0u;
    const int32_t hl = hmove_line(t.ob);
    for (int32_t c = from; c < to;) {  // the columns the span covers, on any of its lines
        const int32_t line = c / kClocksPerLine, l0 = line * kClocksPerLine;
        const int32_t e = to < l0 + kClocksPerLine ? to : l0 + kClocksPerLine;
        int32_t x0 = c - l0 - kHBlank;
        const int32_t x1 = e - l0 - kHBlank;
        x0 = x0 > 0 ? x0 : 0;
        if (line == hl && x0 < 8) x0 = 8;
        if (x1 > x0) {
#pragma unroll
            for (int32_t i = 0; i < 5; ++i) {
                const int32_t a = x0 > 32 * i ? x0 - 32 * i : 0, b = x1 < 32 * i + 32 ? x1 - 32 * i : 32;
                if (b > a) cov.w[i] |= (b - a == 32 ? ~0u : ((1u << (b - a)) - 1u)) << a;
            }
        }
        if ((cov.w[0] & cov.w[1] & cov.w[2] & cov.w[3] & cov.w[4]) == ~0u) break;
        c = e;
    }
    Row160 r[kRows];
    object_rows(r, t);
    constexpr uint8_t kPairs[16][2] = {{R_M0, R_P1}, {R_M0, R_P0}, {R_M1, R_P0}, {R_M1, R_P1}, {R_P0, R_PF},
                                       {R_P0, R_BL}, {R_P1, R_PF}, {R_P1, R_BL}, {R_M0, R_PF}, {R_M0, R_BL},
                                       {R_M1, R_PF}, {R_M1, R_BL}, {R_BL, R_PF}, {R_BL, R_BL}, {R_P0, R_P1},
                                       {R_M0, R_M1}};
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k) {
        if (k == 13) continue;  // CXBLPF bit 6: no pair
        uint32_t any = 0;
#pragma unroll
        for (uint32_t i = 0; i < 5; ++i) any |= r[kPairs[k][0]].w[i] & r[kPairs[k][1]].w[i] & cov.w[i];
        cx |= any ? 1u << k : 0u;
    }
    return cx;
}

// Write the pixels of frame-relative colour clocks [from, to) drawn with TIA
// state t into a frame of T, where objects show or an HMOVE blank lies in the
// frame.  With tan (soft frames), also the position sampler's tangents,
// tan[o][pixel] for o = P0, P1, M0, M1, BL: the colour with object o one column
// further right minus the colour drawn (0 where blanked) -- the derivative of a
// triangular (bilinear) sampler over the object's column at zero sub-pixel
// offset, taken from the right (Sec. "Hard and Soft Execution").
template <typename T>
__host__ __device__ __attribute__((noinline)) void render_span_objects(T *frame, int32_t from, int32_t to, const Tia t,
                                                                       int32_t ystart, uint32_t sub, uint32_t G,
                                                                       float *tan) {
    const uint32_t mask = pf_mask20(t.pf), ctrl = t.pf >> 24;
    const bool objs = objs_shown(t.ob);
    Row160 r[kRows];
    object_rows(r, t);
    const int32_t hl = hmove_line(t.ob) - ystart;  // visible row of an HMOVE blank
    for_each_group(from, to, ystart, sub, G, [&](int32_t y, int32_t g, int32_t xa, int32_t xb) {
        const bool blank = (t.vb & 2u) || (y == hl && g < 2);
        uint32_t c4;
        if (blank) c4 = 0u;
        else if (!objs) c4 = ((t.col >> (8 * group_owner((uint32_t)g, mask, ctrl))) & 0xFEu) * 0x01010101u;
        else c4 = group_colours(r, t, (uint32_t)g);
        T *row = frame + y * kScreenW;
        for (int32_t x = xa; x < xb; ++x) row[x] = (T)((c4 >> (8 * (x - 4 * g))) & 0xFFu);
        if (tan) {
            for (uint32_t o = 0; o < 5; ++o) {
                uint32_t m4 = c4;  // colours with object o one column further right
                if (!blank && objs) {
                    Row160 moved[kRows];
#pragma unroll
                    for (uint32_t q = 0; q < kRows; ++q) moved[q] = q == o ? row_shift1(r[q]) : r[q];
                    m4 = group_colours(moved, t, (uint32_t)g);
                }
                float *tr = tan + (size_t)o * kPixels + y * kScreenW;
                for (int32_t x = xa; x < xb; ++x) {
                    const int32_t sh = 8 * (x - 4 * g);
                    tr[x] = (float)((int32_t)((m4 >> sh) & 0xFFu) - (int32_t)((c4 >> sh) & 0xFFu));
                }
            }
        }
    });
}

// Write the pixels of [from, to) drawn with TIA state t into a frame of T (and
// with tan the sampler's tangents, see render_span_objects).
// Without the object paths (kObj false) no object shows and no HMOVE blank
// falls (the machine stops at the first write that could make either happen).
template <bool kObj = true, typename T>
__host__ __device__ __forceinline__ void render_span(T *frame, int32_t from, int32_t to, const Tia &t,
                                                     int32_t ystart, uint32_t sub, uint32_t G,
                                                     float *tan = nullptr) {
    if constexpr (kObj) {
        if (tan || hmove_line(t.ob) >= 0 || objs_shown(t.ob)) {
            render_span_objects(frame, from, to, t, ystart, sub, G, tan);
            return;
        }
    }
    const uint32_t mask = pf_mask20(t.pf), ctrl = t.pf >> 24;
    for_each_group(from, to, ystart, sub, G, [&](int32_t y, int32_t g, int32_t xa, int32_t xb) {
        const uint32_t c = (t.vb & 2u) ? 0u : ((t.col >> (8 * group_owner((uint32_t)g, mask, ctrl))) & 0xFEu);
        T *row = frame + y * kScreenW;
        if (xb - xa == 4) {
            if constexpr (sizeof(T) == 1) {
                *reinterpret_cast<uint32_t *>(row + xa) = c * 0x01010101u;
            } else {
                const float v = (float)c;
                *reinterpret_cast<float4 *>(row + xa) = make_float4(v, v, v, v);
            }
        } else {
            for (int32_t x = xa; x < xb; ++x) row[x] = (T)c;
        }
    });
}

// ---------------------------------------------------------------------------
// Data classes for the soft backward (where a value comes from / goes to)
// ---------------------------------------------------------------------------
struct ExecInfo {
    uint32_t op_cls, rd_cls, rd_idx, wr_cls, wr_idx, v1, v2, s_before;
};

// Class of a 13-bit data write target.
__host__ __device__ __forceinline__ uint32_t write_class(uint32_t addr, uint32_t *idx) {
    addr &= 0x1FFFu;
    *idx = 0;
    if (addr & 0x1000u) return kClsConst;
    if (!(addr & 0x80u)) {
        const uint32_t reg = addr & 0x3Fu;
        if (reg >= 6 && reg <= 9) {
            *idx = reg - 6;
            return kClsCol;
        }
        return kClsConst;
    }
    if (!(addr & 0x200u)) {
        *idx = addr & 0x7Fu;
        return kClsRam;
    }
    return kClsConst;
}

// ---------------------------------------------------------------------------
// The machine
// ---------------------------------------------------------------------------
// kObj: the machine with the object paths (collision latching, object pixels).
// Without them (the fast variant of the hard kernels) the machine holds no
// object state: obj_stop is raised when the loaded state shows an object, and
// at any write to a register only objects use (NUSIZ, REFP, the strobes, GRP,
// ENAM/ENABL, HMxx, VDEL, RESMP, HMOVE, HMCLR, CXCLR) or read of a collision
// latch.  Until then the object state stays as loaded, nothing shows and
// nothing collides, so the results are the machine's; from then on they are
// void, and the caller reruns the env with the object paths from its starting
// state.  The state record's object fields are left as loaded.
template <class Mem, class Hook, bool kObj = true>
struct Cpu {
    static constexpr bool kObjects = kObj;
    uint32_t a, x, y, s, p, pc, bank, jam;
    uint32_t rn, rz;              // N = bit 7 of rn, Z = (low byte of rz == 0); p holds the other flags
    int32_t cyc;                  // frame-relative CPU cycle
    uint32_t col, pf, vb;         // colour registers, playfield + CTRLPF, VBLANK | VSYNC << 8
    Objs ob;                      // TIA objects
    uint32_t hm;                  // motion nibbles: HMP0 | HMP1 << 4 | HMM0 << 8 | HMM1 << 12 | HMBL << 16
    uint32_t cx;                  // collision latches, bit k = pair k
    int32_t cx_cc;                // frame-relative colour clock up to which cx is current
    bool obj_stop;                // (without the object paths) an object showed
    bool ob_reset;                // (without the object paths) power-on cleared the object state
    const StateRec *ob_src;       // (without the object paths) the record whose object fields hold
    int32_t tim_u, tim_read;
    uint32_t tim_shift;
    uint32_t swcha, inpt4, swchb;
    uint32_t wsync;
    // cartridge format (set_cart): address mask, hotspot range of the 4 KB bank
    // switch, E0 slices (4 bits per quarter of the window), Superchip RAM
    uint32_t amask, hot_lo, hot_n, e0, slices, sc;
    uint32_t fetch_mask, fetch_lim;  // an instruction whose bytes lie in one bank/slice: (pc & mask) <= lim
    Mem mem;
    Hook hook;

    // Cartridge formats (Sec. "Building Two Differentiable VCS Ports": 2K, 4K, F8,
    // F6, F4, their Superchip variants, E0).  F8/F6/F4 select a 4 KB bank on a
    // data access to $1FF8-9 / $1FF6-9 / $1FF4-B; E0 maps 1 KB slices into the
    // window's first three quarters through $1FE0-7 / $1FE8-F / $1FF0-7 (the last
    // quarter is slice 7); Superchip formats add 128 bytes of RAM written at
    // $1000-$107F and read at $1080-$10FF (a read of the write port returns ROM).
    __host__ __device__ __forceinline__ void set_cart(int32_t mapper) {
        amask = mapper == kMapper2K ? 0x7FFu : 0xFFFu;
        const uint32_t nb = mapper_banks(mapper);
        hot_n = nb > 1 ? nb : 0u;
        hot_lo = nb == 2 ? 0x1FF8u : nb == 4 ? 0x1FF6u : 0x1FF4u;
        e0 = mapper == kMapperE0 ? 1u : 0u;
        sc = mapper_sc(mapper) ? 1u : 0u;
        fetch_mask = e0 ? 0x3FFu : 0xFFFu;
        fetch_lim = fetch_mask - 2u;
    }
    __host__ __device__ __forceinline__ uint32_t cart_off(uint32_t addr) const {
        const uint32_t banked = (addr & amask) + (bank << 12);
        const uint32_t sliced = (((slices >> (4u * ((addr >> 10) & 3u))) & 7u) << 10) | (addr & 0x3FFu);
        return e0 ? sliced : banked;
    }

    // processor status byte (B and U as stored in p)
    __host__ __device__ __forceinline__ uint32_t flags() const {
        return (p & ~(kFlagN | kFlagZ)) | (rn & kFlagN) | ((rz & 0xFFu) ? 0u : kFlagZ);
    }
    __host__ __device__ __forceinline__ void set_flags(uint32_t v) {
        p = v;
        rn = v & kFlagN;
        rz = (v & kFlagZ) ? 0u : 1u;
    }
    __host__ __device__ __forceinline__ void set_nz(uint32_t v) { rn = rz = v; }

    __host__ __device__ __forceinline__ uint32_t intim_at(int32_t t) const {
        const int32_t d = t - tim_u;
        return d < 0 ? ((uint32_t)(-1 - (d >> tim_shift)) & 0xFFu) : ((uint32_t)(255 - d) & 0xFFu);
    }
    __host__ __device__ __forceinline__ uint32_t timint_at(int32_t t) const {
        return (t >= tim_u && tim_read < tim_u) ? 0x80u : 0u;
    }
    __host__ __device__ __forceinline__ Tia tia() const {
        if constexpr (kObj) return Tia{col, pf, vb, ob};
        else return Tia{col, pf, vb, Objs{0u, 0u, 0u, 0u}};
    }
    // latch the collisions of the clocks before k
    __host__ __device__ __forceinline__ void cx_upto(int32_t k) {
        if constexpr (kObj) {
            if (k > cx_cc) {
                if (objs_shown(ob)) cx |= collide_span(tia(), cx_cc, k);
                cx_cc = k;
            }
        }
    }
    // TIA read in cycle t: collision latches (registers 0..7), INPT4, INPT5
    __host__ __device__ __forceinline__ uint32_t tia_in(uint32_t addr, int32_t t) {
        const uint32_t r = addr & 0xFu;
        if (r < 8u) {
            if constexpr (!kObj) {
                obj_stop = true;
                return 0u;
            }
            cx_upto(3 * t + 3);
            return (((cx >> (2u * r)) & 1u) << 7) | (((cx >> (2u * r + 1u)) & 1u) << 6);
        }
        return r == 0xCu ? inpt4 : (r == 0xDu ? 0x80u : 0u);
    }
    __host__ __device__ __forceinline__ uint32_t riot_in(uint32_t addr, int32_t t, bool fx) {
        if (!(addr & 4u)) {
            const uint32_t r = addr & 3u;
            return r == 0 ? swcha : (r == 2 ? swchb : 0u);
        }
        if (!(addr & 1u)) {
            const uint32_t v = intim_at(t);
            if (fx) tim_read = t;
            return v;
        }
        return timint_at(t);
    }
    // fetch-type read: no side effects
    __host__ __device__ __forceinline__ uint32_t peek(uint32_t addr, int32_t t) {
        addr &= 0x1FFFu;
        if (sc && (addr & 0x1F80u) == 0x1080u) return mem.sc_byte(addr & 0x7Fu);
        if (addr & 0x1000u) return mem.rom_byte(cart_off(addr));
        if (!(addr & 0x80u)) return tia_in(addr, t);
        if (!(addr & 0x200u)) return mem.ram_byte(addr & 0x7Fu);
        return riot_in(addr, t, false);
    }
    __host__ __device__ __forceinline__ void hotspot(uint32_t addr) {
        if (addr - hot_lo < hot_n) bank = addr - hot_lo;
        if (e0 && addr - 0x1FE0u < 24u) {
            const uint32_t sh = 4u * ((addr - 0x1FE0u) >> 3);
            slices = (slices & ~(0xFu << sh)) | ((addr & 7u) << sh);
        }
    }
    // data read in cycle t
    __host__ __device__ __forceinline__ uint32_t read(uint32_t addr, int32_t t) {
        addr &= 0x1FFFu;
        if (sc && (addr & 0x1F80u) == 0x1080u) return mem.sc_byte(addr & 0x7Fu);
        if (addr & 0x1000u) {
            hotspot(addr);
            return mem.rom_byte(cart_off(addr));
        }
        if (!(addr & 0x80u)) return tia_in(addr, t);
        if (!(addr & 0x200u)) return mem.ram_byte(addr & 0x7Fu);
        return riot_in(addr, t, true);
    }
    // Page 0 and the stack page decode alike (A12 = A9 = 0): TIA below $80,
    // RAM from $80.  These are read/write for such addresses (zero-page modes,
    // zero-page pointers, the stack at $100 | s), with the page bits dropped;
    // t is the cycle of the read.
    __host__ __device__ __forceinline__ uint32_t read_zp(uint32_t a8, int32_t t) {
        if (a8 & 0x80u) return mem.ram_byte(a8 & 0x7Fu);
        return tia_in(a8, t);
    }
    __host__ __device__ __forceinline__ void write_zp(uint32_t a8, uint32_t v, int32_t w) {
        if (a8 & 0x80u) mem.ram_set(a8 & 0x7Fu, v);
        else tia_out(a8 & 0x3Fu, v, w);
    }
    // class of the value a data read at addr returned (after its side effects)
    __host__ __device__ __forceinline__ uint32_t read_class(uint32_t addr, uint32_t *idx) const {
        addr &= 0x1FFFu;
        *idx = 0;
        if (addr & 0x1000u) {
            *idx = cart_off(addr);
            return kClsRom;
        }
        if (!(addr & 0x80u)) return (addr & 0xFu) == 0xCu ? kClsInpt4 : kClsConst;
        if (!(addr & 0x200u)) {
            *idx = addr & 0x7Fu;
            return kClsRam;
        }
        return (!(addr & 4u) && !(addr & 3u)) ? kClsSwcha : kClsConst;
    }
    // a write in cycle w to a register that changes what objects or the playfield
    // show: pixels and collisions before its effect clock keep the old state
    __host__ __device__ __forceinline__ void before_object_write(int32_t w) {
        hook.before_pixel_write(*this, w);
        cx_upto(3 * (w + 1));
    }
    __host__ __device__ __forceinline__ void set_ctl(uint32_t flag, bool on) { ob.ctl = on ? (ob.ctl | flag) : (ob.ctl & ~flag); }
    __host__ __device__ __forceinline__ void set_pos(uint32_t o, uint32_t c) {  // o = 0..3: P0, P1, M0, M1
        ob.pos = (ob.pos & ~(0xFFu << (8u * o))) | (c << (8u * o));
    }
    __host__ __device__ __forceinline__ void tia_out(uint32_t reg, uint32_t v, int32_t w) {
        if constexpr (!kObj) {
            switch (reg) {
                case 0x00: vb = (vb & 0xFFu) | (v << 8); break;
                case 0x01: hook.before_pixel_write(*this, w); vb = (vb & 0xFF00u) | v; break;
                case 0x02: wsync = 1; break;
                case 0x06: case 0x07: case 0x08: case 0x09: {
                    hook.before_pixel_write(*this, w);
                    const uint32_t sh = (reg - 6u) * 8u;
                    col = (col & ~(0xFFu << sh)) | (v << sh);
                    break;
                }
                case 0x0A: hook.before_pixel_write(*this, w); pf = (pf & 0x00FFFFFFu) | (v << 24); break;
                case 0x0D: case 0x0E: case 0x0F: {
                    hook.before_pixel_write(*this, w);
                    const uint32_t sh = (reg - 0x0Du) * 8u;
                    pf = (pf & ~(0xFFu << sh)) | (v << sh);
                    break;
                }
                case 0x03: case 0x15: case 0x16: case 0x17: case 0x18: case 0x19: case 0x1A: break;  // RSYNC, audio
                default: obj_stop = obj_stop || reg <= 0x2Cu; break;  // the object registers; unused above
            }
            return;
        }
        // registers that change what objects or the playfield show: NUSIZ0/1,
        // CTRLPF, REFP0/1, PF0-2, the strobes, GRP0/1, ENAM0/1, ENABL, VDELP0/1,
        // VDELBL, RESMP0/1, HMOVE
        constexpr uint64_t kObjRegs = (3ull << 0x04) | (7ull << 0x0A) | (7ull << 0x0D) | (0x1Full << 0x10) |
                                      (0x1Full << 0x1B) | (0x1Full << 0x25) | (1ull << 0x2A);
        const bool obj_reg = (kObjRegs >> reg) & 1u;
        if (obj_reg) before_object_write(w);
        switch (reg) {
            case 0x00: vb = (vb & 0xFFu) | (v << 8); break;
            case 0x01: hook.before_pixel_write(*this, w); vb = (vb & 0xFF00u) | v; break;
            case 0x02: wsync = 1; break;
            case 0x04: case 0x05: {  // NUSIZ0/1
                const uint32_t sh = (reg - 4u) * 8u;
                ob.ctl = (ob.ctl & ~(0xFFu << sh)) | (v << sh);
                break;
            }
            case 0x06: case 0x07: case 0x08: case 0x09: {
                hook.before_pixel_write(*this, w);
                const uint32_t sh = (reg - 6u) * 8u;
                col = (col & ~(0xFFu << sh)) | (v << sh);
                break;
            }
            case 0x0A: pf = (pf & 0x00FFFFFFu) | (v << 24); break;
            case 0x0B: set_ctl(kObRefp0, v & 8u); break;
            case 0x0C: set_ctl(kObRefp1, v & 8u); break;
            case 0x0D: case 0x0E: case 0x0F: {
                const uint32_t sh = (reg - 0x0Du) * 8u;
                pf = (pf & ~(0xFFu << sh)) | (v << sh);
                break;
            }
            case 0x10: case 0x11: set_pos(reg - 0x10u, strobe_column(3 * (w + 1), 5u)); break;
            case 0x12: case 0x13: set_pos(reg - 0x10u, strobe_column(3 * (w + 1), 4u)); break;
            case 0x14: ob.bl = (ob.bl & ~0xFFu) | strobe_column(3 * (w + 1), 4u); break;
            case 0x1B:  // GRP0; GRP1's old register takes GRP1
                ob.gfx = (ob.gfx & 0x00FFFF00u) | v | ((ob.gfx & 0xFF00u) << 16);
                break;
            case 0x1C:  // GRP1; GRP0's and ENABL's old registers take theirs
                ob.gfx = (ob.gfx & 0xFF0000FFu) | (v << 8) | ((ob.gfx & 0xFFu) << 16);
                set_ctl(kObEnablOld, ob.ctl & kObEnabl);
                break;
            case 0x1D: set_ctl(kObEnam0, v & 2u); break;
            case 0x1E: set_ctl(kObEnam1, v & 2u); break;
            case 0x1F: set_ctl(kObEnabl, v & 2u); break;
            case 0x20: case 0x21: case 0x22: case 0x23: case 0x24: {  // HMP0 .. HMBL: no effect until HMOVE
                const uint32_t sh = (reg - 0x20u) * 4u;
                hm = (hm & ~(0xFu << sh)) | ((v >> 4) << sh);
                break;
            }
            case 0x25: set_ctl(kObVdelp0, v & 1u); break;
            case 0x26: set_ctl(kObVdelp1, v & 1u); break;
            case 0x27: set_ctl(kObVdelbl, v & 1u); break;
            case 0x28: case 0x29: {  // RESMP0/1: on release the missile moves to its player's centre
                const uint32_t i = reg - 0x28u, flag = i ? kObResmp1 : kObResmp0;
                if ((ob.ctl & flag) && !(v & 2u)) {
                    const uint32_t p = (ob.pos >> (8u * i)) & 0xFFu;
                    set_pos(2u + i, wrap160(p + (4u << player_shift(ob.ctl >> (8u * i)))));
                }
                set_ctl(flag, v & 2u);
                break;
            }
            case 0x2A: {  // HMOVE
                uint32_t np = 0;
#pragma unroll
                for (uint32_t o = 0; o < 5; ++o) {
                    const int32_t m = (int32_t)(hm << (28u - 4u * o)) >> 28;  // signed nibble
                    const uint32_t c = o < 4 ? (ob.pos >> (8u * o)) & 0xFFu : ob.bl & 0xFFu;
                    uint32_t q = (uint32_t)((int32_t)c + 160 - m);  // 153..327
                    q = q >= 320u ? q - 320u : q >= 160u ? q - 160u : q;
                    if (o < 4) np |= q << (8u * o);
                    else ob.bl = (ob.bl & ~0xFFu) | q;
                }
                ob.pos = np;
                const int32_t cc = 3 * (w + 1);
                if (cc % kClocksPerLine < kHBlank) ob.bl = (ob.bl & 0xFFu) | ((uint32_t)(cc / kClocksPerLine + 1) << 8);
                break;
            }
            case 0x2B: hm = 0; break;  // HMCLR
            case 0x2C: cx_upto(3 * (w + 1)); cx = 0; break;  // CXCLR
            default: break;  // audio, RSYNC and the unused addresses
        }
    }
    // data write in cycle w
    __host__ __device__ __forceinline__ void write(uint32_t addr, uint32_t v, int32_t w) {
        addr &= 0x1FFFu;
        if (sc && (addr & 0x1F80u) == 0x1000u) {
            mem.sc_set(addr & 0x7Fu, v);
            return;
        }
        if (addr & 0x1000u) {
            hotspot(addr);
            return;
        }
        if (!(addr & 0x80u)) {
            tia_out(addr & 0x3Fu, v, w);
            return;
        }
        if (!(addr & 0x200u)) {
            mem.ram_set(addr & 0x7Fu, v);
            return;
        }
        if ((addr & 0x14u) == 0x14u) {  // TIM1T / TIM8T / TIM64T / T1024T
            const uint32_t k = addr & 3u;
            const uint32_t sh = k == 0 ? 0u : k == 1 ? 3u : k == 2 ? 6u : 10u;
            tim_shift = sh;
            tim_u = w + 1 + (int32_t)(v << sh);
        }
    }
    __host__ __device__ __forceinline__ void push(uint32_t v, int32_t w) {
        write_zp(s, v, w);
        s = (s - 1u) & 0xFFu;
    }
    __host__ __device__ __forceinline__ uint32_t pull(int32_t t) {
        s = (s + 1u) & 0xFFu;
        return read_zp(s, t);
    }

    // NMOS ADC, binary and decimal (decimal: B. Clark, "Decimal Mode", App. A).
    // Both results are formed and D selects, so no lane branches on D.
    __host__ __device__ __forceinline__ uint32_t adc(uint32_t v) {
        const uint32_t c = p & kFlagC;
        const uint32_t sum = a + v + c;
        const uint32_t fb = ((~(a ^ v) & (a ^ sum) & 0x80u) ? kFlagV : 0u) | (sum > 0xFFu ? kFlagC : 0u);
        int32_t lo = (int32_t)((a & 0xFu) + (v & 0xFu) + c);
        lo = lo > 9 ? ((lo + 6) & 0xF) + 0x10 : lo;
        const int32_t hi_s = ((int32_t)((a & 0xF0u) ^ 0x80u) - 128) + ((int32_t)((v & 0xF0u) ^ 0x80u) - 128) + lo;
        int32_t hi_u = (int32_t)(a & 0xF0u) + (int32_t)(v & 0xF0u) + lo;
        hi_u = hi_u >= 0xA0 ? hi_u + 0x60 : hi_u;
        const uint32_t fd = ((hi_s < -128 || hi_s > 127) ? kFlagV : 0u) | (hi_u > 0xFF ? kFlagC : 0u);
        const bool dec = (p & kFlagD) != 0u;
        p = (p & ~(kFlagV | kFlagC)) | (dec ? fd : fb);
        rz = sum & 0xFFu;                              // Z from the binary sum in both modes
        rn = dec ? ((uint32_t)hi_s & 0x80u) : (sum & 0xFFu);  // decimal N from the signed high-digit sum
        return dec ? ((uint32_t)hi_u & 0xFFu) : (sum & 0xFFu);
    }
    __host__ __device__ __forceinline__ uint32_t sbc(uint32_t v) {
        const uint32_t c = p & kFlagC;
        const int32_t diff = (int32_t)a - (int32_t)v - (int32_t)(1u - c);
        const uint32_t bin = (uint32_t)diff & 0xFFu;
        p = (p & ~(kFlagV | kFlagC)) | (((a ^ v) & (a ^ bin) & 0x80u) ? kFlagV : 0u) | (diff >= 0 ? kFlagC : 0u);
        set_nz(bin);  // flags follow the binary difference in both modes
        int32_t lo = (int32_t)(a & 0xFu) - (int32_t)(v & 0xFu) - (int32_t)(1u - c);
        lo = lo < 0 ? ((lo - 6) & 0xF) - 0x10 : lo;
        int32_t r = (int32_t)(a & 0xF0u) - (int32_t)(v & 0xF0u) + lo;
        r = r < 0 ? r - 0x60 : r;
        return (p & kFlagD) ? ((uint32_t)r & 0xFFu) : bin;
    }

    // Execute one instruction whose opcode byte is opc (decode entry d) with
    // operand bytes lo/hi; `info` receives the data classes when recording.
    // On the GPU opc and d are the same in every lane that runs this call, so
    // every test of the mode or class is a wave-uniform branch.  Instructions
    // with one data access run in phases (address, read, operate, write) in
    // which only the read and the write decode addresses per lane; the
    // operate phase has no per-lane branch, so its class switch stays a
    // scalar branch tree.  JSR, RTS, RTI, BRK and JMP (ind) take a separate path.
    __host__ __device__ __forceinline__ void exec(uint32_t opc, uint32_t d, uint32_t lo, uint32_t hi, ExecInfo &info) {
        int32_t t0, n;
        uint32_t ea, r;
        const bool wr = exec_body<false>(opc, d, lo, hi, info, t0, n, ea, r);
        finish(opc, info, t0, n, wr);
    }

    // End of an instruction that started at cycle t0 and took n cycles: the cycle
    // counter, the hook, and the WSYNC stall of an instruction that wrote memory.
    // (wr is the same in every lane; the stall itself is a select, so no lane branches)
    __host__ __device__ __forceinline__ void finish(uint32_t opc, ExecInfo &info, int32_t t0, int32_t n, bool wr) {
        cyc = t0 + n;
        hook.after_exec(*this, opc, t0, cyc, info);
        if (wr) {
            const int32_t q = cyc % kCyclesPerLine;
            cyc = (wsync && q) ? cyc + (kCyclesPerLine - q) : cyc;
            wsync = 0;
        }
    }

    // The instruction up to (kDefer) or including its memory write; returns whether it
    // writes memory.  With kDefer the write (page 0 or stack, at ea with value r, in
    // the last cycle) is left to the caller, which then calls finish().
    template <bool kDefer>
    __host__ __device__ __forceinline__ bool exec_body(uint32_t opc, uint32_t d, uint32_t lo, uint32_t hi,
                                                       ExecInfo &info, int32_t &t0_out, int32_t &n_out,
                                                       uint32_t &ea_out, uint32_t &r_out) {
        constexpr bool R = Hook::kRecord;
        ea_out = r_out = 0;
        (void)opc;
        const uint32_t cls = d & 63u, mode = (d >> 6) & 15u;
        const int32_t t0 = cyc;
        int32_t n = (int32_t)((d >> 10) & 7u);
        const uint32_t pc0 = pc;
        pc = (pc0 + ((d >> 14) & 3u)) & 0xFFFFu;
        if constexpr (R) {
            info.op_cls = cls;
            info.rd_cls = kClsConst;
            info.wr_cls = kClsConst;
            info.rd_idx = info.wr_idx = info.v1 = info.v2 = 0;
            info.s_before = s;
        }
        hook.before_exec(*this);
        const bool multi = cls == C_JSR || cls == C_RTS || cls == C_RTI || cls == C_BRK || mode == M_IND;
        bool wr;  // the instruction writes memory (so it may have written WSYNC)
        if (multi) {
            wr = cls == C_JSR || cls == C_BRK;
            exec_multi(cls, mode, pc0, lo, hi, t0, n);
        } else {
            const bool stack = cls >= C_PHA && cls <= C_PLP;
            const bool zpt = mode == M_ZP || mode == M_ZPX || mode == M_ZPY || stack;  // page-0 / stack access
            const bool load = (cls >= C_LDA && cls <= C_LAX) || (cls >= C_ADC && cls <= C_BIT);
            const bool rmw = cls >= C_ASL && cls <= C_DEC;
            const bool store = cls >= C_STA && cls <= C_SAX;
            const bool rd = (load && mode != M_IMM) || (rmw && mode != M_ACC) || cls == C_PLA || cls == C_PLP;
            wr = store || (rmw && mode != M_ACC) || cls == C_PHA || cls == C_PHP;

            // ---- address
            uint32_t ea = 0;
            switch (mode) {
                case M_IMM: ea = (pc0 + 1u) & 0xFFFFu; break;
                case M_ZP: ea = lo; break;
                case M_ZPX: ea = (lo + x) & 0xFFu; break;
                case M_ZPY: ea = (lo + y) & 0xFFu; break;
                case M_ABS: ea = lo | (hi << 8); break;
                case M_ABX:
                case M_ABY: {
                    const uint32_t base = lo | (hi << 8);
                    ea = (base + (mode == M_ABX ? x : y)) & 0xFFFFu;
                    if ((d >> 13) & 1u) n += ((base ^ ea) >> 8) != 0u ? 1 : 0;
                    break;
                }
                case M_IZX: {
                    const uint32_t z = (lo + x) & 0xFFu;
                    ea = read_zp(z, t0) | (read_zp((z + 1u) & 0xFFu, t0) << 8);
                    break;
                }
                case M_IZY: {
                    const uint32_t base = read_zp(lo, t0) | (read_zp((lo + 1u) & 0xFFu, t0) << 8);
                    ea = (base + y) & 0xFFFFu;
                    if ((d >> 13) & 1u) n += ((base ^ ea) >> 8) != 0u ? 1 : 0;
                    break;
                }
                default: break;
            }
            if (cls == C_PHA || cls == C_PHP) ea = s;                    // push to $100 | s
            else if (cls == C_PLA || cls == C_PLP) ea = (s + 1u) & 0xFFu;  // pull from $100 | s+1
            const int32_t tl = t0 + n - 1;  // last cycle: loads and stores access memory here

            // ---- read (a read-modify-write reads three cycles before its end)
            uint32_t v = lo;
            if (rd) {
                if (zpt) v = read_zp(ea, rmw ? t0 + n - 3 : tl);
                else v = read(ea, rmw ? t0 + n - 3 : tl);
            }
            if constexpr (R) {
                if (load) {
                    info.rd_cls = read_class(ea, &info.rd_idx);  // an immediate is a ROM byte
                } else if (rmw) {
                    if (mode == M_ACC) {
                        info.rd_cls = info.wr_cls = kClsRegA;
                    } else {
                        info.rd_cls = read_class(ea, &info.rd_idx);
                        info.wr_cls = write_class(ea, &info.wr_idx);
                    }
                } else if (store) {
                    info.wr_cls = write_class(ea, &info.wr_idx);
                    info.v1 = a;
                    info.v2 = x;
                } else if (cls == C_PHA) {
                    info.wr_cls = write_class(0x100u | ea, &info.wr_idx);
                } else if (cls == C_PLA) {
                    info.rd_cls = read_class(0x100u | ea, &info.rd_idx);
                }
            }

            // ---- operate
            uint32_t r = 0;  // value to write
            switch (cls) {
                case C_LDA: a = v; set_nz(v); break;
                case C_LDX: x = v; set_nz(v); break;
                case C_LDY: y = v; set_nz(v); break;
                case C_LAX: a = x = v; set_nz(v); break;
                case C_ADC: a = adc(v); break;
                case C_SBC: a = sbc(v); break;
                case C_AND: case C_ORA: case C_EOR:
                    if constexpr (R) {
                        info.v1 = a;
                        info.v2 = v;
                    }
                    a = cls == C_AND ? (a & v) : cls == C_ORA ? (a | v) : (a ^ v);
                    set_nz(a);
                    break;
                case C_BIT:
                    p = (p & ~kFlagV) | (v & kFlagV);
                    rn = v;
                    rz = a & v;
                    break;
                case C_CMP: case C_CPX: case C_CPY: {
                    const uint32_t q = cls == C_CMP ? a : cls == C_CPX ? x : y;
                    p = (p & ~kFlagC) | (q >= v ? kFlagC : 0u);
                    set_nz((q - v) & 0xFFu);
                    break;
                }
                case C_STA: r = a; break;
                case C_STX: r = x; break;
                case C_STY: r = y; break;
                case C_SAX: r = a & x; break;
                case C_ASL: case C_LSR: case C_ROL: case C_ROR: case C_INC: case C_DEC: {
                    const uint32_t src = mode == M_ACC ? a : v;
                    const uint32_t c = p & kFlagC;
                    switch (cls) {
                        case C_ASL: p = (p & ~kFlagC) | (src >> 7); r = (src << 1) & 0xFFu; break;
                        case C_LSR: p = (p & ~kFlagC) | (src & 1u); r = src >> 1; break;
                        case C_ROL: p = (p & ~kFlagC) | (src >> 7); r = ((src << 1) | c) & 0xFFu; break;
                        case C_ROR: p = (p & ~kFlagC) | (src & 1u); r = (src >> 1) | (c << 7); break;
                        case C_INC: r = (src + 1u) & 0xFFu; break;
                        default: r = (src - 1u) & 0xFFu; break;
                    }
                    set_nz(r);
                    if (mode == M_ACC) a = r;
                    break;
                }
                case C_INX: x = (x + 1u) & 0xFFu; set_nz(x); break;
                case C_INY: y = (y + 1u) & 0xFFu; set_nz(y); break;
                case C_DEX: x = (x - 1u) & 0xFFu; set_nz(x); break;
                case C_DEY: y = (y - 1u) & 0xFFu; set_nz(y); break;
                case C_TAX: x = a; set_nz(x); break;
                case C_TAY: y = a; set_nz(y); break;
                case C_TXA: a = x; set_nz(a); break;
                case C_TYA: a = y; set_nz(a); break;
                case C_TSX: x = s; set_nz(x); break;
                case C_TXS: s = x; break;
                case C_PHA: r = a; s = (s - 1u) & 0xFFu; break;
                case C_PHP: r = flags() | kFlagB | kFlagU; s = (s - 1u) & 0xFFu; break;
                case C_PLA: a = v; set_nz(v); s = ea; break;
                case C_PLP: set_flags((v & ~kFlagB) | kFlagU); s = ea; break;
                case C_JMP: pc = ea; break;
                case C_BRANCH: {
                    const uint32_t mask = (d >> 16) & 0xFFu, when_set = (d >> 24) & 1u;
                    const uint32_t f = mask == kFlagN ? (rn >> 7) & 1u
                                     : mask == kFlagZ ? ((rz & 0xFFu) ? 0u : 1u) : ((p & mask) ? 1u : 0u);
                    const bool taken = f == when_set;
                    uint32_t target = (pc + (uint32_t)(int32_t)(int8_t)lo) & 0xFFFFu;
                    if constexpr (Mem::kRelax) target = mem.branch(pc, lo, taken);  // relaxed and cast
                    n += taken ? 1 + (((target ^ pc) & 0xFF00u) ? 1 : 0) : 0;
                    pc = (taken || Mem::kRelax) ? target : pc;
                    break;
                }
                case C_FLAG: {
                    const uint32_t mask = (d >> 16) & 0xFFu;
                    p = ((d >> 24) & 1u) ? (p | mask) : (p & ~mask);
                    break;
                }
                default: break;  // NOP family (operand reads have no side effects)
            }

            // ---- write
            if constexpr (kDefer) {
                ea_out = ea;
                r_out = r;
            } else if (wr) {
                if (zpt) write_zp(ea, r, tl);
                else write(ea, r, tl);
            }
        }
        t0_out = t0;
        n_out = n;
        return wr;
    }

    // JSR, RTS, RTI, BRK (several stack accesses, all in the last cycle) and JMP (ind).
    __host__ __device__ __forceinline__ void exec_multi(uint32_t cls, uint32_t mode, uint32_t pc0, uint32_t lo,
                                                        uint32_t hi, int32_t t0, int32_t n) {
        const int32_t tl = t0 + n - 1;
        switch (cls) {
            case C_JMP: {  // (ind): the pointer's high byte comes from the same page
                const uint32_t ptr = lo | (hi << 8);
                const uint32_t ptr_hi = (ptr & 0xFF00u) | ((ptr + 1u) & 0xFFu);
                pc = peek(ptr, t0) | (peek(ptr_hi, t0) << 8);
                break;
            }
            case C_JSR: {
                const uint32_t ret = (pc - 1u) & 0xFFFFu;
                push(ret >> 8, tl);
                push(ret & 0xFFu, tl);
                pc = lo | (hi << 8);
                break;
            }
            case C_RTS: {
                const uint32_t l = pull(tl);
                const uint32_t h = pull(tl);
                pc = (((h << 8) | l) + 1u) & 0xFFFFu;
                break;
            }
            case C_BRK: {
                const uint32_t ret = (pc0 + 2u) & 0xFFFFu;
                push(ret >> 8, tl);
                push(ret & 0xFFu, tl);
                push(flags() | kFlagB | kFlagU, tl);
                p |= kFlagI;
                pc = peek(0x1FFEu, t0) | (peek(0x1FFFu, t0) << 8);
                break;
            }
            default: {  // RTI
                set_flags((pull(tl) & ~kFlagB) | kFlagU);
                const uint32_t l = pull(tl);
                const uint32_t h = pull(tl);
                pc = (h << 8) | l;
                break;
            }
        }
        (void)mode;
    }

    // Power-on (also the in-run reset): registers, TIA and timer to their
    // power-on values, PC from the reset vector of the power-on bank.
    __host__ __device__ __forceinline__ void power_on() {
        a = x = y = 0;
        s = 0xFDu;
        set_flags(kFlagI | kFlagU);
        bank = hot_n == 2u ? 1u : 0u;            // F8 (and F8SC) start in bank 1, F6/F4 in bank 0
        slices = 4u | (5u << 4) | (6u << 8) | (7u << 12);  // E0: slices 4, 5, 6 and the fixed 7
        jam = 0;
        cyc = 0;
        col = pf = vb = 0;
        ob = Objs{0u, 0u, 0u, 0u};
        hm = cx = 0;
        cx_cc = 0;
        obj_stop = false;
        ob_reset = true;
        ob_src = nullptr;
        tim_u = 0;
        tim_read = 0;
        tim_shift = 10;
        wsync = 0;
        pc = peek(0x1FFCu, 0) | (peek(0x1FFDu, 0) << 8);
    }

    // Frame rollover: cycle counters become relative to the next frame.  Long
    // underflowed timers are renormalised by multiples of 256 cycles, which
    // changes no observable value.
    __host__ __device__ __forceinline__ void next_frame() {
        if constexpr (kObj) {
            cx_upto(3 * cyc);  // the frame's remaining collisions (and those of cycles past its end)
            cx_cc -= kClocksPerFrame;
            const int32_t hl = hmove_line(ob) - kLinesPerFrame;
            ob.bl = (ob.bl & 0xFFu) | (hl >= 0 ? (uint32_t)(hl + 1) << 8 : 0u);
        }
        cyc -= kCyclesPerFrame;
        tim_u -= kCyclesPerFrame;
        tim_read -= kCyclesPerFrame;
        if (tim_read < tim_u - (1 << 20)) tim_read = tim_u - (1 << 20);
        if (tim_u < -(1 << 24)) {
            tim_u += 1 << 24;
            tim_read += 1 << 24;
        }
    }

    __host__ __device__ __forceinline__ void load(const StateRec &r) {
        a = r.a; x = r.x; y = r.y; s = r.s; set_flags(r.p); pc = r.pc; jam = r.status & 1u;
        bank = hot_n ? (r.bank < hot_n ? r.bank : 0u) : 0u;  // only the banked formats have banks
        slices = r.slices;
        cyc = r.cyc; col = r.col; pf = r.pf; vb = r.vblank | ((uint32_t)r.vsync << 8);
        tim_u = r.tim_u; tim_read = r.tim_read; tim_shift = r.tim_shift; wsync = 0;
        if constexpr (kObj) {
            ob = Objs{r.ob_pos, r.ob_gfx, r.ob_ctl, r.ob_bl};
            hm = r.ob_hm; cx = r.cx; cx_cc = r.cx_cc;
            obj_stop = false;
        } else {
            obj_stop = objs_shown(Objs{r.ob_pos, r.ob_gfx, r.ob_ctl, r.ob_bl}) || hmove_line(Objs{0u, 0u, 0u, r.ob_bl}) >= 0;
            ob_reset = false;
            ob_src = &r;
        }
    }
    __host__ __device__ __forceinline__ void store(StateRec &r) const {
        r.magic = kMagic;
        r.a = (uint8_t)a; r.x = (uint8_t)x; r.y = (uint8_t)y; r.s = (uint8_t)s; r.p = (uint8_t)flags();
        r.pc = (uint16_t)pc; r.bank = (uint8_t)bank; r.status = (uint8_t)(jam & 1u); r.slices = (uint16_t)slices;
        r.cyc = cyc; r.col = col; r.pf = pf; r.vblank = (uint8_t)(vb & 0xFFu); r.vsync = (uint8_t)(vb >> 8);
        r.tim_u = tim_u; r.tim_read = tim_read; r.tim_shift = (uint8_t)tim_shift;
        if constexpr (kObj) {
            r.ob_pos = ob.pos; r.ob_gfx = ob.gfx; r.ob_ctl = ob.ctl; r.ob_bl = ob.bl;
            r.ob_hm = hm; r.cx = cx; r.cx_cc = cx_cc;
        } else {  // the object fields as loaded (or cleared by a power-on); nothing collided up to now
            if (ob_reset || !ob_src) {
                r.ob_pos = r.ob_gfx = r.ob_ctl = r.ob_bl = 0u;
                r.ob_hm = r.cx = 0u;
            } else if (ob_src != &r) {
                r.ob_pos = ob_src->ob_pos; r.ob_gfx = ob_src->ob_gfx; r.ob_ctl = ob_src->ob_ctl;
                r.ob_bl = ob_src->ob_bl; r.ob_hm = ob_src->ob_hm; r.cx = ob_src->cx;
            }
            r.cx_cc = 3 * cyc;
        }
    }
};

// The object registers of a state record in the vcs_read_objects layout.
__host__ __device__ __forceinline__ void objects32(const StateRec &r, uint8_t o[32]) {
    const uint32_t c = r.ob_ctl;
    for (int i = 0; i < 4; ++i) o[i] = (uint8_t)(r.ob_pos >> (8 * i));
    o[4] = (uint8_t)r.ob_bl;
    for (int i = 0; i < 4; ++i) o[5 + i] = (uint8_t)(r.ob_gfx >> (8 * i));
    o[9] = (c & kObEnam0) ? 2 : 0;
    o[10] = (c & kObEnam1) ? 2 : 0;
    o[11] = (c & kObEnabl) ? 2 : 0;
    o[12] = (c & kObEnablOld) ? 2 : 0;
    o[13] = (uint8_t)c;
    o[14] = (uint8_t)(c >> 8);
    o[15] = (c & kObRefp0) ? 8 : 0;
    o[16] = (c & kObRefp1) ? 8 : 0;
    o[17] = (c & kObVdelp0) ? 1 : 0;
    o[18] = (c & kObVdelp1) ? 1 : 0;
    o[19] = (c & kObVdelbl) ? 1 : 0;
    o[20] = (c & kObResmp0) ? 2 : 0;
    o[21] = (c & kObResmp1) ? 2 : 0;
    for (int i = 0; i < 5; ++i) o[22 + i] = (uint8_t)(((r.ob_hm >> (4 * i)) & 0xFu) << 4);
    o[27] = (uint8_t)r.cx;
    o[28] = (uint8_t)(r.cx >> 8);
    o[29] = o[30] = o[31] = 0;
}

// ALE joystick action -> port values (SWCHA, INPT4).  Actions 0..17: NOOP FIRE
// UP RIGHT LEFT DOWN UPRIGHT UPLEFT DOWNRIGHT DOWNLEFT UPFIRE RIGHTFIRE LEFTFIRE
// DOWNFIRE UPRIGHTFIRE UPLEFTFIRE DOWNRIGHTFIRE DOWNLEFTFIRE; SWCHA bits 7/6/5/4
// (right/left/down/up) are cleared while held, INPT4 bit 7 clears on fire.
__host__ __device__ __forceinline__ void action_ports(uint32_t action, uint32_t *swcha, uint32_t *inpt4,
                                                      uint32_t *swchb = nullptr) {
    // action 18: the console RESET switch held (SWCHB bit 0 low), joystick idle
    if (swchb) *swchb = action == kActionReset ? 0x0Au : 0x0Bu;
    // direction bits per action: up 1, down 2, left 4, right 8, fire 16
    constexpr uint8_t dirs[18] = {0, 16, 1, 8, 4, 2, 9, 5, 10, 6, 17, 24, 20, 18, 25, 21, 26, 22};
    const uint32_t dm = action < 18 ? dirs[action] : 0u;
    uint32_t v = 0xFFu;
    if (dm & 8u) v &= ~0x80u;
    if (dm & 4u) v &= ~0x40u;
    if (dm & 2u) v &= ~0x20u;
    if (dm & 1u) v &= ~0x10u;
    *swcha = v;
    *inpt4 = (dm & 16u) ? 0x00u : 0x80u;
}

}  // namespace vcs
