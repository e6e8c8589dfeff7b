// Per-env bodies of libvcs's kernels (memory policies, hooks, the step loop
// and the soft backward), written for one env per lane or lane group.  They are
// host/device templates over a wave policy W so that the wave-level
// operations (ballot, readfirstlane) stay in the kernels.
#pragma once

#include <type_traits>

#include "vcs_core.hpp"

namespace vcs {

// ---------------------------------------------------------------------------
// Memory policies
// ---------------------------------------------------------------------------
// LDS with a pre-decoded ROM: word[off].x = byte(off) | byte(off+1) << 8 |
// byte(off+2) << 16 (the successors taken inside the image's 2K mirror or 4K
// bank) and word[off].y = decode entry of byte(off), so one read yields an
// opcode, both operand bytes and the opcode's decode.  dec is the decode
// table (256 entries), also in LDS.
struct LdsWordMem {
    static constexpr bool kRelax = false;
    const uint2 *rom;
    const uint32_t *dec;
    uint8_t *ram;
    uint32_t E, slot;
    uint8_t *sc = nullptr;  // Superchip RAM, in the RAM's layout (NULL: no Superchip image)
    __host__ __device__ __forceinline__ uint32_t rom_byte(uint32_t off) const { return rom[off].x & 0xFFu; }
    __host__ __device__ __forceinline__ uint2 rom_word(uint32_t off) const { return rom[off]; }
    __host__ __device__ __forceinline__ uint32_t ram_byte(uint32_t cell) const {
        return ram[(((cell >> 2) * E + slot) << 2) | (cell & 3u)];
    }
    __host__ __device__ __forceinline__ void ram_set(uint32_t cell, uint32_t v) {
        ram[(((cell >> 2) * E + slot) << 2) | (cell & 3u)] = (uint8_t)v;
    }
    __host__ __device__ __forceinline__ uint32_t ram_word(uint32_t w) const {
        return *reinterpret_cast<const uint32_t *>(ram + ((w * E + slot) << 2));
    }
    __host__ __device__ __forceinline__ void ram_word_set(uint32_t w, uint32_t v) {
        *reinterpret_cast<uint32_t *>(ram + ((w * E + slot) << 2)) = v;
    }
    __host__ __device__ __forceinline__ uint32_t sc_byte(uint32_t cell) const {
        return sc[(((cell >> 2) * E + slot) << 2) | (cell & 3u)];
    }
    __host__ __device__ __forceinline__ void sc_set(uint32_t cell, uint32_t v) {
        sc[(((cell >> 2) * E + slot) << 2) | (cell & 3u)] = (uint8_t)v;
    }
    __host__ __device__ __forceinline__ uint32_t sc_word(uint32_t w) const {
        return *reinterpret_cast<const uint32_t *>(sc + ((w * E + slot) << 2));
    }
    __host__ __device__ __forceinline__ void sc_word_set(uint32_t w, uint32_t v) {
        *reinterpret_cast<uint32_t *>(sc + ((w * E + slot) << 2)) = v;
    }
};

// Successor of ROM offset off inside its 2K mirror (mapper 0) or 4K bank.
__host__ __device__ __forceinline__ uint32_t rom_next(uint32_t off, int32_t mapper) {
    return mapper == 0 ? ((off + 1u) & 0x7FFu) : ((off & ~0xFFFu) | ((off + 1u) & 0xFFFu));
}
__host__ __device__ __forceinline__ uint2 rom_word_at(const uint8_t *rom, uint32_t off, int32_t mapper,
                                                      const uint32_t *decode) {
    const uint32_t o1 = rom_next(off, mapper), o2 = rom_next(o1, mapper);
    const uint32_t b = rom[off];
    uint2 w;
    w.x = b | ((uint32_t)rom[o1] << 8) | ((uint32_t)rom[o2] << 16);
    w.y = decode[b];
    return w;
}

// Opcode and operand bytes at pc (three fetch reads).
template <class C>
__host__ __device__ __forceinline__ void fetch3(C &c, uint32_t &opc, uint32_t &lo, uint32_t &hi) {
    const uint32_t pc = c.pc;
    opc = c.peek(pc, c.cyc);
    lo = c.peek((pc + 1u) & 0xFFFFu, c.cyc);
    hi = c.peek((pc + 2u) & 0xFFFFu, c.cyc);
}

// Opcode, operand bytes and decode entry at pc from a word memory: inside
// $1000-$1FFD the three bytes lie in the cartridge window and the LDS word
// serves them; elsewhere (code in RAM, or an instruction that runs past $1FFF)
// three fetch reads and the decode table.  The word is read for every lane
// (its offset is always inside the image); only when some lane of the wave
// needs the slow fetch does the wave branch.
template <class W, class C>
__host__ __device__ __forceinline__ void fetch_word(C &c, uint32_t &opc, uint32_t &lo, uint32_t &hi, uint32_t &dec) {
    const uint32_t pc = c.pc;
    uint2 w = c.mem.rom_word(c.cart_off(pc));
    W::opaque(w.x);  // both halves now: keeps the word one LDS read
    W::opaque(w.y);
    opc = w.x & 0xFFu;
    lo = (w.x >> 8) & 0xFFu;
    hi = w.x >> 16;
    dec = w.y;
    // the word serves an instruction whose three bytes lie in one bank (E0: one slice)
    // of the cartridge window, outside the Superchip RAM's page
    const bool slow = !(pc & 0x1000u) || (pc & c.fetch_mask) > c.fetch_lim || (c.sc && (pc & 0x1F00u) == 0x1000u);
    if (W::any(slow)) {
        if (slow) {
            fetch3(c, opc, lo, hi);
            dec = c.mem.dec[opc];
        }
    }
}

// Global memory: the env's ROM image and its 128 RAM bytes in the state record.
struct GlobalMem {
    static constexpr bool kRelax = false;
    const uint8_t *rom;
    uint8_t *ram;
    uint8_t *sc;  // the env's Superchip RAM (NULL: no Superchip image)
    __host__ __device__ __forceinline__ uint32_t sc_byte(uint32_t cell) const { return sc[cell]; }
    __host__ __device__ __forceinline__ void sc_set(uint32_t cell, uint32_t v) { sc[cell] = (uint8_t)v; }
    __host__ __device__ __forceinline__ uint32_t sc_word(uint32_t w) const { return reinterpret_cast<const uint32_t *>(sc)[w]; }
    __host__ __device__ __forceinline__ void sc_word_set(uint32_t w, uint32_t v) { reinterpret_cast<uint32_t *>(sc)[w] = v; }
    __host__ __device__ __forceinline__ uint32_t rom_byte(uint32_t off) const { return rom[off]; }
    __host__ __device__ __forceinline__ uint32_t ram_byte(uint32_t cell) const { return ram[cell]; }
    __host__ __device__ __forceinline__ void ram_set(uint32_t cell, uint32_t v) { ram[cell] = (uint8_t)v; }
    __host__ __device__ __forceinline__ uint32_t ram_word(uint32_t w) const { return reinterpret_cast<const uint32_t *>(ram)[w]; }
    __host__ __device__ __forceinline__ void ram_word_set(uint32_t w, uint32_t v) { reinterpret_cast<uint32_t *>(ram)[w] = v; }
};

// FULL relaxed mode (the paper's relaxation without the straight-through
// correction, Table s-modes; Sec. "Forward Bit-Exactness Under Full
// Relaxation"): while an instruction executes, every read of a ROM byte or a
// RAM cell returns the distance-softmax blend of Eq. s-read over the byte and
// its neighbours |k| <= 8 inside the same array (ROM image or the 128 RAM
// cells), with weights e^{-|k|/T}, cast back to a byte (round to nearest,
// ties to even); the branch of Eq. s-branch moves the pc by sigma(alpha z)
// times its offset and is cast likewise (see Cpu::exec_body).  Float32 sums in
// a fixed order without fused multiply-adds, so the casts are those of a
// plain float32 evaluation.  The first instruction whose cast differed from
// the exact value (ndiv, counted from the call's start; -1: none) and the
// number of such casts are recorded; the machine then runs on the cast
// values.  A policy over a memory policy Base, selected at compile time: the
// exact kernels never see it.
struct RelaxConst {
    float u[9];            // u[k] = e^{-k/T} (u[0] = 1)
    float g_taken, g_not;  // sigma(alpha), sigma(-alpha)
};
template <class Base>
struct RelaxMem : Base {
    static constexpr bool kRelax = true;
    RelaxConst rc;
    uint32_t rom_n;   // bytes of the image
    bool active;      // an instruction is executing
    int64_t ninstr;   // instructions completed since the call's start
    int64_t ndiv;
    uint32_t fails;
    __host__ __device__ __forceinline__ void note() {
        if (ndiv < 0) ndiv = ninstr;
        ++fails;
    }
    // Eq. s-read at index a of an array of n bytes read by get(i)
    template <class Get>
    __host__ __device__ __forceinline__ uint32_t blend(Get get, uint32_t a, uint32_t n) {
#pragma clang fp contract(off)
        const uint32_t exact = get(a);
        const float ra = (float)exact;
        float num = 0.f, den = 1.f;
        for (uint32_t k = 1; k <= 8; ++k) {
            const float u = rc.u[k];
            if (a + k < n) {
                num = num + u * ((float)get(a + k) - ra);
                den = den + u;
            }
            if (a >= k) {
                num = num + u * ((float)get(a - k) - ra);
                den = den + u;
            }
        }
        const int32_t v = (int32_t)__builtin_rintf(ra + num / den);
        if (v != (int32_t)exact) note();
        return (uint32_t)v & 0xFFu;
    }
    __host__ __device__ __forceinline__ uint32_t rom_byte(uint32_t off) {
        if (!active) return Base::rom_byte(off);
        return blend([&](uint32_t i) { return Base::rom_byte(i); }, off, rom_n);
    }
    __host__ __device__ __forceinline__ uint32_t ram_byte(uint32_t cell) {
        if (!active) return Base::ram_byte(cell);
        return blend([&](uint32_t i) { return Base::ram_byte(i); }, cell, 128u);
    }
    // Eq. s-branch without the straight-through correction: the flag is crisp
    // (z = +1 taken, -1 not), pc' = round(pc + sigma(alpha z) delta)
    __host__ __device__ __forceinline__ uint32_t branch(uint32_t pc, uint32_t lo, bool taken) {
#pragma clang fp contract(off)
        const float gz = taken ? rc.g_taken : rc.g_not;
        const int32_t cast = (int32_t)__builtin_rintf((float)pc + gz * (float)(int32_t)(int8_t)lo);
        const uint32_t hard = taken ? ((pc + (uint32_t)(int32_t)(int8_t)lo) & 0xFFFFu) : pc;
        const uint32_t got = (uint32_t)cast & 0xFFFFu;
        if (got != hard) note();
        return got;
    }
};

// ---------------------------------------------------------------------------
// Hooks
// ---------------------------------------------------------------------------

// One entry of an env's pixel-write log in translated code (which runs without
// the object paths, so no object shows and no HMOVE blank falls): the effect
// clock of a write, the colour registers, the playfield + CTRLPF, and VBLANK |
// VSYNC << 8, all as before the write.
__host__ __device__ __forceinline__ uint4 log_entry(int32_t clock, const Tia &t) {
    return make_uint4((uint32_t)clock, t.col, t.pf, t.vb);
}

// Upper bound on the polls of a wait between the emulating and the drawing
// lanes (each poll sleeps ~64 clocks, so ~60 ms) with no sign of progress from
// the other side: a wait that long can only be a fault, and giving up keeps every
// wave's exit reachable (the frames are then wrong, not the kernel stuck).
constexpr uint32_t kTrSpinLimit = 1u << 21;
__host__ __device__ __forceinline__ uint32_t ld_ctl(const uint32_t *p) { return *(const volatile uint32_t *)p; }
__host__ __device__ __forceinline__ void st_ctl(uint32_t *p, uint32_t v) { *(volatile uint32_t *)p = v; }

// Draw rows [y0, y1) of a frame from the n entries of a ring starting at entry
// t0 (entry t0 + i at ring slot (t0 + i) mod CAP), the last of which lies past
// the last pixel of row y1 - 1: the pixel at colour clock k shows the state of
// the first entry with an effect clock > k (an entry holds the state before its
// write).  Lane sub of GL takes rows y0 + sub, y0 + sub + GL, ...; a row's first
// entry is found by bisection and the row is walked with the entry pointer, a
// 4-pixel group at a time (one colour unless a write takes effect inside the
// group), 16 pixels per store.
template <int GL, int CAP>
__host__ __device__ __forceinline__ void draw_ring_rows(uint8_t *frame, const uint4 *log, uint32_t t0, uint32_t n,
                                                        int32_t y0, int32_t y1, int32_t ystart, uint32_t sub) {
    constexpr uint32_t M = (uint32_t)CAP - 1u;
    const int32_t vis0 = ystart * kClocksPerLine + kHBlank;  // clock of pixel (0, 0)
    for (int32_t y = y0 + (int32_t)sub; y < y1; y += GL) {
        const int32_t k_row = vis0 + y * kClocksPerLine;
        uint32_t lo = 0, hi = n - 1u;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if ((int32_t)log[(t0 + mid) & M].x > k_row) hi = mid;
            else lo = mid + 1u;
        }
        uint32_t p = lo;
        uint4 e = log[(t0 + p) & M];
        uint32_t mask = pf_mask20(e.z);
        auto advance_past = [&](int32_t k) {  // to the first entry with clock > k
            while ((int32_t)e.x <= k && p + 1u < n) {
                e = log[(t0 + ++p) & M];
                mask = pf_mask20(e.z);
            }
        };
        auto colour = [&](uint32_t g) {
            return (e.w & 2u) ? 0u : ((e.y >> (8 * group_owner(g, mask, e.z >> 24))) & 0xFEu);
        };
        uint8_t *row = frame + y * kScreenW;
        for (int32_t q = 0; q < kScreenW / 16; ++q) {
            uint32_t wd[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t g = (uint32_t)(4 * q + j);
                const int32_t k0 = k_row + 4 * (int32_t)g;
                advance_past(k0);
                if ((int32_t)e.x > k0 + 3) {
                    wd[j] = colour(g) * 0x01010101u;
                } else {  // a write takes effect inside the group, at clock e.x
                    // Effect clocks are multiples of 3, so every entry past those at
                    // e.x lies beyond the group: the pixels before e.x show e, the
                    // rest the first entry past e.x (writes at one clock: the last).
                    const uint32_t c0 = colour(g);
                    const uint32_t m = (1u << (8 * ((int32_t)e.x - k0))) - 1u;  // 1..3 bytes
                    advance_past((int32_t)e.x);
                    wd[j] = ((c0 * 0x01010101u) & m) | ((colour(g) * 0x01010101u) & ~m);
                }
            }
            *reinterpret_cast<uint4 *>(row + 16 * q) = make_uint4(wd[0], wd[1], wd[2], wd[3]);
        }
    }
}

// One round of an env's drawing lanes (lane sub of GL): draw the rows the
// emulation has published and release the entries before the first row not
// drawn (also with no row to draw, once the ring is half full: writes before the
// first visible row fill it with no row to show for them).  Returns whether there
// was anything to do.
template <class W, int GL, int CAP>
__host__ __device__ __forceinline__ bool draw_round(TrCtl *ctl, const uint4 *log, int32_t ystart, uint32_t sub) {
    const uint32_t st = ld_ctl(&ctl->state);
    if (st == 0u) return false;
    const uint32_t ready = ld_ctl(&ctl->ready);
    W::fence();  // the entries and head published with `ready` are visible from here on
    const uint32_t head = ld_ctl(&ctl->head), tail = ld_ctl(&ctl->tail), done = ld_ctl(&ctl->done);
    const bool last = st == 2u && ready >= (uint32_t)kScreenH;
    const uint32_t n = head - tail;
    const bool rows = ready > done;
    if (!rows && !last && n <= (uint32_t)(CAP / 2)) return false;
    const int32_t y1 = ready < (uint32_t)kScreenH ? (int32_t)ready : kScreenH;
    if (n > 0u && (int32_t)done < y1)
        draw_ring_rows<GL, CAP>(ctl->frame, log, tail, n, (int32_t)done, y1, ystart, sub);
    // the first entry past the first pixel of row y1 (earlier ones serve drawn rows only)
    uint32_t keep = n;
    if (y1 < kScreenH) {
        const int32_t cut = ystart * kClocksPerLine + kHBlank + y1 * kClocksPerLine;
        uint32_t lo = 0u;
        while (lo < keep) {
            const uint32_t mid = (lo + keep) >> 1;
            if ((int32_t)log[(tail + mid) & ((uint32_t)CAP - 1u)].x > cut) keep = mid;
            else lo = mid + 1u;
        }
    }
    if (!rows && !last && keep == 0u) return false;  // nothing to release yet
    W::fence();  // this round's reads of the ring are done before the entries are released
    if (sub == 0u) {
        st_ctl(&ctl->done, (uint32_t)y1);
        st_ctl(&ctl->tail, tail + keep);
        if (last) {
            W::fence();
            st_ctl(&ctl->state, 0u);
        }
    }
    W::fence();
    return true;
}

// The drawing wave of translated code: rounds for its envs until each has
// logged its last frame and had it drawn.
template <class W, int GL, int CAP>
__host__ __device__ __forceinline__ void draw_loop(TrCtl *ctl, const uint4 *log, int32_t ystart, uint32_t sub) {
    uint32_t beat = ld_ctl(&ctl->beat);
    for (uint32_t polls = 0; polls < kTrSpinLimit;) {
        const bool fin = ld_ctl(&ctl->fin) != 0u;
        W::fence();
        const bool idle = ld_ctl(&ctl->state) == 0u;
        if (W::all(fin && idle)) break;  // (fin is set after the env's last state change)
        const bool worked = draw_round<W, GL, CAP>(ctl, log, ystart, sub);
        const uint32_t b = ld_ctl(&ctl->beat);
        if (W::any(worked || b != beat)) {
            polls = 0;
        } else {  // idle: poll less often, leaving the SIMD and the LDS to the emulating wave
            W::sleep();
            W::sleep();
            W::sleep();
            W::sleep();
            ++polls;
        }
        beat = b;
    }
}

// Renders the returned frame lazily: before every write that changes pixels
// the pixels up to the write's effect clock are drawn with the old state.  With
// a wave policy W (translated code) a write only appends (effect clock, the TIA
// state before it) to the env's ring log of CAP entries in LDS (lanes without a
// frame write a spare slot: a store with no branch), and flush(), called between
// runs where lanes may branch, publishes how far the entries reach once the ring
// is half full; the drawing wave (draw_loop) turns the covered rows into pixels.
// kAsync false (a build for the host, one lane): the hook draws the rows itself
// at each publish.
struct NoWave {};
template <typename T, class W = NoWave, int GL = 1, int CAP = kTrLogCap, bool kAsync = true>
struct RenderHook {
    static_assert(CAP >= kTrLogCap && (CAP & (CAP - 1)) == 0, "the log holds a row's writes and a run's");
    static constexpr bool kRecord = false;
    T *frame;         // frame being rendered, or nullptr
    float *tan;       // (soft) the frame's position-sampler tangents [5][210][160], or nullptr
    int32_t rend_cc;  // frame-relative colour clock rendered up to
    int32_t pix_cc;   // write point of the last instruction (soft checkpoints)
    int32_t ystart;
    uint32_t sub, G;
    uint4 *log;       // (with W) the env's ring of CAP entries and a spare slot
    TrCtl *ctl;       // (with W) its control block
    uint32_t head;    // (with W) entries appended in the drawn frame
    uint32_t nlog;    // (with W) entries in the ring not yet released, as last seen
    uint32_t pub;     // (with W) head when last published
    template <class C>
    __host__ __device__ __forceinline__ void before_pixel_write(C &c, int32_t w) {
        if constexpr (std::is_same<W, NoWave>::value) {
            if (frame) {
                const int32_t cc = 3 * (w + 1);
                if (cc > rend_cc) {
                    render_span<C::kObjects>(frame, rend_cc, cc, c.tia(), ystart, sub, G, tan);
                    rend_cc = cc;
                }
            }
        } else if (W::any(frame != nullptr)) {  // (wave-uniform) only while some lane draws
            static_assert(!C::kObjects, "translated code runs without the object paths");
            const bool f = frame != nullptr;
            log[f ? (head & (uint32_t)(CAP - 1)) : (uint32_t)CAP] = log_entry(3 * (w + 1), c.tia());
            head += f ? 1u : 0u;
            nlog += f ? 1u : 0u;
        }
    }
    // (with W) a drawn frame starts: wait until the drawing lanes are done with the
    // previous one, then reset the ring
    __host__ __device__ __forceinline__ void begin_frame() {
        if constexpr (!std::is_same<W, NoWave>::value) {
            head = nlog = pub = 0u;
            if (frame) {
                uint32_t polls = 0;
                for (; ld_ctl(&ctl->state) != 0u && polls < kTrSpinLimit; ++polls) W::sleep();
                if (sub == 0u) {
                    if (polls >= kTrSpinLimit) st_ctl(&ctl->stalls, ld_ctl(&ctl->stalls) + 1u);
                    ctl->frame = reinterpret_cast<uint8_t *>(frame);
                    st_ctl(&ctl->head, 0u);
                    st_ctl(&ctl->ready, 0u);
                    st_ctl(&ctl->tail, 0u);
                    st_ctl(&ctl->done, 0u);
                    W::fence();
                    st_ctl(&ctl->state, 1u);
                }
                W::fence();
            }
        }
    }
    // (with W) publish the entries and the rows they determine (rows whose last
    // pixel lies before the last entry's clock; all of them at the frame's end)
    __host__ __device__ __forceinline__ void publish(bool all) {
        const int32_t vis0 = ystart * kClocksPerLine + kHBlank;
        int32_t y_hi = kScreenH;
        if (!all) {
            const int32_t t = (int32_t)log[(head - 1u) & (uint32_t)(CAP - 1)].x - vis0 - (kScreenW - 1);
            y_hi = t <= 0 ? 0 : (t + kClocksPerLine - 1) / kClocksPerLine;
            y_hi = y_hi < kScreenH ? y_hi : kScreenH;
        }
        W::fence();  // the entries before head and ready
        if (sub == 0u) st_ctl(&ctl->head, head);
        W::fence();
        if (sub == 0u) {
            st_ctl(&ctl->ready, (uint32_t)y_hi);
            if (all) {
                W::fence();
                st_ctl(&ctl->state, 2u);
            }
        }
        W::fence();
        pub = head;
        if constexpr (!kAsync) {  // no drawing wave: draw here
            while (draw_round<W, GL, CAP>(ctl, log, ystart, sub)) {
            }
        }
    }
    // (with W) wait until at most `room_left` entries of the ring are unreleased
    __host__ __device__ __forceinline__ void wait_room(uint32_t limit) {
        for (uint32_t polls = 0;; ++polls) {
            nlog = head - ld_ctl(&ctl->tail);
            if (W::all(!frame || nlog <= limit)) break;
            if (polls >= kTrSpinLimit) {
                if (frame && nlog > limit && sub == 0u) st_ctl(&ctl->stalls, ld_ctl(&ctl->stalls) + 1u);
                break;
            }
            W::sleep();
        }
    }
    // (with W) between runs: publish every quarter ring of entries, and make room
    // for the next run once the ring may not hold it
    template <class C>
    __host__ __device__ __forceinline__ void flush(C &) {
        if constexpr (!std::is_same<W, NoWave>::value) {
            static_assert(sizeof(T) == 1, "translated code returns u8 frames");
            const bool f = frame != nullptr;
            const bool due = f && head - pub >= (uint32_t)(CAP / 4);
            const bool full = f && nlog > (uint32_t)(CAP - kTrMaxRun);
            if (W::any(due || full)) {
                if (f && head != pub) publish(false);
                if (W::any(full)) wait_room((uint32_t)(CAP - kTrMaxRun));
            }
        }
    }
    template <class C>
    __host__ __device__ __forceinline__ void before_exec(C &) {}
    template <class C>
    __host__ __device__ __forceinline__ void after_exec(C &, uint32_t, int32_t, int32_t wp, ExecInfo &) {
        pix_cc = 3 * wp;
    }
    template <class C>
    __host__ __device__ __forceinline__ void finish_frame(C &c) {
        if constexpr (std::is_same<W, NoWave>::value) {
            if (frame) render_span<C::kObjects>(frame, rend_cc, kClocksPerFrame, c.tia(), ystart, sub, G, tan);
        } else {
            if (W::any(frame != nullptr)) {  // the rest of the frame with the current state
                wait_room((uint32_t)CAP - 1u);
                const bool f = frame != nullptr;
                log[f ? (head & (uint32_t)(CAP - 1)) : (uint32_t)CAP] = log_entry(kClocksPerFrame, c.tia());
                head += f ? 1u : 0u;
                if (f) publish(true);
            }
            head = nlog = pub = 0u;
            if (sub == 0u) st_ctl(&ctl->beat, ld_ctl(&ctl->beat) + 1u);
        }
    }
    // (with W) the env logs no more frames: the drawing lanes may stop once it is
    // drawn.  A frame still being logged (an env stopped by the first pass of a
    // hard step, whose outputs are void) is abandoned.
    __host__ __device__ __forceinline__ void end_frames() {
        if constexpr (!std::is_same<W, NoWave>::value) {
            W::fence();
            if (sub == 0u) {
                if (ld_ctl(&ctl->state) == 1u) st_ctl(&ctl->state, 0u);
                W::fence();
                st_ctl(&ctl->fin, 1u);
            }
            W::fence();
        }
    }
};

// Per-lane partial sums of dL/dpixel by owner over the groups lane `lane` of
// `width` takes in [from, to), where objects show or an HMOVE blank falls.
struct PixelParts {
    float p[4];
    bool any;
};
__host__ __device__ inline __attribute__((noinline)) PixelParts pixel_parts_objects(const float *gframe, int32_t from,
                                                                            int32_t to, const Tia t, int32_t ystart,
                                                                            uint32_t lane, uint32_t width) {
    PixelParts out{{0.f, 0.f, 0.f, 0.f}, false};
    const uint32_t mask = pf_mask20(t.pf), ctrl = t.pf >> 24;
    const bool objs = objs_shown(t.ob);
    Row160 r[kRows];
    object_rows(r, t);
    const int32_t hl = hmove_line(t.ob) - ystart;
    for_each_group(from, to, ystart, lane, width, [&](int32_t y, int32_t g, int32_t xa, int32_t xb) {
        out.any = true;
        if (y == hl && g < 2) return;  // blanked: constant pixels
        const float *row = gframe + y * kScreenW;
        uint32_t nib[kRows];
        group_occupancy(r, (uint32_t)g, nib);
        for (int32_t x = xa; x < xb; ++x) {
            const uint32_t o = objs ? pixel_owner(nib, (uint32_t)(x - 4 * g), (uint32_t)x, ctrl)
                                    : group_owner((uint32_t)g, mask, ctrl);
            for (uint32_t k = 0; k < 4; ++k) out.p[k] += o == k ? row[x] : 0.f;
        }
    });
    return out;
}

// Per-owner sums of dL/dpixel over [from, to) drawn with state t by the lanes
// of a wave (the soft backward runs one env per wave): lane l takes every
// kWidth-th 4-pixel group of each line, then the wave sums the four partial
// sums.  Returns (the same in every lane) whether any visible pixel lies in the
// span.  Blanked pixels are constants and take no gradient.  kObj false: a
// machine without the object paths (no object shows, no HMOVE blank falls).
template <class W, bool kObj>
__host__ __device__ __forceinline__ bool pixel_sums_wave(const float *gframe, int32_t from, int32_t to, const Tia &t,
                                                         int32_t ystart, float sums[4]) {
    if (t.vb & 2u) return false;
    const int32_t vis0 = ystart * kClocksPerLine, vis1 = vis0 + kScreenH * kClocksPerLine;
    if (to <= vis0 || from >= vis1) return false;
    float part[4] = {0.f, 0.f, 0.f, 0.f};
    bool any = false;
    if (kObj && (hmove_line(t.ob) >= 0 || objs_shown(t.ob))) {
        const PixelParts pp = pixel_parts_objects(gframe, from, to, t, ystart, W::lane(), W::kWidth);
        for (uint32_t k = 0; k < 4; ++k) part[k] = pp.p[k];
        any = pp.any;
    } else {
        const uint32_t mask = pf_mask20(t.pf), ctrl = t.pf >> 24;
        for_each_group(from, to, ystart, W::lane(), W::kWidth, [&](int32_t y, int32_t g, int32_t xa, int32_t xb) {
            const float *row = gframe + y * kScreenW;
            float acc = 0.f;
            for (int32_t x = xa; x < xb; ++x) acc += row[x];
            const uint32_t o = group_owner((uint32_t)g, mask, ctrl);
            for (uint32_t k = 0; k < 4; ++k) part[k] += o == k ? acc : 0.f;  // constant indices: stays in registers
            any = true;
        });
    }
    if (!W::any(any)) return false;
    for (uint32_t k = 0; k < 4; ++k) sums[k] += W::sum(part[k]);
    return true;
}

// Records the recompute tape of the soft backward.  Pixels of the final frame
// are attributed to the instruction during whose span [previous write point,
// this write point) they were drawn, with the state before its write.  Every
// lane of the env's wave runs the recompute; lane 0 stores the records.
template <class W>
struct TapeHook {
    static constexpr bool kRecord = true;
    TapeRec *tape;
    int32_t nrec, max_rec;
    const float *gframe;  // env's dL/dframe while in the final frame, else nullptr
    int32_t pix_cc;
    int32_t ystart;
    uint32_t step;
    Tia save;             // the TIA state before the instruction
    int32_t *overflow;
    bool lead;            // the lane that stores
    float read_T;         // address surrogate (0: off)
    uint32_t rom_n;       // bytes of the image (the relaxed read's array bounds)
    __host__ __device__ __forceinline__ void emit(const TapeRec &r) {
        if (nrec < max_rec) {
            if (lead) tape[nrec] = r;
        } else if (lead) {
            *overflow = 1;
        }
        ++nrec;
    }
    template <class C>
    __host__ __device__ __forceinline__ void before_pixel_write(C &, int32_t) {}
    template <class C>
    __host__ __device__ __forceinline__ void before_exec(C &c) {
        save = c.tia();
    }
    // Instructions whose reverse-sweep rule is the identity need no record unless
    // pixels are attributed to them: branches, flag changes, compares, BIT, NOPs,
    // jumps, returns, PLP, TXS, and stores to registers that carry no content
    // (WSYNC, VBLANK, the timer, ...).
    static constexpr uint64_t kNoContent =
        (1ull << C_BRANCH) | (1ull << C_FLAG) | (1ull << C_CMP) | (1ull << C_CPX) | (1ull << C_CPY) |
        (1ull << C_BIT) | (1ull << C_NOP) | (1ull << C_JMP) | (1ull << C_RTS) | (1ull << C_RTI) |
        (1ull << C_PLP) | (1ull << C_TXS);
    static constexpr uint64_t kStores = (1ull << C_STA) | (1ull << C_STX) | (1ull << C_STY) | (1ull << C_SAX);
    // Slope of Eq. s-read (the distance-softmax read, window |j - a| <= 8 inside the
    // array) at the hard address a, taken symmetrically with coefficients at hard
    // values: (1/T) sum_j w_j sign(j - a) (R[j] - R[a]), w_j = exp(-|j - a|/T) / Z.
    template <class Get>
    __host__ __device__ __forceinline__ float read_slope(Get get, uint32_t a, uint32_t n) const {
        const float ra = (float)get(a);
        float z = 1.f, acc = 0.f;
        for (uint32_t k = 1; k <= 8; ++k) {
            const float w = expf(-(float)k / read_T);
            if (a + k < n) {
                acc += w * ((float)get(a + k) - ra);
                z += w;
            }
            if (a >= k) {
                acc -= w * ((float)get(a - k) - ra);
                z += w;
            }
        }
        return acc / (z * read_T);
    }
    // The words of an instruction's record (w3, the step, is the caller's); returns
    // whether the instruction has content to record.
    __host__ __device__ __forceinline__ static bool instr_words(uint32_t opc, const ExecInfo &info, uint32_t &w0,
                                                                uint32_t &w1, uint32_t &w2) {
        w0 = opc | (info.rd_cls << 8) | (info.wr_cls << 12) | (kRecInstr << 16) | (info.op_cls << 24);
        w1 = info.rd_idx | (info.wr_idx << 16);
        w2 = (info.v1 & 0xFFu) | ((info.v2 & 0xFFu) << 8) | ((info.s_before & 0xFFu) << 16);
        return !(((kNoContent >> info.op_cls) & 1u) ||
                 (((kStores >> info.op_cls) & 1u) && info.wr_cls == kClsConst));
    }
    template <class C>
    __host__ __device__ __forceinline__ void after_exec(C &c, uint32_t opc, int32_t, int32_t wp, ExecInfo &info) {
        TapeRec r;
        bool keep = instr_words(opc, info, r.w0, r.w1, r.w2);
        r.w3 = step;
        // address surrogate: an indexed load or ALU read of a ROM or RAM byte also passes
        // gradient to its index register (read-modify-write forms do not)
        constexpr uint64_t kIndexedReads = (1ull << C_LDA) | (1ull << C_LDX) | (1ull << C_LDY) | (1ull << C_LAX) |
                                           (1ull << C_ADC) | (1ull << C_SBC) | (1ull << C_AND) | (1ull << C_ORA) |
                                           (1ull << C_EOR);
        if (read_T > 0.f && ((kIndexedReads >> info.op_cls) & 1u) &&
            (info.rd_cls == kClsRom || info.rd_cls == kClsRam)) {
            const uint32_t mode = (c.mem.dec[opc] >> 6) & 15u;
            const uint32_t ik = (mode == M_ZPX || mode == M_ABX) ? 1u
                              : (mode == M_ZPY || mode == M_ABY || mode == M_IZY) ? 2u : 0u;
            if (ik) {
                const float kappa = info.rd_cls == kClsRom
                    ? read_slope([&](uint32_t i) { return c.mem.rom_byte(i); }, info.rd_idx, rom_n)
                    : read_slope([&](uint32_t i) { return c.mem.ram_byte(i); }, info.rd_idx, 128u);
                r.w0 |= ik << 21;
                r.w3 = __builtin_bit_cast(uint32_t, kappa);
            }
        }
        r.pix[0] = r.pix[1] = r.pix[2] = r.pix[3] = 0.f;
        if (gframe && pixel_sums_wave<W, C::kObjects>(gframe, pix_cc, 3 * wp, save, ystart, r.pix)) {
            r.w0 |= 1u << 20;
            keep = true;
        }
        pix_cc = 3 * wp;
        if (keep) emit(r);
    }
};

// Hook of a soft forward that keeps its tape: renders as RenderHook and, while
// `taping`, appends every instruction record the backward's recompute would
// make (TapeHook, without the address surrogate) to the env's forward tape, 16
// bytes each (w0..w3 of TapeRec).  The final frame, whose pixels carry the
// loss's gradient, is never taped: its records need dL/dframe.
template <typename T, class W>
struct TapeFwdHook : RenderHook<T> {
    static constexpr bool kRecord = true;
    uint4 *ftape;      // the env's forward tape
    int32_t fcap, fn;  // capacity; records so far (counted on past the capacity)
    uint32_t step;
    bool taping, lead;
    __host__ __device__ __forceinline__ void put(const uint4 &r) {
        if (fn < fcap && lead) ftape[fn] = r;
        ++fn;
    }
    template <class C>
    __host__ __device__ __forceinline__ void after_exec(C &c, uint32_t opc, int32_t x, int32_t wp, ExecInfo &info) {
        RenderHook<T>::after_exec(c, opc, x, wp, info);
        if (taping) {
            uint4 r;
            if (TapeHook<W>::instr_words(opc, info, r.x, r.y, r.z)) {
                r.w = step;
                put(r);
            }
        }
    }
};

// The soft backward's RAM adjoint, 128 floats held across the lanes of the
// env's wave: cell c is element c / kWidth of lane c % kWidth.  Cells are
// addressed by wave-uniform indices (read and written with readlane /
// writelane), so the reverse sweep touches no memory for them.
template <class W>
struct RamAdjoint {
    static constexpr uint32_t NW = W::kWidth, CPL = 128 / NW;
    float v[CPL];
    __host__ __device__ __forceinline__ void zero() {
        for (uint32_t i = 0; i < CPL; ++i) v[i] = 0.f;
    }
    __host__ __device__ __forceinline__ float get(uint32_t c) const {
        if constexpr (NW == 1) {
            return v[c];
        } else {
            float r = v[0];
            for (uint32_t i = 1; i < CPL; ++i) r = (c / NW == i) ? v[i] : r;
            return W::readlane(r, c % NW);
        }
    }
    __host__ __device__ __forceinline__ void set(uint32_t c, float x) {
        if constexpr (NW == 1) {
            v[c] = x;
        } else {
            for (uint32_t i = 0; i < CPL; ++i)
                if (c / NW == i) v[i] = W::writelane(v[i], x, c % NW);
        }
    }
    // element i of this lane is cell lane + NW * i
};

// ---------------------------------------------------------------------------
// Dispatch of one instruction whose opcode u (decode d) is the same in every
// lane of the call.  Opcodes whose data accesses all fall in page 0 or the
// stack (immediate, implied, zero-page, stack and relative forms: most of
// what VCS game code executes) run a copy of the interpreter with the decode
// entry known at compile time, with the page-0 read done branch-free and the
// write, if any, deferred until after the opcode switch.  The switch then has
// no per-lane branch and compiles to a scalar branch tree.  Every other
// opcode takes the generic path.
// ---------------------------------------------------------------------------
constexpr bool fast_form(uint32_t op) {
    const uint32_t d = decode_op(op), cls = d & 63u, mode = (d >> 6) & 15u;
    if (d == 0 || cls == C_JSR || cls == C_BRK || mode == M_IND) return false;
    const bool page0 = mode == M_IMP || mode == M_ACC || mode == M_IMM || mode == M_REL || mode == M_ZP ||
                       mode == M_ZPX || mode == M_ZPY;
    return page0 || (mode == M_ABS && cls == C_JMP);
}

template <uint32_t OP, class C>
__host__ __device__ __forceinline__ bool exec_fast(C &c, uint32_t lo, uint32_t hi, ExecInfo &info, int32_t &t0,
                                                   int32_t &n, uint32_t &ea, uint32_t &r) {
    static_assert(fast_form(OP), "not a page-0 form");
    constexpr uint32_t D = decode_op(OP);
    return c.template exec_body<true>(OP, D, lo, hi, info, t0, n, ea, r);
}

// A page-0 / stack write (address a8 < $100) from every running lane.  When all
// lanes write the same address (lockstep code: STA WSYNC, STA COLUBK, ...) the
// RAM/TIA decision and the TIA register switch are taken once, on a scalar.
template <class W, class C>
__host__ __device__ __forceinline__ void write_page0(C &c, uint32_t a8, uint32_t v, int32_t w) {
    const uint32_t u8 = W::first(a8);
    if (W::all(a8 == u8)) {
        if (u8 & 0x80u) c.mem.ram_set(u8 & 0x7Fu, v);
        else c.tia_out(u8 & 0x3Fu, v, w);
    } else {
        c.write_zp(a8, v, w);
    }
}

template <class W, class C>
__host__ __device__ __forceinline__ void exec_dispatch(C &c, uint32_t u, uint32_t d, uint32_t lo, uint32_t hi,
                                                       ExecInfo &info) {
    bool fast = true, wr = false;
    int32_t t0 = 0, n = 0;
    uint32_t ea = 0, r = 0;
#define VCS_FAST(op) \
    case op: wr = exec_fast<op>(c, lo, hi, info, t0, n, ea, r); break;
    switch (u) {
        VCS_FAST(0x85) VCS_FAST(0x86) VCS_FAST(0x84) VCS_FAST(0x95) VCS_FAST(0x94) VCS_FAST(0x96)  // stores
        VCS_FAST(0xA5) VCS_FAST(0xA6) VCS_FAST(0xA4) VCS_FAST(0xB5) VCS_FAST(0xB4) VCS_FAST(0xB6)  // loads zp
        VCS_FAST(0xA9) VCS_FAST(0xA2) VCS_FAST(0xA0)                                               // loads #
        VCS_FAST(0x10) VCS_FAST(0x30) VCS_FAST(0x50) VCS_FAST(0x70)                                // branches
        VCS_FAST(0x90) VCS_FAST(0xB0) VCS_FAST(0xD0) VCS_FAST(0xF0)
        VCS_FAST(0x48) VCS_FAST(0x68) VCS_FAST(0x08) VCS_FAST(0x28) VCS_FAST(0x60) VCS_FAST(0x40)  // stack, RTS, RTI
        VCS_FAST(0x88) VCS_FAST(0xCA) VCS_FAST(0xC8) VCS_FAST(0xE8)                                // DEY DEX INY INX
        VCS_FAST(0xE6) VCS_FAST(0xC6) VCS_FAST(0xF6) VCS_FAST(0xD6)                                // INC DEC zp, zp,X
        VCS_FAST(0x38) VCS_FAST(0x18) VCS_FAST(0xD8) VCS_FAST(0xF8) VCS_FAST(0x78) VCS_FAST(0x58)  // flags
        VCS_FAST(0xB8)
        VCS_FAST(0x65) VCS_FAST(0xE5) VCS_FAST(0x69) VCS_FAST(0xE9) VCS_FAST(0x75) VCS_FAST(0xF5)  // ADC SBC
        VCS_FAST(0x29) VCS_FAST(0x09) VCS_FAST(0x49) VCS_FAST(0x25) VCS_FAST(0x05) VCS_FAST(0x45)  // AND ORA EOR
        VCS_FAST(0xC9) VCS_FAST(0xE0) VCS_FAST(0xC0) VCS_FAST(0xC5) VCS_FAST(0xE4) VCS_FAST(0xC4)  // CMP CPX CPY
        VCS_FAST(0x24)                                                                             // BIT zp
        VCS_FAST(0x0A) VCS_FAST(0x4A) VCS_FAST(0x2A) VCS_FAST(0x6A)                                // shifts A
        VCS_FAST(0x06) VCS_FAST(0x46) VCS_FAST(0x26) VCS_FAST(0x66)                                // shifts zp
        VCS_FAST(0xAA) VCS_FAST(0xA8) VCS_FAST(0x8A) VCS_FAST(0x98) VCS_FAST(0xBA) VCS_FAST(0x9A)  // transfers
        VCS_FAST(0xEA) VCS_FAST(0x4C)                                                              // NOP, JMP abs
        default: fast = false; break;
    }
#undef VCS_FAST
    // The switch's outcome goes through an opaque scalar so that the optimiser
    // cannot thread the per-lane write below back into the cases (which would
    // put per-lane branches inside the switch).
    uint32_t how = (fast ? 1u : 0u) | (wr ? 2u : 0u);
    W::opaque_uniform(how);
    if (how & 1u) {
        if (how & 2u) write_page0<W>(c, ea, r, t0 + n - 1);
        c.finish(u, info, t0, n, (how & 2u) != 0u);
    } else {
        c.exec(u, d, lo, hi, info);
    }
}

// One page-0 form instruction whose opcode OP is known at compile time
// (translated code), run by lanes that agree on its write address (the
// translated code checks that before it, for the forms whose address is per
// lane): the phases of exec_dispatch's case for OP with the write taken on the
// wave-uniform address, so that the code has no per-lane branch.
template <class W, uint32_t OP, class C>
__host__ __device__ __forceinline__ void exec_static(C &c, uint32_t lo, uint32_t hi) {
    constexpr uint32_t D = decode_op(OP);
    static_assert(D != 0 && fast_form(OP), "a page-0 form");
    ExecInfo info;
    int32_t t0 = 0, n = 0;
    uint32_t ea = 0, r = 0;
    const bool wr = c.template exec_body<true>(OP, D, lo, hi, info, t0, n, ea, r);
    if (wr) {
        const uint32_t u8 = W::first(ea);
        if (u8 & 0x80u) c.mem.ram_set(u8 & 0x7Fu, r);
        else c.tia_out(u8 & 0x3Fu, r, t0 + n - 1);
        // only a WSYNC write ($02 or its mirror $42) can have set the stall flag
        // (it is clear between instructions); for a constant address this folds
        c.finish(OP, info, t0, n, (u8 & 0xBFu) == 0x02u);
    } else {
        c.finish(OP, info, t0, n, false);
    }
}

// One interpreted instruction at each running lane's pc: fetch, decode and a
// dispatch that is wave-uniform when the lanes share the opcode, else a
// waterfall over the distinct opcodes of the wave.
template <class W, bool kPlain, class C>
__host__ __device__ __forceinline__ void interp_one(C &c, const uint32_t *decode) {
    uint32_t opc, lo, hi;
    ExecInfo info;
    if constexpr (std::decay_t<decltype(c.mem)>::kRelax) {
        // FULL relaxed mode: the opcode and both bytes after it are read (relaxed) for
        // every instruction that does not jam, then the lanes' opcodes run one per pass
        c.mem.active = true;
        opc = c.peek(c.pc, c.cyc);
        const uint32_t dj = decode[opc];
        if (dj == 0) {
            c.jam = 1;
        } else {
            lo = c.peek((c.pc + 1u) & 0xFFFFu, c.cyc);
            hi = c.peek((c.pc + 2u) & 0xFFFFu, c.cyc);
        }
        for (bool more = dj != 0; W::any(more);) {
            if (more) {
                const uint32_t u2 = W::first(opc);
                if (opc == u2) {
                    c.exec(u2, W::first(dj), lo, hi, info);
                    ++c.mem.ninstr;
                    more = false;
                }
            }
        }
        c.mem.active = false;
    } else if constexpr (kPlain) {
        fetch3(c, opc, lo, hi);
        const uint32_t d = decode[opc];
        if (d == 0) c.jam = 1;
        else c.exec(opc, d, lo, hi, info);
    } else {
        uint32_t dec;
        fetch_word<W>(c, opc, lo, hi, dec);
        const uint32_t u = W::first(opc);
        const uint32_t d = W::first(dec);
        if (W::all(opc == u)) {
            // the usual case: every running lane has the same opcode
            if (d == 0) c.jam = 1;
            else exec_dispatch<W>(c, u, d, lo, hi, info);
        } else {
            // waterfall: each pass executes one distinct opcode of the
            // wave with a wave-uniform (scalar) decode.  The operands and
            // registers are made opaque per pass so that no case's
            // arithmetic is hoisted out of the loop and run for all cases.
            for (;;) {
                W::opaque(lo);
                W::opaque(hi);
                W::opaque(c.x);
                W::opaque(c.y);
                W::opaque(c.a);
                W::opaque(c.s);
                const uint32_t u2 = W::first(opc);
                const uint32_t d2 = W::first(dec);
                if (opc == u2) {
                    if (d2 == 0) c.jam = 1;
                    else c.exec(u2, d2, lo, hi, info);
                    break;
                }
            }
        }
    }
}

// Lanes of a wave running several envs through the interpreter that are within
// this many CPU cycles of the wave's least advanced env run the next instruction
// together (kSync); the others wait for it.
constexpr int32_t kSyncWindow = 4;

// Executors of the instruction loop of a frame.  The interpreter runs
// interp_one until the lane reaches its cycle limit or jams; translated code
// (generated per ROM image, see the translator) keeps the position of the
// next instruction in its state and runs straight-line code from there.
//
// kSync (a wave of several envs): an env runs its next instruction only while
// it is at most kSyncWindow cycles ahead of the wave's least advanced env.  Envs
// of one image whose paths part (joystick, timer, resets) then meet again where
// their code waits for the same clock (WSYNC, the frame's end) and go on in
// step, one dispatch for all, instead of drifting apart into a waterfall over
// their opcodes for the rest of the frame.  Each env still runs its own
// instructions in order, so the results do not change.
struct InterpExec {
    template <typename T, class W>
    using Hook = RenderHook<T>;
    struct State {};
    template <class C>
    __host__ __device__ __forceinline__ static void init(C &, State &) {}
    template <class W, bool kPlain, bool kSync = false, class C>
    __host__ __device__ __forceinline__ static void run(C &c, State &, bool go, int32_t lim, const uint32_t *decode) {
        if constexpr (kSync) {
            while (W::any(go)) {  // (uniform loop: every lane takes part in the reduction)
                const int32_t least = W::min_i32(go ? c.cyc : 2147483647);
                if (go && c.cyc <= least + kSyncWindow) {
                    interp_one<W, kPlain>(c, decode);
                    go = !c.jam && c.cyc < lim;
                }
            }
        } else {
            while (go) {
                interp_one<W, kPlain>(c, decode);
                go = !c.jam && c.cyc < lim;
            }
        }
    }
};

// The interpreter with a soft forward that keeps its tape (TapeFwdHook).
struct TapeFwdExec : InterpExec {
    template <typename T, class W>
    using Hook = TapeFwdHook<T, W>;
};

// ---------------------------------------------------------------------------
// Per-env bodies of the kernels.  W is the wave policy: any(v) / all(v) (is v
// true in any / every active lane of the wave), first(v) (v of the first active
// lane), table(t, u) (entry u of a constant table, u the same in every active
// lane) and opaque(v) / opaque_uniform(v) (hide a per-lane / wave-uniform v from
// the optimiser); on the GPU they are ballots, readfirstlane, a scalar load and
// empty asm statements, and the ROM image must already be staged in LDS by the
// whole workgroup.
// ---------------------------------------------------------------------------
template <class W, int G, bool kSoft, bool kPlain, class X = InterpExec, bool kObj = true, class Mem>
__host__ __device__ __forceinline__ void step_env(const StepParams &P, int32_t env, uint32_t sub, int32_t mapper,
                                                  Mem mem, const uint32_t *decode,
                                                  typename X::State xs = typename X::State{}) {
    static_assert(!(kSoft && kPlain), "the soft forward uses the grouped kernel");
    constexpr bool kTapeFwd = std::is_same<X, TapeFwdExec>::value;  // a soft forward that keeps its tape
    static_assert(kSoft || !kTapeFwd, "only the soft forward keeps a tape");
    using T = typename std::conditional<kSoft, float, uint8_t>::type;
    // a rerun of flagged envs (P.rerun) leaves the others alone
    const bool live = env >= 0 && (!P.rerun || P.rerun[env]);
    const int32_t S = P.steps, F = P.frame_skip;

    Cpu<Mem, typename X::template Hook<T, W>, kObj> c;
    c.set_cart(mapper);
    c.mem = mem;
    c.hook.frame = nullptr;
    c.hook.tan = nullptr;
    c.hook.rend_cc = 0;
    c.hook.pix_cc = 0;
    c.hook.ystart = P.ystart;
    c.hook.sub = sub;
    c.hook.G = G;
    // frame counts frames since power-on (hard) or since the call's start (soft;
    // frame0 then holds the starting state's count)
    uint32_t frame = 0, frame0 = 0, episode = 0, ep_step = 0;
    const StateRec *src = kSoft ? P.state_in : (P.state_src ? P.state_src : P.state);
    const uint8_t *sc_src = P.sc_src ? P.sc_src : P.sc_state;
    if (live) {
        if (kSoft && !src) {  // soft forward: power-on with the decoded RAM
            const uint32_t *r0 = reinterpret_cast<const uint32_t *>(P.ram0 + (size_t)env * 128);
            for (uint32_t w = sub; w < 32; w += G) c.mem.ram_word_set(w, r0[w]);
            c.power_on();
        } else {
            const StateRec &st = src[env];
            c.load(st);
            frame = st.frame;
            episode = st.episode;
            ep_step = st.ep_step;
            if constexpr (!kPlain) {
                const uint32_t *rw = reinterpret_cast<const uint32_t *>(st.ram);
                for (uint32_t w = sub; w < 32; w += G) c.mem.ram_word_set(w, rw[w]);
                if (c.sc) {  // Superchip RAM, kept after the state records
                    const uint32_t *sw = reinterpret_cast<const uint32_t *>(sc_src + (size_t)env * 128);
                    for (uint32_t w = sub; w < 32; w += G) c.mem.sc_word_set(w, sw[w]);
                }
            }
            if (st.status & 2u) {  // power-on requested by vcs_reset
                c.power_on();
                frame = 0;
            }
            if constexpr (kSoft) {
                frame0 = frame;
                frame = 0;
            }
        }
    }
    X::init(c, xs);
    int32_t seg0 = 0;  // (forward tape) first record of the current segment
    if constexpr (kTapeFwd) {
        c.hook.ftape = live ? P.ftape + (size_t)env * (size_t)P.ftape_cap : nullptr;
        c.hook.fcap = P.ftape_cap;
        c.hook.fn = 0;
        c.hook.step = 0;
        c.hook.taping = live;
        c.hook.lead = sub == 0;
    }

    int32_t s_idx = 0, fstep = 0;
    bool active = live && S > 0;
    bool stopped = false;  // (without the object paths) the env's results are void
    auto set_ports = [&]() {
        const uint32_t act = P.actions ? P.actions[(size_t)env * S + s_idx] : 0u;
        action_ports(act, &c.swcha, &c.inpt4, &c.swchb);
        if constexpr (kTapeFwd) c.hook.step = (uint32_t)s_idx;
    };
    auto start_frame = [&]() {
        c.hook.rend_cc = 0;
        c.hook.frame = nullptr;
        const bool last_of_step = fstep == F - 1;
        if constexpr (kTapeFwd) {
            if (last_of_step && s_idx == S - 1) c.hook.taping = false;  // the final frame is recomputed
        }
        if constexpr (kSoft) {
            if (P.frame_out_f && last_of_step && s_idx == S - 1) {
                c.hook.frame = P.frame_out_f + (size_t)env * kPixels;
                if (P.frame_dpos_f) c.hook.tan = P.frame_dpos_f + (size_t)env * 5 * kPixels;
            }
        } else {
            if (P.frame_out && last_of_step) {
                if (P.frames_mode == 2) c.hook.frame = P.frame_out + ((size_t)env * S + s_idx) * kPixels;
                else if (P.frames_mode == 1 && s_idx == S - 1) c.hook.frame = P.frame_out + (size_t)env * kPixels;
            }
        }
        c.hook.begin_frame();
    };
    if (active) {
        set_ports();
        start_frame();
    }
    // soft forward: hard-state checkpoints, the first at the start, then every K
    // cycles since the start, each taken at the first instruction boundary (or
    // frame end) at or after its multiple of K
    int64_t next_ckpt = P.ckpt_interval;
    int32_t nckpt = 0;
    auto save_checkpoint = [&](int64_t g) {
        if constexpr (kSoft) {
            next_ckpt = (g / P.ckpt_interval + 1) * P.ckpt_interval;
            if constexpr (kTapeFwd) {  // the segment ending here is taped if all of it fit
                if (nckpt > 0 && nckpt <= P.max_ckpt && sub == 0 && c.hook.taping && c.hook.fn <= c.hook.fcap) {
                    StateRec &prev = P.ckpt[(size_t)env * P.max_ckpt + nckpt - 1];
                    prev.tape_off = (uint32_t)seg0;
                    prev.tape_n = c.hook.fn - seg0;
                }
                seg0 = c.hook.fn;
            }
            if (nckpt < P.max_ckpt) {
                StateRec &r = P.ckpt[(size_t)env * P.max_ckpt + nckpt];
                if (sub == 0) {
                    c.store(r);
                    r.frame = frame;
                    r.episode = 0;
                    r.ep_step = (uint32_t)s_idx;
                    r.next_ckpt = next_ckpt;
                    r.pix_cc = c.hook.pix_cc;
                    r.ckpt_index = (uint32_t)nckpt;
                    r.from_tape = src ? 0u : 1u;
                    r.tape_off = 0u;
                    r.tape_n = -1;
                }
                uint32_t *rw = reinterpret_cast<uint32_t *>(r.ram);
                for (uint32_t w = sub; w < 32; w += G) rw[w] = c.mem.ram_word(w);
            }
            ++nckpt;
        }
    };
    auto checkpoint = [&]() {
        if constexpr (kSoft) {
            if (P.ckpt) {
                const int64_t g = (int64_t)frame * kCyclesPerFrame + c.cyc;
                if (g >= next_ckpt) save_checkpoint(g);
            }
        }
    };
    if constexpr (kSoft) {
        if (P.ckpt && active) save_checkpoint((int64_t)c.cyc);
    }

    while (W::any(active)) {
        // ---- the instructions of one frame (the hot loop; a lane leaves it at
        // its frame's end, the wave when every lane has).  A soft forward also
        // leaves it at its next checkpoint cycle, takes the checkpoint and goes on,
        // so the hot loop itself tests no checkpoint condition.
        bool run = active && !c.jam && c.cyc < kCyclesPerFrame;
        for (;;) {
            int32_t lim = kCyclesPerFrame;  // frame-relative cycle at which the lane stops
            if constexpr (kSoft) {
                if (run) {
                    checkpoint();
                    if (P.ckpt) {
                        const int64_t rel = next_ckpt - (int64_t)frame * kCyclesPerFrame;
                        lim = rel < (int64_t)kCyclesPerFrame ? (int32_t)rel : kCyclesPerFrame;
                    }
                }
            }
            const bool go = run && c.cyc < lim;
            X::template run<W, kPlain, (!kPlain && G < (int)W::kWidth)>(c, xs, go, lim, decode);
            run = active && !c.jam && c.cyc < kCyclesPerFrame;
            if constexpr (!kSoft) break;
            if (!W::any(run)) break;
        }
        if (!active) continue;
        if constexpr (!kObj) {
            if (c.obj_stop) {  // an object showed: this env is rerun with the object paths
                stopped = true;
                active = false;
                continue;
            }
        }
        checkpoint();
        // ---- end of frame
        if (c.cyc < kCyclesPerFrame) c.cyc = kCyclesPerFrame;  // a jammed CPU lets the cycles elapse
        c.hook.finish_frame(c);
        c.next_frame();
        c.hook.pix_cc = c.hook.pix_cc > kClocksPerFrame ? c.hook.pix_cc - kClocksPerFrame : 0;
        ++frame;
        if (++fstep == F) {
            // ---- end of env step
            if constexpr (kTapeFwd) {
                if (c.hook.taping) c.hook.put(make_uint4(kRecStepEnd << 16, 0u, 0u, (uint32_t)s_idx));
            }
            if constexpr (kSoft) {
                if (P.ram_out_f) {
                    float4 *o = reinterpret_cast<float4 *>(P.ram_out_f + ((size_t)env * S + s_idx) * 128);
                    for (uint32_t w = sub; w < 32; w += G) {
                        const uint32_t v = c.mem.ram_word(w);
                        o[w] = make_float4((float)(v & 0xFFu), (float)((v >> 8) & 0xFFu),
                                           (float)((v >> 16) & 0xFFu), (float)(v >> 24));
                    }
                }
            } else {
                if (P.ram_out) {
                    uint32_t *o = reinterpret_cast<uint32_t *>(P.ram_out + ((size_t)env * S + s_idx) * 128);
                    for (uint32_t w = sub; w < 32; w += G) o[w] = c.mem.ram_word(w);
                }
            }
            ++ep_step;
            uint32_t done = 0;
            if (P.ep_steps && (int32_t)episode < P.num_episodes &&
                ep_step >= P.ep_steps[(size_t)env * P.num_episodes + episode]) {
                // episode over: in-run reset with SplitMix64 RAM for the next episode
                done = 1;
                ++episode;
                for (uint32_t w = sub; w < 16; w += G) {
                    const uint64_t v = reset_ram_word(P.seed, (uint64_t)env, episode, w);
                    c.mem.ram_word_set(2 * w, (uint32_t)v);
                    c.mem.ram_word_set(2 * w + 1, (uint32_t)(v >> 32));
                }
                if (c.sc) {  // and the Superchip RAM from its own stream
                    for (uint32_t w = sub; w < 16; w += G) {
                        const uint64_t v = reset_ram_word(P.seed ^ kScSeed, (uint64_t)env, episode, w);
                        c.mem.sc_word_set(2 * w, (uint32_t)v);
                        c.mem.sc_word_set(2 * w + 1, (uint32_t)(v >> 32));
                    }
                }
                c.power_on();
                X::init(c, xs);
                frame = 0;
                ep_step = 0;
            }
            if (P.done && sub == 0) P.done[(size_t)env * S + s_idx] = (uint8_t)done;
            fstep = 0;
            if (++s_idx == S) {
                active = false;
            } else {
                set_ports();
            }
        }
        if (active) start_frame();
    }
    c.hook.end_frames();

    // obj_flag: 1 for an env that needs (or ran) the object paths
    if (live && P.obj_flag && sub == 0) P.obj_flag[env] = (kObj || stopped) ? 1u : 0u;
    if (live && !stopped) {
        if (P.state) {
            StateRec &st = P.state[env];
            c.cx_upto(3 * c.cyc);  // collision latches current at the end of the call
            if (sub == 0) {
                c.store(st);
                st.frame = frame0 + frame;
                st.episode = episode;
                st.ep_step = ep_step;
            }
            if constexpr (!kPlain) {
                uint32_t *rw = reinterpret_cast<uint32_t *>(st.ram);
                for (uint32_t w = sub; w < 32; w += G) rw[w] = c.mem.ram_word(w);
                if (c.sc) {
                    uint32_t *sw = reinterpret_cast<uint32_t *>(P.sc_state + (size_t)env * 128);
                    for (uint32_t w = sub; w < 32; w += G) sw[w] = c.mem.sc_word(w);
                }
            }
        }
        if constexpr (kSoft) {
            if (P.ckpt_count && sub == 0) P.ckpt_count[env] = nckpt;
        }
        if constexpr (Mem::kRelax) {
            if (P.relax_out && sub == 0) {
                P.relax_out[(size_t)env * 2] = c.mem.ndiv;
                P.relax_out[(size_t)env * 2 + 1] = (int64_t)c.mem.fails;
            }
        }
    }
}

// Soft backward of one env, run by every lane of its wave: segments from last
// to first are recomputed from their checkpoint into the tape (the env's
// records, contiguous) and swept in reverse.  The sweep reads the records a
// wave-width at a time (lane l loads one record; the next batch is in flight
// while the current one is processed) and takes each one's fields from its lane
// with readlane, so its branches are scalar and no record load waits in the
// loop; the RAM adjoint lives in the lanes' registers (RamAdjoint).  ROM and
// port gradients are accumulated by lane 0 with no-return atomic adds (one
// lane per address: program order, deterministic).
// kObj: recompute with the object paths (an env whose forward needed them);
// without them for the others.
template <class W, bool kObj = true, class Mem>
__host__ __device__ __forceinline__ void bwd_env(const BwdParams &P, int32_t env, uint32_t gslot, uint32_t nslots,
                                                 int32_t mapper, uint32_t rom_n, Mem mem, const uint32_t *decode) {
    constexpr uint32_t NW = W::kWidth;
    (void)decode;  // the tape records carry the opcode class
    const uint32_t lane = W::lane();
    const bool lead = lane == 0;
    const bool live = env >= 0;
    const int32_t S = P.steps, F = P.frame_skip;
    RamAdjoint<W> adj;
    adj.zero();

    Cpu<Mem, TapeHook<W>, kObj> c;
    c.set_cart(mapper);  // (never a Superchip format: the soft path rejects them)
    c.mem = mem;
    c.hook.tape = P.tape + (size_t)gslot * (size_t)P.max_rec;  // the env's records, contiguous
    c.hook.max_rec = P.max_rec;
    c.hook.ystart = P.ystart;
    c.hook.overflow = P.overflow;
    c.hook.lead = lead;
    c.hook.read_T = P.read_T;
    c.hook.rom_n = rom_n;

    float aA = 0.f, aX = 0.f, aY = 0.f;
    float aC[4] = {0.f, 0.f, 0.f, 0.f};
    const float *gframe_env = live ? P.grad_frame + (size_t)env * kPixels : nullptr;
    // segment i starts from checkpoint i (checkpoint 0: the forward's starting state)
    const int32_t nseg = live ? (P.ckpt_count[env] < P.max_ckpt ? P.ckpt_count[env] : P.max_ckpt) : 0;

    float t_rd = 0.f;  // the adjoint the current record delivers to its read value
    auto add_src = [&](uint32_t cls, uint32_t idx, uint32_t step, float t) {
        t_rd = t;
        switch (cls) {
            case kClsRam: adj.set(idx, adj.get(idx) + t); break;
            case kClsRom: if (lead) W::accumulate(&P.gpart[(size_t)idx * nslots + gslot], t); break;
            case kClsSwcha: if (lead) W::accumulate(&P.gport[((size_t)env * S + step) * 2], t); break;
            case kClsInpt4: if (lead) W::accumulate(&P.gport[((size_t)env * S + step) * 2 + 1], t); break;
            case kClsRegA: aA += t; break;
            default: break;
        }
    };
    auto take_dst = [&](uint32_t cls, uint32_t idx) -> float {
        float t = 0.f;
        if (cls == kClsRam) {
            t = adj.get(idx);
            adj.set(idx, 0.f);
        } else if (cls == kClsCol) {
            t = aC[0] * (idx == 0) + aC[1] * (idx == 1) + aC[2] * (idx == 2) + aC[3] * (idx == 3);
            aC[0] = idx == 0 ? 0.f : aC[0];
            aC[1] = idx == 1 ? 0.f : aC[1];
            aC[2] = idx == 2 ? 0.f : aC[2];
            aC[3] = idx == 3 ? 0.f : aC[3];
        } else if (cls == kClsRegA) {
            t = aA;
            aA = 0.f;
        }
        return t;
    };
    auto zero_push = [&](uint32_t cell) {
        uint32_t idx;
        const uint32_t cls = write_class(0x100u | (cell & 0xFFu), &idx);
        (void)take_dst(cls, idx);
    };
    // the reverse-sweep rule of one record (fields already wave-uniform; pix(k) gives
    // its pixel sums, read only by the records that carry them)
    auto sweep_one = [&](uint32_t w0, uint32_t w1, uint32_t w2, uint32_t step, auto pix) {
        const uint32_t kind = (w0 >> 16) & 15u;
        if (kind == kRecStepEnd) {
            if (P.grad_ram_out) {
                const float *gr = P.grad_ram_out + ((size_t)env * S + step) * 128;
                for (uint32_t i = 0; i < RamAdjoint<W>::CPL; ++i) adj.v[i] += gr[lane + NW * i];
            }
            return;
        }
        if (kind == kRecPixels) {
            for (uint32_t k = 0; k < 4; ++k) aC[k] += pix(k);
            return;
        }
        const uint32_t rd = (w0 >> 8) & 15u, wr = (w0 >> 12) & 15u;
        const uint32_t rd_idx = w1 & 0xFFFFu, wr_idx = w1 >> 16;
        const float v1 = (float)(w2 & 0xFFu), v2 = (float)((w2 >> 8) & 0xFFu);
        const uint32_t sb = (w2 >> 16) & 0xFFu;
        const uint32_t cls = (w0 >> 24) & 63u;  // the opcode's class, recorded with it
        t_rd = 0.f;
        switch (cls) {
            case C_LDA: { const float t = aA; aA = 0.f; add_src(rd, rd_idx, step, t); break; }
            case C_LDX: { const float t = aX; aX = 0.f; add_src(rd, rd_idx, step, t); break; }
            case C_LDY: { const float t = aY; aY = 0.f; add_src(rd, rd_idx, step, t); break; }
            case C_LAX: { const float t = aA + aX; aA = aX = 0.f; add_src(rd, rd_idx, step, t); break; }
            case C_STA: aA += take_dst(wr, wr_idx); break;
            case C_STX: aX += take_dst(wr, wr_idx); break;
            case C_STY: aY += take_dst(wr, wr_idx); break;
            case C_SAX: {  // mem = A & X: d/dA = X/255, d/dX = A/255
                const float t = take_dst(wr, wr_idx);
                aA += t * (v2 / 255.f);
                aX += t * (v1 / 255.f);
                break;
            }
            case C_ADC: add_src(rd, rd_idx, step, aA); break;
            case C_SBC: add_src(rd, rd_idx, step, -aA); break;
            case C_AND: {  // A' = A & M with v1 = A, v2 = M
                const float t = aA;
                aA = t * (v2 / 255.f);
                add_src(rd, rd_idx, step, t * (v1 / 255.f));
                break;
            }
            case C_ORA: {
                const float t = aA;
                aA = t * ((255.f - v2) / 255.f);
                add_src(rd, rd_idx, step, t * ((255.f - v1) / 255.f));
                break;
            }
            case C_EOR: {
                const float t = aA;
                aA = t * ((255.f - 2.f * v2) / 255.f);
                add_src(rd, rd_idx, step, t * ((255.f - 2.f * v1) / 255.f));
                break;
            }
            case C_ASL: case C_ROL: case C_LSR: case C_ROR: case C_INC: case C_DEC: {
                const float k = (cls == C_ASL || cls == C_ROL) ? 2.f : (cls == C_LSR || cls == C_ROR) ? 0.5f : 1.f;
                const float t = take_dst(wr, wr_idx) * k;
                add_src(rd, rd_idx, step, t);
                break;
            }
            case C_TAX: aA += aX; aX = 0.f; break;
            case C_TAY: aA += aY; aY = 0.f; break;
            case C_TXA: aX += aA; aA = 0.f; break;
            case C_TYA: aY += aA; aA = 0.f; break;
            case C_TSX: aX = 0.f; break;
            case C_PHA: aA += take_dst(wr, wr_idx); break;
            case C_PLA: { const float t = aA; aA = 0.f; add_src(rd, rd_idx, step, t); break; }
            case C_PHP: zero_push(sb); break;
            case C_JSR: zero_push(sb); zero_push(sb - 1u); break;
            case C_BRK: zero_push(sb); zero_push(sb - 1u); zero_push(sb - 2u); break;
            default: break;  // flags, compares, branches, jumps, pulls into P/PC: no content
        }
        const uint32_t ik = (w0 >> 21) & 3u;  // address surrogate: the index register's share
        if (ik) {
            const float dk = t_rd * __builtin_bit_cast(float, step);
            aX += ik == 1u ? dk : 0.f;
            aY += ik == 2u ? dk : 0.f;
        }
        if (w0 & (1u << 20)) {  // pixels drawn before this instruction's write
            for (uint32_t k = 0; k < 4; ++k) aC[k] += pix(k);
        }
    };
    // reverse sweep of records [0, nrec), a batch of NW records at a time (lane l
    // loads record top - NW + l with load(i, words, pixel sums))
    auto sweep_tape = [&](int32_t nrec, auto load) {
        auto load_batch = [&](int32_t top, uint4 &a, float4 &b) {
            const int32_t i = top - (int32_t)NW + (int32_t)lane;
            if (i >= 0) {
                load(i, a, b);
            } else {
                a = make_uint4(0u, 0u, 0u, 0u);
                b = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        };
        uint4 ca;
        float4 cb;
        load_batch(nrec, ca, cb);
        for (int32_t top = nrec; top > 0; top -= (int32_t)NW) {
            const int32_t base = top - (int32_t)NW;  // lane l holds record base + l
            uint4 na;
            float4 nb;
            load_batch(base, na, nb);  // the next batch, in flight during this one
            const int32_t lo_i = base > 0 ? base : 0;
            for (int32_t i = top - 1; i >= lo_i; --i) {
                const uint32_t j = (uint32_t)(i - base);
                auto pix = [&](uint32_t k) {
                    return W::readlane(k == 0 ? cb.x : k == 1 ? cb.y : k == 2 ? cb.z : cb.w, j);
                };
                sweep_one(W::readlane(ca.x, j), W::readlane(ca.y, j), W::readlane(ca.z, j), W::readlane(ca.w, j),
                          pix);
            }
            ca = na;
            cb = nb;
        }
    };

    for (int32_t seg = nseg - 1; seg >= 0; --seg) {
        const StateRec &r = P.ckpt[(size_t)env * P.max_ckpt + seg];
        // ---- a segment the forward taped is swept from its tape (not with the
        // address surrogate, whose slopes need the arrays at the time of each read)
        const int32_t tape_n = P.ftape && P.read_T == 0.f ? (int32_t)W::first((uint32_t)r.tape_n) : -1;
        if (tape_n >= 0) {
            const uint4 *ft = P.ftape + (size_t)env * (size_t)P.ftape_cap + W::first(r.tape_off);
            sweep_tape(tape_n, [&](int32_t i, uint4 &a, float4 &b) {
                a = ft[i];
                b = make_float4(0.f, 0.f, 0.f, 0.f);
            });
            continue;
        }
        // ---- restore the segment's starting state
        c.load(r);
        const uint32_t *rw = reinterpret_cast<const uint32_t *>(r.ram);
        for (uint32_t w = lane; w < 32; w += NW) c.mem.ram_word_set(w, rw[w]);
        uint32_t frame = r.frame;
        c.hook.pix_cc = r.pix_cc;
        const int64_t seg_end = seg == nseg - 1 ? INT64_MAX : r.next_ckpt;
        int32_t s_idx = (int32_t)(frame / (uint32_t)F), fstep = (int32_t)(frame % (uint32_t)F);
        c.hook.nrec = 0;
        auto set_ports = [&]() {
            action_ports(P.actions[(size_t)env * S + s_idx], &c.swcha, &c.inpt4, &c.swchb);
            c.hook.step = (uint32_t)s_idx;
            c.hook.gframe = (s_idx == S - 1 && fstep == F - 1) ? gframe_env : nullptr;
        };
        bool rec_active = s_idx < S;
        if (rec_active) set_ports();

        // ---- recompute the segment, recording the tape
        while (rec_active) {
            // the instructions of this frame that start before the segment's end run
            // in a tight loop; the frame and segment bookkeeping sits outside it
            const int64_t rel = seg_end - (int64_t)frame * kCyclesPerFrame;  // segment end, frame-relative
            const int32_t lim = rel < (int64_t)kCyclesPerFrame ? (int32_t)rel : kCyclesPerFrame;
            while (!c.jam && c.cyc < lim) {
                uint32_t opc, lo, hi, dec;
                fetch_word<W>(c, opc, lo, hi, dec);
                ExecInfo info;
                // the wave runs one env, so its opcode is wave-uniform
                const uint32_t u = W::first(opc);
                const uint32_t d = W::first(dec);
                if (d == 0) c.jam = 1;
                else exec_dispatch<W>(c, u, d, lo, hi, info);
            }
            const int64_t g = (int64_t)frame * kCyclesPerFrame + c.cyc;
            if (g >= seg_end) {
                rec_active = false;
            } else {  // the frame is over (or the CPU jammed): its end
                if (c.cyc < kCyclesPerFrame) c.cyc = kCyclesPerFrame;
                if (c.hook.gframe) {  // tail of the final frame
                    TapeRec t;
                    t.w0 = kRecPixels << 16;
                    t.w1 = t.w2 = 0;
                    t.w3 = (uint32_t)s_idx;
                    t.pix[0] = t.pix[1] = t.pix[2] = t.pix[3] = 0.f;
                    pixel_sums_wave<W, kObj>(c.hook.gframe, c.hook.pix_cc, kClocksPerFrame, c.tia(), c.hook.ystart,
                                             t.pix);
                    c.hook.emit(t);
                }
                c.next_frame();
                c.hook.pix_cc = c.hook.pix_cc > kClocksPerFrame ? c.hook.pix_cc - kClocksPerFrame : 0;
                ++frame;
                if (++fstep == F) {
                    TapeRec t;
                    t.w0 = kRecStepEnd << 16;
                    t.w1 = t.w2 = 0;
                    t.w3 = (uint32_t)s_idx;
                    t.pix[0] = t.pix[1] = t.pix[2] = t.pix[3] = 0.f;
                    c.hook.emit(t);
                    fstep = 0;
                    if (++s_idx == S) rec_active = false;
                }
                if (rec_active) set_ports();
            }
        }

        // ---- reverse sweep of the segment's tape
        const int32_t nrec = c.hook.nrec < c.hook.max_rec ? c.hook.nrec : c.hook.max_rec;
        const TapeRec *tp = c.hook.tape;
        sweep_tape(nrec, [&](int32_t i, uint4 &a, float4 &b) {
            a = reinterpret_cast<const uint4 *>(tp + i)[0];
            b = reinterpret_cast<const float4 *>(tp + i)[1];
        });
    }
    // the RAM adjoint at the start reaches the tape only when the forward started
    // from power-on with the tape's RAM; a given starting state is a constant
    if (live) {
        const bool tape = nseg > 0 && P.ckpt[(size_t)env * P.max_ckpt].from_tape != 0u;
        for (uint32_t i = 0; i < RamAdjoint<W>::CPL; ++i)
            P.g_ram0[(size_t)env * 128 + lane + NW * i] = tape ? adj.v[i] : 0.f;
    }
}

}  // namespace vcs
