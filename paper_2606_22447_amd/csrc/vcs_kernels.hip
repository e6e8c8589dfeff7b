// HIP kernels of libvcs for gfx950 (MI355X).
//
//  k_step      hard env steps and the soft forward (paper Sec. "Hard and Soft
//              Execution"; Theorem "Exact forward equivalence": the soft forward
//              runs the hard machine on the decoded leaves).
//              PLAIN   = one env per thread, RAM/ROM in global memory, per-lane
//                        opcode switch (the baseline kernel).
//              GROUPED = ROM image and RAM staged in LDS, opcode dispatch made
//                        wave-uniform by a waterfall over the distinct opcodes
//                        of the wave (scalar decode), G lanes per env sharing
//                        the pixel writeback.
//  k_soft_bwd  surrogate backward: per env, segments from last to first are
//              recomputed from their hard-state checkpoint into a tape, then
//              swept in reverse with the straight-through rules.
//  k_decode_*  STE leaves: argmax bytes and softmax statistics (Eq. select).
//  k_*_grad    epilogue: fixed-order reduction of per-env ROM partials and the
//              softmax vector-Jacobian products.
#include <type_traits>

#include "vcs_core.hpp"
#include "vcs_kernels.hpp"

namespace vcs {

__constant__ DecodeTable kDecodeDev = make_decode_table();

// ---------------------------------------------------------------------------
// Memory policies
// ---------------------------------------------------------------------------
// LDS: ROM image bytes; RAM as words [32][E] so that the 4 bytes of a word
// belong to one env and neighbouring envs hit neighbouring banks.
struct LdsMem {
    const uint8_t *rom;
    uint8_t *ram;
    uint32_t E, slot;
    __device__ __forceinline__ uint32_t rom_byte(uint32_t off) const { return rom[off]; }
    __device__ __forceinline__ uint32_t ram_byte(uint32_t cell) const {
        return ram[(((cell >> 2) * E + slot) << 2) | (cell & 3u)];
    }
    __device__ __forceinline__ void ram_set(uint32_t cell, uint32_t v) {
        ram[(((cell >> 2) * E + slot) << 2) | (cell & 3u)] = (uint8_t)v;
    }
    __device__ __forceinline__ uint32_t ram_word(uint32_t w) const {
        return *reinterpret_cast<const uint32_t *>(ram + ((w * E + slot) << 2));
    }
    __device__ __forceinline__ void ram_word_set(uint32_t w, uint32_t v) {
        *reinterpret_cast<uint32_t *>(ram + ((w * E + slot) << 2)) = v;
    }
};

// Global memory: the env's ROM image and its 128 RAM bytes in the state record.
struct GlobalMem {
    const uint8_t *rom;
    uint8_t *ram;
    __device__ __forceinline__ uint32_t rom_byte(uint32_t off) const { return rom[off]; }
    __device__ __forceinline__ uint32_t ram_byte(uint32_t cell) const { return ram[cell]; }
    __device__ __forceinline__ void ram_set(uint32_t cell, uint32_t v) { ram[cell] = (uint8_t)v; }
    __device__ __forceinline__ uint32_t ram_word(uint32_t w) const { return reinterpret_cast<const uint32_t *>(ram)[w]; }
    __device__ __forceinline__ void ram_word_set(uint32_t w, uint32_t v) { reinterpret_cast<uint32_t *>(ram)[w] = v; }
};

// ---------------------------------------------------------------------------
// Hooks
// ---------------------------------------------------------------------------
// Renders the returned frame lazily: before every pixel-register write the
// pixels up to the write's effect clock are drawn with the old state.
template <typename T>
struct RenderHook {
    static constexpr bool kRecord = false;
    T *frame;         // frame being rendered, or nullptr
    int32_t rend_cc;  // frame-relative colour clock rendered up to
    int32_t pix_cc;   // write point of the last instruction (soft checkpoints)
    int32_t ystart;
    uint32_t sub, G;
    template <class C>
    __device__ __forceinline__ void before_pixel_write(C &c, int32_t w) {
        if (frame) {
            const int32_t cc = 3 * (w + 1);
            if (cc > rend_cc) {
                render_span(frame, rend_cc, cc, c.col, c.pf, c.vb, ystart, sub, G);
                rend_cc = cc;
            }
        }
    }
    template <class C>
    __device__ __forceinline__ void before_exec(C &) {}
    template <class C>
    __device__ __forceinline__ void after_exec(C &, uint32_t, int32_t, int32_t wp, ExecInfo &) {
        pix_cc = 3 * wp;
    }
    template <class C>
    __device__ __forceinline__ void finish_frame(C &c) {
        if (frame) render_span(frame, rend_cc, kClocksPerFrame, c.col, c.pf, c.vb, ystart, sub, G);
    }
};

// Records the recompute tape of the soft backward.  Pixels of the final frame
// are attributed to the instruction during whose span [previous write point,
// this write point) they were drawn, with the state before its write.
struct TapeHook {
    static constexpr bool kRecord = true;
    TapeRec *tape;
    uint32_t stride;
    int32_t nrec, max_rec;
    const float *gframe;  // env's dL/dframe while in the final frame, else nullptr
    int32_t pix_cc;
    int32_t ystart;
    uint32_t step;
    uint32_t save_pf, save_vb;
    int32_t *overflow;
    __device__ __forceinline__ void emit(const TapeRec &r) {
        if (nrec < max_rec) tape[(size_t)nrec * stride] = r;
        else *overflow = 1;
        ++nrec;
    }
    template <class C>
    __device__ __forceinline__ void before_pixel_write(C &, int32_t) {}
    template <class C>
    __device__ __forceinline__ void before_exec(C &c) {
        save_pf = c.pf;
        save_vb = c.vb;
    }
    template <class C>
    __device__ __forceinline__ void after_exec(C &, uint32_t opc, int32_t, int32_t wp, ExecInfo &info) {
        TapeRec r;
        r.w0 = opc | (info.rd_cls << 8) | (info.wr_cls << 12) | (kRecInstr << 16);
        r.w1 = info.rd_idx | (info.wr_idx << 16);
        r.w2 = (info.v1 & 0xFFu) | ((info.v2 & 0xFFu) << 8) | ((info.s_before & 0xFFu) << 16);
        r.w3 = step;
        r.pix[0] = r.pix[1] = r.pix[2] = r.pix[3] = 0.f;
        if (gframe && pixel_sums(gframe, pix_cc, 3 * wp, save_pf, save_vb, ystart, r.pix)) r.w0 |= 1u << 20;
        pix_cc = 3 * wp;
        emit(r);
    }
};

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool wave_any(bool v) { return __ballot(v) != 0; }

// ---------------------------------------------------------------------------
// Step kernel (hard steps, soft forward)
// ---------------------------------------------------------------------------
template <int G, int TPB, bool kSoft, bool kPlain>
__global__ __launch_bounds__(TPB) void k_step(StepParams P) {
    static_assert(!(kSoft && kPlain), "the soft forward uses the grouped kernel");
    constexpr int E = TPB / G;
    using T = typename std::conditional<kSoft, float, uint8_t>::type;
    using Mem = typename std::conditional<kPlain, GlobalMem, LdsMem>::type;
    __shared__ __align__(16) uint8_t rom_lds[kPlain ? 16 : 8192];
    __shared__ __align__(16) uint32_t ram_lds[kPlain ? 4 : 32 * E];

    const uint32_t tid = threadIdx.x, slot = tid / G, sub = tid % G;
    const int32_t blk = blockIdx.x;
    const int32_t rom_idx = P.st.main_block_rom[blk];
    const int32_t env = P.st.main_slot_env[blk * E + slot];
    const int32_t rom_base = P.st.rom_off[rom_idx], rom_size = P.st.rom_size[rom_idx];
    const int32_t mapper = P.st.rom_mapper[rom_idx];
    const bool live = env >= 0;
    const int32_t S = P.steps, F = P.frame_skip;

    Cpu<Mem, RenderHook<T>> c;
    c.amask = mapper == 0 ? 0x7FFu : 0xFFFu;
    c.f8 = mapper == 2 ? 1u : 0u;
    if constexpr (kPlain) {
        c.mem.rom = P.rom + rom_base;
        c.mem.ram = live ? P.state[env].ram : nullptr;
    } else {
        for (int32_t i = (int32_t)tid * 16; i < rom_size; i += TPB * 16)
            *reinterpret_cast<uint4 *>(rom_lds + i) = *reinterpret_cast<const uint4 *>(P.rom + rom_base + i);
        c.mem.rom = rom_lds;
        c.mem.ram = reinterpret_cast<uint8_t *>(ram_lds);
        c.mem.E = E;
        c.mem.slot = slot;
    }
    c.hook.frame = nullptr;
    c.hook.rend_cc = 0;
    c.hook.pix_cc = 0;
    c.hook.ystart = P.ystart;
    c.hook.sub = sub;
    c.hook.G = G;
    uint32_t frame = 0, episode = 0, ep_step = 0;
    if (live) {
        if (P.ram0) {  // soft forward: power-on with the decoded RAM
            const uint32_t *r0 = reinterpret_cast<const uint32_t *>(P.ram0 + (size_t)env * 128);
            for (uint32_t w = sub; w < 32; w += G) c.mem.ram_word_set(w, r0[w]);
        } else {
            const StateRec &st = P.state[env];
            c.load(st);
            c.bank &= c.f8;  // only F8 images have a second bank
            frame = st.frame;
            episode = st.episode;
            ep_step = st.ep_step;
            if constexpr (!kPlain) {
                const uint32_t *rw = reinterpret_cast<const uint32_t *>(st.ram);
                for (uint32_t w = sub; w < 32; w += G) c.mem.ram_word_set(w, rw[w]);
            }
        }
    }
    __syncthreads();  // ROM and RAM staged
    if (live && P.ram0) c.power_on();
    if (live && !P.ram0 && (P.state[env].status & 2u)) {  // power-on requested by vcs_reset
        c.power_on();
        frame = 0;
    }

    int32_t s_idx = 0, fstep = 0;
    bool active = live && S > 0;
    auto set_ports = [&]() {
        const uint32_t act = P.actions ? P.actions[(size_t)env * S + s_idx] : 0u;
        action_ports(act, &c.swcha, &c.inpt4);
    };
    auto start_frame = [&]() {
        c.hook.rend_cc = 0;
        c.hook.frame = nullptr;
        const bool last_of_step = fstep == F - 1;
        if constexpr (kSoft) {
            if (P.frame_out_f && last_of_step && s_idx == S - 1) c.hook.frame = P.frame_out_f + (size_t)env * kPixels;
        } else {
            if (P.frame_out && last_of_step) {
                if (P.frames_mode == 2) c.hook.frame = P.frame_out + ((size_t)env * S + s_idx) * kPixels;
                else if (P.frames_mode == 1 && s_idx == S - 1) c.hook.frame = P.frame_out + (size_t)env * kPixels;
            }
        }
    };
    if (active) {
        set_ports();
        start_frame();
    }
    // soft forward: hard-state checkpoints every K cycles since power-on
    int64_t next_ckpt = P.ckpt_interval;
    int32_t nckpt = 0;

    while (wave_any(active)) {
        if (active) {
            if constexpr (kSoft) {
                if (P.ckpt) {
                    const int64_t g = (int64_t)frame * kCyclesPerFrame + c.cyc;
                    if (g >= next_ckpt) {
                        next_ckpt = (g / P.ckpt_interval + 1) * P.ckpt_interval;
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
                            }
                            uint32_t *rw = reinterpret_cast<uint32_t *>(r.ram);
                            for (uint32_t w = sub; w < 32; w += G) rw[w] = c.mem.ram_word(w);
                        }
                        ++nckpt;
                    }
                }
            }
            if (c.jam || c.cyc >= kCyclesPerFrame) {
                // ---- end of frame
                if (c.cyc < kCyclesPerFrame) c.cyc = kCyclesPerFrame;  // a jammed CPU lets the cycles elapse
                c.hook.finish_frame(c);
                c.next_frame();
                c.hook.pix_cc = c.hook.pix_cc > kClocksPerFrame ? c.hook.pix_cc - kClocksPerFrame : 0;
                ++frame;
                if (++fstep == F) {
                    // ---- end of env step
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
                        c.power_on();
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
            } else {
                // ---- one instruction
                const uint32_t pc = c.pc;
                const uint32_t opc = c.peek(pc, c.cyc);
                const uint32_t lo = c.peek((pc + 1u) & 0xFFFFu, c.cyc);
                const uint32_t hi = c.peek((pc + 2u) & 0xFFFFu, c.cyc);
                ExecInfo info;
                if constexpr (kPlain) {
                    const uint32_t d = kDecodeDev.e[opc];
                    if (d == 0) c.jam = 1;
                    else c.exec(opc, d, lo, hi, info);
                } else {
                    // waterfall: each pass executes one distinct opcode of the wave
                    // with a wave-uniform (scalar) decode
                    for (;;) {
                        const uint32_t u = __builtin_amdgcn_readfirstlane(opc);
                        if (opc == u) {
                            const uint32_t d = kDecodeDev.e[u];
                            if (d == 0) c.jam = 1;
                            else c.exec(u, d, lo, hi, info);
                            break;
                        }
                    }
                }
            }
        }
    }

    if (live) {
        if (P.state) {
            StateRec &st = P.state[env];
            if (sub == 0) {
                c.store(st);
                st.frame = frame;
                st.episode = episode;
                st.ep_step = ep_step;
            }
            if constexpr (!kPlain) {
                uint32_t *rw = reinterpret_cast<uint32_t *>(st.ram);
                for (uint32_t w = sub; w < 32; w += G) rw[w] = c.mem.ram_word(w);
            }
        }
        if constexpr (kSoft) {
            if (P.ckpt_count && sub == 0) P.ckpt_count[env] = nckpt;
        }
    }
}

// ---------------------------------------------------------------------------
// Soft backward
// ---------------------------------------------------------------------------
constexpr int kBwdTPB = 64;

__global__ __launch_bounds__(kBwdTPB) void k_soft_bwd(BwdParams P) {
    constexpr int E = kBwdTPB;
    __shared__ __align__(16) uint8_t rom_lds[8192];
    __shared__ __align__(16) uint32_t ram_lds[32 * E];
    __shared__ float adj_ram[128 * E];

    const uint32_t tid = threadIdx.x, slot = tid;
    const int32_t blk = blockIdx.x;
    const uint32_t nslots = (uint32_t)gridDim.x * E;
    const uint32_t gslot = (uint32_t)blk * E + slot;
    const int32_t rom_idx = P.st.bwd_block_rom[blk];
    const int32_t env = P.st.bwd_slot_env[gslot];
    const int32_t rom_base = P.st.rom_off[rom_idx], rom_size = P.st.rom_size[rom_idx];
    const int32_t mapper = P.st.rom_mapper[rom_idx];
    const bool live = env >= 0;
    const int32_t S = P.steps, F = P.frame_skip, K = P.ckpt_interval;

    for (int32_t i = (int32_t)tid * 16; i < rom_size; i += kBwdTPB * 16)
        *reinterpret_cast<uint4 *>(rom_lds + i) = *reinterpret_cast<const uint4 *>(P.rom + rom_base + i);
    for (uint32_t cidx = 0; cidx < 128; ++cidx) adj_ram[cidx * E + slot] = 0.f;
    __syncthreads();

    Cpu<LdsMem, TapeHook> c;
    c.amask = mapper == 0 ? 0x7FFu : 0xFFFu;
    c.f8 = mapper == 2 ? 1u : 0u;
    c.mem.rom = rom_lds;
    c.mem.ram = reinterpret_cast<uint8_t *>(ram_lds);
    c.mem.E = E;
    c.mem.slot = slot;
    c.hook.tape = P.tape + gslot;
    c.hook.stride = nslots;
    c.hook.max_rec = P.max_rec;
    c.hook.ystart = P.ystart;
    c.hook.overflow = P.overflow;

    float aA = 0.f, aX = 0.f, aY = 0.f;
    float aC[4] = {0.f, 0.f, 0.f, 0.f};
    const float *gframe_env = live ? P.grad_frame + (size_t)env * kPixels : nullptr;
    const int32_t nck = live ? (P.ckpt_count[env] < P.max_ckpt ? P.ckpt_count[env] : P.max_ckpt) : 0;
    const int32_t nseg = live ? nck + 1 : 0;
    int32_t seg = nseg - 1;

    auto add_src = [&](uint32_t cls, uint32_t idx, uint32_t step, float t) {
        switch (cls) {
            case kClsRam: adj_ram[idx * E + slot] += t; break;
            case kClsRom: P.gpart[(size_t)idx * nslots + gslot] += t; break;
            case kClsSwcha: P.gport[((size_t)env * S + step) * 2] += t; break;
            case kClsInpt4: P.gport[((size_t)env * S + step) * 2 + 1] += t; break;
            case kClsRegA: aA += t; break;
            default: break;
        }
    };
    auto take_dst = [&](uint32_t cls, uint32_t idx) -> float {
        float t = 0.f;
        if (cls == kClsRam) {
            t = adj_ram[idx * E + slot];
            adj_ram[idx * E + slot] = 0.f;
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

    while (wave_any(seg >= 0)) {
        if (seg >= 0) {
            // ---- restore the segment's starting state
            int64_t seg_end;
            uint32_t frame;
            if (seg == 0) {
                const uint32_t *r0 = reinterpret_cast<const uint32_t *>(P.ram0 + (size_t)env * 128);
                for (uint32_t w = 0; w < 32; ++w) c.mem.ram_word_set(w, r0[w]);
                c.power_on();
                frame = 0;
                c.hook.pix_cc = 0;
                seg_end = K;
            } else {
                const StateRec &r = P.ckpt[(size_t)env * P.max_ckpt + (seg - 1)];
                c.load(r);
                c.bank &= c.f8;
                const uint32_t *rw = reinterpret_cast<const uint32_t *>(r.ram);
                for (uint32_t w = 0; w < 32; ++w) c.mem.ram_word_set(w, rw[w]);
                frame = r.frame;
                c.hook.pix_cc = r.pix_cc;
                seg_end = r.next_ckpt;
            }
            if (seg == nseg - 1) seg_end = INT64_MAX;
            int32_t s_idx = (int32_t)(frame / (uint32_t)F), fstep = (int32_t)(frame % (uint32_t)F);
            c.hook.nrec = 0;
            auto set_ports = [&]() {
                action_ports(P.actions[(size_t)env * S + s_idx], &c.swcha, &c.inpt4);
                c.hook.step = (uint32_t)s_idx;
                c.hook.gframe = (s_idx == S - 1 && fstep == F - 1) ? gframe_env : nullptr;
            };
            bool rec_active = s_idx < S;
            if (rec_active) set_ports();

            // ---- recompute the segment, recording the tape
            while (wave_any(rec_active)) {
                if (rec_active) {
                    const int64_t g = (int64_t)frame * kCyclesPerFrame + c.cyc;
                    if (g >= seg_end) {
                        rec_active = false;
                    } else if (c.jam || c.cyc >= kCyclesPerFrame) {
                        if (c.cyc < kCyclesPerFrame) c.cyc = kCyclesPerFrame;
                        if (c.hook.gframe) {  // tail of the final frame
                            TapeRec r;
                            r.w0 = kRecPixels << 16;
                            r.w1 = r.w2 = 0;
                            r.w3 = (uint32_t)s_idx;
                            r.pix[0] = r.pix[1] = r.pix[2] = r.pix[3] = 0.f;
                            pixel_sums(c.hook.gframe, c.hook.pix_cc, kClocksPerFrame, c.pf, c.vb, c.hook.ystart, r.pix);
                            c.hook.emit(r);
                        }
                        c.next_frame();
                        c.hook.pix_cc = c.hook.pix_cc > kClocksPerFrame ? c.hook.pix_cc - kClocksPerFrame : 0;
                        ++frame;
                        if (++fstep == F) {
                            TapeRec r;
                            r.w0 = kRecStepEnd << 16;
                            r.w1 = r.w2 = 0;
                            r.w3 = (uint32_t)s_idx;
                            r.pix[0] = r.pix[1] = r.pix[2] = r.pix[3] = 0.f;
                            c.hook.emit(r);
                            fstep = 0;
                            if (++s_idx == S) rec_active = false;
                        }
                        if (rec_active) set_ports();
                    } else {
                        const uint32_t pc = c.pc;
                        const uint32_t opc = c.peek(pc, c.cyc);
                        const uint32_t lo = c.peek((pc + 1u) & 0xFFFFu, c.cyc);
                        const uint32_t hi = c.peek((pc + 2u) & 0xFFFFu, c.cyc);
                        ExecInfo info;
                        for (;;) {
                            const uint32_t u = __builtin_amdgcn_readfirstlane(opc);
                            if (opc == u) {
                                const uint32_t d = kDecodeDev.e[u];
                                if (d == 0) c.jam = 1;
                                else c.exec(u, d, lo, hi, info);
                                break;
                            }
                        }
                    }
                }
            }

            // ---- reverse sweep of the segment's tape
            const int32_t nrec = c.hook.nrec < c.hook.max_rec ? c.hook.nrec : c.hook.max_rec;
            for (int32_t i = nrec - 1; i >= 0; --i) {
                const TapeRec r = c.hook.tape[(size_t)i * nslots];
                const uint32_t kind = (r.w0 >> 16) & 15u;
                const uint32_t step = r.w3;
                if (kind == kRecStepEnd) {
                    if (P.grad_ram_out) {
                        const float *gr = P.grad_ram_out + ((size_t)env * S + step) * 128;
                        for (uint32_t cidx = 0; cidx < 128; ++cidx) adj_ram[cidx * E + slot] += gr[cidx];
                    }
                    continue;
                }
                if (kind == kRecPixels) {
                    aC[0] += r.pix[0];
                    aC[1] += r.pix[1];
                    aC[2] += r.pix[2];
                    aC[3] += r.pix[3];
                    continue;
                }
                const uint32_t opc = r.w0 & 0xFFu;
                const uint32_t rd = (r.w0 >> 8) & 15u, wr = (r.w0 >> 12) & 15u;
                const uint32_t rd_idx = r.w1 & 0xFFFFu, wr_idx = r.w1 >> 16;
                const float v1 = (float)(r.w2 & 0xFFu), v2 = (float)((r.w2 >> 8) & 0xFFu);
                const uint32_t sb = (r.w2 >> 16) & 0xFFu;
                const uint32_t d = kDecodeDev.e[opc];
                const uint32_t cls = d & 63u;
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
                if (r.w0 & (1u << 20)) {  // pixels drawn before this instruction's write
                    aC[0] += r.pix[0];
                    aC[1] += r.pix[1];
                    aC[2] += r.pix[2];
                    aC[3] += r.pix[3];
                }
            }
            --seg;
        }
    }
    if (live)
        for (uint32_t cidx = 0; cidx < 128; ++cidx) P.g_ram0[(size_t)env * 128 + cidx] = adj_ram[cidx * E + slot];
}

// ---------------------------------------------------------------------------
// Decode: STE leaves (argmax, lowest index on ties) and softmax statistics
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// (value, index) maximum with ties to the lower index, combined over the wave
__device__ __forceinline__ void wave_argmax(float &v, int &idx) {
    for (int o = 32; o > 0; o >>= 1) {
        const float ov = __shfl_xor(v, o, 64);
        const int oi = __shfl_xor(idx, o, 64);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
}

// Row statistics of 256 logits held as one float4 per lane (k = 4*lane + j):
// max, argmax, Z = sum exp((L-max)/tau), ev = sum k w_k.
struct RowStats {
    float m, z, ev;
    int arg;
};
__device__ __forceinline__ RowStats row_stats(const float4 L, float tau, uint32_t lane) {
    const float l[4] = {L.x, L.y, L.z, L.w};
    float v = l[0];
    int idx = (int)lane * 4;
    for (int j = 1; j < 4; ++j)
        if (l[j] > v) {
            v = l[j];
            idx = (int)lane * 4 + j;
        }
    wave_argmax(v, idx);
    float z = 0.f, e = 0.f;
    for (int j = 0; j < 4; ++j) {
        const float w = expf((l[j] - v) / tau);
        z += w;
        e += w * (float)(lane * 4 + j);
    }
    z = wave_sum(z);
    e = wave_sum(e);
    return RowStats{v, z, e / z, idx};
}

// ROM rows: one wave per row, 4 rows per block.
__global__ __launch_bounds__(256) void k_decode_rom(const float *logits, int64_t rows, float tau, uint8_t *hard,
                                                    float *stats) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (row >= rows) return;
    const float4 L = reinterpret_cast<const float4 *>(logits + row * 256)[lane];
    const RowStats r = row_stats(L, tau, lane);
    if (lane == 0) {
        hard[row] = (uint8_t)r.arg;
        stats[row * 3 + 0] = r.ev;
        stats[row * 3 + 1] = r.m;
        stats[row * 3 + 2] = r.z;
    }
}

// RAM tape rows (content, not logits): argmax and ev = sum_k k P[k].
__global__ __launch_bounds__(256) void k_decode_tape(const float *tape, int64_t rows, uint8_t *hard, float *ev) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (row >= rows) return;
    const float4 P4 = reinterpret_cast<const float4 *>(tape + row * 256)[lane];
    const float p[4] = {P4.x, P4.y, P4.z, P4.w};
    float v = p[0];
    int idx = (int)lane * 4;
    float e = 0.f;
    for (int j = 0; j < 4; ++j) {
        if (j && p[j] > v) {
            v = p[j];
            idx = (int)lane * 4 + j;
        }
        e += (float)(lane * 4 + j) * p[j];
    }
    wave_argmax(v, idx);
    e = wave_sum(e);
    if (lane == 0) {
        hard[row] = (uint8_t)idx;
        ev[row] = e;
    }
}

// Action rows: one thread per (env, step).
__global__ __launch_bounds__(256) void k_decode_act(const float *logits, int64_t rows, float tau, uint8_t *hard,
                                                    float *stats) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= rows) return;
    const float *L = logits + row * 18;
    int best = 0;
    for (int j = 1; j < 18; ++j)
        if (L[j] > L[best]) best = j;
    const float m = L[best];
    float z = 0.f, es = 0.f, ei = 0.f;
    for (int j = 0; j < 18; ++j) {
        const float w = expf((L[j] - m) / tau);
        uint32_t sw, in;
        action_ports((uint32_t)j, &sw, &in);
        z += w;
        es += w * (float)sw;
        ei += w * (float)in;
    }
    hard[row] = (uint8_t)best;
    stats[row * 2 + 0] = es / z;
    stats[row * 2 + 1] = ei / z;
}

// ---------------------------------------------------------------------------
// Epilogue
// ---------------------------------------------------------------------------
// dL/dL[a,k] = g[a] w_k (k - ev_a)/tau, with g[a] the fixed-order (float64)
// sum of the per-env partials of every env that runs ROM r.
__global__ __launch_bounds__(256) void k_rom_grad(const float *logits, const float *stats, const float *gpart,
                                                  int64_t rows, int32_t num_roms, const int32_t *rom_off,
                                                  const int32_t *rom_size, const int32_t *slot_begin,
                                                  const int32_t *slot_end, uint32_t nslots, float tau, float *out) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (row >= rows) return;
    int32_t r = 0;
    while (r + 1 < num_roms && (int64_t)rom_off[r + 1] <= row) ++r;
    const int64_t a = row - rom_off[r];
    double acc = 0.0;
    for (int32_t i = slot_begin[r] + (int32_t)lane; i < slot_end[r]; i += 64) acc += (double)gpart[a * nslots + i];
    const float g = (float)wave_sum_d(acc);
    const float4 L = reinterpret_cast<const float4 *>(logits + row * 256)[lane];
    const float ev = stats[row * 3 + 0], m = stats[row * 3 + 1], z = stats[row * 3 + 2];
    const float l[4] = {L.x, L.y, L.z, L.w};
    float o[4];
    for (int j = 0; j < 4; ++j) {
        const float w = expf((l[j] - m) / tau) / z;
        o[j] = g * w * ((float)(lane * 4 + j) - ev) / tau;
    }
    reinterpret_cast<float4 *>(out + row * 256)[lane] = make_float4(o[0], o[1], o[2], o[3]);
    (void)rom_size;
}

// dL/dP0[c,k] = k * g0[c]
__global__ __launch_bounds__(256) void k_tape_grad(const float *g0, int64_t rows, float *out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;  // float4 index
    if (i >= rows * 64) return;
    const int64_t row = i >> 6;
    const float g = g0[row];
    const float k = (float)((i & 63) * 4);
    reinterpret_cast<float4 *>(out)[i] = make_float4(k * g, (k + 1.f) * g, (k + 2.f) * g, (k + 3.f) * g);
}

// dL/dl[a] = (w_a / tau) (g_sw (SWCHA(a) - E SWCHA) + g_in (INPT4(a) - E INPT4))
__global__ __launch_bounds__(256) void k_act_grad(const float *logits, const float *stats, const float *gport,
                                                  int64_t rows, float tau, float *out) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= rows) return;
    const float *L = logits + row * 18;
    float m = L[0];
    for (int j = 1; j < 18; ++j) m = fmaxf(m, L[j]);
    float z = 0.f;
    for (int j = 0; j < 18; ++j) z += expf((L[j] - m) / tau);
    const float es = stats[row * 2], ei = stats[row * 2 + 1];
    const float gs = gport[row * 2], gi = gport[row * 2 + 1];
    for (int j = 0; j < 18; ++j) {
        uint32_t sw, in;
        action_ports((uint32_t)j, &sw, &in);
        const float w = expf((L[j] - m) / tau) / z;
        out[row * 18 + j] = (w / tau) * (gs * ((float)sw - es) + gi * ((float)in - ei));
    }
}

// ---------------------------------------------------------------------------
// Reset and inspection
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reset(StateRec *state, int32_t B, const uint8_t *mask, const uint8_t *ram0,
                                               uint64_t seed) {
    const int32_t env = blockIdx.x * 256 + threadIdx.x;
    if (env >= B) return;
    if (mask && !mask[env]) return;
    StateRec &r = state[env];
    uint32_t *rw = reinterpret_cast<uint32_t *>(r.ram);
    if (ram0) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(ram0 + (size_t)env * 128);
        for (int w = 0; w < 32; ++w) rw[w] = src[w];
    } else {
        for (uint32_t w = 0; w < 16; ++w) {
            const uint64_t v = reset_ram_word(seed, (uint64_t)env, 0, w);
            rw[2 * w] = (uint32_t)v;
            rw[2 * w + 1] = (uint32_t)(v >> 32);
        }
    }
    r.magic = kMagic;
    r.a = r.x = r.y = 0;
    r.s = 0xFD;
    r.p = (uint8_t)(kFlagI | kFlagU);
    r.pc = 0;
    r.bank = 0;
    r.status = 2;  // power-on pending: the step kernel loads PC from the reset vector
    r.tim_shift = 10;
    r.vblank = r.vsync = 0;
    r.cyc = 0;
    r.frame = 0;
    r.tim_u = 0;
    r.tim_read = 0;
    r.col = r.pf = 0;
    r.episode = 0;
    r.ep_step = 0;
    r.next_ckpt = 0;
    r.pix_cc = 0;
    r.ckpt_index = 0;
}

__global__ __launch_bounds__(256) void k_read_regs(const StateRec *state, int32_t B, uint8_t *out) {
    const int32_t env = blockIdx.x * 256 + threadIdx.x;
    if (env >= B) return;
    const StateRec &r = state[env];
    const int32_t t = r.cyc;
    const int32_t dd = t - r.tim_u;
    const uint32_t intim = dd < 0 ? ((uint32_t)(-1 - (dd >> r.tim_shift)) & 0xFFu) : ((uint32_t)(255 - dd) & 0xFFu);
    const uint32_t timint = (t >= r.tim_u && r.tim_read < r.tim_u) ? 0x80u : 0u;
    uint8_t *o = out + (size_t)env * 16;
    o[0] = r.a; o[1] = r.x; o[2] = r.y; o[3] = r.s; o[4] = r.p;
    o[5] = (uint8_t)(r.pc & 0xFF); o[6] = (uint8_t)(r.pc >> 8); o[7] = r.bank; o[8] = r.status;
    o[9] = (uint8_t)intim; o[10] = (uint8_t)timint; o[11] = r.vblank;
    o[12] = (uint8_t)(r.col & 0xFF); o[13] = (uint8_t)((r.col >> 8) & 0xFF);
    o[14] = (uint8_t)((r.col >> 16) & 0xFF); o[15] = (uint8_t)(r.col >> 24);
}

__global__ void k_fill_zero(uint32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int G, int TPB, bool kSoft, bool kPlain>
static hipError_t launch_step_t(const StepParams &P, int32_t blocks, hipStream_t stream) {
    hipLaunchKernelGGL((k_step<G, TPB, kSoft, kPlain>), dim3(blocks), dim3(TPB), 0, stream, P);
    return hipGetLastError();
}

hipError_t launch_step(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, bool soft, bool plain,
                       hipStream_t stream) {
    if (plain) {
        if (soft || lanes != 1) return hipErrorInvalidValue;
        return tpb == 64 ? launch_step_t<1, 64, false, true>(P, blocks, stream)
                         : launch_step_t<1, 256, false, true>(P, blocks, stream);
    }
#define VCS_STEP_CASE(Gv, Tv)                                                                \
    if (lanes == Gv && tpb == Tv)                                                            \
        return soft ? launch_step_t<Gv, Tv, true, false>(P, blocks, stream)                  \
                    : launch_step_t<Gv, Tv, false, false>(P, blocks, stream);
    VCS_STEP_CASE(1, 64)
    VCS_STEP_CASE(1, 256)
    VCS_STEP_CASE(4, 64)
    VCS_STEP_CASE(4, 256)
    VCS_STEP_CASE(16, 64)
    VCS_STEP_CASE(16, 256)
#undef VCS_STEP_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_soft_bwd(const BwdParams &P, int32_t blocks, hipStream_t stream) {
    hipLaunchKernelGGL(k_soft_bwd, dim3(blocks), dim3(kBwdTPB), 0, stream, P);
    return hipGetLastError();
}

hipError_t launch_decode(const float *rom_logits, int64_t rom_rows, const float *tape, int64_t tape_rows,
                         const float *act_logits, int64_t act_rows, float tau, uint8_t *rom_hard, float *rom_stats,
                         uint8_t *ram0_hard, float *tape_ev, uint8_t *act_hard, float *act_stats, hipStream_t stream) {
    if (rom_rows) hipLaunchKernelGGL(k_decode_rom, dim3((unsigned)((rom_rows + 3) / 4)), dim3(256), 0, stream,
                                     rom_logits, rom_rows, tau, rom_hard, rom_stats);
    if (tape_rows) hipLaunchKernelGGL(k_decode_tape, dim3((unsigned)((tape_rows + 3) / 4)), dim3(256), 0, stream,
                                      tape, tape_rows, ram0_hard, tape_ev);
    if (act_rows) hipLaunchKernelGGL(k_decode_act, dim3((unsigned)((act_rows + 255) / 256)), dim3(256), 0, stream,
                                     act_logits, act_rows, tau, act_hard, act_stats);
    return hipGetLastError();
}

hipError_t launch_epilogue(const float *rom_logits, const float *rom_stats, const float *gpart, int64_t rom_rows,
                           int32_t num_roms, const int32_t *rom_off, const int32_t *rom_size,
                           const int32_t *slot_begin, const int32_t *slot_end, uint32_t nslots, float tau,
                           float *grad_rom, const float *g0, int64_t tape_rows, float *grad_tape,
                           const float *act_logits, const float *act_stats, const float *gport, int64_t act_rows,
                           float *grad_act, hipStream_t stream) {
    if (rom_rows) hipLaunchKernelGGL(k_rom_grad, dim3((unsigned)((rom_rows + 3) / 4)), dim3(256), 0, stream,
                                     rom_logits, rom_stats, gpart, rom_rows, num_roms, rom_off, rom_size, slot_begin,
                                     slot_end, nslots, tau, grad_rom);
    if (tape_rows) hipLaunchKernelGGL(k_tape_grad, dim3((unsigned)((tape_rows * 64 + 255) / 256)), dim3(256), 0,
                                      stream, g0, tape_rows, grad_tape);
    if (act_rows) hipLaunchKernelGGL(k_act_grad, dim3((unsigned)((act_rows + 255) / 256)), dim3(256), 0, stream,
                                     act_logits, act_stats, gport, act_rows, tau, grad_act);
    return hipGetLastError();
}

hipError_t launch_reset(StateRec *state, int32_t B, const uint8_t *mask, const uint8_t *ram0, uint64_t seed,
                        hipStream_t stream) {
    hipLaunchKernelGGL(k_reset, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, state, B, mask, ram0, seed);
    return hipGetLastError();
}

hipError_t launch_read_regs(const StateRec *state, int32_t B, uint8_t *out, hipStream_t stream) {
    hipLaunchKernelGGL(k_read_regs, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, state, B, out);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t stream) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, stream, (uint32_t *)p, n);
    return hipGetLastError();
}

}  // namespace vcs
