// HIP kernels of libvcs for gfx950 (MI355X).
//
//  The step kernels (k_step, k_step_relaxed, k_soft_bwd) are in
//  vcs_step_kernels.hpp and instantiated by vcs_step_hard.hip,
//  vcs_step_soft.hip and vcs_step_relaxed.hip (compiled in parallel).
//  k_decode_*  STE leaves: argmax bytes and softmax statistics (Eq. select).
//  k_*_grad    epilogue: fixed-order reduction of per-env ROM partials and the
//              softmax vector-Jacobian products.
#include "vcs_device.hpp"
#include "vcs_kernels.hpp"

namespace vcs {

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

// Offset of the softmax expectation from the argmax, delta = sum_k (k - arg) w_k,
// accumulated without the cancellation of (k - ev) near the argmax.
__device__ __forceinline__ float row_delta(const float4 L, float tau, uint32_t lane, float m, float z, int arg) {
    const float l[4] = {L.x, L.y, L.z, L.w};
    float d = 0.f;
    for (int j = 0; j < 4; ++j) d += expf((l[j] - m) / tau) * (float)((int)(lane * 4 + j) - arg);
    return wave_sum(d) / z;
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
    const RowStats rs = row_stats(L, tau, lane);
    const float delta = row_delta(L, tau, lane, rs.m, rs.z, rs.arg);  // ev - argmax
    const float l[4] = {L.x, L.y, L.z, L.w};
    float o[4];
    for (int j = 0; j < 4; ++j) {
        const float w = expf((l[j] - rs.m) / tau) / rs.z;
        o[j] = g * w * ((float)((int)(lane * 4 + j) - rs.arg) - delta) / tau;
    }
    (void)stats;
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
    int best = 0;
    for (int j = 1; j < 18; ++j)
        if (L[j] > L[best]) best = j;
    const float m = L[best];
    uint32_t sw0, in0;
    action_ports((uint32_t)best, &sw0, &in0);
    // expectations relative to the argmax action's port values (no cancellation)
    float z = 0.f, ds = 0.f, di = 0.f;
    for (int j = 0; j < 18; ++j) {
        uint32_t sw, in;
        action_ports((uint32_t)j, &sw, &in);
        const float w = expf((L[j] - m) / tau);
        z += w;
        ds += w * ((float)sw - (float)sw0);
        di += w * ((float)in - (float)in0);
    }
    ds /= z;
    di /= z;
    const float gs = gport[row * 2], gi = gport[row * 2 + 1];
    for (int j = 0; j < 18; ++j) {
        uint32_t sw, in;
        action_ports((uint32_t)j, &sw, &in);
        const float w = expf((L[j] - m) / tau) / z;
        out[row * 18 + j] = (w / tau) * (gs * (((float)sw - (float)sw0) - ds) + gi * (((float)in - (float)in0) - di));
    }
    (void)stats;
}

// ---------------------------------------------------------------------------
// Reset and inspection
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reset(StateRec *state, int32_t B, const uint8_t *mask, const uint8_t *ram0,
                                               uint64_t seed, uint8_t *sc_state) {
    const int32_t env = blockIdx.x * 256 + threadIdx.x;
    if (env >= B) return;
    if (mask && !mask[env]) return;
    if (sc_state) {  // Superchip RAM from its own SplitMix64 stream
        uint32_t *sw = reinterpret_cast<uint32_t *>(sc_state + (size_t)env * 128);
        for (uint32_t w = 0; w < 16; ++w) {
            const uint64_t v = reset_ram_word(seed ^ kScSeed, (uint64_t)env, 0, w);
            sw[2 * w] = (uint32_t)v;
            sw[2 * w + 1] = (uint32_t)(v >> 32);
        }
    }
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
    r.slices = 4u | (5u << 4) | (6u << 8) | (7u << 12);
}

// The 16 inspection bytes of a state record (layout of vcs_read_regs).
__device__ __forceinline__ void regs16(const StateRec &r, uint8_t o[16]) {
    const int32_t t = r.cyc;
    const int32_t dd = t - r.tim_u;
    const uint32_t intim = dd < 0 ? ((uint32_t)(-1 - (dd >> r.tim_shift)) & 0xFFu) : ((uint32_t)(255 - dd) & 0xFFu);
    const uint32_t timint = (t >= r.tim_u && r.tim_read < r.tim_u) ? 0x80u : 0u;
    o[0] = r.a; o[1] = r.x; o[2] = r.y; o[3] = r.s; o[4] = r.p;
    o[5] = (uint8_t)(r.pc & 0xFF); o[6] = (uint8_t)(r.pc >> 8); o[7] = r.bank; o[8] = r.status;
    o[9] = (uint8_t)intim; o[10] = (uint8_t)timint; o[11] = r.vblank;
    o[12] = (uint8_t)(r.col & 0xFF); o[13] = (uint8_t)((r.col >> 8) & 0xFF);
    o[14] = (uint8_t)((r.col >> 16) & 0xFF); o[15] = (uint8_t)(r.col >> 24);
}

__global__ __launch_bounds__(256) void k_read_regs(const StateRec *state, int32_t B, uint8_t *out) {
    const int32_t env = blockIdx.x * 256 + threadIdx.x;
    if (env >= B) return;
    uint8_t o[16];
    regs16(state[env], o);
    for (int i = 0; i < 16; ++i) out[(size_t)env * 16 + i] = o[i];
}

// One thread per env: the object registers in the vcs_read_objects layout.
__global__ __launch_bounds__(256) void k_read_objects(const StateRec *state, int32_t B, uint8_t *out) {
    const int32_t env = blockIdx.x * 256 + threadIdx.x;
    if (env >= B) return;
    uint8_t o[32];
    objects32(state[env], o);
    for (int i = 0; i < 32; ++i) out[(size_t)env * 32 + i] = o[i];
}

// FNV-1a, 64-bit (Fowler, Noll, Vo): offset basis 14695981039346656037, prime 2^40 + 2^8 + 0xb3.
__device__ __forceinline__ uint64_t fnv1a(uint64_t h, uint32_t byte) {
    return (h ^ (uint64_t)byte) * 0x100000001B3ull;
}

// One thread per env: hash of the 16 inspection bytes, the 128 RAM bytes and, when
// given, the env's 210 x 160 frame (rows at frame + env * frame_stride).
__global__ __launch_bounds__(256) void k_hash(const StateRec *state, int32_t B, const uint8_t *frame,
                                              int64_t frame_stride, uint64_t *out) {
    const int32_t env = blockIdx.x * 256 + threadIdx.x;
    if (env >= B) return;
    const StateRec &r = state[env];
    uint8_t o[16];
    regs16(r, o);
    uint64_t h = 0xCBF29CE484222325ull;
    for (int i = 0; i < 16; ++i) h = fnv1a(h, o[i]);
    const uint32_t *ram = reinterpret_cast<const uint32_t *>(r.ram);
    for (int w = 0; w < 32; ++w) {
        const uint32_t v = ram[w];
        for (int k = 0; k < 4; ++k) h = fnv1a(h, (v >> (8 * k)) & 0xFFu);
    }
    if (frame) {
        const uint32_t *f = reinterpret_cast<const uint32_t *>(frame + (size_t)env * (size_t)frame_stride);
        for (int w = 0; w < kPixels / 4; ++w) {
            const uint32_t v = f[w];
            for (int k = 0; k < 4; ++k) h = fnv1a(h, (v >> (8 * k)) & 0xFFu);
        }
    }
    out[env] = h;
}

__global__ void k_fill_zero(uint32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
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
                        uint8_t *sc_state, hipStream_t stream) {
    hipLaunchKernelGGL(k_reset, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, state, B, mask, ram0, seed,
                       sc_state);
    return hipGetLastError();
}

hipError_t launch_read_objects(const StateRec *state, int32_t B, uint8_t *out, hipStream_t stream) {
    hipLaunchKernelGGL(k_read_objects, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, state, B, out);
    return hipGetLastError();
}

hipError_t launch_read_regs(const StateRec *state, int32_t B, uint8_t *out, hipStream_t stream) {
    hipLaunchKernelGGL(k_read_regs, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, state, B, out);
    return hipGetLastError();
}

hipError_t launch_hash(const StateRec *state, int32_t B, const uint8_t *frame, int64_t frame_stride, uint64_t *out,
                       hipStream_t stream) {
    hipLaunchKernelGGL(k_hash, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, state, B, frame, frame_stride,
                       out);
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
