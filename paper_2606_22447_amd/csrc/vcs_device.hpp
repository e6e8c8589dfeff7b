// Device side shared by the precompiled kernels of libvcs and the kernels it
// generates at run time for translated ROM images: the wave policy of the
// per-env bodies, the decode table in constant memory and the body of the
// grouped step kernel.
#pragma once

#include "vcs_paths.hpp"

namespace vcs {

static __constant__ DecodeTable kDecodeDev = make_decode_table();

// ---------------------------------------------------------------------------
// Wave policy of the device bodies
// ---------------------------------------------------------------------------
typedef const __attribute__((address_space(4))) uint32_t ConstU32;

struct DeviceWave {
    static constexpr uint32_t kWidth = 64;  // lanes of a wave
    __device__ static __forceinline__ uint32_t lane() { return __lane_id(); }
    // value of v in lane j (j the same in every lane: a scalar)
    __device__ static __forceinline__ uint32_t readlane(uint32_t v, uint32_t j) {
        return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)j);
    }
    __device__ static __forceinline__ float readlane(float v, uint32_t j) {
        return __uint_as_float(readlane(__float_as_uint(v), j));
    }
    // v with lane j's element replaced by x (x and j the same in every lane)
    __device__ static __forceinline__ float writelane(float v, float x, uint32_t j) {
        return lane() == j ? x : v;
    }
    // sum of v over the wave's lanes (every lane gets it)
    __device__ static __forceinline__ float sum(float v) {
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        return v;
    }
    // least v over the active lanes (every lane gets it): start from the first
    // lane's value and move to the first lane below it until none is, with
    // scalar ballots and lane reads (no LDS-pipe shuffles, whose dependent chain
    // costs more than the step it schedules); lanes a few cycles apart take one
    // or two rounds
    __device__ static __forceinline__ int32_t min_i32(int32_t v) {
        int32_t m = __builtin_amdgcn_readfirstlane(v);
        for (;;) {
            const uint64_t lower = __ballot(v < m);
            if (lower == 0u) break;
            m = __builtin_amdgcn_readlane(v, (int)__builtin_ctzll(lower));
        }
        return m;
    }
    __device__ static __forceinline__ bool any(bool v) { return __ballot(v) != 0; }
    __device__ static __forceinline__ bool all(bool v) { return __ballot(v) == __ballot(true); }
    // *p += t without waiting for the result (a no-return atomic add).  Only one lane
    // adds to a given p, so the additions happen in program order.
    __device__ static __forceinline__ void accumulate(float *p, float t) {
        (void)__hip_atomic_fetch_add(p, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static __forceinline__ uint32_t first(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
    // order this wave's LDS and memory accesses before the ones after it, for the
    // other waves of the workgroup
    __device__ static __forceinline__ void fence() { __threadfence_block(); }
    // yield the SIMD for a short while (polling another wave of the workgroup)
    __device__ static __forceinline__ void sleep() { __builtin_amdgcn_s_sleep(1); }
    // makes v opaque to the optimiser (no instruction): code that uses it cannot be
    // hoisted out of the loop that contains this call
    __device__ static __forceinline__ void opaque(uint32_t &v) { asm volatile("" : "+v"(v)); }
    // the same for a wave-uniform value (kept in a scalar register)
    __device__ static __forceinline__ void opaque_uniform(uint32_t &v) { asm volatile("" : "+s"(v)); }
    // entry u (wave-uniform) of a read-only table in constant memory: a scalar
    // load, so that what is derived from it stays in scalar registers and the
    // branches on it are scalar branches
    // (u goes through an empty asm so that the compiler cannot substitute an
    // equal per-lane value for it and turn the load into a vector load).
    __device__ static __forceinline__ uint32_t table(const uint32_t *t, uint32_t u) {
        asm volatile("" : "+s"(u));
        return __builtin_amdgcn_readfirstlane(((ConstU32 *)t)[u]);
    }
};

// Staging of the grouped step kernel by the workgroup's NT threads: the ROM image
// of the workgroup's ROM group as pre-decoded words and the decode table in LDS.
template <int NT>
__device__ __forceinline__ void stage_group(const StepParams &P, uint2 *rom_lds, uint32_t *dec_lds) {
    const uint32_t tid = threadIdx.x;
    const int32_t rom_idx = P.st.main_block_rom[blockIdx.x];
    const int32_t rom_base = P.st.rom_off[rom_idx], rom_size = P.st.rom_size[rom_idx];
    const int32_t mapper = P.st.rom_mapper[rom_idx];
    for (int32_t i = (int32_t)tid; i < rom_size; i += NT)
        rom_lds[i] = rom_word_at(P.rom + rom_base, i, mapper, kDecodeDev.e);
    for (int32_t i = (int32_t)tid; i < 256; i += NT) dec_lds[i] = kDecodeDev.e[i];
    __syncthreads();
}

// The envs of a staged grouped step kernel: E = TPB / G envs, G lanes per env,
// threads [0, TPB) of the workgroup; the envs' RAM in LDS.  state_of(rom) gives
// the executor state of the workgroup's ROM.
template <int G, int TPB, bool kSoft, class X, bool kObj = true, class StateOf>
__device__ __forceinline__ void run_group(const StepParams &P, uint2 *rom_lds, uint32_t *ram_lds, uint32_t *dec_lds,
                                          StateOf state_of) {
    constexpr int E = TPB / G;
    const uint32_t tid = threadIdx.x, slot = tid / G, sub = tid % G;
    const int32_t blk = blockIdx.x;
    const int32_t rom_idx = P.st.main_block_rom[blk];
    const int32_t env = P.st.main_slot_env[blk * E + slot];
    const int32_t mapper = P.st.rom_mapper[rom_idx];
    LdsWordMem m{rom_lds, dec_lds, reinterpret_cast<uint8_t *>(ram_lds), (uint32_t)E, slot};
    // Superchip RAM: [32 words][E] in LDS after the staged image
    if (mapper_sc(mapper)) m.sc = reinterpret_cast<uint8_t *>(rom_lds + P.rom_words);
    step_env<DeviceWave, G, kSoft, false, X, kObj>(P, env, sub, mapper, m, kDecodeDev.e, state_of(rom_idx));
}

// Body of the grouped step kernel: one workgroup per ROM group of E = TPB / G
// envs, G lanes per env; the ROM image (pre-decoded words), the decode table and
// the envs' RAM staged in LDS.
template <int G, int TPB, bool kSoft, class X, bool kObj = true, class StateOf>
__device__ __forceinline__ void step_group(const StepParams &P, uint2 *rom_lds, uint32_t *ram_lds, uint32_t *dec_lds,
                                           StateOf state_of) {
    stage_group<TPB>(P, rom_lds, dec_lds);
    run_group<G, TPB, kSoft, X, kObj>(P, rom_lds, ram_lds, dec_lds, state_of);
}

// Body of the FULL relaxed step kernel: the grouped kernel's layout with the
// relaxing memory policy (hard steps, interpreter only).
template <int G, int TPB>
__device__ __forceinline__ void step_group_relaxed(const StepParams &P, uint2 *rom_lds, uint32_t *ram_lds,
                                                   uint32_t *dec_lds) {
    constexpr int E = TPB / G;
    const uint32_t tid = threadIdx.x, slot = tid / G, sub = tid % G;
    const int32_t blk = blockIdx.x;
    const int32_t rom_idx = P.st.main_block_rom[blk];
    const int32_t env = P.st.main_slot_env[blk * E + slot];
    const int32_t rom_base = P.st.rom_off[rom_idx], rom_size = P.st.rom_size[rom_idx];
    const int32_t mapper = P.st.rom_mapper[rom_idx];
    for (int32_t i = (int32_t)tid; i < rom_size; i += TPB)
        rom_lds[i] = rom_word_at(P.rom + rom_base, i, mapper, kDecodeDev.e);
    for (int32_t i = (int32_t)tid; i < 256; i += TPB) dec_lds[i] = kDecodeDev.e[i];
    __syncthreads();
    RelaxMem<LdsWordMem> m;
    static_cast<LdsWordMem &>(m) = LdsWordMem{rom_lds, dec_lds, reinterpret_cast<uint8_t *>(ram_lds), (uint32_t)E,
                                              slot};
    if (mapper_sc(mapper)) m.sc = reinterpret_cast<uint8_t *>(rom_lds + P.rom_words);
    for (int k = 0; k < 9; ++k) m.rc.u[k] = P.relax_u[k];
    m.rc.g_taken = P.relax_g_taken;
    m.rc.g_not = P.relax_g_not;
    m.rom_n = (uint32_t)rom_size;
    m.active = false;
    m.ninstr = 0;
    m.ndiv = -1;
    m.fails = 0;
    step_env<DeviceWave, G, false, false, InterpExec>(P, env, sub, mapper, m, kDecodeDev.e);
}

}  // namespace vcs
