// Step kernels of libvcs (device templates; instantiated by vcs_step_hard*.hip,
// vcs_step_soft*.hip and vcs_step_relaxed.hip):
//  k_step         hard env steps and the soft forward (paper Sec. "Hard and Soft
//                 Execution"; Theorem "Exact forward equivalence": the soft forward
//                 runs the hard machine on the decoded leaves).
//                 PLAIN   = one env per thread, RAM/ROM in global memory, per-lane
//                           opcode switch (the baseline kernel).
//                 GROUPED = ROM image and RAM staged in LDS, opcode dispatch made
//                           wave-uniform by a waterfall over the distinct opcodes
//                           of the wave (scalar decode), G lanes per env sharing
//                           the pixel writeback.
//  k_step_relaxed FULL relaxed hard steps.
//  k_soft_bwd     the surrogate backward of the soft step.
#pragma once

#include "vcs_device.hpp"
#include "vcs_kernels.hpp"

namespace vcs {

// ---------------------------------------------------------------------------
// Step kernel (hard steps, soft forward): one workgroup per ROM group, G lanes
// per env.
// ---------------------------------------------------------------------------
// kObj: with the object paths (collisions, object pixels); the hard steps run
// first without them (kObj false) and then with them for the envs that showed an
// object (P.rerun), from their starting states.  X: the executor (TapeFwdExec
// for a soft forward that keeps its tape).
template <int G, int TPB, bool kSoft, bool kPlain, bool kObj = true, class X = InterpExec>
__global__ __launch_bounds__(TPB) void k_step(StepParams P) {
    constexpr int E = TPB / G;
    extern __shared__ __align__(16) uint2 rom_lds[];  // pre-decoded ROM words, sized to the largest image
    __shared__ __align__(16) uint32_t ram_lds[kPlain ? 4 : 32 * E];
    __shared__ uint32_t dec_lds[kPlain ? 1 : 256];
    if constexpr (kPlain) {
        const uint32_t tid = threadIdx.x, slot = tid / G, sub = tid % G;
        const int32_t blk = blockIdx.x;
        const int32_t rom_idx = P.st.main_block_rom[blk];
        const int32_t env = P.st.main_slot_env[blk * E + slot];
        if (env >= 0 && P.rerun && P.rerun[env] && P.state_src) {
            // this kernel keeps the env's RAM in its state record: restore the record
            // (and the Superchip RAM) the rerun starts from
            const uint4 *s4 = reinterpret_cast<const uint4 *>(P.state_src + env);
            uint4 *d4 = reinterpret_cast<uint4 *>(P.state + env);
            for (int i = 0; i < (int)(sizeof(StateRec) / 16); ++i) d4[i] = s4[i];
            if (P.sc_state && P.sc_src)
                for (int i = 0; i < 8; ++i)
                    reinterpret_cast<uint4 *>(P.sc_state + (size_t)env * 128)[i] =
                        reinterpret_cast<const uint4 *>(P.sc_src + (size_t)env * 128)[i];
        }
        GlobalMem m{P.rom + P.st.rom_off[rom_idx], env >= 0 ? P.state[env].ram : nullptr,
                    (env >= 0 && P.sc_state) ? P.sc_state + (size_t)env * 128 : nullptr};
        step_env<DeviceWave, G, kSoft, kPlain, InterpExec, kObj>(P, env, sub, P.st.rom_mapper[rom_idx], m,
                                                                  kDecodeDev.e);
    } else {
        step_group<G, TPB, kSoft, X, kObj>(P, rom_lds, ram_lds, dec_lds,
                                           [](int32_t) { return typename X::State{}; });
    }
}

// FULL relaxed hard steps (vcs_step_relaxed): the grouped layout with every ROM
// and RAM read and every branch relaxed and cast (Table s-modes).
template <int G, int TPB>
__global__ __launch_bounds__(TPB) void k_step_relaxed(StepParams P) {
    constexpr int E = TPB / G;
    extern __shared__ __align__(16) uint2 rom_lds[];
    __shared__ __align__(16) uint32_t ram_lds[32 * E];
    __shared__ uint32_t dec_lds[256];
    step_group_relaxed<G, TPB>(P, rom_lds, ram_lds, dec_lds);
}

// ---------------------------------------------------------------------------
// Soft backward: one env per wave (all its lanes), kBwdSlots envs of one ROM
// per workgroup sharing the pre-decoded ROM words in LDS.  The
// recompute-and-reverse chain of an env is serial, so the envs are spread over
// as many waves as possible to interleave their latency.
// ---------------------------------------------------------------------------
constexpr int kBwdTPB = kBwdSlots * 64;

// kObj: the envs whose forward ran with the object paths (P.obj_env), recomputed
// with them; otherwise the others, without them.
template <bool kObj>
__global__ __launch_bounds__(kBwdTPB) void k_soft_bwd(BwdParams P) {
    constexpr int E = kBwdSlots;
    extern __shared__ __align__(16) uint2 rom_lds[];  // pre-decoded ROM words, sized to the largest image
    __shared__ uint32_t dec_lds[256];
    __shared__ __align__(16) uint32_t ram_lds[32 * E];
    const uint32_t tid = threadIdx.x;
    const uint32_t slot = __builtin_amdgcn_readfirstlane(tid / 64);  // the wave's env slot (a scalar)
    const int32_t blk = blockIdx.x;
    const uint32_t nslots = (uint32_t)gridDim.x * E;
    const uint32_t gslot = (uint32_t)blk * E + slot;
    const int32_t rom_idx = P.st.bwd_block_rom[blk];
    const int32_t rom_base = P.st.rom_off[rom_idx], rom_size = P.st.rom_size[rom_idx];
    const int32_t mapper = P.st.rom_mapper[rom_idx];
    for (int32_t i = (int32_t)tid; i < rom_size; i += kBwdTPB)
        rom_lds[i] = rom_word_at(P.rom + rom_base, i, mapper, kDecodeDev.e);
    for (int32_t i = (int32_t)tid; i < 256; i += kBwdTPB) dec_lds[i] = kDecodeDev.e[i];
    __syncthreads();
    const int32_t env0 = P.st.bwd_slot_env[gslot];
    const bool mine = env0 >= 0 && (P.obj_env ? P.obj_env[env0] != 0 : true) == kObj;
    const int32_t env = mine ? env0 : -1;  // another kernel takes the slot's env
    LdsWordMem m{rom_lds, dec_lds, reinterpret_cast<uint8_t *>(ram_lds), (uint32_t)E, slot};
    bwd_env<DeviceWave, kObj>(P, env, gslot, nslots, mapper, (uint32_t)rom_size, m, kDecodeDev.e);
}


template <int G, int TPB, bool kSoft, bool kPlain, bool kObj = true, class X = InterpExec>
hipError_t launch_step_t(const StepParams &P, int32_t blocks, size_t lds, hipStream_t stream) {
    hipLaunchKernelGGL((k_step<G, TPB, kSoft, kPlain, kObj, X>), dim3(blocks), dim3(TPB), kPlain ? 0 : lds, stream,
                       P);
    return hipGetLastError();
}

}  // namespace vcs
