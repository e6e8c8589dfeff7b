// Soft kernels of libvcs: the soft forward (k_step with kSoft) and the
// surrogate backward k_soft_bwd.
#include "vcs_step_kernels.hpp"

namespace vcs {

hipError_t launch_step_soft(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                            hipStream_t stream) {
#define VCS_STEP_CASE(Gv, Tv) \
    if (lanes == Gv && tpb == Tv) return launch_step_t<Gv, Tv, true, false>(P, blocks, lds, stream);
    VCS_STEP_CASE(1, 64)
    VCS_STEP_CASE(1, 256)
    VCS_STEP_CASE(4, 64)
    VCS_STEP_CASE(4, 256)
    VCS_STEP_CASE(16, 64)
    VCS_STEP_CASE(16, 256)
    VCS_STEP_CASE(64, 64)
    VCS_STEP_CASE(64, 256)
    VCS_STEP_CASE(64, 1024)
#undef VCS_STEP_CASE
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Soft backward: one env per wave (all its lanes), kBwdSlots envs of one ROM
// per workgroup sharing the pre-decoded ROM words in LDS.  The
// recompute-and-reverse chain of an env is serial, so the envs are spread over
// as many waves as possible to interleave their latency.
// ---------------------------------------------------------------------------
constexpr int kBwdTPB = kBwdSlots * 64;

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
    const int32_t env = P.st.bwd_slot_env[gslot];
    LdsWordMem m{rom_lds, dec_lds, reinterpret_cast<uint8_t *>(ram_lds), (uint32_t)E, slot};
    bwd_env<DeviceWave>(P, env, gslot, nslots, mapper, (uint32_t)rom_size, m, kDecodeDev.e);
}


hipError_t launch_soft_bwd(const BwdParams &P, int32_t blocks, int32_t max_rom_size, hipStream_t stream) {
    hipLaunchKernelGGL(k_soft_bwd, dim3(blocks), dim3(kBwdTPB), (size_t)max_rom_size * sizeof(uint2), stream, P);
    return hipGetLastError();
}

}  // namespace vcs
