// Soft kernels of libvcs with the object paths: the soft forward and the
// surrogate backward of envs in which a TIA object shows (or every env, when
// the forward writes the position sampler's tangents).
#include "vcs_step_kernels.hpp"

namespace vcs {

hipError_t launch_step_soft_obj(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                                hipStream_t stream) {
#define VCS_STEP_CASE(Gv, Tv) \
    if (lanes == Gv && tpb == Tv) return launch_step_t<Gv, Tv, true, false, true>(P, blocks, lds, stream);
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

hipError_t launch_soft_bwd_obj(const BwdParams &P, int32_t blocks, int32_t max_rom_size, hipStream_t stream) {
    hipLaunchKernelGGL(k_soft_bwd<true>, dim3(blocks), dim3(kBwdTPB), (size_t)max_rom_size * sizeof(uint2), stream,
                       P);
    return hipGetLastError();
}

}  // namespace vcs
