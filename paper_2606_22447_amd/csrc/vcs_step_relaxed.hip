// FULL relaxed step kernels of libvcs (vcs_step_relaxed).
#include "vcs_step_kernels.hpp"

namespace vcs {

hipError_t launch_step_relaxed(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                               hipStream_t stream) {
#define VCS_RELAX_CASE(Gv, Tv)                                                                          \
    if (lanes == Gv && tpb == Tv) {                                                                     \
        hipLaunchKernelGGL((k_step_relaxed<Gv, Tv>), dim3(blocks), dim3(Tv), lds, stream, P);           \
        return hipGetLastError();                                                                       \
    }
    VCS_RELAX_CASE(1, 64)
    VCS_RELAX_CASE(1, 256)
    VCS_RELAX_CASE(4, 64)
    VCS_RELAX_CASE(4, 256)
    VCS_RELAX_CASE(16, 64)
    VCS_RELAX_CASE(16, 256)
    VCS_RELAX_CASE(64, 64)
    VCS_RELAX_CASE(64, 256)
    VCS_RELAX_CASE(64, 1024)
#undef VCS_RELAX_CASE
    return hipErrorInvalidValue;
}

}  // namespace vcs
