// Soft kernels of libvcs without the object paths: the soft forward (k_step
// with kSoft) and the surrogate backward k_soft_bwd, for envs in which no object
// shows (the others run the kernels of vcs_step_soft_obj.hip).
#include "vcs_step_kernels.hpp"

namespace vcs {

hipError_t launch_step_soft_tape(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                                 hipStream_t stream, bool objects);
hipError_t launch_step_soft_obj(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                                hipStream_t stream);

hipError_t launch_step_soft(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                            hipStream_t stream, bool objects) {
    if (P.ftape) return launch_step_soft_tape(P, blocks, lanes, tpb, lds, stream, objects);
    if (objects) return launch_step_soft_obj(P, blocks, lanes, tpb, lds, stream);
#define VCS_STEP_CASE(Gv, Tv) \
    if (lanes == Gv && tpb == Tv) return launch_step_t<Gv, Tv, true, false, false>(P, blocks, lds, stream);
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

hipError_t launch_soft_bwd_obj(const BwdParams &P, int32_t blocks, int32_t max_rom_size, hipStream_t stream);

hipError_t launch_soft_bwd(const BwdParams &P, int32_t blocks, int32_t max_rom_size, hipStream_t stream,
                           bool objects) {
    if (objects) return launch_soft_bwd_obj(P, blocks, max_rom_size, stream);
    hipLaunchKernelGGL(k_soft_bwd<false>, dim3(blocks), dim3(kBwdTPB), (size_t)max_rom_size * sizeof(uint2), stream,
                       P);
    return hipGetLastError();
}

}  // namespace vcs
