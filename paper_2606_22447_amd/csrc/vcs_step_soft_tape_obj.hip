// The soft forward that keeps its tape, with the object paths (envs in which a
// TIA object shows, or every env when the forward writes the sampler's tangents).
#include "vcs_step_kernels.hpp"

namespace vcs {

hipError_t launch_step_soft_tape_obj(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                                     hipStream_t stream) {
#define VCS_STEP_CASE(Gv, Tv) \
    if (lanes == Gv && tpb == Tv) return launch_step_t<Gv, Tv, true, false, true, TapeFwdExec>(P, blocks, lds, stream);
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

}  // namespace vcs
