// The soft forward that keeps its tape for the backward (k_step with the
// TapeFwdExec executor): every segment the forward completes before the final
// frame is swept by the backward from this tape instead of being recomputed.
// These kernels run without the object paths (vcs_step_soft_tape_obj.hip has
// them with).
#include "vcs_step_kernels.hpp"

namespace vcs {

hipError_t launch_step_soft_tape_obj(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                                     hipStream_t stream);

hipError_t launch_step_soft_tape(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                                 hipStream_t stream, bool objects) {
    if (objects) return launch_step_soft_tape_obj(P, blocks, lanes, tpb, lds, stream);
#define VCS_STEP_CASE(Gv, Tv) \
    if (lanes == Gv && tpb == Tv) return launch_step_t<Gv, Tv, true, false, false, TapeFwdExec>(P, blocks, lds, stream);
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
