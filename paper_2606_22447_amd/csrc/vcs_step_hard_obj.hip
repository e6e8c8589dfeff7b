// Hard step kernels of libvcs with the object paths: the rerun of the envs that
// showed an object (and every hard step of the no-allocation entry point),
// including the 32-lane shapes of translated contexts.
#include "vcs_step_kernels.hpp"

namespace vcs {

hipError_t launch_step_objects(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, bool plain,
                               size_t lds, hipStream_t stream) {
    if (plain) {
        if (lanes != 1) return hipErrorInvalidValue;
        return tpb == 64 ? launch_step_t<1, 64, false, true, true>(P, blocks, 0, stream)
                         : launch_step_t<1, 256, false, true, true>(P, blocks, 0, stream);
    }
#define VCS_STEP_CASE(Gv, Tv) \
    if (lanes == Gv && tpb == Tv) return launch_step_t<Gv, Tv, false, false, true>(P, blocks, lds, stream);
    VCS_STEP_CASE(1, 64)
    VCS_STEP_CASE(1, 256)
    VCS_STEP_CASE(4, 64)
    VCS_STEP_CASE(4, 256)
    VCS_STEP_CASE(16, 64)
    VCS_STEP_CASE(16, 256)
    VCS_STEP_CASE(32, 64)
    VCS_STEP_CASE(32, 256)
    VCS_STEP_CASE(64, 64)
    VCS_STEP_CASE(64, 256)
    VCS_STEP_CASE(64, 1024)
#undef VCS_STEP_CASE
    return hipErrorInvalidValue;
}

}  // namespace vcs
