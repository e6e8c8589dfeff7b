// Hard step kernels of libvcs without the object paths (the first pass of a hard
// step), and the launcher of every step kernel shape.
#include "vcs_step_kernels.hpp"

namespace vcs {

hipError_t launch_step_soft(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                            hipStream_t stream, bool objects);
hipError_t launch_step_objects(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, bool plain,
                               size_t lds, hipStream_t stream);

hipError_t launch_step(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, bool soft, bool plain,
                       size_t lds, hipStream_t stream, bool objects) {
    if (soft) {
        if (plain) return hipErrorInvalidValue;
        return launch_step_soft(P, blocks, lanes, tpb, lds, stream, objects);
    }
    if (objects) return launch_step_objects(P, blocks, lanes, tpb, plain, lds, stream);
    if (plain) {
        if (lanes != 1) return hipErrorInvalidValue;
        return tpb == 64 ? launch_step_t<1, 64, false, true, false>(P, blocks, 0, stream)
                         : launch_step_t<1, 256, false, true, false>(P, blocks, 0, stream);
    }
#define VCS_STEP_CASE(Gv, Tv) \
    if (lanes == Gv && tpb == Tv) return launch_step_t<Gv, Tv, false, false, false>(P, blocks, lds, stream);
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
