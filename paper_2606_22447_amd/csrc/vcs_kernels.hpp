// Kernel launchers of libvcs (implemented in vcs_kernels.hip).
#pragma once

#include "vcs_internal.hpp"

namespace vcs {

// lds: bytes of dynamic LDS (the staged ROM image, then Superchip RAM)
// objects: the kernels with the object paths (TIA objects and collisions)
hipError_t launch_step(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, bool soft, bool plain,
                       size_t lds, hipStream_t stream, bool objects = true);
hipError_t launch_step_relaxed(const StepParams &P, int32_t blocks, int32_t lanes, int32_t tpb, size_t lds,
                               hipStream_t stream);
hipError_t launch_soft_bwd(const BwdParams &P, int32_t blocks, int32_t max_rom_size, hipStream_t stream,
                           bool objects);
hipError_t launch_decode(const float *rom_logits, int64_t rom_rows, const float *tape, int64_t tape_rows,
                         const float *act_logits, int64_t act_rows, float tau, uint8_t *rom_hard, float *rom_stats,
                         uint8_t *ram0_hard, float *tape_ev, uint8_t *act_hard, float *act_stats, hipStream_t stream);
hipError_t launch_epilogue(const float *rom_logits, const float *rom_stats, const float *gpart, int64_t rom_rows,
                           int32_t num_roms, const int32_t *rom_off, const int32_t *rom_size,
                           const int32_t *slot_begin, const int32_t *slot_end, uint32_t nslots, float tau,
                           float *grad_rom, const float *g0, int64_t tape_rows, float *grad_tape,
                           const float *act_logits, const float *act_stats, const float *gport, int64_t act_rows,
                           float *grad_act, hipStream_t stream);
hipError_t launch_reset(StateRec *state, int32_t B, const uint8_t *mask, const uint8_t *ram0, uint64_t seed,
                        uint8_t *sc_state, hipStream_t stream);
hipError_t launch_read_regs(const StateRec *state, int32_t B, uint8_t *out, hipStream_t stream);
hipError_t launch_read_objects(const StateRec *state, int32_t B, uint8_t *out, hipStream_t stream);
hipError_t launch_hash(const StateRec *state, int32_t B, const uint8_t *frame, int64_t frame_stride, uint64_t *out,
                       hipStream_t stream);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t stream);

constexpr int kBwdSlots = 16;  // envs per soft-backward workgroup (one wave each)

}  // namespace vcs
