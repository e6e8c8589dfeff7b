/*
 * libvcs -- batched Atari VCS emulation on MI355X (gfx950), hard and soft
 * (straight-through) forms, behind a plain C ABI.
 *
 * The operation is the paper's environment step: state + action -> next
 * state, RAM and frame ("A Differentiable Atari VCS", Sec. "Building Two
 * Differentiable VCS Ports" and Sec. "Evaluation Methodology"), for many
 * independent instances in lockstep.  HARD mode is the bit-exact machine
 * (Sec. "Hard and Soft Execution"); SOFT mode treats the ROM as a weight
 * tensor, the RAM as a soft tape and branches as gates joined to the hard
 * values by the straight-through estimator (Eq. peek, Eq. select, Eq. branch,
 * Eq. ste), so its forward pass equals HARD (Theorem "Exact forward
 * equivalence") and its backward pass is the surrogate gradient of the chosen
 * relaxation (the Corollary after Theorem "Temperature-limit bound").
 *
 * Conventions
 *  - Every function returns a vcs_status (0 = VCS_OK) and never throws.
 *  - Pointers named d_* are DEVICE pointers (HIP device memory on the current
 *    device), owned by the caller; the library allocates no device memory.
 *    Work is enqueued asynchronously on the given stream (NULL = the default
 *    stream); device buffers must stay valid until that work completes.
 *    Pointers without the d_ prefix are host pointers, read synchronously.
 *  - Argument errors are reported synchronously.  HIP launch errors are
 *    reported as VCS_HIP_ERROR by the call that launched; errors raised while a
 *    kernel runs surface on a later synchronising call of the caller's.
 *  - An "env" is one emulated console.  Envs are independent; several envs may
 *    share a ROM image (selected by env_rom[]).
 *  - Frame layout: uint8 (hard) or float32 (soft) [210][160] row-major palette
 *    indices; the visible window is scan lines [ystart, ystart+210) and colour
 *    clocks 68..227 of each line.  Frames are cycle-framed: frame f covers CPU
 *    cycles [f*19912, (f+1)*19912) since power-on (262 lines x 76 cycles).
 *  - An env step applies one action for `frame_skip` frames and ends at the
 *    first instruction boundary at or after the step's cycle budget.
 *  - Actions are the 18 standard ALE joystick actions (0 = NOOP ... 17 =
 *    DOWNLEFTFIRE) and, for hard steps, 18 = the console RESET switch held
 *    (SWCHB bit 0 low, joystick idle): the boot sequence's RESET frames (Table
 *    s-params: 60 NOOP + 4 RESET frames).
 */
#ifndef VCS_H
#define VCS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VCS_ABI_VERSION 4  /* 2: soft forward from a given state; 3: sampler tangents, address surrogate;
                              4: the soft forward's tape (tape_records) */

typedef enum vcs_status {
    VCS_OK = 0,
    VCS_INVALID_ARG = -1,        /* a NULL/out-of-range argument or inconsistent sizes */
    VCS_UNSUPPORTED = -2,        /* a valid request this build does not implement */
    VCS_WORKSPACE_TOO_SMALL = -3,/* the caller's buffer is smaller than the size query returned */
    VCS_HIP_ERROR = -4,          /* a HIP runtime call or kernel launch failed */
    VCS_BAD_STATE_VERSION = -5   /* reserved: state produced by another ABI version */
} vcs_status;

/* Cartridge formats (Sec. "Building Two Differentiable VCS Ports": 2K, 4K, F8,
 * F6, F4, their Superchip variants and E0).
 *  - 2K (2048 bytes, mirrored) and 4K (4096);
 *  - F8 / F6 / F4 (8 / 16 / 32 KB): 4 KB banks selected by a data access (read
 *    or write) to $1FF8-9 / $1FF6-9 / $1FF4-B; power-on bank 1 for F8, 0 for
 *    F6 and F4; a hotspot read returns the newly selected bank's byte;
 *  - F8SC / F6SC / F4SC: the same plus 128 bytes of Superchip RAM written at
 *    $1000-$107F and read at $1080-$10FF (a read of the write port returns the
 *    ROM byte); vcs_reset and in-run resets seed it with SplitMix64 on the seed
 *    XOR 0x5343534352414D00 (env, episode), as RAM;
 *  - E0 (8 KB, eight 1 KB slices): $1FE0-7 / $1FE8-F / $1FF0-7 select the
 *    slice of the window's first / second / third quarter (power-on slices 4,
 *    5, 6); the last quarter is slice 7.
 * Images larger than 16 KB (F4, F4SC) need VCS_KERNEL_PLAIN: the LDS-staged
 * kernels hold an image as 8-byte pre-decoded words in one CU's LDS.  The
 * soft path takes no Superchip format; TRANSLATED takes 2K, 4K and F8. */
typedef enum vcs_mapper {
    VCS_MAPPER_2K = 0, VCS_MAPPER_4K = 1, VCS_MAPPER_F8 = 2, VCS_MAPPER_F6 = 3, VCS_MAPPER_F4 = 4,
    VCS_MAPPER_F8SC = 5, VCS_MAPPER_F6SC = 6, VCS_MAPPER_F4SC = 7, VCS_MAPPER_E0 = 8
} vcs_mapper;

/* Kernel family used for the emulation step. */
typedef enum vcs_kernel {
    VCS_KERNEL_AUTO = 0,    /* the tuned kernel (VCS_KERNEL_GROUPED unless told otherwise) */
    VCS_KERNEL_PLAIN = 1,   /* one env per thread, RAM/ROM in global memory, per-lane dispatch */
    VCS_KERNEL_GROUPED = 2, /* LDS-staged ROM and RAM, wave-uniform grouped dispatch, lane groups */
    VCS_KERNEL_TRANSLATED = 3 /* GROUPED layout running the ROM images' code translated into
                                 straight-line HIP at run time (vcs_translate); hard steps only */
} vcs_kernel;

/* Frame output modes of vcs_step_hard. */
typedef enum vcs_frames {
    VCS_FRAMES_NONE = 0,    /* no frame written (d_frame_out may be NULL) */
    VCS_FRAMES_LAST = 1,    /* d_frame_out is [B][210][160]: last frame of the last step */
    VCS_FRAMES_ALL = 2      /* d_frame_out is [B][S][210][160]: last frame of every step */
} vcs_frames;

typedef struct vcs_config {
    int32_t abi_version;        /* must be VCS_ABI_VERSION */
    int32_t num_envs;           /* B >= 1 */
    int32_t num_roms;           /* R >= 1 */
    const int32_t *rom_size;    /* host [R]: the size of the format (2048 ... 32768 bytes) */
    const int32_t *rom_mapper;  /* host [R]: vcs_mapper matching the size */
    const int32_t *env_rom;     /* host [B]: ROM index of each env */
    int32_t frame_skip;         /* frames per env step, >= 1 */
    int32_t ystart;             /* first visible scan line, 0..52 (34 is the usual value) */
    uint64_t seed;              /* SplitMix64 seed of in-run reset RAM */
    int32_t ckpt_interval;      /* soft backward: hard-state checkpoint every K cycles (>= 64) */
    int32_t kernel;             /* vcs_kernel */
    int32_t lanes_per_env;      /* lanes cooperating on one env (1, 4, 16 or 64, and 32 for TRANSLATED;
                                   0 = auto) */
    int32_t block_threads;      /* threads per workgroup: 64, 256, or 1024 (GROUPED with 64 lanes per
                                   env only); 0 = 1024 for GROUPED with 64 lanes per env, else 256;
                                   TRANSLATED: block_threads / lanes_per_env <= 64, and the
                                   workgroup runs as many drawing threads besides, which turn
                                   the logged pixel-register writes into the returned frames */
    int32_t tape_records;       /* soft forward's tape, 16-byte records per env kept in the residual:
                                   0 = none (the backward recomputes every checkpoint segment);
                                   n > 0 = up to n records; -1 = as many as S steps can need
                                   ((S F - 1) * 9956 + S + 16).  The forward records each segment
                                   it completes before the final frame, while the records fit;
                                   the backward sweeps those from the tape instead of recomputing
                                   them (not with read_T > 0).  Memory for recompute time. */
} vcs_config;

typedef struct vcs_ctx vcs_ctx;

/* Create a host-side context (configuration, launch geometry, env->workgroup
 * grouping by ROM).  Allocates host memory only.  On error *out is NULL. */
int32_t vcs_create(const vcs_config *cfg, vcs_ctx **out);

/* Release the context (host memory only).  NULL is accepted. */
void vcs_destroy(vcs_ctx *ctx);

/* Static text for a status code. */
const char *vcs_status_string(int32_t status);

/* Sizes of caller-allocated device buffers:
 *  - state: B opaque 256-byte records, followed (when some image is a
 *    Superchip format) by B 128-byte Superchip RAM blocks (vcs_state_bytes);
 *  - roms:  the concatenated ROM images (sum of rom_size[]) as uint8;
 *  - workspace for op (VCS_OP_*) and S steps;
 *  - soft residual (saved by the forward, read by the backward) for S steps;
 *  - soft decode output (float32 statistics, layout in vcs_step_soft_fwd). */
enum { VCS_OP_HARD = 0, VCS_OP_SOFT_FWD = 1, VCS_OP_SOFT_BWD = 2 };
int32_t vcs_state_bytes(const vcs_ctx *ctx, size_t *bytes);
int32_t vcs_rom_bytes(const vcs_ctx *ctx, size_t *bytes);
int32_t vcs_workspace_bytes(const vcs_ctx *ctx, int32_t op, int32_t steps, size_t *bytes);
int32_t vcs_residual_bytes(const vcs_ctx *ctx, int32_t steps, size_t *bytes);
int32_t vcs_decode_bytes(const vcs_ctx *ctx, int32_t steps, size_t *bytes);

/* Power-on of the envs selected by d_mask (uint8 [B], nonzero = reset; NULL =
 * all): the console and environment wrapper the paper ports (Sec. "Building
 * Two Differentiable VCS Ports") start an episode from a powered-on machine;
 * the ALE boot sequence of Sec. "Evaluation Methodology" (no-op frames and
 * console resets) is not applied here: the caller's steps follow directly.
 * RAM comes from d_ram0 (uint8 [B][128], 4-byte aligned) when
 * given, otherwise from SplitMix64(seed, env, 0).  CPU: A=X=Y=0, S=$FD, P=$24,
 * TIA registers 0, RIOT timer as if written with 0 at cycle -1 with interval
 * 1024 and its flag clear, episode and step counters 0.  The PC is loaded from
 * the reset vector of the power-on bank (bank 1 for F8) by the next step call,
 * which has the ROM; until then vcs_read_regs shows PC = 0 and status bit 1
 * (power-on pending).  d_state: [B][256] bytes, 16-byte aligned. */
int32_t vcs_reset(vcs_ctx *ctx, void *d_state, const uint8_t *d_mask, const uint8_t *d_ram0, hipStream_t stream);

/* HARD env steps (Sec. "Hard and Soft Execution", hard mode), in place on
 * d_state:
 *  d_rom          uint8 [sum rom_size]: ROM images concatenated in ROM order;
 *  d_state        [B][256] opaque records, updated in place;
 *  d_actions      uint8 [B][S] action per env step (NULL = NOOP);
 *  steps          S >= 1;
 *  d_ram_out      uint8 [B][S][128] RAM after each step (NULL = not written);
 *  frames, d_frame_out  see vcs_frames;
 *  d_done         uint8 [B][S]: 1 when the step ended the env's episode
 *                 (NULL = not written);
 *  d_episode_steps uint32 [B][E] episode lengths in env steps (NULL = no
 *                 episodes): when an env has taken d_episode_steps[b][e] steps
 *                 in episode e < E it is reset in-run (power-on, RAM =
 *                 SplitMix64(seed, env, e+1)) and the next step starts the new
 *                 episode;
 *  d_work         workspace of vcs_workspace_bytes(VCS_OP_HARD): the launch
 *                 tables, a copy of the starting states (and Superchip RAM)
 *                 and one flag byte per env.
 * A call runs in two passes: every env first runs in kernels without the TIA
 * object paths (the translated code, or the interpreter), which are exact while
 * no object shows and flag the envs where one does; those envs are then rerun
 * from the copied starting states by the interpreter with the object paths
 * (collisions, object pixels).  The stream work of a call is one
 * host-to-device copy of the launch tables into d_work, one device-to-device
 * copy of the states (two with Superchip RAM), and the two kernels, so a call
 * can be captured in a HIP graph once the context has made a device call
 * (vcs_reset, or an earlier step); a context's first device call inside a
 * capture returns VCS_UNSUPPORTED. */
int32_t vcs_step_hard(vcs_ctx *ctx, const uint8_t *d_rom, void *d_state, const uint8_t *d_actions, int32_t steps,
                      uint8_t *d_ram_out, int32_t frames, uint8_t *d_frame_out, uint8_t *d_done,
                      const uint32_t *d_episode_steps, int32_t num_episodes, void *d_work, hipStream_t stream);

/* vcs_step_hard for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same arguments without d_work.  The launch tables go to a static device
 * array of the library (1 MiB on each device it runs on, held until the
 * process ends) instead of a caller workspace, and the call allocates
 * nothing: no device, host or pinned memory.
 *  - The context's launch tables must fit: VCS_WORKSPACE_TOO_SMALL when
 *    they exceed 1 MiB (about 80,000 envs).
 *  - The call is one pass of the interpreter with the object paths (no state
 *    copy: that would need a workspace), also for a translated context.
 *  - The context must have made its pinned host copy of the tables (vcs_reset
 *    does; so does an earlier vcs_step_hard): VCS_UNSUPPORTED otherwise.
 *  - All calls on one device share the array, and each call rewrites the
 *    whole of what it uses (nothing in it needs to start at zero): calls whose
 *    stream work overlaps on one device (different streams, no ordering
 *    between them) race on it and must not be issued.
 * Everything else, including results, is as for vcs_step_hard. */
int32_t vcs_step_hard_static(vcs_ctx *ctx, const uint8_t *d_rom, void *d_state, const uint8_t *d_actions,
                             int32_t steps, uint8_t *d_ram_out, int32_t frames, uint8_t *d_frame_out,
                             uint8_t *d_done, const uint32_t *d_episode_steps, int32_t num_episodes,
                             hipStream_t stream);

/* FULL relaxed hard steps: vcs_step_hard (same arguments and outputs, no
 * episodes) with the relaxation applied without the straight-through
 * correction (Table s-modes, "full"; Sec. "Forward Bit-Exactness Under Full
 * Relaxation").  While an instruction executes, every read of a ROM byte or a
 * RAM cell (opcode and the two bytes after it, operands, pointers, pulls)
 * returns the distance-softmax read of Eq. s-read over the byte and its
 * neighbours |k| <= 8 in the same array (ROM image or the 128 RAM cells), with
 * weights e^{-|k|/T} normalised over those, cast back to a byte; every branch
 * moves the pc by sigma(alpha z) times its offset (Eq. s-branch, z = +1
 * taken, -1 not) and is cast.  Sums in float32 without fused multiply-adds,
 * weights e^{-k/T} and sigma(+-alpha) computed in double and stored as float,
 * casts round to nearest (ties to even).  The machine runs on the cast values.
 *  alpha > 0, T > 0   branch sharpness and read temperature;
 *  d_relax_out        int64 [B][2] (8-byte aligned): the first instruction
 *                     (counted from the call's start, 0-based) whose cast
 *                     differed from the exact value, -1 if none (N_div); and
 *                     the number of such casts.
 * The launch geometry is the context's (its lanes per env and threads per
 * workgroup; the interpreter runs whatever the context's kernel). */
int32_t vcs_step_relaxed(vcs_ctx *ctx, const uint8_t *d_rom, void *d_state, const uint8_t *d_actions, int32_t steps,
                         uint8_t *d_ram_out, int32_t frames, uint8_t *d_frame_out, double alpha, double T,
                         int64_t *d_relax_out, void *d_work, hipStream_t stream);

/* SOFT-STE forward of S env steps (Theorem "Exact forward equivalence": its
 * values equal HARD at any tau and alpha), the paper's env step state + action
 * -> next state (Sec. "Building Two Differentiable VCS Ports") taken softly:
 *  d_state_in      [B][256] state records to start from (NULL = power-on with
 *                  the tape's RAM).  From a given state (e.g. after hard steps,
 *                  or a vcs_reset) its registers and RAM are constants of the
 *                  relaxation: the tape is not read (it may be NULL) and its
 *                  gradient is zero.  Frames keep their place on the state's
 *                  frame grid.  May equal d_state_out;
 *  d_rom_logits    float32 [sum rom_size][256]: ROM as a weight tensor; byte a
 *                  = STE(sum_k k softmax(L[a]/tau)_k, argmax_k L[a]) (Eq. select
 *                  over the byte values; lowest index on ties);
 *  d_ram_tape      float32 [B][128][256]: initial RAM as a soft tape of content
 *                  rows; cell c = STE(sum_k k P[c][k], argmax_k P[c][k]);
 *  d_action_logits float32 [B][S][18]: per-step action scores; the ports read
 *                  STE(E_softmax(l/tau)[port(a)], port(argmax l));
 *  tau > 0; alpha > 0 is the branch-gate sharpness of Eq. branch (flags carry
 *  no gradient in this relaxation, so alpha does not change the result);
 *  d_ram_out       float32 [B][S][128] integer-valued RAM after each step;
 *  d_frame_out     float32 [B][210][160] integer-valued final frame;
 *  d_frame_dpos    float32 [B][5][210][160] (NULL = not written; needs
 *                  d_frame_out): the differentiable position sampler of Sec.
 *                  "Hard and Soft Execution" -- for each object (P0, P1, M0, M1,
 *                  BL) the final frame's derivative with respect to the
 *                  object's column through a triangular (bilinear) sampler at
 *                  zero sub-pixel offset, taken from the right: per pixel the
 *                  colour with the object drawn one column further right
 *                  (every span of the frame) minus the colour drawn, 0 where
 *                  VBLANK or an HMOVE blank blacks the pixel out.  A stored
 *                  switch gives no gradient for a strobe-timed column; this is
 *                  the paper's remedy for that one index;
 *  d_decode_out    float32 statistics (NULL = not written), in order:
 *                  ROM rows [sum rom_size][3] = (expected byte, softmax max,
 *                  softmax normaliser); tape [B][128] expected byte; actions
 *                  [B][S][2] = (E[SWCHA], E[INPT4]); the tape rows are zero
 *                  when the forward starts from d_state_in;
 *  d_state_out     [B][256] final hard state (NULL = not written);
 *  d_residual      vcs_residual_bytes(S): saved for the backward;
 *  d_work          vcs_workspace_bytes(VCS_OP_SOFT_FWD, S).
 * Like vcs_step_hard, the forward runs every env first in kernels without the
 * TIA object paths and reruns those in which an object shows with them (the
 * residual records which); with d_frame_dpos every env runs with them.  With
 * tape_records != 0 the forward also writes its tape into d_residual. */
int32_t vcs_step_soft_fwd(vcs_ctx *ctx, const void *d_state_in, const float *d_rom_logits, const float *d_ram_tape,
                          const float *d_action_logits, float tau, float alpha, int32_t steps, float *d_ram_out,
                          float *d_frame_out, float *d_frame_dpos, float *d_decode_out, void *d_state_out,
                          void *d_residual, void *d_work, hipStream_t stream);

/* SOFT-STE backward: surrogate gradients of a loss given dL/d(final frame)
 * (float32 [B][210][160]) and optionally dL/d(RAM out) (float32 [B][S][128],
 * NULL = zero), for the forward whose residual is d_residual (same tau, alpha,
 * inputs and S).  The gradient is the straight-through surrogate of the
 * relaxation (Sec. "Hard and Soft Execution": stored switches, round and
 * clamp with identity backward, straight-through branches; the Corollary after
 * Theorem "Temperature-limit bound": STE as a surrogate-gradient estimator;
 * softmax Jacobians of Eq. select for the leaves).  Sweeps each checkpoint
 * segment's tape in reverse: the forward's tape where it kept one
 * (tape_records), otherwise a tape recorded by recomputing the segment from its
 * hard-state checkpoint; both give the same records, so the gradients do not
 * depend on tape_records or K.  ROM gradients of envs sharing a ROM are summed
 * in a fixed order (deterministic).
 *  read_T               0: addresses carry no gradient (the STE surrogate).  > 0:
 *                       the leaky variant's address surrogate (Eq. s-read taken in
 *                       the backward): an indexed load or ALU read of a ROM or RAM
 *                       byte (zp,X zp,Y abs,X abs,Y (zp),Y; not read-modify-write)
 *                       also passes its value's adjoint to the index register, times
 *                       the slope of the distance-softmax read at temperature
 *                       read_T: (1/T) sum_j w_j sign(j - a) (R[j] - R[a]) over
 *                       |j - a| <= 8 inside the ROM image or the 128 RAM cells,
 *                       w_j = exp(-|j - a|/T) normalised.  Must be finite, >= 0;
 *  d_ram_tape           unused (may be NULL): dL/dP[c][k] = k dL/dcell[c]
 *  d_grad_rom_logits    float32 [sum rom_size][256]  (overwritten)
 *  d_grad_ram_tape      float32 [B][128][256]         (overwritten; NULL = not
 *                       written; zero for a forward from d_state_in)
 *  d_grad_action_logits float32 [B][S][18]            (overwritten)
 *  d_work               vcs_workspace_bytes(VCS_OP_SOFT_BWD, S). */
int32_t vcs_step_soft_bwd(vcs_ctx *ctx, const void *d_residual, const float *d_rom_logits,
                          const float *d_ram_tape, const float *d_action_logits, float tau, float alpha,
                          float read_T, int32_t steps, const float *d_grad_frame, const float *d_grad_ram_out,
                          float *d_grad_rom_logits, float *d_grad_ram_tape, float *d_grad_action_logits,
                          void *d_work, hipStream_t stream);

/* Inspect: per-env registers into d_out uint8 [B][16] = A, X, Y, S, P, PCL,
 * PCH, bank, status (bit0 jammed), INTIM now, TIMINT now, VBLANK, COLUP0,
 * COLUP1, COLUPF, COLUBK. */
int32_t vcs_read_regs(vcs_ctx *ctx, const void *d_state, uint8_t *d_out, hipStream_t stream);

/* Inspect: per-env TIA object registers into d_out uint8 [B][32] (Sec. "Hard
 * and Soft Execution": object priority, sprite bits, strobe-timed columns) =
 * the columns of P0, P1, M0, M1, BL (0..159); GRP0, GRP1 and their old
 * (vertical-delay) registers; ENAM0, ENAM1, ENABL and its old register (bit 1);
 * NUSIZ0, NUSIZ1; REFP0, REFP1 (bit 3); VDELP0, VDELP1, VDELBL (bit 0);
 * RESMP0, RESMP1 (bit 1); the motion registers HMP0, HMP1, HMM0, HMM1, HMBL
 * (high nibble); the collision latches as a 16-bit word (bit 2r: register r's
 * bit 7, bit 2r+1: its bit 6), low byte first; three zero bytes.  The latches
 * are those at the state's cycle. */
int32_t vcs_read_objects(vcs_ctx *ctx, const void *d_state, uint8_t *d_out, hipStream_t stream);

/* Inspect: a 64-bit fingerprint per env for bulk comparisons (the parity
 * protocol compares them step by step against the reference emulator).
 * d_out uint64 [B] (8-byte aligned) = FNV-1a 64 (Fowler/Noll/Vo; offset basis
 * 0xcbf29ce484222325, prime 0x100000001b3) over, in order: the 16 bytes
 * vcs_read_regs gives for the env, its 128 RAM bytes ($80..$FF), and, if
 * d_frame is not NULL, the 33,600 bytes of the env's frame in row-major order
 * at d_frame + env * frame_stride (4-byte aligned; frame_stride >= 33600 and a
 * multiple of 4: 33600 for a [B][210][160] frame buffer, S * 33600 to pick one
 * step of a [B][S][210][160] one). */
int32_t vcs_hash(vcs_ctx *ctx, const void *d_state, const uint8_t *d_frame, int64_t frame_stride, uint64_t *d_out,
                 hipStream_t stream);

/* Number of soft checkpoints the forward wrote for the largest env (host
 * value; valid after the stream has completed the forward). */
int32_t vcs_residual_checkpoints(const vcs_ctx *ctx, int32_t steps, int32_t *count);

/* Soft-backward tape check: after the stream's work completes, *flag (host)
 * = 1 when a recompute segment needed more tape records than the workspace for
 * `steps` holds (that backward's gradients are then invalid), else 0.
 * Synchronises the stream. */
int32_t vcs_bwd_overflow(const vcs_ctx *ctx, const void *d_work, int32_t steps, hipStream_t stream,
                         int32_t *flag);

/* Where the soft backward keeps that flag: *offset = byte offset of an int32
 * in the VCS_OP_SOFT_BWD workspace for `steps` (nonzero after a backward
 * whose tape overflowed), so that callers can test it on the device without
 * synchronising (host only). */
int32_t vcs_bwd_overflow_offset(const vcs_ctx *ctx, int32_t steps, size_t *offset);

/* Content-based format detection (host only; the paper's ports auto-detect
 * the mapper from the image, Sec. "Building Two Differentiable VCS Ports"):
 * 2 KB -> 2K, 4 KB -> 4K; 8 KB -> E0 when the image makes more absolute
 * accesses (LDA/LDX/LDY/STA/STX/STY/BIT/CMP) to the E0 hotspots $xFE0-$xFF7
 * than to the F8 ones $xFF8-9, else F8; 16 KB -> F6, 32 KB -> F4; a banked
 * format is its Superchip variant when the first 256 bytes of every 4 KB bank
 * (the RAM window) hold one repeated value.  *mapper = a vcs_mapper;
 * VCS_INVALID_ARG for other sizes.  A heuristic: an image may defeat it. */
int32_t vcs_detect_mapper(const uint8_t *image, size_t size, int32_t *mapper);

/* Launch geometry chosen at create time (host values; NULL outputs skipped):
 * kernel family, lanes per env, threads per workgroup, step-kernel workgroups,
 * soft-backward workgroups. */
int32_t vcs_launch_info(const vcs_ctx *ctx, int32_t *kernel, int32_t *lanes_per_env, int32_t *block_threads,
                        int32_t *blocks, int32_t *bwd_blocks);

/* Introspection (host only, no GPU work): the library's decoded opcode table,
 * out[256] = op class | mode << 6 | base cycles << 10 | page penalty << 13 |
 * length << 14, with op class 0 for the 67 bytes that jam the CPU. */
int32_t vcs_decode_table(uint32_t *out);

/* Translation of the context's ROM images for VCS_KERNEL_TRANSLATED (the same
 * machine as the interpreting kernels, bit for bit; Sec. "Hard and Soft
 * Execution", hard mode).  The code each image executes is found by a short
 * run of the library's machine core on the host (8 envs x 4 frames, RAM from
 * the context's seed); its immediate / implied / zero-page / stack / relative
 * instructions are grouped into basic blocks, at most max_positions
 * instruction positions per context shared over the images by their envs, and emitted as
 * straight-line HIP with opcodes and operand bytes as compile-time constants;
 * each block is entered through one wave-wide check (cycle limit, common
 * page-0 write addresses).  Everything else (other addressing modes, code the
 * host run did not reach, waves whose envs are at different blocks) runs on
 * the interpreter, one instruction at a time.  The source is compiled for
 * gfx950 with hiprtc (cached per process by source text) and, unless flags
 * has VCS_TRANSLATE_COMPILE_ONLY, loaded as a module on the current device;
 * vcs_step_hard of this context then launches it (on that device only).
 *  roms       host uint8 [sum rom_size]: the images, concatenated in ROM order;
 *             the d_rom of later vcs_step_hard calls must hold the same bytes;
 *  max_positions  instruction positions translated for the context (0 = 256),
 *             1..65536; compile time grows with it;
 *  info       host output (NULL = none);
 *  log        host buffer for the compiler log (NULL = none), NUL-terminated
 *             within log_size bytes.
 * Errors: VCS_UNSUPPORTED if the context's kernel is not TRANSLATED (and from
 * vcs_step_hard of a TRANSLATED context before a loading vcs_translate on the
 * current device); VCS_HIP_ERROR if compilation or module loading fails (see
 * log). */
enum { VCS_TRANSLATE_COMPILE_ONLY = 1 };
typedef struct vcs_translate_info {
    int32_t positions;      /* instruction positions translated over all images */
    int32_t runs;           /* basic blocks (straight-line runs) they form */
    int32_t truncated;      /* 1 if an image executed more positions than its share of the budget */
    int32_t cached;         /* 1 if the code object came from this process's cache */
    double compile_seconds; /* hiprtc time (0 when cached) */
    size_t source_bytes, code_bytes;
} vcs_translate_info;
int32_t vcs_translate(vcs_ctx *ctx, const uint8_t *roms, int32_t max_positions, int32_t flags,
                      vcs_translate_info *info, char *log, size_t log_size);

/* The HIP source vcs_translate compiles for these images and max_positions
 * (host only): copies
 * at most buf_size - 1 bytes and a NUL into buf (NULL = none) and sets *len to
 * the full length. */
int32_t vcs_translated_source(const vcs_ctx *ctx, const uint8_t *roms, int32_t max_positions, char *buf,
                              size_t buf_size, size_t *len);

#ifdef __cplusplus
}
#endif

#endif /* VCS_H */
