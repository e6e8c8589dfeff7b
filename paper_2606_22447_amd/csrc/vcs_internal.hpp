// Internal layouts shared by the HIP kernels and the C-ABI host code of libvcs.
#pragma once

// (run-time compilation of translated ROM code supplies the HIP device
// definitions itself and has no hip_runtime.h)
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

namespace vcs {

constexpr int kCyclesPerLine = 76;
constexpr int kLinesPerFrame = 262;
constexpr int kCyclesPerFrame = kCyclesPerLine * kLinesPerFrame;  // 19912
constexpr int kClocksPerLine = 228;
constexpr int kClocksPerFrame = kClocksPerLine * kLinesPerFrame;  // 59736
constexpr int kHBlank = 68;
constexpr int kScreenW = 160;
constexpr int kScreenH = 210;
constexpr int kPixels = kScreenW * kScreenH;  // 33600
constexpr uint32_t kMagic = 0x31534356u;      // "VCS1"
// Longest straight-line run of translated code, in instructions; also the
// length of an env's pixel-write log there (a run writes at most one pixel
// register per instruction).
constexpr int kTrMaxRun = 32;
// Smallest pixel-write log of an env in translated code, in entries: room for
// one run's writes on top of the entries one row can hold.
constexpr int kTrLogCap = 2 * kTrMaxRun;
// Bytes of one entry of that log (the effect clock and the TIA state before the write).
constexpr int kTrLogEntryBytes = 16;
// Entries of an env's log in translated code with E envs per workgroup: up to
// 256, halved while the workgroup's logs exceed 64 KB (a power of two, >= kTrLogCap).
__host__ __device__ constexpr int tr_log_cap(int E) {
    int cap = 256;
    while (cap > kTrLogCap && E * cap * kTrLogEntryBytes > 65536) cap /= 2;
    return cap;
}
// Control block of an env's pixel-write log in translated code (in LDS).  The
// env's emulating lanes append entries to a ring of CAP entries and publish how
// far the entries reach; the env's drawing lanes, in a wave of their own that
// runs beside the emulating one, turn the covered rows into pixels and release
// the entries no later row needs.  Counters run from the start of the drawn
// frame.
struct TrCtl {
    uint32_t head;   // entries appended (emulation)
    uint32_t ready;  // rows whose pixels the appended entries determine (emulation)
    uint32_t tail;   // first entry a row not drawn yet may need (drawing)
    uint32_t done;   // rows drawn (drawing)
    uint32_t state;  // 0 idle, 1 a frame is being logged, 2 its last entry is in (emulation: 0->1, 1->2; drawing: 2->0)
    uint32_t fin;    // the env logs no more frames (emulation)
    uint32_t beat;   // frames the env has ended (emulation): shows the drawing lanes it is alive
    uint32_t stalls; // waits for the drawing lanes that gave up (emulation; nonzero only after a fault)
    uint8_t *frame;  // the frame being drawn
};

// Cartridge formats (the numbering of vcs_mapper in include/vcs.h).
constexpr int32_t kMapper2K = 0, kMapper4K = 1, kMapperF8 = 2, kMapperF6 = 3, kMapperF4 = 4, kMapperF8SC = 5,
                  kMapperF6SC = 6, kMapperF4SC = 7, kMapperE0 = 8, kMapperCount = 9;
__host__ __device__ constexpr uint32_t mapper_banks(int32_t m) {
    return (m == kMapperF8 || m == kMapperF8SC) ? 2u : (m == kMapperF6 || m == kMapperF6SC) ? 4u
         : (m == kMapperF4 || m == kMapperF4SC) ? 8u : 1u;
}
__host__ __device__ constexpr bool mapper_sc(int32_t m) {
    return m == kMapperF8SC || m == kMapperF6SC || m == kMapperF4SC;
}
__host__ __device__ constexpr int32_t mapper_size(int32_t m) {
    return m == kMapper2K ? 2048 : m == kMapper4K ? 4096 : m == kMapperE0 ? 8192 : 4096 * (int32_t)mapper_banks(m);
}
// Action code of the console RESET switch held (joystick idle); 0..17 are the joystick.
constexpr uint32_t kActionReset = 18;
// Seed offset of the Superchip RAM's SplitMix64 stream ("SCSCRAM\0").
constexpr uint64_t kScSeed = 0x5343534352414D00ull;

// One env's machine state in device memory (opaque to callers, 256 bytes).
// Cycle counters are relative to the start of the current frame so that they
// stay in 32 bits for arbitrarily long episodes.
struct alignas(16) StateRec {
    uint32_t magic;
    uint8_t a, x, y, s;
    uint8_t p, bank, status, tim_shift;  // status bit 0: jammed
    uint16_t pc;
    uint8_t vblank, vsync;
    int32_t cyc;          // CPU cycles since the start of frame `frame`
    uint32_t frame;       // frames since power-on
    int32_t tim_u;        // first cycle (frame-relative) at which the timer reads as underflowed
    int32_t tim_read;     // cycle (frame-relative) of the last INTIM read
    uint32_t col;         // COLUP0 | COLUP1 << 8 | COLUPF << 16 | COLUBK << 24
    uint32_t pf;          // PF0 | PF1 << 8 | PF2 << 16 | CTRLPF << 24
    uint32_t episode;     // episodes completed since the last vcs_reset
    uint32_t ep_step;     // env steps taken in the current episode
    // soft checkpoints only:
    int64_t next_ckpt;    // cycle (since the soft call's start) at which the next checkpoint is due
    int32_t pix_cc;       // frame-relative colour clock of the last instruction's write point
    uint32_t ckpt_index;  // index of this checkpoint
    uint32_t from_tape;   // (checkpoint 0) 1: the RAM came from the soft tape at power-on; 0: a given state
    uint16_t slices;      // E0: the slice of each quarter of the cartridge window, 4 bits each
    uint16_t pad16;
    // TIA objects (layout of vcs::Objs) and collision latches
    uint32_t ob_pos, ob_gfx, ob_ctl, ob_bl;
    uint32_t ob_hm;       // motion registers' high nibbles: HMP0 | HMP1 << 4 | HMM0 << 8 | HMM1 << 12 | HMBL << 16
    uint32_t cx;          // collision latches, bit k = pair k
    int32_t cx_cc;        // frame-relative colour clock up to which the latches are current
    // (soft checkpoints) the forward's tape of the segment that starts here: first
    // record and count in the env's forward tape, tape_n = -1 when not taped
    uint32_t tape_off;
    int32_t tape_n;
    uint32_t pad[5];
    uint8_t ram[128];
};
static_assert(sizeof(StateRec) == 256, "state record must be 256 bytes");

// Static per-context device data (uploaded once per workspace).
struct StaticHdr {
    int32_t num_roms, num_envs;
    int32_t main_slots_per_block, main_blocks;  // hard / soft-forward grouping
    int32_t bwd_slots_per_block, bwd_blocks;    // soft-backward grouping (one lane per env)
    int32_t max_rom_size, total_rom_bytes;
    // byte offsets (from the start of the static region) of the arrays below
    int64_t off_rom_off, off_rom_size, off_rom_mapper;  // int32 [R]
    int64_t off_main_block_rom, off_main_slot_env;      // int32 [blocks], [blocks*slots]
    int64_t off_bwd_block_rom, off_bwd_slot_env;        // int32 [blocks], [blocks*slots]
    int64_t off_env_bwd_slot;                           // int32 [B]
    int64_t off_rom_bwd_slot_begin, off_rom_bwd_slot_end;  // int32 [R]
    int64_t bytes;
};

struct StaticPtrs {
    const int32_t *rom_off, *rom_size, *rom_mapper;
    const int32_t *main_block_rom, *main_slot_env;
    const int32_t *bwd_block_rom, *bwd_slot_env;
    const int32_t *env_bwd_slot;
    const int32_t *rom_bwd_slot_begin, *rom_bwd_slot_end;
};

// Parameters of the emulation-step kernels (hard steps and the soft forward).
struct StepParams {
    StaticPtrs st;
    const uint8_t *rom;        // concatenated ROM images
    StateRec *state;           // [B] in/out (NULL for a soft forward without state output)
    uint8_t *sc_state;         // [B][128] Superchip RAM after the state records, or NULL (no Superchip image)
    int32_t rom_words;         // LDS words staged for the ROM image; Superchip RAM follows them in LDS
    const uint8_t *actions;    // [B][S] or NULL
    int32_t steps;             // S
    int32_t frame_skip;        // F
    int32_t ystart;
    int32_t frames_mode;       // 0 none, 1 last step, 2 every step
    uint8_t *ram_out;          // [B][S][128] u8 (hard) or NULL
    uint8_t *frame_out;        // u8 frames (hard) or NULL
    float *ram_out_f;          // [B][S][128] f32 (soft) or NULL
    float *frame_out_f;        // [B][210][160] f32 (soft) or NULL
    float *frame_dpos_f;       // [B][5][210][160] f32 position-sampler tangents of frame_out_f, or NULL
    uint8_t *done;             // [B][S] or NULL
    const uint32_t *ep_steps;  // [B][E] or NULL
    int32_t num_episodes;
    uint64_t seed;
    // soft forward
    const StateRec *state_in;  // [B]: start every env from this state (NULL: power-on with ram0)
    const uint8_t *ram0;       // [B][128]: decoded RAM of the power-on start
    StateRec *ckpt;            // [B][max_ckpt] or NULL; checkpoint 0 is the starting state
    int32_t *ckpt_count;       // [B]
    int32_t ckpt_interval;
    int32_t max_ckpt;
    uint4 *ftape;              // [B][ftape_cap] the forward's tape records (w0..w3 of TapeRec), or NULL
    int32_t ftape_cap;
    // hard steps in two passes: the kernel without the object paths writes obj_flag[env]
    // (1: an object showed, the env's results are void); the kernel with them then runs
    // only the flagged envs (rerun != NULL) from their starting states state_src/sc_src
    uint8_t *obj_flag;         // [B] or NULL
    const uint8_t *rerun;      // [B] or NULL
    const StateRec *state_src; // [B] starting states of a rerun, or NULL (state)
    const uint8_t *sc_src;     // [B][128] Superchip RAM at the start of a rerun, or NULL (sc_state)
    // FULL relaxed mode (vcs_step_relaxed)
    float relax_u[9];          // e^{-k/T}, k = 0..8
    float relax_g_taken, relax_g_not;
    int64_t *relax_out;        // [B][2]: first diverging instruction (-1: none), casts that differed
};

// One record of the soft backward's recompute tape (32 bytes).
struct alignas(16) TapeRec {
    uint32_t w0;  // opcode | rd_class << 8 | wr_class << 12 | kind << 16 | has_pix << 20 | index << 21 | op class << 24
    uint32_t w1;  // rd_idx | wr_idx << 16
    uint32_t w2;  // v1 | v2 << 8 | s_before << 16
    uint32_t w3;  // env step of the instruction / marker; with index != 0 (1: X, 2: Y) the address
                  // surrogate's slope (float bits) of an indexed ROM or RAM read instead
    float pix[4]; // dL/dpixel summed per owning colour register (COLUP0, COLUP1, COLUPF, COLUBK)
};

enum TapeKind : uint32_t { kRecInstr = 0, kRecStepEnd = 1, kRecPixels = 2 };
enum ValClass : uint32_t { kClsConst = 0, kClsRam = 1, kClsCol = 2, kClsRom = 3, kClsSwcha = 4, kClsInpt4 = 5, kClsRegA = 6 };

// Parameters of the soft backward kernel.
struct BwdParams {
    StaticPtrs st;
    const uint8_t *rom;          // decoded ROM bytes (concatenated)
    const uint8_t *actions;      // [B][S] decoded actions
    const StateRec *ckpt;        // [B][max_ckpt]: segment i starts from checkpoint i (0 = the start)
    const int32_t *ckpt_count;   // [B]
    int32_t max_ckpt;
    int32_t steps, frame_skip, ystart;
    int32_t ckpt_interval;
    const float *grad_frame;     // [B][210][160]
    const float *grad_ram_out;   // [B][S][128] or NULL
    TapeRec *tape;               // [max_rec][bwd slots]
    int32_t max_rec;
    float *gpart;                // [max_rom_size][bwd slots]
    float *gport;                // [B][S][2]
    float *g_ram0;               // [B][128]
    int32_t *overflow;           // set nonzero if a segment needed more than max_rec records
    float read_T;                // address surrogate's read temperature (0: addresses carry no gradient)
    const uint4 *ftape;          // [B][ftape_cap] the forward's tape (segments with tape_n >= 0), or NULL
    int32_t ftape_cap;
    const uint8_t *obj_env;      // [B]: 1 for an env whose forward ran with the object paths, or NULL (all)
};

}  // namespace vcs
