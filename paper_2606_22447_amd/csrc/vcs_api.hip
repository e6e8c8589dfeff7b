// C-ABI of libvcs (declared in include/vcs.h): argument validation, launch
// geometry and the layout of caller-owned device buffers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/vcs.h"
#include "vcs_core.hpp"
#include "vcs_jit.hpp"
#include "vcs_kernels.hpp"

using namespace vcs;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kLdsBytes = 160 * 1024;  // LDS of one CU on gfx950
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

struct vcs_ctx {
    int32_t B = 0, R = 0, F = 1, ystart = 34, K = 1024, kernel = VCS_KERNEL_GROUPED, G = 1, tpb = 256;
    int32_t tape_records = 0;    // soft forward's tape per env (0: none, -1: the bound for S steps)
    uint64_t seed = 0;
    std::vector<int32_t> rom_size, rom_mapper, env_rom, rom_off;
    int32_t max_rom = 0, total_rom = 0;
    bool any_sc = false;         // some image is a Superchip format: its RAM follows the state records
    int32_t main_E = 0, main_blocks = 0, bwd_blocks = 0;
    std::vector<int32_t> main_block_rom, main_slot_env;
    std::vector<int32_t> bwd_block_rom, bwd_slot_env, env_bwd_slot, rom_bwd_begin, rom_bwd_end;
    StaticHdr hdr{};
    std::vector<uint8_t> image;  // host image of the static device region
    uint8_t *pinned = nullptr;   // pinned copy, made on the first upload
    size_t blob_bytes = 0;
    // translated kernel (VCS_KERNEL_TRANSLATED), loaded on one device
    hipModule_t tr_module = nullptr;
    hipFunction_t tr_fn = nullptr;
    int tr_device = -1;
    ~vcs_ctx() {
        if (pinned) (void)hipHostFree(pinned);
        if (tr_module) (void)hipModuleUnload(tr_module);
    }
};

namespace {

// Layout of the soft residual for S steps.
struct ResidualLayout {
    size_t rom_hard, ram0_hard, act_hard, stats, rom_stats, tape_ev, act_stats, ckpt_count, obj_env, ckpt, ftape,
        bytes;
    size_t stats_bytes;
    int32_t max_ckpt;
    int64_t ftape_cap;  // forward-tape records per env (0: no tape)
};
// Records the forward can tape for S steps: every instruction takes at least 2
// cycles, and the final frame is never taped, so (S F - 1) frames of at most
// 9956 instruction records each, plus one step-end record per step.
int64_t ftape_bound(const vcs_ctx *c, int32_t S) {
    return ((int64_t)S * c->F - 1) * (kCyclesPerFrame / 2) + S + 16;
}
ResidualLayout residual_layout(const vcs_ctx *c, int32_t S) {
    ResidualLayout L{};
    size_t o = kAlign;  // header
    L.rom_hard = o;
    o = align_up(o + (size_t)c->total_rom);
    L.ram0_hard = o;
    o = align_up(o + (size_t)c->B * 128);
    L.act_hard = o;
    o = align_up(o + (size_t)c->B * S);
    L.stats = L.rom_stats = o;
    L.tape_ev = L.rom_stats + (size_t)c->total_rom * 3 * sizeof(float);
    L.act_stats = L.tape_ev + (size_t)c->B * 128 * sizeof(float);
    L.stats_bytes = (size_t)c->total_rom * 3 * sizeof(float) + (size_t)c->B * 128 * sizeof(float) +
                    (size_t)c->B * S * 2 * sizeof(float);
    o = align_up(L.rom_stats + L.stats_bytes);
    L.ckpt_count = o;
    o = align_up(o + (size_t)c->B * sizeof(int32_t));
    L.obj_env = o;  // 1 for an env whose forward ran with the object paths
    o = align_up(o + (size_t)c->B);
    // the starting state, one per K cycles, and slack for a start inside a frame
    L.max_ckpt = (int32_t)(((int64_t)S * c->F * kCyclesPerFrame + 256) / c->K + 3);
    L.ckpt = o;
    o = align_up(o + (size_t)c->B * L.max_ckpt * sizeof(StateRec));
    L.ftape_cap = c->tape_records < 0 ? ftape_bound(c, S) : c->tape_records;
    L.ftape = o;
    o = align_up(o + (size_t)c->B * (size_t)L.ftape_cap * 16u);
    L.bytes = o;
    return L;
}
// The forward tape's size is representable (int32 records per env, bytes in 62 bits).
bool ftape_ok(const vcs_ctx *c, const ResidualLayout &L) {
    return L.ftape_cap <= INT32_MAX && (L.ftape_cap == 0 || (uint64_t)c->B <= (1ull << 58) / (uint64_t)L.ftape_cap);
}

// Layout of the soft-backward workspace (after the static region).
// Workspace of a hard step: the launch tables, then for the two passes the
// starting states (and Superchip RAM) and the per-env object flags.
struct HardLayout {
    size_t states, sc, flags, bytes;
};
HardLayout hard_layout(const vcs_ctx *c) {
    HardLayout L{};
    size_t o = align_up(c->blob_bytes);
    L.states = o;
    o = align_up(o + (size_t)c->B * sizeof(StateRec));
    L.sc = o;
    if (c->any_sc) o = align_up(o + (size_t)c->B * 128);
    L.flags = o;
    o = align_up(o + (size_t)c->B);
    L.bytes = o;
    return L;
}

struct BwdLayout {
    size_t tape, gpart, gport, g0, overflow, bytes;
    int32_t max_rec;
    uint32_t nslots;
};
BwdLayout bwd_layout(const vcs_ctx *c, int32_t S) {
    BwdLayout L{};
    L.nslots = (uint32_t)c->bwd_blocks * kBwdSlots;
    L.max_rec = c->K / 2 + 64 + c->K / kCyclesPerFrame + 4;
    size_t o = align_up(c->blob_bytes);
    L.tape = o;
    o = align_up(o + (size_t)L.max_rec * L.nslots * sizeof(TapeRec));
    L.gpart = o;
    o = align_up(o + (size_t)c->max_rom * L.nslots * sizeof(float));
    L.gport = o;
    o = align_up(o + (size_t)c->B * S * 2 * sizeof(float));
    L.g0 = o;
    o = align_up(o + (size_t)c->B * 128 * sizeof(float));
    L.overflow = o;
    o = align_up(o + sizeof(int32_t));
    L.bytes = o;
    return L;
}

StaticPtrs static_ptrs(const vcs_ctx *c, const void *d_work) {
    const uint8_t *b = (const uint8_t *)d_work;
    const StaticHdr &h = c->hdr;
    StaticPtrs p;
    p.rom_off = (const int32_t *)(b + h.off_rom_off);
    p.rom_size = (const int32_t *)(b + h.off_rom_size);
    p.rom_mapper = (const int32_t *)(b + h.off_rom_mapper);
    p.main_block_rom = (const int32_t *)(b + h.off_main_block_rom);
    p.main_slot_env = (const int32_t *)(b + h.off_main_slot_env);
    p.bwd_block_rom = (const int32_t *)(b + h.off_bwd_block_rom);
    p.bwd_slot_env = (const int32_t *)(b + h.off_bwd_slot_env);
    p.env_bwd_slot = (const int32_t *)(b + h.off_env_bwd_slot);
    p.rom_bwd_slot_begin = (const int32_t *)(b + h.off_rom_bwd_slot_begin);
    p.rom_bwd_slot_end = (const int32_t *)(b + h.off_rom_bwd_slot_end);
    return p;
}

// Pinned host copy of the static region, made on the context's first device call.
int32_t ensure_pinned(vcs_ctx *c) {
    if (c->pinned) return VCS_OK;
    if (hipHostMalloc((void **)&c->pinned, c->blob_bytes, hipHostMallocDefault) != hipSuccess) {
        c->pinned = nullptr;
        return VCS_HIP_ERROR;
    }
    std::memcpy(c->pinned, c->image.data(), c->blob_bytes);
    return VCS_OK;
}

// Copy the static region (ROM table, env grouping) into the head of the
// caller's workspace, ordered on the stream before the kernels that read it.
// Inside a stream capture the pinned copy must already exist (allocating host
// memory would invalidate the capture).
int32_t upload_static(vcs_ctx *c, void *d_work, hipStream_t stream) {
    if (!c->pinned) {
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
            return VCS_UNSUPPORTED;
        const int32_t rc = ensure_pinned(c);
        if (rc != VCS_OK) return rc;
    }
    if (hipMemcpyAsync(d_work, c->pinned, c->blob_bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
        return VCS_HIP_ERROR;
    return VCS_OK;
}

int32_t hip_status(hipError_t e) { return e == hipSuccess ? VCS_OK : VCS_HIP_ERROR; }

// Whether the translated kernel fits one CU's LDS: the largest image's words, the
// block tables (4096 16-bit entries per bank), the envs' RAM, the decode table
// and a pixel-write log of at least kTrLogCap entries per env.
bool tr_lds_fits(const vcs_ctx *c) {
    const size_t E = (size_t)(c->tpb / c->G);
    bool f8 = false;
    for (int32_t mp : c->rom_mapper) f8 = f8 || mp == kMapperF8;
    const size_t need = (size_t)c->max_rom * 8 + (f8 ? 2 : 1) * 4096 * 2 + E * 128 + 1024 +
                        E * ((size_t)tr_log_cap((int)E) + 1) * (size_t)kTrLogEntryBytes + E * sizeof(TrCtl);
    return need <= kLdsBytes;
}

// Whether the LDS-staged step kernels fit the context's images and launch shape.
bool lds_fits(const vcs_ctx *c) {
    const size_t E = (size_t)(c->tpb / c->G);
    return (size_t)c->max_rom * 8 + E * 128 * (c->any_sc ? 2 : 1) + 1024 <= kLdsBytes;
}

// The Superchip RAM of a context with a Superchip image: [B][128] after the state records.
uint8_t *sc_state(const vcs_ctx *c, const void *d_state) {
    return c->any_sc ? (uint8_t *)d_state + (size_t)c->B * sizeof(StateRec) : nullptr;
}

// Dynamic LDS of the grouped step kernels: the image's pre-decoded words, then
// (with a Superchip image) the workgroup's Superchip RAM.
size_t step_lds(const vcs_ctx *c) {
    return (size_t)c->max_rom * sizeof(uint2) + (c->any_sc ? (size_t)(c->tpb / c->G) * 128 : 0);
}

// Launch tables of vcs_step_hard_static: a fixed device array, so that the
// entry point needs no caller workspace and allocates nothing.  Every device
// the library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is not a device address in host code).
constexpr size_t kScratchBytes = size_t(1) << 20;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int32_t scratch_on_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return VCS_HIP_ERROR;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VCS_HIP_ERROR;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return VCS_OK;
}

// Envs of every ROM packed into blocks of `per` slots that never mix ROMs.
void group_by_rom(const vcs_ctx *c, int32_t per, std::vector<int32_t> &block_rom, std::vector<int32_t> &slot_env) {
    block_rom.clear();
    slot_env.clear();
    for (int32_t r = 0; r < c->R; ++r) {
        std::vector<int32_t> envs;
        for (int32_t b = 0; b < c->B; ++b)
            if (c->env_rom[b] == r) envs.push_back(b);
        for (size_t i = 0; i < envs.size(); i += (size_t)per) {
            block_rom.push_back(r);
            for (int32_t j = 0; j < per; ++j)
                slot_env.push_back(i + (size_t)j < envs.size() ? envs[i + (size_t)j] : -1);
        }
    }
}

}  // namespace

extern "C" {

const char *vcs_status_string(int32_t status) {
    switch (status) {
        case VCS_OK: return "ok";
        case VCS_INVALID_ARG: return "invalid argument";
        case VCS_UNSUPPORTED: return "unsupported configuration";
        case VCS_WORKSPACE_TOO_SMALL: return "workspace too small";
        case VCS_HIP_ERROR: return "HIP runtime error";
        case VCS_BAD_STATE_VERSION: return "state record of another ABI version";
        default: return "unknown status";
    }
}

int32_t vcs_create(const vcs_config *cfg, vcs_ctx **out) {
    if (!out) return VCS_INVALID_ARG;
    *out = nullptr;
    if (!cfg || cfg->abi_version != VCS_ABI_VERSION) return VCS_INVALID_ARG;
    if (cfg->num_envs < 1 || cfg->num_roms < 1 || !cfg->rom_size || !cfg->rom_mapper || !cfg->env_rom)
        return VCS_INVALID_ARG;
    if (cfg->frame_skip < 1 || cfg->frame_skip > 1000) return VCS_INVALID_ARG;
    if (cfg->ystart < 0 || cfg->ystart + kScreenH > kLinesPerFrame) return VCS_INVALID_ARG;
    if (cfg->ckpt_interval != 0 && (cfg->ckpt_interval < 64 || cfg->ckpt_interval > (1 << 24))) return VCS_INVALID_ARG;
    if (cfg->tape_records < -1) return VCS_INVALID_ARG;
    vcs_ctx *c = new (std::nothrow) vcs_ctx();
    if (!c) return VCS_INVALID_ARG;
    c->B = cfg->num_envs;
    c->R = cfg->num_roms;
    c->F = cfg->frame_skip;
    c->ystart = cfg->ystart;
    c->seed = cfg->seed;
    c->K = cfg->ckpt_interval ? cfg->ckpt_interval : 1024;
    c->tape_records = cfg->tape_records;
    int64_t total = 0;
    for (int32_t r = 0; r < c->R; ++r) {
        const int32_t sz = cfg->rom_size[r], mp = cfg->rom_mapper[r];
        if (mp < 0 || mp >= kMapperCount || sz != mapper_size(mp)) {
            delete c;
            return VCS_INVALID_ARG;
        }
        c->any_sc = c->any_sc || mapper_sc(mp);
        c->rom_size.push_back(sz);
        c->rom_mapper.push_back(mp);
        c->rom_off.push_back((int32_t)total);
        total += sz;
        c->max_rom = std::max(c->max_rom, sz);
    }
    if (total > (1 << 30)) {
        delete c;
        return VCS_INVALID_ARG;
    }
    c->total_rom = (int32_t)total;
    for (int32_t b = 0; b < c->B; ++b) {
        if (cfg->env_rom[b] < 0 || cfg->env_rom[b] >= c->R) {
            delete c;
            return VCS_INVALID_ARG;
        }
        c->env_rom.push_back(cfg->env_rom[b]);
    }
    // kernel family and lane grouping
    c->kernel = cfg->kernel == VCS_KERNEL_AUTO ? VCS_KERNEL_GROUPED : cfg->kernel;
    if (c->kernel != VCS_KERNEL_PLAIN && c->kernel != VCS_KERNEL_GROUPED && c->kernel != VCS_KERNEL_TRANSLATED) {
        delete c;
        return VCS_INVALID_ARG;
    }
    c->tpb = cfg->block_threads;
    if (c->tpb != 0 && c->tpb != 64 && c->tpb != 256 && c->tpb != 1024) {
        delete c;
        return VCS_UNSUPPORTED;
    }
    if (c->kernel == VCS_KERNEL_PLAIN) {
        c->G = 1;
    } else if (cfg->lanes_per_env) {
        c->G = cfg->lanes_per_env;
        // 32 lanes (two envs per wave) only for translated code, which is compiled per shape
        if (c->G != 1 && c->G != 4 && c->G != 16 && c->G != 64 && !(c->G == 32 && c->kernel == VCS_KERNEL_TRANSLATED)) {
            delete c;
            return VCS_UNSUPPORTED;
        }
    } else {
        // Each env is a serial chain whose step latency is set by one wave's
        // instruction issue; a second wave on a SIMD only competes for the same
        // VALU.  Take the widest lane group that keeps about one wave per SIMD
        // (1024 SIMDs = 256 CUs x 4); more envs than that share waves.
        const int64_t lanes_budget = 1024LL * 64;
        c->G = (int64_t)c->B * 64 <= lanes_budget ? 64 : (int64_t)c->B * 16 <= lanes_budget ? 16
             : (int64_t)c->B * 4 <= lanes_budget ? 4 : 1;
    }
    // One env per wave (64 lanes) runs 16 envs per workgroup by default: they share
    // the workgroup's staged ROM image, so a large image does not cap the waves a
    // CU holds.  Otherwise 256 threads.  1024 only with one env per wave and the
    // interpreting kernel.
    if (c->tpb == 0) c->tpb = (c->G == 64 && c->kernel == VCS_KERNEL_GROUPED) ? 1024 : 256;
    if (c->tpb < c->G || (c->tpb == 1024 && (c->G != 64 || c->kernel != VCS_KERNEL_GROUPED))) {
        delete c;
        return VCS_UNSUPPORTED;
    }
    // translated code: at most 64 envs per workgroup (vcs_translate checks that its LDS fits);
    // its translator handles 2K, 4K and F8
    if (c->kernel == VCS_KERNEL_TRANSLATED) {
        bool ok = c->tpb / c->G <= 64;
        for (int32_t mp : c->rom_mapper) ok = ok && (mp == kMapper2K || mp == kMapper4K || mp == kMapperF8);
        if (!ok) {
            delete c;
            return VCS_UNSUPPORTED;
        }
    }
    // the LDS-staged kernels hold the image as 8-byte pre-decoded words, the envs' RAM
    // and Superchip RAM and the decode table in one CU's 160 KB; the plain kernel reads
    // global memory
    if (c->kernel != VCS_KERNEL_PLAIN && !lds_fits(c)) {
        delete c;
        return VCS_UNSUPPORTED;
    }
    c->main_E = c->tpb / c->G;
    group_by_rom(c, c->main_E, c->main_block_rom, c->main_slot_env);
    c->main_blocks = (int32_t)c->main_block_rom.size();
    group_by_rom(c, kBwdSlots, c->bwd_block_rom, c->bwd_slot_env);
    c->bwd_blocks = (int32_t)c->bwd_block_rom.size();
    c->env_bwd_slot.assign((size_t)c->B, -1);
    c->rom_bwd_begin.assign((size_t)c->R, 0);
    c->rom_bwd_end.assign((size_t)c->R, 0);
    for (int32_t blk = 0; blk < c->bwd_blocks; ++blk) {
        const int32_t r = c->bwd_block_rom[(size_t)blk];
        const int32_t first = blk * kBwdSlots;
        if (blk == 0 || c->bwd_block_rom[(size_t)blk - 1] != r) c->rom_bwd_begin[(size_t)r] = first;
        c->rom_bwd_end[(size_t)r] = first + kBwdSlots;
        for (int32_t j = 0; j < kBwdSlots; ++j) {
            const int32_t e = c->bwd_slot_env[(size_t)first + j];
            if (e >= 0) c->env_bwd_slot[(size_t)e] = first + j;
        }
    }
    // static device region image
    StaticHdr &h = c->hdr;
    h.num_roms = c->R;
    h.num_envs = c->B;
    h.main_slots_per_block = c->main_E;
    h.main_blocks = c->main_blocks;
    h.bwd_slots_per_block = kBwdSlots;
    h.bwd_blocks = c->bwd_blocks;
    h.max_rom_size = c->max_rom;
    h.total_rom_bytes = c->total_rom;
    size_t o = align_up(sizeof(StaticHdr));
    auto place = [&](int64_t &off, size_t n) {
        off = (int64_t)o;
        o = align_up(o + n * sizeof(int32_t));
    };
    place(h.off_rom_off, (size_t)c->R);
    place(h.off_rom_size, (size_t)c->R);
    place(h.off_rom_mapper, (size_t)c->R);
    place(h.off_main_block_rom, c->main_block_rom.size());
    place(h.off_main_slot_env, c->main_slot_env.size());
    place(h.off_bwd_block_rom, c->bwd_block_rom.size());
    place(h.off_bwd_slot_env, c->bwd_slot_env.size());
    place(h.off_env_bwd_slot, (size_t)c->B);
    place(h.off_rom_bwd_slot_begin, (size_t)c->R);
    place(h.off_rom_bwd_slot_end, (size_t)c->R);
    h.bytes = (int64_t)o;
    c->blob_bytes = o;
    c->image.assign(o, 0);
    std::memcpy(c->image.data(), &h, sizeof(h));
    auto put = [&](int64_t off, const std::vector<int32_t> &v) {
        if (!v.empty()) std::memcpy(c->image.data() + off, v.data(), v.size() * sizeof(int32_t));
    };
    put(h.off_rom_off, c->rom_off);
    put(h.off_rom_size, c->rom_size);
    put(h.off_rom_mapper, c->rom_mapper);
    put(h.off_main_block_rom, c->main_block_rom);
    put(h.off_main_slot_env, c->main_slot_env);
    put(h.off_bwd_block_rom, c->bwd_block_rom);
    put(h.off_bwd_slot_env, c->bwd_slot_env);
    put(h.off_env_bwd_slot, c->env_bwd_slot);
    put(h.off_rom_bwd_slot_begin, c->rom_bwd_begin);
    put(h.off_rom_bwd_slot_end, c->rom_bwd_end);
    *out = c;
    return VCS_OK;
}

void vcs_destroy(vcs_ctx *ctx) { delete ctx; }

int32_t vcs_state_bytes(const vcs_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return VCS_INVALID_ARG;
    *bytes = (size_t)ctx->B * (sizeof(StateRec) + (ctx->any_sc ? 128 : 0));
    return VCS_OK;
}

int32_t vcs_rom_bytes(const vcs_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return VCS_INVALID_ARG;
    *bytes = (size_t)ctx->total_rom;
    return VCS_OK;
}

int32_t vcs_workspace_bytes(const vcs_ctx *ctx, int32_t op, int32_t steps, size_t *bytes) {
    if (!ctx || !bytes || steps < 1) return VCS_INVALID_ARG;
    switch (op) {
        case VCS_OP_HARD: *bytes = hard_layout(ctx).bytes; return VCS_OK;
        case VCS_OP_SOFT_FWD: *bytes = align_up(ctx->blob_bytes); return VCS_OK;
        case VCS_OP_SOFT_BWD: *bytes = bwd_layout(ctx, steps).bytes; return VCS_OK;
        default: return VCS_INVALID_ARG;
    }
}

int32_t vcs_residual_bytes(const vcs_ctx *ctx, int32_t steps, size_t *bytes) {
    if (!ctx || !bytes || steps < 1) return VCS_INVALID_ARG;
    if (!ftape_ok(ctx, residual_layout(ctx, steps))) return VCS_INVALID_ARG;
    *bytes = residual_layout(ctx, steps).bytes;
    return VCS_OK;
}

int32_t vcs_decode_bytes(const vcs_ctx *ctx, int32_t steps, size_t *bytes) {
    if (!ctx || !bytes || steps < 1) return VCS_INVALID_ARG;
    *bytes = residual_layout(ctx, steps).stats_bytes;
    return VCS_OK;
}

int32_t vcs_residual_checkpoints(const vcs_ctx *ctx, int32_t steps, int32_t *count) {
    if (!ctx || !count || steps < 1) return VCS_INVALID_ARG;
    *count = residual_layout(ctx, steps).max_ckpt;
    return VCS_OK;
}

int32_t vcs_reset(vcs_ctx *ctx, void *d_state, const uint8_t *d_mask, const uint8_t *d_ram0, hipStream_t stream) {
    if (!ctx || !d_state || !aligned16(d_state)) return VCS_INVALID_ARG;
    if (d_ram0 && ((uintptr_t)d_ram0 & 3u)) return VCS_INVALID_ARG;
    const int32_t rc = ensure_pinned(ctx);  // so that later step calls can be captured
    if (rc) return rc;
    return hip_status(launch_reset((StateRec *)d_state, ctx->B, d_mask, d_ram0, ctx->seed, sc_state(ctx, d_state),
                                   stream));
}

}  // extern "C"

namespace {

int32_t check_step_hard_args(const vcs_ctx *ctx, const uint8_t *d_rom, const void *d_state, int32_t steps,
                             const uint8_t *d_ram_out, int32_t frames, const uint8_t *d_frame_out,
                             const uint32_t *d_episode_steps, int32_t num_episodes) {
    if (!ctx || !d_rom || !d_state || steps < 1) return VCS_INVALID_ARG;
    if (!aligned16(d_rom) || !aligned16(d_state)) return VCS_INVALID_ARG;
    if (frames < VCS_FRAMES_NONE || frames > VCS_FRAMES_ALL) return VCS_INVALID_ARG;
    if (frames != VCS_FRAMES_NONE && (!d_frame_out || !aligned16(d_frame_out))) return VCS_INVALID_ARG;
    if (d_ram_out && ((uintptr_t)d_ram_out & 3u)) return VCS_INVALID_ARG;
    if (d_episode_steps && num_episodes < 1) return VCS_INVALID_ARG;
    if ((int64_t)steps * ctx->F > (1 << 24)) return VCS_INVALID_ARG;
    return VCS_OK;
}

// The hard step's launches: the launch tables are already (in stream order) at
// d_tables.  With d_two (the rest of a hard workspace) the step runs in two passes:
// the starting states are copied aside, the kernel without the object paths runs
// every env and flags those that showed an object, and the kernel with them reruns
// the flagged envs from the copies; without it (no workspace) the kernel with the
// object paths runs every env.
int32_t launch_step_hard(vcs_ctx *ctx, const uint8_t *d_rom, void *d_state, const uint8_t *d_actions, int32_t steps,
                         uint8_t *d_ram_out, int32_t frames, uint8_t *d_frame_out, uint8_t *d_done,
                         const uint32_t *d_episode_steps, int32_t num_episodes, const void *d_tables,
                         uint8_t *d_two, hipStream_t stream) {
    StepParams P{};
    P.st = static_ptrs(ctx, d_tables);
    P.rom = d_rom;
    P.state = (StateRec *)d_state;
    P.actions = d_actions;
    P.steps = steps;
    P.frame_skip = ctx->F;
    P.ystart = ctx->ystart;
    P.frames_mode = frames;
    P.ram_out = d_ram_out;
    P.frame_out = frames == VCS_FRAMES_NONE ? nullptr : d_frame_out;
    P.done = d_done;
    P.ep_steps = d_episode_steps;
    P.num_episodes = d_episode_steps ? num_episodes : 0;
    P.seed = ctx->seed;
    P.sc_state = sc_state(ctx, d_state);
    P.rom_words = ctx->max_rom;
    const bool plain = ctx->kernel == VCS_KERNEL_PLAIN;
    if (!d_two)  // one pass with the object paths (the translated code has none: the interpreter runs)
        return hip_status(launch_step(P, ctx->main_blocks, ctx->G, ctx->tpb, false, plain, step_lds(ctx), stream));
    const HardLayout L = hard_layout(ctx);
    uint8_t *work = d_two - align_up(ctx->blob_bytes);  // the workspace's start
    StateRec *copy = (StateRec *)(work + L.states);
    uint8_t *sc_copy = ctx->any_sc ? work + L.sc : nullptr;
    uint8_t *flags = work + L.flags;
    if (hipMemcpyAsync(copy, d_state, (size_t)ctx->B * sizeof(StateRec), hipMemcpyDeviceToDevice, stream) !=
            hipSuccess ||
        (sc_copy && hipMemcpyAsync(sc_copy, P.sc_state, (size_t)ctx->B * 128, hipMemcpyDeviceToDevice, stream) !=
                        hipSuccess))
        return VCS_HIP_ERROR;
    P.obj_flag = flags;
    int32_t rc;
    if (ctx->kernel == VCS_KERNEL_TRANSLATED) {
        int dev = -1;
        if (!ctx->tr_fn || hipGetDevice(&dev) != hipSuccess || dev != ctx->tr_device) return VCS_UNSUPPORTED;
        void *args[] = {&P};
        const size_t lds = (size_t)ctx->max_rom * sizeof(uint2);
        // the emulating waves and as many drawing waves (the returned frames)
        rc = hip_status(hipModuleLaunchKernel(ctx->tr_fn, (unsigned)ctx->main_blocks, 1, 1, 2u * (unsigned)ctx->tpb,
                                              1, 1, (unsigned)lds, stream, args, nullptr));
    } else {
        rc = hip_status(launch_step(P, ctx->main_blocks, ctx->G, ctx->tpb, false, plain, step_lds(ctx), stream,
                                    false));
    }
    if (rc) return rc;
    P.obj_flag = nullptr;
    P.rerun = flags;
    P.state_src = copy;
    P.sc_src = sc_copy;
    return hip_status(launch_step(P, ctx->main_blocks, ctx->G, ctx->tpb, false, plain, step_lds(ctx), stream, true));
}

}  // namespace

extern "C" {

int32_t vcs_step_hard(vcs_ctx *ctx, const uint8_t *d_rom, void *d_state, const uint8_t *d_actions, int32_t steps,
                      uint8_t *d_ram_out, int32_t frames, uint8_t *d_frame_out, uint8_t *d_done,
                      const uint32_t *d_episode_steps, int32_t num_episodes, void *d_work, hipStream_t stream) {
    int32_t rc = check_step_hard_args(ctx, d_rom, d_state, steps, d_ram_out, frames, d_frame_out, d_episode_steps,
                                      num_episodes);
    if (rc) return rc;
    if (!d_work || !aligned16(d_work)) return VCS_INVALID_ARG;
    rc = upload_static(ctx, d_work, stream);
    if (rc) return rc;
    return launch_step_hard(ctx, d_rom, d_state, d_actions, steps, d_ram_out, frames, d_frame_out, d_done,
                            d_episode_steps, num_episodes, d_work, (uint8_t *)d_work + align_up(ctx->blob_bytes),
                            stream);
}

// vcs_step_hard with the launch tables in the library's static device array
// instead of a caller workspace; no allocation of any kind.  The context's
// pinned host copy of the tables must exist already (vcs_reset makes it).
int32_t vcs_step_hard_static(vcs_ctx *ctx, const uint8_t *d_rom, void *d_state, const uint8_t *d_actions,
                             int32_t steps, uint8_t *d_ram_out, int32_t frames, uint8_t *d_frame_out,
                             uint8_t *d_done, const uint32_t *d_episode_steps, int32_t num_episodes,
                             hipStream_t stream) {
    int32_t rc = check_step_hard_args(ctx, d_rom, d_state, steps, d_ram_out, frames, d_frame_out, d_episode_steps,
                                      num_episodes);
    if (rc) return rc;
    if (ctx->blob_bytes > kScratchBytes) return VCS_WORKSPACE_TOO_SMALL;
    if (!ctx->pinned) return VCS_UNSUPPORTED;  // making it would allocate: vcs_reset first
    void *tables = nullptr;
    rc = scratch_on_current_device(&tables);
    if (rc) return rc;
    if (hipMemcpyAsync(tables, ctx->pinned, ctx->blob_bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
        return VCS_HIP_ERROR;
    return launch_step_hard(ctx, d_rom, d_state, d_actions, steps, d_ram_out, frames, d_frame_out, d_done,
                            d_episode_steps, num_episodes, tables, nullptr, stream);
}

// FULL relaxed hard steps: the launch of vcs_step_hard with the relaxing kernel.
int32_t vcs_step_relaxed(vcs_ctx *ctx, const uint8_t *d_rom, void *d_state, const uint8_t *d_actions, int32_t steps,
                         uint8_t *d_ram_out, int32_t frames, uint8_t *d_frame_out, double alpha, double T,
                         int64_t *d_relax_out, void *d_work, hipStream_t stream) {
    int32_t rc = check_step_hard_args(ctx, d_rom, d_state, steps, d_ram_out, frames, d_frame_out, nullptr, 0);
    if (rc) return rc;
    if (!d_work || !aligned16(d_work) || !d_relax_out || ((uintptr_t)d_relax_out & 7u)) return VCS_INVALID_ARG;
    if (!(alpha > 0.0) || !(T > 0.0) || !std::isfinite(alpha) || !std::isfinite(T)) return VCS_INVALID_ARG;
    rc = upload_static(ctx, d_work, stream);
    if (rc) return rc;
    StepParams P{};
    P.st = static_ptrs(ctx, d_work);
    P.rom = d_rom;
    P.state = (StateRec *)d_state;
    P.actions = d_actions;
    P.steps = steps;
    P.frame_skip = ctx->F;
    P.ystart = ctx->ystart;
    P.frames_mode = frames;
    P.ram_out = d_ram_out;
    P.frame_out = frames == VCS_FRAMES_NONE ? nullptr : d_frame_out;
    P.seed = ctx->seed;
    P.sc_state = sc_state(ctx, d_state);
    P.rom_words = ctx->max_rom;
    // the weights and gates in double, stored as float (the kernel sums in float)
    P.relax_u[0] = 1.0f;
    for (int k = 1; k <= 8; ++k) P.relax_u[k] = (float)std::exp(-(double)k / T);
    P.relax_g_taken = (float)(1.0 / (1.0 + std::exp(-alpha)));
    P.relax_g_not = (float)(1.0 / (1.0 + std::exp(alpha)));
    P.relax_out = d_relax_out;
    if (!lds_fits(ctx)) return VCS_UNSUPPORTED;  // the relaxed kernel stages the image in LDS
    return hip_status(launch_step_relaxed(P, ctx->main_blocks, ctx->G, ctx->tpb, step_lds(ctx), stream));
}

int32_t vcs_translated_source(const vcs_ctx *ctx, const uint8_t *roms, int32_t max_positions, char *buf,
                              size_t buf_size, size_t *len) {
    if (!ctx || !roms || !len || max_positions < 0 || max_positions > 65536) return VCS_INVALID_ARG;
    TranslateStats st;
    const std::string src = translated_source(roms, ctx->rom_off, ctx->rom_size, ctx->rom_mapper, ctx->env_rom, ctx->seed,
                                              max_positions ? max_positions : kTranslateBudget, ctx->G, ctx->tpb, st);
    *len = src.size();
    if (buf && buf_size) {
        const size_t n = std::min(buf_size - 1, src.size());
        std::memcpy(buf, src.data(), n);
        buf[n] = '\0';
    }
    return VCS_OK;
}

int32_t vcs_translate(vcs_ctx *ctx, const uint8_t *roms, int32_t max_positions, int32_t flags,
                      vcs_translate_info *info, char *log, size_t log_size) {
    if (!ctx || !roms || (flags & ~VCS_TRANSLATE_COMPILE_ONLY)) return VCS_INVALID_ARG;
    if (max_positions < 0 || max_positions > 65536) return VCS_INVALID_ARG;
    const int budget = max_positions ? max_positions : kTranslateBudget;
    if (ctx->kernel != VCS_KERNEL_TRANSLATED) return VCS_UNSUPPORTED;
    if (!tr_lds_fits(ctx)) return VCS_UNSUPPORTED;  // the pixel logs of this many envs per workgroup do not fit
    if (log && log_size) log[0] = '\0';
    TranslateStats st;
    const std::string src = translated_source(roms, ctx->rom_off, ctx->rom_size, ctx->rom_mapper, ctx->env_rom, ctx->seed,
                                              budget, ctx->G, ctx->tpb, st);
    std::string code, clog;
    double secs = 0.0;
    bool cached = false;
    int32_t rc = jit_compile(src, code, clog, secs, cached);
    if (log && log_size) {
        const size_t n = std::min(log_size - 1, clog.size());
        std::memcpy(log, clog.data(), n);
        log[n] = '\0';
    }
    if (info) {
        info->positions = st.positions;
        info->runs = st.runs;
        info->truncated = st.truncated;
        info->cached = cached ? 1 : 0;
        info->compile_seconds = secs;
        info->source_bytes = src.size();
        info->code_bytes = code.size();
    }
    if (rc != VCS_OK || (flags & VCS_TRANSLATE_COMPILE_ONLY)) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return VCS_HIP_ERROR;
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    if (hipModuleLoadData(&mod, code.data()) != hipSuccess) return VCS_HIP_ERROR;
    if (hipModuleGetFunction(&fn, mod, "vcs_tr_step") != hipSuccess) {
        (void)hipModuleUnload(mod);
        return VCS_HIP_ERROR;
    }
    if (ctx->tr_module) (void)hipModuleUnload(ctx->tr_module);
    ctx->tr_module = mod;
    ctx->tr_fn = fn;
    ctx->tr_device = dev;
    return VCS_OK;
}

int32_t vcs_step_soft_fwd(vcs_ctx *ctx, const void *d_state_in, const float *d_rom_logits, const float *d_ram_tape,
                          const float *d_action_logits, float tau, float alpha, int32_t steps, float *d_ram_out,
                          float *d_frame_out, float *d_frame_dpos, float *d_decode_out, void *d_state_out,
                          void *d_residual, void *d_work, hipStream_t stream) {
    if (!ctx || !d_rom_logits || (!d_ram_tape && !d_state_in) || !d_action_logits || !d_residual || !d_work ||
        steps < 1)
        return VCS_INVALID_ARG;
    if (!(tau > 0.f) || !(alpha > 0.f)) return VCS_INVALID_ARG;
    if (!aligned16(d_rom_logits) || (d_ram_tape && !aligned16(d_ram_tape)) || ((uintptr_t)d_action_logits & 3u) ||
        !aligned16(d_residual) || !aligned16(d_work) || (d_state_in && !aligned16(d_state_in)))
        return VCS_INVALID_ARG;
    if (d_frame_dpos && (!d_frame_out || !aligned16(d_frame_dpos))) return VCS_INVALID_ARG;
    if ((d_ram_out && !aligned16(d_ram_out)) || (d_frame_out && !aligned16(d_frame_out)) ||
        (d_state_out && !aligned16(d_state_out)) || (d_decode_out && ((uintptr_t)d_decode_out & 3u)))
        return VCS_INVALID_ARG;
    if ((int64_t)steps * ctx->F > (1 << 24)) return VCS_INVALID_ARG;
    if (ctx->kernel == VCS_KERNEL_PLAIN || ctx->any_sc) return VCS_UNSUPPORTED;  // no Superchip RAM in the soft graph
    const ResidualLayout L = residual_layout(ctx, steps);
    if (!ftape_ok(ctx, L)) return VCS_INVALID_ARG;
    int32_t rc = upload_static(ctx, d_work, stream);
    if (rc) return rc;
    uint8_t *res = (uint8_t *)d_residual;
    // (from a given state the tape is not read: its statistics are zero)
    hipError_t e = d_ram_tape ? hipSuccess
                              : launch_fill_zero(res + L.tape_ev, (size_t)ctx->B * 128 * sizeof(float), stream);
    if (e != hipSuccess) return VCS_HIP_ERROR;
    e = launch_decode(d_rom_logits, ctx->total_rom, d_ram_tape, d_ram_tape ? (int64_t)ctx->B * 128 : 0,
                      d_action_logits, (int64_t)ctx->B * steps, tau, res + L.rom_hard, (float *)(res + L.rom_stats),
                      res + L.ram0_hard, (float *)(res + L.tape_ev), res + L.act_hard, (float *)(res + L.act_stats),
                      stream);
    if (e != hipSuccess) return VCS_HIP_ERROR;
    StepParams P{};
    P.st = static_ptrs(ctx, d_work);
    P.rom = res + L.rom_hard;
    P.state = (StateRec *)d_state_out;
    P.state_in = (const StateRec *)d_state_in;
    P.actions = res + L.act_hard;
    P.steps = steps;
    P.frame_skip = ctx->F;
    P.ystart = ctx->ystart;
    P.frames_mode = VCS_FRAMES_LAST;
    P.ram_out_f = d_ram_out;
    P.frame_out_f = d_frame_out;
    P.frame_dpos_f = d_frame_dpos;
    P.ram0 = res + L.ram0_hard;
    P.ckpt = (StateRec *)(res + L.ckpt);
    P.ckpt_count = (int32_t *)(res + L.ckpt_count);
    P.ckpt_interval = ctx->K;
    P.max_ckpt = L.max_ckpt;
    P.ftape = L.ftape_cap > 0 ? (uint4 *)(res + L.ftape) : nullptr;
    P.ftape_cap = (int32_t)L.ftape_cap;
    P.rom_words = ctx->max_rom;
    // Two passes, as for the hard steps: every env without the object paths,
    // flagging those in which an object shows, then those with them from the
    // same start.  The sampler's tangents need the object paths everywhere.
    uint8_t *obj_env = res + L.obj_env;
    P.obj_flag = obj_env;
    if (!d_frame_dpos) {
        rc = hip_status(launch_step(P, ctx->main_blocks, ctx->G, ctx->tpb, true, false, step_lds(ctx), stream, false));
        if (rc) return rc;
        P.obj_flag = nullptr;
        P.rerun = obj_env;
    }
    rc = hip_status(launch_step(P, ctx->main_blocks, ctx->G, ctx->tpb, true, false, step_lds(ctx), stream, true));
    if (rc) return rc;
    if (d_decode_out &&
        hipMemcpyAsync(d_decode_out, res + L.stats, L.stats_bytes, hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return VCS_HIP_ERROR;
    (void)alpha;  // flags carry no gradient in this relaxation, so the gate sharpness drops out
    return VCS_OK;
}

int32_t vcs_step_soft_bwd(vcs_ctx *ctx, const void *d_residual, const float *d_rom_logits,
                          const float *d_ram_tape, const float *d_action_logits, float tau, float alpha,
                          float read_T, int32_t steps, const float *d_grad_frame, const float *d_grad_ram_out,
                          float *d_grad_rom_logits, float *d_grad_ram_tape, float *d_grad_action_logits,
                          void *d_work, hipStream_t stream) {
    (void)d_ram_tape;  // dL/dP0[c,k] = k g0[c] needs no tape values
    if (!ctx || !d_residual || !d_rom_logits || !d_action_logits || !d_grad_frame || !d_grad_rom_logits ||
        !d_grad_action_logits || !d_work || steps < 1)
        return VCS_INVALID_ARG;
    if (!(tau > 0.f) || !(alpha > 0.f) || !(read_T >= 0.f) || !std::isfinite(read_T)) return VCS_INVALID_ARG;
    if (!aligned16(d_residual) || !aligned16(d_rom_logits) || !aligned16(d_grad_rom_logits) ||
        (d_grad_ram_tape && !aligned16(d_grad_ram_tape)) || !aligned16(d_work) || ((uintptr_t)d_grad_frame & 3u) ||
        ((uintptr_t)d_action_logits & 3u) || ((uintptr_t)d_grad_action_logits & 3u) ||
        (d_grad_ram_out && ((uintptr_t)d_grad_ram_out & 3u)))
        return VCS_INVALID_ARG;
    if ((int64_t)steps * ctx->F > (1 << 24)) return VCS_INVALID_ARG;
    if (ctx->any_sc || (size_t)ctx->max_rom * 8 + 16 * 128 + 1024 > kLdsBytes) return VCS_UNSUPPORTED;
    int32_t rc = upload_static(ctx, d_work, stream);
    if (rc) return rc;
    const ResidualLayout L = residual_layout(ctx, steps);
    if (!ftape_ok(ctx, L)) return VCS_INVALID_ARG;
    const BwdLayout W = bwd_layout(ctx, steps);
    const uint8_t *res = (const uint8_t *)d_residual;
    uint8_t *work = (uint8_t *)d_work;
    if (launch_fill_zero(work + W.gpart, W.overflow + kAlign - W.gpart, stream) != hipSuccess) return VCS_HIP_ERROR;
    BwdParams P{};
    P.st = static_ptrs(ctx, d_work);
    P.rom = res + L.rom_hard;
    P.actions = res + L.act_hard;
    P.ckpt = (const StateRec *)(res + L.ckpt);
    P.ckpt_count = (const int32_t *)(res + L.ckpt_count);
    P.max_ckpt = L.max_ckpt;
    P.steps = steps;
    P.frame_skip = ctx->F;
    P.ystart = ctx->ystart;
    P.ckpt_interval = ctx->K;
    P.grad_frame = d_grad_frame;
    P.grad_ram_out = d_grad_ram_out;
    P.tape = (TapeRec *)(work + W.tape);
    P.max_rec = W.max_rec;
    P.gpart = (float *)(work + W.gpart);
    P.gport = (float *)(work + W.gport);
    P.g_ram0 = (float *)(work + W.g0);
    P.overflow = (int32_t *)(work + W.overflow);
    P.read_T = read_T;
    P.ftape = L.ftape_cap > 0 ? (const uint4 *)(res + L.ftape) : nullptr;
    P.ftape_cap = (int32_t)L.ftape_cap;
    P.obj_env = res + L.obj_env;
    // the envs whose forward ran without the object paths, then the others
    rc = hip_status(launch_soft_bwd(P, ctx->bwd_blocks, ctx->max_rom, stream, false));
    if (rc) return rc;
    rc = hip_status(launch_soft_bwd(P, ctx->bwd_blocks, ctx->max_rom, stream, true));
    if (rc) return rc;
    const StaticPtrs sp = static_ptrs(ctx, d_work);
    return hip_status(launch_epilogue(d_rom_logits, (const float *)(res + L.rom_stats), P.gpart, ctx->total_rom,
                                      ctx->R, sp.rom_off, sp.rom_size, sp.rom_bwd_slot_begin, sp.rom_bwd_slot_end,
                                      W.nslots, tau, d_grad_rom_logits, P.g_ram0,
                                      d_grad_ram_tape ? (int64_t)ctx->B * 128 : 0, d_grad_ram_tape, d_action_logits, (const float *)(res + L.act_stats), P.gport,
                                      (int64_t)ctx->B * steps, d_grad_action_logits, stream));
}

int32_t vcs_read_regs(vcs_ctx *ctx, const void *d_state, uint8_t *d_out, hipStream_t stream) {
    if (!ctx || !d_state || !d_out || !aligned16(d_state)) return VCS_INVALID_ARG;
    return hip_status(launch_read_regs((const StateRec *)d_state, ctx->B, d_out, stream));
}

int32_t vcs_read_objects(vcs_ctx *ctx, const void *d_state, uint8_t *d_out, hipStream_t stream) {
    if (!ctx || !d_state || !d_out || !aligned16(d_state)) return VCS_INVALID_ARG;
    return hip_status(launch_read_objects((const StateRec *)d_state, ctx->B, d_out, stream));
}

int32_t vcs_hash(vcs_ctx *ctx, const void *d_state, const uint8_t *d_frame, int64_t frame_stride, uint64_t *d_out,
                 hipStream_t stream) {
    if (!ctx || !d_state || !d_out || !aligned16(d_state) || ((uintptr_t)d_out & 7u)) return VCS_INVALID_ARG;
    if (d_frame && (((uintptr_t)d_frame & 3u) || frame_stride < kPixels || (frame_stride & 3))) return VCS_INVALID_ARG;
    return hip_status(launch_hash((const StateRec *)d_state, ctx->B, d_frame, frame_stride, d_out, stream));
}

int32_t vcs_detect_mapper(const uint8_t *image, size_t size, int32_t *mapper) {
    if (!image || !mapper) return VCS_INVALID_ARG;
    if (size == 2048) return *mapper = VCS_MAPPER_2K, VCS_OK;
    if (size == 4096) return *mapper = VCS_MAPPER_4K, VCS_OK;
    if (size != 8192 && size != 16384 && size != 32768) return VCS_INVALID_ARG;
    // absolute accesses (loads, stores, BIT, CMP) to the E0 slice hotspots vs the F8 ones
    size_t e0 = 0, f8 = 0;
    for (size_t i = 0; i + 2 < size; ++i) {
        const uint8_t op = image[i], lo = image[i + 1], hi = image[i + 2];
        const bool abs = op == 0xAD || op == 0x8D || op == 0x2C || op == 0xAE || op == 0xAC || op == 0x8E ||
                         op == 0x8C || op == 0xCD;
        if (!abs || (hi & 0x1F) != 0x1F) continue;
        if (lo >= 0xE0 && lo <= 0xF7) ++e0;
        if (lo == 0xF8 || lo == 0xF9) ++f8;
    }
    if (size == 8192 && e0 > f8) return *mapper = VCS_MAPPER_E0, VCS_OK;
    // Superchip: the first 256 bytes of every bank (the RAM window) hold one repeated value
    bool sc = true;
    for (size_t b = 0; b < size && sc; b += 4096)
        for (size_t i = 1; i < 256 && sc; ++i) sc = image[b + i] == image[b];
    const int32_t base = size == 8192 ? VCS_MAPPER_F8 : size == 16384 ? VCS_MAPPER_F6 : VCS_MAPPER_F4;
    const int32_t with_sc = size == 8192 ? VCS_MAPPER_F8SC : size == 16384 ? VCS_MAPPER_F6SC : VCS_MAPPER_F4SC;
    *mapper = sc ? with_sc : base;
    return VCS_OK;
}

int32_t vcs_decode_table(uint32_t *out) {
    if (!out) return VCS_INVALID_ARG;
    constexpr DecodeTable t = make_decode_table();
    for (int i = 0; i < 256; ++i) out[i] = t.e[i];
    return VCS_OK;
}

// Soft-backward workspace check: copies the tape-overflow flag to the host
// after the stream's work is done (1 = a segment needed more tape records
// than the workspace holds, so that backward's result is invalid).
int32_t vcs_bwd_overflow(const vcs_ctx *ctx, const void *d_work, int32_t steps, hipStream_t stream,
                         int32_t *flag) {
    if (!ctx || !d_work || !flag || steps < 1) return VCS_INVALID_ARG;
    const BwdLayout W = bwd_layout(ctx, steps);
    if (hipMemcpyAsync(flag, (const uint8_t *)d_work + W.overflow, sizeof(int32_t), hipMemcpyDeviceToHost, stream) !=
        hipSuccess)
        return VCS_HIP_ERROR;
    return hip_status(hipStreamSynchronize(stream));
}

// Byte offset of the soft backward's int32 tape-overflow flag in its workspace.
int32_t vcs_bwd_overflow_offset(const vcs_ctx *ctx, int32_t steps, size_t *offset) {
    if (!ctx || !offset || steps < 1) return VCS_INVALID_ARG;
    *offset = bwd_layout(ctx, steps).overflow;
    return VCS_OK;
}

// Launch geometry chosen at create time (host values).
int32_t vcs_launch_info(const vcs_ctx *ctx, int32_t *kernel, int32_t *lanes_per_env, int32_t *block_threads,
                        int32_t *blocks, int32_t *bwd_blocks) {
    if (!ctx) return VCS_INVALID_ARG;
    if (kernel) *kernel = ctx->kernel;
    if (lanes_per_env) *lanes_per_env = ctx->G;
    if (block_threads) *block_threads = ctx->tpb;
    if (blocks) *blocks = ctx->main_blocks;
    if (bwd_blocks) *bwd_blocks = ctx->bwd_blocks;
    return VCS_OK;
}

}  // extern "C"
