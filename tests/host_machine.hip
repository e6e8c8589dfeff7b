// Test harness: the library's per-env machine core and kernel bodies built for
// the host with a one-lane wave policy, so that CPU tests can compare them
// with the oracle (no GPU involved).
#include <cmath>
#include <cstring>
#include <vector>
#include "vcs_paths.hpp"

using namespace vcs;

namespace {
struct OneLane {  // wave policy of a one-lane wave
    static constexpr uint32_t kWidth = 1;
    static uint32_t lane() { return 0; }
    static uint32_t readlane(uint32_t v, uint32_t) { return v; }
    static float readlane(float v, uint32_t) { return v; }
    static float writelane(float, float x, uint32_t) { return x; }
    static float sum(float v) { return v; }
    static bool any(bool v) { return v; }
    static bool all(bool v) { return v; }
    static void opaque(uint32_t &) {}
    static void opaque_uniform(uint32_t &) {}
    static void accumulate(float *p, float t) { *p += t; }
    static uint32_t first(uint32_t v) { return v; }
    static uint32_t table(const uint32_t *t, uint32_t u) { return t[u]; }
};
constexpr DecodeTable kHostDecode = make_decode_table();
}  // namespace

// One env from power-on with RAM ram0 for S steps of F frames through the
// GROUPED interpreter's body (plain = 0: ROM as pre-decoded words, RAM in the
// word layout, wave-uniform dispatch) or the PLAIN kernel's body (plain = 1:
// ROM and RAM in global memory, per-lane switch).  Outputs per step: RAM
// [S][128], frame [S][210][160], done [S]; regs[16] = the inspection bytes
// after the last step (vcs_read_regs layout).
extern "C" int host_interp(int plain, const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0,
                           const uint8_t *actions, int S, int F, const uint32_t *ep_steps, int num_eps,
                           unsigned long long seed, uint8_t *ram_out, uint8_t *frame_out, uint8_t *done,
                           uint8_t *regs, uint8_t *objs) {
    StateRec st{};
    st.status = 2;
    st.tim_shift = 10;
    std::memcpy(st.ram, ram0, 128);
    // Superchip RAM as vcs_reset seeds it (env 0)
    uint8_t sc_state[128];
    for (uint32_t w = 0; w < 16; ++w) {
        const uint64_t v = reset_ram_word(seed ^ kScSeed, 0, 0, w);
        for (int k = 0; k < 8; ++k) sc_state[8 * w + k] = (uint8_t)(v >> (8 * k));
    }
    std::vector<uint32_t> sc_lds(32, 0);
    StepParams P{};
    P.state = &st;
    P.sc_state = mapper_sc(mapper) ? sc_state : nullptr;
    P.actions = actions;
    P.steps = S;
    P.frame_skip = F;
    P.ystart = 34;
    P.frames_mode = 2;
    P.ram_out = ram_out;
    P.frame_out = frame_out;
    P.done = done;
    P.ep_steps = ep_steps;
    P.num_episodes = num_eps;
    P.seed = seed;
    if (plain) {
        GlobalMem m{rom, st.ram, P.sc_state};
        step_env<OneLane, 1, false, true>(P, 0, 0, mapper, m, kHostDecode.e);
    } else {
        std::vector<uint2> words(32768);
        for (int i = 0; i < rom_size; ++i) words[(size_t)i] = rom_word_at(rom, (uint32_t)i, mapper, kHostDecode.e);
        std::vector<uint32_t> ram_lds(32, 0);
        LdsWordMem m{words.data(), kHostDecode.e, reinterpret_cast<uint8_t *>(ram_lds.data()), 1u, 0u};
        if (mapper_sc(mapper)) m.sc = reinterpret_cast<uint8_t *>(sc_lds.data());
        step_env<OneLane, 1, false, false>(P, 0, 0, mapper, m, kHostDecode.e);
    }
    // inspection bytes, as vcs_read_regs forms them
    const int32_t t = st.cyc, dd = t - st.tim_u;
    regs[0] = st.a; regs[1] = st.x; regs[2] = st.y; regs[3] = st.s; regs[4] = st.p;
    regs[5] = (uint8_t)(st.pc & 0xFF); regs[6] = (uint8_t)(st.pc >> 8); regs[7] = st.bank; regs[8] = st.status;
    regs[9] = (uint8_t)(dd < 0 ? (-1 - (dd >> st.tim_shift)) : (255 - dd));
    regs[10] = (uint8_t)((t >= st.tim_u && st.tim_read < st.tim_u) ? 0x80 : 0);
    regs[11] = st.vblank;
    for (int i = 0; i < 4; ++i) regs[12 + i] = (uint8_t)(st.col >> (8 * i));
    if (objs) objects32(st, objs);
    return 0;
}

// The first pass of a hard step: the same env run without the object paths
// (the GROUPED kernel's body, plain = 0, or the PLAIN kernel's, plain = 1).
// flag = 1 when an object showed (the outputs are then void and the step is
// rerun with the object paths); otherwise outputs as host_interp.
extern "C" int host_fast(int plain, const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0,
                         const uint8_t *actions, int S, int F, unsigned long long seed, uint8_t *ram_out,
                         uint8_t *frame_out, uint8_t *flag) {
    StateRec st{};
    st.status = 2;
    st.tim_shift = 10;
    std::memcpy(st.ram, ram0, 128);
    StepParams P{};
    P.state = &st;
    P.actions = actions;
    P.steps = S;
    P.frame_skip = F;
    P.ystart = 34;
    P.frames_mode = 2;
    P.ram_out = ram_out;
    P.frame_out = frame_out;
    P.seed = seed;
    P.obj_flag = flag;
    if (plain) {
        GlobalMem m{rom, st.ram, nullptr};
        step_env<OneLane, 1, false, true, InterpExec, false>(P, 0, 0, mapper, m, kHostDecode.e);
    } else {
        std::vector<uint2> words(32768);
        for (int i = 0; i < rom_size; ++i) words[(size_t)i] = rom_word_at(rom, (uint32_t)i, mapper, kHostDecode.e);
        std::vector<uint32_t> ram_lds(32, 0);
        LdsWordMem m{words.data(), kHostDecode.e, reinterpret_cast<uint8_t *>(ram_lds.data()), 1u, 0u};
        step_env<OneLane, 1, false, false, InterpExec, false>(P, 0, 0, mapper, m, kHostDecode.e);
    }
    return 0;
}

// SOFT-STE forward and the surrogate backward of one env on the host, through
// the soft kernels' bodies: forward on the decoded leaves (rom: decoded bytes,
// actions [S]) with a hard-state checkpoint every K cycles, from power-on with
// RAM ram0 (pre_steps = 0) or from the state after pre_steps hard env steps of
// pre_actions from power-on with ram0 (then the state is a constant and
// g_ram0 is zero); then the backward from dL/dframe [210][160] and
// dL/dRAM_out [S][128] (NULL = zero).  Outputs: ram_out [S][128] and frame
// [210][160] as floats, the per-byte ROM value gradient g_rom [rom_size],
// g_ram0 [128] and the port gradients g_port [S][2] (SWCHA, INPT4), before the
// softmax epilogue, and (frame_dpos not NULL) the position sampler's tangents
// of the final frame [5][210][160]; read_T > 0 turns on the address surrogate.
// Returns the number of checkpoints, or -1 if the tape overflowed.
static int soft_run(const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0, int pre_steps,
                    const uint8_t *pre_actions, const uint8_t *actions, int S, int F, int K, const float *grad_frame,
                    const float *grad_ram, float *ram_out, float *frame_out, float *g_rom, float *g_ram0,
                    float *g_port, float *frame_dpos, float read_T, int tape_cap, int *taped, int objects = 1) {
    std::vector<uint2> words(32768);
    for (int i = 0; i < rom_size; ++i) words[(size_t)i] = rom_word_at(rom, (uint32_t)i, mapper, kHostDecode.e);
    const int max_ckpt = (int)(((int64_t)S * F * kCyclesPerFrame + 256) / K + 3);
    std::vector<StateRec> ckpt((size_t)max_ckpt);
    int32_t nck = 0;
    StateRec st{};
    std::vector<uint4> ftape((size_t)(tape_cap > 0 ? tape_cap : 1));
    if (pre_steps > 0) {  // hard steps from power-on, through the hard interpreter's body
        st.status = 2;
        st.tim_shift = 10;
        std::memcpy(st.ram, ram0, 128);
        StepParams P{};
        P.state = &st;
        P.actions = pre_actions;
        P.steps = pre_steps;
        P.frame_skip = F;
        P.ystart = 34;
        std::vector<uint32_t> ram_lds(32, 0);
        LdsWordMem m{words.data(), kHostDecode.e, reinterpret_cast<uint8_t *>(ram_lds.data()), 1u, 0u};
        step_env<OneLane, 1, false, false>(P, 0, 0, mapper, m, kHostDecode.e);
    }
    {
        StepParams P{};
        P.rom = rom;
        P.actions = actions;
        P.steps = S;
        P.frame_skip = F;
        P.ystart = 34;
        P.frames_mode = 1;
        P.ram_out_f = ram_out;
        P.frame_out_f = frame_out;
        P.frame_dpos_f = frame_dpos;
        P.ram0 = ram0;
        P.state_in = pre_steps > 0 ? &st : nullptr;
        P.ckpt = ckpt.data();
        P.ckpt_count = &nck;
        P.ckpt_interval = K;
        P.max_ckpt = max_ckpt;
        P.ftape = tape_cap > 0 ? ftape.data() : nullptr;
        P.ftape_cap = tape_cap;
        uint8_t flag = 7;
        P.obj_flag = &flag;
        std::vector<uint32_t> ram_lds(32, 0);
        LdsWordMem m{words.data(), kHostDecode.e, reinterpret_cast<uint8_t *>(ram_lds.data()), 1u, 0u};
        if (objects) {
            if (tape_cap > 0) step_env<OneLane, 1, true, false, TapeFwdExec>(P, 0, 0, mapper, m, kHostDecode.e);
            else step_env<OneLane, 1, true, false>(P, 0, 0, mapper, m, kHostDecode.e);
        } else {  // the first pass: an env in which an object shows is flagged (and rerun by the library)
            if (tape_cap > 0) step_env<OneLane, 1, true, false, TapeFwdExec, false>(P, 0, 0, mapper, m, kHostDecode.e);
            else step_env<OneLane, 1, true, false, InterpExec, false>(P, 0, 0, mapper, m, kHostDecode.e);
            if (flag) return -2;
        }
    }
    *taped = 0;
    for (int i = 0; i < nck && i < max_ckpt; ++i) *taped += tape_cap > 0 && ckpt[(size_t)i].tape_n >= 0;
    BwdParams Q{};
    Q.rom = rom;
    Q.actions = actions;
    Q.ckpt = ckpt.data();
    Q.ckpt_count = &nck;
    Q.max_ckpt = max_ckpt;
    Q.steps = S;
    Q.frame_skip = F;
    Q.ystart = 34;
    Q.ckpt_interval = K;
    Q.grad_frame = grad_frame;
    Q.grad_ram_out = grad_ram;
    Q.max_rec = K / 2 + 64 + K / kCyclesPerFrame + 4;
    std::vector<TapeRec> tape((size_t)Q.max_rec);
    Q.tape = tape.data();
    for (int i = 0; i < rom_size; ++i) g_rom[i] = 0.f;
    for (int i = 0; i < 2 * S; ++i) g_port[i] = 0.f;
    Q.gpart = g_rom;
    Q.gport = g_port;
    Q.g_ram0 = g_ram0;
    int32_t overflow = 0;
    Q.overflow = &overflow;
    Q.read_T = read_T;
    Q.ftape = tape_cap > 0 ? ftape.data() : nullptr;
    Q.ftape_cap = tape_cap;
    std::vector<uint32_t> ram_lds(32, 0);
    LdsWordMem m{words.data(), kHostDecode.e, reinterpret_cast<uint8_t *>(ram_lds.data()), 1u, 0u};
    if (objects) bwd_env<OneLane>(Q, 0, 0, 1, mapper, (uint32_t)rom_size, m, kHostDecode.e);
    else bwd_env<OneLane, false>(Q, 0, 0, 1, mapper, (uint32_t)rom_size, m, kHostDecode.e);
    return overflow ? -1 : nck;
}

extern "C" int host_soft(const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0, int pre_steps,
                         const uint8_t *pre_actions, const uint8_t *actions, int S, int F, int K,
                         const float *grad_frame, const float *grad_ram, float *ram_out, float *frame_out,
                         float *g_rom, float *g_ram0, float *g_port, float *frame_dpos, float read_T) {
    int taped = 0;
    return soft_run(rom, rom_size, mapper, ram0, pre_steps, pre_actions, actions, S, F, K, grad_frame, grad_ram,
                    ram_out, frame_out, g_rom, g_ram0, g_port, frame_dpos, read_T, 0, &taped);
}

// host_soft with the forward keeping its tape (tape_cap records, at most; the
// segments it completes before the final frame, while they fit; 0 = none):
// *taped = the number of segments the backward swept from that tape.  objects =
// 0: the forward and backward without the object paths (the library's first
// pass); returns -2 when the forward flags the env (an object showed).
extern "C" int host_soft_tape(const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0, int pre_steps,
                              const uint8_t *pre_actions, const uint8_t *actions, int S, int F, int K,
                              const float *grad_frame, const float *grad_ram, float *ram_out, float *frame_out,
                              float *g_rom, float *g_ram0, float *g_port, float read_T, int tape_cap, int *taped,
                              int objects) {
    return soft_run(rom, rom_size, mapper, ram0, pre_steps, pre_actions, actions, S, F, K, grad_frame, grad_ram,
                    ram_out, frame_out, g_rom, g_ram0, g_port, nullptr, read_T, tape_cap, taped, objects);
}

// FULL relaxed rollout of one env from power-on with RAM ram0 (S steps of F
// frames) through the relaxed kernel's body: the grouped interpreter with the
// relaxing memory policy.  u[0..8] and the gates as vcs_step_relaxed forms them
// (in double, stored as float).  Outputs: RAM [S][128], frames [S][210][160],
// relax[2] = (first diverging instruction or -1, casts that differed).
extern "C" int host_relaxed(const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0,
                            const uint8_t *actions, int S, int F, double alpha, double T, uint8_t *ram_out,
                            uint8_t *frame_out, long long *relax) {
    StateRec st{};
    st.status = 2;
    st.tim_shift = 10;
    std::memcpy(st.ram, ram0, 128);
    int64_t out[2] = {0, 0};
    StepParams P{};
    P.state = &st;
    P.actions = actions;
    P.steps = S;
    P.frame_skip = F;
    P.ystart = 34;
    P.frames_mode = 2;
    P.ram_out = ram_out;
    P.frame_out = frame_out;
    P.relax_out = out;
    std::vector<uint2> words(32768);
    for (int i = 0; i < rom_size; ++i) words[(size_t)i] = rom_word_at(rom, (uint32_t)i, mapper, kHostDecode.e);
    std::vector<uint32_t> ram_lds(32, 0);
    RelaxMem<LdsWordMem> m;
    static_cast<LdsWordMem &>(m) = LdsWordMem{words.data(), kHostDecode.e,
                                              reinterpret_cast<uint8_t *>(ram_lds.data()), 1u, 0u};
    m.rc.u[0] = 1.0f;
    for (int k = 1; k <= 8; ++k) m.rc.u[k] = (float)std::exp(-(double)k / T);
    m.rc.g_taken = (float)(1.0 / (1.0 + std::exp(-alpha)));
    m.rc.g_not = (float)(1.0 / (1.0 + std::exp(alpha)));
    m.rom_n = (uint32_t)rom_size;
    m.active = false;
    m.ninstr = 0;
    m.ndiv = -1;
    m.fails = 0;
    step_env<OneLane, 1, false, false>(P, 0, 0, mapper, m, kHostDecode.e);
    relax[0] = out[0];
    relax[1] = out[1];
    return 0;
}
