// Test harness: a translated step kernel's code (the generated source named by
// TR_SOURCE) run on the host with one lane per wave, through the same per-env
// body as the device kernels.
#include <cstring>
#include <vector>
#define VCS_TR_FN __host__ __device__ __forceinline__
#define VCS_TR_TABLE static const
#define VCS_TR_NO_KERNEL
#define VCS_TR_ASYNC false  // no drawing wave: the hook draws the published rows itself
#include TR_SOURCE

using namespace vcs;

namespace {
struct OneLane {  // wave policy of a one-lane wave
    static constexpr uint32_t kWidth = 1;
    static bool any(bool v) { return v; }
    static bool all(bool v) { return v; }
    static void opaque(uint32_t &) {}
    static void opaque_uniform(uint32_t &) {}
    static void accumulate(float *p, float t) { *p += t; }
    static uint32_t first(uint32_t v) { return v; }
    static void fence() {}
    static void sleep() {}
    static uint32_t table(const uint32_t *t, uint32_t u) { return t[u]; }
};
constexpr DecodeTable kHostDecode = make_decode_table();
}  // namespace

// One env from power-on with RAM ram0 for S steps of F frames; outputs per step
// (RAM [S][128], frame [S][210][160], done [S]) for env index `env`, whose rows
// of ram_out/frame_out/done are written (they hold env + 1 envs' rows).  The
// translated code runs without the object paths: obj_flag[env] = 1 says an
// object showed and the outputs are void (the library then reruns the env).
extern "C" int host_translated(int rom_index, const uint8_t *rom, int rom_size, int mapper, const uint8_t *ram0,
                               const uint8_t *actions, int S, int F, const uint32_t *ep_steps, int num_eps,
                               unsigned long long seed, int env, uint8_t *ram_out, uint8_t *frame_out,
                               uint8_t *done, uint8_t *obj_flag) {
    std::vector<StateRec> st((size_t)env + 1);
    st[(size_t)env].status = 2;
    std::memcpy(st[(size_t)env].ram, ram0, 128);
    StepParams P{};
    P.state = st.data();
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
    P.obj_flag = obj_flag;  // [env + 1]: 1 when an object showed (the outputs are then void)
    std::vector<uint2> words(8192);
    for (int i = 0; i < rom_size; ++i) words[(size_t)i] = rom_word_at(rom, (uint32_t)i, mapper, kHostDecode.e);
    std::vector<uint32_t> ram_lds(32, 0);
    LdsWordMem m{words.data(), kHostDecode.e, reinterpret_cast<uint8_t *>(ram_lds.data()), 1u, 0u};
    std::vector<uint4> log((size_t)tr::kLogCap + 1u);
    TrCtl ctl{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, nullptr};
    step_env<OneLane, 1, false, false, tr::Exec, false>(
        P, env, 0, mapper, m, kHostDecode.e,
        tr::Exec::State{(uint32_t)rom_index, 0u, log.data(), &ctl, tr::kTabAll + tr::kTabOff[rom_index]});
    if (ctl.state != 0u || !ctl.fin) return -1;  // a frame left undrawn
    if (ctl.stalls) return -2;                    // a wait for the drawing gave up
    return 0;
}
