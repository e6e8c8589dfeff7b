// Run-time translation of ROM images into the TRANSLATED step kernel
// (implemented in vcs_jit.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace vcs {

struct TranslateStats {
    int32_t positions = 0;  // instruction positions translated, over all images
    int32_t runs = 0;       // straight-line runs they were emitted as
    int32_t truncated = 0;  // 1 if an image had more positions than the translation holds
};

// HIP source of the translated step kernel `vcs_tr_step` for the given images
// (host bytes, concatenated; offsets, sizes and mappers per image), the envs'
// image indices, the seed of the profiling RAM, the position budget and the
// launch shape (G lanes per env, TPB threads per workgroup).
std::string translated_source(const uint8_t *roms, const std::vector<int32_t> &rom_off,
                              const std::vector<int32_t> &rom_size, const std::vector<int32_t> &rom_mapper,
                              const std::vector<int32_t> &env_rom, uint64_t seed, int budget, int G, int TPB,
                              TranslateStats &stats);

// Instruction positions translated per context (compile time grows faster than
// linearly with the size of the generated function).
constexpr int kTranslateBudget = 256;

// Compile translated source for gfx950 with hiprtc (cached per process by
// source text).  Returns a vcs_status; `log` receives the compiler log.
int32_t jit_compile(const std::string &src, std::string &code, std::string &log, double &seconds, bool &cached);

}  // namespace vcs
