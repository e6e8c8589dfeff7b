// Translation of ROM images into straight-line HIP code, compiled at run time
// (hiprtc) into the TRANSLATED step kernel.
//
// The emulated program is fixed per context, so the interpreter's per-
// instruction work (fetch, decode, opcode dispatch) can be done once, on the
// host.  The code an image executes is found by running it on the host with
// the library's own machine core (a few envs, a few frames); its page-0-form
// instructions (immediate, implied, zero-page, stack, relative: what VCS code
// mostly executes) are grouped into basic blocks ("runs", split where the
// profile entered code other than by falling through), and each run becomes
// one case of a switch over run ids.  A run's body executes its instructions
// with opcodes and operand bytes as compile-time constants (the same machine
// core instantiated per opcode, so the same semantics) and with no exit until
// its end; every lane of the wave checks once, at entry, that all of them
// start before the frame's cycle limit (from a static bound on the run's
// cycles) and that their page-0 writes share addresses, so the body needs no
// per-lane branch.  A wave whose lanes are at different runs, a failed entry
// check, and positions outside the translation (other addressing modes, code
// in RAM, code the profile did not reach) take the interpreter for one
// instruction, after which the next run start is looked up in a table.  The
// kernel therefore runs exactly the interpreter's machine.
#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/vcs.h"
#include "vcs_jit.hpp"
#include "vcs_paths.hpp"

namespace vcs {
namespace {

#include "vcs_jit_headers.inc"  // kJitHeaderNames / kJitHeaderText: the device headers as text


struct Pos {
    uint32_t bank, pc, op, lo, hi, d;
};

struct RomCode {
    std::vector<Pos> pos;                // index = id - 1
    std::map<uint32_t, uint32_t> id_of;  // key bank << 16 | pc
    std::set<uint32_t> leaders;          // keys of positions entered other than by falling through
    std::vector<uint64_t> count;         // executions per position in the profile (index = id - 1)
    int banks = 1;
    bool truncated = false;
};

uint32_t key(uint32_t bank, uint32_t pc) { return (bank << 16) | (pc & 0xFFFFu); }

// Bytes as the CPU fetches them: cartridge offset of address pc in `bank`.
struct Image {
    const uint8_t *img;
    int32_t size, mapper;
    uint32_t byte(uint32_t bank, uint32_t pc) const {
        const uint32_t amask = mapper == 0 ? 0x7FFu : 0xFFFu;
        return img[(pc & amask) + (bank << 12)];
    }
};

// Instruction positions the translated code can hold: opcode and both operand
// bytes inside one cartridge window (what the interpreter serves from its
// pre-decoded words).
bool translatable(uint32_t pc) { return (pc & 0x1000u) && (pc & 0xFFFu) <= 0xFFDu; }

bool accesses_data(uint32_t d) {
    const uint32_t cls = d & 63u, mode = (d >> 6) & 15u;
    const bool load = (cls >= C_LDA && cls <= C_LAX) || (cls >= C_ADC && cls <= C_BIT);
    const bool rmw = cls >= C_ASL && cls <= C_DEC;
    const bool store = cls >= C_STA && cls <= C_SAX;
    return (load && mode != M_IMM) || (rmw && mode != M_ACC) || store;
}

// Whether a data access of this instruction may hit an F8 hotspot ($1FF8/$1FF9
// in the 13-bit bus), which switches the bank under the following code.
bool may_switch_bank(uint32_t d, uint32_t lo, uint32_t hi) {
    if (!accesses_data(d)) return false;
    const uint32_t mode = (d >> 6) & 15u, base = lo | (hi << 8);
    auto hot = [](uint32_t a) { return (a & 0x1FFEu) == 0x1FF8u; };
    switch (mode) {
        case M_ABS: return hot(base);
        case M_ABX:
        case M_ABY:
            for (uint32_t i = 0; i < 256; ++i)
                if (hot((base + i) & 0xFFFFu)) return true;
            return false;
        case M_IZX:
        case M_IZY: return true;
        default: return false;  // page-0 forms
    }
}

enum Flow { kNext, kBranch, kStatic, kDynamic, kJam };

// Control flow after an instruction and its static successors.
Flow flow_of(const Pos &p, int mapper, uint32_t &target) {
    const uint32_t cls = p.d & 63u, mode = (p.d >> 6) & 15u, len = (p.d >> 14) & 3u;
    target = 0;
    if (p.d == 0) return kJam;
    switch (cls) {
        case C_BRANCH: target = (p.pc + 2u + (uint32_t)(int32_t)(int8_t)p.lo) & 0xFFFFu; return kBranch;
        case C_JMP:
            if (mode == M_IND) return kDynamic;
            target = p.lo | (p.hi << 8);
            return kStatic;
        case C_JSR: target = p.lo | (p.hi << 8); return kStatic;
        case C_RTS: case C_RTI: case C_BRK: return kDynamic;
        default: break;
    }
    if (mapper == 2 && may_switch_bank(p.d, p.lo, p.hi)) return kDynamic;
    (void)len;
    return kNext;
}

// Instruction positions worth translating, found by running the image on the
// host with the library's own machine core (the interpreter, one env at a
// time): kProfileEnvs envs with different RAM and joystick inputs for
// kProfileFrames frames each; every translatable position they execute is
// kept with its execution count.  Positions the real envs reach outside this
// set run on the interpreter.
constexpr int kProfileEnvs = 8, kProfileFrames = 4;
constexpr int64_t kProfileMaxInstructions = 1 << 20;

struct Profile {
    std::map<uint32_t, uint64_t> count;  // executions per position
    std::set<uint32_t> leaders;          // positions entered other than by falling through
};

Profile profile(const Image &im, uint64_t seed) {
    Profile pr;
    std::map<uint32_t, uint64_t> &count = pr.count;
    for (int e = 0; e < kProfileEnvs; ++e) {
        uint8_t ram[128];
        for (uint32_t w = 0; w < 16; ++w) {
            const uint64_t v = reset_ram_word(seed, (uint64_t)e, 0, w);
            for (int k = 0; k < 8; ++k) ram[8 * w + k] = (uint8_t)(v >> (8 * k));
        }
        Cpu<GlobalMem, RenderHook<uint8_t>> c;
        c.set_cart(im.mapper);  // 2K, 4K or F8 (the formats the translator takes)
        c.mem = GlobalMem{im.img, ram, nullptr};
        c.hook.frame = nullptr;
        c.hook.tan = nullptr;
        c.hook.rend_cc = c.hook.pix_cc = 0;
        c.hook.ystart = 34;
        c.hook.sub = 0;
        c.hook.G = 1;
        c.bank = 0;
        c.power_on();
        int64_t n = 0;
        uint32_t expect = 0xFFFFFFFFu;  // key of the fall-through successor of the last instruction
        for (int f = 0; f < kProfileFrames && !c.jam && n < kProfileMaxInstructions; ++f) {
            action_ports((uint32_t)(e * 7 + f) % 18u, &c.swcha, &c.inpt4, &c.swchb);
            while (!c.jam && c.cyc < kCyclesPerFrame && n < kProfileMaxInstructions) {
                const uint32_t k = key(c.bank, c.pc);
                if (translatable(c.pc)) {
                    ++count[k];
                    if (k != expect) pr.leaders.insert(k);
                }
                uint32_t opc, lo, hi;
                fetch3(c, opc, lo, hi);
                const uint32_t d = decode_op(opc);
                if (d == 0) {
                    c.jam = 1;
                    break;
                }
                ExecInfo info;
                c.exec(opc, d, lo, hi, info);
                const uint32_t seq = key(k >> 16, ((k & 0xFFFFu) + ((d >> 14) & 3u)) & 0xFFFFu);
                expect = key(c.bank, c.pc) == seq ? seq : 0xFFFFFFFFu;
                ++n;
            }
            if (c.cyc < kCyclesPerFrame) c.cyc = kCyclesPerFrame;
            c.next_frame();
        }
    }
    return pr;
}

// The `budget` most executed positions of the profile.
RomCode select_positions(const Image &im, const Profile &pr, int budget) {
    const std::map<uint32_t, uint64_t> &count = pr.count;
    RomCode rc;
    rc.leaders = pr.leaders;
    rc.banks = im.mapper == 2 ? 2 : 1;
    std::vector<std::pair<uint64_t, uint32_t>> order;
    for (const auto &kv : count) {
        const uint32_t op = im.byte(kv.first >> 16, kv.first & 0xFFFFu);
        if (decode_op(op) == 0 || fast_form(op)) order.push_back({kv.second, kv.first});  // others: interpreter
    }
    std::stable_sort(order.begin(), order.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    budget = std::min(budget, 4095);  // ids fit the lookup table's 12-bit field
    if ((int)order.size() > budget) {
        order.resize((size_t)std::max(budget, 0));
        rc.truncated = true;
    }
    std::sort(order.begin(), order.end(), [](const auto &x, const auto &y) { return x.second < y.second; });
    for (const auto &o : order) {
        Pos p;
        p.bank = o.second >> 16;
        p.pc = o.second & 0xFFFFu;
        p.op = im.byte(p.bank, p.pc);
        p.lo = im.byte(p.bank, (p.pc + 1u) & 0xFFFFu);
        p.hi = im.byte(p.bank, (p.pc + 2u) & 0xFFFFu);
        p.d = decode_op(p.op);
        rc.pos.push_back(p);
        rc.count.push_back(o.first);
        rc.id_of[key(p.bank, p.pc)] = (uint32_t)rc.pos.size();
    }
    return rc;
}

void emit_rom(std::string &s, const Image &im, int r, const RomCode &rc, TranslateStats &stats,
              std::vector<uint16_t> &table) {
    char buf[1024];
    const int nb = rc.banks;
    auto id = [&](uint32_t bank, uint32_t pc) -> uint32_t {
        auto it = rc.id_of.find(key(bank, pc & 0xFFFFu));
        return it == rc.id_of.end() ? 0u : it->second;
    };
    // Straight-line runs (basic blocks of the translated positions), each with
    // one entry, its first position.  A run ends at a branch, jump, return or
    // jam, before a position that is entered other than by falling through (a
    // leader), after TXS, before an indexed page-0 write, and at kMaxRun
    // positions.  A write that may hit WSYNC counts a line (76 cycles) in the
    // run's cycle bound.
    constexpr size_t kMaxRun = (size_t)kTrMaxRun;
    auto write_kind = [](const Pos &p) -> int {  // 0 none, 1 constant address, 2 per-lane address, 3 push
        const uint32_t cls = p.d & 63u, mode = (p.d >> 6) & 15u;
        if (cls == C_PHA || cls == C_PHP) return 3;
        const bool writes = (cls >= C_STA && cls <= C_SAX) || (cls >= C_ASL && cls <= C_DEC && mode != M_ACC);
        if (!writes) return 0;
        return (mode == M_ZPX || mode == M_ZPY) ? 2 : 1;
    };
    auto may_stall = [&](const Pos &p) {  // a write that may be to WSYNC (pushes go to RAM: entry check)
        const int wk = write_kind(p);
        return wk == 2 || (wk == 1 && p.lo < 0x80u && (p.lo & 0x3Fu) == 0x02u);
    };
    std::vector<uint32_t> order(rc.pos.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (uint32_t)i;
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return key(rc.pos[a].bank, rc.pos[a].pc) < key(rc.pos[b].bank, rc.pos[b].pc);
    });
    std::vector<char> done(rc.pos.size(), 0);
    std::vector<std::vector<uint32_t>> runs;
    std::vector<char> starts(rc.pos.size(), 0);
    for (uint32_t start : order) {
        if (done[start]) continue;
        std::vector<uint32_t> run;
        for (uint32_t i = start;;) {
            done[i] = 1;
            run.push_back(i);
            const Pos &p = rc.pos[i];
            uint32_t t;
            if (flow_of(p, im.mapper, t) != kNext) break;
            if ((p.d & 63u) == C_TXS || run.size() >= kMaxRun) break;
            const uint32_t nx = id(p.bank, p.pc + ((p.d >> 14) & 3u));
            if (!nx || done[nx - 1] || write_kind(rc.pos[nx - 1]) == 2) break;
            if (rc.leaders.count(key(rc.pos[nx - 1].bank, rc.pos[nx - 1].pc))) break;
            i = nx - 1;
        }
        starts[run[0]] = 1;
        runs.push_back(run);
    }
    // successor id: a run start, else 0 (the interpreter until the next run start)
    auto sid = [&](uint32_t bank, uint32_t pc) -> uint32_t {
        const uint32_t i = id(bank, pc);
        return i && starts[i - 1] ? i : 0u;
    };
    // lookup table: (bank, pc & 0xFFF) -> run start id | pc >> 12 << 12 (the id
    // counts only when the pc's high bits match)
    table.assign((size_t)nb * 4096, 0);
    for (size_t i = 0; i < rc.pos.size(); ++i) {
        if (!starts[i]) continue;
        const Pos &p = rc.pos[i];
        uint16_t &slot = table[((size_t)p.bank << 12) | (p.pc & 0xFFFu)];
        if (!slot) slot = (uint16_t)((i + 1) | ((p.pc >> 12) << 12));
    }
    std::snprintf(buf, sizeof buf,
                  "template <class W, class C>\n"
                  "VCS_TR_FN void blocks%d(C &c, uint32_t u, uint32_t &blk, uint32_t &fb, int32_t lim, "
                  "const uint16_t *tab) {\n",
                  r);
    s += buf;
    // Each run: the entry check, made once by every lane of the wave (the
    // instructions up to the run's last one all start before the cycle limit;
    // every lane writes the same page-0 / stack addresses: the stack pointer
    // agrees and stays in RAM, an indexed page-0 write, which must start its
    // run, has one address), then the body with no exit until its end.  A
    // failed check sends the wave to the interpreter for one instruction.
    std::vector<std::pair<uint64_t, std::string>> run_code;  // (entries in the profile, code after the case label)
    for (std::vector<uint32_t> run : runs) {
        std::string code;
        const uint64_t entries = rc.count[run[0]];
        const Pos &last = rc.pos[run.back()];
        uint32_t t;
        const Flow f = flow_of(last, im.mapper, t);
        if (f == kJam && run.size() == 1) {
            std::snprintf(buf, sizeof buf, "%u|c.jam = 1; break;\n", run[0] + 1);
            run_code.push_back({0, buf});
            continue;
        }
        if (f == kJam) run.pop_back();  // the jam is then reached through the dispatch
        // cycle bound, and the range of push addresses relative to the entry stack pointer
        int32_t pre = 0, off = 0, lo_push = 1 << 30, hi_push = -(1 << 30);
        for (size_t j = 0; j < run.size(); ++j) {
            const Pos &q = rc.pos[run[j]];
            if (j + 1 < run.size()) pre += (int32_t)((q.d >> 10) & 7u) + (may_stall(q) ? kCyclesPerLine : 0);
            const uint32_t qc = q.d & 63u;
            if (qc == C_PHA || qc == C_PHP) {
                lo_push = std::min(lo_push, off);
                hi_push = std::max(hi_push, off);
                --off;
            } else if (qc == C_PLA || qc == C_PLP) {
                ++off;
            }
        }
        const Pos &p0 = rc.pos[run[0]];
        std::snprintf(buf, sizeof buf, "c.cyc + %d < lim", pre);
        std::string cond = buf;
        if (hi_push >= lo_push) {  // every push lands in RAM ($80-$FF) without wrapping
            std::snprintf(buf, sizeof buf, " && c.s == W::first(c.s) && (int32_t)c.s + %d >= 0x80 && (int32_t)c.s + %d <= 0xFF",
                          lo_push, hi_push);
            cond += buf;
        }
        if (write_kind(p0) == 2) {
            const char *ix = ((p0.d >> 6) & 15u) == M_ZPX ? "x" : "y";
            std::snprintf(buf, sizeof buf, " && ((0x%02Xu + c.%s) & 0xFFu) == W::first((0x%02Xu + c.%s) & 0xFFu)",
                          p0.lo, ix, p0.lo, ix);
            cond += buf;
        }
        std::snprintf(buf, sizeof buf, "%u|E%u: if (!W::all(%s)) { fb = 1u; break; }\n", run[0] + 1, run[0] + 1,
                      cond.c_str());
        code += buf;
        for (uint32_t i : run) {
            const Pos &p = rc.pos[i];
            std::snprintf(buf, sizeof buf, "        c.pc = 0x%04Xu; exec_static<W, 0x%02Xu>(c, 0x%02Xu, 0x%02Xu);\n",
                          p.pc, p.op, p.lo, p.hi);
            code += buf;
        }
        const Pos &e = rc.pos[run.back()];
        const Flow fe = flow_of(e, im.mapper, t);
        if (f == kJam) {
            std::snprintf(buf, sizeof buf, "        blk = %uu; break;\n", id(last.bank, last.pc));
        } else if (fe == kBranch) {
            const uint32_t me = run[0] + 1, bt = sid(e.bank, t), bf = sid(e.bank, e.pc + 2u);
            if (bt == me || bf == me) {
                // a loop onto itself: while every lane takes it, go straight back to
                // the run's entry check, as long as the pixel-write log has room for
                // another pass (it is drained between dispatches) or no lane draws
                int32_t writes = 0;  // pixel-register writes a pass may log (TIA writes)
                for (uint32_t i : run) {
                    const Pos &q = rc.pos[i];
                    const int wk = write_kind(q);
                    if (wk == 2 || (wk == 1 && q.lo < 0x80u)) ++writes;
                }
                std::snprintf(buf, sizeof buf,
                              "        blk = c.pc == 0x%04Xu ? %uu : %uu;\n"
                              "        if (W::all(blk == %uu) && (W::all(c.hook.frame == nullptr) || "
                              "W::all(c.hook.nlog + %du <= (uint32_t)kLogCap))) goto E%u;\n"
                              "        break;\n",
                              t, bt, bf, me, writes, me);
            } else {
                std::snprintf(buf, sizeof buf, "        blk = c.pc == 0x%04Xu ? %uu : %uu; break;\n", t, bt, bf);
            }
        } else if (fe == kStatic) {
            std::snprintf(buf, sizeof buf, "        blk = %uu; break;\n", sid(e.bank, t));
        } else if (fe == kDynamic) {
            std::snprintf(buf, sizeof buf, "        blk = lookup(tab, c.bank, c.pc); break;\n");
        } else {
            std::snprintf(buf, sizeof buf, "        blk = %uu; break;\n", sid(e.bank, e.pc + ((e.d >> 14) & 3u)));
        }
        code += buf;
        run_code.push_back({entries, code});
    }
    // The most entered runs are tested first, one compare each, ahead of the
    // switch's compare tree (each wrapped so that `break` leaves it).
    constexpr size_t kHotRuns = 4;
    std::vector<size_t> rank(run_code.size());
    for (size_t i = 0; i < rank.size(); ++i) rank[i] = i;
    std::stable_sort(rank.begin(), rank.end(), [&](size_t x, size_t y) { return run_code[x].first > run_code[y].first; });
    std::vector<char> hot(run_code.size(), 0);
    for (size_t k = 0; k < rank.size() && k < kHotRuns; ++k) hot[rank[k]] = 1;
    auto split = [](const std::string &c, std::string &rest) {
        const size_t bar = c.find('|');
        rest = c.substr(bar + 1);
        return c.substr(0, bar);
    };
    for (size_t k = 0; k < rank.size() && k < kHotRuns; ++k) {
        std::string rest;
        const std::string idtxt = split(run_code[rank[k]].second, rest);
        s += k ? "      else if (u == " : "      if (u == ";
        s += idtxt + "u) do {\n        " + rest + "      } while (0);\n";
    }
    s += rank.empty() ? "      {\n" : "      else {\n";
    s += "      switch (u) {\n";
    for (size_t i = 0; i < run_code.size(); ++i) {
        if (hot[i]) continue;
        std::string rest;
        const std::string idtxt = split(run_code[i].second, rest);
        s += "      case " + idtxt + ": " + rest;
    }
    s += "      default: fb = 1u; break;\n      }\n      }\n}\n";
    stats.positions += (int32_t)rc.pos.size();
    stats.runs += (int32_t)runs.size();
    if (rc.truncated) stats.truncated = 1;
}

}  // namespace

std::string translated_source(const uint8_t *roms, const std::vector<int32_t> &rom_off,
                              const std::vector<int32_t> &rom_size, const std::vector<int32_t> &rom_mapper,
                              const std::vector<int32_t> &env_rom, uint64_t seed, int budget, int G, int TPB,
                              TranslateStats &stats) {
    stats = TranslateStats{};
    std::string s;
    s.reserve(1 << 20);
    s += "#include \"vcs_device.hpp\"\n#ifndef VCS_TR_FN\n#define VCS_TR_FN __device__ __forceinline__\n"
         "#define VCS_TR_TABLE __device__ const\n#endif\n#ifndef VCS_TR_ASYNC\n#define VCS_TR_ASYNC true\n#endif\n"
         "namespace vcs {\nnamespace tr {\n";
    {  // the env's pixel-write ring: up to 256 entries (+ a spare slot), about 64 KB of LDS per workgroup
        const int log_cap = tr_log_cap(TPB / G);
        char cbuf[64];
        std::snprintf(cbuf, sizeof cbuf, "constexpr int kLogCap = %d;\n", log_cap);
        s += cbuf;
    }
    const int R = (int)rom_off.size();
    // the position budget is shared out over the images in proportion to
    // their envs' share of the executed instructions
    std::vector<Profile> prof((size_t)R);
    std::vector<double> weight((size_t)R, 0.0);
    double wsum = 0.0;
    for (int r = 0; r < R; ++r) {
        const Image im{roms + rom_off[(size_t)r], rom_size[(size_t)r], rom_mapper[(size_t)r]};
        prof[(size_t)r] = profile(im, seed);
        const double envs = (double)std::count(env_rom.begin(), env_rom.end(), r);
        weight[(size_t)r] = envs * (double)(prof[(size_t)r].count.size() ? 1 : 0);
        wsum += weight[(size_t)r];
    }
    // block lookup: (bank, pc) -> run start id, from the image's table (staged in LDS)
    s += "VCS_TR_FN uint32_t lookup(const uint16_t *tab, uint32_t bank, uint32_t pc) {\n"
         "  if (!((pc & 0x1000u) && (pc & 0xFFFu) <= 0xFFDu)) return 0u;\n"
         "  const uint32_t e = tab[(bank << 12) | (pc & 0xFFFu)];\n"
         "  return (e >> 12) == (pc >> 12) ? (e & 0xFFFu) : 0u;\n}\n";
    std::vector<uint16_t> all_tables;
    std::vector<uint32_t> tab_off, tab_banks;
    for (int r = 0; r < R; ++r) {
        const Image im{roms + rom_off[(size_t)r], rom_size[(size_t)r], rom_mapper[(size_t)r]};
        const int share = wsum > 0 ? (int)((double)budget * weight[(size_t)r] / wsum) : 0;
        const RomCode rc = select_positions(im, prof[(size_t)r], share);
        std::vector<uint16_t> table;
        emit_rom(s, im, r, rc, stats, table);
        tab_off.push_back((uint32_t)all_tables.size());
        tab_banks.push_back((uint32_t)rc.banks);
        all_tables.insert(all_tables.end(), table.begin(), table.end());
    }
    char tbuf[64];
    uint32_t max_banks = 1;
    s += "VCS_TR_TABLE uint16_t kTabAll[] = {";
    for (uint16_t v : all_tables) {
        std::snprintf(tbuf, sizeof tbuf, "%u,", v);
        s += tbuf;
    }
    s += "};\nVCS_TR_TABLE uint32_t kTabOff[] = {";
    for (uint32_t v : tab_off) {
        std::snprintf(tbuf, sizeof tbuf, "%u,", v);
        s += tbuf;
    }
    s += "};\nVCS_TR_TABLE uint32_t kTabBanks[] = {";
    for (uint32_t v : tab_banks) {
        std::snprintf(tbuf, sizeof tbuf, "%u,", v);
        s += tbuf;
        max_banks = std::max(max_banks, v);
    }
    s += "};\n";
    // one instruction loop for all images: a wave runs its image's blocks when
    // its lanes agree on the block and the entry check holds, else the
    // interpreter for one instruction (one copy of it, shared by the images)
    char buf[4096];
    std::snprintf(buf, sizeof buf,
                  "struct Exec {\n  template <typename T, class W> using Hook = RenderHook<T, W, %d, kLogCap, VCS_TR_ASYNC>;\n",
                  G);
    s += buf;
    s += ""
         "  struct State { uint32_t rom, blk; uint4 *log; TrCtl *ctl; const uint16_t *tab; };\n"
         "  template <class C> VCS_TR_FN static void init(C &c, State &s) {\n"
         "    s.blk = lookup(s.tab, c.bank, c.pc);\n"
         "    c.hook.log = s.log;\n"
         "    c.hook.ctl = s.ctl;\n"
         "    c.hook.head = c.hook.nlog = c.hook.pub = 0u;\n"
         "  }\n"
         "  template <class W, bool kPlain, bool kSync = false, class C>\n"
         "  VCS_TR_FN static void run(C &c, State &s, bool go, int32_t lim, const uint32_t *decode) {\n"
         "    uint32_t fb = 0u;\n"
         "    while (go) {\n"
         "      bool interp = true;\n"
         "      for (;;) {  // every lane at one block: translated runs back to back, no per-lane loop control\n"
         "        const uint32_t u = W::first(s.blk);\n"
         "        if (fb != 0u || u == 0u || !W::all(s.blk == u)) break;\n"
         "        switch (s.rom) {\n";
    for (int r = 0; r < R; ++r) {
        std::snprintf(buf, sizeof buf, "          case %d: blocks%d<W>(c, u, s.blk, fb, lim, s.tab); break;\n", r, r);
        s += buf;
    }
    s += "          default: fb = 1u; break;\n"
         "        }\n"
         "        if (fb != 0u) break;\n"
         "        interp = false;\n"
         "        if (!W::all(!c.jam && c.cyc < lim)) break;\n"
         "        if (W::any(c.hook.nlog > (uint32_t)(kLogCap - kTrMaxRun))) break;  // drain the pixel log\n"
         "        interp = true;\n"
         "      }\n"
         "      c.hook.flush(c);\n"
         "      go = !c.jam && c.cyc < lim;\n"
         "      if (go && interp) {  // lanes at different blocks, a failed entry check, or untranslated code\n"
         "        interp_one<W, false>(c, decode);\n"
         "        s.blk = lookup(s.tab, c.bank, c.pc);\n"
         "        c.hook.flush(c);\n"
         "        go = !c.jam && c.cyc < lim;\n"
         "      }\n"
         "      fb = 0u;\n"
         "    }\n"
         "  }\n";
    s += "};\n}  // namespace tr\n}  // namespace vcs\n#ifndef VCS_TR_NO_KERNEL\n";
    // The workgroup: TPB emulating threads (G lanes per env) and as many drawing
    // threads, thread TPB + t drawing the rows of thread t's env.
    std::snprintf(buf, sizeof buf,
                  "extern \"C\" __global__ __launch_bounds__(%d) void vcs_tr_step(vcs::StepParams P) {\n"
                  "  extern __shared__ __align__(16) uint2 rom_lds[];\n"
                  "  __shared__ __align__(16) uint32_t ram_lds[32 * %d];\n"
                  "  __shared__ uint32_t dec_lds[256];\n"
                  "  __shared__ uint4 log_lds[%d * (vcs::tr::kLogCap + 1)];\n"
                  "  __shared__ vcs::TrCtl ctl_lds[%d];\n"
                  "  __shared__ uint16_t tab_lds[%u * 4096];\n"
                  "  const bool drawer = threadIdx.x >= %du;\n"
                  "  const uint32_t t = drawer ? threadIdx.x - %du : threadIdx.x;\n"
                  "  uint4 *log = log_lds + (t / %d) * (vcs::tr::kLogCap + 1);\n"
                  "  vcs::TrCtl *ctl = ctl_lds + t / %d;\n"
                  "  if (!drawer && t %% %d == 0u) *ctl = vcs::TrCtl{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, nullptr};\n"
                  "  {\n"
                  "    const int32_t rom = P.st.main_block_rom[blockIdx.x];\n"
                  "    const uint16_t *src = vcs::tr::kTabAll + vcs::tr::kTabOff[rom];\n"
                  "    for (uint32_t i = threadIdx.x; i < vcs::tr::kTabBanks[rom] * 4096u; i += %d) tab_lds[i] = src[i];\n"
                  "  }\n"
                  "  vcs::stage_group<%d>(P, rom_lds, dec_lds);\n"
                  "  if (drawer) {\n"
                  "    vcs::draw_loop<vcs::DeviceWave, %d, vcs::tr::kLogCap>(ctl, log, P.ystart, t %% %du);\n"
                  "  } else {\n"
                  "    vcs::run_group<%d, %d, false, vcs::tr::Exec, false>(P, rom_lds, ram_lds, dec_lds,\n"
                  "        [log, ctl](int32_t r) { return vcs::tr::Exec::State{(uint32_t)r, 0u, log, ctl, tab_lds}; });\n"
                  "  }\n}\n",
                  2 * TPB, TPB / G, TPB / G, TPB / G, max_banks, TPB, TPB, G, G, G, 2 * TPB, 2 * TPB, G, G, G, TPB);
    s += buf;
    s += "#endif\n";
    return s;
}

namespace {
std::mutex g_cache_mu;
std::map<std::string, std::string> g_code_cache;  // source -> code object
}  // namespace

int32_t jit_compile(const std::string &src, std::string &code, std::string &log, double &seconds, bool &cached) {
    cached = false;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_code_cache.find(src);
        if (it != g_code_cache.end()) {
            code = it->second;
            seconds = 0.0;
            cached = true;
            return VCS_OK;
        }
    }
    const auto t0 = std::chrono::steady_clock::now();
    hiprtcProgram prog;
    const int nh = (int)(sizeof(kJitHeaderNames) / sizeof(kJitHeaderNames[0]));
    if (hiprtcCreateProgram(&prog, src.c_str(), "vcs_translated.hip", nh, kJitHeaderText, kJitHeaderNames) !=
        HIPRTC_SUCCESS) {
        log = "hiprtcCreateProgram failed";
        return VCS_HIP_ERROR;
    }
    // gfx950 only; packed-FP32 selection off and uniform regions left
    // unstructurised, as for the precompiled kernels
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Wno-implicit-fallthrough",
                          "-mllvm", "-structurizecfg-skip-uniform-regions=true",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    log.assign(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &log[0]);
    if (rc != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        return VCS_HIP_ERROR;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code.assign(cs, '\0');
    hiprtcGetCode(prog, &code[0]);
    hiprtcDestroyProgram(&prog);
    seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_code_cache[src] = code;
    return VCS_OK;
}

}  // namespace vcs
