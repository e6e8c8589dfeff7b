"""The ROM translator on the CPU: the generated code, built for the host, against the oracle."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import binding as Bd
from paper_2606_22447_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2606_22447_amd", "csrc")


def _ctx(w, G=1, tpb=64):
    return Bd.create([r.size for r in w.roms], [r.mapper for r in w.roms], w.env_rom, w.frame_skip, 34, w.seed, 0,
                     Bd.VCS_KERNEL_TRANSLATED, G, tpb)


def _hetero():
    roms = [I.generate_rom(100 + i, sz, reads_inputs=True, timer_vblank=True)
            for i, sz in enumerate([2048, 4096, 8192, 8192])]
    B, S = 8, 8
    env_rom = (np.arange(B) % 4).astype(np.int32)
    eps = (1 + (np.arange(B)[:, None] * 3 + np.arange(5)[None, :]) % 4).astype(np.uint32)
    return I.Workload("hetero", roms, env_rom, I.initial_ram(9, B), I.action_stream(9, B, S), S, 4,
                      episode_steps=eps, seed=4242)


def test_translated_source_is_basic_blocks_of_page0_forms():
    w = I.config_c1(num_envs=16, steps=2)
    h = _ctx(w, 16, 256)
    src = Bd.translated_source(h, np.concatenate([r.image for r in w.roms]))
    import re
    assert "vcs_tr_step" in src and "exec_static" in src
    loop = src[src.index("void blocks0("):src.index("struct Exec")]
    cases = re.findall(r"^      case \d+: (.*)$", loop, re.M) + re.findall(r"^      (?:else )?if \(u == \d+u\) do \{\n\s+(.*)$", loop, re.M)
    assert 10 < len(cases) < 100  # runs, each one case
    assert src.count("exec_static<W, 0x") > 100  # positions
    # every run is entered through one wave-wide check (or is a lone jam)
    assert all(re.match(r"(E\d+: )?if \(!W::all\(c\.cyc \+ ", c) or c.startswith("c.jam = 1") for c in cases)
    # only page-0 forms are translated (no absolute / indexed-absolute / indirect opcodes)
    dec = Bd.decode_table()
    for op in {int(x, 16) for x in __import__("re").findall(r"exec_static<W, 0x([0-9A-F]{2})u>", src)}:
        mode = (int(dec[op]) >> 6) & 15
        assert mode in (0, 1, 2, 3, 4, 5, 12) or op == 0x4C, hex(op)


def tia_pushes_workload(B: int = 3, S: int = 3) -> I.Workload:
    """A program whose JSRs push onto CTRLPF and COLUBK (stack pointer $0A): two
    pixel-register writes at the same clock.  The two call sites push different
    return addresses, so COLUBK changes at every call, and the 45-cycle loop
    drifts through every pixel alignment of the writes."""
    from tests import asm as A

    def body(b):
        b.ins("LDX", "imm", 0x0A)
        b.ins("TXS")
        for reg, v in ((A.PF0, 0xF0), (A.PF1, 0xAA), (A.PF2, 0x55)):
            b.ins("LDA", "imm", v)
            b.ins("STA", "zp", reg)
        b.label("LOOP")
        b.ins("INC", "zp", 0x80)
        b.ins("LDA", "zp", 0x80)
        b.ins("STA", "zp", A.COLUPF)
        b.ins("INC", "zp", 0x81)
        b.ins("JSR", "abs", "SUBA")
        b.label("BACKA")
        b.ins("JSR", "abs", "SUBB")
        b.label("BACKB")
        b.ins("JMP", "abs", "LOOP")
        for name, back in (("SUBA", "BACKA"), ("SUBB", "BACKB")):
            b.label(name)
            b.ins("LDX", "imm", 0x0A)
            b.ins("TXS")
            b.ins("JMP", "abs", back)

    img = A.program(body)
    return I.Workload("tia_pushes", [I.Rom(0, 4096, 1, img)], np.zeros(B, np.int32), I.initial_ram(21, B),
                      np.zeros((B, S), np.uint8), S, 2, seed=7)


def playfield_modes_workload(B: int = 3, S: int = 3) -> I.Workload:
    """A program that cycles CTRLPF through plain, reflected, score and score +
    reflected playfields in a loop that drifts across the line, with COLUP0,
    COLUP1, COLUPF and COLUBK all different and changing: every owner of a
    playfield group shows up on both halves of the screen."""
    from tests import asm as A

    def body(b):
        for reg, v in ((A.PF0, 0xA0), (A.PF1, 0x96), (A.PF2, 0x3C), (A.COLUP0, 0x44), (A.COLUP1, 0x88),
                       (A.COLUPF, 0xCC), (A.COLUBK, 0x22)):
            b.ins("LDA", "imm", v)
            b.ins("STA", "zp", reg)
        b.label("LOOP")
        for mode in (0x00, 0x01, 0x02, 0x03):
            b.ins("LDA", "imm", mode)
            b.ins("STA", "zp", A.CTRLPF)
            b.ins("INC", "zp", 0x80)
        b.ins("LDA", "zp", 0x80)
        b.ins("STA", "zp", A.COLUP1)
        b.ins("JMP", "abs", "LOOP")

    img = A.program(body)
    return I.Workload("playfield_modes", [I.Rom(0, 4096, 1, img)], np.zeros(B, np.int32), I.initial_ram(22, B),
                      np.zeros((B, S), np.uint8), S, 2, seed=8)


@pytest.mark.parametrize("name", ["c1", "hetero", "tia_pushes", "playfield_modes", "sweep", "sweep_objects", "objects"])
def test_translated_code_on_the_host_matches_the_oracle(name, tmp_path):
    w = {"c1": lambda: I.config_c1(num_envs=6, steps=6), "hetero": _hetero, "tia_pushes": tia_pushes_workload,
         "playfield_modes": playfield_modes_workload,
         "sweep": lambda: I.config_sweep(envs_per_rom=2, steps=3, frame_skip=2, objects=False),
         "sweep_objects": lambda: I.config_sweep(envs_per_rom=2, steps=3, frame_skip=2),
         "objects": lambda: I.config_objects(envs_per_rom=1, steps=3, n_roms=6, frame_skip=2)}[name]()
    h = _ctx(w)
    src = Bd.translated_source(h, np.concatenate([r.image for r in w.roms]))
    gen = tmp_path / "translated.hip"
    gen.write_text(src)
    so = tmp_path / "libhost_translated.so"
    subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared",
                           "-Wno-implicit-fallthrough", "-w", f'-DTR_SOURCE="{gen}"', "-I", CSRC,
                           os.path.join(HERE, "host_translated.hip"), "-o", str(so)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    H = C.CDLL(str(so))
    ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)  # noqa: E731
    flagged = 0
    for b in range(w.num_envs):
        ri = int(w.env_rom[b])
        rom = w.roms[ri]
        acts = np.zeros((b + 1, w.steps), np.uint8)
        acts[b] = w.actions[b]
        ep = None
        if w.episode_steps is not None:
            ep = np.zeros((b + 1, w.episode_steps.shape[1]), np.uint32)
            ep[b] = w.episode_steps[b]
        ref = O.run_env(rom.image, rom.mapper, w.ram0[b], w.actions[b], w.steps, w.frame_skip,
                        ep_steps=None if ep is None else ep[b], seed=w.seed, env_index=b)
        n = (b + 1) * w.steps
        ram = np.zeros((n, 128), np.uint8)
        fr = np.zeros((n, 210, 160), np.uint8)
        dn = np.zeros(n, np.uint8)
        flag = np.full(b + 1, 7, np.uint8)
        rc = H.host_translated(ri, ptr(np.ascontiguousarray(rom.image)), rom.size, rom.mapper,
                               ptr(np.ascontiguousarray(w.ram0[b])), ptr(acts), w.steps, w.frame_skip, ptr(ep),
                               0 if ep is None else ep.shape[1], C.c_ulonglong(w.seed), b, ptr(ram), ptr(fr),
                               ptr(dn), ptr(flag))
        assert rc == 0, (name, b, {-1: "a frame left undrawn", -2: "a wait for the drawing gave up"}.get(rc, rc))
        if name == "objects":  # sprite kernels show objects: the library reruns them with the object paths
            assert flag[b] == 1, b
            continue
        if name == "sweep_objects" and flag[b]:  # reads a collision latch or writes an object register
            assert flag[b] == 1, b
            flagged += 1
            continue
        assert flag[b] == 0, (name, b)
        sl = slice(b * w.steps, None)
        assert (ram[sl] == ref["ram"]).all(), (name, b)
        assert (fr[sl] == ref["frames"]).all(), (name, b)
        assert (dn[sl] == ref["done"]).all(), (name, b)
    if name == "sweep_objects":
        assert 0 < flagged, "the full sweep touches the object registers"


def test_translate_compiles_for_gfx950_without_a_gpu():
    w = I.config_c1(num_envs=8, steps=2)
    info = Bd.translate(_ctx(w, 16, 256), np.concatenate([r.image for r in w.roms]), compile_only=True)
    assert info["positions"] > 100 and info["code_bytes"] > 10000 and not info["truncated"]


def test_translate_rejects_other_kernels():
    w = I.config_c1(num_envs=8, steps=2)
    h = Bd.create([r.size for r in w.roms], [r.mapper for r in w.roms], w.env_rom, 4, 34, 0, 0,
                  Bd.VCS_KERNEL_GROUPED, 16, 256)
    with pytest.raises(Bd.VcsError):
        Bd.translate(h, np.concatenate([r.image for r in w.roms]), compile_only=True)


def test_translate_arguments_and_budget():
    w = I.config_c1(num_envs=8, steps=2)
    h = _ctx(w, 16, 256)
    roms = np.concatenate([r.image for r in w.roms])
    with pytest.raises(Bd.VcsError):
        Bd.translate(h, roms, compile_only=True, max_positions=-1)
    with pytest.raises(Bd.VcsError):
        Bd.translate(h, roms, compile_only=True, max_positions=70000)
    src = Bd.translated_source(h, roms, max_positions=10)
    assert src.count("exec_static<W, 0x") <= 10
    # the translated kernel keeps at most 64 envs per workgroup (the pixel logs live in LDS)
    with pytest.raises(Bd.VcsError):
        Bd.create([r.size for r in w.roms], [r.mapper for r in w.roms], w.env_rom, 4, 34, 0, 0,
                  Bd.VCS_KERNEL_TRANSLATED, 1, 256)
    assert Bd.translate(_ctx(w, 4, 256), roms, compile_only=True)["positions"] > 100
