"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
validates arguments on the host, and its opcode decode agrees with the oracle's
independently written table (no GPU compute is launched here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_22447_amd import binding as Bd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    hdr = open(os.path.join(ROOT, "include", "vcs.h")).read()
    return sorted(set(re.findall(r"^(?:int32_t|void|const char \*)\s*\*?\s*(vcs_\w+)\(", hdr, re.M)))


def test_library_exports_every_declared_symbol():
    L = Bd.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(Bd.EXPORTED) == names


def test_decode_table_agrees_with_oracle():
    t = Bd.decode_table()
    # oracle op ids differ from the library's class ids; compare timing, length and the jam set
    mode_len = {0: 1, 1: 1, 2: 2, 3: 2, 4: 2, 5: 2, 6: 3, 7: 3, 8: 3, 9: 2, 10: 2, 11: 3, 12: 2}
    for op in range(256):
        ok, oop, omode, ocyc, open_ = O.opcode_info(op)
        e = t[op]
        assert (e != 0) == ok, hex(op)
        if not ok:
            continue
        assert (e >> 6) & 15 == omode, hex(op)          # both number the modes IMP..REL alike
        assert (e >> 10) & 7 == ocyc, hex(op)
        assert (e >> 13) & 1 == open_, hex(op)
        assert (e >> 14) & 3 == mode_len[omode], hex(op)


def test_create_validates_arguments():
    with pytest.raises(Bd.VcsError):
        Bd.create([4096], [0], [0])          # 4K image with the 2K mapper
    with pytest.raises(Bd.VcsError):
        Bd.create([2048], [0], [1])          # env uses a ROM that does not exist
    with pytest.raises(Bd.VcsError):
        Bd.create([2048], [0], [0], frame_skip=0)
    with pytest.raises(Bd.VcsError):
        Bd.create([2048], [0], [0], lanes_per_env=3)
    h = Bd.create([2048, 8192], [0, 2], [1, 0, 1], lanes_per_env=4, block_threads=64)
    info = Bd.launch_info(h)
    assert info["lanes_per_env"] == 4 and info["block_threads"] == 64 and info["blocks"] == 2
    assert Bd.size_query("vcs_state_bytes", h) == 3 * 256
    assert Bd.size_query("vcs_rom_bytes", h) == 2048 + 8192
    assert Bd.size_query("vcs_workspace_bytes", h, Bd.VCS_OP_SOFT_BWD, 2) > Bd.size_query(
        "vcs_workspace_bytes", h, Bd.VCS_OP_HARD, 2)
    # step calls reject NULL / misaligned buffers before touching the GPU
    L = Bd.lib()
    rc = L.vcs_step_hard(h, None, None, None, 1, None, 0, None, None, None, 0, None, None)
    assert rc == -1
    rc = L.vcs_step_hard(h, C.c_void_p(16), C.c_void_p(32), None, 1, None, 2, None, None, None, 0, C.c_void_p(64),
                         None)
    assert rc == -1  # frames requested without a frame buffer
    rc = L.vcs_step_soft_fwd(h, None, C.c_void_p(16), C.c_void_p(32), C.c_void_p(48), C.c_float(0.0), C.c_float(6.0), 1,
                             None, None, None, None, None, C.c_void_p(64), C.c_void_p(80), None)
    assert rc == -1  # tau must be > 0
    rc = L.vcs_step_soft_fwd(h, None, C.c_void_p(16), C.c_void_p(32), C.c_void_p(48), C.c_float(1.0), C.c_float(6.0), 1,
                             None, None, C.c_void_p(96), None, None, C.c_void_p(64), C.c_void_p(80), None)
    assert rc == -1  # sampler tangents need the frame they belong to
    assert L.vcs_status_string(-3).decode() == "workspace too small"
    L.vcs_destroy(h)
    np.testing.assert_equal(Bd.ABI_VERSION, 4)
    # the forward's tape: -1 sizes it for every segment before the final frame
    with pytest.raises(Bd.VcsError):
        Bd.create([2048], [0], [0], tape_records=-2)
    h0 = Bd.create([2048], [0], [0, 0], frame_skip=2)
    h1 = Bd.create([2048], [0], [0, 0], frame_skip=2, tape_records=-1)
    h2 = Bd.create([2048], [0], [0, 0], frame_skip=2, tape_records=1000)
    r0, r1, r2 = (Bd.size_query("vcs_residual_bytes", h, 3) for h in (h0, h1, h2))
    assert r1 - r0 >= 2 * ((3 * 2 - 1) * 9956 + 3 + 16) * 16 and r2 - r0 >= 2 * 1000 * 16
    h3 = Bd.create([2048], [0], [0, 0], frame_skip=2, tape_records=-1)
    with pytest.raises(Bd.VcsError):  # more records per env than an int32 counts
        Bd.size_query("vcs_residual_bytes", h3, 1 << 20)
    for h in (h0, h1, h2, h3):
        L.vcs_destroy(h)


def test_autotune_candidates_are_valid_launch_shapes():
    from paper_2606_22447_amd import autotune
    for B in (1, 64, 4096, 16384, 1 << 20):
        c = autotune.hard_candidates(B)
        assert c, B
        for g, t in c:
            assert g in (1, 4, 16, 64) and (t in (64, 256) or (g, t) == (64, 1024)) and t >= g
            waves = B * g / 64
            assert waves <= 1024 * 8 or (g, t) == (1, 64)


def test_fnv1a64_matches_the_published_test_vectors():
    # FNV-1a 64 reference values published with the algorithm: "" , "a", "foobar"
    from tests.fnv import fnv1a64
    assert int(fnv1a64(np.zeros((1, 0), np.uint8))[0]) == 0xCBF29CE484222325
    assert int(fnv1a64(np.frombuffer(b"a", np.uint8)[None])[0]) == 0xAF63DC4C8601EC8C
    assert int(fnv1a64(np.frombuffer(b"foobar", np.uint8)[None])[0]) == 0x85944171F73967E8
