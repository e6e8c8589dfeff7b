"""ctypes binding of libvcs (the C-ABI declared in ``include/vcs.h``).

Argument marshalling only: every step of the emulation runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvcs.so")

VCS_OK = 0
(VCS_MAPPER_2K, VCS_MAPPER_4K, VCS_MAPPER_F8, VCS_MAPPER_F6, VCS_MAPPER_F4, VCS_MAPPER_F8SC, VCS_MAPPER_F6SC,
 VCS_MAPPER_F4SC, VCS_MAPPER_E0) = range(9)
ACTION_RESET = 18  # the console RESET switch held (hard steps)
VCS_KERNEL_AUTO, VCS_KERNEL_PLAIN, VCS_KERNEL_GROUPED, VCS_KERNEL_TRANSLATED = 0, 1, 2, 3
VCS_TRANSLATE_COMPILE_ONLY = 1
VCS_FRAMES_NONE, VCS_FRAMES_LAST, VCS_FRAMES_ALL = 0, 1, 2
VCS_OP_HARD, VCS_OP_SOFT_FWD, VCS_OP_SOFT_BWD = 0, 1, 2
ABI_VERSION = 4
STATE_BYTES = 256

EXPORTED = [
    "vcs_create", "vcs_destroy", "vcs_status_string", "vcs_state_bytes", "vcs_rom_bytes",
    "vcs_workspace_bytes", "vcs_residual_bytes", "vcs_decode_bytes", "vcs_reset", "vcs_step_hard",
    "vcs_step_soft_fwd", "vcs_step_soft_bwd", "vcs_read_regs", "vcs_read_objects", "vcs_residual_checkpoints",
    "vcs_bwd_overflow", "vcs_launch_info", "vcs_decode_table", "vcs_hash", "vcs_translate",
    "vcs_translated_source", "vcs_step_hard_static", "vcs_bwd_overflow_offset", "vcs_step_relaxed",
    "vcs_detect_mapper",
]


class VcsTranslateInfo(C.Structure):
    _fields_ = [
        ("positions", C.c_int32), ("runs", C.c_int32), ("truncated", C.c_int32), ("cached", C.c_int32),
        ("compile_seconds", C.c_double), ("source_bytes", C.c_size_t), ("code_bytes", C.c_size_t),
    ]


class VcsConfig(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("num_envs", C.c_int32), ("num_roms", C.c_int32),
        ("rom_size", C.POINTER(C.c_int32)), ("rom_mapper", C.POINTER(C.c_int32)),
        ("env_rom", C.POINTER(C.c_int32)), ("frame_skip", C.c_int32), ("ystart", C.c_int32),
        ("seed", C.c_uint64), ("ckpt_interval", C.c_int32), ("kernel", C.c_int32),
        ("lanes_per_env", C.c_int32), ("block_threads", C.c_int32), ("tape_records", C.c_int32),
    ]


class VcsError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libvcs.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise VcsError(f"{LIB_PATH} is not built; run `python -m paper_2606_22447_amd.build` "
                           "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32, u64, sz = C.c_void_p, C.c_int32, C.c_uint64, C.c_size_t
        f32 = C.c_float
        L.vcs_create.argtypes = [C.POINTER(VcsConfig), C.POINTER(vp)]
        L.vcs_destroy.argtypes = [vp]
        L.vcs_destroy.restype = None
        L.vcs_status_string.argtypes = [i32]
        L.vcs_status_string.restype = C.c_char_p
        for f in ("vcs_state_bytes", "vcs_rom_bytes"):
            getattr(L, f).argtypes = [vp, C.POINTER(sz)]
        L.vcs_workspace_bytes.argtypes = [vp, i32, i32, C.POINTER(sz)]
        L.vcs_residual_bytes.argtypes = [vp, i32, C.POINTER(sz)]
        L.vcs_decode_bytes.argtypes = [vp, i32, C.POINTER(sz)]
        L.vcs_residual_checkpoints.argtypes = [vp, i32, C.POINTER(i32)]
        L.vcs_reset.argtypes = [vp, vp, vp, vp, vp]
        L.vcs_step_hard.argtypes = [vp, vp, vp, vp, i32, vp, i32, vp, vp, vp, i32, vp, vp]
        L.vcs_step_hard_static.argtypes = [vp, vp, vp, vp, i32, vp, i32, vp, vp, vp, i32, vp]
        L.vcs_step_relaxed.argtypes = [vp, vp, vp, vp, i32, vp, i32, vp, C.c_double, C.c_double, vp, vp, vp]
        L.vcs_step_soft_fwd.argtypes = [vp, vp, vp, vp, vp, f32, f32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.vcs_step_soft_bwd.argtypes = [vp, vp, vp, vp, vp, f32, f32, f32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.vcs_read_regs.argtypes = [vp, vp, vp, vp]
        L.vcs_read_objects.argtypes = [vp, vp, vp, vp]
        L.vcs_bwd_overflow.argtypes = [vp, vp, i32, vp, C.POINTER(i32)]
        L.vcs_bwd_overflow_offset.argtypes = [vp, i32, C.POINTER(sz)]
        L.vcs_launch_info.argtypes = [vp] + [C.POINTER(i32)] * 5
        L.vcs_decode_table.argtypes = [C.POINTER(C.c_uint32)]
        L.vcs_detect_mapper.argtypes = [vp, sz, C.POINTER(i32)]
        L.vcs_translate.argtypes = [vp, vp, i32, i32, C.POINTER(VcsTranslateInfo), C.c_char_p, sz]
        L.vcs_translated_source.argtypes = [vp, vp, i32, C.c_char_p, sz, C.POINTER(sz)]
        for f in EXPORTED:
            fn = getattr(L, f)
            if f not in ("vcs_destroy", "vcs_status_string"):
                fn.restype = i32
        del u64
        _lib = L
    return _lib


def check(rc: int, what: str):
    if rc != VCS_OK:
        msg = lib().vcs_status_string(rc).decode()
        raise VcsError(f"{what} failed: {msg} ({rc})")


def ptr(t):
    """Device (or host) address of a tensor/array, or None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return C.c_void_p(t.data_ptr())
    return t.ctypes.data_as(C.c_void_p)


def detect_mapper(image) -> int:
    """vcs_detect_mapper on a host image (uint8 array)."""
    import numpy as np
    img = np.ascontiguousarray(image, np.uint8)
    out = C.c_int32()
    check(lib().vcs_detect_mapper(img.ctypes.data, img.size, C.byref(out)), "vcs_detect_mapper")
    return out.value


def decode_table():
    out = (C.c_uint32 * 256)()
    check(lib().vcs_decode_table(out), "vcs_decode_table")
    return list(out)


def create(rom_sizes, rom_mappers, env_rom, frame_skip=4, ystart=34, seed=0, ckpt_interval=0,
           kernel=VCS_KERNEL_AUTO, lanes_per_env=0, block_threads=0, tape_records=0):
    R, B = len(rom_sizes), len(env_rom)
    sizes = (C.c_int32 * R)(*[int(v) for v in rom_sizes])
    maps = (C.c_int32 * R)(*[int(v) for v in rom_mappers])
    envr = (C.c_int32 * B)(*[int(v) for v in env_rom])
    cfg = VcsConfig(ABI_VERSION, B, R, sizes, maps, envr, frame_skip, ystart, seed, ckpt_interval, kernel,
                    lanes_per_env, block_threads, tape_records)
    h = C.c_void_p()
    check(lib().vcs_create(C.byref(cfg), C.byref(h)), "vcs_create")
    return h


def size_query(fn, *args) -> int:
    out = C.c_size_t()
    check(getattr(lib(), fn)(*args, C.byref(out)), fn)
    return out.value


def launch_info(h):
    vals = [C.c_int32() for _ in range(5)]
    check(lib().vcs_launch_info(h, *[C.byref(v) for v in vals]), "vcs_launch_info")
    return dict(zip(["kernel", "lanes_per_env", "block_threads", "blocks", "bwd_blocks"], [v.value for v in vals]))


def translate(h, roms: "np.ndarray", compile_only: bool = False, max_positions: int = 0) -> dict:
    """vcs_translate on the host image bytes (uint8, concatenated); returns its info."""
    import numpy as np
    roms = np.ascontiguousarray(roms, np.uint8)
    info = VcsTranslateInfo()
    log = C.create_string_buffer(1 << 16)
    rc = lib().vcs_translate(h, roms.ctypes.data, int(max_positions), VCS_TRANSLATE_COMPILE_ONLY if compile_only else 0,
                             C.byref(info), log, len(log))
    if rc != VCS_OK:
        raise VcsError(f"vcs_translate: {lib().vcs_status_string(rc).decode()}\n{log.value.decode(errors='replace')}")
    return {k: getattr(info, k) for k, _ in VcsTranslateInfo._fields_}


def translated_source(h, roms: "np.ndarray", max_positions: int = 0) -> str:
    import numpy as np
    roms = np.ascontiguousarray(roms, np.uint8)
    n = C.c_size_t(0)
    check(lib().vcs_translated_source(h, roms.ctypes.data, int(max_positions), None, 0, C.byref(n)),
          "vcs_translated_source")
    buf = C.create_string_buffer(n.value + 1)
    check(lib().vcs_translated_source(h, roms.ctypes.data, int(max_positions), buf, len(buf), C.byref(n)),
          "vcs_translated_source")
    return buf.value.decode()
