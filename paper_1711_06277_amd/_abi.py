"""ctypes binding of ``libart.so`` (the C ABI of include/art.h), same names.

Argument marshalling only: every step of the sweep runs in the HIP library.
Loading fails loudly when the library has not been built (there is no CPU
fallback).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libart.so")

ART_OK = 0
ART_ERR_INVALID_ARG = -1
ART_ERR_HIP = -2
ART_ERR_OUT_OF_MEMORY = -3
ART_ERR_QUEUE_OVERFLOW = -4
ART_ERR_SOURCE_OUTSIDE = -5
ART_ERR_DESTROY_COUNT = -6
ART_ERR_NO_FORWARD = -7
ART_ERR_BAD_FIELD = -8
ART_ERR_NO_ADJOINT = -9
ART_ERR_TOO_LARGE = -10
ART_NOALLOC_SCRATCH_MIB = 64
ART_DEPOSIT_ATOMIC = 0
ART_DEPOSIT_DETERMINISTIC = 1
ART_MAX_LEVELS = 16
ART_MAX_BINS = 2

# every symbol declared in include/art.h
EXPORTED = ("art_create", "art_set_stream", "art_trace", "art_get_tape", "art_trace_adjoint",
            "art_trace_adjoint_tape", "art_trace_and_adjoint", "art_sync",
            "art_get_stats", "art_autotune", "art_autotune_adjoint", "art_set_launch",
            "art_set_adjoint_launch", "art_set_wave_sources", "art_set_timing", "art_get_timing",
            "art_set_transparent", "art_set_rotation", "art_random_rotation", "art_get_rotation",
            "art_ion_substep", "art_ion_subcycle", "art_destroy", "art_strerror", "art_trace_noalloc")


class art_params(C.Structure):
    _fields_ = [("level0", C.c_int), ("level_max", C.c_int), ("phi_c", C.c_double),
                ("tau_term", C.c_double), ("s_H", C.c_double), ("s_d", C.c_double),
                ("n_bins", C.c_int), ("rot", C.c_double * 9), ("deposit_mode", C.c_int)]


class art_options(C.Structure):
    _fields_ = [("max_sources", C.c_int), ("enable_adjoint", C.c_int),
                ("pool_rays", C.c_int64), ("pool_mem_fraction", C.c_double),
                ("block_size", C.c_int), ("blocks_per_cu", C.c_int)]


class art_ion_params(C.Structure):
    _fields_ = [("alpha_B", C.c_double), ("gamma_scale", C.c_double), ("C", C.c_double)]


class art_stats(C.Structure):
    _fields_ = [("status", C.c_int), ("n_src", C.c_int), ("n_waves", C.c_int),
                ("segments", C.c_uint64), ("destroy", C.c_uint64),
                ("destroy_expected", C.c_uint64), ("rays_max_wave", C.c_uint64),
                ("created", C.c_uint64 * ART_MAX_LEVELS), ("split", C.c_uint64 * ART_MAX_LEVELS),
                ("exited", C.c_uint64 * ART_MAX_LEVELS),
                ("terminated", C.c_uint64 * ART_MAX_LEVELS)]


class ArtError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


_lib = None


def lib() -> C.CDLL:
    """Load libart.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1711_06277_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.art_create.argtypes = [C.POINTER(vp), C.c_int, C.c_int, C.c_int, C.POINTER(art_params),
                                 C.POINTER(art_options), vp]
        L.art_set_stream.argtypes = [vp, vp]
        L.art_trace.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp, vp, vp]
        L.art_get_tape.argtypes = [vp, C.POINTER(C.c_uint64)]
        L.art_trace_adjoint.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp, vp, vp, vp]
        L.art_trace_adjoint_tape.argtypes = [vp, C.c_uint64, vp, vp, vp, vp, C.c_int, vp, vp, vp, vp]
        L.art_trace_and_adjoint.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp, vp, vp, vp, vp, vp, vp]
        L.art_sync.argtypes = [vp]
        L.art_get_stats.argtypes = [vp, C.POINTER(art_stats), C.c_int, vp, vp, vp, vp, vp, vp, vp, vp]
        L.art_autotune.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp, vp, C.POINTER(C.c_int),
                                   C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_float)]
        L.art_autotune_adjoint.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp, vp, vp, vp, vp, vp,
                                           C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_float)]
        L.art_set_launch.argtypes = [vp, C.c_int, C.c_int]
        L.art_set_adjoint_launch.argtypes = [vp, C.c_int, C.c_int]
        L.art_set_wave_sources.argtypes = [vp, C.c_int]
        L.art_set_timing.argtypes = [vp, C.c_int]
        L.art_get_timing.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_int),
                                     C.POINTER(C.c_float)]
        L.art_set_transparent.argtypes = [vp, vp]
        L.art_set_rotation.argtypes = [vp, C.POINTER(C.c_double)]
        L.art_random_rotation.argtypes = [vp, vp]
        L.art_get_rotation.argtypes = [vp, C.POINTER(C.c_double)]
        L.art_ion_substep.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.POINTER(art_ion_params),
                                      C.c_double, vp, vp, vp, vp, vp]
        L.art_ion_subcycle.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.POINTER(art_ion_params),
                                       C.c_double, C.c_int, vp, vp, vp, vp, C.POINTER(C.c_int),
                                       C.POINTER(C.c_double)]
        L.art_trace_noalloc.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(art_params), vp, vp, vp, vp,
                                        C.c_int, vp, vp, vp, vp, vp]
        L.art_destroy.argtypes = [vp]
        L.art_destroy.restype = None
        L.art_strerror.argtypes = [C.c_int]
        L.art_strerror.restype = C.c_char_p
        for name in EXPORTED:
            if name not in ("art_destroy", "art_strerror"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().art_strerror(int(code)).decode()
    except ImportError:
        return f"error {code}"


def check(code: int, where: str) -> None:
    if code != ART_OK:
        raise ArtError(code, where)


def art_create(nx, ny, nz, params: art_params, opts: art_options, stream: int) -> int:
    h = C.c_void_p()
    check(lib().art_create(C.byref(h), nx, ny, nz, C.byref(params), C.byref(opts),
                           C.c_void_p(stream)), "art_create")
    return h.value


def art_set_stream(ctx, stream):
    check(lib().art_set_stream(C.c_void_p(ctx), C.c_void_p(stream)), "art_set_stream")


def art_trace(ctx, n_H, x_n, src_pos, src_lum, n_src, rate, force, J):
    check(lib().art_trace(C.c_void_p(ctx), n_H, x_n, src_pos, src_lum, int(n_src), rate, force, J),
          "art_trace")


def art_trace_adjoint(ctx, n_H, x_n, src_pos, src_lum, n_src, g_rate, g_force, g_nH, g_xn):
    check(lib().art_trace_adjoint(C.c_void_p(ctx), n_H, x_n, src_pos, src_lum, int(n_src),
                                  g_rate, g_force, g_nH, g_xn), "art_trace_adjoint")


def art_get_tape(ctx) -> int:
    t = C.c_uint64()
    check(lib().art_get_tape(C.c_void_p(ctx), C.byref(t)), "art_get_tape")
    return t.value


def art_trace_adjoint_tape(ctx, tape, n_H, x_n, src_pos, src_lum, n_src, g_rate, g_force, g_nH, g_xn):
    check(lib().art_trace_adjoint_tape(C.c_void_p(ctx), C.c_uint64(int(tape)), n_H, x_n, src_pos, src_lum,
                                       int(n_src), g_rate, g_force, g_nH, g_xn), "art_trace_adjoint_tape")


def art_trace_and_adjoint(ctx, n_H, x_n, src_pos, src_lum, n_src, rate, force, J, g_rate, g_force,
                          g_nH, g_xn):
    check(lib().art_trace_and_adjoint(C.c_void_p(ctx), n_H, x_n, src_pos, src_lum, int(n_src), rate, force,
                                      J, g_rate, g_force, g_nH, g_xn), "art_trace_and_adjoint")


def art_sync(ctx) -> int:
    return lib().art_sync(C.c_void_p(ctx))


def art_get_stats(ctx, n_src_stats, created, split, exited, terminated, escaped, residual,
                  segments, rays_bound=None) -> art_stats:
    st = art_stats()
    check(lib().art_get_stats(C.c_void_p(ctx), C.byref(st), int(n_src_stats), created, split,
                              exited, terminated, escaped, residual, segments, rays_bound), "art_get_stats")
    return st


def art_autotune(ctx, n_H, x_n, src_pos, src_lum, n_src, rate, force):
    bb, bp, bw, ms = C.c_int(), C.c_int(), C.c_int(), C.c_float()
    check(lib().art_autotune(C.c_void_p(ctx), n_H, x_n, src_pos, src_lum, int(n_src), rate, force,
                             C.byref(bb), C.byref(bp), C.byref(bw), C.byref(ms)), "art_autotune")
    return bb.value, bp.value, bw.value, ms.value


def art_autotune_adjoint(ctx, n_H, x_n, src_pos, src_lum, n_src, rate, force, g_rate, g_force, g_nH, g_xn):
    bb, bp, ms = C.c_int(), C.c_int(), C.c_float()
    check(lib().art_autotune_adjoint(C.c_void_p(ctx), n_H, x_n, src_pos, src_lum, int(n_src), rate, force,
                                     g_rate, g_force, g_nH, g_xn, C.byref(bb), C.byref(bp), C.byref(ms)),
          "art_autotune_adjoint")
    return bb.value, bp.value, ms.value


def art_set_launch(ctx, block_size: int, blocks_per_cu: int):
    check(lib().art_set_launch(C.c_void_p(ctx), int(block_size), int(blocks_per_cu)), "art_set_launch")


def art_set_adjoint_launch(ctx, block_size: int, blocks_per_cu: int):
    check(lib().art_set_adjoint_launch(C.c_void_p(ctx), int(block_size), int(blocks_per_cu)),
          "art_set_adjoint_launch")


def art_set_wave_sources(ctx, n: int):
    check(lib().art_set_wave_sources(C.c_void_p(ctx), int(n)), "art_set_wave_sources")


def art_set_timing(ctx, enable: bool):
    check(lib().art_set_timing(C.c_void_p(ctx), 1 if enable else 0), "art_set_timing")


def art_get_timing(ctx):
    s, n, t = C.c_float(), C.c_int(), C.c_float()
    check(lib().art_get_timing(C.c_void_p(ctx), C.byref(s), C.byref(n), C.byref(t)),
          "art_get_timing")
    return s.value, n.value, t.value


def art_set_transparent(ctx, mask):
    check(lib().art_set_transparent(C.c_void_p(ctx), mask), "art_set_transparent")


def art_set_rotation(ctx, rot):
    r = (C.c_double * 9)(*[float(x) for x in rot])
    check(lib().art_set_rotation(C.c_void_p(ctx), r), "art_set_rotation")


def art_random_rotation(ctx, u):
    check(lib().art_random_rotation(C.c_void_p(ctx), u), "art_random_rotation")


def art_get_rotation(ctx):
    r = (C.c_double * 9)()
    check(lib().art_get_rotation(C.c_void_p(ctx), r), "art_get_rotation")
    return list(r)


def art_ion_substep(ctx, n_H, x_n, src_pos, src_lum, n_src, ip: art_ion_params, t_end, t_now,
                    rate, force, J, impulse):
    check(lib().art_ion_substep(C.c_void_p(ctx), n_H, x_n, src_pos, src_lum, int(n_src), C.byref(ip),
                                float(t_end), t_now, rate, force, J, impulse), "art_ion_substep")


def art_ion_subcycle(ctx, n_H, x_n, src_pos, src_lum, n_src, ip: art_ion_params, t_end, max_substeps,
                     rate, force, J, impulse):
    k, t = C.c_int(), C.c_double()
    check(lib().art_ion_subcycle(C.c_void_p(ctx), n_H, x_n, src_pos, src_lum, int(n_src), C.byref(ip),
                                 float(t_end), int(max_substeps), rate, force, J, impulse, C.byref(k),
                                 C.byref(t)), "art_ion_subcycle")
    return k.value, t.value


def art_trace_noalloc(nx, ny, nz, params: art_params, n_H, x_n, src_pos, src_lum, n_src, rate, force, J,
                      status, stream):
    check(lib().art_trace_noalloc(int(nx), int(ny), int(nz), C.byref(params), n_H, x_n, src_pos, src_lum,
                                  int(n_src), rate, force, J, status, C.c_void_p(stream)), "art_trace_noalloc")


def art_destroy(ctx):
    if ctx:
        lib().art_destroy(C.c_void_p(ctx))


def art_strerror(code: int) -> str:
    return strerror(code)
