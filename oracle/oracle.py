"""ctypes wrapper of the FP64 CPU oracle (``art_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``; never by the product path.  It imports nothing
from the HIP package.

Every function takes numpy arrays (float32 inputs are widened to float64 exactly)
and returns float64 results.  Field layout: flat arrays of ``nx*ny*nz`` with x
fastest; ``force``/``v`` are ``[3, N]`` (structure of arrays).
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "art_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_LEVELS = 16
MAX_BINS = 2


# gcc flags of the oracle: no FMA contraction, no fast math (the reference stays
# plain FP64); the timing build adds -O3 -march=native, which leaves every
# result bitwise unchanged under these flags
CFLAGS = ["-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]


def compile_library(src: str, out: str, opt=("-O2",)) -> str:
    """gcc ``src`` into the shared library ``out`` with the oracle's flags."""
    subprocess.check_call(["gcc", *opt, *CFLAGS, "-o", out + ".tmp", src, "-lm"])
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_library(_SRC, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("level0", C.c_int), ("level_max", C.c_int),
                ("phi_c", C.c_double), ("tau_term", C.c_double),
                ("s_H", C.c_double), ("s_d", C.c_double),
                ("n_bins", C.c_int), ("rot", C.c_double * 9)]


class _Stats(C.Structure):
    _fields_ = [("created", C.c_void_p), ("split", C.c_void_p), ("exited", C.c_void_p),
                ("terminated", C.c_void_p), ("segments", C.c_void_p),
                ("escaped", C.c_void_p), ("residual", C.c_void_p),
                ("absorbed", C.c_void_p), ("emitted", C.c_void_p),
                ("destroy", C.c_uint64)]


_lib = None


@contextlib.contextmanager
def using_library(path: str):
    """Run the wrappers below on another build of the oracle's source (a timing
    build, or a test's deliberately altered copy), then restore the default."""
    global _lib
    keep = _lib
    _lib = _bind(C.CDLL(path))
    try:
        yield
    finally:
        _lib = keep


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(C.CDLL(_LIB))
    return _lib


def _bind(lib):
    """Declare the C signatures of the oracle's entry points on a loaded build."""
    P = C.POINTER(_Params)
    d = C.POINTER(C.c_double)
    lib.orc_trace.argtypes = [P, d, d, C.c_int, d, d, C.c_void_p, d, d, C.POINTER(_Stats)]
    lib.orc_trace.restype = C.c_int
    lib.orc_tangent.argtypes = [P, d, d, d, d, C.c_int, d, d, d, d]
    lib.orc_tangent.restype = C.c_int
    lib.orc_adjoint.argtypes = [P, d, d, C.c_int, d, d, d, d, d, d]
    lib.orc_adjoint.restype = C.c_int
    lib.orc_pix2vec_nest.argtypes = [C.c_int, C.c_int64, d]
    lib.orc_pix2vec_nest.restype = None
    lib.orc_pix2ang_nest.argtypes = [C.c_int, C.c_int64, d, d]
    lib.orc_pix2ang_nest.restype = None
    lib.orc_r_max.argtypes = [C.c_double, C.c_int]
    lib.orc_r_max.restype = C.c_double
    lib.orc_ray_segments.argtypes = [C.c_int, C.c_int, C.c_int, d, d, C.c_double,
                                     C.c_double, C.POINTER(C.c_int64), d, C.c_int64]
    lib.orc_ray_segments.restype = C.c_int64
    lib.orc_seed_order.argtypes = [C.c_int, C.POINTER(C.c_int64), C.c_int64]
    lib.orc_seed_order.restype = C.c_int64
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _params(nx, ny, nz, level0, level_max, phi_c, tau_term, s_H, s_d, n_bins, rot=None):
    p = _Params()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.level0, p.level_max = int(level0), int(level_max)
    p.phi_c, p.tau_term = float(phi_c), float(tau_term)
    p.s_H, p.s_d = float(s_H), float(s_d)
    p.n_bins = int(n_bins)
    r = np.eye(3) if rot is None else np.asarray(rot, dtype=np.float64).reshape(3, 3)
    for i in range(9):
        p.rot[i] = float(r.reshape(-1)[i])
    return p


@dataclass
class OracleResult:
    rate: np.ndarray        # [N]
    force: np.ndarray       # [3, N]
    J: np.ndarray           # [n_bins, N]
    created: np.ndarray     # [n_src, 16] int64
    split: np.ndarray
    exited: np.ndarray
    terminated: np.ndarray
    segments: np.ndarray    # [n_src]
    escaped: np.ndarray     # [n_src, n_bins]
    residual: np.ndarray
    absorbed: np.ndarray
    emitted: np.ndarray
    destroy: int


def pix2vec_nest(level: int, pix: int) -> np.ndarray:
    v = np.zeros(3)
    _load().orc_pix2vec_nest(int(level), int(pix), _dp(v))
    return v


def pix2ang_nest(level: int, pix: int):
    z = C.c_double()
    phi = C.c_double()
    _load().orc_pix2ang_nest(int(level), int(pix), C.byref(z), C.byref(phi))
    return z.value, phi.value


def seed_order(level0: int, n: int) -> np.ndarray:
    """The first n level-l0 pixels in the order the oracle traces them (Sec. 2.2, Step 1)."""
    out = np.zeros(n, dtype=np.int64)
    k = _load().orc_seed_order(int(level0), out.ctypes.data_as(C.POINTER(C.c_int64)), int(n))
    return out[:k]


def r_max(phi_c: float, level: int) -> float:
    return _load().orc_r_max(float(phi_c), int(level))


def ray_segments(shape, xs, n, r_a, r_end, cap=100000):
    """(cells, dr) of one ray through an (nx, ny, nz) grid over [r_a, min(r_end, exit)]."""
    nx, ny, nz = shape
    cells = np.zeros(cap, dtype=np.int64)
    drs = np.zeros(cap)
    m = _load().orc_ray_segments(nx, ny, nz, _dp(_f64(xs)), _dp(_f64(n)), float(r_a),
                                 float(r_end), cells.ctypes.data_as(C.POINTER(C.c_int64)),
                                 _dp(drs), cap)
    if m < 0:
        raise RuntimeError("segment buffer too small")
    return cells[:m].copy(), drs[:m].copy()


def _transparent(n_H, transparent):
    """Sink control volumes (Sec. 4.1: the radiation ignores the gas in
    them): the cells flagged in ``transparent`` neither absorb nor receive the
    absorbed photons, which is the sweep with no gas there."""
    nH = _f64(n_H).reshape(-1)
    if transparent is None:
        return nH
    return np.where(np.asarray(transparent).reshape(-1) != 0, 0.0, nH)


def trace(nx, ny, nz, n_H, x_n, src_pos, src_lum, *, s_H, s_d, n_bins, level0=2,
          level_max=13, phi_c=4.0, tau_term=float(np.log(1e10)), rot=None,
          transparent=None) -> OracleResult:
    """Forward ART sweep in FP64 (see art_oracle.c for the definition).
    ``transparent``: optional per-cell flags of sink control volumes."""
    lib = _load()
    N = int(nx) * int(ny) * int(nz)
    nH = _transparent(n_H, transparent)
    xn = _f64(x_n).reshape(-1)
    pos = _f64(src_pos).reshape(-1, 3)
    ns = pos.shape[0]
    lum = _f64(src_lum).reshape(ns, n_bins)
    assert nH.size == N and xn.size == N
    rate = np.zeros(N)
    force = np.zeros((3, N))
    J = np.zeros((n_bins, N))
    st = {k: np.zeros((ns, MAX_LEVELS), dtype=np.int64)
          for k in ("created", "split", "exited", "terminated")}
    segs = np.zeros(ns, dtype=np.int64)
    fl = {k: np.zeros((ns, MAX_BINS)) for k in ("escaped", "residual", "absorbed", "emitted")}
    S = _Stats()
    for k in ("created", "split", "exited", "terminated"):
        setattr(S, k, st[k].ctypes.data)
    S.segments = segs.ctypes.data
    for k in fl:
        setattr(S, k, fl[k].ctypes.data)
    p = _params(nx, ny, nz, level0, level_max, phi_c, tau_term, s_H, s_d, n_bins, rot)
    rc = lib.orc_trace(C.byref(p), _dp(nH), _dp(xn), ns, _dp(pos), _dp(lum),
                       J.ctypes.data, _dp(force), _dp(rate), C.byref(S))
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return OracleResult(rate=rate, force=force, J=J, segments=segs, destroy=int(S.destroy),
                        **st, **{k: v[:, :n_bins].copy() for k, v in fl.items()})


def tangent(nx, ny, nz, n_H, x_n, dn_H, dx_n, src_pos, src_lum, *, s_H, s_d, n_bins,
            level0=2, level_max=13, phi_c=4.0, tau_term=float(np.log(1e10)), rot=None):
    """(d rate, d force) along (dn_H, dx_n), ray tree held fixed."""
    lib = _load()
    N = int(nx) * int(ny) * int(nz)
    pos = _f64(src_pos).reshape(-1, 3)
    ns = pos.shape[0]
    lum = _f64(src_lum).reshape(ns, n_bins)
    drate = np.zeros(N)
    dforce = np.zeros((3, N))
    p = _params(nx, ny, nz, level0, level_max, phi_c, tau_term, s_H, s_d, n_bins, rot)
    rc = lib.orc_tangent(C.byref(p), _dp(_f64(n_H).reshape(-1)), _dp(_f64(x_n).reshape(-1)),
                         _dp(_f64(dn_H).reshape(-1)), _dp(_f64(dx_n).reshape(-1)), ns,
                         _dp(pos), _dp(lum), _dp(drate), _dp(dforce))
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return drate, dforce


def adjoint(nx, ny, nz, n_H, x_n, src_pos, src_lum, w, v, *, s_H, s_d, n_bins, level0=2,
            level_max=13, phi_c=4.0, tau_term=float(np.log(1e10)), rot=None, transparent=None):
    """(dL/dn_H, dL/dx_n) for L = sum w*rate + sum v.force, ray tree held fixed.
    With ``transparent``, the outputs do not depend on the flagged cells' fields,
    whose gradients are zero."""
    if transparent is not None:
        g_nH, g_xn = adjoint(nx, ny, nz, _transparent(n_H, transparent), x_n, src_pos, src_lum, w, v,
                             s_H=s_H, s_d=s_d, n_bins=n_bins, level0=level0, level_max=level_max,
                             phi_c=phi_c, tau_term=tau_term, rot=rot)
        m = np.asarray(transparent).reshape(-1) != 0
        g_nH[m] = 0.0
        g_xn[m] = 0.0
        return g_nH, g_xn
    lib = _load()
    N = int(nx) * int(ny) * int(nz)
    pos = _f64(src_pos).reshape(-1, 3)
    ns = pos.shape[0]
    lum = _f64(src_lum).reshape(ns, n_bins)
    g_nH = np.zeros(N)
    g_xn = np.zeros(N)
    p = _params(nx, ny, nz, level0, level_max, phi_c, tau_term, s_H, s_d, n_bins, rot)
    rc = lib.orc_adjoint(C.byref(p), _dp(_f64(n_H).reshape(-1)), _dp(_f64(x_n).reshape(-1)),
                         ns, _dp(pos), _dp(lum), _dp(_f64(w).reshape(-1)),
                         _dp(_f64(v).reshape(-1)), _dp(g_nH), _dp(g_xn))
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return g_nH, g_xn


def trace_workload(wl, **over) -> OracleResult:
    """Forward sweep of an ``inputs.Workload``-like object (duck-typed)."""
    kw = dict(wl.params())
    kw.update(over)
    return trace(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum, **kw)
