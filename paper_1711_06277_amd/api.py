"""PyTorch-facing wrapper of the HIP ART sweep.

PyTorch supplies device memory and the stream; every step of the sweep runs in
``libart.so`` through the C ABI (``_abi``).  There is no CPU path: without the
built library or a GPU these calls raise.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi as A

TAU_TERM_1E10 = math.log(1.0e10)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, device):
    t = torch.as_tensor(t, dtype=dtype, device=device)
    return t.contiguous()


@dataclass
class TraceStats:
    status: int
    n_src: int
    n_waves: int
    segments: int
    destroy: int
    destroy_expected: int
    rays_max_wave: int
    created: np.ndarray      # [16] totals per level
    split: np.ndarray
    exited: np.ndarray
    terminated: np.ndarray
    src_created: np.ndarray  # [n_src, 16]
    src_split: np.ndarray
    src_exited: np.ndarray
    src_terminated: np.ndarray
    src_escaped: np.ndarray  # [n_src, 2]
    src_residual: np.ndarray
    src_segments: np.ndarray  # [n_src]
    src_rays_bound: np.ndarray  # [n_src] bound on each source's rays (device-planned waves; else 0)


class ArtTracer:
    """One ART context: grid shape, method parameters and the device workspace.

    Parameters follow Sec. 2.1 / 2.3 of the paper: ``level0`` (initial HEALPix
    level), ``level_max``, ``phi_c`` (m_ray), ``tau_term`` (termination optical
    depth), ``s_H`` / ``s_d`` (gas / dust opacity per cell length per unit
    density), ``n_bins`` (1: ionizing, 2: + non-ionizing).
    """

    def __init__(self, nx, ny, nz, *, s_H, s_d, n_bins=1, level0=2, level_max=13, phi_c=4.0,
                 tau_term=TAU_TERM_1E10, rot=None, deterministic=False, max_sources=1,
                 enable_adjoint=False, pool_rays=0, pool_mem_fraction=0.5, block_size=0,
                 blocks_per_cu=0, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("ArtTracer needs a GPU: the sweep has no CPU implementation")
        self.device = torch.device(device)
        self.shape = (int(nx), int(ny), int(nz))
        self.N = int(nx) * int(ny) * int(nz)
        self.n_bins = int(n_bins)
        self.s_H, self.s_d = float(s_H), float(s_d)
        self.max_sources = int(max_sources)
        p = A.art_params()
        p.level0, p.level_max = int(level0), int(level_max)
        p.phi_c, p.tau_term = float(phi_c), float(tau_term)
        p.s_H, p.s_d = self.s_H, self.s_d
        p.n_bins = self.n_bins
        r = np.eye(3) if rot is None else np.asarray(rot, dtype=np.float64).reshape(3, 3)
        for i, x in enumerate(r.reshape(-1)):
            p.rot[i] = float(x)
        p.deposit_mode = A.ART_DEPOSIT_DETERMINISTIC if deterministic else A.ART_DEPOSIT_ATOMIC
        o = A.art_options()
        o.max_sources = self.max_sources
        o.enable_adjoint = 1 if enable_adjoint else 0
        o.pool_rays = int(pool_rays)
        o.pool_mem_fraction = float(pool_mem_fraction)
        o.block_size, o.blocks_per_cu = int(block_size), int(blocks_per_cu)
        self.params, self.options = p, o
        self.last_tape = 0
        self._tape_inputs = None
        with torch.cuda.device(self.device):
            self._ctx = A.art_create(nx, ny, nz, p, o, torch.cuda.current_stream().cuda_stream)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            A.art_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        A.art_set_stream(self._ctx, torch.cuda.current_stream(self.device).cuda_stream)

    # -- calls ---------------------------------------------------------------
    def trace(self, n_H, x_n, src_pos, src_lum, *, want_J=False, out=None, check=True):
        """Forward sweep.  Returns (rate [N], force [3, N]) or (rate, force, J)."""
        d = self.device
        n_H = _dev(n_H, torch.float32, d).reshape(-1)
        x_n = _dev(x_n, torch.float32, d).reshape(-1)
        src_pos = _dev(src_pos, torch.float64, d).reshape(-1, 3)
        n_src = src_pos.shape[0]
        src_lum = _dev(src_lum, torch.float32, d).reshape(n_src, self.n_bins)
        if n_H.numel() != self.N or x_n.numel() != self.N:
            raise ValueError("field size does not match the grid")
        if out is None:
            rate = torch.empty(self.N, dtype=torch.float32, device=d)
            force = torch.empty((3, self.N), dtype=torch.float32, device=d)
            J = torch.empty((self.n_bins, self.N), dtype=torch.float32, device=d) if want_J else None
        else:
            rate, force, J = out
        self._stream()
        A.art_trace(self._ctx, _ptr(n_H), _ptr(x_n), _ptr(src_pos), _ptr(src_lum), n_src,
                    _ptr(rate), _ptr(force), _ptr(J))
        # token of the ray tree this trace left in the pool (0 if none): the inputs
        # it was traced from are kept referenced with it, so that a later
        # adjoint(..., tape=...) passes the very same device buffers
        self.last_tape = A.art_get_tape(self._ctx)
        self._tape_inputs = (n_H, x_n, src_pos, src_lum) if self.last_tape else None
        if check:
            A.check(A.art_sync(self._ctx), "art_trace (device)")
        return (rate, force, J) if want_J else (rate, force)

    # -- sink control volumes (Sec. 4.1) ----------------------------------------
    def set_transparent(self, mask):
        """Flag transparent cells, whose gas the radiation ignores (a uint8 or bool
        device tensor of N cells, kept referenced here), or None to clear."""
        if mask is None:
            self._transparent = None
            A.art_set_transparent(self._ctx, None)
            return
        if not (isinstance(mask, torch.Tensor) and mask.is_cuda and mask.numel() == self.N):
            raise ValueError("mask must be a device tensor of N cells")
        m = mask.reshape(-1).to(torch.uint8).contiguous()
        self._transparent = m
        A.art_set_transparent(self._ctx, _ptr(m))

    # -- rotation of the ray directions (Sec. 2.1) ------------------------------
    def set_rotation(self, rot):
        """Rotate every ray direction by rot (3x3, orthonormal) from the next call on."""
        self._stream()
        A.art_set_rotation(self._ctx, np.asarray(rot, dtype=np.float64).reshape(9))

    def random_rotation(self, u):
        """Draw a uniform random rotation on the device from u, a float64 device tensor
        of three numbers in [0, 1) (graph-capturable: u is read when the call runs)."""
        if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == torch.float64 and u.numel() >= 3
                and u.is_contiguous()):
            raise ValueError("u must be a contiguous float64 device tensor of 3 numbers")
        self._stream()
        A.art_random_rotation(self._ctx, _ptr(u))

    def rotation(self) -> np.ndarray:
        """The current rotation (synchronises)."""
        return np.array(A.art_get_rotation(self._ctx)).reshape(3, 3)

    # -- ionization subcycle (Sec. 2.3) ----------------------------------------
    def _ion_args(self, n_H, x_n, src_pos, src_lum, out):
        d = self.device
        if not (isinstance(x_n, torch.Tensor) and x_n.is_cuda and x_n.dtype == torch.float32
                and x_n.is_contiguous() and x_n.numel() == self.N):
            raise ValueError("x_n must be a contiguous float32 device tensor of N cells (updated in place)")
        n_H = _dev(n_H, torch.float32, d).reshape(-1)
        if n_H.numel() != self.N:
            raise ValueError("field size does not match the grid")
        src_pos = _dev(src_pos, torch.float64, d).reshape(-1, 3)
        n_src = src_pos.shape[0]
        src_lum = _dev(src_lum, torch.float32, d).reshape(n_src, self.n_bins)
        if out is None:
            out = (torch.empty(self.N, dtype=torch.float32, device=d),
                   torch.empty((3, self.N), dtype=torch.float32, device=d),
                   torch.empty((self.n_bins, self.N), dtype=torch.float32, device=d))
        return n_H, src_pos, n_src, src_lum, out

    def ion_substep(self, n_H, x_n, src_pos, src_lum, *, alpha_B, gamma_scale, C=0.1, t_end, t_now,
                    out=None, impulse=None, check=True):
        """One radiation substep: sweep of the current x_n, dt = min(C min(n_H/|I-R|),
        t_end - t_now) (Eq. e:dtss), Method B update of x_n in place (Eq. e:xn3),
        impulse += force * dt, t_now += dt.  x_n: float32 device tensor; t_now: float64
        device tensor of one element.  Returns (rate, force, J) of the substep's sweep."""
        n_H, src_pos, n_src, src_lum, out = self._ion_args(n_H, x_n, src_pos, src_lum, out)
        if not (isinstance(t_now, torch.Tensor) and t_now.is_cuda and t_now.dtype == torch.float64):
            raise ValueError("t_now must be a float64 device tensor")
        ip = A.art_ion_params(float(alpha_B), float(gamma_scale), float(C))
        self._stream()
        A.art_ion_substep(self._ctx, _ptr(n_H), _ptr(x_n), _ptr(src_pos), _ptr(src_lum), n_src, ip,
                          float(t_end), _ptr(t_now), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]),
                          _ptr(impulse))
        if check:
            A.check(A.art_sync(self._ctx), "art_ion_substep (device)")
        return out

    def ion_subcycle(self, n_H, x_n, src_pos, src_lum, *, alpha_B, gamma_scale, C=0.1, t_end,
                     max_substeps=1000000, out=None, impulse=None):
        """Substeps from t = 0 until t_end (synchronises after each).  Returns
        (n_substeps, t_reached); x_n is updated in place."""
        n_H, src_pos, n_src, src_lum, out = self._ion_args(n_H, x_n, src_pos, src_lum, out)
        ip = A.art_ion_params(float(alpha_B), float(gamma_scale), float(C))
        self._stream()
        return A.art_ion_subcycle(self._ctx, _ptr(n_H), _ptr(x_n), _ptr(src_pos), _ptr(src_lum), n_src,
                                  ip, float(t_end), int(max_substeps), _ptr(out[0]), _ptr(out[1]),
                                  _ptr(out[2]), _ptr(impulse))

    def adjoint(self, n_H, x_n, src_pos, src_lum, g_rate, g_force, *, tape=None, out=None, check=True):
        """dL/dn_H, dL/dx_n for L = <g_rate, rate> + <g_force, force>.

        Without ``tape`` the ray tree is traced again from the given inputs.  With
        ``tape`` (the ``last_tape`` of a trace on this tracer, whose inputs must not
        have changed since) the stored tree is reused; the inputs are those that
        trace kept.  Raises ArtError (ART_ERR_NO_FORWARD) if that tape is gone."""
        d = self.device
        if tape:
            if self._tape_inputs is None:
                raise A.ArtError(A.ART_ERR_NO_FORWARD, "adjoint(tape=...)")
            n_H, x_n, src_pos, src_lum = self._tape_inputs
        else:
            n_H = _dev(n_H, torch.float32, d).reshape(-1)
            x_n = _dev(x_n, torch.float32, d).reshape(-1)
            src_pos = _dev(src_pos, torch.float64, d).reshape(-1, 3)
        n_src = src_pos.shape[0]
        src_lum = _dev(src_lum, torch.float32, d).reshape(n_src, self.n_bins)
        g_rate = _dev(g_rate, torch.float32, d).reshape(-1)
        g_force = _dev(g_force, torch.float32, d).reshape(3, -1)
        if out is None:
            g_nH = torch.empty(self.N, dtype=torch.float32, device=d)
            g_xn = torch.empty(self.N, dtype=torch.float32, device=d)
        else:
            g_nH, g_xn = out
        self._stream()
        if tape:
            A.art_trace_adjoint_tape(self._ctx, tape, _ptr(n_H), _ptr(x_n), _ptr(src_pos), _ptr(src_lum),
                                     n_src, _ptr(g_rate), _ptr(g_force), _ptr(g_nH), _ptr(g_xn))
        else:
            A.art_trace_adjoint(self._ctx, _ptr(n_H), _ptr(x_n), _ptr(src_pos), _ptr(src_lum), n_src,
                                _ptr(g_rate), _ptr(g_force), _ptr(g_nH), _ptr(g_xn))
        if check:
            A.check(A.art_sync(self._ctx), "art_trace_adjoint (device)")
        return g_nH, g_xn

    def trace_and_adjoint(self, n_H, x_n, src_pos, src_lum, g_rate, g_force, *, want_J=False, out=None,
                          check=True):
        """Forward sweep and the adjoint of L = <g_rate, rate> + <g_force, force> in one
        call (each source wave's tree is walked back right after it is traced).
        Returns (rate, force[, J], g_nH, g_xn)."""
        d = self.device
        n_H = _dev(n_H, torch.float32, d).reshape(-1)
        x_n = _dev(x_n, torch.float32, d).reshape(-1)
        src_pos = _dev(src_pos, torch.float64, d).reshape(-1, 3)
        n_src = src_pos.shape[0]
        src_lum = _dev(src_lum, torch.float32, d).reshape(n_src, self.n_bins)
        g_rate = _dev(g_rate, torch.float32, d).reshape(-1)
        g_force = _dev(g_force, torch.float32, d).reshape(3, -1)
        if n_H.numel() != self.N or x_n.numel() != self.N:
            raise ValueError("field size does not match the grid")
        if out is None:
            out = (torch.empty(self.N, dtype=torch.float32, device=d),
                   torch.empty((3, self.N), dtype=torch.float32, device=d),
                   torch.empty((self.n_bins, self.N), dtype=torch.float32, device=d) if want_J else None,
                   torch.empty(self.N, dtype=torch.float32, device=d),
                   torch.empty(self.N, dtype=torch.float32, device=d))
        rate, force, J, g_nH, g_xn = out
        self._stream()
        A.art_trace_and_adjoint(self._ctx, _ptr(n_H), _ptr(x_n), _ptr(src_pos), _ptr(src_lum), n_src,
                                _ptr(rate), _ptr(force), _ptr(J), _ptr(g_rate), _ptr(g_force),
                                _ptr(g_nH), _ptr(g_xn))
        self.last_tape = A.art_get_tape(self._ctx)
        self._tape_inputs = (n_H, x_n, src_pos, src_lum) if self.last_tape else None
        if check:
            A.check(A.art_sync(self._ctx), "art_trace_and_adjoint (device)")
        return (rate, force, J, g_nH, g_xn) if want_J else (rate, force, g_nH, g_xn)

    def sync(self) -> int:
        return A.art_sync(self._ctx)

    def stats(self, n_src_stats=None) -> TraceStats:
        ns = self.max_sources if n_src_stats is None else int(n_src_stats)
        L = A.ART_MAX_LEVELS
        arr = {k: np.zeros((ns, L), dtype=np.uint32) for k in ("c", "s", "e", "t")}
        esc = np.zeros((ns, 2))
        res = np.zeros((ns, 2))
        seg = np.zeros(ns, dtype=np.uint64)
        bnd = np.zeros(ns, dtype=np.uint64)
        st = A.art_get_stats(self._ctx, ns, *(arr[k].ctypes.data for k in "cset"),
                             esc.ctypes.data, res.ctypes.data, seg.ctypes.data, bnd.ctypes.data)
        n = min(ns, st.n_src)
        return TraceStats(
            status=st.status, n_src=st.n_src, n_waves=st.n_waves, segments=int(st.segments),
            destroy=int(st.destroy), destroy_expected=int(st.destroy_expected),
            rays_max_wave=int(st.rays_max_wave),
            created=np.array(st.created[:], dtype=np.int64), split=np.array(st.split[:], dtype=np.int64),
            exited=np.array(st.exited[:], dtype=np.int64),
            terminated=np.array(st.terminated[:], dtype=np.int64),
            src_created=arr["c"][:n].astype(np.int64), src_split=arr["s"][:n].astype(np.int64),
            src_exited=arr["e"][:n].astype(np.int64), src_terminated=arr["t"][:n].astype(np.int64),
            src_escaped=esc[:n, : self.n_bins], src_residual=res[:n, : self.n_bins],
            src_segments=seg[:n].astype(np.int64), src_rays_bound=bnd[:n].astype(np.int64))

    def autotune_key(self, n_src: int, kind: str = "sweep") -> str:
        """Cache key of a tuned setting: what is tuned ("sweep": launch shape and sources
        per wave; "adjoint": the adjoint's launch shape), GPU name, grid, sources, bins,
        deposit mode, levels, m_ray, pool capacity."""
        p = self.params
        return "|".join([kind, torch.cuda.get_device_name(self.device), "x".join(map(str, self.shape)),
                         f"src{int(n_src)}", f"bins{self.n_bins}", f"mode{p.deposit_mode}",
                         f"l{p.level0}-{p.level_max}", f"m{p.phi_c:g}", f"adj{self.options.enable_adjoint}",
                         f"pool{self.options.pool_rays}"])

    def _inputs(self, n_H, x_n, src_pos, src_lum):
        d = self.device
        n_H = _dev(n_H, torch.float32, d).reshape(-1)
        x_n = _dev(x_n, torch.float32, d).reshape(-1)
        src_pos = _dev(src_pos, torch.float64, d).reshape(-1, 3)
        src_lum = _dev(src_lum, torch.float32, d).reshape(src_pos.shape[0], self.n_bins)
        return n_H, x_n, src_pos, src_lum

    def autotune(self, n_H, x_n, src_pos, src_lum, *, cache=None):
        """Time the built-in launch shapes, then caps on the sources per wave, on these
        inputs and keep the fastest; returns (block_size, blocks_per_cu, wave_sources, ms),
        wave_sources 0 meaning no cap.  With ``cache`` (a JSON file path, or True for
        $ART_AUTOTUNE_CACHE or ~/.cache/art_mi355x/autotune.json) a setting found before
        for the same key is applied without timing, and new results are stored."""
        n_H, x_n, src_pos, src_lum = self._inputs(n_H, x_n, src_pos, src_lum)
        n_src = int(src_pos.shape[0])
        path = autotune_cache_path(cache)
        key = self.autotune_key(n_src, "sweep")
        if path is not None:
            hit = load_autotune_cache(path).get(key)
            if hit is not None and len(hit) == 4:
                A.art_set_launch(self._ctx, hit[0], hit[1])
                A.art_set_wave_sources(self._ctx, hit[2])
                return int(hit[0]), int(hit[1]), int(hit[2]), float(hit[3])
        rate = torch.empty(self.N, dtype=torch.float32, device=self.device)
        force = torch.empty((3, self.N), dtype=torch.float32, device=self.device)
        self._stream()
        result = A.art_autotune(self._ctx, _ptr(n_H), _ptr(x_n), _ptr(src_pos), _ptr(src_lum), n_src,
                                _ptr(rate), _ptr(force))
        if path is not None:
            store_autotune_cache(path, key, result)
        return result

    def autotune_adjoint(self, n_H, x_n, src_pos, src_lum, g_rate, g_force, *, cache=None):
        """The adjoint sweep's launch shape, likewise; returns (block_size, blocks_per_cu, ms)."""
        n_H, x_n, src_pos, src_lum = self._inputs(n_H, x_n, src_pos, src_lum)
        n_src = int(src_pos.shape[0])
        path = autotune_cache_path(cache)
        key = self.autotune_key(n_src, "adjoint")
        if path is not None:
            hit = load_autotune_cache(path).get(key)
            if hit is not None and len(hit) == 3:
                A.art_set_adjoint_launch(self._ctx, hit[0], hit[1])
                return int(hit[0]), int(hit[1]), float(hit[2])
        d = self.device
        g_rate = _dev(g_rate, torch.float32, d).reshape(-1)
        g_force = _dev(g_force, torch.float32, d).reshape(3, -1)
        rate = torch.empty(self.N, dtype=torch.float32, device=d)
        force = torch.empty((3, self.N), dtype=torch.float32, device=d)
        g_nH = torch.empty(self.N, dtype=torch.float32, device=d)
        g_xn = torch.empty(self.N, dtype=torch.float32, device=d)
        self._stream()
        result = A.art_autotune_adjoint(self._ctx, _ptr(n_H), _ptr(x_n), _ptr(src_pos), _ptr(src_lum), n_src,
                                        _ptr(rate), _ptr(force), _ptr(g_rate), _ptr(g_force), _ptr(g_nH),
                                        _ptr(g_xn))
        self.last_tape = 0
        self._tape_inputs = None
        if path is not None:
            store_autotune_cache(path, key, result)
        return result

    def set_wave_sources(self, n: int):
        """Trace at most n sources per wave (0: as many as the pool holds)."""
        A.art_set_wave_sources(self._ctx, int(n))

    def set_timing(self, enable: bool):
        A.art_set_timing(self._ctx, enable)

    def timing(self):
        """(sum of sweep-kernel durations in ms, number of sweep launches, whole call ms)."""
        return A.art_get_timing(self._ctx)


def autotune_cache_path(cache):
    """None (no cache), an explicit path, or for True the default location."""
    if cache is None or cache is False:
        return None
    if cache is True:
        return os.environ.get("ART_AUTOTUNE_CACHE",
                              os.path.join(os.path.expanduser("~"), ".cache", "art_mi355x", "autotune.json"))
    return str(cache)


def load_autotune_cache(path) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_autotune_cache(path, key, result) -> None:
    """Add one entry (integers, then the time in ms last), replacing the file atomically."""
    data = load_autotune_cache(path)
    data[key] = [int(x) for x in result[:-1]] + [float(result[-1])]
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class ArtTrace(torch.autograd.Function):
    """(rate, force) = ART sweep of (n_H, x_n); backward runs the adjoint sweep."""

    @staticmethod
    def forward(ctx, n_H, x_n, tracer: ArtTracer, src_pos, src_lum):
        rate, force = tracer.trace(n_H, x_n, src_pos, src_lum)
        ctx.tracer = tracer
        ctx.tape = tracer.last_tape
        ctx.save_for_backward(n_H, x_n, src_pos, src_lum)
        return rate, force

    @staticmethod
    def backward(ctx, g_rate, g_force):
        # autograd checks that the saved inputs were not modified in place, so the
        # forward's tree may be reused as long as the tracer still holds it
        n_H, x_n, src_pos, src_lum = ctx.saved_tensors
        tr = ctx.tracer
        if g_rate is None:
            g_rate = torch.zeros(tr.N, dtype=torch.float32, device=n_H.device)
        if g_force is None:
            g_force = torch.zeros((3, tr.N), dtype=torch.float32, device=n_H.device)
        tape = ctx.tape if ctx.tape and ctx.tape == A.art_get_tape(tr._ctx) else None
        g_nH, g_xn = tr.adjoint(n_H, x_n, src_pos, src_lum, g_rate, g_force, tape=tape)
        return g_nH.view_as(n_H), g_xn.view_as(x_n), None, None, None


def art_trace(n_H, x_n, tracer: ArtTracer, src_pos, src_lum):
    """Differentiable forward sweep: returns (rate, force)."""
    return ArtTrace.apply(n_H, x_n, tracer, src_pos, src_lum)
