"""Seeded synthetic inputs for the ART sweep (grids, sources, loss weights).

This module only *draws* inputs; it contains none of the ray-tracing arithmetic.
Both the FP64 oracle tests and the HIP path read their inputs from here, so the
two sides always see bit-identical float32/float64 arrays.

Workloads (stand-ins for the paper's turbulent-cloud snapshots, which are not
available): a lognormal density field ``n_H = exp(g)/<exp(g)>`` where ``g`` is a
periodic Gaussian random field whose per-mode variance falls as ``|k|^-4``
(amplitude ``|k|^-2``), standardised to a given std.  The ``k^-4`` slope follows
the turbulent velocity spectrum the paper uses for its cloud initial conditions
(Sec. 4.1).  Sources are drawn cell-wise with probability proportional to
``n_H`` and jittered by ``U(-0.25, 0.25)`` cells so that no source sits on a
cell face.

Layout conventions shared by every consumer: a 3-D field is a flat float32
array of ``nx*ny*nz`` values with x fastest, i.e. cell ``(i, j, k)`` is element
``(k*ny + j)*nx + i`` and occupies ``[i, i+1) x [j, j+1) x [k, k+1)`` in cell
units.  ``src_pos`` is float64 ``[n_src, 3]`` (x, y, z); ``src_lum`` is float32
``[n_src, n_bins]`` with bin 0 ionizing (gas + dust opacity) and bin 1
non-ionizing (dust only).

Seeds: workload ``c`` uses ``1000*c + {0: density, 1: second field,
2: sources, 3: loss weights}``.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

TAU_TERM_1E10 = math.log(1.0e10)  # photon fraction 1e-10 -> tau = ln(1e10)


def _fft_workers() -> int:
    """Threads for the FFTs (pocketfft splits them into independent 1-D
    transforms, so the result does not depend on the count)."""
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 1


def gaussian_field(n: int, std: float, seed: int) -> np.ndarray:
    """Periodic Gaussian random field on an n^3 grid, per-mode variance ~ |k|^-4.

    Returned as float64 with axes (z, y, x), mean 0 and the requested std.
    """
    import scipy.fft as sfft
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    wk = sfft.rfftn(w, workers=_fft_workers())
    del w
    kz = np.fft.fftfreq(n) * n
    ky = np.fft.fftfreq(n) * n
    kx = np.fft.rfftfreq(n) * n
    k2 = (kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    k2[0, 0, 0] = 1.0
    amp = 1.0 / k2  # |k|^-2 amplitude -> |k|^-4 power
    amp[0, 0, 0] = 0.0
    wk *= amp
    del k2, amp
    g = sfft.irfftn(wk, s=(n, n, n), axes=(0, 1, 2), workers=_fft_workers())
    del wk
    g -= g.mean()
    g *= std / g.std()
    return g


def lognormal_density(n: int, std: float, seed: int) -> np.ndarray:
    """n_H = exp(g) / mean(exp(g)) as a flat float32 array (x fastest)."""
    g = gaussian_field(n, std, seed)
    np.exp(g, out=g)
    g /= g.mean()
    return np.ascontiguousarray(g.astype(np.float32).reshape(-1))


def sigmoid_fraction(n: int, std: float, seed: int) -> np.ndarray:
    """x_n = 1/(1+exp(-h)) with h a second k^-4 field of the given std (flat float32)."""
    h = gaussian_field(n, std, seed)
    x = 1.0 / (1.0 + np.exp(-h))
    return np.ascontiguousarray(x.astype(np.float32).reshape(-1))


def sample_sources(n_H: np.ndarray, n: int, n_src: int, rng: np.random.Generator) -> np.ndarray:
    """Cells drawn with probability ~ n_H (with replacement), centre + U(-0.25,0.25)^3."""
    p = n_H.astype(np.float64)
    p /= p.sum()
    # inverse-CDF draw, the same draws as rng.choice(p.size, n_src, p=p) without its
    # slow validation of p
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    idx = cdf.searchsorted(rng.random(n_src), side="right")
    i = idx % n
    j = (idx // n) % n
    k = idx // (n * n)
    pos = np.stack([i, j, k], axis=1).astype(np.float64) + 0.5
    pos += rng.uniform(-0.25, 0.25, size=(n_src, 3))
    return np.ascontiguousarray(pos)


@dataclass
class Workload:
    """One synthetic ART problem: grid, opacity parameters and sources."""

    name: str
    nx: int
    ny: int
    nz: int
    n_H: np.ndarray            # float32 [nx*ny*nz]
    x_n: np.ndarray            # float32 [nx*ny*nz]
    src_pos: np.ndarray        # float64 [n_src, 3]
    src_lum: np.ndarray        # float32 [n_src, n_bins]
    s_H: float
    s_d: float
    n_bins: int
    level0: int = 2
    level_max: int = 13
    phi_c: float = 4.0
    tau_term: float = TAU_TERM_1E10
    deterministic: bool = False
    w: np.ndarray | None = None   # float32 [N]     d loss / d rate
    v: np.ndarray | None = None   # float32 [3, N]  d loss / d force (SoA)
    extra: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_src(self) -> int:
        return int(self.src_pos.shape[0])

    def params(self) -> dict:
        return dict(level0=self.level0, level_max=self.level_max, phi_c=self.phi_c,
                    tau_term=self.tau_term, s_H=self.s_H, s_d=self.s_d,
                    n_bins=self.n_bins)

    def subset(self, idx) -> "Workload":
        """Same grid, only the sources listed in ``idx``."""
        idx = np.asarray(idx, dtype=np.int64)
        return Workload(name=f"{self.name}[{len(idx)} src]", nx=self.nx, ny=self.ny,
                        nz=self.nz, n_H=self.n_H, x_n=self.x_n,
                        src_pos=np.ascontiguousarray(self.src_pos[idx]),
                        src_lum=np.ascontiguousarray(self.src_lum[idx]),
                        s_H=self.s_H, s_d=self.s_d, n_bins=self.n_bins,
                        level0=self.level0, level_max=self.level_max,
                        phi_c=self.phi_c, tau_term=self.tau_term,
                        deterministic=self.deterministic, w=self.w, v=self.v)


def uniform_workload(n: int, src_pos, lum=1.0, s_H=0.05, s_d=0.0, n_H=1.0, x_n=1.0,
                     n_bins=1, **kw) -> Workload:
    """Uniform medium with sources at the given positions (lum per source and bin)."""
    src_pos = np.ascontiguousarray(np.atleast_2d(np.asarray(src_pos, dtype=np.float64)))
    ns = src_pos.shape[0]
    lum = np.broadcast_to(np.asarray(lum, dtype=np.float32).reshape(-1, 1)
                          if np.ndim(lum) else np.float32(lum), (ns, n_bins))
    return Workload(name=f"uniform{n}", nx=n, ny=n, nz=n,
                    n_H=np.full(n ** 3, n_H, dtype=np.float32),
                    x_n=np.full(n ** 3, x_n, dtype=np.float32),
                    src_pos=src_pos, src_lum=np.array(lum, dtype=np.float32),
                    s_H=s_H, s_d=s_d, n_bins=n_bins, **kw)


def config(c: int, n_src: int | None = None, n: int | None = None) -> Workload:
    """The five benchmark/parity workloads (1-based index).

    ``n_src`` and ``n`` optionally shrink a workload (same recipe) for quick tests.
    """
    if c == 1:
        return uniform_workload(32, [16.3, 16.1, 15.8], lum=1.0, s_H=0.05, s_d=0.0,
                                n_bins=1)._renamed("c1: 32^3 uniform, 1 source")
    if c == 2:
        nn = n or 128
        n_H = lognormal_density(nn, 1.5, 2000)
        idx = int(np.argmax(n_H))
        pos = np.array([[idx % nn, (idx // nn) % nn, idx // (nn * nn)]], dtype=np.float64) + 0.5
        return Workload(name=f"c2: {nn}^3 lognormal std1.5, source at density max",
                        nx=nn, ny=nn, nz=nn, n_H=n_H,
                        x_n=np.ones(nn ** 3, dtype=np.float32), src_pos=pos,
                        src_lum=np.ones((1, 1), dtype=np.float32),
                        s_H=0.02, s_d=0.002, n_bins=1)
    if c == 3:
        nn = n or 256
        ns = n_src or 64
        n_H = lognormal_density(nn, 1.5, 3000)
        rng = np.random.default_rng(3002)
        pos = sample_sources(n_H, nn, ns, rng)
        li = 10.0 ** rng.uniform(0.0, 3.0, size=ns)
        lum = np.stack([li, 1.5 * li], axis=1).astype(np.float32)
        return Workload(name=f"c3: {nn}^3 lognormal std1.5, {ns} sources, 2 bins",
                        nx=nn, ny=nn, nz=nn, n_H=n_H,
                        x_n=np.ones(nn ** 3, dtype=np.float32), src_pos=pos, src_lum=lum,
                        s_H=0.02, s_d=0.002, n_bins=2)
    if c == 4:
        nn = n or 128
        ns = n_src or 8
        n_H = lognormal_density(nn, 1.5, 4000)
        x_n = sigmoid_fraction(nn, 2.0, 4001)
        rng = np.random.default_rng(4002)
        pos = sample_sources(n_H, nn, ns, rng)
        li = 10.0 ** rng.uniform(0.0, 3.0, size=ns)
        lum = np.stack([li, 1.5 * li], axis=1).astype(np.float32)
        w, v = random_adjoint_weights(nn ** 3, seed=4003)
        return Workload(name=f"c4: {nn}^3 lognormal, sigmoid x_n, {ns} sources, adjoint",
                        nx=nn, ny=nn, nz=nn, n_H=n_H, x_n=x_n, src_pos=pos, src_lum=lum,
                        s_H=0.02, s_d=0.002, n_bins=2, w=w, v=v)
    if c == 5:
        nn = n or 512
        ns = n_src or 1024
        n_H = lognormal_density(nn, 2.0, 5000)
        rng = np.random.default_rng(5002)
        pos = sample_sources(n_H, nn, ns, rng)
        u = rng.uniform(0.0, 1.0, size=ns)
        li = 1.0 / (1.0 - u * (1.0 - 1.0e-4))
        lum = np.stack([li, 1.5 * li], axis=1).astype(np.float32)
        w, v = random_adjoint_weights(nn ** 3, seed=5003)
        return Workload(name=f"c5: {nn}^3 lognormal std2, {ns} sources, 2 bins, deterministic",
                        nx=nn, ny=nn, nz=nn, n_H=n_H,
                        x_n=np.ones(nn ** 3, dtype=np.float32), src_pos=pos, src_lum=lum,
                        s_H=0.02, s_d=0.002, n_bins=2, deterministic=True, w=w, v=v)
    raise ValueError(f"unknown workload {c}")


def _renamed(self: Workload, name: str) -> Workload:
    self.name = name
    return self


Workload._renamed = _renamed  # type: ignore[attr-defined]


def random_adjoint_weights(n_cells: int, seed: int):
    """w ~ U[0,1) per cell and v ~ U[0,1)^3 per cell (SoA), drawn as float32."""
    rw = np.random.default_rng(seed)
    w = rw.random(n_cells, dtype=np.float32)
    v = rw.random((3, n_cells), dtype=np.float32)
    return w, np.ascontiguousarray(v)


# Physical constants of the HII-region tests (paper Sec. 3.3.1): cgs.
PC_CM = 3.0857e18
SIGMA_H_CM2 = 6.3e-18        # frequency-averaged H cross section
ALPHA_B_RTYPE = 3.02e-13     # case-B recombination coefficient of the R-type test, cm^3/s
Q_RTYPE = 1.0e49             # ionizing photons per second
N_H_RTYPE = 1.0e2            # cm^-3


@dataclass
class IonProblem:
    """A workload plus the code units of the ionization subcycle.

    Code units: the cell is the unit of length, the background density n0 the
    unit of density, the recombination time t_rec = 1 / (alpha_B n0) the unit of
    time, and the source's photon rate Q the unit of luminosity.  Then
    alpha_B = 1, the optical depth per cell length is s_H n_H with
    s_H = sigma_H dx n0, and Gamma = gamma_scale J_0 with
    gamma_scale = sigma_H Q t_rec / dx^2."""

    wl: Workload
    alpha_B: float
    gamma_scale: float
    R_S: float          # dust-free Stromgren radius in cells
    t_rec: float = 1.0


def rtype_problem(n: int = 128, box_over_rs: float = 2.4) -> IonProblem:
    """R-type ionization front (paper Sec. 3.3.1): uniform neutral hydrogen of
    n_H = 100 cm^-3 around a source of Q = 1e49 photons/s at the box centre, box
    side 2.4 R_S, no dust, one ionizing bin, x_n = 1 at t = 0."""
    r_s_cm = (3.0 * Q_RTYPE / (4.0 * np.pi * ALPHA_B_RTYPE * N_H_RTYPE ** 2)) ** (1.0 / 3.0)
    dx = box_over_rs * r_s_cm / n
    t_rec = 1.0 / (ALPHA_B_RTYPE * N_H_RTYPE)
    s_H = SIGMA_H_CM2 * dx * N_H_RTYPE
    gamma_scale = SIGMA_H_CM2 * Q_RTYPE * t_rec / dx ** 2
    N = n ** 3
    wl = Workload(name=f"R-type front {n}^3", nx=n, ny=n, nz=n,
                  n_H=np.ones(N, dtype=np.float32), x_n=np.ones(N, dtype=np.float32),
                  src_pos=np.array([[n / 2.0, n / 2.0, n / 2.0]]),
                  src_lum=np.ones((1, 1), dtype=np.float32), s_H=float(s_H), s_d=0.0, n_bins=1)
    return IonProblem(wl=wl, alpha_B=1.0, gamma_scale=float(gamma_scale), R_S=r_s_cm / dx)
