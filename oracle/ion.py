"""FP64 CPU oracle of the ionization subcycle around the sweep (paper Sec. 2.3).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the smoke check, never by the
product path.  It imports nothing from the HIP package; the radiation field of a
substep comes from the FP64 sweep oracle (``oracle.trace``).

What is computed (paper Sec. 2.3, on-the-spot approximation, no collisional
ionization, one ionizing bin):

* the neutral fraction obeys  dx_n/dt = alpha_B n_e (1 - x_n) - x_n Gamma   (Eq. e:xn)
  with n_e = n_HII = n_H (1 - x_n), R = alpha_B n_e n_HII and I = Gamma n_HI;
* Gamma = I / n_HI is the photoionization rate per neutral atom.  With the sweep's
  J_0 (sum over rays of L_in dr phi(dtau) in a cell), I = s_H n_HI J_0 / V_cell, so
  Gamma = gamma_scale J_0 with gamma_scale = s_H / V_cell in the caller's units
  (Eq. e:photrate2);
* Method A: the exact solution for Gamma and alpha_B held fixed over the substep
  (Eq. e:xn2), and the Gamma = 0 solution for shielded cells;
* Method B: the solution with n_e also held at its start value (Eq. e:xn3),
  x_n = x_eq0 + (x_0 - x_eq0) exp(-dt / t_ir), t_ir = 1 / (Gamma + alpha_B n_e),
  x_eq0 = alpha_B n_e t_ir -- the method the paper adopts;
* the substep  dt_ss = C min over cells of n_H / |I - R|   (Eq. e:dtss);
* the subcycle: sweep -> Gamma -> dt_ss -> Method B update of x_n, repeated until
  the hydro step is used up (the loop of Sec. 2.3, without the hydro update).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def gamma_from_J(J0, gamma_scale: float) -> np.ndarray:
    """Photoionization rate per neutral atom: Gamma = gamma_scale J_0 (Eq. e:photrate2)."""
    return float(gamma_scale) * np.asarray(J0, dtype=np.float64)


def source_terms(n_H, x_n, Gamma, alpha_B: float):
    """(I, R): ionizations and recombinations per unit volume and time (Sec. 2.3)."""
    n_H = np.asarray(n_H, dtype=np.float64)
    x_n = np.asarray(x_n, dtype=np.float64)
    n_e = n_H * (1.0 - x_n)
    I = np.asarray(Gamma, dtype=np.float64) * n_H * x_n
    R = float(alpha_B) * n_e * n_e
    return I, R


def substep_dt(n_H, x_n, Gamma, alpha_B: float, C: float, transparent=None) -> float:
    """dt_ss = C min(n_H / |I - R|) over cells with gas (Eq. e:dtss); +inf if no cell
    changes.  Cells flagged in ``transparent`` (sink control volumes, Sec. 4.1: the
    radiation ignores their gas, whose state the subcycle leaves alone) set no
    limit."""
    n_H = np.asarray(n_H, dtype=np.float64)
    I, R = source_terms(n_H, x_n, Gamma, alpha_B)
    d = np.abs(I - R)
    ok = (n_H > 0.0) & (d > 0.0)
    if transparent is not None:
        ok &= np.asarray(transparent).reshape(n_H.shape) == 0
    if not ok.any():
        return float("inf")
    return float(C) * float(np.min(n_H[ok] / d[ok]))


def method_b(x0, n_H, Gamma, alpha_B: float, dt: float, transparent=None) -> np.ndarray:
    """Eq. e:xn3: relaxation towards x_eq0 = alpha_B n_e / (Gamma + alpha_B n_e) on
    the time scale t_ir = 1 / (Gamma + alpha_B n_e), with n_e = n_H (1 - x_0).
    Cells flagged in ``transparent`` (sink control volumes) keep x_0."""
    x0 = np.asarray(x0, dtype=np.float64)
    n_e = np.asarray(n_H, dtype=np.float64) * (1.0 - x0)
    a = float(alpha_B) * n_e
    s = np.asarray(Gamma, dtype=np.float64) + a
    out = x0.copy()
    m = s > 0.0
    if transparent is not None:
        m &= np.asarray(transparent).reshape(x0.shape) == 0
    x_eq = np.where(m, a / np.where(m, s, 1.0), 0.0)
    out[m] = x_eq[m] + (x0[m] - x_eq[m]) * np.exp(-float(dt) * s[m])
    return out


def x_eq_exact(n_H, Gamma, alpha_B: float) -> np.ndarray:
    """Equilibrium of Eq. e:xn for fixed Gamma: the root of alpha_B n_H (1 - x)^2 = x Gamma
    in [0, 1], written without cancellation (Sec. 2.3)."""
    a = float(alpha_B) * np.asarray(n_H, dtype=np.float64)
    G = np.asarray(Gamma, dtype=np.float64)
    return 2.0 * a / (G + 2.0 * a + np.sqrt(G * G + 4.0 * a * G))


def method_a(x0, n_H, Gamma, alpha_B: float, dt: float) -> np.ndarray:
    """Eq. e:xn2 (exact for Gamma, alpha_B fixed over dt); the Gamma = 0 solution
    x = (x_0 + (1 - x_0) a t) / (1 + (1 - x_0) a t), a = alpha_B n_H, for shielded cells."""
    x0 = np.asarray(x0, dtype=np.float64)
    n_H = np.broadcast_to(np.asarray(n_H, dtype=np.float64), x0.shape)
    G = np.broadcast_to(np.asarray(Gamma, dtype=np.float64), x0.shape)
    a = float(alpha_B) * n_H
    out = np.empty_like(x0)
    shield = G <= 0.0
    at = a[shield] * float(dt)
    out[shield] = (x0[shield] + (1.0 - x0[shield]) * at) / (1.0 + (1.0 - x0[shield]) * at)
    m = ~shield
    xe = x_eq_exact(n_H[m], G[m], alpha_B)
    xp = 1.0 / xe
    K = np.exp(-(xp - xe) * float(dt) * a[m])
    out[m] = xe + (xp - xe) * (x0[m] - xe) * K / ((xp - x0[m]) + (x0[m] - xe) * K)
    return out


def rhs(x, n_H, Gamma, alpha_B: float):
    """Right-hand side of Eq. e:xn: alpha_B n_e (1 - x_n) - x_n Gamma."""
    n_e = np.asarray(n_H, dtype=np.float64) * (1.0 - x)
    return float(alpha_B) * n_e * (1.0 - x) - x * Gamma


@dataclass
class SubcycleResult:
    x_n: np.ndarray          # final neutral fraction [N]
    t: float                 # time reached
    dts: list                # substep sizes
    impulse: np.ndarray      # sum over substeps of force * dt, [3, N]


def subcycle(nx, ny, nz, n_H, x_n, src_pos, src_lum, *, alpha_B, gamma_scale, C, t_end,
             max_substeps=100000, trace_kw=None, on_substep=None, transparent=None) -> SubcycleResult:
    """The radiation subcycle of one hydro step (Sec. 2.3 without hydro): repeat
    {FP64 sweep of the current x_n; Gamma = gamma_scale J_0; dt = min(dt_ss, t_end - t);
    x_n <- Method B; impulse += force dt} until t = t_end.  ``on_substep(k, t, x_n)``
    is called after every substep.  ``transparent``: sink control volumes, traced
    without gas, with their x_n kept and no substep limit from them."""
    from oracle import oracle as O
    kw = dict(trace_kw or {})
    if transparent is not None:
        kw["transparent"] = transparent
    x = np.asarray(x_n, dtype=np.float64).reshape(-1).copy()
    nH = np.asarray(n_H, dtype=np.float64).reshape(-1)
    imp = np.zeros((3, x.size))
    t = 0.0
    dts = []
    for k in range(max_substeps):
        if t >= t_end:
            break
        res = O.trace(nx, ny, nz, nH, x, src_pos, src_lum, **kw)
        G = gamma_from_J(res.J[0], gamma_scale)
        dt = min(substep_dt(nH, x, G, alpha_B, C, transparent), t_end - t)
        x = method_b(x, nH, G, alpha_B, dt, transparent)
        imp += res.force * dt
        t = t + dt if t + dt < t_end else t_end
        dts.append(dt)
        if on_substep is not None:
            on_substep(k, t, x)
    return SubcycleResult(x_n=x, t=t, dts=dts, impulse=imp)
