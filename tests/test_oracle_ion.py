"""Pins of the ionization-subcycle oracle (paper Sec. 2.3 and the Appendix).

Method A (Eq. e:xn2) and Method B (Eq. e:xn3) are checked against numerical
integration of the ODEs they solve; the substep rule (Eq. e:dtss) against the
bound it is designed to give; the subcycle against the paper's one-cell test and
the analytic R-type front (Eq. e:Rtype)."""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import ion as X
from paper_1711_06277_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def golden(key):
    with open(GOLDEN) as f:
        return json.load(f)[key]


def ode(x0, a, G, t, n_e_fixed=None):
    """Integrate dx/dt = a (1 - x)^2 - G x (Eq. e:xn with a = alpha_B n_H), or, with
    n_e_fixed, dx/dt = alpha n_e (1 - x) - G x, to high accuracy."""
    if n_e_fixed is None:
        f = lambda _t, x: a * (1 - x) ** 2 - G * x
    else:
        f = lambda _t, x: a * n_e_fixed * (1 - x) - G * x
    s = solve_ivp(f, (0.0, t), [x0], method="Radau", rtol=1e-12, atol=1e-15)
    return float(s.y[0, -1])


CASES = [(x0, a, G, t) for x0 in (1.0, 0.5, 1e-3) for a in (1.0, 0.1)
         for G in (0.0, 0.3, 14.0, 1e3) for t in (0.01, 0.5, 3.0)]


@pytest.mark.parametrize("x0,a,G,t", CASES)
def test_method_a_solves_the_ode(x0, a, G, t):
    """Eq. e:xn2 (and the Gamma = 0 solution) is the exact solution of Eq. e:xn."""
    got = X.method_a(np.array([x0]), 1.0, G, a, t)[0]
    assert got == pytest.approx(ode(x0, a, G, t), rel=1e-8, abs=1e-13)


@pytest.mark.parametrize("x0,a,G,t", CASES)
def test_method_b_solves_the_frozen_electron_ode(x0, a, G, t):
    """Eq. e:xn3 is the exact solution when n_e is held at n_H (1 - x_0)."""
    got = X.method_b(np.array([x0]), 1.0, G, a, t)[0]
    assert got == pytest.approx(ode(x0, a, G, t, n_e_fixed=1.0 - x0), rel=1e-8, abs=1e-13)


def test_method_b_properties():
    """x_n stays between x_0 and x_eq0 (the robustness the paper cites); dt = 0 is the
    identity; a neutral, unirradiated cell stays neutral."""
    rng = np.random.default_rng(11)
    n = 2000
    x0 = rng.uniform(0, 1, n)
    nH = 10 ** rng.uniform(-2, 3, n)
    G = np.where(rng.uniform(0, 1, n) < 0.2, 0.0, 10 ** rng.uniform(-3, 4, n))
    dt = 10 ** rng.uniform(-4, 1, n)
    alpha = 0.7
    xb = np.array([X.method_b(x0[i:i + 1], nH[i], G[i], alpha, dt[i])[0] for i in range(n)])
    n_e = nH * (1 - x0)
    xeq = alpha * n_e / (G + alpha * n_e)
    lo, hi = np.minimum(x0, xeq), np.maximum(x0, xeq)
    assert np.all(xb >= lo - 1e-15) and np.all(xb <= hi + 1e-15)
    assert np.allclose(X.method_b(x0, nH, G, alpha, 0.0), x0, rtol=0, atol=2.3e-16)  # x_eq + (x0 - x_eq)
    assert X.method_b(np.array([1.0]), 5.0, 0.0, alpha, 3.0)[0] == 1.0


def test_method_b_is_first_order_consistent_with_the_exact_solution():
    """B differs from A only through the frozen n_e, an O(dt^2) effect: halving dt
    divides the one-step difference by ~4 (a wrong rate term would leave O(dt))."""
    x0, a, G = 0.4, 1.0, 2.0
    d = [abs(X.method_b(np.array([x0]), 1.0, G, a, h)[0] - X.method_a(np.array([x0]), 1.0, G, a, h)[0])
         for h in (1e-2, 5e-3, 2.5e-3)]
    assert 3.6 < d[0] / d[1] < 4.4 and 3.6 < d[1] / d[2] < 4.4


def test_substep_bounds_the_change_of_x():
    """With dt = C min(n_H / |I - R|) (Eq. e:dtss), Method B changes x_n by at most C
    in any cell (exponential relaxation moves less than its initial slope times dt)."""
    rng = np.random.default_rng(5)
    n = 50000
    x0 = rng.uniform(0, 1, n)
    nH = 10 ** rng.uniform(-1, 2, n)
    G = 10 ** rng.uniform(-2, 3, n)
    for C in (0.1, 0.5):
        dt = X.substep_dt(nH, x0, G, 1.3, C)
        assert np.max(np.abs(X.method_b(x0, nH, G, 1.3, dt) - x0)) <= C * (1 + 1e-12)
    dt1 = X.substep_dt(nH, x0, G, 1.3, 0.1)
    assert X.substep_dt(nH, x0, G, 1.3, 0.2) == pytest.approx(2 * dt1, rel=1e-15)
    # cells without gas or in exact balance impose nothing
    nH2 = np.concatenate([nH, [0.0]])
    assert X.substep_dt(nH2, np.concatenate([x0, [0.5]]), np.concatenate([G, [1.0]]), 1.3, 0.1) == dt1
    assert X.substep_dt([1.0], [1.0], [0.0], 1.0, 0.1) == math.inf


def one_cell_gamma(g, alpha):
    """Appendix: the cell's own absorption sets Gamma(x_n)."""
    dx = g["dx_pc"] * I.PC_CM
    nH = g["tau_0"] / (g["sigma_H"] * dx)
    G0 = g["Q_i"] / (nH * dx ** 3)
    tau0 = nH * g["sigma_H"] * dx
    gam = lambda x: G0 * (-np.expm1(-tau0 * x)) / x if x > 0 else G0 * tau0
    return nH, G0, gam


def run_one_cell(method, C, t_end, nH, gam, alpha):
    x, t, traj = 1.0, 0.0, []
    while t < t_end:
        G = gam(x)
        dt = min(X.substep_dt([nH], [x], [G], alpha, C), t_end - t)
        x = float(method(np.array([x]), nH, G, alpha, dt)[0])
        t += dt
        traj.append((t, x))
    return traj


def test_one_cell_appendix():
    """Appendix numbers: Gamma_0 ~ 14 alpha_B n_H; equilibrium x_eq ~ 1.8e-5 for
    t Gamma_0 >~ 1; Methods A and B with C = 0.001 nearly identical, and close to each
    other even for C as large as 1."""
    g = golden("one_cell")
    alpha = 3.03e-13  # alpha_B at T = 8000 K (Sec. 2.3)
    nH, G0, gam = one_cell_gamma(g, alpha)
    assert G0 / (alpha * nH) == pytest.approx(g["gamma0_over_alpha_nH"], rel=0.03)
    t_end = 5.0 / G0
    ref_b = run_one_cell(X.method_b, 0.001, t_end, nH, gam, alpha)
    ref_a = run_one_cell(X.method_a, 0.001, t_end, nH, gam, alpha)
    assert ref_b[-1][1] == pytest.approx(g["x_eq"], rel=0.06)
    # the equilibrium of alpha n (1 - x)^2 = x Gamma(x), solved by bisection
    lo, hi = 1e-8, 1e-3
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if alpha * nH * (1 - mid) ** 2 - mid * gam(mid) > 0:
            lo = mid
        else:
            hi = mid
    assert ref_b[-1][1] == pytest.approx(lo, rel=1e-3)
    ta, xa = np.array(ref_a).T
    tb, xb = np.array(ref_b).T
    assert np.max(np.abs(np.interp(tb, ta, xa) - xb)) < 2e-3
    # A and B stay close even at C = 1, and the error of B against the C = 0.001
    # solution shrinks with C (Gamma is frozen over a substep: first order in C)
    err = {}
    for C in (1.0, 0.1, 0.01):
        cb = np.array(run_one_cell(X.method_b, C, t_end, nH, gam, alpha))
        ca = np.array(run_one_cell(X.method_a, C, t_end, nH, gam, alpha))
        assert np.max(np.abs(np.interp(cb[:, 0], ca[:, 0], ca[:, 1]) - cb[:, 1])) < 0.01
        err[C] = np.max(np.abs(np.interp(cb[:, 0], tb, xb) - cb[:, 1]))
    assert err[0.01] < err[0.1] / 3 < err[1.0] / 3


def rtype_radius(x, shape):
    """Radius of the sphere with the volume of the cells with x_n < 0.5."""
    return (3.0 * float((x < 0.5).sum()) / (4.0 * math.pi)) ** (1.0 / 3.0)


def test_rtype_front_oracle():
    """Sec. 3.3.1: with Method B and C = 0.1 the ionization front follows
    r_IF = R_S (1 - exp(-t/t_rec))^(1/3) within ~5%, better at late times.
    32^3 cells (the paper finds 64^3-256^3 within 2% of each other)."""
    g = golden("r_type")
    p = I.rtype_problem(32)
    wl = p.wl
    marks = {0.25: None, 0.5: None, 1.0: None, 2.0: None, 4.0: None}

    def cb(k, t, x):
        for m in marks:
            if marks[m] is None and t >= m - 1e-12:
                marks[m] = rtype_radius(x, (wl.nx, wl.ny, wl.nz))

    res = X.subcycle(wl.nx, wl.ny, wl.nz, wl.n_H, wl.x_n, wl.src_pos, wl.src_lum,
                     alpha_B=p.alpha_B, gamma_scale=p.gamma_scale, C=0.1, t_end=4.0,
                     trace_kw=dict(s_H=wl.s_H, s_d=0.0, n_bins=1), on_substep=cb)
    assert res.t == 4.0
    for m, r in marks.items():
        ref = p.R_S * (1.0 - math.exp(-m)) ** (1.0 / 3.0)
        assert abs(r / ref - 1.0) < g["front_rel_err_C0.1"], (m, r, ref)
    assert abs(marks[4.0] / (p.R_S * (1 - math.exp(-4.0)) ** (1 / 3)) - 1) < 0.01
    # the momentum given to the gas points away from the source
    c = np.argmax(np.linalg.norm(res.impulse, axis=0))
    k, rem = divmod(int(c), wl.nx * wl.ny)
    j, i = divmod(rem, wl.nx)
    d = np.array([i + 0.5, j + 0.5, k + 0.5]) - wl.src_pos[0]
    assert np.dot(d, res.impulse[:, c]) > 0
