"""Pins of the random rotation of the ray directions (paper Sec. 2.1: the
injection directions are rotated at random every time step; Sec. 3.2: averaging
ten orientations at m_ray = 4 reaches about the accuracy of m_ray = 10)."""
import math

import numpy as np
import pytest

from oracle import rotation as R
from paper_1711_06277_amd import inputs as I
from tests.test_oracle_physics import cell_centres, cell_integral


def test_shoemake_special_cases():
    """u1 = 1 puts all weight on (z, w): u3 = 0 is the identity, u3 = 1/4 the half
    turn about z; u1 = 0, u2 = 1/4 is the half turn about x."""
    assert np.allclose(R.uniform_rotation([1.0, 0.0, 0.0]), np.eye(3), atol=1e-15)
    assert np.allclose(R.uniform_rotation([1.0, 0.0, 0.25]), np.diag([-1.0, -1.0, 1.0]), atol=1e-15)
    assert np.allclose(R.uniform_rotation([0.0, 0.25, 0.7]), np.diag([1.0, -1.0, -1.0]), atol=1e-15)


def test_rotations_are_proper_and_haar_uniform():
    """Every draw is orthonormal with determinant +1; over many seeded draws the
    rotated z axis is uniform on the sphere (mean 0, second moments 1/3), the mean
    trace is 0 and P(angle <= pi/2) = (pi/2 - 1)/pi, as for the Haar measure."""
    rng = np.random.default_rng(21)
    n = 20000
    Ms = np.array([R.uniform_rotation(u) for u in rng.uniform(0.0, 1.0, (n, 3))])
    eye = np.einsum("nij,nkj->nik", Ms, Ms)
    assert np.abs(eye - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(Ms) - 1.0).max() < 1e-13
    z = Ms[:, :, 2]
    assert np.abs(z.mean(axis=0)).max() < 0.02
    assert np.abs((z * z).mean(axis=0) - 1.0 / 3.0).max() < 0.01
    tr = np.trace(Ms, axis1=1, axis2=2)
    assert abs(tr.mean()) < 0.03
    ang = np.arccos(np.clip((tr - 1.0) / 2.0, -1.0, 1.0))
    assert abs((ang <= math.pi / 2).mean() - (math.pi / 2 - 1.0) / math.pi) < 0.01


def test_rotation_averaging_in_vacuum(oracle):
    """Sec. 3.2: the mean of ten randomly oriented traces at (m_ray, l0) = (4, 4) has
    a median error near that of one trace at m_ray = 10, against the exact cell
    average of L / (4 pi r^2)."""
    n, xs = 32, np.array([16.3, 16.1, 15.8])
    exact = cell_integral((n, n, n), xs)
    r = np.linalg.norm(cell_centres(n, n, n) - xs, axis=1)
    far = r > 3.0

    def J(phi_c, rot=None):
        wl = I.uniform_workload(n, xs, lum=1.0, s_H=0.0, s_d=0.0, n_bins=1, phi_c=phi_c, level0=4)
        return oracle.trace_workload(wl, rot=rot).J[0]

    med = lambda j: float(np.median(np.abs(j / exact - 1.0)[far]))
    m4, m10 = med(J(4.0)), med(J(10.0))
    rng = np.random.default_rng(12)
    avg = sum(J(4.0, R.uniform_rotation(rng.uniform(0.0, 1.0, 3))) for _ in range(10)) / 10.0
    mr = med(avg)
    assert mr < m4 / 2.5
    assert mr < 1.5 * m10
