"""Pins of the oracle's HEALPix nested pixel centres (Gorski et al. 2005).

The paper takes its ray directions from the HEALPix nested scheme with
N_ray(l) = 12*4^l equal-area pixels and children at one level higher
(Sec. 2.1, Sec. 2.2 Step-1 ordering).  These tests check the oracle's
pix2vec_nest against the ring-scheme definition of the pixel centres and
the nested-hierarchy property, both written out here independently.
"""
import math

import numpy as np
import pytest


def ring_scheme_centres(level):
    """Pixel centres (z, phi) from the HEALPix ring-scheme formulas."""
    ns = 2 ** level
    out = []
    for i in range(1, 4 * ns):
        if i < ns:
            z = 1.0 - i * i / (3.0 * ns * ns)
            out += [(z, math.pi / (2 * i) * (j - 0.5)) for j in range(1, 4 * i + 1)]
        elif i <= 3 * ns:
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns)
            s = (i - ns + 1) % 2
            out += [(z, math.pi / (2 * ns) * (j - s / 2.0)) for j in range(1, 4 * ns + 1)]
        else:
            ip = 4 * ns - i
            z = -(1.0 - ip * ip / (3.0 * ns * ns))
            out += [(z, math.pi / (2 * ip) * (j - 0.5)) for j in range(1, 4 * ip + 1)]
    return out


def _vec(z, phi):
    st = math.sqrt(max(0.0, (1 - z) * (1 + z)))
    return np.array([st * math.cos(phi), st * math.sin(phi), z])


def nested_vectors(O, level):
    return np.array([O.pix2vec_nest(level, p) for p in range(12 * 4 ** level)])


def test_base_pixels(oracle):
    """nside = 1: four pixels at z = 2/3 and phi = pi/4 + k pi/2, four on the
    equator at phi = k pi/2, four at z = -2/3."""
    got = [oracle.pix2ang_nest(0, p) for p in range(12)]
    for f, (z, phi) in enumerate(got):
        if f < 4:
            assert z == pytest.approx(2 / 3, abs=1e-15)
            assert phi == pytest.approx(math.pi / 4 + f * math.pi / 2, abs=1e-14)
        elif f < 8:
            assert z == pytest.approx(0.0, abs=1e-15)
            assert phi == pytest.approx((f - 4) * math.pi / 2, abs=1e-14)
        else:
            assert z == pytest.approx(-2 / 3, abs=1e-15)
            assert phi == pytest.approx(math.pi / 4 + (f - 8) * math.pi / 2, abs=1e-14)


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_nested_centres_equal_ring_centres(oracle, level):
    """The nested numbering is a permutation of the ring-scheme pixel centres."""
    ring = np.array([_vec(z, p) for z, p in ring_scheme_centres(level)])
    nest = nested_vectors(oracle, level)
    assert ring.shape == nest.shape == (12 * 4 ** level, 3)
    # match every nested centre to its nearest ring centre: must be a bijection
    d = ((nest[:, None, :] - ring[None, :, :]) ** 2).sum(-1)
    nearest = d.argmin(1)
    assert np.unique(nearest).size == nest.shape[0]
    assert np.sqrt(d.min(1)).max() < 1e-12


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_children_nearest_to_parent(oracle, level):
    """Children 4p..4p+3 at level l+1 lie inside parent p: of all level-l
    centres, p's is the nearest one to each child centre."""
    par = nested_vectors(oracle, level)
    chi = nested_vectors(oracle, level + 1)
    dots = chi @ par.T
    assert np.array_equal(dots.argmax(1), np.arange(chi.shape[0]) // 4)


@pytest.mark.parametrize("level", [0, 2, 4])
def test_unit_and_balanced(oracle, level):
    v = nested_vectors(oracle, level)
    assert np.abs(np.linalg.norm(v, axis=1) - 1).max() < 1e-14
    # antipodal symmetry of the pixelisation: the centres sum to zero
    assert np.abs(v.sum(0)).max() < 1e-10


def test_equal_area_neighbour_spacing(oracle):
    """Equal-area pixels: nearest-neighbour angular spacing is close to
    sqrt(Omega) with Omega = 4 pi / N_pix everywhere on the sphere."""
    level = 3
    v = nested_vectors(oracle, level)
    ang = np.arccos(np.clip(v @ v.T, -1, 1))
    np.fill_diagonal(ang, 10)
    nn = ang.min(1)
    omega = 4 * math.pi / v.shape[0]
    assert 0.6 < nn.min() / math.sqrt(omega) and nn.max() / math.sqrt(omega) < 1.3


def test_r_max_definition(oracle):
    """r_max(l) = sqrt(3/(pi m_ray)) 2^l solves (dx/r)^2 = m_ray * 4pi/(12*4^l)."""
    for m_ray in (2.0, 4.0, 10.0):
        for level in range(0, 12):
            r = oracle.r_max(m_ray, level)
            omega = 4 * math.pi / (12 * 4 ** level)
            assert (1.0 / r) ** 2 == pytest.approx(m_ray * omega, rel=1e-14)
