"""Uniform random rotations for the per-step rotation of the ray directions
(paper Sec. 2.1: the injection directions are rotated at random every time step).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; it imports nothing from the HIP
package.  The rotation is drawn from three uniform numbers u in [0, 1) with the
quaternion construction of Shoemake (Graphics Gems III, 1992), which is uniform
(Haar) on SO(3): q = (sqrt(1-u1) sin 2 pi u2, sqrt(1-u1) cos 2 pi u2,
sqrt(u1) sin 2 pi u3, sqrt(u1) cos 2 pi u3) = (x, y, z, w), and the matrix of the
unit quaternion w + x i + y j + z k.  Written here in FP64 with numpy.
"""
from __future__ import annotations

import numpy as np


def quaternion(u) -> np.ndarray:
    """(x, y, z, w) of the uniform random unit quaternion for u = (u1, u2, u3)."""
    u1, u2, u3 = (float(t) for t in u)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    return np.array([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                     b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)])


def matrix(q) -> np.ndarray:
    """Row-major 3x3 rotation of the unit quaternion q = (x, y, z, w): v -> q v q*."""
    x, y, z, w = (float(t) for t in q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def uniform_rotation(u) -> np.ndarray:
    """The rotation matrix drawn from u = (u1, u2, u3) in [0, 1)^3."""
    return matrix(quaternion(u))
