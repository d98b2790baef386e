"""Real spherical harmonics up to degree 3, FP64 (directional emission E_i(omega)).

Parity: pinned (tests compare the basis with SciPy's complex spherical
harmonics and check orthonormality by quadrature).

The paper gives each Gaussian a directional emission E_i(omega) (Sec. 3)
stored as SH coefficients (degree 1 for reconstruction, inherited for
refinement, Sec. 5).  Reading: the orthonormal real basis
    Y_l^m = sqrt(2) Im Y_l^|m|  (m < 0),  Y_l^0,  sqrt(2) Re Y_l^m  (m > 0)
built from the complex harmonics *without* the Condon-Shortley phase, so that
degree 1 is sqrt(3/(4 pi)) * (y, z, x).  Coefficient (l, m) sits at index
l*l + l + m.  The emitted colour is max(0, sum_lm c_lm Y_lm(d) + 1/2) per
channel, d = unit vector from the camera centre to the Gaussian's mean.
"""
import math

import numpy as np


def basis(degree, dirs):
    """[P, (degree+1)^2] real SH values at unit directions dirs [P, 3]."""
    d = np.asarray(dirs, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    out = [np.full_like(x, 0.5 * math.sqrt(1.0 / pi))]
    if degree >= 1:
        c1 = math.sqrt(3.0 / (4.0 * pi))
        out += [c1 * y, c1 * z, c1 * x]
    if degree >= 2:
        out += [0.5 * math.sqrt(15.0 / pi) * x * y,
                0.5 * math.sqrt(15.0 / pi) * y * z,
                0.25 * math.sqrt(5.0 / pi) * (3.0 * z * z - 1.0),
                0.5 * math.sqrt(15.0 / pi) * x * z,
                0.25 * math.sqrt(15.0 / pi) * (x * x - y * y)]
    if degree >= 3:
        out += [0.25 * math.sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y),
                0.5 * math.sqrt(105.0 / pi) * x * y * z,
                0.25 * math.sqrt(21.0 / (2.0 * pi)) * y * (5.0 * z * z - 1.0),
                0.25 * math.sqrt(7.0 / pi) * z * (5.0 * z * z - 3.0),
                0.25 * math.sqrt(21.0 / (2.0 * pi)) * x * (5.0 * z * z - 1.0),
                0.25 * math.sqrt(105.0 / pi) * z * (x * x - y * y),
                0.25 * math.sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y)]
    if degree > 3:
        raise ValueError("SH degree must be 0..3")
    return np.stack(out, axis=1)


def emission(coeffs, degree, dirs):
    """E = max(0, sum_lm coeffs[:, lm, :] * Y_lm(dir) + 0.5): [P, 3]."""
    Y = basis(degree, dirs)                      # [P, K]
    c = np.asarray(coeffs, np.float64)[:, : Y.shape[1], :]
    return np.maximum(np.einsum("pk,pkc->pc", Y, c) + 0.5, 0.0)
