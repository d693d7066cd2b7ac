"""Real spherical-harmonic colour, degrees 0..3 (oracle; test infrastructure).

The basis is the real SH family used by 3D Gaussian Splatting (the paper's
Gaussian representation, Section 3.2): for order m < 0 it is
sqrt(2) Im Y_l^|m|, for m = 0 Y_l^0 and for m > 0 sqrt(2) Re Y_l^m, with the
complex Y_l^m carrying the Condon-Shortley phase.  Each normalisation
constant is computed here from its closed form sqrt((2l+1)/(4 pi) *
(l-|m|)!/(l+|m|)!), so no table of decimal constants is involved.
Coefficients are stored (N, (deg+1)^2, 3) in l-major, m = -l..l order.
"""
from __future__ import annotations

import math

import numpy as np


def _k(l: int, m: int) -> float:
    m = abs(m)
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def basis(dirs: np.ndarray, degree: int) -> np.ndarray:
    """Evaluate the (deg+1)^2 basis functions at unit directions (n,3) -> (n, nc)."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    s2 = math.sqrt(2.0)
    out = [np.full_like(x, _k(0, 0))]
    if degree >= 1:
        # associated Legendre P_1^1 = -sin(theta): x = sin cos(phi), y = sin sin(phi)
        out += [-s2 * _k(1, 1) * y, _k(1, 0) * z, -s2 * _k(1, 1) * x]
    if degree >= 2:
        # P_2^2 = 3 sin^2, P_2^1 = -3 cos sin, P_2^0 = (3 cos^2 - 1)/2
        xx, yy, zz = x * x, y * y, z * z
        out += [s2 * _k(2, 2) * 3.0 * (2.0 * x * y),          # sin^2 sin(2 phi) = 2xy
                -s2 * _k(2, 1) * 3.0 * y * z,
                _k(2, 0) * 0.5 * (2.0 * zz - xx - yy),
                -s2 * _k(2, 1) * 3.0 * x * z,
                s2 * _k(2, 2) * 3.0 * (xx - yy)]
    if degree >= 3:
        xx, yy, zz = x * x, y * y, z * z
        # P_3^3 = -15 sin^3, P_3^2 = 15 cos sin^2, P_3^1 = -1.5 sin (5 cos^2 - 1),
        # P_3^0 = 0.5 (5 cos^3 - 3 cos)
        out += [-s2 * _k(3, 3) * 15.0 * y * (3.0 * xx - yy),          # sin^3 sin(3phi)
                s2 * _k(3, 2) * 15.0 * (2.0 * x * y * z),            # cos sin^2 sin(2phi)
                -s2 * _k(3, 1) * 1.5 * y * (4.0 * zz - xx - yy),
                _k(3, 0) * 0.5 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy),
                -s2 * _k(3, 1) * 1.5 * x * (4.0 * zz - xx - yy),
                s2 * _k(3, 2) * 15.0 * z * (xx - yy),
                -s2 * _k(3, 3) * 15.0 * x * (xx - 3.0 * yy)]
    return np.stack(out, axis=1)


def colour(sh: np.ndarray, dirs: np.ndarray, degree: int) -> np.ndarray:
    """rgb = max(0, sum_lm c_lm Y_lm(dir) + 0.5)  (3DGS colour convention)."""
    B = basis(dirs, degree)                       # (n, nc)
    nc = (degree + 1) ** 2
    raw = np.einsum("nk,nkc->nc", B, sh[:, :nc, :].astype(np.float64))
    return np.maximum(raw + 0.5, 0.0)
