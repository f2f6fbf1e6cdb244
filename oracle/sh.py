"""Real spherical harmonics up to degree 3, built from their definition (oracle; test infrastructure only).

The paper gives each Gaussian SH coefficients for view-dependent colour (Sec. 3.1) without fixing a
basis.  The reading used throughout is the real orthonormal basis with the Condon-Shortley phase,
ordered l-major with m = -l..l (index k = l^2 + l + m):

    Y_l^m  = sqrt(2) K_l^|m| cos(m phi)   P_l^|m|(cos theta)   for m > 0
    Y_l^m  = sqrt(2) K_l^|m| sin(|m| phi) P_l^|m|(cos theta)   for m < 0
    Y_l^0  = K_l^0 P_l(cos theta)
    K_l^m  = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
    P_l^m(z) = (-1)^m (1-z^2)^(m/2) d^m/dz^m P_l(z)

On a unit vector (x, y, z): sin^m(theta) cos(m phi) = Re((x+iy)^m) and sin^m(theta) sin(m phi) = Im((x+iy)^m),
so every Y is a polynomial in (x, y, z) that torch can differentiate.  The Legendre polynomials and their
derivatives come from numpy's Legendre series routines.
"""
from __future__ import annotations

import math

import numpy as np
import numpy.polynomial.legendre as npleg
import numpy.polynomial.polynomial as nppoly
import torch


def _legendre_derivative_coeffs(l: int, m: int) -> np.ndarray:
    """Power-series coefficients (ascending) of d^m/dz^m P_l(z)."""
    c = np.zeros(l + 1)
    c[l] = 1.0
    power = npleg.leg2poly(c)
    return nppoly.polyder(power, m) if m > 0 else power


def _norm(l: int, m: int) -> float:
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def basis(dirs: torch.Tensor, degree: int = 3) -> torch.Tensor:
    """Evaluate the (degree+1)^2 real SH at unit directions ``dirs`` [N,3] -> [N,(degree+1)^2]."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    # Re/Im of (x+iy)^m for m = 0..degree
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for _ in range(degree):
        r, i = re[-1], im[-1]
        re.append(r * x - i * y)
        im.append(r * y + i * x)
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            coeffs = _legendre_derivative_coeffs(l, am)
            poly = torch.zeros_like(z)
            for c in coeffs[::-1]:  # Horner
                poly = poly * z + float(c)
            phase = (-1.0) ** am
            if m == 0:
                out.append(_norm(l, 0) * poly)
            elif m > 0:
                out.append(math.sqrt(2.0) * _norm(l, am) * phase * re[am] * poly)
            else:
                out.append(math.sqrt(2.0) * _norm(l, am) * phase * im[am] * poly)
    return torch.stack(out, dim=1)
