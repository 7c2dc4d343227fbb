"""Closed-form linear wake of a weak, frozen, luminal Gaussian driver.

Independent of the oracle: it comes from linearising the quasi-static system
(paper Sec. III: eqs. (6)-(7), (8), (9), (12)-(14), (18)-(19)) about a cold
uniform plasma at rest, g = 1 + psi ~ 1, for a driver
``n_b = A exp(-r^2/sr^2) exp(-(xi - xc)^2/sz^2)`` switched on at xi = 0.
The electron fluid then obeys ``(d^2/dxi^2 + 1) n1 = -n_b`` transversely
local, which gives

    psi(r, xi) = -A Z(xi) R(r),        Ez = d psi/dxi = -A Z'(xi) R(r),
    B_x = +A exp(-(xi-xc)^2/sz^2) R'(r) y/r,   B_y = -A exp(...) R'(r) x/r,

with ``Z(xi) = int_0^xi sin(xi - s) exp(-(s-xc)^2/sz^2) ds`` and R the decaying
solution of ``(nabla_perp^2 - 1) R = exp(-r^2/sr^2)``:

    R(r)  = -K0(r) int_0^r I0 f s ds - I0(r) int_r^inf K0 f s ds,
    R'(r) = -K1(r)... (see code),  f(s) = exp(-s^2/sr^2).

Used only by the oracle's pin tests.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, special


def _f(s, sr):
    return np.exp(-(s * s) / (sr * sr))


def radial_R(r: float, sr: float) -> float:
    """Solution of (1/r)(r R')' - R = exp(-r^2/sr^2) that is regular at 0 and decays."""
    if r == 0.0:
        val, _ = integrate.quad(lambda s: special.k0(s) * _f(s, sr) * s, 0.0, np.inf, limit=200)
        return -val
    inner, _ = integrate.quad(lambda s: special.i0(s) * _f(s, sr) * s, 0.0, r, limit=200)
    outer, _ = integrate.quad(lambda s: special.k0(s) * _f(s, sr) * s, r, np.inf, limit=200)
    return -special.k0(r) * inner - special.i0(r) * outer


def radial_dR(r: float, sr: float) -> float:
    """dR/dr: K0' = -K1 and I0' = I1 acting on the two Green's-function terms."""
    if r == 0.0:
        return 0.0
    inner, _ = integrate.quad(lambda s: special.i0(s) * _f(s, sr) * s, 0.0, r, limit=200)
    outer, _ = integrate.quad(lambda s: special.k0(s) * _f(s, sr) * s, r, np.inf, limit=200)
    return special.k1(r) * inner - special.i1(r) * outer


def long_Z(xi: float, sz: float, xc: float, deriv: bool = False) -> float:
    if xi <= 0.0:
        return 0.0
    kern = np.cos if deriv else np.sin
    val, _ = integrate.quad(lambda s: kern(xi - s) * np.exp(-((s - xc) ** 2) / (sz * sz)),
                            0.0, xi, limit=200)
    return val


def ez_on_axis(xi, A, sr, sz, xc):
    R0 = radial_R(0.0, sr)
    return np.array([-A * long_Z(float(v), sz, xc, deriv=True) * R0 for v in np.atleast_1d(xi)])


def psi_on_axis(xi, A, sr, sz, xc):
    R0 = radial_R(0.0, sr)
    return np.array([-A * long_Z(float(v), sz, xc) * R0 for v in np.atleast_1d(xi)])


def bperp(x, y, xi, A, sr, sz, xc):
    """(B_x, B_y) of the linear wake at a point."""
    r = float(np.hypot(x, y))
    if r == 0.0:
        return 0.0, 0.0
    e = A * np.exp(-((xi - xc) ** 2) / (sz * sz)) * radial_dR(r, sr)
    return e * y / r, -e * x / r
