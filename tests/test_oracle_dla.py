"""Pins of the oracle's driver push in the laser's fields with sub-cycling
(Sec. IV, eqs. (21)-(26); no GPU).

The laser's fields come from the envelope A-hat (the x-polarised vector
potential A_x = Re(A-hat exp(-i k0 xi))) interpolated between its planes and
its two time levels.  Pins, none of which retypes the field formulas:

* Maxwell's equations that the formulas must obey for any envelope, checked
  by finite differences of the field function: Faraday's law for B_z and for
  B_y (d/dt at fixed z is d_t + d_xi) and, for an envelope constant in t,
  Gauss's law div E = 0 (d/dz at fixed t is -d_xi);
* an electron in fields that do not depend on x keeps its canonical momentum
  p_x - A_x(t, xi) (charge -e), and, when they depend on xi alone (a plane
  wave), also gamma - p_z; the sub-cycled push converges to both at second
  order in the sub-step (with one step per dt it does not follow the
  oscillation at all).
"""
import numpy as np

import wandqs_inputs as wi


def _cfg(N, L, dxi, **kw):
    return wi.scaled(wi.config("C1"), n_cells=N, half_width=L, beams=[], dxi0=dxi, adaptive=0,
                     **kw)


def test_laser_fields_obey_faraday_and_gauss(oracle_mod):
    N, L, dxi, nz, k0, dt = 16, 4.0, 0.1, 40, 3.0, 0.7
    o = oracle_mod.Oracle(_cfg(N, L, dxi))
    rng = np.random.default_rng(5)
    A0 = rng.standard_normal((nz, N + 1, N + 1)) + 1j * rng.standard_normal((nz, N + 1, N + 1))
    A1 = A0 + 0.3 * (rng.standard_normal((nz, N + 1, N + 1)) + 1j * rng.standard_normal((nz, N + 1, N + 1)))
    o.set_laser(A0, k0)
    h = 2 * L / N
    n = 200
    # points inside cells and plane intervals, away from their edges (the
    # interpolant is smooth there)
    ca, cb, cq = rng.integers(1, N - 1, n), rng.integers(1, N - 1, n), rng.integers(1, nz - 2, n)
    fx, fy, fq = rng.uniform(0.2, 0.8, (3, n))
    x, y, xi = -L + (ca + fx) * h, -L + (cb + fy) * h, (cq + fq) * dxi
    tau = rng.uniform(0.2, 0.8, n)
    d = 1e-5

    def F(xx, yy, zz, tt, a0=A0, a1=A1):
        return np.stack([o.laser_fields(dt, tt[i], np.array([[xx[i]], [yy[i]], [zz[i]]]), a0, a1)[:, 0]
                         for i in range(n)], axis=1)

    EX, EZ, BY, BZ = 0, 2, 4, 5
    # Faraday, z: dB_z/dt = -(d_x E_y - d_y E_x) = d_y E_x
    dBz = (F(x, y, xi + d, tau + d / dt)[BZ] - F(x, y, xi - d, tau - d / dt)[BZ]) / (2 * d)
    dEx_y = (F(x, y + d, xi, tau)[EX] - F(x, y - d, xi, tau)[EX]) / (2 * d)
    assert np.abs(dBz - dEx_y).max() < 1e-5 * np.abs(dEx_y).max()
    # Faraday, y: dB_y/dt = -(d_z E_x - d_x E_z) = d_xi E_x + d_x E_z
    dBy = (F(x, y, xi + d, tau + d / dt)[BY] - F(x, y, xi - d, tau - d / dt)[BY]) / (2 * d)
    dEx_xi = (F(x, y, xi + d, tau)[EX] - F(x, y, xi - d, tau)[EX]) / (2 * d)
    dEz_x = (F(x + d, y, xi, tau)[EZ] - F(x - d, y, xi, tau)[EZ]) / (2 * d)
    assert np.abs(dBy - dEx_xi - dEz_x).max() < 1e-5 * np.abs(dBy).max()
    # Gauss with an envelope constant in t: d_x E_x + d_z E_z = d_x E_x - d_xi E_z = 0
    dEx_x = (F(x + d, y, xi, tau, A0, A0)[EX] - F(x - d, y, xi, tau, A0, A0)[EX]) / (2 * d)
    dEz_xi = (F(x, y, xi + d, tau, A0, A0)[EZ] - F(x, y, xi - d, tau, A0, A0)[EZ]) / (2 * d)
    assert np.abs(dEx_x - dEz_xi).max() < 1e-5 * np.abs(dEx_x).max()
    # E_y and B_x are dropped (x-polarised, Sec. IV)
    assert np.all(F(x, y, xi, tau)[[1, 3]] == 0.0)


def _wave(N, nz, dxi, scale=1.0):
    xis = dxi * np.arange(nz)
    prof = 0.5 * np.exp(-(xis - 5.0) ** 2)
    env = np.repeat((scale * prof)[:, None], (N + 1) ** 2, 1).reshape(nz, N + 1, N + 1)
    return xis, prof, env.astype(complex)


def _drift(oracle_mod, nsub, time_varying):
    N, L, dxi, nz, k0, dt = 16, 4.0, 0.05, 240, 5.0, 0.5
    o = oracle_mod.Oracle(_cfg(N, L, dxi, driver_nsub=nsub))
    xis, prof, _ = _wave(N, nz, dxi)
    o.set_laser(_wave(N, nz, dxi)[2], k0)
    amp = (lambda t: 1.0 + 0.1 * t) if time_varying else (lambda t: 1.0)

    def Ax(t, xi):  # the potential of the interpolated envelope (linear in xi and t)
        return np.real(amp(t) * np.interp(xi, xis, prof) * np.exp(-1j * k0 * xi))

    d = np.zeros((8, 3))
    # two electrons at rest ahead of the pulse, one moving with it inside it
    d[0], d[1], d[2] = [0.0, 0.5, -0.3], [0.0, 0.2, 0.1], [0.5, 0.6, 3.5]
    d[5] = [0.0, 0.0, 2.0]
    d[6], d[7] = -1.0, 1.0
    px0 = d[3] - Ax(0.0, d[2])
    lf0 = np.sqrt(1 + (d[3:6] ** 2).sum(0)) - d[5]
    none = np.zeros((1, 5, N + 1, N + 1))
    dev_px = dev_lf = 0.0
    t = 0.0
    for _ in range(24):
        d = o.driver_push(d, dt, np.zeros(0), none, _wave(N, nz, dxi, amp(t))[2],
                          _wave(N, nz, dxi, amp(t + dt))[2])
        t += dt
        dev_px = max(dev_px, np.abs(d[3] - Ax(t, d[2]) - px0).max())
        dev_lf = max(dev_lf, np.abs(np.sqrt(1 + (d[3:6] ** 2).sum(0)) - d[5] - lf0).max())
    assert d[2][:2].min() > 7.0  # the pulse (xi ~ 3 .. 7) has passed the first two
    return dev_px, dev_lf


def test_plane_wave_keeps_canonical_and_light_front_momenta(oracle_mod):
    p8, l8 = _drift(oracle_mod, 8, False)
    p32, l32 = _drift(oracle_mod, 32, False)
    p1, _ = _drift(oracle_mod, 1, False)
    print("canonical", p1, p8, p32, "light front", l8, l32)
    assert p32 < 5e-4 and l32 < 2e-5
    assert p8 / p32 > 6 and l8 / l32 > 12
    assert p1 > 0.05  # one step per dt does not resolve the oscillation


def test_time_varying_envelope_keeps_canonical_momentum(oracle_mod):
    p8, _ = _drift(oracle_mod, 8, True)
    p32, _ = _drift(oracle_mod, 32, True)
    print("canonical (time-varying)", p8, p32)
    assert p32 < 2e-3 and p8 / p32 > 5
