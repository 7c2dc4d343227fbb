"""Pins of the oracle's time loop: driver deposit, wake gather and driver push
(no GPU).

The outer loop of Algorithm 1 advances the driver macroparticles in t by eqs.
(25)-(26) through the wake of the xi-sweep; their current enters the slices'
j_z.  Pins, none of which retypes the oracle's formulas:

* the deposit conserves the driver's charge, and a quiet (lattice) driver
  deposits the analytic Gaussian density on the nodes and planes; a sampled
  driver reproduces the per-plane charge of the analytic profile;
* the push: in a uniform B the momentum's length is conserved exactly and it
  turns by 2 atan(|qm B| dt / 2 gamma) per step; in a uniform E the momentum
  grows exactly linearly and the orbit converges to the closed-form
  hyperbolic motion at second order; a step forward and one back return to the
  start; ahead of the first slice and behind the last there is no force;
* a time step with a quiet driver gives the wake of the frozen analytic
  driver (to the interpolation error in xi), and an electron driver loses
  energy to its wake.
"""
import numpy as np
import pytest

import wandqs_inputs as wi


def _cfg(N=32, L=4.0, **kw):
    return wi.scaled(wi.config("C1"), n_cells=N, half_width=L, beams=[], **kw)


def _uniform_stack(N, L, grad=(0.0, 0.0), ez=0.0, b=(0.0, 0.0, 0.0), xis=(-10.0, 10.0)):
    """Slices with uniform fields: psi linear (its gradient), Ez, Bx, By, Bz."""
    h = 2 * L / N
    g = -L + h * np.arange(N + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    F = np.zeros((len(xis), 5, N + 1, N + 1))
    F[:, 0] = grad[0] * X + grad[1] * Y
    F[:, 1] = ez
    F[:, 2] = b[2]
    F[:, 3] = b[0]
    F[:, 4] = b[1]
    return np.array(xis, dtype=float), F


def _particles(n, seed, gamma=5.0, L=2.0):
    rng = np.random.default_rng(seed)
    d = np.zeros((8, n))
    d[0], d[1] = rng.uniform(-L, L, n), rng.uniform(-L, L, n)
    d[2] = rng.uniform(-1, 1, n)
    p = rng.standard_normal((3, n))
    p *= np.sqrt(gamma ** 2 - 1) / np.linalg.norm(p, axis=0)
    d[3:6] = p
    d[6] = -1.0
    d[7] = 1.0
    return d


def test_deposit_conserves_charge_and_reproduces_a_quiet_driver(oracle_mod):
    N, L, dz, nz, xi0 = 32, 4.0, 0.05, 64, 0.0
    beam = wi.gauss_beam(0.7, 0.6, 0.5, 1.6)
    o = oracle_mod.Oracle(_cfg(N, L))
    d = wi.driver_lattice(beam, N, L, xi0, dz, nz, gamma0=1e4)
    P = o.driver_deposit(d, nz, xi0, dz)
    h = 2 * L / N
    vz = d[5] / np.sqrt(1 + d[5] ** 2)
    assert abs(P.sum() * h * h * dz - (d[7] * vz).sum()) <= 1e-13 * (d[7] * vz).sum()
    g = -L + h * np.arange(N + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    for m in (10, 32, 40):
        xi = xi0 + m * dz
        ref = beam["amp"] * np.exp(-(X ** 2 + Y ** 2) / beam["sigma_r"] ** 2
                                   - (xi - beam["xi_c"]) ** 2 / beam["sigma_z"] ** 2) * vz[0]
        ref[ref < 1e-12 * beam["amp"]] = 0.0
        np.testing.assert_allclose(P[m], ref, rtol=1e-12, atol=1e-15)


def test_sampled_driver_matches_the_profile_per_plane(oracle_mod):
    """200k macroparticles sampled from a Gaussian: the charge per plane
    follows amp pi sr^2 exp(-(xi-xc)^2/sz^2) to the sampling noise."""
    N, L, dz, nz, xi0 = 32, 4.0, 0.1, 40, 0.0
    beam = wi.gauss_beam(2.0, 0.5, 0.6, 2.0)
    d = wi.driver_gaussian(beam, 200_000, seed=12, gamma0=1e4)
    o = oracle_mod.Oracle(_cfg(N, L))
    P = o.driver_deposit(d, nz, xi0, dz)
    h = 2 * L / N
    per_plane = P.sum(axis=(1, 2)) * h * h
    xis = xi0 + dz * np.arange(nz)
    ref = beam["amp"] * np.pi * beam["sigma_r"] ** 2 * np.exp(-(xis - 2.0) ** 2 / 0.36)
    big = ref > 0.2 * ref.max()
    err = np.abs(per_plane[big] - ref[big]) / ref[big]
    print("per-plane charge relative error", err.max())
    assert err.max() < 0.03


def test_push_uniform_b_rotates_exactly(oracle_mod):
    N, L = 16, 8.0
    o = oracle_mod.Oracle(_cfg(N, L))
    B = np.array([0.3, -0.2, 0.9])
    # E_perp = -grad psi - e_z x B_perp vanishes for grad psi = (B_y, -B_x)
    xis, F = _uniform_stack(N, L, grad=(B[1], -B[0]), b=B)
    d0 = _particles(200, 3)
    dt = 0.7
    d1 = o.driver_push(d0, dt, xis, F)
    p0, p1 = d0[3:6], d1[3:6]
    assert np.allclose(np.linalg.norm(p1, axis=0), np.linalg.norm(p0, axis=0), rtol=1e-14)
    gam = np.sqrt(1 + (p0 ** 2).sum(axis=0))
    bn = np.linalg.norm(B)
    # the component along B is unchanged; the perpendicular part turns by the
    # Cayley angle 2 atan(|qm B| dt / 2 gamma) (qm = -1)
    u = B / bn
    par0, par1 = u @ p0, u @ p1
    assert np.allclose(par1, par0, rtol=0, atol=1e-12)
    q0, q1 = p0 - np.outer(u, par0), p1 - np.outer(u, par1)
    cosang = (q0 * q1).sum(axis=0) / (np.linalg.norm(q0, axis=0) * np.linalg.norm(q1, axis=0))
    np.testing.assert_allclose(np.arccos(np.clip(cosang, -1, 1)), 2 * np.arctan(bn * dt / (2 * gam)),
                               rtol=1e-9)
    # the sense of rotation: dp/dt = qm v x B with qm = -1
    cross = np.cross(q0.T, q1.T) @ u
    assert np.all(cross > 0)


def test_push_uniform_e_exact_momentum_second_order_orbit(oracle_mod):
    """dp/dt = qm E: p(t) = p0 + qm E t exactly at every step; the orbit in
    (x, y, xi) against its closed form x(t) = x0 + (gamma(t) - gamma0)/(qm E)
    for E along x (p_y = 0), xi(t) = xi0 + t - p_z0 (asinh(p_x(t)/m) -
    asinh(p_x0/m))/(qm E) with m = sqrt(1 + p_z0^2)."""
    N, L, Ex = 16, 50.0, 0.4
    o = oracle_mod.Oracle(_cfg(N, L))
    xis, F = _uniform_stack(N, L, grad=(-Ex, 0.0))  # E_x = -d_x psi
    d0 = np.zeros((8, 1))
    d0[3, 0], d0[5, 0], d0[6, 0] = 0.5, 3.0, -1.0
    d0[7, 0] = 1.0
    T = 4.0
    errs = []
    for n in (16, 32, 64):
        d = d0.copy()
        for _ in range(n):
            d = o.driver_push(d, T / n, xis, F)
        qE = -Ex
        pxT = 0.5 + qE * T
        assert abs(d[3, 0] - pxT) < 1e-13 and d[4, 0] == 0.0 and d[5, 0] == 3.0
        m = np.sqrt(1 + 3.0 ** 2)
        xT = (np.sqrt(m * m + pxT ** 2) - np.sqrt(m * m + 0.25)) / qE
        xiT = T - 3.0 * (np.arcsinh(pxT / m) - np.arcsinh(0.5 / m)) / qE
        errs.append(max(abs(d[0, 0] - xT), abs(d[2, 0] - xiT)))
    print("orbit errors", errs)
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_push_is_reversible_and_forceless_outside_the_slices(oracle_mod):
    N, L = 16, 8.0
    o = oracle_mod.Oracle(_cfg(N, L))
    xis, F = _uniform_stack(N, L, grad=(0.2, -0.1), ez=0.3, b=(0.1, 0.4, -0.5))
    d0 = _particles(100, 5, gamma=3.0)
    d1 = o.driver_push(d0, 0.6, xis, F)
    d2 = o.driver_push(d1, -0.6, xis, F)
    assert np.abs(d2 - d0).max() < 1e-12
    # slices only over xi in [5, 6]: particles elsewhere drift freely
    xs2, F2 = _uniform_stack(N, L, grad=(0.2, -0.1), ez=0.3, b=(0.1, 0.4, -0.5), xis=(5.0, 6.0))
    d3 = o.driver_push(d0, 0.6, xs2, F2)
    assert np.array_equal(d3[3:6], d0[3:6])


def test_time_step_quiet_driver_gives_the_frozen_wake_and_loses_energy(oracle_mod):
    """C1 (64^2, weak driver) for 60 slices: the wake of the deposited quiet
    driver against the wake of the analytic frozen driver with the same
    parameters (they differ by the linear interpolation between planes,
    dz = 0.0625, and by v_z = 1 - 1/2gamma^2); the driver particles lose
    longitudinal momentum to the wake (E_z > 0 behind the driver centre pulls
    electrons back)."""
    cfg = wi.config("C1")
    beam = cfg["beams"][0]
    n = 60
    dz, xi0, nz = 0.0625, -0.0625, 96
    drv = wi.driver_lattice(beam, cfg["n_cells"], cfg["half_width"], xi0, dz, nz, gamma0=1e4)
    o_ref = oracle_mod.Oracle(cfg)
    st_ref = oracle_mod.initial_state(cfg)
    Fr = o_ref.run(st_ref, n, keep_fields=True)["fields"]
    cfg_d = wi.scaled(cfg, beams=[])
    o = oracle_mod.Oracle(cfg_d)
    st = oracle_mod.initial_state(cfg_d)
    d = drv.copy()
    r = o.time_step(st, d, n, 50.0, nz, xi0, dz, keep_fields=True)
    assert r["status"] == 0
    Fd = r["fields"]
    for k in (0, 3, 4):  # psi, Bx, By
        e = np.abs(Fd[:, k] - Fr[:, k]).max() / np.abs(Fr[:, k]).max()
        print("field", k, "quiet driver vs frozen analytic driver", e)
        assert e < 2e-3
    dpz = (d[5] - drv[5]) * drv[7]
    print("weighted mean dp_z over one step", dpz.sum() / drv[7].sum())
    assert dpz.sum() < 0.0
