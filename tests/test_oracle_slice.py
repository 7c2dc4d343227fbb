"""Pins of the oracle's particle operations and of the whole slice (no GPU).

Each check is independent of the oracle's code: closed forms, invariants fixed
by the paper, special cases that reduce to exact arithmetic, and the paper's
central identity (the explicit xi-derivative of the transverse current,
Sec. III.B eqs. (15)-(19)) tested against finite differences of the particle
motion itself.
"""
import os

import numpy as np
import pytest

import linear_wake as lw
import wandqs_inputs as wi


def _rand_particles(cfg, P, seed):
    rng = np.random.default_rng(seed)
    L = cfg["half_width"]
    return rng.uniform(-L, L, P), rng.uniform(-L, L, P)


# ------------------------------------------------------------------ CIC -----

def test_deposit_partition_of_unity(oracle_mod):
    """Total charge: sum n* h^2 = P w exactly (continuity eq. (8): N is xi-independent)."""
    cfg = wi.scaled(wi.config("C2"), n_cells=32)
    o = oracle_mod.Oracle(cfg)
    x, y = _rand_particles(cfg, 5000, 1)
    x[:4] = [-8.0, 8.0, -8.0, 8.0]   # corners and edges are included
    y[:4] = [-8.0, 8.0, 8.0, -8.0]
    n = o.deposit(x, y)
    w = cfg["n0"] * o.h ** 2 / cfg["ppc_side"] ** 2
    assert abs(n.sum() * o.h ** 2 - x.size * w) <= 1e-13 * x.size * w


def test_lattice_gives_uniform_density(oracle_mod):
    """A cold plasma at rest on the lattice has n* = n0 at every interior node."""
    for name in ("C1",):
        cfg = wi.config(name)
        st = oracle_mod.initial_state(cfg)
        n = oracle_mod.Oracle(cfg).deposit(st["x"], st["y"])
        assert np.abs(n[1:-1, 1:-1] - 1.0).max() <= 1e-14
    cfg = wi.scaled(wi.config("C2"), n_cells=32, jitter=0.0)
    st = oracle_mod.initial_state(cfg)
    n = oracle_mod.Oracle(cfg).deposit(st["x"], st["y"])
    assert np.abs(n[1:-1, 1:-1] - 1.0).max() <= 1e-14


def test_gather_reproduces_bilinear_fields(oracle_mod):
    cfg = wi.scaled(wi.config("C2"), n_cells=16)
    o = oracle_mod.Oracle(cfg)
    g = -o.L + o.h * np.arange(o.N + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    F = 0.3 - 1.7 * X + 0.25 * Y + 0.8 * X * Y   # bilinear on every cell
    x, y = _rand_particles(cfg, 2000, 2)
    got = o.gather(x, y, F)
    ref = 0.3 - 1.7 * x + 0.25 * y + 0.8 * x * y
    assert np.abs(got - ref).max() <= 1e-12


def test_deposit_is_adjoint_of_gather(oracle_mod):
    """<deposit(q), F> h^2 = sum_i w q_i gather(F)_i."""
    cfg = wi.scaled(wi.config("C2"), n_cells=32)
    o = oracle_mod.Oracle(cfg)
    rng = np.random.default_rng(3)
    x, y = _rand_particles(cfg, 3000, 4)
    q = rng.standard_normal(x.size)
    F = rng.standard_normal((o.N + 1, o.N + 1))
    w = cfg["n0"] * o.h ** 2 / cfg["ppc_side"] ** 2
    lhs = (o.deposit(x, y, q) * F).sum() * o.h ** 2
    rhs = (w * q * o.gather(x, y, F)).sum()
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(w * q).sum() * np.abs(F).max())


# --------------------------------------------------------------- pusher -----

def test_push_uniform_bz_is_exact_rotation(oracle_mod):
    """Only (e_z x V) Bz acts: |p| is conserved and p turns counter-clockwise by
    2 atan(Bz dxi / 2g) per step (eq. (7))."""
    P = 7
    rng = np.random.default_rng(5)
    px, py = rng.standard_normal(P), rng.standard_normal(P)
    g = rng.uniform(0.5, 2.0, P)
    Bz = rng.uniform(-3, 3, P)
    dxi = 0.05
    z = np.zeros(P)
    x, y, qx, qy = oracle_mod.push(1e9, dxi, g, z, z, z, z, Bz, z, z, px, py)
    assert np.allclose(np.hypot(qx, qy), np.hypot(px, py), rtol=1e-14, atol=0)
    turn = np.angle((qx + 1j * qy) / (px + 1j * py))
    assert np.allclose(turn, 2 * np.arctan(Bz * dxi / (2 * g)), rtol=1e-12, atol=1e-14)


def test_push_uniform_by_is_exact_drift(oracle_mod):
    """Only e_z x B_perp with B = (0, By): dp_x/dxi = -By exactly, so after n
    steps p_x = -By n dxi; the drift dx = dxi p_new/g is exact for this force."""
    By, dxi, g = 0.7, 0.01, 1.3
    x, y, px, py = (np.zeros(1) for _ in range(4))
    one, z = np.ones(1), np.zeros(1)
    xs = 0.0
    for n in range(1, 51):
        x, y, px, py = oracle_mod.push(1e9, dxi, g * one, z, z, z, By * one, z, x, y, px, py)
        xs += dxi * (-By * n * dxi) / g
        assert abs(px[0] + By * n * dxi) <= 1e-14 * n
    assert abs(x[0] - xs) <= 1e-12


def test_push_gradient_force_uses_gamma(oracle_mod):
    """Only the wake-potential force gamma grad psi / g (eq. (7)) acts on a
    particle at rest: one step gives p = dxi * gamma0 grad psi / g with
    gamma0 = (1 + g^2)/(2g)."""
    g, gx, gy, dxi = 1.2, 0.3, -0.4, 0.02
    one, z = np.ones(1), np.zeros(1)
    x, y, px, py = oracle_mod.push(1e9, dxi, g * one, gx * one, gy * one, z, z, z, z, z, z, z)
    gam0 = (1 + g * g) / (2 * g)
    assert abs(px[0] - dxi * gam0 * gx / g) <= 1e-16
    assert abs(py[0] - dxi * gam0 * gy / g) <= 1e-16
    assert abs(x[0] - dxi * px[0] / g) <= 1e-18


def test_push_wall_reflection(oracle_mod):
    L = 1.0
    one, z = np.ones(1), np.zeros(1)
    x, y, px, py = oracle_mod.push(L, 0.1, one, z, z, z, z, z, 0.99 * one, -0.99 * one,
                                   0.3 * one, -0.3 * one)
    assert np.isclose(x[0], 2 * L - 1.02) and np.isclose(px[0], -0.3)
    assert np.isclose(y[0], -2 * L + 1.02) and np.isclose(py[0], 0.3)


# ----------------------------------------------------------- Algorithm 1 -----

def test_step_size_refinement_table(oracle_mod):
    """Step_Size_Refinement (Algorithm 1) with the refinement floor of Sec. V.A."""
    cfg = wi.scaled(wi.config("C2"), n_cells=256, half_width=8.0, dxi0=0.02, refine_k=8)
    o = oracle_mod.Oracle(cfg)
    V0 = o.h / 0.02
    assert o.next_dxi(0.0) == 0.02
    assert o.next_dxi(0.5 * V0) == 0.02
    assert o.next_dxi(V0) == 0.02
    assert np.isclose(o.next_dxi(2 * V0), 0.01, rtol=1e-15)
    assert np.isclose(o.next_dxi(5 * V0), 0.004, rtol=1e-15)
    assert np.isclose(o.next_dxi(100 * V0), 0.02 / 8, rtol=1e-15)
    for v in (1.5 * V0, 3 * V0, 7.9 * V0):   # floor inactive: a step never crosses a cell
        assert v * o.next_dxi(v) <= o.h * (1 + 1e-15)
    o2 = oracle_mod.Oracle(wi.scaled(cfg, adaptive=0))
    assert o2.next_dxi(100 * V0) == 0.02
    o3 = oracle_mod.Oracle(wi.scaled(cfg, refine_k=0))
    assert np.isclose(o3.next_dxi(100 * V0), 0.0002, rtol=1e-14)


# ------------------------------------------------------------ invariants -----

def test_qs_invariant_formula():
    """gamma = (1 + p^2 + g^2)/(2g) and p_z = gamma - g satisfy the mass shell
    gamma^2 - p_perp^2 - p_z^2 = 1 (Sec. III.A, H - P_z = 1)."""
    rng = np.random.default_rng(9)
    p = rng.standard_normal((2, 1000)) * 3
    g = rng.uniform(0.05, 3.0, 1000)
    gam = (1 + (p ** 2).sum(0) + g * g) / (2 * g)
    pz = gam - g
    assert np.allclose(gam ** 2 - (p ** 2).sum(0) - pz ** 2, 1.0, rtol=0, atol=1e-11 * gam ** 2)


def test_qs_invariant_dynamic(oracle_mod):
    """Carrying p_z with dp_z/dxi = -gamma Ez/g - Vx By + Vy Bx keeps
    gamma - p_z = 1 + psi (exact in the continuum because Ez = d psi/dxi);
    the discrete defect shrinks when the resolution is refined."""
    errs = []
    for N, dxi in ((64, 0.0625), (128, 0.03125)):
        cfg = wi.scaled(wi.config("C1"), n_cells=N, dxi0=dxi)
        cfg["beams"][0]["amp"] = 0.5
        o = oracle_mod.Oracle(cfg)
        st = oracle_mod.initial_state(cfg)
        r = o.run(st, int(round(5.0 / dxi)), carry_pz=True)
        assert r["status"] == 0
        errs.append(max(i.invariant_err for i in r["infos"]))
    assert errs[0] < 1e-2 and errs[1] < 0.6 * errs[0], errs


def test_charge_conserved_over_run(oracle_mod):
    cfg = wi.scaled(wi.config("C2"), n_cells=64, half_width=4.0)
    o = oracle_mod.Oracle(cfg)
    st = oracle_mod.initial_state(cfg)
    n0 = o.deposit(st["x"], st["y"]).sum()
    r = o.run(st, 150)
    assert r["status"] == 0
    assert np.all(np.abs(st["x"]) <= 4.0) and np.all(np.abs(st["y"]) <= 4.0)
    assert abs(o.deposit(st["x"], st["y"]).sum() - n0) <= 1e-12 * n0


# ------------------------------------------------------------ whole slice ----

def _linear_error(oracle_mod, N, dxi, A):
    cfg = wi.scaled(wi.config("C1"), n_cells=N, dxi0=dxi)
    cfg["beams"][0]["amp"] = A
    ns = int(round(8.0 / dxi)) + 1
    o = oracle_mod.Oracle(cfg)
    st = oracle_mod.initial_state(cfg)
    r = o.run(st, ns, keep_fields=True)
    assert r["status"] == 0
    xis = np.arange(ns) * dxi
    ez = r["fields"][:, 1, N // 2, N // 2] / A
    lin = lw.ez_on_axis(xis, 1.0, 0.5, 1.0, 2.0)
    return np.abs(ez - lin).max() / np.abs(lin).max(), r, cfg


# SI constants (CODATA 2018) for the normalised charge k_p^3 q / (4 pi e n0)
_E_CHARGE, _C_LIGHT, _M_E, _EPS0 = 1.602176634e-19, 299792458.0, 9.1093837015e-31, 8.8541878128e-12


def _golden_beams():
    rows = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "beam_charge.txt")
    with open(path) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                f = line.split()
                rows[f[0]] = dict(n0_cm3=float(f[1]), q_nC=float(f[2]),
                                  amp=None if f[3] == "-" else float(f[3]),
                                  sigma_r_um=None if f[4] == "-" else float(f[4]),
                                  sigma_z_um=None if f[5] == "-" else float(f[5]), Q=float(f[6]))
    return rows


def _kp(n0_cm3):
    """Plasma wavenumber omega_p / c in 1/m."""
    n0 = n0_cm3 * 1e6
    return np.sqrt(n0 * _E_CHARGE ** 2 / (_EPS0 * _M_E)) / _C_LIGHT


def test_normalised_charge_definition():
    """Q = k_p^3 q / (4 pi e n0) (Sec. V.A) reproduces both charges the paper
    prints from their plasma densities and bunch charges (Sec. V.A, Sec. VI)."""
    for name, b in _golden_beams().items():
        kp = _kp(b["n0_cm3"])
        Q = kp ** 3 * b["q_nC"] * 1e-9 / (4.0 * np.pi * _E_CHARGE * b["n0_cm3"] * 1e6)
        assert abs(Q - b["Q"]) <= 0.01 * b["Q"], (name, Q)


def test_beam_density_convention_gives_printed_charge(oracle_mod):
    """The oracle's driver density, integrated over the transverse grid and xi
    for the paper's beam-driven bubble (Sec. V.A: 10 n0, sigma_r = 6.6 um,
    sigma_z = 8 um at 6.5e17 cm^-3, in k_p units), gives the normalised charge
    Q = 5.34 that the paper prints for it.  This fixes the Gaussian convention
    exp(-r^2/sigma_r^2 - xi^2/sigma_z^2): with exp(-r^2/(2 sigma^2)) the same
    widths give Q = 15.2.  The widths and the density carry two digits, so the
    printed Q and the one they give agree to about 1%."""
    b = _golden_beams()["beam_driver"]
    kp = _kp(b["n0_cm3"])
    sr, sz = b["sigma_r_um"] * 1e-6 * kp, b["sigma_z_um"] * 1e-6 * kp
    xi_c = 10.0   # well clear of the cut at xi < 0
    cfg = wi._base(n_cells=128, half_width=6.0 * sr, beams=[wi.gauss_beam(b["amp"], sr, sz, xi_c)])
    o = oracle_mod.Oracle(cfg)
    dxi = 0.02
    xis = xi_c + dxi * np.arange(-int(8 * sz / dxi), int(8 * sz / dxi) + 1)
    total = sum(o.beam_density(xi).sum() for xi in xis) * o.h ** 2 * dxi
    Q = total / (4.0 * np.pi)
    assert abs(Q - b["Q"]) <= 0.015 * b["Q"], Q


def test_linear_wake_closed_form(oracle_mod):
    """On-axis Ez of a weak Gaussian driver against the closed-form linear wake,
    and its convergence when h and dxi are halved (C1 and a refined C1)."""
    e64, r, cfg = _linear_error(oracle_mod, 64, 0.0625, 0.1)
    e128, _, _ = _linear_error(oracle_mod, 128, 0.03125, 0.01)
    e256, _, _ = _linear_error(oracle_mod, 256, 0.015625, 0.001)
    print(f"on-axis Ez error vs the linear wake: {e64:.4f}, {e128:.4f}, {e256:.4f}")
    # budget 20% / 6% / 2.5% (measured 16.3% / 5.0% / 1.65%): at C1 the driver
    # spans sigma_r / h = 2.7 cells, so the discretisation error dominates; the
    # pin's strength is that the error keeps falling ~3-4x per halving of h and
    # dxi, which a wrong term would stop at an O(1) floor
    assert e64 < 0.2 and e128 < 0.06 and e256 < 0.025, (e64, e128, e256)
    assert 2.7 < e64 / e128 < 4.5 and 2.7 < e128 / e256 < 4.5, (e64, e128, e256)
    # B_perp of the linear wake at a few points, refined case
    N, dxi = 128, 0.03125
    cfg = wi.scaled(wi.config("C1"), n_cells=N, dxi0=dxi)
    cfg["beams"][0]["amp"] = 0.01
    o = oracle_mod.Oracle(cfg)
    st = oracle_mod.initial_state(cfg)
    F = o.run(st, 100, keep_fields=True)["fields"]
    h = 12.0 / N
    err, ref = 0.0, 0.0
    for j in range(40, 100, 10):
        for a, b in ((N // 2, N // 2 + 5), (N // 2 + 8, N // 2), (N // 2 + 4, N // 2 + 4)):
            bx, by = lw.bperp(-6 + a * h, -6 + b * h, j * dxi, 1.0, 0.5, 1.0, 2.0)
            err = max(err, abs(F[j, 3, b, a] / 0.01 - bx), abs(F[j, 4, b, a] / 0.01 - by))
            ref = max(ref, abs(bx), abs(by))
    assert err < 0.01 * ref


def test_bz_of_a_swirling_plasma(oracle_mod):
    """Bz from eq. (14) for a weak Gaussian swirl of electron momentum
    p = p0 (-(y-y0), x-x0) exp(-r^2/w^2): the continuum solution of
    nabla^2 Bz = e_z.(curl j) with j = n* V ~ p is Bz = -(p0 w^2/2) exp(-r^2/w^2)
    (negative: electrons circulating counter-clockwise are a clockwise current).
    Second-order convergence when h is halved."""
    errs = []
    for N in (64, 128):
        cfg = wi.scaled(wi.config("C1"), n_cells=N, beams=[])
        p0, w = 0.05, 1.0
        st = wi.vortex_state(cfg, p0, w, xi=0.5, x0=0.3, y0=-0.2)
        assert oracle_mod.Oracle(cfg).slice_step(st)["status"] == 0
        h = 12.0 / N
        g = -6 + h * np.arange(N + 1)
        X, Y = np.meshgrid(g, g, indexing="xy")
        ref = -(p0 * w * w / 2) * np.exp(-((X - 0.3) ** 2 + (Y + 0.2) ** 2) / w ** 2)
        errs.append(np.abs(st["fields"][2] - ref).max() / np.abs(ref).max())
    assert errs[0] < 0.04 and errs[1] < 0.01 and errs[0] / errs[1] > 3.5, errs


def test_d4_symmetry(oracle_mod):
    """An axisymmetric driver on the symmetric lattice keeps the square's D4
    symmetry: psi(x,y) = psi(-x,y) = psi(y,x), By(x,y) = -Bx(y,x), Bz = 0."""
    cfg = wi.config("C1")
    o = oracle_mod.Oracle(cfg)
    st = oracle_mod.initial_state(cfg)
    F = o.run(st, 80, keep_fields=True)["fields"][-1]
    psi, Ez, Bz, Bx, By = F
    s = np.abs(psi).max()
    assert np.abs(psi - psi[:, ::-1]).max() <= 1e-12 * s
    assert np.abs(psi - psi.T).max() <= 1e-12 * s
    assert np.abs(Ez - Ez.T).max() <= 1e-12 * np.abs(Ez).max()
    sb = np.abs(Bx).max()
    assert np.abs(By - (-Bx.T)).max() <= 1e-12 * sb
    # Bz is a pseudo-scalar: odd under each mirror of the square.  On the grid it
    # is not identically zero (an O(h^2)-small octupole), but it must be odd.
    assert np.abs(Bz + Bz[:, ::-1]).max() <= 1e-12 * sb
    assert np.abs(Bz + Bz.T).max() <= 1e-12 * sb
    assert np.abs(Bz).max() <= 0.1 * sb


def _fluxpres_error(oracle_mod, cfg, state, n_ramp, dxi_fd):
    """B_perp from the Helmholtz form (eqs. (18)-(19)) against B_perp from the
    non-local form (eq. (15)) with d j_perp/d xi from central differences of
    the deposited current over two particle pushes."""
    o = oracle_mod.Oracle(cfg)
    if n_ramp:
        assert o.run(state, n_ramp)["status"] == 0
    o2 = oracle_mod.Oracle(wi.scaled(cfg, dxi0=dxi_fd))
    state["dxi"] = dxi_fd
    r0 = o2.slice_step(state, want_moments=True)
    r1 = o2.slice_step(state, want_moments=True)
    F1 = state["fields"].copy()
    r2 = o2.slice_step(state, want_moments=True)
    N, h = o.N, o.h
    djx = (r2["moments"][1] - r0["moments"][1]) / (2 * dxi_fd)
    djy = (r2["moments"][2] - r0["moments"][2]) / (2 * dxi_fd)
    jz = r1["extra"][3]
    fx = np.zeros_like(jz)
    fy = np.zeros_like(jz)
    # -e_z x (grad j_z + d j_perp/d xi) = (w_y, -w_x)
    fx[1:-1, 1:-1] = (jz[2:, 1:-1] - jz[:-2, 1:-1]) / (2 * h) + djy[1:-1, 1:-1]
    fy[1:-1, 1:-1] = -((jz[1:-1, 2:] - jz[1:-1, :-2]) / (2 * h) + djx[1:-1, 1:-1])
    _, bx, _, _ = oracle_mod.mg_solve(N, h, fx)
    _, by, _, _ = oracle_mod.mg_solve(N, h, fy)
    num = ((bx - F1[3]) ** 2 + (by - F1[4]) ** 2).sum()
    den = (F1[3] ** 2 + F1[4] ** 2).sum()
    return np.sqrt(num / den), F1


def test_explicit_current_derivative_axisymmetric(oracle_mod):
    """Nonlinear axisymmetric wake: every term of S that involves psi, Ez, T
    or G contributes more than the tolerance here."""
    cfg = wi.scaled(wi.config("C1"), n_cells=128, dxi0=0.02)
    cfg["beams"][0]["amp"] = 4.0
    st = oracle_mod.initial_state(cfg)
    err, F = _fluxpres_error(oracle_mod, cfg, st, 149, 0.002)
    assert err < 0.012, err


def test_explicit_current_derivative_vortex(oracle_mod):
    """A swirling plasma (curl j != 0) exercises the (e_z x j) Bz terms."""
    cfg = wi.scaled(wi.config("C1"), n_cells=128, dxi0=0.004)
    cfg["beams"][0]["amp"] = 1.0
    st = wi.vortex_state(cfg, 0.8, 1.0, xi=1.8)
    oracle_mod.Oracle(cfg).slice_step(st)
    err, F = _fluxpres_error(oracle_mod, cfg, st, 0, 0.004)
    assert np.abs(F[2]).max() > 0.1
    assert err < 0.01, err


def test_nonphysical_reported(oracle_mod):
    """1 + psi <= 0 is an error, never clamped."""
    cfg = wi.scaled(wi.config("C1"), n_cells=32)
    cfg["beams"][0]["amp"] = 1e3
    o = oracle_mod.Oracle(cfg)
    st = oracle_mod.initial_state(cfg)
    st["x"] = st["x"] * 0.0 + 0.01   # all electrons piled on the axis: psi << -1
    st["y"] = st["y"] * 0.0 - 0.01
    r = o.slice_step(st)
    assert r["status"] == oracle_mod.NONPHYS


def test_psi_gradient_boundary_rows(oracle_mod):
    """The node gradient the particle gather uses: central differences inside,
    one-sided differences on the boundary rows and columns.  A linear field's
    gradient is exact on every node, the boundary included; for psi = x^2 the
    interior gradient is exact (2x) and the one-sided boundary values carry
    the first-order error +-h: (x_1^2 - x_0^2)/h = 2 x_0 + h and
    (x_N^2 - x_{N-1}^2)/h = 2 x_N - h.  (A second-order one-sided formula would
    be exact here, a zero or mirrored boundary value would not be 2x +- h.)"""
    N, L = 32, 3.0
    h = 2 * L / N
    g = -L + h * np.arange(N + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    G = oracle_mod.psi_gradient(N, L, 0.7 * X - 1.3 * Y + 0.25)
    assert np.allclose(G[0], 0.7, rtol=0, atol=1e-13) and np.allclose(G[1], -1.3, rtol=0, atol=1e-13)
    G = oracle_mod.psi_gradient(N, L, X * X + 0.5 * Y * Y * Y)
    assert np.allclose(G[0][:, 1:-1], 2 * X[:, 1:-1], rtol=0, atol=1e-12)
    assert np.allclose(G[0][:, 0], 2 * g[0] + h, rtol=0, atol=1e-12)
    assert np.allclose(G[0][:, -1], 2 * g[-1] - h, rtol=0, atol=1e-12)
    # y: central difference of y^3 is 3y^2 + h^2 (exact); one-sided at the edges
    y = g
    assert np.allclose(G[1][1:-1, :].T, 0.5 * (3 * y[1:-1] ** 2 + h * h), rtol=0, atol=1e-11)
    assert np.allclose(G[1][0, :], 0.5 * (y[1] ** 3 - y[0] ** 3) / h, rtol=0, atol=1e-11)
    assert np.allclose(G[1][-1, :], 0.5 * (y[-1] ** 3 - y[-2] ** 3) / h, rtol=0, atol=1e-11)


def _lattice_bin_counts(n_half, p, q, n_bins):
    """Nodes (i, j) of the integer lattice |i|, |j| <= n_half whose distance
    from the origin, in units of the bin width p/q lattice steps, falls in bin
    k: k <= q sqrt(i^2 + j^2) / p < k + 1, decided in exact integer arithmetic
    ((k p)^2 <= q^2 (i^2 + j^2) < ((k+1) p)^2)."""
    i = np.arange(-n_half, n_half + 1, dtype=np.int64)
    d2 = (i[:, None] ** 2 + i[None, :] ** 2) * q * q
    return np.array([np.count_nonzero((d2 >= (k * p) ** 2) & (d2 < ((k + 1) * p) ** 2))
                     for k in range(n_bins)])


@pytest.mark.parametrize("case", ["edges_on_nodes", "edges_between_nodes"])
def test_radial_bin_driver_nodes(oracle_mod, case):
    """Radial-bin driver: bin k holds the nodes with k dr <= r < (k+1) dr around
    its centre (r_max = n_bins dr), its density there is bin_amp[k] times the
    xi factor exp(-(xi-xc)^2/sz^2), and it vanishes for xi < 0.  The node set of
    every bin is checked against an exact integer count of lattice points in
    the annulus; the summed charge per bin, sum n_b h^2, against the annulus
    area pi((k+1)^2 - k^2) dr^2 within the lattice-point bound
    pi((r+h/sqrt2)^2 - (r-h/sqrt2)^2) on each edge.  Two cases: the C4 recipe
    (dr = h, so edges fall on nodes, which belong to the outer bin) and
    dr = 208/25 h off-centre (no node on an edge)."""
    if case == "edges_on_nodes":
        N, L, p, q, nb, cx, cy = 256, 8.0, 1, 1, 32, 0, 0
    else:
        N, L, p, q, nb, cx, cy = 256, 4.0, 208, 25, 9, 3, -5
    h = 2 * L / N
    dr = h * p / q
    x0, y0 = cx * h, cy * h
    n_half = N // 2 - max(abs(cx), abs(cy))
    assert nb * dr < n_half * h  # every annulus lies inside the grid
    exact = _lattice_bin_counts(n_half, p, q, nb)
    xc, sz = 1.5, 0.8
    for k in range(nb):
        amp = np.zeros(nb)
        amp[k] = 1.0 + k
        cfg = wi.scaled(wi.config("C1"), n_cells=N, half_width=L,
                        beams=[wi.radial_bins_beam(amp, nb * dr, sz, xc, x0=x0, y0=y0)])
        o = oracle_mod.Oracle(cfg)
        nbd = o.beam_density(xc)
        on = nbd != 0.0
        assert np.count_nonzero(on) == exact[k], (k, np.count_nonzero(on), exact[k])
        assert np.all(nbd[on] == amp[k])
        q_bin = nbd.sum() * h * h / amp[k]
        area = np.pi * ((k + 1) ** 2 - k ** 2) * dr * dr
        bound = sum(np.pi * ((r + h / np.sqrt(2)) ** 2 - max(r - h / np.sqrt(2), 0.0) ** 2)
                    for r in (k * dr, (k + 1) * dr))
        assert abs(q_bin - area) <= bound, (k, q_bin, area, bound)
        if k == nb // 2:
            np.testing.assert_allclose(o.beam_density(xc + sz)[on], amp[k] * np.exp(-1.0),
                                       rtol=1e-15)
            assert not o.beam_density(-1e-3).any()
