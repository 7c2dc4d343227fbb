"""Pins of the oracle's Runge-Kutta pushers (no GPU).

Besides the Boris-like pusher the paper lists first-, second- and fourth-order
Runge-Kutta for the plasma electrons (Sec. VII.A).  The pins, none of which
retypes the oracle's formulas:

* the first-order scheme agrees with the (separately pinned) Boris-like push
  to first order in dxi: their difference falls 4x per halving of dxi, so the
  two integrate the same equations of motion;
* a uniform B_z with psi = 0 rotates the momentum at the rate B_z: the closed
  form of the orbit, reached at order 1, 2 and 4;
* on fields that the bilinear gather reproduces exactly (linear psi, B_x, B_y,
  uniform B_z) the error against a brute-force solution (a hundred times
  smaller steps of the fourth-order scheme) falls by 2, 4 and 16 per halving.
"""
import numpy as np
import pytest

import wandqs_inputs as wi


def _cfg(pusher, N=32, L=4.0):
    return wi.scaled(wi.config("C1"), n_cells=N, half_width=L, beams=[], pusher=pusher)


def _nodes(N, L):
    g = -L + (2 * L / N) * np.arange(N + 1)
    return np.meshgrid(g, g, indexing="xy")


def _run(o, fields, state, dxi, n):
    x, y, px, py = (np.array(a, dtype=float) for a in state)
    for _ in range(n):
        st, x, y, px, py, _ = o.push_fields(dxi, x, y, px, py, fields)
        assert st == 0
    return np.stack([x, y, px, py])


def test_rk1_agrees_with_boris_to_first_order(oracle_mod):
    N, L = 32, 4.0
    X, Y = _nodes(N, L)
    F = np.zeros((5, N + 1, N + 1))
    F[0] = 0.15 * np.sin(0.7 * X) * np.cos(0.5 * Y)           # psi (g stays near 1)
    F[2] = 0.4 + 0.2 * np.cos(0.3 * X + 0.2 * Y)              # Bz
    F[3] = 0.3 * np.sin(0.4 * Y)                               # Bx
    F[4] = -0.25 * np.cos(0.6 * X)                             # By
    rng = np.random.default_rng(2)
    P = 400
    s0 = (rng.uniform(-2.5, 2.5, P), rng.uniform(-2.5, 2.5, P), rng.uniform(-0.5, 0.5, P),
          rng.uniform(-0.5, 0.5, P))
    rk, bo = oracle_mod.Oracle(_cfg("rk1", N, L)), oracle_mod.Oracle(_cfg("boris", N, L))
    diffs = []
    for dxi in (0.02, 0.01, 0.005):
        a = _run(rk, F, s0, dxi, 1)
        b = _run(bo, F, s0, dxi, 1)
        diffs.append(np.abs(a - b).max())
    print("|rk1 - boris| per step:", diffs)
    assert 3.3 < diffs[0] / diffs[1] < 4.7 and 3.3 < diffs[1] / diffs[2] < 4.7, diffs
    assert diffs[2] < 2.0 * 0.005 ** 2


@pytest.mark.parametrize("pusher,order", [("rk1", 1), ("rk2", 2), ("rk4", 4)])
def test_uniform_bz_closed_form_orbit(oracle_mod, pusher, order):
    """psi = 0, B_perp = 0, uniform B_z: dp/dxi = B_z (-p_y, p_x), dr/dxi = p, so
    p turns by the angle B_z Xi and r follows the closed-form circle."""
    N, L, bz, Xi = 32, 8.0, 1.3, 1.6
    F = np.zeros((5, N + 1, N + 1))
    F[2] = bz
    o = oracle_mod.Oracle(_cfg(pusher, N, L))
    rng = np.random.default_rng(5)
    P = 50
    x0, y0 = rng.uniform(-2, 2, P), rng.uniform(-2, 2, P)
    px0, py0 = rng.uniform(-0.6, 0.6, P), rng.uniform(-0.6, 0.6, P)
    th = bz * Xi
    c, s = np.cos(th), np.sin(th)
    exact = np.stack([x0 + (s * px0 + (c - 1) * py0) / bz, y0 + ((1 - c) * px0 + s * py0) / bz,
                      c * px0 - s * py0, s * px0 + c * py0])
    errs = []
    for n in (8, 16, 32):
        got = _run(o, F, (x0, y0, px0, py0), Xi / n, n)
        errs.append(np.abs(got - exact).max())
    rates = [np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])]
    print(pusher, "errors", errs, "observed orders", rates)
    assert all(abs(r - order) < 0.35 for r in rates), rates


@pytest.mark.parametrize("pusher,order", [("rk1", 1), ("rk2", 2), ("rk4", 4)])
def test_order_on_exactly_gathered_fields(oracle_mod, pusher, order):
    """Linear psi, B_x, B_y and uniform B_z: the gather is exact, so the
    equations of motion are smooth along every orbit and the scheme's order
    shows against a brute-force solution."""
    N, L, Xi = 32, 8.0, 1.2
    X, Y = _nodes(N, L)
    F = np.zeros((5, N + 1, N + 1))
    F[0] = 0.05 * X - 0.03 * Y          # psi: g = 1 + psi within [0.4, 1.6] on the box
    F[2] = 0.7                           # Bz
    F[3] = 0.2 + 0.05 * Y                # Bx
    F[4] = -0.1 + 0.04 * X               # By
    rng = np.random.default_rng(8)
    P = 40
    s0 = (rng.uniform(-2, 2, P), rng.uniform(-2, 2, P), rng.uniform(-0.4, 0.4, P),
          rng.uniform(-0.4, 0.4, P))
    ref = _run(oracle_mod.Oracle(_cfg("rk4", N, L)), F, s0, Xi / 1600, 1600)
    o = oracle_mod.Oracle(_cfg(pusher, N, L))
    errs = [np.abs(_run(o, F, s0, Xi / n, n) - ref).max() for n in (8, 16, 32)]
    rates = [np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])]
    print(pusher, "errors", errs, "observed orders", rates)
    assert all(abs(r - order) < 0.35 for r in rates), rates


def test_rk_slice_runs_and_rejects_the_adjoint(oracle_mod):
    """A whole slice with each Runge-Kutta pusher keeps the charge and stays
    close to the Boris-like slice (same fields, pushes that agree to first
    order); the reverse sweep exists for the Boris-like push only."""
    base = wi.scaled(wi.config("C2"), n_cells=32, half_width=4.0, adaptive=0, dxi0=0.01)
    st0 = wi.synthetic_state(base, seed=3, p_max=0.3, xi=2.0)
    outs = {}
    for pusher in ("boris", "rk1", "rk2", "rk4"):
        cfg = wi.scaled(base, pusher=pusher)
        o = oracle_mod.Oracle(cfg)
        st = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st0.items()}
        r = o.slice_step(st)
        assert r["status"] == 0
        outs[pusher] = np.stack([st["x"], st["y"], st["px"], st["py"]])
        if pusher != "boris":
            stat, _, _ = o.slice_adjoint(st0, st["fields"], [np.zeros_like(st0["x"])] * 4)
            assert stat == oracle_mod.INVALID
    for pusher in ("rk1", "rk2", "rk4"):
        d = np.abs(outs[pusher] - outs["boris"]).max()
        assert d < 5e-4, (pusher, d)
    # the higher orders agree with each other more closely than with the first
    assert np.abs(outs["rk4"] - outs["rk2"]).max() < np.abs(outs["rk4"] - outs["rk1"]).max()
