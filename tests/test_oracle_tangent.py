"""Pins of the oracle's tangent-linear model (forward mode, dual numbers) and,
through it, of the hand-written reverse sweep (no GPU).

The tangent-linear run is the same templated slice code instantiated with dual
numbers.  Its value part follows the plain oracle to rounding (its multigrid
solves run until every derivative has converged too, so they may take a cycle
more), and its derivatives must match central finite differences.  The adjoint is the
transpose of the same derivative: <ybar, J xdot> (tangent) equals
<J^T ybar, xdot> (adjoint) to rounding for random directions and weights.
"""
import numpy as np
import pytest

import wandqs_inputs as wi


def _small_cfg():
    cfg = wi.scaled(wi.config("C2"), n_cells=32, half_width=4.0, jitter=0.25, dxi0=0.02,
                    adaptive=0)
    cfg["beams"][0].update(amp=2.0, sigma_r=0.5, sigma_z=0.7)
    cfg["beams"].append(wi.radial_bins_beam([0.3, 0.7, 0.2], 1.2, 0.6, 2.1, x0=0.3))
    return cfg


def _c4_small(n_bins=8):
    N, L = 32, 4.0
    h = 2 * L / N
    amps = 0.5 + 1.5 * wi.uniform01(40, n_bins)
    return wi.scaled(wi.config("C4"), n_cells=N, half_width=L, dxi0=0.05,
                     beams=[wi.radial_bins_beam(amps, n_bins * h, 0.8, 1.0)],
                     probes=[dict(field=1, slice_begin=30, slice_end=40, r_max=0.5, x0=0.0,
                                  y0=0.0)])


def _copy(st):
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}


def test_tangent_values_equal_the_oracle(oracle_mod):
    cfg = _c4_small()
    a = oracle_mod.initial_state(cfg)
    b = _copy(a)
    assert oracle_mod.Oracle(cfg).run(a, 25)["status"] == 0
    st, *_ = oracle_mod.Oracle(cfg).run_tangent(b, 25, dtheta=np.ones((1, 8)))
    assert st == 0
    for k in ("x", "y", "px", "py", "fields"):
        assert np.abs(a[k] - b[k]).max() <= 1e-13 * np.abs(a[k]).max(), k
    assert a["xi"] == b["xi"] and a["dxi"] == b["dxi"]


def test_tangent_matches_finite_differences(oracle_mod):
    """Directional derivatives of the particles and fields after 3 slices from a
    synthetic state, along random particle and parameter directions."""
    cfg = _small_cfg()
    st0 = wi.synthetic_state(cfg, seed=7, p_max=0.3, xi=2.0)
    P = st0["x"].size
    th0 = oracle_mod.theta_of(cfg)
    rng = np.random.default_rng(3)
    dP = rng.standard_normal((2, 4, P)) * np.array([[0.01], [0.01], [1.0], [1.0]])
    dth = rng.standard_normal((2, th0.size))
    s = _copy(st0)
    st, _, _, dout, dF = oracle_mod.Oracle(cfg).run_tangent(s, 3, dP=dP, dtheta=dth)
    assert st == 0
    eps = 1e-6
    for k in range(2):
        def fwd(e):
            c = oracle_mod.with_theta(cfg, th0 + e * dth[k])
            z = _copy(st0)
            for q, name in enumerate(("x", "y", "px", "py")):
                z[name] = z[name] + e * dP[k, q]
            assert oracle_mod.Oracle(c).run(z, 3)["status"] == 0
            return np.stack([z["x"], z["y"], z["px"], z["py"]]), z["fields"]
        (pp, fp), (pm, fm) = fwd(eps), fwd(-eps)
        fd_p, fd_f = (pp - pm) / (2 * eps), (fp - fm) / (2 * eps)
        assert np.abs(dout[k] - fd_p).max() <= 1e-6 * np.abs(fd_p).max(), k
        assert np.abs(dF[k] - fd_f).max() <= 1e-6 * np.abs(fd_f).max(), k


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dot_product_tangent_vs_adjoint_one_slice(oracle_mod, seed):
    """<ybar, J xdot> = <J^T ybar, xdot> for one slice: output weights on the
    particles and all five fields, directions in the particles and theta."""
    cfg = _small_cfg()
    N = cfg["n_cells"]
    st0 = wi.synthetic_state(cfg, seed=10 + seed, p_max=0.3, xi=2.0)
    P = st0["x"].size
    th0 = oracle_mod.theta_of(cfg)
    rng = np.random.default_rng(seed)
    dP = rng.standard_normal((1, 4, P))
    dth = rng.standard_normal((1, th0.size))
    s = _copy(st0)
    st, _, _, dout, dF = oracle_mod.Oracle(cfg).run_tangent(s, 1, dP=dP, dtheta=dth)
    assert st == 0
    abar = rng.standard_normal((4, P))
    Fbar = rng.standard_normal((5, N + 1, N + 1))
    Fbar[:, [0, -1], :] = 0
    Fbar[:, :, [0, -1]] = 0
    so, ib, tb = oracle_mod.Oracle(cfg).slice_adjoint(st0, s["fields"], abar, Fbar)
    assert so == 0
    lhs_terms = np.concatenate([(abar * dout[0]).ravel(), (Fbar * dF[0]).ravel()])
    rhs_terms = np.concatenate([(np.stack(ib) * dP[0]).ravel(), tb * dth[0]])
    lhs, rhs = lhs_terms.sum(), rhs_terms.sum()
    scale = max(np.abs(lhs_terms).sum(), np.abs(rhs_terms).sum())
    print("dot product", lhs, rhs, abs(lhs - rhs) / scale)
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_run_gradient_tangent_equals_adjoint(oracle_mod):
    """dL/dtheta of the probe loss over 40 slices: the 8 unit directions of the
    tangent-linear run against the reverse sweep."""
    cfg = _c4_small()
    st, L_t, dloss, _, _ = oracle_mod.Oracle(cfg).run_tangent(oracle_mod.initial_state(cfg), 40,
                                                              dtheta=np.eye(8))
    assert st == 0
    sa, L_a, g = oracle_mod.Oracle(cfg).run_loss(oracle_mod.initial_state(cfg), 40, grad=True)
    assert sa == 0
    assert abs(L_t - L_a) <= 1e-13 * abs(L_a)
    print("tangent", dloss, "adjoint", g)
    assert np.linalg.norm(dloss - g) <= 1e-10 * np.linalg.norm(g)
