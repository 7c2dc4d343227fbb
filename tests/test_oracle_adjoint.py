"""Pins of the oracle's reverse-mode slice adjoint (no GPU).

The adjoint is the transpose of the derivative of the discrete slice map; it is
checked against central finite differences of the oracle's forward map
(h = 1e-6), which needs no code of the adjoint: directional derivatives along
random directions in (positions, momenta, driver parameters) with random
weights on every output, and the gradient of a probe loss over a whole run.
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


def _copy(st):
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}


@pytest.mark.parametrize("seed", [1, 2])
def test_slice_adjoint_matches_finite_differences(oracle_mod, seed):
    cfg = _small_cfg()
    N = cfg["n_cells"]
    o = oracle_mod.Oracle(cfg)
    st0 = wi.synthetic_state(cfg, seed=3 + seed, p_max=0.3, xi=2.0)
    th0 = oracle_mod.theta_of(cfg)
    P = st0["x"].size

    def fwd(state, theta):
        oo = oracle_mod.Oracle(oracle_mod.with_theta(cfg, theta))
        s = _copy(state)
        assert oo.slice_step(s)["status"] == 0
        return np.stack([s["x"], s["y"], s["px"], s["py"]]), s["fields"].copy()

    rng = np.random.default_rng(seed)
    abar = rng.standard_normal((4, P))
    Fbar = rng.standard_normal((5, N + 1, N + 1))
    Fbar[:, [0, -1], :] = 0
    Fbar[:, :, [0, -1]] = 0
    _, F0 = fwd(st0, th0)
    stat, ib, tb = o.slice_adjoint(st0, F0, abar, Fbar)
    assert stat == 0 and tb.size == th0.size == 4

    def J(p, F):
        return (abar * p).sum() + (Fbar * F).sum()

    for _ in range(3):
        d = rng.standard_normal((4, P)) * np.array([[0.01], [0.01], [1.0], [1.0]])
        dth = rng.standard_normal(th0.size)
        eps = 1e-6

        def pert(e):
            s = _copy(st0)
            for k, name in enumerate(("x", "y", "px", "py")):
                s[name] = s[name] + e * d[k]
            return fwd(s, th0 + e * dth)

        fd = (J(*pert(eps)) - J(*pert(-eps))) / (2 * eps)
        terms = np.concatenate([(ib[k] * d[k]) for k in range(4)] + [tb * dth])
        ad = terms.sum()
        assert abs(fd - ad) <= 1e-6 * np.abs(terms).sum(), (fd, ad)


def test_run_gradient_matches_finite_differences(oracle_mod):
    """dL/dtheta of a probe loss (mean Ez over a disc and a slice window) for 8
    radial-bin amplitudes, through 40 slices."""
    N, L = 32, 4.0
    h = 2 * L / N
    amps = 0.5 + 1.5 * wi.uniform01(40, 8)
    cfg = wi.scaled(wi.config("C4"), n_cells=N, half_width=L, dxi0=0.05,
                    beams=[wi.radial_bins_beam(amps, 8 * h, 0.8, 1.0)],
                    probes=[dict(field=1, slice_begin=30, slice_end=40, r_max=0.5,
                                 x0=0.0, y0=0.0)])
    th0 = oracle_mod.theta_of(cfg)

    def loss(th, grad=False):
        c = oracle_mod.with_theta(cfg, th)
        return oracle_mod.Oracle(c).run_loss(oracle_mod.initial_state(c), 40, grad=grad)

    st, L0, g = loss(th0, True)
    assert st == 0
    eps = 1e-6
    fd = np.array([(loss(th0 + eps * e)[1] - loss(th0 - eps * e)[1]) / (2 * eps)
                   for e in np.eye(th0.size)])
    assert np.linalg.norm(g - fd) <= 1e-5 * np.linalg.norm(fd), (g, fd)
