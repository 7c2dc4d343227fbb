"""The oracle's results do not depend on its thread count (no GPU).

Every parallel loop of the oracle writes disjoint elements, the deposit gives
each thread a band of node rows that it fills in particle order, and norms are
summed serially, so a run on any number of threads must give the same bits as
a run on one.  Checked on a jittered blowout-like state (particles crowded
across the row bands), for the forward slice, its tangent-linear model and the
reverse sweep.
"""
import numpy as np
import pytest

import wandqs_inputs as wi


@pytest.fixture
def threads(oracle_mod):
    n0 = oracle_mod.get_threads()
    yield oracle_mod.set_threads
    oracle_mod.set_threads(n0)


def _state(cfg):
    st = wi.synthetic_state(cfg, seed=17, p_max=0.6, disp=0.45, xi=1.9, field_amp=0.02)
    # pull a quarter of the particles into a few rows so that band edges fall
    # inside crowded rows
    h = 2 * cfg["half_width"] / cfg["n_cells"]
    st["y"][::4] = np.round(st["y"][::4] / (4 * h)) * 4 * h + 0.3 * h
    return st


def _forward(oracle_mod, cfg, nthreads, n_slices=3):
    oracle_mod.set_threads(nthreads)
    o = oracle_mod.Oracle(cfg)
    st = _state(cfg)
    r = o.run(st, n_slices, keep_fields=True)
    assert r["status"] == 0
    info = [(i.xi, i.dxi, i.vmax, tuple(i.cycles)) for i in r["infos"]]
    return st, r["fields"], info


def test_forward_is_independent_of_threads(oracle_mod, threads):
    cfg = wi.scaled(wi.config("C2"), n_cells=64, half_width=4.0)
    ref_st, ref_F, ref_info = _forward(oracle_mod, cfg, 1)
    for n in (3, 8):
        st, F, info = _forward(oracle_mod, cfg, n)
        assert info == ref_info
        assert np.array_equal(F, ref_F)
        for k in ("x", "y", "px", "py"):
            assert np.array_equal(st[k], ref_st[k]), k


def test_deposit_is_independent_of_threads(oracle_mod, threads):
    cfg = wi.scaled(wi.config("C1"), n_cells=32, half_width=2.0)
    rng = np.random.default_rng(4)
    P = 20000
    x = rng.uniform(-2, 2, P)
    y = np.where(rng.random(P) < 0.5, rng.uniform(-2, 2, P), rng.integers(-16, 16, P) / 8.0)
    q = rng.standard_normal(P)
    threads(1)
    ref = oracle_mod.Oracle(cfg).deposit(x, y, q)
    for n in (2, 5, 7, 33):
        threads(n)
        assert np.array_equal(oracle_mod.Oracle(cfg).deposit(x, y, q), ref), n


def test_tangent_and_adjoint_are_independent_of_threads(oracle_mod, threads):
    cfg = wi.scaled(wi.config("C2"), n_cells=32, half_width=4.0)
    rng = np.random.default_rng(9)
    P = (32 * 2) ** 2
    dP = rng.standard_normal((2, 4, P))
    bars = [rng.standard_normal(P) for _ in range(4)]
    res = []
    for n in (1, 6):
        threads(n)
        o = oracle_mod.Oracle(cfg)
        st = _state(cfg)
        st0 = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in st.items()}
        _, _, _, dout, dF = o.run_tangent(st, 2, dP=dP)
        # reverse of one slice from the same state and its solved fields
        s1 = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in st0.items()}
        o.slice_step(s1)
        stat, ab, tb = o.slice_adjoint(st0, s1["fields"], bars)
        assert stat == 0
        res.append((dout, dF, ab, tb))
    for a, b in zip(res[0], res[1]):
        if isinstance(a, tuple):
            for u, v in zip(a, b):
                assert np.array_equal(u, v)
        else:
            assert np.array_equal(a, b)
