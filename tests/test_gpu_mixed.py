"""Mixed-precision form (FP32 V-cycles inside FP64 defect correction) against
the FP64 CPU oracle.  There is no separate mixed oracle: the mixed path must
stay within 1e-6 relative per field of the FP64 oracle, and, solved to the
rounding floor, it reaches the FP64 answer (iterative refinement).
"""
import numpy as np
import pytest

import wandqs_inputs as wi
from parity import FIELD_TOL, check_fields, rel

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _sim(cfg, n_slices=1):
    from paper_2012_00881_amd import Simulation
    print(f"[case] mixed N={cfg['n_cells']} rtol={cfg['mg_rtol']} inner={cfg.get('mg_inner_cycles', 0)}",
          flush=True)
    return Simulation(cfg, n_slices=n_slices)


def _particles(st):
    return np.stack([st["x"], st["y"], st["px"], st["py"]])


@pytest.mark.parametrize("N", [64, 256, 1024])
@pytest.mark.parametrize("helm", [False, True])
@pytest.mark.parametrize("inner", [1, 2, 3])
def test_mixed_mg_reaches_fp64_solution(torch_cuda, oracle_mod, N, helm, inner):
    L = 8.0
    h = 2 * L / N
    cfg = wi.scaled(wi.config("C2"), n_cells=N, half_width=L, precision="mixed",
                    mg_inner_cycles=inner)
    sim = _sim(cfg)
    rng = np.random.default_rng(N + inner)
    f = np.zeros((2, N + 1, N + 1))
    f[:, 1:-1, 1:-1] = rng.standard_normal((2, N - 1, N - 1))
    k2 = rng.uniform(0.0, 30.0, (N + 1, N + 1)) if helm else None
    st, u, cyc, relres = sim.mg_solve(f, k2=k2)
    assert st == 0, (st, cyc, relres)
    u = u.cpu().numpy()
    for r in range(2):
        so, ref, co, _ = oracle_mod.mg_solve(N, h, f[r], k2=k2)
        assert so == 0
        assert rel(u[r], ref) <= 1e-12, (r, rel(u[r], ref), cyc, co)
    sim.close()


@pytest.mark.parametrize("rtol,tol", [(1e-14, FIELD_TOL), (1e-9, MIXED_TOL)])
def test_mixed_slice_matches_oracle(torch_cuda, oracle_mod, rtol, tol):
    cfg = wi.scaled(wi.config("C3"), precision="mixed", mg_rtol=rtol)
    state = wi.synthetic_state(cfg, seed=21, p_max=0.5, xi=2.0, field_amp=0.01)
    ocfg = wi.scaled(cfg, precision="fp64", mg_rtol=1e-14)
    orc = oracle_mod.Oracle(ocfg)
    ost = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in state.items()}
    assert orc.slice_step(ost)["status"] == 0
    sim = _sim(cfg)
    sim.set_state(particles=_particles(state), fields=state["fields"], xi=state["xi"],
                  dxi=state["dxi"])
    F, info = sim.step(fields=True, info=True)
    print("outer iterations", info["vcycles"])
    check_fields(F.cpu().numpy(), ost["fields"], tol, "mixed slice")
    p = sim.get_state()["particles"].cpu().numpy()
    assert np.abs(p - _particles(ost)).max() <= 100 * tol
    sim.close()


def test_mixed_run_c3_start(torch_cuda, oracle_mod):
    """First 60 slices of the driver + witness case in the mixed form."""
    n = 60
    cfg = wi.scaled(wi.config("C3"), precision="mixed", mg_rtol=1e-9)
    ocfg = wi.scaled(cfg, precision="fp64", mg_rtol=1e-14)
    orc = oracle_mod.Oracle(ocfg)
    st = oracle_mod.initial_state(ocfg)
    assert orc.run(st, n)["status"] == 0
    sim = _sim(cfg, n)
    sim.run(n)
    got = sim.get_state()
    check_fields(got["fields"].cpu().numpy(), st["fields"], MIXED_TOL, "mixed C3 run")
    assert abs(got["xi"] - st["xi"]) <= 1e-9
    sim.close()


@pytest.mark.parametrize("name", ["C3", "C5"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_slice_at_forms_tolerance_matches_oracle(torch_cuda, oracle_mod, name, precision):
    """One slice of the full C3 (512^2) and C5 (1024^2, 4.2M particles) grids
    at the multigrid tolerance the benchmark's FP64-vs-mixed comparison uses,
    in both forms, against the oracle solved to the rounding floor: every
    field within 1e-6 (L2 and node by node)."""
    cfg = wi.scaled(wi.config(name), precision=precision, mg_rtol=wi.FORMS_RTOL)
    state = wi.synthetic_state(cfg, seed=23, p_max=0.5, xi=2.0, field_amp=0.01)
    ocfg = wi.scaled(cfg, precision="fp64", mg_rtol=1e-14)
    ost = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in state.items()}
    assert oracle_mod.Oracle(ocfg).slice_step(ost)["status"] == 0
    sim = _sim(cfg)
    sim.set_state(particles=_particles(state), fields=state["fields"], xi=state["xi"],
                  dxi=state["dxi"])
    F, info = sim.step(fields=True, info=True)
    print(name, precision, "cycles", info["vcycles"])
    check_fields(F.cpu().numpy(), ost["fields"], MIXED_TOL, f"{name} {precision} @ rtol {wi.FORMS_RTOL}")
    sim.close()
