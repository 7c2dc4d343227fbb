"""The non-uniform grid multigrid (Sec. VII.B) through the C ABI against the
oracle: both solve L u = R J to the rounding floor, so the solutions agree to
1e-10 of their largest value, on grids whose spacing jumps by 2x and 3x (the
paper's three regions) and on a smoothly stretched one, for the Poisson form
(M = 0) and the Helmholtz form (M = -n*/(1+psi) < 0), at sizes whose solve
runs in the coarse workgroup alone (16^2, 64^2) and with levels above it
(256^2, 512^2); a uniform grid gives the context's own 5-point solve.  The
four-colour point smoother needs up to ~120 cycles here (white-noise sources,
cells of aspect ratio up to 3), hence mg_max_cycles = 200."""
import numpy as np
import pytest

import wandqs_inputs as wi

pytestmark = pytest.mark.gpu

L = 4.0
TOL = 1e-10


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _problem(N, kind, seed):
    X = wi.nonuniform_axis(N, L, kind)
    Y = wi.nonuniform_axis(N, 1.2 * L, "smooth" if kind == "regions" else "regions")
    u = wi.uniform01(seed, 3 * (N + 1) ** 2).reshape(3, N + 1, N + 1)
    J = u[0] - 0.5
    M = -(0.5 + 3.0 * u[1])
    u0 = 0.1 * (u[2] - 0.5)
    return X, Y, J, M, u0


@pytest.mark.parametrize("N", [16, 64, 256, 512])
@pytest.mark.parametrize("kind", ["regions", "smooth"])
@pytest.mark.parametrize("helm", [False, True])
def test_nu_solve_matches_oracle(torch_cuda, oracle_mod, N, kind, helm):
    from paper_2012_00881_amd import Simulation
    if N == 512 and not (kind == "regions" and helm):
        pytest.skip("one large case")
    print(f"[case] non-uniform solve N={N} {kind} {'helmholtz' if helm else 'poisson'}", flush=True)
    X, Y, J, M, u0 = _problem(N, kind, 50 + N)
    m = M if helm else None
    so, ref, co, _ = oracle_mod.nu_mg_solve(X, Y, J, u0=u0, M=m, max_cycles=200)
    assert so == 0
    sim = Simulation(wi.scaled(wi.config("C1"), n_cells=N, half_width=L, mg_max_cycles=200))
    st, u, cyc, rel = sim.nu_mg_solve(X, Y, J, u0=u0, M=m)
    assert st == 0, (st, cyc, rel)
    u = u.cpu().numpy()
    err = np.abs(u - ref).max() / np.abs(ref).max()
    print(f"cycles gpu {cyc} oracle {co}, rel residual {rel:.2e}, error {err:.2e}", flush=True)
    assert err <= TOL
    sim.close()


def test_uniform_grid_equals_the_five_point_solve(torch_cuda):
    from paper_2012_00881_amd import Simulation
    N = 128
    X = np.linspace(-L, L, N + 1)
    _, _, J, M, _ = _problem(N, "regions", 7)
    sim = Simulation(wi.scaled(wi.config("C1"), n_cells=N, half_width=L))
    st, u, _, _ = sim.nu_mg_solve(X, X, J, M=M)
    assert st == 0
    f = J.copy()
    f[0, :] = f[-1, :] = f[:, 0] = f[:, -1] = 0.0
    st2, v, _, _ = sim.mg_solve(f, k2=-M)  # (L_h - k2) v = f with k2 = -M
    assert st2 == 0
    u, v = u.cpu().numpy(), v.cpu().numpy()[0]
    assert np.abs(u - v).max() <= 1e-11 * np.abs(v).max()
    sim.close()


def test_bad_coordinates_rejected(torch_cuda):
    from paper_2012_00881_amd import Simulation, WandQSError
    N = 16
    sim = Simulation(wi.scaled(wi.config("C1"), n_cells=N, half_width=L))
    X = np.linspace(-L, L, N + 1)
    X[5] = X[4]
    with pytest.raises(WandQSError):
        sim.nu_mg_solve(X, np.linspace(-L, L, N + 1), np.zeros((N + 1, N + 1)))
    sim.close()
