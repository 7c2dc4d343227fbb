"""Pins of the oracle's elliptic solves (no GPU).

The five wakefield equations are 2D Poisson (psi, Ez, Bz: paper Sec. III.B
eqs. (12)-(14)) and Helmholtz-like (B_perp: eq. (18)) problems discretised with
the 5-point Laplacian of Sec. VII.B eq. (33) and solved by multigrid (Sec. II
item 4).  The pins are independent of the oracle's code:

* closed form: the grid functions sin(k pi a/N) sin(l pi b/N) are exact
  eigenvectors of the Dirichlet 5-point Laplacian with eigenvalue
  -(4/h^2)[sin^2(k pi/2N) + sin^2(l pi/2N)];
* a sparse direct solve of a matrix assembled with scipy from Kronecker
  products of the 1D second-difference matrix;
* second-order convergence to a continuous manufactured solution.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _eig(N, h, k, l):
    a = np.arange(N + 1)
    s = np.outer(np.sin(l * np.pi * a / N), np.sin(k * np.pi * a / N))  # [b, a]
    lam = -(4.0 / h**2) * (np.sin(k * np.pi / (2 * N)) ** 2 + np.sin(l * np.pi / (2 * N)) ** 2)
    return s, lam


def _scipy_operator(N, h, k2=None):
    """Dirichlet 5-point operator on the (N-1)^2 interior nodes via Kronecker products."""
    n = N - 1
    d2 = sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1]) / h**2
    I = sp.identity(n)
    A = sp.kron(I, d2) + sp.kron(d2, I)
    if k2 is not None:
        A = A - sp.diags(k2[1:-1, 1:-1].ravel())
    return A.tocsc()


@pytest.mark.parametrize("N", [16, 64])
@pytest.mark.parametrize("kl", [(1, 1), (3, 2), (7, 5)])
def test_poisson_sine_eigenmodes(oracle_mod, N, kl):
    L = 6.0
    h = 2 * L / N
    s, lam = _eig(N, h, *kl)
    st, u, cyc, rel = oracle_mod.mg_solve(N, h, lam * s)
    assert st == 0
    assert np.abs(u - s).max() <= 1e-12 * np.abs(s).max() * max(1.0, abs(lam) * h * h)


@pytest.mark.parametrize("kappa2", [0.5, 7.0, 50.0])
def test_helmholtz_constant_kappa_shift(oracle_mod, kappa2):
    N, L = 32, 4.0
    h = 2 * L / N
    s, lam = _eig(N, h, 2, 3)
    k2 = np.full((N + 1, N + 1), kappa2)
    st, u, cyc, rel = oracle_mod.mg_solve(N, h, (lam - kappa2) * s, k2=k2)
    assert st == 0
    assert np.abs(u - s).max() <= 1e-12


def test_poisson_dense_16(oracle_mod):
    N, L = 16, 3.0
    h = 2 * L / N
    rng = np.random.default_rng(11)
    f = np.zeros((N + 1, N + 1))
    f[1:-1, 1:-1] = rng.standard_normal((N - 1, N - 1))
    ref = np.zeros_like(f)
    ref[1:-1, 1:-1] = spla.spsolve(_scipy_operator(N, h), f[1:-1, 1:-1].ravel()).reshape(N - 1, N - 1)
    st, u, cyc, rel = oracle_mod.mg_solve(N, h, f)
    assert st == 0
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref)


def test_helmholtz_dense_16_random_kappa(oracle_mod):
    N, L = 16, 3.0
    h = 2 * L / N
    rng = np.random.default_rng(12)
    f = np.zeros((N + 1, N + 1))
    f[1:-1, 1:-1] = rng.standard_normal((N - 1, N - 1))
    k2 = rng.uniform(0.0, 50.0, (N + 1, N + 1))
    ref = np.zeros_like(f)
    ref[1:-1, 1:-1] = spla.spsolve(_scipy_operator(N, h, k2), f[1:-1, 1:-1].ravel()).reshape(N - 1, N - 1)
    st, u, cyc, rel = oracle_mod.mg_solve(N, h, f, k2=k2)
    assert st == 0
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref)


def test_apply_matches_scipy_operator(oracle_mod):
    N, L = 16, 2.0
    h = 2 * L / N
    rng = np.random.default_rng(13)
    u = np.zeros((N + 1, N + 1))
    u[1:-1, 1:-1] = rng.standard_normal((N - 1, N - 1))
    k2 = rng.uniform(0.0, 5.0, (N + 1, N + 1))
    out = oracle_mod.apply(N, h, u, k2)
    ref = (_scipy_operator(N, h, k2) @ u[1:-1, 1:-1].ravel()).reshape(N - 1, N - 1)
    assert np.abs(out[1:-1, 1:-1] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(out[0] == 0) and np.all(out[-1] == 0)


def _manufactured(N, L, helm):
    h = 2 * L / N
    g = -L + h * np.arange(N + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    a, b = np.pi / (2 * L), np.pi / L
    u = np.sin(a * (X + L)) * np.sin(b * (Y + L)) * np.exp(X)
    lap = np.exp(X) * np.sin(b * (Y + L)) * ((1 - a * a - b * b) * np.sin(a * (X + L)) +
                                              2 * a * np.cos(a * (X + L)))
    k2 = 1.0 + X * X if helm else None
    f = lap - (k2 * u if helm else 0.0)
    return h, u, f, k2


@pytest.mark.parametrize("helm", [False, True])
def test_second_order_convergence(oracle_mod, helm):
    L = 1.5
    errs = []
    for N in (16, 32, 64):
        h, u, f, k2 = _manufactured(N, L, helm)
        st, v, cyc, rel = oracle_mod.mg_solve(N, h, f, k2=k2)
        assert st == 0
        errs.append(np.abs(v - u).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, errs


def test_vcycle_contraction_and_initial_guess(oracle_mod):
    """V(2,2) cycles reduce the residual by well over 10x each; a good initial
    guess (the previous slice's field, Sec. VII.A) needs fewer cycles."""
    N, L = 128, 6.0
    h = 2 * L / N
    rng = np.random.default_rng(3)
    f = np.zeros((N + 1, N + 1))
    f[1:-1, 1:-1] = rng.standard_normal((N - 1, N - 1))
    st, u, cyc, rel = oracle_mod.mg_solve(N, h, f, rtol=1e-10, atol=0.0)
    assert st == 0 and cyc <= 10
    st2, u2, cyc2, rel2 = oracle_mod.mg_solve(N, h, f * 1.001, u0=u, rtol=1e-10, atol=0.0)
    assert st2 == 0 and cyc2 < cyc


def test_noconv_reported(oracle_mod):
    N, L = 64, 6.0
    h = 2 * L / N
    f = np.zeros((N + 1, N + 1))
    f[1:-1, 1:-1] = 1.0
    st, u, cyc, rel = oracle_mod.mg_solve(N, h, f, rtol=1e-30, atol=0.0, max_cycles=1)
    assert st == oracle_mod.NOCONV and cyc == 1


@pytest.mark.parametrize("helm", [False, True])
def test_zero_rhs_with_nonzero_guess(oracle_mod, helm):
    """f = 0 has the solution 0: from a nonzero initial guess the solve must stop
    (relative to the initial residual) with u ~ rtol * |u0|, not run out of cycles."""
    N, L = 64, 6.0
    h = 2 * L / N
    rng = np.random.default_rng(5)
    u0 = np.zeros((N + 1, N + 1))
    u0[1:-1, 1:-1] = rng.standard_normal((N - 1, N - 1))
    k2 = rng.uniform(0.0, 30.0, (N + 1, N + 1)) if helm else None
    st, u, cyc, rel = oracle_mod.mg_solve(N, h, np.zeros_like(u0), u0=u0, k2=k2)
    assert st == 0 and cyc < 30
    assert np.abs(u).max() <= 1e-12 * np.abs(u0).max()


@pytest.mark.parametrize("helm", [False, True])
@pytest.mark.parametrize("smooth", [False, True])
def test_stop_at_rounding_floor(oracle_mod, helm, smooth):
    """With a tolerance below reach (rtol 1e-16) the floor tests of the stop
    rule end the solve at the rounding floor, not before: one more V-cycle from
    the returned iterate reduces ||r|| by less than 2x.  And not much later:
    the stop comes at most one cycle after the last cycle that still reduced
    ||r|| by more than 2x (the stagnation test needs that one cycle when the
    backward-error test does not fire at the first cycle on the floor)."""
    N, L = 128, 6.0
    h = 2 * L / N
    rng = np.random.default_rng(11)
    if smooth:
        x = np.linspace(-L, L, N + 1)
        X, Y = np.meshgrid(x, x)
        f = np.exp(-(X ** 2 + Y ** 2) / 0.7)
    else:
        f = rng.standard_normal((N + 1, N + 1))
    f[[0, -1], :] = 0
    f[:, [0, -1]] = 0
    k2 = rng.uniform(0.0, 30.0, (N + 1, N + 1)) if helm else None
    A = _scipy_operator(N, h, k2)

    def rnorm(u):
        return np.linalg.norm(f[1:-1, 1:-1].ravel() - A @ u[1:-1, 1:-1].ravel())

    st, u, cyc, _ = oracle_mod.mg_solve(N, h, f, k2=k2, rtol=1e-16)
    assert st == 0 and cyc >= 3
    _, u_prev2, _, _ = oracle_mod.mg_solve(N, h, f, k2=k2, rtol=0.0, max_cycles=cyc - 2)
    _, u_prev, _, _ = oracle_mod.mg_solve(N, h, f, k2=k2, rtol=0.0, max_cycles=cyc - 1)
    _, u_more, c1, _ = oracle_mod.mg_solve(N, h, f, u0=u, k2=k2, rtol=0.0, max_cycles=1)
    assert c1 == 1
    r_prev2, r_prev, r_stop, r_more = rnorm(u_prev2), rnorm(u_prev), rnorm(u), rnorm(u_more)
    print(f"cycles {cyc}: ||r|| {r_prev2:.3e} -> {r_prev:.3e} -> {r_stop:.3e} -> {r_more:.3e}")
    assert r_more > 0.5 * r_stop
    assert r_stop < 0.5 * r_prev or r_prev < 0.5 * r_prev2


def test_vcycle_rate_is_textbook(oracle_mod):
    """V(2,2) cycles of red-black Gauss-Seidel with full weighting and bilinear
    prolongation reduce the residual of the Poisson model problem by a factor
    of 0.04-0.07 per cycle (the textbook rate of this cycle, e.g. Trottenberg,
    Oosterlee & Schueller, Multigrid, Sec. 4.6, about 0.05); a plainer cycle
    (V(1,1)) is slower."""
    N, L = 128, 8.0
    h = 2 * L / N
    rng = np.random.default_rng(1)
    f = np.zeros((N + 1, N + 1))
    f[1:-1, 1:-1] = rng.standard_normal((N - 1, N - 1))
    A = _scipy_operator(N, h)

    def rate(nu):
        r = []
        for m in (4, 5, 6):
            _, u, _, _ = oracle_mod.mg_solve(N, h, f, rtol=0.0, max_cycles=m, nu1=nu, nu2=nu)
            r.append(np.linalg.norm(f[1:-1, 1:-1].ravel() - A @ u[1:-1, 1:-1].ravel()))
        return max(r[1] / r[0], r[2] / r[1])

    r22, r11 = rate(2), rate(1)
    print(f"rate per cycle: V(2,2) {r22:.4f}, V(1,1) {r11:.4f}")
    assert 0.04 <= r22 <= 0.07
    assert r11 > r22
