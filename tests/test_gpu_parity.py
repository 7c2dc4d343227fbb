"""GPU path (through the C ABI) against the CPU oracle, element by element.

Inputs come from the shared seeded input module only; expected values come from
the oracle only.  Field tolerance: 1e-10 relative per field (FP64 path), both as
the relative L2 error over the interior nodes and node by node (max |difference|
over max |field|); the nine node arrays of the slice (moments, k2 and the B_perp
sources) node by node to 1e-10 of their maximum; particle positions and momenta:
1e-10 absolute (lengths ~ 1/k_p, momenta ~ 1).
"""
import numpy as np
import pytest

import wandqs_inputs as wi
from parity import FIELD_TOL, check_fields, check_node_arrays, field_errors, field_maxabs_errors, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _sim(cfg, n_slices=1):
    from paper_2012_00881_amd import Simulation
    print(f"[case] N={cfg['n_cells']} ppc={cfg['ppc_side']**2} beams={len(cfg['beams'])}",
          flush=True)
    return Simulation(cfg, n_slices=n_slices)


def _particles(st):
    return np.stack([st["x"], st["y"], st["px"], st["py"]])


# ------------------------------------------------------------------ init ----

@pytest.mark.parametrize("name,N", [("C1", 64), ("C2", 64), ("C2", 256), ("C5", 1024)])
def test_initial_lattice_bitwise(torch_cuda, name, N):
    cfg = wi.scaled(wi.config(name), n_cells=N)
    sim = _sim(cfg)
    got = sim.get_state()
    x, y, px, py = wi.plasma_lattice(N, cfg["half_width"], cfg["ppc_side"], cfg["jitter"],
                                     cfg["seed"])
    p = got["particles"].cpu().numpy()
    assert np.array_equal(p[0], x) and np.array_equal(p[1], y)
    assert np.all(p[2] == 0) and np.all(p[3] == 0)
    assert got["xi"] == 0.0 and got["dxi"] == cfg["dxi0"]
    assert float(got["fields"].abs().max()) == 0.0
    sim.close()


# -------------------------------------------------------------- multigrid ---

def _rand_rhs(N, seed, nrhs=1):
    rng = np.random.default_rng(seed)
    f = np.zeros((nrhs, N + 1, N + 1))
    f[:, 1:-1, 1:-1] = rng.standard_normal((nrhs, N - 1, N - 1))
    return f


@pytest.mark.parametrize("N,helm,nrhs", [(N, helm, nrhs) for N in (8, 16, 64, 128, 256, 512, 1024)
                                          for helm in (False, True) for nrhs in (1, 2)]
                         + [(2048, False, 2)])
def test_mg_solve_matches_oracle(torch_cuda, oracle_mod, N, helm, nrhs):
    L = 6.0
    h = 2 * L / N
    cfg = wi.scaled(wi.config("C1"), n_cells=N, half_width=L)
    sim = _sim(cfg)
    f = _rand_rhs(N, 100 + N, nrhs)
    k2 = np.random.default_rng(7).uniform(0.0, 30.0, (N + 1, N + 1)) if helm else None
    u0 = 0.1 * _rand_rhs(N, 200 + N, nrhs)
    st, u, cyc, relres = sim.mg_solve(f, u0=u0, k2=k2)
    assert st == 0, (st, cyc, relres)
    u = u.cpu().numpy()
    for r in range(nrhs):
        so, ref, co, _ = oracle_mod.mg_solve(N, h, f[r], u0=u0[r], k2=k2)
        assert so == 0
        assert rel(u[r], ref) <= 1e-12, (r, rel(u[r], ref), cyc, co)
        assert np.all(u[r][0] == 0) and np.all(u[r][-1] == 0)
        assert np.all(u[r][:, 0] == 0) and np.all(u[r][:, -1] == 0)
    sim.close()


@pytest.mark.parametrize("N", [256, 1024, 2048, 4096])
def test_mg_sine_eigenmode_closed_form(torch_cuda, N):
    """GPU solve of L_h u = lambda s recovers the exact eigenvector s, for two
    right-hand sides at once (a smooth and an oscillating mode): the Poisson
    V-cycles end with the fast sine transform solve on level 1 (FFT lengths
    256 .. 4096)."""
    L = 8.0
    h = 2 * L / N
    a = np.arange(N + 1)
    modes = [(5, 3), (N // 2 + 7, N - 9)]
    s = np.stack([np.outer(np.sin(l * np.pi * a / N), np.sin(k * np.pi * a / N)) for k, l in modes])
    lam = np.array([-(4 / h**2) * (np.sin(k * np.pi / (2 * N)) ** 2 + np.sin(l * np.pi / (2 * N)) ** 2)
                    for k, l in modes])
    cfg = wi.scaled(wi.config("C2"), n_cells=N, half_width=L, ppc_side=1)
    sim = _sim(cfg)
    st, u, cyc, _ = sim.mg_solve(lam[:, None, None] * s)
    assert st == 0
    err = np.abs(u.cpu().numpy() - s).max()
    print(f"N={N}: cycles {cyc}, max error {err:.2e}")
    assert err <= 1e-12
    sim.close()


# ------------------------------------------------------------ one slice -----

SLICE_CASES = [
    ("C1", 8, 31, 0.3),     # smallest grid: particle tiles overhang it, one coarse kernel solves
    ("C1", 16, 32, 0.3),
    ("C1", 64, 1, 0.3),
    ("C2", 128, 11, 0.5),
    ("C2", 256, 12, 0.8),
    ("C3", 512, 13, 0.5),
]


def _compare_slice(torch, oracle_mod, cfg, state):
    orc = oracle_mod.Oracle(cfg)
    ost = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in state.items()}
    r = orc.slice_step(ost, want_moments=True)
    assert r["status"] == 0
    sim = _sim(cfg)
    sim.set_state(particles=_particles(state), fields=state["fields"], xi=state["xi"],
                  dxi=state["dxi"])
    F, info = sim.step(fields=True, info=True)
    mom = sim.moments().cpu().numpy()
    got = sim.get_state()
    F = F.cpu().numpy()
    print("cycles gpu", info["vcycles"], "oracle", list(r["info"].cycles))
    check_fields(F, ost["fields"], FIELD_TOL, "slice")
    ref_mom = np.concatenate([r["moments"], r["extra"][:3]])
    check_node_arrays(mom, ref_mom, 1e-10)
    p = got["particles"].cpu().numpy()
    assert np.abs(p - _particles(ost)).max() <= 1e-10
    assert abs(got["xi"] - ost["xi"]) <= 1e-14 and abs(got["dxi"] - ost["dxi"]) <= 1e-12
    assert abs(info["vmax"] - r["info"].vmax) <= 1e-10 * max(1.0, r["info"].vmax)
    sim.close()


@pytest.mark.parametrize("name,N,seed,pmax", SLICE_CASES)
def test_slice_matches_oracle_synthetic(torch_cuda, oracle_mod, name, N, seed, pmax):
    cfg = wi.scaled(wi.config(name), n_cells=N, precision="fp64")
    state = wi.synthetic_state(cfg, seed=seed, p_max=pmax, xi=2.0, field_amp=0.01)
    _compare_slice(torch_cuda, oracle_mod, cfg, state)


def test_slice_crowded_cells_matches_oracle(torch_cuda, oracle_mod):
    """Cells of more than 16 particles take the crowded-cell path of the sort
    (one workgroup per cell).  Three cells of 40, 24 and 17 particles, spread
    over the particle index range so that the scatter interleaves them, then
    one slice against the oracle; the state after it holds every particle
    exactly once (ID order)."""
    cfg = wi.scaled(wi.config("C2"), n_cells=128, precision="fp64")
    state = wi.synthetic_state(cfg, seed=21, p_max=0.3, xi=2.0, field_amp=0.01)
    N, L = cfg["n_cells"], cfg["half_width"]
    h = 2 * L / N
    rng = np.random.default_rng(5)
    P = state["x"].size
    for (ca, cb), n in (((40, 61), 40), ((41, 61), 24), ((90, 30), 17)):
        idx = rng.choice(P, n, replace=False)
        state["x"][idx] = -L + (ca + rng.uniform(0.05, 0.95, n)) * h
        state["y"][idx] = -L + (cb + rng.uniform(0.05, 0.95, n)) * h
    _compare_slice(torch_cuda, oracle_mod, cfg, state)


def test_slice_matches_oracle_vortex(torch_cuda, oracle_mod):
    cfg = wi.scaled(wi.config("C2"), n_cells=256)
    state = wi.vortex_state(cfg, 0.8, 1.0, xi=2.2)
    _compare_slice(torch_cuda, oracle_mod, cfg, state)


def test_slice_matches_oracle_full_size_c5(torch_cuda, oracle_mod):
    """C5 grid and particle count (1024^2, 4.2M particles), one slice from a
    synthetic state in the driver region."""
    cfg = wi.config("C5")
    state = wi.synthetic_state(cfg, seed=15, p_max=0.5, xi=2.0, field_amp=0.01)
    _compare_slice(torch_cuda, oracle_mod, cfg, state)


def test_slice_matches_oracle_largest_grid(torch_cuda, oracle_mod):
    """The largest grid the library accepts, 4096^2 over the C5 box (twelve
    multigrid levels, four on register tiles), with one particle per cell
    (16.8M particles): one slice from a synthetic state in the driver region."""
    cfg = wi.scaled(wi.config("C5"), n_cells=4096, ppc_side=1, precision="fp64")
    state = wi.synthetic_state(cfg, seed=41, p_max=0.5, xi=2.0, field_amp=0.01)
    _compare_slice(torch_cuda, oracle_mod, cfg, state)


# ------------------------------------------------------------------ runs ----

def test_run_c1_matches_oracle(torch_cuda, oracle_mod):
    """The whole C1 run (128 slices, linear regime), compared after 40 slices
    (driver peak) and at the end."""
    cfg = wi.config("C1")
    orc = oracle_mod.Oracle(cfg)
    st = oracle_mod.initial_state(cfg)
    sim = _sim(cfg, cfg["n_slices"])
    for n in (40, cfg["n_slices"] - 40):
        ro = orc.run(st, n)
        assert ro["status"] == 0
        infos, _ = sim.run(n, infos=True)
        got = sim.get_state()
        check_fields(got["fields"].cpu().numpy(), st["fields"], FIELD_TOL, f"C1 run after {n}")
        assert np.abs(got["particles"].cpu().numpy() - _particles(st)).max() <= 1e-10
        for j in (0, n // 2, n - 1):
            assert abs(infos[j]["xi"] - ro["infos"][j].xi) <= 1e-12
    sim.close()


def test_run_c2_start_matches_oracle(torch_cuda, oracle_mod):
    """First 120 slices of the blowout case (adaptive step, jittered plasma)."""
    cfg = wi.config("C2")
    n = 120
    orc = oracle_mod.Oracle(cfg)
    st = oracle_mod.initial_state(cfg)
    ro = orc.run(st, n)
    assert ro["status"] == 0
    sim = _sim(cfg, n)
    infos, _ = sim.run(n, infos=True)
    got = sim.get_state()
    check_fields(got["fields"].cpu().numpy(), st["fields"], FIELD_TOL, "C2 run start")
    assert np.abs(got["particles"].cpu().numpy() - _particles(st)).max() <= 1e-10
    assert abs(got["xi"] - st["xi"]) <= 1e-10
    sim.close()


def test_run_c2_within_oracle_sensitivity(torch_cuda, oracle_mod):
    """Whole-run parity on the blowout case over 320 slices (xi to 6.4: the
    driver and the first bubble behind it), read against the oracle's own
    sensitivity to rounding.  The oracle runs twice, the second time with
    every initial position moved by 1e-15 h (seeded random signs).  Every 80
    slices the GPU run from the unperturbed start must lie within 10x that
    spread of the unperturbed oracle run, per field and for the particles.
    The spread is floored at the per-slice tolerance, which rounding alone
    can reach over a run.  The two oracle runs share no state and run in two
    threads."""
    import threading
    cfg = wi.config("C2")
    chunk, nch = 80, 4
    h = 2 * cfg["half_width"] / cfg["n_cells"]
    orcs = (oracle_mod.Oracle(cfg), oracle_mod.Oracle(cfg))
    a, b = oracle_mod.initial_state(cfg), oracle_mod.initial_state(cfg)
    rng = np.random.default_rng(7)
    b["x"] = b["x"] + 1e-15 * h * rng.choice([-1.0, 1.0], b["x"].size)
    b["y"] = b["y"] + 1e-15 * h * rng.choice([-1.0, 1.0], b["y"].size)
    sim = _sim(cfg, chunk * nch)
    for k in range(nch):
        status = {}

        def go(key, orc, st):
            status[key] = orc.run(st, chunk)["status"]

        ts = [threading.Thread(target=go, args=(key, orc, st))
              for key, orc, st in (("a", orcs[0], a), ("b", orcs[1], b))]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        assert status == {"a": 0, "b": 0}, status
        sim.run(chunk)
        got = sim.get_state()
        spread = field_errors(b["fields"], a["fields"])
        errs = field_errors(got["fields"].cpu().numpy(), a["fields"])
        mspread = field_maxabs_errors(b["fields"], a["fields"])
        merrs = field_maxabs_errors(got["fields"].cpu().numpy(), a["fields"])
        pa, pb = _particles(a), _particles(b)
        pspread = np.abs(pa - pb).max()
        perr = np.abs(got["particles"].cpu().numpy() - pa).max()
        print("C2 slice", (k + 1) * chunk, "xi", a["xi"], "gpu", errs, "oracle spread", spread,
              "particles", perr, pspread, flush=True)
        assert np.all(errs <= np.maximum(10.0 * spread, FIELD_TOL)), (errs, spread)
        assert np.all(merrs <= np.maximum(10.0 * mspread, FIELD_TOL)), (merrs, mspread)
        assert perr <= max(10.0 * pspread, 1e-10), (perr, pspread)
        assert abs(got["xi"] - a["xi"]) <= 1e-10
    sim.close()


def test_bitwise_deterministic(torch_cuda):
    cfg = wi.scaled(wi.config("C2"), n_cells=128)
    outs = []
    for _ in range(2):
        sim = _sim(cfg, 60)
        sim.run(60)
        g = sim.get_state()
        outs.append((g["particles"].cpu().numpy(), g["fields"].cpu().numpy()))
        sim.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_noconv_is_an_error(torch_cuda):
    """A solve that cannot meet its tolerance within mg_max_cycles (here one
    V-cycle, from a state with a nonzero source) returns WANDQS_E_NOCONV and
    names the solve; the context then refuses to step until set_state, after
    which the same slice fails the same way again.  Every kernel completes:
    the host decides non-convergence from the published norms."""
    from paper_2012_00881_amd import WandQSError
    cfg = wi.scaled(wi.config("C2"), n_cells=64, mg_max_cycles=1)
    state = wi.synthetic_state(cfg, seed=3, p_max=0.3, xi=2.0, field_amp=0.01)
    sim = _sim(cfg)
    for _ in range(2):
        sim.set_state(particles=_particles(state), fields=state["fields"], xi=state["xi"],
                      dxi=state["dxi"])
        with pytest.raises(WandQSError) as e:
            sim.step(info=True)
        assert e.value.status == -4, e.value
        assert "psi solve" in str(e.value), e.value
        with pytest.raises(WandQSError) as e2:
            sim.step()
        assert e2.value.status == -6
    sim.close()


def test_nonphysical_is_an_error(torch_cuda):
    from paper_2012_00881_amd import WandQSError
    cfg = wi.scaled(wi.config("C1"), n_cells=32)
    sim = _sim(cfg)
    st = sim.get_state()
    p = st["particles"].cpu().numpy()
    p[0] = 0.01
    p[1] = -0.01
    sim.set_state(particles=p)
    with pytest.raises(WandQSError) as e:
        sim.step(info=True)
    assert e.value.status == -5
    with pytest.raises(WandQSError) as e2:
        sim.step()
    assert e2.value.status == -6
    sim.close()


def test_run_radial_bins_matches_oracle(torch_cuda, oracle_mod):
    """Radial-bin driver (bin width = h, so bin edges pass through grid nodes)
    over 60 slices, with a probe: fields, particles and the probe value."""
    N, L = 64, 4.0
    h = 2 * L / N
    amps = 0.5 + 1.5 * wi.uniform01(40, 16)
    cfg = wi.scaled(wi.config("C4"), n_cells=N, half_width=L, dxi0=0.05,
                    beams=[wi.radial_bins_beam(amps, 16 * h, 0.8, 1.0)],
                    probes=[dict(field=1, slice_begin=30, slice_end=60, r_max=4 * h, x0=0.0,
                                 y0=0.0)])
    n = 60
    orc = oracle_mod.Oracle(cfg)
    st = oracle_mod.initial_state(cfg)
    so, L0, _ = orc.run_loss(st, n)
    assert so == 0
    sim = _sim(cfg, n)
    _, pr = sim.run(n, probes=True)
    got = sim.get_state()
    print("probe", float(pr[0]), L0)
    check_fields(got["fields"].cpu().numpy(), st["fields"], FIELD_TOL, "radial-bin run")
    assert np.abs(got["particles"].cpu().numpy() - _particles(st)).max() <= 1e-10
    assert abs(float(pr[0]) - L0) <= 1e-10 * max(1.0, abs(L0))
    sim.close()


@pytest.mark.parametrize("N", [32, 256])
@pytest.mark.parametrize("helm", [False, True])
def test_mg_zero_rhs_nonzero_guess(torch_cuda, N, helm):
    """f = 0 from a nonzero guess stops on the initial-residual rule with u ~ 0."""
    L = 6.0
    cfg = wi.scaled(wi.config("C1"), n_cells=N, half_width=L)
    sim = _sim(cfg)
    u0 = _rand_rhs(N, 300 + N, 2)
    k2 = np.random.default_rng(8).uniform(0.0, 30.0, (N + 1, N + 1)) if helm else None
    st, u, cyc, relres = sim.mg_solve(np.zeros_like(u0), u0=u0, k2=k2)
    assert st == 0 and cyc < 30, (st, cyc)
    assert float(u.abs().max()) <= 1e-12 * np.abs(u0).max()
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("helm", [False, True])
def test_register_tiles_bitwise_equal_lds_tiles(torch_cuda, monkeypatch, precision, helm):
    """The register-tile pass kernels of the large levels against the LDS tile
    kernels (WANDQS_MG_TILES=lds), and with both right-hand sides in every
    workgroup (WANDQS_MG_SPLIT=0) against one per workgroup: three fixed
    V-cycles on 1024^2 and 2048^2 give the same bits, and so does a full C5
    slice."""
    outs = []
    for mode in (None, "lds", "fused"):
        monkeypatch.delenv("WANDQS_MG_TILES", raising=False)
        monkeypatch.delenv("WANDQS_MG_SPLIT", raising=False)
        if mode == "lds":
            monkeypatch.setenv("WANDQS_MG_TILES", mode)
        elif mode == "fused":
            monkeypatch.setenv("WANDQS_MG_SPLIT", "0")
        res = []
        for N in (1024, 2048):
            cfg = wi.scaled(wi.config("C1"), n_cells=N, half_width=6.0, mg_rtol=0.0,
                            mg_max_cycles=3, precision=precision)
            sim = _sim(cfg)
            f = _rand_rhs(N, N, 2)
            u0 = 0.1 * _rand_rhs(N, N + 1, 2)
            k2 = np.random.default_rng(7).uniform(0.0, 30.0, (N + 1, N + 1)) if helm else None
            st, u, _, _ = sim.mg_solve(f, u0=u0, k2=k2)
            assert st == 0
            res.append(u.cpu().numpy().copy())
            sim.close()
        if not helm:
            cfg = wi.scaled(wi.config("C5"), mg_rtol=0.0, mg_max_cycles=6, precision=precision)
            state = wi.synthetic_state(cfg, seed=15, p_max=0.5, xi=2.0, field_amp=0.01)
            sim = _sim(cfg)
            sim.set_state(particles=_particles(state), fields=state["fields"], xi=state["xi"],
                          dxi=state["dxi"])
            F, _ = sim.step(fields=True)
            res.append(F.cpu().numpy().copy())
            res.append(sim.get_state()["particles"].cpu().numpy().copy())
            sim.close()
        outs.append(res)
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b), float(np.abs(a - b).max())


def test_fused_passes_bitwise_equal_separate(torch_cuda, monkeypatch):
    """Inside a batch of V-cycles the finest level's up pass and the next
    cycle's down pass run as one fused launch; with WANDQS_MG_FUSE=0 they run
    separately.  Solves to the tolerance (batches of several cycles) on 1024^2
    and 2048^2, Poisson and Helmholtz, and six C5 slices give the same bits,
    cycle counts and residuals."""
    outs = []
    for fuse in (None, "0"):
        monkeypatch.delenv("WANDQS_MG_FUSE", raising=False)
        if fuse is not None:
            monkeypatch.setenv("WANDQS_MG_FUSE", fuse)
        res = []
        for N in (1024, 2048):
            for helm in (False, True):
                cfg = wi.scaled(wi.config("C1"), n_cells=N, half_width=6.0)
                sim = _sim(cfg)
                f = _rand_rhs(N, N + 3, 2)
                k2 = np.random.default_rng(9).uniform(0.0, 30.0, (N + 1, N + 1)) if helm else None
                # the second solve's first batch is the first's cycle count
                for rep in range(2):
                    u0 = 0.1 * _rand_rhs(N, N + 4 + rep, 2)
                    st, u, cyc, rr = sim.mg_solve(f, u0=u0, k2=k2)
                    assert st == 0
                    print(f"fuse={fuse} N={N} helm={helm}: cycles {cyc}")
                    res += [u.cpu().numpy().copy(), np.array([cyc]), np.array(rr)]
                sim.close()
        cfg = wi.config("C5")
        state = wi.synthetic_state(cfg, seed=17, p_max=0.5, xi=2.0, field_amp=0.01)
        sim = _sim(cfg, n_slices=6)
        sim.set_state(particles=_particles(state), fields=state["fields"], xi=state["xi"],
                      dxi=state["dxi"])
        infos, _ = sim.run(6, infos=True)
        got = sim.get_state()
        res += [got["fields"].cpu().numpy().copy(), got["particles"].cpu().numpy().copy(),
                np.array([i["vcycles"] for i in infos])]
        print(f"fuse={fuse} C5 cycles", [i["vcycles"] for i in infos])
        sim.close()
        outs.append(res)
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b), float(np.abs(a - b).max())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_bitwise_equal_direct_launches(torch_cuda, monkeypatch, precision):
    """Multigrid cycles replayed as HIP graphs (WANDQS_GRAPHS=1) against
    direct launches: the first 48 slices of the 512^2 case in tolerance mode
    replay every captured cycle many times, with the particle kernels and the
    host's norm reads between replays, and give the same bits, the same cycle
    counts and the same steps."""
    outs = []
    for mode in ("1", None):
        if mode:
            monkeypatch.setenv("WANDQS_GRAPHS", mode)
        else:
            monkeypatch.delenv("WANDQS_GRAPHS", raising=False)
        cfg = wi.scaled(wi.config("C3"), precision=precision)
        sim = _sim(cfg, 48)
        infos, _ = sim.run(48, infos=True)
        got = sim.get_state()
        outs.append((got["fields"].cpu().numpy().copy(), got["particles"].cpu().numpy().copy(),
                     [(i["xi"], i["dxi"], tuple(i["vcycles"])) for i in infos]))
        sim.close()
    (fa, pa, ia), (fb, pb, ib) = outs
    assert np.array_equal(fa, fb), float(np.abs(fa - fb).max())
    assert np.array_equal(pa, pb), float(np.abs(pa - pb).max())
    assert ia == ib


# ------------------------------------------------------------- pushers ------

@pytest.mark.parametrize("pusher", ["rk1", "rk2", "rk4"])
@pytest.mark.parametrize("name,N", [("C2", 256), ("C5", 1024)])
def test_slice_rk_pushers_match_oracle(torch_cuda, oracle_mod, pusher, name, N):
    """The Runge-Kutta pushers (every stage gathers at its own position) on the
    C2 and C5 grids: one slice from a synthetic state against the oracle."""
    cfg = wi.scaled(wi.config(name), n_cells=N, precision="fp64", pusher=pusher)
    state = wi.synthetic_state(cfg, seed=17, p_max=0.5, xi=2.0, field_amp=0.01)
    _compare_slice(torch_cuda, oracle_mod, cfg, state)


@pytest.mark.parametrize("pusher", ["rk2", "rk4"])
def test_run_c2_start_rk_matches_oracle(torch_cuda, oracle_mod, pusher):
    """The first 80 slices of the blowout case (adaptive step) with a
    Runge-Kutta pusher."""
    cfg = wi.scaled(wi.config("C2"), pusher=pusher)
    n = 80
    orc = oracle_mod.Oracle(cfg)
    st = oracle_mod.initial_state(cfg)
    assert orc.run(st, n)["status"] == 0
    sim = _sim(cfg, n)
    sim.run(n)
    got = sim.get_state()
    check_fields(got["fields"].cpu().numpy(), st["fields"], FIELD_TOL, f"C2 run {pusher}")
    assert np.abs(got["particles"].cpu().numpy() - _particles(st)).max() <= 1e-10
    assert abs(got["xi"] - st["xi"]) <= 1e-10
    sim.close()
