"""The laser envelope driver through the C ABI against the oracle.

* the envelope's time step (eq. (20), complex multigrid) plane by plane:
  wandqs_laser_advance against the oracle's oracle_laser_advance, on grids
  whose solve runs in the single workgroup alone (16^2), with one tile level
  above it (64^2) and with several (256^2), in vacuum and with a
  susceptibility chi; both sides converge to the rounding floor, so the planes
  agree to 1e-10 of their largest value;
* slices with a frozen envelope (the ponderomotive terms in the push, in j_z
  and in S), Boris-like and RK4 pushers: fields to 1e-10 (both field
  measures), particles to 1e-10;
* the time loop with a laser: each plane advanced right after its slice with
  that slice's chi, two steps: envelope, fields and particles as above; with
  driver particles pushed through the laser's fields in 16 sub-steps: their
  positions to 1e-10, momenta to 1e-9 of their largest change.
"""
import numpy as np
import pytest

import wandqs_inputs as wi
from parity import FIELD_TOL, check_fields

pytestmark = pytest.mark.gpu

ENV_TOL = 1e-10


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _cfg(N, L, nz, k0, **kw):
    base = dict(beams=[], adaptive=0, laser_nz=nz, laser_k0=k0)
    base.update(kw)
    return wi.scaled(wi.config("C1"), n_cells=N, half_width=L, **base)


def _env_err(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("N", [16, 64, 256])
@pytest.mark.parametrize("medium", ["vacuum", "plasma"])
def test_envelope_advance_matches_oracle(torch_cuda, oracle_mod, N, medium):
    from paper_2012_00881_amd import Simulation
    L, nz, k0, dxi, dt = 6.0, 12, 5.0, 0.25, 2.0
    print(f"[case] envelope advance N={N} {medium}", flush=True)
    cfg = _cfg(N, L, nz, k0, dxi0=dxi)
    env = wi.laser_gaussian(N, L, nz, dxi, 0.8, 1.5, 1.5, 0.8)
    chi = None
    if medium == "plasma":
        u = wi.uniform01(31 + N, nz * (N + 1) ** 2).reshape(nz, N + 1, N + 1)
        chi = 2.0 * u
    o = oracle_mod.Oracle(cfg)
    sim = Simulation(cfg)
    sim.laser_set(env)
    ref = env
    for step in range(2):
        st, ref, cyc_o = o.laser_advance(dt, ref, chi, k0=k0)
        assert st == 0
        cyc = sim.laser_advance(dt, chi)
        got = sim.laser_get().cpu().numpy()
        e = _env_err(got, ref)
        print(f"step {step}: envelope error {e:.2e}, cycles gpu {cyc[:4]} oracle {list(cyc_o[:4])}",
              flush=True)
        assert e <= ENV_TOL
    sim.close()


@pytest.mark.parametrize("N,pusher", [(64, "boris"), (64, "rk4"), (256, "boris")])
def test_frozen_laser_slices_match_oracle(torch_cuda, oracle_mod, N, pusher):
    from paper_2012_00881_amd import Simulation
    L, dxi = 6.0, 0.05
    nz, n = 90, 60
    print(f"[case] frozen laser slices N={N} {pusher}", flush=True)
    cfg = _cfg(N, L, nz, 10.0, dxi0=dxi, ppc_side=2, pusher=pusher)
    env = wi.laser_gaussian(N, L, nz, dxi, 0.6, 1.5, 1.5, 0.6)
    o = oracle_mod.Oracle(cfg)
    o.set_laser(env, 10.0)
    st = oracle_mod.initial_state(cfg)
    r = o.run(st, n)
    assert r["status"] == 0
    sim = Simulation(cfg, n_slices=n)
    sim.laser_set(env)
    sim.run(n)
    got = sim.get_state()
    check_fields(got["fields"].cpu().numpy(), st["fields"], FIELD_TOL, f"laser slices N={N}")
    parts = got["particles"].cpu().numpy()
    d = np.abs(parts - np.stack([st["x"], st["y"], st["px"], st["py"]])).max()
    print("particles", d)
    assert d <= 1e-10
    # the laser is felt: the wake differs from the laser-free plasma's (zero)
    assert np.abs(st["fields"][0]).max() > 1e-3
    sim.close()


def test_time_step_with_laser_matches_oracle(torch_cuda, oracle_mod):
    from paper_2012_00881_amd import Simulation
    N, L, dxi, nz, k0, dt = 64, 6.0, 0.1, 40, 8.0, 5.0
    print("[case] time loop with a laser N=64", flush=True)
    cfg = _cfg(N, L, nz, k0, dxi0=dxi, ppc_side=2)
    env = wi.laser_gaussian(N, L, nz, dxi, 0.7, 1.5, 1.8, 0.6)
    o = oracle_mod.Oracle(cfg)
    o.set_laser(env, k0)
    sim = Simulation(cfg, n_slices=nz)
    sim.laser_set(env)
    none = np.zeros((8, 0))
    for step in range(2):
        st = oracle_mod.initial_state(cfg)
        r = o.time_step(st, none, nz, dt, 2, 0.0, 1.0)
        assert r["status"] == 0
        infos = sim.time_step(dt, nz, infos=True)
        got = sim.get_state()
        check_fields(got["fields"].cpu().numpy(), st["fields"], FIELD_TOL, f"laser time step {step}")
        parts = got["particles"].cpu().numpy()
        assert np.abs(parts - np.stack([st["x"], st["y"], st["px"], st["py"]])).max() <= 1e-10
        e = _env_err(sim.laser_get().cpu().numpy(), o.laser_env)
        print(f"step {step}: envelope error {e:.2e}, laser cycles "
              f"{[i['laser_vcycles'] for i in infos[:5]]}", flush=True)
        assert e <= ENV_TOL
        assert all(i["laser_vcycles"] > 0 for i in infos)
    sim.close()


def test_laser_time_step_needs_fixed_steps(torch_cuda):
    from paper_2012_00881_amd import Simulation, WandQSError
    N, nz = 32, 8
    cfg = _cfg(N, 6.0, nz, 5.0, dxi0=0.1, adaptive=1)
    sim = Simulation(cfg, n_slices=nz)
    sim.laser_set(wi.laser_gaussian(N, 6.0, nz, 0.1, 0.5, 1.5, 0.3, 0.3))
    with pytest.raises(WandQSError):
        sim.time_step(1.0, nz)
    sim.close()
    cfg = _cfg(N, 6.0, nz, 5.0, dxi0=0.1)
    sim = Simulation(cfg, n_slices=nz)
    with pytest.raises(WandQSError):  # no envelope set
        sim.laser_advance(1.0)
    sim.laser_set(wi.laser_gaussian(N, 6.0, nz, 0.1, 0.5, 1.5, 0.3, 0.3))
    with pytest.raises(WandQSError):  # fewer slices than planes
        sim.time_step(1.0, nz - 1)
    sim.close()


def test_time_step_laser_and_subcycled_driver_match_oracle(torch_cuda, oracle_mod):
    """Driver particles inside the laser (gamma 30): the push adds the laser's
    fields from the planes at t and t + dt in 16 sub-steps (Sec. IV)."""
    from paper_2012_00881_amd import Simulation
    N, L, dxi, nz, k0, dt = 64, 6.0, 0.1, 40, 8.0, 4.0
    print("[case] time loop, laser and sub-cycled driver N=64", flush=True)
    beam = wi.gauss_beam(0.05, 0.8, 0.4, 1.8)
    drv = wi.driver_gaussian(beam, 20_000, 41, gamma0=30.0)
    cfg = _cfg(N, L, nz, k0, dxi0=dxi, ppc_side=2, driver_max=drv.shape[1], driver_nz=45,
               driver_xi0=-0.1, driver_dz=0.1, driver_nsub=16)
    env = wi.laser_gaussian(N, L, nz, dxi, 0.7, 1.5, 1.8, 0.6)
    o = oracle_mod.Oracle(cfg)
    o.set_laser(env, k0)
    sim = Simulation(cfg, n_slices=nz)
    sim.laser_set(env)
    sim.driver_set(drv)
    d_orc = drv.copy()
    for step in range(2):
        st = oracle_mod.initial_state(cfg)
        r = o.time_step(st, d_orc, nz, dt, cfg["driver_nz"], cfg["driver_xi0"], cfg["driver_dz"])
        assert r["status"] == 0
        sim.time_step(dt, nz)
        got = sim.get_state()
        check_fields(got["fields"].cpu().numpy(), st["fields"], FIELD_TOL, f"laser+driver step {step}")
        e = _env_err(sim.laser_get().cpu().numpy(), o.laser_env)
        d_gpu = sim.driver_get().cpu().numpy()
        dpos = np.abs(d_gpu[:3] - d_orc[:3]).max()
        scale = np.abs(d_orc[3:6] - drv[3:6]).max()
        dmom = np.abs(d_gpu[3:6] - d_orc[3:6]).max()
        print(f"step {step}: envelope {e:.2e}, driver positions {dpos:.2e}, momenta {dmom:.2e} "
              f"(largest change {scale:.3e})", flush=True)
        assert e <= ENV_TOL
        assert dpos <= 1e-10
        assert dmom <= 1e-9 * scale
    # the laser's oscillating field moves the particles: p_x (the polarisation)
    # quivers by about a0, more than the wake moves p_y
    dpx, dpy = np.abs(d_orc[3] - drv[3]).max(), np.abs(d_orc[4] - drv[4]).max()
    assert dpx > 0.5 and dpx > 1.3 * dpy
    sim.close()
