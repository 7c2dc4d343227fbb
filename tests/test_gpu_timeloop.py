"""The time loop (driver macroparticles, wandqs_time_step) through the C ABI
against the oracle's oracle_time_step.

Each step deposits the driver's current, sweeps the cold plasma through the
slices with it and pushes the driver by dt through the wake.  Compared: the
fields and plasma particles after the sweep (1e-10, as the slice parity) and
the driver particles after the push: positions to 1e-10 absolute, momentum
changes to 1e-9 of their largest size.
"""
import numpy as np
import pytest

import wandqs_inputs as wi
from parity import FIELD_TOL, check_fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(name, N, amp, n_drv, seed, dz, xi0, nz, quiet=False, **kw):
    base = wi.scaled(wi.config(name), n_cells=N, **kw)
    beam = dict(base["beams"][0], amp=amp)
    if quiet:
        drv = wi.driver_lattice(beam, N, base["half_width"], xi0, dz, nz, gamma0=2000.0)
    else:
        drv = wi.driver_gaussian(beam, n_drv, seed, gamma0=2000.0)
    cfg = wi.scaled(base, beams=[], driver_max=max(drv.shape[1], 1), driver_nz=nz,
                    driver_xi0=xi0, driver_dz=dz)
    return cfg, beam, drv


def _compare_steps(torch, oracle_mod, cfg, drv, n_slices, dt, n_steps):
    from paper_2012_00881_amd import Simulation
    print(f"[case] time loop N={cfg['n_cells']} driver={drv.shape[1]} slices={n_slices} "
          f"dt={dt} steps={n_steps}", flush=True)
    orc = oracle_mod.Oracle(cfg)
    sim = Simulation(cfg, n_slices=n_slices)
    sim.driver_set(drv)
    d_orc = drv.copy()
    for step in range(n_steps):
        st = oracle_mod.initial_state(cfg)
        r = orc.time_step(st, d_orc, n_slices, dt, cfg["driver_nz"], cfg["driver_xi0"],
                          cfg["driver_dz"])
        assert r["status"] == 0
        sim.time_step(dt, n_slices)
        got = sim.get_state()
        check_fields(got["fields"].cpu().numpy(), st["fields"], FIELD_TOL, f"time step {step}")
        parts = got["particles"].cpu().numpy()
        assert np.abs(parts - np.stack([st["x"], st["y"], st["px"], st["py"]])).max() <= 1e-10
        d_gpu = sim.driver_get().cpu().numpy()
        dpos = np.abs(d_gpu[:3] - d_orc[:3]).max()
        dp_ref = d_orc[3:6] - drv[3:6] if step == 0 else None
        dmom = np.abs(d_gpu[3:6] - d_orc[3:6]).max()
        scale = np.abs(d_orc[3:6] - drv[3:6]).max()
        print(f"step {step}: driver positions {dpos:.2e}, momenta {dmom:.2e} (largest change "
              f"{scale:.3e})", flush=True)
        assert dpos <= 1e-10
        assert dmom <= 1e-9 * max(scale, 1e-300)
        assert np.array_equal(d_gpu[6:], d_orc[6:])
    sim.close()
    return d_orc


def test_time_step_c1_sampled_driver(torch_cuda, oracle_mod):
    """Linear regime (64^2): 20,000 sampled driver particles of 5x the C1 driver,
    60 slices, two time steps of dt = 25."""
    cfg, beam, drv = _setup("C1", 64, 0.5, 20_000, 21, 0.0625, -2.0, 130)
    d = _compare_steps(torch_cuda, oracle_mod, cfg, drv, 60, 25.0, 2)
    # an electron driver loses energy to its wake
    assert ((d[5] - drv[5]) * drv[7]).sum() < 0.0


def test_time_step_c2_blowout_driver(torch_cuda, oracle_mod):
    """Blowout (256^2, 4 particles per cell, adaptive steps): 100,000 sampled
    particles of the C2 driver, 120 slices, one step of dt = 10."""
    cfg, beam, drv = _setup("C2", 256, 10.0, 100_000, 22, 0.02, -2.0, 300)
    _compare_steps(torch_cuda, oracle_mod, cfg, drv, 120, 10.0, 1)


def test_quiet_driver_reproduces_the_frozen_driver_run(torch_cuda, oracle_mod):
    """A quiet (lattice) driver whose planes coincide with the slices deposits
    the frozen Gaussian driver's density times v_z = 1 - 1/2gamma^2: the time
    step's sweep reproduces the GPU's own frozen-driver run to 1e-6."""
    from paper_2012_00881_amd import Simulation
    cfg, beam, drv = _setup("C1", 64, 0.1, 0, 0, 0.0625, -0.0625, 96, quiet=True)
    sim = Simulation(cfg, n_slices=60)
    sim.driver_set(drv)
    sim.time_step(0.0, 60)
    F = sim.get_state()["fields"].cpu().numpy()
    sim.close()
    ref_cfg = wi.scaled(wi.config("C1"), beams=[beam])
    sim = Simulation(ref_cfg, n_slices=60)
    sim.run(60)
    R = sim.get_state()["fields"].cpu().numpy()
    sim.close()
    check_fields(F, R, 1e-6, "quiet driver vs frozen driver")
