"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""
import ctypes as C
import os
import re

import pytest

import wandqs_inputs as wi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2012_00881_amd import wandqs
    if not os.path.exists(wandqs.LIB_PATH):
        from paper_2012_00881_amd import build
        build.build()
    return wandqs


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "wandqs.h")).read()
    declared = set(re.findall(r"\b(wandqs_[a-z_]+)\s*\(", hdr))
    assert declared == set(lib.EXPORTS)
    L = lib.load()
    for name in declared:
        assert hasattr(L, name), name


def test_struct_sizes_match_header_layout(lib):
    # natural alignment on x86-64: the binding's ctypes structs must match
    assert C.sizeof(lib.Beam) == 4 + 4 + 6 * 8 + 8 + 8 + 8
    assert C.sizeof(lib.SliceInfo) == 3 * 8 + 5 * 4 + 4 + 5 * 8 + 4 + 4


@pytest.mark.parametrize("bad", [
    dict(n_cells=100), dict(n_cells=4), dict(n_cells=8192), dict(half_width=0.0),
    dict(ppc_side=5), dict(ppc_side=2, jitter=0.3), dict(dxi0=0.0), dict(refine_k=-1),
    dict(mg_max_cycles=0), dict(nu_pre=4), dict(nu_post=0), dict(adaptive=2),
    dict(adaptive=1, checkpoint_every=8), dict(adjoint_hold_dxi=2), dict(pusher=3),
    dict(pusher="rk4", checkpoint_every=4, adaptive=0), dict(laser_nz=-1),
    dict(laser_nz=4, laser_k0=0.0), dict(laser_nz=4, laser_k0=5.0, checkpoint_every=4, adaptive=0),
])
def test_invalid_configs_rejected(lib, bad):
    cfg = wi.scaled(wi.config("C2"), **bad)
    with pytest.raises(lib.WandQSError) as e:
        lib.workspace_bytes(cfg, 1)
    assert e.value.status == lib.E_INVALID


def test_invalid_beam_and_probe_rejected(lib):
    cfg = wi.config("C1")
    cfg["beams"][0]["sigma_z"] = 0.0
    with pytest.raises(lib.WandQSError):
        lib.workspace_bytes(cfg, 1)
    cfg = wi.config("C4")
    cfg["probes"][0]["slice_end"] = cfg["probes"][0]["slice_begin"]
    with pytest.raises(lib.WandQSError):
        lib.workspace_bytes(cfg, 1)


def test_workspace_sizes_scale(lib):
    b1 = lib.workspace_bytes(wi.config("C1"), 1)
    b2 = lib.workspace_bytes(wi.config("C2"), 1)
    b5 = lib.workspace_bytes(wi.config("C5"), 4096)
    assert 0 < b1 < b2 < b5 < 2 * 1024**3
    assert b5 % 256 == 0
    # a laser adds two sets of complex planes
    bl = lib.workspace_bytes(wi.scaled(wi.config("C1"), laser_nz=10, laser_k0=5.0), 1)
    assert bl >= b1 + 2 * 10 * 16 * 65 * 65


def test_init_without_gpu_fails_cleanly(lib):
    """On a machine without a GPU, wandqs_init validates, lays out the workspace
    and then reports the HIP failure (no crash).  Skipped where a GPU is visible:
    the fake workspace pointer must never reach a device."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    L = lib.load()
    for name in ("C1", "C4", "C5"):
        c, keep = lib.make_config(wi.config(name) if name != "C4" else wi.config(name))
        n = C.c_size_t(0)
        assert L.wandqs_workspace_bytes(C.byref(c), 8, C.byref(n)) == 0
        ctx = C.c_void_p()
        st = L.wandqs_init(C.byref(c), 8, C.c_void_p(1 << 20), n.value, None, C.byref(ctx))
        assert st == lib.E_HIP and not ctx.value
        assert L.wandqs_last_error(None)
        st = L.wandqs_init(C.byref(c), 8, C.c_void_p(1 << 20), n.value - 256, None, C.byref(ctx))
        assert st == lib.E_NOMEM


def test_missing_library_fails_loudly(lib, monkeypatch, tmp_path):
    """Without libwandqs.so the binding raises, both at load and when a
    Simulation is built; nothing falls back to the CPU or to the oracle."""
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "libwandqs.so"))
    monkeypatch.setattr(lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        lib.load()
    with pytest.raises(RuntimeError, match="missing"):
        lib.Simulation(wi.config("C1"), n_slices=1)
