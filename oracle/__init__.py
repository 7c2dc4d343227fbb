"""CPU oracle for the quasi-static slice step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle_wandqs.so`` (plain
FP64 C++ with OpenMP loops whose results do not depend on the thread count, see
``wandqs_oracle.cpp``) with numpy arrays.  It shares no code with the GPU
library in ``paper_2012_00881_amd``.

The environment variable ``WANDQS_ORACLE_LIB`` names another build of the same
source to load instead (the sanitizer build of the tests).

Every function is pinned by ``tests/test_oracle_*.py`` against facts fixed by the
paper or by mathematics (closed forms, dense direct solves, invariants).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("WANDQS_ORACLE_LIB") or os.path.join(_HERE, "liboracle_wandqs.so")
_lib = None

FIELDS = ("psi", "Ez", "Bz", "Bx", "By")
MOMENTS = ("n", "jx", "jy", "Txx", "Txy", "Tyy")
EXTRA = ("k2", "fBx", "fBy", "jz")

OK, INVALID, NOCONV, NONPHYS = 0, -1, -4, -5
#: plasma pushers: the Boris-like scheme and Runge-Kutta of order 1, 2, 4
PUSHERS = {"boris": 0, "rk1": 1, "rk2": 2, "rk4": 4}

_dp = C.POINTER(C.c_double)


class Beam(C.Structure):
    _fields_ = [("kind", C.c_int), ("amp", C.c_double), ("sigma_r", C.c_double),
                ("sigma_z", C.c_double), ("xi_c", C.c_double), ("x0", C.c_double),
                ("y0", C.c_double), ("n_bins", C.c_int), ("r_max", C.c_double),
                ("bin_amp", _dp)]


class Cfg(C.Structure):
    _fields_ = [("n_cells", C.c_int), ("half_width", C.c_double), ("ppc", C.c_int),
                ("n0", C.c_double), ("dxi0", C.c_double), ("adaptive", C.c_int),
                ("refine_k", C.c_int), ("mg_rtol", C.c_double), ("mg_atol", C.c_double),
                ("mg_max_cycles", C.c_int), ("nu_pre", C.c_int), ("nu_post", C.c_int),
                ("n_beams", C.c_int), ("beams", C.POINTER(Beam)), ("pusher", C.c_int),
                ("drv_planes", _dp), ("drv_nz", C.c_int), ("drv_xi0", C.c_double),
                ("drv_dz", C.c_double), ("las_env", _dp), ("las_nz", C.c_int),
                ("las_k0", C.c_double), ("drv_nsub", C.c_int)]


class Info(C.Structure):
    _fields_ = [("xi", C.c_double), ("dxi", C.c_double), ("dxi_next", C.c_double),
                ("vmax", C.c_double), ("cycles", C.c_int * 5), ("rel_resid", C.c_double * 5),
                ("invariant_err", C.c_double), ("status", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.oracle_next_dxi.restype = C.c_double
        L.oracle_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Holds one workload (a dict from ``wandqs_inputs.config``) as a C config."""

    def __init__(self, cfg: dict):
        self.cfg = cfg
        self.N = int(cfg["n_cells"])
        self.L = float(cfg["half_width"])
        self.h = 2.0 * self.L / self.N
        self.nn = (self.N + 1) ** 2
        self._keep = []
        beams = (Beam * max(1, len(cfg["beams"])))()
        for k, b in enumerate(cfg["beams"]):
            bb = beams[k]
            bb.x0, bb.y0 = b.get("x0", 0.0), b.get("y0", 0.0)
            bb.sigma_z, bb.xi_c = b["sigma_z"], b["xi_c"]
            if b["kind"] == "gauss":
                bb.kind, bb.amp, bb.sigma_r = 0, b["amp"], b["sigma_r"]
            else:
                amp = _f64(b["bin_amp"])
                self._keep.append(amp)
                bb.kind, bb.n_bins, bb.r_max, bb.bin_amp = 1, amp.size, b["r_max"], _p(amp)
                bb.amp, bb.sigma_r = 1.0, 1.0
        self._beams = beams
        c = Cfg()
        c.n_cells, c.half_width = self.N, self.L
        c.ppc = int(cfg["ppc_side"]) ** 2
        c.n0, c.dxi0 = cfg.get("n0", 1.0), cfg["dxi0"]
        c.adaptive, c.refine_k = int(cfg["adaptive"]), int(cfg["refine_k"])
        c.mg_rtol, c.mg_atol = cfg["mg_rtol"], cfg["mg_atol"]
        c.mg_max_cycles, c.nu_pre, c.nu_post = cfg["mg_max_cycles"], cfg["nu_pre"], cfg["nu_post"]
        c.n_beams, c.beams = len(cfg["beams"]), beams
        c.pusher = PUSHERS[cfg.get("pusher", "boris")]
        c.drv_nsub = int(cfg.get("driver_nsub", 1))
        self.c = c
        self.laser_env = None

    # ----------------------------------------------------------------- laser
    def set_laser(self, env, k0):
        """Laser envelope A-hat on planes xi_m = m dxi0: complex [nz][N+1][N+1]
        (None: no laser); k0 = omega0/omega_p."""
        if env is None:
            self.laser_env = None
            self.c.las_env, self.c.las_nz = None, 0
            return
        e = np.ascontiguousarray(env, dtype=np.complex128).reshape(-1, self.N + 1, self.N + 1)
        self.laser_env = e
        self.c.las_env = e.ctypes.data_as(_dp)
        self.c.las_nz, self.c.las_k0 = e.shape[0], float(k0)

    def laser_advance(self, dt, env, chi=None, k0=None):
        """Advance envelope planes env (complex [nz][N+1][N+1]) by dt with the
        susceptibility chi [nz][N+1][N+1] (None: vacuum); returns (status,
        new planes, multigrid cycles per plane)."""
        e = np.ascontiguousarray(env, dtype=np.complex128).reshape(-1, self.N + 1, self.N + 1)
        nz = e.shape[0]
        out = np.zeros_like(e)
        ch = None if chi is None else _f64(chi).reshape(nz, -1)
        cyc = np.zeros(nz, dtype=np.int32)
        c = Cfg.from_buffer_copy(self.c)
        if k0 is not None:
            c.las_k0 = float(k0)
        st = lib().oracle_laser_advance(C.byref(c), C.c_double(dt), nz, e.ctypes.data_as(_dp),
                                        _p(ch), out.ctypes.data_as(_dp),
                                        cyc.ctypes.data_as(C.POINTER(C.c_int)))
        return st, out, cyc

    # ---------------------------------------------------------------- pieces
    def deposit(self, x, y, q=None):
        x, y = _f64(x), _f64(y)
        q = None if q is None else _f64(q)
        out = np.zeros(self.nn)
        lib().oracle_deposit(C.byref(self.c), x.size, _p(x), _p(y), _p(q), _p(out))
        return out.reshape(self.N + 1, self.N + 1)

    def gather(self, x, y, F):
        x, y, F = _f64(x), _f64(y), _f64(F)
        out = np.zeros(x.size)
        lib().oracle_gather(C.byref(self.c), x.size, _p(x), _p(y), _p(F), _p(out))
        return out

    def beam_density(self, xi):
        out = np.zeros(self.nn)
        lib().oracle_beam_density(C.byref(self.c), C.c_double(xi), _p(out))
        return out.reshape(self.N + 1, self.N + 1)

    def assemble(self, xi, moments, psi, Ez, Bz):
        mom = _f64(moments).reshape(6, -1)
        out = np.zeros((4, self.nn))
        st = lib().oracle_assemble(C.byref(self.c), C.c_double(xi), _p(mom), _p(_f64(psi)),
                                   _p(_f64(Ez)), _p(_f64(Bz)), _p(out))
        return st, out.reshape(4, self.N + 1, self.N + 1)

    def push_fields(self, dxi, x, y, px, py, fields, xi=0.0):
        """The particle advance of a slice at xi from its solved fields (the
        configuration's pusher, a laser's ponderomotive terms at xi); returns
        (status, x, y, px, py, vmax)."""
        arrs = [_f64(a).copy() for a in (x, y, px, py)]
        F = _f64(fields).reshape(5, -1)
        vm = C.c_double(0.0)
        st = lib().oracle_push_fields(C.byref(self.c), C.c_double(xi), C.c_double(dxi),
                                      arrs[0].size, _p(F), *[_p(a) for a in arrs], C.byref(vm))
        return (st, *arrs, vm.value)

    # ------------------------------------------------------------ driver
    def driver_deposit(self, drv, nz, xi0, dz):
        """Longitudinal current of driver particles drv [8][n] on nz planes."""
        d = _f64(drv).reshape(8, -1)
        out = np.zeros((nz, self.nn))
        lib().oracle_driver_deposit(C.byref(self.c), d.shape[1], _p(d), int(nz), C.c_double(xi0),
                                    C.c_double(dz), _p(out))
        return out.reshape(nz, self.N + 1, self.N + 1)

    def driver_push(self, drv, dt, xi_s, F_s, env0=None, env1=None):
        """Advance driver particles drv [8][n] by dt through the slices
        (xi_s [ns], F_s [ns][5][N+1][N+1]) and, with env0 and env1 (the laser's
        planes at t and t + dt, complex [nz][N+1][N+1]; k0 from set_laser), the
        laser's fields, in driver_nsub sub-steps; returns the new state."""
        d = _f64(drv).reshape(8, -1).copy()
        xs = _f64(xi_s)
        Fs = _f64(F_s).reshape(max(xs.size, 1), 5, -1)
        e0 = None if env0 is None else np.ascontiguousarray(env0, dtype=np.complex128)
        e1 = None if env1 is None else np.ascontiguousarray(env1, dtype=np.complex128)
        c = Cfg.from_buffer_copy(self.c)
        if e0 is not None:
            c.las_nz = e0.shape[0]
        st = lib().oracle_driver_push(C.byref(c), C.c_double(dt), d.shape[1], _p(d), xs.size,
                                      _p(xs), _p(Fs), None if e0 is None else e0.ctypes.data_as(_dp),
                                      None if e1 is None else e1.ctypes.data_as(_dp))
        assert st == OK
        return d

    def laser_fields(self, dt, tau, pts, env0, env1):
        """The laser's fields at points pts [3][n] (x, y, xi) and time t + tau dt
        from the planes env0 (t) and env1 (t + dt): [6][n] = E_x, E_y, E_z, B_x,
        B_y, B_z (k0 from set_laser)."""
        p = _f64(pts).reshape(3, -1)
        e0 = np.ascontiguousarray(env0, dtype=np.complex128)
        e1 = np.ascontiguousarray(env1, dtype=np.complex128)
        c = Cfg.from_buffer_copy(self.c)
        c.las_nz = e0.shape[0]
        out = np.zeros((6, p.shape[1]))
        lib().oracle_laser_fields(C.byref(c), C.c_double(dt), C.c_double(tau), p.shape[1], _p(p),
                                  e0.ctypes.data_as(_dp), e1.ctypes.data_as(_dp), _p(out))
        return out

    def time_step(self, state, drv, n_slices, dt, nz, xi0, dz, keep_fields=False):
        """One step of the time loop: the driver's current on nz planes, a sweep
        of n_slices slices through `state` (advanced in place), the driver
        (drv [8][n], advanced in place) pushed by dt.  With a laser set
        (set_laser) its envelope is advanced by dt in the same sweep and
        replaces the one set.  Returns dict(status, infos[, xi, fields])."""
        state["fields"] = _f64(state["fields"]).reshape(5, self.N + 1, self.N + 1)
        d = _f64(drv).reshape(8, -1)
        xi = C.c_double(state["xi"])
        dxi = C.c_double(state["dxi"])
        hx = np.zeros(n_slices)
        hF = np.zeros((n_slices, 5, self.nn)) if keep_fields else None
        infos = (Info * n_slices)()
        nxt = None if self.laser_env is None else np.zeros_like(self.laser_env)
        st = lib().oracle_time_step(C.byref(self.c), state["x"].size, _p(state["x"]),
                                    _p(state["y"]), _p(state["px"]), _p(state["py"]),
                                    _p(state["fields"]), C.byref(xi), C.byref(dxi), int(n_slices),
                                    d.shape[1], _p(d), int(nz), C.c_double(xi0), C.c_double(dz),
                                    C.c_double(dt), _p(hx), _p(hF), infos,
                                    None if nxt is None else nxt.ctypes.data_as(_dp))
        state["xi"], state["dxi"] = xi.value, dxi.value
        if nxt is not None and st == OK:
            self.set_laser(nxt, self.c.las_k0)
        out = dict(status=st, infos=list(infos), xi=hx)
        if keep_fields:
            out["fields"] = hF.reshape(n_slices, 5, self.N + 1, self.N + 1)
        return out

    def next_dxi(self, vmax):
        return lib().oracle_next_dxi(C.byref(self.c), C.c_double(vmax))

    # ----------------------------------------------------------------- slice
    def slice_step(self, state: dict, want_moments=False, carry_pz=False):
        """Advance ``state`` (dict x, y, px, py, fields[5,N+1,N+1], xi, dxi[, pz]) in place."""
        for k in ("x", "y", "px", "py"):
            state[k] = _f64(state[k]).copy() if not state[k].flags.writeable else _f64(state[k])
        state["fields"] = _f64(state["fields"]).reshape(5, self.N + 1, self.N + 1)
        xi = C.c_double(state["xi"])
        dxi = C.c_double(state["dxi"])
        info = Info()
        mom = np.zeros((6, self.nn)) if want_moments else None
        extra = np.zeros((4, self.nn)) if want_moments else None
        pz = None
        if carry_pz:
            if "pz" not in state:
                state["pz"] = np.zeros_like(state["x"])
            pz = state["pz"]
        st = lib().oracle_slice_step(C.byref(self.c), state["x"].size, _p(state["x"]),
                                     _p(state["y"]), _p(state["px"]), _p(state["py"]), _p(pz),
                                     _p(state["fields"]), C.byref(xi), C.byref(dxi),
                                     C.byref(info), _p(mom), _p(extra))
        state["xi"], state["dxi"] = xi.value, dxi.value
        out = dict(status=st, info=info)
        if want_moments:
            out["moments"] = mom.reshape(6, self.N + 1, self.N + 1)
            out["extra"] = extra.reshape(4, self.N + 1, self.N + 1)
        return out

    def run(self, state: dict, n_slices: int, keep_fields=False, carry_pz=False):
        infos = (Info * n_slices)()
        hist = np.zeros((n_slices, 5, self.nn)) if keep_fields else None
        state["fields"] = _f64(state["fields"]).reshape(5, self.N + 1, self.N + 1)
        pz = None
        if carry_pz:
            if "pz" not in state:
                state["pz"] = np.zeros_like(state["x"])
            pz = state["pz"]
        xi = C.c_double(state["xi"])
        dxi = C.c_double(state["dxi"])
        st = lib().oracle_run(C.byref(self.c), state["x"].size, _p(state["x"]), _p(state["y"]),
                              _p(state["px"]), _p(state["py"]), _p(pz), _p(state["fields"]),
                              C.byref(xi), C.byref(dxi), n_slices, _p(hist), infos)
        state["xi"], state["dxi"] = xi.value, dxi.value
        res = dict(status=st, infos=list(infos))
        if keep_fields:
            res["fields"] = hist.reshape(n_slices, 5, self.N + 1, self.N + 1)
        return res


def theta_of(cfg: dict) -> np.ndarray:
    """Driver parameters in the adjoint's order: per beam, amp or the bin amplitudes."""
    out = []
    for b in cfg["beams"]:
        out += [b["amp"]] if b["kind"] == "gauss" else list(np.asarray(b["bin_amp"], float))
    return np.array(out, dtype=np.float64)


def with_theta(cfg: dict, theta) -> dict:
    """Copy of cfg with the driver parameters replaced by theta."""
    import wandqs_inputs as wi
    out = wi.scaled(cfg)
    k = 0
    for b in out["beams"]:
        if b["kind"] == "gauss":
            b["amp"] = float(theta[k])
            k += 1
        else:
            n = len(b["bin_amp"])
            b["bin_amp"] = np.array(theta[k:k + n], dtype=np.float64)
            k += n
    return out


def _probe_array(cfg):
    pr = cfg["probes"]
    a = np.array([[p["field"], p["slice_begin"], p["slice_end"], p["r_max"], p.get("x0", 0.0),
                   p.get("y0", 0.0)] for p in pr], dtype=np.float64).reshape(-1, 6)
    return a


def _slice_adjoint(self, state, fields, out_bar, Fbar=None):
    """Reverse of one slice: state = its input particles, fields = its solved
    fields; out_bar = adjoints (x, y, px, py) of its output particles.  Returns
    (adjoints of the input particles, theta_bar)."""
    x, y, px, py = (_f64(state[k]) for k in ("x", "y", "px", "py"))
    xb, yb, pxb, pyb = (_f64(a).copy() for a in out_bar)
    nth = lib().oracle_theta_count(C.byref(self.c))
    tb = np.zeros(max(1, nth))
    Fb = None if Fbar is None else _f64(Fbar).reshape(5, -1)
    st = lib().oracle_slice_adjoint(C.byref(self.c), x.size, _p(x), _p(y), _p(px), _p(py),
                                    _p(_f64(fields)), C.c_double(state["xi"]),
                                    C.c_double(state["dxi"]), _p(xb), _p(yb), _p(pxb), _p(pyb),
                                    _p(Fb), _p(tb))
    return st, (xb, yb, pxb, pyb), tb[:nth]


def _run_loss(self, state, n_slices, weights=None, grad=False):
    """Loss of an n-slice run from `state` (probes of the config); with grad,
    also dL/dtheta by the reverse sweep.  Advances `state`."""
    pr = _probe_array(self.cfg)
    w = np.ones(len(pr)) if weights is None else _f64(weights)
    state["fields"] = _f64(state["fields"]).reshape(5, self.N + 1, self.N + 1)
    xi = C.c_double(state["xi"])
    dxi = C.c_double(state["dxi"])
    loss = C.c_double(0.0)
    nth = lib().oracle_theta_count(C.byref(self.c))
    tb = np.zeros(max(1, nth)) if grad else None
    st = lib().oracle_run_loss(C.byref(self.c), state["x"].size, _p(state["x"]), _p(state["y"]),
                               _p(state["px"]), _p(state["py"]), _p(state["fields"]),
                               C.byref(xi), C.byref(dxi), int(n_slices), len(pr), _p(pr),
                               _p(w), C.byref(loss), _p(tb))
    state["xi"], state["dxi"] = xi.value, dxi.value
    return st, loss.value, (tb[:nth] if grad else None)


def _run_tangent(self, state, n_slices, dP=None, dtheta=None, weights=None):
    """Tangent-linear run (forward mode, up to 8 directions): returns
    (status, loss, dloss[K], dout[K][4][P], dF[K][5][N+1][N+1]).  dP: [K][4][P]
    seeds of the particles, dtheta: [K][n_theta] seeds of the driver
    parameters.  Advances `state` like run()."""
    x, y, px, py = (_f64(state[k]).copy() for k in ("x", "y", "px", "py"))
    P = x.size
    nth = lib().oracle_theta_count(C.byref(self.c))
    K = max(1, (0 if dP is None else np.asarray(dP).shape[0]),
            (0 if dtheta is None else np.asarray(dtheta).shape[0]))
    dPa = None if dP is None else _f64(dP).reshape(K, 4, P)
    dTa = None if dtheta is None else _f64(dtheta).reshape(K, nth)
    pr = _probe_array(self.cfg)
    w = np.ones(len(pr)) if weights is None else _f64(weights)
    fields = _f64(state["fields"]).reshape(5, self.N + 1, self.N + 1).copy()
    xi = C.c_double(state["xi"])
    dxi = C.c_double(state["dxi"])
    loss = C.c_double(0.0)
    dloss = np.zeros(K)
    dout = np.zeros((K, 4, P))
    dF = np.zeros((K, 5, self.N + 1, self.N + 1))
    st = lib().oracle_run_tangent(C.byref(self.c), P, _p(x), _p(y), _p(px), _p(py), _p(fields),
                                  C.byref(xi), C.byref(dxi), int(n_slices), int(K), _p(dPa),
                                  _p(dTa), len(pr), _p(pr), _p(w), C.byref(loss), _p(dloss),
                                  _p(dout), _p(dF))
    state.update(x=x, y=y, px=px, py=py, fields=fields, xi=xi.value, dxi=dxi.value)
    return st, loss.value, dloss, dout, dF


Oracle.slice_adjoint = _slice_adjoint
Oracle.run_tangent = _run_tangent
Oracle.run_loss = _run_loss


def initial_state(cfg: dict) -> dict:
    """Cold plasma at rest at xi = 0 with zero fields (uses the shared input generator)."""
    import wandqs_inputs as wi
    x, y, px, py = wi.plasma_lattice(cfg["n_cells"], cfg["half_width"], cfg["ppc_side"],
                                     cfg["jitter"], cfg["seed"])
    N = cfg["n_cells"]
    return dict(x=x, y=y, px=px, py=py, fields=np.zeros((5, N + 1, N + 1)), xi=0.0,
                dxi=float(cfg["dxi0"]))


def apply(N, h, u, k2=None):
    """L_h u - k2 u at interior nodes (zero on the boundary)."""
    u = _f64(u)
    out = np.zeros_like(u)
    lib().oracle_apply(int(N), C.c_double(h), _p(None if k2 is None else _f64(k2)), _p(u),
                       _p(out))
    return out


def mg_solve(N, h, f, u0=None, k2=None, rtol=1e-14, atol=0.0, max_cycles=50, nu1=2, nu2=2):
    """Multigrid solve of (L_h - k2) u = f with zero Dirichlet boundary: V(nu1, nu2)
    cycles of red-black Gauss-Seidel from the guess u0 (default 0)."""
    f = _f64(f)
    u = np.zeros_like(f) if u0 is None else _f64(u0).copy()
    cyc = C.c_int(0)
    rel = C.c_double(0)
    st = lib().oracle_mg_solve(int(N), C.c_double(h), _p(None if k2 is None else _f64(k2)),
                               _p(f), _p(u), C.c_double(rtol), C.c_double(atol), int(max_cycles),
                               int(nu1), int(nu2), C.byref(cyc), C.byref(rel))
    return st, u, cyc.value, rel.value


def psi_gradient(N, L, psi):
    """Node gradient of psi used by the particle gather: [2][N+1][N+1] (d/dx, d/dy)."""
    psi = _f64(psi)
    out = np.zeros((2,) + psi.shape)
    lib().oracle_psi_gradient(int(N), C.c_double(L), _p(psi), _p(out))
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (the results do not depend on it)."""
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def push(L, dxi, g_i, gx, gy, Bx, By, Bz, x, y, px, py):
    arrs = [_f64(a).copy() for a in (x, y, px, py)]
    ins = [_f64(a) for a in (g_i, gx, gy, Bx, By, Bz)]
    lib().oracle_push(C.c_double(L), C.c_double(dxi), arrs[0].size, *[_p(a) for a in ins],
                      *[_p(a) for a in arrs])
    return arrs


# ------------------------------------------------- non-uniform grids (Sec. VII.B)
def _axes(X, Y):
    X, Y = _f64(X), _f64(Y)
    assert X.size == Y.size
    return X.size - 1, X, Y


def nu_apply(X, Y, u, M=None):
    """L u (the non-uniform grid's nine-point operator with the third-order
    correction, plus the M terms) at the interior nodes; u, M: [N+1][N+1]
    indexed [j][i] (y, x)."""
    N, X, Y = _axes(X, Y)
    u = _f64(u)
    out = np.zeros_like(u)
    st = lib().oracle_nu_apply(N, _p(X), _p(Y), _p(None if M is None else _f64(M)), _p(u), _p(out))
    assert st == OK
    return out


def nu_rhs(X, Y, J):
    """R J, the right-hand side of the discrete equation L u = R J."""
    N, X, Y = _axes(X, Y)
    J = _f64(J)
    out = np.zeros_like(J)
    assert lib().oracle_nu_rhs(N, _p(X), _p(Y), _p(J), _p(out)) == OK
    return out


def nu_restrict(X, Y, v):
    N, X, Y = _axes(X, Y)
    out = np.zeros((N // 2 + 1, N // 2 + 1))
    assert lib().oracle_nu_transfer(N, _p(X), _p(Y), 0, _p(_f64(v)), _p(out)) == OK
    return out


def nu_prolong(X, Y, e):
    N, X, Y = _axes(X, Y)
    out = np.zeros((N + 1, N + 1))
    assert lib().oracle_nu_transfer(N, _p(X), _p(Y), 1, _p(_f64(e)), _p(out)) == OK
    return out


def nu_mg_solve(X, Y, J, u0=None, M=None, rtol=1e-14, atol=0.0, max_cycles=60, nu1=2, nu2=2):
    """Multigrid solve of L u = R J on the non-uniform grid (X, Y), u = 0 on the
    boundary, from the guess u0 (default 0).  Returns (status, u, cycles, rel)."""
    N, X, Y = _axes(X, Y)
    J = _f64(J)
    u = np.zeros_like(J) if u0 is None else _f64(u0).copy()
    cyc = C.c_int(0)
    rel = C.c_double(0)
    st = lib().oracle_nu_mg_solve(N, _p(X), _p(Y), _p(None if M is None else _f64(M)), _p(J),
                                  _p(u), C.c_double(rtol), C.c_double(atol), int(max_cycles),
                                  int(nu1), int(nu2), C.byref(cyc), C.byref(rel))
    return st, u, cyc.value, rel.value
