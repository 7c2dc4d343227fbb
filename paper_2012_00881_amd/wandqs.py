"""ctypes binding of libwandqs.so (C ABI declared in include/wandqs.h).

Argument marshalling only: every step of the slice runs in the HIP library.
PyTorch provides the device workspace, the input/output buffers and the HIP
stream.  There is no fallback: if the library is missing or no GPU is visible,
the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# WANDQS_LIB names another build of the same library (the host code built with
# the address and undefined-behaviour sanitizers, for the CPU tests)
LIB_PATH = os.environ.get("WANDQS_LIB") or os.path.join(_HERE, "libwandqs.so")

OK, E_INVALID, E_NOMEM, E_HIP, E_NOCONV, E_NONPHYS, E_STATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_HIP", -4: "E_NOCONV",
                -5: "E_NONPHYS", -6: "E_STATE"}
FP64, MIXED = 0, 1
#: plasma pushers of wandqs_config.pusher
PUSHERS = {"boris": 0, "rk1": 1, "rk2": 2, "rk4": 4}
BEAM_GAUSS, BEAM_RADIAL_BINS = 0, 1

_dp = C.POINTER(C.c_double)

#: every symbol the header declares
EXPORTS = ("wandqs_workspace_bytes", "wandqs_init", "wandqs_slice_step", "wandqs_run",
           "wandqs_get_state", "wandqs_set_state", "wandqs_mg_solve", "wandqs_get_moments",
           "wandqs_num_particles", "wandqs_destroy", "wandqs_last_error", "wandqs_profile",
           "wandqs_profile_stats", "wandqs_backward", "wandqs_num_theta", "wandqs_tape_slices",
           "wandqs_mg_solve_noalloc", "wandqs_driver_set", "wandqs_driver_get",
           "wandqs_time_step", "wandqs_laser_set", "wandqs_laser_get", "wandqs_laser_advance",
           "wandqs_nu_mg_solve")


class Beam(C.Structure):
    _fields_ = [("kind", C.c_int32), ("amp", C.c_double), ("sigma_r", C.c_double),
                ("sigma_z", C.c_double), ("xi_c", C.c_double), ("x0", C.c_double),
                ("y0", C.c_double), ("n_bins", C.c_int32), ("r_max", C.c_double),
                ("bin_amp", _dp)]


class Probe(C.Structure):
    _fields_ = [("field", C.c_int32), ("slice_begin", C.c_int32), ("slice_end", C.c_int32),
                ("r_max", C.c_double), ("x0", C.c_double), ("y0", C.c_double)]


class Config(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("half_width", C.c_double), ("ppc_side", C.c_int32),
                ("jitter", C.c_double), ("seed", C.c_uint64), ("n0", C.c_double),
                ("dxi0", C.c_double), ("adaptive", C.c_int32), ("refine_k", C.c_int32),
                ("precision", C.c_int32), ("mg_rtol", C.c_double), ("mg_atol", C.c_double),
                ("mg_max_cycles", C.c_int32), ("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("n_beams", C.c_int32), ("beams", C.POINTER(Beam)), ("n_probes", C.c_int32),
                ("probes", C.POINTER(Probe)), ("checkpoint_every", C.c_int32),
                ("mg_inner_cycles", C.c_int32), ("mg_omega", C.c_double),
                ("mg_omega_helm", C.c_double), ("adjoint_hold_dxi", C.c_int32),
                ("pusher", C.c_int32), ("driver_max", C.c_int32), ("driver_nz", C.c_int32),
                ("driver_xi0", C.c_double), ("driver_dz", C.c_double), ("laser_nz", C.c_int32),
                ("laser_k0", C.c_double), ("driver_nsub", C.c_int32)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 56), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("alg_bytes", C.c_double)]


class SliceInfo(C.Structure):
    _fields_ = [("xi", C.c_double), ("dxi", C.c_double), ("vmax", C.c_double),
                ("vcycles", C.c_int32 * 5), ("rel_resid", C.c_double * 5), ("flags", C.c_int32),
                ("laser_vcycles", C.c_int32)]

    def as_dict(self):
        return dict(xi=self.xi, dxi=self.dxi, vmax=self.vmax, vcycles=list(self.vcycles),
                    rel_resid=list(self.rel_resid), flags=self.flags,
                    laser_vcycles=self.laser_vcycles)


_lib = None


def load():
    """Load libwandqs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    L.wandqs_workspace_bytes.argtypes = [C.POINTER(Config), i32, C.POINTER(sz)]
    L.wandqs_init.argtypes = [C.POINTER(Config), i32, vp, sz, vp, C.POINTER(vp)]
    L.wandqs_slice_step.argtypes = [vp, vp, C.POINTER(SliceInfo)]
    L.wandqs_run.argtypes = [vp, i32, vp, C.POINTER(SliceInfo)]
    L.wandqs_get_state.argtypes = [vp, vp, vp, _dp]
    L.wandqs_set_state.argtypes = [vp, vp, vp, _dp]
    L.wandqs_mg_solve.argtypes = [vp, i32, vp, vp, vp, C.POINTER(i32), _dp]
    L.wandqs_get_moments.argtypes = [vp, vp]
    L.wandqs_mg_solve_noalloc.argtypes = [C.POINTER(Config), i32, vp, vp, vp, vp]
    L.wandqs_driver_set.argtypes = [vp, C.c_int64, vp]
    L.wandqs_driver_get.argtypes = [vp, vp]
    L.wandqs_time_step.argtypes = [vp, C.c_double, i32, C.POINTER(SliceInfo)]
    L.wandqs_laser_set.argtypes = [vp, vp]
    L.wandqs_laser_get.argtypes = [vp, vp]
    L.wandqs_laser_advance.argtypes = [vp, C.c_double, vp, C.POINTER(i32)]
    L.wandqs_nu_mg_solve.argtypes = [vp, _dp, _dp, vp, vp, vp, C.POINTER(i32), _dp]
    L.wandqs_num_particles.argtypes = [vp]
    L.wandqs_num_particles.restype = C.c_int64
    L.wandqs_profile.argtypes = [vp, i32]
    L.wandqs_profile_stats.argtypes = [vp, C.POINTER(KernelStat), i32, C.POINTER(i32)]
    L.wandqs_backward.argtypes = [vp, _dp, vp, vp, _dp, vp]
    L.wandqs_num_theta.argtypes = [vp]
    L.wandqs_num_theta.restype = C.c_int32
    L.wandqs_tape_slices.argtypes = [vp]
    L.wandqs_tape_slices.restype = C.c_int64
    L.wandqs_destroy.argtypes = [vp]
    L.wandqs_destroy.restype = None
    L.wandqs_last_error.argtypes = [vp]
    L.wandqs_last_error.restype = C.c_char_p
    for name in ("wandqs_workspace_bytes", "wandqs_init", "wandqs_slice_step", "wandqs_run",
                 "wandqs_get_state", "wandqs_set_state", "wandqs_mg_solve",
                 "wandqs_get_moments", "wandqs_profile", "wandqs_profile_stats",
                 "wandqs_backward", "wandqs_mg_solve_noalloc", "wandqs_driver_set",
                 "wandqs_driver_get", "wandqs_time_step", "wandqs_laser_set", "wandqs_laser_get",
                 "wandqs_laser_advance", "wandqs_nu_mg_solve"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


class WandQSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"wandqs {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def make_config(cfg: dict):
    """C config from a workload dict (see wandqs_inputs.config).  Returns (Config, keep-alive)."""
    keep = []
    beams = (Beam * max(1, len(cfg["beams"])))()
    for k, b in enumerate(cfg["beams"]):
        bb = beams[k]
        bb.sigma_z, bb.xi_c = b["sigma_z"], b["xi_c"]
        bb.x0, bb.y0 = b.get("x0", 0.0), b.get("y0", 0.0)
        if b["kind"] == "gauss":
            bb.kind, bb.amp, bb.sigma_r = BEAM_GAUSS, b["amp"], b["sigma_r"]
        else:
            amp = np.ascontiguousarray(b["bin_amp"], dtype=np.float64)
            keep.append(amp)
            bb.kind, bb.n_bins, bb.r_max = BEAM_RADIAL_BINS, amp.size, b["r_max"]
            bb.bin_amp = amp.ctypes.data_as(_dp)
            bb.amp, bb.sigma_r = 1.0, 1.0
    probes = (Probe * max(1, len(cfg["probes"])))()
    for k, p in enumerate(cfg["probes"]):
        probes[k] = Probe(p["field"], p["slice_begin"], p["slice_end"], p["r_max"],
                          p.get("x0", 0.0), p.get("y0", 0.0))
    keep += [beams, probes]
    c = Config()
    c.n_cells, c.half_width = cfg["n_cells"], cfg["half_width"]
    c.ppc_side, c.jitter, c.seed = cfg["ppc_side"], cfg["jitter"], int(cfg["seed"])
    c.n0, c.dxi0 = cfg.get("n0", 1.0), cfg["dxi0"]
    c.adaptive, c.refine_k = int(cfg["adaptive"]), int(cfg["refine_k"])
    c.precision = MIXED if cfg.get("precision", "fp64") == "mixed" else FP64
    c.mg_rtol, c.mg_atol = cfg["mg_rtol"], cfg["mg_atol"]
    c.mg_max_cycles, c.nu_pre, c.nu_post = cfg["mg_max_cycles"], cfg["nu_pre"], cfg["nu_post"]
    c.n_beams, c.beams = len(cfg["beams"]), beams
    c.n_probes, c.probes = len(cfg["probes"]), probes
    c.checkpoint_every = cfg.get("checkpoint_every", 0)
    c.mg_inner_cycles = cfg.get("mg_inner_cycles", 0)
    c.mg_omega = cfg.get("mg_omega", 0.0)
    c.mg_omega_helm = cfg.get("mg_omega_helm", 0.0)
    c.adjoint_hold_dxi = int(cfg.get("adjoint_hold_dxi", 0))
    pu = cfg.get("pusher", "boris")
    c.pusher = PUSHERS[pu] if isinstance(pu, str) else int(pu)
    c.driver_max = int(cfg.get("driver_max", 0))
    c.driver_nz = int(cfg.get("driver_nz", 0))
    c.driver_xi0 = float(cfg.get("driver_xi0", 0.0))
    c.driver_dz = float(cfg.get("driver_dz", 0.0))
    c.laser_nz = int(cfg.get("laser_nz", 0))
    c.laser_k0 = float(cfg.get("laser_k0", 0.0))
    c.driver_nsub = int(cfg.get("driver_nsub", 0))
    return c, keep


def theta_of(cfg: dict) -> np.ndarray:
    """Driver parameters theta in the library's order: per beam its amp
    (Gaussian) or its bin amplitudes (radial bins)."""
    out = []
    for b in cfg["beams"]:
        if b["kind"] == "gauss":
            out.append(float(b["amp"]))
        else:
            out.extend(float(v) for v in b["bin_amp"])
    return np.asarray(out, dtype=np.float64)


def with_theta(cfg: dict, theta) -> dict:
    """Copy of cfg with the driver parameters replaced by theta."""
    theta = np.asarray(theta, dtype=np.float64)
    beams, k = [], 0
    for b in cfg["beams"]:
        b = dict(b)
        if b["kind"] == "gauss":
            b["amp"] = float(theta[k])
            k += 1
        else:
            n = len(b["bin_amp"])
            b["bin_amp"] = theta[k:k + n].copy()
            k += n
        beams.append(b)
    if k != theta.size:
        raise ValueError(f"theta has {theta.size} entries, the beams take {k}")
    return dict(cfg, beams=beams)


def workspace_bytes(cfg: dict, n_slices: int = 1) -> int:
    L = load()
    c, keep = make_config(cfg)
    n = C.c_size_t(0)
    st = L.wandqs_workspace_bytes(C.byref(c), int(n_slices), C.byref(n))
    if st != OK:
        raise WandQSError(st, L.wandqs_last_error(None).decode())
    return n.value


def mg_solve_noalloc(cfg: dict, f, u0=None, k2=None, stream=None):
    """wandqs_mg_solve_noalloc on cfg's grid: exactly cfg["mg_max_cycles"]
    V-cycles (cfg["mg_rtol"] must be <= 0) on 1 or 2 right-hand sides, with the
    library's static scratch array.  f, u0, k2: [nrhs][N+1][N+1] / [N+1][N+1]
    float64 (device tensors are used in place).  Returns (status, u); the work
    is enqueued on `stream` (default: torch's current stream)."""
    import torch
    L = load()
    c, keep = make_config(cfg)
    dev = torch.device("cuda", torch.cuda.current_device())
    f = torch.as_tensor(f, dtype=torch.float64).to(dev).contiguous()
    if f.dim() == 2:
        f = f.unsqueeze(0)
    u = (torch.zeros_like(f) if u0 is None else
         torch.as_tensor(u0, dtype=torch.float64).to(dev).reshape(f.shape).contiguous().clone())
    kk = None if k2 is None else torch.as_tensor(k2, dtype=torch.float64).to(dev).contiguous()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    st = L.wandqs_mg_solve_noalloc(C.byref(c), int(f.shape[0]),
                                   C.c_void_p(kk.data_ptr()) if kk is not None else None,
                                   C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()),
                                   C.c_void_p(s.cuda_stream))
    if st != OK:
        raise WandQSError(st, L.wandqs_last_error(None).decode())
    return st, u


class Simulation:
    """One context: plasma state, fields and workspace on one GPU."""

    def __init__(self, cfg: dict, n_slices: int = 1, device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.L = load()
        self.cfg = cfg
        self.N = int(cfg["n_cells"])
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._c, self._keep = make_config(cfg)
        nbytes = workspace_bytes(cfg, n_slices)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = (self.ws.data_ptr() + 255) & ~255
        ctx = C.c_void_p()
        st = self.L.wandqs_init(C.byref(self._c), int(n_slices), C.c_void_p(base), nbytes,
                                C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if st != OK:
            raise WandQSError(st, self.L.wandqs_last_error(None).decode())
        self.ctx = ctx
        self.P = int(self.L.wandqs_num_particles(ctx))

    # ------------------------------------------------------------------ util
    def _check(self, st):
        if st != OK:
            raise WandQSError(st, self.L.wandqs_last_error(self.ctx).decode())

    def _nodes(self, k):
        return self.torch.empty((k, self.N + 1, self.N + 1), dtype=self.torch.float64,
                                device=self.device)

    # ------------------------------------------------------------------- API
    def step(self, fields: bool = False, info: bool = False):
        out = self._nodes(5) if fields else None
        inf = SliceInfo() if info else None
        st = self.L.wandqs_slice_step(self.ctx, C.c_void_p(out.data_ptr()) if fields else None,
                                      C.byref(inf) if info else None)
        self._check(st)
        return out, (inf.as_dict() if info else None)

    def run(self, n_slices: int, infos: bool = False, probes: bool = False):
        arr = (SliceInfo * max(1, n_slices))() if infos else None
        pr = self.torch.zeros(max(1, len(self.cfg["probes"])), dtype=self.torch.float64,
                              device=self.device) if probes else None
        st = self.L.wandqs_run(self.ctx, int(n_slices),
                               C.c_void_p(pr.data_ptr()) if probes else None, arr)
        self._check(st)
        return ([a.as_dict() for a in arr[:n_slices]] if infos else None), pr

    def get_state(self):
        parts = self.torch.empty((4, self.P), dtype=self.torch.float64, device=self.device)
        flds = self._nodes(5)
        xd = (C.c_double * 2)()
        self._check(self.L.wandqs_get_state(self.ctx, C.c_void_p(parts.data_ptr()),
                                            C.c_void_p(flds.data_ptr()), xd))
        return dict(particles=parts, fields=flds, xi=xd[0], dxi=xd[1])

    def set_state(self, particles=None, fields=None, xi=None, dxi=None):
        t = self.torch
        p = f = None
        if particles is not None:
            p = t.as_tensor(particles, dtype=t.float64).to(self.device).contiguous()
            assert p.shape == (4, self.P)
        if fields is not None:
            f = t.as_tensor(fields, dtype=t.float64).to(self.device).contiguous()
            assert f.shape == (5, self.N + 1, self.N + 1)
        xd = None
        if xi is not None or dxi is not None:
            cur = self.get_state()
            xd = (C.c_double * 2)(cur["xi"] if xi is None else xi,
                                  cur["dxi"] if dxi is None else dxi)
        self.stream.synchronize()
        self._check(self.L.wandqs_set_state(self.ctx, C.c_void_p(p.data_ptr()) if p is not None else None,
                                            C.c_void_p(f.data_ptr()) if f is not None else None, xd))

    def mg_solve(self, f, u0=None, k2=None):
        """Solve (L_h - k2) u = f for 1 or 2 right-hand sides on this grid."""
        t = self.torch
        f = t.as_tensor(f, dtype=t.float64).to(self.device).contiguous()
        if f.dim() == 2:
            f = f.unsqueeze(0)
        nrhs = f.shape[0]
        u = t.zeros_like(f) if u0 is None else t.as_tensor(u0, dtype=t.float64).to(self.device).reshape(f.shape).contiguous().clone()
        kk = None if k2 is None else t.as_tensor(k2, dtype=t.float64).to(self.device).contiguous()
        cyc = C.c_int32(0)
        rel = (C.c_double * 2)()
        self.stream.synchronize()
        st = self.L.wandqs_mg_solve(self.ctx, nrhs, C.c_void_p(kk.data_ptr()) if kk is not None else None,
                                    C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()),
                                    C.byref(cyc), rel)
        if st not in (OK, E_NOCONV):
            self._check(st)
        return st, u, cyc.value, list(rel)[:nrhs]

    def nu_mg_solve(self, X, Y, J, u0=None, M=None):
        """Solve lap u + M u = J on the non-uniform grid of node coordinates X,
        Y ([N+1] each; arrays [N+1][N+1] indexed [j][i]).  Returns (status, u,
        cycles, rel)."""
        t = self.torch
        Xh = np.ascontiguousarray(X, dtype=np.float64)
        Yh = np.ascontiguousarray(Y, dtype=np.float64)
        assert Xh.size == self.N + 1 and Yh.size == self.N + 1
        Jd = t.as_tensor(J, dtype=t.float64).to(self.device).contiguous()
        u = (t.zeros_like(Jd) if u0 is None else
             t.as_tensor(u0, dtype=t.float64).to(self.device).contiguous().clone())
        Md = None if M is None else t.as_tensor(M, dtype=t.float64).to(self.device).contiguous()
        cyc = C.c_int32(0)
        rel = C.c_double(0.0)
        self.stream.synchronize()
        st = self.L.wandqs_nu_mg_solve(self.ctx, Xh.ctypes.data_as(_dp), Yh.ctypes.data_as(_dp),
                                       C.c_void_p(Md.data_ptr()) if Md is not None else None,
                                       C.c_void_p(Jd.data_ptr()), C.c_void_p(u.data_ptr()),
                                       C.byref(cyc), C.byref(rel))
        if st not in (OK, E_NOCONV):
            self._check(st)
        return st, u, cyc.value, rel.value

    # ------------------------------------------------------------ time loop
    def driver_set(self, state):
        """Driver macroparticles [8][n] (x, y, xi, px, py, pz, q/m, w)."""
        t = self.torch
        d = t.as_tensor(state, dtype=t.float64).to(self.device).contiguous()
        assert d.dim() == 2 and d.shape[0] == 8
        self._ndrv = int(d.shape[1])
        self.stream.synchronize()
        self._check(self.L.wandqs_driver_set(self.ctx, self._ndrv, C.c_void_p(d.data_ptr())))
        self.stream.synchronize()

    def driver_get(self):
        out = self.torch.empty((8, getattr(self, "_ndrv", 0)), dtype=self.torch.float64,
                               device=self.device)
        self._check(self.L.wandqs_driver_get(self.ctx, C.c_void_p(out.data_ptr())))
        return out

    def time_step(self, dt: float, n_slices: int, infos: bool = False):
        """One step of the time loop: a sweep of n_slices slices through the
        cold plasma with the driver's current, then the driver pushed by dt."""
        arr = (SliceInfo * max(1, n_slices))() if infos else None
        self._check(self.L.wandqs_time_step(self.ctx, C.c_double(dt), int(n_slices), arr))
        return [a.as_dict() for a in arr[:n_slices]] if infos else None

    # ---------------------------------------------------------------- laser
    def laser_set(self, env):
        """Laser envelope planes A-hat, complex [laser_nz][N+1][N+1] (None: no laser)."""
        t = self.torch
        if env is None:
            self._check(self.L.wandqs_laser_set(self.ctx, None))
            return
        e = t.as_tensor(env, dtype=t.complex128).to(self.device).contiguous()
        assert tuple(e.shape) == (int(self.cfg["laser_nz"]), self.N + 1, self.N + 1)
        self.stream.synchronize()
        self._check(self.L.wandqs_laser_set(self.ctx, C.c_void_p(e.data_ptr())))
        self.stream.synchronize()

    def laser_get(self):
        out = self.torch.empty((int(self.cfg["laser_nz"]), self.N + 1, self.N + 1),
                               dtype=self.torch.complex128, device=self.device)
        self._check(self.L.wandqs_laser_get(self.ctx, C.c_void_p(out.data_ptr())))
        return out

    def laser_advance(self, dt: float, chi=None):
        """Advance the envelope by dt with the susceptibility chi
        [laser_nz][N+1][N+1] (None: vacuum); returns the V-cycles per plane."""
        t = self.torch
        nz = int(self.cfg["laser_nz"])
        ch = None
        if chi is not None:
            ch = t.as_tensor(chi, dtype=t.float64).to(self.device).contiguous()
            assert tuple(ch.shape) == (nz, self.N + 1, self.N + 1)
        cyc = (C.c_int32 * max(1, nz))()
        self.stream.synchronize()
        self._check(self.L.wandqs_laser_advance(self.ctx, C.c_double(dt),
                                                C.c_void_p(ch.data_ptr()) if ch is not None else None,
                                                cyc))
        return list(cyc[:nz])

    def moments(self):
        out = self._nodes(9)
        self._check(self.L.wandqs_get_moments(self.ctx, C.c_void_p(out.data_ptr())))
        return out

    def profile(self, enable: bool = True):
        """Start (and reset) or stop per-kernel HIP-event timing."""
        self._check(self.L.wandqs_profile(self.ctx, 1 if enable else 0))

    def kernel_stats(self):
        """Per kernel instantiation: launches, total ms, algorithmic bytes."""
        n = C.c_int32(0)
        self._check(self.L.wandqs_profile_stats(self.ctx, None, 0, C.byref(n)))
        arr = (KernelStat * max(1, n.value))()
        self._check(self.L.wandqs_profile_stats(self.ctx, arr, n.value, C.byref(n)))
        return [dict(name=a.name.decode(), launches=a.launches, total_ms=a.total_ms,
                     alg_bytes=a.alg_bytes) for a in arr[:n.value]]

    @property
    def n_theta(self) -> int:
        return int(self.L.wandqs_num_theta(self.ctx))

    def tape_slices(self) -> int:
        return int(self.L.wandqs_tape_slices(self.ctx))

    def backward(self, dL_dprobe=None, dL_dfields=None, dL_dparticles=None,
                 particles_grad: bool = False):
        """Reverse sweep over the taped slices (needs checkpoint_every > 0).

        dL_dprobe: [n_probes] (the last run's probes); dL_dfields: [S][5][N+1][N+1]
        for the S taped slices; dL_dparticles: [4][P] adjoint of the final
        particles (ID order).  Returns (dL/dtheta as numpy, dL/d(initial
        particles) as a [4][P] device tensor or None)."""
        t = self.torch
        pr = None
        if dL_dprobe is not None:
            v = np.ascontiguousarray(np.asarray(dL_dprobe, dtype=np.float64).reshape(-1))
            if v.size != len(self.cfg["probes"]):
                raise ValueError("dL_dprobe needs one entry per probe")
            pr = v
        fb = None
        if dL_dfields is not None:
            fb = t.as_tensor(dL_dfields, dtype=t.float64).to(self.device).contiguous()
            S = self.tape_slices()
            if tuple(fb.shape) != (S, 5, self.N + 1, self.N + 1):
                raise ValueError(f"dL_dfields must be [{S}][5][N+1][N+1]")
        pb = None
        if dL_dparticles is not None:
            pb = t.as_tensor(dL_dparticles, dtype=t.float64).to(self.device).contiguous()
            if tuple(pb.shape) != (4, self.P):
                raise ValueError("dL_dparticles must be [4][P]")
        th = np.zeros(max(1, self.n_theta), dtype=np.float64)
        p0 = t.empty((4, self.P), dtype=t.float64, device=self.device) if particles_grad else None
        self.stream.synchronize()
        st = self.L.wandqs_backward(
            self.ctx, pr.ctypes.data_as(_dp) if pr is not None else None,
            C.c_void_p(fb.data_ptr()) if fb is not None else None,
            C.c_void_p(pb.data_ptr()) if pb is not None else None,
            th.ctypes.data_as(_dp), C.c_void_p(p0.data_ptr()) if p0 is not None else None)
        self._check(st)
        return th[:self.n_theta], p0

    def close(self):
        if getattr(self, "ctx", None):
            self.L.wandqs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_probe_fn = None


def run_probes(theta, cfg: dict, n_slices: int, checkpoint_every: int = 32):
    """Differentiable probe values of a run from the cold plasma: a torch
    function of theta (the driver parameters, see theta_of) whose backward is
    the library's reverse sweep.  Returns a float64 tensor [n_probes] on the
    GPU."""
    global _probe_fn
    import torch
    if _probe_fn is None:
        class _ProbeRun(torch.autograd.Function):
            @staticmethod
            def forward(ctx, th, cfg, n, K):
                c = with_theta(dict(cfg, checkpoint_every=int(K)), th.detach().cpu().numpy())
                sim = Simulation(c, n_slices=n)
                _, pr = sim.run(n, probes=True)
                ctx.sim = sim
                ctx.th_device = th.device
                return pr[:len(cfg["probes"])].clone()

            @staticmethod
            def backward(ctx, g):
                sim = ctx.sim
                try:
                    th, _ = sim.backward(dL_dprobe=g.detach().cpu().numpy())
                finally:
                    sim.close()
                return (torch.as_tensor(th, dtype=torch.float64, device=ctx.th_device),
                        None, None, None)
        _probe_fn = _ProbeRun
    return _probe_fn.apply(theta, cfg, int(n_slices), int(checkpoint_every))
