"""Seeded synthetic inputs for the quasi-static slice step.

This module is shared by the CPU oracle tests and by the GPU path's tests,
benchmark and smoke check.  It holds no arithmetic of the method itself: only
the workload descriptions (grid, box, plasma, driver beams, step size) and the
initial plasma state.

Initial plasma (paper Sec. III.A: a cold homogeneous plasma at rest before the
driver arrives, H = 1 and P = 0 for every electron):

* ``s x s`` macroparticles per cell on a sub-lattice at cell-local offsets
  ``(i + 1/2)/s``, optionally displaced by a uniform jitter of ``+-J`` cells
  per coordinate, transverse momenta zero;
* cells are visited row-major (y index ``b`` outer, x index ``a`` inner), the
  sub-particles of a cell in ``(sy, sx)`` order, and for each particle the x
  jitter is drawn before the y jitter; the particle ID is its place in this
  order;
* the jitter draws come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014), which is counter based: draw
  ``k`` of a stream with seed ``s`` is ``mix64(s + (k + 1) * 0x9E3779B97F4A7C15)``
  and maps to ``[0, 1)`` as ``(z >> 11) * 2**-53``.

The GPU library builds the same lattice itself from the same published
generator; a test asserts that both arrays are bitwise identical.

Workloads (all lengths in 1/k_p, densities in n0, normalisation of the paper's
Sec. III): the Gaussian driver density is ``amp * exp(-r^2/sr^2 - (xi-xc)^2/sz^2)``
(no factor 1/2; this convention reproduces the normalised charge Q = 5.34 quoted
in Sec. V.A for the 2 nC beam).
"""
from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Draws ``start .. start+count-1`` of the SplitMix64 stream with ``seed`` (uint64)."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + k * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """SplitMix64 draws mapped to [0, 1) with 53 random bits."""
    z = splitmix64(seed, count, start)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def plasma_lattice(n_cells: int, half_width: float, ppc_side: int, jitter: float,
                   seed: int):
    """Initial plasma macroparticles in ID order: arrays x, y, px, py (float64)."""
    N, L, s, J = int(n_cells), float(half_width), int(ppc_side), float(jitter)
    h = 2.0 * L / N
    b, a, sy, sx = np.meshgrid(np.arange(N), np.arange(N), np.arange(s), np.arange(s),
                               indexing="ij")
    a = a.ravel().astype(np.float64)
    b = b.ravel().astype(np.float64)
    sx = sx.ravel().astype(np.float64)
    sy = sy.ravel().astype(np.float64)
    P = a.size
    u = uniform01(seed, 2 * P)
    ux, uy = u[0::2], u[1::2]
    x = -L + h * ((a + (sx + 0.5) / s) + J * (2.0 * ux - 1.0))
    y = -L + h * ((b + (sy + 0.5) / s) + J * (2.0 * uy - 1.0))
    z = np.zeros(P)
    return x, y, z.copy(), z.copy()


def normal01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Standard normal draws by the Box-Muller transform (G. E. P. Box and
    M. E. Muller, Ann. Math. Statist. 29, 610 (1958)) of SplitMix64 pairs:
    z = sqrt(-2 ln(1 - u1)) cos(2 pi u2)."""
    u = uniform01(seed, 2 * count, start)
    return np.sqrt(-2.0 * np.log1p(-u[0::2])) * np.cos(2.0 * np.pi * u[1::2])


#: driver state rows: positions, momenta, charge-to-mass ratio (e/m_e units)
#: and weight (number of particles in units of n0 k_p^-3)
DRIVER_ROWS = ("x", "y", "xi", "px", "py", "pz", "qm", "w")


def driver_gaussian(beam: dict, n: int, seed: int, gamma0: float = 2000.0, qm: float = -1.0):
    """n driver macroparticles of equal weight sampled from the density
    amp exp(-r^2/sr^2 - (xi - xc)^2/sz^2) of a Gaussian beam (x, y and xi each
    normal with standard deviation sigma/sqrt 2), all moving along z with
    p_z = sqrt(gamma0^2 - 1) (electrons: qm = -1).  Returns [8][n]."""
    z = normal01(seed, 3 * n)
    sr, sz = beam["sigma_r"] / np.sqrt(2.0), beam["sigma_z"] / np.sqrt(2.0)
    total = beam["amp"] * np.pi * beam["sigma_r"] ** 2 * np.sqrt(np.pi) * beam["sigma_z"]
    out = np.zeros((8, n))
    out[0] = beam.get("x0", 0.0) + sr * z[0::3]
    out[1] = beam.get("y0", 0.0) + sr * z[1::3]
    out[2] = beam["xi_c"] + sz * z[2::3]
    out[5] = np.sqrt(gamma0 * gamma0 - 1.0)
    out[6] = qm
    out[7] = total / n
    return out


def driver_lattice(beam: dict, n_cells: int, half_width: float, xi0: float, dz: float, nz: int,
                   gamma0: float = 2000.0, qm: float = -1.0, cut: float = 1e-12):
    """A quiet driver: one macroparticle on every transverse node x_a, y_b and
    deposit plane xi_m = xi0 + m dz (m = 1 .. nz-2) where the Gaussian density
    exceeds cut times its peak, weighted by that density times h^2 dz, so that
    its deposit is the density itself on the nodes and planes.  Returns [8][n]."""
    N, L = int(n_cells), float(half_width)
    h = 2.0 * L / N
    g = -L + h * np.arange(N + 1)
    xis = xi0 + dz * np.arange(1, nz - 1)
    XI, Y, X = np.meshgrid(xis, g, g, indexing="ij")
    r2 = (X - beam.get("x0", 0.0)) ** 2 + (Y - beam.get("y0", 0.0)) ** 2
    dens = beam["amp"] * np.exp(-r2 / beam["sigma_r"] ** 2 - (XI - beam["xi_c"]) ** 2 / beam["sigma_z"] ** 2)
    keep = (dens > cut * beam["amp"]) & (np.abs(X) < L) & (np.abs(Y) < L)
    n = int(keep.sum())
    out = np.zeros((8, n))
    out[0], out[1], out[2] = X[keep], Y[keep], XI[keep]
    out[5] = np.sqrt(gamma0 * gamma0 - 1.0)
    out[6] = qm
    out[7] = dens[keep] * h * h * dz
    return out


def laser_gaussian(n_cells: int, half_width: float, nz: int, dxi: float, a0: float, w0: float,
                   xi_c: float, sigma_z: float, x0: float = 0.0, y0: float = 0.0):
    """Envelope planes of a Gaussian laser pulse on the nodes, planes xi_m =
    m dxi (m = 0 .. nz-1): a0 exp(-r^2/w0^2 - (xi - xi_c)^2/sigma_z^2), real
    (zero phase), zero on the boundary nodes.  Returns complex [nz][N+1][N+1]."""
    N, L = int(n_cells), float(half_width)
    h = 2.0 * L / N
    g = -L + h * np.arange(N + 1)
    xis = dxi * np.arange(nz)
    XI, Y, X = np.meshgrid(xis, g, g, indexing="ij")
    r2 = (X - x0) ** 2 + (Y - y0) ** 2
    env = a0 * np.exp(-r2 / w0 ** 2 - (XI - xi_c) ** 2 / sigma_z ** 2)
    env[:, 0, :] = env[:, -1, :] = env[:, :, 0] = env[:, :, -1] = 0.0
    return env.astype(np.complex128)


def nonuniform_axis(n_cells: int, half_width: float, kind: str = "regions") -> np.ndarray:
    """Node coordinates x_0 = -L < ... < x_N = L of a non-uniform axis.

    "regions": three regions as in the paper's bubble example, spacing ratio
    1 : 2 : 3 from the axis out (|s| < 1/4, 1/4 <= |s| < 1/2, beyond), with
    abrupt changes; s = -1 + 2a/N is the uniform index coordinate, so the
    region edges fall on nodes for N >= 8 and a refined grid keeps them.
    "smooth": smooth stretching x = L sinh(2 s)/sinh(2), finest at the axis
    (the spacing grows by cosh(2) ~ 3.8 towards the edges)."""
    N, L = int(n_cells), float(half_width)
    s = -1.0 + 2.0 * np.arange(N + 1) / N
    if kind == "smooth":
        return L * np.sinh(2.0 * s) / np.sinh(2.0)
    a = np.abs(s)
    # slope 1, 2, 3 on [0, 1/4), [1/4, 1/2), [1/2, 1]; scaled so x(1) = L
    x = np.where(a < 0.25, a, np.where(a < 0.5, 0.25 + 2 * (a - 0.25), 0.75 + 3 * (a - 0.5)))
    return np.sign(s) * x * (L / 2.25)


def gauss_beam(amp, sigma_r, sigma_z, xi_c, x0=0.0, y0=0.0):
    return dict(kind="gauss", amp=float(amp), sigma_r=float(sigma_r), sigma_z=float(sigma_z),
                xi_c=float(xi_c), x0=float(x0), y0=float(y0))


def radial_bins_beam(bin_amp, r_max, sigma_z, xi_c, x0=0.0, y0=0.0):
    """Driver whose radial profile is piecewise constant on len(bin_amp) equal bins of [0, r_max)."""
    bin_amp = np.asarray(bin_amp, dtype=np.float64)
    return dict(kind="radial_bins", bin_amp=bin_amp, r_max=float(r_max), sigma_z=float(sigma_z),
                xi_c=float(xi_c), x0=float(x0), y0=float(y0), amp=1.0, sigma_r=1.0)


#: multigrid tolerance at which the FP64 and mixed forms are compared for
#: speed (every field must stay within 1e-6 of the oracle there)
FORMS_RTOL = 1e-7


def _base(**kw):
    cfg = dict(n_cells=64, half_width=6.0, ppc_side=1, jitter=0.0, seed=0, n0=1.0,
               dxi0=0.0625, adaptive=0, refine_k=0, precision="fp64",
               mg_rtol=1e-14, mg_atol=0.0, mg_max_cycles=50, nu_pre=2, nu_post=2,
               beams=[], probes=[], checkpoint_every=0, n_slices=128)
    cfg.update(kw)
    return cfg


def config(name: str) -> dict:
    """The five workloads of the build (linear wake, blowout, mixed, adjoint, scale)."""
    if name == "C1":   # linear regime, lattice, fixed step
        return _base(name=name, n_cells=64, half_width=6.0, ppc_side=1, jitter=0.0,
                     dxi0=0.0625, adaptive=0, refine_k=0, n_slices=128,
                     beams=[gauss_beam(0.1, 0.5, 1.0, 2.0)])
    if name == "C2":   # blowout, adaptive step
        return _base(name=name, n_cells=256, half_width=8.0, ppc_side=2, jitter=0.25, seed=2,
                     dxi0=0.02, adaptive=1, refine_k=8, n_slices=1024,
                     beams=[gauss_beam(10.0, 0.3, 0.7, 2.0)])
    if name == "C3":   # driver + witness, mixed precision form
        return _base(name=name, n_cells=512, half_width=8.0, ppc_side=2, jitter=0.25, seed=3,
                     dxi0=0.01, adaptive=1, refine_k=8, n_slices=2048, precision="mixed",
                     beams=[gauss_beam(5.0, 0.4, 0.8, 2.0), gauss_beam(2.0, 0.2, 0.3, 6.5)])
    if name == "C4":   # adjoint: 32 radial-bin amplitudes of the driver
        N, L = 256, 8.0
        h = 2 * L / N
        amps = 0.5 + 1.5 * uniform01(40, 32)
        return _base(name=name, n_cells=N, half_width=L, ppc_side=2, jitter=0.25, seed=4,
                     dxi0=0.02, adaptive=0, refine_k=0, n_slices=512, checkpoint_every=32,
                     beams=[radial_bins_beam(amps, 32 * h, 0.8, 2.0)],
                     probes=[dict(field=1, slice_begin=300, slice_end=351, r_max=0.5,
                                  x0=0.0, y0=0.0)])
    if name == "C5":   # scale run: driver + witness, adaptive step
        return _base(name=name, n_cells=1024, half_width=10.0, ppc_side=2, jitter=0.25, seed=5,
                     dxi0=0.005, adaptive=1, refine_k=8, n_slices=4096,
                     beams=[gauss_beam(20.0, 0.25, 0.6, 2.0), gauss_beam(2.0, 0.2, 0.3, 6.5)])
    raise KeyError(name)


def scaled(cfg: dict, **kw) -> dict:
    """Copy of a workload with some entries replaced (smaller grids for quick cases)."""
    out = dict(cfg)
    out["beams"] = [dict(b) for b in cfg["beams"]]
    out["probes"] = [dict(p) for p in cfg["probes"]]
    out.update(kw)
    return out


def synthetic_state(cfg: dict, seed: int, p_max: float = 0.5, disp: float = 0.45,
                    xi: float = 2.0, dxi: float | None = None, field_amp: float = 0.0):
    """A mid-run-like plasma state for single-slice parity cases.

    Particles start from the lattice of ``cfg`` and are displaced by up to
    ``disp`` cells (uniform, SplitMix64 stream ``seed``), given momenta uniform in
    ``[-p_max, p_max]`` per component, and placed at ``xi`` with step ``dxi``.
    ``field_amp`` scales smooth previous-slice fields used only as multigrid
    initial guesses.  Returns dict(x, y, px, py, fields[5,N+1,N+1], xi, dxi).
    """
    N, L = cfg["n_cells"], cfg["half_width"]
    h = 2.0 * L / N
    x, y, px, py = plasma_lattice(N, L, cfg["ppc_side"], cfg["jitter"], cfg["seed"])
    P = x.size
    u = uniform01(seed, 4 * P, start=0)
    x = x + disp * h * (2.0 * u[0::4] - 1.0)
    y = y + disp * h * (2.0 * u[1::4] - 1.0)
    x = np.clip(x, -L, L)
    y = np.clip(y, -L, L)
    px = p_max * (2.0 * u[2::4] - 1.0)
    py = p_max * (2.0 * u[3::4] - 1.0)
    g = -L + h * np.arange(N + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    fields = np.zeros((5, N + 1, N + 1))
    if field_amp != 0.0:
        base = np.sin(np.pi * (X + L) / (2 * L)) * np.sin(np.pi * (Y + L) / (2 * L))
        for k in range(5):
            fields[k] = field_amp * (k + 1) * base * np.cos(0.3 * k * X)
        fields[:, 0, :] = fields[:, -1, :] = 0.0
        fields[:, :, 0] = fields[:, :, -1] = 0.0
    return dict(x=x, y=y, px=px, py=py, fields=fields, xi=float(xi),
                dxi=float(cfg["dxi0"] if dxi is None else dxi))


def vortex_state(cfg: dict, p0: float, width: float, xi: float = 2.0, dxi: float | None = None,
                 x0: float = 0.3, y0: float = -0.2):
    """Lattice plasma of ``cfg`` with a smooth swirl of transverse momentum.

    ``p = p0 * (-(y - y0), x - x0) * exp(-((x-x0)^2 + (y-y0)^2) / width^2)``; no
    random numbers, so the state is smooth at the grid scale.  The swirl gives the
    plasma current a curl, hence a non-zero Bz, for single-slice cases that must
    exercise every term of the B-perp source.
    """
    N, L = cfg["n_cells"], cfg["half_width"]
    x, y, _, _ = plasma_lattice(N, L, cfg["ppc_side"], 0.0, 0)
    rx, ry = x - x0, y - y0
    env = p0 * np.exp(-(rx * rx + ry * ry) / (width * width))
    return dict(x=x, y=y, px=-ry * env, py=rx * env, fields=np.zeros((5, N + 1, N + 1)),
                xi=float(xi), dxi=float(cfg["dxi0"] if dxi is None else dxi))
