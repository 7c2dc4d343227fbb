"""Parity metrics shared by the GPU tests (no method arithmetic here)."""
import numpy as np

FIELD_NAMES = ("psi", "Ez", "Bz", "Bx", "By")

#: FP64 GPU path vs oracle, relative field error of the FP64 form (1e-10)
FIELD_TOL = 1e-10

_I = (slice(1, -1), slice(1, -1))


def field_errors(gpu, ref):
    """Relative L2 error per field over interior nodes, with a floor of 1e-3 of
    the largest field norm (Bz can vanish for axisymmetric drivers)."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    norms = [np.linalg.norm(ref[k][_I]) for k in range(5)]
    floor = 1e-3 * max(max(norms), 1e-300)
    return np.array([np.linalg.norm((gpu[k] - ref[k])[_I]) / max(norms[k], floor)
                     for k in range(5)])


def field_maxabs_errors(gpu, ref):
    """Node-by-node error per field: max |F_gpu - F_orc| over the interior nodes
    divided by max |F_orc| of that field (floored at 1e-3 of the largest field
    maximum, as above).  A single wrong node fails this where the L2 measure
    averages it away."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    peaks = [np.abs(ref[k][_I]).max() for k in range(5)]
    floor = 1e-3 * max(max(peaks), 1e-300)
    return np.array([np.abs((gpu[k] - ref[k])[_I]).max() / max(peaks[k], floor)
                     for k in range(5)])


def check_fields(gpu, ref, tol, what=""):
    """Both field measures within tol; returns them for printing."""
    e2, emax = field_errors(gpu, ref), field_maxabs_errors(gpu, ref)
    print(f"{what} field errors L2 {np.array2string(e2, precision=2)} "
          f"max-abs {np.array2string(emax, precision=2)}", flush=True)
    assert np.all(e2 <= tol), (what, "L2", e2)
    assert np.all(emax <= tol), (what, "max-abs", emax)
    return e2, emax


def check_node_arrays(gpu, ref, tol, abs_floor=1e-13, what="moment"):
    """Node arrays compared node by node: max |a_gpu - a_ref| <= tol max |a_ref|
    + abs_floor for every array (an all-zero reference must be matched to the
    absolute floor)."""
    for k, (g, r) in enumerate(zip(gpu, ref)):
        d = float(np.abs(np.asarray(g) - np.asarray(r)).max())
        bound = tol * float(np.abs(r).max()) + abs_floor
        assert d <= bound, (what, k, d, bound)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
