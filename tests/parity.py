"""Parity metrics shared by the GPU tests (no method arithmetic here)."""
import numpy as np

FIELD_NAMES = ("psi", "Ez", "Bz", "Bx", "By")

#: FP64 GPU path vs oracle, relative field error (spec tolerance)
FIELD_TOL = 1e-10


def field_errors(gpu, ref):
    """Relative L2 error per field over interior nodes, with a floor of 1e-3 of
    the largest field norm (Bz can vanish for axisymmetric drivers)."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    I = (slice(1, -1), slice(1, -1))
    norms = [np.linalg.norm(ref[k][I]) for k in range(5)]
    floor = 1e-3 * max(max(norms), 1e-300)
    return np.array([np.linalg.norm((gpu[k] - ref[k])[I]) / max(norms[k], floor)
                     for k in range(5)])


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
