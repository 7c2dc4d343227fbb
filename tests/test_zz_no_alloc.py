"""wandqs_mg_solve_noalloc (the solve with the library's static scratch array)
against wandqs_mg_solve on a context made with the same configuration.

Two calls in a row, the second on a smaller grid (the static array then still
holds the first call's larger layout), for each form and operator: the
results must equal the context path's bit for bit, since both run the same
kernels on the same inputs.  A grid above the array's limit and a tolerance
mode are rejected before any work is enqueued.
"""
import numpy as np
import pytest

import wandqs_inputs as wi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _case(N, nrhs, helm, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros((nrhs, N + 1, N + 1))
    f[:, 1:-1, 1:-1] = rng.standard_normal((nrhs, N - 1, N - 1))
    u0 = np.zeros_like(f)
    u0[:, 1:-1, 1:-1] = 0.1 * rng.standard_normal((nrhs, N - 1, N - 1))
    k2 = rng.uniform(0.0, 30.0, (N + 1, N + 1)) if helm else None
    return f, u0, k2


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("helm", [False, True])
def test_noalloc_equals_context_solve(torch_cuda, precision, helm):
    from paper_2012_00881_amd import Simulation, mg_solve_noalloc
    for N, nrhs, cycles, seed in ((256, 2, 3, 1), (128, 1, 2, 2)):
        print(f"[case] noalloc N={N} nrhs={nrhs} {precision} helm={helm} cycles={cycles}", flush=True)
        cfg = wi.scaled(wi.config("C2"), n_cells=N, precision=precision, mg_rtol=0.0,
                        mg_max_cycles=cycles)
        f, u0, k2 = _case(N, nrhs, helm, seed)
        st, u = mg_solve_noalloc(cfg, f, u0=u0, k2=k2)
        assert st == 0
        got = u.cpu().numpy()
        sim = Simulation(cfg)
        st2, ref, _, _ = sim.mg_solve(f, u0=u0, k2=k2)
        assert st2 == 0
        ref = ref.cpu().numpy()
        sim.close()
        d = float(np.abs(got - ref).max())
        print(f"max |noalloc - context| = {d:.3e}", flush=True)
        assert np.array_equal(got, ref), d
        # the solve did something: the residual moved
        assert float(np.abs(got - u0).max()) > 1e-3


def test_noalloc_rejects_what_it_cannot_do(torch_cuda):
    from paper_2012_00881_amd import WandQSError, mg_solve_noalloc
    f, _, _ = _case(512, 1, False, 3)
    with pytest.raises(WandQSError) as e:
        mg_solve_noalloc(wi.scaled(wi.config("C3"), mg_rtol=0.0, mg_max_cycles=1), f)
    assert e.value.status == -1 and "256" in str(e.value)
    f, _, _ = _case(64, 1, False, 4)
    with pytest.raises(WandQSError) as e:
        mg_solve_noalloc(wi.scaled(wi.config("C2"), n_cells=64), f)
    assert e.value.status == -1 and "mg_rtol" in str(e.value)
