"""wandqs: the quasi-static xi-slice step of WAND-PIC (arXiv 2012.00881) on MI355X.

The compute path is the HIP library ``libwandqs.so`` (C ABI in
``include/wandqs.h``); :mod:`paper_2012_00881_amd.wandqs` is its ctypes binding.
"""
from .wandqs import (Simulation, WandQSError, load, make_config, mg_solve_noalloc, workspace_bytes,  # noqa: F401
                     EXPORTS, LIB_PATH, theta_of, with_theta, run_probes)
