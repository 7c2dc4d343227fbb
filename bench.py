#!/usr/bin/env python3
"""Benchmark of the quasi-static xi-slice step on one MI355X.

A step is one xi-slice of the whole hot path: cell sort, deposit of n*, the psi
Poisson solve, deposit of j and T, the Ez/Bz Poisson solves, the B_perp
Helmholtz assembly and solve, gather and push, adaptive step.  The workload is
the scale case: 1024^2 cells over [-10, 10]^2, 4 particles per cell
(4,194,304), Gaussian driver 20 n0 (sigma_r 0.25, sigma_z 0.6) plus a witness,
adaptive dxi (dxi0 = 0.005, refinement k = 8), FP64, multigrid solved to the
rounding floor.  Inputs are synthetic (the cold plasma lattice of the input
module) and resident on the GPU before the timed region.

Timed region: the job runs untimed from xi = 0 to the driver centre (xi >= 2 by
default: inside the blowout, where the solves are hardest and crowded cells
appear), then W warm-up slices, then K timed slices.  Printed value:
particle-slice updates per second (P * K / wall time).  The window's start
state is kept; a second pass over the same K slices from it records every
kernel launch with HIP events for the roofline of the dominant kernel, and the
FP64-vs-mixed comparison and the forward-plus-adjoint timing start from it too.
The CPU oracle is timed on a bounded sample of the same job from its own cold
start (it cannot reach the window within the run's time), on all the threads
it is given and on one.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
WORKLOAD = ("C5 scale run: 1024x1024 cells over [-10,10]^2, 4 particles/cell (4194304), "
            "driver n_b=20 sigma_r=0.25 sigma_z=0.6 at xi=2 + witness n_b=2 sigma_r=0.2 "
            "sigma_z=0.3 at xi=6.5, adaptive dxi0=0.005 k=8, FP64, MG to rounding floor")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2012_00881_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_record():
    """The committed counter summary, or None when it was taken on different
    kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    return rec if rec.get("source_hash") == kernel_source_hash() else None


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None."""
    rec = _traffic_record()
    k = None if rec is None else rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


# the multigrid (V-cycle) kernels: passes, coarse solves, norms, transfers
VCYCLE_PREFIXES = ("k_mg_", "k_coarse", "k_dst", "k_fst", "k_resnorm", "k_reduce_publish", "k_restrict_fw",
                   "k_correct")


def vcycle_bandwidth(stats, tot_ms):
    """Aggregate HBM rate of the V-cycle kernels over the profiled pass: the
    algorithmic bytes, and (when the counter summary matches these sources)
    the counted FETCH + WRITE bytes, each over the summed kernel durations."""
    vs = [s for s in stats if s["name"].startswith(VCYCLE_PREFIXES)]
    ms = sum(s["total_ms"] for s in vs)
    alg = sum(s["alg_bytes"] for s in vs)
    rec = _traffic_record()
    counted = None
    if rec is not None:
        ks = rec.get("kernels", {})
        if all(s["name"] in ks for s in vs):
            counted = sum(ks[s["name"]]["hbm_bytes_per_launch"] * s["launches"] for s in vs)
    out = {"kernels": len(vs), "share_of_kernel_time": round(ms / tot_ms, 4),
           "alg_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
           "alg_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "counted_GBps": None, "counted_frac": None}
    if counted is not None:
        out["counted_GBps"] = round(counted / (ms * 1e-3) / 1e9, 1)
        out["counted_frac"] = round(counted / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(cfg: dict, slices_all: int, slices_one: int, reps: int = 3):
    """The oracle on the first slices of the job from its cold start: `reps`
    runs of `slices_all` slices on all the threads OpenMP is given (the
    OMP_NUM_THREADS share of the host) and of `slices_one` slices on one
    thread; the median of each.  Its results do not depend on the thread
    count.  Returns the record for the all-threads figure."""
    import statistics
    import oracle
    orc = oracle.Oracle(cfg)
    n_all = oracle.get_threads()
    res = {}
    for nt, ns in ((n_all, slices_all), (1, slices_one)):
        oracle.set_threads(nt)
        rates, cyc = [], None
        for _ in range(reps):
            st = oracle.initial_state(cfg)
            t0 = time.perf_counter()
            r = orc.run(st, ns)
            dt = time.perf_counter() - t0
            assert r["status"] == 0, r["status"]
            rates.append(st["x"].size * ns / dt)
            cyc = [sum(i.cycles[k] for i in r["infos"]) / ns for k in range(5)]
        res[nt] = (statistics.median(rates), rates, cyc)
        print(f"[bench] oracle on {nt} thread(s): {ns} slices x {reps}: "
              f"{['%.3e' % v for v in rates]} particle-slice/s", file=sys.stderr, flush=True)
    oracle.set_threads(n_all)
    v_all, r_all, cyc = res[n_all]
    v_one = res[1][0]
    return dict(value=v_all, unit="particle-slice updates/s", cores=n_all, kind="oracle",
                single_core_value=v_one, runs=reps,
                sample=(f"median of {reps} runs of the first {slices_all} slices of the same job "
                        f"from its cold start (xi = 0) on {n_all} OpenMP threads, and of "
                        f"{reps} runs of {slices_one} slices on 1 thread ({v_one:.3e}/s); FP64 "
                        f"oracle, plain V(2,2) Gauss-Seidel, mean V-cycles per solve "
                        f"{[round(c, 2) for c in cyc]}, on {_cpu_model()}"))


def _start(sim, win):
    """Put the window's start state into a fresh context (its tape, if any,
    starts there)."""
    sim.set_state(particles=win["particles"], fields=win["fields"], xi=win["xi"], dxi=win["dxi"])


def adjoint_timing(cfg: dict, win: dict, S: int, K: int):
    """Forward without tape, forward with the tape (checkpoint every K) and the
    reverse sweep over the same S slices from the window's start state.  Loss:
    the mean Ez on a disc over the last S/4 slices plus a random linear
    function of the final particles, so every slice carries nonzero adjoints.
    The adaptive steps are held at the forward's values in the reverse sweep."""
    import numpy as np
    import torch
    from paper_2012_00881_amd import Simulation
    probe = dict(field=1, slice_begin=S - S // 4, slice_end=S, r_max=0.5, x0=0.0, y0=0.0)
    res = {"slices": S, "checkpoint_every": K, "xi_start": win["xi"]}
    for taped in (False, True):
        c = dict(cfg, probes=[probe], checkpoint_every=K if taped else 0, adjoint_hold_dxi=1)
        print(f"[bench] adjoint: forward {S} slices, tape {'on' if taped else 'off'}",
              file=sys.stderr, flush=True)
        sim = Simulation(c, n_slices=S)
        _start(sim, win)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(S, probes=True)
        torch.cuda.synchronize()
        res["forward_taped_s" if taped else "forward_s"] = time.perf_counter() - t0
        if not taped:
            sim.close()
            del sim
            continue
        pbar = torch.as_tensor(np.random.default_rng(1).standard_normal((4, sim.P)),
                               device="cuda")
        print(f"[bench] adjoint: reverse sweep", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        th, _ = sim.backward(dL_dprobe=[1.0], dL_dparticles=pbar)
        torch.cuda.synchronize()
        res["backward_s"] = time.perf_counter() - t0
        res["dL_dtheta"] = [float(v) for v in th]
        P = sim.P
        sim.close()
        del sim
    res["backward_over_forward"] = res["backward_s"] / res["forward_s"]
    # the forward-plus-adjoint form's throughput: particle-slices over the taped
    # forward and the reverse sweep together
    res["fwd_adj_value"] = P * S / (res["forward_taped_s"] + res["backward_s"])
    res["fwd_adj_unit"] = "particle-slice updates/s"
    res["ms_per_slice_backward"] = 1e3 * res["backward_s"] / S
    res["tape_overhead"] = res["forward_taped_s"] / res["forward_s"] - 1.0
    print(f"[bench] adjoint: forward {res['forward_s']:.3f} s, taped {res['forward_taped_s']:.3f} s, "
          f"backward {res['backward_s']:.3f} s ({res['backward_over_forward']:.2f}x forward)",
          file=sys.stderr, flush=True)
    return res


def forms_timing(cfg: dict, win: dict, S: int, rtol: float):
    """The FP64 and the mixed form, both solved to `rtol`, over the same S
    slices from the window's start state, against the FP64 path solved to the
    rounding floor over those slices: time per slice and every field's error
    after the last slice."""
    import numpy as np
    import torch
    import wandqs_inputs as wi
    from paper_2012_00881_amd import Simulation
    print(f"[bench] forms reference (FP64, rtol {cfg['mg_rtol']:g}): {S} slices", file=sys.stderr,
          flush=True)
    sim = Simulation(wi.scaled(cfg, precision="fp64"), n_slices=S)
    _start(sim, win)
    sim.run(S)
    ref = sim.get_state()["fields"].cpu().numpy()
    sim.close()
    del sim
    out = {"rtol": rtol, "steps": S, "xi_start": win["xi"]}
    for prec in ("fp64", "mixed"):
        fc = wi.scaled(cfg, precision=prec, mg_rtol=rtol)
        print(f"[bench] form {prec} @ rtol {rtol:g}: {S} slices", file=sys.stderr, flush=True)
        sim = Simulation(fc, n_slices=S)
        _start(sim, win)
        torch.cuda.synchronize()
        tf = time.perf_counter()
        fi, _ = sim.run(S, infos=True)
        torch.cuda.synchronize()
        tf = time.perf_counter() - tf
        got = sim.get_state()["fields"].cpu().numpy()
        P = sim.P
        sim.close()
        del sim
        # per-field error after the last slice: relative L2 over the interior
        # (floored at 1e-3 of the largest field, for B_z = 0 runs) and node by node
        I = (slice(1, -1), slice(1, -1))
        big = max(float(np.linalg.norm(ref[j][I])) for j in range(5))
        bigm = max(float(np.abs(ref[j][I]).max()) for j in range(5))
        errs = [float(np.linalg.norm((got[k] - ref[k])[I]) /
                      max(np.linalg.norm(ref[k][I]), 1e-3 * big)) for k in range(5)]
        merrs = [float(np.abs((got[k] - ref[k])[I]).max() /
                       max(np.abs(ref[k][I]).max(), 1e-3 * bigm)) for k in range(5)]
        out[prec] = {
            "value": P * S / tf, "ms_per_step": 1e3 * tf / S,
            "mean_vcycles": [round(sum(i["vcycles"][k] for i in fi) / len(fi), 3) for k in range(5)],
            "field_rel_err_vs_fp64_full": [float("%.3g" % e) for e in errs],
            "field_maxabs_err_vs_fp64_full": [float("%.3g" % e) for e in merrs],
            "within_1e-6": bool(max(errs + merrs) <= 1e-6)}
    out["mixed_speedup"] = out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    print(f"[bench] mixed speedup at rtol {rtol:g}: {out['mixed_speedup']:.3f}", file=sys.stderr,
          flush=True)
    return out


def laser_timing(cfg: dict, S: int):
    """The laser-driven time loop on the workload's grid and plasma: a Gaussian
    laser (a0 = 2, w0 = 3, sigma_z = 1, k0 = 20) on S envelope planes with fixed
    steps dxi = 0.02, one time step dt = 10 (the plasma swept through the S
    slices, each advancing its envelope plane): ms per slice, the envelope's
    multigrid cycles per plane, and a profiled step's split between the
    envelope kernels and the rest."""
    import torch
    import wandqs_inputs as wi
    from paper_2012_00881_amd import Simulation
    dxi, k0, dt = 0.02, 20.0, 10.0
    c = wi.scaled(cfg, beams=[], adaptive=0, dxi0=dxi, laser_nz=S, laser_k0=k0)
    env = wi.laser_gaussian(c["n_cells"], c["half_width"], S, dxi, 2.0, 3.0, 0.5 * S * dxi, 1.0)
    env_t = torch.as_tensor(env, device="cuda")
    res = {"slices": S, "dxi": dxi, "dt": dt, "k0": k0, "a0": 2.0, "w0": 3.0, "sigma_z": 1.0}
    sim = Simulation(c, n_slices=S)
    sim.laser_set(env_t)
    print(f"[bench] laser: warm-up time step of {S} slices", file=sys.stderr, flush=True)
    sim.time_step(dt, S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = sim.time_step(dt, S, infos=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter() - t0
    res["ms_per_slice"] = 1e3 * t1 / S
    res["value"] = sim.P * S / t1
    res["unit"] = "particle-slice updates/s (with the envelope advance)"
    res["mean_laser_vcycles"] = sum(i["laser_vcycles"] for i in infos) / S
    res["mean_vcycles"] = [round(sum(i["vcycles"][k] for i in infos) / S, 3) for k in range(5)]
    sim.profile(True)
    sim.time_step(dt, S)
    st = sim.kernel_stats()
    sim.close()
    tot = sum(x["total_ms"] for x in st)
    las = [x for x in st if x["name"].startswith("k_las")]
    lms = sum(x["total_ms"] for x in las)
    res["laser_kernel_share"] = round(lms / tot, 4)
    res["laser_kernel_ms_per_slice"] = round(lms / S, 4)
    res["laser_alg_GBps"] = round(sum(x["alg_bytes"] for x in las) / (lms * 1e-3) / 1e9, 1)
    print(f"[bench] laser: {res}", file=sys.stderr, flush=True)
    return res


def nonuniform_timing(cfg: dict, reps: int = 3):
    """The non-uniform grid solver (Sec. VII.B) on the workload's grid size: the
    three-region axis (spacing 1 : 2 : 3 from the axis out) in x and y, a
    Gaussian source of the bubble's size (the shape of n* - 1), the Poisson
    and the Helmholtz (M = -1) forms from a zero guess to the rounding floor:
    ms per solve, cycles, and the solver kernels' algorithmic HBM rate."""
    import numpy as np
    import torch
    import wandqs_inputs as wi
    from paper_2012_00881_amd import Simulation
    N, L = cfg["n_cells"], cfg["half_width"]
    X = wi.nonuniform_axis(N, L, "regions")
    XX, YY = np.meshgrid(X, X, indexing="xy")
    J = -np.exp(-(XX ** 2 + YY ** 2) / 4.0)
    c = wi.scaled(cfg, mg_max_cycles=200)
    sim = Simulation(c)
    res = {"grid": N, "axis": "three regions, spacing 1:2:3", "source": "Gaussian, width 2"}
    for name, M in (("poisson", None), ("helmholtz", -np.ones_like(J))):
        sim.nu_mg_solve(X, X, J, M=M)  # warm-up
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, u, cyc, rel = sim.nu_mg_solve(X, X, J, M=M)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            assert st == 0, st
        res[name] = {"ms_per_solve": round(1e3 * min(times), 3), "cycles": cyc,
                     "ms_per_cycle": round(1e3 * min(times) / cyc, 4), "rel_resid": rel}
    sim.profile(True)
    sim.nu_mg_solve(X, X, J)
    st = sim.kernel_stats()
    sim.close()
    nu = [x for x in st if x["name"].startswith("k_nu")]
    ms = sum(x["total_ms"] for x in nu)
    res["kernel_alg_GBps"] = round(sum(x["alg_bytes"] for x in nu) / (ms * 1e-3) / 1e9, 1)
    res["kernels"] = {x["name"]: {"launches": x["launches"], "ms": round(x["total_ms"], 3)}
                      for x in sorted(nu, key=lambda x: -x["total_ms"])[:6]}
    print(f"[bench] non-uniform solver: {res}", file=sys.stderr, flush=True)
    return res


def workload_timing(name: str, xi_start: float, steps: int):
    """Another workload's window, timed like the headline: the job run untimed
    to xi_start, `steps` slices timed, then replayed with per-kernel timing
    for the V-cycle kernels' aggregate HBM rate."""
    import torch
    import wandqs_inputs as wi
    from paper_2012_00881_amd import Simulation
    cfg = wi.config(name)
    sim = Simulation(cfg, n_slices=max(steps, 64))
    xi = 0.0
    while xi < xi_start:
        sim.run(64)
        xi = sim.get_state()["xi"]
    win = sim.get_state()
    win = dict(particles=win["particles"].clone(), fields=win["fields"].clone(), xi=win["xi"],
               dxi=win["dxi"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, _ = sim.run(steps, infos=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    P = sim.P
    xi_end = sim.get_state()["xi"]
    sim.close()
    sim = Simulation(cfg, n_slices=steps)
    _start(sim, win)
    sim.profile(True)
    sim.run(steps)
    stats = sim.kernel_stats()
    sim.close()
    groups = {}
    for st in stats:
        g = groups.setdefault(st["name"].split("@")[0], dict(name=st["name"].split("@")[0],
                                                             launches=0, total_ms=0.0, alg_bytes=0.0))
        g["launches"] += st["launches"]
        g["total_ms"] += st["total_ms"]
        g["alg_bytes"] += st["alg_bytes"]
    gl = list(groups.values())
    tot = sum(x["total_ms"] for x in gl)
    res = {"workload": name, "grid": cfg["n_cells"], "particles": P, "slices": steps,
           "value": P * steps / dt, "ms_per_slice": 1e3 * dt / steps, "xi_start": win["xi"],
           "xi_end": xi_end,
           "mean_vcycles": [round(sum(i["vcycles"][k] for i in infos) / steps, 3) for k in range(5)],
           "vcycle_hbm": vcycle_bandwidth(gl, tot)}
    print(f"[bench] {name}: {res}", file=sys.stderr, flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=256)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--xi-start", type=float, default=2.0,
                    help="run the job untimed up to this xi before the warm-up and timed slices "
                         "(default: the driver centre, inside the blowout)")
    ap.add_argument("--workload", default="C5")
    ap.add_argument("--cpu-slices", type=int, default=4,
                    help="oracle slices per timed run on all threads (1 thread: half as many)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile-pass", action="store_true")
    ap.add_argument("--breakdown", default=None, help="write per-kernel stats (JSON) here")
    ap.add_argument("--nu", type=int, default=None, help="pre- and post-smoothing sweeps")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--rtol", type=float, default=None, help="multigrid rtol (default 1e-14)")
    ap.add_argument("--inner", type=int, default=0, help="mixed: FP32 cycles per correction")
    ap.add_argument("--forms-steps", type=int, default=512,
                    help="slices of the FP64-vs-mixed comparison (0: skip)")
    ap.add_argument("--forms-rtol", type=float, default=None,
                    help="multigrid rtol of both forms in that comparison (default: the input "
                         "module's FORMS_RTOL)")
    ap.add_argument("--adjoint-steps", type=int, default=512,
                    help="slices of the taped forward + reverse sweep (0: skip)")
    ap.add_argument("--checkpoint-every", type=int, default=32)
    ap.add_argument("--pusher-steps", type=int, default=128,
                    help="slices timed from the window with each Runge-Kutta pusher (0: skip)")
    ap.add_argument("--laser-steps", type=int, default=256,
                    help="envelope planes (slices) of the laser-driven time step (0: skip)")
    ap.add_argument("--c3-steps", type=int, default=128,
                    help="slices of the C3 (512^2, driver + witness) window, from xi = 2 (0: skip)")
    ap.add_argument("--no-nonuniform", action="store_true",
                    help="skip the non-uniform grid solver timing")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB three times (the "
                         "reference for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the slice step is not sharded "
              "across GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import wandqs_inputs as wi
    from paper_2012_00881_amd import Simulation

    cfg = wi.scaled(wi.config(args.workload), precision=args.precision,
                    mg_inner_cycles=args.inner)
    if args.nu is not None:
        cfg.update(nu_pre=args.nu, nu_post=args.nu)
    if args.rtol is not None:
        cfg.update(mg_rtol=args.rtol)
    K, W = args.steps, args.warmup

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * 2**20 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 x {args.copy_calibration_mib} MiB", file=sys.stderr,
              flush=True)
        del src, dst

    sim = Simulation(cfg, n_slices=max(K, W, 64))
    P = sim.P
    lead = 0
    xi = 0.0
    while xi < args.xi_start:
        sim.run(64)
        lead += 64
        xi = sim.get_state()["xi"]
    print(f"[bench] lead-in: {lead} slices to xi={xi:.4f}; warm-up: {W} slices", file=sys.stderr,
          flush=True)
    if W:
        sim.run(W)
    win = sim.get_state()
    win = dict(particles=win["particles"].clone(), fields=win["fields"].clone(), xi=win["xi"],
               dxi=win["dxi"])
    print(f"[bench] timed: {K} slices from xi={win['xi']:.4f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, _ = sim.run(K, infos=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    final = sim.get_state()
    sim.close()
    del sim
    value = P * K / dt
    cyc = [sum(i["vcycles"][k] for i in infos) / max(1, len(infos)) for k in range(5)]
    print(f"[bench] {K} slices in {dt:.3f} s: {value:.4e} particle-slice/s, xi {win['xi']:.4f} -> "
          f"{final['xi']:.4f}, mean V-cycles per solve {['%.2f' % c for c in cyc]}",
          file=sys.stderr, flush=True)

    roof = None
    vcycle = None
    stats = []
    if not args.no_profile_pass:
        print("[bench] profiled pass (HIP events per launch) over the same slices", file=sys.stderr,
              flush=True)
        sim = Simulation(cfg, n_slices=max(K, 1))
        _start(sim, win)
        sim.profile(True)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        sim.run(K)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        per_level = sorted(sim.kernel_stats(), key=lambda s: -s["total_ms"])
        sim.close()
        del sim
        # group the per-level records by kernel (the unit a profiler reports)
        groups = {}
        for s in per_level:
            g = groups.setdefault(s["name"].split("@")[0], dict(name=s["name"].split("@")[0],
                                                                 launches=0, total_ms=0.0,
                                                                 alg_bytes=0.0))
            g["launches"] += s["launches"]
            g["total_ms"] += s["total_ms"]
            g["alg_bytes"] += s["alg_bytes"]
        stats = sorted(groups.values(), key=lambda s: -s["total_ms"])
        tot = sum(s["total_ms"] for s in stats)
        for s in stats[:14]:
            avg = s["total_ms"] / s["launches"]
            print(f"[bench]   {s['name']:34s} {s['launches']:7d} launches {s['total_ms']:9.2f} ms "
                  f"({100 * s['total_ms'] / tot:5.1f}%) avg {1e3 * avg:8.2f} us "
                  f"{s['alg_bytes'] / (s['total_ms'] * 1e-3) / 1e9:8.1f} GB/s",
                  file=sys.stderr, flush=True)
        for s in per_level:
            if "@" in s["name"] and s["total_ms"] > 0.02 * tot:
                print(f"[bench]     level {s['name']:38s} avg {1e3 * s['total_ms'] / s['launches']:8.2f} us "
                      f"{s['alg_bytes'] / (s['total_ms'] * 1e-3) / 1e9:8.1f} GB/s", file=sys.stderr,
                      flush=True)
        dom = stats[0]
        avg_s = dom["total_ms"] * 1e-3 / dom["launches"]
        bytes_per_launch = dom["alg_bytes"] / dom["launches"]
        achieved = bytes_per_launch / avg_s / 1e9
        traffic = measured_traffic(dom["name"])
        roof = {"bound": "hbm", "kernel": dom["name"], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "alg_bytes_per_launch": round(bytes_per_launch),
                "avg_launch_us": round(avg_s * 1e6, 2), "launches": dom["launches"],
                "share_of_kernel_time": round(dom["total_ms"] / tot, 4),
                "kernel_ms_per_slice": round(tot / K, 4),
                "profiled_pass_s": round(tp, 3)}
        vcycle = vcycle_bandwidth(stats, tot)
        print(f"[bench] V-cycle kernels: {vcycle}", file=sys.stderr, flush=True)
        if args.breakdown:
            os.makedirs(os.path.dirname(os.path.abspath(args.breakdown)), exist_ok=True)
            with open(args.breakdown, "w") as fh:
                json.dump(dict(workload=args.workload, slices=K, particles=P, xi_start=win["xi"],
                               stats=stats, per_level=per_level,
                               source_hash=kernel_source_hash()), fh, indent=1)

    forms = None
    if args.forms_steps > 0:
        forms = forms_timing(cfg, win, args.forms_steps,
                             args.forms_rtol if args.forms_rtol is not None else wi.FORMS_RTOL)

    pushers = None
    if args.pusher_steps > 0:
        # the same window with each Runge-Kutta pusher (the Boris-like one is
        # the headline's)
        pushers = {}
        for pu in ("rk1", "rk2", "rk4"):
            print(f"[bench] pusher {pu}: {args.pusher_steps} slices", file=sys.stderr, flush=True)
            sim = Simulation(wi.scaled(cfg, pusher=pu), n_slices=args.pusher_steps)
            _start(sim, win)
            torch.cuda.synchronize()
            tq = time.perf_counter()
            sim.run(args.pusher_steps)
            torch.cuda.synchronize()
            tq = time.perf_counter() - tq
            sim.close()
            del sim
            pushers[pu] = {"value": P * args.pusher_steps / tq,
                           "ms_per_step": 1e3 * tq / args.pusher_steps}
        pushers["steps"] = args.pusher_steps
        print(f"[bench] pushers: {pushers}", file=sys.stderr, flush=True)

    laser = None
    if args.laser_steps > 0:
        laser = laser_timing(cfg, args.laser_steps)

    c3 = None
    if args.c3_steps > 0:
        c3 = workload_timing("C3", 2.0, args.c3_steps)

    nonuniform = None
    if not args.no_nonuniform:
        nonuniform = nonuniform_timing(cfg)

    adjoint = None
    if args.adjoint_steps > 0:
        adjoint = adjoint_timing(cfg, win, args.adjoint_steps, args.checkpoint_every)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, args.cpu_slices, max(1, args.cpu_slices // 2))

    line = {"metric": "particle-slice updates/s", "value": value,
            "unit": "particle-slice updates/s", "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": 1e3 * dt / K, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f64+f32",
            "data": "synthetic",
            "config": {"workload": WORKLOAD if args.workload == "C5" else args.workload,
                       "grid": cfg["n_cells"], "particles": P, "slices": K,
                       "precision": args.precision, "mg_rtol": cfg["mg_rtol"],
                       "coarse_corrections": "the FP64 form's Helmholtz coarse levels (<= 64^2) "
                                             "sweep in FP32; its Poisson cycles end on level 1 "
                                             "with an FP64 fast-sine-transform solve (an FP32 one "
                                             "at 64^2 on 128^2 grids); the FP64 fine levels' "
                                             "residuals carry the answer to the FP64 rounding floor",
                       "lead_in_slices": lead, "xi_start": win["xi"], "xi_end": final["xi"],
                       "mean_vcycles": [round(c, 3) for c in cyc]},
            "roofline": roof, "vcycle_hbm": vcycle, "cpu_baseline": cpu, "forms": forms,
            "adjoint": adjoint, "pushers": pushers, "laser": laser, "nonuniform": nonuniform,
            "c3": c3}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
