#!/usr/bin/env python3
"""Throughput benchmark of the fused rectangular-lattice CM-LBM step on one GPU.

Default workload: lid-driven cavity on a square physical domain, nx 512 x
ny 1024 nodes at aspect ratio r = dy/dx = 0.5, Re 1000, lid speed 0.05,
FP32-deviation storage, RC collision (the raw-moment RNR variant is timed
beside it).  A step is one collide-and-stream pass over the whole lattice;
every `--check-every` steps the FP64 residual and conservation reductions run
inside the timed region, as in a run to steady state (enqueued without a host
wait and read one interval later, as a monitored production run would).  Inputs (the cavity at
rest, after the warm-up steps) are resident in HBM when timing starts.

Prints ONE JSON line: MLUPS of the whole job, the roofline of the step kernel
(algorithmic bytes per launch / mean launch time from HIP events on the
library's stream), the HBM traffic measured by rocprofv3 counters (when
profiles/ holds a measurement of the current kernel source) and the CPU
oracle timed on a bounded sample on the host.  On the cavity it also times
a cold start to a residual of 1e-8 (in FP64).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2103_02119_amd", "csrc", "lbm_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

WORKLOADS = {
    # name: nx, ny, r, cs2, bc types, wall velocities, Re, lid/velocity scale
    "cavity": dict(nx=512, ny=1024, r=0.5, cs2=0.16, bc=(1, 1, 1, 2), U=0.05, Re=1000.0),
    "tgv": dict(nx=1024, ny=2048, r=0.5, cs2=0.16, bc=(0, 0, 0, 0), U=0.02, nu=0.1),
    # the shear layer's own nu = 1e-4 (tau = 0.5025) is below the scheme's
    # small-tau stability limit on this lattice and blows up within a few
    # hundred steps; the throughput run uses nu = 6e-3 (tau = 0.65), which
    # stays finite for 30 000 steps (the step's cost does not depend on nu)
    "shear": dict(nx=2048, ny=8192, r=0.25, cs2=0.04, bc=(0, 0, 0, 0), U=0.04, nu=6e-3),
}


def kernel_sha():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def setup(name, precision, collision, rows=0):
    from paper_2103_02119_amd import inputs as I
    from paper_2103_02119_amd import lbm as L

    w = WORKLOADS[name]
    nx, ny, r, cs2 = w["nx"], w["ny"], w["r"], w["cs2"]
    nu = w["U"] * nx / w["Re"] if "Re" in w else w["nu"]
    tau = nu / cs2 + 0.5
    rates = [1.0, 1.0, 1.0, 1.0, 1.0 / tau, 1.0 / tau, 1.0, 1.0, 1.0]
    uw = ((0, 0), (0, 0), (0, 0), (w["U"], 0)) if name == "cavity" else ((0, 0),) * 4
    lat = L.Lattice(nx, ny, r, rates, bc_types=w["bc"], u_wall=uw, cs2=cs2,
                    collision=collision, precision=precision, rows_per_wave=rows)
    if name == "cavity":
        lat.set_fields(*I.cavity_rest(nx, ny))
    elif name == "tgv":
        lat.set_fields(*I.taylor_green(nx, ny, r, w["U"], cs2))
    else:
        lat.set_fields(*I.shear_layer(nx, ny, r, u0=w["U"]))
    return lat, dict(nx=nx, ny=ny, r=r, cs2=cs2, tau=tau, nu=nu)


def time_steps(lat, steps, check_every, chunk):
    """Times `steps` steps issued `chunk` launches at a time (one C-level
    loop per chunk), each chunk bracketed by HIP events on torch's current
    stream (the stream the library enqueues on).  Every `check_every` steps
    the FP64 residual and conservation reductions are enqueued without a
    host wait (lbm_check_async), and the previous check's results are read
    then, one interval later, so the queue never drains; the last one is
    read before the clock stops.  Returns the wall time, the per-launch
    kernel times from the events and the step of the first check that
    reported a non-finite field (None if none did)."""
    import torch

    from paper_2103_02119_amd import lbm as L

    s = torch.cuda.current_stream()
    nchunks = (steps + chunk - 1) // chunk
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(nchunks)]
    sizes = []
    blew_up = None
    pending = None  # steps done at the enqueued, unread check

    def read():
        nonlocal blew_up
        try:
            lat.check_result()
        except L.LbmError as e:
            if e.code != L.LBM_E_UNSTABLE:
                raise
            blew_up = pending

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    for c in range(nchunks):
        n = min(chunk, steps - done)
        ev[c][0].record(s)
        lat.step(n)
        ev[c][1].record(s)
        sizes.append(n)
        done += n
        if check_every and done % check_every == 0 and blew_up is None:
            if pending is not None:
                read()
            lat.check_async()
            pending = done
    if pending is not None and blew_up is None:
        read()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_launch = [a.elapsed_time(b) / n for (a, b), n in zip(ev, sizes)]
    return wall, per_launch, blew_up


def cpu_baseline(name, collision, budget_s=10.0):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload (the same lattice advanced from the same start)."""
    import numpy as np

    import oracle as O
    from paper_2103_02119_amd import inputs as I

    w = WORKLOADS[name]
    nx, ny, r, cs2 = w["nx"], w["ny"], w["r"], w["cs2"]
    nu = w["U"] * nx / w["Re"] if "Re" in w else w["nu"]
    tau = nu / cs2 + 0.5
    rates = [1.0, 1.0, 1.0, 1.0, 1.0 / tau, 1.0 / tau, 1.0, 1.0, 1.0]
    uw = ((0, 0), (0, 0), (0, 0), (w["U"], 0)) if name == "cavity" else ((0, 0),) * 4
    p = O.make_params(nx, ny, r, cs2, rates, bc=w["bc"], u_wall=uw, collision=collision)
    if name == "cavity":
        f = O.init(p, *I.cavity_rest(nx, ny))
    elif name == "tgv":
        f = O.init(p, *I.taylor_green(nx, ny, r, w["U"], cs2))
    else:
        f = O.init(p, *I.shear_layer(nx, ny, r, u0=w["U"]))
    f = O.run(p, f, 1)  # first-touch / page-in
    steps, t = 0, 0.0
    chunk = 2
    while t < budget_s:
        t0 = time.perf_counter()
        f = O.run(p, f, chunk)
        t += time.perf_counter() - t0
        steps += chunk
    assert np.isfinite(f).all()
    cores = O.max_threads()
    # the same oracle on one thread, for a quarter of the budget
    O.set_threads(1)
    steps1, t1 = 0, 0.0
    try:
        while t1 < budget_s / 4:
            t0 = time.perf_counter()
            f = O.run(p, f, 1)
            t1 += time.perf_counter() - t0
            steps1 += 1
    finally:
        O.set_threads(cores)
    return dict(value=round(nx * ny * steps / t / 1e6, 3), unit="MLUPS", cores=cores,
                kind="oracle",
                sample=f"{name} {nx}x{ny} r={r}, FP64 oracle, {steps} steps ({t:.1f} s) "
                       f"from the same start, {'RC' if collision == 0 else 'RNR'}",
                single_core_value=round(nx * ny * steps1 / t1 / 1e6, 3))


def time_to_steady(name, tol=1e-8, check_every=1000, cap=2_000_000):
    """Cold start (fluid at rest) to a per-step residual <= tol, in FP64:
    FP32 storage has a residual floor near 1e-7..1e-6 (rounding noise keeps
    the weakly damped acoustic modes alive), so it never reaches 1e-8.
    Returns steps and wall seconds (the residual is checked every
    `check_every` steps, so steps are resolved to that)."""
    import torch

    from paper_2103_02119_amd import lbm as L

    lat, _ = setup(name, L.LBM_FP64, L.LBM_RC)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, R = 0, float("inf")
    while steps < cap:
        lat.step(check_every)
        steps += check_every
        R = lat.residual()
        if R <= tol:
            break
    wall = time.perf_counter() - t0
    lat.close()
    return dict(cold_steps=steps if R <= tol else None, cold_seconds=round(wall, 3),
                residual=R, tol=tol, precision="fp64", collision="RC",
                checked_every=check_every, warm_steps=None, warm_seconds=None,
                warm_start="not on this lattice: the network is trained on 256x128 cavities "
                           "with obstacles (python -m paper_2103_02119_amd.warmstart)")


def bench_sweep(args):
    """The 512-case batch (cavities and channels, nx 64..512, r in
    {0.25, 0.5, 1}, Re 100..5000, FP32 deviations) advanced together by the
    persistent batched kernel, autotuned, graph-replayed."""
    import torch

    from paper_2103_02119_amd import inputs as I
    from paper_2103_02119_amd import lbm as L
    from paper_2103_02119_amd import workloads as W

    prec = L.LBM_FP32_DEV if args.precision == "fp32dev" else L.LBM_FP64
    bytes_per_lu = 72 if prec == L.LBM_FP32_DEV else 144
    params = I.batch_sweep()
    cases = W.sweep_cases(params)
    nodes = sum(c.nx * c.ny for c in cases)
    stream = torch.cuda.Stream()
    b = L.Batch(cases, precision=prec, graph_steps=args.graph_steps, stream=stream.cuda_stream)
    rows, wgs = b.autotune(5)
    tile = b.uses_tile_kernel()
    steps = (args.steps + args.graph_steps - 1) // args.graph_steps * args.graph_steps
    b.step(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    R = b.residuals()
    kern_ms = e0.elapsed_time(e1) / steps
    achieved = bytes_per_lu * nodes / (kern_ms * 1e-3) / 1e9
    out = {
        "metric": "MLUPS + % HBM roofline; time-to-steady-state warm-start vs cold",
        "value": round(nodes * steps / wall / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == L.LBM_FP32_DEV else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"batch sweep {len(cases)} cases ({sum(p['kind'] == 'cavity' for p in params)} "
                        f"cavities, the rest channels), nx 64..512, r in 0.25/0.5/1, Re 100..5000, "
                        f"{nodes} nodes",
            "collision": "RC",
            "rows_per_wave": rows, "workgroups": wgs, "graph_steps": args.graph_steps,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "algorithmic_bytes_per_launch": bytes_per_lu * nodes,
            "kernel": "lbm::batch_tile_kernel" if tile else "lbm::batch_step_kernel",
            "bytes_per_lu": bytes_per_lu,
            "kernel_us": round(1e3 * kern_ms, 3),
        },
        "unstable_cases": int(np.isnan(R).sum()),
    }
    if args.steady_cap:
        t0 = time.perf_counter()
        got = b.run_to_steady(args.steady_tol, args.steady_every, args.steady_cap)
        out["time_to_steady"] = {
            "tol": args.steady_tol, "cap": args.steady_cap, "checked_every": args.steady_every,
            "seconds": round(time.perf_counter() - t0, 3),
            "converged": int((got > 0).sum()), "blew_up": int((got == -1).sum()),
            "not_converged": int((got == -2).sum()),
            "median_steps_converged": int(np.median(got[got > 0])) if (got > 0).any() else None,
        }
    b.close()
    print(json.dumps(out), flush=True)


def copy_probe(nbytes=1 << 30, reps=20):
    """Plain device copy of a known size (counter calibration and the
    achievable HBM bandwidth)."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes": nbytes, "read_plus_write_GBs": round(2 * nbytes / ms / 1e6, 1),
                      "ms": round(ms, 4)}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["sweep"], default="cavity")
    ap.add_argument("--graph-steps", type=int, default=64, help="sweep: steps per captured graph")
    ap.add_argument("--steady-cap", type=int, default=0,
                    help="sweep: also run every case to --steady-tol, at most this many steps")
    ap.add_argument("--steady-tol", type=float, default=1e-6)
    ap.add_argument("--steady-every", type=int, default=1000)
    ap.add_argument("--precision", choices=["fp32dev", "fp64"], default="fp32dev")
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--chunk", type=int, default=100, help="launches per host call")
    ap.add_argument("--rows", type=int, default=0, help="rows per wavefront (0 = automatic)")
    ap.add_argument("--no-rnr", action="store_true", help="skip the RNR side-by-side timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--no-steady", action="store_true",
                    help="skip the cold-start time-to-steady-state run (cavity only)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only; a multi-GPU lattice step would "
              "shard by slabs with a halo exchange, which is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2103_02119_amd import lbm as L

    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()
        return
    if args.workload == "sweep":
        bench_sweep(args)
        return
    prec = L.LBM_FP32_DEV if args.precision == "fp32dev" else L.LBM_FP64
    bytes_per_lu = 72 if prec == L.LBM_FP32_DEV else 144

    lat, info = setup(args.workload, prec, L.LBM_RC, args.rows)
    nodes = info["nx"] * info["ny"]
    lat.step(args.warmup)
    torch.cuda.synchronize()
    wall, kern, blew_up = time_steps(lat, args.steps, args.check_every, args.chunk)
    try:
        R = lat.residual()
        sums = lat.sums()
    except L.LbmError as e:
        if e.code != L.LBM_E_UNSTABLE:
            raise
        R, sums = float("nan"), [float("nan")] * 3
        blew_up = blew_up or args.warmup + args.steps
    rows, wgs = lat.launch_shape()
    lat.close()

    rnr = None
    if not args.no_rnr:
        lat2, _ = setup(args.workload, prec, L.LBM_RNR, args.rows)
        lat2.step(args.warmup)
        wall2, kern2, _ = time_steps(lat2, args.steps, args.check_every, args.chunk)
        lat2.close()
        rnr = dict(mlups=round(nodes * args.steps / wall2 / 1e6, 1),
                   kernel_us=round(1e3 * sum(kern2) / len(kern2), 3))

    mlups = nodes * args.steps / wall / 1e6
    kern_ms = sum(kern) / len(kern)
    achieved = bytes_per_lu * nodes / (kern_ms * 1e-3) / 1e9
    # HBM bytes per launch from the rocprofv3 counters recorded in profiles/,
    # valid only for the kernel source they were measured on
    traffic, traffic_ratio = None, None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        key = f"{args.workload}/{args.precision}"
        if tr.get("kernel_sha") == kernel_sha() and key in tr.get("per_launch", {}):
            traffic = tr["per_launch"][key]["bytes_per_launch"]
            traffic_ratio = tr["per_launch"][key]["ratio"]

    out = {
        "metric": "MLUPS + % HBM roofline; time-to-steady-state warm-start vs cold",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == L.LBM_FP32_DEV else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload} {info['nx']}x{info['ny']} r={info['r']}"
                        + (f" Re={WORKLOADS[args.workload]['Re']:g} lid={WORKLOADS[args.workload]['U']}"
                           if args.workload == "cavity" else ""),
            "collision": "RC (RNR beside it)",
            "storage": "FP32 deviations f - w rho0" if prec == L.LBM_FP32_DEV else "FP64",
            "cs2": info["cs2"], "tau": round(info["tau"], 6),
            "residual_every": args.check_every,
            "residual_read": "asynchronous, one interval later",
            "launches_per_host_call": args.chunk,
            "rows_per_wave": rows, "workgroups": wgs,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_over_algorithmic": traffic_ratio,
            "algorithmic_bytes_per_launch": bytes_per_lu * nodes,
            "kernel": "lbm::tile_step_kernel" if args.rows == 0 else "lbm::step_kernel",
            "bytes_per_lu": bytes_per_lu,
            "kernel_us": round(1e3 * kern_ms, 3),
        },
        "rnr": rnr,
        "final_residual": R,
        "mass": sums[0],
        "nonfinite_at_step": blew_up,
    }
    if args.workload == "cavity" and not args.no_steady:
        out["time_to_steady"] = time_to_steady(args.workload)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, L.LBM_RC, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
