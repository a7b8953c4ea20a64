#!/usr/bin/env python3
"""Throughput benchmark of the fused rectangular-lattice CM-LBM step on one GPU.

Default workload: the doubly periodic shear layer on nx 2048 x ny 8192 nodes
at aspect ratio r = dy/dx = 0.25 (kappa 80, delta 0.05, u0 0.04), FP32
deviation storage, RC collision.  Its two population buffers (1.2 GB) are far
beyond the 256 MB Infinity Cache, so the step is bound by HBM: this is the
roofline workload.  A step is one collide-and-stream pass over the whole
lattice.  The timed region runs `--steps` steps in chunks of `--chunk`; every
chunk's launches fuse two steps each except the last one or two, which fuse
one, and every `--check-every` steps and at the end of the timed region the
FP64 residual and conservation reductions run (enqueued without a host wait;
the last one is read before the clock stops).  Inputs (the shear layer after
the warm-up steps) are resident in HBM when timing starts.

Beside the headline it reports: the library's own streaming copy of one
population buffer (the copy ceiling), the one-step-per-launch kernel, the
same workload in FP64 and with the raw-moment (RNR) collision, the
cache-resident 512 x 1024 cavity, time to steady state (cold and from the
learned warm start), the FP32-storage velocity error against FP64 at the
cavity's converged state and over 50 000 steps of the shear layer, and the
FP64 CPU oracle timed on a bounded sample on the host.

Prints ONE JSON line.  The roofline is that of the dominant kernel: its
algorithmic bytes per launch (9 reads + 9 writes per node) over its mean
launch time from HIP events on the library's stream inside the timed region.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2103_02119_amd", "csrc")
KERNEL_SRCS = ("lbm_device.h", "lbm_tile.hip", "lbm_tile2.hip", "lbm_internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
METRIC = "MLUPS + % HBM roofline; time-to-steady-state warm-start vs cold"

WORKLOADS = {
    # name: nx, ny, r, cs2, bc types, wall velocities, Re or nu, velocity scale
    "cavity": dict(nx=512, ny=1024, r=0.5, cs2=0.16, bc=(1, 1, 1, 2), U=0.05, Re=1000.0),
    "tgv": dict(nx=1024, ny=2048, r=0.5, cs2=0.16, bc=(0, 0, 0, 0), U=0.02, nu=0.1),
    # the shear layer's own nu = 1e-4 (tau = 0.5025) is below the scheme's
    # small-tau stability limit on this lattice and blows up within a few
    # hundred steps; the throughput run uses nu = 6e-3 (tau = 0.65), which
    # stays finite for 30 000 steps (the step's cost does not depend on nu)
    "shear": dict(nx=2048, ny=8192, r=0.25, cs2=0.04, bc=(0, 0, 0, 0), U=0.04, nu=6e-3),
}
# 80% of the 8 TB/s HBM roofline at the one-step traffic of 72 B (FP32
# deviations) or 144 B (FP64) per lattice update, in MLUPS
TARGET_MLUPS = {"fp32dev": 0.8 * HBM_PEAK_GBS * 1e9 / 72 / 1e6,
                "fp64": 0.8 * HBM_PEAK_GBS * 1e9 / 144 / 1e6}


def kernel_sha():
    h = hashlib.sha256()
    for name in KERNEL_SRCS:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def params_of(name):
    w = WORKLOADS[name]
    nx, ny, r, cs2 = w["nx"], w["ny"], w["r"], w["cs2"]
    nu = w["U"] * nx / w["Re"] if "Re" in w else w["nu"]
    tau = nu / cs2 + 0.5
    rates = [1.0, 1.0, 1.0, 1.0, 1.0 / tau, 1.0 / tau, 1.0, 1.0, 1.0]
    uw = ((0, 0), (0, 0), (0, 0), (w["U"], 0)) if name == "cavity" else ((0, 0),) * 4
    return w, nx, ny, r, cs2, nu, tau, rates, uw


def initial_fields(name, nx, ny, r, w, cs2):
    from paper_2103_02119_amd import inputs as I
    if name == "cavity":
        return I.cavity_rest(nx, ny)
    if name == "tgv":
        return I.taylor_green(nx, ny, r, w["U"], cs2)
    return I.shear_layer(nx, ny, r, u0=w["U"])


def setup(name, precision, collision):
    from paper_2103_02119_amd import lbm as L

    w, nx, ny, r, cs2, nu, tau, rates, uw = params_of(name)
    lat = L.Lattice(nx, ny, r, rates, bc_types=w["bc"], u_wall=uw, cs2=cs2,
                    collision=collision, precision=precision)
    lat.set_fields(*initial_fields(name, nx, ny, r, w, cs2))
    return lat, dict(nx=nx, ny=ny, r=r, cs2=cs2, tau=tau, nu=nu)


def time_steps(lat, steps, check_every, chunk, spl):
    """Times `steps` steps in chunks of `chunk`.  With two steps per launch
    (spl = 2) a chunk of c steps is (c - 1) // 2 two-step launches bracketed
    by HIP events on torch's current stream (the library's stream), then one
    or two one-step launches, so that the state one step back exists for the
    check; with spl = 1 the events bracket all c launches.  Every
    `check_every` steps, and once at the end, the FP64 residual and
    conservation reductions are enqueued without a host wait
    (lbm_check_async) and the previous check's results are read then; the
    last one is read before the clock stops.  Returns the wall time, the mean
    time of one bracketed launch, the number of checks and the step of the
    first check that found a non-finite field (None if none did)."""
    import torch

    from paper_2103_02119_amd import lbm as L

    s = torch.cuda.current_stream()
    lat.set_steps_per_launch(spl)
    plan = []
    done = 0
    while done < steps:
        c = min(chunk, steps - done)
        pairs = (c - 1) // 2 if spl == 2 else 0
        plan.append((c, pairs))
        done += c
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in plan]
    blew_up, pending, checks = None, None, 0

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
    for i, (c, pairs) in enumerate(plan):
        if spl == 2:
            ev[i][0].record(s)
            lat.step(2 * pairs)
            ev[i][1].record(s)
            for _ in range(c - 2 * pairs):
                lat.step(1)
        else:
            ev[i][0].record(s)
            lat.step(c)
            ev[i][1].record(s)
        done += c
        last = i == len(plan) - 1
        if (last or (check_every and done % check_every == 0)) and blew_up is None:
            if pending is not None:
                read()
            lat.check_async()
            checks += 1
            pending = done
    if pending is not None and blew_up is None:
        read()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches = [(a.elapsed_time(b), (p if spl == 2 else c)) for (a, b), (c, p) in zip(ev, plan)]
    tot_ms = sum(t for t, n in launches if n > 0)
    tot_n = sum(n for _, n in launches)
    return wall, (tot_ms / tot_n if tot_n else float("nan")), checks, blew_up


def time_launches(lat, spl, n):
    """Mean time (ms) of n back-to-back launches of spl steps each, from HIP
    events on the library's stream (outside the timed region)."""
    import torch

    lat.set_steps_per_launch(spl)
    if spl == 2:
        lat.step(1)  # pull form
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    lat.step(spl * n)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def copy_ceiling(nbytes, reps=10):
    """The library's streaming copy (lbm_stream_copy) of one population
    buffer's size, best over a few grid sizes: the read-plus-write bandwidth
    a plain stream reaches on this GPU."""
    import torch

    from paper_2103_02119_amd import lbm as L

    nbytes = nbytes // 16 * 16
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()
    best = None
    per_grid = {}
    for wgs in (2048, 4096, 8192, 16384, 65536):
        L.lbm_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, wgs, s.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            L.lbm_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, wgs, s.cuda_stream)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = 2 * nbytes / (ms * 1e-3) / 1e9
        per_grid[wgs] = round(gbs, 1)
        if best is None or gbs > best[0]:
            best = (gbs, wgs, ms)
    assert torch.equal(a[:4096], b[:4096])
    del a, b
    torch.cuda.empty_cache()
    return dict(kernel="lbm::stream_copy_kernel (lbm_stream_copy)", bytes_each_way=nbytes,
                GBs=round(best[0], 1), workgroups=best[1], us=round(1e3 * best[2], 2),
                per_workgroups_GBs=per_grid)


def run_workload(name, prec_name, collision, args, spl=0, one_step=True):
    """Setup, warm-up and the timed region for one workload; returns a dict."""
    import torch

    from paper_2103_02119_amd import lbm as L

    prec = L.LBM_FP32_DEV if prec_name == "fp32dev" else L.LBM_FP64
    lat, info = setup(name, prec, collision)
    nodes = info["nx"] * info["ny"]
    k = spl or lat.steps_per_launch()
    lat.set_steps_per_launch(k)
    form = lat.two_step_form()
    lat.step(args.warmup)
    torch.cuda.synchronize()
    wall, kern_ms, checks, blew_up = time_steps(lat, args.steps, args.check_every, args.chunk, k)
    try:
        R = lat.residual()
        sums = lat.sums()
    except L.LbmError as e:
        if e.code != L.LBM_E_UNSTABLE:
            raise
        R, sums = float("nan"), [float("nan")] * 3
        blew_up = blew_up or args.warmup + args.steps
    vb = 4 if prec == L.LBM_FP32_DEV else 8
    kernel = ("lbm::tile_step_kernel" if k == 1 else
              "lbm::tile2_staged_kernel" if form == L.LBM_FORM_STAGED else "lbm::tile2_step_kernel")
    out = dict(nodes=nodes, info=info, wall=wall, steps_per_launch=k, kernel_ms=kern_ms, kernel=kernel,
               mlups=nodes * args.steps / wall / 1e6, checks=checks, residual=R, mass=sums[0],
               nonfinite_at_step=blew_up, value_bytes=vb,
               bytes_per_launch=18 * vb * nodes)
    if one_step:
        out["one_step_ms"] = time_launches(lat, 1, max(args.steps, 10))
        if k == 1:
            out["two_step_ms"] = time_launches(lat, 2, max(args.steps // 2, 5))
    lat.close()
    torch.cuda.empty_cache()
    return out


def roofline_of(r, copy_gbs, traffic=None):
    bpl = r["bytes_per_launch"]
    k = r["steps_per_launch"]
    achieved = bpl / (r["kernel_ms"] * 1e-3) / 1e9
    out = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic[0] if traffic else None,
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "traffic_over_algorithmic": traffic[1] if traffic else None,
        "valu_issue": valu_ceiling_of(r, traffic[2] if traffic else None,
                                      traffic[3] if traffic else None,
                                      "fp32" if r.get("value_bytes", 4) == 4 else "fp64"),
        "kernel": r["kernel"],
        "steps_per_launch": k,
        "algorithmic_bytes_per_launch": bpl,
        "bytes_per_lu": bpl // (k * r["nodes"]),
        "kernel_us": round(1e3 * r["kernel_ms"], 3),
        "kernel_time_from": "HIP events on the library's stream around the timed region's "
                            + ("two-step launches" if k == 2 else "launches"),
    }
    if copy_gbs:
        out["copy_ceiling_GBs"] = copy_gbs
        out["frac_of_copy"] = round(achieved / copy_gbs, 4)
    return out


def one_step_line(r, copy_gbs):
    ms = r.get("one_step_ms")
    if not ms:
        return None
    bpl = r["bytes_per_launch"]
    gbs = bpl / (ms * 1e-3) / 1e9
    d = dict(kernel="lbm::tile_step_kernel", kernel_us=round(1e3 * ms, 3),
             achieved_GBs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
             kernel_mlups=round(r["nodes"] / (ms * 1e-3) / 1e6, 1))
    if copy_gbs:
        d["frac_of_copy"] = round(gbs / copy_gbs, 4)
    return d


def traffic_of(key):
    """HBM bytes per launch from the rocprofv3 counters recorded in profiles/,
    valid only for the kernel source they were measured on."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    if tr.get("kernel_sha") == kernel_sha() and key in tr.get("per_launch", {}):
        e = tr["per_launch"][key]
        return e["bytes_per_launch"], e["ratio"], e.get("valu_insts_per_64_lu"), e.get("flops_per_lu")
    return None


# one wave64 vector instruction per CU per cycle (four SIMDs of 16 lanes)
N_CU, CLOCK_GHZ = 256, 2.4
# MI355X vector peaks (TFLOP/s): FP32 as published (counts packed FP32
# instructions, which this library does not use), FP32 without them (one FMA
# per lane per cycle: 256 CUs x 64 lanes x 2 x 2.4 GHz), FP64
PEAK_TFLOPS = {"fp32": 157.3, "fp32_unpacked": 78.6, "fp64": 78.6}


def valu_ceiling_of(r, valu_per_64, flops_per_lu=None, arith="fp32"):
    """The kernel's vector-ALU issue ceiling in lattice updates per second:
    256 CUs x 2.4 GHz x one wave64 instruction per CU per cycle, over the
    VALU instructions per lattice update that the counters measured; and the
    floating-point rate those counters give, against the vector peaks."""
    if not valu_per_64:
        return None
    peak = N_CU * CLOCK_GHZ * 1e9 / (valu_per_64 / 64) / 1e9  # GLUPS
    got = r["steps_per_launch"] * r["nodes"] / (r["kernel_ms"] * 1e-3) / 1e9
    out = {"bound": "alu", "unit": "GLUPS", "achieved": round(got, 1), "peak": round(peak, 1),
           "frac": round(got / peak, 4), "valu_insts_per_64_lu": valu_per_64,
           "peak_from": "256 CUs x 2.4 GHz x one wave64 VALU instruction per CU per cycle "
                        "(unpacked), over SQ_INSTS_VALU per lattice update (profiles/)"}
    if flops_per_lu:
        tf = got * flops_per_lu / 1e3
        out["flops"] = {"flops_per_lu": flops_per_lu, "achieved_tflops": round(tf, 2),
                        "arithmetic": arith, "peak_tflops": PEAK_TFLOPS[arith],
                        "frac": round(tf / PEAK_TFLOPS[arith], 4)}
        if arith == "fp32":
            out["flops"]["peak_tflops_unpacked"] = PEAK_TFLOPS["fp32_unpacked"]
            out["flops"]["frac_unpacked"] = round(tf / PEAK_TFLOPS["fp32_unpacked"], 4)
        out["flops"]["from"] = "executed FP adds, multiplies, FMAs (x2) and transcendentals " \
                               "counted by rocprofv3 (profiles/traffic.json)"
    return out


def cpu_baseline(name, collision, budget_s=10.0):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload (the same lattice advanced from the same start)."""
    import oracle as O

    w, nx, ny, r, cs2, nu, tau, rates, uw = params_of(name)
    p = O.make_params(nx, ny, r, cs2, rates, bc=w["bc"], u_wall=uw, collision=collision)
    f = O.init(p, *initial_fields(name, nx, ny, r, w, cs2))
    f = O.run(p, f, 1)  # first touch
    steps, t = 0, 0.0
    while t < budget_s:
        t0 = time.perf_counter()
        f = O.run(p, f, 1)
        t += time.perf_counter() - t0
        steps += 1
    assert np.isfinite(f).all()
    cores = O.max_threads()
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
                cpu_model=cpu_model(),
                single_core_value=round(nx * ny * steps1 / t1 / 1e6, 3),
                single_core_sample=f"{steps1} steps ({t1:.1f} s) on one thread")


def cavity_steady(tol=1e-8, check_every=10_000, cap=2_000_000):
    """The 512 x 1024 cavity from rest to a per-step residual <= tol in
    FP64 (cold time to steady state), then both FP32-storage modes for the
    same number of steps: their velocity distance from the FP64 field at
    that converged state (max |du| / max |u|).  FP32 storage itself never
    reaches 1e-8: rounding noise keeps the weakly damped acoustic modes
    alive (residual floor near 1e-7 .. 1e-6)."""
    import torch

    from paper_2103_02119_amd import lbm as L

    lat, _ = setup("cavity", L.LBM_FP64, L.LBM_RC)
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
    progress(f"cavity fp64 from rest: residual {R:.2e} after {steps} steps, {wall:.1f} s")
    _, ux64, uy64 = lat.moments()
    lat.close()
    umax = float(np.hypot(ux64, uy64).max())
    err = {}
    for prec, name in ((L.LBM_FP32_DEV, "fp32_storage_fp32_arithmetic"),
                       (L.LBM_FP32_DEV_F64, "fp32_storage_fp64_arithmetic")):
        lat, _ = setup("cavity", prec, L.LBM_RC)
        lat.step(steps)
        _, ux, uy = lat.moments()
        lat.close()
        err[name] = float(np.hypot(ux - ux64, uy - uy64).max() / umax)
    return dict(workload="cavity 512x1024 r=0.5 Re=1000 lid=0.05, from rest",
                cold_steps=steps if R <= tol else None, cold_seconds=round(wall, 3),
                residual=R, tol=tol, precision="fp64", collision="RC",
                checked_every=check_every), dict(err, steps=steps, bar=1e-5,
                                                 meets_bar=max(err.values()) < 1e-5,
                                                 reference="the FP64 run of the same length")


def progress(msg):
    """A line on stderr as each stage of the benchmark ends."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def shear_fp32_50k(nu=4e-2, steps=50_000, every=5000):
    """FP32 deviation storage against FP64 on the 2048 x 8192 shear layer
    over its configured 50 000 steps, RC, at nu = 4e-2 (tau 1.5): the
    velocity difference (max |du| / max |u|) at every `every` steps.  The
    headline's nu = 6e-3 does not survive 50 000 steps in RC (FP64 blows up
    near 36 000), and at nu <= 2e-2 the roll-up of the layers amplifies
    perturbations of rounding size for a while (stability.py --study fp32)."""
    from paper_2103_02119_amd import lbm as L
    from paper_2103_02119_amd import stability as S

    r = S.shear_layer(nu=nu, steps=steps, check_every=every, compare_every=every,
                      collisions=(L.LBM_RC,))
    x = r["RC"]
    diffs = x["fp32_vs_fp64"]
    return dict(workload="shear 2048x8192 r=0.25 kappa=80 delta=0.05 u0=0.04 doubly periodic",
                nu=nu, tau=r["tau"], cs2=r["cs2"], steps=steps, collision="RC",
                blowup_step_fp64=x["blowup_step_fp64"], blowup_step_fp32=x["blowup_step_fp32"],
                compared_every=every, max_error=x["max_fp32_vs_fp64"],
                final_error=diffs[-1][1] if diffs else None, bar=1e-5,
                meets_bar=(x["max_fp32_vs_fp64"] is not None and len(diffs) == steps // every
                           and x["max_fp32_vs_fp64"] < 1e-5),
                reference="the FP64 run of the same length", seconds=x["seconds"])


def warm_start_section(n_cases=64, max_steps=400_000):
    """The learned warm start on unseen 256 x 128 cavities with obstacles
    (seeded Re in [100, 5000], a in {0.25, 0.5, 1}): steps and wall time to
    a per-step residual of 1e-8 in FP64 from rest (cold), from rest with the
    smoothing step (cold+smooth) and from the network's prediction with the
    smoothing step (warm+smooth), with the committed trained weights."""
    from paper_2103_02119_amd import warmstart as WS

    if not os.path.exists(WS.WEIGHTS):
        return dict(warm_steps=None, reason=f"no trained weights at {WS.WEIGHTS}")
    cmp = WS.evaluate(WS.WEIGHTS, n_test=n_cases, max_steps=max_steps,
                      modes=("cold", "cold+smooth", "warm+smooth"), log=progress)
    ws, cs, cold = cmp["warm+smooth"], cmp["cold+smooth"], cmp["cold"]
    own = cmp["network_gain_warm+smooth_vs_cold+smooth"]
    return dict(workload=f"{n_cases} unseen 256x128 lid-driven cavities with obstacles, "
                         "Re 100..5000, a in 0.25/0.5/1, FP64, per-step residual 1e-8",
                weights=os.path.basename(WS.WEIGHTS),
                cold_reached=cold["reached"], cold_seconds=cold["seconds"],
                cold_smooth_reached=cs["reached"], cold_smooth_seconds=cs["seconds"],
                warm_reached=ws["reached"], warm_seconds=ws["seconds"],
                warm_steps=ws["vs_cold"]["steps_total"],
                cold_steps=ws["vs_cold"]["ref_steps_total"],
                compared_cases=ws["vs_cold"]["compared"],
                step_speedup_vs_cold=round(ws["vs_cold"]["step_speedup_total"], 3),
                wall_speedup_vs_cold=round(cold["seconds"] / ws["seconds"], 3),
                network_own_step_speedup=round(own["step_speedup_total"], 3),
                network_own_wall_speedup=round(own["wall_speedup"], 3),
                network_own_compared_cases=own["compared"],
                target_speedup=3.0,
                note="warm+smooth: the network's prediction set as equilibrium fields and one "
                     "smoothing step after 50 steps; the network's own gain is against "
                     "cold+smooth, the same start-up without the network")


def bench_sweep(args):
    """The 512-case batch (cavities and channels, nx 64..512, r in
    {0.25, 0.5, 1}, Re 100..5000, FP32 deviations) advanced together by the
    persistent batched kernel, autotuned, graph-replayed."""
    import torch

    from paper_2103_02119_amd import inputs as I
    from paper_2103_02119_amd import lbm as L
    from paper_2103_02119_amd import workloads as W

    prec = L.LBM_FP32_DEV if args.precision == "fp32dev" else L.LBM_FP64
    params = I.batch_sweep()
    cases = W.sweep_cases(params)
    nodes = sum(c.nx * c.ny for c in cases)
    stream = torch.cuda.Stream()
    b = L.Batch(cases, precision=prec, graph_steps=args.graph_steps, stream=stream.cuda_stream)
    rows, wgs = b.autotune(5)
    tile = b.uses_tile_kernel()
    spl = b.steps_per_launch()
    # one step moves 9 values in and out per node; a two-step launch moves
    # them once for two steps (the call's last one or two steps are single)
    bytes_per_lu = (72 if prec == L.LBM_FP32_DEV else 144) // spl
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
        "metric": METRIC,
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
            "algorithmic_bytes_per_launch": bytes_per_lu * nodes * spl,
            "kernel": (("lbm::batch_staged_kernel" if b.two_step_form() == L.LBM_FORM_STAGED
                        else "lbm::batch_tile2_kernel") if spl == 2 else
                       "lbm::batch_tile_kernel" if tile else "lbm::batch_step_kernel"),
            "steps_per_launch": spl,
            "bytes_per_lu": bytes_per_lu,
            "kernel_us": round(1e3 * kern_ms * spl, 3),
            "kernel_time_from": "HIP events around the timed call (graph replays of the "
                                "batched launches; with two steps per launch the call's "
                                "last one or two steps are single), per step x steps per launch",
        },
        "unstable_cases": int(np.isnan(R).sum()),
    }
    if args.steady_cap:
        # every case to the tolerance from the state after the timed steps;
        # run_to_steady counts steps from its own start.  --steady-smooth
        # first takes the smoothing step (one step, then the mean of the
        # states before and after it), which removes the staggered mode the
        # impulsive start leaves in the cavities
        t0 = time.perf_counter()
        if args.steady_smooth:
            b.smooth_step()
        got = np.full(len(cases), -2, np.int64)
        seconds = np.full(len(cases), np.nan)
        done = 1 if args.steady_smooth else 0
        while done < args.steady_cap and (got == -2).any():
            n = min(args.steady_cap - done, 20 * args.steady_every)
            g = b.run_to_steady(args.steady_tol, args.steady_every, n)
            now = time.perf_counter() - t0
            for c in range(len(cases)):
                if got[c] == -2 and g[c] != -2:
                    got[c] = g[c] + done if g[c] > 0 else g[c]
                    seconds[c] = now
            done += n
            print(f"sweep steady: {done} steps, {int((got > 0).sum())} converged, "
                  f"{int((got == -1).sum())} blew up, {now:.0f} s", file=sys.stderr, flush=True)
        ok = got > 0
        out["time_to_steady"] = {
            "tol": args.steady_tol, "cap": args.steady_cap, "checked_every": args.steady_every,
            "seconds": round(time.perf_counter() - t0, 3),
            "converged": int(ok.sum()), "blew_up": int((got == -1).sum()),
            "not_converged": int((got == -2).sum()),
            "median_steps_converged": int(np.median(got[ok])) if ok.any() else None,
            "steps_converged_quartiles": [int(v) for v in np.percentile(got[ok], [25, 50, 75])]
            if ok.any() else None,
            "counted_from": f"step {args.warmup + steps} (after the warm-up and timed steps)",
            "smoothing_step": (f"at step {args.warmup + steps}, counted as one step"
                               if args.steady_smooth else None),
        }
        if args.steady_out:
            with open(args.steady_out, "w") as fh:
                json.dump([dict(p, nodes=c.nx * c.ny, steps=int(got[i]),
                                seconds=None if np.isnan(seconds[i]) else round(seconds[i], 3))
                           for i, (p, c) in enumerate(zip(params, cases))], fh)
    b.close()
    print(json.dumps(out), flush=True)


def copy_probe_main(nbytes=1 << 30, reps=20):
    """Plain device copies of a known size by the library's copy kernel
    (counter calibration)."""
    import torch

    from paper_2103_02119_amd import lbm as L

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()
    L.lbm_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, 0, s.cuda_stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        L.lbm_stream_copy(b.data_ptr(), a.data_ptr(), nbytes, 0, s.cuda_stream)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes": nbytes, "read_plus_write_GBs": round(2 * nbytes / ms / 1e6, 1),
                      "ms": round(ms, 4), "dispatches": reps + 1}), flush=True)


SIZES = [(64, 32), (128, 256), (256, 512), (512, 1024), (1024, 1024), (1024, 2048),
         (2048, 2048), (2048, 4096)]


def bench_sizes():
    """Microseconds per step of lid-driven cavities (a = 0.5, cs2 0.16, tau
    0.625, FP32 deviations and FP64) for one step per launch and for two
    steps per launch in each form of the two-step kernel (the staged form
    in FP32 only); best of three runs of back-to-back launches, HIP events
    on the library's stream.  One JSON line."""
    import torch

    from paper_2103_02119_amd import inputs as I
    from paper_2103_02119_amd import lbm as L

    out = {"workload": "cavities, a=0.5, cs2=0.16, tau=0.625, from rest; us per step", "sizes": {}}
    for pname, prec in (("fp32dev", L.LBM_FP32_DEV), ("fp64", L.LBM_FP64)):
        for nx, ny in SIZES:
            steps = min(4000, max(200, int(4e9 / (nx * ny)) // 2 * 2))
            row = {}
            modes = [("one_step", 1, L.LBM_FORM_AUTO), ("two_step_register", 2, L.LBM_FORM_REGISTER)]
            if prec == L.LBM_FP32_DEV:
                modes.append(("two_step_staged", 2, L.LBM_FORM_STAGED))
            for name, spl, form in modes:
                lat = L.Lattice(nx, ny, 0.5, [1, 1, 1, 1, 1.6, 1.6, 1, 1, 1], bc_types=(1, 1, 1, 2),
                                u_wall=((0, 0), (0, 0), (0, 0), (0.05, 0)), cs2=0.16,
                                precision=prec)
                lat.set_fields(*I.cavity_rest(nx, ny))
                lat.set_two_step_form(form)
                lat.step(101)
                best = min(time_launches(lat, spl, steps // spl) for _ in range(3)) / spl
                row[name] = round(1e3 * best, 3)
                lat.close()
            lat = L.Lattice(nx, ny, 0.5, [1, 1, 1, 1, 1.6, 1.6, 1, 1, 1], bc_types=(1, 1, 1, 2),
                            u_wall=((0, 0), (0, 0), (0, 0), (0.05, 0)), cs2=0.16, precision=prec)
            row["automatic"] = {"steps_per_launch": lat.steps_per_launch(),
                                "form": "staged" if lat.two_step_form() == L.LBM_FORM_STAGED
                                else "register"}
            lat.close()
            out["sizes"][f"{pname} {nx}x{ny}"] = row
            print(f"sizes: {pname} {nx}x{ny} {row}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["sweep", "sizes"], default="shear",
                    help="sizes: one step against two steps per launch, and the two forms of the "
                         "two-step kernel, on cavities of 64 x 32 to 2048 x 4096 nodes")
    ap.add_argument("--precision", choices=["fp32dev", "fp64"], default="fp32dev")
    ap.add_argument("--steps-per-launch", type=int, choices=[0, 1, 2], default=0,
                    help="0 = the library's automatic choice")
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--chunk", type=int, default=100, help="steps per host call")
    ap.add_argument("--graph-steps", type=int, default=64, help="sweep: steps per captured graph")
    ap.add_argument("--steady-cap", type=int, default=0,
                    help="sweep: also run every case to --steady-tol, at most this many steps")
    ap.add_argument("--steady-tol", type=float, default=1e-6)
    ap.add_argument("--steady-every", type=int, default=1000)
    ap.add_argument("--steady-smooth", action="store_true",
                    help="sweep: take the smoothing step before running every case to steady state")
    ap.add_argument("--steady-out", default=None,
                    help="sweep: write every case's parameters and steps to steady state here")
    ap.add_argument("--minimal", action="store_true",
                    help="only the headline workload (no copy ceiling, FP64, RNR, cavity, "
                         "time to steady state or CPU baseline); for profiling runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-steady", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--copy-probe", action="store_true")
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
        copy_probe_main()
        return
    if args.workload == "sweep":
        bench_sweep(args)
        return
    if args.workload == "sizes":
        bench_sizes()
        return
    print(f"bench: workload {args.workload} {args.precision}, {args.steps} steps", file=sys.stderr,
          flush=True)
    full = not args.minimal
    vb = 4 if args.precision == "fp32dev" else 8
    w = WORKLOADS[args.workload]
    buf_bytes = L.lbm_required_bytes(w["nx"], w["ny"], L.LBM_FP32_DEV if vb == 4 else L.LBM_FP64)
    # one population buffer copied: the same bytes each way as one step moves
    copy = copy_ceiling(buf_bytes) if full else None
    copy_gbs = copy["GBs"] if copy else None
    main_r = run_workload(args.workload, args.precision, L.LBM_RC, args, args.steps_per_launch,
                          one_step=full)
    info = main_r["info"]
    tr = traffic_of(f"{args.workload}/{args.precision}/{main_r['steps_per_launch']}")
    out = {
        "metric": METRIC,
        "value": round(main_r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * main_r["wall"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if vb == 4 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload} {info['nx']}x{info['ny']} r={info['r']}"
                        + (f" Re={w['Re']:g} lid={w['U']}" if args.workload == "cavity" else "")
                        + (" kappa=80 delta=0.05 u0=0.04 doubly periodic" if args.workload == "shear"
                           else ""),
            "collision": "RC",
            "storage": "FP32 deviations f - w rho0" if vb == 4 else "FP64",
            "cs2": info["cs2"], "nu": info["nu"], "tau": round(info["tau"], 6),
            "population_buffers_bytes": 2 * buf_bytes,
            "steps_per_launch": main_r["steps_per_launch"],
            "checks_in_timed_region": main_r["checks"],
            "check_every": args.check_every,
            "check_read": "asynchronous, one interval later; the last before the clock stops",
            "steps_per_host_call": args.chunk,
        },
        "roofline": roofline_of(main_r, copy_gbs, tr),
        "target_mlups": round(TARGET_MLUPS[args.precision], 1),
        "mlups_vs_target": round(main_r["mlups"] / TARGET_MLUPS[args.precision], 4),
        "one_step_per_launch": one_step_line(main_r, copy_gbs),
        "final_residual": main_r["residual"],
        "mass": main_r["mass"],
        "nonfinite_at_step": main_r["nonfinite_at_step"],
        "copy_ceiling": copy,
    }
    progress(f"headline run done: {out['value']} MLUPS")
    if full:
        if args.precision == "fp32dev":
            r64 = run_workload(args.workload, "fp64", L.LBM_RC, args)
            progress(f"fp64 run done: {r64['mlups']:.1f} MLUPS")
            c64 = copy_gbs  # the copy ceiling does not depend on the value type
            out["fp64"] = dict(mlups=round(r64["mlups"], 1),
                               roofline=roofline_of(r64, c64, traffic_of(
                                   f"{args.workload}/fp64/{r64['steps_per_launch']}")),
                               one_step_per_launch=one_step_line(r64, c64),
                               target_mlups=round(TARGET_MLUPS["fp64"], 1),
                               mlups_vs_target=round(r64["mlups"] / TARGET_MLUPS["fp64"], 4))
        rn = run_workload(args.workload, args.precision, L.LBM_RNR, args, args.steps_per_launch,
                          one_step=False)
        out["rnr"] = dict(mlups=round(rn["mlups"], 1), kernel_us=round(1e3 * rn["kernel_ms"], 3),
                          steps_per_launch=rn["steps_per_launch"])
        progress("rnr run done")
        if args.workload != "cavity":
            cav = run_workload("cavity", args.precision, L.LBM_RC, args)
            d = dict(workload="cavity 512x1024 r=0.5 Re=1000 lid=0.05 (both buffers fit the "
                              "256 MB Infinity Cache: not an HBM roofline)",
                     mlups=round(cav["mlups"], 1), steps_per_launch=cav["steps_per_launch"],
                     kernel_us=round(1e3 * cav["kernel_ms"], 3),
                     one_step_kernel_us=round(1e3 * cav["one_step_ms"], 3))
            if "two_step_ms" in cav:
                d["two_step_kernel_us"] = round(1e3 * cav["two_step_ms"], 3)
            out["cavity_cache_resident"] = d
            progress("cavity run done")
        if not args.no_steady:
            out["time_to_steady"], out["fp32_steady_error"] = cavity_steady()
            progress("cavity to steady state done")
            out["fp32_shear_50k"] = shear_fp32_50k()
            progress(f"shear layer fp32 vs fp64 over 50000 steps done: "
                     f"max {out['fp32_shear_50k']['max_error']:.2e}")
            out["time_to_steady"]["warm_start"] = warm_start_section()
            progress("warm-start section done")
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(args.workload, L.LBM_RC, args.cpu_budget)
    out["kernel_sha"] = kernel_sha()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
