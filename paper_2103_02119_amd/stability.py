"""Stability margins of RC-LBM and RNR-LBM (Sec. 6), run with the batched
solver so that every (parameter, grid, collision) combination of a bisection
round advances in the same launches.

  max_lid_velocity  the largest lid speed U of a lid-driven cavity that stays
                    finite for a given number of steps, against tau
                    (the paper's Fig. 17 study: 21 x 21, 21 x 41, 21 x 61
                    nodes at a = 1, 0.5, 0.3, 100 000 steps);
  max_reynolds      the largest Re = U nx / nu that stays finite at a = 0.5,
                    U = 0.2, cs2 = 0.1 (the paper's Table 6 study);
  shear_layer       the doubly periodic shear layer: the step at which each
                    collision model blows up, and the FP32-deviation run's
                    velocity difference from the FP64 run until then;
  perturbation_growth  the FP64 shear layer's response to a population
                    perturbation of FP32 rounding's size made at a given step.

A case is unstable when a residual check (every `check_every` steps and at
the end) meets a non-finite velocity.
"""
from __future__ import annotations

import time

import numpy as np

from . import lbm as L
from . import workloads as Wk

PAPER_GRIDS = ((21, 21, 1.0), (21, 41, 0.5), (21, 61, 0.3))
TABLE6_GRIDS = ((100, 200), (200, 400), (300, 600))


def _lid_case(nx, ny, a, tau, U, cs2):
    rates = [1.0, 1.0, 1.0, 1.0, 1.0 / tau, 1.0 / tau, 1.0, 1.0, 1.0]
    return L.make_case(nx, ny, a, rates,
                       bc_types=(L.LBM_BC_WALL, L.LBM_BC_WALL, L.LBM_BC_WALL, L.LBM_BC_MOVING_WALL),
                       u_wall=((0, 0), (0, 0), (0, 0), (U, 0)), cs2=cs2)


def _survives(cases, collision, steps, check_every, precision):
    """True per case if no residual check met a non-finite velocity."""
    b = L.Batch(cases, collision=collision, precision=precision)
    out = b.run_to_steady(1e-300, check_every, steps)
    b.close()
    return out != -1


def max_lid_velocity(taus, grids=PAPER_GRIDS, collisions=(L.LBM_RC, L.LBM_RNR), steps=100_000,
                     rounds=10, u_max=0.6, check_every=1000, precision=L.LBM_FP64, cs2_rule=None,
                     log=None):
    """Bisection on U in (0, u_max] for every (tau, grid, collision).
    Returns a list of dicts with the stable / unstable bracket."""
    cs2_rule = cs2_rule or Wk.cavity_cs2
    combos = [(tau, g, coll) for coll in collisions for g in grids for tau in taus]
    lo = np.zeros(len(combos))
    hi = np.full(len(combos), u_max)
    hi_unstable = np.zeros(len(combos), bool)  # has hi been seen to blow up?
    t0 = time.perf_counter()
    for r in range(rounds):
        trial = np.where(hi_unstable, 0.5 * (lo + hi), hi) if r == 0 else 0.5 * (lo + hi)
        ok = np.zeros(len(combos), bool)
        for coll in collisions:
            idx = [i for i, c in enumerate(combos) if c[2] == coll]
            cases = [_lid_case(g[0], g[1], g[2], tau, float(trial[i]), cs2_rule(g[2]))
                     for i in idx for (tau, g, _) in [combos[i]]]
            ok[idx] = _survives(cases, coll, steps, check_every, precision)
        if r == 0:
            # the first round tries u_max itself
            hi_unstable = ~ok
            lo = np.where(ok, trial, lo)
        else:
            lo = np.where(ok, trial, lo)
            hi = np.where(ok, hi, trial)
            hi_unstable |= ~ok
        if log:
            log(f"max_lid_velocity: round {r + 1}/{rounds}, {time.perf_counter() - t0:.1f} s")
    return [dict(tau=tau, nx=g[0], ny=g[1], a=g[2], collision="RC" if coll == L.LBM_RC else "RNR",
                 stable_U=float(lo[i]), unstable_U=float(hi[i]) if hi_unstable[i] else None)
            for i, (tau, g, coll) in enumerate(combos)]


def max_reynolds(grids=TABLE6_GRIDS, a=0.5, U=0.2, cs2=0.1, collisions=(L.LBM_RC, L.LBM_RNR),
                 steps=100_000, rounds=12, re_lo=500.0, re_hi=60_000.0, check_every=1000,
                 precision=L.LBM_FP64, log=None):
    """Bisection on log Re for every (grid, collision); Re = U nx / nu."""
    combos = [(g, coll) for coll in collisions for g in grids]
    lo = np.full(len(combos), np.log(re_lo))
    hi = np.full(len(combos), np.log(re_hi))
    t0 = time.perf_counter()
    for r in range(rounds):
        trial = 0.5 * (lo + hi)
        ok = np.zeros(len(combos), bool)
        for coll in collisions:
            idx = [i for i, c in enumerate(combos) if c[1] == coll]
            cases = []
            for i in idx:
                (nx, ny), _ = combos[i]
                nu = U * nx / np.exp(trial[i])
                cases.append(_lid_case(nx, ny, a, nu / cs2 + 0.5, U, cs2))
            ok[idx] = _survives(cases, coll, steps, check_every, precision)
        lo = np.where(ok, trial, lo)
        hi = np.where(ok, hi, trial)
        if log:
            log(f"max_reynolds: round {r + 1}/{rounds}, {time.perf_counter() - t0:.1f} s")
    return [dict(nx=g[0], ny=g[1], a=a, collision="RC" if coll == L.LBM_RC else "RNR",
                 stable_Re=float(np.exp(lo[i])), unstable_Re=float(np.exp(hi[i])),
                 tau_at_stable=float(U * g[0] / np.exp(lo[i]) / cs2 + 0.5))
            for i, (g, coll) in enumerate(combos)]


def shear_layer(nx=2048, ny=8192, a=0.25, nu=1e-4, u0=0.04, kappa=80.0, delta=0.05, cs2=0.04,
                steps=50_000, check_every=500, compare_every=5000,
                collisions=(L.LBM_RC, L.LBM_RNR), log=None):
    """FP64 and FP32 deviations, per collision model, on the doubly periodic
    shear layer: blow-up step (None if it survives `steps`) and the
    FP32-vs-FP64 velocity difference (max-norm relative to max |u| of the
    FP64 run) at every `compare_every` steps while both are finite."""
    import torch

    from . import inputs as I

    rho0, ux0, uy0 = I.shear_layer(nx, ny, a, u0=u0, kappa=kappa, delta=delta)
    tau = nu / cs2 + 0.5
    rates = [1.0, 1.0, 1.0, 1.0, 1.0 / tau, 1.0 / tau, 1.0, 1.0, 1.0]
    out = {}
    for coll in collisions:
        name = "RC" if coll == L.LBM_RC else "RNR"
        lats = {p: L.Lattice(nx, ny, a, rates, cs2=cs2, collision=coll, precision=p)
                for p in (L.LBM_FP64, L.LBM_FP32_DEV)}
        for lat in lats.values():
            lat.set_fields(rho0, ux0, uy0)
        blow = {p: None for p in lats}
        diffs = []
        done = 0
        t0 = time.perf_counter()
        while done < steps:
            for p, lat in lats.items():
                if blow[p] is None:
                    lat.step(check_every)
            done += check_every
            for p, lat in lats.items():
                if blow[p] is None:
                    try:
                        lat.sums()
                    except L.LbmError as e:
                        if e.code != L.LBM_E_UNSTABLE:
                            raise
                        blow[p] = done
            if done % compare_every == 0 and all(v is None for v in blow.values()):
                _, a64, b64 = lats[L.LBM_FP64].moments()
                _, a32, b32 = lats[L.LBM_FP32_DEV].moments()
                scale = np.hypot(a64, b64).max()
                diffs.append((done, float(np.hypot(a32 - a64, b32 - b64).max() / scale)))
            if all(v is not None for v in blow.values()):
                break
        torch.cuda.synchronize()
        for lat in lats.values():
            lat.close()
        out[name] = dict(blowup_step_fp64=blow[L.LBM_FP64], blowup_step_fp32=blow[L.LBM_FP32_DEV],
                         fp32_vs_fp64=diffs,
                         max_fp32_vs_fp64=max((d for _, d in diffs), default=None),
                         seconds=round(time.perf_counter() - t0, 1))
        if log:
            log(f"shear_layer {name}: {out[name]}")
    return dict(nx=nx, ny=ny, a=a, nu=nu, tau=tau, cs2=cs2, steps=steps, check_every=check_every,
                **out)


def perturbation_growth(nx=2048, ny=8192, a=0.25, nu=1.2e-2, u0=0.04, kappa=80.0, delta=0.05,
                        cs2=0.04, kick_at=36_000, until=40_000, every=1000, amp=1e-7,
                        collision=L.LBM_RC, log=None):
    """How the FP64 scheme itself treats a perturbation of FP32 rounding's
    size: two FP64 runs of the shear layer, one of them with every
    population multiplied by 1 + amp xi (xi ~ U(-1, 1), seeded) at step
    `kick_at`; their velocity difference (max-norm relative to max |u|)
    every `every` steps up to `until`."""
    from . import inputs as I

    rho0, ux0, uy0 = I.shear_layer(nx, ny, a, u0=u0, kappa=kappa, delta=delta)
    tau = nu / cs2 + 0.5
    rates = [1.0, 1.0, 1.0, 1.0, 1.0 / tau, 1.0 / tau, 1.0, 1.0, 1.0]
    ref, kicked = (L.Lattice(nx, ny, a, rates, cs2=cs2, collision=collision, precision=L.LBM_FP64)
                   for _ in range(2))
    for lat in (ref, kicked):
        lat.set_fields(rho0, ux0, uy0)
        lat.step(kick_at)
    f = kicked.get_populations()
    f *= I.relative_noise(6, nx, ny, amp=amp)
    kicked.set_populations(f)
    del f
    diffs = []
    for done in range(kick_at + every, until + 1, every):
        for lat in (ref, kicked):
            lat.step(every)
        _, a0, b0 = ref.moments()
        _, a1, b1 = kicked.moments()
        diffs.append((done, float(np.hypot(a1 - a0, b1 - b0).max() / np.hypot(a0, b0).max())))
        if log:
            log(f"perturbation growth nu={nu:g}: step {done}: {diffs[-1][1]:.3e}")
    ref.close()
    kicked.close()
    return dict(nx=nx, ny=ny, a=a, nu=nu, tau=tau, cs2=cs2, amp=amp, kick_at=kick_at,
                collision="RC" if collision == L.LBM_RC else "RNR", difference=diffs)


def shear_layer_sweep(nus=(1e-4, 2e-4, 4e-4, 8e-4, 1.6e-3), steps=20_000, check_every=100,
                      log=None, **kw):
    """Blow-up steps of both collision models and both storage precisions on
    the shear layer over a range of viscosities (tau = nu / cs2 + 1/2)."""
    out = []
    for nu in nus:
        r = shear_layer(nu=nu, steps=steps, check_every=check_every,
                        compare_every=max(check_every, steps // 4), log=log, **kw)
        out.append(dict(nu=nu, tau=r["tau"],
                        **{f"{c}_{p}": r[c][f"blowup_step_{p}"] for c in ("RC", "RNR")
                           for p in ("fp64", "fp32")}))
    return out


def _shear_survives(nx, ny, a, nu, cs2, coll, precision, steps, check_every, fields):
    tau = nu / cs2 + 0.5
    rates = [1.0, 1.0, 1.0, 1.0, 1.0 / tau, 1.0 / tau, 1.0, 1.0, 1.0]
    lat = L.Lattice(nx, ny, a, rates, cs2=cs2, collision=coll, precision=precision)
    lat.set_fields(*fields)
    ok = True
    for _ in range(steps // check_every):
        lat.step(check_every)
        try:
            lat.sums()
        except L.LbmError as e:
            if e.code != L.LBM_E_UNSTABLE:
                raise
            ok = False
            break
    lat.close()
    return ok


def shear_layer_margin(nx=2048, ny=8192, a=0.25, cs2=0.04, u0=0.04, kappa=80.0, delta=0.05,
                       nu_lo=1e-4, nu_hi=2e-2, rounds=6, steps=20_000, check_every=1000,
                       precision=L.LBM_FP64, log=None):
    """Smallest viscosity at which the shear layer stays finite for `steps`
    steps, per collision model: bisection on log nu (the stable end of the
    final bracket is reported)."""
    from . import inputs as I

    fields = I.shear_layer(nx, ny, a, u0=u0, kappa=kappa, delta=delta)
    out = {}
    for coll in (L.LBM_RC, L.LBM_RNR):
        name = "RC" if coll == L.LBM_RC else "RNR"
        lo, hi = np.log(nu_lo), np.log(nu_hi)
        for r in range(rounds):
            mid = 0.5 * (lo + hi)
            if _shear_survives(nx, ny, a, float(np.exp(mid)), cs2, coll, precision, steps,
                               check_every, fields):
                hi = mid
            else:
                lo = mid
            if log:
                log(f"shear margin {name}: round {r + 1}/{rounds}, bracket "
                    f"[{np.exp(lo):.3g}, {np.exp(hi):.3g}]")
        out[name] = dict(min_stable_nu=float(np.exp(hi)), max_unstable_nu=float(np.exp(lo)),
                         tau_at_min_stable=float(np.exp(hi) / cs2 + 0.5))
    return dict(nx=nx, ny=ny, a=a, cs2=cs2, steps=steps, precision=precision, **out)


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description="stability margins of RC-LBM and RNR-LBM")
    ap.add_argument("--study", choices=["lid", "reynolds", "shear", "margin", "fp32", "all"],
                    default="all")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    log = lambda s: print(s, flush=True)  # noqa: E731
    res = {}
    if args.study in ("lid", "all"):
        taus = (0.505, 0.51, 0.52, 0.55, 0.6, 0.7, 0.8, 1.0, 1.5)
        res["max_lid_velocity"] = max_lid_velocity(taus, log=log)
    if args.study in ("reynolds", "all"):
        res["max_reynolds"] = max_reynolds(log=log)
    if args.study in ("shear", "all"):
        # the configured viscosity, with the blow-up step resolved to 50 steps
        res["shear_layer"] = shear_layer(steps=5000, check_every=50, compare_every=100, log=log)
        res["shear_layer_margin"] = shear_layer_margin(log=log)
        # above both models' limits: FP32 storage against FP64 over 50 000 steps
        res["shear_layer_fp32"] = shear_layer(nu=6e-3, steps=50_000, check_every=1000,
                                              compare_every=5000, log=log)
    if args.study == "margin":
        # the shear layer's viscosity margin over its full 50 000 steps, both precisions
        res["shear_layer_margin_50k"] = [
            shear_layer_margin(nu_lo=1e-3, nu_hi=2e-2, rounds=5, steps=50_000, precision=p, log=log)
            for p in (L.LBM_FP64, L.LBM_FP32_DEV)]
    if args.study == "fp32":
        # FP32 storage against FP64 over the configured 50 000 steps at stable viscosities,
        # and what the FP64 scheme makes of a 1e-7 perturbation during the roll-up
        res["shear_layer_fp32_50k"] = [
            shear_layer(nu=nu, steps=50_000, check_every=2500, compare_every=2500, log=log)
            for nu in (1.2e-2, 2e-2, 4e-2)]
        res["perturbation_growth"] = [perturbation_growth(nu=nu, log=log)
                                      for nu in (1.2e-2, 4e-2)]
    text = json.dumps(res)
    print(text, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
