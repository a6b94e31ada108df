#!/usr/bin/env python3
"""Throughput of the one-loop temperature-flow right-hand side on one MI355X.

Workload (the quasi-particle configuration): square lattice t = 1, t' = 0, mu = 0, U = 3t,
N = 48 angular Fermi-surface patches, L = 128 loop grid, T from 1.0t towards 0.01t with
Dormand-Prince steps in ln T, synthetic Z table on the internal lines, single-precision
right-hand side, double-precision state / error estimate / stop test (stop at max|V| > 20t).

One benchmark step is one complete flow (every right-hand side, stage, error estimate and
stop test until the flow stops) with its inputs already on the device.  The metric counts
3 N^3 L^2 coupling-loop-point updates per right-hand side (the direct form's nominal work).

Prints one JSON line.  --gpus above 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp32_TFs": 157.3, "fp64_TFs": 78.6, "bf16_TFs": 2500.0}
METRIC = "coupling·loop-point updates/s per RHS (N³·L²·3); flows/hour, mixed vs FP64"


# Matrix-core peak of each single-precision phase-2a mode (TFLOP/s): split bf16 issues three
# bf16 products per product.
MFMA_PEAK = {"fp32": PEAK["fp32_TFs"], "bf16": PEAK["bf16_TFs"], "bf16x3": PEAK["bf16_TFs"] / 3.0}


def kernel_work(name, N, L, nP, nD, rsize, nRp=None, nRd=None, nsets=5, prec="fp32"):
    """Algorithmic work of one launch of each timed kernel group for one flow.

    stage_bins: phase 1 of every stage node of a Dormand-Prince step (nsets = 5 distinct
              nodes; the stage argument in the same launch is minor): nsets (nRp + nRd) L^2
              weight derivatives (orbit representatives), each counted as 6 flops (two
              differences, one division, the 1/(4 T L^2) scale and the bin accumulation) --
              the point quantities the kernel evaluates on the fly are not counted
    stage:    the stage argument alone, timed as a middle stage of a step (four earlier k
              slots): V read (f64), the newest slot's three channel parts and the three
              earlier slots' sums read, the newest slot's sum and three operand layouts
              written
    y:        (nP + 3 nD) N^3 multiply-adds on the matrix cores; bytes = representative
              bins read (plus the transposed particle-hole bins) + 3 operand slabs read + Y
              written; bound by whichever roof takes longer at its peak: the matrix cores of
              the mode `prec` (peak MFMA_PEAK[prec]) or HBM
    contract: 4 N^4 multiply-adds; bytes = Y read + operand read + k written
    """
    NN, N3 = N * N, N ** 3
    nRp = nP if nRp is None else nRp
    nRd = nD if nRd is None else nRd
    if name == "stage_bins":
        return {"bound": "alu", "flops": 6.0 * nsets * (nRp + nRd) * L * L}
    if name == "stage":
        return {"bound": "hbm", "bytes": N3 * (8 + (3 + 3) * rsize + (1 + 3) * rsize)}
    if name == "y":
        flops = 2.0 * (nP + 3 * nD) * N3
        nbytes = (nRp + 2 * nRd) * NN * rsize + 3 * N3 * rsize + (nP + 3 * nD) * NN * rsize
        mma = flops / (MFMA_PEAK[prec] * 1e12) > nbytes / (PEAK["hbm_GBs"] * 1e9)
        return {"bound": "mfma" if mma else "hbm", "flops": flops, "bytes": nbytes,
                "peak_TFs": MFMA_PEAK[prec]}
    if name == "contract":
        return {"bound": "hbm", "flops": 8.0 * N ** 4,
                "bytes": (nP + 3 * nD) * NN * rsize + 2 * N3 * rsize}
    return None


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c2.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2005_00827_amd", "csrc", "kernels.hip")


def measured_traffic(group):
    """HBM bytes per launch of a kernel group from the committed counter summary.

    The summary holds FETCH_SIZE + WRITE_SIZE per dispatch (scaled by the copy-kernel
    calibration) and the SHA-256 of the kernel source it was taken with; when the source
    has changed since, the figure no longer describes the kernel and None is returned.
    """
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for ln in fh:
            if ":" in ln and not ln.startswith((" ", "#", "$")):
                k, v = ln.split(":", 1)
                kv[k.strip()] = v.strip()
    with open(KERNEL_SOURCE, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    key = "bytes_per_launch_" + group
    if kv.get("kernel_source_sha256") != sha or key not in kv:
        return None
    return float(kv[key])


def batched_sweep(fm, inputs, torch, dev):
    """The 64-flow sweep (U in {1.0, ..., 4.5} x 8 start temperatures, N=48, L=128, no Z,
    ragged stops) in one batch: flows/hour in single precision and in the plain FP64 path,
    and the largest relative T_c difference between them."""
    w = inputs.workload("C4")
    U, T0 = w["U"], w["T0"]
    out = {}
    tc = {}
    for prec in ("fp32", "fp64"):
        f = fm.Flow(N=w["N"], L=w["L"], U=U[0], T0=max(T0), T_end=w["T_end"], integrator="rk45",
                    precision=prec, max_batch=len(U), device=dev)
        if prec == "fp32":
            f.run_batch(U, T0)          # first call picks the tile shape
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = f.run_batch(U, T0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        f.close()
        tc[prec] = [r["T_c"] for r in res]
        out["flows_per_hour_" + prec] = len(U) / dt * 3600.0
        out["seconds_" + prec] = dt
        out["rhs_" + prec] = int(sum(r["n_rhs"] for r in res))
        out["updates_per_s_" + prec] = out["rhs_" + prec] * 3.0 * w["N"] ** 3 * w["L"] ** 2 / dt
    d = [abs(a / b - 1.0) for a, b in zip(tc["fp32"], tc["fp64"]) if math.isfinite(a) and math.isfinite(b)]
    out["diverged"] = len(d)
    out["Tc_max_rel_diff"] = max(d) if d else None
    return out


def interaction_flow(fm, inputs, torch, dev):
    """The paper's own interaction flow at N=48, L=128 (no Z): the crossover curve U*(T) at
    16 temperatures log-spaced in [0.03, 0.3] from one batched launch of flows with bare
    U = 8 (U* = g*^2 U, so one flow per temperature gives U*(T)), in single and double
    precision, and T*(U) for U = 2, 3, 4 by bisection in ln T to 1e-4."""
    import numpy as np
    N, L, Ub = 48, 128, 8.0
    T = np.geomspace(0.03, 0.3, 16)
    out, ustar = {}, {}
    for prec in ("fp32", "fp64"):
        f = fm.Flow(N=N, L=L, U=Ub, T0=0.1, integrator="rk45", precision=prec,
                    flow="interaction", max_batch=len(T), device=dev)
        if prec == "fp32":
            f.run_batch([Ub] * len(T), T)   # first call picks the tile shape
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = f.run_batch([Ub] * len(T), T)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ustar[prec] = [r["U_star"] for r in res]
        out["seconds_" + prec] = dt
        out["flows_per_hour_" + prec] = len(T) / dt * 3600.0
        out["rhs_" + prec] = int(sum(r["n_rhs"] for r in res))
        out["updates_per_s_" + prec] = out["rhs_" + prec] * 3.0 * N ** 3 * L ** 2 / dt
        if prec == "fp32":
            t0 = time.perf_counter()
            ts, st = f.tstar([2.0, 3.0, 4.0], 0.005, 1.0, rtol=1e-4)
            torch.cuda.synchronize()
            out["tstar_seconds_fp32"] = time.perf_counter() - t0
            out["T_star_fp32"] = {str(u): (float(t) if s == 0 else None)
                                  for u, t, s in zip((2.0, 3.0, 4.0), ts, st)}
        f.close()
    out["T"] = [float(t) for t in T]
    out["U_star_fp64"] = [float(u) for u in ustar["fp64"]]
    d = [abs(a / b - 1.0) for a, b in zip(ustar["fp32"], ustar["fp64"])
         if math.isfinite(a) and math.isfinite(b)]
    out["U_star_max_rel_diff"] = max(d) if d else None
    return out


def large_batch(fm, inputs, torch, dev):
    """16 flows, U = 1 + 3i/15, N=128, L=512, synthetic Z per flow, T 1 -> 0.01: flows/hour for
    the bf16, split-bf16 and fp32 right-hand sides against the plain FP64 path, T_c agreement,
    the per-kernel timings (HIP events, eager replay) of the bf16 run, and for bf16 and fp32
    the roofline of each kernel group with all 16 flows running (10 back-to-back launches on
    the final state, HIP events on the library stream)."""
    import numpy as np
    w = inputs.workload("C5")
    N, L, U, T0 = w["N"], w["L"], w["U"], w["T0"]
    cfg = fm.make_config(N, L)
    _, _, _, nP, nD, _ = fm.geometry_query(cfg)
    nRp, nRd = fm.representative_counts(cfg)
    nf = len(U)
    tabs = [inputs.synthetic_z_table(N, u, 1.0, w["T_end"]) for u in U]
    zl = np.stack([t[0] for t in tabs])
    zt = np.stack([t[1] for t in tabs])
    out, tc = {}, {}
    for prec in ("bf16", "bf16x3", "fp32", "fp64"):
        f = fm.Flow(N=N, L=L, U=U[0], T0=1.0, T_end=w["T_end"], integrator="rk45", precision=prec,
                    z_lnT=zl[0], z_table=zt[0], max_batch=len(U), device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = f.run_batch(U, T0, z_lnT=zl, z_tables=zt)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if prec == "bf16":
            f.set_timing(True)
            f.run_batch(U, T0, z_lnT=zl, z_tables=zt)
            out["kernels_bf16"] = {k: {"launches": n, "avg_us": ms / n * 1e3}
                                   for k, (ms, n) in f.timings().items()}
            f.set_timing(False)
        if prec in ("bf16", "fp32"):
            roof = {}
            for name, gid in (("stage_bins", 0), ("y", 1), ("contract", 2), ("stage", 3)):
                us = f.kernel_time(gid, nf, 10) * 1e3
                wk = kernel_work(name, N, L, nP, nD, 4, nRp, nRd, prec=prec)
                r = {"avg_us": us}
                if wk["bound"] == "hbm":
                    r.update(bound="hbm", achieved_GBs=nf * wk["bytes"] / (us * 1e-6) / 1e9)
                    r["frac"] = r["achieved_GBs"] / PEAK["hbm_GBs"]
                elif wk["bound"] == "mfma":
                    r.update(bound="mfma", achieved_TFs=nf * wk["flops"] / (us * 1e-6) / 1e12,
                             hbm_GBs=nf * wk["bytes"] / (us * 1e-6) / 1e9)
                    r["frac"] = r["achieved_TFs"] / wk["peak_TFs"]
                else:
                    r.update(bound="alu", pair_evals_per_s=nf * wk["flops"] / 6.0 / 2.0 / (us * 1e-6))
                roof[name] = r
            out["roofline_16_flows_" + prec] = roof
        f.close()
        rhs = int(sum(r["n_rhs"] for r in res))
        tc[prec] = [r["T_c"] for r in res]
        out["flows_per_hour_" + prec] = len(U) / dt * 3600.0
        out["seconds_" + prec] = dt
        out["rhs_" + prec] = rhs
        out["updates_per_s_" + prec] = rhs * 3.0 * N ** 3 * L ** 2 / dt
    for prec in ("bf16", "bf16x3", "fp32"):
        d = [abs(a / b - 1.0) for a, b in zip(tc[prec], tc["fp64"])
             if math.isfinite(a) and math.isfinite(b)]
        out["Tc_max_rel_diff_" + prec] = max(d) if d else None
    out["note"] = ("first call of each single-precision mode includes the phase-2a tile tuning; "
                   "bf16 runs at its default rtol 1e-4, the others at 1e-6")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the batched U x T0 sweep (64 flows) in the extra section")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the large batch (16 flows, N=128, L=512) in the extra section")
    ap.add_argument("--no-gflow", action="store_true", help="skip the interaction-flow runs")
    ap.add_argument("--large-only", action="store_true",
                    help="only the 16-flow N=128, L=512 batch (for profiling); prints its record")
    ap.add_argument("--cpu-rhs", type=int, default=6, help="oracle RHS evaluations timed")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain device-to-device copy of this many MiB three times "
                         "(calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path; independent flows "
              "and the per-transfer work would be the units to shard over GPUs.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2005_00827_amd import fm, inputs

    if args.large_only:
        print(json.dumps({"large_16_flows": large_batch(fm, inputs, torch, torch.device("cuda:0"))}))
        return
    w = inputs.workload("C2")
    N, L, U, T0, Te = w["N"], w["L"], w["U"][0], w["T0"][0], w["T_end"]
    zl, zt = inputs.synthetic_z_table(N, U, T0, Te)
    dev = torch.device("cuda:0")
    print("bench: C2 N=%d L=%d U=%g fp32 rhs, rk45, Z table; steps=%d warmup=%d"
          % (N, L, U, args.steps, args.warmup), file=sys.stderr, flush=True)

    def make(prec):
        return fm.Flow(N=N, L=L, U=U, T0=T0, T_end=Te, integrator="rk45", precision=prec,
                       z_lnT=zl, z_table=zt, max_batch=1, device=dev)

    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    flow = make("fp32")
    for _ in range(args.warmup):
        flow.run_batch([U], [T0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [flow.run_batch([U], [T0])[0] for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_rhs = sum(r["n_rhs"] for r in res)
    upd = 3.0 * N ** 3 * L ** 2
    value = n_rhs * upd / wall
    print("bench: timed %d flows in %.3f s, %d rhs, T_c %.6f" % (args.steps, wall, n_rhs, res[0]["T_c"]),
          file=sys.stderr, flush=True)

    # Kernel durations: HIP events on the library's stream around every launch group, over the
    # same flows replayed eagerly (same kernels, same inputs) -- these include host launch
    # gaps; the roofline uses the replay measurement below.
    flow.set_timing(True)
    for _ in range(args.steps):
        flow.run_batch([U], [T0])
    tm = flow.timings()
    flow.set_timing(False)
    cfg = fm.make_config(N, L)
    _, _, _, nP, nD, _ = fm.geometry_query(cfg)
    nRp, nRd = fm.representative_counts(cfg)
    kernels = {}
    for name, (ms, n) in tm.items():
        avg_s = ms / n * 1e-3
        k = {"launches": n, "total_ms": ms, "avg_us": avg_s * 1e6}
        wk = kernel_work(name, N, L, nP, nD, 4, nRp, nRd)
        if wk:
            if wk["bound"] == "hbm":
                k.update(bound="hbm", achieved=wk["bytes"] / avg_s / 1e9, peak=PEAK["hbm_GBs"],
                         unit="GB/s")
            else:
                k.update(bound=wk["bound"], achieved=wk["flops"] / avg_s / 1e12,
                         peak=wk.get("peak_TFs", PEAK["fp32_TFs"]), unit="TFLOP/s")
            k["frac"] = k["achieved"] / k["peak"]
        kernels[name] = k
    # Per-launch durations of the three RHS kernel groups: each launched 200 times back to
    # back on the flow's final state between two HIP events on the library's stream (the
    # serialized-launch cost is included, host gaps are not).
    groups = {"stage_bins": 0, "y": 1, "contract": 2, "stage": 3}
    replay = {name: flow.kernel_time(gid, 1, 200) * 1e3 for name, gid in groups.items()}
    for name, us in replay.items():
        k = kernels.setdefault(name, {})
        k["replay_avg_us"] = us
        wk = kernel_work(name, N, L, nP, nD, 4, nRp, nRd)
        if wk and wk["bound"] == "hbm":
            k["replay_achieved_GBs"] = wk["bytes"] / (us * 1e-6) / 1e9
        elif wk:
            k["replay_achieved_TFs"] = wk["flops"] / (us * 1e-6) / 1e12
    # dominant: the largest share of a flow's time (per-launch duration x launches per flow)
    dom = max(groups, key=lambda n: replay[n] * kernels[n].get("launches", 0))
    wk = kernel_work(dom, N, L, nP, nD, 4, nRp, nRd)
    avg_s = replay[dom] * 1e-6
    if wk["bound"] == "hbm":
        ach, peak, unit = wk["bytes"] / avg_s / 1e9, PEAK["hbm_GBs"], "GB/s"
    else:
        ach, peak, unit = wk["flops"] / avg_s / 1e12, wk.get("peak_TFs", PEAK["fp32_TFs"]), "TFLOP/s"
    roofline = {"kernel": dom, "bound": wk["bound"], "achieved": ach, "peak": peak, "unit": unit,
                "frac": ach / peak, "traffic": measured_traffic(dom), "avg_us": replay[dom],
                "launches_per_flow": kernels[dom].get("launches", 0) / args.steps,
                "timing": "200 back-to-back launches on the flow's final state, HIP events on "
                          "the library stream"}

    extra = {"flows": args.steps, "rhs_per_flow": n_rhs / args.steps,
             "T_c_fp32": res[0]["T_c"], "flows_per_hour_fp32": args.steps / wall * 3600.0,
             "kernels": kernels}
    if not args.no_fp64:
        f64 = make("fp64")
        f64.run_batch([U], [T0])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r64 = f64.run_batch([U], [T0])[0]
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t1
        extra.update(T_c_fp64=r64["T_c"], flows_per_hour_fp64=3600.0 / w64,
                     Tc_rel_diff=abs(res[0]["T_c"] / r64["T_c"] - 1.0),
                     updates_per_s_fp64=r64["n_rhs"] * upd / w64)
        f64.close()

    if not args.no_sweep:
        extra["sweep_64_flows"] = batched_sweep(fm, inputs, torch, dev)
    if not args.no_gflow:
        extra["interaction_flow"] = interaction_flow(fm, inputs, torch, dev)
    if not args.no_large:
        extra["large_16_flows"] = large_batch(fm, inputs, torch, dev)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O   # the checker, timed as the CPU baseline only
        m = O.model(N, L)
        V = inputs.noisy_state(N, U)
        Z = np.array([np.interp(math.log(0.2), zl, zt[:, a]) for a in range(N)])
        O.rhs(O.model(16, 32), 0.2, inputs.noisy_state(16, U))   # load + warm
        tc = time.perf_counter()
        for _ in range(args.cpu_rhs):
            O.rhs(m, 0.2, V, Z=Z)
        tcpu = time.perf_counter() - tc
        cpu = {"value": args.cpu_rhs * upd / tcpu, "unit": "coupling·loop-point updates/s",
               "cores": O.n_threads(), "kind": "oracle",
               "sample": "%d direct-form RHS evaluations of the same workload (N=48, L=128, "
                         "Z on, T=0.2) in %.1f s" % (args.cpu_rhs, tcpu)}

    line = {"metric": METRIC, "value": value, "unit": "coupling·loop-point updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "C2 quasi-particle flow: N=48 patches, L=128 loop grid, "
                                   "U=3t, t'=0, mu=0, T 1.0t->0.01t, Dormand-Prince in ln T, "
                                   "synthetic Z table, f32 RHS, f64 state, stop at max|V|>20t",
                       "N": N, "L": L, "U": U, "flows_per_step": 1},
            "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(line))
    flow.close()


if __name__ == "__main__":
    main()
