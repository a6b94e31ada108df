#!/usr/bin/env python3
"""Throughput of the one-loop temperature-flow right-hand side on one MI355X.

Workload (the large batch): 16 flows with U_i = 1 + 3i/15, square lattice t = 1, t' = 0,
mu = 0, N = 128 angular Fermi-surface patches, L = 512 loop grid, T from 1.0t towards 0.01t
with Dormand-Prince steps in ln T, a synthetic Z table per flow on the internal lines,
single-precision loop sums with the grouped contractions on bf16 matrix cores, double-
precision state / error estimate / stop test (stop at max|V| > 20t).

One benchmark step is the whole 16-flow batch (every right-hand side, stage, error estimate
and stop test until every flow has stopped) with its inputs already on the device.  The
metric counts 3 N^3 L^2 coupling-loop-point updates per right-hand side of each flow (the
direct form's nominal work).  The flows start from V = U and their Z tables depend on the
patch through cos 4 theta only, so every state is invariant under the lattice's point group
and the headline runs the symmetric-state mode (sym_state = 1: phase 2 from the orbit
representatives' products, the same right-hand side); --sym 0 runs the full mode, which the
extra figures also report.

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

PEAK = {"hbm_GBs": 8000.0, "fp32_TFs": 157.3, "fp64_TFs": 78.6, "bf16_TFs": 2500.0,
        # plain (non-packed) vector issue: 256 CUs x 64 lanes x 2.4 GHz; packed FP32 is
        # disabled in these kernels, so a lane-op is one VALU instruction on one lane and an
        # FP32 FMA is 2 flops of a 78.6 TFLOP/s rate
        "valu_TOPs": 256 * 64 * 2.4e9 / 1e12, "fp32_fma_TFs": 256 * 64 * 2 * 2.4e9 / 1e12}
METRIC = "coupling·loop-point updates/s per RHS (N³·L²·3); flows/hour, mixed vs FP64"

# Matrix-core peak of each single-precision phase-2a mode (TFLOP/s): split bf16 issues three
# bf16 products per product.
MFMA_PEAK = {"fp32": PEAK["fp32_TFs"], "bf16": PEAK["bf16_TFs"], "bf16x3": PEAK["bf16_TFs"] / 3.0}

# Lane-ops priced per bubble-weight evaluation in phase 1 (two exponentials, one reciprocal,
# about 25 FMA-class operations and the bin update)
OPS_PER_WEIGHT = 40.0


def bin_density(fm, N, L, stride=16):
    """Fraction of the N x N patch pairs (a', b') that a transfer's bin actually holds (a loop
    point of patch a' whose partner lies in patch b'), averaged over every stride-th distinct
    transfer of each channel kind (the point group maps transfers onto each other with equal
    density).  Returns (rho_pp, rho_ph)."""
    import numpy as np
    cfg = fm.make_config(N, L)
    _, patch, anchor, npp, nph, _ = fm.geometry_query(cfg)
    ax, ay = anchor[:, 0].astype(np.int64), anchor[:, 1].astype(np.int64)
    qpp = np.unique(((ax[:, None] + ax[None, :]) % L) + L * ((ay[:, None] + ay[None, :]) % L))
    qph = np.unique(((ax[:, None] - ax[None, :]) % L) + L * ((ay[:, None] - ay[None, :]) % L))
    j = np.arange(L * L)
    jx, jy = j % L, j // L
    pj = patch.astype(np.int64)
    out = []
    for qs, pp in ((qpp, True), (qph, False)):
        nnz, sel = 0, qs[::stride]
        for q in sel:
            mx, my = q % L, q // L
            if pp:       # partner of k_j in q - k_j on the half-shifted grid
                px, py = (mx - jx - 1) % L, (my - jy - 1) % L
            else:        # partner k_j + q
                px, py = (mx + jx) % L, (my + jy) % L
            nnz += np.unique(pj * N + pj[px + L * py]).size
        out.append(nnz / (len(sel) * N * N))
    return out[0], out[1]


def kernel_work(name, N, L, nP, nD, rsize, nRp, nRd, rho, nsets=5, prec="fp32", nbin_flows=1,
                sym=0):
    """Algorithmic work of one launch of each timed kernel group for one flow (phase 1: for
    nbin_flows flows that bin, one per step-sharing group).

    stage_bins: phase 1 of every stage node of a Dormand-Prince step (nsets = 5 distinct
              nodes) for the orbit representatives, each unordered pair of a transfer's
              involution once: nsets (nRp + nRd) L^2 / 2 weight evaluations at OPS_PER_WEIGHT
              lane-ops each, against the plain vector issue rate (bound "alu")
    y:        the contraction over the bins, weighted by their density rho = (rho_pp, rho_ph):
              2 (nP rho_pp + 3 nD rho_ph) N^3 flops on the matrix cores of the mode (symmetric
              states: the representatives' products, nRp and nRd in place of nP and nD); bytes =
              representative bins (plus the transposed particle-hole bins) + 3 operand slabs
              (the products Y that this build stores between phase 2a and 2b are not the
              method's work and are not counted); bound by HBM or the matrix cores, whichever
              takes longer at its peak
    contract: 4 N^4 multiply-adds (8 N^4 flops) on the vector units (bound "alu" at the plain
              FP32 FMA rate)
    stage:    the stage argument alone, timed as a middle stage of a step (four earlier k
              slots): V read (f64), the newest slot's three channel parts and the three
              earlier slots' sums read, the newest slot's sum and three operand layouts
              written (bound "hbm")
    """
    NN, N3 = N * N, N ** 3
    opsz = 2 if prec == "bf16" else 4
    if name == "stage_bins":
        return {"bound": "alu", "ops": OPS_PER_WEIGHT * nsets * (nRp + nRd) * L * L / 2.0
                * nbin_flows, "peak": PEAK["valu_TOPs"], "unit": "TOP/s (lane-ops)"}
    if name == "stage":
        return {"bound": "hbm", "bytes": N3 * (8 + (3 + 3) * rsize + (1 + 3) * rsize),
                "peak": PEAK["hbm_GBs"], "unit": "GB/s"}
    if name == "y":
        mp, md = (nRp, nRd) if sym else (nP, nD)
        flops = 2.0 * (mp * rho[0] + 3 * md * rho[1]) * N3
        nbytes = (nRp + 2 * nRd) * NN * rsize + 3 * N3 * opsz
        # the binding roof: whichever takes longer at its peak for this work
        if nbytes / (PEAK["hbm_GBs"] * 1e9) > flops / (MFMA_PEAK[prec] * 1e12):
            return {"bound": "hbm", "flops": flops, "bytes": nbytes, "peak": PEAK["hbm_GBs"],
                    "unit": "GB/s"}
        return {"bound": "mfma", "flops": flops, "bytes": nbytes, "peak": MFMA_PEAK[prec],
                "unit": "TFLOP/s"}
    if name == "contract":
        return {"bound": "alu", "flops": 8.0 * N ** 4, "peak": PEAK["fp32_fma_TFs"],
                "unit": "TFLOP/s"}
    return None


def achieved(wk, avg_s, nflows):
    """Achieved rate of one launch in the unit of its roof (per-flow work x flows)."""
    if wk["bound"] == "hbm":
        return wk["bytes"] * nflows / avg_s / 1e9
    if "ops" in wk:
        return wk["ops"] / avg_s / 1e12          # phase 1: already counted for the binning flows
    return wk["flops"] * nflows / avg_s / 1e12


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c5_16flows.txt")
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


def c5_tables(inputs, w):
    import numpy as np
    tabs = [inputs.synthetic_z_table(w["N"], u, 1.0, w["T_end"]) for u in w["U"]]
    return np.stack([t[0] for t in tabs]), np.stack([t[1] for t in tabs])


def c5_flow(fm, w, zl, zt, dev, prec, rtol=0.0, sync=0, sym=0):
    return fm.Flow(N=w["N"], L=w["L"], U=w["U"][0], T0=1.0, T_end=w["T_end"], integrator="rk45",
                   precision=prec, rtol=rtol, z_lnT=zl[0], z_table=zt[0], max_batch=len(w["U"]),
                   sync_batch=sync, sym_state=sym, device=dev)


def timed_batch(f, torch, w, zl, zt):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = f.run_batch(w["U"], w["T0"], z_lnT=zl, z_tables=zt)
    torch.cuda.synchronize()
    return res, time.perf_counter() - t0


def tc_diff(res, ref):
    d = [abs(r["T_c"] / q - 1.0) for r, q in zip(res, ref)
         if math.isfinite(r["T_c"]) and math.isfinite(q)]
    return max(d) if d else None


def c5_other_modes(fm, inputs, torch, dev, w, zl, zt, ref_tc):
    """The 16-flow batch in the full and the symmetric-state mode, with every flow stepping on
    its own, in step-sharing groups of 2 and of all 16, and in the other precisions (each at
    its default rtol): flows/hour, RHS count, the largest T_c difference from the converged
    FP64 reference, and the phase-1 launch."""
    out = {}
    for key, prec, sync, sym in (("bf16_full_sync2", "bf16", 2, 0), ("bf16_sym_independent", "bf16", 0, 1),
                                 ("bf16_sym_sync2", "bf16", 2, 1), ("bf16_sym_sync16", "bf16", 1, 1),
                                 ("bf16x3_sym_sync2", "bf16x3", 2, 1), ("bf16x3_full_sync2", "bf16x3", 2, 0),
                                 ("fp32_sym_sync2", "fp32", 2, 1), ("fp32_full_sync2", "fp32", 2, 0),
                                 ("fp64_full", "fp64", 0, 0), ("fp64_sym", "fp64", 0, 1)):
        f = c5_flow(fm, w, zl, zt, dev, prec, sync=sync, sym=sym)
        if prec != "fp64":    # tuning and the batch's step graph, outside the timed run
            f.run_batch(w["U"], w["T0"], z_lnT=zl, z_tables=zt)
        res, dt = timed_batch(f, torch, w, zl, zt)
        r = {"seconds": dt, "flows_per_hour": len(w["U"]) / dt * 3600.0,
             "rhs": int(sum(x["n_rhs"] for x in res)), "Tc_max_rel_diff": tc_diff(res, ref_tc)}
        r["phase1_launch_us"] = f.kernel_time(0, len(w["U"]), 3) * 1e3
        f.close()
        out[key] = r
    return out


def c2_single_flow(fm, inputs, torch, dev, steps=5):
    """The quasi-particle workload of one flow (N=48, L=128, U=3, Z table, f32): updates/s and
    flows/hour in the full and the symmetric-state mode, and its T_c against the FP64 path."""
    w = inputs.workload("C2")
    N, L, U, Te = w["N"], w["L"], w["U"][0], w["T_end"]
    zl, zt = inputs.synthetic_z_table(N, U, 1.0, Te)
    out = {}
    tc = {}
    for prec, sym in (("fp32", 0), ("fp64", 0), ("fp32", 1)):
        f = fm.Flow(N=N, L=L, U=U, T0=1.0, T_end=Te, integrator="rk45", precision=prec,
                    z_lnT=zl, z_table=zt, sym_state=sym, device=dev)
        f.run_batch([U], [1.0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [f.run_batch([U], [1.0])[0] for _ in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        f.close()
        rhs = sum(r["n_rhs"] for r in res)
        key = prec + ("_sym" if sym else "")
        tc[key] = res[0]["T_c"]
        out["updates_per_s_" + key] = rhs * 3.0 * N ** 3 * L ** 2 / dt
        out["ms_per_flow_" + key] = dt / steps * 1e3
        out["rhs_per_flow_" + key] = rhs / steps
    out["Tc_rel_diff_fp32_fp64"] = abs(tc["fp32"] / tc["fp64"] - 1.0)
    out["Tc_rel_diff_fp32_sym_fp64"] = abs(tc["fp32_sym"] / tc["fp64"] - 1.0)
    return out


def shell_flow(fm, inputs, torch, dev):
    """Energy-shell patching at the paper's 224 patches (7 shells x 32 sectors), L=128, U=3,
    one FP32 flow (phase 2a on the vector units above 128 patches) and the FP64 flow of the
    same workload: seconds, RHS, updates/s and the T_c difference."""
    w = inputs.workload("shells")
    N, L, U = w["N"], w["L"], w["U"][0]
    out, tc = {}, {}
    for prec in ("fp32", "fp64"):
        f = fm.Flow(N=N, L=L, U=U, T0=1.0, T_end=w["T_end"], geometry="shells",
                    n_shells=w["n_shells"], integrator="rk45", precision=prec, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f.run_batch([U], [1.0])[0]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["rhs_ms_" + prec] = f.kernel_time(1, 1, 3) + f.kernel_time(2, 1, 3)
        f.close()
        tc[prec] = r["T_c"]
        out["seconds_" + prec] = dt
        out["rhs_" + prec] = r["n_rhs"]
        out["updates_per_s_" + prec] = r["n_rhs"] * 3.0 * N ** 3 * L ** 2 / dt
    out["T_c_fp64"] = tc["fp64"]
    out["Tc_rel_diff_fp32_fp64"] = abs(tc["fp32"] / tc["fp64"] - 1.0)
    out["note"] = "rhs_ms_*: phase 2a + phase 2b launch of one flow (first call includes tuning)"
    return out


def z_provider(fm, inputs, torch, dev):
    """The quasi-particle weights of second-order perturbation theory (fm_flow_z) at the
    quasi-particle workload's size (N=48, L=128, U=3): time per temperature node (the L^4 sum
    per patch), the range of Z, and the FP32 flow fed by the table on 17 ln T nodes from
    T = 0.025 to 1 against the same flow with the synthetic table."""
    import numpy as np
    w = inputs.workload("C2")
    N, L, U, Te = w["N"], w["L"], w["U"][0], w["T_end"]
    # nodes from T = 0.025, the lowest T whose slope window holds 8 frequency nodes; the
    # table is held at its lowest node below
    lnT = np.linspace(math.log(0.025), 0.0, 17)
    f = fm.Flow(N=N, L=L, U=U, T0=1.0, T_end=Te, integrator="rk45", precision="fp32",
                device=dev)
    f.z(0.3, U)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tab = np.stack([f.z(math.exp(s), U) for s in lnT])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / len(lnT)
    f.close()
    out = {"seconds_per_node": dt, "Z_min": float(tab.min()), "Z_max": float(tab.max()),
           "terms_per_node": N * float(L) ** 4}
    for name, (zl, zt) in (("second_order", (lnT, tab)),
                           ("synthetic", inputs.synthetic_z_table(N, U, 1.0, Te))):
        g = fm.Flow(N=N, L=L, U=U, T0=1.0, T_end=Te, integrator="rk45", precision="fp32",
                    z_lnT=zl, z_table=zt, device=dev)
        r = g.run_batch([U], [1.0])[0]
        g.close()
        out["T_c_" + name] = r["T_c"]
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="bf16", choices=("bf16", "bf16x3", "fp32"),
                    help="precision of the headline right-hand side")
    ap.add_argument("--sync", type=int, default=2,
                    help="step-sharing groups of at most this many flows (0: every flow steps "
                         "on its own)")
    ap.add_argument("--sym", type=int, default=1, choices=(0, 1),
                    help="1: symmetric-state mode (the batch's states are point-group "
                         "invariant); 0: full mode")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline batch (for profiling)")
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the converged FP64 run of the batch (for profiling)")
    ap.add_argument("--cpu-outputs", type=int, default=4096,
                    help="outputs of the 16-flow workload the oracle evaluates for the CPU baseline")
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

    dev = torch.device("cuda:0")
    w = inputs.workload("C5")
    N, L, nf = w["N"], w["L"], len(w["U"])
    zl, zt = c5_tables(inputs, w)
    print("bench: 16 flows N=%d L=%d U=1..4, Z per flow, %s rhs, rk45, sym_state %d; steps=%d "
          "warmup=%d" % (N, L, args.prec, args.sym, args.steps, args.warmup), file=sys.stderr,
          flush=True)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    flow = c5_flow(fm, w, zl, zt, dev, args.prec, sync=args.sync, sym=args.sym)
    for _ in range(args.warmup):          # the first call also times the phase-2a variants
        flow.run_batch(w["U"], w["T0"], z_lnT=zl, z_tables=zt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [flow.run_batch(w["U"], w["T0"], z_lnT=zl, z_tables=zt) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_rhs = sum(r["n_rhs"] for res in runs for r in res)
    upd = 3.0 * N ** 3 * L ** 2
    value = n_rhs * upd / wall
    print("bench: timed %d batches in %.3f s, %d rhs" % (args.steps, wall, n_rhs),
          file=sys.stderr, flush=True)

    # launches and time per batch of each kernel group (HIP events around each launch of one
    # eager batch, whose launches shrink as flows stop; the dominant group is the one with the
    # most time there), then each group's average launch duration: 10 back-to-back launches
    # with all 16 flows running on the batch's final state, between HIP events on the
    # library's stream
    flow.set_timing(True)
    flow.run_batch(w["U"], w["T0"], z_lnT=zl, z_tables=zt)
    tm = flow.timings()
    flow.set_timing(False)
    cfg = fm.make_config(N, L)
    _, _, _, nP, nD, _ = fm.geometry_query(cfg)
    nRp, nRd = fm.representative_counts(cfg)
    rho = bin_density(fm, N, L)
    groups = {"stage_bins": 0, "y": 1, "contract": 2, "stage": 3}
    kernels = {}
    for name, gid in groups.items():
        try:
            us = flow.kernel_time(gid, nf, 10) * 1e3
        except fm.FmError:           # phase 2 runs as one fused launch: no separate phase 2b
            continue
        # flows that bin in phase 1: one per step-sharing group
        nbin = nf if args.sync == 0 else (nf + (args.sync if args.sync > 1 else nf) - 1) // \
            (args.sync if args.sync > 1 else nf)
        wk = kernel_work(name, N, L, nP, nD, 4, nRp, nRd, rho, prec=args.prec, nbin_flows=nbin,
                         sym=args.sym)
        ach = achieved(wk, us * 1e-6, nf)
        batch_ms, launches = tm.get(name, (0.0, 0))
        kernels[name] = {"avg_us": us, "launches_per_batch": launches,
                         "share_ms_per_batch": batch_ms, "bound": wk["bound"],
                         "achieved": ach, "peak": wk["peak"], "unit": wk["unit"],
                         "frac": ach / wk["peak"]}
        if name == "y":
            kernels[name]["achieved_method_GBs"] = wk["bytes"] * nf / (us * 1e-6) / 1e9
    dom = max(kernels, key=lambda k: kernels[k]["share_ms_per_batch"])
    kd = kernels[dom]
    roofline = {"kernel": dom, "bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"],
                "unit": kd["unit"], "frac": kd["frac"], "traffic": measured_traffic(dom),
                "avg_us": kd["avg_us"], "launches_per_batch": kd["launches_per_batch"],
                "timing": "10 back-to-back launches with all 16 flows running, HIP events on "
                          "the library stream"}
    flow.close()

    # the converged FP64 reference of the same batch (rtol 1e-8) for the T_c agreement
    ref_tc, ref_dt = None, None
    if not args.no_reference:
        f64 = c5_flow(fm, w, zl, zt, dev, "fp64", rtol=1e-8)
        ref, ref_dt = timed_batch(f64, torch, w, zl, zt)
        f64.close()
        ref_tc = [r["T_c"] for r in ref]
    extra = {"batches": args.steps, "rhs_per_batch": n_rhs / args.steps,
             "flows_per_hour": args.steps * nf / wall * 3600.0,
             "Tc_max_rel_diff_vs_fp64": tc_diff(runs[0], ref_tc) if ref_tc else None,
             "fp64_reference": {"rtol": 1e-8, "seconds": ref_dt, "T_c": ref_tc},
             "T_c": [r["T_c"] for r in runs[0]], "status": [r["status"] for r in runs[0]],
             "bin_density": rho, "kernels": kernels}
    if not args.no_extra:
        if ref_tc:
            extra["c5_other_modes"] = c5_other_modes(fm, inputs, torch, dev, w, zl, zt, ref_tc)
        extra["c2_single_flow"] = c2_single_flow(fm, inputs, torch, dev)
        extra["sweep_64_flows"] = batched_sweep(fm, inputs, torch, dev)
        extra["interaction_flow"] = interaction_flow(fm, inputs, torch, dev)
        extra["shells_224"] = shell_flow(fm, inputs, torch, dev)
        extra["z_provider"] = z_provider(fm, inputs, torch, dev)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O   # the checker, timed as the CPU baseline only
        m = O.model(N, L)
        V = inputs.noisy_state(N, w["U"][8])
        T = 0.2
        Z = np.array([np.interp(math.log(T), zl[8], zt[8][:, a]) for a in range(N)])
        abc = inputs.sample_indices(N, args.cpu_outputs)
        O.rhs_points(m, T, V, abc[:2], Z=Z)                   # load + warm
        tc0 = time.perf_counter()
        O.rhs_points(m, T, V, abc, Z=Z)
        tcpu = time.perf_counter() - tc0
        cpu = {"value": args.cpu_outputs * 3.0 * L * L / tcpu,
               "unit": "coupling·loop-point updates/s", "cores": O.n_threads(), "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": "%d outputs (a,b,c) of one flow's direct-form RHS at N=128, L=512, "
                         "T=0.2, Z on, each 3 L^2 nominal updates, in %.1f s"
                         % (args.cpu_outputs, tcpu)}

    line = {"metric": METRIC, "value": value, "unit": "coupling·loop-point updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": {"bf16": "bf16 contraction, f32 loop sums, f64 state",
                      "bf16x3": "split-bf16 contraction, f32 loop sums, f64 state",
                      "fp32": "f32, f64 state"}[args.prec],
            "data": "synthetic",
            "config": {"workload": "16 flows, U_i = 1 + 3i/15, N=128 patches, L=512 loop grid, "
                                   "t'=0, mu=0, T 1.0t->0.01t, Dormand-Prince in ln T, synthetic "
                                   "Z table per flow, %s contraction, f64 state, stop at "
                                   "max|V|>20t; one step = the whole 16-flow batch; %s"
                                   % (args.prec, "symmetric-state mode (point-group invariant "
                                      "states: phase 2 from the orbit representatives' "
                                      "products)" if args.sym else "full mode"),
                       "N": N, "L": L, "flows_per_step": nf,
                       "step_sharing_groups": args.sync, "sym_state": args.sym},
            "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
