#!/usr/bin/env python3
"""Benchmark of the parabolic-operator advance on one MI355X.

One step = one pass of the whole hot path over the 151 x 301 x 400 spherical
shell (18.2 M cells): lagged-coefficient set-up, then for both split
operators -- field-aligned Spitzer conduction on T and isotropic viscosity
on three velocity components -- a PTL-cycled RKL2 advance and a PTL-cycled
Backward Euler + Jacobi-PCG advance (tol 1e-10), each over dt = 50 times the
operator's explicit Euler limit.  Every advance starts from the same
seeded synthetic fields (copied on the device inside the timed region).

value = grid-point operator applications per second: cells x components x
(STS stages + PCG iterations) summed over the step, divided by the step
time.  Also reported: seconds per PTL-cycled advance, the roofline of the
dominant kernel (average launch duration from HIP events recorded on the
library's stream during the timed steps), and the CPU oracle on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpts/s per stage & s per PTL-cycled advance; HBM roofline %; PCG iters vs Jacobi"
HBM_PEAK_GBS = 8000.0
XGROUP = 8                    # PCG iterations per x update of the FP64 point-Jacobi solves (PA_PCG_XGROUP)
COPY_ELEMS = 1 << 27          # 1 GiB of FP64 read and 1 GiB written
WORKLOAD = "spherical shell 151x301x400 (18.2M cells): field-aligned conduction + vector viscosity (3 spherical components), PTL-cycled RKL2 and BE+Jacobi-PCG at dt = 50 dt_E"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_launch(op, ncomp, cls, N, NCO, coef_var, stage_k=None, word=8, rows=False):
    """Algorithmic HBM bytes of one launch: every array the kernel needs read
    once, every output written once, `word` bytes per value (8: FP64; 4:
    the FP32 stencil and stage kernels).  Field-aligned coefficients are 3
    values per corner; the 7-point operator reads a cell coefficient array
    only when the coefficient varies.  rows: the point-Jacobi diagonal is
    formed from per-(r, theta) row terms (the advance's `jacobi_rows`), so
    the PCG kernels read no per-cell D (the row terms, 16 B per row and per
    phi index, are under 0.1% of a launch and not counted)."""
    coef = 3 * word * NCO if op == "aligned" else (word * N if coef_var else 0)
    f = word * N * ncomp
    if cls == "first":
        return 2 * f + coef
    if cls == "stage":
        nread = {2: 2, 3: 3}.get(stage_k, 4)
        return (nread + 1) * f + coef
    if cls == "matvec":
        return 2 * f + coef
    dcell = 0 if rows else 8 * N
    if cls == "update":
        return 3 * f + dcell    # r, q, D read; r written
    if cls == "dir":
        return 3 * f + dcell    # r, p, D read; the next direction written
    if cls == "xgroup":
        return 2 * f            # x read and written once per group (plus its directions)
    if cls == "init":
        return 4 * f + 8 * N + dcell   # u, y0 (and diag L) read; r, p, D written
    return 0


def dir_class_bytes(op, ncomp, N, NCO, per_cycle, group=8, rows=False):
    """Bytes of the direction class of an FP64 point-Jacobi BE advance: per
    solve of n iterations, n - 1 direction launches (the iteration that
    stops a solve writes no new direction) and the x updates of the groups
    of `group` iterations (x read and written once per group, each
    iteration's direction read once)."""
    f = 8 * N * ncomp
    tot = 0
    for n in per_cycle:
        n = int(n)
        if n <= 0:
            continue
        tot += (n - 1) * bytes_per_launch(op, ncomp, "dir", N, NCO, False, rows=rows)
        tot += n * f + -(-n // group) * bytes_per_launch(op, ncomp, "xgroup", N, NCO, False)
    return tot


def stage_bytes(op, ncomp, N, NCO, coef_var, per_cycle, word=8):
    """Sum of algorithmic bytes over the stage launches of an STS advance."""
    tot = 0
    for s in per_cycle:
        for k in range(2, int(s) + 1):
            tot += bytes_per_launch(op, ncomp, "stage", N, NCO, coef_var, stage_k=k, word=word)
    return tot


def _host_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def _slab(prob, nlev):
    """The first nlev radial levels of a problem (same theta-phi plane, same
    coefficients; the cut is a Dirichlet face with the field's own values):
    the one-thread sample."""
    import dataclasses
    from paper_2403_01004_amd import inputs as _inp
    m = prob.mesh
    mesh = _inp.Mesh(m.r_faces[:nlev + 1].copy(), m.t_faces, m.p_faces)
    sub = lambda a: None if a is None else a[:nlev].copy()
    B = None if prob.B is None else prob.B[:, :nlev + 1].copy()
    return dataclasses.replace(prob, mesh=mesh, u=prob.u[:, :nlev].copy(),
                               ub_out=prob.u[:, nlev - 1].copy(), T0=sub(prob.T0), B=B,
                               w=sub(prob.w), fc=sub(prob.fc))


def run_cpu_baseline(probs, gpu, slab_levels=8):
    """The oracle (as it stands) on a bounded sample of each benchmarked
    advance: its first cycle, at the cycle length the GPU took, on all host
    threads (full grid) and on one thread (the first slab_levels radial
    levels).  Per advance: oracle Gpts/s per STS stage or PCG iteration and
    the seconds one advance would take at that rate, beside the GPU's."""
    import oracle
    oracle.build(force=False)
    threads = oracle.num_threads()
    out = {}
    tot_units = tot_t = 0.0
    for name, st in gpu.items():
        kind, opn = name.split("_", 1)
        prob = probs[opn]
        dt1 = float(st["dt_cycle"][0])
        res = {}
        for label, p, nth in (("all_threads", prob, threads),
                              ("one_thread", _slab(prob, slab_levels), 1)):
            oracle.set_num_threads(nth)
            try:
                o = oracle.Oracle.from_problem(p)
                t0 = time.perf_counter()
                if kind == "rkl2":
                    _, so = o.advance_sts(p.u, dt1, 1, "rkl2")
                    units = so["s_total"]
                else:
                    _, so = o.advance_be(p.u, dt1, 1e-10, 1)
                    units = so["iters_total"]
                t = time.perf_counter() - t0
            finally:
                oracle.set_num_threads(threads)
            pts = p.mesh.ncells * p.ncomp * units
            res[label] = {"Gpts_s": round(pts / t / 1e9, 5), "s": round(t, 2),
                          "units": int(units), "cells": p.mesh.ncells * p.ncomp}
            if label == "all_threads":
                tot_units += pts
                tot_t += t
        gunits = st["s_total"] if kind == "rkl2" else st["iters_total"]
        rate = res["all_threads"]["Gpts_s"] * 1e9
        res["s_per_advance_est"] = round(prob.mesh.ncells * prob.ncomp * gunits / rate, 2)
        res["gpu_s_per_advance"] = round(st["ms_total"] / 1e3, 4)
        res["gpu_over_oracle"] = round(res["s_per_advance_est"] / res["gpu_s_per_advance"], 1)
        res["unit"] = "STS stage" if kind == "rkl2" else "PCG iteration"
        out[name] = res
    triad = oracle.stream_triad(1 << 26, 5)
    return {"value": round(tot_units / tot_t / 1e9, 5), "unit": "Gpts/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the first cycle of each of the four benchmarked advances at the GPU's "
                      f"cycle length: full grid on {threads} host threads ({_host_model()}); "
                      f"value = grid-point stages and PCG iterations per second over the four; "
                      f"per advance also one thread on the first {slab_levels} radial levels",
            "advances": out, "host_stream_triad_GB_s": round(triad, 1), "nproc": os.cpu_count()}


# committed counter summaries: roofline kernel -> (summary, source file of the kernel)
TRAFFIC_PROFILES = {
    "be_viscosity/update": ("profiles/k_pcg_update_viscosity_151x301x400.md",
                            "paper_2403_01004_amd/csrc/pa_vec.hip"),
    "be_viscosity/dir": ("profiles/k_pcg_dir_viscosity_151x301x400.md",
                         "paper_2403_01004_amd/csrc/pa_vec.hip"),
}


def measured_traffic(kernel, shape):
    """HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE summary of this
    kernel and workload, or None when there is none or the kernel's source
    changed since the counters were taken."""
    import hashlib
    import re
    ent = TRAFFIC_PROFILES.get(kernel)
    if ent is None or tuple(shape) != (151, 301, 400):
        return None
    prof, src = (os.path.join(ROOT, x) for x in ent)
    try:
        txt = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch: (\d+)", txt)
    h = re.search(r"kernel_source_sha256 \([^)]*\): ([0-9a-f]+)", txt)
    if not m or not h or h.group(1) != sha:
        return None
    return int(m.group(1))


def kernel_accounting(s, op, nc, N, NCO, coef_var=False):
    """Per kernel class of one advance's statistics (timing on): [ms,
    effective launches, algorithmic bytes].  Launches a PCG batch queues
    after its solve stopped exit at once: one effective launch per
    iteration, all launch time charged to them."""
    out = {}
    rows = bool(s.get("jacobi_rows", False))
    for cls, ms in s["kernel_ms"].items():
        calls = s["kernel_calls"][cls]
        if calls == 0:
            continue
        if cls in ("matvec", "update", "dir"):
            calls = s["iters_total"]
            if calls == 0:
                continue
        if cls == "stage":
            by = stage_bytes(op, nc, N, NCO, coef_var, s["per_cycle"])
        elif cls == "dir":
            by = dir_class_bytes(op, nc, N, NCO, s["per_cycle"], XGROUP, rows)
        else:
            by = calls * bytes_per_launch(op, nc, cls, N, NCO, coef_var, rows=rows)
        out[cls] = [ms, calls, by]
    return out


def rel_l2(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def fp32_leg(paradv, torch, dev, cond, visc, reps=3):
    """FP32 stencil and STS stages (FP64 recurrence coefficients, combination
    and reductions) and the FP32-matvec BE solve (FP64 defect correction)
    against the FP64 path on the same inputs: seconds per PTL-cycled advance
    and relative L2 error per field.  The FP64 path matches the oracle to
    1e-12, so its result stands in for the oracle's at this size."""
    out = {}
    for name, prob, op, nc, T0, scale, expo in (
            ("conduction", cond, "aligned", 1, cond.T0, 1.0, 2.5),
            ("viscosity", visc, visc.op, 3, None, 1e-3, 0.0)):
        res = {}
        ref = {}
        for prec in ("fp64", "fp32"):
            g = paradv.Operator(prob.mesh, op, nc, "dirichlet", "dirichlet", prec)
            g.set_bc(prob.ub_in, prob.ub_out)
            g.set_coefficients(None if T0 is None else torch.as_tensor(T0, device=dev), scale,
                               expo, None if prob.B is None else torch.as_tensor(prob.B, device=dev))
            dt = 50 * g.dt_explicit()
            u0 = torch.as_tensor(prob.u, device=dev)
            u = torch.empty_like(u0)
            for kind in ("rkl2", "be"):
                times = []
                for k in range(reps + 1):
                    u.copy_(u0)
                    g.bind(u)
                    st = g.advance_rkl2(dt, 0) if kind == "rkl2" else g.advance_be(dt, 1e-10, 0)
                    if k > 0:
                        times.append(st["ms_total"] / 1e3)
                if kind == "rkl2" and prec == "fp32":
                    # one more run with per-class timing: the FP32 PTL pass
                    # and stage kernels against their FP32 bytes
                    g.set_options(timing=1)
                    u.copy_(u0)
                    g.bind(u)
                    tst = g.advance_rkl2(dt, 0)
                    g.set_options()
                    mr, mt, mp = prob.mesh.shape
                    N, NCO = mr * mt * mp, (mr + 1) * (mt + 1) * mp
                    cls_gbs = {}
                    for cls in ("first", "stage"):
                        ms = tst["kernel_ms"][cls]
                        if ms <= 0:
                            continue
                        by = (stage_bytes(op, nc, N, NCO, T0 is not None, tst["per_cycle"], word=4)
                              if cls == "stage" else
                              tst["kernel_calls"][cls] * bytes_per_launch(op, nc, cls, N, NCO,
                                                                          T0 is not None, word=4))
                        cls_gbs[cls] = {"GB_s": round(by / (ms / 1e3) / 1e9, 1),
                                        "frac": round(by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 3)}
                key = f"{kind}_{prec}"
                res[key] = {"s_per_advance": round(min(times), 4), "cycles": st["cycles"],
                            "stages" if kind == "rkl2" else "pcg_iters":
                                st["s_total"] if kind == "rkl2" else st["iters_total"]}
                if prec == "fp64":
                    ref[kind] = u.clone()
                else:
                    res[key]["rel_err_vs_fp64"] = [round(rel_l2(u[c], ref[kind][c]), 9)
                                                   for c in range(nc)]
                    if kind == "rkl2":
                        res[key]["kernels_fp32"] = cls_gbs
                    res[key]["speedup_vs_fp64"] = round(
                        res[f"{kind}_fp64"]["s_per_advance"] / res[key]["s_per_advance"], 3)
            del g
            torch.cuda.empty_cache()
        out[name] = res
    return out


def learned_leg(paradv, inputs, torch, dev, nr, nt, np_, reps=2):
    """BE on the transition-region conduction problem: Jacobi PCG against
    FCG(1) with the learned preconditioner, trained on the GPU on pairs
    from the plain solver at the first cycle's step (training time reported
    separately), same tolerance 1e-10 on the true residual."""
    tr = inputs.transition_region(nr, nt, np_)
    g = paradv.Operator.from_problem(tr)
    u0 = torch.as_tensor(tr.u, device=dev)
    u = torch.empty_like(u0)
    dt = 50 * g.dt_explicit()

    def run(pc):
        g.set_options(pc=paradv.PCS[pc])
        best = None
        for k in range(reps + 1):
            u.copy_(u0)
            g.bind(u)
            st = g.advance_be(dt, 1e-10, 0)
            if k > 0 and (best is None or st["ms_total"] < best["ms_total"]):
                best = st
        return best

    sj = run("jacobi")
    dt1 = float(sj["dt_cycle"][0])
    u.copy_(u0)
    g.bind(u)
    g.lpc_set_weights(paradv.he_init(4300))
    t0 = time.perf_counter()
    rep = g.lpc_train(dt1)
    t_train = time.perf_counter() - t0
    sl = run("learned")
    # the network's step alone, z = P(r) on the first cycle's system, and the
    # least it could cost on this chip: 21.6 kflop per cell on the BF16
    # matrix cores, or the HBM bytes of a fused network reading r, D and the
    # six face couplings and writing z (72 B per cell)
    N = nr * nt * np_
    r = torch.randn(tr.mesh.shape, dtype=torch.float64, device=dev)
    g.lpc_apply(dt1, r)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    napp = 10
    e0.record()
    for _ in range(napp):
        g.lpc_apply(dt1, r)
    e1.record()
    e1.synchronize()
    t_app = e0.elapsed_time(e1) / napp / 1e3
    flop = 21600.0 * N
    t_roof = max(flop / 2.5e15, 72.0 * N / (HBM_PEAK_GBS * 1e9))
    t_jac = sj["ms_total"] / 1e3 / max(sj["iters_total"], 1)
    return {
        "workload": f"transition-region conduction {nr}x{nt}x{np_}, BE PTL-cycled at dt = 50 dt_E, tol 1e-10",
        "jacobi": {"s_per_advance": round(sj["ms_total"] / 1e3, 4), "pcg_iters": sj["iters_total"],
                   "cycles": sj["cycles"]},
        "learned": {"s_per_advance": round(sl["ms_total"] / 1e3, 4), "pcg_iters": sl["iters_total"],
                    "cycles": sl["cycles"], "fallbacks": sl["fallbacks"],
                    "rel_residual": sl["rel_residual"]},
        "iters_ratio": round(sl["iters_total"] / max(sj["iters_total"], 1), 3),
        "speedup_vs_jacobi": round(sj["ms_total"] / max(sl["ms_total"], 1e-9), 3),
        "network": {"ms_per_application": round(1e3 * t_app, 3),
                    "TFLOP_s": round(flop / t_app / 1e12, 1),
                    "frac_of_bf16_peak": round(flop / t_app / 2.5e15, 4),
                    "roofline_ms": round(1e3 * t_roof, 3),
                    "jacobi_ms_per_iteration": round(1e3 * t_jac, 3)},
        # the learned solve pays only if it needs fewer than this fraction of
        # Jacobi's iterations (a step = a Jacobi iteration plus the network)
        "break_even_iters_ratio": {"measured_step": round(t_jac / (t_jac + t_app), 3),
                                   "network_at_roofline": round(t_jac / (t_jac + t_roof), 3)},
        "training": {"s": round(t_train, 2), "pairs": rep["pairs"], "steps": rep["steps"],
                     "snapshots": rep["snapshots"], "ref_iters": rep["ref_iters"],
                     "loss_first": round(rep["loss_first"], 5),
                     "loss_last": round(rep["loss_last"], 5),
                     "ms_pairs": round(rep["ms_pairs"], 1), "ms_train": round(rep["ms_train"], 1)},
    }


def rkg2_leg(paradv, torch, dev, cond, visc, reps=3):
    """The paper's own STS scheme, RKG2 (App. A), PTL-cycled at dt = 50 dt_E on
    both operators, beside BE+Jacobi-PCG on the same fields: seconds per
    advance and the BE / RKG2 ratio (the comparison of Sec. 4.2)."""
    out = {}
    for name, prob in (("conduction", cond), ("viscosity", visc)):
        g = paradv.Operator.from_problem(prob)
        u0 = torch.as_tensor(prob.u, device=dev)
        u = torch.empty_like(u0)
        dt = 50 * g.dt_explicit()
        res = {}
        for kind in ("rkg2", "be"):
            best = None
            for k in range(reps + 1):
                u.copy_(u0)
                g.bind(u)
                st = g.advance_rkg2(dt, 0) if kind == "rkg2" else g.advance_be(dt, 1e-10, 0)
                if k > 0 and (best is None or st["ms_total"] < best["ms_total"]):
                    best = st
            res[kind] = {"s_per_advance": round(best["ms_total"] / 1e3, 4), "cycles": best["cycles"],
                         "stages" if kind == "rkg2" else "pcg_iters":
                             best["s_total"] if kind == "rkg2" else best["iters_total"]}
        res["be_over_rkg2"] = round(res["be"]["s_per_advance"] /
                                    max(res["rkg2"]["s_per_advance"], 1e-9), 2)
        out[name] = res
        del g
        torch.cuda.empty_cache()
    return out


def bilu0_leg(paradv, inputs, torch, dev, visc, nr, nt, np_, reps=3):
    """BE with the block ILU(0) preconditioner (PC2 of Sec. 3.1) against
    point Jacobi (PC1) on the 7-point workloads: the viscosity fields as
    three scalar components and the isotropic heat recipe at the same grid,
    PTL-cycled at dt = 50 dt_E, tol 1e-10; seconds per advance, iterations,
    speedup."""
    out = {"workload": f"{nr}x{nt}x{np_}, BE PTL-cycled at dt = 50 dt_E, tol 1e-10, "
                       "boxes 8x4x16"}
    import dataclasses
    # block ILU(0) is built for the 7-point operator: the viscosity fields as
    # three scalar components
    visc7 = dataclasses.replace(visc, op="iso7")
    for name, prob in (("viscosity", visc7), ("heat", inputs.heat_iso(nr, nt, np_))):
        g = paradv.Operator.from_problem(prob)
        u0 = torch.as_tensor(prob.u, device=dev)
        u = torch.empty_like(u0)
        dt = 50 * g.dt_explicit()
        res = {}
        for pc in ("jacobi", "bilu0"):
            g.set_options(pc=paradv.PCS[pc])
            best = None
            for k in range(reps + 1):
                u.copy_(u0)
                g.bind(u)
                st = g.advance_be(dt, 1e-10, 0)
                if k > 0 and (best is None or st["ms_total"] < best["ms_total"]):
                    best = st
            res[pc] = {"s_per_advance": round(best["ms_total"] / 1e3, 4),
                       "pcg_iters": best["iters_total"], "cycles": best["cycles"],
                       "rel_residual": best["rel_residual"]}
        res["iters_ratio"] = round(res["bilu0"]["pcg_iters"] / max(res["jacobi"]["pcg_iters"], 1), 3)
        res["speedup_vs_jacobi"] = round(res["jacobi"]["s_per_advance"] /
                                         max(res["bilu0"]["s_per_advance"], 1e-9), 3)
        del g
        torch.cuda.empty_cache()
        # block ILU(0) with FP32 matvecs inside the FP64 defect correction
        g32 = paradv.Operator.from_problem(prob, prec="fp32")
        g32.set_options(pc=paradv.PCS["bilu0"])
        best = None
        for k in range(reps + 1):
            u.copy_(u0)
            g32.bind(u)
            st = g32.advance_be(dt, 1e-10, 0)
            if k > 0 and (best is None or st["ms_total"] < best["ms_total"]):
                best = st
        res["bilu0_fp32_matvec"] = {"s_per_advance": round(best["ms_total"] / 1e3, 4),
                                    "pcg_iters": best["iters_total"], "cycles": best["cycles"],
                                    "rel_residual": best["rel_residual"]}
        res["bilu0_fp32_speedup_vs_jacobi"] = round(
            res["jacobi"]["s_per_advance"] / max(res["bilu0_fp32_matvec"]["s_per_advance"], 1e-9), 3)
        out[name] = res
        del g32
        torch.cuda.empty_cache()
    return out


def c1_leg(paradv, inputs, torch, dev, reps=20):
    """The small scalar heat workload, 32 x 32 x 64 (kappa = T^{5/2},
    Dirichlet T): one RKL2 advance of s = 10 stages at dt = 24.3 dt_E and one
    Backward Euler + Jacobi PCG step at the same dt, tol 1e-10.  It fits in
    the caches and is bound by launch latency, so no roofline is attached;
    median of `reps` timed repetitions."""
    prob = inputs.heat_iso(32, 32, 64)
    g = paradv.Operator.from_problem(prob)
    dt = 24.3 * g.dt_explicit()
    u0 = torch.as_tensor(prob.u, device=dev)
    u = torch.empty_like(u0)
    out = {"workload": "32x32x64 scalar heat, kappa = T^(5/2), dt = 24.3 dt_E"}
    N = prob.mesh.ncells
    for kind in ("rkl2", "be"):
        if kind == "rkl2":
            g.set_options(s_override=10, force_odd=0)
        else:
            g.set_options()
        ms, st = [], None
        for k in range(reps + 2):
            u.copy_(u0)
            g.bind(u)
            st = g.advance_rkl2(dt, 1) if kind == "rkl2" else g.advance_be(dt, 1e-10, 1)
            if k >= 2:
                ms.append(st["ms_total"])
        t = sorted(ms)[len(ms) // 2] / 1e3
        units = st["s_total"] if kind == "rkl2" else st["iters_total"]
        out[kind] = {"s_per_advance": round(t, 6), "stages" if kind == "rkl2" else "pcg_iters": units,
                     "Gpts_s": round(N * units / t / 1e9, 3)}
    return out


def unfloored_leg(paradv, torch, dev, cond, visc, reps=2, max_cycles=20000):
    """RKL2 cycled at the paper's limit without the floor of dt_E (ptl_floor
    = 0) beside the floored form, on the benchmark's fields: cycles, stages
    and seconds per advance (max_cycles bounds the unfloored run)."""
    out = {}
    for name, prob in (("conduction", cond), ("viscosity", visc)):
        g = paradv.Operator.from_problem(prob)
        u0 = torch.as_tensor(prob.u, device=dev)
        u = torch.empty_like(u0)
        dt = 50 * g.dt_explicit()
        res = {}
        for label, floor in (("floored", 1.0), ("unfloored", 0.0)):
            g.set_options(ptl_floor=floor, max_cycles=max_cycles)
            best = None
            for k in range(reps + 1):
                u.copy_(u0)
                g.bind(u)
                st = g.advance_rkl2(dt, 0, check=False)
                if k > 0 and (best is None or st["ms_total"] < best["ms_total"]):
                    best = st
            res[label] = {"s_per_advance": round(best["ms_total"] / 1e3, 4),
                          "cycles": best["cycles"], "stages": best["s_total"],
                          "status": paradv.STATUS_NAMES[best["status"]],
                          "dt_ptl_min_over_dtE": float(f"{best['dt_ptl_min'] / g.dt_explicit():.4g}")}
        out[name] = res
        del g
        torch.cuda.empty_cache()
    return out


def c5_leg(paradv, inputs, torch, dev, shape=(256, 512, 1024), reps=2, nseq=20):
    """The largest workload, 256 x 512 x 1024 (134 M cells): transition-region
    conduction (T jump at i_tr = 20 + 4 S(501)) and the vector viscosity.
    Per operator, PTL-cycled at dt = 50 dt_E: FP64 RKL2 and BE + Jacobi PCG
    with seconds per advance, cycles, stages or iterations and algorithmic
    GB/s (fraction of 8 TB/s); FP32-stage RKL2 and FP32-matvec BE with their
    speedup.  Then nseq consecutive FP32-stage RKL2 advances of the
    conduction with the diffusivity recomputed from the current field before
    each (time step fixed from the first)."""
    nr, nt, np_ = shape
    N, NCO = nr * nt * np_, (nr + 1) * (nt + 1) * np_
    t0 = time.perf_counter()
    cond = inputs.transition_region(nr, nt, np_, seed=501, i_tr0=20.0, i_amp=4.0)
    visc = inputs.viscosity_device(nr, nt, np_, torch, dev)
    out = {"workload": f"{nr}x{nt}x{np_}: transition-region conduction and vector viscosity, "
                       "PTL-cycled at dt = 50 dt_E, tol 1e-10",
           "inputs_s": round(time.perf_counter() - t0, 1)}
    for name, prob, op, nc in (("conduction", cond, "aligned", 1), ("viscosity", visc, "viscv", 3)):
        res = {}
        u0 = torch.as_tensor(prob.u, device=dev)
        u = torch.empty_like(u0)
        for prec in ("fp64", "fp32"):
            g = paradv.Operator.from_problem(prob, prec=prec)
            g.set_options(timing=int(prec == "fp64"))
            dt = 50 * g.dt_explicit()
            for kind in ("rkl2", "be"):
                best = None
                for k in range(reps + 1):
                    u.copy_(u0)
                    g.bind(u)
                    st = g.advance_rkl2(dt, 0) if kind == "rkl2" else g.advance_be(dt, 1e-10, 0)
                    if k > 0 and (best is None or st["ms_total"] < best["ms_total"]):
                        best = st
                r = {"s_per_advance": round(best["ms_total"] / 1e3, 4), "cycles": best["cycles"],
                     "stages" if kind == "rkl2" else "pcg_iters":
                         best["s_total"] if kind == "rkl2" else best["iters_total"]}
                if prec == "fp64":
                    by = sum(v[2] for v in kernel_accounting(best, op, nc, N, NCO).values())
                    r["GB_s"] = round(by / (best["ms_total"] / 1e3) / 1e9, 1)
                    r["hbm_frac"] = round(r["GB_s"] / HBM_PEAK_GBS, 3)
                else:
                    r["speedup_vs_fp64"] = round(res[f"{kind}_fp64"]["s_per_advance"] /
                                                 r["s_per_advance"], 3)
                res[f"{kind}_{prec}"] = r
            del g
            torch.cuda.empty_cache()
        out[name] = res
        del u0, u
    # consecutive advances with the diffusivity re-lagged before each
    g = paradv.Operator.from_problem(cond, prec="fp32")
    dt = 50 * g.dt_explicit()
    u = g.bind(cond.u)
    T0 = torch.empty_like(u[0])
    Bd = torch.as_tensor(cond.B, device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cyc = stg = 0
    for k in range(nseq):
        if k:
            T0.copy_(u[0])
            g.set_coefficients(T0, cond.scale, cond.expo, Bd)
        st = g.advance_rkl2(dt, 0)
        cyc += st["cycles"]
        stg += st["s_total"]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t1
    out["sequence"] = {"advances": nseq, "s": round(ts, 3), "s_per_advance": round(ts / nseq, 4),
                       "cycles": cyc, "stages": stg,
                       "what": "FP32-stage RKL2 conduction, diffusivity recomputed from the "
                               "current temperature before each advance"}
    del g, u, Bd
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--shape", default="151,301,400")
    ap.add_argument("--leg-reps", type=int, default=3,
                    help="timed repetitions of each advance in the block ILU(0) leg")
    ap.add_argument("--legs", default="c1,fp32,learned,bilu0,rkg2,unfloored,c5",
                    help="extra legs reported beside the timed step: c1, fp32, learned, bilu0, "
                         "rkg2, unfloored, c5, none")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs the advance on a single "
              "MI355X and does not shard it across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2403_01004_amd import inputs, paradv
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    nr, nt, np_ = (int(x) for x in args.shape.split(","))
    dev = torch.device("cuda:0")
    log(f"building inputs {nr}x{nt}x{np_}")
    cond = inputs.conduction(nr, nt, np_)
    visc = inputs.viscosity(nr, nt, np_, vector=True)
    N = nr * nt * np_
    NCO = (nr + 1) * (nt + 1) * np_

    gc = paradv.Operator(cond.mesh, "aligned", 1, "dirichlet", "dirichlet", "fp64")
    gv = paradv.Operator(visc.mesh, "viscv", 3, "dirichlet", "dirichlet", "fp64")
    gc.set_bc(cond.ub_in, cond.ub_out)
    gv.set_bc(visc.ub_in, visc.ub_out)
    T0 = torch.as_tensor(cond.T0, device=dev)
    B = torch.as_tensor(cond.B, device=dev)
    uc0 = torch.as_tensor(cond.u, device=dev)
    uv0 = torch.as_tensor(visc.u, device=dev)
    uc = torch.empty_like(uc0)
    uv = torch.empty_like(uv0)

    def step(timing):
        for g in (gc, gv):
            g.set_options(timing=int(timing))
        t = {}
        gc.set_coefficients(T0, 1.0, 2.5, B)
        gv.set_coefficients(None, 1e-3, 0.0, None)
        dtc, dtv = 50 * gc.dt_explicit(), 50 * gv.dt_explicit()
        uc.copy_(uc0)
        gc.bind(uc)
        t["rkl2_conduction"] = gc.advance_rkl2(dtc, 0)
        uv.copy_(uv0)
        gv.bind(uv)
        t["rkl2_viscosity"] = gv.advance_rkl2(dtv, 0)
        uc.copy_(uc0)
        gc.bind(uc)
        t["be_conduction"] = gc.advance_be(dtc, 1e-10, 0)
        uv.copy_(uv0)
        gv.bind(uv)
        t["be_viscosity"] = gv.advance_be(dtv, 1e-10, 0)
        return t

    # plain device copy of known size: the achievable-bandwidth reference,
    # and the kernel whose FETCH_SIZE / WRITE_SIZE counters calibrate the
    # HBM traffic of the hot kernels in a --pmc run
    ca = torch.ones(COPY_ELEMS, dtype=torch.float64, device=dev)
    cb = torch.empty_like(ca)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    copy_ms = []
    for k in range(4):
        e0.record()
        cb.copy_(ca)
        e1.record()
        e1.synchronize()
        if k:
            copy_ms.append(e0.elapsed_time(e1))
    copy_gbs = 2 * 8 * COPY_ELEMS / (min(copy_ms) / 1e3) / 1e9
    del ca, cb

    for w in range(args.warmup):
        log(f"warmup {w}")
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        stats.append(step(True))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    ncomp = {"rkl2_conduction": 1, "rkl2_viscosity": 3, "be_conduction": 1, "be_viscosity": 3}
    ops = {"rkl2_conduction": "aligned", "rkl2_viscosity": "viscv", "be_conduction": "aligned",
           "be_viscosity": "viscv"}
    work = 0
    adv = {}
    kern = {}   # (advance, class) -> [ms, calls, bytes]
    for t in stats:
        for name, s in t.items():
            n = s["s_total"] + s["iters_total"]
            work += N * ncomp[name] * n
            a = adv.setdefault(name, {"s": 0.0, "cycles": 0, "stages": 0, "pcg_iters": 0})
            a["s"] += s["ms_total"] / 1e3 / args.steps
            a["cycles"] = s["cycles"]
            a["stages"] = s["s_total"]
            a["pcg_iters"] = s["iters_total"]
            for cls, (ms, calls, by) in kernel_accounting(s, ops[name], ncomp[name], N,
                                                          NCO).items():
                e = kern.setdefault((name, cls), [0.0, 0, 0])
                e[0] += ms
                e[1] += calls
                e[2] += by
    value = work / elapsed / 1e9
    (dname, dcls), (dms, dcalls, dbytes) = max(kern.items(), key=lambda kv: kv[1][0])
    avg_ms = dms / dcalls
    achieved = dbytes / dcalls / (avg_ms / 1e3) / 1e9
    # whole advances: algorithmic bytes of all their kernels over the advance's
    # wall time (host syncs and reductions included)
    for name, a in adv.items():
        by = sum(v[2] for (an, _), v in kern.items() if an == name) / args.steps
        a["GB_s"] = round(by / a["s"] / 1e9, 1) if a["s"] > 0 else None
        a["hbm_frac"] = round(by / a["s"] / 1e9 / HBM_PEAK_GBS, 3) if a["s"] > 0 else None
    kernels = {f"{a}/{c}": {"ms_total": round(v[0] / args.steps, 3), "calls": v[1] // args.steps,
                            "avg_us": round(1e3 * v[0] / v[1], 2),
                            "GB_s": round(v[2] / (v[0] / 1e3) / 1e9, 1) if v[2] else None,
                            "frac": round(v[2] / (v[0] / 1e3) / 1e9 / HBM_PEAK_GBS, 3)
                            if v[2] else None}
               for (a, c), v in sorted(kern.items(), key=lambda kv: -kv[1][0])}
    # the stencil kernels (operator apply inside the PTL pass, the fused STS
    # stage and the PCG matvec) per operator, beside the dominant kernel
    stencil = {}
    for opn in ("conduction", "viscosity"):
        for cls in ("first", "stage", "matvec"):
            ms = by = 0.0
            for (a, c), v in kern.items():
                if a.endswith(opn) and c == cls:
                    ms += v[0]
                    by += v[2]
            if ms > 0:
                stencil[f"{opn}/{cls}"] = {"GB_s": round(by / (ms / 1e3) / 1e9, 1),
                                           "frac": round(by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 3)}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "grid": [nr, nt, np_], "dt_over_dtE": 50,
                   "pcg_tol": 1e-10, "sts": "rkl2", "preconditioner": "jacobi"},
        "s_per_advance": {k: round(v["s"], 4) for k, v in adv.items()},
        "advances": adv,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(f"{dname}/{dcls}", (nr, nt, np_)),
                     "kernel": f"{dname}/{dcls}", "avg_launch_us": round(1e3 * avg_ms, 2),
                     "bytes_per_launch": int(dbytes / dcalls)},
        "stencil_roofline": stencil,
        "kernels": kernels,
        "copy_GB_s": round(copy_gbs, 1),
    }
    # the argmax form of the limit (Eq. ptl3, used by the advances) against
    # the minimum of Eq. (ptl2) over every cell pair, on the step's fields
    ptl = {}
    for name, g, uw, u0 in (("conduction", gc, uc, uc0), ("viscosity", gv, uv, uv0)):
        uw.copy_(u0)
        g.bind(uw)
        da, ka = g.ptl()
        df, kf = g.ptl_full()
        sig = lambda x: float(f"{x:.4g}")
        ptl[name] = {"dt_argmax_over_dtE": sig(da / g.dt_explicit()),
                     "dt_fullgrid_over_dtE": sig(df / g.dt_explicit()),
                     "argmax_over_fullgrid": sig(da / df), "k_argmax": ka, "k_fullgrid": kf}
    out["ptl_argmax_vs_fullgrid"] = ptl
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    if "fp32" in legs:
        log("fp32 leg")
        out["fp32_stages"] = fp32_leg(paradv, torch, dev, cond, visc)
    if "learned" in legs:
        log("learned-preconditioner leg")
        out["learned_pc"] = learned_leg(paradv, inputs, torch, dev, nr, nt, np_)
    if "rkg2" in legs:
        log("RKG2 leg")
        out["rkg2_vs_be"] = rkg2_leg(paradv, torch, dev, cond, visc)
    if "bilu0" in legs:
        log("block ILU(0) leg")
        out["bilu0_pc"] = bilu0_leg(paradv, inputs, torch, dev, visc, nr, nt, np_,
                                    reps=args.leg_reps)
    if "c1" in legs:
        log("32x32x64 leg")
        out["c1"] = c1_leg(paradv, inputs, torch, dev)
    if "unfloored" in legs:
        log("unfloored limit leg")
        out["rkl2_unfloored_ptl"] = unfloored_leg(paradv, torch, dev, cond, visc)
    if "c5" in legs:
        log("256x512x1024 leg")
        out["c5"] = c5_leg(paradv, inputs, torch, dev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = run_cpu_baseline({"conduction": cond, "viscosity": visc}, stats[-1])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
