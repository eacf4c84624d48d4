#!/usr/bin/env python3
"""Throughput of the per-point chemistry path on one MI355X.

One step = species production rates + mixture-averaged transport (mu, lambda,
D_km) for every point of the 53-species / 325-reaction synthetic mechanism
workload (2^20 points, T ~ U[300, 2800] K, p ~ U[1, 40] atm, Y ~ Dirichlet(0.3)),
inputs resident in HBM.  `value` is FP64 Mpoints/s; the mixed-precision path
is timed the same way and reported beside it.  Prints one JSON line on stdout
(progress goes to stderr).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6
FP32_VALU_PEAK_TFLOPS = 157.3
SERVE_SEED = 5
SERVE_LOADS = (0.25, 0.5, 0.75, 0.9, 1.1)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# Sources whose change invalidates a committed traffic measurement of a kernel.
KERNEL_SOURCES = {
    "rates": ["kx_rates.hip", "kx_math.h", "kx_internal.h"],
    "transport": ["kx_transport.hip", "kx_math.h", "kx_internal.h"],
}


def kernel_sources_sha256(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2411_02640_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(kernel, precision="fp64"):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    `kernel` on this workload, or None if there is none or the kernel's sources
    changed since it was taken."""
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_syn53_{precision}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    h = re.search(r"kernel_sources_sha256:\s*([0-9a-f]{64})", text)
    if not m or not h or h.group(1) != kernel_sources_sha256(kernel):
        return None
    return float(m.group(1))


def copy_probe(torch, gib=1):
    """A plain elementwise kernel of known traffic (reads and writes `gib`
    GiB), run three times: its FETCH_SIZE / WRITE_SIZE readings calibrate the
    HBM counters."""
    n = (gib << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def time_path(kx, dm, Td, pd, Yd, outs, steps, warmup, precision, symmetric=False,
              prewarm_s=0.0):
    """Time `steps` steps; returns wall seconds and per-kernel mean ms.  Before
    the `warmup` steps, untimed steps run for at least `prewarm_s` seconds: the
    GPU's clocks rise over the first tens of milliseconds of sustained load (the
    rates kernel's launches go from 1.81 to 1.58 ms over the first 13 of a
    run), so the timed steps see the steady state."""
    import torch
    wdot, (mu, lam, Dm) = outs
    t_end = time.perf_counter() + prewarm_s
    while time.perf_counter() < t_end:
        kx.production_rates(dm, Td, pd, Yd, out=wdot, precision=precision)
        kx.transport(dm, Td, pd, Yd, out=(mu, lam, Dm), precision=precision,
                     symmetric=symmetric)
        torch.cuda.synchronize()
    for _ in range(warmup):
        kx.production_rates(dm, Td, pd, Yd, out=wdot, precision=precision)
        kx.transport(dm, Td, pd, Yd, out=(mu, lam, Dm), precision=precision,
                     symmetric=symmetric)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        kx.production_rates(dm, Td, pd, Yd, out=wdot, precision=precision)
        ev[k][1].record()
        kx.transport(dm, Td, pd, Yd, out=(mu, lam, Dm), precision=precision,
                     symmetric=symmetric)
        ev[k][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r = sorted(e[0].elapsed_time(e[1]) for e in ev)
    t = sorted(e[1].elapsed_time(e[2]) for e in ev)
    time_path.medians = (r[len(r) // 2], t[len(t) // 2])
    return wall, sum(r) / steps, sum(t) / steps


def other_workloads(kx, I, torch, steps, warmup):
    """Kernel times of the other workload sizes, on device-generated states of
    the same distributions (T ~ U[300, 2800] K, p ~ U[1, 40] atm, Y ~
    Dirichlet(0.3)): syn53 at 2^22 points; syn200 at 2^20 points with 1/D_kj fit
    tables (matrix-core transport) and with D_kj fit tables (vector-ALU
    transport); and a sweep of the point count for syn53.  No kernel branches
    on state values other than the NASA temperature range, so the work per
    point does not depend on how the states are drawn."""
    import dataclasses
    from paper_2411_02640_amd import serve_load

    def run(mech, n, seed, nsteps, symmetric=False):
        dm = kx.Mechanism(mech, 0)
        ns = int(mech["n_species"])
        (_, T, p, Y), = serve_load.make_pool(dm, ns, [n], seed)
        kw = dict(dtype=torch.float64, device="cuda:0")
        outs = (torch.empty((ns, n), **kw),
                (torch.empty(n, **kw), torch.empty(n, **kw), torch.empty((ns, n), **kw)))
        entry = {"n_points": n, "n_species": ns, "n_reactions": int(mech["n_reactions"]),
                 "steps": nsteps}
        for prec in ("fp64", "mixed"):
            wall, r, t = time_path(kx, dm, T, p, Y, outs, nsteps, warmup, prec, symmetric)
            entry[prec] = {"Mpoints_s": n * nsteps / wall / 1e6, "rates_ms": r,
                           "transport_ms": t, "rates_ms_median": time_path.medians[0],
                           "transport_ms_median": time_path.medians[1]}
        del outs, T, p, Y
        dm.close()
        torch.cuda.empty_cache()
        return entry

    m53 = I.make_mechanism(I.MECH_53)
    res = {"states": "device-generated (torch generator), seeds 11-13 and 20+"}
    log("syn53 at 2^22 points")
    res["syn53_2p22"] = run(m53, 1 << 22, 11, steps)
    m200 = I.make_mechanism(I.MECH_200)
    log("syn200 at 2^20 points (1/D_kj fits)")
    res["syn200_2p20"] = run(m200, 1 << 20, 12, steps)
    log("syn200 at 2^20 points (D_kj fits)")
    m200d = I.make_mechanism(dataclasses.replace(I.MECH_200, diff_fit_kind=0))
    res["syn200_2p20_dfit"] = run(m200d, 1 << 20, 13, steps)
    # the same tables with each unordered pair's D_kj fit evaluated once
    # (KX_DKJ_SYMMETRIC), and both variants on the 53-species D_kj tables
    log("syn200 at 2^20 points (D_kj fits, symmetric pairs)")
    res["syn200_2p20_dfit_symmetric"] = run(m200d, 1 << 20, 13, steps, symmetric=True)
    m53d = I.make_mechanism(dataclasses.replace(I.MECH_53, diff_fit_kind=0))
    log("syn53 at 2^20 points (D_kj fits, full and symmetric pairs)")
    res["syn53_2p20_dfit"] = run(m53d, 1 << 20, 14, steps)
    res["syn53_2p20_dfit_symmetric"] = run(m53d, 1 << 20, 14, steps, symmetric=True)
    sweep = []
    for e in range(10, 25, 2):
        n = 1 << e
        log(f"sweep n = 2^{e}")
        r = run(m53, n, 20 + e, max(steps, min(400, (1 << 22) // n)))
        sweep.append({"n_points": n, "fp64_Mpoints_s": r["fp64"]["Mpoints_s"],
                      "mixed_Mpoints_s": r["mixed"]["Mpoints_s"],
                      "fp64_rates_ms": r["fp64"]["rates_ms"],
                      "fp64_transport_ms": r["fp64"]["transport_ms"]})
    res["sweep_syn53"] = sweep
    # the analytical Jacobian d wdot / d C: one 53 x 53 matrix per point, 2^16
    # points (1.47 GB of output per launch)
    log("jacobian syn53 at 2^16 points")
    dm = kx.Mechanism(m53, 0)
    nj = 1 << 16
    (_, T, p, Y), = serve_load.make_pool(dm, 53, [nj], 30)
    out = torch.empty((nj, 53, 53), dtype=torch.float64, device="cuda:0")
    for _ in range(warmup):
        kx.jacobian(dm, T, p, Y, out=out)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        kx.jacobian(dm, T, p, Y, out=out)
    ev[1].record()
    torch.cuda.synchronize()
    jms = ev[0].elapsed_time(ev[1]) / steps
    res["jacobian_syn53_2p16"] = {"n_points": nj, "ms": jms, "Mpoints_s": nj / jms / 1e3,
                                  "output_GB_s": nj * 53 * 53 * 8 / (jms * 1e-3) / 1e9}
    del out, T, p, Y
    dm.close()
    # rates of the 53-species mechanism with 6 QSS species: the QSS balances
    # solved per point before the rates, 2^20 points
    log("qss syn53q at 2^20 points")
    mq = I.make_mechanism(I.MECH_53Q)
    dq = kx.Mechanism(mq, 0)
    nq = 1 << 20
    (_, T, p, Y), = serve_load.make_pool(dq, 53, [nq], 31)
    wq = torch.empty((53, nq), dtype=torch.float64, device="cuda:0")
    for _ in range(warmup):
        kx.production_rates(dq, T, p, Y, out=wq)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        kx.production_rates(dq, T, p, Y, out=wq)
    ev[1].record()
    torch.cuda.synchronize()
    qms = ev[0].elapsed_time(ev[1]) / steps
    res["qss_syn53q_2p20"] = {"n_points": nq, "n_qss": int(dq.n_qss), "rates_ms": qms,
                              "Mpoints_s": nq / qms / 1e3}
    del wq, T, p, Y
    dq.close()
    torch.cuda.empty_cache()
    return res


def cpu_baseline(mech, T, p, Y, target_s=12.0, single_s=3.0):
    """The oracle as it stands, on a bounded sample of the same states (the
    first n points, n chosen for about `target_s` seconds), on all host threads
    and on one.  Returns the baseline and the oracle's outputs on the whole
    sample (for the error report)."""
    import numpy as np
    from oracle import oracle as O
    om = O.OracleMech(mech)
    threads = O.max_threads()
    n0 = 4096
    Y0 = np.ascontiguousarray(Y[:, :n0])
    t0 = time.perf_counter()
    om.production_rates(T[:n0], p[:n0], Y0, with_scale=False)
    om.transport(T[:n0], p[:n0], Y0)
    est = (time.perf_counter() - t0) / n0
    n = int(min(T.size, max(n0, target_s / max(est, 1e-9))))
    Ys = np.ascontiguousarray(Y[:, :n])
    t0 = time.perf_counter()
    ref_w, ref_s = om.production_rates(T[:n], p[:n], Ys)
    ref_t = om.transport(T[:n], p[:n], Ys)
    dt = time.perf_counter() - t0
    del Ys
    # single thread, the paper's per-core comparison basis
    n1 = int(max(256, min(n, single_s * n / dt / max(threads, 1))))
    O.set_threads(1)
    Y1 = np.ascontiguousarray(Y[:, :n1])
    t1 = time.perf_counter()
    om.production_rates(T[:n1], p[:n1], Y1, with_scale=False)
    om.transport(T[:n1], p[:n1], Y1)
    dt1 = time.perf_counter() - t1
    O.set_threads(threads)
    base = {"value": n / dt / 1e6, "unit": "Mpoints/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} points of the same workload, production rates (with the "
                      f"conditioning scale s_k) + transport, {dt:.1f} s on {threads} threads",
            "single_thread": {"value": n1 / dt1 / 1e6, "unit": "Mpoints/s", "cores": 1,
                              "sample": f"first {n1} points, {dt1:.1f} s"}}
    return base, (ref_w, ref_s) + tuple(ref_t)


def error_report(gpu, ref, target):
    """Per-output error of GPU outputs against the oracle.  wdot entries above
    1e-10 max|entry| of their point are judged: the strict relative error (max,
    p99.99, median, the count above `target` and, for those entries, their
    cancellation ratio kappa = s_k / |wdot_k| with s_k = sum_i |nu_ki| |R_i|),
    and the conditioned error |d| / s_k.  Transport outputs by the relative
    error (max, p99.99, median, count above `target`)."""
    import numpy as np
    w, mu, lam, Dm = gpu
    rw, rs, rmu, rlam, rDm = ref
    mask = np.abs(rw) > 1e-10 * np.abs(rw).max(axis=0, keepdims=True)
    aref = np.abs(rw)[mask]
    d = np.abs(w - rw)[mask]
    rel = d / aref
    kappa = rs[mask] / aref
    over = rel > target
    worst = np.argsort(rel)[::-1][:5]
    out = {"points": int(rw.shape[1]), "target": target,
           "wdot": {"judged": int(mask.sum()), "max_rel": float(rel.max()),
                    "p9999_rel": float(np.quantile(rel, 0.9999)),
                    "median_rel": float(np.median(rel)),
                    "n_above_target": int(over.sum()),
                    "max_conditioned": float((d / rs[mask]).max()),
                    "kappa_of_entries_above_target": (
                        {"min": float(kappa[over].min()), "median": float(np.median(kappa[over])),
                         "max": float(kappa[over].max())} if over.any() else None),
                    "kappa_all_entries": {"median": float(np.median(kappa)),
                                          "p9999": float(np.quantile(kappa, 0.9999))},
                    "worst": [{"rel": float(rel[i]), "kappa": float(kappa[i])} for i in worst]}}
    for name, g, r in (("mu", mu, rmu), ("lambda", lam, rlam), ("Dmix", Dm, rDm)):
        e = (np.abs(g - r) / np.abs(r)).ravel()
        out[name] = {"max_rel": float(e.max()), "p9999_rel": float(np.quantile(e, 0.9999)),
                     "median_rel": float(np.median(e)), "n_above_target": int((e > target).sum())}
    return out


def cfg3_mixed(kx, mech, steps, warmup):
    """The mixed-precision workload: 2^22 points of the 53-species mechanism,
    three quarters drawn as the FP64 workload and one quarter within 1e-6 of
    constructed equilibrium states (8192 distinct ones, each repeated 128
    times), randomly interleaved.  Times FP64 and mixed on these states and
    reports the mixed (and FP64) error against the oracle on all 8192 distinct
    near-equilibrium states and a stratified sample of 2^15 bulk points."""
    import numpy as np
    import torch
    from oracle import oracle as O
    from paper_2411_02640_amd import inputs as I
    sspec = I.STATES_53_MIXED
    n = sspec.n_points
    nq = n // 4
    om = O.OracleMech(mech)
    log("cfg3: near-equilibrium states")
    ne = 8192
    Te, pe, Ye = O.equilibrium_states(om, ne, seed=sspec.seed + 1000, perturb=1e-6)
    log("cfg3: bulk states")
    T1, p1, Y1 = I.make_states(53, sspec, n_points=n - nq)
    reps = nq // ne
    T = np.concatenate([T1, np.tile(Te, reps)])
    p = np.concatenate([p1, np.tile(pe, reps)])
    src = np.concatenate([np.arange(n - nq), -1 - np.tile(np.arange(ne), reps)])
    perm = np.random.default_rng(sspec.seed).permutation(n)
    T, p, src = T[perm], p[perm], src[perm]
    Y = np.empty((53, n))
    for k in range(53):
        Y[k] = np.concatenate([Y1[k], np.tile(Ye[k], reps)])[perm]
    del Y1
    ns = 53
    dm = kx.Mechanism(mech, 0)
    Td, pd, Yd = [torch.from_numpy(a).to("cuda:0") for a in (T, p, Y)]
    kw = dict(dtype=torch.float64, device="cuda:0")
    outs = (torch.empty((ns, n), **kw),
            (torch.empty(n, **kw), torch.empty(n, **kw), torch.empty((ns, n), **kw)))
    # sample: the first occurrence of every near-equilibrium state and one
    # bulk point from each of 2^15 strata of the bulk positions
    bulk_pos = np.flatnonzero(src >= 0)
    strata = np.array_split(bulk_pos, 1 << 15)
    rng = np.random.default_rng(sspec.seed + 7)
    bulk_idx = np.array([s[rng.integers(s.size)] for s in strata])
    near_pos = np.flatnonzero(src < 0)
    _, first = np.unique(src[near_pos], return_index=True)
    near_idx = near_pos[first]
    res = {"workload": "syn53, 2^22 points: 3/4 T ~ U[300, 2800] K, p ~ U[1, 40] atm, "
                       "Y ~ Dirichlet(0.3); 1/4 within 1e-6 of 8192 constructed equilibrium "
                       "states (element potentials), randomly interleaved",
           "n_points": n, "state_seed": sspec.seed, "steps": steps}
    sample = {}
    for prec in ("fp64", "mixed"):
        log(f"cfg3: {prec} timing")
        wall, r, t = time_path(kx, dm, Td, pd, Yd, outs, steps, warmup, prec)
        res[prec] = {"Mpoints_s": n * steps / wall / 1e6, "rates_ms": r, "transport_ms": t,
                     "rates_ms_median": time_path.medians[0],
                     "transport_ms_median": time_path.medians[1]}
        w_, (mu_, lam_, Dm_) = outs
        for part, idx in (("bulk", bulk_idx), ("near_equilibrium", near_idx)):
            it = torch.from_numpy(idx).to("cuda:0")
            sample[(prec, part)] = (w_[:, it].cpu().numpy(), mu_[it].cpu().numpy(),
                                    lam_[it].cpu().numpy(), Dm_[:, it].cpu().numpy())
    del outs, Td, pd, Yd
    dm.close()
    torch.cuda.empty_cache()
    res["speedup_mixed_vs_fp64"] = res["mixed"]["Mpoints_s"] / res["fp64"]["Mpoints_s"]
    res["rates_speedup_mixed_vs_fp64"] = res["fp64"]["rates_ms"] / res["mixed"]["rates_ms"]
    res["transport_speedup_mixed_vs_fp64"] = (res["fp64"]["transport_ms"] /
                                              res["mixed"]["transport_ms"])
    log("cfg3: oracle on the sample")
    errors = {}
    for part, idx in (("bulk", bulk_idx), ("near_equilibrium", near_idx)):
        Ts, ps, Ys = T[idx], p[idx], np.ascontiguousarray(Y[:, idx])
        ref_w, ref_s = om.production_rates(Ts, ps, Ys)
        ref = (ref_w, ref_s) + tuple(om.transport(Ts, ps, Ys))
        errors[part] = {"mixed": error_report(sample[("mixed", part)], ref, 1e-5),
                        "fp64": error_report(sample[("fp64", part)], ref, 1e-12)}
    res["error_vs_oracle"] = errors
    res["criterion"] = ("mixed wdot passes when |d| <= 1e-5 s_k on every judged entry "
                        "(conditioned error); the plain relative error is reported beside it")
    return res


def serve_bench(kx, args):
    """Served workload: Poisson stream over the 9-, 53- and 200-species
    mechanisms, n = round(10^U(3,6)), ops and precision 50/50, at fractions of
    the measured back-to-back capacity."""
    import numpy as np
    import torch

    from paper_2411_02640_amd import inputs as I
    from paper_2411_02640_amd import serve_load as SL

    rng = np.random.default_rng(SERVE_SEED)
    mechs, pools = {}, {}
    for spec in (I.MECH_9, I.MECH_53, I.MECH_200):
        mech = I.make_mechanism(spec)
        name = mech["name"]
        mechs[name] = kx.Mechanism(mech, 0)
        sizes = np.rint(10.0 ** rng.uniform(3.0, 6.0, args.serve_pool)).astype(int)
        pools[name] = SL.make_pool(mechs[name], mech["n_species"], sizes,
                                   SERVE_SEED * 1000 + spec.n_species)
    srv = kx.Server(0, hbm_budget=args.serve_budget_gb << 30, max_slots=args.serve_slots)
    try:
        for m in mechs.values():   # resident tables and captured graphs before any request
            srv.add_mech(m)
        nw, nm = args.serve_warmup, args.serve_requests
        # warm every (mechanism, precision, ops) graph on every stream
        SL.run_stream(srv, mechs, pools, SL.make_stream(4 * nw, pools, SERVE_SEED + 1), None, 0)
        cap_stream = SL.make_stream(nm, pools, SERVE_SEED + 2)
        rec = SL.run_stream(srv, mechs, pools, cap_stream, None, 0)
        cap = SL.summarize(rec)
        capacity = cap["achieved_rps"]
        log(f"serve capacity {capacity:.1f} req/s, {cap['achieved_Mpoints_s']:.1f} Mpoints/s")
        seq_s = SL.direct_sequential(mechs, pools, cap_stream)
        levels = []
        for k, frac in enumerate(SERVE_LOADS):
            qps = frac * capacity
            stream = SL.make_stream(nw + nm, pools, SERVE_SEED + 10 + k)
            rec = SL.run_stream(srv, mechs, pools, stream, qps, SERVE_SEED + 20 + k)
            s = SL.summarize(rec, skip=nw)
            s.update({"load": frac, "offered_rps": qps})
            log(f"serve load {frac:.2f}: p50 {s['p50_ms']:.2f} ms p99 {s['p99_ms']:.2f} ms "
                f"{s['achieved_rps']:.1f} req/s")
            levels.append(s)
        # the same service for a client whose data live in pinned host memory:
        # inputs copied in at arrival, outputs copied out before the request
        # counts as finished (latency to outputs on the host)
        log("serving with host staging")
        hpools = {name: SL.make_host_pool(pools[name][:args.serve_staged_pool],
                                          mechs[name].n_species) for name in pools}
        ns_, nw_ = args.serve_staged_requests, max(1, args.serve_staged_requests // 10)
        cap_s = SL.make_stream(ns_, hpools, SERVE_SEED + 40)
        rec = SL.run_stream_staged(srv, mechs, hpools, cap_s, None, 0)
        scap = SL.summarize(rec, end="t_host")
        staged = {"capacity_rps": scap["achieved_rps"],
                  "capacity_Mpoints_s": scap["achieved_Mpoints_s"],
                  "input_sets_per_mechanism": args.serve_staged_pool,
                  "measured_requests": ns_, "warmup_requests": nw_, "levels": []}
        log(f"staged capacity {scap['achieved_rps']:.1f} req/s")
        for k, frac in enumerate((0.5, 0.9)):
            qps = frac * scap["achieved_rps"]
            stream = SL.make_stream(nw_ + ns_, hpools, SERVE_SEED + 50 + k)
            rec = SL.run_stream_staged(srv, mechs, hpools, stream, qps, SERVE_SEED + 60 + k)
            sm = SL.summarize(rec, skip=nw_, end="t_host")
            sm.update({"load": frac, "offered_rps": qps})
            log(f"staged load {frac:.2f}: p50 {sm['p50_ms']:.2f} ms p99 {sm['p99_ms']:.2f} ms")
            staged["levels"].append(sm)
        del hpools
        st = srv.stats()
    finally:
        srv.close()
        for m in mechs.values():
            m.close()
    return {"workload": "Poisson arrivals; mechanism uniform over syn9/syn53/syn200, "
                        "n = round(10^U(3,6)), rates-only vs rates+transport 50/50, "
                        "fp64 vs mixed 50/50; inputs device-resident; latency from "
                        "scheduled arrival to outputs ready on the device",
            "seed": SERVE_SEED, "input_sets_per_mechanism": args.serve_pool,
            "warmup_requests": nw, "measured_requests": nm,
            "hbm_budget_bytes": args.serve_budget_gb << 30, "max_slots": args.serve_slots,
            "capacity_rps": capacity, "capacity_Mpoints_s": cap["achieved_Mpoints_s"],
            "direct_sequential_rps": nm / seq_s,
            "direct_sequential_Mpoints_s": sum(pools[nm_][i][0] for nm_, i, _, _ in cap_stream)
                                           / seq_s / 1e6,
            "levels": levels, "batches": st["batches"], "graph_launches": st["graph_launches"],
            "resident_mechs": st["resident_mechs"], "resident_bytes": st["resident_bytes"],
            "host_staged": dict(staged, workload="the same mix with inputs and outputs in "
                                "pinned host memory: inputs copied to the device at arrival, "
                                "latency to outputs copied back to the host")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prewarm-s", type=float, default=0.5,
                    help="untimed steps for at least this many seconds before the warm-up "
                         "steps of the headline workload (clocks settle)")
    ap.add_argument("--points", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 2^22, syn200 and point-count sweep timings")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB elementwise copy first (counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-pool", type=int, default=24)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-budget-gb", type=int, default=48)
    ap.add_argument("--serve-staged-requests", type=int, default=200)
    ap.add_argument("--serve-staged-pool", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: kx has no multi-GPU path "
              "(points shard trivially across GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_02640_amd import inputs as I
    from paper_2411_02640_amd import kx, opcount

    if args.copy_probe:
        copy_probe(torch)

    spec, sspec = I.MECH_53, I.STATES_53
    log("generating mechanism and states")
    mech = I.make_mechanism(spec)
    T, p, Y = I.make_states(spec.n_species, sspec, n_points=args.points)
    n, ns, nr = int(T.size), int(mech["n_species"]), int(mech["n_reactions"])
    dm = kx.Mechanism(mech, 0)
    Td, pd, Yd = [torch.from_numpy(a).to("cuda:0") for a in (T, p, Y)]
    kw = dict(dtype=torch.float64, device="cuda:0")
    outs = (torch.empty((ns, n), **kw),
            (torch.empty(n, **kw), torch.empty(n, **kw), torch.empty((ns, n), **kw)))

    log(f"fp64: {args.warmup} warmup + {args.steps} timed steps, n = {n}")
    wall, r_ms, t_ms = time_path(kx, dm, Td, pd, Yd, outs, args.steps, args.warmup, "fp64",
                                 prewarm_s=args.prewarm_s)
    r_med, t_med = time_path.medians

    def host(o):  # the outputs on the host (judged against the oracle later)
        w_, (mu_, lam_, Dm_) = o
        return (w_.cpu().numpy(), mu_.cpu().numpy(), lam_.cpu().numpy(), Dm_.cpu().numpy())
    gpu64 = host(outs)
    ms_step = wall / args.steps * 1e3
    value = n * args.steps / wall / 1e6
    log(f"fp64 {value:.1f} Mpoints/s (rates {r_ms:.3f} ms, transport {t_ms:.3f} ms)")

    mixed = None
    if not args.no_mixed:
        log("mixed precision")
        mwall, mr, mt = time_path(kx, dm, Td, pd, Yd, outs, args.steps, args.warmup, "mixed",
                                  prewarm_s=args.prewarm_s)
        gpumx = host(outs)
        mixed = {"value": n * args.steps / mwall / 1e6, "unit": "Mpoints/s",
                 "ms_per_step": mwall / args.steps * 1e3,
                 "rates_kernel_ms": mr, "transport_kernel_ms": mt,
                 "rates_kernel_ms_median": time_path.medians[0],
                 "transport_kernel_ms_median": time_path.medians[1],
                 "speedup_vs_fp64": (n * args.steps / mwall) / (n * args.steps / wall)}
        log(f"mixed {mixed['value']:.1f} Mpoints/s")

    ops = opcount.per_point(mech)
    io = opcount.io_bytes(mech)
    kern = {"rates": (r_ms, ops["rates_flops"], io["rates"]),
            "transport": (t_ms, ops["transport_flops"], io["transport"])}
    # the rates kernel runs on the vector ALUs; the transport kernel's pair sums
    # run on the matrix cores for 1/D_kj tables of 24 or more species.  FP64
    # vector and dense FP64 MFMA peaks are both 78.6 TFLOP/s on MI355X.
    mfma_tr = int(mech["diff_fit_kind"]) == 1 and ns >= 24
    bound = {"rates": "alu", "transport": "mfma" if mfma_tr else "alu"}
    dom = max(kern, key=lambda k: kern[k][0])
    ms, fl, by = kern[dom]
    fl, by = float(fl), float(by)
    achieved = fl * n / (ms * 1e-3) / 1e12
    roofline = {"bound": bound[dom], "kernel": dom, "achieved": achieved,
                "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VALU_PEAK_TFLOPS, "traffic": profiled_traffic(dom),
                "flops_per_point": fl, "points_per_launch": n,
                "hbm_gbs_compulsory": by * n / (ms * 1e-3) / 1e9}
    # the same work with the elementary functions priced at their measured
    # cost on this GPU (the library's own sequences, in FP64 FMA issue time):
    # T_min = flops / peak is the least time the FP64 units need for it
    log("elementary-function prices")
    mp = opcount.measure_prices()
    fl_m = opcount.flops_priced(ops[dom], mp["prices"])
    tmin_ms = fl_m * n / (FP64_VALU_PEAK_TFLOPS * 1e12) * 1e3
    roofline.update({"prices_model": dict(opcount.PRICE), "prices_measured": mp["prices"],
                     "mixed_prices_measured": mp["mixed_prices"],
                     "fma_tflops_measured": mp["fma_tflops_measured"],
                     "price_probe_ms": mp["probe_ms"],
                     "flops_per_point_measured_prices": fl_m, "tmin_ms": tmin_ms,
                     "tmin_frac": tmin_ms / ms})
    log(f"prices {json.dumps(mp['prices'])}; T_min {tmin_ms:.3f} ms = "
        f"{tmin_ms / ms:.3f} of the {dom} kernel time")
    other = [k for k in kern if k != dom][0]
    oms, ofl, oby = kern[other]
    ofl = float(ofl)
    roofline["other_kernel"] = {"kernel": other, "bound": bound[other],
                                "achieved": ofl * n / (oms * 1e-3) / 1e12,
                                "frac": ofl * n / (oms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS,
                                "ms": oms, "traffic": profiled_traffic(other)}
    if other == "transport":
        # the matrix-core work the kernel issues (16x16x4 FP64 tiles over the
        # padded species: ceil(ns/16) row blocks x ceil(ns/4) K-steps x
        # (3 Wilke products + one per fit order) per 16 points), against the
        # rate that instruction sustains on this GPU (probe above)
        ns_ = mech["n_species"]
        mb_, ks_ = -(-ns_ // 16), -(-ns_ // 4)
        mfl = mb_ * ks_ * (3 + int(mech["fit_order"])) * 2048 / 16
        rate = mfl * n / (oms * 1e-3) / 1e12
        peak_m = mp["mfma_tflops_measured"]["f64_16x16x4"]
        roofline["other_kernel"].update({
            "mfma_flops_per_point_issued": mfl, "mfma_tflops_issued": rate,
            "mfma_tflops_measured": mp["mfma_tflops_measured"],
            "mfma_frac_of_measured_16x16x4": rate / peak_m})
        log(f"transport issues {rate:.1f} TFLOP/s of 16x16x4 FP64 MFMA work; the "
            f"instruction sustains {peak_m:.1f} on this GPU ({rate / peak_m:.2f})")

    extra = None
    if not args.no_extra:
        extra = other_workloads(kx, I, torch, args.steps, args.warmup)

    served = None
    if not args.no_serve:
        log("serving")
        served = serve_bench(kx, args)

    cpu = errors = mixed3 = None
    if not args.no_cpu_baseline:
        # the legs that run the oracle: the CPU baseline, the error of both
        # paths on its sample, and the mixed-precision workload's accuracy
        log("cpu baseline (oracle)")
        del Td, pd, Yd, outs
        torch.cuda.empty_cache()
        cpu, ref = cpu_baseline(mech, T, p, Y)
        log(f"oracle {cpu['value']:.4f} Mpoints/s on {cpu['cores']} threads, "
            f"{cpu['single_thread']['value']:.5f} on one")
        ns_ = ref[0].shape[1]
        cut = lambda g: (g[0][:, :ns_], g[1][:ns_], g[2][:ns_], g[3][:, :ns_])
        errors = {"fp64": error_report(cut(gpu64), ref, 1e-12)}
        if mixed is not None:
            errors["mixed"] = error_report(cut(gpumx), ref, 1e-5)
        del ref, gpu64
        log("errors vs oracle", json.dumps(errors))
        if not args.no_mixed:
            mixed3 = cfg3_mixed(kx, mech, args.steps, args.warmup)
            log("cfg3", json.dumps({k: mixed3[k] for k in ("fp64", "mixed")}))

    line = {
        "metric": "Mpoints/s wdot+transport (53 sp) FP64 vs mixed; served p50/p99 latency",
        "value": value, "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "prewarm_s": args.prewarm_s, "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "syn53 mechanism (53 species, 325 reactions: 266 elementary, "
                               "30 three-body, 29 Troe), 2^20 points, p 1-40 atm, "
                               "Y ~ Dirichlet(0.3)",
                   "n_points": n, "n_species": ns, "n_reactions": nr,
                   "mechanism_seed": spec.seed, "state_seed": sspec.seed},
        "grxn_per_s": value * 1e6 * nr / 1e9,
        "gdof_per_s": value * 1e6 * (ns + 2) / 1e9,
        "rates_kernel_ms": r_ms, "transport_kernel_ms": t_ms,
        "rates_kernel_ms_median": r_med, "transport_kernel_ms_median": t_med,
        "error_vs_oracle": errors,
        "roofline": roofline, "cpu_baseline": cpu, "mixed": mixed,
        "mixed_workload_2p22": mixed3, "served": served,
        "other_workloads": extra,
    }
    print(json.dumps(line), flush=True)
    dm.close()


if __name__ == "__main__":
    main()
