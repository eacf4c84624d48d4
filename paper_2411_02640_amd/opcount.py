"""Algorithmic FP64 work per grid point, counted from a mechanism.

The count follows the method as the library evaluates it (App. A of the
paper with the per-species Gibbs exponentials for K_c and the beta = E_R = 0
shortcut of eq:k_f), one term per arithmetic operation the formulas need:
add / sub / mul = 1 flop, fused multiply-add = 2 flops, and each elementary
function priced at the flops of a plain FP64 polynomial implementation
(range reduction + minimax polynomial + reconstruction).  The prices are the
model's, stated here so that the roofline fraction can be reproduced:

    exp, exp10: 24    log, log10: 24    division, reciprocal: 8
    sqrt, 1/sqrt: 8

`measure_prices` measures the same classes on the GPU as the library
evaluates them (its exponential, logarithm, reciprocal and reciprocal square
root sequences), in FP64 FMA issue time; with those prices the count gives
T_min = flops / peak, the least time the FP64 vector units need for the
work the method requires.

Counts are per point; a launch processes n points.
"""
from __future__ import annotations

import numpy as np

PRICE = {"exp": 24, "log": 24, "div": 8, "sqrt": 8}

# Probe ops of libkx_micro.so (kx_micro.hip) by price class; a division is the
# library's reciprocal times the numerator, a square root its reciprocal
# square root times the argument (one more multiply each).
_PROBE = {"add": 0, "fma": 1, "exp": 2, "log": 3, "rcp": 4, "rsqrt": 5, "exp_mixed": 6,
          "exp32": 7, "rcp32": 8, "fma32": 9}
# matrix-core probes: op and flops per instruction
_MFMA_PROBE = {"f64_16x16x4": (10, 2048), "f64_4x4x4_4b": (11, 512),
               "f32_16x16x4": (12, 2048), "f32_32x32x2": (13, 4096)}


def measure_prices(iters: int = 400, blocks: int = 256 * 16, reps: int = 5) -> dict:
    """Price of each elementary function as the library evaluates it on this
    GPU, in flops (the issue time of FP64 FMAs, 2 flops each): every probe
    advances eight independent values per lane through one operation and one
    bookkeeping add on a grid filling every SIMD; the add alone is timed and
    subtracted, and the time of the FMA probe is the unit.  Needs a GPU and
    libkx_micro.so."""
    import ctypes
    import os

    import torch
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkx_micro.so")
    if not os.path.exists(path):
        raise RuntimeError("libkx_micro.so is not built (python -m paper_2411_02640_amd.build)")
    lib = ctypes.CDLL(path)
    lib.kx_micro_time.restype = ctypes.c_int
    lib.kx_micro_time.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda:0")
    ms = {}
    for name, op in _PROBE.items():
        t = ctypes.c_double()
        rc = lib.kx_micro_time(op, iters, blocks, reps, ctypes.c_void_p(out.data_ptr()),
                               ctypes.byref(t))
        if rc != 0:
            raise RuntimeError(f"kx_micro_time({name}) failed: {rc}")
        ms[name] = t.value
    torch.cuda.synchronize()
    # an FP64 add issues like an FMA: the add probe is one bookkeeping add per
    # step, the other FP64 probes are one operation + that add per step
    unit = ms["fma"]
    fl = lambda k: 2.0 * (ms[k] - ms["add"]) / unit
    prices = {"exp": fl("exp"), "log": fl("log"), "div": fl("rcp") + 1.0,
              "sqrt": fl("rsqrt") + 1.0}
    # FP32 probes: one operation + one FP32 add per step; an FP32 FMA issues
    # like an FP64 one on gfx950 (packed FP32 is not used)
    fl32 = lambda k: 2.0 * (ms[k] - ms["fma32"]) / unit
    mixed = {"exp_mixed": fl("exp_mixed"), "exp32": fl32("exp32"), "div32": fl32("rcp32") + 1.0,
             "fma32": 2.0 * ms["fma32"] / unit}
    # achieved FP64 FMA rate of the probe (a check of the 78.6 TFLOP/s peak)
    n_fma = blocks * 256 * iters * 8
    rate = 2.0 * n_fma / (ms["fma"] * 1e-3) / 1e12
    # sustained rates of the matrix-core instructions (eight independent
    # accumulators per wave, one MFMA each per step)
    mfma = {}
    for name, (op, flops) in _MFMA_PROBE.items():
        t = ctypes.c_double()
        rc = lib.kx_micro_time(op, iters, blocks, reps, ctypes.c_void_p(out.data_ptr()),
                               ctypes.byref(t))
        if rc != 0:
            raise RuntimeError(f"kx_micro_time({name}) failed: {rc}")
        ms[name] = t.value
        waves = blocks * 256 // 64
        mfma[name] = flops * 8.0 * iters * waves / (t.value * 1e-3) / 1e12
    torch.cuda.synchronize()
    return {"prices": prices, "mixed_prices": mixed, "probe_ms": ms,
            "fma_tflops_measured": rate, "mfma_tflops_measured": mfma}


def flops_priced(counts: dict, prices: dict) -> float:
    """flops of a count with the given prices of the elementary functions."""
    return (2 * counts["fma"] + counts["mul"] + counts["add"]
            + prices["exp"] * counts["exp"] + prices["log"] * counts["log"]
            + prices["div"] * counts["div"] + prices["sqrt"] * counts["sqrt"])


def rates_ops(mech: dict) -> dict:
    ns, nr = mech["n_species"], mech["n_reactions"]
    t = mech["rxn_type"]
    kfconst = (mech["beta"] == 0) & (mech["Ea"] == 0) & (t != 5)
    plog_ptr = mech.get("plog_ptr")
    c = dict(fma=0, mul=0, add=0, exp=0, log=0, div=0, sqrt=0)
    # mixture basics: sum Y/W (fma), C_k (2 mul), one division; ln T, 1/T
    c["fma"] += ns
    c["mul"] += 2 * ns
    c["div"] += 2
    c["log"] += 1
    # species Gibbs (6 fma), exp, a_k (mul), b_k (div)
    c["fma"] += 6 * ns
    c["exp"] += ns
    c["mul"] += ns
    c["div"] += ns
    for i in range(nr):
        r = slice(mech["reac_ptr"][i], mech["reac_ptr"][i + 1])
        p = slice(mech["prod_ptr"][i], mech["prod_ptr"][i + 1])
        if not kfconst[i]:
            c["fma"] += 2
            c["exp"] += 1
        nu_r = int(mech["reac_nu"][r].sum())
        nu_p = int(mech["prod_nu"][p].sum())
        c["mul"] += 2 * nu_r + nu_p + 3      # A', B', B'', c * kf * A' * bracket
        c["add"] += 1                        # bracket
        if t[i] == 5:  # pressure table: two Arrhenius exponents and a lerp in ln p
            if plog_ptr[i + 1] - plog_ptr[i] > 1:
                c["fma"] += 3
                c["mul"] += 1
                c["add"] += 2
        if t[i] in (1, 2, 3, 4):
            ne = mech["eff_ptr"][i + 1] - mech["eff_ptr"][i]
            c["mul"] += 1 + ne
            c["fma"] += ne
        if t[i] in (2, 3, 4):
            c["fma"] += 2
            c["exp"] += 1
            c["mul"] += 2
            c["div"] += 2
            c["add"] += 1
        if t[i] == 4:  # SRI: two exps, a log and the final exp
            c["exp"] += 3
            c["log"] += 1
            c["fma"] += 4
            c["mul"] += 3
            c["div"] += 1
        if t[i] == 3:
            c["exp"] += 3 if not np.isnan(mech["troe"][i, 3]) else 2
            c["log"] += 2
            c["exp"] += 1                    # 10^x
            c["fma"] += 4
            c["mul"] += 3
            c["add"] += 3
            c["div"] += 1
    # stoichiometric accumulation: one fma per non-zero nu_ki
    nnz = 0
    for i in range(nr):
        sp = {}
        for e in range(mech["reac_ptr"][i], mech["reac_ptr"][i + 1]):
            sp[mech["reac_sp"][e]] = sp.get(mech["reac_sp"][e], 0) - mech["reac_nu"][e]
        for e in range(mech["prod_ptr"][i], mech["prod_ptr"][i + 1]):
            sp[mech["prod_sp"][e]] = sp.get(mech["prod_sp"][e], 0) + mech["prod_nu"][e]
        nnz += sum(1 for v in sp.values() if v != 0)
    c["fma"] += nnz
    return c


def transport_ops(mech: dict) -> dict:
    ns, order = mech["n_species"], mech["fit_order"]
    c = dict(fma=0, mul=0, add=0, exp=0, log=0, div=0, sqrt=0)
    c["log"] += 1
    c["fma"] += 1 + ns                       # u, sum Y/W
    c["div"] += 1
    c["mul"] += 2 * ns                       # X_k
    # lambda_k fits, Mathur sums
    c["fma"] += ns * (order - 1) + 2 * ns
    c["div"] += ns + 2
    c["add"] += 1
    # eta_k fits, sqrt / 1/sqrt, Wilke: 3 fma per ordered pair (k, j)
    c["fma"] += ns * (order - 1)
    c["sqrt"] += 2 * ns
    c["mul"] += 2 * ns
    c["fma"] += 3 * ns * ns
    c["fma"] += 2 * ns
    c["div"] += ns
    c["fma"] += ns
    # fits for k != j (full matrix) and the accumulation of X_j / D_kj: with
    # fits of 1/D_kj (kind 1, the paper's form) the fit value multiplies X_j
    # directly; with fits of D_kj (kind 0) a division per pair is needed
    npair = ns * (ns - 1)
    c["fma"] += npair * (order - 1)
    if int(mech.get("diff_fit_kind", 0)) == 1:
        c["fma"] += npair
    else:
        c["div"] += npair
        c["add"] += npair
    c["div"] += 2 * ns
    c["fma"] += 2 * ns
    c["mul"] += ns
    return c


def flops(counts: dict) -> int:
    return (2 * counts["fma"] + counts["mul"] + counts["add"]
            + PRICE["exp"] * counts["exp"] + PRICE["log"] * counts["log"]
            + PRICE["div"] * counts["div"] + PRICE["sqrt"] * counts["sqrt"])


def per_point(mech: dict) -> dict:
    r = rates_ops(mech)
    t = transport_ops(mech)
    return {"rates": r, "transport": t, "rates_flops": flops(r), "transport_flops": flops(t)}


def io_bytes(mech: dict) -> dict:
    """Compulsory HBM bytes per point (inputs read once, outputs written once)."""
    ns = mech["n_species"]
    return {"rates": 8 * (2 * ns + 2), "transport": 8 * (2 * ns + 4),
            "fused": 8 * (3 * ns + 4)}
