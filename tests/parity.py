"""Comparison metrics between the HIP path and the oracle.

wdot (signed sums over reactions): an entry passes when
    |gpu - ref| <= REL * |ref| + EPS_TERM * (s - |ref|)
where s = sum_i |nu_ki| |c_i| (|q_f,i| + |q_r,i|) is the oracle's magnitude of
the terms that cancel into wdot_k (s >= |ref|; s = |ref| without
cancellation, where the bound is the plain relative 1e-12).  EPS_TERM bounds
the relative difference of one term between two correct FP64 evaluations:
each term is a product of up to ~8 exponentials whose arguments reach
|x| ~ 150 for these mechanisms, and rounding the argument changes exp(x) by
|x| u, so 8 * 150 * 2^-53 ~ 1.3e-13 per evaluation, doubled for two
independent evaluations.  Only entries above 1e-10 max|entry| of their point
are judged (per point, per output field); every entry must be finite.

Transport outputs are sums of positive terms and are judged by the plain
relative error.
"""
import numpy as np

REL_FP64 = 1e-12
EPS_TERM = 3e-13
REL_MIXED = 1e-5


def _mask(ref):
    thr = 1e-10 * np.abs(ref).max(axis=0, keepdims=True)
    return np.abs(ref) > thr


def wdot_report(gpu, ref, scale, rel=REL_FP64, eps=EPS_TERM):
    gpu = np.asarray(gpu)
    assert np.isfinite(gpu).all(), "non-finite wdot from the GPU"
    mask = _mask(ref)
    d = np.abs(gpu - ref)
    aref = np.abs(ref)
    tol = rel * aref + eps * np.maximum(scale - aref, 0.0)
    bad = (d > tol) & mask
    strict = np.where(mask, d / np.where(aref > 0, aref, 1.0), 0.0)
    cond = np.where(mask, d / np.where(scale > 0, scale, 1.0), 0.0)
    sm = strict[mask]
    return {
        "ok": not bad.any(),
        "n_judged": int(mask.sum()),
        "n_fail": int(bad.sum()),
        "max_strict_rel": float(sm.max()) if sm.size else 0.0,
        "p9999_strict_rel": float(np.quantile(sm, 0.9999)) if sm.size else 0.0,
        "median_strict_rel": float(np.median(sm)) if sm.size else 0.0,
        "n_strict_above_rel": int((sm > rel).sum()),
        "max_conditioned_rel": float(cond[mask].max()) if sm.size else 0.0,
    }


def mixed_wdot_report(gpu, ref, scale, target=REL_MIXED):
    """Mixed path: conditioned error |gpu - ref| / s must stay below target."""
    r = wdot_report(gpu, ref, scale, rel=target, eps=target)
    return r


def rel_report(gpu, ref, rel):
    gpu = np.asarray(gpu)
    assert np.isfinite(gpu).all(), "non-finite transport output from the GPU"
    mask = _mask(ref)
    e = np.where(mask, np.abs(gpu - ref) / np.where(np.abs(ref) > 0, np.abs(ref), 1.0), 0.0)
    em = e[mask]
    return {
        "ok": bool((em <= rel).all()),
        "max_rel": float(em.max()) if em.size else 0.0,
        "p9999_rel": float(np.quantile(em, 0.9999)) if em.size else 0.0,
        "median_rel": float(np.median(em)) if em.size else 0.0,
        "n_fail": int((em > rel).sum()),
    }
