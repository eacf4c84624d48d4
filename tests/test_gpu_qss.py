"""Parity of the QSS path (kx_production_rates / kx_qss_concentrations on a
mechanism with quasi-steady species) with the FP64 CPU oracle.

Tolerances.  The GPU assembles A and b of the QSS balances from the reaction
terms and eliminates without row exchanges; the oracle takes A and b from
re-evaluations of the plain rates and eliminates with partial pivoting.  Each
entry of A and b is a sum of reaction terms, and a term of two correct FP64
evaluations differs by at most EPS_TERM relative (the exponential arguments,
see tests/parity.py).  A relative perturbation e of the entries moves unknown
i by at most cond_i * e relative, cond_i = (|A^-1| (|A| |x| + |b|))_i / |x_i|
being its componentwise (Skeel) condition, computed from the oracle's system;
both eliminations are backward stable (the columns of A are weakly diagonally
dominant) and add only a few n_qss u on top.  So the test allows
EPS_TERM * cond_i on C_Q.  cond_i is below 10 at most points but reaches ~1e6
where two QSS species exchange fast and drain slowly (a nearly closed
sub-system).  The transported rates inherit the error of C_Q on the terms that
carry a QSS factor, so their conditioned bound per point is the largest
allowance of that point's unknowns (at least EPS_TERM).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_02640_amd import inputs as I

from . import parity as PM
from . import tiny_mechs as TM

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
U = 2.0 ** -53


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kx():
    from paper_2411_02640_amd import kx as K
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    K.lib()
    return K


def to_dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV) for a in arrs]


def run_qss(kx, dm, T, p, Y):
    Td, pd, Yd = to_dev(T, p, Y)
    w = kx.production_rates(dm, Td, pd, Yd)
    Cq = kx.qss_concentrations(dm, Td, pd, Yd)
    torch.cuda.synchronize()
    return w.cpu().numpy(), Cq.cpu().numpy()


def qss_condition(om, T, p, Y, Cq):
    """cond[nq, n]: componentwise condition of each QSS unknown (see above)."""
    cond = np.empty_like(Cq)
    for i in range(T.size):
        A, b = om.qss_system(T[i], p[i], Y[:, i])
        x = Cq[:, i]
        cond[:, i] = (np.abs(np.linalg.inv(A)) @ (np.abs(A) @ np.abs(x) + np.abs(b))) / np.abs(x)
    return cond


def compare(mech, w, Cq, T, p, Y, label):
    om = O.OracleMech(mech)
    ref, s, rCq = om.qss_rates(T, p, Y)
    q = np.flatnonzero(mech["qss"])
    tr = np.flatnonzero(mech["qss"] == 0)
    assert np.isfinite(Cq).all() and np.isfinite(w).all()
    cond = qss_condition(om, T, p, Y, rCq)
    allow = PM.EPS_TERM * np.maximum(cond, 1.0)
    cq_rel = np.abs(Cq - rCq) / np.abs(rCq)
    _say("  ", label, "C_Q max rel", float(cq_rel.max()), "median", float(np.median(cq_rel)),
         "| cond max", float(cond.max()), "median", float(np.median(cond)),
         "| max rel / (u cond)", float((cq_rel / (U * np.maximum(cond, 1.0))).max()))
    assert (cq_rel <= allow).all(), float((cq_rel / allow).max())
    assert (w[q] == 0.0).all()
    # transported rates: the plain-rates bound, with the per-point allowance of
    # the QSS unknowns on the terms that carry them
    gw, rw, sw = w[tr], ref[tr], s[tr]
    eps = np.maximum(PM.EPS_TERM, allow.max(axis=0, keepdims=True))
    mask = np.abs(rw) > 1e-10 * np.abs(rw).max(axis=0, keepdims=True)
    d = np.abs(gw - rw)
    bad = (d > PM.REL_FP64 * np.abs(rw) + eps * sw) & mask
    cond_rel = np.where(mask, d / np.where(sw > 0, sw, 1.0), 0.0)
    _say("  ", label, "wdot judged", int(mask.sum()), "failing", int(bad.sum()),
         "max conditioned", float(cond_rel.max()),
         "max conditioned / allowance", float((cond_rel / eps).max()))
    assert not bad.any()


@pytest.mark.parametrize("qss", [(TM.Q1_, TM.Q2_), (TM.Q1_,)])
def test_qss_chain(kx, qss):
    """The hand-solvable chain mechanism (two coupled QSS species, or one),
    1027 points: every point against the oracle."""
    mech = TM.qss_chain_mechanism(qss)
    T, p, Y = I.make_states(5, I.StateSpec(1027, seed=81, p_atm_range=(0.2, 40.0),
                                           dirichlet_alpha=1.0))
    _say("qss chain", qss, "n =", T.size)
    dm = kx.Mechanism(mech, 0)
    w, Cq = run_qss(kx, dm, T, p, Y)
    compare(mech, w, Cq, T, p, Y, "chain")
    dm.close()


def test_qss_nine_species_lds_path(kx):
    """Nine coupled QSS species (9 x 10 entries of [A | b] exceed one wave, so
    the system is solved in LDS rather than in registers), 517 points."""
    mech = TM.qss_long_chain(9)
    T, p, Y = I.make_states(12, I.StateSpec(517, seed=88, p_atm_range=(0.2, 40.0),
                                            dirichlet_alpha=1.0))
    _say("qss long chain nq = 9, n =", T.size)
    dm = kx.Mechanism(mech, 0)
    w, Cq = run_qss(kx, dm, T, p, Y)
    compare(mech, w, Cq, T, p, Y, "long chain")
    dm.close()


def test_qss_syn200q(kx, mech200q):
    """200 species with 12 QSS species: eight reaction chunks and the LDS
    elimination (12 x 13 entries exceed one wave), 263 points."""
    T, p, Y = I.make_states(200, I.StateSpec(263, seed=89, p_atm_range=(1.0, 40.0),
                                             dirichlet_alpha=0.3))
    _say("qss syn200q n =", T.size)
    dm = kx.Mechanism(mech200q, 0)
    w, Cq = run_qss(kx, dm, T, p, Y)
    compare(mech200q, w, Cq, T, p, Y, "syn200q")
    dm.close()


def test_qss_syn53q_block(kx, mech53q):
    """53 species with 6 QSS species, 4133 points (every point judged)."""
    T, p, Y = I.make_states(53, I.StateSpec(4133, seed=82, p_atm_range=(1.0, 40.0),
                                            dirichlet_alpha=0.3))
    _say("qss syn53q n =", T.size)
    dm = kx.Mechanism(mech53q, 0)
    w, Cq = run_qss(kx, dm, T, p, Y)
    compare(mech53q, w, Cq, T, p, Y, "syn53q")
    dm.close()


def test_qss_further_forms(kx, mech53xq):
    """QSS species in SRI and pressure-table reactions (syn53x with 6 QSS
    species), 1031 points at 0.05-150 atm (below, inside and above the tables)."""
    T, p, Y = I.make_states(53, I.StateSpec(1031, seed=87, p_atm_range=(0.05, 150.0),
                                            dirichlet_alpha=0.3))
    _say("qss syn53xq n =", T.size)
    dm = kx.Mechanism(mech53xq, 0)
    w, Cq = run_qss(kx, dm, T, p, Y)
    compare(mech53xq, w, Cq, T, p, Y, "syn53xq")
    dm.close()


def test_qss_full_size_sampled(kx, mech53q):
    """The 2^20-point workload in the launch configuration the benchmark times
    (the grid strides over points); the oracle checks a sample."""
    T, p, Y = I.make_states(53, I.STATES_53)
    n = T.size
    _say("qss full size syn53q n =", n)
    dm = kx.Mechanism(mech53q, 0)
    w, Cq = run_qss(kx, dm, T, p, Y)
    rng = np.random.default_rng(83)
    idx = np.unique(np.concatenate([rng.choice(n, 800, replace=False),
                                    [0, 1, 32767, 32768, n - 1]]))
    compare(mech53q, w[:, idx], Cq[:, idx], T[idx], p[idx], np.ascontiguousarray(Y[:, idx]),
            "syn53q sampled")
    dm.close()


def test_qss_inputs_not_read_and_deterministic(kx, mech53q):
    """QSS entries of Y change nothing; two launches agree bit for bit; n = 1
    and n = 0 work."""
    T, p, Y = I.make_states(53, I.StateSpec(700, seed=84, p_atm_range=(1.0, 40.0),
                                            dirichlet_alpha=0.3))
    dm = kx.Mechanism(mech53q, 0)
    w1, c1 = run_qss(kx, dm, T, p, Y)
    Y2 = Y.copy()
    q = np.flatnonzero(mech53q["qss"])
    Y2[q] = np.random.default_rng(3).uniform(0.0, 0.5, (len(q), T.size))
    w2, c2 = run_qss(kx, dm, T, p, Y2)
    np.testing.assert_array_equal(w1, w2)
    np.testing.assert_array_equal(c1, c2)
    w3, c3 = run_qss(kx, dm, T[:1], p[:1], np.ascontiguousarray(Y[:, :1]))
    np.testing.assert_array_equal(w3[:, 0], w1[:, 0])
    np.testing.assert_array_equal(c3[:, 0], c1[:, 0])
    e = torch.empty((53, 0), dtype=torch.float64, device=DEV)
    kx.production_rates(dm, torch.empty(0, dtype=torch.float64, device=DEV),
                        torch.empty(0, dtype=torch.float64, device=DEV), e)
    dm.close()


def test_qss_unsupported_calls(kx, mech53q, mech9):
    """Mixed precision, the Jacobian and the request server refuse a QSS
    mechanism; the concentration call refuses a mechanism without QSS species."""
    dm = kx.Mechanism(mech53q, 0)
    T, p, Y = to_dev(*I.make_states(53, I.StateSpec(16, seed=85)))
    for call in (lambda: kx.production_rates(dm, T, p, Y, precision="mixed"),
                 lambda: kx.jacobian(dm, T, p, Y)):
        with pytest.raises(kx.KxError) as ei:
            call()
        assert ei.value.code == kx.KX_EUNSUPPORTED
    srv = kx.Server(0, hbm_budget=1 << 26, max_slots=4)
    with pytest.raises(kx.KxError) as ei:
        srv.submit(dm, T, p, Y)
    assert ei.value.code == kx.KX_EUNSUPPORTED
    srv.close()
    d9 = kx.Mechanism(mech9, 0)
    T9, p9, Y9 = to_dev(*I.make_states(9, I.StateSpec(8, seed=86)))
    d9.n_qss = 0
    with pytest.raises(kx.KxError) as ei:
        kx.qss_concentrations(d9, T9, p9, Y9)
    assert ei.value.code == kx.KX_EINVAL
    d9.close()
    dm.close()
