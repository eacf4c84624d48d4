"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle."""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_02640_amd import inputs as I

from . import parity as PM

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kx():
    from paper_2411_02640_amd import kx as K
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    K.lib()
    return K


_dev_mechs = {}


def dev_mech(kx, mech):
    key = id(mech)
    if key not in _dev_mechs:
        _dev_mechs[key] = (kx.Mechanism(mech, 0), mech)
    return _dev_mechs[key][0]


def to_dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV) for a in arrs]


def run_rates(kx, dm, T, p, Y, precision="fp64"):
    Td, pd, Yd = to_dev(T, p, Y)
    w = kx.production_rates(dm, Td, pd, Yd, precision=precision)
    torch.cuda.synchronize()
    return w.cpu().numpy()


def run_transport(kx, dm, T, p, Y, precision="fp64"):
    Td, pd, Yd = to_dev(T, p, Y)
    mu, lam, Dm = kx.transport(dm, Td, pd, Yd, precision=precision)
    torch.cuda.synchronize()
    return mu.cpu().numpy(), lam.cpu().numpy(), Dm.cpu().numpy()


def check_rates(kx, mech, T, p, Y, label):
    _say("rates fp64", label, mech["name"], "n =", T.size)
    dm = dev_mech(kx, mech)
    w = run_rates(kx, dm, T, p, Y)
    ref, s = O.OracleMech(mech).production_rates(T, p, Y)
    r = PM.wdot_report(w, ref, s)
    _say("  ", r)
    assert r["ok"], r
    return w


def check_transport(kx, mech, T, p, Y, label):
    _say("transport fp64", label, mech["name"], "n =", T.size)
    dm = dev_mech(kx, mech)
    mu, lam, Dm = run_transport(kx, dm, T, p, Y)
    rmu, rlam, rDm = O.OracleMech(mech).transport(T, p, Y)
    for name, g, r in (("mu", mu, rmu), ("lambda", lam, rlam), ("Dmix", Dm, rDm)):
        rep = PM.rel_report(g, r, PM.REL_FP64)
        _say("  ", name, rep)
        assert rep["ok"], (name, rep)


# ------------------------------------------------------------------ FP64 parity
def test_syn9_all_points(kx, mech9):
    T, p, Y = I.make_states(9, I.STATES_9)
    check_rates(kx, mech9, T, p, Y, "4096 points")
    check_transport(kx, mech9, T, p, Y, "4096 points")


def test_syn9_ragged_tail(kx, mech9):
    T, p, Y = I.make_states(9, I.StateSpec(4096 + 37, seed=21))
    check_rates(kx, mech9, T, p, Y, "4133 points")
    check_transport(kx, mech9, T, p, Y, "4133 points")


def test_syn53_block(kx, mech53):
    T, p, Y = I.make_states(53, I.STATES_53, n_points=(1 << 14) + 5)
    check_rates(kx, mech53, T, p, Y, "16389 points")
    check_transport(kx, mech53, T, p, Y, "16389 points")


def test_syn53_full_size_all_points(kx, mech53):
    """The 2^20-point workload in the launch configuration the benchmark times,
    every point judged against the oracle (rates and transport)."""
    T, p, Y = I.make_states(53, I.STATES_53)
    n = T.size
    dm = dev_mech(kx, mech53)
    _say("full size syn53 n =", n)
    w = run_rates(kx, dm, T, p, Y)
    mu, lam, Dm = run_transport(kx, dm, T, p, Y)
    om = O.OracleMech(mech53)
    ref, s = om.production_rates(T, p, Y)
    r = PM.wdot_report(w, ref, s)
    _say("  wdot", r)
    assert r["ok"], r
    del ref, s, w
    rmu, rlam, rDm = om.transport(T, p, Y)
    for name, g, rr in (("mu", mu, rmu), ("lambda", lam, rlam), ("Dmix", Dm, rDm)):
        rep = PM.rel_report(g, rr, PM.REL_FP64)
        _say("  ", name, rep)
        assert rep["ok"], (name, rep)


def _stratified(n, m, seed):
    """One point from each of m equal strata of consecutive points (every tile
    region and, the states being i.i.d., the whole state distribution)."""
    w = n // m
    rng = np.random.default_rng(seed)
    return np.arange(m) * w + rng.integers(0, w, m)


def test_syn200_full_size_stratified(kx, mech200):
    """The 200-species workload at 2^20 points, FP64 and mixed, in the launch
    configuration the benchmark times; a stratified subset of 2^16 points is
    judged against the oracle (one oracle evaluation serves both precisions)."""
    T, p, Y = I.make_states(200, I.STATES_200)
    n = T.size
    dm = dev_mech(kx, mech200)
    idx = _stratified(n, 1 << 16, 17)
    it = torch.from_numpy(idx).to(DEV)
    Td, pd, Yd = to_dev(T, p, Y)
    Ts, ps, Ys = T[idx], p[idx], np.ascontiguousarray(Y[:, idx])
    del Y
    om = O.OracleMech(mech200)
    _say("syn200 oracle on", idx.size, "points")
    ref, s = om.production_rates(Ts, ps, Ys)
    rmu, rlam, rDm = om.transport(Ts, ps, Ys)
    for prec in ("fp64", "mixed"):
        _say("syn200 full size", prec, "n =", n)
        w = kx.production_rates(dm, Td, pd, Yd, precision=prec)[:, it].cpu().numpy()
        mu, lam, Dm = kx.transport(dm, Td, pd, Yd, precision=prec)
        mu, lam, Dm = mu[it].cpu().numpy(), lam[it].cpu().numpy(), Dm[:, it].cpu().numpy()
        torch.cuda.synchronize()
        if prec == "fp64":
            r = PM.wdot_report(w, ref, s)
        else:
            r = PM.mixed_wdot_report(w, ref, s)
        _say("  wdot", prec, r)
        assert r["ok"], (prec, r)
        tol = PM.REL_FP64 if prec == "fp64" else PM.REL_MIXED
        for name, g, rr in (("mu", mu, rmu), ("lambda", lam, rlam), ("Dmix", Dm, rDm)):
            rep = PM.rel_report(g, rr, tol)
            _say("  ", name, prec, rep)
            assert rep["ok"], (name, prec, rep)


def test_syn100_two_species_per_lane(kx, mech100):
    """100 species / 700 reactions: the rates kernel with two species per lane
    and the 32-point matrix-core transport tile (the 65-128-species band), FP64
    and mixed, with a ragged tail; the Jacobian with two waves per point."""
    T, p, Y = I.make_states(100, I.StateSpec((1 << 13) + 13, seed=71, p_atm_range=(1.0, 40.0),
                                             dirichlet_alpha=0.3))
    check_rates(kx, mech100, T, p, Y, "syn100")
    check_transport(kx, mech100, T, p, Y, "syn100")
    dm = dev_mech(kx, mech100)
    om = O.OracleMech(mech100)
    ref, s = om.production_rates(T, p, Y)
    w = run_rates(kx, dm, T, p, Y, precision="mixed")
    r = PM.mixed_wdot_report(w, ref, s)
    _say("  mixed wdot", r)
    assert r["ok"], r
    mu, lam, Dm = run_transport(kx, dm, T, p, Y, precision="mixed")
    rmu, rlam, rDm = om.transport(T, p, Y)
    for name, g, rr in (("mu", mu, rmu), ("lambda", lam, rlam), ("Dmix", Dm, rDm)):
        rep = PM.rel_report(g, rr, PM.REL_MIXED)
        _say("  mixed", name, rep)
        assert rep["ok"], (name, rep)
    Te, pe, Ye = O.equilibrium_states(om, 512, seed=73, perturb=1e-6)
    check_rates(kx, mech100, Te, pe, Ye, "syn100 near equilibrium")
    _check_jacobian(kx, mech100, T[:131], p[:131], np.ascontiguousarray(Y[:, :131]), "syn100")


def test_three_molecule_sides(kx):
    """Reactions with three molecules on a side (AB + A <=> B + 2 A, and the
    explicit-order and every-form reactions of the four-species mechanisms):
    the rates kernel's third molecule slot, FP64 and mixed, at every point of
    4096 plus a ragged tail, at 0.05-50 atm."""
    from . import tiny_mechs as TM
    for mech, seed in ((TM.abx_mechanism(), 81), (TM.all_forms_mechanism(), 82)):
        nr = mech["n_reactions"]
        sides = [int(mech["reac_nu"][mech["reac_ptr"][i]:mech["reac_ptr"][i + 1]].sum())
                 for i in range(nr)] + \
                [int(mech["prod_nu"][mech["prod_ptr"][i]:mech["prod_ptr"][i + 1]].sum())
                 for i in range(nr)]
        assert max(sides) == 3
        mech = dict(mech, name="tiny%d" % seed)
        T, p, Y = I.make_states(4, I.StateSpec(4096 + 29, seed=seed, p_atm_range=(0.05, 50.0),
                                               dirichlet_alpha=1.0))
        check_rates(kx, mech, T, p, Y, "three-molecule side")
        dm = dev_mech(kx, mech)
        w = run_rates(kx, dm, T, p, Y, precision="mixed")
        ref, s = O.OracleMech(mech).production_rates(T, p, Y)
        r = PM.mixed_wdot_report(w, ref, s)
        _say("  mixed", r)
        assert r["ok"], r


def test_syn200_sampled(kx, mech200):
    T, p, Y = I.make_states(200, I.STATES_200, n_points=(1 << 14) + 3)
    dm = dev_mech(kx, mech200)
    _say("syn200 n =", T.size)
    w = run_rates(kx, dm, T, p, Y)
    mu, lam, Dm = run_transport(kx, dm, T, p, Y)
    idx = np.unique(np.concatenate([np.arange(0, T.size, 61), [T.size - 1]]))
    Ts, ps, Ys = T[idx], p[idx], np.ascontiguousarray(Y[:, idx])
    om = O.OracleMech(mech200)
    ref, s = om.production_rates(Ts, ps, Ys)
    r = PM.wdot_report(w[:, idx], ref, s)
    _say("  wdot", r)
    assert r["ok"], r
    rmu, rlam, rDm = om.transport(Ts, ps, Ys)
    for name, g, rr in (("mu", mu[idx], rmu), ("lambda", lam[idx], rlam), ("Dmix", Dm[:, idx], rDm)):
        rep = PM.rel_report(g, rr, PM.REL_FP64)
        _say("  ", name, rep)
        assert rep["ok"], (name, rep)


def test_special_case_mechanism(kx):
    """beta = E_R = 0, integer beta and shared (beta, E_R) reactions."""
    spec = I.MechSpec(53, 266, 30, 0, 29, seed=77, special_cases=True, name="syn53sc")
    m = I.make_mechanism(spec)
    T, p, Y = I.make_states(53, I.STATES_53, n_points=4096)
    check_rates(kx, m, T, p, Y, "special cases")


def test_further_reaction_forms(kx, mech53x):
    """SRI falloff, chemically activated falloff (Lindemann-free Troe and SRI)
    and pressure-table reactions (syn53x: 10 SRI, 8 chemically activated, 20
    PLOG), FP64 and mixed, at pressures from below to above the tables'
    reference pressures (0.1-100 atm), with a ragged tail; and
    near-equilibrium states, where the net rate is a small difference."""
    T, p, Y = I.make_states(53, I.StateSpec(4096 + 11, seed=41, p_atm_range=(0.02, 300.0),
                                            dirichlet_alpha=0.3))
    check_rates(kx, mech53x, T, p, Y, "further forms")
    dm = dev_mech(kx, mech53x)
    w = run_rates(kx, dm, T, p, Y, precision="mixed")
    ref, sc = O.OracleMech(mech53x).production_rates(T, p, Y)
    r = PM.mixed_wdot_report(w, ref, sc)
    _say("  mixed", r)
    assert r["ok"], r
    om = O.OracleMech(mech53x)
    Te, pe, Ye = O.equilibrium_states(om, 1024, seed=43, perturb=1e-6)
    check_rates(kx, mech53x, Te, pe, Ye, "further forms near equilibrium")


def test_explicit_orders(kx, mech53o):
    """20 irreversible reactions with non-integer forward orders (one with a
    non-reactant species), FP64 and mixed."""
    T, p, Y = I.make_states(53, I.StateSpec(4096 + 3, seed=45, p_atm_range=(0.5, 40.0),
                                            dirichlet_alpha=0.3))
    check_rates(kx, mech53o, T, p, Y, "explicit orders")
    dm = dev_mech(kx, mech53o)
    w = run_rates(kx, dm, T, p, Y, precision="mixed")
    ref, sc = O.OracleMech(mech53o).production_rates(T, p, Y)
    r = PM.mixed_wdot_report(w, ref, sc)
    _say("  mixed", r)
    assert r["ok"], r


def test_imported_yaml_mechanism(kx):
    """A mechanism read by the Cantera-YAML importer (the synthetic fixture:
    every reaction form, duplicates, a single-range NASA species, a single
    collider), FP64 rates and transport through the C ABI."""
    import os
    from paper_2411_02640_amd import mech_yaml as MY
    m = MY.load(os.path.join(os.path.dirname(__file__), "golden", "mini_mech.yaml"))
    T, p, Y = I.make_states(m["n_species"], I.StateSpec(3001, seed=51, p_atm_range=(0.05, 50.0),
                                                        dirichlet_alpha=0.5))
    check_rates(kx, m, T, p, Y, "imported")
    check_transport(kx, m, T, p, Y, "imported")


# |J_gpu - J_ref| per entry relative to the largest |J| of its row.  Both sides
# are FP64 sums of the same terms in different orders (complex step on the
# oracle side), so the difference is a few ulps of the row's largest terms;
# 1e-12 leaves a margin of ~20 over the largest difference seen (5e-14).
JAC_TOL = 1e-12


def _check_jacobian(kx, mech, T, p, Y, label):
    _say("jacobian", label, mech.get("name", ""), "n =", T.size)
    dm = dev_mech(kx, mech)
    Td, pd, Yd = to_dev(T, p, Y)
    J = kx.jacobian(dm, Td, pd, Yd).cpu().numpy()
    ref = O.OracleMech(mech).jacobian(T, p, Y)
    assert np.isfinite(J).all()
    row = np.abs(ref).max(axis=2, keepdims=True)
    err = np.abs(J - ref) / np.where(row > 0, row, 1.0)
    _say("   max error / row scale", float(err.max()),
         "median", float(np.median(err)))
    assert err.max() <= JAC_TOL, float(err.max())
    return J, ref


def test_jacobian(kx, mech9, mech53x, mech53o):
    """d wdot / d C through the C ABI against the oracle's complex-step
    Jacobian (a different method: no derivative formulas), for syn9 (all 4096
    points + a ragged tail), a tiny mechanism with one reaction of every form,
    and samples of the 53-species mechanisms with SRI, chemically activated and
    pressure-table reactions and with explicit orders."""
    from . import tiny_mechs as TM
    T, p, Y = I.make_states(9, I.StateSpec(4096 + 7, seed=61))
    _check_jacobian(kx, mech9, T, p, Y, "syn9")
    m = TM.all_forms_mechanism()
    T, p, Y = I.make_states(4, I.StateSpec(2048, seed=62, p_atm_range=(0.1, 20.0),
                                           dirichlet_alpha=1.0))
    _check_jacobian(kx, m, T, p, Y, "all forms")
    for mech, seed in ((mech53x, 63), (mech53o, 64)):
        T, p, Y = I.make_states(53, I.StateSpec(129, seed=seed, p_atm_range=(0.05, 150.0),
                                                dirichlet_alpha=0.3))
        _check_jacobian(kx, mech, T, p, Y, mech["name"])


def test_jacobian_rows_conserve_mass(kx, mech53):
    """sum_k W_k J_kj = 0 (every reaction balanced) on the GPU result for the
    benchmark mechanism, 2^14 points."""
    T, p, Y = I.make_states(53, I.STATES_53, n_points=1 << 14)
    dm = dev_mech(kx, mech53)
    J = kx.jacobian(dm, *to_dev(T, p, Y))
    W = torch.from_numpy(np.asarray(mech53["composition"] @ mech53["elem_mass"], float)).to(DEV)
    s = (W[None, :, None] * J).sum(dim=1)
    a = (W[None, :, None] * J.abs()).sum(dim=1)
    rel = (s.abs() / torch.clamp(a, min=1e-300)).max().item()
    _say("jacobian mass rows: max |W.J| / (W.|J|)", rel)
    assert rel < 1e-13


def test_diffusion_fit_kind_direct(kx):
    """Tables holding fits of D_kj itself (diff_fit_kind = 0): the vector-ALU
    transport kernel with a reciprocal per pair, FP64 and mixed."""
    spec = I.MechSpec(53, 266, 30, 0, 29, seed=53325, diff_fit_kind=0, name="syn53d")
    m = I.make_mechanism(spec)
    T, p, Y = I.make_states(53, I.STATES_53, n_points=4133)
    check_transport(kx, m, T, p, Y, "D fits")
    dm = dev_mech(kx, m)
    mu, lam, Dm = run_transport(kx, dm, T, p, Y, precision="mixed")
    rmu, rlam, rDm = O.OracleMech(m).transport(T, p, Y)
    for name, g, r in (("mu", mu, rmu), ("lambda", lam, rlam), ("Dmix", Dm, rDm)):
        rep = PM.rel_report(g, r, PM.REL_MIXED)
        _say("  mixed", name, rep)
        assert rep["ok"], (name, rep)


def test_symmetric_diffusion_fits(kx):
    """Tables of D_kj fits evaluated once per unordered pair (KX_DKJ_SYMMETRIC,
    the symmetric D_kj of §2.2.2 / §2.3.2), FP64 and mixed, at 53 and 200
    species with a ragged tail, against the oracle (which evaluates every
    ordered pair); the tables of 1/D_kj fits ignore the option."""
    import dataclasses
    for spec, npts in ((I.MechSpec(53, 266, 30, 0, 29, seed=53325, diff_fit_kind=0,
                                   name="syn53d"), 4133),
                       (dataclasses.replace(I.MECH_200, diff_fit_kind=0, name="syn200d"), 1031)):
        m = I.make_mechanism(spec)
        ns = m["n_species"]
        T, p, Y = I.make_states(ns, I.StateSpec(npts, seed=91, p_atm_range=(1.0, 40.0),
                                                dirichlet_alpha=0.3))
        dm = dev_mech(kx, m)
        om = O.OracleMech(m)
        rmu, rlam, rDm = om.transport(T, p, Y)
        Td, pd, Yd = to_dev(T, p, Y)
        for prec, tol in (("fp64", PM.REL_FP64), ("mixed", PM.REL_MIXED)):
            _say("symmetric D_kj", spec.name, prec, "n =", npts)
            out = kx.transport(dm, Td, pd, Yd, precision=prec, symmetric=True)
            torch.cuda.synchronize()
            for name, g, rr in zip(("mu", "lambda", "Dmix"), out, (rmu, rlam, rDm)):
                rep = PM.rel_report(g.cpu().numpy(), rr, tol)
                _say("  ", name, rep)
                assert rep["ok"], (spec.name, prec, name, rep)
    # 1/D_kj tables: the option changes nothing
    m53 = I.make_mechanism(I.MECH_53)
    T, p, Y = I.make_states(53, I.STATES_53, n_points=3000)
    dm = dev_mech(kx, m53)
    Td, pd, Yd = to_dev(T, p, Y)
    a = kx.transport(dm, Td, pd, Yd)
    b = kx.transport(dm, Td, pd, Yd, symmetric=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_other_fit_orders(kx):
    """Transport fits with 3, 4, 7 and 8 coefficients (every other test
    mechanism has 5; these run the kernels' forms for any fit order): the
    matrix-core kernel (1/D_kj fits), the vector-ALU kernel and the symmetric
    evaluation (D_kj fits), FP64 and mixed, 4133 points, against the oracle."""
    import dataclasses
    T, p, Y = I.make_states(53, I.StateSpec(4133, seed=92, p_atm_range=(1.0, 40.0),
                                            dirichlet_alpha=0.3))
    Td, pd, Yd = to_dev(T, p, Y)
    for fo, kind, sym in ((4, 1, False), (8, 1, False), (3, 0, False), (7, 0, True)):
        spec = dataclasses.replace(I.MECH_53, fit_order=fo, diff_fit_kind=kind,
                                   name=f"syn53_fit{fo}_kind{kind}")
        m = I.make_mechanism(spec)
        assert m["fit_order"] == fo
        dm = kx.Mechanism(m, 0)
        try:
            rmu, rlam, rDm = O.OracleMech(m).transport(T, p, Y)
            for prec, tol in (("fp64", PM.REL_FP64), ("mixed", PM.REL_MIXED)):
                _say("fit order", fo, "diffusion fit kind", kind, "symmetric" if sym else "",
                     prec, "n =", T.size)
                out = kx.transport(dm, Td, pd, Yd, precision=prec, symmetric=sym)
                torch.cuda.synchronize()
                for name, g, rr in zip(("mu", "lambda", "Dmix"), out, (rmu, rlam, rDm)):
                    rep = PM.rel_report(g.cpu().numpy(), rr, tol)
                    _say("  ", name, rep)
                    assert rep["ok"], (spec.name, prec, name, rep)
        finally:
            dm.close()


def test_near_equilibrium_states_fp64(kx, mech53):
    om = O.OracleMech(mech53)
    T, p, Y = O.equilibrium_states(om, 2048, seed=31, perturb=1e-6)
    check_rates(kx, mech53, T, p, Y, "near equilibrium")


def test_edge_states(kx, mech53):
    ns = 53
    rows = []
    for T in (200.0, 300.0, np.nextafter(1000.0, 0), 1000.0, 2800.0, 3500.0):
        for patm in (0.01, 1.0, 100.0):
            rows.append((T, patm * O.PATM))
    Ts = np.array([r[0] for r in rows])
    ps = np.array([r[1] for r in rows])
    rng = np.random.default_rng(5)
    Y = rng.dirichlet(np.full(ns, 0.3), size=Ts.size).T.copy()
    # pure species and mixtures with absent species
    pureT = np.full(ns, 1500.0)
    purep = np.full(ns, 2 * O.PATM)
    pureY = np.eye(ns)
    sparse = np.zeros((ns, 8))
    for c in range(8):
        sel = rng.choice(ns - 1, 3, replace=False)
        sparse[sel, c] = rng.dirichlet(np.ones(3))
    T = np.concatenate([Ts, pureT, np.linspace(400, 2500, 8)])
    p = np.concatenate([ps, purep, np.full(8, O.PATM)])
    Yall = np.concatenate([Y, pureY, sparse], axis=1)
    check_rates(kx, mech53, T, p, Yall, "edge states")
    check_transport(kx, mech53, T, p, Yall, "edge states")


def test_single_point_and_empty(kx, mech9):
    T, p, Y = I.make_states(9, I.STATES_9, n_points=1)
    check_rates(kx, mech9, T, p, Y, "n = 1")
    check_transport(kx, mech9, T, p, Y, "n = 1")
    dm = dev_mech(kx, mech9)
    _say("n = 0 no-op")
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    w = kx.production_rates(dm, e, e, torch.empty((9, 0), dtype=torch.float64, device=DEV))
    mu, lam, Dm = kx.transport(dm, e, e, torch.empty((9, 0), dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    assert w.shape == (9, 0) and Dm.shape == (9, 0)


def test_deterministic_and_stream(kx, mech53):
    T, p, Y = I.make_states(53, I.STATES_53, n_points=20000)
    dm = dev_mech(kx, mech53)
    Td, pd, Yd = to_dev(T, p, Y)
    _say("determinism / side stream")
    a = kx.production_rates(dm, Td, pd, Yd)
    mu_a, _, D_a = kx.transport(dm, Td, pd, Yd)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b = kx.production_rates(dm, Td, pd, Yd, stream=s)
        mu_b, _, D_b = kx.transport(dm, Td, pd, Yd, stream=s)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(mu_a, mu_b) and torch.equal(D_a, D_b)


def test_thermo_outputs(kx, mech53):
    T, p, Y = I.make_states(53, I.STATES_53, n_points=5000)
    dm = dev_mech(kx, mech53)
    Td, Yd = to_dev(T, Y)
    _say("thermo n =", T.size)
    cpk, hk, cp = kx.thermo(dm, Td, Yd)
    torch.cuda.synchronize()
    rcpk, rhk, rcp = O.OracleMech(mech53).mixture_thermo(T, Y)
    np.testing.assert_allclose(cpk.cpu().numpy(), rcpk, rtol=1e-13)
    np.testing.assert_allclose(cp.cpu().numpy(), rcp, rtol=1e-13)
    # h_k = H_k/W_k changes sign: judge against the per-species scale
    hg = hk.cpu().numpy()
    scale = np.abs(rhk).max(axis=1, keepdims=True)
    assert (np.abs(hg - rhk) <= 1e-12 * scale).all()


# ------------------------------------------------------------------ mixed path
def _mixed_workload(mech, n, seed):
    """Three quarters as the 53-species FP64 workload, one quarter within 1e-6
    of a constructed equilibrium state, randomly interleaved."""
    om = O.OracleMech(mech)
    nq = n // 4
    T1, p1, Y1 = I.make_states(mech["n_species"], I.StateSpec(
        n - nq, seed=seed, p_atm_range=(1.0, 40.0), dirichlet_alpha=0.3))
    T2, p2, Y2 = O.equilibrium_states(om, nq, seed=seed + 1000, perturb=1e-6)
    T = np.concatenate([T1, T2])
    p = np.concatenate([p1, p2])
    Y = np.concatenate([Y1, Y2], axis=1)
    near = np.concatenate([np.zeros(n - nq, bool), np.ones(nq, bool)])
    perm = np.random.default_rng(seed).permutation(n)
    return T[perm], p[perm], np.ascontiguousarray(Y[:, perm]), near[perm]


def test_mixed_precision_error_report(kx, mech53):
    T, p, Y, near = _mixed_workload(mech53, 1 << 14, seed=3)
    dm = dev_mech(kx, mech53)
    _say("mixed n =", T.size)
    w = run_rates(kx, dm, T, p, Y, precision="mixed")
    mu, lam, Dm = run_transport(kx, dm, T, p, Y, precision="mixed")
    om = O.OracleMech(mech53)
    ref, s = om.production_rates(T, p, Y)
    rmu, rlam, rDm = om.transport(T, p, Y)
    for part, sel in (("bulk", ~near), ("near-equilibrium", near)):
        r = PM.mixed_wdot_report(w[:, sel], ref[:, sel], s[:, sel])
        _say("  wdot", part, r)
        assert r["ok"], (part, r)
        for name, g, rr in (("mu", mu[sel], rmu[sel]), ("lambda", lam[sel], rlam[sel]),
                            ("Dmix", Dm[:, sel], rDm[:, sel])):
            rep = PM.rel_report(g, rr, PM.REL_MIXED)
            _say("  ", name, part, rep)
            assert rep["ok"], (name, part, rep)


def test_mixed_full_size_sampled(kx, mech53):
    """The mixed-precision workload at its full size (2^22 points, a quarter of
    them within 1e-6 of constructed equilibrium states -- 4096 distinct ones,
    each used 256 times), both kernels in the benchmark's launch
    configuration; the oracle checks a sample split into bulk and
    near-equilibrium points."""
    n = I.STATES_53_MIXED.n_points
    nq = n // 4
    om = O.OracleMech(mech53)
    T1, p1, Y1 = I.make_states(53, I.STATES_53_MIXED, n_points=n - nq)
    Te, pe, Ye = O.equilibrium_states(om, 1 << 12, seed=1003, perturb=1e-6)
    reps = nq // Te.size
    T = np.concatenate([T1, np.tile(Te, reps)])
    p = np.concatenate([p1, np.tile(pe, reps)])
    Y = np.ascontiguousarray(np.concatenate([Y1, np.tile(Ye, (1, reps))], axis=1))
    del Y1
    near = np.zeros(n, bool)
    near[n - nq:] = True
    _say("mixed full size n =", n)
    dm = dev_mech(kx, mech53)
    w = run_rates(kx, dm, T, p, Y, precision="mixed")
    mu, lam, Dm = run_transport(kx, dm, T, p, Y, precision="mixed")
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([rng.choice(n - nq, 1000, replace=False),
                                    n - nq + rng.choice(nq, 1000, replace=False),
                                    [0, 7, 8, 63, 64, n - nq - 1, n - nq, n - 1]]))
    Ts, ps, Ys = T[idx], p[idx], np.ascontiguousarray(Y[:, idx])
    ref, sc = om.production_rates(Ts, ps, Ys)
    rmu, rlam, rDm = om.transport(Ts, ps, Ys)
    sel_near = near[idx]
    for part, sel in (("bulk", ~sel_near), ("near-equilibrium", sel_near)):
        r = PM.mixed_wdot_report(w[:, idx][:, sel], ref[:, sel], sc[:, sel])
        _say("  wdot", part, r)
        assert r["ok"], (part, r)
        for name, g, rr in (("mu", mu[idx][sel], rmu[sel]), ("lambda", lam[idx][sel], rlam[sel]),
                            ("Dmix", Dm[:, idx][:, sel], rDm[:, sel])):
            rep = PM.rel_report(g, rr, PM.REL_MIXED)
            _say("  ", name, part, rep)
            assert rep["ok"], (name, part, rep)
