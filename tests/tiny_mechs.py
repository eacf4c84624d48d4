"""Hand-built tiny mechanisms for closed-form and brute-force checks."""
import math

import numpy as np

RCAL = 8.31446261815324 / 4.184
PATM = 1013250.0


def _csr(lists):
    ptr, sp, nu = [0], [], []
    for lst in lists:
        for s, v in lst:
            sp.append(s)
            nu.append(v)
        ptr.append(len(sp))
    return np.array(ptr, np.int32), np.array(sp, np.int32), np.array(nu, np.int32)


def build(species_comp, nasa, reactions, visc=None, cond=None, diff=None):
    """reactions: list of dicts with keys type, reac [(sp, nu)], prod [(sp, nu)],
    A, beta, Ea and optionally A0, beta0, Ea0, troe (4), sri (5), chem_act,
    plog [(p, A, beta, Ea)], ord [(sp, order)], eff {sp: alpha}, eff_default."""
    ns = len(species_comp)
    nr = len(reactions)
    comp = np.array(species_comp, np.int32)
    nasa = np.asarray(nasa, np.float64)
    rp, rs, rn = _csr([r["reac"] for r in reactions])
    pp, ps, pn = _csr([r["prod"] for r in reactions])
    eff_ptr, eff_sp, eff_val = [0], [], []
    for r in reactions:
        for s, a in sorted(r.get("eff", {}).items()):
            eff_sp.append(s)
            eff_val.append(a)
        eff_ptr.append(len(eff_sp))
    extra = {"sri": None, "chem_act": None, "plog_ptr": None, "plog_p": None,
             "plog_A": None, "plog_beta": None, "plog_Ea": None, "ord_ptr": None,
             "ord_sp": None, "ord_val": None}
    if any("ord" in r for r in reactions):
        optr, osp, oval = [0], [], []
        for r in reactions:
            for k, o in r.get("ord", []):
                osp.append(k)
                oval.append(o)
            optr.append(len(osp))
        extra.update(ord_ptr=np.array(optr, np.int32), ord_sp=np.array(osp, np.int32),
                     ord_val=np.array(oval, float))
    if any("sri" in r or "chem_act" in r or "plog" in r for r in reactions):
        extra["sri"] = np.array([r.get("sri", [0.0] * 5) for r in reactions], float)
        extra["chem_act"] = np.array([r.get("chem_act", 0) for r in reactions], np.int32)
        ptr, pts = [0], []
        for r in reactions:
            pts += r.get("plog", [])
            ptr.append(len(pts))
        pts = np.array(pts, float).reshape(-1, 4)
        extra.update(plog_ptr=np.array(ptr, np.int32), plog_p=pts[:, 0].copy(),
                     plog_A=pts[:, 1].copy(), plog_beta=pts[:, 2].copy(),
                     plog_Ea=pts[:, 3].copy())
    fo = 5
    if visc is None:
        visc = np.tile([2e-4, 5e-5, 1e-6, 0.0, 0.0], (ns, 1))
    if cond is None:
        cond = np.tile([5e3, 2e3, 1e2, 0.0, 0.0], (ns, 1))
    if diff is None:
        diff = np.tile([1.0, 0.8, 0.2, 0.0, 0.0], (ns, ns, 1))
    return {
        "name": "tiny", "n_species": ns, "n_reactions": nr, "n_elements": comp.shape[1],
        "elem_mass": np.array([1.008, 15.999, 14.007][: comp.shape[1]]),
        "composition": comp, "nasa_lo": nasa.copy(), "nasa_hi": nasa.copy(),
        "t_mid": np.full(ns, 1000.0),
        "rxn_type": np.array([r["type"] for r in reactions], np.int32),
        "reversible": np.array([r.get("rev", 1) for r in reactions], np.int32),
        "reac_ptr": rp, "reac_sp": rs, "reac_nu": rn,
        "prod_ptr": pp, "prod_sp": ps, "prod_nu": pn,
        "A": np.array([r["A"] for r in reactions], float),
        "beta": np.array([r["beta"] for r in reactions], float),
        "Ea": np.array([r["Ea"] for r in reactions], float),
        "A0": np.array([r.get("A0", 0.0) for r in reactions], float),
        "beta0": np.array([r.get("beta0", 0.0) for r in reactions], float),
        "Ea0": np.array([r.get("Ea0", 0.0) for r in reactions], float),
        "troe": np.array([r.get("troe", [0, 0, 0, 0]) for r in reactions], float),
        "eff_ptr": np.array(eff_ptr, np.int32), "eff_sp": np.array(eff_sp, np.int32),
        "eff_val": np.array(eff_val, float),
        "eff_default": np.array([r.get("eff_default", 1.0) for r in reactions], float),
        "fit_order": fo, "fit_L0": 7.0, "fit_h": 1.2, "diff_fit_kind": 0,
        "visc_fit": np.asarray(visc, float), "cond_fit": np.asarray(cond, float),
        "diff_fit": np.asarray(diff, float),
        **extra,
    }


A_, B_, AB_, D_ = 0, 1, 2, 3
ABX_COMP = [(1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 2)]
ABX_NASA = [
    [2.5, 0.0, 0.0, 0.0, 0.0, 2.5e4, 4.2],
    [2.5, 0.0, 0.0, 0.0, 0.0, 2.9e4, 5.1],
    [3.3, 1.1e-3, -3.0e-7, 4.0e-11, -2.0e-15, 4.5e3, 3.9],
    [3.5, 2.0e-4, 0.0, 0.0, 0.0, -1.0e3, 4.0],
]


def abx_mechanism():
    """{A, B, AB, D}: A + B <=> AB as elementary, three-body, Troe and a
    single-collider Lindemann reaction, plus AB + A <=> B + 2 A."""
    rx = [
        dict(type=0, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=3.0e13, beta=0.4, Ea=1.2e3),
        dict(type=1, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=2.0e15, beta=-0.8, Ea=0.0,
             eff={B_: 2.5, D_: 0.7}),
        dict(type=3, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=1.5e12, beta=0.3, Ea=5.0e3,
             A0=4.0e18, beta0=-1.1, Ea0=2.0e3, troe=[0.62, 150.0, 1800.0, 4500.0],
             eff={AB_: 3.0}),
        dict(type=0, reac=[(AB_, 1), (A_, 1)], prod=[(B_, 1), (A_, 2)], A=7.0e14, beta=0.0,
             Ea=3.1e4),
        dict(type=2, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=9.0e12, beta=0.1, Ea=800.0,
             A0=2.0e17, beta0=-0.5, Ea0=0.0, eff_default=0.0, eff={B_: 1.0}),
    ]
    return build(ABX_COMP, ABX_NASA, rx)


def single_reaction_mech(rtype, A=1e13, beta=0.0, Ea=0.0, A0=0.0, beta0=0.0, Ea0=0.0,
                         troe=(0, 0, 0, 0), eff=None, eff_default=1.0, rev=1, **more):
    """A + B <=> AB of one type; `more` passes sri, chem_act or plog through."""
    rx = [dict(type=rtype, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=A, beta=beta, Ea=Ea,
               A0=A0, beta0=beta0, Ea0=Ea0, troe=list(troe), eff=eff or {},
               eff_default=eff_default, rev=rev, **more)]
    return build(ABX_COMP, ABX_NASA, rx)


def ea_for_half(T):
    """E_a (cal/mol) with exp(-E_a/(R T)) = 1/2 at temperature T."""
    return math.log(2.0) * RCAL * T


def all_forms_mechanism():
    """{A, B, AB, D} with one reaction of every form: elementary, three-body,
    Troe, SRI, chemically activated Troe, a pressure table and explicit orders."""
    base = dict(beta=0.3, Ea=3000.0)
    rx = [
        dict(type=0, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=3e13, **base),
        dict(type=1, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=2e15, beta=-0.8,
             Ea=0.0, eff={B_: 2.5, D_: 0.7}),
        dict(type=3, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=1.5e12, beta=0.3,
             Ea=5e3, A0=4e18, beta0=-1.1, Ea0=2e3, troe=[0.62, 150.0, 1800.0, 4500.0],
             eff={AB_: 3.0}),
        dict(type=4, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=9e12, beta=0.1,
             Ea=800.0, A0=2e17, beta0=-0.5, Ea0=0.0, sri=[0.8, 600.0, 900.0, 1.3, 0.1]),
        dict(type=3, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=1e12, beta=0.0,
             Ea=0.0, A0=1e17, beta0=0.0, Ea0=0.0, troe=[0.5, 200.0, 1500.0, np.nan],
             chem_act=1),
        dict(type=5, reac=[(AB_, 1), (A_, 1)], prod=[(B_, 1), (A_, 2)], A=1.0,
             beta=0.0, Ea=0.0, plog=[(0.5 * PATM, 7e14, 0.0, 3.1e4), (5 * PATM, 2e15, 0.1,
                                                                          3.2e4)]),
        dict(type=0, reac=[(A_, 1), (B_, 1)], prod=[(AB_, 1)], A=3e12, rev=0,
             ord=[(A_, 1.5), (D_, 0.25)], **base),
    ]
    return build(ABX_COMP, ABX_NASA, rx)


# isomers A, Q1, Q2, B (one atom of each of the first two elements) and a bath D
QA_, Q1_, Q2_, QB_, QD_ = 0, 1, 2, 3, 4
QSS_COMP = [(1, 1, 0), (1, 1, 0), (1, 1, 0), (1, 1, 0), (0, 0, 2)]
QSS_NASA = [
    [3.3, 1.1e-3, -3.0e-7, 4.0e-11, -2.0e-15, 4.5e3, 3.9],
    [3.1, 9.0e-4, -2.0e-7, 3.0e-11, -1.0e-15, 1.2e4, 4.4],
    [3.6, 7.0e-4, -1.0e-7, 2.0e-11, -1.0e-15, 9.0e3, 5.0],
    [3.4, 1.0e-3, -2.5e-7, 3.5e-11, -1.5e-15, -2.0e3, 4.1],
    [3.5, 2.0e-4, 0.0, 0.0, 0.0, -1.0e3, 4.0],
]


def qss_chain_mechanism(qss=(Q1_, Q2_)):
    """A <=> Q1 <=> Q2 -> B, Q1 + D -> B + D and Q1 (+M) -> B (+M) with
    efficiency 2 for D; the species in `qss` are quasi-steady."""
    rx = [
        dict(type=0, reac=[(QA_, 1)], prod=[(Q1_, 1)], A=1e10, beta=0.2, Ea=5.0e3),
        dict(type=0, reac=[(Q1_, 1)], prod=[(Q2_, 1)], A=3e11, beta=0.0, Ea=2.0e3),
        dict(type=0, reac=[(Q2_, 1)], prod=[(QB_, 1)], A=5e9, beta=0.5, Ea=1.0e3, rev=0),
        dict(type=0, reac=[(Q1_, 1), (QD_, 1)], prod=[(QB_, 1), (QD_, 1)], A=2e13,
             beta=0.0, Ea=4.0e3, rev=0),
        dict(type=1, reac=[(Q1_, 1)], prod=[(QB_, 1)], A=4e15, beta=-0.5, Ea=0.0, rev=0,
             eff={QD_: 2.0}),
    ]
    m = build(QSS_COMP, QSS_NASA, rx)
    flags = np.zeros(len(QSS_COMP), np.int32)
    flags[list(qss)] = 1
    m["qss"] = flags
    return m


def qss_long_chain(nq=9):
    """A <=> Q1 <=> ... <=> Q_nq -> B (isomers), every Q_i also drained to B
    through the bath D, and one three-body sink; Q_1..Q_nq are quasi-steady.
    nq (nq + 1) > 64 for nq >= 8."""
    ns = nq + 3                       # A, Q1..Qnq, B, D
    a, b, d = 0, nq + 1, nq + 2
    comp = [(1, 1, 0)] * (nq + 2) + [(0, 0, 2)]
    base = np.array([3.3, 1.0e-3, -2.5e-7, 3.0e-11, -1.5e-15, 0.0, 4.0])
    nasa = []
    for k in range(ns):
        row = base.copy()
        row[5] = 4.5e3 + 900.0 * ((k * 7) % 11) if k != d else -1.0e3
        row[6] = 4.0 + 0.1 * k
        nasa.append(row.tolist())
    rx = [dict(type=0, reac=[(a, 1)], prod=[(1, 1)], A=1e10, beta=0.2, Ea=5.0e3)]
    for i in range(1, nq):
        rx.append(dict(type=0, reac=[(i, 1)], prod=[(i + 1, 1)], A=3e11 * (1 + i % 3),
                       beta=0.1 * (i % 2), Ea=2.0e3 + 300.0 * i))
    rx.append(dict(type=0, reac=[(nq, 1)], prod=[(b, 1)], A=5e9, beta=0.5, Ea=1.0e3, rev=0))
    for i in range(1, nq + 1):
        rx.append(dict(type=0, reac=[(i, 1), (d, 1)], prod=[(b, 1), (d, 1)],
                       A=2e12 * (1 + i % 4), beta=0.0, Ea=4.0e3 + 100.0 * i, rev=0))
    rx.append(dict(type=1, reac=[(2, 1)], prod=[(b, 1)], A=4e15, beta=-0.5, Ea=0.0, rev=0,
                   eff={d: 2.0}))
    m = build(comp, nasa, rx)
    flags = np.zeros(ns, np.int32)
    flags[1:nq + 1] = 1
    m["qss"] = flags
    return m
