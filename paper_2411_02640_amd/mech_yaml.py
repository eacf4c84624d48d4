"""Mechanism import from Cantera-format YAML files.

``load(path_or_text)`` turns the species and reactions of a Cantera YAML
mechanism into the mechanism dictionary that ``kx.Mechanism`` hands to
``kx_mech_create`` (the ``kx_mech_desc`` fields, cgs units).  ``dump(mech)``
writes such a dictionary back as YAML (round trips, test fixtures).

What is read:

* ``units`` (length, quantity, activation-energy, pressure; Cantera's defaults
  are m, kmol, J/kmol and Pa) and values written as "number unit" strings for
  activation energies, pressures and temperatures;
* species: ``composition``; ``thermo`` of model NASA7 with one or two
  temperature ranges (App. A.1); ``transport`` of model gas (geometry,
  diameter in Angstrom, well-depth in K, rotational-relaxation);
* reactions (App. A.2): elementary; ``three-body`` (equation with ``+ M``);
  ``falloff`` and ``chemically-activated`` (``(+M)`` or a single collider such
  as ``(+AR)``) with ``low-P-rate-constant`` / ``high-P-rate-constant`` and an
  optional ``Troe`` or ``SRI`` block; ``pressure-dependent-Arrhenius``
  (``rate-constants`` at reference pressures); ``efficiencies`` and
  ``default-efficiency``; ``<=>`` / ``=`` reversible, ``=>`` irreversible;
  ``duplicate`` is accepted (duplicates simply add).

Explicit forward ``orders`` are read for irreversible reactions.

Rejected with ValueError: other thermo models or reaction types (Chebyshev,
Blowers-Masel, surface reactions), ``orders`` on a reversible reaction,
non-integer stoichiometric coefficients, negative pre-exponential factors, A written with
units, efficiencies of undeclared species.

The polynomial transport fits are built from the Lennard-Jones parameters by
kinetic theory (``inputs.transport_fits``: Neufeld-Janzen-Aziz collision
integrals, Warnatz conductivity).  Those integrals are for non-polar
molecules: for a species with a dipole moment the Stockmayer correction is
not applied, and the species is listed in the result's ``_warnings``.
"""
from __future__ import annotations

import re

import numpy as np
import yaml

from . import inputs as I

# Standard atomic weights (IUPAC conventional values), g/mol.
ATOMIC_WEIGHT = {
    "H": 1.008, "D": 2.014, "He": 4.002602, "Li": 6.94, "Be": 9.0121831, "B": 10.81,
    "C": 12.011, "N": 14.007, "O": 15.999, "F": 18.998403163, "Ne": 20.1797,
    "Na": 22.98976928, "Mg": 24.305, "Al": 26.9815385, "Si": 28.085, "P": 30.973761998,
    "S": 32.06, "Cl": 35.45, "Ar": 39.95, "K": 39.0983, "Ca": 40.078, "Fe": 55.845,
    "Br": 79.904, "Kr": 83.798, "I": 126.90447, "Xe": 131.293, "E": 5.48579909065e-4,
}

CAL = 4.184                                  # J per thermochemical calorie
R_CAL = I.R_GAS * 1e-7 / CAL                 # cal / (mol K)
_LENGTH_CM = {"cm": 1.0, "m": 100.0, "mm": 0.1}
_QUANTITY_MOL = {"mol": 1.0, "kmol": 1000.0, "molec": 1.0 / I.N_AVOGADRO}
_ENERGY_CAL_MOL = {"cal/mol": 1.0, "kcal/mol": 1000.0, "J/mol": 1.0 / CAL,
                   "kJ/mol": 1000.0 / CAL, "J/kmol": 1.0 / (1000.0 * CAL),
                   "kJ/kmol": 1.0 / CAL, "K": R_CAL,
                   "eV": 1.602176634e-19 * I.N_AVOGADRO / CAL}
_PRESSURE_DYN = {"Pa": 10.0, "kPa": 1e4, "MPa": 1e7, "bar": 1e6, "atm": 1013250.0,
                 "Torr": 1013250.0 / 760.0, "dyn/cm^2": 1.0}
_GEOMETRY_ATOMS = {"atom": 1, "linear": 2, "nonlinear": 3}


def _num(v):
    """float of a YAML number; YAML 1.1 loaders read forms such as 1.0e10 as
    strings, which are accepted here too.  None if `v` is not a plain number."""
    if isinstance(v, (int, float)) and not isinstance(v, bool):
        return float(v)
    try:
        return float(str(v).strip())
    except ValueError:
        return None


def _f(v) -> float:
    x = _num(v)
    if x is None:
        raise ValueError(f"not a number: {v!r}")
    return x


def _quantity(v, table, default, what):
    """A number in the default unit, or a "number unit" string."""
    if _num(v) is not None:
        return _num(v) * table[default]
    m = re.fullmatch(r"\s*([-+0-9.eE]+)\s+(\S+)\s*", str(v))
    if not m or m.group(2) not in table:
        raise ValueError(f"cannot read {what} {v!r}")
    return float(m.group(1)) * table[m.group(2)]


class _Units:
    def __init__(self, u: dict | None):
        u = u or {}
        self.length = u.get("length", "m")
        self.quantity = u.get("quantity", "kmol")
        self.energy = u.get("activation-energy", "J/kmol")
        self.pressure = u.get("pressure", "Pa")
        if self.length not in _LENGTH_CM or self.quantity not in _QUANTITY_MOL:
            raise ValueError(f"unsupported units {u}")
        if self.energy not in _ENERGY_CAL_MOL or self.pressure not in _PRESSURE_DYN:
            raise ValueError(f"unsupported units {u}")

    def A(self, v, order: float) -> float:
        """A of a rate constant of `order` concentrations, to (cm^3/mol)^(order-1)/s."""
        if _num(v) is None:
            raise ValueError(f"A with explicit units ({v!r}) is not supported")
        f = _LENGTH_CM[self.length] ** 3 / _QUANTITY_MOL[self.quantity]
        return _num(v) * f ** (order - 1)

    def Ea(self, v) -> float:
        return _quantity(v, _ENERGY_CAL_MOL, self.energy, "activation energy")

    def p(self, v) -> float:
        return _quantity(v, _PRESSURE_DYN, self.pressure, "pressure")


def _arrhenius(rc, units, order):
    if "A" not in rc:
        raise ValueError(f"rate constant without A: {rc}")
    A = units.A(rc["A"], order)
    if not A > 0.0:
        raise ValueError("negative or zero pre-exponential factors are not supported")
    return A, _num(rc.get("b", 0.0)), units.Ea(rc.get("Ea", 0.0))


_COLLIDER = re.compile(r"\(\+\s*([^()\s]+)\s*\)")


def _parse_equation(eq: str):
    """(reactants, products, reversible, falloff collider or None, has + M)."""
    colliders = _COLLIDER.findall(eq)
    body = _COLLIDER.sub(" ", eq)
    for arrow, rev in (("<=>", True), ("=>", False), ("=", True)):
        if arrow in body:
            lhs, rhs = body.split(arrow, 1)
            break
    else:
        raise ValueError(f"no reaction arrow in {eq!r}")

    def side(text):
        out, third = [], False
        for term in re.split(r"\s+\+\s+", text.strip()):
            term = term.strip()
            if term == "M":
                third = True
                continue
            m = re.fullmatch(r"(\d+(?:\.\d*)?)\s+(\S+)|(\S+)", term)
            if not m:
                raise ValueError(f"cannot read {term!r} in {eq!r}")
            if m.group(3):
                out.append((m.group(3), 1))
            else:
                nu = float(m.group(1))
                if nu != int(nu) or nu <= 0:
                    raise ValueError(f"non-integer stoichiometry in {eq!r}")
                out.append((m.group(2), int(nu)))
        return out, third

    reac, t1 = side(lhs)
    prod, t2 = side(rhs)
    if len(set(colliders)) > 1:
        raise ValueError(f"two different falloff colliders in {eq!r}")
    return reac, prod, rev, (colliders[0] if colliders else None), (t1 or t2)


def load(src, T_fit=(I.T_FIT_LO, I.T_FIT_HI), qss_species=None) -> dict:
    """Mechanism dictionary (kx_mech_desc fields) from a Cantera YAML file path
    or YAML text.  The transport fits cover T_fit (K).  Cantera's format has no
    notion of quasi-steady species: `qss_species` (names) sets the descriptor's
    qss flags (kx_mech_create checks that they form a linear QSS system)."""
    if (T_fit[0], T_fit[1]) != (I.T_FIT_LO, I.T_FIT_HI):
        raise ValueError("only the default fit range is supported")
    text = src
    if "\n" not in str(src):
        with open(src) as f:
            text = f.read()
    doc = yaml.safe_load(text)
    units = _Units(doc.get("units"))
    spec_list = doc.get("species") or []
    rxn_list = doc.get("reactions") or []
    if not spec_list:
        raise ValueError("no species")
    names = [s["name"] for s in spec_list]
    index = {n: k for k, n in enumerate(names)}
    if len(index) != len(names):
        raise ValueError("duplicate species names")
    elements = []
    for s in spec_list:
        for e in s.get("composition", {}):
            if e not in elements:
                elements.append(e)
    for e in elements:
        if e not in ATOMIC_WEIGHT:
            raise ValueError(f"unknown element {e}")
    ns, ne = len(names), len(elements)
    comp = np.zeros((ns, ne), np.int32)
    nasa_lo = np.empty((ns, 7))
    nasa_hi = np.empty((ns, 7))
    t_mid = np.empty(ns)
    sigma = np.empty(ns)
    eps = np.empty(ns)
    zrot = np.empty(ns)
    natoms = np.empty(ns, np.int64)
    warnings = []
    for k, s in enumerate(spec_list):
        for e, n in s.get("composition", {}).items():
            if n != int(n):
                raise ValueError(f"non-integer atom count in species {s['name']}")
            comp[k, elements.index(e)] = int(n)
        th = s.get("thermo", {})
        if th.get("model") != "NASA7":
            raise ValueError(f"species {s['name']}: only NASA7 thermo is supported")
        data = [list(map(_f, d)) for d in th["data"]]
        ranges = [_f(x) for x in th["temperature-ranges"]]
        if len(data) == 1:
            nasa_lo[k] = nasa_hi[k] = data[0]
            t_mid[k] = ranges[-1]
        elif len(data) == 2:
            nasa_lo[k], nasa_hi[k] = data
            t_mid[k] = ranges[1]
        else:
            raise ValueError(f"species {s['name']}: more than two NASA7 ranges")
        tr = s.get("transport")
        if not tr or tr.get("model", "gas") != "gas":
            raise ValueError(f"species {s['name']}: gas transport data are required")
        sigma[k] = _f(tr["diameter"]) * 1e-8
        eps[k] = _f(tr["well-depth"])
        zrot[k] = _f(tr.get("rotational-relaxation", 0.0))
        natoms[k] = _GEOMETRY_ATOMS[tr["geometry"]]
        if _f(tr.get("dipole", 0.0)) != 0.0:
            warnings.append(f"{s['name']}: dipole moment ignored (non-polar collision "
                            "integrals)")
    elem_mass = np.array([ATOMIC_WEIGHT[e] for e in elements])
    W = comp @ elem_mass

    # ---- reactions
    nr = len(rxn_list)
    rtype = np.zeros(nr, np.int32)
    rev = np.zeros(nr, np.int32)
    A, beta, Ea = np.ones(nr), np.zeros(nr), np.zeros(nr)
    A0, beta0, Ea0 = np.zeros(nr), np.zeros(nr), np.zeros(nr)
    troe = np.zeros((nr, 4))
    sri = np.zeros((nr, 5))
    chem_act = np.zeros(nr, np.int32)
    eff_default = np.ones(nr)
    reac, prod, effs, ords = [], [], [], []
    pptr, pp, pA, pb, pE = [0], [], [], [], []
    for i, r in enumerate(rxn_list):
        eq = r["equation"]
        if r.get("negative-A"):
            raise ValueError(f"{eq}: negative pre-exponential factors are not supported")
        rs, ps, reversible, coll, plus_m = _parse_equation(eq)
        if "orders" in r:
            if reversible:
                raise ValueError(f"{eq}: explicit reaction orders need an irreversible "
                                 "reaction")
            for nm, o in r["orders"].items():
                if nm not in index:
                    raise ValueError(f"{eq}: order of undeclared species {nm}")
                ords.append((i, index[nm], _f(o)))
        for nm, _ in rs + ps:
            if nm not in index:
                raise ValueError(f"{eq}: undeclared species {nm}")
        reac.append([(index[nm], nu) for nm, nu in rs])
        prod.append([(index[nm], nu) for nm, nu in ps])
        rev[i] = 1 if reversible else 0
        order = sum(nu for _, nu in rs)
        if "orders" in r:
            # the units of A follow the sum of the forward orders
            listed = {nm: _f(o) for nm, o in r["orders"].items()}
            order = sum(nu for nm, nu in rs if nm not in listed) + sum(listed.values())
        kind = r.get("type", "elementary")
        eff = dict(r.get("efficiencies", {}) or {})
        if kind == "elementary":
            if plus_m or coll:
                raise ValueError(f"{eq}: third body in an elementary reaction")
            rtype[i] = I.RXN_ELEMENTARY
            A[i], beta[i], Ea[i] = _arrhenius(r["rate-constant"], units, order)
        elif kind == "three-body":
            if not plus_m:
                raise ValueError(f"{eq}: three-body reaction without + M")
            rtype[i] = I.RXN_THREEBODY
            A[i], beta[i], Ea[i] = _arrhenius(r["rate-constant"], units, order + 1)
        elif kind in ("falloff", "chemically-activated"):
            if coll is None:
                raise ValueError(f"{eq}: falloff reaction without (+M)")
            act = kind == "chemically-activated"
            # pressure-dependent falloff: k_inf of `order`, k_0 of order + 1;
            # chemically activated: k_0 of `order`, k_inf of order - 1
            hi_order, lo_order = (order - 1, order) if act else (order, order + 1)
            A[i], beta[i], Ea[i] = _arrhenius(r["high-P-rate-constant"], units, hi_order)
            A0[i], beta0[i], Ea0[i] = _arrhenius(r["low-P-rate-constant"], units, lo_order)
            chem_act[i] = 1 if act else 0
            if "Troe" in r:
                t = r["Troe"]
                rtype[i] = I.RXN_TROE
                troe[i] = (_f(t["A"]), _f(t["T3"]), _f(t["T1"]),
                           _f(t["T2"]) if "T2" in t else np.nan)
            elif "SRI" in r:
                t = r["SRI"]
                rtype[i] = I.RXN_SRI
                sri[i] = (_f(t["A"]), _f(t["B"]), _f(t["C"]),
                          _f(t.get("D", 1.0)), _f(t.get("E", 0.0)))
            else:
                rtype[i] = I.RXN_LINDEMANN
            if coll != "M":
                if coll not in index:
                    raise ValueError(f"{eq}: undeclared collider {coll}")
                eff = {coll: 1.0}
                eff_default[i] = 0.0
        elif kind == "pressure-dependent-Arrhenius":
            rtype[i] = I.RXN_PLOG
            pts = sorted(((units.p(q["P"]), q) for q in r["rate-constants"]),
                         key=lambda x: x[0])
            for j in range(1, len(pts)):
                if pts[j][0] == pts[j - 1][0]:
                    raise ValueError(f"{eq}: several rate constants at one pressure are "
                                     "not supported")
            for pj, q in pts:
                a, b, e = _arrhenius(q, units, order)
                pp.append(pj)
                pA.append(a)
                pb.append(b)
                pE.append(e)
        else:
            raise ValueError(f"{eq}: reaction type {kind!r} is not supported")
        if kind != "three-body" and kind not in ("falloff", "chemically-activated"):
            eff = {}
        if rtype[i] in (I.RXN_THREEBODY, I.RXN_LINDEMANN, I.RXN_TROE, I.RXN_SRI):
            eff_default[i] = _f(r.get("default-efficiency", eff_default[i]))
        for nm in eff:
            if nm not in index:
                raise ValueError(f"{eq}: efficiency of undeclared species {nm}")
        effs.append(sorted((index[nm], _f(a)) for nm, a in eff.items()))
        pptr.append(len(pp))

    def csr(lists):
        ptr, sp, nu = [0], [], []
        for lst in lists:
            merged = {}
            for k, v in lst:
                merged[k] = merged.get(k, 0) + v
            for k in sorted(merged):
                sp.append(k)
                nu.append(merged[k])
            ptr.append(len(sp))
        return np.array(ptr, np.int32), np.array(sp, np.int32), np.array(nu, np.int32)

    reac_ptr, reac_sp, reac_nu = csr(reac)
    prod_ptr, prod_sp, prod_nu = csr(prod)
    eff_ptr = np.array([0] + list(np.cumsum([len(e) for e in effs])), np.int32)
    eff_sp = np.array([k for e in effs for k, _ in e], np.int32)
    eff_val = np.array([a for e in effs for _, a in e], np.float64)

    # ---- transport fits (App. A.3), cp/R of each species from its NASA-7 table
    Tg = I.transport_fit_grid()
    cp_r = np.empty((ns, Tg.size))
    for k in range(ns):
        for g, T in enumerate(Tg):
            a = nasa_lo[k] if T < t_mid[k] else nasa_hi[k]
            cp_r[k, g] = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])))
    visc_fit, cond_fit, diff_fit = I.transport_fits(W, sigma, eps, zrot, natoms, cp_r, 1)

    qss = None
    if qss_species:
        qss = np.zeros(ns, np.int32)
        for nm in qss_species:
            if nm not in index:
                raise ValueError(f"unknown QSS species {nm!r}")
            qss[index[nm]] = 1

    ord_ptr = np.searchsorted([o[0] for o in ords], np.arange(nr + 1)).astype(np.int32)
    ord_sp = np.array([o[1] for o in ords], np.int32)
    ord_val = np.array([o[2] for o in ords], np.float64)
    any_extra = bool((rtype == I.RXN_SRI).any() or chem_act.any()
                     or (rtype == I.RXN_PLOG).any())
    return {
        "name": str(doc.get("description", "imported")).split("\n")[0][:40],
        "n_species": ns, "n_reactions": nr, "n_elements": ne,
        "elem_mass": elem_mass, "composition": comp,
        "nasa_lo": nasa_lo, "nasa_hi": nasa_hi, "t_mid": t_mid,
        "rxn_type": rtype, "reversible": rev,
        "reac_ptr": reac_ptr, "reac_sp": reac_sp, "reac_nu": reac_nu,
        "prod_ptr": prod_ptr, "prod_sp": prod_sp, "prod_nu": prod_nu,
        "A": A, "beta": beta, "Ea": Ea, "A0": A0, "beta0": beta0, "Ea0": Ea0,
        "troe": troe, "eff_ptr": eff_ptr, "eff_sp": eff_sp, "eff_val": eff_val,
        "eff_default": eff_default,
        "fit_order": I.FIT_ORDER, "fit_L0": I.FIT_L0, "fit_h": I.FIT_H, "diff_fit_kind": 1,
        "visc_fit": visc_fit, "cond_fit": cond_fit, "diff_fit": diff_fit,
        "sri": sri if any_extra else None,
        "chem_act": chem_act if any_extra else None,
        "plog_ptr": np.array(pptr, np.int32) if any_extra else None,
        "plog_p": np.array(pp) if any_extra else None,
        "plog_A": np.array(pA) if any_extra else None,
        "plog_beta": np.array(pb) if any_extra else None,
        "plog_Ea": np.array(pE) if any_extra else None,
        "ord_ptr": ord_ptr if ords else None,
        "ord_sp": ord_sp if ords else None,
        "ord_val": ord_val if ords else None,
        "qss": qss,
        "_species_names": names, "_elements": elements, "_warnings": warnings,
    }


def dump(mech: dict, names=None, elements=None, transport=None) -> str:
    """YAML text (units cm, mol, cal/mol, dyn/cm^2 written as Pa / 10) for a
    mechanism dictionary.  `transport` = (sigma_cm, eps, zrot, natoms) per
    species; for the synthetic generator's dictionaries it is taken from their
    metadata."""
    ns, nr = int(mech["n_species"]), int(mech["n_reactions"])
    names = names or mech.get("_species_names") or [f"S{k}" for k in range(ns)]
    elements = elements or mech.get("_elements")
    if elements is None:
        masses = list(mech["elem_mass"])
        elements = []
        for mval in masses:
            cand = [e for e, w in ATOMIC_WEIGHT.items() if w == mval and e not in elements]
            if not cand:
                raise ValueError(f"no element of mass {mval}")
            elements.append(cand[0])
    if transport is None:
        natoms = mech["composition"].sum(axis=1)
        transport = (mech["_sigma_cm"], mech["_eps_k"], mech["_zrot298"], natoms)
    sig, eps, zr, nat = transport
    geom = {1: "atom", 2: "linear"}
    f = repr

    def flt(x):
        return f(float(x))

    lines = ["description: exported kx mechanism",
             "units: {length: cm, quantity: mol, activation-energy: cal/mol, pressure: Pa}",
             "phases:",
             "- name: gas",
             "  thermo: ideal-gas",
             f"  elements: [{', '.join(elements)}]",
             "  species: all",
             "  kinetics: gas",
             "  transport: mixture-averaged",
             "species:"]
    for k in range(ns):
        cmp_ = ", ".join(f"{e}: {int(mech['composition'][k, j])}"
                         for j, e in enumerate(elements) if mech["composition"][k, j])
        lo = ", ".join(flt(x) for x in mech["nasa_lo"][k])
        hi = ", ".join(flt(x) for x in mech["nasa_hi"][k])
        lines += [f"- name: {names[k]}",
                  f"  composition: {{{cmp_}}}",
                  "  thermo:",
                  "    model: NASA7",
                  f"    temperature-ranges: [200.0, {flt(mech['t_mid'][k])}, 3500.0]",
                  f"    data:",
                  f"    - [{lo}]",
                  f"    - [{hi}]",
                  "  transport:",
                  "    model: gas",
                  f"    geometry: {geom.get(int(nat[k]), 'nonlinear')}",
                  f"    diameter: {flt(sig[k] * 1e8)}",
                  f"    well-depth: {flt(eps[k])}",
                  f"    rotational-relaxation: {flt(zr[k])}"]
    lines.append("reactions:")
    rt = mech["rxn_type"]
    chem = mech.get("chem_act")

    def side(ptr, sp, nu, i):
        return " + ".join((f"{int(nu[e])} " if nu[e] > 1 else "") + names[sp[e]]
                          for e in range(ptr[i], ptr[i + 1]))

    for i in range(nr):
        lhs = side(mech["reac_ptr"], mech["reac_sp"], mech["reac_nu"], i)
        rhs = side(mech["prod_ptr"], mech["prod_sp"], mech["prod_nu"], i)
        arrow = "<=>" if mech["reversible"][i] else "=>"
        t = int(rt[i])
        effs = {names[mech["eff_sp"][e]]: float(mech["eff_val"][e])
                for e in range(mech["eff_ptr"][i], mech["eff_ptr"][i + 1])}
        single = None
        if t in (2, 3, 4) and mech["eff_default"][i] == 0.0 and list(effs.values()) == [1.0]:
            single = list(effs)[0]
        if t == 1:
            eq = f"{lhs} + M {arrow} {rhs} + M"
        elif t in (2, 3, 4):
            c = single or "M"
            eq = f"{lhs} (+{c}) {arrow} {rhs} (+{c})"
        else:
            eq = f"{lhs} {arrow} {rhs}"
        rc = lambda a, b, e: f"{{A: {flt(a)}, b: {flt(b)}, Ea: {flt(e)}}}"
        lines.append(f"- equation: {eq}")
        if t == 0:
            lines.append(f"  rate-constant: {rc(mech['A'][i], mech['beta'][i], mech['Ea'][i])}")
        elif t == 1:
            lines += ["  type: three-body",
                      f"  rate-constant: {rc(mech['A'][i], mech['beta'][i], mech['Ea'][i])}"]
        elif t in (2, 3, 4):
            act = chem is not None and chem[i]
            lines += [f"  type: {'chemically-activated' if act else 'falloff'}",
                      f"  low-P-rate-constant: {rc(mech['A0'][i], mech['beta0'][i], mech['Ea0'][i])}",
                      f"  high-P-rate-constant: {rc(mech['A'][i], mech['beta'][i], mech['Ea'][i])}"]
            if t == 3:
                a, t3, t1, t2 = mech["troe"][i]
                tail = "" if np.isnan(t2) else f", T2: {flt(t2)}"
                lines.append(f"  Troe: {{A: {flt(a)}, T3: {flt(t3)}, T1: {flt(t1)}{tail}}}")
            if t == 4:
                a, b, c, d, e = mech["sri"][i]
                lines.append(f"  SRI: {{A: {flt(a)}, B: {flt(b)}, C: {flt(c)}, D: {flt(d)}, "
                             f"E: {flt(e)}}}")
        elif t == 5:
            lines += ["  type: pressure-dependent-Arrhenius", "  rate-constants:"]
            for j in range(mech["plog_ptr"][i], mech["plog_ptr"][i + 1]):
                lines.append(f"  - {{P: {flt(mech['plog_p'][j] / 10.0)}, A: "
                             f"{flt(mech['plog_A'][j])}, b: {flt(mech['plog_beta'][j])}, "
                             f"Ea: {flt(mech['plog_Ea'][j])}}}")
        op = mech.get("ord_ptr")
        if op is not None and op[i + 1] > op[i]:
            lines.append("  orders: {" + ", ".join(
                f"{names[mech['ord_sp'][e]]}: {flt(mech['ord_val'][e])}"
                for e in range(op[i], op[i + 1])) + "}")
        if t in (1, 2, 3, 4) and single is None:
            if effs:
                lines.append("  efficiencies: {" + ", ".join(f"{n}: {flt(v)}"
                                                             for n, v in effs.items()) + "}")
            if mech["eff_default"][i] != 1.0:
                lines.append(f"  default-efficiency: {flt(mech['eff_default'][i])}")
    return "\n".join(lines) + "\n"
