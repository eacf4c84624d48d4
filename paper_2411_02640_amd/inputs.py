"""Seeded synthetic mechanisms and thermochemical states.

This module produces *inputs* only: the mechanism tables that a user would
hand to ``kx_mech_create`` (species composition, NASA-7 thermo fits, reaction
list with Arrhenius / third-body / falloff parameters, and ln T polynomial fits
of the pure-species viscosity, conductivity and binary diffusion coefficients)
and per-point states (T, p, Y).  It never evaluates production rates, Gibbs
energies of reactions, equilibrium constants or mixture-averaged transport: both
the HIP path and the CPU oracle consume the tables built here, so the table
construction itself is not part of what parity checks.

The paper's mechanisms (H2 9/21, GRI-Mech 3.0 53/325, C2H5OH 129/1231; Table
"tab:mech") are not available, so seeded synthetic mechanisms with the same
shapes stand in for them.  Table-building physics used here (setup only):

* NASA-7 coefficients: least-squares fit of a smooth cp/R(T) curve on
  [300, 1000] K and [1000, 3000] K with cp, H and S continuous at T_mid
  (the seven-coefficient form of App. A.1, eq:H_RT / eq:S_R antiderivatives).
* Pure-species viscosity and binary diffusion from Lennard-Jones kinetic
  theory (App. A.3), with the collision integrals from the closed-form
  correlations of Neufeld, Janzen & Aziz, J. Chem. Phys. 57 (1972) 1100, used
  in place of the Monchick-Mason Stockmayer tables (non-polar species only).
* Pure-species conductivity from the Warnatz translational / rotational /
  vibrational split with the Parker / Brau-Jonkman Z_rot(T) (App. A.3).
* Degree-4 polynomial fits in a centred ln T variable u = (ln T - L0) / h
  (App. A.3 "Polynomial fits"; N = 5 coefficients), relative weighting.

Units are cgs throughout: T in K, p in dyn/cm^2, A in (cm^3/mol)^(m-1)/s,
Ea in cal/mol, viscosity in g/(cm s), conductivity in erg/(cm s K),
diffusion in cm^2/s.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Physical constants (CODATA 2018 exact values where applicable), cgs.
K_BOLTZ = 1.380649e-16          # erg / K
N_AVOGADRO = 6.02214076e23      # 1 / mol
R_GAS = 8.31446261815324e7      # erg / (mol K)
P_ATM = 1013250.0               # dyn / cm^2

ELEMENT_MASS = np.array([1.008, 15.999, 14.007])  # two reactive elements + diluent
T_MID = 1000.0
T_FIT_LO, T_FIT_HI = 300.0, 3000.0
FIT_ORDER = 5
FIT_L0 = 0.5 * (math.log(T_FIT_LO) + math.log(T_FIT_HI))
FIT_H = 0.5 * (math.log(T_FIT_HI) - math.log(T_FIT_LO))

RXN_ELEMENTARY, RXN_THREEBODY, RXN_LINDEMANN, RXN_TROE, RXN_SRI, RXN_PLOG = 0, 1, 2, 3, 4, 5


# --------------------------------------------------------------------------
# species
# --------------------------------------------------------------------------
def _species_compositions(ns: int) -> np.ndarray:
    """Element counts [ns, 3]; the last species is the inert diluent (0,0,2).

    Order: the two atoms, the three diatomics, then mixed then pure molecules
    by growing atom count up to 8 atoms, then isomers of polyatomics.
    """
    if ns < 3:
        raise ValueError("need at least 3 species")
    base = [(1, 0), (0, 1), (2, 0), (0, 2), (1, 1)]
    for s in range(3, 9):
        mixed = [(a, s - a) for a in range(s - 1, 0, -1)]
        mixed.sort(key=lambda ab: (abs(ab[0] - ab[1]), -ab[0]))
        base += mixed + [(s, 0), (0, s)]
    poly = [c for c in base if sum(c) >= 3]
    comps = list(base[: ns - 1])
    i = 0
    while len(comps) < ns - 1:
        comps.append(poly[i % len(poly)])
        i += 1
    out = np.zeros((ns, 3), dtype=np.int32)
    out[: ns - 1, :2] = np.array(comps, dtype=np.int32)
    out[ns - 1] = (0, 0, 2)
    return out


# --------------------------------------------------------------------------
# thermo tables
# --------------------------------------------------------------------------
def _cp_model(T, clo, chi, theta):
    """Smooth model heat capacity cp/R rising from clo (300 K) to chi (3000 K)."""
    T = np.asarray(T, dtype=np.float64)
    num = 1.0 - np.exp(-(T - 300.0) / theta)
    den = 1.0 - np.exp(-2700.0 / theta)
    return clo + (chi - clo) * num / den


def _nasa_h_over_r(a, T):
    """Antiderivative of the NASA cp/R polynomial: H/R (K) incl. the a5 constant."""
    return (a[0] * T + a[1] * T**2 / 2 + a[2] * T**3 / 3 + a[3] * T**4 / 4
            + a[4] * T**5 / 5 + a[5])


def _nasa_s_over_r(a, T):
    """Antiderivative of (cp/R)/T: S/R incl. the a6 constant."""
    return (a[0] * math.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3
            + a[4] * T**4 / 4 + a[6])


def _fit_nasa(clo, chi, theta, h298, s298):
    """Two-range NASA-7 fit with cp, H and S continuous at T_MID.

    cp/R is fitted by least squares on 64 points per range with the constraint
    cp_lo(T_MID) = cp_hi(T_MID); a5 / a6 of the low range reproduce the
    requested H(298.15)/R and S(298.15)/R, those of the high range make H and
    S continuous at T_MID.
    """
    Tl = np.linspace(T_FIT_LO, T_MID, 64)
    Th = np.linspace(T_MID, T_FIT_HI, 64)
    sc = 1000.0
    Al = np.vander(Tl / sc, 5, increasing=True)
    Ah = np.vander(Th / sc, 5, increasing=True)
    yl = _cp_model(Tl, clo, chi, theta)
    yh = _cp_model(Th, clo, chi, theta)
    # KKT system for min |Al cl - yl|^2 + |Ah ch - yh|^2  s.t.  b.cl - b.ch = 0
    b = np.vander(np.array([T_MID / sc]), 5, increasing=True)[0]
    K = np.zeros((11, 11))
    K[:5, :5] = 2 * Al.T @ Al
    K[5:10, 5:10] = 2 * Ah.T @ Ah
    K[10, :5] = b
    K[10, 5:10] = -b
    K[:5, 10] = b
    K[5:10, 10] = -b
    rhs = np.concatenate([2 * Al.T @ yl, 2 * Ah.T @ yh, [0.0]])
    sol = np.linalg.solve(K, rhs)
    scale = sc ** -np.arange(5)
    lo = np.zeros(7)
    hi = np.zeros(7)
    lo[:5] = sol[:5] * scale
    hi[:5] = sol[5:10] * scale
    t0 = 298.15
    lo[5] = 0.0
    lo[5] = h298 - _nasa_h_over_r(lo, t0)
    lo[6] = 0.0
    lo[6] = s298 - _nasa_s_over_r(lo, t0)
    hi[5] = 0.0
    hi[5] = _nasa_h_over_r(lo, T_MID) - _nasa_h_over_r(hi, T_MID)
    hi[6] = 0.0
    hi[6] = _nasa_s_over_r(lo, T_MID) - _nasa_s_over_r(hi, T_MID)
    return lo, hi


def species_h_over_r(mech: dict, T: float) -> np.ndarray:
    """H/R (K) of every species at T from its NASA-7 table (setup helper)."""
    out = np.empty(mech["n_species"])
    for k in range(mech["n_species"]):
        a = mech["nasa_lo"][k] if T < mech["t_mid"][k] else mech["nasa_hi"][k]
        out[k] = _nasa_h_over_r(a, T)
    return out


# --------------------------------------------------------------------------
# transport tables (kinetic theory -> ln T fits)
# --------------------------------------------------------------------------
def omega11(tstar):
    """Reduced collision integral Omega(1,1)* for the Lennard-Jones 12-6 potential.

    Neufeld, Janzen & Aziz (1972), eq. (10) with their Table I constants.
    """
    t = np.asarray(tstar, dtype=np.float64)
    return (1.06036 / t**0.15610 + 0.19300 / np.exp(0.47635 * t)
            + 1.03587 / np.exp(1.52996 * t) + 1.76474 / np.exp(3.89411 * t))


def omega22(tstar):
    """Reduced collision integral Omega(2,2)* (Neufeld, Janzen & Aziz 1972, eq. 11)."""
    t = np.asarray(tstar, dtype=np.float64)
    return (1.16145 / t**0.14874 + 0.52487 / np.exp(0.77320 * t)
            + 2.16178 / np.exp(2.43787 * t)
            - 6.435e-4 * t**0.14874 * np.sin(18.0323 * t**-0.76830 - 7.27371))


def _zrot_f(T, eps):
    x = eps / T
    return (1.0 + 0.5 * math.pi**1.5 * np.sqrt(x) + (math.pi**2 / 4 + 2.0) * x
            + math.pi**1.5 * x**1.5)


def _pure_viscosity(T, W, sigma_cm, eps):
    m = W / N_AVOGADRO
    return (5.0 / 16.0) * np.sqrt(math.pi * m * K_BOLTZ * T) / (
        math.pi * sigma_cm**2 * omega22(T / eps))


def _binary_diffusion_1atm(T, Wj, Wk, sj_cm, sk_cm, ej, ek):
    """D_jk at one atmosphere; T broadcasts against the species arguments."""
    mjk = (Wj / N_AVOGADRO) * (Wk / N_AVOGADRO) / ((Wj + Wk) / N_AVOGADRO)
    sjk = 0.5 * (sj_cm + sk_cm)
    ejk = np.sqrt(ej * ek)
    return (3.0 / 16.0) * np.sqrt(2.0 * math.pi * K_BOLTZ**3 * T**3 / mjk) / (
        P_ATM * math.pi * sjk**2 * omega11(T / ejk))


def _pure_conductivity(T, W, eta, rhoD_over_eta, cv_over_r, natoms, zrot298, eps):
    """Warnatz split with the Parker / Brau-Jonkman rotational relaxation number.

    The rotational term follows the Chemkin transport manual form
    B = Z_rot + (2/pi)(5/3 Cv_rot/R + rho D_kk / eta_k); App. A.3 prints this
    term garbled, and the table it feeds is setup data only.
    """
    R = R_GAS
    if natoms == 1:
        return eta / W * 2.5 * 1.5 * R
    cv_trans = 1.5 * R
    if natoms == 2:
        cv_rot = R
        cv_vib = np.maximum(cv_over_r * R - 2.5 * R, 0.0)
    else:
        cv_rot = 1.5 * R
        cv_vib = np.maximum(cv_over_r * R - 3.0 * R, 0.0)
    zrot = zrot298 * _zrot_f(298.0, eps) / _zrot_f(T, eps)
    A = 2.5 - rhoD_over_eta
    B = zrot + (2.0 / math.pi) * (5.0 / 3.0 * cv_rot / R + rhoD_over_eta)
    f_trans = 2.5 * (1.0 - (2.0 / math.pi) * (cv_rot / cv_trans) * (A / B))
    f_rot = rhoD_over_eta * (1.0 + (2.0 / math.pi) * (A / B))
    f_vib = rhoD_over_eta
    return eta / W * (f_trans * cv_trans + f_rot * cv_rot + f_vib * cv_vib)


def _weighted_polyfit(u, y, order):
    """Relative-weight least squares fit, batched over the leading axes of y.

    y: [..., G] samples on the grid u[G]; returns coefficients [..., order]
    (constant term first) of the polynomial in u.
    """
    V = np.vander(u, order, increasing=True)            # [G, order]
    w2 = 1.0 / (y * y)                                  # relative weights
    M = np.einsum("...g,gi,gj->...ij", w2, V, V)
    rhs = np.einsum("...g,gi,...g->...i", w2, V, y)
    return np.linalg.solve(M, rhs[..., None])[..., 0]


def transport_fit_grid():
    """The 64 temperatures (log-spaced on [T_FIT_LO, T_FIT_HI]) the fits use."""
    return np.exp(np.linspace(math.log(T_FIT_LO), math.log(T_FIT_HI), 64))


def transport_fits(W, sigma_cm, eps, zrot298, natoms, cp_over_r, diff_fit_kind: int = 1,
                   order: int = FIT_ORDER):
    """ln T polynomial fits (App. A.3 "Polynomial fits", in the centred variable
    u) of the pure-species viscosity and conductivity and of the binary
    diffusion coefficients at 1 atm (or their reciprocals, diff_fit_kind 1),
    from Lennard-Jones kinetic theory on the grid of transport_fit_grid().

    W[ns] g/mol, sigma_cm[ns], eps[ns] (epsilon/k, K), zrot298[ns], natoms[ns]
    (1 atom, 2 linear, >= 3 nonlinear), cp_over_r[ns, 64] on the grid.
    Returns visc_fit[ns, order], cond_fit[ns, order], diff_fit[ns, ns, order]
    (order coefficients, constant term first).
    """
    ns = len(W)
    Tg = transport_fit_grid()
    ug = (np.log(Tg) - FIT_L0) / FIT_H
    eta = np.empty((ns, Tg.size))
    lam = np.empty((ns, Tg.size))
    Dg = _binary_diffusion_1atm(Tg[None, None, :], W[:, None, None], W[None, :, None],
                                sigma_cm[:, None, None], sigma_cm[None, :, None],
                                eps[:, None, None], eps[None, :, None])
    for k in range(ns):
        eta[k] = _pure_viscosity(Tg, W[k], sigma_cm[k], eps[k])
        rho = P_ATM * W[k] / (R_GAS * Tg)
        rhoD_eta = rho * Dg[k, k] / eta[k]
        cv_r = cp_over_r[k] - 1.0
        lam[k] = _pure_conductivity(Tg, W[k], eta[k], rhoD_eta, cv_r, natoms[k],
                                    zrot298[k], eps[k])
    visc_fit = _weighted_polyfit(ug, eta, order)
    cond_fit = _weighted_polyfit(ug, lam, order)
    iu = np.triu_indices(ns)
    target = Dg[iu] if diff_fit_kind == 0 else 1.0 / Dg[iu]
    dfit_u = _weighted_polyfit(ug, target, order)
    diff_fit = np.empty((ns, ns, order))
    diff_fit[iu] = dfit_u
    diff_fit[(iu[1], iu[0])] = dfit_u
    return visc_fit, cond_fit, diff_fit


# --------------------------------------------------------------------------
# reactions
# --------------------------------------------------------------------------
def _comp_index(comps):
    idx = {}
    for k, c in enumerate(comps):
        idx.setdefault((int(c[0]), int(c[1])), []).append(k)
    return idx


def _association_triples(comps):
    """All (x, y, z) with comp(x) + comp(y) = comp(z), x <= y, reactive species."""
    idx = _comp_index(comps)
    out = []
    for z, cz in enumerate(comps):
        if cz.sum() < 2:
            continue
        for a in range(cz[0] + 1):
            for b in range(cz[1] + 1):
                rest = (int(cz[0] - a), int(cz[1] - b))
                if (a, b) == (0, 0) or rest == (0, 0):
                    continue
                for x in idx.get((a, b), []):
                    for y in idx.get(rest, []):
                        if x <= y:
                            out.append((x, y, z))
    return sorted(set(out))


def _elementary_candidates(comps, rng, count, max_tries=200000):
    """Sample `count` distinct balanced X + Y <=> Z + W reactions."""
    idx = _comp_index(comps)
    nsp = len(comps)
    seen = set()
    out = []
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not sample enough elementary reactions")
        x, y = sorted(rng.integers(0, nsp, size=2).tolist())
        tot = comps[x] + comps[y]
        splits = []
        for a in range(tot[0] + 1):
            for b in range(tot[1] + 1):
                rest = (int(tot[0] - a), int(tot[1] - b))
                if (a, b) == (0, 0) or rest == (0, 0):
                    continue
                for z in idx.get((a, b), []):
                    for w in idx.get(rest, []):
                        if z <= w and (z, w) != (x, y):
                            splits.append((z, w))
        if not splits:
            continue
        z, w = splits[int(rng.integers(0, len(splits)))]
        key = frozenset([(x, y), (z, w)])
        if key in seen:
            continue
        seen.add(key)
        out.append(((x, y), (z, w)))
    return out


@dataclass
class MechSpec:
    """Shape of a synthetic mechanism."""
    n_species: int
    n_elementary: int
    n_threebody: int
    n_lindemann: int
    n_troe: int
    seed: int
    special_cases: bool = False
    # 1: tables hold fits of 1/D_kj, the polynomial the paper's generated
    # routines evaluate directly; 0: fits of D_kj itself (eq:Dkj)
    diff_fit_kind: int = 1
    name: str = ""
    extra: dict = field(default_factory=dict)
    # further reaction forms (App. A.2), made by converting reactions of the
    # base mechanism after all of its draws (the base arrays are unchanged):
    # Troe -> SRI, falloff -> chemically activated, elementary -> PLOG
    n_sri: int = 0
    n_chemact: int = 0
    n_plog: int = 0
    # elementary -> irreversible with explicit forward orders
    n_orders: int = 0
    # species made quasi-steady (linearised QSSA): chosen greedily so that no
    # reaction side holds two QSS molecules, then dropped from the efficiency
    # lists (the third-body sums run over transported species only)
    n_qss: int = 0
    # coefficients of the transport fits (polynomial degree + 1)
    fit_order: int = FIT_ORDER

    @property
    def n_reactions(self) -> int:
        return self.n_elementary + self.n_threebody + self.n_lindemann + self.n_troe


# The three workloads' mechanisms (sizes of Table tab:mech for the first two,
# and a 200-species / 1500-reaction mechanism beyond the paper's largest).
MECH_9 = MechSpec(9, 17, 3, 0, 1, seed=9021, name="syn9")
MECH_53 = MechSpec(53, 266, 30, 0, 29, seed=53325, name="syn53")
MECH_200 = MechSpec(200, 1200, 180, 30, 90, seed=2001500, name="syn200")
# 100 species / 700 reactions (the proportions of the 200-species mechanism):
# the band of 65-128 species, where the kernels take two species per lane
MECH_100 = MechSpec(100, 560, 84, 14, 42, seed=1000700, name="syn100")
# syn53 with part of its reactions in the further forms: 10 SRI, 8 chemically
# activated falloff, 20 pressure-table (PLOG) reactions
MECH_53X = MechSpec(53, 266, 30, 0, 29, seed=53325, name="syn53x", n_sri=10, n_chemact=8,
                    n_plog=20)
# syn53 with 20 irreversible reactions of non-integer forward orders
MECH_53O = MechSpec(53, 266, 30, 0, 29, seed=53325, name="syn53o", n_orders=20)
# syn53 with 6 quasi-steady-state species (the most the greedy choice finds)
MECH_53Q = MechSpec(53, 266, 30, 0, 29, seed=53325, name="syn53q", n_qss=6)
# syn200 with 12 QSS species
MECH_200Q = MechSpec(200, 1200, 180, 30, 90, seed=2001500, name="syn200q", n_qss=12)
# syn53x (SRI, chemically activated, PLOG) with the same 6 QSS species
MECH_53XQ = MechSpec(53, 266, 30, 0, 29, seed=53325, name="syn53xq", n_sri=10, n_chemact=8,
                     n_plog=20, n_qss=6)


def _pick_qss(spec, ns, reac_ptr, reac_sp, reac_nu, prod_ptr, prod_sp, prod_nu, reversible,
              orders, eff_ptr, eff_sp, eff_val):
    """Seeded greedy choice of spec.n_qss quasi-steady species: every reaction
    side keeps at most one QSS molecule, a QSS species is consumed by some
    reaction and takes part in none with explicit orders.  The chosen species
    leave the efficiency lists.  Returns (qss flags, eff_ptr, eff_sp, eff_val)."""
    rng = np.random.Generator(np.random.PCG64(spec.seed + 9999))
    nr = len(reac_ptr) - 1
    sides = []
    for i in range(nr):
        r = {int(k): int(v) for k, v in zip(reac_sp[reac_ptr[i]:reac_ptr[i + 1]],
                                             reac_nu[reac_ptr[i]:reac_ptr[i + 1]])}
        q = {int(k): int(v) for k, v in zip(prod_sp[prod_ptr[i]:prod_ptr[i + 1]],
                                             prod_nu[prod_ptr[i]:prod_ptr[i + 1]])}
        sides.append((r, q))
    banned = set()
    if orders is not None:
        optr, osp = orders["ord_ptr"], orders["ord_sp"]
        for i in range(nr):
            if optr[i + 1] > optr[i]:
                banned |= set(sides[i][0]) | set(sides[i][1])
                banned |= set(int(k) for k in osp[optr[i]:optr[i + 1]])
    # the species in the fewest reactions first (the minor species a reduced
    # mechanism makes quasi-steady), ties in seeded random order
    degree = np.zeros(ns, np.int64)
    for r, p in sides:
        for k in set(r) | set(p):
            degree[k] += 1
    tie = rng.permutation(ns)
    order = sorted(range(ns - 1), key=lambda k: (degree[k], tie[k]))  # bath stays
    chosen = []
    for q in order:
        if len(chosen) == spec.n_qss:
            break
        if q in banned:
            continue
        trial = set(chosen) | {q}
        if any(sum(v for k, v in side.items() if k in trial) > 1
               for r, p in sides for side in (r, p)):
            continue
        consumed = any((r.get(q, 0) > p.get(q, 0)) or (p.get(q, 0) > r.get(q, 0) and
                                                        reversible[i])
                       for i, (r, p) in enumerate(sides))
        if consumed:
            chosen.append(q)
    if len(chosen) < spec.n_qss:
        raise RuntimeError("could not choose that many QSS species")
    qss = np.zeros(ns, np.int32)
    qss[chosen] = 1
    ptr, sp, val = [0], [], []
    for i in range(nr):
        for e in range(eff_ptr[i], eff_ptr[i + 1]):
            if not qss[eff_sp[e]]:
                sp.append(int(eff_sp[e]))
                val.append(float(eff_val[e]))
        ptr.append(len(sp))
    return qss, np.array(ptr, np.int32), np.array(sp, np.int32), np.array(val, np.float64)


def make_mechanism(spec: MechSpec) -> dict:
    """Build a seeded synthetic mechanism descriptor (numpy arrays, cgs units).

    Keys mirror the fields of ``kx_mech_desc``; extra keys starting with an
    underscore carry generator metadata used by tests (targets of the thermo
    fit, Lennard-Jones parameters, species names).
    """
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    ns = spec.n_species
    comps = _species_compositions(ns)
    W = comps @ ELEMENT_MASS
    natoms = comps.sum(axis=1)

    # ---- thermo
    clo = np.empty(ns)
    chi = np.empty(ns)
    theta = np.empty(ns)
    h298 = np.empty(ns)
    s298 = np.empty(ns)
    for k in range(ns):
        if natoms[k] == 1:
            clo[k] = chi[k] = 2.5
            theta[k] = 1000.0
        elif k == ns - 1:
            clo[k], chi[k], theta[k] = 3.5, 4.5, 900.0
        else:
            clo[k] = rng.uniform(2.5, 4.0)
            chi[k] = rng.uniform(4.0, 9.0)
            theta[k] = rng.uniform(400.0, 1500.0)
        homonuclear_diatomic = natoms[k] == 2 and (comps[k] == 2).any()
        h298[k] = 0.0 if homonuclear_diatomic else rng.uniform(-3.0e4, 3.0e4)
        s298[k] = rng.uniform(15.0, 35.0)
    nasa_lo = np.empty((ns, 7))
    nasa_hi = np.empty((ns, 7))
    for k in range(ns):
        nasa_lo[k], nasa_hi[k] = _fit_nasa(clo[k], chi[k], theta[k], h298[k], s298[k])
    t_mid = np.full(ns, T_MID)

    # ---- reactions
    reactive = comps[: ns - 1, :2]
    mech_tmp = {"n_species": ns, "nasa_lo": nasa_lo, "nasa_hi": nasa_hi, "t_mid": t_mid}
    h1000 = species_h_over_r(mech_tmp, 1000.0)

    triples = _association_triples(reactive)
    n_assoc = spec.n_threebody + spec.n_lindemann + spec.n_troe
    if len(triples) < n_assoc:
        raise RuntimeError("not enough association reactions for this species set")
    pick = rng.choice(len(triples), size=n_assoc, replace=False)
    assoc = [triples[i] for i in pick]
    elem = _elementary_candidates(reactive, rng, spec.n_elementary)

    rxns = []  # (type, reactants list, products list)
    for (x, y), (z, w) in elem:
        rxns.append([RXN_ELEMENTARY, [x, y], [z, w]])
    types = ([RXN_THREEBODY] * spec.n_threebody + [RXN_LINDEMANN] * spec.n_lindemann
             + [RXN_TROE] * spec.n_troe)
    for t, (x, y, z) in zip(types, assoc):
        rxns.append([t, [x, y], [z]])
    # orient every reaction exothermic at 1000 K so that k_r stays bounded
    for r in rxns:
        dh = sum(h1000[k] for k in r[2]) - sum(h1000[k] for k in r[1])
        if dh > 0:
            r[1], r[2] = r[2], r[1]
    order = rng.permutation(len(rxns))
    rxns = [rxns[i] for i in order]
    nr = len(rxns)

    def csr(lists):
        ptr = [0]
        sp, nu = [], []
        for lst in lists:
            uniq, cnt = np.unique(np.array(lst, dtype=np.int64), return_counts=True)
            sp += uniq.tolist()
            nu += cnt.tolist()
            ptr.append(len(sp))
        return (np.array(ptr, np.int32), np.array(sp, np.int32), np.array(nu, np.int32))

    reac_ptr, reac_sp, reac_nu = csr([r[1] for r in rxns])
    prod_ptr, prod_sp, prod_nu = csr([r[2] for r in rxns])
    rtype = np.array([r[0] for r in rxns], np.int32)

    A = 10.0 ** rng.uniform(8.0, 18.0, nr)
    beta = rng.uniform(-2.0, 2.0, nr)
    Ea = rng.uniform(0.0, 40000.0, nr)
    A0 = np.zeros(nr)
    beta0 = np.zeros(nr)
    Ea0 = np.zeros(nr)
    troe = np.zeros((nr, 4))
    eff_ptr = [0]
    eff_sp, eff_val = [], []
    eff_default = np.ones(nr)
    for i in range(nr):
        if rtype[i] in (RXN_LINDEMANN, RXN_TROE):
            A0[i] = A[i] * 10.0 ** rng.uniform(3.0, 6.0)
            beta0[i] = rng.uniform(-2.0, 2.0)
            Ea0[i] = rng.uniform(0.0, Ea[i])
        if rtype[i] == RXN_TROE:
            troe[i, 0] = rng.uniform(0.1, 0.9)
            troe[i, 1] = rng.uniform(50.0, 500.0)
            troe[i, 2] = rng.uniform(500.0, 5000.0)
            troe[i, 3] = rng.uniform(2000.0, 8000.0) if rng.random() < 0.5 else np.nan
        if rtype[i] != RXN_ELEMENTARY:
            m = min(6, ns)
            sub = np.sort(rng.choice(ns, size=m, replace=False))
            eff_sp += sub.tolist()
            eff_val += rng.uniform(0.5, 12.0, m).tolist()
        eff_ptr.append(len(eff_sp))

    if spec.special_cases:
        elem_ids = np.flatnonzero(rtype == RXN_ELEMENTARY)
        n0 = int(round(0.27 * nr))
        nint = max(1, int(round(0.006 * nr)))
        nshare = int(round(0.21 * nr))
        sel = rng.permutation(elem_ids)
        zero = sel[:n0]
        ints = sel[n0:n0 + nint]
        beta[zero] = 0.0
        Ea[zero] = 0.0
        beta[ints] = rng.choice([-1.0, 1.0, 2.0], size=len(ints))
        Ea[ints] = 0.0
        others = np.setdiff1d(np.arange(nr), np.concatenate([zero, ints]))
        share = rng.permutation(others)[:nshare]
        donors = rng.choice(others, size=len(share))
        beta[share] = beta[donors]
        Ea[share] = Ea[donors]

    # ---- transport tables
    sigma = rng.uniform(2.5, 5.5, ns) * 1e-8     # cm
    eps = rng.uniform(30.0, 600.0, ns)           # K (epsilon / k_B)
    zrot = rng.uniform(0.0, 4.0, ns)
    Tg = transport_fit_grid()
    cp_r = np.stack([_cp_model(Tg, clo[k], chi[k], theta[k]) for k in range(ns)])
    visc_fit, cond_fit, diff_fit = transport_fits(W, sigma, eps, zrot, natoms, cp_r,
                                                  spec.diff_fit_kind, spec.fit_order)

    sri = chem_act = plog = orders = None
    reversible = np.ones(nr, np.int32)
    if spec.n_orders:
        rng3 = np.random.Generator(np.random.PCG64(spec.seed + 8888))
        elem_ids = np.flatnonzero(rtype == RXN_ELEMENTARY)
        optr, osp, oval = [0], [], []
        conv = set(rng3.choice(elem_ids, size=spec.n_orders, replace=False).tolist())
        for i in range(nr):
            if i in conv:
                reversible[i] = 0
                reac = reac_sp[reac_ptr[i]:reac_ptr[i + 1]]
                for k, nu in zip(reac, reac_nu[reac_ptr[i]:reac_ptr[i + 1]]):
                    osp.append(int(k))
                    oval.append(float(nu) * rng3.uniform(0.5, 1.5))
                if rng3.random() < 0.5:   # a species that is not a reactant
                    cand = [k for k in range(ns - 1) if k not in reac]
                    osp.append(int(rng3.choice(cand)))
                    oval.append(rng3.uniform(0.1, 0.5))
            optr.append(len(osp))
        orders = {"ord_ptr": np.array(optr, np.int32), "ord_sp": np.array(osp, np.int32),
                  "ord_val": np.array(oval)}
    if spec.n_sri or spec.n_chemact or spec.n_plog:
        rng2 = np.random.Generator(np.random.PCG64(spec.seed + 7777))
        troe_ids = np.flatnonzero(rtype == RXN_TROE)
        if spec.n_sri > len(troe_ids):
            raise ValueError("n_sri exceeds the number of Troe reactions")
        sri = np.zeros((nr, 5))
        for i in rng2.choice(troe_ids, size=spec.n_sri, replace=False):
            rtype[i] = RXN_SRI
            troe[i] = 0.0
            # a, b (K), c (K; a very large c drops the second term to 1), d, e
            sri[i] = (rng2.uniform(0.1, 2.0), rng2.uniform(0.0, 2000.0),
                      rng2.uniform(100.0, 3000.0) if rng2.random() < 0.7 else 1e30,
                      rng2.uniform(0.5, 2.0), rng2.uniform(-0.5, 0.5))
        falloff = np.flatnonzero((rtype == RXN_LINDEMANN) | (rtype == RXN_TROE)
                                 | (rtype == RXN_SRI))
        if spec.n_chemact > len(falloff):
            raise ValueError("n_chemact exceeds the number of falloff reactions")
        chem_act = np.zeros(nr, np.int32)
        chem_act[rng2.choice(falloff, size=spec.n_chemact, replace=False)] = 1
        elem_ids = np.flatnonzero(rtype == RXN_ELEMENTARY)
        if spec.n_plog > len(elem_ids):
            raise ValueError("n_plog exceeds the number of elementary reactions")
        conv = set(rng2.choice(elem_ids, size=spec.n_plog, replace=False).tolist())
        pptr, pp, pA, pb, pE = [0], [], [], [], []
        for i in range(nr):
            if i in conv:
                rtype[i] = RXN_PLOG
                npt = int(rng2.integers(1, 5))
                pres = np.sort(10.0 ** rng2.uniform(-1.0, 2.0, npt)) * P_ATM
                pres = np.unique(pres)
                for q in pres:
                    pp.append(q)
                    pA.append(A[i] * 10.0 ** rng2.uniform(-1.0, 1.0))
                    pb.append(beta[i] + rng2.uniform(-0.3, 0.3))
                    pE.append(Ea[i] * rng2.uniform(0.8, 1.2))
            pptr.append(len(pp))
        plog = {"plog_ptr": np.array(pptr, np.int32), "plog_p": np.array(pp),
                "plog_A": np.array(pA), "plog_beta": np.array(pb), "plog_Ea": np.array(pE)}

    qss = None
    eff_ptr = np.array(eff_ptr, np.int32)
    eff_sp = np.array(eff_sp, np.int32)
    eff_val = np.array(eff_val, np.float64)
    if spec.n_qss:
        qss, eff_ptr, eff_sp, eff_val = _pick_qss(
            spec, ns, reac_ptr, reac_sp, reac_nu, prod_ptr, prod_sp, prod_nu, reversible,
            orders, eff_ptr, eff_sp, eff_val)

    return {
        "name": spec.name,
        "n_species": ns,
        "n_reactions": nr,
        "n_elements": 3,
        "elem_mass": ELEMENT_MASS.copy(),
        "composition": comps,
        "nasa_lo": nasa_lo,
        "nasa_hi": nasa_hi,
        "t_mid": t_mid,
        "rxn_type": rtype,
        "reversible": reversible,
        "reac_ptr": reac_ptr, "reac_sp": reac_sp, "reac_nu": reac_nu,
        "prod_ptr": prod_ptr, "prod_sp": prod_sp, "prod_nu": prod_nu,
        "A": A, "beta": beta, "Ea": Ea,
        "A0": A0, "beta0": beta0, "Ea0": Ea0,
        "troe": troe,
        "eff_ptr": eff_ptr,
        "eff_sp": eff_sp,
        "eff_val": eff_val,
        "eff_default": eff_default,
        "fit_order": spec.fit_order,
        "fit_L0": FIT_L0,
        "fit_h": FIT_H,
        "diff_fit_kind": spec.diff_fit_kind,
        "visc_fit": visc_fit,
        "cond_fit": cond_fit,
        "diff_fit": diff_fit,
        "sri": sri,
        "chem_act": chem_act,
        **(plog if plog is not None else
           {"plog_ptr": None, "plog_p": None, "plog_A": None, "plog_beta": None,
            "plog_Ea": None}),
        **(orders if orders is not None else
           {"ord_ptr": None, "ord_sp": None, "ord_val": None}),
        "qss": qss,
        # generator metadata (not part of the descriptor)
        "_h298_over_r": h298,
        "_s298_over_r": s298,
        "_cp_model": np.stack([clo, chi, theta], axis=1),
        "_sigma_cm": sigma,
        "_eps_k": eps,
        "_zrot298": zrot,
        "_seed": spec.seed,
    }


# --------------------------------------------------------------------------
# states
# --------------------------------------------------------------------------
@dataclass
class StateSpec:
    n_points: int
    seed: int
    T_range: tuple = (300.0, 2800.0)
    p_atm_range: tuple = (1.0, 1.0)
    dirichlet_alpha: float = 1.0


STATES_9 = StateSpec(4096, seed=1)
STATES_53 = StateSpec(1 << 20, seed=2, p_atm_range=(1.0, 40.0), dirichlet_alpha=0.3)
STATES_53_MIXED = StateSpec(1 << 22, seed=3, p_atm_range=(1.0, 40.0), dirichlet_alpha=0.3)
STATES_200 = StateSpec(1 << 20, seed=4, p_atm_range=(1.0, 40.0), dirichlet_alpha=0.3)


def make_states(n_species: int, spec: StateSpec, n_points: int | None = None):
    """Seeded states in the structure-of-arrays layout used by the library.

    Returns (T[n], p[n], Y[n_species, n]) as float64 numpy arrays (p in
    dyn/cm^2).  ``n_points`` overrides the spec's count while keeping the same
    random stream prefix for T and p.
    """
    n = spec.n_points if n_points is None else n_points
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    T = rng.uniform(spec.T_range[0], spec.T_range[1], n)
    p = rng.uniform(spec.p_atm_range[0], spec.p_atm_range[1], n) * P_ATM
    g = rng.gamma(spec.dirichlet_alpha, 1.0, size=(n, n_species))
    g /= g.sum(axis=1, keepdims=True)
    Y = np.ascontiguousarray(g.T)
    return T, p, Y
