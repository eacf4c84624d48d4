"""Python access to the plain FP64 CPU oracle (``kx_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this module; the library never does.  It marshals the
generator's mechanism arrays into the oracle's own struct and calls the C
functions; it also builds constructed-equilibrium states (from the oracle's
own Gibbs energies) for the equilibrium pin and the mixed-precision workload.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kx_oracle.c")
_LIB = os.path.join(_HERE, "libkx_oracle.so")

RU = 8.31446261815324e7
PATM = 1013250.0


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable x86-64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _Mech(C.Structure):
    _fields_ = [
        ("ns", C.c_int32), ("nr", C.c_int32), ("ne", C.c_int32),
        ("elem_mass", _dp), ("comp", _ip), ("nasa_lo", _dp), ("nasa_hi", _dp),
        ("t_mid", _dp), ("rtype", _ip), ("rev", _ip),
        ("reac_ptr", _ip), ("reac_sp", _ip), ("reac_nu", _ip),
        ("prod_ptr", _ip), ("prod_sp", _ip), ("prod_nu", _ip),
        ("A", _dp), ("beta", _dp), ("Ea", _dp),
        ("A0", _dp), ("beta0", _dp), ("Ea0", _dp), ("troe", _dp),
        ("eff_ptr", _ip), ("eff_sp", _ip), ("eff_val", _dp), ("eff_default", _dp),
        ("fit_order", C.c_int32), ("fit_L0", C.c_double), ("fit_h", C.c_double),
        ("diff_kind", C.c_int32),
        ("visc_fit", _dp), ("cond_fit", _dp), ("diff_fit", _dp),
        ("sri", _dp), ("chem_act", _ip), ("plog_ptr", _ip), ("plog_p", _dp),
        ("plog_A", _dp), ("plog_beta", _dp), ("plog_Ea", _dp),
        ("ord_ptr", _ip), ("ord_sp", _ip), ("ord_val", _dp),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        L.kxo_thermo.argtypes = [vp, C.c_double, vp, vp, vp, vp]
        L.kxo_mixture_thermo.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp]
        L.kxo_production_rates.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp]
        L.kxo_rates_detail.argtypes = [vp, C.c_double, C.c_double, vp, vp, vp, vp, vp, vp]
        L.kxo_rate_constants.argtypes = [vp, C.c_double, C.c_double, vp, vp]
        L.kxo_troe_F.argtypes = [vp, C.c_double, C.c_double]
        L.kxo_troe_F.restype = C.c_double
        L.kxo_sri_F.argtypes = [vp, C.c_double, C.c_double]
        L.kxo_sri_F.restype = C.c_double
        L.kxo_pure_transport.argtypes = [vp, C.c_double, C.c_double, vp, vp, vp]
        L.kxo_wilke_phi.argtypes = [vp, C.c_double, C.c_int, C.c_int]
        L.kxo_wilke_phi.restype = C.c_double
        L.kxo_transport.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp]
        L.kxo_jacobian.argtypes = [vp, C.c_int64, vp, vp, vp, vp]
        L.kxo_qss_rates.argtypes = [vp, vp, C.c_int64, vp, vp, vp, vp, vp, vp]
        L.kxo_qss_system.argtypes = [vp, vp, C.c_double, C.c_double, vp, vp, vp]
        L.kxo_set_threads.argtypes = [C.c_int]
        L.kxo_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OracleMech:
    """Keeps contiguous copies of a mechanism's arrays alive for the C struct."""

    def __init__(self, mech: dict):
        self.mech = mech
        f64 = lambda k: np.ascontiguousarray(mech[k], dtype=np.float64)
        i32 = lambda k: np.ascontiguousarray(mech[k], dtype=np.int32)
        self._keep = {}
        s = _Mech()
        s.ns, s.nr, s.ne = mech["n_species"], mech["n_reactions"], mech["n_elements"]
        names_f = ["elem_mass", "nasa_lo", "nasa_hi", "t_mid", "A", "beta", "Ea", "A0",
                   "beta0", "Ea0", "troe", "eff_val", "eff_default", "visc_fit",
                   "cond_fit", "diff_fit"]
        names_i = ["composition", "rxn_type", "reversible", "reac_ptr", "reac_sp",
                   "reac_nu", "prod_ptr", "prod_sp", "prod_nu", "eff_ptr", "eff_sp"]
        field_of = {"composition": "comp", "rxn_type": "rtype", "reversible": "rev"}
        for k in names_f:
            a = f64(k)
            self._keep[k] = a
            setattr(s, field_of.get(k, k), a.ctypes.data_as(_dp))
        for k in names_i:
            a = i32(k)
            self._keep[k] = a
            setattr(s, field_of.get(k, k), a.ctypes.data_as(_ip))
        for k, conv, ptr in (("sri", f64, _dp), ("plog_p", f64, _dp), ("plog_A", f64, _dp),
                             ("plog_beta", f64, _dp), ("plog_Ea", f64, _dp),
                             ("chem_act", i32, _ip), ("plog_ptr", i32, _ip),
                             ("ord_ptr", i32, _ip), ("ord_sp", i32, _ip), ("ord_val", f64, _dp)):
            if mech.get(k) is None:
                setattr(s, k, None)
                continue
            a = conv(k)
            self._keep[k] = a
            setattr(s, k, a.ctypes.data_as(ptr))
        s.fit_order = int(mech["fit_order"])
        s.fit_L0 = float(mech["fit_L0"])
        s.fit_h = float(mech["fit_h"])
        s.diff_kind = int(mech["diff_fit_kind"])
        self.struct = s
        self.ns = s.ns
        self.nr = s.nr

    @property
    def ref(self):
        return C.byref(self.struct)

    # ---------------------------------------------------------------- thermo
    def thermo(self, T: float):
        ns = self.ns
        out = [np.empty(ns) for _ in range(4)]
        lib().kxo_thermo(self.ref, float(T), *[_ptr(a) for a in out])
        return tuple(out)  # cp/R, H/RT, S/R, G/RT

    def mixture_thermo(self, T, Y):
        T = np.ascontiguousarray(T, np.float64)
        Y = np.ascontiguousarray(Y, np.float64)
        n = T.size
        cpk = np.empty((self.ns, n))
        hk = np.empty((self.ns, n))
        cp = np.empty(n)
        lib().kxo_mixture_thermo(self.ref, n, _ptr(T), _ptr(Y), _ptr(cpk), _ptr(hk), _ptr(cp))
        return cpk, hk, cp

    # ---------------------------------------------------------------- rates
    def production_rates(self, T, p, Y, with_scale: bool = True):
        T = np.ascontiguousarray(T, np.float64)
        p = np.ascontiguousarray(p, np.float64)
        Y = np.ascontiguousarray(Y, np.float64)
        n = T.size
        assert Y.shape == (self.ns, n)
        wdot = np.empty((self.ns, n))
        scale = np.empty((self.ns, n)) if with_scale else None
        lib().kxo_production_rates(self.ref, n, _ptr(T), _ptr(p), _ptr(Y), _ptr(wdot),
                                   _ptr(scale))
        return (wdot, scale) if with_scale else wdot

    def rates_detail(self, T: float, p: float, Y):
        Y = np.ascontiguousarray(Y, np.float64)
        ns, nr = self.ns, self.nr
        wdot, scale = np.empty(ns), np.empty(ns)
        qf, qr, c = np.empty(nr), np.empty(nr), np.empty(nr)
        lib().kxo_rates_detail(self.ref, float(T), float(p), _ptr(Y), _ptr(wdot),
                               _ptr(scale), _ptr(qf), _ptr(qr), _ptr(c))
        return dict(wdot=wdot, scale=scale, qf=qf, qr=qr, c=c)

    def rate_constants(self, T: float, p: float = PATM):
        """k_f (k_inf for falloff reactions; the interpolated k_f of a pressure
        table at p) and k_0 (falloff only) at temperature T."""
        kf, k0 = np.empty(self.nr), np.empty(self.nr)
        lib().kxo_rate_constants(self.ref, float(T), float(p), _ptr(kf), _ptr(k0))
        return kf, k0

    def jacobian(self, T, p, Y):
        """jac[n, ns, ns]: d wdot_k / d C_j at fixed T (complex step)."""
        T = np.ascontiguousarray(T, np.float64)
        p = np.ascontiguousarray(p, np.float64)
        Y = np.ascontiguousarray(Y, np.float64)
        n = T.size
        jac = np.empty((n, self.ns, self.ns))
        lib().kxo_jacobian(self.ref, n, _ptr(T), _ptr(p), _ptr(Y), _ptr(jac))
        return jac

    def qss_rates(self, T, p, Y, with_scale: bool = True):
        """Rates of a mechanism whose ``qss`` flags mark quasi-steady species:
        (wdot[ns, n], scale[ns, n] or None, Cq[nq, n]).  QSS rows of wdot hold
        the residual of their balance; QSS entries of Y are not read."""
        qss = np.ascontiguousarray(self.mech["qss"], dtype=np.int32)
        nq = int(np.count_nonzero(qss))
        T = np.ascontiguousarray(T, np.float64)
        p = np.ascontiguousarray(p, np.float64)
        Y = np.ascontiguousarray(Y, np.float64)
        n = T.size
        assert Y.shape == (self.ns, n) and qss.shape == (self.ns,)
        wdot = np.empty((self.ns, n))
        scale = np.empty((self.ns, n)) if with_scale else None
        Cq = np.empty((nq, n))
        lib().kxo_qss_rates(self.ref, _ptr(qss), n, _ptr(T), _ptr(p), _ptr(Y), _ptr(wdot),
                            _ptr(scale), _ptr(Cq))
        return wdot, scale, Cq

    def qss_system(self, T: float, p: float, Y):
        """(A[nq, nq], b[nq]) of the QSS balances wdot_Q = A C_Q + b at one point."""
        qss = np.ascontiguousarray(self.mech["qss"], dtype=np.int32)
        nq = int(np.count_nonzero(qss))
        Y = np.ascontiguousarray(Y, np.float64)
        A, b = np.empty((nq, nq)), np.empty(nq)
        lib().kxo_qss_system(self.ref, _ptr(qss), float(T), float(p), _ptr(Y), _ptr(A), _ptr(b))
        return A, b

    # ---------------------------------------------------------------- transport
    def pure_transport(self, T: float, p: float):
        ns = self.ns
        eta, lam, D = np.empty(ns), np.empty(ns), np.empty((ns, ns))
        lib().kxo_pure_transport(self.ref, float(T), float(p), _ptr(eta), _ptr(lam), _ptr(D))
        return eta, lam, D

    def wilke_phi(self, T: float, k: int, j: int) -> float:
        return lib().kxo_wilke_phi(self.ref, float(T), int(k), int(j))

    def transport(self, T, p, Y):
        T = np.ascontiguousarray(T, np.float64)
        p = np.ascontiguousarray(p, np.float64)
        Y = np.ascontiguousarray(Y, np.float64)
        n = T.size
        mu, lam = np.empty(n), np.empty(n)
        Dm = np.empty((self.ns, n))
        lib().kxo_transport(self.ref, n, _ptr(T), _ptr(p), _ptr(Y), _ptr(mu), _ptr(lam),
                            _ptr(Dm))
        return mu, lam, Dm


def troe_F(params4, T: float, Pr: float) -> float:
    a = np.ascontiguousarray(params4, np.float64)
    return lib().kxo_troe_F(_ptr(a), float(T), float(Pr))


def sri_F(params5, T: float, Pr: float) -> float:
    a = np.ascontiguousarray(params5, np.float64)
    return lib().kxo_sri_F(_ptr(a), float(T), float(Pr))


def set_threads(n: int) -> None:
    lib().kxo_set_threads(int(n))


def max_threads() -> int:
    return lib().kxo_max_threads()


# ------------------------------------------------------------------------
# constructed equilibrium states (test-input construction, not the method)
# ------------------------------------------------------------------------
def equilibrium_states(om: OracleMech, n: int, seed: int, T_range=(300.0, 2800.0),
                       p_atm_range=(1.0, 40.0), perturb: float = 1e-6):
    """States whose reactive species sit at chemical equilibrium.

    With element potentials lam_e, C_k = (p_atm/RT) exp(-G_k/RT + sum_e lam_e a_ke)
    makes prod_k C_k^nu_ki = K_c,i for every element-balanced reaction
    (eq:K_p with K_c = K_p (p_atm/RT)^(sum nu)), so q_f = q_r.  The anchors are
    the two homonuclear diatomics (species 2 and 3) with X ~ U[0.05, 0.3]; the
    inert diluent (last species) fills the remaining pressure.  Each Y_k is
    then multiplied by (1 + perturb * U[-1, 1]) and Y renormalised.
    Returns T[n], p[n], Y[ns, n].
    """
    mech = om.mech
    ns = om.ns
    comp = np.asarray(mech["composition"], np.float64)
    W = comp @ np.asarray(mech["elem_mass"], np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    T = rng.uniform(T_range[0], T_range[1], n)
    p = rng.uniform(p_atm_range[0], p_atm_range[1], n) * PATM
    xa = rng.uniform(0.05, 0.3, (n, 2))
    u = rng.uniform(-1.0, 1.0, (n, ns))
    Y = np.empty((ns, n))
    react = np.arange(ns - 1)
    a_re = comp[react, :2]
    for i in range(n):
        g = om.thermo(T[i])[3]
        P0 = PATM / (RU * T[i])
        ctot = p[i] / (RU * T[i])
        # anchors: species 2 = (2,0,0), species 3 = (0,2,0)
        lam = np.empty(2)
        lam[0] = 0.5 * (np.log(xa[i, 0] * ctot / P0) + g[2])
        lam[1] = 0.5 * (np.log(xa[i, 1] * ctot / P0) + g[3])
        lnC = np.log(P0) - g[react] + a_re @ lam
        # lower both potentials by the same amount until the reactive species
        # take at most 90 % of the pressure: f(shift) is decreasing
        na = a_re.sum(axis=1)
        target = np.log(0.9 * ctot)
        f = lambda sh: np.logaddexp.reduce(lnC - sh * na) - target
        shift = 0.0
        if f(0.0) > 0.0:
            lo, hi = 0.0, 1.0
            while f(hi) > 0.0:
                lo, hi = hi, 2.0 * hi
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if f(mid) > 0.0:
                    lo = mid
                else:
                    hi = mid
            shift = hi
        Cr = np.exp(lnC - shift * na)
        X = np.empty(ns)
        X[react] = Cr / ctot
        X[ns - 1] = 1.0 - X[react].sum()
        y = X * W
        y /= y.sum()
        y *= 1.0 + perturb * u[i]
        Y[:, i] = y / y.sum()
    assert (Y >= 0.0).all() and np.isfinite(Y).all()
    return T, p, Y
