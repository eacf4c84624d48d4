"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function that include/kx.h declares, and kx_mech_create_host enforces the
descriptor contract (error codes) without touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2411_02640_amd import kx
from tests import tiny_mechs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "kx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w ]+?\**\s*(kx_\w+)\s*\(", text, re.M)))


def test_header_declares_api():
    names = declared_functions()
    for must in ("kx_mech_create", "kx_mech_create_host", "kx_production_rates",
                 "kx_transport", "kx_thermo", "kx_submit", "kx_server_create"):
        assert must in names


def test_every_declared_symbol_is_exported():
    L = kx.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_version():
    assert "gfx950" in kx.version()


@pytest.mark.parametrize("name", ["mech9", "mech53", "mech200", "mech53x", "mech53o",
                                  "mech53q", "mech53xq", "mech200q"])
def test_host_create(name, request):
    mech = request.getfixturevalue(name)
    m = kx.HostMechanism(mech)
    assert m.n_species == mech["n_species"]
    assert m.n_reactions == mech["n_reactions"]
    assert m.device_bytes > 0
    m.close()


def _tiny():
    return tiny_mechs.abx_mechanism()


def _expect(mech, code, words):
    with pytest.raises(kx.KxError) as ei:
        kx.HostMechanism(mech)
    assert ei.value.code == code, str(ei.value)
    assert words in str(ei.value)


def _mod(**kw):
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in _tiny().items()}
    m.update(kw)
    return m


def test_tiny_is_valid():
    kx.HostMechanism(_tiny()).close()


def test_reject_bad_counts():
    _expect(_mod(n_species=0), kx.KX_EINVAL, "n_species")
    _expect(_mod(n_elements=0), kx.KX_EINVAL, "n_species")


def test_reject_too_many_species(mech9):
    m = dict(mech9)
    m["n_species"] = 257
    _expect(m, kx.KX_EUNSUPPORTED, "256 species")


def test_reject_fit_parameters():
    _expect(_mod(fit_order=0), kx.KX_EINVAL, "fit_order")
    _expect(_mod(fit_order=9), kx.KX_EINVAL, "fit_order")
    _expect(_mod(fit_h=0.0), kx.KX_EINVAL, "fit_h")
    _expect(_mod(fit_L0=float("nan")), kx.KX_EINVAL, "fit_h")
    _expect(_mod(diff_fit_kind=2), kx.KX_EINVAL, "diff_fit_kind")


def test_reject_asymmetric_diffusion_fit():
    m = _mod()
    d = m["diff_fit"].copy()
    d[0, 1, 0] += 1e-3
    m["diff_fit"] = d
    _expect(m, kx.KX_EINVAL, "symmetric")


def test_reject_negative_atoms():
    m = _mod()
    c = m["composition"].copy()
    c[0, 0] = -1
    m["composition"] = c
    _expect(m, kx.KX_EINVAL, "negative atom")


def test_reject_bad_reaction_fields():
    m = _mod()
    m["A"] = m["A"].copy()
    m["A"][0] = 0.0
    _expect(m, kx.KX_EINVAL, "A must be > 0")
    m = _mod()
    m["rxn_type"] = m["rxn_type"].copy()
    m["rxn_type"][0] = 7
    _expect(m, kx.KX_EINVAL, "unknown reaction type")
    m = _mod()
    m["reac_sp"] = m["reac_sp"].copy()
    m["reac_sp"][0] = m["n_species"]
    _expect(m, kx.KX_EINVAL, "out of range")


def test_reject_unbalanced_reaction():
    comp = [[2, 0], [0, 2], [1, 1]]  # H2, O2, HO
    nasa = np.tile([3.5, 0, 0, 0, 0, -1000.0, 3.0], (3, 1))
    rx = [{"type": 0, "reac": [(0, 1), (1, 1)], "prod": [(2, 1)], "A": 1e10, "beta": 0.0,
           "Ea": 0.0}]
    _expect(tiny_mechs.build(comp, nasa, rx), kx.KX_EINVAL, "element-balanced")


def test_reject_four_molecules_on_a_side():
    comp = [[2, 0], [1, 0]]  # H2, H
    nasa = np.tile([3.5, 0, 0, 0, 0, -1000.0, 3.0], (2, 1))
    rx = [{"type": 0, "reac": [(1, 4)], "prod": [(0, 2)], "A": 1e10, "beta": 0.0, "Ea": 0.0}]
    _expect(tiny_mechs.build(comp, nasa, rx), kx.KX_EUNSUPPORTED, "more than 3 molecules")


def test_reject_duplicate_species_on_a_side():
    comp = [[2, 0], [1, 0]]
    nasa = np.tile([3.5, 0, 0, 0, 0, -1000.0, 3.0], (2, 1))
    rx = [{"type": 0, "reac": [(1, 1), (1, 1)], "prod": [(0, 1)], "A": 1e10, "beta": 0.0,
           "Ea": 0.0}]
    _expect(tiny_mechs.build(comp, nasa, rx), kx.KX_EINVAL, "listed twice")


def test_direct_calls_reject_host_mechanism():
    L = kx.lib()
    m = kx.HostMechanism(_tiny())
    rc = L.kx_production_rates(m.handle, 1, None, None, None, None, None)
    assert rc == kx.KX_EINVAL and b"device tables" in L.kx_last_error()
    rc = L.kx_transport(m.handle, 1, None, None, None, None, None, None, None)
    assert rc == kx.KX_EINVAL
    m.close()


def test_null_arguments():
    L = kx.lib()
    assert L.kx_production_rates(None, 1, None, None, None, None, None) == kx.KX_EINVAL
    assert b"NULL" in L.kx_last_error()
    d, keep = kx.make_desc(_tiny())
    L2 = kx._serve_lib()
    assert L2.kx_mech_create_host(C.byref(d), None) == kx.KX_EINVAL
    assert L.kx_mech_destroy(None) == kx.KX_OK


def _one(rtype, **kw):
    base = dict(A=1e12, beta=0.0, Ea=100.0, A0=1e16, beta0=0.0, Ea0=0.0)
    base.update(kw)
    return tiny_mechs.single_reaction_mech(rtype, **base)


def test_further_reaction_forms_accepted():
    for m in (_one(4, sri=[0.5, 300.0, 900.0, 1.0, 0.0]),
              _one(3, troe=(0.5, 100.0, 1000.0, np.nan), chem_act=1),
              _one(5, plog=[(1e5, 1e12, 0.0, 0.0), (1e7, 2e12, 0.1, 50.0)]),
              _one(5, A=0.0, plog=[(1e6, 1e12, 0.0, 0.0)])):
        kx.HostMechanism(m).close()


def test_reject_bad_sri_parameters():
    _expect(_one(4, sri=[0.5, 300.0, 0.0, 1.0, 0.0]), kx.KX_EINVAL, "SRI needs")
    _expect(_one(4, sri=[0.5, 300.0, 900.0, 0.0, 0.0]), kx.KX_EINVAL, "SRI needs")
    _expect(_one(4, sri=[-0.1, 300.0, 900.0, 1.0, 0.0]), kx.KX_EINVAL, "SRI needs")
    _expect(_one(4, sri=[0.5, np.inf, 900.0, 1.0, 0.0]), kx.KX_EINVAL, "finite")
    m = _one(4, sri=[0.5, 300.0, 900.0, 1.0, 0.0])
    m["sri"] = None
    _expect(m, kx.KX_EINVAL, "NULL sri")


def test_reject_bad_pressure_tables():
    _expect(_one(5, plog=[(1e7, 1e12, 0.0, 0.0), (1e5, 2e12, 0.0, 0.0)]), kx.KX_EINVAL,
            "strictly increasing")
    _expect(_one(5, plog=[(1e6, 1e12, 0.0, 0.0), (1e6, 2e12, 0.0, 0.0)]), kx.KX_EINVAL,
            "strictly increasing")
    _expect(_one(5, plog=[(-1.0, 1e12, 0.0, 0.0)]), kx.KX_EINVAL, "strictly increasing")
    _expect(_one(5, plog=[(1e6, 0.0, 0.0, 0.0)]), kx.KX_EINVAL, "PLOG A must be > 0")
    m = _one(5, plog=[(1e6, 1e12, 0.0, 0.0)])
    m["plog_ptr"] = np.array([0, 0], np.int32)
    _expect(m, kx.KX_EINVAL, "without pressures")


def test_reject_chem_act_on_non_falloff():
    _expect(_one(0, chem_act=1), kx.KX_EINVAL, "chem_act")
    _expect(_one(1, chem_act=1), kx.KX_EINVAL, "chem_act")


def _ord(orders, rev=0):
    rx = [dict(type=0, reac=[(tiny_mechs.A_, 1), (tiny_mechs.B_, 1)],
               prod=[(tiny_mechs.AB_, 1)], A=1e12, beta=0.0, Ea=0.0, rev=rev, ord=orders)]
    return tiny_mechs.build(tiny_mechs.ABX_COMP, tiny_mechs.ABX_NASA, rx)


def test_explicit_orders_validation():
    kx.HostMechanism(_ord([(0, 1.5), (3, 0.2)])).close()
    kx.HostMechanism(_ord([(0, 0.0), (1, 0.0), (2, 0.5), (3, 0.2)])).close()  # zeros dropped
    _expect(_ord([(0, 1.5)], rev=1), kx.KX_EINVAL, "irreversible")
    _expect(_ord([(0, -0.5)]), kx.KX_EINVAL, "orders must be finite")
    _expect(_ord([(0, 1.0), (0, 2.0)]), kx.KX_EINVAL, "listed twice")
    _expect(_ord([(9, 1.0)]), kx.KX_EINVAL, "out of range")
    # five species with non-zero orders (two reactants + three more) exceed four
    comp = tiny_mechs.ABX_COMP + [(2, 0, 0)]
    nasa = tiny_mechs.ABX_NASA + [tiny_mechs.ABX_NASA[2]]
    rx = [dict(type=0, reac=[(0, 1), (1, 1)], prod=[(2, 1)], A=1e12, beta=0.0, Ea=0.0, rev=0,
               ord=[(2, 0.1), (3, 0.1), (4, 0.1)])]
    _expect(tiny_mechs.build(comp, nasa, rx), kx.KX_EUNSUPPORTED, "more than 4")


# ------------------------------------------------------------- QSS species
TM = tiny_mechs


def _chain(**kw):
    m = TM.qss_chain_mechanism()
    m.update(kw)
    return m


def test_qss_validation():
    kx.HostMechanism(_chain()).close()
    kx.HostMechanism(TM.qss_chain_mechanism((TM.Q1_,))).close()
    _expect(_chain(qss=np.array([0, 2, 0, 0, 0], np.int32)), kx.KX_EINVAL, "0 or 1")
    _expect(_chain(qss=np.ones(5, np.int32)), kx.KX_EINVAL, "every species is QSS")
    # B is produced only by irreversible reactions: nothing consumes it
    _expect(_chain(qss=np.array([0, 0, 0, 1, 0], np.int32)), kx.KX_EINVAL, "consumed by no")
    # a collider efficiency for a QSS species makes [M] depend on it
    m = TM.qss_chain_mechanism()
    m["eff_sp"] = np.array([TM.Q2_], np.int32)
    _expect(m, kx.KX_EUNSUPPORTED, "efficiency list")
    # two QSS molecules on one side: Q1 + Q2 -> A + B
    m = TM.qss_chain_mechanism()
    comp, nasa = TM.QSS_COMP, TM.QSS_NASA
    rx = [dict(type=0, reac=[(TM.QA_, 1)], prod=[(TM.Q1_, 1)], A=1e10, beta=0.0, Ea=0.0),
          dict(type=0, reac=[(TM.Q1_, 1), (TM.Q2_, 1)], prod=[(TM.QA_, 1), (TM.QB_, 1)],
               A=1e12, beta=0.0, Ea=0.0)]
    bad = TM.build(comp, nasa, rx)
    bad["qss"] = np.array([0, 1, 1, 0, 0], np.int32)
    _expect(bad, kx.KX_EUNSUPPORTED, "two QSS molecules")
    # a QSS species in a reaction with explicit orders
    rx = [dict(type=0, reac=[(TM.QA_, 1)], prod=[(TM.Q1_, 1)], A=1e10, beta=0.0, Ea=0.0),
          dict(type=0, reac=[(TM.Q1_, 1)], prod=[(TM.QB_, 1)], A=1e9, beta=0.0, Ea=0.0,
               rev=0, ord=[(TM.Q1_, 0.5)])]
    bad = TM.build(comp, nasa, rx)
    bad["qss"] = np.array([0, 1, 0, 0, 0], np.int32)
    _expect(bad, kx.KX_EUNSUPPORTED, "explicit orders")


def test_qss_entry_points_reject_what_they_do_not_cover():
    L = kx.lib()
    m = kx.HostMechanism(_tiny())
    # a host-only handle has no device tables; a mechanism without QSS species
    # is refused by the concentration call before any device work
    rc = L.kx_qss_concentrations(m.handle, 1, None, None, None, None, None)
    assert rc == kx.KX_EINVAL
    m.close()
