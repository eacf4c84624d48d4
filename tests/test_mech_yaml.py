"""The Cantera-YAML importer: unit conversions and reaction forms against
closed-form values from a synthetic fixture, round trips of the synthetic
mechanisms through export and import, and the inputs it refuses."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_02640_amd import inputs as I
from paper_2411_02640_amd import kx
from paper_2411_02640_amd import mech_yaml as MY

FIXTURE = os.path.join(os.path.dirname(__file__), "golden", "mini_mech.yaml")
RCAL = 8.31446261815324 / 4.184


def test_fixture_units_and_forms():
    """Cantera's default units (m, kmol, J/kmol, Pa) and explicit-unit values
    converted to cgs / cal/mol: a bimolecular A in m^3/(kmol s) gains 1e3, a
    termolecular one 1e6, a unimolecular one 1; 4.184e7 J/kmol = 1e4 cal/mol;
    500 K = 500 R cal/mol; 1 atm = 101325 Pa = 1013250 dyn/cm^2."""
    m = MY.load(FIXTURE)
    names = m["_species_names"]
    assert names == ["A", "B", "AB", "A2", "B2", "AB2", "X"]
    np.testing.assert_array_equal(m["rxn_type"], [0, 0, 1, 3, 4, 2, 5, 0, 0, 0])
    np.testing.assert_array_equal(m["reversible"], [1, 0, 1, 1, 1, 1, 1, 1, 1, 0])
    assert m["A"][0] == pytest.approx(1e13, rel=1e-15)
    assert m["Ea"][0] == pytest.approx(1e4, rel=1e-15)
    assert m["A"][1] == pytest.approx(2e13, rel=1e-15) and m["Ea"][1] == 1e4
    assert m["A"][2] == pytest.approx(1e16, rel=1e-15)            # + M: one order more
    assert m["A"][3] == pytest.approx(4e12, rel=1e-15)            # k_inf, bimolecular
    assert m["A0"][3] == pytest.approx(3e18, rel=1e-15)           # k_0, termolecular
    assert m["Ea0"][3] == pytest.approx(500.0 * RCAL, rel=1e-15)
    assert m["troe"][3][:3].tolist() == [0.5, 100.0, 2000.0] and np.isnan(m["troe"][3][3])
    assert m["sri"][4].tolist() == [0.8, 300.0, 900.0, 1.0, 0.0]  # D, E defaults
    assert m["eff_default"][4] == 0.0                             # (+X): X alone collides
    sl = slice(m["eff_ptr"][4], m["eff_ptr"][5])
    assert m["eff_sp"][sl].tolist() == [names.index("X")] and m["eff_val"][sl].tolist() == [1.0]
    assert m["chem_act"].tolist() == [0, 0, 0, 0, 0, 1, 0, 0, 0, 0]
    assert m["A0"][5] == pytest.approx(7e13, rel=1e-15)           # k_0 bimolecular
    assert m["A"][5] == pytest.approx(8e7, rel=1e-15)             # k_inf unimolecular
    sl = slice(m["plog_ptr"][6], m["plog_ptr"][7])
    np.testing.assert_allclose(m["plog_p"][sl], [1013250.0, 10132500.0], rtol=1e-15)
    np.testing.assert_allclose(m["plog_A"][sl], [1e13, 3e13], rtol=1e-15)
    np.testing.assert_allclose(m["plog_Ea"][sl], [1000.0, 1000.0], rtol=1e-15)
    sl = slice(m["eff_ptr"][2], m["eff_ptr"][3])
    assert m["eff_sp"][sl].tolist() == [names.index("A2"), names.index("X")]
    assert m["eff_val"][sl].tolist() == [2.5, 0.5]
    # 2 A <=> A2 twice (duplicates add); nu = 2 on the left
    assert m["reac_nu"][m["reac_ptr"][7]] == 2 and m["A"][7] + m["A"][8] == pytest.approx(4e12)
    # explicit orders: A's units follow their sum (1.5 + 0.7 + 0.25 = 2.45)
    sl = slice(m["ord_ptr"][9], m["ord_ptr"][10])
    assert [names[k] for k in m["ord_sp"][sl]] == ["A", "AB2", "B"]
    assert m["ord_val"][sl].tolist() == [1.5, 0.7, 0.25]
    assert m["A"][9] == pytest.approx(5e9 * 1e3 ** 1.45, rel=1e-14)
    # one NASA range: used on both sides of t_mid = its upper end
    k = names.index("AB2")
    assert m["t_mid"][k] == 1000.0 and (m["nasa_lo"][k] == m["nasa_hi"][k]).all()
    assert any("AB" in w for w in m["_warnings"])                 # the polar species
    kx.HostMechanism(m).close()


@pytest.mark.parametrize("name", ["mech9", "mech53x", "mech53o"])
def test_round_trip(name, request):
    """export -> import gives back the kinetics and thermo arrays (and the same
    oracle rates); viscosity and diffusion fits agree; conductivity fits differ
    only through cp, which the importer takes from the NASA-7 tables where the
    generator used its smooth cp model (within the NASA fit error)."""
    m = request.getfixturevalue(name)
    r = MY.load(MY.dump(m))
    plog = m["rxn_type"] == I.RXN_PLOG
    for k in ("n_species", "n_reactions", "n_elements", "fit_order", "fit_L0", "fit_h",
              "diff_fit_kind"):
        assert r[k] == m[k], k
    for k in ("elem_mass", "composition", "nasa_lo", "nasa_hi", "t_mid", "rxn_type",
              "reversible", "reac_ptr", "reac_sp", "reac_nu", "prod_ptr", "prod_sp",
              "prod_nu", "A0", "beta0", "Ea0", "troe", "eff_ptr", "eff_sp", "eff_val",
              "eff_default"):
        np.testing.assert_array_equal(r[k], m[k], err_msg=k)
    for k in ("A", "beta", "Ea"):   # not read for pressure-table reactions
        np.testing.assert_array_equal(r[k][~plog], m[k][~plog], err_msg=k)
    for k in ("sri", "chem_act", "plog_ptr", "plog_A", "plog_beta", "plog_Ea", "ord_ptr",
              "ord_sp", "ord_val"):
        if m[k] is None:
            assert r[k] is None or not np.any(r[k]), k
        else:
            np.testing.assert_array_equal(r[k], m[k], err_msg=k)
    if m["plog_p"] is not None:
        np.testing.assert_allclose(r["plog_p"], m["plog_p"], rtol=1e-15)
    np.testing.assert_allclose(r["visc_fit"], m["visc_fit"], rtol=1e-12)
    np.testing.assert_allclose(r["diff_fit"], m["diff_fit"], rtol=1e-12)
    np.testing.assert_allclose(r["cond_fit"][:, 0], m["cond_fit"][:, 0], rtol=5e-2)
    T, p, Y = I.make_states(m["n_species"], I.StateSpec(64, seed=8, p_atm_range=(0.05, 200.0)))
    w1 = O.OracleMech(m).production_rates(T, p, Y, with_scale=False)
    w2 = O.OracleMech(r).production_rates(T, p, Y, with_scale=False)
    np.testing.assert_allclose(w2, w1, rtol=1e-13, atol=1e-13 * np.abs(w1).max())


@pytest.mark.parametrize("bad, words", [
    ("orders: {A: 1.5}", "irreversible"),
    ("type: Chebyshev", "not supported"),
    ("negative-A: true", "negative"),
])
def test_rejected_reaction_fields(bad, words):
    text = open(FIXTURE).read().replace(
        "- equation: A + B <=> AB\n  rate-constant: {A: 1.0e10, b: 0.5, Ea: 4.184e7}",
        "- equation: A + B <=> AB\n  rate-constant: {A: 1.0e10, b: 0.5, Ea: 4.184e7}\n  " + bad)
    with pytest.raises(ValueError, match=words):
        MY.load(text)


@pytest.mark.parametrize("old, new, words", [
    ("- equation: A + B <=> AB\n", "- equation: 0.5 A + B <=> AB\n", "non-integer"),
    ("- equation: A + B <=> AB\n", "- equation: A + Q <=> AB\n", "undeclared species"),
    ("composition: {Ar: 1}", "composition: {Zz: 1}", "unknown element"),
    ("- name: X\n  composition: {Ar: 1}\n  thermo:\n    model: NASA7",
     "- name: X\n  composition: {Ar: 1}\n  thermo:\n    model: NASA9", "NASA7"),
    ("efficiencies: {AB2: 3.0}", "efficiencies: {Q: 3.0}", "undeclared species"),
])
def test_rejected_inputs(old, new, words):
    text = open(FIXTURE).read()
    assert old in text
    with pytest.raises(ValueError, match=words):
        MY.load(text.replace(old, new, 1))


def test_qss_species_by_name():
    """Species named as quasi-steady become the descriptor's qss flags; an
    unknown name is refused."""
    plain = MY.load(FIXTURE)
    assert plain["qss"] is None
    names = plain["_species_names"]
    m = MY.load(FIXTURE, qss_species=[names[1], names[3]])
    assert m["qss"].tolist() == [1 if k in (1, 3) else 0 for k in range(len(names))]
    with pytest.raises(ValueError, match="unknown QSS species"):
        MY.load(FIXTURE, qss_species=["no-such-species"])
