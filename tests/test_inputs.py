"""Checks of the seeded input generator (setup tables and states)."""
import math

import numpy as np
import pytest

from paper_2411_02640_amd import inputs as I


@pytest.mark.parametrize("spec", [I.MECH_9, I.MECH_53, I.MECH_200], ids=lambda s: s.name)
def test_reaction_counts_and_balance(spec):
    m = I.make_mechanism(spec)
    counts = np.bincount(m["rxn_type"], minlength=4)
    assert counts.tolist() == [spec.n_elementary, spec.n_threebody, spec.n_lindemann,
                               spec.n_troe]
    comp = m["composition"]
    ns = m["n_species"]
    keys = set()
    for i in range(m["n_reactions"]):
        r = slice(m["reac_ptr"][i], m["reac_ptr"][i + 1])
        p = slice(m["prod_ptr"][i], m["prod_ptr"][i + 1])
        left = (m["reac_nu"][r][:, None] * comp[m["reac_sp"][r]]).sum(0)
        right = (m["prod_nu"][p][:, None] * comp[m["prod_sp"][p]]).sum(0)
        assert (left == right).all(), i
        # the diluent only ever acts as a collider
        assert ns - 1 not in m["reac_sp"][r] and ns - 1 not in m["prod_sp"][p]
        key = frozenset([tuple(sorted(np.repeat(m["reac_sp"][r], m["reac_nu"][r]))),
                         tuple(sorted(np.repeat(m["prod_sp"][p], m["prod_nu"][p])))])
        keys.add((key, int(m["rxn_type"][i])))
    assert len(keys) == m["n_reactions"]


def test_determinism():
    a = I.make_mechanism(I.MECH_9)
    b = I.make_mechanism(I.MECH_9)
    for k, v in a.items():
        if isinstance(v, np.ndarray):
            np.testing.assert_array_equal(v, b[k], err_msg=k)
    T1, p1, Y1 = I.make_states(9, I.STATES_9)
    T2, p2, Y2 = I.make_states(9, I.STATES_9)
    np.testing.assert_array_equal(Y1, Y2)
    np.testing.assert_array_equal(T1, T2)


def test_nasa_fit_continuity_and_targets(mech53):
    m = mech53
    for k in range(m["n_species"]):
        lo, hi = m["nasa_lo"][k], m["nasa_hi"][k]
        T = I.T_MID
        cp = lambda a: sum(a[i] * T**i for i in range(5))
        assert cp(lo) == pytest.approx(cp(hi), rel=1e-10)
        assert I._nasa_h_over_r(lo, T) == pytest.approx(I._nasa_h_over_r(hi, T), rel=1e-10,
                                                         abs=1e-8)
        assert I._nasa_s_over_r(lo, T) == pytest.approx(I._nasa_s_over_r(hi, T), rel=1e-12)
        # the fit follows the model cp curve closely on the fitting range
        for TT in (300.0, 600.0, 1500.0, 2800.0):
            a = lo if TT < I.T_MID else hi
            model = I._cp_model(TT, *m["_cp_model"][k])
            fit = sum(a[i] * TT**i for i in range(5))
            assert abs(fit - model) / model < 2e-2


def test_transport_fits_follow_kinetic_theory(mech53):
    """Residual report of the ln T fits against the kinetic-theory values."""
    m = mech53
    W = m["composition"] @ m["elem_mass"]
    T = np.exp(np.linspace(math.log(310.0), math.log(2900.0), 37))
    u = (np.log(T) - m["fit_L0"]) / m["fit_h"]
    V = np.vander(u, m["fit_order"], increasing=True)
    worst_eta = worst_d = 0.0
    for k in range(m["n_species"]):
        eta = I._pure_viscosity(T, W[k], m["_sigma_cm"][k], m["_eps_k"][k])
        worst_eta = max(worst_eta, np.max(np.abs(V @ m["visc_fit"][k] / eta - 1)))
        for j in range(0, m["n_species"], 7):
            D = I._binary_diffusion_1atm(T, W[k], W[j], m["_sigma_cm"][k], m["_sigma_cm"][j],
                                         m["_eps_k"][k], m["_eps_k"][j])
            fit = V @ m["diff_fit"][k, j]
            if m["diff_fit_kind"] == 1:  # the table fits 1/D_kj
                fit = 1.0 / fit
            worst_d = max(worst_d, np.max(np.abs(fit / D - 1)))
    # a degree-4 polynomial in ln T of D ~ T^1.75 / Omega (or of its inverse)
    # carries a few per cent of fit error (the paper's functional form, App. A.3)
    assert worst_eta < 5e-3
    assert worst_d < 5e-2
    np.testing.assert_array_equal(m["diff_fit"], m["diff_fit"].transpose(1, 0, 2))


def test_states_shape_and_ranges():
    T, p, Y = I.make_states(53, I.STATES_53, n_points=1000)
    assert Y.shape == (53, 1000) and Y.flags.c_contiguous
    assert T.min() >= 300.0 and T.max() <= 2800.0
    assert p.min() >= I.P_ATM and p.max() <= 40 * I.P_ATM
    np.testing.assert_allclose(Y.sum(0), 1.0, rtol=1e-14)
    assert (Y >= 0).all()


def test_special_case_fractions():
    spec = I.MechSpec(53, 266, 30, 0, 29, seed=77, special_cases=True, name="syn53sc")
    m = I.make_mechanism(spec)
    zero = (m["beta"] == 0) & (m["Ea"] == 0)
    assert zero.sum() == round(0.27 * 325)
    intb = (m["Ea"] == 0) & (m["beta"] != 0) & (m["beta"] == np.round(m["beta"]))
    assert intb.sum() >= 1
    pairs = {}
    for b, e in zip(m["beta"][~zero], m["Ea"][~zero]):
        pairs[(b, e)] = pairs.get((b, e), 0) + 1
    assert sum(c - 1 for c in pairs.values() if c > 1) >= 0.15 * 325
