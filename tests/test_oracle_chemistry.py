"""Pins of the oracle's thermochemistry (Sections 2.3.1 and 4.1.1): closed
forms, exact equilibria, a stiff library ODE solver, and textbook rates."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

import oracle
import rtgen
from rtgen.configs import CHEM_H, CHEM_HHE, RATES_CASEB_CONST, RATES_HG97

ALPHA_B = 2.59e-13


def h_params(rate_set=RATES_CASEB_CONST, isothermal=1, T=1.0e4, sigma=6.3e-18):
    p = rtgen.default_params(1)
    p.update(chem_mode=CHEM_H, rate_set=rate_set, isothermal=isothermal, T_iso=T)
    p["sigma"][0, 0] = sigma
    return p


def hhe_params(isothermal=1, T=2.0e4, sigma=1e-30):
    p = rtgen.default_params(3)
    p.update(chem_mode=CHEM_HHE, rate_set=RATES_HG97, isothermal=isothermal, T_iso=T, Y_He=0.24)
    # Each bin ionises one species only; sigma tiny so the photon field is
    # effectively fixed over the step.
    p["sigma"][:] = np.diag([sigma, sigma, sigma])
    p["e_heat"][:] = np.diag([2.0, 10.0, 20.0]) * 1.602176634e-12
    return p


def test_pure_recombination_matches_closed_form():
    """dx/dt = -alpha n_H x^2 (no radiation, n_e = n_H x_HII):
    x(t) = x0 / (1 + alpha n_H x0 t)."""
    p = h_params()
    nH = 1.0e-3
    trec = 1.0 / (ALPHA_B * nH)
    for t, x0 in ((0.3 * trec, 1.0), (trec, 1.0), (2.0 * trec, 0.6)):
        out = oracle.chem_cell(p, t, nH, [0.0], np.zeros(3), [1 - x0, x0, 1, 0, 0], 1.0e4)
        assert out["rc"] == 0
        exact = x0 / (1 + ALPHA_B * nH * x0 * t)
        # Backward-Euler steps that change x by ~f_s = 5% carry a local
        # relative error ~f_s^2/2; the controller bounds the total well below 2%.
        assert out["x"][1] == pytest.approx(exact, rel=2e-2, abs=0.0)
        assert out["x"][0] + out["x"][1] == pytest.approx(1.0, abs=1e-14)


def test_photoionisation_equilibrium_is_a_fixed_point():
    """Exact balance Gamma x_HI = alpha n_H x_HII^2 is left unchanged by the
    semi-implicit update, for any step length."""
    p = h_params(sigma=1e-30)
    nH = 1.0e-3
    Gam = 1.0e-12
    N = Gam / (p["c_reduced"] * 1e-30)
    # root of alpha n_H x^2 + Gam x - Gam = 0 in the form without
    # cancellation, and x_HI from the balance itself (1 - x_HII would lose
    # four digits here)
    xII = 2 * Gam / (Gam + np.sqrt(Gam ** 2 + 4 * ALPHA_B * nH * Gam))
    xHI = ALPHA_B * nH * xII ** 2 / Gam
    assert xHI + xII == pytest.approx(1.0, rel=1e-15, abs=0.0)
    for dt in (1e10, 1e13, 1e15):
        out = oracle.chem_cell(p, dt, nH, [N], np.zeros(3), [xHI, xII, 1, 0, 0], 1.0e4)
        assert out["x"][1] == pytest.approx(xII, rel=1e-10, abs=0.0)
        assert out["x"][0] == pytest.approx(xHI, rel=1e-10, abs=0.0)
        assert out["attempts"] == 1


def hhe_equilibrium(p, T, nH, Gam):
    """Ionisation balance of H and He with photoionisation rates Gam[3],
    case-B recombination and collisional ionisation, solved for n_e."""
    r = oracle.rates(p, T)
    yhe = p["Y_He"] / (4 * (1 - p["Y_He"]))

    def fractions(ne):
        ionH = Gam[0] + r["bHI"] * ne
        xII = ionH / (ionH + r["aHII"] * ne)
        # He0 <-> He+ <-> He++ balance
        a = (Gam[1] + r["bHeI"] * ne) / (r["aHeII"] * ne)      # y_II / y_I
        b = (Gam[2] + r["bHeII"] * ne) / (r["aHeIII"] * ne)    # y_III / y_II
        yI = 1.0 / (1 + a + a * b)
        return np.array([1 - xII, xII, yI, a * yI, a * b * yI])

    def resid(ne):
        x = fractions(ne)
        return ne - nH * (x[1] + yhe * (x[3] + 2 * x[4]))

    ne = brentq(resid, 1e-12 * nH, 1.2 * nH, xtol=1e-30, rtol=1e-15)
    return fractions(ne)


@pytest.mark.parametrize("T", [1.5e4, 4.0e4])
def test_hhe_equilibrium_is_a_fixed_point(T):
    p = hhe_params(T=T)
    nH = 2.0e-3
    Gam = np.array([3e-13, 1e-13, 2e-14])
    x = hhe_equilibrium(p, T, nH, Gam)
    N = Gam / (p["c_reduced"] * 1e-30)
    for dt in (1e11, 1e14):
        out = oracle.chem_cell(p, dt, nH, N, np.zeros((3, 3)), x, T)
        assert out["rc"] == 0
        assert np.allclose(out["x"], x, rtol=1e-9, atol=1e-14)


def hhe_rhs(p, T, nH, Gam):
    r = oracle.rates(p, T)
    yhe = p["Y_He"] / (4 * (1 - p["Y_He"]))

    def f(t, x):
        ne = nH * (x[1] + yhe * (x[3] + 2 * x[4]))
        dxII = (Gam[0] + r["bHI"] * ne) * x[0] - r["aHII"] * ne * x[1]
        dyI = r["aHeII"] * ne * x[3] - (Gam[1] + r["bHeI"] * ne) * x[2]
        dyIII = (Gam[2] + r["bHeII"] * ne) * x[3] - r["aHeIII"] * ne * x[4]
        return [-dxII, dxII, dyI, -dyI - dyIII, dyIII]
    return f


@pytest.mark.parametrize("dt_rec", [0.05, 1.0, 20.0])
def test_hhe_kinetics_match_stiff_ode_solver(dt_rec):
    """Ionisation of neutral gas under a fixed radiation field: the adaptive
    semi-implicit integrator follows the rate equations to within the
    controller's few-percent step error."""
    T = 2.0e4
    p = hhe_params(T=T)
    nH = 1.0e-3
    Gam = np.array([2e-13, 5e-14, 1e-14])
    N = Gam / (p["c_reduced"] * 1e-30)
    x0 = np.array([1.0, 0.0, 1.0, 0.0, 0.0])
    t = dt_rec / (ALPHA_B * nH)
    out = oracle.chem_cell(p, t, nH, N, np.zeros((3, 3)), x0, T)
    sol = solve_ivp(hhe_rhs(p, T, nH, Gam), [0, t], x0, method="Radau", rtol=1e-10, atol=1e-14)
    ref = sol.y[:, -1]
    assert np.allclose(out["x"], ref, rtol=3e-2, atol=2e-3)
    assert out["x"][0] + out["x"][1] == pytest.approx(1, abs=1e-14)
    assert out["x"][2:].sum() == pytest.approx(1, abs=1e-14)


def test_coupled_energy_and_abundances_match_stiff_ode_solver():
    """Recombining, cooling gas (no radiation): the explicit energy step under
    the 10% rule plus the implicit abundances follow the coupled system
    dx/dt (rate equations at T(u)), du/dt = -Lambda(T, x)/rho."""
    p = hhe_params(isothermal=0, sigma=1e-30)
    nH = 1.0e-3
    x0 = np.array([1e-3, 1 - 1e-3, 0.2, 0.7, 0.1])
    kB, mp = 1.380649e-16, 1.67262192369e-24
    yhe = 0.24 / (4 * 0.76)
    rho = mp * nH * (1 + 4 * yhe)

    def temp(u, x):
        xe = x[1] + yhe * (x[3] + 2 * x[4])
        mu = (1 + 4 * yhe) / (1 + yhe + xe)
        return (2.0 / 3.0) * mu * mp * u / kB

    def f(_, y):
        x, u = y[:5], y[5]
        T = temp(u, x)
        dx = hhe_rhs(p, T, nH, np.zeros(3))(0, x)
        return list(dx) + [-oracle.cooling(p, T, nH, x) / rho]

    T0 = 3.0e4
    xe0 = x0[1] + yhe * (x0[3] + 2 * x0[4])
    u0 = kB * T0 / ((2.0 / 3.0) * (1 + 4 * yhe) / (1 + yhe + xe0) * mp)
    t = 3e14
    out = oracle.chem_cell(p, t, nH, np.zeros(3), np.zeros((3, 3)), x0, T0)
    sol = solve_ivp(f, [0, t], list(x0) + [u0], method="Radau", rtol=1e-9, atol=1e-14)
    Tref = temp(sol.y[5, -1], sol.y[:5, -1])
    assert Tref < 0.8 * T0                      # the pin is not trivial
    assert out["T"] == pytest.approx(Tref, rel=0.03, abs=0.0)
    assert np.allclose(out["x"], sol.y[:5, -1], rtol=0.05, atol=5e-3)


def test_case_b_recombination_textbook_value():
    p = h_params(rate_set=RATES_HG97)
    r = oracle.rates(p, 1.0e4)
    assert r["aHII"] == pytest.approx(2.59e-13, rel=0.01, abs=0.0)      # Osterbrock & Ferland, case B, 10^4 K
    for T in (3e3, 1e4, 3e4, 1e5):
        # hydrogenic scaling alpha_Z(T) = Z alpha_1(T / Z^2) for He II -> He I I I recombination
        assert oracle.rates(p, T)["aHeIII"] == pytest.approx(2 * oracle.rates(p, T / 4)["aHII"], rel=2e-3, abs=0.0)
    # collisional ionisation switches on steeply with temperature
    assert oracle.rates(p, 5e3)["bHI"] < 1e-6 * oracle.rates(p, 3e4)["bHI"]


def test_controller_rejects_and_rescales():
    """A neutral cell hit by a strong field must take many controlled substeps;
    the result keeps the complement identity and stays in [0, 1]."""
    p = h_params(sigma=6.3e-18)
    nH = 1.0e-3
    out = oracle.chem_cell(p, 1e13, nH, [1e-4], np.array([1e-5, 0, 0]), [1, 0, 1, 0, 0], 1e4)
    assert out["attempts"] > 50
    assert 0 <= out["x"][1] <= 1 and 0 <= out["x"][0] <= 1
    assert out["x"][0] + out["x"][1] == pytest.approx(1, abs=1e-14)
    # photons absorbed, flux scaled by the same factor
    assert out["N"][0] < 1e-4
    assert out["Fh"][0, 0] / out["N"][0] == pytest.approx(1e-5 / 1e-4, rel=1e-12, abs=0.0)


def test_substep_cap_reports_error():
    p = h_params(sigma=6.3e-18)
    p["chem_max_substeps"] = 3
    out = oracle.chem_cell(p, 1e13, 1e-3, [1e-4], np.zeros(3), [1, 0, 1, 0, 0], 1e4)
    assert out["rc"] == -6
