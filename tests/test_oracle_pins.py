"""Pins of the oracle's outflow cap, photoheating, rate fits and cooling, and
the brute-force comparison on the 2x2x2 periodic mesh.

* The outflow cap (the "further limiter" of Sec. 2.3.3) against a
  hand-derived closed form: one free-streaming cell on an unjittered lattice.
* Photoheating (Sec. 2.3.1) against an energy budget: the change of the gas
  energy density over one accepted substep equals the energy of the photons
  actually absorbed (N - N' per bin, shared among the absorbers by their
  opacity) minus cooling times the step.
* The rate-coefficient and cooling fits (rate set 1) against published
  atomic data (tests/golden/atomic_data.json, each entry with its source).
* Whole subcycles on the 2x2x2 jittered periodic mesh against the
  separately written explicit-loop calculator (tests/bruteforce_calc.py) at
  1e-13, with the cap, the face-state admissibility fix and the post-update
  guard all firing, and the event counters equal.
"""
import json
import math
from pathlib import Path

import numpy as np
import pytest

import oracle
import rtgen
from rtgen import fields
from rtgen.configs import CHEM_H, CHEM_HHE, CHEM_NONE, RATES_HG97, _pack

from . import bruteforce_calc as bf

GOLDEN = json.loads((Path(__file__).parent / "golden" / "atomic_data.json").read_text())
KB = 1.380649e-16
EV = 1.602176634e-12


# ---------------------------------------------------------------------------
# outflow cap: closed form
# ---------------------------------------------------------------------------

def test_outflow_cap_closed_form():
    """Unjittered periodic 8^3 lattice (h = 1, c~ = 1), transport only, one
    cell with N0 = 1 streaming freely along +x (Fh = N0 x), all others empty.

    Every limited gradient is zero (the lit cell is the maximum of its
    stencil and its neighbours the minimum of theirs), so the face states are
    the cell averages.  With a = c~ dt / h = 0.3 (3 / 4 pi)^(1/3), the HLL
    fluxes of the lit cell are c~ N0 out through +x, c~ N0 / 2 out through
    each transverse face and 0 through -x.  The cap of the +x face is
    theta = N0 V / (6 c~ N0 dt A) = 1 / (6 a) < 1; the transverse faces ask
    half as much and stay uncapped.  Hence after one subcycle
        lit cell      N = Fh_x = N0 (1 - theta a - 2 a)
        +x neighbour  N = Fh_x = N0 theta a = N0 / 6
        transverse    N = Fh_x = N0 a / 2   (four cells)
        -x neighbour  and every other cell empty,
    with exactly one capped face."""
    n = 8
    m = rtgen.jittered_lattice((n, n, n), 1.0, 0.0, 1, order="lattice")
    p = rtgen.default_params(1)
    p.update(chem_mode=CHEM_NONE, c_reduced=1.0)
    st = rtgen.neutral_state(1, m.n_cells, 1.0, 1.0e4)

    def lex(i, j, k):
        return i + n * (j + n * k)

    lit = lex(3, 3, 3)
    st["N"][0, lit] = 1.0
    st["F"][0, 0, lit] = 1.0
    cfg = _pack("cap_closed_form", m, p, st, np.zeros(0, np.int64), np.zeros((1, 0)), 1, "fp64")
    out = oracle.run(cfg)
    a = 0.3 * (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0)
    theta = 1.0 / (6.0 * a)
    assert theta < 1.0 < 2.0 * theta
    expect = np.zeros(m.n_cells)
    expect[lit] = 1.0 - theta * a - 2.0 * a
    expect[lex(4, 3, 3)] = theta * a
    for c in (lex(3, 4, 3), lex(3, 2, 3), lex(3, 3, 4), lex(3, 3, 2)):
        expect[c] = a / 2.0
    assert out["diag"]["dt"] == pytest.approx(a, rel=1e-15, abs=0.0)
    np.testing.assert_allclose(out["N"][0], expect, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(out["F"][0, 0], expect, rtol=1e-14, atol=1e-16)
    np.testing.assert_array_equal(out["F"][0, 1:], 0.0)
    assert out["diag"]["flux_caps"] == 1
    assert out["diag"]["photon_sum"][0] == pytest.approx(1.0, rel=1e-15, abs=0.0)


# ---------------------------------------------------------------------------
# photoheating: energy budget of one accepted substep
# ---------------------------------------------------------------------------

def _hhe_params():
    p = rtgen.default_params(3)
    sig, eh = fields.blackbody_bin_constants(5.0e4, (13.6, 24.6, 54.4))
    p.update(chem_mode=CHEM_HHE, isothermal=0, rate_set=RATES_HG97, Y_He=0.24, sigma=sig, e_heat=eh)
    return p


def _energy_density(nH, x, T, yhe, gamma):
    """rho u = n_particles k T / (gamma - 1), n_particles = n_H (1 + y_He + x_e)."""
    xe = x[1] + yhe * (x[3] + 2 * x[4])
    return nH * (1 + yhe + xe) * KB * T / (gamma - 1)


@pytest.mark.parametrize("case", ["H", "HHe"])
def test_photoheating_energy_budget(case):
    """One accepted substep: Delta(rho u) = sum_b (N_b - N'_b) e_b - Lambda dt,
    where N_b - N'_b are the photons the cell absorbed in bin b and e_b the
    mean excess energy per absorption, shared among the absorbers in
    proportion to their opacity sigma_bs n_s.  Lambda is the cooling rate of
    the substep-start state (its fits are pinned separately below)."""
    if case == "H":
        p = rtgen.default_params(1)
        p.update(chem_mode=CHEM_H, isothermal=0, rate_set=RATES_HG97, Y_He=0.0)
        p["sigma"][0] = (3.0e-18, 0.0, 0.0)
        p["e_heat"][0] = (4.0 * EV, 0.0, 0.0)
        N = np.array([1.0e-3])
        x = np.array([0.6, 0.4, 1.0, 0.0, 0.0])
    else:
        p = _hhe_params()
        N = np.array([1.0e-3, 2.0e-4, 1.0e-4])
        x = np.array([0.6, 0.4, 0.7, 0.25, 0.05])
    nH, T0, dt = 1.0e-2, 2.0e4, 1.0e10
    yhe = p["Y_He"] / (4 * (1 - p["Y_He"])) if p["chem_mode"] == CHEM_HHE else 0.0
    Fh = np.zeros((p["nb"], 3))
    out = oracle.chem_cell(p, dt, nH, N, Fh, x, T0)
    assert out["rc"] == 0 and out["attempts"] == 1
    sig = np.asarray(p["sigma"]).reshape(-1, 3)
    eh = np.asarray(p["e_heat"]).reshape(-1, 3)
    absorbers = np.array([nH * x[0], yhe * nH * x[2], yhe * nH * x[3]])
    absorbed = N - out["N"]
    assert np.all(absorbed > 0)
    mean_e = (sig * absorbers[None, :] * eh).sum(axis=1) / (sig * absorbers[None, :]).sum(axis=1)
    heating = float((absorbed * mean_e).sum())
    cooling = oracle.cooling(p, T0, nH, x) * dt
    dE = _energy_density(nH, out["x"], out["T"], yhe, p["gamma"]) - _energy_density(nH, x, T0, yhe, p["gamma"])
    # both terms matter, so a wrong heating or cooling term cannot hide
    assert heating > 0.1 * abs(dE) and cooling > 0.1 * abs(dE)
    assert dE == pytest.approx(heating - cooling, rel=1e-10, abs=0.0)


# ---------------------------------------------------------------------------
# rate fits and cooling against published atomic data
# ---------------------------------------------------------------------------

def _hg97_params():
    p = rtgen.default_params(3)
    p.update(chem_mode=CHEM_HHE, rate_set=RATES_HG97, isothermal=0, Y_He=0.24)
    return p


def test_case_b_recombination_published_values():
    g = GOLDEN["case_b_recombination_H"]
    p = _hg97_params()
    for T, ref in zip(g["T"], g["alpha_B"]):
        assert oracle.rates(p, T)["aHII"] == pytest.approx(ref, rel=g["rel_tol"], abs=0.0), T


def test_collisional_ionisation_against_voronov_fit():
    g = GOLDEN["collisional_ionisation_voronov1997"]
    p = _hg97_params()
    kb_ev = KB / EV
    names = {"HI": "bHI", "HeI": "bHeI", "HeII": "bHeII"}
    for sp, c in g["species"].items():
        for T in g["T"]:
            U = c["dE_eV"] / (kb_ev * T)
            ref = c["A"] * (1 + c["P"] * math.sqrt(U)) / (c["X"] + U) * U ** c["K"] * math.exp(-U)
            got = oracle.rates(p, T)[names[sp]]
            assert got == pytest.approx(ref, rel=g["rel_tol"][sp], abs=0.0), (sp, T, got / ref)


def test_free_free_cooling_is_bremsstrahlung():
    """Fully ionised hydrogen at 1e8 K: free-free emission dominates (the
    recombination cooling is ~1e-4 of it), so the cooling per n_e n_p over
    the Rybicki & Lightman coefficient is the mean Gaunt factor."""
    g = GOLDEN["bremsstrahlung"]
    e, h, me, c = 4.80320471e-10, 6.62607015e-27, 9.1093837015e-28, 2.99792458e10
    coef = 2 ** 5 * math.pi * e ** 6 / (3 * h * me * c ** 3) * math.sqrt(2 * math.pi * KB / (3 * me))
    p = rtgen.default_params(1)
    p.update(chem_mode=CHEM_H, rate_set=RATES_HG97, isothermal=0)
    T = g["T"]
    lam = oracle.cooling(p, T, 1.0, np.array([0.0, 1.0, 1.0, 0.0, 0.0]))   # n_e = n_p = 1
    gaunt = lam / (coef * math.sqrt(T))
    assert g["gaunt_range"][0] <= gaunt <= g["gaunt_range"][1], gaunt


def test_collisional_excitation_cooling_matches_collision_strength():
    """Half-ionised hydrogen at 1-2e4 K cools mostly by collisional
    excitation of n = 2 (>= 90 per cent of the total with these fits).  The
    cooling per n_e n_HI divided by E_12 q_12(Upsilon = 1) is the effective
    collision strength; it must be of the order atomic physics gives."""
    g = GOLDEN["collisional_excitation_HI_n2"]
    p = rtgen.default_params(1)
    p.update(chem_mode=CHEM_H, rate_set=RATES_HG97, isothermal=0)
    e12 = 10.2 * EV
    for T in g["T"]:
        x = np.array([0.5, 0.5, 1.0, 0.0, 0.0])
        per_pair = oracle.cooling(p, T, 1.0, x) / (0.5 * 0.5)      # n_e n_HI = 0.25
        q1 = 8.629e-6 / (2.0 * math.sqrt(T)) * math.exp(-e12 / (KB * T))
        upsilon = per_pair / (e12 * q1)
        assert g["upsilon_range"][0] <= upsilon <= g["upsilon_range"][1], (T, upsilon)


# ---------------------------------------------------------------------------
# brute force on the 2x2x2 periodic mesh
# ---------------------------------------------------------------------------

def _errors(a, r, c_red):
    """Largest relative difference per field: N against max(N, 1e-10 max N)
    per bin, Fh against c~ times the same, fractions and T elementwise."""
    worst = {}
    for b in range(r["N"].shape[0]):
        Nr = r["N"][b]
        sc = np.maximum(Nr, 1e-10 * Nr.max())
        worst[f"N[{b}]"] = float((np.abs(a["N"][b] - Nr) / sc).max())
        worst[f"F[{b}]"] = float((np.abs(a["F"][b] - r["F"][b]) / (c_red * sc)[None, :]).max())
    for s in range(5):
        x = r["species"][s]
        worst[f"x[{s}]"] = float((np.abs(a["species"][s] - x) / np.maximum(np.abs(x), 1e-300)).max())
    worst["T"] = float((np.abs(a["T"] - r["T"]) / r["T"]).max())
    return worst


def _radiation(rng, nb, nc, lo, hi, c_red):
    """Nearly free-streaming radiation: N log-uniform in [10^lo, 10^hi],
    |Fh| / N uniform in [0.3, 0.95] in random directions (not 1 exactly, so
    that no admissibility decision of the first subcycle sits at rounding
    level)."""
    N = 10.0 ** rng.uniform(lo, hi, (nb, nc))
    d = rng.normal(size=(nb, 3, nc))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return N, d * (N * rng.uniform(0.3, 0.95, (nb, nc)))[:, None, :] * c_red


def _break_realisability(F, N, cells, c_red, factor=1.5):
    """Inputs with |Fh| = factor N in the given cells, so the post-update
    guard has something to act on (the scheme itself keeps |Fh| <= N: the
    cap bounds each face's outflow and the HLL update of admissible face
    states is realisable, so on valid inputs the guards act only on
    rounding)."""
    F = F.copy()
    for i in cells:
        for b in range(N.shape[0]):
            F[b, :, i] *= factor * N[b, i] * c_red / np.linalg.norm(F[b, :, i])
    return F


def bf_transport_case(seed=2):
    m = rtgen.jittered_lattice((2, 2, 2), 1.0, 0.2, 1000 + seed)
    nb = 2
    p = rtgen.default_params(nb)
    p.update(chem_mode=CHEM_NONE, c_reduced=1.0)
    rng = np.random.default_rng(seed)
    st = rtgen.neutral_state(nb, 8, 1.0, 1.0e4)
    st["N"], F = _radiation(rng, nb, 8, -12, 0, p["c_reduced"])
    # the brightest cells: an inflow from dimmer neighbours cannot restore them
    st["F"] = _break_realisability(F, st["N"], sorted(set(np.argmax(st["N"], axis=1))), p["c_reduced"])
    return _pack("bf_transport", m, p, st, np.zeros(0, np.int64), np.zeros((nb, 0)), 3, "fp64")


def bf_chemistry_case(seed=4):
    m = rtgen.jittered_lattice((2, 2, 2), 0.5 * fields.KPC, 0.2, 1000 + seed)
    p = _hhe_params()
    rng = np.random.default_rng(seed)
    nH = 1.0e-3 * np.exp(rng.normal(0.0, 0.7, 8))
    st = rtgen.neutral_state(3, 8, nH, 100.0)
    st["N"], F = _radiation(rng, 3, 8, -9, -3, p["c_reduced"])
    st["F"] = _break_realisability(F, st["N"], sorted(set(np.argmax(st["N"], axis=1))), p["c_reduced"])
    rate = np.array([1.0, 0.05, 0.03])[:, None] * np.array([[5.0e48, 1.0e48]])
    return _pack("bf_chemistry", m, p, st, np.array([0, 5]), rate, 3, "fp64")


@pytest.mark.parametrize("n_sub", [1, 3])
@pytest.mark.parametrize("make", [bf_transport_case, bf_chemistry_case], ids=["transport", "chemistry"])
def test_oracle_matches_explicit_loop_calculator(make, n_sub):
    cfg = make()
    ref = bf.run(cfg, n_sub)
    out = oracle.run(cfg, n_sub=n_sub)
    errs = _errors(out, ref, cfg["params"]["c_reduced"])
    worst = max(errs, key=errs.get)
    assert errs[worst] <= 1e-13, (worst, errs[worst])
    np.testing.assert_allclose(out["diag"]["photon_sum"], ref["photon_sum"], rtol=1e-13)
    assert out["diag"]["dt"] == pytest.approx(ref["dt"], rel=1e-14, abs=0.0)
    cnt = ref["counters"]
    # a decision taken on a margin at rounding level (|Fh| = N to 1e-12,
    # which the guard's rescaling and free streaming produce) may go either
    # way in two correct implementations; every other decision must agree
    for k, ties in (("adm_F", cnt["adm_ties"]), ("guard_F", cnt["guard_ties"])):
        assert abs(out["diag"][k] - cnt[k]) <= ties, (k, out["diag"][k], cnt[k], ties)
    for k in ("adm_N", "flux_caps", "guard_N", "substeps"):
        assert out["diag"][k] == cnt[k], (k, out["diag"][k], cnt[k])
    # the limiters this pin is about actually act
    assert cnt["flux_caps"] > 0 and cnt["adm_F"] > 0 and cnt["guard_F"] > 0
    if cfg["params"]["chem_mode"] != CHEM_NONE:
        assert cnt["substeps"] > 8 * n_sub


def test_calculator_alone_conserves_and_reduces_to_closed_form():
    """The calculator itself reproduces the cap's closed form on a 4^3
    unjittered lattice (the same derivation as the oracle pin above)."""
    n = 4
    m = rtgen.jittered_lattice((n, n, n), 1.0, 0.0, 1, order="lattice")
    p = rtgen.default_params(1)
    p.update(chem_mode=CHEM_NONE, c_reduced=1.0)
    st = rtgen.neutral_state(1, m.n_cells, 1.0, 1.0e4)
    lit = 1 + n * (1 + n * 1)
    st["N"][0, lit] = 1.0
    st["F"][0, 0, lit] = 1.0
    cfg = _pack("cap_bf", m, p, st, np.zeros(0, np.int64), np.zeros((1, 0)), 1, "fp64")
    out = bf.run(cfg, 1)
    a = 0.3 * (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0)
    assert out["N"][0, lit] == pytest.approx(1.0 - 1.0 / 6.0 - 2.0 * a, rel=1e-14, abs=0.0)
    assert out["N"][0, lit + 1] == pytest.approx(1.0 / 6.0, rel=1e-14, abs=0.0)
    assert out["counters"]["flux_caps"] == 1
    assert out["photon_sum"][0] == pytest.approx(1.0, rel=1e-15, abs=0.0)
