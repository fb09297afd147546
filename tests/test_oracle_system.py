"""Whole-subcycle pins of the oracle: the Stromgren sphere (closed form and
the reduced-speed-of-light photon budget), invariants, symmetries, and the
forward-mode derivative against central finite differences."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import rtgen
from rtgen.fields import C_LIGHT


def stromgren_radius_ode(Q, n, alpha, c, t):
    """I-front radius from the photon budget with photons in flight under the
    reduced speed of light: r' (4 pi n r^2 + Q/c) = Q - (4 pi/3) alpha n^2 r^3."""
    def f(_, y):
        r = y[0]
        return [(Q - 4 * np.pi / 3 * alpha * n * n * r ** 3) / (4 * np.pi * n * r * r + Q / c)]
    sol = solve_ivp(f, [0, max(t)], [1e-6 * (3 * Q / (4 * np.pi * n * n * alpha)) ** (1 / 3)], rtol=1e-10,
                    dense_output=True)
    return np.array([sol.sol(tt)[0] for tt in t])


def front_radius(cfg, out):
    return (3.0 / (4 * np.pi) * np.sum(out["species"][1] * cfg["mesh"]["volume"])) ** (1 / 3)


def advance(cfg, out):
    return dict(cfg, state=dict(N=out["N"], F=out["F"], n_H=out["n_H"], species=out["species"], T=out["T"]))


def test_stromgren_front_follows_photon_budget():
    """Point source in uniform isothermal hydrogen (the Stromgren workload):
    the ionised volume tracks the photon-budget ODE and the closed form
    R_S (1 - exp(-t/t_rec))^(1/3)."""
    cfg = rtgen.stromgren()
    Q, n, a, c = 5e48, 1e-3, 2.59e-13, cfg["params"]["c_reduced"]
    RS = (3 * Q / (4 * np.pi * n * n * a)) ** (1 / 3)
    h = cfg["meta"]["h"]
    assert RS / h == pytest.approx(10.79, abs=0.01)
    radii, times = [], []
    st = cfg
    for k in range(4):
        out = oracle.run(st, n_sub=25)
        times.append(25 * (k + 1) * out["diag"]["dt"])
        radii.append(front_radius(cfg, out))
        st = advance(cfg, out)
    ode = stromgren_radius_ode(Q, n, a, c, times)
    closed = RS * (1 - np.exp(-np.array(times) * n * a)) ** (1 / 3)
    assert np.allclose(radii, ode, rtol=0.05)
    assert np.allclose(radii[1:], closed[1:], rtol=0.15)
    # invariants of the final state
    x = out["species"]
    assert np.all((x >= 0) & (x <= 1))
    assert np.allclose(x[0] + x[1], 1.0, rtol=0, atol=1e-14)
    N = out["N"][0]
    Fh = out["F"][0] / c
    assert np.all(N >= 0)
    assert np.all(np.sqrt((Fh ** 2).sum(0)) <= N * (1 + 1e-12) + 1e-150)


@pytest.mark.slow
def test_stromgren_saturates_at_stromgren_radius():
    """Run to three recombination times with c~ = 0.001c (the front is slow by
    then): the ionised volume reaches the Stromgren radius."""
    cfg = rtgen.stromgren()
    cfg["params"]["c_reduced"] = 1e-3 * C_LIGHT
    Q, n, a = 5e48, 1e-3, 2.59e-13
    RS = (3 * Q / (4 * np.pi * n * n * a)) ** (1 / 3)
    trec = 1 / (n * a)
    dt = oracle.cfl_dt(cfg)
    total = int(np.ceil(3 * trec / dt))
    checkpoints = [int(total * f) for f in (0.25, 0.5, 1.0)]
    st, done = cfg, 0
    for k in checkpoints:
        out = oracle.run(st, n_sub=k - done)
        done = k
        st = advance(cfg, out)
        t = done * dt
        r = front_radius(cfg, out)
        closed = RS * (1 - np.exp(-t / trec)) ** (1 / 3)
        ode = stromgren_radius_ode(Q, n, a, cfg["params"]["c_reduced"], [t])[0]
        assert r == pytest.approx(ode, rel=0.05, abs=0.0)
        assert r == pytest.approx(closed, rel=0.05, abs=0.0)
    assert r == pytest.approx(RS, rel=0.05, abs=0.0)


def small_hhe(n=12, n_src=6, n_sub=4, order="hilbert"):
    return rtgen.cosmological(n, 1.0, 1.0, n_src, 0.01, n_sub, 2, order=order, name="small_hhe")


def test_hhe_invariants_and_photon_balance():
    cfg = small_hhe(n_sub=6)
    out = oracle.run(cfg)
    x = out["species"]
    assert np.all((x >= 0) & (x <= 1))
    assert np.allclose(x[0] + x[1], 1, atol=1e-14)
    assert np.allclose(x[2:].sum(0), 1, atol=1e-14)
    assert np.all(out["T"] > 0)
    assert np.all(out["N"] >= 0)
    c = cfg["params"]["c_reduced"]
    Fm = np.sqrt(((out["F"] / c) ** 2).sum(1))
    assert np.all(Fm <= out["N"] * (1 + 1e-12) + 1e-150)
    # Photons injected minus photons left in the box were absorbed: they must
    # be at least the ionisations they caused (recombination is slow here).
    V = cfg["mesh"]["volume"]
    injected = cfg["sources"]["rate"].sum() * 6 * out["diag"]["dt"]
    left = out["diag"]["photon_sum"].sum()
    nH = cfg["state"]["n_H"]
    yhe = 0.24 / (4 * 0.76)
    ionisations = np.sum(V * nH * (x[1] + yhe * (x[3] + 2 * x[4])))
    assert left < injected
    assert ionisations == pytest.approx(injected - left, rel=0.25, abs=0.0)


def test_cell_permutation_equivariance():
    a = small_hhe(order="hilbert")
    b = small_hhe(order="random")
    oa, ob = oracle.run(a), oracle.run(b)
    la = a["meta"]["lattice_index"]
    lb = b["meta"]["lattice_index"]
    dims = a["meta"]["dims"]
    key = lambda li: li[0] + dims[0] * (li[1] + dims[1] * li[2])  # noqa: E731
    ia, ib = np.argsort(key(la)), np.argsort(key(lb))
    for f in ("N", "species", "T"):
        A = oa[f][..., ia]
        B = ob[f][..., ib]
        assert np.allclose(A, B, rtol=1e-10, atol=1e-12 * np.abs(A).max())


def rotate_cfg(cfg, kind):
    """90-degree rotation about z, or reflection x -> -x, of a cubic periodic
    configuration; cells keep their indices."""
    m = dict(cfg["mesh"])
    L = m["box"][0]

    def pos(p):
        p = np.array(p)
        if kind == "rot":
            return np.stack([L - p[1], p[0], p[2]])
        return np.stack([L - p[0], p[1], p[2]])

    def vec(v):
        v = np.array(v)
        if kind == "rot":
            return np.stack([-v[1], v[0], v[2]])
        return np.stack([-v[0], v[1], v[2]])

    m["centre"] = np.ascontiguousarray(pos(m["centre"]))
    m["face_centre"] = np.ascontiguousarray(pos(m["face_centre"]))
    m["normal"] = np.ascontiguousarray(vec(m["normal"]))
    st = dict(cfg["state"])
    st["F"] = np.ascontiguousarray(np.stack([vec(st["F"][b]) for b in range(st["F"].shape[0])]))
    return dict(cfg, mesh=m, state=st), vec


@pytest.mark.parametrize("kind", ["rot", "refl"])
def test_rotation_and_reflection_equivariance(kind):
    cfg = small_hhe(n_sub=3)
    # give the radiation a direction so the vector part is exercised
    out0 = oracle.run(cfg, n_sub=2)
    cfg = advance(cfg, out0)
    rc, vec = rotate_cfg(cfg, kind)
    oa, ob = oracle.run(cfg), oracle.run(rc)
    assert np.allclose(ob["N"], oa["N"], rtol=1e-10, atol=1e-12 * oa["N"].max())
    Fa = np.stack([vec(oa["F"][b]) for b in range(3)])
    assert np.allclose(ob["F"], Fa, rtol=1e-10, atol=1e-12 * np.abs(Fa).max())
    assert np.allclose(ob["species"], oa["species"], rtol=1e-10, atol=1e-13)


def test_forward_derivative_matches_central_differences():
    """Dual-number derivative of the final x_HI along a source-luminosity and a
    density direction against central differences of the plain run."""
    cfg = small_hhe(n=8, n_src=3, n_sub=3)
    nc = cfg["mesh"]["n_cells"]
    rng = np.random.default_rng(0)
    dlnQ = np.zeros((2, 3))
    dlnQ[0] = rng.normal(size=3)
    dln = np.zeros((2, nc))
    dln[1] = rng.normal(size=nc)
    jv = oracle.run_jvp(cfg, dlnQ, dln)
    w = rng.normal(size=nc)
    h = 1e-6
    base_nH = cfg["state"]["n_H"]
    for k in range(2):
        def loss(eps):
            c2 = dict(cfg, state=dict(cfg["state"], n_H=base_nH * np.exp(eps * dln[k])))
            return w @ oracle.run(c2, rate_scale=np.exp(eps * dlnQ[k]))["species"][0]
        fd = (loss(h) - loss(-h)) / (2 * h)
        assert w @ jv["dxHI"][k] == pytest.approx(fd, rel=1e-5, abs=0.0)
