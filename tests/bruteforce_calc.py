"""Explicit-loop calculator of whole subcycles on very small meshes.

A second, separately written statement of the method, used only to pin the
oracle on meshes of a few cells (the 2x2x2 periodic mesh).  It shares no code
with the oracle or the GPU library and is organised differently from both:

* transport is cell-centric: every cell visits each of its faces and
  computes that face's flux in the face's (L, R) orientation;
* gradients are the weighted least-squares solution of the paper's normal
  equation (Sec. 2.3.2), found with numpy's lstsq on the weighted rows
  instead of an explicit inverse;
* the closure builds the full 3x3 Eddington tensor (eq. edd) and the HLL
  flux is written as the Rusanov average of the physical fluxes with speed
  c~ (Sec. 2.3.3);
* the flux divergence and the photon sums use exactly rounded sums
  (math.fsum);
* the thermal state is carried as the energy density rho u.

Readings of the paper that it follows (the same readings the oracle takes):
photon number density N and Fh = F / c~ per bin; sources, chemistry,
gradients, fluxes and update in the order of Fig. 1; Barth-Jespersen limiter
with the cell in its own min/max and face centres as control points;
admissibility of face states; upwind outflow cap theta = min(1, N_up V_up /
(n_faces(up) |Phi_N| dt A)); post-update guards; semi-implicit chemistry that
absorbs the photons first, with the substep controller of Sec. 4.1.1; Hui &
Gnedin (1997) and Cen (1992) rate fits (rate set 1) or a constant case-B
coefficient (rate set 0).
"""
from __future__ import annotations

import math

import numpy as np

KB = 1.380649e-16
MP = 1.67262192369e-24


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------

def _wrap(x, box):
    return x - box * math.floor(x / box + 0.5) if box > 0 else x


def cell_faces(mesh):
    """Per cell, its faces in face-index order: (face, neighbour, sign, r_own,
    r_nbr), with the minimum-image offsets from the two cell centres to the
    face centre."""
    nc, nf = mesh["n_cells"], mesh["n_faces"]
    fc, s, xf, box = mesh["face_cells"], mesh["centre"], mesh["face_centre"], mesh["box"]
    faces = [[] for _ in range(nc)]
    for f in range(nf):
        L, R = int(fc[0, f]), int(fc[1, f])
        rL = np.array([_wrap(xf[k, f] - s[k, L], box[k]) for k in range(3)])
        rR = np.array([_wrap(xf[k, f] - s[k, R], box[k]) for k in range(3)])
        faces[L].append((f, R, +1, rL, rR))
        faces[R].append((f, L, -1, rR, rL))
    return faces


def lsq_gradient(phi_i, items):
    """Gradient g minimising sum_j A_j ((phi_j - phi_i)/|d_j| - g.u_j)^2 with
    d_j = r_own - r_nbr the separation through the face (eq. S_tot)."""
    rows, rhs = [], []
    for A, d, phi_j in items:
        dl = math.sqrt(float(d @ d))
        w = math.sqrt(A)
        rows.append(w * d / dl)
        rhs.append(w * (phi_j - phi_i) / dl)
    g, *_ = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)
    return g


def limited(phi_i, g, nbr_vals, offsets):
    """Barth-Jespersen: scale g so that phi_i + g.r stays in [min, max] of the
    cell and its neighbours at every face centre r."""
    hi = max([phi_i] + nbr_vals)
    lo = min([phi_i] + nbr_vals)
    a = 1.0
    for r in offsets:
        dlt = float(g @ r)
        if dlt > 0:
            a = min(a, (hi - phi_i) / dlt)
        elif dlt < 0:
            a = min(a, (lo - phi_i) / dlt)
    return a * g


# ---------------------------------------------------------------------------
# face physics
# ---------------------------------------------------------------------------

TIE = 1e-12     # decisions closer than this (relative) to their threshold are rounding-level


def admissible(U, cnt):
    """N >= 0, |Fh| <= N (counts each fix, and each decision taken on a
    rounding-level margin as a tie)."""
    N, F = U[0], U[1:].copy()
    if N < 0:
        N = 0.0
        cnt["adm_N"] += 1
    m = math.sqrt(float(F @ F))
    if abs(m - N) <= TIE * max(m, abs(N)):
        cnt["adm_ties"] += 1
    if m * m > N * N:
        cnt["adm_F"] += 1
        F = np.zeros(3) if N <= 0 else F * (N / m)
    return np.concatenate([[N], F])


def eddington(N, F):
    """Levermore M1 Eddington tensor of (N, Fh)."""
    m = math.sqrt(float(F @ F))
    if N <= 0 or m == 0:
        return np.eye(3) / 3
    f = min(m / N, 1.0)
    chi = (3 + 4 * f * f) / (5 + 2 * math.sqrt(4 - 3 * f * f))
    u = F / m
    return 0.5 * (1 - chi) * np.eye(3) + 0.5 * (3 * chi - 1) * np.outer(u, u)


def physical_flux(U, n, c):
    """Normal flux of (N, Fh): c~ Fh.n and c~ N D n."""
    N, F = U[0], U[1:]
    return np.concatenate([[c * float(F @ n)], c * N * (eddington(N, F) @ n)])


def rusanov(UL, UR, n, c):
    return 0.5 * (physical_flux(UL, n, c) + physical_flux(UR, n, c)) - 0.5 * c * (UR - UL)


# ---------------------------------------------------------------------------
# chemistry
# ---------------------------------------------------------------------------

TH_HI, TH_HEI, TH_HEII = 157807.0, 285335.0, 631515.0


def _hg97_b(lam):
    return 2.753e-14 * lam ** 1.5 / (1 + (lam / 2.740) ** 0.407) ** 2.242


def _hg97_b_cool(T, lam):
    return 3.435e-30 * T * lam ** 1.970 / (1 + (lam / 2.250) ** 0.376) ** 3.720


def _cen_dielectronic(T):
    return T ** -1.5 * math.exp(-470000.0 / T) * (1 + 0.3 * math.exp(-94000.0 / T))


def _hg97_ci(T, lam, a, p1, l0, p2, p3):
    return a * T ** -1.5 * math.exp(-lam / 2) * lam ** p1 / (1 + (lam / l0) ** p2) ** p3


def rate_coefficients(p, T):
    """(alpha_HII, alpha_HeII, alpha_HeIII, beta_HI, beta_HeI, beta_HeII)."""
    if p["rate_set"] == 0:
        return p["alpha_B_const"], 0.0, 0.0, 0.0, 0.0, 0.0
    T = max(T, 1.0)
    lH, lHe, lHe2 = 2 * TH_HI / T, 2 * TH_HEI / T, 2 * TH_HEII / T
    aH = _hg97_b(lH)
    aHe = 1.26e-14 * lHe ** 0.75 + 1.9e-3 * _cen_dielectronic(T)
    aHe2 = 2 * _hg97_b(lHe2)
    bH = _hg97_ci(T, lH, 21.11, -1.089, 0.354, 0.874, 1.101)
    bHe = _hg97_ci(T, lHe, 32.38, -1.146, 0.416, 0.987, 1.056)
    bHe2 = _hg97_ci(T, lHe2, 19.95, -1.089, 0.553, 0.735, 1.275)
    return aH, aHe, aHe2, bH, bHe, bHe2


def cooling_rate(p, T, nH, x, yhe):
    """Cooling per volume (erg cm^-3 s^-1)."""
    if p["rate_set"] == 0:
        return 0.0
    T = max(T, 1.0)
    xHI, xHII, yI, yII, yIII = x
    ne = nH * (xHII + yhe * (yII + 2 * yIII))
    n = dict(HI=nH * xHI, HII=nH * xHII, HeI=yhe * nH * yI, HeII=yhe * nH * yII, HeIII=yhe * nH * yIII)
    lH, lHe, lHe2 = 2 * TH_HI / T, 2 * TH_HEI / T, 2 * TH_HEII / T
    _, _, _, bH, bHe, bHe2 = rate_coefficients(p, T)
    total = 0.0
    total += _hg97_b_cool(T, lH) * n["HII"]
    total += KB * T * 1.26e-14 * lHe ** 0.75 * n["HeII"]
    total += 8 * _hg97_b_cool(T, lHe2) * n["HeIII"]
    total += 1.24e-13 * _cen_dielectronic(T) * n["HeII"]
    total += KB * (TH_HI * bH * n["HI"] + TH_HEI * bHe * n["HeI"] + TH_HEII * bHe2 * n["HeII"])
    root = 1 + math.sqrt(T / 1e5)
    total += 7.5e-19 * math.exp(-118348.0 / T) / root * n["HI"]
    total += 5.54e-17 * T ** -0.397 * math.exp(-473638.0 / T) / root * n["HeII"]
    g = 1.1 + 0.34 * math.exp(-(5.5 - math.log10(T)) ** 2 / 3)
    total += 1.42e-27 * g * math.sqrt(T) * (n["HII"] + n["HeII"] + 4 * n["HeIII"])
    return ne * total


def chemistry(p, Dt, nH, N, Fh, x, E, yhe, cnt):
    """One cell over one subcycle; E = rho u.  Returns (N, Fh, x, E)."""
    c, nb = p["c_reduced"], p["nb"]
    hhe = p["chem_mode"] == 2
    tracked = 5 if hhe else 2
    sig = np.asarray(p["sigma"], float).reshape(nb, 3)
    eh = np.asarray(p["e_heat"], float).reshape(nb, 3)
    gm1 = p["gamma"] - 1
    N, Fh, x = list(N), [np.array(v, float) for v in Fh], list(x)
    tau, d = 0.0, Dt
    att = 0
    while True:
        last = d >= Dt - tau
        if last:
            d = Dt - tau
        att += 1
        if att > p["chem_max_substeps"]:
            raise RuntimeError("substep cap")
        ntot = nH * (1 + yhe + x[1] + yhe * (x[3] + 2 * x[4]))
        T = p["T_iso"] if p["isothermal"] else gm1 * E / (ntot * KB)
        aH, aHe, aHe2, bH, bHe, bHe2 = rate_coefficients(p, T)
        ne = nH * (x[1] + yhe * (x[3] + 2 * x[4]))
        absorbers = (nH * x[0], yhe * nH * x[2], yhe * nH * x[3])
        # photons first: implicit absorption by the substep-start absorbers
        shrink, Nnew = [], []
        for b in range(nb):
            kap = sum(sig[b, s] * absorbers[s] for s in range(3))
            shrink.append(1 + c * d * kap)
            Nnew.append(N[b] / shrink[-1])
        gam = [c * sum(sig[b, s] * Nnew[b] for b in range(nb)) for s in range(3)]
        heat = sum(c * Nnew[b] * sig[b, s] * absorbers[s] * eh[b, s] for b in range(nb) for s in range(3))
        xn = list(x)
        den = 1 + (gam[0] + bH * ne + aH * ne) * d
        xn[0] = (x[0] + aH * ne * d) / den
        xn[1] = (x[1] + (gam[0] + bH * ne) * d) / den
        if hhe:
            xn[2] = (x[2] + aHe * ne * x[3] * d) / (1 + (gam[1] + bHe * ne) * d)
            xn[4] = (x[4] + (gam[2] + bHe2 * ne) * x[3] * d) / (1 + aHe2 * ne * d)
            xn[3] = 1 - xn[2] - xn[4]
            if xn[3] < 0:
                tot = xn[2] + xn[4]
                xn[2], xn[3], xn[4] = xn[2] / tot, 0.0, xn[4] / tot
        En = E
        change = 0.0
        if not p["isothermal"]:
            En = E + d * (heat - cooling_rate(p, T, nH, x, yhe))
            change = abs(En - E) / E
        for s in range(tracked):
            change = max(change, abs(xn[s] - x[s]) / max(x[s], p["chem_xfloor"]))
        if change > p["chem_fmax"]:
            d *= p["chem_fs"] / change
            continue
        N = Nnew
        Fh = [Fh[b] / shrink[b] for b in range(nb)]
        x, E = xn, En
        if last:
            break
        tau += d
        d *= min(p["chem_fs"] / change, p["chem_growth"]) if change > 0 else p["chem_growth"]
    cnt["substeps"] += att
    return N, Fh, x, E


# ---------------------------------------------------------------------------
# a whole run
# ---------------------------------------------------------------------------

def run(cfg, n_sub, dt=None):
    """Advance cfg's state by n_sub subcycles.  Returns the final fields in
    the oracle's layout and the event counters."""
    mesh, p, st = cfg["mesh"], cfg["params"], cfg["state"]
    nc, nb = mesh["n_cells"], p["nb"]
    c = p["c_reduced"]
    V, A, nrm = mesh["volume"], mesh["area"], mesh["normal"]
    faces = cell_faces(mesh)
    yhe = p["Y_He"] / (4 * (1 - p["Y_He"])) if p["chem_mode"] == 2 else 0.0
    if dt is None:
        dt = p["cfl_eta"] * min((3 * v / (4 * math.pi)) ** (1 / 3) for v in V) / c
    # state: U[b][i] = (N, Fh), x[i][5], E[i] = rho u
    U = [[np.concatenate([[st["N"][b, i]], st["F"][b, :, i] / c]) for i in range(nc)] for b in range(nb)]
    x = [list(st["species"][:, i]) for i in range(nc)]
    nH = [float(v) for v in st["n_H"]]
    gm1 = p["gamma"] - 1
    E = [nH[i] * (1 + yhe + x[i][1] + yhe * (x[i][3] + 2 * x[i][4])) * KB * st["T"][i] / gm1 for i in range(nc)]
    src_cell = [int(v) for v in cfg["sources"]["cell"]]
    src_rate = np.asarray(cfg["sources"]["rate"], float).reshape(nb, -1)
    cnt = dict(adm_N=0, adm_F=0, flux_caps=0, guard_N=0, guard_F=0, substeps=0, adm_ties=0, guard_ties=0)
    for _ in range(n_sub):
        for k, i in enumerate(src_cell):
            for b in range(nb):
                U[b][i] = U[b][i].copy()
                U[b][i][0] += src_rate[b, k] * dt / V[i]
        if p["chem_mode"] != 0:
            for i in range(nc):
                Nn, Fn, x[i], E[i] = chemistry(p, dt, nH[i], [U[b][i][0] for b in range(nb)],
                                               [U[b][i][1:] for b in range(nb)], x[i], E[i], yhe, cnt)
                for b in range(nb):
                    U[b][i] = np.concatenate([[Nn[b]], Fn[b]])
        # limited gradients of all cells from the start-of-transport state
        grad = [[None] * nc for _ in range(nb)]
        for b in range(nb):
            for i in range(nc):
                g = np.zeros((4, 3))
                for v in range(4):
                    items = [(A[f], ro - rn, U[b][j][v]) for (f, j, _, ro, rn) in faces[i]]
                    gv = lsq_gradient(U[b][i][v], items)
                    if p["use_limiter"]:
                        gv = limited(U[b][i][v], gv, [U[b][j][v] for (_, j, _, _, _) in faces[i]],
                                     [ro for (_, _, _, ro, _) in faces[i]])
                    g[v] = gv
                grad[b][i] = g
        newU = [[None] * nc for _ in range(nb)]
        for b in range(nb):
            for i in range(nc):
                parts = [[], [], [], []]
                for (f, j, sign, ro, rn) in faces[i]:
                    L, R = (i, j) if sign > 0 else (j, i)
                    rL, rR = (ro, rn) if sign > 0 else (rn, ro)
                    nvec = nrm[:, f]
                    count = sign > 0           # each face counted once, by its L cell
                    scratch = dict(adm_N=0, adm_F=0, adm_ties=0)
                    UL = admissible(U[b][L] + grad[b][L] @ rL, scratch)
                    UR = admissible(U[b][R] + grad[b][R] @ rR, scratch)
                    Phi = rusanov(UL, UR, nvec, c)
                    if Phi[0] != 0:
                        up = L if Phi[0] > 0 else R
                        theta = U[b][up][0] * V[up] / (len(faces[up]) * abs(Phi[0]) * dt * A[f])
                        if theta < 1:
                            Phi = theta * Phi
                            if count:
                                cnt["flux_caps"] += 1
                    if count:
                        for k in scratch:
                            cnt[k] += scratch[k]
                    for v in range(4):
                        parts[v].append(sign * A[f] * Phi[v])
                un = np.array([U[b][i][v] - dt / V[i] * math.fsum(parts[v]) for v in range(4)])
                if un[0] < 0:
                    un[0] = 0.0
                    cnt["guard_N"] += 1
                m = math.sqrt(float(un[1:] @ un[1:]))
                if abs(m - un[0]) <= TIE * max(m, abs(un[0])):
                    cnt["guard_ties"] += 1
                if m * m > un[0] * un[0]:
                    cnt["guard_F"] += 1
                    un[1:] = 0.0 if un[0] <= 0 else un[1:] * (un[0] / m)
                newU[b][i] = un
        U = newU
    out_N = np.array([[U[b][i][0] for i in range(nc)] for b in range(nb)])
    out_F = np.array([[[U[b][i][1 + k] * c for i in range(nc)] for k in range(3)] for b in range(nb)])
    species = np.array(x).T.copy()
    T = np.array([p["T_iso"] if p["isothermal"] else
                  gm1 * E[i] / (nH[i] * (1 + yhe + x[i][1] + yhe * (x[i][3] + 2 * x[i][4])) * KB)
                  for i in range(nc)])
    sums = [math.fsum(out_N[b, i] * V[i] for i in range(nc)) for b in range(nb)]
    return dict(N=out_N, F=out_F, species=species, T=T, counters=cnt, photon_sum=np.array(sums), dt=dt)
