"""Seeded synthetic fields: lognormal density, density peaks, power-law sources,
and per-bin photoionisation cross-sections and excess energies.

None of this is the radiative-transfer method itself: these are the inputs the
method is run on (gas density, source positions and rates, and the per-bin
opacity and heating constants the library takes as parameters).
"""
from __future__ import annotations

import numpy as np

# Physical constants (CODATA 2018), cgs.
K_BOLTZ = 1.380649e-16
H_PLANCK = 6.62607015e-27
EV = 1.602176634e-12
C_LIGHT = 2.99792458e10
KPC = 3.0856775814913673e21

# Ionisation thresholds (eV).
E_HI, E_HEI, E_HEII = 13.6, 24.6, 54.4
# Threshold cross-sections (cm^2) of the hydrogenic nu^-3 laws.
SIGMA0_HI, SIGMA0_HEII = 6.30e-18, 1.58e-18


def gaussian_random_field(dims, h: float, width: float, seed: int) -> np.ndarray:
    """Unit-variance periodic Gaussian random field on the lattice (lexicographic,
    x fastest): white noise filtered in Fourier space by a Gaussian kernel of
    width ``width`` (same length unit as ``h``)."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((nz, ny, nx))
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=h)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=h)
    kz = 2 * np.pi * np.fft.fftfreq(nz, d=h)
    kk = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    g = np.real(np.fft.ifftn(np.fft.fftn(white) * np.exp(-0.5 * kk * width ** 2)))
    g -= g.mean()
    g /= g.std()
    return g.reshape(-1)


def lognormal_density(g: np.ndarray, mean: float, sigma_ln: float) -> np.ndarray:
    """n = mean * exp(sigma_ln g - sigma_ln^2/2): mean-preserving for unit-variance g."""
    return mean * np.exp(sigma_ln * g - 0.5 * sigma_ln ** 2)


def density_peaks(n_lex: np.ndarray, dims, key_lex: np.ndarray, k: int) -> np.ndarray:
    """Lexicographic ids of the k highest strict local maxima (26 periodic
    neighbours), ties broken by the lower Hilbert key.  A lattice too small to
    hold k maxima takes the densest remaining cells after the maxima."""
    nx, ny, nz = dims
    a = n_lex.reshape(nz, ny, nx)
    is_peak = np.ones_like(a, dtype=bool)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == dy == dz == 0:
                    continue
                is_peak &= a > np.roll(a, shift=(dz, dy, dx), axis=(0, 1, 2))
    flat = is_peak.reshape(-1)
    if k > flat.size:
        raise ValueError(f"{k} sources for {flat.size} cells")
    ids = np.arange(flat.size)
    # peaks first, then by density (descending), then Hilbert key
    order = np.lexsort((key_lex, -n_lex, ~flat))
    return ids[order[:k]]


def power_law_luminosities(k: int, lmin: float, lmax: float, seed: int) -> np.ndarray:
    """Inverse-CDF draws from dN/dL ~ L^-2 on [lmin, lmax]."""
    u = np.random.default_rng(seed).uniform(0.0, 1.0, size=k)
    return 1.0 / (1.0 / lmin - u * (1.0 / lmin - 1.0 / lmax))


# --- per-bin cross-sections -------------------------------------------------

def sigma_hi(e_ev):
    e = np.asarray(e_ev, dtype=float)
    return np.where(e >= E_HI, SIGMA0_HI * (e / E_HI) ** -3.0, 0.0)


def sigma_heii(e_ev):
    e = np.asarray(e_ev, dtype=float)
    return np.where(e >= E_HEII, SIGMA0_HEII * (e / E_HEII) ** -3.0, 0.0)


def sigma_hei(e_ev):
    """He I photoionisation cross-section, two-power-law fit of Osterbrock
    (Astrophysics of Gaseous Nebulae, 1989, Table 2.2 form)."""
    e = np.asarray(e_ev, dtype=float)
    y = e / E_HEI
    return np.where(e >= E_HEI, 7.42e-18 * (1.66 * y ** -2.05 - 0.66 * y ** -3.05), 0.0)


def blackbody_bin_constants(t_eff: float, edges_ev, e_max_ev: float = 1000.0, n_grid: int = 20001):
    """Photon-number-weighted mean cross-sections sigma[b][s] (cm^2) and mean
    excess energies per absorption e_heat[b][s] (erg) for species
    s = (HI, HeI, HeII) over bins [edges[b], edges[b+1]) of a black body."""
    edges = list(edges_ev) + [e_max_ev]
    kt = K_BOLTZ * t_eff / EV
    thresholds = (E_HI, E_HEI, E_HEII)
    fns = (sigma_hi, sigma_hei, sigma_heii)
    nb = len(edges) - 1
    sig = np.zeros((nb, 3))
    eh = np.zeros((nb, 3))
    for b in range(nb):
        # midpoint rule on the half-open bin [lo, hi)
        de = (edges[b + 1] - edges[b]) / n_grid
        e = edges[b] + (np.arange(n_grid) + 0.5) * de
        nphot = e ** 2 / np.expm1(e / kt)          # B_nu / (h nu) up to a constant
        norm = nphot.sum()
        for s in range(3):
            sv = fns[s](e)
            w = (sv * nphot).sum()
            sig[b, s] = w / norm
            if w > 0:
                eh[b, s] = (sv * (e - thresholds[s]) * nphot).sum() / w * EV
    return sig, eh
