// Per-cell non-equilibrium H/He photo-thermochemistry on the device.
//
// Zier et al. (2024) Sec. 2.3.1 and Sec. 4.1.1: one lane integrates one cell
// over the subcycle with adaptive semi-implicit substeps held in registers.
// Each substep:
//   * absorbs photons implicitly with the substep-start absorber densities,
//     N' = N / (1 + c~ d sum_s sigma_bs n_s), the flux scaled alike;
//   * updates the abundances implicitly with frozen rates, n_e and the
//     photoionisation rates Gamma_s = c~ sum_b sigma_bs N'_b;
//   * updates the thermal energy explicitly with the photoheating of N'.
// The step is rejected when any of u and the tracked fractions changes by
// more than f_max; the retry uses d f_s / f, an accepted step proposes
// d min(f_s / f, growth) for the next, and the last step is clipped to end
// on the subcycle.
//
// The network constants are not in the paper (it cites Kannan et al. 2019);
// rate set RT_RATES_HG97 uses Hui & Gnedin (1997, MNRAS 292, 27) case-B
// recombination, collisional ionisation and their cooling, and Cen (1992,
// ApJS 78, 341) dielectronic recombination, collisional-excitation cooling and
// the free-free Gaunt factor.  Fits are evaluated at T >= 1 K.
#pragma once

#include <hip/hip_runtime.h>

#include "rt_types.hpp"

namespace rtk {

constexpr double kBoltz = 1.380649e-16;     // erg/K (CODATA 2018)
constexpr double kProtonMass = 1.67262192369e-24;  // g
// Ionisation temperatures chi/k of H I, He I, He II (Hui & Gnedin 1997).
constexpr double kTHI = 157807.0;
constexpr double kTHeI = 285335.0;
constexpr double kTHeII = 631515.0;

struct Rates {
    double rec_HII, rec_HeII, rec_HeIII;    // recombination coefficients, cm^3/s
    double col_HI, col_HeI, col_HeII;       // collisional ionisation, cm^3/s
};

// Case-B hydrogenic recombination of Hui & Gnedin in terms of
// lambda = 2 T_ion / T.
__device__ inline double hg_rec_caseB(double lam) {
    return 2.753e-14 * pow(lam, 1.5) / pow(1.0 + pow(lam * (1.0 / 2.740), 0.407), 2.242);
}
// Matching case-B recombination cooling coefficient (erg cm^3/s).
__device__ inline double hg_rec_cool_caseB(double T, double lam) {
    return 3.435e-30 * T * pow(lam, 1.970) / pow(1.0 + pow(lam * (1.0 / 2.250), 0.376), 3.720);
}
// Temperature shape of dielectronic He II recombination (Cen 1992).
__device__ inline double cen_dielectronic(double T) {
    return pow(T, -1.5) * exp(-470000.0 / T) * (1.0 + 0.3 * exp(-94000.0 / T));
}

__device__ inline Rates network_rates(const ChemParams& P, double T) {
    Rates r;
    if (P.rate_set == 0) {
        r.rec_HII = P.alpha_B;
        r.rec_HeII = r.rec_HeIII = 0.0;
        r.col_HI = r.col_HeI = r.col_HeII = 0.0;
        return r;
    }
    T = fmax(T, 1.0);
    const double lH = 2.0 * kTHI / T, lHe1 = 2.0 * kTHeI / T, lHe2 = 2.0 * kTHeII / T;
    const double t32 = pow(T, -1.5);
    r.rec_HII = hg_rec_caseB(lH);
    r.rec_HeII = 1.26e-14 * pow(lHe1, 0.75) + 1.9e-3 * cen_dielectronic(T);
    r.rec_HeIII = 2.0 * hg_rec_caseB(lHe2);
    r.col_HI = 21.11 * t32 * exp(-0.5 * lH) * pow(lH, -1.089) / pow(1.0 + pow(lH * (1.0 / 0.354), 0.874), 1.101);
    r.col_HeI = 32.38 * t32 * exp(-0.5 * lHe1) * pow(lHe1, -1.146) / pow(1.0 + pow(lHe1 * (1.0 / 0.416), 0.987), 1.056);
    r.col_HeII = 19.95 * t32 * exp(-0.5 * lHe2) * pow(lHe2, -1.089) / pow(1.0 + pow(lHe2 * (1.0 / 0.553), 0.735), 1.275);
    return r;
}

// Radiative cooling per volume (erg cm^-3 s^-1).  x = x_HI, x_HII, y_I, y_II, y_III.
__device__ inline double cooling_rate(const ChemParams& P, double T, double nH, const double* x, const Rates& r) {
    if (P.rate_set == 0) return 0.0;
    T = fmax(T, 1.0);
    const double yhe = P.yhe;
    const double ne = nH * (x[1] + yhe * (x[3] + 2.0 * x[4]));
    const double nHI = nH * x[0], nHII = nH * x[1];
    const double nHe = yhe * nH;
    const double nHeI = nHe * x[2], nHeII = nHe * x[3], nHeIII = nHe * x[4];
    const double lH = 2.0 * kTHI / T, lHe1 = 2.0 * kTHeI / T, lHe2 = 2.0 * kTHeII / T;
    const double sq = 1.0 + sqrt(T * 1.0e-5);
    // recombination (radiative, case B) and dielectronic recombination
    double L = hg_rec_cool_caseB(T, lH) * nHII
             + kBoltz * T * 1.26e-14 * pow(lHe1, 0.75) * nHeII
             + 8.0 * hg_rec_cool_caseB(T, lHe2) * nHeIII
             + 1.24e-13 * cen_dielectronic(T) * nHeII;
    // collisional ionisation: one ionisation energy per event
    L += kBoltz * (kTHI * r.col_HI * nHI + kTHeI * r.col_HeI * nHeI + kTHeII * r.col_HeII * nHeII);
    // collisional excitation of H I and He II
    L += 7.5e-19 * exp(-118348.0 / T) / sq * nHI + 5.54e-17 * pow(T, -0.397) * exp(-473638.0 / T) / sq * nHeII;
    // free-free emission
    const double lg = log10(T) - 5.5;
    const double gff = 1.1 + 0.34 * exp(-lg * lg * (1.0 / 3.0));
    L += 1.42e-27 * gff * sqrt(T) * (nHII + nHeII + 4.0 * nHeIII);
    return ne * L;
}

// Mean particle mass per proton mass for the current ionisation state.
__device__ inline double mean_mass(const ChemParams& P, const double* x) {
    const double xe = x[1] + P.yhe * (x[3] + 2.0 * x[4]);
    return (1.0 + 4.0 * P.yhe) / (1.0 + P.yhe + xe);
}

__device__ inline double temperature(const ChemParams& P, double u, const double* x) {
    return P.gm1 * mean_mass(P, x) * kProtonMass * u / kBoltz;
}

// Integrate one cell over the subcycle Dt.  N[b], Fh[b][3], x[5] and u are
// updated in place; returns the number of attempts (> max_sub on failure).
template <int NB>
__device__ inline int integrate_cell(const ChemParams& P, double Dt, double nH, double* N, double (*Fh)[3],
                                     double* x, double& u) {
    const bool hhe = P.chem_mode == 2;
    const double ct = P.c;
    const double yhe = P.yhe;
    const double rho = kProtonMass * nH * (1.0 + 4.0 * yhe);
    double tau = 0.0;
    double d = Dt;
    int attempts = 0;
    while (true) {
        bool last = false;
        if (d >= Dt - tau) { d = Dt - tau; last = true; }
        if (++attempts > P.max_sub) return attempts;

        const double T = P.isothermal ? P.T_iso : temperature(P, u, x);
        const Rates r = network_rates(P, T);
        const double ne = nH * (x[1] + yhe * (x[3] + 2.0 * x[4]));
        const double nHI = nH * x[0];
        const double nHeI = yhe * nH * x[2];
        const double nHeII = yhe * nH * x[3];

        double fac[NB], Nn[NB];
        double G0 = 0.0, G1 = 0.0, G2 = 0.0, heat = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const double kap = P.sigma[b][0] * nHI + P.sigma[b][1] * nHeI + P.sigma[b][2] * nHeII;
            fac[b] = 1.0 + ct * d * kap;
            Nn[b] = N[b] / fac[b];
            G0 += ct * P.sigma[b][0] * Nn[b];
            G1 += ct * P.sigma[b][1] * Nn[b];
            G2 += ct * P.sigma[b][2] * Nn[b];
            heat += ct * Nn[b] * (P.sigma[b][0] * nHI * P.eheat[b][0] + P.sigma[b][1] * nHeI * P.eheat[b][1] +
                                  P.sigma[b][2] * nHeII * P.eheat[b][2]);
        }

        double xn[5];
        const double den = 1.0 + (G0 + r.col_HI * ne + r.rec_HII * ne) * d;
        xn[0] = (x[0] + r.rec_HII * ne * d) / den;
        xn[1] = (x[1] + (G0 + r.col_HI * ne) * d) / den;
        if (hhe) {
            xn[2] = (x[2] + r.rec_HeII * ne * x[3] * d) / (1.0 + (G1 + r.col_HeI * ne) * d);
            xn[4] = (x[4] + (G2 + r.col_HeII * ne) * x[3] * d) / (1.0 + r.rec_HeIII * ne * d);
            xn[3] = 1.0 - xn[2] - xn[4];
            if (xn[3] < 0.0) {
                xn[3] = 0.0;
                const double s = xn[2] + xn[4];
                xn[2] = xn[2] / s;
                xn[4] = xn[4] / s;
            }
        } else {
            xn[2] = x[2]; xn[3] = x[3]; xn[4] = x[4];
        }

        double un = u;
        double f = 0.0;
        if (!P.isothermal) {
            un = u + d * (heat - cooling_rate(P, T, nH, x, r)) / rho;
            f = fabs(un - u) / u;
        }
        const int ns = hhe ? 5 : 2;
        for (int s = 0; s < ns; ++s) f = fmax(f, fabs(xn[s] - x[s]) / fmax(x[s], P.xfloor));

        if (f > P.fmax) {
            d = d * (P.fs / f);
            continue;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            N[b] = Nn[b];
            Fh[b][0] = Fh[b][0] / fac[b];
            Fh[b][1] = Fh[b][1] / fac[b];
            Fh[b][2] = Fh[b][2] / fac[b];
        }
        for (int s = 0; s < 5; ++s) x[s] = xn[s];
        u = un;
        if (last) break;
        tau = tau + d;
        d = f > 0.0 ? d * fmin(P.fs / f, P.growth) : d * P.growth;
    }
    return attempts;
}

}  // namespace rtk
