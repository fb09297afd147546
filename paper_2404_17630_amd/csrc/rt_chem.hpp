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
//
// Everything is templated on the scalar type R (double in the forward
// kernels, Dual<K> in the adjoint's replay).
#pragma once

#include <hip/hip_runtime.h>

#include "rt_dual.hpp"
#include "rt_types.hpp"

namespace rtk {

constexpr double kBoltz = 1.380649e-16;            // erg/K (CODATA 2018)
constexpr double kProtonMass = 1.67262192369e-24;  // g
// Ionisation temperatures chi/k of H I, He I, He II (Hui & Gnedin 1997).
constexpr double kTHI = 157807.0;
constexpr double kTHeI = 285335.0;
constexpr double kTHeII = 631515.0;

// Every temperature-dependent coefficient of the network: the rates, and
// the cooling per pair of colliding species (erg cm^3/s), so that the
// cooling rate is a sum of products with the current densities.  Powers of
// the same base share one logarithm: x^p = exp(p ln x).
template <typename R>
struct Rates {
    R rec_HII, rec_HeII, rec_HeIII;    // recombination coefficients, cm^3/s
    R col_HI, col_HeI, col_HeII;       // collisional ionisation, cm^3/s
    // cooling coefficients: recombination of H II, He II, He III, dielectronic
    // recombination of He II, collisional excitation of H I and He II, and
    // free-free emission per ion charge weight
    R cr_HII, cr_HeII, cr_HeIII, cd_HeII, ce_HI, ce_HeII, cff;
};

// Every fit below is a product of powers and exponentials, so it is
// evaluated as one exponential of the summed exponent: x^p y^q e^z =
// exp(p ln x + q ln y + z).  A fit then costs one exp, plus one exp and one
// log for its (1 + (lambda/l0)^b)^-c factor.
template <typename R>
__device__ inline R log1p_pow(const R& ln_lam, double ln_l0, double b) {   // ln(1 + (lambda/l0)^b)
    return m_log(1.0 + m_exp(b * (ln_lam - ln_l0)));
}

// Case-B hydrogenic recombination of Hui & Gnedin in terms of
// lambda = 2 T_ion / T (ln lambda given):
// 2.753e-14 lambda^1.5 / (1 + (lambda/2.740)^0.407)^2.242.
template <typename R>
__device__ inline R hg_rec_caseB(const R& ln_lam) {
    return 2.753e-14 * m_exp(1.5 * ln_lam - 2.242 * log1p_pow(ln_lam, 1.007957920399979 /* ln 2.740 */, 0.407));
}
// Matching case-B recombination cooling coefficient (erg cm^3/s):
// 3.435e-30 T lambda^1.970 / (1 + (lambda/2.250)^0.376)^3.720.
template <typename R>
__device__ inline R hg_rec_cool_caseB(const R& T, const R& ln_lam) {
    return 3.435e-30 * T *
           m_exp(1.970 * ln_lam - 3.720 * log1p_pow(ln_lam, 0.8109302162163288 /* ln 2.250 */, 0.376));
}
// Hui & Gnedin collisional ionisation, A T^-3/2 e^(-lambda/2) lambda^-a /
// (1 + (lambda/l0)^b)^c.
template <typename R>
__device__ inline R hg_col(double A, const R& lnT, const R& lam, const R& ln_lam, double a, double ln_l0, double b,
                           double c) {
    return A * m_exp(-1.5 * lnT - 0.5 * lam - a * ln_lam - c * log1p_pow(ln_lam, ln_l0, b));
}

template <typename R>
__device__ inline Rates<R> network_rates(const ChemParams& P, R T) {
    Rates<R> r;
    if (P.rate_set == 0) {
        r.rec_HII = P.alpha_B;
        r.rec_HeII = 0.0; r.rec_HeIII = 0.0;
        r.col_HI = 0.0; r.col_HeI = 0.0; r.col_HeII = 0.0;
        r.cr_HII = 0.0; r.cr_HeII = 0.0; r.cr_HeIII = 0.0; r.cd_HeII = 0.0;
        r.ce_HI = 0.0; r.ce_HeII = 0.0; r.cff = 0.0;
        return r;
    }
    T = m_max(T, R(1.0));
    const R iT = 1.0 / T;
    const R lnT = m_log(T);
    const R lH = (2.0 * kTHI) * iT, lHe1 = (2.0 * kTHeI) * iT, lHe2 = (2.0 * kTHeII) * iT;
    const R ln_lH = 12.662275226919286 /* ln(2 T_HI) */ - lnT;
    const R ln_lHe1 = 13.254566388120152 /* ln(2 T_HeI) */ - lnT;
    const R ln_lHe2 = 14.049024154019651 /* ln(2 T_HeII) */ - lnT;
    const R sqT = m_sqrt(T);
    // Cen (1992) dielectronic recombination shape T^-3/2 e^(-470000/T) (1 + 0.3 e^(-94000/T)),
    // with e^(-470000/T) = (e^(-94000/T))^5
    const R e94 = m_exp(-94000.0 * iT);
    const R e94_2 = e94 * e94;
    const R diel = (iT / sqT) * (e94_2 * e94_2 * e94) * (1.0 + 0.3 * e94);
    const R rHe1 = 1.26e-14 * m_exp(0.75 * ln_lHe1);
    r.rec_HII = hg_rec_caseB(ln_lH);
    r.rec_HeII = rHe1 + 1.9e-3 * diel;
    r.rec_HeIII = 2.0 * hg_rec_caseB(ln_lHe2);
    r.col_HI = hg_col(21.11, lnT, lH, ln_lH, 1.089, -1.0384583658483626 /* ln 0.354 */, 0.874, 1.101);
    r.col_HeI = hg_col(32.38, lnT, lHe1, ln_lHe1, 1.146, -0.8770700187208739 /* ln 0.416 */, 0.987, 1.056);
    r.col_HeII = hg_col(19.95, lnT, lHe2, ln_lHe2, 1.089, -0.5923972774598022 /* ln 0.553 */, 0.735, 1.275);
    const R isq = 1.0 / (1.0 + 0.0031622776601683794 * sqT);   // 1 / (1 + (T / 1e5)^1/2)
    r.cr_HII = hg_rec_cool_caseB(T, ln_lH);
    r.cr_HeII = kBoltz * T * rHe1;
    r.cr_HeIII = 8.0 * hg_rec_cool_caseB(T, ln_lHe2);
    r.cd_HeII = 1.24e-13 * diel;
    r.ce_HI = 7.5e-19 * m_exp(-118348.0 * iT) * isq;
    r.ce_HeII = 5.54e-17 * m_exp(-0.397 * lnT - 473638.0 * iT) * isq;
    const R lg = 0.43429448190325182765 * lnT - 5.5;    // log10 T - 5.5
    r.cff = 1.42e-27 * (1.1 + 0.34 * m_exp(-lg * lg * (1.0 / 3.0))) * sqT;
    return r;
}

// Radiative cooling per volume (erg cm^-3 s^-1).  x = x_HI, x_HII, y_I, y_II, y_III.
template <typename R>
__device__ inline R cooling_rate(const ChemParams& P, const R& nH, const R* x, const Rates<R>& r) {
    if (P.rate_set == 0) return R(0.0);
    const double yhe = P.yhe;
    const R ne = nH * (x[1] + yhe * (x[3] + 2.0 * x[4]));
    const R nHI = nH * x[0], nHII = nH * x[1];
    const R nHe = yhe * nH;
    const R nHeI = nHe * x[2], nHeII = nHe * x[3], nHeIII = nHe * x[4];
    // recombination (radiative, case B) and dielectronic recombination
    R L = r.cr_HII * nHII + r.cr_HeII * nHeII + r.cr_HeIII * nHeIII + r.cd_HeII * nHeII;
    // collisional ionisation: one ionisation energy per event
    L += kBoltz * (kTHI * r.col_HI * nHI + kTHeI * r.col_HeI * nHeI + kTHeII * r.col_HeII * nHeII);
    // collisional excitation of H I and He II
    L += r.ce_HI * nHI + r.ce_HeII * nHeII;
    // free-free emission
    L += r.cff * (nHII + nHeII + 4.0 * nHeIII);
    return ne * L;
}

// Mean particle mass per proton mass for the current ionisation state.
template <typename R>
__device__ inline R mean_mass(const ChemParams& P, const R* x) {
    const R xe = x[1] + P.yhe * (x[3] + 2.0 * x[4]);
    return (1.0 + 4.0 * P.yhe) / (1.0 + P.yhe + xe);
}

template <typename R>
__device__ inline R temperature(const ChemParams& P, const R& u, const R* x) {
    return P.gm1 * mean_mass(P, x) * kProtonMass * u / kBoltz;
}

// Integration state of one cell within a subcycle.
template <int NB, typename R>
struct ChemState {
    R N[NB];
    R Fh[NB][3];
    R x[5];
    R u;
    R tau;       // time integrated so far
    R d;         // proposed step
    int attempts;
};

template <int NB, typename R>
__device__ inline void chem_begin(double Dt, ChemState<NB, R>& s) {
    s.tau = R(0.0);
    s.d = R(Dt);
    s.attempts = 0;
}

// One attempt of the adaptive semi-implicit step.  Returns 1 when the
// subcycle is complete, 0 to continue, -1 when the attempt cap is exceeded.
template <int NB, typename R>
__device__ inline int chem_attempt(const ChemParams& P, double Dt, const R& nH, ChemState<NB, R>& s) {
    const bool hhe = P.chem_mode == 2;
    const double ct = P.c;
    const double yhe = P.yhe;
    bool last = false;
    if (val(s.d) >= val(Dt - s.tau)) { s.d = Dt - s.tau; last = true; }
    if (++s.attempts > P.max_sub) return -1;
    const R d = s.d;
    R* x = s.x;

    const R T = P.isothermal ? R(P.T_iso) : temperature(P, s.u, x);
    const Rates<R> r = network_rates(P, T);
    const R ne = nH * (x[1] + yhe * (x[3] + 2.0 * x[4]));
    const R nHI = nH * x[0];
    const R nHeI = yhe * nH * x[2];
    const R nHeII = yhe * nH * x[3];

    R ifac[NB], Nn[NB];
    R G0 = 0.0, G1 = 0.0, G2 = 0.0, heat = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const R kap = P.sigma[b][0] * nHI + P.sigma[b][1] * nHeI + P.sigma[b][2] * nHeII;
        ifac[b] = 1.0 / (1.0 + ct * d * kap);
        Nn[b] = s.N[b] * ifac[b];
        G0 += ct * P.sigma[b][0] * Nn[b];
        G1 += ct * P.sigma[b][1] * Nn[b];
        G2 += ct * P.sigma[b][2] * Nn[b];
        heat += ct * Nn[b] * (P.sigma[b][0] * nHI * P.eheat[b][0] + P.sigma[b][1] * nHeI * P.eheat[b][1] +
                              P.sigma[b][2] * nHeII * P.eheat[b][2]);
    }

    R xn[5];
    const R iden = 1.0 / (1.0 + (G0 + r.col_HI * ne + r.rec_HII * ne) * d);
    xn[0] = (x[0] + r.rec_HII * ne * d) * iden;
    xn[1] = (x[1] + (G0 + r.col_HI * ne) * d) * iden;
    if (hhe) {
        xn[2] = (x[2] + r.rec_HeII * ne * x[3] * d) / (1.0 + (G1 + r.col_HeI * ne) * d);
        xn[4] = (x[4] + (G2 + r.col_HeII * ne) * x[3] * d) / (1.0 + r.rec_HeIII * ne * d);
        xn[3] = 1.0 - xn[2] - xn[4];
        if (val(xn[3]) < 0.0) {
            xn[3] = 0.0;
            const R sm = xn[2] + xn[4];
            xn[2] = xn[2] / sm;
            xn[4] = xn[4] / sm;
        }
    } else {
        xn[2] = x[2]; xn[3] = x[3]; xn[4] = x[4];
    }

    // Largest relative change: each candidate is a fraction |change| / scale,
    // compared without dividing; one division gives f.
    R un = s.u;
    R fnum = 0.0, fden = 1.0;
    if (!P.isothermal) {
        const R rho = kProtonMass * nH * (1.0 + 4.0 * yhe);
        un = s.u + d * (heat - cooling_rate(P, nH, x, r)) / rho;
        fnum = m_abs(un - s.u);
        fden = s.u;
    }
    const int ns = hhe ? 5 : 2;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        if (q >= ns) break;
        const R num = m_abs(xn[q] - x[q]);
        const R den = m_max(x[q], R(P.xfloor));
        if (val(num) * val(fden) > val(fnum) * val(den)) { fnum = num; fden = den; }
    }
    const R f = fnum / fden;

    if (val(f) > P.fmax) {
        s.d = d * (P.fs / f);
        return 0;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        s.N[b] = Nn[b];
        s.Fh[b][0] = s.Fh[b][0] * ifac[b];
        s.Fh[b][1] = s.Fh[b][1] * ifac[b];
        s.Fh[b][2] = s.Fh[b][2] * ifac[b];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) x[q] = xn[q];
    s.u = un;
    if (last) return 1;
    s.tau = s.tau + d;
    s.d = val(f) > 0.0 ? d * m_min(P.fs / f, R(P.growth)) : d * P.growth;
    return 0;
}

// Integrate one cell over the subcycle Dt; returns the number of attempts
// (> max_sub on failure).
template <int NB, typename R>
__device__ inline int integrate_cell(const ChemParams& P, double Dt, const R& nH, ChemState<NB, R>& s) {
    chem_begin<NB, R>(Dt, s);
    while (true) {
        const int r = chem_attempt<NB, R>(P, Dt, nH, s);
        if (r == 1) break;
        if (r < 0) break;
    }
    return s.attempts;
}

}  // namespace rtk
