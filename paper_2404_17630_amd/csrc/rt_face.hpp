// Face physics of the M1 subcycle (Zier et al. 2024, Sec. 2.3.3), templated
// on the state scalar R (float, double or Dual<K>) and the geometry scalar G
// (float or double):
//   * admissibility of an extrapolated state: N >= 0 and |Fh| <= N;
//   * the M1 Eddington tensor (eq. edd) with the Levermore factor
//     chi(f) = (3 + 4 f^2) / (5 + 2 sqrt(4 - 3 f^2)), f = |Fh| / N clamped to 1;
//   * the HLL flux with wave-speed bounds -c~ and +c~ (the M1 eigenvalues lie
//     in [-c~, c~], so this is the Rusanov flux and needs no rotation to the
//     face frame), in units of c~:
//       Phi_N  = (Fh_L + Fh_R).n / 2 - (N_R - N_L) / 2
//       Phi_Fh = (N_L D_L + N_R D_R) n / 2 - (Fh_R - Fh_L) / 2;
//   * the outflow cap theta = min(1, N_up V_up / (n_faces(up) |Phi_N| c~ dt A))
//     on all four components, with N_up the cell average of the upwind cell.
#pragma once

#include <hip/hip_runtime.h>

#include "rt_dual.hpp"

namespace rtk {

// Relative size below which the flux of N through a face counts as
// rounding noise of its terms and of the two cells' contents (see
// face_flux).
constexpr double kCapNoise = 1.0e-12;

template <typename R, typename G>
__device__ inline void make_admissible(R* U, int& cN, int& cF) {
#pragma clang fp contract(off)
    if (val(U[0]) < 0) { U[0] = R(G(0)); ++cN; }
    const R F2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
    if (val(F2) > val(U[0] * U[0])) {
        ++cF;
        if (val(U[0]) <= 0) {
            U[1] = R(G(0)); U[2] = R(G(0)); U[3] = R(G(0));
        } else {
            const R s = U[0] / m_sqrt(F2);
            U[1] = U[1] * s; U[2] = U[2] * s; U[3] = U[3] * s;
        }
    }
}

// N D n for state U = (N, Fh).
template <typename R, typename G>
__device__ inline void radiation_pressure_n(const R* U, G n0, G n1, G n2, R* P) {
#pragma clang fp contract(off)
    const R N = U[0];
    const R F2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
    // Isotropic when f = |Fh|/N <= 1e-8: the anisotropic part of D is
    // (3 chi - 1)/2 = O(f^2) <= 1e-16, below the rounding of either
    // precision, and the direction of a vanishing Fh (whose derivative is
    // 1/|Fh|) does not enter.
    if (val(N) <= 0 || val(F2) <= G(1e-16) * val(N) * val(N)) {
        const R third = N * G(1.0 / 3.0);
        P[0] = third * n0; P[1] = third * n1; P[2] = third * n2;
        return;
    }
    // D = (1 - chi)/2 I + (3 chi - 1)/2 u u with the unit vector u = Fh / |Fh|;
    // chi depends on f^2 = |Fh|^2 / N^2 only, and (u . n) u = (Fh . n) Fh /
    // |Fh|^2, so the values need no square root of |Fh|^2.  On duals u is
    // formed by dividing by |Fh| rather than |Fh|^2, which keeps the
    // derivative finite down to the smallest |Fh| whose square is nonzero.
    if constexpr (IsDualT<R>::value) {
        const R Fm = m_sqrt(F2);
        R f = Fm / N;
        if (val(f) > 1) f = R(G(1));
        const R f2 = f * f;
        const R chi = (G(3) + G(4) * f2) / (G(5) + G(2) * m_sqrt(G(4) - G(3) * f2));
        const R iso = G(0.5) * (G(1) - chi);
        const R iFm = G(1) / Fm;
        const R u0 = U[1] * iFm, u1 = U[2] * iFm, u2 = U[3] * iFm;
        const R dir = G(0.5) * (G(3) * chi - G(1)) * (u0 * n0 + u1 * n1 + u2 * n2);
        P[0] = N * (iso * n0 + dir * u0);
        P[1] = N * (iso * n1 + dir * u1);
        P[2] = N * (iso * n2 + dir * u2);
    } else {
        R f2 = F2 / (N * N);
        if (val(f2) > 1) f2 = R(G(1));
        const R chi = (G(3) + G(4) * f2) / (G(5) + G(2) * m_sqrt(G(4) - G(3) * f2));
        const R iso = G(0.5) * (G(1) - chi);
        const R dir = G(0.5) * (G(3) * chi - G(1)) * (U[1] * n0 + U[2] * n1 + U[3] * n2) / F2;
        P[0] = N * (iso * n0 + dir * U[1]);
        P[1] = N * (iso * n1 + dir * U[2]);
        P[2] = N * (iso * n2 + dir * U[3]);
    }
}

template <typename R, typename G>
__device__ inline void hll_flux(const R* UL, const R* UR, G n0, G n1, G n2, R* Phi) {
#pragma clang fp contract(off)
    R PL[3], PR[3];
    radiation_pressure_n<R, G>(UL, n0, n1, n2, PL);
    radiation_pressure_n<R, G>(UR, n0, n1, n2, PR);
    const R FLn = UL[1] * n0 + UL[2] * n1 + UL[3] * n2;
    const R FRn = UR[1] * n0 + UR[2] * n1 + UR[3] * n2;
    Phi[0] = G(0.5) * (FLn + FRn) - G(0.5) * (UR[0] - UL[0]);
    Phi[1] = G(0.5) * (PL[0] + PR[0]) - G(0.5) * (UR[1] - UL[1]);
    Phi[2] = G(0.5) * (PL[1] + PR[1]) - G(0.5) * (UR[2] - UL[2]);
    Phi[3] = G(0.5) * (PL[2] + PR[2]) - G(0.5) * (UR[3] - UL[3]);
}

// The face physics is evaluated without contracting products into fused
// multiply-adds, so every kernel that inlines it (the split and fused
// transport, the adjoint) rounds a face's flux the same way.

// Full face flux from the raw extrapolated states sL, sR (modified in place
// by the admissibility fix) and the cell averages NL, NR of the two cells.
// vcL, vcR = V / n_faces of the cells; cdt = c~ dt / h.  Returns capped.
template <typename R, typename G>
__device__ inline bool face_flux(R* sL, R* sR, const R& NL, const R& NR, G vcL, G vcR, G n0, G n1, G n2, G A,
                                 G cdt, R* Phi, int& aN, int& aF) {
#pragma clang fp contract(off)
    make_admissible<R, G>(sL, aN, aF);
    make_admissible<R, G>(sR, aN, aF);
    hll_flux<R, G>(sL, sR, n0, n1, n2, Phi);
    if (val(Phi[0]) != 0) {
        const bool upL = val(Phi[0]) > 0;
        const R Nup = sel(upL, NL, NR);
        const G vc = upL ? vcL : vcR;
        const R q = m_abs(Phi[0]) * cdt * A;
        if (val(Nup) * vc < val(q)) {
            // The flux of N is a difference of terms of size N_L* + N_R*; when
            // it is at their rounding level, or at that of the two cells'
            // contents (free streaming along n into an empty cell, a face
            // state that is the rounding residue of a limited extrapolation),
            // its sign and size are noise, and so is the dependence of theta
            // on the face states: theta is then held constant for the
            // derivative.  The value is the same either way.
            const bool noise = (double)val(m_abs(Phi[0])) <=
                               kCapNoise * ((double)val(sL[0]) + (double)val(sR[0]) + (double)val(NL) +
                                            (double)val(NR));
            if (noise) {
                const auto th = val(Nup) * vc / val(q);
#pragma unroll
                for (int v = 0; v < 4; ++v) Phi[v] = Phi[v] * th;
            } else {
                const R cap = Nup * vc / q;
#pragma unroll
                for (int v = 0; v < 4; ++v) Phi[v] = cap * Phi[v];
            }
            return true;
        }
    }
    return false;
}

// Post-update guards on the new cell state (N >= 0, |Fh| <= N).
template <typename R>
__device__ inline void update_guards(R* un, int& cN, int& cF) {
    if (val(un[0]) < 0.0) { un[0] = R(0.0); ++cN; }
    const R F2 = un[1] * un[1] + un[2] * un[2] + un[3] * un[3];
    if (val(F2) > val(un[0] * un[0])) {
        ++cF;
        if (val(un[0]) <= 0.0) {
            un[1] = R(0.0); un[2] = R(0.0); un[3] = R(0.0);
        } else {
            const R s = un[0] / m_sqrt(F2);
            un[1] = un[1] * s; un[2] = un[2] * s; un[3] = un[3] * s;
        }
    }
}

}  // namespace rtk
