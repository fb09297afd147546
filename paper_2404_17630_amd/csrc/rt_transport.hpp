// Per-cell flux sum of the M1 subcycle: one lane computes, for each face of
// its cell, both extrapolated face states from the start-of-transport
// fields and gradients (U* = U + g . r), the face flux in the face's
// canonical (L, R) orientation (rt_face.hpp), and accumulates sigma A Phi in
// face-index order in FP64.  Shared by the forward flux kernel and by the
// adjoint, which recomputes the pre-guard update.
#pragma once

#include <hip/hip_runtime.h>

#include "rt_face.hpp"
#include "rt_types.hpp"

namespace rtk {

template <typename T>
__device__ inline void cell_flux_sum(int64_t i, int64_t nc, const T* __restrict__ Ub, const T* __restrict__ Gb,
                                     const GeomView<T>& geo, const SellView& sell, T cdt, const T* ui,
                                     const T (*gi)[3], T vcap_i, double* acc, int& cAdmN, int& cAdmF, int& cCap) {
    const int64_t nf = geo.nf;
    const int64_t slice = i / kSlice;
    const int32_t deg = sell.deg[slice];
    const int64_t base = (int64_t)sell.ptr[slice] + (i % kSlice);
    for (int k = 0; k < deg; ++k) {
        const int64_t e = base + (int64_t)k * kSlice;
        const int32_t j = sell.nbr[e];
        if (j < 0) continue;
        const int32_t fs = sell.fsf[e];
        const bool isL = fs >= 0;
        const int64_t f = isL ? fs : ~fs;
        const T A = geo.face[f];
        const T n0 = geo.face[nf + f], n1 = geo.face[2 * nf + f], n2 = geo.face[3 * nf + f];
        T rl[3], rr[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            rl[c] = geo.face[(4 + c) * nf + f];
            rr[c] = geo.face[(7 + c) * nf + f];
        }
        T uj[4], gj[4][3];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            uj[v] = Ub[(int64_t)v * nc + j];
#pragma unroll
            for (int c = 0; c < 3; ++c) gj[v][c] = Gb[(int64_t)(v * 3 + c) * nc + j];
        }
        const T vcap_j = geo.vcap[j];
        // Canonical orientation: L then R, whichever lane computes it.
        T UL[4], UR[4], sL[4], sR[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            UL[v] = isL ? ui[v] : uj[v];
            UR[v] = isL ? uj[v] : ui[v];
            const T gl0 = isL ? gi[v][0] : gj[v][0], gl1 = isL ? gi[v][1] : gj[v][1], gl2 = isL ? gi[v][2] : gj[v][2];
            const T gr0 = isL ? gj[v][0] : gi[v][0], gr1 = isL ? gj[v][1] : gi[v][1], gr2 = isL ? gj[v][2] : gi[v][2];
            sL[v] = UL[v] + (gl0 * rl[0] + gl1 * rl[1] + gl2 * rl[2]);
            sR[v] = UR[v] + (gr0 * rr[0] + gr1 * rr[1] + gr2 * rr[2]);
        }
        int aN = 0, aF = 0;
        T Phi[4];
        const T vcL = isL ? vcap_i : vcap_j, vcR = isL ? vcap_j : vcap_i;
        const bool capped = face_flux<T, T>(sL, sR, UL[0], UR[0], vcL, vcR, n0, n1, n2, A, cdt, Phi, aN, aF);
        if (isL) {
            cAdmN += aN; cAdmF += aF; cCap += capped ? 1 : 0;
        }
        const T sA = isL ? A : -A;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += (double)(sA * Phi[v]);
    }
}

}  // namespace rtk
