// Transport pieces shared by the forward kernels and the adjoint.
//
// Records are read with 16-byte vector loads (one float4 or two double2 per
// four values), so a gathered neighbour record costs one or two memory
// instructions per lane instead of four scalar gathers.
#pragma once

#include <hip/hip_runtime.h>

#include "rt_face.hpp"
#include "rt_types.hpp"

namespace rtk {

__device__ inline void load4(const float* __restrict__ p, float* o) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ inline void load4(const double* __restrict__ p, double* o) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
__device__ inline void store4(float* __restrict__ p, const float* v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ inline void store4(double* __restrict__ p, const double* v) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
}

// The face record: A, n, rL, rR, vcap_L, vcap_R.
template <typename T>
struct FaceRec {
    T A, n0, n1, n2, rl0, rl1, rl2, rr0, rr1, rr2, vcL, vcR;
};
template <typename T>
__device__ inline FaceRec<T> load_face(const T* __restrict__ face, int64_t f) {
    T v[12];
    const T* p = face + f * kFaceRec;
    load4(p, v);
    load4(p + 4, v + 4);
    load4(p + 8, v + 8);
    return FaceRec<T>{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9], v[10], v[11]};
}

// Where the limited face states of a cell's sides are read from: the
// face-state array FV[b][e][4] of the split path, or the LDS tile of the
// fused kernel.
template <typename T>
struct GlobalFaceStates {
    const T* FVb;          // FV of bin b
    const int32_t* opp;
    __device__ const T* own(int64_t e) const { return FVb + e * 4; }
    __device__ const T* other(int64_t e) const { return FVb + (int64_t)opp[e] * 4; }
};
template <typename T>
struct TileFaceStates {
    const T* lds;
    int64_t e0;            // first entry of the tile
    const int32_t* lds_opp;
    __device__ const T* own(int64_t e) const { return lds + (e - e0) * 4; }
    __device__ const T* other(int64_t e) const { return lds + (int64_t)lds_opp[e] * 4; }
};

// Flux sum of cell i (bin b) from the limited face states: each face's
// flux in its canonical (L, R) orientation with the upwind cap, accumulated
// as sigma A Phi in face-index order in FP64.  TA is the arithmetic
// precision of the face physics.
template <typename T, typename TA, typename FS>
__device__ inline void cell_flux_sum(int64_t i, int b, int64_t nc, const T* __restrict__ U, const FS& fsv,
                                     const GeomView<T>& geo, const SellView& sell, TA cdt, TA Ni, double* acc,
                                     int& cAdmN, int& cAdmF, int& cCap) {
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
        const FaceRec<T> fr = load_face(geo.face, f);
        T so[4], sn[4];
        load4(fsv.own(e), so);
        load4(fsv.other(e), sn);
        const TA Nj = (TA)U[urec(b, nc, j)];
        // Canonical orientation: L then R, whichever lane computes it.
        TA sL[4], sR[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            sL[v] = (TA)(isL ? so[v] : sn[v]);
            sR[v] = (TA)(isL ? sn[v] : so[v]);
        }
        const TA NL = isL ? Ni : Nj, NR = isL ? Nj : Ni;
        int aN = 0, aF = 0;
        TA Phi[4];
        const bool capped = face_flux<TA, TA>(sL, sR, NL, NR, (TA)fr.vcL, (TA)fr.vcR, (TA)fr.n0, (TA)fr.n1,
                                             (TA)fr.n2, (TA)fr.A, cdt, Phi, aN, aF);
        if (isL) {
            cAdmN += aN; cAdmF += aF; cCap += capped ? 1 : 0;
        }
        const TA sA = isL ? (TA)fr.A : -(TA)fr.A;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += (double)(sA * Phi[v]);
    }
}

// The limited state of a cell at one of its faces, U_i + g . r_if, rounded
// to the storage precision once.
template <typename T>
__device__ inline void face_state(const double* ui, const double (*g)[3], double r0, double r1, double r2, T* s) {
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] = (T)(ui[v] + (g[v][0] * r0 + g[v][1] * r1 + g[v][2] * r2));
}

// Limited least-squares gradient of the four fields of cell i (bin b) in
// FP64: g = M^-1 sum_j w_ij (phi_j - phi_i), w_ij = A d / |d|^2 with
// d = s_j - s_i through the face, then a Barth-Jespersen factor per variable
// (Sec. 2.3.2).  Returns the cell's fields in ui.
template <typename T>
__device__ inline void limited_gradient(int64_t i, int b, int64_t nc, const T* __restrict__ U, const GeomView<T>& geo,
                                        const SellView& sell, int use_limiter, double* ui, double (*g)[3]) {
    T u0[4];
    load4(U + urec(b, nc, i), u0);
#pragma unroll
    for (int v = 0; v < 4; ++v) ui[v] = (double)u0[v];
    double bs[4][3], umax[4], umin[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        bs[v][0] = bs[v][1] = bs[v][2] = 0.0;
        umax[v] = umin[v] = ui[v];
    }
    const int64_t slice = i / kSlice;
    const int32_t deg = sell.deg[slice];
    const int64_t base = (int64_t)sell.ptr[slice] + (i % kSlice);
    for (int k = 0; k < deg; ++k) {
        const int64_t e = base + (int64_t)k * kSlice;
        const int32_t j = sell.nbr[e];
        if (j < 0) continue;
        const int32_t fs = sell.fsf[e];
        const bool isL = fs >= 0;
        const FaceRec<T> fr = load_face(geo.face, isL ? fs : ~fs);
        // d = r_if - r_jf = s_j - s_i
        const double d0 = isL ? (double)fr.rl0 - (double)fr.rr0 : (double)fr.rr0 - (double)fr.rl0;
        const double d1 = isL ? (double)fr.rl1 - (double)fr.rr1 : (double)fr.rr1 - (double)fr.rl1;
        const double d2 = isL ? (double)fr.rl2 - (double)fr.rr2 : (double)fr.rr2 - (double)fr.rl2;
        const double s = (double)fr.A / (d0 * d0 + d1 * d1 + d2 * d2);
        const double w0 = d0 * s, w1 = d1 * s, w2 = d2 * s;
        T uj[4];
        load4(U + urec(b, nc, j), uj);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double ujv = (double)uj[v];
            const double dphi = ujv - ui[v];
            bs[v][0] += w0 * dphi;
            bs[v][1] += w1 * dphi;
            bs[v][2] += w2 * dphi;
            umax[v] = ujv > umax[v] ? ujv : umax[v];
            umin[v] = ujv < umin[v] ? ujv : umin[v];
        }
    }
    T c[8];
    load4(geo.cell + i * kCellRec, c);
    load4(geo.cell + i * kCellRec + 4, c + 4);
    const double mxx = c[0], myy = c[1], mzz = c[2], mxy = c[3], mxz = c[4], myz = c[5];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        g[v][0] = mxx * bs[v][0] + mxy * bs[v][1] + mxz * bs[v][2];
        g[v][1] = mxy * bs[v][0] + myy * bs[v][1] + myz * bs[v][2];
        g[v][2] = mxz * bs[v][0] + myz * bs[v][1] + mzz * bs[v][2];
    }
    if (!use_limiter) return;
    double alpha[4] = {1.0, 1.0, 1.0, 1.0};
    for (int k = 0; k < deg; ++k) {
        const int64_t e = base + (int64_t)k * kSlice;
        if (sell.nbr[e] < 0) continue;
        const int32_t fs = sell.fsf[e];
        const bool isL = fs >= 0;
        const FaceRec<T> fr = load_face(geo.face, isL ? fs : ~fs);
        const double r0 = isL ? fr.rl0 : fr.rr0, r1 = isL ? fr.rl1 : fr.rr1, r2 = isL ? fr.rl2 : fr.rr2;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double delta = g[v][0] * r0 + g[v][1] * r1 + g[v][2] * r2;
            double psi = 1.0;
            if (delta > 0.0) psi = (umax[v] - ui[v]) / delta;
            else if (delta < 0.0) psi = (umin[v] - ui[v]) / delta;
            alpha[v] = psi < alpha[v] ? psi : alpha[v];
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        g[v][0] *= alpha[v];
        g[v][1] *= alpha[v];
        g[v][2] *= alpha[v];
    }
}

}  // namespace rtk
