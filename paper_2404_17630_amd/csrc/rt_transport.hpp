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
__device__ inline void load2(const float* __restrict__ p, float* o) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    o[0] = v.x; o[1] = v.y;
}
__device__ inline void load2(const double* __restrict__ p, double* o) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    o[0] = v.x; o[1] = v.y;
}
__device__ inline void store4(float* __restrict__ p, const float* v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ inline void store4(double* __restrict__ p, const double* v) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
}
// Store that bypasses the caches' retention (a record no kernel reads again
// soon enough to find it there); the FP64 form is a plain store.
__device__ inline void store4_stream(float* __restrict__ p, const float* v) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f x = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(x, reinterpret_cast<v4f*>(p));
}
__device__ inline void store4_stream(double* __restrict__ p, const double* v) { store4(p, v); }

// a * b rounded on its own: never contracted with the sum it feeds, so a
// face's contribution to a flux sum is the same value in every kernel that
// forms it (the slot-parallel flux kernel passes it through LDS).
template <typename R>
__device__ inline R mul_nc(R a, R b) {
#pragma clang fp contract(off)
    return a * b;
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
// Both also give the numerator N V / n_faces of the outflow cap of a cell:
// the split path reads it as the product k_facestate stored (4 bytes a
// cell, kCapProduct), the fused path forms it from the cell's N and the
// side record's V / n_faces.  Either way it is the same product of the same
// two stored values, rounded once.
template <typename T>
struct GlobalFaceStates {
    static constexpr bool kCapProduct = true;
    const T* FVb;          // FV of bin b
    const int32_t* opp;
    const T* NVb;          // N V / n_faces of every cell of bin b, written by k_facestate
    __device__ const T* own(int64_t e) const { return FVb + e * 4; }
    __device__ const T* other(int64_t e) const { return FVb + (int64_t)opp[e] * 4; }
    // with the entry's opposite entry already loaded
    __device__ const T* other(int64_t e, int32_t eo) const { return FVb + (int64_t)eo * 4; }
    __device__ T cellN(int32_t j) const { return NVb[j]; }
};
template <typename T>
struct TileFaceStates {
    static constexpr bool kCapProduct = false;
    const T* lds;
    int64_t e0;            // first entry of the tile
    const int32_t* lds_opp;
    const T* Ub;           // fields of bin b
    __device__ const T* own(int64_t e) const { return lds + (e - e0) * 4; }
    __device__ const T* other(int64_t e) const { return lds + (int64_t)lds_opp[e] * 4; }
    __device__ const T* other(int64_t e, int32_t) const { return lds + (int64_t)lds_opp[e] * 4; }
    __device__ T cellN(int32_t j) const { return Ub[(int64_t)j * 4]; }
};

// The limited state of a cell at one of its faces, U_i + g . r_if, rounded
// to the storage precision once.
template <typename T>
__device__ inline void face_state(const double* ui, const double (*g)[3], double r0, double r1, double r2, T* s) {
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] = (T)(ui[v] + (g[v][0] * r0 + g[v][1] * r1 + g[v][2] * r2));
}

// Barth-Jespersen factor alpha = min(1, min_k psi_k) of one variable, with
// psi_k = (u_max - u_i) / delta_k for delta_k = g . r_k > 0 and
// (u_min - u_i) / delta_k for delta_k < 0 (Sec. 2.3.2).  All psi_k of one
// sign of delta_k share their numerator (u_max - u_i >= 0, or u_i - u_min),
// so the smallest is the one of the largest |delta_k|: only the largest
// positive and the largest negative extrapolation are kept (add), and
// alpha is the smaller of their two fractions and 1, chosen without
// dividing (n1 d2 < n2 d1), with one division at the end.
struct BJFactor {
    double dpos = 0.0, dneg = 0.0;     // max over delta_k > 0 of delta_k, of -delta_k over delta_k < 0
    __device__ void add(double delta) {
        dpos = fmax(dpos, delta);
        dneg = fmax(dneg, -delta);
    }
    __device__ double alpha(double up, double down) const {   // up = u_max - u_i, down = u_i - u_min
        double num = 1.0, den = 1.0;
        if (dpos > 0.0 && up * den < num * dpos) { num = up; den = dpos; }
        if (dneg > 0.0 && down * den < num * dneg) { num = down; den = dneg; }
        return num / den;
    }
};

// ---------------------------------------------------------------------------
// The same two steps from the per-side records.  DEG > 0: every slice of the
// mesh has exactly DEG slots, the slot loops are unrolled and the face
// offsets stay in registers; DEG == 0: any degree.
// ---------------------------------------------------------------------------

template <int DEG>
struct SlotCount {
    static constexpr int kMax = DEG > 0 ? DEG : 1;
};
// Slots whose gathers are issued together: all of them up to 8, else half
// (the records of 14 slots at once would cost too many registers).
template <int DEG>
struct SlotBatch {
    static constexpr int kSize = DEG <= 8 ? DEG : (DEG + 1) / 2;
};
// The flux sum takes three slots at a time, loading their face records with
// their gathers: the records of all slots held at once cost more in
// occupancy than the extra overlap gains.
template <int DEG>
struct FluxBatch {
    static constexpr int kSize = DEG < 3 ? DEG : 3;
};

// Side records of one cell's DEG slots (DEG > 0) for the gradient: the
// neighbours, the least-squares weights and the face offsets.
template <typename T, int DEG>
struct CellSides {
    int32_t nbr[DEG];
    T w[DEG][3], r[DEG][3];
};
template <typename T, int DEG>
__device__ inline void load_cell_sides(int64_t i, const GeomView<T>& geo, const SellView& sell, CellSides<T, DEG>& cs) {
    const int64_t base = (int64_t)sell.ptr[i / kSlice] + (i % kSlice);
#pragma unroll
    for (int k = 0; k < DEG; ++k) {
        const int64_t e = base + (int64_t)k * kSlice;
        cs.nbr[k] = sell.nbr[e];
        T g0[4], g1[2];
        load4(geo.sg(0, e), g0);
        load2(geo.sg(1, e), g1);
        cs.w[k][0] = g0[0]; cs.w[k][1] = g0[1]; cs.w[k][2] = g0[2];
        cs.r[k][0] = g0[3]; cs.r[k][1] = g1[0]; cs.r[k][2] = g1[1];
    }
}
// Index records of one cell's DEG slots for the flux sum (neighbour,
// opposite entry, orientation), loaded once and reused for every bin; the
// face records (groups 2 and 3 of the side records) are read with each
// batch of slots.
template <typename T, int DEG>
struct CellFaces {
    int32_t nbr[DEG], opp[DEG];
    bool isL[DEG];
    const T* side2;        // (V_L/n, V_R/n) of every entry
    const T* side3;        // (A, n) of every entry
};
template <typename T, int DEG>
__device__ inline void load_cell_faces(int64_t i, const GeomView<T>& geo, const SellView& sell, CellFaces<T, DEG>& cf) {
    const int64_t base = (int64_t)sell.ptr[i / kSlice] + (i % kSlice);
#pragma unroll
    for (int k = 0; k < DEG; ++k) {
        const int64_t e = base + (int64_t)k * kSlice;
        const int2 id = sell.nop[e];
        cf.nbr[k] = id.x;
        cf.isL[k] = id.y >= 0;
        cf.opp[k] = id.y >= 0 ? id.y : ~id.y;
    }
    cf.side2 = geo.sg(2, 0);
    cf.side3 = geo.sg(3, 0);
}

// Limited gradient of cell i (bin b) from its loaded side records (DEG > 0).
template <typename T, int DEG>
__device__ inline void limited_gradient_c(int64_t i, int b, int64_t nc, const T* __restrict__ U, const T* cell,
                                          const CellSides<T, DEG>& cs, int use_limiter, double* ui, double (*g)[3]) {
    T u0[4];
    load4(U + urec(b, nc, i), u0);
#pragma unroll
    for (int v = 0; v < 4; ++v) ui[v] = (double)u0[v];
    // neighbour extrema in the storage precision (exact: they are stored values)
    double bs[4][3];
    T umax[4], umin[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        bs[v][0] = bs[v][1] = bs[v][2] = 0.0;
        umax[v] = umin[v] = u0[v];
    }
    // The neighbour records of a batch of slots are all requested before
    // any is used, so the gathers overlap instead of each waiting for the
    // previous one (a padding slot reads the cell's own record and is
    // skipped below).
    constexpr int P = SlotBatch<DEG>::kSize;
#pragma unroll
    for (int k0 = 0; k0 < DEG; k0 += P) {
        T uj[P][4];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int k = k0 + q;
            if (k < DEG) load4(U + urec(b, nc, cs.nbr[k] >= 0 ? (int64_t)cs.nbr[k] : i), uj[q]);
        }
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int k = k0 + q;
            if (k >= DEG || cs.nbr[k] < 0) continue;
            const double w0 = (double)cs.w[k][0], w1 = (double)cs.w[k][1], w2 = (double)cs.w[k][2];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double ujv = (double)uj[q][v];
                const double dphi = ujv - ui[v];
                bs[v][0] += w0 * dphi;
                bs[v][1] += w1 * dphi;
                bs[v][2] += w2 * dphi;
                // (compare and select: a NaN neighbour leaves the extrema
                // as fmax/fmin would, without their operand quieting)
                umax[v] = uj[q][v] > umax[v] ? uj[q][v] : umax[v];
                umin[v] = uj[q][v] < umin[v] ? uj[q][v] : umin[v];
            }
        }
    }
    const double mxx = cell[0], myy = cell[1], mzz = cell[2], mxy = cell[3], mxz = cell[4], myz = cell[5];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        g[v][0] = mxx * bs[v][0] + mxy * bs[v][1] + mxz * bs[v][2];
        g[v][1] = mxy * bs[v][0] + myy * bs[v][1] + myz * bs[v][2];
        g[v][2] = mxz * bs[v][0] + myz * bs[v][1] + mzz * bs[v][2];
    }
    if (!use_limiter) return;
    BJFactor bj[4];
#pragma unroll
    for (int k = 0; k < DEG; ++k) {
        if (cs.nbr[k] < 0) continue;
        const double r0 = cs.r[k][0], r1 = cs.r[k][1], r2 = cs.r[k][2];
#pragma unroll
        for (int v = 0; v < 4; ++v) bj[v].add(g[v][0] * r0 + g[v][1] * r1 + g[v][2] * r2);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double alpha = bj[v].alpha((double)umax[v] - ui[v], ui[v] - (double)umin[v]);
        g[v][0] *= alpha;
        g[v][1] *= alpha;
        g[v][2] *= alpha;
    }
}

// Flux sum of cell i (bin b) from its loaded face records (DEG > 0).  With
// `prod` the products sigma A Phi of the slots are stored there instead of
// added (a padding slot's are left unset), so that the fused kernel can add
// a cell's tile-interior faces before its cross-tile ones, in the order of
// the split path.
template <typename T, typename TA, int DEG, typename FS>
__device__ inline void cell_flux_sum_c(int64_t i, int b, int64_t nc, const T* __restrict__ U, const FS& fsv,
                                       int64_t base, const CellFaces<T, DEG>& cf, TA cdt, TA Ni, double* acc,
                                       int& cAdmN, int& cAdmF, int& cCap, TA (*prod)[4] = nullptr) {
    // The face records, the two face states and the neighbour's N of a
    // batch of slots are all requested before the batch's first flux is
    // computed, so the gathers overlap (a padding slot reads its own entry
    // and the cell itself, and is skipped below).
    constexpr int P = FluxBatch<DEG>::kSize;
#pragma unroll
    for (int k0 = 0; k0 < DEG; k0 += P) {
        T so[P][4], sn[P][4], nj[P], gv[P][2], ga[P][4];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int k = k0 + q;
            if (k >= DEG) break;
            const int64_t e = base + (int64_t)k * kSlice;
            load2(cf.side2 + e * 2, gv[q]);
            load4(cf.side3 + e * 4, ga[q]);
            const bool pad = cf.nbr[k] < 0;
            load4(fsv.own(e), so[q]);
            load4(pad ? fsv.own(e) : fsv.other(e, cf.opp[k]), sn[q]);
            nj[q] = fsv.cellN(pad ? (int32_t)i : cf.nbr[k]);
        }
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int k = k0 + q;
            if (k >= DEG) break;
            const int32_t j = cf.nbr[k];
            if (j < 0) continue;
            const bool isL = cf.isL[k];
            const TA A = (TA)ga[q][0];
            const TA Nj = (TA)nj[q];
            TA sL[4], sR[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                sL[v] = (TA)(isL ? so[q][v] : sn[q][v]);
                sR[v] = (TA)(isL ? sn[q][v] : so[q][v]);
            }
            const TA NL = isL ? Ni : Nj, NR = isL ? Nj : Ni;
            int aN = 0, aF = 0;
            TA Phi[4];
            const TA vcL = FS::kCapProduct ? (TA)1 : (TA)gv[q][0], vcR = FS::kCapProduct ? (TA)1 : (TA)gv[q][1];
            const bool capped = face_flux<TA, TA>(sL, sR, NL, NR, vcL, vcR, (TA)ga[q][1], (TA)ga[q][2], (TA)ga[q][3],
                                                 A, cdt, Phi, aN, aF);
            if (isL) {
                cAdmN += aN; cAdmF += aF; cCap += capped ? 1 : 0;
            }
            const TA sA = isL ? A : -A;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const TA p = mul_nc(sA, Phi[v]);
                if (prod) prod[k][v] = p;
                else acc[v] += (double)p;
            }
        }
    }
}

// Limited gradient of the four fields of cell i (bin b) in FP64; ui the
// cell's fields; for DEG > 0 the offsets r_if of its slots in rr and their
// validity in ok.
template <typename T, int DEG>
__device__ inline void limited_gradient_s(int64_t i, int b, int64_t nc, const T* __restrict__ U, const GeomView<T>& geo,
                                          const SellView& sell, int use_limiter, double* ui, double (*g)[3],
                                          T (*rr)[3], bool* ok) {
    T u0[4];
    load4(U + urec(b, nc, i), u0);
#pragma unroll
    for (int v = 0; v < 4; ++v) ui[v] = (double)u0[v];
    // neighbour extrema in the storage precision (exact: they are stored values)
    double bs[4][3];
    T umax[4], umin[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        bs[v][0] = bs[v][1] = bs[v][2] = 0.0;
        umax[v] = umin[v] = u0[v];
    }
    const int64_t slice = i / kSlice;
    const int32_t deg = DEG > 0 ? DEG : sell.deg[slice];
    const int64_t base = (int64_t)sell.ptr[slice] + (i % kSlice);
#pragma unroll(SlotCount<DEG>::kMax)
    for (int k = 0; k < (DEG > 0 ? DEG : deg); ++k) {
        const int64_t e = base + (int64_t)k * kSlice;
        const int32_t j = sell.nbr[e];
        if (DEG > 0) {
            rr[k][0] = geo.sv(kSR0, e); rr[k][1] = geo.sv(kSR1, e); rr[k][2] = geo.sv(kSR2, e);
            ok[k] = j >= 0;
        }
        if (j < 0) continue;
        const double w0 = (double)geo.sv(kSW0, e), w1 = (double)geo.sv(kSW1, e), w2 = (double)geo.sv(kSW2, e);
        T uj[4];
        load4(U + urec(b, nc, j), uj);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double ujv = (double)uj[v];
            const double dphi = ujv - ui[v];
            bs[v][0] += w0 * dphi;
            bs[v][1] += w1 * dphi;
            bs[v][2] += w2 * dphi;
            umax[v] = uj[v] > umax[v] ? uj[v] : umax[v];
            umin[v] = uj[v] < umin[v] ? uj[v] : umin[v];
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
    BJFactor bj[4];
#pragma unroll(SlotCount<DEG>::kMax)
    for (int k = 0; k < (DEG > 0 ? DEG : deg); ++k) {
        double r0, r1, r2;
        if (DEG > 0) {
            if (!ok[k]) continue;
            r0 = rr[k][0]; r1 = rr[k][1]; r2 = rr[k][2];
        } else {
            const int64_t e = base + (int64_t)k * kSlice;
            if (sell.nbr[e] < 0) continue;
            r0 = geo.sv(kSR0, e); r1 = geo.sv(kSR1, e); r2 = geo.sv(kSR2, e);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) bj[v].add(g[v][0] * r0 + g[v][1] * r1 + g[v][2] * r2);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double alpha = bj[v].alpha((double)umax[v] - ui[v], ui[v] - (double)umin[v]);
        g[v][0] *= alpha;
        g[v][1] *= alpha;
        g[v][2] *= alpha;
    }
}

// Flux sum of cell i (bin b) from the face states and the per-side records.
template <typename T, typename TA, int DEG, typename FS>
__device__ inline void cell_flux_sum_s(int64_t i, int b, int64_t nc, const T* __restrict__ U, const FS& fsv,
                                       const GeomView<T>& geo, const SellView& sell, TA cdt, TA Ni, double* acc,
                                       int& cAdmN, int& cAdmF, int& cCap) {
    const int64_t slice = i / kSlice;
    const int32_t deg = DEG > 0 ? DEG : sell.deg[slice];
    const int64_t base = (int64_t)sell.ptr[slice] + (i % kSlice);
#pragma unroll(SlotCount<DEG>::kMax)
    for (int k = 0; k < (DEG > 0 ? DEG : deg); ++k) {
        const int64_t e = base + (int64_t)k * kSlice;
        const int32_t j = sell.nbr[e];
        if (j < 0) continue;
        const bool isL = sell.fsf[e] >= 0;
        const TA A = (TA)geo.sv(kSA, e);
        const TA n0 = (TA)geo.sv(kSN0, e), n1 = (TA)geo.sv(kSN1, e), n2 = (TA)geo.sv(kSN2, e);
        const TA vcL = FS::kCapProduct ? (TA)1 : (TA)geo.sv(kSVL, e);
        const TA vcR = FS::kCapProduct ? (TA)1 : (TA)geo.sv(kSVR, e);
        T so[4], sn[4];
        load4(fsv.own(e), so);
        load4(fsv.other(e), sn);
        const TA Nj = (TA)fsv.cellN(j);
        TA sL[4], sR[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            sL[v] = (TA)(isL ? so[v] : sn[v]);
            sR[v] = (TA)(isL ? sn[v] : so[v]);
        }
        const TA NL = isL ? Ni : Nj, NR = isL ? Nj : Ni;
        int aN = 0, aF = 0;
        TA Phi[4];
        const bool capped = face_flux<TA, TA>(sL, sR, NL, NR, vcL, vcR, n0, n1, n2, A, cdt, Phi, aN, aF);
        if (isL) {
            cAdmN += aN; cAdmF += aF; cCap += capped ? 1 : 0;
        }
        const TA sA = isL ? A : -A;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += (double)mul_nc(sA, Phi[v]);
    }
}

}  // namespace rtk
