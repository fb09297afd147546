// Reverse-mode derivative of the radiative-transfer subcycle (FP64).
//
// Given dL/dx_HI of the state after n subcycles, returns dL/d ln Q_k for
// every source (all bins of a source scaled together) and dL/d ln n_H,i of
// the initial density.  The forward pass is the same sequence of kernels as
// rt_subcycle; states are checkpointed every C subcycles and each segment is
// recomputed forward, keeping the pre-chemistry and post-chemistry states of
// its subcycles.  The reverse sweep of one subcycle is, in reverse order of
// the forward steps:
//
//   k_adj_guard   post-update guards (N >= 0, |Fh| <= N)        per (cell, bin)
//   k_adj_flux    face fluxes -> face states -> (U, g)           per (cell, bin)
//   k_adj_grad    gradients + slope limiter -> U                 per (cell, bin)
//   k_adj_gather  sums each cell's share of its neighbours' terms per (cell, bin)
//   k_adj_chem    thermochemistry                                 per cell
//   k_adj_src     point sources -> dL/d ln Q                      per source
//
// Every kernel is a gather: a cell's adjoint is summed from quantities the
// kernel before it stored per cell or per face side, so there are no atomics
// and the result is deterministic.  Local Jacobians (one face's flux, one
// cell's limited gradient, one cell's chemistry over the subcycle, the
// guards) are evaluated by running the forward device code on dual numbers
// with one seeded direction per input; branches are decided on the value
// part, so this is the exact derivative of the branch path the forward pass
// takes (the controller's accept/reject decisions, limiter and cap choices).
// The chemistry replay needs no substep tape: a cell's subcycle map has only
// 7 + nb scalar inputs (five fractions, u, N_b, n_H), and the flux enters
// only through the product of the substep absorption factors.

#include <hip/hip_runtime.h>

#include <cmath>

#include <algorithm>
#include <cstring>
#include <vector>

#include "rt.h"
#include "rt_chem.hpp"
#include "rt_dual.hpp"
#include "rt_face.hpp"
#include "rt_internal.hpp"
#include "rt_transport.hpp"
#include "rt_types.hpp"

namespace rtk {

constexpr int kFaceDirs = 10;   // sL[4], sR[4], N_L, N_R

// Input states of the transport step whose photon density is below
// kAdjFloor times the bin's largest (the leading edge of a front, where
// neighbours differ by tens of orders of magnitude) are held constant: the
// adjoint of the cell's input state and of its gradient is zero (the adjoint
// of its output, which the flux from lit neighbours fills, is kept).  A
// perturbation of the luminosities or densities moves such a state by a
// relative amount of the order of its own, which cannot reach x_HI in FP64;
// the ratio-type local derivatives there (limiter, closure) would otherwise
// multiply the adjoint by up to 1e12 per subcycle and overflow it.  Cells
// with N = 0 are beyond the stencil's reach, so their adjoint is exactly
// zero anyway.
constexpr double kAdjFloor = 1.0e-20;

// Largest N of each bin over the cells: per-block maxima, then one block per
// bin; writes tau[b] = kAdjFloor * max.
__global__ __launch_bounds__(kBlock) void k_adj_binmax(const double* __restrict__ U, int64_t nc, int nb,
                                                       double* __restrict__ part) {
    __shared__ double red[kBlock];
    const int b = (int)(blockIdx.x % nb);
    const int64_t blk = blockIdx.x / nb;
    const int64_t i = blk * kBlock + threadIdx.x;
    red[threadIdx.x] = i < nc ? U[urec(b, nc, i)] : 0.0;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(kBlock) void k_adj_tau(const double* __restrict__ part, int64_t n_blk, int nb,
                                                    double* __restrict__ tau) {
    __shared__ double red[kBlock];
    const int b = blockIdx.x;
    double m = 0.0;
    for (int64_t q = threadIdx.x; q < n_blk; q += kBlock) m = fmax(m, part[q * nb + b]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) tau[b] = kAdjFloor * red[0];
}

__device__ inline bool adj_active(const double* __restrict__ U, const double* __restrict__ tau, int b, int64_t nc,
                                  int64_t i) {
    const double n = U[urec(b, nc, i)];
    return n > 0.0 && n >= tau[b];
}

// ---------------------------------------------------------------------------
// k_adj_guard: lambda_pre = J_guard^T lambda_new, with the pre-guard update
// recomputed from the transport inputs.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_adj_guard(const double* __restrict__ U, const double* __restrict__ FV,
                                                      const double* __restrict__ lam_new, double* __restrict__ lam_pre,
                                                      int64_t nc, int nb, int64_t n_entries, GeomView<double> geo,
                                                      SellView sell, double cdt) {
    const int64_t blk = xcd_logical_block();
    const int b = (int)(blk % nb);
    const int64_t i = (blk / nb) * kBlock + threadIdx.x;
    if (i >= nc) return;
    double ui[4];
    load4(U + urec(b, nc, i), ui);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int c0 = 0, c1 = 0, c2 = 0;
    // the cells' cap numerators N V / n_faces follow the face states in FV
    const GlobalFaceStates<double> fsv{FV + (int64_t)b * n_entries * 4, sell.opp,
                                       FV + (int64_t)nb * n_entries * 4 + (int64_t)b * nc};
    cell_flux_sum_s<double, double, 0>(i, b, nc, U, fsv, geo, sell, cdt, fsv.cellN((int32_t)i), acc, c0, c1, c2);
    const double coef = cdt / geo.cell[i * kCellRec + 6];
    Dual<4> un[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        un[v] = Dual<4>(ui[v] - coef * acc[v]);
        un[v].d[v] = 1.0;
    }
    int g0 = 0, g1 = 0;
    update_guards<Dual<4>>(un, g0, g1);
    const double* ln = lam_new + (int64_t)(b * 4) * nc;
    double lnew[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) lnew[w] = ln[(int64_t)w * nc + i];
    double* lp = lam_pre + (int64_t)(b * 4) * nc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) s += lnew[w] * un[w].d[v];
        lp[(int64_t)v * nc + i] = s;
    }
}

// ---------------------------------------------------------------------------
// k_adj_flux: for each face of the cell, mu = dL/dPhi from both cells'
// lambda_pre (U_new_L = U_L - coef_L A Phi, U_new_R = U_R + coef_R A Phi),
// then the face function's Jacobian on duals; the cell's share gives
// lambda_direct (including the identity term lambda_pre) and lambda_g.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_adj_flux(const double* __restrict__ U, const double* __restrict__ G,
                                                     const double* __restrict__ lam_pre, double* __restrict__ lam_dir,
                                                     double* __restrict__ lam_g, int64_t nc, int nb,
                                                     GeomView<double> geo, SellView sell, double cdt,
                                                     const double* __restrict__ tau) {
    const int64_t blk = xcd_logical_block();
    const int b = (int)(blk % nb);
    const int64_t i = (blk / nb) * kBlock + threadIdx.x;
    if (i >= nc) return;
    if (!adj_active(U, tau, b, nc, i)) {
        double* Ld = lam_dir + (int64_t)(b * 4) * nc;
        double* Lg = lam_g + (int64_t)(b * 12) * nc;
        for (int v = 0; v < 4; ++v) Ld[(int64_t)v * nc + i] = 0.0;
        for (int v = 0; v < 12; ++v) Lg[(int64_t)v * nc + i] = 0.0;
        return;
    }
    const double* Gb = G + (int64_t)(b * 12) * nc;
    const double* Lp = lam_pre + (int64_t)(b * 4) * nc;
    double ui[4], gi[4][3], li[4];
    load4(U + urec(b, nc, i), ui);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        li[v] = Lp[(int64_t)v * nc + i];
#pragma unroll
        for (int c = 0; c < 3; ++c) gi[v][c] = Gb[(int64_t)(v * 3 + c) * nc + i];
    }
    const double coef_i = cdt / geo.cell[i * kCellRec + 6];
    double ld[4] = {li[0], li[1], li[2], li[3]};
    double lg[4][3];
#pragma unroll
    for (int v = 0; v < 4; ++v) lg[v][0] = lg[v][1] = lg[v][2] = 0.0;

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
        const FaceRec<double> fr = load_face(geo.face, f);
        const double A = fr.A;
        const double n0 = fr.n0, n1 = fr.n1, n2 = fr.n2;
        const double rl[3] = {fr.rl0, fr.rl1, fr.rl2}, rr[3] = {fr.rr0, fr.rr1, fr.rr2};
        double uj[4], gj[4][3], lj[4];
        load4(U + urec(b, nc, j), uj);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            lj[v] = Lp[(int64_t)v * nc + j];
#pragma unroll
            for (int c = 0; c < 3; ++c) gj[v][c] = Gb[(int64_t)(v * 3 + c) * nc + j];
        }
        const double coef_j = cdt / geo.cell[(int64_t)j * kCellRec + 6];
        const double coefL = isL ? coef_i : coef_j, coefR = isL ? coef_j : coef_i;
        Dual<kFaceDirs> sL[4], sR[4];
        double mu[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double UL = isL ? ui[v] : uj[v];
            const double UR = isL ? uj[v] : ui[v];
            const double gl0 = isL ? gi[v][0] : gj[v][0], gl1 = isL ? gi[v][1] : gj[v][1], gl2 = isL ? gi[v][2] : gj[v][2];
            const double gr0 = isL ? gj[v][0] : gi[v][0], gr1 = isL ? gj[v][1] : gi[v][1], gr2 = isL ? gj[v][2] : gi[v][2];
            sL[v] = Dual<kFaceDirs>(UL + (gl0 * rl[0] + gl1 * rl[1] + gl2 * rl[2]));
            sR[v] = Dual<kFaceDirs>(UR + (gr0 * rr[0] + gr1 * rr[1] + gr2 * rr[2]));
            sL[v].d[v] = 1.0;
            sR[v].d[4 + v] = 1.0;
            const double lL = isL ? li[v] : lj[v], lR = isL ? lj[v] : li[v];
            mu[v] = A * (coefR * lR - coefL * lL);
        }
        Dual<kFaceDirs> NL(isL ? ui[0] : uj[0]), NR(isL ? uj[0] : ui[0]);
        NL.d[8] = 1.0;
        NR.d[9] = 1.0;
        int aN = 0, aF = 0;
        Dual<kFaceDirs> Phi[4];
        face_flux<Dual<kFaceDirs>, double>(sL, sR, NL, NR, fr.vcL, fr.vcR, n0, n1, n2, A, cdt, Phi, aN, aF);
        const int off = isL ? 0 : 4;
        const double* r = isL ? rl : rr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double ls = 0.0;
#pragma unroll
            for (int w = 0; w < 4; ++w) ls += mu[w] * Phi[w].d[off + v];
            ld[v] += ls;
            lg[v][0] += ls * r[0];
            lg[v][1] += ls * r[1];
            lg[v][2] += ls * r[2];
        }
        double lN = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) lN += mu[w] * Phi[w].d[isL ? 8 : 9];
        ld[0] += lN;
    }
    double* Ld = lam_dir + (int64_t)(b * 4) * nc;
    double* Lg = lam_g + (int64_t)(b * 12) * nc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        Ld[(int64_t)v * nc + i] = ld[v];
#pragma unroll
        for (int c = 0; c < 3; ++c) Lg[(int64_t)(v * 3 + c) * nc + i] = lg[v][c];
    }
}

// ---------------------------------------------------------------------------
// k_adj_grad: the cell's limited gradient of each variable as a function of
// phi_i (direction 0) and its neighbours (direction 1 + slot), contracted
// with lambda_g.  The cell's own coefficient goes to c_self, the neighbour
// coefficients to c_slot in the cell's sliced-ELL slots.
// ---------------------------------------------------------------------------
template <int KG>
__global__ __launch_bounds__(kBlock) void k_adj_grad(const double* __restrict__ U, const double* __restrict__ lam_g,
                                                     double* __restrict__ c_self, double* __restrict__ c_slot,
                                                     int64_t n_entries, int64_t nc, int nb, GeomView<double> geo,
                                                     SellView sell, int use_limiter, const double* __restrict__ tau) {
    const int64_t blk = xcd_logical_block();
    const int b = (int)(blk % nb);
    const int64_t i = (blk / nb) * kBlock + threadIdx.x;
    if (i >= nc) return;
    const double* Lg = lam_g + (int64_t)(b * 12) * nc;
    const int64_t slice = i / kSlice;
    const int32_t deg = sell.deg[slice];
    const int64_t base = (int64_t)sell.ptr[slice] + (i % kSlice);
    if (!adj_active(U, tau, b, nc, i)) {
        for (int v = 0; v < 4; ++v) {
            c_self[(int64_t)(b * 4 + v) * nc + i] = 0.0;
            for (int k = 0; k < deg; ++k)
                c_slot[(int64_t)(b * 4 + v) * n_entries + base + (int64_t)k * kSlice] = 0.0;
        }
        return;
    }
    const double* cr = geo.cell + i * kCellRec;
    const double mxx = cr[0], myy = cr[1], mzz = cr[2], mxy = cr[3], mxz = cr[4], myz = cr[5];
    for (int v = 0; v < 4; ++v) {
        Dual<KG> phi_i(U[urec(b, nc, i) + v]);
        phi_i.d[0] = 1.0;
        Dual<KG> bs[3], umax = phi_i, umin = phi_i;
        // (slot loops unrolled to KG - 1 so that a slot's direction index is a
        // constant and the duals stay in registers)
#pragma unroll
        for (int k = 0; k < KG - 1; ++k) {
            if (k >= deg) break;
            const int64_t e = base + (int64_t)k * kSlice;
            const int32_t j = sell.nbr[e];
            if (j < 0) continue;
            const int32_t fs = sell.fsf[e];
            const bool isL = fs >= 0;
            const FaceRec<double> fr = load_face(geo.face, isL ? fs : ~fs);
            const double d0 = isL ? fr.rl0 - fr.rr0 : fr.rr0 - fr.rl0;
            const double d1 = isL ? fr.rl1 - fr.rr1 : fr.rr1 - fr.rl1;
            const double d2 = isL ? fr.rl2 - fr.rr2 : fr.rr2 - fr.rl2;
            const double s = fr.A / (d0 * d0 + d1 * d1 + d2 * d2);
            Dual<KG> uj(U[urec(b, nc, j) + v]);
            uj.d[1 + k] = 1.0;
            const Dual<KG> dphi = uj - phi_i;
            bs[0] += (d0 * s) * dphi;
            bs[1] += (d1 * s) * dphi;
            bs[2] += (d2 * s) * dphi;
            if (val(uj) > val(umax)) umax = uj;
            if (val(uj) < val(umin)) umin = uj;
        }
        Dual<KG> g[3];
        g[0] = mxx * bs[0] + mxy * bs[1] + mxz * bs[2];
        g[1] = mxy * bs[0] + myy * bs[1] + myz * bs[2];
        g[2] = mxz * bs[0] + myz * bs[1] + mzz * bs[2];
        if (use_limiter) {
            Dual<KG> alpha(1.0);
#pragma unroll
            for (int k = 0; k < KG - 1; ++k) {
                if (k >= deg) break;
                const int64_t e = base + (int64_t)k * kSlice;
                if (sell.nbr[e] < 0) continue;
                const int32_t fs = sell.fsf[e];
                const bool isL = fs >= 0;
                const FaceRec<double> fr = load_face(geo.face, isL ? fs : ~fs);
                const double r0 = isL ? fr.rl0 : fr.rr0, r1 = isL ? fr.rl1 : fr.rr1, r2 = isL ? fr.rl2 : fr.rr2;
                const Dual<KG> delta = g[0] * r0 + g[1] * r1 + g[2] * r2;
                Dual<KG> psi(1.0);
                if (val(delta) > 0.0) psi = (umax - phi_i) / delta;
                else if (val(delta) < 0.0) psi = (umin - phi_i) / delta;
                if (val(psi) < val(alpha)) alpha = psi;
            }
            g[0] = alpha * g[0];
            g[1] = alpha * g[1];
            g[2] = alpha * g[2];
        }
        const double l0 = Lg[(int64_t)(v * 3 + 0) * nc + i];
        const double l1 = Lg[(int64_t)(v * 3 + 1) * nc + i];
        const double l2 = Lg[(int64_t)(v * 3 + 2) * nc + i];
        c_self[(int64_t)(b * 4 + v) * nc + i] = l0 * g[0].d[0] + l1 * g[1].d[0] + l2 * g[2].d[0];
#pragma unroll
        for (int k = 0; k < KG - 1; ++k) {
            if (k >= deg) break;
            const int64_t e = base + (int64_t)k * kSlice;
            c_slot[(int64_t)(b * 4 + v) * n_entries + e] =
                l0 * g[0].d[1 + k] + l1 * g[1].d[1 + k] + l2 * g[2].d[1 + k];
        }
    }
}

// ---------------------------------------------------------------------------
// k_adj_gather: lambda_U = lambda_direct + c_self + sum over the faces of the
// cell of the neighbour's coefficient for this cell (found by face index in
// the neighbour's slots).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_adj_gather(const double* __restrict__ lam_dir,
                                                       const double* __restrict__ c_self,
                                                       const double* __restrict__ c_slot, int64_t n_entries,
                                                       double* __restrict__ lam_U, int64_t nc, int nb, SellView sell,
                                                       const double* __restrict__ U, const double* __restrict__ tau) {
    const int64_t blk = xcd_logical_block();
    const int b = (int)(blk % nb);
    const int64_t i = (blk / nb) * kBlock + threadIdx.x;
    if (i >= nc) return;
    if (!adj_active(U, tau, b, nc, i)) {
#pragma unroll
        for (int v = 0; v < 4; ++v) lam_U[(int64_t)(b * 4 + v) * nc + i] = 0.0;
        return;
    }
    double acc[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
        acc[v] = lam_dir[(int64_t)(b * 4 + v) * nc + i] + c_self[(int64_t)(b * 4 + v) * nc + i];
    const int64_t slice = i / kSlice;
    const int32_t deg = sell.deg[slice];
    const int64_t base = (int64_t)sell.ptr[slice] + (i % kSlice);
    for (int k = 0; k < deg; ++k) {
        const int64_t e = base + (int64_t)k * kSlice;
        const int32_t j = sell.nbr[e];
        if (j < 0) continue;
        const int32_t fs = sell.fsf[e];
        const int32_t f = fs >= 0 ? fs : ~fs;
        const int64_t sj = j / kSlice;
        const int32_t dj = sell.deg[sj];
        const int64_t bj = (int64_t)sell.ptr[sj] + (j % kSlice);
        for (int q = 0; q < dj; ++q) {
            const int64_t ej = bj + (int64_t)q * kSlice;
            const int32_t fq = sell.fsf[ej];
            if (sell.nbr[ej] >= 0 && (fq >= 0 ? fq : ~fq) == f) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] += c_slot[(int64_t)(b * 4 + v) * n_entries + ej];
                break;
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) lam_U[(int64_t)(b * 4 + v) * nc + i] = acc[v];
}

// ---------------------------------------------------------------------------
// k_adj_chem: replay of the cell's chemistry over the subcycle on duals, for
// the 7 + NB input directions (x_HI, x_HII, y_I, y_II, y_III, u, N_b, n_H)
// in passes of KC directions each (a dual of all directions at once does
// not fit in registers); the flux factors Fh'/Fh = prod 1/fac_b are carried
// as duals seeded with 1.  Every pass takes the same branches (the values
// are the same), so the passes' columns make up one Jacobian.
// Overwrites lambda_U (N, Fh parts), lambda_X, lambda_u with the adjoint of
// the pre-chemistry state and adds n_H dL/dn_H to lambda_lnnH.
// ---------------------------------------------------------------------------
template <int NB, int KC>
__global__ __launch_bounds__(kBlock) void k_adj_chem(const double* __restrict__ Upre, const double* __restrict__ Xpre,
                                                     const double* __restrict__ Upre_u, const double* __restrict__ nH,
                                                     double* __restrict__ lam_U, double* __restrict__ lam_X,
                                                     double* __restrict__ lam_u, double* __restrict__ lam_lnnH,
                                                     int32_t* __restrict__ fail, int64_t nc, ChemParams P, double dt) {
    constexpr int K = 7 + NB;                       // input directions
    const int64_t blk = xcd_logical_block();
    const int64_t i = blk * kBlock + threadIdx.x;
    if (i >= nc) return;
    // the adjoint of the post-chemistry state
    double lX[5], lN[NB], lF[NB];
#pragma unroll
    for (int q = 0; q < 5; ++q) lX[q] = lam_X[(int64_t)q * nc + i];
    const double lu = lam_u[i];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        lN[b] = lam_U[(int64_t)(b * 4) * nc + i];
        lF[b] = 0.0;
        for (int c = 0; c < 3; ++c)
            lF[b] += lam_U[(int64_t)(b * 4 + 1 + c) * nc + i] * Upre[urec(b, nc, i) + 1 + c];
    }
    const double nh = nH[i];
    double fac[NB];
    for (int k0 = 0; k0 < K; k0 += KC) {
        // seed directions k0 .. k0 + KC - 1
        auto seed = [&](Dual<KC>& d, int k) {
            if (k >= k0 && k < k0 + KC) d.d[k - k0] = 1.0;
        };
        ChemState<NB, Dual<KC>> s;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            s.N[b] = Dual<KC>(Upre[urec(b, nc, i)]);
            seed(s.N[b], 6 + b);
            s.Fh[b][0] = Dual<KC>(1.0);
            s.Fh[b][1] = Dual<KC>(0.0);
            s.Fh[b][2] = Dual<KC>(0.0);
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            s.x[q] = Dual<KC>(Xpre[(int64_t)q * nc + i]);
            seed(s.x[q], q);
        }
        s.u = Dual<KC>(Upre_u[i]);
        seed(s.u, 5);
        Dual<KC> nHd(nh);
        seed(nHd, 6 + NB);
        const int att = integrate_cell<NB, Dual<KC>>(P, dt, nHd, s);
        if (att > P.max_sub) {
            fail[blockIdx.x] = 1;
            return;
        }
        // the adjoint of input k = k0 + j, written as soon as it is complete
        // (the post-chemistry adjoint it overwrites was read above)
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int k = k0 + j;
            if (k >= K) break;
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 5; ++q) acc += lX[q] * s.x[q].d[j];
            acc += lu * s.u.d[j];
#pragma unroll
            for (int b = 0; b < NB; ++b) acc += lN[b] * s.N[b].d[j] + lF[b] * s.Fh[b][0].d[j];
            if (k < 5) lam_X[(int64_t)k * nc + i] = acc;
            else if (k == 5) lam_u[i] = acc;
            else if (k < 6 + NB) lam_U[(int64_t)((k - 6) * 4) * nc + i] = acc;
            else lam_lnnH[i] += acc * nh;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) fac[b] = s.Fh[b][0].v;
    }
    // The flux itself only scales by the absorption product.
#pragma unroll
    for (int b = 0; b < NB; ++b)
        for (int c = 0; c < 3; ++c) lam_U[(int64_t)(b * 4 + 1 + c) * nc + i] *= fac[b];
}

// ---------------------------------------------------------------------------
// k_adj_src: dL/d ln Q_k += sum_b lambda_N[b][cell_k] Q_bk dt / V (sources in
// their original order; one lane per source).
// ---------------------------------------------------------------------------
__global__ void k_adj_src(const double* __restrict__ lam_U, const int32_t* __restrict__ cell,
                          const double* __restrict__ rate, const double* __restrict__ vphys, int64_t n_src,
                          int64_t nc, int nb, double dt, double* __restrict__ lam_lnQ) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_src) return;
    const int64_t i = cell[k];
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += lam_U[(int64_t)(b * 4) * nc + i] * (rate[(int64_t)b * n_src + k] * dt / vphys[k]);
    lam_lnQ[k] += acc;
}

__global__ void k_seed_lambda(double* __restrict__ lam_X, const double* __restrict__ dL_dxHI, int64_t nc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) lam_X[i] = dL_dxHI[i];
}

}  // namespace rtk

using namespace rtk;

#define RT_HIP_A(expr)                                                                                    \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            return rt_fail(e_ == hipErrorOutOfMemory ? RT_ENOMEM : RT_EDEVICE, "%s failed: %s", #expr,     \
                           hipGetErrorString(e_));                                                        \
    } while (0)

namespace {

unsigned grid1(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Directions per replay of the chemistry adjoint (registers against passes).
#ifndef RT_ADJ_CHEM_DIRS
#define RT_ADJ_CHEM_DIRS 2
#endif
constexpr int kAdjChemDirs = RT_ADJ_CHEM_DIRS;

template <int NB>
void launch_adj_chem_nb(const double* Upre, const double* Xpre, const double* ue, const double* nH, double* lU,
                        double* lX, double* lu, double* lnn, int32_t* fail, int64_t nc, const ChemParams& P,
                        double dt, hipStream_t st) {
    hipLaunchKernelGGL((k_adj_chem<NB, kAdjChemDirs>), dim3(grid1(nc, kBlock)), dim3(kBlock), 0, st, Upre, Xpre, ue, nH,
                       lU, lX, lu, lnn, fail, nc, P, dt);
}

struct Segment {
    DevMem U, X, u;
};

}  // namespace

extern "C" int rt_subcycle_adjoint(const rt_state* initial, int n_subcycles, int checkpoint_every, double dt_in,
                                   const double* dL_dxHI_final, double* dL_dlnQ, double* dL_dln_nH,
                                   void* hip_stream) {
    if (!initial) return rt_fail(RT_EINVAL, "null state");
    if (!std::isfinite(dt_in)) return rt_fail(RT_EINVAL, "dt=%g", dt_in);
    if (!(dt_in <= 0) && !(dt_in <= initial->dt_cfl))
        return rt_fail(RT_EINVAL, "dt=%g above the CFL step %g", dt_in, initial->dt_cfl);
    if (n_subcycles < 0 || checkpoint_every < 1) return rt_fail(RT_EINVAL, "n_subcycles=%d checkpoint_every=%d",
                                                                n_subcycles, checkpoint_every);
    if (!dL_dxHI_final || !dL_dln_nH || (initial->n_src > 0 && !dL_dlnQ)) return rt_fail(RT_EINVAL, "null array");
    if (initial->precision != RT_FP64) return rt_fail(RT_ESTATE, "the adjoint needs an FP64 state");
    if (initial->nb > 4) return rt_fail(RT_ESTATE, "the adjoint supports up to 4 bins");
    if (initial->mesh->max_deg > 16) return rt_fail(RT_ESTATE, "the adjoint supports up to 16 faces per cell");
    rt_mesh* m = initial->mesh;
    int dev_prev = -1;
    (void)hipGetDevice(&dev_prev);
    (void)hipSetDevice(m->device);
    struct Restore {
        int d;
        ~Restore() { if (d >= 0) (void)hipSetDevice(d); }
    } restore{dev_prev};
    hipStream_t st = (hipStream_t)hip_stream;

    // Working copy of the initial state.
    rt_state* w = nullptr;
    int rc = rt_state_clone(initial, &w);
    if (rc) return rc;
    struct Owner {
        rt_state* s;
        ~Owner() { if (s) rt_state_destroy(s); }
    } owner{w};
    // The adjoint recomputes the forward pass on the split path, whose face
    // states it differentiates.
    w->transport_mode = RT_TRANSPORT_SPLIT;
    if ((rc = w->ensure_face_states())) return rc;
    const int64_t nc = w->nc;
    const int nb = w->nb;
    const double dt = dt_in <= 0 ? w->dt_cfl : dt_in;
    const double cdt = w->params.c_reduced * dt / m->h_ref;
    const size_t ub = (size_t)nb * 4 * nc * 8;
    const int C = checkpoint_every;
    const int n = n_subcycles;
    const int n_ck = (n + C - 1) / C;
    const int seg_len = std::min(C, std::max(n, 1));

    // Checkpoints and segment storage.
    std::vector<Segment> ck(n_ck);
    std::vector<DevMem> pre_U(seg_len), pre_X(seg_len), pre_u(seg_len), mid_U(seg_len);
    for (auto& c : ck)
        if ((rc = c.U.alloc(ub)) || (rc = c.X.alloc(5 * nc * 8)) || (rc = c.u.alloc(nc * 8))) return rc;
    for (int j = 0; j < seg_len; ++j)
        if ((rc = pre_U[j].alloc(ub)) || (rc = pre_X[j].alloc(5 * nc * 8)) || (rc = pre_u[j].alloc(nc * 8)) ||
            (rc = mid_U[j].alloc(ub)))
            return rc;
    // Adjoint buffers.
    const int64_t n_entries = m->n_entries;
    DevMem lU, lX, lu, lnn, lq, lpre, ldir, lg, cself, cslot, fail, d_cell, d_rate, d_vp, d_dL, G, tmax, tau;
    if ((rc = lU.alloc(ub)) || (rc = lX.alloc(5 * nc * 8)) || (rc = lu.alloc(nc * 8)) || (rc = lnn.alloc(nc * 8)) ||
        (rc = lq.alloc(std::max<int64_t>(w->n_src, 1) * 8)) || (rc = lpre.alloc(ub)) || (rc = ldir.alloc(ub)) ||
        (rc = lg.alloc(3 * ub)) || (rc = cself.alloc(ub)) || (rc = cslot.alloc((size_t)nb * 4 * n_entries * 8)) ||
        (rc = fail.alloc(grid1(nc, kBlock) * 4)) || (rc = G.alloc(3 * ub)) ||
        (rc = tmax.alloc((size_t)grid1(nc, kBlock) * nb * 8)) || (rc = tau.alloc((size_t)nb * 8)))
        return rc;
    {
        std::vector<int32_t> cell(w->n_src);
        std::vector<double> vp(w->n_src);
        for (int64_t k = 0; k < w->n_src; ++k) {
            cell[k] = (int32_t)w->src_cell[k];
            vp[k] = m->vphys[w->src_cell[k]];
        }
        if ((rc = d_cell.upload(cell.data(), cell.size() * 4)) ||
            (rc = d_rate.upload(w->src_rate.data(), w->src_rate.size() * 8)) ||
            (rc = d_vp.upload(vp.data(), vp.size() * 8)))
            return rc;
        std::vector<double> h(nc);
        hipPointerAttribute_t a;
        bool on_dev = hipPointerGetAttributes(&a, dL_dxHI_final) == hipSuccess &&
                      (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged);
        (void)hipGetLastError();
        if (on_dev) RT_HIP_A(hipMemcpy(h.data(), dL_dxHI_final, nc * 8, hipMemcpyDeviceToHost));
        else std::memcpy(h.data(), dL_dxHI_final, nc * 8);
        if ((rc = d_dL.upload(h.data(), nc * 8))) return rc;
    }

    auto save = [&](DevMem& dU, DevMem& dX, DevMem& du) -> int {
        RT_HIP_A(hipMemcpyAsync(dU.ptr, w->U[w->cur].ptr, ub, hipMemcpyDeviceToDevice, st));
        RT_HIP_A(hipMemcpyAsync(dX.ptr, w->X.ptr, 5 * nc * 8, hipMemcpyDeviceToDevice, st));
        RT_HIP_A(hipMemcpyAsync(du.ptr, w->Ue.ptr, nc * 8, hipMemcpyDeviceToDevice, st));
        return RT_OK;
    };
    auto load = [&](const Segment& c) -> int {
        RT_HIP_A(hipMemcpyAsync(w->U[w->cur].ptr, c.U.ptr, ub, hipMemcpyDeviceToDevice, st));
        RT_HIP_A(hipMemcpyAsync(w->X.ptr, c.X.ptr, 5 * nc * 8, hipMemcpyDeviceToDevice, st));
        RT_HIP_A(hipMemcpyAsync(w->Ue.ptr, c.u.ptr, nc * 8, hipMemcpyDeviceToDevice, st));
        return RT_OK;
    };

    // Forward pass with checkpoints.
    rt_reset_partials(w, st);
    for (int q = 0; q < n_ck; ++q) {
        if ((rc = save(ck[q].U, ck[q].X, ck[q].u))) return rc;
        rt_run_subcycles(w, std::min(C, n - q * C), dt, st);
    }
    int status = 0;
    if ((rc = rt_read_status(w, st, &status))) return rc;
    if (status) return rt_fail(RT_ENUMERIC, "forward pass status 0x%x", status);

    // Seed: lambda_X[x_HI] = dL/dx_HI; everything else zero.
    fill_words(lU.ptr, ub / 4, 0, st);
    fill_words(lX.ptr, 5 * nc * 2, 0, st);
    fill_words(lu.ptr, nc * 2, 0, st);
    fill_words(lnn.ptr, nc * 2, 0, st);
    fill_words(lq.ptr, std::max<int64_t>(w->n_src, 1) * 2, 0, st);
    fill_words(fail.ptr, grid1(nc, kBlock), 0, st);
    hipLaunchKernelGGL(k_seed_lambda, dim3(grid1(nc, 256)), dim3(256), 0, st, (double*)lX.ptr,
                       (const double*)d_dL.ptr, nc);

    const GeomView<double> geo = rt_geo64(m);
    const SellView sell = rt_sell(m);
    const int64_t tblk = transport_blocks(nc, nb);
    for (int q = n_ck - 1; q >= 0; --q) {
        const int len = std::min(C, n - q * C);
        if ((rc = load(ck[q]))) return rc;
        // Recompute the segment, keeping the chemistry input and output.
        for (int j = 0; j < len; ++j) {
            void* U = w->U[w->cur].ptr;
            void* Un = w->U[w->cur ^ 1].ptr;
            rt_step_sources(w, U, dt, st);
            if ((rc = save(pre_U[j], pre_X[j], pre_u[j]))) return rc;
            rt_step_chem(w, U, (double*)w->X.ptr, (double*)w->Ue.ptr, dt, st);
            RT_HIP_A(hipMemcpyAsync(mid_U[j].ptr, U, ub, hipMemcpyDeviceToDevice, st));
            rt_step_facestate(w, U, w->FV.ptr, Un, st, dt, false);
            rt_step_flux(w, U, w->FV.ptr, Un, dt, st);
            w->cur ^= 1;
        }
        // Reverse sweep over the segment.
        for (int j = len - 1; j >= 0; --j) {
            const double* Um = (const double*)mid_U[j].ptr;
            const double* tv = (const double*)tau.ptr;
            rt_step_facestate(w, Um, w->FV.ptr, nullptr, st, dt, true);
            launch_gradient(Um, (double*)G.ptr, nc, nb, geo, sell, w->params.use_limiter, st);
            hipLaunchKernelGGL(k_adj_binmax, dim3((unsigned)tblk), dim3(kBlock), 0, st, Um, nc, nb, (double*)tmax.ptr);
            hipLaunchKernelGGL(k_adj_tau, dim3((unsigned)nb), dim3(kBlock), 0, st, (const double*)tmax.ptr,
                               (int64_t)grid1(nc, kBlock), nb, (double*)tau.ptr);
            hipLaunchKernelGGL(k_adj_guard, dim3((unsigned)tblk), dim3(kBlock), 0, st, Um, (const double*)w->FV.ptr,
                               (const double*)lU.ptr, (double*)lpre.ptr, nc, nb, n_entries, geo, sell, cdt);
            hipLaunchKernelGGL(k_adj_flux, dim3((unsigned)tblk), dim3(kBlock), 0, st, Um, (const double*)G.ptr,
                               (const double*)lpre.ptr, (double*)ldir.ptr, (double*)lg.ptr, nc, nb, geo, sell, cdt,
                               tv);
            if (m->max_deg <= 6)
                hipLaunchKernelGGL(k_adj_grad<7>, dim3((unsigned)tblk), dim3(kBlock), 0, st, Um, (const double*)lg.ptr,
                                   (double*)cself.ptr, (double*)cslot.ptr, n_entries, nc, nb, geo, sell,
                                   w->params.use_limiter, tv);
            else
                hipLaunchKernelGGL(k_adj_grad<17>, dim3((unsigned)tblk), dim3(kBlock), 0, st, Um,
                                   (const double*)lg.ptr, (double*)cself.ptr, (double*)cslot.ptr, n_entries, nc, nb,
                                   geo, sell, w->params.use_limiter, tv);
            hipLaunchKernelGGL(k_adj_gather, dim3((unsigned)tblk), dim3(kBlock), 0, st, (const double*)ldir.ptr,
                               (const double*)cself.ptr, (const double*)cslot.ptr, n_entries, (double*)lU.ptr, nc, nb,
                               sell, Um, tv);
            if (w->params.chem_mode != RT_CHEM_NONE) {
                const double* Up = (const double*)pre_U[j].ptr;
                const double* Xp = (const double*)pre_X[j].ptr;
                const double* up = (const double*)pre_u[j].ptr;
                double* a = (double*)lU.ptr;
                double* bX = (double*)lX.ptr;
                double* c = (double*)lu.ptr;
                double* dn = (double*)lnn.ptr;
                int32_t* fl = (int32_t*)fail.ptr;
                const double* nH = (const double*)w->nH.ptr;
                switch (nb) {
                    case 1: launch_adj_chem_nb<1>(Up, Xp, up, nH, a, bX, c, dn, fl, nc, w->cp, dt, st); break;
                    case 2: launch_adj_chem_nb<2>(Up, Xp, up, nH, a, bX, c, dn, fl, nc, w->cp, dt, st); break;
                    case 3: launch_adj_chem_nb<3>(Up, Xp, up, nH, a, bX, c, dn, fl, nc, w->cp, dt, st); break;
                    default: launch_adj_chem_nb<4>(Up, Xp, up, nH, a, bX, c, dn, fl, nc, w->cp, dt, st); break;
                }
            }
            if (w->n_src > 0)
                hipLaunchKernelGGL(k_adj_src, dim3(grid1(w->n_src, 64)), dim3(64), 0, st, (const double*)lU.ptr,
                                   (const int32_t*)d_cell.ptr, (const double*)d_rate.ptr, (const double*)d_vp.ptr,
                                   w->n_src, nc, nb, dt, (double*)lq.ptr);
        }
    }
    RT_HIP_A(hipGetLastError());
    RT_HIP_A(hipStreamSynchronize(st));
    {
        std::vector<int32_t> hf(grid1(nc, kBlock));
        RT_HIP_A(hipMemcpy(hf.data(), fail.ptr, hf.size() * 4, hipMemcpyDeviceToHost));
        for (int32_t v : hf)
            if (v) return rt_fail(RT_ENUMERIC, "chemistry replay hit the substep cap");
    }
    auto put = [&](double* dst, const DevMem& src, size_t bytes) -> int {
        if (!bytes) return RT_OK;
        hipPointerAttribute_t a;
        bool on_dev = hipPointerGetAttributes(&a, dst) == hipSuccess &&
                      (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged);
        (void)hipGetLastError();
        RT_HIP_A(hipMemcpy(dst, src.ptr, bytes, on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
        return RT_OK;
    };
    if ((rc = put(dL_dln_nH, lnn, nc * 8))) return rc;
    if (w->n_src > 0 && (rc = put(dL_dlnQ, lq, w->n_src * 8))) return rc;
    return RT_OK;
}
