// HIP kernels of the M1 radiative-transfer subcycle for gfx950 (CDNA4).
//
// One subcycle (Zier et al. 2024, Fig. 1) is four launches on one stream:
//   k_sources    point-source injection, one lane per source cell
//   k_chem       thermochemistry + absorption, one lane per cell (FP64)
//   k_facestate  least-squares gradients + slope limiter in FP64 registers,
//                then the limited state at each face centre, one lane per
//                (cell, bin); writes one 4-value record per face side
//   k_flux       face fluxes + divergence update, one lane per (cell, bin)
//   (k_reduce    diagnostics, once per call)
// k_facestate and k_flux are the split form of the transport step; the
// fused k_transport does both per 256-cell tile with the face states in LDS
// and is used whenever the mesh's tiles fit (see k_transport).
// The path is a six-neighbour gather stencil bound by memory traffic, so
// there is no matrix-core work.  Lanes of a wavefront are 64 consecutive
// cells of one bin; fields are 4-value records per (bin, cell) and geometry
// is one record per face and per cell, so a gathered neighbour costs one or
// two 16-byte loads.  Each cell computes the fluxes of its own faces from the
// two face states in the face's canonical (L, R) orientation: the two cells
// of a face obtain bit-identical fluxes of opposite sign, so accumulation is
// deterministic and needs no atomics or face-flux array (the paper's GPU
// design stores fluxes per interface and gathers them in a second kernel,
// Sec. 4.1.3).  T is the storage precision of the transport fields (double,
// or float in the mixed form); gradients and face extrapolation are FP64 in
// registers, flux sums and photon sums FP64, chemistry FP64.

#include <hip/hip_runtime.h>

#include "rt_chem.hpp"
#include "rt_face.hpp"
#include "rt_transport.hpp"
#include "rt_kernels.hpp"
#include "rt_types.hpp"

namespace rtk {

// ---------------------------------------------------------------------------
// Reduction helpers (wave64 shuffles, then the four waves of a block in a
// fixed order).
// ---------------------------------------------------------------------------

template <typename V>
__device__ inline V wave_sum(V v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename V>
__device__ inline V wave_max(V v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        V w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}
__device__ inline int wave_or(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// Sum over the block; the result is valid in thread 0.
template <typename V, int NT = kBlock>
__device__ inline V block_sum(V v, V* lds) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    V s = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) s += lds[k];
    return s;
}
template <typename V>
__device__ inline V block_max(V v, V* lds) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    V s = lds[0];
    if (threadIdx.x == 0)
        for (int k = 1; k < kBlock / 64; ++k) s = lds[k] > s ? lds[k] : s;
    return s;
}
template <int NT = kBlock>
__device__ inline int block_or(int v, int* lds) {
    v = wave_or(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    int s = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) s |= lds[k];
    return s;
}

// ---------------------------------------------------------------------------
// Fill kernels (used instead of memset so every launch is a kernel).
// ---------------------------------------------------------------------------

__global__ void k_fill_bytes(uint32_t* p, int64_t n_words, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_words) p[i] = v;
}

// ---------------------------------------------------------------------------
// k_sources: N_b += Q_bk dt / V_k for the sources of each source cell, in
// source-list order (sources were stably sorted by cell on the host).
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_sources(T* __restrict__ U, int64_t nc, int nb, int32_t n_cells_src,
                          const int32_t* __restrict__ cell, const int32_t* __restrict__ ptr,
                          const double* __restrict__ rate /*[nb][n_src] sorted*/, int64_t n_src,
                          const double* __restrict__ vphys /*[n_src]*/, const double* __restrict__ inv_scale,
                          const double* __restrict__ scale, double dt) {
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells_src) return;
    const int64_t i = cell[c];
    for (int b = 0; b < nb; ++b) {
        T* Nb = U + urec(b, nc, i);
        double N = (double)Nb[0] * scale[b];
        for (int32_t k = ptr[c]; k < ptr[c + 1]; ++k) N = N + rate[(int64_t)b * n_src + k] * dt / vphys[k];
        Nb[0] = (T)(N * inv_scale[b]);
    }
}

// ---------------------------------------------------------------------------
// k_chem: thermochemistry with the adaptive substeps held in registers
// (Sec. 4.1.1).  The number of substeps varies by orders of magnitude between
// cells (an I-front cell takes hundreds, a cell in equilibrium one), so a
// wavefront that gave each lane one fixed cell would run as long as its
// slowest cell with the other lanes idle.  Instead each workgroup owns a
// chunk of cells and a lane that finishes its cell takes the next one from a
// counter in LDS: lanes stay busy until the chunk is exhausted.  Which lane
// integrates a cell does not change its arithmetic, so results are the same
// bit for bit as a one-cell-per-lane launch.
// ---------------------------------------------------------------------------

// Inputs of one cell, as stored.
template <int NB, typename T>
struct ChemInput {
    T U[NB][4];
    double x[5], u, nh;
    int32_t att;           // the cell's attempts so far in this call
};

template <int NB, typename T>
__device__ inline void chem_fetch(const T* __restrict__ U, const double* __restrict__ X, const double* __restrict__ Ue,
                                  const double* __restrict__ nH, const int32_t* __restrict__ att, int64_t nc, int64_t i,
                                  ChemInput<NB, T>& in) {
#pragma unroll
    for (int b = 0; b < NB; ++b) load4(U + urec(b, nc, i), in.U[b]);
#pragma unroll
    for (int q = 0; q < 5; ++q) in.x[q] = X[(int64_t)q * nc + i];
    in.u = Ue[i];
    in.nh = nH[i];
    in.att = att[i];
}

template <int NB, typename T>
__device__ inline void chem_unpack(const ChemInput<NB, T>& in, const double* __restrict__ scale,
                                   ChemState<NB, double>& s) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        s.N[b] = (double)in.U[b][0] * scale[b];
#pragma unroll
        for (int k = 0; k < 3; ++k) s.Fh[b][k] = (double)in.U[b][1 + k] * scale[b];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) s.x[q] = in.x[q];
    s.u = in.u;
}

template <int NB, typename T>
__global__ __launch_bounds__(kBlock) void k_chem(T* __restrict__ U, double* __restrict__ X /*[5][nc]*/,
                                                 double* __restrict__ Ue /*[nc]*/, const double* __restrict__ nH,
                                                 int64_t nc, int64_t cell0, int64_t cell1, int chunk,
                                                 ChemParams P, double dt,
                                                 const double* __restrict__ scale, const double* __restrict__ inv_scale,
                                                 int64_t* __restrict__ part_sum, int64_t* __restrict__ part_max,
                                                 int32_t* __restrict__ part_status, int32_t* __restrict__ att_cell) {
    __shared__ int next;
    __shared__ int64_t lds64[kBlock / 64];
    __shared__ int lds32[kBlock / 64];
    const int64_t blk = xcd_logical_block();
    const int64_t c0 = cell0 + blk * (int64_t)kBlock * chunk;
    const int64_t c1 = c0 + (int64_t)kBlock * chunk < cell1 ? c0 + (int64_t)kBlock * chunk : cell1;
    if (threadIdx.x == 0) next = kBlock;
    __syncthreads();
    int64_t sum_att = 0, max_att = 0;
    int status = 0;
    // The lane's current cell i and the next one it will take, whose inputs
    // are fetched while i is integrated.
    int64_t i = c0 + threadIdx.x;
    bool active = i < c1;
    ChemState<NB, double> s;
    ChemInput<NB, T> pf;
    double nh = 0.0;
    int32_t att0 = 0;
    int64_t inext = c1;
    if (active) {
        chem_fetch<NB, T>(U, X, Ue, nH, att_cell, nc, i, pf);
        chem_unpack<NB, T>(pf, scale, s);
        nh = pf.nh;
        att0 = pf.att;
        chem_begin<NB, double>(dt, s);
        inext = c0 + atomicAdd(&next, 1);
        if (inext < c1) chem_fetch<NB, T>(U, X, Ue, nH, att_cell, nc, inext, pf);
    }
    while (active) {
        const int r = chem_attempt<NB, double>(P, dt, nh, s);
        if (r == 0) continue;
        sum_att += s.attempts;
        max_att = s.attempts > max_att ? s.attempts : max_att;
        att_cell[i] = att0 + (int32_t)s.attempts;
        if (r < 0) {
            status |= 2;            // leave the cell untouched; the call is rolled back
        } else {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                T o[4] = {(T)(s.N[b] * inv_scale[b]), (T)(s.Fh[b][0] * inv_scale[b]), (T)(s.Fh[b][1] * inv_scale[b]),
                          (T)(s.Fh[b][2] * inv_scale[b])};
                store4(U + urec(b, nc, i), o);
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) X[(int64_t)q * nc + i] = s.x[q];
            Ue[i] = s.u;
            if (!isfinite(s.u)) status |= 1;
        }
        i = inext;
        active = i < c1;
        if (active) {
            chem_unpack<NB, T>(pf, scale, s);
            nh = pf.nh;
            att0 = pf.att;
            chem_begin<NB, double>(dt, s);
            inext = c0 + atomicAdd(&next, 1);
            if (inext < c1) chem_fetch<NB, T>(U, X, Ue, nH, att_cell, nc, inext, pf);
        }
    }
    const int64_t sm = block_sum<int64_t>(sum_att, lds64);
    const int64_t mx = block_max<int64_t>(max_att, lds64);
    const int st = block_or(status, lds32);
    if (threadIdx.x == 0) {
        part_sum[blk] += sm;
        part_max[blk] = mx > part_max[blk] ? mx : part_max[blk];
        part_status[blk] |= st;
    }
}

// ---------------------------------------------------------------------------
// k_facestate: limited gradients of N, Fh_x, Fh_y, Fh_z of one bin in FP64
// (Sec. 2.3.2), then the extrapolated state U_i + g . r_if at each face
// centre (Sec. 2.3.3), stored in the transport precision as one record per
// face side: FV[b][e][4]; and the numerator N V / n_faces of the cell's
// outflow cap, NC[b][nc], for the flux kernel.  Keeping g in registers
// means a limited face state is rounded once, relative to its own size (an
// FP32-stored gradient would cancel at steep fronts, where U + g.r is much
// smaller than U).
// ---------------------------------------------------------------------------

// Store the limited state of cell i at each of its faces: entry e goes to
// out[(e - e0) * 4].
template <typename T, int DEG>
__device__ inline void export_face_states(int64_t i, const double* ui, const double (*g)[3], const T (*rr)[3],
                                          const bool* ok, const GeomView<T>& geo, const SellView& sell,
                                          T* __restrict__ out, int64_t e0) {
    const int64_t slice = i / kSlice;
    const int32_t deg = DEG > 0 ? DEG : sell.deg[slice];
    const int64_t base = (int64_t)sell.ptr[slice] + (i % kSlice);
#pragma unroll(SlotCount<DEG>::kMax)
    for (int k = 0; k < (DEG > 0 ? DEG : deg); ++k) {
        const int64_t e = base + (int64_t)k * kSlice;
        double r0, r1, r2;
        if (DEG > 0) {
            if (!ok[k]) continue;
            r0 = rr[k][0]; r1 = rr[k][1]; r2 = rr[k][2];
        } else {
            if (sell.nbr[e] < 0) continue;
            r0 = geo.sv(kSR0, e); r1 = geo.sv(kSR1, e); r2 = geo.sv(kSR2, e);
        }
        T st[4];
        face_state<T>(ui, g, r0, r1, r2, st);
        store4(out + (e - e0) * 4, st);
    }
}

template <typename T, int DEG>
__global__ __launch_bounds__(kBlock) void k_facestate(const T* __restrict__ U, T* __restrict__ FV, T* __restrict__ NC,
                                                      int64_t nc, int nb, int64_t n_entries, GeomView<T> geo,
                                                      SellView sell, int use_limiter) {
    const int64_t blk = xcd_logical_block();
    if constexpr (DEG > 0) {
        // One lane per (cell, bin) with the cell's side records in registers.
        const int b = (int)(blk % nb);
        const int64_t i = (blk / nb) * kBlock + threadIdx.x;
        if (i >= nc) return;
        CellSides<T, DEG> cs;
        load_cell_sides<T, DEG>(i, geo, sell, cs);
        T cell[8];
        load4(geo.cell + i * kCellRec, cell);
        load4(geo.cell + i * kCellRec + 4, cell + 4);
        const int64_t base = (int64_t)sell.ptr[i / kSlice] + (i % kSlice);
        double ui[4], g[4][3];
        limited_gradient_c<T, DEG>(i, b, nc, U, cell, cs, use_limiter, ui, g);
        NC[(int64_t)b * nc + i] = (T)ui[0] * cell[7];
        T* FVb = FV + (int64_t)b * n_entries * 4;
#pragma unroll
        for (int k = 0; k < DEG; ++k) {
            if (cs.nbr[k] < 0) continue;
            T st[4];
            face_state<T>(ui, g, cs.r[k][0], cs.r[k][1], cs.r[k][2], st);
            store4_stream(FVb + (base + (int64_t)k * kSlice) * 4, st);
        }
    } else {
        const int b = (int)(blk % nb);
        const int64_t i = (blk / nb) * kBlock + threadIdx.x;
        if (i >= nc) return;
        double ui[4], g[4][3];
        T rr[SlotCount<DEG>::kMax][3];
        bool ok[SlotCount<DEG>::kMax];
        limited_gradient_s<T, DEG>(i, b, nc, U, geo, sell, use_limiter, ui, g, rr, ok);
        NC[(int64_t)b * nc + i] = (T)ui[0] * geo.cell[i * kCellRec + 7];
        export_face_states<T, DEG>(i, ui, g, rr, ok, geo, sell, FV + (int64_t)b * n_entries * 4, 0);
    }
}

// ---------------------------------------------------------------------------
// k_gradient: the limited gradients themselves, G[b][v*3+c][nc] in FP64
// (used by the adjoint, which differentiates through the extrapolation).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_gradient(const double* __restrict__ U, double* __restrict__ G, int64_t nc,
                                                     int nb, GeomView<double> geo, SellView sell, int use_limiter) {
    const int64_t blk = xcd_logical_block();
    const int b = (int)(blk % nb);
    const int64_t i = (blk / nb) * kBlock + threadIdx.x;
    if (i >= nc) return;
    double ui[4], g[4][3];
    double rr[1][3];
    bool ok[1];
    limited_gradient_s<double, 0>(i, b, nc, U, geo, sell, use_limiter, ui, g, rr, ok);
    double* Gb = G + (int64_t)(b * 12) * nc;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int c = 0; c < 3; ++c) Gb[(int64_t)(v * 3 + c) * nc + i] = g[v][c];
}

// ---------------------------------------------------------------------------
// k_flux: for each face of the cell, the HLL flux of the two face states and
// the outflow cap theta = min(1, N_up V_up / (n_faces(up) |Phi_N| dt A));
// then U_i <- U_i - (dt / V_i) sum_f sigma A Phi in face-index order, with
// post-update guards.  Writes the new fields to Unew (double buffering:
// neighbours still read U).  Per-block partials: sum N V (this bin),
// counters and status, accumulated across the subcycles of one call.
// ---------------------------------------------------------------------------

// Divergence update of cell i from its flux sum, post-update guards and the
// new record; adds the cell's N V, guard counts and status to the thread's.
// Divergence update of cell i (volume vol_t) from its flux sum, post-update
// guards and the new record; adds the cell's N V, guard counts and status to
// the thread's.  Not contracted, so the split and fused paths round it alike.
template <typename T, typename TA>
__device__ inline void update_cell_v(int64_t i, int b, int64_t nc, const T* ui, T vol_t, const double* acc, TA cdt,
                                     T* __restrict__ Unew, double& nv, int& cGN, int& cGF, int& status) {
#pragma clang fp contract(off)
    const double vol = (double)vol_t;
    const double coef = (double)cdt / vol;
    double un[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) un[v] = (double)ui[v] - coef * acc[v];
    update_guards<double>(un, cGN, cGF);
    T o[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        o[v] = (T)un[v];
        if (!isfinite((double)o[v])) status = 1;
    }
    store4(Unew + urec(b, nc, i), o);
    nv += (double)o[0] * vol;
}

// The update of a cell by part of its flux sum, rounded to the field type:
// w = u - (dt / V) acc.  The by-tile paths apply the tile-interior faces'
// sum this way, then the cross-tile faces' sum with update_cell_v.
template <typename T, typename TA, typename UI>
__device__ inline void partial_update(const UI* ui, T vol_t, const double* acc, TA cdt, T* w) {
#pragma clang fp contract(off)
    const double coef = (double)cdt / (double)vol_t;
#pragma unroll
    for (int v = 0; v < 4; ++v) w[v] = (T)((double)ui[v] - coef * acc[v]);
}

template <typename T, typename TA>
__device__ inline void update_cell(int64_t i, int b, int64_t nc, const T* ui, const double* acc, TA cdt,
                                   const GeomView<T>& geo, T* __restrict__ Unew, double& nv, int& cGN, int& cGF,
                                   int& status) {
    update_cell_v<T, TA>(i, b, nc, ui, geo.cell[i * kCellRec + 6], acc, cdt, Unew, nv, cGN, cGF, status);
}

// Adds a workgroup's counts to its partial slots, accumulated across the
// subcycles of one call.  Integer sums do not depend on order, so the adds
// are atomics whose results are not waited for (a load and a store per
// counter would hold the wavefront for a memory round trip each); zero
// counts, the common case, are skipped.
__device__ inline void add_counts(int64_t* __restrict__ part_cnt, int64_t n_blocks, int64_t blk, int64_t c0, int64_t c1,
                                  int64_t c2, int64_t c3, int64_t c4, int32_t status,
                                  int32_t* __restrict__ part_status) {
    const int64_t c[5] = {c0, c1, c2, c3, c4};
#pragma unroll
    for (int q = 0; q < 5; ++q)
        if (c[q] != 0) atomicAdd(reinterpret_cast<unsigned long long*>(part_cnt + q * n_blocks + blk),
                                 (unsigned long long)c[q]);
    if (status != 0) atomicOr(part_status + blk, status);
}

// The partials of a workgroup whose cells are one wavefront (the
// slot-parallel flux kernel): shuffle sums and ballots, no barrier; lane 0
// writes them.
__device__ inline void wave_partials(double nv, int cAdmN, int cAdmF, int cCap, int cGN, int cGF, int status,
                                     int64_t blk, double* __restrict__ part_nv, int64_t* __restrict__ part_cnt,
                                     int32_t* __restrict__ part_status, int64_t n_blocks) {
    const uint64_t packed = (uint64_t)cAdmN | ((uint64_t)cAdmF << 21) | ((uint64_t)cCap << 42);
    const double snv = wave_sum(nv);
    const uint64_t spk = wave_sum(packed);
    const uint64_t bGN = __ballot(cGN != 0), bGF = __ballot(cGF != 0), bST = __ballot(status != 0);
    if ((threadIdx.x & 63) == 0) {
        constexpr uint64_t kField = (1ull << 21) - 1;
        part_nv[blk] = snv;
        add_counts(part_cnt, n_blocks, blk, (int64_t)(spk & kField), (int64_t)((spk >> 21) & kField),
                   (int64_t)((spk >> 42) & kField), (int64_t)__popcll(bGN), (int64_t)__popcll(bGF),
                   bST != 0 ? 1 : 0, part_status);
    }
}

// The block's partials (sum N V of this bin, counters, status), accumulated
// across the subcycles of one call.  Called by every thread of the block.
// Each wave reduces N V and the three per-face counts (packed in 21-bit
// fields of one 64-bit sum; a block's count stays below 2^21 for cells of
// up to kMaxCellFaces faces) with shuffles, the 0/1 guard flags and status
// with ballots; one barrier, then thread 0 adds the waves in order.
template <int NT = kBlock>
__device__ inline void block_partials(double nv, int cAdmN, int cAdmF, int cCap, int cGN, int cGF, int status,
                                      int64_t blk, double* __restrict__ part_nv, int64_t* __restrict__ part_cnt,
                                      int32_t* __restrict__ part_status, int64_t n_blocks) {
    static_assert((int64_t)NT * kMaxCellFaces < (1 << 21), "packed counters overflow");
    __shared__ double ldsd[NT / 64];
    __shared__ uint64_t ldsc[NT / 64];
    __shared__ uint32_t ldsg[NT / 64][3];
    const uint64_t packed = (uint64_t)cAdmN | ((uint64_t)cAdmF << 21) | ((uint64_t)cCap << 42);
    const double snv = wave_sum(nv);
    const uint64_t spk = wave_sum(packed);
    const uint64_t bGN = __ballot(cGN != 0), bGF = __ballot(cGF != 0), bST = __ballot(status != 0);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        ldsd[w] = snv;
        ldsc[w] = spk;
        ldsg[w][0] = (uint32_t)__popcll(bGN);
        ldsg[w][1] = (uint32_t)__popcll(bGF);
        ldsg[w][2] = bST != 0 ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sn = 0.0;
        uint64_t sc = 0;
        int64_t g0 = 0, g1 = 0;
        uint32_t st = 0;
        for (int k = 0; k < NT / 64; ++k) {
            sn += ldsd[k];
            sc += ldsc[k];
            g0 += ldsg[k][0];
            g1 += ldsg[k][1];
            st |= ldsg[k][2];
        }
        constexpr uint64_t kField = (1ull << 21) - 1;
        part_nv[blk] = sn;
        add_counts(part_cnt, n_blocks, blk, (int64_t)(sc & kField), (int64_t)((sc >> 21) & kField),
                   (int64_t)((sc >> 42) & kField), g0, g1, (int32_t)st, part_status);
    }
}

template <typename T, typename TA, int NT = kBlock>
__device__ inline void finish_cell(int64_t i, int b, int64_t nc, const T* ui, const double* acc, TA cdt,
                                   const GeomView<T>& geo, T* __restrict__ Unew, int cAdmN, int cAdmF, int cCap,
                                   int64_t blk, double* __restrict__ part_nv, int64_t* __restrict__ part_cnt,
                                   int32_t* __restrict__ part_status, int64_t n_blocks) {
    int cGN = 0, cGF = 0, status = 0;
    double nv = 0.0;
    if (i < nc) update_cell<T, TA>(i, b, nc, ui, acc, cdt, geo, Unew, nv, cGN, cGF, status);
    block_partials<NT>(nv, cAdmN, cAdmF, cCap, cGN, cGF, status, blk, part_nv, part_cnt, part_status, n_blocks);
}

// General meshes (any degree): one lane per (cell, bin), the cell's slots in
// a loop.
template <typename T, typename TA>
__global__ __launch_bounds__(kFluxBlock) void k_flux(const T* __restrict__ U, const T* __restrict__ FV,
                                                 const T* __restrict__ NC, T* __restrict__ Unew,
                                                 int64_t nc, int nb, int64_t n_entries, GeomView<T> geo, SellView sell,
                                                 TA cdt, double* __restrict__ part_nv, int64_t* __restrict__ part_cnt,
                                                 int32_t* __restrict__ part_status, int64_t n_blocks, int64_t slice0) {
    const int64_t blk = slice0 * nb + xcd_logical_block();   // partial slot: (slice, bin) of the whole mesh
    const int b = (int)(blk % nb);
    const int64_t i = (blk / nb) * kFluxBlock + threadIdx.x;
    int cAdmN = 0, cAdmF = 0, cCap = 0;
    T ui[4] = {0, 0, 0, 0};
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < nc) {
        load4(U + urec(b, nc, i), ui);
        const GlobalFaceStates<T> fsv{FV + (int64_t)b * n_entries * 4, sell.opp, NC + (int64_t)b * nc};
        cell_flux_sum_s<T, TA, 0>(i, b, nc, U, fsv, geo, sell, cdt, (TA)fsv.cellN((int32_t)i), acc, cAdmN, cAdmF,
                                  cCap);
    }
    finish_cell<T, TA, kFluxBlock>(i, b, nc, ui, acc, cdt, geo, Unew, cAdmN, cAdmF, cCap, blk, part_nv, part_cnt,
                                   part_status, n_blocks);
}

// Meshes whose slices all have DEG slots: one workgroup per (64-cell slice,
// bin).  Its threads share out the slice's face evaluations (the mesh's
// fitem list): a face whose two sides are both in the slice is evaluated
// once, from its L side, and its R side takes the negated product, which is
// the value that side would compute itself (the flux is formed in the
// face's canonical orientation, so it is the same to the last bit); a face
// that crosses to another slice is evaluated here for this slice's side.
// On a Hilbert-ordered lattice a 64-cell slice is a 4x4x4 block whose 144
// inner faces are evaluated once: 240 evaluations instead of 384.  Each
// evaluation's loads are its entry's index, face record and face state and
// the cell's cap numerator, then the opposite face state and the
// neighbour's cap numerator.  The products sigma A Phi go through LDS by
// entry; after one barrier the first wavefront adds each cell's slots in
// slot (face-index) order in FP64, as the one-lane form does, and updates
// the cell.
template <typename T, typename TA, int DEG>
__global__ __launch_bounds__(kFluxPairThreads) void k_flux_pairs(
    const T* __restrict__ U, const T* __restrict__ FV, const T* __restrict__ NC, T* __restrict__ Unew, int64_t nc,
    int nb, int64_t n_entries, GeomView<T> geo, SellView sell, TA cdt, double* __restrict__ part_nv,
    int64_t* __restrict__ part_cnt, int32_t* __restrict__ part_status, int64_t n_blocks, int64_t slice0) {
    static_assert(DEG > 0, "uniform-degree meshes");
    constexpr int kPer = DEG * kSlice;                 // entries of a slice
    __shared__ TA lflux[4][kPer];
    __shared__ uint8_t lcnt[kPer];                    // bits 0-1, 2-3, 4: admissibility N, F, cap (L side)
    const uint32_t blk32 = xcd_logical_block32();
    const int b = (int)(blk32 % (uint32_t)nb);
    const int64_t sl = slice0 + blk32 / (uint32_t)nb;
    const int64_t blk = sl * nb + b;                   // partial slot of the whole mesh
    const T* FVb = FV + (int64_t)b * n_entries * 4;
    const T* NCb = NC + (int64_t)b * nc;
    const int l = threadIdx.x % kSlice;
    const int64_t i = sl * kSlice + l;
    const int64_t ic = i < nc ? i : nc - 1;
    // The first wavefront's cell record and volume, for the update (every
    // wavefront requests them: under a branch they would be waited for at
    // once; the others find them in the cache).
    T ui[4];
    load4(U + urec(b, nc, ic), ui);
    const T vol = geo.vol[ic];
    const int32_t it0 = sell.fitem_ptr[sl], it1 = sell.fitem_ptr[sl + 1];
    for (int32_t it = it0 + (int32_t)threadIdx.x; it < it1; it += kFluxPairThreads) {
        const int2 item = sell.fitem[it];
        const bool pair = (item.x & kFluxPairBit) != 0;
        const int64_t e = item.x & ~kFluxPairBit;
        const int32_t os = item.y;
        T ga[4], so[4], sn[4];
        load4(geo.sg(3, e), ga);
        load4(FVb + e * 4, so);
        const int64_t ci = (e / kPer) * kSlice + e % kSlice;     // the entry's cell
        const T ni = NCb[ci];
        const bool isL = os >= 0;
        const int64_t eo = isL ? os : ~os;
        const int64_t j = (eo / kPer) * kSlice + eo % kSlice;    // the neighbour
        const T nj = NCb[j];
        load4(FVb + eo * 4, sn);
        __builtin_amdgcn_sched_barrier(0);
        const TA A = (TA)ga[0];
        TA sL[4], sR[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            sL[v] = (TA)(isL ? so[v] : sn[v]);
            sR[v] = (TA)(isL ? sn[v] : so[v]);
        }
        const TA NL = (TA)(isL ? ni : nj), NR = (TA)(isL ? nj : ni);   // cap numerators N V / n_faces
        int aN = 0, aF = 0;
        TA Phi[4];
        const bool capped = face_flux<TA, TA>(sL, sR, NL, NR, (TA)1, (TA)1, (TA)ga[1], (TA)ga[2], (TA)ga[3], A, cdt,
                                             Phi, aN, aF);
        const TA sA = isL ? A : -A;
        const int q = (int)(e - sl * kPer);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const TA ph = mul_nc(sA, Phi[v]);
            lflux[v][q] = ph;
            if (pair) lflux[v][(int)(eo - sl * kPer)] = -ph;
        }
        lcnt[q] = (uint8_t)(isL ? ((uint32_t)aN | ((uint32_t)aF << 2) | ((capped ? 1u : 0u) << 4)) : 0u);
        if (pair) lcnt[(int)(eo - sl * kPer)] = 0;
    }
    __syncthreads();
    if (threadIdx.x >= kSlice) return;
    int cAdmN = 0, cAdmF = 0, cCap = 0, cGN = 0, cGF = 0, status = 0;
    double nv = 0.0;
    if (i < nc) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < DEG; ++k) {
            const int q = k * kSlice + l;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += (double)lflux[v][q];
            const uint32_t c = lcnt[q];
            cAdmN += (int)(c & 3u);
            cAdmF += (int)((c >> 2) & 3u);
            cCap += (int)((c >> 4) & 1u);
        }
        update_cell_v<T, TA>(i, b, nc, ui, vol, acc, cdt, Unew, nv, cGN, cGF, status);
    }
    wave_partials(nv, cAdmN, cAdmF, cCap, cGN, cGF, status, blk, part_nv, part_cnt, part_status, n_blocks);
}

// ---------------------------------------------------------------------------
// Split transport on six-slot meshes, by tile of kTileCells cells (the fused
// kernel's tiles), one workgroup per (tile, bin), one thread per tile cell:
//   k_facestate_tile  each cell's limited gradient and its six face states
//                     into LDS; the states of faces that cross to another
//                     tile, with the cell's cap numerator, also to HBM,
//                     packed in boundary-item order; then every
//                     tile-interior face's flux, once, from the two states
//                     in LDS; then each cell's FP64 sum over its
//                     tile-interior faces in slot order, applied to the
//                     cell (partial_update) and stored to the new fields;
//   k_flux_tile       the fluxes of the tile's boundary items (own and
//                     opposite state read by item: the own ones contiguous);
//                     each cell sums them in slot order and finishes its
//                     update in place.
// Only the cross-tile face states (one a cell on a Hilbert-ordered
// lattice, against six) and the partly updated cell go through HBM between
// the two passes.  A cell is updated by its tile-interior faces, rounded to
// the field type, then by its cross-tile ones, each sum in slot order, as
// the fused kernel does too, so the two paths agree bit for bit.
// ---------------------------------------------------------------------------

// Cell (relative to the tile) of an entry relative to the tile's first
// entry, on a six-slot mesh.
__device__ inline int tile_cell_of(int q) { return (q / (6 * kSlice)) * kSlice + q % kSlice; }

// Boundary items of the calling lane's cell in slot order: item of slot k
// (when bit k of bm is set) = first + (items of slots < k in the wavefront's
// slice) + (lanes below with slot k set).  Called by whole wavefronts of
// one slice (lanes past the last cell with bm = 0).
struct SliceItems {
    uint64_t bal[6];
    __device__ void init(uint32_t bm) {
#pragma unroll
        for (int k = 0; k < 6; ++k) bal[k] = __ballot((bm >> k) & 1u);
    }
    // items of slots below k, then the rank within slot k
    __device__ int32_t rank(int k) const {
        const uint64_t lt = (1ull << (threadIdx.x & 63)) - 1ull;
        int32_t r = __popcll(bal[k] & lt);
#pragma unroll
        for (int kk = 0; kk < 6; ++kk)
            if (kk < k) r += __popcll(bal[kk]);
        return r;
    }
};

template <typename T, typename TA>
__global__ __launch_bounds__(kTileThreads) void k_facestate_tile(
    const T* __restrict__ U, T* __restrict__ BS, T* __restrict__ BN, T* __restrict__ Unew, int64_t nc, int nb,
    GeomView<T> geo, SellView sell, TileFaceView tf, int use_limiter, TA cdt, int64_t* __restrict__ part_cnt,
    int32_t* __restrict__ part_status, int64_t n_blocks) {
    constexpr int DEG = 6;
    constexpr int kPer = DEG * kTileCells;           // entries of a tile
    __shared__ TA lst[4][kPer];                      // face states, then the products sigma A Phi
    __shared__ TA lnv[kTileCells];                   // cap numerators N V / n_faces
    __shared__ uint64_t lcnt[kTileThreads / 64];     // packed face counts per wavefront
    const uint32_t blk32 = xcd_logical_block32();
    const int b = (int)(blk32 % (uint32_t)nb);
    const int64_t t = blk32 / (uint32_t)nb;
    const int tid = threadIdx.x;
    const int64_t c0 = t * kTileCells;
    const int64_t i = c0 + tid;
    const int64_t e0 = t * kPer;
    T* BSb = BS + (int64_t)b * tf.n_bnd * 4;
    T* BNb = BN + (int64_t)b * tf.n_bnd;
    // The tile's interior faces, at most three per thread (a face takes two
    // of the tile's 6 kTileCells sides): their indices are requested first,
    // their records before the barrier, so that the face phase waits on no
    // global load.
    constexpr int kRounds = 3;
    const int32_t p0 = tf.pair_ptr[t], p1 = tf.pair_ptr[t + 1];
    int32_t pk[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const int32_t p = p0 + tid + r * kTileThreads;
        pk[r] = p < p1 ? tf.pair[p] : -1;
    }
    const uint32_t bm = i < nc ? tf.bmask[i] : 0u;
    T nv = (T)0;
    if (i < nc) {
        CellSides<T, DEG> cs;
        load_cell_sides<T, DEG>(i, geo, sell, cs);
        T cell[8];
        load4(geo.cell + i * kCellRec, cell);
        load4(geo.cell + i * kCellRec + 4, cell + 4);
        double ui[4], g[4][3];
        limited_gradient_c<T, DEG>(i, b, nc, U, cell, cs, use_limiter, ui, g);
        nv = (T)ui[0] * cell[7];
        lnv[tid] = (TA)nv;
        const int64_t base = (int64_t)sell.ptr[i / kSlice] + (i % kSlice);
#pragma unroll
        for (int k = 0; k < DEG; ++k) {
            T st[4];
            face_state<T>(ui, g, cs.r[k][0], cs.r[k][1], cs.r[k][2], st);
            const int q = (int)(base + (int64_t)k * kSlice - e0);
#pragma unroll
            for (int v = 0; v < 4; ++v) lst[v][q] = (TA)st[v];
        }
    }
    T gar[kRounds][4];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) load4(geo.sg(3, e0 + (pk[r] >= 0 ? (pk[r] & 0xffff) : 0)), gar[r]);
    __syncthreads();
    // the states of the cell's cross-tile sides (still in LDS: the face
    // phase overwrites interior sides only) to their boundary items
    {
        SliceItems si;
        si.init(bm);
        if (bm) {
            const int64_t item0 = tf.bnd_sptr[i / kSlice];
            const int64_t base = (i / kSlice) * (DEG * kSlice) + (i % kSlice);
#pragma unroll
            for (int k = 0; k < DEG; ++k) {
                if (!((bm >> k) & 1u)) continue;
                const int q = (int)(base + (int64_t)k * kSlice - e0);
                const int64_t it = item0 + si.rank(k);
                T st[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) st[v] = (T)lst[v][q];
                store4_stream(BSb + it * 4, st);
                BNb[it] = nv;
            }
        }
    }
    int cAdmN = 0, cAdmF = 0, cCap = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        if (pk[r] < 0) continue;
        const int ql = pk[r] & 0xffff, qr = pk[r] >> 16;
        const T* ga = gar[r];
        TA sL[4], sR[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            sL[v] = lst[v][ql];
            sR[v] = lst[v][qr];
        }
        const TA A = (TA)ga[0];
        int aN = 0, aF = 0;
        TA Phi[4];
        const bool capped = face_flux<TA, TA>(sL, sR, lnv[tile_cell_of(ql)], lnv[tile_cell_of(qr)], (TA)1, (TA)1,
                                             (TA)ga[1], (TA)ga[2], (TA)ga[3], A, cdt, Phi, aN, aF);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const TA ph = mul_nc(A, Phi[v]);
            lst[v][ql] = ph;
            lst[v][qr] = -ph;
        }
        cAdmN += aN;
        cAdmF += aF;
        cCap += capped ? 1 : 0;
    }
    const uint64_t packed = (uint64_t)cAdmN | ((uint64_t)cAdmF << 21) | ((uint64_t)cCap << 42);
    const uint64_t spk = wave_sum(packed);
    if ((tid & 63) == 0) lcnt[tid >> 6] = spk;
    // the cell and its volume again (cache hits), requested before the barrier
    const int64_t ic = i < nc ? i : nc - 1;
    T ui[4];
    load4(U + urec(b, nc, ic), ui);
    const T vi = geo.cell[ic * kCellRec + 6];
    __syncthreads();
    if (i < nc) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const int64_t base = (int64_t)sell.ptr[i / kSlice] + (i % kSlice);
#pragma unroll
        for (int k = 0; k < DEG; ++k) {
            if ((bm >> k) & 1u) continue;
            const int q = (int)(base + (int64_t)k * kSlice - e0);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += (double)lst[v][q];
        }
        T w[4];
        partial_update<T, TA>(ui, vi, acc, cdt, w);
        store4(Unew + urec(b, nc, i), w);
    }
    if (tid == 0) {
        constexpr uint64_t kField = (1ull << 21) - 1;
        uint64_t c = 0;
        for (int w = 0; w < kTileThreads / 64; ++w) c += lcnt[w];
        add_counts(part_cnt, n_blocks, (t * kTileSlices) * nb + b, (int64_t)(c & kField),
                   (int64_t)((c >> 21) & kField), (int64_t)((c >> 42) & kField), 0, 0, 0, part_status);
    }
}

// Products of the boundary items live in dynamic LDS, bnd_max records of
// four TA per workgroup, at the item's index relative to the tile's first.
// Unew holds the cells as k_facestate_tile left them (updated by their
// tile-interior faces); each thread finishes its own cell in place.
template <typename T, typename TA>
__global__ __launch_bounds__(kTileThreads) void k_flux_tile(
    const T* __restrict__ BS, const T* __restrict__ BN,
    T* __restrict__ Unew, int64_t nc, int nb, const T* __restrict__ vol, const T* __restrict__ bgeo,
    TileFaceView tf, TA cdt, double* __restrict__ part_nv, int64_t* __restrict__ part_cnt,
    int32_t* __restrict__ part_status, int64_t n_blocks) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    TA* lph = reinterpret_cast<TA*>(lds_raw);
    __shared__ uint64_t lcnt[kTileThreads / 64];     // packed face counts per wavefront
    constexpr int DEG = 6;
    const uint32_t blk32 = xcd_logical_block32();
    const int b = (int)(blk32 % (uint32_t)nb);
    const int64_t t = blk32 / (uint32_t)nb;
    const int tid = threadIdx.x;
    const int64_t c0 = t * kTileCells;
    const int64_t i = c0 + tid;
    const int64_t ic = i < nc ? i : nc - 1;
    const T* BSb = BS + (int64_t)b * tf.n_bnd * 4;
    const T* BNb = BN + (int64_t)b * tf.n_bnd;
    // the cell's inputs of the update, requested before the face work
    T ui[4];
    load4(Unew + urec(b, nc, ic), ui);
    const T vi = vol[ic];
    const uint32_t bm = i < nc ? tf.bmask[i] : 0u;
    const int32_t item0 = tf.bnd_sptr[ic / kSlice];
    int cAdmN = 0, cAdmF = 0, cCap = 0;
    const int32_t it0 = tf.bnd_ptr[t], it1 = tf.bnd_ptr[t + 1];
    for (int32_t it = it0 + tid; it < it1; it += kTileThreads) {
        const int32_t os = tf.bnd_opp[it];
        const bool isL = os >= 0;
        const int64_t o = isL ? os : ~os;
        T ga[4], so[4], sn[4];
        load4(bgeo + (int64_t)it * 4, ga);
        load4(BSb + (int64_t)it * 4, so);
        load4(BSb + o * 4, sn);
        const T ni = BNb[it], nj = BNb[o];
        __builtin_amdgcn_sched_barrier(0);
        TA sL[4], sR[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            sL[v] = (TA)(isL ? so[v] : sn[v]);
            sR[v] = (TA)(isL ? sn[v] : so[v]);
        }
        const TA A = (TA)ga[0];
        int aN = 0, aF = 0;
        TA Phi[4];
        const bool capped = face_flux<TA, TA>(sL, sR, (TA)(isL ? ni : nj), (TA)(isL ? nj : ni), (TA)1, (TA)1,
                                             (TA)ga[1], (TA)ga[2], (TA)ga[3], A, cdt, Phi, aN, aF);
        const TA sA = isL ? A : -A;
        TA* dst = lph + (int64_t)(it - it0) * 4;
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[v] = mul_nc(sA, Phi[v]);
        if (isL) {
            cAdmN += aN;
            cAdmF += aF;
            cCap += capped ? 1 : 0;
        }
    }
    const uint64_t packed = (uint64_t)cAdmN | ((uint64_t)cAdmF << 21) | ((uint64_t)cCap << 42);
    const uint64_t spk = wave_sum(packed);
    if ((tid & 63) == 0) lcnt[tid >> 6] = spk;
    SliceItems si;
    si.init(bm);
    __syncthreads();
    int cGN = 0, cGF = 0, status = 0;
    double nv = 0.0;
    if (i < nc) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < DEG; ++k) {
            if (!((bm >> k) & 1u)) continue;
            const TA* src = lph + (int64_t)(item0 - it0 + si.rank(k)) * 4;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += (double)src[v];
        }
        update_cell_v<T, TA>(i, b, nc, ui, vi, acc, cdt, Unew, nv, cGN, cGF, status);
    }
    // photon sum, guards and status per slice; the face counts of the tile
    // to its first slice
    const int64_t sl = c0 / kSlice + tid / kSlice;
    if (sl * kSlice < nc) wave_partials(nv, 0, 0, 0, cGN, cGF, status, sl * nb + b, part_nv, part_cnt, part_status,
                                        n_blocks);
    if (tid == 0) {
        constexpr uint64_t kField = (1ull << 21) - 1;
        uint64_t c = 0;
        for (int w = 0; w < kTileThreads / 64; ++w) c += lcnt[w];
        add_counts(part_cnt, n_blocks, (t * kTileSlices) * nb + b, (int64_t)(c & kField),
                   (int64_t)((c >> 21) & kField), (int64_t)((c >> 42) & kField), 0, 0, 0, part_status);
    }
}

// ---------------------------------------------------------------------------
// k_transport: gradients, face states and fluxes of one 256-cell tile and
// one bin in a single launch, with the face states in LDS instead of HBM.
// The work items are the tile's cells (all their sides) and its halo cells
// (only their sides that face the tile); both go through the same code, so
// a face state is bit-identical in every tile that computes it and the two
// cells of a face still obtain fluxes of exactly opposite sign.
// ---------------------------------------------------------------------------

template <typename T, typename TA, int DEG>
__global__ __launch_bounds__(kTileThreads) void k_transport(const T* __restrict__ U, T* __restrict__ Unew, int64_t nc,
                                                      int nb, GeomView<T> geo, SellView sell, TileView tile,
                                                      int use_limiter, TA cdt, double* __restrict__ part_nv,
                                                      int64_t* __restrict__ part_cnt,
                                                      int32_t* __restrict__ part_status, int64_t n_blocks) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* lds = reinterpret_cast<T*>(lds_raw);
    const int64_t blk = xcd_logical_block();
    const int b = (int)(blk % nb);
    const int64_t t = blk / nb;
    const int64_t c0 = t * kTileCells;
    const int64_t e0 = sell.ptr[t * kTileSlices];
    const int64_t sl_end = (t + 1) * kTileSlices < tile.n_slices ? (t + 1) * kTileSlices : tile.n_slices;
    const int64_t tile_sides = (int64_t)sell.ptr[sl_end] - e0;
    const int32_t hq0 = tile.halo_ptr[t], hq1 = tile.halo_ptr[t + 1];
    const int32_t hs0 = tile.hside_ptr[hq0];
    const int64_t n_items = kTileCells + (hq1 - hq0);

    for (int64_t item = threadIdx.x; item < n_items; item += kTileThreads) {
        const bool own = item < kTileCells;
        const int64_t c = own ? c0 + item : (int64_t)tile.halo_cell[hq0 + (item - kTileCells)];
        if (c >= nc) continue;
        double uc[4], g[4][3];
        T rr[SlotCount<DEG>::kMax][3];
        bool ok[SlotCount<DEG>::kMax];
        if constexpr (DEG > 0) {
            CellSides<T, DEG> cs;
            load_cell_sides<T, DEG>(c, geo, sell, cs);
            T cell[8];
            load4(geo.cell + c * kCellRec, cell);
            load4(geo.cell + c * kCellRec + 4, cell + 4);
            limited_gradient_c<T, DEG>(c, b, nc, U, cell, cs, use_limiter, uc, g);
#pragma unroll
            for (int k = 0; k < DEG; ++k) {
                rr[k][0] = cs.r[k][0]; rr[k][1] = cs.r[k][1]; rr[k][2] = cs.r[k][2];
                ok[k] = cs.nbr[k] >= 0;
            }
        } else {
            limited_gradient_s<T, DEG>(c, b, nc, U, geo, sell, use_limiter, uc, g, rr, ok);
        }
        if (own) {
            export_face_states<T, DEG>(c, uc, g, rr, ok, geo, sell, lds, e0);
        } else {
            const int32_t sp = tile.hside_ptr[hq0 + (item - kTileCells)];
            const int32_t n_sides = tile.hside_ptr[hq0 + (item - kTileCells) + 1] - sp;
            for (int32_t q = 0; q < n_sides; ++q) {
                const int64_t e = tile.hside_entry[sp + q];
                T st[4];
                face_state<T>(uc, g, geo.sv(kSR0, e), geo.sv(kSR1, e), geo.sv(kSR2, e), st);
                store4(lds + (tile_sides + (sp + q - hs0)) * 4, st);
            }
        }
    }
    __syncthreads();

    int cAdmN = 0, cAdmF = 0, cCap = 0, cGN = 0, cGF = 0, status = 0;
    double nv = 0.0;
    const TileFaceStates<T> fsv{lds, e0, tile.lds_opp, U + (int64_t)b * nc * 4};
    const int64_t i = c0 + threadIdx.x;
    if (i < nc) {
        T ui[4];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        load4(U + urec(b, nc, i), ui);
        if constexpr (DEG == 6) {
            // the tile-interior faces first, then the cross-tile ones, each in
            // slot order: the order of the split path on six-slot meshes
            CellFaces<T, DEG> cf;
            load_cell_faces<T, DEG>(i, geo, sell, cf);
            const int64_t base = (int64_t)sell.ptr[i / kSlice] + (i % kSlice);
            const uint32_t bm = tile.bmask ? tile.bmask[i] : 0u;     // none: the per-slice kernels' slot order
            TA prod[DEG][4];
            cell_flux_sum_c<T, TA, DEG>(i, b, nc, U, fsv, base, cf, cdt, (TA)ui[0], acc, cAdmN, cAdmF, cCap, prod);
#pragma unroll
            for (int k = 0; k < DEG; ++k) {
                if (cf.nbr[k] < 0 || ((bm >> k) & 1u)) continue;
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] += (double)prod[k][v];
            }
            if (tile.bmask) {
                // as the split path by tile: the cell updated by its
                // tile-interior faces and rounded, then by the others
                T w[4];
                partial_update<T, TA>(ui, geo.cell[i * kCellRec + 6], acc, cdt, w);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    ui[v] = w[v];
                    acc[v] = 0.0;
                }
#pragma unroll
                for (int k = 0; k < DEG; ++k) {
                    if (cf.nbr[k] < 0 || !((bm >> k) & 1u)) continue;
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[v] += (double)prod[k][v];
                }
            }
        } else if constexpr (DEG > 0) {
            CellFaces<T, DEG> cf;
            load_cell_faces<T, DEG>(i, geo, sell, cf);
            cell_flux_sum_c<T, TA, DEG>(i, b, nc, U, fsv, (int64_t)sell.ptr[i / kSlice] + (i % kSlice), cf, cdt,
                                        (TA)ui[0], acc, cAdmN, cAdmF, cCap);
        } else {
            cell_flux_sum_s<T, TA, DEG>(i, b, nc, U, fsv, geo, sell, cdt, (TA)ui[0], acc, cAdmN, cAdmF, cCap);
        }
        update_cell<T, TA>(i, b, nc, ui, acc, cdt, geo, Unew, nv, cGN, cGF, status);
    }
    // Partials go to the slot of the tile's first 256-cell block, so that
    // they are laid out as those of the split kernels.
    block_partials<kTileThreads>(nv, cAdmN, cAdmF, cCap, cGN, cGF, status, (t * kTileBlocks) * nb + b, part_nv,
                                 part_cnt, part_status, n_blocks);
}

// ---------------------------------------------------------------------------
// k_reduce: the per-block partials folded in a fixed order into the
// diagnostics record (deterministic).
// ---------------------------------------------------------------------------

// Two stages: kReduceBlocks workgroups fold fixed, contiguous ranges of the
// partials into one record each, then one workgroup folds those records.
// The partition and the order of every sum are fixed, so the diagnostics
// are reproducible bit for bit.
__global__ __launch_bounds__(kBlock) void k_reduce_part(const double* __restrict__ part_nv,
                                                        const int64_t* __restrict__ part_cnt,
                                                        const int32_t* __restrict__ part_fstatus, int64_t n_fblocks,
                                                        int nb, const int64_t* __restrict__ chem_sum,
                                                        const int64_t* __restrict__ chem_max,
                                                        const int32_t* __restrict__ chem_status, int64_t n_cblocks,
                                                        DiagDev* __restrict__ parts) {
    __shared__ double ldsd[kBlock / 64];
    __shared__ int64_t ldsi[kBlock / 64];
    __shared__ int ldss[kBlock / 64];
    const int64_t g = blockIdx.x;
    const int64_t rows = n_fblocks / nb;                  // 256-cell blocks
    const int64_t rper = (rows + kReduceBlocks - 1) / kReduceBlocks;
    const int64_t r0 = g * rper < rows ? g * rper : rows, r1 = r0 + rper < rows ? r0 + rper : rows;
    const int64_t cper = (n_cblocks + kReduceBlocks - 1) / kReduceBlocks;
    const int64_t q0 = g * cper < n_cblocks ? g * cper : n_cblocks;
    const int64_t q1 = q0 + cper < n_cblocks ? q0 + cper : n_cblocks;
    DiagDev& o = parts[g];
    for (int b = 0; b < nb; ++b) {
        double sm = 0.0;
        for (int64_t k = r0 + threadIdx.x; k < r1; k += kBlock) sm += part_nv[k * nb + b];
        sm = block_sum<double>(sm, ldsd);
        if (threadIdx.x == 0) o.photon_sum[b] = sm;
    }
    for (int c = 0; c < 5; ++c) {
        int64_t sm = 0;
        for (int64_t k = r0 * nb + threadIdx.x; k < r1 * nb; k += kBlock) sm += part_cnt[c * n_fblocks + k];
        sm = block_sum<int64_t>(sm, ldsi);
        if (threadIdx.x == 0) o.counters[c] = sm;
    }
    int st = 0;
    for (int64_t k = r0 * nb + threadIdx.x; k < r1 * nb; k += kBlock) st |= part_fstatus[k];
    for (int64_t k = q0 + threadIdx.x; k < q1; k += kBlock) st |= chem_status[k];
    st = block_or(st, ldss);
    int64_t cs = 0, cm = 0;
    for (int64_t k = q0 + threadIdx.x; k < q1; k += kBlock) {
        cs += chem_sum[k];
        cm = chem_max[k] > cm ? chem_max[k] : cm;
    }
    cs = block_sum<int64_t>(cs, ldsi);
    cm = block_max<int64_t>(cm, ldsi);
    if (threadIdx.x == 0) {
        o.status = st;
        o.substeps = cs;
        o.max_substeps = cm;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce(const DiagDev* __restrict__ parts, int nb,
                                                   const double* __restrict__ nv_scale /*[nb] scale*h^3*/,
                                                   DiagDev* __restrict__ out) {
    __shared__ double ldsd[kBlock / 64];
    __shared__ int64_t ldsi[kBlock / 64];
    __shared__ int ldss[kBlock / 64];
    const int k = threadIdx.x;
    const bool in = k < kReduceBlocks;
    for (int b = 0; b < nb; ++b) {
        const double sm = block_sum<double>(in ? parts[k].photon_sum[b] : 0.0, ldsd);
        if (threadIdx.x == 0) out->photon_sum[b] = sm * nv_scale[b];
    }
    for (int c = 0; c < 5; ++c) {
        const int64_t sm = block_sum<int64_t>(in ? parts[k].counters[c] : 0, ldsi);
        if (threadIdx.x == 0) out->counters[c] = sm;
    }
    const int st = block_or(in ? parts[k].status : 0, ldss);
    const int64_t cs = block_sum<int64_t>(in ? parts[k].substeps : 0, ldsi);
    const int64_t cm = block_max<int64_t>(in ? parts[k].max_substeps : 0, ldsi);
    if (threadIdx.x == 0) {
        out->status = st;
        out->substeps = cs;
        out->max_substeps = cm;
    }
}

// ---------------------------------------------------------------------------
// CFL length: min_i (3 V_i / 4 pi)^(1/3) by a two-pass wave64 min-reduction.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_min_cfl_length(const double* __restrict__ vphys, int64_t nc,
                                                           double* __restrict__ part) {
    __shared__ double lds[kBlock / 64];
    double m = INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nc; i += (int64_t)gridDim.x * kBlock)
        m = fmin(m, cbrt(3.0 * vphys[i] / (4.0 * M_PI)));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / 64; ++k) m = fmin(m, lds[k]);
        part[blockIdx.x] = fmin(m, lds[0]);
    }
}

// ---------------------------------------------------------------------------
// Field conversion between the caller's FP64 layout and the internal one.
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_get_fields(const T* __restrict__ U, const double* __restrict__ X, const double* __restrict__ Ue,
                             int64_t nc, int nb, int field, const double* __restrict__ scale, double c_red,
                             ChemParams P, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    if (field == 0) {
        for (int b = 0; b < nb; ++b) out[(int64_t)b * nc + i] = (double)U[urec(b, nc, i)] * scale[b];
    } else if (field == 1) {
        for (int b = 0; b < nb; ++b)
            for (int k = 0; k < 3; ++k)
                out[(int64_t)(b * 3 + k) * nc + i] = (double)U[urec(b, nc, i) + 1 + k] * scale[b] * c_red;
    } else if (field == 4) {
        double x[5];
        for (int s = 0; s < 5; ++s) x[s] = X[(int64_t)s * nc + i];
        out[i] = P.isothermal ? P.T_iso : temperature(P, Ue[i], x);
    }
}

template <typename T>
__global__ void k_set_fields(T* __restrict__ U, const double* __restrict__ X, double* __restrict__ Ue, int64_t nc,
                             int nb, int field, const double* __restrict__ inv_scale, double c_red, ChemParams P,
                             const double* __restrict__ in) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    if (field == 0) {
        for (int b = 0; b < nb; ++b) U[urec(b, nc, i)] = (T)(in[(int64_t)b * nc + i] * inv_scale[b]);
    } else if (field == 1) {
        for (int b = 0; b < nb; ++b)
            for (int k = 0; k < 3; ++k)
                U[urec(b, nc, i) + 1 + k] = (T)(in[(int64_t)(b * 3 + k) * nc + i] / c_red * inv_scale[b]);
    } else if (field == 4) {
        // thermal energy from T and the current fractions
        double x[5];
        for (int s = 0; s < 5; ++s) x[s] = X[(int64_t)s * nc + i];
        Ue[i] = kBoltz * in[i] / (P.gm1 * mean_mass(P, x) * kProtonMass);
    }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------

static inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

void fill_words(void* p, int64_t n_words, uint32_t v, hipStream_t s) {
    if (n_words <= 0) return;
    hipLaunchKernelGGL(k_fill_bytes, dim3(grid_for(n_words, 256)), dim3(256), 0, s, (uint32_t*)p, n_words, v);
}

template <typename T>
void launch_sources(T* U, int64_t nc, int nb, int32_t n_cells_src, const int32_t* cell, const int32_t* ptr,
                    const double* rate, int64_t n_src, const double* vphys, const double* inv_scale,
                    const double* scale, double dt, hipStream_t s) {
    if (n_cells_src <= 0) return;
    hipLaunchKernelGGL(k_sources<T>, dim3(grid_for(n_cells_src, 64)), dim3(64), 0, s, U, nc, nb, n_cells_src, cell,
                       ptr, rate, n_src, vphys, inv_scale, scale, dt);
}

// Cells per lane of k_chem: as asked, else up to 32 while keeping at least
// about 1024 workgroups.  Longer chunks spread each workgroup's start and
// its slowest cells over more work (on 16.8M cells, 8 cells a lane took
// 1.47 ms, 32 took 1.37 ms).
int chem_chunk(int64_t nc, int per_lane) {
    if (per_lane > 0) return per_lane;
    int64_t c = nc / ((int64_t)kBlock * 1024);
    return (int)(c < 1 ? 1 : (c > 32 ? 32 : c));
}

template <typename T, int NB>
static void launch_chem_nb(T* U, double* X, double* Ue, const double* nH, int64_t nc, int64_t cell0, int64_t cell1,
                           const ChemParams& P, double dt, const double* scale, const double* inv_scale, int64_t* ps,
                           int64_t* pm, int32_t* pst, int32_t* att, hipStream_t s) {
    const int64_t n = cell1 - cell0;
    if (n <= 0) return;
    const int chunk = chem_chunk(n, P.cells_per_lane);
    hipLaunchKernelGGL((k_chem<NB, T>), dim3((unsigned)chem_blocks(n, P.cells_per_lane)), dim3(kBlock), 0, s, U, X, Ue,
                       nH, nc, cell0,
                       cell1, chunk, P, dt, scale, inv_scale, ps, pm, pst, att);
}

template <typename T>
void launch_chem(T* U, double* X, double* Ue, const double* nH, int64_t nc, int64_t cell0, int64_t cell1,
                 const ChemParams& P, double dt, const double* scale, const double* inv_scale, int64_t* ps,
                 int64_t* pm, int32_t* pst, int32_t* att, hipStream_t s) {
    switch (P.nb) {
#define RT_CHEM_CASE(K) \
    case K: launch_chem_nb<T, K>(U, X, Ue, nH, nc, cell0, cell1, P, dt, scale, inv_scale, ps, pm, pst, att, s); break;
        RT_CHEM_CASE(1) RT_CHEM_CASE(2) RT_CHEM_CASE(3) RT_CHEM_CASE(4)
        RT_CHEM_CASE(5) RT_CHEM_CASE(6) RT_CHEM_CASE(7) RT_CHEM_CASE(8)
#undef RT_CHEM_CASE
        default: break;
    }
}

int64_t chem_blocks(int64_t nc, int per_lane) {
    return (int64_t)grid_for(nc, (int64_t)kBlock * chem_chunk(nc, per_lane));
}
int64_t transport_blocks(int64_t nc, int nb) { return (int64_t)grid_for(nc, kBlock) * nb; }
int64_t partial_blocks(int64_t nc, int nb) { return (int64_t)grid_for(nc, kFluxBlock) * nb; }

// The transport kernels are specialised for meshes whose slices all have 6
// slots (lattices) or 14 (the staggered BCC mesh); other meshes take the
// general form.
#define RT_DEG_DISPATCH(deg, CALL) \
    switch (deg) {                 \
        case 6: CALL(6); break;    \
        case 14: CALL(14); break;  \
        default: CALL(0); break;   \
    }

template <typename T>
void launch_facestate(const T* U, T* FV, T* NC, int64_t nc, int nb, int64_t n_entries, const GeomView<T>& geo,
                      const SellView& sell, int use_limiter, hipStream_t s) {
#define RT_CALL(D)                                                                                             \
    hipLaunchKernelGGL((k_facestate<T, D>), dim3((unsigned)transport_blocks(nc, nb)), dim3(kBlock), 0, s, U, FV,    \
                       NC, nc, nb, n_entries, geo, sell, use_limiter)
    RT_DEG_DISPATCH(sell.uniform_deg, RT_CALL)
#undef RT_CALL
}

void launch_gradient(const double* U, double* G, int64_t nc, int nb, const GeomView<double>& geo, const SellView& sell,
                     int use_limiter, hipStream_t s) {
    hipLaunchKernelGGL(k_gradient, dim3((unsigned)transport_blocks(nc, nb)), dim3(kBlock), 0, s, U, G, nc, nb, geo,
                       sell, use_limiter);
}

template <typename T>
void launch_flux(const T* U, const T* FV, const T* NC, T* Unew, int64_t nc, int nb, int64_t n_entries,
                 const GeomView<T>& geo, const SellView& sell, double cdt, double* part_nv, int64_t* part_cnt,
                 int32_t* part_status, int64_t slice0, int64_t slice1, hipStream_t s) {
    const int64_t nblk = partial_blocks(nc, nb);          // partial slots of the whole mesh
    const int64_t grid = (slice1 - slice0) * nb;
    if (grid <= 0) return;
    switch (sell.uniform_deg) {
#define RT_CALL(D)                                                                                               \
    hipLaunchKernelGGL((k_flux_pairs<T, T, D>), dim3((unsigned)grid), dim3(kFluxPairThreads), 0, s, U, FV, NC, Unew, \
                       nc, nb, n_entries, geo, sell, (T)cdt, part_nv, part_cnt, part_status, nblk, slice0)
        case 6: RT_CALL(6); break;
        case 14: RT_CALL(14); break;
#undef RT_CALL
        default:
            hipLaunchKernelGGL((k_flux<T, T>), dim3((unsigned)grid), dim3(kFluxBlock), 0, s, U, FV, NC, Unew, nc, nb,
                               n_entries, geo, sell, (T)cdt, part_nv, part_cnt, part_status, nblk, slice0);
            break;
    }
}

template <typename T>
void launch_facestate_tile(const T* U, T* BS, T* BN, T* Unew, int64_t nc, int nb, const GeomView<T>& geo,
                           const SellView& sell, const TileFaceView& tf, int use_limiter, double cdt,
                           int64_t* part_cnt, int32_t* part_status, hipStream_t s) {
    const int64_t nblk = partial_blocks(nc, nb);
    const int64_t grid = (int64_t)grid_for(nc, kTileCells) * nb;
    hipLaunchKernelGGL((k_facestate_tile<T, T>), dim3((unsigned)grid), dim3(kTileThreads), 0, s, U, BS, BN, Unew, nc,
                       nb, geo, sell, tf, use_limiter, (T)cdt, part_cnt, part_status, nblk);
}

template <typename T>
void launch_flux_tile(const T* BS, const T* BN, T* Unew, int64_t nc, int nb, const T* vol, const T* bgeo,
                      const TileFaceView& tf, double cdt, double* part_nv, int64_t* part_cnt, int32_t* part_status,
                      hipStream_t s) {
    const int64_t nblk = partial_blocks(nc, nb);
    const int64_t grid = (int64_t)grid_for(nc, kTileCells) * nb;
    const size_t lds = (size_t)(tf.bnd_max > 0 ? tf.bnd_max : 1) * 4 * sizeof(T);   // at most 6 kTileCells items
    hipLaunchKernelGGL((k_flux_tile<T, T>), dim3((unsigned)grid), dim3(kTileThreads), lds, s, BS, BN, Unew, nc, nb,
                       vol, bgeo, tf, (T)cdt, part_nv, part_cnt, part_status, nblk);
}

template <typename T, int D>
static void launch_transport_deg(const T* U, T* Unew, int64_t nc, int nb, const GeomView<T>& geo,
                                 const SellView& sell, const TileView& tile, size_t lds_bytes, int use_limiter,
                                 double cdt, double* part_nv, int64_t* part_cnt, int32_t* part_status, hipStream_t s) {
    const int64_t nblk = partial_blocks(nc, nb);                // partial slots
    const int64_t ntile_blk = (int64_t)grid_for(nc, kTileCells) * nb;
    if (lds_bytes > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_transport<T, T, D>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    hipLaunchKernelGGL((k_transport<T, T, D>), dim3((unsigned)ntile_blk), dim3(kTileThreads), lds_bytes, s, U, Unew, nc, nb,
                       geo, sell, tile, use_limiter, (T)cdt, part_nv, part_cnt, part_status, nblk);
}

template <typename T>
void launch_transport(const T* U, T* Unew, int64_t nc, int nb, const GeomView<T>& geo, const SellView& sell,
                      const TileView& tile, size_t lds_bytes, int use_limiter, double cdt, double* part_nv,
                      int64_t* part_cnt, int32_t* part_status, hipStream_t s) {
#define RT_CALL(D)                                                                                            \
    launch_transport_deg<T, D>(U, Unew, nc, nb, geo, sell, tile, lds_bytes, use_limiter, cdt, part_nv, part_cnt, \
                               part_status, s)
    RT_DEG_DISPATCH(sell.uniform_deg, RT_CALL)
#undef RT_CALL
}

void launch_reduce(const double* part_nv, const int64_t* part_cnt, const int32_t* part_fstatus, int64_t n_fblocks,
                   int nb, const int64_t* chem_sum, const int64_t* chem_max, const int32_t* chem_status,
                   int64_t n_cblocks, const double* nv_scale, DiagDev* parts, DiagDev* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_part, dim3(kReduceBlocks), dim3(kBlock), 0, s, part_nv, part_cnt, part_fstatus,
                       n_fblocks, nb, chem_sum, chem_max, chem_status, n_cblocks, parts);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, parts, nb, nv_scale, out);
}

int64_t cfl_partials(int64_t nc) {
    int64_t g = grid_for(nc, kBlock);
    return g < 1024 ? g : 1024;
}

void launch_min_cfl_length(const double* vphys, int64_t nc, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_min_cfl_length, dim3((unsigned)cfl_partials(nc)), dim3(kBlock), 0, s, vphys, nc, part);
}

template <typename T>
void launch_get_fields(const T* U, const double* X, const double* Ue, int64_t nc, int nb, int field,
                       const double* scale, double c_red, const ChemParams& P, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_get_fields<T>, dim3(grid_for(nc, 256)), dim3(256), 0, s, U, X, Ue, nc, nb, field, scale,
                       c_red, P, out);
}

template <typename T>
void launch_set_fields(T* U, const double* X, double* Ue, int64_t nc, int nb, int field, const double* inv_scale,
                       double c_red, const ChemParams& P, const double* in, hipStream_t s) {
    hipLaunchKernelGGL(k_set_fields<T>, dim3(grid_for(nc, 256)), dim3(256), 0, s, U, X, Ue, nc, nb, field, inv_scale,
                       c_red, P, in);
}

#define RT_INSTANTIATE(T)                                                                                          \
    template void launch_sources<T>(T*, int64_t, int, int32_t, const int32_t*, const int32_t*, const double*,       \
                                    int64_t, const double*, const double*, const double*, double, hipStream_t);    \
    template void launch_chem<T>(T*, double*, double*, const double*, int64_t, int64_t, int64_t, const ChemParams&,  \
                                 double, const double*, const double*, int64_t*, int64_t*, int32_t*, int32_t*,     \
                                 hipStream_t);                                                                      \
    template void launch_facestate<T>(const T*, T*, T*, int64_t, int, int64_t, const GeomView<T>&, const SellView&, int, \
                                      hipStream_t);                                                                \
    template void launch_facestate_tile<T>(const T*, T*, T*, T*, int64_t, int, const GeomView<T>&,                \
                                           const SellView&, const TileFaceView&, int, double, int64_t*, int32_t*,  \
                                           hipStream_t);                                                           \
    template void launch_flux_tile<T>(const T*, const T*, T*, int64_t, int, const T*, const T*,                    \
                                      const TileFaceView&, double, double*, int64_t*, int32_t*, hipStream_t);      \
    template void launch_flux<T>(const T*, const T*, const T*, T*, int64_t, int, int64_t, const GeomView<T>&, const SellView&, \
                                 double, double*, int64_t*, int32_t*, int64_t, int64_t, hipStream_t);               \
    template void launch_transport<T>(const T*, T*, int64_t, int, const GeomView<T>&, const SellView&,             \
                                      const TileView&, size_t, int, double, double*, int64_t*, int32_t*,           \
                                      hipStream_t);                                                                \
    template void launch_get_fields<T>(const T*, const double*, const double*, int64_t, int, int, const double*,   \
                                       double, const ChemParams&, double*, hipStream_t);                           \
    template void launch_set_fields<T>(T*, const double*, double*, int64_t, int, int, const double*, double,       \
                                       const ChemParams&, const double*, hipStream_t);

RT_INSTANTIATE(double)
RT_INSTANTIATE(float)

}  // namespace rtk
