// Launchers of the M1 radiative-transfer kernels (rt_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt_types.hpp"

namespace rtk {

// Diagnostics record written by k_reduce.
struct DiagDev {
    double photon_sum[kMaxBins];
    int64_t counters[5];     // adm_N, adm_F, flux_caps, guard_N, guard_F
    int64_t substeps;
    int64_t max_substeps;
    int32_t status;
    int32_t pad_;
};

// Workgroups of the first stage of the diagnostics reduction (one DiagDev
// record each; no more than the threads of one workgroup).
constexpr int kReduceBlocks = 256;
static_assert(kReduceBlocks <= kBlock, "the second stage folds one record per thread");

void fill_words(void* p, int64_t n_words, uint32_t v, hipStream_t s);

// Cells per lane of k_chem over nc cells (per_lane > 0: that many), and its
// workgroup count.
constexpr int kMaxChemCellsPerLane = 1024;
int chem_chunk(int64_t nc, int per_lane);
int64_t chem_blocks(int64_t nc, int per_lane);
int64_t transport_blocks(int64_t nc, int nb);   // workgroups of kBlock cells, times nb
int64_t partial_blocks(int64_t nc, int nb);     // per-block partial slots (kFluxBlock cells), times nb
int64_t cfl_partials(int64_t nc);

template <typename T>
void launch_sources(T* U, int64_t nc, int nb, int32_t n_cells_src, const int32_t* cell, const int32_t* ptr,
                    const double* rate, int64_t n_src, const double* vphys, const double* inv_scale,
                    const double* scale, double dt, hipStream_t s);

// Cells [cell0, cell1) of the mesh's nc; the partial arrays start at the
// range's first chemistry workgroup (chem_blocks(cell1 - cell0) of them).
template <typename T>
void launch_chem(T* U, double* X, double* Ue, const double* nH, int64_t nc, int64_t cell0, int64_t cell1,
                 const ChemParams& P, double dt, const double* scale, const double* inv_scale, int64_t* part_sum,
                 int64_t* part_max, int32_t* part_status, int32_t* att_cell /*[nc] attempts of each cell, accumulated*/,
                 hipStream_t s);

// FV[b][e][4]: face states; NC[b][nc]: each cell's N V / n_faces (the
// numerator of the outflow cap, one product of the stored N and V / n_faces),
// which launch_flux gathers instead of a 16-byte field record and a side
// record of V / n_faces.
template <typename T>
void launch_facestate(const T* U, T* FV, T* NC, int64_t nc, int nb, int64_t n_entries, const GeomView<T>& geo,
                      const SellView& sell, int use_limiter, hipStream_t s);

void launch_gradient(const double* U, double* G, int64_t nc, int nb, const GeomView<double>& geo, const SellView& sell,
                     int use_limiter, hipStream_t s);

// Split transport on six-slot meshes by tile (see k_facestate_tile): the
// face states of cross-tile faces to BS [nb][n_bnd][4] and their cells' cap
// numerators to BN [nb][n_bnd], by boundary item; every cell updated by its
// tile-interior faces to Unew; then the cross-tile fluxes and the rest of
// the update, in place in Unew.  bgeo [n_bnd][4]: A, n of each boundary
// item.
template <typename T>
void launch_facestate_tile(const T* U, T* BS, T* BN, T* Unew, int64_t nc, int nb, const GeomView<T>& geo,
                           const SellView& sell, const TileFaceView& tf, int use_limiter, double cdt,
                           int64_t* part_cnt, int32_t* part_status, hipStream_t s);
template <typename T>
void launch_flux_tile(const T* BS, const T* BN, T* Unew, int64_t nc, int nb, const T* vol, const T* bgeo,
                      const TileFaceView& tf, double cdt, double* part_nv, int64_t* part_cnt, int32_t* part_status,
                      hipStream_t s);

// Slices [slice0, slice1); the partial arrays are those of the whole mesh.
template <typename T>
void launch_flux(const T* U, const T* FV, const T* NC, T* Unew, int64_t nc, int nb, int64_t n_entries,
                 const GeomView<T>& geo, const SellView& sell, double cdt, double* part_nv, int64_t* part_cnt,
                 int32_t* part_status, int64_t slice0, int64_t slice1, hipStream_t s);

template <typename T>
void launch_transport(const T* U, T* Unew, int64_t nc, int nb, const GeomView<T>& geo, const SellView& sell,
                      const TileView& tile, size_t lds_bytes, int use_limiter, double cdt, double* part_nv,
                      int64_t* part_cnt, int32_t* part_status, hipStream_t s);

void launch_reduce(const double* part_nv, const int64_t* part_cnt, const int32_t* part_fstatus, int64_t n_fblocks,
                   int nb, const int64_t* chem_sum, const int64_t* chem_max, const int32_t* chem_status,
                   int64_t n_cblocks, const double* nv_scale, DiagDev* parts, DiagDev* out, hipStream_t s);

void launch_min_cfl_length(const double* vphys, int64_t nc, double* part, hipStream_t s);

template <typename T>
void launch_get_fields(const T* U, const double* X, const double* Ue, int64_t nc, int nb, int field,
                       const double* scale, double c_red, const ChemParams& P, double* out, hipStream_t s);

template <typename T>
void launch_set_fields(T* U, const double* X, double* Ue, int64_t nc, int nb, int field, const double* inv_scale,
                       double c_red, const ChemParams& P, const double* in, hipStream_t s);

}  // namespace rtk
