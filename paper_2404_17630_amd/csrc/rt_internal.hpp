// Internal host-side structures of the M1 radiative-transfer library.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <utility>
#include <vector>

#include "rt.h"
#include "rt_kernels.hpp"
#include "rt_types.hpp"

// Sets the thread-local error message and returns `code`.
int rt_fail(int code, const char* fmt, ...);

// Return RT_ENOMEM or RT_EDEVICE with a message when a HIP call fails.
#define RT_HIP(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) {                                                                        \
            int code_ = (e_ == hipErrorOutOfMemory) ? RT_ENOMEM : RT_EDEVICE;                          \
            return rt_fail(code_, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
        }                                                                                              \
    } while (0)

// Makes `dev` the current device for a scope and restores the previous one.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (dev < 0) return;    // host-only mesh: no device to select
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Owning device allocation.
struct DevMem {
    void* ptr = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() { release(); }
    int alloc(size_t nbytes);
    int upload(const void* src, size_t nbytes);
    void release();
};

struct rt_mesh {
    int device = 0;
    int64_t nc = 0, nf = 0;
    double h_ref = 1.0;          // length unit of the stored geometry: <V>^(1/3)
    double dx_min = 0.0;         // min_i (3 V_i / 4 pi)^(1/3), cm
    int32_t max_deg = 0;
    std::atomic<int> refs{0};
    // Host copies (FP64, units of h_ref).
    std::vector<double> face;    // [nf][kFaceRec]: A, n, rL, rR, vcap_L, vcap_R
    std::vector<double> cell;    // [nc][kCellRec]: M^-1 (xx yy zz xy xz yz), V, vcap
    std::vector<double> vphys;   // [nc] cm^3
    std::vector<int32_t> deg;    // faces per cell
    std::vector<int32_t> nbr, fsf, opp, sptr, sdeg;   // sliced ELL
    int64_t n_entries = 0;       // sliced-ELL slots (face sides plus padding)
    // Device copies.
    DevMem d_face64, d_cell64, d_vphys;
    DevMem d_face32, d_cell32;
    bool geo32_ready = false;
    DevMem d_side32, d_side64;   // per face side records (rtk::SideComp), built on first use
    int32_t uniform_deg = 0;     // rtk::SellView::uniform_deg
    DevMem d_nbr, d_fsf, d_opp, d_sptr, d_sdeg, d_idx;
    DevMem d_vol32, d_vol64;     // [nc] V in units of h_ref^3
    // Tiles of the fused transport kernel (rtk::TileView).
    std::vector<int32_t> lds_opp, halo_ptr, halo_cell, hside_ptr, hside_entry;
    int64_t tile_max_sides = 0;  // largest tile + halo side count
    double halo_ratio = 0.0;     // halo cells / cells, over all tiles
    size_t lds_limit = 0;        // LDS bytes a workgroup may use on the device
    DevMem d_lds_opp, d_halo_ptr, d_halo_cell, d_hside_ptr, d_hside_entry;

    // Face evaluations of the flux kernel on uniform-degree meshes: per
    // slice, the entries whose face is evaluated there, fitem_ptr [n_slices
    // + 1] into the pairs of fitem: the entry, with kFluxPairBit set when the
    // face's other side is in the same slice and takes the negated result,
    // and the signed opposite entry (opp for an L side, ~opp for an R side).
    std::vector<int32_t> fitem_ptr, fitem;
    DevMem d_fitem_ptr, d_fitem;
    // Faces of the split transport on six-slot meshes, per kTileCells-cell
    // tile (rtk::TileFaceView): the faces with both sides in the tile
    // (tpair: L and R entries relative to the tile's first entry, 16 bits
    // each); the face sides whose face crosses to another tile, numbered in
    // entry order ("boundary items"; tbnd: entry and the opposite side's item,
    // complemented for an R side), with the first item of every tile
    // (tbnd_ptr) and of every slice (tbnd_sptr); per cell the slots of such
    // faces (bmask).  The device keeps the opposite items only (d_tbnd_opp)
    // and each item's face area and normal in the transport precision
    // (d_bgeo32/64: A, n_x, n_y, n_z).
    std::vector<int32_t> tpair_ptr, tpair, tbnd_ptr, tbnd, tbnd_sptr;
    std::vector<uint8_t> bmask;
    int64_t tbnd_max = 0;        // most boundary items of one tile
    DevMem d_tpair_ptr, d_tpair, d_tbnd_ptr, d_tbnd_opp, d_tbnd_sptr, d_bmask, d_bgeo32, d_bgeo64;
    int64_t n_bnd() const { return (int64_t)tbnd.size() / 2; }

    int build_float_geometry();
    void build_flux_items();
    void build_tile_faces();
    int build_side_geometry(size_t tbytes);
    void build_tiles();
    size_t tile_lds_bytes(size_t tbytes) const { return (size_t)tile_max_sides * 4 * tbytes; }
};

void rt_mesh_release(rt_mesh* m);

// Where the kernels of a call write their per-block partials and the
// diagnostics record: normally the state's own buffers; rt_subcycle_noalloc
// points them into its static device array for the duration of its call.
struct PartialBufs {
    double* nv = nullptr;          // [n_fblk] photon sums of the flux workgroups
    int64_t* cnt = nullptr;        // [5][n_fblk] admissibility, cap and guard counts
    int32_t* fst = nullptr;        // [n_fblk] status bits of the flux workgroups
    int64_t* csum = nullptr;       // [n_cblk] chemistry attempts
    int64_t* cmax = nullptr;       // [n_cblk] largest attempts of one cell
    int32_t* cst = nullptr;        // [n_cblk] status bits of the chemistry workgroups
    rtk::DiagDev* red = nullptr;   // [kReduceBlocks] first-stage reduction records
    rtk::DiagDev* diag = nullptr;  // the folded diagnostics record
};
// Bytes of the partials above for n_fblk flux and n_cblk chemistry
// workgroups, each array starting on a 256-byte boundary.
size_t rt_partial_bytes(int64_t n_fblk, int64_t n_cblk);
// Carve the partials out of `base` (rt_partial_bytes bytes, 256-byte aligned).
PartialBufs rt_partials_at(void* base, int64_t n_fblk, int64_t n_cblk);

struct rt_state {
    rt_mesh* mesh = nullptr;
    rt_params params{};
    rtk::ChemParams cp{};
    int precision = RT_FP64;
    int transport_mode = RT_TRANSPORT_AUTO;
    int nb = 1;
    int64_t nc = 0;
    double dt_cfl = 0.0;

    // Fields: U[b][nc][4] = (N, Fh_x, Fh_y, Fh_z) / scale_b in the transport
    // precision, double-buffered; face states FV[b][entry][4] followed by
    // the cells' cap numerators N V / n_faces [b][nc] (split path only,
    // allocated with the state); chemistry FP64.
    DevMem U[2];
    int cur = 0;
    DevMem FV;
    DevMem X, Ue, nH;            // [5][nc], [nc], [nc]
    DevMem att;                  // [nc] int32 chemistry attempts of each cell in the current call
    double scale[RT_MAX_BINS];
    DevMem d_scale, d_inv_scale, d_nv_scale;

    // Sources (original order on the host; sorted by cell on the device).
    int64_t n_src = 0;
    std::vector<int64_t> src_cell;
    std::vector<double> src_rate;    // [nb][n_src]
    int32_t n_src_cells = 0;
    DevMem d_src_cell, d_src_ptr, d_src_rate, d_src_vphys;

    // Per-block partials and the diagnostics record.
    int64_t n_fblk = 0, n_cblk = 0;
    DevMem part_mem;             // the state's own partials (rt_partial_bytes)
    PartialBufs pb;              // the buffers the kernels use (part_mem unless redirected)
    rtk::DiagDev* h_diag = nullptr;
    rt_diag diag{};

    // Entry copy for roll-back on error.
    DevMem bU, bX, bUe;

    // Profiling.
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    int prof_open = -1;
    int prof_kernel = 0;
    std::vector<std::pair<int, int>> ev_marks;
    int64_t launches[RT_N_KERNELS] = {0, 0, 0, 0, 0, 0};
    double total_ms[RT_N_KERNELS] = {0, 0, 0, 0, 0, 0};

    ~rt_state();
    bool fused() const;
    size_t tbytes() const;
    int ensure_face_states();
    int alloc_buffers();
    int upload_scales();
    int upload_sources();
    void prof_begin(int kernel, hipStream_t st);
    void prof_end(hipStream_t st);
    int prof_collect();
};

// Pieces of a subcycle on explicit buffers (U, G in the state's precision);
// used by rt_subcycle and by the adjoint's recomputation.
rtk::GeomView<double> rt_geo64(const rt_mesh* m);
rtk::SellView rt_sell(const rt_mesh* m);
void rt_step_sources(rt_state* s, void* U, double dt, hipStream_t st, int32_t src0 = 0, int32_t src1 = -1);
void rt_step_chem(rt_state* s, void* U, double* X, double* Ue, double dt, hipStream_t st, int64_t cell0 = 0,
                  int64_t cell1 = -1, int64_t cblk0 = 0);
// Face states of the split path; where the mesh has tile tables also the
// tile-interior faces' fluxes, with every cell updated by them into Un,
// unless all_states asks for every face state in FV (the adjoint's reverse
// sweep; Un is unused, and rt_step_flux must not follow it then).
// rt_step_flux then updates the whole mesh into Un.
void rt_step_facestate(rt_state* s, const void* U, void* FV, void* Un, hipStream_t st, double dt, bool all_states);
void rt_step_flux(rt_state* s, const void* U, const void* FV, void* Un, double dt, hipStream_t st);
void rt_step_transport(rt_state* s, const void* U, void* Un, double dt, hipStream_t st);
rtk::TileView rt_tiles(const rt_mesh* m);
void rt_run_subcycles(rt_state* s, int n, double dt, hipStream_t st);
void rt_reset_partials(rt_state* s, hipStream_t st);
// Folds the partials and returns the status word (synchronises the stream).
int rt_read_status(rt_state* s, hipStream_t st, int* status);
// Body of rt_subcycle after argument checks: n subcycles of length `step`,
// the diagnostics fold and read-back into s->diag.  With `rollback` the
// fields are copied at entry (into buffers the state allocates on first use)
// and restored on RT_ENUMERIC; without it nothing is allocated and a failed
// call leaves the state as the failing subcycle left it.
int rt_subcycle_run(rt_state* s, int n, double step, hipStream_t st, bool rollback);
