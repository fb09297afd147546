// Device-side parameter blocks and launch helpers shared by the kernels and
// the host driver of the M1 radiative-transfer library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtk {

constexpr int kMaxBins = 8;
constexpr int kBlock = 256;          // threads per workgroup (four wave64s)
constexpr int kSlice = 64;           // cells per SELL slice = one wavefront
constexpr int kMaxCellFaces = 4096;    // faces a cell may have (rt_mesh_create rejects more)
constexpr int kNumXcd = 8;           // MI355X: 8 XCDs, workgroups dispatched round-robin

// Chemistry constants (from rt_params).
struct ChemParams {
    int nb, chem_mode, isothermal, rate_set, max_sub;
    int cells_per_lane;     // of a chemistry workgroup's share; 0: chosen by the cell count
    double c, T_iso, yhe, alpha_B, gm1, fmax, fs, growth, xfloor;
    double sigma[kMaxBins][3];
    double eheat[kMaxBins][3];
};

// Field layout: one record of four values per (bin, cell), U[(b nc + i) 4 + v]
// with v = N, Fh_x, Fh_y, Fh_z, so a neighbour's state is one 16-byte (FP32)
// or 32-byte (FP64) load.
__host__ __device__ inline int64_t urec(int b, int64_t nc, int64_t i) { return ((int64_t)b * nc + i) * 4; }

// Geometry of one precision variant (lengths in units of h_ref).
//   face [nf][kFaceRec]: A, n_x, n_y, n_z, rL_x, rL_y, rL_z, rR_x, rR_y, rR_z,
//     vcap_L, vcap_R (rL = minimum-image offset from the L cell centre to the
//     face centre; vcap = V / number of faces of the cell)
//   cell [nc][kCellRec]: inverse geometry matrix xx, yy, zz, xy, xz, yz; V; vcap
constexpr int kFaceRec = 12;
constexpr int kCellRec = 8;
// Per face side (sliced-ELL entry e), twelve values in four groups, each
// group a structure of arrays of records side[g][e][w] of width w, so that
// a kernel reads exactly the groups it uses:
//   g = 0 (w 4): w_x, w_y, w_z, r_x   w = A d / |d|^2 with d = s_j - s_i
//   g = 1 (w 2): r_y, r_z             r = r_if, offset from the cell centre
//   g = 2 (w 2): vcap_L, vcap_R       vcap = V / n_faces of the L and R cells
//   g = 3 (w 4): A, n_x, n_y, n_z     n from L to R
// (the gradient reads groups 0 and 1, the flux groups 2 and 3); zeros for
// padding entries.  A wavefront reads a group of a slot as one contiguous
// run.
enum SideComp { kSW0 = 0, kSW1, kSW2, kSR0, kSR1, kSR2, kSVL, kSVR, kSA, kSN0, kSN1, kSN2, kSideComps };
constexpr int kSideGroups = 4;
constexpr int kSideGroupFirst[kSideGroups + 1] = {0, 4, 6, 8, 12};   // first component of each group
template <typename T>
struct GeomView {
    const T* face;
    const T* cell;
    const T* side;
    const T* vol;          // [nc] V (the cell record's V as its own array, for the flux update)
    int64_t nf;
    int64_t ne;
    // group g of entry e (kSideGroupFirst[g+1] - kSideGroupFirst[g] values)
    __host__ __device__ const T* sg(int g, int64_t e) const {
        const int w = kSideGroupFirst[g + 1] - kSideGroupFirst[g];
        return side + (int64_t)kSideGroupFirst[g] * ne + e * w;
    }
    // component c (SideComp) of entry e
    __host__ __device__ T sv(int c, int64_t e) const {
        const int g = c < 4 ? 0 : c < 6 ? 1 : c < 8 ? 2 : 3;
        return sg(g, e)[c - kSideGroupFirst[g]];
    }
};

// Face sides of each cell in sliced-ELL order: slice s (cells 64s..64s+63)
// holds deg[s] slots; slot k of lane l is entry ptr[s] + 64 k + l.  nbr is
// the neighbour cell (-1 for padding), fsf the face index (f when the cell is
// the face's L cell, ~f when it is R), opp the entry of the same face in the
// neighbour's list.  Slots are in increasing face index.
struct SellView {
    const int32_t* nbr;
    const int32_t* fsf;
    const int32_t* opp;
    const int32_t* ptr;
    const int32_t* deg;
    const int2* nop;       // (nbr, opp for an L side or ~opp for an R side) of each entry, one 8-byte load
    const int32_t* fitem_ptr;   // face evaluations per slice (uniform-degree meshes; see kFluxPairBit)
    const int2* fitem;          // (entry | kFluxPairBit if paired, signed opposite entry) of each evaluation
    int32_t uniform_deg;   // slots of every slice when all are equal and specialised (6, 14), else 0
};

// Faces of the split transport on six-slot meshes by tile (rt_mesh
// tpair/tbnd/bmask): the tile-interior faces, as (L, R) entries relative to
// the tile's first entry in the low and high 16 bits; the face sides whose
// face crosses to another tile ("boundary items", numbered in entry order,
// so a tile's and a slice's items are contiguous: bnd_ptr per tile,
// bnd_sptr per slice), with the opposite side's item (complemented for an
// R side); per cell the slots of cross-tile faces.  Within a slice the
// items of a cell follow from the slot masks of the slice's cells:
// slot-major, then lane order.
struct TileFaceView {
    const int32_t* pair_ptr;
    const int32_t* pair;
    const int32_t* bnd_ptr;
    const int32_t* bnd_sptr;
    const int32_t* bnd_opp;
    const uint8_t* bmask;
    int64_t n_bnd;          // boundary items of the mesh
    int64_t bnd_max;        // most boundary items of one tile
};

// A face whose two sides are in one slice is evaluated once there, from its
// L side; the item carries this bit and the R side takes the negated
// product.  Entries stay below 2^30 (rt_mesh_create), so the bit is free.
constexpr int32_t kFluxPairBit = 1 << 30;

// Tiles of the fused transport kernel: tile t is cells [T t, T t + T) with
// T = kTileCells (whole slices, so its face sides are the contiguous entries
// ptr[t T/64] .. ptr[(t+1) T/64]).  Face states live in LDS: first the tile's own
// sides at (entry - ptr[4t]), then the halo sides: the sides of cells
// outside the tile that face a tile cell, grouped by halo cell.
//   lds_opp[e]     LDS slot of the state on the other side of entry e
//   halo_ptr[t]    first halo cell of tile t in halo_cell / hside_ptr
//   halo_cell[q]   halo cell id
//   hside_ptr[q]   first halo side of halo cell q in hside_entry; the LDS
//                  slot of halo side s of tile t is
//                  (tile sides) + s - hside_ptr[halo_ptr[t]]
//   hside_entry[s] sliced-ELL entry of the halo side
constexpr int kTileCells = 256;                 // cells per tile (RT_TILE_CELLS)
constexpr int kTileThreads = 256;               // threads per tile workgroup: one per tile cell
constexpr int kTileSlices = kTileCells / kSlice;
// Cells per workgroup of the flux kernels (one slice), which is also the
// granularity of the per-block partials (photon sums, counters, status) of
// both paths.
constexpr int kFluxBlock = kSlice;
constexpr int kFluxPairThreads = 256;           // threads of the flux workgroup of uniform-degree meshes
constexpr int kTileBlocks = kTileCells / kFluxBlock;  // partial slots per tile
struct TileView {
    const int32_t* lds_opp;
    const int32_t* halo_ptr;
    const int32_t* halo_cell;
    const int32_t* hside_ptr;
    const int32_t* hside_entry;
    int64_t n_slices;
    const uint8_t* bmask;   // six-slot meshes: per cell the slots of cross-tile faces (else null)
};

// Workgroup id -> logical block: hardware hands workgroups to the 8 XCDs in
// turn, so consecutive logical blocks (neighbouring cells in a locality
// order) are remapped to run on the same XCD and share its L2.
// (32-bit arithmetic: grids stay below 2^31 workgroups.)
__device__ inline uint32_t xcd_logical_block32() {
    const uint32_t w = blockIdx.x;
    const uint32_t G = gridDim.x;
    const uint32_t xcd = w % kNumXcd;
    const uint32_t local = w / kNumXcd;
    const uint32_t per = G / kNumXcd;
    const uint32_t rem = G % kNumXcd;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}
__device__ inline int64_t xcd_logical_block() { return (int64_t)xcd_logical_block32(); }

}  // namespace rtk
