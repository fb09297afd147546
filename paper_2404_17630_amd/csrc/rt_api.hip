// Host side of the C ABI declared in include/rt.h: argument validation, the
// one-time mesh preparation (minimum-image face offsets, least-squares
// geometry matrices and their inverses, sliced-ELL face lists), state
// allocation, the subcycle driver and field conversion.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "rt.h"
#include "rt_internal.hpp"
#include "rt_kernels.hpp"

using namespace rtk;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

int rt_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

extern "C" const char* rt_last_error(void) { return g_last_error.c_str(); }


namespace {

// True if p points into device memory (device or managed allocation).  With
// no usable device the runtime reports an error and p is host memory.
bool is_device_pointer(const void* p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Copies n elements from a host or device pointer into a host vector.
template <typename V>
int fetch(const V* src, size_t n, std::vector<V>& dst, const char* what) {
    if (n == 0) { dst.clear(); return RT_OK; }
    if (!src) return rt_fail(RT_EINVAL, "null pointer for %s", what);
    try {
        dst.resize(n);
    } catch (const std::bad_alloc&) {
        return rt_fail(RT_ENOMEM, "host allocation for %s", what);
    }
    if (is_device_pointer(src)) RT_HIP(hipMemcpy(dst.data(), src, n * sizeof(V), hipMemcpyDeviceToHost));
    else std::memcpy(dst.data(), src, n * sizeof(V));
    return RT_OK;
}

bool finite_all(const std::vector<double>& v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}


constexpr double kBoltzH = 1.380649e-16;
constexpr double kProtonMassH = 1.67262192369e-24;

}  // namespace

// ---------------------------------------------------------------------------
// Device buffers
// ---------------------------------------------------------------------------

int DevMem::alloc(size_t nbytes) {
    release();
    if (nbytes == 0) return RT_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return rt_fail(e == hipErrorOutOfMemory ? RT_ENOMEM : RT_EDEVICE, "hipMalloc(%zu bytes): %s", nbytes,
                       hipGetErrorString(e));
    }
    ptr = p;
    bytes = nbytes;
    return RT_OK;
}

void DevMem::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

int DevMem::upload(const void* src, size_t nbytes) {
    int rc = alloc(nbytes);
    if (rc) return rc;
    if (nbytes) RT_HIP(hipMemcpy(ptr, src, nbytes, hipMemcpyHostToDevice));
    return RT_OK;
}

// ---------------------------------------------------------------------------
// Mesh
// ---------------------------------------------------------------------------

extern "C" int rt_params_default(int32_t nb, rt_params* p) {
    if (!p) return rt_fail(RT_EINVAL, "null params");
    if (nb < 1 || nb > RT_MAX_BINS) return rt_fail(RT_EINVAL, "nb=%d outside 1..%d", nb, RT_MAX_BINS);
    std::memset(p, 0, sizeof(*p));
    p->nb = nb;
    p->chem_mode = RT_CHEM_H;
    p->isothermal = 1;
    p->rate_set = RT_RATES_CASEB_CONST;
    p->use_limiter = 1;
    p->chem_max_substeps = 100000;
    p->c_reduced = 0.01 * 2.99792458e10;
    p->cfl_eta = 0.3;
    p->T_iso = 1.0e4;
    p->Y_He = 0.0;
    p->alpha_B_const = 2.59e-13;
    p->gamma = 5.0 / 3.0;
    p->chem_fmax = 0.1;
    p->chem_fs = 0.05;
    p->chem_growth = 2.0;
    p->chem_xfloor = 1.0e-6;
    return RT_OK;
}

static double min_image(double x, double box) {
    if (box > 0) x -= box * std::floor(x / box + 0.5);
    return x;
}

static int upload_volumes(rt_mesh* m, bool fp32);

int rt_mesh::build_float_geometry() {
    if (geo32_ready) return RT_OK;
    std::vector<float> f(face.size()), c(cell.size());
    for (size_t q = 0; q < face.size(); ++q) f[q] = (float)face[q];
    for (size_t q = 0; q < cell.size(); ++q) c[q] = (float)cell[q];
    int rc;
    if ((rc = d_face32.upload(f.data(), f.size() * 4))) return rc;
    if ((rc = d_cell32.upload(c.data(), c.size() * 4))) return rc;
    if ((rc = upload_volumes(this, true))) return rc;
    geo32_ready = true;
    return RT_OK;
}

// Face evaluations of the flux kernel on a uniform-degree mesh: slice s
// evaluates the faces of its entries, once for a face whose other side is in
// the slice too (from the L side, with kFluxPairBit), once per side for a
// face that crosses to another slice.  Each item is the entry and its signed
// opposite entry (opp for an L side, ~opp for an R side).
void rt_mesh::build_flux_items() {
    fitem_ptr.clear();
    fitem.clear();
    if (uniform_deg == 0) return;
    const int64_t ns = (int64_t)sdeg.size();
    const int64_t per = (int64_t)uniform_deg * kSlice;
    fitem_ptr.assign(ns + 1, 0);
    fitem.reserve(2 * n_entries);
    for (int64_t s = 0; s < ns; ++s) {
        for (int64_t q = 0; q < per; ++q) {
            const int64_t e = s * per + q;
            if (nbr[e] < 0) continue;
            const bool same = (int64_t)opp[e] / per == s;
            if (same && fsf[e] < 0) continue;      // evaluated from its L side
            fitem.push_back((int32_t)e | (same ? kFluxPairBit : 0));
            fitem.push_back(fsf[e] >= 0 ? opp[e] : ~opp[e]);
        }
        fitem_ptr[s + 1] = (int32_t)(fitem.size() / 2);
    }
}

// Faces of the split transport on six-slot meshes, by tile of kTileCells
// cells (the fused kernel's tiles): a face with both sides in the tile is
// evaluated by the face-state kernel from its face states in LDS (once, the
// R side taking the negated product); a face that crosses to another tile
// is evaluated by the flux kernel for each side.
void rt_mesh::build_tile_faces() {
    tpair_ptr.clear(); tpair.clear(); tbnd_ptr.clear(); tbnd.clear(); tbnd_sptr.clear(); bmask.clear();
    tbnd_max = 0;
    if (uniform_deg != 6) return;
    const int64_t per = (int64_t)uniform_deg * kTileCells;     // entries of a tile
    const int64_t sper = (int64_t)uniform_deg * kSlice;        // entries of a slice
    const int64_t nt = (nc + kTileCells - 1) / kTileCells;
    const int64_t ns = (int64_t)sdeg.size();
    tpair_ptr.assign(nt + 1, 0);
    tbnd_ptr.assign(nt + 1, 0);
    tbnd_sptr.assign(ns + 1, 0);
    bmask.assign(nc, 0);
    std::vector<int32_t> item(n_entries, -1);
    int32_t n_items = 0;
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t e0 = t * per;
        for (int64_t q = 0; q < per && e0 + q < n_entries; ++q) {
            const int64_t e = e0 + q;
            if (nbr[e] < 0) continue;
            const int64_t qo = (int64_t)opp[e] - e0;
            const int64_t cell = t * kTileCells + (q / sper) * kSlice + q % kSlice;
            const int k = (int)((q % sper) / kSlice);
            if (qo >= 0 && qo < per) {
                if (fsf[e] >= 0) tpair.push_back((int32_t)(q | (qo << 16)));
            } else {
                item[e] = n_items++;
                tbnd.push_back((int32_t)e);
                tbnd.push_back(0);
                bmask[cell] |= (uint8_t)(1u << k);
                ++tbnd_sptr[e / sper + 1];
            }
        }
        tpair_ptr[t + 1] = (int32_t)tpair.size();
        tbnd_ptr[t + 1] = n_items;
        tbnd_max = std::max<int64_t>(tbnd_max, tbnd_ptr[t + 1] - tbnd_ptr[t]);
        // a face takes two of the tile's sides, so a tile has at most
        // 3 kTileCells interior faces: the face-state kernel's three per thread
        if (tpair_ptr[t + 1] - tpair_ptr[t] > 3 * kTileCells) {
            tpair_ptr.clear(); tpair.clear(); tbnd_ptr.clear(); tbnd.clear(); tbnd_sptr.clear(); bmask.clear();
            tbnd_max = 0;
            return;
        }
    }
    for (int64_t s = 0; s < ns; ++s) tbnd_sptr[s + 1] += tbnd_sptr[s];
    // The tile split pays off when tiles are compact (a Hilbert-ordered
    // lattice has about one cross-tile side per cell); with more than two a
    // cell (an unordered mesh: up to all six) the per-slice kernels are used.
    if (n_items > 2 * nc) {
        tpair_ptr.clear(); tpair.clear(); tbnd_ptr.clear(); tbnd.clear(); tbnd_sptr.clear(); bmask.clear();
        tbnd_max = 0;
        return;
    }
    // the opposite side of a boundary item is a boundary item of its own tile
    for (int32_t q = 0; q < n_items; ++q) {
        const int32_t e = tbnd[2 * q];
        const int32_t o = item[opp[e]];
        tbnd[2 * q + 1] = fsf[e] >= 0 ? o : ~o;
    }
}

// Tiles of kTileCells cells for the fused transport kernel: the LDS slot of every
// face side's opposite state, and the halo cells with the sides they
// contribute, grouped per tile in (cell, entry) order.
static_assert(kTileCells == RT_TILE_CELLS, "tile size of the header and the kernels");
static_assert(kTileCells % kBlock == 0 && kTileCells % kSlice == 0, "tiles are whole blocks and slices");
static_assert(kTileThreads == kTileCells, "one thread per tile cell in the flux phase");
static_assert(kTileCells % kFluxBlock == 0 && kFluxBlock % 64 == 0, "tiles hold whole flux workgroups of whole waves");

void rt_mesh::build_tiles() {
    const int64_t ns = (int64_t)sdeg.size();
    const int64_t ntiles = (nc + kTileCells - 1) / kTileCells;
    lds_opp.assign(n_entries, -1);
    halo_ptr.assign(ntiles + 1, 0);
    halo_cell.clear();
    hside_ptr.clear();
    hside_entry.clear();
    tile_max_sides = 0;
    struct Ext {
        int32_t j, eo;
        int64_t e;
    };
    std::vector<Ext> ext;
    for (int64_t t = 0; t < ntiles; ++t) {
        const int64_t c0 = t * kTileCells, c1 = std::min<int64_t>(nc, c0 + kTileCells);
        const int64_t e0 = sptr[t * kTileSlices];
        const int64_t tile_sides = (int64_t)sptr[std::min<int64_t>(ns, (t + 1) * kTileSlices)] - e0;
        ext.clear();
        for (int64_t i = c0; i < c1; ++i) {
            const int64_t sl = i / kSlice;
            for (int64_t k = 0; k < sdeg[sl]; ++k) {
                const int64_t e = sptr[sl] + k * kSlice + i % kSlice;
                const int32_t j = nbr[e];
                if (j < 0) continue;
                if (j >= c0 && j < c1) lds_opp[e] = (int32_t)(opp[e] - e0);
                else ext.push_back({j, opp[e], e});
            }
        }
        std::stable_sort(ext.begin(), ext.end(),
                         [](const Ext& a, const Ext& b) { return a.j != b.j ? a.j < b.j : a.eo < b.eo; });
        const int64_t hs0 = (int64_t)hside_entry.size();
        for (size_t q = 0; q < ext.size(); ++q) {
            if (q == 0 || ext[q].j != ext[q - 1].j) {
                halo_cell.push_back(ext[q].j);
                hside_ptr.push_back((int32_t)hside_entry.size());
            }
            lds_opp[ext[q].e] = (int32_t)(tile_sides + (int64_t)hside_entry.size() - hs0);
            hside_entry.push_back(ext[q].eo);
        }
        halo_ptr[t + 1] = (int32_t)halo_cell.size();
        tile_max_sides = std::max<int64_t>(tile_max_sides, tile_sides + (int64_t)ext.size());
    }
    hside_ptr.push_back((int32_t)hside_entry.size());
    halo_ratio = (double)halo_cell.size() / (double)nc;
}

// Per face side records in the transport precision (rtk::SideComp), one
// group at a time.
int rt_mesh::build_side_geometry(size_t tbytes) {
    DevMem& d = tbytes == 4 ? d_side32 : d_side64;
    if (d.ptr) return RT_OK;
    const int64_t ne = n_entries;
    int rc;
    if ((rc = d.alloc((size_t)kSideComps * ne * tbytes))) return rc;
    // all components of every entry, then each group as its own array
    std::vector<double> all((size_t)kSideComps * ne, 0.0);
    for (int64_t e = 0; e < ne; ++e) {
        if (nbr[e] < 0) continue;
        const bool isL = fsf[e] >= 0;
        const double* rec = &face[(size_t)(isL ? fsf[e] : ~fsf[e]) * kFaceRec];
        const double* ro = isL ? rec + 4 : rec + 7;     // own offset
        const double* rn = isL ? rec + 7 : rec + 4;     // neighbour's offset
        double* a = &all[(size_t)kSideComps * e];
        const double d0 = ro[0] - rn[0], d1 = ro[1] - rn[1], d2 = ro[2] - rn[2];
        const double sc = rec[0] / (d0 * d0 + d1 * d1 + d2 * d2);
        a[kSW0] = d0 * sc; a[kSW1] = d1 * sc; a[kSW2] = d2 * sc;
        a[kSR0] = ro[0]; a[kSR1] = ro[1]; a[kSR2] = ro[2];
        a[kSA] = rec[0];
        a[kSN0] = rec[1]; a[kSN1] = rec[2]; a[kSN2] = rec[3];
        a[kSVL] = rec[10]; a[kSVR] = rec[11];
    }
    std::vector<double> grp((size_t)kSideComps * ne);
    for (int g = 0; g < kSideGroups; ++g) {
        const int c0 = kSideGroupFirst[g], w = kSideGroupFirst[g + 1] - c0;
        for (int64_t e = 0; e < ne; ++e)
            for (int q = 0; q < w; ++q) grp[(size_t)c0 * ne + (size_t)e * w + q] = all[(size_t)kSideComps * e + c0 + q];
    }
    hipError_t err;
    if (tbytes == 4) {
        std::vector<float> g32(grp.begin(), grp.end());
        err = hipMemcpy(d.ptr, g32.data(), g32.size() * 4, hipMemcpyHostToDevice);
    } else {
        err = hipMemcpy(d.ptr, grp.data(), grp.size() * 8, hipMemcpyHostToDevice);
    }
    if (err != hipSuccess) return rt_fail(RT_EDEVICE, "side geometry upload: %s", hipGetErrorString(err));
    // area and normal of every boundary item of the split transport by tile
    if (!tbnd.empty()) {
        const int64_t nq = n_bnd();
        std::vector<double> bg((size_t)nq * 4);
        for (int64_t q = 0; q < nq; ++q) {
            const int32_t e = tbnd[2 * q];
            const double* rec = &face[(size_t)(fsf[e] >= 0 ? fsf[e] : ~fsf[e]) * kFaceRec];
            for (int v = 0; v < 4; ++v) bg[(size_t)q * 4 + v] = rec[v];
        }
        if (tbytes == 4) {
            std::vector<float> b32(bg.begin(), bg.end());
            if ((rc = d_bgeo32.upload(b32.data(), b32.size() * 4))) return rc;
        } else if ((rc = d_bgeo64.upload(bg.data(), bg.size() * 8))) {
            return rc;
        }
    }
    return RT_OK;
}

// (nbr, opp for an L side or ~opp for an R side) of every sliced-ELL entry
// as one 8-byte record.
static int upload_packed_index(rt_mesh* m) {
    std::vector<int32_t> p((size_t)2 * m->n_entries, 0);
    for (int64_t e = 0; e < m->n_entries; ++e) {
        p[2 * e] = m->nbr[e];
        p[2 * e + 1] = m->nbr[e] < 0 ? 0 : (m->fsf[e] >= 0 ? m->opp[e] : ~m->opp[e]);
    }
    return m->d_idx.upload(p.data(), p.size() * 4);
}

// The opposite item of every boundary item (the device's part of tbnd).
static int upload_bnd_opp(rt_mesh* m) {
    std::vector<int32_t> o((size_t)m->n_bnd());
    for (size_t q = 0; q < o.size(); ++q) o[q] = m->tbnd[2 * q + 1];
    return m->d_tbnd_opp.upload(o.data(), o.size() * 4);
}

// The cells' V (units of h_ref^3) as one array per precision.
static int upload_volumes(rt_mesh* m, bool fp32) {
    std::vector<double> v(m->nc);
    for (int64_t i = 0; i < m->nc; ++i) v[i] = m->cell[(size_t)i * kCellRec + 6];
    if (!fp32) return m->d_vol64.upload(v.data(), v.size() * 8);
    std::vector<float> f(v.begin(), v.end());
    return m->d_vol32.upload(f.data(), f.size() * 4);
}

extern "C" int rt_mesh_create(int64_t n_cells, const double* volume, const double* centre, int64_t n_faces,
                              const int64_t* face_cells, const double* area, const double* normal,
                              const double* face_centre, const double box_in[3], int device, rt_mesh** out) {
    if (!out) return rt_fail(RT_EINVAL, "null output handle");
    *out = nullptr;
    if (n_cells < 1 || n_faces < 1) return rt_fail(RT_EINVAL, "n_cells=%lld n_faces=%lld", (long long)n_cells,
                                                   (long long)n_faces);
    if (n_cells >= INT32_MAX / 2 || n_faces >= INT32_MAX / 2)
        return rt_fail(RT_EINVAL, "mesh too large for 32-bit face indices");
    if (!box_in) return rt_fail(RT_EINVAL, "null box");

    const int64_t nc = n_cells, nf = n_faces;
    std::vector<double> V, S, A, Nrm, Xf;
    std::vector<int64_t> FC;
    int rc;
    if ((rc = fetch(volume, nc, V, "volume"))) return rc;
    if ((rc = fetch(centre, 3 * nc, S, "centre"))) return rc;
    if ((rc = fetch(face_cells, 2 * nf, FC, "face_cells"))) return rc;
    if ((rc = fetch(area, nf, A, "area"))) return rc;
    if ((rc = fetch(normal, 3 * nf, Nrm, "normal"))) return rc;
    if ((rc = fetch(face_centre, 3 * nf, Xf, "face_centre"))) return rc;
    double box[3] = {box_in[0], box_in[1], box_in[2]};
    for (int k = 0; k < 3; ++k)
        if (!(box[k] >= 0) || !std::isfinite(box[k])) return rt_fail(RT_EINVAL, "box[%d]=%g", k, box[k]);
    if (!finite_all(S) || !finite_all(Xf)) return rt_fail(RT_EMESH, "non-finite centre or face centre");
    for (int64_t i = 0; i < nc; ++i)
        if (!(V[i] > 0) || !std::isfinite(V[i])) return rt_fail(RT_EMESH, "cell %lld: volume %g", (long long)i, V[i]);
    std::vector<int32_t> deg(nc, 0);
    for (int64_t f = 0; f < nf; ++f) {
        int64_t L = FC[f], R = FC[nf + f];
        if (L < 0 || L >= nc || R < 0 || R >= nc)
            return rt_fail(RT_EMESH, "face %lld: cell index out of range (%lld, %lld)", (long long)f, (long long)L,
                           (long long)R);
        if (L == R) return rt_fail(RT_EMESH, "face %lld joins cell %lld to itself", (long long)f, (long long)L);
        if (!(A[f] > 0) || !std::isfinite(A[f])) return rt_fail(RT_EMESH, "face %lld: area %g", (long long)f, A[f]);
        double nn = std::sqrt(Nrm[f] * Nrm[f] + Nrm[nf + f] * Nrm[nf + f] + Nrm[2 * nf + f] * Nrm[2 * nf + f]);
        if (!(std::fabs(nn - 1.0) <= 1e-12)) return rt_fail(RT_EMESH, "face %lld: |n| = %.17g", (long long)f, nn);
        ++deg[L];
        ++deg[R];
    }
    for (int64_t i = 0; i < nc; ++i) {
        if (deg[i] < 4) return rt_fail(RT_EMESH, "cell %lld has %d faces (< 4)", (long long)i, deg[i]);
        if (deg[i] > kMaxCellFaces)
            return rt_fail(RT_EMESH, "cell %lld has %d faces (> %d)", (long long)i, deg[i], kMaxCellFaces);
    }

    rt_mesh* m = new (std::nothrow) rt_mesh();
    if (!m) return rt_fail(RT_ENOMEM, "mesh handle");
    m->device = device;
    m->nc = nc;
    m->nf = nf;
    double vsum = 0;
    for (double v : V) vsum += v;
    const double h = std::cbrt(vsum / (double)nc);
    m->h_ref = h;
    const double h2 = h * h, h3 = h2 * h;

    // Per-face geometry in units of h: A, n, r_Lf, r_Rf (minimum image); the
    // cells' V / n_faces are filled in below.
    m->face.assign((size_t)kFaceRec * nf, 0.0);
    for (int64_t f = 0; f < nf; ++f) {
        int64_t L = FC[f], R = FC[nf + f];
        double* rec = &m->face[(size_t)f * kFaceRec];
        rec[0] = A[f] / h2;
        for (int k = 0; k < 3; ++k) {
            rec[1 + k] = Nrm[k * nf + f];
            rec[4 + k] = min_image(Xf[k * nf + f] - S[k * nc + L], box[k]) / h;
            rec[7 + k] = min_image(Xf[k * nf + f] - S[k * nc + R], box[k]) / h;
        }
    }
    // Face sides per cell in face-index order (counting sort keeps the order).
    std::vector<int64_t> off(nc + 1, 0);
    for (int64_t i = 0; i < nc; ++i) off[i + 1] = off[i] + deg[i];
    std::vector<int32_t> side_face(2 * nf), side_nbr(2 * nf);
    std::vector<uint8_t> side_isL(2 * nf);
    {
        std::vector<int64_t> fill(off.begin(), off.end() - 1);
        for (int64_t f = 0; f < nf; ++f) {
            int64_t L = FC[f], R = FC[nf + f];
            int64_t eL = fill[L]++, eR = fill[R]++;
            side_face[eL] = (int32_t)f; side_nbr[eL] = (int32_t)R; side_isL[eL] = 1;
            side_face[eR] = (int32_t)f; side_nbr[eR] = (int32_t)L; side_isL[eR] = 0;
        }
    }
    // Geometry matrix M_i = sum A u u^T (u = unit separation through the face),
    // its inverse by the adjugate, and a Frobenius condition-number check.
    m->cell.assign((size_t)kCellRec * nc, 0.0);
    m->vphys = V;
    for (int64_t i = 0; i < nc; ++i) {
        double M[6] = {0, 0, 0, 0, 0, 0};   // xx yy zz xy xz yz
        for (int64_t e = off[i]; e < off[i + 1]; ++e) {
            const int64_t f = side_face[e];
            const bool isL = side_isL[e];
            const double* rec = &m->face[(size_t)f * kFaceRec];
            double d[3];
            for (int k = 0; k < 3; ++k) d[k] = isL ? rec[4 + k] - rec[7 + k] : rec[7 + k] - rec[4 + k];
            const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(dd > 0)) {
                delete m;
                return rt_fail(RT_EMESH, "cell %lld: coincident neighbour centre through face %lld", (long long)i,
                               (long long)f);
            }
            const double Af = rec[0] / dd;
            M[0] += Af * d[0] * d[0]; M[1] += Af * d[1] * d[1]; M[2] += Af * d[2] * d[2];
            M[3] += Af * d[0] * d[1]; M[4] += Af * d[0] * d[2]; M[5] += Af * d[1] * d[2];
        }
        const double a = M[0], b = M[1], c = M[2], dxy = M[3], exz = M[4], fyz = M[5];
        const double det = a * (b * c - fyz * fyz) - dxy * (dxy * c - fyz * exz) + exz * (dxy * fyz - b * exz);
        double inv[6];
        inv[0] = (b * c - fyz * fyz) / det;
        inv[1] = (a * c - exz * exz) / det;
        inv[2] = (a * b - dxy * dxy) / det;
        inv[3] = (exz * fyz - dxy * c) / det;
        inv[4] = (dxy * fyz - b * exz) / det;
        inv[5] = (dxy * exz - a * fyz) / det;
        double nM = a * a + b * b + c * c + 2 * (dxy * dxy + exz * exz + fyz * fyz);
        double nI = inv[0] * inv[0] + inv[1] * inv[1] + inv[2] * inv[2] +
                    2 * (inv[3] * inv[3] + inv[4] * inv[4] + inv[5] * inv[5]);
        double cond = std::sqrt(nM * nI);
        if (!(det != 0) || !std::isfinite(cond) || cond > 1e12) {
            delete m;
            return rt_fail(RT_EMESH, "cell %lld: geometry matrix condition number %g", (long long)i, cond);
        }
        double* rec = &m->cell[(size_t)i * kCellRec];
        for (int q = 0; q < 6; ++q) rec[q] = inv[q];
        rec[6] = V[i] / h3;
        rec[7] = rec[6] / (double)deg[i];
    }
    for (int64_t f = 0; f < nf; ++f) {
        m->face[(size_t)f * kFaceRec + 10] = m->cell[(size_t)FC[f] * kCellRec + 7];
        m->face[(size_t)f * kFaceRec + 11] = m->cell[(size_t)FC[nf + f] * kCellRec + 7];
    }
    // Sliced ELL with 64-cell slices.
    const int64_t ns = (nc + kSlice - 1) / kSlice;
    m->sdeg.assign(ns, 0);
    m->sptr.assign(ns + 1, 0);
    for (int64_t s = 0; s < ns; ++s) {
        int32_t mx = 0;
        for (int64_t i = s * kSlice; i < std::min<int64_t>(nc, (s + 1) * kSlice); ++i) mx = std::max(mx, deg[i]);
        m->sdeg[s] = mx;
        m->sptr[s + 1] = m->sptr[s] + mx * kSlice;
        if ((int64_t)m->sptr[s + 1] > INT32_MAX / 2) {
            delete m;
            return rt_fail(RT_EINVAL, "too many face sides");
        }
    }
    const int64_t ne = m->sptr[ns];
    m->n_entries = ne;
    m->nbr.assign(ne, -1);
    m->fsf.assign(ne, 0);
    m->opp.assign(ne, 0);
    std::vector<int64_t> entry_of_side(2 * nf);   // CSR face side -> sliced-ELL entry
    for (int64_t i = 0; i < nc; ++i) {
        const int64_t s = i / kSlice, lane = i % kSlice;
        for (int64_t k = 0; k < deg[i]; ++k) {
            const int64_t e = m->sptr[s] + k * kSlice + lane;
            const int64_t src = off[i] + k;
            m->nbr[e] = side_nbr[src];
            m->fsf[e] = side_isL[src] ? side_face[src] : ~side_face[src];
            entry_of_side[src] = e;
        }
    }
    {
        // the two sides of each face point at each other
        std::vector<int64_t> side_of_face(2 * nf, -1);
        for (int64_t src = 0; src < 2 * nf; ++src) side_of_face[2 * (int64_t)side_face[src] + (side_isL[src] ? 0 : 1)] = src;
        for (int64_t f = 0; f < nf; ++f) {
            const int64_t eL = entry_of_side[side_of_face[2 * f]], eR = entry_of_side[side_of_face[2 * f + 1]];
            m->opp[eL] = (int32_t)eR;
            m->opp[eR] = (int32_t)eL;
        }
    }
    m->max_deg = *std::max_element(deg.begin(), deg.end());
    {
        const int32_t d0 = m->sdeg[0];
        bool uniform = (d0 == 6 || d0 == 14);
        for (int64_t q = 0; q < nc && uniform; ++q) uniform = deg[q] == d0;
        m->uniform_deg = uniform ? d0 : 0;
    }
    m->deg = std::move(deg);
    if ((int64_t)m->n_entries + (int64_t)2 * nf >= INT32_MAX / 2) {
        delete m;
        return rt_fail(RT_EINVAL, "too many face sides for the tile tables");
    }
    m->build_tiles();
    m->build_flux_items();
    m->build_tile_faces();
    if (device == RT_DEVICE_HOST_ONLY) {
        m->refs.store(1);
        *out = m;
        return RT_OK;
    }

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) {
        (void)hipGetLastError();
        ndev = 0;
    }
    if (device < 0 || device >= ndev) {
        delete m;
        return rt_fail(RT_EDEVICE, "device %d of %d", device, ndev);
    }
    DeviceGuard dg(device);

    if ((rc = m->d_face64.upload(m->face.data(), m->face.size() * 8)) ||
        (rc = m->d_cell64.upload(m->cell.data(), m->cell.size() * 8)) || (rc = upload_volumes(m, false)) ||
        (rc = m->d_vphys.upload(m->vphys.data(), m->vphys.size() * 8)) ||
        (rc = m->d_nbr.upload(m->nbr.data(), m->nbr.size() * 4)) ||
        (rc = m->d_fsf.upload(m->fsf.data(), m->fsf.size() * 4)) ||
        (rc = m->d_opp.upload(m->opp.data(), m->opp.size() * 4)) ||
        (rc = m->d_sptr.upload(m->sptr.data(), m->sptr.size() * 4)) ||
        (rc = m->d_sdeg.upload(m->sdeg.data(), m->sdeg.size() * 4)) || (rc = upload_packed_index(m)) ||
        (rc = m->d_lds_opp.upload(m->lds_opp.data(), m->lds_opp.size() * 4)) ||
        (rc = m->d_halo_ptr.upload(m->halo_ptr.data(), m->halo_ptr.size() * 4)) ||
        (rc = m->d_halo_cell.upload(m->halo_cell.data(), m->halo_cell.size() * 4)) ||
        (rc = m->d_hside_ptr.upload(m->hside_ptr.data(), m->hside_ptr.size() * 4)) ||
        (rc = m->d_hside_entry.upload(m->hside_entry.data(), m->hside_entry.size() * 4)) ||
        (rc = m->d_fitem_ptr.upload(m->fitem_ptr.data(), m->fitem_ptr.size() * 4)) ||
        (rc = m->d_fitem.upload(m->fitem.data(), m->fitem.size() * 4)) ||
        (rc = m->d_tpair_ptr.upload(m->tpair_ptr.data(), m->tpair_ptr.size() * 4)) ||
        (rc = m->d_tpair.upload(m->tpair.data(), m->tpair.size() * 4)) ||
        (rc = m->d_tbnd_ptr.upload(m->tbnd_ptr.data(), m->tbnd_ptr.size() * 4)) ||
        (rc = upload_bnd_opp(m)) ||
        (rc = m->d_tbnd_sptr.upload(m->tbnd_sptr.data(), m->tbnd_sptr.size() * 4)) ||
        (rc = m->d_bmask.upload(m->bmask.data(), m->bmask.size()))) {
        delete m;
        return rc;
    }
    {
        // LDS available to one workgroup, less the fused kernel's static use.
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) {
            (void)hipGetLastError();
            lds = 0;
        }
        m->lds_limit = lds > 1024 ? (size_t)lds - 1024 : 0;
    }
    // CFL length min_i (3V/4pi)^(1/3) by the device min-reduction.
    {
        DevMem part;
        const int64_t np = cfl_partials(nc);
        if ((rc = part.alloc(np * 8))) { delete m; return rc; }
        launch_min_cfl_length((const double*)m->d_vphys.ptr, nc, (double*)part.ptr, nullptr);
        std::vector<double> hp(np);
        hipError_t e = hipMemcpy(hp.data(), part.ptr, np * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) { delete m; return rt_fail(RT_EDEVICE, "CFL reduction: %s", hipGetErrorString(e)); }
        m->dx_min = *std::min_element(hp.begin(), hp.end());
    }
    m->refs.store(1);
    *out = m;
    return RT_OK;
}

void rt_mesh_release(rt_mesh* m) {
    if (m && m->refs.fetch_sub(1) == 1) {
        DeviceGuard dg(m->device);
        delete m;
    }
}

extern "C" int rt_mesh_table(const rt_mesh* m, int table, const int32_t** data, int64_t* length) {
    if (!m || !data || !length) return rt_fail(RT_EINVAL, "null argument");
    const std::vector<int32_t>* v = nullptr;
    switch (table) {
        case RT_TABLE_NBR: v = &m->nbr; break;
        case RT_TABLE_FSF: v = &m->fsf; break;
        case RT_TABLE_OPP: v = &m->opp; break;
        case RT_TABLE_SPTR: v = &m->sptr; break;
        case RT_TABLE_SDEG: v = &m->sdeg; break;
        case RT_TABLE_LDS_OPP: v = &m->lds_opp; break;
        case RT_TABLE_HALO_PTR: v = &m->halo_ptr; break;
        case RT_TABLE_HALO_CELL: v = &m->halo_cell; break;
        case RT_TABLE_HSIDE_PTR: v = &m->hside_ptr; break;
        case RT_TABLE_HSIDE_ENTRY: v = &m->hside_entry; break;
        case RT_TABLE_FITEM_PTR: v = &m->fitem_ptr; break;
        case RT_TABLE_FITEM: v = &m->fitem; break;
        case RT_TABLE_TPAIR_PTR: v = &m->tpair_ptr; break;
        case RT_TABLE_TPAIR: v = &m->tpair; break;
        case RT_TABLE_TBND_PTR: v = &m->tbnd_ptr; break;
        case RT_TABLE_TBND: v = &m->tbnd; break;
        case RT_TABLE_TBND_SPTR: v = &m->tbnd_sptr; break;
        default: return rt_fail(RT_EINVAL, "table %d", table);
    }
    *data = v->data();
    *length = (int64_t)v->size();
    return RT_OK;
}

extern "C" int rt_mesh_destroy(rt_mesh* m) {
    if (!m) return rt_fail(RT_EINVAL, "null mesh");
    rt_mesh_release(m);
    return RT_OK;
}

// ---------------------------------------------------------------------------
// State
// ---------------------------------------------------------------------------

static int check_params(const rt_params* p) {
    if (!p) return rt_fail(RT_EINVAL, "null params");
    if (p->nb < 1 || p->nb > RT_MAX_BINS) return rt_fail(RT_EINVAL, "nb=%d", p->nb);
    if (p->chem_mode < RT_CHEM_NONE || p->chem_mode > RT_CHEM_HHE) return rt_fail(RT_EINVAL, "chem_mode=%d", p->chem_mode);
    if (p->rate_set != RT_RATES_CASEB_CONST && p->rate_set != RT_RATES_HG97)
        return rt_fail(RT_EINVAL, "rate_set=%d", p->rate_set);
    if (p->rate_set == RT_RATES_CASEB_CONST && p->chem_mode == RT_CHEM_HHE)
        return rt_fail(RT_EINVAL, "constant case-B rates are hydrogen-only");
    if (p->rate_set == RT_RATES_CASEB_CONST && p->chem_mode != RT_CHEM_NONE && !p->isothermal)
        return rt_fail(RT_EINVAL, "constant case-B rates need an isothermal run");
    if (!(p->c_reduced > 0) || !std::isfinite(p->c_reduced)) return rt_fail(RT_EINVAL, "c_reduced=%g", p->c_reduced);
    if (!(p->cfl_eta > 0 && p->cfl_eta <= 1)) return rt_fail(RT_EINVAL, "cfl_eta=%g", p->cfl_eta);
    if (p->isothermal && !(p->T_iso > 0)) return rt_fail(RT_EINVAL, "T_iso=%g", p->T_iso);
    if (!(p->Y_He >= 0 && p->Y_He < 1)) return rt_fail(RT_EINVAL, "Y_He=%g", p->Y_He);
    if (!(p->gamma > 1)) return rt_fail(RT_EINVAL, "gamma=%g", p->gamma);
    if (!(p->chem_fmax > 0) || !(p->chem_fs > 0) || !(p->chem_growth >= 1) || !(p->chem_xfloor > 0) ||
        p->chem_max_substeps < 1)
        return rt_fail(RT_EINVAL, "chemistry controller parameters");
    if (p->chem_cells_per_lane < 0 || p->chem_cells_per_lane > kMaxChemCellsPerLane)
        return rt_fail(RT_EINVAL, "chem_cells_per_lane=%d (0..%d)", p->chem_cells_per_lane, kMaxChemCellsPerLane);
    if (p->rate_set == RT_RATES_CASEB_CONST && !(p->alpha_B_const >= 0)) return rt_fail(RT_EINVAL, "alpha_B_const");
    for (int b = 0; b < p->nb; ++b)
        for (int s = 0; s < 3; ++s)
            if (!(p->sigma[b][s] >= 0) || !std::isfinite(p->sigma[b][s]) || !(p->e_heat[b][s] >= 0) ||
                !std::isfinite(p->e_heat[b][s]))
                return rt_fail(RT_EINVAL, "sigma/e_heat[%d][%d]", b, s);
    return RT_OK;
}

static ChemParams chem_params_of(const rt_params& p) {
    ChemParams c;
    std::memset(&c, 0, sizeof(c));
    c.nb = p.nb;
    c.chem_mode = p.chem_mode;
    c.isothermal = p.isothermal;
    c.rate_set = p.rate_set;
    c.max_sub = p.chem_max_substeps;
    c.cells_per_lane = p.chem_cells_per_lane;
    c.c = p.c_reduced;
    c.T_iso = p.T_iso;
    c.yhe = p.chem_mode == RT_CHEM_HHE ? p.Y_He / (4.0 * (1.0 - p.Y_He)) : 0.0;
    c.alpha_B = p.alpha_B_const;
    c.gm1 = p.gamma - 1.0;
    c.fmax = p.chem_fmax;
    c.fs = p.chem_fs;
    c.growth = p.chem_growth;
    c.xfloor = p.chem_xfloor;
    for (int b = 0; b < p.nb; ++b)
        for (int s = 0; s < 3; ++s) {
            c.sigma[b][s] = p.sigma[b][s];
            c.eheat[b][s] = p.e_heat[b][s];
        }
    return c;
}

static double pow2_at_least(double m) {
    if (!(m > 0) || !std::isfinite(m)) return 1.0;
    int e;
    double fr = std::frexp(m, &e);   // m = fr * 2^e, fr in [0.5, 1)
    (void)fr;
    return std::ldexp(1.0, e);
}

size_t rt_state::tbytes() const { return precision == RT_MIXED ? 4 : 8; }

// The face-state array of the split path, allocated when a state is created,
// cloned or switched to that path.
int rt_state::ensure_face_states() {
    if (FV.ptr) return RT_OK;
    // face states [nb][n_entries][4], then the cells' cap numerators N V / n_faces [nb][nc]
    // (by tile on six-slot meshes: the boundary items' states and cap
    // numerators [nb][n_bnd][5])
    const size_t n = std::max((size_t)nb * 4 * mesh->n_entries + (size_t)nb * nc, (size_t)nb * 5 * mesh->n_bnd());
    return FV.alloc(n * tbytes());
}

static size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t rt_partial_bytes(int64_t n_fblk, int64_t n_cblk) {
    return align256(n_fblk * 8) + align256(5 * n_fblk * 8) + align256(n_fblk * 4) + align256(n_cblk * 8) +
           align256(n_cblk * 8) + align256(n_cblk * 4) + align256(kReduceBlocks * sizeof(DiagDev)) +
           align256(sizeof(DiagDev));
}

PartialBufs rt_partials_at(void* base, int64_t n_fblk, int64_t n_cblk) {
    char* p = (char*)base;
    PartialBufs b;
    b.nv = (double*)p;         p += align256(n_fblk * 8);
    b.cnt = (int64_t*)p;       p += align256(5 * n_fblk * 8);
    b.fst = (int32_t*)p;       p += align256(n_fblk * 4);
    b.csum = (int64_t*)p;      p += align256(n_cblk * 8);
    b.cmax = (int64_t*)p;      p += align256(n_cblk * 8);
    b.cst = (int32_t*)p;       p += align256(n_cblk * 4);
    b.red = (DiagDev*)p;       p += align256(kReduceBlocks * sizeof(DiagDev));
    b.diag = (DiagDev*)p;
    return b;
}

int rt_state::alloc_buffers() {
    const size_t t = tbytes();
    int rc;
    if ((rc = U[0].alloc((size_t)nb * 4 * nc * t)) || (rc = U[1].alloc((size_t)nb * 4 * nc * t)) ||
        (rc = X.alloc(5 * nc * 8)) || (rc = Ue.alloc(nc * 8)) || (rc = nH.alloc(nc * 8)) ||
        (rc = att.alloc(nc * 4)))
        return rc;
    n_fblk = partial_blocks(nc, nb);
    n_cblk = chem_blocks(nc, cp.cells_per_lane);
    if ((rc = part_mem.alloc(rt_partial_bytes(n_fblk, n_cblk)))) return rc;
    pb = rt_partials_at(part_mem.ptr, n_fblk, n_cblk);
    RT_HIP(hipHostMalloc((void**)&h_diag, sizeof(DiagDev), hipHostMallocDefault));
    return RT_OK;
}

int rt_state::upload_scales() {
    std::vector<double> s(nb), inv(nb), nvs(nb);
    for (int b = 0; b < nb; ++b) {
        s[b] = scale[b];
        inv[b] = 1.0 / scale[b];
        nvs[b] = scale[b] * mesh->h_ref * mesh->h_ref * mesh->h_ref;
    }
    int rc;
    if ((rc = d_scale.upload(s.data(), nb * 8)) || (rc = d_inv_scale.upload(inv.data(), nb * 8)) ||
        (rc = d_nv_scale.upload(nvs.data(), nb * 8)))
        return rc;
    return RT_OK;
}

int rt_state::upload_sources() {
    // Stable sort of the sources by cell; each source cell adds its sources
    // in list order.
    std::vector<int64_t> order(n_src);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return src_cell[a] < src_cell[b]; });
    std::vector<int32_t> cells, ptr;
    std::vector<double> rate((size_t)nb * n_src), vp(n_src);
    for (int64_t q = 0; q < n_src; ++q) {
        const int64_t k = order[q];
        if (cells.empty() || cells.back() != (int32_t)src_cell[k]) {
            cells.push_back((int32_t)src_cell[k]);
            ptr.push_back((int32_t)q);
        }
        for (int b = 0; b < nb; ++b) rate[(size_t)b * n_src + q] = src_rate[(size_t)b * n_src + k];
        vp[q] = mesh->vphys[src_cell[k]];
    }
    ptr.push_back((int32_t)n_src);
    n_src_cells = (int32_t)cells.size();

    int rc;
    if ((rc = d_src_cell.upload(cells.data(), cells.size() * 4)) || (rc = d_src_ptr.upload(ptr.data(), ptr.size() * 4)) ||
        (rc = d_src_rate.upload(rate.data(), rate.size() * 8)) || (rc = d_src_vphys.upload(vp.data(), vp.size() * 8)))
        return rc;
    return RT_OK;
}

extern "C" int rt_state_create(const rt_mesh* mesh_c, const rt_params* params, int precision, const double* N,
                               const double* F, const double* n_H, const double* species, const double* T,
                               int64_t n_src, const int64_t* src_cell, const double* src_rate, rt_state** out) {
    if (!out) return rt_fail(RT_EINVAL, "null output handle");
    *out = nullptr;
    if (!mesh_c) return rt_fail(RT_EINVAL, "null mesh");
    rt_mesh* mesh = const_cast<rt_mesh*>(mesh_c);
    if (mesh->device < 0) return rt_fail(RT_EDEVICE, "the mesh was created host-only");
    int rc;
    if ((rc = check_params(params))) return rc;
    if (precision != RT_FP64 && precision != RT_MIXED) return rt_fail(RT_EINVAL, "precision=%d", precision);
    if (n_src < 0) return rt_fail(RT_EINVAL, "n_src=%lld", (long long)n_src);
    DeviceGuard dg(mesh->device);
    const int64_t nc = mesh->nc;
    const int nb = params->nb;
    std::vector<double> hN, hF, hnH, hX, hT, hR;
    std::vector<int64_t> hC;
    if ((rc = fetch(N, (size_t)nb * nc, hN, "N")) || (rc = fetch(F, (size_t)nb * 3 * nc, hF, "F")) ||
        (rc = fetch(n_H, nc, hnH, "n_H")) || (rc = fetch(species, 5 * nc, hX, "species")) ||
        (rc = fetch(T, nc, hT, "T")) || (rc = fetch(src_cell, n_src, hC, "src_cell")) ||
        (rc = fetch(src_rate, (size_t)nb * n_src, hR, "src_rate")))
        return rc;
    for (int64_t q = 0; q < (int64_t)hN.size(); ++q)
        if (!(hN[q] >= 0) || !std::isfinite(hN[q])) return rt_fail(RT_EINVAL, "N[%lld]=%g", (long long)q, hN[q]);
    if (!finite_all(hF)) return rt_fail(RT_EINVAL, "non-finite F");
    for (int64_t i = 0; i < nc; ++i) {
        if (!(hnH[i] > 0) || !std::isfinite(hnH[i])) return rt_fail(RT_EINVAL, "n_H[%lld]=%g", (long long)i, hnH[i]);
        if (!(hT[i] > 0) || !std::isfinite(hT[i])) return rt_fail(RT_EINVAL, "T[%lld]=%g", (long long)i, hT[i]);
        for (int s = 0; s < 5; ++s) {
            double x = hX[s * nc + i];
            if (!(x >= 0 && x <= 1)) return rt_fail(RT_EINVAL, "species[%d][%lld]=%g", s, (long long)i, x);
        }
    }
    for (int64_t k = 0; k < n_src; ++k) {
        if (hC[k] < 0 || hC[k] >= nc) return rt_fail(RT_EINVAL, "src_cell[%lld]=%lld", (long long)k, (long long)hC[k]);
        for (int b = 0; b < nb; ++b) {
            double r = hR[(size_t)b * n_src + k];
            if (!(r >= 0) || !std::isfinite(r)) return rt_fail(RT_EINVAL, "src_rate[%d][%lld]=%g", b, (long long)k, r);
        }
    }
    if (precision == RT_MIXED && (rc = mesh->build_float_geometry())) return rc;
    if ((rc = mesh->build_side_geometry(precision == RT_MIXED ? 4 : 8))) return rc;

    rt_state* s = new (std::nothrow) rt_state();
    if (!s) return rt_fail(RT_ENOMEM, "state handle");
    mesh->refs.fetch_add(1);
    s->mesh = mesh;
    s->params = *params;
    s->cp = chem_params_of(*params);
    s->precision = precision;
    s->nb = nb;
    s->nc = nc;
    s->dt_cfl = params->cfl_eta * mesh->dx_min / params->c_reduced;
    s->n_src = n_src;
    s->src_cell = hC;
    s->src_rate = hR;
    // Per-bin storage scale (power of two: scaling is exact).
    for (int b = 0; b < RT_MAX_BINS; ++b) s->scale[b] = 1.0;
    if (precision == RT_MIXED) {
        for (int b = 0; b < nb; ++b) {
            double mx = 0;
            for (int64_t i = 0; i < nc; ++i) {
                mx = std::max(mx, hN[(size_t)b * nc + i]);
                for (int k = 0; k < 3; ++k) mx = std::max(mx, std::fabs(hF[((size_t)b * 3 + k) * nc + i]) / params->c_reduced);
            }
            for (int64_t k = 0; k < n_src; ++k)
                mx = std::max(mx, hR[(size_t)b * n_src + k] * s->dt_cfl / mesh->vphys[hC[k]]);
            s->scale[b] = pow2_at_least(mx);
        }
    }
    if ((rc = s->alloc_buffers()) || (rc = s->upload_scales()) || (rc = s->upload_sources()) ||
        (!s->fused() && (rc = s->ensure_face_states()))) {
        rt_state_destroy(s);
        return rc;
    }
    // Fields in the internal layout U[b][nc][4] = (N, F/c~) / scale.
    {
        std::vector<double> U((size_t)nb * 4 * nc);
        for (int b = 0; b < nb; ++b) {
            const double inv = 1.0 / s->scale[b];
            for (int64_t i = 0; i < nc; ++i) {
                U[urec(b, nc, i)] = hN[(size_t)b * nc + i] * inv;
                for (int k = 0; k < 3; ++k)
                    U[urec(b, nc, i) + 1 + k] = hF[((size_t)b * 3 + k) * nc + i] / params->c_reduced * inv;
            }
        }
        hipError_t e;
        if (precision == RT_MIXED) {
            std::vector<float> Uf(U.size());
            for (size_t q = 0; q < U.size(); ++q) Uf[q] = (float)U[q];
            e = hipMemcpy(s->U[0].ptr, Uf.data(), Uf.size() * 4, hipMemcpyHostToDevice);
        } else {
            e = hipMemcpy(s->U[0].ptr, U.data(), U.size() * 8, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) { rt_state_destroy(s); return rt_fail(RT_EDEVICE, "upload U: %s", hipGetErrorString(e)); }
        // Thermal energy u = k_B T / ((gamma - 1) mu m_p).
        std::vector<double> ue(nc);
        const double yhe = s->cp.yhe;
        for (int64_t i = 0; i < nc; ++i) {
            const double xe = hX[1 * nc + i] + yhe * (hX[3 * nc + i] + 2.0 * hX[4 * nc + i]);
            const double mu = (1.0 + 4.0 * yhe) / (1.0 + yhe + xe);
            ue[i] = kBoltzH * hT[i] / ((params->gamma - 1.0) * mu * kProtonMassH);
        }
        if ((e = hipMemcpy(s->X.ptr, hX.data(), hX.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(s->Ue.ptr, ue.data(), nc * 8, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(s->nH.ptr, hnH.data(), nc * 8, hipMemcpyHostToDevice)) != hipSuccess) {
            rt_state_destroy(s);
            return rt_fail(RT_EDEVICE, "upload state: %s", hipGetErrorString(e));
        }
    }
    s->cur = 0;
    std::memset(&s->diag, 0, sizeof(s->diag));
    s->diag.dt = s->dt_cfl;
    for (int b = 0; b < RT_MAX_BINS; ++b) s->diag.scale[b] = s->scale[b];
    *out = s;
    return RT_OK;
}

rt_state::~rt_state() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);

    if (h_diag) (void)hipHostFree(h_diag);
}

extern "C" int rt_state_destroy(rt_state* s) {
    if (!s) return rt_fail(RT_EINVAL, "null state");
    rt_mesh* m = s->mesh;
    {
        DeviceGuard dg(m ? m->device : 0);
        delete s;
    }
    rt_mesh_release(m);
    return RT_OK;
}

static int copy_dev(DevMem& dst, const DevMem& src) {
    int rc = dst.alloc(src.bytes);
    if (rc) return rc;
    if (src.bytes) RT_HIP(hipMemcpy(dst.ptr, src.ptr, src.bytes, hipMemcpyDeviceToDevice));
    return RT_OK;
}

extern "C" int rt_state_clone(const rt_state* src, rt_state** out) {
    if (!src || !out) return rt_fail(RT_EINVAL, "null argument");
    *out = nullptr;
    DeviceGuard dg(src->mesh->device);
    rt_state* s = new (std::nothrow) rt_state();
    if (!s) return rt_fail(RT_ENOMEM, "state handle");
    src->mesh->refs.fetch_add(1);
    s->mesh = src->mesh;
    s->params = src->params;
    s->cp = src->cp;
    s->precision = src->precision;
    s->transport_mode = src->transport_mode;
    s->nb = src->nb;
    s->nc = src->nc;
    s->dt_cfl = src->dt_cfl;
    s->n_src = src->n_src;
    s->src_cell = src->src_cell;
    s->src_rate = src->src_rate;
    std::memcpy(s->scale, src->scale, sizeof(s->scale));
    int rc;
    if ((rc = s->alloc_buffers()) || (rc = s->upload_scales()) || (rc = s->upload_sources()) ||
        (rc = copy_dev(s->U[0], src->U[src->cur])) || (rc = copy_dev(s->X, src->X)) ||
        (rc = copy_dev(s->Ue, src->Ue)) || (rc = copy_dev(s->nH, src->nH)) ||
        (!s->fused() && (rc = s->ensure_face_states()))) {
        rt_state_destroy(s);
        return rc;
    }
    s->cur = 0;
    s->diag = src->diag;
    *out = s;
    return RT_OK;
}

// ---------------------------------------------------------------------------
// Subcycle driver
// ---------------------------------------------------------------------------

void rt_state::prof_begin(int kernel, hipStream_t st) {
    if (!prof) return;
    if (ev_used + 2 > ev_pool.size()) {
        for (int q = 0; q < 64; ++q) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            ev_pool.push_back(e);
        }
    }
    prof_open = (int)ev_used;
    prof_kernel = kernel;
    (void)hipEventRecord(ev_pool[ev_used++], st);
}

void rt_state::prof_end(hipStream_t st) {
    if (!prof || prof_open < 0) return;
    (void)hipEventRecord(ev_pool[ev_used++], st);
    ev_marks.push_back({prof_kernel, prof_open});
    prof_open = -1;
}

int rt_state::prof_collect() {
    if (!prof) return RT_OK;
    for (const auto& mk : ev_marks) {
        float ms = 0;
        RT_HIP(hipEventElapsedTime(&ms, ev_pool[mk.second], ev_pool[mk.second + 1]));
        launches[mk.first] += 1;
        total_ms[mk.first] += ms;
    }
    ev_marks.clear();
    ev_used = 0;
    return RT_OK;
}

template <typename T>
static GeomView<T> geom_view(const rt_mesh* m) {
    GeomView<T> geo;
    if (sizeof(T) == 8) {
        geo.face = (const T*)m->d_face64.ptr;
        geo.cell = (const T*)m->d_cell64.ptr;
    } else {
        geo.face = (const T*)m->d_face32.ptr;
        geo.cell = (const T*)m->d_cell32.ptr;
    }
    geo.side = (const T*)(sizeof(T) == 8 ? m->d_side64.ptr : m->d_side32.ptr);
    geo.vol = (const T*)(sizeof(T) == 8 ? m->d_vol64.ptr : m->d_vol32.ptr);
    geo.nf = m->nf;
    geo.ne = m->n_entries;
    return geo;
}

GeomView<double> rt_geo64(const rt_mesh* m) { return geom_view<double>(m); }

SellView rt_sell(const rt_mesh* m) {
    return SellView{(const int32_t*)m->d_nbr.ptr, (const int32_t*)m->d_fsf.ptr, (const int32_t*)m->d_opp.ptr,
                    (const int32_t*)m->d_sptr.ptr, (const int32_t*)m->d_sdeg.ptr, (const int2*)m->d_idx.ptr,
                    (const int32_t*)m->d_fitem_ptr.ptr, (const int2*)m->d_fitem.ptr, m->uniform_deg};
}

// One piece of a subcycle on explicit buffers (U, G in the state's precision).
// Sources of the source cells [src0, src1) of the cell-sorted list (all by
// default).
void rt_step_sources(rt_state* s, void* U, double dt, hipStream_t st, int32_t src0, int32_t src1) {
    if (src1 < 0) src1 = s->n_src_cells;
    const int32_t n = src1 - src0;
    if (n <= 0) return;
    const int32_t* cell = (const int32_t*)s->d_src_cell.ptr + src0;
    const int32_t* ptr = (const int32_t*)s->d_src_ptr.ptr + src0;
    s->prof_begin(RT_KERNEL_SOURCES, st);
    if (s->precision == RT_MIXED)
        launch_sources<float>((float*)U, s->nc, s->nb, n, cell, ptr, (const double*)s->d_src_rate.ptr, s->n_src,
                              (const double*)s->d_src_vphys.ptr, (const double*)s->d_inv_scale.ptr,
                              (const double*)s->d_scale.ptr, dt, st);
    else
        launch_sources<double>((double*)U, s->nc, s->nb, n, cell, ptr, (const double*)s->d_src_rate.ptr, s->n_src,
                               (const double*)s->d_src_vphys.ptr, (const double*)s->d_inv_scale.ptr,
                               (const double*)s->d_scale.ptr, dt, st);
    s->prof_end(st);
}

// Chemistry of cells [cell0, cell1) (all by default), its partials from
// chemistry slot cblk0.
void rt_step_chem(rt_state* s, void* U, double* X, double* Ue, double dt, hipStream_t st, int64_t cell0,
                  int64_t cell1, int64_t cblk0) {
    if (s->params.chem_mode == RT_CHEM_NONE) return;
    if (cell1 < 0) cell1 = s->nc;
    if (cell1 <= cell0) return;
    s->prof_begin(RT_KERNEL_CHEM, st);
    if (s->precision == RT_MIXED)
        launch_chem<float>((float*)U, X, Ue, (const double*)s->nH.ptr, s->nc, cell0, cell1, s->cp, dt,
                           (const double*)s->d_scale.ptr, (const double*)s->d_inv_scale.ptr, s->pb.csum + cblk0,
                           s->pb.cmax + cblk0, s->pb.cst + cblk0, (int32_t*)s->att.ptr, st);
    else
        launch_chem<double>((double*)U, X, Ue, (const double*)s->nH.ptr, s->nc, cell0, cell1, s->cp, dt,
                            (const double*)s->d_scale.ptr, (const double*)s->d_inv_scale.ptr, s->pb.csum + cblk0,
                            s->pb.cmax + cblk0, s->pb.cst + cblk0, (int32_t*)s->att.ptr, st);
    s->prof_end(st);
}

static TileFaceView rt_tile_faces(const rt_mesh* m) {
    return TileFaceView{(const int32_t*)m->d_tpair_ptr.ptr, (const int32_t*)m->d_tpair.ptr,
                        (const int32_t*)m->d_tbnd_ptr.ptr,  (const int32_t*)m->d_tbnd_sptr.ptr,
                        (const int32_t*)m->d_tbnd_opp.ptr,  (const uint8_t*)m->d_bmask.ptr,
                        m->n_bnd(),                         m->tbnd_max};
}

// Whether the split path of a state runs by tile (six-slot meshes with
// compact tiles, where the mesh kept its tile tables): the face-state pass
// then also evaluates the tile-interior faces and applies them to the new
// fields, and the flux pass finishes the update there.
static bool tile_split(const rt_state* s) { return !s->mesh->tpair_ptr.empty(); }

void rt_step_facestate(rt_state* s, const void* U, void* FV, void* Un, hipStream_t st, double dt, bool all_states) {
    s->prof_begin(RT_KERNEL_GRADIENT, st);
    const int64_t nfv = (int64_t)s->nb * 4 * s->mesh->n_entries;   // the cells' cap numerators follow the face states
    const double cdt = s->params.c_reduced * dt / s->mesh->h_ref;
    if (!all_states && tile_split(s)) {
        // boundary-item states [nb][n_bnd][4], then their cap numerators [nb][n_bnd], in FV
        const int64_t nbs = (int64_t)s->nb * 4 * s->mesh->n_bnd();
        if (s->precision == RT_MIXED)
            launch_facestate_tile<float>((const float*)U, (float*)FV, (float*)FV + nbs, (float*)Un, s->nc,
                                         s->nb, geom_view<float>(s->mesh), rt_sell(s->mesh), rt_tile_faces(s->mesh),
                                         s->params.use_limiter, cdt, s->pb.cnt, s->pb.fst, st);
        else
            launch_facestate_tile<double>((const double*)U, (double*)FV, (double*)FV + nbs, (double*)Un, s->nc,
                                          s->nb, geom_view<double>(s->mesh), rt_sell(s->mesh), rt_tile_faces(s->mesh),
                                          s->params.use_limiter, cdt, s->pb.cnt, s->pb.fst, st);
    } else if (s->precision == RT_MIXED) {
        launch_facestate<float>((const float*)U, (float*)FV, (float*)FV + nfv, s->nc, s->nb, s->mesh->n_entries,
                                geom_view<float>(s->mesh), rt_sell(s->mesh), s->params.use_limiter, st);
    } else {
        launch_facestate<double>((const double*)U, (double*)FV, (double*)FV + nfv, s->nc, s->nb, s->mesh->n_entries,
                                 geom_view<double>(s->mesh), rt_sell(s->mesh), s->params.use_limiter, st);
    }
    s->prof_end(st);
}

// Fluxes and update of the whole mesh, from what rt_step_facestate wrote
// (by tile: in place in Un).
void rt_step_flux(rt_state* s, const void* U, const void* FV, void* Un, double dt, hipStream_t st) {
    const int64_t slice0 = 0, slice1 = (int64_t)s->mesh->sdeg.size();
    const double cdt = s->params.c_reduced * dt / s->mesh->h_ref;
    s->prof_begin(RT_KERNEL_FLUX, st);
    const int64_t nfv = (int64_t)s->nb * 4 * s->mesh->n_entries;   // the cells' cap numerators follow the face states
    if (tile_split(s)) {
        const int64_t nbs = (int64_t)s->nb * 4 * s->mesh->n_bnd();
        if (s->precision == RT_MIXED)
            launch_flux_tile<float>((const float*)FV, (const float*)FV + nbs, (float*)Un, s->nc, s->nb,
                                    (const float*)s->mesh->d_vol32.ptr, (const float*)s->mesh->d_bgeo32.ptr,
                                    rt_tile_faces(s->mesh), cdt, s->pb.nv, s->pb.cnt, s->pb.fst, st);
        else
            launch_flux_tile<double>((const double*)FV, (const double*)FV + nbs, (double*)Un, s->nc, s->nb,
                                     (const double*)s->mesh->d_vol64.ptr, (const double*)s->mesh->d_bgeo64.ptr,
                                     rt_tile_faces(s->mesh), cdt, s->pb.nv, s->pb.cnt, s->pb.fst, st);
    } else if (s->precision == RT_MIXED)
        launch_flux<float>((const float*)U, (const float*)FV, (const float*)FV + nfv, (float*)Un, s->nc, s->nb,
                           s->mesh->n_entries, geom_view<float>(s->mesh), rt_sell(s->mesh), cdt, s->pb.nv, s->pb.cnt,
                           s->pb.fst, slice0, slice1, st);
    else
        launch_flux<double>((const double*)U, (const double*)FV, (const double*)FV + nfv, (double*)Un, s->nc, s->nb,
                            s->mesh->n_entries, geom_view<double>(s->mesh), rt_sell(s->mesh), cdt, s->pb.nv,
                            s->pb.cnt, s->pb.fst, slice0, slice1, st);
    s->prof_end(st);
}

TileView rt_tiles(const rt_mesh* m) {
    return TileView{(const int32_t*)m->d_lds_opp.ptr, (const int32_t*)m->d_halo_ptr.ptr,
                    (const int32_t*)m->d_halo_cell.ptr, (const int32_t*)m->d_hside_ptr.ptr,
                    (const int32_t*)m->d_hside_entry.ptr, (int64_t)m->sdeg.size(),
                    (const uint8_t*)m->d_bmask.ptr};
}

// Halo cells per cell up to which AUTO takes the fused path.  The fused
// kernel computes the gradient of every halo cell once more per tile; a
// 256-cell tile of a Hilbert-ordered lattice has 256 halo cells (ratio 1),
// and there the split path is measured faster (the gradient, not the
// face-state traffic, dominates), so AUTO keeps the split path unless the
// halos are much smaller than the tiles.
static constexpr double kMaxHaloRatio = 0.5;

bool rt_state::fused() const {
    if (transport_mode == RT_TRANSPORT_SPLIT) return false;
    if (mesh->tile_lds_bytes(tbytes()) > mesh->lds_limit) return false;
    return transport_mode == RT_TRANSPORT_FUSED || mesh->halo_ratio <= kMaxHaloRatio;
}

void rt_step_transport(rt_state* s, const void* U, void* Un, double dt, hipStream_t st) {
    const double cdt = s->params.c_reduced * dt / s->mesh->h_ref;
    const size_t lds = s->mesh->tile_lds_bytes(s->tbytes());
    s->prof_begin(RT_KERNEL_TRANSPORT, st);
    if (s->precision == RT_MIXED)
        launch_transport<float>((const float*)U, (float*)Un, s->nc, s->nb, geom_view<float>(s->mesh),
                                rt_sell(s->mesh), rt_tiles(s->mesh), lds, s->params.use_limiter, cdt,
                                s->pb.nv, s->pb.cnt, s->pb.fst, st);
    else
        launch_transport<double>((const double*)U, (double*)Un, s->nc, s->nb, geom_view<double>(s->mesh),
                                 rt_sell(s->mesh), rt_tiles(s->mesh), lds, s->params.use_limiter, cdt,
                                 s->pb.nv, s->pb.cnt, s->pb.fst, st);
    s->prof_end(st);
}

void rt_run_subcycles(rt_state* s, int n, double dt, hipStream_t st) {
    const bool fused = s->fused();
    for (int it = 0; it < n; ++it) {
        void* U = s->U[s->cur].ptr;
        void* Un = s->U[s->cur ^ 1].ptr;
        rt_step_sources(s, U, dt, st);
        rt_step_chem(s, U, (double*)s->X.ptr, (double*)s->Ue.ptr, dt, st);
        if (fused) {
            rt_step_transport(s, U, Un, dt, st);
        } else {
            rt_step_facestate(s, U, s->FV.ptr, Un, st, dt, false);
            rt_step_flux(s, U, s->FV.ptr, Un, dt, st);
        }
        s->cur ^= 1;
    }
}

extern "C" int rt_state_set_transport(rt_state* s, int mode) {
    if (!s) return rt_fail(RT_EINVAL, "null state");
    if (mode != RT_TRANSPORT_AUTO && mode != RT_TRANSPORT_FUSED && mode != RT_TRANSPORT_SPLIT)
        return rt_fail(RT_EINVAL, "transport mode %d", mode);
    if (mode == RT_TRANSPORT_FUSED && s->mesh->tile_lds_bytes(s->tbytes()) > s->mesh->lds_limit)
        return rt_fail(RT_ESTATE, "fused transport needs %zu bytes of LDS per workgroup, the device has %zu",
                       s->mesh->tile_lds_bytes(s->tbytes()), s->mesh->lds_limit);
    s->transport_mode = mode;
    DeviceGuard dg(s->mesh->device);
    if (!s->fused()) return s->ensure_face_states();
    return RT_OK;
}

extern "C" int rt_state_transport(const rt_state* s, int32_t* fused) {
    if (!s || !fused) return rt_fail(RT_EINVAL, "null argument");
    *fused = s->fused() ? 1 : 0;
    return RT_OK;
}

void rt_reset_partials(rt_state* s, hipStream_t st) {
    fill_words(s->att.ptr, s->nc, 0, st);
    fill_words(s->pb.cnt, 5 * s->n_fblk * 2, 0, st);
    fill_words(s->pb.fst, s->n_fblk, 0, st);
    fill_words(s->pb.nv, s->n_fblk * 2, 0, st);
    fill_words(s->pb.csum, s->n_cblk * 2, 0, st);
    fill_words(s->pb.cmax, s->n_cblk * 2, 0, st);
    fill_words(s->pb.cst, s->n_cblk, 0, st);
}

int rt_read_status(rt_state* s, hipStream_t st, int* status) {
    launch_reduce(s->pb.nv, s->pb.cnt, s->pb.fst,
                  s->n_fblk, s->nb, s->pb.csum, s->pb.cmax,
                  s->pb.cst, s->n_cblk, (const double*)s->d_nv_scale.ptr, s->pb.red,
                  s->pb.diag,
                  st);
    RT_HIP(hipGetLastError());
    RT_HIP(hipMemcpyAsync(s->h_diag, s->pb.diag, sizeof(DiagDev), hipMemcpyDeviceToHost, st));
    RT_HIP(hipStreamSynchronize(st));
    *status = s->h_diag->status;
    return RT_OK;
}

int rt_subcycle_run(rt_state* s, int n, double step, hipStream_t st, bool rollback) {
    const size_t t = s->tbytes();
    const size_t ubytes = (size_t)s->nb * 4 * s->nc * t;
    int rc;
    const int cur0 = s->cur;
    if (rollback) {
        // Entry copy for roll-back on error.
        if ((!s->bU.ptr && (rc = s->bU.alloc(ubytes))) || (!s->bX.ptr && (rc = s->bX.alloc(5 * s->nc * 8))) ||
            (!s->bUe.ptr && (rc = s->bUe.alloc(s->nc * 8))))
            return rc;
        RT_HIP(hipMemcpyAsync(s->bU.ptr, s->U[cur0].ptr, ubytes, hipMemcpyDeviceToDevice, st));
        RT_HIP(hipMemcpyAsync(s->bX.ptr, s->X.ptr, 5 * s->nc * 8, hipMemcpyDeviceToDevice, st));
        RT_HIP(hipMemcpyAsync(s->bUe.ptr, s->Ue.ptr, s->nc * 8, hipMemcpyDeviceToDevice, st));
    }
    if (!s->fused() && !s->FV.ptr) return rt_fail(RT_ESTATE, "the split transport path has no face-state buffer");
    rt_reset_partials(s, st);
    rt_run_subcycles(s, n, step, st);
    s->prof_begin(RT_KERNEL_REDUCE, st);
    launch_reduce(s->pb.nv, s->pb.cnt, s->pb.fst, s->n_fblk, s->nb, s->pb.csum, s->pb.cmax, s->pb.cst, s->n_cblk,
                  (const double*)s->d_nv_scale.ptr, s->pb.red, s->pb.diag, st);
    s->prof_end(st);
    RT_HIP(hipGetLastError());
    RT_HIP(hipMemcpyAsync(s->h_diag, s->pb.diag, sizeof(DiagDev), hipMemcpyDeviceToHost, st));
    RT_HIP(hipStreamSynchronize(st));
    if ((rc = s->prof_collect())) return rc;
    const DiagDev& d = *s->h_diag;
    rt_diag& o = s->diag;
    o.dt = step;
    for (int b = 0; b < RT_MAX_BINS; ++b) {
        o.photon_sum[b] = b < s->nb ? d.photon_sum[b] : 0.0;
        o.scale[b] = s->scale[b];
    }
    o.adm_N = d.counters[0]; o.adm_F = d.counters[1]; o.flux_caps = d.counters[2];
    o.guard_N = d.counters[3]; o.guard_F = d.counters[4];
    o.substeps = d.substeps; o.max_substeps = d.max_substeps;
    o.status = d.status;
    o.n_subcycles = n;
    if (n > 0 && d.status != 0) {
        const char* what = (d.status & 1) ? ((d.status & 2) ? "non-finite value, chemistry substep cap"
                                                             : "non-finite value")
                                          : "chemistry substep cap";
        if (!rollback) return rt_fail(RT_ENUMERIC, "subcycle status 0x%x (%s); state not restored", d.status, what);
        // Roll back to the entry state.
        s->cur = cur0;
        RT_HIP(hipMemcpyAsync(s->U[cur0].ptr, s->bU.ptr, ubytes, hipMemcpyDeviceToDevice, st));
        RT_HIP(hipMemcpyAsync(s->X.ptr, s->bX.ptr, 5 * s->nc * 8, hipMemcpyDeviceToDevice, st));
        RT_HIP(hipMemcpyAsync(s->Ue.ptr, s->bUe.ptr, s->nc * 8, hipMemcpyDeviceToDevice, st));
        RT_HIP(hipStreamSynchronize(st));
        return rt_fail(RT_ENUMERIC, "subcycle status 0x%x (%s); state restored", d.status, what);
    }
    return RT_OK;
}

extern "C" int rt_subcycle(rt_state* s, int n, double dt, void* hip_stream) {
    if (!s) return rt_fail(RT_EINVAL, "null state");
    if (n < 0) return rt_fail(RT_EINVAL, "n_subcycles=%d", n);
    if (!(dt <= 0) && !(dt <= s->dt_cfl)) return rt_fail(RT_EINVAL, "dt=%g above the CFL step %g", dt, s->dt_cfl);
    if (!std::isfinite(dt)) return rt_fail(RT_EINVAL, "dt=%g", dt);
    DeviceGuard dg(s->mesh->device);
    int rc;
    if (!s->fused() && (rc = s->ensure_face_states())) return rc;
    return rt_subcycle_run(s, n, dt <= 0 ? s->dt_cfl : dt, (hipStream_t)hip_stream, true);
}

// ---------------------------------------------------------------------------
// Fields, info, diagnostics, profiling
// ---------------------------------------------------------------------------

static size_t field_count(const rt_state* s, int field) {
    switch (field) {
        case RT_FIELD_N: return (size_t)s->nb * s->nc;
        case RT_FIELD_F: return (size_t)s->nb * 3 * s->nc;
        case RT_FIELD_NH: return s->nc;
        case RT_FIELD_SPECIES: return 5 * s->nc;
        case RT_FIELD_T: return s->nc;
        case RT_FIELD_ATTEMPTS: return s->nc;
        default: return 0;
    }
}

extern "C" int rt_state_get_field(const rt_state* s, int field, double* out, int out_on_device) {
    (void)out_on_device;
    if (!s || !out) return rt_fail(RT_EINVAL, "null argument");
    const size_t n = field_count(s, field);
    if (!n) return rt_fail(RT_EINVAL, "field=%d", field);
    DeviceGuard dg(s->mesh->device);
    if (field == RT_FIELD_NH) { RT_HIP(hipMemcpy(out, s->nH.ptr, n * 8, hipMemcpyDefault)); return RT_OK; }
    if (field == RT_FIELD_SPECIES) { RT_HIP(hipMemcpy(out, s->X.ptr, n * 8, hipMemcpyDefault)); return RT_OK; }
    if (field == RT_FIELD_ATTEMPTS) {
        std::vector<int32_t> a(n);
        RT_HIP(hipMemcpy(a.data(), s->att.ptr, n * 4, hipMemcpyDeviceToHost));
        std::vector<double> d(a.begin(), a.end());
        RT_HIP(hipMemcpy(out, d.data(), n * 8, hipMemcpyDefault));
        return RT_OK;
    }
    DevMem tmp;
    int rc = tmp.alloc(n * 8);
    if (rc) return rc;
    if (s->precision == RT_MIXED)
        launch_get_fields<float>((const float*)s->U[s->cur].ptr, (const double*)s->X.ptr, (const double*)s->Ue.ptr,
                                 s->nc, s->nb, field, (const double*)s->d_scale.ptr, s->params.c_reduced, s->cp,
                                 (double*)tmp.ptr, nullptr);
    else
        launch_get_fields<double>((const double*)s->U[s->cur].ptr, (const double*)s->X.ptr, (const double*)s->Ue.ptr,
                                  s->nc, s->nb, field, (const double*)s->d_scale.ptr, s->params.c_reduced, s->cp,
                                  (double*)tmp.ptr, nullptr);
    RT_HIP(hipGetLastError());
    RT_HIP(hipMemcpy(out, tmp.ptr, n * 8, hipMemcpyDefault));
    return RT_OK;
}

extern "C" int rt_state_set_field(rt_state* s, int field, const double* in, int in_on_device) {
    (void)in_on_device;
    if (!s || !in) return rt_fail(RT_EINVAL, "null argument");
    if (field == RT_FIELD_NH) return rt_fail(RT_EINVAL, "n_H is fixed at create time");
    if (field == RT_FIELD_ATTEMPTS) return rt_fail(RT_EINVAL, "the attempt counts are read only");
    const size_t n = field_count(s, field);
    if (!n) return rt_fail(RT_EINVAL, "field=%d", field);
    DeviceGuard dg(s->mesh->device);
    std::vector<double> h;
    int rc = fetch(in, n, h, "field");
    if (rc) return rc;
    if (!finite_all(h)) return rt_fail(RT_EINVAL, "non-finite field values");
    if (field == RT_FIELD_SPECIES) {
        for (double x : h)
            if (!(x >= 0 && x <= 1)) return rt_fail(RT_EINVAL, "species outside [0, 1]");
        RT_HIP(hipMemcpy(s->X.ptr, h.data(), n * 8, hipMemcpyHostToDevice));
        return RT_OK;
    }
    if (field == RT_FIELD_N)
        for (double x : h)
            if (!(x >= 0)) return rt_fail(RT_EINVAL, "negative N");
    if (field == RT_FIELD_T)
        for (double x : h)
            if (!(x > 0)) return rt_fail(RT_EINVAL, "non-positive T");
    DevMem tmp;
    if ((rc = tmp.upload(h.data(), n * 8))) return rc;
    if (s->precision == RT_MIXED)
        launch_set_fields<float>((float*)s->U[s->cur].ptr, (const double*)s->X.ptr, (double*)s->Ue.ptr, s->nc, s->nb,
                                 field, (const double*)s->d_inv_scale.ptr, s->params.c_reduced, s->cp,
                                 (const double*)tmp.ptr, nullptr);
    else
        launch_set_fields<double>((double*)s->U[s->cur].ptr, (const double*)s->X.ptr, (double*)s->Ue.ptr, s->nc, s->nb,
                                  field, (const double*)s->d_inv_scale.ptr, s->params.c_reduced, s->cp,
                                  (const double*)tmp.ptr, nullptr);
    RT_HIP(hipGetLastError());
    RT_HIP(hipDeviceSynchronize());
    return RT_OK;
}

extern "C" int rt_state_info(const rt_state* s, int64_t* n_cells, int32_t* nb, int64_t* n_src, int32_t* precision,
                             double* dt_cfl) {
    if (!s) return rt_fail(RT_EINVAL, "null state");
    if (n_cells) *n_cells = s->nc;
    if (nb) *nb = s->nb;
    if (n_src) *n_src = s->n_src;
    if (precision) *precision = s->precision;
    if (dt_cfl) *dt_cfl = s->dt_cfl;
    return RT_OK;
}

extern "C" int rt_state_diagnostics(const rt_state* s, rt_diag* out) {
    if (!s || !out) return rt_fail(RT_EINVAL, "null argument");
    *out = s->diag;
    return RT_OK;
}

extern "C" int rt_profile_enable(rt_state* s, int enable) {
    if (!s) return rt_fail(RT_EINVAL, "null state");
    s->prof = enable != 0;
    return RT_OK;
}

extern "C" int rt_profile_reset(rt_state* s) {
    if (!s) return rt_fail(RT_EINVAL, "null state");
    for (int k = 0; k < RT_N_KERNELS; ++k) { s->launches[k] = 0; s->total_ms[k] = 0; }
    return RT_OK;
}

extern "C" int rt_profile_read(const rt_state* s, int kernel, int64_t* launches, double* total_ms) {
    if (!s || kernel < 0 || kernel >= RT_N_KERNELS) return rt_fail(RT_EINVAL, "bad argument");
    if (launches) *launches = s->launches[kernel];
    if (total_ms) *total_ms = s->total_ms[kernel];
    return RT_OK;
}
