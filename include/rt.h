/*
 * rt.h -- C ABI of the M1 radiative-transfer subcycle on one MI355X (gfx950).
 *
 * The library advances the photon fields and the gas chemistry of a static
 * mesh by radiative-transfer subcycles, as in Zier et al. (2024), "Adapting
 * AREPO-RT for Exascale Computing", Sections 2.2-2.3 and 4.1: the M1 moment
 * equations (eq. E, eq. F) for the photon number density N_b and flux F_b of
 * each frequency bin, closed by the M1 Eddington tensor (eq. edd) and written
 * in finite-volume form (eq. RT_flux); the per-cell non-equilibrium H/He
 * thermochemistry of Section 2.3.1 integrated with the adaptive semi-implicit
 * scheme of Section 4.1.1.  One subcycle is, in the order of Fig. 1:
 * point sources, thermochemistry, gradients (Sec. 2.3.2), fluxes and update
 * (Sec. 2.3.3).
 *
 * Conventions
 *  - Every function returns an int status: RT_OK (0) or a negative RT_E*
 *    code; rt_last_error() returns a thread-local message for the last
 *    failure on the calling thread.
 *  - Arrays are structure-of-arrays in the CALLER's cell and face order
 *    ("[3][nc]" = three contiguous arrays of nc values).  The library never
 *    reorders cells: a locality-friendly order (e.g. Peano-Hilbert) is the
 *    caller's choice.  Units are cgs.
 *  - Input pointers may be host or device memory (detected per pointer); the
 *    library copies every input at create time and the caller keeps
 *    ownership of its buffers.
 *  - Handles are owned by the caller until destroyed.  A state keeps its mesh
 *    alive: destroying a mesh that still has states only drops the caller's
 *    reference.
 *  - On any error a state is left unchanged.
 *  - Calls on one state are not thread-safe; distinct states may be used from
 *    distinct threads.
 */
#ifndef RT_H
#define RT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define RT_OK        0
#define RT_EINVAL   -1   /* bad argument (null pointer, size, parameter out of range, dt above the CFL step) */
#define RT_EMESH    -2   /* bad mesh: index out of range, L == R, V <= 0, A <= 0, |n| != 1 +- 1e-12,
                            a cell with fewer than 4 faces, or cond(M_i) > 1e12 */
#define RT_ESTATE   -3   /* state/mesh mismatch, or an operation the state does not support */
#define RT_EDEVICE  -4   /* HIP runtime error */
#define RT_ENOMEM   -5   /* allocation failure */
#define RT_ENUMERIC -6   /* a non-finite value appeared, or a cell hit the chemistry substep cap */

/* ---- enumerations ---------------------------------------------------- */
#define RT_MAX_BINS 8

#define RT_FP64  0        /* transport, chemistry and sums in FP64 */
#define RT_MIXED 1        /* transport in FP32 with per-bin power-of-two scaling of N and F;
                             chemistry, flux sums and photon sums in FP64 (Sec. 6.2) */

#define RT_CHEM_NONE 0    /* transport only (no absorption, no chemistry) */
#define RT_CHEM_H    1    /* hydrogen only */
#define RT_CHEM_HHE  2    /* hydrogen and helium */

#define RT_RATES_CASEB_CONST 0   /* constant case-B recombination alpha_B_const, no collisional
                                    ionisation, no cooling; hydrogen only, isothermal */
#define RT_RATES_HG97        1   /* Hui & Gnedin (1997) case-B recombination, collisional ionisation
                                    and their cooling; Cen (1992) dielectronic recombination,
                                    collisional-excitation cooling and free-free emission */

/* Fields for rt_state_get_field / rt_state_set_field (FP64, caller order). */
#define RT_FIELD_N       0   /* [nb][nc]    photon number density, cm^-3 */
#define RT_FIELD_F       1   /* [nb][3][nc] photon flux, cm^-2 s^-1 */
#define RT_FIELD_NH      2   /* [nc]        hydrogen number density, cm^-3 (get only) */
#define RT_FIELD_SPECIES 3   /* [5][nc]     x_HI, x_HII, y_HeI, y_HeII, y_HeIII */
#define RT_FIELD_T       4   /* [nc]        gas temperature, K */
#define RT_FIELD_ATTEMPTS 5  /* [nc]        chemistry step attempts of each cell (accepted and rejected,
                                            Sec. 4.1.1), summed over the subcycles of the last
                                            rt_subcycle call (get only) */

/* Kernel ids for the profiling counters. */
#define RT_KERNEL_SOURCES  0
#define RT_KERNEL_CHEM     1
#define RT_KERNEL_GRADIENT 2
#define RT_KERNEL_FLUX     3
#define RT_KERNEL_REDUCE   4
#define RT_KERNEL_TRANSPORT 5   /* fused gradient + face states + fluxes */
#define RT_N_KERNELS       6

/* Transport path (rt_state_set_transport).  The split path runs the
 * gradient/face-state kernel and the flux kernel with the face states in
 * device memory; the fused path runs both per 256-cell tile in one kernel
 * with the face states in LDS.  Both sum a cell's face fluxes in the same
 * order and round the update at the same points, so they give the same
 * fields bit for bit. */
#define RT_TRANSPORT_AUTO  0   /* fused when the tiles fit in LDS and their halos are
                                  at most half the tile size, else split */
#define RT_TRANSPORT_FUSED 1   /* fused whenever the tiles fit in LDS */
#define RT_TRANSPORT_SPLIT 2   /* always split */

/* ---- parameters ------------------------------------------------------ */
/* Every constant the paper leaves open.  rt_params_default fills the values
 * used throughout (eta = 0.3 per eq. timestep; f_max = 0.1, f_s = 0.05 and the
 * doubling cap per Sec. 4.1.1). */
typedef struct rt_params {
    int32_t nb;                 /* frequency bins, 1..RT_MAX_BINS */
    int32_t chem_mode;          /* RT_CHEM_* */
    int32_t isothermal;         /* 1: T fixed at T_iso, no energy equation */
    int32_t rate_set;           /* RT_RATES_* */
    int32_t use_limiter;        /* 1: slope limiter on (Sec. 2.3.2) */
    int32_t chem_max_substeps;  /* attempts per cell and subcycle before RT_ENUMERIC */
    int32_t chem_cells_per_lane;/* cells per lane in each chemistry workgroup's share, which its
                                   lanes draw from as they finish cells (lane refill): 0 =
                                   automatic (up to 32, keeping about 1024 workgroups); 1 = one
                                   cell per lane, no refill; at most 1024.  Results do not
                                   depend on it. */
    int32_t reserved0;          /* 0 */
    double c_reduced;           /* reduced speed of light c~, cm/s (Sec. 2.2, RSLA) */
    double cfl_eta;             /* Courant number eta (eq. timestep) */
    double T_iso;               /* K, isothermal runs */
    double Y_He;                /* helium mass fraction (RT_CHEM_HHE) */
    double alpha_B_const;       /* cm^3/s, RT_RATES_CASEB_CONST */
    double gamma;               /* adiabatic index */
    double chem_fmax;           /* reject a chemistry step if the largest relative change exceeds this */
    double chem_fs;             /* target relative change per step */
    double chem_growth;         /* largest step growth factor between steps */
    double chem_xfloor;         /* floor of the fraction in the relative-change denominator */
    double sigma[RT_MAX_BINS][3];   /* mean cross-section per bin for HI, HeI, HeII, cm^2 */
    double e_heat[RT_MAX_BINS][3];  /* mean excess energy per absorption, erg */
} rt_params;

/* Diagnostics of the last rt_subcycle call (sums over its subcycles). */
typedef struct rt_diag {
    double dt;                          /* subcycle length used, s */
    double photon_sum[RT_MAX_BINS];     /* sum_i N_i V_i per bin after the call (FP64) */
    double scale[RT_MAX_BINS];          /* per-bin FP32 storage scale (RT_MIXED), 1 in RT_FP64 */
    int64_t guard_N, guard_F;           /* post-update clamps N < 0 and |F|/c~ > N */
    int64_t adm_N, adm_F;               /* face-state admissibility fixes, counted once per face */
    int64_t flux_caps;                  /* faces whose outflow cap was active */
    int64_t substeps;                   /* chemistry step attempts, summed over cells */
    int64_t max_substeps;               /* largest attempts of one cell in one subcycle */
    int32_t status;                     /* bit 0: non-finite value, bit 1: substep cap */
    int32_t n_subcycles;                /* subcycles in the call */
} rt_diag;

typedef struct rt_mesh rt_mesh;
typedef struct rt_state rt_state;

/* Message of the last failure on this thread ("" if none). */
const char* rt_last_error(void);

/* Fill *p with the defaults for nb bins (hydrogen, isothermal 1e4 K, rate set
 * 0, c~ = 0.01 c, eta = 0.3, limiter on, controller 0.1 / 0.05 / 2 / 1e-6 /
 * 1e5, gamma = 5/3, zero cross-sections). */
int rt_params_default(int32_t nb, rt_params* p);

/* `device` value of rt_mesh_create that builds and validates the mesh's
 * host tables only (for inspection with rt_mesh_table; no state can be
 * created on such a mesh). */
#define RT_DEVICE_HOST_ONLY (-1)

/* Create a static mesh on HIP device `device`.
 *   volume [nc] cm^3, centre [3][nc] cm (the point gradients are taken about,
 *   s_i of Sec. 2.3.2), face_cells [2][nf] (L, R) cell indices, area [nf] cm^2,
 *   normal [3][nf] unit normal pointing from L to R, face_centre [3][nf] cm,
 *   box[3] periodic box lengths (0 = open axis; offsets use the minimum image).
 * Precomputes the minimum-image face offsets, the least-squares geometry
 * matrices M_i = sum_j A_ij n_ji n_ji^T and their inverses (Sec. 2.3.2: the
 * matrix depends on geometry only and is reused between subcycles), the
 * per-cell face lists in face-index order (Sec. 4.1.4) and the CFL length
 * (3V/4pi)^(1/3) (eq. timestep).  Every cell must have between 4 and 4096
 * faces.  Errors: RT_EINVAL, RT_EMESH, RT_EDEVICE, RT_ENOMEM. */
int rt_mesh_create(int64_t n_cells, const double* volume, const double* centre,
                   int64_t n_faces, const int64_t* face_cells, const double* area,
                   const double* normal, const double* face_centre, const double box[3],
                   int device, rt_mesh** out);
int rt_mesh_destroy(rt_mesh* mesh);

/* Read-only view of one of the mesh's int32 index tables (host memory owned
 * by the mesh, valid until rt_mesh_destroy).  Sliced ELL with 64-cell
 * slices: slice s holds sdeg[s] slots from sptr[s]; slot k of cell i is entry
 * sptr[i/64] + 64 k + i%64, with nbr (neighbour, -1 for padding), fsf (face
 * index f, or ~f when the cell is the face's R cell) and opp (the entry of
 * the same face in the neighbour's slots).  Tiles of the fused transport
 * kernel (cells T t .. T t + T - 1 with T = RT_TILE_CELLS, face states in
 * LDS): lds_opp (LDS slot of the opposite state of each entry; the tile's
 * own entries occupy slots 0 .. ptr[(t+1) T/64] - ptr[t T/64] - 1 in entry
 * order, its halo sides follow),
 * halo_ptr [n_tiles + 1] into halo_cell (cells outside the tile that share
 * a face with it), hside_ptr [n_halo + 1] into hside_entry (the entries of
 * each halo cell that face the tile, in the order of their LDS slots). */
#define RT_TILE_CELLS        256   /* cells per tile of the fused transport kernel */
#define RT_TABLE_NBR         0
#define RT_TABLE_FSF         1
#define RT_TABLE_OPP         2
#define RT_TABLE_SPTR        3
#define RT_TABLE_SDEG        4
#define RT_TABLE_LDS_OPP     5
#define RT_TABLE_HALO_PTR    6
#define RT_TABLE_HALO_CELL   7
#define RT_TABLE_HSIDE_PTR   8
#define RT_TABLE_HSIDE_ENTRY 9
/* Face evaluations of the flux kernel on meshes whose slices all have 6 or
 * 14 slots (empty otherwise): slice s evaluates items fitem_ptr[s] ..
 * fitem_ptr[s+1] - 1; item q is the pair fitem[2q], fitem[2q+1]: the entry,
 * with bit 30 set when the face's other side is in the same slice
 * (evaluated once, from its L side), and the opposite entry (complemented
 * for an R side). */
#define RT_TABLE_FITEM_PTR   10
#define RT_TABLE_FITEM       11
/* Faces of the split transport on meshes whose slices all have 6 slots
 * (empty otherwise), by tile of RT_TILE_CELLS cells: tile t's faces with
 * both sides in the tile are tpair[tpair_ptr[t] .. tpair_ptr[t+1]), each the
 * L side's entry relative to the tile's first entry (6 RT_TILE_CELLS t) in
 * the low 16 bits and the R side's in the high 16 bits.  The face sides
 * whose face crosses to another tile are the boundary items q, numbered in
 * entry order: tbnd[2q] is the entry and tbnd[2q+1] the opposite side's item
 * (complemented for an R side); tile t holds items tbnd_ptr[t] ..
 * tbnd_ptr[t+1] - 1 and slice s items tbnd_sptr[s] .. tbnd_sptr[s+1] - 1. */
#define RT_TABLE_TPAIR_PTR   12
#define RT_TABLE_TPAIR       13
#define RT_TABLE_TBND_PTR    14
#define RT_TABLE_TBND        15
#define RT_TABLE_TBND_SPTR   16
int rt_mesh_table(const rt_mesh* mesh, int table, const int32_t** data, int64_t* length);

/* Create a radiation + gas state on a mesh.
 *   precision: RT_FP64 or RT_MIXED.
 *   N [nb][nc] photon number density (cm^-3), F [nb][3][nc] photon flux
 *   (cm^-2 s^-1; |F| <= c~ N), n_H [nc] (cm^-3), species [5][nc] = x_HI,
 *   x_HII, y_HeI, y_HeII, y_HeIII (helium fractions of helium), T [nc] (K).
 *   Sources: src_cell [n_src] cell indices, src_rate [nb][n_src] photons/s.
 * The subcycle length is the global CFL step eta min_i (3V_i/4pi)^(1/3) / c~
 * (eq. timestep with v_c = 0), computed here by a device min-reduction.
 * Errors: RT_EINVAL (parameters or arrays), RT_EDEVICE, RT_ENOMEM. */
int rt_state_create(const rt_mesh* mesh, const rt_params* params, int precision,
                    const double* N, const double* F, const double* n_H,
                    const double* species, const double* T,
                    int64_t n_src, const int64_t* src_cell, const double* src_rate,
                    rt_state** out);
/* Deep copy of a state (same mesh, parameters, sources and fields). */
int rt_state_clone(const rt_state* state, rt_state** out);
int rt_state_destroy(rt_state* state);

/* Advance n_subcycles subcycles on `hip_stream` (a hipStream_t; NULL = the
 * null stream).  dt <= 0 selects the CFL step; dt above it is RT_EINVAL.
 * Each subcycle: sources, chemistry, gradients, fluxes and update.  The call
 * synchronises the stream once at the end to read the status word; on
 * RT_ENUMERIC the state is restored to its value at entry. */
int rt_subcycle(rt_state* state, int n_subcycles, double dt, void* hip_stream);

/* rt_subcycle for callers that cannot allocate device memory during the call
 * (code under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as rt_subcycle (bit for
 * bit), with two differences:
 *  - the per-workgroup partials, reduction records and diagnostics record
 *    live in one static device array of RT_NOALLOC_SCRATCH_MB MiB per device
 *    (held until the process ends) instead of the state's buffers; a state
 *    whose partials need more (52 bytes per 64 cells and bin: about 80 M
 *    cells x bins at 64 MiB) is RT_EINVAL, and rt_subcycle serves it;
 *  - no entry copy is kept: on RT_ENUMERIC the state is left as the failing
 *    subcycle left it (rt_subcycle restores it).
 * Every call on one device shares that array: calls that overlap on one
 * device (several host threads, or several streams in flight) race.  The
 * call synchronises `hip_stream` once at the end, like rt_subcycle.  The
 * state's fields and its face-state buffer are allocated when it is created
 * (or switched to the split path by rt_state_set_transport), so the call
 * allocates nothing; profiling (rt_profile_enable) is ignored for it. */
#define RT_NOALLOC_SCRATCH_MB 64
int rt_subcycle_noalloc(rt_state* state, int n_subcycles, double dt, void* hip_stream);

/* Reverse-mode derivative of L(x_HI after n_subcycles of length dt from
 * `initial`) given dL/dx_HI [nc] of the final state (host or device); dt as
 * in rt_subcycle (<= 0: the CFL step; above it: RT_EINVAL), so the gradient
 * is that of the run the caller made:
 *   dL_dlnQ [n_src]  derivative with respect to the log of each source's rate
 *                    (all bins of a source scaled together),
 *   dL_dln_nH [nc]   derivative with respect to the log of the initial n_H.
 * Outputs may be host or device memory.  The forward pass is recomputed from
 * checkpoints taken every `checkpoint_every` subcycles; `initial` is not
 * modified.  FP64 states only (RT_ESTATE otherwise). */
int rt_subcycle_adjoint(const rt_state* initial, int n_subcycles, int checkpoint_every, double dt,
                        const double* dL_dxHI_final, double* dL_dlnQ, double* dL_dln_nH,
                        void* hip_stream);

/* Copy a field out (FP64, caller order) to host or device memory, or set one
 * (RT_FIELD_N, _F, _SPECIES, _T).  Synchronous. */
int rt_state_get_field(const rt_state* state, int field, double* out, int out_on_device);
int rt_state_set_field(rt_state* state, int field, const double* in, int in_on_device);

/* Sizes and the subcycle length of a state. */
int rt_state_info(const rt_state* state, int64_t* n_cells, int32_t* nb, int64_t* n_src,
                  int32_t* precision, double* dt_cfl);

/* Choose the transport path of a state (RT_TRANSPORT_*; default AUTO).
 * RT_ESTATE if RT_TRANSPORT_FUSED is asked for and the mesh's tiles do not
 * fit in the device's LDS at the state's precision.  rt_state_transport
 * reports the path the next subcycle takes (1 fused, 0 split).  The adjoint
 * recomputes its forward pass on the split path. */
int rt_state_set_transport(rt_state* state, int mode);
int rt_state_transport(const rt_state* state, int32_t* fused);

/* Diagnostics of the last rt_subcycle call. */
int rt_state_diagnostics(const rt_state* state, rt_diag* out);

/* Per-kernel timing: when enabled, every kernel launch of rt_subcycle is
 * bracketed by HIP events on the caller's stream; rt_profile_read returns the
 * number of launches and the summed duration (ms) of kernel `kernel`
 * (RT_KERNEL_*) since the last reset. */
int rt_profile_enable(rt_state* state, int enable);
int rt_profile_reset(rt_state* state);
int rt_profile_read(const rt_state* state, int kernel, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */
