/*
 * Plain FP64 CPU oracle of the M1 radiative-transfer subcycle.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a slow, obviously correct statement of the method.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product path never does.  It shares no code, header, constant or
 * helper with the GPU library.
 *
 * Method (Zier et al. 2024, Section 2.2-2.3, following Kannan et al. 2019):
 * photon number density N_b and reduced flux Fh_b = F_b / c~ per frequency
 * bin on a static mesh; per subcycle, in the order of Fig. 1:
 *   O1 point sources            N += Q dt / V
 *   O2 thermochemistry          adaptive semi-implicit H/He network (Sec. 2.3.1, 4.1.1)
 *   O3 gradients + limiter      weighted least squares (Sec. 2.3.2, eq. normalEquation)
 *   O4 face fluxes              extrapolate, M1 closure (eq. edd), HLL (Sec. 2.3.3)
 *   O5 update                   finite-volume divergence (Sec. 2.1, eq. RT_flux)
 *   O6 diagnostics              per-bin sum of N V
 * All arrays are SoA in the caller's cell order, cgs units.
 */
#ifndef M1RT_ORACLE_H
#define M1RT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_MAX_BINS 8

enum { OR_CHEM_NONE = 0, OR_CHEM_H = 1, OR_CHEM_HHE = 2 };
enum { OR_RATES_CASEB_CONST = 0, OR_RATES_HG97 = 1 };

typedef struct oracle_params {
    int32_t nb, chem_mode, isothermal, rate_set, use_limiter, chem_max_substeps;
    double c_reduced, cfl_eta, T_iso, Y_He, alpha_B_const, gamma;
    double chem_fmax, chem_fs, chem_growth, chem_xfloor;
    double sigma[ORACLE_MAX_BINS][3];   /* cm^2, species HI, HeI, HeII */
    double e_heat[ORACLE_MAX_BINS][3];  /* erg per absorption */
} oracle_params;

typedef struct oracle_mesh {
    int64_t nc;
    const double* volume;       /* [nc] */
    const double* centre;       /* [3][nc] */
    int64_t nf;
    const int64_t* face_cells;  /* [2][nf] (L, R) */
    const double* area;         /* [nf] */
    const double* normal;       /* [3][nf] unit, L -> R */
    const double* face_centre;  /* [3][nf] */
    double box[3];              /* periodic lengths, 0 = open */
} oracle_mesh;

/* Per-run counters; sums are taken after the last subcycle. */
typedef struct oracle_diag {
    double dt;
    double photon_sum[ORACLE_MAX_BINS];   /* sum_i N_i V_i per bin */
    int64_t guard_N, guard_F;             /* post-update clamps */
    int64_t adm_N, adm_F;                 /* face-state admissibility fixes */
    int64_t flux_caps;                    /* faces with theta < 1 */
    int64_t substeps, max_substeps;       /* chemistry attempts (total, max per cell-subcycle) */
    int32_t status;                       /* 0 ok, -6 substep cap hit */
    double loop_seconds;                  /* wall time of the subcycle loop (steady clock) */
} oracle_diag;

/* Host threads of the subcycle loop (default 1).  With more than one, the
 * per-cell loops are shared out and the face loop becomes a pass over the
 * faces and a per-cell pass that adds each cell's faces in face-index order:
 * the results are the same bit for bit.  Returns 0, or -1 for n < 1. */
int oracle_set_threads(int n);

/* Global CFL step eta * min (3V/4pi)^(1/3) / c~ (eq. timestep, v_c = 0). */
double oracle_cfl_dt(const oracle_mesh* m, const oracle_params* p);

/* Run n_sub subcycles in place.  N [nb][nc], F [nb][3][nc] (cgs photon flux),
 * species [5][nc] = x_HI, x_HII, y_HeI, y_HeII, y_HeIII, T [nc] K.
 * dt <= 0 selects the CFL step.  Returns 0, -1 (bad argument) or -6. */
int oracle_run(const oracle_mesh* m, const oracle_params* p,
               double* N, double* F, const double* n_H, double* species, double* T,
               int64_t n_src, const int64_t* src_cell, const double* src_rate,
               int n_sub, double dt, oracle_diag* diag);

/* Forward-mode derivative of the same run along n_dir directions of
 * (ln Q per source, ln n_H per cell): dlnQ [n_dir][n_src], dln_nH [n_dir][nc].
 * Writes the directional derivatives of the final x_HI into dxHI [n_dir][nc]
 * and advances the primal state like oracle_run.  The derivative is that of
 * the executed branch path, with three values held constant (derivative
 * zero): the direction of a nearly isotropic flux (|Fh|^2 <= 1e-16 N^2, where
 * the Eddington tensor is taken as I/3), the outflow cap's factor where the
 * face's flux of N is rounding noise, and the state and limited gradient of
 * a cell whose N is not above 1e-20 of its bin's largest at the start of a
 * transport step. */
int oracle_run_jvp(const oracle_mesh* m, const oracle_params* p,
                   double* N, double* F, const double* n_H, double* species, double* T,
                   int64_t n_src, const int64_t* src_cell, const double* src_rate,
                   int n_sub, double dt, int n_dir, const double* dlnQ, const double* dln_nH,
                   double* dxHI, oracle_diag* diag);

/* Pieces exposed for the oracle's own pins. */
int oracle_gradients(const oracle_mesh* m, const double* phi, int use_limiter, double* grad /*[3][nc]*/);
int oracle_geometry(const oracle_mesh* m, double* Minv /*[6][nc] xx,yy,zz,xy,xz,yz*/);
double oracle_chi(double f);
void oracle_hll_flux(const double* UL, const double* UR, const double* n, double c, double* out);
int oracle_chem_cell(const oracle_params* p, double dt, double n_H, double* N /*[nb]*/,
                     double* Fh /*[nb][3]*/, double* x /*[5]*/, double* T, int64_t* n_attempts);
/* Rate coefficients and cooling of rate set 1 (Hui & Gnedin 1997, Cen 1992).
 * Pinned against published atomic data: case-B recombination of H, the
 * hydrogenic He III recombination, collisional ionisation of H I, He I and
 * He II, free-free and H I collisional-excitation cooling.  Parity unpinned
 * (checked only against the 8-cell calculator, which restates the same
 * fits): He I recombination, dielectronic recombination, and the
 * recombination, collisional-ionisation and He II excitation cooling terms. */
void oracle_rates(const oracle_params* p, double T, double* out /*[7]: aHII aHeII aHeIII bHI bHeI bHeII ad*/);
double oracle_cooling(const oracle_params* p, double T, double n_H, const double* x /*[5]*/);

#ifdef __cplusplus
}
#endif
#endif
