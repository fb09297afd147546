// Plain FP64 CPU oracle of the M1 radiative-transfer subcycle.
//
// TEST INFRASTRUCTURE ONLY (see m1rt_oracle.h).  Written for a reader who
// checks it against the paper by eye: one loop per step of the method, in the
// order of the paper's Fig. 1, no blocking, fusion or reordering.  Every
// function is templated on the scalar type R so that the same code runs in
// plain double and in forward-mode dual numbers (the reference derivative of
// the adjoint).  Branches take the decision on the value part only, so the
// dual run differentiates exactly the branch path that the double run takes.
//
// Readings of the places where the paper is silent are stated where they are
// used; the paper cites Kannan et al. (2019) for the RT solver, M1 closure and
// chemistry without restating them.

#include "m1rt_oracle.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Scalar types
// ---------------------------------------------------------------------------

template <int K>
struct Dual {
    double v;
    double d[K];
    Dual() : v(0) { for (int k = 0; k < K; ++k) d[k] = 0; }
    Dual(double x) : v(x) { for (int k = 0; k < K; ++k) d[k] = 0; }  // NOLINT
};

template <int K> Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r; r.v = a.v + b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k]; return r;
}
template <int K> Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r; r.v = a.v - b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k]; return r;
}
template <int K> Dual<K> operator-(const Dual<K>& a) {
    Dual<K> r; r.v = -a.v; for (int k = 0; k < K; ++k) r.d[k] = -a.d[k]; return r;
}
template <int K> Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r; r.v = a.v * b.v; for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r;
}
// (a/b)' = (a' - (a/b) b') / b, which stays finite where b^2 would underflow
// (states of 1e-160 and below occur at the leading edge of a front).
template <int K> Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r; r.v = a.v / b.v;
    for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
}
template <int K> Dual<K> operator+(const Dual<K>& a, double b) { return a + Dual<K>(b); }
template <int K> Dual<K> operator+(double a, const Dual<K>& b) { return Dual<K>(a) + b; }
template <int K> Dual<K> operator-(const Dual<K>& a, double b) { return a - Dual<K>(b); }
template <int K> Dual<K> operator-(double a, const Dual<K>& b) { return Dual<K>(a) - b; }
template <int K> Dual<K> operator*(const Dual<K>& a, double b) { return a * Dual<K>(b); }
template <int K> Dual<K> operator*(double a, const Dual<K>& b) { return Dual<K>(a) * b; }
template <int K> Dual<K> operator/(const Dual<K>& a, double b) { return a / Dual<K>(b); }
template <int K> Dual<K> operator/(double a, const Dual<K>& b) { return Dual<K>(a) / b; }
template <int K> Dual<K>& operator+=(Dual<K>& a, const Dual<K>& b) { a = a + b; return a; }
template <int K> Dual<K>& operator-=(Dual<K>& a, const Dual<K>& b) { a = a - b; return a; }
template <int K> Dual<K>& operator*=(Dual<K>& a, const Dual<K>& b) { a = a * b; return a; }
template <int K> Dual<K>& operator/=(Dual<K>& a, const Dual<K>& b) { a = a / b; return a; }

inline double val(double x) { return x; }
template <int K> double val(const Dual<K>& x) { return x.v; }

template <int K> Dual<K> chain(const Dual<K>& a, double f, double df) {
    Dual<K> r; r.v = f; for (int k = 0; k < K; ++k) r.d[k] = df * a.d[k]; return r;
}
template <int K> Dual<K> sqrt(const Dual<K>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int K> Dual<K> exp(const Dual<K>& a) { double e = std::exp(a.v); return chain(a, e, e); }
template <int K> Dual<K> log(const Dual<K>& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
template <int K> Dual<K> log10(const Dual<K>& a) { return chain(a, std::log10(a.v), 1.0 / (a.v * std::log(10.0))); }
template <int K> Dual<K> pow(const Dual<K>& a, double p) {
    double r = std::pow(a.v, p); return chain(a, r, p * std::pow(a.v, p - 1.0));
}
using std::sqrt; using std::exp; using std::log; using std::log10; using std::pow;

// min / max / abs decide on the value part.
template <class R> R rmax(const R& a, const R& b) { return val(a) >= val(b) ? a : b; }
template <class R> R rmin(const R& a, const R& b) { return val(a) <= val(b) ? a : b; }
template <class R> R rabs(const R& a) { return val(a) < 0 ? -a : a; }

// ---------------------------------------------------------------------------
// How the forward derivative (dual numbers) treats values that are rounding
// noise or negligible.  These hold only in the dual-number instantiation:
// the values of the plain FP64 run are untouched.  They define the
// derivative that the reverse-mode adjoint computes (the paper has no
// adjoint; these are this build's readings), so that the two can be
// compared on workloads where the exact branch-path derivative overflows:
//  * a nearly isotropic state, |Fh|^2 <= 1e-16 N^2, takes the Eddington
//    tensor I/3 (its anisotropic part is O(f^2), below one rounding; the
//    direction of a vanishing Fh has derivative 1/|Fh|);
//  * the outflow cap's factor is held constant where the flux of N through
//    the face is at the rounding level of its terms and of the two cells'
//    contents, |Phi_N| <= 1e-12 (N_L* + N_R* + N_L + N_R);
//  * at the start of a transport step, the state of a cell whose N is not
//    above 1e-20 of the bin's largest N (or is zero), and its limited
//    gradient, are held constant; what its neighbours' fluxes bring into it
//    is kept.
// ---------------------------------------------------------------------------
template <class R> struct IsDual : std::false_type {};
template <int K> struct IsDual<Dual<K>> : std::true_type {};
constexpr double kIsotropicF2 = 1e-16;
constexpr double kCapNoiseRel = 1e-12;
constexpr double kNegligibleN = 1e-20;
template <class R> R held(const R& x) { return R(val(x)); }   // the value, derivative zero

// Physical constants (CODATA 2018), cgs.
constexpr double K_BOLTZ = 1.380649e-16;
constexpr double M_PROTON = 1.67262192369e-24;
constexpr double PI = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// O0  Mesh preparation (static between subcycles: Sec. 2.3.2 reuses the
//     geometry matrix; Sec. 4.1.4 keeps per-cell face lists).
// ---------------------------------------------------------------------------

struct FaceSide {
    int64_t face;   // face index
    int64_t nbr;    // the cell on the other side
    int sign;       // +1 if this cell is the face's L cell, -1 if R
    double r[3];    // r_if = x_f - s_i (minimum image)
    double w[3];    // least-squares weight A u / |d|, d = s_j - s_i via the face
};

struct Geometry {
    int64_t nc = 0, nf = 0;
    std::vector<std::vector<FaceSide>> sides;   // per cell, in face-index order
    std::vector<double> Minv;                   // [nc][6] xx yy zz xy xz yz
    std::vector<double> V;
    std::vector<double> A, n;                   // [nf], [nf][3]
    std::vector<double> rL, rR;                 // [nf][3]: r_Lf, r_Rf
    std::vector<int64_t> L, R;
};

double min_image(double x, double box) {
    if (box > 0) x -= box * std::floor(x / box + 0.5);
    return x;
}

bool build_geometry(const oracle_mesh* m, Geometry& g) {
    g.nc = m->nc; g.nf = m->nf;
    g.sides.assign(g.nc, {});
    g.V.assign(m->volume, m->volume + g.nc);
    g.A.assign(m->area, m->area + g.nf);
    g.n.resize(3 * g.nf); g.rL.resize(3 * g.nf); g.rR.resize(3 * g.nf);
    g.L.resize(g.nf); g.R.resize(g.nf);
    for (int64_t f = 0; f < g.nf; ++f) {
        int64_t L = m->face_cells[f], R = m->face_cells[g.nf + f];
        if (L < 0 || R < 0 || L >= g.nc || R >= g.nc || L == R) return false;
        g.L[f] = L; g.R[f] = R;
        double rL[3], rR[3];
        for (int k = 0; k < 3; ++k) {
            g.n[3 * f + k] = m->normal[k * g.nf + f];
            double xf = m->face_centre[k * g.nf + f];
            rL[k] = min_image(xf - m->centre[k * g.nc + L], m->box[k]);
            rR[k] = min_image(xf - m->centre[k * g.nc + R], m->box[k]);
            g.rL[3 * f + k] = rL[k];
            g.rR[3 * f + k] = rR[k];
        }
        // Face-side of L (neighbour R) and of R (neighbour L).  The separation
        // s_j - s_i is taken through the face centre, r_if - r_jf, which is
        // unambiguous on periodic meshes where two faces join the same pair.
        for (int side = 0; side < 2; ++side) {
            FaceSide fs;
            fs.face = f;
            const double* ri = side == 0 ? rL : rR;
            const double* rj = side == 0 ? rR : rL;
            fs.nbr = side == 0 ? R : L;
            fs.sign = side == 0 ? +1 : -1;
            double d[3], dd = 0;
            for (int k = 0; k < 3; ++k) { fs.r[k] = ri[k]; d[k] = ri[k] - rj[k]; dd += d[k] * d[k]; }
            double dl = std::sqrt(dd);
            for (int k = 0; k < 3; ++k) fs.w[k] = g.A[f] * (d[k] / dl) / dl;
            g.sides[side == 0 ? L : R].push_back(fs);
        }
    }
    // Geometry matrix of the normal equation, sum_j A_ij n_ji n_ji^T, and its
    // inverse by the adjugate.
    g.Minv.assign(6 * g.nc, 0.0);
    for (int64_t i = 0; i < g.nc; ++i) {
        double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (const FaceSide& fs : g.sides[i]) {
            int64_t f = fs.face;
            double d[3], dd = 0;
            const double* rj = fs.sign > 0 ? &g.rR[3 * f] : &g.rL[3 * f];
            for (int k = 0; k < 3; ++k) { d[k] = fs.r[k] - rj[k]; dd += d[k] * d[k]; }
            double dl = std::sqrt(dd);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) M[a][b] += g.A[f] * (d[a] / dl) * (d[b] / dl);
        }
        double a = M[0][0], b = M[1][1], c = M[2][2], d = M[0][1], e = M[0][2], f = M[1][2];
        double det = a * (b * c - f * f) - d * (d * c - f * e) + e * (d * f - b * e);
        if (!(std::fabs(det) > 0)) return false;
        double* o = &g.Minv[6 * i];
        o[0] = (b * c - f * f) / det;
        o[1] = (a * c - e * e) / det;
        o[2] = (a * b - d * d) / det;
        o[3] = (e * f - d * c) / det;
        o[4] = (d * f - b * e) / det;
        o[5] = (d * e - a * f) / det;
    }
    return true;
}

double cfl_dt(const Geometry& g, const oracle_params* p) {
    // Effective cell width: radius of the sphere of equal volume.
    double dxmin = INFINITY;
    for (int64_t i = 0; i < g.nc; ++i) dxmin = std::min(dxmin, std::cbrt(3.0 * g.V[i] / (4.0 * PI)));
    return p->cfl_eta * dxmin / p->c_reduced;
}

// ---------------------------------------------------------------------------
// State
// ---------------------------------------------------------------------------

template <class R>
struct State {
    int nb = 0;
    int64_t nc = 0;
    std::vector<R> N;     // [nb][nc]
    std::vector<R> Fh;    // [nb][3][nc], F / c~
    std::vector<R> nH;    // [nc]
    std::vector<R> x;     // [5][nc] x_HI, x_HII, y_HeI, y_HeII, y_HeIII
    std::vector<R> u;     // [nc] specific thermal energy, erg/g
    R& Nb(int b, int64_t i) { return N[b * nc + i]; }
    R& Fb(int b, int k, int64_t i) { return Fh[(b * 3 + k) * nc + i]; }
};

double helium_ratio(const oracle_params* p) {
    // y_He = n_He / n_H for helium mass fraction Y.
    return p->chem_mode == OR_CHEM_HHE ? p->Y_He / (4.0 * (1.0 - p->Y_He)) : 0.0;
}

template <class R>
R electron_fraction(const R* x, double yhe) { return x[1] + yhe * (x[3] + 2.0 * x[4]); }

// T = (gamma - 1) mu m_p u / k_B, mu = (1 + 4 y_He) / (1 + y_He + x_e).
template <class R>
R temperature_of(const oracle_params* p, const R& u, const R* x) {
    double yhe = helium_ratio(p);
    R mu = (1.0 + 4.0 * yhe) / (1.0 + yhe + electron_fraction(x, yhe));
    return (p->gamma - 1.0) * mu * M_PROTON * u / K_BOLTZ;
}

template <class R>
R energy_of(const oracle_params* p, const R& T, const R* x) {
    double yhe = helium_ratio(p);
    R mu = (1.0 + 4.0 * yhe) / (1.0 + yhe + electron_fraction(x, yhe));
    return K_BOLTZ * T / ((p->gamma - 1.0) * mu * M_PROTON);
}

// ---------------------------------------------------------------------------
// Rate coefficients and cooling (the paper defers the network to Kannan et
// al. 2019).  Reading: rate set 0 = constant case-B recombination, no
// collisional ionisation, no cooling (the Stromgren test); rate set 1 =
// Hui & Gnedin (1997) case-B recombination, collisional ionisation and their
// cooling, plus Cen (1992) dielectronic recombination, collisional excitation
// cooling and free-free emission.  Temperatures are floored at 1 K for the
// fits.
// ---------------------------------------------------------------------------

constexpr double T_HI = 157807.0, T_HEI = 285335.0, T_HEII = 631515.0;

template <class R>
struct Rates {
    R aHII, aHeII, aHeIII;      // recombination (He II includes dielectronic)
    R bHI, bHeI, bHeII;         // collisional ionisation
    R ad;                       // dielectronic part of aHeII (reported)
};

template <class R> R hg97_caseB_H(const R& lam) {
    return 2.753e-14 * pow(lam, 1.5) / pow(1.0 + pow(lam / 2.740, 0.407), 2.242);
}
template <class R> R hg97_caseB_H_cool(const R& T, const R& lam) {
    return 3.435e-30 * T * pow(lam, 1.970) / pow(1.0 + pow(lam / 2.250, 0.376), 3.720);
}
template <class R> R cen92_dielectronic_shape(const R& T) {
    return pow(T, -1.5) * exp(-470000.0 / T) * (1.0 + 0.3 * exp(-94000.0 / T));
}

template <class R>
Rates<R> rates_of(const oracle_params* p, R T) {
    Rates<R> r;
    if (p->rate_set == OR_RATES_CASEB_CONST) {
        r.aHII = p->alpha_B_const;
        r.aHeII = 0.0; r.aHeIII = 0.0; r.bHI = 0.0; r.bHeI = 0.0; r.bHeII = 0.0; r.ad = 0.0;
        return r;
    }
    T = rmax(T, R(1.0));
    R lHI = 2.0 * T_HI / T, lHeI = 2.0 * T_HEI / T, lHeII = 2.0 * T_HEII / T;
    r.aHII = hg97_caseB_H(lHI);
    r.ad = 1.9e-3 * cen92_dielectronic_shape(T);
    r.aHeII = 1.26e-14 * pow(lHeI, 0.75) + r.ad;
    r.aHeIII = 2.0 * hg97_caseB_H(lHeII);
    r.bHI = 21.11 * pow(T, -1.5) * exp(-lHI / 2.0) * pow(lHI, -1.089) / pow(1.0 + pow(lHI / 0.354, 0.874), 1.101);
    r.bHeI = 32.38 * pow(T, -1.5) * exp(-lHeI / 2.0) * pow(lHeI, -1.146) / pow(1.0 + pow(lHeI / 0.416, 0.987), 1.056);
    r.bHeII = 19.95 * pow(T, -1.5) * exp(-lHeII / 2.0) * pow(lHeII, -1.089) / pow(1.0 + pow(lHeII / 0.553, 0.735), 1.275);
    return r;
}

// Net cooling rate per volume (erg cm^-3 s^-1) of gas with n_H and fractions x.
template <class R>
R cooling_of(const oracle_params* p, R T, const R& nH, const R* x) {
    if (p->rate_set == OR_RATES_CASEB_CONST) return R(0.0);
    T = rmax(T, R(1.0));
    double yhe = helium_ratio(p);
    R ne = nH * electron_fraction(x, yhe);
    R nHI = nH * x[0], nHII = nH * x[1];
    R nHeI = yhe * nH * x[2], nHeII = yhe * nH * x[3], nHeIII = yhe * nH * x[4];
    R lHI = 2.0 * T_HI / T, lHeI = 2.0 * T_HEI / T, lHeII = 2.0 * T_HEII / T;
    Rates<R> r = rates_of(p, T);
    R sq5 = 1.0 + sqrt(T / 1.0e5);
    // recombination (case B), Hui & Gnedin 1997
    R rec = hg97_caseB_H_cool(T, lHI) * nHII
          + K_BOLTZ * T * (1.26e-14 * pow(lHeI, 0.75)) * nHeII
          + 8.0 * hg97_caseB_H_cool(T, lHeII) * nHeIII;
    // dielectronic recombination, Cen 1992
    R die = 1.24e-13 * cen92_dielectronic_shape(T) * nHeII;
    // collisional ionisation: one ionisation potential per event
    R cion = K_BOLTZ * T_HI * r.bHI * nHI + K_BOLTZ * T_HEI * r.bHeI * nHeI + K_BOLTZ * T_HEII * r.bHeII * nHeII;
    // collisional excitation, Cen 1992
    R cex = 7.5e-19 * exp(-118348.0 / T) / sq5 * nHI
          + 5.54e-17 * pow(T, -0.397) * exp(-473638.0 / T) / sq5 * nHeII;
    // free-free, Cen 1992 Gaunt factor
    R lt = log10(T);
    R gff = 1.1 + 0.34 * exp(-(5.5 - lt) * (5.5 - lt) / 3.0);
    R ff = 1.42e-27 * gff * sqrt(T) * (nHII + nHeII + 4.0 * nHeIII);
    return ne * (rec + die + cion + cex + ff);
}

// ---------------------------------------------------------------------------
// O2  Thermochemistry of one cell over one subcycle (Sec. 2.3.1, 4.1.1).
//
// Semi-implicit step of length d from the substep-start state: abundances
// implicit with frozen rates, n_e and photoionisation rates; thermal energy
// explicit.  Adaptive control: f is the largest relative change of u and of
// the tracked fractions; f > f_max rejects and retries with d f_s / f; an
// accepted step proposes d min(f_s / f, growth) for the next one.  Readings:
// d restarts at the subcycle length every subcycle, the relative change of a
// fraction is measured against max(x, x_floor), the last step is clipped to
// end exactly on the subcycle, f = 0 proposes growth * d.
// ---------------------------------------------------------------------------

template <class R>
struct CellChem {
    R N[ORACLE_MAX_BINS];
    R Fh[ORACLE_MAX_BINS][3];
    R x[5];
    R u;
    R nH;
};

template <class R>
int chem_cell(const oracle_params* p, double Dt, CellChem<R>& c, int64_t* attempts) {
    const int nb = p->nb;
    const double ct = p->c_reduced;
    const double yhe = helium_ratio(p);
    const bool hhe = p->chem_mode == OR_CHEM_HHE;
    const int nspec = hhe ? 5 : 2;
    R tau = 0.0;
    R d = Dt;
    int64_t n = 0;
    for (;;) {
        bool last = false;
        if (val(d) >= val(Dt - tau)) { d = Dt - tau; last = true; }
        if (++n > p->chem_max_substeps) { *attempts = n; return -6; }

        // Frozen quantities at the substep start.
        R T = p->isothermal ? R(p->T_iso) : temperature_of(p, c.u, c.x);
        Rates<R> r = rates_of(p, T);
        R ne = c.nH * electron_fraction(c.x, yhe);
        R nHI = c.nH * c.x[0];
        R nHeI = yhe * c.nH * c.x[2];
        R nHeII = yhe * c.nH * c.x[3];
        // Photons first: implicit absorption by the substep-start absorbers,
        // N' = N / (1 + c~ d kappa); photoionisation and photoheating then use
        // the absorbed-to density N', so that an optically thick substep
        // cannot ionise more atoms than it removes photons.
        R fac[ORACLE_MAX_BINS];
        R Nn[ORACLE_MAX_BINS];
        R Gam[3] = {0.0, 0.0, 0.0};            // photoionisation rate per atom
        R heat = 0.0;                           // photoheating per volume
        for (int b = 0; b < nb; ++b) {
            R kap = p->sigma[b][0] * nHI + p->sigma[b][1] * nHeI + p->sigma[b][2] * nHeII;
            fac[b] = 1.0 + ct * d * kap;
            Nn[b] = c.N[b] / fac[b];
            for (int s = 0; s < 3; ++s) Gam[s] += ct * p->sigma[b][s] * Nn[b];
            heat += ct * Nn[b] * (p->sigma[b][0] * nHI * p->e_heat[b][0]
                                  + p->sigma[b][1] * nHeI * p->e_heat[b][1]
                                  + p->sigma[b][2] * nHeII * p->e_heat[b][2]);
        }

        // Trial abundances.
        R xn[5];
        R den = 1.0 + (Gam[0] + r.bHI * ne + r.aHII * ne) * d;
        xn[0] = (c.x[0] + r.aHII * ne * d) / den;
        xn[1] = (c.x[1] + (Gam[0] + r.bHI * ne) * d) / den;
        if (hhe) {
            xn[2] = (c.x[2] + r.aHeII * ne * c.x[3] * d) / (1.0 + (Gam[1] + r.bHeI * ne) * d);
            xn[4] = (c.x[4] + (Gam[2] + r.bHeII * ne) * c.x[3] * d) / (1.0 + r.aHeIII * ne * d);
            xn[3] = 1.0 - xn[2] - xn[4];
            if (val(xn[3]) < 0.0) {
                xn[3] = 0.0;
                R s = xn[2] + xn[4];
                xn[2] = xn[2] / s;
                xn[4] = xn[4] / s;
            }
        } else {
            xn[2] = c.x[2]; xn[3] = c.x[3]; xn[4] = c.x[4];
        }

        // Trial thermal energy (explicit).
        R un = c.u;
        if (!p->isothermal) {
            R rho = M_PROTON * c.nH * (1.0 + 4.0 * yhe);
            un = c.u + d * (heat - cooling_of(p, T, c.nH, c.x)) / rho;
        }

        // Largest relative change.
        R f = 0.0;
        if (!p->isothermal) f = rabs(un - c.u) / c.u;
        for (int s = 0; s < nspec; ++s)
            f = rmax(f, rabs(xn[s] - c.x[s]) / rmax(c.x[s], R(p->chem_xfloor)));

        if (val(f) > p->chem_fmax) {          // reject
            d = d * (p->chem_fs / f);
            continue;
        }

        // Accept.
        for (int b = 0; b < nb; ++b) {
            c.N[b] = Nn[b];
            for (int k = 0; k < 3; ++k) c.Fh[b][k] = c.Fh[b][k] / fac[b];
        }
        for (int s = 0; s < 5; ++s) c.x[s] = xn[s];
        c.u = un;
        if (last) break;
        tau = tau + d;
        if (val(f) > 0.0) d = d * rmin(R(p->chem_fs) / f, R(p->chem_growth));
        else d = d * p->chem_growth;
    }
    *attempts = n;
    return 0;
}

// ---------------------------------------------------------------------------
// O3  Least-squares gradients with the slope limiter (Sec. 2.3.2).
// For each scalar phi: g = M^-1 sum_j w_ij (phi_j - phi_i); then a
// Barth-Jespersen factor keeps the extrapolation to every face centre inside
// [min, max] of the cell and its neighbours (reading of the "constant
// factor" of the paper).
// ---------------------------------------------------------------------------

template <class R>
void gradient_of(const Geometry& g, int64_t i, const R* phi, bool limit, R out[3]) {
    R b[3] = {0.0, 0.0, 0.0};
    R pmax = phi[i], pmin = phi[i];
    for (const FaceSide& fs : g.sides[i]) {
        R dphi = phi[fs.nbr] - phi[i];
        for (int k = 0; k < 3; ++k) b[k] += fs.w[k] * dphi;
        pmax = rmax(pmax, phi[fs.nbr]);
        pmin = rmin(pmin, phi[fs.nbr]);
    }
    const double* mi = &g.Minv[6 * i];
    const double Mi[3][3] = {{mi[0], mi[3], mi[4]}, {mi[3], mi[1], mi[5]}, {mi[4], mi[5], mi[2]}};
    for (int a = 0; a < 3; ++a) out[a] = Mi[a][0] * b[0] + Mi[a][1] * b[1] + Mi[a][2] * b[2];
    if (!limit) return;
    R alpha = 1.0;
    for (const FaceSide& fs : g.sides[i]) {
        R delta = out[0] * fs.r[0] + out[1] * fs.r[1] + out[2] * fs.r[2];
        R psi = 1.0;
        if (val(delta) > 0.0) psi = (pmax - phi[i]) / delta;
        else if (val(delta) < 0.0) psi = (pmin - phi[i]) / delta;
        alpha = rmin(alpha, psi);
    }
    for (int a = 0; a < 3; ++a) out[a] = alpha * out[a];
}

// ---------------------------------------------------------------------------
// O4  Face flux (Sec. 2.3.3): extrapolate both cells to the face centre,
// enforce N >= 0 and |Fh| <= N on each face state, M1 closure (eq. edd) with
// the Levermore Eddington factor, HLL flux with the wave-speed bounds -c~ and
// +c~ (every M1 eigenvalue lies in [-c~, c~], so HLL with these bounds is the
// Rusanov flux and the rotation to the face frame and back is the identity).
// State U = (N, Fh); flux of N is c~ Fh.n, flux of Fh is c~ N D n.
// ---------------------------------------------------------------------------

template <class R>
R chi_of(const R& f) {
    // Levermore (1984) M1 Eddington factor.
    return (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f));
}

template <class R>
void eddington_tensor(const R& N, const R* Fh, R D[3][3]) {
    R F2 = Fh[0] * Fh[0] + Fh[1] * Fh[1] + Fh[2] * Fh[2];
    if (val(N) <= 0.0 || val(F2) <= 0.0 ||
        (IsDual<R>::value && val(F2) <= kIsotropicF2 * val(N) * val(N))) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) D[a][b] = a == b ? R(1.0 / 3.0) : R(0.0);
        return;
    }
    R Fm = sqrt(F2);
    // The Levermore factor is defined for f in [0, 1]; near the underflow
    // threshold the rounded |Fh| can exceed N slightly, so f is clamped.
    R f = rmin(Fm / N, R(1.0));
    R chi = chi_of(f);
    R uhat[3] = {Fh[0] / Fm, Fh[1] / Fm, Fh[2] / Fm};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            D[a][b] = 0.5 * (3.0 * chi - 1.0) * uhat[a] * uhat[b] + (a == b ? 0.5 * (1.0 - chi) : R(0.0));
}

template <class R>
void hll_flux(const R UL[4], const R UR[4], const double n[3], double ct, R out[4]) {
    R DL[3][3], DR[3][3];
    eddington_tensor(UL[0], &UL[1], DL);
    eddington_tensor(UR[0], &UR[1], DR);
    R FLn = UL[1] * n[0] + UL[2] * n[1] + UL[3] * n[2];
    R FRn = UR[1] * n[0] + UR[2] * n[1] + UR[3] * n[2];
    out[0] = ct * (0.5 * (FLn + FRn) - 0.5 * (UR[0] - UL[0]));
    for (int a = 0; a < 3; ++a) {
        R PLn = UL[0] * (DL[a][0] * n[0] + DL[a][1] * n[1] + DL[a][2] * n[2]);
        R PRn = UR[0] * (DR[a][0] * n[0] + DR[a][1] * n[1] + DR[a][2] * n[2]);
        out[1 + a] = ct * (0.5 * (PLn + PRn) - 0.5 * (UR[1 + a] - UL[1 + a]));
    }
}

// Face-state admissibility: N >= 0, |Fh| <= N.
template <class R>
void make_admissible(R U[4], int64_t* cntN, int64_t* cntF) {
    if (val(U[0]) < 0.0) { U[0] = 0.0; ++*cntN; }
    R F2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
    if (val(F2) > val(U[0] * U[0])) {
        ++*cntF;
        if (val(U[0]) <= 0.0) { U[1] = 0.0; U[2] = 0.0; U[3] = 0.0; }
        else { R s = U[0] / sqrt(F2); for (int k = 1; k < 4; ++k) U[k] = U[k] * s; }
    }
}

// ---------------------------------------------------------------------------
// One subcycle.
// ---------------------------------------------------------------------------

// Host threads of a subcycle (oracle_set_threads).  With one thread the
// subcycle runs as the plain loops below; with more, the per-cell loops are
// shared out and the face loop becomes two passes (every face's flux, then
// each cell's sum over its faces in face-index order), which adds the same
// terms in the same order, so the results are the same bit for bit.
int g_threads = 1;

template <class R>
struct Sources {
    int64_t n = 0;
    const int64_t* cell = nullptr;
    std::vector<R> rate;    // [nb][n]
};

// The negligible states of a transport step (dual numbers only, see
// kNegligibleN): neg[b][i] set, and the cell's N and Fh of bin b held.
template <class R>
void hold_negligible(State<R>& s, int nb, int64_t nc, std::vector<char>& neg) {
    neg.assign((size_t)nb * nc, 0);
    for (int b = 0; b < nb; ++b) {
        double mx = 0.0;
        for (int64_t i = 0; i < nc; ++i) mx = std::max(mx, val(s.Nb(b, i)));
        for (int64_t i = 0; i < nc; ++i) {
            const double n = val(s.Nb(b, i));
            if (n > 0.0 && n >= kNegligibleN * mx) continue;
            neg[(size_t)b * nc + i] = 1;
            s.Nb(b, i) = held(s.Nb(b, i));
            for (int k = 0; k < 3; ++k) s.Fb(b, k, i) = held(s.Fb(b, k, i));
        }
    }
}

template <class R>
int subcycle_threads(const Geometry& g, const oracle_params* p, double Dt, State<R>& s, const Sources<R>& src,
                     oracle_diag* dg);

template <class R>
int subcycle(const Geometry& g, const oracle_params* p, double Dt, State<R>& s, const Sources<R>& src,
             oracle_diag* dg) {
    if (g_threads > 1) return subcycle_threads(g, p, Dt, s, src, dg);
    const int nb = p->nb;
    const int64_t nc = g.nc;
    const double ct = p->c_reduced;

    // O1  point sources, in source-list order.
    for (int64_t k = 0; k < src.n; ++k) {
        int64_t i = src.cell[k];
        for (int b = 0; b < nb; ++b) s.Nb(b, i) += src.rate[b * src.n + k] * Dt / g.V[i];
    }

    // O2  thermochemistry, independently per cell.
    if (p->chem_mode != OR_CHEM_NONE) {
        for (int64_t i = 0; i < nc; ++i) {
            CellChem<R> c;
            for (int b = 0; b < nb; ++b) {
                c.N[b] = s.Nb(b, i);
                for (int k = 0; k < 3; ++k) c.Fh[b][k] = s.Fb(b, k, i);
            }
            for (int q = 0; q < 5; ++q) c.x[q] = s.x[q * nc + i];
            c.u = s.u[i];
            c.nH = s.nH[i];
            int64_t att = 0;
            int rc = chem_cell(p, Dt, c, &att);
            dg->substeps += att;
            dg->max_substeps = std::max<int64_t>(dg->max_substeps, att);
            if (rc) { dg->status = rc; return rc; }
            for (int b = 0; b < nb; ++b) {
                s.Nb(b, i) = c.N[b];
                for (int k = 0; k < 3; ++k) s.Fb(b, k, i) = c.Fh[b][k];
            }
            for (int q = 0; q < 5; ++q) s.x[q * nc + i] = c.x[q];
            s.u[i] = c.u;
        }
    }

    // O3  gradients of N and of the three components of Fh, per bin.
    std::vector<char> neg;
    if (IsDual<R>::value) hold_negligible(s, nb, nc, neg);
    std::vector<R> grad((size_t)nb * 4 * 3 * nc);   // [nb][4][3][nc]
    for (int b = 0; b < nb; ++b)
        for (int v = 0; v < 4; ++v) {
            const R* phi = v == 0 ? &s.N[(size_t)b * nc] : &s.Fh[((size_t)b * 3 + (v - 1)) * nc];
            for (int64_t i = 0; i < nc; ++i) {
                R gi[3];
                gradient_of(g, i, phi, p->use_limiter != 0, gi);
                for (int k = 0; k < 3; ++k)
                    grad[(((size_t)b * 4 + v) * 3 + k) * nc + i] = neg.empty() || !neg[(size_t)b * nc + i] ? gi[k] : held(gi[k]);
            }
        }

    // O4  face fluxes from the start-of-transport states, one face at a time;
    // O5  accumulation into both cells in face-index order.
    std::vector<R> acc((size_t)nb * 4 * nc, R(0.0));   // [nb][4][nc]
    for (int64_t f = 0; f < g.nf; ++f) {
        const int64_t L = g.L[f], Rr = g.R[f];
        const double* n = &g.n[3 * f];
        for (int b = 0; b < nb; ++b) {
            R UL[4], UR[4];
            for (int v = 0; v < 4; ++v) {
                const R* phi = v == 0 ? &s.N[(size_t)b * nc] : &s.Fh[((size_t)b * 3 + (v - 1)) * nc];
                const R* gv = &grad[(((size_t)b * 4 + v) * 3) * nc];
                UL[v] = phi[L] + gv[L] * g.rL[3 * f] + gv[nc + L] * g.rL[3 * f + 1] + gv[2 * nc + L] * g.rL[3 * f + 2];
                UR[v] = phi[Rr] + gv[Rr] * g.rR[3 * f] + gv[nc + Rr] * g.rR[3 * f + 1] + gv[2 * nc + Rr] * g.rR[3 * f + 2];
            }
            make_admissible(UL, &dg->adm_N, &dg->adm_F);
            make_admissible(UR, &dg->adm_N, &dg->adm_F);
            R Phi[4];
            hll_flux(UL, UR, n, ct, Phi);
            // Positivity limiter: the upwind cell may lose through this face at
            // most its 1/n_faces share of the photons it holds (reading of the
            // "further limiter" of Sec. 2.3.3); symmetric, so conservative.
            if (val(Phi[0]) != 0.0) {
                int64_t up = val(Phi[0]) > 0.0 ? L : Rr;
                double nfs = (double)g.sides[up].size();
                R cap = s.Nb(b, up) * g.V[up] / (nfs * rabs(Phi[0]) * Dt * g.A[f]);
                if (IsDual<R>::value && val(rabs(Phi[0])) <= kCapNoiseRel * (val(UL[0]) + val(UR[0]) +
                                                                              val(s.Nb(b, L)) + val(s.Nb(b, Rr))))
                    cap = held(cap);
                if (val(cap) < 1.0) {
                    ++dg->flux_caps;
                    for (int v = 0; v < 4; ++v) Phi[v] = cap * Phi[v];
                }
            }
            for (int v = 0; v < 4; ++v) {
                acc[((size_t)b * 4 + v) * nc + L] += g.A[f] * Phi[v];
                acc[((size_t)b * 4 + v) * nc + Rr] -= g.A[f] * Phi[v];
            }
        }
    }
    for (int b = 0; b < nb; ++b)
        for (int64_t i = 0; i < nc; ++i) {
            R U[4];
            U[0] = s.Nb(b, i) - (Dt / g.V[i]) * acc[((size_t)b * 4) * nc + i];
            for (int k = 0; k < 3; ++k)
                U[1 + k] = s.Fb(b, k, i) - (Dt / g.V[i]) * acc[((size_t)b * 4 + 1 + k) * nc + i];
            // Post-update guards.
            if (val(U[0]) < 0.0) { U[0] = 0.0; ++dg->guard_N; }
            R F2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
            if (val(F2) > val(U[0] * U[0])) {
                ++dg->guard_F;
                if (val(U[0]) <= 0.0) { U[1] = 0.0; U[2] = 0.0; U[3] = 0.0; }
                else { R sc = U[0] / sqrt(F2); for (int k = 1; k < 4; ++k) U[k] = U[k] * sc; }
            }
            s.Nb(b, i) = U[0];
            for (int k = 0; k < 3; ++k) s.Fb(b, k, i) = U[1 + k];
        }
    return 0;
}

// The same subcycle on g_threads host threads (see g_threads).
template <class R>
int subcycle_threads(const Geometry& g, const oracle_params* p, double Dt, State<R>& s, const Sources<R>& src,
                     oracle_diag* dg) {
    const int nb = p->nb;
    const int64_t nc = g.nc, nf = g.nf;
    const double ct = p->c_reduced;
    const int nt = g_threads;

    for (int64_t k = 0; k < src.n; ++k) {
        int64_t i = src.cell[k];
        for (int b = 0; b < nb; ++b) s.Nb(b, i) += src.rate[b * src.n + k] * Dt / g.V[i];
    }

    if (p->chem_mode != OR_CHEM_NONE) {
        int64_t sum_att = 0, max_att = 0;
        int err = 0;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 256) reduction(+ : sum_att) reduction(max : max_att) \
    reduction(min : err)
        for (int64_t i = 0; i < nc; ++i) {
            CellChem<R> c;
            for (int b = 0; b < nb; ++b) {
                c.N[b] = s.Nb(b, i);
                for (int k = 0; k < 3; ++k) c.Fh[b][k] = s.Fb(b, k, i);
            }
            for (int q = 0; q < 5; ++q) c.x[q] = s.x[q * nc + i];
            c.u = s.u[i];
            c.nH = s.nH[i];
            int64_t att = 0;
            int rc = chem_cell(p, Dt, c, &att);
            sum_att += att;
            max_att = std::max<int64_t>(max_att, att);
            if (rc) { err = std::min(err, rc); continue; }
            for (int b = 0; b < nb; ++b) {
                s.Nb(b, i) = c.N[b];
                for (int k = 0; k < 3; ++k) s.Fb(b, k, i) = c.Fh[b][k];
            }
            for (int q = 0; q < 5; ++q) s.x[q * nc + i] = c.x[q];
            s.u[i] = c.u;
        }
        dg->substeps += sum_att;
        dg->max_substeps = std::max<int64_t>(dg->max_substeps, max_att);
        if (err) { dg->status = err; return err; }
    }

    std::vector<char> neg;
    if (IsDual<R>::value) hold_negligible(s, nb, nc, neg);
    std::vector<R> grad((size_t)nb * 4 * 3 * nc);
    for (int b = 0; b < nb; ++b)
        for (int v = 0; v < 4; ++v) {
            const R* phi = v == 0 ? &s.N[(size_t)b * nc] : &s.Fh[((size_t)b * 3 + (v - 1)) * nc];
#pragma omp parallel for num_threads(nt) schedule(static)
            for (int64_t i = 0; i < nc; ++i) {
                R gi[3];
                gradient_of(g, i, phi, p->use_limiter != 0, gi);
                for (int k = 0; k < 3; ++k)
                    grad[(((size_t)b * 4 + v) * 3 + k) * nc + i] = neg.empty() || !neg[(size_t)b * nc + i] ? gi[k] : held(gi[k]);
            }
        }

    // Pass 1: A_f Phi_f of every face and bin.
    std::vector<R> aphi((size_t)nf * nb * 4);
    int64_t admN = 0, admF = 0, caps = 0;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : admN, admF, caps)
    for (int64_t f = 0; f < nf; ++f) {
        const int64_t L = g.L[f], Rr = g.R[f];
        const double* n = &g.n[3 * f];
        for (int b = 0; b < nb; ++b) {
            R UL[4], UR[4];
            for (int v = 0; v < 4; ++v) {
                const R* phi = v == 0 ? &s.N[(size_t)b * nc] : &s.Fh[((size_t)b * 3 + (v - 1)) * nc];
                const R* gv = &grad[(((size_t)b * 4 + v) * 3) * nc];
                UL[v] = phi[L] + gv[L] * g.rL[3 * f] + gv[nc + L] * g.rL[3 * f + 1] + gv[2 * nc + L] * g.rL[3 * f + 2];
                UR[v] = phi[Rr] + gv[Rr] * g.rR[3 * f] + gv[nc + Rr] * g.rR[3 * f + 1] + gv[2 * nc + Rr] * g.rR[3 * f + 2];
            }
            make_admissible(UL, &admN, &admF);
            make_admissible(UR, &admN, &admF);
            R Phi[4];
            hll_flux(UL, UR, n, ct, Phi);
            if (val(Phi[0]) != 0.0) {
                int64_t up = val(Phi[0]) > 0.0 ? L : Rr;
                double nfs = (double)g.sides[up].size();
                R cap = s.Nb(b, up) * g.V[up] / (nfs * rabs(Phi[0]) * Dt * g.A[f]);
                if (IsDual<R>::value && val(rabs(Phi[0])) <= kCapNoiseRel * (val(UL[0]) + val(UR[0]) +
                                                                              val(s.Nb(b, L)) + val(s.Nb(b, Rr))))
                    cap = held(cap);
                if (val(cap) < 1.0) {
                    ++caps;
                    for (int v = 0; v < 4; ++v) Phi[v] = cap * Phi[v];
                }
            }
            for (int v = 0; v < 4; ++v) aphi[((size_t)f * nb + b) * 4 + v] = g.A[f] * Phi[v];
        }
    }
    dg->adm_N += admN; dg->adm_F += admF; dg->flux_caps += caps;
    // Pass 2: each cell's sum over its faces in face-index order, then the
    // update and the guards.
    int64_t gN = 0, gF = 0;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : gN, gF)
    for (int64_t i = 0; i < nc; ++i) {
        for (int b = 0; b < nb; ++b) {
            R a[4] = {R(0.0), R(0.0), R(0.0), R(0.0)};
            for (const FaceSide& fs : g.sides[i])
                for (int v = 0; v < 4; ++v) {
                    const R& t = aphi[((size_t)fs.face * nb + b) * 4 + v];
                    if (fs.sign > 0) a[v] += t; else a[v] -= t;
                }
            R U[4];
            U[0] = s.Nb(b, i) - (Dt / g.V[i]) * a[0];
            for (int k = 0; k < 3; ++k) U[1 + k] = s.Fb(b, k, i) - (Dt / g.V[i]) * a[1 + k];
            if (val(U[0]) < 0.0) { U[0] = 0.0; ++gN; }
            R F2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
            if (val(F2) > val(U[0] * U[0])) {
                ++gF;
                if (val(U[0]) <= 0.0) { U[1] = 0.0; U[2] = 0.0; U[3] = 0.0; }
                else { R sc = U[0] / sqrt(F2); for (int k = 1; k < 4; ++k) U[k] = U[k] * sc; }
            }
            s.Nb(b, i) = U[0];
            for (int k = 0; k < 3; ++k) s.Fb(b, k, i) = U[1 + k];
        }
    }
    dg->guard_N += gN; dg->guard_F += gF;
    return 0;
}

// Pairwise summation (O6).
double pairwise_sum(const double* a, int64_t n) {
    if (n <= 8) { double s = 0; for (int64_t i = 0; i < n; ++i) s += a[i]; return s; }
    int64_t h = n / 2;
    return pairwise_sum(a, h) + pairwise_sum(a + h, n - h);
}

bool check_params(const oracle_params* p) {
    return p && p->nb >= 1 && p->nb <= ORACLE_MAX_BINS && p->c_reduced > 0 && p->cfl_eta > 0 &&
           p->chem_mode >= 0 && p->chem_mode <= 2 && p->chem_max_substeps > 0;
}

template <class R>
void load_state(const oracle_params* p, int64_t nc, const double* N, const double* F, const double* species,
                const double* T, State<R>& s) {
    const int nb = p->nb;
    s.nb = nb; s.nc = nc;
    s.N.assign(N, N + (size_t)nb * nc);
    s.Fh.resize((size_t)nb * 3 * nc);
    for (size_t q = 0; q < s.Fh.size(); ++q) s.Fh[q] = F[q] / p->c_reduced;
    s.x.assign(species, species + 5 * nc);
    s.u.resize(nc);
    for (int64_t i = 0; i < nc; ++i) {
        R xi[5];
        for (int q = 0; q < 5; ++q) xi[q] = s.x[q * nc + i];
        s.u[i] = energy_of(p, R(T[i]), xi);
    }
}

template <class R>
void store_state(const oracle_params* p, const State<R>& s, double* N, double* F, double* species, double* T) {
    const int64_t nc = s.nc;
    for (size_t q = 0; q < s.N.size(); ++q) N[q] = val(s.N[q]);
    for (size_t q = 0; q < s.Fh.size(); ++q) F[q] = val(s.Fh[q]) * p->c_reduced;
    for (size_t q = 0; q < s.x.size(); ++q) species[q] = val(s.x[q]);
    for (int64_t i = 0; i < nc; ++i) {
        if (p->isothermal) { T[i] = p->T_iso; continue; }
        R xi[5];
        for (int q = 0; q < 5; ++q) xi[q] = s.x[q * nc + i];
        T[i] = val(temperature_of(p, s.u[i], xi));
    }
}

template <class R>
int run(const oracle_mesh* m, const oracle_params* p, State<R>& s, const Sources<R>& src, int n_sub,
        double dt, oracle_diag* diag) {
    Geometry g;
    if (!build_geometry(m, g)) return -1;
    double dtc = cfl_dt(g, p);
    double Dt = dt <= 0 ? dtc : dt;
    if (dt > dtc) return -1;
    oracle_diag local;
    std::memset(&local, 0, sizeof(local));
    local.dt = Dt;
    int rc = 0;
    auto t0 = std::chrono::steady_clock::now();
    for (int it = 0; it < n_sub && rc == 0; ++it) rc = subcycle(g, p, Dt, s, src, &local);
    local.loop_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::vector<double> nv(s.nc);
    for (int b = 0; b < p->nb; ++b) {
        for (int64_t i = 0; i < s.nc; ++i) nv[i] = val(s.N[(size_t)b * s.nc + i]) * g.V[i];
        local.photon_sum[b] = pairwise_sum(nv.data(), s.nc);
    }
    local.status = rc;
    if (diag) *diag = local;
    return rc;
}

template <int K>
int run_jvp_block(const oracle_mesh* m, const oracle_params* p, double* N, double* F, const double* n_H,
                  double* species, double* T, int64_t n_src, const int64_t* src_cell, const double* src_rate,
                  int n_sub, double dt, int ndir, const double* dlnQ, const double* dln_nH, double* dxHI,
                  oracle_diag* diag) {
    using D = Dual<K>;
    const int64_t nc = m->nc;
    State<D> s;
    load_state(p, nc, N, F, species, T, s);
    s.nH.resize(nc);
    for (int64_t i = 0; i < nc; ++i) {
        s.nH[i] = D(n_H[i]);
        for (int k = 0; k < ndir; ++k) s.nH[i].d[k] = n_H[i] * dln_nH[(size_t)k * nc + i];
    }
    Sources<D> src;
    src.n = n_src; src.cell = src_cell;
    src.rate.resize((size_t)p->nb * n_src);
    for (int b = 0; b < p->nb; ++b)
        for (int64_t q = 0; q < n_src; ++q) {
            double Q = src_rate[b * n_src + q];
            D v(Q);
            for (int k = 0; k < ndir; ++k) v.d[k] = Q * dlnQ[(size_t)k * n_src + q];
            src.rate[b * n_src + q] = v;
        }
    int rc = run(m, p, s, src, n_sub, dt, diag);
    store_state(p, s, N, F, species, T);
    for (int k = 0; k < ndir; ++k)
        for (int64_t i = 0; i < nc; ++i) dxHI[(size_t)k * nc + i] = s.x[i].d[k];
    return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// C entry points
// ---------------------------------------------------------------------------

extern "C" int oracle_set_threads(int n) {
    if (n < 1) return -1;
    g_threads = n;
    return 0;
}

extern "C" double oracle_cfl_dt(const oracle_mesh* m, const oracle_params* p) {
    Geometry g;
    if (!check_params(p) || !build_geometry(m, g)) return -1.0;
    return cfl_dt(g, p);
}

extern "C" int oracle_run(const oracle_mesh* m, const oracle_params* p, double* N, double* F, const double* n_H,
                          double* species, double* T, int64_t n_src, const int64_t* src_cell,
                          const double* src_rate, int n_sub, double dt, oracle_diag* diag) {
    if (!check_params(p) || !m || m->nc <= 0 || n_sub < 0) return -1;
    for (int64_t k = 0; k < n_src; ++k)
        if (src_cell[k] < 0 || src_cell[k] >= m->nc) return -1;
    State<double> s;
    load_state(p, m->nc, N, F, species, T, s);
    s.nH.assign(n_H, n_H + m->nc);
    Sources<double> src;
    src.n = n_src; src.cell = src_cell;
    src.rate.assign(src_rate, src_rate + (size_t)p->nb * n_src);
    int rc = run(m, p, s, src, n_sub, dt, diag);
    store_state(p, s, N, F, species, T);
    return rc;
}

extern "C" int oracle_run_jvp(const oracle_mesh* m, const oracle_params* p, double* N, double* F,
                              const double* n_H, double* species, double* T, int64_t n_src,
                              const int64_t* src_cell, const double* src_rate, int n_sub, double dt, int n_dir,
                              const double* dlnQ, const double* dln_nH, double* dxHI, oracle_diag* diag) {
    if (!check_params(p) || !m || m->nc <= 0 || n_sub < 0 || n_dir < 1 || n_dir > 8) return -1;
    for (int64_t k = 0; k < n_src; ++k)
        if (src_cell[k] < 0 || src_cell[k] >= m->nc) return -1;
    if (n_dir == 1)
        return run_jvp_block<1>(m, p, N, F, n_H, species, T, n_src, src_cell, src_rate, n_sub, dt, 1, dlnQ,
                                dln_nH, dxHI, diag);
    return run_jvp_block<8>(m, p, N, F, n_H, species, T, n_src, src_cell, src_rate, n_sub, dt, n_dir, dlnQ,
                            dln_nH, dxHI, diag);
}

extern "C" int oracle_gradients(const oracle_mesh* m, const double* phi, int use_limiter, double* grad) {
    Geometry g;
    if (!build_geometry(m, g)) return -1;
    for (int64_t i = 0; i < g.nc; ++i) {
        double gi[3];
        gradient_of(g, i, phi, use_limiter != 0, gi);
        for (int k = 0; k < 3; ++k) grad[k * g.nc + i] = gi[k];
    }
    return 0;
}

extern "C" int oracle_geometry(const oracle_mesh* m, double* Minv) {
    Geometry g;
    if (!build_geometry(m, g)) return -1;
    for (int64_t i = 0; i < g.nc; ++i)
        for (int q = 0; q < 6; ++q) Minv[q * g.nc + i] = g.Minv[6 * i + q];
    return 0;
}

extern "C" double oracle_chi(double f) { return chi_of(f); }

extern "C" void oracle_hll_flux(const double* UL, const double* UR, const double* n, double c, double* out) {
    hll_flux(UL, UR, n, c, out);
}

extern "C" int oracle_chem_cell(const oracle_params* p, double dt, double n_H, double* N, double* Fh, double* x,
                                double* T, int64_t* n_attempts) {
    if (!check_params(p)) return -1;
    CellChem<double> c;
    for (int b = 0; b < p->nb; ++b) {
        c.N[b] = N[b];
        for (int k = 0; k < 3; ++k) c.Fh[b][k] = Fh[3 * b + k];
    }
    for (int q = 0; q < 5; ++q) c.x[q] = x[q];
    c.nH = n_H;
    c.u = energy_of(p, *T, c.x);
    int rc = chem_cell(p, dt, c, n_attempts);
    for (int b = 0; b < p->nb; ++b) {
        N[b] = c.N[b];
        for (int k = 0; k < 3; ++k) Fh[3 * b + k] = c.Fh[b][k];
    }
    for (int q = 0; q < 5; ++q) x[q] = c.x[q];
    *T = p->isothermal ? p->T_iso : temperature_of(p, c.u, c.x);
    return rc;
}

extern "C" void oracle_rates(const oracle_params* p, double T, double* out) {
    Rates<double> r = rates_of(p, T);
    out[0] = r.aHII; out[1] = r.aHeII; out[2] = r.aHeIII;
    out[3] = r.bHI; out[4] = r.bHeI; out[5] = r.bHeII; out[6] = r.ad;
}

extern "C" double oracle_cooling(const oracle_params* p, double T, double n_H, const double* x) {
    return cooling_of(p, T, n_H, x);
}
