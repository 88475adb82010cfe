/*
 * pmc_oracle.c - plain double-precision CPU reference of condensed-history
 * proton transport with dose scoring (Wan Chan Tseung, Ma & Beltran,
 * arXiv:1409.8336, Sec. II.A "Simulation model" and Sec. II.B.2 "Software
 * structure").
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code,
 * header, table or constant generator with the HIP engine; both read the same
 * seeded inputs and follow the same written reading of the paper.
 *
 * The code follows the paper's step structure in its own order and notation,
 * favouring obviousness over speed: libm everywhere, no fast-math, tables on a
 * fine grid with exact derivatives, one history at a time depth-first.
 *
 * Parity status of each part (what pins it in the CPU test-suite):
 *   Philox4x32-10 ............ pinned (bit-exact against rocRAND's host engine)
 *   normal quantile .......... pinned (scipy.stats.norm.ppf)
 *   Bethe-Bloch S(E) ......... pinned (published water stopping powers)
 *   CSDA range / inverse ..... pinned (independent scipy quadrature)
 *   Eq. 1/2 scaling .......... pinned (deterministic stopping depths)
 *   radiation lengths ........ pinned (published X0 values)
 *   Highland MCS ............. pinned (hand-evaluated worked value; thin-slab
 *                              exit-angle width; Moliere core within 11%)
 *   random hinge ............. pinned (thin-slab exit displacement: the
 *                              thin-layer moments <x^2> = s^2<theta^2>/3,
 *                              <x theta> = s<theta^2>/2; face landing against
 *                              the plain hinge)
 *   source lateral profile ... pinned (per-axis SD = the spot's sigma_x,
 *                              sigma_y on an anisotropic grid; KS normality)
 *   straggling ............... pinned (Bohr variance of one step; worked value)
 *   attenuation .............. pinned (exp(-n sigma L), constant sigma)
 *   elastic (Eq. 3) .......... pinned (KS against the integrated Eq. 3, and
 *                              four-momentum conservation)
 *   target / process choice .. pinned (frequencies vs n_i sigma_i)
 *   secondary sampler ........ pinned (multiplicity / marginals vs table)
 *   energy ledger ............ pinned (conservation identity)
 *   10-group variance ........ pinned (numpy on the batch tallies; Eq. 5)
 *   composed transport ....... pinned (all physics on: a half slab of bone or
 *                              lung shifts R80 by t (rho f - 1), the water
 *                              side's R80 sits at the PSTAR CSDA range)
 *   full 3-D heterogeneous dose  parity unpinned beyond the pieces above
 */
#include "pmc_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- physical constants (CODATA 2018 / PDG) ---- */
#define M_PROTON 938.272088      /* MeV */
#define M_ELECTRON 0.51099895    /* MeV */
#define M_AMU 931.49410242       /* MeV */
#define K_BETHE 0.307075         /* 4 pi N_A r_e^2 m_e c^2, MeV cm^2 / mol */
#define N_AVOGADRO 6.02214076e23
#define ALPHA_FS (1.0 / 137.035999084)
#define X0_CONST 716.408         /* g cm^-2: A / (4 alpha r_e^2 N_A) */
#define MEV_PER_GY_FACTOR 1.602176634e-10 /* MeV/g -> Gy */
#define BARN_CM2 1.0e-24

#define E_CUT 0.1                /* termination energy, Sec. II.A.3 */
#define GRID_EMIN 0.1
#define GRID_EMAX 250.0
#define E_REF 100.0              /* energy at which f_m is evaluated */
#define WATER_I_EV 75.0

static const double EL_Z[ORA_NEL] = {1, 6, 7, 8, 15, 20, 22};
static const double EL_A[ORA_NEL] = {1.00794, 12.0107, 14.0067, 15.9994,
                                     30.973762, 40.078, 47.867};
static const int EL_MASS_NUMBER[ORA_NEL] = {1, 12, 14, 16, 31, 40, 48};

enum { LIM_NUC = 0, LIM_BND = 1 };

static double vav_quantile(const double* t, double kappa, double beta2, double z);

/* ======================================================================
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11), keyed by the run
 * seed, counter = (uid lo, uid hi, step index k, tag).  Tags: 0 birth,
 * 1 step, 3 and 4 nuclear event, 16+j secondary j, 0xC0000000|j uid of
 * secondary j.
 * ====================================================================== */
void oracle_philox4x32_10(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t k0 = key[0], k1 = key[1];
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod1;
        uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* (x >> 9 + 1/2) / 2^23: strictly inside (0,1), exact in float and double */
double oracle_u01(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

static void draw4(uint64_t seed, uint64_t uid, uint32_t k, uint32_t tag, double u[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)uid, (uint32_t)(uid >> 32), k, tag};
    uint32_t out[4];
    oracle_philox4x32_10(key, ctr, out);
    for (int i = 0; i < 4; ++i) u[i] = oracle_u01(out[i]);
}

static uint64_t child_uid(uint64_t seed, uint64_t uid, uint32_t k, uint32_t j)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)uid, (uint32_t)(uid >> 32), k, 0xC0000000u | j};
    uint32_t out[4];
    oracle_philox4x32_10(key, ctr, out);
    return (uint64_t)out[0] | ((uint64_t)out[1] << 32);
}

static double std_normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* Inverse of the standard normal CDF by bracketed Newton iteration. */
double oracle_normal_quantile(double u)
{
    if (!(u > 0.0 && u < 1.0)) return NAN;
    if (u == 0.5) return 0.0;
    if (u > 0.5) return -oracle_normal_quantile(1.0 - u);
    double lo = -40.0, hi = 0.0;
    double x = -sqrt(-2.0 * log(u));
    for (int it = 0; it < 200; ++it) {
        double f = std_normal_cdf(x) - u;
        if (f > 0.0) hi = x; else lo = x;
        double pdf = exp(-0.5 * x * x) / sqrt(2.0 * M_PI);
        double xn = (pdf > 0.0) ? x - f / pdf : 0.5 * (lo + hi);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 1e-15 * fabs(x)) { x = xn; break; }
        x = xn;
    }
    return x;
}

/* ======================================================================
 * Stopping power and CSDA range (Sec. II.A.2).  The paper's Geant4 tables are
 * replaced by the Bethe-Bloch mass stopping power without shell, density or
 * Barkas terms.  Below the energy of its maximum the formula is unphysical
 * (it falls to zero); there the value at the maximum is used.
 * ====================================================================== */
double oracle_bethe_bloch(double t, double za, double i_ev)
{
    double i_mev = i_ev * 1e-6;
    double tau = t / M_PROTON;
    double gamma = 1.0 + tau;
    double b2g2 = tau * (tau + 2.0);            /* (beta gamma)^2 */
    double beta2 = b2g2 / (gamma * gamma);
    double r = M_ELECTRON / M_PROTON;
    double wmax = 2.0 * M_ELECTRON * b2g2 / (1.0 + 2.0 * gamma * r + r * r);
    double bracket = 0.5 * log(2.0 * M_ELECTRON * b2g2 * wmax / (i_mev * i_mev)) - beta2;
    return K_BETHE * za / beta2 * bracket;      /* MeV cm^2 / g */
}

double oracle_bb_peak_energy(double za, double i_ev)
{
    /* golden-section search for the maximum over ln T in [1 keV, 10 MeV] */
    const double g = 0.5 * (sqrt(5.0) - 1.0);
    double a = log(1e-3), b = log(10.0);
    double c = b - g * (b - a), d = a + g * (b - a);
    double fc = oracle_bethe_bloch(exp(c), za, i_ev);
    double fd = oracle_bethe_bloch(exp(d), za, i_ev);
    for (int it = 0; it < 300 && (b - a) > 1e-14; ++it) {
        if (fc > fd) {
            b = d; d = c; fd = fc;
            c = b - g * (b - a);
            fc = oracle_bethe_bloch(exp(c), za, i_ev);
        } else {
            a = c; c = d; fc = fd;
            d = a + g * (b - a);
            fd = oracle_bethe_bloch(exp(d), za, i_ev);
        }
    }
    return exp(0.5 * (a + b));
}

double oracle_stopping_power(double t, double za, double i_ev)
{
    double e_star = oracle_bb_peak_energy(za, i_ev);
    return oracle_bethe_bloch(t > e_star ? t : e_star, za, i_ev);
}

double oracle_water_z_over_a(void)
{
    return (2.0 * EL_Z[0] + EL_Z[3]) / (2.0 * EL_A[0] + EL_A[3]);
}

/* Range table R(E) = int_{E_cut}^{E} dE'/S(E') on a fine log grid,
 * integrated cell by cell with 5-point Gauss-Legendre in ln E, interpolated
 * by cubic Hermite using the exact derivative dR/dE = 1/S(E). */
#define RT_N 32769
#define RT_EMAX 300.0
typedef struct {
    double za, i_ev, e_star, ln_e0, h;
    double* e;
    double* r;
    double* inv_s;
} rtable;

static double rt_s(const rtable* t, double e)
{
    return oracle_bethe_bloch(e > t->e_star ? e : t->e_star, t->za, t->i_ev);
}

static int rt_build(rtable* t, double za, double i_ev)
{
    static const double gx[5] = {0.0, -0.5384693101056831, 0.5384693101056831,
                                 -0.9061798459386640, 0.9061798459386640};
    static const double gw[5] = {0.5688888888888889, 0.4786286704993665, 0.4786286704993665,
                                 0.2369268850561891, 0.2369268850561891};
    t->za = za;
    t->i_ev = i_ev;
    t->e_star = oracle_bb_peak_energy(za, i_ev);
    t->ln_e0 = log(E_CUT);
    t->h = (log(RT_EMAX) - t->ln_e0) / (RT_N - 1);
    t->e = (double*)malloc(sizeof(double) * RT_N);
    t->r = (double*)malloc(sizeof(double) * RT_N);
    t->inv_s = (double*)malloc(sizeof(double) * RT_N);
    if (!t->e || !t->r || !t->inv_s) return -3;
    for (int j = 0; j < RT_N; ++j) {
        t->e[j] = exp(t->ln_e0 + t->h * j);
        t->inv_s[j] = 1.0 / rt_s(t, t->e[j]);
    }
    t->e[0] = E_CUT;
    t->r[0] = 0.0;
    for (int j = 1; j < RT_N; ++j) {
        double xa = t->ln_e0 + t->h * (j - 1), half = 0.5 * t->h, acc = 0.0;
        for (int q = 0; q < 5; ++q) {
            double e = exp(xa + half * (1.0 + gx[q]));
            acc += gw[q] * e / rt_s(t, e);    /* dR/dlnE = E/S */
        }
        t->r[j] = t->r[j - 1] + half * acc;
    }
    return 0;
}

static void rt_free(rtable* t)
{
    free(t->e); free(t->r); free(t->inv_s);
    t->e = t->r = t->inv_s = NULL;
}

static int rt_cell(const rtable* t, double e)
{
    int j = (int)floor((log(e) - t->ln_e0) / t->h);
    if (j < 0) j = 0;
    if (j > RT_N - 2) j = RT_N - 2;
    /* guard against ln/exp rounding at cell edges */
    while (j > 0 && e < t->e[j]) --j;
    while (j < RT_N - 2 && e >= t->e[j + 1]) ++j;
    return j;
}

static double hermite(const rtable* t, int j, double e, double* deriv)
{
    double e0 = t->e[j], e1 = t->e[j + 1], len = e1 - e0;
    double s = (e - e0) / len, s2 = s * s, s3 = s2 * s;
    double h00 = 2 * s3 - 3 * s2 + 1, h10 = s3 - 2 * s2 + s;
    double h01 = -2 * s3 + 3 * s2, h11 = s3 - s2;
    double r = h00 * t->r[j] + h10 * len * t->inv_s[j] + h01 * t->r[j + 1] + h11 * len * t->inv_s[j + 1];
    if (deriv) {
        double d00 = 6 * s2 - 6 * s, d10 = 3 * s2 - 4 * s + 1, d01 = -6 * s2 + 6 * s, d11 = 3 * s2 - 2 * s;
        *deriv = (d00 * t->r[j] + d01 * t->r[j + 1]) / len + d10 * t->inv_s[j] + d11 * t->inv_s[j + 1];
    }
    return r;
}

static double rt_range(const rtable* t, double e)
{
    if (e <= E_CUT) return 0.0;
    return hermite(t, rt_cell(t, e), e, NULL);
}

static double rt_energy(const rtable* t, double r)
{
    if (r <= 0.0) return E_CUT;
    int lo = 0, hi = RT_N - 1;
    if (r >= t->r[hi]) return t->e[hi];
    while (hi - lo > 1) {               /* largest j with R_j <= r */
        int mid = (lo + hi) / 2;
        if (t->r[mid] <= r) lo = mid; else hi = mid;
    }
    double a = t->e[lo], b = t->e[lo + 1];
    double x = a + (b - a) * (r - t->r[lo]) / (t->r[lo + 1] - t->r[lo]);
    for (int it = 0; it < 60; ++it) {   /* bracketed Newton on the Hermite cubic */
        double dr;
        double f = hermite(t, lo, x, &dr) - r;
        if (f > 0) b = x; else a = x;
        double xn = (dr > 0) ? x - f / dr : 0.5 * (a + b);
        if (!(xn >= a && xn <= b)) xn = 0.5 * (a + b);
        if (fabs(xn - x) <= 4e-16 * x) { x = xn; break; }
        x = xn;
    }
    return x;
}

/* ======================================================================
 * Materials (Sec. II.A.1-2): per HU bin the composition fixes Z/A, the
 * water-equivalence factor f_m of Eq. 1 (ratio of Bethe-Bloch stopping powers
 * at 100 MeV, energy independent), the radiation length (Tsai's formula,
 * Bragg additivity in 1/X0) and the nuclei per gram.
 * ====================================================================== */
static double element_x0(int e)
{
    double z = EL_Z[e], a = EL_A[e];
    double az = ALPHA_FS * z, a2 = az * az;
    double fz = a2 * (1.0 / (1.0 + a2) + 0.20206 - 0.0369 * a2 + 0.0083 * a2 * a2 - 0.002 * a2 * a2 * a2);
    double lrad, lrad_p;
    if (z == 1.0) { lrad = 5.31; lrad_p = 6.144; }
    else { lrad = log(184.15 * pow(z, -1.0 / 3.0)); lrad_p = log(1194.0 * pow(z, -2.0 / 3.0)); }
    return X0_CONST * a / (z * z * (lrad - fz) + z * lrad_p);
}

double oracle_radiation_length(const double w[ORA_NEL])
{
    double inv = 0.0;
    for (int e = 0; e < ORA_NEL; ++e) inv += w[e] / element_x0(e);
    return 1.0 / inv;
}

typedef struct {
    int hu_lo, hu_hi;
    double rho_lo, rho_hi, i_ev, za, f, x0, w[ORA_NEL], n_per_g[ORA_NEL];
    int own;
    rtable own_rt;
} omat;

/* ======================================================================
 * Context
 * ====================================================================== */
struct ora_ctx {
    ora_params p;
    int have_physics, have_geometry;
    double sig[2][ORA_NEL][ORA_NE];      /* [elastic, non-elastic] barn */
    double mult[ORA_SEC_NUCLEI][ORA_SEC_EBINS][ORA_SEC_MULT];
    double floc[ORA_SEC_NUCLEI][ORA_SEC_EBINS];
    double xcdf[ORA_SEC_NUCLEI][ORA_SEC_EBINS][ORA_SEC_NCDF + 1];
    double mucdf[ORA_SEC_NUCLEI][ORA_SEC_EBINS][ORA_SEC_NCDF + 1];
    rtable water;
    double* vav;                         /* Vavilov quantile nodes (ORA_VAVILOV) */
    double* mol;                         /* Molière ln R table (ORA_MOLIERE) */
    int nmat;
    omat mat[16];
    int n[3];
    double vs[3];
    size_t nvox;
    unsigned char* vmat;
    double* vrho;
};

int oracle_create(ora_ctx** out, const ora_params* p)
{
    if (!out || !p) return -1;
    if (p->k_batches < 2 || p->f_mcs < 0 || p->s_min_cm <= 0) return -1;
    ora_ctx* c = (ora_ctx*)calloc(1, sizeof(ora_ctx));
    if (!c) return -3;
    c->p = *p;
    if (rt_build(&c->water, oracle_water_z_over_a(), WATER_I_EV)) { free(c); return -3; }
    if (p->flags & ORA_VAVILOV) {
        c->vav = (double*)malloc(sizeof(double) * ORA_VAV_NB * ORA_VAV_NK * ORA_VAV_NZ);
        if (!c->vav || oracle_vavilov_table(c->vav)) {
            free(c->vav);
            rt_free(&c->water);
            free(c);
            return -3;
        }
    }
    if (p->flags & ORA_MOLIERE) {
        c->mol = (double*)malloc(sizeof(double) * ORA_MOL_NX * ORA_MOL_NQ);
        if (!c->mol || oracle_moliere_table(c->mol)) {
            free(c->mol);
            free(c->vav);
            rt_free(&c->water);
            free(c);
            return -3;
        }
    }
    *out = c;
    return 0;
}

double oracle_vavilov_quantile(const ora_ctx* c, double kappa, double beta2, double z)
{
    if (!c || !c->vav) return NAN;
    return vav_quantile(c->vav, kappa, beta2, z);
}

static void free_geometry(ora_ctx* c)
{
    for (int m = 0; m < c->nmat; ++m)
        if (c->mat[m].own) rt_free(&c->mat[m].own_rt);
    free(c->vmat); free(c->vrho);
    c->vmat = NULL; c->vrho = NULL; c->nmat = 0; c->have_geometry = 0;
}

int oracle_destroy(ora_ctx* c)
{
    if (!c) return 0;
    free_geometry(c);
    rt_free(&c->water);
    free(c->vav);
    free(c->mol);
    free(c);
    return 0;
}

int oracle_load_physics(ora_ctx* c, const ora_nuclear_data* nd)
{
    if (!c || !nd || !nd->sigma_ne || !nd->sigma_el || !nd->mult_cdf || !nd->f_local ||
        !nd->x_cdf || !nd->mu_cdf) return -1;
    for (int e = 0; e < ORA_NEL; ++e)
        for (int i = 0; i < ORA_NE; ++i) {
            c->sig[0][e][i] = nd->sigma_el[e * ORA_NE + i];
            c->sig[1][e][i] = nd->sigma_ne[e * ORA_NE + i];
            if (c->sig[0][e][i] < 0 || c->sig[1][e][i] < 0) return -1;
        }
    for (int n = 0; n < ORA_SEC_NUCLEI; ++n)
        for (int j = 0; j < ORA_SEC_EBINS; ++j) {
            int b = n * ORA_SEC_EBINS + j;
            for (int m = 0; m < ORA_SEC_MULT; ++m) c->mult[n][j][m] = nd->mult_cdf[b * ORA_SEC_MULT + m];
            c->floc[n][j] = nd->f_local[b];
            for (int i = 0; i <= ORA_SEC_NCDF; ++i) {
                c->xcdf[n][j][i] = nd->x_cdf[b * (ORA_SEC_NCDF + 1) + i];
                c->mucdf[n][j][i] = nd->mu_cdf[b * (ORA_SEC_NCDF + 1) + i];
            }
            if (c->mult[n][j][ORA_SEC_MULT - 1] != 1.0 || c->xcdf[n][j][0] != 0.0 ||
                c->xcdf[n][j][ORA_SEC_NCDF] != 1.0 || c->mucdf[n][j][0] != 0.0 ||
                c->mucdf[n][j][ORA_SEC_NCDF] != 1.0) return -1;
        }
    c->have_physics = 1;
    return 0;
}

int oracle_load_geometry(ora_ctx* c, const int16_t* hu, int nx, int ny, int nz,
                         float dx, float dy, float dz, const ora_material_table* mt)
{
    if (!c || !hu || !mt || nx <= 0 || ny <= 0 || nz <= 0 || !(dx > 0) || !(dy > 0) || !(dz > 0))
        return -1;
    if (mt->n_bins < 1 || mt->n_bins > 16 || !mt->hu_lo || !mt->rho_lo || !mt->rho_hi ||
        !mt->mass_frac || !mt->i_ev || !mt->own_table) return -1;
    if (mt->hu_lo[0] > -1000) return -1;
    for (int b = 1; b < mt->n_bins; ++b)
        if (mt->hu_lo[b] <= mt->hu_lo[b - 1] || mt->hu_lo[b] > 3000) return -1;
    free_geometry(c);
    double za_w = oracle_water_z_over_a();
    double s_water_ref = oracle_bethe_bloch(E_REF, za_w, WATER_I_EV);
    c->nmat = mt->n_bins;
    for (int b = 0; b < mt->n_bins; ++b) {
        omat* m = &c->mat[b];
        memset(m, 0, sizeof(*m));
        m->hu_lo = mt->hu_lo[b];
        m->hu_hi = (b + 1 < mt->n_bins) ? mt->hu_lo[b + 1] : 3000;
        m->rho_lo = mt->rho_lo[b];
        m->rho_hi = mt->rho_hi[b];
        m->i_ev = mt->i_ev[b];
        m->own = mt->own_table[b] != 0;
        if (!(m->rho_lo > 0) || !(m->rho_hi > 0) || !(m->i_ev > 0)) { c->nmat = b; free_geometry(c); return -1; }
        double sum = 0.0;
        for (int e = 0; e < ORA_NEL; ++e) {
            m->w[e] = mt->mass_frac[b * ORA_NEL + e];
            if (m->w[e] < 0) { c->nmat = b; free_geometry(c); return -1; }
            sum += m->w[e];
        }
        if (fabs(sum - 1.0) > 1e-4) { c->nmat = b; free_geometry(c); return -1; }
        m->za = 0.0;
        for (int e = 0; e < ORA_NEL; ++e) {
            m->za += m->w[e] * EL_Z[e] / EL_A[e];
            m->n_per_g[e] = m->w[e] * N_AVOGADRO / EL_A[e];
        }
        m->x0 = oracle_radiation_length(m->w);
        if (m->own) {
            m->f = 1.0;
            if (rt_build(&m->own_rt, m->za, m->i_ev)) { c->nmat = b + 1; free_geometry(c); return -3; }
        } else {
            m->f = oracle_bethe_bloch(E_REF, m->za, m->i_ev) / s_water_ref;   /* Eq. 1 */
        }
    }
    c->n[0] = nx; c->n[1] = ny; c->n[2] = nz;
    c->vs[0] = dx; c->vs[1] = dy; c->vs[2] = dz;
    c->nvox = (size_t)nx * ny * nz;
    c->vmat = (unsigned char*)malloc(c->nvox);
    c->vrho = (double*)malloc(sizeof(double) * c->nvox);
    if (!c->vmat || !c->vrho) { free_geometry(c); return -3; }
    for (size_t v = 0; v < c->nvox; ++v) {
        int h = hu[v];
        if (h < -1000) h = -1000;
        if (h > 3000) h = 3000;
        int b = 0;
        while (b + 1 < c->nmat && c->mat[b + 1].hu_lo <= h) ++b;
        const omat* m = &c->mat[b];
        double rho = m->rho_lo;
        if (m->hu_hi > m->hu_lo)
            rho = m->rho_lo + (m->rho_hi - m->rho_lo) * (double)(h - m->hu_lo) / (double)(m->hu_hi - m->hu_lo);
        c->vmat[v] = (unsigned char)b;
        c->vrho[v] = rho;
    }
    c->have_geometry = 1;
    return 0;
}

static const rtable* table_of(const ora_ctx* c, int m)
{
    return c->mat[m].own ? &c->mat[m].own_rt : &c->water;
}

double oracle_range(const ora_ctx* c, int table, double t)
{
    if (table == 0) return rt_range(&c->water, t);
    return rt_range(&c->mat[table - 1].own_rt, t);
}

double oracle_energy_at_range(const ora_ctx* c, int table, double r)
{
    if (table == 0) return rt_energy(&c->water, r);
    return rt_energy(&c->mat[table - 1].own_rt, r);
}

int oracle_material_info(const ora_ctx* c, int m, double out[6])
{
    if (!c || m < 0 || m >= c->nmat) return -1;
    double n = 0.0;
    for (int e = 0; e < ORA_NEL; ++e) n += c->mat[m].n_per_g[e];
    out[0] = c->mat[m].za; out[1] = c->mat[m].i_ev; out[2] = c->mat[m].f;
    out[3] = c->mat[m].x0; out[4] = c->mat[m].own; out[5] = n;
    return 0;
}

/* ======================================================================
 * Cross sections (Sec. II.A.3-5): tabulated per element, linear in ln E.
 * ====================================================================== */
static double grid_interp(const double* tab, double t)
{
    double x = (log(t) - log(GRID_EMIN)) / (log(GRID_EMAX / GRID_EMIN) / (ORA_NE - 1));
    int i = (int)floor(x);
    if (i < 0) { i = 0; x = 0.0; }
    if (i > ORA_NE - 2) { i = ORA_NE - 2; x = ORA_NE - 1; }
    double f = x - i;
    return tab[i] + f * (tab[i + 1] - tab[i]);
}

double oracle_sigma(const ora_ctx* c, int process, int element, double t)
{
    return grid_interp(c->sig[process][element], t);
}

/* macroscopic cross section per unit density, cm^2/g, for one process */
static double sigma_per_g(const ora_ctx* c, const omat* m, int process, double t, double part[ORA_NEL])
{
    double sum = 0.0;
    for (int e = 0; e < ORA_NEL; ++e) {
        double v = (m->w[e] > 0) ? m->n_per_g[e] * grid_interp(c->sig[process][e], t) * BARN_CM2 : 0.0;
        if (part) part[e] = v;
        sum += v;
    }
    return sum;
}

/* ======================================================================
 * Multiple scattering and straggling (Sec. II.A.2)
 * ====================================================================== */
double oracle_highland_theta0(double t, double s, double x0_cm, double f)
{
    double e_tot = t + M_PROTON;
    double pv = t * (t + 2.0 * M_PROTON) / e_tot;               /* p beta c, MeV */
    double beta2 = t * (t + 2.0 * M_PROTON) / (e_tot * e_tot);
    double bracket = 1.0 + 0.038 * log(s / (x0_cm * beta2));
    if (bracket < 0.0) bracket = 0.0;
    return f * 13.6 / pv * sqrt(s / x0_cm) * bracket;
}

double oracle_straggling_variance(double t, double s, double rho, double za)
{
    double gamma = 1.0 + t / M_PROTON;
    double e_tot = t + M_PROTON;
    double beta2 = t * (t + 2.0 * M_PROTON) / (e_tot * e_tot);
    return K_BETHE * M_ELECTRON * rho * za * s * gamma * gamma * (1.0 - 0.5 * beta2);
}

/* ======================================================================
 * Vavilov straggling (Sec. II.A.2: a Vavilov-Gaussian model of the energy
 * loss fluctuations)
 *
 * The loss of a step is <Delta> + sigma W, sigma^2 the Bohr variance above
 * and W standardised (mean 0, variance 1).  With the Vavilov parameter
 * kappa = xi / T_max in [0.01, 10), W follows Vavilov's distribution for
 * (kappa, beta^2); outside that range W is standard normal.  Vavilov's
 * model: free-electron collisions with energy transfers v T_max, v in
 * (0, 1], occurring with density kappa (1 - beta^2 v) / v^2.  Then
 * X = (Delta - <Delta>) / T_max has
 *   ln E[exp(i t X)] = kappa (A(t) + i B(t)),
 *   A(t) = Int_0^1 (1 - beta^2 v)(cos tv - 1) / v^2 dv,
 *   B(t) = Int_0^1 (1 - beta^2 v)(sin tv - tv) / v^2 dv,
 * and W = X / sqrt(kappa (1 - beta^2 / 2)).  Here A and B come from running
 * integrals of the integrands after substituting x = t v:
 *   A = t J2(t) - beta^2 J1(t),  B = t K2(t) - beta^2 K1(t),
 *   J2 = Int_0^t (cos x - 1)/x^2, J1 = Int_0^t (cos x - 1)/x,
 *   K2 = Int_0^t (sin x - x)/x^2, K1 = Int_0^t (sin x - x)/x,
 * accumulated by Simpson's rule, and the distribution function from the
 * Gil-Pelaez inversion
 *   F(x) = 1/2 - (1/pi) Int_0^inf exp(kappa A) sin(kappa B - t x) / t dt.
 * The sampler maps z = Phi^-1(u) through the quantile function
 * W = G(z) = F_W^-1(Phi(z)), tabulated at z = -6 + i/8 (97 nodes),
 * log10 kappa = -2 + j/10 (31 nodes) and beta^2 = k/10 (k = 0..4), and
 * interpolated trilinearly (beta^2 clamped to [0, 0.4]).
 * ====================================================================== */
#define VAV_DU 0.01              /* running-integral step */
#define VAV_UMAX 12000.0         /* supports kappa >= 0.0025 */
static double* vav_run = NULL;   /* [n][4]: J2, J1, K2, K1 at u = k VAV_DU */
static long vav_n = 0;

static void vav_integrands(double x, double f[4])
{
    if (x < 0.02) {              /* series: the closed forms cancel badly near 0 */
        double x2 = x * x;
        f[0] = -0.5 + x2 / 24.0 - x2 * x2 / 720.0;
        f[1] = x * (-0.5 + x2 / 24.0 - x2 * x2 / 720.0);
        f[2] = x * (-1.0 / 6.0 + x2 / 120.0 - x2 * x2 / 5040.0);
        f[3] = x2 * (-1.0 / 6.0 + x2 / 120.0 - x2 * x2 / 5040.0);
        return;
    }
    double c = cos(x) - 1.0, sn = sin(x) - x;
    f[0] = c / (x * x);
    f[1] = c / x;
    f[2] = sn / (x * x);
    f[3] = sn / x;
}

static int vav_build_running(void)
{
    int ok = 1;
#pragma omp critical(vav_running)
    {
        if (!vav_run) {
            long n = (long)(VAV_UMAX / VAV_DU) + 2;
            double* r = (double*)malloc(sizeof(double) * 4 * (size_t)n);
            if (!r) ok = 0;
            else {
                double acc[4] = {0, 0, 0, 0}, f0[4], fm[4], f1[4];
                vav_integrands(0.0, f0);
                for (int q = 0; q < 4; ++q) r[q] = 0.0;
                for (long k = 1; k < n; ++k) {
                    double a = (k - 1) * VAV_DU, b = k * VAV_DU;
                    vav_integrands(0.5 * (a + b), fm);
                    vav_integrands(b, f1);
                    for (int q = 0; q < 4; ++q) {
                        acc[q] += VAV_DU / 6.0 * (f0[q] + 4.0 * fm[q] + f1[q]);
                        r[4 * k + q] = acc[q];
                        f0[q] = f1[q];
                    }
                }
                vav_n = n;
                vav_run = r;
            }
        }
    }
    return ok && vav_run != NULL;
}

/* kappa A and kappa B at t = k VAV_DU */
static void vav_ab(long k, double kappa, double beta2, double* ka, double* kb)
{
    const double t = k * VAV_DU;
    const double* r = vav_run + 4 * k;
    *ka = kappa * (t * r[0] - beta2 * r[1]);
    *kb = kappa * (t * r[2] - beta2 * r[3]);
}

/* support window of X used for the inversion step: the distribution has
 * negligible mass (far below 1e-9) outside it */
static void vav_window(double kappa, double* lo, double* hi)
{
    *lo = -8.0 * sqrt(kappa) - 0.1;
    *hi = 4.0 + 8.0 * sqrt(kappa);
}

/* Gil-Pelaez sums for the points x[0..nx): F[i] = P(X <= x[i]) */
static int vav_cdf_points(double kappa, double beta2, const double* x, int nx, double* F)
{
    if (!(kappa > 0.0) || beta2 < 0.0 || beta2 >= 1.0 || !vav_build_running()) return -1;
    double lo, hi;
    vav_window(kappa, &lo, &hi);
    /* midpoint rule, step dt = 2 m VAV_DU with 2 pi / dt at least twice the window */
    long m = (long)floor(M_PI / (hi - lo) / (2.0 * VAV_DU));
    if (m < 1) m = 1;
    const double dt = 2.0 * m * VAV_DU;
    /* nodes t_j = (j + 1/2) dt = (2j + 1) m VAV_DU while exp(kappa A) > e^-45 */
    long nt = 0;
    while (1) {
        long k = (2 * nt + 1) * m;
        if (k >= vav_n) return -2;
        double ka, kb;
        vav_ab(k, kappa, beta2, &ka, &kb);
        if (ka < -45.0) break;
        ++nt;
    }
    double* amp = (double*)malloc(sizeof(double) * 3 * (size_t)(nt > 0 ? nt : 1));
    if (!amp) return -3;
    for (long j = 0; j < nt; ++j) {
        long k = (2 * j + 1) * m;
        double ka, kb;
        vav_ab(k, kappa, beta2, &ka, &kb);
        double t = k * VAV_DU;
        amp[3 * j] = exp(ka) / t;
        amp[3 * j + 1] = kb;
        amp[3 * j + 2] = t;
    }
    for (int i = 0; i < nx; ++i) {
        double sum = 0.0;
        for (long j = 0; j < nt; ++j) sum += amp[3 * j] * sin(amp[3 * j + 1] - amp[3 * j + 2] * x[i]);
        F[i] = 0.5 - sum * dt / M_PI;
    }
    free(amp);
    return 0;
}

double oracle_vavilov_cdf(double kappa, double beta2, double x)
{
    double f;
    if (vav_cdf_points(kappa, beta2, &x, 1, &f)) return NAN;
    return f;
}

static double std_normal_cdf_z(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

/* quantile nodes of W for one (kappa, beta^2): G[i] at z = -6 + i/8 */
static int vav_nodes(double kappa, double beta2, double* G)
{
    const double euler = 0.57721566490153286;
    double lo, hi;
    vav_window(kappa, &lo, &hi);
    /* points: uniform in lambda = X/kappa - (1 - euler) - ln kappa (step
     * 1/40) over the Landau-like core, then uniform in X to the window end */
    const double l0 = fmax(-8.0, lo / kappa - (1.0 - euler) - log(kappa));
    const double l_hi = hi / kappa - (1.0 - euler) - log(kappa);
    const double l1 = fmin(25.0, l_hi);
    int n1 = (int)ceil((l1 - l0) * 40.0) + 1, n2 = l_hi > l1 ? 400 : 0;
    int nx = n1 + n2;
    double* x = (double*)malloc(sizeof(double) * 2 * (size_t)nx);
    if (!x) return -3;
    double* F = x + nx;
    for (int i = 0; i < n1; ++i) {
        double l = l0 + (l1 - l0) * i / (n1 - 1);
        x[i] = kappa * (l + (1.0 - euler) + log(kappa));
    }
    for (int i = 0; i < n2; ++i) x[n1 + i] = x[n1 - 1] + (hi - x[n1 - 1]) * (i + 1) / n2;
    int rc = vav_cdf_points(kappa, beta2, x, nx, F);
    if (rc) { free(x); return rc; }
    for (int i = 0; i < nx; ++i) {          /* a distribution function: in [0, 1], non-decreasing */
        if (F[i] < 0.0) F[i] = 0.0;
        if (F[i] > 1.0) F[i] = 1.0;
        if (i > 0 && F[i] < F[i - 1]) F[i] = F[i - 1];
    }
    const double c = sqrt(kappa * (1.0 - 0.5 * beta2));
    int at = 0;
    for (int q = 0; q < ORA_VAV_NZ; ++q) {
        double u = std_normal_cdf_z(-6.0 + q / 8.0);
        while (at < nx - 1 && F[at] < u) ++at;
        double xq;
        if (at == 0) xq = x[0];
        else if (F[at] < u) xq = x[nx - 1];
        else {
            double fa = F[at - 1], fb = F[at];
            xq = fb > fa ? x[at - 1] + (x[at] - x[at - 1]) * (u - fa) / (fb - fa) : x[at];
        }
        G[q] = xq / c;
    }
    free(x);
    return 0;
}

int oracle_vavilov_table(double* out)
{
    if (!out) return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int jb = 0; jb < ORA_VAV_NB * ORA_VAV_NK; ++jb) {
        const int b = jb / ORA_VAV_NK, j = jb % ORA_VAV_NK;
        const double kappa = pow(10.0, -2.0 + j / 10.0);
        if (vav_nodes(kappa, 0.1 * b, out + (size_t)jb * ORA_VAV_NZ)) bad = 1;
    }
    return bad ? -2 : 0;
}

/* W for normal score z at (kappa, beta^2) from the table t (trilinear) */
static double vav_quantile(const double* t, double kappa, double beta2, double z)
{
    if (!(kappa >= 0.01 && kappa < 10.0)) return z;
    double fk = (log10(kappa) + 2.0) * 10.0;
    int j = (int)floor(fk);
    if (j > ORA_VAV_NK - 2) j = ORA_VAV_NK - 2;
    fk -= j;
    double fb = fmin(fmax(beta2, 0.0), 0.4) * 10.0;
    int b = (int)floor(fb);
    if (b > ORA_VAV_NB - 2) b = ORA_VAV_NB - 2;
    fb -= b;
    double fz = (z + 6.0) * 8.0;
    int q = (int)floor(fz);
    if (q < 0) q = 0;
    if (q > ORA_VAV_NZ - 2) q = ORA_VAV_NZ - 2;
    fz -= q;                      /* beyond the end nodes: linear extrapolation */
    double acc = 0.0;
    for (int db = 0; db < 2; ++db)
        for (int dj = 0; dj < 2; ++dj) {
            const double* row = t + ((size_t)(b + db) * ORA_VAV_NK + (j + dj)) * ORA_VAV_NZ;
            double g = row[q] + fz * (row[q + 1] - row[q]);
            acc += (db ? fb : 1.0 - fb) * (dj ? fk : 1.0 - fk) * g;
        }
    return acc;
}

/* Vavilov parameter of a step: xi / T_max */
double oracle_vavilov_kappa(double t, double s, double rho, double za)
{
    const double gamma = 1.0 + t / M_PROTON;
    const double e_tot = t + M_PROTON;
    const double beta2 = t * (t + 2.0 * M_PROTON) / (e_tot * e_tot);
    const double xi = 0.5 * K_BETHE * za * rho * s / beta2;
    const double r = M_ELECTRON / M_PROTON;
    const double tmax = 2.0 * M_ELECTRON * beta2 * gamma * gamma / (1.0 + 2.0 * gamma * r + r * r);
    return xi / tmax;
}

/* ======================================================================
 * Molière multiple scattering (Sec. II.A.2 names a full Molière option
 * beside the scaled Highland formula), in Bethe's form:
 *   f(theta) theta dtheta = v dv [f0(v) + f1(v)/B + f2(v)/B^2],
 *   v = theta / (chi_c sqrt B), f0 = 2 exp(-v^2),
 *   fn(v) = (1/n!) Int_0^inf u J0(v u) exp(-u^2/4) [(u^2/4) ln(u^2/4)]^n du,
 * chi_c^2 = 4 pi N_A e^4 (rho s) sum_i w_i Z_i (Z_i + 1) / A_i / (p beta)^2,
 * the screening angle of element i chi_a,i^2 = chi_0,i^2 (1.13 + 3.76
 * (Z_i alpha / beta)^2), chi_0,i = hbar c Z_i^(1/3) / (0.885 a_0 p c),
 * combined as ln chi_a^2 = sum_i w_i Z_i (Z_i + 1)/A_i ln chi_a,i^2 / sum of
 * the same weights, and B from B - ln B = ln(chi_c^2 / (1.167 chi_a^2)).
 * The expansion needs B >= 4.5; a step with fewer collisions keeps the
 * scaled Highland Gaussian.
 * Sampling: with q = -ln u, v^2 = q R(q, 1/B), the function ln R tabulated
 * at q = k/8 (k <= 160) and 1/B = 1/20 + j (2/9 - 1/20)/12 (j <= 12; 1/B
 * clamped to that range), interpolated bilinearly (linear extrapolation in
 * q beyond 20); theta = min(pi, chi_c sqrt(B) v), azimuth uniform.
 * The distribution functions Fn(v) = Int_0^v fn v' dv' =
 * (v/n!) Int_0^inf J1(v u) exp(-u^2/4) [(u^2/4) ln(u^2/4)]^n du are
 * integrated by Simpson's rule on v <= 20 and continued beyond by their
 * asymptotic forms F1 = -(v^-2 + 2 v^-4), F2 proportional to ln v / v^4.
 * ====================================================================== */
#define MOL_VMAX 20.0
#define MOL_DV 0.02
#define MOL_NV 1001                  /* v grid 0 .. 20 */
static double* mol_F = NULL;         /* [MOL_NV][2]: F1, F2 */

static double mol_g(double u, int n)
{
    const double y = 0.25 * u * u;
    if (y <= 0.0) return 0.0;
    const double t = y * log(y);
    return exp(-y) * (n == 1 ? t : 0.5 * t * t);
}

double oracle_moliere_f(int n, double v)
{
    if (n == 0) return 2.0 * exp(-v * v);
    if (n != 1 && n != 2) return NAN;
    const int N = 28000;                /* u in [0, 14], step 5e-4 */
    const double h = 14.0 / N;
    double s = 0.0;
    for (int k = 0; k <= N; ++k) {
        const double u = k * h;
        const double w = (k == 0 || k == N) ? 1.0 : (k & 1 ? 4.0 : 2.0);
        s += w * u * j0(v * u) * mol_g(u, n);
    }
    return s * h / 3.0;
}

static double mol_F_direct(int n, double v)
{
    const int N = 14000;                /* u in [0, 14], step 1e-3 */
    const double h = 14.0 / N;
    double s = 0.0;
    for (int k = 0; k <= N; ++k) {
        const double u = k * h;
        const double w = (k == 0 || k == N) ? 1.0 : (k & 1 ? 4.0 : 2.0);
        s += w * j1(v * u) * mol_g(u, n);
    }
    return v * s * h / 3.0;
}

static int mol_build_F(void)
{
    int ok = 1;
#pragma omp critical(mol_F)
    {
        if (!mol_F) {
            double* t = (double*)malloc(sizeof(double) * 2 * MOL_NV);
            if (!t) ok = 0;
            else {
#pragma omp parallel for schedule(dynamic, 8)
                for (int i = 0; i < MOL_NV; ++i) {
                    t[2 * i] = mol_F_direct(1, i * MOL_DV);
                    t[2 * i + 1] = mol_F_direct(2, i * MOL_DV);
                }
                mol_F = t;
            }
        }
    }
    return ok && mol_F;
}

/* F1 and F2 at v */
static void mol_F12(double v, double* f1, double* f2)
{
    if (v >= MOL_VMAX) {
        const double r = MOL_VMAX / v;
        *f1 = -(1.0 / (v * v) + 2.0 / (v * v * v * v));
        *f2 = mol_F[2 * (MOL_NV - 1) + 1] * r * r * r * r * log(v) / log(MOL_VMAX);
        return;
    }
    const double x = v / MOL_DV;
    int i = (int)x;
    if (i > MOL_NV - 2) i = MOL_NV - 2;
    const double fr = x - i;
    *f1 = mol_F[2 * i] + fr * (mol_F[2 * i + 2] - mol_F[2 * i]);
    *f2 = mol_F[2 * i + 1] + fr * (mol_F[2 * i + 3] - mol_F[2 * i + 1]);
}

/* P(V > v) for 1/B = x */
double oracle_moliere_survival(double x, double v)
{
    if (!mol_build_F()) return NAN;
    double f1, f2;
    mol_F12(v, &f1, &f2);
    return exp(-v * v) - x * f1 - x * x * f2;
}

static double mol_x_node(int j) { return 0.05 + j * (2.0 / 9.0 - 0.05) / (ORA_MOL_NX - 1); }

int oracle_moliere_table(double* out)
{
    if (!out || !mol_build_F()) return -1;
    const double euler = 0.57721566490153286;
    const double f1_0 = 2.0 * (1.0 - euler);
    const double f2_0 = 2.0 * ((1.5 - euler) * (1.5 - euler) + M_PI * M_PI / 6.0 - 1.25);
#pragma omp parallel for
    for (int j = 0; j < ORA_MOL_NX; ++j) {
        const double x = mol_x_node(j);
        for (int k = 0; k < ORA_MOL_NQ; ++k) {
            const double q = k / 8.0;
            if (k == 0) {                       /* small v: F = f(0) v^2 / 2 */
                out[j * ORA_MOL_NQ] = log(2.0 / (2.0 + x * f1_0 + x * x * f2_0));
                continue;
            }
            const double target = exp(-q);     /* P(V > v) = 1 - u = e^-q */
            double lo = 0.0, hi = 1.0e5;
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (oracle_moliere_survival(x, mid) > target) lo = mid;
                else hi = mid;
            }
            const double v = 0.5 * (lo + hi);
            out[j * ORA_MOL_NQ + k] = log(v * v / q);
        }
    }
    return 0;
}

/* ln chi_c^2, ln chi_a^2 and B of a step; returns 0 when B < 4.5 */
static int mol_step(const omat* m, double t, double rho, double s, double* chi_c2, double* bB)
{
    const double e_tot = t + M_PROTON;
    const double pc = sqrt(t * (t + 2.0 * M_PROTON));
    const double beta2 = pc * pc / (e_tot * e_tot);
    const double pbeta = pc * pc / e_tot;
    double s1 = 0.0, la = 0.0;
    for (int e = 0; e < ORA_NEL; ++e) {
        if (m->w[e] <= 0.0) continue;
        const double z = EL_Z[e];
        const double wt = m->w[e] * z * (z + 1.0) / EL_A[e];
        const double chi0 = 0.0042134917 * cbrt(z) / pc;
        const double za = z * ALPHA_FS;
        s1 += wt;
        la += wt * log(chi0 * chi0 * (1.13 + 3.76 * za * za / beta2));
    }
    la /= s1;
    const double lc = log(K_BETHE * M_ELECTRON * s1 * rho * s / (pbeta * pbeta));
    const double b = lc - log(1.167) - la;
    if (b < 4.5 - log(4.5)) return 0;
    double B = b + log(b);
    for (int it = 0; it < 30; ++it) B -= (B - log(B) - b) / (1.0 - 1.0 / B);
    *chi_c2 = exp(lc);
    *bB = B;
    return 1;
}

/* polar angle for uniform u (q = -ln u) from the table */
static double mol_theta(const double* tab, double chi_c2, double B, double u)
{
    double x = 1.0 / B;
    if (x < 0.05) x = 0.05;
    if (x > 2.0 / 9.0) x = 2.0 / 9.0;
    double fx = (x - 0.05) / ((2.0 / 9.0 - 0.05) / (ORA_MOL_NX - 1));
    int j = (int)fx;
    if (j > ORA_MOL_NX - 2) j = ORA_MOL_NX - 2;
    fx -= j;
    const double q = -log(u);
    double fq = q * 8.0;
    int k = (int)fq;
    if (k > ORA_MOL_NQ - 2) k = ORA_MOL_NQ - 2;
    fq -= k;
    const double* r0 = tab + j * ORA_MOL_NQ;
    const double* r1 = r0 + ORA_MOL_NQ;
    const double a = r0[k] + fq * (r0[k + 1] - r0[k]);
    const double c = r1[k] + fq * (r1[k + 1] - r1[k]);
    const double v2 = q * exp(a + fx * (c - a));
    const double th = sqrt(chi_c2 * B * v2);
    return th < M_PI ? th : M_PI;
}

double oracle_moliere_theta(const ora_ctx* c, int material, double t_mev, double rho, double s_cm,
                            double u, double* b_out)
{
    if (!c || !c->mol || material < 0 || material >= c->nmat) return NAN;
    double chi_c2, B;
    if (!mol_step(&c->mat[material], t_mev, rho, s_cm, &chi_c2, &B)) {
        if (b_out) *b_out = 0.0;
        return NAN;
    }
    if (b_out) *b_out = B;
    return mol_theta(c->mol, chi_c2, B, u);
}

void oracle_rotate(double d[3], double ct, double st, double phi_rev)
{
    double cp = cos(2.0 * M_PI * phi_rev), sp = sin(2.0 * M_PI * phi_rev);
    double u = d[0], v = d[1], w = d[2];
    double perp = sqrt(u * u + v * v);
    if (perp < 1e-6) {
        d[0] = st * cp;
        d[1] = st * sp;
        d[2] = (w >= 0.0 ? 1.0 : -1.0) * ct;
        return;
    }
    d[0] = u * ct + st * (u * w * cp - v * sp) / perp;
    d[1] = v * ct + st * (v * w * cp + u * sp) / perp;
    d[2] = w * ct - st * cp * perp;
}

/* ======================================================================
 * Nuclear elastic scattering (Sec. II.A.5, Eq. 3): momentum transfer from
 * Ranft's two-exponential form (A >= 2) or isotropic in the CM (p-p), exact
 * relativistic two-body kinematics on a target of mass A u at rest.
 * ====================================================================== */
int oracle_elastic_sample(int a, double t, double u_comp, double u_t, double out[7])
{
    double m = M_PROTON;
    double big_m = (a == 1) ? M_PROTON : a * M_AMU;
    double s_mand = (m + big_m) * (m + big_m) + 2.0 * big_m * t;
    double pcm2 = big_m * big_m * t * (t + 2.0 * m) / s_mand;      /* MeV^2 */
    double tabs;
    if (a == 1) {
        tabs = 4.0 * pcm2 * (1.0 - u_t);                            /* cos_cm = 2u - 1 */
    } else {
        double a1, b1, a2, b2;
        if (a <= 62) { a1 = pow(a, 1.63); b1 = 14.5 * pow(a, 0.66); a2 = 1.4 * pow(a, 0.33); b2 = 10.0; }
        else { a1 = pow(a, 1.33); b1 = 60.0 * pow(a, 0.33); a2 = 0.4 * pow(a, 0.4); b2 = 10.0; }
        double tmax = 4.0 * pcm2 * 1e-6;                            /* (GeV/c)^2 */
        double c1 = -expm1(-b1 * tmax), c2 = -expm1(-b2 * tmax);
        double w1 = a1 * c1 / b1, w2 = a2 * c2 / b2;
        double b = b2, cc = c2;
        if (u_comp * (w1 + w2) < w1) { b = b1; cc = c1; }
        tabs = -log1p(-u_t * cc) / b * 1e6;
    }
    double tr = tabs / (2.0 * big_m);
    double tn = t - tr;
    double p = sqrt(t * (t + 2.0 * m));
    double pn = sqrt(tn > 0 ? tn * (tn + 2.0 * m) : 0.0);
    double ct = 1.0, st = 0.0, cr = 1.0, sr = 0.0;
    if (pn > 0.0 && tr > 0.0) {
        double dp = tr * (t + tn + 2.0 * m) / (p + pn);
        double q2 = tr * (tr + 2.0 * big_m);
        double omc = (q2 - dp * dp) / (2.0 * p * pn);
        if (omc < 0.0) omc = 0.0;
        if (omc > 2.0) omc = 2.0;
        ct = 1.0 - omc;
        st = sqrt(omc * (2.0 - omc));
        double pr = sqrt(q2);
        cr = (dp + pn * omc) / pr;
        sr = pn * st / pr;
    }
    out[0] = tabs; out[1] = tr; out[2] = tn; out[3] = ct; out[4] = st; out[5] = cr; out[6] = sr;
    return 0;
}

/* ======================================================================
 * Non-elastic secondaries (Sec. II.A.4, replaced by a synthetic table).
 * ====================================================================== */
static double inverse_cdf(const double* cdf, double u, double lo, double hi)
{
    int i = ORA_SEC_NCDF - 1;
    while (i > 0 && cdf[i] > u) --i;    /* largest bin whose lower CDF edge <= u */
    double frac = (u - cdf[i]) / (cdf[i + 1] - cdf[i]);
    return lo + (hi - lo) * (i + frac) / ORA_SEC_NCDF;
}

static int sec_bin(double t)
{
    int j = (int)floor(t / 10.0);
    if (j < 0) j = 0;
    if (j > ORA_SEC_EBINS - 1) j = ORA_SEC_EBINS - 1;
    return j;
}

int oracle_secondary_sample(const ora_ctx* c, int element, double t, uint64_t uid, uint32_t k,
                            uint64_t seed, double u_mult, int* n_out, double e_out[4],
                            double mu_out[4], double* f_local)
{
    if (element < 1 || element >= ORA_NEL) return -1;
    int nu = element - 1, j = sec_bin(t);
    int n = 0;
    while (n < ORA_SEC_MULT - 1 && !(u_mult < c->mult[nu][j][n])) ++n;
    double fl = c->floc[nu][j];
    double sum = 0.0;
    for (int q = 0; q < n; ++q) {
        double u[4];
        draw4(seed, uid, k, 16u + (uint32_t)(q + 1), u);
        e_out[q] = inverse_cdf(c->xcdf[nu][j], u[0], 0.0, 1.0) * t;
        mu_out[q] = inverse_cdf(c->mucdf[nu][j], u[1], -1.0, 1.0);
        sum += e_out[q];
    }
    double avail = (1.0 - fl) * t;
    if (sum > avail) {
        double r = avail / sum;
        for (int q = 0; q < n; ++q) e_out[q] *= r;
    }
    *n_out = n;
    *f_local = fl;
    return 0;
}

/* ======================================================================
 * Transport (Sec. II.A.3 transport mechanics, one history per worker,
 * Sec. II.B.1)
 * ====================================================================== */
typedef struct {
    double p[3];     /* position in voxel units */
    double d[3];     /* direction cosines */
    double e, mfp, w;
    uint64_t uid;
    uint32_t k;
    int batch, primary;
} opart;

typedef struct {
    opart* a;
    size_t n, cap;
} ostack;

typedef struct {
    double escaped, neutral;
    uint64_t steps, secondaries, n_el, n_ne, n_short;
    uint64_t inter[2][ORA_NEL];
} oacc;

typedef struct {
    uint64_t seed;
    double* tally;   /* nvox x K */
    ora_diag* diag;
    double* let_num; /* nvox: sum of w * eps * L over proton steps (NULL = not scored) */
    double* let_den; /* nvox: sum of w * eps over the same steps */
} orun;

static void push(ostack* s, const opart* q)
{
    if (s->n == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 64;
        s->a = (opart*)realloc(s->a, s->cap * sizeof(opart));
    }
    s->a[s->n++] = *q;
}

static void deposit(const ora_ctx* c, const orun* r, size_t v, int batch, double amount)
{
    double* slot = &r->tally[v * (size_t)c->p.k_batches + batch];
#pragma omp atomic
    *slot += amount;
}

/* Dose-averaged LET (Sec. III, LET_d maps): a proton step that starts in
 * voxel v and deposits eps there adds w * eps * L to the numerator and
 * w * eps to the denominator, L being the stopping power of v's medium
 * averaged over the step's mean (CSDA) energy loss, in MeV/cm.  Deposits
 * that belong to no step (recoil nuclei, the local share of a non-elastic
 * event, secondaries below the cut-off, the sub-cut-off rest of a track) are
 * not scored. */
static void score_let(const orun* r, size_t v, double amount, double l_mev_cm)
{
    if (!r->let_num) return;
#pragma omp atomic
    r->let_num[v] += amount * l_mev_cm;
#pragma omp atomic
    r->let_den[v] += amount;
}

static int locate(const ora_ctx* c, const double p[3], const double d[3], int v[3])
{
    for (int a = 0; a < 3; ++a) {
        double f = floor(p[a]);
        if (!(f > -2.0 && f < (double)c->n[a] + 2.0)) return 0;
        int i = (int)f;
        if (p[a] == f && d[a] < 0.0) i -= 1;    /* on a face: the voxel being entered */
        if (i < 0 || i >= c->n[a]) return 0;
        v[a] = i;
    }
    return 1;
}

static size_t vindex(const ora_ctx* c, const int v[3])
{
    return ((size_t)v[2] * c->n[1] + v[1]) * c->n[0] + v[0];
}

static void log_escape(const ora_ctx* c, const orun* r, const opart* q)
{
    ora_diag* dg = r->diag;
    if (!dg || !dg->escape_log) return;
    uint64_t slot;
#pragma omp atomic capture
    slot = dg->escape_count++;
    if (slot >= dg->escape_cap) return;
    double* o = dg->escape_log + 8 * slot;
    for (int a = 0; a < 3; ++a) { o[a] = q->p[a] * c->vs[a]; o[3 + a] = q->d[a]; }
    o[6] = q->e; o[7] = q->w;
}

static void birth(const orun* r, opart* q)
{
    double u[4];
    draw4(r->seed, q->uid, 0, 0, u);
    q->mfp = -log(u[2]);
}

/* One nuclear event at the end of a step; returns 1 if the proton survives. */
static int interact(const ora_ctx* c, const orun* r, opart* q, const int v[3], uint32_t ks,
                    ostack* st, oacc* acc)
{
    size_t vi = vindex(c, v);
    const omat* m = &c->mat[c->vmat[vi]];
    double t = q->e;
    double part_el[ORA_NEL], part_ne[ORA_NEL];
    double s_el = sigma_per_g(c, m, 0, t, part_el);
    double s_ne = sigma_per_g(c, m, 1, t, part_ne);
    double u[4];
    draw4(r->seed, q->uid, ks, 3, u);
    if (!(s_el + s_ne > 0.0)) { q->mfp = -log(u[3]); return 1; }
    int elastic = u[0] * (s_el + s_ne) < s_el;
    const double* part = elastic ? part_el : part_ne;
    double target = u[1] * (elastic ? s_el : s_ne), cum = 0.0;
    int el = -1;
    for (int e = 0; e < ORA_NEL; ++e) {
        if (part[e] <= 0.0) continue;
        el = e;
        cum += part[e];
        if (target < cum) break;
    }
    if (r->diag && r->diag->first_nuclear_z_cm && q->primary &&
        isnan(r->diag->first_nuclear_z_cm[q->uid]))
        r->diag->first_nuclear_z_cm[q->uid] = q->p[2] * c->vs[2];
    acc->inter[elastic ? 0 : 1][el]++;
    double u4[4];
    draw4(r->seed, q->uid, ks, 4, u4);
    if (elastic) {
        acc->n_el++;
        double o[7];
        oracle_elastic_sample(EL_MASS_NUMBER[el], t, u[2], u4[0], o);
        double tn = o[2], tr = t - tn;
        if (el == 0 && tr > E_CUT) {          /* recoil proton is transported */
            opart ch = *q;
            ch.d[0] = q->d[0]; ch.d[1] = q->d[1]; ch.d[2] = q->d[2];
            oracle_rotate(ch.d, o[5], o[6], u4[1] + 0.5);
            ch.e = tr;
            ch.uid = child_uid(r->seed, q->uid, ks, 0);
            ch.k = 0;
            ch.primary = 0;
            birth(r, &ch);
            push(st, &ch);
            acc->secondaries++;
        } else {
            deposit(c, r, vi, q->batch, q->w * tr);   /* recoil nucleus: local */
        }
        oracle_rotate(q->d, o[3], o[4], u4[1]);
        q->e = tn;
        if (q->e <= E_CUT) {
            deposit(c, r, vi, q->batch, q->w * q->e);
            return 0;
        }
        q->mfp = -log(u[3]);
        return 1;
    }
    acc->n_ne++;
    if (c->p.flags & ORA_INC) {
        /* intranuclear cascade and evaporation (Sec. II.A.4): protons above
         * the cut-off are transported, neutrons dropped (neutral ledger, with
         * the separation energies and the excitation left for photons), the
         * kinetic energy of heavier fragments and of sub-cut-off protons
         * deposited here */
        ora_inc_result ir;
        oracle_inc_event(el, t, r->seed, q->uid, ks, 1, &ir);
        double local = 0.0, neutral = ir.binding + ir.e_star_fin;
        for (int i = 0; i < ir.n; ++i) {
            if (ir.kind[i] == ORA_EJ_N) { neutral += ir.t[i]; continue; }
            if (ir.kind[i] != ORA_EJ_P || ir.t[i] <= E_CUT) { local += ir.t[i]; continue; }
            opart ch = *q;
            const double* e = ir.dir[i];
            oracle_rotate(ch.d, e[2], sqrt(e[0] * e[0] + e[1] * e[1]), atan2(e[1], e[0]) / (2.0 * M_PI));
            ch.e = ir.t[i];
            ch.uid = child_uid(r->seed, q->uid, ks, ir.id[i]);
            ch.k = 0;
            ch.primary = 0;
            birth(r, &ch);
            push(st, &ch);
            acc->secondaries++;
        }
        deposit(c, r, vi, q->batch, q->w * local);
        acc->neutral += q->w * neutral;
        return 0;
    }
    int n;
    double es[4], mus[4], fl;
    oracle_secondary_sample(c, el, t, q->uid, ks, r->seed, u4[0], &n, es, mus, &fl);
    double local = fl * t, carried = 0.0;
    for (int j = 0; j < n; ++j) {
        carried += es[j];
        if (es[j] <= E_CUT) { local += es[j]; continue; }
        double uc[4];
        draw4(r->seed, q->uid, ks, 16u + (uint32_t)(j + 1), uc);
        opart ch = *q;
        oracle_rotate(ch.d, mus[j], sqrt(fmax(0.0, 1.0 - mus[j] * mus[j])), uc[2]);
        ch.e = es[j];
        ch.uid = child_uid(r->seed, q->uid, ks, (uint32_t)(j + 1));
        ch.k = 0;
        ch.primary = 0;
        birth(r, &ch);
        push(st, &ch);
        acc->secondaries++;
    }
    deposit(c, r, vi, q->batch, q->w * local);
    acc->neutral += q->w * (t - fl * t - carried);
    return 0;
}

static void transport(const ora_ctx* c, const orun* r, opart* q, ostack* st, oacc* acc)
{
    const uint32_t flags = c->p.flags;
    int v[3];
    if (!locate(c, q->p, q->d, v)) {
        acc->escaped += q->w * q->e;
        log_escape(c, r, q);
        return;
    }
    for (;;) {
        size_t vi = vindex(c, v);
        const int mi = c->vmat[vi];
        const omat* m = &c->mat[mi];
        const double rho = c->vrho[vi];
        const rtable* rt = table_of(c, mi);
        const double scale = m->own ? rho : rho * m->f;               /* Eq. 1-2 */
        const double range = rt_range(rt, q->e);
        const double s_range = range / scale;
        const double sig = (flags & ORA_NO_NUCLEAR) ? 0.0
            : rho * (sigma_per_g(c, m, 0, q->e, NULL) + sigma_per_g(c, m, 1, q->e, NULL));
        const double s_nuc = sig > 0.0 ? q->mfp / sig : INFINITY;
        double d = INFINITY;
        int axis = -1;
        for (int a = 0; a < 3; ++a) {
            double da;
            if (q->d[a] > 0.0) da = (v[a] + 1 - q->p[a]) * c->vs[a] / q->d[a];
            else if (q->d[a] < 0.0) da = (v[a] - q->p[a]) * c->vs[a] / q->d[a];
            else continue;
            if (da < d) { d = da; axis = a; }
        }
        /* range-limited step: the proton stops in this voxel; its stopping
         * power averaged over the residual range (R(E_CUT) = 0) */
        if (s_range <= d && s_range <= s_nuc) {
            deposit(c, r, vi, q->batch, q->w * q->e);
            score_let(r, vi, q->w * q->e, (q->e - E_CUT) / s_range);
            return;
        }
        const int lim = (s_nuc < d) ? LIM_NUC : LIM_BND;
        double s = (lim == LIM_NUC) ? s_nuc : d;
        const int short_step = s < c->p.s_min_cm;
        if (short_step) s = c->p.s_min_cm;
        if (s >= s_range) {
            deposit(c, r, vi, q->batch, q->w * q->e);
            score_let(r, vi, q->w * q->e, (q->e - E_CUT) / s_range);
            return;
        }
        /* mean loss from the range table, Eq. 2 water-equivalent path */
        const double e1 = rt_energy(rt, range - s * scale);
        const double de_mean = q->e - e1;
        const double e_mid = q->e - 0.5 * de_mean;
        double u[4];
        const uint32_t ks = q->k;
        draw4(r->seed, q->uid, ks, 1, u);
        double de = de_mean;
        if (!(flags & ORA_NO_STRAGGLE)) {
            double var = oracle_straggling_variance(e_mid, s, rho, m->za);
            double z = oracle_normal_quantile(u[3]);
            if (flags & ORA_VAVILOV) {
                /* Vavilov-Gaussian: the normal score mapped through the
                 * Vavilov quantile function of the step's (kappa, beta^2) */
                const double e_tot = e_mid + M_PROTON;
                const double b2 = e_mid * (e_mid + 2.0 * M_PROTON) / (e_tot * e_tot);
                z = vav_quantile(c->vav, oracle_vavilov_kappa(e_mid, s, rho, m->za), b2, z);
            }
            de = de_mean + sqrt(var) * z;
            if (de < 0.0) de = 0.0;
            if (de > q->e) de = q->e;
        }
        double theta = 0.0;
        if (!(flags & ORA_NO_MCS))
        {
            double chi_c2, B;
            if ((flags & ORA_MOLIERE) && mol_step(m, e_mid, rho, s, &chi_c2, &B))
                theta = mol_theta(c->mol, chi_c2, B, u[1]);
            else
                theta = oracle_highland_theta0(e_mid, s, m->x0 / rho, c->p.f_mcs) * sqrt(-2.0 * log(u[1]));
        }
        /* random hinge: deflect at a uniform fraction u0 of the step.  On a
         * boundary-limited step the remaining segment runs along the new
         * direction to the crossed face plane and ends exactly on it, unless
         * the deflection turned the proton back or that segment would exceed
         * twice its nominal length. */
        for (int a = 0; a < 3; ++a) q->p[a] += u[0] * s * q->d[a] / c->vs[a];
        const double d_axis_before = q->d[axis];
        if (theta != 0.0) oracle_rotate(q->d, cos(theta), sin(theta), u[2]);
        double rest = (1.0 - u[0]) * s;
        int on_face = 0;
        const double face = (d_axis_before > 0.0) ? (double)(v[axis] + 1) : (double)v[axis];
        if (lim == LIM_BND && !(flags & ORA_PLAIN_HINGE) && q->d[axis] * d_axis_before > 0.0) {
            const double l2 = (face - q->p[axis]) * c->vs[axis] / q->d[axis];
            if (l2 >= 0.0 && l2 <= 2.0 * rest) {
                rest = l2;
                on_face = 1;
            }
        }
        for (int a = 0; a < 3; ++a) q->p[a] += rest * q->d[a] / c->vs[a];
        if (on_face) q->p[axis] = face;
        const double e_new = q->e - de;
        deposit(c, r, vi, q->batch, q->w * (q->e - e_new));
        score_let(r, vi, q->w * (q->e - e_new), de_mean / s);
        q->mfp = (lim == LIM_NUC) ? 0.0 : fmax(q->mfp - sig * s, 0.0);
        q->e = e_new;
        q->k = ks + 1;
        acc->steps++;
        acc->n_short += short_step;
        if (q->e <= E_CUT) {
            deposit(c, r, vi, q->batch, q->w * q->e);
            return;
        }
        if (!locate(c, q->p, q->d, v)) {
            acc->escaped += q->w * q->e;
            log_escape(c, r, q);
            return;
        }
        if (lim == LIM_NUC && !interact(c, r, q, v, ks, st, acc)) return;
    }
}

/* ======================================================================
 * Runs: spot allocation, source (Gaussian spots on the z = 0 face),
 * 10 statistical groups and dose statistics (Sec. II.B.2)
 * ====================================================================== */
typedef struct { double rem; int idx; } remk;

static int cmp_rem(const void* a, const void* b)
{
    const remk* x = (const remk*)a;
    const remk* y = (const remk*)b;
    if (x->rem > y->rem) return -1;
    if (x->rem < y->rem) return 1;
    return x->idx - y->idx;
}

static int run_impl(ora_ctx* c, const ora_spot* spots, int n_spots, uint64_t n_hist,
                    uint64_t seed, double* dose, double* var, double* let, ora_summary* sum,
                    ora_diag* diag)
{
    if (!c || !dose || !var || !sum) return -1;
    if (!c->have_physics || !c->have_geometry) return -6;
    if (n_hist > 0 && (n_spots <= 0 || !spots)) return -1;
    const int K = c->p.k_batches;
    double wsum = 0.0;
    for (int s = 0; s < n_spots; ++s) {
        if (!(spots[s].e_mev > E_CUT && spots[s].e_mev <= GRID_EMAX)) return -2;
        if (!(spots[s].weight >= 0.0) || !(spots[s].sigma_x_cm >= 0.0) || !(spots[s].sigma_y_cm >= 0.0)) return -2;
        wsum += spots[s].weight;
    }
    if (n_hist > 0 && !(wsum > 0.0)) return -2;
    memset(sum, 0, sizeof(*sum));
    double t0 = 0.0;
#ifdef _OPENMP
    t0 = omp_get_wtime();
#endif
    /* histories per spot by largest remainder, proportional to weight */
    uint64_t* ns = (uint64_t*)calloc(n_spots > 0 ? n_spots : 1, sizeof(uint64_t));
    uint64_t* start = (uint64_t*)calloc((n_spots > 0 ? n_spots : 1) + 1, sizeof(uint64_t));
    double* omega = (double*)calloc(n_spots > 0 ? n_spots : 1, sizeof(double));
    remk* rk = (remk*)calloc(n_spots > 0 ? n_spots : 1, sizeof(remk));
    double* tally = (double*)calloc(c->nvox * (size_t)K, sizeof(double));
    double* let_nd = let ? (double*)calloc(2 * c->nvox, sizeof(double)) : NULL;
    if (!ns || !start || !omega || !rk || !tally || (let && !let_nd)) {
        free(ns); free(start); free(omega); free(rk); free(tally); free(let_nd);
        return -3;
    }
    if (n_hist > 0) {
        uint64_t assigned = 0;
        for (int s = 0; s < n_spots; ++s) {
            double q = (double)n_hist * spots[s].weight / wsum;
            ns[s] = (uint64_t)floor(q);
            rk[s].rem = q - floor(q);
            rk[s].idx = s;
            assigned += ns[s];
        }
        qsort(rk, n_spots, sizeof(remk), cmp_rem);
        for (uint64_t i = 0; assigned + i < n_hist; ++i) ns[rk[i % n_spots].idx]++;
    }
    double wtot = 0.0;
    for (int s = 0; s < n_spots; ++s) {
        start[s + 1] = start[s] + ns[s];
        omega[s] = ns[s] ? (spots[s].weight / wsum) * (double)n_hist / (double)ns[s] : 0.0;
        wtot += (double)ns[s] * omega[s];
    }
    uint64_t h0 = 0, h1 = n_hist;
    if (diag && diag->uid_end > 0) {
        h0 = diag->uid_begin;
        h1 = diag->uid_end < n_hist ? diag->uid_end : n_hist;
    }
    if (diag) diag->escape_count = 0;
    if (diag && diag->first_nuclear_z_cm)
        for (uint64_t h = 0; h < n_hist; ++h) diag->first_nuclear_z_cm[h] = NAN;
    orun run = {seed, tally, diag, let_nd, let_nd ? let_nd + c->nvox : NULL};
    double incident = 0.0, escaped = 0.0, neutral = 0.0;
    uint64_t steps = 0, secs = 0, nel = 0, nne = 0, nshort = 0, inter[2][ORA_NEL];
    memset(inter, 0, sizeof(inter));
    int nthreads = 1;
#pragma omp parallel num_threads(c->p.n_threads > 0 ? c->p.n_threads : omp_get_max_threads()) \
    reduction(+ : incident, escaped, neutral, steps, secs, nel, nne, nshort)
    {
#ifdef _OPENMP
#pragma omp single
        nthreads = omp_get_num_threads();
#endif
        ostack st = {NULL, 0, 0};
        oacc acc;
        memset(&acc, 0, sizeof(acc));
#pragma omp for schedule(dynamic, 64)
        for (int64_t hh = (int64_t)h0; hh < (int64_t)h1; ++hh) {
            uint64_t h = (uint64_t)hh;
            int lo = 0, hi = n_spots;               /* spot s with start[s] <= h < start[s+1] */
            while (hi - lo > 1) {
                int mid = (lo + hi) / 2;
                if (start[mid] <= h) lo = mid; else hi = mid;
            }
            const int s = lo;
            const ora_spot* sp = &spots[s];
            opart q;
            double u[4];
            draw4(seed, h, 0, 0, u);
            double rr = sqrt(-2.0 * log(u[0]));
            double x = sp->x_cm + sp->sigma_x_cm * rr * cos(2.0 * M_PI * u[1]);
            double y = sp->y_cm + sp->sigma_y_cm * rr * sin(2.0 * M_PI * u[1]);
            q.p[0] = x / c->vs[0];
            q.p[1] = y / c->vs[1];
            q.p[2] = 0.0;
            q.d[0] = 0.0; q.d[1] = 0.0; q.d[2] = 1.0;
            q.e = sp->e_mev;
            q.w = omega[s];
            q.mfp = -log(u[2]);
            q.uid = h;
            q.k = 0;
            q.batch = (int)((h - start[s]) * (uint64_t)K / ns[s]);
            q.primary = 1;
            incident += q.w * q.e;
            push(&st, &q);
            while (st.n) {
                opart cur = st.a[--st.n];
                transport(c, &run, &cur, &st, &acc);
            }
        }
        free(st.a);
        escaped += acc.escaped;
        neutral += acc.neutral;
        steps += acc.steps;
        secs += acc.secondaries;
        nel += acc.n_el;
        nne += acc.n_ne;
        nshort += acc.n_short;
#pragma omp critical
        for (int a = 0; a < 2; ++a)
            for (int e = 0; e < ORA_NEL; ++e) inter[a][e] += acc.inter[a][e];
    }
    /* dose statistics: total and variance of the total from K groups */
    const double vol = c->vs[0] * c->vs[1] * c->vs[2];
    double deposited = 0.0;
    for (size_t v = 0; v < c->nvox; ++v) {
        const double* tb = &tally[v * K];
        double tot = 0.0;
        for (int b = 0; b < K; ++b) tot += tb[b];
        double ss = 0.0;
        for (int b = 0; b < K; ++b) {
            double dd = tb[b] - tot / K;
            ss += dd * dd;
        }
        double conv = (wtot > 0.0) ? MEV_PER_GY_FACTOR / (c->vrho[v] * vol * wtot) : 0.0;
        dose[v] = tot * conv;
        var[v] = (double)K / (K - 1) * ss * conv * conv;
        deposited += tot;
    }
    /* LET_d in keV/um (1 MeV/cm = 0.1 keV/um); 0 where no step deposited */
    if (let)
        for (size_t v = 0; v < c->nvox; ++v) {
            const double num = let_nd[v], den = let_nd[c->nvox + v];
            let[v] = (den > 0.0) ? 0.1 * num / den : 0.0;
        }
    if (diag && diag->batch_tally) memcpy(diag->batch_tally, tally, sizeof(double) * c->nvox * K);
    sum->incident = incident;
    sum->deposited = deposited;
    sum->escaped = escaped;
    sum->neutral = neutral;
    sum->histories = h1 > h0 ? h1 - h0 : 0;
    sum->steps = steps;
    sum->secondaries = secs;
    sum->n_elastic = nel;
    sum->n_nonelastic = nne;
    memcpy(sum->interactions, inter, sizeof(inter));
    sum->total_weight = wtot;
    sum->n_short_steps = nshort;
    sum->threads = nthreads;
#ifdef _OPENMP
    sum->wall_s = omp_get_wtime() - t0;
#endif
    free(ns); free(start); free(omega); free(rk); free(tally); free(let_nd);
    return 0;
}

int oracle_run_spots(ora_ctx* c, const ora_spot* spots, int n_spots, uint64_t n_hist,
                     uint64_t seed, double* dose, double* var, ora_summary* sum, ora_diag* diag)
{
    return run_impl(c, spots, n_spots, n_hist, seed, dose, var, NULL, sum, diag);
}

int oracle_run_spots_let(ora_ctx* c, const ora_spot* spots, int n_spots, uint64_t n_hist,
                         uint64_t seed, double* dose, double* var, double* let_kev_um,
                         ora_summary* sum, ora_diag* diag)
{
    if (!let_kev_um) return -1;
    return run_impl(c, spots, n_spots, n_hist, seed, dose, var, let_kev_um, sum, diag);
}
