/*
 * pmc_oracle.h - plain double-precision CPU reference of condensed-history
 * proton transport with dose scoring, after Wan Chan Tseung, Ma & Beltran,
 * "A fast GPU-based Monte Carlo simulation of proton transport with detailed
 * modeling of non-elastic interactions" (arXiv:1409.8336), Sec. II.A-II.B.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP engine) never calls it and shares no code with it.
 *
 * Conventions (identical to the engine's public interface, restated here):
 *   - HU grid, dose and variance are [nz][ny][nx], x fastest.
 *   - The grid occupies [0,nx*dx) x [0,ny*dy) x [0,nz*dz) cm; spots start on
 *     the z = 0 face travelling along +z.
 *   - Element order everywhere: H, C, N, O, P, Ca, Ti.
 *   - Tabulated cross sections live on E_i = 0.1*2500^(i/999) MeV, i<1000,
 *     and are interpolated linearly in ln E.
 * All functions return 0 on success and a negative code on error.
 */
#ifndef PMC_ORACLE_H
#define PMC_ORACLE_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define ORA_NEL 7
#define ORA_NE 1000
#define ORA_SEC_NUCLEI 6
#define ORA_SEC_EBINS 25
#define ORA_SEC_MULT 5
#define ORA_SEC_NCDF 32

/* ORA_VAVILOV: Vavilov-Gaussian straggling instead of Gaussian (Sec. II.A.2) */
/* ORA_MOLIERE: Molière multiple scattering instead of the scaled Highland
   Gaussian where B >= 4.5 (Sec. II.A.2) */
/* ORA_PLAIN_HINGE (test only): the second hinge segment always keeps its
   nominal length (1 - u) s, without the landing on the crossed face plane;
   used to measure what that landing changes */
/* ORA_INC: non-elastic events by the intranuclear cascade and evaporation
   below (Sec. II.A.4) instead of the synthetic secondary table */
enum { ORA_NO_STRAGGLE = 1, ORA_NO_MCS = 2, ORA_NO_NUCLEAR = 4, ORA_VAVILOV = 8, ORA_MOLIERE = 16,
       ORA_PLAIN_HINGE = 32, ORA_INC = 64 };

/* Molière sampling table: [1/B = 1/20 + j (2/9 - 1/20)/12, j < 13][q = k/8, k < 161]
   of ln(v^2 / q), v the reduced angle, q = -ln u */
#define ORA_MOL_NX 13
#define ORA_MOL_NQ 161

/* Vavilov quantile table: [beta^2 = k/10, k < 5][log10 kappa = -2 + j/10, j < 31]
   [z = -6 + i/8, i < 97] */
#define ORA_VAV_NB 5
#define ORA_VAV_NK 31
#define ORA_VAV_NZ 97

typedef struct {
    double f_mcs;        /* Highland multiplier (1.07, Sec. II.A.2) */
    double s_min_cm;     /* shortest non-range-limited step (1e-4 cm) */
    int32_t k_batches;   /* statistical groups (10, Sec. II.B.2) */
    uint32_t flags;      /* ORA_NO_* switches for the closed-form pins */
    int32_t n_threads;   /* OpenMP threads, 0 = runtime default */
} ora_params;

typedef struct {
    int32_t n_bins;
    const int16_t* hu_lo;
    const float* rho_lo;
    const float* rho_hi;
    const float* mass_frac;  /* n_bins x 7 */
    const float* i_ev;
    const int32_t* own_table;
} ora_material_table;

typedef struct {
    const float* sigma_ne;   /* 7 x 1000 barn */
    const float* sigma_el;   /* 7 x 1000 barn */
    const float* mult_cdf;   /* 6 x 25 x 5 */
    const float* f_local;    /* 6 x 25 */
    const float* x_cdf;      /* 6 x 25 x 33 */
    const float* mu_cdf;     /* 6 x 25 x 33 */
} ora_nuclear_data;

typedef struct {
    float x_cm, y_cm, e_mev, sigma_x_cm, sigma_y_cm, weight;
} ora_spot;

typedef struct {
    double incident, deposited, escaped, neutral;   /* weighted MeV */
    uint64_t histories, steps, secondaries, n_elastic, n_nonelastic;
    uint64_t interactions[2][ORA_NEL];              /* [elastic, non-elastic][element] */
    double total_weight;
    double wall_s;
    int32_t threads;
    uint64_t n_short_steps;                         /* steps lengthened to s_min */
} ora_summary;

/* Optional diagnostics; any pointer may be NULL. */
typedef struct {
    uint64_t uid_begin, uid_end;   /* simulate only these primaries (end 0 = all) */
    double* batch_tally;           /* nvox x K raw weighted MeV */
    double* first_nuclear_z_cm;    /* per primary uid: depth of its first nuclear event, NaN if none */
    double* escape_log;            /* cap x 8: x,y,z (cm), u,v,w, E, weight */
    uint64_t escape_cap;
    uint64_t escape_count;         /* out */
} ora_diag;

typedef struct ora_ctx ora_ctx;

int oracle_create(ora_ctx** out, const ora_params* p);
int oracle_destroy(ora_ctx* c);
int oracle_load_physics(ora_ctx* c, const ora_nuclear_data* nd);
int oracle_load_geometry(ora_ctx* c, const int16_t* hu, int nx, int ny, int nz,
                         float dx, float dy, float dz, const ora_material_table* mt);
int oracle_run_spots(ora_ctx* c, const ora_spot* spots, int n_spots, uint64_t n_histories,
                     uint64_t seed, double* dose_gy, double* var_gy2, ora_summary* s,
                     ora_diag* diag);
/* As oracle_run_spots, and the dose-averaged LET of every voxel (Sec. III,
 * LET_d maps) in keV/um into let_kev_um (nx*ny*nz doubles):
 * sum(w eps L) / sum(w eps) over the proton steps that start in the voxel,
 * eps the step's deposit and L the stopping power of the voxel's medium
 * averaged over the step's mean energy loss (a range-limited step: over the
 * residual range).  Local deposits of nuclear events and the sub-cut-off rest
 * of a track are not scored.  0 where no step deposited. */
int oracle_run_spots_let(ora_ctx* c, const ora_spot* spots, int n_spots, uint64_t n_histories,
                         uint64_t seed, double* dose_gy, double* var_gy2, double* let_kev_um,
                         ora_summary* s, ora_diag* diag);

/* ---- individual pieces, exported for the closed-form pins ---- */
void oracle_philox4x32_10(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4]);
double oracle_u01(uint32_t x);
double oracle_normal_quantile(double u);
double oracle_bethe_bloch(double t_mev, double z_over_a, double i_ev);
double oracle_stopping_power(double t_mev, double z_over_a, double i_ev);
double oracle_bb_peak_energy(double z_over_a, double i_ev);
double oracle_radiation_length(const double w[ORA_NEL]);
double oracle_water_z_over_a(void);
/* table 0 = water; table m+1 = own table of material bin m */
double oracle_range(const ora_ctx* c, int table, double t_mev);
double oracle_energy_at_range(const ora_ctx* c, int table, double r);
int oracle_material_info(const ora_ctx* c, int m, double out[6]); /* za, I, f, X0 g/cm2, own, n/rho total */
double oracle_highland_theta0(double t_mev, double s_cm, double x0_cm, double f);
double oracle_straggling_variance(double t_mev, double s_cm, double rho, double za);
double oracle_sigma(const ora_ctx* c, int process, int element, double t_mev);
/* Ranft elastic (A>=2) or isotropic p-p (A==1) at kinetic energy T:
   out = {|t| MeV^2, recoil kinetic energy, scattered kinetic energy,
          cos theta_lab, sin theta_lab, cos recoil, sin recoil} */
int oracle_elastic_sample(int mass_number, double t_mev, double u_comp, double u_t, double out[7]);
/* Non-elastic secondaries on nucleus element index e (1..6) at T.
   Writes n (<=4) energies, cosines and the local fraction. */
int oracle_secondary_sample(const ora_ctx* c, int element, double t_mev, uint64_t uid,
                            uint32_t k, uint64_t seed, double u_mult, int* n_out,
                            double e_out[4], double mu_out[4], double* f_local);
void oracle_rotate(double dir[3], double cos_t, double sin_t, double phi_rev);
/* Vavilov straggling: distribution function of X = (Delta - <Delta>)/T_max
   (Gil-Pelaez inversion of the characteristic function), the quantile
   nodes of W = X / sqrt(kappa (1 - beta^2/2)) at the table's grid
   (out: 5 x 31 x 97), the step's kappa = xi / T_max, and the trilinear
   quantile the transport draws with (context created with ORA_VAVILOV). */
double oracle_vavilov_cdf(double kappa, double beta2, double x);
int oracle_vavilov_table(double* out);
double oracle_vavilov_kappa(double t_mev, double s_cm, double rho, double za);
double oracle_vavilov_quantile(const ora_ctx* c, double kappa, double beta2, double z);
/* Molière: Bethe's f0, f1, f2 at reduced angle v (n = 0, 1, 2), the
   survival P(V > v) at 1/B = x, the sampling table (out: 13 x 161), and the
   transport's polar angle for material bin m at kinetic energy t, density
   rho, step s and uniform u (context created with ORA_MOLIERE; NaN and
   *b_out = 0 where B < 4.5, i.e. the step keeps Highland) */
double oracle_moliere_f(int n, double v);
double oracle_moliere_survival(double x, double v);
int oracle_moliere_table(double* out);
double oracle_moliere_theta(const ora_ctx* c, int material, double t_mev, double rho, double s_cm,
                            double u, double* b_out);

/* ---- Intranuclear cascade and evaporation (Sec. II.A.4), test pieces ----
 * Targets: element index 1..6 = C-12, N-14, O-16, P-31, Ca-40, Ti-48. */
#define ORA_INC_SHELLS 15
#define ORA_INC_MAX_OUT 96
enum { ORA_EJ_N = 0, ORA_EJ_P = 1, ORA_EJ_D = 2, ORA_EJ_T = 3, ORA_EJ_HE3 = 4, ORA_EJ_ALPHA = 5 };

typedef struct {
    int32_t z, a;
    double radius_ws, diffuseness, r_out;        /* fm */
    double r[ORA_INC_SHELLS + 1];                /* shell boundaries, fm */
    double rho_p[ORA_INC_SHELLS], rho_n[ORA_INC_SHELLS];   /* fm^-3 */
    double tf_p[ORA_INC_SHELLS], tf_n[ORA_INC_SHELLS];     /* Fermi kinetic energies, MeV */
} ora_nucleus;

typedef struct {
    int32_t n;                                   /* emitted particles */
    int32_t kind[ORA_INC_MAX_OUT];               /* ORA_EJ_* */
    int32_t stage[ORA_INC_MAX_OUT];              /* 0 cascade, 1 evaporation */
    uint32_t id[ORA_INC_MAX_OUT];                /* child id (uid draw tag 0xC0000000 | id) */
    double t[ORA_INC_MAX_OUT];                   /* kinetic energy, MeV */
    double dir[ORA_INC_MAX_OUT][3];              /* direction, incident proton along +z */
    int32_t z_res, a_res;                        /* residual after the cascade */
    double e_star;                               /* its excitation (from the energy balance) */
    double e_star_sum;                           /* the same from the holes and trapped particles */
    int32_t n_coll, n_blocked, attempts, n_esc;  /* allowed / Pauli-blocked collisions, entries */
    int32_t compound;                            /* no allowed collision in 64 entries: absorbed */
    int32_t z_fin, a_fin;                        /* after evaporation */
    double e_star_fin;                           /* excitation left (photons, not followed) */
    double binding;                              /* (n_esc - 1) S + sum of evaporation separation energies */
    double pauli_min;                            /* least (product kinetic energy - its Fermi energy)
                                                    over the allowed collisions (INFINITY if none) */
} ora_inc_result;

int oracle_inc_nucleus(int element, ora_nucleus* out);
double oracle_nn_sigma_mb(int same_species, double t_lab_mev);
double oracle_nn_slope(double p_lab_gev);
/* One non-elastic event of a proton of t_mev on element (1..6), random
   stream (seed, uid, ks); evaporate = 0 stops after the cascade. */
int oracle_inc_event(int element, double t_mev, uint64_t seed, uint64_t uid, uint32_t ks, int evaporate,
                     ora_inc_result* out);
/* Evaporation of a nucleus (z, a, e_star) alone, emissions numbered from 0. */
int oracle_evaporate(int z, int a, double e_star, uint64_t seed, uint64_t uid, uint32_t ks, ora_inc_result* out);
double oracle_binding_energy(int z, int a);      /* MeV; -INFINITY where unbound */
/* the cascade's sub-steps, as it calls them: a Fermi-sea partner momentum
   (MeV/c) in shell k from uniforms u[0] (magnitude), u[1] (cos theta),
   u[2] (azimuth); the crossing of a spherical shell boundary (returns 1 if
   crossed, 0 if reflected; t and d updated); an elastic NN collision */
void oracle_fermi_momentum(double p_fermi, const double u[3], double p[3]);
int oracle_inc_refract(double t, double v_from, double v_to, const double x[3], double d[3], double* t_out);
void oracle_nn_collide(const double p1[3], const double p2[3], double u_t, double u_phi, double o1[3], double o2[3]);
/* Relative emission width of ejectile kind from (z, a, e_star) by quadrature,
   and its separation energy and Coulomb barrier. */
double oracle_evap_width(int z, int a, double e_star, int kind, double* sep, double* barrier);

#ifdef __cplusplus
}
#endif
#endif
