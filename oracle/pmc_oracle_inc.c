/*
 * pmc_oracle_inc.c - plain double-precision reference of the non-elastic
 * proton-nucleus model of Wan Chan Tseung, Ma & Beltran (arXiv:1409.8336),
 * Sec. II.A.4: a Bertini-style intranuclear cascade (INC) followed by
 * evaporation of the excited residual nucleus.
 *
 * TEST INFRASTRUCTURE ONLY (see pmc_oracle.h): never called by the product
 * path, shares no code with the HIP engine.
 *
 * What the paper fixes, in its order:
 *   - the target is picked by the relative non-elastic cross sections (done
 *     by the transport), a random entry point is chosen and the proton is
 *     propagated through nuclear matter, repeated until the cascade has at
 *     least one Pauli-allowed nucleon-nucleon collision;
 *   - the nucleus is a two-component Fermi gas of neutrons and protons whose
 *     density follows a Woods-Saxon form approximated by 15 constant-density
 *     shells;
 *   - the incident proton and every collision product are followed until
 *     they leave the nucleus or are trapped; reflection and refraction at the
 *     shell boundaries;
 *   - Pauli blocking: every collision product's kinetic energy must exceed
 *     its Fermi energy;
 *   - below 250 MeV only elastic nucleon-nucleon collisions;
 *   - the residual nucleus de-excites by particle evaporation (GEM in the
 *     paper), isotropic in its rest frame; no photon evaporation,
 *     pre-equilibrium, fission or Fermi break-up;
 *   - only protons are transported further; neutrons are dropped; the
 *     kinetic energy of heavier charged particles is deposited locally.
 * Where the paper is silent or names models whose parameters are not
 * available here (Cugnon's NN cross sections, GEM's level densities and
 * inverse cross sections), the readings are stated at each function; the
 * HIP engine implements the same readings.
 *
 * Random numbers follow the transport's draw contract: Philox4x32-10 blocks
 * keyed by the run seed with counter (uid, ks, tag), the event at step ks of
 * history uid.  Cascade particle j's m-th block in entry attempt e uses tag
 * 0x40000000 | e << 20 | j << 12 | m; evaporation emission i uses tag
 * 0x50000000 | i << 8 | r (r = 0 channel and direction, r >= 1 energy
 * attempts).  So a particle's draws do not depend on the order in which the
 * cascade is processed.
 */
#include "pmc_oracle.h"

#include <math.h>
#include <string.h>

#define HBARC 197.3269804        /* MeV fm */
#define M_NUCLEON 938.918754     /* one nucleon mass inside the cascade (p and n averaged), MeV */
#define S_SEP 7.0                /* separation energy of a nucleon from the Fermi surface, MeV */
#define WS_DIFFUSE 0.55          /* Woods-Saxon diffuseness, fm */
#define E2_MEVFM 1.439964548     /* e^2 / (4 pi eps0), MeV fm */
#define MAX_ATTEMPTS 64
#define MAX_PARTICLES 64
#define MAX_FLIGHTS 4096
#define MAX_REFLECT 32

static const int INC_Z[7] = {1, 6, 7, 8, 15, 20, 22};
static const int INC_A[7] = {1, 12, 14, 16, 31, 40, 48};

static void draw(uint64_t seed, uint64_t uid, uint32_t ks, uint32_t tag, double u[4])
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint32_t ctr[4] = {(uint32_t)uid, (uint32_t)(uid >> 32), ks, tag};
    uint32_t o[4];
    oracle_philox4x32_10(key, ctr, o);
    for (int i = 0; i < 4; ++i) u[i] = oracle_u01(o[i]);
}

/* ======================================================================
 * The nucleus: Woods-Saxon density rho(r) = rho0 / (1 + exp((r - R)/a)),
 * R = 1.16 A^(1/3) (1 - 1.16 A^(-2/3)) fm, a = 0.55 fm (readings), cut at
 * R + 5a and split into 15 shells of equal thickness, each with the
 * Woods-Saxon average density over its volume; rho0 normalises the shells to
 * A nucleons.  Protons carry Z/A of each shell's density, neutrons N/A.
 * Per shell and species: Fermi momentum (3 pi^2 rho)^(1/3) hbar c, Fermi
 * kinetic energy, and a well depth of Fermi energy + S (S = 7 MeV), so that
 * the Fermi surface lies S below the continuum everywhere.
 * ====================================================================== */
static double ws(double r, double R, double a) { return 1.0 / (1.0 + exp((r - R) / a)); }

int oracle_inc_nucleus(int element, ora_nucleus* nu)
{
    if (!nu || element < 1 || element > 6) return -1;
    memset(nu, 0, sizeof(*nu));
    const int Z = INC_Z[element], A = INC_A[element];
    const double a3 = cbrt((double)A);
    nu->z = Z;
    nu->a = A;
    nu->radius_ws = 1.16 * a3 * (1.0 - 1.16 / (a3 * a3));
    nu->diffuseness = WS_DIFFUSE;
    nu->r_out = nu->radius_ws + 5.0 * WS_DIFFUSE;
    double count[ORA_INC_SHELLS], vol[ORA_INC_SHELLS], total = 0.0;
    for (int k = 0; k <= ORA_INC_SHELLS; ++k) nu->r[k] = nu->r_out * k / ORA_INC_SHELLS;
    for (int k = 0; k < ORA_INC_SHELLS; ++k) {
        /* Simpson's rule for the nucleons of the shell (unnormalised) */
        const int n = 400;
        const double lo = nu->r[k], hi = nu->r[k + 1], h = (hi - lo) / n;
        double s = 0.0;
        for (int i = 0; i <= n; ++i) {
            const double r = lo + i * h;
            const double f = 4.0 * M_PI * r * r * ws(r, nu->radius_ws, WS_DIFFUSE);
            s += f * (i == 0 || i == n ? 1.0 : (i % 2 ? 4.0 : 2.0));
        }
        count[k] = s * h / 3.0;
        vol[k] = 4.0 / 3.0 * M_PI * (hi * hi * hi - lo * lo * lo);
        total += count[k];
    }
    for (int k = 0; k < ORA_INC_SHELLS; ++k) {
        const double rho = A * count[k] / total / vol[k];
        nu->rho_p[k] = rho * Z / A;
        nu->rho_n[k] = rho * (A - Z) / A;
        const double pp = HBARC * cbrt(3.0 * M_PI * M_PI * nu->rho_p[k]);
        const double pn = HBARC * cbrt(3.0 * M_PI * M_PI * nu->rho_n[k]);
        nu->tf_p[k] = sqrt(pp * pp + M_NUCLEON * M_NUCLEON) - M_NUCLEON;
        nu->tf_n[k] = sqrt(pn * pn + M_NUCLEON * M_NUCLEON) - M_NUCLEON;
    }
    return 0;
}

/* ======================================================================
 * Free elastic nucleon-nucleon cross sections and angular slope.  The paper
 * uses Cugnon et al.'s parameterisation, which is not available here; the
 * stand-ins below keep the shape of the measured free cross sections below
 * 250 MeV (pp flat near 23 mb above 150 MeV and rising steeply at low
 * energy; np about twice pp): sigma_pp = 22 + 1000/T mb, sigma_np = 30 +
 * 3000/T mb, T the lab kinetic energy on a nucleon at rest (>= 1 MeV).  The
 * CM angle follows dsigma/dt ~ exp(B t), B = 5.5 p^8 / (7.7 + p^8)
 * (GeV/c)^-2, p the lab momentum in GeV/c (Cugnon's form of the slope;
 * nearly isotropic at these energies); np pairs are symmetric about 90
 * degrees (identities exchanged with probability 1/2).
 * ====================================================================== */
double oracle_nn_sigma_mb(int same_species, double t)
{
    const double tt = t > 1.0 ? t : 1.0;
    return same_species ? 22.0 + 1000.0 / tt : 30.0 + 3000.0 / tt;
}

double oracle_nn_slope(double p)
{
    const double p8 = pow(p, 8.0);
    return 5.5 * p8 / (7.7 + p8);
}

/* a partner nucleon of the Fermi sea: |p| uniform in p^3 up to the Fermi
 * momentum (a full sphere in momentum space), direction isotropic */
void oracle_fermi_momentum(double p_fermi, const double u[3], double p[3])
{
    const double pm = p_fermi * cbrt(u[0]);
    const double ct = 2.0 * u[1] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
    p[0] = pm * st * cos(2.0 * M_PI * u[2]);
    p[1] = pm * st * sin(2.0 * M_PI * u[2]);
    p[2] = pm * ct;
}

/* ---- the cascade ---- */
typedef struct {
    int species;        /* 0 neutron, 1 proton */
    int shell;          /* 0..14 */
    int index;          /* particle index (draw stream) */
    int m;              /* next draw block of its stream */
    int reflections;
    double x[3];        /* position, fm */
    double d[3];        /* direction */
    double t;           /* kinetic energy above the local well bottom, MeV */
} cpart;

static double well(const ora_nucleus* nu, int species, int k)
{
    return (species ? nu->tf_p[k] : nu->tf_n[k]) + S_SEP;
}

static double fermi(const ora_nucleus* nu, int species, int k)
{
    return species ? nu->tf_p[k] : nu->tf_n[k];
}

/* distance along d from x to the sphere of radius r (the nearest positive
 * root), or INFINITY */
static double to_sphere(const double x[3], const double d[3], double r, int outward)
{
    const double b = x[0] * d[0] + x[1] * d[1] + x[2] * d[2];
    const double c = x[0] * x[0] + x[1] * x[1] + x[2] * x[2] - r * r;
    const double disc = b * b - c;
    if (disc < 0.0) return INFINITY;
    const double q = sqrt(disc);
    if (outward) {
        const double s = -b + q;
        return s > 0.0 ? s : 0.0;
    }
    const double s = -b - q;
    return s > 0.0 ? s : INFINITY;
}

/* crossing from shell k into shell j (j = 15: outside) at the surface point
 * x: total energy conserved, the momentum component along the surface
 * normal changes, the tangential one is kept; total reflection when the new
 * kinetic energy cannot carry the tangential momentum.  Returns 1 if the
 * particle crossed. */
int oracle_inc_refract(double t, double v_from, double v_to, const double x[3], double d[3], double* t_out)
{
    const double rr = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double n[3] = {x[0] / rr, x[1] / rr, x[2] / rr};
    const double p = sqrt(t * (t + 2.0 * M_NUCLEON));
    const double dn = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
    double pt[3];
    for (int a = 0; a < 3; ++a) pt[a] = p * (d[a] - dn * n[a]);
    const double pt2 = pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2];
    const double t2 = t - v_from + v_to;
    const double p2 = t2 > 0.0 ? t2 * (t2 + 2.0 * M_NUCLEON) : 0.0;
    if (t2 <= 0.0 || p2 <= pt2) {
        for (int a = 0; a < 3; ++a) d[a] -= 2.0 * dn * n[a];   /* reflected */
        *t_out = t;
        return 0;
    }
    const double pn = (dn >= 0.0 ? 1.0 : -1.0) * sqrt(p2 - pt2);
    const double pm = sqrt(p2);
    for (int a = 0; a < 3; ++a) d[a] = (pt[a] + pn * n[a]) / pm;
    *t_out = t2;
    return 1;
}

static int refract(const ora_nucleus* nu, cpart* q, int j)
{
    const double vk = well(nu, q->species, q->shell);
    const double vj = j < ORA_INC_SHELLS ? well(nu, q->species, j) : 0.0;
    double t2;
    if (!oracle_inc_refract(q->t, vk, vj, q->x, q->d, &t2)) return 0;
    q->t = t2;
    q->shell = j;
    return 1;
}

/* elastic collision of (p1, E1) and (p2, E2), equal masses M: the CM
 * direction of particle 1 turned by theta* (from exp(B t)) and azimuth
 * phi* (revolutions) about its incoming CM direction; outputs lab momenta */
void oracle_nn_collide(const double p1[3], const double p2[3], double u_t, double u_phi, double o1[3], double o2[3])
{
    const double M = M_NUCLEON;
    const double e1 = sqrt(p1[0] * p1[0] + p1[1] * p1[1] + p1[2] * p1[2] + M * M);
    const double e2 = sqrt(p2[0] * p2[0] + p2[1] * p2[1] + p2[2] * p2[2] + M * M);
    const double E = e1 + e2;
    double P[3] = {p1[0] + p2[0], p1[1] + p2[1], p1[2] + p2[2]};
    const double P2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
    const double s = E * E - P2;
    const double W = sqrt(s);
    /* boost of particle 1 into the CM frame (velocity P/E) */
    double b[3] = {P[0] / E, P[1] / E, P[2] / E};
    const double b2 = P2 / (E * E);
    const double g = E / W;
    const double bp = b[0] * p1[0] + b[1] * p1[1] + b[2] * p1[2];
    double q[3];
    for (int a = 0; a < 3; ++a) q[a] = p1[a] + ((g - 1.0) * bp / (b2 > 0.0 ? b2 : 1.0) - g * e1) * b[a];
    if (b2 <= 0.0)
        for (int a = 0; a < 3; ++a) q[a] = p1[a];
    const double ps2 = s / 4.0 - M * M;
    const double ps = sqrt(ps2 > 0.0 ? ps2 : 0.0);
    double dq[3];
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    for (int a = 0; a < 3; ++a) dq[a] = qn > 0.0 ? q[a] / qn : (a == 2 ? 1.0 : 0.0);
    /* momentum transfer t in [-4 p*^2, 0] with density ~ exp(B t) */
    const double plab = sqrt((s - 2.0 * M * M) * (s - 2.0 * M * M) - 4.0 * M * M * M * M) / (2.0 * M) * 1e-3;
    const double B = oracle_nn_slope(plab);
    const double ps2g = ps * ps * 1e-6;   /* (GeV/c)^2 */
    const double x = 4.0 * ps2g * B;
    double tt;
    if (x < 1e-6) tt = -4.0 * ps2g * u_t;
    else tt = log(1.0 - u_t * (1.0 - exp(-x))) / B;
    double ct = ps2g > 0.0 ? 1.0 + tt / (2.0 * ps2g) : 1.0;
    if (ct > 1.0) ct = 1.0;
    if (ct < -1.0) ct = -1.0;
    const double st = sqrt(1.0 - ct * ct);
    oracle_rotate(dq, ct, st, u_phi);
    /* back to the nucleus frame */
    for (int k = 0; k < 2; ++k) {
        const double sg = k == 0 ? 1.0 : -1.0;
        double c[3] = {sg * ps * dq[0], sg * ps * dq[1], sg * ps * dq[2]};
        const double ec = W / 2.0;
        const double bc = b[0] * c[0] + b[1] * c[1] + b[2] * c[2];
        double* o = k == 0 ? o1 : o2;
        for (int a = 0; a < 3; ++a)
            o[a] = c[a] + ((g - 1.0) * bc / (b2 > 0.0 ? b2 : 1.0) + g * ec) * b[a];
        if (b2 <= 0.0)
            for (int a = 0; a < 3; ++a) o[a] = c[a];
    }
}

static void emit(ora_inc_result* r, int kind, int stage, uint32_t id, double t, const double d[3])
{
    if (r->n >= ORA_INC_MAX_OUT) return;
    const int i = r->n++;
    r->kind[i] = kind;
    r->stage[i] = stage;
    r->id[i] = id;
    r->t[i] = t;
    for (int a = 0; a < 3; ++a) r->dir[i][a] = d[a];
}

static uint32_t ctag(int attempt, int index, int m)
{
    return 0x40000000u | ((uint32_t)attempt << 20) | ((uint32_t)index << 12) | (uint32_t)m;
}

/* One entry of the incident proton and the cascade it starts.  Returns the
 * number of allowed collisions; fills r (emissions, holes, trapped). */
static int cascade(const ora_nucleus* nu, double t_in, uint64_t seed, uint64_t uid, uint32_t ks, int attempt,
                   ora_inc_result* r, double* e_star_sum, int* n_esc, int* n_esc_p)
{
    cpart stack[MAX_PARTICLES];
    int ns = 0, next_index = 1, n_coll = 0;
    int left_p = nu->z, left_n = nu->a - nu->z;     /* target nucleons not yet struck */
    const int r_first = r->n;
    double u[4];
    /* entry: impact parameter uniform over the disc of radius r_out */
    draw(seed, uid, ks, ctag(attempt, 0, 0), u);
    cpart q;
    memset(&q, 0, sizeof(q));
    const double b = nu->r_out * sqrt(u[0]);
    const double ph = 2.0 * M_PI * u[1];
    q.x[0] = b * cos(ph);
    q.x[1] = b * sin(ph);
    q.x[2] = -sqrt(fmax(nu->r_out * nu->r_out - b * b, 0.0));
    q.d[2] = 1.0;
    q.species = 1;
    q.index = 0;
    q.m = 1;
    q.t = t_in;
    q.shell = ORA_INC_SHELLS;     /* outside, about to enter the outermost shell */
    int entered;
    {
        /* entering: the refraction into shell 14 from outside (potential 0) */
        const double v = well(nu, 1, ORA_INC_SHELLS - 1);
        cpart tmp = q;
        tmp.shell = ORA_INC_SHELLS - 1;
        tmp.t = t_in + v;          /* kinetic energy inside */
        /* inward refraction: tangential momentum kept, normal grows */
        const double rr = nu->r_out;
        double n[3] = {q.x[0] / rr, q.x[1] / rr, q.x[2] / rr};
        const double p_out = sqrt(t_in * (t_in + 2.0 * M_NUCLEON));
        const double p_in = sqrt(tmp.t * (tmp.t + 2.0 * M_NUCLEON));
        const double dn = q.d[0] * n[0] + q.d[1] * n[1] + q.d[2] * n[2];
        double pt[3];
        for (int a = 0; a < 3; ++a) pt[a] = p_out * (q.d[a] - dn * n[a]);
        const double pt2 = pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2];
        const double pn = -sqrt(fmax(p_in * p_in - pt2, 0.0));
        for (int a = 0; a < 3; ++a) tmp.d[a] = (pt[a] + pn * n[a]) / p_in;
        q = tmp;
        entered = b < nu->r_out;
    }
    if (!entered) return 0;
    stack[ns++] = q;
    while (ns > 0) {
        cpart c = stack[--ns];
        int done = 0;
        for (int flight = 0; !done && flight < MAX_FLIGHTS; ++flight) {
            const int k = c.shell;
            /* trapped: bound below the continuum, it can never leave */
            if (c.t - well(nu, c.species, k) <= 0.0 || c.reflections > MAX_REFLECT) {
                *e_star_sum += c.t - fermi(nu, c.species, k);
                done = 1;
                break;
            }
            /* distances to the shell's outer and inner spheres */
            const double s_out = to_sphere(c.x, c.d, nu->r[k + 1], 1);
            const double s_in = k > 0 ? to_sphere(c.x, c.d, nu->r[k], 0) : INFINITY;
            const double s_b = s_in < s_out ? s_in : s_out;
            /* mean free path from the free cross sections at the local
             * kinetic energy on a nucleon at rest; partner densities of the
             * species still present */
            const double rp = left_p > 0 ? nu->rho_p[k] : 0.0, rn = left_n > 0 ? nu->rho_n[k] : 0.0;
            const double sg_p = oracle_nn_sigma_mb(c.species == 1, c.t), sg_n = oracle_nn_sigma_mb(c.species == 0, c.t);
            const double Sig = 0.1 * (rp * sg_p + rn * sg_n);   /* 1 mb = 0.1 fm^2 */
            draw(seed, uid, ks, ctag(attempt, c.index, c.m), u);
            c.m++;
            const double s_c = Sig > 0.0 ? -log(u[0]) / Sig : INFINITY;
            if (s_c >= s_b) {
                for (int a = 0; a < 3; ++a) c.x[a] += s_b * c.d[a];
                const int j = s_in < s_out ? k - 1 : k + 1;
                const int crossed = refract(nu, &c, j);
                if (!crossed) {
                    c.reflections++;
                    continue;
                }
                if (c.shell == ORA_INC_SHELLS) {
                    /* left the nucleus: kinetic energy outside */
                    emit(r, c.species ? ORA_EJ_P : ORA_EJ_N, 0, 0x100u + (uint32_t)c.index, c.t, c.d);
                    (*n_esc)++;
                    if (c.species) (*n_esc_p)++;
                    done = 1;
                }
                continue;
            }
            /* a collision candidate at distance s_c */
            for (int a = 0; a < 3; ++a) c.x[a] += s_c * c.d[a];
            const int partner = (u[1] * (rp * sg_p + rn * sg_n) < rp * sg_p) ? 1 : 0;
            const double pf = HBARC * cbrt(3.0 * M_PI * M_PI * (partner ? nu->rho_p[k] : nu->rho_n[k]));
            double u2[4];
            draw(seed, uid, ks, ctag(attempt, c.index, c.m), u2);
            c.m++;
            const double uf[3] = {u[2], u[3], u2[0]};
            double p2[3];
            oracle_fermi_momentum(pf, uf, p2);
            const double t2 = sqrt(p2[0] * p2[0] + p2[1] * p2[1] + p2[2] * p2[2] + M_NUCLEON * M_NUCLEON) - M_NUCLEON;
            const double pc = sqrt(c.t * (c.t + 2.0 * M_NUCLEON));
            const double p1[3] = {pc * c.d[0], pc * c.d[1], pc * c.d[2]};
            double o1[3], o2[3];
            oracle_nn_collide(p1, p2, u2[1], u2[2], o1, o2);
            int sp1 = c.species, sp2 = partner;
            if (sp1 != sp2 && u2[3] < 0.5) {       /* np: symmetric about 90 degrees */
                sp1 = partner;
                sp2 = c.species;
            }
            const double t1o = sqrt(o1[0] * o1[0] + o1[1] * o1[1] + o1[2] * o1[2] + M_NUCLEON * M_NUCLEON) - M_NUCLEON;
            const double t2o = sqrt(o2[0] * o2[0] + o2[1] * o2[1] + o2[2] * o2[2] + M_NUCLEON * M_NUCLEON) - M_NUCLEON;
            /* Pauli blocking: both products above their Fermi energies, and
             * room for one more particle in the cascade */
            if (!(t1o > fermi(nu, sp1, k) && t2o > fermi(nu, sp2, k)) || next_index >= MAX_PARTICLES ||
                ns + 2 > MAX_PARTICLES) {
                r->n_blocked++;
                continue;
            }
            n_coll++;
            r->n_coll++;
            {
                const double m1 = t1o - fermi(nu, sp1, k), m2 = t2o - fermi(nu, sp2, k);
                const double mm = m1 < m2 ? m1 : m2;
                if (mm < r->pauli_min) r->pauli_min = mm;
            }
            if (partner) left_p--;
            else left_n--;
            *e_star_sum += fermi(nu, partner, k) - t2;       /* the hole */
            cpart a1 = c, a2 = c;
            a1.species = sp1;
            a1.t = t1o;
            a2.species = sp2;
            a2.t = t2o;
            a2.index = next_index++;
            a2.m = 0;
            a2.reflections = 0;
            const double n1 = sqrt(o1[0] * o1[0] + o1[1] * o1[1] + o1[2] * o1[2]);
            const double n2 = sqrt(o2[0] * o2[0] + o2[1] * o2[1] + o2[2] * o2[2]);
            for (int a = 0; a < 3; ++a) {
                a1.d[a] = o1[a] / n1;
                a2.d[a] = o2[a] / n2;
            }
            stack[ns++] = a1;      /* the projectile continues after its partner */
            stack[ns++] = a2;
            done = 1;
        }
        if (!done) *e_star_sum += c.t - fermi(nu, c.species, c.shell);   /* flight cap: trapped */
    }
    if (n_coll == 0) r->n = r_first;     /* a pass without collision leaves nothing */
    return n_coll;
}

/* ======================================================================
 * Evaporation (stand-in for GEM: Weisskopf-Ewing emission of n, p, d, t,
 * 3He and alpha).  Readings: binding energies from the Weizsaecker mass
 * formula (a_v 15.75, a_s 17.8, a_c 0.711, a_a 23.7, pairing 11.18/sqrt(A)
 * MeV), measured values for A <= 4; Coulomb barrier V = e^2 z (Z - z) /
 * (1.5 (A_d^(1/3) + a^(1/3)) fm); level density exp(2 sqrt(a U)) with a =
 * A_d / 8 MeV^-1; inverse cross section pi R^2 (1 - V/eps) above the
 * barrier.  The width of channel j is then proportional to g_j mu_j R_j^2
 * integral_V^(E*-S_j) (eps - V) exp(2 sqrt(a (E* - S_j - eps))) d eps, g the
 * spin degeneracy, mu the reduced mass number, R = 1.5 (A_d^(1/3) +
 * a^(1/3)) fm; the kinetic energy follows the integrand.  Emission stops when
 * no channel is open or A <= 4.
 * ====================================================================== */
static const int EJ_Z[6] = {0, 1, 1, 1, 2, 2};
static const int EJ_A[6] = {1, 1, 2, 3, 3, 4};
static const double EJ_G[6] = {2.0, 2.0, 3.0, 2.0, 2.0, 1.0};

double oracle_binding_energy(int z, int a)
{
    if (a < 1 || z < 0 || z > a) return -INFINITY;
    if (a == 1) return 0.0;
    if (a <= 4) {
        if (z == 1 && a == 2) return 2.224566;
        if (z == 1 && a == 3) return 8.481798;
        if (z == 2 && a == 3) return 7.718043;
        if (z == 2 && a == 4) return 28.295673;
        return -INFINITY;
    }
    const int n = a - z;
    const double A = a, a13 = cbrt(A);
    double b = 15.75 * A - 17.8 * a13 * a13 - 0.711 * z * (z - 1) / a13 - 23.7 * (double)(n - z) * (n - z) / A;
    if (z % 2 == 0 && n % 2 == 0) b += 11.18 / sqrt(A);
    else if (z % 2 == 1 && n % 2 == 1) b -= 11.18 / sqrt(A);
    return b;
}

static int channel(int z, int a, double e_star, int j, double* sep, double* barrier, double* x_max, double* lda,
                   double* weight)
{
    const int zd = z - EJ_Z[j], ad = a - EJ_A[j];
    if (ad < 1 || zd < 0 || zd > ad) return 0;
    const double bd = oracle_binding_energy(zd, ad), bp = oracle_binding_energy(z, a);
    const double be = oracle_binding_energy(EJ_Z[j], EJ_A[j]);
    if (!isfinite(bd) || !isfinite(bp)) return 0;
    *sep = bp - bd - be;
    const double rad = 1.5 * (cbrt((double)ad) + cbrt((double)EJ_A[j]));
    *barrier = EJ_Z[j] ? E2_MEVFM * EJ_Z[j] * zd / rad : 0.0;
    *x_max = e_star - *sep - *barrier;
    *lda = ad / 8.0;
    const double mu = (double)EJ_A[j] * ad / (EJ_A[j] + ad);
    *weight = EJ_G[j] * mu * rad * rad;
    return *x_max > 0.0;
}

double oracle_evap_width(int z, int a, double e_star, int j, double* sep, double* barrier)
{
    double s = 0, v = 0, x = 0, la = 0, w = 0;
    if (j < 0 || j > 5) return 0.0;
    const int open = channel(z, a, e_star, j, &s, &v, &x, &la, &w);
    if (sep) *sep = s;
    if (barrier) *barrier = v;
    if (!open) return 0.0;
    /* Simpson's rule for integral_0^X (X - y) exp(2 sqrt(a y)) dy (y = the
     * residual excitation), on a grid fine in sqrt(y) */
    const int n = 4000;
    double sum = 0.0;
    for (int i = 0; i <= n; ++i) {
        const double sq = sqrt(x) * i / n;          /* y = sq^2, dy = 2 sq dsq */
        const double y = sq * sq;
        const double f = (x - y) * exp(2.0 * sqrt(la) * sq) * 2.0 * sq;
        sum += f * (i == 0 || i == n ? 1.0 : (i % 2 ? 4.0 : 2.0));
    }
    return w * sum * (sqrt(x) / n) / 3.0;
}

int oracle_evaporate(int z, int a, double e_star, uint64_t seed, uint64_t uid, uint32_t ks, ora_inc_result* r)
{
    double u[4];
    for (int i = 0; i < 255 && a > 4 && r->n < ORA_INC_MAX_OUT; ++i) {
        double width[6], total = 0.0;
        for (int j = 0; j < 6; ++j) {
            width[j] = oracle_evap_width(z, a, e_star, j, NULL, NULL);
            total += width[j];
        }
        if (!(total > 0.0)) break;
        draw(seed, uid, ks, 0x50000000u | ((uint32_t)i << 8), u);
        int j = 0;
        double cum = 0.0;
        for (j = 0; j < 6; ++j) {
            if (width[j] <= 0.0) continue;
            cum += width[j];
            if (u[0] * total < cum) break;
        }
        if (j == 6)
            for (j = 5; width[j] <= 0.0; --j) {}
        double sep, v, x, la, w;
        channel(z, a, e_star, j, &sep, &v, &x, &la, &w);
        /* kinetic energy above the barrier y in (0, x], density ~ y exp(2
         * sqrt(la (x - y))): rejection from y = x sqrt(u) (Y = 2 sqrt(la x)
         * < 2) or from a Gamma(2, sqrt(x / la)) proposal (Y >= 2), both
         * dominating the density */
        const double Y = 2.0 * sqrt(la * x), t0 = sqrt(x / la);
        double y = 0.5 * x;
        for (int att = 1; att < 256; ++att) {
            double v4[4];
            draw(seed, uid, ks, 0x50000000u | ((uint32_t)i << 8) | (uint32_t)att, v4);
            double cand, acc;
            if (Y < 2.0) {
                cand = x * sqrt(v4[0]);
                acc = exp(2.0 * sqrt(la * (x - cand)) - Y);
            } else {
                cand = -t0 * log(v4[0] * v4[1]);
                if (cand > x) continue;
                acc = exp(2.0 * sqrt(la * (x - cand)) - Y + cand / t0);
            }
            if (v4[2] < acc) {
                y = cand;
                break;
            }
        }
        const double eps = v + y;
        const double ct = 2.0 * u[1] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
        const double d[3] = {st * cos(2.0 * M_PI * u[2]), st * sin(2.0 * M_PI * u[2]), ct};
        emit(r, j, 1, 0x400u + (uint32_t)i, eps, d);
        r->binding += sep;
        e_star -= sep + eps;
        z -= EJ_Z[j];
        a -= EJ_A[j];
    }
    r->z_fin = z;
    r->a_fin = a;
    r->e_star_fin = e_star;
    return 0;
}

int oracle_inc_event(int element, double t_mev, uint64_t seed, uint64_t uid, uint32_t ks, int evaporate,
                     ora_inc_result* r)
{
    if (!r || element < 1 || element > 6 || !(t_mev > 0.0)) return -1;
    memset(r, 0, sizeof(*r));
    ora_nucleus nu;
    oracle_inc_nucleus(element, &nu);
    int n_esc = 0, n_esc_p = 0;
    double e_sum = 0.0;
    int attempt;
    for (attempt = 0; attempt < MAX_ATTEMPTS; ++attempt) {
        r->n = 0;
        n_esc = n_esc_p = 0;
        e_sum = 0.0;
        r->n_coll = 0;
        r->pauli_min = INFINITY;
        if (cascade(&nu, t_mev, seed, uid, ks, attempt, r, &e_sum, &n_esc, &n_esc_p) > 0) break;
    }
    r->attempts = attempt < MAX_ATTEMPTS ? attempt + 1 : MAX_ATTEMPTS;
    if (attempt == MAX_ATTEMPTS) {
        /* never an allowed collision: the proton is absorbed (compound nucleus) */
        r->n = 0;
        n_esc = n_esc_p = 0;
        r->compound = 1;
        e_sum = t_mev + S_SEP;
    }
    r->n_esc = n_esc;
    r->z_res = nu.z + 1 - n_esc_p;
    r->a_res = nu.a + 1 - n_esc;
    double out = 0.0;
    for (int i = 0; i < r->n; ++i) out += r->t[i];
    r->e_star = t_mev - out - (n_esc - 1) * S_SEP;
    r->e_star_sum = e_sum;
    r->binding = (n_esc - 1) * S_SEP;
    r->z_fin = r->z_res;
    r->a_fin = r->a_res;
    r->e_star_fin = r->e_star;
    if (evaporate && r->e_star > 0.0) oracle_evaporate(r->z_res, r->a_res, r->e_star, seed, uid, ks, r);
    return 0;
}
