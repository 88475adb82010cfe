// Non-elastic proton-nucleus events on the GPU (arXiv:1409.8336, Sec.
// II.A.4): a Bertini-style intranuclear cascade in a two-component Fermi gas
// of 15 Woods-Saxon shells, then evaporation of the residual nucleus.  The
// transport writes each non-elastic event to an event list and stops the
// proton; after each transport generation one launch of inc_transport_kernel
// works the list, one event per lane, in FP64: protons it emits above the
// cut-off join the next generation's queue, neutrons and binding energy go to
// the neutral ledger, heavier fragments and sub-cut-off protons deposit their
// kinetic energy in the event's voxel (Sec. II.B.2 runs the cascade and
// evaporation as kernels of their own between transport passes).
//
// Readings where the paper is silent or names models whose parameters are
// not available here (Cugnon's nucleon-nucleon cross sections, GEM's level
// densities and inverse cross sections) are stated at each function.
//
// Random numbers: Philox4x32-10 keyed by the run (plan) key, counter (uid,
// ks, tag) for the event at step ks of history uid.  Cascade particle j's
// m-th block in entry attempt e: tag 0x40000000 | e << 20 | j << 12 | m;
// evaporation step i: tag 0x50000000 | i << 8 | r (r = 0 channel and
// direction, r >= 1 energy attempts).  A child proton's uid is the first two
// words of the block with tag 0xC0000000 | id.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "device.hpp"
#include "inc.hpp"
#include "pmc.h"
#include "rng.hpp"

namespace pmc {

namespace {

#define HD __host__ __device__ __forceinline__

constexpr double kHbarC = 197.3269804;   // MeV fm
constexpr double kMN = 938.918754;       // nucleon mass inside the cascade (mean of p and n), MeV
constexpr double kSep = 7.0;             // binding of a nucleon at the Fermi surface, MeV
constexpr double kDiffuse = 0.55;        // Woods-Saxon diffuseness, fm
constexpr double kE2 = 1.439964548;      // e^2 / (4 pi eps0), MeV fm
constexpr double kPi = 3.14159265358979323846;
constexpr double kECutD = 0.1;           // transport cut-off, MeV
constexpr double kInfD = 1.0e300;

// ------------------------------------------------------------ evaporation
// Weisskopf-Ewing emission of n, p, d, t, 3He and alpha (stand-in for GEM).
// Readings: binding energies from the Weizsaecker formula (volume 15.75,
// surface 17.8, Coulomb 0.711, asymmetry 23.7, pairing 11.18/sqrt(A) MeV),
// measured values for A <= 4; Coulomb barrier e^2 z (Z - z) / R with R =
// 1.5 (A_d^(1/3) + a^(1/3)) fm; level density exp(2 sqrt(a U)), a = A_d/8
// per MeV; inverse cross section pi R^2 (1 - V/eps) above the barrier.
// Channel j's width is then g_j mu_j R_j^2 times
//   I(X) = integral_0^X (X - y) exp(2 sqrt(a y)) dy,  X = E* - S_j - V_j,
// y the daughter's excitation; the ejectile's energy above the barrier
// follows the integrand.
constexpr int kEjZ[6] = {0, 1, 1, 1, 2, 2};
constexpr int kEjA[6] = {1, 1, 2, 3, 3, 4};
constexpr double kEjG[6] = {2.0, 2.0, 3.0, 2.0, 2.0, 1.0};

HD bool bound_nucleus(int z, int a, double* b)
{
    if (a < 1 || z < 0 || z > a) return false;
    if (a == 1) { *b = 0.0; return true; }
    if (a <= 4) {
        if (z == 1 && a == 2) { *b = 2.224566; return true; }
        if (z == 1 && a == 3) { *b = 8.481798; return true; }
        if (z == 2 && a == 3) { *b = 7.718043; return true; }
        if (z == 2 && a == 4) { *b = 28.295673; return true; }
        return false;
    }
    const int n = a - z;
    const double A = (double)a, a13 = cbrt(A);
    double v = 15.75 * A - 17.8 * a13 * a13 - 0.711 * (double)z * (double)(z - 1) / a13 -
               23.7 * (double)(n - z) * (double)(n - z) / A;
    const double pair = 11.18 / sqrt(A);
    if ((z & 1) == 0 && (n & 1) == 0) v += pair;
    else if ((z & 1) == 1 && (n & 1) == 1) v -= pair;
    *b = v;
    return true;
}

struct Channel {
    double sep, barrier, x, la, weight;
};

// channel j of nucleus (z, a) at excitation es; false when closed.  The
// binding energies and cube roots come from the host-built table t
// (z <= kIncZMax, a <= kIncAMax: every nucleus an event can reach)
HD bool evap_channel(const IncTab& t, int z, int a, double es, int j, Channel* ch)
{
    const int zd = z - kEjZ[j], ad = a - kEjA[j];
    if (ad < 1 || zd < 0 || zd > ad) return false;
    const double bd = t.bind[zd][ad], bp = t.bind[z][a];
    if (!(bd > -kInfD) || !(bp > -kInfD)) return false;   // unbound
    const double be = t.bind[kEjZ[j]][kEjA[j]];
    ch->sep = bp - bd - be;
    const double rad = 1.5 * (t.cbrt_a[ad] + t.cbrt_a[kEjA[j]]);
    ch->barrier = kEjZ[j] ? kE2 * (double)kEjZ[j] * (double)zd / rad : 0.0;
    ch->x = es - ch->sep - ch->barrier;
    ch->la = (double)ad / 8.0;
    const double mu = (double)kEjA[j] * (double)ad / (double)(kEjA[j] + ad);
    ch->weight = kEjG[j] * mu * rad * rad;
    return ch->x > 0.0;
}

// I(X) in closed form: with c = 2 sqrt(a), q = c sqrt(X), two integrations
// by parts of (X - s^2) e^(c s) 2 s ds give
//   I = 2 [e^q (2 q^2 - 6 q + 6) + q^2 - 6] / c^4;
// below q = 1 the terms cancel, and the power series of the exponential,
//   I = X^2 sum_k q^k / (k! (k/2 + 1)(k/2 + 2)),
// is used instead.
HD double level_integral(double x, double la)
{
    const double c = 2.0 * sqrt(la), q = c * sqrt(x);
    if (q >= 1.0) {
        const double c2 = c * c;
        return 2.0 * (exp(q) * (2.0 * q * q - 6.0 * q + 6.0) + q * q - 6.0) / (c2 * c2);
    }
    double term = 1.0, sum = 0.0;
    for (int k = 0; k < 40; ++k) {
        if (k) term *= q / (double)k;
        sum += term / ((0.5 * k + 1.0) * (0.5 * k + 2.0));
        if (term < 1e-18 * sum) break;
    }
    return x * x * sum;
}

HD double evap_width(const IncTab& t, int z, int a, double es, int j, Channel* ch)
{
    if (!evap_channel(t, z, a, es, j, ch)) return 0.0;
    return ch->weight * level_integral(ch->x, ch->la);
}

// ---------------------------------------------------------------- cascade
// Free nucleon-nucleon elastic cross sections, mb (stand-ins keeping the
// shape of the measured ones below 250 MeV): like nucleons 22 + 1000/T,
// unlike 30 + 3000/T, T the lab kinetic energy on a nucleon at rest (at
// least 1 MeV).  The CM angle follows d sigma/dt ~ exp(B t), B = 5.5 p^8 /
// (7.7 + p^8) (GeV/c)^-2 with p the lab momentum in GeV/c (Cugnon's slope).
HD double nn_sigma(bool same, double t)
{
    const double tt = t > 1.0 ? t : 1.0;
    return same ? 22.0 + 1000.0 / tt : 30.0 + 3000.0 / tt;
}

struct Stream {
    uint32_t k0, k1, uid_lo, uid_hi, ks;
};

HD void draw4(const Stream& s, uint32_t tag, double u[4])
{
    const uint4 r = philox(s.uid_lo, s.uid_hi, s.ks, tag, s.k0, s.k1);
    u[0] = (double)u01(r.x);
    u[1] = (double)u01(r.y);
    u[2] = (double)u01(r.z);
    u[3] = (double)u01(r.w);
}

HD uint32_t cascade_tag(int attempt, int index, uint32_t m)
{
    return 0x40000000u | ((uint32_t)attempt << 20) | ((uint32_t)index << 12) | m;
}

// rotate unit vector d by polar (ct, st) and azimuth phi (revolutions); a
// vector along z takes the frame of the axes
HD void rotate_d(double d[3], double ct, double st, double phi)
{
    const double cp = cos(2.0 * kPi * phi), sp = sin(2.0 * kPi * phi);
    const double u = d[0], v = d[1], w = d[2];
    const double perp = sqrt(u * u + v * v);
    if (perp < 1e-6) {
        d[0] = st * cp;
        d[1] = st * sp;
        d[2] = (w >= 0.0 ? ct : -ct);
        return;
    }
    d[0] = u * ct + st * (u * w * cp - v * sp) / perp;
    d[1] = v * ct + st * (v * w * cp + u * sp) / perp;
    d[2] = w * ct - st * cp * perp;
}

// A cascade particle: position (fm), direction, kinetic energy above the
// local well bottom; its draw stream (index, next block m); species (0 n,
// 1 p), shell (15 = outside) and reflections.  64 bytes.
struct Part {
    double x[3], d[3], t;
    uint32_t m;
    uint32_t bits;   // species | shell << 1 | index << 6 | reflections << 13
};
HD int p_species(const Part& p) { return (int)(p.bits & 1u); }
HD int p_shell(const Part& p) { return (int)((p.bits >> 1) & 31u); }
HD int p_index(const Part& p) { return (int)((p.bits >> 6) & 127u); }
HD int p_refl(const Part& p) { return (int)(p.bits >> 13); }
HD uint32_t p_bits(int species, int shell, int index, int refl)
{
    return (uint32_t)species | ((uint32_t)shell << 1) | ((uint32_t)index << 6) | ((uint32_t)refl << 13);
}

// well depth of a species in shell k: Fermi energy + separation energy (the
// Fermi surface lies kSep below the continuum in every shell)
HD double well(const IncNucleus& nu, int sp, int k) { return nu.tf[sp][k] + kSep; }

// path length along d from x to the sphere of radius r: the exit root
// (outward, at least 0) or the nearer entry root (inward; none: kInfD)
HD double to_sphere(const double x[3], const double d[3], double r, bool outward)
{
    const double b = x[0] * d[0] + x[1] * d[1] + x[2] * d[2];
    const double c = x[0] * x[0] + x[1] * x[1] + x[2] * x[2] - r * r;
    const double disc = b * b - c;
    if (disc < 0.0) return kInfD;
    const double q = sqrt(disc);
    if (outward) return fmax(q - b, 0.0);
    const double s = -b - q;
    return s > 0.0 ? s : kInfD;
}

// Crossing a shell boundary at surface point x from a well of depth v_from
// into one of depth v_to: the total energy is conserved and only the
// momentum component along the surface normal changes; when the new kinetic
// energy cannot carry the tangential momentum the particle is reflected.
// Returns true (and the new kinetic energy in *t_out) when it crossed.
__host__ __device__ bool refract(double t, double v_from, double v_to, const double x[3], double d[3], double* t_out)
{
    const double rr = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double n[3] = {x[0] / rr, x[1] / rr, x[2] / rr};
    const double p = sqrt(t * (t + 2.0 * kMN));
    const double dn = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
    const double pt[3] = {p * (d[0] - dn * n[0]), p * (d[1] - dn * n[1]), p * (d[2] - dn * n[2])};
    const double pt2 = pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2];
    const double tn = t - v_from + v_to;
    const double pn2 = tn > 0.0 ? tn * (tn + 2.0 * kMN) : 0.0;
    if (tn <= 0.0 || pn2 <= pt2) {
        for (int i = 0; i < 3; ++i) d[i] -= 2.0 * dn * n[i];
        *t_out = t;
        return false;
    }
    const double pn = (dn >= 0.0 ? 1.0 : -1.0) * sqrt(pn2 - pt2);
    const double pm = sqrt(pn2);
    for (int i = 0; i < 3; ++i) d[i] = (pt[i] + pn * n[i]) / pm;
    *t_out = tn;
    return true;
}

// Elastic collision of two nucleons of momenta p1, p2 (MeV/c, equal masses
// kMN): boost to the CM frame, turn particle 1's CM direction by the polar
// angle from d sigma/dt ~ exp(B t) (t in [-4 p*^2, 0]) and azimuth u_phi
// (revolutions) about its incoming CM direction, boost back.
__host__ __device__ void nn_collide(const double p1[3], const double p2[3], double u_t, double u_phi, double o1[3],
                           double o2[3])
{
    const double m2 = kMN * kMN;
    const double e1 = sqrt(p1[0] * p1[0] + p1[1] * p1[1] + p1[2] * p1[2] + m2);
    const double e2 = sqrt(p2[0] * p2[0] + p2[1] * p2[1] + p2[2] * p2[2] + m2);
    const double E = e1 + e2;
    const double P[3] = {p1[0] + p2[0], p1[1] + p2[1], p1[2] + p2[2]};
    const double P2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
    const double s = E * E - P2;
    const double W = sqrt(s);
    const double beta[3] = {P[0] / E, P[1] / E, P[2] / E};
    const double b2 = P2 / (E * E);
    const double g = E / W;
    const bool moving = b2 > 0.0;
    // particle 1 in the CM frame
    double q[3];
    const double bp = beta[0] * p1[0] + beta[1] * p1[1] + beta[2] * p1[2];
    const double f1 = moving ? (g - 1.0) * bp / b2 - g * e1 : 0.0;
    for (int i = 0; i < 3; ++i) q[i] = p1[i] + f1 * beta[i];
    const double ps = sqrt(fmax(0.25 * s - m2, 0.0));
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    double dq[3];
    for (int i = 0; i < 3; ++i) dq[i] = qn > 0.0 ? q[i] / qn : (i == 2 ? 1.0 : 0.0);
    // lab momentum of the pair's invariant mass on a nucleon at rest, GeV/c
    const double sm = s - 2.0 * m2;
    const double plab = sqrt(sm * sm - 4.0 * m2 * m2) / (2.0 * kMN) * 1e-3;
    const double pl2 = plab * plab, pl4 = pl2 * pl2, pl8 = pl4 * pl4;
    const double B = 5.5 * pl8 / (7.7 + pl8);
    const double ps2g = ps * ps * 1e-6;   // (GeV/c)^2
    const double xx = 4.0 * ps2g * B;
    const double tt = xx < 1e-6 ? -4.0 * ps2g * u_t : log(1.0 - u_t * (1.0 - exp(-xx))) / B;
    double ct = ps2g > 0.0 ? 1.0 + tt / (2.0 * ps2g) : 1.0;
    ct = fmin(1.0, fmax(-1.0, ct));
    rotate_d(dq, ct, sqrt(1.0 - ct * ct), u_phi);
    // back to the nucleus frame: +p* dq and -p* dq, each with energy W/2
    for (int k = 0; k < 2; ++k) {
        const double sg = k == 0 ? ps : -ps;
        const double c[3] = {sg * dq[0], sg * dq[1], sg * dq[2]};
        const double bc = beta[0] * c[0] + beta[1] * c[1] + beta[2] * c[2];
        const double f = moving ? (g - 1.0) * bc / b2 + g * (0.5 * W) : 0.0;
        double* o = k == 0 ? o1 : o2;
        for (int i = 0; i < 3; ++i) o[i] = c[i] + f * beta[i];
    }
}

HD double kinetic(const double p[3])
{
    return sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + kMN * kMN) - kMN;
}

// ------------------------------------------------------ one event, in steps
// An event runs as a sequence of steps over a per-event state, so that a
// wave can run its lanes' events side by side, each lane at its own step:
//   entry       one entry attempt of the incident proton (impact parameter
//               uniform over the outer disc, refraction into the outer shell);
//   flight      one flight of the particle in flight (taken from the
//               cascade's stack when none is): to the next shell boundary
//               (refraction or reflection; leaving through the outer one
//               emits it) or to a collision candidate;
//   collide     the candidate collision: a Fermi-sea partner (|p| = p_F
//               u^(1/3), isotropic), the NN kinematics, Pauli blocking (both
//               products above their Fermi energies, room in the cascade);
//               an allowed collision stacks both products (the projectile
//               continues after its partner);
//   attempt end the cascade of an attempt that had an allowed collision
//               ends the cascade; otherwise the next attempt (after
//               kIncMaxAttempts the proton is absorbed: a compound nucleus);
//   evaporate   one emission of the residual nucleus (channel by width,
//               energy above the barrier y in (0, X] with density ~ y
//               exp(2 sqrt(a (X - y))) -- the width's integrand with the
//               daughter at X - y -- by rejection from y = X sqrt(u) when
//               2 sqrt(a X) < 2, else from a Gamma(2, sqrt(X/a)) proposal,
//               both dominating the density; direction isotropic), until no
//               channel is open, A <= 4 or the event holds kIncMaxOut
//               particles.
// The steps take the draws of the event's stream in the same order whatever
// the interleaving.  Particles that leave are emitted only once the attempt
// has had a collision (an attempt without one is discarded, and its only
// escape is the incident proton); emitted kinetic energy and nucleon count
// give the residual's excitation.
enum : int { kPhIdle = 0, kPhEntry, kPhFlight, kPhCollide, kPhAttemptEnd, kPhEvap, kPhDone };

struct EvState {
    Stream st;
    double t_in;
    int element;                 // 1..6
    int phase;
    bool evap;                   // evaporate after the cascade
    int attempt, n_coll, next_index, ns, left_n, left_p;
    int n_esc, n_esc_p, n_kept;
    double e_sum, out_sum;
    Part c;                      // the particle in flight
    int flight;                  // its flights since it left the stack
    bool live;
    int partner;                 // pending collision: partner species and the two Fermi-sea draws
    double uf0, uf1;
    int ez, ea, ei;              // evaporation: the nucleus and the next emission
    double es;
    IncResult r;                 // the outcome
};

HD void ev_begin(EvState& s, int element, double t, const Stream& st, bool evap)
{
    s.st = st;
    s.t_in = t;
    s.element = element;
    s.evap = evap;
    s.attempt = 0;
    s.r = IncResult{};
    s.phase = kPhEntry;
}

HD void ev_entry(EvState& s, const IncNucleus& nu)
{
    s.ns = 0;
    s.next_index = 1;
    s.n_coll = 0;
    s.left_n = nu.a - nu.z;
    s.left_p = nu.z;
    s.n_esc = s.n_esc_p = s.n_kept = 0;
    s.e_sum = s.out_sum = 0.0;
    const double ro = nu.r[kIncShells];
    double u[4];
    draw4(s.st, cascade_tag(s.attempt, 0, 0), u);
    const double b = ro * sqrt(u[0]);
    if (!(b < ro)) {
        s.phase = kPhAttemptEnd;
        return;
    }
    Part& q = s.c;
    q.x[0] = b * cos(2.0 * kPi * u[1]);
    q.x[1] = b * sin(2.0 * kPi * u[1]);
    q.x[2] = -sqrt(fmax(ro * ro - b * b, 0.0));
    // into the outer shell from outside: tangential momentum kept, the
    // normal component grows with the well depth
    const double t_inside = s.t_in + well(nu, 1, kIncShells - 1);
    const double n[3] = {q.x[0] / ro, q.x[1] / ro, q.x[2] / ro};
    const double p_out = sqrt(s.t_in * (s.t_in + 2.0 * kMN));
    const double p_in = sqrt(t_inside * (t_inside + 2.0 * kMN));
    const double dn = n[2];
    const double pt[3] = {-p_out * dn * n[0], -p_out * dn * n[1], p_out * (1.0 - dn * n[2])};
    const double pt2 = pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2];
    const double pn = -sqrt(fmax(p_in * p_in - pt2, 0.0));
    for (int i = 0; i < 3; ++i) q.d[i] = (pt[i] + pn * n[i]) / p_in;
    q.t = t_inside;
    q.m = 1;
    q.bits = p_bits(1, kIncShells - 1, 0, 0);
    s.flight = 0;
    s.live = true;
    s.phase = kPhFlight;
}

template <class Emit>
HD void ev_flight(EvState& s, const IncNucleus& nu, Part* stack, Emit& emit)
{
    if (!s.live) {
        if (s.ns == 0) {
            s.phase = kPhAttemptEnd;
            return;
        }
        s.c = stack[--s.ns];
        s.flight = 0;
        s.live = true;
    }
    Part& c = s.c;
    const int k = p_shell(c), sp = p_species(c);
    if (s.flight >= kIncMaxFlights) {   // flight limit: trapped
        s.e_sum += c.t - nu.tf[sp][k];
        s.live = false;
        return;
    }
    ++s.r.n_flights;
    if (c.t - well(nu, sp, k) <= 0.0 || p_refl(c) > kIncMaxReflect) {   // trapped
        s.e_sum += c.t - nu.tf[sp][k];
        s.live = false;
        return;
    }
    const double s_out = to_sphere(c.x, c.d, nu.r[k + 1], true);
    const double s_in = k > 0 ? to_sphere(c.x, c.d, nu.r[k], false) : kInfD;
    const double s_b = s_in < s_out ? s_in : s_out;
    const double rp = s.left_p > 0 ? nu.rho[1][k] : 0.0, rn = s.left_n > 0 ? nu.rho[0][k] : 0.0;
    const double sg_p = nn_sigma(sp == 1, c.t), sg_n = nn_sigma(sp == 0, c.t);
    const double sig = 0.1 * (rp * sg_p + rn * sg_n);   // 1 mb = 0.1 fm^2
    double u[4];
    draw4(s.st, cascade_tag(s.attempt, p_index(c), c.m), u);
    c.m++;
    const double s_c = sig > 0.0 ? -log(u[0]) / sig : kInfD;
    if (s_c >= s_b) {
        for (int i = 0; i < 3; ++i) c.x[i] += s_b * c.d[i];
        const int j = s_in < s_out ? k - 1 : k + 1;
        const double vj = j < kIncShells ? well(nu, sp, j) : 0.0;
        double tn;
        if (!refract(c.t, well(nu, sp, k), vj, c.x, c.d, &tn)) {
            c.bits += 1u << 13;   // one more reflection
            s.flight++;
            return;
        }
        c.t = tn;
        c.bits = p_bits(sp, j, p_index(c), p_refl(c));
        if (j == kIncShells) {
            if (s.n_coll > 0 && s.n_kept < kIncMaxOut) {
                emit(sp ? kEjP : kEjN, 0, 0x100u + (uint32_t)p_index(c), c.t, c.d, s.n_kept);
                s.n_kept++;
                s.out_sum += c.t;
            }
            s.n_esc++;
            s.n_esc_p += sp;
            s.live = false;
            return;
        }
        s.flight++;
        return;
    }
    // a collision candidate at distance s_c
    for (int i = 0; i < 3; ++i) c.x[i] += s_c * c.d[i];
    s.partner = (u[1] * (rp * sg_p + rn * sg_n) < rp * sg_p) ? 1 : 0;
    s.uf0 = u[2];
    s.uf1 = u[3];
    s.phase = kPhCollide;
}

HD void ev_collide(EvState& s, const IncNucleus& nu, Part* stack)
{
    Part& c = s.c;
    const int k = p_shell(c), sp = p_species(c), partner = s.partner;
    double u2[4];
    draw4(s.st, cascade_tag(s.attempt, p_index(c), c.m), u2);
    c.m++;
    s.phase = kPhFlight;
    double p2[3];
    {
        const double pm = nu.pf[partner][k] * cbrt(s.uf0);
        const double ct = 2.0 * s.uf1 - 1.0, stt = sqrt(fmax(0.0, 1.0 - ct * ct));
        p2[0] = pm * stt * cos(2.0 * kPi * u2[0]);
        p2[1] = pm * stt * sin(2.0 * kPi * u2[0]);
        p2[2] = pm * ct;
    }
    const double t2 = kinetic(p2);
    const double pc = sqrt(c.t * (c.t + 2.0 * kMN));
    const double p1[3] = {pc * c.d[0], pc * c.d[1], pc * c.d[2]};
    double o1[3], o2[3];
    nn_collide(p1, p2, u2[1], u2[2], o1, o2);
    int sp1 = sp, sp2 = partner;
    if (sp1 != sp2 && u2[3] < 0.5) {   // n-p: identities exchanged (symmetric about 90 degrees)
        sp1 = partner;
        sp2 = sp;
    }
    const double t1o = kinetic(o1), t2o = kinetic(o2);
    if (!(t1o > nu.tf[sp1][k] && t2o > nu.tf[sp2][k]) || s.next_index >= kIncMaxParticles ||
        s.ns + 2 > kIncMaxParticles) {
        s.r.n_blocked++;
        s.flight++;
        return;
    }
    s.n_coll++;
    if (partner) s.left_p--;
    else s.left_n--;
    s.e_sum += nu.tf[partner][k] - t2;   // the hole
    Part a1 = c, a2 = c;
    a1.t = t1o;
    a1.bits = p_bits(sp1, k, p_index(c), p_refl(c));
    a2.t = t2o;
    a2.m = 0;
    a2.bits = p_bits(sp2, k, s.next_index++, 0);
    const double n1 = sqrt(o1[0] * o1[0] + o1[1] * o1[1] + o1[2] * o1[2]);
    const double n2 = sqrt(o2[0] * o2[0] + o2[1] * o2[1] + o2[2] * o2[2]);
    for (int i = 0; i < 3; ++i) {
        a1.d[i] = o1[i] / n1;
        a2.d[i] = o2[i] / n2;
    }
    stack[s.ns++] = a1;   // the projectile continues after its partner
    stack[s.ns++] = a2;
    s.live = false;
}

// the residual after the cascade (or the compound nucleus), and whether it
// evaporates
HD void ev_cascade_done(EvState& s, const IncNucleus& nu, bool compound)
{
    IncResult& r = s.r;
    r.attempts = compound ? kIncMaxAttempts : s.attempt + 1;
    r.compound = compound ? 1 : 0;
    r.n_coll = s.n_coll;
    r.n_esc = s.n_esc;
    r.z_res = nu.z + 1 - s.n_esc_p;
    r.a_res = nu.a + 1 - s.n_esc;
    r.e_star = s.t_in - s.out_sum - (double)(s.n_esc - 1) * kSep;
    r.e_star_sum = s.e_sum;
    r.binding = (double)(s.n_esc - 1) * kSep;
    r.z_fin = r.z_res;
    r.a_fin = r.a_res;
    r.e_star_fin = r.e_star;
    if (s.evap && r.e_star > 0.0) {
        s.ez = r.z_res;
        s.ea = r.a_res;
        s.es = r.e_star;
        s.ei = 0;
        s.phase = kPhEvap;
    } else {
        s.phase = kPhDone;
    }
}

HD void ev_attempt_end(EvState& s, const IncNucleus& nu)
{
    if (s.n_coll > 0) {
        ev_cascade_done(s, nu, false);
        return;
    }
    if (++s.attempt < kIncMaxAttempts) {
        s.phase = kPhEntry;
        return;
    }
    // never an allowed collision: the proton is absorbed
    s.n_kept = 0;
    s.n_esc = s.n_esc_p = 0;
    s.out_sum = 0.0;
    s.e_sum = s.t_in + kSep;
    ev_cascade_done(s, nu, true);
}

template <class Emit>
HD void ev_evaporate(EvState& s, const IncTab& tab, Emit& emit)
{
    IncResult& r = s.r;
    double width[6], total = 0.0;
    Channel ch;
    if (s.ei < 255 && s.ea > 4 && s.n_kept < kIncMaxOut) {
        for (int j = 0; j < 6; ++j) {
            width[j] = evap_width(tab, s.ez, s.ea, s.es, j, &ch);
            total += width[j];
        }
    }
    if (!(total > 0.0)) {
        r.z_fin = s.ez;
        r.a_fin = s.ea;
        r.e_star_fin = s.es;
        s.phase = kPhDone;
        return;
    }
    const uint32_t tag = 0x50000000u | ((uint32_t)s.ei << 8);
    double u[4];
    draw4(s.st, tag, u);
    int j = 0;
    double cum = 0.0;
    for (j = 0; j < 6; ++j) {
        if (width[j] <= 0.0) continue;
        cum += width[j];
        if (u[0] * total < cum) break;
    }
    if (j == 6)
        for (j = 5; width[j] <= 0.0; --j) {}
    evap_channel(tab, s.ez, s.ea, s.es, j, &ch);
    const double x = ch.x, la = ch.la;
    const double Y = 2.0 * sqrt(la * x), t0 = sqrt(x / la);
    double y = 0.5 * x;
    for (uint32_t att = 1; att < 256; ++att) {
        double v[4];
        draw4(s.st, tag | att, v);
        double cand, acc;
        if (Y < 2.0) {
            cand = x * sqrt(v[0]);
            acc = exp(2.0 * sqrt(la * (x - cand)) - Y);
        } else {
            cand = -t0 * log(v[0] * v[1]);
            if (cand > x) continue;
            acc = exp(2.0 * sqrt(la * (x - cand)) - Y + cand / t0);
        }
        if (v[2] < acc) {
            y = cand;
            break;
        }
    }
    const double eps = ch.barrier + y;
    const double ct = 2.0 * u[1] - 1.0, stt = sqrt(fmax(0.0, 1.0 - ct * ct));
    const double d[3] = {stt * cos(2.0 * kPi * u[2]), stt * sin(2.0 * kPi * u[2]), ct};
    emit(j, 1, 0x400u + (uint32_t)s.ei, eps, d, s.n_kept);
    s.n_kept++;
    r.binding += ch.sep;
    s.es -= ch.sep + eps;
    s.ez -= kEjZ[j];
    s.ea -= kEjA[j];
    s.ei++;
}

// One event, its steps in sequence (the reference order; host and device).
template <class Emit>
HD void inc_event(const IncNucleus& nu, const IncTab& tab, double t, const Stream& st, bool evap, Part* stack,
                  IncResult& r, Emit& emit)
{
    EvState s;
    ev_begin(s, 0, t, st, evap);
    while (s.phase != kPhDone) {
        switch (s.phase) {
        case kPhEntry: ev_entry(s, nu); break;
        case kPhFlight: ev_flight(s, nu, stack, emit); break;
        case kPhCollide: ev_collide(s, nu, stack); break;
        case kPhAttemptEnd: ev_attempt_end(s, nu); break;
        case kPhEvap: ev_evaporate(s, tab, emit); break;
        default: s.phase = kPhDone; break;
        }
    }
    r = s.r;
    r.n_out = s.n_kept;
}

// copy n bytes (a multiple of 8) from global memory into LDS, all lanes
__device__ __forceinline__ void stage_words(void* dst, const void* src, int bytes)
{
    const double* s = reinterpret_cast<const double*>(src);
    double* d = reinterpret_cast<double*>(dst);
    for (int i = threadIdx.x; i < bytes / 8; i += blockDim.x) d[i] = s[i];
}

// ----------------------------------------------------------------- kernels

// ------------------------------------------------------- wave scheduling
// A wave runs its 64 lanes' events side by side, one step per lane and loop
// iteration, and gives an idle lane a new event as soon as six are idle,
// so lanes are not held by the longest event of a batch.  The expensive
// steps wait for company: a collision runs once kCollBatch lanes have one
// pending (or too few lanes are still flying for that to happen), an
// evaporation step once kEvapBatch lanes are evaporating, an entry attempt
// once kEntryBatch lanes are entering; meanwhile the other lanes keep
// flying.
constexpr int kCollBatch = 24, kEvapBatch = 12, kEntryBatch = 8, kRefillIdle = 6;
constexpr int kClaimRanges = 8;   // the event list in 8 ranges, each with its own claim counter

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ int wave_mbcnt(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Src: n (events), claim(count) -> first index or >= n; begin(i, s);
// emit(i, s, kind, stage, id, t, d, j); finish(i, s); flush(force)
template <class Src>
__device__ void run_events(Src& src, const IncNucleus* nuc, const IncTab& tab, Part* stack)
{
    EvState s;
    s.phase = kPhIdle;
    unsigned long long ev = 0;
    // (wave-uniform) the last claim found events: a claim returns fewer than
    // asked near the end of a range of the list, none once every range is
    // used up, and only that ends the wave's claims
    bool more = src.n > 0;
    for (;;) {
        // refill: idle lanes take new events, one claim for the wave
        const unsigned long long idle = __ballot(s.phase == kPhIdle);
        const int n_idle = __popcll(idle);
        if (more && (n_idle >= kRefillIdle || n_idle == 64)) {
            int got = 0;
            const unsigned long long base = src.claim(n_idle, &got);
            if (got == 0) more = false;
            if (s.phase == kPhIdle) {
                const int rank = wave_mbcnt(idle);
                if (rank < got) {
                    ev = base + (unsigned long long)rank;
                    src.begin(ev, s);
                }
            }
        }
        if (__ballot(s.phase != kPhIdle) == 0ull) {
            if (!more) break;
            continue;
        }
        auto emit = [&](int kind, int stage, uint32_t id, double t, const double d[3], int j) {
            src.emit(ev, s, kind, stage, id, t, d, j);
        };
        // entry attempts in batches too (an event makes two or three)
        {
            const int n_entry = __popcll(__ballot(s.phase == kPhEntry));
            const int n_fly = __popcll(__ballot(s.phase == kPhFlight));
            if (n_entry >= kEntryBatch || n_fly < kCollBatch) {
                if (s.phase == kPhEntry) ev_entry(s, nuc[s.element - 1]);
            }
        }
        if (s.phase == kPhFlight) ev_flight(s, nuc[s.element - 1], stack, emit);
        if (s.phase == kPhAttemptEnd) ev_attempt_end(s, nuc[s.element - 1]);
        const int n_run = __popcll(__ballot(s.phase == kPhEntry || s.phase == kPhFlight ||
                                            s.phase == kPhAttemptEnd));
        const int n_col = __popcll(__ballot(s.phase == kPhCollide));
        if (n_col >= kCollBatch || (n_col > 0 && n_run < kCollBatch)) {
            if (s.phase == kPhCollide) ev_collide(s, nuc[s.element - 1], stack);
        }
        const int n_ev = __popcll(__ballot(s.phase == kPhEvap));
        if (n_ev >= kEvapBatch || (n_ev > 0 && n_run + n_col < kEvapBatch)) {
            if (s.phase == kPhEvap) ev_evaporate(s, tab, emit);
        }
        if (s.phase == kPhDone) {
            s.r.n_out = s.n_kept;
            src.finish(ev, s);
            s.phase = kPhIdle;
        }
        src.flush(false);
    }
    src.flush(true);
}

// the event list split into kClaimRanges ranges with a counter each: a wave
// claims from its workgroup's range first (spreading the atomics over 8
// addresses), then from the others
struct RangeClaim {
    unsigned long long* ctr;
    unsigned long long n;
    int home;
    __device__ unsigned long long claim(int want, int* got)
    {
        unsigned long long base = 0;
        int g = 0;
        if (lane_id() == 0) {
            // (a range's counter may run past its end: the claim then
            // moves on to the next range)
            for (int k = 0; k < kClaimRanges && g == 0; ++k) {
                const int rr = (home + k) % kClaimRanges;
                const unsigned long long lo = n * (unsigned long long)rr / kClaimRanges;
                const unsigned long long hi = n * (unsigned long long)(rr + 1) / kClaimRanges;
                if (lo == hi) continue;
                const unsigned long long off = atomicAdd(&ctr[rr], (unsigned long long)want);
                if (lo + off < hi) {
                    base = lo + off;
                    g = (int)min((unsigned long long)want, hi - base);
                }
            }
        }
        *got = __shfl(g, 0);
        return __shfl(base, 0);
    }
};

// Inspection: event i on element[i] at t[i], stream (uid[i], ks[i]); the
// outcome to res[i], the emitted particles to out[i * kIncMaxOut + j].
// Scheduled as in the transport (ctr: kClaimRanges zeroed counters).
struct InspectSrc {
    RangeClaim rc;
    unsigned long long n;
    const int32_t* element;
    const double* t;
    const unsigned long long* uid;
    const uint32_t* ks;
    uint32_t k0, k1;
    bool evap;
    IncResult* res;
    IncParticle* out;
    __device__ unsigned long long claim(int want, int* got) { return rc.claim(want, got); }
    __device__ void begin(unsigned long long i, EvState& s)
    {
        const Stream st{k0, k1, (uint32_t)uid[i], (uint32_t)(uid[i] >> 32), ks[i]};
        ev_begin(s, element[i], t[i], st, evap);
    }
    __device__ void emit(unsigned long long i, const EvState&, int kind, int stage, uint32_t id, double tt,
                         const double d[3], int j)
    {
        IncParticle p;
        p.kind = kind;
        p.stage = stage;
        p.id = id;
        p.pad = 0;
        p.t = tt;
        p.dir[0] = d[0];
        p.dir[1] = d[1];
        p.dir[2] = d[2];
        out[i * kIncMaxOut + (unsigned long long)j] = p;
    }
    __device__ void finish(unsigned long long i, const EvState& s) { res[i] = s.r; }
    __device__ void flush(bool) {}
};

__global__ void __launch_bounds__(256) inc_inspect_kernel(const IncNucleus* __restrict__ nuclei,
                                                          const IncTab* __restrict__ tab,
                                                          const int32_t* __restrict__ element,
                                                          const double* __restrict__ t,
                                                          const unsigned long long* __restrict__ uid,
                                                          const uint32_t* __restrict__ ks, int n, uint32_t k0,
                                                          uint32_t k1, int evap, unsigned long long* ctr,
                                                          IncResult* __restrict__ res,
                                                          IncParticle* __restrict__ out)
{
    __shared__ IncNucleus nuc[kIncTargets];
    __shared__ IncTab tb;
    stage_words(nuc, nuclei, (int)sizeof(nuc));
    stage_words(&tb, tab, (int)sizeof(IncTab));
    __syncthreads();
    Part stack[kIncMaxParticles];
    InspectSrc src{{ctr, (unsigned long long)n, (int)(blockIdx.x % kClaimRanges)}, (unsigned long long)n, element,
                   t, uid, ks, k0, k1, evap != 0, res, out};
    run_events(src, nuc, tb, stack);
}

}  // namespace


namespace {

constexpr int kIncBlock = 256;
constexpr int kIncWaves = kIncBlock / 64;
constexpr int kStageW = 512;      // children a wave stages in LDS before writing them out
constexpr int kStageFlush = 384;  // write out at this fill (an iteration adds at most 128)
constexpr int kStageWords = 6;    // event index, child id, energy (FP32), direction (3 x FP32)

// One child proton of event ev into slot of the next generation's queue
// (overflow when the queue is full): its direction is the emission
// direction d (in the frame where the parent moves along +z) turned into the
// parent's frame -- the rotation that takes +z to the parent's direction u
// with the azimuth convention of the transport's scattering, written with
// cos and sin of the emission azimuth as d_x / sin(theta), d_y / sin(theta);
// its uid the first two words of the event's block with tag 0xC0000000 | id.
__device__ __noinline__ bool write_child(const IncLaunch& a, const PlanDesc* pds, const IncEvent& ev, uint32_t id,
                                         float tf, float dx, float dy, float dz, unsigned long long slot)
{
    if (slot >= a.q_cap) return false;
    const PlanDesc& pd = pds[ev.plan];
    const float u = ev.ux, v = ev.uy, w = ev.uz;
    const float perp = sqrtf(u * u + v * v);
    float cx, cy, cz;
    if (perp < 1e-6f) {
        cx = dx;
        cy = dy;
        cz = w >= 0.f ? dz : -dz;
    } else {
        cx = u * dz + (u * w * dx - v * dy) / perp;
        cy = v * dz + (v * w * dx + u * dy) / perp;
        cz = w * dz - dx * perp;
    }
    const uint4 cu = philox(ev.uid_lo, ev.uid_hi, ev.ks, 0xC0000000u | id, pd.key_lo, pd.key_hi);
    const uint32_t e[kQueuePlanes] = {__float_as_uint(ev.px), __float_as_uint(ev.py), __float_as_uint(ev.pz),
                                      __float_as_uint(cx), __float_as_uint(cy), __float_as_uint(cz),
                                      __float_as_uint(tf), __float_as_uint(ev.w), cu.x, cu.y, ev.batch, ev.plan};
    for (int p = 0; p < kQueuePlanes; ++p) a.q_out[(size_t)p * a.q_cap + slot] = e[p];
    return true;
}

// The transport's events: emitted protons above the cut-off are staged in
// the wave's part of LDS and written to the next generation's queue with one
// reservation per write-out; local deposits (fragments, sub-cut-off
// protons) go to the event's voxel and group; neutrons, separation energies
// and the excitation left for photons to the neutral ledger; per-plan sums
// and counters collect in LDS.
struct TransportSrc {
    const IncLaunch& a;
    RangeClaim rc;
    unsigned long long n;
    uint32_t* stg;                 // this wave's stage
    uint32_t* n_staged;            // its fill
    double (*led)[2];
    unsigned long long (*cnt)[3];
    const PlanDesc* pds;           // the plan descriptors (LDS copy)
    // the lane's event
    double local, neutral, ovf;
    unsigned long long n_sec;
    __device__ unsigned long long claim(int want, int* got) { return rc.claim(want, got); }
    __device__ void begin(unsigned long long i, EvState& s)
    {
        const IncEvent& ev = a.ev[i];
        const PlanDesc& pd = pds[ev.plan];
        const Stream st{pd.key_lo, pd.key_hi, ev.uid_lo, ev.uid_hi, ev.ks};
        local = neutral = ovf = 0.0;
        n_sec = 0;
        if (ev.element >= 1 && ev.element <= (uint32_t)kIncTargets) {
            ev_begin(s, (int)ev.element, (double)ev.e, st, true);
        } else {
            // no cascade target (never listed by the transport): deposited
            ev_begin(s, 1, (double)ev.e, st, true);
            s.phase = kPhDone;
            local = (double)ev.e;
        }
    }
    __device__ void emit(unsigned long long i, const EvState&, int kind, int, uint32_t id, double tt,
                         const double d[3], int)
    {
        if (kind == kEjN) {
            neutral += tt;
            return;
        }
        if (kind != kEjP || tt <= kECutD) {
            local += tt;
            return;
        }
        // the queue holds FP32 energies: the rounding stays here, so that
        // the ledger closes exactly
        const float tf = (float)tt;
        local += tt - (double)tf;
        ++n_sec;
        const uint32_t j = atomicAdd(n_staged, 1u);
        if (j < (uint32_t)kStageW) {
            uint32_t* e = stg + j * kStageWords;
            e[0] = (uint32_t)i;
            e[1] = id;
            e[2] = __float_as_uint(tf);
            e[3] = __float_as_uint((float)d[0]);
            e[4] = __float_as_uint((float)d[1]);
            e[5] = __float_as_uint((float)d[2]);
            return;
        }
        // the stage is full: this child reserves its own slot
        const IncEvent ev = a.ev[i];
        if (!write_child(a, pds, ev, id, tf, (float)d[0], (float)d[1], (float)d[2], atomicAdd(a.out_reserve, 1ull)))
            ovf += (double)ev.w * (double)tf;
    }
    __device__ void finish(unsigned long long i, const EvState& s)
    {
        const IncEvent& ev = a.ev[i];
        const PlanDesc& pd = pds[ev.plan];
        const double w = (double)ev.w;
        if (s.r.attempts > 0) neutral += s.r.binding + s.r.e_star_fin;
        if (local != 0.0) {
            const int K = a.k_batches;
            const unsigned long long vi = ((unsigned long long)ev.vi_hi << 32) | ev.vi_lo;
            __hip_atomic_fetch_add(pd.tally + vi * K + ev.batch, w * local, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            if (a.score_let) {
                const unsigned long long nv = (unsigned long long)pd.nx * pd.ny * pd.nz;
                __hip_atomic_fetch_add(pd.tally + nv * (K + 1) + vi, w * local, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        atomicAdd(&led[ev.plan][0], w * neutral);
        if (ovf != 0.0) atomicAdd(&led[ev.plan][1], ovf);
        atomicAdd(&cnt[ev.plan][0], 1ull);
        if (n_sec) atomicAdd(&cnt[ev.plan][1], n_sec);
        atomicAdd(&cnt[ev.plan][2], (unsigned long long)s.r.n_coll);
    }
    // the staged children to the queue, one reservation for the wave (the
    // wave's LDS writes are complete and visible to its lanes after the fence)
    __device__ void flush(bool force)
    {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint32_t fill = *n_staged;
        if (fill == 0u || (!force && fill < (uint32_t)kStageFlush)) return;
        const uint32_t ns = min(fill, (uint32_t)kStageW);
        unsigned long long qb = 0;
        if (lane_id() == 0) qb = atomicAdd(a.out_reserve, (unsigned long long)ns);
        qb = __shfl(qb, 0);
        for (uint32_t j = (uint32_t)lane_id(); j < ns; j += 64u) {
            const uint32_t* e = stg + j * kStageWords;
            const IncEvent ev = a.ev[e[0]];
            const float tf = __uint_as_float(e[2]);
            if (!write_child(a, pds, ev, e[1], tf, __uint_as_float(e[3]), __uint_as_float(e[4]), __uint_as_float(e[5]),
                             qb + j))
                atomicAdd(&led[ev.plan][1], (double)ev.w * (double)tf);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane_id() == 0) *n_staged = 0u;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
};

__global__ void __launch_bounds__(kIncBlock) inc_transport_kernel(IncLaunch a)
{
    __shared__ IncNucleus nuc[kIncTargets];
    __shared__ IncTab tb;
    __shared__ double led[kMaxPlans][2];
    __shared__ unsigned long long cnt[kMaxPlans][3];
    __shared__ uint32_t stage[kIncWaves][kStageW * kStageWords];
    __shared__ uint32_t n_staged[kIncWaves];
    __shared__ PlanDesc pds[kMaxPlans];
    stage_words(nuc, a.nuclei, (int)sizeof(nuc));
    stage_words(&tb, a.tab, (int)sizeof(IncTab));
    stage_words(pds, a.plans, a.n_plans * (int)sizeof(PlanDesc));
    for (int p = threadIdx.x; p < a.n_plans; p += blockDim.x) {
        led[p][0] = led[p][1] = 0.0;
        cnt[p][0] = cnt[p][1] = cnt[p][2] = 0ull;
    }
    if (threadIdx.x < kIncWaves) n_staged[threadIdx.x] = 0u;
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const unsigned long long rec = *a.ev_count;
    const unsigned long long n = rec < a.ev_cap ? rec : a.ev_cap;
    Part stack[kIncMaxParticles];
    TransportSrc src{a, {a.claim, n, (int)(blockIdx.x % kClaimRanges)}, n, stage[wave], &n_staged[wave], led, cnt,
                     pds, 0.0, 0.0, 0.0, 0ull};
    run_events(src, nuc, tb, stack);
    __syncthreads();
    for (int p = threadIdx.x; p < a.n_plans; p += blockDim.x) {
        if (led[p][0] != 0.0) unsafeAtomicAdd(&a.ledger[4 * p + 1], led[p][0]);
        if (led[p][1] != 0.0) unsafeAtomicAdd(&a.ledger[4 * p + 2], led[p][1]);
        unsigned long long* C = a.counters + (size_t)kPlanCounters * p;
        if (cnt[p][0]) atomicAdd(&C[kCtrIncEvents], cnt[p][0]);
        if (cnt[p][1]) atomicAdd(&C[kCtrIncSecondaries], cnt[p][1]);
        if (cnt[p][2]) atomicAdd(&C[kCtrIncCollisions], cnt[p][2]);
    }
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n)
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

// The target nucleus: Woods-Saxon density rho0 / (1 + exp((r - R)/a)),
// R = 1.16 A^(1/3) (1 - 1.16 A^(-2/3)) fm, a = 0.55 fm, cut at R + 5a and
// split into 15 shells of equal thickness, each at the profile's mean
// density over its volume, normalised to A nucleons; protons carry Z/A of
// it, neutrons N/A.  Per shell and species: Fermi momentum (3 pi^2
// rho)^(1/3) hbar c and Fermi kinetic energy.
void build_inc_nucleus(int element, IncNucleus* out)
{
    static const int kZ[7] = {1, 6, 7, 8, 15, 20, 22};
    static const int kA[7] = {1, 12, 14, 16, 31, 40, 48};
    std::memset(out, 0, sizeof(*out));
    if (element < 1 || element > kIncTargets) return;
    const int Z = kZ[element], A = kA[element];
    const double a3 = std::cbrt((double)A);
    const double R = 1.16 * a3 * (1.0 - 1.16 / (a3 * a3));
    const double r_out = R + 5.0 * kDiffuse;
    out->z = Z;
    out->a = A;
    out->radius_ws = R;
    for (int k = 0; k <= kIncShells; ++k) out->r[k] = r_out * k / kIncShells;
    std::vector<double> gx, gw;
    gauss_legendre(24, gx, gw);
    double count[kIncShells], total = 0.0;
    for (int k = 0; k < kIncShells; ++k) {
        // 4 panels of 24-point Gauss-Legendre per shell
        double s = 0.0;
        const double lo = out->r[k], hi = out->r[k + 1];
        for (int pnl = 0; pnl < 4; ++pnl) {
            const double a0 = lo + (hi - lo) * pnl / 4.0, a1 = lo + (hi - lo) * (pnl + 1) / 4.0;
            const double hm = 0.5 * (a1 - a0), cm = 0.5 * (a1 + a0);
            for (size_t g = 0; g < gx.size(); ++g) {
                const double r = cm + hm * gx[g];
                s += gw[g] * hm * 4.0 * kPi * r * r / (1.0 + std::exp((r - R) / kDiffuse));
            }
        }
        count[k] = s;
        total += s;
    }
    for (int k = 0; k < kIncShells; ++k) {
        const double lo = out->r[k], hi = out->r[k + 1];
        const double vol = 4.0 / 3.0 * kPi * (hi * hi * hi - lo * lo * lo);
        const double rho = (double)A * count[k] / total / vol;
        out->rho[1][k] = rho * Z / A;
        out->rho[0][k] = rho * (A - Z) / A;
        for (int sp = 0; sp < 2; ++sp) {
            const double pf = kHbarC * std::cbrt(3.0 * kPi * kPi * out->rho[sp][k]);
            out->pf[sp][k] = pf;
            out->tf[sp][k] = std::sqrt(pf * pf + kMN * kMN) - kMN;
        }
    }
}

// The evaporation constants: binding energies from the formula above for
// every (Z, A) up to (kIncZMax, kIncAMax), -infinity where unbound, and the
// cube roots of A.
void build_inc_table(IncTab* out)
{
    for (int z = 0; z <= kIncZMax; ++z)
        for (int a = 0; a <= kIncAMax; ++a) {
            double b = 0.0;
            out->bind[z][a] = bound_nucleus(z, a, &b) ? b : -HUGE_VAL;
        }
    for (int a = 0; a <= kIncAMax; ++a) out->cbrt_a[a] = std::cbrt((double)a);
}

hipError_t launch_inc_transport(const IncLaunch& a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(inc_transport_kernel, dim3(grid), dim3(kIncBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t inc_transport_occupancy(int* blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)inc_transport_kernel, kIncBlock,
                                                        0);
}

hipError_t launch_inc_inspect(const IncNucleus* nuclei, const IncTab* tab, const int32_t* element, const double* t,
                              const unsigned long long* uid, const uint32_t* ks, int n, uint64_t seed, int evap,
                              unsigned long long* ctr, IncResult* res, IncParticle* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int grid = std::min((n + 255) / 256, 1024);
    hipLaunchKernelGGL(inc_inspect_kernel, dim3(grid), dim3(256), 0, st, nuclei, tab, element, t, uid, ks, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32), evap, ctr, res, out);
    return hipGetLastError();
}

}  // namespace pmc

// ------------------------------------------------------------ host C ABI

extern "C" pmc_status pmc_inc_nucleus(int32_t element, double* out, int32_t n_doubles)
{
    if (!out || n_doubles < 78 || element < 1 || element > pmc::kIncTargets) return PMC_ERR_ARG;
    pmc::IncNucleus nu;
    pmc::build_inc_nucleus(element, &nu);
    int j = 0;
    for (int k = 0; k <= pmc::kIncShells; ++k) out[j++] = nu.r[k];
    for (int sp = 1; sp >= 0; --sp)
        for (int k = 0; k < pmc::kIncShells; ++k) out[j++] = nu.rho[sp][k];
    for (int sp = 1; sp >= 0; --sp)
        for (int k = 0; k < pmc::kIncShells; ++k) out[j++] = nu.tf[sp][k];
    out[j++] = nu.radius_ws;
    out[j++] = (double)nu.a;
    return PMC_OK;
}

extern "C" double pmc_inc_width(int32_t z, int32_t a, double e_star, int32_t kind, double* sep, double* barrier)
{
    pmc::Channel ch{0, 0, 0, 0, 0};
    if (kind < 0 || kind > 5 || z < 0 || a < 1 || z > pmc::kIncZMax || a > pmc::kIncAMax) return 0.0;
    static pmc::IncTab tab;
    static std::once_flag once;
    std::call_once(once, [] { pmc::build_inc_table(&tab); });
    const double w = pmc::evap_width(tab, z, a, e_star, kind, &ch);
    if (sep) *sep = ch.sep;
    if (barrier) *barrier = ch.barrier;
    return w;
}
