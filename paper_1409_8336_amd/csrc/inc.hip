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

// channel j of nucleus (z, a) at excitation es; false when closed
HD bool evap_channel(int z, int a, double es, int j, Channel* ch)
{
    const int zd = z - kEjZ[j], ad = a - kEjA[j];
    if (ad < 1 || zd < 0 || zd > ad) return false;
    double bd, bp, be;
    if (!bound_nucleus(zd, ad, &bd) || !bound_nucleus(z, a, &bp)) return false;
    bound_nucleus(kEjZ[j], kEjA[j], &be);
    ch->sep = bp - bd - be;
    const double rad = 1.5 * (cbrt((double)ad) + cbrt((double)kEjA[j]));
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

HD double evap_width(int z, int a, double es, int j, Channel* ch)
{
    if (!evap_channel(z, a, es, j, ch)) return 0.0;
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

// Per-attempt bookkeeping of the cascade.
struct Tally {
    int n_esc, n_esc_p, n_kept;
    double e_sum, out_sum;
};

// One entry of the incident proton into the nucleus and the cascade it
// starts: entry point uniform over the disc of the outer radius, refraction
// into the outer shell; each particle flies to its next collision (free path
// from the free NN cross sections at its local kinetic energy, on the
// partners of the species not yet exhausted) or shell boundary; a collision
// takes a Fermi-sea partner (|p| uniform in p^3 up to the shell's Fermi
// momentum, isotropic) and is allowed only if both products end above their
// Fermi energies (Pauli) and the cascade has room; particles leave through
// the outer boundary or are trapped (below the continuum, or after too many
// reflections).  The struck nucleon's hole and trapped particles add to the
// excitation sum.  Returns the allowed collisions; emit() gets every
// particle that leaves once a collision has happened (an attempt without
// one is discarded, and its only escape is the incident proton).
template <class Emit>
__host__ __device__ int cascade(const IncNucleus& nu, double t_in, const Stream& st, int attempt, Part* stack, IncResult& r,
                       Tally& ta, Emit& emit)
{
    int ns = 0, next_index = 1, n_coll = 0;
    int left[2] = {nu.a - nu.z, nu.z};   // target nucleons not yet struck, n and p
    const double ro = nu.r[kIncShells];
    double u[4];
    draw4(st, cascade_tag(attempt, 0, 0), u);
    const double b = ro * sqrt(u[0]);
    if (!(b < ro)) return 0;
    Part q;
    q.x[0] = b * cos(2.0 * kPi * u[1]);
    q.x[1] = b * sin(2.0 * kPi * u[1]);
    q.x[2] = -sqrt(fmax(ro * ro - b * b, 0.0));
    {
        // into the outer shell from outside: tangential momentum kept, the
        // normal component grows with the well depth
        const double t_inside = t_in + well(nu, 1, kIncShells - 1);
        const double n[3] = {q.x[0] / ro, q.x[1] / ro, q.x[2] / ro};
        const double p_out = sqrt(t_in * (t_in + 2.0 * kMN));
        const double p_in = sqrt(t_inside * (t_inside + 2.0 * kMN));
        const double dn = n[2];
        const double pt[3] = {-p_out * dn * n[0], -p_out * dn * n[1], p_out * (1.0 - dn * n[2])};
        const double pt2 = pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2];
        const double pn = -sqrt(fmax(p_in * p_in - pt2, 0.0));
        for (int i = 0; i < 3; ++i) q.d[i] = (pt[i] + pn * n[i]) / p_in;
        q.t = t_inside;
    }
    q.m = 1;
    q.bits = p_bits(1, kIncShells - 1, 0, 0);
    stack[ns++] = q;
    while (ns > 0) {
        Part c = stack[--ns];
        bool done = false;
        for (int flight = 0; !done && flight < kIncMaxFlights; ++flight) {
            const int k = p_shell(c), sp = p_species(c);
            if (c.t - well(nu, sp, k) <= 0.0 || p_refl(c) > kIncMaxReflect) {
                ta.e_sum += c.t - nu.tf[sp][k];
                done = true;
                break;
            }
            const double s_out = to_sphere(c.x, c.d, nu.r[k + 1], true);
            const double s_in = k > 0 ? to_sphere(c.x, c.d, nu.r[k], false) : kInfD;
            const double s_b = s_in < s_out ? s_in : s_out;
            const double rp = left[1] > 0 ? nu.rho[1][k] : 0.0, rn = left[0] > 0 ? nu.rho[0][k] : 0.0;
            const double sg_p = nn_sigma(sp == 1, c.t), sg_n = nn_sigma(sp == 0, c.t);
            const double sig = 0.1 * (rp * sg_p + rn * sg_n);   // 1 mb = 0.1 fm^2
            draw4(st, cascade_tag(attempt, p_index(c), c.m), u);
            c.m++;
            const double s_c = sig > 0.0 ? -log(u[0]) / sig : kInfD;
            if (s_c >= s_b) {
                for (int i = 0; i < 3; ++i) c.x[i] += s_b * c.d[i];
                const int j = s_in < s_out ? k - 1 : k + 1;
                const double vj = j < kIncShells ? well(nu, sp, j) : 0.0;
                double tn;
                if (!refract(c.t, well(nu, sp, k), vj, c.x, c.d, &tn)) {
                    c.bits += 1u << 13;   // one more reflection
                    continue;
                }
                c.t = tn;
                c.bits = p_bits(sp, j, p_index(c), p_refl(c));
                if (j == kIncShells) {
                    if (n_coll > 0 && ta.n_kept < kIncMaxOut) {
                        emit(sp ? kEjP : kEjN, 0, 0x100u + (uint32_t)p_index(c), c.t, c.d, ta.n_kept);
                        ta.n_kept++;
                        ta.out_sum += c.t;
                    }
                    ta.n_esc++;
                    ta.n_esc_p += sp;
                    done = true;
                }
                continue;
            }
            // a collision candidate at distance s_c
            for (int i = 0; i < 3; ++i) c.x[i] += s_c * c.d[i];
            const int partner = (u[1] * (rp * sg_p + rn * sg_n) < rp * sg_p) ? 1 : 0;
            double u2[4];
            draw4(st, cascade_tag(attempt, p_index(c), c.m), u2);
            c.m++;
            // the partner from the Fermi sea: |p| = p_F u^(1/3), isotropic
            double p2[3];
            {
                const double pm = nu.pf[partner][k] * cbrt(u[2]);
                const double ct = 2.0 * u[3] - 1.0, stt = sqrt(fmax(0.0, 1.0 - ct * ct));
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
            if (!(t1o > nu.tf[sp1][k] && t2o > nu.tf[sp2][k]) || next_index >= kIncMaxParticles ||
                ns + 2 > kIncMaxParticles) {
                r.n_blocked++;
                continue;
            }
            n_coll++;
            left[partner]--;
            ta.e_sum += nu.tf[partner][k] - t2;   // the hole
            Part a1 = c, a2 = c;
            a1.t = t1o;
            a1.bits = p_bits(sp1, k, p_index(c), p_refl(c));
            a2.t = t2o;
            a2.m = 0;
            a2.bits = p_bits(sp2, k, next_index++, 0);
            const double n1 = sqrt(o1[0] * o1[0] + o1[1] * o1[1] + o1[2] * o1[2]);
            const double n2 = sqrt(o2[0] * o2[0] + o2[1] * o2[1] + o2[2] * o2[2]);
            for (int i = 0; i < 3; ++i) {
                a1.d[i] = o1[i] / n1;
                a2.d[i] = o2[i] / n2;
            }
            stack[ns++] = a1;   // the projectile continues after its partner
            stack[ns++] = a2;
            done = true;
        }
        if (!done) ta.e_sum += c.t - nu.tf[p_species(c)][p_shell(c)];   // flight limit: trapped
    }
    return n_coll;
}

// Evaporation of nucleus (z, a) at excitation es until no channel is open,
// A <= 4 or the event holds kIncMaxOut particles: the channel by its width;
// the ejectile's kinetic energy above the barrier, y in (0, X], with density
// ~ y exp(2 sqrt(a (X - y))) (the width's integrand, the daughter left at
// X - y), by rejection from y = X sqrt(u) (when 2 sqrt(a X) < 2) or from a
// Gamma(2, sqrt(X/a)) proposal (otherwise), both dominating the density;
// direction isotropic.
template <class Emit>
__host__ __device__ void evaporate(int z, int a, double es, const Stream& st, IncResult& r, int& n_kept, Emit& emit)
{
    double u[4];
    for (int i = 0; i < 255 && a > 4 && n_kept < kIncMaxOut; ++i) {
        double width[6], total = 0.0;
        Channel ch;
        for (int j = 0; j < 6; ++j) {
            width[j] = evap_width(z, a, es, j, &ch);
            total += width[j];
        }
        if (!(total > 0.0)) break;
        const uint32_t tag = 0x50000000u | ((uint32_t)i << 8);
        draw4(st, tag, u);
        int j = 0;
        double cum = 0.0;
        for (j = 0; j < 6; ++j) {
            if (width[j] <= 0.0) continue;
            cum += width[j];
            if (u[0] * total < cum) break;
        }
        if (j == 6)
            for (j = 5; width[j] <= 0.0; --j) {}
        evap_channel(z, a, es, j, &ch);
        const double x = ch.x, la = ch.la;
        const double Y = 2.0 * sqrt(la * x), t0 = sqrt(x / la);
        double y = 0.5 * x;
        for (uint32_t att = 1; att < 256; ++att) {
            double v[4];
            draw4(st, tag | att, v);
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
        emit(j, 1, 0x400u + (uint32_t)i, eps, d, n_kept);
        n_kept++;
        r.binding += ch.sep;
        es -= ch.sep + eps;
        z -= kEjZ[j];
        a -= kEjA[j];
    }
    r.z_fin = z;
    r.a_fin = a;
    r.e_star_fin = es;
}

// One non-elastic event of a proton of kinetic energy t on nucleus nu:
// entry attempts until one has an allowed collision (none in
// kIncMaxAttempts: the proton is absorbed into a compound nucleus), the
// residual's excitation from the energy balance (every escaping nucleon
// beyond the incident one costs the separation energy), then evaporation.
template <class Emit>
__host__ __device__ void inc_event(const IncNucleus& nu, double t, const Stream& st, bool evap, Part* stack, IncResult& r,
                          Emit& emit)
{
    r = IncResult{};
    Tally ta{};
    int attempt;
    for (attempt = 0; attempt < kIncMaxAttempts; ++attempt) {
        ta = Tally{};
        r.n_coll = cascade(nu, t, st, attempt, stack, r, ta, emit);
        if (r.n_coll > 0) break;
    }
    r.attempts = attempt < kIncMaxAttempts ? attempt + 1 : kIncMaxAttempts;
    if (attempt == kIncMaxAttempts) {
        ta = Tally{};
        r.compound = 1;
        ta.e_sum = t + kSep;
    }
    r.n_esc = ta.n_esc;
    r.z_res = nu.z + 1 - ta.n_esc_p;
    r.a_res = nu.a + 1 - ta.n_esc;
    r.e_star = t - ta.out_sum - (double)(ta.n_esc - 1) * kSep;
    r.e_star_sum = ta.e_sum;
    r.binding = (double)(ta.n_esc - 1) * kSep;
    r.z_fin = r.z_res;
    r.a_fin = r.a_res;
    r.e_star_fin = r.e_star;
    int n_kept = ta.n_kept;
    if (evap && r.e_star > 0.0) evaporate(r.z_res, r.a_res, r.e_star, st, r, n_kept, emit);
    r.n_out = n_kept;
}

__device__ __forceinline__ void stage_nuclei(IncNucleus* dst, const IncNucleus* src)
{
    const double* s = reinterpret_cast<const double*>(src);
    double* d = reinterpret_cast<double*>(dst);
    for (int i = threadIdx.x; i < kIncTargets * (int)(sizeof(IncNucleus) / 8); i += blockDim.x) d[i] = s[i];
}

// ----------------------------------------------------------------- kernels

// Inspection: event i on element[i] at t[i], stream (uid[i], ks[i]); the
// outcome to res[i], the emitted particles to out[i * kIncMaxOut + j].
__global__ void __launch_bounds__(256) inc_inspect_kernel(const IncNucleus* __restrict__ nuclei,
                                                          const int32_t* __restrict__ element,
                                                          const double* __restrict__ t,
                                                          const unsigned long long* __restrict__ uid,
                                                          const uint32_t* __restrict__ ks, int n, uint32_t k0,
                                                          uint32_t k1, int evap, IncResult* __restrict__ res,
                                                          IncParticle* __restrict__ out)
{
    __shared__ IncNucleus nuc[kIncTargets];
    stage_nuclei(nuc, nuclei);
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Part stack[kIncMaxParticles];
    const Stream st{k0, k1, (uint32_t)uid[i], (uint32_t)(uid[i] >> 32), ks[i]};
    IncParticle* o = out + (size_t)i * kIncMaxOut;
    auto emit = [&](int kind, int stage, uint32_t id, double tt, const double d[3], int j) {
        IncParticle p;
        p.kind = kind;
        p.stage = stage;
        p.id = id;
        p.pad = 0;
        p.t = tt;
        p.dir[0] = d[0];
        p.dir[1] = d[1];
        p.dir[2] = d[2];
        o[j] = p;
    };
    IncResult r;
    inc_event(nuc[element[i] - 1], t[i], st, evap != 0, stack, r, emit);
    res[i] = r;
}

}  // namespace


namespace {

constexpr int kIncBlock = 256;
constexpr int kIncStage = 512;   // children a workgroup stages in LDS per round

// One event per lane in rounds of a workgroup's 256 lanes: the cascade and
// evaporation of the event; emitted protons above the cut-off are staged in
// LDS and written to the next generation's queue with one reservation per
// workgroup and round; local deposits (fragments, sub-cut-off protons) go to
// the event's voxel and group; neutrons, separation energies and the
// excitation left for photons to the neutral ledger.
__global__ void __launch_bounds__(kIncBlock) inc_transport_kernel(IncLaunch a)
{
    __shared__ IncNucleus nuc[kIncTargets];
    __shared__ double led[kMaxPlans][2];
    __shared__ unsigned long long cnt[kMaxPlans][3];
    __shared__ uint32_t stage_w[kIncStage][kQueuePlanes];
    __shared__ uint32_t n_staged;
    __shared__ unsigned long long stage_base;
    stage_nuclei(nuc, a.nuclei);
    for (int p = threadIdx.x; p < a.n_plans; p += blockDim.x) {
        led[p][0] = led[p][1] = 0.0;
        cnt[p][0] = cnt[p][1] = cnt[p][2] = 0ull;
    }
    if (threadIdx.x == 0) n_staged = 0u;
    __syncthreads();
    const unsigned long long rec = *a.ev_count;
    const unsigned long long n = rec < a.ev_cap ? rec : a.ev_cap;
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    const int K = a.k_batches;
    Part stack[kIncMaxParticles];
    for (unsigned long long base = (unsigned long long)blockIdx.x * blockDim.x; base < n; base += stride) {
        const unsigned long long i = base + threadIdx.x;
        if (i < n) {
            const IncEvent ev = a.ev[i];
            const PlanDesc& pd = a.plans[ev.plan];
            const Stream st{pd.key_lo, pd.key_hi, ev.uid_lo, ev.uid_hi, ev.ks};
            const double w = (double)ev.w;
            double local = 0.0, neutral = 0.0, ovf = 0.0;
            unsigned long long n_sec = 0;
            auto emit = [&](int kind, int, uint32_t id, double tt, const double d[3], int) {
                if (kind == kEjN) {
                    neutral += tt;
                    return;
                }
                if (kind != kEjP || tt <= kECutD) {
                    local += tt;
                    return;
                }
                // the child: the parent's direction turned by the emission angle
                double cd[3] = {(double)ev.ux, (double)ev.uy, (double)ev.uz};
                rotate_d(cd, d[2], sqrt(d[0] * d[0] + d[1] * d[1]), atan2(d[1], d[0]) / (2.0 * kPi));
                const uint4 cu = philox(ev.uid_lo, ev.uid_hi, ev.ks, 0xC0000000u | id, pd.key_lo, pd.key_hi);
                // the queue holds FP32 energies: the rounding stays here, so
                // that the ledger closes exactly
                const float tf = (float)tt;
                local += tt - (double)tf;
                const uint32_t e[kQueuePlanes] = {
                    __float_as_uint(ev.px), __float_as_uint(ev.py), __float_as_uint(ev.pz),
                    __float_as_uint((float)cd[0]), __float_as_uint((float)cd[1]), __float_as_uint((float)cd[2]),
                    __float_as_uint(tf), __float_as_uint(ev.w), cu.x, cu.y, ev.batch, ev.plan};
                ++n_sec;
                const uint32_t j = atomicAdd(&n_staged, 1u);
                if (j < (uint32_t)kIncStage) {
                    for (int p = 0; p < kQueuePlanes; ++p) stage_w[j][p] = e[p];
                    return;
                }
                // the stage is full: this child reserves its own slot
                const unsigned long long slot = atomicAdd(a.out_reserve, 1ull);
                if (slot < a.q_cap) {
                    for (int p = 0; p < kQueuePlanes; ++p) a.q_out[(size_t)p * a.q_cap + slot] = e[p];
                } else {
                    ovf += w * (double)tf;
                }
            };
            IncResult r;
            if (ev.element >= 1 && ev.element <= (uint32_t)kIncTargets) {
                inc_event(nuc[ev.element - 1], (double)ev.e, st, true, stack, r, emit);
                neutral += r.binding + r.e_star_fin;
            } else {
                // no cascade target (never listed by the transport): deposited
                r = IncResult{};
                local += (double)ev.e;
            }
            if (local != 0.0) {
                const unsigned long long vi = ((unsigned long long)ev.vi_hi << 32) | ev.vi_lo;
                double* tally = pd.tally;
                __hip_atomic_fetch_add(tally + vi * K + ev.batch, w * local, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                if (a.score_let) {
                    const unsigned long long nv = (unsigned long long)pd.nx * pd.ny * pd.nz;
                    __hip_atomic_fetch_add(tally + nv * (K + 1) + vi, w * local, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            atomicAdd(&led[ev.plan][0], w * neutral);
            if (ovf != 0.0) atomicAdd(&led[ev.plan][1], ovf);
            atomicAdd(&cnt[ev.plan][0], 1ull);
            if (n_sec) atomicAdd(&cnt[ev.plan][1], n_sec);
            atomicAdd(&cnt[ev.plan][2], (unsigned long long)r.n_coll);
        }
        // the round's staged children to the queue: one reservation per workgroup
        __syncthreads();
        const uint32_t ns = n_staged < (uint32_t)kIncStage ? n_staged : (uint32_t)kIncStage;
        if (threadIdx.x == 0 && ns > 0) stage_base = atomicAdd(a.out_reserve, (unsigned long long)ns);
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < ns; j += blockDim.x) {
            const unsigned long long slot = stage_base + j;
            if (slot < a.q_cap) {
                for (int p = 0; p < kQueuePlanes; ++p) a.q_out[(size_t)p * a.q_cap + slot] = stage_w[j][p];
            } else {
                const double ev_w = (double)__uint_as_float(stage_w[j][7]);
                const double ev_e = (double)__uint_as_float(stage_w[j][6]);
                atomicAdd(&led[stage_w[j][11]][1], ev_w * ev_e);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) n_staged = 0u;
        __syncthreads();
    }
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

hipError_t launch_inc_inspect(const IncNucleus* nuclei, const int32_t* element, const double* t,
                              const unsigned long long* uid, const uint32_t* ks, int n, uint64_t seed, int evap,
                              IncResult* res, IncParticle* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int grid = (n + 255) / 256;
    hipLaunchKernelGGL(inc_inspect_kernel, dim3(grid), dim3(256), 0, st, nuclei, element, t, uid, ks, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32), evap, res, out);
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
    if (kind < 0 || kind > 5) return 0.0;
    const double w = pmc::evap_width(z, a, e_star, kind, &ch);
    if (sep) *sep = ch.sep;
    if (barrier) *barrier = ch.barrier;
    return w;
}
