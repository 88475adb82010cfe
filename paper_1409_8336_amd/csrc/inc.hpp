// Non-elastic proton-nucleus events by an intranuclear cascade followed by
// evaporation (arXiv:1409.8336, Sec. II.A.4): data layout shared by the
// cascade kernels and the host engine.
//
// The nucleus is a two-component Fermi gas in 15 constant-density shells of
// a Woods-Saxon profile; the incident proton and every collision product are
// followed through the shells (refraction and reflection at the shell
// boundaries, elastic nucleon-nucleon collisions with Pauli blocking) until
// they leave or are trapped; the excited residual nucleus then emits n, p,
// d, t, 3He and alpha by Weisskopf-Ewing evaporation.  Targets: the six
// nuclei C-12, N-14, O-16, P-31, Ca-40, Ti-48 (element indices 1..6 of the
// material compositions; hydrogen has no non-elastic channel).
#pragma once

#include <cstdint>

namespace pmc {

constexpr int kIncShells = 15;
constexpr int kIncTargets = 6;
constexpr int kIncMaxOut = 96;          // emitted particles kept per event
constexpr int kIncMaxParticles = 64;    // cascade particles per entry attempt
constexpr int kIncMaxAttempts = 64;     // entry attempts before the proton counts as absorbed
constexpr int kIncMaxFlights = 4096;    // flights of one particle between collisions
constexpr int kIncMaxReflect = 32;      // reflections after which a particle counts as trapped

// ejectile kinds
constexpr int kEjN = 0, kEjP = 1, kEjD = 2, kEjT = 3, kEjHe3 = 4, kEjAlpha = 5;

// One target nucleus: shell boundaries and, per species (0 neutron, 1
// proton) and shell, the density, the Fermi momentum and Fermi kinetic
// energy.  1024 bytes (staged into LDS by the event kernel).
struct IncNucleus {
    double r[16];              // shell boundaries, fm (r[0] = 0, r[15] = outer radius)
    double rho[2][kIncShells];  // nucleons per fm^3
    double pf[2][kIncShells];   // Fermi momentum, MeV/c
    double tf[2][kIncShells];   // Fermi kinetic energy, MeV
    int32_t z, a;
    double radius_ws;           // Woods-Saxon half-density radius, fm
    double pad[20];
};
static_assert(sizeof(IncNucleus) == 1024, "IncNucleus is 1 KiB");

// Evaporation constants by nucleus, built on the host: binding energies of
// every (Z, A) an event can reach (the heaviest target plus the proton;
// -infinity where the nucleus is not bound) and the cube roots of A.
constexpr int kIncZMax = 23, kIncAMax = 49;
struct IncTab {
    double bind[kIncZMax + 1][kIncAMax + 1];
    double cbrt_a[kIncAMax + 1];
};

// A non-elastic event the transport hands to the cascade kernel (64 bytes):
// the proton at the interaction point (position in voxel units of its plan,
// direction, kinetic energy, weight), its random stream (uid, the step index
// of the event), statistical group, plan, the struck element (1..6) and the
// voxel the local deposit goes to.
struct IncEvent {
    float px, py, pz, ux, uy, uz, e, w;
    uint32_t uid_lo, uid_hi, batch, plan, ks, element, vi_lo, vi_hi;
};
static_assert(sizeof(IncEvent) == 64, "IncEvent is 64 bytes");

// Per-event outcome (the inspection entry point returns it; the transport
// path keeps only what the ledger needs).
struct IncResult {
    int32_t n_out, n_coll, n_blocked, attempts, n_esc, compound, z_res, a_res, z_fin, a_fin;
    int32_t n_flights;   // flights of all cascade particles, all attempts
    int32_t pad;
    double e_star, e_star_sum, e_star_fin, binding;
};

struct IncParticle {
    int32_t kind, stage;   // kEj*, 0 cascade / 1 evaporation
    uint32_t id;           // child id: 0x100 + cascade particle index, 0x400 + evaporation step
    int32_t pad;
    double t;              // kinetic energy, MeV
    double dir[3];         // direction in the frame where the incident proton moves along +z
};

// The transport's non-elastic events of one generation.
struct PlanDesc;
struct IncLaunch {
    const IncEvent* ev;
    const unsigned long long* ev_count;   // events recorded (beyond ev_cap: counted as overflow)
    unsigned long long ev_cap;
    const IncNucleus* nuclei;             // the six targets
    const IncTab* tab;                    // evaporation constants
    unsigned long long* claim;            // events taken by waves (zeroed per generation)
    const PlanDesc* plans;                // plan descriptors of the run
    int n_plans;
    int k_batches;
    int score_let;                        // the LET_d local-deposit plane exists
    uint32_t* q_out;                      // next generation's queue (kQueuePlanes planes of q_cap)
    unsigned long long q_cap;
    unsigned long long* out_reserve;      // entries produced for the next generation
    double* ledger;                       // [plan][4]: escaped, neutral, overflow, deposited
    unsigned long long* counters;         // [plan][kPlanCounters]
};

// Host: the six target nuclei (Woods-Saxon shells by Gauss-Legendre
// quadrature), element = 1..6; the evaporation table.
void build_inc_nucleus(int element, IncNucleus* out);
void build_inc_table(IncTab* out);

}  // namespace pmc
