// Device-side data layout shared by the transport kernels and the host
// engine.  Everything the hot loop touches per step is either in registers
// (particle state), in LDS (range and cross-section tables) or one 8-byte
// voxel record gather plus one FP64 atomic tally update.
#pragma once

#include <cstdint>

namespace pmc {

constexpr int kWave = 64;
constexpr int kQueuePlanes = 12;   // px py pz ux uy uz E w uid_lo uid_hi batch plan
constexpr int kMaxPlans = 64;
constexpr int kMaxGenerations = 64;
// counters a workgroup accumulates per plan: steps, elastic, non-elastic,
// short steps, deposits, tally atomics, of which cache-flush atomics,
// secondaries queued in the workgroup's own queue; with the ledger (escaped,
// neutral, overflow: 3 doubles) the per-plan LDS block of a batched launch
constexpr int kWgCounters = 8;
constexpr int kPlanLdsBytes = 8 * (3 + kWgCounters);
// device counters per plan (u64): the kWgCounters above, then at index 8 the
// count of workgroups that stopped at the epoch limit (plan 0 only)
constexpr int kPlanCounters = 16;
constexpr int kCtrAborted = 8;
// non-elastic events worked by the cascade kernel, the protons it queued and
// the allowed nucleon-nucleon collisions of their cascades (flag PMC_INC)
constexpr int kCtrIncEvents = 9;
constexpr int kCtrIncSecondaries = 10;
constexpr int kCtrIncCollisions = 11;
// LDS control words of a workgroup (u32), after the deposit cache: own
// secondary queue produced / claimed / published, alive lanes at the epoch
// end, primaries exhausted, workgroup done
constexpr int kWgCtlWords = 8;
// a workgroup's own secondary queue entry: 12 u32 (px py pz ux uy uz E w
// uid_lo uid_hi group plan), 48 bytes
constexpr int kLocEntryWords = 12;
// epochs after which a workgroup stops (a guard against a non-terminating
// launch; reported as an error)
constexpr uint32_t kMaxEpochs = 1u << 21;

// LDS blob layout, in 32-bit words
constexpr int kOffLnrWater = 0;
constexpr int kOffLnrOwn = 1000;
constexpr int kOffInvWater = 2000;   // 1024 uint16 = 512 words
constexpr int kOffInvOwn = 2512;
constexpr int kOffSigma = 3024;      // n_mat x 1000 total cross section per gram
// then n_mat x 4 words: f (Eq. 1; 1 for own-table bins), X0 (g/cm^2), Z/A, own flag

// Run flag set by the engine (beside the public PMC_NO_* switches, bits 0-2)
// when LET_d is scored: the tally of a plan then holds, after its
// [nvox][k_batches] dose groups, two planes of nvox doubles: the LET
// numerator (sum of w eps L over proton steps) and the energy deposited
// outside any step (nuclear-event local deposits, sub-cut-off rests).
constexpr uint32_t kScoreLet = 1u << 8;
// Run flag of a measurement run (single plan, optional-path instantiation):
// every loop iteration each lane records the tally element its step deposited
// into, voxel * K + group (its voxel-record gather is element / K;
// 0xFFFFFFFF for no step) at trace[(epoch * epoch_iters + iteration) *
// trace_lanes + global lane], and each workgroup its epoch count; the
// roofline replay re-issues that stream.
constexpr uint32_t kTrace = 1u << 9;
// Public flag PMC_INC: a non-elastic event is written to the generation's
// event list (IncEvent) for the cascade kernel, and the proton stops.
constexpr uint32_t kInc = 64u;
constexpr uint32_t kTraceNone = 0xFFFFFFFFu;

// One plan: its geometry (voxel record = {density as float bits, material
// bin}), its dose tally and its random-number key.  64 bytes.
struct PlanDesc {
    int nx, ny, nz, pad;
    float vs[3];        // voxel size, cm
    float ivs[3];       // 1 / voxel size
    const uint2* vox;
    double* tally;      // [nvox][k_batches] weighted MeV (+ 2 x [nvox] with LET_d scoring)
    uint32_t key_lo, key_hi;
};
static_assert(sizeof(PlanDesc) == 64, "PlanDesc is 16 words");

// Arguments the step loop does not read every step: staged in LDS at the
// start of the transport kernel and read there at their use sites, so that
// they do not hold scalar registers across the loop.
struct alignas(8) LdsArgs {
    const float* el_sig;
    const float* mat_npg;
    const float* elem;
    const float* sec_mult;
    const float* sec_floc;
    const float* sec_x;
    const float* sec_mu;
    const float* spots;
    const unsigned long long* order;
    const float* vav;  // Vavilov straggling quantile table (flag PMC_VAVILOV), or NULL
    const float* mol;     // Molière sampling table (flag PMC_MOLIERE), or NULL
    const float* molmat;  // [n_mat][16] Molière material constants, or NULL
    const uint32_t* q_in;
    uint32_t* q_out;
    unsigned long long q_cap;
    double* ledger;
    unsigned long long* counters;
    uint32_t* q_loc;   // this launch's per-workgroup queues (loc_cap entries each)
    void* inc_ev;      // flag PMC_INC: this generation's event list (IncEvent entries)
    unsigned long long* inc_count;   // events recorded in it
    unsigned long long inc_cap;
    int n_spots;
    int loc_cap;
};

struct KernelArgs {
    PlanDesc single;            // the plan of a single-plan launch
    const PlanDesc* plans;      // batched launch: n_plans descriptors, staged into LDS
    int n_plans;
    int pd_offset;              // LDS word offset of the staged descriptors
    // hot tables (staged into LDS)
    const float* blob;
    int blob_words;
    int n_mat;
    float r_first[2];   // range at grid point 1 (water, own)
    float ln_r1[2];     // ln of it
    float inv_step[2];  // coarse-index cells per unit ln(range)
    // rare-path tables (global / L2)
    const float* el_sig;    // [2][7][1000] barn, process 0 elastic, 1 non-elastic
    const float* mat_npg;   // [n_mat][7] nuclei per gram per barn
    const float* elem;      // [7][8]: target mass MeV, a1, b1, a2, b2 (Eq. 3)
    const float* sec_mult;  // [6][25][5]
    const float* sec_floc;  // [6][25]
    const float* sec_x;     // [6][25][33]
    const float* sec_mu;    // [6][25][33]
    const float* vav;       // [5][31][97] Vavilov quantiles (flag PMC_VAVILOV), or NULL
    const float* mol;       // [13][161] Molière ln R (flag PMC_MOLIERE), or NULL
    const float* molmat;    // [n_mat][16] Molière material constants
    // run
    int k_batches;
    uint32_t flags;
    float f_mcs, s_min;
    // primaries (generation 0): spots[s*8 + {x/dx, y/dy, E, sx/dx, sy/dy, weight,
    // plan (bits), first index of the spot within its plan (bits)}].  They are
    // worked in batch-major order: all of statistical group 0 of every spot,
    // then group 1, ...  order[b * (n_spots + 1) + s] is the work index where
    // group b of spot s starts (entry n_spots: where group b ends), and
    // order[K * (n_spots + 1) + b * n_spots + s] the history index within its
    // plan (the random-number stream) of that part's first history
    const float* spots;
    const unsigned long long* order;
    int n_spots;
    unsigned long long n_primary;
    // secondary queues: plane p of entry i at q[p * q_cap + i]
    const uint32_t* q_in;
    uint32_t* q_out;
    unsigned long long q_cap;
    unsigned long long* gen_counters;   // [gen][2] = {entries produced for gen, entries claimed}
    int gen;
    // outputs, per plan
    double* ledger;                 // [plan][4]: escaped, neutral, overflow, deposited
    unsigned long long* counters;   // [plan][kPlanCounters]: the counters above
    int refill_lanes;
    int batch_events;
    // workgroup deposit cache in LDS: cache_slots sums (double) then as many
    // keys (tally index as uint32; in a batch of plans, plan << 32 | index as
    // uint64) at the even LDS word offset cache_off, flushed to the tallies
    // every epoch_iters loop iterations; 0 slots = off
    int cache_slots;
    int cache_off;
    // LDS word offsets of the cache keys, their LET numerators, the control
    // words and a batch's per-plan ledgers and counters (computed and checked
    // on the host with the rest of the launch layout)
    int key_off, num_off, ctl_off, led_off, cnt_off;
    int epoch_iters;
    int cache_probes;   // slots tried (linear probing) before a deposit goes to the tally
    // work claims: workgroup b of a launch of G workgroups takes its j-th
    // index from its own counter wg_claims[gen * G + b] and maps it to
    // ((j >> c) * G + b) << c | (j & (2^c - 1)), i.e. runs of 2^c consecutive
    // indices dealt round-robin; c is at most claim_log2 and small enough
    // that every workgroup gets about four runs of the generation's work
    unsigned long long* wg_claims;
    int claim_log2;
    int args_off;   // LDS word offset (even) of the staged LdsArgs
    // secondaries a workgroup emits go first to its own queue (loc_cap AoS
    // entries of kLocEntryWords at q_loc + b * loc_cap * kLocEntryWords),
    // published at the next epoch boundary and taken by its own idle lanes;
    // what does not fit goes to the next generation's queue; 0 = off
    uint32_t* q_loc;
    int loc_cap;
    // flag kTrace: the address trace (see kTrace), iterations it holds per
    // lane, lanes of the launch, and each workgroup's epoch count
    uint32_t* trace;
    unsigned long long trace_iters;
    unsigned long long trace_lanes;
    uint32_t* trace_epochs;
    // flag PMC_INC: the generation's non-elastic event list (IncEvent, 64 B
    // each), its counter and capacity
    void* inc_ev;
    unsigned long long* inc_count;
    unsigned long long inc_cap;
};

}  // namespace pmc
