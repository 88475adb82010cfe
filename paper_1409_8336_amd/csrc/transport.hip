// Transport kernels for gfx950: persistent condensed-history stepping of
// proton histories (arXiv:1409.8336, Sec. II.A.2-5 physics, Sec. II.B
// parallelisation: one history per lane), dose statistics and helpers.
//
// Design (CDNA4):
//   - one history per lane, state in registers for its whole residency;
//   - persistent waves refill idle lanes from a global claim counter (primary
//     uids in generation 0, the previous generation's secondary queue later)
//     with one atomic per wave, so lanes stay busy without any host loop;
//   - nuclear events are rare and long: lanes that reach one wait, and the
//     wave processes several of them together, then appends the emitted
//     protons to the next generation's queue with one atomic per wave;
//   - range/cross-section tables live in LDS; the voxel record is one 8-byte
//     gather; the dose is one FP64 atomic add per step into [voxel][group].
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"
#include "cache.hpp"
#include "rng.hpp"

// Multiply-adds are fused only where one source expression holds both
// (not across statements after inlining): the single-plan and batched
// instantiations then round every step identically, so a batch reproduces
// single-plan runs history by history.
#pragma clang fp contract(on)

namespace pmc {

#define DEV __device__ __forceinline__
// Pointers the kernel reads from LDS (a batch's plan table, the staged
// arguments) are generic to the compiler; casting them to the global address
// space gives global instead of flat memory instructions, which do not make
// the wave wait for its LDS operations as well.
#define GLOBAL __attribute__((address_space(1)))
// 16-byte vector for global-space loads and stores (the HIP vector types do
// not bind to address-space-qualified references)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <typename T>
DEV GLOBAL T* gbl(T* p)
{
    return (GLOBAL T*)p;
}

constexpr float kMp = 938.272088f;
constexpr float kECut = 0.1f;
constexpr float kLnE0 = -2.302585093f;            // ln 0.1
constexpr float kInvH = 999.0f / 7.824046011f;    // 1 / (ln(2500)/999)
constexpr float kH = 7.824046011f / 999.0f;
constexpr float kStraggleK = 0.156914976f;        // K m_e c^2, MeV^2 cm^2 / g
// Vavilov kappa = xi / T_max = (K/2)(Z/A) rho s / beta^2 over
// 2 m_e beta^2 gamma^2 / (1 + 2 gamma m_e/M + (m_e/M)^2); the (m_e/M)^2 term
// (3e-7) is dropped
constexpr float kVavXi = 0.150233246f;             // (K/2) / (2 m_e c^2), cm^2 / g
constexpr float kMeOverMp = 5.44617021e-4f;
constexpr float kInf = 3.0e38f;
constexpr uint32_t kMaxSteps = 1u << 20;
constexpr uint32_t kNoStraggle = 1u, kNoMcs = 2u, kNoNuclear = 4u, kVavilov = 8u, kMoliere = 16u;

// ---------------------------------------------------------------- helpers

DEV float fln(float x) { return __builtin_amdgcn_logf(x) * 0.693147181f; }
DEV float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.442695041f); }
DEV float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
DEV float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
DEV float fsin_rev(float r) { return __builtin_amdgcn_sinf(r); }   // sin(2 pi r)
DEV float fcos_rev(float r) { return __builtin_amdgcn_cosf(r); }   // cos(2 pi r)

// Inverse error function for |x| < 1 in the two-region form of Giles (2010,
// "Approximating the erfinv function"): with w = -ln(1 - x^2), erfinv(x) / x
// is a degree-8 polynomial in w - 2.5 for w < 5 and in sqrt(w) - 3 beyond.
// The coefficients are this project's least-squares fits in relative error
// (csrc/erfinv_fit.py); evaluated in FP32 the result stays within 5e-7 of
// erfinv(x) for every x = 2u - 1 that u01 can produce (4e-7 measured).
DEV float inv_erf(float x)
{
    const float w = -fln((1.f - x) * (1.f + x));
    float p;
    if (w < 5.f) {
        const float t = w - 2.5f;
        p = 2.771113862e-08f;
        p = fmaf(p, t, 3.502618917e-07f);
        p = fmaf(p, t, -3.515215773e-06f);
        p = fmaf(p, t, -4.458842729e-06f);
        p = fmaf(p, t, 2.185349323e-04f);
        p = fmaf(p, t, -1.253544576e-03f);
        p = fmaf(p, t, -4.177604915e-03f);
        p = fmaf(p, t, 2.466406246e-01f);
        p = fmaf(p, t, 1.501409398e+00f);
    } else {
        const float t = fsqrt(w) - 3.f;
        p = -1.968507892e-04f;
        p = fmaf(p, t, 8.508432244e-05f);
        p = fmaf(p, t, 1.354683624e-03f);
        p = fmaf(p, t, -3.657624243e-03f);
        p = fmaf(p, t, 5.733725080e-03f);
        p = fmaf(p, t, -7.627108717e-03f);
        p = fmaf(p, t, 9.440027455e-03f);
        p = fmaf(p, t, 1.001674451e+00f);
        p = fmaf(p, t, 2.832976890e+00f);
    }
    return p * x;
}

DEV int mbcnt(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

DEV unsigned long long bcast0(unsigned long long v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// rotate direction by polar cos/sin and azimuth phi (revolutions); a
// direction along the z axis (every primary's first step) takes the frame of
// the axes, without a branch
DEV void rotate(float& ux, float& uy, float& uz, float ct, float st, float phi)
{
    const float cp = fcos_rev(phi), sp = fsin_rev(phi);
    const float perp = fsqrt(ux * ux + uy * uy);
    const bool axial = perp < 1.0e-6f;
    const float ip = frcp(axial ? 1.f : perp);
    const float nx = ux * ct + st * (ux * uz * cp - uy * sp) * ip;
    const float ny = uy * ct + st * (uy * uz * cp + ux * sp) * ip;
    const float nz = uz * ct - st * cp * perp;
    ux = axial ? st * cp : nx;
    uy = axial ? st * sp : ny;
    uz = axial ? (uz >= 0.f ? ct : -ct) : nz;
}

// voxel containing p (voxel units); on a face, the voxel being entered
DEV bool locate_axis(float p, float d, int n, int& v)
{
    const float f = floorf(p);
    int i = (int)f;
    if (p == f && d < 0.f) --i;
    v = i;
    return i >= 0 && i < n;
}

// grid position of energy e: bin i in [0, 998] and fraction t
DEV void grid_pos(float e, int& i, float& t)
{
    const float x = (fln(e) - kLnE0) * kInvH;
    int j = (int)x;
    j = j < 0 ? 0 : (j > 998 ? 998 : j);
    float f = x - (float)j;
    f = f < 0.f ? 0.f : (f > 1.f ? 1.f : f);
    i = j;
    t = f;
}

// x at CDF value u of a 33-point table (CDF at lo + (hi - lo) i / 32, linear
// between the points): the largest i in [0, 31] with cdf[i] <= u, found in two
// rounds of independent loads (every fourth point, then the three inside the
// bracket) instead of a chain of dependent ones; the CDF is non-decreasing,
// so counting the points <= u gives the same index a bisection would
DEV float inv_cdf33(const GLOBAL float* __restrict__ cdf, float u, float lo, float hi)
{
    float c4[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) c4[i] = cdf[4 * i];
    int l = 0;
#pragma unroll
    for (int i = 1; i < 8; ++i) l += (int)(c4[i] <= u);
    l *= 4;
    const float f1 = cdf[l + 1], f2 = cdf[l + 2], f3 = cdf[l + 3];
    int k = (int)(f1 <= u) + (int)(f2 <= u) + (int)(f3 <= u);
    float c_hi = c4[l / 4 + 1];
    const float c0 = k == 0 ? c4[l / 4] : (k == 1 ? f1 : (k == 2 ? f2 : f3));
    const float c1 = k == 0 ? f1 : (k == 1 ? f2 : (k == 2 ? f3 : c_hi));
    l += k;
    const float frac = (u - c0) / (c1 - c0);
    return lo + (hi - lo) * ((float)l + frac) * (1.0f / 32.0f);
}

// ------------------------------------------------------ plan descriptors

// Geometry, tally and random-number key of the plan a particle belongs to:
// kernel arguments for a single plan, an LDS table for a batch of plans.
template <bool kMulti>
struct Plans;

template <>
struct Plans<false> {
    const KernelArgs& a;
    const PlanDesc* pd;
    DEV int nx(uint32_t) const { return a.single.nx; }
    DEV int ny(uint32_t) const { return a.single.ny; }
    DEV int nz(uint32_t) const { return a.single.nz; }
    DEV float vs(uint32_t, int i) const { return a.single.vs[i]; }
    DEV float ivs(uint32_t, int i) const { return a.single.ivs[i]; }
    DEV const uint2* vox(uint32_t) const { return a.single.vox; }
    DEV double* tally(uint32_t) const { return a.single.tally; }
    DEV uint32_t key_lo(uint32_t) const { return a.single.key_lo; }
    DEV uint32_t key_hi(uint32_t) const { return a.single.key_hi; }
};

template <>
struct Plans<true> {
    const KernelArgs& a;
    const PlanDesc* pd;
    DEV int nx(uint32_t p) const { return pd[p].nx; }
    DEV int ny(uint32_t p) const { return pd[p].ny; }
    DEV int nz(uint32_t p) const { return pd[p].nz; }
    DEV float vs(uint32_t p, int i) const { return pd[p].vs[i]; }
    DEV float ivs(uint32_t p, int i) const { return pd[p].ivs[i]; }
    DEV const uint2* vox(uint32_t p) const { return pd[p].vox; }
    DEV double* tally(uint32_t p) const { return pd[p].tally; }
    DEV uint32_t key_lo(uint32_t p) const { return pd[p].key_lo; }
    DEV uint32_t key_hi(uint32_t p) const { return pd[p].key_hi; }
};

// -------------------------------------------------------------- the kernel

// kOpt: the instantiation with the optional paths (LET_d scoring, Vavilov
// straggling, Molière scattering; each still selected by its run flag); the
// other one carries none of their code
template <bool kMulti, bool kOpt>
__global__ void __launch_bounds__(1024) transport_kernel(KernelArgs a)
{
    // all LDS is the dynamic allocation (no static __shared__ variables, so
    // that it starts at byte 0 and the cache's doubles are 8-byte aligned)
    extern __shared__ float lds[];
    for (int i = threadIdx.x; i < a.blob_words; i += blockDim.x) lds[i] = a.blob[i];
    if constexpr (kMulti) {
        uint32_t* dst = reinterpret_cast<uint32_t*>(lds + a.pd_offset);
        const uint32_t* src = reinterpret_cast<const uint32_t*>(a.plans);
        for (int i = threadIdx.x; i < a.n_plans * 16; i += blockDim.x) dst[i] = src[i];
    }
    // deposit cache at an even word offset: slot values (double), slot keys
    // (tally index; in a batch of plans, plan << 32 | tally index), with
    // LET_d scoring the slots' LET numerators (float partial sums, flushed to
    // the FP64 numerator plane), then the workgroup's control words
    using Key = std::conditional_t<kMulti, unsigned long long, uint32_t>;
    constexpr Key kEmptySlot = ~Key(0);
    const int n_slots = a.cache_slots;
    const bool use_cache = n_slots > 0;
    const bool score_let = kOpt && (a.flags & kScoreLet) != 0u;
    double* const cval = reinterpret_cast<double*>(lds + a.cache_off);
    Key* const ckey = reinterpret_cast<Key*>(lds + a.key_off);
    float* const cnum = reinterpret_cast<float*>(lds + a.num_off);
    uint32_t* const ctl = reinterpret_cast<uint32_t*>(lds + a.ctl_off);
    uint32_t* const loc_produced = ctl + 0;   // entries reserved in the own queue
    uint32_t* const loc_claimed = ctl + 1;    // entries taken by lanes
    uint32_t* const loc_avail = ctl + 2;      // entries published (written before the last epoch end)
    uint32_t* const wg_busy = ctl + 3;        // alive lanes counted at the epoch end
    uint32_t* const prim_done = ctl + 4;      // some wave found the work list exhausted
    uint32_t* const wg_done = ctl + 5;
    for (int i = threadIdx.x; i < n_slots; i += blockDim.x) {
        cval[i] = 0.0;
        ckey[i] = kEmptySlot;
        if (score_let) cnum[i] = 0.f;
    }
    if (threadIdx.x < kWgCtlWords) ctl[threadIdx.x] = 0u;
    LdsArgs* const L = reinterpret_cast<LdsArgs*>(lds + a.args_off);
    // batched launches: per-plan ledger (escaped, neutral, overflow) and
    // counters of the workgroup, accumulated in LDS and written out once at
    // the end (lanes change plan at nearly every refill of a secondary
    // generation; flushing to the same few device addresses each time
    // serialised on the memory-side atomics)
    double* const wg_led = reinterpret_cast<double*>(lds + a.led_off);
    unsigned long long* const wg_cnt = reinterpret_cast<unsigned long long*>(lds + a.cnt_off);
    if constexpr (kMulti) {
        for (int i = threadIdx.x; i < 3 * a.n_plans; i += blockDim.x) wg_led[i] = 0.0;
        for (int i = threadIdx.x; i < kWgCounters * a.n_plans; i += blockDim.x) wg_cnt[i] = 0ull;
    }
    if (threadIdx.x == 0) {
        L->el_sig = a.el_sig;
        L->mat_npg = a.mat_npg;
        L->elem = a.elem;
        L->sec_mult = a.sec_mult;
        L->sec_floc = a.sec_floc;
        L->sec_x = a.sec_x;
        L->sec_mu = a.sec_mu;
        L->vav = a.vav;
        L->mol = a.mol;
        L->molmat = a.molmat;
        L->spots = a.spots;
        L->order = a.order;
        L->q_in = a.q_in;
        L->q_out = a.q_out;
        L->q_cap = a.q_cap;
        L->ledger = a.ledger;
        L->counters = a.counters;
        L->n_spots = a.n_spots;
        L->loc_cap = a.loc_cap;
        L->q_loc = a.q_loc + (size_t)blockIdx.x * (size_t)a.loc_cap * kLocEntryWords;
        L->inc_ev = a.inc_ev;
        L->inc_count = a.inc_count;
        L->inc_cap = a.inc_cap;
    }
    __syncthreads();
    const PlanDesc* pds = reinterpret_cast<const PlanDesc*>(lds + a.pd_offset);
    const Plans<kMulti> P{a, pds};

    const uint16_t* lds16 = reinterpret_cast<const uint16_t*>(lds);
    const float* sig = lds + kOffSigma;
    const float* mc = lds + kOffSigma + 1000 * a.n_mat;

    const int lane = threadIdx.x & (kWave - 1);
    const int gen = a.gen;
    unsigned long long* const out_reserve = &a.gen_counters[2 * (gen + 1)];
    unsigned long long limit = a.n_primary;
    if (gen > 0) {
        const unsigned long long produced = a.gen_counters[2 * gen];
        limit = produced < a.q_cap ? produced : a.q_cap;
    }
    unsigned long long* const claim = &a.wg_claims[(size_t)gen * gridDim.x + blockIdx.x];
    // run length: the largest power of two up to 2^claim_log2 that still
    // gives every workgroup about four runs of this generation's work
    const unsigned long long per_wg = limit / (4ull * gridDim.x);
    uint32_t cl2 = 0;
    while (cl2 < (uint32_t)a.claim_log2 && (2ull << cl2) <= per_wg) ++cl2;
    const unsigned long long cmask = (1ull << cl2) - 1ull;
    // the workgroup's j-th claim -> index into the generation's work list
    auto claim_index = [&](unsigned long long j) {
        return ((((j >> cl2) * gridDim.x) + blockIdx.x) << cl2) | (j & cmask);
    };
    const int K = a.k_batches;
    const uint32_t flags = a.flags;

    // particle state
    float px = 0, py = 0, pz = 0, ux = 0, uy = 0, uz = 1, E = 0, mfp = 0, w = 0;
    uint32_t uid_lo = 0, uid_hi = 0, k = 0, batch = 0, plan = 0;
    int vx = 0, vy = 0, vz = 0;
    bool alive = false, pend = false;

    // per-lane ledger and counters of the lane's current plan
    double acc_esc = 0.0, acc_neu = 0.0, acc_ovf = 0.0;
    uint32_t n_steps = 0, n_el = 0, n_ne = 0, n_short = 0, n_dep = 0, n_glob = 0, n_flush = 0, n_locq = 0;
    auto flush = [&](uint32_t pl) {
        if constexpr (kMulti) {
            double* LG = wg_led + 3 * pl;
            unsigned long long* C = wg_cnt + kWgCounters * pl;
            if (acc_esc != 0.0) unsafeAtomicAdd(&LG[0], acc_esc);
            if (acc_neu != 0.0) unsafeAtomicAdd(&LG[1], acc_neu);
            if (acc_ovf != 0.0) unsafeAtomicAdd(&LG[2], acc_ovf);
            if (n_steps) atomicAdd(&C[0], (unsigned long long)n_steps);
            if (n_el) atomicAdd(&C[1], (unsigned long long)n_el);
            if (n_ne) atomicAdd(&C[2], (unsigned long long)n_ne);
            if (n_short) atomicAdd(&C[3], (unsigned long long)n_short);
            if (n_dep) atomicAdd(&C[4], (unsigned long long)n_dep);
            if (n_glob) atomicAdd(&C[5], (unsigned long long)n_glob);
            if (n_flush) atomicAdd(&C[6], (unsigned long long)n_flush);
            if (n_locq) atomicAdd(&C[7], (unsigned long long)n_locq);
            acc_esc = acc_neu = acc_ovf = 0.0;
            n_steps = n_el = n_ne = n_short = n_dep = n_glob = n_flush = n_locq = 0;
            return;
        }
        double* LG = L->ledger + 4 * pl;
        unsigned long long* C = L->counters + kPlanCounters * pl;
        if (acc_esc != 0.0) unsafeAtomicAdd(&LG[0], acc_esc);
        if (acc_neu != 0.0) unsafeAtomicAdd(&LG[1], acc_neu);
        if (acc_ovf != 0.0) unsafeAtomicAdd(&LG[2], acc_ovf);
        if (n_steps) atomicAdd(&C[0], (unsigned long long)n_steps);
        if (n_el) atomicAdd(&C[1], (unsigned long long)n_el);
        if (n_ne) atomicAdd(&C[2], (unsigned long long)n_ne);
        if (n_short) atomicAdd(&C[3], (unsigned long long)n_short);
        if (n_dep) atomicAdd(&C[4], (unsigned long long)n_dep);
        if (n_glob) atomicAdd(&C[5], (unsigned long long)n_glob);
        if (n_flush) atomicAdd(&C[6], (unsigned long long)n_flush);
        if (n_locq) atomicAdd(&C[7], (unsigned long long)n_locq);
        acc_esc = acc_neu = acc_ovf = 0.0;
        n_steps = n_el = n_ne = n_short = n_dep = n_glob = n_flush = n_locq = 0;
    };
    // one deposit into tally element idx of the current plan: through the
    // workgroup's LDS cache when the slot is free or already holds idx,
    // else straight to the FP64 tally.  With a LET_d numerator (a step's
    // deposit, idx = voxel * K + group) the numerator shares the dose's slot,
    // or goes to the numerator plane element num_idx beside it.
    auto deposit = [&](unsigned long long idx, double v, bool with_num = false, double num = 0.0,
                       unsigned long long num_idx = 0ull) {
        ++n_dep;
        if (use_cache) {
            Key key = (Key)(uint32_t)idx;
            uint32_t h = (uint32_t)idx * 0x9E3779B1u;
            if constexpr (kMulti) {
                key |= (Key)plan << 32;
                h ^= plan * 0x85EBCA6Bu;
            }
            // multiplicative hash; a slot is ours if it holds the key or we
            // claim it empty
            const int slot = cache_slot(ckey, key, h, (uint32_t)n_slots, a.cache_probes);
            if (slot >= 0) {
                unsafeAtomicAdd(&cval[slot], v);
                if (with_num) atomicAdd(&cnum[slot], (float)num);
                return;
            }
        }
        __hip_atomic_fetch_add(gbl(P.tally(plan)) + idx, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ++n_glob;
        if (with_num) {
            __hip_atomic_fetch_add(gbl(P.tally(plan)) + num_idx, num, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ++n_glob;
        }
    };
    // a deposit that belongs to no proton step (Sec. III LET_d leaves out
    // such local deposits): into the dose, and with LET_d scoring also into
    // the plane that the LET denominator subtracts from the dose
    auto deposit_local = [&](unsigned long long vi, double v) {
        deposit(vi * K + batch, v);
        if (kOpt && (flags & kScoreLet)) {
            const unsigned long long nv = (unsigned long long)P.nx(plan) * P.ny(plan) * P.nz(plan);
            deposit(nv * (K + 1) + vi, v);
        }
    };
    bool exhausted = false;
    uint32_t epoch = 0;

    // epochs: between them the workgroup flushes its deposit cache, publishes
    // the secondaries its lanes queued in its own queue and decides whether
    // it is done
    for (;;) {
    for (int it = 0; it < a.epoch_iters; ++it) {
        // ---------------------------------------------------------- refill
        // idle lanes take first the published entries of the workgroup's own
        // queue, then indices of the generation's work list
        const unsigned long long idle = __ballot(!alive);
        const int n_idle = __popcll(idle);
        if (n_idle > 0 && (n_idle == kWave || n_idle >= a.refill_lanes || exhausted)) {
            const int rank = mbcnt(idle);
            uint32_t n_sec = 0, sec_base = 0;
            if (lane == 0 && L->loc_cap > 0) {
                // claim up to n_idle published entries: compare-and-swap on the
                // LDS counter (a failed swap means another wave claimed)
                const uint32_t av = *loc_avail;
                uint32_t c = *loc_claimed;
                while (c < av) {
                    const uint32_t take = min(av - c, (uint32_t)n_idle);
                    const uint32_t prev = atomicCAS(loc_claimed, c, c + take);
                    if (prev == c) {
                        sec_base = c;
                        n_sec = take;
                        break;
                    }
                    c = prev;
                }
            }
            n_sec = __builtin_amdgcn_readfirstlane(n_sec);
            sec_base = __builtin_amdgcn_readfirstlane(sec_base);
            const int n_rest = n_idle - (int)n_sec;
            const bool take_prim = !exhausted && n_rest > 0;
            unsigned long long base = 0;
            if (take_prim) {
                if (lane == 0) base = atomicAdd(claim, (unsigned long long)n_rest);
                base = bcast0(base);
                if (claim_index(base + (unsigned long long)n_rest) >= limit) exhausted = true;
            }
            if (!alive) {
                bool got = false;
                if (rank < (int)n_sec) {
                    // a secondary of this workgroup (48-byte entry)
                    const GLOBAL u32x4* q4 = reinterpret_cast<const GLOBAL u32x4*>(
                        gbl(L->q_loc) + (size_t)(sec_base + (uint32_t)rank) * kLocEntryWords);
                    const u32x4 e0 = q4[0], e1 = q4[1], e2 = q4[2];
                    px = __uint_as_float(e0.x);
                    py = __uint_as_float(e0.y);
                    pz = __uint_as_float(e0.z);
                    ux = __uint_as_float(e0.w);
                    uy = __uint_as_float(e1.x);
                    uz = __uint_as_float(e1.y);
                    E = __uint_as_float(e1.z);
                    w = __uint_as_float(e1.w);
                    uid_lo = e2.x;
                    uid_hi = e2.y;
                    batch = e2.z;
                    if constexpr (kMulti) {
                        if (e2.w != plan) {
                            flush(plan);
                            plan = e2.w;
                        }
                    }
                    const uint4 r = philox<!kMulti>(uid_lo, uid_hi, 0u, 0u, P.key_lo(plan), P.key_hi(plan));
                    mfp = -fln(u01(r.z));
                    got = true;
                }
                const unsigned long long idx =
                    claim_index(base + (unsigned long long)(rank - (int)n_sec));
                if (!got && take_prim && idx < limit) {
                    got = true;
                    if (gen == 0) {
                        // source: Gaussian spot on the z = 0 face (K1 role).
                        // Work index -> statistical group b, then spot s within
                        // the group's part of the list, then the history.
                        // The refilled lanes of a wave take consecutive work
                        // indices (within a claim run): the first one's place
                        // is searched once for the wave (uniform, scalar
                        // code), the others step forward from it, and a lane
                        // that lands past a run boundary searches on its own.
                        const int nsp = L->n_spots;
                        const int ns1 = nsp + 1;
                        const GLOBAL unsigned long long* ord = gbl(L->order);
                        auto locate_work = [&](unsigned long long x, int& b_out, int& s_out) {
                            int b0 = 0, hb = K;
                            while (hb - b0 > 1) {
                                const int mid = (b0 + hb) >> 1;
                                if (ord[mid * ns1] <= x) b0 = mid;
                                else hb = mid;
                            }
                            const GLOBAL unsigned long long* rw = ord + b0 * ns1;
                            int s0 = 0, hs = nsp;
                            while (hs - s0 > 1) {
                                const int mid = (s0 + hs) >> 1;
                                if (rw[mid] <= x) s0 = mid;
                                else hs = mid;
                            }
                            b_out = b0;
                            s_out = s0;
                        };
                        int bg, lo;
                        locate_work(claim_index(base), bg, lo);
                        // (a run holds consecutive indices; idx < n_primary
                        // keeps the walk inside the table: the last group's
                        // row ends at n_primary)
                        for (int walk = 0; walk < 4 && idx >= ord[bg * ns1 + lo + 1]; ++walk) {
                            if (++lo == nsp) {
                                lo = 0;
                                ++bg;
                            }
                        }
                        if (idx < ord[bg * ns1 + lo] || idx >= ord[bg * ns1 + lo + 1]) locate_work(idx, bg, lo);
                        const GLOBAL unsigned long long* row = ord + bg * ns1;
                        const GLOBAL float* sp = gbl(L->spots) + 8 * lo;
                        const unsigned long long uid = ord[K * ns1 + bg * L->n_spots + lo] + (idx - row[lo]);
                        if constexpr (kMulti) {
                            const uint32_t np = __float_as_uint(sp[6]);
                            if (np != plan) {
                                flush(plan);
                                plan = np;
                            }
                        }
                        uid_lo = (uint32_t)uid;
                        uid_hi = (uint32_t)(uid >> 32);
                        const uint4 r = philox<!kMulti>(uid_lo, uid_hi, 0u, 0u, P.key_lo(plan), P.key_hi(plan));
                        const float rr = fsqrt(-2.0f * fln(u01(r.x)));
                        const float ph = u01(r.y);
                        px = sp[0] + sp[3] * rr * fcos_rev(ph);
                        py = sp[1] + sp[4] * rr * fsin_rev(ph);
                        pz = 0.f;
                        ux = 0.f;
                        uy = 0.f;
                        uz = 1.f;
                        E = sp[2];
                        w = sp[5];
                        mfp = -fln(u01(r.z));
                        batch = (uint32_t)bg;
                    } else {
                        const GLOBAL uint32_t* q = gbl(L->q_in) + idx;
                        const unsigned long long c = L->q_cap;
                        px = __uint_as_float(q[0]);
                        py = __uint_as_float(q[c]);
                        pz = __uint_as_float(q[2 * c]);
                        ux = __uint_as_float(q[3 * c]);
                        uy = __uint_as_float(q[4 * c]);
                        uz = __uint_as_float(q[5 * c]);
                        E = __uint_as_float(q[6 * c]);
                        w = __uint_as_float(q[7 * c]);
                        uid_lo = q[8 * c];
                        uid_hi = q[9 * c];
                        batch = q[10 * c];
                        if constexpr (kMulti) {
                            const uint32_t np = q[11 * c];
                            if (np != plan) {
                                flush(plan);
                                plan = np;
                            }
                        }
                        const uint4 r = philox<!kMulti>(uid_lo, uid_hi, 0u, 0u, P.key_lo(plan), P.key_hi(plan));
                        mfp = -fln(u01(r.z));
                    }
                }
                if (got) {
                    k = 0;
                    alive = locate_axis(px, ux, P.nx(plan), vx) && locate_axis(py, uy, P.ny(plan), vy) &&
                            locate_axis(pz, uz, P.nz(plan), vz);
                    if (!alive) acc_esc += (double)w * (double)E;
                }
            }
        }
        const unsigned long long busy = __ballot(alive);
        if (busy == 0) {
            // nothing to run: with the work list exhausted and nothing
            // published in the own queue, wait for the epoch end
            if (exhausted) break;
            continue;
        }

        // ------------------------------------------------------------ step
        bool stepped = false, short_step = false;
        uint32_t tr_key = kTraceNone;   // measurement trace (flag kTrace)
        if (alive && !pend) {
            const unsigned long long vi = ((unsigned long long)vz * P.ny(plan) + vy) * P.nx(plan) + vx;
            if constexpr (kOpt && !kMulti) tr_key = (uint32_t)(vi * K + batch);
            const unsigned long long rec = gbl(reinterpret_cast<const unsigned long long*>(P.vox(plan)))[vi];
            // what does not depend on the voxel record is computed while its
            // gather is in flight: the step's random numbers, the energy's
            // grid position and the distance to the voxel boundary
            const uint4 r = philox<!kMulti>(uid_lo, uid_hi, k, 1u, P.key_lo(plan), P.key_hi(plan));
            int gi;
            float gt;
            grid_pos(E, gi, gt);
            // range-table entries of both stopping tables (water-scaled and
            // the material's own): which one applies is known only from the
            // record, and reading both keeps them off the dependent chain
            const float lw0 = lds[kOffLnrWater + gi], lw1 = lds[kOffLnrWater + gi + 1];
            const float lo0 = lds[kOffLnrOwn + gi], lo1 = lds[kOffLnrOwn + gi + 1];
            float d = kInf;
            int axis = 2;
            {
                // (evaluated for every axis; one with no direction component
                // is then excluded by the selects)
                const float tx = ((float)(ux > 0.f ? vx + 1 : vx) - px) * P.vs(plan, 0) * frcp(ux);
                const float ty = ((float)(uy > 0.f ? vy + 1 : vy) - py) * P.vs(plan, 1) * frcp(uy);
                const float tz = ((float)(uz > 0.f ? vz + 1 : vz) - pz) * P.vs(plan, 2) * frcp(uz);
                const float dx = ux != 0.f ? tx : kInf;
                const float dy = uy != 0.f ? ty : kInf;
                const float dz = uz != 0.f ? tz : kInf;
                d = dx;
                axis = 0;
                if (dy < d) { d = dy; axis = 1; }
                if (dz < d) { d = dz; axis = 2; }
            }
            // an empty asm that takes the record only after those values
            // exist: it keeps the compiler from moving their arithmetic behind
            // the wait for the gather
            uint32_t rec_x = (uint32_t)rec, rec_y = (uint32_t)(rec >> 32);
            asm volatile("" : "+v"(rec_x), "+v"(rec_y) : "v"(r.x), "v"(r.y), "v"(r.z), "v"(r.w), "v"(d), "v"(gt),
                         "v"(lw0), "v"(lw1), "v"(lo0), "v"(lo1));
            const float rho = __uint_as_float(rec_x);
            const int m = (int)rec_y;
            const float mf = mc[4 * m + 0];
            const float mx0 = mc[4 * m + 1];
            const float mza = mc[4 * m + 2];
            const bool own = mc[4 * m + 3] != 0.f;
            const float scale = rho * mf;                          // Eq. 1-2
            // (table offsets selected, not pointers: the addresses stay LDS ones)
            const float* lnr = lds + (own ? kOffLnrOwn : kOffLnrWater);
            const uint16_t* inv = lds16 + 2 * (own ? kOffInvOwn : kOffInvWater);
            const float r_first = own ? a.r_first[1] : a.r_first[0];
            const float ln_r1 = own ? a.ln_r1[1] : a.ln_r1[0];
            const float inv_step = own ? a.inv_step[1] : a.inv_step[0];

            const float l_a = own ? lo0 : lw0, l_b = own ? lo1 : lw1;
            const float range_tab = fexp(l_a + gt * (l_b - l_a));
            const float range = gi == 0 ? gt * r_first : range_tab;
            const float s_range = range * frcp(scale);
            float sigma = 0.f;
            if (!(flags & kNoNuclear)) {
                const float* sm = sig + 1000 * m;
                sigma = rho * (sm[gi] + gt * (sm[gi + 1] - sm[gi]));
            }
            const float s_nuc = sigma > 0.f ? mfp * frcp(sigma) : kInf;
            bool stop_here = (s_range <= d && s_range <= s_nuc);
            const bool nuc = s_nuc < d;
            float s = nuc ? s_nuc : d;
            short_step = s < a.s_min;
            s = short_step ? a.s_min : s;
            stop_here = stop_here || s >= s_range;
            // The step is evaluated also when the range ends it (the proton
            // then deposits all of E here and its new state is discarded):
            // one path without branches around it.
            // mean loss from the range table (Eq. 2 water-equivalent path)
            const float r1 = range - s * scale;
            float e1;
            {
                const float lr = fln(fmaxf(r1, r_first));
                int c = (int)((lr - ln_r1) * inv_step);
                c = c < 0 ? 0 : (c > 1023 ? 1023 : c);
                // a coarse cell spans at most about one grid interval: two
                // unconditional advances (reads clamped into the table), then
                // a loop that practically never runs
                // j = inv[c] <= 998: the four entries j..j+3 are read at once
                // (j+2, j+3 may lie past this table's end inside the LDS
                // blob; they are used only where j + 1 < 998)
                int j = inv[c];
                const float q0 = lnr[j], q1 = lnr[j + 1], q2 = lnr[j + 2], q3 = lnr[j + 3];
                const bool adv1 = j < 998 && q1 <= lr;
                const bool adv2 = adv1 && j + 1 < 998 && q2 <= lr;
                float lo_l = adv2 ? q2 : (adv1 ? q1 : q0);
                float hi_l = adv2 ? q3 : (adv1 ? q2 : q1);
                j += (int)adv1 + (int)adv2;
                if (j < 998 && hi_l <= lr) {
                    // more than two grid intervals in one coarse cell (not
                    // the case for these tables; kept for safety)
                    while (j < 998 && lnr[j + 1] <= lr) ++j;
                    lo_l = lnr[j];
                    hi_l = lnr[j + 1];
                }
                const float tt = (lr - lo_l) * frcp(hi_l - lo_l);
                const float e_tab = fexp(kLnE0 + ((float)j + tt) * kH);
                const float e_low = fexp(kLnE0 + (r1 > 0.f ? r1 : 0.f) * frcp(r_first) * kH);
                e1 = r1 <= r_first ? e_low : e_tab;
            }
            float de_mean = E - e1;
            de_mean = de_mean > 0.f ? de_mean : 0.f;
            const float emid = E - 0.5f * de_mean;
            const float e_tot = emid + kMp;
            const float ie_tot = frcp(e_tot);
            const float pv = emid * (emid + 2.f * kMp) * ie_tot;      // p beta c
            const float b2 = pv * ie_tot;
            float de = de_mean;
            if (!(flags & kNoStraggle)) {
                const float g = e_tot * (1.0f / kMp);
                const float var = kStraggleK * rho * mza * s * g * g * (1.f - 0.5f * b2);
                float z = 1.414213562f * inv_erf(2.f * u01(r.w) - 1.f);
                if (kOpt && (flags & kVavilov)) {
                    // Vavilov-Gaussian (Sec. II.A.2): the normal score through
                    // the Vavilov quantile function of the step's kappa =
                    // xi / T_max and beta^2, tabulated at log10 kappa = -2 +
                    // j/10, beta^2 = k/10, z = -6 + i/8 (trilinear); outside
                    // kappa in [0.01, 10) the loss stays Gaussian
                    const float kappa = kVavXi * mza * rho * s * (1.f + 2.f * g * kMeOverMp) * frcp(b2 * b2 * g * g);
                    const float lk = fln(kappa) * 0.4342944819f;
                    if (lk >= -2.f && lk < 1.f) {
                        float fk = (lk + 2.f) * 10.f;
                        const int j = min((int)fk, 29);
                        fk -= (float)j;
                        float fb = fminf(fmaxf(b2, 0.f), 0.4f) * 10.f;
                        const int kb = min((int)fb, 3);
                        fb -= (float)kb;
                        float fz = (z + 6.f) * 8.f;
                        const int q = min(max((int)floorf(fz), 0), 95);
                        fz -= (float)q;
                        const GLOBAL float* t0 = gbl(L->vav) + (kb * 31 + j) * 97 + q;
                        const GLOBAL float* t1 = t0 + 31 * 97;
                        const float g00 = t0[0] + fz * (t0[1] - t0[0]);
                        const float g01 = t0[97] + fz * (t0[98] - t0[97]);
                        const float g10 = t1[0] + fz * (t1[1] - t1[0]);
                        const float g11 = t1[97] + fz * (t1[98] - t1[97]);
                        const float ga = g00 + fk * (g01 - g00), gb = g10 + fk * (g11 - g10);
                        z = ga + fb * (gb - ga);
                    }
                }
                de = de_mean + fsqrt(var) * z;
                de = de < 0.f ? 0.f : (de > E ? E : de);
            }
            float theta = 0.f;
            if (!(flags & kNoMcs)) {
                bool moliere = false;
                if (kOpt && (flags & kMoliere)) {
                    // Molière (Sec. II.A.2 option), Bethe's form: chi_c^2 =
                    // K m_e c^2 sum w Z(Z+1)/A rho s / (p beta)^2; the
                    // screening angle from the Z(Z+1)/A-weighted logs of the
                    // elements' chi_a^2 = chi_0^2 (1.13 + 3.76 (Z alpha/beta)^2);
                    // B - ln B = ln(chi_c^2 / 1.167 chi_a^2); B >= 4.5 only
                    const GLOBAL float* mm = gbl(L->molmat) + 16 * m;   // 16 floats per material
                    const float lc = fln(kStraggleK * mm[0] * rho * s) - 2.f * fln(pv);
                    const float ib2 = frcp(b2);
                    float la = mm[1] - fln(pv * e_tot);
#pragma unroll
                    for (int el = 0; el < 7; ++el) {
                        const float om = mm[2 + el];
                        if (om > 0.f) la += om * fln(1.13f + mm[9 + el] * ib2);
                    }
                    const float bb = lc - 0.154436f - la;          // ln 1.167
                    if (bb >= 2.9959226f) {                         // 4.5 - ln 4.5
                        float B = bb + fln(bb);
#pragma unroll
                        for (int it = 0; it < 4; ++it) B -= (B - fln(B) - bb) * frcp(1.f - frcp(B));
                        // reduced angle v^2 = q R(q, 1/B), q = -ln u; ln R
                        // bilinear in (1/B, q) on [1/20, 2/9] x [0, 20]
                        const float x = fminf(fmaxf(frcp(B), 0.05f), 0.2222222f);
                        float fx = (x - 0.05f) * (12.f / (0.2222222f - 0.05f));
                        const int jx = min((int)fx, 11);
                        fx -= (float)jx;
                        const float q = -fln(u01(r.y));
                        float fq = q * 8.f;
                        const int kq = min((int)fq, 159);
                        fq -= (float)kq;
                        const GLOBAL float* t0 = gbl(L->mol) + jx * 161 + kq;
                        const float ra = t0[0] + fq * (t0[1] - t0[0]);
                        const float rb = t0[161] + fq * (t0[162] - t0[161]);
                        const float v2 = q * fexp(ra + fx * (rb - ra));
                        theta = fminf(fsqrt(fexp(lc) * B * v2), 3.14159265f);
                        moliere = true;
                    }
                }
                if (!moliere) {
                    const float x0 = mx0 * frcp(rho);
                    float br = 1.f + 0.038f * fln(s * frcp(x0 * b2));
                    br = br > 0.f ? br : 0.f;
                    const float th0 = a.f_mcs * 13.6f * frcp(pv) * fsqrt(s * frcp(x0)) * br;
                    theta = th0 * fsqrt(-2.f * fln(u01(r.y)));
                }
            }
            // random hinge at a uniform fraction of the step; on a
            // boundary-limited step the second segment runs along the new
            // direction to the crossed face plane and ends on it
            const float h1 = u01(r.x) * s;
            float h2 = s - h1;
            px += h1 * ux * P.ivs(plan, 0);
            py += h1 * uy * P.ivs(plan, 1);
            pz += h1 * uz * P.ivs(plan, 2);
            const float da_before = axis == 0 ? ux : (axis == 1 ? uy : uz);
            const int va = axis == 0 ? vx : (axis == 1 ? vy : vz);
            const float face = (float)(da_before > 0.f ? va + 1 : va);
            {
                // theta = 0 (no scattering) leaves the direction as it is
                const float tr = theta * 0.159154943f;
                float nx = ux, ny = uy, nz = uz;
                rotate(nx, ny, nz, fcos_rev(tr), fsin_rev(tr), u01(r.z));
                const bool turn = theta != 0.f;
                ux = turn ? nx : ux;
                uy = turn ? ny : uy;
                uz = turn ? nz : uz;
            }
            const float da = axis == 0 ? ux : (axis == 1 ? uy : uz);
            const float pa = axis == 0 ? px : (axis == 1 ? py : pz);
            const float vsa = axis == 0 ? P.vs(plan, 0) : (axis == 1 ? P.vs(plan, 1) : P.vs(plan, 2));
            const float l2 = (face - pa) * vsa * frcp(da);
            const bool on_face = !nuc && da * da_before > 0.f && l2 >= 0.f && l2 <= 2.f * h2;
            h2 = on_face ? l2 : h2;
            px += h2 * ux * P.ivs(plan, 0);
            py += h2 * uy * P.ivs(plan, 1);
            pz += h2 * uz * P.ivs(plan, 2);
            px = on_face && axis == 0 ? face : px;
            py = on_face && axis == 1 ? face : py;
            pz = on_face && axis == 2 ? face : pz;
            const float e_new = E - de;
            // range-limited: the proton stops in this voxel with all of E
            const double dep = stop_here ? (double)w * (double)E : (double)w * ((double)E - (double)e_new);
            if (kOpt && (flags & kScoreLet)) {
                // LET_d numerator: the deposit times the medium's stopping
                // power averaged over the step's mean loss (over the residual
                // range when the range ends the step), MeV/cm
                const float l = stop_here ? (E - kECut) * frcp(s_range) : de_mean * frcp(s);
                const unsigned long long nv = (unsigned long long)P.nx(plan) * P.ny(plan) * P.nz(plan);
                deposit(vi * K + batch, dep, true, dep * (double)l, nv * K + vi);
            } else {
                deposit(vi * K + batch, dep);
            }
            if (stop_here) {
                alive = false;
            } else {
                mfp = nuc ? 0.f : fmaxf(mfp - sigma * s, 0.f);
                E = e_new;
                ++k;
                stepped = true;
                const bool inside = locate_axis(px, ux, P.nx(plan), vx) & locate_axis(py, uy, P.ny(plan), vy) &
                                    locate_axis(pz, uz, P.nz(plan), vz);
                if (E <= kECut || k >= kMaxSteps) {
                    // below the cut-off (or past the step cap that guards
                    // against non-terminating histories): deposit the rest
                    deposit_local(vi, (double)w * (double)E);
                    alive = false;
                } else if (!inside) {
                    acc_esc += (double)w * (double)E;
                    alive = false;
                } else if (nuc) {
                    pend = true;
                }
            }
        }
        n_steps += stepped;
        n_short += stepped && short_step;
        if constexpr (kOpt && !kMulti) {
            if (flags & kTrace) {
                const unsigned long long n = (unsigned long long)epoch * (unsigned)a.epoch_iters + (unsigned)it;
                if (n < a.trace_iters)
                    a.trace[n * a.trace_lanes + blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x] =
                        tr_key;
            }
        }

        // ------------------------------------------- batched nuclear events
        const unsigned long long pm = __ballot(pend);
        if (pm == 0) continue;
        {
            const int np = __popcll(pm);
            const int occ = __popcll(__ballot(alive));
            int need = occ >> 3;
            need = need < 1 ? 1 : need;
            need = need < a.batch_events ? need : a.batch_events;
            if (np < need && np < occ) continue;
        }
        int n_out = 0;
        float ce0 = 0.f, ce1 = 0.f, ce2 = 0.f, ce3 = 0.f;   // emitted energies (0 = not emitted)
        float rdx = 0.f, rdy = 0.f, rdz = 0.f;              // recoil-proton direction
        float odx = ux, ody = uy, odz = uz;                 // parent direction at the event
        float ox = px, oy = py, oz = pz;
        bool recoil = false, ev_el = false, ev_ne = false;
        uint32_t ks = k - 1u;
        int sec_row = 0;
        // flag PMC_INC: the event goes to the cascade kernel's list
        bool inc_ev = false;
        int inc_el = 0;
        float inc_t = 0.f;
        unsigned long long inc_vi = 0;
        if (pend) {
            pend = false;
            const unsigned long long vi = ((unsigned long long)vz * P.ny(plan) + vy) * P.nx(plan) + vx;
            const unsigned long long rec = gbl(reinterpret_cast<const unsigned long long*>(P.vox(plan)))[vi];
            const int m = (int)(uint32_t)(rec >> 32);
            const float T = E;
            int gi;
            float gt;
            grid_pos(T, gi, gt);
            const uint4 r3 = philox<!kMulti>(uid_lo, uid_hi, ks, 3u, P.key_lo(plan), P.key_hi(plan));
            float pe[7], pn[7];
            float s_el = 0.f, s_ne = 0.f;
#pragma unroll
            for (int e = 0; e < 7; ++e) {
                const float npg = gbl(L->mat_npg)[7 * m + e];
                const GLOBAL float* te = gbl(L->el_sig) + e * 1000;
                const GLOBAL float* tn = gbl(L->el_sig) + (7 + e) * 1000;
                pe[e] = npg > 0.f ? npg * (te[gi] + gt * (te[gi + 1] - te[gi])) : 0.f;
                pn[e] = npg > 0.f ? npg * (tn[gi] + gt * (tn[gi + 1] - tn[gi])) : 0.f;
                s_el += pe[e];
                s_ne += pn[e];
            }
            if (!(s_el + s_ne > 0.f)) {
                mfp = -fln(u01(r3.w));
            } else {
                const bool elastic = u01(r3.x) * (s_el + s_ne) < s_el;
                const float target = u01(r3.y) * (elastic ? s_el : s_ne);
                float cum = 0.f;
                int el = 0;
                bool done = false;
#pragma unroll
                for (int e = 0; e < 7; ++e) {
                    const float part = elastic ? pe[e] : pn[e];
                    if (!done && part > 0.f) {
                        el = e;
                        cum += part;
                        if (target < cum) done = true;
                    }
                }
                const uint4 r4 = philox<!kMulti>(uid_lo, uid_hi, ks, 4u, P.key_lo(plan), P.key_hi(plan));
                const GLOBAL float* ec = gbl(L->elem) + 8 * el;
                ev_el = elastic;
                ev_ne = !elastic;
                if (elastic) {
                    // Eq. 3 (A >= 2) or isotropic-CM p-p; exact two-body kinematics
                    const float bm = ec[0];
                    const float sm = (kMp + bm) * (kMp + bm) + 2.f * bm * T;
                    const float pcm2 = bm * bm * T * (T + 2.f * kMp) / sm;
                    float tabs;
                    if (el == 0) {
                        tabs = 4.f * pcm2 * (1.f - u01(r4.x));
                    } else {
                        const float tmax = 4.f * pcm2 * 1.0e-6f;
                        const float c1 = -expm1f(-ec[2] * tmax), c2 = -expm1f(-ec[4] * tmax);
                        const float w1 = ec[1] * c1 / ec[2], w2 = ec[3] * c2 / ec[4];
                        const bool first = u01(r3.z) * (w1 + w2) < w1;
                        const float b = first ? ec[2] : ec[4];
                        const float cc = first ? c1 : c2;
                        tabs = -log1pf(-u01(r4.x) * cc) / b * 1.0e6f;
                    }
                    const float trr = tabs / (2.f * bm);
                    const float tn = T - trr;
                    const float p = sqrtf(T * (T + 2.f * kMp));
                    const float pn2 = tn > 0.f ? tn * (tn + 2.f * kMp) : 0.f;
                    const float pnn = sqrtf(pn2);
                    float ct = 1.f, st = 0.f, cr = 1.f, sr = 0.f;
                    if (pnn > 0.f && trr > 0.f) {
                        const float dp = trr * (T + tn + 2.f * kMp) / (p + pnn);
                        const float q2 = trr * (trr + 2.f * bm);
                        float omc = (q2 - dp * dp) / (2.f * p * pnn);
                        omc = omc < 0.f ? 0.f : (omc > 2.f ? 2.f : omc);
                        ct = 1.f - omc;
                        st = sqrtf(omc * (2.f - omc));
                        const float pr = sqrtf(q2);
                        cr = (dp + pnn * omc) / pr;
                        sr = pnn * st / pr;
                    }
                    const float phi = u01(r4.y);
                    const float tn_f = tn;
                    const float tr_f = T - tn_f;
                    if (el == 0 && tr_f > kECut) {
                        recoil = true;
                        ce0 = tr_f;
                        n_out = 1;
                        rdx = ux;
                        rdy = uy;
                        rdz = uz;
                        rotate(rdx, rdy, rdz, cr, sr, phi + 0.5f);
                        const double resid = (double)T - (double)tn_f - (double)tr_f;
                        if (resid != 0.0) {
                            deposit_local(vi, (double)w * resid);
                        }
                    } else {
                        deposit_local(vi, (double)w * ((double)T - (double)tn_f));
                    }
                    rotate(ux, uy, uz, ct, st, phi);
                    E = tn_f;
                    if (E <= kECut) {
                        deposit_local(vi, (double)w * (double)E);
                        alive = false;
                    } else {
                        mfp = -fln(u01(r3.w));
                    }
                } else if (kOpt && (flags & kInc)) {
                    // non-elastic, intranuclear cascade: the event is listed
                    // for the cascade kernel, which emits the secondaries
                    inc_ev = true;
                    inc_el = el;
                    inc_t = T;
                    inc_vi = vi;
                    alive = false;
                } else {
                    // non-elastic: secondary protons from the per-nucleus table
                    const int nu = el - 1;
                    int j = (int)(T * 0.1f);
                    j = j > 24 ? 24 : j;
                    const int row = nu * 25 + j;
                    sec_row = row;
                    const GLOBAL float* mc5 = gbl(L->sec_mult) + 5 * row;
                    const float um = u01(r4.x);
                    int n = 0;
                    while (n < 4 && !(um < mc5[n])) ++n;
                    const float fl = gbl(L->sec_floc)[row];
                    const GLOBAL float* xr = gbl(L->sec_x) + 33 * row;
                    float sum = 0.f;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        float ev = 0.f;
                        if (c < n) {
                            const uint4 rc = philox<!kMulti>(uid_lo, uid_hi, ks, 17u + c, P.key_lo(plan), P.key_hi(plan));
                            ev = inv_cdf33(xr, u01(rc.x), 0.f, 1.f) * T;
                        }
                        if (c == 0) ce0 = ev;
                        if (c == 1) ce1 = ev;
                        if (c == 2) ce2 = ev;
                        if (c == 3) ce3 = ev;
                        sum += ev;
                    }
                    const float avail = (1.f - fl) * T;
                    if (sum > avail) {
                        const float rs = avail / sum;
                        ce0 *= rs;
                        ce1 *= rs;
                        ce2 *= rs;
                        ce3 *= rs;
                    }
                    const double loc = (double)fl * (double)T;
                    double local = loc;
                    const double carried = (double)ce0 + (double)ce1 + (double)ce2 + (double)ce3;
                    if (n > 0 && ce0 <= kECut) { local += ce0; ce0 = 0.f; }
                    if (n > 1 && ce1 <= kECut) { local += ce1; ce1 = 0.f; }
                    if (n > 2 && ce2 <= kECut) { local += ce2; ce2 = 0.f; }
                    if (n > 3 && ce3 <= kECut) { local += ce3; ce3 = 0.f; }
                    n_out = (ce0 > 0.f) + (ce1 > 0.f) + (ce2 > 0.f) + (ce3 > 0.f);
                    deposit_local(vi, (double)w * local);
                    acc_neu += (double)w * ((double)T - loc - carried);
                    alive = false;
                }
            }
        }
        n_el += ev_el;
        n_ne += ev_ne;
        if constexpr (kOpt) {
            // the wave's cascade events to the generation's list, one
            // reservation per wave
            const unsigned long long bm = __ballot(inc_ev);
            if (bm != 0ull) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(L->inc_count, (unsigned long long)__popcll(bm));
                base = bcast0(base);
                if (inc_ev) {
                    const unsigned long long idx = base + (unsigned long long)mbcnt(bm);
                    if (idx < L->inc_cap) {
                        GLOBAL u32x4* e4 = reinterpret_cast<GLOBAL u32x4*>(
                            reinterpret_cast<GLOBAL unsigned char*>(gbl(L->inc_ev)) + idx * 64ull);
                        e4[0] = u32x4{__float_as_uint(ox), __float_as_uint(oy), __float_as_uint(oz),
                                      __float_as_uint(odx)};
                        e4[1] = u32x4{__float_as_uint(ody), __float_as_uint(odz), __float_as_uint(inc_t),
                                      __float_as_uint(w)};
                        e4[2] = u32x4{uid_lo, uid_hi, batch, plan};
                        e4[3] = u32x4{ks, (uint32_t)inc_el, (uint32_t)inc_vi, (uint32_t)(inc_vi >> 32)};
                    } else {
                        acc_ovf += (double)w * (double)inc_t;
                    }
                }
            }
        }
        // append emitted protons: to the workgroup's own queue (entries
        // lbase + i while below its capacity), what does not fit to the next
        // generation's queue
        {
            const unsigned long long b0 = __ballot(n_out & 1), b1 = __ballot(n_out & 2),
                                     b2 = __ballot(n_out & 4);
            const int total = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
            if (total == 0) continue;
            const int off = mbcnt(b0) + 2 * mbcnt(b1) + 4 * mbcnt(b2);
            const uint32_t lcap = (uint32_t)L->loc_cap;
            uint32_t lbase = 0;
            if (lane == 0 && lcap > 0) lbase = atomicAdd(loc_produced, (uint32_t)total);
            lbase = __builtin_amdgcn_readfirstlane(lbase);
            const uint32_t first_over = lcap > lbase ? lcap : lbase;
            const uint32_t end = lbase + (uint32_t)total;
            const uint32_t n_over = end > first_over ? end - first_over : 0u;
            unsigned long long gbase = 0;
            if (n_over > 0) {
                if (lane == 0) gbase = atomicAdd(out_reserve, (unsigned long long)n_over);
                gbase = bcast0(gbase);
            }
            if (n_out > 0) {
                uint32_t li = lbase + (uint32_t)off;
                const unsigned long long cap = L->q_cap;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float ev = c == 0 ? ce0 : (c == 1 ? ce1 : (c == 2 ? ce2 : ce3));
                    if (ev > 0.f) {
                        float dx = rdx, dy = rdy, dz = rdz;
                        const uint32_t jj = recoil ? 0u : (uint32_t)(c + 1);
                        if (!recoil) {
                            const uint4 rc = philox<!kMulti>(uid_lo, uid_hi, ks, 16u + jj, P.key_lo(plan), P.key_hi(plan));
                            const float mu = inv_cdf33(gbl(L->sec_mu) + 33 * sec_row, u01(rc.y), -1.f, 1.f);
                            dx = odx;
                            dy = ody;
                            dz = odz;
                            rotate(dx, dy, dz, mu, sqrtf(fmaxf(0.f, 1.f - mu * mu)), u01(rc.z));
                        }
                        const uint4 cu = philox<!kMulti>(uid_lo, uid_hi, ks, 0xC0000000u | jj, P.key_lo(plan),
                                                P.key_hi(plan));
                        const unsigned long long slot = gbase + (unsigned long long)(li - first_over);
                        if (li < lcap) {
                            GLOBAL u32x4* q4 = reinterpret_cast<GLOBAL u32x4*>(gbl(L->q_loc) +
                                                                               (size_t)li * kLocEntryWords);
                            q4[0] = u32x4{__float_as_uint(ox), __float_as_uint(oy), __float_as_uint(oz),
                                          __float_as_uint(dx)};
                            q4[1] = u32x4{__float_as_uint(dy), __float_as_uint(dz), __float_as_uint(ev),
                                          __float_as_uint(w)};
                            q4[2] = u32x4{cu.x, cu.y, batch, plan};
                            ++n_locq;
                        } else if (slot < cap) {
                            GLOBAL uint32_t* q = gbl(L->q_out) + slot;
                            q[0] = __float_as_uint(ox);
                            q[cap] = __float_as_uint(oy);
                            q[2 * cap] = __float_as_uint(oz);
                            q[3 * cap] = __float_as_uint(dx);
                            q[4 * cap] = __float_as_uint(dy);
                            q[5 * cap] = __float_as_uint(dz);
                            q[6 * cap] = __float_as_uint(ev);
                            q[7 * cap] = __float_as_uint(w);
                            q[8 * cap] = cu.x;
                            q[9 * cap] = cu.y;
                            q[10 * cap] = batch;
                            q[11 * cap] = plan;
                        } else {
                            acc_ovf += (double)w * (double)ev;
                        }
                        ++li;
                    }
                }
            }
        }
    }   // iterations of one epoch
    // epoch end: every wave reports its alive lanes (pending events
    // included) and whether it found the work list exhausted
    {
        const int n_alive = __popcll(__ballot(alive));
        if (lane == 0) {
            if (n_alive > 0) atomicAdd(wg_busy, (uint32_t)n_alive);
            if (exhausted) *prim_done = 1u;
        }
    }
    ++epoch;
    __syncthreads();
    // write the epoch's cached sums to the tally and clear the cache
    for (int i = threadIdx.x; i < n_slots; i += blockDim.x) {
        const Key key = ckey[i];
        if (key != kEmptySlot) {
            if constexpr (kMulti)
                __hip_atomic_fetch_add(gbl(P.tally((uint32_t)(key >> 32))) + (uint32_t)key, cval[i], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            else unsafeAtomicAdd(&a.single.tally[key], cval[i]);
            ++n_glob;
            ++n_flush;
            if (score_let) {
                // the slot's LET numerator, if it held step deposits (key =
                // voxel * K + group), to element voxel of the numerator plane
                const float nm = cnum[i];
                if (nm != 0.f) {
                    const uint32_t pk = kMulti ? (uint32_t)(key >> 32) : 0u;
                    const uint32_t t = (uint32_t)key;
                    const unsigned long long nv = (unsigned long long)P.nx(pk) * P.ny(pk) * P.nz(pk);
                    __hip_atomic_fetch_add(gbl(P.tally(pk)) + nv * K + t / (uint32_t)K, (double)nm,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ++n_glob;
                    ++n_flush;
                }
                cnum[i] = 0.f;
            }
            ckey[i] = kEmptySlot;
            cval[i] = 0.0;
        }
    }
    // publish what the lanes queued this epoch (written before the barrier
    // above); the workgroup is done when the work list is exhausted, no lane
    // is alive and every published entry has been taken
    if (threadIdx.x == 0) {
        const uint32_t lcap = (uint32_t)L->loc_cap;
        const uint32_t prod = min(*loc_produced, lcap);
        *loc_avail = prod;
        const bool done = *prim_done != 0u && *wg_busy == 0u && *loc_claimed >= prod;
        const bool stop = !done && epoch >= kMaxEpochs;
        if (stop) atomicAdd(&L->counters[kCtrAborted], 1ull);
        *wg_done = (done || stop) ? 1u : 0u;
        *wg_busy = 0u;
    }
    __syncthreads();
    if (*wg_done) break;
    }   // epochs

    if constexpr (kOpt && !kMulti) {
        if ((flags & kTrace) && threadIdx.x == 0) a.trace_epochs[blockIdx.x] = epoch;
    }
    // -------------------------------------------------- flush the ledger
    if constexpr (kMulti) {
        flush(plan);
        __syncthreads();
        for (int i = threadIdx.x; i < 3 * a.n_plans; i += blockDim.x) {
            const int pl = i / 3, f = i - 3 * pl;
            if (wg_led[i] != 0.0) unsafeAtomicAdd(&L->ledger[4 * pl + f], wg_led[i]);
        }
        for (int i = threadIdx.x; i < kWgCounters * a.n_plans; i += blockDim.x) {
            const int pl = i / kWgCounters, f = i - kWgCounters * pl;
            if (wg_cnt[i] != 0ull) atomicAdd(&L->counters[kPlanCounters * pl + f], wg_cnt[i]);
        }
    } else {
        for (int o = 32; o > 0; o >>= 1) {
            acc_esc += __shfl_xor(acc_esc, o);
            acc_neu += __shfl_xor(acc_neu, o);
            acc_ovf += __shfl_xor(acc_ovf, o);
            n_steps += __shfl_xor(n_steps, o);
            n_el += __shfl_xor(n_el, o);
            n_ne += __shfl_xor(n_ne, o);
            n_short += __shfl_xor(n_short, o);
            n_dep += __shfl_xor(n_dep, o);
            n_glob += __shfl_xor(n_glob, o);
            n_flush += __shfl_xor(n_flush, o);
            n_locq += __shfl_xor(n_locq, o);
        }
        if (lane == 0) flush(0);
    }
}

// Achievable-rate probe for the tally atomics: every lane walks straight
// tracks along z from lateral starts inside the central 40x40-voxel window of
// the loaded grid (the footprint of a treatment field), adding 0 into
// tally[voxel][lane % K] once per voxel, the same FP64 atomic the transport
// issues per step.  Adding 0 leaves the tally unchanged.
__global__ void __launch_bounds__(256) atomic_probe_kernel(double* tally, int nx, int ny, int nz,
                                                           int K, unsigned long long per_lane)
{
    const unsigned gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t s = 2654435761u * gid + 12345u;
    const int b = (int)(gid % (unsigned)K);
    const int wx = nx < 40 ? nx : 40, wy = ny < 40 ? ny : 40;
    const int x0 = (nx - wx) / 2, y0 = (ny - wy) / 2;
    int x = 0, y = 0, z = nz;
    for (unsigned long long i = 0; i < per_lane; ++i) {
        if (z >= nz) {
            s = s * 1664525u + 1013904223u;
            x = x0 + (int)((s >> 8) % (uint32_t)wx);
            s = s * 1664525u + 1013904223u;
            y = y0 + (int)((s >> 8) % (uint32_t)wy);
            z = 0;
        }
        const unsigned long long v = ((unsigned long long)z * ny + y) * nx + x;
        unsafeAtomicAdd(&tally[v * K + b], 0.0);
        ++z;
    }
}

hipError_t launch_atomic_probe(double* tally, int nx, int ny, int nz, int K, int grid,
                               unsigned long long per_lane, hipStream_t st)
{
    hipLaunchKernelGGL(atomic_probe_kernel, dim3(grid), dim3(256), 0, st, tally, nx, ny, nz, K, per_lane);
    return hipGetLastError();
}

// dose statistics over the K groups: total, variance of the total, and the
// deposited-energy sum (Sec. II.B.2); with LET_d scoring also the LET_d of
// every voxel from the two planes after the groups
// A block takes kStatsVox consecutive voxels at a time: their [voxel][K]
// tally rows form one contiguous run, read with 16-byte unit-stride loads
// into LDS rows padded to an odd number of doubles (fewer bank conflicts),
// then each lane reduces its voxel's K groups from LDS.  With kPre (K <= 16:
// a run is at most kStatsPre 16-byte loads per lane) the next run's loads are
// issued into registers before the current run is reduced, so that they are
// in flight during the reduction.
constexpr int kStatsVox = 128;
constexpr int kStatsPre = 8;
template <bool kPre>
__global__ void __launch_bounds__(kStatsVox) stats_kernel(const double* __restrict__ tally,
                                                          const uint2* __restrict__ vox,
                                                          unsigned long long nvox, int K, uint32_t k_magic,
                                                          double inv_k, double k_ratio, double conv0,
                                                          double* __restrict__ dose,
                                                          double* __restrict__ var, double* dep_sum,
                                                          const double* __restrict__ let_nd,
                                                          double* __restrict__ let)
{
    extern __shared__ double rows[];   // kStatsVox * (K | 1)
    const int pitch = K | 1;
    const unsigned long long stride = (unsigned long long)gridDim.x * kStatsVox;
    double part = 0.0;
    // element e of a run lies in row e / K, computed as a high product with
    // k_magic = ceil(2^32 / K) (exact for e < 2^32 / K^2, here e < 8192)
    auto put = [&](int i, const double2& q) {
        const uint32_t e0 = 2u * (uint32_t)i, e1 = e0 + 1u;
        const uint32_t r0 = __umulhi(e0, k_magic), r1 = __umulhi(e1, k_magic);
        rows[r0 * pitch + (e0 - r0 * K)] = q.x;
        rows[r1 * pitch + (e1 - r1 * K)] = q.y;
    };
    // pairs of doubles of the run that starts at voxel w (16-byte aligned:
    // it starts at w * K doubles, w a multiple of kStatsVox)
    auto pairs = [&](unsigned long long w) {
        const unsigned long long left = nvox - w;
        return ((left < (unsigned long long)kStatsVox ? (int)left : kStatsVox) * K) >> 1;
    };
    double2 pre[kPre ? kStatsPre : 1];
    if (kPre && blockIdx.x * (unsigned long long)kStatsVox < nvox) {
        const unsigned long long w = blockIdx.x * (unsigned long long)kStatsVox;
        const double2* src2 = reinterpret_cast<const double2*>(tally + w * K);
        const int np = pairs(w);
#pragma unroll
        for (int j = 0; j < (kPre ? kStatsPre : 1); ++j) {
            const int i = (int)threadIdx.x + j * kStatsVox;
            if (i < np) pre[j] = src2[i];
        }
    }
    for (unsigned long long v0 = blockIdx.x * (unsigned long long)kStatsVox; v0 < nvox; v0 += stride) {
        const unsigned long long left = nvox - v0;
        const int nv = left < (unsigned long long)kStatsVox ? (int)left : kStatsVox;
        const int n = nv * K;                      // doubles in this run
        // the voxel's record is read before the barrier, off the dependent path
        const unsigned long long v = v0 + threadIdx.x;
        const float rho = (int)threadIdx.x < nv ? __uint_as_float(vox[v].x) : 1.f;
        __syncthreads();
        if (kPre) {
#pragma unroll
            for (int j = 0; j < (kPre ? kStatsPre : 1); ++j) {
                const int i = (int)threadIdx.x + j * kStatsVox;
                if (i < (n >> 1)) put(i, pre[j]);
            }
        } else {
            const double2* src2 = reinterpret_cast<const double2*>(tally + v0 * K);
            for (int i = threadIdx.x; i < (n >> 1); i += kStatsVox) put(i, src2[i]);
        }
        if ((n & 1) && threadIdx.x == 0) rows[((n - 1) / K) * pitch + (n - 1) % K] = tally[v0 * K + n - 1];
        __syncthreads();
        if (kPre && v0 + stride < nvox) {
            // the next run's loads, in flight while this run is reduced
            const unsigned long long w = v0 + stride;
            const double2* src2 = reinterpret_cast<const double2*>(tally + w * K);
            const int np = pairs(w);
#pragma unroll
            for (int j = 0; j < (kPre ? kStatsPre : 1); ++j) {
                const int i = (int)threadIdx.x + j * kStatsVox;
                if (i < np) pre[j] = src2[i];
            }
        }
        if ((int)threadIdx.x >= nv) continue;
        const double* t = rows + threadIdx.x * pitch;
        double tot = 0.0;
        for (int b = 0; b < K; ++b) tot += t[b];
        const double mean = tot * inv_k;
        double ss = 0.0;
        for (int b = 0; b < K; ++b) {
            const double dd = t[b] - mean;
            ss += dd * dd;
        }
        // conv0 / rho: an FP32 reciprocal refined by two Newton steps in FP64
        const double rd = (double)rho;
        double ir = (double)frcp(rho);
        ir = ir * (2.0 - rd * ir);
        ir = ir * (2.0 - rd * ir);
        const double conv = conv0 * ir;
        dose[v] = tot * conv;
        if (var) var[v] = k_ratio * ss * conv * conv;
        part += tot;
        if (let) {
            // LET_d (keV/um; 1 MeV/cm = 0.1 keV/um): numerator over the
            // energy of the proton steps, i.e. the dose minus what was
            // deposited outside any step
            const double num = let_nd[v], den = tot - let_nd[nvox + v];
            let[v] = (num > 0.0 && den > 0.0) ? 0.1 * num / den : 0.0;
        }
    }
    // one atomic per workgroup: the workgroups' partial sums all go to one
    // address, where memory-side atomics serialise (one per wave of 65536
    // workgroups took most of the kernel's time)
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) rows[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < kStatsVox / 64; ++w) sum += rows[w];
        if (sum != 0.0) unsafeAtomicAdd(dep_sum, sum);
    }
}

__global__ void density_kernel(const uint2* __restrict__ vox, unsigned long long nvox, float* __restrict__ rho)
{
    for (unsigned long long v = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; v < nvox;
         v += (unsigned long long)gridDim.x * blockDim.x)
        rho[v] = __uint_as_float(vox[v].x);
}

__global__ void zero_kernel(unsigned long long* __restrict__ p, unsigned long long n)
{
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// ------------------------------------------------------------- launchers

namespace {
// the instantiation for a launch: batched or not, with the optional paths if
// any of their flags is set
const void* kernel_for(bool multi, bool opt)
{
    if (multi) return opt ? (const void*)transport_kernel<true, true> : (const void*)transport_kernel<true, false>;
    return opt ? (const void*)transport_kernel<false, true> : (const void*)transport_kernel<false, false>;
}
}  // namespace

bool transport_needs_options(uint32_t flags)
{
    return (flags & (kScoreLet | kVavilov | kMoliere | kTrace | kInc)) != 0u;
}

hipError_t launch_transport(const KernelArgs& a, bool multi, int grid, int block, size_t lds_bytes,
                            hipStream_t s)
{
    const bool opt = transport_needs_options(a.flags);
    if (multi) {
        if (opt) hipLaunchKernelGGL((transport_kernel<true, true>), dim3(grid), dim3(block), lds_bytes, s, a);
        else hipLaunchKernelGGL((transport_kernel<true, false>), dim3(grid), dim3(block), lds_bytes, s, a);
    } else {
        if (opt) hipLaunchKernelGGL((transport_kernel<false, true>), dim3(grid), dim3(block), lds_bytes, s, a);
        else hipLaunchKernelGGL((transport_kernel<false, false>), dim3(grid), dim3(block), lds_bytes, s, a);
    }
    return hipGetLastError();
}

hipError_t transport_max_block(bool multi, uint32_t flags, int* max_threads)
{
    hipFuncAttributes attr;
    const void* f = kernel_for(multi, transport_needs_options(flags));
    hipError_t e = hipFuncGetAttributes(&attr, f);
    if (e != hipSuccess) return e;
    // the LDS layout assumes the dynamic allocation starts at byte 0
    if (attr.sharedSizeBytes != 0) return hipErrorInvalidConfiguration;
    *max_threads = attr.maxThreadsPerBlock;
    return hipSuccess;
}

hipError_t transport_occupancy(bool multi, uint32_t flags, int block, size_t lds_bytes, int* blocks_per_cu)
{
    const void* f = kernel_for(multi, transport_needs_options(flags));
    if (lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, block, lds_bytes);
}

hipError_t launch_stats(const double* tally, const uint2* vox, unsigned long long nvox, int K,
                        double conv0, double* dose, double* var, double* dep_sum, double* let,
                        hipStream_t s)
{
    if (K < 2 || K > 64) return hipErrorInvalidValue;
    const size_t bytes = (size_t)kStatsVox * (K | 1) * sizeof(double);
    // registers hold a whole run when it is at most kStatsPre loads per lane
    const bool pre = (size_t)kStatsVox * K / 2 <= (size_t)kStatsPre * kStatsVox;
    if (bytes > 65536) {
        const hipError_t ea = hipFuncSetAttribute(pre ? (const void*)stats_kernel<true> : (const void*)stats_kernel<false>,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (ea != hipSuccess) return ea;
    }
    // as many workgroups as are resident at once (a second, partial wave of
    // workgroups would run after the first), each looping over runs of voxels
    const void* kfn = pre ? (const void*)stats_kernel<true> : (const void*)stats_kernel<false>;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kStatsVox, bytes);
    if (e != hipSuccess) return e;
    const unsigned long long resident = (unsigned long long)std::max(1, cus) * (unsigned long long)std::max(1, per_cu);
    unsigned long long blocks = (nvox + kStatsVox - 1) / kStatsVox;
    if (blocks > resident) blocks = resident;
    if (blocks == 0) blocks = 1;
    const uint32_t k_magic = (uint32_t)((0x100000000ull + (unsigned)K - 1) / (unsigned)K);
    const double* let_nd = let ? tally + nvox * (unsigned long long)K : nullptr;
    if (pre)
        hipLaunchKernelGGL(stats_kernel<true>, dim3((unsigned)blocks), dim3(kStatsVox), bytes, s, tally, vox, nvox, K,
                           k_magic, 1.0 / K, (double)K / (K - 1), conv0, dose, var, dep_sum, let_nd, let);
    else
        hipLaunchKernelGGL(stats_kernel<false>, dim3((unsigned)blocks), dim3(kStatsVox), bytes, s, tally, vox, nvox, K,
                           k_magic, 1.0 / K, (double)K / (K - 1), conv0, dose, var, dep_sum, let_nd, let);
    return hipGetLastError();
}

hipError_t launch_density(const uint2* vox, unsigned long long nvox, float* rho, hipStream_t s)
{
    unsigned long long blocks = (nvox + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(density_kernel, dim3((unsigned)blocks), dim3(256), 0, s, vox, nvox, rho);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s)
{
    const unsigned long long n = bytes / 8;
    if (n == 0) return hipSuccess;
    unsigned long long blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       (unsigned long long*)p, n);
    return hipGetLastError();
}

}  // namespace pmc
