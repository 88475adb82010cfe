// C ABI of the engine (include/pmc.h): context and device-buffer ownership,
// uploads of nuclear data and geometries, the autotuner and the run driver
// that launches one persistent transport grid per secondary generation
// followed by the dose-statistics pass (arXiv:1409.8336, Sec. II.B.2-3).
// A single-plan run and a batch of plans share the driver; a batch runs in
// one persistent launch per generation with per-plan tallies and ledgers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "device.hpp"
#include "inc.hpp"
#include "layout.hpp"
#include "pmc.h"
#include "tables.hpp"

namespace pmc {
hipError_t launch_transport(const KernelArgs& a, bool multi, int grid, int block, size_t lds_bytes,
                            hipStream_t s);
hipError_t transport_occupancy(bool multi, uint32_t flags, int block, size_t lds_bytes, int* blocks_per_cu);
hipError_t transport_max_block(bool multi, uint32_t flags, int* max_threads);
hipError_t launch_stats(const double* tally, const uint2* vox, unsigned long long nvox, int K,
                        double conv0, double* dose, double* var, double* dep_sum, double* let,
                        hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_density(const uint2* vox, unsigned long long nvox, float* rho, hipStream_t s);
hipError_t launch_atomic_probe(double* tally, int nx, int ny, int nz, int K, int grid,
                               unsigned long long per_lane, hipStream_t st);
hipError_t launch_replay(int mode, const uint32_t* trace, unsigned long long trace_iters, unsigned long long lanes,
                         const uint32_t* epochs, int epoch_iters, int K, const uint2* vox, double* tally,
                         int n_slots, int probes, int grid, int block, unsigned long long* sink, hipStream_t st);
hipError_t launch_stream_read(const void* p, size_t bytes, unsigned long long* sink, int grid, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, int grid, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, unsigned long long n, uint32_t v, hipStream_t st);
hipError_t launch_count_steps(const uint32_t* trace, unsigned long long n, unsigned long long* out, hipStream_t st);
hipError_t launch_inc_transport(const IncLaunch& a, int grid, hipStream_t st);
hipError_t inc_transport_occupancy(int* blocks_per_cu);
hipError_t launch_inc_inspect(const IncNucleus* nuclei, const IncTab* tab, const int32_t* element, const double* t,
                              const unsigned long long* uid, const uint32_t* ks, int n, uint64_t seed, int evap,
                              unsigned long long* ctr, IncResult* res, IncParticle* out, hipStream_t st);
}  // namespace pmc

using namespace pmc;

namespace {

thread_local std::string g_create_error;

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t count)
    {
        if (count <= n && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) n = std::max<size_t>(count, 1);
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { release(); }
};

struct Geometry {
    int nx = 0, ny = 0, nz = 0;
    float vs[3] = {0, 0, 0};
    DevBuf<uint2> vox;
    DevBuf<double> tally;        // [nvox][K] for runs on this geometry
    size_t nvox() const { return (size_t)nx * ny * nz; }
};

// launch shape chosen by the autotuner (or fixed by the caller)
struct Shape {
    int block = 256, blocks_per_cu = 0, refill = 16, batch = 4;
    int cache = 0;   // deposit cache when the caller leaves it automatic: 0 sized from LDS, -1 off
};

// one plan of a run, host side
struct PlanIn {
    Geometry* g;
    const pmc_spot* spots;
    int n_spots;
    unsigned long long n_hist;
    uint64_t seed;
    double* d_dose;
    double* d_var;
    pmc_summary* summary;
    double* d_let;   // LET_d output (nvox doubles) or NULL
};

}  // namespace

struct pmc_ctx {
    int device = 0;
    pmc_params p{};
    std::string err;
    int num_cu = 0;
    bool have_phys = false;
    // host copies of the nuclear data
    std::vector<float> sig_el, sig_ne, mult, floc, xcdf, mucdf;
    // host tables
    RangeTable water, own;
    std::vector<Material> mats;
    std::vector<float> blob;
    int own_bin = -1;
    // geometries: slot 0 is pmc_load_geometry's, slots >= 1 from pmc_load_geometry_slot
    std::vector<std::unique_ptr<Geometry>> geoms;
    // device tables
    DevBuf<float> d_blob, d_el_sig, d_npg, d_elem, d_mult, d_floc, d_xcdf, d_mucdf;
    // run buffers
    DevBuf<double> d_dose, d_var, d_let, d_ledger;
    DevBuf<float> d_vav;       // Vavilov quantile table (PMC_VAVILOV)
    DevBuf<float> d_mol, d_molmat;  // Molière table and material constants (PMC_MOLIERE)
    DevBuf<uint32_t> d_q[2];
    DevBuf<unsigned long long> d_gc, d_counters, d_order, d_wgc;
    DevBuf<uint32_t> d_qloc;   // per-workgroup secondary queues
    DevBuf<float> d_spots;
    DevBuf<PlanDesc> d_plans;
    DevBuf<uint32_t> d_trace, d_trace_epochs;   // roofline replay: address trace (kTrace)
    // intranuclear cascade (PMC_INC): the six target nuclei, the event list
    // of a generation (IncEvent) and each generation's event count
    DevBuf<IncNucleus> d_inc_nuc;
    DevBuf<IncTab> d_inc_tab;
    DevBuf<IncEvent> d_inc_ev;
    DevBuf<unsigned long long> d_inc_count;
    int inc_grid = 0;
    hipEvent_t ev_inc[2 * kMaxGenerations] = {};
    DevBuf<unsigned long long> d_sink;
    unsigned long long* h_pinned = nullptr;   // pinned read-back area
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_gen[2 * kMaxGenerations] = {};
    std::map<std::tuple<int, int, int, int>, Shape> tuned;   // workload signature -> shape
};

namespace {

constexpr size_t kPinnedBytes = 65536;
constexpr int kGenGroup = 6;   // generations launched per host synchronisation

pmc_status fail(pmc_ctx* c, pmc_status s, const std::string& msg)
{
    if (c) c->err = msg;
    return s;
}

pmc_status hip_fail(pmc_ctx* c, hipError_t e, const char* what)
{
    return fail(c, e == hipErrorOutOfMemory ? PMC_ERR_NOMEM : PMC_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr, what)                                      \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return hip_fail(c, _e, what);     \
    } while (0)

bool have_geometry(const pmc_ctx* c) { return !c->geoms.empty() && c->geoms[0] && c->geoms[0]->nx > 0; }

// the hot tables staged into LDS by every transport workgroup
void build_blob(pmc_ctx* c)
{
    const int nm = (int)c->mats.size();
    c->blob.assign(kOffSigma + 1000 * nm + 4 * nm, 0.f);
    const RangeTable& own = c->own_bin >= 0 ? c->own : c->water;
    std::copy(c->water.lnr.begin(), c->water.lnr.end(), c->blob.begin() + kOffLnrWater);
    std::copy(own.lnr.begin(), own.lnr.end(), c->blob.begin() + kOffLnrOwn);
    std::memcpy(c->blob.data() + kOffInvWater, c->water.inv.data(), kInvN * sizeof(uint16_t));
    std::memcpy(c->blob.data() + kOffInvOwn, own.inv.data(), kInvN * sizeof(uint16_t));
    for (int m = 0; m < nm; ++m) {
        const Material& mt = c->mats[m];
        for (int i = 0; i < kNE; ++i) {
            double s = 0.0;
            for (int e = 0; e < kNEl; ++e)
                s += mt.nuclei_per_g_barn[e] * ((double)c->sig_el[e * kNE + i] + (double)c->sig_ne[e * kNE + i]);
            c->blob[kOffSigma + 1000 * m + i] = (float)s;
        }
        float* mc = c->blob.data() + kOffSigma + 1000 * nm + 4 * m;
        mc[0] = (float)mt.f;
        mc[1] = (float)mt.x0;
        mc[2] = (float)mt.za;
        mc[3] = mt.own ? 1.f : 0.f;
    }
}

template <class T>
pmc_status upload(pmc_ctx* c, DevBuf<T>& b, const std::vector<T>& v, const char* what)
{
    HIPCHK(b.ensure(v.size()), what);
    HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), what);
    return PMC_OK;
}

pmc_status upload_tables(pmc_ctx* c)
{
    if (!c->have_phys || c->mats.empty()) return PMC_OK;
    build_blob(c);
    pmc_status s = upload(c, c->d_blob, c->blob, "upload tables");
    if (s != PMC_OK) return s;
    const int nm = (int)c->mats.size();
    std::vector<float> npg(nm * kNEl);
    for (int m = 0; m < nm; ++m)
        for (int e = 0; e < kNEl; ++e) npg[m * kNEl + e] = (float)c->mats[m].nuclei_per_g_barn[e];
    s = upload(c, c->d_npg, npg, "upload nuclei per gram");
    if (s != PMC_OK) return s;
    static_assert(kMolMatFloats == 16, "the transport kernel reads 16 Moliere floats per material");
    std::vector<float> mol((size_t)nm * kMolMatFloats);
    for (int m = 0; m < nm; ++m) moliere_material(c->mats[m].w, &mol[(size_t)m * kMolMatFloats]);
    return upload(c, c->d_molmat, mol, "upload Moliere material constants");
}

bool params_ok(const pmc_params& p, std::string& why)
{
    if (!(p.f_mcs >= 0.0 && p.f_mcs < 10.0)) { why = "f_mcs out of range"; return false; }
    if (!(p.s_min_cm > 0.0 && p.s_min_cm < 1.0)) { why = "s_min_cm out of range"; return false; }
    if (p.k_batches < 2 || p.k_batches > 64) { why = "k_batches must be in [2, 64]"; return false; }
    if (p.flags & ~(31u | (uint32_t)PMC_INC)) { why = "unknown flags"; return false; }
    if (p.block_threads != 0 && (p.block_threads < 64 || p.block_threads > 1024 || p.block_threads % 64))
    { why = "block_threads must be 0 or a multiple of 64 in [64, 1024]"; return false; }
    if (p.blocks_per_cu < 0 || p.blocks_per_cu > 64) { why = "blocks_per_cu out of range"; return false; }
    if (p.refill_lanes < 0 || p.refill_lanes > 64) { why = "refill_lanes out of range"; return false; }
    if (p.batch_events < 0 || p.batch_events > 64) { why = "batch_events out of range"; return false; }
    if (p.tally_cache != 0 && p.tally_cache != -1 && (p.tally_cache < 512 || p.tally_cache > 16384))
    { why = "tally_cache must be -1, 0 or in [512, 16384]"; return false; }
    if (p.epoch_steps < 0 || p.epoch_steps > 4096) { why = "epoch_steps must be in [0, 4096]"; return false; }
    if (p.cache_probes < 0 || p.cache_probes > 16) { why = "cache_probes must be in [0, 16]"; return false; }
    if (p.claim_run_log2 != 0 && (p.claim_run_log2 < 4 || p.claim_run_log2 > 16))
    { why = "claim_run_log2 must be 0 or in [4, 16]"; return false; }
    if (p.local_queue < -1 || p.local_queue > 65536) { why = "local_queue must be -1, 0 or in [1, 65536]"; return false; }
    return true;
}

bool same_materials(const std::vector<Material>& a, const std::vector<Material>& b)
{
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i) {
        if (a[i].hu_lo != b[i].hu_lo || a[i].hu_hi != b[i].hu_hi || a[i].rho_lo != b[i].rho_lo ||
            a[i].rho_hi != b[i].rho_hi || a[i].i_ev != b[i].i_ev || a[i].own != b[i].own)
            return false;
        for (int e = 0; e < kNEl; ++e)
            if (a[i].w[e] != b[i].w[e]) return false;
    }
    return true;
}

// HU grid -> voxel records of one geometry (Sec. II.A.1)
pmc_status build_geometry(pmc_ctx* c, Geometry& g, const int16_t* hu, int nx, int ny, int nz, float dx,
                          float dy, float dz, const std::vector<Material>& mats)
{
    const size_t nv = (size_t)nx * ny * nz;
    std::vector<uint2> rec(nv);
    const int nb = (int)mats.size();
    for (size_t v = 0; v < nv; ++v) {
        int h = hu[v];
        h = h < -1000 ? -1000 : (h > 3000 ? 3000 : h);
        int b = 0;
        while (b + 1 < nb && mats[b + 1].hu_lo <= h) ++b;
        const Material& m = mats[b];
        double rho = m.rho_lo;
        if (m.hu_hi > m.hu_lo) rho = m.rho_lo + (m.rho_hi - m.rho_lo) * double(h - m.hu_lo) / double(m.hu_hi - m.hu_lo);
        const float rf = (float)rho;
        uint32_t bits;
        std::memcpy(&bits, &rf, 4);
        rec[v] = make_uint2(bits, (uint32_t)b);
    }
    pmc_status s = upload(c, g.vox, rec, "upload voxel records");
    if (s != PMC_OK) return s;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.vs[0] = dx; g.vs[1] = dy; g.vs[2] = dz;
    return PMC_OK;
}

pmc_status load_geometry_common(pmc_ctx* c, int slot, const int16_t* hu, int nx, int ny, int nz, float dx,
                                float dy, float dz, const pmc_material_table* mt)
{
    if (!hu || !mt) return fail(c, PMC_ERR_ARG, "geometry: NULL pointer");
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(c, PMC_ERR_ARG, "geometry: dimensions must be > 0");
    if (!(dx > 0.f) || !(dy > 0.f) || !(dz > 0.f)) return fail(c, PMC_ERR_ARG, "geometry: voxel size must be > 0");
    if ((double)nx * ny * nz > 4.0e9) return fail(c, PMC_ERR_ARG, "geometry: too many voxels");
    std::vector<Material> mats;
    std::string why = build_materials(mt->n_bins, mt->hu_lo, mt->rho_lo, mt->rho_hi, mt->mass_frac,
                                      mt->i_ev, mt->own_table, mats);
    if (!why.empty()) return fail(c, PMC_ERR_ARG, why);
    const bool others = c->geoms.size() > 1 || (slot != 0 && have_geometry(c));
    if (others && !c->mats.empty() && !same_materials(mats, c->mats))
        return fail(c, PMC_ERR_ARG, "all geometries of a context must use the same material table");
    HIPCHK(hipSetDevice(c->device), "set device");
    if (c->geoms.empty()) c->geoms.emplace_back(new Geometry());
    if (slot >= (int)c->geoms.size()) c->geoms.emplace_back(new Geometry());
    pmc_status s = build_geometry(c, *c->geoms[slot], hu, nx, ny, nz, dx, dy, dz, mats);
    if (s != PMC_OK) return s;
    if (c->mats.empty() || !same_materials(mats, c->mats)) {
        c->mats = mats;
        c->own_bin = -1;
        for (int b = 0; b < (int)mats.size(); ++b)
            if (mats[b].own) {
                c->own_bin = b;
                c->own = build_range_table(mats[b].za, mats[b].i_ev);
            }
    }
    if (c->water.lnr.empty()) c->water = build_range_table(water_z_over_a(), kWaterIeV);
    return upload_tables(c);
}

pmc_status check_spots(pmc_ctx* c, const pmc_spot* spots, int n_spots, unsigned long long n_hist,
                       double* wsum_out)
{
    if (n_spots < 0) return fail(c, PMC_ERR_ARG, "n_spots < 0");
    if (n_hist > 0 && (n_spots <= 0 || !spots)) return fail(c, PMC_ERR_ARG, "no spots");
    if (n_hist >= (1ull << 32)) return fail(c, PMC_ERR_ARG, "at most 2^32-1 histories per plan");
    double wsum = 0.0;
    for (int s = 0; s < n_spots; ++s) {
        const pmc_spot& sp = spots[s];
        if (!(sp.e_mev > (float)kEMin && sp.e_mev <= (float)kEMax))
            return fail(c, PMC_ERR_RANGE, "spot energy outside (0.1, 250] MeV");
        if (!(sp.weight >= 0.f) || !(sp.sigma_x_cm >= 0.f) || !(sp.sigma_y_cm >= 0.f) ||
            !std::isfinite(sp.x_cm) || !std::isfinite(sp.y_cm) || !std::isfinite(sp.weight) ||
            !std::isfinite(sp.sigma_x_cm) || !std::isfinite(sp.sigma_y_cm))
            return fail(c, PMC_ERR_RANGE, "spot weight/width must be finite and >= 0");
        wsum += sp.weight;
    }
    if (n_hist > 0 && !(wsum > 0.0)) return fail(c, PMC_ERR_RANGE, "spot weights sum to zero");
    *wsum_out = wsum;
    return PMC_OK;
}

// histories per spot: largest remainder, proportional to weight
void allocate(const pmc_spot* spots, int n_spots, unsigned long long n_hist, double wsum,
              std::vector<unsigned long long>& ns)
{
    ns.assign(std::max(n_spots, 1), 0);
    if (n_hist == 0) return;
    std::vector<std::pair<double, int>> rem(n_spots);
    unsigned long long assigned = 0;
    for (int s = 0; s < n_spots; ++s) {
        const double q = (double)n_hist * spots[s].weight / wsum;
        ns[s] = (unsigned long long)std::floor(q);
        rem[s] = {q - std::floor(q), s};
        assigned += ns[s];
    }
    std::sort(rem.begin(), rem.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
        return a.first != b.first ? a.first > b.first : a.second < b.second;
    });
    for (unsigned long long i = 0; assigned + i < n_hist; ++i) ns[rem[i % n_spots].second]++;
}

float u2f(uint32_t u)
{
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// The cascade's target nuclei on the device and the event kernel's grid
// (built once per context, on the first run or inspection that needs them).
pmc_status ensure_inc(pmc_ctx* c)
{
    if (c->d_inc_nuc.p && c->inc_grid > 0) return PMC_OK;
    std::vector<IncNucleus> nu(kIncTargets);
    for (int e = 1; e <= kIncTargets; ++e) build_inc_nucleus(e, &nu[e - 1]);
    HIPCHK(c->d_inc_nuc.ensure(kIncTargets), "alloc nuclei");
    HIPCHK(hipMemcpy(c->d_inc_nuc.p, nu.data(), kIncTargets * sizeof(IncNucleus), hipMemcpyHostToDevice),
           "upload nuclei");
    IncTab tab;
    build_inc_table(&tab);
    HIPCHK(c->d_inc_tab.ensure(1), "alloc evaporation table");
    HIPCHK(hipMemcpy(c->d_inc_tab.p, &tab, sizeof(IncTab), hipMemcpyHostToDevice), "upload evaporation table");
    int per_cu = 0;
    HIPCHK(inc_transport_occupancy(&per_cu), "cascade kernel occupancy");
    c->inc_grid = c->num_cu * std::max(1, std::min(per_cu, 4));
    return PMC_OK;
}

struct RunResult {
    double transport_ms = 0, device_ms = 0, first_ms = 0;
    int generations = 0;
};

// a traced run (kTrace, first generation only): iterations to hold per lane
// in, the launch shape and trace extent out
struct TraceReq {
    unsigned long long iters = 0;
    int grid = 0, block = 0, slots = 0, epoch_iters = 0, probes = 0;
    unsigned long long lanes = 0;
};

// The driver.  tuning = a calibration run: no statistics, no outputs.
pmc_status run_driver(pmc_ctx* c, std::vector<PlanIn>& plans, bool multi, const Shape& shape,
                      hipStream_t st, bool tuning, RunResult* rr, TraceReq* trace = nullptr)
{
    if (trace && (multi || plans.size() != 1)) return fail(c, PMC_ERR_ARG, "a traced run has one plan");
    const int K = c->p.k_batches;
    const int np = (int)plans.size();
    // LET_d is scored for the whole launch when any plan asks for it: every
    // plan's tally then carries the two LET planes after its dose groups
    bool let = false;
    for (const PlanIn& q : plans) let = let || q.d_let != nullptr;
    const int planes = K + (let ? 2 : 0);
    for (int p = 0; p < np; ++p)
        for (int q = 0; q < p; ++q)
            if (plans[p].g == plans[q].g) return fail(c, PMC_ERR_ARG, "two plans of one run share a geometry");
    // spots of every plan, flattened, each tagged with its plan and its first
    // history index within the plan
    std::vector<float> sp;
    std::vector<unsigned long long> start(1, 0), first;
    std::vector<double> incident(np, 0.0), wtot(np, 0.0);
    unsigned long long total = 0;
    for (int p = 0; p < np; ++p) {
        const PlanIn& pl = plans[p];
        double wsum = 0.0;
        pmc_status s = check_spots(c, pl.spots, pl.n_spots, pl.n_hist, &wsum);
        if (s != PMC_OK) return s;
        std::vector<unsigned long long> ns;
        allocate(pl.spots, pl.n_spots, pl.n_hist, wsum, ns);
        unsigned long long local = 0;
        for (int s2 = 0; s2 < pl.n_spots && pl.n_hist > 0; ++s2) {
            const pmc_spot& q = pl.spots[s2];
            const double om = ns[s2] ? (q.weight / wsum) * (double)pl.n_hist / (double)ns[s2] : 0.0;
            const float omf = (float)om;
            const float rec[8] = {q.x_cm / pl.g->vs[0], q.y_cm / pl.g->vs[1], q.e_mev,
                                  q.sigma_x_cm / pl.g->vs[0], q.sigma_y_cm / pl.g->vs[1], omf,
                                  u2f((uint32_t)p), u2f((uint32_t)local)};
            sp.insert(sp.end(), rec, rec + 8);
            start.push_back(start.back() + ns[s2]);
            first.push_back(local);
            local += ns[s2];
            incident[p] += (double)ns[s2] * (double)omf * (double)q.e_mev;
            wtot[p] += (double)ns[s2] * (double)omf;
        }
        total += pl.n_hist;
    }
    const int n_spots = (int)start.size() - 1;
    if (sp.empty()) sp.assign(8, 0.f);
    // batch-major work order of the primaries (Sec. II.B.2 groups): statistical
    // group b of a spot with n histories holds its histories at positions
    // [ceil(b n / K), ceil((b + 1) n / K)); the primaries are worked group by
    // group, so that a workgroup's run of consecutive work indices stays in
    // one group (one tally column) while it moves across neighbouring spots.
    // The history index (random-number stream) and the group of every
    // primary are those of the spot-major numbering.
    const size_t ns1 = (size_t)n_spots + 1;
    std::vector<unsigned long long> order((size_t)K * ns1 + (size_t)K * n_spots + 1, 0ull);
    {
        unsigned long long at = 0;
        for (int b = 0; b < K; ++b) {
            for (int s2 = 0; s2 < n_spots; ++s2) {
                const unsigned long long n = start[s2 + 1] - start[s2];
                const unsigned long long p0 = ((unsigned long long)b * n + K - 1) / K;
                const unsigned long long p1 = ((unsigned long long)(b + 1) * n + K - 1) / K;
                order[b * ns1 + s2] = at;
                order[(size_t)K * ns1 + (size_t)b * n_spots + s2] = first[s2] + p0;
                at += p1 - p0;
            }
            order[b * ns1 + n_spots] = at;
        }
        if (at != total) return fail(c, PMC_ERR_ARG, "internal: work order does not cover the histories");
    }
    HIPCHK(hipSetDevice(c->device), "set device");
    const unsigned long long cap = c->p.queue_capacity ? c->p.queue_capacity
                                                       : std::max<unsigned long long>(65536ull, total);
    std::vector<PlanDesc> pd(np);
    for (int p = 0; p < np; ++p) {
        Geometry& g = *plans[p].g;
        HIPCHK(g.tally.ensure(g.nvox() * planes), "alloc tally");
        PlanDesc& d = pd[p];
        std::memset(&d, 0, sizeof(d));
        d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
        for (int i = 0; i < 3; ++i) { d.vs[i] = g.vs[i]; d.ivs[i] = 1.0f / g.vs[i]; }
        d.vox = g.vox.p;
        d.tally = g.tally.p;
        d.key_lo = (uint32_t)plans[p].seed;
        d.key_hi = (uint32_t)(plans[p].seed >> 32);
    }
    HIPCHK(c->d_q[0].ensure(cap * kQueuePlanes), "alloc queue");
    HIPCHK(c->d_q[1].ensure(cap * kQueuePlanes), "alloc queue");
    HIPCHK(c->d_gc.ensure(2 * (kMaxGenerations + 2)), "alloc counters");
    HIPCHK(c->d_counters.ensure((size_t)kPlanCounters * np), "alloc counters");
    HIPCHK(c->d_ledger.ensure(4 * np), "alloc ledger");
    HIPCHK(c->d_spots.ensure(sp.size()), "alloc spots");
    HIPCHK(c->d_order.ensure(order.size()), "alloc spots");
    HIPCHK(c->d_plans.ensure(np), "alloc plans");
    HIPCHK(hipMemcpyAsync(c->d_spots.p, sp.data(), sp.size() * 4, hipMemcpyHostToDevice, st), "upload spots");
    HIPCHK(hipMemcpyAsync(c->d_order.p, order.data(), order.size() * 8, hipMemcpyHostToDevice, st), "upload spots");
    HIPCHK(hipMemcpyAsync(c->d_plans.p, pd.data(), np * sizeof(PlanDesc), hipMemcpyHostToDevice, st), "upload plans");
    HIPCHK(hipEventRecord(c->ev0, st), "event");
    for (int p = 0; p < np; ++p)
        HIPCHK(launch_zero(pd[p].tally, plans[p].g->nvox() * planes * 8, st), "zero tally");
    HIPCHK(launch_zero(c->d_gc.p, c->d_gc.n * 8, st), "zero counters");
    HIPCHK(launch_zero(c->d_counters.p, 8 * (size_t)kPlanCounters * np, st), "zero counters");
    HIPCHK(launch_zero(c->d_ledger.p, 32 * (size_t)np, st), "zero ledger");

    KernelArgs a{};
    a.single = pd[0];
    a.plans = c->d_plans.p;
    a.n_plans = np;
    a.blob = c->d_blob.p;
    a.blob_words = (int)c->blob.size();
    a.pd_offset = (a.blob_words + 3) & ~3;
    a.n_mat = (int)c->mats.size();
    const RangeTable& own = c->own_bin >= 0 ? c->own : c->water;
    a.r_first[0] = (float)c->water.r_first; a.r_first[1] = (float)own.r_first;
    a.ln_r1[0] = (float)c->water.ln_r1; a.ln_r1[1] = (float)own.ln_r1;
    a.inv_step[0] = (float)c->water.inv_step; a.inv_step[1] = (float)own.inv_step;
    a.el_sig = c->d_el_sig.p; a.mat_npg = c->d_npg.p; a.elem = c->d_elem.p;
    a.sec_mult = c->d_mult.p; a.sec_floc = c->d_floc.p; a.sec_x = c->d_xcdf.p; a.sec_mu = c->d_mucdf.p;
    a.vav = c->d_vav.p;
    a.mol = c->d_mol.p;
    a.molmat = c->d_molmat.p;
    a.k_batches = K;
    a.flags = c->p.flags | (let ? kScoreLet : 0u);
    a.f_mcs = (float)c->p.f_mcs;
    a.s_min = (float)c->p.s_min_cm;
    a.spots = c->d_spots.p;
    a.order = c->d_order.p;
    a.n_spots = n_spots;
    a.n_primary = total;
    a.q_cap = cap;
    a.gen_counters = c->d_gc.p;
    a.ledger = c->d_ledger.p;
    a.counters = c->d_counters.p;
    a.refill_lanes = shape.refill;
    a.batch_events = shape.batch;

    const int block = shape.block;
    // launch layout (LDS regions, buffer sizes): computed and checked by
    // plan_layout, which the kernel's offsets come from; the grid-dependent
    // parts once the occupancy has fixed the grid
    LayoutQuery lq;
    lq.block = block;
    lq.n_plans = np;
    lq.multi = multi;
    lq.score_let = let;
    lq.k_batches = K;
    lq.n_mat = a.n_mat;
    lq.cache_request = c->p.tally_cache != 0 ? c->p.tally_cache : shape.cache;
    lq.local_queue = c->p.local_queue;
    lq.queue_capacity = c->p.queue_capacity;
    lq.n_histories = total;
    lq.n_spots = n_spots;
    for (const PlanIn& q : plans) {
        lq.max_nvox = std::max<unsigned long long>(lq.max_nvox, q.g->nvox());
        lq.max_plan_histories = std::max<unsigned long long>(lq.max_plan_histories, q.n_hist);
    }
    LaunchLayout lay;
    std::string why = plan_layout(lq, &lay);
    if (!why.empty()) return fail(c, PMC_ERR_ARG, "launch layout: " + why);
    if (lay.blob_words != a.blob_words || lay.pd_off != a.pd_offset || lay.q_cap != cap ||
        lay.planes != planes || lay.order_words != order.size())
        return fail(c, PMC_ERR_DEVICE, "internal: launch layout disagrees with the run's buffers");
    const int slots = lay.cache_slots;
    a.cache_slots = slots;
    a.cache_off = lay.cache_off;
    a.key_off = lay.key_off;
    a.num_off = lay.num_off;
    a.ctl_off = lay.ctl_off;
    a.args_off = lay.args_off;
    a.led_off = lay.led_off;
    a.cnt_off = lay.cnt_off;
    a.epoch_iters = c->p.epoch_steps ? c->p.epoch_steps : 32;
    a.cache_probes = c->p.cache_probes ? c->p.cache_probes : 3;
    const size_t lds = lay.lds_bytes;
    int max_block = 0;
    HIPCHK(transport_max_block(multi, a.flags, &max_block), "kernel attributes");
    if (block > max_block) return fail(c, PMC_ERR_ARG, "block_threads exceeds the transport kernel's limit");
    int bpc = shape.blocks_per_cu, fit = 0;
    HIPCHK(transport_occupancy(multi, a.flags, block, lds, &fit), "occupancy");
    if (fit < 1) return fail(c, PMC_ERR_DEVICE, "transport kernel does not fit on a CU");
    if (bpc == 0 || bpc > fit) bpc = fit;
    const int grid = c->num_cu * bpc;
    lq.grid = grid;
    why = plan_layout(lq, &lay);
    if (!why.empty()) return fail(c, PMC_ERR_ARG, "launch layout: " + why);
    if (lay.lds_bytes != lds) return fail(c, PMC_ERR_DEVICE, "internal: launch layout changed with the grid");
    // per-workgroup claim counters of every generation
    HIPCHK(c->d_wgc.ensure(lay.claim_words), "alloc claim counters");
    HIPCHK(launch_zero(c->d_wgc.p, lay.claim_words * 8, st), "zero claim counters");
    a.wg_claims = c->d_wgc.p;
    // per-workgroup secondary queues (48-byte entries); automatic: up to
    // 65536 entries per workgroup within 1 GiB for the whole grid (a
    // workgroup of the 16-plan batch emits about 40000 secondaries)
    a.loc_cap = lay.loc_cap;
    if (a.loc_cap > 0) {
        HIPCHK(c->d_qloc.ensure(lay.qloc_words), "alloc workgroup queues");
        a.q_loc = c->d_qloc.p;
    }
    if (trace) {
        // the address trace of generation 0: trace->iters loop iterations of
        // every lane, pre-filled with "no step"
        const unsigned long long lanes = (unsigned long long)grid * block;
        HIPCHK(c->d_trace.ensure(trace->iters * lanes), "alloc trace");
        HIPCHK(c->d_trace_epochs.ensure(grid), "alloc trace");
        HIPCHK(launch_fill_u32(c->d_trace.p, trace->iters * lanes, kTraceNone, st), "clear trace");
        HIPCHK(launch_fill_u32(c->d_trace_epochs.p, grid, 0u, st), "clear trace");
        a.trace = c->d_trace.p;
        a.trace_iters = trace->iters;
        a.trace_lanes = lanes;
        a.trace_epochs = c->d_trace_epochs.p;
        trace->grid = grid;
        trace->block = block;
        trace->slots = slots;
        trace->epoch_iters = a.epoch_iters;
        trace->probes = a.cache_probes;
        trace->lanes = lanes;
    }
    // non-elastic events by the intranuclear cascade: one event list per
    // generation, worked by the cascade kernel right after the transport
    const bool inc = (a.flags & kInc) != 0u;
    if (inc) {
        pmc_status si = ensure_inc(c);
        if (si != PMC_OK) return si;
        HIPCHK(c->d_inc_ev.ensure(cap), "alloc event list");
        // per generation: events recorded; then per generation the eight
        // claim counters of the cascade kernel's waves
        HIPCHK(c->d_inc_count.ensure(9 * kMaxGenerations), "alloc event counters");
        HIPCHK(launch_zero(c->d_inc_count.p, 9 * kMaxGenerations * 8, st), "zero event counters");
        a.inc_ev = c->d_inc_ev.p;
        a.inc_cap = cap;
    }
    const uint32_t run_flags = a.flags;
    int gens = 0;
    unsigned long long produced_total = 0, overflow_n = 0;
    // generations are launched in groups without waiting: each launch reads
    // its own work count on the device (an empty generation exits at once),
    // and the host reads the produced counts once per group
    int launched = 0;
    // with the workgroups' own queues the next generation only holds what
    // overflowed them, almost always nothing: launch one at a time, so that a
    // run is one launch unless its workgroup queues overflowed
    const int group = a.loc_cap > 0 ? 1 : kGenGroup;
    if (total > 0) {
        bool done = false;
        while (!done) {
            const int g0 = launched;
            const int g1 = std::min(g0 + group, kMaxGenerations);
            if (g0 >= kMaxGenerations) return fail(c, PMC_ERR_DEVICE, "secondary generations exceed limit");
            for (int gidx = g0; gidx < g1; ++gidx) {
                a.gen = gidx;
                // primaries in runs of up to 1024 consecutive histories (a
                // pencil's worth, for the deposit cache), secondaries in runs of 64
                a.claim_log2 = gidx == 0 ? (c->p.claim_run_log2 ? c->p.claim_run_log2 : 10) : 6;
                a.q_in = c->d_q[gidx & 1].p;
                a.q_out = c->d_q[(gidx + 1) & 1].p;
                a.flags = run_flags | (trace && gidx == 0 ? kTrace : 0u);
                a.inc_count = inc ? c->d_inc_count.p + gidx : nullptr;
                HIPCHK(hipEventRecord(c->ev_gen[2 * gidx], st), "event");
                HIPCHK(launch_transport(a, multi, grid, block, lds, st), "transport launch");
                HIPCHK(hipEventRecord(c->ev_gen[2 * gidx + 1], st), "event");
                if (inc) {
                    // this generation's events; their protons join the next
                    // generation's queue
                    IncLaunch il{c->d_inc_ev.p, c->d_inc_count.p + gidx, cap, c->d_inc_nuc.p, c->d_inc_tab.p,
                                 c->d_inc_count.p + kMaxGenerations + 8 * gidx, c->d_plans.p,
                                 np, K, let ? 1 : 0, a.q_out, cap, &c->d_gc.p[2 * (gidx + 1)],
                                 c->d_ledger.p, c->d_counters.p};
                    HIPCHK(hipEventRecord(c->ev_inc[2 * gidx], st), "event");
                    HIPCHK(launch_inc_transport(il, c->inc_grid, st), "cascade launch");
                    HIPCHK(hipEventRecord(c->ev_inc[2 * gidx + 1], st), "event");
                }
            }
            launched = g1;
            // produced counts of generations g0+1 .. g1: words 2(g0+1) .. 2 g1
            HIPCHK(hipMemcpyAsync(c->h_pinned, c->d_gc.p + 2 * (g0 + 1), 8 * (2 * (g1 - g0) - 1),
                                  hipMemcpyDeviceToHost, st), "read counters");
            HIPCHK(hipStreamSynchronize(st), "transport");
            for (int gidx = g0; gidx < g1; ++gidx) {
                const unsigned long long prod = c->h_pinned[2 * (gidx - g0)];
                ++gens;
                produced_total += prod;
                if (prod > cap) overflow_n += prod - cap;
                if (prod == 0) {
                    done = true;
                    break;
                }
            }
        }
    }
    if (!tuning) {
        for (int p = 0; p < np; ++p) {
            const Geometry& g = *plans[p].g;
            const double vol = (double)g.vs[0] * g.vs[1] * g.vs[2];
            const double conv0 = wtot[p] > 0.0 ? 1.602176634e-10 / (vol * wtot[p]) : 0.0;
            HIPCHK(launch_stats(g.tally.p, g.vox.p, g.nvox(), K, conv0, plans[p].d_dose, plans[p].d_var,
                                c->d_ledger.p + 4 * p + 3, plans[p].d_let, st), "stats launch");
        }
    }
    HIPCHK(hipEventRecord(c->ev1, st), "event");
    const size_t led_words = 4 * (size_t)np, cnt_words = (size_t)kPlanCounters * np;
    if ((led_words + cnt_words) * 8 > kPinnedBytes) return fail(c, PMC_ERR_ARG, "too many plans");
    HIPCHK(hipMemcpyAsync(c->h_pinned, c->d_ledger.p, led_words * 8, hipMemcpyDeviceToHost, st), "read ledger");
    HIPCHK(hipMemcpyAsync(c->h_pinned + led_words, c->d_counters.p, cnt_words * 8, hipMemcpyDeviceToHost, st), "read counters");
    HIPCHK(hipStreamSynchronize(st), "run");
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1), "event time");
    double transport_ms = 0.0, first_ms = 0.0, inc_ms = 0.0;
    for (int gidx = 0; gidx < launched; ++gidx) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, c->ev_gen[2 * gidx], c->ev_gen[2 * gidx + 1]), "event time");
        transport_ms += t;
        if (gidx == 0) first_ms = t;
        if (inc) {
            HIPCHK(hipEventElapsedTime(&t, c->ev_inc[2 * gidx], c->ev_inc[2 * gidx + 1]), "event time");
            inc_ms += t;
        }
    }
    if (inc && launched > 0) {
        // events beyond the list's capacity were counted as overflow
        std::vector<unsigned long long> ec(launched);
        HIPCHK(hipMemcpy(ec.data(), c->d_inc_count.p, 8 * (size_t)launched, hipMemcpyDeviceToHost), "read events");
        for (int gidx = 0; gidx < launched; ++gidx)
            if (ec[gidx] > cap) overflow_n += ec[gidx] - cap;
    }
    if (rr) {
        rr->transport_ms = transport_ms;
        rr->first_ms = first_ms;
        rr->device_ms = ms;
        rr->generations = gens;
    }
    if (!tuning) {
        const double* led = reinterpret_cast<const double*>(c->h_pinned);
        const unsigned long long* cnt = c->h_pinned + led_words;
        for (int p = 0; p < np; ++p) {
            pmc_summary* sm = plans[p].summary;
            if (!sm) continue;
            std::memset(sm, 0, sizeof(*sm));
            sm->incident = incident[p];
            sm->escaped = led[4 * p + 0];
            sm->neutral = led[4 * p + 1];
            sm->overflow = led[4 * p + 2];
            sm->deposited = led[4 * p + 3];
            sm->histories = plans[p].n_hist;
            const unsigned long long* cp = cnt + (size_t)kPlanCounters * p;
            sm->steps = cp[0];
            sm->n_elastic = cp[1];
            sm->n_nonelastic = cp[2];
            sm->n_short_steps = cp[3];
            sm->tally_atomics = cp[4];
            sm->global_atomics = cp[5];
            sm->cache_flush_atomics = cp[6];
            sm->refill_lanes = shape.refill;
            sm->batch_events = shape.batch;
            sm->block_threads = block;
            sm->grid_blocks = grid;
            sm->cache_slots = slots;
            sm->epoch_steps = a.epoch_iters;
            // taken by the emitting workgroup (this plan), plus those that
            // went through the generation queues (the whole run)
            sm->secondaries = cp[7] + produced_total;
            sm->n_overflow = overflow_n;
            sm->total_weight = wtot[p];
            sm->device_ms = ms;
            sm->transport_ms = transport_ms;
            sm->first_launch_ms = first_ms;
            sm->generations = gens;
            sm->launches = launched;
            sm->inc_events = cp[kCtrIncEvents];
            sm->inc_secondaries = cp[kCtrIncSecondaries];
            sm->inc_collisions = cp[kCtrIncCollisions];
            sm->inc_ms = inc_ms;
        }
    }
    if (c->h_pinned[led_words + kCtrAborted] != 0)
        return fail(c, PMC_ERR_DEVICE, "transport workgroups stopped at the epoch limit: dose incomplete");
    if (overflow_n) return fail(c, PMC_ERR_QUEUE_OVERFLOW, "secondary queue overflow: raise queue_capacity");
    return PMC_OK;
}

// Launch shape of a run: the caller's fixed values, and for the fields left
// at 0 the fastest of a few candidates timed on a scaled-down copy of the
// workload (2e5 histories), remembered per workload signature.
pmc_status choose_shape(pmc_ctx* c, std::vector<PlanIn>& plans, bool multi, hipStream_t st, Shape* out)
{
    Shape s;
    s.block = c->p.block_threads ? c->p.block_threads : 256;
    s.blocks_per_cu = c->p.blocks_per_cu;
    s.refill = c->p.refill_lanes ? c->p.refill_lanes : 16;
    s.batch = c->p.batch_events ? c->p.batch_events : 4;
    const bool tune = c->p.block_threads == 0 || c->p.refill_lanes == 0 || c->p.batch_events == 0;
    unsigned long long total = 0, vox = 0;
    for (const PlanIn& p : plans) {
        total += p.n_hist;
        vox += p.g->nvox();
    }
    if (!tune || total < 200000ull) {
        *out = s;
        return PMC_OK;
    }
    auto log2i = [](unsigned long long v) { int l = 0; while (v >>= 1) ++l; return l; };
    bool let = false;
    for (const PlanIn& p : plans) let = let || p.d_let != nullptr;
    const auto key = std::make_tuple((int)multi + 2 * (int)let, (int)plans.size(), log2i(total), log2i(vox));
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
        *out = it->second;
        return PMC_OK;
    }
    // every plan contributes eight runs of consecutive spots spread evenly
    // over its list (every energy layer of a field is represented), with
    // their own history counts, up to a fraction f of its work: consecutive
    // spots keep the spatial coherence the deposit cache relies on
    constexpr int kCalBlocks = 8;
    auto sample = [&](double f, std::vector<PlanIn>& cal, std::vector<std::vector<pmc_spot>>& cal_spots) {
        cal = plans;
        cal_spots.assign(cal.size(), {});
        for (size_t pi = 0; pi < cal.size(); ++pi) {
            PlanIn& p = cal[pi];
            p.summary = nullptr;
            if (f >= 1.0) continue;
            double wsum = 0.0;
            for (int i = 0; i < p.n_spots; ++i) wsum += p.spots[i].weight;
            const double goal = f * (double)p.n_hist;
            std::vector<pmc_spot>& sel = cal_spots[pi];
            double acc = 0.0;
            for (int blk = 0; blk < kCalBlocks; ++blk) {
                int m = (int)(((long long)blk * p.n_spots) / kCalBlocks);
                const double blk_goal = goal * (blk + 1) / kCalBlocks;
                while (m < p.n_spots && (acc < blk_goal || sel.empty())) {
                    acc += wsum > 0.0 ? (double)p.n_hist * p.spots[m].weight / wsum : 0.0;
                    sel.push_back(p.spots[m]);
                    ++m;
                }
            }
            p.spots = sel.data();
            p.n_spots = (int)sel.size();
            p.n_hist =
                std::max<unsigned long long>(1ull, (unsigned long long)std::llround(std::min(acc, (double)p.n_hist)));
        }
    };
    // calibration work: a fifth of the run, 2e5 to 2e6 histories, enough to
    // reach the steady state of a full grid of 1024-lane workgroups
    const double cal_hist = std::min(2.0e6, std::max(2.0e5, 0.2 * (double)total));
    std::vector<PlanIn> cal;
    std::vector<std::vector<pmc_spot>> cal_spots;
    sample(cal_hist / (double)total, cal, cal_spots);
    std::vector<Shape> cands;
    for (int b : {256, 512, 1024})
        for (int r : {8, 16})
            for (int e : {4, 8})
                for (int ch : {0, -1}) {
                    Shape x;
                    x.block = c->p.block_threads ? c->p.block_threads : b;
                    x.blocks_per_cu = c->p.blocks_per_cu;
                    x.refill = c->p.refill_lanes ? c->p.refill_lanes : r;
                    x.batch = c->p.batch_events ? c->p.batch_events : e;
                    // the cache is only worth a choice where it fits next to the tables
                    x.cache = (c->p.tally_cache != 0 || x.block < 512) ? 0 : ch;
                    bool dup = false;
                    for (const Shape& y : cands)
                        dup |= (y.block == x.block && y.refill == x.refill && y.batch == x.batch &&
                                y.cache == x.cache);
                    if (!dup) cands.push_back(x);
                }
    // every candidate once, then the three fastest twice more: a shape is
    // rated by the best of its three times, which keeps one noisy
    // calibration launch from deciding (neighbouring shapes differ by a few
    // per cent)
    std::vector<std::pair<double, int>> times;
    for (size_t i = 0; i < cands.size(); ++i) {
        RunResult r;
        pmc_status st2 = run_driver(c, cal, multi, cands[i], st, true, &r);
        if (st2 != PMC_OK) return st2;
        times.push_back({r.transport_ms, (int)i});
    }
    std::sort(times.begin(), times.end());
    const size_t n_final = std::min<size_t>(3, times.size());
    for (int rep = 0; rep < 2; ++rep)
        for (size_t k = 0; k < n_final; ++k) {
            RunResult r;
            pmc_status st2 = run_driver(c, cal, multi, cands[times[k].second], st, true, &r);
            if (st2 != PMC_OK) return st2;
            times[k].first = std::min(times[k].first, r.transport_ms);
        }
    std::sort(times.begin(), times.end());
    int best_i = times[0].second;
    // the best shape of each workgroup size once more on a sample as large
    // as the run (up to 2e7 histories, best of two each): the workgroup size
    // sets the occupancy and the cache size, and shapes that come out within
    // a few per cent on the calibration sample can differ by more on the
    // whole field
    if (total > (unsigned long long)cal_hist) {
        std::vector<int> finalists;
        for (const auto& t : times) {
            bool seen = false;
            for (int f : finalists) seen |= cands[f].block == cands[t.second].block;
            if (!seen) finalists.push_back(t.second);
        }
        if (finalists.size() > 1) {
            std::vector<PlanIn> big;
            std::vector<std::vector<pmc_spot>> big_spots;
            sample(std::min(1.0, 2.0e7 / (double)total), big, big_spots);
            double best_t = 1e300;
            for (int f : finalists) {
                double t_f = 1e300;
                for (int rep = 0; rep < 2; ++rep) {
                    RunResult r;
                    pmc_status st2 = run_driver(c, big, multi, cands[f], st, true, &r);
                    if (st2 != PMC_OK) return st2;
                    t_f = std::min(t_f, r.transport_ms);
                }
                if (t_f < best_t) {
                    best_t = t_f;
                    best_i = f;
                }
            }
        }
    }
    const Shape best_s = cands[best_i];
    c->tuned[key] = best_s;
    *out = best_s;
    return PMC_OK;
}

pmc_status run_plans_impl(pmc_ctx* c, std::vector<PlanIn>& plans, bool multi, hipStream_t st)
{
    if (!c->have_phys || !have_geometry(c)) return fail(c, PMC_ERR_STATE, "load physics and geometry first");
    for (const PlanIn& p : plans) {
        double w;
        pmc_status s = check_spots(c, p.spots, p.n_spots, p.n_hist, &w);
        if (s != PMC_OK) return s;
    }
    Shape shape;
    pmc_status s = choose_shape(c, plans, multi, st, &shape);
    if (s != PMC_OK) return s;
    return run_driver(c, plans, multi, shape, st, false, nullptr);
}

}  // namespace

extern "C" {

pmc_status pmc_default_params(pmc_params* p)
{
    if (!p) return PMC_ERR_ARG;
    std::memset(p, 0, sizeof(*p));
    p->f_mcs = 1.07;
    p->s_min_cm = 1e-4;
    p->k_batches = 10;
    return PMC_OK;
}

const char* pmc_version(void) { return "pmc 0.3 gfx950"; }

const char* pmc_last_error(const pmc_ctx* c)
{
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

pmc_status pmc_create(pmc_ctx** out, int device, const pmc_params* p)
{
    g_create_error.clear();
    if (!out) { g_create_error = "out is NULL"; return PMC_ERR_ARG; }
    pmc_params prm;
    if (p) prm = *p;
    else pmc_default_params(&prm);
    std::string why;
    if (!params_ok(prm, why)) { g_create_error = why; return PMC_ERR_ARG; }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        g_create_error = std::string("no HIP device: ") + hipGetErrorString(e);
        return PMC_ERR_DEVICE;
    }
    if (device < 0 || device >= ndev) { g_create_error = "device index out of range"; return PMC_ERR_ARG; }
    pmc_ctx* c = new (std::nothrow) pmc_ctx();
    if (!c) { g_create_error = "host allocation failed"; return PMC_ERR_NOMEM; }
    c->device = device;
    c->p = prm;
    hipDeviceProp_t prop;
    if ((e = hipSetDevice(device)) != hipSuccess || (e = hipGetDeviceProperties(&prop, device)) != hipSuccess ||
        (e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess ||
        (e = hipHostMalloc((void**)&c->h_pinned, kPinnedBytes, hipHostMallocDefault)) != hipSuccess) {
        g_create_error = std::string("device setup: ") + hipGetErrorString(e);
        pmc_destroy(c);
        return PMC_ERR_DEVICE;
    }
    for (int i = 0; i < 2 * kMaxGenerations; ++i)
        if ((e = hipEventCreate(&c->ev_gen[i])) != hipSuccess || (e = hipEventCreate(&c->ev_inc[i])) != hipSuccess) {
            g_create_error = std::string("device setup: ") + hipGetErrorString(e);
            pmc_destroy(c);
            return PMC_ERR_DEVICE;
        }
    c->num_cu = prop.multiProcessorCount;
    if (prm.flags & PMC_MOLIERE) {
        const std::vector<float>& t = moliere_table();
        if ((e = c->d_mol.ensure(t.size())) != hipSuccess ||
            (e = hipMemcpy(c->d_mol.p, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) {
            g_create_error = std::string("Moliere table upload: ") + hipGetErrorString(e);
            pmc_destroy(c);
            return PMC_ERR_DEVICE;
        }
    }
    if (prm.flags & PMC_VAVILOV) {
        const std::vector<float>& t = vavilov_table();
        if ((e = c->d_vav.ensure(t.size())) != hipSuccess ||
            (e = hipMemcpy(c->d_vav.p, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) {
            g_create_error = std::string("Vavilov table upload: ") + hipGetErrorString(e);
            pmc_destroy(c);
            return PMC_ERR_DEVICE;
        }
    }
    *out = c;
    return PMC_OK;
}

pmc_status pmc_moliere_table(float* out, int32_t n_floats)
{
    const std::vector<float>& t = moliere_table();
    if (!out || n_floats < (int32_t)t.size()) return PMC_ERR_ARG;
    std::copy(t.begin(), t.end(), out);
    return PMC_OK;
}

pmc_status pmc_vavilov_table(float* out, int32_t n_floats)
{
    const std::vector<float>& t = vavilov_table();
    if (!out || n_floats < (int32_t)t.size()) return PMC_ERR_ARG;
    std::copy(t.begin(), t.end(), out);
    return PMC_OK;
}

pmc_status pmc_destroy(pmc_ctx* c)
{
    if (!c) return PMC_OK;
    (void)hipSetDevice(c->device);
    c->geoms.clear();
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    for (int i = 0; i < 2 * kMaxGenerations; ++i) {
        if (c->ev_gen[i]) (void)hipEventDestroy(c->ev_gen[i]);
        if (c->ev_inc[i]) (void)hipEventDestroy(c->ev_inc[i]);
    }
    delete c;   // the DevBuf destructors release the remaining device buffers
    return PMC_OK;
}

pmc_status pmc_load_physics(pmc_ctx* c, const pmc_nuclear_data* nd)
{
    if (!c) return PMC_ERR_ARG;
    if (!nd || !nd->sigma_ne_barn || !nd->sigma_el_barn || !nd->mult_cdf || !nd->f_local ||
        !nd->x_cdf || !nd->mu_cdf)
        return fail(c, PMC_ERR_ARG, "nuclear data: NULL array");
    const size_t ns = kNEl * kNE, nrow = kSecNuc * kSecBins;
    for (size_t i = 0; i < ns; ++i)
        if (!(nd->sigma_ne_barn[i] >= 0.f) || !(nd->sigma_el_barn[i] >= 0.f) ||
            !std::isfinite(nd->sigma_ne_barn[i]) || !std::isfinite(nd->sigma_el_barn[i]))
            return fail(c, PMC_ERR_ARG, "nuclear data: negative or non-finite cross section");
    for (int i = 0; i < kNE; ++i)
        if (nd->sigma_ne_barn[i] != 0.f) return fail(c, PMC_ERR_ARG, "nuclear data: hydrogen has no non-elastic channel");
    for (size_t r = 0; r < nrow; ++r) {
        if (nd->mult_cdf[r * kSecMult + kSecMult - 1] != 1.f) return fail(c, PMC_ERR_ARG, "nuclear data: multiplicity CDF must end at 1");
        for (int m = 0; m + 1 < kSecMult; ++m)
            if (nd->mult_cdf[r * kSecMult + m + 1] < nd->mult_cdf[r * kSecMult + m] || nd->mult_cdf[r * kSecMult + m] < 0.f)
                return fail(c, PMC_ERR_ARG, "nuclear data: multiplicity CDF must not decrease");
        if (nd->x_cdf[r * kSecCdf] != 0.f || nd->x_cdf[r * kSecCdf + 32] != 1.f ||
            nd->mu_cdf[r * kSecCdf] != 0.f || nd->mu_cdf[r * kSecCdf + 32] != 1.f)
            return fail(c, PMC_ERR_ARG, "nuclear data: CDFs must run from 0 to 1");
        for (int i = 0; i < 32; ++i)
            if (nd->x_cdf[r * kSecCdf + i + 1] < nd->x_cdf[r * kSecCdf + i] ||
                nd->mu_cdf[r * kSecCdf + i + 1] < nd->mu_cdf[r * kSecCdf + i])
                return fail(c, PMC_ERR_ARG, "nuclear data: CDFs must not decrease");
        if (!(nd->f_local[r] >= 0.f && nd->f_local[r] <= 1.f)) return fail(c, PMC_ERR_ARG, "nuclear data: f_local outside [0,1]");
    }
    HIPCHK(hipSetDevice(c->device), "set device");
    c->sig_ne.assign(nd->sigma_ne_barn, nd->sigma_ne_barn + ns);
    c->sig_el.assign(nd->sigma_el_barn, nd->sigma_el_barn + ns);
    c->mult.assign(nd->mult_cdf, nd->mult_cdf + nrow * kSecMult);
    c->floc.assign(nd->f_local, nd->f_local + nrow);
    c->xcdf.assign(nd->x_cdf, nd->x_cdf + nrow * kSecCdf);
    c->mucdf.assign(nd->mu_cdf, nd->mu_cdf + nrow * kSecCdf);
    std::vector<float> el(2 * ns);
    std::copy(c->sig_el.begin(), c->sig_el.end(), el.begin());
    std::copy(c->sig_ne.begin(), c->sig_ne.end(), el.begin() + ns);
    // per-element target constants: mass and Eq. 3 coefficients
    std::vector<float> elem(kNEl * 8, 0.f);
    for (int e = 0; e < kNEl; ++e) {
        const double a = kElemMassNumber[e];
        elem[8 * e + 0] = (float)(e == 0 ? kProtonMeV : a * kAmuMeV);
        if (a <= 62) {
            elem[8 * e + 1] = (float)std::pow(a, 1.63);
            elem[8 * e + 2] = (float)(14.5 * std::pow(a, 0.66));
            elem[8 * e + 3] = (float)(1.4 * std::pow(a, 0.33));
        } else {
            elem[8 * e + 1] = (float)std::pow(a, 1.33);
            elem[8 * e + 2] = (float)(60.0 * std::pow(a, 0.33));
            elem[8 * e + 3] = (float)(0.4 * std::pow(a, 0.4));
        }
        elem[8 * e + 4] = 10.f;
    }
    pmc_status s;
    if ((s = upload(c, c->d_el_sig, el, "upload cross sections")) != PMC_OK) return s;
    if ((s = upload(c, c->d_elem, elem, "upload element constants")) != PMC_OK) return s;
    if ((s = upload(c, c->d_mult, c->mult, "upload multiplicities")) != PMC_OK) return s;
    if ((s = upload(c, c->d_floc, c->floc, "upload local fractions")) != PMC_OK) return s;
    if ((s = upload(c, c->d_xcdf, c->xcdf, "upload energy CDFs")) != PMC_OK) return s;
    if ((s = upload(c, c->d_mucdf, c->mucdf, "upload angle CDFs")) != PMC_OK) return s;
    if (c->water.lnr.empty()) c->water = build_range_table(water_z_over_a(), kWaterIeV);
    c->have_phys = true;
    return upload_tables(c);
}

pmc_status pmc_load_geometry(pmc_ctx* c, const int16_t* hu, int nx, int ny, int nz, float dx,
                             float dy, float dz, const pmc_material_table* mt)
{
    if (!c) return PMC_ERR_ARG;
    return load_geometry_common(c, 0, hu, nx, ny, nz, dx, dy, dz, mt);
}

pmc_status pmc_load_geometry_slot(pmc_ctx* c, int* geometry_id_out, const int16_t* hu, int nx, int ny,
                                  int nz, float dx, float dy, float dz, const pmc_material_table* mt)
{
    if (!c) return PMC_ERR_ARG;
    if (!geometry_id_out) return fail(c, PMC_ERR_ARG, "geometry_id_out is NULL");
    if (!have_geometry(c)) return fail(c, PMC_ERR_STATE, "load the base geometry first (pmc_load_geometry)");
    if ((int)c->geoms.size() >= kMaxPlans) return fail(c, PMC_ERR_ARG, "too many geometry slots");
    const int slot = (int)c->geoms.size();
    pmc_status s = load_geometry_common(c, slot, hu, nx, ny, nz, dx, dy, dz, mt);
    if (s != PMC_OK) {
        if ((int)c->geoms.size() > slot) c->geoms.resize(slot);
        return s;
    }
    *geometry_id_out = slot;
    return PMC_OK;
}

pmc_status pmc_inspect_tables(const pmc_ctx* c, float* lnr_w, float* lnr_o, float* sigma_per_g,
                              double* material, int32_t* n_bins)
{
    if (!c) return PMC_ERR_ARG;
    if (!c->have_phys || !have_geometry(c)) return PMC_ERR_STATE;
    const int nm = (int)c->mats.size();
    if (n_bins) *n_bins = nm;
    if (lnr_w) {
        std::copy(c->water.lnr.begin(), c->water.lnr.end(), lnr_w);
        lnr_w[0] = -INFINITY;
    }
    if (lnr_o) {
        if (c->own_bin >= 0) {
            std::copy(c->own.lnr.begin(), c->own.lnr.end(), lnr_o);
            lnr_o[0] = -INFINITY;
        } else {
            std::fill(lnr_o, lnr_o + kNE, 0.f);
        }
    }
    if (sigma_per_g) std::copy(c->blob.begin() + kOffSigma, c->blob.begin() + kOffSigma + 1000 * nm, sigma_per_g);
    if (material)
        for (int m = 0; m < nm; ++m) {
            material[4 * m + 0] = c->mats[m].f;
            material[4 * m + 1] = c->mats[m].x0;
            material[4 * m + 2] = c->mats[m].za;
            material[4 * m + 3] = c->mats[m].own ? 1.0 : 0.0;
        }
    return PMC_OK;
}

pmc_status pmc_geometry_density(pmc_ctx* c, int32_t geometry_id, float* d_rho, void* stream)
{
    if (!c) return PMC_ERR_ARG;
    if (!have_geometry(c)) return fail(c, PMC_ERR_STATE, "density: no geometry loaded");
    if (!d_rho || geometry_id < 0 || geometry_id >= (int32_t)c->geoms.size() || !c->geoms[geometry_id] ||
        c->geoms[geometry_id]->nx <= 0)
        return fail(c, PMC_ERR_ARG, "density: bad geometry id or NULL output");
    HIPCHK(hipSetDevice(c->device), "set device");
    const Geometry& g = *c->geoms[geometry_id];
    HIPCHK(launch_density((const uint2*)g.vox.p, g.nvox(), d_rho, (hipStream_t)stream), "density");
    return PMC_OK;
}

pmc_status pmc_run_spots_dev(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                             uint64_t seed, double* d_dose, double* d_var, void* hip_stream,
                             pmc_summary* summary)
{
    if (!c) return PMC_ERR_ARG;
    if (!d_dose) return fail(c, PMC_ERR_ARG, "d_dose is NULL");
    if (!c->have_phys || !have_geometry(c)) return fail(c, PMC_ERR_STATE, "load physics and geometry first");
    std::vector<PlanIn> plans{{c->geoms[0].get(), spots, n_spots, n_histories, seed, d_dose, d_var, summary,
                               nullptr}};
    return run_plans_impl(c, plans, false, (hipStream_t)hip_stream);
}

pmc_status pmc_run_spots_let_dev(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                                 uint64_t seed, double* d_dose, double* d_var, double* d_let,
                                 void* hip_stream, pmc_summary* summary)
{
    if (!c) return PMC_ERR_ARG;
    if (!d_dose || !d_let) return fail(c, PMC_ERR_ARG, "d_dose or d_let is NULL");
    if (!c->have_phys || !have_geometry(c)) return fail(c, PMC_ERR_STATE, "load physics and geometry first");
    std::vector<PlanIn> plans{{c->geoms[0].get(), spots, n_spots, n_histories, seed, d_dose, d_var, summary,
                               d_let}};
    return run_plans_impl(c, plans, false, (hipStream_t)hip_stream);
}

pmc_status pmc_run_spots(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                         uint64_t seed, double* dose_out, double* var_out, pmc_summary* summary)
{
    if (!c) return PMC_ERR_ARG;
    if (!dose_out || !var_out) return fail(c, PMC_ERR_ARG, "dose/var output is NULL");
    if (!c->have_phys || !have_geometry(c)) return fail(c, PMC_ERR_STATE, "load physics and geometry first");
    HIPCHK(hipSetDevice(c->device), "set device");
    const size_t nv = c->geoms[0]->nvox();
    HIPCHK(c->d_dose.ensure(nv), "alloc dose");
    HIPCHK(c->d_var.ensure(nv), "alloc var");
    std::vector<PlanIn> plans{{c->geoms[0].get(), spots, n_spots, n_histories, seed, c->d_dose.p, c->d_var.p, summary,
                               nullptr}};
    pmc_status s = run_plans_impl(c, plans, false, nullptr);
    if (s != PMC_OK && s != PMC_ERR_QUEUE_OVERFLOW) return s;
    HIPCHK(hipMemcpy(dose_out, c->d_dose.p, nv * 8, hipMemcpyDeviceToHost), "read dose");
    HIPCHK(hipMemcpy(var_out, c->d_var.p, nv * 8, hipMemcpyDeviceToHost), "read variance");
    return s;
}

pmc_status pmc_run_spots_let(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                             uint64_t seed, double* dose_out, double* var_out, double* let_out,
                             pmc_summary* summary)
{
    if (!c) return PMC_ERR_ARG;
    if (!dose_out || !var_out || !let_out) return fail(c, PMC_ERR_ARG, "dose/var/let output is NULL");
    if (!c->have_phys || !have_geometry(c)) return fail(c, PMC_ERR_STATE, "load physics and geometry first");
    HIPCHK(hipSetDevice(c->device), "set device");
    const size_t nv = c->geoms[0]->nvox();
    HIPCHK(c->d_dose.ensure(nv), "alloc dose");
    HIPCHK(c->d_var.ensure(nv), "alloc var");
    HIPCHK(c->d_let.ensure(nv), "alloc let");
    std::vector<PlanIn> plans{{c->geoms[0].get(), spots, n_spots, n_histories, seed, c->d_dose.p, c->d_var.p, summary,
                               c->d_let.p}};
    pmc_status s = run_plans_impl(c, plans, false, nullptr);
    if (s != PMC_OK && s != PMC_ERR_QUEUE_OVERFLOW) return s;
    HIPCHK(hipMemcpy(dose_out, c->d_dose.p, nv * 8, hipMemcpyDeviceToHost), "read dose");
    HIPCHK(hipMemcpy(var_out, c->d_var.p, nv * 8, hipMemcpyDeviceToHost), "read variance");
    HIPCHK(hipMemcpy(let_out, c->d_let.p, nv * 8, hipMemcpyDeviceToHost), "read LET");
    return s;
}

pmc_status pmc_run_plans(pmc_ctx* c, const pmc_plan* plans, int n_plans, uint64_t seed, void* hip_stream)
{
    if (!c) return PMC_ERR_ARG;
    if (!plans || n_plans <= 0 || n_plans > kMaxPlans) return fail(c, PMC_ERR_ARG, "n_plans must be in [1, 64]");
    if (!c->have_phys || !have_geometry(c)) return fail(c, PMC_ERR_STATE, "load physics and geometry first");
    std::vector<PlanIn> v;
    for (int p = 0; p < n_plans; ++p) {
        const pmc_plan& q = plans[p];
        if (q.geometry_id < 0 || q.geometry_id >= (int)c->geoms.size())
            return fail(c, PMC_ERR_ARG, "unknown geometry_id");
        if (!q.d_dose) return fail(c, PMC_ERR_ARG, "plan d_dose is NULL");
        v.push_back({c->geoms[q.geometry_id].get(), q.spots, q.n_spots, q.n_histories, seed + (uint64_t)p,
                     q.d_dose, q.d_var, q.summary, q.d_let});
    }
    return run_plans_impl(c, v, true, (hipStream_t)hip_stream);
}

pmc_status pmc_roofline_replay(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                               uint64_t seed, void* hip_stream, pmc_replay_result* out)
{
    if (!c) return PMC_ERR_ARG;
    if (!out) return fail(c, PMC_ERR_ARG, "out is NULL");
    if (!c->have_phys || !have_geometry(c)) return fail(c, PMC_ERR_STATE, "load physics and geometry first");
    if (n_histories == 0) return fail(c, PMC_ERR_ARG, "n_histories is 0");
    HIPCHK(hipSetDevice(c->device), "set device");
    hipStream_t st = (hipStream_t)hip_stream;
    Geometry& g = *c->geoms[0];
    const size_t nv = g.nvox();
    HIPCHK(c->d_dose.ensure(nv), "alloc dose");
    HIPCHK(c->d_var.ensure(nv), "alloc var");
    pmc_summary s0;
    std::vector<PlanIn> plans{{&g, spots, n_spots, n_histories, seed, c->d_dose.p, c->d_var.p, &s0, nullptr}};
    pmc_status s = run_plans_impl(c, plans, false, st);
    if (s != PMC_OK) return s;
    Shape shape;
    shape.block = s0.block_threads;
    shape.blocks_per_cu = s0.grid_blocks / std::max(1, c->num_cu);
    shape.refill = s0.refill_lanes;
    shape.batch = s0.batch_events;
    shape.cache = s0.cache_slots > 0 ? s0.cache_slots : -1;
    // the traced run, with the same launch shape; iterations per lane from
    // the untraced run's steps, doubled until the trace holds every epoch
    TraceReq tr;
    const unsigned long long lanes = (unsigned long long)s0.grid_blocks * (unsigned long long)s0.block_threads;
    tr.iters = 2 * s0.steps / std::max<unsigned long long>(lanes, 1) + 4096;
    std::vector<uint32_t> epochs;
    for (int attempt = 0;; ++attempt) {
        pmc_summary s1;
        plans[0].summary = &s1;
        RunResult r1;
        s = run_driver(c, plans, false, shape, st, false, &r1, &tr);
        if (s != PMC_OK) { c->d_trace.release(); return s; }
        if (tr.grid != s0.grid_blocks || tr.block != s0.block_threads || s1.steps != s0.steps)
        { c->d_trace.release(); return fail(c, PMC_ERR_DEVICE, "internal: the traced run differs from the run"); }
        epochs.assign(tr.grid, 0u);
        HIPCHK(hipMemcpy(epochs.data(), c->d_trace_epochs.p, tr.grid * 4, hipMemcpyDeviceToHost), "read epochs");
        const unsigned long long need = (unsigned long long)*std::max_element(epochs.begin(), epochs.end()) *
                                        (unsigned long long)tr.epoch_iters;
        if (need <= tr.iters) break;
        if (attempt == 2) { c->d_trace.release(); return fail(c, PMC_ERR_DEVICE, "trace does not fit"); }
        tr.iters = need + 4096;
    }
    HIPCHK(c->d_sink.ensure(2), "alloc sink");
    HIPCHK(launch_zero(c->d_sink.p, 16, st), "zero sink");
    HIPCHK(launch_count_steps(c->d_trace.p, tr.iters * tr.lanes, c->d_sink.p + 1, st), "count trace");
    unsigned long long traced = 0;
    HIPCHK(hipMemcpyAsync(&traced, c->d_sink.p + 1, 8, hipMemcpyDeviceToHost, st), "read count");
    HIPCHK(hipStreamSynchronize(st), "count trace");
    auto timed = [&](int mode, double* ms) -> pmc_status {
        double best = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCHK(hipEventRecord(c->ev0, st), "event");
            HIPCHK(launch_replay(mode, c->d_trace.p, tr.iters, tr.lanes, c->d_trace_epochs.p, tr.epoch_iters,
                                 c->p.k_batches, g.vox.p, g.tally.p, tr.slots, tr.probes, tr.grid, tr.block,
                                 c->d_sink.p, st), "replay launch");
            HIPCHK(hipEventRecord(c->ev1, st), "event");
            HIPCHK(hipEventSynchronize(c->ev1), "replay");
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, c->ev0, c->ev1), "event time");
            best = std::min(best, (double)t);
        }
        *ms = best;
        return PMC_OK;
    };
    std::memset(out, 0, sizeof(*out));
    const int modes[5] = {0, 1, 2, 6, 7};
    double* dst[5] = {&out->trace_only_ms, &out->gather_ms, &out->atomic_ms, &out->cached_atomic_ms,
                      &out->combined_ms};
    for (int i = 0; i < 5; ++i) {
        if (modes[i] >= 6 && tr.slots == 0) {   // no cache in this shape: the direct atomics
            *dst[i] = modes[i] == 6 ? out->atomic_ms : 0.0;
            if (modes[i] == 7 && (s = timed(3, dst[i])) != PMC_OK) { c->d_trace.release(); return s; }
            continue;
        }
        if ((s = timed(modes[i], dst[i])) != PMC_OK) { c->d_trace.release(); return s; }
    }
    c->d_trace.release();
    out->transport_ms = s0.first_launch_ms;
    out->steps = s0.steps;
    out->steps_traced = traced;
    out->deposits = s0.tally_atomics;
    out->trace_iters = tr.iters;
    out->grid_blocks = tr.grid;
    out->block_threads = tr.block;
    out->cache_slots = tr.slots;
    out->epoch_steps = tr.epoch_iters;
    return PMC_OK;
}

static_assert(sizeof(pmc_inc_result) == sizeof(IncResult), "pmc_inc_result mirrors IncResult");
static_assert(sizeof(pmc_inc_particle) == sizeof(IncParticle), "pmc_inc_particle mirrors IncParticle");

pmc_status pmc_inc_events(pmc_ctx* c, const int32_t* element, const double* t_mev, const uint64_t* uid,
                          const uint32_t* ks, int32_t n, uint64_t seed, int32_t evaporate, pmc_inc_result* results,
                          pmc_inc_particle* particles)
{
    if (!c) return PMC_ERR_ARG;
    if (n < 0 || (n > 0 && (!element || !t_mev || !uid || !ks || !results || !particles)))
        return fail(c, PMC_ERR_ARG, "NULL event arrays or outputs, or n < 0");
    for (int i = 0; i < n; ++i) {
        if (element[i] < 1 || element[i] > kIncTargets) return fail(c, PMC_ERR_ARG, "element outside 1..6");
        if (!(t_mev[i] > 0.0 && t_mev[i] <= 1000.0)) return fail(c, PMC_ERR_RANGE, "kinetic energy outside (0, 1000] MeV");
    }
    if (n == 0) return PMC_OK;
    HIPCHK(hipSetDevice(c->device), "set device");
    pmc_status s = ensure_inc(c);
    if (s != PMC_OK) return s;
    DevBuf<int32_t> d_el;
    DevBuf<double> d_t;
    DevBuf<unsigned long long> d_uid;
    DevBuf<uint32_t> d_ks;
    DevBuf<IncResult> d_res;
    DevBuf<IncParticle> d_out;
    DevBuf<unsigned long long> d_ctr;
    HIPCHK(d_el.ensure(n), "alloc events");
    HIPCHK(d_t.ensure(n), "alloc events");
    HIPCHK(d_uid.ensure(n), "alloc events");
    HIPCHK(d_ks.ensure(n), "alloc events");
    HIPCHK(d_res.ensure(n), "alloc results");
    HIPCHK(hipMemset(d_res.p, 0, sizeof(IncResult) * (size_t)n), "clear results");   // (unworked: attempts 0)
    HIPCHK(d_out.ensure((size_t)n * kIncMaxOut), "alloc particles");
    HIPCHK(d_ctr.ensure(8), "alloc claim counters");
    HIPCHK(hipMemset(d_ctr.p, 0, 64), "zero claim counters");
    HIPCHK(hipMemcpy(d_el.p, element, 4 * (size_t)n, hipMemcpyHostToDevice), "upload events");
    HIPCHK(hipMemcpy(d_t.p, t_mev, 8 * (size_t)n, hipMemcpyHostToDevice), "upload events");
    HIPCHK(hipMemcpy(d_uid.p, uid, 8 * (size_t)n, hipMemcpyHostToDevice), "upload events");
    HIPCHK(hipMemcpy(d_ks.p, ks, 4 * (size_t)n, hipMemcpyHostToDevice), "upload events");
    HIPCHK(launch_inc_inspect(c->d_inc_nuc.p, c->d_inc_tab.p, d_el.p, d_t.p, d_uid.p, d_ks.p, n, seed, evaporate, d_ctr.p, d_res.p, d_out.p,
                              nullptr), "cascade launch");
    HIPCHK(hipDeviceSynchronize(), "cascade");
    HIPCHK(hipMemcpy(results, d_res.p, sizeof(IncResult) * (size_t)n, hipMemcpyDeviceToHost), "read results");
    HIPCHK(hipMemcpy(particles, d_out.p, sizeof(IncParticle) * (size_t)n * kIncMaxOut, hipMemcpyDeviceToHost),
           "read particles");
    return PMC_OK;
}

pmc_status pmc_stream_probe(pmc_ctx* c, uint64_t bytes, void* hip_stream, double* read_ms, double* copy_ms)
{
    if (!c) return PMC_ERR_ARG;
    if (!read_ms || !copy_ms || bytes < (1ull << 20) || bytes % 16)
        return fail(c, PMC_ERR_ARG, "bytes must be a multiple of 16 of at least 1 MiB; outputs non-NULL");
    HIPCHK(hipSetDevice(c->device), "set device");
    hipStream_t st = (hipStream_t)hip_stream;
    DevBuf<uint4> a, b;
    HIPCHK(a.ensure(bytes / 16), "alloc probe");
    HIPCHK(b.ensure(bytes / 16), "alloc probe");
    HIPCHK(c->d_sink.ensure(2), "alloc sink");
    HIPCHK(launch_zero(a.p, bytes, st), "fill probe");
    const int grid = 8 * c->num_cu;
    for (int which = 0; which < 2; ++which) {
        double best = 1e300;
        for (int rep = 0; rep < 4; ++rep) {   // the first launch warms up
            HIPCHK(hipEventRecord(c->ev0, st), "event");
            if (which == 0) HIPCHK(launch_stream_read(a.p, bytes, c->d_sink.p, grid, st), "read probe");
            else HIPCHK(launch_copy(a.p, b.p, bytes, grid, st), "copy probe");
            HIPCHK(hipEventRecord(c->ev1, st), "event");
            HIPCHK(hipEventSynchronize(c->ev1), "probe");
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, c->ev0, c->ev1), "event time");
            if (rep > 0) best = std::min(best, (double)t);
        }
        *(which == 0 ? read_ms : copy_ms) = best;
    }
    return PMC_OK;
}

pmc_status pmc_atomic_probe(pmc_ctx* c, uint64_t n_atomics, void* hip_stream, double* ms_out)
{
    if (!c) return PMC_ERR_ARG;
    if (!ms_out || n_atomics == 0) return fail(c, PMC_ERR_ARG, "ms_out is NULL or n_atomics is 0");
    if (!have_geometry(c)) return fail(c, PMC_ERR_STATE, "load a geometry first");
    HIPCHK(hipSetDevice(c->device), "set device");
    hipStream_t st = (hipStream_t)hip_stream;
    const int K = c->p.k_batches;
    Geometry& g = *c->geoms[0];
    HIPCHK(g.tally.ensure(g.nvox() * K), "alloc tally");
    const int grid = c->num_cu * 4;
    const unsigned long long lanes = (unsigned long long)grid * 256;
    const unsigned long long per_lane = (n_atomics + lanes - 1) / lanes;
    HIPCHK(launch_atomic_probe(g.tally.p, g.nx, g.ny, g.nz, K, grid, 1, st), "probe warm-up");
    HIPCHK(hipEventRecord(c->ev0, st), "event");
    HIPCHK(launch_atomic_probe(g.tally.p, g.nx, g.ny, g.nz, K, grid, per_lane, st), "probe launch");
    HIPCHK(hipEventRecord(c->ev1, st), "event");
    HIPCHK(hipEventSynchronize(c->ev1), "probe");
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1), "event time");
    *ms_out = (double)ms * (double)n_atomics / (double)(per_lane * lanes);
    return PMC_OK;
}

}  // extern "C"
