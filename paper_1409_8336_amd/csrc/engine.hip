// C ABI of the engine (include/pmc.h): context and device-buffer ownership,
// uploads of nuclear data and geometry, and the run driver that launches one
// persistent transport grid per secondary generation followed by the
// dose-statistics pass (arXiv:1409.8336, Sec. II.B.2-3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "device.hpp"
#include "pmc.h"
#include "tables.hpp"

namespace pmc {
hipError_t launch_transport(const KernelArgs& a, int grid, int block, size_t lds_bytes, hipStream_t s);
hipError_t transport_occupancy(int block, size_t lds_bytes, int* blocks_per_cu);
hipError_t transport_max_block(int* max_threads);
hipError_t launch_stats(const double* tally, const uint2* vox, unsigned long long nvox, int K,
                        double conv0, double* dose, double* var, double* dep_sum, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
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
};

}  // namespace

struct pmc_ctx {
    int device = 0;
    pmc_params p{};
    std::string err;
    int num_cu = 0;
    bool have_phys = false, have_geom = false;
    // host copies of the nuclear data
    std::vector<float> sig_el, sig_ne, mult, floc, xcdf, mucdf;
    // host tables
    RangeTable water, own;
    std::vector<Material> mats;
    std::vector<float> blob;
    int own_bin = -1;
    // geometry
    int nx = 0, ny = 0, nz = 0;
    float vs[3] = {0, 0, 0};
    DevBuf<uint2> d_vox;
    // device tables
    DevBuf<float> d_blob, d_el_sig, d_npg, d_elem, d_mult, d_floc, d_xcdf, d_mucdf;
    // run buffers
    DevBuf<double> d_tally, d_dose, d_var, d_ledger;
    DevBuf<uint32_t> d_q[2];
    DevBuf<unsigned long long> d_gc, d_counters, d_spot_start;
    DevBuf<float> d_spots;
    unsigned long long* h_pinned = nullptr;   // small pinned read-back area
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_gen[2 * kMaxGenerations] = {};
};

namespace {

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

#define HIPCHK(expr, what)                        \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) return hip_fail(c, _e, what); \
    } while (0)

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

pmc_status upload_tables(pmc_ctx* c)
{
    if (!c->have_phys || !c->have_geom) return PMC_OK;
    build_blob(c);
    HIPCHK(c->d_blob.ensure(c->blob.size()), "alloc tables");
    HIPCHK(hipMemcpy(c->d_blob.p, c->blob.data(), c->blob.size() * 4, hipMemcpyHostToDevice), "upload tables");
    const int nm = (int)c->mats.size();
    std::vector<float> npg(nm * kNEl);
    for (int m = 0; m < nm; ++m)
        for (int e = 0; e < kNEl; ++e) npg[m * kNEl + e] = (float)c->mats[m].nuclei_per_g_barn[e];
    HIPCHK(c->d_npg.ensure(npg.size()), "alloc npg");
    HIPCHK(hipMemcpy(c->d_npg.p, npg.data(), npg.size() * 4, hipMemcpyHostToDevice), "upload npg");
    return PMC_OK;
}

template <class T>
pmc_status upload(pmc_ctx* c, DevBuf<T>& b, const std::vector<T>& v, const char* what)
{
    HIPCHK(b.ensure(v.size()), what);
    HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), what);
    return PMC_OK;
}

bool params_ok(const pmc_params& p, std::string& why)
{
    if (!(p.f_mcs >= 0.0 && p.f_mcs < 10.0)) { why = "f_mcs out of range"; return false; }
    if (!(p.s_min_cm > 0.0 && p.s_min_cm < 1.0)) { why = "s_min_cm out of range"; return false; }
    if (p.k_batches < 2 || p.k_batches > 64) { why = "k_batches must be in [2, 64]"; return false; }
    if (p.flags & ~7u) { why = "unknown flags"; return false; }
    if (p.block_threads != 0 && (p.block_threads < 64 || p.block_threads > 1024 || p.block_threads % 64))
    { why = "block_threads must be 0 or a multiple of 64 in [64, 1024]"; return false; }
    if (p.blocks_per_cu < 0 || p.blocks_per_cu > 64) { why = "blocks_per_cu out of range"; return false; }
    if (p.refill_lanes < 0 || p.refill_lanes > 64) { why = "refill_lanes out of range"; return false; }
    if (p.batch_events < 0 || p.batch_events > 64) { why = "batch_events out of range"; return false; }
    return true;
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
    p->flags = 0;
    p->queue_capacity = 0;
    p->block_threads = 0;
    p->blocks_per_cu = 0;
    p->refill_lanes = 0;
    p->batch_events = 0;
    return PMC_OK;
}

const char* pmc_version(void) { return "pmc 0.1 gfx950"; }

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
    if (c->p.block_threads == 0) c->p.block_threads = 256;
    if (c->p.refill_lanes == 0) c->p.refill_lanes = 16;
    if (c->p.batch_events == 0) c->p.batch_events = 4;
    hipDeviceProp_t prop;
    if ((e = hipSetDevice(device)) != hipSuccess || (e = hipGetDeviceProperties(&prop, device)) != hipSuccess ||
        (e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess ||
        (e = hipHostMalloc((void**)&c->h_pinned, 4096, hipHostMallocDefault)) != hipSuccess) {
        g_create_error = std::string("device setup: ") + hipGetErrorString(e);
        pmc_destroy(c);
        return PMC_ERR_DEVICE;
    }
    for (int i = 0; i < 2 * kMaxGenerations; ++i)
        if ((e = hipEventCreate(&c->ev_gen[i])) != hipSuccess) {
        g_create_error = std::string("device setup: ") + hipGetErrorString(e);
        pmc_destroy(c);
        return PMC_ERR_DEVICE;
    }
    c->num_cu = prop.multiProcessorCount;
    *out = c;
    return PMC_OK;
}

pmc_status pmc_destroy(pmc_ctx* c)
{
    if (!c) return PMC_OK;
    (void)hipSetDevice(c->device);
    c->d_vox.release();
    c->d_blob.release(); c->d_el_sig.release(); c->d_npg.release(); c->d_elem.release();
    c->d_mult.release(); c->d_floc.release(); c->d_xcdf.release(); c->d_mucdf.release();
    c->d_tally.release(); c->d_dose.release(); c->d_var.release(); c->d_ledger.release();
    c->d_q[0].release(); c->d_q[1].release();
    c->d_gc.release(); c->d_counters.release(); c->d_spot_start.release(); c->d_spots.release();
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    for (int i = 0; i < 2 * kMaxGenerations; ++i)
        if (c->ev_gen[i]) (void)hipEventDestroy(c->ev_gen[i]);
    delete c;
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
        if (!(nd->sigma_ne_barn[i] >= 0.f) || !(nd->sigma_el_barn[i] >= 0.f))
            return fail(c, PMC_ERR_ARG, "nuclear data: negative or NaN cross section");
    if (nd->sigma_ne_barn[0 * kNE] != 0.f) {
        for (int i = 0; i < kNE; ++i)
            if (nd->sigma_ne_barn[i] != 0.f) return fail(c, PMC_ERR_ARG, "nuclear data: hydrogen has no non-elastic channel");
    }
    for (size_t r = 0; r < nrow; ++r) {
        if (nd->mult_cdf[r * kSecMult + kSecMult - 1] != 1.f) return fail(c, PMC_ERR_ARG, "nuclear data: multiplicity CDF must end at 1");
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
    if (!hu || !mt) return fail(c, PMC_ERR_ARG, "geometry: NULL pointer");
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(c, PMC_ERR_ARG, "geometry: dimensions must be > 0");
    if (!(dx > 0.f) || !(dy > 0.f) || !(dz > 0.f)) return fail(c, PMC_ERR_ARG, "geometry: voxel size must be > 0");
    if ((double)nx * ny * nz > 4.0e9) return fail(c, PMC_ERR_ARG, "geometry: too many voxels");
    std::vector<Material> mats;
    std::string why = build_materials(mt->n_bins, mt->hu_lo, mt->rho_lo, mt->rho_hi, mt->mass_frac,
                                      mt->i_ev, mt->own_table, mats);
    if (!why.empty()) return fail(c, PMC_ERR_ARG, why);
    HIPCHK(hipSetDevice(c->device), "set device");
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
        float rf = (float)rho;
        uint32_t bits;
        std::memcpy(&bits, &rf, 4);
        rec[v] = make_uint2(bits, (uint32_t)b);
    }
    pmc_status s = upload(c, c->d_vox, rec, "upload voxel records");
    if (s != PMC_OK) return s;
    c->mats = mats;
    c->own_bin = -1;
    for (int b = 0; b < nb; ++b)
        if (mats[b].own) {
            c->own_bin = b;
            c->own = build_range_table(mats[b].za, mats[b].i_ev);
        }
    c->nx = nx; c->ny = ny; c->nz = nz;
    c->vs[0] = dx; c->vs[1] = dy; c->vs[2] = dz;
    if (c->water.lnr.empty()) c->water = build_range_table(water_z_over_a(), kWaterIeV);
    c->have_geom = true;
    return upload_tables(c);
}

pmc_status pmc_inspect_tables(const pmc_ctx* c, float* lnr_w, float* lnr_o, float* sigma_per_g,
                              double* material, int32_t* n_bins)
{
    if (!c) return PMC_ERR_ARG;
    if (!c->have_phys || !c->have_geom) return PMC_ERR_STATE;
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

static pmc_status run_impl(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_hist,
                           uint64_t seed, double* d_dose, double* d_var, hipStream_t st,
                           pmc_summary* summary)
{
    if (!c->have_phys || !c->have_geom) return fail(c, PMC_ERR_STATE, "load physics and geometry first");
    if (n_hist > 0 && (n_spots <= 0 || !spots)) return fail(c, PMC_ERR_ARG, "no spots");
    if (n_spots < 0) return fail(c, PMC_ERR_ARG, "n_spots < 0");
    double wsum = 0.0;
    for (int s = 0; s < n_spots; ++s) {
        const pmc_spot& sp = spots[s];
        if (!(sp.e_mev > (float)kEMin && sp.e_mev <= (float)kEMax)) return fail(c, PMC_ERR_RANGE, "spot energy outside (0.1, 250] MeV");
        if (!(sp.weight >= 0.f) || !(sp.sigma_x_cm >= 0.f) || !(sp.sigma_y_cm >= 0.f) ||
            !std::isfinite(sp.x_cm) || !std::isfinite(sp.y_cm) || !std::isfinite(sp.weight))
            return fail(c, PMC_ERR_RANGE, "spot weight/width must be finite and >= 0");
        wsum += sp.weight;
    }
    if (n_hist > 0 && !(wsum > 0.0)) return fail(c, PMC_ERR_RANGE, "spot weights sum to zero");
    HIPCHK(hipSetDevice(c->device), "set device");
    const int K = c->p.k_batches;
    const size_t nv = (size_t)c->nx * c->ny * c->nz;

    // histories per spot: largest remainder, proportional to weight
    std::vector<unsigned long long> ns(std::max(n_spots, 1), 0), start(n_spots + 1, 0);
    if (n_hist > 0) {
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
    std::vector<float> sp(8 * std::max(n_spots, 1), 0.f);
    double incident = 0.0, wtot = 0.0;
    for (int s = 0; s < n_spots; ++s) {
        start[s + 1] = start[s] + ns[s];
        const double om = ns[s] ? (spots[s].weight / wsum) * (double)n_hist / (double)ns[s] : 0.0;
        const float omf = (float)om;
        sp[8 * s + 0] = spots[s].x_cm / c->vs[0];
        sp[8 * s + 1] = spots[s].y_cm / c->vs[1];
        sp[8 * s + 2] = spots[s].e_mev;
        sp[8 * s + 3] = spots[s].sigma_x_cm / c->vs[0];
        sp[8 * s + 4] = spots[s].sigma_y_cm / c->vs[1];
        sp[8 * s + 5] = omf;
        incident += (double)ns[s] * (double)omf * (double)spots[s].e_mev;
        wtot += (double)ns[s] * (double)omf;
    }
    // buffers
    unsigned long long cap = c->p.queue_capacity ? c->p.queue_capacity
                                                 : std::max<unsigned long long>(65536ull, n_hist);
    HIPCHK(c->d_tally.ensure(nv * K), "alloc tally");
    HIPCHK(c->d_q[0].ensure(cap * kQueuePlanes), "alloc queue");
    HIPCHK(c->d_q[1].ensure(cap * kQueuePlanes), "alloc queue");
    HIPCHK(c->d_gc.ensure(2 * (kMaxGenerations + 2)), "alloc counters");
    HIPCHK(c->d_counters.ensure(8), "alloc counters");
    HIPCHK(c->d_ledger.ensure(8), "alloc ledger");
    HIPCHK(c->d_spots.ensure(sp.size()), "alloc spots");
    HIPCHK(c->d_spot_start.ensure(start.size()), "alloc spots");
    HIPCHK(hipMemcpyAsync(c->d_spots.p, sp.data(), sp.size() * 4, hipMemcpyHostToDevice, st), "upload spots");
    HIPCHK(hipMemcpyAsync(c->d_spot_start.p, start.data(), start.size() * 8, hipMemcpyHostToDevice, st), "upload spots");
    HIPCHK(hipEventRecord(c->ev0, st), "event");
    HIPCHK(launch_zero(c->d_tally.p, nv * K * 8, st), "zero tally");
    HIPCHK(launch_zero(c->d_gc.p, c->d_gc.n * 8, st), "zero counters");
    HIPCHK(launch_zero(c->d_counters.p, 64, st), "zero counters");
    HIPCHK(launch_zero(c->d_ledger.p, 64, st), "zero ledger");

    KernelArgs a{};
    a.vox = c->d_vox.p;
    a.nx = c->nx; a.ny = c->ny; a.nz = c->nz;
    for (int i = 0; i < 3; ++i) { a.vs[i] = c->vs[i]; a.ivs[i] = 1.0f / c->vs[i]; }
    a.blob = c->d_blob.p;
    a.blob_words = (int)c->blob.size();
    a.n_mat = (int)c->mats.size();
    const RangeTable& own = c->own_bin >= 0 ? c->own : c->water;
    a.r_first[0] = (float)c->water.r_first; a.r_first[1] = (float)own.r_first;
    a.ln_r1[0] = (float)c->water.ln_r1; a.ln_r1[1] = (float)own.ln_r1;
    a.inv_step[0] = (float)c->water.inv_step; a.inv_step[1] = (float)own.inv_step;
    a.el_sig = c->d_el_sig.p; a.mat_npg = c->d_npg.p; a.elem = c->d_elem.p;
    a.sec_mult = c->d_mult.p; a.sec_floc = c->d_floc.p; a.sec_x = c->d_xcdf.p; a.sec_mu = c->d_mucdf.p;
    a.seed_lo = (uint32_t)seed; a.seed_hi = (uint32_t)(seed >> 32);
    a.k_batches = K;
    a.flags = c->p.flags;
    a.f_mcs = (float)c->p.f_mcs;
    a.s_min = (float)c->p.s_min_cm;
    a.spots = c->d_spots.p;
    a.spot_start = c->d_spot_start.p;
    a.n_spots = n_spots;
    a.n_primary = n_hist;
    a.q_cap = cap;
    a.gen_counters = c->d_gc.p;
    a.tally = c->d_tally.p;
    a.ledger = c->d_ledger.p;
    a.counters = c->d_counters.p;
    a.refill_lanes = c->p.refill_lanes;
    a.batch_events = c->p.batch_events;

    const int block = c->p.block_threads;
    const size_t lds = c->blob.size() * 4;
    int max_block = 0;
    HIPCHK(transport_max_block(&max_block), "kernel attributes");
    if (block > max_block) return fail(c, PMC_ERR_ARG, "block_threads exceeds the transport kernel's limit");
    int bpc = c->p.blocks_per_cu;
    if (bpc == 0) {
        HIPCHK(transport_occupancy(block, lds, &bpc), "occupancy");
        if (bpc < 1) return fail(c, PMC_ERR_DEVICE, "transport kernel does not fit on a CU");
    } else if (lds > 65536) {
        int dummy;
        HIPCHK(transport_occupancy(block, lds, &dummy), "occupancy");
    }
    const int grid = c->num_cu * bpc;
    int gens = 0;
    unsigned long long produced_total = 0, overflow_n = 0;
    if (n_hist > 0) {
        for (int g = 0;; ++g) {
            if (g >= kMaxGenerations) return fail(c, PMC_ERR_DEVICE, "secondary generations exceed limit");
            a.gen = g;
            a.q_in = c->d_q[g & 1].p;
            a.q_out = c->d_q[(g + 1) & 1].p;
            HIPCHK(hipEventRecord(c->ev_gen[2 * g], st), "event");
            HIPCHK(launch_transport(a, grid, block, lds, st), "transport launch");
            HIPCHK(hipEventRecord(c->ev_gen[2 * g + 1], st), "event");
            ++gens;
            HIPCHK(hipMemcpyAsync(c->h_pinned, c->d_gc.p + 2 * (g + 1), 8, hipMemcpyDeviceToHost, st), "read counters");
            HIPCHK(hipStreamSynchronize(st), "transport");
            const unsigned long long prod = c->h_pinned[0];
            produced_total += prod;
            if (prod > cap) overflow_n += prod - cap;
            if (prod == 0) break;
        }
    }
    const double vol = (double)c->vs[0] * c->vs[1] * c->vs[2];
    const double conv0 = wtot > 0.0 ? 1.602176634e-10 / (vol * wtot) : 0.0;
    HIPCHK(launch_stats(c->d_tally.p, c->d_vox.p, nv, K, conv0, d_dose, d_var, c->d_ledger.p + 3, st), "stats launch");
    HIPCHK(hipEventRecord(c->ev1, st), "event");
    HIPCHK(hipMemcpyAsync(c->h_pinned, c->d_ledger.p, 64, hipMemcpyDeviceToHost, st), "read ledger");
    HIPCHK(hipMemcpyAsync(c->h_pinned + 8, c->d_counters.p, 64, hipMemcpyDeviceToHost, st), "read counters");
    HIPCHK(hipStreamSynchronize(st), "run");
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1), "event time");
    double led[8];
    std::memcpy(led, c->h_pinned, 64);
    double transport_ms = 0.0;
    for (int g = 0; g < gens; ++g) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, c->ev_gen[2 * g], c->ev_gen[2 * g + 1]), "event time");
        transport_ms += t;
    }
    if (summary) {
        std::memset(summary, 0, sizeof(*summary));
        summary->incident = incident;
        summary->escaped = led[0];
        summary->neutral = led[1];
        summary->overflow = led[2];
        summary->deposited = led[3];
        summary->histories = n_hist;
        summary->steps = c->h_pinned[8];
        summary->n_elastic = c->h_pinned[9];
        summary->n_nonelastic = c->h_pinned[10];
        summary->secondaries = produced_total;
        summary->n_overflow = overflow_n;
        summary->n_short_steps = c->h_pinned[11];
        summary->total_weight = wtot;
        summary->device_ms = ms;
        summary->transport_ms = transport_ms;
        summary->generations = gens;
    }
    if (overflow_n) return fail(c, PMC_ERR_QUEUE_OVERFLOW, "secondary queue overflow: raise queue_capacity");
    return PMC_OK;
}

pmc_status pmc_run_spots_dev(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                             uint64_t seed, double* d_dose, double* d_var, void* hip_stream,
                             pmc_summary* summary)
{
    if (!c) return PMC_ERR_ARG;
    if (!d_dose) return fail(c, PMC_ERR_ARG, "d_dose is NULL");
    return run_impl(c, spots, n_spots, n_histories, seed, d_dose, d_var, (hipStream_t)hip_stream, summary);
}

pmc_status pmc_run_spots(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                         uint64_t seed, double* dose_out, double* var_out, pmc_summary* summary)
{
    if (!c) return PMC_ERR_ARG;
    if (!dose_out || !var_out) return fail(c, PMC_ERR_ARG, "dose/var output is NULL");
    if (!c->have_phys || !c->have_geom) return fail(c, PMC_ERR_STATE, "load physics and geometry first");
    HIPCHK(hipSetDevice(c->device), "set device");
    const size_t nv = (size_t)c->nx * c->ny * c->nz;
    HIPCHK(c->d_dose.ensure(nv), "alloc dose");
    HIPCHK(c->d_var.ensure(nv), "alloc var");
    pmc_status s = run_impl(c, spots, n_spots, n_histories, seed, c->d_dose.p, c->d_var.p, nullptr, summary);
    if (s != PMC_OK && s != PMC_ERR_QUEUE_OVERFLOW) return s;
    HIPCHK(hipMemcpy(dose_out, c->d_dose.p, nv * 8, hipMemcpyDeviceToHost), "read dose");
    HIPCHK(hipMemcpy(var_out, c->d_var.p, nv * 8, hipMemcpyDeviceToHost), "read variance");
    return s;
}

}  // extern "C"
