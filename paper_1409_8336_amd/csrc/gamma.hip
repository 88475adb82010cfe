// 3-D gamma index (Low et al.; the paper evaluates its plan re-calculations
// with the 3-D gamma computed on the GPU, Sec. II.D): one reference voxel per
// lane, a cubic search grid around its centre with trilinear interpolation of
// the evaluated distribution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "pmc_unet.h"

namespace pmc {

namespace {

// trilinear interpolation at continuous voxel coordinates (voxel centres at
// integers); the caller keeps the point inside [0, n-1] on every axis
__device__ double trilinear(const double* __restrict__ e, int nx, int ny, int nz, float fx, float fy, float fz)
{
    const int x0 = min((int)fx, nx - 1), y0 = min((int)fy, ny - 1), z0 = min((int)fz, nz - 1);
    const int x1 = min(x0 + 1, nx - 1), y1 = min(y0 + 1, ny - 1), z1 = min(z0 + 1, nz - 1);
    const double tx = fx - x0, ty = fy - y0, tz = fz - z0;
    auto at = [&](int x, int y, int z) { return e[((size_t)z * ny + y) * nx + x]; };
    const double c00 = at(x0, y0, z0) * (1 - tx) + at(x1, y0, z0) * tx;
    const double c10 = at(x0, y1, z0) * (1 - tx) + at(x1, y1, z0) * tx;
    const double c01 = at(x0, y0, z1) * (1 - tx) + at(x1, y0, z1) * tx;
    const double c11 = at(x0, y1, z1) * (1 - tx) + at(x1, y1, z1) * tx;
    const double c0 = c00 * (1 - ty) + c10 * ty, c1 = c01 * (1 - ty) + c11 * ty;
    return c0 * (1 - tz) + c1 * tz;
}

__global__ void max_abs_kernel(const double* __restrict__ a, size_t n, unsigned long long* __restrict__ out)
{
    double m = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        m = fmax(m, a[i]);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0 && m > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void gamma_kernel(const double* __restrict__ ref, const double* __restrict__ ev, int nx, int ny, int nz,
                             float dx, float dy, float dz, const unsigned long long* __restrict__ maxbits,
                             float dose_frac, float dta, float cutoff, float search, float step,
                             float* __restrict__ gamma, unsigned long long* __restrict__ counts)
{
    const double dmax = __longlong_as_double((long long)maxbits[0]);
    const double crit = dose_frac * dmax;
    const int nsteps = (int)floorf(search / step + 1e-4f);
    unsigned long long n_eval = 0, n_pass = 0;
    const size_t nv = (size_t)nx * ny * nz;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < nv; v += (size_t)gridDim.x * blockDim.x) {
        const double r = ref[v];
        if (!(r >= cutoff * dmax) || dmax <= 0.0) {
            if (gamma) gamma[v] = -1.f;
            continue;
        }
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((size_t)nx * ny));
        // the zero offset first (interpolation at a voxel centre is exact), so
        // that every farther offset whose distance term alone exceeds it is
        // skipped without a lookup
        const double d0 = (ev[v] - r) / crit;
        double best = d0 * d0;
        for (int k = -nsteps; k <= nsteps; ++k)
            for (int j = -nsteps; j <= nsteps; ++j)
                for (int i = -nsteps; i <= nsteps; ++i) {
                    const float ox = i * step, oy = j * step, oz = k * step;
                    const float d2 = ox * ox + oy * oy + oz * oz;
                    if (d2 > search * search * (1.0f + 1e-6f)) continue;
                    const double dist = d2 / (dta * dta);
                    if (dist >= best) continue;
                    const float px = x + ox / dx, py = y + oy / dy, pz = z + oz / dz;
                    // points outside the grid carry no evaluated dose: skipped
                    if (px < 0.f || py < 0.f || pz < 0.f || px > nx - 1 || py > ny - 1 || pz > nz - 1) continue;
                    const double e = trilinear(ev, nx, ny, nz, px, py, pz);
                    const double dd = (e - r) / crit;
                    const double g2 = dist + dd * dd;
                    if (g2 < best) best = g2;
                }
        const double g = sqrt(best);
        if (gamma) gamma[v] = (float)g;
        ++n_eval;
        n_pass += g <= 1.0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        n_eval += __shfl_xor(n_eval, o);
        n_pass += __shfl_xor(n_pass, o);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&counts[0], n_eval);
        atomicAdd(&counts[1], n_pass);
    }
}

__global__ void disagreement_kernel(const float* __restrict__ den, const double* __restrict__ mc,
                                    const double* __restrict__ var, size_t n,
                                    const unsigned long long* __restrict__ maxbits, float cutoff, float k,
                                    unsigned long long* __restrict__ counts)
{
    const double thr = cutoff * __longlong_as_double((long long)maxbits[0]);
    unsigned long long above = 0, off = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double m = mc[i];
        if (!(m >= thr) || m <= 0.0) continue;
        ++above;
        off += fabs((double)den[i] - m) > k * sqrt(fmax(var[i], 0.0));
    }
    for (int o = 32; o > 0; o >>= 1) {
        above += __shfl_xor(above, o);
        off += __shfl_xor(off, o);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&counts[0], above);
        atomicAdd(&counts[1], off);
    }
}

// The reduction counters of the two entry points below (maximum and two
// counts): allocated on a device's first call and kept, so that a call
// allocates nothing; the calls are serialised within the process, since
// they share a device's counters until the result has been read back.
std::mutex g_counter_mu;
std::map<int, unsigned long long*> g_counters;

hipError_t device_counters(unsigned long long** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    auto it = g_counters.find(dev);
    if (it == g_counters.end()) {
        unsigned long long* p = nullptr;
        e = hipMalloc((void**)&p, 4 * sizeof(unsigned long long));
        if (e != hipSuccess) return e;
        it = g_counters.emplace(dev, p).first;
    }
    *out = it->second;
    return hipSuccess;
}

}  // namespace

}  // namespace pmc

extern "C" pmc_status pmc_denoise_disagreement(const float* den, const double* mc, const double* var, int64_t n,
                                              float cutoff, float k, double* frac_out, int64_t* n_out, void* stream)
{
    if (!den || !mc || !var || !frac_out || n <= 0 || !(cutoff >= 0) || !(k > 0)) return PMC_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(pmc::g_counter_mu);
    unsigned long long* buf = nullptr;
    if (pmc::device_counters(&buf) != hipSuccess) return PMC_ERR_NOMEM;
    hipError_t e = hipMemsetAsync(buf, 0, 3 * sizeof(unsigned long long), s);
    const unsigned blocks = (unsigned)std::min<size_t>(((size_t)n + 255) / 256, 4096);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pmc::max_abs_kernel, dim3(blocks), dim3(256), 0, s, mc, (size_t)n, buf);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pmc::disagreement_kernel, dim3(blocks), dim3(256), 0, s, den, mc, var, (size_t)n, buf,
                           cutoff, k, buf + 1);
        e = hipGetLastError();
    }
    unsigned long long h[3] = {0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, buf, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return PMC_ERR_DEVICE;
    *frac_out = h[1] ? (double)h[2] / (double)h[1] : 0.0;
    if (n_out) *n_out = (int64_t)h[1];
    return PMC_OK;
}

extern "C" pmc_status pmc_gamma_index(const double* ref, const double* ev, int nx, int ny, int nz, float dx,
                                      float dy, float dz, float dose_frac, float dta, float cutoff, float search,
                                      float step, float* gamma, double* pass_rate, int64_t* n_eval, void* stream)
{
    if (!ref || !ev || !pass_rate || nx <= 0 || ny <= 0 || nz <= 0 || !(dx > 0) || !(dy > 0) || !(dz > 0) ||
        !(dose_frac > 0) || !(dta > 0) || !(cutoff >= 0) || !(search >= 0) || !(step > 0) || search / step > 64)
        return PMC_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(pmc::g_counter_mu);
    unsigned long long* buf = nullptr;
    if (pmc::device_counters(&buf) != hipSuccess) return PMC_ERR_NOMEM;
    const size_t nv = (size_t)nx * ny * nz;
    hipError_t e = hipMemsetAsync(buf, 0, 3 * sizeof(unsigned long long), s);
    unsigned blocks = (unsigned)std::min<size_t>((nv + 255) / 256, 8192);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pmc::max_abs_kernel, dim3(blocks), dim3(256), 0, s, ref, nv, buf);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pmc::gamma_kernel, dim3(blocks), dim3(256), 0, s, ref, ev, nx, ny, nz, dx, dy, dz, buf,
                           dose_frac, dta, cutoff, search, step, gamma, buf + 1);
        e = hipGetLastError();
    }
    unsigned long long h[3] = {0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, buf, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return PMC_ERR_DEVICE;
    *pass_rate = h[1] ? (double)h[2] / (double)h[1] : 1.0;
    if (n_eval) *n_eval = (int64_t)h[1];
    return PMC_OK;
}
