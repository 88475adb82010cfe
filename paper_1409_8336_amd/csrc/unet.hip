// Host side of the dose denoiser (include/pmc_unet.h): parameters,
// activation buffers and the forward / backward / Adam sequences built from
// the kernels in unet_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "pmc_unet.h"

namespace pmc {
hipError_t nn_conv3d_fwd(const uint16_t* in, const uint16_t* wt, const float* bias, uint16_t* out, int N,
                         int D, int H, int W, int Cin, int Cout, int Kp, int relu, hipStream_t s);
hipError_t nn_conv3d_fwd_cat(const uint16_t* in, const uint16_t* coarse, int Cc, const uint16_t* wt,
                             const float* bias, uint16_t* out, int N, int D, int H, int W, int Cin, int Cout,
                             int Kp, int relu, hipStream_t s);
hipError_t nn_flip_weights(const uint16_t* w, uint16_t* wf, int Cin, int Cout, int Kp, int Kpf, hipStream_t s);
hipError_t nn_conv3d_wgrad(const uint16_t* in, const uint16_t* dout, float* dw, int N, int D, int H, int W,
                           int Cin, int Cout, int Kp, hipStream_t s);
hipError_t nn_relu_bias_bwd(uint16_t* dy, const uint16_t* y, float* db, size_t nvox, int C, hipStream_t s);
hipError_t nn_pool_fwd(const uint16_t* in, uint16_t* out, int N, int D, int H, int W, int C, hipStream_t s);
hipError_t nn_pool_bwd(const uint16_t* dout, const uint16_t* add, uint16_t* din, int N, int D, int H, int W, int C,
                       hipStream_t s);
hipError_t nn_up_concat(const uint16_t* coarse, const uint16_t* skip, uint16_t* cat, int N, int D, int H, int W,
                        int Cc, int Cs, hipStream_t s);
hipError_t nn_up_concat_bwd(const uint16_t* dcat, uint16_t* dcoarse, uint16_t* dskip, int N, int D, int H, int W,
                            int Cc, int Cs, hipStream_t s);
hipError_t nn_make_input(const float* dose, const float* rho, float* scale, uint16_t* x, size_t nvox, int N, int D,
                         int H, int W, int d, int h, int w, hipStream_t s);
hipError_t nn_head_fwd(const uint16_t* d1, const float* w, const float* b, const float* dose, const float* scale,
                       float* out, size_t nvox, int C, int D, int H, int W, int d, int h, int wd, hipStream_t s);
hipError_t nn_loss_head_bwd(const float* out, const float* target, const float* dose, const float* scale,
                            unsigned int* region, const uint16_t* d1, const float* w, uint16_t* dd1, float* dw,
                            float* db, double* loss, size_t nvox, int C, hipStream_t s);
hipError_t nn_adam(float* p, float* g, float* m1, float* m2, uint16_t* p_bf, size_t n, float lr, float b1, float b2,
                   float eps, float c1, float c2, float gs, hipStream_t s);
hipError_t nn_sqnorm(const float* g, size_t n, double* out, hipStream_t s);
hipError_t nn_f32_to_bf16(const float* a, uint16_t* b, size_t n, hipStream_t s);
hipError_t nn_mfma_probe(int grid, int iters, float* sink, hipStream_t s);
}  // namespace pmc

using namespace pmc;

// the flipped-weight workspace of pmc_nn_conv3d_backward_data_noalloc (see
// flip_scratch below): 2^20 BF16 entries, 2 MiB
constexpr size_t kFlipScratchElems = size_t(1) << 20;
static __device__ __align__(256) uint16_t scratch[kFlipScratchElems];

namespace {

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Workspace of the data gradient that allocates nothing
// (pmc_nn_conv3d_backward_data_noalloc): the flipped weights [cin][kpf] as
// BF16, at most kFlipScratchElems entries (2 MiB), in a device-resident array
// that every GPU the library runs on holds until the process ends.  Host code
// never passes the array's name to a kernel (on the host it only stands for
// the symbol): the address of each device's copy is looked up once per
// device, with that device current, and used instead.

std::mutex g_scratch_mu;
std::map<int, uint16_t*> g_scratch_ptr;   // device -> address of its copy of scratch

hipError_t flip_scratch(uint16_t** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
        it = g_scratch_ptr.emplace(dev, static_cast<uint16_t*>(ptr)).first;
    }
    *out = it->second;
    return hipSuccess;
}

struct Conv {
    int cin, cout, kp, kpf;
    size_t off_w, off_b;      // offsets in the FP32 parameter vector
    size_t off_wbf;           // offset of the BF16 weights
    size_t off_wf;            // offset of the flipped BF16 weights (data gradient)
};

// one activation / gradient tensor: channels-last BF16 at a level
struct Act {
    uint16_t* p = nullptr;
    size_t nvox = 0;
    int c = 0;
};

}  // namespace

struct pmc_unet {
    int device = 0;
    int N = 0, D = 0, H = 0, W = 0;
    std::string err;
    Conv conv[7];             // enc1..enc4, dec3, dec2, dec1
    size_t n_params = 0, off_hw = 0, off_hb = 0, n_wbf = 0, n_wf = 0;
    float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    uint16_t *wbf = nullptr, *wf = nullptr;
    int step = 0;
    // activations
    Act x, e1, p1, e2, p2, e3, p3, e4, c3, d3, c2, d2, c1, d1;
    // gradients
    Act g_d1, g_c1, g_d2, g_e1s, g_c2, g_d3, g_e2s, g_c3, g_e4, g_e3s, g_p3, g_e3, g_p2, g_e2, g_p1, g_e1;
    float* out = nullptr;     // FP32 network output (denoised dose)
    float* scale = nullptr;
    unsigned int* region = nullptr;   // voxels in the dose region (loss normalisation)
    double* loss = nullptr;
    double* gnorm2 = nullptr;   // squared gradient norm (pmc_unet_grad_norm)
    std::vector<void*> allocs;
};

namespace {

pmc_status ufail(pmc_unet* u, pmc_status s, const std::string& m)
{
    if (u) u->err = m;
    return s;
}

#define UCHK(expr, what)                                                                  \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess)                                                             \
            return ufail(u, _e == hipErrorOutOfMemory ? PMC_ERR_NOMEM : PMC_ERR_DEVICE,   \
                         std::string(what) + ": " + hipGetErrorString(_e));               \
    } while (0)

template <class T>
hipError_t ualloc(pmc_unet* u, T** p, size_t count)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
        u->allocs.push_back(q);
        *p = (T*)q;
    }
    return e;
}

hipError_t act(pmc_unet* u, Act& a, int level, int c)
{
    a.nvox = (size_t)u->N * (u->D >> level) * (u->H >> level) * (u->W >> level);
    a.c = c;
    return ualloc(u, &a.p, a.nvox * c);
}

// runs one convolution of the network: forward
hipError_t conv_fwd(pmc_unet* u, const Conv& c, const Act& in, Act& out, int level, hipStream_t s)
{
    return nn_conv3d_fwd(in.p, u->wbf + c.off_wbf, u->p + c.off_b, out.p, u->N, u->D >> level, u->H >> level,
                         u->W >> level, c.cin, c.cout, c.kp, 1, s);
}

// a decoder convolution whose input is [upsampled coarse, skip]: either from
// the concatenation, formed first (training keeps it for the weight
// gradient), or read from both sources by the convolution itself
hipError_t dec_fwd(pmc_unet* u, const Conv& c, const Act& coarse, const Act& skip, Act& cat, Act& out, int level,
                   bool keep_cat, hipStream_t s)
{
    const int d = u->D >> level, h = u->H >> level, w = u->W >> level;
    if (keep_cat) {
        hipError_t e = nn_up_concat(coarse.p, skip.p, cat.p, u->N, d, h, w, coarse.c, skip.c, s);
        if (e != hipSuccess) return e;
        return conv_fwd(u, c, cat, out, level, s);
    }
    return nn_conv3d_fwd_cat(skip.p, coarse.p, coarse.c, u->wbf + c.off_wbf, u->p + c.off_b, out.p, u->N, d, h, w,
                             c.cin, c.cout, c.kp, 1, s);
}

// backward of one conv + ReLU layer: dy (gradient at the ReLU output, made
// the pre-activation gradient in place), its input x and output y; writes
// the input gradient dx unless dx is NULL
hipError_t conv_bwd(pmc_unet* u, const Conv& c, const Act& x, const Act& y, Act& dy, Act* dx, int level,
                    hipStream_t s)
{
    const int d = u->D >> level, h = u->H >> level, w = u->W >> level;
    hipError_t e;
    if ((e = nn_relu_bias_bwd(dy.p, y.p, u->g + c.off_b, dy.nvox, c.cout, s)) != hipSuccess) return e;
    if ((e = nn_conv3d_wgrad(x.p, dy.p, u->g + c.off_w, u->N, d, h, w, c.cin, c.cout, c.kp, s)) != hipSuccess) return e;
    if (!dx) return hipSuccess;
    if ((e = nn_flip_weights(u->wbf + c.off_wbf, u->wf + c.off_wf, c.cin, c.cout, c.kp, c.kpf, s)) != hipSuccess)
        return e;
    return nn_conv3d_fwd(dy.p, u->wf + c.off_wf, nullptr, dx->p, u->N, d, h, w, c.cout, c.cin, c.kpf, 0, s);
}

// train: keep what the backward pass reads; out: the head's output; the
// caller's grid is d x h x w inside the network's (the whole of it in
// training)
hipError_t forward(pmc_unet* u, const float* dose, const float* rho, bool train, float* out, int d, int h, int w,
                   hipStream_t s)
{
    hipError_t e;
    const size_t nv = u->x.nvox;
    if ((e = hipMemsetAsync(u->scale, 0, sizeof(float), s)) != hipSuccess) return e;
    if ((e = nn_make_input(dose, rho, u->scale, u->x.p, nv, u->N, u->D, u->H, u->W, d, h, w, s)) != hipSuccess)
        return e;
    const int N = u->N, D = u->D, H = u->H, W = u->W;
    if ((e = conv_fwd(u, u->conv[0], u->x, u->e1, 0, s)) != hipSuccess) return e;
    if ((e = nn_pool_fwd(u->e1.p, u->p1.p, N, D, H, W, 16, s)) != hipSuccess) return e;
    if ((e = conv_fwd(u, u->conv[1], u->p1, u->e2, 1, s)) != hipSuccess) return e;
    if ((e = nn_pool_fwd(u->e2.p, u->p2.p, N, D >> 1, H >> 1, W >> 1, 32, s)) != hipSuccess) return e;
    if ((e = conv_fwd(u, u->conv[2], u->p2, u->e3, 2, s)) != hipSuccess) return e;
    if ((e = nn_pool_fwd(u->e3.p, u->p3.p, N, D >> 2, H >> 2, W >> 2, 64, s)) != hipSuccess) return e;
    if ((e = conv_fwd(u, u->conv[3], u->p3, u->e4, 3, s)) != hipSuccess) return e;
    if ((e = dec_fwd(u, u->conv[4], u->e4, u->e3, u->c3, u->d3, 2, train, s)) != hipSuccess) return e;
    if ((e = dec_fwd(u, u->conv[5], u->d3, u->e2, u->c2, u->d2, 1, train, s)) != hipSuccess) return e;
    if ((e = dec_fwd(u, u->conv[6], u->d2, u->e1, u->c1, u->d1, 0, train, s)) != hipSuccess) return e;
    return nn_head_fwd(u->d1.p, u->p + u->off_hw, u->p + u->off_hb, dose, u->scale, out, nv, 16, D, H, W, d, h, w, s);
}

hipError_t backward(pmc_unet* u, const float* dose, const float* target, hipStream_t s)
{
    hipError_t e;
    const int N = u->N, D = u->D, H = u->H, W = u->W;
    const size_t nv = u->x.nvox;
    if ((e = hipMemsetAsync(u->loss, 0, sizeof(double), s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(u->region, 0, sizeof(unsigned int), s)) != hipSuccess) return e;
    if ((e = nn_loss_head_bwd(u->out, target, dose, u->scale, u->region, u->d1.p, u->p + u->off_hw, u->g_d1.p,
                              u->g + u->off_hw, u->g + u->off_hb, u->loss, nv, 16, s)) != hipSuccess)
        return e;
    // dec1: c1 (48) -> d1 (16)
    if ((e = conv_bwd(u, u->conv[6], u->c1, u->d1, u->g_d1, &u->g_c1, 0, s)) != hipSuccess) return e;
    if ((e = nn_up_concat_bwd(u->g_c1.p, u->g_d2.p, u->g_e1s.p, N, D, H, W, 32, 16, s)) != hipSuccess) return e;
    // dec2: c2 (96) -> d2 (32)
    if ((e = conv_bwd(u, u->conv[5], u->c2, u->d2, u->g_d2, &u->g_c2, 1, s)) != hipSuccess) return e;
    if ((e = nn_up_concat_bwd(u->g_c2.p, u->g_d3.p, u->g_e2s.p, N, D >> 1, H >> 1, W >> 1, 64, 32, s)) != hipSuccess)
        return e;
    // dec3: c3 (192) -> d3 (64)
    if ((e = conv_bwd(u, u->conv[4], u->c3, u->d3, u->g_d3, &u->g_c3, 2, s)) != hipSuccess) return e;
    if ((e = nn_up_concat_bwd(u->g_c3.p, u->g_e4.p, u->g_e3s.p, N, D >> 2, H >> 2, W >> 2, 128, 64, s)) != hipSuccess)
        return e;
    // enc4: p3 (64) -> e4 (128)
    if ((e = conv_bwd(u, u->conv[3], u->p3, u->e4, u->g_e4, &u->g_p3, 3, s)) != hipSuccess) return e;
    if ((e = nn_pool_bwd(u->g_p3.p, u->g_e3s.p, u->g_e3.p, N, D >> 2, H >> 2, W >> 2, 64, s)) != hipSuccess) return e;
    // enc3: p2 (32) -> e3 (64)
    if ((e = conv_bwd(u, u->conv[2], u->p2, u->e3, u->g_e3, &u->g_p2, 2, s)) != hipSuccess) return e;
    if ((e = nn_pool_bwd(u->g_p2.p, u->g_e2s.p, u->g_e2.p, N, D >> 1, H >> 1, W >> 1, 32, s)) != hipSuccess) return e;
    // enc2: p1 (16) -> e2 (32)
    if ((e = conv_bwd(u, u->conv[1], u->p1, u->e2, u->g_e2, &u->g_p1, 1, s)) != hipSuccess) return e;
    if ((e = nn_pool_bwd(u->g_p1.p, u->g_e1s.p, u->g_e1.p, N, D, H, W, 16, s)) != hipSuccess) return e;
    // enc1: x (8) -> e1 (16), no input gradient
    return conv_bwd(u, u->conv[0], u->x, u->e1, u->g_e1, nullptr, 0, s);
}

hipError_t refresh_bf16(pmc_unet* u, hipStream_t s)
{
    for (int i = 0; i < 7; ++i) {
        const Conv& c = u->conv[i];
        hipError_t e = nn_f32_to_bf16(u->p + c.off_w, u->wbf + c.off_wbf, (size_t)c.cout * c.kp, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

pmc_status pmc_unet_create(pmc_unet** out, int device, int n, int d, int h, int w, uint64_t seed)
{
    if (!out) return PMC_ERR_ARG;
    if (n < 1 || d < 8 || h < 8 || w < 8 || d % 8 || h % 8 || w % 8) return PMC_ERR_ARG;
    if ((double)n * d * h * w > 2.0e9) return PMC_ERR_ARG;
    pmc_unet* u = new (std::nothrow) pmc_unet();
    if (!u) return PMC_ERR_NOMEM;
    u->device = device;
    u->N = n; u->D = d; u->H = h; u->W = w;
    const int cin[7] = {8, 16, 32, 64, 192, 96, 48};
    const int cout[7] = {16, 32, 64, 128, 64, 32, 16};
    size_t off = 0, offb = 0, offf = 0;
    for (int i = 0; i < 7; ++i) {
        Conv& c = u->conv[i];
        c.cin = cin[i];
        c.cout = cout[i];
        c.kp = round_up(27 * c.cin, 32);
        c.kpf = round_up(27 * c.cout, 32);
        c.off_w = off;
        off += (size_t)c.cout * c.kp;
        c.off_b = off;
        off += c.cout;
        c.off_wbf = offb;
        offb += (size_t)c.cout * c.kp;
        c.off_wf = offf;
        offf += (size_t)c.cin * c.kpf;
    }
    u->off_hw = off;
    off += 16;
    u->off_hb = off;
    off += 1;
    u->n_params = off;
    u->n_wbf = offb;
    u->n_wf = offf;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) { pmc_unet_destroy(u); return PMC_ERR_DEVICE; }
#define A(expr)                                                                       \
    do {                                                                              \
        if ((e = (expr)) != hipSuccess) {                                             \
            pmc_unet_destroy(u);                                                      \
            return e == hipErrorOutOfMemory ? PMC_ERR_NOMEM : PMC_ERR_DEVICE;         \
        }                                                                             \
    } while (0)
    A(ualloc(u, &u->p, u->n_params));
    A(ualloc(u, &u->g, u->n_params));
    A(ualloc(u, &u->m1, u->n_params));
    A(ualloc(u, &u->m2, u->n_params));
    A(ualloc(u, &u->wbf, u->n_wbf));
    A(ualloc(u, &u->wf, u->n_wf));
    A(act(u, u->x, 0, 8));
    A(act(u, u->e1, 0, 16));
    A(act(u, u->p1, 1, 16));
    A(act(u, u->e2, 1, 32));
    A(act(u, u->p2, 2, 32));
    A(act(u, u->e3, 2, 64));
    A(act(u, u->p3, 3, 64));
    A(act(u, u->e4, 3, 128));
    A(act(u, u->c3, 2, 192));
    A(act(u, u->d3, 2, 64));
    A(act(u, u->c2, 1, 96));
    A(act(u, u->d2, 1, 32));
    A(act(u, u->c1, 0, 48));
    A(act(u, u->d1, 0, 16));
    A(act(u, u->g_d1, 0, 16));
    A(act(u, u->g_c1, 0, 48));
    A(act(u, u->g_d2, 1, 32));
    A(act(u, u->g_e1s, 0, 16));
    A(act(u, u->g_c2, 1, 96));
    A(act(u, u->g_d3, 2, 64));
    A(act(u, u->g_e2s, 1, 32));
    A(act(u, u->g_c3, 2, 192));
    A(act(u, u->g_e4, 3, 128));
    A(act(u, u->g_e3s, 2, 64));
    A(act(u, u->g_p3, 3, 64));
    A(act(u, u->g_e3, 2, 64));
    A(act(u, u->g_p2, 2, 32));
    A(act(u, u->g_e2, 1, 32));
    A(act(u, u->g_p1, 1, 16));
    A(act(u, u->g_e1, 0, 16));
    A(ualloc(u, &u->out, u->x.nvox));
    A(ualloc(u, &u->scale, 1));
    A(ualloc(u, &u->region, 1));
    A(ualloc(u, &u->loss, 1));
    A(ualloc(u, &u->gnorm2, 1));
    // initial parameters
    std::vector<float> hp(u->n_params, 0.f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.f, 1.f);
    for (int i = 0; i < 7; ++i) {
        const Conv& c = u->conv[i];
        const int fan_in = 27 * (i == 0 ? 2 : c.cin);
        const float sd = std::sqrt(2.0f / fan_in);
        for (int co = 0; co < c.cout; ++co)
            for (int k = 0; k < 27 * c.cin; ++k) {
                const int ci = k % c.cin;
                hp[c.off_w + (size_t)co * c.kp + k] = (i == 0 && ci >= 2) ? 0.f : sd * nd(rng);
            }
    }
    // the head starts at zero: the network starts as the identity on the
    // input dose and learns the correction
    A(hipMemcpy(u->p, hp.data(), u->n_params * 4, hipMemcpyHostToDevice));
    A(hipMemset(u->g, 0, u->n_params * 4));
    A(hipMemset(u->m1, 0, u->n_params * 4));
    A(hipMemset(u->m2, 0, u->n_params * 4));
    A(refresh_bf16(u, nullptr));
    A(hipDeviceSynchronize());
#undef A
    *out = u;
    return PMC_OK;
}

pmc_status pmc_unet_destroy(pmc_unet* u)
{
    if (!u) return PMC_OK;
    (void)hipSetDevice(u->device);
    for (void* q : u->allocs) (void)hipFree(q);
    delete u;
    return PMC_OK;
}

const char* pmc_unet_last_error(const pmc_unet* u) { return u ? u->err.c_str() : ""; }

pmc_status pmc_unet_param_count(const pmc_unet* u, int64_t* count)
{
    if (!u || !count) return PMC_ERR_ARG;
    *count = (int64_t)u->n_params;
    return PMC_OK;
}

pmc_status pmc_unet_get_params(pmc_unet* u, float* host)
{
    if (!u || !host) return PMC_ERR_ARG;
    UCHK(hipSetDevice(u->device), "set device");
    UCHK(hipMemcpy(host, u->p, u->n_params * 4, hipMemcpyDeviceToHost), "read params");
    return PMC_OK;
}

pmc_status pmc_unet_set_params(pmc_unet* u, const float* host)
{
    if (!u || !host) return PMC_ERR_ARG;
    UCHK(hipSetDevice(u->device), "set device");
    UCHK(hipMemcpy(u->p, host, u->n_params * 4, hipMemcpyHostToDevice), "write params");
    UCHK(refresh_bf16(u, nullptr), "convert weights");
    UCHK(hipDeviceSynchronize(), "convert weights");
    return PMC_OK;
}

pmc_status pmc_unet_get_grads(pmc_unet* u, float* host)
{
    if (!u || !host) return PMC_ERR_ARG;
    UCHK(hipSetDevice(u->device), "set device");
    UCHK(hipMemcpy(host, u->g, u->n_params * 4, hipMemcpyDeviceToHost), "read grads");
    return PMC_OK;
}

pmc_status pmc_unet_zero_grads(pmc_unet* u, void* stream)
{
    if (!u) return PMC_ERR_ARG;
    UCHK(hipSetDevice(u->device), "set device");
    UCHK(hipMemsetAsync(u->g, 0, u->n_params * 4, (hipStream_t)stream), "zero grads");
    return PMC_OK;
}

pmc_status pmc_unet_forward(pmc_unet* u, const float* dose, const float* rho, float* d_out, void* stream)
{
    if (!u) return PMC_ERR_ARG;
    return pmc_unet_forward_region(u, dose, rho, u->D, u->H, u->W, d_out, stream);
}

pmc_status pmc_unet_forward_region(pmc_unet* u, const float* dose, const float* rho, int d, int h, int w,
                                   float* d_out, void* stream)
{
    if (!u) return PMC_ERR_ARG;
    if (!dose || !rho || !d_out) return ufail(u, PMC_ERR_ARG, "NULL tensor");
    if (d < 1 || h < 1 || w < 1 || d > u->D || h > u->H || w > u->W)
        return ufail(u, PMC_ERR_ARG, "the grid must fit inside the network's shape");
    UCHK(hipSetDevice(u->device), "set device");
    hipStream_t s = (hipStream_t)stream;
    UCHK(forward(u, dose, rho, false, d_out, d, h, w, s), "forward");
    return PMC_OK;
}

pmc_status pmc_unet_backward(pmc_unet* u, const float* dose, const float* rho, const float* target,
                             double* loss_out, void* stream)
{
    if (!u) return PMC_ERR_ARG;
    if (!dose || !rho || !target) return ufail(u, PMC_ERR_ARG, "NULL tensor");
    UCHK(hipSetDevice(u->device), "set device");
    hipStream_t s = (hipStream_t)stream;
    UCHK(forward(u, dose, rho, true, u->out, u->D, u->H, u->W, s), "forward");
    UCHK(backward(u, dose, target, s), "backward");
    if (loss_out) {
        UCHK(hipMemcpyAsync(loss_out, u->loss, 8, hipMemcpyDeviceToHost, s), "read loss");
        UCHK(hipStreamSynchronize(s), "backward");
    }
    return PMC_OK;
}

pmc_status pmc_unet_grad_norm(pmc_unet* u, double* norm_out, void* stream)
{
    if (!u) return PMC_ERR_ARG;
    if (!norm_out) return ufail(u, PMC_ERR_ARG, "NULL output");
    UCHK(hipSetDevice(u->device), "set device");
    hipStream_t s = (hipStream_t)stream;
    UCHK(hipMemsetAsync(u->gnorm2, 0, sizeof(double), s), "zero norm");
    UCHK(nn_sqnorm(u->g, u->n_params, u->gnorm2, s), "gradient norm");
    double n2 = 0.0;
    UCHK(hipMemcpyAsync(&n2, u->gnorm2, sizeof(double), hipMemcpyDeviceToHost, s), "read norm");
    UCHK(hipStreamSynchronize(s), "gradient norm");
    *norm_out = std::sqrt(n2);
    return PMC_OK;
}

pmc_status pmc_unet_adam_step(pmc_unet* u, float lr, float grad_scale, void* stream)
{
    if (!u) return PMC_ERR_ARG;
    if (!(lr > 0.f)) return ufail(u, PMC_ERR_ARG, "lr must be > 0");
    if (!(grad_scale > 0.f) || !(grad_scale <= 1.f)) return ufail(u, PMC_ERR_ARG, "grad_scale must be in (0, 1]");
    UCHK(hipSetDevice(u->device), "set device");
    hipStream_t s = (hipStream_t)stream;
    u->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, (float)u->step), c2 = 1.f - std::pow(b2, (float)u->step);
    for (int i = 0; i < 7; ++i) {
        const Conv& c = u->conv[i];
        const size_t nw = (size_t)c.cout * c.kp;
        UCHK(nn_adam(u->p + c.off_w, u->g + c.off_w, u->m1 + c.off_w, u->m2 + c.off_w, u->wbf + c.off_wbf, nw, lr,
                     b1, b2, eps, c1, c2, grad_scale, s), "adam");
        UCHK(nn_adam(u->p + c.off_b, u->g + c.off_b, u->m1 + c.off_b, u->m2 + c.off_b, nullptr, c.cout, lr, b1, b2,
                     eps, c1, c2, grad_scale, s), "adam");
    }
    UCHK(nn_adam(u->p + u->off_hw, u->g + u->off_hw, u->m1 + u->off_hw, u->m2 + u->off_hw, nullptr, 17, lr, b1, b2,
                 eps, c1, c2, grad_scale, s), "adam");
    return PMC_OK;
}

pmc_status pmc_nn_conv3d_forward(const uint16_t* x, const uint16_t* w, const float* bias, uint16_t* y, int n, int d,
                                 int h, int wd, int cin, int cout, int relu, void* stream)
{
    if (!x || !w || !y || n < 1 || d < 1 || h < 1 || wd < 1 || cin < 8 || cout < 8 || cin % 8 || cout % 8)
        return PMC_ERR_ARG;
    hipError_t e = nn_conv3d_fwd(x, w, bias, y, n, d, h, wd, cin, cout, round_up(27 * cin, 32), relu,
                                 (hipStream_t)stream);
    return e == hipSuccess ? PMC_OK : PMC_ERR_DEVICE;
}

pmc_status pmc_nn_conv3d_backward_data(const uint16_t* dy, const uint16_t* w, uint16_t* dx, int n, int d, int h,
                                       int wd, int cin, int cout, void* stream)
{
    if (!dy || !w || !dx || n < 1 || d < 1 || h < 1 || wd < 1 || cin < 8 || cout < 8 || cin % 8 || cout % 8)
        return PMC_ERR_ARG;
    const int kp = round_up(27 * cin, 32), kpf = round_up(27 * cout, 32);
    uint16_t* wf = nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (hipMalloc((void**)&wf, (size_t)cin * kpf * 2) != hipSuccess) return PMC_ERR_NOMEM;
    hipError_t e = nn_flip_weights(w, wf, cin, cout, kp, kpf, s);
    if (e == hipSuccess) e = nn_conv3d_fwd(dy, wf, nullptr, dx, n, d, h, wd, cout, cin, kpf, 0, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(wf);
    return e == hipSuccess ? PMC_OK : PMC_ERR_DEVICE;
}

pmc_status pmc_nn_conv3d_backward_data_noalloc(const uint16_t* dy, const uint16_t* w, uint16_t* dx, int n, int d,
                                               int h, int wd, int cin, int cout, void* stream)
{
    if (!dy || !w || !dx || n < 1 || d < 1 || h < 1 || wd < 1 || cin < 8 || cout < 8 || cin % 8 || cout % 8)
        return PMC_ERR_ARG;
    const int kp = round_up(27 * cin, 32), kpf = round_up(27 * cout, 32);
    // the flipped weights must fit the device-resident workspace
    if ((size_t)cin * (size_t)kpf > kFlipScratchElems) return PMC_ERR_RANGE;
    uint16_t* wf = nullptr;
    if (flip_scratch(&wf) != hipSuccess) return PMC_ERR_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = nn_flip_weights(w, wf, cin, cout, kp, kpf, s);
    if (e == hipSuccess) e = nn_conv3d_fwd(dy, wf, nullptr, dx, n, d, h, wd, cout, cin, kpf, 0, s);
    return e == hipSuccess ? PMC_OK : PMC_ERR_DEVICE;
}

pmc_status pmc_nn_mfma_probe(int32_t iters, void* stream, double* ms_out, double* flop_out)
{
    if (iters < 1 || !ms_out || !flop_out) return PMC_ERR_ARG;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return PMC_ERR_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    const int grid = 8 * cus;   // eight 4-wave workgroups per CU: eight waves per SIMD
    float* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc((void**)&sink, (size_t)grid * 256 * sizeof(float)) != hipSuccess) return PMC_ERR_NOMEM;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {   // the first launch warms up
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = nn_mfma_probe(grid, iters, sink, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e == hipSuccess && rep > 0) best = std::min(best, t);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (e != hipSuccess) return PMC_ERR_DEVICE;
    *ms_out = best;
    *flop_out = (double)grid * 4.0 * (double)iters * 8.0 * 16384.0;
    return PMC_OK;
}

pmc_status pmc_nn_conv3d_backward_weight(const uint16_t* x, const uint16_t* dy, float* dw, int n, int d, int h,
                                         int wd, int cin, int cout, void* stream)
{
    if (!x || !dy || !dw || n < 1 || d < 1 || h < 1 || wd < 1 || cin < 8 || cout < 8 || cin % 8 || cout % 8)
        return PMC_ERR_ARG;
    hipError_t e = nn_conv3d_wgrad(x, dy, dw, n, d, h, wd, cin, cout, round_up(27 * cin, 32), (hipStream_t)stream);
    return e == hipSuccess ? PMC_OK : PMC_ERR_DEVICE;
}

}  // extern "C"
