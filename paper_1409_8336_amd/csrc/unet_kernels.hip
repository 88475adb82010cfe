// Kernels of the 3-D U-Net dose denoiser (gfx950): BF16 activations and
// weights on the matrix cores (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation, channels-last tensors [n][z][y][x][c].
//
// Convolutions are 3x3x3, stride 1, zero padding 1, as implicit GEMMs:
//   forward       out[v][co]  = sum_{tap,ci} in[v+off(tap)][ci] * W[co][tap*Cin+ci]
//   data grad     din[v][ci]  = forward of dout with W'[ci][tap'*Cout+co] = W[co][(26-tap')*Cin+ci]
//   weight grad   dW[co][tap*Cin+ci] = sum_v dout[v][co] * in[v+off(tap)][ci]
// MFMA operand layout (16x16x32, verified on gfx950): lane l holds
// A[l%16][8(l/16)..+7], B[8(l/16)..+7][l%16]; the result D[4(l/16)+i][l%16].
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pmc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#define GLOBAL __attribute__((address_space(1)))
#define LOCAL __attribute__((address_space(3)))

#define DEV __device__ __forceinline__

// negative slope of the leaky ReLU after every convolution
constexpr float kLeak = 0.01f;

DEV float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round-to-nearest-even float -> bf16 bits (finite inputs)
DEV uint16_t f2bf(float f)
{
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

// ------------------------------------------------------------ convolution

// Forward convolution, pipelined through LDS.  A workgroup computes a
// 64 (x) x TY (y) x TZ (z) block of output voxels (TY x TZ = 4R rows; wave w
// owns rows wR .. wR+R-1, each as four 16-voxel M tiles) for 16*NB output
// channels.  The input is consumed 8 channels (one 16-byte voxel entry) at a
// time: the block's halo (66 x (TY+2) x (TZ+2) entries) and the chunk's
// weights (28 taps x 16*NB output channels, tap 27 the zero padding of K to
// 7 x 32) are copied straight from global memory into LDS
// (global_load_lds_dwordx4, out-of-range voxels from a zero page), into one of
// two buffers while the MFMAs read the other, so every operand comes from
// LDS and the copies of chunk c+1 overlap the arithmetic of chunk c (kPipe;
// a one-chunk input uses a single buffer).  K order inside a chunk: 4 taps x
// 8 channels per MFMA K-step (lane group g takes tap 4*s + g), i.e. weight
// column tap*Cin + 8*c + e.  With a coarse source (Cc > 0) the input is the
// decoder's concatenation [nearest upsampling of coarse (Cc channels, half
// resolution), in (Cin - Cc channels)], read from both without forming it.
__device__ const u32x4 kZero16[4] = {};

// TX: tile width in x (64, 32 or 16; a 64-voxel row of a wave covers TX
// voxels in x and 64 / TX in y, so narrow levels waste no lanes)
template <int NB, int R, int TX>
struct FwdTile {
    static constexpr int XT = TX / 16, YR = 4 / XT;          // M tiles per row in x; y values per row
    static constexpr int RY = R >= 2 ? 4 : 2, RZ = R >= 4 ? 4 : 2;   // rows in y, in z
    static constexpr int TY = RY * YR, TZ = RZ;
    static constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
    static constexpr int NHALO = HX * HY * HZ;
    static constexpr int NWT = 28 * 16 * NB;
    static constexpr int NENT = (NHALO + NWT + 63) / 64 * 64;   // whole 64-entry blocks
};

template <int NB, int R, int TX, bool kPipe>
__global__ void __launch_bounds__(256) conv3d_fwd_kernel(const uint16_t* __restrict__ in,
                                                         const uint16_t* __restrict__ coarse, int Cc,
                                                         const uint16_t* __restrict__ wt,
                                                         const float* __restrict__ bias,
                                                         uint16_t* __restrict__ out, int D, int H,
                                                         int W, int Cin, int Cout, int Kp, int relu)
{
    using T = FwdTile<NB, R, TX>;
    // two distinct LDS objects, so that the compiler's wait for the copies
    // into one is not placed before reads of the other
    __shared__ __attribute__((aligned(16))) u32x4 buf0[T::NENT];
    __shared__ __attribute__((aligned(16))) u32x4 buf1[kPipe ? T::NENT : 4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int n_yb = (H + T::TY - 1) / T::TY;
    const int yb = blockIdx.y % n_yb, cg = blockIdx.y / n_yb;
    const int n_zb = (D + T::TZ - 1) / T::TZ;
    const int zb = blockIdx.z % n_zb, n = blockIdx.z / n_zb;
    const int x0 = blockIdx.x * TX, y0 = T::TY * yb, z0 = T::TZ * zb;
    const int co0 = cg * 16 * NB;
    const size_t plane = (size_t)H * W;
    const size_t nbase = (size_t)n * D * plane;
    const int n_chunks = Cin / 8;
    const int Cs = Cin - Cc;   // channels of `in`
    const int Hc = H >> 1, Wc = W >> 1;
    const size_t nbase_c = (size_t)n * (D >> 1) * Hc * Wc;
    // copy chunk c (halo, then weights) into dst: 64-entry blocks dealt to
    // the waves in turn, lane l of a block writing entry 64 * blk + l.  The
    // element offsets of a lane's entries do not depend on the chunk (which
    // only adds 8 c): computed once, -1 for the zero page.
    constexpr int kBlk = T::NENT / 64, kPer = (kBlk + 3) / 4;
    int off_in[kPer], off_co[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int e = (wave + 4 * q) * 64 + lane;
        off_in[q] = -1;
        off_co[q] = -1;
        if (e < T::NHALO) {
            const int hx = e % T::HX, r2 = e / T::HX;
            const int hy = r2 % T::HY, hz = r2 / T::HY;
            const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
            if (x >= 0 && x < W && y >= 0 && y < H && z >= 0 && z < D) {
                off_in[q] = (int)((nbase + (size_t)z * plane + (size_t)y * W + x) * Cs);
                if (Cc) off_co[q] = (int)((nbase_c + ((size_t)(z >> 1) * Hc + (y >> 1)) * Wc + (x >> 1)) * Cc);
            }
        } else if (e < T::NHALO + T::NWT) {
            const int qq = e - T::NHALO, tap = qq / (16 * NB), co = co0 + qq % (16 * NB);
            if (tap < 27 && co < Cout) off_in[q] = co * Kp + tap * Cin;
        }
    }
    auto issue = [&](int c, u32x4* dst) {
        const bool from_coarse = 8 * c < Cc;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int blk = wave + 4 * q;
            if (kBlk % 4 != 0 && blk >= kBlk) break;
            const int e = blk * 64 + lane;
            const GLOBAL void* src = (const GLOBAL void*)&kZero16[0];
            if (e < T::NHALO) {
                if (from_coarse) {
                    if (off_co[q] >= 0) src = (const GLOBAL void*)(coarse + off_co[q] + 8 * c);
                } else if (off_in[q] >= 0) {
                    src = (const GLOBAL void*)(in + off_in[q] + (8 * c - Cc));
                }
            } else if (off_in[q] >= 0) {
                src = (const GLOBAL void*)(wt + off_in[q] + 8 * c);
            }
            __builtin_amdgcn_global_load_lds(src, (LOCAL void*)(dst + blk * 64), 16, 0, 0);
        }
    };
    f32x4 acc[R][4][NB];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[i][t][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    auto compute = [&](const u32x4* bf) {
#pragma unroll
        for (int s = 0; s < 7; ++s) {
            const int tap = 4 * s + g;
            const bool real = tap < 27;
            const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
            bf16x8 b[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) b[j] = __builtin_bit_cast(bf16x8, bf[T::NHALO + tap * 16 * NB + 16 * j + m]);
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = wave * R + i, ry = r % T::RY, rz = r / T::RY;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int xl = 16 * (t % T::XT), yl = ry * T::YR + t / T::XT;
                    // (for the padding tap the index stays inside the buffer;
                    // the entry read is discarded)
                    const u32x4 q = bf[((rz + kz) * T::HY + (yl + ky)) * T::HX + xl + m + kx];
                    const bf16x8 a = real ? __builtin_bit_cast(bf16x8, q) : (bf16x8){};
#pragma unroll
                    for (int j = 0; j < NB; ++j)
                        acc[i][t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][t][j], 0, 0, 0);
                }
            }
        }
    };
    // vmcnt(0), other counters untouched: this wave's copies have landed
    constexpr int kWaitCopies = 0x0F70;
    if constexpr (kPipe) {
        issue(0, buf0);
        for (int c = 0; c < n_chunks; c += 2) {
            __builtin_amdgcn_s_waitcnt(kWaitCopies);
            __syncthreads();   // chunk c in buf0 complete; buf1 no longer read
            if (c + 1 < n_chunks) issue(c + 1, buf1);
            compute(buf0);
            if (c + 1 >= n_chunks) break;
            __builtin_amdgcn_s_waitcnt(kWaitCopies);
            __syncthreads();   // chunk c+1 in buf1 complete; buf0 no longer read
            if (c + 2 < n_chunks) issue(c + 2, buf0);
            compute(buf1);
        }
    } else {
        for (int c = 0; c < n_chunks; ++c) {
            if (c) __syncthreads();   // buf0 no longer read
            issue(c, buf0);
            __builtin_amdgcn_s_waitcnt(kWaitCopies);
            __syncthreads();
            compute(buf0);
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int r = wave * R + i, ry = r % T::RY, z = z0 + r / T::RY;
        if (z >= D) continue;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int co = co0 + 16 * j + m;
            if (co >= Cout) continue;
            const float bv = bias ? bias[co] : 0.f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int y = y0 + ry * T::YR + t / T::XT;
                if (y >= H) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int x = x0 + 16 * (t % T::XT) + 4 * g + q;
                    if (x >= W) continue;
                    float v = acc[i][t][j][q] + bv;
                    if (relu) v = v > 0.f ? v : kLeak * v;
                    out[(nbase + (size_t)z * plane + (size_t)y * W + x) * Cout + co] = f2bf(v);
                }
            }
        }
    }
}

// W'[ci][tap'*Cout + co] = W[co][(26 - tap')*Cin + ci]  (row length Kp')
__global__ void flip_weights_kernel(const uint16_t* __restrict__ w, uint16_t* __restrict__ wf, int Cin,
                                    int Cout, int Kp, int Kpf)
{
    const int total = Cin * Kpf;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int ci = i / Kpf, kk = i - ci * Kpf;
        uint16_t v = 0;
        if (kk < 27 * Cout) {
            const int tp = kk / Cout, co = kk - tp * Cout;
            v = w[(size_t)co * Kp + (26 - tp) * Cin + ci];
        }
        wf[i] = v;
    }
}

// Weight gradient.  Workgroup = (a run of rows) x kz x (32-channel input
// block) x (64-channel output block).  For tap (kz, ky, kx):
//   dW[co][ci] += sum_x dout[x][co] in[x + kx - 1][ci]
//               = sum_x' dout[x' - kx + 1][co] in[x'][ci],
// so per 64-voxel segment of a row the input rows are staged once (aligned,
// no halo) and the output gradient three times, shifted by kx, both
// transposed in LDS (voxel index fastest): every MFMA operand is one aligned
// 16-byte LDS read, A = output-gradient rows (16 channels x 32 voxels), B =
// input columns (32 voxels x 16 channels).  The waves split the 16-channel
// output tiles of the block; where the block has fewer than four of them,
// they also split the two 32-voxel K-steps and the two input tiles.
// Staging: a thread takes an 8-voxel x 8-channel block (one 16-byte load per
// voxel), transposes it in registers and writes eight 16-byte rows (8 voxels
// of one channel) to LDS; the three x-shifted output-gradient copies come
// from one load of 10 voxels, and the block walks its rows with the input
// rows in a three-slot ring (one new row per row where the plane continues).
constexpr int kWgSeg = 64;              // voxels per staged segment (two MFMA K-steps)
constexpr int kWgPitch = kWgSeg + 8;    // LDS row pitch in elements (16-byte multiple)
// kOneCt (Cout <= 16): every wave owns one input tile and one K-step half,
// so it accumulates 9 tiles (the taps) instead of 18: half the accumulator
// registers, three workgroups per CU instead of two
template <bool kOneCt>
__global__ void __launch_bounds__(256) conv3d_wgrad_kernel(const uint16_t* __restrict__ in,
                                                           const uint16_t* __restrict__ dout,
                                                           float* __restrict__ dw, int N, int D,
                                                           int H, int W, int Cin, int Cout, int Kp,
                                                           int rows_per_block)
{
    __shared__ __attribute__((aligned(16))) uint16_t sdo[3][64][kWgPitch];
    __shared__ __attribute__((aligned(16))) uint16_t sin[3][32][kWgPitch];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int n_ci_blk = (Cin + 31) / 32;
    const int kz = blockIdx.y % 3;
    const int cib = (blockIdx.y / 3) % n_ci_blk;
    const int cob = blockIdx.y / (3 * n_ci_blk);
    const int ci0 = cib * 32, co0 = cob * 64;
    // this wave's share: output tile ct, K-steps and input tiles (an input
    // block with 16 channels or fewer has one input tile: the second is
    // neither staged nor multiplied)
    const int n_cot = min(4, (Cout - co0 + 15) / 16);
    const int n_cit = min(2, (Cin - ci0 + 15) / 16);
    int ct, ks_sel = -1, cit_sel = -1;
    if (n_cot >= 3) {
        ct = wave;
    } else if (n_cot == 2) {
        ct = wave & 1;
        ks_sel = wave >> 1;
    } else {
        ct = 0;
        ks_sel = wave & 1;
        cit_sel = wave >> 1;
    }
    const bool active = ct < n_cot && (cit_sel < 0 || cit_sel < n_cit);
    const int total_rows = N * D * H;
    const int row0 = blockIdx.x * rows_per_block;
    const int r_end = min(row0 + rows_per_block, total_rows);
    const size_t plane = (size_t)H * W;
    constexpr int kTiles = kOneCt ? 9 : 18;
    f32x4 acc[kTiles];
#pragma unroll
    for (int t = 0; t < kTiles; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    // 8 voxels of one channel group -> 8 LDS rows (channel c = 2 q + h of
    // voxel j is half h of word q of v[j]; a row packs the voxels in pairs)
    auto put = [](uint16_t* dst, const uint4* v) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t w[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) w[j] = q == 0 ? v[j].x : (q == 1 ? v[j].y : (q == 2 ? v[j].z : v[j].w));
            uint4 lo, hi;
            lo.x = (w[0] & 0xFFFFu) | (w[1] << 16);
            lo.y = (w[2] & 0xFFFFu) | (w[3] << 16);
            lo.z = (w[4] & 0xFFFFu) | (w[5] << 16);
            lo.w = (w[6] & 0xFFFFu) | (w[7] << 16);
            hi.x = (w[0] >> 16) | (w[1] & 0xFFFF0000u);
            hi.y = (w[2] >> 16) | (w[3] & 0xFFFF0000u);
            hi.z = (w[4] >> 16) | (w[5] & 0xFFFF0000u);
            hi.w = (w[6] >> 16) | (w[7] & 0xFFFF0000u);
            *reinterpret_cast<uint4*>(dst + (2 * q) * kWgPitch) = lo;
            *reinterpret_cast<uint4*>(dst + (2 * q + 1) * kWgPitch) = hi;
        }
    };
    // x segments outside, the block's rows inside: the input rows of row r
    // (y + ky - 1, ky < 3) sit in the ring slot (y + ky - 1 + 3) % 3, and the
    // next row of the same plane stages only its new row y + 2
    for (int xb = 0; xb < W; xb += kWgSeg) {
        int prev_nz = -1, prev_y = -2;
        for (int r = row0; r < r_end; ++r) {
            const int y = r % H, nz = r / H, z = nz % D;
            const size_t nbase = (size_t)(nz - z) * plane;
            const int zz = z + kz - 1;
            const bool zin = zz >= 0 && zz < D;
            const bool slide = nz == prev_nz && y == prev_y + 1;
            prev_nz = nz;
            prev_y = y;
            const int n_new = slide ? 1 : 3;            // input rows to stage
            __syncthreads();
            const int i = threadIdx.x;
            if (i < 64) {
                // output gradient of row r, channels co0 + 8 cg .., voxels
                // x = xb + 8 vg - 1 .. + 8 loaded once; copy kx holds slot
                // xp = x - xb + kx - 1 (the voxel x = xb + xp + 1 - kx)
                const int cg = i & 7, vg = i >> 3;
                const int c0 = co0 + 8 * cg;
                if (c0 < Cout) {
                    const uint16_t* src = dout + (nbase + (size_t)z * plane + (size_t)y * W) * Cout + c0;
                    uint4 u[10];
#pragma unroll
                    for (int k = 0; k < 10; ++k) {
                        const int x = xb + 8 * vg - 1 + k;
                        u[k] = make_uint4(0u, 0u, 0u, 0u);
                        if (x >= 0 && x < W) u[k] = *reinterpret_cast<const uint4*>(src + (size_t)x * Cout);
                    }
#pragma unroll
                    for (int kx = 0; kx < 3; ++kx) put(&sdo[kx][8 * cg][8 * vg], u + 2 - kx);
                }
            } else if (i < 64 + 32 * n_new) {
                // input row yy = y + 1 (slide) or y - 1 + k, channels
                // ci0 + 8 cg .., x = xb + 8 vg ..; input rows past Cin
                // inside a used tile are staged as zeros
                const int t = i - 64;
                const int cg = t & 3, vg = (t >> 2) & 7, k = t >> 5;
                if (cg < 2 * n_cit) {
                    const int yy = slide ? y + 1 : y - 1 + k;
                    const int c0 = ci0 + 8 * cg;
                    const bool ok = zin && yy >= 0 && yy < H && c0 < Cin;
                    const uint16_t* src = in + (nbase + (size_t)zz * plane + (size_t)yy * W) * Cin + c0;
                    uint4 v[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int x = xb + 8 * vg + j;
                        v[j] = make_uint4(0u, 0u, 0u, 0u);
                        if (ok && x < W) v[j] = *reinterpret_cast<const uint4*>(src + (size_t)x * Cin);
                    }
                    put(&sin[(yy + 3) % 3][8 * cg][8 * vg], v);
                }
            }
            __syncthreads();
            if (!active) continue;
#pragma unroll
            for (int kh = 0; kh < kWgSeg / 32; ++kh) {
                if (ks_sel >= 0 && kh != ks_sel) continue;
                const int ks = 32 * kh;
                bf16x8 av[3];
#pragma unroll
                for (int kx = 0; kx < 3; ++kx)
                    av[kx] = *reinterpret_cast<const bf16x8*>(&sdo[kx][ct * 16 + m][ks + 8 * g]);
#pragma unroll
                for (int cit = 0; cit < 2; ++cit) {
                    if ((cit_sel >= 0 && cit != cit_sel) || cit >= n_cit) continue;
#pragma unroll
                    for (int ky = 0; ky < 3; ++ky) {
                        const int sl = (y + ky - 1 + 3) % 3;
                        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&sin[sl][cit * 16 + m][ks + 8 * g]);
#pragma unroll
                        for (int kx = 0; kx < 3; ++kx) {
                            const int t = kOneCt ? ky * 3 + kx : (ky * 3 + kx) * 2 + cit;
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[kx], bv, acc[t], 0, 0, 0);
                        }
                    }
                }
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int t = 0; t < kTiles; ++t) {
        const int kyx = kOneCt ? t : t >> 1, cit = kOneCt ? cit_sel : t & 1;
        const int tap = kz * 9 + kyx;
        const int ci = ci0 + cit * 16 + m;
        if (ci >= Cin) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = co0 + ct * 16 + 4 * g + i;
            if (co < Cout && acc[t][i] != 0.f) atomicAdd(&dw[(size_t)co * Kp + tap * Cin + ci], acc[t][i]);
        }
    }
}

// ------------------------------------------------------------ elementwise

// Leaky-ReLU backward through the stored output (which has the sign of the
// pre-activation) and the bias gradient in one pass: dy *= (y > 0 ? 1 :
// kLeak), rounded to BF16 in place, and db[c] += sum_v dy[v][c] of the
// rounded values.  A lane takes 8 channels (16 bytes) of a voxel; the
// block's partial sums meet in LDS, one atomic per (block, channel).
// C is a multiple of 8 with C / 8 dividing 256.
__global__ void __launch_bounds__(256) relu_bias_bwd_kernel(uint16_t* __restrict__ dy,
                                                            const uint16_t* __restrict__ y,
                                                            float* __restrict__ db, size_t nvox, int C)
{
    __shared__ float part[256 * 8];
    const int G = C / 8;                       // channel groups per voxel
    const int g = threadIdx.x % G;
    const int lanes_per_g = blockDim.x / G;
    const int sub = threadIdx.x / G;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (size_t v = (size_t)blockIdx.x * lanes_per_g + sub; v < nvox; v += (size_t)gridDim.x * lanes_per_g) {
        uint4* pd = reinterpret_cast<uint4*>(dy + v * C + 8 * g);
        const uint4 yv = *reinterpret_cast<const uint4*>(y + v * C + 8 * g);
        uint4 dv = *pd;
        uint32_t dw[4] = {dv.x, dv.y, dv.z, dv.w};
        const uint32_t yw[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t out = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint16_t d = (uint16_t)(dw[q] >> (16 * h));
                const uint16_t yy = (uint16_t)(yw[q] >> (16 * h));
                if (!(bf2f(yy) > 0.f)) d = f2bf(kLeak * bf2f(d));
                acc[2 * q + h] += bf2f(d);
                out |= (uint32_t)d << (16 * h);
            }
            dw[q] = out;
        }
        *pd = make_uint4(dw[0], dw[1], dw[2], dw[3]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) part[threadIdx.x * 8 + k] = acc[k];
    __syncthreads();
    if ((int)threadIdx.x < C) {
        const int cg = threadIdx.x / 8, k = threadIdx.x % 8;
        float t = 0.f;
        for (int j = 0; j < lanes_per_g; ++j) t += part[(j * G + cg) * 8 + k];
        atomicAdd(&db[threadIdx.x], t);
    }
}

// 2x2x2 average pooling, channels-last
__global__ void pool_fwd_kernel(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int N, int D,
                                int H, int W, int C)
{
    // 8 channels (16 bytes) per lane; C a multiple of 8; the eight children
    // summed in the same order as element by element
    const int Do = D / 2, Ho = H / 2, Wo = W / 2, C8 = C >> 3;
    const size_t total = (size_t)N * Do * Ho * Wo * C8;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int c8 = (int)(i % C8);
        size_t r = i / C8;
        const int x = (int)(r % Wo); r /= Wo;
        const int y = (int)(r % Ho); r /= Ho;
        const int z = (int)(r % Do);
        const int n = (int)(r / Do);
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const uint4 v = *reinterpret_cast<const uint4*>(
                        in + ((((size_t)n * D + 2 * z + dz) * H + 2 * y + dy) * W + 2 * x + dx) * C + 8 * c8);
                    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int k = 0; k < 8; ++k) acc[k] += bf2f((uint16_t)(w[k >> 1] >> (16 * (k & 1))));
                }
        uint32_t o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            o[q] = (uint32_t)f2bf(0.125f * acc[2 * q]) | ((uint32_t)f2bf(0.125f * acc[2 * q + 1]) << 16);
        *reinterpret_cast<uint4*>(out + 8 * i) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

// d_in[v][c] = add[v][c] + d_out[parent(v)][c] / 8   (add may be NULL)
__global__ void pool_bwd_kernel(const uint16_t* __restrict__ dout, const uint16_t* __restrict__ add,
                                uint16_t* __restrict__ din, int N, int D, int H, int W, int C)
{
    // 8 channels (16 bytes) per lane; C a multiple of 8
    const int C8 = C >> 3;
    const size_t total = (size_t)N * D * H * W * C8;
    const int Ho = H / 2, Wo = W / 2, Do = D / 2;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int c8 = (int)(i % C8);
        size_t r = i / C8;
        const int x = (int)(r % W); r /= W;
        const int y = (int)(r % H); r /= H;
        const int z = (int)(r % D);
        const int n = (int)(r / D);
        const size_t p = ((((size_t)n * Do + z / 2) * Ho + y / 2) * Wo + x / 2) * C + 8 * c8;
        const uint4 dv = *reinterpret_cast<const uint4*>(dout + p);
        const uint4 av = add ? *reinterpret_cast<const uint4*>(add + 8 * i) : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t dw[4] = {dv.x, dv.y, dv.z, dv.w}, aw[4] = {av.x, av.y, av.z, av.w};
        uint32_t ow[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t o = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float v = 0.125f * bf2f((uint16_t)(dw[q] >> (16 * h)));
                if (add) v += bf2f((uint16_t)(aw[q] >> (16 * h)));
                o |= (uint32_t)f2bf(v) << (16 * h);
            }
            ow[q] = o;
        }
        *reinterpret_cast<uint4*>(din + 8 * i) = make_uint4(ow[0], ow[1], ow[2], ow[3]);
    }
}

// cat[v] = (coarse[parent(v)][0..Cc), skip[v][0..Cs))  -- nearest 2x upsampling + concat;
// 8 channels (16 bytes) per lane, Cc and Cs multiples of 8
__global__ void up_concat_kernel(const uint16_t* __restrict__ coarse, const uint16_t* __restrict__ skip,
                                 uint16_t* __restrict__ cat, int N, int D, int H, int W, int Cc, int Cs)
{
    const int C8 = (Cc + Cs) >> 3, Cc8 = Cc >> 3, Cs8 = Cs >> 3;
    const size_t total = (size_t)N * D * H * W * C8;
    const int Ho = H / 2, Wo = W / 2, Do = D / 2;
    const uint4* cs = reinterpret_cast<const uint4*>(coarse);
    const uint4* ss = reinterpret_cast<const uint4*>(skip);
    uint4* dst = reinterpret_cast<uint4*>(cat);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C8);
        const size_t v = i / C8;
        uint4 val;
        if (c < Cc8) {
            size_t r = v;
            const int x = (int)(r % W); r /= W;
            const int y = (int)(r % H); r /= H;
            const int z = (int)(r % D);
            const int n = (int)(r / D);
            val = cs[((((size_t)n * Do + z / 2) * Ho + y / 2) * Wo + x / 2) * Cc8 + c];
        } else {
            val = ss[v * Cs8 + (c - Cc8)];
        }
        dst[i] = val;
    }
}

// backward of up_concat: d_coarse[p][c] = sum over the 8 children of dcat[v][c];
// d_skip[v][c] = dcat[v][Cc + c]
__global__ void up_concat_bwd_coarse_kernel(const uint16_t* __restrict__ dcat, uint16_t* __restrict__ dcoarse,
                                            int N, int D, int H, int W, int Cc, int Cs)
{
    // 8 channels (16 bytes) per lane; Cc and Cs multiples of 8
    const int C = Cc + Cs, Cc8 = Cc >> 3;
    const int Do = D / 2, Ho = H / 2, Wo = W / 2;
    const size_t total = (size_t)N * Do * Ho * Wo * Cc8;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int c8 = (int)(i % Cc8);
        size_t r = i / Cc8;
        const int x = (int)(r % Wo); r /= Wo;
        const int y = (int)(r % Ho); r /= Ho;
        const int z = (int)(r % Do);
        const int n = (int)(r / Do);
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const uint4 v = *reinterpret_cast<const uint4*>(
                        dcat + ((((size_t)n * D + 2 * z + dz) * H + 2 * y + dy) * W + 2 * x + dx) * C + 8 * c8);
                    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int k = 0; k < 8; ++k) acc[k] += bf2f((uint16_t)(w[k >> 1] >> (16 * (k & 1))));
                }
        uint32_t o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = (uint32_t)f2bf(acc[2 * q]) | ((uint32_t)f2bf(acc[2 * q + 1]) << 16);
        *reinterpret_cast<uint4*>(dcoarse + 8 * i) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

__global__ void up_concat_bwd_skip_kernel(const uint16_t* __restrict__ dcat, uint16_t* __restrict__ dskip,
                                          size_t nvox, int Cc, int Cs)
{
    const int C8 = (Cc + Cs) >> 3, Cc8 = Cc >> 3, Cs8 = Cs >> 3;
    const size_t total = nvox * Cs8;
    const uint4* src = reinterpret_cast<const uint4*>(dcat);
    uint4* dst = reinterpret_cast<uint4*>(dskip);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const size_t v = i / Cs8;
        const int c = (int)(i % Cs8);
        dst[i] = src[v * C8 + Cc8 + c];
    }
}

// network input: x[v] = (dose[v] * inv_scale, density[v] * 0.5, 0 x 6)
// Grids: the network's [n][D][H][W] and the caller's compact [n][d][h][w]
// (d <= D, h <= H, w <= W) placed at its origin; outside it the input is
// zero (no dose, density 0) and no output is written.
struct Region {
    int D, H, W, d, h, w;
    // compact index of network voxel v, or -1 outside the caller's grid
    DEV long long compact(size_t v) const
    {
        const int x = (int)(v % W);
        size_t r = v / W;
        const int y = (int)(r % H);
        r /= H;
        const int z = (int)(r % D);
        const size_t n = r / D;
        if (x >= w || y >= h || z >= d) return -1;
        return (long long)(((n * d + z) * h + y) * w + x);
    }
};

__global__ void make_input_kernel(const float* __restrict__ dose, const float* __restrict__ rho,
                                  const float* __restrict__ scale, uint16_t* __restrict__ x, size_t nvox, Region rg)
{
    const float inv = 1.0f / fmaxf(scale[0], 1e-30f);
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < nvox; v += (size_t)gridDim.x * blockDim.x) {
        const long long vc = rg.compact(v);
        uint16_t* o = x + 8 * v;
        o[0] = vc >= 0 ? f2bf(dose[vc] * inv) : (uint16_t)0;
        o[1] = vc >= 0 ? f2bf(rho[vc] * 0.5f) : (uint16_t)0;
#pragma unroll
        for (int c = 2; c < 8; ++c) o[c] = 0;
    }
}

// scale[0] = max_v dose[v]  (non-negative input; scale must start at 0);
// one atomic per block
__global__ void __launch_bounds__(256) max_kernel(const float* __restrict__ a, size_t n, float* __restrict__ scale)
{
    __shared__ float part[4];
    float m = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        m = fmaxf(m, a[i]);
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]));
        atomicMax(reinterpret_cast<unsigned int*>(scale), __float_as_uint(m));
    }
}

// region[0] += number of voxels with dose >= frac * scale (the dose region
// that normalises the loss); one atomic per block
__global__ void __launch_bounds__(256) region_count_kernel(const float* __restrict__ dose, size_t n,
                                                           const float* __restrict__ scale, float frac,
                                                           unsigned int* __restrict__ region)
{
    __shared__ unsigned int part[4];
    const float thr = frac * scale[0];
    unsigned int c = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        c += dose[i] >= thr;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(region, part[0] + part[1] + part[2] + part[3]);
}

// head: out[v] = scale * (dose[v]/scale + sum_c w[c] d1[v][c] + b)  (1x1x1, 16 -> 1, residual)
__global__ void head_fwd_kernel(const uint16_t* __restrict__ d1, const float* __restrict__ w,
                                const float* __restrict__ b, const float* __restrict__ dose,
                                const float* __restrict__ scale, float* __restrict__ out, size_t nvox, int C,
                                Region rg)
{
    const float sc = fmaxf(scale[0], 1e-30f);
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < nvox; v += (size_t)gridDim.x * blockDim.x) {
        const long long vc = rg.compact(v);
        if (vc < 0) continue;
        float s = b[0];
        if (C == 16) {
            // the voxel's 32-byte row in two 16-byte loads (same sum order)
            const uint4* r = reinterpret_cast<const uint4*>(d1 + v * 16);
            const uint4 q0 = r[0], q1 = r[1];
            const uint32_t u[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                s += w[2 * k] * __uint_as_float(u[k] << 16);
                s += w[2 * k + 1] * __uint_as_float(u[k] & 0xFFFF0000u);
            }
        } else {
            for (int c = 0; c < C; ++c) s += w[c] * bf2f(d1[v * C + c]);
        }
        out[vc] = dose[vc] + sc * s;
    }
}

// Squared error in normalised units over the dose region,
// L = sum_v ((out_v - t_v) / scale)^2 / n_region (every voxel contributes;
// n_region, the count of voxels with dose >= 1% of scale, sets the scale of
// the gradients), and the head backward: g_v = dL/d(head pre-activation) =
// 2 (out_v - t_v) / scale / n_region; dd1[v][c] = g_v w[c];
// dw[c] += sum_v g_v d1[v][c]; db += sum_v g_v; loss += L.  C = 16
// channels: one 32-byte row per voxel.  Block partial sums meet in LDS; one
// atomic per block and quantity.
__global__ void __launch_bounds__(256) loss_head_bwd_kernel(const float* __restrict__ out,
                                                            const float* __restrict__ target,
                                                            const float* __restrict__ scale,
                                                            const uint16_t* __restrict__ d1,
                                                            const float* __restrict__ w,
                                                            uint16_t* __restrict__ dd1, float* __restrict__ dw,
                                                            float* __restrict__ db, double* __restrict__ loss,
                                                            size_t nvox, const unsigned int* __restrict__ region)
{
    const float inv_count = 1.0f / (float)max(1u, region[0]);
    __shared__ float sg[4][17];
    __shared__ double sl[4];
    const float sc = fmaxf(scale[0], 1e-30f);
    const float isc = 1.0f / sc;
    float wv[16], gw[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        wv[c] = w[c];
        gw[c] = 0.f;
    }
    float gb = 0.f;
    double l = 0.0;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < nvox; v += (size_t)gridDim.x * blockDim.x) {
        const float e = (out[v] - target[v]) * isc;
        l += (double)e * e;
        const float g = 2.f * e * inv_count;
        gb += g;
        const uint4* src = reinterpret_cast<const uint4*>(d1 + v * 16);
        uint4* dst = reinterpret_cast<uint4*>(dd1 + v * 16);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint4 q = src[h];
            const uint32_t in[4] = {q.x, q.y, q.z, q.w};
            uint32_t o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int c = 8 * h + 2 * k;
                gw[c] += g * __uint_as_float(in[k] << 16);
                gw[c + 1] += g * __uint_as_float(in[k] & 0xFFFF0000u);
                o[k] = (uint32_t)f2bf(g * wv[c]) | ((uint32_t)f2bf(g * wv[c + 1]) << 16);
            }
            dst[h] = make_uint4(o[0], o[1], o[2], o[3]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        gb += __shfl_xor(gb, o);
        l += __shfl_xor(l, o);
#pragma unroll
        for (int c = 0; c < 16; ++c) gw[c] += __shfl_xor(gw[c], o);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int c = 0; c < 16; ++c) sg[wave][c] = gw[c];
        sg[wave][16] = gb;
        sl[wave] = l;
    }
    __syncthreads();
    if (threadIdx.x < 17) {
        const float t = sg[0][threadIdx.x] + sg[1][threadIdx.x] + sg[2][threadIdx.x] + sg[3][threadIdx.x];
        atomicAdd(threadIdx.x < 16 ? &dw[threadIdx.x] : db, t);
    } else if (threadIdx.x == 32) {
        atomicAdd(loss, (sl[0] + sl[1] + sl[2] + sl[3]) * inv_count);
    }
}

// Adam on FP32 master parameters; refreshes the BF16 copies of the
// convolution weights (p_bf == NULL for parameters kept in FP32)
// sum of squares of a float vector into *out (FP64; one atomic per block)
__global__ void __launch_bounds__(256) sqnorm_kernel(const float* __restrict__ g, size_t n, double* out)
{
    __shared__ double part[4];
    double acc = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double v = (double)g[i];
        acc += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = part[0] + part[1] + part[2] + part[3];
        if (t != 0.0) unsafeAtomicAdd(out, t);
    }
}

// Adam on gradient gs * g (gs: the caller's clipping factor, 1 = plain)
__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ g, float* __restrict__ m1,
                            float* __restrict__ m2, uint16_t* __restrict__ p_bf, size_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2, float gs)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = gs * g[i];
        const float a = b1 * m1[i] + (1.f - b1) * gi;
        const float s = b2 * m2[i] + (1.f - b2) * gi * gi;
        m1[i] = a;
        m2[i] = s;
        const float v = p[i] - lr * (a / c1) / (sqrtf(s / c2) + eps);
        p[i] = v;
        g[i] = 0.f;
        if (p_bf) p_bf[i] = f2bf(v);
    }
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ a, uint16_t* __restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = f2bf(a[i]);
}

__global__ void bf16_to_f32_kernel(const uint16_t* __restrict__ a, float* __restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = bf2f(a[i]);
}

// ------------------------------------------------------------ launchers

static unsigned grid_for(size_t n, unsigned block = 256, unsigned cap = 65536)
{
    size_t g = (n + block - 1) / block;
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return (unsigned)g;
}

template <int NB, int TX, bool kPipe>
static hipError_t launch_fwd(const uint16_t* in, const uint16_t* coarse, int Cc, const uint16_t* wt, const float* bias,
                             uint16_t* out, int N, int D, int H, int W, int Cin, int Cout, int Kp, int relu,
                             hipStream_t s)
{
    using T = FwdTile<NB, 1, TX>;
    const int cgroups = (Cout + 16 * NB - 1) / (16 * NB);
    dim3 grid((W + TX - 1) / TX, ((H + T::TY - 1) / T::TY) * cgroups, N * ((D + T::TZ - 1) / T::TZ));
    hipLaunchKernelGGL((conv3d_fwd_kernel<NB, 1, TX, kPipe>), grid, dim3(256), 0, s, in, coarse, Cc, wt, bias, out, D,
                       H, W, Cin, Cout, Kp, relu);
    return hipGetLastError();
}

hipError_t nn_conv3d_fwd_cat(const uint16_t* in, const uint16_t* coarse, int Cc, const uint16_t* wt,
                             const float* bias, uint16_t* out, int N, int D, int H, int W, int Cin, int Cout,
                             int Kp, int relu, hipStream_t s)
{
    // Tiles of 4 rows of 64 voxels (TX in x by 64 / TX in y; two rows in y,
    // two in z); 16 output channels per workgroup (three workgroups per CU)
    // or 32 (two per CU).  The copies in flight per CU set the pace (a
    // 64 x 4 x 2 tile, fewer halo bytes per voxel but two workgroups per CU,
    // was 4% slower at 160 x 128 x 128; 64 x 4 x 4, one workgroup per CU, 19%
    // slower).  A one-chunk input (Cin = 8) is single-buffered.
    if (Cin % 8 || Cin < 8 || Kp < 27 * Cin || Cc % 8 || Cc < 0 || Cc >= Cin || (Cc && !coarse) ||
        (Cc && (D % 2 || H % 2 || W % 2)))
        return hipErrorInvalidValue;
    // the kernel keeps element offsets in 32 bits
    if ((size_t)N * D * H * W * (size_t)Cin >= (size_t)0x7FFFFFFF || (size_t)Cout * Kp >= (size_t)0x7FFFFFFF)
        return hipErrorInvalidValue;
    // tile width: the grid's x extent up to 64
    const int tx = W >= 64 ? 64 : (W >= 32 ? 32 : 16);
#define PMC_FWD(NB, TX, PIPE) \
    launch_fwd<NB, TX, PIPE>(in, coarse, Cc, wt, bias, out, N, D, H, W, Cin, Cout, Kp, relu, s)
    if (Cout <= 16) {
        if (Cin == 8 && tx == 64) return PMC_FWD(1, 64, false);
        if (tx == 64) return PMC_FWD(1, 64, true);
        if (tx == 32) return PMC_FWD(1, 32, true);
        return PMC_FWD(1, 16, true);
    }
    if (tx == 64) return PMC_FWD(2, 64, true);
    if (tx == 32) return PMC_FWD(2, 32, true);
    return PMC_FWD(2, 16, true);
#undef PMC_FWD
}

hipError_t nn_conv3d_fwd(const uint16_t* in, const uint16_t* wt, const float* bias, uint16_t* out, int N,
                         int D, int H, int W, int Cin, int Cout, int Kp, int relu, hipStream_t s)
{
    return nn_conv3d_fwd_cat(in, nullptr, 0, wt, bias, out, N, D, H, W, Cin, Cout, Kp, relu, s);
}

hipError_t nn_flip_weights(const uint16_t* w, uint16_t* wf, int Cin, int Cout, int Kp, int Kpf, hipStream_t s)
{
    hipLaunchKernelGGL(flip_weights_kernel, dim3(grid_for((size_t)Cin * Kpf)), dim3(256), 0, s, w, wf, Cin, Cout, Kp, Kpf);
    return hipGetLastError();
}

hipError_t nn_conv3d_wgrad(const uint16_t* in, const uint16_t* dout, float* dw, int N, int D, int H, int W,
                           int Cin, int Cout, int Kp, hipStream_t s)
{
    const int total_rows = N * D * H;
    const int n_ci = (Cin + 31) / 32, n_co = (Cout + 63) / 64;
    const int others = 3 * n_ci * n_co;
    // enough workgroups to fill the chip, each with a run of rows
    int blocks_x = (2048 + others - 1) / others;
    if (blocks_x > total_rows) blocks_x = total_rows;
    if (blocks_x < 1) blocks_x = 1;
    const int rows = (total_rows + blocks_x - 1) / blocks_x;
    blocks_x = (total_rows + rows - 1) / rows;
    if (Cout <= 16)
        hipLaunchKernelGGL(conv3d_wgrad_kernel<true>, dim3(blocks_x, others), dim3(256), 0, s, in, dout, dw, N, D, H,
                           W, Cin, Cout, Kp, rows);
    else
        hipLaunchKernelGGL(conv3d_wgrad_kernel<false>, dim3(blocks_x, others), dim3(256), 0, s, in, dout, dw, N, D,
                           H, W, Cin, Cout, Kp, rows);
    return hipGetLastError();
}


hipError_t nn_relu_bias_bwd(uint16_t* dy, const uint16_t* y, float* db, size_t nvox, int C, hipStream_t s)
{
    if (C < 8 || C > 256 || C % 8 || 256 % (C / 8)) return hipErrorInvalidValue;
    // a few hundred workgroups: each adds C partial sums to the same C addresses
    hipLaunchKernelGGL(relu_bias_bwd_kernel, dim3(grid_for(nvox, 256 / (C / 8), 512)), dim3(256), 0, s, dy, y, db,
                       nvox, C);
    return hipGetLastError();
}

hipError_t nn_pool_fwd(const uint16_t* in, uint16_t* out, int N, int D, int H, int W, int C, hipStream_t s)
{
    if (C % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pool_fwd_kernel, dim3(grid_for((size_t)N * (D / 2) * (H / 2) * (W / 2) * (C / 8))), dim3(256), 0,
                       s, in, out, N, D, H, W, C);
    return hipGetLastError();
}

hipError_t nn_pool_bwd(const uint16_t* dout, const uint16_t* add, uint16_t* din, int N, int D, int H, int W, int C,
                       hipStream_t s)
{
    if (C % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pool_bwd_kernel, dim3(grid_for((size_t)N * D * H * W * (C / 8))), dim3(256), 0, s, dout, add,
                       din, N, D, H, W, C);
    return hipGetLastError();
}

hipError_t nn_up_concat(const uint16_t* coarse, const uint16_t* skip, uint16_t* cat, int N, int D, int H, int W,
                        int Cc, int Cs, hipStream_t s)
{
    if ((Cc | Cs) & 7) return hipErrorInvalidValue;
    hipLaunchKernelGGL(up_concat_kernel, dim3(grid_for((size_t)N * D * H * W * (Cc + Cs) / 8)), dim3(256), 0, s, coarse,
                       skip, cat, N, D, H, W, Cc, Cs);
    return hipGetLastError();
}

hipError_t nn_up_concat_bwd(const uint16_t* dcat, uint16_t* dcoarse, uint16_t* dskip, int N, int D, int H, int W,
                            int Cc, int Cs, hipStream_t s)
{
    if ((Cc | Cs) & 7) return hipErrorInvalidValue;
    hipLaunchKernelGGL(up_concat_bwd_coarse_kernel, dim3(grid_for((size_t)N * (D / 2) * (H / 2) * (W / 2) * (Cc / 8))),
                       dim3(256), 0, s, dcat, dcoarse, N, D, H, W, Cc, Cs);
    hipLaunchKernelGGL(up_concat_bwd_skip_kernel, dim3(grid_for((size_t)N * D * H * W * Cs / 8)), dim3(256), 0, s, dcat,
                       dskip, (size_t)N * D * H * W, Cc, Cs);
    return hipGetLastError();
}

// nvox: voxels of the network grid; the region gives the caller's (compact)
// grid inside it, whose ncomp = n d h w voxels hold dose and density
hipError_t nn_make_input(const float* dose, const float* rho, float* scale, uint16_t* x, size_t nvox, int N, int D,
                         int H, int W, int d, int h, int w, hipStream_t s)
{
    const Region rg{D, H, W, d, h, w};
    const size_t ncomp = (size_t)N * d * h * w;
    hipLaunchKernelGGL(max_kernel, dim3(grid_for(ncomp, 256, 1024)), dim3(256), 0, s, dose, ncomp, scale);
    hipLaunchKernelGGL(make_input_kernel, dim3(grid_for(nvox)), dim3(256), 0, s, dose, rho, scale, x, nvox, rg);
    return hipGetLastError();
}

hipError_t nn_head_fwd(const uint16_t* d1, const float* w, const float* b, const float* dose, const float* scale,
                       float* out, size_t nvox, int C, int D, int H, int W, int d, int h, int wd, hipStream_t s)
{
    const Region rg{D, H, W, d, h, wd};
    hipLaunchKernelGGL(head_fwd_kernel, dim3(grid_for(nvox)), dim3(256), 0, s, d1, w, b, dose, scale, out, nvox, C, rg);
    return hipGetLastError();
}

hipError_t nn_loss_head_bwd(const float* out, const float* target, const float* dose, const float* scale,
                            unsigned int* region, const uint16_t* d1, const float* w, uint16_t* dd1, float* dw,
                            float* db, double* loss, size_t nvox, int C, hipStream_t s)
{
    if (C != 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(region_count_kernel, dim3(grid_for(nvox, 256, 1024)), dim3(256), 0, s, dose, nvox, scale, 0.01f,
                       region);
    hipLaunchKernelGGL(loss_head_bwd_kernel, dim3(grid_for(nvox, 256, 1024)), dim3(256), 0, s, out, target, scale, d1, w,
                       dd1, dw, db, loss, nvox, (const unsigned int*)region);
    return hipGetLastError();
}

hipError_t nn_adam(float* p, float* g, float* m1, float* m2, uint16_t* p_bf, size_t n, float lr, float b1, float b2,
                   float eps, float c1, float c2, float gs, hipStream_t s)
{
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, g, m1, m2, p_bf, n, lr, b1, b2, eps, c1, c2,
                       gs);
    return hipGetLastError();
}

hipError_t nn_sqnorm(const float* g, size_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(sqnorm_kernel, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, g, n, out);
    return hipGetLastError();
}

hipError_t nn_f32_to_bf16(const float* a, uint16_t* b, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

// Matrix-core throughput probe: every wave issues `iters` rounds of eight
// independent v_mfma_f32_16x16x32_bf16 on register operands (no memory
// traffic in the loop); the accumulators are written out once so that the
// work stays live.  16,384 FLOP per instruction.  The instructions are
// written out so that each accumulates in place: from the builtin the
// register allocator rotated the eight accumulators through other registers
// every iteration (about 18 register moves per 8 MFMAs), which measured the
// moves, not the matrix cores.
__global__ void __launch_bounds__(256) mfma_probe_kernel(int iters, float* __restrict__ sink)
{
    const int lane = threadIdx.x & 63;
    bf16x8 a, b;
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(0.001f * (float)(lane + i));
        b[i] = (__bf16)(0.002f * (float)(lane - i));
    }
    f32x4 acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %2, %0" : "+a"(acc[k]) : "v"(a), "v"(b));
    }
    // the compiler does not track these instructions' results: wait out the
    // last MFMA's passes before the accumulators are read (the accumulators
    // pass through the wait, so no read is scheduled ahead of it)
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7"
                 : "+a"(acc[0]), "+a"(acc[1]), "+a"(acc[2]), "+a"(acc[3]), "+a"(acc[4]), "+a"(acc[5]),
                   "+a"(acc[6]), "+a"(acc[7]));
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) t += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

hipError_t nn_mfma_probe(int grid, int iters, float* sink, hipStream_t s)
{
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(grid), dim3(256), 0, s, iters, sink);
    return hipGetLastError();
}

hipError_t nn_bf16_to_f32(const uint16_t* a, float* b, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(bf16_to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

}  // namespace pmc
