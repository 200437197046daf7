// unet.hip -- warm-start network of the T2-Shuffling solver on gfx950: a 4-level
// U-Net on 2K real channels (NHWC, bf16 activations, fp32 accumulation) whose
// convolutions are implicit GEMMs on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16 in the convolutions, forward and data gradient;
// v_mfma_f32_16x16x16_bf16 in the weight gradients), trained with Adam on solver outputs.
//
// Layer order, shapes and the packed parameter layout (per layer W[KH][KW][Cout][Cin]
// then bias[Cout], forward order) are those of the FP64 reference used by the tests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdint>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/t2s.h"

namespace unetk {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));   // operand type of the 32-deep MFMA
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16;

__host__ __device__ inline bf16 f2bf(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16)((u >> 16) | 0x40);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                        // round to nearest even
    return (bf16)(u >> 16);
}
__host__ __device__ inline float bf2f(bf16 h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

constexpr int kNT = 256;

// D += A B over 32 reduction indices (v_mfma_f32_16x16x32_bf16): lane l supplies
// A[l % 16][8 (l / 16) + r] and B[8 (l / 16) + r][l % 16], r < 8 (layout checked by
// t2s_unet_mfma_probe32)
__device__ __forceinline__ floatx4 mfma32(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, a), __builtin_bit_cast(bf16v8, b), c, 0,
                                                   0, 0);
}
__device__ __forceinline__ void Bv8_load(bf16x8& dst, bool ok, const uint16_t* p) {
    dst = ok ? *(const bf16x8*)p : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
}

// ---------------------------------------------------------------------------
// implicit-GEMM convolution: out[p][co] = bias[co] + sum_{tap, ci} W[tap][co][ci] in[p + off(tap)][ci]
// C[co][p] = A[co][k] B[k][p] with k = (tap, ci); 16x16x16 bf16 MFMA, lane layout:
//   A: lane l holds A[l % 16][4 (l / 16) + r], B: B[4 (l / 16) + r][l % 16],
//   D: D[4 (l / 16) + r][l % 16], r = 0..3.
// Workgroup = 4 waves = 64 output channels x 64 pixels; each wave 32 x 32 (2 x 2 MFMA tiles).
// ---------------------------------------------------------------------------
struct ConvArgs {
    const bf16* in;
    int ldi, ci_off;        // input channel stride and offset
    const bf16* w;          // [KS*KS][coutp][cinp]
    const float* bias;      // [cout_bias] or nullptr
    void* out;
    int ldo, co_off;        // output channel stride and offset
    int B, H, W;            // input grid (output grid equals it, or doubles with shuffle)
    int cinp, coutp;        // padded GEMM sizes (multiples of 16)
    int cout;               // channels actually stored (<= coutp)
    int relu, out_f32, shuffle;
};

template <int KS>
__global__ __launch_bounds__(kNT) void k_conv(ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int P = a.B * a.H * a.W;
    const int co_w = blockIdx.y * 64 + (wave >> 1) * 32;
    const int p_w = blockIdx.x * 64 + (wave & 1) * 32;
    if (co_w >= a.coutp) return;   // whole wave idle (no barriers in this kernel)
    const int r16 = lane & 15, q = lane >> 4;
    // pixel coordinates of the two B column groups this lane loads
    int pb[2], py[2], px[2];
    bool pv[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int p = p_w + j * 16 + r16;
        pv[j] = p < P;
        const int pp = pv[j] ? p : 0;
        px[j] = pp % a.W;
        const int t = pp / a.W;
        py[j] = t % a.H;
        pb[j] = t / a.H;
    }
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int tap = 0; tap < KS * KS; ++tap) {
        const int dy = tap / KS - KS / 2, dx = tap % KS - KS / 2;
        const bf16* src[2];
        bool ok[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int y = py[j] + dy, x = px[j] + dx;
            ok[j] = pv[j] && y >= 0 && y < a.H && x >= 0 && x < a.W;
            src[j] = a.in + ((size_t)(pb[j] * a.H + (ok[j] ? y : 0)) * a.W + (ok[j] ? x : 0)) * a.ldi + a.ci_off;
        }
        const bf16* wt = a.w + (size_t)tap * a.coutp * a.cinp;
        int ci0 = 0;
        // 32 channels per step: each lane loads 8 consecutive channels (16 bytes) of A and B,
        // the operands of one 32-deep MFMA
        for (; ci0 + 32 <= a.cinp; ci0 += 32) {
            const int ci = ci0 + 8 * q;
            bf16x8 A8[2], B8[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int co = co_w + i * 16 + r16;
                A8[i] = co < a.coutp ? *(const bf16x8*)(wt + (size_t)co * a.cinp + ci) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) Bv8_load(B8[j], ok[j], src[j] + ci);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma32(A8[i], B8[j], acc[i][j]);
        }
        for (; ci0 < a.cinp; ci0 += 16) {
            const int ci = ci0 + 4 * q;
            bf16x4 A[2], Bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int co = co_w + i * 16 + r16;
                A[i] = co < a.coutp ? *(const bf16x4*)(wt + (size_t)co * a.cinp + ci) : bf16x4{0, 0, 0, 0};
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) Bv[j] = ok[j] ? *(const bf16x4*)(src[j] + ci) : bf16x4{0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[i], Bv[j], acc[i][j], 0, 0, 0);
        }
    }
    // epilogue: lane holds rows co = co_w + 16 i + 4 q + r of pixel column p_w + 16 j + r16
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (!pv[j]) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int co0 = co_w + i * 16 + 4 * q;
            if (co0 >= a.cout) continue;
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float t = acc[i][j][r];
                if (a.bias) {
                    const int cb = a.shuffle ? (co0 + r) % (a.cout / 4) : co0 + r;
                    t += a.bias[cb];
                }
                if (a.relu) t = fmaxf(t, 0.f);
                v[r] = t;
            }
            size_t base;
            if (a.shuffle) {
                // output channel co4 = (2 i + j) Cout + co goes to pixel (2 y + i, 2 x + j)
                const int cq = a.cout / 4;
                const int sub = co0 / cq, co = co0 - sub * cq;
                const int oy = 2 * py[j] + (sub >> 1), ox = 2 * px[j] + (sub & 1);
                base = ((size_t)(pb[j] * 2 * a.H + oy) * 2 * a.W + ox) * a.ldo + a.co_off + co;
            } else {
                base = (size_t)(p_w + j * 16 + r16) * a.ldo + a.co_off + co0;
            }
            const int nr = min(4, a.cout - co0);
            if (a.out_f32) {
                float* o = (float*)a.out + base;
                for (int r = 0; r < nr; ++r) o[r] = v[r];
            } else {
                bf16* o = (bf16*)a.out + base;
                for (int r = 0; r < nr; ++r) o[r] = f2bf(v[r]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: part[split][tap][co][ci] = sum_{p in split} dout[p][co] in[p + off(tap)][ci]
// GEMM over pixels; tiles of 32 pixels staged through LDS (pixel-major as loaded).
// ---------------------------------------------------------------------------
struct WgradArgs {
    const bf16* dout;
    int ldo, co_off, coutp;
    const bf16* in;
    int ldi, ci_off, cinp;
    int B, H, W, KS;
    float* part;             // [nsplit][KS*KS][coutp][cinp]
    int pix_per_split;
};

__global__ __launch_bounds__(kNT) void k_wgrad(WgradArgs a) {
    constexpr int TP = 32;   // pixels per LDS tile
    __shared__ bf16 sA[TP][64 + 2];
    __shared__ bf16 sB[TP][64 + 2];
    const int taps = a.KS * a.KS;
    const int tap = blockIdx.z % taps, split = blockIdx.z / taps;
    const int dy = tap / a.KS - a.KS / 2, dx = tap % a.KS - a.KS / 2;
    const int co0 = blockIdx.y * 64, ci0 = blockIdx.x * 64;
    const int P = a.B * a.H * a.W;
    const int pbeg = split * a.pix_per_split;
    const int pend = min(P, pbeg + a.pix_per_split);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, q = lane >> 4;
    const int wco = (wave >> 1) * 32, wci = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // loader mapping: 256 threads x 4 channels = 32 pixels x 32 channel quads? -> two passes of 16 pixels
    const int lc = (threadIdx.x & 15) * 4;      // channel quad within the 64-wide tile
    const int lp = threadIdx.x >> 4;            // pixel row 0..15
    for (int p0 = pbeg; p0 < pend; p0 += TP) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int pr = lp + 16 * h;
            const int p = p0 + pr;
            bf16x4 va = bf16x4{0, 0, 0, 0}, vb = bf16x4{0, 0, 0, 0};
            if (p < pend) {
                if (co0 + lc < a.coutp) va = *(const bf16x4*)(a.dout + (size_t)p * a.ldo + a.co_off + co0 + lc);
                const int x = p % a.W, t = p / a.W, y = t % a.H, b = t / a.H;
                const int ys = y + dy, xs = x + dx;
                if (ys >= 0 && ys < a.H && xs >= 0 && xs < a.W && ci0 + lc < a.cinp)
                    vb = *(const bf16x4*)(a.in + ((size_t)(b * a.H + ys) * a.W + xs) * a.ldi + a.ci_off + ci0 + lc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sA[pr][lc + r] = (bf16)va[r];
                sB[pr][lc + r] = (bf16)vb[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < TP; ks += 16) {
            bf16x4 A[2], Bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) A[i][r] = (short)sA[ks + 4 * q + r][wco + 16 * i + r16];
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) Bv[j][r] = (short)sB[ks + 4 * q + r][wci + 16 * j + r16];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[i], Bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    float* out = a.part + ((size_t)split * taps + tap) * a.coutp * a.cinp;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = co0 + wco + 16 * i + 4 * q + r;
                const int ci = ci0 + wci + 16 * j + r16;
                if (co < a.coutp && ci < a.cinp) out[(size_t)co * a.cinp + ci] = acc[i][j][r];
            }
}

// grad[tap][co][ci] (packed, real sizes) = sum over splits of part (padded sizes)
__global__ void k_wgrad_reduce(const float* part, int nsplit, int taps, int coutp, int cinp, int cout, int cin,
                               float* grad) {
    const int n = taps * cout * cin;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ci = i % cin, t = i / cin, co = t % cout, tap = t / cout;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(((size_t)k * taps + tap) * coutp + co) * cinp + ci];
    grad[i] = (float)s;
}

// bias gradient partials: part[split][c] = sum_{p in split} dout[p][co_off + c], c < C.
// The 256 threads cover rows = 256 / C pixels at a time (channel fastest, so a wave
// reads whole pixel rows of channels), each summing every rows-th pixel of the split;
// the rows are then added in LDS in a fixed order.
__global__ void k_bias_part(const bf16* dout, int ldo, int co_off, int C, int P, int pix_per_split, float* part) {
    __shared__ float red[256];
    const int split = blockIdx.x;
    const int p0 = split * pix_per_split, p1 = min(P, p0 + pix_per_split);
    const int tid = threadIdx.x;
    for (int cb = 0; cb < C; cb += 256) {
        const int cw = min(256, C - cb);          // channels of this pass
        const int rows = 256 / cw;
        const int c = cb + tid % cw, row = tid / cw;
        float s = 0.f;
        if (row < rows)
            for (int p = p0 + row; p < p1; p += rows) s += bf2f(dout[(size_t)p * ldo + co_off + c]);
        __syncthreads();
        red[tid] = s;
        __syncthreads();
        if (tid < cw) {
            float t = 0.f;
            for (int r = 0; r < rows; ++r) t += red[r * cw + tid];
            part[(size_t)split * C + cb + tid] = t;
        }
    }
}

// grad_b[c] = sum over splits and `fold` groups of part[split][g * cout + c]: 16
// channels per workgroup, 16 lanes per channel each summing every 16th split (FP64),
// the lane sums combined in a fixed order (deterministic)
constexpr int kBiasCh = 16, kBiasLanes = 16;
__global__ __launch_bounds__(kBiasCh * kBiasLanes) void k_bias_reduce(const float* part, int nsplit, int C, int fold,
                                                                       float* grad) {
    __shared__ double red[kBiasLanes][kBiasCh];
    const int cout = C / fold;
    const int ch = threadIdx.x % kBiasCh, lane = threadIdx.x / kBiasCh;
    const int c = blockIdx.x * kBiasCh + ch;
    double s = 0.0;
    if (c < cout)
        for (int k = lane; k < nsplit; k += kBiasLanes)
            for (int g = 0; g < fold; ++g) s += part[(size_t)k * C + g * cout + c];
    red[lane][ch] = s;
    __syncthreads();
    if (lane == 0 && c < cout) {
        double t = 0.0;
        for (int l = 0; l < kBiasLanes; ++l) t += red[l][ch];
        grad[c] = (float)t;
    }
}

// ---------------------------------------------------------------------------
// elementwise pieces
// ---------------------------------------------------------------------------

// 2x2 max-pool of channels [off, off + C) of in (stride ld) -> out [B][H/2][W/2][C]
__global__ void k_pool(const bf16* in, int ld, int off, int C, int B, int H, int W, bf16* out) {
    const size_t n = (size_t)B * (H / 2) * (W / 2) * C;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = i % C;
    size_t t = i / C;
    const int x = t % (W / 2);
    t /= (W / 2);
    const int y = t % (H / 2);
    const int b = t / (H / 2);
    float m = -INFINITY;
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) m = fmaxf(m, bf2f(in[((size_t)(b * H + 2 * y + dy) * W + 2 * x + dx) * ld + off + c]));
    out[i] = f2bf(m);
}

// dcat[p][off + c] += gradient of the pool routed to the first maximum of its window
__global__ void k_pool_bwd_add(const bf16* fwd, const bf16* dpool, int ld, int off, int C, int B, int H, int W,
                               bf16* dcat) {
    const size_t n = (size_t)B * (H / 2) * (W / 2) * C;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = i % C;
    size_t t = i / C;
    const int x = t % (W / 2);
    t /= (W / 2);
    const int y = t % (H / 2);
    const int b = t / (H / 2);
    float m = -INFINITY;
    int arg = 0;
    for (int k = 0; k < 4; ++k) {
        const float v = bf2f(fwd[((size_t)(b * H + 2 * y + k / 2) * W + 2 * x + k % 2) * ld + off + c]);
        if (v > m) {
            m = v;
            arg = k;
        }
    }
    const size_t o = ((size_t)(b * H + 2 * y + arg / 2) * W + 2 * x + arg % 2) * ld + off + c;
    dcat[o] = f2bf(bf2f(dcat[o]) + bf2f(dpool[i]));
}

// g[p][off + c] *= (y[p][off + c] > 0)
__global__ void k_relu_bwd(bf16* g, const bf16* y, int ld, int off, int C, size_t P) {
    const size_t n = P * C;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t o = (i / C) * ld + off + i % C;
    if (!(bf2f(y[o]) > 0.f)) g[o] = 0;
}

// d4[b][y][x][(2 i + j) C + c] = dup[b][2 y + i][2 x + j][off + c]  (gradient of the 2x2 stride-2 up)
__global__ void k_unshuffle(const bf16* dup, int ld, int off, int C, int B, int H, int W, bf16* d4) {
    const size_t n = (size_t)B * H * W * 4 * C;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c4 = i % (4 * C);
    const size_t p = i / (4 * C);
    const int x = p % W, t = p / W, y = t % H, b = t / H;
    const int sub = c4 / C, c = c4 % C;
    d4[i] = dup[((size_t)(b * 2 * H + 2 * y + sub / 2) * 2 * W + 2 * x + sub % 2) * ld + off + c];
}

// per-slice scale s = max |b0| (FP64 reduction per slice, one workgroup per slice)
// scale[s] = max |b0| over slice s (0 for an all-zero slice): k_zero_scale, then
// kScaleBlocks workgroups per slice fold their maxima in with an integer atomic max
// (non-negative floats order like their bit patterns)
constexpr int kScaleBlocks = 64;
__global__ void k_zero_scale(float* scale, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) scale[i] = 0.f;
}

__global__ void k_slice_scale(const float2* b0, int K, int N, float* scale) {
    __shared__ float red[kNT];
    const int s = blockIdx.y;
    const size_t n = (size_t)K * N;
    const float2* v0 = b0 + (size_t)s * n;
    float m = 0.f;
    for (size_t i = (size_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (size_t)kScaleBlocks * kNT) {
        const float2 v = v0[i];
        m = fmaxf(m, sqrtf(v.x * v.x + v.y * v.y));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = kNT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax((unsigned int*)scale + s, __float_as_uint(red[0]));
}

// complex [S][K][H][W] / scale[s] -> fp32 [S][H][W][2K] and bf16 [S][H][W][ldb] (zero padded)
__global__ void k_pack(const float2* src, const float* scale, int K, int HW, float* x32, bf16* xb, int ldb) {
    const size_t n = (size_t)gridDim.y * HW;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= (size_t)HW) return;
    const float inv = scale[s] > 0.f ? 1.f / scale[s] : 0.f;
    const size_t p = (size_t)s * HW + i;
    for (int k = 0; k < K; ++k) {
        const float2 v = src[((size_t)s * K + k) * HW + i];
        if (x32) {
            x32[p * 2 * K + 2 * k] = v.x * inv;
            x32[p * 2 * K + 2 * k + 1] = v.y * inv;
        }
        if (xb) {
            xb[p * ldb + 2 * k] = f2bf(v.x * inv);
            xb[p * ldb + 2 * k + 1] = f2bf(v.y * inv);
        }
    }
    if (xb)
        for (int c = 2 * K; c < ldb; ++c) xb[p * ldb + c] = 0;
    (void)n;
}

// alpha0[s][k][i] = scale[s] (x + y)[s][i][2k, 2k+1]  (an all-zero input slice has
// scale 0 and gets alpha0 = 0: the solution for no data is zero)
__global__ void k_unpack(const float* x32, const float* y32, int ldy, const float* scale, int K, int HW, float2* dst) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= (size_t)HW) return;
    const size_t p = (size_t)s * HW + i;
    for (int k = 0; k < K; ++k) {
        const float re = x32[p * 2 * K + 2 * k] + y32[p * ldy + 2 * k];
        const float im = x32[p * 2 * K + 2 * k + 1] + y32[p * ldy + 2 * k + 1];
        dst[((size_t)s * K + k) * HW + i] = make_float2(scale[s] * re, scale[s] * im);
    }
}

// MSE: d = x + y - t over the 2K channels; dy (bf16, ld) = 2 d / n; partial sums of d^2
__global__ void k_mse(const float* x32, const float* y32, int ldy, const float* t32, int C, size_t P, float inv_n,
                      bf16* dy, int lddy, double* part) {
    __shared__ double red[kNT];
    double acc = 0.0;
    for (size_t p = (size_t)blockIdx.x * kNT + threadIdx.x; p < P; p += (size_t)gridDim.x * kNT) {
        for (int c = 0; c < lddy; ++c) {
            float g = 0.f;
            if (c < C) {
                const float d = x32[p * C + c] + y32[p * ldy + c] - t32[p * C + c];
                acc += (double)d * d;
                g = 2.f * d * inv_n;
            }
            dy[p * lddy + c] = f2bf(g);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kNT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// bf16 compute weights from the fp32 master copy: forward [tap][coutp][cinp] and the
// data-gradient weights [tap'][cinp][coutp] with tap' the point-reflected tap.
__global__ void k_prep(const float* master, int KS, int cout, int cin, int coutp, int cinp, bf16* wf, bf16* wb) {
    const int taps = KS * KS;
    const size_t n = (size_t)taps * coutp * cinp;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ci = i % cinp;
    const size_t t = i / cinp;
    const int co = t % coutp, tap = t / coutp;
    const float v = (co < cout && ci < cin) ? master[((size_t)tap * cout + co) * cin + ci] : 0.f;
    wf[i] = f2bf(v);
    if (wb) wb[((size_t)(taps - 1 - tap) * cinp + ci) * coutp + co] = f2bf(v);
}

// omb1 = 1 - b1, omb2 = 1 - b2 and the bias corrections c1, c2 come from the host in
// double precision (1 - b2 formed in fp32 from 0.999f would be off by 1.3e-5)
__global__ void k_adam(float* w, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2,
                       float omb1, float omb2, float eps, float c1, float c2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// MFMA check: D = A B (16 x 16 x 16, bf16 in, fp32 out), row-major operands; tile
// blockIdx.x of consecutive 256-element tiles
__global__ void k_mfma_probe(const bf16* A, const bf16* B, float* D) {
    const int l = threadIdx.x;
    A += blockIdx.x * 256;
    B += blockIdx.x * 256;
    D += blockIdx.x * 256;
    bf16x4 a, b;
    for (int r = 0; r < 4; ++r) {
        a[r] = (short)A[(l % 16) * 16 + 4 * (l / 16) + r];
        b[r] = (short)B[(4 * (l / 16) + r) * 16 + l % 16];
    }
    floatx4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    for (int r = 0; r < 4; ++r) D[(4 * (l / 16) + r) * 16 + l % 16] = d[r];
}

// the same for the 32-deep product: D = A B, A 16 x 32, B 32 x 16
__global__ void k_mfma_probe32(const bf16* A, const bf16* B, float* D) {
    const int l = threadIdx.x;
    bf16x8 a, b;
    for (int r = 0; r < 8; ++r) {
        a[r] = (short)A[(l % 16) * 32 + 8 * (l / 16) + r];
        b[r] = (short)B[(8 * (l / 16) + r) * 16 + l % 16];
    }
    const floatx4 d = mfma32(a, b, floatx4{0.f, 0.f, 0.f, 0.f});
    for (int r = 0; r < 4; ++r) D[(4 * (l / 16) + r) * 16 + l % 16] = d[r];
}

// Staging of the allocation-free probe (t2s_unet_mfma_probe_static): up to
// kProbeMaxTiles A and B tiles (bf16) and D tiles (fp32).  Each device holds its own
// copy; host code reaches it only through the address hipGetSymbolAddress returns.
constexpr int kProbeMaxTiles = 8;
__device__ __align__(256) unsigned char scratch[kProbeMaxTiles * (512 + 512 + 1024)];

}  // namespace unetk

// ===========================================================================
// host side: network description, workspace, forward / backward / Adam
// ===========================================================================
namespace {

}  // namespace
namespace t2s {
int set_error(int code, const std::string& msg);   // shared last-error slot (api.cpp)
}
namespace {
int ufail(int code, const std::string& m) { return t2s::set_error(code, m); }
#define UHIP(expr)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return ufail(T2S_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)
#define ULAUNCH()                                                                              \
    do {                                                                                       \
        hipError_t e_ = hipGetLastError();                                                     \
        if (e_ != hipSuccess) return ufail(T2S_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

int pad16(int c) { return (c + 15) / 16 * 16; }
size_t al(size_t v) { return (v + 255) / 256 * 256; }

struct Layer {
    int KS, cin, cout;       // packed (real) sizes; up layers: cout = 4 * c (GEMM rows), bias c
    int cinp, coutp;         // GEMM sizes
    int nbias;
    size_t woff, boff;       // offsets in the packed parameter vector
    size_t o_wf, o_wb;       // bf16 weights in the workspace
    bool up;
};

struct Act {
    size_t off;              // byte offset in the workspace
    int C, H, W;
};

}  // namespace

struct t2s_unet {
    int K, base, levels, maxB, H, W, cx, cxp;
    std::vector<Layer> L;    // enc{l}a, enc{l}b ..., bota, botb, (up{l}, dec{l}a, dec{l}b) ..., final
    size_t nparams = 0;
    // workspace offsets
    size_t o_master = 0, o_m = 0, o_v = 0, o_g = 0, o_part = 0, o_bpart = 0, o_scale = 0, o_loss = 0;
    size_t part_floats = 0, bpart_floats = 0;
    size_t o_x32 = 0, o_t32 = 0, o_xb = 0, o_y32 = 0, o_dy = 0;
    std::vector<Act> a, cat, pool, da, dcat, dpool;   // per level
    std::vector<Act> deca, decb, ddeca, ddecb, d4;     // decoder, per level
    Act bota{}, botb{}, dbota{}, dbotb{};
    size_t bytes = 0;
    char* ws = nullptr;
    int step = 0;
    int loss_blocks = 1024;
};

namespace {

using unetk::bf16;

template <typename T>
T* at(t2s_unet* u, size_t off) {
    return (T*)(u->ws + off);
}

int launch_conv(t2s_unet* u, const Layer& Ly, const bf16* w, int cinp, int coutp, int cout, const bf16* in, int ldi,
                int ci_off, void* out, int ldo, int co_off, int B, int H, int W, const float* bias, int relu,
                int out_f32, int shuffle, hipStream_t st) {
    unetk::ConvArgs a;
    a.in = in;
    a.ldi = ldi;
    a.ci_off = ci_off;
    a.w = w;
    a.bias = bias;
    a.out = out;
    a.ldo = ldo;
    a.co_off = co_off;
    a.B = B;
    a.H = H;
    a.W = W;
    a.cinp = cinp;
    a.coutp = coutp;
    a.cout = cout;
    a.relu = relu;
    a.out_f32 = out_f32;
    a.shuffle = shuffle;
    const int P = B * H * W;
    dim3 grid((P + 63) / 64, (coutp + 63) / 64);
    if (Ly.KS == 3)
        hipLaunchKernelGGL(unetk::k_conv<3>, grid, dim3(unetk::kNT), 0, st, a);
    else
        hipLaunchKernelGGL(unetk::k_conv<1>, grid, dim3(unetk::kNT), 0, st, a);
    ULAUNCH();
    return 0;
}

}  // namespace


namespace {

using unetk::bf16;

// forward of layer `Ly` (not up): out = relu(conv(in) + b)
int fwd_conv(t2s_unet* u, const Layer& Ly, const Act& in, int ldi, int ci_off, void* out, int ldo, int co_off, int B,
             int relu, int out_f32, hipStream_t st) {
    return launch_conv(u, Ly, at<bf16>(u, Ly.o_wf), Ly.cinp, Ly.coutp, Ly.cout, at<bf16>(u, in.off), ldi, ci_off, out,
                       ldo, co_off, B, in.H, in.W, at<float>(u, u->o_master + Ly.boff * 4), relu, out_f32, 0, st);
}

// weight + bias gradient of a layer: dout (channels co_off.. of ldo) against input in
int wgrad(t2s_unet* u, const Layer& Ly, const bf16* dout, int ldo, int co_off, const bf16* in, int ldi, int ci_off,
          int B, int H, int W, int bias_fold, hipStream_t st) {
    const int P = B * H * W;
    const int taps = Ly.KS * Ly.KS;
    const int tiles = ((Ly.coutp + 63) / 64) * ((Ly.cinp + 63) / 64) * taps;
    int nsplit = std::max(1, std::min((1024 + tiles - 1) / tiles, std::max(1, P / 256)));
    int pps = (P + nsplit - 1) / nsplit;
    pps = (pps + 31) / 32 * 32;
    nsplit = (P + pps - 1) / pps;
    if ((size_t)nsplit * taps * Ly.coutp * Ly.cinp > u->part_floats) return ufail(T2S_ENOMEM, "wgrad partial buffer");
    unetk::WgradArgs a;
    a.dout = dout;
    a.ldo = ldo;
    a.co_off = co_off;
    a.coutp = Ly.coutp;
    a.in = in;
    a.ldi = ldi;
    a.ci_off = ci_off;
    a.cinp = Ly.cinp;
    a.B = B;
    a.H = H;
    a.W = W;
    a.KS = Ly.KS;
    a.part = at<float>(u, u->o_part);
    a.pix_per_split = pps;
    hipLaunchKernelGGL(unetk::k_wgrad, dim3((Ly.cinp + 63) / 64, (Ly.coutp + 63) / 64, taps * nsplit),
                       dim3(unetk::kNT), 0, st, a);
    ULAUNCH();
    const int n = taps * Ly.cout * Ly.cin;
    hipLaunchKernelGGL(unetk::k_wgrad_reduce, dim3((n + 255) / 256), dim3(256), 0, st, at<float>(u, u->o_part),
                       nsplit, taps, Ly.coutp, Ly.cinp, Ly.cout, Ly.cin, at<float>(u, u->o_g + Ly.woff * 4));
    ULAUNCH();
    // bias: sum of dout over pixels (folding the 4 sub-pixel groups of an up layer)
    const int C = Ly.cout;
    const int bsplit = std::max(1, std::min(1024, P / 256));
    const int bpps = (P + bsplit - 1) / bsplit;
    if ((size_t)bsplit * C > u->bpart_floats) return ufail(T2S_ENOMEM, "bias partial buffer");
    hipLaunchKernelGGL(unetk::k_bias_part, dim3(bsplit), dim3(256), 0, st, dout, ldo, co_off, C, P, bpps,
                       at<float>(u, u->o_bpart));
    ULAUNCH();
    hipLaunchKernelGGL(unetk::k_bias_reduce, dim3((C / bias_fold + unetk::kBiasCh - 1) / unetk::kBiasCh),
                       dim3(unetk::kBiasCh * unetk::kBiasLanes), 0, st, at<float>(u, u->o_bpart), bsplit, C, bias_fold,
                       at<float>(u, u->o_g + Ly.boff * 4));
    ULAUNCH();
    return 0;
}

// data gradient: din = conv^T(dout) using the reflected / transposed weights
int dgrad(t2s_unet* u, const Layer& Ly, const bf16* dout, int ldo, int co_off, bf16* din, int ldi, int ci_off, int B,
          int H, int W, hipStream_t st) {
    // GEMM: input channels = coutp of the layer, output channels = cinp (stored: cin)
    Layer T = Ly;
    return launch_conv(u, T, at<bf16>(u, Ly.o_wb), Ly.coutp, Ly.cinp, Ly.cin, dout, ldo, co_off, din, ldi, ci_off, B, H,
                       W, nullptr, 0, 0, 0, st);
}

int relu_bwd(t2s_unet* u, bf16* g, const bf16* y, int ld, int off, int C, size_t P, hipStream_t st) {
    const size_t n = P * C;
    hipLaunchKernelGGL(unetk::k_relu_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, y, ld, off, C, P);
    ULAUNCH();
    return 0;
}

int prep_all(t2s_unet* u, hipStream_t st) {
    for (const Layer& Ly : u->L) {
        const size_t n = (size_t)Ly.KS * Ly.KS * Ly.coutp * Ly.cinp;
        hipLaunchKernelGGL(unetk::k_prep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           at<float>(u, u->o_master + Ly.woff * 4), Ly.KS, Ly.cout, Ly.cin, Ly.coutp, Ly.cinp,
                           at<bf16>(u, Ly.o_wf), at<bf16>(u, Ly.o_wb));
        ULAUNCH();
    }
    return 0;
}

// Device address of unetk::scratch on the current device, looked up once per device
// (the array's name is only a host-side stand-in for it).
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};
int static_scratch(void** out) {
    int dev = 0;
    UHIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return ufail(T2S_EHIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        UHIP(hipGetSymbolAddress(&p, HIP_SYMBOL(unetk::scratch)));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

// One Adam step (Kingma & Ba, with bias correction) on the fp32 master weights from
// the gradient buffer, then the bf16 weight copies; advances the step counter.
int adam_update(t2s_unet* u, float lr, hipStream_t st) {
    u->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const double c1 = 1.0 - std::pow(b1, (double)u->step), c2 = 1.0 - std::pow(b2, (double)u->step);
    hipLaunchKernelGGL(unetk::k_adam, dim3((unsigned)((u->nparams + 255) / 256)), dim3(256), 0, st,
                       at<float>(u, u->o_master), at<float>(u, u->o_g), at<float>(u, u->o_m), at<float>(u, u->o_v),
                       u->nparams, lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, (float)c1,
                       (float)c2);
    ULAUNCH();
    return prep_all(u, st);
}

// forward pass on normalised input (x32, xb filled); y32 = net output (2K channels, ld cxp)
int forward(t2s_unet* u, int B, hipStream_t st) {
    const int nl = u->levels;
    int li = 0;
    Act in = Act{u->o_xb, u->cxp, u->H, u->W};
    int ldin = u->cxp, offin = 0;
    for (int l = 0; l < nl - 1; ++l) {
        const int c = u->base << l;
        if (int e = fwd_conv(u, u->L[li++], in, ldin, offin, at<bf16>(u, u->a[l].off), c, 0, B, 1, 0, st)) return e;
        if (int e = fwd_conv(u, u->L[li++], u->a[l], c, 0, at<bf16>(u, u->cat[l].off), 2 * c, c, B, 1, 0, st)) return e;
        const Act& cl = u->cat[l];
        const size_t n = (size_t)B * (cl.H / 2) * (cl.W / 2) * c;
        hipLaunchKernelGGL(unetk::k_pool, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           at<bf16>(u, cl.off), 2 * c, c, c, B, cl.H, cl.W, at<bf16>(u, u->pool[l].off));
        ULAUNCH();
        in = u->pool[l];
        ldin = c;
        offin = 0;
    }
    const int cb = u->base << (nl - 1);
    if (int e = fwd_conv(u, u->L[li++], in, ldin, 0, at<bf16>(u, u->bota.off), cb, 0, B, 1, 0, st)) return e;
    if (int e = fwd_conv(u, u->L[li++], u->bota, cb, 0, at<bf16>(u, u->botb.off), cb, 0, B, 1, 0, st)) return e;
    Act below = u->botb;
    int cbelow = cb;
    for (int l = nl - 2; l >= 0; --l) {
        const int c = u->base << l;
        const Layer& U = u->L[li++];
        // up: 1x1 GEMM to 4c channels, shuffled into channels [0, c) of the concat buffer
        if (int e = launch_conv(u, U, at<bf16>(u, U.o_wf), U.cinp, U.coutp, U.cout, at<bf16>(u, below.off), cbelow,
                                0, at<bf16>(u, u->cat[l].off), 2 * c, 0, B, below.H, below.W,
                                at<float>(u, u->o_master + U.boff * 4), 0, 0, 1, st))
            return e;
        if (int e = fwd_conv(u, u->L[li++], u->cat[l], 2 * c, 0, at<bf16>(u, u->deca[l].off), c, 0, B, 1, 0, st)) return e;
        if (int e = fwd_conv(u, u->L[li++], u->deca[l], c, 0, at<bf16>(u, u->decb[l].off), c, 0, B, 1, 0, st)) return e;
        below = u->decb[l];
        cbelow = c;
    }
    const Layer& F = u->L[li++];
    return fwd_conv(u, F, u->decb[0], u->base, 0, at<float>(u, u->o_y32), u->cxp, 0, B, 0, 1, st);
}

// backward pass from dy (bf16, ld cxp): fills the packed gradient vector
int backward(t2s_unet* u, int B, hipStream_t st) {
    const int nl = u->levels;
    const int nL = (int)u->L.size();
    int li = nL - 1;
    const Layer& F = u->L[li--];
    const bf16* dy = at<bf16>(u, u->o_dy);
    const int c0 = u->base;
    const size_t P0 = (size_t)B * u->H * u->W;
    if (int e = wgrad(u, F, dy, u->cxp, 0, at<bf16>(u, u->decb[0].off), c0, 0, B, u->H, u->W, 1, st)) return e;
    if (int e = dgrad(u, F, dy, u->cxp, 0, at<bf16>(u, u->ddecb[0].off), c0, 0, B, u->H, u->W, st)) return e;
    // decoder, top level first
    for (int l = 0; l <= nl - 2; ++l) {
        const int c = u->base << l;
        const int Hl = u->H >> l, Wl = u->W >> l;
        const size_t Pl = (size_t)B * Hl * Wl;
        const Layer& Db = u->L[li--];
        const Layer& Da = u->L[li--];
        const Layer& Up = u->L[li--];
        bf16* ddb = at<bf16>(u, u->ddecb[l].off);
        if (int e = relu_bwd(u, ddb, at<bf16>(u, u->decb[l].off), c, 0, c, Pl, st)) return e;
        if (int e = wgrad(u, Db, ddb, c, 0, at<bf16>(u, u->deca[l].off), c, 0, B, Hl, Wl, 1, st)) return e;
        bf16* dda = at<bf16>(u, u->ddeca[l].off);
        if (int e = dgrad(u, Db, ddb, c, 0, dda, c, 0, B, Hl, Wl, st)) return e;
        if (int e = relu_bwd(u, dda, at<bf16>(u, u->deca[l].off), c, 0, c, Pl, st)) return e;
        if (int e = wgrad(u, Da, dda, c, 0, at<bf16>(u, u->cat[l].off), 2 * c, 0, B, Hl, Wl, 1, st)) return e;
        bf16* dcat = at<bf16>(u, u->dcat[l].off);
        if (int e = dgrad(u, Da, dda, c, 0, dcat, 2 * c, 0, B, Hl, Wl, st)) return e;
        // up layer: gather the gradient of its shuffled output, then 1x1 GEMM gradients
        const int Hb = Hl / 2, Wb = Wl / 2;
        const size_t n4 = (size_t)B * Hb * Wb * 4 * c;
        bf16* d4 = at<bf16>(u, u->d4[l].off);
        hipLaunchKernelGGL(unetk::k_unshuffle, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st, dcat, 2 * c, 0,
                           c, B, Hb, Wb, d4);
        ULAUNCH();
        const int cbl = u->base << (l + 1);
        const Act& belowA = (l + 1 <= nl - 2) ? u->decb[l + 1] : u->botb;
        bf16* dbelow = at<bf16>(u, ((l + 1 <= nl - 2) ? u->ddecb[l + 1] : u->dbotb).off);
        if (int e = wgrad(u, Up, d4, 4 * c, 0, at<bf16>(u, belowA.off), cbl, 0, B, Hb, Wb, 4, st)) return e;
        if (int e = dgrad(u, Up, d4, 4 * c, 0, dbelow, cbl, 0, B, Hb, Wb, st)) return e;
    }
    // bottleneck
    {
        const int l = nl - 1;
        const int c = u->base << l;
        const int Hl = u->H >> l, Wl = u->W >> l;
        const size_t Pl = (size_t)B * Hl * Wl;
        const Layer& Bb = u->L[li--];
        const Layer& Ba = u->L[li--];
        bf16* dbb = at<bf16>(u, u->dbotb.off);
        if (int e = relu_bwd(u, dbb, at<bf16>(u, u->botb.off), c, 0, c, Pl, st)) return e;
        if (int e = wgrad(u, Bb, dbb, c, 0, at<bf16>(u, u->bota.off), c, 0, B, Hl, Wl, 1, st)) return e;
        bf16* dba = at<bf16>(u, u->dbota.off);
        if (int e = dgrad(u, Bb, dbb, c, 0, dba, c, 0, B, Hl, Wl, st)) return e;
        if (int e = relu_bwd(u, dba, at<bf16>(u, u->bota.off), c, 0, c, Pl, st)) return e;
        const int cin = u->base << (l - 1);
        if (int e = wgrad(u, Ba, dba, c, 0, at<bf16>(u, u->pool[l - 1].off), cin, 0, B, Hl, Wl, 1, st)) return e;
        if (int e = dgrad(u, Ba, dba, c, 0, at<bf16>(u, u->dpool[l - 1].off), cin, 0, B, Hl, Wl, st)) return e;
    }
    // encoder, deepest first
    for (int l = nl - 2; l >= 0; --l) {
        const int c = u->base << l;
        const int Hl = u->H >> l, Wl = u->W >> l;
        const size_t Pl = (size_t)B * Hl * Wl;
        const Layer& Eb = u->L[li--];
        const Layer& Ea = u->L[li--];
        bf16* dcat = at<bf16>(u, u->dcat[l].off);
        const size_t np = (size_t)B * (Hl / 2) * (Wl / 2) * c;
        hipLaunchKernelGGL(unetk::k_pool_bwd_add, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st,
                           at<bf16>(u, u->cat[l].off), at<bf16>(u, u->dpool[l].off), 2 * c, c, c, B, Hl, Wl, dcat);
        ULAUNCH();
        if (int e = relu_bwd(u, dcat, at<bf16>(u, u->cat[l].off), 2 * c, c, c, Pl, st)) return e;
        if (int e = wgrad(u, Eb, dcat, 2 * c, c, at<bf16>(u, u->a[l].off), c, 0, B, Hl, Wl, 1, st)) return e;
        bf16* da = at<bf16>(u, u->da[l].off);
        if (int e = dgrad(u, Eb, dcat, 2 * c, c, da, c, 0, B, Hl, Wl, st)) return e;
        if (int e = relu_bwd(u, da, at<bf16>(u, u->a[l].off), c, 0, c, Pl, st)) return e;
        if (l == 0) {
            if (int e = wgrad(u, Ea, da, c, 0, at<bf16>(u, u->o_xb), u->cxp, 0, B, Hl, Wl, 1, st)) return e;
        } else {
            const int cin = u->base << (l - 1);
            if (int e = wgrad(u, Ea, da, c, 0, at<bf16>(u, u->pool[l - 1].off), cin, 0, B, Hl, Wl, 1, st)) return e;
            if (int e = dgrad(u, Ea, da, c, 0, at<bf16>(u, u->dpool[l - 1].off), cin, 0, B, Hl, Wl, st)) return e;
        }
    }
    (void)P0;
    return 0;
}

int loss_and_dy(t2s_unet* u, int B, double* loss, hipStream_t st) {
    const size_t P = (size_t)B * u->H * u->W;
    const float inv_n = 1.f / (float)(P * u->cx);
    hipLaunchKernelGGL(unetk::k_mse, dim3(u->loss_blocks), dim3(unetk::kNT), 0, st, at<float>(u, u->o_x32),
                       at<float>(u, u->o_y32), u->cxp, at<float>(u, u->o_t32), u->cx, P, inv_n, at<bf16>(u, u->o_dy),
                       u->cxp, at<double>(u, u->o_loss));
    ULAUNCH();
    if (loss) {
        std::vector<double> part(u->loss_blocks);
        UHIP(hipMemcpyAsync(part.data(), at<double>(u, u->o_loss), part.size() * 8, hipMemcpyDeviceToHost, st));
        UHIP(hipStreamSynchronize(st));
        double s = 0;
        for (double v : part) s += v;
        *loss = s / (double)(P * u->cx);
    }
    return 0;
}

int pack_complex(t2s_unet* u, const void* src, int B, float* x32, bf16* xb, hipStream_t st) {
    const int HW = u->H * u->W;
    hipLaunchKernelGGL(unetk::k_pack, dim3((HW + 255) / 256, B), dim3(256), 0, st, (const float2*)src,
                       at<float>(u, u->o_scale), u->K, HW, x32, xb, u->cxp);
    ULAUNCH();
    return 0;
}

}  // namespace

extern "C" {

int t2s_unet_create(int K, int base, int levels, int max_batch, int H, int W, t2s_unet** out) {
    if (!out) return ufail(T2S_EINVAL, "out is NULL");
    *out = nullptr;
    // every inner channel count must be a multiple of the 16-wide GEMM step
    if (K < 1 || K > T2S_MAX_K || base < 16 || base % 16 || levels < 2 || levels > 6 || max_batch < 1)
        return ufail(T2S_EINVAL, "K in [1, 8], base a positive multiple of 16, levels in [2, 6], max_batch >= 1");
    if (H % (1 << (levels - 1)) || W % (1 << (levels - 1)) || H < 2 || W < 2)
        return ufail(T2S_ESHAPE, "H and W must be divisible by 2^(levels-1)");
    t2s_unet* u = new t2s_unet();
    u->K = K;
    u->base = base;
    u->levels = levels;
    u->maxB = max_batch;
    u->H = H;
    u->W = W;
    u->cx = 2 * K;
    u->cxp = pad16(2 * K);
    // layers in forward order (same packing as the reference)
    size_t off = 0;
    auto add = [&](int KS, int cin, int cout_w, int nbias, bool up) {
        Layer Ly{};
        Ly.KS = KS;
        Ly.cin = cin;
        Ly.cout = cout_w;
        Ly.cinp = pad16(cin);
        Ly.coutp = pad16(cout_w);
        Ly.nbias = nbias;
        Ly.up = up;
        Ly.woff = off;
        off += (size_t)KS * KS * cout_w * cin;
        Ly.boff = off;
        off += nbias;
        u->L.push_back(Ly);
    };
    int prev = u->cx;
    for (int l = 0; l < levels - 1; ++l) {
        const int c = base << l;
        add(3, prev, c, c, false);
        add(3, c, c, c, false);
        prev = c;
    }
    const int cb = base << (levels - 1);
    add(3, prev, cb, cb, false);
    add(3, cb, cb, cb, false);
    int below = cb;
    for (int l = levels - 2; l >= 0; --l) {
        const int c = base << l;
        add(1, below, 4 * c, c, true);   // 2x2 stride-2 transposed conv as a 1x1 GEMM to 4c channels
        add(3, 2 * c, c, c, false);
        add(3, c, c, c, false);
        below = c;
    }
    add(1, base, u->cx, u->cx, false);
    u->nparams = off;
    // workspace
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o = al(o + std::max<size_t>(b, 1));
        return r;
    };
    u->o_master = take(off * 4);
    u->o_m = take(off * 4);
    u->o_v = take(off * 4);
    u->o_g = take(off * 4);
    for (Layer& Ly : u->L) {
        const size_t nw = (size_t)Ly.KS * Ly.KS * Ly.coutp * Ly.cinp;
        Ly.o_wf = take(nw * 2);
        Ly.o_wb = take(nw * 2);
    }
    // weight-gradient split-K partials: the largest need over layers at full batch
    // (the split count grows with the pixel count, so the full batch bounds it)
    size_t partmax = 0;
    for (int l = 0; l < levels; ++l) {
        const size_t P = (size_t)max_batch * (H >> l) * (W >> l);
        for (const Layer& Ly : u->L) {
            const int taps = Ly.KS * Ly.KS;
            const int tiles = ((Ly.coutp + 63) / 64) * ((Ly.cinp + 63) / 64) * taps;
            int nsplit = std::max(1, std::min((1024 + tiles - 1) / tiles, std::max(1, (int)(P / 256))));
            partmax = std::max(partmax, (size_t)(nsplit + 1) * taps * Ly.coutp * Ly.cinp);
        }
    }
    u->part_floats = partmax;
    u->o_part = take(u->part_floats * 4);
    u->bpart_floats = (size_t)256 * 4 * (base << (levels - 1)) * 4;
    u->o_bpart = take(u->bpart_floats * 4);
    u->o_scale = take((size_t)max_batch * 4);
    u->o_loss = take((size_t)u->loss_blocks * 8);
    const size_t P0 = (size_t)max_batch * H * W;
    u->o_x32 = take(P0 * u->cx * 4);
    u->o_t32 = take(P0 * u->cx * 4);
    u->o_xb = take(P0 * u->cxp * 2);
    u->o_y32 = take(P0 * u->cxp * 4);
    u->o_dy = take(P0 * u->cxp * 2);
    auto act = [&](int C, int l) {
        Act A;
        A.C = C;
        A.H = H >> l;
        A.W = W >> l;
        A.off = take((size_t)max_batch * A.H * A.W * C * 2);
        return A;
    };
    for (int l = 0; l < levels - 1; ++l) {
        const int c = base << l;
        u->a.push_back(act(c, l));
        u->cat.push_back(act(2 * c, l));
        u->pool.push_back(act(c, l + 1));
        u->da.push_back(act(c, l));
        u->dcat.push_back(act(2 * c, l));
        u->dpool.push_back(act(c, l + 1));
        u->deca.push_back(act(c, l));
        u->decb.push_back(act(c, l));
        u->ddeca.push_back(act(c, l));
        u->ddecb.push_back(act(c, l));
        u->d4.push_back(act(4 * c, l + 1));
    }
    u->bota = act(cb, levels - 1);
    u->botb = act(cb, levels - 1);
    u->dbota = act(cb, levels - 1);
    u->dbotb = act(cb, levels - 1);
    u->bytes = o;
    *out = u;
    return 0;
}

int t2s_unet_destroy(t2s_unet* u) {
    delete u;
    return 0;
}

int t2s_unet_param_count(const t2s_unet* u, size_t* n) {
    if (!u || !n) return ufail(T2S_EINVAL, "NULL argument");
    *n = u->nparams;
    return 0;
}

int t2s_unet_get_shape(const t2s_unet* u, int* K, int* max_batch, int* H, int* W) {
    if (!u) return ufail(T2S_EINVAL, "NULL argument");
    if (K) *K = u->K;
    if (max_batch) *max_batch = u->maxB;
    if (H) *H = u->H;
    if (W) *W = u->W;
    return 0;
}

int t2s_unet_workspace_bytes(const t2s_unet* u, size_t* bytes) {
    if (!u || !bytes) return ufail(T2S_EINVAL, "NULL argument");
    *bytes = u->bytes;
    return 0;
}

int t2s_unet_bind_workspace(t2s_unet* u, void* dev, size_t bytes, void* stream) {
    if (!u) return ufail(T2S_EINVAL, "NULL network");
    if (!dev || bytes < u->bytes) return ufail(T2S_ENOMEM, "workspace too small: need " + std::to_string(u->bytes));
    if ((uintptr_t)dev % 256) return ufail(T2S_EINVAL, "workspace must be 256-byte aligned");
    u->ws = (char*)dev;
    hipStream_t st = (hipStream_t)stream;
    // activations and gradients start at zero (padded channels are read by the GEMMs)
    UHIP(hipMemsetAsync(u->ws, 0, u->bytes, st));
    UHIP(hipStreamSynchronize(st));
    return 0;
}

int t2s_unet_set_params(t2s_unet* u, const float* host, void* stream) {
    if (!u || !host) return ufail(T2S_EINVAL, "NULL argument");
    if (!u->ws) return ufail(T2S_ESTATE, "workspace not bound");
    for (size_t i = 0; i < u->nparams; ++i)
        if (!std::isfinite(host[i])) return ufail(T2S_ENONFINITE, "parameters contain NaN/Inf");
    hipStream_t st = (hipStream_t)stream;
    UHIP(hipMemcpyAsync(u->ws + u->o_master, host, u->nparams * 4, hipMemcpyHostToDevice, st));
    UHIP(hipMemsetAsync(u->ws + u->o_m, 0, u->nparams * 4, st));
    UHIP(hipMemsetAsync(u->ws + u->o_v, 0, u->nparams * 4, st));
    u->step = 0;
    if (int e = prep_all(u, st)) return e;
    UHIP(hipStreamSynchronize(st));
    return 0;
}

int t2s_unet_get_params(t2s_unet* u, float* host, void* stream) {
    if (!u || !host) return ufail(T2S_EINVAL, "NULL argument");
    if (!u->ws) return ufail(T2S_ESTATE, "workspace not bound");
    hipStream_t st = (hipStream_t)stream;
    UHIP(hipMemcpyAsync(host, u->ws + u->o_master, u->nparams * 4, hipMemcpyDeviceToHost, st));
    UHIP(hipStreamSynchronize(st));
    return 0;
}

int t2s_unet_forward(t2s_unet* u, const void* b0, void* alpha0, int B, void* stream) {
    if (!u || !b0 || !alpha0) return ufail(T2S_EINVAL, "NULL argument");
    if (!u->ws) return ufail(T2S_ESTATE, "workspace not bound");
    if (B < 1 || B > u->maxB) return ufail(T2S_EINVAL, "batch out of range");
    hipStream_t st = (hipStream_t)stream;
    const int HW = u->H * u->W;
    hipLaunchKernelGGL(unetk::k_zero_scale, dim3((B + 63) / 64), dim3(64), 0, st, at<float>(u, u->o_scale), B);
    hipLaunchKernelGGL(unetk::k_slice_scale, dim3(unetk::kScaleBlocks, B), dim3(unetk::kNT), 0, st, (const float2*)b0,
                       u->K, HW, at<float>(u, u->o_scale));
    ULAUNCH();
    if (int e = pack_complex(u, b0, B, at<float>(u, u->o_x32), at<bf16>(u, u->o_xb), st)) return e;
    if (int e = forward(u, B, st)) return e;
    hipLaunchKernelGGL(unetk::k_unpack, dim3((HW + 255) / 256, B), dim3(256), 0, st, at<float>(u, u->o_x32),
                       at<float>(u, u->o_y32), u->cxp, at<float>(u, u->o_scale), u->K, HW, (float2*)alpha0);
    ULAUNCH();
    return 0;
}

int t2s_unet_train_step(t2s_unet* u, const void* b0, const void* target, int B, float lr, double* loss,
                        void* stream) {
    if (!u || !b0 || !target) return ufail(T2S_EINVAL, "NULL argument");
    if (!u->ws) return ufail(T2S_ESTATE, "workspace not bound");
    if (B < 1 || B > u->maxB) return ufail(T2S_EINVAL, "batch out of range");
    if (!(lr > 0) || !std::isfinite(lr)) return ufail(T2S_EINVAL, "learning rate must be > 0");
    hipStream_t st = (hipStream_t)stream;
    const int HW = u->H * u->W;
    hipLaunchKernelGGL(unetk::k_zero_scale, dim3((B + 63) / 64), dim3(64), 0, st, at<float>(u, u->o_scale), B);
    hipLaunchKernelGGL(unetk::k_slice_scale, dim3(unetk::kScaleBlocks, B), dim3(unetk::kNT), 0, st, (const float2*)b0,
                       u->K, HW, at<float>(u, u->o_scale));
    ULAUNCH();
    if (int e = pack_complex(u, b0, B, at<float>(u, u->o_x32), at<bf16>(u, u->o_xb), st)) return e;
    if (int e = pack_complex(u, target, B, at<float>(u, u->o_t32), nullptr, st)) return e;
    if (int e = forward(u, B, st)) return e;
    if (int e = loss_and_dy(u, B, loss, st)) return e;
    if (int e = backward(u, B, st)) return e;
    return adam_update(u, lr, st);
}

int t2s_unet_adam_apply(t2s_unet* u, const float* grad, float lr, void* stream) {
    if (!u || !grad) return ufail(T2S_EINVAL, "NULL argument");
    if (!u->ws) return ufail(T2S_ESTATE, "workspace not bound");
    if (!(lr > 0) || !std::isfinite(lr)) return ufail(T2S_EINVAL, "learning rate must be > 0");
    for (size_t i = 0; i < u->nparams; ++i)
        if (!std::isfinite(grad[i])) return ufail(T2S_ENONFINITE, "gradient contains NaN/Inf");
    hipStream_t st = (hipStream_t)stream;
    UHIP(hipMemcpyAsync(u->ws + u->o_g, grad, u->nparams * 4, hipMemcpyHostToDevice, st));
    if (int e = adam_update(u, lr, st)) return e;
    UHIP(hipStreamSynchronize(st));
    return 0;
}

int t2s_unet_get_adam_state(t2s_unet* u, float* m, float* v, int* step, void* stream) {
    if (!u || !m || !v || !step) return ufail(T2S_EINVAL, "NULL argument");
    if (!u->ws) return ufail(T2S_ESTATE, "workspace not bound");
    hipStream_t st = (hipStream_t)stream;
    UHIP(hipMemcpyAsync(m, u->ws + u->o_m, u->nparams * 4, hipMemcpyDeviceToHost, st));
    UHIP(hipMemcpyAsync(v, u->ws + u->o_v, u->nparams * 4, hipMemcpyDeviceToHost, st));
    UHIP(hipStreamSynchronize(st));
    *step = u->step;
    return 0;
}

int t2s_unet_loss_grad(t2s_unet* u, const float* x, const float* t, int B, double* loss, float* grad, void* stream) {
    if (!u || !x || !t || !grad) return ufail(T2S_EINVAL, "NULL argument");
    if (!u->ws) return ufail(T2S_ESTATE, "workspace not bound");
    if (B < 1 || B > u->maxB) return ufail(T2S_EINVAL, "batch out of range");
    hipStream_t st = (hipStream_t)stream;
    const size_t P = (size_t)B * u->H * u->W;
    std::vector<bf16> xb(P * u->cxp, 0);
    for (size_t p = 0; p < P; ++p)
        for (int c = 0; c < u->cx; ++c) xb[p * u->cxp + c] = unetk::f2bf(x[p * u->cx + c]);
    UHIP(hipMemcpyAsync(u->ws + u->o_x32, x, P * u->cx * 4, hipMemcpyHostToDevice, st));
    UHIP(hipMemcpyAsync(u->ws + u->o_t32, t, P * u->cx * 4, hipMemcpyHostToDevice, st));
    UHIP(hipMemcpyAsync(u->ws + u->o_xb, xb.data(), xb.size() * 2, hipMemcpyHostToDevice, st));
    if (int e = forward(u, B, st)) return e;
    if (int e = loss_and_dy(u, B, loss, st)) return e;
    if (int e = backward(u, B, st)) return e;
    UHIP(hipMemcpyAsync(grad, u->ws + u->o_g, u->nparams * 4, hipMemcpyDeviceToHost, st));
    UHIP(hipStreamSynchronize(st));
    return 0;
}

int t2s_unet_init_params(const t2s_unet* u, uint64_t seed, float* host) {
    if (!u || !host) return ufail(T2S_EINVAL, "NULL argument");
    // He-normal weights (std sqrt(2 / fan_in)), zero biases, final 1x1 layer scaled by
    // 0.1 so the untrained network is close to the identity through its residual
    std::mt19937_64 gen(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (size_t li = 0; li < u->L.size(); ++li) {
        const Layer& Ly = u->L[li];
        const int fan_in = Ly.up ? Ly.cin : Ly.KS * Ly.KS * Ly.cin;
        double sd = std::sqrt(2.0 / fan_in);
        if (li + 1 == u->L.size()) sd *= 0.1;
        const size_t nw = (size_t)Ly.KS * Ly.KS * Ly.cout * Ly.cin;
        for (size_t i = 0; i < nw; ++i) host[Ly.woff + i] = (float)(sd * nd(gen));
        for (int i = 0; i < Ly.nbias; ++i) host[Ly.boff + i] = 0.f;
    }
    return 0;
}

int t2s_unet_mfma_probe_static(const float* A, const float* B, float* D, int count) {
    if (!A || !B || !D) return ufail(T2S_EINVAL, "NULL argument");
    if (count < 1 || count > unetk::kProbeMaxTiles)
        return ufail(T2S_EINVAL, "count must be in [1, " + std::to_string(unetk::kProbeMaxTiles) +
                                     "]: the static staging buffer holds that many tiles");
    bf16 a[unetk::kProbeMaxTiles * 256], b[unetk::kProbeMaxTiles * 256];
    for (int i = 0; i < count * 256; ++i) {
        a[i] = unetk::f2bf(A[i]);
        b[i] = unetk::f2bf(B[i]);
    }
    void* sp = nullptr;
    if (int e = static_scratch(&sp)) return e;
    bf16* da = (bf16*)sp;
    bf16* db = da + unetk::kProbeMaxTiles * 256;
    float* dd = (float*)(db + unetk::kProbeMaxTiles * 256);
    UHIP(hipMemcpy(da, a, (size_t)count * 512, hipMemcpyHostToDevice));
    UHIP(hipMemcpy(db, b, (size_t)count * 512, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(unetk::k_mfma_probe, dim3(count), dim3(64), 0, 0, (const bf16*)da, (const bf16*)db, dd);
    ULAUNCH();
    UHIP(hipMemcpy(D, dd, (size_t)count * 1024, hipMemcpyDeviceToHost));
    return 0;
}

int t2s_unet_mfma_probe32(const float* A, const float* B, float* D) {
    if (!A || !B || !D) return ufail(T2S_EINVAL, "NULL argument");
    std::vector<bf16> a(512), b(512);
    for (int i = 0; i < 512; ++i) {
        a[i] = unetk::f2bf(A[i]);
        b[i] = unetk::f2bf(B[i]);
    }
    void *da = nullptr, *db = nullptr, *dd = nullptr;
    UHIP(hipMalloc(&da, 1024));
    UHIP(hipMalloc(&db, 1024));
    UHIP(hipMalloc(&dd, 1024));
    UHIP(hipMemcpy(da, a.data(), 1024, hipMemcpyHostToDevice));
    UHIP(hipMemcpy(db, b.data(), 1024, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(unetk::k_mfma_probe32, dim3(1), dim3(64), 0, 0, (const bf16*)da, (const bf16*)db, (float*)dd);
    ULAUNCH();
    UHIP(hipMemcpy(D, dd, 1024, hipMemcpyDeviceToHost));
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(dd);
    return 0;
}

int t2s_unet_mfma_probe(const float* A, const float* B, float* D) {
    if (!A || !B || !D) return ufail(T2S_EINVAL, "NULL argument");
    std::vector<bf16> a(256), b(256);
    for (int i = 0; i < 256; ++i) {
        a[i] = unetk::f2bf(A[i]);
        b[i] = unetk::f2bf(B[i]);
    }
    void *da = nullptr, *db = nullptr, *dd = nullptr;
    UHIP(hipMalloc(&da, 512));
    UHIP(hipMalloc(&db, 512));
    UHIP(hipMalloc(&dd, 1024));
    UHIP(hipMemcpy(da, a.data(), 512, hipMemcpyHostToDevice));
    UHIP(hipMemcpy(db, b.data(), 512, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(unetk::k_mfma_probe, dim3(1), dim3(64), 0, 0, (const bf16*)da, (const bf16*)db, (float*)dd);
    ULAUNCH();
    UHIP(hipMemcpy(D, dd, 1024, hipMemcpyDeviceToHost));
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(dd);
    return 0;
}

}  // extern "C"
