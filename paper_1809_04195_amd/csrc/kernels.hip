// kernels.hip -- gfx950 kernels of the T2-Shuffling slice solver.
//
// Normal operator M p = S^H F^H Psi F S p + rho p (Sec. IV-B, eqs. commute /
// normaleq; fused three-pass schedule after Alg. 1):
//   pass A  (Alg. 1, first panel loop):  per (slice, 16-row tile, k): p = r + beta p
//           (CG direction update, fused), then for every coil c: S_c p_k and an
//           nz-point FFT of each row; written column-major in 16 x 16 tiles
//           (y fastest) so pass B reads whole columns -- the paper's "leave it
//           transposed" shortcut of Fig. 3 that saves two of four transposes.
//   pass B  (second loop, with the forward column FFT before Psi that the
//           printed loop omits): per (slice, coil, column tile): ny-point FFT of
//           every column of all K coefficient images, the K x K real symmetric
//           mix Psi(n) at every k-space location, ny-point inverse FFT.
//   pass C  (third loop): per (slice, 16-row tile, k): inverse nz-point FFT of
//           the rows of every coil, sum_c conj(S_c) (.), + rho p.  Inside CG the
//           vector update is fused here: the step length needs <p, M p>, which is
//           known before pass C starts, because F is unitary and so
//           <p, A^H A p> = sum_c sum_n (F S_c p)(n)^H Psi(n) (F S_c p)(n) is summed in
//           pass B (which holds both sides in registers) and ||p||^2 in pass A.
//           w = M p therefore never goes to memory.
// The centring of F and the 1/N of the unnormalised FFT pair are folded into the
// kernel table (uncentred order, / N), so no phase-modulation pass exists.
//
// LLR z-step (Sec. II-B eq. llr, blocked form; single pass of Sec. IV-C): one
// 64-lane wavefront per strip of 64/b blocks; lane = voxel column, b rows per lane;
// Gram matrix per block by cross-lane sums, complex Jacobi eigen-decomposition in
// FP64, W = V diag(max(sigma - tau, 0) / sigma) V^H, z = v W, fused with the ADMM
// u- and residual updates.
#include <algorithm>
#include <cmath>

#include "fft.hpp"
#include "kernels.hpp"

namespace t2s {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ double partial_sum(PartialSrc g, int s) {
    if (g.base == nullptr) return 0.0;
    const double* q = g.base + (size_t)s * g.stride;
    double acc = 0.0;
    for (int i = 0; i < g.count; ++i) acc += q[i];
    return acc;
}

// sum over the workgroup (fixed order); result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

// sum over a workgroup of any size >= 64 whose last wave may be partial (lanes past
// blockDim hold no data, so the cross-lane steps run only in the full first wave);
// sh: blockDim doubles of LDS; fixed order; result valid in thread 0
__device__ __forceinline__ double block_sum_ragged(double v, double* sh) {
    const int tid = threadIdx.x, n = blockDim.x;
    __syncthreads();
    sh[tid] = v;
    __syncthreads();
    double r = 0.0;
    if (tid < 64) {
        for (int i = tid; i < n; i += 64) r += sh[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o);
    }
    return r;
}

// Workgroup coordinates (x = row tile, y = coefficient k, z = slice).  The
// dispatcher deals linear workgroup ids round-robin over the 8 XCDs (each with its
// own L2); with `grouped`, id i is given the work item j = (i mod 8) * (total / 8) +
// i / 8 (when 8 divides the total), so each XCD works through a contiguous run of
// work items, decoded with k fastest: the K workgroups that read the same coil-map
// rows run back to back on one XCD and share them through its L2.  Which order
// streams better depends on the shape, so it is a per-class schedule choice.
struct Blk {
    int x, y, z;
};
__device__ __forceinline__ Blk block_coords(bool grouped) {
    const int gx = gridDim.x, gy = gridDim.y;
    const int total = gx * gy * gridDim.z;
    if (!grouped || (total & 7) != 0) return Blk{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z};
    int i = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    i = (i & 7) * (total >> 3) + (i >> 3);
    return Blk{(i / gy) % gx, i % gy, i / (gx * gy)};
}

// Pass intermediate layout: each ny x nz k-space image is stored as 16 x 16 tiles
// (2 KiB), tile (y / 16, z / 16) at ((z / 16) (ny / 16) + y / 16) * 256, inside a tile
// y fastest.  A 16-row tile of a row pass and a 16-column tile of pass B are then
// whole 2 KiB tiles, and a wave's access is one 512-byte run in every pass (with a
// plain [z][y] image the row passes touch 128-byte pieces of 2 KiB columns).
__device__ __forceinline__ size_t tile_col(int z, int ny) { return (size_t)(z >> 4) * (ny >> 4) * 256 + ((z & 15) << 4); }
__device__ __forceinline__ int tile_row(int y) { return ((y >> 4) << 8) + (y & 15); }
__device__ __forceinline__ size_t tix(int y, int z, int ny) { return tile_col(z, ny) + tile_row(y); }
// elements of one tiled image: nz rounded up to whole 16-column tiles (ny is a multiple of 16)
__host__ __device__ __forceinline__ size_t tmp_image(int ny, int nz) { return (size_t)ny * ((nz + 15) & ~15); }

// The pass intermediate is streamed: each pass reads or writes every element once and
// the next pass finds it in HBM, not in cache (a class's intermediate is gigabytes).
// Nontemporal loads and stores of it keep the cache for what a class shares (the Psi
// table, twiddles, partial sums).  NT selects them; plain accesses otherwise.
typedef float f2vec __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ float2 ld_stream(const float2* p) {
    if constexpr (NT) {
        const f2vec r = __builtin_nontemporal_load(reinterpret_cast<const f2vec*>(p));
        return make_float2(r.x, r.y);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
    if constexpr (NT) {
        f2vec r;
        r.x = v.x;
        r.y = v.y;
        __builtin_nontemporal_store(r, reinterpret_cast<f2vec*>(p));
    } else {
        *p = v;
    }
}
// Pass B streams its intermediate nontemporally at every length (at 384 points this
// gained 10 % once the Psi table is shared through each XCD's L2, at 256 points 6 %).
template <int L>
constexpr bool passB_nt() { return true; }

__device__ __forceinline__ bool slice_active(const ClassArgs& a, int s) { return a.state[4 * s] != 0; }

__host__ __device__ __forceinline__ uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// x * W_L^(+-e) with the twiddle read from the LDS table (0 <= e < L; the table's
// entry 0 is exactly 1, so e = 0 needs no branch, which would diverge in a wave)
template <bool INV>
__device__ __forceinline__ float2 tw_mul(float2 x, const float2* tw, int e) {
    float2 w = tw[e];
    if (INV) w.y = -w.y;
    return cmul(x, w);
}

template <int L>
using RowGeom = RegGeom<L, RowPlan<L>>;
template <int L>
constexpr int rows_threads() { return kRowTile * RowGeom<L>::P; }
// Pass C's LDS exchange can be double-buffered (kOrderLds2C): the waves that finished
// reading coil c's exchange then transform coil c + 1 into the other buffer without
// waiting for the rest, one barrier per coil instead of two.  It pays where one
// workgroup fills a CU anyway (384 points: 21.8 -> 20.0 ms per 512-slice launch) and
// costs workgroups per CU where the second buffer does not fit beside the others; the
// variant exists from 256 points on and the autotuner picks per class.  (Pass A
// measured 2 % slower with two buffers at 384 points and keeps one.)
template <int L>
constexpr bool passC_lds2_ok() { return L >= 256; }
// Occupancy targets of the row passes.  Left free, the register scheduler trades the
// batched issue of a coil's loads for one more wave per SIMD and then waits on every
// load in turn, which costs far more than the extra wave gains.
// Pass A: three waves while a thread holds at most 16 values per row, else two
// (24 values per thread at ny = 384 need the larger register budget).
template <int L>
constexpr int passA_waves() { return RowGeom<L>::P <= 16 ? 3 : 2; }
// Pass C: a three-wave budget (168 registers) still keeps the batched loads of the CG
// update at ny = 256 and lets the fused update run at three waves per SIMD; larger
// rows take more registers and run at two.
constexpr int kPassCWavesPerSimd = 3;

// p = r (first) or r + beta p on the R1 positions R2 n1 + t of one row: every load is
// issued before the first store (restrict: r and p never overlap), the new p is kept
// in pv and stored; returns the thread's part of ||p||^2
template <int R1, int R2>
__device__ __forceinline__ double direction_update(const float2* __restrict__ r, float2* __restrict__ p, int t,
                                                   int first, float beta, float2 (&pv)[R1]) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) pv[n1] = r[R2 * n1 + t];
    if (!first) {
        float2 po[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) po[n1] = p[R2 * n1 + t];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) pv[n1] = make_float2(pv[n1].x + beta * po[n1].x, pv[n1].y + beta * po[n1].y);
    }
    double pp = 0.0;
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
        p[R2 * n1 + t] = pv[n1];
        pp += (double)pv[n1].x * pv[n1].x + (double)pv[n1].y * pv[n1].y;
    }
    return pp;
}

// CG update on the R1 positions R2 m of one row (pointers offset by the thread's t),
// with w = acc + rho p in registers: x += alpha p, r -= alpha w; loads before stores (restrict: the three
// vectors never overlap), in two halves to bound the registers; returns the thread's
// part of ||r||^2
template <int R1, int R2>
__device__ __forceinline__ double cg_row_update(const float2 (&acc)[R1], const float2* __restrict__ p,
                                                float2* __restrict__ x, float2* __restrict__ r, float rho,
                                                float alpha) {
    constexpr int H = (R1 >= 8 && R1 % 2 == 0) ? R1 / 2 : R1;   // odd R1 (13, 15): one pass
    static_assert(R1 % H == 0, "the halves must tile the row");
    double dot = 0.0;
#pragma unroll
    for (int h = 0; h < R1; h += H) {
        float2 pv[H], xv[H], rv[H];
#pragma unroll
        for (int m = 0; m < H; ++m) pv[m] = p[R2 * (h + m)];
#pragma unroll
        for (int m = 0; m < H; ++m) xv[m] = x[R2 * (h + m)];
#pragma unroll
        for (int m = 0; m < H; ++m) rv[m] = r[R2 * (h + m)];
#pragma unroll
        for (int m = 0; m < H; ++m) {
            const float2 w = make_float2(acc[h + m].x + rho * pv[m].x, acc[h + m].y + rho * pv[m].y);
            xv[m].x += alpha * pv[m].x;
            xv[m].y += alpha * pv[m].y;
            rv[m].x -= alpha * w.x;
            rv[m].y -= alpha * w.y;
            dot += (double)rv[m].x * rv[m].x + (double)rv[m].y * rv[m].y;
        }
#pragma unroll
        for (int m = 0; m < H; ++m) x[R2 * (h + m)] = xv[m];
#pragma unroll
        for (int m = 0; m < H; ++m) r[R2 * (h + m)] = rv[m];
    }
    return dot;
}

// ---------------------------------------------------------------------------
// pass A: per (row tile, k): p = r + beta p, then per coil S_c p_k and the row FFT
// (register two-step plan), stored column-major in 16 x 16 tiles.  Two thread
// mappings meet at the LDS exchange: row-major lanes for the coalesced row loads,
// row-fastest lanes for the stores (a wave writes one 512-byte run of a tile).
// ---------------------------------------------------------------------------
// M: coil-map sets (soft-SENSE, Sec. II-A): coil c sees sum_m S_(c,m) p_(m,k); the
// coefficient vectors hold M K images per slice ([M][K][ny][nz]), the maps C M per
// slice ([C][M][ny][nz])
template <int L, int M>
__global__ __launch_bounds__(rows_threads<L>()) __attribute__((amdgpu_waves_per_eu(1, passA_waves<L>())))
void k_passA(ClassArgs a, int s0, const float2* __restrict__ src,
                                                              int src_s0, int first, PartialSrc gc, PartialSrc gp,
                                                              int want_pp) {
    const Blk bk = block_coords(a.order & kOrderXcdA);
    using G = RowGeom<L>;
    constexpr int R1 = G::R1, R2 = G::R2, P = G::P, TB = G::TB, RT = kRowTile, NT = RT * P;
    static_assert(NT % 64 == 0, "block_sum needs whole waves");
    __shared__ float2 tw[L];
    __shared__ float2 xb[RT * TB];
    __shared__ double red[16];

    const int s = s0 + bk.z;
    if (!slice_active(a, s)) return;
    const int k = bk.y;
    const int y0 = bk.x * RT;
    const int ny = a.ny;
    const size_t N = (size_t)ny * L;
    const size_t NTI = tmp_image(ny, L);
    const int tid = threadIdx.x;
    for (int i = tid; i < L; i += NT) tw[i] = a.twz[i];

    const int r1 = tid / P, t1 = tid - r1 * P;   // mapping 1 (t fastest)
    const bool on1 = R2 == P || t1 < R2;         // every lane when R2 == P (known at compile time)
    const int r3 = tid % RT, t3 = tid / RT;      // mapping 3 (row fastest)
    const bool on3 = t3 < R1;

    float beta = 0.0f;
    if (!first) {
        const double g1 = partial_sum(gc, s), g0 = partial_sum(gp, s);
        beta = g0 > 0.0 ? (float)(g1 / g0) : 0.0f;
    }
    const size_t rowoff = (size_t)(y0 + r1) * L;
    const int KM = M * a.K;
    float2 pv[M][R1];
    double pp = 0.0;
    if (on1) {
#pragma unroll
        for (int m = 0; m < M; ++m)
            pp += direction_update<R1, R2>(src + ((size_t)(s - src_s0) * KM + m * a.K + k) * N + rowoff,
                                           a.p + ((size_t)s * KM + m * a.K + k) * N + rowoff, t1, first, beta, pv[m]);
    }
    if (want_pp) {
        const double tot = block_sum(pp, red);
        if (tid == 0) a.pa[(size_t)s * a.nrw + bk.y * gridDim.x + bk.x] = tot;
    }
    __syncthreads();
    float2* xr1 = xb + r1 * TB;
    const float2* xr3 = xb + r3 * TB;
    // the next coil's map row is loaded while the current one is transformed (up to 24
    // values per thread; 32 at 512 points leave no registers for it), into the same
    // registers once the current row has been used: a copy "v = next" before the loads
    // would be merged at the end of the on1 block and wait there for the loads in
    // flight, before the exchange barrier
    constexpr bool kPrefetch = M == 1 && R1 <= 24;
    const float2* S0 = a.sens + (size_t)s * a.C * M * N + rowoff + t1;
    float2 sn[R1];
    if (on1 && kPrefetch) {
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) sn[n1] = S0[R2 * n1];
    }
    for (int c = 0; c < a.C; ++c) {
        if (on1) {
            float2 v[R1];
            if constexpr (kPrefetch) {
#pragma unroll
                for (int n1 = 0; n1 < R1; ++n1) v[n1] = cmul(sn[n1], pv[0][n1]);
                __builtin_amdgcn_sched_barrier(0);
                if (c + 1 < a.C) {
                    const float2* S = S0 + (size_t)(c + 1) * N;
#pragma unroll
                    for (int n1 = 0; n1 < R1; ++n1) sn[n1] = S[R2 * n1];
                }
                // all of the next coil's loads issued before the transform (the
                // scheduler would otherwise interleave load / wait / use)
                __builtin_amdgcn_sched_barrier(0);
            } else {
                // sum over the map sets of S_(c,m) p_(m,k)
#pragma unroll
                for (int n1 = 0; n1 < R1; ++n1) v[n1] = make_float2(0.f, 0.f);
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const float2* S = S0 + ((size_t)c * M + m) * N;
                    float2 sm[R1];
#pragma unroll
                    for (int n1 = 0; n1 < R1; ++n1) sm[n1] = S[R2 * n1];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int n1 = 0; n1 < R1; ++n1) v[n1] = cadd(v[n1], cmul(sm[n1], pv[m][n1]));
                }
            }
            dft_dir<R1, false>(v);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) xr1[k1 * (R2 + 1) + t1] = tw_mul<false>(v[k1], tw, t1 * k1);
        }
        __syncthreads();
        if (on3) {
            float2 b[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) b[n2] = xr3[t3 * (R2 + 1) + n2];
            dft_dir<R2, false>(b);
            float2* out = a.tmp + (((size_t)s * a.C + c) * a.K + k) * NTI + tile_row(y0 + r3);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) st_stream<true>(&out[tile_col(t3 + R1 * k2, ny)], b[k2]);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// pass B: per (coil, column tile): forward column FFT of all K images, the K x K
// Psi mix at every frequency (all K spectra of a column are held by the same
// thread), inverse column FFT; in place.  MODE 1 (adjoint): inverse FFT only of
// natural-order spectra.
// ---------------------------------------------------------------------------
template <int L>
constexpr int colB() { return 256 / RegGeom<L>::P; }

template <int L, int K>
__global__ __launch_bounds__(colB<L>() * RegGeom<L>::P) void k_passB(ClassArgs a, int s0, int want_quad) {
    using G = RegGeom<L>;
    constexpr int R1 = G::R1, R2 = G::R2, P = G::P, TB = G::TB, W = colB<L>(), NT = W * P;
    static_assert(NT >= 64, "block_sum_ragged needs a full first wave");
    __shared__ float2 tw[L];
    __shared__ float2 xb[W * TB];

    // With kOrderXcdB (the default when the class's Psi table exceeds 2 MB, more than
    // stays in an XCD's L2 while the pass streams) the workgroups go coil fastest, each
    // XCD a contiguous run of (slice, column tile), so the C workgroups that read the
    // same columns of the table run back to back on one XCD and share them through its
    // L2 (the 384 x 384, K = 5 table is 9.4 MB; dealt round-robin, every coil re-read
    // it from the Infinity Cache and the pass fetched 2.6x its algorithmic bytes)
    const Blk bk = block_coords(a.order & kOrderXcdB);
    const int s = s0 + bk.z;
    if (!slice_active(a, s)) return;
    const int c = bk.y;
    const int tid = threadIdx.x;
    const int w = tid / P, t = tid - w * P;
    const int nz = a.nz;
    const int z = bk.x * W + w;
    const bool colok = z < nz;
    const size_t N = tmp_image(L, nz);   // image stride of the tiled intermediate
    for (int i = tid; i < L; i += NT) tw[i] = a.twy[i];
    __syncthreads();
    // columns past nz (last tile) read column 0 and are never stored: no selects between
    // the loads and their first use, so the next coefficient's loads stay in flight
    // this thread's first element: column z, row t (t < 16); row R2 n1 + t of the column
    // is then a compile-time offset tile_row(R2 n1) away (R2 divides 16)
    static_assert(16 % R2 == 0, "tile rows: R2 must divide 16");
    float2* col = a.tmp + ((size_t)s * a.C + c) * (size_t)K * N + tile_col(colok ? z : 0, L) + t;
    float2* xw = xb + w * TB;

    float2 F[K][R2];
    // coefficient k's column is in col2[k & 1]; the next one loads into the other buffer
    // while k is transformed.  Two buffers rather than a copy "v = next": where only
    // some lanes load (R2 < P, e.g. 16 of 24 at 384 points) such a copy is merged at the
    // end of their block, and the merge waits for the loads in flight, before the
    // exchange barrier; with alternating buffers the loads stay in flight across it.
    float2 col2[2][R1];
    if (t < R2) {
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) col2[0][n1] = ld_stream<passB_nt<L>()>(&col[tile_row(R2 * n1)]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (t < R2) {
            if (k + 1 < K) {
#pragma unroll
                for (int n1 = 0; n1 < R1; ++n1)
                    col2[(k + 1) & 1][n1] = ld_stream<passB_nt<L>()>(&col[(size_t)(k + 1) * N + tile_row(R2 * n1)]);
            }
            float2(&v)[R1] = col2[k & 1];
            dft_dir<R1, false>(v);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) xw[k1 * (R2 + 1) + t] = tw_mul<false>(v[k1], tw, t * k1);
        }
        __syncthreads();
        if (t < R1) {
            float2 b[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) b[n2] = xw[t * (R2 + 1) + n2];
            dft_dir<R2, false>(b);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) F[k][k2] = b[k2];
        }
        __syncthreads();
    }
    double quad = 0.0;   // sum over this thread's frequencies of v^H Psi v
    if (t < R1 && colok) {
        // kernel table in pass-B order: float4 groups of the KP (>= K(K+1)/2, multiple
        // of 4) values of frequency t + R1 k2 of column z, thread index fastest
        constexpr int KT = K * (K + 1) / 2;
        constexpr int KP = (KT + 3) / 4 * 4;
        const float4* psi = (const float4*)a.psi + (size_t)z * R2 * (KP / 4) * R1 + t;
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
            float q[KP];
#pragma unroll
            for (int j = 0; j < KP / 4; ++j) {
                const float4 w = psi[(k2 * (KP / 4) + j) * R1];
                q[4 * j] = w.x;
                q[4 * j + 1] = w.y;
                q[4 * j + 2] = w.z;
                q[4 * j + 3] = w.w;
            }
            float2 v[K];
#pragma unroll
            for (int kk = 0; kk < K; ++kk) v[kk] = F[kk][k2];
            float qf = 0.0f;
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
                float2 acc = make_float2(0.f, 0.f);
#pragma unroll
                for (int l = 0; l < K; ++l) {
                    const int lo = kk < l ? kk : l, hi = kk < l ? l : kk;
                    const int tri = lo * K - (lo * (lo - 1)) / 2 + (hi - lo);
                    acc.x += q[tri] * v[l].x;
                    acc.y += q[tri] * v[l].y;
                }
                F[kk][k2] = acc;
                qf += v[kk].x * acc.x + v[kk].y * acc.y;
            }
            quad += (double)qf;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (t < R1) {
            float2 b[R2];
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) b[k2] = F[k][k2];
            dft_dir<R2, true>(b);
#pragma unroll
            for (int m1 = 0; m1 < R2; ++m1) xw[m1 * (R1 + 1) + t] = tw_mul<true>(b[m1], tw, t * m1);
        }
        __syncthreads();
        if (t < R2) {
            float2 v[R1];
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) v[k1] = xw[t * (R1 + 1) + k1];
            dft_dir<R1, true>(v);
            if (colok) {
#pragma unroll
                for (int m2 = 0; m2 < R1; ++m2) st_stream<passB_nt<L>()>(&col[(size_t)k * N + tile_row(R2 * m2)], v[m2]);
            }
        }
        __syncthreads();
    }
    if (want_quad) {
        // W P threads need not fill whole waves (e.g. 12 x 20 for ny = 320); the
        // exchange buffer is free after the last transform and holds the partials
        static_assert(W * TB * sizeof(float2) >= NT * sizeof(double), "exchange buffer too small");
        const double tot = block_sum_ragged(quad, reinterpret_cast<double*>(xb));
        if (tid == 0) a.pb[(size_t)s * a.npb + c * gridDim.x + bk.x] = tot;
    }
}

template <int L>
__global__ __launch_bounds__(colB<L>() * RegGeom<L>::P) void k_passB_inv(ClassArgs a, int s0) {
    using G = RegGeom<L>;
    constexpr int R1 = G::R1, R2 = G::R2, P = G::P, TB = G::TB, W = colB<L>(), NT = W * P;
    __shared__ float2 tw[L];
    __shared__ float2 xb[W * TB];

    const int s = s0 + blockIdx.z;
    if (!slice_active(a, s)) return;
    const int c = blockIdx.y;
    const int tid = threadIdx.x;
    const int w = tid / P, t = tid - w * P;
    const int nz = a.nz;
    const int z = blockIdx.x * W + w;
    const bool colok = z < nz;
    const size_t N = tmp_image(L, nz);   // image stride of the tiled intermediate
    for (int i = tid; i < L; i += NT) tw[i] = a.twy[i];
    __syncthreads();
    float2* col = a.tmp + ((size_t)s * a.C + c) * (size_t)a.K * N + tile_col(colok ? z : 0, L);
    float2* xw = xb + w * TB;
    for (int k = 0; k < a.K; ++k) {
        if (t < R1) {
            float2 b[R2];
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2)
                b[k2] = col[(size_t)k * N + tile_row(t + R1 * k2)];
            dft_dir<R2, true>(b);
#pragma unroll
            for (int m1 = 0; m1 < R2; ++m1) xw[m1 * (R1 + 1) + t] = tw_mul<true>(b[m1], tw, t * m1);
        }
        __syncthreads();
        if (t < R2) {
            float2 v[R1];
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) v[k1] = xw[t * (R1 + 1) + k1];
            dft_dir<R1, true>(v);
            if (colok) {
#pragma unroll
                for (int m2 = 0; m2 < R1; ++m2) col[(size_t)k * N + tile_row(t + R2 * m2)] = v[m2];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// pass C: per (row tile, k): for every coil, read the tiled spectra (row-fastest
// lanes), inverse row FFT, conj(S_c) (.) accumulated in registers; then
// out = acc + rho_add p (MODE 0), out = acc (MODE 1), or the CG step (MODE 2):
// w = acc + rho p, a = gamma / <p, M p>, x += a p, r -= a w, partial <r, r>.
// ---------------------------------------------------------------------------
template <int L, int MODE, int M, int NBUF>
__global__ __launch_bounds__(rows_threads<L>()) __attribute__((amdgpu_waves_per_eu(1, kPassCWavesPerSimd)))
void k_passC(ClassArgs a, int s0, float rho_add,
                                                              float2* __restrict__ outp, int out_s0, PartialSrc gc,
                                                              int out_buf) {
    const Blk bk = block_coords(a.order & kOrderXcdC);
    using G = RowGeom<L>;
    constexpr int R1 = G::R1, R2 = G::R2, P = G::P, TB = G::TB, RT = kRowTile, NT = RT * P;
    static_assert(NT % 64 == 0, "block_sum needs whole waves");
    static_assert(NBUF == 1 || (NBUF == 2 && passC_lds2_ok<L>()), "pass C LDS buffers");
    __shared__ float2 tw[L];
    __shared__ float2 xb[NBUF * RT * TB];
    __shared__ double red[16];

    const int s = s0 + bk.z;
    if (!slice_active(a, s)) return;
    const int k = bk.y;
    const int y0 = bk.x * RT;
    const int ny = a.ny;
    const size_t N = (size_t)ny * L;
    const size_t NTI = tmp_image(ny, L);
    const int tid = threadIdx.x;
    for (int i = tid; i < L; i += NT) tw[i] = a.twz[i];
    __syncthreads();

    const int r1 = tid / P, t1 = tid - r1 * P;
    const bool on1 = t1 < R2;
    const int r3 = tid % RT, t3 = tid / RT;
    const bool on3 = t3 < R1;
    const size_t rowoff = (size_t)(y0 + r1) * L;

    const int KM = M * a.K;
    float2 acc[M][R1];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int i = 0; i < R1; ++i) acc[m][i] = make_float2(0.f, 0.f);
    // spectra of the next coil are loaded while the current one is transformed
    const float2* T0 = a.tmp + ((size_t)s * a.C * a.K + k) * NTI + tile_row(y0 + r3);
    const size_t cstride = (size_t)a.K * NTI;
    float2 nb[R2];
    if (on3) {
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) nb[k2] = ld_stream<true>(&T0[tile_col(t3 + R1 * k2, ny)]);
    }
    for (int c = 0; c < a.C; ++c) {
        float2* xc = xb + (NBUF == 2 ? (c & 1) * RT * TB : 0);
        float2* xr1 = xc + r1 * TB;
        float2* xr3 = xc + r3 * TB;
        if (on3) {
            float2 b[R2];
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) b[k2] = nb[k2];
            if (c + 1 < a.C) {
                const float2* in = T0 + (size_t)(c + 1) * cstride;
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) nb[k2] = ld_stream<true>(&in[tile_col(t3 + R1 * k2, ny)]);
            }
            dft_dir<R2, true>(b);
#pragma unroll
            for (int m1 = 0; m1 < R2; ++m1) xr3[m1 * (R1 + 1) + t3] = tw_mul<true>(b[m1], tw, t3 * m1);
        }
        __syncthreads();
        if (on1) {
            const float2* S = a.sens + ((size_t)s * a.C + c) * M * N + rowoff;
            if constexpr (M == 1 && R1 <= 24) {
                // the coil's map is loaded first, in flight during the LDS reads and the
                // FFT (R1 = 32 has no registers to spare for it)
                float2 sv[R1];
#pragma unroll
                for (int m2 = 0; m2 < R1; ++m2) sv[m2] = S[t1 + R2 * m2];
                __builtin_amdgcn_sched_barrier(0);
                float2 v[R1];
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1) v[k1] = xr1[t1 * (R1 + 1) + k1];
                dft_dir<R1, true>(v);
#pragma unroll
                for (int m2 = 0; m2 < R1; ++m2) acc[0][m2] = cadd(acc[0][m2], cmulc(v[m2], sv[m2]));
            } else {
                float2 v[R1];
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1) v[k1] = xr1[t1 * (R1 + 1) + k1];
                dft_dir<R1, true>(v);
                // every map set combines the same coil image: acc_m += conj(S_(c,m)) (.)
#pragma unroll
                for (int m = 0; m < M; ++m)
#pragma unroll
                    for (int m2 = 0; m2 < R1; ++m2)
                        acc[m][m2] = cadd(acc[m][m2], cmulc(v[m2], S[(size_t)m * N + t1 + R2 * m2]));
            }
        }
        if constexpr (NBUF == 1) __syncthreads();
    }
    if constexpr (MODE == 2) {
        // <p, M p> = <p, A^H A p> (pass-B partials) + rho ||p||^2 (pass-A partials)
        const double gamma = partial_sum(gc, s);
        const double pmp = partial_sum(PartialSrc{a.pb, a.npb, a.npb}, s) +
                           (double)a.rho * partial_sum(PartialSrc{a.pa, a.nrw, a.nrw}, s);
        const float alpha = (gamma > 0.0 && pmp > 0.0) ? (float)(gamma / pmp) : 0.0f;
        double dot = 0.0;
        if (on1) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const size_t vo = ((size_t)s * KM + m * a.K + k) * N + rowoff + t1;
                dot += cg_row_update<R1, R2>(acc[m], a.p + vo, a.x + vo, a.r + vo, a.rho, alpha);
            }
        }
        const double tot = block_sum(dot, red);
        if (tid == 0) a.rr[((size_t)s * 2 + out_buf) * a.nrw + bk.y * gridDim.x + bk.x] = tot;
    } else {
        if (on1) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                float2* out = outp + ((size_t)(s - out_s0) * KM + m * a.K + k) * N + rowoff;
                const float2* pp = a.p + ((size_t)s * KM + m * a.K + k) * N + rowoff;
#pragma unroll
                for (int m2 = 0; m2 < R1; ++m2) {
                    const int pos = t1 + R2 * m2;
                    float2 w = acc[m][m2];
                    if constexpr (MODE == 0) {
                        const float2 pv = pp[pos];
                        w = make_float2(w.x + rho_add * pv.x, w.y + rho_add * pv.y);
                    }
                    out[pos] = w;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// projection of the samples onto the basis (adjoint input), uncentred, in the tiled
// layout: tmp[c][k] at (y', z') for q = z' ny + y', value
// (-1)^(y'+z') / sqrt(N) * sum_{samples at the centred location of q} phi[t][k] y_c
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_project(ClassArgs a, int s0) {
    const int s = s0 + blockIdx.z;
    const int c = blockIdx.y;
    const int ny = a.ny, nz = a.nz;
    const int N = ny * nz;
    const int q = blockIdx.x * kThreads + threadIdx.x;
    if (q >= N) return;
    const int K = a.K;
    const float2* y = a.ksp + ((size_t)s * a.C + c) * a.P;
    float2 acc[kMaxK];
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) acc[k] = make_float2(0.f, 0.f);
    const int e0 = a.row_ptr[q], e1 = a.row_ptr[q + 1];
    for (int e = e0; e < e1; ++e) {
        const int t = a.ent_t[e];
        const float2 v = y[a.ent_p[e]];
#pragma unroll
        for (int k = 0; k < kMaxK; ++k)
            if (k < K) {
                const float f = a.phi[t * K + k];
                acc[k].x += f * v.x;
                acc[k].y += f * v.y;
            }
    }
    const int yp = q % ny, zp = q / ny;
    const float sc = (((yp + zp) & 1) ? -1.0f : 1.0f) / sqrtf((float)N);
    const size_t NTI = tmp_image(ny, nz);
    float2* out = a.tmp + ((size_t)s * a.C + c) * K * NTI + tix(yp, zp, ny);
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
        if (k < K) out[(size_t)k * NTI] = cscale(acc[k], sc);
}

// ---------------------------------------------------------------------------
// state initialisation: x = z = alpha0 (or 0), u = 0, r = b0 - (sub_w ? w : 0)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_init(ClassArgs a, int s0, const float2* __restrict__ alpha0, int sub_w) {
    __shared__ double red[kThreads / 64];
    const int s = s0 + blockIdx.z;
    const size_t n = (size_t)a.M * a.K * a.ny * a.nz;
    const size_t base = (size_t)s * n;
    const float2* a0 = alpha0 ? alpha0 + (size_t)(s - s0) * n : nullptr;
    double dot = 0.0, bb = 0.0;
    for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += (size_t)gridDim.x * kThreads) {
        const float2 xv = a0 ? a0[e] : make_float2(0.f, 0.f);
        const float2 bv = a.b0[base + e];
        float2 rv = bv;
        if (sub_w) rv = csub(rv, a.w[base + e]);
        a.x[base + e] = xv;
        a.z[base + e] = xv;
        a.u[base + e] = make_float2(0.f, 0.f);
        a.r[base + e] = rv;
        dot += (double)rv.x * rv.x + (double)rv.y * rv.y;
        bb += (double)bv.x * bv.x + (double)bv.y * bv.y;
    }
    const double tot = block_sum(dot, red);
    if (threadIdx.x == 0) a.g0[(size_t)s * a.nllr + blockIdx.x] = tot;
    const double tb = block_sum(bb, red);
    if (threadIdx.x == 0) a.b0n[(size_t)s * a.nllr + blockIdx.x] = tb;
}

// ---------------------------------------------------------------------------
// LLR: complex Hermitian Jacobi (cyclic, FP64) on the K x K Gram matrix
// ---------------------------------------------------------------------------
struct cd2 {
    double x, y;
};
__device__ __forceinline__ cd2 dmul(cd2 a, cd2 b) { return cd2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd2 dconj(cd2 a) { return cd2{a.x, -a.y}; }

template <int K>
__device__ __forceinline__ void jacobi_eig(cd2 (&A)[K][K], cd2 (&V)[K][K]) {
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) V[i][j] = cd2{i == j ? 1.0 : 0.0, 0.0};
    for (int sweep = 0; sweep < 12; ++sweep) {
        double off = 0.0, dia = 0.0;
#pragma unroll
        for (int p = 0; p < K; ++p) {
            dia += A[p][p].x * A[p][p].x;
#pragma unroll
            for (int q = p + 1; q < K; ++q) off += A[p][q].x * A[p][q].x + A[p][q].y * A[p][q].y;
        }
        if (off <= 1e-30 * dia || off == 0.0) break;
#pragma unroll
        for (int p = 0; p < K; ++p) {
#pragma unroll
            for (int q = p + 1; q < K; ++q) {
                const cd2 apq = A[p][q];
                const double g = sqrt(apq.x * apq.x + apq.y * apq.y);
                if (g == 0.0) continue;
                const cd2 e = cd2{apq.x / g, apq.y / g};  // phase of a_pq
                const double th = (A[q][q].x - A[p][p].x) / (2.0 * g);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double sn = t * c;
                const cd2 ec = dconj(e);
                // columns p, q:  A <- A J,  J = [[c, sn], [-sn conj(e), c conj(e)]]
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const cd2 aip = A[i][p], aiq = A[i][q];
                    const cd2 t1 = dmul(ec, aiq);
                    A[i][p] = cd2{c * aip.x - sn * t1.x, c * aip.y - sn * t1.y};
                    A[i][q] = cd2{sn * aip.x + c * t1.x, sn * aip.y + c * t1.y};
                    const cd2 vip = V[i][p], viq = V[i][q];
                    const cd2 t2 = dmul(ec, viq);
                    V[i][p] = cd2{c * vip.x - sn * t2.x, c * vip.y - sn * t2.y};
                    V[i][q] = cd2{sn * vip.x + c * t2.x, sn * vip.y + c * t2.y};
                }
                // rows p, q:  A <- J^H A
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const cd2 apj = A[p][j], aqj = A[q][j];
                    const cd2 t1 = dmul(e, aqj);
                    A[p][j] = cd2{c * apj.x - sn * t1.x, c * apj.y - sn * t1.y};
                    A[q][j] = cd2{sn * apj.x + c * t1.x, sn * apj.y + c * t1.y};
                }
                A[p][q] = cd2{0.0, 0.0};
                A[q][p] = cd2{0.0, 0.0};
                A[p][p].y = 0.0;
                A[q][q].y = 0.0;
            }
        }
    }
}

// FISTA point of one voxel and coefficient: the gradient step y - step (A^H A y - b0)
// from the momentum point y (held in z), A^H A y (in w) and b0 = A^H y_data
__device__ __forceinline__ float2 fista_point(const ClassArgs& a, size_t i, float step) {
    const float2 y = a.z[i], g = csub(a.w[i], a.b0[i]);
    return make_float2(y.x - step * g.x, y.y - step * g.y);
}

constexpr int pow2_at_least(int b) { return b <= 1 ? 1 : 2 * pow2_at_least((b + 1) / 2); }

// MODE kLlrAdmm: z = SVT(x + u) with the ADMM u and right-hand-side updates.
// MODE kLlrProx: out = SVT(in) at an explicit shift.
// MODE kLlrFista: x_new = SVT(y - step (A^H A y - b0)), the next momentum point
// y = x_new + (t_k - 1) / t_(k+1) (x_new - x) into z (Beck & Teboulle's momentum
// sequence t_0 = 1, t_(k+1) = (1 + sqrt(1 + 4 t_k^2)) / 2, from the iteration counter).
// At K = 5 the Gram and eigenvector matrices (FP64 complex, 5 x 5 each) take the
// kernel just past the registers of two waves per SIMD (256 + 27); asking for two
// waves spills 112 bytes per lane and still runs 22 % faster (10.96 -> 8.56 ms per
// 512-slice launch at 384^2).  Larger K would spill far more and keep one wave.
template <int K>
constexpr int llr_min_waves() { return K == 5 ? 2 : 1; }

template <int K, int B, int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(llr_min_waves<K>())))
void k_llr(ClassArgs a, int s0, int kouter, const float2* __restrict__ inp,
                                                   float2* __restrict__ outp, float tau, int sy_arg, int sz_arg,
                                                   float step) {
    __shared__ double red[kThreads / 64];
    constexpr bool kState = MODE == kLlrAdmm || MODE == kLlrFista;   // class vectors, device counter
    const int s = s0 + blockIdx.z;
    if (kState && !slice_active(a, s)) return;
    const int ny = a.ny, nz = a.nz;
    const size_t N = (size_t)ny * nz;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // a wave holds BW blocks side by side, GW lanes each (B of them active: one lane per
    // block column); the last block row / column is partial when B does not divide the
    // grid
    constexpr int GW = pow2_at_least(B), BW = 64 / GW;
    const int nby = (ny + B - 1) / B, nbz = (nz + B - 1) / B;
    const int nsz = (nbz + BW - 1) / BW;
    const int nstrips = nby * nsz;
    // every map set (soft-SENSE) has its own blocks of its K images: the a.nllr
    // workgroups of a slice are a.M runs of nllr / M
    const int wpm = a.nllr / a.M;
    const int mset = blockIdx.x / wpm;
    const int st = (blockIdx.x - mset * wpm) * (kThreads / 64) + wave;

    int sy = sy_arg, sz = sz_arg;
    if (kState) {
        // outer index from the device counter (so an outer iteration can be replayed
        // from a captured graph); a frozen shift overrides it
        const int fk = a.state[4 * s + 1];
        const uint64_t kk = (uint64_t)(fk >= 0 ? fk : a.state[4 * s + 2]);
        const uint64_t h = sm64(sm64(sm64(a.seed) ^ (uint64_t)a.state[4 * s + 3]) ^ kk);
        sy = (int)((h & 0xFFFFFFFFull) % (uint64_t)B);
        sz = (int)((h >> 32) % (uint64_t)B);
    }
    const size_t vb = ((size_t)(kState ? s : s - s0) * a.M + mset) * K * N;
    float mom = 0.0f;
    if (MODE == kLlrFista) {
        const int kk = a.state[4 * s + 2];
        double t = 1.0;
        for (int j = 0; j < kk; ++j) t = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        mom = (float)((t - 1.0) / (0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t))));
    }
    const bool valid = st < nstrips;
    const int prow = valid ? st / nsz : 0;
    const int jl = lane % GW;
    const int col = ((valid ? (st % nsz) : 0) * BW + lane / GW) * B + jl;
    const bool act = valid && jl < B && col < nz;
    const int zc = (col + sz) % nz;
    const int nrows = min(B, ny - prow * B);   // rows of this block row (partial at the end)

    // ---- Gram matrix of this lane's block (FP64) ----
    cd2 G[K][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int l = 0; l < K; ++l) G[k][l] = cd2{0.0, 0.0};
    if (act) {
        for (int i = 0; i < B; ++i) {
            if (i >= nrows) break;
            const int yr = (prow * B + i + sy) % ny;
            const size_t idx = (size_t)yr * nz + zc;
            float2 v[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (MODE == kLlrAdmm) v[k] = cadd(a.x[vb + k * N + idx], a.u[vb + k * N + idx]);
                else if (MODE == kLlrFista) v[k] = fista_point(a, vb + k * N + idx, step);
                else v[k] = inp[vb + k * N + idx];
            }
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int l = k; l < K; ++l) {
                    // conj(v_k) v_l
                    G[k][l].x += (double)v[k].x * v[l].x + (double)v[k].y * v[l].y;
                    G[k][l].y += (double)v[k].x * v[l].y - (double)v[k].y * v[l].x;
                }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int l = k; l < K; ++l) {
#pragma unroll
            for (int o = 1; o < GW; o <<= 1) {
                G[k][l].x += __shfl_xor(G[k][l].x, o);
                G[k][l].y += __shfl_xor(G[k][l].y, o);
            }
        }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        G[k][k].y = 0.0;
#pragma unroll
        for (int l = 0; l < k; ++l) G[k][l] = dconj(G[l][k]);
    }
    // ---- eigen-decomposition and shrinkage matrix W = V diag(f) V^H ----
    cd2 V[K][K];
    jacobi_eig<K>(G, V);
    double f[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const double lam = G[i][i].x;
        const double sg = lam > 0.0 ? sqrt(lam) : 0.0;
        f[i] = sg > (double)tau ? (sg - (double)tau) / sg : 0.0;
    }
    float2 Wm[K][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int l = 0; l < K; ++l) {
            double wx = 0.0, wy = 0.0;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const cd2 t = dmul(V[k][i], dconj(V[l][i]));
                wx += f[i] * t.x;
                wy += f[i] * t.y;
            }
            Wm[k][l] = make_float2((float)wx, (float)wy);
        }
    // ---- apply: z_l = sum_k v_k W_kl, fused ADMM updates ----
    double s_az = 0.0, s_zz = 0.0, s_a = 0.0, s_z = 0.0, s_u = 0.0, s_r = 0.0;
    if (act) {
        for (int i = 0; i < B; ++i) {
            if (i >= nrows) break;
            const int yr = (prow * B + i + sy) % ny;
            const size_t idx = vb + (size_t)yr * nz + zc;
            float2 v[K], xv[K], uv[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (MODE == kLlrAdmm) {
                    xv[k] = a.x[idx + k * N];
                    uv[k] = a.u[idx + k * N];
                    v[k] = cadd(xv[k], uv[k]);
                } else if (MODE == kLlrFista) {
                    xv[k] = a.x[idx + k * N];
                    v[k] = fista_point(a, idx + k * N, step);
                } else {
                    v[k] = inp[idx + k * N];
                }
            }
#pragma unroll
            for (int l = 0; l < K; ++l) {
                float2 zl = make_float2(0.f, 0.f);
#pragma unroll
                for (int k = 0; k < K; ++k) zl = cadd(zl, cmul(v[k], Wm[k][l]));
                if (MODE == kLlrAdmm) {
                    const float2 zo = a.z[idx + l * N];
                    const float2 rv = a.r[idx + l * N];
                    const float2 un = csub(v[l], zl);
                    // r += rho ((z - u_new) - (z_old - u_old))
                    const float2 d = csub(csub(zl, un), csub(zo, uv[l]));
                    const float2 rn = make_float2(rv.x + a.rho * d.x, rv.y + a.rho * d.y);
                    a.z[idx + l * N] = zl;
                    a.u[idx + l * N] = un;
                    a.r[idx + l * N] = rn;
                    const float2 az = csub(xv[l], zl), dz = csub(zl, zo);
                    s_az += (double)az.x * az.x + (double)az.y * az.y;
                    s_zz += (double)dz.x * dz.x + (double)dz.y * dz.y;
                    s_a += (double)xv[l].x * xv[l].x + (double)xv[l].y * xv[l].y;
                    s_z += (double)zl.x * zl.x + (double)zl.y * zl.y;
                    s_u += (double)un.x * un.x + (double)un.y * un.y;
                    s_r += (double)rn.x * rn.x + (double)rn.y * rn.y;
                } else if (MODE == kLlrFista) {
                    const float2 dx = csub(zl, xv[l]);
                    a.x[idx + l * N] = zl;
                    a.z[idx + l * N] = make_float2(zl.x + mom * dx.x, zl.y + mom * dx.y);
                    s_az += (double)dx.x * dx.x + (double)dx.y * dx.y;
                    s_a += (double)xv[l].x * xv[l].x + (double)xv[l].y * xv[l].y;
                    s_z += (double)zl.x * zl.x + (double)zl.y * zl.y;
                } else {
                    outp[idx + l * N] = zl;
                }
            }
        }
    }
    if (kState) {
        // FISTA: slot 0 ||x_new - x||^2, 2 ||x||^2, 3 ||x_new||^2 (1, 4, 5 stay 0)
        double sums[6] = {s_az, s_zz, s_a, s_z, s_u, s_r};
        double* dst = a.llr + ((size_t)s * a.nllr + blockIdx.x) * 8;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const double t = block_sum(sums[j], red);
            if (threadIdx.x == 0) {
                dst[j] = t;
                if (MODE == kLlrAdmm && j == 5) a.g0[(size_t)s * a.nllr + blockIdx.x] = t;
            }
        }
    }
}

__global__ void k_llr_finalize(ClassArgs a, int s0) {
    const int s = s0 + blockIdx.x;
    if (!slice_active(a, s)) return;
    const int j = threadIdx.x;
    const int k = a.state[4 * s + 2];
    if (j < 6 && k < a.hist_len) {
        double acc = 0.0;
        for (int i = 0; i < a.nllr; ++i) acc += a.llr[((size_t)s * a.nllr + i) * 8 + j];
        a.hist[((size_t)s * a.hist_len + k) * 8 + j] = acc;
    }
    __syncthreads();
    if (j == 0) a.state[4 * s + 2] = k + 1;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

bool fft_col_supported(int L) { return fft_col_length_supported(L); }
bool fft_row_supported(int L) { return fft_row_length_supported(L); }

int llr_workgroups(int ny, int nz, int b) {
    if (b != 4 && b != 8 && b != 12 && b != 16) return 0;
    // one wave per strip of b rows x (64 / GW) blocks, GW = b rounded up to a power of two
    const int bw = 64 / pow2_at_least(b);
    const int nby = (ny + b - 1) / b, nbz = (nz + b - 1) / b;
    const int strips = nby * ((nbz + bw - 1) / bw);
    return (strips + kThreads / 64 - 1) / (kThreads / 64);
}

bool reg_plan(int L, int* R1, int* R2) {
    switch (L) {
#define X(n)                          \
    case n:                           \
        *R1 = RegPlan<n>::R1;         \
        *R2 = RegPlan<n>::R2;         \
        return true;
        X(16) X(32) X(48) X(64) X(96) X(128) X(160) X(192) X(240) X(256) X(320) X(384) X(512)
#undef X
    }
    return false;
}

// LDS of the row passes (pass C's with two buffers where it has them, the largest)
template <int L>
static size_t rows_lds() {
    return (L + (passC_lds2_ok<L>() ? 2 : 1) * kRowTile * RowGeom<L>::TB) * sizeof(float2) + 16 * sizeof(double);
}
template <int L>
static size_t cols_lds() { return (L + colB<L>() * RegGeom<L>::TB) * sizeof(float2); }

// column lengths (every pass) and the row-only lengths (passes A and C)
#define T2S_FOR_LENGTHS(X) \
    X(16) X(32) X(48) X(64) X(96) X(128) X(160) X(192) X(240) X(256) X(320) X(384) X(512)
#define T2S_FOR_ROW_LENGTHS(X) T2S_FOR_LENGTHS(X) X(260)

size_t lds_bytes_passA(int nz) {
    switch (nz) {
#define X(L) case L: return rows_lds<L>();
        T2S_FOR_ROW_LENGTHS(X)
#undef X
    }
    return 0;
}

size_t lds_bytes_passB(int ny, int) {
    switch (ny) {
#define X(L) case L: return cols_lds<L>();
        T2S_FOR_LENGTHS(X)
#undef X
    }
    return 0;
}

int passB_columns(int ny, int) {
    switch (ny) {
#define X(L) case L: return colB<L>();
        T2S_FOR_LENGTHS(X)
#undef X
    }
    return 1;
}

hipError_t launch_passA(const ClassArgs& a, int s0, int count, const float2* src, int src_s0, int first,
                        PartialSrc gc, PartialSrc gp, int want_pp, hipStream_t st) {
    const dim3 grid(a.ny / kRowTile, a.K, count);
    switch (a.nz) {
#define X(L)                                                                                                       \
    case L:                                                                                                        \
        if (a.M == 2)                                                                                              \
            hipLaunchKernelGGL((k_passA<L, 2>), grid, dim3(rows_threads<L>()), 0, st, a, s0, src, src_s0, first,   \
                               gc, gp, want_pp);                                                                   \
        else                                                                                                       \
            hipLaunchKernelGGL((k_passA<L, 1>), grid, dim3(rows_threads<L>()), 0, st, a, s0, src, src_s0, first,   \
                               gc, gp, want_pp);                                                                   \
        break;
        T2S_FOR_ROW_LENGTHS(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L>
static hipError_t launch_passB_L(const ClassArgs& a, int s0, int count, int mode, int wq, hipStream_t st) {
    constexpr int W = colB<L>();
    const dim3 grid((a.nz + W - 1) / W, a.C, count);
    const dim3 block(W * RegGeom<L>::P);
    if (mode == 1) {
        hipLaunchKernelGGL(k_passB_inv<L>, grid, block, 0, st, a, s0);
        return hipGetLastError();
    }
    switch (a.K) {
        case 1: hipLaunchKernelGGL((k_passB<L, 1>), grid, block, 0, st, a, s0, wq); break;
        case 2: hipLaunchKernelGGL((k_passB<L, 2>), grid, block, 0, st, a, s0, wq); break;
        case 3: hipLaunchKernelGGL((k_passB<L, 3>), grid, block, 0, st, a, s0, wq); break;
        case 4: hipLaunchKernelGGL((k_passB<L, 4>), grid, block, 0, st, a, s0, wq); break;
        case 5: hipLaunchKernelGGL((k_passB<L, 5>), grid, block, 0, st, a, s0, wq); break;
        case 6: hipLaunchKernelGGL((k_passB<L, 6>), grid, block, 0, st, a, s0, wq); break;
        case 7: hipLaunchKernelGGL((k_passB<L, 7>), grid, block, 0, st, a, s0, wq); break;
        case 8: hipLaunchKernelGGL((k_passB<L, 8>), grid, block, 0, st, a, s0, wq); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_passB(const ClassArgs& a, int s0, int count, int mode, int want_quad, hipStream_t st) {
    switch (a.ny) {
#define X(L) case L: return launch_passB_L<L>(a, s0, count, mode, want_quad, st);
        T2S_FOR_LENGTHS(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
}

// pass C with one or two LDS buffers as the class's schedule flags say
template <int L, int MODE, int M>
static void launch_passC_t(const ClassArgs& a, dim3 grid, int s0, float rho_add, float2* out, int out_s0,
                           PartialSrc gc, int out_buf, hipStream_t st) {
    if constexpr (passC_lds2_ok<L>()) {
        if (a.order & kOrderLds2C) {
            hipLaunchKernelGGL((k_passC<L, MODE, M, 2>), grid, dim3(rows_threads<L>()), 0, st, a, s0, rho_add, out,
                               out_s0, gc, out_buf);
            return;
        }
    }
    hipLaunchKernelGGL((k_passC<L, MODE, M, 1>), grid, dim3(rows_threads<L>()), 0, st, a, s0, rho_add, out, out_s0,
                       gc, out_buf);
}

hipError_t launch_passC(const ClassArgs& a, int s0, int count, int mode, float rho_add, float2* out,
                        int out_s0, hipStream_t st) {
    const dim3 grid(a.ny / kRowTile, a.K, count);
    const PartialSrc none{nullptr, 0, 0};
    switch (a.nz) {
#define X(L)                                                                                 \
    case L:                                                                                  \
        if (mode == 0 && a.M == 2)                                                           \
            launch_passC_t<L, 0, 2>(a, grid, s0, rho_add, out, out_s0, none, 0, st);         \
        else if (mode == 0)                                                                  \
            launch_passC_t<L, 0, 1>(a, grid, s0, rho_add, out, out_s0, none, 0, st);         \
        else if (a.M == 2)                                                                   \
            launch_passC_t<L, 1, 2>(a, grid, s0, rho_add, out, out_s0, none, 0, st);         \
        else                                                                                 \
            launch_passC_t<L, 1, 1>(a, grid, s0, rho_add, out, out_s0, none, 0, st);         \
        break;
        T2S_FOR_ROW_LENGTHS(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_passC_cg(const ClassArgs& a, int s0, int count, PartialSrc gc, int out_buf, hipStream_t st) {
    const dim3 grid(a.ny / kRowTile, a.K, count);
    switch (a.nz) {
#define X(L)                                                                    \
    case L:                                                                     \
        if (a.M == 2)                                                           \
            launch_passC_t<L, 2, 2>(a, grid, s0, 0.0f, nullptr, 0, gc, out_buf, st); \
        else                                                                    \
            launch_passC_t<L, 2, 1>(a, grid, s0, 0.0f, nullptr, 0, gc, out_buf, st); \
        break;
        T2S_FOR_ROW_LENGTHS(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool passC_lds2_supported(int nz) {
    switch (nz) {
#define X(L) case L: return passC_lds2_ok<L>();
        T2S_FOR_ROW_LENGTHS(X)
#undef X
    }
    return false;
}

int default_order(int ny, int nz, int K) {
    const size_t psi_bytes = (size_t)ny * nz * ((K * (K + 1) / 2 + 3) / 4 * 16);
    return (psi_bytes > (2u << 20) ? kOrderXcdB : 0) | (nz >= 384 ? kOrderLds2C : 0);
}

hipError_t launch_project(const ClassArgs& a, int s0, int count, hipStream_t st) {
    const int N = a.ny * a.nz;
    const dim3 grid((N + kThreads - 1) / kThreads, a.C, count);
    hipLaunchKernelGGL(k_project, grid, dim3(kThreads), 0, st, a, s0);
    return hipGetLastError();
}

hipError_t launch_init(const ClassArgs& a, int s0, int count, const float2* alpha0, int sub_w, hipStream_t st) {
    const dim3 grid(a.nllr, 1, count);
    hipLaunchKernelGGL(k_init, grid, dim3(kThreads), 0, st, a, s0, alpha0, sub_w);
    return hipGetLastError();
}

template <int K, int B>
static void launch_llr_kb(const ClassArgs& a, int s0, int count, int mode, int k, const float2* in, float2* out,
                          float tau, int sy, int sz, float step, hipStream_t st) {
    const dim3 grid(a.nllr, 1, count);
    if (mode == kLlrAdmm)
        hipLaunchKernelGGL((k_llr<K, B, kLlrAdmm>), grid, dim3(kThreads), 0, st, a, s0, k, in, out, tau, sy, sz, step);
    else if (mode == kLlrFista)
        hipLaunchKernelGGL((k_llr<K, B, kLlrFista>), grid, dim3(kThreads), 0, st, a, s0, k, in, out, tau, sy, sz,
                           step);
    else
        hipLaunchKernelGGL((k_llr<K, B, kLlrProx>), grid, dim3(kThreads), 0, st, a, s0, k, in, out, tau, sy, sz, step);
}

template <int B>
static hipError_t launch_llr_b(const ClassArgs& a, int s0, int count, int mode, int k, const float2* in,
                               float2* out, float tau, int sy, int sz, float step, hipStream_t st) {
    switch (a.K) {
        case 1: launch_llr_kb<1, B>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st); break;
        case 2: launch_llr_kb<2, B>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st); break;
        case 3: launch_llr_kb<3, B>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st); break;
        case 4: launch_llr_kb<4, B>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st); break;
        case 5: launch_llr_kb<5, B>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st); break;
        case 6: launch_llr_kb<6, B>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st); break;
        case 7: launch_llr_kb<7, B>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st); break;
        case 8: launch_llr_kb<8, B>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_llr(const ClassArgs& a, int s0, int count, int mode, int k, const float2* in, float2* out,
                      float tau, int sy, int sz, float step, hipStream_t st) {
    switch (a.block) {
        case 4: return launch_llr_b<4>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st);
        case 8: return launch_llr_b<8>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st);
        case 12: return launch_llr_b<12>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st);
        case 16: return launch_llr_b<16>(a, s0, count, mode, k, in, out, tau, sy, sz, step, st);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// readout pre-step: the 1D unitary inverse DFT along the fully sampled readout that
// decouples a 3D acquisition into independent slices (Sec. II-A end, Sec. IV-A).
// in [C][P][L]: per coil and per sampled (echo, y, z) entry in mask order, the L
// readout samples; out [L][C][P]: slice x, coil, sample (what t2s_load_slices reads).
// Centred like the 2D transform: index kx is frequency kx - L/2 and x is position
// x - L/2, so X[x] = (-1)^(x + L/2) L^-1/2 sum_kx (-1)^kx Y[kx] exp(+2 pi i kx x / L).
// A workgroup transforms `readout_lines` consecutive entries of one coil with the
// register two-step plan of the solver passes (one LDS exchange per transform) and
// stages the result through the same LDS so the stores go out with the entry index
// fastest: 16 entries give 128-byte runs (74 KB of LDS at 512 points; 8 entries there
// measured 11 % slower).  The LDS Stockham version (4 or 8 entries per workgroup) ran
// at 1.2-2.5 TB/s.
// ---------------------------------------------------------------------------
template <int L>
constexpr int readout_lines() { return 16; }
template <int L>
constexpr int readout_lds() {
    constexpr int a = readout_lines<L>() * RegGeom<L>::TB, b = L * (readout_lines<L>() + 1);
    return a > b ? a : b;
}

template <int L>
__global__ __launch_bounds__(readout_lines<L>() * RegGeom<L>::P) void k_readout_ifft(const float2* __restrict__ in,
                                                                                   float2* __restrict__ out, int C,
                                                                                   int P) {
    using G = RegGeom<L>;
    constexpr int R1 = G::R1, R2 = G::R2, PT = G::P, TB = G::TB, LT = readout_lines<L>(), NT = LT * PT;
    __shared__ float2 tw[L];
    __shared__ float2 xb[readout_lds<L>()];
    const int c = blockIdx.y;
    const int p0 = blockIdx.x * LT;
    const int tid = threadIdx.x;
    const int line = tid / PT, th = tid - line * PT;
    const bool ok = p0 + line < P;
    for (int m = tid; m < L; m += NT) {
        double sn, cs;
        sincospi(-2.0 * m / L, &sn, &cs);
        tw[m] = make_float2((float)cs, (float)sn);
    }
    __syncthreads();
    float2* xw = xb + line * TB;
    // step 1: thread th < R1 holds Y[th + R1 k2] (k2 < R2), with the (-1)^kx centring sign
    if (th < R1) {
        const float2* src = in + ((size_t)c * P + p0 + line) * L + th;
        float2 b[R2];
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
            float2 v = make_float2(0.f, 0.f);
            if (ok) v = ld_stream<true>(&src[R1 * k2]);
            b[k2] = ((th + R1 * k2) & 1) ? make_float2(-v.x, -v.y) : v;
        }
        dft_dir<R2, true>(b);
#pragma unroll
        for (int m1 = 0; m1 < R2; ++m1) xw[m1 * (R1 + 1) + th] = tw_mul<true>(b[m1], tw, th * m1);
    }
    __syncthreads();
    // step 3: thread th < R2 ends with x[th + R2 m2] (m2 < R1)
    float2 v[R1];
    if (th < R2) {
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) v[k1] = xw[th * (R1 + 1) + k1];
        dft_dir<R1, true>(v);
    }
    __syncthreads();
    if (th < R2) {
#pragma unroll
        for (int m2 = 0; m2 < R1; ++m2) xb[(th + R2 * m2) * (LT + 1) + line] = v[m2];
    }
    __syncthreads();
    const float sc = (float)(1.0 / sqrt((double)L));
    for (int i = tid; i < LT * L; i += NT) {
        const int x = i / LT, t = i - x * LT;
        if (p0 + t < P) {
            const float2 r = xb[x * (LT + 1) + t];
            const float f = ((x + L / 2) & 1) ? -sc : sc;
            st_stream<true>(&out[((size_t)x * C + c) * P + p0 + t], make_float2(r.x * f, r.y * f));
        }
    }
}

hipError_t launch_readout_ifft(int nx, int C, int P, const float2* in, float2* out, hipStream_t st) {
    if (P == 0) return hipSuccess;
    switch (nx) {
#define X(L)                                                                                                   \
    case L: {                                                                                                  \
        const dim3 grid((P + readout_lines<L>() - 1) / readout_lines<L>(), C);                                 \
        hipLaunchKernelGGL(k_readout_ifft<L>, grid, dim3(readout_lines<L>() * RegGeom<L>::P), 0, st, in, out, C, P); \
        break;                                                                                                 \
    }
        X(16) X(32) X(48) X(64) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(512)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// post-step (Sec. II-B end; Sec. IV-A post-processing): spatial wavelet
// soft-threshold of every coefficient image, then back-projection x_t = sum_k
// phi_tk alpha_k at chosen echo times (eq. backproj).
// Wavelet: orthonormal separable 2D Haar, `levels` <= 4.  A J-level Haar transform
// only combines values inside aligned 2^J x 2^J squares, so 16 x 16 tiles are
// transformed independently.  One 2 x 2 Haar step maps a block (a b; c d) to LL, LH
// (z detail), HL (y detail), HH; the higher levels run in place on the approximation
// grid: at stride h the block (y, z), (y, z+h), (y+h, z), (y+h, z+h) becomes LL, LH,
// HL, HH in the same places.  Every position that is not a final approximation then
// holds a detail coefficient and is shrunk: c -> c max(1 - thr / |c|, 0).  The
// inverse levels undo the steps (the step is its own inverse).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void haar_block(float2& a, float2& b, float2& c, float2& d) {
    const float2 s0 = cadd(a, b), d0 = csub(a, b), s1 = cadd(c, d), d1 = csub(c, d);
    a = make_float2(0.5f * (s0.x + s1.x), 0.5f * (s0.y + s1.y));
    b = make_float2(0.5f * (d0.x + d1.x), 0.5f * (d0.y + d1.y));
    c = make_float2(0.5f * (s0.x - s1.x), 0.5f * (s0.y - s1.y));
    d = make_float2(0.5f * (d0.x - d1.x), 0.5f * (d0.y - d1.y));
}

__device__ __forceinline__ float2 shrink(float2 v, float thr) {
    const float r = sqrtf(v.x * v.x + v.y * v.y);
    const float f = r > thr ? 1.0f - thr / r : 0.0f;
    return make_float2(v.x * f, v.y * f);
}

// Four 16 x 16 tiles per workgroup (consecutive in row-major tile order), 64 threads
// per tile.  Level 1 runs in registers: each thread owns one 2 x 2 block (two 16-byte
// row loads); its three details stay in registers and its approximation goes to an
// 8 x 8 LDS grid per tile, where levels 2..J run with the in-place scheme above.
constexpr int kHaarTiles = kThreads / 64;

__global__ __launch_bounds__(kThreads) void k_haar_denoise(ClassArgs a, int s0, int levels, float thr) {
    __shared__ float2 t[kHaarTiles][8][9];
    const int s = s0 + blockIdx.z;
    const int k = blockIdx.y;
    const int w = threadIdx.x / 64, q = threadIdx.x % 64;
    const int ntz = a.nz / 16, ntiles = (a.ny / 16) * ntz;
    const int tile = blockIdx.x * kHaarTiles + w;
    const bool on = tile < ntiles;               // uniform over each wave
    const int by = q / 8, bz = q % 8;
    float2* img = a.x + ((size_t)s * a.M * a.K + k) * a.ny * a.nz;   // k: image index over M K
    const size_t g0 = on ? (size_t)((tile / ntz) * 16 + 2 * by) * a.nz + (tile % ntz) * 16 + 2 * bz : 0;
    float2 v00, v01, v10, v11;
    if (on) {
        v00 = img[g0];
        v01 = img[g0 + 1];
        v10 = img[g0 + a.nz];
        v11 = img[g0 + a.nz + 1];
        haar_block(v00, v01, v10, v11);
        v01 = shrink(v01, thr);
        v10 = shrink(v10, thr);
        v11 = shrink(v11, thr);
        t[w][by][bz] = v00;
    }
    __syncthreads();
    for (int j = 1, h = 1; j < levels; ++j, h <<= 1) {
        const int nb = 4 / h;
        if (on && q < nb * nb) {
            const int y = (q / nb) * 2 * h, z = (q % nb) * 2 * h;
            haar_block(t[w][y][z], t[w][y][z + h], t[w][y + h][z], t[w][y + h][z + h]);
        }
        __syncthreads();
    }
    const int m = (1 << (levels - 1)) - 1;
    if (on && ((by & m) || (bz & m))) t[w][by][bz] = shrink(t[w][by][bz], thr);
    __syncthreads();
    for (int j = levels - 1; j >= 1; --j) {
        const int h = 1 << (j - 1), nb = 4 / h;
        if (on && q < nb * nb) {
            const int y = (q / nb) * 2 * h, z = (q % nb) * 2 * h;
            haar_block(t[w][y][z], t[w][y][z + h], t[w][y + h][z], t[w][y + h][z + h]);
        }
        __syncthreads();
    }
    if (on) {
        v00 = t[w][by][bz];
        haar_block(v00, v01, v10, v11);
        img[g0] = v00;
        img[g0 + 1] = v01;
        img[g0 + a.nz] = v10;
        img[g0 + a.nz + 1] = v11;
    }
}

hipError_t launch_haar_denoise(const ClassArgs& a, int s0, int count, int levels, float thr, hipStream_t st) {
    const int ntiles = (a.ny / 16) * (a.nz / 16);
    const dim3 grid((ntiles + kHaarTiles - 1) / kHaarTiles, a.M * a.K, count);
    hipLaunchKernelGGL(k_haar_denoise, grid, dim3(kThreads), 0, st, a, s0, levels, thr);
    return hipGetLastError();
}

// out[s][m][j][n] = sum_k phi_te[j][k] alpha[s][m][k][n] for slices [s0, s0 + count) and
// map sets m (out holds slices from s0 on); one thread per voxel, all echo times at once
struct PhiTe {
    float v[kMaxK * kMaxK];
};
__global__ __launch_bounds__(kThreads) void k_backproject(ClassArgs a, int s0, int nte, PhiTe ph, float2* out) {
    const int s = s0 + blockIdx.y, m = blockIdx.z;
    const size_t N = (size_t)a.ny * a.nz;
    const int K = a.K;
    const float2* al = a.x + ((size_t)s * a.M + m) * K * N;
    float2* o = out + ((size_t)(s - s0) * a.M + m) * nte * N;
    for (size_t n = (size_t)blockIdx.x * kThreads + threadIdx.x; n < N; n += (size_t)gridDim.x * kThreads) {
        float2 v[kMaxK];
#pragma unroll
        for (int k = 0; k < kMaxK; ++k) v[k] = k < K ? al[k * N + n] : make_float2(0.f, 0.f);
        for (int j = 0; j < nte; ++j) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int k = 0; k < kMaxK; ++k) {
                const float w = ph.v[j * kMaxK + k];   // 0 for k >= K
                acc.x += w * v[k].x;
                acc.y += w * v[k].y;
            }
            o[j * N + n] = acc;
        }
    }
}

hipError_t launch_backproject(const ClassArgs& a, int s0, int count, int nte, const float* phi_te, float2* out,
                              hipStream_t st) {
    PhiTe ph{};
    for (int j = 0; j < nte; ++j)
        for (int k = 0; k < a.K; ++k) ph.v[j * kMaxK + k] = phi_te[j * a.K + k];
    const size_t N = (size_t)a.ny * a.nz;
    const int gx = (int)std::min<size_t>((N + kThreads - 1) / kThreads, 1024);
    hipLaunchKernelGGL(k_backproject, dim3(gx, count, a.M), dim3(kThreads), 0, st, a, s0, nte, ph, out);
    return hipGetLastError();
}

// v[s] /= ||p[s]|| with ||p||^2 from the pass-A partials (0 when the norm is 0): the
// renormalisation of the power iteration for the largest eigenvalue of A^H A
__global__ __launch_bounds__(kThreads) void k_normalize(ClassArgs a, int s0, float2* v) {
    __shared__ float fac;
    const int s = s0 + blockIdx.y;
    if (threadIdx.x == 0) {
        const double nn = partial_sum(PartialSrc{a.pa, a.nrw, a.nrw}, s);
        fac = nn > 0.0 ? (float)(1.0 / sqrt(nn)) : 0.0f;
    }
    __syncthreads();
    const size_t n = (size_t)a.M * a.K * a.ny * a.nz;
    float2* vs = v + (size_t)s * n;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
        vs[i] = make_float2(vs[i].x * fac, vs[i].y * fac);
}

hipError_t launch_normalize(const ClassArgs& a, int s0, int count, float2* v, hipStream_t st) {
    const size_t n = (size_t)a.M * a.K * a.ny * a.nz;
    const int gx = (int)std::min<size_t>((n + kThreads - 1) / kThreads, 1024);
    hipLaunchKernelGGL(k_normalize, dim3(gx, count), dim3(kThreads), 0, st, a, s0, v);
    return hipGetLastError();
}

__global__ void k_set_state(ClassArgs a, int s0, int count, int active, int frozen, int kreset, int gfirst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        a.state[4 * (s0 + i)] = active;
        a.state[4 * (s0 + i) + 1] = frozen;
        if (kreset >= 0) a.state[4 * (s0 + i) + 2] = kreset;
        if (gfirst >= 0) a.state[4 * (s0 + i) + 3] = gfirst + i;
    }
}

hipError_t launch_set_state(const ClassArgs& a, int s0, int count, int active, int frozen, int kreset,
                            hipStream_t st, int gfirst) {
    hipLaunchKernelGGL(k_set_state, dim3((count + 63) / 64), dim3(64), 0, st, a, s0, count, active, frozen, kreset,
                       gfirst);
    return hipGetLastError();
}

// empty kernel: marks where the library's event timing starts and stops in an
// external kernel trace
__global__ void k_profile_mark() {}

hipError_t launch_profile_mark(hipStream_t st) {
    hipLaunchKernelGGL(k_profile_mark, dim3(1), dim3(64), 0, st);
    return hipGetLastError();
}

hipError_t launch_llr_finalize(const ClassArgs& a, int s0, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_llr_finalize, dim3(count), dim3(64), 0, st, a, s0);
    return hipGetLastError();
}

}  // namespace t2s
