// kernels.hpp -- device-side data description and launchers of the T2-Shuffling
// slice solver kernels (gfx950).  Shared by kernels.hip and api.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace t2s {

constexpr int kThreads = 256;   // threads per workgroup of every kernel
constexpr int kRowTile = 16;    // rows per workgroup of the row-FFT passes
constexpr int kMaxK = 8;

// Sum of `count` per-workgroup partial sums of slice s, in a fixed order.
struct PartialSrc {
    const double* base;  // slice s at base + s * stride (nullptr: the sum is 0)
    int stride;
    int count;
};

// Device view of one shape class (all slices of the class in one allocation).
struct ClassArgs {
    int ny, nz, C, K, T, P;      // grid, coils, subspace, echoes, samples per coil
    int M;                       // coil-map sets (soft-SENSE): coefficient vectors hold M K
                                 // images per slice, the maps C M
    int nrw, npb, nllr;          // partial-sum counts per slice: row-pass workgroups (passes A
                                 // and C: ny / kRowTile * K), pass-B workgroups, LLR workgroups
                                 // (M runs, one per map set)
    int hist_len;                // outer-iteration capacity of the residual history
    int block;                   // LLR block edge
    int order;                   // kernel schedule flags (kOrder*): XCD-grouped workgroup
                                 // orders of passes A, C and B, pass C's LDS buffers
    float tau, rho;              // LLR threshold lambda / rho, ADMM penalty
    uint64_t seed;
    const float* psi;            // upper triangle of Psi, uncentred, / (ny nz), in pass-B order:
                                 // [nz][R2][KP/4][R1][4] for frequency y' = t + R1 k2 (t < R1,
                                 // k2 < R2), KP = K(K+1)/2 rounded up to a multiple of 4
    const float2* twy;           // W_ny^m, m < ny
    const float2* twz;           // W_nz^m, m < nz
    const float* phi;            // [T][K]
    const int* row_ptr;          // [ny nz + 1] over uncentred transposed positions q = z' ny + y'
    const int* ent_t;            // echo of each sample entry
    const int* ent_p;            // sample index (within a coil's P) of each entry
    float2* sens;                // [S][C][M][ny][nz]
    float2* ksp;                 // [S][C][P]
    float2 *b0, *x, *r, *p, *w, *z, *u;   // [S][M][K][ny][nz]
    float2* tmp;                 // [S][C][K][nz/16][ny/16][16][16]  pass intermediate (k-space,
                                 // 16 x 16 tiles, y fastest inside a tile)
    double* pa;                  // [S][nrw]    ||p||^2 partials of pass A
    double* pb;                  // [S][npb]    k-space partials of <p, A^H A p> (pass B)
    double* rr;                  // [S][2][nrw] <r, r> partials of the CG update (pass C)
    double* g0;                  // [S][nllr]   <r, r> at the start of an outer iteration
    double* b0n;                 // [S][nllr]   ||b0||^2 partials (written with the state init)
    double* llr;                 // [S][nllr][8] residual partial sums of the z-step
    double* hist;                // [S][hist_len][8] per-outer residual sums
    int* state;                  // [S][4]: active flag, frozen outer index (-1: none), outer counter,
                                 // global slice index (the block-shift schedule's g)
};

constexpr int kOrderXcdA = 1;    // pass A workgroups dealt to the XCDs in runs of row tiles
constexpr int kOrderXcdC = 2;    // the same for pass C
constexpr int kOrderXcdB = 4;    // pass B coil-fastest, dealt in runs (coils of a column tile share Psi)
constexpr int kOrderLds2C = 8;   // pass C double-buffers its LDS exchange (row lengths >= 256)
constexpr int kOrderAll = 15;

// schedule flags a class starts with before any tuning: pass B's coil-fastest order
// when the class's Psi table exceeds 2 MB, pass C's two LDS buffers from 384 points
int default_order(int ny, int nz, int K);
// whether pass C has its two-buffer variant at this row length
bool passC_lds2_supported(int nz);

// LLR kernel flavours
enum LlrMode { kLlrAdmm = 0, kLlrProx = 1, kLlrFista = 2 };

// ---- launchers (return hipSuccess or the launch error) ----
// s0/count: slices [s0, s0 + count) of the class.

// p = first ? src : r + beta p (beta from gc / gp); tmp[c][k] = FFT_z(S_c p_k), transposed
// (src holds slices [src_s0, ...): slice s reads src + (s - src_s0) K N); with
// want_pp the partial ||p||^2 of every workgroup goes to pa
hipError_t launch_passA(const ClassArgs& a, int s0, int count, const float2* src, int src_s0, int first,
                        PartialSrc gc, PartialSrc gp, int want_pp, hipStream_t st);
// mode 0: column FFT, Psi mix, column IFFT (in place on tmp), with want_quad the
// partial k-space sums of <p, A^H A p> to pb; mode 1: column IFFT only
hipError_t launch_passB(const ClassArgs& a, int s0, int count, int mode, int want_quad, hipStream_t st);
// mode 0: out = sum_c conj(S_c) IFFT_z(tmp) + rho_add p
// mode 1: out = sum_c conj(S_c) IFFT_z(tmp)
// (out holds slices [out_s0, ...))
hipError_t launch_passC(const ClassArgs& a, int s0, int count, int mode, float rho_add, float2* out,
                        int out_s0, hipStream_t st);
// CG step with the update fused: w = sum_c conj(S_c) IFFT_z(tmp) + rho p stays in
// registers; a = gamma / (sum pb + rho sum pa) with gamma from gc; x += a p,
// r -= a w; partial <r, r> into rr[out_buf]
hipError_t launch_passC_cg(const ClassArgs& a, int s0, int count, PartialSrc gc, int out_buf, hipStream_t st);
// tmp[c][k] = projected, sign-modulated, uncentred k-space of the samples (adjoint input)
hipError_t launch_project(const ClassArgs& a, int s0, int count, hipStream_t st);
// x = z = alpha0 (or 0), u = 0, r = b0 - (sub_w ? w : 0); partial <r, r> into g0 and
// ||b0||^2 into b0n
hipError_t launch_init(const ClassArgs& a, int s0, int count, const float2* alpha0, int sub_w, hipStream_t st);
// ADMM z/u/r update with the shift of the slice's outer counter (mode kLlrAdmm;
// k unused), out = prox(in) at the explicit shift (mode kLlrProx), or one FISTA step
// x = prox(z - step (w - b0)), z = x + momentum (x - x_old) with the shift and the
// momentum of the slice's counter (mode kLlrFista; step used only there)
hipError_t launch_llr(const ClassArgs& a, int s0, int count, int mode, int k, const float2* in, float2* out,
                      float tau, int sy, int sz, float step, hipStream_t st);
// post-step: in-place `levels`-level (1..4) orthonormal 2D Haar soft-threshold of every
// coefficient image of alpha (ny, nz multiples of 16), slices [s0, s0 + count)
hipError_t launch_haar_denoise(const ClassArgs& a, int s0, int count, int levels, float thr, hipStream_t st);
// out[s - s0][j] = sum_k phi_te[j][k] alpha[s][k] (phi_te host [nte][K], nte <= kMaxK)
hipError_t launch_backproject(const ClassArgs& a, int s0, int count, int nte, const float* phi_te, float2* out,
                              hipStream_t st);
// readout pre-step: out[x][c][p] = centred unitary inverse DFT over kx of in[c][p][kx]
// (nx a supported FFT length, 0 < C <= 65535, P >= 0; in and out must not overlap)
hipError_t launch_readout_ifft(int nx, int C, int P, const float2* in, float2* out, hipStream_t st);
// v[s] /= sqrt(sum of the pass-A partials pa[s]) for slices [s0, s0 + count)
hipError_t launch_normalize(const ClassArgs& a, int s0, int count, float2* v, hipStream_t st);
// state[s] = (active, frozen[, counter = kreset if kreset >= 0][, global index = gfirst + s - s0
// if gfirst >= 0]) for slices [s0, s0 + count)
hipError_t launch_set_state(const ClassArgs& a, int s0, int count, int active, int frozen, int kreset,
                            hipStream_t st, int gfirst = -1);
// an empty kernel marking where event timing starts / stops (for external traces)
hipError_t launch_profile_mark(hipStream_t st);
// hist[s][counter] = sum of the LLR partials of slice s; counter += 1
hipError_t launch_llr_finalize(const ClassArgs& a, int s0, int count, hipStream_t st);

// lengths with an FFT plan: as a column length ny (all passes) / as a row length nz
bool fft_col_supported(int L);
bool fft_row_supported(int L);
// workgroups of the LLR kernel per slice (one partial-sum slot each); 0 for an
// unsupported block size
int llr_workgroups(int ny, int nz, int b);
// two-step register plan L = R1 * R2 of the passes (false if L has no plan)
bool reg_plan(int L, int* R1, int* R2);
size_t lds_bytes_passA(int nz);
size_t lds_bytes_passB(int ny, int K);
int passB_columns(int ny, int K);

}  // namespace t2s
