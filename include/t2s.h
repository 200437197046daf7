/*
 * t2s.h -- C ABI of the MI355X (gfx950) T2-Shuffling slice reconstruction library.
 *
 * The library solves, independently for every readout slice, the subspace-
 * constrained PICS problem of the paper (Anderson, Tamir et al., arXiv 1809.04195,
 * Sec. II-B, eq. t2shpics):
 *
 *     argmin_alpha  1/2 || y - P F S Phi alpha ||_2^2  +  lambda * sum_blocks || R(alpha) ||_*
 *
 * with y the measured k-space samples of every echo and coil in truncated form
 * (Sec. II-A: P in {0,1}^{P x N}), S the coil maps, F the centred unitary 2D DFT,
 * Phi in R^{T x K} the temporal basis (eq. backproj) and R the extraction of
 * non-overlapping b x b blocks of the K coefficient images under a random circular
 * shift drawn anew every iteration (Sec. II-B, end; single-pass form Sec. IV-C).
 * The solver is scaled ADMM whose alpha-step runs CG on A^H A + rho I, with the
 * normal operator applied through the space-time kernel Psi(n) = Phi^T P(n) Phi
 * (Sec. IV-B, eqs. commute / normaleq, Alg. 1).
 *
 * Conventions
 * -----------
 *  * Return value: 0 = success, > 0 = warning, < 0 = error (T2S_E*).  The message
 *    of the last non-zero return of the calling thread is t2s_last_error().
 *  * Complex data are complex64: interleaved (re, im) float32 pairs.
 *  * Image-domain arrays are row-major [..][ny][nz] (nz contiguous).  Mask and
 *    k-space index j means frequency j - n/2 (centred; DC at (ny/2, nz/2)).
 *  * Samples ("ksp") of one slice are [ncoils][P_tot] in mask order: echo-major,
 *    then row-major (y, z) position inside the echo's mask.
 *  * `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    Calls are stream-ordered and asynchronous unless stated otherwise.
 *  * `mem` is T2S_HOST or T2S_DEVICE and says where a caller buffer lives.
 *    Host buffers are copied before the call returns.  Device buffers must stay
 *    valid until the stream has executed the operation.  The library never frees
 *    caller memory.
 *  * Argument validation (shapes, pointers, finiteness of host inputs) happens
 *    before any HIP call, so every error path can be exercised without a GPU.
 *  * A plan is not thread-safe; distinct plans are independent.
 */
#ifndef T2S_H
#define T2S_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define T2S_OK 0
#define T2S_WNOTCONVERGED 1   /* tolerance mode: some slice hit n_outer before tol   */
#define T2S_EINVAL (-1)       /* null pointer, bad enum, bad numeric parameter       */
#define T2S_ESHAPE (-2)       /* odd or non-multiple-of-block dims, K > 8, K > T ... */
#define T2S_ENOMEM (-3)       /* workspace missing or too small                      */
#define T2S_EHIP (-4)         /* HIP runtime error (message carries its text)        */
#define T2S_ESTATE (-5)       /* call out of order (e.g. reconstruct before load)    */
#define T2S_ENONFINITE (-6)   /* NaN / Inf in Phi, parameters, maps or samples       */
#define T2S_EUNSUPPORTED (-7) /* grid length without a compiled FFT plan             */

#define T2S_HOST 0
#define T2S_DEVICE 1

#define T2S_BATCHED 0        /* launches cover the slices of a class (per its schedule) */
#define T2S_PER_SLICE 1      /* one launch sequence per slice (baseline schedule)       */
#define T2S_BATCHED_GRAPH 2  /* T2S_BATCHED with one outer iteration captured in a HIP
                                graph and replayed (falls back to T2S_BATCHED while
                                kernel timing is enabled)                              */

#define T2S_ALPHA 0
#define T2S_Z 1
#define T2S_U 2
#define T2S_ADJOINT 3   /* b0 = A^H y of the loaded samples */
#define T2S_RESIDUAL 4  /* CG residual r = b0 + rho (z - u) - (A^H A + rho I) alpha, kept
                           up to date by the z-step for the next alpha-step */

#define T2S_MAX_K 8

/* Solver parameters shared by all shape classes of a plan. */
typedef struct t2s_params {
    int T;                 /* echoes (rows of phi)                                   */
    int K;                 /* subspace size (columns of phi), 1..T2S_MAX_K, K <= T   */
    const float* phi;      /* host, real [T][K] row-major; copied at plan creation   */
    float lambda;          /* LLR weight (absolute; data are not rescaled)           */
    float rho;             /* ADMM penalty; LLR threshold is lambda / rho            */
    int block;             /* LLR block edge b (ny, nz multiples of b)               */
    int n_outer;           /* outer iterations (fixed mode) or cap (tolerance mode)  */
    int n_cg;              /* CG iterations per outer iteration (>= 1)               */
    float tol;             /* 0: fixed iterations; > 0: stop at max(r_p, r_d) <= tol */
    uint64_t seed;         /* block-shift schedule seed (SplitMix64)                 */
    int freeze_window;     /* tolerance mode: stall window (outer iterations)        */
    float freeze_stall;    /* tolerance mode: relative fall below which shifts freeze */
    int check_every;       /* tolerance mode: decisions every this many iterations   */
} t2s_params;

/* One shape class: slices sharing grid, coil count and sampling masks. */
typedef struct t2s_class {
    int ny, nz;            /* slice grid: ny a column length with an FFT plan (a     */
                           /* multiple of 16: 16 ... 512), nz a row length (those or  */
                           /* 260); blocks are partial where b does not divide them   */
    int ncoils;            /* C >= 1                                                 */
    int nslices;           /* slices of this class held by the plan                  */
    const uint8_t* masks;  /* host [T][ny][nz], 1 = sampled; copied at creation      */
    int nmaps;             /* coil-map sets M (soft-SENSE, Sec. II-A; Alg. 1's maps  */
                           /* S_(i,0), S_(i,1)): 0 or 1 = one set, 2 = two.  With M   */
                           /* sets the maps are [C][M][ny][nz] per slice, the unknown */
                           /* has M K images ([M][K][ny][nz] per slice: K coefficient */
                           /* images per set), coil c sees sum_m S_(c,m) x_m, and the */
                           /* LLR blocks are taken per set                            */
} t2s_class;

/* Per-slice outcome of the last t2s_reconstruct. */
typedef struct t2s_slice_report {
    int outer_iterations;  /* outer iterations run                                   */
    int k_freeze;          /* outer index whose shift was frozen (-1: never)         */
    int converged;         /* tolerance mode: 1 if max(r_p, r_d) <= tol             */
    double r_primal;       /* ||alpha - z|| / d after the last outer iteration, with */
                           /* d = max(||alpha||, ||z||, 0.01 ||b0||) (0 when d = 0)   */
    double r_dual;         /* ||z - z_prev|| / d (dual residual rho (z - z_prev)      */
                           /* relative to rho times the solution scale)               */
} t2s_slice_report;

typedef struct t2s_plan t2s_plan;

/* Library version (major * 10000 + minor * 100 + patch). */
int t2s_version(void);

/* Thread-local message for the last non-zero return (never NULL). */
const char* t2s_last_error(void);

/* Validate parameters and classes, build the host-side plan: the space-time kernel
 * Psi(n) = sum_{t: m_t(n)=1} phi_t^T phi_t (Sec. IV-B) in FP64, stored as its upper
 * triangle (k <= l), real, shifted to uncentred FFT order and scaled by 1/(ny nz)
 * (fp32), and the location -> sample map used to project the samples onto the
 * basis (Sec. III-A, "re-sort and project").  No HIP call is made.
 * Errors: T2S_EINVAL, T2S_ESHAPE, T2S_ENONFINITE, T2S_EUNSUPPORTED. */
int t2s_plan_create(const t2s_params* params, const t2s_class* classes, int n_classes,
                    t2s_plan** out);

/* Free host state.  Device memory is the caller's and is not touched. */
int t2s_plan_destroy(t2s_plan* plan);

/* Device workspace (bytes) needed by the plan: kernel tables, per-slice coil maps,
 * samples, solver vectors and pass intermediates. */
int t2s_plan_workspace_bytes(const t2s_plan* plan, size_t* bytes);

/* Bind caller-owned device memory (>= t2s_plan_workspace_bytes, 256-byte aligned)
 * and upload the plan tables on `stream`.  Errors: T2S_ENOMEM, T2S_EHIP. */
int t2s_plan_bind_workspace(t2s_plan* plan, void* device_ptr, size_t bytes, void* stream);

/* Load slices [first, first + count) of class `cls`: coil maps sens
 * (complex64 [count][ncoils][ny][nz]) and samples ksp (complex64
 * [count][ncoils][P_tot], mask order), both in `mem`, and compute the adjoint
 * b0 = A^H y = sum_c conj(S_c) F^H (Phi^T P^H y_c) on the device.
 * The samples are the data y of eq. t2shpics (Sec. II-B) in the truncated form of
 * Sec. II-A (P in {0,1}^{P x N} keeps only the acquired entries of each echo); the
 * projection onto the basis and the re-sorting by k-space location are the "re-sort
 * and project" step of Sec. III-A, done here per slice on the device; the maps are
 * S of eq. coilmodel.  Resets the slices to the cold start alpha = z = u = 0.
 * Host inputs are checked for NaN / Inf (T2S_ENONFINITE).  Host buffers are copied
 * before the call returns; device buffers must stay valid until `stream` has run
 * the load.  Errors: T2S_EINVAL (NULL, class or slice range, mem), T2S_ESTATE
 * (workspace not bound), T2S_ENONFINITE, T2S_EHIP. */
int t2s_load_slices(t2s_plan* plan, int cls, int first, int count, const void* sens,
                    const void* ksp, int mem, void* stream);

/* Warm start: alpha = z = alpha0 (complex64 [count][K][ny][nz] in `mem`), u = 0, and
 * the CG residual r = b0 - A^H A alpha0.  The paper starts its iteration from zero
 * (Sec. II-A: FISTA on eq. t2shpics); any start reaches the same minimiser of the
 * convex problem at a fixed block shift, so the start only changes how many
 * iterations the stop rule of t2s_reconstruct needs.  Must follow t2s_load_slices
 * for these slices.  Host alpha0 is checked for NaN / Inf and copied before the call
 * returns.  Errors: T2S_EINVAL, T2S_ESTATE (slice not loaded), T2S_ENONFINITE,
 * T2S_EHIP. */
int t2s_set_initial(t2s_plan* plan, int cls, int first, int count, const void* alpha0,
                    int mem, void* stream);

/* Solve eq. t2shpics (Sec. II-B) for every loaded slice independently (the
 * per-slice decoupling of Sec. II-A end / Sec. IV-E): scaled ADMM (Boyd et al. 2011,
 * Sec. 3.1.1) with z-step = the blocked LLR prox of Sec. II-B end / Sec. IV-C at
 * threshold lambda / rho, u-step u += alpha - z, and alpha-step n_cg CG iterations on
 * (A^H A + rho I) alpha = b0 + rho (z - u) with A^H A applied through Psi (Sec. IV-B,
 * Alg. 1).  mode = T2S_BATCHED, T2S_BATCHED_GRAPH or T2S_PER_SLICE (same
 * arithmetic, different launch schedule).  Errors: T2S_EINVAL (mode), T2S_ESTATE
 * (workspace not bound or a slice not loaded), T2S_EHIP.  Fixed mode (tol == 0) is fully
 * asynchronous.  Tolerance mode synchronises `stream` every check_every outer
 * iterations to read the per-slice residuals and decides per slice, in this order:
 * stop if max(r_p, r_d) <= tol; else freeze the block shift at the current draw if
 * max(r_p, r_d) fell by less than freeze_stall over freeze_window iterations (with a
 * new shift every iteration ADMM has no fixed point and the residual stalls well
 * above tol).  Returns T2S_WNOTCONVERGED if a slice reached n_outer without meeting
 * tol. */
int t2s_reconstruct(t2s_plan* plan, int mode, void* stream);

/* Batching schedule of class `cls`: pass launches cover `chunk` slices (0 = all
 * slices of the class) and are spread round-robin over `nstreams` (1..8)
 * library-owned streams, so the pass intermediate of the slices in flight stays in
 * the on-package cache between passes; the caller's stream waits for all of them.
 * Same arithmetic for every schedule. */
int t2s_set_schedule(t2s_plan* plan, int cls, int chunk, int nstreams);
int t2s_get_schedule(const t2s_plan* plan, int cls, int* chunk, int* nstreams);

/* Kernel schedule flags of class `cls` (the passes of Alg. 1, Sec. IV-B):
 * T2S_ORDER_XCD_PASS_A (T2S_ORDER_XCD_PASS_C): the workgroups of pass A (C) are dealt
 * to the device's 8 XCDs in contiguous runs of row tiles instead of round-robin;
 * T2S_ORDER_XCD_PASS_B: pass B's workgroups go coil-fastest in contiguous runs, so the
 * coils of a column tile share its Psi entries in one XCD's L2;
 * T2S_ORDER_PASS_C_LDS2: pass C double-buffers its LDS exchange (one barrier per coil
 * instead of two; row lengths >= 256, ignored below).  A new class starts with
 * T2S_ORDER_XCD_PASS_B when its Psi table exceeds 2 MB and T2S_ORDER_PASS_C_LDS2 from
 * 384 points; t2s_autotune times every combination.  Which runs faster depends on the
 * shape; same arithmetic, bitwise identical results.  Errors: T2S_EINVAL. */
#define T2S_ORDER_XCD_PASS_A 1
#define T2S_ORDER_XCD_PASS_C 2
#define T2S_ORDER_XCD_PASS_B 4
#define T2S_ORDER_PASS_C_LDS2 8
int t2s_set_order(t2s_plan* plan, int cls, int order);

/* Global index of class `cls`'s slice 0 in the block-shift schedule (default: the
 * number of slices in the classes before it).  Lets a volume be split over several
 * plans (or devices) with every slice keeping the shifts, and so the result, it has
 * in one plan.  Host-side: it reaches the device with the next t2s_load_slices,
 * t2s_set_initial, t2s_reconstruct or t2s_fista.  Errors: T2S_EINVAL. */
int t2s_set_slice_offset(t2s_plan* plan, int cls, int first_global);
int t2s_get_order(const t2s_plan* plan, int cls, int* order);

/* Pick every class's schedule by timing `reps` CG steps of passes A/B/C per
 * candidate (all slices at once; chunks of 32/16/8/4/2 slices over 1, 2 or 4
 * streams; then every combination of the kernel schedule flags of t2s_set_order with
 * the best of those) on
 * the loaded slices, on `stream`.  Results are cached per process by (ny, nz,
 * ncoils, K, slices, device architecture).  Solver state is untouched.
 * Synchronises `stream`. */
int t2s_autotune(t2s_plan* plan, int reps, void* stream);

/* Copy out alpha, z, u, b0 or r (which = T2S_ALPHA / T2S_Z / T2S_U / T2S_ADJOINT /
 * T2S_RESIDUAL) of slices [first, first + count) as complex64 [count][K][ny][nz] into
 * `out` (`mem`).  alpha is the solution of eq. t2shpics: the subspace coefficient
 * images of eq. backproj (Sec. II-B), from which x_t = sum_k Phi_tk alpha_k gives the
 * image at echo t (t2s_backproject).  A host destination synchronises `stream`.
 * Errors: T2S_EINVAL (NULL, range, which, mem), T2S_ESTATE, T2S_EHIP. */
int t2s_read_coeffs(t2s_plan* plan, int cls, int first, int count, void* out, int which,
                    int mem, void* stream);

/* Per-slice report of the last reconstruct (synchronous host call; call after the
 * stream has finished the reconstruct): outer iterations, frozen shift, convergence
 * and the final residuals.  The time per phase of the solve (passes A / B / C, LLR
 * z-step, load) comes from the plan's event timing: t2s_profile_enable before the
 * solve, t2s_profile_read after it (launches and summed milliseconds per kernel
 * family; with all slices of a class per launch the phases are shared by the slices,
 * so the timing is per plan, not per slice). */
int t2s_get_slice_report(const t2s_plan* plan, int cls, int slice, t2s_slice_report* out);

/* ---- Operator entry points (same kernels as the solver; used for verification) ---- */

/* out = A^H A in + rho_add * in for slices [first, first + count) of `cls`, using
 * their loaded coil maps and the class's Psi (Sec. IV-B, Alg. 1).  `in`, `out`:
 * device complex64 [count][K][ny][nz], must not overlap. */
int t2s_apply_normal(t2s_plan* plan, int cls, int first, int count, const void* in,
                     void* out, float rho_add, void* stream);

/* out = LLR prox with threshold tau of `in` (device complex64 [count][K][ny][nz]):
 * every non-overlapping b x b block of the K images, shifted by shifts[2 i],
 * shifts[2 i + 1] (host int, s_y, s_z in [0, b)) for slice i, replaced by its
 * singular-value soft threshold (Sec. II-B eq. llr; single pass of Sec. IV-C). */
int t2s_apply_llr(t2s_plan* plan, int cls, int first, int count, const void* in, void* out,
                  float tau, const int* shifts, void* stream);

/* ---- Readout pre-step (Sec. II-A end; Sec. IV-A, PICS reconstruction) ---- */

/* Decouple a 3D Cartesian acquisition into readout slices: the 1D unitary inverse
 * DFT along the fully sampled readout direction, centred like the 2D transform
 * (index kx is frequency kx - nx/2, x is position x - nx/2):
 *     out[x][c][p] = (1/sqrt(nx)) sum_kx in[c][p][kx] exp(+2 pi i (kx - nx/2)(x - nx/2) / nx).
 * in: device complex64 [ncoils][nsamples][nx], for every coil and every sampled
 * (echo, y, z) entry in mask order (echo-major, then row-major position inside
 * mask_t) the nx readout samples; out: device complex64 [nx][ncoils][nsamples],
 * slice x's samples in the layout t2s_load_slices reads (slices [x0, x0 + count) at
 * out + x0 * ncoils * nsamples).  Stream-ordered, asynchronous; no plan needed.
 * nx must be one of the supported FFT lengths (16 ... 512, those of the solver).
 * nsamples = 0 does nothing (in and out may then be NULL).
 * Errors: T2S_EINVAL (NULL, in and out overlap), T2S_ESHAPE (nx, ncoils outside
 * [1, 65535], nsamples < 0), T2S_EHIP. */
int t2s_readout_ifft(int nx, int ncoils, int nsamples, const void* in, void* out, void* stream);

/* ---- Post-step (Sec. II-B end, eq. backproj; Sec. IV-A post-processing) ---- */

/* Spatial wavelet soft-threshold of every coefficient image of alpha, in place, for
 * slices [first, first + count) of class `cls`: orthonormal separable 2D Haar
 * transform with `levels` (1..4) levels, every detail coefficient c replaced by
 * c max(1 - thresh / |c|, 0) (the final approximation band is kept), inverse
 * transform.  ny and nz must be multiples of 16.  Run it after the solver; the
 * result is read with t2s_read_coeffs (T2S_ALPHA).  Errors: T2S_EINVAL (levels,
 * thresh not finite or < 0, class or slice range), T2S_ESHAPE, T2S_ESTATE, T2S_EHIP. */
int t2s_wavelet_denoise(t2s_plan* plan, int cls, int first, int count, int levels, float thresh,
                        void* stream);

/* Back-projection onto echo times (eq. backproj): out[i][j] = sum_k phi_te[j][k]
 * alpha_k of slice first + i (with M coil-map sets, out[i][m][j] for every set m), for n_te (1..8) echo times whose basis rows phi_te
 * (host float [n_te][K], copied before the call returns) the caller gives, e.g. rows
 * of Phi at the desired echoes (the paper's TE 21 / 50 / 90 ms).  out: device
 * complex64 [count][n_te][ny][nz].  Errors: T2S_EINVAL, T2S_ENONFINITE, T2S_ESTATE,
 * T2S_EHIP. */
int t2s_backproject(t2s_plan* plan, int cls, int first, int count, int n_te, const float* phi_te,
                    void* out, void* stream);

/* ---- FISTA (the paper's own solver, Sec. II-A and Table 1) ---- */

/* Largest eigenvalue of A^H A for every slice of class `cls` by `iters` power
 * iterations started from b0 = A^H y (the loaded adjoint): v <- A^H A v / ||v||, and
 * L[s] = <v, A^H A v> / <v, v> of the last iteration (0 for a slice whose b0 is 0).
 * L: host double [nslices of the class].  Synchronises `stream`.  Overwrites the
 * solver's scratch vectors p and w (not alpha, z, u or the loaded data).  Errors:
 * T2S_EINVAL, T2S_ESTATE (workspace not bound or a slice not loaded), T2S_EHIP. */
int t2s_lipschitz(t2s_plan* plan, int cls, int iters, double* L, void* stream);

/* n_iter FISTA iterations (proximal gradient with Beck & Teboulle's momentum) on
 * eq. t2shpics for every slice of every class, from the current alpha (the loaded
 * start or the result of an earlier call):
 *     x_(k+1) = prox_{lambda step}( y_k - step (A^H A y_k - A^H y) ),
 *     y_(k+1) = x_(k+1) + (t_k - 1) / t_(k+1) (x_(k+1) - x_k),
 * t_0 = 1, t_(k+1) = (1 + sqrt(1 + 4 t_k^2)) / 2, y_0 = x_0 = alpha.  The prox is the
 * LLR singular-value threshold lambda * step at the block shift of slice g and
 * iteration k (the same shift schedule as the ADMM z-step, Sec. IV-C).  step must be
 * <= 1 / L for convergence (t2s_lipschitz).  mode: T2S_BATCHED (all slices of a
 * class per launch) or T2S_PER_SLICE (same arithmetic, one slice per launch).  The
 * result is alpha (t2s_read_coeffs T2S_ALPHA); the momentum point y is left in z.
 * The slice report then gives outer_iterations = n_iter and in r_primal the relative
 * size of the last step ||x_(k+1) - x_k|| / max(||x_k||, ||x_(k+1)||, 0.01 ||b0||)
 * (NaN when n_iter exceeds n_outer + 1, the history length); r_dual is 0.  The ADMM
 * state (z, u, r) is overwritten: load again (or t2s_set_initial) before an ADMM
 * reconstruct.  Errors: T2S_EINVAL (mode, n_iter < 0, step not finite or <= 0),
 * T2S_ESTATE, T2S_EHIP. */
int t2s_fista(t2s_plan* plan, int mode, int n_iter, float step, void* stream);

/* Copy the class's fp32 kernel table (upper triangle, [K(K+1)/2][nz][ny] in
 * uncentred order, scaled by 1/(ny nz)) into host memory `out`. */
int t2s_get_psi(const t2s_plan* plan, int cls, float* out);

/* ---- Kernel timing (HIP events on the plan's stream, recorded around launches) ---- */

#define T2S_KERNEL_PASS_A 0    /* S p + row FFT (first loop of Alg. 1)             */
#define T2S_KERNEL_PASS_B 1    /* column FFT, Psi mix, column IFFT (second loop)    */
#define T2S_KERNEL_PASS_C 2    /* row IFFT, coil combine, + rho p (third loop); in  */
                               /* CG fused with the x, r update                     */
#define T2S_KERNEL_LLR 3       /* LLR z-step fused with the ADMM updates            */
#define T2S_KERNEL_LOAD 4      /* projection + adjoint of load_slices               */
#define T2S_KERNEL_COUNT 5

/* Enable (1) or disable (0) event timing of every launch; enabling clears the totals.
 * With a bound workspace each call also launches an empty kernel (k_profile_mark) on
 * the plan's last stream, so a kernel trace can cut out the launches that were timed. */
int t2s_profile_enable(t2s_plan* plan, int enable);

/* Launch count and summed duration (ms) of kernel family `kernel` since the last
 * enable.  Synchronises the events (call after the stream has finished). */
int t2s_profile_read(t2s_plan* plan, int kernel, int* launches, double* total_ms);

/* The library's own block-shift schedule: SplitMix64 (Steele, Lea & Flood 2014),
 * h = sm(sm(sm(seed) ^ g) ^ k), s_y = (h mod 2^32) mod b, s_z = (h >> 32) mod b, for
 * global slice index g (class-major order) and outer iteration k.  Host only. */
int t2s_block_shift(uint64_t seed, int g, int k, int b, int* sy, int* sz);

/* ---- Learned warm start: U-Net on the zero-filled adjoint (bf16 matrix cores) ----
 *
 * Not part of the paper's method (its reconstruction is plain iterative); it
 * predicts the solver's output alpha from b0 = A^H y so that ADMM starts closer to
 * its fixed point, and the ADMM that follows still runs to the same residual.
 * Network: input b0 of each slice packed as 2K real channels (Re, Im per
 * coefficient image) divided by s = max |b0| of the slice; `levels` levels of two
 * 3x3 convolutions + ReLU with base, 2 base, 4 base ... channels, 2x2 max-pool
 * down, 2x2 stride-2 transposed convolution up with skip concatenation; final 1x1
 * convolution and a global residual; output times s.  NHWC bf16 activations, fp32
 * accumulation and fp32 master weights; parameters packed per layer in forward order
 * as W[KH][KW][Cout][Cin] followed by bias[Cout] (a transposed convolution stores
 * W[2][2][Cout][Cin]). */
typedef struct t2s_unet t2s_unet;

/* Describe a network for batches of up to max_batch slices of H x W (H, W divisible
 * by 2^(levels-1)).  No HIP call.  Errors: T2S_EINVAL, T2S_ESHAPE. */
int t2s_unet_create(int K, int base, int levels, int max_batch, int H, int W, t2s_unet** out);
int t2s_unet_destroy(t2s_unet* net);
int t2s_unet_param_count(const t2s_unet* net, size_t* count);
int t2s_unet_workspace_bytes(const t2s_unet* net, size_t* bytes);
/* Bind caller-owned device memory (256-byte aligned) and clear it. */
int t2s_unet_bind_workspace(t2s_unet* net, void* device_ptr, size_t bytes, void* stream);
/* Load (host fp32, packed) / read back the parameters; loading resets Adam.  Synchronous. */
int t2s_unet_set_params(t2s_unet* net, const float* params, void* stream);
int t2s_unet_get_params(t2s_unet* net, float* params, void* stream);
/* alpha0 = s (x + net(x)) with x = pack(b0) / s; b0, alpha0: device complex64
 * [B][K][H][W], 1 <= B <= max_batch.  An all-zero slice (s = 0) gets alpha0 = 0.
 * Asynchronous. */
int t2s_unet_forward(t2s_unet* net, const void* b0, void* alpha0, int B, void* stream);
/* One Adam step (lr; beta 0.9 / 0.999, eps 1e-8) on the mean squared error between
 * x + net(x) and target / s (target: device complex64 [B][K][H][W]).  If `loss` is not
 * NULL the loss before the step is returned (synchronises `stream`). */
int t2s_unet_train_step(t2s_unet* net, const void* b0, const void* target, int B, float lr, double* loss,
                        void* stream);
/* Verification entry: loss and packed parameter gradient for host fp32 inputs x and
 * targets t, both [B][H][W][2K] (already normalised).  Synchronous. */
int t2s_unet_loss_grad(t2s_unet* net, const float* x, const float* t, int B, double* loss, float* grad,
                       void* stream);
/* Verification entries of the optimiser: one Adam step of the training path (the
 * update t2s_unet_train_step applies after its backward pass: beta 0.9 / 0.999,
 * eps 1e-8, bias-corrected moments, step counter + 1, then the bf16 weight copies)
 * with the gradient taken from host `grad` (param_count floats, checked for NaN /
 * Inf) instead of the backward pass; synchronous.  And the optimiser state: first and
 * second moments m, v (host, param_count floats each) and the step count.
 * Errors: T2S_EINVAL, T2S_ESTATE (workspace not bound), T2S_ENONFINITE, T2S_EHIP. */
int t2s_unet_adam_apply(t2s_unet* net, const float* grad, float lr, void* stream);
int t2s_unet_get_adam_state(t2s_unet* net, float* m, float* v, int* step, void* stream);

/* Initial parameters into host `params` (param_count floats): He-normal weights
 * (standard deviation sqrt(2 / fan_in)) from a 64-bit Mersenne twister seeded with
 * `seed`, zero biases, the final 1x1 layer scaled by 0.1. */
int t2s_unet_init_params(const t2s_unet* net, uint64_t seed, float* params);

/* Shape of a network: K (complex channels), max_batch, H, W.  Any pointer may be NULL. */
int t2s_unet_get_shape(const t2s_unet* net, int* K, int* max_batch, int* H, int* W);

/* ---- Streaming a volume through a plan's slices (continuous batching) ----
 *
 * The per-slice problems of eq. t2shpics are independent (Sec. II-A: after the
 * readout transform every slice is reconstructed on its own; Sec. IV-E spreads them
 * over machines), and in tolerance mode they stop after different numbers of outer
 * iterations.  Instead of solving fixed batches, whose launches thin out as slices
 * stop, a one-class plan's S slices become slots fed from a queue of slices: at every
 * stop decision (each check_every outer iterations of a slot) the slots whose slice
 * stopped are refilled with the next queued slices in queue order (load: projection
 * and adjoint; optional network warm start; then the slot joins the next outer
 * iteration), so a caller that queues its most expensive slices first keeps the end of
 * a volume from waiting on them.  Every
 * slice runs exactly the arithmetic, stop and freeze decisions it has in
 * t2s_reconstruct (its own outer counter from 0, its own global index in the shift
 * schedule), so results equal those of a batch solve of the same slices.
 *
 * t2s_stream_open: start streaming on plan class `cls` (the plan must have exactly
 * one class, a bound workspace and tol > 0 or a fixed n_outer), all slots idle, queue
 * empty.  `net` (may be NULL: cold start) gives each loaded slice alpha0 = net(b0) as
 * t2s_set_initial does; it must have K, H = ny, W = nz of the class and M = 1.  `mode`
 * is T2S_BATCHED or T2S_BATCHED_GRAPH (an outer iteration replayed from a captured
 * graph; profiling forces eager launches).  Errors: T2S_EINVAL, T2S_ESHAPE (net shape),
 * T2S_ESTATE (workspace not bound).
 *
 * t2s_stream_submit: append `count` slices to the queue (no GPU work): their coil maps
 * `sens` (device complex64 [count][C][M][ny][nz]) and samples `ksp` (device complex64
 * [count][C][P], P the class's samples per coil), global indices first_global .. +
 * count - 1 in the shift schedule, and where to put the results: `alpha_out` (device
 * complex64 [count][M][K][ny][nz]) and `reports` (host, count entries, or NULL).  The
 * arrays must stay valid until the slices completed; the same arrays may be submitted
 * again.  Errors: T2S_EINVAL, T2S_ESTATE (not open).
 *
 * t2s_stream_run: refill, iterate and decide until at least `min_done` more slices
 * completed in this call (min_done <= 0: until the queue is empty and every slot idle)
 * or nothing is left; `status` (may be NULL) receives the counts since open.  The
 * results of completed slices are written on `stream` (synchronise it before reading
 * them).  A slice that reaches n_outer before tol completes with converged = 0 and the
 * call returns T2S_WNOTCONVERGED after finishing its work.  Errors: T2S_ESTATE (not
 * open), T2S_EHIP.
 *
 * t2s_stream_close: end streaming (queued slices are dropped); the plan can then be
 * used with t2s_load_slices / t2s_reconstruct again. */
typedef struct t2s_stream_status {
    int done;              /* slices completed since open                            */
    int in_flight;         /* slices loaded or queued and not completed              */
    int64_t loaded;        /* slices loaded into slots since open                    */
    int64_t slice_outer;   /* outer iterations run, summed over slices, since open   */
} t2s_stream_status;
int t2s_stream_open(t2s_plan* plan, int cls, t2s_unet* net, int mode);
int t2s_stream_submit(t2s_plan* plan, int count, int first_global, const void* sens, const void* ksp,
                      void* alpha_out, t2s_slice_report* reports);
int t2s_stream_run(t2s_plan* plan, int min_done, t2s_stream_status* status, void* stream);
int t2s_stream_close(t2s_plan* plan);

/* One 16x16x16 bf16 matrix-core product D = A B (host fp32 row-major, rounded to bf16
 * on input) -- a check of the lane layout the weight-gradient kernels assume. */
int t2s_unet_mfma_probe(const float* A, const float* B, float* D);
/* The same for the 32-deep product of the convolution kernels: A [16][32], B [32][16],
 * D [16][16] host fp32 row-major (A and B rounded to bf16). */
int t2s_unet_mfma_probe32(const float* A, const float* B, float* D);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the product of t2s_unet_mfma_probe
 * for `count` tiles (A, B, D host fp32 [count][16][16], D[i] = A[i] B[i]) with its
 * device staging in a static per-device buffer of the library instead of memory it
 * allocates, so the call performs no device allocation.  count must be in [1, 8] (the
 * buffer holds 8 tiles, 16 KiB); larger counts return T2S_EINVAL.  Synchronous.
 * Every call on a device shares that device's buffer: calls that overlap on one GPU
 * (from several host threads) race.  Errors: T2S_EINVAL, T2S_EHIP. */
int t2s_unet_mfma_probe_static(const float* A, const float* B, float* D, int count);

#ifdef __cplusplus
}
#endif

#endif /* T2S_H */
