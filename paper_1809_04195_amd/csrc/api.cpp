// api.cpp -- C ABI of the T2-Shuffling slice solver: validation, plan tables,
// workspace layout and the ADMM / CG launch schedule.  See include/t2s.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/t2s.h"
#include "kernels.hpp"

using t2s::ClassArgs;
using t2s::PartialSrc;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(T2S_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct ClassPlan {
    int ny = 0, nz = 0, C = 0, S = 0, P = 0, gbase = 0;
    int M = 1;                              // coil-map sets (soft-SENSE)
    int nrw = 0, npb = 0, nllr = 0;
    std::vector<float> psi;                 // [K(K+1)/2][nz][ny] (host copy, documented layout)
    std::vector<float> psi_dev;             // pass-B order (see kernels.hpp)
    std::vector<int> row_ptr, ent_t, ent_p;
    std::vector<float> twy, twz;            // interleaved (re, im)
    size_t o_psi = 0, o_twy = 0, o_twz = 0, o_phi = 0, o_rowptr = 0, o_entt = 0, o_entp = 0;
    size_t o_sens = 0, o_ksp = 0, o_vec[7] = {}, o_tmp = 0, o_pa = 0, o_pb = 0, o_rr = 0, o_g0 = 0, o_b0n = 0, o_llr = 0,
           o_hist = 0, o_state = 0;
    std::vector<int> loaded;
    std::vector<int> outer_run, k_freeze, converged;
    int chunk = 0;      // slices per pass launch (0: all slices of the class in one launch)
    int nstreams = 1;   // streams the chunks are spread over
    int order = 0;      // workgroup order of passes A / C (T2S_ORDER_* flags)
    ClassArgs args{};
};

// Autotuned schedules, shared by every plan of the process, keyed by the shape of
// the class and the device architecture.
using SchedKey = std::tuple<int, int, int, int, int, std::string>;   // ny, nz, C, M K, slices, arch
struct Sched {
    int chunk, nstreams, order;
};
std::mutex g_sched_mu;
std::map<SchedKey, Sched> g_sched;

// Continuous batching: a queue of submitted slice ranges and the slot each slice of
// the one-class plan holds.
struct StreamItem {
    int count = 0, g0 = 0, next = 0;        // slices, global index of the first, next one to load
    const char* sens = nullptr;
    const char* ksp = nullptr;
    char* out = nullptr;
    t2s_slice_report* rep = nullptr;
};
struct StreamSlot {
    int item = -1;                          // queue entry of the slice held (-1: idle)
    int j = 0;                              // slice within the entry
    int k = 0;                              // outer iterations run since the load
};
struct StreamState {
    bool open = false, fresh = false;
    int cls = 0, mode = 0;
    t2s_unet* net = nullptr;
    int net_batch = 0;
    std::vector<StreamItem> items;
    size_t head = 0;                        // first entry with slices left to load
    std::vector<StreamSlot> slots;
    long done = 0;
    int64_t loaded = 0, slice_outer = 0;
    double* hpin = nullptr;                 // pinned host copies of the history and ||b0||^2 partials
    size_t hpin_len = 0;
};

}  // namespace

namespace t2s {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace t2s

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;             // free events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> open[T2S_KERNEL_COUNT];
    int launches[T2S_KERNEL_COUNT] = {};
    double ms[T2S_KERNEL_COUNT] = {};
};

struct t2s_plan {
    Profiler prof;
    std::vector<hipStream_t> aux;        // library-owned streams for chunked passes (default priority)
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    hipStream_t cap = nullptr;           // capture stream of the outer-iteration graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::string gkey;                    // schedule the graph was captured with
    std::string arch;
    t2s_params prm{};
    std::vector<float> phi;
    std::vector<ClassPlan> cls;
    size_t ws_bytes = 0;
    char* ws = nullptr;
    bool bound = false;
    int hist_len = 0;
    bool reconstructed = false;
    hipStream_t last_stream = nullptr;
    StreamState stream;
};

namespace {

bool finite_f(float v) { return std::isfinite(v); }

int check_class_index(const t2s_plan* plan, int cls, int first, int count) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    if (cls < 0 || cls >= (int)plan->cls.size()) return fail(T2S_EINVAL, "class index out of range");
    const ClassPlan& c = plan->cls[cls];
    if (count < 1 || first < 0 || first + count > c.S) return fail(T2S_EINVAL, "slice range out of bounds");
    return 0;
}

void roots(int L, std::vector<float>& out) {
    out.resize(2 * L);
    for (int m = 0; m < L; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)L;
        out[2 * m] = (float)std::cos(a);
        out[2 * m + 1] = (float)std::sin(a);
    }
}

// coefficient images per slice: K per coil-map set
size_t vec_bytes(const ClassPlan& c, int K) { return (size_t)c.S * c.M * K * c.ny * c.nz * 8; }
size_t slice_images(const ClassPlan& c, int K) { return (size_t)c.M * K * c.ny * c.nz; }

void fill_args(t2s_plan* plan, ClassPlan& c) {
    char* b = plan->ws;
    ClassArgs& a = c.args;
    a.ny = c.ny;
    a.nz = c.nz;
    a.C = c.C;
    a.M = c.M;
    a.K = plan->prm.K;
    a.T = plan->prm.T;
    a.P = c.P;
    a.nrw = c.nrw;
    a.npb = c.npb;
    a.nllr = c.nllr;
    a.hist_len = plan->hist_len;
    a.block = plan->prm.block;
    a.order = c.order;
    a.tau = plan->prm.lambda / plan->prm.rho;
    a.rho = plan->prm.rho;
    a.seed = plan->prm.seed;
    a.psi = (const float*)(b + c.o_psi);
    a.twy = (const float2*)(b + c.o_twy);
    a.twz = (const float2*)(b + c.o_twz);
    a.phi = (const float*)(b + c.o_phi);
    a.row_ptr = (const int*)(b + c.o_rowptr);
    a.ent_t = (const int*)(b + c.o_entt);
    a.ent_p = (const int*)(b + c.o_entp);
    a.sens = (float2*)(b + c.o_sens);
    a.ksp = (float2*)(b + c.o_ksp);
    a.b0 = (float2*)(b + c.o_vec[0]);
    a.x = (float2*)(b + c.o_vec[1]);
    a.r = (float2*)(b + c.o_vec[2]);
    a.p = (float2*)(b + c.o_vec[3]);
    a.w = (float2*)(b + c.o_vec[4]);
    a.z = (float2*)(b + c.o_vec[5]);
    a.u = (float2*)(b + c.o_vec[6]);
    a.tmp = (float2*)(b + c.o_tmp);
    a.pa = (double*)(b + c.o_pa);
    a.pb = (double*)(b + c.o_pb);
    a.rr = (double*)(b + c.o_rr);
    a.g0 = (double*)(b + c.o_g0);
    a.b0n = (double*)(b + c.o_b0n);
    a.llr = (double*)(b + c.o_llr);
    a.hist = (double*)(b + c.o_hist);
    a.state = (int*)(b + c.o_state);
}

hipEvent_t prof_event(Profiler& p) {
    if (!p.pool.empty()) {
        hipEvent_t e = p.pool.back();
        p.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Collect finished intervals of one kernel family into the totals.
int prof_drain(Profiler& p, int kind) {
    for (auto& pr : p.open[kind]) {
        HIP_TRY(hipEventSynchronize(pr.second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
        p.ms[kind] += ms;
        p.launches[kind] += 1;
        p.pool.push_back(pr.first);
        p.pool.push_back(pr.second);
    }
    p.open[kind].clear();
    return 0;
}

struct TimedLaunch {
    Profiler* p;
    int kind;
    hipStream_t st;
    hipEvent_t e0 = nullptr;
    TimedLaunch(Profiler* p_, int k, hipStream_t s) : p(p_), kind(k), st(s) {
        if (p && p->on) {
            if (p->open[kind].size() > 4096) prof_drain(*p, kind);
            e0 = prof_event(*p);
            if (e0) (void)hipEventRecord(e0, st);
        }
    }
    ~TimedLaunch() {
        if (e0) {
            hipEvent_t e1 = prof_event(*p);
            if (e1) {
                (void)hipEventRecord(e1, st);
                p->open[kind].push_back({e0, e1});
            }
        }
    }
};

thread_local Profiler* g_prof = nullptr;   // profiler of the plan being driven

#define TIMED(kind) TimedLaunch timed_##__LINE__(g_prof, kind, st)
#define TIMED_ON(kind, stream) TimedLaunch timed_on_##__LINE__(g_prof, kind, stream)

PartialSrc rr_src(const ClassArgs& a, int buf) { return PartialSrc{a.rr + (size_t)buf * a.nrw, 2 * a.nrw, a.nrw}; }
PartialSrc g0_src(const ClassArgs& a) { return PartialSrc{a.g0, a.nllr, a.nllr}; }

#define HIP_CHECK_LAUNCH(expr)                                                                 \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(T2S_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_));     \
    } while (0)

// w = (A^H A + rho_add) applied to src (slices [s0, s0+count), src indexed from src_s0)
int run_normal(const ClassArgs& a, int s0, int count, const float2* src, int src_s0, float rho_add, float2* out,
               int out_s0, hipStream_t st) {
    {
        TIMED(T2S_KERNEL_PASS_A);
        HIP_CHECK_LAUNCH(t2s::launch_passA(a, s0, count, src, src_s0, 1, PartialSrc{nullptr, 0, 0},
                                           PartialSrc{nullptr, 0, 0}, 0, st));
    }
    {
        TIMED(T2S_KERNEL_PASS_B);
        HIP_CHECK_LAUNCH(t2s::launch_passB(a, s0, count, 0, 0, st));
    }
    {
        TIMED(T2S_KERNEL_PASS_C);
        HIP_CHECK_LAUNCH(t2s::launch_passC(a, s0, count, 0, rho_add, out, out_s0, st));
    }
    return 0;
}

// CG step i for slices [s0, s0 + count) as passes A, B, C with the vector update
// fused into pass C: in one launch each, or in chunks of `chunk` slices spread
// round-robin over `ns` library streams, so that the pass intermediate of the slices
// in flight can stay in the on-package cache between the passes.  The caller's
// stream waits for every chunk before it continues.
// <r, r> partials: g0 at the start of the outer iteration (LLR kernel), then
// rr[(i + 1) % 2] after step i.  With `update` false (schedule timing) pass C writes
// M p to w instead, and x, r and the partial sums stay untouched.
int run_passes(t2s_plan* plan, const ClassArgs& a, int s0, int count, int i, int chunk, int ns, bool update,
               hipStream_t st) {
    const PartialSrc none{nullptr, 0, 0};
    const PartialSrc gcA = (i == 0) ? none : rr_src(a, i % 2);
    const PartialSrc gpA = (i == 0) ? none : (i == 1 ? g0_src(a) : rr_src(a, (i - 1) % 2));
    const PartialSrc gcC = (i == 0) ? g0_src(a) : rr_src(a, i % 2);
    if (chunk <= 0 || chunk >= count) {
        chunk = count;
        ns = 1;
    }
    const int nchunks = (count + chunk - 1) / chunk;
    ns = std::max(1, std::min(ns, std::min(nchunks, (int)plan->aux.size())));
    if (ns > 1) {
        HIP_TRY(hipEventRecord(plan->ev_fork, st));
        for (int j = 0; j < ns; ++j) HIP_TRY(hipStreamWaitEvent(plan->aux[j], plan->ev_fork, 0));
    }
    for (int q = 0; q < nchunks; ++q) {
        hipStream_t sq = ns > 1 ? plan->aux[q % ns] : st;
        const int c0 = s0 + q * chunk;
        const int cn = std::min(chunk, s0 + count - c0);
        {
            TIMED_ON(T2S_KERNEL_PASS_A, sq);
            HIP_CHECK_LAUNCH(t2s::launch_passA(a, c0, cn, a.r, 0, i == 0 ? 1 : 0, gcA, gpA, update, sq));
        }
        {
            TIMED_ON(T2S_KERNEL_PASS_B, sq);
            HIP_CHECK_LAUNCH(t2s::launch_passB(a, c0, cn, 0, update, sq));
        }
        {
            TIMED_ON(T2S_KERNEL_PASS_C, sq);
            if (update)
                HIP_CHECK_LAUNCH(t2s::launch_passC_cg(a, c0, cn, gcC, (i + 1) % 2, sq));
            else
                HIP_CHECK_LAUNCH(t2s::launch_passC(a, c0, cn, 0, a.rho, a.w, 0, sq));
        }
    }
    if (ns > 1) {
        for (int j = 0; j < ns; ++j) {
            HIP_TRY(hipEventRecord(plan->ev_join[j], plan->aux[j]));
            HIP_TRY(hipStreamWaitEvent(st, plan->ev_join[j], 0));
        }
    }
    return 0;
}

// one ADMM outer iteration for slices [s0, s0 + count) (the outer index lives in the
// device-side slice state, so the same launch sequence serves every iteration)
int run_outer(t2s_plan* plan, const ClassArgs& a, int s0, int count, int chunk, int ns, hipStream_t st) {
    const int ncg = plan->prm.n_cg;
    for (int i = 0; i < ncg; ++i)
        if (int e = run_passes(plan, a, s0, count, i, chunk, ns, true, st)) return e;
    {
        TIMED(T2S_KERNEL_LLR);
        HIP_CHECK_LAUNCH(t2s::launch_llr(a, s0, count, t2s::kLlrAdmm, 0, nullptr, nullptr, a.tau, 0, 0, 0.f, st));
    }
    HIP_CHECK_LAUNCH(t2s::launch_llr_finalize(a, s0, count, st));
    return 0;
}

// one outer iteration of every class of the plan
int run_outer_all(t2s_plan* plan, int mode, hipStream_t st) {
    for (ClassPlan& c : plan->cls) {
        if (mode == T2S_PER_SLICE) {
            for (int s = 0; s < c.S; ++s)
                if (int e = run_outer(plan, c.args, s, 1, 0, 1, st)) return e;
        } else {
            if (int e = run_outer(plan, c.args, 0, c.S, c.chunk, c.nstreams, st)) return e;
        }
    }
    return 0;
}

std::string sched_signature(const t2s_plan* plan, int mode) {
    std::string k = std::to_string(mode);
    for (const ClassPlan& c : plan->cls)
        k += "/" + std::to_string(c.chunk) + "x" + std::to_string(c.nstreams) + "o" + std::to_string(c.order);
    return k;
}

int ensure_streams(t2s_plan* plan, int n) {
    while ((int)plan->aux.size() < n) {
        hipStream_t s = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        plan->aux.push_back(s);
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        plan->ev_join.push_back(e);
    }
    if (!plan->ev_fork) HIP_TRY(hipEventCreateWithFlags(&plan->ev_fork, hipEventDisableTiming));
    if (!plan->cap) HIP_TRY(hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking));
    return 0;
}

void drop_graph(t2s_plan* plan) {
    if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    plan->gexec = nullptr;
    plan->graph = nullptr;
    plan->gkey.clear();
}

// Capture one outer iteration of every class into a graph (once per schedule).
int ensure_graph(t2s_plan* plan, int mode) {
    const std::string key = sched_signature(plan, mode);
    if (plan->gexec && plan->gkey == key) return 0;
    drop_graph(plan);
    Profiler* saved = g_prof;
    g_prof = nullptr;   // no timing events inside a captured graph
    HIP_TRY(hipStreamBeginCapture(plan->cap, hipStreamCaptureModeRelaxed));
    int e = run_outer_all(plan, mode == T2S_BATCHED_GRAPH ? T2S_BATCHED : mode, plan->cap);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(plan->cap, &g);
    g_prof = saved;
    if (e) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    if (ce != hipSuccess) return fail(T2S_EHIP, std::string("graph capture: ") + hipGetErrorString(ce));
    plan->graph = g;
    HIP_TRY(hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0));
    plan->gkey = key;
    return 0;
}

// relative primal / dual residuals from the per-outer sums (alpha - z, z - z_prev,
// alpha, z, u, r squared norms): both relative to max(||alpha||, ||z||)
// Relative ADMM residuals of one outer iteration from its summed squares (h[0] =
// ||alpha - z||^2, h[1] = ||z - z_prev||^2, h[2] = ||alpha||^2, h[3] = ||z||^2),
// scaled by max(||alpha||, ||z||, kResidualScaleFloor ||b0||)
constexpr double kResidualScaleFloor = 0.01;
void residuals_from_hist(const double* h, double b0_norm, double* rp, double* rd) {
    const double na = std::sqrt(h[2]), nzz = std::sqrt(h[3]);
    const double den = std::max(std::max(na, nzz), kResidualScaleFloor * b0_norm);
    *rp = den > 0 ? std::sqrt(h[0]) / den : 0.0;
    *rd = den > 0 ? std::sqrt(h[1]) / den : 0.0;
}

// Stop / freeze decision of slice s of class c after its k-th outer iteration (k >= 1;
// hs: the slice's history rows, b0_norm: ||b0||): stop when max(r_p, r_d) <= tol
// (converged); otherwise, once k - 1 >= freeze_window, freeze the shift at draw k - 1
// if the residual fell by less than freeze_stall over the last freeze_window outer
// iterations.  A stopped slice is marked inactive on the device.
int tol_decide(const t2s_params& prm, ClassPlan& c, int s, int k, const double* hs, double b0_norm, hipStream_t st,
               bool* stop) {
    double rp, rd;
    residuals_from_hist(hs + (size_t)(k - 1) * 8, b0_norm, &rp, &rd);
    const double r = std::max(rp, rd);
    *stop = false;
    if (r <= prm.tol) {
        *stop = true;
        c.converged[s] = 1;
    } else if (c.k_freeze[s] < 0 && k - 1 >= prm.freeze_window) {
        double rpo, rdo;
        residuals_from_hist(hs + (size_t)(k - 1 - prm.freeze_window) * 8, b0_norm, &rpo, &rdo);
        if (r > (1.0 - prm.freeze_stall) * std::max(rpo, rdo)) {
            c.k_freeze[s] = k - 1;
            HIP_CHECK_LAUNCH(t2s::launch_set_state(c.args, s, 1, 1, k - 1, -1, st));
        }
    }
    if (*stop) HIP_CHECK_LAUNCH(t2s::launch_set_state(c.args, s, 1, 0, c.k_freeze[s], -1, st));
    return 0;
}

// Copy the coil maps and samples of slices [first, first + count) of class c in, mark
// them active with outer counter 0 and global indices gfirst.., and form b0 = A^H y
// (projection, inverse column and row transforms, coil combine) and the initial
// x = z = u = 0, r = b0 (with their partial sums).
// Copy the coil maps and samples of `count` slices into slices first.. of class c and
// mark them active with outer counter 0 and global indices gfirst, gfirst + 1, ...
int load_copy(ClassPlan& c, int first, int count, const void* sens, const void* ksp, hipMemcpyKind kind, int gfirst,
              hipStream_t st) {
    const size_t N = (size_t)c.ny * c.nz;
    const ClassArgs& a = c.args;
    const size_t ns = (size_t)count * c.C * c.M * N * 8, nk = (size_t)count * c.C * c.P * 8;
    HIP_TRY(hipMemcpyAsync(a.sens + (size_t)first * c.C * c.M * N, sens, ns, kind, st));
    if (nk) HIP_TRY(hipMemcpyAsync(a.ksp + (size_t)first * c.C * c.P, ksp, nk, kind, st));
    HIP_CHECK_LAUNCH(t2s::launch_set_state(a, first, count, 1, -1, 0, st, gfirst));
    return 0;
}

// b0 = A^H y of slices [first, first + count) (projection, inverse column and row
// transforms, coil combine) and the initial x = z = u = 0, r = b0 with their partial sums
int load_compute(ClassPlan& c, int first, int count, hipStream_t st) {
    const ClassArgs& a = c.args;
    TIMED(T2S_KERNEL_LOAD);
    HIP_CHECK_LAUNCH(t2s::launch_project(a, first, count, st));
    HIP_CHECK_LAUNCH(t2s::launch_passB(a, first, count, 1, 0, st));
    HIP_CHECK_LAUNCH(t2s::launch_passC(a, first, count, 1, 0.0f, a.b0, 0, st));
    HIP_CHECK_LAUNCH(t2s::launch_init(a, first, count, nullptr, 0, st));
    return 0;
}

int load_range(ClassPlan& c, int first, int count, const void* sens, const void* ksp, hipMemcpyKind kind, int gfirst,
               hipStream_t st) {
    if (int e = load_copy(c, first, count, sens, ksp, kind, gfirst, st)) return e;
    return load_compute(c, first, count, st);
}

// Load queued slices into the idle slots of the streaming class: each run of
// consecutive idle slots takes the next queued slices in queue order (across queue
// entries; one copy per slice, or one per stretch taken from one entry), then one
// set of load launches over the run, the network warm start when one is set, and the
// warm start's normal operator.
int stream_refill(t2s_plan* plan, StreamState& q, ClassPlan& c, hipStream_t st) {
    const size_t N = (size_t)c.ny * c.nz;
    const size_t n = slice_images(c, plan->prm.K);
    const ClassArgs& a = c.args;
    int s = 0;
    while (s < c.S) {
        if (q.slots[s].item >= 0) {
            ++s;
            continue;
        }
        int r = 0;
        while (s + r < c.S && q.slots[s + r].item < 0) {
            while (q.head < q.items.size() && q.items[q.head].next >= q.items[q.head].count) ++q.head;
            if (q.head == q.items.size()) break;
            StreamItem& it = q.items[q.head];
            // as many consecutive slices of this entry as there are idle slots in a row
            int m = 0;
            while (s + r + m < c.S && q.slots[s + r + m].item < 0 && it.next + m < it.count) ++m;
            const int j0 = it.next;
            it.next += m;
            if (int e = load_copy(c, s + r, m, it.sens + (size_t)j0 * c.C * c.M * N * 8,
                                  it.ksp + (size_t)j0 * c.C * c.P * 8, hipMemcpyDeviceToDevice, it.g0 + j0, st))
                return e;
            for (int i = 0; i < m; ++i) {
                q.slots[s + r + i] = StreamSlot{(int)q.head, j0 + i, 0};
                c.outer_run[s + r + i] = 0;
                c.k_freeze[s + r + i] = -1;
                c.converged[s + r + i] = 0;
            }
            r += m;
        }
        if (r == 0) break;
        q.loaded += r;
        if (int e = load_compute(c, s, r, st)) return e;
        if (q.net) {
            // alpha0 = net(b0) straight into x, then r = b0 - A^H A alpha0 (t2s_set_initial)
            for (int i = 0; i < r; i += q.net_batch) {
                const int b = std::min(q.net_batch, r - i);
                if (int e = t2s_unet_forward(q.net, a.b0 + (size_t)(s + i) * n, a.x + (size_t)(s + i) * n, b, st))
                    return e;
            }
            if (int e = run_normal(a, s, r, a.x, 0, 0.0f, a.w, 0, st)) return e;
            HIP_CHECK_LAUNCH(t2s::launch_init(a, s, r, a.x + (size_t)s * n, 1, st));
        }
        s += r;
    }
    return 0;
}

// Slot s finished its slice: result and report out, slot idle.
int stream_complete(t2s_plan* plan, StreamState& q, ClassPlan& c, int s, const double* hist, double b0_norm,
                    hipStream_t st) {
    StreamSlot& sl = q.slots[s];
    StreamItem& it = q.items[sl.item];
    const size_t n = slice_images(c, plan->prm.K);
    HIP_TRY(hipMemcpyAsync(it.out + (size_t)sl.j * n * 8, c.args.x + (size_t)s * n, n * 8, hipMemcpyDeviceToDevice,
                           st));
    if (it.rep) {
        t2s_slice_report& r = it.rep[sl.j];
        r.outer_iterations = sl.k;
        r.k_freeze = c.k_freeze[s];
        r.converged = c.converged[s];
        r.r_primal = r.r_dual = std::numeric_limits<double>::quiet_NaN();
        if (sl.k > 0 && sl.k <= plan->hist_len)
            residuals_from_hist(hist + (size_t)(sl.k - 1) * 8, b0_norm, &r.r_primal, &r.r_dual);
    }
    sl.item = -1;
    ++q.done;
    return 0;
}

}  // namespace

extern "C" {

int t2s_version(void) { return 104; }

const char* t2s_last_error(void) { return g_err.c_str(); }

int t2s_block_shift(uint64_t seed, int g, int k, int b, int* sy, int* sz) {
    if (!sy || !sz) return fail(T2S_EINVAL, "null output");
    if (b < 1 || g < 0 || k < 0) return fail(T2S_EINVAL, "bad block shift arguments");
    auto sm = [](uint64_t x) {
        uint64_t z = x + 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    const uint64_t h = sm(sm(sm(seed) ^ (uint64_t)g) ^ (uint64_t)k);
    *sy = (int)((h & 0xFFFFFFFFull) % (uint64_t)b);
    *sz = (int)((h >> 32) % (uint64_t)b);
    return 0;
}

int t2s_plan_create(const t2s_params* p, const t2s_class* classes, int n_classes, t2s_plan** out) {
    if (!out) return fail(T2S_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(T2S_EINVAL, "params is NULL");
    if (!p->phi) return fail(T2S_EINVAL, "phi is NULL");
    if (!classes || n_classes < 1) return fail(T2S_EINVAL, "no shape classes");
    if (p->T < 1) return fail(T2S_ESHAPE, "T must be >= 1");
    if (p->K < 1 || p->K > T2S_MAX_K) return fail(T2S_ESHAPE, "K must be in [1, 8]");
    if (p->K > p->T) return fail(T2S_ESHAPE, "K must not exceed T");
    if (!finite_f(p->lambda) || !finite_f(p->rho) || !finite_f(p->tol) || !finite_f(p->freeze_stall))
        return fail(T2S_ENONFINITE, "non-finite solver parameter");
    if (p->lambda < 0) return fail(T2S_EINVAL, "lambda must be >= 0");
    if (!(p->rho > 0)) return fail(T2S_EINVAL, "rho must be > 0");
    if (p->block != 4 && p->block != 8 && p->block != 12 && p->block != 16)
        return fail(T2S_EINVAL, "block must be 4, 8, 12 or 16");
    if (p->n_outer < 1 || p->n_cg < 1) return fail(T2S_EINVAL, "n_outer and n_cg must be >= 1");
    if (p->tol < 0) return fail(T2S_EINVAL, "tol must be >= 0");
    if (p->tol > 0 && (p->freeze_window < 1 || p->check_every < 1 || p->freeze_stall < 0 || p->freeze_stall >= 1))
        return fail(T2S_EINVAL, "tolerance mode needs freeze_window >= 1, check_every >= 1, 0 <= freeze_stall < 1");
    const int T = p->T, K = p->K;
    for (int i = 0; i < T * K; ++i)
        if (!finite_f(p->phi[i])) return fail(T2S_ENONFINITE, "phi has NaN/Inf");
    for (int ci = 0; ci < n_classes; ++ci) {
        const t2s_class& c = classes[ci];
        if (!c.masks) return fail(T2S_EINVAL, "class " + std::to_string(ci) + ": masks is NULL");
        if (c.ncoils < 1 || c.nslices < 1) return fail(T2S_ESHAPE, "class " + std::to_string(ci) + ": ncoils and nslices must be >= 1");
        if (c.nmaps < 0 || c.nmaps > 2) return fail(T2S_ESHAPE, "class " + std::to_string(ci) + ": nmaps must be 0, 1 or 2");
        if (c.ny < 16 || c.nz < 16 || c.ny % 16 || c.ny < p->block || c.nz < p->block)
            return fail(T2S_ESHAPE, "class " + std::to_string(ci) +
                                        ": ny must be a multiple of 16, ny and nz at least the block size");
        if (!t2s::fft_col_supported(c.ny) || !t2s::fft_row_supported(c.nz))
            return fail(T2S_EUNSUPPORTED, "class " + std::to_string(ci) + ": no FFT plan for this grid length");
        const size_t tot = (size_t)T * c.ny * c.nz;
        for (size_t i = 0; i < tot; ++i)
            if (c.masks[i] > 1) return fail(T2S_EINVAL, "class " + std::to_string(ci) + ": mask values must be 0 or 1");
    }

    t2s_plan* plan = new t2s_plan();
    plan->prm = *p;
    plan->phi.assign(p->phi, p->phi + T * K);
    plan->prm.phi = nullptr;
    plan->hist_len = p->n_outer + 1;
    const int kk2 = K * (K + 1) / 2;
    int gbase = 0;
    for (int ci = 0; ci < n_classes; ++ci) {
        const t2s_class& src = classes[ci];
        ClassPlan c;
        c.ny = src.ny;
        c.nz = src.nz;
        c.C = src.ncoils;
        c.M = src.nmaps <= 1 ? 1 : src.nmaps;
        c.S = src.nslices;
        c.gbase = gbase;
        gbase += src.nslices;
        c.order = t2s::default_order(c.ny, c.nz, K);
        const int ny = c.ny, nz = c.nz, N = ny * nz;
        // space-time kernel, FP64, upper triangle, uncentred + transposed, / N
        std::vector<double> acc((size_t)kk2 * N, 0.0);
        std::vector<int> cnt(N + 1, 0);
        int P = 0;
        for (int t = 0; t < T; ++t)
            for (int y = 0; y < ny; ++y)
                for (int z = 0; z < nz; ++z) {
                    if (!src.masks[((size_t)t * ny + y) * nz + z]) continue;
                    const int q = ((z + nz / 2) % nz) * ny + (y + ny / 2) % ny;
                    int tri = 0;
                    for (int k = 0; k < K; ++k)
                        for (int l = k; l < K; ++l, ++tri)
                            acc[(size_t)tri * N + q] += (double)plan->phi[t * K + k] * (double)plan->phi[t * K + l];
                    cnt[q + 1]++;
                    ++P;
                }
        c.P = P;
        c.psi.resize((size_t)kk2 * N);
        for (size_t i = 0; i < c.psi.size(); ++i) c.psi[i] = (float)(acc[i] / (double)N);
        {
            int R1 = 0, R2 = 0;
            t2s::reg_plan(ny, &R1, &R2);
            const int KP = (kk2 + 3) / 4 * 4;
            c.psi_dev.assign((size_t)nz * ny * KP, 0.f);
            for (int zq = 0; zq < nz; ++zq)
                for (int t = 0; t < R1; ++t)
                    for (int k2 = 0; k2 < R2; ++k2) {
                        const int yq = t + R1 * k2;
                        for (int tri = 0; tri < kk2; ++tri)
                            c.psi_dev[((((size_t)zq * R2 + k2) * (KP / 4) + tri / 4) * R1 + t) * 4 + tri % 4] =
                                c.psi[(size_t)tri * N + (size_t)zq * ny + yq];
                    }
        }
        c.row_ptr.assign(N + 1, 0);
        for (int q = 0; q < N; ++q) c.row_ptr[q + 1] = c.row_ptr[q] + cnt[q + 1];
        c.ent_t.assign(std::max(P, 1), 0);
        c.ent_p.assign(std::max(P, 1), 0);
        std::vector<int> fillp(c.row_ptr.begin(), c.row_ptr.end() - 1);
        int pidx = 0;
        for (int t = 0; t < T; ++t)
            for (int y = 0; y < ny; ++y)
                for (int z = 0; z < nz; ++z) {
                    if (!src.masks[((size_t)t * ny + y) * nz + z]) continue;
                    const int q = ((z + nz / 2) % nz) * ny + (y + ny / 2) % ny;
                    const int e = fillp[q]++;
                    c.ent_t[e] = t;
                    c.ent_p[e] = pidx++;
                }
        roots(ny, c.twy);
        roots(nz, c.twz);
        c.nrw = (ny / t2s::kRowTile) * K;
        const int wb = t2s::passB_columns(ny, K);
        c.npb = ((nz + wb - 1) / wb) * c.C;
        c.nllr = c.M * t2s::llr_workgroups(ny, nz, p->block);   // one run per map set
        c.loaded.assign(c.S, 0);
        c.outer_run.assign(c.S, 0);
        c.k_freeze.assign(c.S, -1);
        c.converged.assign(c.S, 0);
        plan->cls.push_back(std::move(c));
    }
    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    for (ClassPlan& c : plan->cls) {
        const size_t N = (size_t)c.ny * c.nz;
        c.o_psi = take(c.psi_dev.size() * 4);
        c.o_twy = take((size_t)c.ny * 8);
        c.o_twz = take((size_t)c.nz * 8);
        c.o_phi = take((size_t)T * K * 4);
        c.o_rowptr = take((N + 1) * 4);
        c.o_entt = take(c.ent_t.size() * 4);
        c.o_entp = take(c.ent_p.size() * 4);
        c.o_sens = take((size_t)c.S * c.C * c.M * N * 8);
        c.o_ksp = take((size_t)c.S * c.C * std::max(c.P, 1) * 8);
        for (int v = 0; v < 7; ++v) c.o_vec[v] = take(vec_bytes(c, K));
        c.o_tmp = take((size_t)c.S * c.C * K * ((size_t)c.ny * ((c.nz + 15) & ~15)) * 8);   // 16-column tiles
        c.o_pa = take((size_t)c.S * c.nrw * 8);
        c.o_pb = take((size_t)c.S * c.npb * 8);
        c.o_rr = take((size_t)c.S * 2 * c.nrw * 8);
        c.o_g0 = take((size_t)c.S * c.nllr * 8);
        c.o_b0n = take((size_t)c.S * c.nllr * 8);
        c.o_llr = take((size_t)c.S * c.nllr * 8 * 8);
        c.o_hist = take((size_t)c.S * plan->hist_len * 8 * 8);
        c.o_state = take((size_t)c.S * 4 * 4);
    }
    plan->ws_bytes = off;
    *out = plan;
    return 0;
}

int t2s_plan_destroy(t2s_plan* plan) {
    if (plan) {
        for (int k = 0; k < T2S_KERNEL_COUNT; ++k)
            for (auto& pr : plan->prof.open[k]) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
        for (hipEvent_t e : plan->prof.pool) (void)hipEventDestroy(e);
        if (g_prof == &plan->prof) g_prof = nullptr;
        drop_graph(plan);
        for (hipStream_t x : plan->aux) (void)hipStreamDestroy(x);
        for (hipEvent_t e : plan->ev_join) (void)hipEventDestroy(e);
        if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
        if (plan->cap) (void)hipStreamDestroy(plan->cap);
        if (plan->stream.hpin) (void)hipHostFree(plan->stream.hpin);
    }
    delete plan;
    return 0;
}

int t2s_profile_enable(t2s_plan* plan, int enable) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    Profiler& p = plan->prof;
    for (int k = 0; k < T2S_KERNEL_COUNT; ++k) {
        if (int e = prof_drain(p, k)) return e;
        p.launches[k] = 0;
        p.ms[k] = 0.0;
    }
    p.on = enable != 0;
    if (plan->bound) HIP_CHECK_LAUNCH(t2s::launch_profile_mark(plan->last_stream));
    return 0;
}

int t2s_profile_read(t2s_plan* plan, int kernel, int* launches, double* total_ms) {
    if (!plan || !launches || !total_ms) return fail(T2S_EINVAL, "NULL argument");
    if (kernel < 0 || kernel >= T2S_KERNEL_COUNT) return fail(T2S_EINVAL, "bad kernel id");
    if (int e = prof_drain(plan->prof, kernel)) return e;
    *launches = plan->prof.launches[kernel];
    *total_ms = plan->prof.ms[kernel];
    return 0;
}

int t2s_plan_workspace_bytes(const t2s_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return fail(T2S_EINVAL, "NULL argument");
    *bytes = plan->ws_bytes;
    return 0;
}

int t2s_plan_bind_workspace(t2s_plan* plan, void* dev, size_t bytes, void* stream) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    if (!dev) return fail(T2S_ENOMEM, "workspace pointer is NULL");
    if (bytes < plan->ws_bytes)
        return fail(T2S_ENOMEM, "workspace too small: need " + std::to_string(plan->ws_bytes) + " bytes");
    if ((uintptr_t)dev % kAlign) return fail(T2S_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    int dev_id = 0, max_lds = 0;
    HIP_TRY(hipGetDevice(&dev_id));
    HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_id));
    for (const ClassPlan& c : plan->cls) {
        const size_t need = std::max(t2s::lds_bytes_passA(c.nz), t2s::lds_bytes_passB(c.ny, plan->prm.K)) + 64;
        if (need > (size_t)max_lds)
            return fail(T2S_EUNSUPPORTED, "grid needs " + std::to_string(need) + " bytes of LDS per workgroup, device has " +
                                              std::to_string(max_lds));
    }
    plan->ws = (char*)dev;
    drop_graph(plan);   // kernel arguments of a captured graph point into the old workspace
    for (ClassPlan& c : plan->cls) {
        fill_args(plan, c);
        char* b = plan->ws;
        HIP_TRY(hipMemcpyAsync(b + c.o_psi, c.psi_dev.data(), c.psi_dev.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(b + c.o_twy, c.twy.data(), c.twy.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(b + c.o_twz, c.twz.data(), c.twz.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(b + c.o_phi, plan->phi.data(), plan->phi.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(b + c.o_rowptr, c.row_ptr.data(), c.row_ptr.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(b + c.o_entt, c.ent_t.data(), c.ent_t.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(b + c.o_entp, c.ent_p.data(), c.ent_p.size() * 4, hipMemcpyHostToDevice, st));
        HIP_CHECK_LAUNCH(t2s::launch_set_state(c.args, 0, c.S, 0, -1, 0, st, c.gbase));
        std::fill(c.loaded.begin(), c.loaded.end(), 0);
    }
    HIP_TRY(hipStreamSynchronize(st));   // host tables are pageable: finish before returning
    plan->bound = true;
    return 0;
}

int t2s_load_slices(t2s_plan* plan, int cls, int first, int count, const void* sens, const void* ksp, int mem,
                    void* stream) {
    if (int e = check_class_index(plan, cls, first, count)) return e;
    if (!sens || !ksp) return fail(T2S_EINVAL, "sens or ksp is NULL");
    if (mem != T2S_HOST && mem != T2S_DEVICE) return fail(T2S_EINVAL, "mem must be T2S_HOST or T2S_DEVICE");
    if (!plan->bound) return fail(T2S_ESTATE, "workspace not bound");
    ClassPlan& c = plan->cls[cls];
    const size_t N = (size_t)c.ny * c.nz;
    const size_t ns = (size_t)count * c.C * c.M * N * 2, nk = (size_t)count * c.C * c.P * 2;
    if (mem == T2S_HOST) {
        const float* fs = (const float*)sens;
        const float* fk = (const float*)ksp;
        for (size_t i = 0; i < ns; ++i)
            if (!finite_f(fs[i])) return fail(T2S_ENONFINITE, "coil maps contain NaN/Inf");
        for (size_t i = 0; i < nk; ++i)
            if (!finite_f(fk[i])) return fail(T2S_ENONFINITE, "samples contain NaN/Inf");
    }
    hipStream_t st = (hipStream_t)stream;
    const hipMemcpyKind kind = mem == T2S_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    g_prof = &plan->prof;
    if (int e = load_range(c, first, count, sens, ksp, kind, c.gbase + first, st)) return e;
    if (mem == T2S_HOST) HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < count; ++i) c.loaded[first + i] = 1;
    plan->last_stream = st;
    return 0;
}

int t2s_set_initial(t2s_plan* plan, int cls, int first, int count, const void* alpha0, int mem, void* stream) {
    if (int e = check_class_index(plan, cls, first, count)) return e;
    if (!alpha0) return fail(T2S_EINVAL, "alpha0 is NULL");
    if (mem != T2S_HOST && mem != T2S_DEVICE) return fail(T2S_EINVAL, "mem must be T2S_HOST or T2S_DEVICE");
    ClassPlan& c = plan->cls[cls];
    for (int i = 0; i < count; ++i)
        if (!c.loaded[first + i]) return fail(T2S_ESTATE, "slice not loaded");
    const int K = plan->prm.K;
    const size_t n = (size_t)count * slice_images(c, K) * 2;
    if (mem == T2S_HOST) {
        const float* f = (const float*)alpha0;
        for (size_t i = 0; i < n; ++i)
            if (!finite_f(f[i])) return fail(T2S_ENONFINITE, "alpha0 contains NaN/Inf");
    }
    hipStream_t st = (hipStream_t)stream;
    g_prof = &plan->prof;
    const ClassArgs& a = c.args;
    float2* xs = a.x + (size_t)first * slice_images(c, K);
    HIP_TRY(hipMemcpyAsync(xs, alpha0, n * 4, mem == T2S_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
    HIP_CHECK_LAUNCH(t2s::launch_set_state(a, first, count, 1, -1, 0, st, c.gbase + first));
    // r = b0 + rho z - (A^H A + rho) alpha0 with z = alpha0, u = 0  =>  r = b0 - A^H A alpha0
    if (int e = run_normal(a, first, count, a.x, 0, 0.0f, a.w, 0, st)) return e;
    HIP_CHECK_LAUNCH(t2s::launch_init(a, first, count, xs, 1, st));
    if (mem == T2S_HOST) HIP_TRY(hipStreamSynchronize(st));
    return 0;
}

int t2s_reconstruct(t2s_plan* plan, int mode, void* stream) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    if (mode != T2S_BATCHED && mode != T2S_PER_SLICE && mode != T2S_BATCHED_GRAPH) return fail(T2S_EINVAL, "bad mode");
    if (!plan->bound) return fail(T2S_ESTATE, "workspace not bound");
    for (const ClassPlan& c : plan->cls)
        for (int s = 0; s < c.S; ++s)
            if (!c.loaded[s]) return fail(T2S_ESTATE, "not every slice is loaded");
    hipStream_t st = (hipStream_t)stream;
    plan->last_stream = st;
    g_prof = &plan->prof;
    const t2s_params& prm = plan->prm;
    const bool tolmode = prm.tol > 0;
    int maxns = 1;
    for (const ClassPlan& c : plan->cls) maxns = std::max(maxns, c.nstreams);
    if (int e = ensure_streams(plan, maxns)) return e;
    for (ClassPlan& c : plan->cls) {
        HIP_CHECK_LAUNCH(t2s::launch_set_state(c.args, 0, c.S, 1, -1, 0, st, c.gbase));
        std::fill(c.outer_run.begin(), c.outer_run.end(), 0);
        std::fill(c.k_freeze.begin(), c.k_freeze.end(), -1);
        std::fill(c.converged.begin(), c.converged.end(), 0);
    }
    // graphs carry no timing events: profiling falls back to eager launches
    const bool use_graph = mode == T2S_BATCHED_GRAPH && !plan->prof.on;
    if (use_graph) {
        if (int e = ensure_graph(plan, mode)) return e;
    }
    auto outer_once = [&]() -> int {
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(plan->gexec, st));
            return 0;
        }
        return run_outer_all(plan, mode == T2S_BATCHED_GRAPH ? T2S_BATCHED : mode, st);
    };
    int warn = 0;
    if (!tolmode) {
        for (int k = 0; k < prm.n_outer; ++k)
            if (int e = outer_once()) return e;
        for (ClassPlan& c : plan->cls) std::fill(c.outer_run.begin(), c.outer_run.end(), prm.n_outer);
    } else {
        // per-slice decisions every check_every outer iterations (see t2s.h)
        std::vector<std::vector<int>> active(plan->cls.size());
        for (size_t ci = 0; ci < plan->cls.size(); ++ci) active[ci].assign(plan->cls[ci].S, 1);
        std::vector<double> hbuf;
        // ||b0|| of every slice (partials written when the slice was loaded, on this
        // stream: wait for them before the synchronous read)
        HIP_TRY(hipStreamSynchronize(st));
        std::vector<std::vector<double>> b0norm(plan->cls.size());
        for (size_t ci = 0; ci < plan->cls.size(); ++ci) {
            const ClassPlan& c = plan->cls[ci];
            std::vector<double> part((size_t)c.S * c.nllr);
            HIP_TRY(hipMemcpy(part.data(), c.args.b0n, part.size() * 8, hipMemcpyDeviceToHost));
            b0norm[ci].assign(c.S, 0.0);
            for (int s = 0; s < c.S; ++s) {
                double acc = 0.0;
                for (int j = 0; j < c.nllr; ++j) acc += part[(size_t)s * c.nllr + j];
                b0norm[ci][s] = std::sqrt(acc);
            }
        }
        int k = 0;
        bool any = true;
        while (k < prm.n_outer && any) {
            const int kend = std::min(prm.n_outer, k + prm.check_every);
            for (; k < kend; ++k)
                if (int e = outer_once()) return e;
            HIP_TRY(hipStreamSynchronize(st));
            any = false;
            for (size_t ci = 0; ci < plan->cls.size(); ++ci) {
                ClassPlan& c = plan->cls[ci];
                hbuf.resize((size_t)c.S * plan->hist_len * 8);
                HIP_TRY(hipMemcpy(hbuf.data(), c.args.hist, hbuf.size() * 8, hipMemcpyDeviceToHost));
                for (int s = 0; s < c.S; ++s) {
                    if (!active[ci][s]) continue;
                    c.outer_run[s] = k;
                    bool stop = false;
                    if (int e = tol_decide(prm, c, s, k, &hbuf[(size_t)s * plan->hist_len * 8], b0norm[ci][s], st,
                                           &stop))
                        return e;
                    if (stop) {
                        active[ci][s] = 0;
                    } else {
                        any = true;
                    }
                }
            }
        }
        for (size_t ci = 0; ci < plan->cls.size(); ++ci)
            for (int s = 0; s < plan->cls[ci].S; ++s)
                if (active[ci][s]) warn = T2S_WNOTCONVERGED;
    }
    plan->reconstructed = true;
    if (warn) return fail(warn, "tolerance not met by n_outer for some slices");
    return 0;
}

int t2s_set_schedule(t2s_plan* plan, int cls, int chunk, int nstreams) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    if (cls < 0 || cls >= (int)plan->cls.size()) return fail(T2S_EINVAL, "class index out of range");
    if (chunk < 0 || nstreams < 1 || nstreams > 8) return fail(T2S_EINVAL, "chunk must be >= 0, nstreams in [1, 8]");
    plan->cls[cls].chunk = chunk;
    plan->cls[cls].nstreams = nstreams;
    return 0;
}

int t2s_set_order(t2s_plan* plan, int cls, int order) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    if (cls < 0 || cls >= (int)plan->cls.size()) return fail(T2S_EINVAL, "class index out of range");
    if (order & ~t2s::kOrderAll) return fail(T2S_EINVAL, "unknown schedule flags");
    plan->cls[cls].order = order;
    plan->cls[cls].args.order = order;
    return 0;
}

int t2s_set_slice_offset(t2s_plan* plan, int cls, int first_global) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    if (cls < 0 || cls >= (int)plan->cls.size()) return fail(T2S_EINVAL, "class index out of range");
    if (first_global < 0) return fail(T2S_EINVAL, "first_global must be >= 0");
    // kept on the host: the device-side global index of every slice is written from it
    // when slices are loaded and when a solve starts
    plan->cls[cls].gbase = first_global;
    return 0;
}

int t2s_get_order(const t2s_plan* plan, int cls, int* order) {
    if (!plan || !order) return fail(T2S_EINVAL, "NULL argument");
    if (cls < 0 || cls >= (int)plan->cls.size()) return fail(T2S_EINVAL, "class index out of range");
    *order = plan->cls[cls].order;
    return 0;
}

int t2s_get_schedule(const t2s_plan* plan, int cls, int* chunk, int* nstreams) {
    if (!plan || !chunk || !nstreams) return fail(T2S_EINVAL, "NULL argument");
    if (cls < 0 || cls >= (int)plan->cls.size()) return fail(T2S_EINVAL, "class index out of range");
    *chunk = plan->cls[cls].chunk;
    *nstreams = plan->cls[cls].nstreams;
    return 0;
}

int t2s_autotune(t2s_plan* plan, int reps, void* stream) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    if (!plan->bound) return fail(T2S_ESTATE, "workspace not bound");
    for (const ClassPlan& c : plan->cls)
        for (int s = 0; s < c.S; ++s)
            if (!c.loaded[s]) return fail(T2S_ESTATE, "autotuning runs on loaded slices");
    if (reps < 1) reps = 3;
    hipStream_t st = (hipStream_t)stream;
    Profiler* saved = g_prof;
    g_prof = nullptr;
    if (int e = ensure_streams(plan, 4)) return e;
    if (plan->arch.empty()) {
        int dev = 0;
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipGetDeviceProperties(&prop, dev));
        plan->arch = prop.gcnArchName;
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    for (ClassPlan& c : plan->cls) {
        const SchedKey key{c.ny, c.nz, c.C, c.M * plan->prm.K, c.S, plan->arch};
        {
            std::lock_guard<std::mutex> lk(g_sched_mu);
            auto it = g_sched.find(key);
            if (it != g_sched.end()) {
                c.chunk = it->second.chunk;
                c.nstreams = it->second.nstreams;
                c.order = c.args.order = it->second.order;
                continue;
            }
        }
        // candidates: everything in one launch, or chunks of 32..2 slices over 1, 2 or 4
        // streams, with the class's default schedule flags; then every combination of
        // the kernel schedule flags (XCD-grouped orders of passes A, C and B, pass C's
        // one or two LDS buffers) with the best of those
        auto time_it = [&](const Sched& cand, float* ms) -> int {
            c.args.order = cand.order;
            // one warm-up, then `reps` timed CG steps (passes only, pass C writing M p to
            // w: the solver state is untouched)
            for (int r = 0; r <= reps; ++r) {
                if (r == 1) HIP_TRY(hipEventRecord(e0, st));
                if (int e = run_passes(plan, c.args, 0, c.S, 0, cand.chunk, cand.nstreams, false, st)) return e;
            }
            HIP_TRY(hipEventRecord(e1, st));
            HIP_TRY(hipEventSynchronize(e1));
            HIP_TRY(hipEventElapsedTime(ms, e0, e1));
            return 0;
        };
        const int o0 = t2s::default_order(c.ny, c.nz, plan->prm.K);
        std::vector<Sched> cands{{0, 1, o0}};
        for (int ch : {32, 16, 8, 4, 2})
            if (ch < c.S)
                for (int ns : {1, 2, 4}) cands.push_back({ch, ns, o0});
        float best = 1e30f;
        Sched pick{0, 1, o0};
        for (int phase = 0; phase < 2; ++phase) {
            if (phase == 1) {
                cands.clear();
                for (int o = 0; o <= t2s::kOrderAll; ++o) {
                    // the two-buffer flag only exists where pass C has that variant
                    if ((o & t2s::kOrderLds2C) && !t2s::passC_lds2_supported(c.nz)) continue;
                    if (o != o0) cands.push_back({pick.chunk, pick.nstreams, o});
                }
            }
            for (const Sched& cand : cands) {
                float ms = 0.f;
                if (int e = time_it(cand, &ms)) {
                    c.args.order = c.order;
                    g_prof = saved;
                    return e;
                }
                if (ms < best) {
                    best = ms;
                    pick = cand;
                }
            }
        }
        c.chunk = pick.chunk;
        c.nstreams = pick.nstreams;
        c.order = c.args.order = pick.order;
        std::lock_guard<std::mutex> lk(g_sched_mu);
        g_sched[key] = pick;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g_prof = saved;
    return 0;
}

int t2s_read_coeffs(t2s_plan* plan, int cls, int first, int count, void* out, int which, int mem, void* stream) {
    if (int e = check_class_index(plan, cls, first, count)) return e;
    if (!out) return fail(T2S_EINVAL, "out is NULL");
    if (mem != T2S_HOST && mem != T2S_DEVICE) return fail(T2S_EINVAL, "mem must be T2S_HOST or T2S_DEVICE");
    if (!plan->bound) return fail(T2S_ESTATE, "workspace not bound");
    const ClassPlan& c = plan->cls[cls];
    const ClassArgs& a = c.args;
    const float2* src = nullptr;
    switch (which) {
        case T2S_ALPHA: src = a.x; break;
        case T2S_Z: src = a.z; break;
        case T2S_U: src = a.u; break;
        case T2S_ADJOINT: src = a.b0; break;
        case T2S_RESIDUAL: src = a.r; break;
        default: return fail(T2S_EINVAL, "bad `which`");
    }
    const size_t n = slice_images(c, plan->prm.K);
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(out, src + (size_t)first * n, (size_t)count * n * 8,
                           mem == T2S_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
    if (mem == T2S_HOST) HIP_TRY(hipStreamSynchronize(st));
    return 0;
}

int t2s_get_slice_report(const t2s_plan* plan, int cls, int slice, t2s_slice_report* out) {
    if (int e = check_class_index(plan, cls, slice, 1)) return e;
    if (!out) return fail(T2S_EINVAL, "out is NULL");
    if (!plan->reconstructed) return fail(T2S_ESTATE, "no reconstruct has run");
    const ClassPlan& c = plan->cls[cls];
    const int k = c.outer_run[slice];
    out->outer_iterations = k;
    out->k_freeze = c.k_freeze[slice];
    out->converged = c.converged[slice];
    out->r_primal = out->r_dual = std::numeric_limits<double>::quiet_NaN();
    if (k > 0 && k <= plan->hist_len) {
        double h[8];
        HIP_TRY(hipStreamSynchronize(plan->last_stream));
        HIP_TRY(hipMemcpy(h, c.args.hist + ((size_t)slice * plan->hist_len + (k - 1)) * 8, sizeof(h),
                          hipMemcpyDeviceToHost));
        std::vector<double> part(c.nllr);
        HIP_TRY(hipMemcpy(part.data(), c.args.b0n + (size_t)slice * c.nllr, part.size() * 8, hipMemcpyDeviceToHost));
        double bb = 0.0;
        for (double v : part) bb += v;
        residuals_from_hist(h, std::sqrt(bb), &out->r_primal, &out->r_dual);
    }
    return 0;
}

int t2s_apply_normal(t2s_plan* plan, int cls, int first, int count, const void* in, void* out, float rho_add,
                     void* stream) {
    if (int e = check_class_index(plan, cls, first, count)) return e;
    if (!in || !out) return fail(T2S_EINVAL, "in or out is NULL");
    if (in == out) return fail(T2S_EINVAL, "in and out must not overlap");
    if (!finite_f(rho_add)) return fail(T2S_ENONFINITE, "rho_add is NaN/Inf");
    ClassPlan& c = plan->cls[cls];
    for (int i = 0; i < count; ++i)
        if (!c.loaded[first + i]) return fail(T2S_ESTATE, "slice not loaded");
    hipStream_t st = (hipStream_t)stream;
    g_prof = &plan->prof;
    HIP_CHECK_LAUNCH(t2s::launch_set_state(c.args, first, count, 1, -1, -1, st));
    return run_normal(c.args, first, count, (const float2*)in, first, rho_add, (float2*)out, first, st);
}

int t2s_apply_llr(t2s_plan* plan, int cls, int first, int count, const void* in, void* out, float tau,
                  const int* shifts, void* stream) {
    if (int e = check_class_index(plan, cls, first, count)) return e;
    if (!in || !out || !shifts) return fail(T2S_EINVAL, "NULL argument");
    if (!finite_f(tau) || tau < 0) return fail(T2S_EINVAL, "tau must be finite and >= 0");
    if (!plan->bound) return fail(T2S_ESTATE, "workspace not bound");
    const int b = plan->prm.block;
    for (int i = 0; i < count; ++i)
        if (shifts[2 * i] < 0 || shifts[2 * i] >= b || shifts[2 * i + 1] < 0 || shifts[2 * i + 1] >= b)
            return fail(T2S_EINVAL, "shift out of [0, block)");
    const ClassPlan& c = plan->cls[cls];
    const size_t n = slice_images(c, plan->prm.K);
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < count; ++i)
        HIP_CHECK_LAUNCH(t2s::launch_llr(c.args, first + i, 1, t2s::kLlrProx, 0, (const float2*)in + i * n,
                                         (float2*)out + i * n, tau, shifts[2 * i], shifts[2 * i + 1], 0.f, st));
    return 0;
}

int t2s_lipschitz(t2s_plan* plan, int cls, int iters, double* L, void* stream) {
    if (int e = check_class_index(plan, cls, 0, 1)) return e;
    if (!L) return fail(T2S_EINVAL, "L is NULL");
    if (iters < 1) return fail(T2S_EINVAL, "iters must be >= 1");
    if (!plan->bound) return fail(T2S_ESTATE, "workspace not bound");
    ClassPlan& c = plan->cls[cls];
    for (int s = 0; s < c.S; ++s)
        if (!c.loaded[s]) return fail(T2S_ESTATE, "not every slice of the class is loaded");
    const ClassArgs& a = c.args;
    const size_t n = slice_images(c, plan->prm.K);
    hipStream_t st = (hipStream_t)stream;
    g_prof = &plan->prof;
    HIP_CHECK_LAUNCH(t2s::launch_set_state(a, 0, c.S, 1, -1, -1, st));
    HIP_TRY(hipMemcpyAsync(a.w, a.b0, (size_t)c.S * n * 8, hipMemcpyDeviceToDevice, st));
    const PartialSrc none{nullptr, 0, 0};
    for (int j = 0; j < iters; ++j) {
        // v <- A^H A v with ||v||^2 (pass A partials) and <v, A^H A v> (pass B partials)
        if (j > 0) HIP_CHECK_LAUNCH(t2s::launch_normalize(a, 0, c.S, a.w, st));
        {
            TIMED(T2S_KERNEL_PASS_A);
            HIP_CHECK_LAUNCH(t2s::launch_passA(a, 0, c.S, a.w, 0, 1, none, none, 1, st));
        }
        {
            TIMED(T2S_KERNEL_PASS_B);
            HIP_CHECK_LAUNCH(t2s::launch_passB(a, 0, c.S, 0, 1, st));
        }
        {
            TIMED(T2S_KERNEL_PASS_C);
            HIP_CHECK_LAUNCH(t2s::launch_passC(a, 0, c.S, 0, 0.f, a.w, 0, st));
        }
    }
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<double> pa((size_t)c.S * c.nrw), pb((size_t)c.S * c.npb);
    HIP_TRY(hipMemcpy(pa.data(), a.pa, pa.size() * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(pb.data(), a.pb, pb.size() * 8, hipMemcpyDeviceToHost));
    for (int s = 0; s < c.S; ++s) {
        double vv = 0.0, vnv = 0.0;
        for (int i = 0; i < c.nrw; ++i) vv += pa[(size_t)s * c.nrw + i];
        for (int i = 0; i < c.npb; ++i) vnv += pb[(size_t)s * c.npb + i];
        L[s] = vv > 0.0 ? vnv / vv : 0.0;
    }
    return 0;
}

int t2s_fista(t2s_plan* plan, int mode, int n_iter, float step, void* stream) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    if (mode != T2S_BATCHED && mode != T2S_PER_SLICE) return fail(T2S_EINVAL, "mode must be BATCHED or PER_SLICE");
    if (n_iter < 0) return fail(T2S_EINVAL, "n_iter must be >= 0");
    if (!finite_f(step) || !(step > 0.f)) return fail(T2S_EINVAL, "step must be finite and > 0");
    if (!plan->bound) return fail(T2S_ESTATE, "workspace not bound");
    for (const ClassPlan& c : plan->cls)
        for (int s = 0; s < c.S; ++s)
            if (!c.loaded[s]) return fail(T2S_ESTATE, "not every slice is loaded");
    hipStream_t st = (hipStream_t)stream;
    plan->last_stream = st;
    g_prof = &plan->prof;
    const float tau = plan->prm.lambda * step;
    for (ClassPlan& c : plan->cls) {
        // every slice active, no frozen shift, iteration counter 0; momentum point y = x
        HIP_CHECK_LAUNCH(t2s::launch_set_state(c.args, 0, c.S, 1, -1, 0, st, c.gbase));
        const size_t n = slice_images(c, plan->prm.K);
        HIP_TRY(hipMemcpyAsync(c.args.z, c.args.x, (size_t)c.S * n * 8, hipMemcpyDeviceToDevice, st));
    }
    auto step_range = [&](const ClassArgs& a, int s0, int count) -> int {
        // A^H A y into w (pass C without the rho term), then the fused prox and momentum
        if (int e = run_normal(a, s0, count, a.z, 0, 0.f, a.w, 0, st)) return e;   // class arrays: slice s at s K N
        {
            TIMED(T2S_KERNEL_LLR);
            HIP_CHECK_LAUNCH(t2s::launch_llr(a, s0, count, t2s::kLlrFista, 0, nullptr, nullptr, tau, 0, 0, step, st));
        }
        HIP_CHECK_LAUNCH(t2s::launch_llr_finalize(a, s0, count, st));
        return 0;
    };
    for (int it = 0; it < n_iter; ++it) {
        for (ClassPlan& c : plan->cls) {
            if (mode == T2S_PER_SLICE) {
                for (int s = 0; s < c.S; ++s)
                    if (int e = step_range(c.args, s, 1)) return e;
            } else if (int e = step_range(c.args, 0, c.S)) {
                return e;
            }
        }
    }
    for (ClassPlan& c : plan->cls) {
        std::fill(c.outer_run.begin(), c.outer_run.end(), n_iter);
        std::fill(c.k_freeze.begin(), c.k_freeze.end(), -1);
        std::fill(c.converged.begin(), c.converged.end(), 0);
    }
    plan->reconstructed = true;
    return 0;
}

int t2s_readout_ifft(int nx, int ncoils, int nsamples, const void* in, void* out, void* stream) {
    if (!t2s::fft_col_supported(nx)) return fail(T2S_ESHAPE, "unsupported readout length " + std::to_string(nx));
    if (ncoils < 1 || ncoils > 65535) return fail(T2S_ESHAPE, "ncoils must be in [1, 65535]");
    if (nsamples < 0) return fail(T2S_ESHAPE, "nsamples must be >= 0");
    if (nsamples == 0) return 0;   // nothing to transform (empty arrays may come as NULL)
    if (!in || !out) return fail(T2S_EINVAL, "in or out is NULL");
    const size_t bytes = (size_t)nx * ncoils * nsamples * 8;
    const char* a = (const char*)in;
    const char* b = (const char*)out;
    if (bytes > 0 && a < b + bytes && b < a + bytes) return fail(T2S_EINVAL, "in and out must not overlap");
    HIP_CHECK_LAUNCH(t2s::launch_readout_ifft(nx, ncoils, nsamples, (const float2*)in, (float2*)out,
                                              (hipStream_t)stream));
    return 0;
}

int t2s_wavelet_denoise(t2s_plan* plan, int cls, int first, int count, int levels, float thresh, void* stream) {
    if (int e = check_class_index(plan, cls, first, count)) return e;
    if (levels < 1 || levels > 4) return fail(T2S_EINVAL, "levels must be in [1, 4]");
    if (!finite_f(thresh) || thresh < 0) return fail(T2S_EINVAL, "thresh must be finite and >= 0");
    if (!plan->bound) return fail(T2S_ESTATE, "workspace not bound");
    const ClassPlan& c = plan->cls[cls];
    if (c.ny % 16 || c.nz % 16) return fail(T2S_ESHAPE, "ny and nz must be multiples of 16");
    if (count == 0) return 0;
    HIP_CHECK_LAUNCH(t2s::launch_haar_denoise(c.args, first, count, levels, thresh, (hipStream_t)stream));
    return 0;
}

int t2s_backproject(t2s_plan* plan, int cls, int first, int count, int n_te, const float* phi_te, void* out,
                    void* stream) {
    if (int e = check_class_index(plan, cls, first, count)) return e;
    if (!phi_te || (!out && count > 0)) return fail(T2S_EINVAL, "phi_te or out is NULL");
    if (n_te < 1 || n_te > t2s::kMaxK) return fail(T2S_EINVAL, "n_te must be in [1, 8]");
    for (int i = 0; i < n_te * plan->prm.K; ++i)
        if (!finite_f(phi_te[i])) return fail(T2S_ENONFINITE, "phi_te has NaN/Inf");
    if (!plan->bound) return fail(T2S_ESTATE, "workspace not bound");
    if (count == 0) return 0;
    HIP_CHECK_LAUNCH(t2s::launch_backproject(plan->cls[cls].args, first, count, n_te, phi_te, (float2*)out,
                                             (hipStream_t)stream));
    return 0;
}

int t2s_get_psi(const t2s_plan* plan, int cls, float* out) {
    if (int e = check_class_index(plan, cls, 0, 1)) return e;
    if (!out) return fail(T2S_EINVAL, "out is NULL");
    const ClassPlan& c = plan->cls[cls];
    std::memcpy(out, c.psi.data(), c.psi.size() * 4);
    return 0;
}

int t2s_stream_open(t2s_plan* plan, int cls, t2s_unet* net, int mode) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    if (plan->cls.size() != 1 || cls != 0) return fail(T2S_EINVAL, "streaming needs a one-class plan (cls 0)");
    if (mode != T2S_BATCHED && mode != T2S_BATCHED_GRAPH) return fail(T2S_EINVAL, "mode must be BATCHED or BATCHED_GRAPH");
    if (!plan->bound) return fail(T2S_ESTATE, "workspace not bound");
    if (plan->prm.n_outer < 1) return fail(T2S_EINVAL, "streaming needs n_outer >= 1");
    ClassPlan& c = plan->cls[cls];
    int nb = 0;
    if (net) {
        int K = 0, H = 0, W = 0;
        if (int e = t2s_unet_get_shape(net, &K, &nb, &H, &W)) return e;
        if (K != plan->prm.K || H != c.ny || W != c.nz || c.M != 1)
            return fail(T2S_ESHAPE, "network shape does not match the class (K, ny, nz, one map set)");
    }
    StreamState& q = plan->stream;
    double* keep = q.hpin;
    const size_t keep_len = q.hpin_len;
    q = StreamState{};
    q.hpin = keep;
    q.hpin_len = keep_len;
    const size_t need = (size_t)c.S * plan->hist_len * 8 + (size_t)c.S * c.nllr;
    if (q.hpin_len < need) {
        if (q.hpin) (void)hipHostFree(q.hpin);
        q.hpin = nullptr;
        q.hpin_len = 0;
        HIP_TRY(hipHostMalloc((void**)&q.hpin, need * sizeof(double), hipHostMallocDefault));
        q.hpin_len = need;
    }
    q.open = q.fresh = true;
    q.cls = cls;
    q.mode = mode;
    q.net = net;
    q.net_batch = nb;
    q.slots.assign(c.S, StreamSlot{});
    std::fill(c.loaded.begin(), c.loaded.end(), 0);   // t2s_reconstruct needs fresh loads afterwards
    return 0;
}

int t2s_stream_submit(t2s_plan* plan, int count, int first_global, const void* sens, const void* ksp,
                      void* alpha_out, t2s_slice_report* reports) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    if (!plan->stream.open) return fail(T2S_ESTATE, "stream not open");
    if (count < 1 || first_global < 0) return fail(T2S_EINVAL, "count must be >= 1, first_global >= 0");
    if (!sens || !ksp || !alpha_out) return fail(T2S_EINVAL, "sens, ksp or alpha_out is NULL");
    StreamItem it;
    it.count = count;
    it.g0 = first_global;
    it.sens = (const char*)sens;
    it.ksp = (const char*)ksp;
    it.out = (char*)alpha_out;
    it.rep = reports;
    plan->stream.items.push_back(it);
    return 0;
}

int t2s_stream_run(t2s_plan* plan, int min_done, t2s_stream_status* status, void* stream) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    StreamState& q = plan->stream;
    if (!q.open) return fail(T2S_ESTATE, "stream not open");
    hipStream_t st = (hipStream_t)stream;
    plan->last_stream = st;
    g_prof = &plan->prof;
    ClassPlan& c = plan->cls[q.cls];
    const t2s_params& prm = plan->prm;
    const bool tolmode = prm.tol > 0;
    // outer iterations between decisions (in fixed-iteration mode a slot stops at n_outer only)
    const int ce = tolmode ? prm.check_every : prm.n_outer;
    if (q.fresh) {
        HIP_CHECK_LAUNCH(t2s::launch_set_state(c.args, 0, c.S, 0, -1, 0, st));   // every slot idle
        q.fresh = false;
    }
    if (int e = ensure_streams(plan, c.nstreams)) return e;
    const bool use_graph = q.mode == T2S_BATCHED_GRAPH && !plan->prof.on;
    if (use_graph) {
        if (int e = ensure_graph(plan, T2S_BATCHED_GRAPH)) return e;
    }
    const size_t hn = (size_t)c.S * plan->hist_len * 8;
    double* hist = q.hpin;
    double* b0p = q.hpin + hn;
    const long done0 = q.done;
    int warn = 0;
    for (;;) {
        if (int e = stream_refill(plan, q, c, st)) return e;
        int chunk = ce, nact = 0;
        for (const StreamSlot& sl : q.slots) {
            if (sl.item < 0) continue;
            ++nact;
            chunk = std::min(chunk, std::min(ce - sl.k % ce, prm.n_outer - sl.k));
        }
        if (nact == 0) break;
        // once the queue is empty and fewer than half the slots hold a slice, the
        // XCD-grouped orders (contiguous slot ranges per XCD) would leave some XCDs
        // without work: the remaining launches deal workgroups round-robin (same
        // arithmetic; eager launches only, a captured graph keeps its order)
        bool queued = false;
        for (size_t i = q.head; i < q.items.size() && !queued; ++i) queued = q.items[i].next < q.items[i].count;
        const bool drained = !queued && 2 * nact < c.S;
        c.args.order = (drained && !use_graph) ? (c.order & t2s::kOrderLds2C) : c.order;
        q.slice_outer += (int64_t)nact * chunk;
        for (int i = 0; i < chunk; ++i) {
            if (use_graph) {
                HIP_TRY(hipGraphLaunch(plan->gexec, st));
            } else if (int e = run_outer_all(plan, T2S_BATCHED, st)) {
                return e;
            }
        }
        HIP_TRY(hipMemcpyAsync(hist, c.args.hist, hn * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(b0p, c.args.b0n, (size_t)c.S * c.nllr * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int s = 0; s < c.S; ++s) {
            StreamSlot& sl = q.slots[s];
            if (sl.item < 0) continue;
            sl.k += chunk;
            c.outer_run[s] = sl.k;
            double bb = 0.0;
            for (int j = 0; j < c.nllr; ++j) bb += b0p[(size_t)s * c.nllr + j];
            const double b0_norm = std::sqrt(bb);
            const double* hs = hist + (size_t)s * plan->hist_len * 8;
            bool stop = false;
            if (tolmode && (sl.k % ce == 0 || sl.k >= prm.n_outer)) {
                if (int e = tol_decide(prm, c, s, sl.k, hs, b0_norm, st, &stop)) return e;
            }
            if (!stop && sl.k >= prm.n_outer) {
                stop = true;
                if (tolmode) warn = T2S_WNOTCONVERGED;
                HIP_CHECK_LAUNCH(t2s::launch_set_state(c.args, s, 1, 0, c.k_freeze[s], -1, st));
            }
            if (stop) {
                if (int e = stream_complete(plan, q, c, s, hs, b0_norm, st)) return e;
            }
        }
        if (min_done > 0 && q.done - done0 >= min_done) break;
    }
    c.args.order = c.order;
    plan->reconstructed = true;
    if (status) {
        long f = 0;
        for (const StreamSlot& sl : q.slots) f += sl.item >= 0;
        for (size_t i = q.head; i < q.items.size(); ++i) f += q.items[i].count - q.items[i].next;
        status->done = (int)q.done;
        status->in_flight = (int)f;
        status->loaded = q.loaded;
        status->slice_outer = q.slice_outer;
    }
    if (warn) return fail(warn, "tolerance not met by n_outer for some slices");
    return 0;
}

int t2s_stream_close(t2s_plan* plan) {
    if (!plan) return fail(T2S_EINVAL, "plan is NULL");
    StreamState& q = plan->stream;
    q.open = false;
    q.items.clear();
    q.slots.clear();
    q.head = 0;
    q.net = nullptr;
    return 0;
}

}  // extern "C"
