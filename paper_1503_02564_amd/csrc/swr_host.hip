// swr_host.hip -- C ABI of the SWR library: context, memory plan and the
// orchestration of the hot path (Besse & Xing, arXiv 1503.02564).
//
// Phases of one solve with a time-independent potential (Sec. 4, "New
// algorithm"):
//   1. assembly + factorisation of every subdomain matrix      (factor_kernel)
//   2. ONE launch of all impulse sweeps (first columns of L, Sec. 4.1) and
//      all d = R 0 sweeps                                       (sweep_kernel)
//   3. interface solve of (I - L) g = d: causal forward substitution, GMRES
//      or fixed point                                           (swr_iface)
//   4. final sweep with the converged g -> u(T), R g           (sweep_kernel)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "swr.h"
#include "swr_common.h"


using namespace swr;

// One interface operator built from impulse responses (Sec. 4.1): the first
// columns of its blocks, the factor records its impulse sweeps use, and the
// state of the causal solver built on it.
struct Iface {
    cd* cols = nullptr;     // [nv][N][4][nt]
    cd* fac = nullptr;      // factor records [nv*N][fields][64]
    cd* lfac = nullptr;     // long-chunk factor records [nv*N][fac_fields(Qmax)][64]
    Task* tasks = nullptr;  // impulse tasks
    int ntasks = 0;
    int nv = 1;
    bool dirty = true;      // columns rebuilt since the causal setup
    int path = 0;           // causal solver: 1 = one-wave block PCR, 2 = workgroup block
                            // PCR, 3 = dense inverse, 0 = not offered (valid once !dirty)
    cd* pcr = nullptr;
    size_t pcr_size = 0;
    double* eta = nullptr;
    int levels = 0;         // PCR levels run per step (coupling left <= 2^-60)
    double eta0 = 0;        // block dominance measure of (I - C_0)
    cd* Minv = nullptr;
    cd* Mwork = nullptr;
    int* piv = nullptr;
    int built_version = -1;  // potential version the causal set-up above was built from
};

// A run of tasks of one chunk width: tasks [start, start + count) of a task
// list, whose subdomains all have P = ceil((J_k + 1) / 64) nodes per lane.
// Every task list is ordered by width (widest first), so each width is one
// launch of the sweep kernel instantiated for it: a subdomain of 41 nodes
// no longer runs with the registers and padded rows of the widest one.
struct WidthRun {
    int P, start, count;
    int pstart, pcount;   // its waves of two tasks in the list's pair table
    // its workgroups of at most g tasks of one factor record in the list's
    // group table of size g (g = 2 .. kGroupMax)
    int gstart[kGroupMax + 1], gcount[kGroupMax + 1];
};

struct swr_ctx {
    // problem
    double a0 = 0, b0 = 0, h = 0, dt = 0;
    int N = 0, nt = 0, nx = 0, nc = 0, ns = 0, B = 1, vk = 0, tr = 0, nv = 1, P = 1;
    cd sigma{}, c2{};
    swr_opts o{};
    hipStream_t st = nullptr;
    std::vector<int> J, off;
    // device memory
    int* dJ = nullptr;
    int* dOff = nullptr;
    double* dV = nullptr;
    double* dBeta = nullptr;
    cd* dHist = nullptr;
    EndCoef* dEndc = nullptr; // [nv][N][2] higher-order transmission coefficients
    cd* dPade = nullptr;      // Pade strategy: [2][m+1] coefficients a_s, d_s
    cd* dPadeStB = nullptr;   // ... its auxiliary functions between chunk launches (build, final)
    cd* dPadeStF = nullptr;
    cd* dEnds = nullptr;
    Task* dBuild = nullptr;   // impulses + d sweeps of the potential (static V)
    int nBuild = 0;
    Task* dSub = nullptr;     // one task per (problem, subdomain)
    int nSub = 0;
    std::vector<int> Pk;      // chunk width of each subdomain (c->P is the largest up to kMaxP;
                              // wider subdomains run the long-chunk sweep)
    int Qlong = 0;            // largest long-chunk width (0: none)
    size_t lfstride = 0;      // complex entries per long factor record
    size_t lwrec = 0;         // complex entries per task work record of the long sweep
    cd* dLwork = nullptr;     // [max tasks][lwrec]
    int* dPk = nullptr;
    std::vector<WidthRun> runs_build, runs_sub, runs_L0;
    int2* dPairsB = nullptr;  // pair tables of the build and the per-(problem, subdomain) lists
    int2* dPairsS = nullptr;
    int2* dGroupsB[kGroupMax + 1] = {};   // group tables of the two lists, by group size
    int2* dGroupsS[kGroupMax + 1] = {};
    int n_launch_sweep = 0;   // sweep kernel launches of the current call
    Iface L, L0;              // interface operator of V and of V = 0
    cd* dD = nullptr;
    cd* dG = nullptr;
    cd* dG2 = nullptr;
    cd* dT1 = nullptr;        // work vectors [B][ns][nt]
    cd* dT2 = nullptr;
    cd* dZero = nullptr;      // [B][ns][nt] zeros
    unsigned long long* dMax = nullptr;
    int* dNl = nullptr;       // |u|^2 inner statistics
    int inner_iters = 0;      // inner BiCGStab iterations of P^{-1} (this call)
    // GMRES workspace
    int gm_m = 0;
    cd* dBasis = nullptr;
    cd* dW = nullptr;
    cd* dH = nullptr;
    cd* dCs = nullptr;
    cd* dSn = nullptr;
    cd* dE = nullptr;
    cd* dHp = nullptr;
    cd* dHp2 = nullptr;
    cd* dY = nullptr;
    double* dPart = nullptr;
    double* dNrm = nullptr;
    double* dBn = nullptr;
    double* dRes = nullptr;
    int* dAct = nullptr;
    cd* dBi = nullptr;        // BiCGStab work vectors r, r^, p, v, s, t: [6][B][ns][nt]
    cd* dCoef = nullptr;      // [B][3] per-problem coefficients of lincomb
    cd* dDot = nullptr;       // [B] complex dot products
    cd* dFar = nullptr;       // causal dense path
    cd* dFacc = nullptr;      // causal PCR paths: [seg][B][ns][256] contribution of each
                              // finished super-block to the current one
    cd* dBase = nullptr;      // causal PCR path
    int base_tb = 0;
    // adjoint
    int Jc = 0;
    cd* dCkpt = nullptr;
    cd* dSeg = nullptr;
    cd* dHist2 = nullptr;
    cd* dGfwd = nullptr;
    cd* dDadj = nullptr;
    cd* dGadj = nullptr;
    double* dGends = nullptr;
    cd* dWends = nullptr;
    cd* dUT = nullptr;
    // pipelined static solve: two more streams, carried sweep state, the
    // build sweeps' own S0^2 history, and per-chunk events
    hipStream_t s2 = nullptr, s3 = nullptr;
    cd* dStateB = nullptr;    // [nBuild][2][P][64]
    cd* dStateL = nullptr;    // [L0 impulse tasks][2][P][64]
    // S0^2 split at super-chunks: old far-history parts of the current
    // super-chunk, [list tasks][2][kFarSuper], one buffer per task list
    cd* dFarB = nullptr;
    cd* dFarS = nullptr;
    cd* dFarL = nullptr;
    cd* dStateF = nullptr;    // [nSub][2][P][64]
    cd* dHistB = nullptr;     // [nBuild][2][nt+1]
    std::vector<hipEvent_t> evSync, evTime;
    // snapshots: end-node values [B][S][N][2] (averaged into the output)
    cd* dSnapEnds = nullptr;
    size_t snap_ends_size = 0;
    // convergence history of the last call (swr_info.history)
    std::vector<double> hist;
    // schedule (swr_tune / the tuning cache): pipeline chunk of the static
    // causal solve (0 = staged), S0^2 helper-wave task bound, GMRES restart
    int pipe_chunk = 0;
    int help_max = kHelpMaxTasks;
    int pair_from = kPairFrom;   // two tasks per wave from this chunk width on (9: never)
    int group = kGroupDefault;   // tasks of one factor record per workgroup (1: one per wave)
    int graph = 0;               // 1: capture the static causal solve once, replay it
    int gm_check = 4;            // GMRES: read the residual estimates back every this many steps
    double* dResHist = nullptr;  // GMRES: [restart][B] residual estimate after every inner step
    std::vector<double> hResHist;
    int v_version = 0;           // bumped whenever the potential changes
    // the captured solve and the arguments it was captured with
    hipGraph_t g_graph = nullptr;
    hipGraphExec_t g_exec = nullptr;
    hipStream_t gs = nullptr;    // capture stream (the caller's may be the null stream)
    struct GraphKey {
        const void* u0;
        void *uT, *g, *tr, *sn;
        int pipe, help, pair, group, vver;
        bool operator==(const GraphKey& o) const {
            return u0 == o.u0 && uT == o.uT && g == o.g && tr == o.tr && sn == o.sn && pipe == o.pipe &&
                   help == o.help && pair == o.pair && group == o.group && vver == o.vver;
        }
    } g_key{};
    // arguments of the last uncaptured static causal solve that succeeded:
    // every buffer, stream and event a capture with them uses exists
    GraphKey warm_key{};
    bool warm = false;
    std::string cache_path;   // opts.tune_cache, copied (the caller's string may not outlive setup)
    // this context's GPU and its copy of the static scratch array
    int dev = 0;
    void* scratch = nullptr;
    // host staging (pinned)
    double* hRes = nullptr;
    int* hAct = nullptr;
    hipEvent_t ev[6] = {};
    std::vector<void*> allocs;
};

// with SWR_DEBUG set in the environment, a failing HIP call is reported on
// stderr (call, file, line, HIP error) before the status is returned
static void report_hip_error(hipError_t e, const char* what, const char* file, int line) {
    static const bool on = std::getenv("SWR_DEBUG") != nullptr;
    if (on) std::fprintf(stderr, "swr: %s failed at %s:%d: %s\n", what, file, line, hipGetErrorName(e));
}
#define HIPCHK(x)                                      \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) {                        \
            report_hip_error(e_, #x, __FILE__, __LINE__); \
            return SWR_EDEVICE;                        \
        }                                              \
    } while (0)
#define CHK(x)                                         \
    do {                                               \
        swr_status s_ = (x);                           \
        if (s_ != SWR_OK) return s_;                   \
    } while (0)

template <class T>
static swr_status dalloc(swr_ctx* c, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    void* q = nullptr;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return SWR_ENOMEM;
    c->allocs.push_back(q);
    // SWR_DEBUG_POISON: every buffer starts as all-ones bytes (NaN as a
    // double), so a read before the first write shows up in the results
    static const bool poison = std::getenv("SWR_DEBUG_POISON") != nullptr;
    if (poison && hipMemset(q, 0xff, count * sizeof(T)) != hipSuccess) return SWR_EDEVICE;
    *p = static_cast<T*>(q);
    return SWR_OK;
}
// setup-time allocation: a failure releases the half-built context
#define ALLOC(p, n)                                     \
    do {                                                \
        swr_status s_ = dalloc(c, &(p), (size_t)(n));   \
        if (s_ != SWR_OK) { swr_destroy(c); return s_; } \
    } while (0)
// allocation inside a call on a live context: report, keep the context
#define ALLOC_LIVE(p, n)                                \
    do {                                                \
        swr_status s_ = dalloc(c, &(p), (size_t)(n));   \
        if (s_ != SWR_OK) return s_;                    \
    } while (0)

// ---------------------------------------------------------------------------
// Scratch of the entry point that allocates nothing (swr_apply_R_noalloc): the
// S0^2 boundary history of every sweep task, the end values of u(T) and the
// max-change word live in this file-scope device array of fixed size instead
// of context memory.  Every GPU holds its own copy, at its own address, until
// the process ends; host code never uses the array's name as an address, only
// the pointer hipGetSymbolAddress returns for the current device, taken once
// per device when the first context is set up on it.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)16 << 20;   // 16 MiB per GPU
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];
static bool g_scratch_done[kMaxDevices];

// device address of `scratch` on device `dev` (the current device), looked up
// once per device; null if the lookup failed
static void* scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            report_hip_error(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
            (void)hipGetLastError();   // the failure must not surface in a later error check
            p = nullptr;
        }
        g_scratch_ptr[dev] = p;
        g_scratch_done[dev] = true;
    }
    return g_scratch_ptr[dev];
}

__global__ void zero_word_kernel(unsigned long long* w) { *w = 0ull; }
// graph-safe fills and copies (kernels, not memset/memcpy nodes)
__global__ void zero_ints_kernel(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
__global__ void copy_cd_kernel(const cd* src, cd* dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}
static hipError_t launch_copy_cd(const cd* src, cd* dst, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    copy_cd_kernel<<<(unsigned)blocks, 256, 0, st>>>(src, dst, n);
    return hipGetLastError();
}
__global__ void word_to_double_kernel(const unsigned long long* w, double* out) {
    *out = __longlong_as_double((long long)*w);
}

extern "C" void swr_default_opts(swr_opts* o) {
    if (!o) return;
    o->tol = 1e-10;
    o->max_iter = 20000;
    o->restart = 30;
    o->solver = SWR_SOLVER_CAUSAL;
    o->precond = 1;
    o->batch = 1;
    o->v_per_problem = 0;
    o->checkpoint_K = 64;
    o->nl_max_iter = 100;
    o->nl_tol = 1e-14;
    o->pipeline = -1;
    o->plain = 0;
    o->snapshot_stride = 0;
    o->tune_cache = nullptr;
    o->pade_m = 20;
    o->pade_theta = M_PI / 4;
}

extern "C" const char* swr_strerror(swr_status s) {
    switch (s) {
        case SWR_OK: return "ok";
        case SWR_EINVAL: return "invalid argument";
        case SWR_ENOMEM: return "device allocation failed";
        case SWR_EDEVICE: return "HIP call or kernel launch failed";
        case SWR_ENOCONV: return "iteration limit reached without convergence";
        case SWR_ENAN: return "non-finite interface residual";
    }
    return "unknown status";
}

static int vof(const swr_ctx* c, int b) { return (c->o.v_per_problem && c->vk == SWR_V_STATIC) ? b : 0; }

static std::vector<Task> impulse_tasks(int N, int nv) {
    std::vector<Task> t;
    for (int v = 0; v < nv; ++v)
        for (int k = 0; k < N; ++k) {
            if (k >= 1) t.push_back(Task{k, 0, v * N + k, T_IMP_L | T_OUT_COLS});
            if (k <= N - 2) t.push_back(Task{k, 0, v * N + k, T_IMP_R | T_OUT_COLS});
        }
    return t;
}

static void load_schedule(swr_ctx* c, const char* path);

// transmissions whose history is a convolution over the stored boundary values
static bool conv_hist(int tr) { return tr != SWR_ROBIN && tr <= SWR_S14; }

// S0^2 sweeps of the register form split their far history at super-chunks
// (old part precomputed on the matrix cores; far_sum_s02, launch_widths).
// Static potentials always do (every static form then sums alike); V(t,x)
// and |u|^2 contexts only when their sweeps fill the GPU with one-wave tasks
// -- with few tasks the S0^2 helper wave already sums the far history beside
// the sweep, and the extra launches of the split cost more than they save
// (|u|^2 on 128 x 256 cells, 4000 steps: 815 ms split, 750 ms not).
// Contexts with long-chunk subdomains sum it in one piece.
static bool far_split(const swr_ctx* c) {
    return c->tr == SWR_S02 && !c->Qlong && (c->vk == SWR_V_STATIC || c->nSub > kHelpMaxTasks);
}

// Pade strategy (Sec. 2.2): sqrt(z) ~ sum_{s=0}^m a_s - sum_{s=1}^m a_s d_s/(z + d_s)
// from the partial fractions of the diagonal [m/m] Pade approximant of
// sqrt(1 + w), R_m(w) = 1 + sum_s A_s w/(1 + B_s w) with A_s = 2/(2m+1)
// sin^2(s pi/(2m+1)) and B_s = cos^2(s pi/(2m+1)), used as
// sqrt(z) = e^{i theta/2} sqrt(1 + w), w = e^{-i theta} z - 1 (branch cut
// rotated by theta): d_s = e^{i theta}(1 - B_s)/B_s, a_s = e^{i theta/2}
// A_s/(B_s(1 - B_s)), a_0 = e^{i theta/2} R_m(-1).  Returns [a_0..a_m, d_0..d_m].
static std::vector<cd> pade_coefficients(int m, double theta) {
    std::vector<cd> out(2 * (size_t)(m + 1), mk(0, 0));
    const double ch = std::cos(theta / 2), sh = std::sin(theta / 2);
    const double ct = std::cos(theta), st = std::sin(theta);
    double r_m1 = 1.0;   // R_m(-1)
    for (int s = 1; s <= m; ++s) {
        const double ang = s * M_PI / (2.0 * m + 1.0);
        const double A = 2.0 / (2.0 * m + 1.0) * std::sin(ang) * std::sin(ang);
        const double B = std::cos(ang) * std::cos(ang);
        const double as = A / (B * (1.0 - B)), ds = (1.0 - B) / B;
        out[s] = mk(ch * as, sh * as);
        out[m + 1 + s] = mk(ct * ds, st * ds);
        r_m1 -= A / (1.0 - B);
    }
    out[0] = mk(ch * r_m1, sh * r_m1);
    return out;
}

extern "C" swr_status swr_setup(double a0, double b0, int N, const int* J, double dt, double T,
                                int vk, const double* V, int tr, double s_re, double s_im,
                                const swr_opts* opts, void* stream, swr_ctx** out) {
    if (!out) return SWR_EINVAL;
    *out = nullptr;
    swr_opts o;
    swr_default_opts(&o);
    if (opts) o = *opts;
    if (!(a0 < b0) || N < 1 || !J || !(dt > 0) || !(T > 0)) return SWR_EINVAL;
    if (!std::isfinite(a0) || !std::isfinite(b0) || !std::isfinite(dt) || !std::isfinite(T)) return SWR_EINVAL;
    const double ntd = T / dt;
    const double ntr = std::round(ntd);
    if (ntr < 1 || std::fabs(ntd - ntr) > 1e-9 * ntd || ntr > 1e8) return SWR_EINVAL;
    if (vk < SWR_V_STATIC || vk > SWR_V_CUBIC || tr < SWR_ROBIN || tr > SWR_P24) return SWR_EINVAL;
    if (tr >= SWR_P22 && (o.pade_m < 1 || o.pade_m > kPadeMax || !(o.pade_theta > 0) ||
                          !(o.pade_theta < M_PI)))
        return SWR_EINVAL;
    // the order-4 operators carry dn W; with |u|^2 the paper finds no
    // discretisation of dn f(u) that keeps the interfaces continuous
    if ((tr == SWR_S04 || tr == SWR_S14 || tr == SWR_P24) && vk == SWR_V_CUBIC) return SWR_EINVAL;
    if (tr == SWR_ROBIN && s_re == 0.0 && s_im == 0.0) return SWR_EINVAL;
    if (!std::isfinite(s_re) || !std::isfinite(s_im)) return SWR_EINVAL;
    if (o.batch < 1 || o.restart < 1 || o.max_iter < 1 || !(o.tol > 0)) return SWR_EINVAL;
    if (o.nl_max_iter < 1 || !(o.nl_tol > 0) || o.checkpoint_K < 1) return SWR_EINVAL;
    if (o.pipeline < -1 || (o.pipeline > 0 && o.pipeline % kWave != 0)) return SWR_EINVAL;
    if (o.snapshot_stride < 0) return SWR_EINVAL;
    if (vk == SWR_V_TIME && !V) return SWR_EINVAL;
    if (vk == SWR_V_CUBIC && V) return SWR_EINVAL;
    if (vk != SWR_V_STATIC && o.v_per_problem) return SWR_EINVAL;
    long nc = 0;
    int nmax = 0;
    for (int k = 0; k < N; ++k) {
        if (J[k] < 1) return SWR_EINVAL;
        nc += J[k];
        nmax = J[k] + 1 > nmax ? J[k] + 1 : nmax;
    }
    if (nmax > kWave * kLongMaxQ || nc > (1L << 30)) return SWR_EINVAL;
    // subdomains beyond 64 * kMaxP nodes (long-chunk sweep): Robin and S0^2
    if (nmax > kWave * kMaxP && tr != SWR_ROBIN && tr != SWR_S02) return SWR_EINVAL;

    swr_ctx* c = new (std::nothrow) swr_ctx();
    if (!c) return SWR_ENOMEM;
    c->a0 = a0; c->b0 = b0; c->dt = dt; c->N = N; c->nt = (int)ntr; c->nc = (int)nc;
    c->nx = (int)nc + 1; c->h = (b0 - a0) / (double)nc; c->ns = 2 * N - 2; c->B = o.batch;
    c->vk = vk; c->tr = tr; c->o = o; c->st = (hipStream_t)stream;
    if (const hipError_t e = hipGetDevice(&c->dev); e != hipSuccess) {
        report_hip_error(e, "hipGetDevice", __FILE__, __LINE__);
        delete c;
        return SWR_EDEVICE;
    }
    c->scratch = scratch_address(c->dev);
    c->nv = (vk == SWR_V_STATIC && o.v_per_problem) ? o.batch : 1;
    c->P = std::min((nmax + kWave - 1) / kWave, kMaxP);
    c->Qlong = nmax > kWave * kMaxP ? (nmax + kWave - 1) / kWave : 0;
    c->c2 = mk(std::cos(-M_PI / 4) * std::sqrt(2.0 / dt), std::sin(-M_PI / 4) * std::sqrt(2.0 / dt));
    // S0^2: the implicit coefficient of c2 sum beta_{n-s} v_s is c2 beta_0 = c2
    c->sigma = (tr == SWR_ROBIN) ? mk(s_re, s_im) : c->c2;
    c->J.assign(J, J + N);
    c->off.resize(N);
    for (int k = 0, acc = 0; k < N; ++k) { c->off[k] = acc; acc += J[k]; }

    const int nt = c->nt, B = c->B, ns = c->ns, nv = c->nv;
    c->Pk.resize(N);
    for (int k = 0; k < N; ++k) c->Pk[k] = (J[k] + 1 + kWave - 1) / kWave;
    // task lists, each ordered by chunk width (widest first; stable within a width)
    std::vector<Task> build = impulse_tasks(N, nv), sub, imp0 = impulse_tasks(N, 1);
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < N; ++k) build.push_back(Task{k, b, vof(c, b) * N + k, T_DATA_U0 | T_OUT_G});
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < N; ++k) sub.push_back(Task{k, b, vof(c, b) * N + k, 0});
    // ordered by width, then by factor record, so that tasks sharing a record
    // are neighbours; each run of a width is cut into waves of two tasks of
    // one record (a record with an odd count leaves a single)
    auto by_width = [c](std::vector<Task>& list, std::vector<WidthRun>& runs, std::vector<int2>* pairs) {
        std::stable_sort(list.begin(), list.end(), [c](const Task& x, const Task& y) {
            if (c->Pk[x.k] != c->Pk[y.k]) return c->Pk[x.k] > c->Pk[y.k];
            return x.f < y.f;
        });
        runs.clear();
        for (int i = 0; i < (int)list.size(); ++i) {
            const int P = c->Pk[list[i].k];
            if (runs.empty() || runs.back().P != P) runs.push_back(WidthRun{P, i, 0, 0, 0});
            ++runs.back().count;
        }
        if (!pairs) return;
        pairs->clear();
        for (WidthRun& r : runs) {
            r.pstart = (int)pairs->size();
            for (int i = r.start; i < r.start + r.count;) {
                const bool two = i + 1 < r.start + r.count && list[i + 1].f == list[i].f;
                pairs->push_back(make_int2(i, two ? i + 1 : -1));
                i += two ? 2 : 1;
            }
            r.pcount = (int)pairs->size() - r.pstart;
        }
    };
    // ... and, for every group size g, into workgroups of at most g tasks of
    // one record
    auto by_group = [](const std::vector<Task>& list, std::vector<WidthRun>& runs, std::vector<int2>* groups) {
        for (int g = 2; g <= kGroupMax; ++g) {
            groups[g].clear();
            for (WidthRun& r : runs) {
                r.gstart[g] = (int)groups[g].size();
                for (int i = r.start; i < r.start + r.count;) {
                    int j = i + 1;
                    while (j < r.start + r.count && j - i < g && list[j].f == list[i].f) ++j;
                    groups[g].push_back(make_int2(i, j - i));
                    i = j;
                }
                r.gcount[g] = (int)groups[g].size() - r.gstart[g];
            }
        }
    };
    std::vector<int2> pairs_build, pairs_sub, groups_build[kGroupMax + 1], groups_sub[kGroupMax + 1];
    by_width(build, c->runs_build, &pairs_build);
    by_width(sub, c->runs_sub, &pairs_sub);
    by_width(imp0, c->runs_L0, nullptr);
    by_group(build, c->runs_build, groups_build);
    by_group(sub, c->runs_sub, groups_sub);
    c->nBuild = (int)build.size();
    // default schedule; a tuning cache entry for this problem replaces it
    c->pipe_chunk = o.pipeline >= 0 ? o.pipeline : kPipeChunk;
    if (o.tune_cache) {
        c->cache_path = o.tune_cache;
        load_schedule(c, o.tune_cache);
    }
    c->o.tune_cache = nullptr;
    c->nSub = (int)sub.size();
    const size_t vec = (size_t)B * ns * nt;
    const size_t max_tasks = std::max(build.size(), std::max(sub.size(), imp0.size()));
    const int fields = fac_fields(c->P);
    if (c->Qlong) {
        c->lfstride = (size_t)fac_fields(c->Qlong) * kWave;
        c->lwrec = (size_t)(3 * c->Qlong + (vk == SWR_V_TIME ? fac_fields(c->Qlong) : 0)) * kWave;
        ALLOC(c->dLwork, max_tasks * c->lwrec);
    }
    ALLOC(c->dJ, N);
    ALLOC(c->dOff, N);
    ALLOC(c->dPk, N);
    // beta_0 .. beta_{nt+64}, and at least beta_0 .. beta_{2*64-1} (the
    // sweep's LDS copy of the first 128 weights)
    const int nbeta = std::max(nt, kWave) + kWave + 1;
    ALLOC(c->dBeta, nbeta);
    ALLOC(c->dHist, conv_hist(tr) ? max_tasks * 2 * (nt + 1) : 1);
    if (tr > SWR_S02) ALLOC(c->dEndc, (size_t)nv * N * 2);
    std::vector<cd> pade;
    if (tr >= SWR_P22) {
        pade = pade_coefficients(o.pade_m, o.pade_theta);
        ALLOC(c->dPade, pade.size());
    }
    ALLOC(c->dEnds, (size_t)B * N * 2);
    ALLOC(c->dBuild, build.size());
    ALLOC(c->dSub, sub.size());
    ALLOC(c->dPairsB, pairs_build.size());
    ALLOC(c->dPairsS, pairs_sub.size());
    for (int g = 2; g <= kGroupMax; ++g) {
        ALLOC(c->dGroupsB[g], groups_build[g].size());
        ALLOC(c->dGroupsS[g], groups_sub[g].size());
    }
    ALLOC(c->dD, vec);
    ALLOC(c->dG, vec);
    ALLOC(c->dG2, vec);
    ALLOC(c->dT1, vec);
    ALLOC(c->dT2, vec);
    ALLOC(c->dZero, vec);
    ALLOC(c->dMax, 1);
    ALLOC(c->dNl, 2);
    ALLOC(c->dPart, (size_t)B * kRedBlocks * 2 * (o.restart + 2));
    ALLOC(c->dNrm, B);
    ALLOC(c->dBn, B);
    ALLOC(c->dRes, B);
    ALLOC(c->dAct, B);
    // interface operator of the potential (static V) ...
    c->L.nv = nv;
    c->L.tasks = c->dBuild;   // its impulse tasks lead the build list
    c->L.ntasks = (int)impulse_tasks(N, nv).size();
    if (vk == SWR_V_STATIC) {
        ALLOC(c->L.fac, (size_t)nv * N * fields * kWave);
        ALLOC(c->L.cols, (size_t)nv * N * 4 * nt);
        if (c->Qlong) ALLOC(c->L.lfac, (size_t)nv * N * c->lfstride);
    }
    // ... and of the zero potential (preconditioner; also the V-free factors
    // of the |u|^2 scheme)
    if (vk != SWR_V_STATIC) {
        c->L0.nv = 1;
        c->L0.ntasks = (int)imp0.size();
        ALLOC(c->L0.fac, (size_t)N * fields * kWave);
        ALLOC(c->L0.cols, (size_t)N * 4 * nt);
        if (c->Qlong) ALLOC(c->L0.lfac, (size_t)N * c->lfstride);
        ALLOC(c->L0.tasks, imp0.size());
    }
    // S0^2 sweeps carry their state across super-chunk launches and read the
    // old far-history parts of their super-chunk (see launch_widths)
    if (far_split(c)) {
        const size_t st_rec = (size_t)2 * c->P * kWave;
        ALLOC(c->dStateB, build.size() * st_rec);
        ALLOC(c->dStateF, sub.size() * st_rec);
        ALLOC(c->dFarB, build.size() * 2 * kFarSuper);
        ALLOC(c->dFarS, sub.size() * 2 * kFarSuper);
        if (c->L0.tasks) {
            ALLOC(c->dStateL, imp0.size() * st_rec);
            ALLOC(c->dFarL, imp0.size() * 2 * kFarSuper);
        }
    }
    if (vk != SWR_V_CUBIC) {
        // the library's own copy of the potential (zeros when V is NULL)
        const size_t vn = (vk == SWR_V_TIME) ? (size_t)c->nx * (nt + 1)
                                             : (size_t)c->nx * (o.v_per_problem ? B : 1);
        ALLOC(c->dV, vn);
        if (V) HIPCHK(hipMemcpyAsync(c->dV, V, vn * sizeof(double), hipMemcpyDeviceToDevice, c->st));
        else HIPCHK(hipMemsetAsync(c->dV, 0, vn * sizeof(double), c->st));
    }
    if (hipHostMalloc(&c->hRes, sizeof(double) * B) != hipSuccess ||
        hipHostMalloc(&c->hAct, sizeof(int) * B) != hipSuccess) { swr_destroy(c); return SWR_ENOMEM; }
    for (auto& e : c->ev)
        if (const hipError_t er = hipEventCreate(&e); er != hipSuccess) {
            report_hip_error(er, "hipEventCreate", __FILE__, __LINE__);
            swr_destroy(c);
            return SWR_EDEVICE;
        }
    HIPCHK(hipMemcpyAsync(c->dJ, c->J.data(), N * sizeof(int), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->dOff, c->off.data(), N * sizeof(int), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->dPk, c->Pk.data(), N * sizeof(int), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->dBuild, build.data(), build.size() * sizeof(Task), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->dSub, sub.data(), sub.size() * sizeof(Task), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->dPairsB, pairs_build.data(), pairs_build.size() * sizeof(int2),
                          hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->dPairsS, pairs_sub.data(), pairs_sub.size() * sizeof(int2),
                          hipMemcpyHostToDevice, c->st));
    for (int g = 2; g <= kGroupMax; ++g) {
        HIPCHK(hipMemcpyAsync(c->dGroupsB[g], groups_build[g].data(), groups_build[g].size() * sizeof(int2),
                              hipMemcpyHostToDevice, c->st));
        HIPCHK(hipMemcpyAsync(c->dGroupsS[g], groups_sub[g].data(), groups_sub[g].size() * sizeof(int2),
                              hipMemcpyHostToDevice, c->st));
    }
    if (c->L0.tasks)
        HIPCHK(hipMemcpyAsync(c->L0.tasks, imp0.data(), imp0.size() * sizeof(Task), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemsetAsync(c->dZero, 0, vec * sizeof(cd), c->st));
    if (c->L.cols) HIPCHK(hipMemsetAsync(c->L.cols, 0, (size_t)nv * N * 4 * nt * sizeof(cd), c->st));
    if (c->L0.cols) HIPCHK(hipMemsetAsync(c->L0.cols, 0, (size_t)N * 4 * nt * sizeof(cd), c->st));
    HIPCHK(launch_beta(nbeta, c->dBeta, c->st));
    if (c->dPade)
        HIPCHK(hipMemcpyAsync(c->dPade, pade.data(), pade.size() * sizeof(cd), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    *out = c;
    return SWR_OK;
}

extern "C" void swr_destroy(swr_ctx* c) {
    if (!c) return;
    if (c->st) hipStreamSynchronize(c->st);
    else hipDeviceSynchronize();
    if (c->g_exec) hipGraphExecDestroy(c->g_exec);
    if (c->g_graph) hipGraphDestroy(c->g_graph);
    if (c->gs) hipStreamDestroy(c->gs);
    if (c->s2) hipStreamSynchronize(c->s2);
    if (c->s3) hipStreamSynchronize(c->s3);
    for (void* p : c->allocs) hipFree(p);
    if (c->hRes) hipHostFree(c->hRes);
    if (c->hAct) hipHostFree(c->hAct);
    for (auto& e : c->ev)
        if (e) hipEventDestroy(e);
    for (auto e : c->evSync) hipEventDestroy(e);
    for (auto e : c->evTime) hipEventDestroy(e);
    if (c->s2) { hipStreamSynchronize(c->s2); hipStreamDestroy(c->s2); }
    if (c->s3) { hipStreamSynchronize(c->s3); hipStreamDestroy(c->s3); }
    delete c;
}

static int nsnaps(const swr_ctx* c);

extern "C" swr_status swr_sizes(const swr_ctx* c, int* nt, int* nx, int* B, int* nv, int* N, int* vk,
                                int* S) {
    if (!c) return SWR_EINVAL;
    if (nt) *nt = c->nt;
    if (nx) *nx = c->nx;
    if (B) *B = c->B;
    if (nv) *nv = c->nv;
    if (N) *N = c->N;
    if (vk) *vk = c->vk;
    if (S) *S = nsnaps(c);
    return SWR_OK;
}

// ---------------------------------------------------------------------------
// Sweep launches
// ---------------------------------------------------------------------------
struct SweepIO {
    const cd* u0 = nullptr;     // data (null: zero data and zero v_0 history)
    const cd* g_in = nullptr;
    cd* g_out = nullptr;
    cd* uT = nullptr;
    cd* trace = nullptr;
    cd* snaps = nullptr;        // [B][S][nx] snapshots every c->o.snapshot_stride steps
    bool maxdiff = false;
    bool ckpt = false;
};

// number of snapshots of a solve: steps 0, s, 2s, ... <= nt
static int nsnaps(const swr_ctx* c) {
    return c->o.snapshot_stride > 0 ? c->nt / c->o.snapshot_stride + 1 : 0;
}

// kernel form of the transmission operator: Robin, S0^2, or the general
// convolution form of the higher-order operators
static int ktr(const swr_ctx* c) {
    if (c->tr >= SWR_P22) return TR_PADE;
    return c->tr == SWR_ROBIN ? TR_ROBIN : (c->tr == SWR_S02 ? TR_S02 : TR_GEN);
}

static SweepArgs sweep_args(swr_ctx* c, const Task* tasks, int ntasks, const cd* fac, cd* cols) {
    SweepArgs a{};
    a.N = c->N; a.nt = c->nt; a.B = c->B; a.nx = c->nx; a.ns = c->ns; a.ntasks = ntasks;
    a.P = c->P;
    a.kappa = c->h / (3.0 * c->dt);
    a.h = c->h;
    a.sigma = c->sigma;
    a.c2 = c->c2;
    a.J = c->dJ; a.off = c->dOff; a.tasks = tasks; a.fac = fac; a.beta = c->dBeta;
    a.cols = cols; a.hist = c->dHist; a.ends = c->dEnds; a.maxdiff = c->dMax;
    a.endc = c->dEndc;
    a.tr = c->tr;
    a.dt = c->dt;
    a.pade = c->dPade;
    a.pade_m = c->o.pade_m;
    a.pade_order = c->tr == SWR_P24 ? 4 : 2;
    a.pstate = nullptr;
    a.Vt = (c->vk == SWR_V_TIME) ? c->dV : nullptr;
    a.nl_maxit = c->o.nl_max_iter;
    a.nl_tol = c->o.nl_tol;
    a.nl_stats = c->dNl;
    a.flags_and = ~0;
    a.flags_or = 0;
    a.help_max = c->help_max;
    a.pstride = c->P;
    a.fstride = (size_t)fac_fields(c->P) * kWave;
    a.lfac = fac == c->L.fac ? c->L.lfac : (fac == c->L0.fac ? c->L0.lfac : nullptr);
    a.lfstride = c->lfstride;
    a.lwork = c->dLwork;
    a.lq = 0;
    a.task0 = 0;
    a.n_begin = 0;
    a.n_end = c->nt;
    a.state = nullptr;
    return a;
}

// factor records of a static potential (V = null: zero potential)
static swr_status run_factor(swr_ctx* c, const double* V, int nv, cd* fac) {
    FactorArgs f{};
    f.N = c->N; f.nx = c->nx; f.nf = nv * c->N; f.P = c->P; f.h = c->h; f.dt = c->dt;
    f.sigma = c->sigma; f.J = c->dJ; f.off = c->dOff; f.V = V; f.fac = fac;
    f.tr = c->tr; f.c2 = c->c2; f.endc = c->dEndc;
    f.pade = c->dPade; f.pade_m = c->o.pade_m;
    f.Pk = c->dPk;
    f.fstride = (size_t)fac_fields(c->P) * kWave;
    // one launch per chunk width present; each builds the records of its width
    std::vector<int> widths(c->Pk);
    std::sort(widths.begin(), widths.end());
    widths.erase(std::unique(widths.begin(), widths.end()), widths.end());
    cd* lfac = fac == c->L.fac ? c->L.lfac : (fac == c->L0.fac ? c->L0.lfac : nullptr);
    for (int P : widths) {
        f.P = P;
        if (P <= kMaxP) {
            HIPCHK(launch_factor(f, c->st));
        } else {
            // long-chunk records (swr_sweep_long.hip)
            if (!lfac) return SWR_EINVAL;
            FactorArgs fl = f;
            fl.fac = lfac;
            fl.fstride = c->lfstride;
            HIPCHK(launch_factor_long(fl, P, c->st));
        }
    }
    return SWR_OK;
}

// the factor records used by the per-(problem, subdomain) sweeps
static const cd* main_fac(swr_ctx* c) { return c->vk == SWR_V_STATIC ? c->L.fac : c->L0.fac; }

// every (problem, subdomain) swept once with the fluxes io.g_in (null: zero)
static SweepArgs sub_args(swr_ctx* c, const SweepIO& io) {
    SweepArgs a = sweep_args(c, c->dSub, c->nSub, main_fac(c), nullptr);
    a.u0 = io.u0;
    a.g_in = io.g_in ? io.g_in : c->dZero;
    a.g_out = io.g_out;
    a.uT = io.uT;
    a.trace = io.trace;
    a.flags_and = 0;
    a.flags_or = (io.u0 ? T_DATA_U0 : 0) | (io.g_in ? T_FLUX_G : 0) | (io.g_out ? T_OUT_G : 0) |
                 (io.uT ? T_OUT_UT : 0) | (io.trace ? T_OUT_TRACE : 0) | (io.maxdiff ? T_MAXDIFF : 0) |
                 (io.ckpt ? T_CKPT : 0) | (io.snaps ? T_OUT_SNAP : 0);
    a.ckpt = c->dCkpt;
    a.Jc = c->Jc;
    a.snaps = io.snaps;
    a.snap_ends = c->dSnapEnds;
    a.snap_stride = c->o.snapshot_stride;
    a.nsnap = nsnaps(c);
    return a;
}

// the width runs of a task list
static const std::vector<WidthRun>& runs_of(const swr_ctx* c, const Task* tasks) {
    if (tasks == c->dBuild) return c->runs_build;
    if (tasks == c->dSub) return c->runs_sub;
    return c->runs_L0;
}

// the old-far-part buffer and the state buffer of a task list
static cd* far_old_of(const swr_ctx* c, const Task* tasks) {
    if (tasks == c->dBuild) return c->dFarB;
    if (tasks == c->dSub) return c->dFarS;
    if (tasks == c->L0.tasks) return c->dFarL;
    return nullptr;
}

static cd* state_of(const swr_ctx* c, const Task* tasks) {
    if (tasks == c->dBuild) return c->dStateB;
    if (tasks == c->dSub) return c->dStateF;
    if (tasks == c->L0.tasks) return c->dStateL;
    return nullptr;
}

static const int2* pairs_of(const swr_ctx* c, const Task* tasks) {
    if (tasks == c->dBuild) return c->dPairsB;
    if (tasks == c->dSub) return c->dPairsS;
    return nullptr;
}

static const int2* groups_of(const swr_ctx* c, const Task* tasks, int g) {
    if (tasks == c->dBuild) return c->dGroupsB[g];
    if (tasks == c->dSub) return c->dGroupsS[g];
    return nullptr;
}

// largest group size at most g whose workgroup (the width-P factor record and
// the waves' staging) fits the 64 KiB of LDS a workgroup may use by default
static int group_fit(int P, int g) {
    auto lds = [P](int q) {
        return sizeof(cd) * ((size_t)fac_fields(P) * kWave + (size_t)q * 2 * kWave) +
               sizeof(double) * (size_t)q * 2 * kWave + sizeof(double) * 2 * kWave;
    };
    while (g > 1 && lds(g) > 65536) --g;
    return g;
}

// all tasks of a's list (a.task0 = 0, a.ntasks = the whole list), one launch
// per chunk width, in order on one stream; *launches counts the kernels.  A
// run that fills the GPU with one-wave tasks (more than help_max of them) of
// a static potential with Robin or S0^2 runs two tasks per wave where it has
// pairs from width pair_from on, else, with group >= 2 and tasks that share
// factor records (two or more per record on average), workgroups of up to
// group tasks of one record reading one LDS copy of it: the same arithmetic
// per task in every form.
static hipError_t launch_widths_range(const swr_ctx* c, SweepArgs a, int vk, hipStream_t st, bool plain,
                                      int* launches) {
    const int2* pairs = pairs_of(c, a.tasks);
    const int tr = ktr(c);
    for (const WidthRun& r : runs_of(c, a.tasks)) {
        a.P = r.P;
        if (r.P > kMaxP) {
            // subdomains beyond 64 * kMaxP nodes: the long-chunk sweep, one launch
            a.task0 = r.start;
            a.ntasks = r.count;
            a.lq = r.P;
            const hipError_t e = launch_sweep_long(a, tr, vk, st);
            if (e != hipSuccess) return e;
            if (launches) *launches += 1;
            continue;
        }
        const bool two = !plain && pairs && vk == SWR_V_STATIC && (tr == TR_S02 || tr == TR_ROBIN) &&
                         r.P >= c->pair_from && r.count > c->help_max && 4 * r.pcount <= 3 * r.count;
        const int gsz = group_fit(r.P, c->group);
        const bool grp = !two && !plain && gsz >= 2 && vk == SWR_V_STATIC && (tr == TR_S02 || tr == TR_ROBIN) &&
                         r.count > c->help_max && groups_of(c, a.tasks, gsz) && 2 * r.gcount[gsz] <= r.count;
        hipError_t e;
        if (two) {
            a.pairs = pairs;
            a.task0 = r.pstart;
            a.ntasks = r.pcount;
            e = launch_sweep_pairs(a, tr, st);
        } else if (grp) {
            a.groups = groups_of(c, a.tasks, gsz);
            a.task0 = r.gstart[gsz];
            a.ntasks = r.gcount[gsz];
            e = launch_sweep_groups(a, tr, gsz, st);
        } else {
            a.task0 = r.start;
            a.ntasks = r.count;
            e = launch_sweep(a, tr, vk, st, plain);
        }
        if (e != hipSuccess) return e;
        if (launches) *launches += plain ? r.count : 1;
    }
    return hipSuccess;
}

// S0^2 (register sweeps): the steps a.n_begin+1 .. a.n_end are launched in
// pieces that end at super-chunk boundaries (multiples of kFarSuper), each
// super-chunk after the first preceded by the batched product of its old
// far-history parts (far_old_kernel); the sweeps carry their state across
// the pieces in the list's state buffer.  Every S0^2 sweep of a context goes
// through here, so all its forms sum the far history alike.
static hipError_t launch_widths(const swr_ctx* c, SweepArgs a, int vk, hipStream_t st, bool plain,
                                int* launches = nullptr) {
    cd* fo = far_split(c) ? far_old_of(c, a.tasks) : nullptr;
    if (!fo) {
        a.far_old = nullptr;
        return launch_widths_range(c, a, vk, st, plain, launches);
    }
    if (!a.state) a.state = state_of(c, a.tasks);
    if (!a.state) return hipErrorInvalidValue;
    a.far_old = fo;
    const int n1 = a.n_end;
    for (int s0 = a.n_begin; s0 < n1;) {
        const int s1 = std::min(n1, (s0 / kFarSuper + 1) * kFarSuper);
        if (s0 > 0 && s0 % kFarSuper == 0) {
            FarOldArgs f{};
            f.hist = a.hist;
            f.beta = a.beta;
            f.out = fo;
            f.ntasks = a.ntasks;
            f.nt = c->nt;
            f.C = s0;
            const hipError_t e = launch_far_old(f, st);
            if (e != hipSuccess) return e;
        }
        a.n_begin = s0;
        a.n_end = s1;
        const hipError_t e = launch_widths_range(c, a, vk, st, plain, launches);
        if (e != hipSuccess) return e;
        s0 = s1;
    }
    return hipSuccess;
}

static swr_status run_sweeps(swr_ctx* c, const SweepIO& io) {
    SweepArgs a = sub_args(c, io);
    if (io.maxdiff) HIPCHK(hipMemsetAsync(c->dMax, 0, sizeof(unsigned long long), c->st));
    HIPCHK(launch_widths(c, a, c->vk, c->st, c->o.plain, &c->n_launch_sweep));
    if (io.uT) HIPCHK(launch_finalize_ut(c->N, c->nx, c->B, c->dOff, c->dEnds, io.uT, c->st));
    if (io.snaps)
        HIPCHK(launch_finalize_snaps(c->N, c->nx, c->B, nsnaps(c), c->dOff, c->dSnapEnds, io.snaps, c->st));
    return SWR_OK;
}

// static potential: impulse sweeps of L and the d sweeps in ONE launch
static swr_status run_build(swr_ctx* c, const double* u0) {
    SweepArgs a = sweep_args(c, c->dBuild, c->nBuild, c->L.fac, c->L.cols);
    a.u0 = reinterpret_cast<const cd*>(u0);
    a.g_in = c->dZero;
    a.g_out = c->dD;
    HIPCHK(launch_widths(c, a, SWR_V_STATIC, c->st, c->o.plain, &c->n_launch_sweep));
    c->L.dirty = true;
    return SWR_OK;
}

// impulse sweeps of the zero-potential operator L_0 (Sec. 5)
static swr_status run_build_L0(swr_ctx* c) {
    CHK(run_factor(c, nullptr, 1, c->L0.fac));
    SweepArgs a = sweep_args(c, c->L0.tasks, c->L0.ntasks, c->L0.fac, c->L0.cols);
    a.g_in = c->dZero;
    HIPCHK(launch_widths(c, a, SWR_V_STATIC, c->st, c->o.plain));
    c->L0.dirty = true;
    return SWR_OK;
}

static LttArgs ltt_args(swr_ctx* c, const Iface& I, const cd* x, cd* y) {
    LttArgs l{};
    l.N = c->N; l.nt = c->nt; l.ns = c->ns; l.B = c->B; l.per_problem = I.nv > 1;
    l.cols = I.cols; l.x = x; l.y = y; l.base = x; l.sign = -1.0;
    l.n_lo = 0; l.n_hi = c->nt; l.s_hi = c->nt; l.y_ld = c->nt;
    return l;
}

// ---------------------------------------------------------------------------
// Interface solvers
// ---------------------------------------------------------------------------
using Op = std::function<swr_status(const cd* x, cd* y)>;

// GMRES(m) for A x = rhs, all problems of the batch at once (each with its
// own Krylov space); classical Gram-Schmidt applied twice; x holds the
// initial guess on entry.  Convergence: ||rhs - A x|| <= tol ||rhs|| per
// problem, confirmed on the true residual at a restart.
static swr_status run_gmres(swr_ctx* c, const Op& A, const cd* rhs, cd* x, int* iters_out) {
    const int m = c->o.restart, B = c->B;
    const long M = (long)c->ns * c->nt;
    if (c->gm_m != m) {
        ALLOC_LIVE(c->dBasis, (size_t)(m + 1) * B * M);
        ALLOC_LIVE(c->dW, (size_t)B * M);
        ALLOC_LIVE(c->dH, (size_t)B * (m + 1) * m);
        ALLOC_LIVE(c->dCs, (size_t)B * m);
        ALLOC_LIVE(c->dSn, (size_t)B * m);
        ALLOC_LIVE(c->dE, (size_t)B * (m + 1));
        ALLOC_LIVE(c->dHp, (size_t)B * (m + 1));
        ALLOC_LIVE(c->dHp2, (size_t)B * (m + 1));
        ALLOC_LIVE(c->dY, (size_t)B * (m + 1));
        ALLOC_LIVE(c->dResHist, (size_t)B * m);
        c->hResHist.assign((size_t)B * m, 0.0);
        c->gm_m = m;
    }
    hipStream_t st = c->st;
    HIPCHK(launch_norm(rhs, M, B, c->dPart, c->dBn, st));
    int its = 0;
    bool conv = false;
    while (true) {
        // r = rhs - A x -> basis[0]
        CHK(A(x, c->dW));
        HIPCHK(launch_axpby(rhs, 1.0, c->dW, -1.0, c->dBasis, (long)B * M, st));
        HIPCHK(launch_norm(c->dBasis, M, B, c->dPart, c->dNrm, st));
        HIPCHK(launch_gmres_init(m, B, c->dNrm, c->dE, c->dAct, c->dBn, c->o.tol, c->dRes, st));
        HIPCHK(hipMemcpyAsync(c->hAct, c->dAct, sizeof(int) * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(c->hRes, c->dRes, sizeof(double) * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool any = false;
        for (int b = 0; b < B; ++b) {
            if (!std::isfinite(c->hRes[b])) return SWR_ENAN;
            any |= c->hAct[b] != 0;
        }
        if (!any) { conv = true; break; }
        if (its >= c->o.max_iter) break;
        HIPCHK(launch_scale(c->dBasis, c->dNrm, c->dBasis, M, B, nullptr, st));
        // The residual estimates of the inner steps are read back every
        // gm_check steps (and at the cycle's and the budget's end), not after
        // each: the steps between two reads run without a host round trip.
        // The first step at which every active problem has converged is found
        // among them afterwards, and the solve uses exactly the columns up to
        // it (later steps only add Hessenberg columns and rotate e below it),
        // so the iterate is the one of a check after every step.
        int jj = 0, j0 = 0;
        bool done = false;
        for (int j = 0; j < m; ++j) {
            if (its + (j - j0) >= c->o.max_iter) break;
            cd* vj = c->dBasis + (size_t)j * B * M;
            cd* vn = c->dBasis + (size_t)(j + 1) * B * M;
            CHK(A(vj, c->dW));
            HIPCHK(launch_multidot(c->dBasis, j + 1, c->dW, M, B, c->dPart, c->dHp, m + 1, 0, st));
            HIPCHK(launch_multiaxpy(c->dBasis, j + 1, c->dHp, m + 1, -1.0, c->dW, M, B, st));
            HIPCHK(launch_multidot(c->dBasis, j + 1, c->dW, M, B, c->dPart, c->dHp2, m + 1, 0, st));
            HIPCHK(launch_multiaxpy(c->dBasis, j + 1, c->dHp2, m + 1, -1.0, c->dW, M, B, st));
            HIPCHK(launch_axpby(c->dHp, 1.0, c->dHp2, 1.0, c->dHp, (long)B * (m + 1), st));
            HIPCHK(launch_norm(c->dW, M, B, c->dPart, c->dNrm, st));
            HIPCHK(launch_scale(c->dW, c->dNrm, vn, M, B, nullptr, st));
            HIPCHK(launch_givens(j, m, B, c->dHp, c->dNrm, c->dH, c->dCs, c->dSn, c->dE, c->dBn,
                                 c->dResHist + (size_t)j * B, c->dAct, st));
            const int pending = j + 1 - j0;
            if (pending < c->gm_check && j < m - 1 && its + pending < c->o.max_iter) continue;
            HIPCHK(hipMemcpyAsync(c->hResHist.data(), c->dResHist + (size_t)j0 * B,
                                  sizeof(double) * B * pending, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int q = 0; q < pending && !done; ++q) {
                const double* r = c->hResHist.data() + (size_t)q * B;
                ++its;
                jj = j0 + q + 1;
                done = true;
                double worst = 0;
                for (int b = 0; b < B; ++b) {
                    // (inactive problems' slots are not written in this cycle)
                    if (c->hAct[b] && !std::isfinite(r[b])) return SWR_ENAN;
                    if (c->hAct[b] && r[b] > c->o.tol) done = false;
                    if (c->hAct[b]) worst = std::max(worst, r[b]);
                }
                c->hist.push_back(worst);
            }
            j0 = j + 1;
            if (done) break;
        }
        HIPCHK(launch_gmres_solve(jj, m, B, c->dH, c->dE, c->dY, c->dAct, st));
        HIPCHK(launch_multiaxpy(c->dBasis, jj, c->dY, m + 1, 1.0, x, M, B, st));
    }
    *iters_out = its;
    return conv ? SWR_OK : SWR_ENOCONV;
}

// BiCGStab (van der Vorst 1992) on A x = rhs for all problems of the batch,
// each with its own scalars; x starts at 0.  Stops per problem when
// ||r||_2 <= tol ||rhs||_2, checked on s after the half step and on r after
// the full step; finished problems keep their x (zero coefficients).
static swr_status run_bicgstab(swr_ctx* c, const Op& A, const cd* rhs, cd* x, int* iters_out,
                               double tol, int max_iter, bool record = true) {
    const int B = c->B;
    const long M = (long)c->ns * c->nt;
    const size_t vec = (size_t)B * M;
    hipStream_t st = c->st;
    if (!c->dBi) {
        ALLOC_LIVE(c->dBi, 6 * vec);
        ALLOC_LIVE(c->dCoef, (size_t)3 * B);
        ALLOC_LIVE(c->dDot, (size_t)B);
    }
    cd *r = c->dBi, *rh = r + vec, *p = rh + vec, *v = p + vec, *s = v + vec, *t = s + vec;
    std::vector<cd> coef(3 * (size_t)B), dot(B), rho(B, mk(1, 0)), alpha(B, mk(1, 0)), omega(B, mk(1, 0)),
        rho_new(B);
    std::vector<double> bn(B), nr(B);
    std::vector<char> act(B), half(B);
    auto dots = [&](const cd* u, const cd* w) -> swr_status {   // dot[b] = <u_b, w_b>
        HIPCHK(launch_multidot(u, 1, w, M, B, c->dPart, c->dDot, 1, 0, st));
        HIPCHK(hipMemcpyAsync(dot.data(), c->dDot, sizeof(cd) * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return SWR_OK;
    };
    auto norms = [&](const cd* w, std::vector<double>& out) -> swr_status {
        HIPCHK(launch_norm(w, M, B, c->dPart, c->dNrm, st));
        HIPCHK(hipMemcpyAsync(out.data(), c->dNrm, sizeof(double) * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return SWR_OK;
    };
    auto comb = [&](const cd* x0, const cd* x1, const cd* x2, cd* z) -> swr_status {
        HIPCHK(hipMemcpyAsync(c->dCoef, coef.data(), sizeof(cd) * 3 * B, hipMemcpyHostToDevice, st));
        HIPCHK(launch_lincomb(x0, x1, x2, c->dCoef, z, M, B, st));
        return SWR_OK;
    };
    auto set = [&](int b, cd a0, cd a1, cd a2) { coef[3 * b] = a0; coef[3 * b + 1] = a1; coef[3 * b + 2] = a2; };
    const cd one = mk(1, 0), zero = mk(0, 0);
    HIPCHK(hipMemsetAsync(x, 0, vec * sizeof(cd), st));
    HIPCHK(hipMemsetAsync(p, 0, vec * sizeof(cd), st));
    HIPCHK(hipMemsetAsync(v, 0, vec * sizeof(cd), st));
    HIPCHK(hipMemcpyAsync(r, rhs, vec * sizeof(cd), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(rh, rhs, vec * sizeof(cd), hipMemcpyDeviceToDevice, st));
    CHK(norms(rhs, bn));
    bool any = false;
    for (int b = 0; b < B; ++b) { act[b] = bn[b] > 0; any |= act[b] != 0; }
    int its = 0;
    while (any && its < max_iter) {
        ++its;
        CHK(dots(rh, r));
        for (int b = 0; b < B; ++b) {
            rho_new[b] = dot[b];
            if (act[b]) {
                const cd beta = (rho_new[b] * inv(rho[b])) * (alpha[b] * inv(omega[b]));
                set(b, one, beta, -(beta * omega[b]));
            } else {
                set(b, zero, one, zero);
            }
        }
        CHK(comb(r, p, v, p));                                   // p = r + beta (p - omega v)
        CHK(A(p, v));
        CHK(dots(rh, v));
        for (int b = 0; b < B; ++b) {
            alpha[b] = act[b] ? rho_new[b] * inv(dot[b]) : zero;
            set(b, one, -alpha[b], zero);
        }
        CHK(comb(r, v, nullptr, s));                             // s = r - alpha v
        CHK(norms(s, nr));
        for (int b = 0; b < B; ++b) {
            if (!std::isfinite(nr[b])) return SWR_ENAN;
            half[b] = act[b] && nr[b] <= tol * bn[b];
        }
        CHK(A(s, t));
        CHK(dots(t, s));
        std::vector<cd> ts = dot;
        CHK(dots(t, t));
        for (int b = 0; b < B; ++b) {
            omega[b] = (act[b] && !half[b]) ? ts[b] * inv(dot[b]) : zero;
            set(b, one, act[b] ? alpha[b] : zero, omega[b]);
        }
        CHK(comb(x, p, s, x));                                   // x += alpha p + omega s
        for (int b = 0; b < B; ++b) set(b, one, -omega[b], zero);
        CHK(comb(s, t, nullptr, r));                             // r = s - omega t
        CHK(norms(r, nr));
        any = false;
        double worst = 0;
        for (int b = 0; b < B; ++b) {
            if (!std::isfinite(nr[b])) return SWR_ENAN;
            if (act[b] && bn[b] > 0) worst = std::max(worst, (half[b] ? 0.0 : nr[b]) / bn[b]);
            if (half[b] || nr[b] <= tol * bn[b]) act[b] = 0;
            any |= act[b] != 0;
            rho[b] = rho_new[b];
        }
        if (record) c->hist.push_back(worst);
    }
    *iters_out = its;
    return any ? SWR_ENOCONV : SWR_OK;
}

// The causal solve needs the per-step block system (I - C_0) in a form it
// can solve quickly: block PCR on one wave or one workgroup, or a dense
// inverse for at most kDenseMaxSlots slots.  Beyond that it is not offered:
// (I - L) g = d is solved by BiCGStab on the same operator instead, and P^{-1}
// of the preconditioned iterations by an inner BiCGStab (the paper's own way
// of applying P^{-1}, Sec. 5) to a relative residual of kInnerTol.
constexpr int kDenseMaxSlots = 512;
constexpr double kInnerTol = 1e-13;
// internal status (never crosses the ABI): the causal solve is not offered
// for this system; the caller switches to BiCGStab
constexpr swr_status kCausalOff = static_cast<swr_status>(7);

// block PCR on one wave (fast) or on one workgroup (general)
static bool causal_fast_ok(const swr_ctx* c) { return c->ns <= kNearSlots && c->N - 1 <= kWave; }
static bool causal_gen_ok(const swr_ctx* c) {
    return c->N - 1 <= kGenMaxIf && gen_shm(c->N) <= 160 * 1024;
}

static bool causal_sized(const swr_ctx* c) {
    if (!c->L.dirty && c->L.path == 0 && c->vk == SWR_V_STATIC) return false;
    return causal_fast_ok(c) || causal_gen_ok(c) || c->ns <= kDenseMaxSlots;
}

static swr_status run_causal(swr_ctx* c, Iface& I, const cd* d, cd* g, hipStream_t st,
                             int n_lo, int n_hi);

// (I - L) g = d of the static potential by BiCGStab on the MFMA operator
static swr_status static_bicgstab(swr_ctx* c, const cd* d, cd* g, int* iters) {
    Op A = [c](const cd* x, cd* y) -> swr_status {
        LttArgs l = ltt_args(c, c->L, x, y);
        HIPCHK(launch_ltt(l, c->st));
        return SWR_OK;
    };
    return run_bicgstab(c, A, d, g, iters, c->o.tol, c->o.max_iter);
}

// x = (I - L_I)^{-1} rhs over the whole window: the causal solve, or an inner
// BiCGStab when the causal solve is not offered at this size
static swr_status apply_inverse(swr_ctx* c, Iface& I, const cd* rhs, cd* x) {
    if (causal_sized(c) && !(!I.dirty && I.path == 0)) {
        const swr_status rs = run_causal(c, I, rhs, x, c->st, 0, c->nt);
        if (rs != kCausalOff) return rs;
    }
    Op A = [c, &I](const cd* z, cd* y) -> swr_status {
        LttArgs l = ltt_args(c, I, z, y);
        HIPCHK(launch_ltt(l, c->st));
        return SWR_OK;
    };
    // the inner solve has its own cap (opts.max_iter bounds the outer
    // iteration): information crosses one interface per Krylov step, so it
    // needs a multiple of the interface count
    int its = 0;
    const int cap = std::max(c->o.max_iter, 20 * c->ns);
    const swr_status rs = run_bicgstab(c, A, rhs, x, &its, kInnerTol, cap, false);
    c->inner_iters += its;
    return rs == SWR_ENOCONV ? SWR_ENOCONV : rs;
}

// causal forward substitution in time for (I - L) g = d with the operator I
// (exact up to rounding).  Block PCR per step when the block system is
// certified diagonally dominant: on one wave for N - 1 <= 64 interfaces, on
// a workgroup up to kGenMaxIf; otherwise (at most kDenseMaxSlots slots) a
// dense (I - C_0)^{-1} by Gauss-Jordan with partial pivoting.
static swr_status run_causal(swr_ctx* c, Iface& I, const cd* d, cd* g, hipStream_t st,
                             int n_lo, int n_hi) {
    const int ns = c->ns, nt = c->nt, B = c->B, ni = c->N - 1;
    const bool fast_ok = causal_fast_ok(c);
    const bool gen_ok = causal_gen_ok(c);
    // the impulse responses were rebuilt from the same potential as at the
    // last set-up: same columns bit for bit, so the PCR records, the level
    // count and the path stay valid (no set-up kernels, no host read-back)
    const int ver = (&I == &c->L) ? c->v_version : 0;
    if (I.dirty && I.built_version == ver) I.dirty = false;
    if (I.dirty) {
        I.built_version = ver;
        I.path = 3;
        if (fast_ok || gen_ok) {
            const size_t rec = fast_ok ? causal_fast_rec() : (size_t)pcr_rec_gen(c->N);
            if (!I.pcr || I.pcr_size < rec * I.nv) {
                ALLOC_LIVE(I.pcr, rec * I.nv);
                I.pcr_size = rec * I.nv;
            }
            // eta[v][l]: ||D_l^{-1}|| (||L_l|| + ||U_l||) of the system before level l
            const int ld = fast_ok ? kPcrLevels + 1 : kGenLevelsMax + 1;
            const int L = fast_ok ? kPcrLevels : pcr_levels_for(ni);
            if (!I.eta) ALLOC_LIVE(I.eta, (size_t)I.nv * (kGenLevelsMax + 1));
            if (fast_ok) HIPCHK(launch_causal_pcr_setup(c->N, nt, I.nv, I.cols, I.pcr, I.eta, st));
            else HIPCHK(launch_causal_pcr_setup_gen(c->N, nt, I.nv, I.cols, I.pcr, I.eta, st));
            std::vector<double> eta((size_t)I.nv * ld);
            HIPCHK(hipMemcpyAsync(eta.data(), I.eta, sizeof(double) * eta.size(), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            // block diagonal dominance (eta_0 < 1) makes block PCR stable and
            // squares the coupling every level; levels past the first l with
            // eta_l <= 2^-60 change no FP64 result and are skipped
            bool ok = true;
            int lev = 0;
            for (int v = 0; v < I.nv; ++v) {
                const double* ev = eta.data() + (size_t)v * ld;
                ok = ok && std::isfinite(ev[0]) && ev[0] < 1.0;
                int lv = L;
                for (int l = 0; l <= L; ++l)
                    if (std::isfinite(ev[l]) && ev[l] <= kPcrNegligible) { lv = l; break; }
                lev = std::max(lev, lv);
            }
            I.levels = lev;
            I.eta0 = 0;
            for (int v = 0; v < I.nv; ++v) I.eta0 = std::max(I.eta0, eta[(size_t)v * ld]);
            if (ok) I.path = fast_ok ? 1 : 2;
        }
        // no dominance certificate and too many slots for a dense inverse
        if (I.path == 3 && ns > kDenseMaxSlots) I.path = 0;
        if (I.path == 3) {
            if (!I.Minv) {
                ALLOC_LIVE(I.Minv, (size_t)I.nv * ns * ns);
                ALLOC_LIVE(I.Mwork, (size_t)I.nv * ns * ns);
                ALLOC_LIVE(I.piv, I.nv);
            }
            HIPCHK(launch_c0_inverse(c->N, ns, nt, I.nv, I.cols, I.Mwork, I.Minv, I.piv, st));
        }
        I.dirty = false;
    }
    if (I.path == 0) return kCausalOff;
    if (I.path == 1 || I.path == 2) {
        const int tb = I.path == 1 ? kNearTb : gen_tb(c->N);
        if (!c->dBase || c->base_tb < tb) {
            ALLOC_LIVE(c->dBase, (size_t)B * ns * tb);
            c->base_tb = tb;
        }
        const int max_seg = (nt - 1) / kCausalSuper;
        if (!c->dFacc && max_seg > 0)
            ALLOC_LIVE(c->dFacc, (size_t)max_seg * B * ns * kCausalSuper);
        // super-blocks are the absolute windows [S, S + kCausalSuper); the
        // steps [a0, a1) of one of them take the contribution of the finished
        // super-blocks (steps < S) from one block-Toeplitz product, which
        // reads lags < a1 only (written once the impulse sweeps reach a1),
        // and the steps S <= s < n from the far kernel.  Where a call's range
        // starts or ends therefore changes no arithmetic.
        for (int a0 = n_lo; a0 < n_hi;) {
            const int S = a0 / kCausalSuper * kCausalSuper;
            const int a1 = std::min(n_hi, S + kCausalSuper);
            if (S > 0) {
                // one partial per finished super-block (split over the sources)
                LttArgs l{};
                l.N = c->N; l.nt = nt; l.ns = ns; l.B = B; l.per_problem = I.nv > 1;
                l.cols = I.cols; l.x = g; l.y = c->dFacc + (a0 - S); l.base = nullptr;
                l.sign = 1.0; l.n_lo = a0; l.n_hi = a1; l.s_lo = 0; l.s_hi = S;
                l.y_ld = kCausalSuper; l.s_seg = kCausalSuper;
                l.y_seg_stride = (size_t)B * ns * kCausalSuper;
                HIPCHK(launch_ltt(l, st));
            }
            const cd* facc = S > 0 ? c->dFacc : nullptr;
            if (I.path == 1)
                HIPCHK(launch_causal_fast(c->N, nt, ns, B, I.nv > 1, I.cols, I.pcr, I.levels, d,
                                          c->dBase, g, a0, a1, facc, S, st));
            else
                HIPCHK(launch_causal_gen(c->N, nt, ns, B, I.nv > 1, I.cols, I.pcr, I.levels, d,
                                         c->dBase, g, a0, a1, facc, S, st));
            a0 = a1;
        }
        return SWR_OK;
    }
    if (!c->dFar) ALLOC_LIVE(c->dFar, (size_t)B * ns * kCausalTb);
    for (int n0 = n_lo; n0 < n_hi; n0 += kCausalTb) {
        const int nb = std::min(kCausalTb, n_hi - n0);
        LttArgs l{};
        l.N = c->N; l.nt = nt; l.ns = ns; l.B = B; l.per_problem = I.nv > 1;
        l.cols = I.cols; l.x = g; l.y = c->dFar; l.base = nullptr; l.sign = 1.0;
        l.n_lo = n0; l.n_hi = n0 + nb; l.s_hi = n0; l.y_ld = kCausalTb;
        HIPCHK(launch_ltt(l, st));
        CausalArgs ca{};
        ca.N = c->N; ca.nt = nt; ca.ns = ns; ca.B = B; ca.per_problem = I.nv > 1;
        ca.n0 = n0; ca.nb = nb; ca.cols = I.cols; ca.Minv = I.Minv; ca.d = d;
        ca.far = c->dFar; ca.g = g;
        HIPCHK(launch_causal_block(ca, st));
    }
    return SWR_OK;
}

static swr_status read_max(swr_ctx* c, double* out) {
    unsigned long long bits = 0;
    HIPCHK(hipMemcpyAsync(&bits, c->dMax, sizeof(bits), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    std::memcpy(out, &bits, sizeof(double));
    return SWR_OK;
}

// classical algorithm: g <- R g until max |g^{k+1} - g^k| < tol (Sec. 4)
static swr_status run_classical(swr_ctx* c, const cd* u0, int* iters, double* last) {
    const size_t vec = (size_t)c->B * c->ns * c->nt;
    HIPCHK(hipMemsetAsync(c->dG, 0, vec * sizeof(cd), c->st));
    cd* gi = c->dG;
    cd* go = c->dG2;
    *last = INFINITY;
    swr_status rs = SWR_ENOCONV;
    for (int it = 1; it <= c->o.max_iter; ++it) {
        SweepIO io;
        io.u0 = u0; io.g_in = gi; io.g_out = go; io.maxdiff = true;
        CHK(run_sweeps(c, io));
        double d;
        CHK(read_max(c, &d));
        *last = d;
        *iters = it;
        c->hist.push_back(d);
        std::swap(gi, go);
        if (!std::isfinite(d)) return SWR_ENAN;
        if (d < c->o.tol) { rs = SWR_OK; break; }
    }
    if (gi != c->dG) HIPCHK(hipMemcpyAsync(c->dG, gi, vec * sizeof(cd), hipMemcpyDeviceToDevice, c->st));
    return rs;
}

// V(t,x): GMRES on (I - L) g = d with L x = R(x) - R(0) applied by one
// zero-data sweep (Sec. 4 "Classical algorithm, version 2"), right
// preconditioned by P = I - L_0 (Sec. 5, eq. chp2_algopd_Lpf) whose inverse is
// applied exactly by the causal solver.
static swr_status run_precond_time(swr_ctx* c, int* iters) {
    const size_t vec = (size_t)c->B * c->ns * c->nt;
    const bool pc = c->o.precond != 0;
    Op A = [c, pc, vec](const cd* z, cd* y) -> swr_status {
        const cd* w = z;
        if (pc) {
            CHK(apply_inverse(c, c->L0, z, c->dT1));
            w = c->dT1;
        }
        SweepIO io;
        io.g_in = w; io.g_out = c->dT2;
        CHK(run_sweeps(c, io));                                   // L w
        HIPCHK(launch_axpby(w, 1.0, c->dT2, -1.0, y, (long)vec, c->st));
        return SWR_OK;
    };
    HIPCHK(hipMemsetAsync(c->dG2, 0, vec * sizeof(cd), c->st));   // y (preconditioned unknown)
    swr_status rs = run_gmres(c, A, c->dD, c->dG2, iters);
    if (rs != SWR_OK && rs != SWR_ENOCONV) return rs;
    if (pc) CHK(apply_inverse(c, c->L0, c->dG2, c->dG));
    else HIPCHK(hipMemcpyAsync(c->dG, c->dG2, vec * sizeof(cd), hipMemcpyDeviceToDevice, c->st));
    return rs;
}

// |u|^2: preconditioned fixed point g <- g - P^{-1}(g - R_nl g) (Sec. 5,
// eq. chp2_algopd_NL read as in the surrounding text) until
// max |g^{k+1} - g^k| < tol.
static swr_status run_precond_cubic(swr_ctx* c, const cd* u0, int* iters, double* last) {
    const size_t vec = (size_t)c->B * c->ns * c->nt;
    const long M = (long)c->ns * c->nt;
    HIPCHK(hipMemsetAsync(c->dG, 0, vec * sizeof(cd), c->st));
    *last = INFINITY;
    for (int it = 1; it <= c->o.max_iter; ++it) {
        SweepIO io;
        io.u0 = u0; io.g_in = c->dG; io.g_out = c->dT2;
        CHK(run_sweeps(c, io));                                          // R_nl g
        HIPCHK(launch_axpby(c->dG, 1.0, c->dT2, -1.0, c->dT2, (long)vec, c->st));   // g - R_nl g
        const cd* z = c->dT2;
        if (c->o.precond) {
            CHK(apply_inverse(c, c->L0, c->dT2, c->dT1));
            z = c->dT1;
        }
        HIPCHK(launch_axpby(c->dG, 1.0, z, -1.0, c->dG, (long)vec, c->st));
        HIPCHK(launch_maxabs(z, M, c->B, c->dPart, c->dNrm, c->st));
        HIPCHK(launch_maxabs(c->dG, M, c->B, c->dPart, c->dBn, c->st));
        std::vector<double> m(c->B), gm(c->B);
        HIPCHK(hipMemcpyAsync(m.data(), c->dNrm, sizeof(double) * c->B, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipMemcpyAsync(gm.data(), c->dBn, sizeof(double) * c->B, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        // change relative to the size of the traces once they exceed 1 (they
        // scale like sqrt(2/dt) |v|, so an absolute bound can sit below FP64
        // resolution)
        double d = 0;
        for (int b = 0; b < c->B; ++b) d = std::max(d, m[b] / std::max(1.0, gm[b]));
        *last = d;
        *iters = it;
        c->hist.push_back(d);
        if (!std::isfinite(d)) return SWR_ENAN;
        if (d < c->o.tol) return SWR_OK;
    }
    return SWR_ENOCONV;
}

static double elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    hipEventElapsedTime(&ms, a, b);
    return ms;
}

// ---------------------------------------------------------------------------
// Static potential with the causal interface solve, pipelined in time.
// Every stage is causal: step n of the impulse responses and of d needs
// steps <= n of the build sweeps, g_n needs them and g_s for s < n, and step n
// of the final sweep needs g_s for s <= n.  The time window is cut into chunks
// of o.pipeline steps; chunk j of the build sweeps (stream st), of the
// interface solve (s2) and of the final sweep (s3) wait only for chunk j of
// the stage before, so the three stages run concurrently on different CUs.
// The sweeps carry their state between chunk launches (dStateB / dStateF)
// and keep their S0^2 boundary history in separate buffers.
// ---------------------------------------------------------------------------
struct PipeTimes {
    double build = 0, iface = 0, fin = 0, sweep_sum = 0;
    int n_sweep = 0;
};

static bool pipelined(const swr_ctx* c) {
    // (the long-chunk sweep runs the whole window in one launch)
    return c->vk == SWR_V_STATIC && c->o.solver == SWR_SOLVER_CAUSAL && c->pipe_chunk > 0 && !c->Qlong &&
           !c->o.plain && causal_sized(c) &&
           c->ns > 0 && c->nt > c->pipe_chunk;
}

static swr_status pipe_resources(swr_ctx* c, int K) {
    if (!c->s2) HIPCHK(hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking));
    if (!c->s3) HIPCHK(hipStreamCreateWithFlags(&c->s3, hipStreamNonBlocking));
    const size_t st_rec = (size_t)2 * c->P * kWave;
    if (!c->dStateB) ALLOC_LIVE(c->dStateB, (size_t)c->nBuild * st_rec);
    if (!c->dStateF) ALLOC_LIVE(c->dStateF, (size_t)c->nSub * st_rec);
    if (!c->dHistB && conv_hist(c->tr)) ALLOC_LIVE(c->dHistB, (size_t)c->nBuild * 2 * (c->nt + 1));
    if (c->tr >= SWR_P22) {
        if (!c->dPadeStB) ALLOC_LIVE(c->dPadeStB, (size_t)c->nBuild * 6 * kWave);
        if (!c->dPadeStF) ALLOC_LIVE(c->dPadeStF, (size_t)c->nSub * 6 * kWave);
    }
    // sync events: fork, build j, causal j, join; timing events: 2 per sweep
    // launch plus the two ends of the interface solve
    while ((int)c->evSync.size() < 2 * K + 2) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->evSync.push_back(e);
    }
    while ((int)c->evTime.size() < 4 * K + 2) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c->evTime.push_back(e);
    }
    return SWR_OK;
}

static swr_status run_static_pipelined(swr_ctx* c, const cd* u0, cd* g, const SweepIO& fin,
                                       PipeTimes* tm, bool timing = true) {
    const int nt = c->nt, ch = c->pipe_chunk;
    // chunk boundaries: a short first chunk (64 steps) so the interface solve
    // starts early, then multiples of ch up to nt.  (A short last chunk, so
    // that the final sweep would end sooner after the interface solve, cost
    // more in launches than it saved: 106.0 against 103.4 ms per
    // batched-uneven solve, 3.62 against 3.56 ms on static-packet.)
    std::vector<int> cut{0};
    auto push = [&](int x) { if (x > cut.back() && x < nt) cut.push_back(x); };
    push(kWave);
    for (int x = ch; x < nt; x += ch) push(x);
    cut.push_back(nt);
    const int K = (int)cut.size() - 1;
    CHK(pipe_resources(c, K));
    hipStream_t st = c->st, s2 = c->s2, s3 = c->s3;
    hipEvent_t* es = c->evSync.data();
    hipEvent_t* et = c->evTime.data();
    hipEvent_t ev_fork = es[0], ev_join = es[1];
    // fork: the side streams start after everything queued so far on st
    HIPCHK(hipEventRecord(ev_fork, st));
    HIPCHK(hipStreamWaitEvent(s2, ev_fork, 0));
    HIPCHK(hipStreamWaitEvent(s3, ev_fork, 0));

    SweepArgs ab = sweep_args(c, c->dBuild, c->nBuild, c->L.fac, c->L.cols);
    ab.u0 = u0;
    ab.g_in = c->dZero;
    ab.g_out = c->dD;
    ab.state = c->dStateB;
    ab.pstate = c->dPadeStB;
    if (c->dHistB) ab.hist = c->dHistB;
    SweepArgs af = sub_args(c, fin);
    af.state = c->dStateF;
    af.pstate = c->dPadeStF;
    c->L.dirty = true;
    int launches = 0;

    // stage 1: impulse + d sweeps, chunk by chunk on st
    for (int j = 0; j < K; ++j) {
        ab.n_begin = cut[j];
        ab.n_end = cut[j + 1];
        if (timing) HIPCHK(hipEventRecord(et[2 * j], st));
        HIPCHK(launch_widths(c, ab, SWR_V_STATIC, st, false, &launches));
        if (timing) HIPCHK(hipEventRecord(et[2 * j + 1], st));
        HIPCHK(hipEventRecord(es[2 + j], st));
    }
    // stage 2: causal interface solve on s2 (its set-up reads the first
    // step of the impulse responses, i.e. chunk 0), and stage 3: final sweep
    // on s3.  Chunk j of the final sweep is queued right after chunk j of
    // the interface solve: queued after all of stage 2, it would wait for
    // the host to issue every interface launch first.
    for (int j = 0; j < K; ++j) {
        HIPCHK(hipStreamWaitEvent(s2, es[2 + j], 0));
        if (timing && j == 0) HIPCHK(hipEventRecord(et[4 * K], s2));
        CHK(run_causal(c, c->L, c->dD, g, s2, cut[j], cut[j + 1]));
        HIPCHK(hipEventRecord(es[2 + K + j], s2));
        if (timing && j == K - 1) HIPCHK(hipEventRecord(et[4 * K + 1], s2));
        HIPCHK(hipStreamWaitEvent(s3, es[2 + K + j], 0));
        af.n_begin = cut[j];
        af.n_end = cut[j + 1];
        if (timing) HIPCHK(hipEventRecord(et[2 * K + 2 * j], s3));
        HIPCHK(launch_widths(c, af, c->vk, s3, false, &launches));
        if (timing) HIPCHK(hipEventRecord(et[2 * K + 2 * j + 1], s3));
    }
    if (fin.uT) HIPCHK(launch_finalize_ut(c->N, c->nx, c->B, c->dOff, c->dEnds, fin.uT, s3));
    if (fin.snaps)
        HIPCHK(launch_finalize_snaps(c->N, c->nx, c->B, nsnaps(c), c->dOff, c->dSnapEnds, fin.snaps, s3));
    // join back onto st
    HIPCHK(hipEventRecord(ev_join, s3));
    HIPCHK(hipStreamWaitEvent(st, ev_join, 0));
    if (tm && timing) {
        HIPCHK(hipEventSynchronize(ev_join));
        tm->build = elapsed(et[0], et[2 * K - 1]);
        tm->iface = elapsed(et[4 * K], et[4 * K + 1]);
        tm->fin = elapsed(et[2 * K], et[4 * K - 1]);
        tm->sweep_sum = 0;
        for (int j = 0; j < 2 * K; ++j) tm->sweep_sum += elapsed(et[2 * j], et[2 * j + 1]);
        tm->n_sweep = launches;
    }
    return SWR_OK;
}

// ---------------------------------------------------------------------------
// The static causal solve as one HIP graph (schedule option graph).  Once the
// causal set-up is cached (the second solve with the same potential), every
// step of the solve -- factorisation, impulse and d sweeps, causal interface
// solve, final sweep, the residual's norms -- is a kernel on the context's
// streams with no host decision in between, so it is captured once per set of
// output pointers and schedule and replayed; only the residual's read-back
// stays outside.  Same kernels, same arguments, same order: the replay is
// bitwise the uncaptured solve.  The graph holds kernels and event waits only
// (no memset or memcpy nodes).
// ---------------------------------------------------------------------------
static swr_ctx::GraphKey graph_key(const swr_ctx* c, const double* u0, double* uT, double* g,
                                   double* tr, double* sn) {
    return swr_ctx::GraphKey{u0, uT, g, tr, sn, c->pipe_chunk, c->help_max, c->pair_from, c->group,
                             c->v_version};
}

static bool graph_ready(const swr_ctx* c, const swr_ctx::GraphKey& key) {
    const bool shape = c->graph && c->vk == SWR_V_STATIC && c->o.solver == SWR_SOLVER_CAUSAL &&
                       !c->o.plain && c->ns > 0 && c->L.built_version == c->v_version &&
                       (c->L.path == 1 || c->L.path == 2 || c->L.path == 3);
    return shape && ((c->warm && key == c->warm_key) || (c->g_exec && key == c->g_key));
}

// everything of a static causal solve up to the residual's norms (dNrm, dBn)
static swr_status enqueue_static_causal(swr_ctx* c, const cd* u0, cd* uT, cd* g, cd* utrace, cd* snaps) {
    const size_t vec = (size_t)c->B * c->ns * c->nt;
    hipStream_t st = c->st;
    CHK(run_factor(c, c->dV, c->nv, c->L.fac));
    SweepIO io;
    io.u0 = u0; io.g_in = c->dG; io.g_out = c->dG2;
    io.uT = uT; io.trace = utrace; io.snaps = snaps;
    if (pipelined(c)) {
        CHK(run_static_pipelined(c, u0, c->dG, io, nullptr, false));
    } else {
        CHK(run_build(c, reinterpret_cast<const double*>(u0)));
        const swr_status rs = run_causal(c, c->L, c->dD, c->dG, st, 0, c->nt);
        if (rs != SWR_OK) return rs == kCausalOff ? SWR_EINVAL : rs;
        CHK(run_sweeps(c, io));
    }
    if (g) HIPCHK(launch_copy_cd(c->dG, g, vec, st));
    const long M = (long)c->ns * c->nt;
    HIPCHK(launch_axpby(c->dG, 1.0, c->dG2, -1.0, c->dT1, (long)vec, st));
    HIPCHK(launch_norm(c->dT1, M, c->B, c->dPart, c->dNrm, st));
    HIPCHK(launch_norm(c->dD, M, c->B, c->dPart, c->dBn, st));
    return SWR_OK;
}

static swr_status solve_graph(swr_ctx* c, const swr_ctx::GraphKey& key, const double* u0d, double* uT,
                              double* g, double* utrace, double* snaps, swr_info* info) {
    hipStream_t st = c->st;
    if (!c->g_exec || !(key == c->g_key)) {
        if (c->g_exec) { hipGraphExecDestroy(c->g_exec); c->g_exec = nullptr; }
        if (c->g_graph) { hipGraphDestroy(c->g_graph); c->g_graph = nullptr; }
        // captured on a stream of the context's own (the null stream cannot
        // be captured): every helper enqueues on c->st, so it points there
        // while the capture runs; nothing executes until the launch below
        if (!c->gs) HIPCHK(hipStreamCreateWithFlags(&c->gs, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(c->gs, hipStreamCaptureModeRelaxed));
        c->st = c->gs;
        const swr_status es = enqueue_static_causal(c, reinterpret_cast<const cd*>(u0d), reinterpret_cast<cd*>(uT),
                                                    reinterpret_cast<cd*>(g), reinterpret_cast<cd*>(utrace),
                                                    reinterpret_cast<cd*>(snaps));
        c->st = st;
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(c->gs, &graph);
        if (es != SWR_OK || ee != hipSuccess || !graph) {
            if (graph) hipGraphDestroy(graph);
            return es != SWR_OK ? es : SWR_EDEVICE;
        }
        if (hipGraphInstantiate(&c->g_exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(graph);
            c->g_exec = nullptr;
            return SWR_EDEVICE;
        }
        c->g_graph = graph;
        c->g_key = key;
    }
    HIPCHK(hipEventRecord(c->ev[0], st));
    HIPCHK(hipGraphLaunch(c->g_exec, st));
    HIPCHK(hipEventRecord(c->ev[4], st));
    std::vector<double> a(c->B), bnv(c->B);
    int nl[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(a.data(), c->dNrm, sizeof(double) * c->B, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(bnv.data(), c->dBn, sizeof(double) * c->B, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(nl, c->dNl, sizeof(nl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double res = 0;
    for (int b = 0; b < c->B; ++b) {
        const double r = bnv[b] > 0 ? a[b] / bnv[b] : a[b];
        if (!std::isfinite(r)) return SWR_ENAN;
        res = std::max(res, r);
    }
    c->hist.push_back(res);
    if (info) {
        // one pass, timed as a whole (no per-stage events inside the graph)
        *info = swr_info{};
        info->iters = 1;
        info->residual = res;
        info->nl_worst = nl[0];
        info->t_total_ms = elapsed(c->ev[0], c->ev[4]);
        info->history = c->hist.data();
        info->history_len = (int)c->hist.size();
    }
    return nl[1] ? SWR_ENOCONV : SWR_OK;
}

extern "C" swr_status swr_solve(swr_ctx* c, const double* u0d, double* uT, double* g, double* utrace,
                                double* snaps, swr_info* info) {
    if (!c || !u0d || !uT) return SWR_EINVAL;
    if (snaps && c->o.snapshot_stride <= 0) return SWR_EINVAL;
    if (snaps) {
        const size_t need = (size_t)c->B * nsnaps(c) * c->N * 2;
        if (c->snap_ends_size < need) {
            ALLOC_LIVE(c->dSnapEnds, need);
            c->snap_ends_size = need;
        }
    }
    c->hist.clear();
    c->n_launch_sweep = 0;
    const cd* u0 = reinterpret_cast<const cd*>(u0d);
    const size_t vec = (size_t)c->B * c->ns * c->nt;
    hipStream_t st = c->st;
    swr_status rs = SWR_OK;
    int iters = 0;
    double fixed_last = 0;
    c->inner_iters = 0;
    zero_ints_kernel<<<1, 2, 0, st>>>(c->dNl, 2);
    HIPCHK(hipGetLastError());
    const swr_ctx::GraphKey gkey = graph_key(c, u0d, uT, g, utrace, snaps);
    if (graph_ready(c, gkey)) return solve_graph(c, gkey, u0d, uT, g, utrace, snaps, info);
    HIPCHK(hipEventRecord(c->ev[0], st));
    // 1. assembly + factorisation
    if (c->vk == SWR_V_STATIC) CHK(run_factor(c, c->dV, c->nv, c->L.fac));
    else CHK(run_build_L0(c));   // zero-potential factors + impulses of L_0
    HIPCHK(hipEventRecord(c->ev[1], st));
    const bool fixed = c->vk == SWR_V_STATIC && c->o.solver == SWR_SOLVER_FIXED;
    PipeTimes tm;
    const bool pipe = pipelined(c);
    if (pipe) {
        // 2-4 overlapped in time: build sweeps, causal solve, final sweep
        SweepIO io;
        io.u0 = u0; io.g_in = c->dG; io.g_out = c->dG2;
        io.uT = reinterpret_cast<cd*>(uT); io.trace = reinterpret_cast<cd*>(utrace);
        io.snaps = reinterpret_cast<cd*>(snaps);
        const swr_status ps = run_static_pipelined(c, u0, c->dG, io, info ? &tm : nullptr);
        if (ps == kCausalOff) {
            // the causal solve turned out not to be offered for this system
            // (found once the first impulse responses existed): let the
            // streams drain, then solve again in the staged form
            if (c->s2) HIPCHK(hipStreamSynchronize(c->s2));
            if (c->s3) HIPCHK(hipStreamSynchronize(c->s3));
            HIPCHK(hipStreamSynchronize(st));
            return swr_solve(c, u0d, uT, g, utrace, snaps, info);
        }
        CHK(ps);
        iters = 1;
        HIPCHK(hipEventRecord(c->ev[2], st));
        HIPCHK(hipEventRecord(c->ev[3], st));
        HIPCHK(hipEventRecord(c->ev[4], st));
    } else {
    // 2. explicit interface problem (static V) or d = R 0
    if (c->vk == SWR_V_STATIC) {
        if (!fixed) CHK(run_build(c, u0d));
    } else {
        SweepIO io;
        io.u0 = u0; io.g_out = c->dD;
        CHK(run_sweeps(c, io));
    }
    HIPCHK(hipEventRecord(c->ev[2], st));
    // 3. interface solve
    if (c->ns == 0) {
        rs = SWR_OK;
    } else if (c->vk == SWR_V_TIME) {
        rs = run_precond_time(c, &iters);
    } else if (c->vk == SWR_V_CUBIC) {
        rs = run_precond_cubic(c, u0, &iters, &fixed_last);
    } else if (fixed) {
        rs = run_classical(c, u0, &iters, &fixed_last);
    } else if (c->o.solver == SWR_SOLVER_GMRES) {
        HIPCHK(hipMemsetAsync(c->dG, 0, vec * sizeof(cd), st));
        Op A = [c](const cd* x, cd* y) -> swr_status {
            LttArgs l = ltt_args(c, c->L, x, y);
            HIPCHK(launch_ltt(l, c->st));
            return SWR_OK;
        };
        rs = run_gmres(c, A, c->dD, c->dG, &iters);
    } else if (c->o.solver == SWR_SOLVER_BICGSTAB ||
               (c->o.solver == SWR_SOLVER_CAUSAL && !causal_sized(c))) {
        // (the causal solve is not offered at this many interfaces: the same
        // system by BiCGStab)
        Op A = [c](const cd* x, cd* y) -> swr_status {
            LttArgs l = ltt_args(c, c->L, x, y);
            HIPCHK(launch_ltt(l, c->st));
            return SWR_OK;
        };
        rs = run_bicgstab(c, A, c->dD, c->dG, &iters, c->o.tol, c->o.max_iter);
    } else if (c->o.solver == SWR_SOLVER_CAUSAL) {
        rs = run_causal(c, c->L, c->dD, c->dG, c->st, 0, c->nt);
        iters = 1;
        if (rs == kCausalOff) rs = static_bicgstab(c, c->dD, c->dG, &iters);
    } else {
        return SWR_EINVAL;
    }
    if (rs != SWR_OK && rs != SWR_ENOCONV) return rs;
    HIPCHK(hipEventRecord(c->ev[3], st));
    // 4. final sweep: u(T) and R g
    {
        SweepIO io;
        io.u0 = u0; io.g_in = c->ns ? c->dG : nullptr; io.g_out = c->dG2;
        io.uT = reinterpret_cast<cd*>(uT); io.trace = reinterpret_cast<cd*>(utrace);
        io.snaps = reinterpret_cast<cd*>(snaps);
        CHK(run_sweeps(c, io));
    }
    HIPCHK(hipEventRecord(c->ev[4], st));
    }
    if (g && vec) HIPCHK(hipMemcpyAsync(g, c->dG, vec * sizeof(cd), hipMemcpyDeviceToDevice, st));
    // certified residual ||g - R g|| / ||R 0|| (R 0 = d; the classical
    // algorithm reports its last change instead)
    double res = 0;
    if (c->ns > 0) {
        const long M = (long)c->ns * c->nt;
        if (!fixed) {
            HIPCHK(launch_axpby(c->dG, 1.0, c->dG2, -1.0, c->dT1, (long)vec, st));
            HIPCHK(launch_norm(c->dT1, M, c->B, c->dPart, c->dNrm, st));
            HIPCHK(launch_norm(c->dD, M, c->B, c->dPart, c->dBn, st));
            std::vector<double> a(c->B), bnv(c->B);
            HIPCHK(hipMemcpyAsync(a.data(), c->dNrm, sizeof(double) * c->B, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(bnv.data(), c->dBn, sizeof(double) * c->B, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int b = 0; b < c->B; ++b) {
                const double r = bnv[b] > 0 ? a[b] / bnv[b] : a[b];
                if (!std::isfinite(r)) return SWR_ENAN;
                res = r > res ? r : res;
            }
        } else {
            res = fixed_last;
        }
    }
    int nl[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(nl, c->dNl, sizeof(nl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (info) {
        *info = swr_info{};
        info->iters = iters;
        info->residual = res;
        info->t_factor_ms = elapsed(c->ev[0], c->ev[1]);
        info->t_build_ms = elapsed(c->ev[1], c->ev[2]);
        info->t_iface_ms = elapsed(c->ev[2], c->ev[3]);
        info->t_final_ms = elapsed(c->ev[3], c->ev[4]);
        info->nl_worst = nl[0];
        info->t_total_ms = elapsed(c->ev[0], c->ev[4]);
        info->t_sweep_ms = 0;
        info->n_sweep = 0;
        info->inner_iters = c->inner_iters;
        // Krylov and fixed-point solvers recorded every iteration; the
        // causal solve (one pass) has the certified residual
        if (c->hist.empty()) c->hist.push_back(res);
        info->history = c->hist.data();
        info->history_len = (int)c->hist.size();
        if (pipe) {
            info->t_build_ms = tm.build;
            info->t_iface_ms = tm.iface;
            info->t_final_ms = tm.fin;
            info->t_sweep_ms = tm.sweep_sum;
            info->n_sweep = tm.n_sweep;
        } else if (c->vk == SWR_V_STATIC && !fixed) {
            info->t_sweep_ms = info->t_build_ms + info->t_final_ms;
            info->n_sweep = c->n_launch_sweep;
        }
    }
    if (nl[1]) return SWR_ENOCONV;
    if (rs == SWR_OK && c->vk == SWR_V_STATIC && c->o.solver == SWR_SOLVER_CAUSAL) {
        c->warm_key = gkey;
        c->warm = true;
    }
    return rs;
}

extern "C" swr_status swr_apply_R(swr_ctx* c, const double* u0, const double* g_in, double* g_out,
                                  double* uT, double* maxdiff) {
    if (!c || !g_in || !g_out) return SWR_EINVAL;
    if (c->vk == SWR_V_STATIC) CHK(run_factor(c, c->dV, c->nv, c->L.fac));
    else CHK(run_factor(c, nullptr, 1, c->L0.fac));
    SweepIO io;
    io.u0 = reinterpret_cast<const cd*>(u0);
    io.g_in = reinterpret_cast<const cd*>(g_in);
    io.g_out = reinterpret_cast<cd*>(g_out);
    io.uT = reinterpret_cast<cd*>(uT);
    io.maxdiff = maxdiff != nullptr;
    CHK(run_sweeps(c, io));
    if (maxdiff) CHK(read_max(c, maxdiff));
    HIPCHK(hipStreamSynchronize(c->st));
    return SWR_OK;
}

extern "C" swr_status swr_apply_R_noalloc(swr_ctx* c, const double* u0, const double* g_in,
                                          double* g_out, double* uT, double* maxdiff) {
    if (!c || !g_in || !g_out) return SWR_EINVAL;
    if (!c->scratch) return SWR_EDEVICE;
    // scratch layout: [max word, padded to 256 B][ends B*N*2][history nSub*2*(nt+1)]
    const size_t ends = (size_t)c->B * c->N * 2;
    const size_t hist = conv_hist(c->tr) ? (size_t)c->nSub * 2 * (c->nt + 1) : 0;
    if (256 + (ends + hist) * sizeof(cd) > kScratchBytes) return SWR_EINVAL;
    unsigned char* base = static_cast<unsigned char*>(c->scratch);
    auto* word = reinterpret_cast<unsigned long long*>(base);
    cd* dEnds = reinterpret_cast<cd*>(base + 256);
    cd* dHist = dEnds + ends;
    if (c->vk == SWR_V_STATIC) CHK(run_factor(c, c->dV, c->nv, c->L.fac));
    else CHK(run_factor(c, nullptr, 1, c->L0.fac));
    SweepIO io;
    io.u0 = reinterpret_cast<const cd*>(u0);
    io.g_in = reinterpret_cast<const cd*>(g_in);
    io.g_out = reinterpret_cast<cd*>(g_out);
    io.uT = reinterpret_cast<cd*>(uT);
    io.maxdiff = maxdiff != nullptr;
    SweepArgs a = sub_args(c, io);
    a.hist = dHist;
    a.ends = dEnds;
    a.maxdiff = word;
    // the max-change word starts at zero (a kernel, not a memset: capturable)
    if (maxdiff) {
        zero_word_kernel<<<1, 1, 0, c->st>>>(word);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(launch_widths(c, a, c->vk, c->st, c->o.plain));
    if (uT) HIPCHK(launch_finalize_ut(c->N, c->nx, c->B, c->dOff, dEnds, io.uT, c->st));
    if (maxdiff) {
        word_to_double_kernel<<<1, 1, 0, c->st>>>(word, maxdiff);
        HIPCHK(hipGetLastError());
    }
    return SWR_OK;
}

// ---------------------------------------------------------------------------
// Schedule tuning.  The schedule parameters change no arithmetic of any
// result (the pipelined and staged solves, and both sweep workgroup forms,
// are bitwise equal; the GMRES restart changes the iterate, not the
// tolerance it meets): pipeline chunk of the static causal solve, the task
// bound of the S0^2 helper wave, the GMRES restart.  swr_tune times candidate
// schedules on the caller's input and keeps the fastest; the tuning cache
// (opts.tune_cache, a text file of "key value..." lines) remembers it per
// problem shape so a later swr_setup starts from it.
// ---------------------------------------------------------------------------
static std::string schedule_key(const swr_ctx* c) {
    uint64_t h = 1469598103934665603ull;                 // FNV-1a over the subdomain sizes
    for (int j : c->J) {
        for (int b = 0; b < 4; ++b) { h ^= (uint64_t)((j >> (8 * b)) & 0xff); h *= 1099511628211ull; }
    }
    std::ostringstream k;
    k << "N" << c->N << "_nt" << c->nt << "_B" << c->B << "_nv" << c->nv << "_vk" << c->vk << "_tr"
      << c->tr << "_solver" << c->o.solver;
    if (c->tr >= SWR_P22) k << "_m" << c->o.pade_m;
    k << "_J" << std::hex << h;
    return k.str();
}

static void load_schedule(swr_ctx* c, const char* path) {
    std::ifstream f(path);
    if (!f) return;
    const std::string key = schedule_key(c);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string k;
        int pipe = 0, help = 0, restart = 0, pair = 0;
        if (!(in >> k >> pipe >> help >> restart >> pair) || k != key) continue;
        if (pipe < 0 || (pipe > 0 && pipe % kWave != 0) || help < 0 || restart < 1 || pair < 1) continue;
        // then "graph check group ms"; lines written before those options
        // have "graph check ms", "graph ms" or "ms" alone
        std::vector<std::string> rest;
        for (std::string t; in >> t;) rest.push_back(t);
        c->pipe_chunk = pipe;
        c->help_max = help;
        c->o.restart = restart;
        c->pair_from = pair;
        c->graph = rest.size() >= 2 && rest[0] == "1" ? 1 : 0;
        if (rest.size() >= 3) {
            const int chk = std::atoi(rest[1].c_str());
            if (chk >= 1) c->gm_check = chk;
        }
        if (rest.size() >= 4) {
            const int grp = std::atoi(rest[2].c_str());
            if (grp >= 1 && grp <= kGroupMax) c->group = grp;
        }
    }
}

static bool store_schedule(const swr_ctx* c, const char* path, double ms) {
    const std::string key = schedule_key(c);
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        while (f && std::getline(f, line)) {
            std::istringstream in(line);
            std::string k;
            if ((in >> k) && k == key) continue;
            if (!line.empty()) keep.push_back(line);
        }
    }
    std::ofstream f(path, std::ios::trunc);
    if (!f) return false;
    for (const auto& l : keep) f << l << "\n";
    f << key << " " << c->pipe_chunk << " " << c->help_max << " " << c->o.restart << " " << c->pair_from
      << " " << c->graph << " " << c->gm_check << " " << c->group << " " << ms << "\n";
    return (bool)f;
}

extern "C" swr_status swr_tune(swr_ctx* c, const double* u0, double budget_ms, swr_schedule* chosen) {
    if (!c || !u0 || !(budget_ms > 0)) return SWR_EINVAL;
    if (!c->dUT) ALLOC_LIVE(c->dUT, (size_t)c->B * c->nx);
    double* uT = reinterpret_cast<double*>(c->dUT);
    // candidate values (the current schedule first)
    std::vector<int> pipes{c->pipe_chunk}, helps{c->help_max}, restarts{c->o.restart}, pairs{c->pair_from},
        graphs{c->graph}, checks{c->gm_check}, groups{c->group};
    if (c->vk == SWR_V_STATIC && c->tr <= SWR_S02)
        for (int g : {1, 2, 4, 8})
            if (std::find(groups.begin(), groups.end(), g) == groups.end()) groups.push_back(g);
    if (c->o.solver == SWR_SOLVER_GMRES || c->vk == SWR_V_TIME)
        for (int q : {1, 4, 16})
            if (std::find(checks.begin(), checks.end(), q) == checks.end()) checks.push_back(q);
    if (c->vk == SWR_V_STATIC && c->o.solver == SWR_SOLVER_CAUSAL) graphs.push_back(1 - c->graph);
    if (c->vk == SWR_V_STATIC && c->o.solver == SWR_SOLVER_CAUSAL)
        for (int p : {0, 128, 256, 512, 1024})
            if (p < c->nt && std::find(pipes.begin(), pipes.end(), p) == pipes.end()) pipes.push_back(p);
    if (c->tr == SWR_S02)
        for (int h : {0, kHelpMaxTasks, 1 << 30})
            if (std::find(helps.begin(), helps.end(), h) == helps.end()) helps.push_back(h);
    if (c->o.solver == SWR_SOLVER_GMRES || c->vk == SWR_V_TIME)
        for (int m : {20, 30, 60, 120})
            if (std::find(restarts.begin(), restarts.end(), m) == restarts.end()) restarts.push_back(m);
    if (c->vk == SWR_V_STATIC && c->tr <= SWR_S02)
        for (int w : {1, 4, kMaxP + 1})
            if (std::find(pairs.begin(), pairs.end(), w) == pairs.end()) pairs.push_back(w);
    const int p0 = c->pipe_chunk, h0 = c->help_max, m0 = c->o.restart, w0 = c->pair_from, q0 = c->graph,
              k0 = c->gm_check, g0 = c->group;
    double best = INFINITY;
    int bp = p0, bh = h0, bm = m0, bw = w0, bq = q0, bk = k0, bg = g0, tried = 0;
    double spent = 0;
    auto t_now = [] { return std::chrono::steady_clock::now(); };
    const auto t_start = t_now();
    for (int m : restarts)
        for (int kc : checks)
        for (int gz : groups)
        for (int w : pairs)
        for (int q : graphs)
        for (int p : pipes)
            for (int h : helps) {
                if (tried > 0 && spent > budget_ms) break;
                c->pipe_chunk = p;
                c->help_max = h;
                c->o.restart = m;
                c->pair_from = w;
                c->graph = q;
                c->gm_check = kc;
                c->group = gz;
                // warm-up (with a graph: the uncaptured solve, then the capture)
                swr_status rs = swr_solve(c, u0, uT, nullptr, nullptr, nullptr, nullptr);
                if (rs == SWR_OK && q) rs = swr_solve(c, u0, uT, nullptr, nullptr, nullptr, nullptr);
                if (rs != SWR_OK) continue;
                double ms = INFINITY;
                for (int r = 0; r < 2; ++r) {
                    HIPCHK(hipStreamSynchronize(c->st));
                    const auto t0 = t_now();
                    rs = swr_solve(c, u0, uT, nullptr, nullptr, nullptr, nullptr);
                    HIPCHK(hipStreamSynchronize(c->st));
                    if (rs != SWR_OK) break;
                    ms = std::min(ms, std::chrono::duration<double, std::milli>(t_now() - t0).count());
                }
                ++tried;
                if (ms < best) { best = ms; bp = p; bh = h; bm = m; bw = w; bq = q; bk = kc; bg = gz; }
                spent = std::chrono::duration<double, std::milli>(t_now() - t_start).count();
            }
    c->pipe_chunk = bp;
    c->help_max = bh;
    c->o.restart = bm;
    c->pair_from = bw;
    c->graph = bq;
    c->gm_check = bk;
    c->group = bg;
    if (chosen) {
        chosen->pipeline = bp;
        chosen->help_max = bh;
        chosen->restart = bm;
        chosen->pair_from = bw;
        chosen->graph = bq;
        chosen->check = bk;
        chosen->group = bg;
        chosen->ms = best;
        chosen->candidates = tried;
    }
    if (!std::isfinite(best)) return SWR_ENOCONV;
    if (!c->cache_path.empty() && !store_schedule(c, c->cache_path.c_str(), best)) return SWR_EINVAL;
    return SWR_OK;
}

extern "C" swr_status swr_set_schedule(swr_ctx* c, const swr_schedule* s) {
    if (!c || !s) return SWR_EINVAL;
    if (s->pipeline < 0 || (s->pipeline > 0 && s->pipeline % kWave != 0) || s->help_max < 0 ||
        s->restart < 1 || s->pair_from < 1 || s->check < 1 || s->group < 1 || s->group > kGroupMax)
        return SWR_EINVAL;
    c->pipe_chunk = s->pipeline;
    c->help_max = s->help_max;
    c->o.restart = s->restart;
    c->pair_from = s->pair_from;
    c->graph = s->graph ? 1 : 0;
    c->gm_check = s->check;
    c->group = s->group;
    return SWR_OK;
}

extern "C" swr_status swr_get_schedule(const swr_ctx* c, swr_schedule* s) {
    if (!c || !s) return SWR_EINVAL;
    s->pipeline = c->pipe_chunk;
    s->help_max = c->help_max;
    s->restart = c->o.restart;
    s->pair_from = c->pair_from;
    s->graph = c->graph;
    s->check = c->gm_check;
    s->group = c->group;
    s->ms = 0;
    s->candidates = 0;
    return SWR_OK;
}

extern "C" swr_status swr_build_interface(swr_ctx* c, const double* u0, double* cols, double* d) {
    if (!c || !u0) return SWR_EINVAL;
    if (c->vk == SWR_V_STATIC) {
        CHK(run_factor(c, c->dV, c->nv, c->L.fac));
        CHK(run_build(c, u0));
        if (cols) HIPCHK(hipMemcpyAsync(cols, c->L.cols, (size_t)c->nv * c->N * 4 * c->nt * sizeof(cd),
                                        hipMemcpyDeviceToDevice, c->st));
    } else {
        // the operator that exists for a general potential is L_0 (Sec. 5)
        CHK(run_build_L0(c));
        SweepIO io;
        io.u0 = reinterpret_cast<const cd*>(u0); io.g_out = c->dD;
        CHK(run_sweeps(c, io));
        if (cols) HIPCHK(hipMemcpyAsync(cols, c->L0.cols, (size_t)c->N * 4 * c->nt * sizeof(cd),
                                        hipMemcpyDeviceToDevice, c->st));
    }
    if (d) HIPCHK(hipMemcpyAsync(d, c->dD, (size_t)c->B * c->ns * c->nt * sizeof(cd),
                                 hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return SWR_OK;
}

extern "C" swr_status swr_set_potential(swr_ctx* c, const double* V) {
    if (!c || !V || c->vk == SWR_V_CUBIC || !c->dV) return SWR_EINVAL;
    const size_t vn = (c->vk == SWR_V_TIME) ? (size_t)c->nx * (c->nt + 1)
                                            : (size_t)c->nx * (c->o.v_per_problem ? c->B : 1);
    HIPCHK(hipMemcpyAsync(c->dV, V, vn * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    c->L.dirty = true;
    ++c->v_version;
    return SWR_OK;
}

extern "C" swr_status swr_interface_matvec(swr_ctx* c, const double* x, double* y) {
    if (!c || !x || !y) return SWR_EINVAL;
    Iface& I = c->vk == SWR_V_STATIC ? c->L : c->L0;
    LttArgs l = ltt_args(c, I, reinterpret_cast<const cd*>(x), reinterpret_cast<cd*>(y));
    HIPCHK(launch_ltt(l, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return SWR_OK;
}

// the interface solve of (I - L) g = d with the configured solver
static swr_status solve_interface(swr_ctx* c, const cd* d, cd* g, int* iters) {
    const size_t vec = (size_t)c->B * c->ns * c->nt;
    if (c->ns == 0) return SWR_OK;
    if (c->o.solver == SWR_SOLVER_GMRES) {
        HIPCHK(hipMemsetAsync(g, 0, vec * sizeof(cd), c->st));
        Op A = [c](const cd* x, cd* y) -> swr_status {
            LttArgs l = ltt_args(c, c->L, x, y);
            HIPCHK(launch_ltt(l, c->st));
            return SWR_OK;
        };
        return run_gmres(c, A, d, g, iters);
    }
    if (c->o.solver == SWR_SOLVER_BICGSTAB || !causal_sized(c)) {
        Op A = [c](const cd* x, cd* y) -> swr_status {
            LttArgs l = ltt_args(c, c->L, x, y);
            HIPCHK(launch_ltt(l, c->st));
            return SWR_OK;
        };
        return run_bicgstab(c, A, d, g, iters, c->o.tol, c->o.max_iter);
    }
    *iters = 1;
    const swr_status rs = run_causal(c, c->L, d, g, c->st, 0, c->nt);
    return rs == kCausalOff ? static_bicgstab(c, d, g, iters) : rs;
}

static AdjArgs adj_args(swr_ctx* c) {
    AdjArgs a{};
    a.N = c->N; a.nt = c->nt; a.B = c->B; a.nx = c->nx; a.ns = c->ns; a.ntasks = c->nSub;
    a.P = c->P; a.Jc = c->Jc;
    a.kappa = c->h / (3.0 * c->dt);
    a.h = c->h;
    a.sigma = c->sigma;
    a.c2 = c->c2;
    a.J = c->dJ; a.off = c->dOff; a.tasks = c->dSub; a.fac = c->L.fac; a.beta = c->dBeta;
    a.hist = c->dHist2;
    a.ckpt = c->dCkpt; a.g_fwd = c->dGfwd; a.hist_fwd = c->dHist; a.seg = c->dSeg;
    a.gends = c->dGends; a.wends = c->dWends;
    a.task0 = 0;
    a.pstride = c->P;
    a.fstride = (size_t)fac_fields(c->P) * kWave;
    return a;
}

// the adjoint sweep over every (problem, subdomain), one launch per chunk width
static hipError_t launch_adjoint_widths(const swr_ctx* c, AdjArgs a, hipStream_t st) {
    for (const WidthRun& r : c->runs_sub) {
        a.P = r.P;
        a.task0 = r.start;
        a.ntasks = r.count;
        const hipError_t e = launch_adjoint(a, ktr(c), st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

extern "C" swr_status swr_grad(swr_ctx* c, const double* u0d, const double* gbar, double* dJdV,
                               double* dJdu0, swr_info* info) {
    if (!c || !u0d || !gbar || !dJdV || !dJdu0) return SWR_EINVAL;
    if (c->vk != SWR_V_STATIC || c->o.solver == SWR_SOLVER_FIXED || c->o.checkpoint_K != kWave)
        return SWR_EINVAL;
    if (c->tr > SWR_S02) return SWR_EINVAL;   // adjoint provided for Robin and S0^2
    if (c->Qlong) return SWR_EINVAL;          // ... and subdomains of at most 64 * kMaxP nodes
    const cd* u0 = reinterpret_cast<const cd*>(u0d);
    const size_t vec = (size_t)c->B * c->ns * c->nt;
    hipStream_t st = c->st;
    if (!c->dCkpt) {
        c->Jc = (c->nt + kWave - 1) / kWave;
        ALLOC_LIVE(c->dCkpt, (size_t)c->nSub * (c->Jc + 1) * c->P * kWave);
        ALLOC_LIVE(c->dSeg, (size_t)c->nSub * kWave * c->P * kWave);
        ALLOC_LIVE(c->dHist2, (size_t)c->nSub * 2 * (c->nt + 1));
        ALLOC_LIVE(c->dGfwd, vec);
        ALLOC_LIVE(c->dDadj, vec);
        ALLOC_LIVE(c->dGadj, vec);
        ALLOC_LIVE(c->dGends, (size_t)c->B * c->N * 2);
        ALLOC_LIVE(c->dWends, (size_t)c->B * c->N * 2);
        ALLOC_LIVE(c->dUT, (size_t)c->B * c->nx);
    }
    int it_f = 0, it_b = 0;
    // ---- forward: factor, impulses + d, interface solve, final sweep with
    //      checkpoints (the S0^2 boundary history of this sweep stays in dHist)
    HIPCHK(hipEventRecord(c->ev[0], st));
    CHK(run_factor(c, c->dV, c->nv, c->L.fac));
    swr_status rf = SWR_OK;
    if (pipelined(c)) {
        SweepIO io;
        io.u0 = u0; io.g_in = c->dGfwd; io.g_out = c->dG2; io.uT = c->dUT;
        io.ckpt = true;
        const swr_status ps = run_static_pipelined(c, u0, c->dGfwd, io, nullptr);
        if (ps == kCausalOff) {
            if (c->s2) HIPCHK(hipStreamSynchronize(c->s2));
            if (c->s3) HIPCHK(hipStreamSynchronize(c->s3));
            HIPCHK(hipStreamSynchronize(st));
            return swr_grad(c, u0d, gbar, dJdV, dJdu0, info);
        }
        CHK(ps);
        it_f = 1;
    } else {
        CHK(run_build(c, u0d));
        rf = solve_interface(c, c->dD, c->dGfwd, &it_f);
        if (rf != SWR_OK && rf != SWR_ENOCONV) return rf;
        SweepIO io;
        io.u0 = u0; io.g_in = c->ns ? c->dGfwd : nullptr; io.g_out = c->dG2; io.uT = c->dUT;
        io.ckpt = true;
        CHK(run_sweeps(c, io));
    }
    HIPCHK(hipEventRecord(c->ev[1], st));
    // ---- adjoint: d of the adjoint interface problem (dual data, zero fluxes)
    AdjArgs a = adj_args(c);
    a.gbar = reinterpret_cast<const cd*>(gbar);
    a.g_in = nullptr;
    a.g_out = c->ns ? c->dDadj : nullptr;
    a.grad = 0;
    HIPCHK(launch_adjoint_widths(c, a, st));
    HIPCHK(hipEventRecord(c->ev[2], st));
    c->hist.clear();   // the history reported is the adjoint interface solve's
    swr_status rb = solve_interface(c, c->dDadj, c->dGadj, &it_b);
    if (rb != SWR_OK && rb != SWR_ENOCONV) return rb;
    HIPCHK(hipEventRecord(c->ev[3], st));
    // ---- adjoint final sweep with forward replay and dJ/dV accumulation
    a.g_in = c->ns ? c->dGadj : nullptr;
    a.g_out = c->ns ? c->dT1 : nullptr;
    a.grad = 1;
    a.dV = dJdV;
    a.du0 = reinterpret_cast<cd*>(dJdu0);
    HIPCHK(launch_adjoint_widths(c, a, st));
    HIPCHK(launch_finalize_grad(c->N, c->nx, c->B, c->dOff, c->dGends, c->dWends, dJdV,
                                reinterpret_cast<cd*>(dJdu0), st));
    HIPCHK(hipEventRecord(c->ev[4], st));
    // certified residual of the adjoint interface problem
    double res = 0;
    if (c->ns > 0) {
        const long M = (long)c->ns * c->nt;
        HIPCHK(launch_axpby(c->dGadj, 1.0, c->dT1, -1.0, c->dT2, (long)vec, st));
        HIPCHK(launch_norm(c->dT2, M, c->B, c->dPart, c->dNrm, st));
        HIPCHK(launch_norm(c->dDadj, M, c->B, c->dPart, c->dBn, st));
        std::vector<double> x(c->B), y(c->B);
        HIPCHK(hipMemcpyAsync(x.data(), c->dNrm, sizeof(double) * c->B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(y.data(), c->dBn, sizeof(double) * c->B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int b = 0; b < c->B; ++b) {
            const double r = y[b] > 0 ? x[b] / y[b] : x[b];
            if (!std::isfinite(r)) return SWR_ENAN;
            res = std::max(res, r);
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    if (info) {
        *info = swr_info{};
        info->iters = it_b;
        info->residual = res;
        info->t_factor_ms = elapsed(c->ev[0], c->ev[1]);   // the whole forward solve
        info->t_build_ms = elapsed(c->ev[1], c->ev[2]);    // adjoint d sweep
        info->t_iface_ms = elapsed(c->ev[2], c->ev[3]);    // adjoint interface solve
        info->t_final_ms = elapsed(c->ev[3], c->ev[4]);    // replay + adjoint sweep + dJ/dV
        info->nl_worst = it_f;
        if (c->hist.empty()) c->hist.push_back(res);
        info->history = c->hist.data();
        info->history_len = (int)c->hist.size();
    }
    return (rf == SWR_ENOCONV || rb == SWR_ENOCONV) ? SWR_ENOCONV : SWR_OK;
}
