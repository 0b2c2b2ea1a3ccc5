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

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "swr.h"
#include "swr_common.h"


using namespace swr;

struct swr_ctx {
    // problem
    double a0 = 0, b0 = 0, h = 0, dt = 0;
    int N = 0, nt = 0, nx = 0, nc = 0, ns = 0, B = 1, vk = 0, tr = 0, nv = 1, P = 1;
    cd sigma{}, c2{};
    swr_opts o{};
    hipStream_t st = nullptr;
    std::vector<int> J, off;
    std::vector<Task> build_tasks, final_tasks;
    // device memory
    int* dJ = nullptr;
    int* dOff = nullptr;
    double* dV = nullptr;
    double* dBeta = nullptr;
    cd* dFac = nullptr;
    cd* dCols = nullptr;
    cd* dHist = nullptr;
    cd* dEnds = nullptr;
    Task* dBuild = nullptr;
    Task* dFinal = nullptr;
    cd* dD = nullptr;
    cd* dG = nullptr;
    cd* dG2 = nullptr;
    cd* dZero = nullptr;   // [B][ns][nt] zeros
    unsigned long long* dMax = nullptr;
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
    // causal workspace
    cd* dMinv = nullptr;
    cd* dMwork = nullptr;
    cd* dFar = nullptr;
    int* dPivOk = nullptr;
    cd* dPcr = nullptr;
    cd* dBase = nullptr;
    double* dEta = nullptr;
    int causal_path = 0;   // 1 = block PCR, 2 = dense inverse
    bool built = false;
    // host staging (pinned)
    double* hRes = nullptr;
    int* hAct = nullptr;
    hipEvent_t ev[6] = {};
    std::vector<void*> allocs;
};

#define HIPCHK(x)                                      \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) {                        \
            return SWR_EDEVICE;                        \
        }                                              \
    } while (0)

template <class T>
static swr_status dalloc(swr_ctx* c, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    void* q = nullptr;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return SWR_ENOMEM;
    c->allocs.push_back(q);
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
    if (vk < SWR_V_STATIC || vk > SWR_V_CUBIC || (tr != SWR_ROBIN && tr != SWR_S02)) return SWR_EINVAL;
    if (tr == SWR_ROBIN && s_re == 0.0 && s_im == 0.0) return SWR_EINVAL;
    if (!std::isfinite(s_re) || !std::isfinite(s_im)) return SWR_EINVAL;
    if (o.batch < 1 || o.restart < 1 || o.max_iter < 1 || !(o.tol > 0)) return SWR_EINVAL;
    if (vk == SWR_V_TIME && !V) return SWR_EINVAL;
    if (vk != SWR_V_STATIC && o.v_per_problem) return SWR_EINVAL;
    long nc = 0;
    int nmax = 0;
    for (int k = 0; k < N; ++k) {
        if (J[k] < 1) return SWR_EINVAL;
        nc += J[k];
        nmax = J[k] + 1 > nmax ? J[k] + 1 : nmax;
    }
    if (nmax > kWave * kMaxP || nc > (1L << 30)) return SWR_EINVAL;
    // only the static potential is served by this build
    if (vk != SWR_V_STATIC) return SWR_EINVAL;

    swr_ctx* c = new (std::nothrow) swr_ctx();
    if (!c) return SWR_ENOMEM;
    c->a0 = a0; c->b0 = b0; c->dt = dt; c->N = N; c->nt = (int)ntr; c->nc = (int)nc;
    c->nx = (int)nc + 1; c->h = (b0 - a0) / (double)nc; c->ns = 2 * N - 2; c->B = o.batch;
    c->vk = vk; c->tr = tr; c->o = o; c->st = (hipStream_t)stream;
    c->nv = (vk == SWR_V_STATIC && o.v_per_problem) ? o.batch : 1;
    c->P = (nmax + kWave - 1) / kWave;
    c->c2 = mk(std::cos(-M_PI / 4) * std::sqrt(2.0 / dt), std::sin(-M_PI / 4) * std::sqrt(2.0 / dt));
    // S0^2: the implicit coefficient of c2 sum beta_{n-s} v_s is c2 beta_0 = c2
    c->sigma = (tr == SWR_S02) ? c->c2 : mk(s_re, s_im);
    c->J.assign(J, J + N);
    c->off.resize(N);
    for (int k = 0, acc = 0; k < N; ++k) { c->off[k] = acc; acc += J[k]; }

    const int nt = c->nt, B = c->B, ns = c->ns, nv = c->nv;
    // task lists: impulses (per potential) + d sweeps (per problem); final sweeps
    for (int v = 0; v < nv; ++v)
        for (int k = 0; k < N; ++k) {
            if (k >= 1) c->build_tasks.push_back(Task{k, 0, v * N + k, T_IMP_L | T_OUT_COLS});
            if (k <= N - 2) c->build_tasks.push_back(Task{k, 0, v * N + k, T_IMP_R | T_OUT_COLS});
        }
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < N; ++k) c->build_tasks.push_back(Task{k, b, vof(c, b) * N + k, T_DATA_U0 | T_OUT_G});
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < N; ++k)
            c->final_tasks.push_back(Task{k, b, vof(c, b) * N + k, T_DATA_U0 | T_FLUX_G | T_OUT_G});

    const size_t vec = (size_t)B * ns * nt;
    const size_t max_tasks = c->build_tasks.size() > c->final_tasks.size() ? c->build_tasks.size()
                                                                            : c->final_tasks.size();
    ALLOC(c->dJ, N);
    ALLOC(c->dOff, N);
    ALLOC(c->dBeta, nt + kWave + 1);
    ALLOC(c->dFac, (size_t)nv * N * fac_fields(c->P) * kWave);
    ALLOC(c->dCols, (size_t)nv * N * 4 * nt);
    ALLOC(c->dHist, (tr == SWR_S02) ? max_tasks * 2 * (nt + 1) : 1);
    ALLOC(c->dEnds, (size_t)B * N * 2);
    ALLOC(c->dBuild, c->build_tasks.size());
    ALLOC(c->dFinal, c->final_tasks.size());
    ALLOC(c->dD, vec);
    ALLOC(c->dG, vec);
    ALLOC(c->dG2, vec);
    ALLOC(c->dZero, vec);
    ALLOC(c->dMax, 1);
    ALLOC(c->dPart, (size_t)B * kRedBlocks * 2 * (o.restart + 2));
    ALLOC(c->dNrm, B);
    ALLOC(c->dBn, B);
    ALLOC(c->dRes, B);
    ALLOC(c->dAct, B);
    if (V) {
        const size_t vn = (size_t)c->nx * (o.v_per_problem ? B : 1);
        ALLOC(c->dV, vn);
        HIPCHK(hipMemcpyAsync(c->dV, V, vn * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    }
    if (hipHostMalloc(&c->hRes, sizeof(double) * B) != hipSuccess ||
        hipHostMalloc(&c->hAct, sizeof(int) * B) != hipSuccess) { swr_destroy(c); return SWR_ENOMEM; }
    for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) { swr_destroy(c); return SWR_EDEVICE; }
    HIPCHK(hipMemcpyAsync(c->dJ, c->J.data(), N * sizeof(int), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->dOff, c->off.data(), N * sizeof(int), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->dBuild, c->build_tasks.data(), c->build_tasks.size() * sizeof(Task),
                          hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->dFinal, c->final_tasks.data(), c->final_tasks.size() * sizeof(Task),
                          hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemsetAsync(c->dZero, 0, vec * sizeof(cd), c->st));
    HIPCHK(hipMemsetAsync(c->dCols, 0, (size_t)nv * N * 4 * nt * sizeof(cd), c->st));
    HIPCHK(launch_beta(nt + kWave + 1, c->dBeta, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    *out = c;
    return SWR_OK;
}

extern "C" void swr_destroy(swr_ctx* c) {
    if (!c) return;
    if (c->st) hipStreamSynchronize(c->st);
    else hipDeviceSynchronize();
    for (void* p : c->allocs) hipFree(p);
    if (c->hRes) hipHostFree(c->hRes);
    if (c->hAct) hipHostFree(c->hAct);
    for (auto& e : c->ev)
        if (e) hipEventDestroy(e);
    delete c;
}

extern "C" swr_status swr_sizes(const swr_ctx* c, int* nt, int* nx, int* B, int* nv) {
    if (!c) return SWR_EINVAL;
    if (nt) *nt = c->nt;
    if (nx) *nx = c->nx;
    if (B) *B = c->B;
    if (nv) *nv = c->nv;
    return SWR_OK;
}

// ---------------------------------------------------------------------------
static SweepArgs sweep_args(swr_ctx* c, const Task* tasks, int ntasks) {
    SweepArgs a{};
    a.N = c->N; a.nt = c->nt; a.B = c->B; a.nx = c->nx; a.ns = c->ns; a.ntasks = ntasks;
    a.P = c->P;
    a.kappa = c->h / (3.0 * c->dt);
    a.sigma = c->sigma;
    a.c2 = c->c2;
    a.J = c->dJ; a.off = c->dOff; a.tasks = tasks; a.fac = c->dFac; a.beta = c->dBeta;
    a.cols = c->dCols; a.hist = c->dHist; a.ends = c->dEnds; a.maxdiff = c->dMax;
    return a;
}

static swr_status run_factor(swr_ctx* c) {
    FactorArgs f{};
    f.N = c->N; f.nx = c->nx; f.nf = c->nv * c->N; f.P = c->P; f.h = c->h; f.dt = c->dt;
    f.sigma = c->sigma; f.J = c->dJ; f.off = c->dOff; f.V = c->dV; f.fac = c->dFac;
    HIPCHK(launch_factor(f, c->st));
    return SWR_OK;
}

// impulse sweeps + d sweeps in one launch (Sec. 4.1)
static swr_status run_build(swr_ctx* c, const double* u0) {
    SweepArgs a = sweep_args(c, c->dBuild, (int)c->build_tasks.size());
    a.u0 = reinterpret_cast<const cd*>(u0);
    a.g_in = c->dZero;
    a.g_out = c->dD;
    HIPCHK(launch_sweep(a, c->tr, c->st));
    c->built = true;
    return SWR_OK;
}

// sweeps of every (problem, subdomain) with fluxes g_in
static swr_status run_sweeps(swr_ctx* c, const cd* u0, const cd* g_in, cd* g_out, cd* uT,
                             cd* trace, bool maxdiff) {
    std::vector<Task>& tl = c->final_tasks;
    // flags vary per call: rebuild the list only when they change
    int want = (u0 ? T_DATA_U0 : 0) | T_FLUX_G | T_OUT_G | (uT ? T_OUT_UT : 0) |
               (trace ? T_OUT_TRACE : 0) | (maxdiff ? T_MAXDIFF : 0);
    if (tl.empty() || tl[0].flags != want) {
        for (auto& t : tl) t.flags = want;
        HIPCHK(hipMemcpyAsync(c->dFinal, tl.data(), tl.size() * sizeof(Task), hipMemcpyHostToDevice,
                              c->st));
    }
    SweepArgs a = sweep_args(c, c->dFinal, (int)tl.size());
    a.u0 = u0;
    a.g_in = g_in;
    a.g_out = g_out;
    a.uT = uT;
    a.trace = trace;
    if (maxdiff) HIPCHK(hipMemsetAsync(c->dMax, 0, sizeof(unsigned long long), c->st));
    HIPCHK(launch_sweep(a, c->tr, c->st));
    if (uT) HIPCHK(launch_finalize_ut(c->N, c->nx, c->B, c->dOff, c->dEnds, uT, c->st));
    return SWR_OK;
}

static LttArgs ltt_args(swr_ctx* c, const cd* x, cd* y) {
    LttArgs l{};
    l.N = c->N; l.nt = c->nt; l.ns = c->ns; l.B = c->B; l.per_problem = c->nv > 1;
    l.cols = c->dCols; l.x = x; l.y = y; l.base = x; l.sign = -1.0;
    l.n_lo = 0; l.n_hi = c->nt; l.s_hi = c->nt; l.y_ld = c->nt;
    return l;
}

// GMRES(m) on (I - L) g = d, all problems of the batch at once (each with its
// own Krylov space); classical Gram-Schmidt applied twice.
static swr_status run_gmres(swr_ctx* c, int* iters_out) {
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
        c->gm_m = m;
    }
    hipStream_t st = c->st;
    cd* x = c->dG;
    HIPCHK(hipMemsetAsync(x, 0, (size_t)B * M * sizeof(cd), st));
    HIPCHK(launch_norm(c->dD, M, B, c->dPart, c->dBn, st));
    int its = 0;
    bool conv = false;
    while (its < c->o.max_iter && !conv) {
        // r = d - (I - L) x  -> basis[0]
        LttArgs l = ltt_args(c, x, c->dW);
        HIPCHK(launch_ltt(l, st));
        HIPCHK(launch_axpby(c->dD, 1.0, c->dW, -1.0, c->dBasis, (long)B * M, st));
        HIPCHK(launch_norm(c->dBasis, M, B, c->dPart, c->dNrm, st));
        HIPCHK(launch_gmres_init(m, B, c->dNrm, c->dE, c->dAct, c->dBn, c->o.tol, c->dRes, st));
        HIPCHK(hipMemcpyAsync(c->hAct, c->dAct, sizeof(int) * B, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool any = false;
        for (int b = 0; b < B; ++b) any |= c->hAct[b] != 0;
        if (!any) { conv = true; break; }
        HIPCHK(launch_scale(c->dBasis, c->dNrm, c->dBasis, M, B, nullptr, st));
        int jj = 0;
        for (int j = 0; j < m && its < c->o.max_iter; ++j) {
            cd* vj = c->dBasis + (size_t)j * B * M;
            cd* vn = c->dBasis + (size_t)(j + 1) * B * M;
            LttArgs lj = ltt_args(c, vj, c->dW);
            HIPCHK(launch_ltt(lj, st));
            HIPCHK(launch_multidot(c->dBasis, j + 1, c->dW, M, B, c->dPart, c->dHp, m + 1, 0, st));
            HIPCHK(launch_multiaxpy(c->dBasis, j + 1, c->dHp, m + 1, -1.0, c->dW, M, B, st));
            HIPCHK(launch_multidot(c->dBasis, j + 1, c->dW, M, B, c->dPart, c->dHp2, m + 1, 0, st));
            HIPCHK(launch_multiaxpy(c->dBasis, j + 1, c->dHp2, m + 1, -1.0, c->dW, M, B, st));
            HIPCHK(launch_axpby(c->dHp, 1.0, c->dHp2, 1.0, c->dHp, (long)B * (m + 1), st));
            HIPCHK(launch_norm(c->dW, M, B, c->dPart, c->dNrm, st));
            HIPCHK(launch_scale(c->dW, c->dNrm, vn, M, B, nullptr, st));
            HIPCHK(launch_givens(j, m, B, c->dHp, c->dNrm, c->dH, c->dCs, c->dSn, c->dE, c->dBn,
                                 c->dRes, c->dAct, st));
            HIPCHK(hipMemcpyAsync(c->hRes, c->dRes, sizeof(double) * B, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            ++its;
            jj = j + 1;
            bool done = true;
            for (int b = 0; b < B; ++b) {
                if (!std::isfinite(c->hRes[b])) return SWR_ENAN;
                if (c->hAct[b] && c->hRes[b] > c->o.tol) done = false;
            }
            if (done) { conv = true; break; }
        }
        HIPCHK(launch_gmres_solve(jj, m, B, c->dH, c->dE, c->dY, c->dAct, st));
        HIPCHK(launch_multiaxpy(c->dBasis, jj, c->dY, m + 1, 1.0, x, M, B, st));
        if (conv) {
            // confirm with the true residual at the next cycle start
            conv = false;
        }
    }
    *iters_out = its;
    return its >= c->o.max_iter ? SWR_ENOCONV : SWR_OK;
}

// causal forward substitution in time (exact up to rounding).  Block PCR
// per step when it applies (N - 1 <= 64, ns <= 128) and the block system is
// certified diagonally dominant; otherwise a dense (I - C_0)^{-1} by
// Gauss-Jordan with partial pivoting.
static swr_status run_causal(swr_ctx* c) {
    const int ns = c->ns, nt = c->nt, B = c->B;
    hipStream_t st = c->st;
    if (ns <= kNearSlots && c->N - 1 <= kWave) {
        if (!c->dPcr) {
            ALLOC_LIVE(c->dPcr, (size_t)c->nv * kPcrRec * kWave);
            ALLOC_LIVE(c->dBase, (size_t)B * ns * kNearTb);
            ALLOC_LIVE(c->dEta, c->nv);
        }
        HIPCHK(launch_causal_pcr_setup(c->N, nt, c->nv, c->dCols, c->dPcr, c->dEta, st));
        std::vector<double> eta(c->nv);
        HIPCHK(hipMemcpyAsync(eta.data(), c->dEta, sizeof(double) * c->nv, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool ok = true;
        for (double e : eta) ok = ok && std::isfinite(e) && e < 1.0;
        if (ok) {
            c->causal_path = 1;
            HIPCHK(launch_causal_fast(c->N, nt, ns, B, c->nv > 1, c->dCols, c->dPcr, c->dD, c->dBase,
                                      c->dG, st));
            return SWR_OK;
        }
    }
    c->causal_path = 2;
    if (!c->dMinv) {
        ALLOC_LIVE(c->dMinv, (size_t)c->nv * ns * ns);
        ALLOC_LIVE(c->dMwork, (size_t)c->nv * ns * ns);
        ALLOC_LIVE(c->dFar, (size_t)B * ns * kCausalTb);
        ALLOC_LIVE(c->dPivOk, c->nv);
    }
    HIPCHK(launch_c0_inverse(c->N, ns, nt, c->nv, c->dCols, c->dMwork, c->dMinv, c->dPivOk, st));
    for (int n0 = 0; n0 < nt; n0 += kCausalTb) {
        const int nb = std::min(kCausalTb, nt - n0);
        LttArgs l{};
        l.N = c->N; l.nt = nt; l.ns = ns; l.B = B; l.per_problem = c->nv > 1;
        l.cols = c->dCols; l.x = c->dG; l.y = c->dFar; l.base = nullptr; l.sign = 1.0;
        l.n_lo = n0; l.n_hi = n0 + nb; l.s_hi = n0; l.y_ld = kCausalTb;
        HIPCHK(launch_ltt(l, st));
        CausalArgs ca{};
        ca.N = c->N; ca.nt = nt; ca.ns = ns; ca.B = B; ca.per_problem = c->nv > 1;
        ca.n0 = n0; ca.nb = nb; ca.cols = c->dCols; ca.Minv = c->dMinv; ca.d = c->dD;
        ca.far = c->dFar; ca.g = c->dG;
        HIPCHK(launch_causal_block(ca, st));
    }
    return SWR_OK;
}

// classical algorithm: g <- R g until max |g^{k+1} - g^k| < tol (Sec. 4)
static swr_status run_classical(swr_ctx* c, const double* u0, int* iters, double* last) {
    const size_t vec = (size_t)c->B * c->ns * c->nt;
    HIPCHK(hipMemsetAsync(c->dG, 0, vec * sizeof(cd), c->st));
    cd* gi = c->dG;
    cd* go = c->dG2;
    const cd* u = reinterpret_cast<const cd*>(u0);
    *last = INFINITY;
    for (int it = 1; it <= c->o.max_iter; ++it) {
        swr_status s = run_sweeps(c, u, gi, go, nullptr, nullptr, true);
        if (s != SWR_OK) return s;
        unsigned long long bits = 0;
        HIPCHK(hipMemcpyAsync(&bits, c->dMax, sizeof(bits), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        double d;
        std::memcpy(&d, &bits, sizeof(d));
        *last = d;
        *iters = it;
        std::swap(gi, go);
        if (!std::isfinite(d)) return SWR_ENAN;
        if (d < c->o.tol) {
            if (gi != c->dG) HIPCHK(hipMemcpyAsync(c->dG, gi, vec * sizeof(cd), hipMemcpyDeviceToDevice, c->st));
            return SWR_OK;
        }
    }
    if (gi != c->dG) HIPCHK(hipMemcpyAsync(c->dG, gi, vec * sizeof(cd), hipMemcpyDeviceToDevice, c->st));
    return SWR_ENOCONV;
}

static double elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    hipEventElapsedTime(&ms, a, b);
    return ms;
}

extern "C" swr_status swr_solve(swr_ctx* c, const double* u0, double* uT, double* g, double* utrace,
                                swr_info* info) {
    if (!c || !u0 || !uT) return SWR_EINVAL;
    const size_t vec = (size_t)c->B * c->ns * c->nt;
    hipStream_t st = c->st;
    swr_status rs = SWR_OK;
    int iters = 0;
    double fixed_last = 0;
    HIPCHK(hipEventRecord(c->ev[0], st));
    swr_status s = run_factor(c);
    if (s != SWR_OK) return s;
    HIPCHK(hipEventRecord(c->ev[1], st));
    if (c->o.solver != SWR_SOLVER_FIXED) {
        s = run_build(c, u0);
        if (s != SWR_OK) return s;
    }
    HIPCHK(hipEventRecord(c->ev[2], st));
    if (c->ns == 0) {
        HIPCHK(hipMemsetAsync(c->dG, 0, sizeof(cd), st));
    } else if (c->o.solver == SWR_SOLVER_FIXED) {
        rs = run_classical(c, u0, &iters, &fixed_last);
    } else if (c->o.solver == SWR_SOLVER_GMRES) {
        rs = run_gmres(c, &iters);
    } else if (c->o.solver == SWR_SOLVER_CAUSAL) {
        rs = run_causal(c);
        iters = 1;
    } else {
        return SWR_EINVAL;
    }
    if (rs != SWR_OK && rs != SWR_ENOCONV) return rs;
    HIPCHK(hipEventRecord(c->ev[3], st));
    s = run_sweeps(c, reinterpret_cast<const cd*>(u0), c->dG, c->dG2, reinterpret_cast<cd*>(uT),
                   reinterpret_cast<cd*>(utrace), false);
    if (s != SWR_OK) return s;
    HIPCHK(hipEventRecord(c->ev[4], st));
    if (g) HIPCHK(hipMemcpyAsync(g, c->dG, vec * sizeof(cd), hipMemcpyDeviceToDevice, st));
    // certified residual ||g - R g|| / ||R 0||; R 0 = d for the built path
    double res = 0;
    if (c->ns > 0) {
        const long M = (long)c->ns * c->nt;
        HIPCHK(launch_axpby(c->dG, 1.0, c->dG2, -1.0, c->dW ? c->dW : c->dG2, (long)vec, st));
        if (c->o.solver != SWR_SOLVER_FIXED) {
            HIPCHK(launch_norm(c->dW ? c->dW : c->dG2, M, c->B, c->dPart, c->dNrm, st));
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
    HIPCHK(hipStreamSynchronize(st));
    if (info) {
        info->iters = iters;
        info->residual = res;
        info->t_factor_ms = elapsed(c->ev[0], c->ev[1]);
        info->t_build_ms = elapsed(c->ev[1], c->ev[2]);
        info->t_iface_ms = elapsed(c->ev[2], c->ev[3]);
        info->t_final_ms = elapsed(c->ev[3], c->ev[4]);
        info->nl_worst = 0;
    }
    return rs;
}

extern "C" swr_status swr_apply_R(swr_ctx* c, const double* u0, const double* g_in, double* g_out,
                                  double* uT, double* maxdiff) {
    if (!c || !g_in || !g_out) return SWR_EINVAL;
    swr_status s = run_factor(c);
    if (s != SWR_OK) return s;
    s = run_sweeps(c, reinterpret_cast<const cd*>(u0), reinterpret_cast<const cd*>(g_in),
                   reinterpret_cast<cd*>(g_out), reinterpret_cast<cd*>(uT), nullptr, maxdiff != nullptr);
    if (s != SWR_OK) return s;
    if (maxdiff) {
        unsigned long long bits = 0;
        HIPCHK(hipMemcpyAsync(&bits, c->dMax, sizeof(bits), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        std::memcpy(maxdiff, &bits, sizeof(double));
    }
    HIPCHK(hipStreamSynchronize(c->st));
    return SWR_OK;
}

extern "C" swr_status swr_build_interface(swr_ctx* c, const double* u0, double* cols, double* d) {
    if (!c || !u0) return SWR_EINVAL;
    swr_status s = run_factor(c);
    if (s != SWR_OK) return s;
    s = run_build(c, u0);
    if (s != SWR_OK) return s;
    if (cols) HIPCHK(hipMemcpyAsync(cols, c->dCols, (size_t)c->nv * c->N * 4 * c->nt * sizeof(cd),
                                    hipMemcpyDeviceToDevice, c->st));
    if (d) HIPCHK(hipMemcpyAsync(d, c->dD, (size_t)c->B * c->ns * c->nt * sizeof(cd),
                                 hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return SWR_OK;
}

extern "C" swr_status swr_interface_matvec(swr_ctx* c, const double* x, double* y) {
    if (!c || !x || !y || !c->built) return SWR_EINVAL;
    LttArgs l = ltt_args(c, reinterpret_cast<const cd*>(x), reinterpret_cast<cd*>(y));
    HIPCHK(launch_ltt(l, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return SWR_OK;
}

extern "C" swr_status swr_grad(swr_ctx* c, const double* u0, const double* gbar, double* dJdV,
                               double* dJdu0, swr_info* info) {
    (void)u0; (void)gbar; (void)dJdV; (void)dJdu0; (void)info;
    if (!c) return SWR_EINVAL;
    return SWR_EINVAL;
}
