// swr_causal.hip -- exact causal solve of the interface problem
// (I - L) g = d for a time-independent potential (Besse & Xing,
// arXiv 1503.02564, Secs. 3-4).
//
// Every block of L is lower triangular in time (Props. 3-4), so with C_m the
// matrix of the m-th Toeplitz coefficients of all blocks, time step n reads
//     (I - C_0) g_n = d_n + sum_{s<n} C_{n-s} g_s.
// Per time step the unknowns of interface j (between subdomains j and j+1)
// are p_j = (r_j, l_{j+1}) (slots 2j, 2j+1).  Row r_j is subdomain j+1's left
// output, row l_{j+1} subdomain j's right output, so (I - C_0) is block
// tridiagonal with 2x2 blocks
//     D_j = [[1, -x1_{j+1}], [-x4_j, 1]],  U_j = [[-x2_{j+1}, 0], [0, 0]],
//     L_j = [[0, 0], [0, -x3_j]]
// (x_p^{k} the lag-0 entry of X^{k,p}).  It is reduced by block parallel
// cyclic reduction, whose multipliers are computed once; the reduction is
// stable when the system is block diagonally dominant
// (max_j ||D_j^{-1}|| (||L_j|| + ||U_j||) < 1), which setup checks.
//
// Time is processed in super-blocks of 256 steps (absolute windows) and,
// inside them, in blocks of kTb steps.  The contribution of every earlier
// super-block to the outputs being solved is formed by one block-Toeplitz
// product on the matrix cores (launch_ltt).  `causal_far_kernel` adds to d that product and
// the contribution of the earlier blocks of the current super-block (a short
// rectangle, one workgroup per output slot);
// `causal_near_kernel` then
// marches through the block on one workgroup per problem: wave 0 runs the
// per-step PCR solve while waves 1..8 gather the in-block history (lags >= 2)
// of the next step, from the block's g kept in LDS and the lag coefficients
// kept in registers.
#include "swr_common.h"

namespace swr {

constexpr int kTb = kNearTb;                  // near block (time steps)

struct C2x2 { cd a, b, c, d; };   // [[a, b], [c, d]]

__device__ inline C2x2 m2(cd a, cd b, cd c, cd d) { C2x2 r; r.a = a; r.b = b; r.c = c; r.d = d; return r; }
__device__ inline C2x2 operator*(const C2x2& x, const C2x2& y) {
    return m2(madd(x.a * y.a, x.b, y.c), madd(x.a * y.b, x.b, y.d),
              madd(x.c * y.a, x.d, y.c), madd(x.c * y.b, x.d, y.d));
}
__device__ inline C2x2 operator-(const C2x2& x, const C2x2& y) {
    return m2(x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d);
}
__device__ inline C2x2 neg(const C2x2& x) { return m2(-x.a, -x.b, -x.c, -x.d); }
__device__ inline C2x2 inv2(const C2x2& x) {
    const cd idet = inv(x.a * x.d - x.b * x.c);
    return m2(x.d * idet, -(x.b * idet), -(x.c * idet), x.a * idet);
}
__device__ inline double norm_inf(const C2x2& x) {
    return fmax(sqrt(abs2(x.a)) + sqrt(abs2(x.b)), sqrt(abs2(x.c)) + sqrt(abs2(x.d)));
}
__device__ inline C2x2 shfl_up_m(const C2x2& x, int d, const C2x2& fill) {
    return m2(shfl_up_c(x.a, d, fill.a), shfl_up_c(x.b, d, fill.b), shfl_up_c(x.c, d, fill.c),
              shfl_up_c(x.d, d, fill.d));
}
__device__ inline C2x2 shfl_dn_m(const C2x2& x, int d, const C2x2& fill) {
    return m2(shfl_dn_c(x.a, d, fill.a), shfl_dn_c(x.b, d, fill.b), shfl_dn_c(x.c, d, fill.c),
              shfl_dn_c(x.d, d, fill.d));
}

// Block PCR multipliers of (I - C_0), one wave per potential, lane j =
// interface j (N - 1 <= 64 interfaces).  Record per lane: for each level
// K1 (4), K2 (4), then D^{-1} (4).  eta[v] = block dominance measure.
__global__ __launch_bounds__(64) void causal_pcr_setup_kernel(int N, int nt, const cd* cols, cd* pcr,
                                                              double* eta) {
    const int v = blockIdx.x, j = threadIdx.x;
    const int ni = N - 1;
    const cd* base = cols + (size_t)v * N * 4 * nt;
    auto col0 = [&](int k, int p) { return base[((size_t)k * 4 + p) * nt]; };
    const cd zero = mk(0, 0), one = mk(1, 0);
    const C2x2 I = m2(one, zero, zero, one), Z = m2(zero, zero, zero, zero);
    C2x2 D = I, Lm = Z, U = Z;
    if (j < ni) {
        const cd x1 = col0(j + 1, 0);
        const cd x2 = (j + 1 <= N - 2) ? col0(j + 1, 1) : zero;
        const cd x3 = (j >= 1) ? col0(j, 2) : zero;
        const cd x4 = col0(j, 3);
        D = m2(one, -x1, -x4, one);
        U = m2(-x2, zero, zero, zero);
        Lm = m2(zero, zero, zero, -x3);
    }
    double e = norm_inf(inv2(D)) * (norm_inf(Lm) + norm_inf(U));
    e = wave_max(e);
    if (j == 0) eta[v] = e;
    cd* rec = pcr + (size_t)v * kPcrRec * kWave + j;
    // runs once per solve: keep the level loop rolled (the fully unrolled
    // chain of 2x2 complex products is very slow to compile)
#pragma unroll 1
    for (int l = 0; l < kPcrLevels; ++l) {
        const int d = 1 << l;
        const C2x2 Dm = shfl_up_m(D, d, I), Lmm = shfl_up_m(Lm, d, Z), Um = shfl_up_m(U, d, Z);
        const C2x2 Dp = shfl_dn_m(D, d, I), Lp = shfl_dn_m(Lm, d, Z), Up = shfl_dn_m(U, d, Z);
        const C2x2 K1 = (j - d >= 0) ? Lm * inv2(Dm) : Z;
        const C2x2 K2 = (j + d < kWave) ? U * inv2(Dp) : Z;
        const C2x2 Dn = D - K1 * Um - K2 * Lp;
        const C2x2 Ln = neg(K1 * Lmm), Un = neg(K2 * Up);
        D = Dn;
        Lm = Ln;
        U = Un;
        cd* r = rec + (size_t)l * 8 * kWave;
        r[0 * kWave] = K1.a; r[1 * kWave] = K1.b; r[2 * kWave] = K1.c; r[3 * kWave] = K1.d;
        r[4 * kWave] = K2.a; r[5 * kWave] = K2.b; r[6 * kWave] = K2.c; r[7 * kWave] = K2.d;
    }
    const C2x2 Di = inv2(D);
    cd* r = rec + (size_t)kPcrLevels * 8 * kWave;
    r[0 * kWave] = Di.a; r[1 * kWave] = Di.b; r[2 * kWave] = Di.c; r[3 * kWave] = Di.d;
}

__device__ inline void slot_src(int o, int N, int& k, int& pl, int& pr, int& sl, int& sr) {
    if ((o & 1) == 0) { k = o / 2 + 1; pl = 0; pr = 1; }
    else { k = (o - 1) / 2; pl = 2; pr = 3; }
    sl = (k >= 1) ? 2 * k - 1 : -1;
    sr = (k <= N - 2) ? 2 * k : -1;
}

struct FarArgs {
    int N, nt, ns, per_problem;
    int n0, nb;
    const cd* cols;    // [nv][N][4][nt]
    const cd* d;       // [B][ns][nt]
    const cd* g;       // [B][ns][nt]
    cd* out;           // [B][ns][kTb]  = d + contribution of steps s < n0
    const cd* facc;    // [B][ns][nt] contribution of steps s < s_from (null: none)
    int s_from;        // this kernel sums steps s_from <= s < n0
};

// one workgroup per (slot, problem); thread (i, split): output step n0+i,
// inputs s in the split's share of [0, n0).  out = d + that contribution.
template <int TB>
__global__ __launch_bounds__(256) void causal_far_kernel(FarArgs f) {
    constexpr int SPLITS = 256 / TB;
    __shared__ cd part[SPLITS][TB];
    const int o = blockIdx.x, b = blockIdx.y;
    const int i = threadIdx.x % TB, sp = threadIdx.x / TB;
    int k, pl, pr, sl, sr;
    slot_src(o, f.N, k, pl, pr, sl, sr);
    const int v = f.per_problem ? b : 0;
    const cd* cl = f.cols + ((size_t)(v * f.N + k) * 4 + pl) * f.nt;
    const cd* cr = f.cols + ((size_t)(v * f.N + k) * 4 + pr) * f.nt;
    const cd* gl = sl >= 0 ? f.g + ((size_t)b * f.ns + sl) * f.nt : nullptr;
    const cd* gr = sr >= 0 ? f.g + ((size_t)b * f.ns + sr) * f.nt : nullptr;
    const int n = f.n0 + i;
    const int per = (f.n0 - f.s_from + SPLITS - 1) / SPLITS;
    const int s_lo = f.s_from + sp * per, s_hi = min(f.n0, s_lo + per);
    double ax = 0, ay = 0;
    if (i < f.nb) {
        for (int s = s_lo; s < s_hi; ++s) {
            if (gl) {
                const cd c = cl[n - s], x = gl[s];
                ax += c.x * x.x - c.y * x.y;
                ay += c.x * x.y + c.y * x.x;
            }
            if (gr) {
                const cd c = cr[n - s], x = gr[s];
                ax += c.x * x.x - c.y * x.y;
                ay += c.x * x.y + c.y * x.x;
            }
        }
    }
    part[sp][i] = mk(ax, ay);
    __syncthreads();
    if (sp == 0 && i < f.nb) {
        cd r = f.d[((size_t)b * f.ns + o) * f.nt + n];
        if (f.facc) r = r + f.facc[((size_t)b * f.ns + o) * f.nt + n];
        for (int q = 0; q < SPLITS; ++q) r = r + part[q][i];
        f.out[((size_t)b * f.ns + o) * TB + i] = r;
    }
}

struct NearArgs {
    int N, nt, ns, per_problem;
    int n0, nb;
    const cd* cols;
    const cd* pcr;     // [nv][kPcrRec][64]
    const cd* base;    // [B][ns][kTb]: d + far part
    cd* g;             // [B][ns][nt]
};

constexpr int kNearThreads = 64 + 4 * kNearSlots;

// one workgroup per problem; wave 0 = PCR solver, waves 1..8 = gather
__global__ __launch_bounds__(kNearThreads) void causal_near_kernel(NearArgs a) {
    __shared__ cd gh[kTb][kNearSlots];
    __shared__ cd rhs[kNearSlots];
    __shared__ cd gn[kNearSlots];
    __shared__ cd spcr[kPcrRec][kWave];
    const int b = blockIdx.x, v = a.per_problem ? b : 0;
    const int tid = threadIdx.x;
    const int ns = a.ns, nt = a.nt, n0 = a.n0, nb = a.nb;
    const int ni = a.N - 1;
    const cd zero = mk(0, 0);
    cd* gb = a.g + (size_t)b * ns * nt;
    const cd* bb = a.base + (size_t)b * ns * kTb;

    // PCR multipliers -> LDS
    for (int e = tid; e < kPcrRec * kWave; e += blockDim.x)
        (&spcr[0][0])[e] = a.pcr[(size_t)v * kPcrRec * kWave + e];

    // gather role: slot o, lag class c (lags c+1, c+5, ..., c+29)
    const int gt = tid - kWave;
    const int o = gt >> 2, c = gt & 3;
    const bool gather = tid >= kWave && o < ns;
    int sl = -1, sr = -1;
    cd cl[8], cr[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) { cl[m] = zero; cr[m] = zero; }
    if (gather) {
        int k, pl, pr;
        slot_src(o, a.N, k, pl, pr, sl, sr);
        const cd* base = a.cols + (size_t)(v * a.N + k) * 4 * nt;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int lag = c + 1 + 4 * m;
            if (lag < nt) {
                if (sl >= 0) cl[m] = base[(size_t)pl * nt + lag];
                if (sr >= 0) cr[m] = base[(size_t)pr * nt + lag];
            }
        }
        if (c == 0) rhs[o] = bb[(size_t)o * kTb + 0];   // step n0: no in-block history
    }
    __syncthreads();

    for (int i = 0; i < nb; ++i) {
        if (tid < kWave) {
            // per-step solve of (I - C_0) g = rhs by block PCR; lane j = interface j
            const int j = tid;
            cd p0 = zero, p1 = zero;
            if (j < ni) { p0 = rhs[2 * j]; p1 = rhs[2 * j + 1]; }
#pragma unroll
            for (int l = 0; l < kPcrLevels; ++l) {
                const int d = 1 << l;
                const cd q0m = shfl_up_c(p0, d, zero), q1m = shfl_up_c(p1, d, zero);
                const cd q0p = shfl_dn_c(p0, d, zero), q1p = shfl_dn_c(p1, d, zero);
                const cd* K = &spcr[l * 8][j];
                const cd k1a = K[0 * kWave], k1b = K[1 * kWave], k1c = K[2 * kWave], k1d = K[3 * kWave];
                const cd k2a = K[4 * kWave], k2b = K[5 * kWave], k2c = K[6 * kWave], k2d = K[7 * kWave];
                p0 = msub(msub(msub(msub(p0, k1a, q0m), k1b, q1m), k2a, q0p), k2b, q1p);
                p1 = msub(msub(msub(msub(p1, k1c, q0m), k1d, q1m), k2c, q0p), k2d, q1p);
            }
            const cd* Di = &spcr[kPcrLevels * 8][j];
            const cd x0 = madd(Di[0] * p0, Di[1 * kWave], p1);
            const cd x1 = madd(Di[2 * kWave] * p0, Di[3 * kWave], p1);
            if (j < ni) {
                gh[i][2 * j] = x0;
                gh[i][2 * j + 1] = x1;
                gb[(size_t)(2 * j) * nt + n0 + i] = x0;
                gb[(size_t)(2 * j + 1) * nt + n0 + i] = x1;
            }
        } else if (i + 1 < nb) {
            // history of step i+1 from in-block steps up to i-1 (lags >= 2)
            cd part = zero;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int lag = c + 1 + 4 * m;
                if (lag >= 2 && lag <= i + 1) {
                    const int s = i + 1 - lag;
                    if (sl >= 0) part = madd(part, cl[m], gh[s][sl]);
                    if (sr >= 0) part = madd(part, cr[m], gh[s][sr]);
                }
            }
            part = mk(part.x + __shfl_xor(part.x, 1), part.y + __shfl_xor(part.y, 1));
            part = mk(part.x + __shfl_xor(part.x, 2), part.y + __shfl_xor(part.y, 2));
            if (gather && c == 0) gn[o] = part + bb[(size_t)o * kTb + i + 1];
        }
        __syncthreads();
        if (gather && c == 0 && i + 1 < nb) {
            // lag 1 needs the step just solved
            cd r = gn[o];
            if (sl >= 0) r = madd(r, cl[0], gh[i][sl]);
            if (sr >= 0) r = madd(r, cr[0], gh[i][sr]);
            rhs[o] = r;
        }
        __syncthreads();
    }
}

hipError_t launch_causal_pcr_setup(int N, int nt, int nv, const cd* cols, cd* pcr, double* eta,
                                   hipStream_t st) {
    causal_pcr_setup_kernel<<<nv, 64, 0, st>>>(N, nt, cols, pcr, eta);
    return hipGetLastError();
}

template <int TB>
static hipError_t launch_causal_far(int N, int nt, int ns, int B, int per_problem, int n0, int nb,
                                    const cd* cols, const cd* d, const cd* g, cd* out,
                                    const cd* facc, int s_from, hipStream_t st) {
    FarArgs f{N, nt, ns, per_problem, n0, nb, cols, d, g, out, facc, s_from};
    causal_far_kernel<TB><<<dim3(ns, B), 256, 0, st>>>(f);
    return hipGetLastError();
}

hipError_t launch_causal_near(int N, int nt, int ns, int B, int per_problem, int n0, int nb,
                              const cd* cols, const cd* pcr, const cd* base, cd* g, hipStream_t st) {
    if (ns > kNearSlots || N - 1 > kWave) return hipErrorInvalidValue;
    NearArgs a{N, nt, ns, per_problem, n0, nb, cols, pcr, base, g};
    causal_near_kernel<<<B, kNearThreads, 0, st>>>(a);
    return hipGetLastError();
}

// the whole forward substitution: far part then near march, block by block
hipError_t launch_causal_fast(int N, int nt, int ns, int B, int per_problem, const cd* cols,
                              const cd* pcr, const cd* d, cd* base, cd* g, int n_lo, int n_hi,
                              const cd* facc, int s_from, hipStream_t st) {
    if (n_lo % kTb != 0 || n_lo < 0 || n_hi > nt || s_from < 0 || s_from > n_lo)
        return hipErrorInvalidValue;
    for (int n0 = n_lo; n0 < n_hi; n0 += kTb) {
        const int nb = min(kTb, n_hi - n0);
        hipError_t e = launch_causal_far<kTb>(N, nt, ns, B, per_problem, n0, nb, cols, d, g, base,
                                              facc, s_from, st);
        if (e != hipSuccess) return e;
        e = launch_causal_near(N, nt, ns, B, per_problem, n0, nb, cols, pcr, base, g, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// General path: up to kGenMaxIf interfaces.  Same algebra as above with the
// block PCR spread over the workgroup (one thread per interface, exchange
// through LDS) and a short near block of kGenTb steps.
// ---------------------------------------------------------------------------
constexpr int kGenThreads = 512;

__device__ inline int pcr_levels(int ni) {
    int l = 0;
    while ((1 << l) < ni) ++l;
    return l;
}

// multipliers [nv][levels][8][ni] then D^{-1} [nv][4][ni] (after the levels)
__global__ __launch_bounds__(kGenThreads) void causal_pcr_setup_gen_kernel(int N, int nt, const cd* cols,
                                                                          cd* pcr, int rec, double* eta) {
    __shared__ C2x2 sD[kGenMaxIf], sL[kGenMaxIf], sU[kGenMaxIf];
    __shared__ double se[kGenThreads / kWave];
    const int v = blockIdx.x, j = threadIdx.x;
    const int ni = N - 1, lv = pcr_levels(ni);
    const cd* base = cols + (size_t)v * N * 4 * nt;
    auto col0 = [&](int k, int p) { return base[((size_t)k * 4 + p) * nt]; };
    const cd zero = mk(0, 0), one = mk(1, 0);
    const C2x2 I = m2(one, zero, zero, one), Z = m2(zero, zero, zero, zero);
    C2x2 D = I, Lm = Z, U = Z;
    if (j < ni) {
        const cd x1 = col0(j + 1, 0);
        const cd x2 = (j + 1 <= N - 2) ? col0(j + 1, 1) : zero;
        const cd x3 = (j >= 1) ? col0(j, 2) : zero;
        const cd x4 = col0(j, 3);
        D = m2(one, -x1, -x4, one);
        U = m2(-x2, zero, zero, zero);
        Lm = m2(zero, zero, zero, -x3);
    }
    double e = (j < ni) ? norm_inf(inv2(D)) * (norm_inf(Lm) + norm_inf(U)) : 0.0;
    e = wave_max(e);
    if ((j & (kWave - 1)) == 0) se[j / kWave] = e;
    __syncthreads();
    if (j == 0) {
        double m = 0;
        for (int w = 0; w < kGenThreads / kWave; ++w) m = fmax(m, se[w]);
        eta[v] = m;
    }
    cd* rec_v = pcr + (size_t)v * rec;
#pragma unroll 1
    for (int l = 0; l < lv; ++l) {
        const int d = 1 << l;
        if (j < ni) { sD[j] = D; sL[j] = Lm; sU[j] = U; }
        __syncthreads();
        C2x2 K1 = Z, K2 = Z;
        if (j < ni) {
            const bool hm = j - d >= 0, hp = j + d < ni;
            const C2x2 Dm = hm ? sD[j - d] : I, Lmm = hm ? sL[j - d] : Z, Um = hm ? sU[j - d] : Z;
            const C2x2 Dp = hp ? sD[j + d] : I, Lp = hp ? sL[j + d] : Z, Up = hp ? sU[j + d] : Z;
            K1 = hm ? Lm * inv2(Dm) : Z;
            K2 = hp ? U * inv2(Dp) : Z;
            const C2x2 Dn = D - K1 * Um - K2 * Lp;
            const C2x2 Ln = neg(K1 * Lmm), Un = neg(K2 * Up);
            D = Dn;
            Lm = Ln;
            U = Un;
            cd* r = rec_v + (size_t)l * 8 * ni + j;
            r[0 * ni] = K1.a; r[1 * ni] = K1.b; r[2 * ni] = K1.c; r[3 * ni] = K1.d;
            r[4 * ni] = K2.a; r[5 * ni] = K2.b; r[6 * ni] = K2.c; r[7 * ni] = K2.d;
        }
        __syncthreads();
    }
    if (j < ni) {
        const C2x2 Di = inv2(D);
        cd* r = rec_v + (size_t)lv * 8 * ni + j;
        r[0 * ni] = Di.a; r[1 * ni] = Di.b; r[2 * ni] = Di.c; r[3 * ni] = Di.d;
    }
}

struct NearGenArgs {
    int N, nt, ns, per_problem;
    int n0, nb, rec;
    const cd* cols;
    const cd* pcr;     // [nv][rec]
    const cd* base;    // [B][ns][kGenTb]: d + far part
    cd* g;             // [B][ns][nt]
};

// one workgroup per problem; per step: gather the in-block history of every
// slot (coefficients of lags 1..kGenTb-1 in registers), then block PCR
__global__ __launch_bounds__(kGenThreads) void causal_near_gen_kernel(NearGenArgs a) {
    extern __shared__ cd smem[];
    const int ns = a.ns, nt = a.nt, n0 = a.n0, nb = a.nb, ni = a.N - 1;
    cd* gh = smem;                          // [kGenTb][ns]
    cd* rhs = gh + (size_t)kGenTb * ns;     // [ns]
    cd* ex = rhs + ns;                      // [ni][2] PCR exchange
    const int b = blockIdx.x, v = a.per_problem ? b : 0;
    const int tid = threadIdx.x;
    const int lv = pcr_levels(ni);
    const cd zero = mk(0, 0);
    cd* gb = a.g + (size_t)b * ns * nt;
    const cd* bb = a.base + (size_t)b * ns * kGenTb;
    const cd* rec = a.pcr + (size_t)v * a.rec;
    // slots handled by this thread: o0 = tid, o1 = tid + kGenThreads
    int sl[2], sr[2];
    cd cl[2][kGenTb - 1], cr[2][kGenTb - 1];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int o = tid + h * kGenThreads;
        sl[h] = sr[h] = -1;
#pragma unroll
        for (int m = 0; m < kGenTb - 1; ++m) { cl[h][m] = zero; cr[h][m] = zero; }
        if (o < ns) {
            int k, pl, pr;
            slot_src(o, a.N, k, pl, pr, sl[h], sr[h]);
            const cd* base = a.cols + (size_t)(v * a.N + k) * 4 * nt;
#pragma unroll
            for (int m = 0; m < kGenTb - 1; ++m) {
                const int lag = m + 1;
                if (lag < nt) {
                    if (sl[h] >= 0) cl[h][m] = base[(size_t)pl * nt + lag];
                    if (sr[h] >= 0) cr[h][m] = base[(size_t)pr * nt + lag];
                }
            }
        }
    }
    for (int i = 0; i < nb; ++i) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int o = tid + h * kGenThreads;
            if (o < ns) {
                cd r = bb[(size_t)o * kGenTb + i];
#pragma unroll
                for (int m = 0; m < kGenTb - 1; ++m) {
                    const int lag = m + 1;
                    if (lag <= i) {
                        if (sl[h] >= 0) r = madd(r, cl[h][m], gh[(size_t)(i - lag) * ns + sl[h]]);
                        if (sr[h] >= 0) r = madd(r, cr[h][m], gh[(size_t)(i - lag) * ns + sr[h]]);
                    }
                }
                rhs[o] = r;
            }
        }
        __syncthreads();
        // block PCR, one thread per interface
        const int j = tid;
        cd p0 = zero, p1 = zero;
        if (j < ni) { p0 = rhs[2 * j]; p1 = rhs[2 * j + 1]; }
        for (int l = 0; l < lv; ++l) {
            const int d = 1 << l;
            if (j < ni) { ex[2 * j] = p0; ex[2 * j + 1] = p1; }
            __syncthreads();
            if (j < ni) {
                const bool hm = j - d >= 0, hp = j + d < ni;
                const cd q0m = hm ? ex[2 * (j - d)] : zero, q1m = hm ? ex[2 * (j - d) + 1] : zero;
                const cd q0p = hp ? ex[2 * (j + d)] : zero, q1p = hp ? ex[2 * (j + d) + 1] : zero;
                const cd* K = rec + (size_t)l * 8 * ni + j;
                p0 = msub(msub(msub(msub(p0, K[0 * ni], q0m), K[1 * ni], q1m), K[4 * ni], q0p), K[5 * ni], q1p);
                p1 = msub(msub(msub(msub(p1, K[2 * ni], q0m), K[3 * ni], q1m), K[6 * ni], q0p), K[7 * ni], q1p);
            }
            __syncthreads();
        }
        if (j < ni) {
            const cd* Di = rec + (size_t)lv * 8 * ni + j;
            const cd x0 = madd(Di[0] * p0, Di[1 * ni], p1);
            const cd x1 = madd(Di[2 * ni] * p0, Di[3 * ni], p1);
            gh[(size_t)i * ns + 2 * j] = x0;
            gh[(size_t)i * ns + 2 * j + 1] = x1;
            gb[(size_t)(2 * j) * nt + n0 + i] = x0;
            gb[(size_t)(2 * j + 1) * nt + n0 + i] = x1;
        }
        __syncthreads();
    }
}

hipError_t launch_causal_pcr_setup_gen(int N, int nt, int nv, const cd* cols, cd* pcr, double* eta,
                                       hipStream_t st) {
    if (N - 1 > kGenMaxIf) return hipErrorInvalidValue;
    causal_pcr_setup_gen_kernel<<<nv, kGenThreads, 0, st>>>(N, nt, cols, pcr, pcr_rec_gen(N), eta);
    return hipGetLastError();
}

hipError_t launch_causal_gen(int N, int nt, int ns, int B, int per_problem, const cd* cols,
                             const cd* pcr, const cd* d, cd* base, cd* g, int n_lo, int n_hi,
                             const cd* facc, int s_from, hipStream_t st) {
    const size_t shm = ((size_t)kGenTb * ns + ns + 2 * (size_t)(N - 1)) * sizeof(cd);
    if (N - 1 > kGenMaxIf || N - 1 > kGenThreads || ns > 2 * kGenThreads || shm > 160 * 1024)
        return hipErrorInvalidValue;
    if (n_lo % kGenTb != 0 || n_lo < 0 || n_hi > nt || s_from < 0 || s_from > n_lo)
        return hipErrorInvalidValue;
    for (int n0 = n_lo; n0 < n_hi; n0 += kGenTb) {
        const int nb = min(kGenTb, n_hi - n0);
        hipError_t e = launch_causal_far<kGenTb>(N, nt, ns, B, per_problem, n0, nb, cols, d, g, base,
                                                 facc, s_from, st);
        if (e != hipSuccess) return e;
        NearGenArgs na{N, nt, ns, per_problem, n0, nb, pcr_rec_gen(N), cols, pcr, base, g};
        causal_near_gen_kernel<<<B, kGenThreads, shm, st>>>(na);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace swr
