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
// rectangle, one workgroup per subdomain and pair of problems; for a batch of
// eight or more problems with one potential `causal_far_mfma_kernel`, one
// wave per subdomain and eight problems on the matrix cores);
// `causal_near_kernel` then
// marches through the block on one workgroup per problem: wave 0 runs the
// per-step PCR solve and adds the lag-1 and lag-2 history, while the other
// waves gather the lags >= 3 of the step two ahead, from the block's g kept in
// LDS and the lag coefficients kept in registers.
#include "swr_common.h"

namespace swr {

constexpr int kTb = kNearTb;                  // near block (time steps)
constexpr int kNearClasses = 4;                            // gather threads per subdomain
constexpr int kNearLags = kTb / kNearClasses;              // lags per thread: c+3, c+3+C, ...
constexpr int kNearGroup = 4;                              // lags whose loads are issued together
// gather threads: kNearClasses per subdomain, N <= kWave + 1 subdomains
constexpr int kNearGather = (kNearClasses * (kWave + 1) + kWave - 1) / kWave * kWave;
constexpr int kNearThreads = kWave + kNearGather;
constexpr int kNearCols = kNearSlots + 2;                  // slot q in column q + 1; 0 and ns + 1 stay zero
static_assert(kTb % (kNearClasses * kNearGroup) == 0, "near block: whole lag groups");
// per-potential record of the one-wave form: PCR multipliers and inverse
// diagonals [kPcrRec][64], then the near kernel's lag coefficients packed by
// thread: gather [kNearLags][4][kNearGather] (lags >= 3), solver [2][4][64]
// (lags 1, 2), zero where the coupling does not exist
constexpr size_t kNearPackG = (size_t)kNearLags * 4 * kNearGather;
constexpr size_t kFastRec = (size_t)kPcrRec * kWave + kNearPackG + 2 * 4 * kWave;
size_t causal_fast_rec() { return kFastRec; }

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
    cd* rec = pcr + (size_t)v * kFastRec + j;
    // per level: the coupling measure and the inverse diagonal block of the
    // current system, then one reduction.  Runs once per solve: keep the
    // loop rolled (the unrolled chain of 2x2 products is slow to compile).
#pragma unroll 1
    for (int l = 0; l <= kPcrLevels; ++l) {
        double e = norm_inf(inv2(D)) * (norm_inf(Lm) + norm_inf(U));
        e = wave_max(e);
        if (j == 0) eta[(size_t)v * (kPcrLevels + 1) + l] = e;
        const C2x2 Di = inv2(D);
        cd* r = rec + (size_t)(kPcrLevels * 8 + 4 * l) * kWave;
        r[0 * kWave] = Di.a; r[1 * kWave] = Di.b; r[2 * kWave] = Di.c; r[3 * kWave] = Di.d;
        if (l == kPcrLevels) break;
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
        cd* q = rec + (size_t)l * 8 * kWave;
        q[0 * kWave] = K1.a; q[1 * kWave] = K1.b; q[2 * kWave] = K1.c; q[3 * kWave] = K1.d;
        q[4 * kWave] = K2.a; q[5 * kWave] = K2.b; q[6 * kWave] = K2.c; q[7 * kWave] = K2.d;
    }
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
    const cd* facc;    // [nseg][B][ns][kCausalSuper]: contribution of each finished
                       // super-block to steps s_from .. s_from + kCausalSuper - 1
    int nseg;          // number of finished super-blocks (facc null when 0)
    int s_from;        // this kernel sums steps s_from <= s < n0
    int B;             // problems
};

// One workgroup per (subdomain k, PB problems).  Subdomain k feeds the
// output slots 2k - 2 (if k >= 1) and 2k + 1 (if k <= N - 2); both read the
// same two source rows, g of slots 2k - 1 and 2k, and with one potential the
// problems read the same coefficients, so each row is staged in LDS once for
// all its readers.  Thread (h, bb, split, i): output step n0 + i of slot
// 2k - 2 (h = 0) or 2k + 1 (h = 1) for problem b0 + bb, inputs s in the
// split's share of [s_from, n0).  out = d + the finished super-blocks'
// partials + that contribution.  The source rows over [s_from, n0) and the
// coefficient window they meet (lags 1 .. n0 + TB - s_from) are staged with
// coalesced loads (the range is less than one 256-step super-block).  Per
// output, the source split, the order of terms in each partial sum and the
// order in which the partials are added depend on TB and the range only.
// PB problems per workgroup: 2, or 1 for a single problem (no idle half)
template <int TB, int PB>
__global__ __launch_bounds__(2 * PB * 256) void causal_far_kernel(FarArgs f) {
    constexpr int SPLITS = 256 / TB;
    constexpr int kWin = kCausalSuper + TB;
    constexpr int NT = 2 * PB * 256;
    __shared__ cd part[2][PB][SPLITS][TB];
    __shared__ cd sg[2][PB][kCausalSuper];
    __shared__ cd sc[PB][4][kWin];       // [problem or 0][coefficient row p][lag]
    const int k = blockIdx.x, b0 = blockIdx.y * PB, t = threadIdx.x;
    const int i = t % TB, sp = (t / TB) % SPLITS, bb = (t / 256) % PB, h = t / (256 * PB);
    const bool hasl = k >= 1, hasr = k <= f.N - 2;      // source rows 2k - 1, 2k
    const bool act = h == 0 ? hasl : hasr;              // output slot exists
    const int o = h == 0 ? 2 * k - 2 : 2 * k + 1;
    const int b = b0 + bb;
    const int len = f.n0 - f.s_from;                    // < kCausalSuper
    const int n = f.n0 + i;
    const bool out_ok = act && b < f.B && i < f.nb;
    // d plus the finished super-blocks' partials, in that order, loaded
    // before the staging so their latency overlaps it
    cd r = mk(0, 0);
    if (out_ok && sp == 0) {
        r = f.d[((size_t)b * f.ns + o) * f.nt + n];
        const size_t seg_stride = (size_t)f.B * f.ns * kCausalSuper;
        const cd* fp = f.facc + ((size_t)b * f.ns + o) * kCausalSuper + (n - f.s_from);
        for (int q = 0; q < f.nseg; ++q) r = r + fp[q * seg_stride];
    }
    // sources: thread t stages entry e of row q for problem bq (one each);
    // coefficients: row p of subdomain k (p = 0, 1: slot 2k - 2 with the left,
    // right source; p = 2, 3: slot 2k + 1), one copy per problem if each has
    // its own potential.  All loads are issued before any store.
    static_assert(kCausalSuper == 256 && TB <= 256, "far kernel staging: one source entry per thread");
    constexpr int kCoef = PB * 4 * kWin, kCoefTrips = (kCoef + NT - 1) / NT;
    const int nc = f.per_problem ? kCoef : 4 * kWin;
    cd x = mk(0, 0), c[kCoefTrips];
    {
        const int q = t / (PB * 256), bq = (t / 256) % PB, e = t % 256;
        if ((q == 0 ? hasl : hasr) && b0 + bq < f.B && e < len)
            x = f.g[((size_t)(b0 + bq) * f.ns + 2 * k - 1 + q) * f.nt + f.s_from + e];
    }
#pragma unroll
    for (int m = 0; m < kCoefTrips; ++m) {
        const int u = t + m * NT, cb = u / (4 * kWin), p = (u / kWin) % 4, e = u % kWin;
        const bool row_ok = (p == 0 || p == 2 ? hasl : hasr) && (p < 2 ? hasl : hasr);
        const int v = f.per_problem ? b0 + cb : 0;
        c[m] = mk(0, 0);
        if (u < nc && row_ok && e < len + TB && e < f.nt && (!f.per_problem || v < f.B))
            c[m] = f.cols[((size_t)(v * f.N + k) * 4 + p) * f.nt + e];
    }
    (&sg[0][0][0])[t] = x;
#pragma unroll
    for (int m = 0; m < kCoefTrips; ++m) {
        const int u = t + m * NT;
        if (u < nc) (&sc[0][0][0])[u] = c[m];
    }
    __syncthreads();
    const int per = (len + SPLITS - 1) / SPLITS;
    const int s_lo = f.s_from + sp * per, s_hi = min(f.n0, s_lo + per);
    const cd* cl = sc[f.per_problem ? bb : 0][2 * h];
    const cd* cr = sc[f.per_problem ? bb : 0][2 * h + 1];
    double ax = 0, ay = 0;
    if (out_ok) {
        for (int s = s_lo; s < s_hi; ++s) {
            const int e = s - f.s_from, lag = n - s;
            if (hasl) {
                const cd cc = cl[lag], xx = sg[0][bb][e];
                ax += cc.x * xx.x - cc.y * xx.y;
                ay += cc.x * xx.y + cc.y * xx.x;
            }
            if (hasr) {
                const cd cc = cr[lag], xx = sg[1][bb][e];
                ax += cc.x * xx.x - cc.y * xx.y;
                ay += cc.x * xx.y + cc.y * xx.x;
            }
        }
    }
    part[h][bb][sp][i] = mk(ax, ay);
    __syncthreads();
    if (out_ok && sp == 0) {
        for (int q = 0; q < SPLITS; ++q) r = r + part[h][bb][q][i];
        f.out[((size_t)b * f.ns + o) * TB + i] = r;
    }
}

// Matrix-core form of the same sums for a batch with one potential (at least
// 8 problems, TB = 8 or 32).  One wave per (subdomain k, 8 problems): the
// rows of the product are the block's TB outputs of the two slots subdomain
// k feeds (slot 2k - 2, then slot 2k + 1: 2 TB rows in 16-row blocks), the
// columns the 8 problems' real and imaginary parts, and K runs over the
// sources s in [s_from, n0) of the left row (g of slot 2k - 1), then of the
// right row (slot 2k), four per instruction.  Two accumulators per row block
// collect Re C [Re x | Im x] and Im C [Re x | Im x]; neighbouring lanes
// combine them (Re y = Re C Re x - Im C Im x, Im y = Re C Im x + Im C Re x).
// At N = 500, B = 32 a launch has 2000 waves where the form above has
// 128000, so it finds room quickly beside the sweeps that run concurrently
// on the other streams.  Per output: d, the finished super-blocks' partials,
// then the product (sources ascending in fours, left row before right).
typedef double fd4 __attribute__((ext_vector_type(4)));
static __device__ inline fd4 far_mfma(double a, double b, fd4 c) {
    // lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator register
    // q of lane l is D[l/16 + 4q][l%16]
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
static __device__ inline double far_swap_pair(double v) {   // the value of lane l ^ 1
    int2 t = *reinterpret_cast<int2*>(&v);
    t.x = __builtin_amdgcn_mov_dpp(t.x, 0xB1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
    t.y = __builtin_amdgcn_mov_dpp(t.y, 0xB1, 0xf, 0xf, false);
    return *reinterpret_cast<double*>(&t);
}
constexpr int kFarMfmaB = 8;    // problems per wave of the matrix-core form

template <int TB>
__global__ __launch_bounds__(64) void causal_far_mfma_kernel(FarArgs f) {
    static_assert((2 * TB) % 16 == 0, "whole 16-row blocks");
    constexpr int RB = 2 * TB / 16;
    const int k = blockIdx.x, b0 = blockIdx.y * kFarMfmaB;
    const int lane = threadIdx.x, r = lane & 15, kq = lane >> 4;
    const bool hasl = k >= 1, hasr = k <= f.N - 2;       // source rows 2k - 1, 2k
    const cd* crow = f.cols + (size_t)k * 4 * f.nt;       // coefficient rows p = 0..3
    // B operand column r: problem b0 + r / 2, real (r even) or imaginary part
    const int bcol = b0 + (r >> 1), part = r & 1;
    const bool col_ok = bcol < f.B;
    fd4 d1[RB], d2[RB];
#pragma unroll
    for (int I = 0; I < RB; ++I) {
        d1[I] = fd4{0.0, 0.0, 0.0, 0.0};
        d2[I] = fd4{0.0, 0.0, 0.0, 0.0};
    }
    // operands of U k-steps are loaded one group ahead of the instructions
    // that use them (k-steps past the range load zeros)
    constexpr int U = RB == 1 ? 4 : 2;
    const int nblk = (f.n0 - f.s_from + 3) / 4;
    for (int side = 0; side < 2; ++side) {
        if (side == 0 ? !hasl : !hasr) continue;          // uniform over the wave
        const double* gs = reinterpret_cast<const double*>(
                               f.g + ((size_t)(col_ok ? bcol : 0) * f.ns + 2 * k - 1 + side) * f.nt) + part;
        double bv[2][U];
        cd av[2][U][RB];
        auto fetch = [&](int buf, int j0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int s = f.s_from + 4 * (j0 + u) + kq;
                const bool s_ok = s < f.n0;
                bv[buf][u] = (col_ok && s_ok) ? gs[2 * (size_t)s] : 0.0;
#pragma unroll
                for (int I = 0; I < RB; ++I) {
                    // A row r of block I: output R = 16 I + r, slot h = R / TB,
                    // step i = R % TB
                    const int R = 16 * I + r, h = R / TB, lag = f.n0 + R % TB - s;
                    const bool a_ok = s_ok && (h == 0 ? hasl : hasr) && lag < f.nt;
                    av[buf][u][I] = a_ok ? crow[(size_t)(2 * h + side) * f.nt + lag] : mk(0, 0);
                }
            }
        };
        auto apply = [&](int buf) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int I = 0; I < RB; ++I) {
                    d1[I] = far_mfma(av[buf][u][I].x, bv[buf][u], d1[I]);
                    d2[I] = far_mfma(av[buf][u][I].y, bv[buf][u], d2[I]);
                }
            }
        };
        fetch(0, 0);
        for (int j0 = 0; j0 < nblk; j0 += 2 * U) {
            fetch(1, j0 + U);
            apply(0);
            if (j0 + U >= nblk) break;
            fetch(0, j0 + 2 * U);
            apply(1);
        }
    }
    const size_t seg_stride = (size_t)f.B * f.ns * kCausalSuper;
#pragma unroll
    for (int I = 0; I < RB; ++I) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double other = far_swap_pair(d2[I][q]);
            const double v = part ? d1[I][q] + other : d1[I][q] - other;
            const int R = 16 * I + kq + 4 * q, h = R / TB, i = R % TB;
            if (col_ok && (h == 0 ? hasl : hasr) && i < f.nb) {
                const int o = h == 0 ? 2 * k - 2 : 2 * k + 1, n = f.n0 + i;
                const size_t row = (size_t)bcol * f.ns + o;
                double acc = reinterpret_cast<const double*>(f.d + row * f.nt + n)[part];
                for (int q2 = 0; q2 < f.nseg; ++q2)
                    acc += reinterpret_cast<const double*>(f.facc + q2 * seg_stride + row * kCausalSuper +
                                                           (n - f.s_from))[part];
                reinterpret_cast<double*>(f.out + row * TB + i)[part] = acc + v;
            }
        }
    }
}

struct NearArgs {
    int N, nt, ns, per_problem;
    int n0, nb;
    const cd* cols;
    const cd* pcr;     // [nv][kFastRec]
    int levels;        // PCR levels run per step (the rest of the coupling is negligible)
    const cd* base;    // [B][ns][kTb]: d + far part
    cd* g;             // [B][ns][nt]
};


// neighbour values for the lag-1/lag-2 history: lane j - 1 / j + 1 (zero outside)
__device__ inline cd lane_up1(cd v) { return shfl_up1z(v); }
__device__ inline cd lane_dn1(cd v) { return shfl_dn1z(v); }

// sum over the four lanes of a quad (DPP quad permutations); every lane of
// the quad gets the same bits
template <int CTRL>
__device__ inline double quad_move(double v) {
    int2 t = *reinterpret_cast<int2*>(&v);
    t.x = __builtin_amdgcn_update_dpp(0, t.x, CTRL, 0xf, 0xf, false);
    t.y = __builtin_amdgcn_update_dpp(0, t.y, CTRL, 0xf, 0xf, false);
    return *reinterpret_cast<double*>(&t);
}
__device__ inline cd quad_sum(cd v) {
    v = mk(v.x + quad_move<0xB1>(v.x), v.y + quad_move<0xB1>(v.y));   // lanes (1,0,3,2)
    return mk(v.x + quad_move<0x4E>(v.x), v.y + quad_move<0x4E>(v.y)); // lanes (2,3,0,1)
}

// One workgroup per problem.  Wave 0 solves the per-step block system; lane
// j owns interface j, i.e. slots 2j (r_j) and 2j+1 (l_{j+1}), and adds the
// lag-1 and lag-2 history itself from the solutions of the two previous
// steps it keeps in registers (slot 2j reads x1 of lane j and x0 of lane j+1
// through X^{j+1,1}, X^{j+1,2}; slot 2j+1 reads x1 of lane j-1 and x0 of lane
// j through X^{j,3}, X^{j,4}).  The other waves gather lags >= 3 of the step
// two ahead from the block's g kept in LDS, so a step costs one barrier and
// the solver never waits for LDS written in the same step.  They work per
// subdomain k: its two outgoing traces (slots 2k-1, 2k) enter exactly the
// slots 2k-2 (through X^{k,1}, X^{k,2}) and 2k+1 (through X^{k,3}, X^{k,4}),
// so each pair of LDS values read serves two slots; kNearClasses threads
// split the lags of one subdomain and sum through DPP.  Lags are taken in
// groups whose LDS loads are issued together: a source before the block or
// outside the interface range reads the zero row / zero columns of `gh`,
// which adds exact zeros.  Row s + 1 of `gh` holds, in turn, the base of step
// s (staged at the start), its full right-hand side (written by the gather
// two steps before) and its solution (written by the solver at step s).
__global__ __launch_bounds__(kNearThreads) void causal_near_kernel(NearArgs a) {
    __shared__ cd gh[kTb + 1][kNearCols];
    __shared__ cd spcr[kPcrLevels * 8 + 4][kWave];
    const int b = blockIdx.x, v = a.per_problem ? b : 0;
    const int tid = threadIdx.x;
    const int ns = a.ns, nt = a.nt, n0 = a.n0, nb = a.nb;
    const int ni = a.N - 1;
    const cd zero = mk(0, 0);
    cd* gb = a.g + (size_t)b * ns * nt;
    const cd* bb = a.base + (size_t)b * ns * kTb;
    const cd* prec = a.pcr + (size_t)v * kFastRec;
    const cd* pk = prec + (size_t)kPcrRec * kWave;   // packed lag coefficients

    // gather role: subdomain k, lag class c (lags c+3, c+3+C, c+3+2C, ...).
    // wa*: slot 2k-2 from slots 2k-1, 2k; wb*: slot 2k+1 from the same pair.
    const int gt = tid - kWave;
    const int k = gt / kNearClasses, c = gt % kNearClasses;
    const bool gather = tid >= kWave && k < a.N;
    // a gather wave with no subdomain at all skips the sums (it would add
    // zeros and hold its SIMD)
    const bool gwave = tid >= kWave && ((tid & ~(kWave - 1)) - kWave) / kNearClasses < a.N;
    const bool has_a = gather && k >= 1, has_b = gather && k <= a.N - 2;
    const int kk = gather ? k : 0;
    // (coalesced reads of the table packed once per solve)
    cd wa0[kNearLags], wa1[kNearLags], wb0[kNearLags], wb1[kNearLags];
#pragma unroll
    for (int m = 0; m < kNearLags; ++m) { wa0[m] = zero; wa1[m] = zero; wb0[m] = zero; wb1[m] = zero; }
    if (tid >= kWave) {
#pragma unroll
        for (int m = 0; m < kNearLags; ++m) {
            const cd* q = pk + (size_t)m * 4 * kNearGather + gt;
            wa0[m] = q[0];
            wa1[m] = q[kNearGather];
            wb0[m] = q[2 * kNearGather];
            wb1[m] = q[3 * kNearGather];
        }
    }
    // solver role: lag-1 and lag-2 coefficients of my two slots
    const int j = tid;
    cd a0[2] = {zero, zero}, a1[2] = {zero, zero}, a2[2] = {zero, zero}, a3[2] = {zero, zero};
    if (tid < kWave) {
        const cd* q = pk + kNearPackG + j;
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            a0[l] = q[(l * 4 + 0) * kWave];
            a1[l] = q[(l * 4 + 1) * kWave];
            a2[l] = q[(l * 4 + 2) * kWave];
            a3[l] = q[(l * 4 + 3) * kWave];
        }
    }
    // base (d + far part) of every step of the block -> its row of gh; then
    // the multipliers of the levels run and the matching inverse diagonal ->
    // LDS.  The lag coefficients above and the base are in flight together,
    // so the set-up waits for one round of memory latency (two when PCR
    // levels run).
    const int lev = a.levels;
    {
        constexpr int kIt = (kNearSlots * kTb + kNearThreads - 1) / kNearThreads;
        const int lim = ns * nb;
        // q = e / nb as (e * ceil(2^32 / nb)) >> 32: exact for e < 2^32 / kTb
        const unsigned long long rnb = (0x100000000ull + nb - 1) / nb;
        cd t[kIt];
#pragma unroll
        for (int u = 0; u < kIt; ++u) {
            const int e = tid + u * kNearThreads;
            const int q = (int)(((unsigned long long)e * rnb) >> 32), s = e - q * nb;
            t[u] = zero;
            if (e < lim) t[u] = bb[(size_t)q * kTb + s];
        }
#pragma unroll
        for (int u = 0; u < kIt; ++u) {
            const int e = tid + u * kNearThreads;
            const int q = (int)(((unsigned long long)e * rnb) >> 32), s = e - q * nb;
            if (e < lim) gh[s + 1][q + 1] = t[u];
        }
    }
    {
        constexpr int kIt = (kPcrLevels * 8 * kWave + kNearThreads - 1) / kNearThreads;
        const int lim = lev * 8 * kWave;
        cd t[kIt];
        cd di = zero;
#pragma unroll
        for (int u = 0; u < kIt; ++u) {
            const int e = tid + u * kNearThreads;
            t[u] = zero;
            if (e < lim) t[u] = prec[e];
        }
        if (tid < 4 * kWave) di = prec[(size_t)(kPcrLevels * 8 + 4 * lev) * kWave + tid];
#pragma unroll
        for (int u = 0; u < kIt; ++u) {
            const int e = tid + u * kNearThreads;
            if (e < lim) (&spcr[0][0])[e] = t[u];
        }
        if (tid < 4 * kWave) (&spcr[kPcrLevels * 8][0])[tid] = di;
    }
    // zero row (steps before the block) and zero columns (no such slot)
    for (int e = tid; e < kNearCols; e += kNearThreads) gh[0][e] = zero;
    for (int e = tid; e < kTb; e += kNearThreads) {
        gh[e + 1][0] = zero;
        gh[e + 1][ns + 1] = zero;
    }
    cd x0 = zero, x1 = zero, y0 = zero, y1 = zero;   // solutions of steps i-1 and i-2
    __syncthreads();
    // every load of the set-up has landed: the step loop then waits on no
    // memory counter, so its stores never hold a step
    __builtin_amdgcn_s_waitcnt(0);
    // lag-1 and lag-2 part of the next step's right-hand side, formed from
    // the solver's own registers before the step's barrier
    cd h0 = zero, h1 = zero;
    // neighbour values of the previous step's solution (lane j+1's x0, lane
    // j-1's x1): this step's lag-2 neighbours, shuffled once
    cd x0p = zero, x1m = zero;

    for (int i = 0; i < nb; ++i) {
        if (tid < kWave) {
            // right-hand side: base + lags >= 3 (gathered; steps 0 and 1 have
            // none in the block) + lags 1, 2 (h); lags reaching before the
            // block are in base
            cd p0 = zero, p1 = zero;
            if (j < ni) { p0 = gh[i + 1][2 * j + 1] + h0; p1 = gh[i + 1][2 * j + 2] + h1; }
#pragma unroll
            for (int l = 0; l < kPcrLevels; ++l) {
                if (l >= lev) break;                    // uniform over the workgroup
                // the multipliers are zero on lanes without a partner
                const int d = 1 << l;
                const cd q0m = shfl_up_raw(p0, d), q1m = shfl_up_raw(p1, d);
                const cd q0p = shfl_dn_raw(p0, d), q1p = shfl_dn_raw(p1, d);
                const cd* K = &spcr[l * 8][j];
                const cd k1a = K[0 * kWave], k1b = K[1 * kWave], k1c = K[2 * kWave], k1d = K[3 * kWave];
                const cd k2a = K[4 * kWave], k2b = K[5 * kWave], k2c = K[6 * kWave], k2d = K[7 * kWave];
                p0 = msub(msub(msub(msub(p0, k1a, q0m), k1b, q1m), k2a, q0p), k2b, q1p);
                p1 = msub(msub(msub(msub(p1, k1c, q0m), k1d, q1m), k2c, q0p), k2d, q1p);
            }
            const cd* Di = &spcr[kPcrLevels * 8][j];
            y0 = x0;
            y1 = x1;
            x0 = madd(Di[0] * p0, Di[1 * kWave], p1);
            x1 = madd(Di[2 * kWave] * p0, Di[3 * kWave], p1);
            if (j >= ni) { x0 = zero; x1 = zero; }
            if (j < ni) {
                gh[i + 1][2 * j + 1] = x0;
                gh[i + 1][2 * j + 2] = x1;
                gb[(size_t)(2 * j) * nt + n0 + i] = x0;
                gb[(size_t)(2 * j + 1) * nt + n0 + i] = x1;
            }
            // lags 1 (this step) and 2 (the step before) for step i+1
            const cd y0p = x0p, y1m = x1m;
            x0p = lane_dn1(x0);
            x1m = lane_up1(x1);
            h0 = madd(a1[0] * x0p, a0[0], x1);
            h1 = madd(a3[0] * x0, a2[0], x1m);
            if (i >= 1) {
                h0 = madd(madd(h0, a0[1], y1), a1[1], y0p);
                h1 = madd(madd(h1, a2[1], y1m), a3[1], y0);
            }
        } else if (gwave && i + 2 < nb) {
            // lags >= 3 of step i+2, from in-block steps up to i-1: lag
            // c+3+C*m reads row i - c - C*m (step i+2-lag), row 0 if earlier
            cd pa = zero, pb = zero;
#pragma unroll
            for (int g0 = 0; g0 < kNearLags; g0 += kNearGroup) {
                // first lag of the group: 3 + C*g0 <= i + 2 for some class
                if (i >= 1 + kNearClasses * g0) {
                    cd xl[kNearGroup], xr[kNearGroup];
#pragma unroll
                    for (int u = 0; u < kNearGroup; ++u) {
                        const int r = max(i - c - kNearClasses * (g0 + u), 0);
                        xl[u] = gh[r][2 * kk];
                        xr[u] = gh[r][2 * kk + 1];
                    }
#pragma unroll
                    for (int u = 0; u < kNearGroup; ++u) {
                        pa = madd(madd(pa, wa0[g0 + u], xl[u]), wa1[g0 + u], xr[u]);
                        pb = madd(madd(pb, wb0[g0 + u], xl[u]), wb1[g0 + u], xr[u]);
                    }
                }
            }
            pa = quad_sum(pa);
            pb = quad_sum(pb);
            if (c == 0 && has_a) gh[i + 3][2 * k - 1] = gh[i + 3][2 * k - 1] + pa;   // slot 2k-2
            if (c == 1 && has_b) gh[i + 3][2 * k + 2] = gh[i + 3][2 * k + 2] + pb;   // slot 2k+1
        }
        __syncthreads();
    }
}

// The near kernel's lag coefficients of one potential, packed by thread so
// that every launch reads them with coalesced loads: gather thread gt
// (subdomain k = gt / C, class c) gets, for lag c+3+C*m, X^{k,1..4} (those of
// slot 2k-2 from slots 2k-1, 2k and of slot 2k+1 from the same pair); solver
// lane j gets the lag-1 and lag-2 values of its two slots.  Zero where the
// slot or the source does not exist, or the lag is past nt or the near block.
__global__ __launch_bounds__(kNearGather) void causal_near_pack_kernel(int N, int nt, const cd* cols,
                                                                       cd* pcr) {
    const int v = blockIdx.x, gt = threadIdx.x;
    const cd zero = mk(0, 0);
    const cd* cbase = cols + (size_t)v * N * 4 * nt;
    cd* pk = pcr + (size_t)v * kFastRec + (size_t)kPcrRec * kWave;
    const int k = gt / kNearClasses, c = gt % kNearClasses;
    const bool gather = k < N;
    const bool has_a = gather && k >= 1, has_b = gather && k <= N - 2;
    const cd* cb = cbase + (size_t)(gather ? k : 0) * 4 * nt;
    for (int m = 0; m < kNearLags; ++m) {
        const int lag = c + 3 + kNearClasses * m;
        cd w0 = zero, w1 = zero, w2 = zero, w3 = zero;
        if (lag < nt && lag < kTb) {
            if (has_a) {
                w0 = cb[lag];
                if (k <= N - 2) w1 = cb[(size_t)nt + lag];
            }
            if (has_b) {
                if (k >= 1) w2 = cb[(size_t)2 * nt + lag];
                w3 = cb[(size_t)3 * nt + lag];
            }
        }
        cd* q = pk + (size_t)m * 4 * kNearGather + gt;
        q[0] = w0;
        q[kNearGather] = w1;
        q[2 * kNearGather] = w2;
        q[3 * kNearGather] = w3;
    }
    if (gt < kWave) {
        const int j = gt, ni = N - 1;
        cd* q = pk + kNearPackG + j;
        for (int l = 0; l < 2; ++l) {
            const int lag = l + 1;
            cd x0 = zero, x1 = zero, x2 = zero, x3 = zero;
            if (j < ni && lag < nt) {
                x0 = cbase[((size_t)(j + 1) * 4 + 0) * nt + lag];                        // x1_j
                if (j + 1 <= N - 2) x1 = cbase[((size_t)(j + 1) * 4 + 1) * nt + lag];   // x0_{j+1}
                if (j >= 1) x2 = cbase[((size_t)j * 4 + 2) * nt + lag];                  // x1_{j-1}
                x3 = cbase[((size_t)j * 4 + 3) * nt + lag];                              // x0_j
            }
            q[(l * 4 + 0) * kWave] = x0;
            q[(l * 4 + 1) * kWave] = x1;
            q[(l * 4 + 2) * kWave] = x2;
            q[(l * 4 + 3) * kWave] = x3;
        }
    }
}

hipError_t launch_causal_pcr_setup(int N, int nt, int nv, const cd* cols, cd* pcr, double* eta,
                                   hipStream_t st) {
    if (N > kWave + 1) return hipErrorInvalidValue;
    causal_pcr_setup_kernel<<<nv, 64, 0, st>>>(N, nt, cols, pcr, eta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    causal_near_pack_kernel<<<nv, kNearGather, 0, st>>>(N, nt, cols, pcr);
    return hipGetLastError();
}

template <int TB>
static hipError_t launch_causal_far(int N, int nt, int ns, int B, int per_problem, int n0, int nb,
                                    const cd* cols, const cd* d, const cd* g, cd* out,
                                    const cd* facc, int s_from, hipStream_t st) {
    // the staged rows hold less than one super-block of sources
    if (n0 - s_from < 0 || n0 - s_from >= kCausalSuper) return hipErrorInvalidValue;
    if (ns != 2 * (N - 1)) return hipErrorInvalidValue;
    FarArgs f{N, nt, ns, per_problem, n0, nb, cols, d, g, out, facc,
              facc ? s_from / kCausalSuper : 0, s_from, B};
    if constexpr (TB == 8 || TB == 32) {
        if (!per_problem && B >= kFarMfmaB) {
            causal_far_mfma_kernel<TB><<<dim3(N, (B + kFarMfmaB - 1) / kFarMfmaB), 64, 0, st>>>(f);
            return hipGetLastError();
        }
    }
    if (B == 1) causal_far_kernel<TB, 1><<<dim3(N, 1), 2 * 256, 0, st>>>(f);
    else causal_far_kernel<TB, 2><<<dim3(N, (B + 1) / 2), 2 * 2 * 256, 0, st>>>(f);
    return hipGetLastError();
}

hipError_t launch_causal_near(int N, int nt, int ns, int B, int per_problem, int n0, int nb,
                              const cd* cols, const cd* pcr, int levels, const cd* base, cd* g,
                              hipStream_t st) {
    if (ns > kNearSlots || N - 1 > kWave || levels < 0 || levels > kPcrLevels)
        return hipErrorInvalidValue;
    NearArgs a{N, nt, ns, per_problem, n0, nb, cols, pcr, levels, base, g};
    causal_near_kernel<<<B, kNearThreads, 0, st>>>(a);
    return hipGetLastError();
}

// the whole forward substitution: far part then near march, block by block
hipError_t launch_causal_fast(int N, int nt, int ns, int B, int per_problem, const cd* cols,
                              const cd* pcr, int levels, const cd* d, cd* base, cd* g, int n_lo,
                              int n_hi, const cd* facc, int s_from, hipStream_t st) {
    if (n_lo % kTb != 0 || n_lo < 0 || n_hi > nt || s_from < 0 || s_from > n_lo)
        return hipErrorInvalidValue;
    for (int n0 = n_lo; n0 < n_hi; n0 += kTb) {
        const int nb = min(kTb, n_hi - n0);
        hipError_t e = launch_causal_far<kTb>(N, nt, ns, B, per_problem, n0, nb, cols, d, g, base,
                                              facc, s_from, st);
        if (e != hipSuccess) return e;
        e = launch_causal_near(N, nt, ns, B, per_problem, n0, nb, cols, pcr, levels, base, g, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// General path: up to kGenMaxIf interfaces.  Same algebra as above with the
// block PCR spread over the workgroup (one thread per interface, exchange
// through LDS) and a short near block of TB steps (gen_threads / gen_tb).
// ---------------------------------------------------------------------------

// multipliers [nv][levels][8][ni] then D^{-1} [nv][4][ni] (after the levels).
// The neighbours' blocks are exchanged through LDS in two rounds (D and L,
// then U), so 1024 interfaces fit.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void causal_pcr_setup_gen_kernel(int N, int nt, const cd* cols,
                                                                      cd* pcr, int rec, double* eta) {
    __shared__ C2x2 sA[THREADS], sB[THREADS];
    __shared__ double se[THREADS / kWave];
    const int v = blockIdx.x, j = threadIdx.x;
    const int ni = N - 1, lv = pcr_levels_for(ni);
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
    cd* rec_v = pcr + (size_t)v * rec;
    // per level: coupling measure and inverse diagonal block of the current
    // system (eta[v][l], Dinv block l), then one reduction
#pragma unroll 1
    for (int l = 0; l <= lv; ++l) {
        double e = (j < ni) ? norm_inf(inv2(D)) * (norm_inf(Lm) + norm_inf(U)) : 0.0;
        e = wave_max(e);
        if ((j & (kWave - 1)) == 0) se[j / kWave] = e;
        __syncthreads();
        if (j == 0) {
            double m = 0;
            for (int w = 0; w < THREADS / kWave; ++w) m = fmax(m, se[w]);
            eta[(size_t)v * (kGenLevelsMax + 1) + l] = m;
        }
        if (j < ni) {
            const C2x2 Di = inv2(D);
            cd* r = rec_v + ((size_t)lv * 8 + 4 * l) * ni + j;
            r[0 * ni] = Di.a; r[1 * ni] = Di.b; r[2 * ni] = Di.c; r[3 * ni] = Di.d;
        }
        if (l == lv) break;
        const int d = 1 << l;
        const bool hm = j - d >= 0, hp = j + d < ni;
        if (j < ni) { sA[j] = D; sB[j] = Lm; }
        __syncthreads();
        C2x2 Dm = I, Lmm = Z, Dp = I, Lp = Z, Um = Z, Up = Z;
        if (j < ni) {
            if (hm) { Dm = sA[j - d]; Lmm = sB[j - d]; }
            if (hp) { Dp = sA[j + d]; Lp = sB[j + d]; }
        }
        __syncthreads();
        if (j < ni) sA[j] = U;
        __syncthreads();
        if (j < ni) {
            if (hm) Um = sA[j - d];
            if (hp) Up = sA[j + d];
        }
        C2x2 K1 = Z, K2 = Z;
        if (j < ni) {
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
}

struct NearGenArgs {
    int N, nt, ns, per_problem;
    int n0, nb, rec;
    int levels;        // PCR levels run per step (the rest of the coupling is negligible)
    const cd* cols;
    const cd* pcr;     // [nv][rec]
    const cd* base;    // [B][ns][TB]: d + far part
    cd* g;             // [B][ns][nt]
};

// one workgroup per problem; per step: gather the in-block history of every
// slot (coefficients of lags 1..TB-1 in registers), then block PCR
// One thread per interface j (slots 2j, 2j+1).  Per step: the right-hand
// side from the base and the in-block lags (coefficients in registers,
// earlier solutions in LDS), then the levels of block PCR exchanging through
// two alternating LDS buffers (one barrier per level), with the multipliers
// of the next level loaded while the current one runs.
template <int THREADS, int TB>
__global__ __launch_bounds__(THREADS) void causal_near_gen_kernel(NearGenArgs a) {
    extern __shared__ cd smem[];
    const int ns = a.ns, nt = a.nt, n0 = a.n0, nb = a.nb, ni = a.N - 1;
    cd* gh = smem;                          // [TB][ns]
    cd* xa = gh + (size_t)TB * ns;          // [ns] exchange, even levels
    cd* xb = xa + ns;                       // [ns] exchange, odd levels
    const int b = blockIdx.x, v = a.per_problem ? b : 0;
    const int j = threadIdx.x;
    const bool act = j < ni;
    const bool has_r = j + 1 <= a.N - 2, has_l = j >= 1;
    const int lv = pcr_levels_for(ni);
    const cd zero = mk(0, 0);
    cd* gb = a.g + (size_t)b * ns * nt;
    const cd* bb = a.base + (size_t)b * ns * TB;
    const cd* rec = a.pcr + (size_t)v * a.rec;
    const cd* cb = a.cols + (size_t)v * a.N * 4 * nt;
    // lag m+1 coefficients: slot 2j <- x1_j (c0), x0_{j+1} (c1);
    //                       slot 2j+1 <- x1_{j-1} (c2), x0_j (c3)
    cd c0[TB - 1], c1[TB - 1], c2[TB - 1], c3[TB - 1];
#pragma unroll
    for (int m = 0; m < TB - 1; ++m) {
        const int lag = m + 1;
        c0[m] = c1[m] = c2[m] = c3[m] = zero;
        if (act && lag < nt) {
            c0[m] = cb[((size_t)(j + 1) * 4 + 0) * nt + lag];
            if (has_r) c1[m] = cb[((size_t)(j + 1) * 4 + 1) * nt + lag];
            if (has_l) c2[m] = cb[((size_t)j * 4 + 2) * nt + lag];
            c3[m] = cb[((size_t)j * 4 + 3) * nt + lag];
        }
    }
    const int lev = a.levels;
    cd di0 = zero, di1 = zero, di2 = zero, di3 = zero;
    if (act) {
        const cd* Di = rec + ((size_t)lv * 8 + 4 * lev) * ni + j;
        di0 = Di[0]; di1 = Di[1 * ni]; di2 = Di[2 * ni]; di3 = Di[3 * ni];
    }
    auto loadK = [rec, ni, j, act](int l, cd (&K)[8]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) K[q] = act ? rec[((size_t)l * 8 + q) * ni + j] : mk(0, 0);
    };
    // the 512-thread form loads the next level's multipliers while the
    // current level runs; the 1024-thread form (128 registers) loads each
    // level's when it starts
    constexpr bool kPrefetch = THREADS <= 512;
    cd Kc[8], Kn[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) Kc[q] = zero;
    if (lev > 0) loadK(0, Kc);
    // base of my two slots for every step of the block -> their entries of
    // gh (only this thread reads them before its step overwrites them with
    // the solution); the step loop touches no global memory
    if (act) {
        cd t0[TB], t1[TB];
#pragma unroll
        for (int i = 0; i < TB; ++i) {
            t0[i] = zero;
            t1[i] = zero;
            if (i < nb) {
                t0[i] = bb[(size_t)(2 * j) * TB + i];
                t1[i] = bb[(size_t)(2 * j + 1) * TB + i];
            }
        }
#pragma unroll
        for (int i = 0; i < TB; ++i) {
            if (i < nb) {
                gh[(size_t)i * ns + 2 * j] = t0[i];
                gh[(size_t)i * ns + 2 * j + 1] = t1[i];
            }
        }
    }

#pragma unroll
    for (int i = 0; i < TB; ++i) {
        if (i < nb) {
            cd p0 = zero, p1 = zero;
            if (act) {
                p0 = gh[(size_t)i * ns + 2 * j];
                p1 = gh[(size_t)i * ns + 2 * j + 1];
#pragma unroll
                for (int m = 0; m < TB - 1; ++m) {
                    const int lag = m + 1;
                    if (lag <= i) {
                        const cd* gs = gh + (size_t)(i - lag) * ns;
                        p0 = madd(p0, c0[m], gs[2 * j + 1]);
                        if (has_r) p0 = madd(p0, c1[m], gs[2 * j + 2]);
                        if (has_l) p1 = madd(p1, c2[m], gs[2 * j - 1]);
                        p1 = madd(p1, c3[m], gs[2 * j]);
                    }
                }
            }
            for (int l = 0; l < lev; ++l) {
                const int d = 1 << l;
                if (kPrefetch) loadK(l + 1 < lev ? l + 1 : 0, Kn);   // next level (or next step's first)
                else loadK(l, Kc);
                cd* ex = (l & 1) ? xb : xa;
                if (act) { ex[2 * j] = p0; ex[2 * j + 1] = p1; }
                __syncthreads();
                if (act) {
                    const bool hm = j - d >= 0, hp = j + d < ni;
                    const cd q0m = hm ? ex[2 * (j - d)] : zero, q1m = hm ? ex[2 * (j - d) + 1] : zero;
                    const cd q0p = hp ? ex[2 * (j + d)] : zero, q1p = hp ? ex[2 * (j + d) + 1] : zero;
                    p0 = msub(msub(msub(msub(p0, Kc[0], q0m), Kc[1], q1m), Kc[4], q0p), Kc[5], q1p);
                    p1 = msub(msub(msub(msub(p1, Kc[2], q0m), Kc[3], q1m), Kc[6], q0p), Kc[7], q1p);
                }
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (kPrefetch) Kc[q] = Kn[q];
            }
            if (act) {
                const cd x0 = madd(di0 * p0, di1, p1);
                const cd x1 = madd(di2 * p0, di3, p1);
                gh[(size_t)i * ns + 2 * j] = x0;
                gh[(size_t)i * ns + 2 * j + 1] = x1;
            }
            __syncthreads();
        }
    }
    // my two slots' solutions of the block -> memory (kept out of the step
    // loop: its multiplier loads would otherwise wait for these stores)
    if (act) {
#pragma unroll
        for (int i = 0; i < TB; ++i) {
            if (i < nb) {
                gb[(size_t)(2 * j) * nt + n0 + i] = gh[(size_t)i * ns + 2 * j];
                gb[(size_t)(2 * j + 1) * nt + n0 + i] = gh[(size_t)i * ns + 2 * j + 1];
            }
        }
    }
}

hipError_t launch_causal_pcr_setup_gen(int N, int nt, int nv, const cd* cols, cd* pcr, double* eta,
                                       hipStream_t st) {
    if (N - 1 > kGenMaxIf) return hipErrorInvalidValue;
    if (gen_threads(N) == 512)
        causal_pcr_setup_gen_kernel<512><<<nv, 512, 0, st>>>(N, nt, cols, pcr, pcr_rec_gen(N), eta);
    else
        causal_pcr_setup_gen_kernel<1024><<<nv, 1024, 0, st>>>(N, nt, cols, pcr, pcr_rec_gen(N), eta);
    return hipGetLastError();
}

hipError_t launch_causal_gen(int N, int nt, int ns, int B, int per_problem, const cd* cols,
                             const cd* pcr, int levels, const cd* d, cd* base, cd* g, int n_lo,
                             int n_hi, const cd* facc, int s_from, hipStream_t st) {
    const size_t shm = gen_shm(N);
    const int tb = gen_tb(N), threads = gen_threads(N);
    if (N - 1 > kGenMaxIf || N - 1 > threads || ns != 2 * (N - 1) || shm > 160 * 1024)
        return hipErrorInvalidValue;
    if (levels < 0 || levels > pcr_levels_for(N - 1)) return hipErrorInvalidValue;
    if (n_lo % tb != 0 || n_lo < 0 || n_hi > nt || s_from < 0 || s_from > n_lo)
        return hipErrorInvalidValue;
    for (int n0 = n_lo; n0 < n_hi; n0 += tb) {
        const int nb = min(tb, n_hi - n0);
        hipError_t e = (tb == 8)
            ? launch_causal_far<8>(N, nt, ns, B, per_problem, n0, nb, cols, d, g, base, facc, s_from, st)
            : launch_causal_far<2>(N, nt, ns, B, per_problem, n0, nb, cols, d, g, base, facc, s_from, st);
        if (e != hipSuccess) return e;
        NearGenArgs na{N, nt, ns, per_problem, n0, nb, pcr_rec_gen(N), levels, cols, pcr, base, g};
        if (tb == 8) causal_near_gen_kernel<512, 8><<<B, 512, shm, st>>>(na);
        else causal_near_gen_kernel<1024, 2><<<B, 1024, shm, st>>>(na);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace swr
