// swr_common.h -- types and wave-level helpers shared by the SWR kernels.
//
// All arithmetic is FP64 complex, interleaved (re, im) -- the layout of
// std::complex<double> / torch.complex128.  One wavefront is 64 lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swr {

constexpr int kWave = 64;

struct __align__(16) cd {
    double x, y;
};

__host__ __device__ inline cd mk(double x, double y) { cd r; r.x = x; r.y = y; return r; }
__host__ __device__ inline cd operator+(cd a, cd b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cd operator-(cd a, cd b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cd operator-(cd a) { return mk(-a.x, -a.y); }
__host__ __device__ inline cd operator*(cd a, cd b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline cd operator*(double s, cd a) { return mk(s * a.x, s * a.y); }
__host__ __device__ inline cd conjc(cd a) { return mk(a.x, -a.y); }
__host__ __device__ inline double abs2(cd a) { return a.x * a.x + a.y * a.y; }
// 1/z as conj(z)/|z|^2 (reciprocal-multiply; only used outside the time loop)
__host__ __device__ inline cd inv(cd a) { double s = 1.0 / abs2(a); return mk(a.x * s, -a.y * s); }
// i*a
__host__ __device__ inline cd mul_i(cd a) { return mk(-a.y, a.x); }
// a - b*c (one complex multiply-subtract)
__host__ __device__ inline cd msub(cd a, cd b, cd c) {
    return mk(a.x - b.x * c.x + b.y * c.y, a.y - b.x * c.y - b.y * c.x);
}
// a + b*c
__host__ __device__ inline cd madd(cd a, cd b, cd c) {
    return mk(a.x + b.x * c.x - b.y * c.y, a.y + b.x * c.y + b.y * c.x);
}

__device__ inline int lane_id() { return __lane_id(); }

__device__ inline double rdlane(double v, int l) {
    int2 t = *reinterpret_cast<int2*>(&v);
    t.x = __builtin_amdgcn_readlane(t.x, l);
    t.y = __builtin_amdgcn_readlane(t.y, l);
    return *reinterpret_cast<double*>(&t);
}
__device__ inline cd rdlane(cd v, int l) { return mk(rdlane(v.x, l), rdlane(v.y, l)); }

// whole-wave shift of one double by one lane through DPP (CTRL 0x138: lane
// i reads lane i - 1; 0x130: lane i reads lane i + 1); the lane without a
// source reads 0 (bound_ctrl: no old value to materialise)
template <int CTRL>
__device__ inline double dpp_shift(double v) {
    int2 t = *reinterpret_cast<int2*>(&v);
    t.x = __builtin_amdgcn_mov_dpp(t.x, CTRL, 0xf, 0xf, true);
    t.y = __builtin_amdgcn_mov_dpp(t.y, CTRL, 0xf, 0xf, true);
    return *reinterpret_cast<double*>(&t);
}

// Row moves of one double through the gfx950 lane swaps (rows = 16 lanes).
// With both operands equal to x, v_permlane16_swap returns
//   first  = (x.row0, x.row0, x.row2, x.row2)   second = (x.row1, x.row1, x.row3, x.row3)
// and v_permlane32_swap returns
//   first  = (x.row0, x.row1, x.row0, x.row1)   second = (x.row2, x.row3, x.row2, x.row3).
struct RowPair { double first, second; };
__device__ inline RowPair swap16(double v) {
    int2 t = *reinterpret_cast<int2*>(&v);
    const auto lo = __builtin_amdgcn_permlane16_swap(t.x, t.x, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(t.y, t.y, false, false);
    int2 f = make_int2(lo[0], hi[0]), s = make_int2(lo[1], hi[1]);
    return RowPair{*reinterpret_cast<double*>(&f), *reinterpret_cast<double*>(&s)};
}
__device__ inline RowPair swap32(double v) {
    int2 t = *reinterpret_cast<int2*>(&v);
    const auto lo = __builtin_amdgcn_permlane32_swap(t.x, t.x, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(t.y, t.y, false, false);
    int2 f = make_int2(lo[0], hi[0]), s = make_int2(lo[1], hi[1]);
    return RowPair{*reinterpret_cast<double*>(&f), *reinterpret_cast<double*>(&s)};
}
// value of lane - 16 (rows 1..3) and of lane + 16 (rows 0..2)
__device__ inline double up16(double v) {
    const RowPair a = swap16(v);
    const double r2 = swap32(a.second).first;          // row 2 <- row 1
    const int row = lane_id() >> 4;
    return row == 2 ? r2 : a.first;                    // rows 1, 3 <- rows 0, 2
}
__device__ inline double dn16(double v) {
    const RowPair a = swap16(v);
    const double r1 = swap32(a.first).second;          // row 1 <- row 2
    const int row = lane_id() >> 4;
    return row == 1 ? r1 : a.second;                   // rows 0, 2 <- rows 1, 3
}

// value of lane (lane - d); lanes below d receive `fill`.  Distance 1 is a
// DPP wave shift, distances 16 and 32 are lane swaps (no LDS round trip),
// other distances a permute.  All run on every lane of the wave.
__device__ inline cd shfl_up_c(cd v, int d, cd fill) {
    if (d == 1) {
        const cd r = mk(dpp_shift<0x138>(v.x), dpp_shift<0x138>(v.y));
        return lane_id() == 0 ? fill : r;
    }
    if (d == 32) {
        const cd r = mk(swap32(v.x).first, swap32(v.y).first);
        return lane_id() < 32 ? fill : r;
    }
    if (d == 16) {
        const cd r = mk(up16(v.x), up16(v.y));
        return lane_id() < 16 ? fill : r;
    }
    int src = lane_id() - d;
    cd r = mk(__shfl(v.x, src < 0 ? 0 : src), __shfl(v.y, src < 0 ? 0 : src));
    return src < 0 ? fill : r;
}
// value of lane (lane + d); lanes with lane + d >= 64 receive `fill`
__device__ inline cd shfl_dn_c(cd v, int d, cd fill) {
    if (d == 1) {
        const cd r = mk(dpp_shift<0x130>(v.x), dpp_shift<0x130>(v.y));
        return lane_id() == kWave - 1 ? fill : r;
    }
    if (d == 32) {
        const cd r = mk(swap32(v.x).second, swap32(v.y).second);
        return lane_id() >= 32 ? fill : r;
    }
    if (d == 16) {
        const cd r = mk(dn16(v.x), dn16(v.y));
        return lane_id() >= kWave - 16 ? fill : r;
    }
    int src = lane_id() + d;
    cd r = mk(__shfl(v.x, src > 63 ? 63 : src), __shfl(v.y, src > 63 ? 63 : src));
    return src > 63 ? fill : r;
}

// Value of lane - 1 / lane + 1 with zero where there is none: the DPP shift
// already reads zero there, so no select is needed
__device__ inline cd shfl_up1z(cd v) { return mk(dpp_shift<0x138>(v.x), dpp_shift<0x138>(v.y)); }
__device__ inline cd shfl_dn1z(cd v) { return mk(dpp_shift<0x130>(v.x), dpp_shift<0x130>(v.y)); }

// The same moves without the fill: lanes with no source get some other
// lane's (finite) value.  For reductions whose multiplier is exactly zero on
// those lanes (the PCR levels), the product is zero and the select is saved.
__device__ inline cd shfl_up_raw(cd v, int d) {
    if (d == 1) return mk(dpp_shift<0x138>(v.x), dpp_shift<0x138>(v.y));
    if (d == 32) return mk(swap32(v.x).first, swap32(v.y).first);
    if (d == 16) return mk(up16(v.x), up16(v.y));
    const int src = (lane_id() - d) & (kWave - 1);
    return mk(__shfl(v.x, src), __shfl(v.y, src));
}
__device__ inline cd shfl_dn_raw(cd v, int d) {
    if (d == 1) return mk(dpp_shift<0x130>(v.x), dpp_shift<0x130>(v.y));
    if (d == 32) return mk(swap32(v.x).second, swap32(v.y).second);
    if (d == 16) return mk(dn16(v.x), dn16(v.y));
    const int src = (lane_id() + d) & (kWave - 1);
    return mk(__shfl(v.x, src), __shfl(v.y, src));
}

__device__ inline double wave_max(double v) {
    for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d));
    return v;
}
__device__ inline double wave_sum(double v) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// ---------------------------------------------------------------------------
// Problem-wide constants handed to every kernel.
// ---------------------------------------------------------------------------
// kernel forms of the transmission operator: Robin, S0^2, the general
// convolution form that carries S0^3, S0^4, S1^2 and S1^4 (EndCoef), and the
// Pade strategy's auxiliary-function form (S2^{2,m}, S2^{4,m})
enum Trans { TR_ROBIN = 0, TR_S02 = 1, TR_GEN = 2, TR_PADE = 3 };
// Pade strategy: at most two auxiliary functions of each end per lane
constexpr int kPadeMax = 2 * 64;

// Coefficients of the higher-order transmission operators at one interface
// end for a time-independent potential (Sec. 2.2).  With x_s = e^{-i calW_s}
// v_s the stored boundary history (calW_s = (s - 1/2) omega, calW_0 = 0;
// omega = W dt for the gauge strategy, 0 for the potential strategy):
//   Sbar v_n = sig v_n + e^{i calW_n} [ cp E_n + cm O_n + a G_n ]
//   E_n / O_n = sum over s < n with n-s even / odd of beta_{n-s} x_s
//   G_n = 2 sum_{s<n} x_s
// where cp = c2 + d, cm = c2 - d, d = -e^{i pi/4} sqrt(dt/2) W/2 (S0^3, S0^4;
// alpha_k = +-beta_k splits the alpha sum by parity), a = -i (dn W/4)(dt/2)
// (S0^4, S1^4), sig = c2 + d + a.  The part that crosses the interface drops
// the a terms: sig_s = c2 + d.
// Pade strategy (c = 2i/dt, W and dn W at the end node):
//   sig_s = -i sum_{s=0}^m a_s + i sum_{s=1}^m a_s d_s / (c + W + d_s),
//   sig = sig_s + (dn W/4) / (c + W) at order 4 (else sig_s),
//   cp = 1/(c + W), omega = W, pad = dn W.
struct EndCoef {
    cd sig, sig_s, cp, cm, a;
    double omega, pad;
};
enum VKind { VK_STATIC = 0, VK_TIME = 1, VK_CUBIC = 2 };

// Task flags: one sweep of one subdomain of one problem.
enum TaskFlags {
    T_DATA_U0   = 1 << 0,   // initial data from u0 (else zero data, zero v_0 history)
    T_FLUX_G    = 1 << 1,   // incoming fluxes l_k, r_k from g_in slots
    T_IMP_L     = 1 << 2,   // l_{k,1} = 1, everything else 0
    T_IMP_R     = 1 << 3,   // r_{k,1} = 1
    T_OUT_G     = 1 << 4,   // outgoing fluxes -> g_out slots
    T_OUT_COLS  = 1 << 5,   // outgoing fluxes -> first-column store
    T_OUT_UT    = 1 << 6,   // u(T) -> uT (interior nodes) + ends
    T_OUT_TRACE = 1 << 7,   // u_n at the two end nodes -> trace store
    T_MAXDIFF   = 1 << 8,   // fold max |g_out - g_in| over written slots
    T_CKPT      = 1 << 9,   // store u at steps nt - 64 j (and u_0) for the adjoint
    T_OUT_SNAP  = 1 << 10,  // u at steps 0, s, 2s, ... -> snapshot store
};

struct Task {
    int k;      // subdomain
    int b;      // problem (batch member)
    int f;      // factor set (potential index)
    int flags;
};

// Layout of the per-lane factor record of one subdomain (see factor kernel).
// For a chunk of up to P nodes per lane: P-1 interior nodes with
// {inv, ainv, cp, alpha, gamma}, then {a_sep, c_sep}, then PCR {k1[6], k2[6]},
// then 1/B of the decoupled reduced equation.
constexpr int kPcrLevels = 6;
__host__ __device__ constexpr int fac_fields(int P) { return 5 * (P - 1) + 2 + 2 * kPcrLevels + 1; }
constexpr int kMaxP = 8;
// subdomains of more than 64 * kMaxP nodes run the long-chunk sweep
// (swr_sweep_long.hip) with up to this many nodes per lane
constexpr int kLongMaxQ = 8192;
// default schedule: the S0^2 helper wave up to this many tasks per launch (every
// wave then has a SIMD of its own); the static causal solve pipelined in
// chunks of this many steps (measured on batched-uneven, whose sweeps fill the
// GPU: 172 ms per solve pipelined, 175.5 ms staged, 202 ms with 128-step and
// 176 ms with 512-step chunks)
constexpr int kHelpMaxTasks = 512;
constexpr int kPipeChunk = 256;
// chunk width from which filled launches run two tasks per wave (a schedule
// parameter; kMaxP + 1 = never).  Measured on the batched-uneven workload the
// one-task sweep is bound by instruction issue, not by its dependency chain:
// two tasks per wave take twice as long per step (widths 4-7: 14.1-16.2 ms
// per launch of two-task waves against 10.3-12.8 ms of one-task waves for
// the same tasks), so the default is never
constexpr int kPairFrom = kMaxP + 1;
// largest group of tasks (one subdomain, one potential) that run as the
// waves of one workgroup sharing an LDS copy of their factor record, and the
// default group size (a schedule parameter; 1 = one task per workgroup)
constexpr int kGroupMax = 8;
constexpr int kGroupDefault = 4;

// S0^2: the time window is cut into super-chunks of this many steps for the
// far history (the part of a block's far sum older than its super-chunk is
// one batched Toeplitz product on the matrix cores per super-chunk; a
// multiple of 256).  Measured on batched-uneven (32 problems, 2000 steps,
// pipelined solve): 256 steps 146.1 ms, 512 steps 146.6 ms; the shorter one
// keeps each lane's chain of recent terms shorter (at most 193 terms)
constexpr int kFarSuper = 256;

struct SweepArgs {
    int N, nt, B, nx, ns;        // ns = 2N-2 interface slots
    int ntasks;
    int P;                       // nodes-per-lane bound the factors were built for
    double kappa;                // h / (3 dt):  c M = i kappa * tridiag(1,4,1)
    cd sigma;                    // implicit transmission coefficient
    cd c2;                       // S0^2 history prefactor e^{-i pi/4} sqrt(2/dt)
    const int* J;                // [N] cells per subdomain
    const int* off;              // [N] first global node
    const Task* tasks;
    const cd* fac;               // [nf][fac_fields(P)][64]
    const double* beta;          // [nt + 65]
    const cd* u0;                // [B][nx]
    const cd* g_in;              // [B][ns][nt]
    cd* g_out;                   // [B][ns][nt]
    cd* cols;                    // [nf/N ... ] first columns [nv][N][4][nt]
    cd* hist;                    // [ntasks][2][nt+1] boundary v_n history
    cd* uT;                      // [B][nx]
    cd* ends;                    // [B][N][2] u(T) at the two end nodes
    cd* trace;                   // [B][N][2][nt+1] u_n at the two end nodes
    unsigned long long* maxdiff; // max |g_out - g_in| as ordered bits
    double h;                    // mesh size
    const double* Vt;            // [nt+1][nx] time-dependent potential
    int nl_maxit;                // |u|^2 inner fixed point: cap and tolerance
    double nl_tol;
    int* nl_stats;               // [0] largest inner count, [1] nonconvergence flag
    int flags_and, flags_or;     // per-launch override of the task flags
    cd* ckpt;                    // [ntasks][Jc+1][P][64] checkpoints of u
    int Jc;                      // ceil(nt / 64)
    int task0;                   // this launch runs tasks task0 .. task0 + ntasks - 1
    int n_begin, n_end;          // steps n_begin+1 .. n_end of this launch (n_begin % 64 == 0)
    cd* state;                   // [ntasks][2][P][64] u_n and v_n carried between launches
    const EndCoef* endc;         // TR_GEN: [nf][2] end coefficients (left, right)
    int help_max;                // S0^2: launches of at most this many tasks use the helper wave
    const int2* pairs;           // two-task waves: [.] task indices (second -1 for a single)
    const int2* groups;          // shared-factor workgroups: [.] (first task, task count)
    int pstride;                 // chunk-width stride of the per-task state and checkpoint
                                 // records (the context's largest width; a launch's own P may
                                 // be smaller: subdomains are grouped by width)
    size_t fstride;              // complex entries per subdomain factor record
    cd* snaps;                   // [B][nsnap][nx] u at steps 0, snap_stride, ... (interior nodes)
    cd* snap_ends;               // [B][nsnap][N][2] the same at the two end nodes
    int snap_stride, nsnap;
    int tr;                      // swr_transmission code (time-dependent end coefficients)
    // Pade strategy
    double dt;
    const cd* pade;              // [2][m+1]: a_0..a_m, then d_0..d_m (d_0 unused)
    int pade_m, pade_order;      // auxiliary functions per end; 2 or 4
    cd* pstate;                  // [ntasks][6][64] auxiliary functions carried between launches
                                 // (phi of the left end: slots 0, 1; right end: 2, 3; psi: 4, 5)
    // long-chunk sweep (subdomains of more than 64 * kMaxP nodes)
    int lq;                      // nodes per lane of this launch
    cd* lfac;                    // [nf][fac_fields(lq max)][64] factor records (static, |u|^2)
    size_t lfstride;             // complex entries per long factor record
    cd* lwork;                   // [ntasks][3 Q (+ fac_fields(Q) for V(t,x))][64] per-task arrays
    // S0^2 split at super-chunks: [list tasks][2][kFarSuper] the old part of
    // the far sums of the launch's super-chunk (null: the far sums run from
    // q = 0; the launch then need not end at a super-chunk boundary)
    const cd* far_old;
};

// far_old_kernel: for the super-chunk starting at step C (> 0), every task
// t < ntasks of a list, both ends e and outputs j < kFarSuper (step C+1+j <=
// nt): out[t][e][j] = sum_{q <= C-65} beta_{C+1+j-q} x_q, x the task's
// boundary history hist[t][e][.] ([ntasks][2][nt+1]).
struct FarOldArgs {
    const cd* hist;
    const double* beta;          // [nt + 65]
    cd* out;
    int ntasks, nt, C;
};

struct FactorArgs {
    int N, nx, nf, P;
    double h, dt;
    cd sigma;                    // Robin / S0^2: implicit coefficient at both ends
    int tr;                      // swr_transmission code; 2..7 fill endc
    cd c2;                       // e^{-i pi/4} sqrt(2/dt)
    EndCoef* endc;               // [nf][2] output for the higher-order operators
    const int* Pk;               // [N] chunk width of each subdomain (this launch builds width P)
    size_t fstride;              // complex entries per subdomain factor record
    const int* J;
    const int* off;
    const double* V;             // [nv][nx] static potential (nullptr = 0)
    cd* fac;
    const cd* pade;              // Pade strategy: [2][m+1] coefficients a, d
    int pade_m;
};

struct LttArgs {
    int N, nt, ns, B;
    int per_problem;       // cols indexed by problem (1) or shared (0)
    const cd* cols;        // [nv][N][4][nt]
    const cd* x;           // [B][ns][nt]
    cd* y;                 // output, see y_ld / n_lo
    const cd* base;        // y = base + sign * L x  (base may be x itself or null)
    double sign;
    int n_lo, n_hi;        // output time window
    int s_lo, s_hi;        // only inputs s_lo <= s < s_hi contribute (and s <= n)
    int y_ld;              // leading dimension of y / base per (b, slot)
    int s_seg;             // > 0: split the inputs into segments of s_seg steps, segment z
                           // writing its own partial at y + z * y_seg_stride (base ignored)
    size_t y_seg_stride;
};

// In-block forward substitution of the causal interface solve.
struct CausalArgs {
    int N, nt, ns, B, per_problem;
    int n0, nb;
    const cd* cols;
    const cd* Minv;    // [nv][ns][ns]  (I - C_0)^{-1}
    const cd* d;       // [B][ns][nt]
    const cd* far;     // [B][ns][kCausalTb]
    cd* g;             // [B][ns][nt]
};
constexpr int kCausalTb = 64;
constexpr int kRedBlocks = 240;   // partial-sum blocks per problem
constexpr int kRedThreads = 256;

// launchers (swr_sweep.hip)
hipError_t launch_factor(const FactorArgs& a, hipStream_t st);
hipError_t launch_sweep(const SweepArgs& a, int trans, int vk, hipStream_t st, bool plain = false);
hipError_t launch_sweep_static(const SweepArgs& a, int trans, hipStream_t st);
hipError_t launch_sweep_static_s02(const SweepArgs& a, hipStream_t st);
hipError_t launch_sweep_static_pade(const SweepArgs& a, hipStream_t st);
// subdomains of more than 64 * kMaxP nodes (swr_sweep_long.hip): a.lq nodes per lane
hipError_t launch_sweep_long(const SweepArgs& a, int trans, int vk, hipStream_t st);
hipError_t launch_factor_long(const FactorArgs& a, int Q, hipStream_t st);
hipError_t launch_sweep_time(const SweepArgs& a, int trans, hipStream_t st);
hipError_t launch_sweep_cubic(const SweepArgs& a, int trans, hipStream_t st);
// static potential, Robin or S0^2: a.ntasks waves of two tasks each, the
// pairs a.pairs[a.task0 ..] (swr_sweep_pair.hip)
hipError_t launch_sweep_pairs(const SweepArgs& a, int trans, hipStream_t st);
// static potential, Robin or S0^2: a.ntasks workgroups of gsize waves, the
// task groups a.groups[a.task0 ..] (swr_sweep_group.hip)
hipError_t launch_sweep_groups(const SweepArgs& a, int trans, int gsize, hipStream_t st);
// the old part of the S0^2 far sums of one super-chunk (swr_sweep.hip)
hipError_t launch_far_old(const FarOldArgs& a, hipStream_t st);
hipError_t launch_finalize_ut(int N, int nx, int B, const int* off, const cd* ends, cd* uT,
                              hipStream_t st);
// the same for every snapshot: ends [B][S][N][2] -> snaps [B][S][nx]
hipError_t launch_finalize_snaps(int N, int nx, int B, int S, const int* off, const cd* ends,
                                 cd* snaps, hipStream_t st);
hipError_t launch_beta(int n, double* beta, hipStream_t st);
// launchers (swr_iface.hip)
hipError_t launch_ltt(const LttArgs& a, hipStream_t st);
hipError_t launch_lincomb(const cd* x0, const cd* x1, const cd* x2, const cd* coef, cd* z, long M,
                          int B, hipStream_t st);
hipError_t launch_multidot(const cd* basis, int nv, const cd* w, long M, int B, double* partial,
                           cd* out, int out_ld, int accumulate, hipStream_t st);
hipError_t launch_multiaxpy(const cd* basis, int nv, const cd* coef, int coef_ld, double sign,
                            cd* w, long M, int B, hipStream_t st);
hipError_t launch_norm(const cd* w, long M, int B, double* partial, double* nrm, hipStream_t st);
hipError_t launch_scale(const cd* src, const double* den, cd* dst, long M, int B, const int* active,
                        hipStream_t st);
hipError_t launch_givens(int j, int m, int B, const cd* hproj, const double* hnext, cd* H, cd* cs,
                         cd* sn, cd* e, const double* bnorm, double* resid, int* active,
                         hipStream_t st);
hipError_t launch_gmres_solve(int jj, int m, int B, const cd* H, const cd* e, cd* y,
                              const int* active, hipStream_t st);
hipError_t launch_gmres_init(int m, int B, const double* beta, cd* e, int* active,
                             const double* bnorm, double tol, double* resid, hipStream_t st);
hipError_t launch_c0_inverse(int N, int ns, int nt, int nv, const cd* cols, cd* work, cd* Minv,
                             int* piv_ok, hipStream_t st);
hipError_t launch_causal_block(const CausalArgs& a, hipStream_t st);
// launchers (swr_causal.hip): block-PCR causal solve for N - 1 <= 64
// interfaces and ns <= kNearSlots slots
constexpr int kNearTb = 32;
constexpr int kNearSlots = 128;
// PCR record per lane: multipliers of every level, then the inverse of the
// reduced diagonal block after 0 .. kPcrLevels levels
constexpr int kPcrRec = kPcrLevels * 8 + (kPcrLevels + 1) * 4;
// remaining coupling below which further PCR levels cannot change an FP64
// result: ||D_l^{-1}|| (||L_l|| + ||U_l||) <= 2^-60 (unit roundoff is 2^-53)
constexpr double kPcrNegligible = 8.673617379884035e-19;
// eta: [nv][levels + 1] coupling measure of the system before each level
// per-potential record size (complex values) of the one-wave causal form:
// PCR multipliers plus the near kernel's packed lag coefficients
size_t causal_fast_rec();
hipError_t launch_causal_pcr_setup(int N, int nt, int nv, const cd* cols, cd* pcr, double* eta,
                                   hipStream_t st);
hipError_t launch_causal_fast(int N, int nt, int ns, int B, int per_problem, const cd* cols,
                              const cd* pcr, int levels, const cd* d, cd* base, cd* g, int n_lo,
                              int n_hi, const cd* facc, int s_from, hipStream_t st);
// general block-PCR causal solve for up to kGenMaxIf interfaces: one
// thread per interface, 512 threads and near blocks of 8 steps up to 512
// interfaces, 1024 threads and near blocks of 2 steps (so the LDS of the
// near march fits) up to 1024
constexpr int kCausalSuper = 256;    // causal solve super-block (time steps)
constexpr int kGenMaxIf = 1024;
constexpr int kGenLevelsMax = 10;    // pcr_levels_for(kGenMaxIf)
__host__ __device__ constexpr int gen_threads(int N) { return N - 1 <= 512 ? 512 : 1024; }
__host__ __device__ constexpr int gen_tb(int N) { return N - 1 <= 512 ? 8 : 2; }
// dynamic LDS of the general near march: [tb][ns] solutions + two exchange rows
__host__ __device__ constexpr size_t gen_shm(int N) {
    return ((size_t)gen_tb(N) * (2 * N - 2) + 2 * (size_t)(2 * N - 2)) * sizeof(cd);
}
// number of block-PCR levels that decouple ni interfaces completely
__host__ __device__ constexpr int pcr_levels_for(int ni) {
    return ni <= 1 ? 0 : (32 - __builtin_clz((unsigned)(ni - 1)));
}
__host__ __device__ constexpr int pcr_rec_gen(int N) {
    // complex entries per potential: levels * 8 * ni multipliers, then
    // (levels + 1) * 4 * ni inverse diagonal blocks
    return (N - 1) * 8 * pcr_levels_for(N - 1) + (pcr_levels_for(N - 1) + 1) * 4 * (N - 1);
}
hipError_t launch_causal_pcr_setup_gen(int N, int nt, int nv, const cd* cols, cd* pcr, double* eta,
                                       hipStream_t st);
hipError_t launch_causal_gen(int N, int nt, int ns, int B, int per_problem, const cd* cols,
                             const cd* pcr, int levels, const cd* d, cd* base, cd* g, int n_lo,
                             int n_hi, const cd* facc, int s_from, hipStream_t st);
struct AdjArgs {
    int N, nt, B, nx, ns, ntasks, P, Jc;
    int task0, pstride;          // this launch runs tasks task0 ..; record stride as SweepArgs
    size_t fstride;
    double kappa, h;
    cd sigma, c2;
    const int* J;
    const int* off;
    const Task* tasks;
    const cd* fac;
    const double* beta;
    const cd* gbar;          // [B][nx]
    const cd* g_in;          // adjoint fluxes [B][ns][nt] (null: zero)
    cd* g_out;               // outgoing adjoint fluxes (null: not written)
    cd* hist;                // adjoint boundary history [ntasks][2][nt+1]
    int grad;                // replay the forward and accumulate dJ/dV
    const cd* ckpt;          // [ntasks][Jc+1][P][64]
    const cd* g_fwd;         // forward converged fluxes
    const cd* hist_fwd;      // forward boundary history [ntasks][2][nt+1]
    cd* seg;                 // [ntasks][64][P][64] forward v of one block
    double* dV;              // [B][nx] (nodes interior to a subdomain)
    cd* du0;                 // [B][nx] (nodes interior to a subdomain)
    double* gends;           // [B][N][2] dJ/dV partial sums at the end nodes
    cd* wends;               // [B][N][2] w at the end nodes
};
hipError_t launch_adjoint(const AdjArgs& a, int trans, hipStream_t st);
hipError_t launch_finalize_grad(int N, int nx, int B, const int* off, const double* gends,
                                const cd* wends, double* dV, cd* du0, hipStream_t st);
hipError_t launch_maxabs(const cd* x, long M, int B, double* partial, double* out, hipStream_t st);
hipError_t launch_axpby(const cd* x, double a, const cd* y, double b, cd* z, long n, hipStream_t st);

}  // namespace swr
