// swr_sweep.hip -- subdomain Crank-Nicolson sweeps of Schwarz waveform
// relaxation (Besse & Xing, arXiv 1503.02564), hand-written for gfx950.
//
// One wavefront owns one sweep task (subdomain k of problem b over the whole
// time window).  Its J_k + 1 nodes are split into 64 contiguous chunks, one per
// lane; the tridiagonal system of eq. AvML is solved every step by the
// partition method:
//   * each lane eliminates its chunk interior against the two neighbouring
//     separators (last node of each chunk),
//   * the 64 separators form a tridiagonal reduced system solved by parallel
//     cyclic reduction across lanes (6 levels),
//   * each lane recovers its interior nodes.
// For a time-independent potential the matrix is constant, so every
// coefficient (pivots, spikes, PCR multipliers) is computed once by
// `factor_kernel` and kept in VGPRs for all steps; a step touches only
// right-hand sides.  State u_{n-1} also lives in VGPRs.
//
// Transmission (eq. TransmissionCondlocal, eq. TransmissionCond_disc):
//   (A - sigma E) v_n = c M u_{n-1} + E (h_n - flux_n),   u_n = 2 v_n - u_{n-1}
//   rho_n = -flux_n + 2 (sigma v_n + h_n)  at each interface end
// with h_n = c2 sum_{s<n} beta_{n-s} v_s for S0^2 (Sec. 2.2) and h = 0 for
// Robin.  The S0^2 history is blocked by 64 steps: lane j carries the output
// step n0+1+j.  Its "far" part, s <= n0 - 64, is summed from the boundary
// history stored in global memory -- by a second wave of the workgroup while
// the sweep runs the block before (launches of up to 512 tasks, where every
// wave gets a SIMD of its own), or at the block start by the sweeping wave
// itself (larger launches), with the same arithmetic; the 64 terms of the
// block before, and every step's newest value for the current block, are
// added by the sweeping wave with one fused multiply-add per lane each.
//
// The kernel template itself is in swr_sweep_kernel.h; swr_sweep_static.hip,
// swr_sweep_static_s02.hip, swr_sweep_time.hip and swr_sweep_cubic.hip
// instantiate it.
#include "swr_lane.h"

namespace swr {

// ---------------------------------------------------------------------------
// Assembly + factorisation for a static potential: one wave per
// (potential, subdomain).
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(64) void factor_kernel(FactorArgs a) {
    const int f = blockIdx.x;
    const int k = f % a.N, v = f / a.N;
    if (a.Pk && a.Pk[k] != P) return;    // another width's launch builds this record
    const int t = threadIdx.x;
    const int n = a.J[k] + 1, o = a.off[k];
    const bool lif = k > 0, rif = k < a.N - 1;
    const double kap = a.h / (3.0 * a.dt);
    const double* W = a.V ? a.V + (size_t)v * a.nx + o : nullptr;
    const int s = t * P;
    double w[P];
#pragma unroll
    for (int q = 0; q < P; ++q) w[q] = (W && s + q < n) ? W[s + q] : 0.0;
    double wL, wR;
    neighbour_w(w, wL, wR);
    cd sigL = a.sigma, sigR = a.sigma;
    if (a.tr >= 2) {
        // higher-order and Pade operators (Sec. 2.2) at the two interface ends: W and
        // its outward normal derivative (centred difference on the global
        // mesh) at the end node
        const double* Vg = a.V ? a.V + (size_t)v * a.nx : nullptr;
        const cd eP = mk(M_SQRT1_2, M_SQRT1_2);                 // e^{i pi/4}
        EndCoef e[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int g = o + (side ? n - 1 : 0);
            const bool iface = side ? rif : lif;
            double We = 0.0, dWe = 0.0;
            if (Vg && iface) {
                We = Vg[g];
                dWe = (side ? 1.0 : -1.0) * (Vg[g + 1] - Vg[g - 1]) / (2.0 * a.h);
            }
            if (a.tr >= 6) {
                // Pade strategy: the implicit part of Sbar v_n (see EndCoef)
                const cd cc = mk(0.0, 2.0 / a.dt);
                const cd* pa = a.pade;
                const cd* pd = a.pade + a.pade_m + 1;
                cd asum = mk(0, 0);
                for (int q = 0; q <= a.pade_m; ++q) asum = asum + pa[q];
                cd s2 = -mul_i(asum);
                for (int q = 1; q <= a.pade_m; ++q) {
                    const cd den = mk(cc.x + We + pd[q].x, cc.y + pd[q].y);
                    s2 = s2 + mul_i(pa[q] * pd[q]) * inv(den);
                }
                const cd rho = inv(mk(cc.x + We, cc.y));
                e[side].cp = rho;
                e[side].cm = mk(0, 0);
                e[side].a = mk(0, 0);
                e[side].sig_s = s2;
                e[side].sig = (a.tr == 7) ? s2 + (dWe / 4.0) * rho : s2;
                e[side].omega = We;
                e[side].pad = dWe;
                continue;
            }
            const bool pot = a.tr == 2 || a.tr == 3, ord4 = a.tr == 3 || a.tr == 5;
            const cd d = pot ? (-(sqrt(0.5 * a.dt) * 0.5 * We)) * eP : mk(0, 0);
            const cd aa = ord4 ? mk(0.0, -(dWe / 4.0) * (0.5 * a.dt)) : mk(0, 0);
            e[side].cp = a.c2 + d;
            e[side].cm = a.c2 - d;
            e[side].a = aa;
            e[side].sig_s = a.c2 + d;
            e[side].sig = (a.c2 + d) + aa;
            e[side].omega = (a.tr >= 4) ? We * a.dt : 0.0;
            e[side].pad = 0.0;
        }
        sigL = e[0].sig;
        sigR = e[1].sig;
        if (t == 0) {
            a.endc[(size_t)f * 2 + 0] = e[0];
            a.endc[(size_t)f * 2 + 1] = e[1];
        }
    }
    cd ra[P], rb[P], rc[P];
    chunk_rows<P>(s, n, lif, rif, a.h, kap, sigL, sigR, w, wL, wR, ra, rb, rc);
    LaneFac<P> F;
    lane_factor<P>(ra, rb, rc, F);
    store_fac<P>(a.fac + (size_t)f * a.fstride + t, F);
}


// u(T) at the nodes shared by two subdomains: average of the two sides;
// walls take their subdomain's value.
__global__ void finalize_ut_kernel(int N, int nx, int B, const int* off, const cd* ends, cd* uT) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * (N + 1)) return;
    const int b = idx / (N + 1), j = idx % (N + 1);
    const cd* e = ends + (size_t)b * N * 2;
    cd* u = uT + (size_t)b * nx;
    if (j == 0) u[0] = e[0];
    else if (j == N) u[nx - 1] = e[(N - 1) * 2 + 1];
    else u[off[j]] = 0.5 * (e[(j - 1) * 2 + 1] + e[j * 2 + 0]);
}

// the same per snapshot: one thread per (problem, snapshot, end node)
__global__ void finalize_snaps_kernel(int N, int nx, int B, int S, const int* off, const cd* ends,
                                      cd* snaps) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)B * S * (N + 1)) return;
    const long bs = idx / (N + 1);
    const int j = (int)(idx % (N + 1));
    const cd* e = ends + (size_t)bs * N * 2;
    cd* u = snaps + (size_t)bs * nx;
    if (j == 0) u[0] = e[0];
    else if (j == N) u[nx - 1] = e[(N - 1) * 2 + 1];
    else u[off[j]] = 0.5 * (e[(j - 1) * 2 + 1] + e[j * 2 + 0]);
}

// beta_s = (-1)^s alpha_s, alpha_{2m} = alpha_{2m+1} = (2m-1)!!/(2m)!!
// (Sec. 2.2), tabulated for s = 0..n-1 by one thread.
__global__ void beta_table_kernel(int n, double* beta) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double a = 1.0;
    for (int s = 0; s < n; ++s) {
        if (s >= 2 && (s % 2) == 0) a *= (double)(s - 1) / (double)s;
        beta[s] = (s % 2) ? -a : a;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from swr_host.hip).
// ---------------------------------------------------------------------------
hipError_t launch_factor(const FactorArgs& a, hipStream_t st) {
    switch (a.P) {
#define CASE(PP) case PP: factor_kernel<PP><<<a.nf, 64, 0, st>>>(a); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t launch_sweep_once(const SweepArgs& a, int trans, int vk, hipStream_t st) {
    if (vk == VK_TIME) return launch_sweep_time(a, trans, st);
    if (vk == VK_CUBIC) return launch_sweep_cubic(a, trans, st);
    return launch_sweep_static(a, trans, st);
}

// All tasks in one launch, or (plain) one launch per task on the stream:
// the unbatched form, kept as the reference the batched one is compared to.
hipError_t launch_sweep(const SweepArgs& a, int trans, int vk, hipStream_t st, bool plain) {
    if (a.ntasks == 0) return hipSuccess;
    if (a.P < 1 || a.P > kMaxP) return hipErrorInvalidValue;
    if (!plain) return launch_sweep_once(a, trans, vk, st);
    SweepArgs one = a;
    one.ntasks = 1;
    for (int i = 0; i < a.ntasks; ++i) {
        one.task0 = a.task0 + i;
        const hipError_t e = launch_sweep_once(one, trans, vk, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// The old part of the S0^2 far sums of one super-chunk (see far_sum_s02): for
// every task of a list, a lower-triangular Toeplitz product of the beta
// sequence with the task's two boundary histories, on the matrix cores
// (v_mfma_f64_16x16x4_f64; lane l supplies A[l%16][l/16] and B[l/16][l%16],
// accumulator register k of lane l is D[l/16 + 4k][l%16]).  A workgroup
// takes four tasks, whose 16 (task, end, part) columns fill the instruction's
// N dimension, and 64 RT output rows (blockIdx.y of the super-chunk's
// kFarSuper / (64 RT)); its wave w takes RT row tiles of 16 rows (one
// accumulator each, one B operand for all of them).  RT = 4 for long task
// lists, RT = 1 for short ones, so that few tasks still spread over many
// waves; each output adds the same terms in the same order either way.  Sources come in groups of four, q = 4g ..
// 4g+3, and every output adds its groups in ascending g, one instruction per
// group: A[r][k] = beta_{C+1+j-4g-k} (j = 16 RT + r), B[k][.] = x_{4g+k};
// sources past C - 65, absent tasks and outputs past nt give zero operands.
// Algorithmic work: 4 (C - 64) flops per output per end per task.
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int RT>
__global__ __launch_bounds__(256) void far_old_kernel(FarOldArgs a) {
    const int t = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int r = t & 15, kq = t >> 4;
    const int p = r >> 2, e = (r >> 1) & 1, part = r & 1;
    const int task = blockIdx.x * 4 + p;
    const int row0 = (blockIdx.y * 4 + w) * 16 * RT;   // first output row of this wave
    const bool has = task < a.ntasks;
    const int C = a.C, nt = a.nt;
    const int qmax = C - kWave - 1;                 // old part: q <= C - 65
    const int ng = (qmax + 4) / 4;                  // source groups 0 .. ng-1
    const int amax = nt + kWave;                    // last beta index held
    const double* hs = has ? reinterpret_cast<const double*>(a.hist + ((size_t)task * 2 + e) * (nt + 1)) + part
                           : nullptr;
    f64x4 acc[RT];
#pragma unroll
    for (int rr = 0; rr < RT; ++rr) acc[rr] = f64x4{0.0, 0.0, 0.0, 0.0};
    constexpr int U = RT == 1 ? 8 : 4;
    double an[U][RT], bn[U];
    auto fetch = [&](int gs) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int g = gs + u;
            const int q = 4 * g + kq;
            bn[u] = (hs && q <= qmax) ? hs[2 * q] : 0.0;
#pragma unroll
            for (int rr = 0; rr < RT; ++rr) {
                const int ia = C + 1 + row0 + 16 * rr + r - 4 * g - kq;
                an[u][rr] = (ia >= 0 && ia <= amax) ? a.beta[ia] : 0.0;
            }
        }
    };
    if (ng > 0) fetch(0);
    for (int g = 0; g < ng; g += U) {
        double ac[U][RT], bc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            bc[u] = bn[u];
#pragma unroll
            for (int rr = 0; rr < RT; ++rr) ac[u][rr] = an[u][rr];
        }
        if (g + U < ng) fetch(g + U);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int rr = 0; rr < RT; ++rr)
                acc[rr] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[u][rr], bc[u], acc[rr], 0, 0, 0);
    }
    if (!has) return;
    double* o = reinterpret_cast<double*>(a.out + ((size_t)task * 2 + e) * kFarSuper) + part;
#pragma unroll
    for (int rr = 0; rr < RT; ++rr)
#pragma unroll
        for (int k = 0; k < 4; ++k) o[2 * (row0 + 16 * rr + kq + 4 * k)] = acc[rr][k];
}

// Long task lists: the same product with the operands staged in LDS.  The
// workgroup loads each chunk of 64 sources of its four tasks' histories (16
// columns) and the 319-entry beta window the chunk meets for its 256 rows with
// coalesced loads, the next chunk's loads in flight while the current one is
// multiplied (double buffer, two barriers per chunk).  Each output adds the
// same groups in the same ascending order as far_old_kernel (the chunks'
// padding groups past C - 65 add exact zeros).
__global__ __launch_bounds__(256) void far_old_staged_kernel(FarOldArgs a) {
    __shared__ double sB[2][kWave][16];           // [buffer][source in chunk][column]
    __shared__ double sA[2][kWave + 256];         // [buffer][beta window]
    const int tid = threadIdx.x, t = tid & (kWave - 1), w = tid / kWave;
    const int r = t & 15, kq = t >> 4;
    const int p = r >> 2, e = (r >> 1) & 1, part = r & 1;
    const int task0 = blockIdx.x * 4;
    const int row_base = blockIdx.y * 256;
    const int rw = 64 * w;                          // first row of this wave within the workgroup's
    const int C = a.C, nt = a.nt;
    const int qmax = C - kWave - 1;
    const int amax = nt + kWave;
    const int nch = (qmax + kWave) / kWave;         // chunks of 64 sources covering 0 .. qmax
    // staging: thread tid loads sources i2 and i2 + 32 of history (task, end)
    // pe = tid / 32, and two beta entries
    const int pe = tid >> 5, i2 = tid & 31;
    const int stask = task0 + (pe >> 1);
    const cd* sx = stask < a.ntasks ? a.hist + ((size_t)stask * 2 + (pe & 1)) * (nt + 1) : nullptr;
    cd xv0, xv1;
    double bv0, bv1;
    auto fetch = [&](int c) {
        const int q0 = c * kWave;
        xv0 = (sx && q0 + i2 <= qmax) ? sx[q0 + i2] : mk(0, 0);
        xv1 = (sx && q0 + 32 + i2 <= qmax) ? sx[q0 + 32 + i2] : mk(0, 0);
        const int base = C + 1 + row_base - q0 - (kWave - 1);   // beta index of sA[0]
        const int i0 = base + tid, i1 = base + 256 + tid;
        bv0 = (i0 >= 0 && i0 <= amax) ? a.beta[i0] : 0.0;
        bv1 = (tid < kWave - 1 && i1 >= 0 && i1 <= amax) ? a.beta[i1] : 0.0;
    };
    auto stage = [&](int buf) {
        sB[buf][i2][2 * pe] = xv0.x;
        sB[buf][i2][2 * pe + 1] = xv0.y;
        sB[buf][32 + i2][2 * pe] = xv1.x;
        sB[buf][32 + i2][2 * pe + 1] = xv1.y;
        sA[buf][tid] = bv0;
        if (tid < kWave - 1) sA[buf][256 + tid] = bv1;
    };
    f64x4 acc[4];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[rr] = f64x4{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    stage(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) fetch(c + 1);
#pragma unroll 4
        for (int gl = 0; gl < 16; ++gl) {
            const double bvv = sB[buf][4 * gl + kq][r];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const double avv = sA[buf][rw + 16 * rr + r - 4 * gl - kq + (kWave - 1)];
                acc[rr] = __builtin_amdgcn_mfma_f64_16x16x4f64(avv, bvv, acc[rr], 0, 0, 0);
            }
        }
        if (c + 1 < nch) stage(buf ^ 1);
        __syncthreads();
    }
    const int task = task0 + p;
    if (task >= a.ntasks) return;
    double* o = reinterpret_cast<double*>(a.out + ((size_t)task * 2 + e) * kFarSuper) + part;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
        for (int k = 0; k < 4; ++k) o[2 * (row_base + rw + 16 * rr + kq + 4 * k)] = acc[rr][k];
}

hipError_t launch_far_old(const FarOldArgs& a, hipStream_t st) {
    if (a.ntasks == 0) return hipSuccess;
    if (a.C <= 0 || a.C % kFarSuper != 0 || !a.hist || !a.beta || !a.out) return hipErrorInvalidValue;
    static_assert(kFarSuper % 256 == 0, "far_old_kernel covers the super-chunk in 256-row blocks");
    const unsigned gx = (unsigned)(a.ntasks + 3) / 4;
    if (a.ntasks >= 4096)
        far_old_staged_kernel<<<dim3(gx, kFarSuper / 256), 256, 0, st>>>(a);
    else
        far_old_kernel<1><<<dim3(gx, kFarSuper / 64), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_finalize_ut(int N, int nx, int B, const int* off, const cd* ends, cd* uT,
                              hipStream_t st) {
    const int tot = B * (N + 1);
    finalize_ut_kernel<<<(tot + 255) / 256, 256, 0, st>>>(N, nx, B, off, ends, uT);
    return hipGetLastError();
}

hipError_t launch_finalize_snaps(int N, int nx, int B, int S, const int* off, const cd* ends,
                                 cd* snaps, hipStream_t st) {
    const long tot = (long)B * S * (N + 1);
    finalize_snaps_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(N, nx, B, S, off, ends, snaps);
    return hipGetLastError();
}

hipError_t launch_beta(int n, double* beta, hipStream_t st) {
    beta_table_kernel<<<1, 1, 0, st>>>(n, beta);
    return hipGetLastError();
}

}  // namespace swr
