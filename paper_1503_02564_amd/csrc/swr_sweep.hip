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
// step n0+1+j; at each block start it sums the "far" past s <= n0 from the
// boundary history stored in global memory, and every step adds the newest
// boundary value with one fused multiply-add per lane.  The critical path of
// a step therefore carries no O(n) history work.
#include "swr_common.h"

namespace swr {

// Lane t owns the P consecutive nodes t*P .. t*P+P-1 of its subdomain; nodes
// at or beyond n = J_k + 1 are padding with a decoupled identity row, so every
// lane runs the same straight-line code with compile-time register indices.

// Row i of the subdomain matrix  c M - S + M_W - sigma E  (P1 elements on a
// uniform mesh, eq. AvML; the generalised mass integrates W interpolated in
// P1).  a = coupling to node i-1, b = diagonal, c = coupling to node i+1.
__device__ inline void subdomain_row(int i, int n, bool left_if, bool right_if, double h,
                                     double kap, cd sigma, const double* W, cd& ra, cd& rb,
                                     cd& rc) {
    ra = mk(0, 0);
    rb = mk(0, 0);
    rc = mk(0, 0);
    if (i >= n) { rb = mk(1, 0); return; }   // padding
    const double wi = W ? W[i] : 0.0;
    if (i > 0) {
        const double wm = W ? W[i - 1] : 0.0;
        rb = rb + mk(-1.0 / h + h / 12.0 * (wm + 3.0 * wi), 2.0 * kap);
        ra = mk(1.0 / h + h / 12.0 * (wm + wi), kap);
    }
    if (i < n - 1) {
        const double wp = W ? W[i + 1] : 0.0;
        rb = rb + mk(-1.0 / h + h / 12.0 * (3.0 * wi + wp), 2.0 * kap);
        rc = mk(1.0 / h + h / 12.0 * (wi + wp), kap);
    }
    if (i == 0 && left_if) rb = rb - sigma;
    if (i == n - 1 && right_if) rb = rb - sigma;
}

// Field offsets inside one lane's factor record.
template <int P>
struct FacLayout {
    static constexpr int inv(int q) { return 5 * q + 0; }
    static constexpr int ainv(int q) { return 5 * q + 1; }
    static constexpr int cp(int q) { return 5 * q + 2; }
    static constexpr int al(int q) { return 5 * q + 3; }
    static constexpr int ga(int q) { return 5 * q + 4; }
    static constexpr int ae = 5 * (P - 1);
    static constexpr int ce = ae + 1;
    static constexpr int k1(int l) { return ce + 1 + l; }
    static constexpr int k2(int l) { return ce + 1 + kPcrLevels + l; }
    static constexpr int invB = ce + 1 + 2 * kPcrLevels;
    static constexpr int total = invB + 1;
};
static_assert(FacLayout<5>::total == fac_fields(5), "factor layout");

// ---------------------------------------------------------------------------
// Assembly + factorisation: one wave per (potential, subdomain).
//
// Chunk of lane t: interior nodes q = 0..P-2, separator q = P-1 (X_t).  The
// interior solves  T_t x = rhs - a_0 X_{t-1} e_0 - c_{P-2} X_t e_{P-2},
// giving x_q = y_q + alpha_q X_{t-1} + gamma_q X_t, where y is the Thomas
// solution for the right-hand side and alpha, gamma are the responses to the
// two separators.  Substituting into the separator rows leaves a tridiagonal
// system in X_0..X_63 (A X_{t-1} + B X_t + C X_{t+1} = D), reduced here by
// parallel cyclic reduction; only the multipliers k1, k2 and the final 1/B are
// stored.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(64) void factor_kernel(FactorArgs a) {
    using L = FacLayout<P>;
    const int f = blockIdx.x;
    const int k = f % a.N, v = f / a.N;
    const int t = threadIdx.x;
    const int n = a.J[k] + 1, o = a.off[k];
    const bool lif = k > 0, rif = k < a.N - 1;
    const double kap = a.h / (3.0 * a.dt);
    const double* W = a.V ? a.V + (size_t)v * a.nx + o : nullptr;
    const int s = t * P;
    cd* F = a.fac + (size_t)f * L::total * kWave + t;
    const cd zero = mk(0, 0), one = mk(1, 0);

    constexpr int PI = P > 1 ? P - 1 : 1;
    cd iinv[PI], icp[PI], ial[PI], iga[PI];
    cd cpp = zero, alp = zero, last_c = zero;
#pragma unroll
    for (int q = 0; q < P - 1; ++q) {
        cd ra, rb, rc;
        subdomain_row(s + q, n, lif, rif, a.h, kap, a.sigma, W, ra, rb, rc);
        const cd piv = (q == 0) ? rb : msub(rb, ra, cpp);
        const cd iv = inv(piv);
        const cd ai = ra * iv;
        const cd cp = rc * iv;
        alp = (q == 0) ? -(ra * iv) : -(ai * alp);   // forward sweep of alpha
        cpp = cp;
        last_c = rc;
        F[L::inv(q) * kWave] = iv;
        F[L::ainv(q) * kWave] = ai;
        F[L::cp(q) * kWave] = cp;
        iinv[q] = iv;
        icp[q] = cp;
        ial[q] = alp;
    }
    // back substitution of alpha and gamma (gamma' = -c_{P-2} inv_{P-2} at the
    // last interior node and zero above it)
    if (P > 1) {
        cd an = ial[P - 2], gn = -(last_c * iinv[P - 2]);
        iga[P - 2] = gn;
#pragma unroll
        for (int q = P - 3; q >= 0; --q) {
            gn = -(icp[q] * gn);
            an = msub(ial[q], icp[q], an);
            ial[q] = an;
            iga[q] = gn;
        }
    }
#pragma unroll
    for (int q = 0; q < P - 1; ++q) {
        F[L::al(q) * kWave] = ial[q];
        F[L::ga(q) * kWave] = iga[q];
    }

    // separator row and the reduced system
    cd ae, rbs, ce;
    subdomain_row(s + P - 1, n, lif, rif, a.h, kap, a.sigma, W, ae, rbs, ce);
    const cd aL = (P > 1) ? ial[PI - 1] : one;
    const cd gL = (P > 1) ? iga[PI - 1] : zero;
    // the right neighbour's first node: (alpha_0, gamma_0), or its separator
    const cd aF = (P > 1) ? ial[0] : zero;
    const cd gF = (P > 1) ? iga[0] : one;
    const cd aR = shfl_dn_c(aF, 1, zero);
    const cd gR = shfl_dn_c(gF, 1, zero);
    cd At = ae * aL;
    cd Bt = madd(madd(rbs, ae, gL), ce, aR);
    cd Ct = ce * gR;
    F[L::ae * kWave] = ae;
    F[L::ce * kWave] = ce;

#pragma unroll
    for (int l = 0; l < kPcrLevels; ++l) {
        const int d = 1 << l;
        const cd Am = shfl_up_c(At, d, zero), Bm = shfl_up_c(Bt, d, one), Cm = shfl_up_c(Ct, d, zero);
        const cd Ap = shfl_dn_c(At, d, zero), Bp = shfl_dn_c(Bt, d, one), Cp = shfl_dn_c(Ct, d, zero);
        const cd k1 = (t - d >= 0) ? At * inv(Bm) : zero;
        const cd k2 = (t + d < kWave) ? Ct * inv(Bp) : zero;
        At = -(k1 * Am);
        Ct = -(k2 * Cp);
        Bt = msub(msub(Bt, k1, Cm), k2, Ap);
        F[L::k1(l) * kWave] = k1;
        F[L::k2(l) * kWave] = k2;
    }
    F[L::invB * kWave] = inv(Bt);
}

// ---------------------------------------------------------------------------
// The sweep.
// ---------------------------------------------------------------------------
template <int P, int TR>
__global__ __launch_bounds__(64) void sweep_kernel(SweepArgs a) {
    using L = FacLayout<P>;
    constexpr int PI = P > 1 ? P - 1 : 1;
    __shared__ double sbeta[kWave + 1];
    __shared__ cd sha[kWave], shb[kWave];     // staged chunk of the boundary history
    __shared__ double sb[2 * kWave];          // beta window of that chunk
    const Task task = a.tasks[blockIdx.x];
    const int k = task.k, b = task.b, f = task.f, fl = task.flags;
    const int t = threadIdx.x;
    const int n = a.J[k] + 1, o = a.off[k];
    const int nt = a.nt;
    const bool lif = k > 0, rif = k < a.N - 1;
    const int s = t * P;
    const int lastl = (n - 1) / P;          // lane holding node n-1
    const cd zero = mk(0, 0);

    if (TR == TR_S02) {
        sbeta[t] = a.beta[t];
        if (t == 0) sbeta[kWave] = a.beta[kWave];
        __syncthreads();
    }

    // factors -> registers
    const cd* F = a.fac + (size_t)f * L::total * kWave + t;
    cd f_inv[PI], f_ainv[PI], f_cp[PI], f_al[PI], f_ga[PI];
#pragma unroll
    for (int q = 0; q < P - 1; ++q) {
        f_inv[q] = F[L::inv(q) * kWave];
        f_ainv[q] = F[L::ainv(q) * kWave];
        f_cp[q] = F[L::cp(q) * kWave];
        f_al[q] = F[L::al(q) * kWave];
        f_ga[q] = F[L::ga(q) * kWave];
    }
    const cd f_ae = F[L::ae * kWave], f_ce = F[L::ce * kWave], f_invB = F[L::invB * kWave];
    cd f_k1[kPcrLevels], f_k2[kPcrLevels];
#pragma unroll
    for (int l = 0; l < kPcrLevels; ++l) {
        f_k1[l] = F[L::k1(l) * kWave];
        f_k2[l] = F[L::k2(l) * kWave];
    }

    // per-node constants: mass stencil weights (P1 mass: 1,4,1 inside,
    // 2,1 / 1,2 at the ends, zero on padding) and the mask of node n-1
    double wl[P], wr[P], wlast[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int i = s + q;
        wl[q] = (i >= 1 && i <= n - 1) ? 1.0 : 0.0;
        wr[q] = (i <= n - 2) ? 1.0 : 0.0;
        wlast[q] = (i == n - 1) ? 1.0 : 0.0;
    }

    // state u_0
    cd u[P];
    const bool data = (fl & T_DATA_U0) != 0;
    const cd* u0 = a.u0 + (size_t)b * a.nx + o;
#pragma unroll
    for (int q = 0; q < P; ++q) u[q] = (data && s + q < n) ? u0[s + q] : zero;
    auto at_last = [&](const cd (&arr)[P]) {
        cd r = zero;
#pragma unroll
        for (int q = 0; q < P; ++q) r = mk(r.x + wlast[q] * arr[q].x, r.y + wlast[q] * arr[q].y);
        return rdlane(r, lastl);
    };

    const double kap = a.kappa;
    cd* Ha = a.hist ? a.hist + (size_t)blockIdx.x * 2 * (nt + 1) : nullptr;
    cd* Hb = Ha ? Ha + (nt + 1) : nullptr;
    const cd va0 = rdlane(u[0], 0);
    const cd vb0 = at_last(u);
    if (TR == TR_S02 && t == 0) {
        Ha[0] = va0;
        Hb[0] = vb0;
    }
    cd* trace_a = (fl & T_OUT_TRACE) ? a.trace + ((size_t)(b * a.N + k) * 2) * (nt + 1) : nullptr;
    cd* trace_b = trace_a ? trace_a + (nt + 1) : nullptr;
    if (trace_a && t == 0) {
        trace_a[0] = va0;
        trace_b[0] = vb0;
    }

    const int ns = a.ns;
    const cd* gin_l = (lif && (fl & T_FLUX_G)) ? a.g_in + ((size_t)b * ns + 2 * k - 1) * nt : nullptr;
    const cd* gin_r = (rif && (fl & T_FLUX_G)) ? a.g_in + ((size_t)b * ns + 2 * k) * nt : nullptr;
    cd* out_l = nullptr;
    cd* out_r = nullptr;
    const cd* old_l = nullptr;
    const cd* old_r = nullptr;
    if (fl & T_OUT_G) {
        if (lif) out_l = a.g_out + ((size_t)b * ns + 2 * k - 2) * nt;
        if (rif) out_r = a.g_out + ((size_t)b * ns + 2 * k + 1) * nt;
        if (fl & T_MAXDIFF) {
            if (lif) old_l = a.g_in + ((size_t)b * ns + 2 * k - 2) * nt;
            if (rif) old_r = a.g_in + ((size_t)b * ns + 2 * k + 1) * nt;
        }
    } else if (fl & T_OUT_COLS) {
        const int pl = (fl & T_IMP_L) ? 0 : 1;
        if (lif) out_l = a.cols + ((size_t)f * 4 + pl) * nt;
        if (rif) out_r = a.cols + ((size_t)f * 4 + pl + 2) * nt;
    }
    double maxd = 0.0;

    for (int n0 = 0; n0 < nt; n0 += kWave) {
        const int nb = min(kWave, nt - n0);
        const bool act = t < nb;
        // incoming fluxes of this block: lane j <-> step n0+1+j
        cd lb = zero, rb = zero;
        if (act) {
            if (gin_l) lb = gin_l[n0 + t];
            if (gin_r) rb = gin_r[n0 + t];
            if ((fl & T_IMP_L) && n0 + t == 0) lb = mk(1, 0);
            if ((fl & T_IMP_R) && n0 + t == 0) rb = mk(1, 0);
        }
        // far part of the S0^2 history for the outputs of this block:
        // acc_j = sum_{q <= n0} beta_{n0+1+j-q} v_q, over chunks of 64 past
        // values staged in LDS with one coalesced load each, together with
        // the 127-entry window of beta the chunk needs
        cd acc_a = zero, acc_b = zero;
        if (TR == TR_S02) {
            __threadfence_block();
            const int nj = n0 + 1 + t;
            for (int q0 = 0; q0 <= n0; q0 += kWave) {
                const int qn = min(kWave, n0 + 1 - q0);
                const int bbase = n0 - q0 - (kWave - 2);   // beta index of sb[0]
                sha[t] = (t < qn) ? Ha[q0 + t] : zero;
                shb[t] = (t < qn) ? Hb[q0 + t] : zero;
                const int i0 = bbase + t, i1 = bbase + kWave + t;
                sb[t] = (i0 >= 0) ? a.beta[i0] : 0.0;
                sb[kWave + t] = (i1 >= 0) ? a.beta[i1] : 0.0;
                __syncthreads();
                const double* bw = sb + (nj - q0 - bbase);  // beta_{nj - q0 - i} = bw[-i]
                for (int i = 0; i < qn; ++i) {
                    const double bt = bw[-i];
                    const cd ha = sha[i], hb = shb[i];
                    acc_a = mk(acc_a.x + bt * ha.x, acc_a.y + bt * ha.y);
                    acc_b = mk(acc_b.x + bt * hb.x, acc_b.y + bt * hb.y);
                }
                __syncthreads();
            }
        }
        cd rl_b = zero, rr_b = zero, va_b = zero, vb_b = zero, ua_b = zero, ub_b = zero;

        for (int i = 0; i < nb; ++i) {
            const cd ln = rdlane(lb, i), rn = rdlane(rb, i);
            cd hA = zero, hB = zero;
            if (TR == TR_S02) {
                hA = a.c2 * rdlane(acc_a, i);
                hB = a.c2 * rdlane(acc_b, i);
            }
            // right-hand side c M u_{n-1} + boundary terms
            const cd uL = shfl_up_c(u[P - 1], 1, zero);
            const cd uR = shfl_dn_c(u[0], 1, zero);
            const cd tb = rif ? (hB - rn) : zero;
            cd d[P];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const cd up = (q == 0) ? uL : u[q - 1];
                const cd un = (q + 1 < P) ? u[q + 1] : uR;
                const double wc = 2.0 * (wl[q] + wr[q]);
                const cd sum = mk(wl[q] * up.x + wc * u[q].x + wr[q] * un.x,
                                  wl[q] * up.y + wc * u[q].y + wr[q] * un.y);
                d[q] = kap * mul_i(sum);
                d[q] = mk(d[q].x + wlast[q] * tb.x, d[q].y + wlast[q] * tb.y);
            }
            if (lif && t == 0) d[0] = d[0] + (hA - ln);
            // interior forward / backward elimination
            cd y[PI];
            cd yp = zero;
#pragma unroll
            for (int q = 0; q < P - 1; ++q) {
                yp = msub(d[q] * f_inv[q], f_ainv[q], yp);
                y[q] = yp;
            }
#pragma unroll
            for (int q = P - 3; q >= 0; --q) y[q] = msub(y[q], f_cp[q], y[q + 1]);
            // reduced right-hand side at my separator, then PCR
            const cd yL = (P > 1) ? y[PI - 1] : zero;
            const cd yR = (P > 1) ? shfl_dn_c(y[0], 1, zero) : zero;
            cd D = msub(msub(d[P - 1], f_ae, yL), f_ce, yR);
#pragma unroll
            for (int l = 0; l < kPcrLevels; ++l) {
                const int dd = 1 << l;
                const cd Dm = shfl_up_c(D, dd, zero), Dp = shfl_dn_c(D, dd, zero);
                D = msub(msub(D, f_k1[l], Dm), f_k2[l], Dp);
            }
            const cd X = D * f_invB;
            const cd Xm = shfl_up_c(X, 1, zero);
            // recover the chunk and advance u_n = 2 v_n - u_{n-1}
            cd x[P];
#pragma unroll
            for (int q = 0; q < P - 1; ++q) x[q] = madd(madd(y[q], f_al[q], Xm), f_ga[q], X);
            x[P - 1] = X;
#pragma unroll
            for (int q = 0; q < P; ++q) u[q] = mk(2.0 * x[q].x - u[q].x, 2.0 * x[q].y - u[q].y);
            const cd va = rdlane(x[0], 0);
            const cd vb = at_last(x);
            const cd rhoL = (2.0 * madd(hA, a.sigma, va)) - ln;
            const cd rhoR = (2.0 * madd(hB, a.sigma, vb)) - rn;
            if (t == i) {
                rl_b = rhoL;
                rr_b = rhoR;
                va_b = va;
                vb_b = vb;
            }
            if (trace_a) {
                const cd ua = rdlane(u[0], 0), ub = at_last(u);
                if (t == i) { ua_b = ua; ub_b = ub; }
            }
            if (TR == TR_S02 && t > i) {
                const double bt = sbeta[t - i];
                acc_a = acc_a + bt * va;
                acc_b = acc_b + bt * vb;
            }
        }
        // block epilogue: coalesced stores
        if (act) {
            if (out_l) out_l[n0 + t] = rl_b;
            if (out_r) out_r[n0 + t] = rr_b;
            if (old_l) maxd = fmax(maxd, sqrt(abs2(rl_b - old_l[n0 + t])));
            if (old_r) maxd = fmax(maxd, sqrt(abs2(rr_b - old_r[n0 + t])));
            if (TR == TR_S02) {
                Ha[n0 + 1 + t] = va_b;
                Hb[n0 + 1 + t] = vb_b;
            }
            if (trace_a) {
                trace_a[n0 + 1 + t] = ua_b;
                trace_b[n0 + 1 + t] = ub_b;
            }
        }
    }

    if (fl & T_OUT_UT) {
        cd* uT = a.uT + (size_t)b * a.nx + o;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int gi = s + q;
            if (gi > 0 && gi < n - 1) uT[gi] = u[q];
        }
        const cd ua = rdlane(u[0], 0), ub = at_last(u);
        if (t == 0) {
            a.ends[((size_t)b * a.N + k) * 2 + 0] = ua;
            a.ends[((size_t)b * a.N + k) * 2 + 1] = ub;
        }
    }
    if (fl & T_MAXDIFF) {
        maxd = wave_max(maxd);
        if (t == 0 && maxd > 0.0)
            atomicMax(a.maxdiff, (unsigned long long)__double_as_longlong(maxd));
    }
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

hipError_t launch_sweep(const SweepArgs& a, int trans, hipStream_t st) {
    if (a.ntasks == 0) return hipSuccess;
#define CASE(PP)                                                                    \
    case PP:                                                                        \
        if (trans == TR_S02) sweep_kernel<PP, TR_S02><<<a.ntasks, 64, 0, st>>>(a);  \
        else sweep_kernel<PP, TR_ROBIN><<<a.ntasks, 64, 0, st>>>(a);                \
        break;
    switch (a.P) {
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef CASE
    return hipGetLastError();
}

hipError_t launch_finalize_ut(int N, int nx, int B, const int* off, const cd* ends, cd* uT,
                              hipStream_t st) {
    const int tot = B * (N + 1);
    finalize_ut_kernel<<<(tot + 255) / 256, 256, 0, st>>>(N, nx, B, off, ends, uT);
    return hipGetLastError();
}

hipError_t launch_beta(int n, double* beta, hipStream_t st) {
    beta_table_kernel<<<1, 1, 0, st>>>(n, beta);
    return hipGetLastError();
}

}  // namespace swr
