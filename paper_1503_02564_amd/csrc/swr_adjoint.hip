// swr_adjoint.hip -- discrete adjoint of the subdomain Crank-Nicolson scheme,
// solved through the same Schwarz decomposition (static real potential).
//
// Forward (eq. CNS_L with P1): A v_n = c M u_{n-1}, u_n = 2 v_n - u_{n-1},
// A = c M - S + M_V complex symmetric.  For a real objective J(u_nt) with
// upstream gradient gbar = dJ/dRe + i dJ/dIm, write P_n for the conjugate of
// the gradient with respect to u_n.  The chain rule gives
//   P_nt = conj(gbar);  A Q_n = P_n;  P_{n-1} = 2 c M Q_n - P_n;
//   dJ/dV_i = -2 Re sum_n Q_n^T (dM_V/dV_i) v_n,   dJ/du0 = conj(P_0).
// With w = P this is the forward recursion written on dual vectors
// (A x = w_prev, w_new = 2 c M x - w_prev): the same subdomain matrices, the
// same transmission and so the same interface operator L; only the data
// differ.  Subdomain k carries the local part w_k of the assembled dual vector
// (a node shared by two subdomains is split half/half; the split only changes
// the iterates, not the converged result); the S0^2 history starts from
// v_0 = 0 on both sides of every interface.
//
// adjoint_kernel runs one wave per (problem, subdomain) task.  Without
// gradient it is the dual sweep (d of the adjoint interface problem, or one
// adjoint SWR iteration).  With gradient it walks the 64-step blocks of the
// adjoint time m = nt - n + 1 in order; for each block it first replays the
// forward steps of that block from a checkpoint of u (stored by the forward
// final sweep every 64 steps counted back from nt), with the forward fluxes
// and the forward S0^2 history, keeping the forward v_n of the block in a
// per-task buffer; then it advances the adjoint over the block, consuming v_n
// in reverse and accumulating dJ/dV per node.
#include "swr_lane.h"

namespace swr {


// far part of the S0^2 history for outputs n0+1+lane:
// sum_{q <= n0} beta_{n0+1+lane-q} H[q] (both ends), staged through LDS in
// chunks of 64; the loads of the next chunk are issued before the current
// one is summed
__device__ inline void far_history(const cd* Ha, const cd* Hb, const double* beta, int n0,
                                   cd* sha, cd* shb, double* sb, cd& acc_a, cd& acc_b) {
    const int t = lane_id();
    const cd zero = mk(0, 0);
    acc_a = zero;
    acc_b = zero;
    __threadfence_block();
    const int nj = n0 + 1 + t;
    cd pa = zero, pb = zero;
    double p0 = 0.0, p1 = 0.0;
    auto fetch = [&](int q0) {
        const int qn = min(kWave, n0 + 1 - q0);
        const int bbase = n0 - q0 - (kWave - 2);
        // (assignments, not a conditional of two lvalues: that would put
        // the zero constant in scratch memory)
        pa = zero;
        pb = zero;
        if (t < qn) { pa = Ha[q0 + t]; pb = Hb[q0 + t]; }
        const int i0 = bbase + t, i1 = bbase + kWave + t;
        p0 = 0.0;
        p1 = 0.0;
        if (i0 >= 0) p0 = beta[i0];
        if (i1 >= 0) p1 = beta[i1];
    };
    if (n0 >= 0) fetch(0);
    for (int q0 = 0; q0 <= n0; q0 += kWave) {
        const int bbase = n0 - q0 - (kWave - 2);
        sha[t] = pa;
        shb[t] = pb;
        sb[t] = p0;
        sb[kWave + t] = p1;
        if (q0 + kWave <= n0) fetch(q0 + kWave);
        __syncthreads();
        const double* bw = sb + (nj - q0 - bbase);
        // all 64 entries: the staged chunk is zero past qn and the beta
        // window bw[-i], i < 64, stays inside sb, so the loop unrolls and
        // its LDS reads overlap
        #pragma unroll 16
        for (int i = 0; i < kWave; ++i) {
            const double bt = bw[-i];
            const cd ha = sha[i], hb = shb[i];
            acc_a = mk(acc_a.x + bt * ha.x, acc_a.y + bt * ha.y);
            acc_b = mk(acc_b.x + bt * hb.x, acc_b.y + bt * hb.y);
        }
        __syncthreads();
    }
}

template <int P, int TR>
__global__ __launch_bounds__(64) void adjoint_kernel(AdjArgs a) {
    __shared__ double sbeta[kWave + 1];
    __shared__ cd sha[kWave], shb[kWave];
    __shared__ double sb[2 * kWave];
    // widths 7 and 8: the factor record is read from an LDS copy every step
    // instead of being held in VGPRs, where it would not fit beside the rest
    // of the state without spilling to scratch memory (bitwise the same
    // solve: the two forms of lane_solve_with round alike)
    constexpr bool kFacLds = P >= 7;
    __shared__ cd sfac[kFacLds ? fac_fields(P) * kWave : 1];
    const int tix = a.task0 + blockIdx.x;   // task index (per-task buffers)
    const Task task = a.tasks[tix];
    const int k = task.k, b = task.b, f = task.f;
    const int t = threadIdx.x;
    const int n = a.J[k] + 1, o = a.off[k];
    const int nt = a.nt, ns_ = a.ns;
    const bool lif = k > 0, rif = k < a.N - 1;
    const int s = t * P;
    const int lastl = (n - 1) / P;
    const cd zero = mk(0, 0);
    const double kap = a.kappa, hk = a.h / 12.0;

    if (TR == TR_S02) {
        sbeta[t] = a.beta[t];
        if (t == 0) sbeta[kWave] = a.beta[kWave];
        __syncthreads();
    }
    LaneFac<P> F;
    if (kFacLds) {
        const cd* src = a.fac + (size_t)f * a.fstride;
        for (int i = t; i < fac_fields(P) * kWave; i += kWave) sfac[i] = src[i];
        __syncthreads();
    } else {
        load_fac<P>(a.fac + (size_t)f * a.fstride + t, F);
    }
    // one solve of the step (kFacLds: the record is read anew every step --
    // the compiler would otherwise keep it in VGPRs across the time loop)
    auto solve = [&](const cd (&dd)[P], cd (&xx)[P]) {
        if constexpr (kFacLds) {
            asm volatile("" ::: "memory");
            lane_solve_with<P>(FacLds<P>{sfac + t}, dd, xx);
        } else {
            lane_solve<P>(F, dd, xx);
        }
    };

    double wl[P], wr[P], wlast[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int i = s + q;
        wl[q] = (i >= 1 && i <= n - 1) ? 1.0 : 0.0;
        wr[q] = (i <= n - 2) ? 1.0 : 0.0;
        wlast[q] = (i == n - 1) ? 1.0 : 0.0;
    }
    auto at_last = [&](const cd (&arr)[P]) {
        cd r = zero;
#pragma unroll
        for (int q = 0; q < P; ++q) r = mk(r.x + wlast[q] * arr[q].x, r.y + wlast[q] * arr[q].y);
        return rdlane(r, lastl);
    };
    // c M x at my nodes (local P1 mass: 1,4,1 inside, 2,1 / 1,2 at the ends)
    auto mass = [&](const cd (&xx)[P], cd (&out)[P]) {
        const cd xL = shfl_up1z(xx[P - 1]);
        const cd xR = shfl_dn1z(xx[0]);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const cd up = (q == 0) ? xL : xx[q - 1];
            const cd un = (q + 1 < P) ? xx[q + 1] : xR;
            const double wc = 2.0 * (wl[q] + wr[q]);
            const cd sum = mk(wl[q] * up.x + wc * xx[q].x + wr[q] * un.x,
                              wl[q] * up.y + wc * xx[q].y + wr[q] * un.y);
            out[q] = kap * mul_i(sum);
        }
    };

    // adjoint dual data: conj(gbar), split half/half at interface nodes
    cd w[P];
    const cd* gb = a.gbar + (size_t)b * a.nx + o;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int i = s + q;
        cd v = (i < n) ? conjc(gb[i]) : zero;
        if ((i == 0 && lif) || (i == n - 1 && rif)) v = 0.5 * v;
        w[q] = v;
    }
    double gv[P];
#pragma unroll
    for (int q = 0; q < P; ++q) gv[q] = 0.0;

    cd* Ha = a.hist + (size_t)tix * 2 * (nt + 1);
    cd* Hb = Ha + (nt + 1);
    if (TR == TR_S02 && t == 0) { Ha[0] = zero; Hb[0] = zero; }
    const cd* gin_l = (lif && a.g_in) ? a.g_in + ((size_t)b * ns_ + 2 * k - 1) * nt : nullptr;
    const cd* gin_r = (rif && a.g_in) ? a.g_in + ((size_t)b * ns_ + 2 * k) * nt : nullptr;
    cd* out_l = (lif && a.g_out) ? a.g_out + ((size_t)b * ns_ + 2 * k - 2) * nt : nullptr;
    cd* out_r = (rif && a.g_out) ? a.g_out + ((size_t)b * ns_ + 2 * k + 1) * nt : nullptr;
    // forward replay
    const cd* fw_l = (lif && a.grad) ? a.g_fwd + ((size_t)b * ns_ + 2 * k - 1) * nt : nullptr;
    const cd* fw_r = (rif && a.grad) ? a.g_fwd + ((size_t)b * ns_ + 2 * k) * nt : nullptr;
    const cd* Fa = a.grad ? a.hist_fwd + (size_t)tix * 2 * (nt + 1) : nullptr;
    const cd* Fb = Fa ? Fa + (nt + 1) : nullptr;
    cd* seg = a.grad ? a.seg + (size_t)tix * kWave * a.pstride * kWave + t : nullptr;

    for (int m0 = 0; m0 < nt; m0 += kWave) {
        const int nb = min(kWave, nt - m0);
        const bool act = t < nb;
        if (a.grad) {
            // ---- replay forward steps ns+1 .. ns+nb from the checkpoint ----
            const int jj = m0 / kWave + 1;
            const int nsf = max(0, nt - kWave * jj);
            cd uf[P];
            const cd* ck = a.ckpt + (((size_t)tix * (a.Jc + 1) + jj) * a.pstride) * kWave + t;
#pragma unroll
            for (int q = 0; q < P; ++q) uf[q] = ck[q * kWave];
            cd lf = zero, rf = zero;
            if (act) {
                if (fw_l) lf = fw_l[nsf + t];
                if (fw_r) rf = fw_r[nsf + t];
            }
            cd fa = zero, fb = zero;
            if (TR == TR_S02) far_history(Fa, Fb, a.beta, nsf, sha, shb, sb, fa, fb);
            for (int i = 0; i < nb; ++i) {
                const cd ln = rdlane(lf, i), rn = rdlane(rf, i);
                cd hA = zero, hB = zero;
                if (TR == TR_S02) {
                    hA = a.c2 * rdlane(fa, i);
                    hB = a.c2 * rdlane(fb, i);
                }
                cd d[P];
                mass(uf, d);
                const cd tb = rif ? (hB - rn) : zero;
#pragma unroll
                for (int q = 0; q < P; ++q) d[q] = mk(d[q].x + wlast[q] * tb.x, d[q].y + wlast[q] * tb.y);
                if (lif && t == 0) d[0] = d[0] + (hA - ln);
                cd x[P];
                solve(d, x);
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    uf[q] = mk(2.0 * x[q].x - uf[q].x, 2.0 * x[q].y - uf[q].y);
                    seg[((size_t)i * a.pstride + q) * kWave] = x[q];
                }
                if (TR == TR_S02) {
                    // boundary values by cross-lane reads: every lane must take part
                    const cd va = rdlane(x[0], 0), vb = at_last(x);
                    if (t > i) {
                        const double bt = sbeta[t - i];
                        fa = fa + bt * va;
                        fb = fb + bt * vb;
                    }
                }
            }
        }
        // ---- adjoint steps m0+1 .. m0+nb (forward steps ne .. ne-nb+1) ----
        cd lb = zero, rb = zero;
        if (act) {
            if (gin_l) lb = gin_l[m0 + t];
            if (gin_r) rb = gin_r[m0 + t];
        }
        cd acc_a = zero, acc_b = zero;
        if (TR == TR_S02) far_history(Ha, Hb, a.beta, m0, sha, shb, sb, acc_a, acc_b);
        cd rl_b = zero, rr_b = zero, va_b = zero, vb_b = zero;
        for (int i = 0; i < nb; ++i) {
            const cd ln = rdlane(lb, i), rn = rdlane(rb, i);
            cd hA = zero, hB = zero;
            if (TR == TR_S02) {
                hA = a.c2 * rdlane(acc_a, i);
                hB = a.c2 * rdlane(acc_b, i);
            }
            cd d[P];
            const cd tb = rif ? (hB - rn) : zero;
#pragma unroll
            for (int q = 0; q < P; ++q) d[q] = mk(w[q].x + wlast[q] * tb.x, w[q].y + wlast[q] * tb.y);
            if (lif && t == 0) d[0] = d[0] + (hA - ln);
            cd x[P];
            solve(d, x);
            // w_m = 2 c M Q - w_{m-1}
            cd cm[P];
            mass(x, cm);
#pragma unroll
            for (int q = 0; q < P; ++q) w[q] = mk(2.0 * cm[q].x - w[q].x, 2.0 * cm[q].y - w[q].y);
            if (a.grad) {
                // dJ/dV_i -= 2 Re Q^T (dM_V/dV_i) v over the elements of node i
                const int is = nb - 1 - i;            // forward step ns+1+is
                cd v[P];
#pragma unroll
                for (int q = 0; q < P; ++q) v[q] = seg[((size_t)is * a.pstride + q) * kWave];
                const cd xL = shfl_up1z(x[P - 1]), xR = shfl_dn1z(x[0]);
                const cd vL = shfl_up1z(v[P - 1]), vR = shfl_dn1z(v[0]);
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const cd qm = (q == 0) ? xL : x[q - 1], qp = (q + 1 < P) ? x[q + 1] : xR;
                    const cd am = (q == 0) ? vL : v[q - 1], ap = (q + 1 < P) ? v[q + 1] : vR;
                    const cd qi = x[q], ai = v[q];
                    double r = 0.0;
                    if (wl[q] != 0.0) r += ((madd(qm * (am + ai), qi, am + 3.0 * ai))).x;
                    if (wr[q] != 0.0) r += ((madd(qi * (3.0 * ai + ap), qp, ai + ap))).x;
                    gv[q] -= 2.0 * hk * r;
                }
            }
            const cd va = rdlane(x[0], 0), vb = at_last(x);
            const cd rhoL = (2.0 * madd(hA, a.sigma, va)) - ln;
            const cd rhoR = (2.0 * madd(hB, a.sigma, vb)) - rn;
            if (t == i) { rl_b = rhoL; rr_b = rhoR; va_b = va; vb_b = vb; }
            if (TR == TR_S02 && t > i) {
                const double bt = sbeta[t - i];
                acc_a = acc_a + bt * va;
                acc_b = acc_b + bt * vb;
            }
        }
        if (act) {
            if (out_l) out_l[m0 + t] = rl_b;
            if (out_r) out_r[m0 + t] = rr_b;
            if (TR == TR_S02) {
                Ha[m0 + 1 + t] = va_b;
                Hb[m0 + 1 + t] = vb_b;
            }
        }
    }

    if (a.grad) {
        double* dV = a.dV + (size_t)b * a.nx + o;
        cd* du = a.du0 + (size_t)b * a.nx + o;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int gi = s + q;
            if (gi > 0 && gi < n - 1) {
                dV[gi] = gv[q];
                du[gi] = conjc(w[q]);
            }
        }
        double g_first = rdlane(gv[0], 0), g_last = 0.0;
        {
            double r = 0.0;
#pragma unroll
            for (int q = 0; q < P; ++q) r += wlast[q] * gv[q];
            g_last = rdlane(r, lastl);
        }
        const cd w_first = rdlane(w[0], 0), w_last = at_last(w);
        if (t == 0) {
            a.gends[((size_t)b * a.N + k) * 2 + 0] = g_first;
            a.gends[((size_t)b * a.N + k) * 2 + 1] = g_last;
            a.wends[((size_t)b * a.N + k) * 2 + 0] = w_first;
            a.wends[((size_t)b * a.N + k) * 2 + 1] = w_last;
        }
    }
}

// dJ/dV and dJ/du0 at nodes shared by two subdomains: the two local parts
// add (element sums of dJ/dV; pieces of the assembled dual vector P_0).
__global__ void finalize_grad_kernel(int N, int nx, int B, const int* off, const double* gends,
                                     const cd* wends, double* dV, cd* du0) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * (N + 1)) return;
    const int b = idx / (N + 1), j = idx % (N + 1);
    const double* ge = gends + (size_t)b * N * 2;
    const cd* we = wends + (size_t)b * N * 2;
    double* v = dV + (size_t)b * nx;
    cd* u = du0 + (size_t)b * nx;
    if (j == 0) { v[0] = ge[0]; u[0] = conjc(we[0]); }
    else if (j == N) { v[nx - 1] = ge[(N - 1) * 2 + 1]; u[nx - 1] = conjc(we[(N - 1) * 2 + 1]); }
    else {
        v[off[j]] = ge[(j - 1) * 2 + 1] + ge[j * 2 + 0];
        u[off[j]] = conjc(we[(j - 1) * 2 + 1] + we[j * 2 + 0]);
    }
}

template <int P>
static void launch_adj_p(const AdjArgs& a, int trans, hipStream_t st) {
    if (trans == TR_S02) adjoint_kernel<P, TR_S02><<<a.ntasks, 64, 0, st>>>(a);
    else adjoint_kernel<P, TR_ROBIN><<<a.ntasks, 64, 0, st>>>(a);
}

hipError_t launch_adjoint(const AdjArgs& a, int trans, hipStream_t st) {
    if (a.ntasks == 0) return hipSuccess;
    switch (a.P) {
        case 1: launch_adj_p<1>(a, trans, st); break;
        case 2: launch_adj_p<2>(a, trans, st); break;
        case 3: launch_adj_p<3>(a, trans, st); break;
        case 4: launch_adj_p<4>(a, trans, st); break;
        case 5: launch_adj_p<5>(a, trans, st); break;
        case 6: launch_adj_p<6>(a, trans, st); break;
        case 7: launch_adj_p<7>(a, trans, st); break;
        case 8: launch_adj_p<8>(a, trans, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finalize_grad(int N, int nx, int B, const int* off, const double* gends,
                                const cd* wends, double* dV, cd* du0, hipStream_t st) {
    const int tot = B * (N + 1);
    finalize_grad_kernel<<<(tot + 255) / 256, 256, 0, st>>>(N, nx, B, off, gends, wends, dV, du0);
    return hipGetLastError();
}

}  // namespace swr
