// swr_sweep_pair_kernel.h -- the subdomain sweep of two tasks per wavefront.
//
// Two sweep tasks of the same subdomain and the same potential (two problems
// of a batch, or the two impulse responses of a subdomain) share one factor
// record, so one wave can run both: every lane holds the factors of its chunk
// once and the states of both tasks, and each step interleaves the two
// independent dependency chains (right-hand side, chunk elimination, the
// cross-lane reduction of the separators, recovery, traces).  A step of one
// task is a long chain of dependent FP64 operations and cross-lane moves; a
// wave that has two of them in flight keeps the SIMD busy where one leaves
// it waiting.  Used for launches that fill the GPU with one-wave tasks
// (static potential, Robin or S0^2 transmission); every task's arithmetic is
// the one-task kernel's, term for term and in the same order, so results are
// bitwise those of swr_sweep_kernel.h.
#pragma once
#include "swr_sweep_kernel.h"

namespace swr {

constexpr int kPair = 2;

template <int P, int TR>
__global__ __launch_bounds__(kWave) void sweep_pair_kernel(SweepArgs a) {
    static_assert(TR == TR_S02 || TR == TR_ROBIN, "pairs: Robin and S0^2");
    constexpr int K = kPair;
    __shared__ double sbeta[2 * kWave];       // beta_0 .. beta_127
    __shared__ cd sha[kWave], shb[kWave];     // staged chunk of the boundary history
    __shared__ double sb[2 * kWave];          // beta window of that chunk
    const int2 pr = a.pairs[a.task0 + blockIdx.x];
    const int t = threadIdx.x;
    // the second slot of a pair that has one task repeats the first task's
    // arithmetic and stores nothing
    const int tix[K] = {pr.x, pr.y >= 0 ? pr.y : pr.x};
    const bool live[K] = {true, pr.y >= 0};
    Task task[K];
    int fl[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        task[c] = a.tasks[tix[c]];
        fl[c] = (task[c].flags & a.flags_and) | a.flags_or;
    }
    const int k = task[0].k, f = task[0].f;   // shared by both tasks
    const int n = a.J[k] + 1, o = a.off[k];
    const int nt = a.nt;
    const bool lif = k > 0, rif = k < a.N - 1;
    const int s = t * P;
    const int lastl = (n - 1) / P;
    const cd zero = mk(0, 0);

    if (TR == TR_S02) {
        sbeta[t] = a.beta[t];
        sbeta[kWave + t] = a.beta[kWave + t];
        __syncthreads();
    }
    cd* Ha[K];
    cd* Hb[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        Ha[c] = a.hist ? a.hist + (size_t)tix[c] * 2 * (nt + 1) : nullptr;
        Hb[c] = Ha[c] ? Ha[c] + (nt + 1) : nullptr;
    }
    LaneFac<P> F;
    load_fac<P>(a.fac + (size_t)f * a.fstride + t, F);
    const int nbeg = a.n_begin, nend = a.n_end;
    const bool first = nbeg == 0, last = nend == nt;
    cd* stp[K];
#pragma unroll
    for (int c = 0; c < K; ++c)
        stp[c] = a.state ? a.state + (size_t)tix[c] * 2 * a.pstride * kWave + t : nullptr;

    double wl[P], wr[P], wlast[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int i = s + q;
        wl[q] = (i >= 1 && i <= n - 1) ? 1.0 : 0.0;
        wr[q] = (i <= n - 2) ? 1.0 : 0.0;
        wlast[q] = (i == n - 1) ? 1.0 : 0.0;
    }
    cd u[K][P];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const bool data = (fl[c] & T_DATA_U0) != 0;
        const cd* u0 = a.u0 + (size_t)task[c].b * a.nx + o;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (first) {
                u[c][q] = zero;
                if (data && s + q < n) u[c][q] = u0[s + q];
            } else {
                u[c][q] = stp[c][q * kWave];
            }
        }
    }
    auto at_last = [&](const cd (&arr)[P]) {
        cd r = zero;
#pragma unroll
        for (int q = 0; q < P; ++q) r = mk(r.x + wlast[q] * arr[q].x, r.y + wlast[q] * arr[q].y);
        return rdlane(r, lastl);
    };
    const double kap = a.kappa;
    const int ns = a.ns;
    cd* ck[K];
    cd* trace_a[K];
    cd* trace_b[K];
    const cd* gin_l[K];
    const cd* gin_r[K];
    cd* out_l[K];
    cd* out_r[K];
    const cd* old_l[K];
    const cd* old_r[K];
    bool snap[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const int b = task[c].b;
        const cd va0 = rdlane(u[c][0], 0);
        const cd vb0 = at_last(u[c]);
        if (TR == TR_S02 && t == 0 && first && live[c]) {
            Ha[c][0] = va0;
            Hb[c][0] = vb0;
        }
        ck[c] = (fl[c] & T_CKPT) && live[c]
                    ? a.ckpt + ((size_t)tix[c] * (a.Jc + 1) * a.pstride) * kWave + t : nullptr;
        if (ck[c] && first) {
#pragma unroll
            for (int q = 0; q < P; ++q) ck[c][((size_t)a.Jc * a.pstride + q) * kWave] = u[c][q];
        }
        snap[c] = (fl[c] & T_OUT_SNAP) != 0 && live[c];
        trace_a[c] = (fl[c] & T_OUT_TRACE) && live[c]
                         ? a.trace + ((size_t)(b * a.N + k) * 2) * (nt + 1) : nullptr;
        trace_b[c] = trace_a[c] ? trace_a[c] + (nt + 1) : nullptr;
        if (trace_a[c] && t == 0 && first) {
            trace_a[c][0] = va0;
            trace_b[c][0] = vb0;
        }
        gin_l[c] = (lif && (fl[c] & T_FLUX_G)) ? a.g_in + ((size_t)b * ns + 2 * k - 1) * nt : nullptr;
        gin_r[c] = (rif && (fl[c] & T_FLUX_G)) ? a.g_in + ((size_t)b * ns + 2 * k) * nt : nullptr;
        out_l[c] = out_r[c] = nullptr;
        old_l[c] = old_r[c] = nullptr;
        if (!live[c]) continue;
        if (fl[c] & T_OUT_G) {
            if (lif) out_l[c] = a.g_out + ((size_t)b * ns + 2 * k - 2) * nt;
            if (rif) out_r[c] = a.g_out + ((size_t)b * ns + 2 * k + 1) * nt;
            if (fl[c] & T_MAXDIFF) {
                if (lif) old_l[c] = a.g_in + ((size_t)b * ns + 2 * k - 2) * nt;
                if (rif) old_r[c] = a.g_in + ((size_t)b * ns + 2 * k + 1) * nt;
            }
        } else if (fl[c] & T_OUT_COLS) {
            const int pl = (fl[c] & T_IMP_L) ? 0 : 1;
            if (lif) out_l[c] = a.cols + ((size_t)f * 4 + pl) * nt;
            if (rif) out_r[c] = a.cols + ((size_t)f * 4 + pl + 2) * nt;
        }
    }
    auto put_snap = [&](int c, int nstep) {
        const int j = nstep / a.snap_stride;
        const int b = task[c].b;
        cd* sp = a.snaps + ((size_t)b * a.nsnap + j) * a.nx + o;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int gi = s + q;
            if (gi > 0 && gi < n - 1) sp[gi] = u[c][q];
        }
        const cd ua = rdlane(u[c][0], 0), ub = at_last(u[c]);
        if (t == 0) {
            cd* se = a.snap_ends + (((size_t)b * a.nsnap + j) * a.N + k) * 2;
            se[0] = ua;
            se[1] = ub;
        }
    };
#pragma unroll
    for (int c = 0; c < K; ++c)
        if (snap[c] && first) put_snap(c, 0);
    double maxd[K] = {0.0, 0.0};

    // S0^2: the 64 history terms of the block before this launch's first
    cd nxt_a[K], nxt_b[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
        nxt_a[c] = zero;
        nxt_b[c] = zero;
    }
    if (TR == TR_S02) {
        __threadfence_block();
#pragma unroll 8
        for (int i = 0; i < kWave; ++i) {
            const int q = nbeg - kWave + 1 + i;
            if (q >= 0) {
                const double bt = sbeta[kWave + t - i];
#pragma unroll
                for (int c = 0; c < K; ++c) {
                    const cd xa = Ha[c][q], xb = Hb[c][q];
                    nxt_a[c] = mk(fma(bt, xa.x, nxt_a[c].x), fma(bt, xa.y, nxt_a[c].y));
                    nxt_b[c] = mk(fma(bt, xb.x, nxt_b[c].x), fma(bt, xb.y, nxt_b[c].y));
                }
            }
        }
    }

    for (int n0 = nbeg; n0 < nend; n0 += kWave) {
        const int nb = min(kWave, nend - n0);
        const bool act = t < nb;
        cd lb[K], rb[K], acc_a[K], acc_b[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            lb[c] = zero;
            rb[c] = zero;
            if (act) {
                if (gin_l[c]) lb[c] = gin_l[c][n0 + t];
                if (gin_r[c]) rb[c] = gin_r[c][n0 + t];
                if ((fl[c] & T_IMP_L) && n0 + t == 0) lb[c] = mk(1, 0);
                if ((fl[c] & T_IMP_R) && n0 + t == 0) rb[c] = mk(1, 0);
            }
            acc_a[c] = zero;
            acc_b[c] = zero;
        }
        if (TR == TR_S02) {
#pragma unroll
            for (int c = 0; c < K; ++c) {
                cd fa = zero, fb = zero;
                __threadfence_block();
                far_sum_s02(a, Ha[c], Hb[c], n0, t, sha, shb, sb, fa, fb,
                            a.far_old ? a.far_old + (size_t)tix[c] * 2 * kFarSuper : nullptr);
                acc_a[c] = fa + nxt_a[c];
                acc_b[c] = fb + nxt_b[c];
                nxt_a[c] = zero;
                nxt_b[c] = zero;
            }
        }
        cd rl_b[K], rr_b[K], va_b[K], vb_b[K], ua_b[K], ub_b[K];
#pragma unroll
        for (int c = 0; c < K; ++c) rl_b[c] = rr_b[c] = va_b[c] = vb_b[c] = ua_b[c] = ub_b[c] = zero;

        for (int i = 0; i < nb; ++i) {
            const int nstep = n0 + 1 + i;
            cd x[K][P];
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const cd ln = rdlane(lb[c], i), rn = rdlane(rb[c], i);
                cd hA = zero, hB = zero;
                if (TR == TR_S02) {
                    hA = a.c2 * rdlane(acc_a[c], i);
                    hB = a.c2 * rdlane(acc_b[c], i);
                }
                const cd uL = shfl_up1z(u[c][P - 1]);
                const cd uR = shfl_dn1z(u[c][0]);
                const cd tb = rif ? (hB - rn) : zero;
                cd d[P];
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const cd up = (q == 0) ? uL : u[c][q - 1];
                    const cd un = (q + 1 < P) ? u[c][q + 1] : uR;
                    const double wc = 2.0 * (wl[q] + wr[q]);
                    const cd sum = mk(wl[q] * up.x + wc * u[c][q].x + wr[q] * un.x,
                                      wl[q] * up.y + wc * u[c][q].y + wr[q] * un.y);
                    d[q] = kap * mul_i(sum);
                    d[q] = mk(d[q].x + wlast[q] * tb.x, d[q].y + wlast[q] * tb.y);
                }
                if (lif && t == 0) d[0] = d[0] + (hA - ln);
                lane_solve<P>(F, d, x[c]);
#pragma unroll
                for (int q = 0; q < P; ++q)
                    u[c][q] = mk(2.0 * x[c][q].x - u[c][q].x, 2.0 * x[c][q].y - u[c][q].y);
                if (ck[c] && nstep < nt && ((nt - nstep) & (kWave - 1)) == 0) {
                    const int jj = (nt - nstep) / kWave;
#pragma unroll
                    for (int q = 0; q < P; ++q) ck[c][((size_t)jj * a.pstride + q) * kWave] = u[c][q];
                }
                if (snap[c] && nstep % a.snap_stride == 0) put_snap(c, nstep);
                const cd va = rdlane(x[c][0], 0);
                const cd vb = at_last(x[c]);
                const cd rhoL = (2.0 * madd(hA, a.sigma, va)) - ln;
                const cd rhoR = (2.0 * madd(hB, a.sigma, vb)) - rn;
                if (t == i) {
                    rl_b[c] = rhoL;
                    rr_b[c] = rhoR;
                    va_b[c] = va;
                    vb_b[c] = vb;
                }
                if (trace_a[c]) {
                    const cd ua = rdlane(u[c][0], 0), ub = at_last(u[c]);
                    if (t == i) { ua_b[c] = ua; ub_b[c] = ub; }
                }
                if (TR == TR_S02) {
                    if (t > i) {
                        const double bt = sbeta[t - i];
                        acc_a[c] = acc_a[c] + bt * va;
                        acc_b[c] = acc_b[c] + bt * vb;
                    }
                    const double bn = sbeta[kWave + t - i];
                    nxt_a[c] = mk(fma(bn, va.x, nxt_a[c].x), fma(bn, va.y, nxt_a[c].y));
                    nxt_b[c] = mk(fma(bn, vb.x, nxt_b[c].x), fma(bn, vb.y, nxt_b[c].y));
                }
            }
        }
        // block epilogue: coalesced stores
        if (act) {
#pragma unroll
            for (int c = 0; c < K; ++c) {
                if (out_l[c]) out_l[c][n0 + t] = rl_b[c];
                if (out_r[c]) out_r[c][n0 + t] = rr_b[c];
                if (old_l[c]) maxd[c] = fmax(maxd[c], sqrt(abs2(rl_b[c] - old_l[c][n0 + t])));
                if (old_r[c]) maxd[c] = fmax(maxd[c], sqrt(abs2(rr_b[c] - old_r[c][n0 + t])));
                if (TR == TR_S02 && live[c]) {
                    Ha[c][n0 + 1 + t] = va_b[c];
                    Hb[c][n0 + 1 + t] = vb_b[c];
                }
                if (trace_a[c]) {
                    trace_a[c][n0 + 1 + t] = ua_b[c];
                    trace_b[c][n0 + 1 + t] = ub_b[c];
                }
            }
        }
    }

#pragma unroll
    for (int c = 0; c < K; ++c) {
        if (!live[c]) continue;
        const int b = task[c].b;
        if (!last && stp[c]) {
#pragma unroll
            for (int q = 0; q < P; ++q) stp[c][q * kWave] = u[c][q];
        }
        if ((fl[c] & T_OUT_UT) && last) {
            cd* uT = a.uT + (size_t)b * a.nx + o;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int gi = s + q;
                if (gi > 0 && gi < n - 1) uT[gi] = u[c][q];
            }
            const cd ua = rdlane(u[c][0], 0), ub = at_last(u[c]);
            if (t == 0) {
                a.ends[((size_t)b * a.N + k) * 2 + 0] = ua;
                a.ends[((size_t)b * a.N + k) * 2 + 1] = ub;
            }
        }
        if (fl[c] & T_MAXDIFF) {
            const double m = wave_max(maxd[c]);
            if (t == 0 && m > 0.0) atomicMax(a.maxdiff, (unsigned long long)__double_as_longlong(m));
        }
    }
}

}  // namespace swr
