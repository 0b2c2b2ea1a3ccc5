// swr_sweep_long.hip -- subdomain sweeps for subdomains of more than 64 * 8
// nodes (the paper's finest grid: 4201-node subdomains at N = 1000).
//
// One wave per task as in the register sweep (swr_sweep_kernel.h), with the
// same partition solve: lane t owns the Q = ceil(n/64) consecutive nodes
// tQ .. tQ+Q-1, eliminates its chunk interior against the two neighbouring
// separators, the 64 separators are solved by the 6-level cross-lane cyclic
// reduction, and each lane recovers its interior.  What differs is where the
// per-node arrays live: a chunk of up to thousands of nodes does not fit in
// registers, so the factor record (pivot inverses, multipliers, spikes), the
// state u_{n-1}, the Thomas intermediate y and (|u|^2) the inner iterate
// live in global memory, laid out [field][64] per record so that a wave's
// access to one field is one coalesced 1 KiB transaction; each step streams
// them through the three passes of the partition solve (forward, backward,
// recovery).  The S0^2 history uses the register sweep's arithmetic
// (far_sum_s02 plus the block-before and in-block terms, same order).
// Transmissions: Robin and S0^2; potentials: static, V(t,x) (the task's own
// record refactorised every step), |u|^2 (inner fixed point of eq. AvMNL).
#include "swr_sweep_kernel.h"

namespace swr {

// W at subdomain node j (global node o + j) of a nodal row (nullptr = 0)
struct WRow {
    const double* a;      // row n (or the static potential)
    const double* b;      // row n - 1 (V(t,x): W = (a + b)/2), nullptr = static
    __device__ double operator()(int g) const {
        if (!a) return 0.0;
        return b ? 0.5 * (a[g] + b[g]) : a[g];
    }
};

// Row i of (A - sigma E) for subdomain node i (the register sweep's
// chunk_rows for one node, with W read at the node and its neighbours).
__device__ inline void long_row(int i, int n, int o, bool lif, bool rif, double h, double kap,
                                cd sigL, cd sigR, const WRow& W, cd& ra, cd& rb, cd& rc) {
    ra = rb = rc = mk(0, 0);
    if (i >= n) {
        rb = mk(1, 0);
        return;
    }
    const double wi = W(o + i);
    if (i > 0) {
        const double wm = W(o + i - 1);
        rb = rb + mk(-1.0 / h + h / 12.0 * (wm + 3.0 * wi), 2.0 * kap);
        ra = mk(1.0 / h + h / 12.0 * (wm + wi), kap);
    }
    if (i < n - 1) {
        const double wp = W(o + i + 1);
        rb = rb + mk(-1.0 / h + h / 12.0 * (3.0 * wi + wp), 2.0 * kap);
        rc = mk(1.0 / h + h / 12.0 * (wi + wp), kap);
    }
    if (i == 0 && lif) rb = rb - sigL;
    if (i == n - 1 && rif) rb = rb - sigR;
}

// Factor record of lane t's chunk (fields as FacLayout for P = Q, each field
// at R[field * 64]); all 64 lanes take part (separator reduction).
__device__ inline void long_factor(cd* R, int Q, int n, int o, bool lif, bool rif, double h,
                                   double kap, cd sigL, cd sigR, const WRow& W) {
    const int t = lane_id();
    const int s = t * Q;
    const cd zero = mk(0, 0), one = mk(1, 0);
    auto F = [&](int field) -> cd& { return R[(size_t)field * kWave]; };
    const int ae_f = 5 * (Q - 1), ce_f = ae_f + 1, invB_f = ce_f + 1 + 2 * kPcrLevels;
    // forward: pivots, multipliers and the left spike alpha
    cd cpp = zero, alp = zero, ra, rb, rc;
    for (int q = 0; q < Q - 1; ++q) {
        long_row(s + q, n, o, lif, rif, h, kap, sigL, sigR, W, ra, rb, rc);
        const cd piv = (q == 0) ? rb : msub(rb, ra, cpp);
        const cd iv = inv(piv);
        const cd ai = ra * iv;
        const cd cp = rc * iv;
        alp = (q == 0) ? -(ra * iv) : -(ai * alp);
        cpp = cp;
        F(5 * q + 0) = iv;
        F(5 * q + 1) = ai;
        F(5 * q + 2) = cp;
        F(5 * q + 3) = alp;
    }
    // backward: alpha and the right spike gamma
    cd aL = one, gL = zero, aF = zero, gF = one;
    if (Q > 1) {
        long_row(s + Q - 2, n, o, lif, rif, h, kap, sigL, sigR, W, ra, rb, rc);
        cd an = F(5 * (Q - 2) + 3), gn = -(rc * F(5 * (Q - 2) + 0));
        F(5 * (Q - 2) + 4) = gn;
        aL = an;
        gL = gn;
        for (int q = Q - 3; q >= 0; --q) {
            const cd cp = F(5 * q + 2);
            gn = -(cp * gn);
            an = msub(F(5 * q + 3), cp, an);
            F(5 * q + 3) = an;
            F(5 * q + 4) = gn;
        }
        aF = F(3);
        gF = F(4);
    }
    // separator row and the reduced system
    long_row(s + Q - 1, n, o, lif, rif, h, kap, sigL, sigR, W, ra, rb, rc);
    const cd ae = ra, rbs = rb, ce = rc;
    const cd aR = shfl_dn1z(aF);
    const cd gR = shfl_dn1z(gF);
    cd At = ae * aL;
    cd Bt = madd(madd(rbs, ae, gL), ce, aR);
    cd Ct = ce * gR;
    F(ae_f) = ae;
    F(ce_f) = ce;
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
        F(ce_f + 1 + l) = k1;
        F(ce_f + 1 + kPcrLevels + l) = k2;
    }
    F(invB_f) = inv(Bt);
}

// factor records of the long subdomains of one width Q (static potential or
// none): one wave per (potential, subdomain)
__global__ __launch_bounds__(64) void factor_long_kernel(FactorArgs a, int Q) {
    const int f = blockIdx.x;
    const int k = f % a.N, v = f / a.N;
    if (a.Pk[k] != Q) return;
    const int n = a.J[k] + 1, o = a.off[k];
    const double kap = a.h / (3.0 * a.dt);
    WRow W{a.V ? a.V + (size_t)v * a.nx : nullptr, nullptr};
    long_factor(a.fac + (size_t)f * a.fstride + lane_id(), Q, n, o, k > 0, k < a.N - 1, a.h, kap,
                a.sigma, a.sigma, W);
}

// ---------------------------------------------------------------------------
// The sweep.  Per task the work record holds U (u_{n-1}), Y (the Thomas
// intermediate), Z (|u|^2: the inner iterate; v_{n-1} at a step start), and
// for V(t,x) the task's own factor record, each field [64] per lane.
// ---------------------------------------------------------------------------
template <int TR, int VK>
__global__ __launch_bounds__(64) void sweep_long_kernel(SweepArgs a) {
    __shared__ double sbeta[2 * kWave];
    __shared__ cd sha[kWave], shb[kWave];
    __shared__ double sb[2 * kWave];
    const int Q = a.lq;
    const int tix = a.task0 + blockIdx.x;
    const Task task = a.tasks[tix];
    const int k = task.k, b = task.b, f = task.f;
    const int fl = (task.flags & a.flags_and) | a.flags_or;
    const int t = threadIdx.x;
    const int n = a.J[k] + 1, o = a.off[k];
    const int nt = a.nt;
    const bool lif = k > 0, rif = k < a.N - 1;
    const int s = t * Q;
    const int lastl = (n - 1) / Q;          // lane holding node n-1
    const int qlast = (n - 1) - lastl * Q;  // its position in that chunk
    const cd zero = mk(0, 0);
    const double kap = a.kappa;

    if (TR == TR_S02) {
        sbeta[t] = a.beta[t];
        sbeta[kWave + t] = a.beta[kWave + t];
        __syncthreads();
    }
    cd* Ha = (TR == TR_S02) ? a.hist + (size_t)tix * 2 * (nt + 1) : nullptr;
    cd* Hb = Ha ? Ha + (nt + 1) : nullptr;

    // the task's work record
    const int fields = 5 * (Q - 1) + 2 + 2 * kPcrLevels + 1;
    const size_t wrec = (size_t)(3 * Q + (VK == VK_TIME ? fields : 0)) * kWave;
    cd* wk = a.lwork + (size_t)tix * wrec + t;
    cd* U = wk;
    cd* Y = wk + (size_t)Q * kWave;
    cd* Z = wk + (size_t)2 * Q * kWave;
    cd* R = (VK == VK_TIME) ? wk + (size_t)3 * Q * kWave : a.lfac + (size_t)f * a.lfstride + t;
    auto at = [&](cd* base, int q) -> cd& { return base[(size_t)q * kWave]; };
    const int ae_f = 5 * (Q - 1), ce_f = ae_f + 1, invB_f = ce_f + 1 + 2 * kPcrLevels;

    // u_0 (and v_0 = u_0: the |u|^2 iteration's first start)
    const bool data = (fl & T_DATA_U0) != 0;
    const cd* u0 = a.u0 + (size_t)b * a.nx + o;
    for (int q = 0; q < Q; ++q) {
        const cd uq = (data && s + q < n) ? u0[s + q] : zero;
        at(U, q) = uq;
        if (VK == VK_CUBIC) at(Z, q) = uq;
    }
    auto node = [&](cd* base, int lane, int q) {   // value at (lane, q), every lane calls
        return rdlane(at(base, min(q, Q - 1)), lane);
    };
    const cd va0 = node(U, 0, 0), vb0 = node(U, lastl, qlast);
    if (TR == TR_S02 && t == 0) {
        Ha[0] = va0;
        Hb[0] = vb0;
    }
    const bool snap = (fl & T_OUT_SNAP) != 0;
    auto put_snap = [&](int nstep) {
        const int j = nstep / a.snap_stride;
        cd* sp = a.snaps + ((size_t)b * a.nsnap + j) * a.nx + o;
        for (int q = 0; q < Q; ++q) {
            const int gi = s + q;
            if (gi > 0 && gi < n - 1) sp[gi] = at(U, q);
        }
        const cd ua = node(U, 0, 0), ub = node(U, lastl, qlast);
        if (t == 0) {
            cd* se = a.snap_ends + (((size_t)b * a.nsnap + j) * a.N + k) * 2;
            se[0] = ua;
            se[1] = ub;
        }
    };
    if (snap) put_snap(0);
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
    int nl_worst = 0, nl_fail = 0;

    // c M u_{n-1} at my node q (P1 mass: 1, 4, 1 inside; 2, 1 / 1, 2 at the
    // ends) given u at q - 1, q, q + 1
    auto mass_rhs = [&](int q, cd um, cd uq, cd up) {
        const int i = s + q;
        const double wl = (i >= 1 && i <= n - 1) ? 1.0 : 0.0;
        const double wr = (i <= n - 2) ? 1.0 : 0.0;
        const double wc = 2.0 * (wl + wr);
        const cd sum = mk(wl * um.x + wc * uq.x + wr * up.x, wl * um.y + wc * uq.y + wr * up.y);
        return kap * mul_i(sum);
    };
    // generalised mass of |z|^2 applied to z at node q (eq. AvMNL, R2)
    auto nl_term = [&](int q, cd zm, cd zq, cd zp) {
        const int i = s + q;
        const double hk = a.h / 12.0;
        const double fm = abs2(zm), fi = abs2(zq), fp = abs2(zp);
        cd r = zero;
        if (i >= 1 && i <= n - 1) r = r + hk * ((fm + fi) * zm + (fm + 3.0 * fi) * zq);
        if (i <= n - 2) r = r + hk * ((3.0 * fi + fp) * zq + (fi + fp) * zp);
        return r;
    };

    // S0^2: the terms of the "block before" the first one, i.e. v_0 (lag 64 + t
    // - 63 from the first block's point of view), as the register sweep adds
    // them at a launch start
    cd nxt_a = zero, nxt_b = zero;
    if (TR == TR_S02) {
        const double bt = sbeta[kWave + t - (kWave - 1)];
        nxt_a = mk(fma(bt, va0.x, nxt_a.x), fma(bt, va0.y, nxt_a.y));
        nxt_b = mk(fma(bt, vb0.x, nxt_b.x), fma(bt, vb0.y, nxt_b.y));
    }

    for (int n0 = 0; n0 < nt; n0 += kWave) {
        const int nb = min(kWave, nt - n0);
        const bool act = t < nb;
        cd lb = zero, rb = zero;
        if (act) {
            if (gin_l) lb = gin_l[n0 + t];
            if (gin_r) rb = gin_r[n0 + t];
            if ((fl & T_IMP_L) && n0 + t == 0) lb = mk(1, 0);
            if ((fl & T_IMP_R) && n0 + t == 0) rb = mk(1, 0);
        }
        cd acc_a = zero, acc_b = zero;
        if (TR == TR_S02) {
            cd fa, fb;
            __threadfence_block();
            far_sum_s02(a, Ha, Hb, n0, t, sha, shb, sb, fa, fb,
                        a.far_old ? a.far_old + (size_t)tix * 2 * kFarSuper : nullptr);
            acc_a = fa + nxt_a;
            acc_b = fb + nxt_b;
            nxt_a = zero;
            nxt_b = zero;
        }
        cd rl_b = zero, rr_b = zero, va_b = zero, vb_b = zero, ua_b = zero, ub_b = zero;

        for (int i = 0; i < nb; ++i) {
            const int nstep = n0 + 1 + i;
            if (VK == VK_TIME) {
                // W_n = (V_n + V_{n-1})/2 (eq. CNS_L): the task's record for this step
                WRow W{a.Vt + (size_t)nstep * a.nx, a.Vt + (size_t)(nstep - 1) * a.nx};
                long_factor(R, Q, n, o, lif, rif, a.h, kap, a.sigma, a.sigma, W);
            }
            const cd ln = rdlane(lb, i), rn = rdlane(rb, i);
            cd hA = zero, hB = zero;
            if (TR == TR_S02) {
                hA = a.c2 * rdlane(acc_a, i);
                hB = a.c2 * rdlane(acc_b, i);
            }
            const cd bA = lif ? (hA - ln) : zero;   // boundary term of node 0
            const cd bB = rif ? (hB - rn) : zero;   // boundary term of node n-1
            // u at the neighbouring chunks' edge nodes
            const cd uL = shfl_up_c(at(U, Q - 1), 1, zero);
            const cd uR = shfl_dn_c(at(U, 0), 1, zero);
            // one partition solve of (A - sigma E) x = d(z) into Y / x (z: |u|^2 inner iterate)
            auto solve = [&](bool nonlin, cd& X) {
                cd zL = zero, zR = zero;
                if (nonlin) {
                    zL = shfl_up_c(at(Z, Q - 1), 1, zero);
                    zR = shfl_dn_c(at(Z, 0), 1, zero);
                }
                // forward pass: right-hand side and the Thomas sweep of the interior
                cd um = uL, uq = at(U, 0);
                cd zm = zL, zq = nonlin ? at(Z, 0) : zero;
                cd yp = zero, dsep = zero;
                for (int q = 0; q < Q; ++q) {
                    const cd up = (q + 1 < Q) ? at(U, q + 1) : uR;
                    cd d = mass_rhs(q, um, uq, up);
                    if (s + q == 0) d = d + bA;
                    if (s + q == n - 1) d = d + bB;
                    if (nonlin) {
                        const cd zp = (q + 1 < Q) ? at(Z, q + 1) : zR;
                        d = d - nl_term(q, zm, zq, zp);
                        zm = zq;
                        zq = zp;
                    }
                    if (q < Q - 1) {
                        yp = msub(d * at(R, 5 * q + 0), at(R, 5 * q + 1), yp);
                        at(Y, q) = yp;
                    } else {
                        dsep = d;
                    }
                    um = uq;
                    uq = up;
                }
                // backward pass
                cd yn = (Q > 1) ? at(Y, Q - 2) : zero;
                const cd yL = yn;
                for (int q = Q - 3; q >= 0; --q) {
                    yn = msub(at(Y, q), at(R, 5 * q + 2), yn);
                    at(Y, q) = yn;
                }
                const cd yR = (Q > 1) ? shfl_dn1z(yn) : zero;
                cd D = msub(msub(dsep, at(R, ae_f), yL), at(R, ce_f), yR);
#pragma unroll
                for (int l = 0; l < kPcrLevels; ++l) {
                    const int dd = 1 << l;
                    const cd Dm = shfl_up_raw(D, dd), Dp = shfl_dn_raw(D, dd);
                    D = msub(msub(D, at(R, ce_f + 1 + l), Dm), at(R, ce_f + 1 + kPcrLevels + l), Dp);
                }
                X = D * at(R, invB_f);
            };
            cd X;
            if (VK == VK_CUBIC) {
                // inner fixed point of eq. AvMNL from zeta^0 = v_{n-1} (in Z)
                int it = 1;
                bool conv = false;
                for (; it <= a.nl_maxit; ++it) {
                    solve(true, X);
                    const cd Xm = shfl_up1z(X);
                    double dm = 0.0, zm2 = 0.0;
                    for (int q = 0; q < Q; ++q) {
                        const cd x = (q < Q - 1) ? madd(madd(at(Y, q), at(R, 5 * q + 3), Xm), at(R, 5 * q + 4), X) : X;
                        const cd z = at(Z, q);
                        if (s + q < n) {
                            dm = fmax(dm, abs2(x - z));
                            zm2 = fmax(zm2, abs2(z));
                        }
                        at(Z, q) = x;
                    }
                    const double dmax = sqrt(wave_max(dm)), zmax = sqrt(wave_max(zm2));
                    if (dmax <= a.nl_tol * fmax(1.0, zmax)) { conv = true; break; }
                }
                if (!conv) nl_fail = 1;
                nl_worst = max(nl_worst, conv ? it : a.nl_maxit);
            } else {
                solve(false, X);
                const cd Xm = shfl_up1z(X);
                for (int q = 0; q < Q; ++q)
                    at(Z, q) = (q < Q - 1) ? madd(madd(at(Y, q), at(R, 5 * q + 3), Xm), at(R, 5 * q + 4), X) : X;
            }
            // v_n in Z; u_n = 2 v_n - u_{n-1}
            for (int q = 0; q < Q; ++q) {
                const cd x = at(Z, q), uo = at(U, q);
                at(U, q) = mk(2.0 * x.x - uo.x, 2.0 * x.y - uo.y);
            }
            if (snap && nstep % a.snap_stride == 0) put_snap(nstep);
            const cd va = node(Z, 0, 0), vb = node(Z, lastl, qlast);
            const cd rhoL = (2.0 * madd(hA, a.sigma, va)) - ln;
            const cd rhoR = (2.0 * madd(hB, a.sigma, vb)) - rn;
            if (t == i) {
                rl_b = rhoL;
                rr_b = rhoR;
                va_b = va;
                vb_b = vb;
            }
            if (trace_a) {
                const cd ua = node(U, 0, 0), ub = node(U, lastl, qlast);
                if (t == i) { ua_b = ua; ub_b = ub; }
            }
            if (TR == TR_S02) {
                if (t > i) {
                    const double bt = sbeta[t - i];
                    acc_a = acc_a + bt * va;
                    acc_b = acc_b + bt * vb;
                }
                const double bn = sbeta[kWave + t - i];
                nxt_a = mk(fma(bn, va.x, nxt_a.x), fma(bn, va.y, nxt_a.y));
                nxt_b = mk(fma(bn, vb.x, nxt_b.x), fma(bn, vb.y, nxt_b.y));
            }
        }
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
        for (int q = 0; q < Q; ++q) {
            const int gi = s + q;
            if (gi > 0 && gi < n - 1) uT[gi] = at(U, q);
        }
        const cd ua = node(U, 0, 0), ub = node(U, lastl, qlast);
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
    if (VK == VK_CUBIC && t == 0 && a.nl_stats) {
        atomicMax(&a.nl_stats[0], nl_worst);
        if (nl_fail) atomicMax(&a.nl_stats[1], 1);
    }
}

hipError_t launch_factor_long(const FactorArgs& a, int Q, hipStream_t st) {
    if (Q <= kMaxP || Q > kLongMaxQ) return hipErrorInvalidValue;
    factor_long_kernel<<<a.nf, 64, 0, st>>>(a, Q);
    return hipGetLastError();
}

hipError_t launch_sweep_long(const SweepArgs& a, int trans, int vk, hipStream_t st) {
    if (a.ntasks == 0) return hipSuccess;
    if (a.lq <= kMaxP || a.lq > kLongMaxQ || !a.lwork) return hipErrorInvalidValue;
    if (vk != VK_TIME && !a.lfac) return hipErrorInvalidValue;
    // one launch over the whole window (no chunked launches, no checkpoints)
    if (a.n_begin != 0 || a.n_end != a.nt) return hipErrorInvalidValue;
    const dim3 g(a.ntasks), blk(64);
    if (trans == TR_S02) {
        if (vk == VK_TIME) sweep_long_kernel<TR_S02, VK_TIME><<<g, blk, 0, st>>>(a);
        else if (vk == VK_CUBIC) sweep_long_kernel<TR_S02, VK_CUBIC><<<g, blk, 0, st>>>(a);
        else sweep_long_kernel<TR_S02, VK_STATIC><<<g, blk, 0, st>>>(a);
    } else if (trans == TR_ROBIN) {
        if (vk == VK_TIME) sweep_long_kernel<TR_ROBIN, VK_TIME><<<g, blk, 0, st>>>(a);
        else if (vk == VK_CUBIC) sweep_long_kernel<TR_ROBIN, VK_CUBIC><<<g, blk, 0, st>>>(a);
        else sweep_long_kernel<TR_ROBIN, VK_STATIC><<<g, blk, 0, st>>>(a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace swr
