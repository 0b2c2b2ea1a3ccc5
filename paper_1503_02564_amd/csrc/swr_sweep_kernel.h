// swr_sweep_kernel.h -- the subdomain sweep kernel template (see the
// description at the top of swr_sweep.hip).  Included by the three
// translation units that instantiate it for one potential kind each, so
// the instantiations compile in parallel.
#pragma once
#include "swr_lane.h"

namespace swr {

// Threads per workgroup of the sweep: with HELP (S0^2, launches of at most
// SweepArgs::help_max tasks -- by default kHelpMaxTasks, so that every wave
// has a SIMD of its own; a schedule parameter) a second wave sums the far
// history beside the sweep (far_helper below); otherwise one wave does
// everything, with the same arithmetic in the same order.
__host__ __device__ constexpr int sweep_threads(bool help) { return help ? 2 * kWave : kWave; }

// The far part of the S0^2 history on the workgroup's second wave.  The main
// wave marches blocks of 64 steps, n0 = nbeg, nbeg + 64, ...; for block n0 it
// needs, in lane j (output step n0+1+j), sum_{s <= n0} beta_{n0+1+j-s} x_s.
// The terms s <= n0 - 64 use values stored at least one block earlier: this
// wave sums them for the next block while the main wave runs the current one
// and hands them over through LDS (double buffer, one barrier per block, the
// same count as the main wave's).  The main wave adds the 64 terms of the
// block just finished, which it accumulates step by step.
//
// The sum itself (far_sum_s02): lane t, output step nj = n0 + 1 + t, adds
// beta_{nj-q} x_q for q = 0 .. n0 - 64 in ascending order (one FMA chain per
// component).  The past values come in chunks of 64 staged in LDS with one
// coalesced load each, together with the 127-entry window of beta the chunk
// meets; the loads of the next chunk are issued before the current one is
// summed, so the wave waits for memory about once per chunk boundary instead
// of once per few terms.  Only the calling wave touches the staging buffers,
// and a wave's LDS operations complete in order, so no workgroup barrier is
// needed (the helper wave cannot take one: the main wave does not join).
// Positions past the last term hold zeros, which add exact zeros.
//
// Split at super-chunks (fo non-null): the time window is cut into
// super-chunks of kFarSuper steps, and for a block of the super-chunk that
// starts at step C > 0 the terms q <= C - 65 (the "old" part, the same for
// all its blocks) come precomputed from far_old_kernel as one lower-triangular
// Toeplitz product per super-chunk on the matrix cores, fo[e * kFarSuper +
// j] for the super-chunk's output j and end e; the chain here starts from
// that value and adds q = C - 64 .. n0 - 64 (at most kFarSuper - 63 terms)
// in ascending order.  Launches of such sweeps end at super-chunk
// boundaries.
__device__ inline void far_sum_s02(const SweepArgs& a, const cd* Ha, const cd* Hb, int n0, int t,
                                   cd* sha, cd* shb, double* sb, cd& fa, cd& fb, const cd* fo) {
    const cd zero = mk(0, 0);
    const int qmax = n0 - kWave;
    const int nj = n0 + 1 + t;
    fa = zero;
    fb = zero;
    const int C = n0 - n0 % kFarSuper;
    int q0s = 0;
    if (fo && C > 0) {
        fa = fo[(n0 - C) + t];
        fb = fo[kFarSuper + (n0 - C) + t];
        q0s = C - kWave;
    }
    cd pa = zero, pb = zero;
    double p0 = 0.0, p1 = 0.0;
    auto fetch = [&](int q0) {
        const int qn = min(kWave, qmax + 1 - q0);
        const int bbase = n0 - q0 - (kWave - 2);   // beta index of sb[0]
        pa = zero;
        pb = zero;
        if (t < qn) { pa = Ha[q0 + t]; pb = Hb[q0 + t]; }
        p0 = 0.0;
        p1 = 0.0;
        if (bbase + t >= 0) p0 = a.beta[bbase + t];
        if (bbase + kWave + t >= 0) p1 = a.beta[bbase + kWave + t];
    };
    if (qmax >= q0s) fetch(q0s);
    for (int q0 = q0s; q0 <= qmax; q0 += kWave) {
        const int bbase = n0 - q0 - (kWave - 2);
        sha[t] = pa;
        shb[t] = pb;
        sb[t] = p0;
        sb[kWave + t] = p1;
        if (q0 + kWave <= qmax) fetch(q0 + kWave);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double* bw = sb + (nj - q0 - bbase);  // beta_{nj - q0 - i} = bw[-i]
#pragma unroll 16
        for (int i = 0; i < kWave; ++i) {
            const double bt = bw[-i];
            const cd ha = sha[i], hb = shb[i];
            fa = mk(fma(bt, ha.x, fa.x), fma(bt, ha.y, fa.y));
            fb = mk(fma(bt, hb.x, fb.x), fma(bt, hb.y, fb.y));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

__device__ inline void far_helper(const SweepArgs& a, const cd* Ha, const cd* Hb, int t,
                                  cd (*ffa)[kWave], cd (*ffb)[kWave], cd* sha, cd* shb,
                                  double* sb, const cd* fo) {
    const int nbeg = a.n_begin, nend = a.n_end;
    auto far = [&](int n0, int buf) {
        cd fa, fb;
        far_sum_s02(a, Ha, Hb, n0, t, sha, shb, sb, fa, fb, fo);
        ffa[buf][t] = fa;
        ffb[buf][t] = fb;
    };
    far(nbeg, 0);
    __syncthreads();
    int kb = 0;
    for (int n0 = nbeg; n0 < nend; n0 += kWave, ++kb) {
        if (n0 + kWave < nend) far(n0 + kWave, (kb + 1) & 1);
        __syncthreads();
    }
}

// Coefficients of the higher-order operators at one interface end for end
// data W, dn W (Sec. 2.2; the EndCoef form, see swr_common.h): cp, cm of the
// parity-split beta/alpha sums, the order-4 prefactor aa of e^{i calW_n} G_n
// with the weight gw of each stored value in G (S0^4: aa = -i (dn W/4)(dt/2),
// gw = 1; S1^4: aa = -i sgn(dn W) q (dt/2), gw = q = sqrt|dn W|/2), the
// implicit coefficient sig and the exchanged sig_s (without order-4 terms).
__device__ inline void gen_end_coef(int tr, double W, double dW, double dt, cd c2, cd& cp, cd& cm,
                                    cd& aa, cd& sig, cd& sig_s, double& gw) {
    const bool pot = tr == 2 || tr == 3, ord4 = tr == 3 || tr == 5;
    const cd eP = mk(M_SQRT1_2, M_SQRT1_2);                 // e^{i pi/4}
    const cd d = pot ? (-(sqrt(0.5 * dt) * 0.5 * W)) * eP : mk(0, 0);
    cp = c2 + d;
    cm = c2 - d;
    sig_s = c2 + d;
    aa = mk(0, 0);
    gw = 1.0;
    cd s4 = mk(0, 0);
    if (ord4 && pot) {
        aa = mk(0.0, -(dW / 4.0) * (0.5 * dt));
        s4 = aa;
    } else if (ord4) {
        const double q = 0.5 * sqrt(fabs(dW));
        const double sg = dW > 0.0 ? 1.0 : (dW < 0.0 ? -1.0 : 0.0);
        aa = mk(0.0, -(sg * q) * (0.5 * dt));
        s4 = q * aa;
        gw = q;
    }
    sig = sig_s + s4;
}

// ---------------------------------------------------------------------------
// The sweep.  VK selects the potential: static (factors loaded once), time
// dependent (rows rebuilt and refactored every step from the streamed V rows)
// or |u|^2 (V-free factors, inner fixed point of eq. AvMNL every step).
// ---------------------------------------------------------------------------
//
// GRP: the workgroup's waves run a group of tasks that share one factor record
// (one subdomain, one potential: the problems of a batch, the impulse tasks),
// a.groups[task0 + blockIdx.x] = (first task, count); the record is copied
// once into LDS and every wave's solve reads it from there instead of holding
// it in VGPRs, which leaves room for more waves per SIMD.  The arithmetic is
// the one-wave form's, term for term.  Dynamic LDS: the record, then per wave
// the staging of the far history (2 * 64 complex + 2 * 64 doubles).
template <int P, int TR, int VK, bool HELP = false, bool GRP = false>
__global__ __launch_bounds__(GRP ? kGroupMax * kWave : sweep_threads(HELP)) void sweep_kernel(SweepArgs a) {
    static_assert(!HELP || TR == TR_S02, "the helper wave serves S0^2");
    static_assert(!GRP || (!HELP && VK == VK_STATIC && (TR == TR_S02 || TR == TR_ROBIN)),
                  "shared-factor groups: static potential, Robin or S0^2");
    __shared__ double sbeta[2 * kWave];       // beta_0 .. beta_127
    __shared__ cd ffa[2][kWave], ffb[2][kWave];   // S0^2: far sums from the helper wave
    __shared__ cd sha[kWave], shb[kWave];     // staged chunk of the boundary history
    __shared__ double sb[2 * kWave];          // beta window of that chunk
    extern __shared__ cd sgrp[];              // GRP: factor record, then per-wave staging
    constexpr int kFacN = fac_fields(P) * kWave;
    const int t = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;     // 1: the S0^2 helper wave; GRP: the group member
    int tix = a.task0 + blockIdx.x;         // task index (per-task buffers)
    int gcount = 1;
    if (GRP) {
        const int2 g = a.groups[a.task0 + blockIdx.x];
        gcount = g.y;
        tix = g.x + min(wv, g.y - 1);
    }
    const Task task = a.tasks[tix];
    const int k = task.k, b = task.b, f = task.f;
    const int fl = (task.flags & a.flags_and) | a.flags_or;
    const int n = a.J[k] + 1, o = a.off[k];
    const int nt = a.nt;
    const bool lif = k > 0, rif = k < a.N - 1;
    const int s = t * P;
    const int lastl = (n - 1) / P;          // lane holding node n-1
    const cd zero = mk(0, 0);

    if (GRP) {
        // every task of the group has this record (f)
        const cd* src = a.fac + (size_t)f * a.fstride;
        for (int i = threadIdx.x; i < kFacN; i += blockDim.x) sgrp[i] = src[i];
    }
    if (TR == TR_S02 || TR == TR_GEN || GRP) {
        if (wv == 0 && (TR == TR_S02 || TR == TR_GEN)) {
            sbeta[t] = a.beta[t];
            sbeta[kWave + t] = a.beta[kWave + t];
        }
        __syncthreads();
    }
    if (GRP && wv >= gcount) return;        // a short group: no later workgroup barrier
    // this wave's staging of the far history
    cd* wsha = sha;
    cd* wshb = shb;
    double* wsb = sb;
    if (GRP) {
        wsha = sgrp + kFacN + wv * 2 * kWave;
        wshb = wsha + kWave;
        wsb = reinterpret_cast<double*>(sgrp + kFacN + (blockDim.x / kWave) * 2 * kWave) + wv * 2 * kWave;
    }
    cd* Ha = a.hist ? a.hist + (size_t)tix * 2 * (nt + 1) : nullptr;
    cd* Hb = Ha ? Ha + (nt + 1) : nullptr;
    // S0^2 split at super-chunks: this task's old far-history part
    const cd* fo = a.far_old ? a.far_old + (size_t)tix * 2 * kFarSuper : nullptr;
    if (HELP && wv == 1) {
        far_helper(a, Ha, Hb, t, ffa, ffb, sha, shb, sb, fo);
        return;
    }
    // higher-order and Pade operators: coefficients of the two ends (left, right)
    EndCoef ea{}, eb{};
    if (TR == TR_GEN || TR == TR_PADE) {
        ea = a.endc[(size_t)f * 2 + 0];
        eb = a.endc[(size_t)f * 2 + 1];
    }

    LaneFac<P> F;
    // this launch advances steps nbeg+1 .. nend; a launch that does not
    // start at step 0 resumes from the state the previous one saved
    const int nbeg = a.n_begin, nend = a.n_end;
    const bool first = nbeg == 0, last = nend == nt;
    cd* stp = a.state ? a.state + (size_t)tix * 2 * a.pstride * kWave + t : nullptr;

    // Pade strategy (Sec. 2.2): lane t carries the auxiliary functions
    // s = t + 1 and s = t + 65 of both ends, with r_s = 1/(c + W + d_s),
    // c r_s, and the history weight w_s = i a_s d_s c r_s (c = 2i/dt); psi of
    // the order-4 operator is wave-uniform.  ph[e] = sum_s w_s phi^s_{n-1}
    // (a wave sum, every lane holds it) is ready before each step.
    // Time-dependent or |u|^2 potential with the higher-order or Pade
    // operators (Sec. 2.2): the end coefficients change every step and are
    // formed per step, wave-uniform, from W_n and dn W_n at the end node --
    // V(t,x): W_n = (V_n + V_{n-1})/2, which lane j reads for step n0+1+j at
    // each block start; |u|^2: W_n = |v_{n-1}|^2 at the end node, the inner
    // fixed point's starting value (dn W unused: order 2 and 3 only).  The
    // history keeps its even- and odd-lag beta sums apart (E, O) until the
    // step's coefficients are known; the gauge phase is advanced step by step
    // (calV_n = calV_{n-1} + dt W_n, calW_n the mean of the two, as in the
    // oracle) and the order-4 sum G_n = 2 sum_{s<n} q_s x_s (q_s =
    // sqrt|dn W_s|/2 for S1^4, 1 for S0^4) is a running sum; both are carried
    // across launches in the second half of the state record.
    constexpr bool TEND = (VK == VK_TIME || VK == VK_CUBIC) && (TR == TR_GEN || TR == TR_PADE);
    const int trc = a.tr;
    const bool g_gauge = trc == 4 || trc == 5;
    cd Ga = zero, Gb = zero;          // TR_GEN: G_n of the two ends
    double cvA = 0.0, cvB = 0.0;      // TEND gauge: calV_{n-1} of the two ends
    // W_n and dn W_n at global node g (outward sign ns), rows n and n-1 of V
    auto end_data = [&](int nj, int g, double ns, double& W, double& dW) {
        const double* Vn = a.Vt + (size_t)nj * a.nx;
        const double* Vm = a.Vt + (size_t)(nj > 0 ? nj - 1 : 0) * a.nx;
        W = 0.5 * (Vn[g] + Vm[g]);
        const double wm = 0.5 * (Vn[g - 1] + Vm[g - 1]), wp = 0.5 * (Vn[g + 1] + Vm[g + 1]);
        dW = ns * (wp - wm) / (2.0 * a.h);
    };

    cd pr[2][2], pkr[2][2], pw[2][2], pphi[2][2], ppsi[2], ph[2], pad[2];
    double pq[2] = {0.0, 0.0}, psg[2] = {0.0, 0.0};
    cd pkrho[2], prho[2], pasum = zero;
    const bool ord4 = TR == TR_PADE && a.pade_order == 4;
    cd* pst = (TR == TR_PADE && a.pstate) ? a.pstate + (size_t)tix * 6 * kWave + t : nullptr;
    const cd pcc = mk(0.0, 2.0 / a.dt);
    auto pade_sum = [&](int e) {
        const cd p = pw[e][0] * pphi[e][0] + pw[e][1] * pphi[e][1];
        return mk(wave_sum(p.x), wave_sum(p.y));
    };
    // r_s = 1/(c + W + d_s), c r_s, w_s = i a_s d_s c r_s at end e for the
    // end potential W; rho = 1/(c + W) and the order-4 weight from dn W
    auto pade_coef = [&](int e, double W, double dW) {
        const cd* pd = a.pade + a.pade_m + 1;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int sl = t + 1 + j * kWave;
            pr[e][j] = pkr[e][j] = pw[e][j] = zero;
            if (sl <= a.pade_m) {
                pr[e][j] = inv(mk(pcc.x + W + pd[sl].x, pcc.y + pd[sl].y));
                pkr[e][j] = pcc * pr[e][j];
                pw[e][j] = pad[j] * pkr[e][j];
            }
        }
        prho[e] = inv(mk(pcc.x + W, pcc.y));
        pkrho[e] = pcc * prho[e];
        pq[e] = ord4 ? 0.5 * sqrt(fabs(dW)) : 0.0;
        psg[e] = dW > 0.0 ? 1.0 : (dW < 0.0 ? -1.0 : 0.0);
    };
    if (TR == TR_PADE) {
        const cd* pa = a.pade;
        const cd* pd = a.pade + a.pade_m + 1;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int sl = t + 1 + j * kWave;
            pad[j] = (sl <= a.pade_m) ? mul_i(pa[sl] * pd[sl]) : zero;
        }
        for (int q = 0; q <= a.pade_m; ++q) pasum = pasum + pa[q];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
                pphi[e][j] = (!first && pst && t + 1 + j * kWave <= a.pade_m) ? pst[(2 * e + j) * kWave] : zero;
            ppsi[e] = (ord4 && !first && pst) ? pst[(4 + e) * kWave] : zero;
            if (!TEND) {
                const EndCoef& ec = e ? eb : ea;
                pade_coef(e, ec.omega, ec.pad);
                ph[e] = pade_sum(e);
            }
        }
    }

    // time-dependent potential: rows n and n+1 of V at my nodes
    double vprev[P], vnext[P];
    const double* Vt = (VK == VK_TIME) ? a.Vt + o : nullptr;
    if (VK == VK_TIME) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            vprev[q] = (s + q < n) ? Vt[(size_t)nbeg * a.nx + s + q] : 0.0;
            vnext[q] = (s + q < n) ? Vt[(size_t)(nbeg + 1) * a.nx + s + q] : 0.0;
        }
    } else if (!GRP) {
        load_fac<P>(a.fac + (size_t)f * a.fstride + t, F);
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

    // state u_0 (and v_0 = u_0, the first guess of the |u|^2 inner iteration)
    cd u[P], vlast[P];
    const bool data = (fl & T_DATA_U0) != 0;
    const cd* u0 = a.u0 + (size_t)b * a.nx + o;
    if (first) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            u[q] = zero;
            if (data && s + q < n) u[q] = u0[s + q];
            vlast[q] = u[q];
        }
    } else {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            u[q] = stp[q * kWave];
            vlast[q] = (VK == VK_CUBIC) ? stp[(a.pstride + q) * kWave] : u[q];
        }
    }
    auto at_last = [&](const cd (&arr)[P]) {
        cd r = zero;
#pragma unroll
        for (int q = 0; q < P; ++q) r = mk(r.x + wlast[q] * arr[q].x, r.y + wlast[q] * arr[q].y);
        return rdlane(r, lastl);
    };

    const double kap = a.kappa;
    const cd va0 = rdlane(u[0], 0);
    const cd vb0 = at_last(u);
    // history value at step 0: v_0 (calW_0 = 0, so also x_0 = v_0)
    if ((TR == TR_S02 || TR == TR_GEN) && t == 0 && first) {
        Ha[0] = va0;
        Hb[0] = vb0;
    }
    // checkpoints for the adjoint: u at forward steps max(0, nt - 64 jj), jj = 1..Jc
    cd* ck = (fl & T_CKPT) ? a.ckpt + ((size_t)tix * (a.Jc + 1) * a.pstride) * kWave + t : nullptr;
    if (ck && first) {
#pragma unroll
        for (int q = 0; q < P; ++q) ck[((size_t)a.Jc * a.pstride + q) * kWave] = u[q];
    }
    // snapshots u_n, n = 0, stride, 2 stride, ...: interior nodes straight to
    // the output, the two end nodes to a side store (averaged across the
    // interface afterwards, as u(T))
    const bool snap = (fl & T_OUT_SNAP) != 0;
    auto put_snap = [&](int nstep) {
        const int j = nstep / a.snap_stride;
        cd* sp = a.snaps + ((size_t)b * a.nsnap + j) * a.nx + o;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int gi = s + q;
            if (gi > 0 && gi < n - 1) sp[gi] = u[q];
        }
        const cd ua = rdlane(u[0], 0), ub = at_last(u);
        if (t == 0) {
            cd* se = a.snap_ends + (((size_t)b * a.nsnap + j) * a.N + k) * 2;
            se[0] = ua;
            se[1] = ub;
        }
    };
    if (snap && first) put_snap(0);
    cd* trace_a = (fl & T_OUT_TRACE) ? a.trace + ((size_t)(b * a.N + k) * 2) * (nt + 1) : nullptr;
    cd* trace_b = trace_a ? trace_a + (nt + 1) : nullptr;
    if (trace_a && t == 0 && first) {
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

    // S0^2: the 64 history terms of the block before the first one of this
    // launch (s in (nbeg-64, nbeg]), in the order in which a running block
    // accumulates them for its successor, then the barrier that pairs with
    // the helper's first one
    cd nxt_a = zero, nxt_b = zero;
    if (TR == TR_S02) {
        __threadfence_block();
#pragma unroll 8
        for (int i = 0; i < kWave; ++i) {
            const int q = nbeg - kWave + 1 + i;
            if (q >= 0) {
                const double bt = sbeta[kWave + t - i];
                const cd xa = Ha[q], xb = Hb[q];
                nxt_a = mk(fma(bt, xa.x, nxt_a.x), fma(bt, xa.y, nxt_a.y));
                nxt_b = mk(fma(bt, xb.x, nxt_b.x), fma(bt, xb.y, nxt_b.y));
            }
        }
        if (HELP) __syncthreads();
    }

    // TEND: G and calV at the launch start (the state record's second half
    // carries them across launches: lane 0 G of the left end, lane 1 of the
    // right end, lane 2 the two calV)
    if (TEND && TR == TR_GEN) {
        if (first) {
            double w0, dw0, gw0a = 1.0, gw0b = 1.0;
            if (trc == 5 && lif) { end_data(0, o, -1.0, w0, dw0); gw0a = 0.5 * sqrt(fabs(dw0)); }
            if (trc == 5 && rif) { end_data(0, o + n - 1, 1.0, w0, dw0); gw0b = 0.5 * sqrt(fabs(dw0)); }
            Ga = (2.0 * gw0a) * va0;
            Gb = (2.0 * gw0b) * vb0;
        } else if (stp) {
            const cd sv = stp[a.pstride * kWave];
            Ga = rdlane(sv, 0);
            Gb = rdlane(sv, 1);
            const cd cv = rdlane(sv, 2);
            cvA = cv.x;
            cvB = cv.y;
        }
    }

    int kb = 0;
    for (int n0 = nbeg; n0 < nend; n0 += kWave, ++kb) {
        const int nb = min(kWave, nend - n0);
        const bool act = t < nb;
        // incoming fluxes of this block: lane j <-> step n0+1+j
        cd lb = zero, rb = zero;
        if (act) {
            if (gin_l) lb = gin_l[n0 + t];
            if (gin_r) rb = gin_r[n0 + t];
            if ((fl & T_IMP_L) && n0 + t == 0) lb = mk(1, 0);
            if ((fl & T_IMP_R) && n0 + t == 0) rb = mk(1, 0);
        }
        // far part of the history for the outputs of this block,
        // acc_j = sum_{q <= n0} beta_{n0+1+j-q} x_q.  S0^2: the helper
        // wave's terms q <= n0 - 64 plus the running sum of the block before.
        // Higher-order operators: summed here over chunks of 64 past values
        // staged in LDS with one coalesced load each, together with the
        // 127-entry window of beta the chunk needs, split by the parity of i
        // (acc for even i, acc1 for odd i), with each lane's running sum of
        // the staged values for G
        cd acc_a = zero, acc_b = zero, acc_a1 = zero, acc_b1 = zero, gs_a = zero, gs_b = zero;
        if (TR == TR_S02) {
            // terms s <= n0 - 64 (from the helper wave, or summed here in the
            // same order over staged chunks) plus the block before
            cd fa = zero, fb = zero;
            if (HELP) {
                fa = ffa[kb & 1][t];
                fb = ffb[kb & 1][t];
            } else {
                __threadfence_block();
                far_sum_s02(a, Ha, Hb, n0, t, wsha, wshb, wsb, fa, fb, fo);
            }
            acc_a = fa + nxt_a;
            acc_b = fb + nxt_b;
            nxt_a = zero;
            nxt_b = zero;
        }
        if (TR == TR_GEN) {
            __threadfence_block();
            const int nj = n0 + 1 + t;
            // the loads of chunk q0 + 64 are issued before chunk q0 is summed
            cd pa = zero, pb = zero;
            double pb0 = 0.0, pb1 = 0.0;
            auto fetch = [&](int q0) {
                const int qn = min(kWave, n0 + 1 - q0);
                const int bbase = n0 - q0 - (kWave - 2);   // beta index of sb[0]
                pa = (t < qn) ? Ha[q0 + t] : mk(0, 0);
                pb = (t < qn) ? Hb[q0 + t] : mk(0, 0);
                const int i0 = bbase + t, i1 = bbase + kWave + t;
                pb0 = (i0 >= 0) ? a.beta[i0] : 0.0;
                pb1 = (i1 >= 0) ? a.beta[i1] : 0.0;
            };
            fetch(0);
            for (int q0 = 0; q0 <= n0; q0 += kWave) {
                const int qn = min(kWave, n0 + 1 - q0);
                const int bbase = n0 - q0 - (kWave - 2);   // beta index of sb[0]
                sha[t] = pa;
                shb[t] = pb;
                gs_a = gs_a + pa;
                gs_b = gs_b + pb;
                sb[t] = pb0;
                sb[kWave + t] = pb1;
                if (q0 + kWave <= n0) fetch(q0 + kWave);
                __syncthreads();
                const double* bw = sb + (nj - q0 - bbase);  // beta_{nj - q0 - i} = bw[-i]
                // all 64 entries: the staged chunk is zero past qn and the beta
                // window bw[-i], i < 64, stays inside sb, so the loop unrolls and
                // its LDS reads overlap
                #pragma unroll 8
                for (int i = 0; i < kWave; i += 2) {
                    const double b0 = bw[-i], b1 = bw[-i - 1];
                    const cd h0 = sha[i], h1 = sha[i + 1], k0 = shb[i], k1 = shb[i + 1];
                    acc_a = mk(acc_a.x + b0 * h0.x, acc_a.y + b0 * h0.y);
                    acc_a1 = mk(acc_a1.x + b1 * h1.x, acc_a1.y + b1 * h1.y);
                    acc_b = mk(acc_b.x + b0 * k0.x, acc_b.y + b0 * k0.y);
                    acc_b1 = mk(acc_b1.x + b1 * k1.x, acc_b1.y + b1 * k1.y);
                }
                __syncthreads();
            }
        }
        // higher-order operators: lane j's history Hl = cp E + cm O of step
        // nj = n0+1+j (lag nj - q0 - i has the parity of nj - i, q0 being a
        // multiple of 64), its phase e^{i calW_nj}, and the wave-uniform
        // G = 2 sum_{s <= n0} x_s
        // static: Hl = cp E + cm O; TEND: Hl = E and Ho = O (coefficients per step)
        cd Hl_a = zero, Hl_b = zero, Ho_a = zero, Ho_b = zero, pha = mk(1, 0), phb = mk(1, 0);
        double eWa = 0.0, edWa = 0.0, eWb = 0.0, edWb = 0.0;   // V(t,x): lane j's step
        if (TEND && VK == VK_TIME) {
            const int nj = min(n0 + 1 + t, nt);
            if (lif) end_data(nj, o, -1.0, eWa, edWa);
            if (rif) end_data(nj, o + n - 1, 1.0, eWb, edWb);
        }
        if (TR == TR_GEN) {
            const int nj = n0 + 1 + t;
            const bool odd = (nj & 1) != 0;
            if (TEND) {
                Hl_a = odd ? acc_a1 : acc_a;
                Ho_a = odd ? acc_a : acc_a1;
                Hl_b = odd ? acc_b1 : acc_b;
                Ho_b = odd ? acc_b : acc_b1;
            } else {
                Hl_a = ea.cp * (odd ? acc_a1 : acc_a) + ea.cm * (odd ? acc_a : acc_a1);
                Hl_b = eb.cp * (odd ? acc_b1 : acc_b) + eb.cm * (odd ? acc_b : acc_b1);
            }
            if (!TEND) {
                Ga = 2.0 * mk(wave_sum(gs_a.x), wave_sum(gs_a.y));
                Gb = 2.0 * mk(wave_sum(gs_b.x), wave_sum(gs_b.y));
                double sn, cs;
                sincos(((double)nj - 0.5) * ea.omega, &sn, &cs);
                pha = mk(cs, sn);
                sincos(((double)nj - 0.5) * eb.omega, &sn, &cs);
                phb = mk(cs, sn);
            }
        }
        cd rl_b = zero, rr_b = zero, va_b = zero, vb_b = zero, ua_b = zero, ub_b = zero;

        for (int i = 0; i < nb; ++i) {
            const int nstep = n0 + 1 + i;
            // GRP: read the LDS factor record anew every step (the compiler
            // would otherwise keep it in VGPRs across the loop)
            if (GRP) asm volatile("" ::: "memory");
            // implicit coefficients of this step's boundary rows and of the
            // exchange (static potential: constant)
            cd sgA_n = a.sigma, sgB_n = a.sigma, sgsA_n = a.sigma, sgsB_n = a.sigma;
            cd phA = mk(1, 0), phB = mk(1, 0);
            // end data of this step (TEND)
            double WA_n = 0.0, dWA_n = 0.0, WB_n = 0.0, dWB_n = 0.0;
            if (TEND && VK == VK_TIME) {
                WA_n = rdlane(eWa, i);
                dWA_n = rdlane(edWa, i);
                WB_n = rdlane(eWb, i);
                dWB_n = rdlane(edWb, i);
            }
            if (TEND && VK == VK_CUBIC) {
                WA_n = abs2(rdlane(vlast[0], 0));
                WB_n = abs2(at_last(vlast));
            }
            cd cpA_n = ea.cp, cmA_n = ea.cm, cpB_n = eb.cp, cmB_n = eb.cm, aA_n = ea.a, aB_n = eb.a;
            double gwA_n = 1.0, gwB_n = 1.0;
            if (TR == TR_GEN) {
                sgsA_n = ea.sig_s;
                sgsB_n = eb.sig_s;
                sgA_n = ea.sig;
                sgB_n = eb.sig;
                if (TEND) {
                    gen_end_coef(trc, WA_n, dWA_n, a.dt, a.c2, cpA_n, cmA_n, aA_n, sgA_n, sgsA_n, gwA_n);
                    gen_end_coef(trc, WB_n, dWB_n, a.dt, a.c2, cpB_n, cmB_n, aB_n, sgB_n, sgsB_n, gwB_n);
                    if (g_gauge) {
                        // calV_n = calV_{n-1} + dt W_n, calW_n = (calV_n + calV_{n-1})/2
                        const double wa = WA_n, wb = WB_n;
                        const double na = cvA + a.dt * wa, nbv = cvB + a.dt * wb;
                        double sn, cs;
                        sincos(0.5 * (na + cvA), &sn, &cs);
                        phA = mk(cs, sn);
                        sincos(0.5 * (nbv + cvB), &sn, &cs);
                        phB = mk(cs, sn);
                        cvA = na;
                        cvB = nbv;
                    }
                } else {
                    phA = rdlane(pha, i);
                    phB = rdlane(phb, i);
                }
            }
            if (TR == TR_PADE) {
                if (TEND) {
                    // this step's r_s, w_s from W_n; history sums; implicit part
                    // -i sum a_s + i sum a_s d_s r_s (+ (dn W/4) rho at order 4)
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const double we = e ? WB_n : WA_n, dwe = e ? dWB_n : dWA_n;
                        pade_coef(e, we, dwe);
                        ph[e] = pade_sum(e);
                        const cd p = pad[0] * pr[e][0] + pad[1] * pr[e][1];
                        const cd ss = mk(wave_sum(p.x), wave_sum(p.y)) - mul_i(pasum);
                        const cd sg = ord4 ? ss + (dwe / 4.0) * prho[e] : ss;
                        if (e) { sgsB_n = ss; sgB_n = sg; } else { sgsA_n = ss; sgA_n = sg; }
                    }
                } else {
                    sgsA_n = ea.sig_s;
                    sgsB_n = eb.sig_s;
                }
            }
            if (VK == VK_TIME) {
                // W_n = (V_n + V_{n-1})/2 (eq. CNS_L); refactor for this step
                double w[P];
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    w[q] = 0.5 * (vnext[q] + vprev[q]);
                    vprev[q] = vnext[q];
                }
                if (nstep < nt) {
#pragma unroll
                    for (int q = 0; q < P; ++q)
                        vnext[q] = (s + q < n) ? Vt[(size_t)(nstep + 1) * a.nx + s + q] : 0.0;
                }
                double wL, wR;
                neighbour_w(w, wL, wR);
                cd ra[P], rbr[P], rc[P];
                chunk_rows<P>(s, n, lif, rif, a.h, kap, sgA_n, sgB_n, w, wL, wR, ra, rbr, rc);
                lane_factor<P>(ra, rbr, rc, F);
            }
            if (VK == VK_CUBIC && TEND) {
                // |u|^2 with a W-dependent operator: the V-free matrix with this
                // step's implicit coefficients, fixed over the inner iteration
                double w[P];
#pragma unroll
                for (int q = 0; q < P; ++q) w[q] = 0.0;
                cd ra[P], rbr[P], rc[P];
                chunk_rows<P>(s, n, lif, rif, a.h, kap, sgA_n, sgB_n, w, 0.0, 0.0, ra, rbr, rc);
                lane_factor<P>(ra, rbr, rc, F);
            }
            const cd ln = rdlane(lb, i), rn = rdlane(rb, i);
            // history part of Sbar v_n at each end: hA (all terms, boundary
            // condition) and hAs (without the order-4 term, the exchange)
            cd hA = zero, hB = zero, hAs = zero, hBs = zero;
            if (TR == TR_S02) {
                hA = a.c2 * rdlane(acc_a, i);
                hB = a.c2 * rdlane(acc_b, i);
                hAs = hA;
                hBs = hB;
            }
            if (TR == TR_GEN) {
                if (TEND) {
                    hAs = phA * (cpA_n * rdlane(Hl_a, i) + cmA_n * rdlane(Ho_a, i));
                    hBs = phB * (cpB_n * rdlane(Hl_b, i) + cmB_n * rdlane(Ho_b, i));
                } else {
                    hAs = phA * rdlane(Hl_a, i);
                    hBs = phB * rdlane(Hl_b, i);
                }
                hA = hAs + aA_n * (phA * Ga);
                hB = hBs + aB_n * (phB * Gb);
            }
            if (TR == TR_PADE) {
                hAs = ph[0];
                hBs = ph[1];
                hA = hAs;
                hB = hBs;
                if (ord4) {
                    // + sgn(dn W) (sqrt|dn W|/2) c psi_{n-1} / (c + W)
                    hA = hA + (psg[0] * pq[0]) * (pkrho[0] * ppsi[0]);
                    hB = hB + (psg[1] * pq[1]) * (pkrho[1] * ppsi[1]);
                }
            }
            // right-hand side c M u_{n-1} + boundary terms
            const cd uL = shfl_up1z(u[P - 1]);
            const cd uR = shfl_dn1z(u[0]);
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
            cd x[P];
            if (VK == VK_CUBIC) {
                // inner fixed point of eq. AvMNL from zeta^0 = v_{n-1}:
                // (cM - S - sigma E) zeta^{s+1} = rhs - M_{|zeta^s|^2} zeta^s
                cd z[P];
#pragma unroll
                for (int q = 0; q < P; ++q) z[q] = vlast[q];
                const double hk = a.h / 12.0;
                int it = 1;
                bool conv = false;
                for (; it <= a.nl_maxit; ++it) {
                    double Fz[P];
#pragma unroll
                    for (int q = 0; q < P; ++q) Fz[q] = abs2(z[q]);
                    const cd zL = shfl_up1z(z[P - 1]), zR = shfl_dn1z(z[0]);
                    // neighbours' |zeta|^2: the shuffles run on every lane
                    // (a lane left out of a permute hands zero to its reader)
                    const double FLs = __shfl(Fz[P - 1], t > 0 ? t - 1 : 0);
                    const double FRs = __shfl(Fz[0], t < kWave - 1 ? t + 1 : kWave - 1);
                    const double FL = t > 0 ? FLs : 0.0;
                    const double FR = t < kWave - 1 ? FRs : 0.0;
                    cd r[P];
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        // generalised mass with nodal weight |zeta|^2 (same
                        // element matrix as M_W)
                        const cd zm = (q == 0) ? zL : z[q - 1];
                        const cd zp = (q == P - 1) ? zR : z[q + 1];
                        const double fm = (q == 0) ? FL : Fz[q - 1];
                        const double fp = (q == P - 1) ? FR : Fz[q + 1];
                        const double fi = Fz[q];
                        cd nl = zero;
                        if (wl[q] != 0.0) nl = nl + hk * ((fm + fi) * zm + (fm + 3.0 * fi) * z[q]);
                        if (wr[q] != 0.0) nl = nl + hk * ((3.0 * fi + fp) * z[q] + (fi + fp) * zp);
                        r[q] = d[q] - nl;
                    }
                    lane_solve<P>(F, r, x);
                    double dm = 0.0, zm2 = 0.0;
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        if (s + q < n) {
                            dm = fmax(dm, abs2(x[q] - z[q]));
                            zm2 = fmax(zm2, abs2(z[q]));
                        }
                        z[q] = x[q];
                    }
                    const double dmax = sqrt(wave_max(dm)), zmax = sqrt(wave_max(zm2));
                    if (dmax <= a.nl_tol * fmax(1.0, zmax)) { conv = true; break; }
                }
                if (!conv) nl_fail = 1;
                nl_worst = max(nl_worst, conv ? it : a.nl_maxit);
#pragma unroll
                for (int q = 0; q < P; ++q) vlast[q] = x[q];
            } else if (GRP) {
                lane_solve_with<P>(FacLds<P>{sgrp + t}, d, x);
            } else {
                lane_solve<P>(F, d, x);
            }
            // advance u_n = 2 v_n - u_{n-1}
#pragma unroll
            for (int q = 0; q < P; ++q) u[q] = mk(2.0 * x[q].x - u[q].x, 2.0 * x[q].y - u[q].y);
            if (snap && nstep % a.snap_stride == 0) put_snap(nstep);
            if (ck && nstep < nt && ((nt - nstep) & (kWave - 1)) == 0) {
                const int jj = (nt - nstep) / kWave;
#pragma unroll
                for (int q = 0; q < P; ++q) ck[((size_t)jj * a.pstride + q) * kWave] = u[q];
            }
            const cd va = rdlane(x[0], 0);
            const cd vb = at_last(x);
            const cd sgA = sgsA_n;
            const cd sgB = sgsB_n;
            const cd rhoL = (2.0 * madd(hAs, sgA, va)) - ln;
            const cd rhoR = (2.0 * madd(hBs, sgB, vb)) - rn;
            // stored history value: x_n = e^{-i calW_n} v_n (= v_n for S0^2)
            const cd xa = (TR == TR_GEN) ? conjc(phA) * va : va;
            const cd xb = (TR == TR_GEN) ? conjc(phB) * vb : vb;
            if (t == i) {
                rl_b = rhoL;
                rr_b = rhoR;
                va_b = xa;
                vb_b = xb;
            }
            if (trace_a) {
                const cd ua = rdlane(u[0], 0), ub = at_last(u);
                if (t == i) { ua_b = ua; ub_b = ub; }
            }
            if (TR == TR_S02) {
                if (t > i) {
                    const double bt = sbeta[t - i];
                    acc_a = acc_a + bt * va;
                    acc_b = acc_b + bt * vb;
                }
                // this value's term for the next block (lag 64 + t - i)
                const double bn = sbeta[kWave + t - i];
                nxt_a = mk(fma(bn, va.x, nxt_a.x), fma(bn, va.y, nxt_a.y));
                nxt_b = mk(fma(bn, vb.x, nxt_b.x), fma(bn, vb.y, nxt_b.y));
            }
            if (TR == TR_PADE) {
                // phi^s_n = 2 r_s (v_n + c phi^s_{n-1}) - phi^s_{n-1}, psi alike;
                // then the history sums of the next step
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const cd ve = e ? vb : va;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const cd half = pr[e][j] * ve + pkr[e][j] * pphi[e][j];
                        pphi[e][j] = 2.0 * half - pphi[e][j];
                    }
                    if (ord4) {
                        const cd half = (pq[e] * ve) * prho[e] + pkrho[e] * ppsi[e];
                        ppsi[e] = 2.0 * half - ppsi[e];
                    }
                    if (!TEND) ph[e] = pade_sum(e);
                }
            }
            if (TR == TR_GEN) {
                if (t > i) {
                    const int lag = t - i;
                    const double bt = sbeta[lag];
                    if (TEND) {
                        if (lag & 1) {
                            Ho_a = Ho_a + bt * xa;
                            Ho_b = Ho_b + bt * xb;
                        } else {
                            Hl_a = Hl_a + bt * xa;
                            Hl_b = Hl_b + bt * xb;
                        }
                    } else {
                        Hl_a = Hl_a + (bt * ((lag & 1) ? ea.cm : ea.cp)) * xa;
                        Hl_b = Hl_b + (bt * ((lag & 1) ? eb.cm : eb.cp)) * xb;
                    }
                }
                if (TEND) {
                    Ga = Ga + (2.0 * gwA_n) * xa;
                    Gb = Gb + (2.0 * gwB_n) * xb;
                } else {
                    Ga = Ga + 2.0 * xa;
                    Gb = Gb + 2.0 * xb;
                }
            }
        }
        // block epilogue: coalesced stores
        if (act) {
            if (out_l) out_l[n0 + t] = rl_b;
            if (out_r) out_r[n0 + t] = rr_b;
            if (old_l) maxd = fmax(maxd, sqrt(abs2(rl_b - old_l[n0 + t])));
            if (old_r) maxd = fmax(maxd, sqrt(abs2(rr_b - old_r[n0 + t])));
            if (TR == TR_S02 || TR == TR_GEN) {
                Ha[n0 + 1 + t] = va_b;
                Hb[n0 + 1 + t] = vb_b;
            }
            if (trace_a) {
                trace_a[n0 + 1 + t] = ua_b;
                trace_b[n0 + 1 + t] = ub_b;
            }
        }
        // S0^2: the block's history values are stored; the helper's sums
        // for the next block are in LDS
        if (HELP) __syncthreads();
    }

    if (!last && stp) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            stp[q * kWave] = u[q];
            if (VK == VK_CUBIC) stp[(a.pstride + q) * kWave] = vlast[q];
        }
    }
    if (TEND && TR == TR_GEN && !last && stp)
        stp[a.pstride * kWave] = (t == 0) ? Ga : ((t == 1) ? Gb : mk(cvA, cvB));
    if (TR == TR_PADE && !last && pst) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
#pragma unroll
            for (int j = 0; j < 2; ++j) pst[(2 * e + j) * kWave] = pphi[e][j];
            pst[(4 + e) * kWave] = ppsi[e];
        }
    }
    if ((fl & T_OUT_UT) && last) {
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
    if (VK == VK_CUBIC && t == 0 && a.nl_stats) {
        atomicMax(&a.nl_stats[0], nl_worst);
        if (nl_fail) atomicMax(&a.nl_stats[1], 1);
    }
}

}  // namespace swr
