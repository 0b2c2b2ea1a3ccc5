// swr_lane.h -- per-wavefront building blocks of the subdomain solver:
// assembly of the subdomain rows, the partition factorisation (per-lane Thomas
// on 64 chunks + parallel cyclic reduction of the separator system) and its
// right-hand-side solve.  Shared by the forward sweep and the adjoint sweep.
#pragma once
#include "swr_common.h"

namespace swr {

// Lane t owns the P consecutive nodes t*P .. t*P+P-1 of its subdomain; nodes
// at or beyond n = J_k + 1 are padding with a decoupled identity row, so every
// lane runs the same straight-line code with compile-time register indices.

// Rows of the subdomain matrix  c M - S + M_W - sig E  at my P nodes (P1
// elements on a uniform mesh, eq. AvML; the generalised mass integrates W
// interpolated in P1; sig = sigL at an interface left end, sigR at an
// interface right end).  w[q] = W at node s+q, wL / wR = W at nodes s-1 and
// s+P.  ra = coupling to node i-1, rb = diagonal, rc = coupling to node i+1.
template <int P>
__device__ inline void chunk_rows(int s, int n, bool lif, bool rif, double h, double kap, cd sigL, cd sigR,
                                  const double (&w)[P], double wL, double wR, cd (&ra)[P],
                                  cd (&rb)[P], cd (&rc)[P]) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int i = s + q;
        const double wm = (q == 0) ? wL : w[q - 1];
        const double wi = w[q];
        const double wp = (q == P - 1) ? wR : w[q + 1];
        cd a = mk(0, 0), b = mk(0, 0), c = mk(0, 0);
        if (i >= n) {
            b = mk(1, 0);                       // padding
        } else {
            if (i > 0) {
                b = b + mk(-1.0 / h + h / 12.0 * (wm + 3.0 * wi), 2.0 * kap);
                a = mk(1.0 / h + h / 12.0 * (wm + wi), kap);
            }
            if (i < n - 1) {
                b = b + mk(-1.0 / h + h / 12.0 * (3.0 * wi + wp), 2.0 * kap);
                c = mk(1.0 / h + h / 12.0 * (wi + wp), kap);
            }
            if (i == 0 && lif) b = b - sigL;
            if (i == n - 1 && rif) b = b - sigR;
        }
        ra[q] = a;
        rb[q] = b;
        rc[q] = c;
    }
}

// Per-lane factor record of the partition solve.  Chunk interior q =
// 0..P-2 is eliminated against the separators X_{t-1} (left) and X_t (right,
// node q = P-1): x_q = y_q + al_q X_{t-1} + ga_q X_t, y the Thomas solution
// for the right-hand side (pivot inverses inv, multipliers ainv = a inv,
// cp = c inv).  The separator rows then form a tridiagonal system in
// X_0..X_63 whose parallel cyclic reduction multipliers k1, k2 and final
// 1/B are kept; a step replays them on its right-hand side.
template <int P>
struct LaneFac {
    static constexpr int PI = P > 1 ? P - 1 : 1;
    cd inv[PI], ainv[PI], cp[PI], al[PI], ga[PI];
    cd ae, ce, invB;
    cd k1[kPcrLevels], k2[kPcrLevels];
};

// Field offsets inside one lane's stored factor record.
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

// Factorisation of my chunk given its rows (all 64 lanes take part: the
// separator system couples neighbouring lanes).
template <int P>
__device__ inline void lane_factor(const cd (&ra)[P], const cd (&rb)[P], const cd (&rc)[P],
                                   LaneFac<P>& F) {
    constexpr int PI = LaneFac<P>::PI;
    const int t = lane_id();
    const cd zero = mk(0, 0), one = mk(1, 0);
    cd alp = zero, cpp = zero;
#pragma unroll
    for (int q = 0; q < P - 1; ++q) {
        const cd piv = (q == 0) ? rb[q] : msub(rb[q], ra[q], cpp);
        const cd iv = inv(piv);
        const cd ai = ra[q] * iv;
        const cd cp = rc[q] * iv;
        alp = (q == 0) ? -(ra[q] * iv) : -(ai * alp);   // forward sweep of alpha
        cpp = cp;
        F.inv[q] = iv;
        F.ainv[q] = ai;
        F.cp[q] = cp;
        F.al[q] = alp;
    }
    // back substitution of alpha and gamma (gamma' = -c_{P-2} inv_{P-2} at the
    // last interior node and zero above it)
    if (P > 1) {
        cd an = F.al[PI - 1], gn = -(rc[PI - 1] * F.inv[PI - 1]);
        F.ga[PI - 1] = gn;
#pragma unroll
        for (int q = P - 3; q >= 0; --q) {
            gn = -(F.cp[q] * gn);
            an = msub(F.al[q], F.cp[q], an);
            F.al[q] = an;
            F.ga[q] = gn;
        }
    }
    // separator row and the reduced system A X_{t-1} + B X_t + C X_{t+1}
    const cd ae = ra[P - 1], rbs = rb[P - 1], ce = rc[P - 1];
    const cd aL = (P > 1) ? F.al[PI - 1] : one;
    const cd gL = (P > 1) ? F.ga[PI - 1] : zero;
    const cd aF = (P > 1) ? F.al[0] : zero;     // right neighbour's first node
    const cd gF = (P > 1) ? F.ga[0] : one;
    const cd aR = shfl_dn1z(aF);
    const cd gR = shfl_dn1z(gF);
    cd At = ae * aL;
    cd Bt = madd(madd(rbs, ae, gL), ce, aR);
    cd Ct = ce * gR;
    F.ae = ae;
    F.ce = ce;
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
        F.k1[l] = k1;
        F.k2[l] = k2;
    }
    F.invB = inv(Bt);
}

template <int P>
__device__ inline void store_fac(cd* Fp, const LaneFac<P>& F) {
    using L = FacLayout<P>;
#pragma unroll
    for (int q = 0; q < P - 1; ++q) {
        Fp[L::inv(q) * kWave] = F.inv[q];
        Fp[L::ainv(q) * kWave] = F.ainv[q];
        Fp[L::cp(q) * kWave] = F.cp[q];
        Fp[L::al(q) * kWave] = F.al[q];
        Fp[L::ga(q) * kWave] = F.ga[q];
    }
    Fp[L::ae * kWave] = F.ae;
    Fp[L::ce * kWave] = F.ce;
#pragma unroll
    for (int l = 0; l < kPcrLevels; ++l) {
        Fp[L::k1(l) * kWave] = F.k1[l];
        Fp[L::k2(l) * kWave] = F.k2[l];
    }
    Fp[L::invB * kWave] = F.invB;
}

template <int P>
__device__ inline void load_fac(const cd* Fp, LaneFac<P>& F) {
    using L = FacLayout<P>;
#pragma unroll
    for (int q = 0; q < P - 1; ++q) {
        F.inv[q] = Fp[L::inv(q) * kWave];
        F.ainv[q] = Fp[L::ainv(q) * kWave];
        F.cp[q] = Fp[L::cp(q) * kWave];
        F.al[q] = Fp[L::al(q) * kWave];
        F.ga[q] = Fp[L::ga(q) * kWave];
    }
    F.ae = Fp[L::ae * kWave];
    F.ce = Fp[L::ce * kWave];
#pragma unroll
    for (int l = 0; l < kPcrLevels; ++l) {
        F.k1[l] = Fp[L::k1(l) * kWave];
        F.k2[l] = Fp[L::k2(l) * kWave];
    }
    F.invB = Fp[L::invB * kWave];
}

// Where a right-hand-side solve reads the factor record: the lane's VGPRs
// (FacRegs) or the workgroup's LDS copy of the record (FacLds, p = the copy +
// lane id, fields kWave apart as in global memory).  Both hand the solve the
// same values, so the two forms are bitwise equal.
template <int P>
struct FacRegs {
    const LaneFac<P>& F;
    __device__ cd inv(int q) const { return F.inv[q]; }
    __device__ cd ainv(int q) const { return F.ainv[q]; }
    __device__ cd cp(int q) const { return F.cp[q]; }
    __device__ cd al(int q) const { return F.al[q]; }
    __device__ cd ga(int q) const { return F.ga[q]; }
    __device__ cd ae() const { return F.ae; }
    __device__ cd ce() const { return F.ce; }
    __device__ cd k1(int l) const { return F.k1[l]; }
    __device__ cd k2(int l) const { return F.k2[l]; }
    __device__ cd invB() const { return F.invB; }
};

template <int P>
struct FacLds {
    using L = FacLayout<P>;
    const cd* p;
    __device__ cd inv(int q) const { return p[L::inv(q) * kWave]; }
    __device__ cd ainv(int q) const { return p[L::ainv(q) * kWave]; }
    __device__ cd cp(int q) const { return p[L::cp(q) * kWave]; }
    __device__ cd al(int q) const { return p[L::al(q) * kWave]; }
    __device__ cd ga(int q) const { return p[L::ga(q) * kWave]; }
    __device__ cd ae() const { return p[L::ae * kWave]; }
    __device__ cd ce() const { return p[L::ce * kWave]; }
    __device__ cd k1(int l) const { return p[L::k1(l) * kWave]; }
    __device__ cd k2(int l) const { return p[L::k2(l) * kWave]; }
    __device__ cd invB() const { return p[L::invB * kWave]; }
};

// Complex products of the right-hand-side solve with every rounding fixed by
// explicit fused multiply-adds.  Left to the compiler, a*b - c*d may be fused
// around either product, and which one it picks depends on how the operands
// reach the expression (a factor held in a VGPR across the time loop, whose
// negation is hoisted out of it, or one read from LDS every step); with the
// roundings spelled out, the VGPR and LDS forms of the solve are bitwise equal.
__device__ inline cd cmul_x(cd a, cd b) {
#pragma clang fp contract(off)
    const double yy = a.y * b.y, yx = a.y * b.x;
    return mk(fma(a.x, b.x, -yy), fma(a.x, b.y, yx));
}
__device__ inline cd msub_x(cd a, cd b, cd c) {   // a - b c
    return mk(fma(b.y, c.y, fma(-b.x, c.x, a.x)), fma(-b.y, c.x, fma(-b.x, c.y, a.y)));
}
__device__ inline cd madd_x(cd a, cd b, cd c) {   // a + b c
    return mk(fma(-b.y, c.y, fma(b.x, c.x, a.x)), fma(b.y, c.x, fma(b.x, c.y, a.y)));
}

// Solve (A - sigma E) x = d for my chunk (all lanes take part).
template <int P, class FA>
__device__ inline void lane_solve_with(const FA& F, const cd (&d)[P], cd (&x)[P]) {
    constexpr int PI = LaneFac<P>::PI;
    const cd zero = mk(0, 0);
    cd y[PI];
    cd yp = zero;
#pragma unroll
    for (int q = 0; q < P - 1; ++q) {
        yp = msub_x(cmul_x(d[q], F.inv(q)), F.ainv(q), yp);
        y[q] = yp;
    }
#pragma unroll
    for (int q = P - 3; q >= 0; --q) y[q] = msub_x(y[q], F.cp(q), y[q + 1]);
    const cd yL = (P > 1) ? y[PI - 1] : zero;
    const cd yR = (P > 1) ? shfl_dn1z(y[0]) : zero;
    cd D = msub_x(msub_x(d[P - 1], F.ae(), yL), F.ce(), yR);
#pragma unroll
    for (int l = 0; l < kPcrLevels; ++l) {
        // k1 (k2) is zero on lanes without a partner at -dd (+dd)
        const int dd = 1 << l;
        const cd Dm = shfl_up_raw(D, dd), Dp = shfl_dn_raw(D, dd);
        D = msub_x(msub_x(D, F.k1(l), Dm), F.k2(l), Dp);
    }
    const cd X = cmul_x(D, F.invB());
    const cd Xm = shfl_up1z(X);
#pragma unroll
    for (int q = 0; q < P - 1; ++q) x[q] = madd_x(madd_x(y[q], F.al(q), Xm), F.ga(q), X);
    x[P - 1] = X;
}

template <int P>
__device__ inline void lane_solve(const LaneFac<P>& F, const cd (&d)[P], cd (&x)[P]) {
    lane_solve_with<P>(FacRegs<P>{F}, d, x);
}

// W at my nodes and at the two neighbouring nodes from a nodal array (static
// potential: V; time-dependent: (V_n + V_{n-1})/2 built by the caller).
template <int P>
__device__ inline void neighbour_w(const double (&w)[P], double& wL, double& wR) {
    const int t = lane_id();
    const double l = __shfl(w[P - 1], t > 0 ? t - 1 : 0);
    const double r = __shfl(w[0], t < kWave - 1 ? t + 1 : kWave - 1);
    wL = t > 0 ? l : 0.0;
    wR = t < kWave - 1 ? r : 0.0;
}

}  // namespace swr
