// swr_iface.hip -- the interface problem (I - L) g = d of Schwarz waveform
// relaxation (Besse & Xing, arXiv 1503.02564, Secs. 3-4) on gfx950.
//
// L is stored as the first columns of its blocks X^{k,p} (Sec. 4.1); every
// block is lower-triangular Toeplitz (Props. 3-4), so a block product is the
// causal convolution  y_n = sum_{s<=n} c_{n-s} x_s.
//
// Slot algebra (Sec. 3, vector g; eq. chp1_L_N):  output slot 2k-2 (r_{k-1})
// is written by subdomain k from columns p = 0, 1 (X^{k,1} l_k + X^{k,2} r_k);
// output slot 2k+1 (l_{k+1}) from p = 2, 3 (X^{k,3} l_k + X^{k,4} r_k); l_k
// lives in slot 2k-1 and r_k in slot 2k.
#include <algorithm>

#include "swr_common.h"

namespace swr {


__device__ inline void slot_sources(int o, int N, int& k, int& pl, int& pr, int& sl, int& sr) {
    if ((o & 1) == 0) { k = o / 2 + 1; pl = 0; pr = 1; }
    else { k = (o - 1) / 2; pl = 2; pr = 3; }
    sl = (k >= 1) ? 2 * k - 1 : -1;
    sr = (k <= N - 2) ? 2 * k : -1;
}

// ---------------------------------------------------------------------------
// Block products of L on FP64 matrix cores.
//
// For one output slot o and one source slot (column c of X^{k,p}), the part
// of y on targets n = n_lo + 16 I + row from sources s = s_lo + 16 J + kk is
//     y_I += T_{I-J} x_J,   T_m[row][kk] = c[delta + 16 m + row - kk],
// delta = n_lo - s_lo: every 16 x 16 block of a lower-triangular Toeplitz
// matrix is itself Toeplitz, fixed by the lag block m = I - J.  One wave owns
// 16 consecutive target blocks I0 .. I0+15 (256 outputs) as the columns of a
// 16 x 16 accumulator and, for each lag block m, multiplies T_m (A operand,
// 16 x 16 in four k-slices of 4) by the 16 source blocks I0+col-m (B
// operand) with v_mfma_f64_16x16x4_f64.  Complex products use the real
// embedding: Re y += Re T Re x - Im T Im x, Im y += Re T Im x + Im T Re x.
// Lags < 0 (s > n) and sources outside [s_lo, s_hi) enter as zeros.
// Operand layout of the instruction (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; accumulator register q of lane l is D[l/16+4q][l%16]
// (checked on the device against a host product).
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// With one 256-step target tile and a source range of at most 256 steps (the
// causal solve's history products), the workgroup first stages the sources
// and the coefficient window they meet (at most 511 lags) in LDS with
// coalesced loads by all four waves, so the lag-block loop reads its operands
// from LDS instead of waiting on memory every block.  The four waves then
// share the tile: wave w takes k-slice w (sources 4w .. 4w+3 of every
// 16-step source block) of every lag block, with one accumulator pair per
// side (four independent MFMA chains), and the partial sums are added in a
// fixed order (sides, then waves).  For a given output the terms and their
// order do not depend on the output range of the call, so splitting a range
// changes no result bit; the rounding differs from the one-wave form used
// for longer ranges by the order of the sum.
constexpr int kLttStage = 256;

// staged sources: entry e at e + e / 16, so the 16 B-operand lanes of one
// instruction (sources 16 apart) fall in different LDS banks
__device__ inline int ltt_xpad(int e) { return e + (e >> 4); }

__global__ __launch_bounds__(256) void ltt_mfma_kernel(LttArgs a) {
    __shared__ cd st_x[2][kLttStage + kLttStage / 16], st_c[2][2 * kLttStage];
    __shared__ d4 red[4][2][kWave];               // staged form: the waves' accumulators
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int tile = blockIdx.x * 4 + w;
    const int o = blockIdx.y;
    const int b = a.s_seg > 0 ? blockIdx.z % a.B : blockIdx.z;
    const int seg = a.s_seg > 0 ? blockIdx.z / a.B : 0;
    const int nlen = a.n_hi - a.n_lo;
    const int s_lo0 = a.s_seg > 0 ? a.s_lo + seg * a.s_seg : a.s_lo;
    const int s_hi0 = a.s_seg > 0 ? min(a.s_hi, s_lo0 + a.s_seg) : a.s_hi;
    const bool staged = nlen <= kLttStage && s_hi0 - s_lo0 <= kLttStage;   // uniform per workgroup
    if (!staged && tile * 256 >= nlen) return;       // whole wave leaves together
    const int s_lo = s_lo0;
    const int s_hi = s_hi0;
    int k, pl, pr, sl, sr;
    slot_sources(o, a.N, k, pl, pr, sl, sr);
    const int v = a.per_problem ? b : 0;
    const cd* cl = a.cols + ((size_t)(v * a.N + k) * 4 + pl) * a.nt;
    const cd* cr = a.cols + ((size_t)(v * a.N + k) * 4 + pr) * a.nt;
    const cd* xl = sl >= 0 ? a.x + ((size_t)b * a.ns + sl) * a.nt + s_lo : nullptr;
    const cd* xr = sr >= 0 ? a.x + ((size_t)b * a.ns + sr) * a.nt + s_lo : nullptr;
    // staged form: sources s_lo + [0, slen) and lags lag0 + [0, nlen + slen - 1)
    const int lag0 = a.n_lo - s_hi + 1;
    if (staged) {
        const int slen0 = s_hi - s_lo, nlag = nlen + slen0 - 1;
        for (int e = threadIdx.x; e < kLttStage; e += blockDim.x) {
            cd x0 = mk(0, 0), x1 = mk(0, 0);
            if (xl && e < slen0) x0 = xl[e];
            if (xr && e < slen0) x1 = xr[e];
            st_x[0][ltt_xpad(e)] = x0;
            st_x[1][ltt_xpad(e)] = x1;
        }
        for (int e = threadIdx.x; e < 2 * kLttStage; e += blockDim.x) {
            const int lag = lag0 + e;
            const bool ok = e < nlag && lag >= 0 && lag < a.nt;
            cd c0 = mk(0, 0), c1 = mk(0, 0);
            if (xl && ok) c0 = cl[lag];
            if (xr && ok) c1 = cr[lag];
            st_c[0][e] = c0;
            st_c[1][e] = c1;
        }
        __syncthreads();
    }
    const int r = lane & 15, kq = lane >> 4;
    const int I0 = staged ? 0 : tile * 16;
    const int slen = s_hi - s_lo;
    const int Jn = (slen + 15) / 16;
    const int delta = a.n_lo - s_lo;
    // lag blocks that can meet a source block J in [0, Jn) and a lag >= 0
    const int q = -delta - 15;
    const int m_lag = q >= 0 ? (q + 15) / 16 : -((-q) / 16);
    const int m_lo = max(I0 - (Jn - 1), m_lag);
    const int m_hi = slen > 0 ? I0 + 15 : m_lo - 1;
    d4 yr = {0, 0, 0, 0}, yi = {0, 0, 0, 0};
    // the lag-block loop of the one-wave form, operands from memory
    auto blocks = [&](auto opA, auto opB) {
        for (int m = m_lo; m <= m_hi; ++m) {
            const int J = I0 + r - m;               // source block of B column r
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                const int kk = 4 * kc + kq;
                const int lag = delta + 16 * m + r - kk;
                const int si = 16 * J + kk;
                const bool sok = J >= 0 && si < slen;
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    if (side == 0 ? !xl : !xr) continue;
                    const cd av = opA(side, lag);
                    cd bv = mk(0, 0);
                    if (sok) bv = opB(side, si);
                    yr = mfma16(av.x, bv.x, yr);
                    yr = mfma16(-av.y, bv.y, yr);
                    yi = mfma16(av.x, bv.y, yi);
                    yi = mfma16(av.y, bv.x, yi);
                }
            }
        }
    };
    if (staged) {
        // a lag outside the window pairs only with sources outside [0, slen)
        // or outputs past nlen, i.e. with a zero operand or a dropped result
        const int kk = 4 * w + kq;
        d4 ar0 = {0, 0, 0, 0}, ai0 = {0, 0, 0, 0}, ar1 = {0, 0, 0, 0}, ai1 = {0, 0, 0, 0};
        for (int m = m_lo; m <= m_hi; ++m) {
            const int J = I0 + r - m;               // source block of B column r
            const int le = delta + 16 * m + r - kk - lag0;
            const int si = 16 * J + kk;
            const bool sok = J >= 0 && si < slen;
            const bool lok = le >= 0 && le < 2 * kLttStage;
            if (xl) {
                cd av = mk(0, 0), bv = mk(0, 0);
                if (lok) av = st_c[0][le];
                if (sok) bv = st_x[0][ltt_xpad(si)];
                ar0 = mfma16(av.x, bv.x, ar0);
                ar0 = mfma16(-av.y, bv.y, ar0);
                ai0 = mfma16(av.x, bv.y, ai0);
                ai0 = mfma16(av.y, bv.x, ai0);
            }
            if (xr) {
                cd av = mk(0, 0), bv = mk(0, 0);
                if (lok) av = st_c[1][le];
                if (sok) bv = st_x[1][ltt_xpad(si)];
                ar1 = mfma16(av.x, bv.x, ar1);
                ar1 = mfma16(-av.y, bv.y, ar1);
                ai1 = mfma16(av.x, bv.y, ai1);
                ai1 = mfma16(av.y, bv.x, ai1);
            }
        }
        red[w][0][lane] = ar0 + ar1;
        red[w][1][lane] = ai0 + ai1;
        __syncthreads();
        if (w != 0) return;
        yr = red[0][0][lane];
        yi = red[0][1][lane];
#pragma unroll
        for (int u = 1; u < 4; ++u) {
            yr = yr + red[u][0][lane];
            yi = yi + red[u][1][lane];
        }
    } else {
        blocks([&](int side, int lag) {
                   cd c = mk(0, 0);
                   if (lag >= 0 && lag < a.nt) c = (side ? cr : cl)[lag];
                   return c;
               },
               [&](int side, int si) { return (side ? xr : xl)[si]; });
    }
    const size_t yb = ((size_t)b * a.ns + o) * a.y_ld + (size_t)seg * a.y_seg_stride;
    const cd* base = a.s_seg > 0 ? nullptr : a.base;
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const int nrel = 16 * (I0 + r) + kq + 4 * qq;
        if (nrel < nlen) {
            cd out = mk(a.sign * yr[qq], a.sign * yi[qq]);
            if (base) out = out + base[yb + nrel];
            a.y[yb + nrel] = out;
        }
    }
}

// ---------------------------------------------------------------------------
// Batched form of the staged product (at most 256 outputs and 256 sources per
// segment, one potential for the whole batch): the problems of the batch,
// which share every coefficient, fill the instruction's N dimension instead
// of the output blocks.  A workgroup takes one slot, one segment and eight
// problems; the columns are (problem, real / imaginary part of x), and two
// accumulators per 16-output block collect Re T [Re x | Im x] and
// Im T [Re x | Im x], combined at the end (Re y = Re T Re x - Im T Im x, Im y
// = Re T Im x + Im T Re x) between neighbouring lanes.  Every (output block,
// source block) pair does useful work, where the one-problem form's columns
// (output blocks) meet a lag block's sources only partly (about half of its
// products are zero operands on a 256 x 256 tile).  The workgroup stages the
// sources of its eight problems (2 sides x 256 x 16 doubles) and the
// coefficient window (2 x 512) in LDS (80 KiB); wave w takes the output blocks
// 4w .. 4w+3.  The sources sit at the end of their 16-aligned block (zeros
// first), so the lag index of every (output, source) pair of the tiles lies in
// [0, 511) and each A operand is one LDS read at a constant offset from a
// per-lane base, with no range test in the product loop.  Sum order: source blocks ascending, k-slices ascending, the
// two sides, per output; it differs from the one-problem form's, so a batch
// of eight or more problems and the same problem alone agree to rounding.
// ---------------------------------------------------------------------------
constexpr int kLttBatch = 8;      // problems per workgroup of the batched form
static_assert(2 * kLttBatch == 16, "the 16 columns of a tile are 8 problems x (re, im)");
constexpr int kLttScLen = 2 * kLttStage;   // coefficient window per side

__device__ inline double swap_pair(double v) {   // the value of lane l ^ 1
    int2 t = *reinterpret_cast<int2*>(&v);
    t.x = __builtin_amdgcn_mov_dpp(t.x, 0xB1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
    t.y = __builtin_amdgcn_mov_dpp(t.y, 0xB1, 0xf, 0xf, false);
    return *reinterpret_cast<double*>(&t);
}

__global__ __launch_bounds__(256) void ltt_batch_kernel(LttArgs a) {
    extern __shared__ double lds[];
    double* sx = lds;                                            // [2][256][16]
    cd* sc = reinterpret_cast<cd*>(lds + 2 * kLttStage * 16);    // [2][kLttScLen]
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int r = lane & 15, kq = lane >> 4;
    const int o = blockIdx.x, b0 = blockIdx.y * kLttBatch, seg = blockIdx.z;
    const int nlen = a.n_hi - a.n_lo;
    const int s_lo = a.s_seg > 0 ? a.s_lo + seg * a.s_seg : a.s_lo;
    const int s_hi = a.s_seg > 0 ? min(a.s_hi, s_lo + a.s_seg) : a.s_hi;
    const int slen = s_hi - s_lo;
    int k, pl, pr, sl, sr;
    slot_sources(o, a.N, k, pl, pr, sl, sr);
    const cd* cl = a.cols + ((size_t)k * 4 + pl) * a.nt;
    const cd* cr = a.cols + ((size_t)k * 4 + pr) * a.nt;
    // sources: position p of a side holds source p - pad0 of the eight
    // problems (positions below pad0 zero) as 8 complex values in a row; item
    // u = (side, p, bb) goes to thread u mod 256, so a wave writes one
    // contiguous 1 KiB span of LDS
    const int Jn = (slen + 15) / 16, pad0 = 16 * Jn - slen;
    {
        cd* sxc = reinterpret_cast<cd*>(sx);
        const int bb = tid & (kLttBatch - 1), b = b0 + bb;
#pragma unroll
        for (int it = 0; it < 2 * kLttStage * kLttBatch / 256; ++it) {
            const int u = it * 256 + tid, side = u / (kLttStage * kLttBatch);
            const int pos = (u / kLttBatch) % kLttStage, src = pos - pad0;
            const int srow = side ? sr : sl;
            cd x = mk(0, 0);
            if (srow >= 0 && b < a.B && src >= 0 && src < slen) x = a.x[((size_t)b * a.ns + srow) * a.nt + s_lo + src];
            sxc[u] = x;
        }
    }
    // coefficients: lags lag0 + e, e < nlen + slen - 1
    const int lag0 = a.n_lo - s_hi + 1, nlag = nlen + slen - 1;
    for (int e = tid; e < kLttScLen; e += blockDim.x) {
        const int lag = lag0 + e;
        const bool ok = e < nlag && lag >= 0 && lag < a.nt;
        sc[e] = (ok && sl >= 0) ? cl[lag] : mk(0, 0);
        sc[kLttScLen + e] = (ok && sr >= 0) ? cr[lag] : mk(0, 0);
    }
    __syncthreads();
    // a wave whose four output blocks all lie past the call's range (a short
    // last piece of the solve) has nothing to write; no barrier follows
    if (64 * w >= nlen) return;
    d4 d1[4], d2[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        d1[i] = d4{0.0, 0.0, 0.0, 0.0};
        d2[i] = d4{0.0, 0.0, 0.0, 0.0};
    }
    // per-lane bases: B[kq][col r] = position 16 J + 4 ks + kq of column r;
    // A[row r][kq] = lag index e = 16 (I - J) + r - (4 ks + kq) + 16 Jn - 1,
    // in [0, 16 Jn + 255) for every output row and position
    const double* bx = sx + kq * 16 + r;
    const cd* ac = sc + 64 * w + r - kq + 16 * Jn - 1;
    for (int J = 0; J < Jn; ++J) {
        const double* bxj = bx + 16 * 16 * J;
        const cd* acj = ac - 16 * J;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                // a side without a neighbour has zero sources and
                // coefficients: no branch here, which would move the
                // accumulators out of the matrix registers around it
                const double bv = bxj[(side * kLttStage + 4 * ks) * 16];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const cd av = acj[side * kLttScLen + 16 * i - 4 * ks];
                    d1[i] = mfma16(av.x, bv, d1[i]);
                    d2[i] = mfma16(av.y, bv, d2[i]);
                }
            }
        }
    }
    // lane with column r = 2 bb + part: part 0 gives Re y = Re T Re x - Im T Im x
    // (d1 here, d2 of the odd neighbour), part 1 Im y = Re T Im x + Im T Re x
    const int bb = r >> 1, part = r & 1;
    const int b = b0 + bb;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double other = swap_pair(d2[i][q]);
            const double v = part ? d1[i][q] + other : d1[i][q] - other;
            const int nrel = 16 * (4 * w + i) + kq + 4 * q;
            if (b < a.B && nrel < nlen) {
                const size_t yb = ((size_t)b * a.ns + o) * a.y_ld + (size_t)seg * a.y_seg_stride;
                double* y = reinterpret_cast<double*>(a.y + yb + nrel) + part;
                double val = a.sign * v;
                if (a.s_seg <= 0 && a.base) val += reinterpret_cast<const double*>(a.base + yb + nrel)[part];
                *y = val;
            }
        }
    }
}

hipError_t launch_ltt(const LttArgs& a, hipStream_t st) {
    if (a.ns == 0 || a.n_hi <= a.n_lo) return hipSuccess;
    if (a.s_lo < 0 || a.s_hi > a.nt || a.n_lo < 0 || a.n_hi > a.nt) return hipErrorInvalidValue;
    const int tiles = (a.n_hi - a.n_lo + 255) / 256;
    const int nseg = a.s_seg > 0 ? (a.s_hi - a.s_lo + a.s_seg - 1) / a.s_seg : 1;
    if ((size_t)a.B * nseg > 65535) return hipErrorInvalidValue;
    const int slen_max = a.s_seg > 0 ? std::min(a.s_seg, a.s_hi - a.s_lo) : a.s_hi - a.s_lo;
    if (a.B >= kLttBatch && !a.per_problem && a.n_hi - a.n_lo <= kLttStage && slen_max <= kLttStage) {
        const size_t lds = sizeof(double) * 2 * kLttStage * 16 + sizeof(cd) * 2 * kLttScLen;
        dim3 grid(a.ns, (a.B + kLttBatch - 1) / kLttBatch, nseg);
        ltt_batch_kernel<<<grid, 256, lds, st>>>(a);
        return hipGetLastError();
    }
    dim3 grid((tiles + 3) / 4, a.ns, a.B * nseg);
    ltt_mfma_kernel<<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched vector kernels for GMRES.  Vectors are [B][M] complex; the Krylov
// basis is V[i] = basis + i * B * M.  Reductions are two-stage and
// deterministic: per-block partials, then one reduction kernel.
// ---------------------------------------------------------------------------

__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) r += sh[i];
    __syncthreads();
    return r;
}

// partial[b][blk][i] = sum over the block's range of conj(V_i) w,  i < nv
__global__ __launch_bounds__(kRedThreads) void multidot_kernel(const cd* basis, int nv, const cd* w,
                                                              long M, int B, double* partial) {
    __shared__ double sh[8];
    const int b = blockIdx.y;
    const long per = (M + gridDim.x - 1) / gridDim.x;
    const long lo = blockIdx.x * per, hi = min(M, lo + per);
    const cd* wb = w + (size_t)b * M;
    for (int i = 0; i < nv; ++i) {
        const cd* vb = basis + ((size_t)i * B + b) * M;
        double sx = 0, sy = 0;
        for (long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
            const cd p = vb[e], q = wb[e];
            sx += p.x * q.x + p.y * q.y;
            sy += p.x * q.y - p.y * q.x;
        }
        const double tx = block_sum(sx, sh);
        const double ty = block_sum(sy, sh);
        if (threadIdx.x == 0) {
            double* pp = partial + (((size_t)b * gridDim.x + blockIdx.x) * nv + i) * 2;
            pp[0] = tx;
            pp[1] = ty;
        }
    }
}

// out[b][i] (+)= sum over blocks of partial[b][blk][i]
__global__ void reduce_partials_kernel(const double* partial, int nblk, int nv, int B, cd* out,
                                       int out_ld, int accumulate) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * nv) return;
    const int b = idx / nv, i = idx % nv;
    double sx = 0, sy = 0;
    for (int k = 0; k < nblk; ++k) {
        const double* pp = partial + (((size_t)b * nblk + k) * nv + i) * 2;
        sx += pp[0];
        sy += pp[1];
    }
    cd r = mk(sx, sy);
    cd* o = out + (size_t)b * out_ld + i;
    if (accumulate) r = r + *o;
    *o = r;
}

// w[b] += sign * sum_{i<nv} coef[b][i] V_i[b]
__global__ __launch_bounds__(256) void multiaxpy_kernel(const cd* basis, int nv, const cd* coef,
                                                        int coef_ld, double sign, cd* w, long M,
                                                        int B) {
    const int b = blockIdx.y;
    const cd* cb = coef + (size_t)b * coef_ld;
    cd* wb = w + (size_t)b * M;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < M; e += (long)gridDim.x * blockDim.x) {
        cd acc = wb[e];
        for (int i = 0; i < nv; ++i) {
            const cd c = sign * cb[i];
            acc = madd(acc, c, basis[((size_t)i * B + b) * M + e]);
        }
        wb[e] = acc;
    }
}

// partial[b][blk] = sum |w|^2 over the block's range
__global__ __launch_bounds__(kRedThreads) void norm2_kernel(const cd* w, long M, double* partial) {
    __shared__ double sh[8];
    const int b = blockIdx.y;
    const long per = (M + gridDim.x - 1) / gridDim.x;
    const long lo = blockIdx.x * per, hi = min(M, lo + per);
    const cd* wb = w + (size_t)b * M;
    double s = 0;
    for (long e = lo + threadIdx.x; e < hi; e += blockDim.x) s += abs2(wb[e]);
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) partial[(size_t)b * gridDim.x + blockIdx.x] = t;
}

// partial[b][blk] = max |w| over the block's range
__global__ __launch_bounds__(kRedThreads) void maxabs_kernel(const cd* w, long M, double* partial) {
    __shared__ double sh[8];
    const int b = blockIdx.y;
    const long per = (M + gridDim.x - 1) / gridDim.x;
    const long lo = blockIdx.x * per, hi = min(M, lo + per);
    const cd* wb = w + (size_t)b * M;
    double m = 0;
    for (long e = lo + threadIdx.x; e < hi; e += blockDim.x) m = fmax(m, abs2(wb[e]));
    m = wave_max(m);
    const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) sh[wv] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) r = fmax(r, sh[i]);
        partial[(size_t)b * gridDim.x + blockIdx.x] = r;
    }
}

__global__ void reduce_max_kernel(const double* partial, int nblk, int B, double* out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double m = 0;
    for (int k = 0; k < nblk; ++k) m = fmax(m, partial[(size_t)b * nblk + k]);
    out[b] = sqrt(m);
}

// nrm[b] = sqrt(sum partial[b][:])
__global__ void reduce_norm_kernel(const double* partial, int nblk, int B, double* nrm) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double s = 0;
    for (int k = 0; k < nblk; ++k) s += partial[(size_t)b * nblk + k];
    nrm[b] = sqrt(s);
}

// dst[b] = src[b] * (1 / den[b]) (den == 0 -> zero)
__global__ __launch_bounds__(256) void scale_kernel(const cd* src, const double* den, cd* dst, long M,
                                                    int B, const int* active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    const double s = den[b] != 0.0 ? 1.0 / den[b] : 0.0;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < M; e += (long)gridDim.x * blockDim.x)
        dst[(size_t)b * M + e] = s * src[(size_t)b * M + e];
}

// Arnoldi column j of problem b: H[b] (m+1) x m column-major in hcol, Givens
// rotations cs/sn, residual vector e.  hcol[b][0..j] holds the projections,
// hnext[b] = ||w||.  Writes the residual estimate |e_{j+1}| / bnorm.
__global__ void givens_kernel(int j, int m, int B, const cd* hproj, const double* hnext, cd* H,
                              cd* cs, cd* sn, cd* e, const double* bnorm, double* resid,
                              int* active) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B || !active[b]) return;
    cd* Hb = H + (size_t)b * (m + 1) * m;
    cd* col = Hb + (size_t)j * (m + 1);
    for (int i = 0; i <= j; ++i) col[i] = hproj[(size_t)b * (m + 1) + i];
    col[j + 1] = mk(hnext[b], 0);
    cd* c = cs + (size_t)b * m;
    cd* s = sn + (size_t)b * m;
    cd* eb = e + (size_t)b * (m + 1);
    // earlier rotations [[conj c, conj s], [-s, c]] (unitary; the same map
    // that annihilated their own subdiagonal entries and updated e)
    for (int i = 0; i < j; ++i) {
        const cd t = conjc(c[i]) * col[i] + conjc(s[i]) * col[i + 1];
        col[i + 1] = c[i] * col[i + 1] - s[i] * col[i];
        col[i] = t;
    }
    const double den = sqrt(abs2(col[j]) + abs2(col[j + 1]));
    cd cj = mk(1, 0), sj = mk(0, 0);
    if (den > 0) { cj = (1.0 / den) * col[j]; sj = (1.0 / den) * col[j + 1]; }
    c[j] = cj;
    s[j] = sj;
    col[j] = conjc(cj) * col[j] + conjc(sj) * col[j + 1];
    col[j + 1] = mk(0, 0);
    eb[j + 1] = -(sj * eb[j]);
    eb[j] = conjc(cj) * eb[j];
    resid[b] = sqrt(abs2(eb[j + 1])) / bnorm[b];
}

// Back substitution H y = e on the leading jj x jj block; y stored in ycoef.
__global__ void gmres_solve_kernel(int jj, int m, int B, const cd* H, const cd* e, cd* y,
                                   const int* active) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    cd* yb = y + (size_t)b * (m + 1);
    if (!active[b]) {
        for (int i = 0; i <= m; ++i) yb[i] = mk(0, 0);
        return;
    }
    const cd* Hb = H + (size_t)b * (m + 1) * m;
    const cd* eb = e + (size_t)b * (m + 1);
    for (int i = jj - 1; i >= 0; --i) {
        cd r = eb[i];
        for (int q = i + 1; q < jj; ++q) r = msub(r, Hb[(size_t)q * (m + 1) + i], yb[q]);
        yb[i] = r * inv(Hb[(size_t)i * (m + 1) + i]);
    }
    for (int i = jj; i <= m; ++i) yb[i] = mk(0, 0);
}

// e[b] = (beta_b, 0, ...), cycle initialisation
__global__ void gmres_init_kernel(int m, int B, const double* beta, cd* e, int* active,
                                  const double* bnorm, double tol, double* resid) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    cd* eb = e + (size_t)b * (m + 1);
    for (int i = 0; i <= m; ++i) eb[i] = mk(0, 0);
    eb[0] = mk(beta[b], 0);
    resid[b] = bnorm[b] > 0 ? beta[b] / bnorm[b] : 0.0;
    active[b] = (bnorm[b] > 0 && beta[b] > tol * bnorm[b]) ? 1 : 0;
}

// z_b = c0_b x0_b + c1_b x1_b + c2_b x2_b with complex per-problem
// coefficients coef[b][0..2]; a null x_k is skipped; z may alias any x_k
__global__ __launch_bounds__(256) void lincomb_kernel(const cd* x0, const cd* x1, const cd* x2,
                                                      const cd* coef, cd* z, long M) {
    const int b = blockIdx.y;
    const cd c0 = coef[3 * b], c1 = coef[3 * b + 1], c2 = coef[3 * b + 2];
    const size_t o = (size_t)b * M;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < M; e += (long)gridDim.x * blockDim.x) {
        cd acc = mk(0, 0);
        if (x0) acc = madd(acc, c0, x0[o + e]);
        if (x1) acc = madd(acc, c1, x1[o + e]);
        if (x2) acc = madd(acc, c2, x2[o + e]);
        z[o + e] = acc;
    }
}

hipError_t launch_lincomb(const cd* x0, const cd* x1, const cd* x2, const cd* coef, cd* z, long M,
                          int B, hipStream_t st) {
    const int blocks = (int)std::min<long>(1024, (M + 255) / 256);
    lincomb_kernel<<<dim3(blocks, B), 256, 0, st>>>(x0, x1, x2, coef, z, M);
    return hipGetLastError();
}

hipError_t launch_multidot(const cd* basis, int nv, const cd* w, long M, int B, double* partial,
                           cd* out, int out_ld, int accumulate, hipStream_t st) {
    multidot_kernel<<<dim3(kRedBlocks, B), kRedThreads, 0, st>>>(basis, nv, w, M, B, partial);
    reduce_partials_kernel<<<(B * nv + 127) / 128, 128, 0, st>>>(partial, kRedBlocks, nv, B, out,
                                                                  out_ld, accumulate);
    return hipGetLastError();
}
hipError_t launch_multiaxpy(const cd* basis, int nv, const cd* coef, int coef_ld, double sign,
                            cd* w, long M, int B, hipStream_t st) {
    const int blocks = (int)std::min<long>(1024, (M + 255) / 256);
    multiaxpy_kernel<<<dim3(blocks, B), 256, 0, st>>>(basis, nv, coef, coef_ld, sign, w, M, B);
    return hipGetLastError();
}
hipError_t launch_norm(const cd* w, long M, int B, double* partial, double* nrm, hipStream_t st) {
    norm2_kernel<<<dim3(kRedBlocks, B), kRedThreads, 0, st>>>(w, M, partial);
    reduce_norm_kernel<<<(B + 63) / 64, 64, 0, st>>>(partial, kRedBlocks, B, nrm);
    return hipGetLastError();
}
hipError_t launch_maxabs(const cd* x, long M, int B, double* partial, double* out, hipStream_t st) {
    maxabs_kernel<<<dim3(kRedBlocks, B), kRedThreads, 0, st>>>(x, M, partial);
    reduce_max_kernel<<<(B + 63) / 64, 64, 0, st>>>(partial, kRedBlocks, B, out);
    return hipGetLastError();
}
hipError_t launch_scale(const cd* src, const double* den, cd* dst, long M, int B, const int* active,
                        hipStream_t st) {
    const int blocks = (int)std::min<long>(1024, (M + 255) / 256);
    scale_kernel<<<dim3(blocks, B), 256, 0, st>>>(src, den, dst, M, B, active);
    return hipGetLastError();
}
hipError_t launch_givens(int j, int m, int B, const cd* hproj, const double* hnext, cd* H, cd* cs,
                         cd* sn, cd* e, const double* bnorm, double* resid, int* active,
                         hipStream_t st) {
    givens_kernel<<<(B + 63) / 64, 64, 0, st>>>(j, m, B, hproj, hnext, H, cs, sn, e, bnorm, resid,
                                                active);
    return hipGetLastError();
}
hipError_t launch_gmres_solve(int jj, int m, int B, const cd* H, const cd* e, cd* y,
                              const int* active, hipStream_t st) {
    gmres_solve_kernel<<<(B + 63) / 64, 64, 0, st>>>(jj, m, B, H, e, y, active);
    return hipGetLastError();
}
hipError_t launch_gmres_init(int m, int B, const double* beta, cd* e, int* active,
                             const double* bnorm, double tol, double* resid, hipStream_t st) {
    gmres_init_kernel<<<(B + 63) / 64, 64, 0, st>>>(m, B, beta, e, active, bnorm, tol, resid);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Causal forward substitution for (I - L) g = d.
// Every block of L is lower triangular in time (Props. 3-4), so with C_m the
// ns x ns matrix of m-th Toeplitz coefficients, step n reads
//   (I - C_0) g_n = d_n + sum_{s<n} C_{n-s} g_s.
// (I - C_0)^{-1} is formed once (Gauss-Jordan, partial pivoting); time is
// processed in blocks of kCausalTb steps: the contribution of all earlier
// blocks comes from the LTT apply kernel, the in-block part is summed here.
// ---------------------------------------------------------------------------
// C0 assembly: M = I - C_0 for potential v, row-major ns x ns.
__global__ void c0_assemble_kernel(int N, int ns, int nt, const cd* cols, cd* Mat) {
    const int v = blockIdx.y;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ns * ns) return;
    const int o = idx / ns, in = idx % ns;
    int k, pl, pr, sl, sr;
    slot_sources(o, N, k, pl, pr, sl, sr);
    cd val = mk(o == in ? 1.0 : 0.0, 0);
    const cd* base = cols + (size_t)(v * N + k) * 4 * nt;
    if (in == sl) val = val - base[(size_t)pl * nt];
    if (in == sr) val = val - base[(size_t)pr * nt];
    Mat[(size_t)v * ns * ns + idx] = val;
}

// In-place Gauss-Jordan inverse with partial pivoting, one workgroup per
// potential.  A: [ns][ns] row-major (destroyed), Ainv: [ns][ns].
__global__ __launch_bounds__(256) void gauss_jordan_kernel(int ns, cd* A, cd* Ainv, int* piv_ok) {
    const int v = blockIdx.x;
    cd* a = A + (size_t)v * ns * ns;
    cd* x = Ainv + (size_t)v * ns * ns;
    __shared__ int s_piv;
    __shared__ double s_val[256];
    __shared__ int s_idx[256];
    for (int i = threadIdx.x; i < ns * ns; i += blockDim.x) x[i] = mk((i / ns) == (i % ns) ? 1 : 0, 0);
    __syncthreads();
    for (int c = 0; c < ns; ++c) {
        double best = -1;
        int bi = c;
        for (int r = c + threadIdx.x; r < ns; r += blockDim.x) {
            const double m2 = abs2(a[(size_t)r * ns + c]);
            if (m2 > best) { best = m2; bi = r; }
        }
        s_val[threadIdx.x] = best;
        s_idx[threadIdx.x] = bi;
        __syncthreads();
        if (threadIdx.x == 0) {
            double bb = -1;
            int ii = c;
            for (int q = 0; q < (int)blockDim.x; ++q)
                if (s_val[q] > bb) { bb = s_val[q]; ii = s_idx[q]; }
            s_piv = ii;
            if (bb <= 0) piv_ok[v] = 0;
        }
        __syncthreads();
        const int p = s_piv;
        if (p != c) {
            for (int q = threadIdx.x; q < ns; q += blockDim.x) {
                cd t = a[(size_t)c * ns + q]; a[(size_t)c * ns + q] = a[(size_t)p * ns + q]; a[(size_t)p * ns + q] = t;
                t = x[(size_t)c * ns + q]; x[(size_t)c * ns + q] = x[(size_t)p * ns + q]; x[(size_t)p * ns + q] = t;
            }
        }
        __syncthreads();
        const cd pinv = inv(a[(size_t)c * ns + c]);
        __syncthreads();
        for (int q = threadIdx.x; q < ns; q += blockDim.x) {
            a[(size_t)c * ns + q] = pinv * a[(size_t)c * ns + q];
            x[(size_t)c * ns + q] = pinv * x[(size_t)c * ns + q];
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < ns * ns; idx += blockDim.x) {
            const int r = idx / ns, q = idx % ns;
            if (r == c) continue;
            const cd f = a[(size_t)r * ns + c];
            if (q == c) continue;
            a[(size_t)r * ns + q] = msub(a[(size_t)r * ns + q], f, a[(size_t)c * ns + q]);
            x[(size_t)r * ns + q] = msub(x[(size_t)r * ns + q], f, x[(size_t)c * ns + q]);
        }
        __syncthreads();
        for (int r = threadIdx.x; r < ns; r += blockDim.x) {
            if (r == c) continue;
            const cd f = a[(size_t)r * ns + c];
            x[(size_t)r * ns + c] = msub(x[(size_t)r * ns + c], f, x[(size_t)c * ns + c]);
            a[(size_t)r * ns + c] = mk(0, 0);
        }
        __syncthreads();
    }
}


__global__ __launch_bounds__(256) void causal_block_kernel(CausalArgs a) {
    extern __shared__ cd s_rhs[];
    const int b = blockIdx.x;
    const int v = a.per_problem ? b : 0;
    const cd* Mi = a.Minv + (size_t)v * a.ns * a.ns;
    cd* gb = a.g + (size_t)b * a.ns * a.nt;
    for (int i = 0; i < a.nb; ++i) {
        const int n = a.n0 + i;
        for (int o = threadIdx.x; o < a.ns; o += blockDim.x) {
            int k, pl, pr, sl, sr;
            slot_sources(o, a.N, k, pl, pr, sl, sr);
            const cd* base = a.cols + (size_t)(v * a.N + k) * 4 * a.nt;
            cd r = a.d[((size_t)b * a.ns + o) * a.nt + n] + a.far[((size_t)b * a.ns + o) * kCausalTb + i];
            for (int s = a.n0; s < n; ++s) {
                if (sl >= 0) r = madd(r, base[(size_t)pl * a.nt + (n - s)], gb[(size_t)sl * a.nt + s]);
                if (sr >= 0) r = madd(r, base[(size_t)pr * a.nt + (n - s)], gb[(size_t)sr * a.nt + s]);
            }
            s_rhs[o] = r;
        }
        __syncthreads();
        for (int o = threadIdx.x; o < a.ns; o += blockDim.x) {
            cd r = mk(0, 0);
            const cd* row = Mi + (size_t)o * a.ns;
            for (int q = 0; q < a.ns; ++q) r = madd(r, row[q], s_rhs[q]);
            gb[(size_t)o * a.nt + n] = r;
        }
        __threadfence_block();
        __syncthreads();
    }
}

// z = a x + b y (elementwise, complex vectors of n entries; z may alias x or y)
__global__ __launch_bounds__(256) void axpby_kernel(const cd* x, double a, const cd* y, double b,
                                                    cd* z, long n) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
        z[e] = a * x[e] + b * y[e];
}
hipError_t launch_axpby(const cd* x, double a, const cd* y, double b, cd* z, long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>(2048, (n + 255) / 256);
    axpby_kernel<<<blocks, 256, 0, st>>>(x, a, y, b, z, n);
    return hipGetLastError();
}

hipError_t launch_c0_inverse(int N, int ns, int nt, int nv, const cd* cols, cd* work, cd* Minv,
                             int* piv_ok, hipStream_t st) {
    if (ns == 0) return hipSuccess;
    c0_assemble_kernel<<<dim3((ns * ns + 255) / 256, nv), 256, 0, st>>>(N, ns, nt, cols, work);
    gauss_jordan_kernel<<<nv, 256, 0, st>>>(ns, work, Minv, piv_ok);
    return hipGetLastError();
}

hipError_t launch_causal_block(const CausalArgs& a, hipStream_t st) {
    causal_block_kernel<<<a.B, 256, a.ns * sizeof(cd), st>>>(a);
    return hipGetLastError();
}

}  // namespace swr
