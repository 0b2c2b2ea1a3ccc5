/*
 * swr_oracle.c -- plain, slow, single-threaded CPU reference ("oracle") for the
 * Schwarz waveform relaxation (SWR) method of Besse & Xing, "Schwarz waveform
 * relaxation method for one dimensional Schroedinger equation with general
 * potential" (arXiv 1503.02564).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path.
 *
 * Everything is IEEE FP64 complex (C99 `double complex`).  No blocking, no
 * fusion, no reordering beyond what the paper's definitions state.
 *
 * Notation (paper Sec. 2.2):
 *   c      = 2i/dt                               (eq. CNS_L)
 *   A      = c M - S + M_W   (P1 mass, stiffness, generalised mass; eq. AvML)
 *   v_n    = (u_n + u_{n-1})/2,   u_n = 2 v_n - u_{n-1}            (eq. CNS_L)
 *   W_n    = (V_n + V_{n-1})/2                                     (eq. CNS_L)
 *   S0^2 : Sbar v_n = c2 sum_{s=0}^{n} beta_{n-s} v_s, c2 = e^{-i pi/4} sqrt(2/dt)
 *   S0^3 : adds - e^{i pi/4} sqrt(dt/2) (W_n/2) sum_{s=0}^{n} alpha_{n-s} v_s
 *   S0^4 : adds - i (dn W_n / 4) (dt/2) sum_{s=0}^{n} gamma_{n-s} v_s
 *   S1^2 : Sbar v_n = c2 e^{i calW_n} sum_{s=0}^{n} beta_{n-s} e^{-i calW_s} v_s
 *   S1^4 : adds - i sgn(dn W_n) q_n e^{i calW_n} (dt/2) sum gamma_{n-s} q_s e^{-i calW_s} v_s,
 *          q_n = sqrt(|dn W_n|)/2
 *   Robin: Sbar v_n = sigma v_n (the caller passes the complex sigma of dn + sigma)
 *   S2^{2,m}, S2^{4,m} (Pade strategy): Sbar v_n from m auxiliary functions
 *          phi^s (and psi for order 4), see orc_pade_coef / pade_parts
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Convolution weights of the potential strategy (Sec. 2.2, "Potential       */
/* strategy l=0"): alpha_0 = alpha_1 = 1, alpha_{2m} = alpha_{2m+1} =         */
/* (2m-1)!!/(2m)!!, beta_s = (-1)^s alpha_s, gamma = (1,2,2,2,...).           */
/* ------------------------------------------------------------------------ */
void orc_alpha(int n, double *alpha)
{
    for (int s = 0; s < n; ++s) {
        int m = s / 2;               /* alpha_{2m} = alpha_{2m+1} */
        double a = 1.0;              /* (2m-1)!!/(2m)!! as a running product */
        for (int q = 1; q <= m; ++q) a *= (2.0 * q - 1.0) / (2.0 * q);
        alpha[s] = a;
    }
}

void orc_beta(int n, double *beta)
{
    orc_alpha(n, beta);
    for (int s = 1; s < n; s += 2) beta[s] = -beta[s];
}

/* ------------------------------------------------------------------------ */
/* P1 finite elements on a uniform mesh of n nodes, spacing h (Sec. 2.2:      */
/* "classical P1 finite element method"; matrices named in eq. AvML).         */
/* Element [x_e, x_{e+1}] contributes                                         */
/*   mass      (h/6)  [[2,1],[1,2]]                                           */
/*   stiffness (1/h)  [[1,-1],[-1,1]]                                         */
/*   gen. mass (h/12) [[3W_e+W_{e+1}, W_e+W_{e+1}],[W_e+W_{e+1}, W_e+3W_{e+1}]] */
/* (the last one: integral of W phi_a phi_b with W interpolated in P1).       */
/* Assembles the symmetric tridiagonal of  coef_m*M - S + M_W.                */
/* ------------------------------------------------------------------------ */
void orc_assemble(int n, double h, double coef_re, double coef_im, const double *W,
                  cplx *diag, cplx *off)
{
    const cplx coef_m = coef_re + I * coef_im;
    for (int i = 0; i < n; ++i) diag[i] = 0;
    for (int i = 0; i + 1 < n; ++i) off[i] = 0;
    for (int e = 0; e + 1 < n; ++e) {
        double w0 = W ? W[e] : 0.0, w1 = W ? W[e + 1] : 0.0;
        double m00 = 2.0 * h / 6.0, m01 = h / 6.0, m11 = 2.0 * h / 6.0;
        double s00 = 1.0 / h, s01 = -1.0 / h, s11 = 1.0 / h;
        double g00 = h / 12.0 * (3.0 * w0 + w1);
        double g01 = h / 12.0 * (w0 + w1);
        double g11 = h / 12.0 * (w0 + 3.0 * w1);
        diag[e]     += coef_m * m00 - s00 + g00;
        diag[e + 1] += coef_m * m11 - s11 + g11;
        off[e]      += coef_m * m01 - s01 + g01;
    }
}

/* y = M x  (P1 mass matrix, same element matrices as orc_assemble). */
void orc_mass_apply(int n, double h, const cplx *x, cplx *y)
{
    for (int i = 0; i < n; ++i) y[i] = 0;
    for (int e = 0; e + 1 < n; ++e) {
        y[e]     += (2.0 * h / 6.0) * x[e] + (h / 6.0) * x[e + 1];
        y[e + 1] += (h / 6.0) * x[e] + (2.0 * h / 6.0) * x[e + 1];
    }
}

/* y = M_F x, generalised mass with nodal weight F (same element matrix as the
 * M_W block of orc_assemble).  Used for the nonlinear term b_{f(v)} of
 * eq. AvMNL with F_i = |v_i|^2. */
void orc_genmass_apply(int n, double h, const double *F, const cplx *x, cplx *y)
{
    for (int i = 0; i < n; ++i) y[i] = 0;
    for (int e = 0; e + 1 < n; ++e) {
        double f0 = F[e], f1 = F[e + 1];
        double g00 = h / 12.0 * (3.0 * f0 + f1);
        double g01 = h / 12.0 * (f0 + f1);
        double g11 = h / 12.0 * (f0 + 3.0 * f1);
        y[e]     += g00 * x[e] + g01 * x[e + 1];
        y[e + 1] += g01 * x[e] + g11 * x[e + 1];
    }
}

/* Thomas algorithm (no pivoting) for the symmetric tridiagonal system
 * off[i-1] x[i-1] + diag[i] x[i] + off[i] x[i+1] = rhs[i].  The paper's
 * matrices are tridiagonal and symmetric (Sec. 6); they are strictly
 * diagonally dominant for the step sizes used, so no pivoting is needed. */
int orc_thomas(int n, const cplx *diag, const cplx *off, const cplx *rhs, cplx *x)
{
    cplx *cp = malloc(sizeof(cplx) * (size_t)n);
    cplx *dp = malloc(sizeof(cplx) * (size_t)n);
    if (!cp || !dp) { free(cp); free(dp); return -1; }
    cplx piv = diag[0];
    if (piv == 0) { free(cp); free(dp); return -2; }
    cp[0] = (n > 1) ? off[0] / piv : 0;
    dp[0] = rhs[0] / piv;
    for (int i = 1; i < n; ++i) {
        piv = diag[i] - off[i - 1] * cp[i - 1];
        if (piv == 0) { free(cp); free(dp); return -2; }
        cp[i] = (i + 1 < n) ? off[i] / piv : 0;
        dp[i] = (rhs[i] - off[i - 1] * dp[i - 1]) / piv;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    free(cp); free(dp);
    return 0;
}

/* Potential kinds */
enum { ORC_V_STATIC = 0, ORC_V_TIME = 1, ORC_V_CUBIC = 2 };
/* Transmission kinds */
enum { ORC_ROBIN = 0, ORC_S02 = 1, ORC_S03 = 2, ORC_S04 = 3, ORC_S12 = 4, ORC_S14 = 5,
       ORC_P22 = 6, ORC_P24 = 7 };
#define ORC_PADE_MAX 1024

/* W_n on n nodes starting at global node offset `off0`.
 * Static: W = V(x).  Time dependent: W_n = (V_n + V_{n-1})/2 (eq. CNS_L),
 * V stored row-major [nt+1][nx_global]. */
static void weight_at_step(int vkind, const double *V, int nx_global, int off0,
                           int n, int step, double *W)
{
    if (vkind == ORC_V_STATIC) {
        for (int i = 0; i < n; ++i) W[i] = V ? V[off0 + i] : 0.0;
    } else if (vkind == ORC_V_TIME) {
        const double *Vn = V + (size_t)step * nx_global + off0;
        const double *Vm = V + (size_t)(step - 1) * nx_global + off0;
        for (int i = 0; i < n; ++i) W[i] = 0.5 * (Vn[i] + Vm[i]);
    } else {
        for (int i = 0; i < n; ++i) W[i] = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Inner fixed point of the nonlinear scheme (eq. CNS_NL / AvMNL):           */
/*   (c M - S - B) zeta^{s+1} = c M u_{n-1} - M_{|zeta^s|^2} zeta^s + bnd     */
/* starting from zeta^0 = v_{n-1}.  `diag/off` hold the factor-free matrix    */
/* c M - S - B, `base` the data-dependent right-hand side c M u + bnd.        */
/* Stops when max_i |zeta^{s+1}-zeta^s| <= tol * max(1, max_i |zeta^s|).      */
/* Returns iterations used, or -1 if `maxit` is reached.                     */
/* ------------------------------------------------------------------------ */
static int nonlinear_step(int n, double h, const cplx *diag, const cplx *off,
                          const cplx *base, cplx *zeta, int maxit, double tol,
                          cplx *work_rhs, cplx *work_nl, double *work_F, cplx *work_new)
{
    for (int it = 1; it <= maxit; ++it) {
        for (int i = 0; i < n; ++i) work_F[i] = creal(zeta[i] * conj(zeta[i]));
        orc_genmass_apply(n, h, work_F, zeta, work_nl);
        for (int i = 0; i < n; ++i) work_rhs[i] = base[i] - work_nl[i];
        if (orc_thomas(n, diag, off, work_rhs, work_new)) return -2;
        double dmax = 0.0, zmax = 0.0;
        for (int i = 0; i < n; ++i) {
            double d = cabs(work_new[i] - zeta[i]);
            double z = cabs(zeta[i]);
            if (d > dmax) dmax = d;
            if (z > zmax) zmax = z;
        }
        memcpy(zeta, work_new, sizeof(cplx) * (size_t)n);
        if (dmax <= tol * (zmax > 1.0 ? zmax : 1.0)) return it;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Monodomain Crank-Nicolson, P1 in space, homogeneous Neumann walls          */
/* (eq. Schequ with the scheme eq. CNS_L; nonlinear: eq. CNS_NL).            */
/* nx nodes, spacing h, nt steps of size dt.  u0[nx] in, uT[nx] out,          */
/* u_all[(nt+1)*nx] (optional) receives every u_n, v_all[nt*nx] (optional)    */
/* every v_n (n = 1..nt).  Returns 0, or <0 on failure; *nl_worst receives    */
/* the largest inner iteration count (nonlinear only).                        */
/* ------------------------------------------------------------------------ */
int orc_mono_cn(int nx, double h, double dt, int nt, int vkind, const double *V,
                const cplx *u0, cplx *uT, cplx *u_all, cplx *v_all,
                int nl_maxit, double nl_tol, int *nl_worst)
{
    const cplx c = 2.0 * I / dt;
    cplx *diag = malloc(sizeof(cplx) * (size_t)nx), *off = malloc(sizeof(cplx) * (size_t)(nx > 1 ? nx - 1 : 1));
    cplx *u = malloc(sizeof(cplx) * (size_t)nx), *v = malloc(sizeof(cplx) * (size_t)nx);
    cplx *rhs = malloc(sizeof(cplx) * (size_t)nx), *w1 = malloc(sizeof(cplx) * (size_t)nx);
    cplx *w2 = malloc(sizeof(cplx) * (size_t)nx), *w3 = malloc(sizeof(cplx) * (size_t)nx);
    double *W = malloc(sizeof(double) * (size_t)nx);
    int rc = 0, worst = 0;
    memcpy(u, u0, sizeof(cplx) * (size_t)nx);
    memcpy(v, u0, sizeof(cplx) * (size_t)nx);           /* v_0 = u_0 (Sec. 2.2) */
    if (u_all) memcpy(u_all, u0, sizeof(cplx) * (size_t)nx);
    if (vkind == ORC_V_STATIC || vkind == ORC_V_CUBIC) {
        weight_at_step(vkind, V, nx, 0, nx, 0, W);
        orc_assemble(nx, h, creal(c), cimag(c), vkind == ORC_V_CUBIC ? NULL : W, diag, off);
    }
    for (int n = 1; n <= nt && rc == 0; ++n) {
        if (vkind == ORC_V_TIME) {
            weight_at_step(vkind, V, nx, 0, nx, n, W);
            orc_assemble(nx, h, creal(c), cimag(c), W, diag, off);
        }
        orc_mass_apply(nx, h, u, rhs);
        for (int i = 0; i < nx; ++i) rhs[i] *= c;
        if (vkind == ORC_V_CUBIC) {
            /* zeta^0 = v_{n-1}; v holds v_{n-1} here */
            int it = nonlinear_step(nx, h, diag, off, rhs, v, nl_maxit, nl_tol, w1, w2, W, w3);
            if (it < 0) { rc = -3; break; }
            if (it > worst) worst = it;
        } else {
            if (orc_thomas(nx, diag, off, rhs, v)) { rc = -2; break; }
        }
        for (int i = 0; i < nx; ++i) u[i] = 2.0 * v[i] - u[i];
        if (u_all) memcpy(u_all + (size_t)n * nx, u, sizeof(cplx) * (size_t)nx);
        if (v_all) memcpy(v_all + (size_t)(n - 1) * nx, v, sizeof(cplx) * (size_t)nx);
    }
    if (rc == 0) memcpy(uT, u, sizeof(cplx) * (size_t)nx);
    if (nl_worst) *nl_worst = worst;
    free(diag); free(off); free(u); free(v); free(rhs); free(w1); free(w2); free(w3); free(W);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Potential data the transmission operators need at one interface end       */
/* (Sec. 2.2, "Potential strategy" and "Gauge change strategy"), for steps   */
/* n = 0..nt at global node g:                                               */
/*   W[n]    = W_n(x_g) (static: V(x_g); time dependent: (V_n + V_{n-1})/2)   */
/*   dW[n]   = outward normal derivative of W_n at x_g, by the centred        */
/*             difference (W_n(x_{g+1}) - W_n(x_{g-1}))/(2h) times nsign      */
/*             (+1 at a right end b_j, -1 at a left end a_j)                  */
/*   calW[n] = (calV_n + calV_{n-1})/2 with calV_n = int_0^{t_n} V(s, x_g) ds */
/*             by the trapezoid rule on the time grid, calV_n = calV_{n-1} +  */
/*             dt W_n                                                         */
/* Step 0 has no V_{-1}: W_0 = V_0 and calW_0 = calV_0 = 0 (v_0 = u_0 is the   */
/* state at t = 0).  Interior interfaces only (g-1 and g+1 exist).            */
/* ------------------------------------------------------------------------ */
void orc_end_data(int vkind, const double *V, int nx_global, int g, int nsign, double h,
                  double dt, int nt, double *W, double *dW, double *calW)
{
    double calV_prev = 0.0;
    for (int n = 0; n <= nt; ++n) {
        double w = 0.0, wm = 0.0, wp = 0.0;
        if (V && vkind == ORC_V_STATIC) {
            w = V[g]; wm = V[g - 1]; wp = V[g + 1];
        } else if (V && vkind == ORC_V_TIME) {
            const double *Vn = V + (size_t)n * nx_global;
            const double *Vm = V + (size_t)(n > 0 ? n - 1 : 0) * nx_global;
            w = 0.5 * (Vn[g] + Vm[g]);
            wm = 0.5 * (Vn[g - 1] + Vm[g - 1]);
            wp = 0.5 * (Vn[g + 1] + Vm[g + 1]);
        }
        W[n] = w;
        dW[n] = nsign * (wp - wm) / (2.0 * h);
        if (n == 0) {
            calW[0] = 0.0;
        } else {
            double calV = calV_prev + dt * w;
            calW[n] = 0.5 * (calV + calV_prev);
            calV_prev = calV;
        }
    }
}

static double sgn(double x) { return (x > 0.0) - (x < 0.0); }

/* ------------------------------------------------------------------------ */
/* The semi-discrete transmission operator Sbar at step n and one end        */
/* (Sec. 2.2), written as                                                    */
/*     Sbar v_n = sig v_n + hist,     hist = the terms with s < n,            */
/* for the S0^2, S0^3, S0^4, S1^2 and S1^4 operators.  (sig_s, hist_s) is     */
/* the same split without the order-4 normal-derivative term: that term      */
/* changes sign with the normal, so in the exchange of eq. TransmisionCond   */
/* it cancels and 2 (Sbar without it) v is what crosses the interface.       */
/* v[0..n-1] are the past values at this end; W, dW, calW as orc_end_data.   */
/* alpha, beta: weights of at least n+1 entries; gamma = (1, 2, 2, ...).     */
/* ------------------------------------------------------------------------ */
void orc_sbar_parts(int kind, int n, double dt, const cplx *v, const double *W,
                    const double *dW, const double *calW, const double *alpha,
                    const double *beta, cplx *sig, cplx *hist, cplx *sig_s, cplx *hist_s)
{
    const cplx c2 = cexp(-I * M_PI / 4.0) * sqrt(2.0 / dt);
    cplx s2 = 0, h2 = 0, s4 = 0, h4 = 0;
    if (kind == ORC_S02 || kind == ORC_S03 || kind == ORC_S04) {
        cplx b = 0;
        for (int s = 0; s < n; ++s) b += beta[n - s] * v[s];
        s2 = c2 * beta[0];
        h2 = c2 * b;
        if (kind != ORC_S02) {
            /* - e^{i pi/4} sqrt(dt/2) (W_n/2) sum alpha_{n-s} v_s */
            const cplx c3 = -cexp(I * M_PI / 4.0) * sqrt(dt / 2.0) * (W[n] / 2.0);
            cplx a = 0;
            for (int s = 0; s < n; ++s) a += alpha[n - s] * v[s];
            s2 += c3 * alpha[0];
            h2 += c3 * a;
        }
        if (kind == ORC_S04) {
            /* - i (dn W_n / 4) (dt/2) sum gamma_{n-s} v_s */
            const cplx c4 = -I * (dW[n] / 4.0) * (dt / 2.0);
            cplx gsum = 0;
            for (int s = 0; s < n; ++s) gsum += 2.0 * v[s];
            s4 = c4 * 1.0;
            h4 = c4 * gsum;
        }
    } else if (kind == ORC_S12 || kind == ORC_S14) {
        /* c2 e^{i calW_n} sum beta_{n-s} e^{-i calW_s} v_s; the s = n term is
           c2 beta_0 v_n */
        cplx b = 0;
        for (int s = 0; s < n; ++s) b += beta[n - s] * cexp(-I * calW[s]) * v[s];
        s2 = c2 * beta[0];
        h2 = c2 * cexp(I * calW[n]) * b;
        if (kind == ORC_S14) {
            const double qn = sqrt(fabs(dW[n])) / 2.0;
            const cplx c4 = -I * sgn(dW[n]) * qn * cexp(I * calW[n]) * (dt / 2.0);
            cplx gsum = 0;
            for (int s = 0; s < n; ++s) gsum += 2.0 * (sqrt(fabs(dW[s])) / 2.0) * cexp(-I * calW[s]) * v[s];
            s4 = c4 * 1.0 * qn * cexp(-I * calW[n]);
            h4 = c4 * gsum;
        }
    }
    *sig = s2 + s4;
    *hist = h2 + h4;
    *sig_s = s2;
    *hist_s = h2;
}

/* Sbar v_n for n = 0..nt of a given sequence v (test access to the operator):
   out[n] with every term, out_s[n] without the order-4 term. */
void orc_sbar_apply(int kind, int nt, double dt, const cplx *v, const double *W,
                    const double *dW, const double *calW, cplx *out, cplx *out_s)
{
    double *alpha = malloc(sizeof(double) * (size_t)(nt + 1));
    double *beta = malloc(sizeof(double) * (size_t)(nt + 1));
    orc_alpha(nt + 1, alpha);
    orc_beta(nt + 1, beta);
    for (int n = 0; n <= nt; ++n) {
        cplx sg, hs, sgs, hss;
        orc_sbar_parts(kind, n, dt, v, W, dW, calW, alpha, beta, &sg, &hs, &sgs, &hss);
        out[n] = sg * v[n] + hs;
        out_s[n] = sgs * v[n] + hss;
    }
    free(alpha); free(beta);
}

/* ------------------------------------------------------------------------ */
/* Pade approximation strategy (Sec. 2.1 "l=2", Sec. 2.2).  S2^2 is           */
/* -i sqrt(i d_t + V) with the square root replaced by the rational function  */
/*     sqrt(z) ~ sum_{s=0}^m a_s - sum_{s=1}^m a_s d_s / (z + d_s),           */
/* whose coefficients the paper takes from its references without stating   */
/* them.  Reading: the diagonal [m/m] Pade approximant of sqrt(1 + w) at     */
/* w = 0 in its partial-fraction form                                        */
/*     R_m(w) = 1 + sum_{s=1}^m A_s w / (1 + B_s w),                           */
/*     A_s = 2/(2m+1) sin^2(s pi/(2m+1)),  B_s = cos^2(s pi/(2m+1))            */
/* (Baker & Graves-Morris, "Pade Approximants"; Milinazzo, Zala & Brooke,    */
/* J. Acoust. Soc. Am. 101 (1997), which also rotates the branch cut), with  */
/* the cut rotated by theta: sqrt(z) = e^{i theta/2} sqrt(1 + w),            */
/* w = e^{-i theta} z - 1.  From w/(1 + B w) = (1 - 1/(1 + B w))/B and       */
/* 1 + B w = B e^{-i theta} (z + e^{i theta}(1 - B)/B) the paper's form has  */
/*     d_s = e^{i theta} (1 - B_s) / B_s,                                      */
/*     a_s = e^{i theta/2} A_s / (B_s (1 - B_s))            (s >= 1),          */
/*     a_0 = e^{i theta/2} R_m(-1)            (the value of the form at z = 0).*/
/* a[0..m], d[0..m] (d[0] = 0, unused).                                      */
/* ------------------------------------------------------------------------ */
void orc_pade_coef(int m, double theta, cplx *a, cplx *d)
{
    const cplx rot = cexp(I * theta / 2.0);
    double r_at_minus1 = 1.0;
    a[0] = 0;
    d[0] = 0;
    for (int s = 1; s <= m; ++s) {
        const double ang = s * M_PI / (2.0 * m + 1.0);
        const double A = 2.0 / (2.0 * m + 1.0) * sin(ang) * sin(ang);
        const double B = cos(ang) * cos(ang);
        d[s] = cexp(I * theta) * (1.0 - B) / B;
        a[s] = rot * A / (B * (1.0 - B));
        r_at_minus1 += A * (-1.0) / (1.0 - B);
    }
    a[0] = rot * r_at_minus1;
}

/* The rational function above at z (test access to the coefficients). */
void orc_pade_eval(int m, double theta, double zr, double zi, double *out)
{
    cplx *a = malloc(sizeof(cplx) * (size_t)(m + 1)), *d = malloc(sizeof(cplx) * (size_t)(m + 1));
    orc_pade_coef(m, theta, a, d);
    const cplx z = zr + I * zi;
    cplx r = 0;
    for (int s = 0; s <= m; ++s) r += a[s];
    for (int s = 1; s <= m; ++s) r -= a[s] * d[s] / (z + d[s]);
    out[0] = creal(r);
    out[1] = cimag(r);
    free(a); free(d);
}

/* Sbar_2^{2,m} / Sbar_2^{4,m} at step n and one end (Sec. 2.2), with c =     */
/* 2i/dt, W = W_n and dW = dn W_n at the end:                                 */
/*   Sbar_2^2 v_n = -i (sum_{s=0}^m a_s) v_n                                  */
/*                  + i sum_s a_s d_s [ v_n + c phi^s_{n-1} ] / (c + W + d_s)  */
/*   Sbar_2^4 v_n = Sbar_2^2 v_n + (dW/4) v_n / (c + W)                       */
/*                  + sgn(dW) (sqrt|dW|/2) c psi_{n-1} / (c + W)              */
/* written as sig v_n + hist; (sig_s, hist_s) drops the order-4 terms, which  */
/* change sign with the normal (as for S0^4).  The paper's third term writes  */
/* d_k^m in its denominator: read as d_s^m.                                   */
static void pade_parts(int order, int m, const cplx *a, const cplx *d, double dt, double W,
                       double dW, const cplx *phi, cplx psi, cplx *sig, cplx *hist, cplx *sig_s,
                       cplx *hist_s)
{
    const cplx c = 2.0 * I / dt;
    cplx asum = 0, s2, h2 = 0;
    for (int s = 0; s <= m; ++s) asum += a[s];
    s2 = -I * asum;
    for (int s = 1; s <= m; ++s) {
        const cplx den = c + W + d[s];
        s2 += I * a[s] * d[s] * (1.0 / den);
        h2 += I * a[s] * d[s] * (c / den) * phi[s];
    }
    *sig_s = s2;
    *hist_s = h2;
    if (order == 4) {
        const double q = sqrt(fabs(dW)) / 2.0;
        s2 += (dW / 4.0) * (1.0 / (c + W));
        h2 += sgn(dW) * q * (c / (c + W)) * psi;
    }
    *sig = s2;
    *hist = h2;
}

/* The auxiliary functions once v_n is known (Sec. 2.2):                      */
/*   phi^s_{n-1/2} = v_n/(c + W + d_s) + c phi^s_{n-1}/(c + W + d_s),         */
/*   phi^s_n = 2 phi^s_{n-1/2} - phi^s_{n-1},  phi^s_0 = 0;                    */
/*   psi_{n-1/2} = (sqrt|dW|/2) v_n/(c + W) + c psi_{n-1}/(c + W),             */
/*   psi_n = 2 psi_{n-1/2} - psi_{n-1},  psi_0 = 0.                            */
static void pade_advance(int order, int m, const cplx *d, double dt, double W, double dW, cplx v,
                         cplx *phi, cplx *psi)
{
    const cplx c = 2.0 * I / dt;
    for (int s = 1; s <= m; ++s) {
        const cplx den = c + W + d[s];
        const cplx half = v * (1.0 / den) + (c / den) * phi[s];
        phi[s] = 2.0 * half - phi[s];
    }
    if (order == 4) {
        const double q = sqrt(fabs(dW)) / 2.0;
        const cplx half = q * v * (1.0 / (c + W)) + (c / (c + W)) * *psi;
        *psi = 2.0 * half - *psi;
    }
}

/* Sbar v_n, n = 1..nt, of S2^{order,m} on a given sequence v (test access;   */
/* v_0 plays no part: phi_0 = psi_0 = 0); out[0] = out_s[0] = 0.  W, dW as    */
/* orc_end_data.  Returns -5 for a bad order or m.                            */
int orc_pade_apply(int order, int m, double theta, int nt, double dt, const cplx *v,
                   const double *W, const double *dW, cplx *out, cplx *out_s)
{
    if ((order != 2 && order != 4) || m < 1 || m > ORC_PADE_MAX) return -5;
    cplx *a = malloc(sizeof(cplx) * (size_t)(m + 1)), *d = malloc(sizeof(cplx) * (size_t)(m + 1));
    cplx *phi = calloc((size_t)(m + 1), sizeof(cplx));
    cplx psi = 0;
    orc_pade_coef(m, theta, a, d);
    out[0] = 0;
    out_s[0] = 0;
    for (int n = 1; n <= nt; ++n) {
        cplx sg, hs, sgs, hss;
        pade_parts(order, m, a, d, dt, W[n], dW[n], phi, psi, &sg, &hs, &sgs, &hss);
        out[n] = sg * v[n] + hs;
        out_s[n] = sgs * v[n] + hss;
        pade_advance(order, m, d, dt, W[n], dW[n], v[n], phi, &psi);
    }
    free(a); free(d); free(phi);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One subdomain over the whole time window (eq. AvML for linear V,          */
/* eq. AvMNL for f(u) = |u|^2), with the transmission conditions written by  */
/* fluxes (eq. TransmissionCondlocal) and the exchange of                    */
/* eq. TransmissionCond_disc:                                                */
/*                                                                           */
/*  (A_n - B_n) v_n = c M u_{n-1} + b_n - Q^T (l_n, r_n)^T                   */
/*  Sbar v_n = sig_n v_n + h_n at each end (orc_sbar_parts; Robin: sig_n =  */
/*        sigma, h_n = 0), with v_0 = u_0 at the boundary node                */
/*  B_n = sig_n E   (E picks the interface ends; walls keep Neumann)         */
/*  b_n = Q^T (h_n(a), h_n(b))                                               */
/*  outgoing fluxes:  rhoL_n = -l_n + 2 (sig'_n v_n(a) + h'_n(a))            */
/*                    rhoR_n = -r_n + 2 (sig'_n v_n(b) + h'_n(b))            */
/*  where ' drops the order-4 normal-derivative term (S0^4, S1^4, S2^4).     */
/*  trans: 0 Robin, 1 S0^2, 2 S0^3, 3 S0^4, 4 S1^2, 5 S1^4, 6 S2^{2,m},      */
/*  7 S2^{4,m} (pade_m auxiliary functions, branch rotation pade_theta); the */
/*  order-4 operators need a linear potential (returns -4 with |u|^2); with  */
/*  |u|^2 the others take W_n = |v_{n-1}|^2 at the end node.                 */
/*                                                                           */
/* The subdomain has n nodes starting at global node `off0` of a mesh with   */
/* nx_global nodes (V is indexed globally).  left_iface/right_iface say      */
/* whether each end is an interface (1) or a Neumann wall (0).               */
/* u0: local initial data (NULL = zero).  hist0: value used for v_0 in the   */
/* history of Sbar at each end (NULL = u0 ends, as in the paper).            */
/* l, r: incoming fluxes for n = 1..nt (index 0..nt-1); NULL = zero.         */
/* Outputs (each optional): rhoL/rhoR[nt], uT[n], va/vb[nt+1] (v_n at the    */
/* two ends, n = 0..nt), v_all[nt*n].                                        */
/* ------------------------------------------------------------------------ */
int orc_sub_sweep(int n, double h, double dt, int nt, int vkind, const double *V,
                  int nx_global, int off0, int left_iface, int right_iface,
                  int trans, double sigma_re, double sigma_im, const double *beta,
                  const cplx *u0, const cplx *hist0,
                  const cplx *l, const cplx *r,
                  cplx *rhoL, cplx *rhoR, cplx *uT, cplx *va, cplx *vb, cplx *v_all,
                  int nl_maxit, double nl_tol, int *nl_worst, int pade_m, double pade_theta)
{
    const cplx c = 2.0 * I / dt;
    const int pade = trans == ORC_P22 || trans == ORC_P24;
    const int conv = trans != ORC_ROBIN && !pade;     /* a convolution-type Sbar */
    const int porder = trans == ORC_P24 ? 4 : 2;
    /* the order-4 operators carry dn W_n; with f(u) = |u|^2 the paper finds
       no discretisation of dn f(u) that keeps the interfaces continuous */
    if ((trans == ORC_S04 || trans == ORC_S14 || trans == ORC_P24) && vkind == ORC_V_CUBIC) return -4;
    if (trans < ORC_ROBIN || trans > ORC_P24) return -5;
    if (pade && (pade_m < 1 || pade_m > ORC_PADE_MAX)) return -5;
    cplx *diag = malloc(sizeof(cplx) * (size_t)n), *off = malloc(sizeof(cplx) * (size_t)(n > 1 ? n - 1 : 1));
    cplx *u = malloc(sizeof(cplx) * (size_t)n), *v = malloc(sizeof(cplx) * (size_t)n);
    cplx *rhs = malloc(sizeof(cplx) * (size_t)n), *w1 = malloc(sizeof(cplx) * (size_t)n);
    cplx *w2 = malloc(sizeof(cplx) * (size_t)n), *w3 = malloc(sizeof(cplx) * (size_t)n);
    double *W = malloc(sizeof(double) * (size_t)n);
    cplx *ta = malloc(sizeof(cplx) * (size_t)(nt + 1)), *tb = malloc(sizeof(cplx) * (size_t)(nt + 1));
    double *alpha = malloc(sizeof(double) * (size_t)(nt + 1));
    double *ed = malloc(sizeof(double) * (size_t)(nt + 1) * 6);   /* W, dW, calW at a and b */
    double *Wa = ed, *dWa = ed + (nt + 1), *cWa = ed + 2 * (nt + 1);
    double *Wb = ed + 3 * (nt + 1), *dWb = ed + 4 * (nt + 1), *cWb = ed + 5 * (nt + 1);
    int rc = 0, worst = 0;
    /* Pade: coefficients and the auxiliary functions of the two ends */
    const int pm = pade ? pade_m : 0;
    cplx *pa = malloc(sizeof(cplx) * (size_t)(pm + 1)), *pd = malloc(sizeof(cplx) * (size_t)(pm + 1));
    cplx *phiA = calloc((size_t)(pm + 1), sizeof(cplx)), *phiB = calloc((size_t)(pm + 1), sizeof(cplx));
    cplx psiA = 0, psiB = 0;
    if (pade) orc_pade_coef(pm, pade_theta, pa, pd);

    orc_alpha(nt + 1, alpha);
    memset(ed, 0, sizeof(double) * (size_t)(nt + 1) * 6);
    if (trans > ORC_S02) {
        if (left_iface)  orc_end_data(vkind, V, nx_global, off0, -1, h, dt, nt, Wa, dWa, cWa);
        if (right_iface) orc_end_data(vkind, V, nx_global, off0 + n - 1, +1, h, dt, nt, Wb, dWb, cWb);
    }
    for (int i = 0; i < n; ++i) u[i] = u0 ? u0[i] : 0;
    memcpy(v, u, sizeof(cplx) * (size_t)n);                      /* v_0 = u_0 */
    ta[0] = hist0 ? hist0[0] : u[0];
    tb[0] = hist0 ? hist0[1] : u[n - 1];

    double cvA = 0.0, cvB = 0.0;     /* |u|^2: calV_{n-1} at the two ends */
    for (int step = 1; step <= nt && rc == 0; ++step) {
        if (vkind == ORC_V_CUBIC && trans > ORC_S02) {
            /* W_n = f(u) at the end node, taken at the start of the step's
               inner fixed point (zeta^0 = v_{n-1}), so that B_n stays fixed
               over the inner iteration as eq. AvMNL writes it; dn W is not
               used (order 2 and 3 only); calV, calW as for a linear potential */
            Wa[step] = creal(v[0]) * creal(v[0]) + cimag(v[0]) * cimag(v[0]);
            Wb[step] = creal(v[n - 1]) * creal(v[n - 1]) + cimag(v[n - 1]) * cimag(v[n - 1]);
            const double nA = cvA + dt * Wa[step], nB = cvB + dt * Wb[step];
            cWa[step] = 0.5 * (nA + cvA);
            cWb[step] = 0.5 * (nB + cvB);
            cvA = nA;
            cvB = nB;
        }
        /* A_n = cM - S + M_{W_n} (rebuilt every step: W_n and the implicit
           part of Sbar may change with n) */
        weight_at_step(vkind, V, nx_global, off0, n, vkind == ORC_V_TIME ? step : 0, W);
        orc_assemble(n, h, creal(c), cimag(c), vkind == ORC_V_CUBIC ? NULL : W, diag, off);
        /* Sbar v_n = sig v_n + hist at each interface end */
        cplx sgA = sigma_re + I * sigma_im, sgB = sgA, hA = 0, hB = 0;
        cplx sgAs = sgA, sgBs = sgB, hAs = 0, hBs = 0;
        if (conv) {
            orc_sbar_parts(trans, step, dt, ta, Wa, dWa, cWa, alpha, beta, &sgA, &hA, &sgAs, &hAs);
            orc_sbar_parts(trans, step, dt, tb, Wb, dWb, cWb, alpha, beta, &sgB, &hB, &sgBs, &hBs);
        }
        if (pade) {
            pade_parts(porder, pm, pa, pd, dt, Wa[step], dWa[step], phiA, psiA, &sgA, &hA, &sgAs, &hAs);
            pade_parts(porder, pm, pa, pd, dt, Wb[step], dWb[step], phiB, psiB, &sgB, &hB, &sgBs, &hBs);
        }
        if (left_iface)  diag[0]     -= sgA;
        if (right_iface) diag[n - 1] -= sgB;
        cplx ln = l ? l[step - 1] : 0, rn = r ? r[step - 1] : 0;
        orc_mass_apply(n, h, u, rhs);
        for (int i = 0; i < n; ++i) rhs[i] *= c;
        if (left_iface)  rhs[0]     += hA - ln;
        if (right_iface) rhs[n - 1] += hB - rn;
        if (vkind == ORC_V_CUBIC) {
            int it = nonlinear_step(n, h, diag, off, rhs, v, nl_maxit, nl_tol, w1, w2, W, w3);
            if (it < 0) { rc = -3; break; }
            if (it > worst) worst = it;
        } else {
            if (orc_thomas(n, diag, off, rhs, v)) { rc = -2; break; }
        }
        for (int i = 0; i < n; ++i) u[i] = 2.0 * v[i] - u[i];
        ta[step] = v[0]; tb[step] = v[n - 1];
        if (pade) {
            pade_advance(porder, pm, pd, dt, Wa[step], dWa[step], v[0], phiA, &psiA);
            pade_advance(porder, pm, pd, dt, Wb[step], dWb[step], v[n - 1], phiB, &psiB);
        }
        if (rhoL) rhoL[step - 1] = left_iface  ? -ln + 2.0 * (sgAs * v[0] + hAs) : 0;
        if (rhoR) rhoR[step - 1] = right_iface ? -rn + 2.0 * (sgBs * v[n - 1] + hBs) : 0;
        if (v_all) memcpy(v_all + (size_t)(step - 1) * n, v, sizeof(cplx) * (size_t)n);
    }
    if (rc == 0) {
        if (uT) memcpy(uT, u, sizeof(cplx) * (size_t)n);
        if (va) memcpy(va, ta, sizeof(cplx) * (size_t)(nt + 1));
        if (vb) memcpy(vb, tb, sizeof(cplx) * (size_t)(nt + 1));
    }
    if (nl_worst) *nl_worst = worst;
    free(diag); free(off); free(u); free(v); free(rhs); free(w1); free(w2); free(w3);
    free(W); free(ta); free(tb); free(alpha); free(ed);
    free(pa); free(pd); free(phiA); free(phiB);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The monodomain Crank-Nicolson solve of orc_mono_cn in extended precision  */
/* (x87 80-bit long double: 64-bit significand, unit roundoff 5.4e-20), for  */
/* grids where one FP64 Thomas sweep over the whole domain is itself the     */
/* largest error: with dt/h^2 = 1e5 the elimination over 1e4-1e5 nodes of    */
/* c M - S (nearly a discrete Laplacian with a small imaginary shift) loses  */
/* about 1e-9 relative in FP64.  Same definitions, element matrices and      */
/* inner fixed point as above; inputs and outputs are FP64.                  */
/* ------------------------------------------------------------------------ */
typedef long double complex lcplx;
typedef long double lreal;

static void ld_assemble(int n, lreal h, lcplx coef_m, const lreal *W, lcplx *diag, lcplx *off)
{
    for (int i = 0; i < n; ++i) diag[i] = 0;
    for (int i = 0; i + 1 < n; ++i) off[i] = 0;
    for (int e = 0; e + 1 < n; ++e) {
        lreal w0 = W ? W[e] : 0.0L, w1 = W ? W[e + 1] : 0.0L;
        lreal m00 = 2.0L * h / 6.0L, m01 = h / 6.0L, m11 = 2.0L * h / 6.0L;
        lreal s00 = 1.0L / h, s01 = -1.0L / h, s11 = 1.0L / h;
        lreal g00 = h / 12.0L * (3.0L * w0 + w1);
        lreal g01 = h / 12.0L * (w0 + w1);
        lreal g11 = h / 12.0L * (w0 + 3.0L * w1);
        diag[e]     += coef_m * m00 - s00 + g00;
        diag[e + 1] += coef_m * m11 - s11 + g11;
        off[e]      += coef_m * m01 - s01 + g01;
    }
}

static void ld_mass_apply(int n, lreal h, const lcplx *x, lcplx *y)
{
    for (int i = 0; i < n; ++i) y[i] = 0;
    for (int e = 0; e + 1 < n; ++e) {
        y[e]     += (2.0L * h / 6.0L) * x[e] + (h / 6.0L) * x[e + 1];
        y[e + 1] += (h / 6.0L) * x[e] + (2.0L * h / 6.0L) * x[e + 1];
    }
}

static void ld_genmass_apply(int n, lreal h, const lreal *F, const lcplx *x, lcplx *y)
{
    for (int i = 0; i < n; ++i) y[i] = 0;
    for (int e = 0; e + 1 < n; ++e) {
        lreal f0 = F[e], f1 = F[e + 1];
        lreal g00 = h / 12.0L * (3.0L * f0 + f1);
        lreal g01 = h / 12.0L * (f0 + f1);
        lreal g11 = h / 12.0L * (f0 + 3.0L * f1);
        y[e]     += g00 * x[e] + g01 * x[e + 1];
        y[e + 1] += g01 * x[e] + g11 * x[e + 1];
    }
}

static int ld_thomas(int n, const lcplx *diag, const lcplx *off, const lcplx *rhs, lcplx *x,
                     lcplx *cp, lcplx *dp)
{
    lcplx piv = diag[0];
    if (piv == 0) return -2;
    cp[0] = (n > 1) ? off[0] / piv : 0;
    dp[0] = rhs[0] / piv;
    for (int i = 1; i < n; ++i) {
        piv = diag[i] - off[i - 1] * cp[i - 1];
        if (piv == 0) return -2;
        cp[i] = (i + 1 < n) ? off[i] / piv : 0;
        dp[i] = (rhs[i] - off[i - 1] * dp[i - 1]) / piv;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    return 0;
}

/* Same interface as orc_mono_cn (no u_all / v_all).  The |u|^2 inner fixed */
/* point stops on max |zeta^{s+1} - zeta^s| <= tol max(1, max |zeta^s|).     */
int orc_mono_cn_ld(int nx, double h_, double dt_, int nt, int vkind, const double *V,
                   const cplx *u0, cplx *uT, int nl_maxit, double nl_tol, int *nl_worst)
{
    const lreal h = h_, dt = dt_;
    const lcplx c = 2.0L * I / dt;
    lcplx *diag = malloc(sizeof(lcplx) * (size_t)nx), *off = malloc(sizeof(lcplx) * (size_t)(nx > 1 ? nx - 1 : 1));
    lcplx *u = malloc(sizeof(lcplx) * (size_t)nx), *v = malloc(sizeof(lcplx) * (size_t)nx);
    lcplx *rhs = malloc(sizeof(lcplx) * (size_t)nx), *base = malloc(sizeof(lcplx) * (size_t)nx);
    lcplx *nl = malloc(sizeof(lcplx) * (size_t)nx), *z = malloc(sizeof(lcplx) * (size_t)nx);
    lcplx *cp = malloc(sizeof(lcplx) * (size_t)nx), *dp = malloc(sizeof(lcplx) * (size_t)nx);
    lreal *W = malloc(sizeof(lreal) * (size_t)nx);
    int rc = 0, worst = 0;
    for (int i = 0; i < nx; ++i) { u[i] = u0[i]; v[i] = u0[i]; }     /* v_0 = u_0 */
    if (vkind != ORC_V_TIME) {
        for (int i = 0; i < nx; ++i) W[i] = (vkind == ORC_V_STATIC && V) ? V[i] : 0.0L;
        ld_assemble(nx, h, c, vkind == ORC_V_CUBIC ? NULL : W, diag, off);
    }
    for (int n = 1; n <= nt && rc == 0; ++n) {
        if (vkind == ORC_V_TIME) {
            const double *Vn = V + (size_t)n * nx, *Vm = V + (size_t)(n - 1) * nx;
            for (int i = 0; i < nx; ++i) W[i] = 0.5L * ((lreal)Vn[i] + (lreal)Vm[i]);
            ld_assemble(nx, h, c, W, diag, off);
        }
        ld_mass_apply(nx, h, u, base);
        for (int i = 0; i < nx; ++i) base[i] *= c;
        if (vkind == ORC_V_CUBIC) {
            /* inner fixed point from zeta^0 = v_{n-1} (eq. AvMNL) */
            int it = 1, conv = 0;
            for (; it <= nl_maxit; ++it) {
                for (int i = 0; i < nx; ++i) W[i] = creall(v[i]) * creall(v[i]) + cimagl(v[i]) * cimagl(v[i]);
                ld_genmass_apply(nx, h, W, v, nl);
                for (int i = 0; i < nx; ++i) rhs[i] = base[i] - nl[i];
                if (ld_thomas(nx, diag, off, rhs, z, cp, dp)) { rc = -2; break; }
                lreal dmax = 0, zmax = 0;
                for (int i = 0; i < nx; ++i) {
                    lreal d = cabsl(z[i] - v[i]), a = cabsl(v[i]);
                    if (d > dmax) dmax = d;
                    if (a > zmax) zmax = a;
                }
                memcpy(v, z, sizeof(lcplx) * (size_t)nx);
                if (dmax <= nl_tol * (zmax > 1.0L ? zmax : 1.0L)) { conv = 1; break; }
            }
            if (rc) break;
            if (!conv) { rc = -3; break; }
            if (it > worst) worst = it;
        } else {
            if (ld_thomas(nx, diag, off, base, v, cp, dp)) { rc = -2; break; }
        }
        for (int i = 0; i < nx; ++i) u[i] = 2.0L * v[i] - u[i];
    }
    if (rc == 0) for (int i = 0; i < nx; ++i) uT[i] = (cplx)u[i];
    if (nl_worst) *nl_worst = worst;
    free(diag); free(off); free(u); free(v); free(rhs); free(base); free(nl); free(z);
    free(cp); free(dp); free(W);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the monodomain CN map for a static real V(x).         */
/* Forward:  A v_n = c M u_{n-1},  u_n = 2 v_n - u_{n-1},  A = cM - S + M_V.  */
/* A is complex symmetric (A^T = A).  For a real objective J(u_nt) with       */
/* upstream gradient gbar = dJ/dRe(u_nt) + i dJ/dIm(u_nt), write              */
/* P_n = conj(lambda_n) (lambda_n the gradient w.r.t. u_n).  Then             */
/*   P_nt = conj(gbar);  for n = nt..1:  A Q_n = P_n,                          */
/*   dJ/dV_i -= 2 Re( Q_n^T (dM_V/dV_i) v_n ),  P_{n-1} = 2 c M Q_n - P_n,    */
/* and dJ/du0 = conj(P_0).  This is the chain rule applied to eq. CNS_L;       */
/* v_all[nt*nx] holds the forward v_n, n = 1..nt.                             */
/* Outputs: dV[nx] (real), du0[nx].                                           */
/* ------------------------------------------------------------------------ */
int orc_mono_adjoint(int nx, double h, double dt, int nt, const double *V,
                     const cplx *v_all, const cplx *gbar, double *dV, cplx *du0)
{
    const cplx c = 2.0 * I / dt;
    cplx *diag = malloc(sizeof(cplx) * (size_t)nx), *off = malloc(sizeof(cplx) * (size_t)(nx > 1 ? nx - 1 : 1));
    cplx *P = malloc(sizeof(cplx) * (size_t)nx), *Q = malloc(sizeof(cplx) * (size_t)nx);
    cplx *MQ = malloc(sizeof(cplx) * (size_t)nx);
    int rc = 0;
    orc_assemble(nx, h, creal(c), cimag(c), V, diag, off);
    for (int i = 0; i < nx; ++i) { P[i] = conj(gbar[i]); dV[i] = 0.0; }
    for (int n = nt; n >= 1 && rc == 0; --n) {
        if (orc_thomas(nx, diag, off, P, Q)) { rc = -2; break; }
        const cplx *vn = v_all + (size_t)(n - 1) * nx;
        /* dM_V/dV_i: element [e,e+1] contributes (h/12)[[3,1],[1,1]] for
           i = e and (h/12)[[1,1],[1,3]] for i = e+1 (derivative of the
           generalised-mass element matrix above). */
        for (int e = 0; e + 1 < nx; ++e) {
            cplx q0 = Q[e], q1 = Q[e + 1], a0 = vn[e], a1 = vn[e + 1];
            cplx t_left  = (h / 12.0) * (q0 * (3.0 * a0 + a1) + q1 * (a0 + a1));
            cplx t_right = (h / 12.0) * (q0 * (a0 + a1) + q1 * (a0 + 3.0 * a1));
            dV[e]     -= 2.0 * creal(t_left);
            dV[e + 1] -= 2.0 * creal(t_right);
        }
        orc_mass_apply(nx, h, Q, MQ);
        for (int i = 0; i < nx; ++i) P[i] = 2.0 * c * MQ[i] - P[i];
    }
    if (rc == 0) for (int i = 0; i < nx; ++i) du0[i] = conj(P[i]);
    free(diag); free(off); free(P); free(Q); free(MQ);
    return rc;
}
