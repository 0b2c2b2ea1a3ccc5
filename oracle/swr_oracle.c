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
 *   Robin: Sbar v_n = sigma v_n (the caller passes the complex sigma of dn + sigma)
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
enum { ORC_ROBIN = 0, ORC_S02 = 1 };

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
/* One subdomain over the whole time window (eq. AvML for linear V,          */
/* eq. AvMNL for f(u) = |u|^2), with the transmission conditions written by  */
/* fluxes (eq. TransmissionCondlocal) and the exchange of                    */
/* eq. TransmissionCond_disc:                                                */
/*                                                                           */
/*  (A_n - B_n) v_n = c M u_{n-1} + b_n - Q^T (l_n, r_n)^T                   */
/*  B_n = sigma E   (E picks the interface ends; walls keep Neumann)         */
/*  b_n = Q^T (h_n(a), h_n(b)),  h_n = c2 sum_{s=0}^{n-1} beta_{n-s} v_s      */
/*        (S0^2; zero for Robin), with v_0 = u_0 at the boundary node         */
/*  outgoing fluxes:  rhoL_n = -l_n + 2 (sigma v_n(a) + h_n(a))              */
/*                    rhoR_n = -r_n + 2 (sigma v_n(b) + h_n(b))              */
/*                                                                           */
/* The subdomain has n nodes starting at global node `off0` of a mesh with   */
/* nx_global nodes (V is indexed globally).  left_iface/right_iface say      */
/* whether each end is an interface (1) or a Neumann wall (0).               */
/* u0: local initial data (NULL = zero).  hist0: value used for v_0 in the   */
/* S0^2 history at each end (NULL = u0 ends, as in the paper).               */
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
                  int nl_maxit, double nl_tol, int *nl_worst)
{
    const cplx c = 2.0 * I / dt;
    const cplx c2 = cexp(-I * M_PI / 4.0) * sqrt(2.0 / dt);
    /* S0^2: the s = n term of c2 sum beta_{n-s} v_s is the implicit part,
       coefficient c2 beta_0; Robin: the caller's sigma. */
    const cplx sigma = (trans == ORC_S02) ? c2 * beta[0] : sigma_re + I * sigma_im;
    cplx *diag = malloc(sizeof(cplx) * (size_t)n), *off = malloc(sizeof(cplx) * (size_t)(n > 1 ? n - 1 : 1));
    cplx *u = malloc(sizeof(cplx) * (size_t)n), *v = malloc(sizeof(cplx) * (size_t)n);
    cplx *rhs = malloc(sizeof(cplx) * (size_t)n), *w1 = malloc(sizeof(cplx) * (size_t)n);
    cplx *w2 = malloc(sizeof(cplx) * (size_t)n), *w3 = malloc(sizeof(cplx) * (size_t)n);
    double *W = malloc(sizeof(double) * (size_t)n);
    cplx *ha = malloc(sizeof(cplx) * (size_t)(nt + 1)), *hb = malloc(sizeof(cplx) * (size_t)(nt + 1));
    cplx *ta = malloc(sizeof(cplx) * (size_t)(nt + 1)), *tb = malloc(sizeof(cplx) * (size_t)(nt + 1));
    int rc = 0, worst = 0;

    for (int i = 0; i < n; ++i) u[i] = u0 ? u0[i] : 0;
    memcpy(v, u, sizeof(cplx) * (size_t)n);                      /* v_0 = u_0 */
    ta[0] = hist0 ? hist0[0] : u[0];
    tb[0] = hist0 ? hist0[1] : u[n - 1];

    if (vkind != ORC_V_TIME) {
        weight_at_step(vkind, V, nx_global, off0, n, 0, W);
        orc_assemble(n, h, creal(c), cimag(c), vkind == ORC_V_CUBIC ? NULL : W, diag, off);
        if (left_iface)  diag[0]     -= sigma;
        if (right_iface) diag[n - 1] -= sigma;
    }
    for (int step = 1; step <= nt && rc == 0; ++step) {
        if (vkind == ORC_V_TIME) {
            weight_at_step(vkind, V, nx_global, off0, n, step, W);
            orc_assemble(n, h, creal(c), cimag(c), W, diag, off);
            if (left_iface)  diag[0]     -= sigma;
            if (right_iface) diag[n - 1] -= sigma;
        }
        /* history part b_n of the S0^2 operator */
        cplx hA = 0, hB = 0;
        if (trans == ORC_S02) {
            for (int s = 0; s < step; ++s) {
                hA += beta[step - s] * ta[s];
                hB += beta[step - s] * tb[s];
            }
            hA *= c2; hB *= c2;
        }
        ha[step] = hA; hb[step] = hB;
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
        if (rhoL) rhoL[step - 1] = left_iface  ? -ln + 2.0 * (sigma * v[0] + hA) : 0;
        if (rhoR) rhoR[step - 1] = right_iface ? -rn + 2.0 * (sigma * v[n - 1] + hB) : 0;
        if (v_all) memcpy(v_all + (size_t)(step - 1) * n, v, sizeof(cplx) * (size_t)n);
    }
    if (rc == 0) {
        if (uT) memcpy(uT, u, sizeof(cplx) * (size_t)n);
        if (va) memcpy(va, ta, sizeof(cplx) * (size_t)(nt + 1));
        if (vb) memcpy(vb, tb, sizeof(cplx) * (size_t)(nt + 1));
    }
    if (nl_worst) *nl_worst = worst;
    free(diag); free(off); free(u); free(v); free(rhs); free(w1); free(w2); free(w3);
    free(W); free(ha); free(hb); free(ta); free(tb);
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
