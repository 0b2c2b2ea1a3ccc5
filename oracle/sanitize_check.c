/*
 * sanitize_check.c -- runs every entry point of the oracle's C core
 * (swr_oracle.c) on small inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py).  TEST
 * INFRASTRUCTURE ONLY, like the oracle itself.
 *
 * Covered: the alpha/beta weights, P1 assembly and mass products, Thomas, the
 * monodomain Crank-Nicolson scheme in FP64 and extended precision for static,
 * time-dependent and |u|^2 potentials, the interface data and Sbar of every
 * transmission operator, one subdomain sweep per operator and potential kind
 * (interface and wall ends, with and without data and incoming fluxes), and
 * the discrete adjoint.  Prints "ok" and exits 0 when every call returned its
 * success code; the sanitizers abort on the first invalid access.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

void orc_alpha(int n, double *alpha);
void orc_beta(int n, double *beta);
void orc_assemble(int n, double h, double coef_re, double coef_im, const double *W,
                  cplx *diag, cplx *off);
void orc_mass_apply(int n, double h, const cplx *x, cplx *y);
void orc_genmass_apply(int n, double h, const double *F, const cplx *x, cplx *y);
int orc_thomas(int n, const cplx *diag, const cplx *off, const cplx *rhs, cplx *x);
int orc_mono_cn(int nx, double h, double dt, int nt, int vkind, const double *V,
                const cplx *u0, cplx *uT, cplx *u_all, cplx *v_all,
                int nl_maxit, double nl_tol, int *nl_worst);
int orc_mono_cn_ld(int nx, double h, double dt, int nt, int vkind, const double *V,
                   const cplx *u0, cplx *uT, int nl_maxit, double nl_tol, int *nl_worst);
void orc_end_data(int vkind, const double *V, int nx_global, int g, int nsign, double h,
                  double dt, int nt, double *W, double *dW, double *calW);
void orc_sbar_apply(int kind, int nt, double dt, const cplx *v, const double *W,
                    const double *dW, const double *calW, cplx *out, cplx *out_s);
int orc_sub_sweep(int n, double h, double dt, int nt, int vkind, const double *V,
                  int nx_global, int off0, int left_iface, int right_iface,
                  int trans, double sigma_re, double sigma_im, const double *beta,
                  const cplx *u0, const cplx *hist0, const cplx *l, const cplx *r,
                  cplx *rhoL, cplx *rhoR, cplx *uT, cplx *va, cplx *vb, cplx *v_all,
                  int nl_maxit, double nl_tol, int *nl_worst, int pade_m, double pade_theta);
void orc_pade_coef(int m, double theta, cplx *a, cplx *d);
void orc_pade_eval(int m, double theta, double zr, double zi, double *out);
int orc_pade_apply(int order, int m, double theta, int nt, double dt, const cplx *v,
                   const double *W, const double *dW, cplx *out, cplx *out_s);
int orc_mono_adjoint(int nx, double h, double dt, int nt, const double *V,
                     const cplx *v_all, const cplx *gbar, double *dV, cplx *du0);

static int fails = 0;
#define EXPECT(x) do { if (!(x)) { fprintf(stderr, "failed: %s (line %d)\n", #x, __LINE__); ++fails; } } while (0)

int main(void)
{
    enum { NX = 33, NT = 9, NSUB = 12 };
    const double a0 = -4.0, h = 8.0 / (NX - 1), dt = 0.05;
    double Vs[NX], Vt[(NT + 1) * NX], beta[NT + 70], alpha[NT + 1];
    cplx u0[NX], uT[NX], u_all[(NT + 1) * NX], v_all[NT * NX], du0[NX];
    double dV[NX];
    for (int i = 0; i < NX; ++i) {
        const double x = a0 + i * h;
        Vs[i] = -0.3 * x * x + sin(x);
        u0[i] = cexp(-(x - 0.5) * (x - 0.5) + 1.5 * I * x);
    }
    for (int n = 0; n <= NT; ++n)
        for (int i = 0; i < NX; ++i) Vt[n * NX + i] = 5.0 * cos(n * dt) * (a0 + i * h);
    orc_alpha(NT + 1, alpha);
    orc_beta(NT + 70, beta);

    /* P1 pieces and Thomas */
    cplx diag[NX], off[NX - 1], y[NX], x[NX];
    orc_assemble(NX, h, 0.0, 2.0 / dt, Vs, diag, off);
    orc_mass_apply(NX, h, u0, y);
    orc_genmass_apply(NX, h, Vs, u0, y);
    EXPECT(orc_thomas(NX, diag, off, y, x) == 0);
    EXPECT(orc_thomas(1, diag, off, y, x) == 0);

    /* monodomain: static (all outputs), time dependent, |u|^2; extended precision */
    int worst = 0;
    EXPECT(orc_mono_cn(NX, h, dt, NT, 0, Vs, u0, uT, u_all, v_all, 100, 1e-14, &worst) == 0);
    EXPECT(orc_mono_cn(NX, h, dt, NT, 1, Vt, u0, uT, NULL, NULL, 100, 1e-14, &worst) == 0);
    EXPECT(orc_mono_cn(NX, h, dt, NT, 2, NULL, u0, uT, NULL, v_all, 100, 1e-14, &worst) == 0);
    EXPECT(orc_mono_cn_ld(NX, h, dt, NT, 0, Vs, u0, uT, 100, 1e-17, &worst) == 0);
    EXPECT(orc_mono_cn_ld(NX, h, dt, NT, 1, Vt, u0, uT, 100, 1e-17, &worst) == 0);
    EXPECT(orc_mono_cn_ld(NX, h, dt, NT, 2, NULL, u0, uT, 200, 1e-17, &worst) == 0);

    /* adjoint of the static run */
    EXPECT(orc_mono_cn(NX, h, dt, NT, 0, Vs, u0, uT, NULL, v_all, 100, 1e-14, &worst) == 0);
    EXPECT(orc_mono_adjoint(NX, h, dt, NT, Vs, v_all, uT, dV, du0) == 0);

    /* interface data and Sbar of every operator, static and time dependent */
    double W[NT + 1], dW[NT + 1], calW[NT + 1];
    cplx vend[NT + 1], out[NT + 1], out_s[NT + 1];
    for (int n = 0; n <= NT; ++n) vend[n] = u0[n];
    for (int vk = 0; vk <= 1; ++vk) {
        orc_end_data(vk, vk ? Vt : Vs, NX, NSUB, +1, h, dt, NT, W, dW, calW);
        for (int kind = 1; kind <= 5; ++kind) orc_sbar_apply(kind, NT, dt, vend, W, dW, calW, out, out_s);
        for (int order = 2; order <= 4; order += 2)
            EXPECT(orc_pade_apply(order, 7, M_PI / 4, NT, dt, vend, W, dW, out, out_s) == 0);
    }
    EXPECT(orc_pade_apply(3, 7, M_PI / 4, NT, dt, vend, W, dW, out, out_s) == -5);
    {
        cplx pa[8], pd[8];
        double z[2];
        orc_pade_coef(7, M_PI / 4, pa, pd);
        orc_pade_eval(7, M_PI / 4, 1.0, 2000.0, z);
    }

    /* one subdomain sweep per operator and potential kind: nodes NSUB..NSUB+NSUB
       of the global mesh, both ends interfaces, data, fluxes and every output;
       then a wall-ended sweep without data or fluxes */
    const int n = NSUB + 1;
    cplx l[NT], r[NT], rhoL[NT], rhoR[NT], uTs[NSUB + 1], va[NT + 1], vb[NT + 1], vsub[NT * (NSUB + 1)];
    for (int i = 0; i < NT; ++i) { l[i] = 0.1 * i + 0.2 * I; r[i] = -0.05 * i + 0.1 * I; }
    for (int trans = 0; trans <= 7; ++trans)
        for (int vk = 0; vk <= 2; ++vk) {
            const double *V = vk == 0 ? Vs : (vk == 1 ? Vt : NULL);
            const int rc = orc_sub_sweep(n, h, dt, NT, vk, V, NX, NSUB, 1, 1, trans, 1.0, -1.0, beta,
                                         u0 + NSUB, NULL, l, r, rhoL, rhoR, uTs, va, vb, vsub,
                                         100, 1e-14, &worst, 7, M_PI / 4);
            /* the order-4 operators are refused with |u|^2 */
            EXPECT(rc == (((trans == 3 || trans == 5 || trans == 7) && vk == 2) ? -4 : 0));
        }
    EXPECT(orc_sub_sweep(n, h, dt, NT, 0, Vs, NX, 0, 0, 1, 1, 0.0, 0.0, beta, NULL, NULL, NULL,
                         NULL, NULL, NULL, uTs, NULL, NULL, NULL, 100, 1e-14, &worst, 0, 0.0) == 0);
    EXPECT(orc_sub_sweep(n, h, dt, NT, 0, Vs, NX, NX - n, 1, 0, 1, 0.0, 0.0, beta, NULL, NULL, NULL,
                         NULL, NULL, NULL, uTs, NULL, NULL, NULL, 100, 1e-14, &worst, 0, 0.0) == 0);
    /* a Pade sweep with no auxiliary functions is refused */
    EXPECT(orc_sub_sweep(n, h, dt, NT, 0, Vs, NX, NSUB, 1, 1, 6, 0.0, 0.0, beta, NULL, NULL, NULL,
                         NULL, NULL, NULL, uTs, NULL, NULL, NULL, 100, 1e-14, &worst, 0, 0.0) == -5);
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
