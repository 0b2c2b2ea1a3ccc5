/*
 * swr.h -- C ABI of the MI355X (gfx950) Schwarz waveform relaxation library
 * for the 1-D Schroedinger equation  i u_t + u_xx + V u = 0  on (a0, b0) with
 * homogeneous Neumann walls (Besse & Xing, arXiv 1503.02564, eq. Schequ).
 *
 * Method (paper Secs. 2-5):
 *   - N non-overlapping subdomains, each solved over the whole time window by
 *     Crank-Nicolson in the v-form of eq. CNS_L with P1 finite elements
 *     (eq. AvML; nonlinear |u|^2: eq. CNS_NL / AvMNL);
 *   - transmission B = dn + S written with fluxes (eq. TransmissionCondlocal)
 *     and exchanged as in eq. TransmissionCond_disc; S is either Robin
 *     (dn u + s u, complex s) or the potential strategy of order 2, S0^2;
 *   - the interface vector g = (r_1 | l_2, r_2 | ... | l_N) of Sec. 3 and the
 *     affine map g -> R g = L g + d (Props. 1-2);
 *   - for time-independent V, L is built from impulse responses (Sec. 4.1;
 *     every block lower-triangular Toeplitz, Props. 3-4) and (I - L) g = d is
 *     solved on the device (Sec. 4 "New algorithm");
 *   - for V(t,x) and |u|^2 the iteration is preconditioned by P = I - L_0,
 *     L_0 the interface operator of the zero potential (Sec. 5).
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer (e.g. torch .data_ptr()) unless
 *     marked "host".  Complex arrays are interleaved FP64 (re, im) pairs, i.e.
 *     double[2] per entry (torch.complex128 / std::complex<double>).
 *   - The caller owns every argument buffer.  The library copies what it
 *     needs at setup (potential, mesh tables) into device memory it owns until
 *     swr_destroy.  Outputs are written asynchronously on the context's stream;
 *     the call returns after the last host read-back it needs (convergence
 *     scalars), so outputs are complete when the stream is synchronised.
 *   - Mesh: uniform, nc = sum(J) cells, h = (b0 - a0)/nc, nodes x_i = a0 + i h,
 *     nx = nc + 1.  Subdomain k (0-based) owns nodes o_k .. o_k + J_k with
 *     o_0 = 0, o_{k+1} = o_k + J_k; the node shared by two subdomains is
 *     duplicated internally and reported as the average of the two sides.
 *   - Time: nt = round(T/dt) steps; V(t,x) rows are t_n = n dt, n = 0..nt.
 *   - Interface vectors g are [B][2N-2][nt]: slot 2k-1 holds l_k (k >= 1),
 *     slot 2k holds r_k (k <= N-2); entry n-1 of a slot is time step n.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - With SWR_DEBUG set in the environment a failing HIP call is reported on
 *     stderr (call, source line, HIP error name) before SWR_EDEVICE is returned;
 *     with SWR_DEBUG_POISON set, every device buffer the library allocates is
 *     filled with all-ones bytes (NaN as a double) when it is allocated, so a
 *     read before the first write shows in the results.
 *   - Errors are status codes; nothing is thrown across the ABI.  After any
 *     status other than SWR_OK or SWR_ENOCONV the context remains valid for
 *     swr_destroy.
 */
#ifndef SWR_H
#define SWR_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct swr_ctx swr_ctx;

typedef enum {
    SWR_OK = 0,
    SWR_EINVAL = 1,   /* invalid argument (see swr_setup / each call) */
    SWR_ENOMEM = 2,   /* device allocation failed */
    SWR_EDEVICE = 3,  /* a HIP call or kernel launch failed */
    SWR_ENOCONV = 4,  /* iteration limit reached; outputs hold the last iterate */
    SWR_ENAN = 5      /* NaN/Inf met in the interface residual */
} swr_status;

/* transmission operator S of B = dn + S (Sec. 2.1), discretised as in Sec. 2.2:
 *   SWR_ROBIN  S = s (the complex s_re + i s_im of swr_setup)
 *   SWR_S02    potential strategy, order 2: e^{-i pi/4} d_t^{1/2}
 *   SWR_S03    order 3: S0^2 - e^{i pi/4} (W/2) I_t^{1/2}
 *   SWR_S04    order 4: S0^3 - i (dn W / 4) I_t
 *   SWR_S12    gauge change strategy, order 2: e^{-i pi/4} e^{i calW} d_t^{1/2} e^{-i calW}
 *   SWR_S14    order 4: S1^2 - i sgn(dn W) (|dn W|^{1/2}/2) e^{i calW} I_t (|dn W|^{1/2}/2) e^{-i calW}
 *   SWR_P22    Pade approximation strategy, order 2: -i sqrt(i d_t + W) with the square
 *              root replaced by sum_{s=0}^m a_s - sum_{s=1}^m a_s d_s / (z + d_s), applied
 *              through m auxiliary functions per interface end (Sec. 2.2); a_s, d_s are the
 *              partial fractions of the diagonal [m/m] Pade approximant of sqrt(1 + w) with
 *              the branch cut rotated by theta (opts.pade_m, opts.pade_theta)
 *   SWR_P24    order 4: S2^2 + sgn(dn W) (|dn W|^{1/2}/2) (i d_t + W)^{-1} (|dn W|^{1/2}/2)
 *              (one more auxiliary function)
 * W is the potential at the interface node, dn W its outward normal derivative
 * (centred difference on the mesh), calW the gauge phase (time integral of V by
 * the trapezoid rule, averaged over the two ends of the step); with V(t,x) all of
 * them follow W_n = (V_n + V_{n-1})/2 step by step; with |u|^2 (SWR_V_CUBIC)
 * W_n = |v_{n-1}|^2 at the end node (the inner fixed point's starting value) and
 * the order-4 operators S04, S14, P24 are refused (they carry dn f(u)).  The
 * order-4 terms flip sign with the normal and cancel in the exchange, which
 * transmits S without them. */
typedef enum {
    SWR_ROBIN = 0, SWR_S02 = 1, SWR_S03 = 2, SWR_S04 = 3, SWR_S12 = 4, SWR_S14 = 5,
    SWR_P22 = 6, SWR_P24 = 7
} swr_transmission;

/* potential: static V(x) [nx] | time dependent V(t,x) [nt+1][nx] | |u|^2 (V NULL) */
typedef enum { SWR_V_STATIC = 0, SWR_V_TIME = 1, SWR_V_CUBIC = 2 } swr_vkind;

/* interface solver */
typedef enum {
    SWR_SOLVER_FIXED = 0,   /* fixed point g <- R g (Sec. 4 "Classical algorithm") */
    SWR_SOLVER_GMRES = 1,   /* restarted GMRES on (I - L) g = d (Sec. 4) */
    SWR_SOLVER_CAUSAL = 2,  /* exact forward substitution in time on (I - L) g = d; offered up to
                               512 interface slots, or 513 subdomains when the per-step block
                               system is block diagonally dominant (block PCR).  Beyond that the
                               same system is solved by BiCGStab, and P^{-1} of the V_TIME /
                               V_CUBIC iterations by an inner BiCGStab to relative residual
                               1e-13 (the paper's way of applying P^{-1}, Sec. 5) */
    SWR_SOLVER_BICGSTAB = 3 /* BiCGStab on (I - L) g = d (the Krylov solver of Sec. 6) */
} swr_solver;

typedef struct {
    double tol;        /* FIXED: max |g^{k+1} - g^k| < tol; GMRES, BICGSTAB: ||d - (I-L)g||_2 <= tol ||d||_2;
                          |u|^2 preconditioned fixed point: max |g^{k+1} - g^k| <
                          tol max(1, max |g^{k+1}|) (per problem).  default 1e-10 */
    int max_iter;      /* iteration cap (default 20000) */
    int restart;       /* GMRES restart length m (default 30) */
    int solver;        /* swr_solver (default SWR_SOLVER_CAUSAL) */
    int precond;       /* V_TIME / V_CUBIC: 1 = precondition with P = I - L_0 (default 1) */
    int batch;         /* B independent problems sharing mesh and transmission (default 1) */
    int v_per_problem; /* V_STATIC only: V is [B][nx], one potential per problem (default 0) */
    int checkpoint_K;  /* adjoint checkpoint interval in steps (default 64) */
    int nl_max_iter;   /* |u|^2 inner fixed point cap per step (default 100) */
    double nl_tol;     /* |u|^2 inner fixed point tolerance (default 1e-14) */
    int pipeline;      /* static V with SWR_SOLVER_CAUSAL: cut the time window into chunks of
                          this many steps (a multiple of 64) and overlap the impulse/d sweeps,
                          the interface solve and the final sweep chunk by chunk on two extra
                          internal streams (joined back to the context's stream before the call
                          returns); 0 = one stage after the other; -1 = chosen by the library
                          (default): 256; a tuning-cache entry (tune_cache) overrides the
                          choice */
    int plain;         /* 1 = launch the subdomain sweeps one task (one subdomain of one problem)
                          per launch on the context's stream, staged: the unbatched form, for
                          comparison with the batched launches (default 0) */
    int snapshot_stride; /* > 0: swr_solve may return u(t_n, x) at n = 0, s, 2s, ... <= nt
                            (s = this stride) in its snaps argument; 0 = no snapshots (default 0) */
    const char* tune_cache; /* host path of the schedule cache written by swr_tune and read by
                               swr_setup (NULL = no cache, built-in schedule; default NULL) */
    int pade_m;        /* SWR_P22 / SWR_P24: auxiliary functions per interface end, 1..128
                          (default 20; the paper runs 20, 50 and 100) */
    double pade_theta; /* SWR_P22 / SWR_P24: rotation of the square root's branch cut in
                          (0, pi) (default pi/4) */
} swr_opts;

typedef struct {
    int iters;          /* interface iterations (FIXED/GMRES), 1 for CAUSAL */
    double residual;    /* certified ||g - R g||_2 / ||R 0||_2 of the final sweep
                           (max over the batch); FIXED: last max change */
    double t_factor_ms; /* assembly + factorisation */
    double t_build_ms;  /* impulse sweeps and d (Sec. 4.1); with opts.pipeline the three
                           phases overlap and each figure is the span of its own stream */
    double t_iface_ms;  /* interface solve */
    double t_final_ms;  /* final sweep and u(T) */
    int nl_worst;       /* |u|^2: largest inner iteration count */
    double t_total_ms;  /* the whole call on the device, factorisation to u(T) */
    double t_sweep_ms;  /* static V, new algorithm: summed durations of the subdomain sweep
                           launches (impulse/d sweeps and final sweep) ... */
    int n_sweep;        /* ... and their number (0 when not measured) */
    int inner_iters;    /* V_TIME / V_CUBIC with more interfaces than the causal solve takes:
                           total inner BiCGStab iterations spent applying P^{-1} (else 0) */
    const double* history; /* host array owned by the context, valid until the next call on it:
                              the convergence measure after every interface iteration (max over
                              the batch): GMRES / BiCGStab relative residual estimate, fixed
                              point max trace change, causal solve the certified residual */
    int history_len;    /* entries of history */
} swr_info;

/* A schedule: parameters that change how the work is launched, not what is
 * computed (results are bitwise the same for every pipeline chunk and helper
 * bound; the GMRES restart changes the iterate, not the tolerance met). */
typedef struct {
    int pipeline;     /* pipeline chunk of the static causal solve, 0 = staged */
    int help_max;     /* S0^2 sweeps: launches of at most this many tasks give every task a
                         second wave that sums the far boundary history */
    int restart;      /* GMRES restart length */
    int pair_from;    /* static Robin / S0^2 sweeps: launches that fill the GPU with one-wave
                         tasks run two tasks of one subdomain per wave from this chunk width
                         (ceil((J_k + 1) / 64) nodes per lane) on; 9 = never (default) */
    int graph;        /* static causal solve: 1 = from the second solve with the same potential,
                         output pointers and schedule, replay the whole solve as one HIP graph
                         captured on the context's streams (bitwise the same results; no
                         per-stage timings in swr_info); 0 = launch kernel by kernel (default) */
    int check;        /* GMRES: read the inner residual estimates back every this many steps
                         (default 4); the iterate and the iteration count are those of a check
                         after every step, the steps between reads need no host round trip */
    int group;        /* static Robin / S0^2 sweeps: launches that fill the GPU with one-wave
                         tasks run up to this many tasks of one subdomain and one potential (the
                         problems of a batch) as the waves of one workgroup, reading one LDS
                         copy of the subdomain's factors; 1..8, 1 = one task per workgroup
                         (default 4); bitwise the same results */
    double ms;        /* swr_tune: wall time of the chosen schedule's solve */
    int candidates;   /* swr_tune: schedules timed */
} swr_schedule;

/* Fill *o with the defaults listed above. */
void swr_default_opts(swr_opts* o);

/* Create a context.
 *   a0 < b0: the domain.  N >= 1 subdomains with J[k] >= 1 cells each (J: host
 *   array of N ints).  dt > 0, T > 0 with T/dt an integer to 1e-9 relative.
 *   vk: potential kind; V: device array [nx] (STATIC), [B][nx] (STATIC with
 *   opts->v_per_problem), [nt+1][nx] (TIME), or NULL (CUBIC; also allowed for
 *   STATIC, meaning V = 0).  tr: transmission (swr_transmission); s_re + i s_im
 *   is the Robin coefficient s of dn u + s u (ignored otherwise; must be
 *   nonzero for Robin).
 *   opts: NULL for defaults.  stream: hipStream_t the work is enqueued on
 *   (NULL = default stream).  *out receives the context.
 * Errors: SWR_EINVAL for any violated condition above, tr beyond SWR_S02 with
 * a potential that is not STATIC, a nonzero-size
 * subdomain larger than the kernel's node bound (512 nodes per subdomain),
 * batch < 1, or CUBIC combined with batch > 1 problems of different V;
 * SWR_ENOMEM / SWR_EDEVICE on allocation / launch failure. */
swr_status swr_setup(double a0, double b0, int N, const int* J, double dt, double T,
                     int vk, const double* V, int tr, double s_re, double s_im,
                     const swr_opts* opts, void* stream, swr_ctx** out);

/* Solve the B problems with initial data u0 [B][nx] complex.
 * Static V: Sec. 4 "New algorithm" -- factorise, impulse sweeps for L and the
 * d sweep (one launch), interface solve by opts.solver, final sweep.  V(t,x) /
 * |u|^2: Sec. 5 preconditioned iteration.  Outputs: uT [B][nx] complex
 * (required); g [B][2N-2][nt] converged interface vector (NULL to skip);
 * utrace [B][N][2][nt+1]: u_n at the left/right end node of every subdomain,
 * n = 0..nt (NULL to skip); snaps [B][S][nx] complex with S = nt/s + 1
 * (integer division, s = opts.snapshot_stride): u(t_n, x) at n = 0, s, 2s, ...
 * from the final sweep, the node shared by two subdomains the average of the
 * two sides as in uT (NULL to skip; SWR_EINVAL when given with a stride of 0).
 * info: host struct (NULL to skip).
 * Returns SWR_ENOCONV if the solver hit max_iter (outputs hold the last
 * iterate), SWR_ENAN on a non-finite residual. */
swr_status swr_solve(swr_ctx* ctx, const double* u0, double* uT, double* g, double* utrace,
                     double* snaps, swr_info* info);

/* Gradient of a real objective J(u(T)) with respect to the static potential
 * and the initial data, by the discrete adjoint of the Crank-Nicolson scheme
 * solved through the same decomposition (STATIC potential only; the adjoint
 * uses the same interface operator L as the forward).
 *   u0 [B][nx] complex; gbar [B][nx] complex upstream gradient
 *   dJ/dRe u(T) + i dJ/dIm u(T) (for J = sum |u(T) - u*|^2 it is 2(u(T) - u*)).
 *   dJdV [B][nx] real (per problem; with a shared V sum over the batch),
 *   dJdu0 [B][nx] complex (same convention).
 * The call runs the forward solve (final sweep checkpointing u every 64 steps
 * counted back from nt), the adjoint interface problem, and one adjoint sweep
 * that replays each 64-step forward segment from its checkpoint and consumes
 * it in reverse.  opts.checkpoint_K must be 64, the solver not FIXED and the
 * transmission Robin or S0^2 (SWR_EINVAL otherwise).  info: iters / residual of the adjoint interface
 * solve; t_factor_ms = whole forward, t_build_ms = adjoint d sweep,
 * t_iface_ms = adjoint interface solve, t_final_ms = replay + adjoint sweep. */
swr_status swr_grad(swr_ctx* ctx, const double* u0, const double* gbar, double* dJdV,
                    double* dJdu0, swr_info* info);

/* ---- step-level entry points (each one row of the hot path) ------------ */

/* One SWR iteration for all B problems (Sec. 3, eq. interfacepbR):
 * g_out = R g_in, i.e. every subdomain swept with the fluxes of g_in and the
 * data u0 (NULL = zero data and zero history, which gives g_out = L g_in).
 * g_in, g_out: [B][2N-2][nt]; must not overlap.  uT [B][nx] (NULL to skip)
 * receives u(T) of this sweep.  maxdiff (host, NULL to skip) receives
 * max |g_out - g_in|. */
swr_status swr_apply_R(swr_ctx* ctx, const double* u0, const double* g_in, double* g_out,
                       double* uT, double* maxdiff);

/* swr_apply_R for callers that cannot allocate device memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same sweeps and the same results as swr_apply_R, but its
 * scratch -- the S0^2 boundary history of every (problem, subdomain) sweep,
 * the end values of u(T) and the max-change word -- is a fixed 16 MiB device
 * array of the library (one copy per GPU, held until the process ends) instead
 * of context memory; the call allocates nothing, never synchronises and enqueues
 * only kernels on the context's stream.  maxdiff is a DEVICE double (NULL to
 * skip) that receives max |g_out - g_in| when the stream reaches it.
 * Requires 256 + 16 (B N 2 + B N 2 (nt + 1)) bytes <= 16 MiB (the history term
 * only for the convolution-type transmissions); SWR_EINVAL beyond, and for the
 * argument errors of swr_apply_R.  All calls on one GPU share the array: calls
 * that overlap in time on one GPU (other streams, other threads) race and
 * corrupt each other's results. */
swr_status swr_apply_R_noalloc(swr_ctx* ctx, const double* u0, const double* g_in, double* g_out,
                               double* uT, double* maxdiff);

/* Build the explicit interface problem (Sec. 4.1, static V): impulse sweeps
 * give the first columns of all blocks X^{k,p}, cols [nv][N][4][nt] (p = 0..3
 * for X^{k,1..4}; entries of absent blocks are left untouched), and
 * d = R 0 [B][2N-2][nt] from the data u0.  Either output may be NULL. */
swr_status swr_build_interface(swr_ctx* ctx, const double* u0, double* cols, double* d);

/* y = x - L x for [B][2N-2][nt] vectors with L from the last build: the
 * operator of the interface problem (I - L) g = d (Sec. 4, "New algorithm";
 * the matrix its Krylov solvers iterate with), L applied block by block as
 * lower-triangular Toeplitz products fixed by the impulse-response first
 * columns (Props. 3-4, Sec. 4.1).  Static V: L of the potential; V(t,x) and
 * |u|^2: L_0 of the zero potential (Sec. 5).  x and y must not overlap. */
swr_status swr_interface_matvec(swr_ctx* ctx, const double* x, double* y);

/* Replace the potential of a context (same layout as the V of swr_setup:
 * [nx], [B][nx] with v_per_problem, or [nt+1][nx] for V_TIME); the next
 * solve refactorises and rebuilds the interface problem.  SWR_EINVAL for a
 * cubic context or a NULL V. */
swr_status swr_set_potential(swr_ctx* ctx, const double* V);

/* The autotuner: times candidate schedules (pipeline chunks 0, 128, 256, 512,
 * 1024 for the static causal solve; helper-wave bounds 0, 512, all for S0^2;
 * two-task waves from widths 1, 4 or never for static Robin / S0^2 sweeps;
 * graph replay on and off for the static causal solve; restarts 20, 30, 60,
 * 120 and residual read-back periods 1, 4, 16 for GMRES and the V(t,x)
 * iteration) with full
 * solves of the caller's u0 [B][nx] (one warm-up and the best of two timed
 * solves each), until budget_ms of wall time is spent, and keeps the fastest
 * on the context.  With opts.tune_cache the choice is written to that file
 * under a key of the problem's shape (sizes, batch, potential kind,
 * transmission, solver) and applied by every later swr_setup of the same
 * shape.  chosen (host, NULL to skip) receives it.  May allocate; synchronises.
 * SWR_EINVAL on bad arguments or an unwritable cache file, SWR_ENOCONV when no
 * candidate solve converged. */
swr_status swr_tune(swr_ctx* ctx, const double* u0, double budget_ms, swr_schedule* chosen);

/* The schedule a context runs with (host out). */
swr_status swr_get_schedule(const swr_ctx* ctx, swr_schedule* s);

/* Set the schedule of a context (host in; ms and candidates are ignored).
 * SWR_EINVAL for a pipeline chunk that is negative or not a multiple of 64, a
 * negative helper bound, a restart, pair width or check period below 1. */
swr_status swr_set_schedule(swr_ctx* ctx, const swr_schedule* s);

/* Release the context and all device memory it owns. */
void swr_destroy(swr_ctx* ctx);

/* Static description of a status code. */
const char* swr_strerror(swr_status s);

/* Sizes of a context (host ints, each pointer may be NULL): time steps nt,
 * global nodes nx, problems B, potentials nv (B with opts.v_per_problem, else
 * 1), subdomains N, the potential kind vk (swr_vkind) and the snapshot count S
 * of swr_solve (0 without opts.snapshot_stride).  They fix the element counts
 * of every array argument above. */
swr_status swr_sizes(const swr_ctx* ctx, int* nt, int* nx, int* B, int* nv, int* N, int* vk,
                     int* S);

#ifdef __cplusplus
}
#endif
#endif /* SWR_H */
