/*
 * FP64 CPU oracle for the ADER-DG hot path (test infrastructure).
 *
 * This is NOT part of the product.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * HIP library: it has its own Gauss-Legendre rule, Lagrange basis, operator
 * tables, PDE fluxes and Riemann solver.
 *
 * What it computes (Dumbser, Fambri, Tavelli, Bader, Weinzierl, "Efficient
 * implementation of ADER discontinuous Galerkin schemes for a scalable
 * hyperbolic PDE engine", 2018):
 *   - PDE class  Q_t + div F(Q) + B(Q).grad Q = S(Q)            (Sec. 2, eq. pde)
 *   - nodal tensor basis on N+1 Gauss-Legendre nodes on [0,1]   (Sec. 2.1, eq. ansatz.uh)
 *   - element-local space-time predictor, Picard iteration       (Sec. 2.2, eqs. spacetime, pde.st2)
 *   - corrector with path-conservative Rusanov jump term         (Sec. 2.1, eqs. pde.nc.gw2, pc.scheme, rusanov)
 *   - CFL time step, alpha = cfl*alpha_N below 1/(2N+1)          (Sec. 3, CFL condition)
 *
 * Layout (shared with the library's public layout, which is part of the
 * interface, not of the arithmetic):
 *   u[e][v][k]      e = ix + nx*(iy + ny*iz),  k = k1 + n*(k2 + n*k3), n = N+1
 *   qhat[e][v][l0][k]   space-time predictor DOFs, l0 = time node
 *
 * Parity status: every function below is pinned by a CPU test (see the
 * oracle tests).  The absolute error values of the isentropic vortex, which
 * the paper quotes from another work without the vortex parameters, final
 * time or error variable, are compared only loosely (density L2 error within
 * a factor of 3 of the printed values at the two coarsest meshes of
 * N = 3, 4, 5, with the parameters the tests assume); their orders are
 * pinned.
 */
#ifndef ADER_ORACLE_H
#define ADER_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXN 8 /* largest n = N+1 */

enum { ORC_EULER = 0, ORC_ELASTIC = 1 };

typedef struct {
  int dim;          /* 2 or 3 (elasticity: 3) */
  int N;            /* polynomial degree, 0..7 */
  int nel[3];       /* elements per axis (nel[2] = 1 when dim = 2) */
  double lo[3], hi[3];
  int pde;          /* ORC_EULER or ORC_ELASTIC */
  double gamma;     /* Euler: ratio of specific heats */
  const double *material; /* ELASTIC: [E][3] = (rho, lambda, mu) */
  int picard;       /* number of Picard sweeps; 0 -> max(1, N+1-guess), 1 for guess 3 */
  double cfl;       /* dt = cfl*alpha_N / max_e sum_d lambda_d/h_d */
  int guess;        /* initial guess of the Picard iteration (Sec. 2.2):
                       0  q0 = u_h(t^n), constant in time;
                       1  second-order MUSCL-Hancock type
                          q0(t) = u + (t - t^n) L(u);
                       2  third-order Taylor type
                          q0(t) = u + (t - t^n) k1 + (t - t^n)^2 (k2 - k1) / (2 dt),
                          k1 = L(u), k2 = L(u + dt k1);
                       3  extrapolation of the previous interval's predictor
                          q_h^{n-1} (a polynomial of degree N in time on
                          [t^{n-1}, t^n]) into [t^n, t^{n+1}], shifted to start
                          at the corrected state:
                          q0(t) = u + q_h^{n-1}(t) - q_h^{n-1}(t^n);
                          without a previous interval (the first step) the
                          constant guess with N+1 sweeps;
                       L = S - div F - B.grad, the collocated right-hand side. */
  int face_avg;     /* face integrals from time-averaged traces (see orc_corrector) */
} orc_problem;

/* Picard sweeps used for a problem: picard, or max(1, N+1-guess), or 1 for
 * guess 3 (with a previous interval; N+1 without one). */
int orc_sweeps(const orc_problem *p);

/* A posteriori detection of troubled elements (Sec. 2.3: the checks that
 * decide which cells the subcell limiter recomputes), on a candidate state
 * u_new after a step from u_old.  flags[e] (host [E]) is a bit set:
 *   1  a value of u_new(e) is NaN or infinite;
 *   2  Euler: rho <= 0 or p <= 0 at a node of u_new(e);
 *   4  relaxed discrete maximum principle violated: for some variable v a
 *      nodal value of u_new(e) lies outside [m - delta, M + delta], where m
 *      and M are the minimum and maximum of the nodal values of u_old over
 *      e and every element sharing a vertex with it (3^d elements,
 *      periodic), and delta = max(1e-4, 1e-3 (M - m)).
 * (Readings: nodal values as the points of the polynomial DMP; the
 * vertex neighbourhood; the constants 1e-4 and 1e-3.)  Returns 0. */
int orc_detect(const orc_problem *p, const double *u_old, const double *u_new, int *flags);

/* 1-D basis on [0,1] (Sec. 2.1). */
int orc_gauss_legendre(int n, double *xi, double *w);
double orc_lagrange(int n, const double *xi, int k, double x);
double orc_lagrange_deriv(int n, const double *xi, int k, double x);
/* Operator tables, all n x n row-major except F0/F1 (length n):
 *   Dhat[k][j] = phi_j'(xi_k); F0[k] = phi_k(0); F1[k] = phi_k(1);
 *   K[j][k] = int phi_j phi_k' = w_j phi_k'(xi_j);  K1 = F1 F1^T - K^T;
 *   T = K1^{-1} W  (time operator of the predictor). */
int orc_operators(int N, double *xi, double *w, double *Dhat, double *F0,
                  double *F1, double *K, double *K1, double *T);

/* Number of variables m of the problem. */
int orc_nvar(const orc_problem *p);
/* Stability coefficient alpha_N of the CFL rule (1-D von Neumann limit of
 * the scheme, rounded down; always below the paper's bound 1/(2N+1) for N>=2). */
double orc_stability_alpha(int N);
/* Unclipped CFL step (Sec. 3): dt = cfl*alpha_N / max_e sum_d lambda_d/h_d.  Returns a negative value when a node is
 * non-finite or non-physical (rho <= 0 or p <= 0). */
double orc_cfl_dt(const orc_problem *p, const double *u);
/* Space-time predictor (Sec. 2.2) for every element; qhat is [E][m][n][n^d].
 * Returns 0 on success. */
int orc_predictor(const orc_problem *p, const double *u, double dt, double *qhat);
/* Picard sweeps actually needed until max|dq| <= tol*max|q| (diagnostic). */
int orc_predictor_converge(const orc_problem *p, const double *u, double dt,
                           double tol, int max_sweeps, double *qhat);
/* Corrector (Sec. 2.1, eq. pde.nc.gw2): unew = u + dt*R(qhat). */
/* With p->face_avg the face integral of every face node is taken from
 * time averages: qbar, the time average of the boundary-extrapolated state,
 * and Fbar, the time average of the flux of that state,
 * sum_l0 w_l0 F(sum_j phi_j(side) q(l0, node j)) (the flux of the trace at
 * each time node, as in the per-time-node integral):
 *   G = 1/2 (Fbar+ + Fbar-).n + 1/2 (int_0^1 B(psi).n ds - s_max I)(qbar+ - qbar-),
 * path and s_max from the averaged states.  For elasticity (no flux; B and
 * s_max depend only on the material) this equals the per-time-node integral. */
int orc_corrector(const orc_problem *p, const double *u, const double *qhat,
                  double dt, double *unew);
/* One full step with dt = min(cfl dt, t_end - t); updates u and *t in place.
 * Returns 0, or -1 on a non-physical state. *dt_out may be NULL. */
int orc_step(const orc_problem *p, double *u, double *t, double t_end, double *dt_out);
/* Predictor with the previous interval's predictor qprev ([E][m][n][n^d],
 * step dtprev) for guess 3; qprev = NULL or dtprev <= 0: no previous
 * interval (constant guess, N+1 sweeps). */
int orc_predictor_hist(const orc_problem *p, const double *u, double dt, const double *qprev,
                       double dtprev, double *qhat);
/* The initial guess alone (no sweep), with the previous interval as in
 * orc_predictor_hist; q0 is [E][m][n][n^d]. */
int orc_guess_hist(const orc_problem *p, const double *u, double dt, const double *qprev, double dtprev,
                   double *q0);
/* orc_step that carries the previous interval for guess 3: qprev
 * ([E][m][n][n^d]) and *dtprev hold it when *has is set; on return they hold
 * this step's predictor and step, and *has is set. */
int orc_step_hist(const orc_problem *p, double *u, double *t, double t_end, double *dt_out, double *qprev,
                  double *dtprev, int *has);
/* Integral of every variable over the domain (Neumaier summation): sums[m]. */
int orc_totals(const orc_problem *p, const double *u, double *sums);
/* Threads the OpenMP runtime will use. */
int orc_num_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
