/*
 * FP64 CPU oracle of the ADER-DG hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct C99: one element at a time, every sum
 * written out as a loop, no blocking or fusion beyond what the paper's
 * formulas state.  OpenMP only distributes whole elements over threads.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library; the HIP library never does.
 *
 * Paper: Dumbser et al., "Efficient implementation of ADER discontinuous
 * Galerkin schemes for a scalable hyperbolic PDE engine" (2018).
 * Readings where the paper is silent or garbled are marked "reading:".
 */
#include "ader_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXM 9

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Thread count of the OpenMP loops (timing of the oracle only). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* 1-D basis (Sec. 2.1, paragraph after eq. ansatz.uh): Lagrange        */
/* polynomials through the N+1 Gauss-Legendre nodes of [0,1].           */
/* ------------------------------------------------------------------ */

/* Legendre P_n(z) and P_n'(z) by the three-term recurrence. */
static void legendre(int n, double z, double *pn, double *dpn) {
  double p_prev = 1.0, p = z;
  if (n == 0) {
    *pn = 1.0;
    *dpn = 0.0;
    return;
  }
  for (int j = 2; j <= n; j++) {
    double p_next = ((2.0 * j - 1.0) * z * p - (j - 1.0) * p_prev) / j;
    p_prev = p;
    p = p_next;
  }
  *pn = p;
  *dpn = n * (z * p - p_prev) / (z * z - 1.0);
}

/* Gauss-Legendre nodes (ascending) and weights on [0,1]: Newton's method on
 * the roots of P_n in [-1,1], then the affine map z -> (1-z)/2. */
int orc_gauss_legendre(int n, double *xi, double *w) {
  if (n < 1 || n > 64) return -1;
  for (int i = 0; i < n; i++) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double pn, dpn;
    for (int it = 0; it < 100; it++) {
      legendre(n, z, &pn, &dpn);
      double dz = pn / dpn;
      z -= dz;
      if (fabs(dz) < 1e-15) break;
    }
    legendre(n, z, &pn, &dpn);
    xi[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dpn * dpn); /* = (2/((1-z^2)P'^2)) / 2 */
  }
  return 0;
}

double orc_lagrange(int n, const double *xi, int k, double x) {
  double r = 1.0;
  for (int j = 0; j < n; j++)
    if (j != k) r *= (x - xi[j]) / (xi[k] - xi[j]);
  return r;
}

/* Product rule applied to prod_{j!=k} (x - xi_j)/(xi_k - xi_j). */
double orc_lagrange_deriv(int n, const double *xi, int k, double x) {
  double s = 0.0;
  for (int i = 0; i < n; i++) {
    if (i == k) continue;
    double term = 1.0 / (xi[k] - xi[i]);
    for (int j = 0; j < n; j++)
      if (j != k && j != i) term *= (x - xi[j]) / (xi[k] - xi[j]);
    s += term;
  }
  return s;
}

/* Solve A X = B for X (n x n, row-major) by Gauss-Jordan elimination with
 * partial pivoting.  A and B are overwritten. */
static int solve_dense(int n, double *A, double *B) {
  for (int c = 0; c < n; c++) {
    int piv = c;
    for (int r = c + 1; r < n; r++)
      if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return -1;
    if (piv != c)
      for (int j = 0; j < n; j++) {
        double t = A[c * n + j]; A[c * n + j] = A[piv * n + j]; A[piv * n + j] = t;
        t = B[c * n + j]; B[c * n + j] = B[piv * n + j]; B[piv * n + j] = t;
      }
    double d = A[c * n + c];
    for (int j = 0; j < n; j++) {
      A[c * n + j] /= d;
      B[c * n + j] /= d;
    }
    for (int r = 0; r < n; r++) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; j++) {
        A[r * n + j] -= f * A[c * n + j];
        B[r * n + j] -= f * B[c * n + j];
      }
    }
  }
  return 0;
}

/* Operators of the scheme.  The time operator comes from the predictor's
 * weak form (eq. pde.st2) after the time integration by parts: with the
 * collocated right-hand side R at the space-time nodes, the coefficients of
 * one spatial node obey  K1 q = F0 u + dt W R,  K1 = F1 F1^T - K^T, hence
 * q = K1^{-1} F0 u + dt T R with T = K1^{-1} W (and K1^{-1} F0 = 1). */
int orc_operators(int N, double *xi, double *w, double *Dhat, double *F0,
                  double *F1, double *K, double *K1, double *T) {
  int n = N + 1;
  if (N < 0 || n > ORC_MAXN) return -1;
  orc_gauss_legendre(n, xi, w);
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++) Dhat[k * n + j] = orc_lagrange_deriv(n, xi, j, xi[k]);
  for (int k = 0; k < n; k++) {
    F0[k] = orc_lagrange(n, xi, k, 0.0);
    F1[k] = orc_lagrange(n, xi, k, 1.0);
  }
  /* K[j][k] = int_0^1 phi_j phi_k' dxi, exact with the n-point rule. */
  for (int j = 0; j < n; j++)
    for (int k = 0; k < n; k++) K[j * n + k] = w[j] * Dhat[j * n + k];
  for (int a = 0; a < n; a++)
    for (int b = 0; b < n; b++) K1[a * n + b] = F1[a] * F1[b] - K[b * n + a];
  double A[ORC_MAXN * ORC_MAXN], B[ORC_MAXN * ORC_MAXN];
  memcpy(A, K1, sizeof(double) * n * n);
  for (int a = 0; a < n; a++)
    for (int b = 0; b < n; b++) B[a * n + b] = (a == b) ? w[a] : 0.0;
  if (solve_dense(n, A, B)) return -2;
  memcpy(T, B, sizeof(double) * n * n);
  return 0;
}

/* ------------------------------------------------------------------ */
/* PDE systems (Sec. 3.1 Euler; Sec. 3.2 elasticity with alpha = 1).    */
/* ------------------------------------------------------------------ */

int orc_nvar(const orc_problem *p) {
  return p->pde == ORC_EULER ? p->dim + 2 : 9;
}

/* Euler, eq. euler: state (rho, rho v, rho E), ideal gas
 * p = (gamma-1)(rho E - rho |v|^2 / 2). */
static void euler_flux(int d, double gamma, const double *q, int a, double *F) {
  double rho = q[0];
  double ke = 0.0;
  for (int i = 0; i < d; i++) ke += q[1 + i] * q[1 + i];
  ke = 0.5 * ke / rho;
  double pr = (gamma - 1.0) * (q[d + 1] - ke);
  double va = q[1 + a] / rho;
  F[0] = q[1 + a];
  for (int i = 0; i < d; i++) F[1 + i] = q[1 + i] * va + (i == a ? pr : 0.0);
  F[d + 1] = (q[d + 1] + pr) * va;
}

static double euler_pressure(int d, double gamma, const double *q) {
  double ke = 0.0;
  for (int i = 0; i < d; i++) ke += q[1 + i] * q[1 + i];
  return (gamma - 1.0) * (q[d + 1] - 0.5 * ke / q[0]);
}

/* Largest |eigenvalue| of dF_a/dQ: |v_a| + c, c = sqrt(gamma p / rho). */
static double euler_speed(int d, double gamma, const double *q, int a) {
  double pr = euler_pressure(d, gamma, q);
  return fabs(q[1 + a] / q[0]) + sqrt(gamma * pr / q[0]);
}

/* Linear elasticity in velocity-stress form (eqs. 3.00-3.1 with alpha = 1):
 *   v_t - (1/rho) div sigma = 0,
 *   sigma_t - lambda (div v) I - mu (grad v + grad v^T) = 0,
 * written as B(Q).grad Q.  Variables: (u, v, w, sxx, syy, szz, sxy, syz, sxz).
 * grad[a][c] = d q_c / d x_a.  out = B(Q).grad Q. */
static const int SIG[3][3] = {{3, 6, 8}, {6, 4, 7}, {8, 7, 5}};
static void elastic_ncp(const double *mat, const double grad[3][MAXM], double *out) {
  double rho = mat[0], lam = mat[1], mu = mat[2];
  for (int i = 0; i < 3; i++) {
    double divs = 0.0;
    for (int j = 0; j < 3; j++) divs += grad[j][SIG[i][j]];
    out[i] = -divs / rho;
  }
  double divv = grad[0][0] + grad[1][1] + grad[2][2];
  for (int i = 0; i < 3; i++)
    for (int j = i; j < 3; j++) {
      double s = mu * (grad[i][j] + grad[j][i]);
      if (i == j) s += lam * divv;
      out[SIG[i][j]] = -s;
    }
}

static double elastic_speed(const double *mat) {
  return sqrt((mat[1] + 2.0 * mat[2]) / mat[0]); /* c_p */
}

typedef struct {
  int d, n, m, nd, nst, E;
  int str[3];    /* node stride of axis a inside an element: n^a */
  double h[3];
  double xi[ORC_MAXN], w[ORC_MAXN], Dhat[ORC_MAXN * ORC_MAXN];
  double F0[ORC_MAXN], F1[ORC_MAXN], K[ORC_MAXN * ORC_MAXN];
  double K1[ORC_MAXN * ORC_MAXN], T[ORC_MAXN * ORC_MAXN];
  double gx[3], gw[3]; /* 3-point Gauss-Legendre rule for the path integral */
} setup_t;

static int setup(const orc_problem *p, setup_t *s) {
  if (p->dim < 1 || p->dim > 3 || p->N < 0 || p->N + 1 > ORC_MAXN) return -1;
  if (p->guess < 0 || p->guess > 3) return -1;
  if (p->pde == ORC_ELASTIC && (p->dim != 3 || !p->material)) return -1;
  s->d = p->dim;
  s->n = p->N + 1;
  s->m = orc_nvar(p);
  s->nd = 1;
  s->E = 1;
  for (int a = 0; a < s->d; a++) {
    s->str[a] = s->nd;
    s->nd *= s->n;
    s->E *= p->nel[a];
    s->h[a] = (p->hi[a] - p->lo[a]) / p->nel[a];
  }
  s->nst = s->nd * s->n;
  if (orc_operators(p->N, s->xi, s->w, s->Dhat, s->F0, s->F1, s->K, s->K1, s->T)) return -1;
  orc_gauss_legendre(3, s->gx, s->gw);
  return 0;
}

static const double *elem_mat(const orc_problem *p, int e) {
  return p->pde == ORC_ELASTIC ? p->material + 3 * (size_t)e : NULL;
}

static void pde_flux(const orc_problem *p, const setup_t *s, const double *q, int a, double *F) {
  if (p->pde == ORC_EULER) euler_flux(s->d, p->gamma, q, a, F);
  else for (int v = 0; v < s->m; v++) F[v] = 0.0;
}

/* B(Q).grad Q for gradient grad[a][v]. */
static void pde_ncp(const orc_problem *p, const setup_t *s, const double *q, const double *mat,
                    const double grad[3][MAXM], double *out) {
  (void)q;
  if (p->pde == ORC_ELASTIC) elastic_ncp(mat, grad, out);
  else for (int v = 0; v < s->m; v++) out[v] = 0.0;
}

static double pde_speed(const orc_problem *p, const setup_t *s, const double *q, const double *mat, int a) {
  if (p->pde == ORC_EULER) return euler_speed(s->d, p->gamma, q, a);
  return elastic_speed(mat);
}

/* Algebraic source S(Q): zero for both systems of this library. */
static void pde_source(const orc_problem *p, const setup_t *s, const double *q, double *S) {
  (void)p; (void)q;
  for (int v = 0; v < s->m; v++) S[v] = 0.0;
}

/* Path-conservative jump term of eq. pc.scheme for an element face with
 * outward normal n = sgn * e_a, inside state qm (q_h^-) and outside state
 * qp (q_h^+):
 *   D^- . n = 1/2 (F(qp) + F(qm)).n + 1/2 ( int_0^1 B(psi).n ds - Theta ) (qp - qm),
 * straight-line path psi(s) = qm + s (qp - qm), 3-point Gauss-Legendre rule
 * for the path integral, Rusanov Theta = s_max I with s_max the larger
 * |eigenvalue| of A.n on the two sides (eq. rusanov).
 * Reading (material across a face): the material parameters are carried
 * along the same straight path as the state. */
static void dminus(const orc_problem *p, const setup_t *s, const double *qm, const double *qp,
                   const double *matm, const double *matp, int a, double sgn, double *D) {
  int m = s->m;
  double Fm[MAXM], Fp[MAXM], dq[MAXM], path[MAXM];
  pde_flux(p, s, qm, a, Fm);
  pde_flux(p, s, qp, a, Fp);
  for (int v = 0; v < m; v++) {
    dq[v] = qp[v] - qm[v];
    path[v] = 0.0;
  }
  if (p->pde == ORC_ELASTIC) {
    for (int g = 0; g < 3; g++) {
      double psi[MAXM], matg[3], grad[3][MAXM], out[MAXM];
      for (int v = 0; v < m; v++) psi[v] = qm[v] + s->gx[g] * dq[v];
      for (int c = 0; c < 3; c++) matg[c] = matm[c] + s->gx[g] * (matp[c] - matm[c]);
      /* B(psi).n dq is B.grad with the gradient n (x) dq. */
      for (int b = 0; b < 3; b++)
        for (int v = 0; v < m; v++) grad[b][v] = (b == a) ? sgn * dq[v] : 0.0;
      pde_ncp(p, s, psi, matg, grad, out);
      for (int v = 0; v < m; v++) path[v] += s->gw[g] * out[v];
    }
  }
  double smax = fmax(pde_speed(p, s, qm, matm, a), pde_speed(p, s, qp, matp, a));
  for (int v = 0; v < m; v++)
    D[v] = 0.5 * (Fp[v] + Fm[v]) * sgn + 0.5 * (path[v] - smax * dq[v]);
}

/* The jump term from time-averaged traces qm, qp and time-averaged
 * fluxes Fm, Fp (face_avg): the same formula as dminus with the averaged
 * quantities; the path and s_max come from the averaged states. */
static void dminus_avg(const orc_problem *p, const setup_t *s, const double *qm, const double *qp,
                       const double *Fm, const double *Fp, const double *matm, const double *matp,
                       int a, double sgn, double *D) {
  int m = s->m;
  double dq[MAXM], path[MAXM];
  for (int v = 0; v < m; v++) {
    dq[v] = qp[v] - qm[v];
    path[v] = 0.0;
  }
  if (p->pde == ORC_ELASTIC) {
    for (int g = 0; g < 3; g++) {
      double psi[MAXM], matg[3], grad[3][MAXM], out[MAXM];
      for (int v = 0; v < m; v++) psi[v] = qm[v] + s->gx[g] * dq[v];
      for (int c = 0; c < 3; c++) matg[c] = matm[c] + s->gx[g] * (matp[c] - matm[c]);
      for (int b = 0; b < 3; b++)
        for (int v = 0; v < m; v++) grad[b][v] = (b == a) ? sgn * dq[v] : 0.0;
      pde_ncp(p, s, psi, matg, grad, out);
      for (int v = 0; v < m; v++) path[v] += s->gw[g] * out[v];
    }
  }
  double smax = fmax(pde_speed(p, s, qm, matm, a), pde_speed(p, s, qp, matp, a));
  for (int v = 0; v < m; v++)
    D[v] = 0.5 * (Fp[v] + Fm[v]) * sgn + 0.5 * (path[v] - smax * dq[v]);
}

/* ------------------------------------------------------------------ */
/* Space-time predictor (Sec. 2.2).                                     */
/* ------------------------------------------------------------------ */

static int axis_index(const setup_t *s, int k, int a) { return (k / s->str[a]) % s->n; }

/* Collocated right-hand side of the predictor at every space-time node of
 * one element (reading: the flux divergence is the derivative of the nodal
 * interpolant of F, and the sign is -div F as in eq. pde; the printed "+"
 * in eq. pde.st2 contradicts eq. pde and the operator L that follows it):
 *   R = S(q) - sum_a (1/h_a) Dhat_a F_a(q) - B(q) . sum_a (1/h_a) Dhat_a q.
 * q, R are [m][n][nd]; F is scratch [3][m][n*nd]. */
static void predictor_rhs(const orc_problem *p, const setup_t *s, const double *mat,
                          const double *q, double *F, double *R) {
  int m = s->m, nd = s->nd, nst = s->nst, n = s->n;
  for (int l0 = 0; l0 < n; l0++)
    for (int k = 0; k < nd; k++) {
      double qv[MAXM], Fv[MAXM];
      for (int v = 0; v < m; v++) qv[v] = q[(v * n + l0) * nd + k];
      for (int a = 0; a < s->d; a++) {
        pde_flux(p, s, qv, a, Fv);
        for (int v = 0; v < m; v++) F[(a * m + v) * nst + l0 * nd + k] = Fv[v];
      }
    }
  for (int l0 = 0; l0 < n; l0++)
    for (int k = 0; k < nd; k++) {
      double qv[MAXM], Sv[MAXM], grad[3][MAXM], ncp[MAXM];
      for (int v = 0; v < m; v++) qv[v] = q[(v * n + l0) * nd + k];
      pde_source(p, s, qv, Sv);
      for (int a = 0; a < 3; a++)
        for (int v = 0; v < m; v++) grad[a][v] = 0.0;
      double divF[MAXM];
      for (int v = 0; v < m; v++) divF[v] = 0.0;
      for (int a = 0; a < s->d; a++) {
        int ka = axis_index(s, k, a);
        int base = k - ka * s->str[a];
        for (int v = 0; v < m; v++) {
          double dF = 0.0, dq = 0.0;
          for (int j = 0; j < n; j++) {
            int kj = base + j * s->str[a];
            dF += s->Dhat[ka * n + j] * F[(a * m + v) * nst + l0 * nd + kj];
            dq += s->Dhat[ka * n + j] * q[(v * n + l0) * nd + kj];
          }
          divF[v] += dF / s->h[a];
          grad[a][v] = dq / s->h[a];
        }
      }
      pde_ncp(p, s, qv, mat, grad, ncp);
      for (int v = 0; v < m; v++) R[(v * n + l0) * nd + k] = Sv[v] - divF[v] - ncp[v];
    }
}

/* L(w) = S - div F - B.grad of a state w(k) constant in time, at the
 * spatial nodes: the collocated right-hand side of the time-constant
 * space-time polynomial (all its time slices are equal; slice 0 is kept). */
static void rhs_of_state(const orc_problem *p, const setup_t *s, const double *mat,
                         const double *w, double *q, double *F, double *R, double *out) {
  int m = s->m, nd = s->nd, n = s->n;
  for (int v = 0; v < m; v++)
    for (int l0 = 0; l0 < n; l0++)
      for (int k = 0; k < nd; k++) q[(v * n + l0) * nd + k] = w[v * nd + k];
  predictor_rhs(p, s, mat, q, F, R);
  for (int v = 0; v < m; v++)
    for (int k = 0; k < nd; k++) out[v * nd + k] = R[(v * n + 0) * nd + k];
}

int orc_sweeps(const orc_problem *p) {
  if (p->picard > 0) return p->picard;
  if (p->guess == 3) return 1;
  int g = p->guess > 0 ? p->guess : 0;
  return p->N + 1 - g > 1 ? p->N + 1 - g : 1;
}

/* Picard iteration of one element (Sec. 2.2), a fixed number of sweeps
 *   q^{r}(l0,k) = u(k) + dt * sum_j0 T[l0][j0] R(q^{r-1})(j0,k),
 * from the initial guess q^0 selected by p->guess (evaluated at the time
 * nodes t = t^n + xi_l0 dt, see orc_problem).  Returns the number of sweeps
 * done; stops early only when tol > 0 and the update fell to tol * max|q|. */
static int element_predictor(const orc_problem *p, const setup_t *s, const double *mat,
                             const double *ue, double dt, int sweeps, double tol,
                             double *q, double *F, double *R, const double *qprev, double ratio) {
  int m = s->m, nd = s->nd, n = s->n;
  if (p->guess == 3 && qprev) {
    /* the previous interval's polynomial q_h^{n-1}(tau), tau in [0,1] on
     * [t^{n-1}, t^n], evaluated at the new time nodes t^n + xi_l dt, i.e.
     * tau = 1 + xi_l dt/dt_prev, minus its value at tau = 1 */
    for (int v = 0; v < m; v++)
      for (int l0 = 0; l0 < n; l0++) {
        const double tau = 1.0 + s->xi[l0] * ratio;
        for (int k = 0; k < nd; k++) {
          double g = ue[v * nd + k];
          for (int j = 0; j < n; j++)
            g += qprev[(v * n + j) * nd + k] *
                 (orc_lagrange(n, s->xi, j, tau) - orc_lagrange(n, s->xi, j, 1.0));
          q[(v * n + l0) * nd + k] = g;
        }
      }
  } else if (p->guess == 0 || p->guess == 3) {
    for (int v = 0; v < m; v++)
      for (int l0 = 0; l0 < n; l0++)
        for (int k = 0; k < nd; k++) q[(v * n + l0) * nd + k] = ue[v * nd + k];
  } else {
    double k1[MAXM * ORC_MAXN * ORC_MAXN * ORC_MAXN], k2[MAXM * ORC_MAXN * ORC_MAXN * ORC_MAXN];
    rhs_of_state(p, s, mat, ue, q, F, R, k1);
    if (p->guess == 2) {
      double w[MAXM * ORC_MAXN * ORC_MAXN * ORC_MAXN];
      for (int i = 0; i < m * nd; i++) w[i] = ue[i] + dt * k1[i];
      rhs_of_state(p, s, mat, w, q, F, R, k2);
    }
    for (int v = 0; v < m; v++)
      for (int l0 = 0; l0 < n; l0++)
        for (int k = 0; k < nd; k++) {
          const int i = v * nd + k;
          const double tau = s->xi[l0] * dt;  /* t - t^n */
          double g = ue[i] + tau * k1[i];
          if (p->guess == 2) g += tau * tau * (k2[i] - k1[i]) / (2.0 * dt);
          q[(v * n + l0) * nd + k] = g;
        }
  }
  int r;
  for (r = 1; r <= sweeps; r++) {
    predictor_rhs(p, s, mat, q, F, R);
    double dmax = 0.0, qmax = 0.0;
    for (int v = 0; v < m; v++)
      for (int l0 = 0; l0 < n; l0++)
        for (int k = 0; k < nd; k++) {
          double acc = 0.0;
          for (int j0 = 0; j0 < n; j0++) acc += s->T[l0 * n + j0] * R[(v * n + j0) * nd + k];
          double qn = ue[v * nd + k] + dt * acc;
          double *qo = &q[(v * n + l0) * nd + k];
          dmax = fmax(dmax, fabs(qn - *qo));
          qmax = fmax(qmax, fabs(qn));
          *qo = qn;
        }
    if (tol > 0.0 && dmax <= tol * qmax) break;
  }
  return r > sweeps ? sweeps : r;
}

static int run_predictor(const orc_problem *p, const double *u, double dt, int sweeps,
                         double tol, double *qhat, const double *qprev, double ratio) {
  setup_t s;
  if (setup(p, &s)) return -1;
  int maxused = 0, fail = 0;
#pragma omp parallel
  {
    double *F = malloc(sizeof(double) * 3 * s.m * s.nst);
    double *R = malloc(sizeof(double) * s.m * s.nst);
    int used_local = 0;
    if (!F || !R) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(static)
      for (int e = 0; e < s.E; e++) {
        int used = element_predictor(p, &s, elem_mat(p, e), u + (size_t)e * s.m * s.nd, dt,
                                     sweeps, tol, qhat + (size_t)e * s.m * s.nst, F, R,
                                     qprev ? qprev + (size_t)e * s.m * s.nst : NULL, ratio);
        if (used > used_local) used_local = used;
      }
    }
#pragma omp critical
    if (used_local > maxused) maxused = used_local;
    free(F);
    free(R);
  }
  return fail ? -1 : maxused;
}

int orc_predictor(const orc_problem *p, const double *u, double dt, double *qhat) {
  return orc_predictor_hist(p, u, dt, NULL, 0.0, qhat);
}

int orc_guess_hist(const orc_problem *p, const double *u, double dt, const double *qprev, double dtprev,
                   double *q0) {
  const int hist = p->guess == 3 && qprev && dtprev > 0.0;
  return run_predictor(p, u, dt, 0, 0.0, q0, hist ? qprev : NULL, hist ? dt / dtprev : 0.0) < 0 ? -1 : 0;
}

int orc_predictor_hist(const orc_problem *p, const double *u, double dt, const double *qprev,
                       double dtprev, double *qhat) {
  const int hist = p->guess == 3 && qprev && dtprev > 0.0;
  /* guess 3 without a previous interval: the plain scheme (constant guess, N+1 sweeps) */
  const int sweeps = (p->guess == 3 && !hist) ? p->N + 1 : orc_sweeps(p);
  return run_predictor(p, u, dt, sweeps, 0.0, qhat, hist ? qprev : NULL, hist ? dt / dtprev : 0.0) < 0 ? -1 : 0;
}

int orc_predictor_converge(const orc_problem *p, const double *u, double dt, double tol,
                           int max_sweeps, double *qhat) {
  return run_predictor(p, u, dt, max_sweeps, tol, qhat, NULL, 0.0);
}

/* ------------------------------------------------------------------ */
/* Corrector (Sec. 2.1, eq. pde.nc.gw2), divided by the diagonal mass   */
/* matrix |Omega| w_k.  All integrals use the GL nodes in space and     */
/* time; the face term is integrated node by node in space and time     */
/* (reading: the Riemann solver is evaluated at every face-node and     */
/* time-node pair).                                                     */
/* ------------------------------------------------------------------ */

static int neighbour(const orc_problem *p, int e, int a, int dir) {
  int idx[3] = {0, 0, 0}, rem = e;
  for (int b = 0; b < p->dim; b++) {
    idx[b] = rem % p->nel[b];
    rem /= p->nel[b];
  }
  idx[a] = (idx[a] + dir + p->nel[a]) % p->nel[a]; /* periodic */
  int r = 0;
  for (int b = p->dim - 1; b >= 0; b--) r = r * p->nel[b] + idx[b];
  return r;
}

static void element_corrector(const orc_problem *p, const setup_t *s, int e, const double *u,
                              const double *qhat, double dt, double *unew, double *Fl,
                              double *G) {
  int m = s->m, nd = s->nd, n = s->n, nst = s->nst;
  const double *q = qhat + (size_t)e * m * nst;
  const double *mat = elem_mat(p, e);
  const double *ue = u + (size_t)e * m * nd;
  double *un = unew + (size_t)e * m * nd;
  double V[MAXM * ORC_MAXN * ORC_MAXN * ORC_MAXN];
  for (int i = 0; i < m * nd; i++) V[i] = 0.0;

  /* Volume terms: + int grad(Phi_k).F - int Phi_k B.grad q + int Phi_k S. */
  for (int l0 = 0; l0 < n; l0++) {
    for (int k = 0; k < nd; k++) {
      double qv[MAXM], Fv[MAXM];
      for (int v = 0; v < m; v++) qv[v] = q[(v * n + l0) * nd + k];
      for (int a = 0; a < s->d; a++) {
        pde_flux(p, s, qv, a, Fv);
        for (int v = 0; v < m; v++) Fl[(a * m + v) * nd + k] = Fv[v];
      }
    }
    for (int k = 0; k < nd; k++) {
      double qv[MAXM], grad[3][MAXM], ncp[MAXM], Sv[MAXM], vol[MAXM];
      for (int v = 0; v < m; v++) {
        qv[v] = q[(v * n + l0) * nd + k];
        vol[v] = 0.0;
      }
      for (int a = 0; a < 3; a++)
        for (int v = 0; v < m; v++) grad[a][v] = 0.0;
      for (int a = 0; a < s->d; a++) {
        int ka = axis_index(s, k, a);
        int base = k - ka * s->str[a];
        for (int v = 0; v < m; v++) {
          /* (1/w_ka) sum_j w_j phi_ka'(xi_j) F(j) = stiffness term / mass */
          double sF = 0.0, dq = 0.0;
          for (int j = 0; j < n; j++) {
            int kj = base + j * s->str[a];
            sF += s->w[j] * s->Dhat[j * n + ka] * Fl[(a * m + v) * nd + kj];
            dq += s->Dhat[ka * n + j] * q[(v * n + l0) * nd + kj];
          }
          vol[v] += sF / (s->w[ka] * s->h[a]);
          grad[a][v] = dq / s->h[a];
        }
      }
      pde_ncp(p, s, qv, mat, grad, ncp);
      pde_source(p, s, qv, Sv);
      for (int v = 0; v < m; v++) V[v * nd + k] += s->w[l0] * (vol[v] - ncp[v] + Sv[v]);
    }
  }

  /* Face terms: - (1/h_a) phi_ka(side)/w_ka * sum_l0 w_l0 D^-(q_in, q_out).n */
  for (int a = 0; a < s->d; a++) {
    for (int side = 0; side < 2; side++) {
      int nb = neighbour(p, e, a, side ? +1 : -1);
      const double *qn = qhat + (size_t)nb * m * nst;
      const double *matn = elem_mat(p, nb);
      const double *phin = side ? s->F1 : s->F0;  /* inside trace: this face */
      const double *phout = side ? s->F0 : s->F1; /* outside: neighbour's opposite face */
      double sgn = side ? 1.0 : -1.0;
      for (int i = 0; i < m * nd; i++) G[i] = 0.0;
      for (int k = 0; k < nd && p->face_avg; k++) {
        if (axis_index(s, k, a) != 0) continue;
        /* time averages, over the time nodes, of the boundary-extrapolated
         * states and of the flux evaluated at those states */
        double qi[MAXM], qo[MAXM], Fi[MAXM], Fo[MAXM];
        for (int v = 0; v < m; v++) qi[v] = qo[v] = Fi[v] = Fo[v] = 0.0;
        for (int l0 = 0; l0 < n; l0++) {
          double tin[MAXM], tout[MAXM], fin[MAXM], fout[MAXM];
          for (int v = 0; v < m; v++) {
            double si = 0.0, so = 0.0;
            for (int j = 0; j < n; j++) {
              si += phin[j] * q[(v * n + l0) * nd + k + j * s->str[a]];
              so += phout[j] * qn[(v * n + l0) * nd + k + j * s->str[a]];
            }
            tin[v] = si;
            tout[v] = so;
          }
          pde_flux(p, s, tin, a, fin);
          pde_flux(p, s, tout, a, fout);
          for (int v = 0; v < m; v++) {
            qi[v] += s->w[l0] * tin[v];
            qo[v] += s->w[l0] * tout[v];
            Fi[v] += s->w[l0] * fin[v];
            Fo[v] += s->w[l0] * fout[v];
          }
        }
        double D[MAXM];
        dminus_avg(p, s, qi, qo, Fi, Fo, mat, matn, a, sgn, D);
        for (int v = 0; v < m; v++) G[v * nd + k] = D[v];
      }
      for (int k = 0; k < nd && !p->face_avg; k++) {
        if (axis_index(s, k, a) != 0) continue; /* k enumerates the face nodes */
        for (int l0 = 0; l0 < n; l0++) {
          double qin[MAXM], qout[MAXM], D[MAXM];
          for (int v = 0; v < m; v++) {
            double si = 0.0, so = 0.0;
            for (int j = 0; j < n; j++) {
              si += phin[j] * q[(v * n + l0) * nd + k + j * s->str[a]];
              so += phout[j] * qn[(v * n + l0) * nd + k + j * s->str[a]];
            }
            qin[v] = si;
            qout[v] = so;
          }
          dminus(p, s, qin, qout, mat, matn, a, sgn, D);
          for (int v = 0; v < m; v++) G[v * nd + k] += s->w[l0] * D[v];
        }
      }
      for (int k = 0; k < nd; k++) {
        int ka = axis_index(s, k, a);
        int kf = k - ka * s->str[a];
        double lift = (side ? s->F1[ka] : s->F0[ka]) / (s->w[ka] * s->h[a]);
        for (int v = 0; v < m; v++) V[v * nd + k] -= lift * G[v * nd + kf];
      }
    }
  }
  for (int i = 0; i < m * nd; i++) un[i] = ue[i] + dt * V[i];
}

int orc_corrector(const orc_problem *p, const double *u, const double *qhat, double dt,
                  double *unew) {
  setup_t s;
  if (setup(p, &s)) return -1;
  int fail = 0;
#pragma omp parallel
  {
    double *Fl = malloc(sizeof(double) * 3 * s.m * s.nd);
    double *G = malloc(sizeof(double) * s.m * s.nd);
    if (!Fl || !G) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(static)
      for (int e = 0; e < s.E; e++) element_corrector(p, &s, e, u, qhat, dt, unew, Fl, G);
    }
    free(Fl);
    free(G);
  }
  return fail ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Time step (Sec. 3, CFL condition).  The paper bounds the coefficient */
/* by alpha < 1/(2N+1) and takes its value from a von Neumann analysis. */
/* Reading: alpha = cfl * alpha_N, where alpha_N is the 1-D von Neumann */
/* limit of this very scheme (linear advection, upwind flux, converged  */
/* predictor; largest Courant number with spectral radius <= 1 + 1e-4), */
/* rounded down to 3 significant digits.  The wave speeds are the       */
/* per-element maxima over the nodes of u^n, per axis.                  */
/* ------------------------------------------------------------------ */

double orc_stability_alpha(int N) {
  static const double alpha[ORC_MAXN] = {1.00, 0.333, 0.170, 0.103, 0.0698, 0.0501, 0.0355, 0.0256};
  return (N >= 0 && N < ORC_MAXN) ? alpha[N] : -1.0;
}

double orc_cfl_dt(const orc_problem *p, const double *u) {
  setup_t s;
  if (setup(p, &s)) return -1.0;
  double S = 0.0;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : S) reduction(| : bad)
  for (int e = 0; e < s.E; e++) {
    const double *mat = elem_mat(p, e);
    double lmax[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < s.nd; k++) {
      double qv[MAXM];
      for (int v = 0; v < s.m; v++) {
        qv[v] = u[((size_t)e * s.m + v) * s.nd + k];
        if (!isfinite(qv[v])) bad = 1;
      }
      if (p->pde == ORC_EULER && (qv[0] <= 0.0 || euler_pressure(s.d, p->gamma, qv) <= 0.0))
        bad = 1;
      for (int a = 0; a < s.d; a++) {
        double l = pde_speed(p, &s, qv, mat, a);
        if (!(l == l)) bad = 1;
        if (l > lmax[a]) lmax[a] = l;
      }
    }
    double se = 0.0;
    for (int a = 0; a < s.d; a++) se += lmax[a] / s.h[a];
    if (se > S) S = se;
  }
  if (bad || !(S > 0.0) || !isfinite(S)) return -1.0;
  return (p->cfl * orc_stability_alpha(p->N)) / S;
}

int orc_step(const orc_problem *p, double *u, double *t, double t_end, double *dt_out) {
  return orc_step_hist(p, u, t, t_end, dt_out, NULL, NULL, NULL);
}

int orc_step_hist(const orc_problem *p, double *u, double *t, double t_end, double *dt_out, double *qprev,
                  double *dtprev, int *has) {
  setup_t s;
  if (setup(p, &s)) return -1;
  double dt = orc_cfl_dt(p, u);
  if (dt < 0.0) return -1;
  double tn;
  if (t_end - *t <= dt) {
    dt = t_end - *t; /* the last step lands exactly on t_end */
    tn = t_end;
  } else {
    tn = *t + dt;
  }
  if (dt < 0.0) dt = 0.0;
  size_t nq = (size_t)s.E * s.m * s.nst, nu = (size_t)s.E * s.m * s.nd;
  double *qhat = malloc(sizeof(double) * nq);
  double *un = malloc(sizeof(double) * nu);
  int rc = -1;
  const int hist = qprev && dtprev && has && *has;
  if (qhat && un && orc_predictor_hist(p, u, dt, hist ? qprev : NULL, hist ? *dtprev : 0.0, qhat) == 0 &&
      orc_corrector(p, u, qhat, dt, un) == 0) {
    memcpy(u, un, sizeof(double) * nu);
    *t = tn;
    if (dt_out) *dt_out = dt;
    if (qprev && dtprev && has) {  /* this interval becomes the previous one */
      memcpy(qprev, qhat, sizeof(double) * nq);
      *dtprev = dt;
      *has = 1;
    }
    rc = 0;
  }
  free(qhat);
  free(un);
  return rc;
}

/* Domain integral of each variable: sum_e |Omega_e| sum_k (prod_a w_ka) u,
 * accumulated with Neumaier's compensated summation in element order. */
/* ------------------------------------------------------------------ */
/* A posteriori detection (Sec. 2.3, detection criteria of the limiter) */
/* ------------------------------------------------------------------ */

int orc_detect(const orc_problem *p, const double *u_old, const double *u_new, int *flags) {
  setup_t s;
  if (setup(p, &s)) return -1;
  const int m = s.m, nd = s.nd, d = s.d;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < s.E; e++) {
    const double *un = u_new + (size_t)e * m * nd;
    int f = 0;
    for (int i = 0; i < m * nd; i++)
      if (!isfinite(un[i])) f |= 1;
    if (p->pde == ORC_EULER)
      for (int k = 0; k < nd; k++) {
        double qv[MAXM];
        for (int v = 0; v < m; v++) qv[v] = un[v * nd + k];
        if (!(qv[0] > 0.0) || !(euler_pressure(d, p->gamma, qv) > 0.0)) f |= 2;
      }
    /* the vertex neighbourhood: offsets in {-1,0,1}^d */
    int idx[3] = {0, 0, 0}, rem = e;
    for (int b = 0; b < d; b++) {
      idx[b] = rem % p->nel[b];
      rem /= p->nel[b];
    }
    int nb = 1;
    for (int b = 0; b < d; b++) nb *= 3;
    for (int v = 0; v < m; v++) {
      double lo = INFINITY, hi = -INFINITY;
      for (int o = 0; o < nb; o++) {
        int r = o, j[3] = {0, 0, 0};
        for (int b = 0; b < d; b++) {
          j[b] = (idx[b] + (r % 3) - 1 + p->nel[b]) % p->nel[b];
          r /= 3;
        }
        int en = 0;
        for (int b = d - 1; b >= 0; b--) en = en * p->nel[b] + j[b];
        const double *uo = u_old + ((size_t)en * m + v) * nd;
        for (int k = 0; k < nd; k++) {
          lo = fmin(lo, uo[k]);
          hi = fmax(hi, uo[k]);
        }
      }
      const double delta = fmax(1e-4, 1e-3 * (hi - lo));
      const double lo_r = lo - delta, hi_r = hi + delta;
      for (int k = 0; k < nd; k++) {
        const double x = un[v * nd + k];
        if (x < lo_r || x > hi_r) f |= 4;
      }
    }
    flags[e] = f;
  }
  return 0;
}

int orc_totals(const orc_problem *p, const double *u, double *sums) {
  setup_t s;
  if (setup(p, &s)) return -1;
  double vol = 1.0;
  for (int a = 0; a < s.d; a++) vol *= s.h[a];
  for (int v = 0; v < s.m; v++) {
    double sum = 0.0, c = 0.0;
    for (int e = 0; e < s.E; e++)
      for (int k = 0; k < s.nd; k++) {
        double wk = vol;
        for (int a = 0; a < s.d; a++) wk *= s.w[axis_index(&s, k, a)];
        double x = wk * u[((size_t)e * s.m + v) * s.nd + k];
        double t = sum + x;
        if (fabs(sum) >= fabs(x)) c += (sum - t) + x;
        else c += (x - t) + sum;
        sum = t;
      }
    sums[v] = sum + c;
  }
  return 0;
}
