// Host construction of the 1-D operator tables (Sec. 2.1 and Sec. 2.2).
//
// Gauss-Legendre points and weights come from the Golub-Welsch method: the
// points are the eigenvalues of the symmetric tridiagonal Jacobi matrix of
// the Legendre recurrence, the weights the squared first components of its
// normalised eigenvectors; the eigenproblem is solved with cyclic Jacobi
// rotations.  Lagrange derivatives and end-point values use the barycentric
// form of the interpolant; the time operator is obtained by an LU solve.
#include <math.h>
#include <string.h>

#include "ader_common.hpp"

namespace ader {

namespace {

// Cyclic Jacobi eigen-solver for a symmetric n x n matrix A (row-major);
// on return the diagonal of A holds the eigenvalues and the columns of Z the
// eigenvectors.
void jacobi_eigen(int n, double *A, double *Z) {
  for (int i = 0; i < n * n; i++) Z[i] = 0.0;
  for (int i = 0; i < n; i++) Z[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0.0;
    for (int p = 0; p < n; p++)
      for (int q = p + 1; q < n; q++) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-60) break;
    for (int p = 0; p < n; p++)
      for (int q = p + 1; q < n; q++) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; k++) {  // A <- A J  (columns p, q)
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; k++) {  // A <- J^T A  (rows p, q)
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; k++) {
          double zkp = Z[k * n + p], zkq = Z[k * n + q];
          Z[k * n + p] = c * zkp - s * zkq;
          Z[k * n + q] = s * zkp + c * zkq;
        }
      }
  }
}

void golub_welsch01(int n, double *x, double *w) {
  double J[kMaxN * kMaxN] = {0}, Z[kMaxN * kMaxN];
  for (int k = 1; k < n; k++) {
    double b = k / sqrt(4.0 * k * k - 1.0);
    J[(k - 1) * n + k] = b;
    J[k * n + (k - 1)] = b;
  }
  jacobi_eigen(n, J, Z);
  double z[kMaxN], wz[kMaxN];
  for (int i = 0; i < n; i++) {
    z[i] = J[i * n + i];
    wz[i] = Z[0 * n + i] * Z[0 * n + i];  // (2 v0^2) on [-1,1] -> v0^2 on [0,1]
  }
  // sort ascending
  for (int i = 0; i < n; i++)
    for (int j = i + 1; j < n; j++)
      if (z[j] < z[i]) {
        double t = z[i]; z[i] = z[j]; z[j] = t;
        t = wz[i]; wz[i] = wz[j]; wz[j] = t;
      }
  for (int i = 0; i < n; i++) {
    x[i] = 0.5 * (1.0 + z[i]);
    w[i] = wz[i];
  }
  // the rule is symmetric about 1/2: average mirrored pairs
  for (int i = 0; i < n / 2; i++) {
    int j = n - 1 - i;
    double xs = 0.5 * (x[i] + (1.0 - x[j]));
    double ws = 0.5 * (w[i] + w[j]);
    x[i] = xs; x[j] = 1.0 - xs;
    w[i] = ws; w[j] = ws;
  }
  if (n % 2) x[n / 2] = 0.5;
}

// Solve A X = B in place of B with LU decomposition and partial pivoting.
int lu_solve(int n, double *A, double *B) {
  int piv[kMaxN];
  for (int k = 0; k < n; k++) {
    int p = k;
    for (int i = k + 1; i < n; i++)
      if (fabs(A[i * n + k]) > fabs(A[p * n + k])) p = i;
    if (A[p * n + k] == 0.0) return -1;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; j++) {
        double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t;
      }
    for (int i = k + 1; i < n; i++) {
      A[i * n + k] /= A[k * n + k];
      for (int j = k + 1; j < n; j++) A[i * n + j] -= A[i * n + k] * A[k * n + j];
    }
  }
  for (int c = 0; c < n; c++) {
    double y[kMaxN];
    for (int i = 0; i < n; i++) y[i] = B[i * n + c];
    for (int k = 0; k < n; k++)
      if (piv[k] != k) { double t = y[k]; y[k] = y[piv[k]]; y[piv[k]] = t; }
    for (int i = 0; i < n; i++)
      for (int j = 0; j < i; j++) y[i] -= A[i * n + j] * y[j];
    for (int i = n - 1; i >= 0; i--) {
      for (int j = i + 1; j < n; j++) y[i] -= A[i * n + j] * y[j];
      y[i] /= A[i * n + i];
    }
    for (int i = 0; i < n; i++) B[i * n + c] = y[i];
  }
  return 0;
}

}  // namespace

int build_ops(int N, Ops *o) {
  const int n = N + 1;
  if (N < 0 || n > kMaxN) return -1;
  memset(o, 0, sizeof(*o));
  golub_welsch01(n, o->xi, o->w);
  const double *x = o->xi;
  double lam[kMaxN];  // barycentric weights
  for (int j = 0; j < n; j++) {
    double p = 1.0;
    for (int k = 0; k < n; k++)
      if (k != j) p *= (x[j] - x[k]);
    lam[j] = 1.0 / p;
  }
  double Dn[kMaxN * kMaxN];
  for (int i = 0; i < n; i++) {
    double diag = 0.0;
    for (int j = 0; j < n; j++) {
      if (j == i) continue;
      double d = (lam[j] / lam[i]) / (x[i] - x[j]);
      Dn[i * n + j] = d;
      diag -= d;
    }
    Dn[i * n + i] = diag;
  }
  for (int s = 0; s < 2; s++) {  // end-point values, second barycentric form
    double xe = s ? 1.0 : 0.0, den = 0.0, t[kMaxN];
    for (int j = 0; j < n; j++) { t[j] = lam[j] / (xe - x[j]); den += t[j]; }
    for (int j = 0; j < n; j++) (s ? o->F1 : o->F0)[j] = t[j] / den;
  }
  // K1 = F1 F1^T - K^T with K[j][k] = w_j phi_k'(xi_j); T = K1^{-1} W
  double K1[kMaxN * kMaxN], W[kMaxN * kMaxN];
  for (int a = 0; a < n; a++)
    for (int b = 0; b < n; b++) {
      K1[a * n + b] = o->F1[a] * o->F1[b] - o->w[b] * Dn[b * n + a];
      W[a * n + b] = (a == b) ? o->w[a] : 0.0;
    }
  if (lu_solve(n, K1, W)) return -2;
  for (int a = 0; a < n; a++)
    for (int b = 0; b < n; b++) {
      o->D[a * kMaxN + b] = Dn[a * n + b];
      o->T[a * kMaxN + b] = W[a * n + b];
      o->V[a * kMaxN + b] = o->w[b] * Dn[b * n + a] / o->w[a];
    }
  // Taylor coefficients of the basis about tau = 1: with V[l][p] = (xi_l - 1)^p,
  // phi_j(tau) = sum_p (V^{-1})[p][j] (tau - 1)^p
  {
    double V[kMaxN * kMaxN], Id[kMaxN * kMaxN];
    for (int l = 0; l < n; l++)
      for (int q = 0; q < n; q++) {
        double pw = 1.0;
        for (int r = 0; r < q; r++) pw *= (x[l] - 1.0);
        V[l * n + q] = pw;
        Id[l * n + q] = (l == q) ? 1.0 : 0.0;
      }
    if (lu_solve(n, V, Id)) return -3;
    for (int q = 0; q < n; q++)
      for (int j = 0; j < n; j++) o->TE[q * kMaxN + j] = Id[q * n + j];
  }
  for (int k = 0; k < n; k++) {
    o->L0[k] = o->F0[k] / o->w[k];
    o->L1[k] = o->F1[k] / o->w[k];
    double r = 0.0;
    for (int j = 0; j < n; j++) r += o->T[k * kMaxN + j];
    o->Trow[k] = r;
  }
  return 0;
}

// alpha_N: largest Courant number of the 1-D scheme for linear advection
// (upwind flux, converged predictor) at which no Fourier mode grows by more
// than 1e-4 per step, rounded down to three significant digits.  The paper
// requires alpha < 1/(2N+1) and takes alpha from such an analysis (Sec. 3).
double stability_alpha(int N) {
  static const double a[kMaxN] = {1.00, 0.333, 0.170, 0.103, 0.0698, 0.0501, 0.0355, 0.0256};
  return (N >= 0 && N < kMaxN) ? a[N] : -1.0;
}

void line_slots(int D, int N, int A, uint16_t *out) {
  const int n = N + 1;
  int nd = 1;
  for (int a = 0; a < D; a++) nd *= n;
  const int nf = nd / n, nl = nd;  // lines of one axis phase: n time slices x n^(D-1)
  int st = 1;
  for (int a = 0; a < A; a++) st *= n;
  const int waves = (nl + 63) / 64;
  for (int s = 0; s < kMaxSlots; s++) out[s] = kEmptySlot;
  // line L: time slice l0 = L / nf, face index r = L % nf over the other axes
  int rest[kMaxSlots], nrest = nl;
  for (int L = 0; L < nl; L++) {
    const int l0 = L / nf, r = L % nf;
    rest[L] = l0 * nd + r % st + (r / st) * st * n;
  }
  for (int w = 0; w < waves; w++) {
    int keep = 0;
    for (int i = 0; i < nrest; i++) {
      const int b = rest[i], s = w * 64 + b % 64;
      if (out[s] == kEmptySlot) out[s] = (uint16_t)b;
      else rest[keep++] = b;
    }
    nrest = keep;
  }
  for (int i = 0, s = 0; i < nrest; i++) {  // lines left over: first free slots
    while (out[s] != kEmptySlot) s++;
    out[s] = (uint16_t)rest[i];
  }
}

}  // namespace ader
