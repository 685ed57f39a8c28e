// Device kernels of the ADER-DG step, templated on space dimension D,
// degree N and PDE system.  One workgroup owns one element in the predictor;
// the face and update kernels are one thread per face node / per DOF.
#pragma once
#include "ader_common.hpp"

namespace ader {

// ------------------------------------------------------------ PDE systems

// Compressible Euler equations (Sec. 3.1, eq. euler), ideal gas.
template <int D>
struct Euler {
  static constexpr int M = D + 2;
  static constexpr bool kConservative = true;   // B = 0: face integral single-valued
  static constexpr bool kElastic = false;
};

// Linear elasticity, velocity-stress form (Sec. 3.2 with volume fraction 1).
struct Elastic {
  static constexpr int M = 9;
  static constexpr bool kConservative = false;  // B != 0: two face integrals
  static constexpr bool kElastic = true;
};

// Flux F_A(q) of the Euler equations; p = (gamma-1)(rho E - |rho v|^2/(2 rho)).
template <int D, int A, typename R>
__device__ __forceinline__ void euler_flux(const R *q, R gm1, R *F) {
  const R ir = R(1) / q[0];
  R ke = R(0);
#pragma unroll
  for (int i = 0; i < D; i++) ke += q[1 + i] * q[1 + i];
  const R p = gm1 * (q[D + 1] - R(0.5) * ke * ir);
  const R va = q[1 + A] * ir;
  F[0] = q[1 + A];
#pragma unroll
  for (int i = 0; i < D; i++) F[1 + i] = q[1 + i] * va;
  F[1 + A] += p;
  F[D + 1] = (q[D + 1] + p) * va;
}

// Pressure and largest |eigenvalue| |v_A| + c of the Euler flux Jacobian.
template <int D>
__device__ __forceinline__ double euler_pressure(const double *q, double gamma) {
  double ke = 0.0;
#pragma unroll
  for (int i = 0; i < D; i++) ke += q[1 + i] * q[1 + i];
  return (gamma - 1.0) * (q[D + 1] - 0.5 * ke / q[0]);
}

// Index of stress component s_{iA} in the elastic state vector.
__device__ __forceinline__ constexpr int sig(int i, int j) {
  return (i == j) ? 3 + i : ((i + j == 1) ? 6 : ((i + j == 3) ? 7 : 8));
}

// B_A g for the elastic system, g = d q / d x_A:
//   velocity rows: -(1/rho) d s_{iA}/dx_A,
//   stress rows:   -(lambda delta_ij dv_A/dx_A + mu (delta_iA dv_j/dx_A + delta_jA dv_i/dx_A)).
template <int A, typename R>
__device__ __forceinline__ void elastic_bg(const R *g, R irho, R lam, R mu, R *out) {
#pragma unroll
  for (int i = 0; i < 3; i++) out[i] = -irho * g[sig(i, A)];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    R s = lam * g[A];
    if (i == A) s += R(2) * mu * g[A];
    out[3 + i] = -s;
  }
  // off-diagonal (i,j) = (0,1), (1,2), (0,2) stored at 6, 7, 8
  out[6] = -mu * ((A == 0 ? g[1] : R(0)) + (A == 1 ? g[0] : R(0)));
  out[7] = -mu * ((A == 1 ? g[2] : R(0)) + (A == 2 ? g[1] : R(0)));
  out[8] = -mu * ((A == 0 ? g[2] : R(0)) + (A == 2 ? g[0] : R(0)));
}

__device__ __forceinline__ int64_t neighbour(int64_t e, int A, int dir, const int *nel) {
  int64_t ix = e % nel[0];
  int64_t r = e / nel[0];
  int64_t iy = r % nel[1];
  int64_t iz = r / nel[1];
  if (A == 0) ix = (ix + dir + nel[0]) % nel[0];
  if (A == 1) iy = (iy + dir + nel[1]) % nel[1];
  if (A == 2) iz = (iz + dir + nel[2]) % nel[2];
  return ix + (int64_t)nel[0] * (iy + (int64_t)nel[1] * iz);
}

// ------------------------------------------------------------ predictor

struct PredArgs {
  Ops ops;
  Geom g;
  const double *u;      // [E][M][ND]
  const double *dt;     // device scalar
  const double *mat;    // elastic: [E][3]
  double *ustar;        // [E][M][ND]  u + dt * volume terms
  double *trace[3][2];  // [E][M][n][ND/n] per axis and side (0: x_A = 0, 1: x_A = 1)
  double *qhat;         // optional [E][M][n][ND]
  double *acc_glob;     // accumulator when it does not fit in LDS: [E][M][max(NST,2ND)]
  int sweeps;
};

template <int D, int N>
struct Shape {
  static constexpr int n = N + 1;
  static constexpr int ND = ipow(n, D);
  static constexpr int NST = ND * n;
  static constexpr int NF = ND / n;   // face nodes
  static constexpr int ACC = (NST > 2 * ND) ? NST : 2 * ND;
};

// Collocated right-hand side along axis A for all lines of the element:
//   R -= (1/h_A) Dhat_A F_A(q)           (Euler)
//   R -= (1/h_A) B_A (Dhat_A q)          (elasticity)
// Lines are enumerated over (l0, the other spatial indices).
template <int D, int N, class PDE, int A>
__device__ __forceinline__ void rhs_axis(const PredArgs &P, const double *sq, double *sacc,
                                         double irho, double lam, double mu) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST, NF = S::NF;
  constexpr int ST = ipow(n, A);
  const double ih = P.g.inv_h[A];
  for (int L = threadIdx.x; L < NST / n; L += kBlock) {
    const int l0 = L / NF, r = L - l0 * NF;
    const int lo = r % ST, hi = r / ST;
    const int base = l0 * ND + lo + hi * ST * n;
    double qv[n][M];
#pragma unroll
    for (int j = 0; j < n; j++)
#pragma unroll
      for (int v = 0; v < M; v++) qv[j][v] = sq[v * NST + base + j * ST];
    double out[n][M];
    if constexpr (!PDE::kElastic) {
      double F[n][M];
#pragma unroll
      for (int j = 0; j < n; j++) euler_flux<D, A>(qv[j], P.g.gamma - 1.0, F[j]);
#pragma unroll
      for (int k = 0; k < n; k++)
#pragma unroll
        for (int v = 0; v < M; v++) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < n; j++) s += P.ops.D[k * kMaxN + j] * F[j][v];
          out[k][v] = -s * ih;
        }
    } else {
#pragma unroll
      for (int k = 0; k < n; k++) {
        double gk[M], bg[M];
#pragma unroll
        for (int v = 0; v < M; v++) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < n; j++) s += P.ops.D[k * kMaxN + j] * qv[j][v];
          gk[v] = s;
        }
        elastic_bg<A>(gk, irho, lam, mu, bg);
#pragma unroll
        for (int v = 0; v < M; v++) out[k][v] = -bg[v] * ih;
      }
    }
#pragma unroll
    for (int k = 0; k < n; k++)
#pragma unroll
      for (int v = 0; v < M; v++) {
        const int idx = v * NST + base + k * ST;
        if (A == 0) sacc[idx] = out[k][v];
        else sacc[idx] += out[k][v];
      }
  }
}

// Euler volume term along axis A from the time-integrated flux:
//   V += (1/h_A) Vop_A [ sum_l0 w_l0 F_A(q(l0)) ]
template <int D, int N, class PDE, int A>
__device__ __forceinline__ void volume_axis_euler(const PredArgs &P, const double *sq, double *sV) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST, NF = S::NF;
  constexpr int ST = ipow(n, A);
  const double ih = P.g.inv_h[A];
  for (int L = threadIdx.x; L < NF; L += kBlock) {
    const int lo = L % ST, hi = L / ST;
    const int base = lo + hi * ST * n;
    double Fb[n][M];
#pragma unroll
    for (int j = 0; j < n; j++)
#pragma unroll
      for (int v = 0; v < M; v++) Fb[j][v] = 0.0;
    for (int l0 = 0; l0 < n; l0++) {
      const double wl = P.ops.w[l0];
#pragma unroll
      for (int j = 0; j < n; j++) {
        double qv[M], F[M];
#pragma unroll
        for (int v = 0; v < M; v++) qv[v] = sq[v * NST + l0 * ND + base + j * ST];
        euler_flux<D, A>(qv, P.g.gamma - 1.0, F);
#pragma unroll
        for (int v = 0; v < M; v++) Fb[j][v] += wl * F[v];
      }
    }
#pragma unroll
    for (int k = 0; k < n; k++)
#pragma unroll
      for (int v = 0; v < M; v++) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < n; j++) s += P.ops.V[k * kMaxN + j] * Fb[j][v];
        const int idx = v * ND + base + k * ST;
        if (A == 0) sV[idx] = s * ih;
        else sV[idx] += s * ih;
      }
  }
}

// Elastic volume term along axis A: V -= (1/h_A) B_A Dhat_A qbar,
// qbar = sum_l0 w_l0 q(l0) (B is constant in the element).
template <int D, int N, int A>
__device__ __forceinline__ void volume_axis_elastic(const PredArgs &P, const double *sQ, double *sV,
                                                    double irho, double lam, double mu) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = 9, ND = S::ND, NF = S::NF;
  constexpr int ST = ipow(n, A);
  const double ih = P.g.inv_h[A];
  for (int L = threadIdx.x; L < NF; L += kBlock) {
    const int lo = L % ST, hi = L / ST;
    const int base = lo + hi * ST * n;
    double qv[n][M];
#pragma unroll
    for (int j = 0; j < n; j++)
#pragma unroll
      for (int v = 0; v < M; v++) qv[j][v] = sQ[v * ND + base + j * ST];
#pragma unroll
    for (int k = 0; k < n; k++) {
      double gk[M], bg[M];
#pragma unroll
      for (int v = 0; v < M; v++) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < n; j++) s += P.ops.D[k * kMaxN + j] * qv[j][v];
        gk[v] = s;
      }
      elastic_bg<A>(gk, irho, lam, mu, bg);
#pragma unroll
      for (int v = 0; v < M; v++) {
        const int idx = v * ND + base + k * ST;
        if (A == 0) sV[idx] = -bg[v] * ih;
        else sV[idx] -= bg[v] * ih;
      }
    }
  }
}

// Boundary-extrapolated traces on both faces normal to axis A:
// trace_s(v, l0, face node) = sum_j phi_j(s) q(v, l0, node with k_A = j).
template <int D, int N, class PDE, int A>
__device__ __forceinline__ void traces_axis(const PredArgs &P, const double *sq, int64_t e) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST, NF = S::NF;
  constexpr int ST = ipow(n, A);
  double *t0 = P.trace[A][0] + e * (int64_t)(M * ND);
  double *t1 = P.trace[A][1] + e * (int64_t)(M * ND);
  for (int i = threadIdx.x; i < M * ND; i += kBlock) {
    const int v = i / ND, r = i - v * ND;
    const int l0 = r / NF, kf = r - l0 * NF;
    const int lo = kf % ST, hi = kf / ST;
    const double *line = sq + v * NST + l0 * ND + lo + hi * ST * n;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int j = 0; j < n; j++) {
      const double qj = line[j * ST];
      a0 += P.ops.F0[j] * qj;
      a1 += P.ops.F1[j] * qj;
    }
    t0[i] = a0;
    t1[i] = a1;
  }
}

// Space-time predictor (Sec. 2.2) of one element per workgroup, FP64.
// LDS: sq[M][NST] (space-time DOFs, layout [v][l0][k]) and, when it fits,
// the accumulator sacc[M][ACC]; otherwise the accumulator lives in HBM.
template <int D, int N, class PDE, bool kAccLds>
__global__ void __launch_bounds__(kBlock) k_predictor(const PredArgs P) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST;
  extern __shared__ double smem[];
  const int64_t e = blockIdx.x;
  double *sq = smem;
  double *sacc = kAccLds ? smem + M * NST : P.acc_glob + e * (int64_t)(M * S::ACC);
  const double *ue = P.u + e * (int64_t)(M * ND);
  const double dt = *P.dt;
  double irho = 0.0, lam = 0.0, mu = 0.0;
  if constexpr (PDE::kElastic) {
    irho = 1.0 / P.mat[3 * e + 0];
    lam = P.mat[3 * e + 1];
    mu = P.mat[3 * e + 2];
  }
  // q^0 = u_h(t^n), constant in time (K1^{-1} F0 = 1)
  for (int i = threadIdx.x; i < M * ND; i += kBlock) {
    const double val = ue[i];
    const int v = i / ND, k = i - v * ND;
#pragma unroll
    for (int l0 = 0; l0 < n; l0++) sq[v * NST + l0 * ND + k] = val;
  }
  __syncthreads();
  for (int s = 0; s < P.sweeps; s++) {
    rhs_axis<D, N, PDE, 0>(P, sq, sacc, irho, lam, mu);
    __syncthreads();
    if constexpr (D > 1) {
      rhs_axis<D, N, PDE, 1>(P, sq, sacc, irho, lam, mu);
      __syncthreads();
    }
    if constexpr (D > 2) {
      rhs_axis<D, N, PDE, 2>(P, sq, sacc, irho, lam, mu);
      __syncthreads();
    }
    // q(l0,k) = u(k) + dt sum_j0 T[l0][j0] R(j0,k)
    for (int i = threadIdx.x; i < M * ND; i += kBlock) {
      const int v = i / ND, k = i - v * ND;
      double r[n];
#pragma unroll
      for (int j = 0; j < n; j++) r[j] = sacc[v * NST + j * ND + k];
      const double u0 = ue[i];
#pragma unroll
      for (int l = 0; l < n; l++) {
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < n; j++) a += P.ops.T[l * kMaxN + j] * r[j];
        sq[v * NST + l * ND + k] = u0 + dt * a;
      }
    }
    __syncthreads();
  }
  if (P.qhat) {
    double *qo = P.qhat + e * (int64_t)(M * NST);
    for (int i = threadIdx.x; i < M * NST; i += kBlock) qo[i] = sq[i];
  }
  traces_axis<D, N, PDE, 0>(P, sq, e);
  if constexpr (D > 1) traces_axis<D, N, PDE, 1>(P, sq, e);
  if constexpr (D > 2) traces_axis<D, N, PDE, 2>(P, sq, e);
  // volume terms into sV = sacc[0 .. M*ND)
  double *sV = sacc;
  if constexpr (N == 0) {
    for (int i = threadIdx.x; i < M * ND; i += kBlock) sV[i] = 0.0;
  } else if constexpr (!PDE::kElastic) {
    volume_axis_euler<D, N, PDE, 0>(P, sq, sV);
    __syncthreads();
    if constexpr (D > 1) {
      volume_axis_euler<D, N, PDE, 1>(P, sq, sV);
      __syncthreads();
    }
    if constexpr (D > 2) volume_axis_euler<D, N, PDE, 2>(P, sq, sV);
  } else {
    double *sQ = sacc + M * ND;
    for (int i = threadIdx.x; i < M * ND; i += kBlock) {
      const int v = i / ND, k = i - v * ND;
      double a = 0.0;
#pragma unroll
      for (int l = 0; l < n; l++) a += P.ops.w[l] * sq[v * NST + l * ND + k];
      sQ[i] = a;
    }
    __syncthreads();
    volume_axis_elastic<D, N, 0>(P, sQ, sV, irho, lam, mu);
    __syncthreads();
    volume_axis_elastic<D, N, 1>(P, sQ, sV, irho, lam, mu);
    __syncthreads();
    volume_axis_elastic<D, N, 2>(P, sQ, sV, irho, lam, mu);
  }
  __syncthreads();
  double *us = P.ustar + e * (int64_t)(M * ND);
  // dt = 0 (flagged state or t already at t_end) leaves the state untouched
  for (int i = threadIdx.x; i < M * ND; i += kBlock) us[i] = dt == 0.0 ? ue[i] : ue[i] + dt * sV[i];
}

// ------------------------------------------------------------ faces

struct FaceArgs {
  Ops ops;
  Geom g;
  const double *trace0;  // side-0 traces of axis A (the + neighbour reads these)
  const double *trace1;  // side-1 traces of axis A
  const double *mat;
  double *GL;            // [E][M][NF] face integral for the element on the - side
  double *GR;            // [E][M][NF] for the element on the + side (non-conservative only)
};

// Path-conservative Rusanov jump term (eqs. pc.scheme, rusanov) at every
// face node and time node of the face between element e (side 1) and its +A
// neighbour (side 0), integrated in time with the GL weights.  One thread
// per (face, face node).
template <int D, int N, class PDE, int A>
__global__ void __launch_bounds__(kBlock) k_face(const FaceArgs F) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NF = S::NF;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= F.g.E * NF) return;
  const int64_t e = t / NF;
  const int kf = (int)(t - e * NF);
  const int64_t eR = neighbour(e, A, +1, F.g.nel);
  const double *tm = F.trace1 + e * (int64_t)(M * ND) + kf;
  const double *tp = F.trace0 + eR * (int64_t)(M * ND) + kf;
  double GL[M], GR[M];
#pragma unroll
  for (int v = 0; v < M; v++) GL[v] = GR[v] = 0.0;
  if constexpr (!PDE::kElastic) {
    const double gamma = F.g.gamma;
    for (int l0 = 0; l0 < n; l0++) {
      double qm[M], qp[M], Fm[M], Fp[M];
#pragma unroll
      for (int v = 0; v < M; v++) {
        qm[v] = tm[(v * n + l0) * NF];
        qp[v] = tp[(v * n + l0) * NF];
      }
      euler_flux<D, A>(qm, gamma - 1.0, Fm);
      euler_flux<D, A>(qp, gamma - 1.0, Fp);
      const double sm = fabs(qm[1 + A] / qm[0]) + sqrt(gamma * euler_pressure<D>(qm, gamma) / qm[0]);
      const double sp = fabs(qp[1 + A] / qp[0]) + sqrt(gamma * euler_pressure<D>(qp, gamma) / qp[0]);
      const double smax = fmax(sm, sp);
      const double wl = F.ops.w[l0];
#pragma unroll
      for (int v = 0; v < M; v++)
        GL[v] += wl * (0.5 * (Fp[v] + Fm[v]) - 0.5 * smax * (qp[v] - qm[v]));
    }
    double *gl = F.GL + e * (int64_t)(M * NF) + kf;
#pragma unroll
    for (int v = 0; v < M; v++) gl[v * NF] = GL[v];
  } else {
    // material path integral with the 3-point Gauss-Legendre rule on [0,1]
    const double rL = F.mat[3 * e], lL = F.mat[3 * e + 1], mL = F.mat[3 * e + 2];
    const double rR = F.mat[3 * eR], lR = F.mat[3 * eR + 1], mR = F.mat[3 * eR + 2];
    const double gs[3] = {0.5 - 0.1 * sqrt(15.0), 0.5, 0.5 + 0.1 * sqrt(15.0)};
    const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    double irho = 0.0, lam = 0.0, mu = 0.0;
#pragma unroll
    for (int g = 0; g < 3; g++) {
      irho += gw[g] / (rL + gs[g] * (rR - rL));
      lam += gw[g] * (lL + gs[g] * (lR - lL));
      mu += gw[g] * (mL + gs[g] * (mR - mL));
    }
    const double smax = fmax(sqrt((lL + 2.0 * mL) / rL), sqrt((lR + 2.0 * mR) / rR));
    for (int l0 = 0; l0 < n; l0++) {
      double dq[M], bd[M];
#pragma unroll
      for (int v = 0; v < M; v++) dq[v] = tp[(v * n + l0) * NF] - tm[(v * n + l0) * NF];
      elastic_bg<A>(dq, irho, lam, mu, bd);
      const double wl = F.ops.w[l0];
#pragma unroll
      for (int v = 0; v < M; v++) {
        GL[v] += wl * (0.5 * (bd[v] - smax * dq[v]));
        GR[v] += wl * (0.5 * (bd[v] + smax * dq[v]));
      }
    }
    double *gl = F.GL + e * (int64_t)(M * NF) + kf;
    double *gr = F.GR + e * (int64_t)(M * NF) + kf;
#pragma unroll
    for (int v = 0; v < M; v++) {
      gl[v * NF] = GL[v];
      gr[v * NF] = GR[v];
    }
  }
}

// ------------------------------------------------------------ update

struct UpdArgs {
  Ops ops;
  Geom g;
  const double *ustar;
  const double *dt;
  const double *GL[3];
  const double *GR[3];
  double *u;
};

// u^{n+1} = u* - dt sum_A (1/h_A) [ L1_kA G_+face + L0_kA G_-face ]  (FP64)
template <int D, int N, class PDE>
__global__ void __launch_bounds__(kBlock) k_update(const UpdArgs U) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NF = S::NF;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= U.g.E * (M * ND)) return;
  const int64_t e = t / (M * ND);
  const int r = (int)(t - e * (M * ND));
  const int v = r / ND, k = r - v * ND;
  double acc = 0.0;
#pragma unroll
  for (int A = 0; A < D; A++) {
    const int ST = ipow(n, A);
    const int ka = (k / ST) % n;
    const int kf = (k % ST) + (k / (ST * n)) * ST;
    const int64_t eL = neighbour(e, A, -1, U.g.nel);
    const double gplus = U.GL[A][e * (M * NF) + v * NF + kf];
    const double gminus = PDE::kConservative ? -U.GL[A][eL * (M * NF) + v * NF + kf]
                                             : U.GR[A][eL * (M * NF) + v * NF + kf];
    acc += U.g.inv_h[A] * (U.ops.L1[ka] * gplus + U.ops.L0[ka] * gminus);
  }
  const double dt = *U.dt;
  U.u[t] = dt == 0.0 ? U.ustar[t] : U.ustar[t] - dt * acc;
}

// ------------------------------------------------------------ time step

struct CflArgs {
  Geom g;
  double h[3];
  const double *u;
  const double *mat;
  unsigned long long *smax_bits;  // max over elements of sum_A lambda_A/h_A (double bits)
  int *err;
};

// One wavefront per element: per-axis maxima of |lambda| over the nodes,
// S_e = sum_A max_A / h_A, then a block max and one atomicMax on the bit
// pattern (order independent: positive doubles order like their bits).
template <int D, int N, class PDE>
__global__ void __launch_bounds__(kBlock) k_cfl(const CflArgs C) {
  using S = Shape<D, N>;
  constexpr int M = PDE::M, ND = S::ND;
  __shared__ double red[kBlock / 64];
  __shared__ int bad_any;
  if (threadIdx.x == 0) bad_any = 0;
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t e = (int64_t)blockIdx.x * (kBlock / 64) + wave;
  double se = 0.0;
  int bad = 0;
  if (e < C.g.E) {
    double lm[3] = {0.0, 0.0, 0.0};
    const double *ue = C.u + e * (int64_t)(M * ND);
    for (int k = lane; k < ND; k += 64) {
      double q[M];
#pragma unroll
      for (int v = 0; v < M; v++) {
        q[v] = ue[v * ND + k];
        if (!isfinite(q[v])) bad = 1;
      }
      if constexpr (!PDE::kElastic) {
        const double p = euler_pressure<D>(q, C.g.gamma);
        if (!(q[0] > 0.0) || !(p > 0.0)) bad = 1;
        const double c = sqrt(C.g.gamma * p / q[0]);
#pragma unroll
        for (int A = 0; A < D; A++) {
          const double l = fabs(q[1 + A] / q[0]) + c;
          if (!(l >= 0.0)) bad = 1;
          lm[A] = fmax(lm[A], l);
        }
      }
    }
    if constexpr (PDE::kElastic) {
      const double cp = sqrt((C.mat[3 * e + 1] + 2.0 * C.mat[3 * e + 2]) / C.mat[3 * e]);
      if (!(cp > 0.0)) bad = 1;
#pragma unroll
      for (int A = 0; A < D; A++) lm[A] = cp;
    }
#pragma unroll
    for (int A = 0; A < D; A++)
      for (int off = 32; off > 0; off >>= 1) lm[A] = fmax(lm[A], __shfl_xor(lm[A], off, 64));
#pragma unroll
    for (int A = 0; A < D; A++) se += lm[A] / C.h[A];
  }
  if (bad) atomicOr(&bad_any, 1);
  if (lane == 0) red[wave] = se;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int i = 1; i < kBlock / 64; i++) m = fmax(m, red[i]);
    atomicMax(C.smax_bits, (unsigned long long)__double_as_longlong(m));
    if (bad_any) atomicOr(C.err, 1);
  }
}

}  // namespace ader
