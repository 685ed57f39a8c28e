// Shared declarations of the ADER-DG library (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ader {

constexpr int kMaxN = 8;      // largest n = N+1
constexpr int kBlock = 256;   // threads per workgroup of the element kernels

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// 1-D tables of one degree, FP64 (Sec. 2.1: nodal Lagrange basis on the
// Gauss-Legendre points of [0,1]).  Row stride kMaxN.
struct Ops {
  double xi[kMaxN], w[kMaxN];
  double D[kMaxN * kMaxN];   // D[k][j] = phi_j'(xi_k): derivative of the interpolant
  double T[kMaxN * kMaxN];   // predictor time operator K1^{-1} W
  double V[kMaxN * kMaxN];   // volume operator V[k][j] = w_j phi_k'(xi_j) / w_k
  double F0[kMaxN], F1[kMaxN];  // phi_k(0), phi_k(1): face extrapolation
  double L0[kMaxN], L1[kMaxN];  // lifting phi_k(0)/w_k, phi_k(1)/w_k
  double Trow[kMaxN];           // row sums of T (applied to a time-constant right-hand side)
};

// Host: build the tables of degree N (0..7).  Returns 0 on success.
int build_ops(int N, Ops *out);
// Host: CFL coefficient alpha_N (1-D von Neumann limit of the scheme).
double stability_alpha(int N);

// Per-problem geometry/physics handed to the kernels by value.
struct Geom {
  int nel[3];
  double inv_h[3];
  double gamma;
  int64_t E;
};

}  // namespace ader
