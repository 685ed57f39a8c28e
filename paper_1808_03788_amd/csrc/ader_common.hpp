// Shared declarations of the ADER-DG library (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ader {

constexpr int kMaxN = 8;      // largest n = N+1
constexpr int kBlock = 256;   // threads per workgroup of the element kernels

// Iterative, so that it always inlines: the recursive form was left as a
// device call in some kernels, with a dynamic stack and spills.
__host__ __device__ __forceinline__ constexpr int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; i++) r *= b;
  return r;
}

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
  double TE[kMaxN * kMaxN];     // TE[p][j]: coefficient of (tau - 1)^p in phi_j(tau) (Taylor
                                // coefficients about the end of the interval, p = 0..N)
};

// Host: build the tables of degree N (0..7).  Returns 0 on success.
int build_ops(int N, Ops *out);
// Host: CFL coefficient alpha_N (1-D von Neumann limit of the scheme).
double stability_alpha(int N);

// Lines of one axis phase of the predictor are assigned to slots (slot s:
// wavefront s / 64, lane s % 64); at most kMaxSlots slots per axis (n^D
// lines rounded up to whole wavefronts, n^D <= 512).  An entry is the LDS
// offset of the line's first node in the space-time element, or
// kEmptySlot.
constexpr int kMaxSlots = 512;
constexpr uint16_t kEmptySlot = 0xffff;
// Host: the slot table of axis A for dimension D and degree N: within every
// wavefront, the line whose base is congruent to r modulo 64 goes to lane
// r where possible, so that the 4-byte (and 8-byte) LDS accesses of a
// phase fall in distinct banks; lines that cannot be placed so take the
// remaining free slots.
void line_slots(int D, int N, int A, uint16_t *out);

// Per-problem geometry/physics handed to the kernels by value.
struct Geom {
  int nel[3];
  double inv_h[3];
  double gamma;
  int64_t E;
};

}  // namespace ader
