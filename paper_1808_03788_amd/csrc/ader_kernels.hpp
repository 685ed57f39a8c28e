// Device kernels of the ADER-DG step, templated on space dimension D,
// degree N and PDE system.  One workgroup owns one element in the predictor;
// the face and update kernels are one thread per face node / per DOF.
#pragma once
#include <type_traits>

#include "ader_common.hpp"

namespace ader {

// Read-only operator tables: loads through the constant address space, so
// that uniform indices become scalar loads even after the kernel has
// written global memory (the tables are never written by a kernel).
template <typename T>
__device__ __forceinline__ T cload(const T *p) {
  if constexpr (__is_arithmetic(T) || __is_pointer(T)) {
    return *(const __attribute__((address_space(4))) T *)p;
  } else {  // argument records: copied word by word
    static_assert(sizeof(T) % 4 == 0, "record size");
    T out;
    const __attribute__((address_space(4))) uint32_t *src = (const __attribute__((address_space(4))) uint32_t *)p;
    uint32_t *dst = (uint32_t *)&out;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); i++) dst[i] = src[i];
    return out;
  }
}

// Buffer pointers read from argument records are generic; accesses through
// these global-address-space views compile to global (not flat) loads and
// stores, with scalar base addresses.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *as_global(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

// Tiles of a batched launch.  Problem p of the batch owns the tiles
// [start[p], start[p+1]); a kernel walks the tiles start[0]..start[np]-1
// with a grid-stride loop (persistent workgroups), so one launch covers any
// number of problems of one kernel class.
struct Batch {
  const int64_t *start;  // device [np + 1]
  int np;
};

// Row-chunk tiles of the face and update kernels, listed explicitly: the
// problem and the chunk's (x-chunk, y, z) position.  A table read replaces
// the search and the integer divisions of the decomposition.
struct RowTile {
  int p;     // problem within the launch's argument records
  int pidx;  // problem index in the context (its dt)
  int bx;    // chunk along the x-row
  uint32_t yz;  // iy | iz << 16 (each < 65536)
};

// The problem that owns `tile` (uniform: binary search on scalar loads).
__device__ __forceinline__ int tile_problem(const Batch &b, int64_t tile) {
  int lo = 0, hi = b.np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cload(&b.start[mid]) <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

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

// 1/x.  FP64: the hardware reciprocal estimate refined by two Newton-Raphson
// steps r <- r + r (1 - x r) (each squares the relative error), which ends
// within about one ulp of the correctly rounded quotient at a third of the
// instructions of an IEEE division; x is a positive normal density here.
// FP32: the hardware reciprocal (1 ulp), where the Picard sweeps are later
// corrected by an FP64 sweep.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Flux F_A(q) of the Euler equations; p = (gamma-1)(rho E - |rho v|^2/(2 rho)).
template <int D, int A, typename R>
__device__ __forceinline__ void euler_flux(const R *q, R gm1, R *F) {
  const R ir = recip(q[0]);
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

// |v_A| + c with one division: 1/rho, then products.
template <int D, int A>
__device__ __forceinline__ double euler_speed(const double *q, double gamma) {
  const double ir = 1.0 / q[0];
  double ke = 0.0;
#pragma unroll
  for (int i = 0; i < D; i++) ke += q[1 + i] * q[1 + i];
  const double p = (gamma - 1.0) * (q[D + 1] - 0.5 * ke * ir);
  return fabs(q[1 + A] * ir) + sqrt(gamma * p * ir);
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

// ------------------------------------------------------------ predictor

// Precision modes of the predictor's Picard sweeps.
enum Prec : int { kFP64 = 0, kFP32 = 1, kBF16 = 2 };

// Sweep operators of one problem, FP64 and FP32 copies, read through a
// device pointer (uniform addresses: scalar loads).  DA[A] = -(1/h_A) Dhat
// carries the mesh width and sign of the axis-A term, so the contraction
// accumulates straight into the right-hand side; T is the time operator and
// Trow its row sums.
struct OpsSweep {
  double DA[3][kMaxN * kMaxN];
  double T[kMaxN * kMaxN];
  double Trow[kMaxN];
  float DAf[3][kMaxN * kMaxN];
  float Tf[kMaxN * kMaxN];
  float Trowf[kMaxN];
  float Dhf[kMaxN * kMaxN];  // unscaled Dhat (MFMA sweeps)
  uint16_t ls[3][kMaxSlots];  // per axis: slot -> line base (line_slots), kEmptySlot if none
  double VA[3][kMaxN * kMaxN];  // (1/h_A) V: volume operator of axis A
  double xi[kMaxN];             // time nodes (initial guesses)
  float xif[kMaxN];
};

struct PredArgs {
  const OpsSweep *sw;   // sweep operators
  const Ops *ops;     // device copy of all FP64 tables (outputs index them per lane)
  Geom g;
  int64_t u_off;        // offset of the problem's u[E][M][ND] in the state buffer
  int64_t q_off;        // offset of its q-hat in the optional q-hat buffer
  int pidx;             // problem index: its time step is dt[pidx]
  const double *mat;    // elastic: [E][3]
  double *ustar;        // [E][M][ND]  u + dt * volume terms
  void *trace[3][2];    // [E][M][n][ND/n] per axis and side (0: x_A = 0, 1: x_A = 1);
                        // double for FP64, float for the mixed modes
  double *acc_glob;     // FP64 accumulator when it does not fit in LDS: [E][M][ACC]
  int sweeps;
  int guess;            // initial guess: 0 constant, 1 MUSCL-Hancock type, 2 third-order Taylor type,
                        // 3 extrapolation of the previous interval
  void *hist;           // guess 3: [E][M][N][ND] Taylor coefficients (orders 1..N) of the last
                        // interval's predictor about its end; double (FP64) or float (mixed)
  const double *dtprev; // guess 3: [nprob] step of that interval
  const int *hist_ok;   // guess 3: the history holds the interval before the state in u
  int face_avg;         // traces as time averages (qbar and, for Euler, Fbar_A) instead of per time node
};

// Values per face node of a time-averaged trace: qbar, and for Euler the
// time-averaged normal flux Fbar_A (the elastic jump term needs qbar only).
template <class PDE>
constexpr int avg_comps() { return PDE::kElastic ? PDE::M : 2 * PDE::M; }
// Argument records are read in place through the constant address space:
// every field load is a scalar load, whatever the kernel has written.
using PArg = const __attribute__((address_space(4))) PredArgs;


template <int D, int N>
struct Shape {
  static constexpr int n = N + 1;
  static constexpr int ND = ipow(n, D);
  static constexpr int NST = ND * n;
  static constexpr int NF = ND / n;   // face nodes
  static constexpr int ACC = (NST > D * ND) ? NST : D * ND;  // also holds D*M*ND output scratch
};

// LDS bytes of the predictor: region A holds the space-time DOFs q in the
// sweep precision (and, in the mixed modes, the output scratch); region R
// the right-hand-side accumulator (and, in the mixed modes, the FP64 final
// iterate).
__host__ __device__ constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }

template <int D, int N, int M, int PREC>
struct PredLds {
  using S = Shape<D, N>;
  // region R starts 256-byte aligned so that its FP64 accesses stay aligned
  static constexpr size_t A = round256(
      PREC == kFP64 ? (size_t)M * S::NST * 8
                    : ((size_t)M * S::NST * 4 > (size_t)D * M * S::ND * 8 ? (size_t)M * S::NST * 4
                                                                            : (size_t)D * M * S::ND * 8));
  // (M * ACC doubles: the space-time accumulator or FP64 iterate, and at
  // least the D per-axis parts of a one-slice right-hand side)
  static constexpr size_t R = round256((size_t)M * S::ACC * 8);
  // FP64 row-group sweeps (elasticity): q in region A, then the stress-row
  // accumulator (M - 3 variables), which also holds the per-axis parts of a
  // one-slice right-hand side and the output scratch
  static constexpr size_t G = round256(
      (size_t)(M - 3) * S::NST * 8 > (size_t)D * M * S::ND * 8 ? (size_t)(M - 3) * S::NST * 8
                                                                : (size_t)D * M * S::ND * 8);
};

// Threads per workgroup of the predictor: the number of lines of one axis
// phase (n^D) rounded up to whole wavefronts, times a tuning factor (1 or
// 2), at most 256, or 512 when a phase has more than 256 lines (one line
// per thread with factor 2; these elements fill most of the LDS, so a
// single workgroup per CU needs the larger block).  Factor kSplitLines
// (elasticity): two threads per line, one for the velocity rows and one for
// the stress rows of the right-hand side, each half of the block n^D
// rounded up to whole wavefronts.
constexpr int kSplitLines = 4;
// Factor kRowGroups (FP64 elasticity): one thread per line, the two row
// groups of a sweep one after the other (elastic_group_sweep).
constexpr int kRowGroups = 8;
__host__ __device__ constexpr int round64(int x) { return (x + 63) / 64 * 64; }
// Factor kWide (elements with more than 128 lines per axis phase, whose LDS
// footprint leaves one or two workgroups per CU): 512 threads (1024 above
// 256 lines), four wavefronts per SIMD instead of two, and room to pair
// two axis phases.
constexpr int kWide = 16;
__host__ __device__ constexpr int pred_block_cap(int D, int N) { return ipow(N + 1, D) > 256 ? 512 : 256; }
__host__ __device__ constexpr int pred_block(int D, int N, int factor = 1) {
  return factor == kWide ? (ipow(N + 1, D) > 256 ? 1024 : (ipow(N + 1, D) > 128 ? 512 : pred_block(D, N, 2)))
         : factor == kRowGroups ? pred_block(D, N, 1)
         : factor == kSplitLines
             ? 2 * round64(ipow(N + 1, D))
             : ((ipow(N + 1, D) <= 64 ? 64 : (ipow(N + 1, D) <= 128 ? 128 : 256)) * factor > pred_block_cap(D, N)
                    ? pred_block_cap(D, N)
                    : (ipow(N + 1, D) <= 64 ? 64 : (ipow(N + 1, D) <= 128 ? 128 : 256)) * factor);
}

// Rows of the elastic right-hand side along axis A that one line task
// computes: kPart 0 all of them; 1 the velocity rows, which need only the
// gradients of the three stress components sig(i, A); 2 the stress rows,
// which need only the velocity gradients.
template <class PDE, int A, int kPart>
__device__ __forceinline__ constexpr bool part_reads(int v) {
  return kPart == 0 || (kPart == 1 ? (v == sig(0, A) || v == sig(1, A) || v == sig(2, A)) : v < 3);
}
template <int kPart>
__device__ __forceinline__ constexpr bool part_writes(int v) {
  return kPart == 0 || (kPart == 1 ? v < 3 : v >= 3);
}

template <typename T>
__device__ __forceinline__ T opD(PArg &P, int A, int i);
template <>
__device__ __forceinline__ double opD<double>(PArg &P, int A, int i) { return cload(&P.sw->DA[A][i]); }
template <>
__device__ __forceinline__ float opD<float>(PArg &P, int A, int i) { return cload(&P.sw->DAf[A][i]); }
// Round to the nearest bfloat16 (ties to even), kept in a float register.
__device__ __forceinline__ float round_bf16(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7fffu + ((b >> 16) & 1u);
  return __uint_as_float(b & 0xffff0000u);
}

// Collocated right-hand side along axis A on one line of n nodes (starting
// at offset `base`, stride n^A; variables VS apart), in arithmetic T, reading
// q stored as TQ:
//   R -= (1/h_A) Dhat_A F_A(q)           (Euler)
//   R -= (1/h_A) B_A (Dhat_A q)          (elasticity)
// With kAcc the result is added to the values already in sacc, else it is
// stored.  With kRoundBF the contraction inputs are rounded to bfloat16.
// kPart (elasticity only) restricts the line to one row group; variable v
// of the accumulator is held at (v - kAccShift) * VS.  With kHold the n x M
// results go to held[k * M + v] (registers of the caller) instead of sacc.
// The accumulator is stored as TA (T, or FP32 partial sums of the FP64
// residual sweep).  Only the output nodes KLO <= k < KHI of the line are
// computed (the flux still at all n nodes).
template <int D, int N, class PDE, int A, typename T, typename TQ, bool kRoundBF, int VS, bool kAcc, int kPart = 0,
          int kAccShift = 0, bool kHold = false, typename TA = T, int KLO = 0, int KHI = N + 1>
__device__ __forceinline__ void line_rhs(PArg &P, const TQ *sq, TA *sacc, int base, T irho, T lam, T mu,
                                         T *held = nullptr) {
  constexpr int n = N + 1, M = PDE::M;
  constexpr int ST = ipow(n, A);
  static_assert(kPart == 0 || PDE::kElastic, "row groups are an elasticity split");
  T qv[n][M];
#pragma unroll
  for (int j = 0; j < n; j++)
#pragma unroll
    for (int v = 0; v < M; v++) qv[j][v] = part_reads<PDE, A, kPart>(v) ? (T)sq[v * VS + base + j * ST] : T(0);
  // the accumulated right-hand side of the earlier axes
  T acc[n][M];
#pragma unroll
  for (int k = KLO; k < KHI; k++)
#pragma unroll
    for (int v = 0; v < M; v++)
      acc[k][v] = (kAcc && part_writes<kPart>(v)) ? (T)sacc[(v - kAccShift) * VS + base + k * ST] : T(0);
  if constexpr (!PDE::kElastic) {
    T F[n][M];
#pragma unroll
    for (int j = 0; j < n; j++) {
      euler_flux<D, A, T>(qv[j], (T)(P.g.gamma - 1.0), F[j]);
      if constexpr (kRoundBF)
#pragma unroll
        for (int v = 0; v < M; v++) F[j][v] = round_bf16(F[j][v]);
    }
#pragma unroll
    for (int k = KLO; k < KHI; k++)
#pragma unroll
      for (int v = 0; v < M; v++)
#pragma unroll
        for (int j = 0; j < n; j++) acc[k][v] += opD<T>(P, A, k * kMaxN + j) * F[j][v];
  } else {
    if constexpr (kRoundBF)
#pragma unroll
      for (int j = 0; j < n; j++)
#pragma unroll
        for (int v = 0; v < M; v++) qv[j][v] = round_bf16(qv[j][v]);
#pragma unroll
    for (int k = KLO; k < KHI; k++) {
      T gk[M], bg[M];
#pragma unroll
      for (int v = 0; v < M; v++) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < n; j++) s += opD<T>(P, A, k * kMaxN + j) * qv[j][v];
        gk[v] = s;
      }
      elastic_bg<A, T>(gk, irho, lam, mu, bg);
#pragma unroll
      for (int v = 0; v < M; v++) acc[k][v] += bg[v];
    }
  }
#pragma unroll
  for (int k = KLO; k < KHI; k++)
#pragma unroll
    for (int v = 0; v < M; v++) {
      if constexpr (kHold)
        held[k * M + v] = acc[k][v];
      else if (part_writes<kPart>(v))
        sacc[(v - kAccShift) * VS + base + k * ST] = (TA)acc[k][v];
    }
}

// Lines of an axis phase in slots: slot s of axis A holds the line whose
// first node sits at P.sw->ls[A][s] (the slot tables of line_slots), so
// that the lanes of a wavefront hit distinct LDS banks; n^D lines in
// round64(n^D) slots.
template <int D, int N>
__host__ __device__ constexpr int line_slots_count() { return round64(ipow(N + 1, D)); }
// Degrees whose slot tables differ from the plain line order by enough to
// matter (from a model of the bank conflicts of each order: at n = 4 and
// n = 8 no order of the lines removes them); the others use the plain
// order, computed, and keep no table.
template <int D, int N>
__host__ __device__ constexpr bool slot_tables() {
  return D == 3 ? (N == 2 || N == 4 || N == 5 || N == 6) : (N >= 3 && N <= 6);
}
// The predictor copies the slot tables of its problem into the first
// slot_table_bytes of its LDS (the regions A and R follow them).
template <int D, int N>
__host__ __device__ constexpr size_t slot_table_bytes() {
  return slot_tables<D, N>() ? round256((size_t)3 * line_slots_count<D, N>() * 2) : 0;
}
template <int D, int N, int A>
__device__ __forceinline__ int slot_base(int s) {
  if constexpr (slot_tables<D, N>()) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    return ((const uint16_t *)smem_raw)[A * line_slots_count<D, N>() + s];
  } else {  // plain order: line s is (time slice s / NF, face index s % NF over the other axes)
    using S = Shape<D, N>;
    constexpr int ST = ipow(N + 1, A);
    if (s >= S::ND) return kEmptySlot;
    const int l0 = s / S::NF, r = s - l0 * S::NF;
    return l0 * S::ND + r % ST + (r / ST) * ST * S::n;
  }
}

// The axis that runs alone after the paired axes, adding to the first
// accumulator: the one whose slot order leaves the fewest LDS bank
// conflicts for its three accesses (read q, read and write the
// accumulator), from a model of the slot tables (-1 in 2-D: no third axis).
__host__ __device__ constexpr int third_axis(int D, int N) {
  return D < 3 ? -1 : ((N == 3 || N == 5 || N == 7) ? 2 : 0);
}

// Right-hand side along axis A for all lines of the space-time element
// (one thread per slot), stored (kAcc false) or accumulated onto the
// earlier axes.  With kSplit (elasticity, BS = 2 * slots) the first half of
// the block takes the velocity rows of every line and the second half the
// stress rows (whole wavefronts on each side).
template <int D, int N, class PDE, int A, typename T, typename TQ, bool kRoundBF, int BS, bool kSplit = false,
          bool kAcc = (A > 0), typename TA = T, bool kHalfK = false>
__device__ __forceinline__ void rhs_axis(PArg &P, const TQ *sq, TA *sacc, T irho, T lam, T mu) {
  constexpr int NS = line_slots_count<D, N>(), NST = Shape<D, N>::NST;
  if constexpr (kHalfK) {
    // two threads per line, on two halves of whole wavefronts: the first
    // computes the output nodes k < KH, the second the others (both
    // evaluate the line's fluxes)
    static_assert(!kSplit && BS >= 2 * NS, "two halves of whole wavefronts");
    constexpr int KH = (N + 2) / 2;
    const int half = threadIdx.x / NS, L = threadIdx.x - half * NS;
    const int base = half < 2 ? slot_base<D, N, A>(L) : (int)kEmptySlot;
    if (base != kEmptySlot) {
      if (half == 0)
        line_rhs<D, N, PDE, A, T, TQ, kRoundBF, NST, kAcc, 0, 0, false, TA, 0, KH>(P, sq, sacc, base, irho, lam, mu);
      else
        line_rhs<D, N, PDE, A, T, TQ, kRoundBF, NST, kAcc, 0, 0, false, TA, KH, N + 1>(P, sq, sacc, base, irho, lam,
                                                                                       mu);
    }
  } else if constexpr (kSplit) {
    static_assert(BS == 2 * NS && PDE::kElastic, "two threads per line");
    const int half = threadIdx.x / NS, L = threadIdx.x - half * NS;
    const int base = slot_base<D, N, A>(L);
    if (base != kEmptySlot) {
      if (half == 0)
        line_rhs<D, N, PDE, A, T, TQ, kRoundBF, NST, kAcc, 1>(P, sq, sacc, base, irho, lam, mu);
      else
        line_rhs<D, N, PDE, A, T, TQ, kRoundBF, NST, kAcc, 2>(P, sq, sacc, base, irho, lam, mu);
    }
  } else {
    for (int L = threadIdx.x; L < NS; L += BS) {
      const int base = slot_base<D, N, A>(L);
      if (base != kEmptySlot)
        line_rhs<D, N, PDE, A, T, TQ, kRoundBF, NST, kAcc, 0, 0, false, TA>(P, sq, sacc, base, irho, lam, mu);
    }
  }
}

// The right-hand side of a time-constant state w (compact [M][ND]) on one
// time slice, all axes at once: wavefront W takes the lines of axis W (and
// W + BS/64, ...), one lane per line (n^(D-1) <= 64 lines per axis), and
// stores that axis's contribution in part[A][M][ND]; the sum over A is left
// to the consumer.  With kSplit (elasticity) the tasks are (axis, row
// group) pairs, wavefront W taking task W, W + BS/64, ...
template <int D, int N, class PDE, int A, typename T, bool kRoundBF, int kPart>
__device__ __forceinline__ void slice_lines(PArg &P, const T *w, T *part, int L, T irho, T lam, T mu) {
  constexpr int n = N + 1, M = PDE::M, ND = ipow(n, D);
  constexpr int ST = ipow(n, A);
  const int base = L % ST + (L / ST) * ST * n;
  line_rhs<D, N, PDE, A, T, T, kRoundBF, ND, false, kPart>(P, w, part + A * M * ND, base, irho, lam, mu);
}

template <int D, int N, class PDE, int A, typename T, bool kRoundBF, bool kSplit>
__device__ __forceinline__ void slice_task(PArg &P, const T *w, T *part, int L, int g, T irho, T lam, T mu) {
  if constexpr (kSplit) {
    if (g == 1)
      slice_lines<D, N, PDE, A, T, kRoundBF, 1>(P, w, part, L, irho, lam, mu);
    else
      slice_lines<D, N, PDE, A, T, kRoundBF, 2>(P, w, part, L, irho, lam, mu);
  } else {
    slice_lines<D, N, PDE, A, T, kRoundBF, 0>(P, w, part, L, irho, lam, mu);
  }
}

template <int D, int N, class PDE, typename T, bool kRoundBF, int BS, bool kSplit = false>
__device__ __forceinline__ void rhs_slice(PArg &P, const T *w, T *part, T irho, T lam, T mu) {
  using S = Shape<D, N>;
  constexpr int NF = S::NF;
  static_assert(NF <= 64, "one wavefront per axis");
  constexpr int NT = kSplit ? 2 * D : D;  // tasks
  const int wave = threadIdx.x >> 6, L = threadIdx.x & 63;
  for (int t = wave; t < NT; t += BS / 64) {
    if (L < NF) {
      const int A = kSplit ? t >> 1 : t;
      const int g = kSplit ? 1 + (t & 1) : 0;
      if (A == 0) {
        slice_task<D, N, PDE, 0, T, kRoundBF, kSplit>(P, w, part, L, g, irho, lam, mu);
      } else if (A == 1) {
        if constexpr (D > 1) slice_task<D, N, PDE, 1, T, kRoundBF, kSplit>(P, w, part, L, g, irho, lam, mu);
      } else {
        if constexpr (D > 2) slice_task<D, N, PDE, 2, T, kRoundBF, kSplit>(P, w, part, L, g, irho, lam, mu);
      }
    }
  }
}

// Number of (v,k) time lines each thread owns in the time phase.
template <int D, int N, int M, int BS>
struct TimeItems {
  static constexpr int value = (M * ipow(N + 1, D) + BS - 1) / BS;
};

// Time contraction q(l0,k) = u(k) + dt sum_j0 T[l0][j0] R(j0,k), in arithmetic
// T, writing q as TO (may alias R: every thread reads its whole time line
// before writing it back).  Thread tid owns the time lines tid + r*BS, whose
// u values it keeps in ureg[r] across sweeps.
template <typename T>
__device__ __forceinline__ T opT(PArg &P, int i);
template <>
__device__ __forceinline__ double opT<double>(PArg &P, int i) { return cload(&P.sw->T[i]); }
template <>
__device__ __forceinline__ float opT<float>(PArg &P, int i) { return cload(&P.sw->Tf[i]); }
template <typename T>
__device__ __forceinline__ T opTrow(PArg &P, int l);
template <>
__device__ __forceinline__ double opTrow<double>(PArg &P, int l) { return cload(&P.sw->Trow[l]); }
template <>
__device__ __forceinline__ float opTrow<float>(PArg &P, int l) { return cload(&P.sw->Trowf[l]); }

template <int D, int N, class PDE, typename T, typename TO, int BS, bool kTwo = false, typename TA = T>
__device__ __forceinline__ void time_phase(PArg &P, const TA *sacc, TO *qout, const double *ureg, T dt,
                                           const TA *sacc2 = nullptr) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST;
  constexpr int NU = TimeItems<D, N, M, BS>::value;
  // a wider iterate written over narrower partial sums (the FP64 iterate of
  // the residual sweep over its FP32 accumulators) overlaps the values other
  // threads still read: every thread reads first, then writes after a barrier
  constexpr bool kWiden = sizeof(TO) > sizeof(TA);
  T rr[kWiden ? NU : 1][n];
#pragma unroll
  for (int r = 0; r < NU; r++) {
    const int i = threadIdx.x + r * BS;
    const int rs = kWiden ? r : 0;
    if (i < M * ND) {
      const int v = i / ND, k = i - v * ND;
#pragma unroll
      for (int j = 0; j < n; j++) {
        rr[rs][j] = (T)sacc[v * NST + j * ND + k];
        if constexpr (kTwo) rr[rs][j] += (T)sacc2[v * NST + j * ND + k];
      }
    }
    if constexpr (!kWiden) {
      if (i < M * ND) {
        const int v = i / ND, k = i - v * ND;
        const T u0 = (T)ureg[r];
#pragma unroll
        for (int l = 0; l < n; l++) {
          T a = T(0);
#pragma unroll
          for (int j = 0; j < n; j++) a += opT<T>(P, l * kMaxN + j) * rr[0][j];
          qout[v * NST + l * ND + k] = (TO)(u0 + dt * a);
        }
      }
    }
  }
  if constexpr (kWiden) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NU; r++) {
      const int i = threadIdx.x + r * BS;
      if (i < M * ND) {
        const int v = i / ND, k = i - v * ND;
        const T u0 = (T)ureg[r];
#pragma unroll
        for (int l = 0; l < n; l++) {
          T a = T(0);
#pragma unroll
          for (int j = 0; j < n; j++) a += opT<T>(P, l * kMaxN + j) * rr[r][j];
          qout[v * NST + l * ND + k] = (TO)(u0 + dt * a);
        }
      }
    }
  }
}

// Sum of the D per-axis parts of a one-slice right-hand side for the
// values this thread owns (ureg layout: i = threadIdx.x + r*BS).
template <int D, int N, class PDE, typename T, int BS>
__device__ __forceinline__ void gather_parts(const T *part, T (&out)[TimeItems<D, N, PDE::M, BS>::value]) {
  constexpr int M = PDE::M, ND = Shape<D, N>::ND;
  constexpr int NU = TimeItems<D, N, M, BS>::value;
#pragma unroll
  for (int r = 0; r < NU; r++) {
    const int i = threadIdx.x + r * BS;
    T a = T(0);
    if (i < M * ND)
#pragma unroll
      for (int A = 0; A < D; A++) a += part[A * M * ND + i];
    out[r] = a;
  }
}

// Whether a block of BS threads holds the lines of two axes at once, each
// set on its own half of whole wavefronts (one thread per slot).
template <int D, int N, int BS>
__host__ __device__ constexpr bool pair_axes() {
  return D >= 2 && BS >= 2 * round64(ipow(N + 1, D));
}
// The two axes of the pair: the ones other than third_axis (0 and 1 in 2-D).
template <int D, int N>
__host__ __device__ constexpr int pair_a() { return third_axis(D, N) == 0 ? 1 : 0; }
template <int D, int N>
__host__ __device__ constexpr int pair_b() { return third_axis(D, N) == 2 || D < 3 ? 1 : 2; }

// The paired axes at the same time: the first half of the block stores the
// lines of axis pair_a into sacc, the second half those of axis pair_b into
// sacc2 (the time phase adds the two).
template <int D, int N, class PDE, typename T, typename TQ, bool kRoundBF, int BS, typename TA = T>
__device__ __forceinline__ void rhs_pair(PArg &P, const TQ *sq, TA *sacc, TA *sacc2, T irho, T lam, T mu) {
  constexpr int NS = line_slots_count<D, N>(), NST = Shape<D, N>::NST;
  constexpr int a = pair_a<D, N>(), b = pair_b<D, N>();
  static_assert(pair_axes<D, N, BS>(), "two halves of whole wavefronts");
  const int half = threadIdx.x / NS, L = threadIdx.x - half * NS;
  if (half == 0) {
    const int base = slot_base<D, N, a>(L);
    if (base != kEmptySlot)
      line_rhs<D, N, PDE, a, T, TQ, kRoundBF, NST, false, 0, 0, false, TA>(P, sq, sacc, base, irho, lam, mu);
  } else if (half == 1) {
    const int base = slot_base<D, N, b>(L);
    if (base != kEmptySlot)
      line_rhs<D, N, PDE, b, T, TQ, kRoundBF, NST, false, 0, 0, false, TA>(P, sq, sacc2, base, irho, lam, mu);
  }
}

// The paired axes with one accumulator: the first half of the block stores
// the lines of axis pair_a into sacc while the second half computes those of
// axis pair_b into registers, and adds them after a barrier (used where
// region R has no room for a second accumulator).
template <int D, int N, class PDE, typename T, typename TQ, bool kRoundBF, int BS>
__device__ __forceinline__ void rhs_pair_held(PArg &P, const TQ *sq, T *sacc, T irho, T lam, T mu) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, NST = S::NST;
  constexpr int NS = line_slots_count<D, N>();
  constexpr int a = pair_a<D, N>(), b = pair_b<D, N>();
  constexpr int STb = ipow(n, b);
  static_assert(pair_axes<D, N, BS>(), "two halves of whole wavefronts");
  const int half = threadIdx.x / NS, L = threadIdx.x - half * NS;
  const int base = half == 0 ? slot_base<D, N, a>(L) : (half == 1 ? slot_base<D, N, b>(L) : (int)kEmptySlot);
  const bool active = base != kEmptySlot;
  T held[n * M];
  if (active) {
    if (half == 0)
      line_rhs<D, N, PDE, a, T, TQ, kRoundBF, NST, false>(P, sq, sacc, base, irho, lam, mu);
    else
      line_rhs<D, N, PDE, b, T, TQ, kRoundBF, NST, false, 0, 0, true>(P, sq, sacc, base, irho, lam, mu, held);
  }
  __syncthreads();
  if (active && half == 1)
#pragma unroll
    for (int k = 0; k < n; k++)
#pragma unroll
      for (int v = 0; v < M; v++) sacc[v * NST + base + k * STb] += held[k * M + v];
}

// One Picard sweep: R(q) over all axes, then the time contraction.  With
// kPair (pair_axes) the axes pair_a and pair_b run at the same time:
// kPairTwo with a second accumulator sacc2 of M NST values, kPairHeld with
// the pair_b results held in registers; third_axis then accumulates onto
// sacc.
constexpr int kPairTwo = 1, kPairHeld = 2;
template <int D, int N, class PDE, typename T, typename TQ, typename TO, bool kRoundBF, int BS, bool kSplit = false,
          int kPair = 0, typename TA = T>
__device__ __forceinline__ void picard_sweep(PArg &P, const TQ *sq, TA *sacc, TO *qout,
                                             const double *ureg, T dt, T irho, T lam, T mu, TA *sacc2 = nullptr) {
  static_assert(std::is_same<TA, T>::value || kPair != kPairHeld, "narrow accumulators are not held");
  if constexpr (kPair != 0) {
    static_assert(!kSplit, "one thread per line");
    if constexpr (kPair == kPairTwo)
      rhs_pair<D, N, PDE, T, TQ, kRoundBF, BS, TA>(P, sq, sacc, sacc2, irho, lam, mu);
    else
      rhs_pair_held<D, N, PDE, T, TQ, kRoundBF, BS>(P, sq, sacc, irho, lam, mu);
    __syncthreads();
    if constexpr (D > 2) {
      // the third axis alone: its lines split by output nodes over the
      // whole block (not in the 512/1024-thread blocks, whose 128
      // registers would spill)
      rhs_axis<D, N, PDE, third_axis(D, N), T, TQ, kRoundBF, BS, false, true, TA, (BS <= 256)>(P, sq, sacc, irho, lam,
                                                                                              mu);
      __syncthreads();
    }
    time_phase<D, N, PDE, T, TO, BS, kPair == kPairTwo, TA>(P, sacc, qout, ureg, dt, sacc2);
    __syncthreads();
    return;
  }
  rhs_axis<D, N, PDE, 0, T, TQ, kRoundBF, BS, kSplit, false, TA>(P, sq, sacc, irho, lam, mu);
  __syncthreads();
  if constexpr (D > 1) {
    rhs_axis<D, N, PDE, 1, T, TQ, kRoundBF, BS, kSplit, true, TA>(P, sq, sacc, irho, lam, mu);
    __syncthreads();
  }
  if constexpr (D > 2) {
    rhs_axis<D, N, PDE, 2, T, TQ, kRoundBF, BS, kSplit, true, TA>(P, sq, sacc, irho, lam, mu);
    __syncthreads();
  }
  time_phase<D, N, PDE, T, TO, BS, false, TA>(P, sacc, qout, ureg, dt);
  __syncthreads();
}

// Lines of axis A for one row group kPart, one thread per line, accumulator
// variable v at (v - kShift) * NST of sacc.
template <int D, int N, class PDE, int A, int kPart, int kShift, int BS>
__device__ __forceinline__ void rhs_axis_group(PArg &P, const double *sq, double *sacc, double irho, double lam,
                                               double mu) {
  using S = Shape<D, N>;
  constexpr int NST = S::NST, NS = line_slots_count<D, N>();
  for (int L = threadIdx.x; L < NS; L += BS) {
    const int base = slot_base<D, N, A>(L);
    if (base != kEmptySlot)
      line_rhs<D, N, PDE, A, double, double, false, NST, (A > 0), kPart, kShift>(P, sq, sacc, base, irho, lam, mu);
  }
}

// Time contraction of the variables v0 <= v < v1 only: q(l0, k) = u(k) +
// dt sum_j0 T[l0][j0] R(j0, k), R of variable v at (v - shift) * NST of
// sacc, written to (v - shift) * NST of qout (same owners as time_phase).
template <int D, int N, class PDE, int BS>
__device__ __forceinline__ void time_phase_vars(PArg &P, const double *sacc, double *qout, int shift,
                                                const double *ureg, double dt, int v0, int v1) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST;
  constexpr int NU = TimeItems<D, N, M, BS>::value;
#pragma unroll
  for (int r = 0; r < NU; r++) {
    const int i = threadIdx.x + r * BS;
    const int v = i / ND, k = i - v * ND;
    if (i < M * ND && v >= v0 && v < v1) {
      double rr[n];
#pragma unroll
      for (int j = 0; j < n; j++) rr[j] = sacc[(v - shift) * NST + j * ND + k];
#pragma unroll
      for (int l = 0; l < n; l++) {
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < n; j++) a += opT<double>(P, l * kMaxN + j) * rr[j];
        qout[(v - shift) * NST + l * ND + k] = ureg[r] + dt * a;
      }
    }
  }
}

// One FP64 elastic Picard sweep by row groups, in LDS q ([M][NST]) plus an
// accumulator sS of the M-3 stress variables.  The stress rows need only
// the velocity gradients and the velocity rows only the stress gradients,
// so: (1) the stress rows into sS, time-contracted there; (2) the velocity
// rows into the velocity slots of q (their old values are no longer read),
// time-contracted in place, from the old stresses still in q; (3) the new
// stresses copied into q.  Every row is a function of the previous iterate,
// as in picard_sweep.
template <int D, int N, class PDE, int BS>
__device__ __forceinline__ void elastic_group_sweep(PArg &P, double *sq, double *sS, const double *ureg,
                                                    double dt, double irho, double lam, double mu) {
  static_assert(PDE::kElastic && D == 3, "row groups: 3-D elasticity");
  constexpr int M = PDE::M, NST = Shape<D, N>::NST;
  rhs_axis_group<D, N, PDE, 0, 2, 3, BS>(P, sq, sS, irho, lam, mu);
  __syncthreads();
  rhs_axis_group<D, N, PDE, 1, 2, 3, BS>(P, sq, sS, irho, lam, mu);
  __syncthreads();
  rhs_axis_group<D, N, PDE, 2, 2, 3, BS>(P, sq, sS, irho, lam, mu);
  __syncthreads();
  time_phase_vars<D, N, PDE, BS>(P, sS, sS, 3, ureg, dt, 3, M);
  rhs_axis_group<D, N, PDE, 0, 1, 0, BS>(P, sq, sq, irho, lam, mu);
  __syncthreads();
  rhs_axis_group<D, N, PDE, 1, 1, 0, BS>(P, sq, sq, irho, lam, mu);
  __syncthreads();
  rhs_axis_group<D, N, PDE, 2, 1, 0, BS>(P, sq, sq, irho, lam, mu);
  __syncthreads();
  time_phase_vars<D, N, PDE, BS>(P, sq, sq, 0, ureg, dt, 0, 3);
  for (int i = threadIdx.x; i < (M - 3) * NST; i += BS) sq[3 * NST + i] = sS[i];
  __syncthreads();
}

// The first sweep from the time-constant iterate q^0 = u (compact [M][ND]
// in w): R is the same at every time node, so it is evaluated on one time
// slice (D per-axis parts in `part`, D M ND values) and the time operator
// reduces to its row sums -- the same values as a full sweep up to rounding.
// The sums are taken into registers before any write, so qout may overlap
// `part`.
template <int D, int N, class PDE, typename T, typename TO, bool kRoundBF, int BS, bool kSplit = false>
__device__ __forceinline__ void first_sweep(PArg &P, const T *w, T *part, TO *qout, const double *ureg, T dt,
                                            T irho, T lam, T mu) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST;
  constexpr int NU = TimeItems<D, N, M, BS>::value;
  rhs_slice<D, N, PDE, T, kRoundBF, BS, kSplit>(P, w, part, irho, lam, mu);
  __syncthreads();
  T r0[NU];
  gather_parts<D, N, PDE, T, BS>(part, r0);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NU; r++) {
    const int i = threadIdx.x + r * BS;
    if (i < M * ND) {
      const int v = i / ND, k = i - v * ND;
      const T u0 = (T)ureg[r];
#pragma unroll
      for (int l = 0; l < n; l++) qout[v * NST + l * ND + k] = (TO)(u0 + dt * (opTrow<T>(P, l) * r0[r]));
    }
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ T opXi(PArg &P, int l);
template <>
__device__ __forceinline__ double opXi<double>(PArg &P, int l) { return cload(&P.sw->xi[l]); }
template <>
__device__ __forceinline__ float opXi<float>(PArg &P, int l) { return cload(&P.sw->xif[l]); }

// Initial guess of the Picard iteration (Sec. 2.2), as a Taylor polynomial
// in t - t^n = xi_l dt evaluated at the time nodes:
//   guess 1: q0 = u + (t - t^n) k1,                                  k1 = L(u)
//   guess 2: q0 = u + (t - t^n) k1 + (t - t^n)^2 (k2 - k1) / (2 dt),  k2 = L(u + dt k1).
// On entry sq holds u in the compact [M][ND] layout, on exit the guess in
// the space-time layout [M][n][ND]; sk is scratch for D M ND values that
// does not overlap sq.
template <int D, int N, class PDE, typename T, bool kRoundBF, int BS, bool kSplit = false>
__device__ __forceinline__ void initial_guess(PArg &P, T *sq, T *sk, const double *ureg, T dt, T irho, T lam,
                                              T mu) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST;
  constexpr int NU = TimeItems<D, N, M, BS>::value;
  rhs_slice<D, N, PDE, T, kRoundBF, BS, kSplit>(P, sq, sk, irho, lam, mu);
  __syncthreads();
  T k1[NU], c2[NU];
  gather_parts<D, N, PDE, T, BS>(sk, k1);
  const bool third = P.guess == 2;
  if (third) {
#pragma unroll
    for (int r = 0; r < NU; r++) {
      const int i = threadIdx.x + r * BS;
      if (i < M * ND) sq[i] = (T)ureg[r] + dt * k1[r];
    }
    __syncthreads();
    rhs_slice<D, N, PDE, T, kRoundBF, BS, kSplit>(P, sq, sk, irho, lam, mu);
    __syncthreads();
    gather_parts<D, N, PDE, T, BS>(sk, c2);
#pragma unroll
    for (int r = 0; r < NU; r++) c2[r] = T(0.5) * (c2[r] - k1[r]);
  } else {
#pragma unroll
    for (int r = 0; r < NU; r++) c2[r] = T(0);
  }
#pragma unroll
  for (int r = 0; r < NU; r++) {
    const int i = threadIdx.x + r * BS;
    if (i < M * ND) {
      const int v = i / ND, k = i - v * ND;
      const T u0 = (T)ureg[r];
#pragma unroll
      for (int l = 0; l < n; l++) {
        const T x = opXi<T>(P, l);
        sq[v * NST + l * ND + k] = u0 + dt * (x * k1[r] + x * x * c2[r]);
      }
    }
  }
  __syncthreads();
}

// Initial guess 3 (Sec. 2.2: extrapolation of q_h from the previous time
// interval): the previous interval's predictor, continued to the new time
// nodes and shifted to start at the corrected state,
//   q0(l, k) = u(k) + sum_{p=1..N} c_p(k) (xi_l r)^p,   r = dt / dt_prev,
// c_p the Taylor coefficients of that predictor about the end of its
// interval (written by write_history).  Fills sq in the space-time layout
// from the u values each thread holds.
template <int D, int N, class PDE, typename T, int BS, typename TH>
__device__ __forceinline__ void extrap_guess(PArg &P, T *sq, const double *ureg, const TH *he, T r) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST;
  constexpr int NU = TimeItems<D, N, M, BS>::value;
#pragma unroll
  for (int it = 0; it < NU; it++) {
    const int i = threadIdx.x + it * BS;
    if (i < M * ND) {
      const int v = i / ND, k = i - v * ND;
      T c[N > 0 ? N : 1];
#pragma unroll
      for (int p = 0; p < N; p++) c[p] = (T)he[(v * N + p) * ND + k];
      const T u0 = (T)ureg[it];
#pragma unroll
      for (int l = 0; l < n; l++) {
        const T x = opXi<T>(P, l) * r;
        T acc = u0, xp = x;
#pragma unroll
        for (int p = 0; p < N; p++) {
          acc += c[p] * xp;
          xp *= x;
        }
        sq[v * NST + l * ND + k] = acc;
      }
    }
  }
}

// Taylor coefficients (orders 1..N) about the end of the interval of the
// final predictor qf, stored as TH for the next step's guess 3.
template <int D, int N, class PDE, typename TH, int BS>
__device__ __forceinline__ void write_history(PArg &P, const double *qf, int64_t e) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST;
  if constexpr (N > 0) {
    auto *he = as_global((TH *)P.hist + e * (int64_t)(M * N * ND));
    for (int i = threadIdx.x; i < M * ND; i += BS) {
      const int v = i / ND, k = i - v * ND;
      double q[n];
#pragma unroll
      for (int j = 0; j < n; j++) q[j] = qf[v * NST + j * ND + k];
#pragma unroll
      for (int p = 1; p <= N; p++) {
        double c = 0.0;
#pragma unroll
        for (int j = 0; j < n; j++) c += cload(&P.ops->TE[p * kMaxN + j]) * q[j];
        he[(v * N + p - 1) * ND + k] = (TH)c;
      }
    }
  }
}

// ---------------------------------------------------------------- MFMA sweep
//
// FP32 Picard sweep whose operator contractions run on v_mfma_f32_4x4x1_16b:
// 16 independent 4x4 outer-product blocks per instruction.  Lane 4b+i of a
// wavefront supplies row i of block b (A operand), lane 4b+j supplies column
// j (B operand); the 4x4 result of block b lands in lane 4b+j, register i.
// Every lane owns one line (n nodes of one axis, all M variables) and feeds
// its own value at node j as B; the A operand of lane 4b+i is the operator
// entry Op[4c+i][j].  One instruction per node j (K = 1, no padding) and per
// group c of four output rows thus leaves out[k = 4c+i] = sum_j Op[k][j] X[j]
// of the lane's own line in register i: no data moves between lanes.
//
// Output rows go in groups of four to the matrix cores while a group is at
// least 3/4 full; the rest (one row at n = 5, two at n = 6) is computed on
// VALU FMAs with the operator row as a scalar operand, concurrently with
// the matrix cores.  The MFMA accumulators start from the value to add (the
// earlier axes' sum, or u in the time contraction), so no extra add is
// needed.

typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));  // four bfloat16 values

// BF16 variant of the spatial contractions: v_mfma_f32_4x4x4bf16_1k takes
// four bfloat16 values of K per lane, A[i][kk] from lane 4b+i and B[kk][j]
// from lane 4b+j, so a lane supplies four consecutive nodes of its own line
// as B and the operator row chunk as A; n nodes take ceil(n/4) instructions
// per row group.  The contraction inputs (flux, or q for elasticity) are
// rounded to bfloat16 as in the BF16 VALU sweeps; the operator is split into
// a bfloat16 high part and a bfloat16 remainder (two instructions per chunk,
// operator accurate to about 2^-16 instead of 2^-8); FP32 accumulation.  The
// time contraction stays on the FP32 MFMA path.
__device__ __forceinline__ short bf16_bits(float x) { return (short)(__float_as_uint(round_bf16(x)) >> 16); }

// Row groups of four on MFMA, and rows left to VALU, for n nodes.
__host__ __device__ constexpr int mfma_groups(int n) { return (n == 5 || n == 6) ? 1 : (n + 3) / 4; }
__host__ __device__ constexpr int mfma_valu_rows(int n) { return n - 4 * mfma_groups(n) > 0 ? n - 4 * mfma_groups(n) : 0; }

// MFMA operands of a lane, loaded once per element: rows 4c + (lane & 3) of
// the unscaled Dhat (zero past row n-1) and of (-dt/h_0) T (Euler) or dt T
// (elasticity).  The Euler sweeps
// accumulate S = sum_A (h_0/h_A) Dhat_A F_A (Euler; the factor is applied
// to the flux only when h_A != h_0) and the time contraction multiplies by
// -dt/h_0, so one operand set serves every axis.  Elasticity applies -1/h_A
// through the coefficients of B_A.
template <int N>
struct MfmaOps {
  static constexpr int n = N + 1, G = mfma_groups(N + 1), JC = (N + 4) / 4;
  float D[G][n];
  float T[G][n];
  s4v Dh[G][JC], Dl[G][JC];  // BF16 variant: high part and remainder, nodes 4jc .. 4jc+3
};

template <int N, class PDE, bool kBF = false>
__device__ __forceinline__ void load_mfma_ops(PArg &P, float dt, MfmaOps<N> &o) {
  constexpr int n = N + 1, G = mfma_groups(n), JC = MfmaOps<N>::JC;
  const int lane = threadIdx.x & 63;
  const float sT = PDE::kElastic ? dt : -dt * (float)P.g.inv_h[0];
#pragma unroll
  for (int c = 0; c < G; c++) {
    const int k = 4 * c + (lane & 3);
#pragma unroll
    for (int j = 0; j < n; j++) {
      o.D[c][j] = k < n ? P.sw->Dhf[k * kMaxN + j] : 0.f;
      o.T[c][j] = k < n ? sT * P.sw->Tf[k * kMaxN + j] : 0.f;
    }
    if constexpr (kBF)
#pragma unroll
      for (int jc = 0; jc < JC; jc++)
#pragma unroll
        for (int kk = 0; kk < 4; kk++) {
          const int j = 4 * jc + kk;
          const float d = (k < n && j < n) ? P.sw->Dhf[k * kMaxN + j] : 0.f;
          const float hi = round_bf16(d);
          o.Dh[c][jc][kk] = bf16_bits(hi);
          o.Dl[c][jc][kk] = bf16_bits(d - hi);
        }
  }
}

// Right-hand side along axis A for the lines L0 + lane of one wavefront
// (all lanes take part in the MFMAs; lanes past the last line compute on
// the line L0 and store nothing), written to sacc (kAcc: added to it), in
// the scaling of MfmaOps.
template <int D, int N, class PDE, int A, bool kAcc, bool kBF = false>
__device__ __forceinline__ void mfma_lines(PArg &P, const MfmaOps<N> &o, const float *sq, float *sacc, int L0,
                                           float irho, float lam, float mu) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, NST = S::NST;
  constexpr int ST = ipow(n, A);
  constexpr int G = mfma_groups(n), VR = mfma_valu_rows(n);
  const int lane = threadIdx.x & 63;
  const int sb = slot_base<D, N, A>(L0 + lane);
  const bool own = sb != kEmptySlot;
  const int base = own ? sb : 0;  // an empty slot computes on line 0 and stores nothing
  float X[n][M];
  // Euler: flux scale h_0/h_A (1 on cubic elements: no multiply)
  const float fs = (float)(P.g.inv_h[A] / P.g.inv_h[0]);
  const bool scale = !PDE::kElastic && A > 0 && P.g.inv_h[A] != P.g.inv_h[0];
#pragma unroll
  for (int j = 0; j < n; j++) {
    float q[M];
#pragma unroll
    for (int v = 0; v < M; v++) q[v] = sq[v * NST + base + j * ST];
    if constexpr (!PDE::kElastic) {
      euler_flux<D, A, float>(q, (float)(P.g.gamma - 1.0), X[j]);
      if (scale)
#pragma unroll
        for (int v = 0; v < M; v++) X[j][v] *= fs;
    } else {
#pragma unroll
      for (int v = 0; v < M; v++) X[j][v] = q[v];
    }
  }
  f4v acc[G][M];
  float accv[VR > 0 ? VR : 1][M];
#pragma unroll
  for (int v = 0; v < M; v++) {
#pragma unroll
    for (int c = 0; c < G; c++) {
      // Euler: start from the earlier axes' sum (elasticity adds after B_A)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int k = 4 * c + i;
        acc[c][v][i] = (!PDE::kElastic && kAcc && own && k < n) ? sacc[v * NST + base + k * ST] : 0.f;
      }
    }
#pragma unroll
    for (int r = 0; r < VR; r++)
      accv[r][v] = (!PDE::kElastic && kAcc && own) ? sacc[v * NST + base + (4 * G + r) * ST] : 0.f;
  }
  if constexpr (kBF) {
    constexpr int JC = MfmaOps<N>::JC;
#pragma unroll
    for (int j = 0; j < n; j++)
#pragma unroll
      for (int v = 0; v < M; v++) X[j][v] = round_bf16(X[j][v]);
#pragma unroll
    for (int v = 0; v < M; v++)
#pragma unroll
      for (int jc = 0; jc < JC; jc++) {
        s4v xb;
#pragma unroll
        for (int kk = 0; kk < 4; kk++) xb[kk] = 4 * jc + kk < n ? bf16_bits(X[4 * jc + kk < n ? 4 * jc + kk : 0][v]) : 0;
#pragma unroll
        for (int c = 0; c < G; c++) {
          acc[c][v] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(o.Dh[c][jc], xb, acc[c][v], 0, 0, 0);
          acc[c][v] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(o.Dl[c][jc], xb, acc[c][v], 0, 0, 0);
        }
      }
#pragma unroll
    for (int j = 0; j < n; j++)
#pragma unroll
      for (int v = 0; v < M; v++)
#pragma unroll
        for (int r = 0; r < VR; r++) accv[r][v] += cload(&P.sw->Dhf[(4 * G + r) * kMaxN + j]) * X[j][v];
  } else {
#pragma unroll
    for (int j = 0; j < n; j++)
#pragma unroll
      for (int v = 0; v < M; v++) {
#pragma unroll
        for (int c = 0; c < G; c++)
          acc[c][v] = __builtin_amdgcn_mfma_f32_4x4x1f32(o.D[c][j], X[j][v], acc[c][v], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < VR; r++) accv[r][v] += cload(&P.sw->Dhf[(4 * G + r) * kMaxN + j]) * X[j][v];
      }
  }
  if (!own) return;
  // elasticity: B_A with -1/h_A folded into its coefficients
  const float sh = PDE::kElastic ? -(float)P.g.inv_h[A] : 1.f;
  const float irh = irho * sh, lah = lam * sh, muh = mu * sh;
#pragma unroll
  for (int k = 0; k < n; k++) {
    float g[M];
#pragma unroll
    for (int v = 0; v < M; v++) g[v] = k < 4 * G ? acc[k / 4][v][k % 4] : accv[k >= 4 * G ? k - 4 * G : 0][v];
    if constexpr (PDE::kElastic) {
      float bg[M];
      elastic_bg<A, float>(g, irh, lah, muh, bg);
#pragma unroll
      for (int v = 0; v < M; v++) {
        const int idx = v * NST + base + k * ST;
        sacc[idx] = kAcc ? sacc[idx] + bg[v] : bg[v];
      }
    } else {
#pragma unroll
      for (int v = 0; v < M; v++) sacc[v * NST + base + k * ST] = g[v];
    }
  }
}

template <int D, int N, class PDE, int A, bool kAcc, int WAVES, int W0 = 0, bool kBF = false>
__device__ __forceinline__ void mfma_axis(PArg &P, const MfmaOps<N> &o, const float *sq, float *sacc, float irho,
                                          float lam, float mu) {
  constexpr int NS = line_slots_count<D, N>();
  const int wave = (threadIdx.x >> 6) - W0;
  for (int L0 = wave * 64; L0 < NS; L0 += WAVES * 64)
    mfma_lines<D, N, PDE, A, kAcc, kBF>(P, o, sq, sacc, L0, irho, lam, mu);
}

// Time contraction on MFMA: the lane owns the time line (v, k), thread
// i = threadIdx.x + r BS as in time_phase; q(l) = u + sum_j (c T)[l][j] S(j)
// with S the sum of the accumulators (two with kTwo) and c = -dt/h_0 for
// Euler (the accumulators hold the unscaled sum) or dt for elasticity.
template <int D, int N, class PDE, int BS, bool kTwo>
__device__ __forceinline__ void mfma_time(PArg &P, const MfmaOps<N> &o, const float *sacc, const float *sacc2,
                                          float *sq, const double *ureg, float dt) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST;
  constexpr int NTL = M * ND;
  constexpr int G = mfma_groups(n), VR = mfma_valu_rows(n);
  constexpr int NU = TimeItems<D, N, M, BS>::value;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float cT = PDE::kElastic ? dt : -dt * (float)P.g.inv_h[0];
#pragma unroll
  for (int r = 0; r < NU; r++) {
    const int T0 = wave * 64 + r * BS;
    if (T0 >= NTL) break;  // uniform over the wavefront
    const bool own = T0 + lane < NTL;
    const int Lt = own ? T0 + lane : T0;
    const int v = Lt / ND, k = Lt - v * ND;
    float b[n];
#pragma unroll
    for (int j = 0; j < n; j++) {
      b[j] = sacc[v * NST + j * ND + k];
      if constexpr (kTwo) b[j] += sacc2[v * NST + j * ND + k];
    }
    const float u0 = (float)ureg[r];
    f4v acc[G];
    float accv[VR > 0 ? VR : 1];
#pragma unroll
    for (int c = 0; c < G; c++) acc[c] = f4v{u0, u0, u0, u0};
#pragma unroll
    for (int q = 0; q < VR; q++) accv[q] = u0;
#pragma unroll
    for (int j = 0; j < n; j++) {
#pragma unroll
      for (int c = 0; c < G; c++) acc[c] = __builtin_amdgcn_mfma_f32_4x4x1f32(o.T[c][j], b[j], acc[c], 0, 0, 0);
#pragma unroll
      for (int q = 0; q < VR; q++) accv[q] += (cT * opT<float>(P, (4 * G + q) * kMaxN + j)) * b[j];
    }
    if (own)
#pragma unroll
      for (int l = 0; l < n; l++) sq[v * NST + l * ND + k] = l < 4 * G ? acc[l / 4][l % 4] : accv[l >= 4 * G ? l - 4 * G : 0];
  }
}

// One FP32 Picard sweep with MFMA contractions.  With pair_axes the lines
// of axes pair_a and pair_b run at the same time on the two halves of the
// block into two accumulators (as rhs_pair); third_axis then accumulates
// onto the first.
template <int D, int N, class PDE, int BS, bool kBF = false>
__device__ __forceinline__ void picard_sweep_mfma(PArg &P, const MfmaOps<N> &o, float *sq, float *sacc, float *sacc2,
                                                  const double *ureg, float dt, float irho, float lam, float mu) {
  constexpr int NW = BS / 64;
  constexpr bool kPair = pair_axes<D, N, BS>();
  if constexpr (kPair) {
    constexpr int HW = round64(ipow(N + 1, D)) / 64;  // wavefronts per half
    if ((int)(threadIdx.x >> 6) < HW)
      mfma_axis<D, N, PDE, pair_a<D, N>(), false, HW, 0, kBF>(P, o, sq, sacc, irho, lam, mu);
    else if ((int)(threadIdx.x >> 6) < 2 * HW)
      mfma_axis<D, N, PDE, pair_b<D, N>(), false, HW, HW, kBF>(P, o, sq, sacc2, irho, lam, mu);
    __syncthreads();
    if constexpr (D > 2) {
      mfma_axis<D, N, PDE, third_axis(D, N), true, NW, 0, kBF>(P, o, sq, sacc, irho, lam, mu);
      __syncthreads();
    }
  } else {
    mfma_axis<D, N, PDE, 0, false, NW, 0, kBF>(P, o, sq, sacc, irho, lam, mu);
    __syncthreads();
    if constexpr (D > 1) {
      mfma_axis<D, N, PDE, 1, true, NW, 0, kBF>(P, o, sq, sacc, irho, lam, mu);
      __syncthreads();
    }
    if constexpr (D > 2) {
      mfma_axis<D, N, PDE, 2, true, NW, 0, kBF>(P, o, sq, sacc, irho, lam, mu);
      __syncthreads();
    }
  }
  mfma_time<D, N, PDE, BS, kPair>(P, o, sacc, sacc2, sq, ureg, dt);
  __syncthreads();
}

// Euler volume term, step 1: time-integrated flux of every axis at every
// spatial node, FB[A][v][k] = sum_l0 w_l0 F_A(q(l0,k)) (one thread per node).
template <int D, int N, class PDE, int BS>
__device__ __forceinline__ void euler_time_flux(PArg &P, const double *qf, double *FB) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST;
  const double gm1 = P.g.gamma - 1.0;
  for (int k = threadIdx.x; k < ND; k += BS) {
    double fb[D][M];
#pragma unroll
    for (int a = 0; a < D; a++)
#pragma unroll
      for (int v = 0; v < M; v++) fb[a][v] = 0.0;
    for (int l0 = 0; l0 < n; l0++) {
      double q[M], F[M];
#pragma unroll
      for (int v = 0; v < M; v++) q[v] = qf[v * NST + l0 * ND + k];
      const double wl = cload(&P.ops->w[l0]);
      euler_flux<D, 0, double>(q, gm1, F);
#pragma unroll
      for (int v = 0; v < M; v++) fb[0][v] += wl * F[v];
      if constexpr (D > 1) {
        euler_flux<D, 1, double>(q, gm1, F);
#pragma unroll
        for (int v = 0; v < M; v++) fb[1][v] += wl * F[v];
      }
      if constexpr (D > 2) {
        euler_flux<D, 2, double>(q, gm1, F);
#pragma unroll
        for (int v = 0; v < M; v++) fb[2][v] += wl * F[v];
      }
    }
#pragma unroll
    for (int a = 0; a < D; a++)
#pragma unroll
      for (int v = 0; v < M; v++) FB[(a * M + v) * ND + k] = fb[a][v];
  }
}

// Work split of an output phase over ITEMS independent items (lines or
// nodes) and the M variables: VG groups of VPG variables, so that up to
// ITEMS*VG threads of the block have work and the index arithmetic of an
// item is done once for all its variables.
template <int ITEMS, int M, int BS>
struct Split {
  static constexpr int VG = BS / ITEMS < 1 ? 1 : (BS / ITEMS > M ? M : BS / ITEMS);
  static constexpr int VPG = (M + VG - 1) / VG;
};

// Euler volume term, step 2, all axes at once (the axes read and write
// disjoint parts of FB): whole wavefronts per axis, one thread per line of
// the axis and variable group,
//   V_A(v,k) = (1/h_A) sum_j Vop[k_A][j] FB[A][v](k_A = j), written over FB[A].
template <int D, int N, class PDE, int BS>
__device__ __forceinline__ void euler_volume_axes(PArg &P, double *FB) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NF = S::NF;
  constexpr int TPA = round64(NF);  // threads per axis
  using SP = Split<NF, M, TPA>;
  for (int it = threadIdx.x; it < D * TPA; it += BS) {
    const int A = __builtin_amdgcn_readfirstlane(it / TPA);  // uniform over a wavefront
    const int r = it - A * TPA;
    if (r < NF * SP::VG) {
      const int g = r / NF, t = r - g * NF;
      const int ST = A == 0 ? 1 : (A == 1 ? n : n * n);
      const int base = t % ST + (t / ST) * ST * n;
#pragma unroll
      for (int vv = 0; vv < SP::VPG; vv++) {
        const int v = g * SP::VPG + vv;
        if (v < M) {
          double *line = FB + (A * M + v) * ND + base;
          double f[n];
#pragma unroll
          for (int j = 0; j < n; j++) f[j] = line[j * ST];
#pragma unroll
          for (int k = 0; k < n; k++) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < n; j++) acc += cload(&P.sw->VA[A][k * kMaxN + j]) * f[j];
            line[k * ST] = acc;
          }
        }
      }
    }
  }
}

// u* = u + dt (V_0 + ... + V_{D-1}) from the per-axis volume terms V_A[v][k]
// at A*M*ND of V (one thread per DOF; DOF threadIdx.x + r*BS is the one
// whose u the thread holds in ureg[r]).
template <int D, int N, class PDE, int BS>
__device__ __forceinline__ void ustar_update(const double *V, const double *ureg, double *us, double dt) {
  constexpr int M = PDE::M, ND = Shape<D, N>::ND;
  constexpr int NU = TimeItems<D, N, M, BS>::value;
#pragma unroll
  for (int r = 0; r < NU; r++) {
    const int i = threadIdx.x + r * BS;
    if (i < M * ND) {
      double vs = V[i];
#pragma unroll
      for (int A = 1; A < D; A++) vs += V[A * M * ND + i];
      // dt = 0 (flagged state or t already at t_end) leaves the state untouched
      us[i] = dt == 0.0 ? ureg[r] : ureg[r] + dt * vs;
    }
  }
}

// Elastic volume term (one thread per node), fused with u* = u + dt V:
//   V = -sum_A (1/h_A) B_A Dhat_A qbar,  qbar = sum_l0 w_l0 q(l0)  (B constant in the element)
// Rows of row group kPart (part_writes) from the gradients they need
// (part_reads).
template <int D, int N, int kPart>
__device__ __forceinline__ void elastic_volume_node(PArg &P, const double *QB, const double *ue, double *us,
                                                    int k, double dt, double irho, double lam, double mu) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = 9, ND = S::ND;
  double V[M];
#pragma unroll
  for (int v = 0; v < M; v++) V[v] = 0.0;
  auto axis = [&](auto Ac) {
    constexpr int A = decltype(Ac)::value;
    constexpr int st = ipow(n, A);
    const int ka = (k / st) % n;
    const double *base = QB + (k - ka * st);
    double g[M], bg[M];
#pragma unroll
    for (int v = 0; v < M; v++) {
      double s = 0.0;
      if (part_reads<Elastic, A, kPart>(v))
#pragma unroll
        for (int j = 0; j < n; j++) s += cload(&P.ops->D[ka * kMaxN + j]) * base[v * ND + j * st];
      g[v] = s;
    }
    elastic_bg<A, double>(g, irho, lam, mu, bg);
#pragma unroll
    for (int v = 0; v < M; v++) V[v] -= bg[v] * P.g.inv_h[A];
  };
  axis(std::integral_constant<int, 0>{});
  axis(std::integral_constant<int, 1>{});
  axis(std::integral_constant<int, 2>{});
#pragma unroll
  for (int v = 0; v < M; v++) {
    if (!part_writes<kPart>(v)) continue;
    const int i = v * ND + k;
    us[i] = dt == 0.0 ? ue[i] : ue[i] + dt * V[v];
  }
}

// All nodes of the element: one thread per node, or with kSplit (BS = 2 *
// round64(n^D)) the velocity rows on the first half of the block and the
// stress rows on the second.
template <int D, int N, int BS, bool kSplit = false>
__device__ __forceinline__ void elastic_volume_update(PArg &P, const double *QB, const double *ue,
                                                      double *us, double dt, double irho, double lam,
                                                      double mu) {
  constexpr int ND = Shape<D, N>::ND;
  if constexpr (kSplit) {
    constexpr int H = round64(ND);
    static_assert(BS == 2 * H, "two threads per node");
    const int half = threadIdx.x / H, k = threadIdx.x - half * H;
    if (k < ND) {
      if (half == 0)
        elastic_volume_node<D, N, 1>(P, QB, ue, us, k, dt, irho, lam, mu);
      else
        elastic_volume_node<D, N, 2>(P, QB, ue, us, k, dt, irho, lam, mu);
    }
  } else {
    for (int k = threadIdx.x; k < ND; k += BS) elastic_volume_node<D, N, 0>(P, QB, ue, us, k, dt, irho, lam, mu);
  }
}

// Boundary-extrapolated traces on both faces normal to axis A:
// trace_s(v, l0, face node) = sum_j phi_j(s) q(v, l0, node with k_A = j),
// computed in FP64 and stored as TT.  One thread per (l0, face node) pair
// and variable group; consecutive threads store consecutive trace values.
// The BS threads from T0 on take part.
template <int D, int N, class PDE, int A, typename TT, int BS, int T0 = 0>
__device__ __forceinline__ void traces_axis(PArg &P, const double *sq, int64_t e) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST, NF = S::NF;
  constexpr int ST = ipow(n, A);
  using SP = Split<ND, M, BS>;
  TT *t0 = (TT *)P.trace[A][0] + e * (int64_t)(M * ND);
  TT *t1 = (TT *)P.trace[A][1] + e * (int64_t)(M * ND);
  for (int it = (int)threadIdx.x - T0; it < ND * SP::VG; it += BS) {
    const int g = it / ND, t = it - g * ND;  // t = l0 * NF + kf
    const int l0 = t / NF, kf = t - l0 * NF;
    const int base = l0 * ND + kf % ST + (kf / ST) * ST * n;
#pragma unroll
    for (int vv = 0; vv < SP::VPG; vv++) {
      const int v = g * SP::VPG + vv;
      if (v < M) {
        const double *line = sq + v * NST + base;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int j = 0; j < n; j++) {
          const double qj = line[j * ST];
          a0 += cload(&P.ops->F0[j]) * qj;
          a1 += cload(&P.ops->F1[j]) * qj;
        }
        t0[v * ND + t] = (TT)a0;
        t1[v * ND + t] = (TT)a1;
      }
    }
  }
}

// Time-averaged trace of variable v at face node kf of the faces normal to
// axis A, both sides (elasticity: the jump term is linear with
// time-independent coefficients, so qbar is all it needs): qbar =
// sum_j phi_j(side) QB(node j), QB the time average sum_l0 w_l0 q(l0) at the
// volume nodes.  Stored as TT in [avg_comps][NF] per element and side.
template <int D, int N, class PDE, int A, typename TT>
__device__ __forceinline__ void trace_avg_value(PArg &P, const double *QB, int64_t e, int v, int kf) {
  using S = Shape<D, N>;
  constexpr int n = S::n, ND = S::ND, NF = S::NF;
  constexpr int ST = ipow(n, A), NC = avg_comps<PDE>();
  const int base = kf % ST + (kf / ST) * ST * n;
  TT *t0 = (TT *)P.trace[A][0] + e * (int64_t)(NC * NF) + kf;
  TT *t1 = (TT *)P.trace[A][1] + e * (int64_t)(NC * NF) + kf;
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int j = 0; j < n; j++) {
    const double qb = QB[v * ND + base + j * ST];
    a0 += cload(&P.ops->F0[j]) * qb;
    a1 += cload(&P.ops->F1[j]) * qb;
  }
  t0[v * NF] = (TT)a0;
  t1[v * NF] = (TT)a1;
}

// Averaged traces of all 2D faces for elasticity: one thread per (axis,
// variable, face node), both sides.
template <int D, int N, class PDE, typename TT, int BS>
__device__ __forceinline__ void traces_avg(PArg &P, const double *QB, int64_t e) {
  constexpr int M = PDE::M, NF = Shape<D, N>::NF;
  for (int it = threadIdx.x; it < D * M * NF; it += BS) {
    const int A = it / (M * NF), r = it - A * (M * NF);
    const int v = r / NF, kf = r - v * NF;
    if (A == 0) trace_avg_value<D, N, PDE, 0, TT>(P, QB, e, v, kf);
    else if (A == 1) {
      if constexpr (D > 1) trace_avg_value<D, N, PDE, 1, TT>(P, QB, e, v, kf);
    } else {
      if constexpr (D > 2) trace_avg_value<D, N, PDE, 2, TT>(P, QB, e, v, kf);
    }
  }
}

// Time-averaged Euler trace at face node kf of the faces normal to axis A
// on one side (0: the face at xi = 0): at each time node l0 the trace
// t(l0) = sum_j phi_j(side) q(l0, node j) of every variable and its flux
// F_A(t(l0)); stored are qbar = sum_l0 w_l0 t(l0) and Fbar = sum_l0 w_l0
// F_A(t(l0)), so that the averaged central flux equals the time integral of
// the per-time-node one.  Layout as trace_avg_value.
template <int D, int N, class PDE, int A, typename TT>
__device__ __forceinline__ void trace_avg_euler(PArg &P, const double *qf, int64_t e, int side, int kf) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST, NF = S::NF;
  constexpr int ST = ipow(n, A), NC = avg_comps<PDE>();
  const int base = kf % ST + (kf / ST) * ST * n;
  const double *phi = side ? P.ops->F1 : P.ops->F0;
  const double gm1 = P.g.gamma - 1.0;
  double qb[M], fb[M];
#pragma unroll
  for (int v = 0; v < M; v++) qb[v] = fb[v] = 0.0;
  // the time loop kept rolled (one time node's loads in flight at once, but
  // no more: this phase must not raise the kernel's register count)
#pragma unroll 1
  for (int l0 = 0; l0 < n; l0++) {
    double t[M], F[M];
#pragma unroll
    for (int v = 0; v < M; v++) t[v] = 0.0;
#pragma unroll
    for (int j = 0; j < n; j++) {
      const double pj = cload(&phi[j]);
      const double *qj = qf + l0 * ND + base + j * ST;
#pragma unroll
      for (int v = 0; v < M; v++) t[v] += pj * qj[v * NST];
    }
    euler_flux<D, A, double>(t, gm1, F);
    const double wl = cload(&P.ops->w[l0]);
#pragma unroll
    for (int v = 0; v < M; v++) {
      qb[v] += wl * t[v];
      fb[v] += wl * F[v];
    }
  }
  TT *o = (TT *)P.trace[A][side] + e * (int64_t)(NC * NF) + kf;
#pragma unroll
  for (int v = 0; v < M; v++) {
    o[v * NF] = (TT)qb[v];
    o[(M + v) * NF] = (TT)fb[v];
  }
}

// Averaged Euler traces of all 2D faces: one thread per (axis, side, face
// node).
template <int D, int N, class PDE, typename TT, int BS>
__device__ __forceinline__ void traces_avg_euler(PArg &P, const double *qf, int64_t e) {
  constexpr int NF = Shape<D, N>::NF;
  for (int it = threadIdx.x; it < D * 2 * NF; it += BS) {
    const int A = it / (2 * NF), r = it - A * (2 * NF);
    const int side = r / NF, kf = r - side * NF;
    if (A == 0) trace_avg_euler<D, N, PDE, 0, TT>(P, qf, e, side, kf);
    else if (A == 1) {
      if constexpr (D > 1) trace_avg_euler<D, N, PDE, 1, TT>(P, qf, e, side, kf);
    } else {
      if constexpr (D > 2) trace_avg_euler<D, N, PDE, 2, TT>(P, qf, e, side, kf);
    }
  }
}

// Predictor outputs from the final FP64 iterate qf: optional qhat copy, the
// face traces, the volume terms (scratch of D*M*ND doubles) and
// u* = u + dt V.
template <int D, int N, class PDE, typename TT, int BS, bool kSplit = false>
__device__ __forceinline__ void predictor_outputs(PArg &P, const double *qf, double *scratch,
                                                  const double *ue, const double *ureg, double dt, int64_t e,
                                                  double *qo, double irho, double lam, double mu) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NST = S::NST;
  if (qo)
    for (int i = threadIdx.x; i < M * NST; i += BS) qo[i] = qf[i];
  if (P.guess == 3) write_history<D, N, PDE, TT, BS>(P, qf, e);
  double *us = P.ustar + e * (int64_t)(M * ND);
  // Euler with two halves of whole wavefronts: the traces on the second
  // half while the first computes the time-integrated fluxes (both only
  // read qf)
  constexpr int HB = BS / 2;
  constexpr bool kHalves = !PDE::kElastic && N > 0 && HB % 64 == 0 && HB >= ND;
  if (kHalves && !P.face_avg) {
    if ((int)threadIdx.x >= HB) {
      traces_axis<D, N, PDE, 0, TT, HB, HB>(P, qf, e);
      if constexpr (D > 1) traces_axis<D, N, PDE, 1, TT, HB, HB>(P, qf, e);
      if constexpr (D > 2) traces_axis<D, N, PDE, 2, TT, HB, HB>(P, qf, e);
    } else {
      euler_time_flux<D, N, PDE, HB>(P, qf, scratch);
    }
    __syncthreads();
  } else if (!P.face_avg) {
    traces_axis<D, N, PDE, 0, TT, BS>(P, qf, e);
    if constexpr (D > 1) traces_axis<D, N, PDE, 1, TT, BS>(P, qf, e);
    if constexpr (D > 2) traces_axis<D, N, PDE, 2, TT, BS>(P, qf, e);
  }
  if constexpr (!PDE::kElastic) {
    if (P.face_avg) traces_avg_euler<D, N, PDE, TT, BS>(P, qf, e);  // reads qf only
    if (!(kHalves && !P.face_avg) && N > 0) {  // not yet computed by the first half
      euler_time_flux<D, N, PDE, BS>(P, qf, scratch);
      __syncthreads();
    }
    if constexpr (N == 0) {
      for (int i = threadIdx.x; i < M * ND; i += BS) us[i] = ue[i];  // no volume term at N = 0
    } else {
      euler_volume_axes<D, N, PDE, BS>(P, scratch);
      __syncthreads();
      ustar_update<D, N, PDE, BS>(scratch, ureg, us, dt);
    }
  } else {
    for (int i = threadIdx.x; i < M * ND; i += BS) {
      const int v = i / ND, k = i - v * ND;
      double a = 0.0;
#pragma unroll
      for (int l = 0; l < n; l++) a += cload(&P.ops->w[l]) * qf[v * NST + l * ND + k];
      scratch[i] = a;
    }
    __syncthreads();
    if (P.face_avg) traces_avg<D, N, PDE, TT, BS>(P, scratch, e);
    if constexpr (N == 0) {
      for (int i = threadIdx.x; i < M * ND; i += BS) us[i] = ue[i];  // no volume term at N = 0
    } else {
      elastic_volume_update<D, N, BS, kSplit>(P, scratch, ue, us, dt, irho, lam, mu);
    }
  }
}

// q^0 = u (as TQ) in the compact [M][ND] layout of the time-constant first
// sweep, from the u values each thread keeps in registers (ureg[r] holds
// u[i], i = threadIdx.x + r*BS).
template <int D, int N, class PDE, typename TQ, int BS>
__device__ __forceinline__ void stage_slice0(TQ *sq, const double *ureg) {
  constexpr int M = PDE::M, ND = Shape<D, N>::ND;
  constexpr int NU = TimeItems<D, N, M, BS>::value;
#pragma unroll
  for (int r = 0; r < NU; r++) {
    const int i = threadIdx.x + r * BS;
    if (i < M * ND) sq[i] = (TQ)ureg[r];
  }
}

// Space-time predictor (Sec. 2.2) of one element per workgroup.
//  PREC == kFP64: every sweep in FP64; q in LDS region A, the accumulator in
//    region R (or in HBM when kAccLds is false).
//  PREC == kFP32/kBF16: sweeps 1..P-1 in FP32 on an FP32 copy of q (region
//    A), the last sweep in FP64 from that copy; its iterate lands in region
//    R and feeds the FP64 outputs; traces are stored in FP32.
//  kMfma: the FP32 (or BF16-input) sweeps contract on MFMA instead of VALU FMAs.
//  kBFac: block-size factor (threads = pred_block(D, N, kBFac)); kSplitLines
//    splits every line of the Picard sweeps into its two elastic row groups.
template <int D, int N, class PDE, int PREC, bool kAccLds, bool kMfma, int kBFac>
__device__ __forceinline__ void predictor_element(PArg &P, int64_t e, const double *ue, double dt,
                                                  double *qo, unsigned char *smem_raw) {
  constexpr int BS = pred_block(D, N, kBFac);
  constexpr bool kSplit = kBFac == kSplitLines;
  static_assert(!kSplit || (PDE::kElastic && !kMfma), "row-group split: elasticity, VALU sweeps");
  using S = Shape<D, N>;
  using L = PredLds<D, N, PDE::M, PREC>;
  constexpr int M = PDE::M, ND = S::ND;
  double irho = 0.0, lam = 0.0, mu = 0.0;
  if constexpr (PDE::kElastic) {
    irho = 1.0 / P.mat[3 * e + 0];
    lam = P.mat[3 * e + 1];
    mu = P.mat[3 * e + 2];
  }
  constexpr int NU = TimeItems<D, N, M, BS>::value;
  double ureg[NU];  // u of the time lines this thread owns, kept for every sweep
#pragma unroll
  for (int r = 0; r < NU; r++) {
    const int i = threadIdx.x + r * BS;
    ureg[r] = i < M * ND ? ue[i] : 0.0;
  }
  // guess and sweep count of this step; guess 3 without a usable previous
  // interval (the first step, or one after a zero step) is the plain
  // scheme: constant guess, N+1 sweeps
  int sweeps = P.sweeps, gm = P.guess;
  double ratio = 0.0;
  if (gm == 3) {
    const double dp = (N > 0 && cload(P.hist_ok) != 0) ? cload(&P.dtprev[P.pidx]) : 0.0;
    if (dp > 0.0) {
      ratio = dt / dp;
    } else {
      gm = 0;
      sweeps = N + 1;
    }
  }
  const int64_t hoff = e * (int64_t)(M * (N > 0 ? N : 1) * ND);
  if constexpr (PREC == kFP64 && kBFac == kRowGroups) {
    static_assert(PDE::kElastic && kAccLds && !kMfma, "row groups: FP64 elasticity, accumulator in LDS");
    double *sq = (double *)smem_raw;
    double *sS = (double *)(smem_raw + L::A);
    stage_slice0<D, N, PDE, double, BS>(sq, ureg);
    __syncthreads();
    int full = sweeps;
    if (gm == 0) {
      first_sweep<D, N, PDE, double, double, false, BS>(P, sq, sS, sq, ureg, dt, irho, lam, mu);
      full -= 1;
    } else if (gm == 3) {
      extrap_guess<D, N, PDE, double, BS, double>(P, sq, ureg, (const double *)P.hist + hoff, ratio);
      __syncthreads();
    } else {
      initial_guess<D, N, PDE, double, false, BS>(P, sq, sS, ureg, dt, irho, lam, mu);
    }
    for (int s = 0; s < full; s++) elastic_group_sweep<D, N, PDE, BS>(P, sq, sS, ureg, dt, irho, lam, mu);
    predictor_outputs<D, N, PDE, double, BS>(P, sq, sS, ue, ureg, dt, e, qo, irho, lam, mu);
  } else if constexpr (PREC == kFP64) {
    double *sq = (double *)smem_raw;
    double *sacc = kAccLds ? (double *)(smem_raw + L::A) : P.acc_glob + e * (int64_t)(M * S::ACC);
    // q^0 = u_h(t^n), constant in time (K1^{-1} F0 = 1): the first sweep
    // reads only its time slice 0
    stage_slice0<D, N, PDE, double, BS>(sq, ureg);
    __syncthreads();
    int full = sweeps;  // sweeps over all time slices
    if (gm == 0) {
      // the first sweep starts from the time-constant iterate q^0 = u
      first_sweep<D, N, PDE, double, double, false, BS, kSplit>(P, sq, sacc, sq, ureg, dt, irho, lam, mu);
      full -= 1;
    } else if (gm == 3) {
      extrap_guess<D, N, PDE, double, BS, double>(P, sq, ureg, (const double *)P.hist + hoff, ratio);
      __syncthreads();
    } else {
      initial_guess<D, N, PDE, double, false, BS, kSplit>(P, sq, sacc, ureg, dt, irho, lam, mu);
    }
    // no room for a second FP64 accumulator: paired axes hold axis 1 in
    // registers (not in 1024-thread blocks, which have 128 registers)
    constexpr int kPair64 = (!kSplit && kBFac != kWide && pair_axes<D, N, BS>()) ? kPairHeld : 0;
    for (int s = 0; s < full; s++)
      picard_sweep<D, N, PDE, double, double, double, false, BS, kSplit, kPair64>(P, sq, sacc, sq, ureg, dt, irho,
                                                                                 lam, mu);
    predictor_outputs<D, N, PDE, double, BS, kSplit>(P, sq, sacc, ue, ureg, dt, e, qo, irho, lam, mu);
  } else {
    constexpr bool kBF = PREC == kBF16;
    float *sq32 = (float *)smem_raw;
    double *sR = (double *)(smem_raw + L::A);
    float *sacc32 = (float *)sR;
    if (sweeps == 1 && gm == 0) {
      // a single sweep is the FP64 one, from q^0 = u itself: region A holds
      // u (compact), region R the per-axis parts and then the iterate
      static_assert(D * M * ND * 8 <= L::R, "region R holds the per-axis parts");
      double *su = (double *)smem_raw;
      stage_slice0<D, N, PDE, double, BS>(su, ureg);
      __syncthreads();
      first_sweep<D, N, PDE, double, double, false, BS, kSplit>(P, su, sR, sR, ureg, dt, irho, lam, mu);
      predictor_outputs<D, N, PDE, float, BS, kSplit>(P, sR, (double *)smem_raw, ue, ureg, dt, e, qo, irho, lam,
                                                      mu);
      return;
    }
    stage_slice0<D, N, PDE, float, BS>(sq32, ureg);
    __syncthreads();
    const float dtf = (float)dt;
    // FP32 sweeps over all time slices before the FP64 one
    int full32 = sweeps - 1;
    if (gm == 0) {
      // first sweep from the time-constant iterate q^0 = u
      first_sweep<D, N, PDE, float, float, kBF, BS, kSplit>(P, sq32, sacc32, sq32, ureg, dtf, (float)irho, (float)lam,
                                                    (float)mu);
      full32 -= 1;
    } else if (gm == 3) {
      // with one sweep (the default) it is the FP64 one, from this guess
      extrap_guess<D, N, PDE, float, BS, float>(P, sq32, ureg, (const float *)P.hist + hoff, (float)ratio);
      __syncthreads();
    } else {
      initial_guess<D, N, PDE, float, kBF, BS, kSplit>(P, sq32, sacc32, ureg, dtf, (float)irho, (float)lam,
                                                     (float)mu);
    }
    if constexpr (kMfma) {
      float *sacc32b = pair_axes<D, N, BS>() ? sacc32 + M * S::NST : nullptr;
      static_assert(!pair_axes<D, N, BS>() || 2 * M * S::NST * sizeof(float) <= L::R, "two FP32 accumulators");
      MfmaOps<N> mo;
      load_mfma_ops<N, PDE, kBF>(P, dtf, mo);
      for (int s = 0; s < full32; s++)
        picard_sweep_mfma<D, N, PDE, BS, kBF>(P, mo, sq32, sacc32, sacc32b, ureg, dtf, (float)irho, (float)lam,
                                              (float)mu);
    } else if constexpr (!kSplit && pair_axes<D, N, BS>()) {
      // the FP32 accumulator fills half of region R: the second one takes the other half
      static_assert(2 * M * S::NST * sizeof(float) <= L::R, "two FP32 accumulators in region R");
      float *sacc32b = sacc32 + M * S::NST;
      for (int s = 0; s < full32; s++)
        picard_sweep<D, N, PDE, float, float, float, kBF, BS, false, kPairTwo>(P, sq32, sacc32, sq32, ureg, dtf,
                                                                          (float)irho, (float)lam, (float)mu,
                                                                          sacc32b);
    } else {
      for (int s = 0; s < full32; s++)
        picard_sweep<D, N, PDE, float, float, float, kBF, BS, kSplit>(P, sq32, sacc32, sq32, ureg, dtf,
                                                                  (float)irho, (float)lam, (float)mu);
    }
    // FP64 residual sweep from the FP32 iterate, into region R
    if constexpr (kBFac != kWide) {
      // FP64 arithmetic with the partial sums stored in FP32: they enter the
      // iterate multiplied by dt, so their rounding is 2^-24 of the one-step
      // change, not of the state; two FP32 accumulators fill region R (axes
      // paired where an axis phase spans more than one wavefront), and the
      // time phase writes the FP64 iterate over them
      float *ra = (float *)sR, *rb = ra + M * S::NST;
      static_assert(2 * M * S::NST * sizeof(float) <= L::R, "two FP32 accumulators in region R");
      constexpr int kPairR = (!kSplit && pair_axes<D, N, BS>() && ipow(N + 1, D) > 64) ? kPairTwo : 0;
      picard_sweep<D, N, PDE, double, float, double, false, BS, kSplit, kPairR, float>(P, sq32, ra, sR, ureg, dt,
                                                                                       irho, lam, mu, rb);
    } else {
      // FP64 accumulator, unpaired (the 512/1024-thread blocks, whose 128
      // registers hold no more)
      picard_sweep<D, N, PDE, double, float, double, false, BS, kSplit>(P, sq32, sR, sR, ureg, dt, irho, lam, mu);
    }
    predictor_outputs<D, N, PDE, float, BS, kSplit>(P, sR, (double *)smem_raw, ue, ureg, dt, e, qo, irho, lam, mu);
  }
}

// Dynamic LDS bytes of a predictor variant: the slot tables, region A and
// region R (or G for the FP64 row-group sweeps; only A when the FP64
// accumulator lives in HBM).
template <int D, int N, int M, int PREC, bool kAccLds, int kBFac>
__host__ __device__ constexpr size_t pred_lds_bytes() {
  return slot_table_bytes<D, N>() +
         ((PREC == kFP64 && !kAccLds) ? PredLds<D, N, M, PREC>::A
          : (kBFac == kRowGroups ? PredLds<D, N, M, PREC>::A + PredLds<D, N, M, PREC>::G
                                 : PredLds<D, N, M, PREC>::A + PredLds<D, N, M, PREC>::R));
}

// Waves per SIMD the register allocation must allow: as many as the LDS
// footprint lets reside (more registers than that would cost occupancy the
// LDS leaves room for).
template <int D, int N, int M, int PREC, bool kAccLds, int kBFac>
__host__ __device__ constexpr int pred_waves_per_eu() {
  constexpr size_t lds = pred_lds_bytes<D, N, M, PREC, kAccLds, kBFac>();
  constexpr int blocks = (int)((160u * 1024u) / lds);
  constexpr int w = blocks * pred_block(D, N, kBFac) / 64 / 4;
  return w < 1 ? 1 : (w > 4 ? 4 : w);  // at most 4: small elements keep 128 registers
}

// Batched predictor: workgroup b owns tile b, one element of one problem of
// the batch (one launch per kernel class; the grid is the total tile count).
// A grid-stride loop over tiles would let the compiler keep every per-thread
// index of the element phases live across iterations and cost occupancy, so
// each workgroup takes a single element.  u, dt and the optional q-hat output
// are the call's buffers (per-problem offsets in the record).
template <int D, int N, class PDE, int PREC, bool kAccLds, bool kMfma, int kBFac>
__global__ void __launch_bounds__(pred_block(D, N, kBFac))
    __attribute__((amdgpu_waves_per_eu(pred_waves_per_eu<D, N, PDE::M, PREC, kAccLds, kBFac>())))
    k_predictor(const PredArgs *args, const Batch b, const double *u, const double *dt, double *qhat) {
  constexpr int M = PDE::M, ND = Shape<D, N>::ND, NST = Shape<D, N>::NST;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t tile = blockIdx.x;
  const int p = tile_problem(b, tile);
  PArg &P = *(PArg *)&args[p];
  const int64_t e = tile - cload(&b.start[p]);
  const double *ue = u + P.u_off + e * (int64_t)(M * ND);
  double *qo = qhat ? qhat + P.q_off + e * (int64_t)(M * NST) : nullptr;
  // slot tables of the line phases into the head of the LDS (read by
  // slot_base; the element's staging ends with a barrier before any line
  // phase)
  constexpr int NS = line_slots_count<D, N>();
  if constexpr (slot_tables<D, N>())
    for (int i = threadIdx.x; i < 3 * NS; i += pred_block(D, N, kBFac))
      ((uint16_t *)smem_raw)[i] = P.sw->ls[i / NS][i - (i / NS) * NS];
  predictor_element<D, N, PDE, PREC, kAccLds, kMfma, kBFac>(P, e, ue, cload(&dt[P.pidx]), qo,
                                                            smem_raw + slot_table_bytes<D, N>());
}

// ------------------------------------------------------------ faces

struct FaceArgs {
  const Ops *ops;
  Geom g;
  const void *trace0;  // side-0 traces of axis A (the + neighbour reads these)
  const void *trace1;  // side-1 traces of axis A
  const double *mat;
  void *GL;            // [E][M][NF] face integral for the element on the - side (GT)
  void *GR;            // [E][M][NF] for the element on the + side (non-conservative only)
  int cx;              // x-chunks of face_per_block faces per x-row
};

// Faces handled by one workgroup of the face kernel: as many whole faces as
// fit n*NF (time node, face node) pairs into 256 threads, at least one.
__host__ __device__ constexpr int face_per_block(int D, int N) {
  return kBlock / (ipow(N + 1, D)) > 0 ? kBlock / (ipow(N + 1, D)) : 1;
}

// Path-conservative Rusanov jump term (eqs. pc.scheme, rusanov) at every
// face node and time node of the face between element e (side 1) and its +A
// neighbour (side 0), integrated in time with the GL weights, in FP64 from
// traces stored as TT, stored as GT.  One thread per (face, time node, face node), so that
// consecutive threads read consecutive trace values; the time integral is
// summed through LDS in time-node order.  A tile is chunk bx of FPB faces of
// the x-row (iy, iz).
template <int D, int N, class PDE, int A, typename TT, typename GT>
__device__ __forceinline__ void face_tile(const FaceArgs &F, int bx, int iy, int iz, double *sDraw) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NF = S::NF;
  constexpr int FPB = face_per_block(D, N);
  constexpr int NI = FPB * n * NF;            // (face, l0, kf) items of the block
  constexpr int NG = PDE::kConservative ? 1 : 2;
  double(*sD)[FPB][M][n * NF] = (double(*)[FPB][M][n * NF])sDraw;  // w_l0 * D^-(l0, kf) per face
  const int nx = F.g.nel[0], ny = F.g.nel[1], nz = F.g.nel[2];
  for (int it = threadIdx.x; it < NI; it += kBlock) {
    const int f = it / (n * NF), r = it - f * (n * NF);  // r = l0 * NF + kf
    const int l0 = r / NF;
    const int ix = bx * FPB + f;
    if (ix >= nx) continue;
    const int64_t e = ix + (int64_t)nx * (iy + (int64_t)ny * iz);
    const int jx = (A == 0) ? (ix + 1 == nx ? 0 : ix + 1) : ix;
    const int jy = (A == 1) ? (iy + 1 == ny ? 0 : iy + 1) : iy;
    const int jz = (A == 2) ? (iz + 1 == nz ? 0 : iz + 1) : iz;
    const int64_t eR = jx + (int64_t)nx * (jy + (int64_t)ny * jz);
    const auto *tm = as_global((const TT *)F.trace1 + e * (int64_t)(M * ND) + r);
    const auto *tp = as_global((const TT *)F.trace0 + eR * (int64_t)(M * ND) + r);
    double qm[M], qp[M];
#pragma unroll
    for (int v = 0; v < M; v++) {
      qm[v] = (double)tm[v * n * NF];
      qp[v] = (double)tp[v * n * NF];
    }
    const double wl = cload(&F.ops->w[l0]);
    if constexpr (!PDE::kElastic) {
      const double gamma = F.g.gamma;
      double Fm[M], Fp[M];
      euler_flux<D, A, double>(qm, gamma - 1.0, Fm);
      euler_flux<D, A, double>(qp, gamma - 1.0, Fp);
      const double smax = fmax(euler_speed<D, A>(qm, gamma), euler_speed<D, A>(qp, gamma));
#pragma unroll
      for (int v = 0; v < M; v++)
        sD[0][f][v][r] = wl * (0.5 * (Fp[v] + Fm[v]) - 0.5 * smax * (qp[v] - qm[v]));
    } else {
      // material path integral with the 3-point Gauss-Legendre rule on [0,1]
      const auto *mat = as_global(F.mat);
      const double rL = mat[3 * e], lL = mat[3 * e + 1], mL = mat[3 * e + 2];
      const double rR = mat[3 * eR], lR = mat[3 * eR + 1], mR = mat[3 * eR + 2];
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
      double dq[M], bd[M];
#pragma unroll
      for (int v = 0; v < M; v++) dq[v] = qp[v] - qm[v];
      elastic_bg<A, double>(dq, irho, lam, mu, bd);
#pragma unroll
      for (int v = 0; v < M; v++) {
        sD[0][f][v][r] = wl * (0.5 * (bd[v] - smax * dq[v]));
        sD[NG - 1][f][v][r] = wl * (0.5 * (bd[v] + smax * dq[v]));
      }
    }
  }
  __syncthreads();
  // G(v, kf) = sum over time nodes, in time-node order
  for (int it = threadIdx.x; it < FPB * M * NF; it += kBlock) {
    const int f = it / (M * NF), r = it - f * (M * NF);
    const int v = r / NF, kf = r - v * NF;
    const int ix = bx * FPB + f;
    if (ix >= nx) continue;
    const int64_t e = ix + (int64_t)nx * (iy + (int64_t)ny * iz);
#pragma unroll
    for (int g = 0; g < NG; g++) {
      double acc = 0.0;
#pragma unroll
      for (int l0 = 0; l0 < n; l0++) acc += sD[g][f][v][l0 * NF + kf];
      as_global((GT *)(g == 0 ? F.GL : F.GR))[e * (int64_t)(M * NF) + r] = (GT)acc;
    }
  }
}

template <int D, int N, class PDE, int A, typename TT, typename GT>
__global__ void __launch_bounds__(kBlock) k_face(const FaceArgs *args, const RowTile *tiles, int64_t ntiles) {
  using S = Shape<D, N>;
  constexpr int n = S::n, M = PDE::M, NF = S::NF;
  constexpr int FPB = face_per_block(D, N);
  constexpr int NG = PDE::kConservative ? 1 : 2;
  __shared__ double sD[NG * FPB * M * n * NF];
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const RowTile t = cload(&tiles[tile]);
    const FaceArgs F = cload(&args[t.p]);
    face_tile<D, N, PDE, A, TT, GT>(F, t.bx, (int)(t.yz & 0xffffu), (int)(t.yz >> 16), sD);
    __syncthreads();  // the next tile overwrites the LDS
  }
}

// Faces per workgroup of the face kernel on averaged traces (one thread per
// face node).
__host__ __device__ constexpr int face_avg_per_block(int D, int N) {
  return kBlock / ipow(N + 1, D - 1) > 0 ? kBlock / ipow(N + 1, D - 1) : 1;
}

// The jump term of a face node from time-averaged traces (option
// face_avg): G = 1/2 (Fbar+ + Fbar-) - 1/2 s_max (qbar+ - qbar-) for Euler
// with s_max from the averaged states; for elasticity the per-time-node
// term integrated exactly (it is linear in the traces with time-independent
// coefficients).  One thread per (face, face node); a tile is chunk bx of
// face_avg_per_block faces of the x-row (iy, iz).
template <int D, int N, class PDE, int A, typename TT, typename GT>
__device__ __forceinline__ void face_avg_tile(const FaceArgs &F, int bx, int iy, int iz) {
  using S = Shape<D, N>;
  constexpr int M = PDE::M, NF = S::NF, NC = avg_comps<PDE>();
  constexpr int FPB = face_avg_per_block(D, N);
  const int nx = F.g.nel[0], ny = F.g.nel[1], nz = F.g.nel[2];
  for (int it = threadIdx.x; it < FPB * NF; it += kBlock) {
    const int f = it / NF, kf = it - f * NF;
    const int ix = bx * FPB + f;
    if (ix >= nx) continue;
    const int64_t e = ix + (int64_t)nx * (iy + (int64_t)ny * iz);
    const int jx = (A == 0) ? (ix + 1 == nx ? 0 : ix + 1) : ix;
    const int jy = (A == 1) ? (iy + 1 == ny ? 0 : iy + 1) : iy;
    const int jz = (A == 2) ? (iz + 1 == nz ? 0 : iz + 1) : iz;
    const int64_t eR = jx + (int64_t)nx * (jy + (int64_t)ny * jz);
    const auto *tm = as_global((const TT *)F.trace1 + e * (int64_t)(NC * NF) + kf);
    const auto *tp = as_global((const TT *)F.trace0 + eR * (int64_t)(NC * NF) + kf);
    double qm[M], qp[M];
#pragma unroll
    for (int v = 0; v < M; v++) {
      qm[v] = (double)tm[v * NF];
      qp[v] = (double)tp[v * NF];
    }
    auto *gl = as_global((GT *)F.GL + e * (int64_t)(M * NF) + kf);
    if constexpr (!PDE::kElastic) {
      const double gamma = F.g.gamma;
      const double smax = fmax(euler_speed<D, A>(qm, gamma), euler_speed<D, A>(qp, gamma));
#pragma unroll
      for (int v = 0; v < M; v++)
        gl[v * NF] = (GT)(0.5 * ((double)tp[(M + v) * NF] + (double)tm[(M + v) * NF]) - 0.5 * smax * (qp[v] - qm[v]));
    } else {
      const auto *mat = as_global(F.mat);
      const double rL = mat[3 * e], lL = mat[3 * e + 1], mL = mat[3 * e + 2];
      const double rR = mat[3 * eR], lR = mat[3 * eR + 1], mR = mat[3 * eR + 2];
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
      double dq[M], bd[M];
#pragma unroll
      for (int v = 0; v < M; v++) dq[v] = qp[v] - qm[v];
      elastic_bg<A, double>(dq, irho, lam, mu, bd);
      auto *gr = as_global((GT *)F.GR + e * (int64_t)(M * NF) + kf);
#pragma unroll
      for (int v = 0; v < M; v++) {
        gl[v * NF] = (GT)(0.5 * (bd[v] - smax * dq[v]));
        gr[v * NF] = (GT)(0.5 * (bd[v] + smax * dq[v]));
      }
    }
  }
}

template <int D, int N, class PDE, int A, typename TT, typename GT>
__global__ void __launch_bounds__(kBlock) k_face_avg(const FaceArgs *args, const RowTile *tiles, int64_t ntiles) {
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const RowTile t = cload(&tiles[tile]);
    const FaceArgs F = cload(&args[t.p]);
    face_avg_tile<D, N, PDE, A, TT, GT>(F, t.bx, (int)(t.yz & 0xffffu), (int)(t.yz >> 16));
  }
}

// ------------------------------------------------------------ update

// Largest |eigenvalue| of the Euler flux Jacobian along each axis at one
// node, lm[A] = |v_A| + c (Sec. 3, CFL condition), and whether the node is
// unusable (a value not finite, rho <= 0 or p <= 0).  The time-step kernel
// and the update (which takes the maxima of the state it writes) both call
// this function, so that the two give the same bits.
template <int D>
__device__ __forceinline__ bool euler_node_speeds(const double *q, double gamma, double *lm) {
  bool bad = false;
#pragma unroll
  for (int v = 0; v < D + 2; v++)
    if (!isfinite(q[v])) bad = true;
  const double ir = 1.0 / q[0];
  double ke = 0.0;
#pragma unroll
  for (int i = 0; i < D; i++) ke += q[1 + i] * q[1 + i];
  const double p = (gamma - 1.0) * (q[D + 1] - 0.5 * ke * ir);
  if (!(q[0] > 0.0) || !(p > 0.0)) bad = true;
  const double c = sqrt(gamma * p * ir);
#pragma unroll
  for (int A = 0; A < D; A++) {
    const double l = fabs(q[1 + A] * ir) + c;
    if (!(l >= 0.0)) bad = true;
    lm[A] = l;
  }
  return bad;
}

// P-wave speed of an element's material (elasticity: the largest
// |eigenvalue| along every axis).
__device__ __forceinline__ double elastic_cp(const double *mat, int64_t e) {
  return sqrt((mat[3 * e + 1] + 2.0 * mat[3 * e + 2]) / mat[3 * e]);
}

struct UpdArgs {
  const Ops *ops;
  Geom g;
  const double *ustar;
  const double *dt;
  const void *GL[3];   // GT
  const void *GR[3];
  int64_t u_off;       // offset of the problem's u in the state buffer
  int pidx;            // problem index: its time step is dt[pidx]
  int cx;              // tiles of upd_elems(D, N, M) elements per x-row
  double h[3];         // mesh widths (wave-speed maxima of the new state)
  const double *mat;   // elasticity: [E][3] material
};

// The wave-speed maximum of a problem is collected in kSmaxSlots slots, one
// 128-byte line apart: each workgroup of the update or time-step kernel
// takes the slot of its tile or row, so that the atomics of many workgroups
// do not queue on one address (one address per problem serialises them at
// about 13 ns each, which bounded the update at 262144 tiles).  The
// time-step finalisation takes the maximum over the slots and clears them.
constexpr int kSmaxSlots = 32;
constexpr int kSmaxStride = 16;  // unsigned long longs from one slot to the next
constexpr int kSmaxPerProblem = kSmaxSlots * kSmaxStride;
__device__ __forceinline__ unsigned long long *smax_slot(unsigned long long *bits, int pidx, int64_t key) {
  return bits + (int64_t)pidx * kSmaxPerProblem + (key & (kSmaxSlots - 1)) * kSmaxStride;
}

// u^{n+1} = u* - dt sum_A (1/h_A) [ L1_kA G_+face + L0_kA G_-face ]  (FP64
// arithmetic; face integrals stored as GT).  A tile is a chunk of
// upd_elems() whole elements of the x-row (iy, iz).  The workgroup first
// copies the tile's face integrals into LDS with contiguous loads: per axis
// the elements' own (+) faces and the lower neighbours' faces (the x
// neighbours of a conservative system share one chunk, shifted by one
// element), together with the lifting coefficients, and issues the loads of
// u* for its nodes; then one thread per node and round updates all M
// variables, reading the face values from LDS.  The new state is written
// with non-temporal stores (nothing reads it again in the step).  Measured
// at 64^3 elements, N = 4 (FP32 face integrals): 0.95 ms with per-node
// global loads of the face values and 1024-node tiles, 0.65 ms so.
//
// With smax_bits set the tile also takes the wave-speed maxima of the state
// it writes, the reduction the next step's time step needs (the same
// per-element quantity as k_cfl), so a step of ader_step does not read u
// again for it.
//
// Elements per tile: at most 256 nodes for Euler and 512 for elasticity
// (measured: Euler 64^3 N=4 0.79 -> 0.67 ms from 512 to 256 nodes,
// elasticity 48^3 N=5 0.93 -> 1.13 ms, one 216-node element per tile), and
// at most 32 KB of staged FP64 face values (2D faces of M * n^(D-1) values
// per element).
__host__ __device__ constexpr int upd_elems(int D, int N, int M) {
  const int nd = ipow(N + 1, D), nf = ipow(N + 1, D - 1);
  const int by_nodes = (M >= 9 ? 512 : 256) / nd, by_lds = 32768 / (2 * D * M * nf * 8);
  const int e = by_nodes < by_lds ? by_nodes : by_lds;
  return e > 0 ? e : 1;
}

template <int D, int N, class PDE, typename GT>
struct UpdLds {
  static constexpr int NF = Shape<D, N>::NF, EPT = upd_elems(D, N, PDE::M);
  static constexpr int EB = PDE::M * NF;  // face values of one element and axis
  // x faces: conservative systems keep one chunk of EPT + 1 elements (the
  // lower neighbour of the tile's first element, then the tile), others an
  // own chunk and a neighbour chunk; axes 1.. an own and a neighbour chunk
  static constexpr int XS = PDE::kConservative ? (EPT + 1) * EB : 2 * EPT * EB;
  static constexpr int YS = EPT * EB;
  static constexpr int SIZE = XS + 2 * (D - 1) * YS;
  __device__ static constexpr int own(int A, int el) {
    return A == 0 ? (PDE::kConservative ? (el + 1) * EB : el * EB) : XS + 2 * (A - 1) * YS + el * EB;
  }
  __device__ static constexpr int nbr(int A, int el) {
    return A == 0 ? (PDE::kConservative ? el * EB : YS + el * EB) : XS + (2 * (A - 1) + 1) * YS + el * EB;
  }
};

// One step of a maximum over runs of lanes within 16-lane rows: lane i takes
// the value of lane i + OFF (a DPP row shift, no LDS traffic) when that lane
// is in the same row and holds a node of the same element (node index / ND).
// Sources beyond the row or the tile read 0, which leaves speeds >= 0 alone.
template <int ND, int OFF, int D>
__device__ __forceinline__ void row_run_max(double (&x)[D], int loc, int lane) {
  const bool take = (lane & 15) + OFF < 16 && (loc + OFF) / ND == loc / ND;
#pragma unroll
  for (int A = 0; A < D; A++) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x[A]), 0x100 + OFF, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x[A]), 0x100 + OFF, 0xf, 0xf, true);
    if (take) x[A] = fmax(x[A], __hiloint2double(hi, lo));
  }
}

// Copy of `count` face values (whole elements of EB values) from HBM into
// LDS, in 16-byte pieces where an element's values fill whole pieces (then
// every element, and every LDS chunk of whole elements, starts 16-byte
// aligned), else value by value.
typedef double d2v __attribute__((ext_vector_type(2)));
template <typename GT, int EB>
__device__ __forceinline__ void stage_chunk(GT *dst, const __attribute__((address_space(1))) GT *src, int count) {
  if constexpr ((EB * sizeof(GT)) % 16 == 0) {
    using V = typename std::conditional<sizeof(GT) == 4, f4v, d2v>::type;
    constexpr int W = 16 / sizeof(GT);
    const auto *vs = (const __attribute__((address_space(1))) V *)src;
    V *vd = (V *)dst;
    for (int i = threadIdx.x; i < count / W; i += kBlock) vd[i] = vs[i];
  } else {
    for (int i = threadIdx.x; i < count; i += kBlock) dst[i] = src[i];
  }
}

template <int D, int N, class PDE, typename GT>
__global__ void __launch_bounds__(kBlock) k_update(const UpdArgs *args, const RowTile *tiles, int64_t ntiles,
                                                   double *u, const double *dt, unsigned long long *smax_bits,
                                                   int *err) {
  using S = Shape<D, N>;
  using L = UpdLds<D, N, PDE, GT>;
  constexpr int n = S::n, M = PDE::M, ND = S::ND, NF = S::NF;
  constexpr int EPT = L::EPT, EB = L::EB;
  constexpr int ROUNDS = (EPT * ND + kBlock - 1) / kBlock;
  __shared__ __align__(16) GT sg[L::SIZE];
  __shared__ double coef[2][D][n];  // (1/h_A) L1[k], -+(1/h_A) L0[k]
  __shared__ double lam[EPT][D];    // per element of the tile: max over its nodes of lambda_A
  __shared__ int bad_any;
  const bool speeds = smax_bits != nullptr;
  const int lane = threadIdx.x & 63;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const RowTile t = cload(&tiles[tile]);
    const UpdArgs U = cload(&args[t.p]);
    const double d = cload(&dt[t.pidx]);
    const int iy = (int)(t.yz & 0xffffu), iz = (int)(t.yz >> 16);
    const int nx = U.g.nel[0], ny = U.g.nel[1], nz = U.g.nel[2];
    const int e0 = t.bx * EPT;
    const int ne = nx - e0 < EPT ? nx - e0 : EPT;
    const int64_t erow = (int64_t)nx * (iy + (int64_t)ny * iz);
    const auto *ustar = as_global(U.ustar);
    // u* of this thread's nodes, loaded before the face values arrive
    double us[ROUNDS][M];
#pragma unroll
    for (int r = 0; r < ROUNDS; r++) {
      const int loc = r * kBlock + threadIdx.x;
      if (loc < ne * ND) {
        const int el = loc / ND, k = loc - el * ND;
        const int64_t base = (erow + e0 + el) * (M * ND) + k;
#pragma unroll
        for (int v = 0; v < M; v++) us[r][v] = ustar[base + v * ND];
      }
    }
    if (threadIdx.x < 2 * D * n) {
      const int side = threadIdx.x / (D * n), A = (threadIdx.x / n) % D, ka = threadIdx.x % n;
      const double ih = args[t.p].g.inv_h[A];  // through the pointer: A differs between lanes
      (&coef[0][0][0])[threadIdx.x] = side == 0 ? ih * cload(&U.ops->L1[ka])
                                                : (PDE::kConservative ? -ih : ih) * cload(&U.ops->L0[ka]);
    }
    if (speeds) {
      for (int i = threadIdx.x; i < EPT * D; i += kBlock) (&lam[0][0])[i] = 0.0;
      if (threadIdx.x == 0) bad_any = 0;
    }
    {
      const auto *gx = as_global((const GT *)U.GL[0]);
      const int64_t exm = erow + (e0 == 0 ? nx - 1 : e0 - 1);  // lower x neighbour of the first element
      if constexpr (PDE::kConservative) {
        stage_chunk<GT, EB>(sg, gx + exm * EB, EB);
        stage_chunk<GT, EB>(sg + EB, gx + (erow + e0) * EB, ne * EB);
      } else {
        const auto *gxr = as_global((const GT *)U.GR[0]);
        stage_chunk<GT, EB>(sg, gx + (erow + e0) * EB, ne * EB);
        stage_chunk<GT, EB>(sg + EPT * EB, gxr + exm * EB, EB);
        stage_chunk<GT, EB>(sg + EPT * EB + EB, gxr + (erow + e0) * EB, (ne - 1) * EB);
      }
#pragma unroll
      for (int A = 1; A < D; A++) {
        const auto *ga = as_global((const GT *)U.GL[A]);
        const auto *gn = as_global((const GT *)(PDE::kConservative ? U.GL[A] : U.GR[A]));
        const int jy = (A == 1) ? (iy == 0 ? ny - 1 : iy - 1) : iy;
        const int jz = (A == 2) ? (iz == 0 ? nz - 1 : iz - 1) : iz;
        const int64_t enb = (int64_t)nx * (jy + (int64_t)ny * jz) + e0;
        stage_chunk<GT, EB>(sg + L::own(A, 0), ga + (erow + e0) * EB, ne * EB);
        stage_chunk<GT, EB>(sg + L::nbr(A, 0), gn + enb * EB, ne * EB);
      }
    }
    __syncthreads();
    bool bad = false;
#pragma unroll
    for (int r = 0; r < ROUNDS; r++) {
      const int loc = r * kBlock + threadIdx.x;  // node of the tile
      const bool act = loc < ne * ND;
      double qn[M];
      if (act) {
        const int el = loc / ND, k = loc - el * ND;
        int oo[D], on[D];
        double cp[D], cm[D];
#pragma unroll
        for (int A = 0; A < D; A++) {
          const int ST = ipow(n, A);
          const int ka = (k / ST) % n;
          const int kf = (k % ST) + (k / (ST * n)) * ST;
          oo[A] = L::own(A, el) + kf;
          on[A] = L::nbr(A, el) + kf;
          cp[A] = coef[0][A][ka];
          cm[A] = coef[1][A][ka];
        }
        double *ug = u + U.u_off + (erow + e0 + el) * (M * ND) + k;
#pragma unroll
        for (int v = 0; v < M; v++) {
          double acc = 0.0;
#pragma unroll
          for (int A = 0; A < D; A++) acc += cp[A] * (double)sg[oo[A] + v * NF] + cm[A] * (double)sg[on[A] + v * NF];
          qn[v] = d == 0.0 ? us[r][v] : us[r][v] - d * acc;
          __builtin_nontemporal_store(qn[v], ug + v * ND);
        }
      }
      if constexpr (!PDE::kElastic) {
        if (speeds) {
          double lm[D];
#pragma unroll
          for (int A = 0; A < D; A++) lm[A] = 0.0;
          if (act) {
            bad |= euler_node_speeds<D>(qn, U.g.gamma, lm);
#pragma unroll
            for (int A = 0; A < D; A++) lm[A] = fmax(0.0, lm[A]);  // a NaN speed raises the flag instead
          }
          // maximum over the lanes of one element within each 16-lane row
          // (elements are contiguous runs of lanes; the speeds are >= 0),
          // then one LDS atomic per run and row and axis
          const int key = loc / ND;
          row_run_max<ND, 1, D>(lm, loc, lane);
          row_run_max<ND, 2, D>(lm, loc, lane);
          row_run_max<ND, 4, D>(lm, loc, lane);
          row_run_max<ND, 8, D>(lm, loc, lane);
          if (act && ((lane & 15) == 0 || loc % ND == 0))
#pragma unroll
            for (int A = 0; A < D; A++)
              atomicMax((unsigned long long *)&lam[key][A], (unsigned long long)__double_as_longlong(lm[A]));
        }
      } else {
        if (speeds && act)
#pragma unroll
          for (int v = 0; v < M; v++)
            if (!isfinite(qn[v])) bad = true;
      }
    }
    if (speeds) {
      if (bad) atomicOr(&bad_any, 1);
      __syncthreads();
      if (threadIdx.x < 64) {
        // S_e = sum_A lm_A / h_A per element, then the tile maximum
        double smx = 0.0;
        bool badm = false;
        for (int el = lane; el < ne; el += 64) {
          double se = 0.0;
          if constexpr (PDE::kElastic) {
            const double cpe = elastic_cp(U.mat, erow + e0 + el);
            if (!(cpe > 0.0)) badm = true;
#pragma unroll
            for (int A = 0; A < D; A++) se += cpe / U.h[A];
          } else {
#pragma unroll
            for (int A = 0; A < D; A++) se += lam[el][A] / U.h[A];
          }
          smx = fmax(smx, se);
        }
        for (int off = 32; off > 0; off >>= 1) smx = fmax(smx, __shfl_xor(smx, off, 64));
        if (__any(badm)) bad_any = 1;  // wave 0 only; the other waves wrote bad_any before the barrier
        if (threadIdx.x == 0) {
          atomicMax(smax_slot(smax_bits, t.pidx, tile), (unsigned long long)__double_as_longlong(smx));
          if (bad_any) atomicOr(err, 1);
        }
      }
    }
    __syncthreads();  // sg, coef, lam and bad_any are reused by the next tile
  }
}

// ------------------------------------------------------------ time step

struct CflArgs {
  Geom g;
  double h[3];
  int64_t u_off;                  // offset of the problem's u in the state buffer
  const double *mat;
  int pidx;                       // problem index: the slots smax_slot(., pidx, .) collect its maximum
  double *summ;                   // optional [E][M][2]: min and max of every variable per element
};

// Per-element wave speed S_e = sum_A (max_k |lambda_A(u_k)|) / h_A and its
// maximum over the mesh.  A tile is one x-row of elements (tile = iy + ny iz):
// the workgroup walks it one wavefront per element at a time and issues a
// single atomicMax on the bit pattern of the row maximum into the row's slot
// (positive doubles order like their bits, so the result does not depend on
// the order).
template <int D, int N, class PDE>
__device__ __forceinline__ void cfl_row(const CflArgs &C, int64_t row, const double *u,
                                        unsigned long long *smax_bits, int *err, double *red, int *bad_any) {
  using S = Shape<D, N>;
  constexpr int M = PDE::M, ND = S::ND;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int nx = C.g.nel[0];
  double smax = 0.0;
  int bad = 0;
  for (int ix = wave; ix < nx; ix += kBlock / 64) {
    const int64_t e = row * nx + ix;
    double lm[3] = {0.0, 0.0, 0.0};
    double vmin[M], vmax[M];
#pragma unroll
    for (int v = 0; v < M; v++) {
      vmin[v] = INFINITY;
      vmax[v] = -INFINITY;
    }
    const auto *ue = as_global(u + C.u_off + e * (int64_t)(M * ND));
    for (int k = lane; k < ND; k += 64) {
      double q[M];
#pragma unroll
      for (int v = 0; v < M; v++) {
        q[v] = ue[v * ND + k];
        if (!isfinite(q[v])) bad = 1;
        vmin[v] = fmin(vmin[v], q[v]);
        vmax[v] = fmax(vmax[v], q[v]);
      }
      if constexpr (!PDE::kElastic) {
        double ln[D];
        if (euler_node_speeds<D>(q, C.g.gamma, ln)) bad = 1;
#pragma unroll
        for (int A = 0; A < D; A++) lm[A] = fmax(lm[A], ln[A]);
      }
    }
    if constexpr (PDE::kElastic) {
      const double cp = elastic_cp(C.mat, e);
      if (!(cp > 0.0)) bad = 1;
#pragma unroll
      for (int A = 0; A < D; A++) lm[A] = cp;
    }
    double se = 0.0;
#pragma unroll
    for (int A = 0; A < D; A++) {
      for (int off = 32; off > 0; off >>= 1) lm[A] = fmax(lm[A], __shfl_xor(lm[A], off, 64));
      se += lm[A] / C.h[A];
    }
    smax = fmax(smax, se);
    if (C.summ) {  // per-element bounds for the detection after the step
#pragma unroll
      for (int v = 0; v < M; v++) {
        for (int off = 32; off > 0; off >>= 1) {
          vmin[v] = fmin(vmin[v], __shfl_xor(vmin[v], off, 64));
          vmax[v] = fmax(vmax[v], __shfl_xor(vmax[v], off, 64));
        }
        if (lane == 0) {
          as_global(C.summ)[(e * M + v) * 2] = vmin[v];
          as_global(C.summ)[(e * M + v) * 2 + 1] = vmax[v];
        }
      }
    }
  }
  if (bad) atomicOr(bad_any, 1);
  if (lane == 0) red[wave] = smax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int i = 1; i < kBlock / 64; i++) m = fmax(m, red[i]);
    atomicMax(smax_slot(smax_bits, C.pidx, row), (unsigned long long)__double_as_longlong(m));
    if (*bad_any) atomicOr(err, 1);
    *bad_any = 0;
  }
  __syncthreads();  // red and bad_any are reused by the next row
}

template <int D, int N, class PDE>
__global__ void __launch_bounds__(kBlock) k_cfl(const CflArgs *args, const Batch b, const double *u,
                                                unsigned long long *smax_bits, int *err) {
  __shared__ double red[kBlock / 64];
  __shared__ int bad_any;
  if (threadIdx.x == 0) bad_any = 0;
  __syncthreads();
  const int64_t total = cload(&b.start[b.np]);
  for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const int p = tile_problem(b, tile);
    const CflArgs C = cload(&args[p]);
    cfl_row<D, N, PDE>(C, tile - cload(&b.start[p]), u, smax_bits, err, red, &bad_any);
  }
}

// ------------------------------------------------------------ detection

struct DetArgs {
  Geom g;
  int64_t u_off;        // offset of the problem's u in the state buffer
  const double *summ;   // [E][M][2] min/max per element of the state before the step
  int *flags;           // [E] troubled-element bits of the problem
};

// A posteriori detection (Sec. 2.3) on the state u after a step: bit 1 a
// value is NaN or infinite, bit 2 (Euler) rho <= 0 or p <= 0 at a node,
// bit 4 the relaxed discrete maximum principle fails for some variable: a
// nodal value outside [m - delta, M + delta], with m, M the extremes of the
// previous state over the element and the 3^D elements sharing a vertex
// with it (periodic) and delta = max(1e-4, 1e-3 (M - m)).  A tile is one
// x-row (tile = iy + ny iz), one wavefront per element.
template <int D, int N, class PDE>
__device__ __forceinline__ void detect_row(const DetArgs &A, int64_t row, const double *u) {
  using S = Shape<D, N>;
  constexpr int M = PDE::M, ND = S::ND;
  constexpr int NB = ipow(3, D);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int nx = A.g.nel[0], ny = A.g.nel[1], nz = A.g.nel[2];
  const int iy = (int)(row % ny), iz = (int)(row / ny);
  for (int ix = wave; ix < nx; ix += kBlock / 64) {
    const int64_t e = row * nx + ix;
    const auto *ue = as_global(u + A.u_off + e * (int64_t)(M * ND));
    int f = 0;
    for (int k = lane; k < ND; k += 64) {
      double q[M];
#pragma unroll
      for (int v = 0; v < M; v++) {
        q[v] = ue[v * ND + k];
        if (!isfinite(q[v])) f |= 1;
      }
      if constexpr (!PDE::kElastic)
        if (!(q[0] > 0.0) || !(euler_pressure<D>(q, A.g.gamma) > 0.0)) f |= 2;
    }
    // neighbour of lane j: offsets (j % 3 - 1, j / 3 % 3 - 1, j / 9 - 1)
    int64_t en = e;
    if (lane < NB) {
      const int jx = (ix + lane % 3 - 1 + nx) % nx;
      const int jy = D > 1 ? (iy + lane / 3 % 3 - 1 + ny) % ny : iy;
      const int jz = D > 2 ? (iz + lane / 9 - 1 + nz) % nz : iz;
      en = jx + (int64_t)nx * (jy + (int64_t)ny * jz);
    }
#pragma unroll
    for (int v = 0; v < M; v++) {
      double lo = lane < NB ? as_global(A.summ)[(en * M + v) * 2] : INFINITY;
      double hi = lane < NB ? as_global(A.summ)[(en * M + v) * 2 + 1] : -INFINITY;
      for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
      }
      const double delta = fmax(1e-4, 1e-3 * (hi - lo));
      const double lo_r = lo - delta, hi_r = hi + delta;
      for (int k = lane; k < ND; k += 64) {
        const double x = ue[v * ND + k];
        if (x < lo_r || x > hi_r) f |= 4;
      }
    }
    for (int off = 32; off > 0; off >>= 1) f |= __shfl_xor(f, off, 64);
    if (lane == 0) as_global(A.flags)[e] = f;
  }
}

template <int D, int N, class PDE>
__global__ void __launch_bounds__(kBlock) k_detect(const DetArgs *args, const Batch b, const double *u) {
  const int64_t total = cload(&b.start[b.np]);
  for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const int p = tile_problem(b, tile);
    const DetArgs A = cload(&args[p]);
    detect_row<D, N, PDE>(A, tile - cload(&b.start[p]), u);
  }
}

}  // namespace ader
