// Tables of kernel entry points per (dimension, PDE, degree).
#pragma once
#include "ader_kernels.hpp"

namespace ader {

struct KernelSet {
  const void *pred_lds = nullptr;   // predictor, accumulator in LDS
  const void *pred_glob = nullptr;  // predictor, accumulator in HBM
  const void *face[3] = {nullptr, nullptr, nullptr};
  const void *update = nullptr;
  const void *cfl = nullptr;
  int M = 0, n = 0, ND = 0, NST = 0, NF = 0, ACC = 0;
};

template <int D, int N, class PDE>
KernelSet make_kernel_set() {
  using S = Shape<D, N>;
  KernelSet k;
  k.pred_lds = (const void *)&k_predictor<D, N, PDE, true>;
  k.pred_glob = (const void *)&k_predictor<D, N, PDE, false>;
  k.face[0] = (const void *)&k_face<D, N, PDE, 0>;
  if constexpr (D > 1) k.face[1] = (const void *)&k_face<D, N, PDE, 1>;
  if constexpr (D > 2) k.face[2] = (const void *)&k_face<D, N, PDE, 2>;
  k.update = (const void *)&k_update<D, N, PDE>;
  k.cfl = (const void *)&k_cfl<D, N, PDE>;
  k.M = PDE::M;
  k.n = S::n;
  k.ND = S::ND;
  k.NST = S::NST;
  k.NF = S::NF;
  k.ACC = S::ACC;
  return k;
}

// Defined in the per-family instantiation units.
KernelSet kernels_euler2(int N);
KernelSet kernels_euler3(int N);
KernelSet kernels_elastic3(int N);

}  // namespace ader
