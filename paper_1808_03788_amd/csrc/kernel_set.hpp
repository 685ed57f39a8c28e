// Tables of kernel entry points per (dimension, PDE, degree).
#pragma once
#include "ader_kernels.hpp"

namespace ader {

// One predictor entry point and its launch shape.
struct PredVariant {
  const void *fn = nullptr;
  int threads = 0;
  size_t lds = 0;
  int prec = 0;       // Prec
  bool acc_lds = true;
  bool mfma = false;
  const char *name = "";
};

constexpr int kMaxVariants = 24;

struct KernelSet {
  PredVariant pred[kMaxVariants];
  int npred = 0;
  const void *face64[3] = {nullptr, nullptr, nullptr};  // FP64 traces and face integrals
  const void *face32[3] = {nullptr, nullptr, nullptr};  // FP32 traces and face integrals
  const void *faceavg64[3] = {nullptr, nullptr, nullptr};  // from time-averaged traces
  const void *faceavg32[3] = {nullptr, nullptr, nullptr};
  const void *update64 = nullptr;                       // FP64 face integrals
  const void *update32 = nullptr;                       // FP32 face integrals
  const void *cfl = nullptr;
  const void *detect = nullptr;
  int M = 0, n = 0, ND = 0, NST = 0, NF = 0, ACC = 0;
};

template <int D, int N, class PDE, int PREC, bool kAccLds, bool kMfma, int kBFac>
void add_variant(KernelSet &k, const char *name) {
  PredVariant v;
  v.fn = (const void *)&k_predictor<D, N, PDE, PREC, kAccLds, kMfma, kBFac>;
  v.threads = pred_block(D, N, kBFac);
  v.lds = pred_lds_bytes<D, N, PDE::M, PREC, kAccLds, kBFac>();
  v.prec = PREC;
  v.acc_lds = kAccLds;
  v.mfma = kMfma;
  v.name = name;
  k.pred[k.npred++] = v;
}

template <int D, int N, class PDE>
KernelSet make_kernel_set() {
  using S = Shape<D, N>;
  KernelSet k;
  add_variant<D, N, PDE, kFP64, true, false, 1>(k, "fp64-valu-b1");
  add_variant<D, N, PDE, kFP64, true, false, 2>(k, "fp64-valu-b2");
  add_variant<D, N, PDE, kFP64, false, false, 1>(k, "fp64-valu-hbmacc-b1");
  add_variant<D, N, PDE, kFP32, true, false, 1>(k, "fp32-valu-b1");
  add_variant<D, N, PDE, kFP32, true, false, 2>(k, "fp32-valu-b2");
  add_variant<D, N, PDE, kFP32, true, true, 1>(k, "fp32-mfma-b1");
  add_variant<D, N, PDE, kFP32, true, true, 2>(k, "fp32-mfma-b2");
  add_variant<D, N, PDE, kBF16, true, false, 1>(k, "bf16-valu-b1");
  add_variant<D, N, PDE, kBF16, true, false, 2>(k, "bf16-valu-b2");
  add_variant<D, N, PDE, kBF16, true, true, 1>(k, "bf16-mfma-b1");
  add_variant<D, N, PDE, kBF16, true, true, 2>(k, "bf16-mfma-b2");
  if constexpr (ipow(N + 1, D) > 128) {
    // one or two workgroups per CU: also 512- or 1024-thread blocks (the
    // FP64 and MFMA line phases of these elements do not fit the 128
    // registers they allow)
    add_variant<D, N, PDE, kFP32, true, false, kWide>(k, "fp32-valu-w4");
    add_variant<D, N, PDE, kBF16, true, false, kWide>(k, "bf16-valu-w4");
  }
  if constexpr (PDE::kElastic && D == 3) {
    add_variant<D, N, PDE, kFP64, true, false, kSplitLines>(k, "fp64-valu-split");
    add_variant<D, N, PDE, kFP64, false, false, kSplitLines>(k, "fp64-valu-hbmacc-split");
    add_variant<D, N, PDE, kFP32, true, false, kSplitLines>(k, "fp32-valu-split");
    add_variant<D, N, PDE, kBF16, true, false, kSplitLines>(k, "bf16-valu-split");
    add_variant<D, N, PDE, kFP64, true, false, kRowGroups>(k, "fp64-valu-groups");
  }
  k.face64[0] = (const void *)&k_face<D, N, PDE, 0, double, double>;
  k.face32[0] = (const void *)&k_face<D, N, PDE, 0, float, float>;
  k.faceavg64[0] = (const void *)&k_face_avg<D, N, PDE, 0, double, double>;
  k.faceavg32[0] = (const void *)&k_face_avg<D, N, PDE, 0, float, float>;
  if constexpr (D > 1) {
    k.face64[1] = (const void *)&k_face<D, N, PDE, 1, double, double>;
    k.face32[1] = (const void *)&k_face<D, N, PDE, 1, float, float>;
    k.faceavg64[1] = (const void *)&k_face_avg<D, N, PDE, 1, double, double>;
    k.faceavg32[1] = (const void *)&k_face_avg<D, N, PDE, 1, float, float>;
  }
  if constexpr (D > 2) {
    k.face64[2] = (const void *)&k_face<D, N, PDE, 2, double, double>;
    k.face32[2] = (const void *)&k_face<D, N, PDE, 2, float, float>;
    k.faceavg64[2] = (const void *)&k_face_avg<D, N, PDE, 2, double, double>;
    k.faceavg32[2] = (const void *)&k_face_avg<D, N, PDE, 2, float, float>;
  }
  k.update64 = (const void *)&k_update<D, N, PDE, double>;
  k.update32 = (const void *)&k_update<D, N, PDE, float>;
  k.cfl = (const void *)&k_cfl<D, N, PDE>;
  k.detect = (const void *)&k_detect<D, N, PDE>;
  k.M = PDE::M;
  k.n = S::n;
  k.ND = S::ND;
  k.NST = S::NST;
  k.NF = S::NF;
  k.ACC = S::ACC;
  return k;
}

// Defined in the per-(family, degree) instantiation units (inst_degree.hip).
#define ADER_DECLARE_FAMILY(fam)                                                                      \
  KernelSet fam##_N0();                                                                                 \
  KernelSet fam##_N1();                                                                                 \
  KernelSet fam##_N2();                                                                                 \
  KernelSet fam##_N3();                                                                                 \
  KernelSet fam##_N4();                                                                                 \
  KernelSet fam##_N5();                                                                                 \
  KernelSet fam##_N6();                                                                                 \
  KernelSet fam##_N7();                                                                                 \
  inline KernelSet fam(int N) {                                                                         \
    switch (N) {                                                                                        \
      case 0: return fam##_N0();                                                                        \
      case 1: return fam##_N1();                                                                        \
      case 2: return fam##_N2();                                                                        \
      case 3: return fam##_N3();                                                                        \
      case 4: return fam##_N4();                                                                        \
      case 5: return fam##_N5();                                                                        \
      case 6: return fam##_N6();                                                                        \
      case 7: return fam##_N7();                                                                        \
      default: return KernelSet{};                                                                      \
    }                                                                                                   \
  }
ADER_DECLARE_FAMILY(kernels_euler2)
ADER_DECLARE_FAMILY(kernels_euler3)
ADER_DECLARE_FAMILY(kernels_elastic3)
#undef ADER_DECLARE_FAMILY

}  // namespace ader
