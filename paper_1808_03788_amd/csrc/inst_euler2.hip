// Instantiations of the euler2 kernels for degrees 0..7.
#include "kernel_set.hpp"

namespace ader {

KernelSet kernels_euler2(int N) {
  switch (N) {
    case 0: return make_kernel_set<2, 0, Euler<2>>();
    case 1: return make_kernel_set<2, 1, Euler<2>>();
    case 2: return make_kernel_set<2, 2, Euler<2>>();
    case 3: return make_kernel_set<2, 3, Euler<2>>();
    case 4: return make_kernel_set<2, 4, Euler<2>>();
    case 5: return make_kernel_set<2, 5, Euler<2>>();
    case 6: return make_kernel_set<2, 6, Euler<2>>();
    case 7: return make_kernel_set<2, 7, Euler<2>>();
    default: return KernelSet{};
  }
}

}  // namespace ader
