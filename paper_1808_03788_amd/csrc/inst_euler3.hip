// Instantiations of the euler3 kernels for degrees 0..7.
#include "kernel_set.hpp"

namespace ader {

KernelSet kernels_euler3(int N) {
  switch (N) {
    case 0: return make_kernel_set<3, 0, Euler<3>>();
    case 1: return make_kernel_set<3, 1, Euler<3>>();
    case 2: return make_kernel_set<3, 2, Euler<3>>();
    case 3: return make_kernel_set<3, 3, Euler<3>>();
    case 4: return make_kernel_set<3, 4, Euler<3>>();
    case 5: return make_kernel_set<3, 5, Euler<3>>();
    case 6: return make_kernel_set<3, 6, Euler<3>>();
    case 7: return make_kernel_set<3, 7, Euler<3>>();
    default: return KernelSet{};
  }
}

}  // namespace ader
