// Instantiations of the elastic3 kernels for degrees 0..7.
#include "kernel_set.hpp"

namespace ader {

KernelSet kernels_elastic3(int N) {
  switch (N) {
    case 0: return make_kernel_set<3, 0, Elastic>();
    case 1: return make_kernel_set<3, 1, Elastic>();
    case 2: return make_kernel_set<3, 2, Elastic>();
    case 3: return make_kernel_set<3, 3, Elastic>();
    case 4: return make_kernel_set<3, 4, Elastic>();
    case 5: return make_kernel_set<3, 5, Elastic>();
    case 6: return make_kernel_set<3, 6, Elastic>();
    case 7: return make_kernel_set<3, 7, Elastic>();
    default: return KernelSet{};
  }
}

}  // namespace ader
