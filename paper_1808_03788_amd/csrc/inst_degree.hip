// Kernel instantiations of one family and one degree.  The build compiles
// this unit once per (family, degree) with
//   -DADER_DIM=<2|3> -DADER_ELASTIC=<0|1> -DADER_DEGREE=<0..7>
// so that the heavy template instantiations compile in parallel.
#include "kernel_set.hpp"

#if !defined(ADER_DIM) || !defined(ADER_ELASTIC) || !defined(ADER_DEGREE)
#error "compile with -DADER_DIM, -DADER_ELASTIC and -DADER_DEGREE"
#endif

#define ADER_CAT3_(a, b, c) a##b##c
#define ADER_CAT3(a, b, c) ADER_CAT3_(a, b, c)

namespace ader {

#if ADER_ELASTIC
KernelSet ADER_CAT3(kernels_elastic3_, N, ADER_DEGREE)() { return make_kernel_set<3, ADER_DEGREE, Elastic>(); }
#elif ADER_DIM == 2
KernelSet ADER_CAT3(kernels_euler2_, N, ADER_DEGREE)() { return make_kernel_set<2, ADER_DEGREE, Euler<2>>(); }
#else
KernelSet ADER_CAT3(kernels_euler3_, N, ADER_DEGREE)() { return make_kernel_set<3, ADER_DEGREE, Euler<3>>(); }
#endif

}  // namespace ader
