// FP32 instances of the pass kernels (twiddles and propagator coefficients are formed
// in FP64 and rounded; invariant partial sums are accumulated in FP64).
#include "passes_impl.h"

namespace eifp {
EIFP_INSTANTIATE(float)
}
