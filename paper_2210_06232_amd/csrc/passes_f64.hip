// FP64 instances of the pass kernels.
#include "passes_impl.h"

namespace eifp {
EIFP_INSTANTIATE(double)
}
