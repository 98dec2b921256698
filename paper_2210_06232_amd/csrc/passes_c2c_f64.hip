// FP64 instances of the strided single-component pass (k_c2c), built with the
// memory-clause scheduling strategy (see build.py).
#include "passes_impl.h"

namespace eifp {
EIFP_INSTANTIATE_C2C(double)
}
