// Kernel instantiations for n = 24 (both precisions).
#include "kernels.h"

PST_INSTANTIATE_N(24)
