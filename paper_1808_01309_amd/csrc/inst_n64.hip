// Kernel instantiations for n = 64 (both precisions).
#include "kernels.h"

PST_INSTANTIATE_N(64)
