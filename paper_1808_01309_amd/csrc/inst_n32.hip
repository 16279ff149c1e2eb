// Kernel instantiations for n = 32 (both precisions).
#include "kernels.h"

PST_INSTANTIATE_N(32)
