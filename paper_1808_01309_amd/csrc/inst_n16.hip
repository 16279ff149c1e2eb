// Kernel instantiations for n = 16 (both precisions).
#include "kernels.h"

PST_INSTANTIATE_N(16)
