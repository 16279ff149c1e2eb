// Kernel instantiations for n = 128 (both precisions).
#include "kernels.h"

PST_INSTANTIATE_N(128)
