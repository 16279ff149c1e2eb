// Kernel instantiations for n = 256 (both precisions).
#include "kernels.h"

PST_INSTANTIATE_N(256)
