// Kernel instantiations for n = 96 (both precisions).
#include "kernels.h"

PST_INSTANTIATE_N(96)
