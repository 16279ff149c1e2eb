// Kernel instantiations for n = 1024 (both precisions).
#include "kernels.h"

PST_INSTANTIATE_N(1024)
