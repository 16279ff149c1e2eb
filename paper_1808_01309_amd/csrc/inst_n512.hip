// Kernel instantiations for n = 512 (both precisions).
#include "kernels.h"

PST_INSTANTIATE_N(512)
