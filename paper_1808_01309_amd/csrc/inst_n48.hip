// Kernel instantiations for n = 48 (both precisions).
#include "kernels.h"

PST_INSTANTIATE_N(48)
