// Ensemble kernels for schedule variant 1 (radix order 1, tile lines full).
#include "ensemble_kernels.h"

PST_ENS_VARIANT(1)
