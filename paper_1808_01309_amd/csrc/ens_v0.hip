// Ensemble kernels for schedule variant 0 (radix order 0, tile lines full).
#include "ensemble_kernels.h"

PST_ENS_VARIANT(0)
