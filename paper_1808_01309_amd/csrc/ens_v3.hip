// Ensemble kernels for schedule variant 3 (radix order 1, tile lines halved).
#include "ensemble_kernels.h"

PST_ENS_VARIANT(3)
