// Ensemble kernels for schedule variant 2 (radix order 0, tile lines halved).
#include "ensemble_kernels.h"

PST_ENS_VARIANT(2)
