// Launchers of the L-templated kernels for L = 16..16 (see dr_kernels.h).
#include "dr_kernels.h"

DR_LAUNCHERS(, 16)
