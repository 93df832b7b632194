// Launchers of the L-templated kernels for L = 14..15 (see dr_kernels.h).
#include "dr_kernels.h"

DR_LAUNCHERS(, 14)
DR_LAUNCHERS(, 15)
