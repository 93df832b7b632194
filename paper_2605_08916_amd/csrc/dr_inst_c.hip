// Launchers of the L-templated kernels for L = 12..13 (see dr_kernels.h).
#include "dr_kernels.h"

DR_LAUNCHERS(, 12)
DR_LAUNCHERS(, 13)
