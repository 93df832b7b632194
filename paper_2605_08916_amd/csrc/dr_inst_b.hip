// Launchers of the L-templated kernels for L = 9..11 (see dr_kernels.h).
#include "dr_kernels.h"

DR_LAUNCHERS(, 9)
DR_LAUNCHERS(, 10)
DR_LAUNCHERS(, 11)
