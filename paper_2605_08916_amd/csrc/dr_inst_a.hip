// Launchers of the L-templated kernels for L = 2..8 (see dr_kernels.h).
#include "dr_kernels.h"

DR_LAUNCHERS(, 2)
DR_LAUNCHERS(, 3)
DR_LAUNCHERS(, 4)
DR_LAUNCHERS(, 5)
DR_LAUNCHERS(, 6)
DR_LAUNCHERS(, 7)
DR_LAUNCHERS(, 8)
