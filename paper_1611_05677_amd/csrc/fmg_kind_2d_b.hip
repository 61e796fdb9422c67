// Nonlinearity-dependent kernels, dimension 2, catalogue entries 4, 5, 6 (see fmg_launch.h).
#include "fmg_launch_impl.h"

FMG_INSTANTIATE_KIND(2, 4)
FMG_INSTANTIATE_KIND(2, 5)
FMG_INSTANTIATE_KIND(2, 6)
