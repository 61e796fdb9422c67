// Nonlinearity-dependent kernels, dimension 2, catalogue entries 0, 1, 2, 3 (see fmg_launch.h).
#include "fmg_launch_impl.h"

FMG_INSTANTIATE_KIND(2, 0)
FMG_INSTANTIATE_KIND(2, 1)
FMG_INSTANTIATE_KIND(2, 2)
FMG_INSTANTIATE_KIND(2, 3)
