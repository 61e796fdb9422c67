// Nonlinearity-dependent kernels, dimension 3, catalogue entries 4, 5, 6 (see fmg_launch.h).
#include "fmg_launch_impl.h"

FMG_INSTANTIATE_KIND(3, 4)
FMG_INSTANTIATE_FINISH(3, 4)
FMG_INSTANTIATE_KIND(3, 5)
FMG_INSTANTIATE_FINISH(3, 5)
FMG_INSTANTIATE_KIND(3, 6)
FMG_INSTANTIATE_FINISH(3, 6)
