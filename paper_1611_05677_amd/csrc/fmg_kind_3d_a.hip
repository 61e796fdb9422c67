// Nonlinearity-dependent kernels, dimension 3, catalogue entries 0, 1, 2, 3 (see fmg_launch.h).
#include "fmg_launch_impl.h"

FMG_INSTANTIATE_KIND(3, 0)
FMG_INSTANTIATE_FINISH(3, 0)
FMG_INSTANTIATE_KIND(3, 1)
FMG_INSTANTIATE_FINISH(3, 1)
FMG_INSTANTIATE_KIND(3, 2)
FMG_INSTANTIATE_FINISH(3, 2)
FMG_INSTANTIATE_KIND(3, 3)
FMG_INSTANTIATE_FINISH(3, 3)
