// Variable-coefficient kernels, dimension 3, every catalogue entry (see fmg_launch_impl.h).
#include "fmg_launch_impl.h"

FMG_INSTANTIATE_VAR(3, 0)
FMG_INSTANTIATE_VAR(3, 1)
FMG_INSTANTIATE_VAR(3, 2)
FMG_INSTANTIATE_VAR(3, 3)
FMG_INSTANTIATE_VAR(3, 4)
FMG_INSTANTIATE_VAR(3, 5)
FMG_INSTANTIATE_VAR(3, 6)
