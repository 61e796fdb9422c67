// Variable-coefficient kernels, dimension 2, every catalogue entry (see fmg_launch_impl.h).
#include "fmg_launch_impl.h"

FMG_INSTANTIATE_VAR(2, 0)
FMG_INSTANTIATE_VAR(2, 1)
FMG_INSTANTIATE_VAR(2, 2)
FMG_INSTANTIATE_VAR(2, 3)
FMG_INSTANTIATE_VAR(2, 4)
FMG_INSTANTIATE_VAR(2, 5)
FMG_INSTANTIATE_VAR(2, 6)
