// First phase of the two-phase operator (local output y_L), degrees 1..8, each
// under its default FP64 tile schedule.
#include "ax_impl.h"

HB_AX_INSTANCE_LOCAL(1, 1)
HB_AX_INSTANCE_LOCAL(2, 3)
HB_AX_INSTANCE_LOCAL(3, 1)
HB_AX_INSTANCE_LOCAL(4, 3)
HB_AX_INSTANCE_LOCAL(5, 0)
HB_AX_INSTANCE_LOCAL(6, 0)
HB_AX_INSTANCE_LOCAL(7, 3)
HB_AX_INSTANCE_LOCAL(8, 0)
