// First phase of the two-phase operator (local output y_L), degrees 9..15, each
// under its default FP64 tile schedule.
#include "ax_impl.h"

HB_AX_INSTANCE_LOCAL(9, 0)
HB_AX_INSTANCE_LOCAL(10, 0)
HB_AX_INSTANCE_LOCAL(11, 1)
HB_AX_INSTANCE_LOCAL(12, 4)
HB_AX_INSTANCE_LOCAL(13, 5)
HB_AX_INSTANCE_LOCAL(14, 5)
HB_AX_INSTANCE_LOCAL(15, 5)
