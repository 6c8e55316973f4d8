// Operator instantiations for Dirichlet boxes, degrees 11..15 (one translation unit per range keeps builds
// parallel).
#include "ax_impl.h"

HB_AX_INSTANCE_DIRICHLET(11)
HB_AX_INSTANCE_DIRICHLET(12)
HB_AX_INSTANCE_DIRICHLET(13)
HB_AX_INSTANCE_DIRICHLET(14)
HB_AX_INSTANCE_DIRICHLET(15)
