// Operator instantiations for Dirichlet boxes, degrees 6..10 (one translation unit per range keeps builds
// parallel).
#include "ax_impl.h"

HB_AX_INSTANCE_DIRICHLET(6)
HB_AX_INSTANCE_DIRICHLET(7)
HB_AX_INSTANCE_DIRICHLET(8)
HB_AX_INSTANCE_DIRICHLET(9)
HB_AX_INSTANCE_DIRICHLET(10)
