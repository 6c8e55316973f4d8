// Operator instantiations for Dirichlet boxes, degrees 1..5 (one translation unit per range keeps builds
// parallel).
#include "ax_impl.h"

HB_AX_INSTANCE_DIRICHLET(1)
HB_AX_INSTANCE_DIRICHLET(2)
HB_AX_INSTANCE_DIRICHLET(3)
HB_AX_INSTANCE_DIRICHLET(4)
HB_AX_INSTANCE_DIRICHLET(5)
