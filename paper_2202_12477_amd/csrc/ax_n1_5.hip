// Operator instantiations for degrees 1..5 (one translation unit per range keeps builds parallel).
#include "ax_impl.h"

HB_AX_INSTANCE(1)
HB_AX_INSTANCE(2)
HB_AX_INSTANCE(3)
HB_AX_INSTANCE(4)
HB_AX_INSTANCE(5)
