// Operator instantiations for degrees 6..10 (one translation unit per range keeps builds parallel).
#include "ax_impl.h"

HB_AX_INSTANCE(6)
HB_AX_INSTANCE(7)
HB_AX_INSTANCE(8)
HB_AX_INSTANCE(9)
HB_AX_INSTANCE(10)
