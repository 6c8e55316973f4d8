// Operator instantiations for degrees 11..15 (one translation unit per range keeps builds parallel).
#include "ax_impl.h"

HB_AX_INSTANCE(11)
HB_AX_INSTANCE(12)
HB_AX_INSTANCE(13)
HB_AX_INSTANCE(14)
HB_AX_INSTANCE(15)
