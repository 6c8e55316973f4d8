// Dispatch of the fused operator by polynomial degree (compile-time N).
#include "common.h"

namespace hb {

#define HB_DECL_AX(n)                                                                                              \
    hb_status launch_ax_##n(const hb_mesh_s *, double, const double *, double *, double *, CgState *, int, hipStream_t); \
    int ax_grid_##n(int64_t);
HB_DECL_AX(1) HB_DECL_AX(2) HB_DECL_AX(3) HB_DECL_AX(4) HB_DECL_AX(5) HB_DECL_AX(6) HB_DECL_AX(7) HB_DECL_AX(8)
HB_DECL_AX(9) HB_DECL_AX(10) HB_DECL_AX(11) HB_DECL_AX(12) HB_DECL_AX(13) HB_DECL_AX(14) HB_DECL_AX(15)
#undef HB_DECL_AX

hb_status launch_ax(const hb_mesh_s *m, double lambda, const double *x, double *y, double *partial, CgState *st,
                    int j, hipStream_t s)
{
    switch (m->N) {
#define HB_CASE(n) \
    case n: return launch_ax_##n(m, lambda, x, y, partial, st, j, s);
        HB_CASE(1) HB_CASE(2) HB_CASE(3) HB_CASE(4) HB_CASE(5) HB_CASE(6) HB_CASE(7) HB_CASE(8)
        HB_CASE(9) HB_CASE(10) HB_CASE(11) HB_CASE(12) HB_CASE(13) HB_CASE(14) HB_CASE(15)
#undef HB_CASE
    default: return fail(HB_ERR_INVALID_ARG, "unsupported degree N");
    }
}

int ax_blocks(const hb_mesh_s *m)
{
    switch (m->N) {
#define HB_CASE(n) \
    case n: return ax_grid_##n(m->E);
        HB_CASE(1) HB_CASE(2) HB_CASE(3) HB_CASE(4) HB_CASE(5) HB_CASE(6) HB_CASE(7) HB_CASE(8)
        HB_CASE(9) HB_CASE(10) HB_CASE(11) HB_CASE(12) HB_CASE(13) HB_CASE(14) HB_CASE(15)
#undef HB_CASE
    default: return 0;
    }
}

}  // namespace hb
