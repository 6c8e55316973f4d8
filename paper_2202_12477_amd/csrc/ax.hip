// Dispatch of the fused operator by polynomial degree (compile-time N).
#include "common.h"

namespace hb {

#define HB_DECL_AX(n)                                                                                           \
    hb_status launch_ax_##n(const hb_mesh_s *, double, const double *, double *, double *, CgState *,           \
                            hipStream_t);                                                                       \
    hb_status launch_ax32_##n(const hb_mesh_s *, double, const double *, float *, double *, CgState *,          \
                              hipStream_t);                                                                     \
    int ax_grid_##n(int64_t);
HB_DECL_AX(1) HB_DECL_AX(2) HB_DECL_AX(3) HB_DECL_AX(4) HB_DECL_AX(5) HB_DECL_AX(6) HB_DECL_AX(7) HB_DECL_AX(8)
HB_DECL_AX(9) HB_DECL_AX(10) HB_DECL_AX(11) HB_DECL_AX(12) HB_DECL_AX(13) HB_DECL_AX(14) HB_DECL_AX(15)
#undef HB_DECL_AX

#define HB_ALL_N(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

hb_status launch_ax(const hb_mesh_s *m, double lambda, const double *x, double *y, double *partial, CgState *st,
                    hipStream_t s)
{
    switch (m->N) {
#define HB_CASE(n) \
    case n: return launch_ax_##n(m, lambda, x, y, partial, st, s);
        HB_ALL_N(HB_CASE)
#undef HB_CASE
    default: return fail(HB_ERR_INVALID_ARG, "unsupported degree N");
    }
}

hb_status launch_ax32(const hb_mesh_s *m, double lambda, const double *x, float *y, double *partial, CgState *st,
                      hipStream_t s)
{
    if (!m->geo32) return fail(HB_ERR_INVALID_ARG, "the FP32 operator needs a mesh built with HB_MESH_FP32");
    switch (m->N) {
#define HB_CASE(n) \
    case n: return launch_ax32_##n(m, lambda, x, y, partial, st, s);
        HB_ALL_N(HB_CASE)
#undef HB_CASE
    default: return fail(HB_ERR_INVALID_ARG, "unsupported degree N");
    }
}

int ax_blocks(const hb_mesh_s *m)
{
    switch (m->N) {
#define HB_CASE(n) \
    case n: return ax_grid_##n(m->E);
        HB_ALL_N(HB_CASE)
#undef HB_CASE
    default: return 0;
    }
}

}  // namespace hb
