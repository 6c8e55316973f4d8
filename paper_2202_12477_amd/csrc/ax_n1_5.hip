// Operator instantiations for degrees 1..5 (one translation unit per range keeps builds parallel).
#include "ax_impl.h"

namespace hb {
hb_status launch_ax_1(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<1>(m, l, x, y, p, st, j, s); }
int ax_grid_1(int64_t E) { return ax_grid<1>(E); }
hb_status launch_ax_2(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<2>(m, l, x, y, p, st, j, s); }
int ax_grid_2(int64_t E) { return ax_grid<2>(E); }
hb_status launch_ax_3(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<3>(m, l, x, y, p, st, j, s); }
int ax_grid_3(int64_t E) { return ax_grid<3>(E); }
hb_status launch_ax_4(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<4>(m, l, x, y, p, st, j, s); }
int ax_grid_4(int64_t E) { return ax_grid<4>(E); }
hb_status launch_ax_5(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<5>(m, l, x, y, p, st, j, s); }
int ax_grid_5(int64_t E) { return ax_grid<5>(E); }
}  // namespace hb
