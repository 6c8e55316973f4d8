// Operator instantiations for degrees 6..10 (one translation unit per range keeps builds parallel).
#include "ax_impl.h"

namespace hb {
hb_status launch_ax_6(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<6>(m, l, x, y, p, st, j, s); }
int ax_grid_6(int64_t E) { return ax_grid<6>(E); }
hb_status launch_ax_7(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<7>(m, l, x, y, p, st, j, s); }
int ax_grid_7(int64_t E) { return ax_grid<7>(E); }
hb_status launch_ax_8(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<8>(m, l, x, y, p, st, j, s); }
int ax_grid_8(int64_t E) { return ax_grid<8>(E); }
hb_status launch_ax_9(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<9>(m, l, x, y, p, st, j, s); }
int ax_grid_9(int64_t E) { return ax_grid<9>(E); }
hb_status launch_ax_10(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<10>(m, l, x, y, p, st, j, s); }
int ax_grid_10(int64_t E) { return ax_grid<10>(E); }
}  // namespace hb
