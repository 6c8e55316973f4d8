// Operator instantiations for degrees 11..15 (one translation unit per range keeps builds parallel).
#include "ax_impl.h"

namespace hb {
hb_status launch_ax_11(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<11>(m, l, x, y, p, st, j, s); }
int ax_grid_11(int64_t E) { return ax_grid<11>(E); }
hb_status launch_ax_12(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<12>(m, l, x, y, p, st, j, s); }
int ax_grid_12(int64_t E) { return ax_grid<12>(E); }
hb_status launch_ax_13(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<13>(m, l, x, y, p, st, j, s); }
int ax_grid_13(int64_t E) { return ax_grid<13>(E); }
hb_status launch_ax_14(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<14>(m, l, x, y, p, st, j, s); }
int ax_grid_14(int64_t E) { return ax_grid<14>(E); }
hb_status launch_ax_15(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st, int j, hipStream_t s) { return launch_ax_n<15>(m, l, x, y, p, st, j, s); }
int ax_grid_15(int64_t E) { return ax_grid<15>(E); }
}  // namespace hb
