// Dispatch of the fused operator by polynomial degree (compile-time N) and
// tile schedule (run-time table per degree and precision).
#include <algorithm>
#include <atomic>
#include <mutex>

#include "common.h"

namespace hb {

#define HB_DECL_AX(n)                                                                                           \
    hb_status launch_ax_##n(const hb_mesh_s *, double, const double *, double *, double *, CgState *,           \
                            hipStream_t);                                                                       \
    hb_status launch_ax32_##n(const hb_mesh_s *, double, const double *, float *, double *, CgState *,          \
                              hipStream_t);                                                                     \
    hb_status launch_batch_ax_##n(int, const void *, bool, const WorkItem *, int, const BatchProb *, hipStream_t); \
    hb_status launch_ax_d_##n(const hb_mesh_s *, double, const double *, double *, double *, CgState *,         \
                              hipStream_t);                                                                     \
    hb_status launch_ax32_d_##n(const hb_mesh_s *, double, const double *, float *, double *, CgState *,        \
                                hipStream_t);                                                                   \
    hb_status launch_batch_ax_d_##n(int, const void *, bool, const WorkItem *, int, const BatchProb *,           \
                                    hipStream_t);                                                             \
    int ax_epb_##n(int);                                                                                        \
    TileWalk ax_walk_##n(int64_t, int64_t, int64_t, int);
HB_DECL_AX(1) HB_DECL_AX(2) HB_DECL_AX(3) HB_DECL_AX(4) HB_DECL_AX(5) HB_DECL_AX(6) HB_DECL_AX(7) HB_DECL_AX(8)
HB_DECL_AX(9) HB_DECL_AX(10) HB_DECL_AX(11) HB_DECL_AX(12) HB_DECL_AX(13) HB_DECL_AX(14) HB_DECL_AX(15)
#undef HB_DECL_AX

#define HB_ALL_N(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

namespace {

// Default schedules (bit 0: D^T in LDS; bit 1: one-wave workgroups, N <= 7;
// bit 2: lean registers with two waves per SIMD, N >= 8; bit 3: merged row
// assembly, N <= 10; bit 4: the three-wave form of 5, N >= 8): the autotuner's
// choices on this part at about 2^24 local nodes per degree (the order-sweep
// size), kept where the winner beat the plain schedule by more than ~1.5%.
constexpr int kDefaultSched[2][kMaxN + 1] = {
    // N: 0  1  2  3  4  5  6  7  8  9 10 11 12 13 14 15
    {0, 1, 1, 9, 3, 1, 8, 9, 8, 29, 8, 21, 21, 5, 5, 5},  // FP64
    {0, 8, 1, 8, 1, 9, 9, 8, 9, 9, 9, 21, 0, 21, 5, 4},   // FP32
};

std::atomic<int> g_sched[2][kMaxN + 1] = {};
std::atomic<bool> g_explicit[2][kMaxN + 1] = {};  // set by a caller or the autotuner
std::atomic<int> g_epoch{0};
std::once_flag g_init;

void init_table()
{
    std::call_once(g_init, [] {
        for (int p = 0; p < 2; ++p)
            for (int n = 0; n <= kMaxN; ++n) g_sched[p][n].store(kDefaultSched[p][n]);
    });
}

}  // namespace

int ax_schedule(int N, bool fp32)
{
    init_table();
    if (N < 1 || N > kMaxN) return 0;
    return g_sched[fp32 ? 1 : 0][N].load(std::memory_order_relaxed);
}

bool ax_schedule_legal(int N, int v)
{
    const bool small = (N + 1) * (N + 1) <= 64;   // an element fits in a wave
    const bool merge = (N + 1) * (N + 1) <= 128;  // a 256-thread tile holds two or more elements
    const int lean_cols = kSchedLean | kSchedColsLds;
    // merging goes with the 256-thread schedules and with the full three-wave form (29) only
    const int rest = v & ~kSchedMerge;
    const bool merge_ok = merge && !(v & kSchedWave) &&
                          (!(v & (kSchedLean | kSchedThree)) || rest == (lean_cols | kSchedThree));
    return N >= 1 && N <= kMaxN && v >= 0 && v < kNumSched && (!(v & kSchedWave) || small) &&
           (!(v & kSchedLean) || !small) && (!(v & kSchedMerge) || merge_ok) &&
           (!(v & kSchedThree) || (v & lean_cols) == lean_cols);
}

void set_ax_schedule(int N, bool fp32, int v)
{
    init_table();
    g_sched[fp32 ? 1 : 0][N].store(v, std::memory_order_relaxed);
    g_explicit[fp32 ? 1 : 0][N].store(true, std::memory_order_relaxed);
    g_epoch.fetch_add(1);
}

int ax_schedule_epoch() { return g_epoch.load(); }

hb_status launch_ax(const hb_mesh_s *m, double lambda, const double *x, double *y, double *partial, CgState *st,
                    hipStream_t s)
{
    if (m->desc.flags & HB_MESH_GATHER) return launch_ax_two_phase(m, lambda, x, y, partial, st, false, s);
    const bool d = (m->desc.flags & HB_MESH_DIRICHLET) != 0;
    switch (m->N) {
#define HB_CASE(n) \
    case n: return d ? launch_ax_d_##n(m, lambda, x, y, partial, st, s) : launch_ax_##n(m, lambda, x, y, partial, st, s);
        HB_ALL_N(HB_CASE)
#undef HB_CASE
    default: return fail(HB_ERR_INVALID_ARG, "unsupported degree N");
    }
}

hb_status launch_ax32(const hb_mesh_s *m, double lambda, const double *x, float *y, double *partial, CgState *st,
                      hipStream_t s)
{
    if (!m->geo32) return fail(HB_ERR_INVALID_ARG, "the FP32 operator needs a mesh built with HB_MESH_FP32");
    const bool d = (m->desc.flags & HB_MESH_DIRICHLET) != 0;
    switch (m->N) {
#define HB_CASE(n)                                                                \
    case n:                                                                       \
        return d ? launch_ax32_d_##n(m, lambda, x, y, partial, st, s)             \
                 : launch_ax32_##n(m, lambda, x, y, partial, st, s);
        HB_ALL_N(HB_CASE)
#undef HB_CASE
    default: return fail(HB_ERR_INVALID_ARG, "unsupported degree N");
    }
}

hb_status launch_batch_ax(int N, int sched, const void *D, bool fp32, bool dirichlet, const WorkItem *items,
                          int nitems, const BatchProb *probs, hipStream_t s)
{
    switch (N) {
#define HB_CASE(n)                                                                       \
    case n:                                                                              \
        return dirichlet ? launch_batch_ax_d_##n(sched, D, fp32, items, nitems, probs, s) \
                         : launch_batch_ax_##n(sched, D, fp32, items, nitems, probs, s);
        HB_ALL_N(HB_CASE)
#undef HB_CASE
    default: return fail(HB_ERR_INVALID_ARG, "unsupported degree N");
    }
}

TileWalk ax_walk_for(int N, int64_t nx, int64_t ny, int64_t nz, int sched)
{
    switch (N) {
#define HB_CASE(n) \
    case n: return ax_walk_##n(nx, ny, nz, sched);
        HB_ALL_N(HB_CASE)
#undef HB_CASE
    default: return TileWalk{};
    }
}

int ax_epb_for(int N, int sched)
{
    switch (N) {
#define HB_CASE(n) \
    case n: return ax_epb_##n(sched);
        HB_ALL_N(HB_CASE)
#undef HB_CASE
    default: return 1;
    }
}

int ax_grid_for(int N, int64_t E, int64_t nx, int64_t ny, int64_t nz, int sched)
{
    return static_cast<int>(walk_tiles(ax_walk_for(N, nx, ny, nz, sched), E, ax_epb_for(N, sched)));
}

int unmerged_if_sparse(int N, bool fp32, int v, int64_t elements, int64_t tiles)
{
    if (!(v & kSchedMerge) || g_explicit[fp32 ? 1 : 0][N].load(std::memory_order_relaxed)) return v;
    const double slots = static_cast<double>(tiles) * ax_epb_for(N, v);
    return static_cast<double>(elements) < kMergeFill * slots ? (v & ~kSchedMerge) : v;
}

int mesh_schedule(const hb_mesh_s *m, bool fp32)
{
    int v = ax_schedule(m->N, fp32);
    if (g_explicit[fp32 ? 1 : 0][m->N].load(std::memory_order_relaxed)) return v;  // a chosen schedule, as is
    if (v & kSchedMerge)
        v = unmerged_if_sparse(m->N, fp32, v, m->E, ax_grid_for(m->N, m->E, m->desc.nx, m->desc.ny, m->desc.nz, v));
    const int wave = (v & kSchedColsLds) | kSchedWave;
    // a launch of fewer workgroups than the device has CUs is latency-bound:
    // one-wave workgroups (more of them) where an element fits a wave
    if (!(v & kSchedWave) && ax_schedule_legal(m->N, wave) &&
        ax_grid_for(m->N, m->E, m->desc.nx, m->desc.ny, m->desc.nz, v) < kSmallLaunch)
        return wave;
    return v;
}

int ax_blocks(const hb_mesh_s *m, bool fp32)
{
    if (!fp32 && (m->desc.flags & HB_MESH_GATHER)) return ax_local_blocks(m);
    return ax_grid_for(m->N, m->E, m->desc.nx, m->desc.ny, m->desc.nz, mesh_schedule(m, fp32));
}

int ax_blocks_max(const hb_mesh_s *m)
{
    int g = 0;
    for (int v = 0; v < kNumSched; ++v)
        if (ax_schedule_legal(m->N, v))
            g = std::max(g, ax_grid_for(m->N, m->E, m->desc.nx, m->desc.ny, m->desc.nz, v));
    return g;
}

}  // namespace hb
