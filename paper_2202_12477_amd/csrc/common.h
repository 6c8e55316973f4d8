// Internal declarations shared by the HIP translation units of libhbmi.
// Not installed; the public interface is include/hbmi.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "hbmi.h"
#include "walk.h"

namespace hb {

constexpr int kMaxN = 15;
// Operator tile schedules (bit flags): D^T read from LDS; one-wave workgroups
// (N <= 7); lean registers with two waves per SIMD (N >= 8); assembly of four
// x-consecutive elements merged in LDS (N <= 10; at N = 7 an element is one
// wave); the three-wave form of the lean schedule with D^T in LDS (N >= 8,
// with both; merged too as 29 at N = 8-10).
constexpr int kSchedColsLds = 1, kSchedWave = 2, kSchedLean = 4, kSchedMerge = 8, kSchedThree = 16,
              kNumSched = 32;
constexpr int kGeo = 7;  // G_rr, G_rs, G_rt, G_ss, G_st, G_tt, c

// Thread-local error message behind hb_last_error().
void set_error(const std::string &msg);
hb_status fail(hb_status st, const std::string &msg);
hb_status hip_fail(hipError_t err, const char *what);

// Device allocation that reports HB_ERR_OUT_OF_MEMORY and adds to *tally.
template <typename T>
inline hb_status dev_alloc(T **p, size_t count, size_t *tally)
{
    if (hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * count) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(HB_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(sizeof(T) * count) + " bytes failed");
    }
    *tally += sizeof(T) * count;
    return HB_OK;
}

#define HB_HIP(call)                                      \
    do {                                                  \
        hipError_t err_ = (call);                         \
        if (err_ != hipSuccess) return hb::hip_fail(err_, #call); \
    } while (0)

// Device-resident state of one CG solve (Algorithm 1).  Scalars never leave
// the device and no kernel takes the iteration number as an argument, so one
// captured iteration can be replayed and problems at different iterations can
// share launches.  Fields are written only by single-block kernels and read by
// later kernels:
//   alpha (first single-block kernel of an iteration): turns `pending` into
//     `done`, else advances `it` and computes alpha (or sets `done` on breakdown);
//   beta: records rho_{it+1}, beta, the history and `iters`; a stop decided
//     here only sets `pending`, so this iteration's update still runs.
// Every streaming kernel returns at once when `done` is set (an operator call
// issued after `pending` was set is wasted but harmless: it touches only Ap).
struct CgState {
    double bb;         // b . b
    double alpha;      // alpha of the current iteration
    double beta;       // beta of the current iteration
    double pAp;        // p . A p of the current iteration
    double rtol;       // < 0 in fixed-iteration mode
    double stop_res;   // stop once ||r_j|| <= stop_res (< 0: never; set from rtol ||b|| at the start)
    int32_t max_iter;
    int32_t it;        // index of the current iteration (-1 before the first)
    int32_t iters;     // completed iterations
    int32_t done;      // no further kernel of this solve does anything
    int32_t pending;   // stop after the current iteration's update
    int32_t status;    // hb_status of the solve
};

// One problem of a batched solve, as the batched kernels see it (device copy).
struct BatchProb {
    const int32_t *map;
    const double *geo;
    const float *geo32;
    const double *D;
    const float *D32;
    double lambda;
    double *x, *r, *p, *Ap;
    float *Ap32;
    double *rho, *hist, *part_ax, *part_vec;
    CgState *st;
    int64_t E, NG;
    int32_t N, ax_tiles, vec_chunks, use32;  // use32: the operator of this problem is the FP32 one
    int32_t nx, ny, nz;                      // the box (host side: the order of the operator tiles)
    int32_t dirichlet;                       // a Dirichlet box (host side: its class of operator launches)
    const double *inv;                       // Jacobi: 1 / diag(A) (nullptr: no preconditioner)
};

// A unit of batched work: problem index and tile (operator) or chunk (vectors).
struct WorkItem {
    int32_t prob, idx;
};

// The persistent batched launch (persist.hip): workgroup -> (problem, rank
// among the problem's workgroups), and per problem its workgroup count, its
// iteration budget for the launch, its operator tiles and their order.
struct PersistWg {
    int32_t prob, rank;
};
struct PersistSlot {
    TileWalk walk;
    int32_t tiles, nwg, iters, pad;
};

// Per-mesh CG workspace (device), allocated on first use.
struct CgWork {
    int64_t n = 0;         // N_G it was sized for
    int32_t hist_len = 0;  // entries in hist
    double *r = nullptr, *p = nullptr, *Ap = nullptr;
    double *part_ax = nullptr;  // operator block partials of p.Ap (>= operator grid)
    double *part_vec = nullptr; // vector-kernel block partials (>= 2 * vector grid)
    int32_t part_ax_len = 0, part_vec_len = 0;
    double *rho = nullptr;      // r_j . r_j (r_j . z_j with the Jacobi preconditioner), j = 0..max_iter
    // mixed-precision refinement: outer residual, correction, FP32 operator output
    double *rout = nullptr, *d = nullptr;
    float *Ap32 = nullptr;
    double *hist = nullptr;     // ||r_j||, j = 0..max_iter
    CgState *state = nullptr;
    double *dnorm = nullptr;        // one device scalar (a squared norm)
    CgState *host_state = nullptr;  // pinned mirror for read-back
    double *host_norm = nullptr;    // pinned mirror of dnorm
    size_t bytes = 0;               // device bytes held (counted in the mesh's device_bytes)
    // captured iteration graphs (hb_cg_opts.graph_k), keyed by their arguments
    struct Graph {
        hipGraphExec_t exec = nullptr;
        int elem = 0;   // bytes per operator output entry (8: FP64 operator, 4: FP32)
        int epoch = 0;  // schedule-table version the kernels were captured under
        int k = 0;
        double lambda = 0.0;
        const void *x = nullptr, *Ap = nullptr;
        bool pc = false;  // Jacobi-preconditioned iteration
    };
    Graph graphs[2];
    int graph_next = 0;
    int graph_k = 0;           // the current solve's graph length (0: plain launches)
    hipStream_t cap = nullptr; // private stream the graphs are captured on
    // Jacobi preconditioner: 1 / diag(A) for lambda = jlambda (allocated on first use)
    double *jinv = nullptr;
    double jlambda = 0.0;
    bool jvalid = false;
    bool pc = false;           // the current solve is preconditioned (iterations use jinv)
};

}  // namespace hb

// Global nodes (DOFs) of a box mesh: every GLL node of the box, or only the
// interior ones with HB_MESH_DIRICHLET.
inline int64_t box_global_nodes(const hb_mesh_desc &d)
{
    const int64_t gx = (int64_t)d.nx * d.N + 1, gy = (int64_t)d.ny * d.N + 1, gz = (int64_t)d.nz * d.N + 1;
    return (d.flags & HB_MESH_DIRICHLET) ? (gx - 2) * (gy - 2) * (gz - 2) : gx * gy * gz;
}

struct hb_mesh_s {
    hb_mesh_desc desc;
    int N = 0;
    int64_t E = 0, NL = 0, NG = 0;
    int32_t *map = nullptr;   // [E][(N+1)^3] global index per local node (rows of Z)
    double *geo = nullptr;    // [E][N+1 layers][7 factors][(N+1)^2]: each element layer-major
    double *D = nullptr;      // [(N+1)^2] row-major
    double *xi = nullptr, *w = nullptr;  // device copies of the GLL nodes and weights
    float *geo32 = nullptr;   // FP32 copy of geo (HB_MESH_FP32), rounded once
    float *D32 = nullptr;     // FP32 copy of D
    // two-phase operator (HB_MESH_GATHER): the local output y_L [E][(N+1)^3] and
    // Z^T as CSR rows (row g: the local nodes mapped to g, ascending)
    double *yl = nullptr;
    uint32_t *zt_off = nullptr;  // [N_G + 1]
    uint32_t *zt_idx = nullptr;  // [local nodes that carry a DOF]
    double h_xi[hb::kMaxN + 1], h_w[hb::kMaxN + 1], h_D[(hb::kMaxN + 1) * (hb::kMaxN + 1)];
    hb::CgWork cg;
    size_t device_bytes = 0;
};

namespace hb {

// Host-side 1D basis (basis.cpp): GLL nodes ascending, weights, D[i][j] = l_j'(xi_i).
void gll_basis(int N, double *xi, double *w, double *D);

// Setup kernels (setup.hip).
hb_status build_geometry(hb_mesh_s *m, hipStream_t s);
hb_status launch_rhs(int64_t n, uint64_t seed, double *b, hipStream_t s);

// Operator (ax*.hip).  y += A x (y is assembled by atomic addition, so a
// fresh result needs y = 0 first).  With st != nullptr this is the operator
// step of CG: it returns at once if the solve is done, and each block also
// writes its share of sum_e x_e . y_e (= x . A x) to partial[block].
hb_status launch_ax(const hb_mesh_s *m, double lambda, const double *x, double *y, double *partial, CgState *st,
                    hipStream_t s);
// The two-phase operator of an HB_MESH_GATHER mesh (gather.hip): y_L by the
// element kernel, then y (+)= Z^T y_L by a deterministic gather (overwrite:
// y = Z^T y_L, no zeroing needed).  launch_ax routes such meshes here (adding).
hb_status launch_ax_two_phase(const hb_mesh_s *m, double lambda, const double *x, double *y, double *partial,
                              CgState *st, bool overwrite, hipStream_t s);
int ax_local_blocks(const hb_mesh_s *m);
hb_status build_gather(hb_mesh_s *m, hipStream_t s);
// The FP32 operator (mesh built with HB_MESH_FP32): x FP64, y FP32.
hb_status launch_ax32(const hb_mesh_s *m, double lambda, const double *x, float *y, double *partial, CgState *st,
                      hipStream_t s);
// Operator blocks (tiles) of a mesh under the current schedule of its degree
// and the given precision; the largest over all schedules (sizes partials).
int ax_blocks(const hb_mesh_s *m, bool fp32);
int ax_blocks_max(const hb_mesh_s *m);
// Operator tiles of a box of E = nx*ny*nz elements under a schedule (padded rows included).
int ax_grid_for(int N, int64_t E, int64_t nx, int64_t ny, int64_t nz, int sched);
// The order of the operator's tiles on an nx x ny x nz box under a schedule.
TileWalk ax_walk_for(int N, int64_t nx, int64_t ny, int64_t nz, int sched);
// The autotuner (tune.hip): time every legal schedule of a class on a synthetic
// box of about local_nodes local nodes and install the fastest; the cached
// form tunes each (degree, precision, power-of-two size class) once per
// process and installs its winner on later calls.
hb_status tune_class(int N, bool fp32, int64_t local_nodes, int reps, hb_tune_result *out, hipStream_t s);
int tune_size_class(int64_t local_nodes);
hb_status tune_class_cached(int N, bool fp32, int64_t local_nodes, hipStream_t s, int *schedule);
// The schedule a single-problem launch on this mesh uses: the table's; while
// the class's entry is the built-in default (no hb_set_schedule or autotuning
// for it yet), launches of fewer than kSmallLaunch workgroups where an element
// fits a wave take its one-wave form (the small configuration: 13.4 us per CG
// iteration against 14.5 us).  Likewise a default merged schedule whose padded
// rows would leave more than 15% of the tile slots empty (rows of few elements)
// runs unmerged.  ax_blocks counts the workgroups of the one chosen.
constexpr int kSmallLaunch = 256;
constexpr double kMergeFill = 0.85;
int mesh_schedule(const hb_mesh_s *m, bool fp32);
// v without its merge bit where `elements` fill less than kMergeFill of the
// slots of `tiles` merged tiles and the class's schedule is the built-in default.
int unmerged_if_sparse(int N, bool fp32, int v, int64_t elements, int64_t tiles);
// Schedule table (per degree and precision), shared by every solve path.
int ax_schedule(int N, bool fp32);
bool ax_schedule_legal(int N, int sched);
void set_ax_schedule(int N, bool fp32, int sched);
int ax_schedule_epoch();

// Vector kernels of CG (cg.hip).  TAp is the type of the operator output Ap
// (double for the FP64 operator, float for the FP32 one); every other vector
// and every dot product is FP64.
int vec_blocks(int64_t n);
hb_status launch_zero(double *v, int64_t n, hipStream_t s);
hb_status launch_zero(float *v, int64_t n, hipStream_t s);
hb_status launch_cg_setup_state(CgState *st, int max_iter, double rtol, hipStream_t s);
template <typename TAp>
hb_status launch_cg_init(int64_t n, const double *b, double *x, double *r, double *p, TAp *Ap, int x0_zero,
                         CgWork &w, CgState *st, hipStream_t s);
hb_status launch_cg_alpha(CgWork &w, int ax_grid, CgState *st, hipStream_t s);
template <typename TAp>
hb_status launch_cg_residual(int64_t n, double *r, const TAp *Ap, CgWork &w, CgState *st, hipStream_t s);
hb_status launch_cg_beta(int64_t n, CgWork &w, CgState *st, hipStream_t s);
// alpha, residual, beta and update in one workgroup (vectors of at most
// kCgTailMax entries, four per thread; nax: the operator's partials).  Measured
// per CG iteration: 2197 DOFs 14.4 us against 16.4-17.1 us with the four
// launches, 6859 DOFs 19.0 against 17.5 us (one workgroup's bandwidth).
constexpr int64_t kCgTailMax = 4096;
template <typename TAp>
hb_status launch_cg_tail(int64_t n, double *x, double *p, double *r, TAp *Ap, const double *inv, CgWork &w, int nax,
                         CgState *st, hipStream_t s);
template <typename TAp>
hb_status launch_cg_update(int64_t n, double *x, double *p, const double *r, TAp *Ap, const double *inv, CgState *st,
                          hipStream_t s);
// 1 / diag(A) into inv (Jacobi preconditioner), for the mesh's operator at lambda.
hb_status launch_jacobi_inverse(const hb_mesh_s *m, double lambda, double *inv, hipStream_t s);
// Residual replacement after the completed iterations: r = b - t (t = A x
// from the FP64 operator), rho_iters = r.r (r.z with the Jacobi inverse
// diagonal inv), history entry iters = ||r||, *out = r.r; then the solve
// resumes with a new stopping threshold on ||r||.
hb_status launch_cg_replace(int64_t n, const double *b, const double *t, double *r, CgWork &w, CgState *st,
                            double *out, const double *inv, hipStream_t s);
hb_status launch_cg_resume(CgState *st, double stop_res, hipStream_t s);
// Refinement helpers: r = b - t with ||r||^2 into *out (one block finishes), and x += d.
hb_status launch_residual_norm(int64_t n, const double *b, const double *t, double *r, CgWork &w, double *out,
                               hipStream_t s);
hb_status launch_axpy(int64_t n, double *x, const double *d, hipStream_t s);
// FP64 -> FP32 rounding of an array (geometry and D of HB_MESH_FP32 meshes).
hb_status launch_round_f32(const double *in, float *out, int64_t n, hipStream_t s);

// Batched kernels (batch.hip).  Vector chunks hold kBatchChunk entries (four per
// thread: 4096-entry chunks ran the 64-problem batch 6% slower).
constexpr int kBatchChunk = 1024;
// sched: the class's tile schedule (the one its work list was built for);
// D: the degree's derivative matrix (FP32 copy when fp32), shared by the class;
// dirichlet: the class's problems are Dirichlet boxes.
hb_status launch_batch_ax(int N, int sched, const void *D, bool fp32, bool dirichlet, const WorkItem *items,
                          int nitems, const BatchProb *probs, hipStream_t s);
hb_status launch_batch_alpha(const int32_t *plist, int np, const BatchProb *probs, hipStream_t s);
hb_status launch_batch_residual(const WorkItem *items, int nitems, const BatchProb *probs, hipStream_t s);
hb_status launch_batch_beta(const int32_t *plist, int np, const BatchProb *probs, hipStream_t s);
hb_status launch_batch_update(const WorkItem *items, int nitems, const BatchProb *probs, hipStream_t s);

// The persistent batched launch (persist.hip): every running problem advances
// up to slots[p].iters iterations inside one cooperative launch of `nwg`
// workgroups, each problem on its own workgroups (wgs), synchronised by
// per-problem barriers over the counters bar[p] (zero before the launch).  A
// barrier wait that exceeds its spin limit sets *err and ends the launch.
// Degrees the kernel is compiled for, its workgroup size, and how many of its
// workgroups the device holds at once (0 if it cannot be launched).
bool persist_degree(int N);
constexpr int kPersistThreads = 256;
int persist_capacity();
// Operator tiles of an N-degree box of E elements in the persistent kernel, and their walk.
int persist_tiles(int N, int64_t E);
TileWalk persist_walk(int N, int64_t nx, int64_t ny, int64_t nz);
hb_status launch_batch_persistent(bool dirichlet, const PersistWg *wgs, int nwg, const PersistSlot *slots,
                                  const BatchProb *probs, uint32_t *bar, int32_t *err, hipStream_t s);

// 8:1 streaming probe (stream.hip).
hb_status launch_stream_probe(const double *in, double *out, int64_t n, hipStream_t s);

}  // namespace hb
