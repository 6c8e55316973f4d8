/*
 * hbmi.h -- C ABI of an MI355X-native assembled spectral-element screened
 * Poisson operator and the conjugate-gradient solve around it.
 *
 * The method is hipBone's (Chalmers, Karakus, Austin, Swirydowicz &
 * Warburton, arXiv:2202.12477): a box mesh of E hexahedra of degree N,
 * the screened Poisson operator A = S + lambda*(mass) of eq. (poisson), with the
 * stiffness S = Z^T S_L Z of eq. (stiffness), S_L^e = D^T G^e D, applied
 * matrix-free to an *assembled* DOF vector (DOF Storage section), inside
 * Algorithm 1 (unpreconditioned CG; optionally with a Jacobi
 * preconditioner) with fused vector kernels (Conjugate gradient Iteration
 * section).
 *
 * Conventions shared by every entry point:
 *  - Every function returns hb_status and never throws.  On failure a
 *    thread-local message is available from hb_last_error().
 *  - "dev_" pointers are device (HBM) pointers of the current HIP device,
 *    8-byte aligned, not aliasing each other; the caller owns them.
 *  - "stream" is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it; functions that return host results synchronise it.
 *  - Assembled vectors have N_G = (nx*N+1)(ny*N+1)(nz*N+1) entries in
 *    lexicographic global order g = I + gx*(J + gy*K), gx = nx*N+1,
 *    gy = ny*N+1, where global node (I,J,K) = (ex*N+a, ey*N+b, ez*N+c) for local
 *    GLL node (a,b,c) of element (ex,ey,ez).  No boundary node is masked,
 *    except on meshes built with HB_MESH_DIRICHLET: there only the interior
 *    nodes carry DOFs, g = (I-1) + (gx-2)((J-1) + (gy-2)(K-1)).
 *  - A mesh object is not thread-safe: calls on one mesh from several host
 *    threads, or on several streams at once, must be serialised by the caller
 *    (the CG workspace is owned by the mesh).
 */
#ifndef HBMI_H
#define HBMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HB_OK = 0,
    HB_ERR_INVALID_ARG = 1,   /* null pointer, N outside 1..15, n < 1, lambda <= 0, jitter outside [0,0.5), ... */
    HB_ERR_OUT_OF_MEMORY = 2, /* device allocation failed */
    HB_ERR_DEVICE = 3,        /* no HIP device, or a HIP runtime error (message in hb_last_error) */
    HB_ERR_NOT_CONVERGED = 4, /* tolerance not met within max_iter (results are still filled) */
    HB_ERR_BREAKDOWN = 5,     /* p.Ap <= 0 or not finite during CG */
    HB_ERR_NONFINITE = 6,     /* the initial residual r0.r0 is NaN or Inf */
    HB_ERR_BUDGET = 7,        /* an engine request larger than the engine's whole memory budget */
    HB_ERR_BUSY = 8           /* reserved */
} hb_status;

/* Mass coefficient c of the lambda term (7th geometric value per node).
 * HB_MASS_GWJ: c = w_a w_b w_c J (GLL weight times Jacobian): A = S + lambda*M.
 * HB_MASS_INVDEG: c = 1/multiplicity of the node's global DOF, the inverse
 * degree weights W of the Poisson Operator section (Z^T W Z = I), giving
 * A = S + lambda*I exactly as eq. (poisson) writes it. */
typedef enum { HB_MASS_GWJ = 0, HB_MASS_INVDEG = 1 } hb_mass;

/* Mesh flags. */
enum {
    HB_MESH_FP32 = 1,     /* also keep FP32 geometric factors and D, for hb_ax_f32 and FP32 refinement */
    HB_MESH_DIRICHLET = 2, /* homogeneous Dirichlet box (the paper's experiments): the nodes on the boundary of
                             [0,1]^3 carry no DOF, so N_G = (nx N - 1)(ny N - 1)(nz N - 1), numbered
                             lexicographically over the interior nodes; needs nx N, ny N, nz N >= 2 */
    HB_MESH_GATHER = 4    /* two-phase operator (the Poisson Operator section's own form): the element kernel
                             (under the degree's default FP64 tile schedule; the schedule table does not apply)
                             writes the local vector y_L (8 N_L bytes kept with the mesh), then a gather sums
                             each DOF's local copies in ascending local order (Z^T as CSR rows, 4 (N_G + 1)
                             + 4 N_L bytes, built at creation from the map on the host).  Every hb_ax, hb_ax_add
                             and FP64 hb_cg_solve on the mesh uses it; its results are bit-identical from run
                             to run.  FP64 only: not with HB_MESH_FP32; not accepted by hb_batch_solve or the
                             engine; needs fewer than 2^32 local nodes */
};

/* Precision of hb_cg_solve. */
typedef enum {
    HB_PREC_FP64 = 0,     /* Algorithm 1 with the FP64 operator */
    HB_PREC_FP32_IR = 1,  /* FP64 iterative refinement, each correction solved by CG with the FP32 operator */
    HB_PREC_FP32_RR = 2   /* one CG with the FP32 operator and FP64 residual replacement */
} hb_prec;                /* both mixed modes need HB_MESH_FP32 */

/* Preconditioner of hb_cg_solve.  The paper's benchmark runs CG without one;
 * NekBone (whose benchmark hipBone re-implements) offers the Jacobi option. */
typedef enum {
    HB_PRECOND_NONE = 0,
    HB_PRECOND_JACOBI = 1 /* M = diag(A) (computed on the device per mesh and lambda, 8 N_G bytes kept with the
                             mesh's CG workspace): z = M^{-1} r replaces r in rho = r.z and p = z + beta p; the
                             residual history and the stop test stay on ||r|| */
} hb_precond;

typedef struct hb_mesh_s *hb_mesh;

/* Box mesh on [0,1]^3 (NekBone section: a regular mesh of E hexahedra with
 * (N+1)^3 GLL nodes each).  Trilinear elements: vertices strictly inside the
 * box are moved by h_d*jitter*(2U-1) per coordinate d, U uniform in [0,1) from
 * the splitmix64 stream d+1 of `seed` at the vertex's lexicographic index
 * i + (nx+1)(j + (ny+1)k) (the same counter-based generator as hb_rhs_uniform). */
typedef struct {
    int32_t nx, ny, nz; /* elements per direction, >= 1 */
    int32_t N;          /* polynomial degree, 1..15 */
    double jitter;      /* 0 <= jitter < 0.5 (0: affine box) */
    uint64_t seed;      /* jitter seed */
    int32_t mass;       /* hb_mass */
    int32_t flags;      /* HB_MESH_FP32 | HB_MESH_DIRICHLET, or 0 */
} hb_mesh_desc;

typedef struct {
    int64_t n_elem;       /* E */
    int64_t n_local;      /* N_L = E (N+1)^3 */
    int64_t n_global;     /* N_G */
    int32_t N;
    int32_t reserved;
    size_t device_bytes;  /* device memory currently held by the mesh (geometry, map, D, CG workspace) */
} hb_mesh_info;

/* Build the mesh on the device: GLL nodes/weights and the 1D derivative
 * matrix D (NekBone section), the scatter map Z as int32 [E][(N+1)^3], and the
 * geometric factors G_rr, G_rs, G_rt, G_ss, G_st, G_tt and c in FP64
 * (G_dd' = w_a w_b w_c J sum_i dxi_d/dx_i dxi_d'/dx_i, the metric tensor
 * combined with the GLL weights), 56 bytes per local node, stored per element
 * layer by layer ([E][N+1][7][(N+1)^2]) so the operator reads each element's
 * factors as one sequential stream (hb_mesh_export returns [E][7][(N+1)^3]).
 * With HB_MESH_FP32 the mesh also keeps the factors and D rounded once to FP32
 * (28 more bytes per local node).  Synchronises `stream`.
 * Errors: HB_ERR_INVALID_ARG (bad desc, N_G or N_L >= 2^31, non-positive
 * Jacobian), HB_ERR_OUT_OF_MEMORY, HB_ERR_DEVICE.  *out is NULL on failure. */
hb_status hb_mesh_create(const hb_mesh_desc *desc, void *stream, hb_mesh *out);

/* Release every device buffer of the mesh.  NULL is accepted (no-op). */
hb_status hb_mesh_destroy(hb_mesh mesh);

hb_status hb_mesh_query(hb_mesh mesh, hb_mesh_info *info);

/* Copy mesh data to host memory (any pointer may be NULL to skip it):
 * host_geo: 7*N_L doubles, layout [E][7][(N+1)^3]; host_map: N_L int32
 * (-1 for a boundary node of a HB_MESH_DIRICHLET mesh);
 * host_D: (N+1)^2 doubles row-major, D[i][j] = l_j'(xi_i);
 * host_xi, host_w: N+1 doubles each (GLL nodes ascending, weights).
 * Synchronous. */
hb_status hb_mesh_export(hb_mesh mesh, double *host_geo, int32_t *host_map, double *host_D, double *host_xi,
                         double *host_w);

/* Forcing vector (HipBone section: filled once by a pseudo-random kernel):
 * dev_b[g] = 2U - 1 in [-1,1), U from splitmix64 (Steele, Lea & Flood 2014)
 * stream 0 of `seed`: the stream starts at output number 0 of the sequence
 * started at `seed`; U is the top 53 bits of that stream's output number g,
 * times 2^-53.  Asynchronous.  n >= 0. */
hb_status hb_rhs_uniform(int64_t n, uint64_t seed, double *dev_b, void *stream);

/* y = A x (eq. poisson / eq. stiffness, fused): gather x through Z, apply
 * D (r,s,t), the 6 symmetric G factors and lambda*c, apply D^T, and assemble
 * with Z^T into y.  x and y are FP64 device vectors of N_G entries and must not
 * overlap.  y is overwritten.  lambda > 0 (with no masked boundary S has
 * the constants in its null space, so lambda = 0 makes A singular).
 * Asynchronous; assembly uses device atomics, so results may differ between
 * calls in the last bits (summation order).  Not thread-safe per mesh. */
hb_status hb_ax(hb_mesh mesh, double lambda, const double *dev_x, double *dev_y, void *stream);

/* y += A x: the same fused operator, assembling into y without clearing it
 * first (hb_ax = clear y, then this).  Same arguments and rules as hb_ax. */
hb_status hb_ax_add(hb_mesh mesh, double lambda, const double *dev_x, double *dev_y, void *stream);

/* y = A x with the FP32 operator: x is read as FP64 and rounded to FP32; the
 * FP32 geometric factors and D, FP32 arithmetic and FP32 atomic assembly give
 * y (FP32, N_G entries, overwritten).  Needs a mesh built with HB_MESH_FP32.
 * Same rules as hb_ax otherwise.  The paper is FP64 throughout; this is the
 * reduced-precision operator of the mixed-precision solver. */
hb_status hb_ax_f32(hb_mesh mesh, double lambda, const double *dev_x, float *dev_y, void *stream);

/* Options of hb_cg_solve (Algorithm 1). */
typedef struct {
    int32_t max_iter;    /* FP64: iteration cap (>= 0), in fixed mode the exact count;
                            FP32_IR / FP32_RR: cap on the CG iterations in total */
    int32_t fixed_iters; /* 1: run exactly max_iter iterations (the benchmark's 100); 0: stop on rtol.
                            the mixed modes require 0. */
    double rtol;         /* FP64: stop once ||r_j|| <= rtol ||b|| (recursive residual);
                            FP32_IR / FP32_RR: stop once ||b - A x|| <= rtol ||b|| with the FP64 operator */
    int32_t x0_zero;     /* 1: ignore dev_x on entry and start from x0 = 0 (r0 = b, no operator call) */
    int32_t check_every; /* tolerance mode: read the device state back every this many iterations (<=0: 25) */
    int32_t prec;        /* hb_prec */
    int32_t max_outer;   /* FP32_IR: cap on refinement steps (<=0: 60); FP32_RR: cap on replacements (<=0: none) */
    double inner_rtol;   /* FP32_IR: inner solves reduce ||r|| by this factor; FP32_RR: replace the residual
                            each time the recursive ||r|| has dropped by this factor (<=0: 1e-3) */
    int32_t graph_k;     /* hb_cg_solve: > 0 enqueues the iterations as replays of one captured HIP graph of
                            graph_k iterations (cached per mesh for the same lambda, x and precision; a replay
                            past the stop is a no-op on the device); 0: one launch per kernel.
                            hb_batch_solve: > 0 makes each segment graph_k iterations long (instead of
                            check_every) and replays it from a captured graph until the set of running
                            problems changes. At most 4096. */
    int32_t precond;     /* hb_precond: HB_PRECOND_JACOBI in every precision (HB_PREC_FP32_RR: each residual
                            replacement also recomputes r.z; HB_PREC_FP32_IR: the inner FP32 solves and the
                            FP64 fallback are preconditioned); hb_batch_solve: not with HB_PREC_FP32_IR */
    int32_t persistent;  /* hb_batch_solve: 1 runs each segment of iterations as ONE persistent cooperative launch
                            holding every running problem (each on its own workgroups, synchronised by barriers
                            among those workgroups only; the whole iteration -- operator with p.Ap, alpha,
                            residual with r.r, beta, update -- inside the launch), instead of one launch per
                            (degree, precision) class and four per step and iteration.  Used for the segments
                            whose running problems all have N in {3, 5, 7, 9} and are all plain or all Dirichlet
                            boxes (others use the per-step launches); same results up to the order of the
                            floating-point sums.  A barrier wait that times out ends the launch and the solve
                            with HB_ERR_DEVICE.  Ignored by hb_cg_solve.  0: per-step launches */
    int32_t autotune;    /* hb_batch_solve: 1 first sets the tile schedule of each (degree, operator precision)
                            class in the batch by timing every legal schedule on a synthetic box of the class's
                            total local nodes (rounded down to a power of two in [2^16, 2^26]; each such size
                            class is timed once per process, later calls install the cached winner).  Changes
                            the process-wide schedule table (hb_get_schedule).  Ignored by hb_cg_solve.
                            0: the table as it stands */
} hb_cg_opts;

typedef struct {
    int32_t iters;       /* CG iterations completed (FP32_IR: inner iterations in total) */
    int32_t status;      /* hb_status of the solve */
    double res0;         /* ||r_0|| */
    double res;          /* FP64: ||r_iters|| (recursive); mixed: ||b - A x|| (FP64 operator) at exit */
    double bnorm;        /* ||b|| */
    int32_t outer_iters; /* FP32_IR: refinement steps; FP32_RR: replacements (0 in FP64 mode) */
    int32_t fp64_iters;  /* mixed: FP64 CG iterations run after the FP32 operator stalled (0 if it did not) */
    int32_t persistent_segments; /* hb_batch_solve with opts->persistent: segments of this problem's iterations
                                    run inside persistent launches (0 elsewhere) */
} hb_cg_result;

/* Algorithm 1 on the assembled system A x = b: r0 = b - A x0, p = r0; per
 * iteration Ap = A p (with p.Ap fused into the operator), alpha = r.r / p.Ap,
 * x += alpha p, r -= alpha Ap fused with r.r, beta = r'.r' / r.r, p = r + beta p.
 * All scalars stay on the device; dot products are two-stage FP64 reductions
 * with a fixed final order.  Stops early (status) on p.Ap <= 0 (BREAKDOWN),
 * a non-finite r0.r0 (NONFINITE) or r.r == 0 (exact solution, OK).
 * dev_b: N_G doubles; dev_x: N_G doubles, initial guess in, solution out.
 * host_res_hist: NULL or room for max_iter+1 doubles, receives ||r_j||, j = 0..iters
 * (FP32_IR: the true residual ||b - A x_k|| of each refinement step k = 0..outer_iters).
 *
 * FP32_IR (mixed precision): x_0 = x0; repeat { r = b - A x_k with the FP64
 * operator; stop if ||r|| <= rtol ||b||; solve A_32 d = r by CG (FP32 operator,
 * FP64 vectors, dot products, residual updates) from d = 0 to
 * ||r_in|| <= eta_k ||r||, eta_k = max(inner_rtol, min(1/2, rtol ||b|| / (2 ||r||)))
 * (no tighter than the remaining reduction needs); x_{k+1} = x_k + d }.  If a refinement step
 * reduces ||r|| by less than a factor 2 (the FP32 operator's error times the
 * condition number is too large), the solve continues with FP64 CG from x and
 * reports it in fp64_iters.
 *
 * FP32_RR (mixed precision, keeps the Krylov sequence): CG whose operator is
 * the FP32 one; whenever the recursive ||r|| has dropped by inner_rtol since
 * the last replacement, r is replaced by b - A x computed with the FP64
 * operator (residual replacement, van der Vorst & Ye 2000) and the iteration
 * continues with the same search direction.  It stops when a replacement gives
 * ||b - A x|| <= rtol ||b||.  If a replacement shows less than a halving of the
 * true residual, the remaining iterations use the FP64 operator (fp64_iters).
 * outer_iters counts the replacements; iters the CG iterations in total;
 * host_res_hist receives the true residual at the start and at each replacement.
 * Synchronises `stream` before returning.  Returns the solve's status
 * (HB_OK, HB_ERR_NOT_CONVERGED, HB_ERR_BREAKDOWN, HB_ERR_NONFINITE) or an
 * argument/device error. */
hb_status hb_cg_solve(hb_mesh mesh, double lambda, const double *dev_b, double *dev_x, const hb_cg_opts *opts,
                      hb_cg_result *result, double *host_res_hist, void *stream);

/* hb_cg_solve without any allocation, for callers that cannot allocate device
 * memory (code under HIP stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, algorithm, kernels and results as
 * hb_cg_solve in HB_PREC_FP64 (plain or HB_PRECOND_JACOBI, fixed count or
 * tolerance), but the workspace (r, p, Ap, block partials, device state, the
 * rho and ||r|| histories, 1/diag(A)) lives in one static device buffer of
 * 64 MiB per GPU that the library holds until the process ends; no hipMalloc,
 * hipFree, pinned host allocation or graph is made.  The workspace needs
 * 24 N_G (32 N_G with Jacobi) + 16 (max_iter + 1) bytes plus the block
 * partials: N_G up to about 2.7M DOFs at 100 iterations.  Larger solves,
 * opts->prec other than HB_PREC_FP64 and opts->graph_k != 0 are rejected with
 * HB_ERR_INVALID_ARG before any device work.  Every call on one GPU shares
 * that GPU's buffer: calls that overlap in time on the same GPU (other host
 * threads, or other streams with work still in flight) race and give wrong
 * results; calls serialised on one stream are safe.  The Jacobi diagonal is
 * recomputed on every call (the buffer keeps no state between calls).
 * Synchronises `stream` before returning; returns what hb_cg_solve returns. */
hb_status hb_cg_solve_noalloc(hb_mesh mesh, double lambda, const double *dev_b, double *dev_x,
                              const hb_cg_opts *opts, hb_cg_result *result, double *host_res_hist, void *stream);

/* Batched solve of independent problems (each its own mesh, lambda, b, x):
 * every problem runs the same algorithm as hb_cg_solve (HB_PREC_FP64, fixed
 * count or tolerance; or HB_PREC_FP32_RR), but all problems advance together:
 * an iteration is one operator launch per (degree, precision) class over a
 * work list of (problem, element tile), then one launch each for the alpha,
 * residual, beta and update steps of all problems.  Each problem has its own
 * device state, so problems that stop early simply drop out of the work lists
 * at the next read-back (every opts->check_every iterations, default 25).
 * meshes[i] must be distinct (the CG workspace belongs to the mesh).
 * results[i] is filled for every problem; the return value is HB_OK if all
 * problems succeeded, else the status of the first that did not.
 * HB_PREC_FP32_IR is not available here.  Synchronises `stream`. */
hb_status hb_batch_solve(int32_t nprob, const hb_mesh *meshes, const double *lambdas, const double *const *dev_b,
                         double *const *dev_x, const hb_cg_opts *opts, hb_cg_result *results, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving engine: continuous batching of independent solve requests.       */
/* A request is a box mesh (hb_mesh_desc), lambda, a forcing seed (the       */
/* hb_rhs_uniform vector) and a tolerance.  hb_engine_step admits queued     */
/* requests first-in first-out while a slot is free and the request's device */
/* footprint fits in the budget (its mesh and forcing are built on the       */
/* device at admission), advances every admitted request by a number of CG   */
/* iterations in shared launches (as hb_batch_solve), and retires finished   */
/* requests: the solution is copied to host memory (kept until polled) and   */
/* the request's device memory is released.  An engine is not thread-safe.   */
/* ------------------------------------------------------------------------ */
typedef struct hb_engine_s *hb_engine;

typedef struct {
    size_t hbm_budget;      /* device bytes the admitted requests may hold in total */
    int32_t max_slots;      /* requests solved at once */
    int32_t prec;           /* HB_PREC_FP64 or HB_PREC_FP32_RR */
    int32_t max_iter;       /* per-request CG iteration cap */
    int32_t iters_per_step; /* iterations per hb_engine_step when its argument is <= 0 (<= 0: 25) */
    double inner_rtol;      /* HB_PREC_FP32_RR replacement factor (<= 0: 1e-3) */
    int32_t max_quota;      /* iteration quota per step: a request whose iteration costs at most 1/2^k of
                               the costliest running request's advances 2^k times the step's iterations,
                               capped at max_quota (<= 0: 64; 1: every request advances equally) */
    int32_t graphs;         /* 1: a step's launches are replays of a captured HIP graph, re-captured whenever
                               the set of running requests (or the step length) changes; 0: plain launches */
    int32_t precond;        /* hb_precond: HB_PRECOND_JACOBI solves every request with the Jacobi
                               preconditioner (either precision), its 1 / diag(A) (8 N_G bytes) part of the
                               footprint */
    int32_t autotune;       /* 1: at each admission, set the tile schedule of the request's (degree, operator
                               precision) class for the class's running local nodes, as hb_cg_opts.autotune
                               (each size class timed once per process); 0: the table as it stands */
} hb_engine_opts;

typedef struct {
    int32_t running;        /* admitted requests still iterating */
    int32_t queued;         /* submitted, not yet admitted */
    int32_t completed;      /* finished, not yet polled */
    int32_t reserved;
    size_t used_bytes;      /* footprint of the admitted requests */
    double admit_s;         /* host wall seconds spent admitting requests (mesh, forcing, CG start), since
                               creation: the device runs nothing of the engine's meanwhile */
    double iterate_s;       /* host wall seconds inside the steps' iterations (launches and their completion) */
    double retire_s;        /* host wall seconds retiring requests (solution to host memory, release) */
} hb_engine_info;

/* Device bytes a request holds while admitted (pure host arithmetic), without a
 * preconditioner (an engine with HB_PRECOND_JACOBI adds 8 N_G). */
hb_status hb_engine_footprint(const hb_mesh_desc *desc, int32_t prec, int32_t max_iter, size_t *bytes);
hb_status hb_engine_create(const hb_engine_opts *opts, void *stream, hb_engine *out);
/* Releases every device buffer (admitted requests are dropped).  NULL is accepted. */
hb_status hb_engine_destroy(hb_engine engine);
/* Queue a request; HB_ERR_BUDGET if its footprint exceeds the whole budget
 * (it could never be admitted).  Of desc->flags only HB_MESH_DIRICHLET is
 * taken; the engine adds HB_MESH_FP32 itself in mixed precision. */
hb_status hb_engine_submit(hb_engine engine, const hb_mesh_desc *desc, double lambda, uint64_t rhs_seed, double rtol,
                           uint64_t *ticket);
/* Admit, run `iters` iterations (<= 0: the engine default) of every admitted
 * request (cheaper requests up to max_quota times as many, see
 * hb_engine_opts), retire finished ones.  info may be NULL.  Synchronises the
 * stream. */
hb_status hb_engine_step(hb_engine engine, int32_t iters, hb_engine_info *info);
/* *done = 1 and the results (host_x: N_G doubles, may be NULL) if the request
 * has finished; the engine then forgets it.  *done = 0 otherwise. */
hb_status hb_engine_poll(hb_engine engine, uint64_t ticket, int32_t *done, double *host_x, hb_cg_result *result);

/* ------------------------------------------------------------------------ */
/* Operator tile schedules and their autotuner.                              */
/* The operator (single, CG and batched launches) runs one of the compiled  */
/* tile schedules per (degree, precision) class: bit 0 (1) reads the        */
/* columns of D for the divergence from LDS instead of registers; bit 1 (2)  */
/* uses one-wave workgroups instead of 256-thread workgroups (N <= 7, where  */
/* an element fits in a wave); bit 2 (4) keeps no f_t array and targets two  */
/* waves per SIMD (N >= 8); bit 3 (8, N <= 10, not with bit 1; with bits 2  */
/* and 4 only as 29, the merged three-wave form, N = 8-10) makes the k       */
/* elements of a 256-thread workgroup x-consecutive (k = 4 at               */
/* N = 7), sums their shared faces in LDS and assembles each row of kN+1    */
/* DOFs once (where k does not divide nx, each row of the box ends in a     */
/* shorter tile);                                                           */
/* bit 4 (16, N >= 8, only with bits 0 and 2: value 21, or 29) also reads   */
/* the rows of D from LDS, keeps the map column in LDS between gather and    */
/* assembly, prefetches one geometry layer instead of two (FP64) and targets */
/* three waves per SIMD.                                                     */
/* Schedule values are 0..31.  While a class's entry is the built-in default */
/* (neither set nor autotuned), a single-problem launch of fewer than 256    */
/* workgroups (a tiny mesh) uses the one-wave form of that schedule where    */
/* an element fits a wave, and a merged schedule (bit 3) runs without bit 3  */
/* where its padded rows would fill less than 85% of the tile slots (per     */
/* mesh; per class over the running problems in batched solves).  The       */
/* choice changes the reduction grouping of p.Ap, the order of assembly      */
/* atomics and of the t-part sums only (results                              */
/* agree to rounding).  The table is process-wide, starts from measured      */
/* defaults, and must not be changed while solves are in flight.  `prec`:    */
/* HB_PREC_FP64 selects the FP64 operator's entry, either mixed precision    */
/* the FP32 one.                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t schedule;   /* the schedule chosen (now in the table) */
    int32_t candidates; /* schedules timed */
    double us[32];      /* mean launch time per schedule value in microseconds; < 0: not available here */
} hb_tune_result;

/* Current schedule of a class. */
hb_status hb_get_schedule(int32_t N, int32_t prec, int32_t *schedule);
/* Pin a class's schedule (HB_ERR_INVALID_ARG if it is not available at N). */
hb_status hb_set_schedule(int32_t N, int32_t prec, int32_t schedule);
/* Time every available schedule of a class on a synthetic jittered cubic box
 * of about `local_nodes` local nodes (<= 0: 2^22; at most 2^30; the best
 * schedule depends on the problem size, so tune at the size that will run),
 * built and freed here (device allocation), `reps` back-to-back y += A x
 * launches each (<= 0: 20; at most 10000) after 128 untimed launches that
 * bring the device up to speed, and put the fastest in the table.
 * out may be NULL.  Synchronises `stream`. */
hb_status hb_autotune(int32_t N, int32_t prec, int64_t local_nodes, int32_t reps, hb_tune_result *out,
                      void *stream);

/* Empirical streaming probe of the Computational Tests section: every thread
 * reads 8 FP64 values and writes one (8:1 read:write), dev_out[i] =
 * sum_k dev_in[k*n + i], k = 0..7.  dev_in: 8n doubles, dev_out: n doubles.
 * Asynchronous. */
hb_status hb_stream_probe(const double *dev_in, double *dev_out, int64_t n, void *stream);

const char *hb_status_string(hb_status status);
const char *hb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HBMI_H */
