// Host-side drivers of the CG solves: the per-mesh workspace, Algorithm 1 on
// one problem, and the residual-replacement controller of the mixed-precision
// solve (also used by the batched runner and the serving engine).
#include <algorithm>
#include <cmath>
#include <string>

#include "common.h"
#include "solver.h"

namespace hb {

static void drop_graphs(CgWork &w)
{
    for (CgWork::Graph &g : w.graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = CgWork::Graph{};
    }
}

void free_cg(hb_mesh_s *m)
{
    CgWork &w = m->cg;
    for (double *p : {w.r, w.p, w.Ap, w.part_ax, w.part_vec, w.rho, w.hist, w.rout, w.d, w.dnorm, w.jinv})
        if (p) (void)hipFree(p);
    if (w.Ap32) (void)hipFree(w.Ap32);
    if (w.state) (void)hipFree(w.state);
    if (w.host_state) (void)hipHostFree(w.host_state);
    if (w.host_norm) (void)hipHostFree(w.host_norm);
    drop_graphs(w);
    if (w.cap) (void)hipStreamDestroy(w.cap);
    m->device_bytes -= w.bytes;
    w = CgWork{};
}

// Size the CG workspace for this mesh and iteration cap.  mixed: also the
// FP32 operator output; refine: also the outer residual and correction of the
// restarted refinement.
hb_status ensure_cg(hb_mesh_s *m, int max_iter, bool mixed, bool refine)
{
    CgWork &w = m->cg;
    const int need_ax = ax_blocks_max(m);  // any schedule of either precision
    // three partial arrays for the first step of the preconditioned iteration,
    // two per chunk for the batched preconditioned one
    const int need_vec = static_cast<int>(
        std::max<int64_t>(3 * vec_blocks(m->NG), 2 * ((m->NG + kBatchChunk - 1) / kBatchChunk)));
    if (w.r && w.n == m->NG && w.hist_len >= max_iter + 1 && w.part_ax_len >= need_ax &&
        w.part_vec_len >= need_vec && (!mixed || w.Ap32) && (!refine || w.rout))
        return HB_OK;
    const int hist_len = std::max(max_iter + 1, w.hist_len);
    mixed = mixed || w.Ap32 || refine;
    refine = refine || w.rout;
    if (w.r) free_cg(m);
    size_t tally = 0;
    hb_status st;
    if ((st = dev_alloc(&w.r, m->NG, &tally)) || (st = dev_alloc(&w.p, m->NG, &tally)) ||
        (st = dev_alloc(&w.Ap, m->NG, &tally)) || (st = dev_alloc(&w.part_ax, need_ax, &tally)) ||
        (st = dev_alloc(&w.part_vec, need_vec, &tally)) || (st = dev_alloc(&w.rho, hist_len, &tally)) ||
        (st = dev_alloc(&w.hist, hist_len, &tally)) || (st = dev_alloc(&w.state, 1, &tally)) ||
        (st = dev_alloc(&w.dnorm, 1, &tally)) || (mixed && (st = dev_alloc(&w.Ap32, m->NG, &tally))) ||
        (refine && ((st = dev_alloc(&w.rout, m->NG, &tally)) || (st = dev_alloc(&w.d, m->NG, &tally))))) {
        w.bytes = tally;
        m->device_bytes += tally;
        free_cg(m);
        return st;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&w.host_state), sizeof(CgState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&w.host_norm), sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        w.bytes = tally;
        m->device_bytes += tally;
        free_cg(m);
        return fail(HB_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
    }
    w.n = m->NG;
    w.hist_len = hist_len;
    w.part_ax_len = need_ax;
    w.part_vec_len = need_vec;
    w.bytes = tally;
    m->device_bytes += tally;
    return HB_OK;
}

// The operator for each output type: FP64 operator into double, FP32 into float.
hb_status apply_op(const hb_mesh_s *m, double l, const double *x, double *y, double *part, CgState *st, hipStream_t s)
{
    return launch_ax(m, l, x, y, part, st, s);
}
hb_status apply_op(const hb_mesh_s *m, double l, const double *x, float *y, double *part, CgState *st, hipStream_t s)
{
    return launch_ax32(m, l, x, y, part, st, s);
}

hb_status read_state(CgWork &w, hipStream_t s)
{
    HB_HIP(hipMemcpyAsync(w.host_state, w.state, sizeof(CgState), hipMemcpyDeviceToHost, s));
    HB_HIP(hipStreamSynchronize(s));
    return HB_OK;
}

// One CG iteration (Algorithm 1, loop body) with the operator whose output
// type is TAp: Ap = A p with p.Ap fused, alpha, r -= alpha Ap with r.r, beta,
// x += alpha p and p = r + beta p (which also clears Ap for the next operator).
template <typename TAp>
hb_status enqueue_iteration(hb_mesh_s *m, CgWork &w, double lambda, double *x, TAp *Ap, hipStream_t s)
{
    const int64_t n = m->NG;
    hb_status e;
    if ((e = apply_op(m, lambda, w.p, Ap, w.part_ax, w.state, s))) return e;
    if (n <= kCgTailMax)  // short vectors: the four steps after the operator in one workgroup
        return launch_cg_tail<TAp>(n, x, w.p, w.r, Ap, w.pc ? w.jinv : nullptr, w, ax_blocks(m, sizeof(TAp) == 4),
                                   w.state, s);
    if ((e = launch_cg_alpha(w, ax_blocks(m, sizeof(TAp) == 4), w.state, s))) return e;
    if ((e = launch_cg_residual<TAp>(n, w.r, Ap, w, w.state, s))) return e;
    if ((e = launch_cg_beta(n, w, w.state, s))) return e;
    return launch_cg_update<TAp>(n, x, w.p, w.r, Ap, w.pc ? w.jinv : nullptr, w.state, s);
}

// k iterations as one executable graph: the cached one with the same
// arguments, else captured on the workspace's private stream (every step of
// an iteration is a kernel launch, so the graph holds kernel nodes only).
template <typename TAp>
static hb_status iteration_graph(hb_mesh_s *m, double lambda, double *x, TAp *Ap, int k, hipGraphExec_t *out)
{
    CgWork &w = m->cg;
    for (const CgWork::Graph &g : w.graphs) {
        if (g.exec && g.elem == static_cast<int>(sizeof(TAp)) && g.k == k && g.lambda == lambda && g.x == x &&
            g.Ap == Ap && g.epoch == ax_schedule_epoch() && g.pc == w.pc) {
            *out = g.exec;
            return HB_OK;
        }
    }
    if (!w.cap) HB_HIP(hipStreamCreateWithFlags(&w.cap, hipStreamNonBlocking));
    CgWork::Graph &g = w.graphs[w.graph_next];
    w.graph_next ^= 1;
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = CgWork::Graph{};
    const int epoch = ax_schedule_epoch();
    HB_HIP(hipStreamBeginCapture(w.cap, hipStreamCaptureModeThreadLocal));
    hb_status st = HB_OK;
    for (int i = 0; i < k && st == HB_OK; ++i) st = enqueue_iteration<TAp>(m, w, lambda, x, Ap, w.cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(w.cap, &graph);
    if (st != HB_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != HB_OK ? st : hip_fail(e, "hipStreamEndCapture");
    }
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        g.exec = nullptr;
        return hip_fail(ei, "hipGraphInstantiate");
    }
    g.elem = static_cast<int>(sizeof(TAp));
    g.epoch = epoch;
    g.k = k;
    g.lambda = lambda;
    g.x = x;
    g.Ap = Ap;
    g.pc = w.pc;
    *out = g.exec;
    return HB_OK;
}

// Enqueue CG iterations with the operator whose output type is TAp until
// the device state stops the solve or max_iter iterations are complete; the
// state is left in w.host_state.  Fixed mode (every iteration runs) enqueues
// everything at once; otherwise the state is read back every `check_every`
// iterations.  With w.graph_k > 0 the iterations are replays of a captured
// graph of graph_k iterations; replays past the device's stop do nothing.
template <typename TAp>
hb_status cg_iterate(hb_mesh_s *m, double lambda, double *x, TAp *Ap, int max_iter, bool fixed, int check_every,
                     hipStream_t s)
{
    CgWork &w = m->cg;
    hb_status st;
    if ((st = read_state(w, s))) return st;
    int done_iters = w.host_state->iters;
    auto stopped = [&]() { return w.host_state->done || w.host_state->pending; };
    const int chunk = fixed ? std::max(max_iter - done_iters, 1) : (check_every > 0 ? check_every : 25);
    hipGraphExec_t graph = nullptr;
    if (w.graph_k > 0 && done_iters < max_iter && !stopped() &&
        (st = iteration_graph<TAp>(m, lambda, x, Ap, w.graph_k, &graph)))
        return st;
    while (done_iters < max_iter && !stopped()) {
        const int k = std::min(chunk, max_iter - done_iters);
        if (graph) {
            for (int i = 0; i < (k + w.graph_k - 1) / w.graph_k; ++i) HB_HIP(hipGraphLaunch(graph, s));
        } else {
            for (int i = 0; i < k; ++i)
                if ((st = enqueue_iteration<TAp>(m, w, lambda, x, Ap, s))) return st;
        }
        if ((st = read_state(w, s))) return st;
        done_iters = w.host_state->iters;
    }
    return HB_OK;
}

// Algorithm 1: r0 = b - A x0, p = r0, then iterations until the stop test.
template <typename TAp>
hb_status run_cg(hb_mesh_s *m, double lambda, const double *b, double *x, TAp *Ap, int x0_zero, int max_iter,
                 double rtol, int check_every, hipStream_t s)
{
    CgWork &w = m->cg;
    const int64_t n = m->NG;
    hb_status st;
    if ((st = launch_cg_setup_state(w.state, max_iter, rtol, s))) return st;
    if (!x0_zero) {
        if ((st = launch_zero(Ap, n, s)) || (st = apply_op(m, lambda, x, Ap, nullptr, nullptr, s))) return st;
    }
    if ((st = launch_cg_init<TAp>(n, b, x, w.r, w.p, Ap, x0_zero, w, w.state, s))) return st;
    return cg_iterate<TAp>(m, lambda, x, Ap, max_iter, rtol < 0.0, check_every, s);
}

// The Jacobi preconditioner's 1 / diag(A) for this lambda (the workspace must
// be sized; computed again only when lambda changes).
hb_status ensure_jacobi(hb_mesh_s *m, double lambda, hipStream_t s)
{
    CgWork &w = m->cg;
    if (!w.jinv) {
        size_t tally = 0;
        hb_status st = dev_alloc(&w.jinv, m->NG, &tally);
        if (st) return st;
        w.bytes += tally;
        m->device_bytes += tally;
        w.jvalid = false;
    }
    if (w.jvalid && w.jlambda == lambda) return HB_OK;
    hb_status st = launch_jacobi_inverse(m, lambda, w.jinv, s);
    if (st) return st;
    w.jlambda = lambda;
    w.jvalid = true;
    return HB_OK;
}

// ||b - A x||^2 with the FP64 operator (t = A x in w.Ap, r = b - t in w.rout).
hb_status true_residual_sq(hb_mesh_s *m, double lambda, const double *b, const double *x, hipStream_t s, double *out)
{
    CgWork &w = m->cg;
    hb_status st;
    if ((st = launch_zero(w.Ap, m->NG, s)) || (st = launch_ax(m, lambda, x, w.Ap, nullptr, nullptr, s)) ||
        (st = launch_residual_norm(m->NG, b, w.Ap, w.rout, w, w.dnorm, s)))
        return st;
    HB_HIP(hipMemcpyAsync(w.host_norm, w.dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
    HB_HIP(hipStreamSynchronize(s));
    *out = *w.host_norm;
    return HB_OK;
}

hb_status read_norm(CgWork &w, hipStream_t s, double *out)
{
    HB_HIP(hipMemcpyAsync(w.host_norm, w.dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
    HB_HIP(hipStreamSynchronize(s));
    *out = *w.host_norm;
    return HB_OK;
}

// Start a solve on the device: state, r0 = b - A x0, p = r0 (FP64 operator),
// zero FP32 operator output when mixed.
hb_status cg_start(hb_mesh_s *m, double lambda, const double *b, double *x, CgState *st, int x0_zero, int max_iter,
                   double rtol, bool mixed, hipStream_t s)
{
    CgWork &w = m->cg;
    const int64_t n = m->NG;
    hb_status e;
    if ((e = launch_cg_setup_state(st, max_iter, rtol, s))) return e;
    if (!x0_zero) {
        if ((e = launch_zero(w.Ap, n, s)) || (e = launch_ax(m, lambda, x, w.Ap, nullptr, nullptr, s))) return e;
    }
    if ((e = launch_cg_init<double>(n, b, x, w.r, w.p, w.Ap, x0_zero, w, st, s))) return e;
    if (mixed && (e = launch_zero(w.Ap32, n, s))) return e;
    return HB_OK;
}

// CG with the FP32 operator and FP64 residual replacement (one problem).
hb_status solve_replace(hb_mesh_s *m, double lambda, const double *b, double *x, const hb_cg_opts *opts,
                        hb_cg_result *result, double *hist, hipStream_t s)
{
    CgWork &w = m->cg;
    hb_status st;
    if ((st = cg_start(m, lambda, b, x, w.state, opts->x0_zero, opts->max_iter, opts->rtol, true, s)) ||
        (st = read_state(w, s)))
        return st;
    double res0 = 0.0;  // ||r0|| (the first history entry, also when preconditioned)
    HB_HIP(hipMemcpy(&res0, w.hist, sizeof(double), hipMemcpyDeviceToHost));
    Replacer rp;
    rp.inv = w.pc ? w.jinv : nullptr;
    rp.start(opts, res0, std::sqrt(w.host_state->bb), w.host_state->done != 0,
             static_cast<hb_status>(w.host_state->status));
    if (hist && opts->max_iter >= 0) hist[0] = rp.res0;
    if (!rp.finished && (st = launch_cg_resume(w.state, rp.threshold(), s))) return st;
    while (!rp.finished) {
        st = rp.use32 ? cg_iterate<float>(m, lambda, x, w.Ap32, opts->max_iter, false, opts->check_every, s)
                      : cg_iterate<double>(m, lambda, x, w.Ap, opts->max_iter, false, opts->check_every, s);
        if (st) return st;
        const CgState hs = *w.host_state;
        bool enq = false;
        if ((st = rp.replace(m, lambda, b, x, w.state, hs, w.dnorm, s, &enq))) return st;
        if (!enq) break;
        double rr = 0.0;
        if ((st = read_norm(w, s, &rr)) || (st = rp.decide(m, w.state, hs.iters, rr, hist, s))) return st;
    }
    HB_HIP(hipStreamSynchronize(s));
    if ((st = read_state(w, s))) return st;
    rp.fill(result, w.host_state->iters);
    return rp.status;
}


template hb_status enqueue_iteration<double>(hb_mesh_s *, CgWork &, double, double *, double *, hipStream_t);
template hb_status cg_iterate<double>(hb_mesh_s *, double, double *, double *, int, bool, int, hipStream_t);
template hb_status cg_iterate<float>(hb_mesh_s *, double, double *, float *, int, bool, int, hipStream_t);
template hb_status run_cg<double>(hb_mesh_s *, double, const double *, double *, double *, int, int, double, int,
                                  hipStream_t);
template hb_status run_cg<float>(hb_mesh_s *, double, const double *, double *, float *, int, int, double, int,
                                 hipStream_t);

}  // namespace hb
