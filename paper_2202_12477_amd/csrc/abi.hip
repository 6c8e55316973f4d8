// The extern "C" entry points declared in include/hbmi.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "solver.h"

namespace hb {

namespace {
thread_local std::string g_last_error;

hb_status check_device()
{
    int n = 0;
    const hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
        (void)hipGetLastError();
        return fail(HB_ERR_DEVICE, "no HIP device available");
    }
    return HB_OK;
}



void free_mesh(hb_mesh_s *m)
{
    if (!m) return;
    free_cg(m);
    if (m->map) (void)hipFree(m->map);
    for (double *p : {m->geo, m->D, m->xi, m->w, m->yl})
        if (p) (void)hipFree(p);
    for (uint32_t *p : {m->zt_off, m->zt_idx})
        if (p) (void)hipFree(p);
    for (float *p : {m->geo32, m->D32})
        if (p) (void)hipFree(p);
    delete m;
}

}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

hb_status fail(hb_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

hb_status hip_fail(hipError_t err, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(err);
    return HB_ERR_DEVICE;
}

}  // namespace hb

using namespace hb;

extern "C" {

const char *hb_status_string(hb_status s)
{
    switch (s) {
    case HB_OK: return "HB_OK";
    case HB_ERR_INVALID_ARG: return "HB_ERR_INVALID_ARG";
    case HB_ERR_OUT_OF_MEMORY: return "HB_ERR_OUT_OF_MEMORY";
    case HB_ERR_DEVICE: return "HB_ERR_DEVICE";
    case HB_ERR_NOT_CONVERGED: return "HB_ERR_NOT_CONVERGED";
    case HB_ERR_BREAKDOWN: return "HB_ERR_BREAKDOWN";
    case HB_ERR_NONFINITE: return "HB_ERR_NONFINITE";
    case HB_ERR_BUDGET: return "HB_ERR_BUDGET";
    case HB_ERR_BUSY: return "HB_ERR_BUSY";
    }
    return "HB_UNKNOWN_STATUS";
}

const char *hb_last_error(void) { return g_last_error.c_str(); }

hb_status hb_mesh_create(const hb_mesh_desc *desc, void *stream, hb_mesh *out)
{
    if (out) *out = nullptr;
    if (!desc || !out) return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: null argument");
    const hb_mesh_desc d = *desc;
    if (d.N < 1 || d.N > kMaxN) return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: N must be in 1..15");
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: element counts must be >= 1");
    if (!(d.jitter >= 0.0 && d.jitter < 0.5)) return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: jitter must be in [0, 0.5)");
    if (d.mass != HB_MASS_GWJ && d.mass != HB_MASS_INVDEG) return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: bad mass kind");
    if (d.flags & ~(HB_MESH_FP32 | HB_MESH_DIRICHLET | HB_MESH_GATHER))
        return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: unknown flag");
    if ((d.flags & HB_MESH_GATHER) && (d.flags & HB_MESH_FP32))
        return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: the two-phase operator is FP64 only (HB_MESH_GATHER excludes HB_MESH_FP32)");
    if ((d.flags & HB_MESH_DIRICHLET) && ((int64_t)d.nx * d.N < 2 || (int64_t)d.ny * d.N < 2 || (int64_t)d.nz * d.N < 2))
        return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: a Dirichlet box needs interior nodes (n*N >= 2)");
    const int64_t n1 = d.N + 1;
    const double E_d = (double)d.nx * d.ny * d.nz;
    const double NL_d = E_d * n1 * n1 * n1;
    const double NG_d = ((double)d.nx * d.N + 1) * ((double)d.ny * d.N + 1) * ((double)d.nz * d.N + 1);  // bound
    if (NL_d >= 2147483647.0 || NG_d >= 2147483647.0)
        return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: local or global node count exceeds the int32 map");
    hb_status st = check_device();
    if (st) return st;

    hb_mesh_s *m = new (std::nothrow) hb_mesh_s();
    if (!m) return fail(HB_ERR_OUT_OF_MEMORY, "hb_mesh_create: host allocation failed");
    m->desc = d;
    m->N = d.N;
    m->E = (int64_t)d.nx * d.ny * d.nz;
    m->NL = m->E * n1 * n1 * n1;
    m->NG = box_global_nodes(d);
    gll_basis(d.N, m->h_xi, m->h_w, m->h_D);
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t tally = 0;
    if ((st = dev_alloc(&m->map, m->NL, &tally)) || (st = dev_alloc(&m->geo, kGeo * m->NL, &tally)) ||
        (st = dev_alloc(&m->D, n1 * n1, &tally)) || (st = dev_alloc(&m->xi, n1, &tally)) ||
        (st = dev_alloc(&m->w, n1, &tally))) {
        free_mesh(m);
        return st;
    }
    m->device_bytes = tally;
    hipError_t e;
    if ((e = hipMemcpyAsync(m->D, m->h_D, sizeof(double) * n1 * n1, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(m->xi, m->h_xi, sizeof(double) * n1, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(m->w, m->h_w, sizeof(double) * n1, hipMemcpyHostToDevice, s)) != hipSuccess) {
        free_mesh(m);
        return hip_fail(e, "hb_mesh_create: copy of the 1D basis");
    }
    if ((st = build_geometry(m, s))) {
        free_mesh(m);
        return st;
    }
    if ((d.flags & HB_MESH_GATHER) && (st = build_gather(m, s))) {
        free_mesh(m);
        return st;
    }
    if (d.flags & HB_MESH_FP32) {
        if ((st = dev_alloc(&m->geo32, kGeo * m->NL, &m->device_bytes)) ||
            (st = dev_alloc(&m->D32, n1 * n1, &m->device_bytes)) ||
            (st = launch_round_f32(m->geo, m->geo32, kGeo * m->NL, s)) ||
            (st = launch_round_f32(m->D, m->D32, n1 * n1, s))) {
            free_mesh(m);
            return st;
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) {
            free_mesh(m);
            return hip_fail(e, "hb_mesh_create: FP32 geometry");
        }
    }
    *out = m;
    return HB_OK;
}

hb_status hb_mesh_destroy(hb_mesh mesh)
{
    if (!mesh) return HB_OK;
    free_mesh(mesh);
    return HB_OK;
}

hb_status hb_mesh_query(hb_mesh m, hb_mesh_info *info)
{
    if (!m || !info) return fail(HB_ERR_INVALID_ARG, "hb_mesh_query: null argument");
    info->n_elem = m->E;
    info->n_local = m->NL;
    info->n_global = m->NG;
    info->N = m->N;
    info->reserved = 0;
    info->device_bytes = m->device_bytes;
    return HB_OK;
}

hb_status hb_mesh_export(hb_mesh m, double *host_geo, int32_t *host_map, double *host_D, double *host_xi, double *host_w)
{
    if (!m) return fail(HB_ERR_INVALID_ARG, "hb_mesh_export: null mesh");
    const int n1 = m->N + 1;
    if (host_geo) {
        // the device keeps each element layer-major ([E][layer][factor][(N+1)^2]);
        // the exported format is factor-major ([E][factor][(N+1)^3])
        std::vector<double> dev(static_cast<size_t>(kGeo) * m->NL);
        HB_HIP(hipMemcpy(dev.data(), m->geo, sizeof(double) * dev.size(), hipMemcpyDeviceToHost));
        const int64_t np2 = (int64_t)n1 * n1, np3 = np2 * n1;
        for (int64_t e = 0; e < m->E; ++e)
            for (int64_t c = 0; c < n1; ++c)
                for (int f = 0; f < kGeo; ++f)
                    std::memcpy(host_geo + (e * kGeo + f) * np3 + c * np2, dev.data() + ((e * n1 + c) * kGeo + f) * np2,
                                sizeof(double) * np2);
    }
    if (host_map) HB_HIP(hipMemcpy(host_map, m->map, sizeof(int32_t) * m->NL, hipMemcpyDeviceToHost));
    if (host_D) std::memcpy(host_D, m->h_D, sizeof(double) * n1 * n1);
    if (host_xi) std::memcpy(host_xi, m->h_xi, sizeof(double) * n1);
    if (host_w) std::memcpy(host_w, m->h_w, sizeof(double) * n1);
    return HB_OK;
}

hb_status hb_rhs_uniform(int64_t n, uint64_t seed, double *dev_b, void *stream)
{
    if (n < 0 || (n > 0 && !dev_b)) return fail(HB_ERR_INVALID_ARG, "hb_rhs_uniform: bad arguments");
    hb_status st = check_device();
    if (st) return st;
    return launch_rhs(n, seed, dev_b, static_cast<hipStream_t>(stream));
}

hb_status hb_ax(hb_mesh m, double lambda, const double *dev_x, double *dev_y, void *stream)
{
    if (!m || !dev_x || !dev_y) return fail(HB_ERR_INVALID_ARG, "hb_ax: null argument");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(HB_ERR_INVALID_ARG, "hb_ax: lambda must be finite and > 0");
    if (dev_x == dev_y) return fail(HB_ERR_INVALID_ARG, "hb_ax: x and y must not alias");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (m->desc.flags & HB_MESH_GATHER) return launch_ax_two_phase(m, lambda, dev_x, dev_y, nullptr, nullptr, true, s);
    hb_status st = launch_zero(dev_y, m->NG, s);
    if (st) return st;
    return launch_ax(m, lambda, dev_x, dev_y, nullptr, nullptr, s);
}

hb_status hb_ax_add(hb_mesh m, double lambda, const double *dev_x, double *dev_y, void *stream)
{
    if (!m || !dev_x || !dev_y) return fail(HB_ERR_INVALID_ARG, "hb_ax_add: null argument");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(HB_ERR_INVALID_ARG, "hb_ax_add: lambda must be finite and > 0");
    if (dev_x == dev_y) return fail(HB_ERR_INVALID_ARG, "hb_ax_add: x and y must not alias");
    return launch_ax(m, lambda, dev_x, dev_y, nullptr, nullptr, static_cast<hipStream_t>(stream));
}

hb_status hb_ax_f32(hb_mesh m, double lambda, const double *dev_x, float *dev_y, void *stream)
{
    if (!m || !dev_x || !dev_y) return fail(HB_ERR_INVALID_ARG, "hb_ax_f32: null argument");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(HB_ERR_INVALID_ARG, "hb_ax_f32: lambda must be finite and > 0");
    if (!m->geo32) return fail(HB_ERR_INVALID_ARG, "hb_ax_f32: the mesh was built without HB_MESH_FP32");
    if (static_cast<const void *>(dev_x) == static_cast<const void *>(dev_y))
        return fail(HB_ERR_INVALID_ARG, "hb_ax_f32: x and y must not alias");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hb_status st = launch_zero(dev_y, m->NG, s);
    if (st) return st;
    return launch_ax32(m, lambda, dev_x, dev_y, nullptr, nullptr, s);
}

hb_status hb_cg_solve(hb_mesh m, double lambda, const double *dev_b, double *dev_x, const hb_cg_opts *opts,
                      hb_cg_result *result, double *host_res_hist, void *stream)
{
    if (!m || !dev_b || !dev_x || !opts) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: null argument");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: lambda must be finite and > 0");
    if (opts->max_iter < 0) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: max_iter must be >= 0");
    if (!opts->fixed_iters && !(opts->rtol >= 0.0)) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: rtol must be >= 0");
    if (dev_b == dev_x) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: b and x must not alias");
    if (opts->graph_k < 0 || opts->graph_k > 4096)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: graph_k must be in [0, 4096]");
    if (opts->prec != HB_PREC_FP64 && opts->prec != HB_PREC_FP32_IR && opts->prec != HB_PREC_FP32_RR)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: unknown precision");
    const bool mixed = opts->prec != HB_PREC_FP64;
    if (mixed && opts->fixed_iters)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: mixed precision needs a tolerance (fixed_iters = 0)");
    if (mixed && !m->geo32)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: mixed precision needs a mesh built with HB_MESH_FP32");
    if (opts->precond != HB_PRECOND_NONE && opts->precond != HB_PRECOND_JACOBI)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: unknown preconditioner");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hb_status st = ensure_cg(m, opts->max_iter, mixed, opts->prec == HB_PREC_FP32_IR);
    if (st) return st;
    CgWork &w = m->cg;
    w.graph_k = opts->graph_k;
    const bool pc = opts->precond == HB_PRECOND_JACOBI;
    if (pc && (st = ensure_jacobi(m, lambda, s))) return st;
    // every CG iteration of this solve (inner solves of the refinement included)
    // is preconditioned; the flag is cleared on every way out
    struct PcScope {
        CgWork &w;
        PcScope(CgWork &w_, bool on) : w(w_) { w.pc = on; }
        ~PcScope() { w.pc = false; }
    } pc_scope(w, pc);
    if (opts->prec == HB_PREC_FP32_RR) return solve_replace(m, lambda, dev_b, dev_x, opts, result, host_res_hist, s);
    if (!mixed) {
        st = run_cg<double>(m, lambda, dev_b, dev_x, w.Ap, opts->x0_zero, opts->max_iter,
                            opts->fixed_iters ? -1.0 : opts->rtol, opts->check_every, s);
        if (st) return st;
        const CgState hs = *w.host_state;
        // ||r_0|| and ||r_iters|| (hist holds the residual norms in both forms of the iteration)
        double res0 = 0.0, res_last = 0.0;
        HB_HIP(hipMemcpy(&res0, w.hist, sizeof(double), hipMemcpyDeviceToHost));
        HB_HIP(hipMemcpy(&res_last, w.hist + hs.iters, sizeof(double), hipMemcpyDeviceToHost));
        if (host_res_hist)
            HB_HIP(hipMemcpy(host_res_hist, w.hist, sizeof(double) * (hs.iters + 1), hipMemcpyDeviceToHost));
        if (result) {
            *result = hb_cg_result{};
            result->iters = hs.iters;
            result->status = hs.status;
            result->res0 = res0;
            result->res = res_last;
            result->bnorm = std::sqrt(hs.bb);
        }
        return static_cast<hb_status>(hs.status);
    }

    // FP64 iterative refinement around CG with the FP32 operator.
    const int max_outer = opts->max_outer > 0 ? opts->max_outer : 60;
    const double eta = opts->inner_rtol > 0.0 ? opts->inner_rtol : 1e-3;
    const int64_t n = m->NG;
    if (opts->x0_zero && (st = launch_zero(dev_x, n, s))) return st;
    double bb = 0.0;
    {
        // ||b||: r = b - 0
        if ((st = launch_zero(w.Ap, n, s)) || (st = launch_residual_norm(n, dev_b, w.Ap, w.rout, w, w.dnorm, s)))
            return st;
        HB_HIP(hipMemcpyAsync(w.host_norm, w.dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
        HB_HIP(hipStreamSynchronize(s));
        bb = *w.host_norm;
    }
    const double bnorm = std::sqrt(bb);
    if (!std::isfinite(bnorm)) {
        if (result) {
            *result = hb_cg_result{};
            result->status = HB_ERR_NONFINITE;
        }
        return HB_ERR_NONFINITE;
    }
    int outer = 0, inner_total = 0, fp64_iters = 0;
    hb_status status = HB_ERR_NOT_CONVERGED;
    double res = 0.0, res_prev = 0.0, res0 = 0.0;
    for (;; ++outer) {
        double rr = 0.0;
        if ((st = true_residual_sq(m, lambda, dev_b, dev_x, s, &rr))) return st;
        res = std::sqrt(rr);
        if (outer == 0) res0 = res;
        if (host_res_hist && outer <= opts->max_iter) host_res_hist[outer] = res;
        if (!std::isfinite(res)) {
            status = outer == 0 ? HB_ERR_NONFINITE : HB_ERR_BREAKDOWN;
            break;
        }
        if (res <= opts->rtol * bnorm) {
            status = HB_OK;
            break;
        }
        const bool stalled = outer > 0 && res > 0.5 * res_prev;
        if (stalled) {
            // The FP32 operator cannot reduce this residual any further: finish
            // with FP64 CG from the current iterate (true residual computed again below).
            const int budget = std::max(opts->max_iter - inner_total, 0);
            if ((st = run_cg<double>(m, lambda, dev_b, dev_x, w.Ap, 0, budget, opts->rtol, opts->check_every, s)))
                return st;
            fp64_iters = w.host_state->iters;
            if ((st = true_residual_sq(m, lambda, dev_b, dev_x, s, &rr))) return st;
            res = std::sqrt(rr);
            status = res <= opts->rtol * bnorm ? HB_OK : static_cast<hb_status>(
                w.host_state->status == HB_OK ? HB_ERR_NOT_CONVERGED : w.host_state->status);
            break;
        }
        if (outer >= max_outer || inner_total >= opts->max_iter) break;
        res_prev = res;
        // inner solve A_32 d = r (r = b - A x is in w.rout), to eta, or only as far as the
        // remaining reduction needs (with a factor 2 to spare, and never looser than 1/2)
        // when that is less
        const double inner = std::max(eta, std::min(0.5, 0.5 * opts->rtol * bnorm / res));
        if ((st = run_cg<float>(m, lambda, w.rout, w.d, w.Ap32, 1, opts->max_iter - inner_total, inner,
                                opts->check_every, s)))
            return st;
        inner_total += w.host_state->iters;
        if ((st = launch_axpy(n, dev_x, w.d, s))) return st;
    }
    HB_HIP(hipStreamSynchronize(s));
    if (result) {
        *result = hb_cg_result{};
        result->iters = inner_total;
        result->status = status;
        result->res0 = res0;
        result->res = res;
        result->bnorm = bnorm;
        result->outer_iters = outer;
        result->fp64_iters = fp64_iters;
    }
    return status;
}

hb_status hb_stream_probe(const double *dev_in, double *dev_out, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!dev_in || !dev_out))) return fail(HB_ERR_INVALID_ARG, "hb_stream_probe: bad arguments");
    return launch_stream_probe(dev_in, dev_out, n, static_cast<hipStream_t>(stream));
}

}  // extern "C"
