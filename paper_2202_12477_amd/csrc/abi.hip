// The extern "C" entry points declared in include/hbmi.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"

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

template <typename T>
hb_status dev_alloc(T **p, size_t count, size_t *tally)
{
    if (hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * count) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(HB_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(sizeof(T) * count) + " bytes failed");
    }
    *tally += sizeof(T) * count;
    return HB_OK;
}

void free_cg(hb_mesh_s *m)
{
    CgWork &w = m->cg;
    for (double *p : {w.r, w.p, w.Ap, w.part_ax, w.part_vec, w.rho, w.hist, w.rout, w.d, w.dnorm})
        if (p) (void)hipFree(p);
    if (w.Ap32) (void)hipFree(w.Ap32);
    if (w.state) (void)hipFree(w.state);
    if (w.host_state) (void)hipHostFree(w.host_state);
    if (w.host_norm) (void)hipHostFree(w.host_norm);
    m->device_bytes -= w.bytes;
    w = CgWork{};
}

void free_mesh(hb_mesh_s *m)
{
    if (!m) return;
    free_cg(m);
    if (m->map) (void)hipFree(m->map);
    for (double *p : {m->geo, m->D, m->xi, m->w})
        if (p) (void)hipFree(p);
    for (float *p : {m->geo32, m->D32})
        if (p) (void)hipFree(p);
    delete m;
}

// Size the CG workspace for this mesh and iteration cap.
hb_status ensure_cg(hb_mesh_s *m, int max_iter, bool mixed)
{
    CgWork &w = m->cg;
    const int need_ax = ax_blocks(m);
    const int need_vec = static_cast<int>(std::max<int64_t>(2 * vec_blocks(m->NG), (m->NG + kBatchChunk - 1) / kBatchChunk));
    if (w.r && w.n == m->NG && w.hist_len >= max_iter + 1 && w.part_ax_len >= need_ax &&
        w.part_vec_len >= need_vec && (!mixed || w.Ap32))
        return HB_OK;
    const int hist_len = std::max(max_iter + 1, w.hist_len);
    mixed = mixed || w.Ap32;
    if (w.r) free_cg(m);
    size_t tally = 0;
    hb_status st;
    if ((st = dev_alloc(&w.r, m->NG, &tally)) || (st = dev_alloc(&w.p, m->NG, &tally)) ||
        (st = dev_alloc(&w.Ap, m->NG, &tally)) || (st = dev_alloc(&w.part_ax, need_ax, &tally)) ||
        (st = dev_alloc(&w.part_vec, need_vec, &tally)) || (st = dev_alloc(&w.rho, hist_len, &tally)) ||
        (st = dev_alloc(&w.hist, hist_len, &tally)) || (st = dev_alloc(&w.state, 1, &tally)) ||
        (st = dev_alloc(&w.dnorm, 1, &tally)) ||
        (mixed && ((st = dev_alloc(&w.rout, m->NG, &tally)) || (st = dev_alloc(&w.d, m->NG, &tally)) ||
                   (st = dev_alloc(&w.Ap32, m->NG, &tally))))) {
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

// Enqueue CG iterations with the operator whose output type is TAp until
// the device state stops the solve or max_iter iterations are complete; the
// state is left in w.host_state.  Fixed mode (every iteration runs) enqueues
// everything at once; otherwise the state is read back every `check_every`
// iterations.
template <typename TAp>
hb_status cg_iterate(hb_mesh_s *m, double lambda, double *x, TAp *Ap, int max_iter, bool fixed, int check_every,
                     hipStream_t s)
{
    CgWork &w = m->cg;
    const int64_t n = m->NG;
    const int axg = ax_blocks(m);
    hb_status st;
    auto enqueue_iteration = [&]() -> hb_status {
        hb_status e;
        if ((e = apply_op(m, lambda, w.p, Ap, w.part_ax, w.state, s))) return e;
        if ((e = launch_cg_alpha(w, axg, w.state, s))) return e;
        if ((e = launch_cg_residual<TAp>(n, w.r, Ap, w, w.state, s))) return e;
        if ((e = launch_cg_beta(n, w, w.state, s))) return e;
        return launch_cg_update<TAp>(n, x, w.p, w.r, Ap, w.state, s);
    };
    if ((st = read_state(w, s))) return st;
    int done_iters = w.host_state->iters;
    auto stopped = [&]() { return w.host_state->done || w.host_state->pending; };
    const int chunk = fixed ? std::max(max_iter - done_iters, 1) : (check_every > 0 ? check_every : 25);
    while (done_iters < max_iter && !stopped()) {
        const int k = std::min(chunk, max_iter - done_iters);
        for (int i = 0; i < k; ++i)
            if ((st = enqueue_iteration())) return st;
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

// Host-side control of one residual-replacement solve (FP32 operator, FP64
// replacements).  After the device has stopped a segment of iterations (the
// recursive residual met the segment's threshold, the iteration cap, or a
// breakdown), `replace` recomputes r = b - A x with the FP64 operator on the
// stream and `decide` (after the norm has been read back) either finishes the
// solve or resumes it with the next threshold, switching to the FP64 operator
// for good if the true residual fell by less than a factor 2 since the last
// replacement.
struct Replacer {
    double eta = 1e-3, rtol = 0.0, bnorm = 0.0, ref = 0.0, res = 0.0, res0 = 0.0;
    int max_iter = 0, max_outer = 0, outer = 0, fp64_from = -1;
    bool use32 = true, finished = false, breakdown = false;
    hb_status status = HB_ERR_NOT_CONVERGED;

    void start(const hb_cg_opts *o, double res0_, double bnorm_, bool already_done, hb_status st0)
    {
        eta = o->inner_rtol > 0.0 ? o->inner_rtol : 1e-3;
        rtol = o->rtol;
        max_iter = o->max_iter;
        max_outer = o->max_outer > 0 ? o->max_outer : 1000000;
        bnorm = bnorm_;
        res = ref = res0 = res0_;
        if (already_done) {
            finished = true;
            status = st0;
        }
    }
    double threshold() const { return use32 ? std::max(eta * ref, rtol * bnorm) : rtol * bnorm; }

    // Enqueue the replacement; returns true if one was enqueued.
    hb_status replace(hb_mesh_s *m, double lambda, const double *b, const double *x, CgState *st,
                      const CgState &hs, double *norm_out, hipStream_t s, bool *enqueued)
    {
        *enqueued = false;
        breakdown = hs.status == HB_ERR_BREAKDOWN;
        if (breakdown && !use32) {
            finished = true;
            status = HB_ERR_BREAKDOWN;
            return HB_OK;
        }
        CgWork &w = m->cg;
        hb_status e;
        if ((e = launch_zero(w.Ap, m->NG, s)) || (e = launch_ax(m, lambda, x, w.Ap, nullptr, nullptr, s)) ||
            (e = launch_cg_replace(m->NG, b, w.Ap, w.r, w, st, norm_out, s)))
            return e;
        *enqueued = true;
        return HB_OK;
    }

    // After the replacement's squared norm `rr` is on the host.
    hb_status decide(hb_mesh_s *m, CgState *st, int iters, double rr, double *hist, hipStream_t s)
    {
        ++outer;
        res = std::sqrt(rr);
        if (hist && outer <= max_iter) hist[outer] = res;
        if (!std::isfinite(res)) {
            finished = true;
            status = HB_ERR_BREAKDOWN;
            return HB_OK;
        }
        if (res <= rtol * bnorm) {
            finished = true;
            status = HB_OK;
            return HB_OK;
        }
        if (iters >= max_iter || outer >= max_outer) {
            finished = true;
            status = HB_ERR_NOT_CONVERGED;
            return HB_OK;
        }
        if (use32 && (breakdown || res > 0.5 * ref)) {
            use32 = false;
            fp64_from = iters;
        }
        ref = res;
        CgWork &w = m->cg;
        hb_status e;
        // both operator outputs start the next segment at zero (w.Ap held A x)
        if ((e = launch_zero(w.Ap, m->NG, s)) || (e = launch_zero(w.Ap32, m->NG, s)) ||
            (e = launch_cg_resume(st, threshold(), s)))
            return e;
        return HB_OK;
    }

    void fill(hb_cg_result *r, int iters) const
    {
        if (!r) return;
        *r = hb_cg_result{};
        r->iters = iters;
        r->status = status;
        r->res0 = res0;
        r->res = res;
        r->bnorm = bnorm;
        r->outer_iters = outer;
        r->fp64_iters = fp64_from >= 0 ? iters - fp64_from : 0;
    }
};

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
    double rho0 = 0.0;
    HB_HIP(hipMemcpy(&rho0, w.rho, sizeof(double), hipMemcpyDeviceToHost));
    Replacer rp;
    rp.start(opts, std::sqrt(rho0), std::sqrt(w.host_state->bb), w.host_state->done != 0,
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
    if (d.flags & ~HB_MESH_FP32) return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: unknown flag");
    const int64_t n1 = d.N + 1;
    const double E_d = (double)d.nx * d.ny * d.nz;
    const double NL_d = E_d * n1 * n1 * n1;
    const double NG_d = ((double)d.nx * d.N + 1) * ((double)d.ny * d.N + 1) * ((double)d.nz * d.N + 1);
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
    m->NG = ((int64_t)d.nx * d.N + 1) * ((int64_t)d.ny * d.N + 1) * ((int64_t)d.nz * d.N + 1);
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
    if (host_geo) HB_HIP(hipMemcpy(host_geo, m->geo, sizeof(double) * kGeo * m->NL, hipMemcpyDeviceToHost));
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
    if (opts->prec != HB_PREC_FP64 && opts->prec != HB_PREC_FP32_IR && opts->prec != HB_PREC_FP32_RR)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: unknown precision");
    const bool mixed = opts->prec != HB_PREC_FP64;
    if (mixed && opts->fixed_iters)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: mixed precision needs a tolerance (fixed_iters = 0)");
    if (mixed && !m->geo32)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: mixed precision needs a mesh built with HB_MESH_FP32");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hb_status st = ensure_cg(m, opts->max_iter, mixed);
    if (st) return st;
    CgWork &w = m->cg;
    if (opts->prec == HB_PREC_FP32_RR) return solve_replace(m, lambda, dev_b, dev_x, opts, result, host_res_hist, s);
    if (!mixed) {
        if ((st = run_cg<double>(m, lambda, dev_b, dev_x, w.Ap, opts->x0_zero, opts->max_iter,
                                 opts->fixed_iters ? -1.0 : opts->rtol, opts->check_every, s)))
            return st;
        const CgState hs = *w.host_state;
        double rho0 = 0.0, rho_last = 0.0;
        HB_HIP(hipMemcpy(&rho0, w.rho, sizeof(double), hipMemcpyDeviceToHost));
        HB_HIP(hipMemcpy(&rho_last, w.rho + hs.iters, sizeof(double), hipMemcpyDeviceToHost));
        if (host_res_hist)
            HB_HIP(hipMemcpy(host_res_hist, w.hist, sizeof(double) * (hs.iters + 1), hipMemcpyDeviceToHost));
        if (result) {
            *result = hb_cg_result{};
            result->iters = hs.iters;
            result->status = hs.status;
            result->res0 = std::sqrt(rho0);
            result->res = std::sqrt(rho_last);
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
        // inner solve A_32 d = r (r = b - A x is in w.rout)
        if ((st = run_cg<float>(m, lambda, w.rout, w.d, w.Ap32, 1, opts->max_iter - inner_total, eta,
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

hb_status hb_batch_solve(int32_t nprob, const hb_mesh *meshes, const double *lambdas, const double *const *dev_b,
                         double *const *dev_x, const hb_cg_opts *opts, hb_cg_result *results, void *stream)
{
    if (nprob < 0 || (nprob > 0 && (!meshes || !lambdas || !dev_b || !dev_x || !results)) || !opts)
        return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: null argument");
    if (opts->prec != HB_PREC_FP64 && opts->prec != HB_PREC_FP32_RR)
        return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: precision must be HB_PREC_FP64 or HB_PREC_FP32_RR");
    const bool mixed = opts->prec == HB_PREC_FP32_RR;
    const bool fixed = opts->fixed_iters != 0;
    if (opts->max_iter < 0) return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: max_iter must be >= 0");
    if (mixed && fixed) return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: mixed precision needs a tolerance");
    if (!fixed && !(opts->rtol >= 0.0)) return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: rtol must be >= 0");
    for (int i = 0; i < nprob; ++i) {
        if (!meshes[i] || !dev_b[i] || !dev_x[i] || dev_b[i] == dev_x[i])
            return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: problem " + std::to_string(i) + ": bad pointers");
        if (!(lambdas[i] > 0.0) || !std::isfinite(lambdas[i]))
            return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: problem " + std::to_string(i) + ": lambda must be > 0");
        if (mixed && !meshes[i]->geo32)
            return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: problem " + std::to_string(i) + " has no FP32 data");
        for (int k = 0; k < i; ++k)
            if (meshes[k] == meshes[i])
                return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: a mesh appears twice (its workspace is per mesh)");
    }
    if (nprob == 0) return HB_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hb_status st;
    for (int i = 0; i < nprob; ++i)
        if ((st = ensure_cg(meshes[i], opts->max_iter, mixed))) return st;

    // batch tables: descriptors, states, work lists (device) and their host staging (pinned)
    int64_t cap_ax = 0, cap_vec = 0;
    for (int i = 0; i < nprob; ++i) {
        cap_ax += ax_blocks(meshes[i]);
        cap_vec += (meshes[i]->NG + kBatchChunk - 1) / kBatchChunk;
    }
    if (cap_ax + cap_vec > INT32_MAX) return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: batch too large");
    struct Buffers {
        BatchProb *probs = nullptr, *h_probs = nullptr;
        CgState *states = nullptr, *h_states = nullptr;
        WorkItem *items = nullptr, *h_items = nullptr;
        int32_t *plist = nullptr, *h_plist = nullptr;
        double *norms = nullptr, *h_norms = nullptr, *h_rho = nullptr;
        ~Buffers()
        {
            for (void *p : {(void *)probs, (void *)states, (void *)items, (void *)plist, (void *)norms})
                if (p) (void)hipFree(p);
            for (void *p : {(void *)h_probs, (void *)h_states, (void *)h_items, (void *)h_plist, (void *)h_norms,
                            (void *)h_rho})
                if (p) (void)hipHostFree(p);
        }
    } B;
    const size_t n_items = static_cast<size_t>(cap_ax + cap_vec);
    if (hipMalloc(&B.probs, sizeof(BatchProb) * nprob) != hipSuccess ||
        hipMalloc(&B.states, sizeof(CgState) * nprob) != hipSuccess ||
        hipMalloc(&B.items, sizeof(WorkItem) * n_items) != hipSuccess ||
        hipMalloc(&B.plist, sizeof(int32_t) * nprob) != hipSuccess ||
        hipMalloc(&B.norms, sizeof(double) * nprob) != hipSuccess ||
        hipHostMalloc(&B.h_probs, sizeof(BatchProb) * nprob, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&B.h_states, sizeof(CgState) * nprob, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&B.h_items, sizeof(WorkItem) * n_items, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&B.h_plist, sizeof(int32_t) * nprob, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&B.h_norms, sizeof(double) * nprob, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&B.h_rho, sizeof(double) * nprob, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(HB_ERR_OUT_OF_MEMORY, "hb_batch_solve: batch table allocation failed");
    }

    // start every problem (r0, p0 with the FP64 operator) and read the states back
    const double rtol = fixed ? -1.0 : opts->rtol;
    for (int i = 0; i < nprob; ++i) {
        hb_mesh_s *m = meshes[i];
        if ((st = cg_start(m, lambdas[i], dev_b[i], dev_x[i], B.states + i, opts->x0_zero, opts->max_iter, rtol,
                           mixed, s)))
            return st;
        HB_HIP(hipMemcpyAsync(B.h_rho + i, m->cg.rho, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HB_HIP(hipMemcpyAsync(B.h_states, B.states, sizeof(CgState) * nprob, hipMemcpyDeviceToHost, s));
    HB_HIP(hipStreamSynchronize(s));
    std::vector<Replacer> rp(nprob);
    std::vector<char> finished(nprob, 0);
    for (int i = 0; i < nprob; ++i) {
        const CgState &hs = B.h_states[i];
        if (mixed) {
            rp[i].start(opts, std::sqrt(B.h_rho[i]), std::sqrt(hs.bb), hs.done != 0, static_cast<hb_status>(hs.status));
            finished[i] = rp[i].finished;
            if (!finished[i] && (st = launch_cg_resume(B.states + i, rp[i].threshold(), s))) return st;
        } else {
            finished[i] = hs.done != 0;
        }
        hb_mesh_s *m = meshes[i];
        CgWork &w = m->cg;
        BatchProb &P = B.h_probs[i];
        P.map = m->map;
        P.geo = m->geo;
        P.geo32 = m->geo32;
        P.D = m->D;
        P.D32 = m->D32;
        P.lambda = lambdas[i];
        P.x = dev_x[i];
        P.r = w.r;
        P.p = w.p;
        P.Ap = w.Ap;
        P.Ap32 = w.Ap32;
        P.rho = w.rho;
        P.hist = w.hist;
        P.part_ax = w.part_ax;
        P.part_vec = w.part_vec;
        P.st = B.states + i;
        P.E = m->E;
        P.NG = m->NG;
        P.N = m->N;
        P.ax_tiles = ax_blocks(m);
        P.vec_chunks = static_cast<int32_t>((m->NG + kBatchChunk - 1) / kBatchChunk);
        P.use32 = mixed ? 1 : 0;
    }
    const int chunk = fixed ? std::max(opts->max_iter, 1) : (opts->check_every > 0 ? opts->check_every : 25);
    bool probs_dirty = true;
    for (;;) {
        // work lists of the running problems: operator items grouped by (degree, precision)
        std::vector<int> running;
        for (int i = 0; i < nprob; ++i)
            if (!finished[i]) running.push_back(i);
        if (running.empty()) break;
        if (probs_dirty) {
            HB_HIP(hipMemcpyAsync(B.probs, B.h_probs, sizeof(BatchProb) * nprob, hipMemcpyHostToDevice, s));
            probs_dirty = false;
        }
        struct Class {
            int N;
            bool fp32;
            int off, count;
            const void *D;  // the class's derivative matrix (any of its meshes)
        };
        std::vector<Class> classes;
        int nit = 0;
        for (int N = 1; N <= kMaxN; ++N)
            for (int f = 0; f < 2; ++f) {
                const int off = nit;
                const void *D = nullptr;
                for (int i : running) {
                    const BatchProb &P = B.h_probs[i];
                    if (P.N != N || P.use32 != f) continue;
                    D = f ? static_cast<const void *>(P.D32) : static_cast<const void *>(P.D);
                    for (int t = 0; t < P.ax_tiles; ++t) B.h_items[nit++] = WorkItem{i, t};
                }
                if (nit > off) classes.push_back(Class{N, f != 0, off, nit - off, D});
            }
        const int vec_off = nit;
        for (int i : running)
            for (int c = 0; c < B.h_probs[i].vec_chunks; ++c) B.h_items[nit++] = WorkItem{i, c};
        const int nvec = nit - vec_off;
        const int np = static_cast<int>(running.size());
        for (int k = 0; k < np; ++k) B.h_plist[k] = running[k];
        HB_HIP(hipMemcpyAsync(B.items, B.h_items, sizeof(WorkItem) * nit, hipMemcpyHostToDevice, s));
        HB_HIP(hipMemcpyAsync(B.plist, B.h_plist, sizeof(int32_t) * np, hipMemcpyHostToDevice, s));
        for (int it = 0; it < chunk; ++it) {
            for (const Class &c : classes)
                if ((st = launch_batch_ax(c.N, c.D, c.fp32, B.items + c.off, c.count, B.probs, s))) return st;
            if ((st = launch_batch_alpha(B.plist, np, B.probs, s)) ||
                (st = launch_batch_residual(B.items + vec_off, nvec, B.probs, s)) ||
                (st = launch_batch_beta(B.plist, np, B.probs, s)) ||
                (st = launch_batch_update(B.items + vec_off, nvec, B.probs, s)))
                return st;
        }
        HB_HIP(hipMemcpyAsync(B.h_states, B.states, sizeof(CgState) * nprob, hipMemcpyDeviceToHost, s));
        HB_HIP(hipStreamSynchronize(s));
        std::vector<int> replaced;
        for (int i : running) {
            const CgState &hs = B.h_states[i];
            const bool stopped = hs.done || hs.pending || hs.iters >= opts->max_iter;
            if (!stopped) continue;
            if (!mixed) {
                finished[i] = 1;
                continue;
            }
            bool enq = false;
            if ((st = rp[i].replace(meshes[i], lambdas[i], dev_b[i], dev_x[i], B.states + i, hs, B.norms + i, s,
                                    &enq)))
                return st;
            if (enq) replaced.push_back(i);
            else finished[i] = 1;
        }
        if (!replaced.empty()) {
            HB_HIP(hipMemcpyAsync(B.h_norms, B.norms, sizeof(double) * nprob, hipMemcpyDeviceToHost, s));
            HB_HIP(hipStreamSynchronize(s));
            for (int i : replaced) {
                const bool was32 = rp[i].use32;
                if ((st = rp[i].decide(meshes[i], B.states + i, B.h_states[i].iters, B.h_norms[i], nullptr, s)))
                    return st;
                finished[i] = rp[i].finished;
                if (was32 != rp[i].use32) {
                    B.h_probs[i].use32 = rp[i].use32 ? 1 : 0;
                    probs_dirty = true;
                }
            }
        }
    }
    HB_HIP(hipMemcpyAsync(B.h_states, B.states, sizeof(CgState) * nprob, hipMemcpyDeviceToHost, s));
    for (int i = 0; i < nprob; ++i) {
        const int iters = B.h_states[i].iters;
        HB_HIP(hipMemcpyAsync(B.h_norms + i, meshes[i]->cg.rho + iters, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HB_HIP(hipStreamSynchronize(s));
    hb_status worst = HB_OK;
    for (int i = 0; i < nprob; ++i) {
        const CgState &hs = B.h_states[i];
        if (mixed) {
            rp[i].fill(&results[i], hs.iters);
        } else {
            results[i] = hb_cg_result{};
            results[i].iters = hs.iters;
            results[i].status = hs.status;
            results[i].res0 = std::sqrt(B.h_rho[i]);
            results[i].res = std::sqrt(B.h_norms[i]);
            results[i].bnorm = std::sqrt(hs.bb);
        }
        if (worst == HB_OK && results[i].status != HB_OK) worst = static_cast<hb_status>(results[i].status);
    }
    return worst;
}

hb_status hb_stream_probe(const double *dev_in, double *dev_out, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!dev_in || !dev_out))) return fail(HB_ERR_INVALID_ARG, "hb_stream_probe: bad arguments");
    return launch_stream_probe(dev_in, dev_out, n, static_cast<hipStream_t>(stream));
}

}  // extern "C"
