// The extern "C" entry points declared in include/hbmi.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

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
    for (double *p : {w.r, w.p, w.Ap, w.part_ax, w.part_vec, w.rho, w.hist})
        if (p) (void)hipFree(p);
    if (w.state) (void)hipFree(w.state);
    if (w.host_state) (void)hipHostFree(w.host_state);
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
    delete m;
}

// Size the CG workspace for this mesh and iteration cap.
hb_status ensure_cg(hb_mesh_s *m, int max_iter)
{
    CgWork &w = m->cg;
    const int need_ax = ax_blocks(m), need_vec = 2 * vec_blocks(m->NG);
    if (w.r && w.n == m->NG && w.hist_len >= max_iter + 1 && w.part_ax_len >= need_ax && w.part_vec_len >= need_vec)
        return HB_OK;
    const int hist_len = std::max(max_iter + 1, w.hist_len);
    if (w.r) free_cg(m);
    size_t tally = 0;
    hb_status st;
    if ((st = dev_alloc(&w.r, m->NG, &tally)) || (st = dev_alloc(&w.p, m->NG, &tally)) ||
        (st = dev_alloc(&w.Ap, m->NG, &tally)) || (st = dev_alloc(&w.part_ax, need_ax, &tally)) ||
        (st = dev_alloc(&w.part_vec, need_vec, &tally)) || (st = dev_alloc(&w.rho, hist_len, &tally)) ||
        (st = dev_alloc(&w.hist, hist_len, &tally)) || (st = dev_alloc(&w.state, 1, &tally))) {
        w.bytes = tally;
        m->device_bytes += tally;
        free_cg(m);
        return st;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&w.host_state), sizeof(CgState), hipHostMallocDefault) != hipSuccess) {
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
    if (d.reserved != 0) return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: reserved field must be 0");
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
    return launch_ax(m, lambda, dev_x, dev_y, nullptr, nullptr, 0, s);
}

hb_status hb_ax_add(hb_mesh m, double lambda, const double *dev_x, double *dev_y, void *stream)
{
    if (!m || !dev_x || !dev_y) return fail(HB_ERR_INVALID_ARG, "hb_ax_add: null argument");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(HB_ERR_INVALID_ARG, "hb_ax_add: lambda must be finite and > 0");
    if (dev_x == dev_y) return fail(HB_ERR_INVALID_ARG, "hb_ax_add: x and y must not alias");
    return launch_ax(m, lambda, dev_x, dev_y, nullptr, nullptr, 0, static_cast<hipStream_t>(stream));
}

hb_status hb_cg_solve(hb_mesh m, double lambda, const double *dev_b, double *dev_x, const hb_cg_opts *opts,
                      hb_cg_result *result, double *host_res_hist, void *stream)
{
    if (!m || !dev_b || !dev_x || !opts) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: null argument");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: lambda must be finite and > 0");
    if (opts->max_iter < 0) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: max_iter must be >= 0");
    if (!opts->fixed_iters && !(opts->rtol >= 0.0)) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: rtol must be >= 0");
    if (dev_b == dev_x) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve: b and x must not alias");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hb_status st = ensure_cg(m, opts->max_iter);
    if (st) return st;
    CgWork &w = m->cg;
    const int64_t n = m->NG;
    const double rtol = opts->fixed_iters ? -1.0 : opts->rtol;
    if ((st = launch_cg_setup_state(w.state, opts->max_iter, rtol, s))) return st;
    if (!opts->x0_zero) {
        if ((st = launch_zero(w.Ap, n, s)) || (st = launch_ax(m, lambda, dev_x, w.Ap, nullptr, nullptr, 0, s))) return st;
    }
    if ((st = launch_cg_init(n, dev_b, dev_x, w.r, w.p, w.Ap, opts->x0_zero, w, w.state, s))) return st;

    const int axg = ax_blocks(m);
    auto enqueue_iteration = [&](int j) -> hb_status {
        hb_status e;
        if ((e = launch_ax(m, lambda, w.p, w.Ap, w.part_ax, w.state, j, s))) return e;
        if ((e = launch_cg_alpha(w, axg, w.state, j, s))) return e;
        if ((e = launch_cg_residual(n, w.r, w.Ap, w, w.state, j, s))) return e;
        if ((e = launch_cg_beta(n, w, w.state, j, s))) return e;
        return launch_cg_update(n, dev_x, w.p, w.r, w.Ap, w.state, j, s);
    };
    auto read_state = [&]() -> hb_status {
        HB_HIP(hipMemcpyAsync(w.host_state, w.state, sizeof(CgState), hipMemcpyDeviceToHost, s));
        HB_HIP(hipStreamSynchronize(s));
        return HB_OK;
    };
    // Fixed mode enqueues every iteration at once; tolerance mode reads the
    // device state back every `chunk` iterations to stop launching.
    const int chunk = opts->fixed_iters ? std::max(opts->max_iter, 1)
                                        : (opts->check_every > 0 ? opts->check_every : 25);
    int enqueued = 0;
    if (!opts->fixed_iters && (st = read_state())) return st;
    while (enqueued < opts->max_iter && (opts->fixed_iters || w.host_state->done_at > enqueued)) {
        const int k = std::min(chunk, opts->max_iter - enqueued);
        for (int i = 0; i < k; ++i)
            if ((st = enqueue_iteration(enqueued + i))) return st;
        enqueued += k;
        if (!opts->fixed_iters && (st = read_state())) return st;
    }
    if ((st = read_state())) return st;
    const CgState hs = *w.host_state;
    double rho0 = 0.0, rho_last = 0.0;
    HB_HIP(hipMemcpy(&rho0, w.rho, sizeof(double), hipMemcpyDeviceToHost));
    HB_HIP(hipMemcpy(&rho_last, w.rho + hs.iters, sizeof(double), hipMemcpyDeviceToHost));
    if (host_res_hist) HB_HIP(hipMemcpy(host_res_hist, w.hist, sizeof(double) * (hs.iters + 1), hipMemcpyDeviceToHost));
    if (result) {
        result->iters = hs.iters;
        result->status = hs.status;
        result->res0 = std::sqrt(rho0);
        result->res = std::sqrt(rho_last);
        result->bnorm = std::sqrt(hs.bb);
    }
    return static_cast<hb_status>(hs.status);
}

hb_status hb_stream_probe(const double *dev_in, double *dev_out, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!dev_in || !dev_out))) return fail(HB_ERR_INVALID_ARG, "hb_stream_probe: bad arguments");
    return launch_stream_probe(dev_in, dev_out, n, static_cast<hipStream_t>(stream));
}

}  // extern "C"
