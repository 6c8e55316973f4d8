// hb_cg_solve_noalloc: FP64 CG (Algorithm 1, optionally Jacobi-preconditioned)
// whose whole workspace lives in one file-scope device array, for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc).  The kernels are the ones
// hb_cg_solve launches; only where their workspace lives differs.
//
// The array is a static __device__ object: every GPU the library runs on holds
// its own copy until the process ends.  In host code its name is a host-side
// stand-in, not a device address, so the address of this device's copy is
// looked up once per device with hipGetSymbolAddress and only that address is
// ever handed to kernels or copies.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "common.h"
#include "solver.h"

namespace hb {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on first use).
hb_status scratch_ptr(unsigned char **out)
{
    int dev = 0;
    HB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HB_ERR_DEVICE, "hb_cg_solve_noalloc: device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return e != hipSuccess ? hip_fail(e, "hipGetSymbolAddress(scratch)")
                                   : fail(HB_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned no address");
        }
        g_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_ptr[dev]);
    return HB_OK;
}

// Carves aligned pieces off the front of a byte range (or, with base ==
// nullptr, only counts the bytes the pieces need).
struct Carver {
    unsigned char *base;
    size_t used = 0;
    template <typename T>
    T *take(size_t count)
    {
        used = (used + kAlign - 1) / kAlign * kAlign;
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += sizeof(T) * count;
        return p;
    }
};

// The workspace of one solve, laid out in `base` (nullptr: size only).
size_t layout(const hb_mesh_s *m, int max_iter, bool pc, unsigned char *base, CgWork *w)
{
    Carver c{base};
    const size_t ng = static_cast<size_t>(m->NG);
    w->state = c.take<CgState>(1);
    w->dnorm = c.take<double>(1);
    w->part_ax = c.take<double>(static_cast<size_t>(std::max(ax_blocks_max(m), 1)));
    w->part_vec = c.take<double>(static_cast<size_t>(3 * vec_blocks(m->NG)));
    w->rho = c.take<double>(static_cast<size_t>(max_iter) + 1);
    w->hist = c.take<double>(static_cast<size_t>(max_iter) + 1);
    w->r = c.take<double>(ng);
    w->p = c.take<double>(ng);
    w->Ap = c.take<double>(ng);
    w->jinv = pc ? c.take<double>(ng) : nullptr;
    return c.used;
}

hb_status read_state_sync(const CgWork &w, CgState *out, hipStream_t s)
{
    HB_HIP(hipMemcpyAsync(out, w.state, sizeof(CgState), hipMemcpyDeviceToHost, s));
    HB_HIP(hipStreamSynchronize(s));
    return HB_OK;
}

}  // namespace
}  // namespace hb

using namespace hb;

extern "C" hb_status hb_cg_solve_noalloc(hb_mesh m, double lambda, const double *dev_b, double *dev_x,
                                         const hb_cg_opts *opts, hb_cg_result *result, double *host_res_hist,
                                         void *stream)
{
    if (!m || !dev_b || !dev_x || !opts) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve_noalloc: null argument");
    if (!(lambda > 0.0) || !std::isfinite(lambda))
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve_noalloc: lambda must be finite and > 0");
    if (opts->max_iter < 0) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve_noalloc: max_iter must be >= 0");
    if (!opts->fixed_iters && !(opts->rtol >= 0.0))
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve_noalloc: rtol must be >= 0");
    if (dev_b == dev_x) return fail(HB_ERR_INVALID_ARG, "hb_cg_solve_noalloc: b and x must not alias");
    if (opts->prec != HB_PREC_FP64)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve_noalloc: only HB_PREC_FP64 runs without allocation");
    if (opts->graph_k != 0)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve_noalloc: graph_k must be 0 (a graph is an allocation)");
    if (opts->precond != HB_PRECOND_NONE && opts->precond != HB_PRECOND_JACOBI)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve_noalloc: unknown preconditioner");
    const bool pc = opts->precond == HB_PRECOND_JACOBI;
    CgWork w;
    const size_t need = layout(m, opts->max_iter, pc, nullptr, &w);
    if (need > kScratchBytes)
        return fail(HB_ERR_INVALID_ARG, "hb_cg_solve_noalloc: the solve needs " + std::to_string(need) +
                                            " bytes of workspace, more than the " + std::to_string(kScratchBytes) +
                                            "-byte no-allocation buffer (N_G <= ~2.7M DOFs at 100 iterations)");
    unsigned char *base = nullptr;
    hb_status st = scratch_ptr(&base);
    if (st) return st;
    layout(m, opts->max_iter, pc, base, &w);
    w.n = m->NG;
    w.pc = pc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = m->NG;
    const int max_iter = opts->max_iter;
    const double rtol = opts->fixed_iters ? -1.0 : opts->rtol;
    if (pc && (st = launch_jacobi_inverse(m, lambda, w.jinv, s))) return st;
    // r0 = b - A x0, p = r0 (z0 with the preconditioner); every value the
    // iterations read is written first by these kernels, whatever the buffer held
    if ((st = launch_cg_setup_state(w.state, max_iter, rtol, s))) return st;
    if (!opts->x0_zero) {
        if ((st = launch_zero(w.Ap, n, s)) || (st = launch_ax(m, lambda, dev_x, w.Ap, nullptr, nullptr, s))) return st;
    }
    if ((st = launch_cg_init<double>(n, dev_b, dev_x, w.r, w.p, w.Ap, opts->x0_zero, w, w.state, s))) return st;
    CgState hs{};
    if ((st = read_state_sync(w, &hs, s))) return st;
    const int chunk = rtol < 0.0 ? std::max(max_iter, 1) : (opts->check_every > 0 ? opts->check_every : 25);
    while (hs.iters < max_iter && !hs.done && !hs.pending) {
        const int k = std::min(chunk, max_iter - hs.iters);
        for (int i = 0; i < k; ++i)
            if ((st = enqueue_iteration<double>(m, w, lambda, dev_x, w.Ap, s))) return st;
        if ((st = read_state_sync(w, &hs, s))) return st;
    }
    double res0 = 0.0, res_last = 0.0;
    HB_HIP(hipMemcpyAsync(&res0, w.hist, sizeof(double), hipMemcpyDeviceToHost, s));
    HB_HIP(hipMemcpyAsync(&res_last, w.hist + hs.iters, sizeof(double), hipMemcpyDeviceToHost, s));
    if (host_res_hist)
        HB_HIP(hipMemcpyAsync(host_res_hist, w.hist, sizeof(double) * (hs.iters + 1), hipMemcpyDeviceToHost, s));
    HB_HIP(hipStreamSynchronize(s));
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
