// Batched CG over independent problems of different sizes and degrees.
//
// All problems advance together: one iteration is one operator launch per
// (degree, precision) class over a work list of (problem, element tile), then
// one launch each for alpha, the residual, beta and the update over all
// problems.  Each problem keeps its own device state (CgState), so problems
// at different iterations, or already finished, share the same launches
// (finished ones return at once).  The host rebuilds the work lists only when
// the set of running problems changes.  This file holds the vector and scalar
// steps; the batched operator kernel is instantiated with the single-problem
// operator, per degree range (ax_impl.h, ax_n*.hip), and launched through the
// schedule table (ax.hip).
#include "ax_impl.h"
#include "cg_steps.h"
#include "common.h"
#include "reduce.h"

namespace hb {
namespace {

constexpr int kVecThreads = 256;

__global__ __launch_bounds__(kFinThreads) void batch_alpha_kernel(const int32_t *__restrict__ plist,
                                                                 const BatchProb *__restrict__ probs)
{
    const BatchProb &P = probs[plist[blockIdx.x]];
    alpha_step(P.part_ax, P.ax_tiles, P.st, P.rho);
}

__global__ __launch_bounds__(kFinThreads) void batch_beta_kernel(const int32_t *__restrict__ plist,
                                                                const BatchProb *__restrict__ probs)
{
    const BatchProb &P = probs[plist[blockIdx.x]];
    beta_step(P.part_vec, P.vec_chunks, P.st, P.rho, P.hist, P.inv != nullptr);
}

// r -= alpha Ap on one chunk; the chunk's partial of r.r (Jacobi: of r.z, z =
// inv r, and of r.r in the second half of the partials).
__global__ __launch_bounds__(kVecThreads) void batch_residual_kernel(const WorkItem *__restrict__ items,
                                                                    const BatchProb *__restrict__ probs)
{
    __shared__ double red[kVecThreads / 64];
    const WorkItem it = items[blockIdx.x];
    const int32_t prob = uniform(it.prob), chunk = uniform(it.idx);
    const BatchProb &P = probs[prob];
    const auto st = to_global(uniform(P.st));
    if (uniform(st->done)) return;
    const double alpha = uniform(st->alpha);
    const int64_t NG = uniform(P.NG);
    const int64_t lo = (int64_t)chunk * kBatchChunk;
    const int64_t hi = lo + kBatchChunk < NG ? lo + kBatchChunk : NG;
    const auto r = to_global(uniform(P.r));
    double rr = 0.0;
    if (uniform(P.inv)) {
        const auto inv = to_global(uniform(P.inv));
        double rz = 0.0;
        auto sweep = [&](auto Ap) {
            for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
                const double ri = __builtin_nontemporal_load(&r[i]) -
                                  alpha * static_cast<double>(__builtin_nontemporal_load(&Ap[i]));
                __builtin_nontemporal_store(ri, &r[i]);
                rr += ri * ri;
                rz += ri * (inv[i] * ri);
            }
        };
        if (uniform(P.use32))
            sweep(to_global(uniform(P.Ap32)));
        else
            sweep(to_global(uniform(P.Ap)));
        rr = block_sum(rr, red);
        rz = block_sum(rz, red);
        if (threadIdx.x == 0) {
            to_global(uniform(P.part_vec))[chunk] = rz;
            to_global(uniform(P.part_vec))[uniform(P.vec_chunks) + chunk] = rr;
        }
        return;
    }
    if (uniform(P.use32)) {
        const auto Ap = to_global(uniform(P.Ap32));
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const double ri = __builtin_nontemporal_load(&r[i]) -
                              alpha * static_cast<double>(__builtin_nontemporal_load(&Ap[i]));
            __builtin_nontemporal_store(ri, &r[i]);
            rr += ri * ri;
        }
    } else {
        const auto Ap = to_global(uniform(P.Ap));
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const double ri = __builtin_nontemporal_load(&r[i]) - alpha * __builtin_nontemporal_load(&Ap[i]);
            __builtin_nontemporal_store(ri, &r[i]);
            rr += ri * ri;
        }
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) to_global(uniform(P.part_vec))[chunk] = rr;
}

// x += alpha p; p = r + beta p (Jacobi: p = inv r + beta p); Ap = 0 on one chunk.
// x, r and Ap are accessed non-temporally here and in the residual step (as in
// the single-problem kernels); p keeps plain stores for the operator's gather.
__global__ __launch_bounds__(kVecThreads) void batch_update_kernel(const WorkItem *__restrict__ items,
                                                                  const BatchProb *__restrict__ probs)
{
    const WorkItem it = items[blockIdx.x];
    const int32_t prob = uniform(it.prob), chunk = uniform(it.idx);
    const BatchProb &P = probs[prob];
    const auto st = to_global(uniform(P.st));
    if (uniform(st->done)) return;
    const double alpha = uniform(st->alpha), beta = uniform(st->beta);
    const int64_t NG = uniform(P.NG);
    const int64_t lo = (int64_t)chunk * kBatchChunk;
    const int64_t hi = lo + kBatchChunk < NG ? lo + kBatchChunk : NG;
    const auto x = to_global(uniform(P.x));
    const auto p = to_global(uniform(P.p));
    const auto r = to_global(uniform(P.r));
    if (uniform(P.inv)) {
        const auto inv = to_global(uniform(P.inv));
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const double pi = p[i];
            __builtin_nontemporal_store(__builtin_nontemporal_load(&x[i]) + alpha * pi, &x[i]);
            p[i] = inv[i] * __builtin_nontemporal_load(&r[i]) + beta * pi;
        }
    } else {
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const double pi = p[i];
            __builtin_nontemporal_store(__builtin_nontemporal_load(&x[i]) + alpha * pi, &x[i]);
            p[i] = __builtin_nontemporal_load(&r[i]) + beta * pi;
        }
    }
    if (uniform(P.use32)) {
        const auto Ap = to_global(uniform(P.Ap32));
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) __builtin_nontemporal_store(0.0f, &Ap[i]);
    } else {
        const auto Ap = to_global(uniform(P.Ap));
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) __builtin_nontemporal_store(0.0, &Ap[i]);
    }
}

}  // namespace

hb_status launch_batch_alpha(const int32_t *plist, int np, const BatchProb *probs, hipStream_t s)
{
    if (np == 0) return HB_OK;
    batch_alpha_kernel<<<np, kFinThreads, 0, s>>>(plist, probs);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_batch_beta(const int32_t *plist, int np, const BatchProb *probs, hipStream_t s)
{
    if (np == 0) return HB_OK;
    batch_beta_kernel<<<np, kFinThreads, 0, s>>>(plist, probs);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_batch_residual(const WorkItem *items, int nitems, const BatchProb *probs, hipStream_t s)
{
    if (nitems == 0) return HB_OK;
    batch_residual_kernel<<<nitems, kVecThreads, 0, s>>>(items, probs);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_batch_update(const WorkItem *items, int nitems, const BatchProb *probs, hipStream_t s)
{
    if (nitems == 0) return HB_OK;
    batch_update_kernel<<<nitems, kVecThreads, 0, s>>>(items, probs);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

}  // namespace hb
