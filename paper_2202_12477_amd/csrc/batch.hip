// Batched CG over independent problems of different sizes and degrees.
//
// All problems advance together: one iteration is one operator launch per
// (degree, precision) class over a work list of (problem, element tile), then
// one launch each for alpha, the residual, beta and the update over all
// problems.  Each problem keeps its own device state (CgState), so problems
// at different iterations, or already finished, share the same launches
// (finished ones return at once).  The host rebuilds the work lists only when
// the set of running problems changes.
#include "ax_impl.h"
#include "cg_steps.h"
#include "common.h"
#include "reduce.h"

namespace hb {
namespace {

constexpr int kVecThreads = 256;

// Values read from the work list and the problem table are the same for the
// whole block; saying so lets the compiler keep them (and everything derived
// from them, such as the uniform entries of D) in scalar registers.
__device__ inline int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uniform(int64_t v)
{
    const uint64_t u = static_cast<uint64_t>(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}
template <typename T>
__device__ inline T *uniform(T *p)
{
    return reinterpret_cast<T *>(uniform(reinterpret_cast<int64_t>(p)));
}
__device__ inline double uniform(double v)
{
    return __builtin_bit_cast(double, uniform(__builtin_bit_cast(int64_t, v)));
}

// D depends only on the degree, so all problems of a class share it; as a
// read-only kernel argument its block-uniform entries come through scalar loads.
template <int N, typename T>
__global__ __launch_bounds__(AxShape<N>::threads) void batch_ax_kernel(const WorkItem *__restrict__ items,
                                                                      const BatchProb *__restrict__ probs,
                                                                      const T *__restrict__ Dm)
{
    const WorkItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    const int32_t prob = uniform(it.prob), tile = uniform(it.idx);
    const BatchProb &P = probs[prob];
    // a stopped problem, or one whose stop the next alpha step will apply, needs no operator
    const auto st = to_global(uniform(P.st));
    if (uniform(st->done) | uniform(st->pending)) return;
    const int64_t E = uniform(P.E);
    const auto map = to_global(uniform(P.map));
    const auto x = to_global(uniform(P.p));
    const auto part = to_global(uniform(P.part_ax) + tile);
    if constexpr (sizeof(T) == 4)
        ax_tile<N, true, float>(E, tile, map, to_global(uniform(P.geo32)), to_global(Dm),
                                static_cast<float>(uniform(P.lambda)), x, to_global(uniform(P.Ap32)), part);
    else
        ax_tile<N, true, double>(E, tile, map, to_global(uniform(P.geo)), to_global(Dm), uniform(P.lambda), x,
                                 to_global(uniform(P.Ap)), part);
}

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
    beta_step(P.part_vec, P.vec_chunks, P.st, P.rho, P.hist);
}

// r -= alpha Ap on one chunk; the chunk's partial of r.r.
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
    if (uniform(P.use32)) {
        const auto Ap = to_global(uniform(P.Ap32));
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const double ri = r[i] - alpha * static_cast<double>(Ap[i]);
            r[i] = ri;
            rr += ri * ri;
        }
    } else {
        const auto Ap = to_global(uniform(P.Ap));
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const double ri = r[i] - alpha * Ap[i];
            r[i] = ri;
            rr += ri * ri;
        }
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) to_global(uniform(P.part_vec))[chunk] = rr;
}

// x += alpha p; p = r + beta p; Ap = 0 on one chunk.
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
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double pi = p[i];
        x[i] += alpha * pi;
        p[i] = r[i] + beta * pi;
    }
    if (uniform(P.use32)) {
        const auto Ap = to_global(uniform(P.Ap32));
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) Ap[i] = 0.0f;
    } else {
        const auto Ap = to_global(uniform(P.Ap));
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) Ap[i] = 0.0;
    }
}

template <int N>
hb_status batch_ax_n(const void *D, bool fp32, const WorkItem *items, int nitems, const BatchProb *probs,
                     hipStream_t s)
{
    if (fp32)
        batch_ax_kernel<N, float><<<nitems, AxShape<N>::threads, 0, s>>>(items, probs, static_cast<const float *>(D));
    else
        batch_ax_kernel<N, double><<<nitems, AxShape<N>::threads, 0, s>>>(items, probs, static_cast<const double *>(D));
    HB_HIP(hipGetLastError());
    return HB_OK;
}

}  // namespace

int batch_ax_threads(int N)
{
    switch (N) {
#define HB_CASE(n) \
    case n: return AxShape<n>::threads;
        HB_CASE(1) HB_CASE(2) HB_CASE(3) HB_CASE(4) HB_CASE(5) HB_CASE(6) HB_CASE(7) HB_CASE(8)
        HB_CASE(9) HB_CASE(10) HB_CASE(11) HB_CASE(12) HB_CASE(13) HB_CASE(14) HB_CASE(15)
#undef HB_CASE
    default: return 0;
    }
}

hb_status launch_batch_ax(int N, const void *D, bool fp32, const WorkItem *items, int nitems, const BatchProb *probs,
                          hipStream_t s)
{
    if (nitems == 0) return HB_OK;
    switch (N) {
#define HB_CASE(n) \
    case n: return batch_ax_n<n>(D, fp32, items, nitems, probs, s);
        HB_CASE(1) HB_CASE(2) HB_CASE(3) HB_CASE(4) HB_CASE(5) HB_CASE(6) HB_CASE(7) HB_CASE(8)
        HB_CASE(9) HB_CASE(10) HB_CASE(11) HB_CASE(12) HB_CASE(13) HB_CASE(14) HB_CASE(15)
#undef HB_CASE
    default: return fail(HB_ERR_INVALID_ARG, "unsupported degree N");
    }
}

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
