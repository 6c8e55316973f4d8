// Batched CG in one persistent launch (Algorithm 1 for many independent
// problems; the latency model of the DOF Storage section, t = alpha + beta B,
// is why small problems want no per-step launches).
//
// The launch holds every running problem at once: problem p owns nwg_p
// workgroups, and those run its iterations back to back, each iteration three
// phases separated by a barrier among the problem's workgroups only:
//   operator  Ap += A p over the problem's tiles (Ap is zero), partial of p.Ap
//   residual  alpha = rho_j / p.Ap from all partials (every workgroup sums
//             them in the same fixed order, so all hold the same alpha),
//             r -= alpha Ap over the workgroup's slice, partial of r.r (r.z)
//   update    beta = rho_{j+1} / rho_j likewise, x += alpha p,
//             p = r (or M^-1 r) + beta p, Ap = 0 over the slice.
// So no problem waits for another, and the host sees the device only between
// launches.  The stop tests, the history and the device state follow the
// single-block alpha and beta steps of the per-step runner exactly (cg_steps.h),
// so the host's handling of finished problems and of residual replacement is
// the same for both.
//
// Deadlock freedom: the launch is cooperative (the runtime guarantees that all
// its workgroups are resident at once, or refuses it), and a workgroup only
// waits for workgroups of its own problem.  Every wait is bounded: a barrier
// that spins past its limit raises *err and the launch ends.
//
// The kernel inlines the operator of each degree it is compiled for (one tile
// routine per degree and precision), so it runs at the occupancy of the most
// demanding of them (one wave per SIMD: a workgroup per compute unit); tiles use
// the 256-thread shape with D^T read from LDS.  That suits the regime it is for,
// many small problems whose iterations are bound by the latency of dependent
// steps rather than by bandwidth; the host keeps large problems on the
// per-step launches.
#include <cmath>
#include <mutex>

#include "ax_impl.h"
#include "cg_steps.h"
#include "common.h"
#include "reduce.h"

namespace hb {
namespace {

// tile schedule of every degree in the launch: 256-thread tiles, D^T in LDS
template <int N>
constexpr int kPV = kSchedColsLds;
constexpr uint32_t kSpinLimit = 1u << 22;  // polls of a barrier counter before giving up (~0.3 s)

// Arrive at barrier number `target / nwg` of one problem and wait for its other
// workgroups: the workgroup's writes are released (agent scope) before the
// arrival is counted, and acquired after the count is complete.  Returns false
// (every thread) if the wait timed out or another workgroup reported an error.
__device__ bool group_barrier(uint32_t *ctr, uint32_t target, int32_t *err, int *s_ok)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __threadfence();
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Ap += A p over tiles rank, rank + nwg, ... of the problem's walk; the
// workgroup's sum of the tiles' p_e . (A p)_e.  The arrays come in as
// non-aliasing parameters: read from the problem table, the compiler would
// otherwise have to assume that the operator's output may alias its inputs
// across the tiles of the loop (which costs it the register budget of two
// waves per SIMD).
template <int N, typename T, bool MASK>
__device__ __attribute__((always_inline)) inline double operator_tiles(
    int64_t E, const TileWalk &walk, int tiles, int rank, int nwg, gptr<const int32_t> __restrict__ map,
    gptr<const T> __restrict__ geo, gptr<const T> __restrict__ D, T lam, gptr<const double> __restrict__ x,
    gptr<T> __restrict__ y)
{
    double dot = 0.0;
    for (int i = rank; i < tiles; i += nwg)
        dot += ax_tile<N, true, T, kPV<N>, MASK>(
            tile_span(walk, walk_tile(walk, static_cast<uint32_t>(i)), E, AxShape<N, kPV<N>>::epb), map, geo, D, lam,
            x, y, nullptr);
    return dot;
}

template <int N, typename T, bool MASK>
__device__ __attribute__((always_inline)) inline double operator_share(const BatchProb &P, const TileWalk &walk,
                                                                       int tiles, int rank, int nwg)
{
    const int64_t E = uniform(P.E);
    const auto map = to_global(uniform(P.map));
    const auto x = to_global(uniform(P.p));
    if constexpr (sizeof(T) == 4)
        return operator_tiles<N, float, MASK>(E, walk, tiles, rank, nwg, map, to_global(uniform(P.geo32)),
                                              to_global(uniform(P.D32)), static_cast<float>(uniform(P.lambda)), x,
                                              to_global(uniform(P.Ap32)));
    else
        return operator_tiles<N, double, MASK>(E, walk, tiles, rank, nwg, map, to_global(uniform(P.geo)),
                                               to_global(uniform(P.D)), uniform(P.lambda), x,
                                               to_global(uniform(P.Ap)));
}

template <bool MASK>
__device__ double operator_any(const BatchProb &P, int N, bool fp32, const TileWalk &walk, int tiles, int rank,
                               int nwg)
{
    switch (N) {
#define HB_PCASE(n)                                                                    \
    case n:                                                                            \
        return fp32 ? operator_share<n, float, MASK>(P, walk, tiles, rank, nwg)        \
                    : operator_share<n, double, MASK>(P, walk, tiles, rank, nwg);
        HB_PCASE(3)
        HB_PCASE(5)
        HB_PCASE(7)
        HB_PCASE(9)
#undef HB_PCASE
    default: return 0.0;  // not reached: the host launches listed degrees only
    }
}

template <bool MASK>
__global__ __launch_bounds__(kPersistThreads) void persist_kernel(const PersistWg *__restrict__ wgs,
                                                                 const PersistSlot *__restrict__ slots,
                                                                 const BatchProb *__restrict__ probs,
                                                                 uint32_t *__restrict__ bar, int32_t *__restrict__ err)
{
    __shared__ double red[kPersistThreads / 64];
    __shared__ int s_ok;
    const int t = threadIdx.x;
    const int32_t prob = uniform(wgs[blockIdx.x].prob), rank = uniform(wgs[blockIdx.x].rank);
    const PersistSlot &sl = slots[prob];
    const int32_t nwg = uniform(sl.nwg), budget = uniform(sl.iters), tiles = uniform(sl.tiles);
    const TileWalk walk{static_cast<uint32_t>(uniform(static_cast<int32_t>(sl.walk.txn))),
                        static_cast<uint32_t>(uniform(static_cast<int32_t>(sl.walk.ny))),
                        static_cast<uint32_t>(uniform(static_cast<int32_t>(sl.walk.nz))),
                        static_cast<uint32_t>(uniform(static_cast<int32_t>(sl.walk.ys)))};
    const BatchProb &P = probs[prob];
    CgState *st = uniform(P.st);
    const int N = uniform(P.N);
    const bool fp32 = uniform(P.use32) != 0;
    const int64_t n = uniform(P.NG);
    double *rho = uniform(P.rho), *hist = uniform(P.hist);
    double *part_ax = uniform(P.part_ax), *part_vec = uniform(P.part_vec);
    const auto x = to_global(uniform(P.x)), r = to_global(uniform(P.r)), p = to_global(uniform(P.p));
    const auto Ap = to_global(uniform(P.Ap));
    const auto Ap32 = to_global(uniform(P.Ap32));
    const auto inv = to_global(uniform(P.inv));
    uint32_t *ctr = bar + prob;
    uint32_t passed = 0;

    // the starting state, read by every workgroup before any of them changes it
    int32_t it = uniform(st->it), iters = uniform(st->iters), done = uniform(st->done);
    int32_t pending = uniform(st->pending), status = uniform(st->status);
    const int32_t max_iter = uniform(st->max_iter);
    const double stop_res = uniform(st->stop_res), rtol = uniform(st->rtol);
    double alpha = uniform(st->alpha), beta = uniform(st->beta), pAp = uniform(st->pAp);
    double rho_j = (done | pending) ? 0.0 : uniform(rho[it + 1]);
    if (!group_barrier(ctr, ++passed * nwg, err, &s_ok)) return;

    const int64_t first = static_cast<int64_t>(rank) * kPersistThreads + t;
    const int64_t stride = static_cast<int64_t>(nwg) * kPersistThreads;
    for (int k = 0; k < budget; ++k) {
        // alpha step: a stop decided by the last beta step takes effect here
        if (done) break;
        if (pending) {
            done = 1;
            break;
        }
        const double d = MASK ? operator_any<true>(P, N, fp32, walk, tiles, rank, nwg)
                              : operator_any<false>(P, N, fp32, walk, tiles, rank, nwg);
        if (t == 0) part_ax[rank] = d;
        if (!group_barrier(ctr, ++passed * nwg, err, &s_ok)) return;
        pAp = uniform(sum_partials(part_ax, nwg, red));
        const int j = it + 1;
        it = j;
        if (!(pAp > 0.0) || !isfinite(pAp)) {
            done = 1;
            status = HB_ERR_BREAKDOWN;
            break;
        }
        alpha = uniform(rho_j / pAp);

        // residual step
        double rr = 0.0, rz = 0.0;
        for (int64_t i = first; i < n; i += stride) {
            const double api = fp32 ? static_cast<double>(Ap32[i]) : Ap[i];
            const double ri = r[i] - alpha * api;
            r[i] = ri;
            rr += ri * ri;
            if (inv) rz += ri * (inv[i] * ri);
        }
        rr = block_sum(rr, red);
        if (inv) rz = block_sum(rz, red);
        if (t == 0) {
            part_vec[rank] = inv ? rz : rr;
            if (inv) part_vec[nwg + rank] = rr;
        }
        if (!group_barrier(ctr, ++passed * nwg, err, &s_ok)) return;
        const double rho_new = uniform(sum_partials(part_vec, nwg, red));
        const double rrs = inv ? uniform(sum_partials(part_vec + nwg, nwg, red)) : rho_new;

        // beta step (as beta_step): history, stop tests; the update below still runs
        beta = uniform(rho_new / rho_j);
        if (rank == 0 && t == 0) {
            rho[j + 1] = rho_new;
            hist[j + 1] = sqrt(rrs);
        }
        iters = j + 1;
        if (!isfinite(rho_new) || !isfinite(rrs)) {
            pending = 1;
            status = HB_ERR_BREAKDOWN;
        } else if (rho_new == 0.0 || sqrt(rrs) <= stop_res) {
            pending = 1;
            status = HB_OK;
        } else if (j + 1 >= max_iter) {
            pending = 1;
            status = rtol >= 0.0 ? HB_ERR_NOT_CONVERGED : HB_OK;
        }
        rho_j = rho_new;

        // update step
        for (int64_t i = first; i < n; i += stride) {
            const double pi = p[i];
            x[i] += alpha * pi;
            p[i] = (inv ? inv[i] * r[i] : r[i]) + beta * pi;
            if (fp32)
                Ap32[i] = 0.0f;
            else
                Ap[i] = 0.0;
        }
        if (!group_barrier(ctr, ++passed * nwg, err, &s_ok)) return;
    }
    if (rank == 0 && t == 0) {
        st->it = it;
        st->iters = iters;
        st->alpha = alpha;
        st->beta = beta;
        st->pAp = pAp;
        st->done = done;
        st->pending = pending;
        st->status = status;
    }
}

std::once_flag g_cap_once;
int g_cap = 0;

}  // namespace

bool persist_degree(int N) { return N == 3 || N == 5 || N == 7 || N == 9; }

int persist_capacity()
{
    std::call_once(g_cap_once, [] {
        int dev = 0, cus = 0, coop = 0, per_cu = 0, per_cu_d = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_kernel<false>, kPersistThreads, 0) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_d, persist_kernel<true>, kPersistThreads, 0) !=
                hipSuccess) {
            (void)hipGetLastError();
            g_cap = 0;
            return;
        }
        g_cap = cus * std::min(per_cu, per_cu_d);
    });
    return g_cap;
}

int persist_tiles(int N, int64_t E)
{
    switch (N) {
    case 3: return ax_grid<3, kPV<3>>(E);
    case 5: return ax_grid<5, kPV<5>>(E);
    case 7: return ax_grid<7, kPV<7>>(E);
    case 9: return ax_grid<9, kPV<9>>(E);
    default: return 0;
    }
}

TileWalk persist_walk(int N, int64_t nx, int64_t ny, int64_t nz)
{
    switch (N) {
    case 3: return make_walk(nx, ny, nz, AxShape<3, kPV<3>>::epb);
    case 5: return make_walk(nx, ny, nz, AxShape<5, kPV<5>>::epb);
    case 7: return make_walk(nx, ny, nz, AxShape<7, kPV<7>>::epb);
    case 9: return make_walk(nx, ny, nz, AxShape<9, kPV<9>>::epb);
    default: return TileWalk{};
    }
}

hb_status launch_batch_persistent(bool dirichlet, const PersistWg *wgs, int nwg, const PersistSlot *slots,
                                  const BatchProb *probs, uint32_t *bar, int32_t *err, hipStream_t s)
{
    static_assert(AxShape<3, kPV<3>>::threads == kPersistThreads && AxShape<5, kPV<5>>::threads == kPersistThreads &&
                      AxShape<7, kPV<7>>::threads == kPersistThreads && AxShape<9, kPV<9>>::threads == kPersistThreads,
                  "every degree of the persistent kernel tiles with its workgroup size");
    if (nwg == 0) return HB_OK;
    if (nwg > persist_capacity())
        return fail(HB_ERR_INVALID_ARG, "persistent batch: more workgroups than the device holds at once");
    void *args[] = {&wgs, &slots, &probs, &bar, &err};
    const void *fn = dirichlet ? reinterpret_cast<const void *>(&persist_kernel<true>)
                               : reinterpret_cast<const void *>(&persist_kernel<false>);
    HB_HIP(hipLaunchCooperativeKernel(fn, dim3(nwg), dim3(kPersistThreads), args, 0, s));
    return HB_OK;
}

}  // namespace hb
