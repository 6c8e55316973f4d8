// The two single-block scalar steps of a CG iteration (Algorithm 1), shared
// by the one-problem kernels and the batched kernels (one block per problem).
#pragma once

#include <cmath>

#include "common.h"
#include "reduce.h"

namespace hb {

constexpr int kFinThreads = 1024;

// Fixed-order sum of partial[0..n) by one block (call from every thread).
// The partials were written by an earlier kernel on the stream.
__device__ inline double sum_partials(const double *partial, int n, double *scratch)
{
    // eight loads in flight per thread, added in index order (the same sums as a
    // plain strided loop, without waiting on each load; past the end a thread
    // adds zeros, which leaves its sum unchanged)
    double s = 0.0;
    const int step = blockDim.x;
    for (int i = threadIdx.x; i < n; i += 8 * step) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = i + k * step < n ? partial[i + k * step] : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
    return block_sum(s, scratch);
}

// Start of iteration j = it + 1: alpha = rho_j / p.Ap, or stop on breakdown
// (p.Ap <= 0 or not finite), or apply a stop decided by the previous beta.
__device__ inline void alpha_step(const double *__restrict__ partial, int nblk, CgState *st,
                                  const double *__restrict__ rho)
{
    __shared__ double red[kFinThreads / 64];
    if (st->done) return;
    if (st->pending) {
        if (threadIdx.x == 0) st->done = 1;
        return;
    }
    const double pAp = sum_partials(partial, nblk, red);
    if (threadIdx.x != 0) return;
    const int j = st->it + 1;
    st->it = j;
    st->pAp = pAp;
    if (!(pAp > 0.0) || !isfinite(pAp)) {
        st->done = 1;
        st->status = HB_ERR_BREAKDOWN;
    } else {
        st->alpha = rho[j] / pAp;
    }
}

// rho_{j+1} = r.r, beta, history, convergence / iteration-cap test.  With the
// Jacobi preconditioner (pc) the partials hold r.z and then r.r: rho and beta
// use r.z, the history and the stop test ||r||.
__device__ inline void beta_step(const double *__restrict__ partial, int nblk, CgState *st, double *__restrict__ rho,
                                 double *__restrict__ hist, bool pc = false)
{
    __shared__ double red[kFinThreads / 64];
    if (st->done) return;
    const double rho_new = sum_partials(partial, nblk, red);
    const double rr = pc ? sum_partials(partial + nblk, nblk, red) : rho_new;
    if (threadIdx.x != 0) return;
    const int j = st->it;
    st->beta = rho_new / rho[j];
    rho[j + 1] = rho_new;
    hist[j + 1] = sqrt(rr);
    st->iters = j + 1;
    // this iteration's update still runs; the next alpha turns pending into done
    if (!isfinite(rho_new) || !isfinite(rr)) {
        st->pending = 1;
        st->status = HB_ERR_BREAKDOWN;
    } else if (rho_new == 0.0 || sqrt(rr) <= st->stop_res) {
        st->pending = 1;
        st->status = HB_OK;
    } else if (j + 1 >= st->max_iter) {
        st->pending = 1;
        st->status = st->rtol >= 0.0 ? HB_ERR_NOT_CONVERGED : HB_OK;
    }
}

}  // namespace hb
