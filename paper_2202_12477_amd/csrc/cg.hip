// Kernels of the conjugate-gradient iteration (Algorithm 1; fused as in the
// Conjugate gradient Iteration section, with every scalar kept on the device so
// the host never waits inside an iteration).
//
// An iteration is five launches on one stream, identical for every iteration
// (the iteration number lives in the device state):
//   operator  Ap = A p, block partials of p.Ap              (ax*.hip)
//   alpha     one block: j = it + 1, p.Ap from the partials, alpha = rho_j / p.Ap
//   residual  r -= alpha Ap, block partials of r.r
//   beta      one block: rho_{j+1} = r.r, beta = rho_{j+1} / rho_j, history, stop test
//   update    x += alpha p; p = r + beta p; Ap = 0 for the next assembly
// Streaming kernels never wait for each other's blocks and issue no
// device-scope fences: the single-block kernels finish the reductions in a
// fixed order after the kernel boundary has made the partials visible.
#include <climits>
#include <cmath>

#include "cg_steps.h"
#include "common.h"
#include "reduce.h"

namespace hb {
namespace {

constexpr int kVecThreads = 256;


template <typename V>
__global__ __launch_bounds__(kVecThreads) void zero_kernel(V *__restrict__ v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = V(0);
}

__global__ void setup_state_kernel(CgState *st, int max_iter, double rtol)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->bb = st->alpha = st->beta = st->pAp = 0.0;
    st->rtol = rtol;
    st->stop_res = -1.0;
    st->max_iter = max_iter;
    st->it = -1;
    st->iters = 0;
    st->done = 0;
    st->pending = 0;
    st->status = HB_OK;
}

// r0 = b - A x0 (Ap holds A x0 unless x0 = 0), p = r0, Ap = 0; partials of r0.r0 and b.b.
// PC (Jacobi): p = z0 = inv r0, and a third partial array of r0.z0.
template <typename TAp, bool PC>
__global__ __launch_bounds__(kVecThreads) void init_kernel(int64_t n, const double *__restrict__ b,
                                                          double *__restrict__ x, double *__restrict__ r,
                                                          double *__restrict__ p, TAp *__restrict__ Ap,
                                                          int x0_zero, const double *__restrict__ inv,
                                                          double *__restrict__ partial)
{
    __shared__ double red[kVecThreads / 64];
    double rr = 0.0, bb = 0.0, rz = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double bi = b[i];
        const double ri = x0_zero ? bi : bi - static_cast<double>(Ap[i]);
        r[i] = ri;
        if constexpr (PC) {
            const double zi = inv[i] * ri;
            p[i] = zi;
            rz += ri * zi;
        } else {
            p[i] = ri;
        }
        Ap[i] = TAp(0);
        if (x0_zero) x[i] = 0.0;
        rr += ri * ri;
        bb += bi * bi;
    }
    rr = block_sum(rr, red);
    bb = block_sum(bb, red);
    if constexpr (PC) rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = rr;
        partial[gridDim.x + blockIdx.x] = bb;
        if constexpr (PC) partial[2 * gridDim.x + blockIdx.x] = rz;
    }
}

__global__ __launch_bounds__(kFinThreads) void init_finish_kernel(const double *__restrict__ partial, int nblk,
                                                                 int pc, CgState *st, double *__restrict__ rho,
                                                                 double *__restrict__ hist)
{
    __shared__ double red[kFinThreads / 64];
    const double rho0 = sum_partials(partial, nblk, red);  // r0.r0: the stop tests
    const double bb = sum_partials(partial + nblk, nblk, red);
    const double rz0 = pc ? sum_partials(partial + 2 * nblk, nblk, red) : rho0;
    if (threadIdx.x != 0) return;
    st->bb = bb;
    rho[0] = rz0;
    hist[0] = sqrt(rho0);
    st->stop_res = st->rtol >= 0.0 ? st->rtol * sqrt(bb) : -1.0;
    if (!isfinite(rho0)) {
        st->done = 1;
        st->status = HB_ERR_NONFINITE;
    } else if (rho0 == 0.0 || sqrt(rho0) <= st->stop_res) {
        st->done = 1;  // already solved
    } else if (st->max_iter == 0) {
        st->done = 1;
        st->status = st->rtol >= 0.0 ? HB_ERR_NOT_CONVERGED : HB_OK;
    }
}

__global__ __launch_bounds__(kFinThreads) void alpha_kernel(const double *__restrict__ partial, int nblk, CgState *st,
                                                           const double *__restrict__ rho)
{
    alpha_step(partial, nblk, st, rho);
}

// r -= alpha Ap; partials of r.r (PC: of r.z, z = inv r, then of r.r).
template <typename TAp, bool PC>
__global__ __launch_bounds__(kVecThreads) void residual_kernel(int64_t n, double *__restrict__ r,
                                                              const TAp *__restrict__ Ap,
                                                              const double *__restrict__ inv,
                                                              double *__restrict__ partial, const CgState *st)
{
    if (st->done) return;
    __shared__ double red[kVecThreads / 64];
    const double alpha = st->alpha;
    double rr = 0.0, rz = 0.0;
    // non-temporal: r and Ap are streamed once here; the operator reads p next,
    // and the geometry it streams would evict these lines before their next use
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ri = __builtin_nontemporal_load(&r[i]) -
                          alpha * static_cast<double>(__builtin_nontemporal_load(&Ap[i]));
        __builtin_nontemporal_store(ri, &r[i]);
        rr += ri * ri;
        if constexpr (PC) rz += ri * (inv[i] * ri);
    }
    rr = block_sum(rr, red);
    if constexpr (PC) {
        rz = block_sum(rz, red);
        if (threadIdx.x == 0) {
            partial[blockIdx.x] = rz;
            partial[gridDim.x + blockIdx.x] = rr;
        }
    } else {
        if (threadIdx.x == 0) partial[blockIdx.x] = rr;
    }
}

__global__ __launch_bounds__(kFinThreads) void beta_kernel(const double *__restrict__ partial, int nblk, int pc,
                                                          CgState *st, double *__restrict__ rho,
                                                          double *__restrict__ hist)
{
    beta_step(partial, nblk, st, rho, hist, pc != 0);
}

// x += alpha p; p = r + beta p (PC: p = inv r + beta p); Ap = 0 (the next
// operator call assembles into it).
template <typename TAp, bool PC, bool AP_CACHED>
__global__ __launch_bounds__(kVecThreads) void update_kernel(int64_t n, double *__restrict__ x, double *__restrict__ p,
                                                            const double *__restrict__ r, TAp *__restrict__ Ap,
                                                            const double *__restrict__ inv, const CgState *st)
{
    if (st->done) return;
    const double alpha = st->alpha, beta = st->beta;
    // x and r non-temporal (not read again before the next update or residual
    // step); p with plain stores, which the operator gathers next.  Ap with
    // plain stores where it fits the last-level cache with room to spare
    // (AP_CACHED), so the operator's memory-side atomic adds find its lines
    // there; non-temporal otherwise.
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double pi = p[i];
        __builtin_nontemporal_store(__builtin_nontemporal_load(&x[i]) + alpha * pi, &x[i]);
        const double ri = __builtin_nontemporal_load(&r[i]);
        if constexpr (PC)
            p[i] = inv[i] * ri + beta * pi;
        else
            p[i] = ri + beta * pi;
        if constexpr (AP_CACHED)
            Ap[i] = TAp(0);
        else
            __builtin_nontemporal_store(TAp(0), &Ap[i]);
    }
}

// The four steps after the operator -- alpha, r -= alpha Ap with r.r, beta,
// x += alpha p; p = r + beta p (PC: p = inv r + beta p); Ap = 0 -- in one
// workgroup, for vectors so short that one workgroup streams them in less time
// than four dependent launches take.  The same steps and state transitions as
// alpha_kernel, residual_kernel, beta_kernel and update_kernel; r.r is summed
// over the one workgroup (one partial), so only the grouping of its additions
// differs.
template <typename TAp, bool PC>
__global__ __launch_bounds__(kFinThreads) void tail_kernel(int64_t n, double *__restrict__ x, double *__restrict__ p,
                                                          double *__restrict__ r, TAp *__restrict__ Ap,
                                                          const double *__restrict__ inv,
                                                          const double *__restrict__ part_ax, int nax,
                                                          double *__restrict__ part_vec, CgState *st,
                                                          double *__restrict__ rho, double *__restrict__ hist)
{
    // each thread holds its K entries (i = threadIdx.x + k blockDim.x) in
    // registers from the residual to the update, every load of a pass in flight
    constexpr int K = static_cast<int>(kCgTailMax / kFinThreads);
    __shared__ double red[kFinThreads / 64];
    alpha_step(part_ax, nax, st, rho);
    __syncthreads();  // thread 0's state update, seen by the whole workgroup
    if (st->done) return;
    const double alpha = st->alpha;
    const int t = threadIdx.x, step = blockDim.x;
    double rv[K], zv[PC ? K : 1];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t i = t + static_cast<int64_t>(k) * step;
        rv[k] = i < n ? r[i] - alpha * static_cast<double>(Ap[i]) : 0.0;
        if constexpr (PC) zv[k] = i < n ? inv[i] : 0.0;
    }
    double rr = 0.0, rz = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t i = t + static_cast<int64_t>(k) * step;
        if (i < n) r[i] = rv[k];
        rr += rv[k] * rv[k];
        if constexpr (PC) rz += rv[k] * (zv[k] * rv[k]);
    }
    rr = block_sum(rr, red);
    if constexpr (PC) rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        part_vec[0] = PC ? rz : rr;
        if (PC) part_vec[1] = rr;
    }
    __syncthreads();
    beta_step(part_vec, 1, st, rho, hist, PC);
    __syncthreads();
    const double beta = st->beta;
    double pv[K], xv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t i = t + static_cast<int64_t>(k) * step;
        pv[k] = i < n ? p[i] : 0.0;
        xv[k] = i < n ? x[i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t i = t + static_cast<int64_t>(k) * step;
        if (i >= n) continue;
        x[i] = xv[k] + alpha * pv[k];
        if constexpr (PC)
            p[i] = zv[k] * rv[k] + beta * pv[k];
        else
            p[i] = rv[k] + beta * pv[k];
        Ap[i] = TAp(0);
    }
}

// Diagonal of the assembled operator, one thread per local node: at node
// (a,b,c) of an element, (D^T G D + lambda C)_ii = sum_m D[m][a]^2 G_rr(m,b,c)
// + sum_m D[m][b]^2 G_ss(a,m,c) + sum_m D[m][c]^2 G_tt(a,b,m)
// + 2 (D_aa D_bb G_rs + D_aa D_cc G_rt + D_bb D_cc G_st)(i) + lambda c(i),
// assembled by atomic addition (the cross terms meet only at the node itself).
__global__ __launch_bounds__(256) void jacobi_diag_kernel(int64_t nl, int N, const int32_t *__restrict__ map,
                                                          const double *__restrict__ geo,
                                                          const double *__restrict__ Dm, double lambda,
                                                          double *__restrict__ diag)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nl) return;
    const int32_t g = map[t];
    if (g < 0) return;
    const int n1 = N + 1;
    const int64_t np2 = (int64_t)n1 * n1, np3 = np2 * n1;
    const int64_t e = t / np3;
    const int n = static_cast<int>(t - e * np3);
    const int a = n % n1, b = (n / n1) % n1, c = n / (n1 * n1);
    // layer-major geometry: factor f of node (a', b', c') at [(e np3 + c' np2) 7 + f np2 + a' + n1 b']
    auto G = [&](int f, int aa, int bb, int cc) {
        return geo[(e * np3 + cc * np2) * kGeo + f * np2 + aa + n1 * bb];
    };
    double s = 0.0;
    for (int m = 0; m < n1; ++m) {
        s += Dm[m * n1 + a] * Dm[m * n1 + a] * G(0, m, b, c);
        s += Dm[m * n1 + b] * Dm[m * n1 + b] * G(3, a, m, c);
        s += Dm[m * n1 + c] * Dm[m * n1 + c] * G(5, a, b, m);
    }
    const double Daa = Dm[a * n1 + a], Dbb = Dm[b * n1 + b], Dcc = Dm[c * n1 + c];
    s += 2.0 * Daa * Dbb * G(1, a, b, c) + 2.0 * Daa * Dcc * G(2, a, b, c) + 2.0 * Dbb * Dcc * G(4, a, b, c);
    atomicAdd(&diag[g], s + lambda * G(6, a, b, c));
}

__global__ __launch_bounds__(kVecThreads) void invert_kernel(int64_t n, double *__restrict__ v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = 1.0 / v[i];
}

// r = b - t; partials of r.r (and, with inv, of r.z, z = inv r, after them).
__global__ __launch_bounds__(kVecThreads) void residual_norm_kernel(int64_t n, const double *__restrict__ b,
                                                                   const double *__restrict__ t,
                                                                   double *__restrict__ r,
                                                                   const double *__restrict__ inv,
                                                                   double *__restrict__ partial)
{
    __shared__ double red[kVecThreads / 64];
    double rr = 0.0, rz = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ri = b[i] - t[i];
        r[i] = ri;
        rr += ri * ri;
        if (inv) rz += ri * (inv[i] * ri);
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = rr;
    if (inv) {
        rz = block_sum(rz, red);
        if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = rz;
    }
}

// rho_iters = r.r (Jacobi, pc: r.z), history entry iters = ||r||, *out = r.r.
__global__ __launch_bounds__(kFinThreads) void replace_finish_kernel(const double *__restrict__ partial, int nblk,
                                                                    int pc, CgState *st, double *__restrict__ rho,
                                                                    double *__restrict__ hist,
                                                                    double *__restrict__ out)
{
    __shared__ double red[kFinThreads / 64];
    const double rr = sum_partials(partial, nblk, red);
    const double rz = pc ? sum_partials(partial + nblk, nblk, red) : rr;
    if (threadIdx.x != 0) return;
    const int j = st->iters;
    rho[j] = rz;
    hist[j] = sqrt(rr);
    *out = rr;
}

// Continue after a residual replacement: the next alpha starts iteration `iters`.
__global__ void resume_kernel(CgState *st, double stop_res)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->stop_res = stop_res;
    st->it = st->iters - 1;
    st->done = 0;
    st->pending = 0;
    st->status = HB_OK;
}

__global__ __launch_bounds__(kFinThreads) void sum_kernel(const double *__restrict__ partial, int nblk,
                                                         double *__restrict__ out)
{
    __shared__ double red[kFinThreads / 64];
    const double s = sum_partials(partial, nblk, red);
    if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(kVecThreads) void axpy_kernel(int64_t n, double *__restrict__ x,
                                                          const double *__restrict__ d)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += d[i];
}

__global__ __launch_bounds__(kVecThreads) void round_f32_kernel(const double *__restrict__ in, float *__restrict__ out,
                                                               int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = static_cast<float>(in[i]);  // round to nearest
}

}  // namespace

// Two entries per thread, up to 32768 workgroups: with 2048 workgroups (four or
// more entries each) a CG iteration at 32^3 N=7 took 378 us against 357 us, and
// the streaming kernels need many loads in flight (see also zero_blocks).
int vec_blocks(int64_t n)
{
    const int64_t want = (n + kVecThreads * 2 - 1) / (kVecThreads * 2);
    return static_cast<int>(want < 1 ? 1 : (want > 32768 ? 32768 : want));
}

// Clearing takes one entry per thread and up to 32768 workgroups: a store-only
// kernel needs many more stores in flight than the vector kernels' 2048-workgroup
// grid gives (the 32^3 N=7 vector: 15.7 us against 18.4 us with 2048 workgroups).
inline int zero_blocks(int64_t n)
{
    const int64_t want = (n + kVecThreads - 1) / kVecThreads;
    return static_cast<int>(want < 1 ? 1 : (want > 32768 ? 32768 : want));
}

template <typename V>
hb_status zero_any(V *v, int64_t n, hipStream_t s)
{
    if (n == 0) return HB_OK;
    zero_kernel<V><<<zero_blocks(n), kVecThreads, 0, s>>>(v, n);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_zero(double *v, int64_t n, hipStream_t s) { return zero_any(v, n, s); }
hb_status launch_zero(float *v, int64_t n, hipStream_t s) { return zero_any(v, n, s); }

hb_status launch_cg_setup_state(CgState *st, int max_iter, double rtol, hipStream_t s)
{
    setup_state_kernel<<<1, 64, 0, s>>>(st, max_iter, rtol);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

template <typename TAp>
hb_status launch_cg_init(int64_t n, const double *b, double *x, double *r, double *p, TAp *Ap, int x0_zero,
                         CgWork &w, CgState *st, hipStream_t s)
{
    const int g = vec_blocks(n);
    if (w.pc)
        init_kernel<TAp, true><<<g, kVecThreads, 0, s>>>(n, b, x, r, p, Ap, x0_zero, w.jinv, w.part_vec);
    else
        init_kernel<TAp, false><<<g, kVecThreads, 0, s>>>(n, b, x, r, p, Ap, x0_zero, nullptr, w.part_vec);
    init_finish_kernel<<<1, kFinThreads, 0, s>>>(w.part_vec, g, w.pc ? 1 : 0, st, w.rho, w.hist);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_cg_alpha(CgWork &w, int ax_grid, CgState *st, hipStream_t s)
{
    alpha_kernel<<<1, kFinThreads, 0, s>>>(w.part_ax, ax_grid, st, w.rho);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

template <typename TAp>
hb_status launch_cg_residual(int64_t n, double *r, const TAp *Ap, CgWork &w, CgState *st, hipStream_t s)
{
    if (w.pc)
        residual_kernel<TAp, true><<<vec_blocks(n), kVecThreads, 0, s>>>(n, r, Ap, w.jinv, w.part_vec, st);
    else
        residual_kernel<TAp, false><<<vec_blocks(n), kVecThreads, 0, s>>>(n, r, Ap, nullptr, w.part_vec, st);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_cg_beta(int64_t n, CgWork &w, CgState *st, hipStream_t s)
{
    beta_kernel<<<1, kFinThreads, 0, s>>>(w.part_vec, vec_blocks(n), w.pc ? 1 : 0, st, w.rho, w.hist);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

template <typename TAp>
hb_status launch_cg_update(int64_t n, double *x, double *p, const double *r, TAp *Ap, const double *inv, CgState *st,
                           hipStream_t s)
{
    // Ap of at most 128 MB (half the last-level cache) is cleared with plain
    // stores: at 32^3 N=7 (91 MB) a CG iteration took 336 us against 345 us with
    // non-temporal stores, on the 50^3 Dirichlet box (340 MB) 1493 us against 1481 us
    const bool cached = static_cast<uint64_t>(n) * sizeof(TAp) <= (uint64_t(128) << 20);
    const int g = vec_blocks(n);
    if (inv) {
        if (cached)
            update_kernel<TAp, true, true><<<g, kVecThreads, 0, s>>>(n, x, p, r, Ap, inv, st);
        else
            update_kernel<TAp, true, false><<<g, kVecThreads, 0, s>>>(n, x, p, r, Ap, inv, st);
    } else {
        if (cached)
            update_kernel<TAp, false, true><<<g, kVecThreads, 0, s>>>(n, x, p, r, Ap, nullptr, st);
        else
            update_kernel<TAp, false, false><<<g, kVecThreads, 0, s>>>(n, x, p, r, Ap, nullptr, st);
    }
    HB_HIP(hipGetLastError());
    return HB_OK;
}

template <typename TAp>
hb_status launch_cg_tail(int64_t n, double *x, double *p, double *r, TAp *Ap, const double *inv, CgWork &w, int nax,
                         CgState *st, hipStream_t s)
{
    if (inv)
        tail_kernel<TAp, true><<<1, kFinThreads, 0, s>>>(n, x, p, r, Ap, inv, w.part_ax, nax, w.part_vec, st, w.rho,
                                                         w.hist);
    else
        tail_kernel<TAp, false><<<1, kFinThreads, 0, s>>>(n, x, p, r, Ap, nullptr, w.part_ax, nax, w.part_vec, st,
                                                          w.rho, w.hist);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_jacobi_inverse(const hb_mesh_s *m, double lambda, double *inv, hipStream_t s)
{
    if (m->NG == 0) return HB_OK;
    zero_kernel<double><<<vec_blocks(m->NG), kVecThreads, 0, s>>>(inv, m->NG);
    jacobi_diag_kernel<<<static_cast<unsigned>((m->NL + 255) / 256), 256, 0, s>>>(m->NL, m->N, m->map, m->geo, m->D,
                                                                                   lambda, inv);
    invert_kernel<<<vec_blocks(m->NG), kVecThreads, 0, s>>>(m->NG, inv);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

template hb_status launch_cg_init<double>(int64_t, const double *, double *, double *, double *, double *, int,
                                          CgWork &, CgState *, hipStream_t);
template hb_status launch_cg_init<float>(int64_t, const double *, double *, double *, double *, float *, int,
                                         CgWork &, CgState *, hipStream_t);
template hb_status launch_cg_tail<double>(int64_t, double *, double *, double *, double *, const double *, CgWork &,
                                          int, CgState *, hipStream_t);
template hb_status launch_cg_tail<float>(int64_t, double *, double *, double *, float *, const double *, CgWork &,
                                         int, CgState *, hipStream_t);
template hb_status launch_cg_residual<double>(int64_t, double *, const double *, CgWork &, CgState *, hipStream_t);
template hb_status launch_cg_residual<float>(int64_t, double *, const float *, CgWork &, CgState *, hipStream_t);
template hb_status launch_cg_update<double>(int64_t, double *, double *, const double *, double *, const double *,
                                            CgState *, hipStream_t);
template hb_status launch_cg_update<float>(int64_t, double *, double *, const double *, float *, const double *,
                                           CgState *, hipStream_t);

hb_status launch_residual_norm(int64_t n, const double *b, const double *t, double *r, CgWork &w, double *out,
                               hipStream_t s)
{
    const int g = vec_blocks(n);
    residual_norm_kernel<<<g, kVecThreads, 0, s>>>(n, b, t, r, nullptr, w.part_vec);
    sum_kernel<<<1, kFinThreads, 0, s>>>(w.part_vec, g, out);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_cg_replace(int64_t n, const double *b, const double *t, double *r, CgWork &w, CgState *st,
                            double *out, const double *inv, hipStream_t s)
{
    const int g = vec_blocks(n);
    residual_norm_kernel<<<g, kVecThreads, 0, s>>>(n, b, t, r, inv, w.part_vec);
    replace_finish_kernel<<<1, kFinThreads, 0, s>>>(w.part_vec, g, inv ? 1 : 0, st, w.rho, w.hist, out);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_cg_resume(CgState *st, double stop_res, hipStream_t s)
{
    resume_kernel<<<1, 64, 0, s>>>(st, stop_res);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_axpy(int64_t n, double *x, const double *d, hipStream_t s)
{
    axpy_kernel<<<vec_blocks(n), kVecThreads, 0, s>>>(n, x, d);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status launch_round_f32(const double *in, float *out, int64_t n, hipStream_t s)
{
    if (n == 0) return HB_OK;
    round_f32_kernel<<<vec_blocks(n), kVecThreads, 0, s>>>(in, out, n);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

}  // namespace hb
