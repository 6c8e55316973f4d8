// The two-phase form of the assembled operator (the Poisson Operator section:
// the element operator writes the local vector y_L, then Z^T assembles it as a
// gather): y_L = (S_L + lambda C) Z x in the first kernel, y_g = sum of y_L
// over the local copies of DOF g in the second.  Each DOF's copies are summed
// in ascending local order by one thread, so the result does not depend on
// scheduling: repeated applications (and whole CG solves) are bit-identical.
#include <vector>

#include "common.h"

namespace hb {

#define HB_DECL_LOCAL(n)                                                                                       \
    hb_status launch_ax_local_##n(const hb_mesh_s *, double, const double *, double *, double *, CgState *,    \
                                  hipStream_t);                                                                \
    int ax_local_grid_##n(int64_t);
HB_DECL_LOCAL(1) HB_DECL_LOCAL(2) HB_DECL_LOCAL(3) HB_DECL_LOCAL(4) HB_DECL_LOCAL(5) HB_DECL_LOCAL(6)
HB_DECL_LOCAL(7) HB_DECL_LOCAL(8) HB_DECL_LOCAL(9) HB_DECL_LOCAL(10) HB_DECL_LOCAL(11) HB_DECL_LOCAL(12)
HB_DECL_LOCAL(13) HB_DECL_LOCAL(14) HB_DECL_LOCAL(15)
#undef HB_DECL_LOCAL
#define HB_LOCAL_ALL_N(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

namespace {

constexpr int kGatherThreads = 256;

// y_g (+)= sum_{k in row g} y_L[idx[k]], one thread per DOF.  Inside CG (st set)
// it returns when the operator phase did (solve done or stopping).
__global__ __launch_bounds__(kGatherThreads) void gather_kernel(int64_t n, const uint32_t *__restrict__ off,
                                                                const uint32_t *__restrict__ idx,
                                                                const double *__restrict__ yl, double *__restrict__ y,
                                                                int add, const CgState *__restrict__ st)
{
    if (st && (st->done | st->pending)) return;
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n) return;
    const uint32_t b = off[g], e = off[g + 1];
    double s = add ? y[g] : 0.0;
    for (uint32_t k = b; k < e; ++k) s += yl[idx[k]];
    y[g] = s;
}

}  // namespace

int ax_local_blocks(const hb_mesh_s *m)
{
    switch (m->N) {
#define HB_CASE(n) \
    case n: return ax_local_grid_##n(m->E);
        HB_LOCAL_ALL_N(HB_CASE)
#undef HB_CASE
    default: return 0;
    }
}

hb_status launch_ax_two_phase(const hb_mesh_s *m, double lambda, const double *x, double *y, double *partial,
                              CgState *st, bool overwrite, hipStream_t s)
{
    hb_status e = HB_ERR_INVALID_ARG;
    switch (m->N) {
#define HB_CASE(n) \
    case n: e = launch_ax_local_##n(m, lambda, x, m->yl, partial, st, s); break;
        HB_LOCAL_ALL_N(HB_CASE)
#undef HB_CASE
    default: return fail(HB_ERR_INVALID_ARG, "unsupported degree N");
    }
    if (e) return e;
    if (m->NG == 0) return HB_OK;
    const unsigned grid = static_cast<unsigned>((m->NG + kGatherThreads - 1) / kGatherThreads);
    gather_kernel<<<grid, kGatherThreads, 0, s>>>(m->NG, m->zt_off, m->zt_idx, m->yl, y, overwrite ? 0 : 1, st);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

// The rows of Z^T as CSR (row g: the local nodes whose map entry is g, in
// ascending order), built on the host from the device map by a counting sort,
// and the y_L buffer.
hb_status build_gather(hb_mesh_s *m, hipStream_t s)
{
    if (m->NL >= (int64_t{1} << 32))
        return fail(HB_ERR_INVALID_ARG, "hb_mesh_create: the two-phase operator needs fewer than 2^32 local nodes");
    std::vector<int32_t> map;
    std::vector<uint32_t> off, idx;
    try {
        map.resize(m->NL);
        off.assign(m->NG + 1, 0u);
    } catch (...) {
        return fail(HB_ERR_OUT_OF_MEMORY, "hb_mesh_create: host memory for the gather rows");
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(map.data(), m->map, sizeof(int32_t) * m->NL, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "hb_mesh_create: map read-back");
    for (int64_t l = 0; l < m->NL; ++l)
        if (map[l] >= 0) ++off[map[l] + 1];
    for (int64_t g = 0; g < m->NG; ++g) off[g + 1] += off[g];
    try {
        idx.resize(off[m->NG]);
    } catch (...) {
        return fail(HB_ERR_OUT_OF_MEMORY, "hb_mesh_create: host memory for the gather rows");
    }
    {
        std::vector<uint32_t> next(off.begin(), off.end() - 1);
        for (int64_t l = 0; l < m->NL; ++l)
            if (map[l] >= 0) idx[next[map[l]]++] = static_cast<uint32_t>(l);
    }
    hb_status st;
    if ((st = dev_alloc(&m->zt_off, m->NG + 1, &m->device_bytes)) ||
        (st = dev_alloc(&m->zt_idx, std::max<size_t>(idx.size(), 1), &m->device_bytes)) ||
        (st = dev_alloc(&m->yl, m->NL, &m->device_bytes)))
        return st;
    if ((e = hipMemcpyAsync(m->zt_off, off.data(), sizeof(uint32_t) * off.size(), hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (idx.size() &&
         (e = hipMemcpyAsync(m->zt_idx, idx.data(), sizeof(uint32_t) * idx.size(), hipMemcpyHostToDevice, s)) !=
             hipSuccess) ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "hb_mesh_create: copy of the gather rows");
    return HB_OK;
}

}  // namespace hb
