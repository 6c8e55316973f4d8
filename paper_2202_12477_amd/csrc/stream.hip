// Empirical streaming-rate probe (Computational Tests section): each thread
// reads 8 FP64 values and writes one, the 8:1 read:write mix of the operator.
#include "common.h"

namespace hb {
namespace {

__global__ __launch_bounds__(256) void stream8to1_kernel(int64_t n, const double *__restrict__ in,
                                                         double *__restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) s += __builtin_nontemporal_load(&in[k * n + i]);
        __builtin_nontemporal_store(s, &out[i]);
    }
}

}  // namespace

hb_status launch_stream_probe(const double *in, double *out, int64_t n, hipStream_t s)
{
    if (n == 0) return HB_OK;
    const int64_t want = (n + 255) / 256;
    const unsigned grid = static_cast<unsigned>(want < 65536 ? want : 65536);
    stream8to1_kernel<<<grid, 256, 0, s>>>(n, in, out);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

}  // namespace hb
