// Mesh setup on the device: vertex jitter, the scatter map Z, the geometric
// factors G (NekBone section: the symmetric 3x3 block of diagonal matrices of
// metric terms combined with GLL weights) and the mass coefficient c; plus the
// pseudo-random forcing kernel of the HipBone section.
//
// Random numbers: splitmix64 (Steele, Lea & Flood, OOPSLA 2014).  A stream's
// start state is the generator's output number `stream` from state `seed`;
// value number i of the stream is the generator's output number i from that
// start state.  Output number i from state s is finalise(s + (i+1) * gamma).
#include <cmath>
#include <vector>

#include "common.h"

namespace hb {
namespace {

__host__ __device__ inline uint64_t sm64(uint64_t state, uint64_t i)
{
    uint64_t z = state + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ inline double unit_uniform(uint64_t stream_start, uint64_t i)
{
    return static_cast<double>(sm64(stream_start, i) >> 11) * 0x1.0p-53;
}

__global__ void rhs_kernel(int64_t n, uint64_t start, double *__restrict__ b)
{
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
        b[g] = 2.0 * unit_uniform(start, static_cast<uint64_t>(g)) - 1.0;
}

// Vertex coordinates [(nx+1)(ny+1)(nz+1)][3]; interior vertices are jittered.
__global__ void vertex_kernel(int nx, int ny, int nz, double jitter, uint64_t sx, uint64_t sy, uint64_t sz,
                              double *__restrict__ V)
{
    const int64_t nv = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int i = static_cast<int>(v % (nx + 1));
    const int j = static_cast<int>((v / (nx + 1)) % (ny + 1));
    const int k = static_cast<int>(v / ((int64_t)(nx + 1) * (ny + 1)));
    double c[3] = {(double)i / nx, (double)j / ny, (double)k / nz};
    const bool interior = i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz;
    if (interior && jitter != 0.0) {
        const uint64_t st[3] = {sx, sy, sz};
        const int n[3] = {nx, ny, nz};
        for (int d = 0; d < 3; ++d)
            c[d] += (jitter / n[d]) * (2.0 * unit_uniform(st[d], static_cast<uint64_t>(v)) - 1.0);
    }
    V[3 * v + 0] = c[0];
    V[3 * v + 1] = c[1];
    V[3 * v + 2] = c[2];
}

// One thread per local node: Z row, Jacobian of the trilinear map, G and c.
__global__ void geometry_kernel(int nx, int ny, int nz, int N, const double *__restrict__ V,
                                const double *__restrict__ xi, const double *__restrict__ w, int mass_invdeg,
                                int dirichlet, int32_t *__restrict__ map, double *__restrict__ geo,
                                int *__restrict__ bad)
{
    const int n1 = N + 1;
    const int64_t np3 = (int64_t)n1 * n1 * n1;
    const int64_t E = (int64_t)nx * ny * nz;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= E * np3) return;
    const int64_t e = t / np3;
    const int n = static_cast<int>(t - e * np3);
    const int a = n % n1, b = (n / n1) % n1, c = n / (n1 * n1);
    const int ex = static_cast<int>(e % nx), ey = static_cast<int>((e / nx) % ny), ez = static_cast<int>(e / ((int64_t)nx * ny));

    const int64_t gx = (int64_t)nx * N + 1, gy = (int64_t)ny * N + 1, gz = (int64_t)nz * N + 1;
    const int64_t gi = (int64_t)ex * N + a, gj = (int64_t)ey * N + b, gk = (int64_t)ez * N + c;
    if (!dirichlet)
        map[t] = static_cast<int32_t>(gi + gx * (gj + gy * gk));
    else if (gi == 0 || gj == 0 || gk == 0 || gi == gx - 1 || gj == gy - 1 || gk == gz - 1)
        map[t] = -1;  // boundary node: no DOF
    else
        map[t] = static_cast<int32_t>((gi - 1) + (gx - 2) * ((gj - 1) + (gy - 2) * (gk - 1)));

    // Trilinear map x(r) = sum over corners of X_corner * prod_d (1 +- r_d)/2.
    const double r = xi[a], s = xi[b], tt = xi[c];
    const double lo[3] = {0.5 * (1.0 - r), 0.5 * (1.0 - s), 0.5 * (1.0 - tt)};
    const double hi[3] = {0.5 * (1.0 + r), 0.5 * (1.0 + s), 0.5 * (1.0 + tt)};
    double jac[3][3] = {{0.0}};  // jac[i][d] = d x_i / d r_d
    for (int corner = 0; corner < 8; ++corner) {
        const int dx = corner & 1, dy = (corner >> 1) & 1, dz = corner >> 2;
        const int64_t v = (ex + dx) + (int64_t)(nx + 1) * ((ey + dy) + (int64_t)(ny + 1) * (ez + dz));
        const double fx = dx ? hi[0] : lo[0], fy = dy ? hi[1] : lo[1], fz = dz ? hi[2] : lo[2];
        const double gxr = (dx ? 0.5 : -0.5) * fy * fz;
        const double gys = fx * (dy ? 0.5 : -0.5) * fz;
        const double gzt = fx * fy * (dz ? 0.5 : -0.5);
        for (int i = 0; i < 3; ++i) {
            const double X = V[3 * v + i];
            jac[i][0] += X * gxr;
            jac[i][1] += X * gys;
            jac[i][2] += X * gzt;
        }
    }
    // cofactors: inv[d][i] = d r_d / d x_i = cof[i][d] / J
    const double c00 = jac[1][1] * jac[2][2] - jac[1][2] * jac[2][1];
    const double c01 = jac[1][2] * jac[2][0] - jac[1][0] * jac[2][2];
    const double c02 = jac[1][0] * jac[2][1] - jac[1][1] * jac[2][0];
    const double c10 = jac[0][2] * jac[2][1] - jac[0][1] * jac[2][2];
    const double c11 = jac[0][0] * jac[2][2] - jac[0][2] * jac[2][0];
    const double c12 = jac[0][1] * jac[2][0] - jac[0][0] * jac[2][1];
    const double c20 = jac[0][1] * jac[1][2] - jac[0][2] * jac[1][1];
    const double c21 = jac[0][2] * jac[1][0] - jac[0][0] * jac[1][2];
    const double c22 = jac[0][0] * jac[1][1] - jac[0][1] * jac[1][0];
    const double J = jac[0][0] * c00 + jac[0][1] * c01 + jac[0][2] * c02;
    if (!(J > 0.0)) atomicOr(bad, 1);
    const double invJ = 1.0 / J;
    // rows of the inverse Jacobian: grad r, grad s, grad t
    const double gr[3] = {c00 * invJ, c10 * invJ, c20 * invJ};
    const double gs[3] = {c01 * invJ, c11 * invJ, c21 * invJ};
    const double gt[3] = {c02 * invJ, c12 * invJ, c22 * invJ};
    const double wJ = w[a] * w[b] * w[c] * J;
    auto dot3 = [](const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
    // layer-major per element: [E][N+1 layers][7 factors][(N+1)^2 nodes of the layer]
    const int64_t np2 = (int64_t)n1 * n1;
    double *g = geo + (e * np3 + c * np2) * kGeo + (n - c * np2);
    g[0 * np2] = wJ * dot3(gr, gr);
    g[1 * np2] = wJ * dot3(gr, gs);
    g[2 * np2] = wJ * dot3(gr, gt);
    g[3 * np2] = wJ * dot3(gs, gs);
    g[4 * np2] = wJ * dot3(gs, gt);
    g[5 * np2] = wJ * dot3(gt, gt);
    g[6 * np2] = mass_invdeg ? 0.0 : wJ;
}

__global__ void count_kernel(int64_t nl, const int32_t *__restrict__ map, int32_t *__restrict__ mult)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < nl && map[t] >= 0) atomicAdd(&mult[map[t]], 1);
}

__global__ void invdeg_kernel(int64_t nl, int64_t np3, int64_t np2, const int32_t *__restrict__ map,
                              const int32_t *__restrict__ mult, double *__restrict__ geo)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nl) return;
    const int64_t e = t / np3, n = t - e * np3, c = n / np2;
    const int32_t g = map[t];
    geo[(e * np3 + c * np2) * kGeo + 6 * np2 + (n - c * np2)] = g >= 0 ? 1.0 / static_cast<double>(mult[g]) : 0.0;
}

inline unsigned blocks_for(int64_t n, int threads) { return static_cast<unsigned>((n + threads - 1) / threads); }

}  // namespace

hb_status launch_rhs(int64_t n, uint64_t seed, double *b, hipStream_t s)
{
    if (n == 0) return HB_OK;
    const int threads = 256;
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>(blocks_for(n, threads), 8192));
    rhs_kernel<<<grid, threads, 0, s>>>(n, sm64(seed, 0), b);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

hb_status build_geometry(hb_mesh_s *m, hipStream_t s)
{
    const hb_mesh_desc &d = m->desc;
    const int64_t nv = (int64_t)(d.nx + 1) * (d.ny + 1) * (d.nz + 1);
    const int64_t np3 = (int64_t)(m->N + 1) * (m->N + 1) * (m->N + 1);
    double *V = nullptr;
    int *bad = nullptr;
    int32_t *mult = nullptr;
    hb_status st = HB_OK;
    int h_bad = 0;
    auto cleanup = [&]() {
        if (V) (void)hipFree(V);
        if (bad) (void)hipFree(bad);
        if (mult) (void)hipFree(mult);
    };
    if (hipMalloc(&V, sizeof(double) * 3 * nv) != hipSuccess || hipMalloc(&bad, sizeof(int)) != hipSuccess) {
        cleanup();
        return fail(HB_ERR_OUT_OF_MEMORY, "hb_mesh_create: setup scratch allocation failed");
    }
    do {
        hipError_t e;
        if ((e = hipMemsetAsync(bad, 0, sizeof(int), s)) != hipSuccess) { st = hip_fail(e, "memset"); break; }
        vertex_kernel<<<blocks_for(nv, 256), 256, 0, s>>>(d.nx, d.ny, d.nz, d.jitter, sm64(d.seed, 1),
                                                           sm64(d.seed, 2), sm64(d.seed, 3), V);
        if ((e = hipGetLastError()) != hipSuccess) { st = hip_fail(e, "vertex_kernel"); break; }
        geometry_kernel<<<blocks_for(m->NL, 256), 256, 0, s>>>(d.nx, d.ny, d.nz, m->N, V, m->xi, m->w,
                                                                 d.mass == HB_MASS_INVDEG,
                                                                 (d.flags & HB_MESH_DIRICHLET) != 0, m->map, m->geo,
                                                                 bad);
        if ((e = hipGetLastError()) != hipSuccess) { st = hip_fail(e, "geometry_kernel"); break; }
        if (d.mass == HB_MASS_INVDEG) {
            if ((e = hipMalloc(&mult, sizeof(int32_t) * m->NG)) != hipSuccess) {
                st = fail(HB_ERR_OUT_OF_MEMORY, "hb_mesh_create: multiplicity allocation failed");
                break;
            }
            if ((e = hipMemsetAsync(mult, 0, sizeof(int32_t) * m->NG, s)) != hipSuccess) { st = hip_fail(e, "memset"); break; }
            count_kernel<<<blocks_for(m->NL, 256), 256, 0, s>>>(m->NL, m->map, mult);
            invdeg_kernel<<<blocks_for(m->NL, 256), 256, 0, s>>>(m->NL, np3, (int64_t)(m->N + 1) * (m->N + 1),
                                                                   m->map, mult, m->geo);
            if ((e = hipGetLastError()) != hipSuccess) { st = hip_fail(e, "invdeg_kernel"); break; }
        }
        if ((e = hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) {
            st = hip_fail(e, "hipMemcpyAsync");
            break;
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) { st = hip_fail(e, "hipStreamSynchronize"); break; }
        if (h_bad) st = fail(HB_ERR_INVALID_ARG, "hb_mesh_create: non-positive Jacobian (jitter too large?)");
    } while (false);
    cleanup();
    return st;
}

}  // namespace hb
