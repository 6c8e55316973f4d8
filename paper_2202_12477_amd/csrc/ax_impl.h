// The fused assembled screened-Poisson operator y = Z^T (S_L + lambda C) Z x
// (eq. poisson and eq. stiffness; the fused gather of the Poisson Operator
// section, with the Z^T assembly fused as well).
//
// Work decomposition (gfx950, wave64): a thread owns one (a,b) column of one
// element and walks its N+1 nodes along t, so
//   - the t-derivative and the t-part of D^T are register-only;
//   - the r/s derivatives of layer c read one (N+1)^2 slice from LDS, and the
//     r/s parts of D^T read one slice of f_r, f_s;
//   - the rows of D a thread needs live in registers (reused by every layer),
//     and so do its columns unless the schedule puts D^T in LDS;
//     D[c][*] is uniform across the block and comes through the scalar cache;
//   - each workgroup holds EPB elements (EPB*(N+1)^2 <= 256 threads, or <= 64
//     under the one-wave schedule), so N=7 is one wave per element and low
//     orders pack several elements per wave.
// HBM streams: map (4 B/node) and the 7 geometric values once, coalesced per
// layer (G two layers ahead, non-temporal where an element's run of a factor
// fills a cache line; stored layer-major per element, so an element's factors
// are one sequential read); x through an indirect (cache-friendly) gather; y
// by device-scope atomic adds into a zeroed vector (atomics on every node:
// mixing plain stores into lines that other elements update atomically
// measured far slower), with face-shared nodes of neighbouring elements in one
// wave merged first.  On a box the tiles are visited in a walk that keeps each
// XCD's neighbouring elements close in time (walk.h), so the lines of x and y
// they share meet in that XCD's L2.
//
// T is the arithmetic type: double (the method's FP64 operator) or float (the
// FP32 operator of the mixed-precision solver: FP32 geometry and D, x rounded
// to FP32 on load, FP32 accumulation and assembly).  x is FP64 in both.
#pragma once

#include <type_traits>

#include "common.h"
#include "reduce.h"
#include "walk.h"

namespace hb {

// Pointers into device (global) memory.  The tile routine takes them in the
// global address space explicitly: callers that read pointers from a table in
// memory would otherwise hand the compiler generic pointers, and every access
// would become a flat access (which also waits on the LDS counter).
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

template <typename T>
__device__ inline gptr<T> to_global(T *p)
{
    return (gptr<T>)p;
}

// Tile schedules of the operator, chosen per (degree, precision) class at run
// time (a table filled with measured defaults and rewritten by the autotuner):
//   kSchedColsLds - a thread reads the columns of D for D^T from LDS instead of
//                   keeping them in registers (frees 2(N+1) registers);
//   kSchedWave    - one-wave workgroups of floor(64/(N+1)^2) elements instead of
//                   256-thread workgroups: no element spans two waves, so the
//                   per-layer barriers are wave-local (legal for N <= 7);
//   kSchedLean    - no f_t array (the t-part of D^T is added per layer) and a
//                   target of two waves per SIMD, for the high degrees whose
//                   registers otherwise allow one (legal for N >= 8).
template <int N>
constexpr bool kWaveLegal = (N + 1) * (N + 1) <= 64;
template <int N>
constexpr bool kLeanLegal = !kWaveLegal<N>;
//   kSchedMerge   - (N <= 10, where a 256-thread workgroup holds two or more
//                   elements) the workgroup's epb elements are x-consecutive in
//                   one row of the box; at the end it sums the epb-1 faces they
//                   share in LDS and assembles each of the tile's (N+1)^2 rows
//                   of epb N + 1 consecutive DOFs once.  Each atomic add is a
//                   read-modify-write at the memory side on this part, and a
//                   row of 29 DOFs (N = 7) goes out in fewer, fuller requests
//                   than four rows of 8.  At N = 7 an element is exactly one
//                   wave, and the layer loops synchronise within their wave.
template <int N>
constexpr bool kMergeLegal = (N + 1) * (N + 1) <= 128;
//   kSchedThree   - (with kSchedLean and kSchedColsLds) D's rows and the map
//                   column also live in LDS, FP64 prefetches one geometry layer
//                   instead of two, and the target is three waves per SIMD: at
//                   the degrees where that fits without spills (FP64 N = 9, 11,
//                   12) the third wave hides more of the layer loop's latency
//                   than the extra LDS reads cost.
template <int V>
constexpr int kWavesTarget = (V & kSchedLean) ? ((V & kSchedThree) ? 3 : 2) : 1;
// the merged schedule's tiles lie in one row of the box, so its walk pads the rows
template <int N, int V>
constexpr bool kPadRows = (V & kSchedMerge) != 0 && kMergeLegal<N>;

template <int N, int V = 0>
struct AxShape {
    static constexpr int n1 = N + 1;
    static constexpr int np2 = n1 * n1;
    static constexpr int np3 = np2 * n1;
    static constexpr int target = ((V & kSchedWave) && kWaveLegal<N>) ? 64 : 256;
    static constexpr int epb = (target / np2) > 0 ? (target / np2) : 1;
    static constexpr int threads = (epb * np2 + 63) / 64 * 64;
};

// Geometry layers in flight ahead of the one being computed.
constexpr int kPrefetch = 2;

// Map entry of a node without a DOF (the boundary of a Dirichlet box): the
// gather reads 0 there and the assembly skips it.
constexpr uint32_t kNoDof = 0xffffffffu;

// Materialise a value here: stops the compiler from sinking a layer's
// arithmetic to the end of the kernel, which would keep every layer's LDS
// operands live at once.
template <typename T>
__device__ inline void pin(T &v)
{
    asm volatile("" : "+v"(v));
}

// Geometry loads.  Non-temporal where one element's run of a factor within a
// layer ((N+1)^2 values) fills at least a 128-byte line; below that (FP64 N <= 2,
// FP32 N <= 4) a load instruction touches many partial lines that the next
// factors' loads touch again, and plain loads, which keep the lines in L2 for
// them, measured up to 1.6x faster.
template <bool NT, typename T>
__device__ inline T geo_load(gptr<const T> p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <typename T>
__device__ inline void atomic_add(gptr<T> p, T v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One tile of up to EPB consecutive elements (sp.e0 .. sp.e0 + sp.n - 1): y += A x on them and,
// with DOT, this block's sum of x_e . y_e, returned in every thread and written
// to *dot_out (thread 0) unless dot_out is null.
// Every thread of the block must call it (it synchronises the block).
// (Always inlined: the single-problem and the batched kernel both call it, and
// an out-of-line call would spill the whole register set.)
// rows: the tile's elements are x-consecutive in one row of the box (the
// merged assembly needs it; without it that schedule assembles node by node).
// map_nt (CG form): stream the map non-temporally.
template <int N, bool DOT, typename T, int V, bool MASK, bool LOCAL = false>
__device__ __attribute__((always_inline)) inline double ax_tile(TileSpan sp, gptr<const int32_t> __restrict__ map,
                               gptr<const T> __restrict__ geo, gptr<const T> __restrict__ Dm, T lambda,
                               gptr<const double> __restrict__ x, gptr<T> __restrict__ y,
                               gptr<double> __restrict__ dot_out, bool rows = false, bool map_nt = true)
{
    using S = AxShape<N, V>;
    constexpr int n1 = S::n1, np2 = S::np2, np3 = S::np3, epb = S::epb;
    // From N = 11 on (an element spans several waves, and the counters show the
    // waves waiting at the per-layer barriers for 41-53% of their lives) the
    // (N+1)^2 slices of q, f_r and f_s are double-buffered: a layer writes its
    // f_r, f_s and the next layer's q slice before ONE barrier, after which it
    // reads f_r, f_s (for D^T) and the next layer reads its q slice.  A tile then
    // takes N+2 workgroup barriers instead of 2(N+1); the arithmetic and its order
    // are unchanged.  (Measured 2-5% faster at N = 12-15, within 1% at N = 11, and
    // 3-5% slower at N = 9, 10 and for the FP32 N = 1 operator, so not below 11.)
    constexpr bool pipe = N >= 11;
    constexpr int nbuf = pipe ? 2 : 1;
    __shared__ T sq[nbuf][epb][np2];
    __shared__ T sr[nbuf][epb][np2];
    __shared__ T ss[nbuf][epb][np2];
    __shared__ double red[S::threads / 64];

    const int t = threadIdx.x;
    const bool lane_used = t < epb * np2;
    const int el = lane_used ? t / np2 : epb - 1;  // spare lanes mirror the last element, inactive
    const int ab = lane_used ? t - el * np2 : 0;
    const int a = ab % n1, b = ab / n1;
    const bool active = lane_used && el < sp.n;
    const int64_t eo = sp.e0 + (el < sp.n ? el : sp.n - 1);  // inactive lanes read a valid element and discard it
    // rows a, b of D in registers, loaded once; columns a, b likewise, or D^T in LDS
    constexpr bool cols_lds = (V & kSchedColsLds) != 0;
    __shared__ T sDt[cols_lds ? np2 : 1];
    // three-wave form: rows of D in LDS as well, and the map column parked there
    // between the gather and the assembly
    constexpr bool three = (V & kSchedThree) != 0 && cols_lds && (V & kSchedLean) != 0;
    __shared__ T sD[three ? np2 : 1];
    __shared__ uint32_t sidx[three && !LOCAL ? epb * np3 : 1];
    T Da[three ? 1 : n1], Db[three ? 1 : n1], DaT[cols_lds ? 1 : n1], DbT[cols_lds ? 1 : n1];
#pragma unroll
    for (int m = 0; m < n1; ++m) {
        if constexpr (!three) {
            Da[m] = Dm[a * n1 + m];
            Db[m] = Dm[b * n1 + m];
        }
        if constexpr (!cols_lds) {
            DaT[m] = Dm[m * n1 + a];
            DbT[m] = Dm[m * n1 + b];
        }
    }
    // merged assembly at N = 7: each wave holds one element and its own LDS slices,
    // so the layer loop synchronises within the wave (LDS writes complete before
    // the reads); at the other degrees elements share waves and the workgroup syncs
    constexpr bool merge = (V & kSchedMerge) != 0 && kMergeLegal<N> && !LOCAL;
    constexpr bool wave_sync = merge && np2 == 64;
    auto layer_sync = [] {
        if constexpr (wave_sync) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        } else {
            __syncthreads();
        }
    };
    if constexpr (cols_lds) {
        // sDt[i][m] = D[m][i]; the first layer's barriers order these stores before any read
        for (int i = t; i < np2; i += S::threads) sDt[(i % n1) * n1 + i / n1] = Dm[i];
        if constexpr (three)
            for (int i = t; i < np2; i += S::threads) sD[i] = Dm[i];
        if constexpr (wave_sync) __syncthreads();  // filled by the first wave, read by all
    }

    // gather through Z: the (a,b) column of the element
    uint32_t idx[n1];
    T q[n1];
    gptr<const uint32_t> me = (gptr<const uint32_t>)map + eo * np3 + ab;
#pragma unroll
    for (int c = 0; c < n1; ++c) {
        // back to back, the map itself is reused from the last-level cache;
        // inside CG (DOT) too where map, p and Ap fit that cache together, else
        // a non-temporal map stream keeps p and Ap there
        if (DOT && map_nt)
            idx[c] = __builtin_nontemporal_load(&me[c * np2]);
        else
            idx[c] = me[c * np2];
    }
    if constexpr (MASK) {
#pragma unroll
        for (int c = 0; c < n1; ++c) {
            const bool dof = idx[c] != kNoDof;
            const double v = x[dof ? idx[c] : 0u];
            q[c] = dof ? static_cast<T>(v) : T(0);
        }
    } else {
#pragma unroll
        for (int c = 0; c < n1; ++c) q[c] = static_cast<T>(x[idx[c]]);
    }
    if constexpr (three && !LOCAL) {
        // read back by the same thread before its atomics
        if (lane_used) {
#pragma unroll
            for (int c = 0; c < n1; ++c) sidx[el * np3 + c * np2 + ab] = idx[c];
        }
    }

    // G is streamed once: non-temporal loads keep it from evicting x and y from
    // the caches (above a line per element and factor, geo_load).  Layers c+1 .. c+PF are in flight while layer c is computed
    // (a ring of PF register sets; the loop is unrolled, so slots are static).
    constexpr int PF = (three && sizeof(T) == 8) ? 1 : (kPrefetch < n1 ? kPrefetch : n1);
    // geometry layout [E][layer c][factor f][(N+1)^2 nodes of the layer]
    gptr<const T> ge = geo + eo * kGeo * np3 + ab;
    constexpr bool geo_nt = np2 * sizeof(T) >= 128;
    T Gq[PF][kGeo];
#pragma unroll
    for (int p = 0; p < PF; ++p) {
#pragma unroll
        for (int f = 0; f < kGeo; ++f) Gq[p][f] = geo_load<geo_nt>(&ge[(p * kGeo + f) * np2]);
    }
    // lean schedule: the t-part of D^T is added into the column as each layer's
    // f_t appears, so no f_t array is kept (2(N+1) fewer registers)
    constexpr bool lean = (V & kSchedLean) != 0;
    T ft[lean ? 1 : n1], yv[n1];
    if constexpr (lean) {
#pragma unroll
        for (int c = 0; c < n1; ++c) yv[c] = 0;
    }
    if constexpr (pipe) {
        if (lane_used) sq[0][el][ab] = q[0];
        layer_sync();
    }
#pragma unroll
    for (int c = 0; c < n1; ++c) {
        const int cb = pipe ? (c & 1) : 0;  // this layer's buffers
        // keep each layer's instructions together: stops the scheduler from
        // hoisting every layer's loads (and spilling them)
        __builtin_amdgcn_sched_barrier(0);
        T G[kGeo];
#pragma unroll
        for (int f = 0; f < kGeo; ++f) G[f] = Gq[c % PF][f];
        if (c + PF < n1) {
#pragma unroll
            for (int f = 0; f < kGeo; ++f)
                Gq[c % PF][f] = geo_load<geo_nt>(&ge[((c + PF) * kGeo + f) * np2]);
        }
        // t-derivative from registers; D[c][*] is uniform (scalar loads)
        T qt = 0;
#pragma unroll
        for (int m = 0; m < n1; ++m) qt += Dm[c * n1 + m] * q[m];
        if constexpr (!pipe) {
            if (lane_used) sq[0][el][ab] = q[c];
            layer_sync();
        }
        T qr = 0, qs = 0;
#pragma unroll
        for (int m = 0; m < n1; ++m) {
            if constexpr (three) {
                qr += sD[a * n1 + m] * sq[cb][el][b * n1 + m];
                qs += sD[b * n1 + m] * sq[cb][el][m * n1 + a];
            } else {
                qr += Da[m] * sq[cb][el][b * n1 + m];
                qs += Db[m] * sq[cb][el][m * n1 + a];
            }
        }
        const T fr = G[0] * qr + G[1] * qs + G[2] * qt;
        const T fs = G[1] * qr + G[3] * qs + G[4] * qt;
        if constexpr (lean) {
            T f = G[2] * qr + G[4] * qs + G[5] * qt;
            pin(f);
#pragma unroll
            for (int k = 0; k < n1; ++k) yv[k] += Dm[c * n1 + k] * f;
        } else {
            ft[c] = G[2] * qr + G[4] * qs + G[5] * qt;
            pin(ft[c]);
        }
        T acc = lambda * G[6] * q[c];
        if (lane_used) {
            sr[cb][el][ab] = fr;
            ss[cb][el][ab] = fs;
            if (pipe && c + 1 < n1) sq[cb ^ 1][el][ab] = q[c + 1];
        }
        layer_sync();
        if constexpr (sizeof(T) == 8) {
            // FP64: the r half, then the s half.  Issued together, the two
            // halves' LDS operands are the register peak of the kernel (at N=7
            // the difference between two and three waves per SIMD).
            if constexpr (cols_lds) {
#pragma unroll
                for (int m = 0; m < n1; ++m) acc += sDt[a * n1 + m] * sr[cb][el][b * n1 + m];
#pragma unroll
                for (int m = 0; m < n1; ++m) acc += sDt[b * n1 + m] * ss[cb][el][m * n1 + a];
            } else {
#pragma unroll
                for (int m = 0; m < n1; ++m) acc += DaT[m] * sr[cb][el][b * n1 + m];
#pragma unroll
                for (int m = 0; m < n1; ++m) acc += DbT[m] * ss[cb][el][m * n1 + a];
            }
        } else if constexpr (cols_lds) {
#pragma unroll
            for (int m = 0; m < n1; ++m)
                acc += sDt[a * n1 + m] * sr[cb][el][b * n1 + m] + sDt[b * n1 + m] * ss[cb][el][m * n1 + a];
        } else {
#pragma unroll
            for (int m = 0; m < n1; ++m) acc += DaT[m] * sr[cb][el][b * n1 + m] + DbT[m] * ss[cb][el][m * n1 + a];
        }
        pin(acc);
        if constexpr (lean)
            yv[c] += acc;
        else
            yv[c] = acc;
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (!lean) {
        // t-part of D^T from registers
#pragma unroll
        for (int c = 0; c < n1; ++c) {
            T s = 0;
#pragma unroll
            for (int m = 0; m < n1; ++m) s += Dm[m * n1 + c] * ft[m];
            yv[c] += s;
        }
    }
    if constexpr (MASK) {
        // materialise the outputs here: the assembly below is conditional per
        // node, and the compiler would otherwise sink each output's last sums
        // into its own branch and serialise them
#pragma unroll
        for (int c = 0; c < n1; ++c) pin(yv[c]);
    }
    if constexpr (LOCAL) {
        // the two-phase form: y is the unassembled local vector y_L, [E][(N+1)^3]
        // in the map's order, written with plain coalesced stores (the gather
        // that assembles it reads it back while it is still in the caches)
        if (active) {
            gptr<T> yl = y + eo * np3 + ab;
#pragma unroll
            for (int c = 0; c < n1; ++c) yl[c * np2] = yv[c];
        }
    } else {
    bool assembled = false;
    if constexpr (merge) {
        if (rows) {
            // the tile's (N+1)^2 rows of n N + 1 DOFs (n = sp.n elements): every
            // element stores its a < N nodes (the last one also a = N), then the
            // a = N nodes of the others are added to the a = 0 nodes of their right
            // neighbours, then each row goes out as one run of atomic adds (the
            // indices come from the lanes' own map entries; a shared face's two
            // copies agree)
            static_assert(epb >= 2, "a merged tile holds two or more elements");
            constexpr int L = epb * N + 1;
            __shared__ T sy[n1][n1][L];
            __shared__ uint32_t sid[n1][n1][L];
            const int last = sp.n - 1;
            if (active && (a < N || el == last)) {
#pragma unroll
                for (int c = 0; c < n1; ++c) {
                    sy[c][b][N * el + a] = yv[c];
                    uint32_t id = idx[c];
                    if constexpr (three) id = sidx[el * np3 + c * np2 + ab];  // parked in LDS
                    sid[c][b][N * el + a] = id;
                }
            }
            __syncthreads();
            if (active && a == N && el < last) {
#pragma unroll
                for (int c = 0; c < n1; ++c) sy[c][b][N * el + N] += yv[c];
            }
            __syncthreads();
            const T *flat_y = &sy[0][0][0];
            const uint32_t *flat_i = &sid[0][0][0];
            const int used = N * sp.n + 1;  // entries of a row that a short tile fills
            for (int k = t; k < n1 * n1 * L; k += S::threads) {
                const uint32_t id = flat_i[k];
                if ((sp.n == epb || k % L < used) && (!MASK || id != kNoDof)) atomic_add(&y[id], flat_y[k]);
            }
            assembled = true;
        }
    }
    if (!assembled) {
    // assemble through Z^T.  Where several elements share a wave, the a = 0 face
    // node of an element is the a = N face node of the previous one whenever the
    // two are neighbours along r: the lanes holding them then see the same index,
    // and the a = N lane adds its partner's value and issues the only atomic
    // (half as many atomics at N = 1, a quarter fewer at N = 3, and no two lanes
    // of one atomic instruction hitting the same address along r).
    constexpr int kShift = np2 - N;  // lane distance from an a = N node to the next element's a = 0 node
    if constexpr (epb > 1 && np2 < 64) {
        const int lane = t & 63;
        const int act = active ? 1 : 0;
        const int next_act = __shfl(act, lane + kShift);
        const int prev_act = __shfl(act, lane - kShift);
        const bool may_recv = act && a == N && lane + kShift < 64 && next_act;
        const bool may_send = act && a == 0 && lane >= kShift && prev_act;
#pragma unroll
        for (int c = 0; c < n1; ++c) {
            const int id = static_cast<int>(idx[c]);
            const int id_next = __shfl(id, lane + kShift);
            const int id_prev = __shfl(id, lane - kShift);
            const T v_next = __shfl(yv[c], lane + kShift);
            const bool recv = may_recv && id_next == id;
            const bool sent = may_send && id_prev == id;
            if (active && !sent && (!MASK || id != static_cast<int>(kNoDof)))
                atomic_add(&y[idx[c]], recv ? yv[c] + v_next : yv[c]);
        }
    } else if (active) {
        if constexpr (three) {
#pragma unroll
            for (int c = 0; c < n1; ++c) idx[c] = sidx[el * np3 + c * np2 + ab];
        }
        if constexpr (MASK) {
#pragma unroll
            for (int c = 0; c < n1; ++c)
                if (idx[c] != kNoDof) atomic_add(&y[idx[c]], yv[c]);
        } else {
#pragma unroll
            for (int c = 0; c < n1; ++c) atomic_add(&y[idx[c]], yv[c]);
        }
    }
    }
    }
    if constexpr (DOT) {
        // sum_e x_e . y_e = x . Z^T y_L = x . A x, accumulated in FP64
        double v = 0.0;
        if (active) {
#pragma unroll
            for (int c = 0; c < n1; ++c) v += static_cast<double>(q[c]) * static_cast<double>(yv[c]);
        }
        v = block_sum(v, red);
        if (t == 0 && dot_out) *dot_out = v;
        return v;
    }
    return 0.0;
}

template <int N, bool DOT, typename T, int V, bool MASK>
__global__ __launch_bounds__((AxShape<N, V>::threads))
__attribute__((amdgpu_waves_per_eu(kWavesTarget<V>))) void ax_kernel(
    int64_t E, TileWalk walk, const int32_t *__restrict__ map, const T *__restrict__ geo, const T *__restrict__ Dm,
    T lambda, const double *__restrict__ x, T *__restrict__ y, double *__restrict__ partial,
    const CgState *__restrict__ st, int map_nt)
{
    if constexpr (DOT) {
        // stopped, or stopping at the next alpha step (which reads no partials)
        if (st->done | st->pending) return;
    }
    // rows: the walk is defined (whole or padded rows), so every tile is
    // x-consecutive elements of one row
    const TileSpan sp = tile_span(walk, walk_tile(walk, xcd_remap(blockIdx.x, gridDim.x)), E, AxShape<N, V>::epb);
    ax_tile<N, DOT, T, V, MASK>(sp, to_global(map), to_global(geo), to_global(Dm), lambda, to_global(x),
                                to_global(y), to_global(DOT ? partial + blockIdx.x : partial), walk.txn != 0,
                                map_nt != 0);
}

// First phase of the two-phase operator: y_L = (S_L + lambda C) Z x per element
// (no assembly), with the same tiles and optional p.Ap partials as ax_kernel.
template <int N, bool DOT, int V, bool MASK>
__global__ __launch_bounds__((AxShape<N, V>::threads))
__attribute__((amdgpu_waves_per_eu(kWavesTarget<V>))) void ax_local_kernel(
    int64_t E, TileWalk walk, const int32_t *__restrict__ map, const double *__restrict__ geo,
    const double *__restrict__ Dm, double lambda, const double *__restrict__ x, double *__restrict__ yl,
    double *__restrict__ partial, const CgState *__restrict__ st)
{
    if constexpr (DOT) {
        if (st->done | st->pending) return;
    }
    const TileSpan sp = tile_span(walk, walk_tile(walk, xcd_remap(blockIdx.x, gridDim.x)), E, AxShape<N, V>::epb);
    ax_tile<N, DOT, double, V, MASK, true>(sp, to_global(map),
                                           to_global(geo), to_global(Dm), lambda, to_global(x), to_global(yl),
                                           to_global(DOT ? partial + blockIdx.x : partial));
}

// Values read from a work list or a problem table are the same for the whole
// block; saying so lets the compiler keep them (and everything derived from
// them, such as the uniform entries of D) in scalar registers.
__device__ inline int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uniform(int64_t v)
{
    const uint64_t u = static_cast<uint64_t>(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}
template <typename P>
__device__ inline P *uniform(P *p)
{
    return reinterpret_cast<P *>(uniform(reinterpret_cast<int64_t>(p)));
}
__device__ inline double uniform(double v)
{
    return __builtin_bit_cast(double, uniform(__builtin_bit_cast(int64_t, v)));
}

// The batched operator: one block per (problem, tile) item of a class's work
// list, with p.Ap fused.  D depends only on the degree, so all problems of a
// class share it; as a read-only kernel argument its block-uniform entries come
// through scalar loads.
template <int N, typename T, int V, bool MASK>
__global__ __launch_bounds__((AxShape<N, V>::threads))
__attribute__((amdgpu_waves_per_eu(kWavesTarget<V>))) void batch_ax_kernel(const WorkItem *__restrict__ items,
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
    // the list holds tiles of the same walk as the single-problem launch (padded
    // rows under the merged schedule); with whole or padded rows a tile lies in one x-row
    constexpr int epb = AxShape<N, V>::epb;
    const int32_t nx = uniform(P.nx);
    const TileWalk w = make_walk(nx, 1, 1, epb, kPadRows<N, V>);
    const TileSpan sp = tile_span(w, static_cast<uint32_t>(tile), E, epb);
    const bool rows = nx > 0 && w.txn != 0;
    if constexpr (sizeof(T) == 4)
        ax_tile<N, true, float, V, MASK>(sp, map, to_global(uniform(P.geo32)), to_global(Dm),
                                   static_cast<float>(uniform(P.lambda)), x, to_global(uniform(P.Ap32)), part, rows);
    else
        ax_tile<N, true, double, V, MASK>(sp, map, to_global(uniform(P.geo)), to_global(Dm), uniform(P.lambda), x,
                                    to_global(uniform(P.Ap)), part, rows);
}

template <int N, int V>
int ax_grid(int64_t E)
{
    return static_cast<int>((E + AxShape<N, V>::epb - 1) / AxShape<N, V>::epb);
}

// The tile order of a box under schedule V, and its tile count.
template <int N, int V>
TileWalk ax_walk(int64_t nx, int64_t ny, int64_t nz)
{
    return make_walk(nx, ny, nz, AxShape<N, V>::epb, kPadRows<N, V>);
}

// Run-time schedule -> compile-time instantiation.  Bits not available at
// this degree are dropped (the host validates schedules before they reach
// the table, so this only bounds the instantiations).
template <int N>
constexpr int legal_sched(int v)
{
    // merging needs the 256-thread tile: it drops the one-wave bit
    const int m = v & (kMergeLegal<N> ? kSchedMerge : 0);
    // the three-wave form needs the lean schedule with D^T in LDS
    constexpr int both = kSchedColsLds | kSchedLean;
    const int three = kLeanLegal<N> && (v & both) == both ? (v & kSchedThree) : 0;
    return (v & (kSchedColsLds | (kWaveLegal<N> && !m ? kSchedWave : 0) | (kLeanLegal<N> ? kSchedLean : 0))) | m |
           three;
}
template <int N, typename F>
decltype(auto) with_schedule(int v, F &&f)
{
    switch (legal_sched<N>(v)) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, legal_sched<N>(2)>{});
    case 3: return f(std::integral_constant<int, legal_sched<N>(3)>{});
    case 4: return f(std::integral_constant<int, legal_sched<N>(4)>{});
    case 5: return f(std::integral_constant<int, legal_sched<N>(5)>{});
    case 8: return f(std::integral_constant<int, legal_sched<N>(8)>{});
    case 9: return f(std::integral_constant<int, legal_sched<N>(9)>{});
    case 21: return f(std::integral_constant<int, legal_sched<N>(21)>{});
    case 29: return f(std::integral_constant<int, legal_sched<N>(29)>{});
    default: return f(std::integral_constant<int, 0>{});
    }
}

template <int N>
int ax_epb_sched(int v)
{
    return with_schedule<N>(v, [&](auto VV) { return AxShape<N, decltype(VV)::value>::epb; });
}

template <int N>
TileWalk ax_walk_sched(int64_t nx, int64_t ny, int64_t nz, int v)
{
    return with_schedule<N>(v, [&](auto VV) { return ax_walk<N, decltype(VV)::value>(nx, ny, nz); });
}

template <int N, typename T, bool MASK>
hb_status launch_ax_n(const hb_mesh_s *m, const T *geo, const T *D, double lambda, const double *x, T *y,
                      double *partial, CgState *st, hipStream_t s)
{
    return with_schedule<N>(mesh_schedule(m, sizeof(T) == 4), [&](auto VV) -> hb_status {
        constexpr int V = decltype(VV)::value;
        const TileWalk walk = ax_walk<N, V>(m->desc.nx, m->desc.ny, m->desc.nz);
        const int grid = static_cast<int>(walk_tiles(walk, m->E, AxShape<N, V>::epb));
        if (grid == 0) return HB_OK;
        const T lam = static_cast<T>(lambda);
        // CG: map (4 N_L bytes), p (8 N_G) and Ap (sizeof(T) N_G) within the
        // 256 MB last-level cache: plain map loads (32^3 N=7, 249 MB: 333 against
        // 338 us per iteration); above it non-temporal (50^3 Dirichlet: 1488
        // against 1504 us)
        const bool map_nt = static_cast<uint64_t>(m->NL) * 4 + static_cast<uint64_t>(m->NG) * (8 + sizeof(T)) >
                            (uint64_t(256) << 20);
        if (st)
            ax_kernel<N, true, T, V, MASK><<<grid, AxShape<N, V>::threads, 0, s>>>(m->E, walk, m->map, geo, D, lam, x,
                                                                             y, partial, st, map_nt ? 1 : 0);
        else
            ax_kernel<N, false, T, V, MASK><<<grid, AxShape<N, V>::threads, 0, s>>>(m->E, walk, m->map, geo, D, lam, x,
                                                                              y, nullptr, nullptr, 0);
        HB_HIP(hipGetLastError());
        return HB_OK;
    });
}

// The first phase under the degree's default FP64 schedule (V): y_L for every
// local node of the mesh.
template <int N, int V, bool MASK>
hb_status launch_ax_local_n(const hb_mesh_s *m, double lambda, const double *x, double *yl, double *partial,
                            CgState *st, hipStream_t s)
{
    const int grid = ax_grid<N, V>(m->E);
    if (grid == 0) return HB_OK;
    const TileWalk walk = make_walk(m->desc.nx, m->desc.ny, m->desc.nz, AxShape<N, V>::epb);
    if (st)
        ax_local_kernel<N, true, V, MASK><<<grid, AxShape<N, V>::threads, 0, s>>>(m->E, walk, m->map, m->geo, m->D,
                                                                                lambda, x, yl, partial, st);
    else
        ax_local_kernel<N, false, V, MASK><<<grid, AxShape<N, V>::threads, 0, s>>>(m->E, walk, m->map, m->geo, m->D,
                                                                                 lambda, x, yl, nullptr, nullptr);
    HB_HIP(hipGetLastError());
    return HB_OK;
}

template <int N, bool MASK>
hb_status launch_batch_ax_n(int sched, const void *D, bool fp32, const WorkItem *items, int nitems,
                            const BatchProb *probs, hipStream_t s)
{
    if (nitems == 0) return HB_OK;
    return with_schedule<N>(sched, [&](auto VV) -> hb_status {
        constexpr int V = decltype(VV)::value;
        if (fp32)
            batch_ax_kernel<N, float, V, MASK><<<nitems, AxShape<N, V>::threads, 0, s>>>(items, probs,
                                                                                  static_cast<const float *>(D));
        else
            batch_ax_kernel<N, double, V, MASK><<<nitems, AxShape<N, V>::threads, 0, s>>>(items, probs,
                                                                                   static_cast<const double *>(D));
        HB_HIP(hipGetLastError());
        return HB_OK;
    });
}

}  // namespace hb

// One degree's entry points (FP64 and FP32 operator, batched operator, grid
// size per schedule), expanded in the per-range translation units so the
// instantiations compile in parallel.
#define HB_AX_INSTANCE(n)                                                                                      \
    namespace hb {                                                                                             \
    hb_status launch_ax_##n(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st,  \
                            hipStream_t s)                                                                     \
    {                                                                                                          \
        return launch_ax_n<n, double, false>(m, m->geo, m->D, l, x, y, p, st, s);                              \
    }                                                                                                          \
    hb_status launch_ax32_##n(const hb_mesh_s *m, double l, const double *x, float *y, double *p, CgState *st, \
                              hipStream_t s)                                                                   \
    {                                                                                                          \
        return launch_ax_n<n, float, false>(m, m->geo32, m->D32, l, x, y, p, st, s);                           \
    }                                                                                                          \
    hb_status launch_batch_ax_##n(int v, const void *D, bool fp32, const WorkItem *it, int ni,                 \
                                  const BatchProb *pr, hipStream_t s)                                          \
    {                                                                                                          \
        return launch_batch_ax_n<n, false>(v, D, fp32, it, ni, pr, s);                                         \
    }                                                                                                          \
    int ax_epb_##n(int v) { return ax_epb_sched<n>(v); }                                                       \
    TileWalk ax_walk_##n(int64_t nx, int64_t ny, int64_t nz, int v) { return ax_walk_sched<n>(nx, ny, nz, v); }\
    }

// The same entry points for Dirichlet boxes (boundary nodes without DOFs:
// guarded gather and assembly), in translation units of their own.
#define HB_AX_INSTANCE_DIRICHLET(n)                                                                            \
    namespace hb {                                                                                             \
    hb_status launch_ax_d_##n(const hb_mesh_s *m, double l, const double *x, double *y, double *p, CgState *st,\
                              hipStream_t s)                                                                   \
    {                                                                                                          \
        return launch_ax_n<n, double, true>(m, m->geo, m->D, l, x, y, p, st, s);                               \
    }                                                                                                          \
    hb_status launch_ax32_d_##n(const hb_mesh_s *m, double l, const double *x, float *y, double *p,            \
                                CgState *st, hipStream_t s)                                                    \
    {                                                                                                          \
        return launch_ax_n<n, float, true>(m, m->geo32, m->D32, l, x, y, p, st, s);                            \
    }                                                                                                          \
    hb_status launch_batch_ax_d_##n(int v, const void *D, bool fp32, const WorkItem *it, int ni,               \
                                    const BatchProb *pr, hipStream_t s)                                        \
    {                                                                                                          \
        return launch_batch_ax_n<n, true>(v, D, fp32, it, ni, pr, s);                                          \
    }                                                                                                          \
    }

// The first phase of the two-phase operator for one degree (plain and
// Dirichlet meshes), under schedule v, in a translation unit of its own.
#define HB_AX_INSTANCE_LOCAL(n, v)                                                                             \
    namespace hb {                                                                                             \
    hb_status launch_ax_local_##n(const hb_mesh_s *m, double l, const double *x, double *yl, double *p,        \
                                  CgState *st, hipStream_t s)                                                  \
    {                                                                                                          \
        return (m->desc.flags & HB_MESH_DIRICHLET) ? launch_ax_local_n<n, v, true>(m, l, x, yl, p, st, s)      \
                                                   : launch_ax_local_n<n, v, false>(m, l, x, yl, p, st, s);    \
    }                                                                                                          \
    int ax_local_grid_##n(int64_t E) { return ax_grid<n, v>(E); }                                              \
    }
