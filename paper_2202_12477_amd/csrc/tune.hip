// Autotuner of the operator's tile schedules.
//
// For one (degree, precision) class it builds a synthetic jittered box of a
// requested size (about 2^22 local nodes by default), times every schedule
// that is legal at that degree (y += A x launched back to back, HIP events on
// the caller's stream), and writes the fastest into the process-wide schedule
// table that the operator, CG and batched launches read.  Get/set let a
// caller inspect or pin entries.
#include <cmath>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"

using namespace hb;

namespace {

constexpr int kTuneWarm = 128;  // untimed launches before the first candidate

hb_status check_class(int32_t N, int32_t prec, const char *who)
{
    if (N < 1 || N > kMaxN) return fail(HB_ERR_INVALID_ARG, std::string(who) + ": N must be in [1, 15]");
    if (prec != HB_PREC_FP64 && prec != HB_PREC_FP32_IR && prec != HB_PREC_FP32_RR)
        return fail(HB_ERR_INVALID_ARG, std::string(who) + ": unknown precision");
    return HB_OK;
}

struct TuneScratch {
    hb_mesh mesh = nullptr;
    double *x = nullptr;
    void *y = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneScratch()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (x) (void)hipFree(x);
        if (y) (void)hipFree(y);
        if (mesh) (void)hb_mesh_destroy(mesh);
    }
};

}  // namespace

extern "C" {

hb_status hb_get_schedule(int32_t N, int32_t prec, int32_t *schedule)
{
    hb_status st;
    if ((st = check_class(N, prec, "hb_get_schedule"))) return st;
    if (!schedule) return fail(HB_ERR_INVALID_ARG, "hb_get_schedule: null argument");
    *schedule = ax_schedule(N, prec != HB_PREC_FP64);
    return HB_OK;
}

hb_status hb_set_schedule(int32_t N, int32_t prec, int32_t schedule)
{
    hb_status st;
    if ((st = check_class(N, prec, "hb_set_schedule"))) return st;
    if (!ax_schedule_legal(N, schedule))
        return fail(HB_ERR_INVALID_ARG, "hb_set_schedule: schedule not available at this degree");
    set_ax_schedule(N, prec != HB_PREC_FP64, schedule);
    return HB_OK;
}

hb_status hb_autotune(int32_t N, int32_t prec, int64_t local_nodes, int32_t reps, hb_tune_result *out,
                      void *stream)
{
    hb_status st;
    if ((st = check_class(N, prec, "hb_autotune"))) return st;
    if (reps > 10000) return fail(HB_ERR_INVALID_ARG, "hb_autotune: reps must be <= 10000");
    if (local_nodes > (int64_t(1) << 30))
        return fail(HB_ERR_INVALID_ARG, "hb_autotune: local_nodes must be <= 2^30");
    if (reps <= 0) reps = 20;
    if (local_nodes <= 0) local_nodes = int64_t(1) << 22;
    return tune_class(N, prec != HB_PREC_FP64, local_nodes, reps, out, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace hb {

hb_status tune_class(int N, bool fp32, int64_t local_nodes, int reps, hb_tune_result *out, hipStream_t s)
{
    hb_status st;
    void *stream = s;
    const int n = std::max(1, static_cast<int>(std::lround(std::cbrt(static_cast<double>(local_nodes) /
                                                                     std::pow(N + 1.0, 3)))));
    hb_mesh_desc d{};
    d.nx = d.ny = d.nz = n;
    d.N = N;
    d.jitter = 0.05;
    d.seed = 1;
    d.mass = HB_MASS_GWJ;
    d.flags = fp32 ? HB_MESH_FP32 : 0;
    TuneScratch t;
    if ((st = hb_mesh_create(&d, stream, &t.mesh))) return st;
    const int64_t NG = t.mesh->NG;
    size_t tally = 0;
    if ((st = dev_alloc(&t.x, NG, &tally)) || (st = launch_rhs(NG, 7, t.x, s))) return st;
    if (fp32) {
        float *y = nullptr;
        if ((st = dev_alloc(&y, NG, &tally))) return st;
        t.y = y;
        if ((st = launch_zero(y, NG, s))) return st;
    } else {
        double *y = nullptr;
        if ((st = dev_alloc(&y, NG, &tally))) return st;
        t.y = y;
        if ((st = launch_zero(y, NG, s))) return st;
    }
    HB_HIP(hipEventCreate(&t.e0));
    HB_HIP(hipEventCreate(&t.e1));
    auto apply = [&]() -> hb_status {
        return fp32 ? launch_ax32(t.mesh, 1.0, t.x, static_cast<float *>(t.y), nullptr, nullptr, s)
                    : launch_ax(t.mesh, 1.0, t.x, static_cast<double *>(t.y), nullptr, nullptr, s);
    };
    const int prev = ax_schedule(N, fp32);
    hb_tune_result res{};
    res.schedule = prev;
    for (double &u : res.us) u = -1.0;
    double best_us = std::numeric_limits<double>::infinity();
    // The device has been idle while the host built the box, and its first
    // ~100 launches run up to 15% slow (FP64 N = 9-12 on the order-sweep
    // boxes); the first candidate would pay for that.  Warm it up first.
    for (int w = 0; w < kTuneWarm; ++w) {
        const hb_status e = apply();
        if (e) return e;
    }
    for (int v = 0; v < kNumSched; ++v) {
        if (!ax_schedule_legal(N, v)) continue;
        set_ax_schedule(N, fp32, v);
        hb_status e = HB_OK;
        for (int w = 0; w < 2 && !e; ++w) e = apply();
        hipError_t he = e ? hipSuccess : hipEventRecord(t.e0, s);
        for (int r = 0; r < reps && !e && he == hipSuccess; ++r) e = apply();
        if (!e && he == hipSuccess) he = hipEventRecord(t.e1, s);
        if (!e && he == hipSuccess) he = hipEventSynchronize(t.e1);
        float ms = 0.0f;
        if (!e && he == hipSuccess) he = hipEventElapsedTime(&ms, t.e0, t.e1);
        if (e || he != hipSuccess) {
            set_ax_schedule(N, fp32, prev);
            return e ? e : hip_fail(he, "autotune: timing");
        }
        res.us[v] = 1e3 * ms / reps;
        ++res.candidates;
        if (res.us[v] < best_us) {
            best_us = res.us[v];
            res.schedule = v;
        }
    }
    set_ax_schedule(N, fp32, res.schedule);
    if (out) *out = res;
    return HB_OK;
}

namespace {

// Winners per (degree, precision, size class), for the life of the process.
struct TuneCache {
    std::mutex m;
    std::map<std::tuple<int, bool, int>, int> winner;
};
TuneCache &tune_cache()
{
    static TuneCache c;
    return c;
}

}  // namespace

int tune_size_class(int64_t local_nodes)
{
    // powers of two, clamped to [2^16, 2^26] local nodes
    int k = 16;
    while (k < 26 && (int64_t(1) << (k + 1)) <= local_nodes) ++k;
    return k;
}

hb_status tune_class_cached(int N, bool fp32, int64_t local_nodes, hipStream_t s, int *schedule)
{
    const int k = tune_size_class(local_nodes);
    const auto key = std::make_tuple(N, fp32, k);
    TuneCache &c = tune_cache();
    std::lock_guard<std::mutex> lock(c.m);
    auto it = c.winner.find(key);
    if (it == c.winner.end()) {
        hb_tune_result r{};
        hb_status st = tune_class(N, fp32, int64_t(1) << k, 20, &r, s);
        if (st) return st;
        it = c.winner.emplace(key, r.schedule).first;
    }
    if (ax_schedule(N, fp32) != it->second) set_ax_schedule(N, fp32, it->second);
    if (schedule) *schedule = it->second;
    return HB_OK;
}

}  // namespace hb
