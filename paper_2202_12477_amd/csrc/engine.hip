// Batched CG runner and the continuous-batching serving engine.
//
// BatchRunner keeps a changing set of independent CG solves on the device and
// advances all of them together (one operator launch per (degree, precision)
// class, one launch per vector/scalar step; see batch.hip).  Problems join
// between segments of iterations and leave as soon as they finish, so work
// that arrives while others run is overlapped with them.  A segment's launches
// can be replayed from a captured HIP graph, re-captured whenever the running
// set (and with it the work lists) changes.
//
// The engine puts a request queue in front of it: a request (box mesh, degree,
// lambda, forcing seed, tolerance) is admitted first-in first-out when a slot
// is free and its device footprint fits the memory budget; admission builds
// its mesh and forcing on the device; a finished request's solution is copied
// to host memory and its device memory is released for the next admission.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "solver.h"

namespace hb {

// ---------------------------------------------------------------------------
// BatchRunner
// ---------------------------------------------------------------------------
class BatchRunner {
  public:
    BatchRunner(int capacity, hipStream_t s) : cap_(capacity), s_(s) {}
    ~BatchRunner()
    {
        if (gexec_) (void)hipGraphExecDestroy(gexec_);
        if (cap_s_) (void)hipStreamDestroy(cap_s_);
        for (void *p : {(void *)probs_, (void *)states_, (void *)items_, (void *)plist_, (void *)norms_,
                        (void *)pwgs_, (void *)pslots_, (void *)pbar_})
            if (p) (void)hipFree(p);
        for (void *p : {(void *)h_probs_, (void *)h_states_, (void *)h_items_, (void *)h_plist_, (void *)h_norms_,
                        (void *)h_rho_, (void *)h_pwgs_, (void *)h_pslots_, (void *)h_perr_})
            if (p) (void)hipHostFree(p);
    }

    hb_status init()
    {
        slots_.resize(cap_);
        if (hipMalloc(&probs_, sizeof(BatchProb) * cap_) != hipSuccess ||
            hipMalloc(&states_, sizeof(CgState) * cap_) != hipSuccess ||
            hipMalloc(&plist_, sizeof(int32_t) * cap_) != hipSuccess ||
            hipMalloc(&norms_, sizeof(double) * cap_) != hipSuccess ||
            hipHostMalloc(&h_probs_, sizeof(BatchProb) * cap_, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&h_states_, sizeof(CgState) * cap_, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&h_plist_, sizeof(int32_t) * cap_, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&h_norms_, sizeof(double) * cap_, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&h_rho_, sizeof(double) * cap_, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HB_ERR_OUT_OF_MEMORY, "batch runner: table allocation failed");
        }
        return HB_OK;
    }

    // Run each step as one persistent launch when the running problems allow it
    // (persist.hip); otherwise, and for the steps where they do not, per-step launches.
    void use_persistent(bool on) { persistent_ = on; }
    // Steps run as one persistent launch so far.
    int persistent_steps() const { return persist_steps_; }

    int free_slot() const
    {
        for (int i = 0; i < cap_; ++i)
            if (!slots_[i].used) return i;
        return -1;
    }
    int running() const
    {
        int n = 0;
        for (const Slot &q : slots_) n += q.used && !q.finished;
        return n;
    }
    bool finished(int i) const { return slots_[i].used && slots_[i].finished; }
    hb_cg_result result(int i) const
    {
        hb_cg_result r = slots_[i].result;
        r.persistent_segments = slots_[i].psegments;
        return r;
    }
    void release(int i)
    {
        slots_[i] = Slot{};
        dirty_ = pdirty_ = true;
    }

    // Start a solve in slot i (enqueued; its first state is read at the next step).
    hb_status add(int i, hb_mesh_s *m, double lambda, const double *b, double *x, const hb_cg_opts &o)
    {
        const bool mixed = o.prec == HB_PREC_FP32_RR;
        hb_status st;
        if ((st = ensure_cg(m, o.max_iter, mixed))) return st;
        Slot &q = slots_[i];
        q = Slot{};
        q.used = true;
        q.starting = true;
        q.mesh = m;
        q.lambda = lambda;
        q.b = b;
        q.x = x;
        q.opts = o;
        q.mixed = mixed;
        const double rtol = o.fixed_iters ? -1.0 : o.rtol;
        const bool pc = o.precond == HB_PRECOND_JACOBI;
        if (pc && (st = ensure_jacobi(m, lambda, s_))) return st;
        m->cg.pc = pc;  // the first step (r0, z0 = inv r0, p0 = z0, r0.z0)
        st = cg_start(m, lambda, b, x, states_ + i, o.x0_zero, o.max_iter, rtol, mixed, s_);
        m->cg.pc = false;
        if (st) return st;
        // ||r0|| from the residual history (r0.r0 is not kept when the iteration
        // is preconditioned)
        HB_HIP(hipMemcpyAsync(h_rho_ + i, m->cg.hist, sizeof(double), hipMemcpyDeviceToHost, s_));
        CgWork &w = m->cg;
        BatchProb &P = h_probs_[i];
        P.map = m->map;
        P.geo = m->geo;
        P.geo32 = m->geo32;
        P.D = m->D;
        P.D32 = m->D32;
        P.lambda = lambda;
        P.x = x;
        P.r = w.r;
        P.p = w.p;
        P.Ap = w.Ap;
        P.Ap32 = w.Ap32;
        P.rho = w.rho;
        P.hist = w.hist;
        P.part_ax = w.part_ax;
        P.part_vec = w.part_vec;
        P.st = states_ + i;
        P.E = m->E;
        P.NG = m->NG;
        P.N = m->N;
        P.nx = m->desc.nx;
        P.ny = m->desc.ny;
        P.nz = m->desc.nz;
        P.dirichlet = (m->desc.flags & HB_MESH_DIRICHLET) ? 1 : 0;
        P.ax_tiles = ax_blocks(m, mixed);  // recomputed with the lists (schedule, precision)
        P.vec_chunks = static_cast<int32_t>((m->NG + kBatchChunk - 1) / kBatchChunk);
        P.use32 = mixed ? 1 : 0;
        P.inv = pc ? w.jinv : nullptr;
        q.rp.inv = P.inv;
        dirty_ = pdirty_ = true;
        return HB_OK;
    }

    // Advance the running problems, then handle the ones the device stopped
    // (finish, or replace the residual and resume).  Every problem advances
    // `iters` iterations times its quota multiplier: 1 with max_quota = 1;
    // otherwise a problem whose iteration costs at most 1/2^k of the costliest
    // running one's gets 2^k (capped at max_quota), so small problems are not
    // held to the large ones' pace.  Sub-iteration j launches only the problems
    // whose quota exceeds j: the lists are sorted by multiplier, so those are a
    // prefix of each list.
    hb_status step(int iters, int max_quota = 1)
    {
        hb_status st;
        if ((st = start_pending())) return st;
        std::vector<int> run;
        for (int i = 0; i < cap_; ++i)
            if (slots_[i].used && !slots_[i].finished) run.push_back(i);
        if (run.empty()) return HB_OK;
        max_quota = std::max(max_quota, 1);
        if (persistent_ && persist_eligible(run)) return step_persistent(run, iters, max_quota);
        // the lists depend on the running set, the quotas and the schedule
        // table (tile counts and order): rebuilt when any of them changed
        if ((dirty_ || max_quota != built_quota_ || ax_schedule_epoch() != built_epoch_) &&
            (st = build_lists(run, max_quota)))
            return st;
        if (graphs_) {
            hipGraphExec_t g = nullptr;
            if ((st = step_graph(iters, &g))) return st;
            HB_HIP(hipGraphLaunch(g, s_));
        } else if ((st = enqueue_step(iters, s_))) {
            return st;
        }
        return handle_stops(run);
    }

    // Replay each step's launches from a captured graph (rebuilt whenever the
    // lists or the step length change).
    void use_graphs(bool on) { graphs_ = on; }

  private:
    struct Slot {
        bool used = false, starting = false, finished = false, mixed = false;
        hb_mesh_s *mesh = nullptr;
        double lambda = 0.0;
        const double *b = nullptr;
        double *x = nullptr;
        hb_cg_opts opts{};
        Replacer rp;
        hb_cg_result result{};
        int psegments = 0;  // steps of this problem inside persistent launches
    };
    // Cumulative list length after the problems whose multiplier is >= mult.
    struct Level {
        int mult, count;
    };
    struct Class {
        int N, sched;
        bool fp32, dirichlet;
        int off;
        const void *D;              // the class's derivative matrix (any of its meshes)
        std::vector<Level> levels;  // items of the class's problems, by multiplier (descending)
    };
    // The persistent launch takes problems of the degrees it is compiled for, on
    // boxes of one kind (plain or Dirichlet), at most one per workgroup the
    // device holds.
    bool persist_eligible(const std::vector<int> &run) const
    {
        const int cap = persist_capacity();
        if (cap == 0 || static_cast<int>(run.size()) > cap) return false;
        for (int i : run) {
            const BatchProb &P = h_probs_[i];
            if (!persist_degree(P.N) || P.dirichlet != h_probs_[run.front()].dirichlet) return false;
        }
        return true;
    }

    // Per-problem bytes streamed by one iteration: operator (60 N_L FP64,
    // 32 N_L FP32) plus vectors (~88 N_G).
    double iteration_cost(int i) const
    {
        const BatchProb &P = h_probs_[i];
        const double nl = static_cast<double>(P.E) * (P.N + 1) * (P.N + 1) * (P.N + 1);
        return (P.use32 ? 32.0 : 60.0) * nl + 88.0 * static_cast<double>(P.NG);
    }

    // Quota multipliers (as build_lists) and the workgroups of each problem in
    // the persistent launch: one each, the rest of the device's workgroups in
    // proportion to the bytes each problem streams during the launch, each
    // capped by its operator tiles and by its partial-sum arrays.
    hb_status build_persist(const std::vector<int> &run, int max_quota)
    {
        HB_HIP(hipStreamSynchronize(s_));  // earlier launches may still read the tables
        const int cap = persist_capacity();
        if (!pwgs_) {
            if (hipMalloc(&pwgs_, sizeof(PersistWg) * cap) != hipSuccess ||
                hipMalloc(&pslots_, sizeof(PersistSlot) * cap_) != hipSuccess ||
                hipMalloc(&pbar_, sizeof(uint32_t) * cap_ + sizeof(int32_t)) != hipSuccess ||
                hipHostMalloc(&h_pwgs_, sizeof(PersistWg) * cap, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc(&h_pslots_, sizeof(PersistSlot) * cap_, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc(&h_perr_, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return fail(HB_ERR_OUT_OF_MEMORY, "batch runner: persistent launch tables");
            }
        }
        double wmax = 0.0, total = 0.0;
        for (int i : run) wmax = std::max(wmax, iteration_cost(i));
        mult_.assign(cap_, 1);
        for (int i : run) {
            int m = 1;
            while (m * 2 <= max_quota && iteration_cost(i) * (m * 2) <= wmax) m *= 2;
            mult_[i] = m;
            total += iteration_cost(i) * m;
        }
        std::vector<int> nwg(cap_, 0), top(cap_, 0);
        int used = 0;
        for (int i : run) {
            const BatchProb &P = h_probs_[i];
            const int64_t vec_len = std::max<int64_t>(3 * vec_blocks(P.NG), 2 * ((P.NG + kBatchChunk - 1) / kBatchChunk));
            const int64_t lanes = (P.NG + kPersistThreads - 1) / kPersistThreads;
            top[i] = static_cast<int>(std::max<int64_t>(
                1, std::min<int64_t>({persist_tiles(P.N, P.E), vec_len / 2, lanes})));
            nwg[i] = 1;
            ++used;
        }
        // the remaining workgroups, one at a time to the problem with the most bytes per workgroup
        while (used < cap) {
            int best = -1;
            double best_load = 0.0;
            for (int i : run) {
                if (nwg[i] >= top[i]) continue;
                const double load = iteration_cost(i) * mult_[i] / nwg[i];
                if (load > best_load) {
                    best_load = load;
                    best = i;
                }
            }
            if (best < 0) break;
            ++nwg[best];
            ++used;
        }
        int k = 0;
        for (int i : run) {
            const BatchProb &P = h_probs_[i];
            PersistSlot &sl = h_pslots_[i];
            sl.walk = persist_walk(P.N, P.nx, P.ny, P.nz);
            sl.tiles = persist_tiles(P.N, P.E);
            sl.nwg = nwg[i];
            sl.iters = 0;
            sl.pad = 0;
            for (int r = 0; r < nwg[i]; ++r) h_pwgs_[k++] = PersistWg{i, r};
        }
        persist_nwg_ = k;
        (void)total;
        HB_HIP(hipMemcpyAsync(probs_, h_probs_, sizeof(BatchProb) * cap_, hipMemcpyHostToDevice, s_));
        HB_HIP(hipMemcpyAsync(pwgs_, h_pwgs_, sizeof(PersistWg) * k, hipMemcpyHostToDevice, s_));
        pquota_ = max_quota;
        pdirty_ = false;
        return HB_OK;
    }

    // One step as one persistent launch: every running problem advances
    // `iters` iterations times its quota multiplier.
    hb_status step_persistent(const std::vector<int> &run, int iters, int max_quota)
    {
        hb_status st;
        if ((pdirty_ || max_quota != pquota_) && (st = build_persist(run, max_quota))) return st;
        for (int i : run) h_pslots_[i].iters = iters * mult_[i];
        HB_HIP(hipMemcpyAsync(pslots_, h_pslots_, sizeof(PersistSlot) * cap_, hipMemcpyHostToDevice, s_));
        int32_t *err = reinterpret_cast<int32_t *>(pbar_ + cap_);
        HB_HIP(hipMemsetAsync(pbar_, 0, sizeof(uint32_t) * cap_ + sizeof(int32_t), s_));
        if ((st = launch_batch_persistent(h_probs_[run.front()].dirichlet != 0, pwgs_, persist_nwg_, pslots_, probs_,
                                          pbar_, err, s_)))
            return st;
        HB_HIP(hipMemcpyAsync(h_perr_, err, sizeof(int32_t), hipMemcpyDeviceToHost, s_));
        ++persist_steps_;
        for (int i : run) ++slots_[i].psegments;
        if ((st = handle_stops(run))) return st;  // synchronises the stream
        if (*h_perr_)
            return fail(HB_ERR_DEVICE, "persistent batch: a barrier among a problem's workgroups timed out");
        return HB_OK;
    }

    // The launches of one step: `iters` iterations of every running problem
    // (times its quota multiplier), on stream s.
    hb_status enqueue_step(int iters, hipStream_t s)
    {
        hb_status st;
        const int64_t sub_iters = static_cast<int64_t>(iters) * top_mult_;
        for (int64_t j = 0; j < sub_iters; ++j) {
            const int need = static_cast<int>(j / iters) + 1;  // multiplier a problem needs to run sub-iteration j
            for (const Class &c : classes_) {
                const int n = count_at(c.levels, need);
                if (n > 0 && (st = launch_batch_ax(c.N, c.sched, c.D, c.fp32, c.dirichlet, items_ + c.off, n, probs_, s)))
                    return st;
            }
            const int nrun = count_at(run_levels_, need), nvec = count_at(vec_levels_, need);
            if ((st = launch_batch_alpha(plist_, nrun, probs_, s)) ||
                (st = launch_batch_residual(items_ + vec_off_, nvec, probs_, s)) ||
                (st = launch_batch_beta(plist_, nrun, probs_, s)) ||
                (st = launch_batch_update(items_ + vec_off_, nvec, probs_, s)))
                return st;
        }
        return HB_OK;
    }

    // The step as an executable graph: the cached one if the lists and the
    // step length are unchanged, else captured on a private stream (every
    // launch of a step is a kernel, so the graph holds kernel nodes only).
    hb_status step_graph(int iters, hipGraphExec_t *out)
    {
        if (gexec_ && g_iters_ == iters && g_version_ == lists_version_) {
            *out = gexec_;
            return HB_OK;
        }
        if (!cap_s_) HB_HIP(hipStreamCreateWithFlags(&cap_s_, hipStreamNonBlocking));
        HB_HIP(hipStreamBeginCapture(cap_s_, hipStreamCaptureModeThreadLocal));
        const hb_status st = enqueue_step(iters, cap_s_);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(cap_s_, &graph);
        if (st != HB_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return st != HB_OK ? st : hip_fail(e, "hipStreamEndCapture");
        }
        if (gexec_) {
            // the same launches with other lists and grids (a problem retired or
            // joined, the class set unchanged): update the executable graph in
            // place instead of instantiating a new one
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult why{};
            if (hipGraphExecUpdate(gexec_, graph, &bad, &why) == hipSuccess && why == hipGraphExecUpdateSuccess) {
                (void)hipGraphDestroy(graph);
                ++g_updates_;
                g_iters_ = iters;
                g_version_ = lists_version_;
                *out = gexec_;
                return HB_OK;
            }
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(gexec_);
            gexec_ = nullptr;
        }
        const hipError_t ei = hipGraphInstantiate(&gexec_, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            gexec_ = nullptr;
            return hip_fail(ei, "hipGraphInstantiate");
        }
        g_iters_ = iters;
        g_version_ = lists_version_;
        *out = gexec_;
        return HB_OK;
    }

    static int count_at(const std::vector<Level> &levels, int need)
    {
        int n = 0;
        for (const Level &l : levels) {
            if (l.mult < need) break;
            n = l.count;
        }
        return n;
    }

    // First state of newly added problems (one read-back for all of them).
    hb_status start_pending()
    {
        bool any = false;
        for (const Slot &q : slots_) any = any || (q.used && q.starting);
        if (!any) return HB_OK;
        HB_HIP(hipMemcpyAsync(h_states_, states_, sizeof(CgState) * cap_, hipMemcpyDeviceToHost, s_));
        HB_HIP(hipStreamSynchronize(s_));
        for (int i = 0; i < cap_; ++i) {
            Slot &q = slots_[i];
            if (!q.used || !q.starting) continue;
            q.starting = false;
            const CgState &hs = h_states_[i];
            if (q.mixed) {
                q.rp.start(&q.opts, h_rho_[i], std::sqrt(hs.bb), hs.done != 0,
                           static_cast<hb_status>(hs.status));
                if (q.rp.finished) {
                    finish(i, hs.iters);
                } else {
                    hb_status st = launch_cg_resume(states_ + i, q.rp.threshold(), s_);
                    if (st) return st;
                }
            } else if (hs.done) {
                q.result = hb_cg_result{};
                q.result.status = hs.status;
                q.result.res0 = q.result.res = h_rho_[i];
                q.result.bnorm = std::sqrt(hs.bb);
                q.finished = true;
            }
        }
        dirty_ = pdirty_ = true;
        return HB_OK;
    }

    hb_status grow_items(size_t n)
    {
        if (n <= items_cap_) return HB_OK;
        size_t cap = std::max<size_t>(n, items_cap_ * 2);
        if (items_) (void)hipFree(items_);
        if (h_items_) (void)hipHostFree(h_items_);
        items_ = nullptr;
        h_items_ = nullptr;
        items_cap_ = 0;
        if (hipMalloc(&items_, sizeof(WorkItem) * cap) != hipSuccess ||
            hipHostMalloc(&h_items_, sizeof(WorkItem) * cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(HB_ERR_OUT_OF_MEMORY, "batch runner: work list allocation failed");
        }
        items_cap_ = cap;
        return HB_OK;
    }

    // Work lists of the running problems: operator items grouped by (degree,
    // precision), vector chunks and the problem list, each ordered by quota
    // multiplier (descending).  A problem's cost per iteration is its bytes
    // streamed: operator (60 N_L FP64, 32 N_L FP32) plus vectors (~88 N_G).
    hb_status build_lists(std::vector<int> run, int max_quota)
    {
        // enqueued kernels may still read the previous lists and copies the
        // host staging: wait before rewriting either
        HB_HIP(hipStreamSynchronize(s_));
        built_epoch_ = ax_schedule_epoch();  // read before the schedules themselves
        ++lists_version_;
        // each class's schedule: the table's, unmerged where its problems' rows
        // leave the merged tiles sparse
        int sched[kMaxN + 1][2];
        int64_t elems[kMaxN + 1][2] = {}, tiles[kMaxN + 1][2] = {};
        for (int N = 1; N <= kMaxN; ++N)
            for (int f = 0; f < 2; ++f) sched[N][f] = ax_schedule(N, f != 0);
        for (int i : run) {
            const BatchProb &P = h_probs_[i];
            const int f = P.use32 != 0;
            elems[P.N][f] += P.E;
            tiles[P.N][f] += ax_grid_for(P.N, P.E, P.nx, P.ny, P.nz, sched[P.N][f]);
        }
        for (int N = 1; N <= kMaxN; ++N)
            for (int f = 0; f < 2; ++f) sched[N][f] = unmerged_if_sparse(N, f != 0, sched[N][f], elems[N][f], tiles[N][f]);
        // operator tiles under the schedule of each problem's class (sets the
        // list lengths, so before sizing the lists)
        for (int i : run) {
            BatchProb &P = h_probs_[i];
            P.ax_tiles = ax_grid_for(P.N, P.E, P.nx, P.ny, P.nz, sched[P.N][P.use32 != 0]);
        }
        size_t need = 0;
        for (int i : run) need += h_probs_[i].ax_tiles + h_probs_[i].vec_chunks;
        hb_status st;
        if ((st = grow_items(need))) return st;
        auto cost = [&](int i) {
            const BatchProb &P = h_probs_[i];
            const double nl = static_cast<double>(P.E) * (P.N + 1) * (P.N + 1) * (P.N + 1);
            return (P.use32 ? 32.0 : 60.0) * nl + 88.0 * static_cast<double>(P.NG);
        };
        HB_HIP(hipMemcpyAsync(probs_, h_probs_, sizeof(BatchProb) * cap_, hipMemcpyHostToDevice, s_));
        double wmax = 0.0;
        for (int i : run) wmax = std::max(wmax, cost(i));
        mult_.assign(cap_, 1);
        for (int i : run) {
            int m = 1;
            while (m * 2 <= max_quota && cost(i) * (m * 2) <= wmax) m *= 2;
            mult_[i] = m;
        }
        std::stable_sort(run.begin(), run.end(), [&](int a, int b) { return mult_[a] > mult_[b]; });
        top_mult_ = mult_[run.front()];
        classes_.clear();
        int nit = 0;
        for (int N = 1; N <= kMaxN; ++N)
            for (int k = 0; k < 4; ++k) {
                const int f = k & 1, dir = k >> 1;
                Class c{N, sched[N][f], f != 0, dir != 0, nit, nullptr, {}};
                for (int i : run) {
                    const BatchProb &P = h_probs_[i];
                    if (P.N != N || P.use32 != f || P.dirichlet != dir) continue;
                    c.D = f ? static_cast<const void *>(P.D32) : static_cast<const void *>(P.D);
                    // the single-problem launch's tile order (locality of the shared lines)
                    const TileWalk w = ax_walk_for(P.N, P.nx, P.ny, P.nz, c.sched);
                    for (int t = 0; t < P.ax_tiles; ++t)
                        h_items_[nit++] = WorkItem{i, static_cast<int32_t>(walk_tile(w, static_cast<uint32_t>(t)))};
                    c.levels.push_back(Level{mult_[i], nit - c.off});
                }
                if (!c.levels.empty()) classes_.push_back(std::move(c));
            }
        vec_off_ = nit;
        vec_levels_.clear();
        run_levels_.clear();
        for (size_t k = 0; k < run.size(); ++k) {
            const int i = run[k];
            for (int c = 0; c < h_probs_[i].vec_chunks; ++c) h_items_[nit++] = WorkItem{i, c};
            vec_levels_.push_back(Level{mult_[i], nit - vec_off_});
            run_levels_.push_back(Level{mult_[i], static_cast<int>(k) + 1});
            h_plist_[k] = i;
        }
        const int nrun = static_cast<int>(run.size());
        HB_HIP(hipMemcpyAsync(items_, h_items_, sizeof(WorkItem) * nit, hipMemcpyHostToDevice, s_));
        HB_HIP(hipMemcpyAsync(plist_, h_plist_, sizeof(int32_t) * nrun, hipMemcpyHostToDevice, s_));
        built_quota_ = max_quota;
        dirty_ = false;
        pdirty_ = true;  // mult_ was rewritten
        return HB_OK;
    }

    hb_status handle_stops(const std::vector<int> &run)
    {
        HB_HIP(hipMemcpyAsync(h_states_, states_, sizeof(CgState) * cap_, hipMemcpyDeviceToHost, s_));
        HB_HIP(hipStreamSynchronize(s_));
        std::vector<int> replaced, done64;
        hb_status st;
        for (int i : run) {
            Slot &q = slots_[i];
            const CgState &hs = h_states_[i];
            const bool stopped = hs.done || hs.pending || hs.iters >= q.opts.max_iter;
            if (!stopped) continue;
            if (!q.mixed) {
                done64.push_back(i);
                HB_HIP(hipMemcpyAsync(h_norms_ + i, q.mesh->cg.hist + hs.iters, sizeof(double),
                                      hipMemcpyDeviceToHost, s_));
                continue;
            }
            bool enq = false;
            if ((st = q.rp.replace(q.mesh, q.lambda, q.b, q.x, states_ + i, hs, norms_ + i, s_, &enq))) return st;
            if (enq) {
                replaced.push_back(i);
                HB_HIP(hipMemcpyAsync(h_norms_ + i, norms_ + i, sizeof(double), hipMemcpyDeviceToHost, s_));
            } else {
                finish(i, hs.iters);
            }
        }
        if (replaced.empty() && done64.empty()) return HB_OK;
        HB_HIP(hipStreamSynchronize(s_));
        for (int i : done64) {
            Slot &q = slots_[i];
            const CgState &hs = h_states_[i];
            q.result = hb_cg_result{};
            q.result.iters = hs.iters;
            q.result.status = hs.status;
            q.result.res0 = h_rho_[i];
            q.result.res = h_norms_[i];
            q.result.bnorm = std::sqrt(hs.bb);
            q.finished = true;
            dirty_ = pdirty_ = true;
        }
        for (int i : replaced) {
            Slot &q = slots_[i];
            const bool was32 = q.rp.use32;
            if ((st = q.rp.decide(q.mesh, states_ + i, h_states_[i].iters, h_norms_[i], nullptr, s_))) return st;
            if (q.rp.finished) finish(i, h_states_[i].iters);
            if (was32 != q.rp.use32) {
                h_probs_[i].use32 = q.rp.use32 ? 1 : 0;
                dirty_ = pdirty_ = true;
            }
        }
        return HB_OK;
    }

    void finish(int i, int iters)
    {
        Slot &q = slots_[i];
        q.rp.fill(&q.result, iters);
        q.finished = true;
        dirty_ = pdirty_ = true;
    }

    int cap_;
    hipStream_t s_;
    std::vector<Slot> slots_;
    BatchProb *probs_ = nullptr, *h_probs_ = nullptr;
    CgState *states_ = nullptr, *h_states_ = nullptr;
    WorkItem *items_ = nullptr, *h_items_ = nullptr;
    size_t items_cap_ = 0;
    int32_t *plist_ = nullptr, *h_plist_ = nullptr;
    double *norms_ = nullptr, *h_norms_ = nullptr, *h_rho_ = nullptr;
    std::vector<Class> classes_;
    std::vector<Level> vec_levels_, run_levels_;
    std::vector<int> mult_;
    int vec_off_ = 0, top_mult_ = 1, built_quota_ = 0, built_epoch_ = -1;
    bool dirty_ = true;
    // persistent launches
    bool persistent_ = false, pdirty_ = true;  // pdirty_: the persistent tables are stale
    int pquota_ = 0;
    PersistWg *pwgs_ = nullptr, *h_pwgs_ = nullptr;
    PersistSlot *pslots_ = nullptr, *h_pslots_ = nullptr;
    uint32_t *pbar_ = nullptr;  // a barrier counter per slot, then the error flag
    int32_t *h_perr_ = nullptr;
    int persist_nwg_ = 0, persist_steps_ = 0;
    // graph replay of steps
    bool graphs_ = false;
    hipStream_t cap_s_ = nullptr;
    hipGraphExec_t gexec_ = nullptr;
    int g_iters_ = 0;
    int g_updates_ = 0;  // executable graphs updated in place (instead of instantiated anew)
    uint64_t lists_version_ = 0, g_version_ = 0;
};

// ---------------------------------------------------------------------------
// Serving engine
// ---------------------------------------------------------------------------

// Device bytes one request holds while it is admitted (mesh, FP32 copy,
// CG workspace, b and x, histories).
size_t request_footprint(const hb_mesh_desc &d, int prec, int max_iter, bool jacobi)
{
    const double n1 = d.N + 1.0;
    const double NL = (double)d.nx * d.ny * d.nz * n1 * n1 * n1;
    const double NG = static_cast<double>(box_global_nodes(d));
    const bool mixed = prec == HB_PREC_FP32_RR;
    double bytes = NL * (4.0 + 8.0 * kGeo) + (mixed ? NL * 4.0 * kGeo : 0.0);  // map, geometry
    bytes += NG * (8.0 * 3 + (mixed ? 4.0 : 0.0));                               // r, p, Ap (+ FP32 Ap)
    bytes += NG * 16.0;                                                          // b, x
    if (jacobi) bytes += NG * 8.0;                                               // 1 / diag(A)
    bytes += 16.0 * (max_iter + 1.0) + 8.0 * (NL / 16.0 + NG / 512.0) + 4096.0;  // histories, partials, small
    return static_cast<size_t>(bytes);
}

}  // namespace hb

struct hb_engine_s {
    struct Request {
        uint64_t ticket;
        hb_mesh_desc desc;
        double lambda;
        uint64_t rhs_seed;
        double rtol;
        size_t footprint;
    };
    struct Active {
        Request req;
        hb_mesh mesh = nullptr;
        double *b = nullptr, *x = nullptr;
        int slot = -1;
    };
    struct Done {
        hb_cg_result result;
        std::vector<double> x;
    };
    hb_engine_opts opts;
    hipStream_t s;
    std::unique_ptr<hb::BatchRunner> runner;
    std::deque<Request> queue;
    std::vector<Active> active;
    std::unordered_map<uint64_t, Done> done;
    size_t used = 0;
    uint64_t next_ticket = 1;
    double admit_s = 0.0, iterate_s = 0.0, retire_s = 0.0;  // host wall time per phase of the steps

    void release(Active &a)
    {
        if (a.b) (void)hipFree(a.b);
        if (a.x) (void)hipFree(a.x);
        if (a.mesh) hb_mesh_destroy(a.mesh);
        used -= a.req.footprint;
        a = Active{};
    }
};

using namespace hb;

extern "C" {

hb_status hb_batch_solve(int32_t nprob, const hb_mesh *meshes, const double *lambdas, const double *const *dev_b,
                         double *const *dev_x, const hb_cg_opts *opts, hb_cg_result *results, void *stream)
{
    if (nprob < 0 || (nprob > 0 && (!meshes || !lambdas || !dev_b || !dev_x || !results)) || !opts)
        return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: null argument");
    if (opts->prec != HB_PREC_FP64 && opts->prec != HB_PREC_FP32_RR)
        return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: precision must be HB_PREC_FP64 or HB_PREC_FP32_RR");
    const bool mixed = opts->prec == HB_PREC_FP32_RR;
    const bool fixed = opts->fixed_iters != 0;
    if (opts->max_iter < 0) return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: max_iter must be >= 0");
    if (mixed && fixed) return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: mixed precision needs a tolerance");
    if (!fixed && !(opts->rtol >= 0.0)) return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: rtol must be >= 0");
    if (opts->graph_k < 0 || opts->graph_k > 4096)
        return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: graph_k must be in [0, 4096]");
    if (opts->precond != HB_PRECOND_NONE && opts->precond != HB_PRECOND_JACOBI)
        return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: unknown preconditioner");
    if (opts->precond == HB_PRECOND_JACOBI && opts->prec == HB_PREC_FP32_IR)
        return fail(HB_ERR_INVALID_ARG,
                    "hb_batch_solve: the Jacobi preconditioner is available with HB_PREC_FP64 and HB_PREC_FP32_RR only");
    for (int i = 0; i < nprob; ++i) {
        if (!meshes[i] || !dev_b[i] || !dev_x[i] || dev_b[i] == dev_x[i])
            return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: problem " + std::to_string(i) + ": bad pointers");
        if (!(lambdas[i] > 0.0) || !std::isfinite(lambdas[i]))
            return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: problem " + std::to_string(i) + ": lambda must be > 0");
        if (meshes[i]->desc.flags & HB_MESH_GATHER)
            return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: two-phase (HB_MESH_GATHER) meshes are solved one at a time");
        if (mixed && !meshes[i]->geo32)
            return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: problem " + std::to_string(i) + " has no FP32 data");
        for (int k = 0; k < i; ++k)
            if (meshes[k] == meshes[i])
                return fail(HB_ERR_INVALID_ARG, "hb_batch_solve: a mesh appears twice (its workspace is per mesh)");
    }
    if (nprob == 0) return HB_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hb_status st;
    if (opts->autotune) {
        // each (degree, operator precision) class at its total local nodes
        std::map<int, int64_t> nodes;
        for (int i = 0; i < nprob; ++i) nodes[meshes[i]->N] += meshes[i]->NL;
        for (const auto &kv : nodes)
            if ((st = tune_class_cached(kv.first, mixed, kv.second, s, nullptr))) return st;
    }
    BatchRunner runner(nprob, s);
    if ((st = runner.init())) return st;
    for (int i = 0; i < nprob; ++i)
        if ((st = runner.add(i, meshes[i], lambdas[i], dev_b[i], dev_x[i], *opts))) return st;
    int chunk = fixed ? std::max(opts->max_iter, 1) : (opts->check_every > 0 ? opts->check_every : 25);
    if (opts->graph_k > 0) {
        chunk = fixed ? std::min(chunk, opts->graph_k) : opts->graph_k;
        runner.use_graphs(true);
    }
    runner.use_persistent(opts->persistent != 0);
    do {
        if ((st = runner.step(chunk))) return st;
    } while (runner.running() > 0);
    hb_status worst = HB_OK;
    for (int i = 0; i < nprob; ++i) {
        results[i] = runner.result(i);
        if (worst == HB_OK && results[i].status != HB_OK) worst = static_cast<hb_status>(results[i].status);
    }
    return worst;
}

hb_status hb_engine_footprint(const hb_mesh_desc *desc, int32_t prec, int32_t max_iter, size_t *bytes)
{
    if (!desc || !bytes || max_iter < 0) return fail(HB_ERR_INVALID_ARG, "hb_engine_footprint: bad arguments");
    *bytes = request_footprint(*desc, prec, max_iter, false);
    return HB_OK;
}

hb_status hb_engine_create(const hb_engine_opts *opts, void *stream, hb_engine *out)
{
    if (out) *out = nullptr;
    if (!opts || !out) return fail(HB_ERR_INVALID_ARG, "hb_engine_create: null argument");
    if (opts->max_slots < 1 || opts->hbm_budget == 0 || opts->max_iter < 1 ||
        (opts->prec != HB_PREC_FP64 && opts->prec != HB_PREC_FP32_RR) ||
        (opts->precond != HB_PRECOND_NONE && opts->precond != HB_PRECOND_JACOBI))
        return fail(HB_ERR_INVALID_ARG, "hb_engine_create: bad options");

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(HB_ERR_DEVICE, "no HIP device available");
    }
    hb_engine_s *e = new (std::nothrow) hb_engine_s();
    if (!e) return fail(HB_ERR_OUT_OF_MEMORY, "hb_engine_create: host allocation failed");
    e->opts = *opts;
    e->s = static_cast<hipStream_t>(stream);
    e->runner.reset(new (std::nothrow) BatchRunner(opts->max_slots, e->s));
    if (e->runner) e->runner->use_graphs(opts->graphs != 0);
    e->active.resize(opts->max_slots);
    hb_status st = e->runner ? e->runner->init() : fail(HB_ERR_OUT_OF_MEMORY, "hb_engine_create: host allocation");
    if (st) {
        delete e;
        return st;
    }
    *out = e;
    return HB_OK;
}

hb_status hb_engine_destroy(hb_engine e)
{
    if (!e) return HB_OK;
    (void)hipStreamSynchronize(e->s);
    for (hb_engine_s::Active &a : e->active)
        if (a.mesh) e->release(a);
    delete e;
    return HB_OK;
}

hb_status hb_engine_submit(hb_engine e, const hb_mesh_desc *desc, double lambda, uint64_t rhs_seed, double rtol,
                           uint64_t *ticket)
{
    if (!e || !desc || !ticket) return fail(HB_ERR_INVALID_ARG, "hb_engine_submit: null argument");
    if (desc->N < 1 || desc->N > kMaxN || desc->nx < 1 || desc->ny < 1 || desc->nz < 1 ||
        !(desc->jitter >= 0.0 && desc->jitter < 0.5) || (desc->mass != HB_MASS_GWJ && desc->mass != HB_MASS_INVDEG))
        return fail(HB_ERR_INVALID_ARG, "hb_engine_submit: bad mesh descriptor");
    if (desc->flags & HB_MESH_GATHER)
        return fail(HB_ERR_INVALID_ARG, "hb_engine_submit: the engine runs the fused operator (no HB_MESH_GATHER)");
    if ((desc->flags & HB_MESH_DIRICHLET) &&
        ((int64_t)desc->nx * desc->N < 2 || (int64_t)desc->ny * desc->N < 2 || (int64_t)desc->nz * desc->N < 2))
        return fail(HB_ERR_INVALID_ARG, "hb_engine_submit: a Dirichlet box needs interior nodes (n*N >= 2)");
    if (!(lambda > 0.0) || !std::isfinite(lambda) || !(rtol > 0.0))
        return fail(HB_ERR_INVALID_ARG, "hb_engine_submit: lambda and rtol must be > 0");
    const size_t fp = request_footprint(*desc, e->opts.prec, e->opts.max_iter, e->opts.precond == HB_PRECOND_JACOBI);
    if (fp > e->opts.hbm_budget)
        return fail(HB_ERR_BUDGET, "hb_engine_submit: the request needs " + std::to_string(fp) +
                                       " device bytes, more than the whole budget");
    hb_engine_s::Request r{e->next_ticket++, *desc, lambda, rhs_seed, rtol, fp};
    r.desc.flags = (desc->flags & HB_MESH_DIRICHLET) | (e->opts.prec == HB_PREC_FP32_RR ? HB_MESH_FP32 : 0);
    e->queue.push_back(r);
    *ticket = r.ticket;
    return HB_OK;
}

hb_status hb_engine_step(hb_engine e, int32_t iters, hb_engine_info *info)
{
    if (!e) return fail(HB_ERR_INVALID_ARG, "hb_engine_step: null engine");
    hb_status st;
    using clock = std::chrono::steady_clock;
    auto since = [](clock::time_point t0) { return std::chrono::duration<double>(clock::now() - t0).count(); };
    auto t0 = clock::now();
    // admission: first in, first out, while a slot is free and the footprint fits
    while (!e->queue.empty()) {
        const hb_engine_s::Request &r = e->queue.front();
        const int slot = e->runner->free_slot();
        if (slot < 0 || e->used + r.footprint > e->opts.hbm_budget) break;
        hb_engine_s::Active a;
        a.req = r;
        a.slot = slot;
        e->used += r.footprint;
        if ((st = hb_mesh_create(&r.desc, e->s, &a.mesh))) {
            e->release(a);
            return st;
        }
        if (e->opts.autotune) {
            // the class's running local nodes with this request
            int64_t nodes = a.mesh->NL;
            for (const hb_engine_s::Active &o : e->active)
                if (o.mesh && o.mesh->N == a.mesh->N) nodes += o.mesh->NL;
            if ((st = tune_class_cached(a.mesh->N, e->opts.prec == HB_PREC_FP32_RR, nodes, e->s, nullptr))) {
                e->release(a);
                return st;
            }
        }
        const int64_t NG = a.mesh->NG;
        size_t tally = 0;
        if ((st = dev_alloc(&a.b, NG, &tally)) || (st = dev_alloc(&a.x, NG, &tally)) ||
            (st = launch_rhs(NG, r.rhs_seed, a.b, e->s))) {
            e->release(a);
            return st;
        }
        hb_cg_opts o{};
        o.max_iter = e->opts.max_iter;
        o.fixed_iters = 0;
        o.rtol = r.rtol;
        o.x0_zero = 1;
        o.prec = e->opts.prec;
        o.inner_rtol = e->opts.inner_rtol;
        o.precond = e->opts.precond;
        if ((st = e->runner->add(slot, a.mesh, r.lambda, a.b, a.x, o))) {
            e->release(a);
            return st;
        }
        e->active[slot] = a;
        e->queue.pop_front();
    }
    e->admit_s += since(t0);
    t0 = clock::now();
    const int k = iters > 0 ? iters : (e->opts.iters_per_step > 0 ? e->opts.iters_per_step : 25);
    if ((st = e->runner->step(k, e->opts.max_quota > 0 ? e->opts.max_quota : 64))) return st;
    e->iterate_s += since(t0);
    t0 = clock::now();
    // retire finished requests: solution to host memory, device memory released
    for (int i = 0; i < e->opts.max_slots; ++i) {
        hb_engine_s::Active &a = e->active[i];
        if (!a.mesh || !e->runner->finished(i)) continue;
        hb_engine_s::Done d;
        d.result = e->runner->result(i);
        d.x.resize(a.mesh->NG);
        HB_HIP(hipMemcpyAsync(d.x.data(), a.x, sizeof(double) * a.mesh->NG, hipMemcpyDeviceToHost, e->s));
        HB_HIP(hipStreamSynchronize(e->s));
        e->done.emplace(a.req.ticket, std::move(d));
        e->runner->release(i);
        e->release(a);
    }
    e->retire_s += since(t0);
    if (info) {
        info->running = e->runner->running();
        info->queued = static_cast<int32_t>(e->queue.size());
        info->completed = static_cast<int32_t>(e->done.size());
        info->reserved = 0;
        info->used_bytes = e->used;
        info->admit_s = e->admit_s;
        info->iterate_s = e->iterate_s;
        info->retire_s = e->retire_s;
    }
    return HB_OK;
}

hb_status hb_engine_poll(hb_engine e, uint64_t ticket, int32_t *done, double *host_x, hb_cg_result *result)
{
    if (!e || !done) return fail(HB_ERR_INVALID_ARG, "hb_engine_poll: null argument");
    auto it = e->done.find(ticket);
    if (it == e->done.end()) {
        *done = 0;
        return HB_OK;
    }
    *done = 1;
    if (host_x) std::memcpy(host_x, it->second.x.data(), sizeof(double) * it->second.x.size());
    if (result) *result = it->second.result;
    e->done.erase(it);
    return HB_OK;
}

}  // extern "C"
