// Host-side CG drivers shared by the C ABI, the batched runner and the
// serving engine (definitions in solver.hip).
#pragma once

#include <algorithm>
#include <cmath>

#include "common.h"

namespace hb {

void free_cg(hb_mesh_s *m);
// Size the CG workspace of a mesh for an iteration cap (mixed: the FP32
// operator output; refine: the buffers of the restarted refinement).
hb_status ensure_cg(hb_mesh_s *m, int max_iter, bool mixed, bool refine = false);
// 1 / diag(A) for the Jacobi preconditioner, computed for this lambda if needed.
hb_status ensure_jacobi(hb_mesh_s *m, double lambda, hipStream_t s);
hb_status read_state(CgWork &w, hipStream_t s);
hb_status read_norm(CgWork &w, hipStream_t s, double *out);
hb_status apply_op(const hb_mesh_s *m, double l, const double *x, double *y, double *part, CgState *st, hipStream_t s);
hb_status apply_op(const hb_mesh_s *m, double l, const double *x, float *y, double *part, CgState *st, hipStream_t s);
// One CG iteration (Algorithm 1, loop body) on the workspace w: the operator
// step with p.Ap, alpha, the residual step with r.r, beta, the update.
template <typename TAp>
hb_status enqueue_iteration(hb_mesh_s *m, CgWork &w, double lambda, double *x, TAp *Ap, hipStream_t s);
template <typename TAp>
hb_status cg_iterate(hb_mesh_s *m, double lambda, double *x, TAp *Ap, int max_iter, bool fixed, int check_every,
                     hipStream_t s);
template <typename TAp>
hb_status run_cg(hb_mesh_s *m, double lambda, const double *b, double *x, TAp *Ap, int x0_zero, int max_iter,
                 double rtol, int check_every, hipStream_t s);
hb_status true_residual_sq(hb_mesh_s *m, double lambda, const double *b, const double *x, hipStream_t s, double *out);
hb_status cg_start(hb_mesh_s *m, double lambda, const double *b, double *x, CgState *st, int x0_zero, int max_iter,
                   double rtol, bool mixed, hipStream_t s);
hb_status solve_replace(hb_mesh_s *m, double lambda, const double *b, double *x, const hb_cg_opts *opts,
                        hb_cg_result *result, double *hist, hipStream_t s);

// Host-side control of one residual-replacement solve (FP32 operator, FP64
// replacements).  After the device has stopped a segment of iterations (the
// recursive residual met the segment's threshold, the iteration cap, or a
// breakdown), `replace` recomputes r = b - A x with the FP64 operator on the
// stream and `decide` (after the norm has been read back) either finishes the
// solve or resumes it with the next threshold, switching to the FP64 operator
// for good if the true residual fell by less than a factor 2 since the last
// replacement.
struct Replacer {
    double eta = 1e-3, rtol = 0.0, bnorm = 0.0, ref = 0.0, res = 0.0, res0 = 0.0;
    int max_iter = 0, max_outer = 0, outer = 0, fp64_from = -1;
    bool use32 = true, finished = false, breakdown = false;
    const double *inv = nullptr;  // Jacobi: 1 / diag(A) (the replacement then also recomputes r.z)
    hb_status status = HB_ERR_NOT_CONVERGED;

    void start(const hb_cg_opts *o, double res0_, double bnorm_, bool already_done, hb_status st0)
    {
        eta = o->inner_rtol > 0.0 ? o->inner_rtol : 1e-3;
        rtol = o->rtol;
        max_iter = o->max_iter;
        max_outer = o->max_outer > 0 ? o->max_outer : 1000000;
        bnorm = bnorm_;
        res = ref = res0 = res0_;
        if (already_done) {
            finished = true;
            status = st0;
        }
    }
    double threshold() const { return use32 ? std::max(eta * ref, rtol * bnorm) : rtol * bnorm; }

    // Enqueue the replacement; returns true if one was enqueued.
    hb_status replace(hb_mesh_s *m, double lambda, const double *b, const double *x, CgState *st,
                      const CgState &hs, double *norm_out, hipStream_t s, bool *enqueued)
    {
        *enqueued = false;
        breakdown = hs.status == HB_ERR_BREAKDOWN;
        if (breakdown && !use32) {
            finished = true;
            status = HB_ERR_BREAKDOWN;
            return HB_OK;
        }
        CgWork &w = m->cg;
        hb_status e;
        if ((e = launch_zero(w.Ap, m->NG, s)) || (e = launch_ax(m, lambda, x, w.Ap, nullptr, nullptr, s)) ||
            (e = launch_cg_replace(m->NG, b, w.Ap, w.r, w, st, norm_out, inv, s)))
            return e;
        *enqueued = true;
        return HB_OK;
    }

    // After the replacement's squared norm `rr` is on the host.
    hb_status decide(hb_mesh_s *m, CgState *st, int iters, double rr, double *hist, hipStream_t s)
    {
        ++outer;
        res = std::sqrt(rr);
        if (hist && outer <= max_iter) hist[outer] = res;
        if (!std::isfinite(res)) {
            finished = true;
            status = HB_ERR_BREAKDOWN;
            return HB_OK;
        }
        if (res <= rtol * bnorm) {
            finished = true;
            status = HB_OK;
            return HB_OK;
        }
        if (iters >= max_iter || outer >= max_outer) {
            finished = true;
            status = HB_ERR_NOT_CONVERGED;
            return HB_OK;
        }
        if (use32 && (breakdown || res > 0.5 * ref)) {
            use32 = false;
            fp64_from = iters;
        }
        ref = res;
        CgWork &w = m->cg;
        hb_status e;
        // both operator outputs start the next segment at zero (w.Ap held A x)
        if ((e = launch_zero(w.Ap, m->NG, s)) || (e = launch_zero(w.Ap32, m->NG, s)) ||
            (e = launch_cg_resume(st, threshold(), s)))
            return e;
        return HB_OK;
    }

    void fill(hb_cg_result *r, int iters) const
    {
        if (!r) return;
        *r = hb_cg_result{};
        r->iters = iters;
        r->status = status;
        r->res0 = res0;
        r->res = res;
        r->bnorm = bnorm;
        r->outer_iters = outer;
        r->fp64_iters = fp64_from >= 0 ? iters - fp64_from : 0;
    }
};

}  // namespace hb
