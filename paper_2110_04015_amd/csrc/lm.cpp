// Levenberg-Marquardt outer loop (Sec. 4.1) over the library's own entry points:
// residuals and Jacobians of the nine-parameter camera on the device (k_lm.hip), the
// reduced camera system built once and updated in place, PCG or MCG for the damped
// normal equation, back-substitution, and the accept/reject damping rule.  The host
// reads back one scalar per iteration (F at the moved state) to decide.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <string>

#include "ba_internal.h"
#include "kernels.h"

using namespace ba;

namespace {

#define LMCHK(expr)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return set_error(BA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

ba_status check_scene(const ba_scene_desc *sc) {
    if (!sc) return set_error(BA_ERR_INVALID_ARG, "scene is NULL");
    if (sc->n_cams < 1 || sc->n_lms < 1 || sc->n_obs < 1)
        return set_error(BA_ERR_INVALID_ARG, "n_cams, n_lms and n_obs must be positive");
    if (!sc->obs_cam || !sc->obs_lm || !sc->u_obs) return set_error(BA_ERR_INVALID_ARG, "a scene array is NULL");
    return BA_OK;
}

// device buffers of one LM run, released together
struct LMBuffers {
    double *Jp = nullptr, *Jl = nullptr, *r = nullptr;   // linearisation at the current state
    double *cams_c = nullptr, *X_c = nullptr;             // the moved (candidate) state
    double *dxp = nullptr, *dxl = nullptr;
    double *partials = nullptr;                           // project_blocks(m) + 1 (F)
    ~LMBuffers() {
        for (double *p : {Jp, Jl, r, cams_c, X_c, dxp, dxl, partials})
            if (p) (void)hipFree(p);
    }
};

ba_status alloc(double **p, size_t count) {
    if (hipMalloc((void **)p, count * sizeof(double)) != hipSuccess) {
        *p = nullptr;
        return set_error(BA_ERR_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(double)) + " bytes failed");
    }
    return BA_OK;
}

double ms_since(std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

}  // namespace

extern "C" {

void ba_default_lm_opts(ba_lm_opts *o) {
    if (!o) return;
    *o = ba_lm_opts{};
    o->max_iter = 25;
    o->solver = 0;
    o->n_groups = 1;
    o->tau = 3.3;
    o->lambda0 = 1e-4;
    o->ftol = 1e-6;
    o->lambda_factor = 10.0;
    ba_default_solve_opts(&o->solve);
}

ba_status ba_project(const ba_scene_desc *sc, const double *cams, const double *X, double *J_p, double *J_l,
                     double *r, double *cost, void *stream) {
    ba_status st = check_scene(sc);
    if (st != BA_OK) return st;
    if (!cams || !X) return set_error(BA_ERR_INVALID_ARG, "cams or X is NULL");
    if ((J_p == nullptr) != (J_l == nullptr)) return set_error(BA_ERR_INVALID_ARG, "J_p and J_l go together");
    hipStream_t q = (hipStream_t)stream;
    double *part = nullptr;
    if ((st = alloc(&part, (size_t)project_blocks(sc->n_obs) + 1)) != BA_OK) return st;
    double *dcost = part + project_blocks(sc->n_obs);
    launch_project(sc->n_obs, sc->obs_cam, sc->obs_lm, cams, X, sc->u_obs, J_p, J_l, r, part, dcost, q);
    double h = 0.0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&h, dcost, sizeof(double), hipMemcpyDeviceToHost, q);
    if (e == hipSuccess) e = hipStreamSynchronize(q);
    (void)hipFree(part);
    if (e != hipSuccess) return set_error(BA_ERR_HIP, std::string("ba_project: ") + hipGetErrorString(e));
    if (cost) *cost = h;
    return BA_OK;
}

ba_status ba_apply_step(int32_t n_cams, int32_t n_lms, const double *cams, const double *X, const double *dxp,
                        const double *dxl, double *cams_out, double *X_out, void *stream) {
    if (n_cams < 1 || n_lms < 1) return set_error(BA_ERR_INVALID_ARG, "n_cams and n_lms must be positive");
    if (!cams || !X || !dxp || !dxl || !cams_out || !X_out) return set_error(BA_ERR_INVALID_ARG, "NULL argument");
    launch_apply_step(n_cams, n_lms, cams, X, dxp, dxl, cams_out, X_out, (hipStream_t)stream);
    LMCHK(hipGetLastError());
    return BA_OK;
}

ba_status ba_lm_solve(const ba_scene_desc *sc, double *cams, double *X, const ba_lm_opts *opts_in, void *stream,
                      ba_lm_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    ba_status st = check_scene(sc);
    if (st != BA_OK) return st;
    if (!cams || !X) return set_error(BA_ERR_INVALID_ARG, "cams or X is NULL");
    ba_lm_opts o;
    if (opts_in) o = *opts_in;
    else ba_default_lm_opts(&o);
    if (o.max_iter < 0 || (o.solver != 0 && o.solver != 1) || (o.solver == 1 && o.n_groups < 1))
        return set_error(BA_ERR_INVALID_ARG, "max_iter >= 0, solver 0 (PCG) or 1 (MCG), n_groups >= 1");
    if (!std::isfinite(o.lambda0) || o.lambda0 < 0.0 || !(o.lambda_factor > 1.0) || !(o.ftol >= 0.0))
        return set_error(BA_ERR_INVALID_ARG, "lambda0 >= 0, lambda_factor > 1 and ftol >= 0 are required");
    hipStream_t q = (hipStream_t)stream;
    const int64_t m = sc->n_obs;
    const int np = sc->n_cams, nl = sc->n_lms;
    const int pb = project_blocks(m);
    LMBuffers b;
    if ((st = alloc(&b.Jp, (size_t)m * 18)) != BA_OK || (st = alloc(&b.Jl, (size_t)m * 6)) != BA_OK ||
        (st = alloc(&b.r, (size_t)m * 2)) != BA_OK || (st = alloc(&b.cams_c, (size_t)np * 15)) != BA_OK ||
        (st = alloc(&b.X_c, (size_t)nl * 3)) != BA_OK || (st = alloc(&b.dxp, (size_t)np * 9)) != BA_OK ||
        (st = alloc(&b.dxl, (size_t)nl * 3)) != BA_OK || (st = alloc(&b.partials, (size_t)pb + 1)) != BA_OK)
        return st;
    double *dcost = b.partials + pb;
    double t_solve = 0.0, t_lin = 0.0;
    // F (and with `jac` the linearisation) of a state, read back
    auto evaluate = [&](const double *c, const double *x, bool jac, double *F) -> ba_status {
        launch_project(m, sc->obs_cam, sc->obs_lm, c, x, sc->u_obs, jac ? b.Jp : nullptr, jac ? b.Jl : nullptr,
                       jac ? b.r : nullptr, b.partials, dcost, q);
        LMCHK(hipGetLastError());
        LMCHK(hipMemcpyAsync(F, dcost, sizeof(double), hipMemcpyDeviceToHost, q));
        LMCHK(hipStreamSynchronize(q));
        return BA_OK;
    };
    auto tl = std::chrono::steady_clock::now();
    double F = 0.0;
    if ((st = evaluate(cams, X, true, &F)) != BA_OK) return st;
    if (!std::isfinite(F)) return set_error(BA_ERR_NONFINITE, "F is not finite at the start state");
    double lam = o.lambda0;
    ba_problem_desc d{};
    d.n_cams = np;
    d.n_lms = nl;
    d.n_obs = m;
    d.d_p = 9;
    d.obs_cam = sc->obs_cam;
    d.obs_lm = sc->obs_lm;
    d.J_p = b.Jp;
    d.J_l = b.Jl;
    d.r = b.r;
    d.lambda = lam;
    ba_system *sys = nullptr;
    if ((st = ba_build_system(&d, &o.build, stream, &sys)) != BA_OK) return st;
    // the subsets' layout depends on the observations only: set up once, with the system
    if (o.solver == 1 && (st = prepare_mcg(sys, o.n_groups, o.solve.precision)) != BA_OK) {
        ba_free_system(sys);
        return st;
    }
    t_lin += ms_since(tl);
    const double cost0 = F;
    int it = 0, accepted_n = 0;
    int64_t solver_its = 0;
    ba_status result = BA_OK;
    for (; it < o.max_iter;) {
        if (F == 0.0) break;
        // the damped normal equation through S (eq. (13)), then the landmarks (eq. (16), corrected)
        ba_solve_stats ss{};
        auto ts = std::chrono::steady_clock::now();
        st = o.solver == 0 ? ba_pcg_solve(sys, nullptr, b.dxp, &o.solve, &ss)
                           : ba_mcg_solve(sys, o.n_groups, o.tau, nullptr, b.dxp, &o.solve, &ss);
        const double solve_ms = ms_since(ts);
        t_solve += solve_ms;
        if (st != BA_OK && st != BA_MAXITER) {
            result = st;
            break;
        }
        if ((st = ba_back_substitute(sys, b.dxp, b.dxl)) != BA_OK) {
            result = st;
            break;
        }
        tl = std::chrono::steady_clock::now();
        launch_apply_step(np, nl, cams, X, b.dxp, b.dxl, b.cams_c, b.X_c, q);
        double Fn = 0.0;
        if ((st = evaluate(b.cams_c, b.X_c, false, &Fn)) != BA_OK) {
            result = st;
            break;
        }
        const bool accept = Fn < F;   // false for a non-finite F_new
        const double change = std::fabs(F - Fn) / F;
        if (stats && it < stats->trace_cap) {
            if (stats->trace_lambda) stats->trace_lambda[it] = lam;
            if (stats->trace_cost) stats->trace_cost[it] = Fn;
            if (stats->trace_accepted) stats->trace_accepted[it] = accept ? 1 : 0;
            if (stats->trace_solver_iterations) stats->trace_solver_iterations[it] = ss.iterations;
            if (stats->trace_solve_ms) stats->trace_solve_ms[it] = solve_ms;
        }
        ++it;
        solver_its += ss.iterations;
        if (accept) {
            ++accepted_n;
            if (hipMemcpyAsync(cams, b.cams_c, (size_t)np * 15 * sizeof(double), hipMemcpyDeviceToDevice, q) !=
                    hipSuccess ||
                hipMemcpyAsync(X, b.X_c, (size_t)nl * 3 * sizeof(double), hipMemcpyDeviceToDevice, q) != hipSuccess) {
                result = set_error(BA_ERR_HIP, "state copy failed");
                break;
            }
            F = Fn;
            lam /= o.lambda_factor;
        } else {
            lam *= o.lambda_factor;
        }
        const bool stop = change < o.ftol || it >= o.max_iter || F == 0.0;
        if (!stop) {
            // relinearise at the accepted state, or keep the linearisation with the new lambda
            if (accept && (st = evaluate(cams, X, true, &Fn)) != BA_OK) {
                result = st;
                break;
            }
            // a rejected step keeps J and r: only the values that depend on lambda change
            st = accept ? ba_update_system(sys, b.Jp, b.Jl, b.r, lam) : ba_set_lambda(sys, lam);
            if (st != BA_OK) {
                result = st;
                break;
            }
        }
        t_lin += ms_since(tl);
        if (stop) break;
    }
    ba_free_system(sys);
    if (hipStreamSynchronize(q) != hipSuccess && result == BA_OK)
        result = set_error(BA_ERR_HIP, "stream synchronisation failed");
    if (stats) {
        stats->iterations = it;
        stats->accepted = accepted_n;
        stats->status = result;
        stats->solver_iterations = (int32_t)solver_its;
        stats->cost0 = cost0;
        stats->cost = F;
        stats->t_total_ms = ms_since(t0);
        stats->t_solve_ms = t_solve;
        stats->t_linearize_ms = t_lin;
    }
    return result;
}

}  // extern "C"
