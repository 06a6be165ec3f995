// Host engine and C ABI of the periodic thermal homogenization library.
//
// One context = one design cell of n^3 voxels on the current HIP device.  All
// per-iteration work runs in the kernels of otm_kernels.hip on the context's
// stream; the host only sequences launches, reads back a few scalars (PCG
// convergence flags, the 6-vector tensor, reduction sums) and runs the scalar
// logic of the adaptive volume governor (Algorithm 1) and the objective.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "opentm_amd.h"
#include "otm_internal.h"

using namespace otm;

#define OTM_VERSION "opentm-amd 0.1 (gfx950)"

struct otm_ctx {
    otm_problem prob;
    otm_solver_opts so;
    otm_oc_opts oc;
    otm_governor_opts go;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    int n = 0;
    int64_t nn = 0;
    int64_t dev_bytes = 0;  // device memory this context holds

    // fields (float64)
    double* rho = nullptr;
    double* rhof = nullptr;
    double* k = nullptr;
    double* dinv = nullptr;
    double* b = nullptr;    // 3 nn
    double* x = nullptr;    // 3 nn, solution chi
    double* st = nullptr;   // element sensitivity before the filter transpose
    double* sens = nullptr; // after
    double* ocq = nullptr;  // OC numerator q_e
    // FP64 Krylov vectors
    double* r64 = nullptr;
    double* p64[2] = {nullptr, nullptr};
    double* q64 = nullptr;
    double* r64b = nullptr;  // second r, q of the fused iteration (ping-pong)
    double* q64b = nullptr;
    // mixed-precision Krylov vectors
    float* k32 = nullptr;
    float* dinv32 = nullptr;
    float* x32 = nullptr;
    float* r32 = nullptr;
    float* p32[2] = {nullptr, nullptr};
    float* q32 = nullptr;
    float* r32b = nullptr;
    float* q32b = nullptr;

    double* partials = nullptr;
    unsigned* counter = nullptr;
    Scalars* sc = nullptr;
    Scalars* h_sc = nullptr;  // pinned host mirror
    int max_blocks = 0;
    int pbuf = 0;
    TileShape tile;   // one-node-per-thread kernels (ring, march)
    TileShape tile2;  // pair kernel (even n)
    bool use_pair = false;
    bool use_fused = false;  // one pass per PCG iteration (otm_fused.hip)
    bool fused_chain = false;  // passes within a check interval reduce their predecessor's sums
    double tune_us = 0.0;  // autotuned time of one PCG iteration's passes
    otm_nn* net = nullptr;
    int learned_used = 0;  // last solve started from the network's prediction

    // multigrid preconditioner (float32 V-cycle, captured as a graph)
    bool use_mg = false;
    MgHierarchy mg;
    std::vector<void*> mg_bufs;
    float* ones32 = nullptr;       // D^-1 := 1 for the direction pass and the update (mixed)
    double* ones64 = nullptr;      // the same for float64 contexts
    const float* mg_z = nullptr;   // z = M^-1 r written by the captured cycle
    int mg_nb = 0;                 // blocks of its r.z partial sums
    hipGraph_t mg_graph = nullptr;
    hipGraphExec_t mg_exec = nullptr;

    bool have_density = false;
    bool prepared = false;
    bool homogenized = false;
    bool have_sens = false;
    bool have_solution = false;
    bool have_user_guess = false;

    double kappa[6] = {0, 0, 0, 0, 0, 0};
    double g = 0.0;
    double w[6] = {0, 0, 0, 0, 0, 0};
    double volume = 0.0, low_bound = 0.0;

    // adaptive volume bound (Algorithm 1) and the design iteration count
    VolumeBound vb;
    int iter = 0;

    otm_solve_stats last_stats{};
    double timings[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    hipEvent_t ev[8] = {};
    // live timing of the dominant solver kernel: one sampled launch per
    // check interval with every load active, bracketed by the launch's own
    // start/end events (hipExtLaunchKernelGGL)
    hipEvent_t pev[2] = {};
    hipEvent_t cev = nullptr;  // marks the scalar copy of a check (no timing)
    double pass_ms = 0.0;
    int64_t pass_count = 0;
    double pass_bytes = 0.0;  // algorithmic bytes of one sampled launch
    int pass_kind = 0;        // 4: fused pass, 0: direction+operator pass
    std::string err;

    Workspace ws() const { return Workspace{partials, counter, sc, max_blocks}; }
};

namespace {

int fail(otm_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(c, call)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            return fail((c), OTM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));        \
        }                                                                                            \
    } while (0)

int check_launch(otm_ctx* c, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, OTM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return OTM_OK;
}

template <typename T>
int dalloc(otm_ctx* c, T** p, int64_t count) {
    if (hipMalloc((void**)p, (size_t)count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, OTM_ENOMEM, "device allocation of " + std::to_string((long long)count * sizeof(T)) + " bytes failed");
    }
    c->dev_bytes += count * (int64_t)sizeof(T);
    return OTM_OK;
}

bool finite6(const double* v) {
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

int sync_scalars(otm_ctx* c) {
    HIPCHK(c, hipMemcpyAsync(c->h_sc, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return OTM_OK;
}

int validate_problem(const otm_problem* p, std::string& why) {
    if (!p) {
        why = "problem is NULL";
        return OTM_EINVAL;
    }
    if (p->n < 4 || p->n > 1024) {
        why = "n must be in [4, 1024]";
        return OTM_EINVAL;
    }
    if (!(std::isfinite(p->k0) && std::isfinite(p->kmin) && p->kmin > 0.0 && p->k0 > p->kmin)) {
        why = "need 0 < kmin < k0, finite";
        return OTM_EINVAL;
    }
    if (!(std::isfinite(p->penal) && p->penal >= 1.0)) {
        why = "penal must be >= 1";
        return OTM_EINVAL;
    }
    if (!(std::isfinite(p->filter_radius) && p->filter_radius < 5.0)) {
        why = "filter_radius must be finite and < 5";
        return OTM_EINVAL;
    }
    if (!(std::isfinite(p->vf) && p->vf > 0.0 && p->vf <= 1.0)) {
        why = "vf must be in (0, 1]";
        return OTM_EINVAL;
    }
    if (!finite6(p->target)) {
        why = "target must be finite";
        return OTM_EINVAL;
    }
    if (p->objective != OTM_OBJ_MSE && p->objective != OTM_OBJ_REL && p->objective != OTM_OBJ_L1) {
        why = "unsupported objective";
        return OTM_EUNSUPPORTED;
    }
    if (p->objective == OTM_OBJ_REL)
        for (int q = 0; q < 6; ++q)
            if (p->target[q] == 0.0) {
                why = "the relative objective needs every target component nonzero";
                return OTM_EINVAL;
            }
    if (p->symmetry != OTM_SYM_NONE && p->symmetry != OTM_SYM_CENTRAL) {
        why = "unknown symmetry";
        return OTM_EINVAL;
    }
    return OTM_OK;
}

// ------------------------------------------------------------------ timing
struct EvTimer {
    otm_ctx* c;
    int a, b;
    EvTimer(otm_ctx* c_, int a_, int b_) : c(c_), a(a_), b(b_) { (void)hipEventRecord(c->ev[a], c->stream); }
    void stop() { (void)hipEventRecord(c->ev[b], c->stream); }
};

double ev_ms(otm_ctx* c, int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0;
    }
    return (double)ms;
}

// ------------------------------------------------------------------ prepare
// filter + SIMP + macro loads + diagonal, b projected to zero mean
int prepare(otm_ctx* c) {
    if (!c->have_density) return fail(c, OTM_ESTATE, "no density set");
    const Workspace w = c->ws();
    if (c->prob.symmetry == OTM_SYM_CENTRAL) launch_sym_central(c->n, c->rho, c->stream);
    launch_filter_simp(c->n, c->prob.filter_radius, c->rho, c->rhof, c->k, c->k32, c->prob.k0, c->prob.kmin,
                       c->prob.penal, w, c->stream);
    launch_setup_nodes(c->n, c->k, c->b, c->dinv, c->dinv32, w, c->stream);
    launch_sub_mean3(c->n, c->b, 1, w, c->stream);
    if (c->use_mg) {
        // coarse conductivities and diagonals, inverse of the coarsest operator
        const MgHierarchy& H = c->mg;
        for (int l = 1; l < H.levels; ++l)
            launch_mg_coarsen(H.lv[l].n, H.lv[l - 1].k, H.lv[l].kc, H.lv[l].dinvc, c->stream);
        launch_mg_coarse_setup(H.lv[H.levels - 1].n, H.lv[H.levels - 1].k, H.minv, c->stream);
    }
    int rc = check_launch(c, "prepare");
    if (rc) return rc;
    c->prepared = true;
    return OTM_OK;
}

// ------------------------------------------------------------------ PCG
bool all_inactive(const Scalars* s) { return !s->active[0] && !s->active[1] && !s->active[2]; }
bool all_active(const Scalars* s) { return s->active[0] && s->active[1] && s->active[2]; }
int max_iters(const Scalars* s) {
    int m = s->iters[0];
    if (s->iters[1] > m) m = s->iters[1];
    if (s->iters[2] > m) m = s->iters[2];
    return m;
}

// Stagnation and divergence watch over the host checks of one solve: the
// best recursive residual of every active load must halve (its square drop
// to a quarter) within `window` iterations of that load; a non-finite
// residual is divergence.  The mixed-precision paths' recursive residual is
// refreshed from the float64 one, so a float32 recursion that has lost
// touch with the true residual stops improving the best value and trips it.
struct SolveWatch {
    double best[3] = {0, 0, 0};
    int at[3] = {0, 0, 0};
    int window = 0;
    int verdict = 0;  // 0 running, 1 stalled, 2 non-finite residual
    void start(const Scalars* s, int w) {
        window = w;
        verdict = 0;
        for (int l = 0; l < 3; ++l) {
            best[l] = s->rr[l];
            at[l] = s->iters[l];
        }
    }
    // true when the solve should stop
    bool stop(const Scalars* s) {
        bool stuck = false;
        for (int l = 0; l < 3; ++l) {
            if (!s->active[l]) continue;
            if (!std::isfinite(s->rr[l])) {
                verdict = 2;
                return true;
            }
            if (s->rr[l] <= 0.25 * best[l]) {
                best[l] = s->rr[l];
                at[l] = s->iters[l];
            } else if (s->iters[l] - at[l] > window) {
                stuck = true;
            }
        }
        if (stuck) verdict = 1;
        return stuck;
    }
};

// Iterations without progress before a solve counts as stagnant.
int stall_window(const otm_ctx* c) {
    return c->so.stall_window > 0 ? c->so.stall_window : 200 + 10 * c->n;
}

// Reset the solver part of the scalar block (the fields before sum_rho) and
// set tol^2; the reduction results of prepare() that follow are left intact.
int reset_solver_scalars(otm_ctx* c) {
    const size_t head = offsetof(Scalars, sum_rho);
    std::memset(c->h_sc, 0, head);
    c->h_sc->tol2 = c->so.tol * c->so.tol;
    HIPCHK(c, hipMemcpyAsync(c->sc, c->h_sc, head, hipMemcpyHostToDevice, c->stream));
    return OTM_OK;
}

// Adds the sampled launch of the last check interval (if any) to the live timing.
void collect_pass_sample(otm_ctx* c, bool sampled, double bytes, int kind) {
    if (!sampled) return;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->pev[0], c->pev[1]) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    c->pass_ms += (double)ms;
    c->pass_count += 1;
    c->pass_bytes = bytes;
    c->pass_kind = kind;
}

// One pass and one reduction per iteration (otm_fused.hip).  r[cur], q[cur],
// p[cur] hold what the next pass reads; x is the float64 solution (FP64) or the
// float32 increment folded into it at each residual refresh (mixed).
template <typename T>
struct FusedBufs {
    T* r[2];
    T* q[2];
    T* p[2];
    T* x;
    const T* dinv;
    const T* k;
};

template <typename T>
int solve_fused(otm_ctx* c, bool x_zero, bool mixed, const FusedBufs<T>& B, otm_solve_stats* st) {
    const Workspace w = c->ws();
    const int n = c->n;
    int rc;
    if ((rc = reset_solver_scalars(c))) return rc;
    if (x_zero) HIPCHK(c, hipMemsetAsync(c->x, 0, (size_t)3 * c->nn * sizeof(double), c->stream));
    if (mixed) HIPCHK(c, hipMemsetAsync(c->x32, 0, (size_t)3 * c->nn * sizeof(float), c->stream));
    int cur = 0;
    launch_residual_f<T>(n, c->k, c->b, c->x, B.r[cur], nullptr, B.dinv, true, x_zero ? 1 : 0, w, c->stream);
    if ((rc = check_launch(c, "residual"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    double rr_ref[3] = {c->h_sc->rr_true[0], c->h_sc->rr_true[1], c->h_sc->rr_true[2]};
    const double d2 = c->so.reliable_delta * c->so.reliable_delta;
    int refreshes = 0, launches = 0;
    SolveWatch watch;
    watch.start(c->h_sc, stall_window(c));
    // The host reads a check's scalars while one more pass (the bridge) runs,
    // so the copy's round trip does not leave the device idle.  What the
    // host decides from them still holds a pass later: a load that converged
    // is left unchanged by the passes after it (no step, no count), and a
    // residual refresh may come one pass late.  The next chunk is one pass
    // shorter, so the checks stay check_every passes apart.
    int bridged = 0;
    while (!all_inactive(c->h_sc) && max_iters(c->h_sc) < c->so.max_iter) {
        const bool all = all_active(c->h_sc);
        const int len = c->so.check_every - bridged;
        // h_sc is not read again until the copy below has landed
        const bool bridge = max_iters(c->h_sc) + c->so.check_every < c->so.max_iter;
        bool sampled = false;
        for (int it = 0; it < len; ++it) {
            const int nx = cur ^ 1;
            // sample the chunk's last pass when every load takes a full step
            const bool sample = all && launches > 0 && it == len - 1;
            // chained: passes after the first of a chunk reduce their
            // predecessor's sums themselves and the chunk's last pass is closed
            // by a finalize; else a finalize follows every pass
            const bool chained = c->fused_chain && it > 0;
            const bool fin = !c->fused_chain || it == len - 1;
            launch_fused<T>(n, c->tile2, all, B.r[cur], B.q[cur], B.p[cur], B.r[nx], B.q[nx], B.p[nx], B.x, B.dinv,
                            B.k, w, c->stream, cur, chained, fin, sample ? c->pev[0] : nullptr,
                            sample ? c->pev[1] : nullptr);
            sampled = sampled || sample;
            cur = nx;
            ++launches;
        }
        HIPCHK(c, hipMemcpyAsync(c->h_sc, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipEventRecord(c->cev, c->stream));
        bridged = 0;
        if (bridge) {
            const int nx = cur ^ 1;
            launch_fused<T>(n, c->tile2, all, B.r[cur], B.q[cur], B.p[cur], B.r[nx], B.q[nx], B.p[nx], B.x, B.dinv,
                            B.k, w, c->stream, cur, false, true, nullptr, nullptr);
            cur = nx;
            ++launches;
            bridged = 1;
        }
        if ((rc = check_launch(c, "pcg fused"))) return rc;
        HIPCHK(c, hipEventSynchronize(c->cev));
        // fused pass: r, q, p, x read and written, D^-1 and k read (three loads);
        // the sample counts only if every load still ran its last pass
        collect_pass_sample(c, sampled && all_active(c->h_sc), (double)c->nn * (8.0 * 3 + 1 + 1) * sizeof(T), 4);
        bool refresh = all_inactive(c->h_sc);
        if (mixed)
            for (int l = 0; l < 3; ++l)
                if (c->h_sc->active[l] && c->h_sc->rr[l] < d2 * rr_ref[l]) refresh = true;
        if (refresh) {
            // float64 residual of the current solution; loads whose true
            // residual misses the tolerance go on (or restart)
            if (mixed) launch_accumulate(n, c->x, c->x32, c->stream);
            launch_residual_f<T>(n, c->k, c->b, c->x, B.r[cur], B.q[cur], B.dinv, false, 0, w, c->stream);
            if ((rc = check_launch(c, "refresh"))) return rc;
            if ((rc = sync_scalars(c))) return rc;
            for (int l = 0; l < 3; ++l) rr_ref[l] = c->h_sc->rr_true[l];
            if (mixed) ++refreshes;
            bridged = 0;  // the scalars now describe the current state
        }
        if (watch.stop(c->h_sc)) break;
    }
    if (mixed) launch_accumulate(n, c->x, c->x32, c->stream);
    // a stopped solve reports the true residual of the solution it returns
    if (watch.verdict) launch_residual_f<T>(n, c->k, c->b, c->x, B.r[cur], B.q[cur], B.dinv, false, 0, w, c->stream);
    launch_sum3(n, c->x, 0, w, c->stream);
    launch_sub_mean3(n, c->x, 0, w, c->stream);
    if ((rc = check_launch(c, "project"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    for (int l = 0; l < 3; ++l) {
        st->iterations[l] = c->h_sc->iters[l];
        st->rel_residual[l] = c->h_sc->bb[l] > 0.0 ? std::sqrt(c->h_sc->rr_true[l] / c->h_sc->bb[l]) : 0.0;
    }
    st->converged = all_inactive(c->h_sc) ? 1 : 0;
    st->refreshes = refreshes;
    st->stalled = watch.verdict;
    c->timings[7] = (double)launches;
    return OTM_OK;
}

// Float64 CG preconditioned by the float32 V-cycle: r is rounded to float32
// for the cycle and z widened as the direction pass reads it; the Krylov vectors, dots and convergence
// test stay float64 (the true residual confirms convergence, as in the Jacobi
// path).  CG restarts (beta = 0) after such a confirmation.
int solve_mg64(otm_ctx* c, bool x_zero, otm_solve_stats* st) {
    const Workspace w = c->ws();
    const int n = c->n;
    const int64_t n3 = 3 * c->nn;
    int rc;
    if ((rc = reset_solver_scalars(c))) return rc;
    if (x_zero) HIPCHK(c, hipMemsetAsync(c->x, 0, (size_t)n3 * sizeof(double), c->stream));
    launch_residual<double>(n, c->k, c->b, c->x, c->r64, c->p64[c->pbuf], c->dinv, RES_START, x_zero ? 1 : 0, w,
                            c->stream);
    if ((rc = check_launch(c, "residual"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    int launches = 0;
    bool restart = true;
    const int check = c->so.check_every < 2 ? c->so.check_every : 2;
    SolveWatch watch;
    watch.start(c->h_sc, stall_window(c));
    while (!all_inactive(c->h_sc) && max_iters(c->h_sc) < c->so.max_iter) {
        const bool all = all_active(c->h_sc);
        bool sampled = false;
        for (int it = 0; it < check; ++it) {
            // the update writes the float32 copy of r; after a residual kernel it is cast here
            if (restart) launch_cast_f64_f32(n3, c->r64, c->r32, c->stream);
            HIPCHK(c, hipGraphLaunch(c->mg_exec, c->stream));
            launch_finalize(restart ? FIN_MG_RZ0 : FIN_MG_RZ, c->mg_nb, w, c->stream);
            restart = false;
            double* po = c->p64[c->pbuf];
            double* pn = c->p64[c->pbuf ^ 1];
            const bool sample = all && it == check - 1;
            // the direction pass reads the cycle's float32 output directly
            launch_dir_march2_zf(n, c->tile2, all, c->mg_z, c->ones64, po, pn, c->k, c->q64, w, c->stream,
                                 sample ? c->pev[0] : nullptr, sample ? c->pev[1] : nullptr);
            sampled = sampled || sample;
            launch_update_vec<double>(n, c->x, c->r64, pn, c->q64, c->ones64, w, c->stream, true, FIN_MG_UPDATE,
                                      c->r32);
            c->pbuf ^= 1;
            ++launches;
        }
        if ((rc = check_launch(c, "mg-pcg64"))) return rc;
        if ((rc = sync_scalars(c))) return rc;
        // direction pass: z (float32) read, p read and written, q written, ones and k read
        collect_pass_sample(c, sampled, (double)c->nn * (3.0 * sizeof(float) + 11.0 * sizeof(double)), 0);
        if (all_inactive(c->h_sc)) {
            // confirm with the true residual; loads that fail restart
            launch_residual<double>(n, c->k, c->b, c->x, c->r64, c->p64[c->pbuf], c->dinv, RES_START, 0, w,
                                    c->stream);
            if ((rc = sync_scalars(c))) return rc;
            restart = true;
        }
        if (watch.stop(c->h_sc)) break;
    }
    // a stopped solve reports the true residual of the solution it returns
    if (watch.verdict)
        launch_residual<double>(n, c->k, c->b, c->x, c->r64, c->p64[c->pbuf], c->dinv, RES_START, 0, w, c->stream);
    launch_sum3(n, c->x, 0, w, c->stream);
    launch_sub_mean3(n, c->x, 0, w, c->stream);
    if ((rc = check_launch(c, "project"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    for (int l = 0; l < 3; ++l) {
        st->iterations[l] = c->h_sc->iters[l];
        st->rel_residual[l] = c->h_sc->bb[l] > 0.0 ? std::sqrt(c->h_sc->rr_true[l] / c->h_sc->bb[l]) : 0.0;
    }
    st->converged = all_inactive(c->h_sc) ? 1 : 0;
    st->refreshes = 0;
    st->stalled = watch.verdict;
    c->timings[7] = (double)launches;
    return OTM_OK;
}

// Float64 Jacobi-PCG with the two-pass iteration (direction + operator pass,
// then the vector update); also the fallback of the float32 paths.
int solve_fp64_twopass(otm_ctx* c, bool x_zero, otm_solve_stats* st) {
    const Workspace w = c->ws();
    const int n = c->n;
    int rc;
    if ((rc = reset_solver_scalars(c))) return rc;
    if (x_zero) HIPCHK(c, hipMemsetAsync(c->x, 0, (size_t)3 * c->nn * sizeof(double), c->stream));
    launch_residual<double>(n, c->k, c->b, c->x, c->r64, c->p64[c->pbuf], c->dinv, RES_START, x_zero ? 1 : 0, w,
                            c->stream);
    if ((rc = check_launch(c, "residual"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    int launches = 0;
    SolveWatch watch;
    watch.start(c->h_sc, stall_window(c));
    while (!all_inactive(c->h_sc) && max_iters(c->h_sc) < c->so.max_iter) {
        const bool all = all_active(c->h_sc);
        bool sampled = false;
        for (int it = 0; it < c->so.check_every; ++it) {
            double* po = c->p64[c->pbuf];
            double* pn = c->p64[c->pbuf ^ 1];
            if (c->so.kernel_variant == 1) {
                launch_dir<double>(n, c->r64, c->dinv, po, pn, w, c->stream);
                launch_apply_pq<double>(n, c->k, pn, c->q64, w, c->stream);
                launch_update<double>(n, c->x, c->r64, pn, c->q64, c->dinv, w, c->stream);
            } else {
                if (c->so.kernel_variant == 2)
                    launch_dir_apply<double>(n, c->tile, c->r64, c->dinv, po, pn, c->k, c->q64, w, c->stream);
                else if (c->use_pair) {
                    const bool sample = all && it == c->so.check_every - 1;
                    launch_dir_march2<double>(n, c->tile2, all, c->r64, c->dinv, po, pn, c->k, c->q64, w, c->stream, true,
                                           sample ? c->pev[0] : nullptr, sample ? c->pev[1] : nullptr);
                    sampled = sampled || sample;
                }
                else
                    launch_dir_march<double>(n, c->tile, c->r64, c->dinv, po, pn, c->k, c->q64, w, c->stream);
                launch_update_vec<double>(n, c->x, c->r64, pn, c->q64, c->dinv, w, c->stream);
            }
            c->pbuf ^= 1;
            ++launches;
        }
        if ((rc = check_launch(c, "pcg"))) return rc;
        if ((rc = sync_scalars(c))) return rc;
        // direction+operator pass: r, p_old read, p, q written, D^-1 and k read
        collect_pass_sample(c, sampled, (double)c->nn * (4.0 * 3 + 1 + 1) * sizeof(double), 0);
        if (all_inactive(c->h_sc)) {
            // confirm with the true residual; loads that fail restart
            launch_residual<double>(n, c->k, c->b, c->x, c->r64, c->p64[c->pbuf], c->dinv, RES_START, 0, w,
                                    c->stream);
            if ((rc = sync_scalars(c))) return rc;
        }
        if (watch.stop(c->h_sc)) break;
    }
    // a stopped solve reports the true residual of the solution it returns
    if (watch.verdict)
        launch_residual<double>(n, c->k, c->b, c->x, c->r64, c->p64[c->pbuf], c->dinv, RES_START, 0, w, c->stream);
    launch_sum3(n, c->x, 0, w, c->stream);
    launch_sub_mean3(n, c->x, 0, w, c->stream);
    if ((rc = check_launch(c, "project"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    int conv = all_inactive(c->h_sc) ? 1 : 0;
    for (int l = 0; l < 3; ++l) {
        st->iterations[l] = c->h_sc->iters[l];
        st->rel_residual[l] = c->h_sc->bb[l] > 0.0 ? std::sqrt(c->h_sc->rr_true[l] / c->h_sc->bb[l]) : 0.0;
    }
    st->converged = conv;
    st->refreshes = 0;
    st->stalled = watch.verdict;
    c->timings[7] = (double)launches;
    return OTM_OK;
}

int solve_fp64(otm_ctx* c, bool x_zero, otm_solve_stats* st) {
    if (c->use_mg) return solve_mg64(c, x_zero, st);
    if (c->use_fused) {
        const FusedBufs<double> B{{c->r64, c->r64b}, {c->q64, c->q64b}, {c->p64[0], c->p64[1]}, c->x, c->dinv, c->k};
        return solve_fused<double>(c, x_zero, false, B, st);
    }
    return solve_fp64_twopass(c, x_zero, st);
}

// Multigrid-preconditioned CG in float32 with float64 residual refreshes
// (the refresh rule of the Jacobi path); z = M^-1 r by the captured V-cycle.
// PCG restarts (beta = 0) after each refresh.
int solve_mg(otm_ctx* c, bool x_zero, otm_solve_stats* st) {
    const Workspace w = c->ws();
    const int n = c->n;
    int rc;
    if ((rc = reset_solver_scalars(c))) return rc;
    if (x_zero) HIPCHK(c, hipMemsetAsync(c->x, 0, (size_t)3 * c->nn * sizeof(double), c->stream));
    HIPCHK(c, hipMemsetAsync(c->x32, 0, (size_t)3 * c->nn * sizeof(float), c->stream));
    launch_residual<float>(n, c->k, c->b, c->x, c->r32, c->p32[c->pbuf], c->dinv32, RES_START, x_zero ? 1 : 0, w,
                           c->stream);
    if ((rc = check_launch(c, "residual"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    double rr_ref[3] = {c->h_sc->rr_true[0], c->h_sc->rr_true[1], c->h_sc->rr_true[2]};
    const double d2 = c->so.reliable_delta * c->so.reliable_delta;
    int refreshes = 0, launches = 0;
    bool restart = true;
    // a V-cycle costs several operator passes and few are needed: check often
    const int check = c->so.check_every < 2 ? c->so.check_every : 2;
    SolveWatch watch;
    watch.start(c->h_sc, stall_window(c));
    while (!all_inactive(c->h_sc) && max_iters(c->h_sc) < c->so.max_iter) {
        const bool all = all_active(c->h_sc);
        bool sampled = false;
        for (int it = 0; it < check; ++it) {
            HIPCHK(c, hipGraphLaunch(c->mg_exec, c->stream));
            launch_finalize(restart ? FIN_MG_RZ0 : FIN_MG_RZ, c->mg_nb, w, c->stream);
            restart = false;
            float* po = c->p32[c->pbuf];
            float* pn = c->p32[c->pbuf ^ 1];
            const bool sample = all && it == check - 1;
            launch_dir_march2<float>(n, c->tile2, all, c->mg_z, c->ones32, po, pn, c->k32, c->q32, w, c->stream, true,
                                     sample ? c->pev[0] : nullptr, sample ? c->pev[1] : nullptr);
            sampled = sampled || sample;
            launch_update_vec<float>(n, c->x32, c->r32, pn, c->q32, c->ones32, w, c->stream, true, FIN_MG_UPDATE);
            c->pbuf ^= 1;
            ++launches;
        }
        if ((rc = check_launch(c, "mg-pcg"))) return rc;
        if ((rc = sync_scalars(c))) return rc;
        collect_pass_sample(c, sampled, (double)c->nn * (4.0 * 3 + 1 + 1) * sizeof(float), 0);
        bool refresh = all_inactive(c->h_sc);
        for (int l = 0; l < 3; ++l)
            if (c->h_sc->active[l] && c->h_sc->rr[l] < d2 * rr_ref[l]) refresh = true;
        if (refresh) {
            launch_accumulate(n, c->x, c->x32, c->stream);
            launch_residual<float>(n, c->k, c->b, c->x, c->r32, c->p32[c->pbuf], c->dinv32, RES_REFRESH, 0, w,
                                   c->stream);
            if ((rc = check_launch(c, "refresh"))) return rc;
            if ((rc = sync_scalars(c))) return rc;
            for (int l = 0; l < 3; ++l) rr_ref[l] = c->h_sc->rr_true[l];
            ++refreshes;
            restart = true;
        }
        if (watch.stop(c->h_sc)) break;
    }
    launch_accumulate(n, c->x, c->x32, c->stream);
    // a stopped solve reports the true residual of the solution it returns
    if (watch.verdict)
        launch_residual<float>(n, c->k, c->b, c->x, c->r32, c->p32[c->pbuf], c->dinv32, RES_REFRESH, 0, w, c->stream);
    launch_sum3(n, c->x, 0, w, c->stream);
    launch_sub_mean3(n, c->x, 0, w, c->stream);
    if ((rc = check_launch(c, "project"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    for (int l = 0; l < 3; ++l) {
        st->iterations[l] = c->h_sc->iters[l];
        st->rel_residual[l] = c->h_sc->bb[l] > 0.0 ? std::sqrt(c->h_sc->rr_true[l] / c->h_sc->bb[l]) : 0.0;
    }
    st->converged = all_inactive(c->h_sc) ? 1 : 0;
    st->refreshes = refreshes;
    st->stalled = watch.verdict;
    c->timings[7] = (double)launches;
    return OTM_OK;
}

int solve_mixed(otm_ctx* c, bool x_zero, otm_solve_stats* st) {
    if (c->use_mg) return solve_mg(c, x_zero, st);
    if (c->use_fused) {
        const FusedBufs<float> B{{c->r32, c->r32b}, {c->q32, c->q32b}, {c->p32[0], c->p32[1]}, c->x32, c->dinv32,
                                 c->k32};
        return solve_fused<float>(c, x_zero, true, B, st);
    }
    const Workspace w = c->ws();
    const int n = c->n;
    int rc;
    if ((rc = reset_solver_scalars(c))) return rc;
    if (x_zero) HIPCHK(c, hipMemsetAsync(c->x, 0, (size_t)3 * c->nn * sizeof(double), c->stream));
    HIPCHK(c, hipMemsetAsync(c->x32, 0, (size_t)3 * c->nn * sizeof(float), c->stream));
    launch_residual<float>(n, c->k, c->b, c->x, c->r32, c->p32[c->pbuf], c->dinv32, RES_START, x_zero ? 1 : 0, w,
                           c->stream);
    if ((rc = check_launch(c, "residual"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    double rr_ref[3] = {c->h_sc->rr_true[0], c->h_sc->rr_true[1], c->h_sc->rr_true[2]};
    const double d2 = c->so.reliable_delta * c->so.reliable_delta;
    int refreshes = 0, launches = 0;
    SolveWatch watch;
    watch.start(c->h_sc, stall_window(c));
    while (!all_inactive(c->h_sc) && max_iters(c->h_sc) < c->so.max_iter) {
        const bool all = all_active(c->h_sc);
        bool sampled = false;
        for (int it = 0; it < c->so.check_every; ++it) {
            float* po = c->p32[c->pbuf];
            float* pn = c->p32[c->pbuf ^ 1];
            if (c->so.kernel_variant == 1) {
                launch_dir<float>(n, c->r32, c->dinv32, po, pn, w, c->stream);
                launch_apply_pq<float>(n, c->k32, pn, c->q32, w, c->stream);
                launch_update<float>(n, c->x32, c->r32, pn, c->q32, c->dinv32, w, c->stream);
            } else {
                if (c->so.kernel_variant == 2)
                    launch_dir_apply<float>(n, c->tile, c->r32, c->dinv32, po, pn, c->k32, c->q32, w, c->stream);
                else if (c->use_pair) {
                    const bool sample = all && it == c->so.check_every - 1;
                    launch_dir_march2<float>(n, c->tile2, all, c->r32, c->dinv32, po, pn, c->k32, c->q32, w, c->stream, true,
                                           sample ? c->pev[0] : nullptr, sample ? c->pev[1] : nullptr);
                    sampled = sampled || sample;
                }
                else
                    launch_dir_march<float>(n, c->tile, c->r32, c->dinv32, po, pn, c->k32, c->q32, w, c->stream);
                launch_update_vec<float>(n, c->x32, c->r32, pn, c->q32, c->dinv32, w, c->stream);
            }
            c->pbuf ^= 1;
            ++launches;
        }
        if ((rc = check_launch(c, "pcg32"))) return rc;
        if ((rc = sync_scalars(c))) return rc;
        // direction+operator pass: r, p_old read, p, q written, D^-1 and k read
        collect_pass_sample(c, sampled, (double)c->nn * (4.0 * 3 + 1 + 1) * sizeof(float), 0);
        bool refresh = all_inactive(c->h_sc);
        for (int l = 0; l < 3; ++l)
            if (c->h_sc->active[l] && c->h_sc->rr[l] < d2 * rr_ref[l]) refresh = true;
        if (refresh) {
            launch_accumulate(n, c->x, c->x32, c->stream);
            launch_residual<float>(n, c->k, c->b, c->x, c->r32, c->p32[c->pbuf], c->dinv32, RES_REFRESH, 0, w,
                                   c->stream);
            if ((rc = check_launch(c, "refresh"))) return rc;
            if ((rc = sync_scalars(c))) return rc;
            for (int l = 0; l < 3; ++l) rr_ref[l] = c->h_sc->rr_true[l];
            ++refreshes;
        }
        if (watch.stop(c->h_sc)) break;
    }
    // fold any remaining float32 increment into the float64 solution
    launch_accumulate(n, c->x, c->x32, c->stream);
    // a stopped solve reports the true residual of the solution it returns
    if (watch.verdict)
        launch_residual<float>(n, c->k, c->b, c->x, c->r32, c->p32[c->pbuf], c->dinv32, RES_REFRESH, 0, w, c->stream);
    launch_sum3(n, c->x, 0, w, c->stream);
    launch_sub_mean3(n, c->x, 0, w, c->stream);
    if ((rc = check_launch(c, "project"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    for (int l = 0; l < 3; ++l) {
        st->iterations[l] = c->h_sc->iters[l];
        st->rel_residual[l] = c->h_sc->bb[l] > 0.0 ? std::sqrt(c->h_sc->rr_true[l] / c->h_sc->bb[l]) : 0.0;
    }
    st->converged = all_inactive(c->h_sc) ? 1 : 0;
    st->refreshes = refreshes;
    st->stalled = watch.verdict;
    c->timings[7] = (double)launches;
    return OTM_OK;
}

// The float64 Krylov vectors of the two-pass iteration, allocated on the
// first fallback of a mixed-precision context (which does not hold them).
int ensure_fp64_vectors(otm_ctx* c) {
    int rc = OTM_OK;
    const int64_t n3 = 3 * c->nn;
    if (!c->r64) rc = dalloc(c, &c->r64, n3);
    if (!rc && !c->q64) rc = dalloc(c, &c->q64, n3);
    for (int q = 0; q < 2 && !rc; ++q)
        if (!c->p64[q]) {
            rc = dalloc(c, &c->p64[q], n3);
            if (!rc) HIPCHK(c, hipMemsetAsync(c->p64[q], 0, (size_t)n3 * sizeof(double), c->stream));
        }
    return rc;
}

int homogenize(otm_ctx* c, double kappa6[6], otm_solve_stats* st_out) {
    int rc;
    EvTimer t0(c, 0, 1);
    if ((rc = prepare(c))) return rc;
    t0.stop();
    // warm starts: the previous solution, a user field or the network's
    // prediction, each load scaled by its energy-minimising factor
    bool have_guess = false;
    if (c->so.guess == OTM_GUESS_PREVIOUS && c->have_solution) have_guess = true;
    if (c->so.guess == OTM_GUESS_USER && c->have_user_guess) have_guess = true;
    c->learned_used = 0;
    if (c->so.guess == OTM_GUESS_LEARNED && c->net && c->n % 16 == 0) {
        // the network runs on its own stream: it starts after prepare() and
        // the solve after it, ordered by events on the device (no host wait)
        const hipStream_t ns = nn_stream(c->net);
        HIPCHK(c, hipEventRecord(c->cev, c->stream));
        HIPCHK(c, hipStreamWaitEvent(ns, c->cev, 0));
        rc = otm_nn_forward(c->net, c->n, c->rhof, c->x);
        if (rc) return fail(c, rc, "network forward failed");
        HIPCHK(c, hipEventRecord(c->cev, ns));
        HIPCHK(c, hipStreamWaitEvent(c->stream, c->cev, 0));
        have_guess = true;
    }
    bool x_zero = true;
    if (have_guess) {
        launch_guess_scale(c->n, c->k, c->b, c->x, c->ws(), c->stream);
        if ((rc = check_launch(c, "guess scale"))) return rc;
        if ((rc = sync_scalars(c))) return rc;
        const double* gs = c->h_sc->gscale;
        x_zero = !(gs[0] > 0.0 || gs[1] > 0.0 || gs[2] > 0.0);
        if (c->so.guess == OTM_GUESS_LEARNED) c->learned_used = x_zero ? 0 : 1;
    }
    otm_solve_stats st{};
    (void)hipEventRecord(c->ev[2], c->stream);
    auto t_start = std::chrono::steady_clock::now();
    rc = (c->so.precision == OTM_MIXED) ? solve_mixed(c, x_zero, &st) : solve_fp64(c, x_zero, &st);
    if (rc) return rc;
    if (c->so.precision == OTM_MIXED && st.stalled) {
        // the float32 recursion stopped making progress (or its residual left
        // the finite range): finish in float64 from the current solution, or
        // from zero after a non-finite residual
        if ((rc = ensure_fp64_vectors(c))) return rc;
        otm_solve_stats s2{};
        rc = solve_fp64_twopass(c, st.stalled == 2, &s2);
        if (rc) return rc;
        for (int l = 0; l < 3; ++l) {
            s2.iterations[l] += st.iterations[l];
        }
        s2.refreshes = st.refreshes;
        s2.fallback = 1;
        st = s2;
    }
    (void)hipEventRecord(c->ev[3], c->stream);
    auto t_end = std::chrono::steady_clock::now();
    st.ms_solve = std::chrono::duration<double, std::milli>(t_end - t_start).count();
    c->have_solution = true;
    c->have_user_guess = false;
    const Workspace w = c->ws();
    launch_energy(c->n, c->k, c->x, w, c->stream);
    if ((rc = check_launch(c, "energy"))) return rc;
    (void)hipEventRecord(c->ev[4], c->stream);
    if ((rc = sync_scalars(c))) return rc;
    for (int q = 0; q < 6; ++q) c->kappa[q] = c->h_sc->kappa_sum[q] / (double)c->nn;
    c->volume = c->h_sc->sum_rho / (double)c->nn;
    c->low_bound = c->h_sc->sum_rhofp / (double)c->nn;
    c->timings[0] = ev_ms(c, 0, 1);
    c->timings[6] = (double)c->learned_used;
    c->timings[1] = ev_ms(c, 2, 3);
    c->timings[2] = ev_ms(c, 3, 4);
    if (!finite6(c->kappa)) return fail(c, OTM_ENONFINITE, "non-finite homogenized tensor");
    if (kappa6) std::memcpy(kappa6, c->kappa, sizeof(c->kappa));
    c->last_stats = st;
    if (st_out) *st_out = st;
    c->homogenized = true;
    c->have_sens = false;
    return st.converged ? OTM_OK : OTM_NOT_CONVERGED;
}

int sensitivity(otm_ctx* c, const double w6[6]) {
    if (!c->homogenized) return fail(c, OTM_ESTATE, "sensitivity needs a prior homogenize");
    if (!finite6(w6)) return fail(c, OTM_ENONFINITE, "non-finite dg/dkappa");
    (void)hipEventRecord(c->ev[4], c->stream);
    launch_sens(c->n, c->rhof, c->x, w6, c->prob.k0, c->prob.kmin, c->prob.penal, c->st, c->stream);
    launch_filter(c->n, c->prob.filter_radius, c->st, c->sens, c->stream);
    if (c->prob.symmetry == OTM_SYM_CENTRAL) launch_sym_central(c->n, c->sens, c->stream);
    (void)hipEventRecord(c->ev[5], c->stream);
    int rc = check_launch(c, "sensitivity");
    if (rc) return rc;
    c->have_sens = true;
    return OTM_OK;
}

int oc_update(otm_ctx* c, double vstar, double move, double* lambda_out) {
    if (!c->have_sens) return fail(c, OTM_ESTATE, "OC update needs sensitivities");
    if (!std::isfinite(vstar)) return fail(c, OTM_EINVAL, "non-finite V*");
    const Workspace w = c->ws();
    const int n = c->n;
    (void)hipEventRecord(c->ev[5], c->stream);
    int prep_blocks = 0;
    launch_oc_prepare(n, c->rho, c->sens, c->oc.eta, move, c->oc.rho_min, c->ocq, w, c->stream, &prep_blocks);
    launch_oc_init(vstar, n, c->oc.eta, prep_blocks, w, c->stream);
    const int max_passes = kOcMaxPasses;
    int rc;
    for (int pass = 0; pass < max_passes; pass += 4) {
        for (int q = 0; q < 4; ++q) launch_oc_pass(n, c->rho, c->ocq, move, c->oc.rho_min, c->oc.eta, w, c->stream);
        if ((rc = check_launch(c, "oc pass"))) return rc;
        if ((rc = sync_scalars(c))) return rc;
        if (c->h_sc->oc_done) break;
    }
    launch_oc_apply(n, c->rho, c->ocq, c->oc.eta, move, c->oc.rho_min, w, c->stream);
    (void)hipEventRecord(c->ev[6], c->stream);
    if ((rc = check_launch(c, "oc apply"))) return rc;
    if ((rc = sync_scalars(c))) return rc;
    c->timings[4] = ev_ms(c, 5, 6);
    if (lambda_out) *lambda_out = c->h_sc->lam;
    c->homogenized = false;
    c->have_sens = false;
    c->prepared = false;
    return OTM_OK;
}

int free_all(otm_ctx* c) {
    void* bufs[] = {c->rho, c->rhof, c->k, c->dinv, c->b, c->x, c->st, c->sens, c->ocq, c->r64, c->p64[0], c->p64[1],
                    c->q64, c->k32, c->dinv32, c->x32, c->r32, c->p32[0], c->p32[1], c->q32, c->partials, c->counter,
                    c->sc, c->r64b, c->q64b, c->r32b, c->q32b};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    for (void* p : c->mg_bufs)
        if (p) (void)hipFree(p);
    if (c->mg_exec) (void)hipGraphExecDestroy(c->mg_exec);
    if (c->mg_graph) (void)hipGraphDestroy(c->mg_graph);
    if (c->h_sc) (void)hipHostFree(c->h_sc);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : c->pev)
        if (e) (void)hipEventDestroy(e);
    if (c->cev) (void)hipEventDestroy(c->cev);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    return 0;
}

// ------------------------------------------------------------------ multigrid
// Levels n, n/2, ... while the side is even and above 4; the coarsest side
// must end at 3 or 4 (at most 64 nodes, solved directly), with at least one
// level above it.
int mg_levels(int n, int* ns) {
    int L = 0, m = n;
    ns[L++] = m;
    while (m % 2 == 0 && m > 4 && L < kMgMaxLevels) {
        m /= 2;
        ns[L++] = m;
    }
    if (m > 4 || L < 2) return 0;
    return L;
}

template <typename T>
int mg_alloc(otm_ctx* c, T** p, int64_t count) {
    int rc = dalloc(c, p, count);
    if (!rc) c->mg_bufs.push_back((void*)*p);
    return rc;
}

// Buffers of every level and the captured V-cycle (fixed pointers).
int mg_build(otm_ctx* c) {
    MgHierarchy& H = c->mg;
    int ns[kMgMaxLevels];
    H.levels = mg_levels(c->n, ns);
    if (!H.levels) return fail(c, OTM_EINVAL, "multigrid needs n = m 2^j with m in {3, 4} and n >= 6");
    H.sweeps = c->so.mg_sweeps;
    H.coarse_sweeps = c->so.mg_coarse_sweeps > 0 ? c->so.mg_coarse_sweeps : c->so.mg_sweeps;
    H.gs = c->so.mg_smoother == OTM_MG_GS8;
    int rc = OTM_OK;
    for (int l = 0; l < H.levels && !rc; ++l) {
        MgLevel& a = H.lv[l];
        a.n = ns[l];
        const int64_t m = (int64_t)a.n * a.n * a.n;
        rc = rc ? rc : mg_alloc(c, &a.x[0], 3 * m);
        rc = rc ? rc : mg_alloc(c, &a.x[1], 3 * m);
        rc = rc ? rc : mg_alloc(c, &a.t, 3 * m);
        if (l == 0) {
            a.k = c->k32;
            a.dinv = c->dinv32;
            a.f = c->r32;
        } else {
            rc = rc ? rc : mg_alloc(c, &a.kc, m);
            rc = rc ? rc : mg_alloc(c, &a.dinvc, m);
            rc = rc ? rc : mg_alloc(c, &a.f, 3 * m);
            a.k = a.kc;
            a.dinv = a.dinvc;
        }
        a.tile = choose_tile2(a.n, c->max_blocks, 0, 0);
    }
    rc = rc ? rc : mg_alloc(c, &H.minv, (int64_t)kMgCoarseMax * kMgCoarseMax);
    if (c->so.precision == OTM_MIXED) {
        rc = rc ? rc : mg_alloc(c, &c->ones32, c->nn);
    } else {
        rc = rc ? rc : mg_alloc(c, &c->ones64, c->nn);
    }
    if (rc) return rc;
    if (c->ones32) launch_fill_const<float>(c->ones32, c->nn, 1.0f, c->stream);
    if (c->ones64) launch_fill_const<double>(c->ones64, c->nn, 1.0, c->stream);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // capture on a private stream (the context's may be the legacy default stream)
    hipStream_t cs = nullptr;
    HIPCHK(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        c->mg_nb = mg_vcycle(H, c->partials, c->max_blocks, cs, &c->mg_z);
        e = hipStreamEndCapture(cs, &c->mg_graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&c->mg_exec, c->mg_graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, OTM_EDEVICE, std::string("multigrid graph capture: ") + hipGetErrorString(e));
    }
    return OTM_OK;
}

// ------------------------------------------------------------------ autotune
// Picks the PCG iteration scheme and operator kernel for this n and precision
// by timing them on the context's own buffers: the fused single pass (even n),
// or a direction+operator pass (two-node or one-node z-march) followed by the
// vector update, over tile widths and march lengths.  Results are cached per
// process and, with OTM_TUNE_CACHE set, in that file (per architecture).  A
// candidate displaces the best so far only when it is more than 2 % faster,
// so near-ties resolve to the earlier candidate instead of to timing noise.
struct TuneChoice {
    bool pair, fused, chain;
    int tx, tz;
    double us;  // one PCG iteration (passes and finalizes)
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int>, TuneChoice> g_tune_cache;
constexpr double kTuneMargin = 0.98;

template <typename F>
double time_us(otm_ctx* c, F run, int reps) {
    run();
    run();
    (void)hipEventRecord(c->ev[6], c->stream);
    for (int i = 0; i < reps; ++i) run();
    (void)hipEventRecord(c->ev[7], c->stream);
    if (hipEventSynchronize(c->ev[7]) != hipSuccess) {
        (void)hipGetLastError();
        return 1e30;
    }
    return 1000.0 * ev_ms(c, 6, 7) / reps;
}

void apply_choice(otm_ctx* c, const TuneChoice& ch) {
    c->use_pair = ch.pair;
    c->use_fused = ch.fused;
    c->fused_chain = ch.chain;
    if (ch.pair)
        c->tile2 = choose_tile2(c->n, c->max_blocks, ch.tz, ch.tx);
    else
        c->tile = choose_tile(c->n, c->max_blocks, ch.tz, ch.tx);
}

// Scalar state for timing: every load active with a non-zero step and
// direction weight, so each candidate does its full work.
int upload_timing_scalars(otm_ctx* c) {
    const size_t head = offsetof(Scalars, sum_rho);
    std::memset(c->h_sc, 0, head);
    for (int l = 0; l < 3; ++l) {
        c->h_sc->active[l] = 1;
        c->h_sc->alpha[l] = 0.5;
        c->h_sc->beta[l] = 0.5;
        c->h_sc->rz[l] = 1.0;
    }
    HIPCHK(c, hipMemcpyAsync(c->sc, c->h_sc, head, hipMemcpyHostToDevice, c->stream));
    return OTM_OK;
}

template <typename T>
int tune_precision(otm_ctx* c, T* r, T* rb, T* q, T* qb, T* p0, T* p1, T* x, T* dinv, T* k, TuneChoice& best) {
    const Workspace w = c->ws();
    const int n = c->n;
    const int reps = c->nn >= (1 << 20) ? 6 : 12;
    const int tzs[] = {4, 8, 16, 32};
    int rc;
    best = TuneChoice{false, false, false, 32, 8, 1e30};
    // fused candidates: a finalize after every pass, or chains of passes that
    // reduce their predecessor's sums (closing finalize amortized over the
    // check interval)
    double fin_us = 0.0, upd_us = 0.0;
    if ((rc = upload_timing_scalars(c))) return rc;
    if (rb && qb) {
        fin_us = time_us(c, [&]() { launch_finalize(FIN_PQ, 512, w, c->stream); }, reps);
        if ((rc = upload_timing_scalars(c))) return rc;
        for (int chain = 0; chain < 2; ++chain)
            for (int tx : {64, 32})
                for (int tz : tzs) {
                    if (tz > n) continue;
                    const TileShape t = choose_tile2(n, c->max_blocks, tz, tx);
                    if (t.tz != tz || t.blocks > c->max_blocks) continue;
                    int par = 0, calls = 0;
                    double us = time_us(
                        c,
                        [&]() {
                            T* ri = par ? rb : r;
                            T* ro = par ? r : rb;
                            T* qi = par ? qb : q;
                            T* qo = par ? q : qb;
                            T* pi = par ? p1 : p0;
                            T* po = par ? p0 : p1;
                            launch_fused<T>(n, t, true, ri, qi, pi, ro, qo, po, x, dinv, k, w, c->stream, par,
                                            chain && calls > 0, !chain);
                            par ^= 1;
                            ++calls;
                        },
                        reps);
                    if (chain) us += fin_us / c->so.check_every;
                    if (us < kTuneMargin * best.us) best = TuneChoice{true, true, chain != 0, tx, tz, us};
                    if ((rc = upload_timing_scalars(c))) return rc;
                }
        upd_us = time_us(c, [&]() { launch_update_vec<T>(n, x, r, p0, q, dinv, w, c->stream, false); }, reps);
        if ((rc = upload_timing_scalars(c))) return rc;
    }
    // direction+operator pass (its finalize included) + update + finalize
    std::vector<std::tuple<bool, int, int>> cands;
    if (n % 2 == 0)
        for (int tx : {32, 64})
            for (int tz : tzs)
                if (tz <= n) cands.emplace_back(true, tx, tz);
    for (int tx : {16, 32, 64})
        for (int tz : tzs)
            if (tz <= n) cands.emplace_back(false, tx, tz);
    for (auto& cd : cands) {
        const bool pair = std::get<0>(cd);
        const int tx = std::get<1>(cd), tz = std::get<2>(cd);
        const TileShape t = pair ? choose_tile2(n, c->max_blocks, tz, tx) : choose_tile(n, c->max_blocks, tz, tx);
        if (t.tz != tz || t.blocks > c->max_blocks) continue;
        const double us = time_us(
                              c,
                              [&]() {
                                  if (pair)
                                      launch_dir_march2<T>(n, t, true, r, dinv, p0, p1, k, q, w, c->stream);
                                  else
                                      launch_dir_march<T>(n, t, r, dinv, p0, p1, k, q, w, c->stream);
                              },
                              reps) +
                          upd_us + fin_us;
        if (us < kTuneMargin * best.us) best = TuneChoice{pair, false, false, tx, tz, us};
    }
    return check_launch(c, "autotune");
}

std::string tune_key(const otm_ctx* c) {
    return "context_n" + std::to_string(c->n) + (c->so.precision == OTM_MIXED ? "_mixed" : "_fp64");
}

// A stored choice is used only if this context could have picked it itself.
bool choice_valid(const otm_ctx* c, const TuneChoice& ch, bool have_fused_bufs) {
    if (ch.chain && !ch.fused) return false;
    if (ch.fused && (!ch.pair || !have_fused_bufs)) return false;
    if (ch.pair && (c->n % 2 != 0 || (ch.tx != 32 && ch.tx != 64))) return false;
    if (!ch.pair && ch.tx != 16 && ch.tx != 32 && ch.tx != 64) return false;
    if (ch.tz != 4 && ch.tz != 8 && ch.tz != 16 && ch.tz != 32) return false;
    if (ch.tz > c->n) return false;
    const TileShape t = ch.pair ? choose_tile2(c->n, c->max_blocks, ch.tz, ch.tx)
                                : choose_tile(c->n, c->max_blocks, ch.tz, ch.tx);
    return t.tz == ch.tz && t.blocks <= c->max_blocks;
}

int autotune(otm_ctx* c) {
    const int prec = c->so.precision;
    const auto key = std::make_tuple(c->n, prec);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            apply_choice(c, it->second);
            return OTM_OK;
        }
    }
    const bool mixed = prec == OTM_MIXED;
    const bool fused_bufs = mixed ? (c->r32b && c->q32b) : (c->r64b && c->q64b);
    {
        std::vector<double> v(6);
        if (tune_cache_lookup(tune_key(c), v)) {
            const TuneChoice ch{v[0] != 0.0, v[1] != 0.0, v[2] != 0.0, (int)v[3], (int)v[4], v[5]};
            if (choice_valid(c, ch, fused_bufs)) {
                apply_choice(c, ch);
                c->tune_us = ch.us;
                std::lock_guard<std::mutex> g(g_tune_mu);
                g_tune_cache[key] = ch;
                return OTM_OK;
            }
        }
    }
    // zeroed vectors and coefficients: every candidate computes on zeros
    const size_t es = mixed ? sizeof(float) : sizeof(double);
    const size_t v3 = 3 * (size_t)c->nn * es;
    void* vecs[] = {mixed ? (void*)c->r32 : (void*)c->r64, mixed ? (void*)c->q32 : (void*)c->q64,
                    mixed ? (void*)c->r32b : (void*)c->r64b, mixed ? (void*)c->q32b : (void*)c->q64b,
                    mixed ? (void*)c->p32[0] : (void*)c->p64[0], mixed ? (void*)c->p32[1] : (void*)c->p64[1],
                    mixed ? (void*)c->x32 : nullptr};
    for (void* v : vecs)
        if (v) HIPCHK(c, hipMemsetAsync(v, 0, v3, c->stream));
    // a residual of hashed values, unit conductivities and a constant diagonal:
    // the timed passes are genuine iterations (non-zero steps, all loads active)
    if (mixed) {
        launch_fill_hash<float>(c->r32, 3 * c->nn, 12345u, c->stream);
        launch_fill_const<float>(c->k32, c->nn, 1.0f, c->stream);
        launch_fill_const<float>(c->dinv32, c->nn, 0.375f, c->stream);
    } else {
        launch_fill_hash<double>(c->r64, 3 * c->nn, 12345u, c->stream);
        launch_fill_const<double>(c->k, c->nn, 1.0, c->stream);
        launch_fill_const<double>(c->dinv, c->nn, 0.375, c->stream);
    }
    // FP64 timing updates a scratch x: the solution buffer is restored below
    TuneChoice best;
    int rc;
    if (mixed)
        rc = tune_precision<float>(c, c->r32, c->r32b, c->q32, c->q32b, c->p32[0], c->p32[1], c->x32, c->dinv32,
                                   c->k32, best);
    else
        rc = tune_precision<double>(c, c->r64, c->r64b, c->q64, c->q64b, c->p64[0], c->p64[1], c->x, c->dinv, c->k,
                                    best);
    if (rc) return rc;
    for (void* v : vecs)
        if (v) HIPCHK(c, hipMemsetAsync(v, 0, v3, c->stream));
    HIPCHK(c, hipMemsetAsync(c->x, 0, 3 * (size_t)c->nn * sizeof(double), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    apply_choice(c, best);
    c->tune_us = best.us;
    tune_cache_store(tune_key(c), {best.pair ? 1.0 : 0.0, best.fused ? 1.0 : 0.0, best.chain ? 1.0 : 0.0,
                                   (double)best.tx, (double)best.tz, best.us});
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = best;
    return OTM_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

void otm_default_options(otm_solver_opts* s, otm_oc_opts* o, otm_governor_opts* g) {
    if (s) {
        s->precision = OTM_FP64;
        s->guess = OTM_GUESS_ZERO;
        s->tol = 1e-8;
        s->max_iter = 20000;
        s->check_every = 16;
        s->reliable_delta = 1e-2;
        s->kernel_variant = 0;
        s->tile_tz = 0;
        s->tile_tx = 0;
        s->autotune = 1;
        s->preconditioner = OTM_PRECOND_JACOBI;
        s->mg_sweeps = 1;
        s->mg_coarse_sweeps = 2;
        s->stall_window = 0;
        s->mg_smoother = OTM_MG_JACOBI;
    }
    if (o) {
        o->move = 0.05;
        o->eta = 0.5;
        o->rho_min = 1e-3;
        o->move_min = 0.0;
    }
    if (g) {
        g->bound = 1e-4;
        g->dg_small = 1e-6;
        g->dv_small = 1e-3;
        g->decay = 0.8;
        g->rebound = 0.3;
        g->g_tol = 1e-6;
        g->patience = 5;
        g->stall_iters = 3;
    }
}

const char* otm_version(void) { return OTM_VERSION; }

const char* otm_strerror(int s) {
    switch (s) {
        case OTM_OK: return "ok";
        case OTM_NOT_CONVERGED: return "solver did not converge (outputs filled)";
        case OTM_EINVAL: return "invalid argument";
        case OTM_ENOMEM: return "out of memory";
        case OTM_EDEVICE: return "HIP device error";
        case OTM_ENONFINITE: return "non-finite value";
        case OTM_EUNSUPPORTED: return "unsupported";
        case OTM_ESTATE: return "call order violated";
        case OTM_EIO: return "file could not be opened, read or written, or is malformed";
        default: return "unknown status";
    }
}

const char* otm_last_error(const otm_ctx* c) { return c ? c->err.c_str() : "null context"; }

int otm_create(const otm_problem* problem, const otm_solver_opts* solver, const otm_oc_opts* oc,
               const otm_governor_opts* gov, void* stream, otm_ctx** out) {
    if (!out) return OTM_EINVAL;
    *out = nullptr;
    std::string why;
    int rc = validate_problem(problem, why);
    if (rc) return rc;
    otm_ctx* c = new (std::nothrow) otm_ctx();
    if (!c) return OTM_ENOMEM;
    c->prob = *problem;
    otm_default_options(&c->so, &c->oc, &c->go);
    if (solver) c->so = *solver;
    if (oc) c->oc = *oc;
    if (gov) c->go = *gov;
    if (!(c->so.tol > 0.0 && c->so.max_iter > 0 && c->so.check_every >= 1 && c->so.reliable_delta > 0.0 &&
          c->so.reliable_delta < 1.0 && (c->so.precision == OTM_FP64 || c->so.precision == OTM_MIXED) &&
          c->so.guess >= OTM_GUESS_ZERO && c->so.guess <= OTM_GUESS_LEARNED &&
          c->so.kernel_variant >= 0 && c->so.kernel_variant <= 5 && c->so.tile_tz >= 0 && c->so.stall_window >= 0 &&
          (c->so.tile_tx == 0 || c->so.tile_tx == 16 || c->so.tile_tx == 32 || c->so.tile_tx == 64) &&
          (c->so.preconditioner == OTM_PRECOND_JACOBI || c->so.preconditioner == OTM_PRECOND_MG))) {
        delete c;
        return OTM_EINVAL;
    }
    if (c->so.preconditioner == OTM_PRECOND_MG) {
        int ns[kMgMaxLevels];
        if (c->so.kernel_variant != 0 || c->so.mg_sweeps < 1 ||
            c->so.mg_sweeps > 8 || c->so.mg_coarse_sweeps < 0 || c->so.mg_coarse_sweeps > 8 || (c->so.tile_tx != 0 && c->so.tile_tx != 32 && c->so.tile_tx != 64) ||
            (c->so.mg_smoother != OTM_MG_JACOBI && c->so.mg_smoother != OTM_MG_GS8) ||
            !mg_levels(problem->n, ns)) {
            delete c;
            return OTM_EINVAL;
        }
        c->use_mg = true;
    }
    if (!(c->oc.move > 0.0 && c->oc.eta > 0.0 && c->oc.rho_min > 0.0 && c->oc.rho_min < 1.0 &&
          c->oc.move_min >= 0.0 && c->oc.move_min <= c->oc.move) ||
        !governor_opts_valid(c->go)) {
        delete c;
        return OTM_EINVAL;
    }
    c->n = problem->n;
    c->nn = (int64_t)c->n * c->n * c->n;
    // device check: this library carries gfx950 code only
    hipDeviceProp_t prop;
    if (hipGetDevice(&c->device) != hipSuccess || hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return OTM_EDEVICE;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        delete c;
        return OTM_EDEVICE;
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return OTM_EDEVICE;
        }
        c->own_stream = true;
    }
    const int64_t nn = c->nn;
    c->max_blocks = kMaxBlocks;
    c->tile = choose_tile(c->n, c->max_blocks, c->so.tile_tz, c->so.tile_tx);
    c->tile2 = choose_tile2(c->n, c->max_blocks, c->so.tile_tz, c->so.tile_tx);
    c->use_pair = (c->so.kernel_variant == 0 || c->so.kernel_variant >= 4) && (c->n % 2 == 0);
    c->use_fused = (c->so.kernel_variant >= 4);
    c->fused_chain = (c->so.kernel_variant == 5);
    if (c->use_fused && c->n % 2 != 0) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return OTM_EINVAL;
    }
    // the fused iteration needs second r, q buffers (automatic choice or forced)
    const bool fused_bufs = c->use_pair && (c->so.kernel_variant >= 4 || (c->so.kernel_variant == 0 && c->so.autotune &&
                                                                        c->so.tile_tx == 0 && c->so.tile_tz == 0));
    rc = OTM_OK;
    rc = rc ? rc : dalloc(c, &c->rho, nn);
    rc = rc ? rc : dalloc(c, &c->rhof, nn);
    rc = rc ? rc : dalloc(c, &c->k, nn);
    rc = rc ? rc : dalloc(c, &c->dinv, nn);
    rc = rc ? rc : dalloc(c, &c->b, 3 * nn);
    rc = rc ? rc : dalloc(c, &c->x, 3 * nn);
    rc = rc ? rc : dalloc(c, &c->st, nn);
    rc = rc ? rc : dalloc(c, &c->sens, nn);
    rc = rc ? rc : dalloc(c, &c->ocq, nn);
    if (c->so.precision == OTM_FP64) {
        if (c->use_mg) {  // the V-cycle runs in float32: its level-0 inputs
            rc = rc ? rc : dalloc(c, &c->k32, nn);
            rc = rc ? rc : dalloc(c, &c->dinv32, nn);
            rc = rc ? rc : dalloc(c, &c->r32, 3 * nn);
        }
        rc = rc ? rc : dalloc(c, &c->r64, 3 * nn);
        rc = rc ? rc : dalloc(c, &c->p64[0], 3 * nn);
        rc = rc ? rc : dalloc(c, &c->p64[1], 3 * nn);
        rc = rc ? rc : dalloc(c, &c->q64, 3 * nn);
        if (fused_bufs) {
            rc = rc ? rc : dalloc(c, &c->r64b, 3 * nn);
            rc = rc ? rc : dalloc(c, &c->q64b, 3 * nn);
        }
    } else {
        rc = rc ? rc : dalloc(c, &c->k32, nn);
        rc = rc ? rc : dalloc(c, &c->dinv32, nn);
        rc = rc ? rc : dalloc(c, &c->x32, 3 * nn);
        rc = rc ? rc : dalloc(c, &c->r32, 3 * nn);
        rc = rc ? rc : dalloc(c, &c->p32[0], 3 * nn);
        rc = rc ? rc : dalloc(c, &c->p32[1], 3 * nn);
        rc = rc ? rc : dalloc(c, &c->q32, 3 * nn);
        if (fused_bufs) {
            rc = rc ? rc : dalloc(c, &c->r32b, 3 * nn);
            rc = rc ? rc : dalloc(c, &c->q32b, 3 * nn);
        }
    }
    rc = rc ? rc : dalloc(c, &c->partials, (int64_t)c->max_blocks * kMaxReduce);
    rc = rc ? rc : dalloc(c, &c->counter, 64);
    rc = rc ? rc : dalloc(c, &c->sc, (int64_t)sizeof(Scalars));
    if (!rc && hipHostMalloc((void**)&c->h_sc, sizeof(Scalars), hipHostMallocDefault) != hipSuccess) rc = OTM_ENOMEM;
    for (int q = 0; q < 8 && !rc; ++q)
        if (hipEventCreate(&c->ev[q]) != hipSuccess) rc = OTM_EDEVICE;
    for (int q = 0; q < 2 && !rc; ++q)
        if (hipEventCreate(&c->pev[q]) != hipSuccess) rc = OTM_EDEVICE;
    if (!rc && hipEventCreateWithFlags(&c->cev, hipEventDisableTiming) != hipSuccess) rc = OTM_EDEVICE;
    if (rc) {
        free_all(c);
        delete c;
        return rc;
    }
    launch_fill_u32(c->counter, 64, 0u, c->stream);
    (void)hipMemsetAsync(c->x, 0, (size_t)3 * nn * sizeof(double), c->stream);
    if (c->p64[0]) {
        (void)hipMemsetAsync(c->p64[0], 0, (size_t)3 * nn * sizeof(double), c->stream);
        (void)hipMemsetAsync(c->p64[1], 0, (size_t)3 * nn * sizeof(double), c->stream);
    }
    if (c->p32[0]) {
        (void)hipMemsetAsync(c->p32[0], 0, (size_t)3 * nn * sizeof(float), c->stream);
        (void)hipMemsetAsync(c->p32[1], 0, (size_t)3 * nn * sizeof(float), c->stream);
        (void)hipMemsetAsync(c->x32, 0, (size_t)3 * nn * sizeof(float), c->stream);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        free_all(c);
        delete c;
        return OTM_EDEVICE;
    }
    if (c->use_mg) {
        rc = mg_build(c);
        if (rc) {
            free_all(c);
            delete c;
            return rc;
        }
    }
    if (!c->use_mg && c->so.kernel_variant == 0 && c->so.tile_tx == 0 && c->so.tile_tz == 0 && c->so.autotune) {
        rc = autotune(c);
        if (rc) {
            free_all(c);
            delete c;
            return rc;
        }
    }
    c->vb.vstar = problem->vf;
    *out = c;
    return OTM_OK;
}

void otm_destroy(otm_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

static int set_density_common(otm_ctx* c) {
    launch_clamp(c->n, c->rho, c->oc.rho_min, 1.0, c->stream);
    int rc = check_launch(c, "clamp");
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_density = true;
    c->prepared = c->homogenized = c->have_sens = false;
    return OTM_OK;
}

int otm_set_density(otm_ctx* c, const double* rho, int64_t count) {
    if (!c || !rho) return OTM_EINVAL;
    if (count != c->nn) return fail(c, OTM_EINVAL, "density count must be n^3");
    for (int64_t e = 0; e < count; ++e)
        if (!std::isfinite(rho[e])) return fail(c, OTM_ENONFINITE, "non-finite density value");
    HIPCHK(c, hipMemcpyAsync(c->rho, rho, (size_t)count * sizeof(double), hipMemcpyHostToDevice, c->stream));
    return set_density_common(c);
}

int otm_set_density_device(otm_ctx* c, const void* rho_dev, int64_t count) {
    if (!c || !rho_dev) return OTM_EINVAL;
    if (count != c->nn) return fail(c, OTM_EINVAL, "density count must be n^3");
    HIPCHK(c, hipMemcpyAsync(c->rho, rho_dev, (size_t)count * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return set_density_common(c);
}

int otm_prepare(otm_ctx* c) {
    if (!c) return OTM_EINVAL;
    int rc = prepare(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return OTM_OK;
}

int otm_homogenize(otm_ctx* c, double kappa6[6], otm_solve_stats* stats) {
    if (!c) return OTM_EINVAL;
    return homogenize(c, kappa6, stats);
}

int otm_sensitivity(otm_ctx* c, const double dg_dkappa6[6], double* out) {
    if (!c || !dg_dkappa6) return OTM_EINVAL;
    int rc = sensitivity(c, dg_dkappa6);
    if (rc) return rc;
    if (out) HIPCHK(c, hipMemcpyAsync(out, c->sens, (size_t)c->nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return OTM_OK;
}

int otm_oc_update(otm_ctx* c, double vstar, double* rho_out, double* lambda_out) {
    if (!c) return OTM_EINVAL;
    int rc = oc_update(c, vstar, c->oc.move, lambda_out);
    if (rc) return rc;
    if (rho_out) HIPCHK(c, hipMemcpyAsync(rho_out, c->rho, (size_t)c->nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return OTM_OK;
}

int otm_step(otm_ctx* c, otm_iter_record* rec) {
    if (!c) return OTM_EINVAL;
    auto t0 = std::chrono::steady_clock::now();
    otm_solve_stats st{};
    int hrc = homogenize(c, nullptr, &st);
    if (hrc < 0) return hrc;
    double g, w6[6];
    objective_grad(c->prob.objective, c->kappa, c->prob.target, &g, w6);
    c->g = g;
    std::memcpy(c->w, w6, sizeof(w6));
    int rc = sensitivity(c, w6);
    if (rc) return rc;
    const double vol = c->volume, low = c->low_bound;
    const double move = next_move(c->oc, c->vb, g);
    advance_volume_bound(c->go, c->oc.rho_min, c->vb, g, low, vol);
    const double vstar = c->vb.vstar;
    double lam = 0.0;
    rc = oc_update(c, vstar, move, &lam);
    if (rc) return rc;
    c->timings[3] = ev_ms(c, 4, 5);
    auto t1 = std::chrono::steady_clock::now();
    c->timings[5] = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (rec) {
        rec->iter = c->iter;
        rec->g = g;
        std::memcpy(rec->kappa, c->kappa, sizeof(c->kappa));
        rec->volume = vol;
        rec->low_bound = low;
        rec->vstar = vstar;
        rec->lambda = lam;
        for (int l = 0; l < 3; ++l) {
            rec->pcg_iters[l] = st.iterations[l];
            rec->rel_residual[l] = st.rel_residual[l];
        }
        rec->ms_total = c->timings[5];
        rec->ms_solve = st.ms_solve;
        rec->stop = c->vb.flat >= c->go.stall_iters ? 1 : 0;
        rec->move = move;
        rec->stalled = st.stalled;
    }
    c->iter += 1;
    return hrc;
}

int otm_optimize(otm_ctx* c, int32_t max_iter, double* rho_out, otm_iter_record* log, int32_t cap, int32_t* done) {
    if (!c || max_iter < 0) return OTM_EINVAL;
    int it = 0, last = OTM_OK;
    for (; it < max_iter; ++it) {
        otm_iter_record r{};
        int rc = otm_step(c, &r);
        if (rc < 0) return rc;
        last = rc;
        if (log && it < cap) log[it] = r;
        if (r.stop) {
            ++it;
            break;
        }
    }
    if (done) *done = it;
    if (rho_out) {
        HIPCHK(c, hipMemcpyAsync(rho_out, c->rho, (size_t)c->nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return last;
}

int otm_get_field(otm_ctx* c, int32_t field, double* out, int64_t count) {
    if (!c || !out) return OTM_EINVAL;
    const double* src = nullptr;
    int64_t size = c->nn;
    switch (field) {
        case OTM_FIELD_RHO: src = c->rho; break;
        case OTM_FIELD_RHOF: src = c->rhof; break;
        case OTM_FIELD_K: src = c->k; break;
        case OTM_FIELD_B: src = c->b; size = 3 * c->nn; break;
        case OTM_FIELD_DIAG: src = c->dinv; break;
        case OTM_FIELD_CHI: src = c->x; size = 3 * c->nn; break;
        case OTM_FIELD_SENS_ELEM: src = c->st; break;
        case OTM_FIELD_SENS: src = c->sens; break;
        default: return fail(c, OTM_EINVAL, "unknown field");
    }
    if (count != size) return fail(c, OTM_EINVAL, "field count mismatch");
    HIPCHK(c, hipMemcpyAsync(out, src, (size_t)size * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (field == OTM_FIELD_DIAG)
        for (int64_t v = 0; v < size; ++v) out[v] = 1.0 / out[v];
    return OTM_OK;
}

int otm_set_field(otm_ctx* c, int32_t field, const double* in, int64_t count) {
    if (!c || !in) return OTM_EINVAL;
    if (field == OTM_FIELD_RHO) return otm_set_density(c, in, count);
    const int64_t size = field == OTM_FIELD_CHI ? 3 * c->nn : c->nn;
    if (field != OTM_FIELD_CHI && field != OTM_FIELD_SENS) return fail(c, OTM_EINVAL, "field is not settable");
    if (count != size) return fail(c, OTM_EINVAL, "field count mismatch");
    for (int64_t v = 0; v < count; ++v)
        if (!std::isfinite(in[v])) return fail(c, OTM_ENONFINITE, "non-finite field value");
    if (field == OTM_FIELD_CHI && !c->prepared) return fail(c, OTM_ESTATE, "set chi needs prepared conductivities");
    double* dst = field == OTM_FIELD_CHI ? c->x : c->sens;
    HIPCHK(c, hipMemcpyAsync(dst, in, (size_t)size * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (field == OTM_FIELD_CHI) {
        c->homogenized = true;
        c->have_sens = false;
    } else {
        c->have_sens = true;
    }
    return OTM_OK;
}

int otm_set_guess(otm_ctx* c, const double* chi, int64_t count) {
    if (!c || !chi) return OTM_EINVAL;
    if (count != 3 * c->nn) return fail(c, OTM_EINVAL, "guess count must be 3 n^3");
    for (int64_t v = 0; v < count; ++v)
        if (!std::isfinite(chi[v])) return fail(c, OTM_ENONFINITE, "non-finite guess");
    HIPCHK(c, hipMemcpyAsync(c->x, chi, (size_t)count * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_user_guess = true;
    return OTM_OK;
}

int otm_get_governor(const otm_ctx* c, double s[8]) {
    if (!c || !s) return OTM_EINVAL;
    s[0] = c->vb.vstar;
    s[1] = c->vb.df;
    s[2] = (double)c->vb.stalls;
    s[3] = c->vb.gap;
    s[4] = c->vb.g_prev;
    s[5] = (double)c->vb.flat;
    s[6] = (double)c->iter;
    s[7] = c->vb.move;
    return OTM_OK;
}

int otm_set_governor(otm_ctx* c, const double s[8]) {
    if (!c || !s) return OTM_EINVAL;
    for (int q = 0; q < 8; ++q)
        if (!std::isfinite(s[q])) return fail(c, OTM_ENONFINITE, "non-finite governor state");
    c->vb.vstar = s[0];
    c->vb.df = s[1];
    c->vb.stalls = (int)s[2];
    c->vb.gap = s[3];
    c->vb.g_prev = s[4];
    c->vb.flat = (int)s[5];
    c->iter = (int)s[6];
    c->vb.move = s[7] > 0.0 ? s[7] : 0.0;
    return OTM_OK;
}

// ---- checkpoint / resume -----------------------------------------------------
// A design run's state, in one little-endian binary file written here:
//   "OTMSTATE" | u32 version 2 | i32 n | u32 flags (bit 0: solution present) |
//   u32 0 | f64 problem[11] (k0, kmin, penal, filter radius, target[6],
//   objective) | f64 governor[8] (as otm_get_governor) | f64 the objective's
//   last change (the adaptive OC step's memory) | f64 rho[n^3] |
//   f64 chi[3 n^3] if bit 0 | u64 FNV-1a hash of every preceding byte.
// Version 1 files (without the objective's last change, read as 0) load too.
// The file is written under path.tmp and renamed over path, so a crash while
// saving leaves any earlier checkpoint whole.
namespace {

const char kStateMagic[8] = {'O', 'T', 'M', 'S', 'T', 'A', 'T', 'E'};
constexpr uint32_t kStateVersion = 2;

}  // namespace

int otm_save_state(otm_ctx* c, const char* path) {
    if (!c || !path || !path[0]) return OTM_EINVAL;
    if (!c->have_density) return fail(c, OTM_ESTATE, "no density to save");
    std::vector<double> rho((size_t)c->nn), chi;
    HIPCHK(c, hipMemcpyAsync(rho.data(), c->rho, (size_t)c->nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (c->have_solution) {
        chi.resize((size_t)(3 * c->nn));
        HIPCHK(c, hipMemcpyAsync(chi.data(), c->x, chi.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const uint32_t version = kStateVersion, flags = c->have_solution ? 1u : 0u, zero = 0u;
    const int32_t n = c->n;
    double sig[11], gov[8];
    problem_signature(c->prob, sig);
    otm_get_governor(c, gov);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(c, OTM_EIO, "cannot open " + tmp + " for writing");
    Fnv1a h;
    bool ok = true;
    auto put = [&](const void* p, size_t len) {
        if (!ok || len == 0) return;
        h.add(p, len);
        ok = std::fwrite(p, 1, len, f) == len;
    };
    put(kStateMagic, 8);
    put(&version, 4);
    put(&n, 4);
    put(&flags, 4);
    put(&zero, 4);
    put(sig, sizeof(sig));
    put(gov, sizeof(gov));
    put(&c->vb.dg_prev, sizeof(double));
    put(rho.data(), rho.size() * sizeof(double));
    put(chi.data(), chi.size() * sizeof(double));
    const uint64_t digest = h.h;
    ok = ok && std::fwrite(&digest, 1, 8, f) == 8;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(c, OTM_EIO, std::string("cannot write ") + path);
    }
    return OTM_OK;
}

int otm_load_state(otm_ctx* c, const char* path) {
    if (!c || !path || !path[0]) return OTM_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(c, OTM_EIO, std::string("cannot open ") + path);
    std::vector<unsigned char> buf;
    unsigned char chunk[1 << 16];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) buf.insert(buf.end(), chunk, chunk + got);
    const bool read_err = std::ferror(f) != 0;
    std::fclose(f);
    if (read_err) return fail(c, OTM_EIO, std::string("cannot read ") + path);
    const size_t head1 = 8 + 4 * 4 + 11 * 8 + 8 * 8;
    if (buf.size() < head1 + 8 || std::memcmp(buf.data(), kStateMagic, 8) != 0)
        return fail(c, OTM_EIO, std::string(path) + " is not a state file");
    uint32_t version, flags;
    int32_t n;
    std::memcpy(&version, &buf[8], 4);
    std::memcpy(&n, &buf[12], 4);
    std::memcpy(&flags, &buf[16], 4);
    if (version != 1 && version != kStateVersion) return fail(c, OTM_EIO, "unsupported state file version");
    const size_t head = head1 + (version >= 2 ? 8 : 0);
    if (n != c->n) return fail(c, OTM_EINVAL, "state file holds another resolution");
    const size_t body = (size_t)c->nn * sizeof(double) * ((flags & 1u) ? 4 : 1);
    if (buf.size() != head + body + 8) return fail(c, OTM_EIO, "state file size does not match its header");
    Fnv1a h;
    h.add(buf.data(), head + body);
    uint64_t digest;
    std::memcpy(&digest, &buf[head + body], 8);
    if (digest != h.h) return fail(c, OTM_EIO, "state file checksum mismatch");
    double sig[11], mine[11], gov[8];
    std::memcpy(sig, &buf[24], sizeof(sig));
    std::memcpy(gov, &buf[24 + sizeof(sig)], sizeof(gov));
    problem_signature(c->prob, mine);
    if (std::memcmp(sig, mine, sizeof(sig)) != 0)
        return fail(c, OTM_EINVAL, "state file was written for another problem (constants, target or objective)");
    std::vector<double> vals((size_t)(body / sizeof(double)));
    std::memcpy(vals.data(), &buf[head], body);
    for (double v : vals)
        if (!std::isfinite(v)) return fail(c, OTM_ENONFINITE, "non-finite value in state file");
    double dg_prev = 0.0;
    if (version >= 2) std::memcpy(&dg_prev, &buf[head1], 8);
    if (!std::isfinite(dg_prev)) return fail(c, OTM_ENONFINITE, "non-finite value in state file");
    int rc = otm_set_governor(c, gov);
    if (rc) return rc;
    c->vb.dg_prev = dg_prev;
    HIPCHK(c, hipMemcpyAsync(c->rho, vals.data(), (size_t)c->nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (flags & 1u)
        HIPCHK(c, hipMemcpyAsync(c->x, vals.data() + c->nn, (size_t)(3 * c->nn) * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream));
    rc = set_density_common(c);  // synchronises the stream, so vals may go
    if (rc) return rc;
    c->have_solution = (flags & 1u) != 0;
    c->have_user_guess = false;
    return OTM_OK;
}

int otm_apply(otm_ctx* c, int32_t precision, const double* xh, double* yh) {
    if (!c || !xh || !yh) return OTM_EINVAL;
    if (!c->prepared) return fail(c, OTM_ESTATE, "apply needs prepared conductivities");
    // temporaries, freed before return: not part of what the context holds
    struct HeldBytes {
        otm_ctx* c;
        int64_t v;
        ~HeldBytes() { c->dev_bytes = v; }
    } held{c, c->dev_bytes};
    const int64_t cnt = 3 * c->nn;
    int rc = OTM_OK;
    if (precision == OTM_FP64) {
        double *xd = nullptr, *yd = nullptr;
        if ((rc = dalloc(c, &xd, cnt))) return rc;
        if ((rc = dalloc(c, &yd, cnt))) {
            (void)hipFree(xd);
            return rc;
        }
        (void)hipMemcpyAsync(xd, xh, cnt * sizeof(double), hipMemcpyHostToDevice, c->stream);
        const TileShape t = choose_tile(c->n, 1 << 30, c->so.tile_tz, c->so.tile_tx);
        if (c->so.kernel_variant == 1)
            launch_apply<double>(c->n, c->k, xd, yd, c->stream);
        else if (c->so.kernel_variant == 2)
            launch_apply_tiled<double>(c->n, t, c->k, xd, yd, c->stream);
        else if (c->use_pair)
            launch_apply_march2<double>(c->n, choose_tile2(c->n, 1 << 30, c->so.tile_tz, c->so.tile_tx), c->k, xd,
                                        yd, c->stream);
        else
            launch_apply_march<double>(c->n, t, c->k, xd, yd, c->stream);
        (void)hipMemcpyAsync(yh, yd, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        rc = check_launch(c, "apply");
        hipError_t e = hipStreamSynchronize(c->stream);
        (void)hipFree(xd);
        (void)hipFree(yd);
        if (!rc && e != hipSuccess) rc = fail(c, OTM_EDEVICE, hipGetErrorString(e));
        return rc;
    }
    if (precision != OTM_MIXED) return fail(c, OTM_EINVAL, "precision");
    double* xd = nullptr;
    float *x32 = nullptr, *y32 = nullptr, *k32 = nullptr;
    if ((rc = dalloc(c, &xd, cnt))) return rc;
    rc = rc ? rc : dalloc(c, &x32, cnt);
    rc = rc ? rc : dalloc(c, &y32, cnt);
    rc = rc ? rc : dalloc(c, &k32, c->nn);
    if (!rc) {
        (void)hipMemcpyAsync(xd, xh, cnt * sizeof(double), hipMemcpyHostToDevice, c->stream);
        launch_cast_f64_f32(cnt, xd, x32, c->stream);
        launch_cast_f64_f32(c->nn, c->k, k32, c->stream);
        const TileShape t = choose_tile(c->n, 1 << 30, c->so.tile_tz, c->so.tile_tx);
        if (c->so.kernel_variant == 1)
            launch_apply<float>(c->n, k32, x32, y32, c->stream);
        else if (c->so.kernel_variant == 2)
            launch_apply_tiled<float>(c->n, t, k32, x32, y32, c->stream);
        else if (c->use_pair)
            launch_apply_march2<float>(c->n, choose_tile2(c->n, 1 << 30, c->so.tile_tz, c->so.tile_tx), k32, x32,
                                       y32, c->stream);
        else
            launch_apply_march<float>(c->n, t, k32, x32, y32, c->stream);
        launch_cast_f32_f64(cnt, y32, xd, c->stream);
        (void)hipMemcpyAsync(yh, xd, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        rc = check_launch(c, "apply32");
        hipError_t e = hipStreamSynchronize(c->stream);
        if (!rc && e != hipSuccess) rc = fail(c, OTM_EDEVICE, hipGetErrorString(e));
    }
    if (xd) (void)hipFree(xd);
    if (x32) (void)hipFree(x32);
    if (y32) (void)hipFree(y32);
    if (k32) (void)hipFree(k32);
    return rc;
}

static int apply_device_impl(int32_t n, int32_t precision, int32_t variant, int32_t tx, int32_t tz, const void* k,
                             const void* x, void* y, void* stream) {
    if (n < 4 || n > 1024 || !k || !x || !y) return OTM_EINVAL;
    if (x == y || variant < 0 || variant > 3) return OTM_EINVAL;
    if (!(tx == 0 || tx == 16 || tx == 32 || tx == 64) || tz < 0) return OTM_EINVAL;
    if (variant == 0 && n % 2 != 0) variant = 3;
    if (variant == 0 && tx == 16) return OTM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const TileShape t = choose_tile(n, 1 << 30, tz, tx);
    const TileShape t2 = choose_tile2(n, 1 << 30, tz, tx);
    if (precision == OTM_FP64) {
        const double *kd = (const double*)k, *xd = (const double*)x;
        double* yd = (double*)y;
        if (variant == 0)
            launch_apply_march2<double>(n, t2, kd, xd, yd, s);
        else if (variant == 1)
            launch_apply<double>(n, kd, xd, yd, s);
        else if (variant == 2)
            launch_apply_tiled<double>(n, t, kd, xd, yd, s);
        else
            launch_apply_march<double>(n, t, kd, xd, yd, s);
    } else if (precision == OTM_MIXED) {
        const float *kf = (const float*)k, *xf = (const float*)x;
        float* yf = (float*)y;
        if (variant == 0)
            launch_apply_march2<float>(n, t2, kf, xf, yf, s);
        else if (variant == 1)
            launch_apply<float>(n, kf, xf, yf, s);
        else if (variant == 2)
            launch_apply_tiled<float>(n, t, kf, xf, yf, s);
        else
            launch_apply_march<float>(n, t, kf, xf, yf, s);
    } else {
        return OTM_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? OTM_OK : OTM_EDEVICE;
}

int otm_apply_device(int32_t n, int32_t precision, int32_t variant, const void* k, const void* x, void* y,
                     void* stream) {
    return apply_device_impl(n, precision, variant, 0, 0, k, x, y, stream);
}

int otm_apply_device_tiled(int32_t n, int32_t precision, int32_t variant, int32_t tx, int32_t tz, const void* k,
                           const void* x, void* y, void* stream) {
    return apply_device_impl(n, precision, variant, tx, tz, k, x, y, stream);
}

int otm_time_apply_device(int32_t n, int32_t precision, int32_t variant, int32_t tx, int32_t tz, const void* k,
                          const void* x, void* y, void* stream, int32_t reps, double* us) {
    if (reps < 1 || !us) return OTM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return OTM_EDEVICE;
    int rc = apply_device_impl(n, precision, variant, tx, tz, k, x, y, stream);  // warm
    if (rc) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return rc;
    }
    (void)hipEventRecord(a, s);
    for (int q = 0; q < reps; ++q) (void)apply_device_impl(n, precision, variant, tx, tz, k, x, y, stream);
    (void)hipEventRecord(b, s);
    if (hipEventSynchronize(b) != hipSuccess) return OTM_EDEVICE;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    *us = 1000.0 * (double)ms / (double)reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return OTM_OK;
}

int otm_set_network(otm_ctx* c, otm_nn* net) {
    if (!c) return OTM_EINVAL;
    c->net = net;
    return OTM_OK;
}

int otm_pass_timing(otm_ctx* c, int32_t reset, double out4[4]) {
    if (!c || !out4) return OTM_EINVAL;
    out4[0] = (double)c->pass_count;
    out4[1] = c->pass_count ? 1000.0 * c->pass_ms / (double)c->pass_count : 0.0;
    out4[2] = c->pass_bytes;
    out4[3] = (double)c->pass_kind;
    if (reset) {
        c->pass_ms = 0.0;
        c->pass_count = 0;
    }
    return OTM_OK;
}

int otm_get_tile(const otm_ctx* c, int32_t tile4[4]) {
    if (!c || !tile4) return OTM_EINVAL;
    const TileShape& t = c->use_pair ? c->tile2 : c->tile;
    tile4[0] = c->use_fused ? (c->fused_chain ? 5 : 4)
                            : (c->so.kernel_variant == 0 ? (c->use_pair ? 0 : 3) : c->so.kernel_variant);
    tile4[1] = t.tx;
    tile4[2] = t.tz;
    tile4[3] = t.blocks;
    return OTM_OK;
}

int otm_get_timings(const otm_ctx* c, double t8[8]) {
    if (!c || !t8) return OTM_EINVAL;
    std::memcpy(t8, c->timings, sizeof(c->timings));
    return OTM_OK;
}

int otm_device_bytes(const otm_ctx* c, int64_t* bytes) {
    if (!c || !bytes) return OTM_EINVAL;
    *bytes = c->dev_bytes;
    return OTM_OK;
}

}  // extern "C"
