// Host engine for batches of designs with uneven n (float64, or mixed
// precision: float32 operator and Krylov vectors with float64 residual
// refreshes, as a single context's OTM_MIXED solve).
//
// All designs of a batch share one set of arenas; every phase of a design
// iteration is one launch over the batch's work list (otm_kernels.hip,
// otm_stencil.hip, otm_march2.hip), with per-design device scalars and a
// per-design finalize.  A chunk of PCG iterations -- the fused single pass
// with its per-design finalize (otm_fused.hip), or the two-pass iteration
// (direction+operator pass, finalize, update, finalize) -- is captured once
// as a hipGraph and replayed until every design has converged; the
// iteration kind, tile width and march length are chosen by timing whole
// iterations of the candidates on the batch itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "opentm_amd.h"
#include "otm_internal.h"

using namespace otm;

struct otm_batch {
    int count = 0;
    int64_t dev_bytes = 0;  // device memory this batch holds
    std::vector<otm_problem> prob;
    otm_solver_opts so;
    otm_oc_opts oc;
    otm_governor_opts go;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t total = 0;
    std::vector<int64_t> off;

    // work lists
    std::vector<BatchDesc> hdesc;
    BatchDesc* ddesc = nullptr;
    int* eb_design = nullptr;
    int* mb_design = nullptr;
    int eb_cap = 0, mb_cap = 0;
    BatchTab tab{};
    int wx = 16;  // z-march tile: WX threads x TY rows (tx = 2 WX nodes)
    int march_grid = 1024, update_grid = 1024;

    // arenas
    double *rho = nullptr, *rhof = nullptr, *k = nullptr, *dinv = nullptr, *b = nullptr, *x = nullptr;
    double *st = nullptr, *sens = nullptr, *ocq = nullptr, *r = nullptr, *p[2] = {nullptr, nullptr}, *q = nullptr;
    double *r2 = nullptr, *q2 = nullptr;  // second r, q of the fused iteration (ping-pong)
    bool fused = false;                   // fused single-pass iteration chosen
    int fbuf = 0;                         // fused iteration: which r, q, p the next pass reads
    // mixed precision (fused iteration only): float32 r, q, p (ping-pong), the
    // float32 iterate folded into x at each refresh, float32 k and D^-1
    bool mixed = false;
    float *r32[2] = {nullptr, nullptr}, *q32[2] = {nullptr, nullptr}, *p32[2] = {nullptr, nullptr};
    float *x32 = nullptr, *k32 = nullptr, *dinv32 = nullptr;
    int refreshes = 0;  // float64 residual refreshes of the last solve
    std::vector<int> stalled;  // per design: 0, 1 stagnated, 2 non-finite residual (last solve)
    W6* dw6 = nullptr;
    double* dvstar = nullptr;
    double* dmove = nullptr;  // OC move limit per design
    double* partials = nullptr;
    int partial_slots = 0;
    Scalars* sc = nullptr;
    Scalars* h_sc = nullptr;
    int pbuf = 0;

    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    std::vector<VolumeBound> gov;
    std::vector<double> kappa, g, volume, low;
    std::vector<int> have_density;
    bool have_solution = false;
    int iter = 0;
    double tune_us = 0.0;
    double t_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    std::string err;
};

namespace {

int bfail(otm_batch* c, int code, const std::string& m) {
    if (c) c->err = m;
    return code;
}

#define BCHK(c, call)                                                                                \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return bfail((c), OTM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int blaunch_ok(otm_batch* c, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(c, OTM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return OTM_OK;
}

template <typename T>
int balloc(otm_batch* c, T** p, int64_t n) {
    if (hipMalloc((void**)p, (size_t)n * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return bfail(c, OTM_ENOMEM, "device allocation failed");
    }
    c->dev_bytes += n * (int64_t)sizeof(T);
    return OTM_OK;
}

// Work lists for a given z-march tile (tx = 2 wx nodes wide, 256/wx rows) and
// march length tz; element sweeps give each thread at least four elements and
// use up to 256 blocks per design.
void build_tables(otm_batch* c, int wx, int tz) {
    const int tx = 2 * wx, ty = kBlock / wx;
    c->hdesc.resize(c->count);
    std::vector<int> ebd, mbd;
    for (int d = 0; d < c->count; ++d) {
        BatchDesc& D = c->hdesc[d];
        const int n = c->prob[d].n;
        const int64_t nn = (int64_t)n * n * n;
        D.n = n;
        D.off = c->off[d];
        D.eb_start = (int)ebd.size();
        // at least four elements per thread: the element sweeps end in block
        // reductions (up to 31 values for the OC bisection) that a block
        // with one element per thread spends most of its time on
        int64_t nb = (nn + 4 * kBlock - 1) / (4 * kBlock);
        D.eb_count = (int)std::min<int64_t>(nb, 256);
        for (int q = 0; q < D.eb_count; ++q) ebd.push_back(d);
        D.ntx = (n + tx - 1) / tx;
        D.nty = (n + ty - 1) / ty;
        D.tz = std::min(tz, n);
        D.mb_start = (int)mbd.size();
        D.mb_count = D.ntx * D.nty * ((n + D.tz - 1) / D.tz);
        for (int q = 0; q < D.mb_count; ++q) mbd.push_back(d);
        D.k0 = c->prob[d].k0;
        D.kmin = c->prob[d].kmin;
        D.penal = c->prob[d].penal;
        D.fw = filter_weights(c->prob[d].filter_radius);
    }
    c->tab.count = c->count;
    c->tab.eb_total = (int)ebd.size();
    c->tab.mb_total = (int)mbd.size();
    c->wx = wx;
    (void)hipMemcpyAsync(c->ddesc, c->hdesc.data(), c->count * sizeof(BatchDesc), hipMemcpyHostToDevice, c->stream);
    (void)hipMemcpyAsync(c->eb_design, ebd.data(), ebd.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    (void)hipMemcpyAsync(c->mb_design, mbd.data(), mbd.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    c->tab.desc = c->ddesc;
    c->tab.eb_design = c->eb_design;
    c->tab.mb_design = c->mb_design;
    c->march_grid = std::min(c->tab.mb_total, 1024);
    c->update_grid = std::min(c->tab.eb_total, 2048);
    // the host tables are staged from pageable memory: finish before they go away
    (void)hipStreamSynchronize(c->stream);
}

void march_pass(otm_batch* c, const double* po, double* pn, bool fin) {
    if (c->wx == 32)
        launch_b_dir_march2<32, 8>(c->tab, c->march_grid, c->r, c->dinv, po, pn, c->k, c->q, c->partials, c->sc,
                                   fin, c->stream);
    else
        launch_b_dir_march2<16, 16>(c->tab, c->march_grid, c->r, c->dinv, po, pn, c->k, c->q, c->partials, c->sc,
                                    fin, c->stream);
}

// check_every PCG iterations (even, so the direction buffers end where they began)
void pcg_chunk(otm_batch* c) {
    for (int it = 0; it < c->so.check_every; ++it) {
        double* po = c->p[c->pbuf];
        double* pn = c->p[c->pbuf ^ 1];
        march_pass(c, po, pn, true);
        launch_b_update_vec(c->tab, c->update_grid, c->x, c->r, pn, c->q, c->dinv, c->partials, c->sc, true,
                            c->stream);
        c->pbuf ^= 1;
    }
}

// One fused pass reading buffer set par and writing set par ^ 1.
void fused_pass(otm_batch* c, int par, bool fin) {
    const int nx = par ^ 1;
    if (c->mixed) {
        launch_b_fused<float>(c->tab, c->wx, c->march_grid, c->r32[par], c->q32[par], c->p32[par], c->r32[nx],
                              c->q32[nx], c->p32[nx], c->x32, c->dinv32, c->k32, c->partials, c->sc, par, fin,
                              c->stream);
    } else {
        double* R[2] = {c->r, c->r2};
        double* Q[2] = {c->q, c->q2};
        launch_b_fused<double>(c->tab, c->wx, c->march_grid, R[par], Q[par], c->p[par], R[nx], Q[nx], c->p[nx], c->x,
                               c->dinv, c->k, c->partials, c->sc, par, fin, c->stream);
    }
}

// check_every fused passes (even: the buffers end where they began)
void fused_chunk(otm_batch* c) {
    for (int it = 0; it < c->so.check_every; ++it) {
        fused_pass(c, c->fbuf, true);
        c->fbuf ^= 1;
    }
}

// float64 residual of every design from its float64 x (start, or a refresh
// with the pending step of buffer set fbuf)
void residual_f(otm_batch* c, bool start, bool x_zero) {
    if (c->mixed) {
        launch_b_residual_f<float>(c->tab, c->k, c->b, c->x, c->r32[c->fbuf], start ? nullptr : c->q32[c->fbuf],
                                   c->dinv32, start, x_zero ? 1 : 0, c->partials, c->sc, c->stream);
    } else {
        double* R[2] = {c->r, c->r2};
        double* Q[2] = {c->q, c->q2};
        launch_b_residual_f<double>(c->tab, c->k, c->b, c->x, R[c->fbuf], start ? nullptr : Q[c->fbuf], c->dinv,
                                    start, x_zero ? 1 : 0, c->partials, c->sc, c->stream);
    }
}

int sync_sc(otm_batch* c) {
    BCHK(c, hipMemcpyAsync(c->h_sc, c->sc, c->count * sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
    BCHK(c, hipStreamSynchronize(c->stream));
    return OTM_OK;
}

// The solver part of every design's scalar block reset (one launch on the
// device, the host mirror alike); a copy per design cost a blit each.
int reset_solver(otm_batch* c) {
    const size_t head = offsetof(Scalars, sum_rho);
    const double tol2 = c->so.tol * c->so.tol;
    for (int d = 0; d < c->count; ++d) {
        std::memset(&c->h_sc[d], 0, head);
        c->h_sc[d].tol2 = tol2;
    }
    launch_b_reset_solver(c->sc, c->count, tol2, c->stream);
    return blaunch_ok(c, "solver reset");
}

bool all_inactive(const otm_batch* c) {
    for (int d = 0; d < c->count; ++d)
        for (int l = 0; l < 3; ++l)
            if (c->h_sc[d].active[l]) return false;
    return true;
}

// Stagnation watch per design, the rule a context's solve uses: a design
// whose running loads have not cut their recursive residual 4x within its
// window of iterations (stall_window, else 200 + 10 n), or whose residual is
// not finite, stops: its loads are switched off on the device and stay off
// through later confirmation refreshes, and the step reports it.
struct BatchWatch {
    std::vector<double> best;
    std::vector<int> at, window;
    void start(otm_batch* c) {
        best.assign(3 * (size_t)c->count, 0.0);
        at.assign(3 * (size_t)c->count, 0);
        window.resize(c->count);
        c->stalled.assign(c->count, 0);
        for (int d = 0; d < c->count; ++d) {
            window[d] = c->so.stall_window > 0 ? c->so.stall_window : 200 + 10 * c->prob[d].n;
            for (int l = 0; l < 3; ++l) {
                best[3 * d + l] = c->h_sc[d].rr[l];
                at[3 * d + l] = c->h_sc[d].iters[l];
            }
        }
    }
    // after a chunk: true when some design got a verdict now
    bool check(otm_batch* c) {
        bool any = false;
        for (int d = 0; d < c->count; ++d) {
            if (c->stalled[d]) continue;
            for (int l = 0; l < 3; ++l) {
                const Scalars& s = c->h_sc[d];
                if (!s.active[l]) continue;
                const size_t i = 3 * (size_t)d + l;
                if (!std::isfinite(s.rr[l])) {
                    c->stalled[d] = 2;
                } else if (s.rr[l] <= 0.25 * best[i]) {
                    best[i] = s.rr[l];
                    at[i] = s.iters[l];
                } else if (s.iters[l] - at[i] > window[d]) {
                    c->stalled[d] = 1;
                }
                if (c->stalled[d]) {
                    any = true;
                    break;
                }
            }
        }
        return any;
    }
};

// Switch off the loads of every design with a verdict (host copy and device;
// after a scalar sync the two agree).
int hold_stalled(otm_batch* c) {
    const size_t head = offsetof(Scalars, sum_rho);
    for (int d = 0; d < c->count; ++d) {
        if (!c->stalled[d]) continue;
        Scalars& s = c->h_sc[d];
        if (!(s.active[0] || s.active[1] || s.active[2])) continue;
        for (int l = 0; l < 3; ++l) {
            s.active[l] = 0;
            s.alpha[l] = 0.0;
            s.beta[l] = 0.0;
        }
        BCHK(c, hipMemcpyAsync(&c->sc[d], &c->h_sc[d], head, hipMemcpyHostToDevice, c->stream));
    }
    return OTM_OK;
}

int max_iters(const otm_batch* c) {
    int m = 0;
    for (int d = 0; d < c->count; ++d)
        for (int l = 0; l < 3; ++l) m = std::max(m, c->h_sc[d].iters[l]);
    return m;
}

int run_chunk(otm_batch* c) {
    if (!c->use_graph) {
        if (c->fused)
            fused_chunk(c);
        else
            pcg_chunk(c);
        return blaunch_ok(c, "pcg chunk");
    }
    if (!c->gexec) {
        const int pb = c->pbuf, fb = c->fbuf;
        BCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        if (c->fused)
            fused_chunk(c);
        else
            pcg_chunk(c);
        hipGraph_t g = nullptr;
        BCHK(c, hipStreamEndCapture(c->stream, &g));
        c->graph = g;
        BCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
        c->pbuf = pb;  // capture did not run anything
        c->fbuf = fb;
    }
    BCHK(c, hipGraphLaunch(c->gexec, c->stream));
    // the chunk has an even number of iterations: pbuf is unchanged
    return OTM_OK;
}

// The fused iteration (one pass and one per-design finalize per iteration);
// converged designs are confirmed with their true residual, and loads that
// miss the tolerance restart.  Mixed precision: the float32 iterate is folded
// into the float64 x and the float64 residual replaces the recursive one when
// every design has stopped, or when some running load's recursive residual
// has fallen by reliable_delta since its last refresh (the refresh covers
// every design: a refresh at any chunk boundary is a valid step).
int solve_fused(otm_batch* c, bool x_zero) {
    int rc;
    if ((rc = reset_solver(c))) return rc;
    if (x_zero) BCHK(c, hipMemsetAsync(c->x, 0, (size_t)3 * c->total * sizeof(double), c->stream));
    if (c->mixed) BCHK(c, hipMemsetAsync(c->x32, 0, (size_t)3 * c->total * sizeof(float), c->stream));
    c->fbuf = 0;
    c->refreshes = 0;
    residual_f(c, true, x_zero);
    if ((rc = blaunch_ok(c, "residual"))) return rc;
    if ((rc = sync_sc(c))) return rc;
    std::vector<double> rr_ref(3 * (size_t)c->count);
    for (int d = 0; d < c->count; ++d)
        for (int l = 0; l < 3; ++l) rr_ref[3 * d + l] = c->h_sc[d].rr_true[l];
    const double d2 = c->so.reliable_delta * c->so.reliable_delta;
    BatchWatch watch;
    watch.start(c);
    while (!all_inactive(c) && max_iters(c) < c->so.max_iter) {
        if ((rc = run_chunk(c))) return rc;
        if ((rc = sync_sc(c))) return rc;
        if (watch.check(c) && (rc = hold_stalled(c))) return rc;
        bool refresh = all_inactive(c);
        if (c->mixed)
            for (int d = 0; d < c->count && !refresh; ++d)
                for (int l = 0; l < 3; ++l)
                    if (c->h_sc[d].active[l] && c->h_sc[d].rr[l] < d2 * rr_ref[3 * d + l]) refresh = true;
        if (refresh) {
            if (c->mixed) launch_b_accumulate(c->tab, c->x, c->x32, c->stream);
            residual_f(c, false, false);
            if ((rc = blaunch_ok(c, "refresh"))) return rc;
            if ((rc = sync_sc(c))) return rc;
            if ((rc = hold_stalled(c))) return rc;  // a refresh restarts loads that miss the tolerance
            for (int d = 0; d < c->count; ++d)
                for (int l = 0; l < 3; ++l) rr_ref[3 * d + l] = c->h_sc[d].rr_true[l];
            if (c->mixed) ++c->refreshes;
        }
    }
    if (c->mixed) launch_b_accumulate(c->tab, c->x, c->x32, c->stream);
    launch_b_sum3(c->tab, c->x, 0, c->partials, c->sc, c->stream);
    launch_b_sub_mean3(c->tab, c->x, 0, c->sc, c->stream);
    return blaunch_ok(c, "project");
}

int solve(otm_batch* c, bool x_zero) {
    if (c->fused) return solve_fused(c, x_zero);
    int rc;
    if ((rc = reset_solver(c))) return rc;
    if (x_zero) BCHK(c, hipMemsetAsync(c->x, 0, (size_t)3 * c->total * sizeof(double), c->stream));
    launch_b_residual(c->tab, c->k, c->b, c->x, c->r, c->p[c->pbuf], c->dinv, RES_START, x_zero ? 1 : 0, c->partials,
                      c->sc, c->stream);
    if ((rc = blaunch_ok(c, "residual"))) return rc;
    if ((rc = sync_sc(c))) return rc;
    BatchWatch watch;
    watch.start(c);
    while (!all_inactive(c) && max_iters(c) < c->so.max_iter) {
        if ((rc = run_chunk(c))) return rc;
        if ((rc = sync_sc(c))) return rc;
        if (watch.check(c) && (rc = hold_stalled(c))) return rc;
        if (all_inactive(c)) {
            launch_b_residual(c->tab, c->k, c->b, c->x, c->r, c->p[c->pbuf], c->dinv, RES_START, 0, c->partials, c->sc,
                              c->stream);
            if ((rc = sync_sc(c))) return rc;
            if ((rc = hold_stalled(c))) return rc;
        }
    }
    launch_b_sum3(c->tab, c->x, 0, c->partials, c->sc, c->stream);
    launch_b_sub_mean3(c->tab, c->x, 0, c->sc, c->stream);
    return blaunch_ok(c, "project");
}

// Time one PCG iteration of a (tile width, march length) candidate: the
// fused pass, or the direction+operator pass and the update.  The per-design
// finalizes (one block per design) are left out of both kinds, so that every
// timed pass runs with the same all-active state.  The fused kind needs at
// most kMaxBlocks work items.
double time_candidate(otm_batch* c, int wx, int tz, bool fused) {
    build_tables(c, wx, tz);
    if (fused && (c->tab.mb_total > kMaxBlocks || !(c->r2 || c->mixed))) return 1e30;
    auto iteration = [&](int par) {
        if (fused) {
            fused_pass(c, par, false);
        } else {
            march_pass(c, c->p[par], c->p[par ^ 1], false);
            launch_b_update_vec(c->tab, c->update_grid, c->x, c->r, c->p[par ^ 1], c->q, c->dinv, c->partials,
                                c->sc, false, c->stream);
        }
    };
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    iteration(0);
    iteration(1);
    (void)hipEventRecord(a, c->stream);
    const int reps = 6;
    for (int i = 0; i < reps; ++i) iteration(i & 1);
    (void)hipEventRecord(b, c->stream);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (hipGetLastError() != hipSuccess) return 1e30;
    return 1000.0 * ms / reps;
}

std::mutex g_btune_mu;
std::map<std::vector<int>, std::pair<int, int>> g_btune;

int autotune_batch(otm_batch* c) {
    std::vector<int> key;
    for (auto& p : c->prob) key.push_back(p.n);
    std::sort(key.begin(), key.end());
    // fused only: mixed precision, or kernel variant 4
    const bool fused_only = c->mixed || c->so.kernel_variant == 4;
    std::string fkey = "batch";
    for (size_t i = 0; i < key.size();) {
        size_t j = i;
        while (j < key.size() && key[j] == key[i]) ++j;
        fkey += "_" + std::to_string(key[i]) + "x" + std::to_string(j - i);
        i = j;
    }
    if (c->mixed) fkey += "_mixed";
    key.insert(key.begin(), {c->mixed ? 1 : 0, fused_only ? 1 : 0});
    {
        std::lock_guard<std::mutex> g(g_btune_mu);
        auto it = g_btune.find(key);
        if (it != g_btune.end()) {  // a negative width marks the fused iteration
            build_tables(c, std::abs(it->second.first), it->second.second);
            c->fused = it->second.first < 0;
            return OTM_OK;
        }
    }
    // the persistent cache: keyed by the multiset of n (count of each size)
    // and the precision
    {
        std::vector<double> v(4);
        if (tune_cache_lookup(fkey, v)) {
            const int wx = (int)v[0], tz = (int)v[1];
            const bool fused = v[2] != 0.0;
            if ((wx == 16 || wx == 32) && (tz == 4 || tz == 8 || tz == 16 || tz == 32)) {
                build_tables(c, wx, tz);
                if (fused ? ((c->r2 || c->mixed) && c->tab.mb_total <= kMaxBlocks) : !fused_only) {
                    c->fused = fused;
                    c->tune_us = v[3];
                    std::lock_guard<std::mutex> g(g_btune_mu);
                    g_btune[key] = {fused ? -wx : wx, tz};
                    return OTM_OK;
                }
            }
        }
    }
    // valid timing state: every load active, beta != 0, zeroed vectors
    const size_t head = offsetof(Scalars, sum_rho);
    for (int d = 0; d < c->count; ++d) {
        std::memset(&c->h_sc[d], 0, head);
        for (int l = 0; l < 3; ++l) {
            c->h_sc[d].active[l] = 1;
            c->h_sc[d].alpha[l] = 0.5;
            c->h_sc[d].beta[l] = 0.5;
            c->h_sc[d].rz[l] = 1.0;
        }
        BCHK(c, hipMemcpyAsync(&c->sc[d], &c->h_sc[d], head, hipMemcpyHostToDevice, c->stream));
    }
    const size_t v3 = (size_t)3 * c->total * sizeof(double), v1 = (size_t)c->total * sizeof(double);
    for (double* v : {c->r, c->q, c->r2, c->q2, c->p[0], c->p[1], c->x})
        if (v) BCHK(c, hipMemsetAsync(v, 0, v3, c->stream));
    for (float* v : {c->r32[0], c->r32[1], c->q32[0], c->q32[1], c->p32[0], c->p32[1], c->x32})
        if (v) BCHK(c, hipMemsetAsync(v, 0, v3 / 2, c->stream));
    for (float* v : {c->k32, c->dinv32})
        if (v) BCHK(c, hipMemsetAsync(v, 0, v1 / 2, c->stream));
    BCHK(c, hipMemsetAsync(c->k, 0, v1, c->stream));
    BCHK(c, hipMemsetAsync(c->dinv, 0, v1, c->stream));
    int best_wx = 16, best_tz = 8;
    bool best_fused = false;
    double best = 1e30;
    const int fz_min = fused_only ? 1 : 0;
    for (int fz = ((c->r2 || c->mixed) ? 1 : 0); fz >= fz_min; --fz)
        for (int wx : {16, 32})
            for (int tz : {4, 8, 16, 32}) {
                const double us = time_candidate(c, wx, tz, fz != 0);
                if (us < 0.98 * best) {  // near-ties keep the earlier candidate
                    best = us;
                    best_wx = wx;
                    best_tz = tz;
                    best_fused = fz != 0;
                }
            }
    if (c->mixed && !best_fused)
        return bfail(c, OTM_EUNSUPPORTED, "a mixed-precision batch needs at most 4096 (design, tile) items");
    for (double* v : {c->p[0], c->p[1], c->x})
        if (v) BCHK(c, hipMemsetAsync(v, 0, v3, c->stream));
    for (float* v : {c->q32[0], c->q32[1], c->p32[0], c->p32[1], c->x32})
        if (v) BCHK(c, hipMemsetAsync(v, 0, v3 / 2, c->stream));
    build_tables(c, best_wx, best_tz);
    c->fused = best_fused;
    BCHK(c, hipStreamSynchronize(c->stream));
    c->tune_us = best;
    tune_cache_store(fkey, {(double)best_wx, (double)best_tz, best_fused ? 1.0 : 0.0, best});
    std::lock_guard<std::mutex> g(g_btune_mu);
    g_btune[key] = {best_fused ? -best_wx : best_wx, best_tz};
    return OTM_OK;
}

void free_batch(otm_batch* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    void* bufs[] = {c->rho,    c->rhof,   c->k,      c->dinv,     c->b,      c->x,        c->st,
                    c->sens,   c->ocq,    c->r,      c->p[0],     c->p[1],   c->q,        c->r2,
                    c->q2,     c->r32[0], c->r32[1], c->q32[0],   c->q32[1], c->p32[0],   c->p32[1],
                    c->x32,    c->k32,    c->dinv32, c->dw6,      c->dvstar, c->dmove,    c->partials,
                    c->sc,     c->ddesc,  c->eb_design, c->mb_design};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    if (c->h_sc) (void)hipHostFree(c->h_sc);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

}  // namespace

extern "C" {

int otm_batch_create(const otm_problem* problems, int32_t count, const otm_solver_opts* solver,
                     const otm_oc_opts* oc, const otm_governor_opts* gov, void* stream, otm_batch** out) {
    if (!out || !problems || count < 1 || count > 4096) return OTM_EINVAL;
    *out = nullptr;
    for (int d = 0; d < count; ++d) {
        const otm_problem& p = problems[d];
        if (p.n < 4 || p.n > 1024 || (p.n % 2) != 0) return OTM_EINVAL;  // the batched kernels need even n
        if (!(p.kmin > 0.0 && p.k0 > p.kmin && p.penal >= 1.0 && p.filter_radius < 5.0 && p.vf > 0.0 && p.vf <= 1.0))
            return OTM_EINVAL;
        for (int q = 0; q < 6; ++q)
            if (!std::isfinite(p.target[q])) return OTM_EINVAL;
        if (p.objective != OTM_OBJ_MSE && p.objective != OTM_OBJ_REL && p.objective != OTM_OBJ_L1)
            return OTM_EUNSUPPORTED;
        if (p.objective == OTM_OBJ_REL)
            for (int q = 0; q < 6; ++q)
                if (p.target[q] == 0.0) return OTM_EINVAL;
        if (p.symmetry != OTM_SYM_NONE) return OTM_EUNSUPPORTED;
    }
    otm_batch* c = new (std::nothrow) otm_batch();
    if (!c) return OTM_ENOMEM;
    c->count = count;
    c->prob.assign(problems, problems + count);
    otm_default_options(&c->so, &c->oc, &c->go);
    if (solver) c->so = *solver;
    if (oc) c->oc = *oc;
    if (gov) c->go = *gov;
    c->mixed = c->so.precision == OTM_MIXED;
    // mixed precision runs the fused iteration only (kernel variant 0 or 4)
    const bool supported = (c->so.precision == OTM_FP64 || (c->mixed && (c->so.kernel_variant == 0 ||
                                                                          c->so.kernel_variant == 4))) &&
                           c->so.preconditioner == OTM_PRECOND_JACOBI;
    if (!supported || !(c->so.tol > 0.0) || c->so.max_iter < 1 || c->so.check_every < 1 ||
        c->so.kernel_variant < 0 || c->so.kernel_variant > 5 || !(c->so.reliable_delta > 0.0) ||
        c->so.stall_window < 0) {
        const bool known = (c->so.precision == OTM_FP64 || c->mixed) && c->so.kernel_variant >= 0 &&
                           c->so.kernel_variant <= 5 &&
                           (c->so.preconditioner == OTM_PRECOND_JACOBI || c->so.preconditioner == OTM_PRECOND_MG);
        const int code = (known && !supported) ? OTM_EUNSUPPORTED : OTM_EINVAL;
        delete c;
        return code;
    }
    if (!(c->oc.move > 0.0 && c->oc.eta > 0.0 && c->oc.rho_min > 0.0 && c->oc.rho_min < 1.0 &&
          c->oc.move_min >= 0.0 && c->oc.move_min <= c->oc.move) ||
        !governor_opts_valid(c->go)) {
        delete c;
        return OTM_EINVAL;
    }
    if (c->so.check_every % 2) c->so.check_every += 1;
    hipDeviceProp_t prop;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        (void)hipGetLastError();
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
    c->off.resize(count);
    int64_t total = 0;
    int64_t max_eb = 0, max_mb = 0;
    for (int d = 0; d < count; ++d) {
        c->off[d] = total;
        const int n = problems[d].n;
        total += (int64_t)n * n * n;
        max_eb += 256;
        // smallest tile (32 x 16 nodes) and march (4 planes) bound the item count
        max_mb += (int64_t)((n + 31) / 32) * ((n + 7) / 8) * ((n + 3) / 4);
    }
    c->total = total;
    int rc = OTM_OK;
    rc = rc ? rc : balloc(c, &c->rho, total);
    rc = rc ? rc : balloc(c, &c->rhof, total);
    rc = rc ? rc : balloc(c, &c->k, total);
    rc = rc ? rc : balloc(c, &c->dinv, total);
    rc = rc ? rc : balloc(c, &c->b, 3 * total);
    rc = rc ? rc : balloc(c, &c->x, 3 * total);
    rc = rc ? rc : balloc(c, &c->st, total);
    rc = rc ? rc : balloc(c, &c->sens, total);
    rc = rc ? rc : balloc(c, &c->ocq, total);
    // the fused iteration (kernel variant 0 with autotuning, or 4; always in
    // mixed precision) ping-pongs r and q
    const bool may_fuse = c->mixed || c->so.kernel_variant == 4 || (c->so.kernel_variant == 0 && c->so.autotune);
    if (c->mixed) {
        for (int i = 0; i < 2; ++i) {
            rc = rc ? rc : balloc(c, &c->r32[i], 3 * total);
            rc = rc ? rc : balloc(c, &c->q32[i], 3 * total);
            rc = rc ? rc : balloc(c, &c->p32[i], 3 * total);
        }
        rc = rc ? rc : balloc(c, &c->x32, 3 * total);
        rc = rc ? rc : balloc(c, &c->k32, total);
        rc = rc ? rc : balloc(c, &c->dinv32, total);
    } else {
        rc = rc ? rc : balloc(c, &c->r, 3 * total);
        rc = rc ? rc : balloc(c, &c->p[0], 3 * total);
        rc = rc ? rc : balloc(c, &c->p[1], 3 * total);
        rc = rc ? rc : balloc(c, &c->q, 3 * total);
        if (may_fuse) {
            rc = rc ? rc : balloc(c, &c->r2, 3 * total);
            rc = rc ? rc : balloc(c, &c->q2, 3 * total);
        }
    }
    rc = rc ? rc : balloc(c, &c->dw6, count);
    rc = rc ? rc : balloc(c, &c->dvstar, count);
    rc = rc ? rc : balloc(c, &c->dmove, count);
    c->partial_slots = (int)std::max(max_eb, max_mb);
    rc = rc ? rc : balloc(c, &c->partials, std::max((int64_t)c->partial_slots * kMaxReduce,
                                                    may_fuse ? 2 * kFusedStride : (int64_t)0));
    rc = rc ? rc : balloc(c, &c->sc, count);
    rc = rc ? rc : balloc(c, &c->ddesc, count);
    rc = rc ? rc : balloc(c, &c->eb_design, max_eb);
    rc = rc ? rc : balloc(c, &c->mb_design, max_mb);
    if (!rc && hipHostMalloc((void**)&c->h_sc, count * sizeof(Scalars), hipHostMallocDefault) != hipSuccess)
        rc = OTM_ENOMEM;
    if (rc) {
        free_batch(c);
        delete c;
        return rc;
    }
    c->gov.resize(count);
    for (int d = 0; d < count; ++d) c->gov[d].vstar = problems[d].vf;
    c->kappa.assign(6 * count, 0.0);
    c->g.assign(count, 0.0);
    c->volume.assign(count, 0.0);
    c->low.assign(count, 0.0);
    c->have_density.assign(count, 0);
    for (double* v : {c->x, c->p[0], c->p[1]})
        if (v) (void)hipMemsetAsync(v, 0, (size_t)3 * total * sizeof(double), c->stream);
    for (float* v : {c->q32[0], c->q32[1], c->p32[0], c->p32[1], c->x32})
        if (v) (void)hipMemsetAsync(v, 0, (size_t)3 * total * sizeof(float), c->stream);
    if (c->so.autotune && c->so.tile_tz == 0 && c->so.tile_tx == 0) {
        rc = autotune_batch(c);
    } else {
        const int wx = c->so.tile_tx == 64 ? 32 : 16;
        build_tables(c, wx, c->so.tile_tz > 0 ? std::max(4, c->so.tile_tz) : 8);
        c->fused = (c->mixed || c->so.kernel_variant == 4) && (c->r2 || c->mixed) && c->tab.mb_total <= kMaxBlocks;
        if (c->mixed && !c->fused)
            rc = bfail(c, OTM_EUNSUPPORTED, "a mixed-precision batch needs at most 4096 (design, tile) items");
    }
    if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = OTM_EDEVICE;
    if (rc) {
        free_batch(c);
        delete c;
        return rc;
    }
    *out = c;
    return OTM_OK;
}

void otm_batch_destroy(otm_batch* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_batch(c);
    delete c;
}

int otm_batch_set_graph(otm_batch* c, int32_t use_graph) {
    if (!c) return OTM_EINVAL;
    c->use_graph = use_graph != 0;
    return OTM_OK;
}

int otm_batch_set_density(otm_batch* c, int32_t d, const double* rho, int64_t count) {
    if (!c || !rho || d < 0 || d >= c->count) return OTM_EINVAL;
    const int n = c->prob[d].n;
    if (count != (int64_t)n * n * n) return bfail(c, OTM_EINVAL, "density count must be n^3");
    for (int64_t e = 0; e < count; ++e)
        if (!std::isfinite(rho[e])) return bfail(c, OTM_ENONFINITE, "non-finite density");
    BCHK(c, hipMemcpyAsync(c->rho + c->off[d], rho, count * sizeof(double), hipMemcpyHostToDevice, c->stream));
    BCHK(c, hipStreamSynchronize(c->stream));
    c->have_density[d] = 1;
    return OTM_OK;
}

int otm_batch_get_field(otm_batch* c, int32_t d, int32_t field, double* out, int64_t count) {
    if (!c || !out || d < 0 || d >= c->count) return OTM_EINVAL;
    const int64_t nn = (int64_t)c->prob[d].n * c->prob[d].n * c->prob[d].n;
    const double* src = nullptr;
    int64_t size = nn;
    switch (field) {
        case OTM_FIELD_RHO: src = c->rho + c->off[d]; break;
        case OTM_FIELD_RHOF: src = c->rhof + c->off[d]; break;
        case OTM_FIELD_K: src = c->k + c->off[d]; break;
        case OTM_FIELD_CHI: src = c->x + 3 * c->off[d]; size = 3 * nn; break;
        case OTM_FIELD_SENS: src = c->sens + c->off[d]; break;
        case OTM_FIELD_SENS_ELEM: src = c->st + c->off[d]; break;
        default: return bfail(c, OTM_EINVAL, "field not available for batches");
    }
    if (count != size) return bfail(c, OTM_EINVAL, "field count mismatch");
    BCHK(c, hipMemcpyAsync(out, src, size * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    BCHK(c, hipStreamSynchronize(c->stream));
    return OTM_OK;
}

int otm_batch_step(otm_batch* c, otm_iter_record* recs) {
    if (!c) return OTM_EINVAL;
    for (int d = 0; d < c->count; ++d)
        if (!c->have_density[d]) return bfail(c, OTM_ESTATE, "every design needs a density");
    int rc;
    auto t0 = std::chrono::steady_clock::now();
    // densities clamped to [rho_min, 1]
    launch_b_clamp(c->tab, c->rho, c->oc.rho_min, 1.0, c->stream);
    // filter + SIMP + loads + diagonal
    launch_b_filter_simp(c->tab, c->rho, c->rhof, c->k, c->partials, c->sc, c->stream);
    launch_b_setup_nodes(c->tab, c->k, c->b, c->dinv, c->partials, c->sc, c->stream);
    launch_b_sub_mean3(c->tab, c->b, 1, c->sc, c->stream);
    if (c->mixed) launch_b_to_f32(c->tab, c->k, c->dinv, c->k32, c->dinv32, c->stream);
    if ((rc = blaunch_ok(c, "prepare"))) return rc;
    auto t1 = std::chrono::steady_clock::now();
    const bool x_zero = !(c->so.guess == OTM_GUESS_PREVIOUS && c->have_solution);
    if ((rc = solve(c, x_zero))) return rc;
    c->have_solution = true;
    auto t2 = std::chrono::steady_clock::now();
    launch_b_energy(c->tab, c->k, c->x, c->partials, c->sc, c->stream);
    if ((rc = sync_sc(c))) return rc;
    std::vector<W6> w6(c->count);
    std::vector<double> vstar(c->count), moves(c->count);
    bool conv = true;
    for (int d = 0; d < c->count; ++d) {
        const double nn = (double)c->prob[d].n * c->prob[d].n * c->prob[d].n;
        const Scalars& s = c->h_sc[d];
        double gg = 0.0;
        for (int q = 0; q < 6; ++q) c->kappa[6 * d + q] = s.kappa_sum[q] / nn;
        objective_grad(c->prob[d].objective, c->kappa.data() + 6 * d, c->prob[d].target, &gg, w6[d].w);
        if (!std::isfinite(gg)) return bfail(c, OTM_ENONFINITE, "non-finite tensor");
        c->g[d] = gg;
        c->volume[d] = s.sum_rho / nn;
        c->low[d] = s.sum_rhofp / nn;
        for (int l = 0; l < 3; ++l)
            if (s.active[l]) conv = false;
        if (c->stalled[d]) conv = false;
        if (recs) {
            otm_iter_record& R = recs[d];
            R.iter = c->iter;
            R.g = gg;
            std::memcpy(R.kappa, &c->kappa[6 * d], 6 * sizeof(double));
            R.volume = c->volume[d];
            R.low_bound = c->low[d];
            for (int l = 0; l < 3; ++l) {
                R.pcg_iters[l] = s.iters[l];
                R.rel_residual[l] = s.bb[l] > 0.0 ? std::sqrt(s.rr_true[l] / s.bb[l]) : 0.0;
            }
            R.stalled = c->stalled[d];
        }
        moves[d] = next_move(c->oc, c->gov[d], gg);
        advance_volume_bound(c->go, c->oc.rho_min, c->gov[d], gg, c->low[d], c->volume[d]);
        vstar[d] = c->gov[d].vstar;
    }
    BCHK(c, hipMemcpyAsync(c->dw6, w6.data(), c->count * sizeof(W6), hipMemcpyHostToDevice, c->stream));
    BCHK(c, hipMemcpyAsync(c->dvstar, vstar.data(), c->count * sizeof(double), hipMemcpyHostToDevice, c->stream));
    BCHK(c, hipMemcpyAsync(c->dmove, moves.data(), c->count * sizeof(double), hipMemcpyHostToDevice, c->stream));
    // sensitivities and filter transpose
    launch_b_sens(c->tab, c->rhof, c->x, c->dw6, c->st, c->stream);
    launch_b_filter(c->tab, c->st, c->sens, c->stream);
    // OC bisection for every design
    launch_b_oc_prepare(c->tab, c->rho, c->sens, c->oc.eta, c->ocq, c->stream);
    launch_b_oc_init(c->tab, c->sc, c->dvstar, c->oc.eta, c->stream);
    const int max_passes = kOcMaxPasses;
    for (int pass = 0; pass < max_passes; pass += 4) {
        for (int q = 0; q < 4; ++q)
            launch_b_oc_pass(c->tab, c->rho, c->ocq, c->dmove, c->oc.rho_min, c->oc.eta, c->partials, c->sc,
                             c->stream);
        if ((rc = sync_sc(c))) return rc;
        bool done = true;
        for (int d = 0; d < c->count; ++d) done = done && c->h_sc[d].oc_done;
        if (done) break;
    }
    launch_b_oc_apply(c->tab, c->rho, c->ocq, c->oc.eta, c->dmove, c->oc.rho_min, c->sc, c->stream);
    if ((rc = sync_sc(c))) return rc;
    auto t3 = std::chrono::steady_clock::now();
    if (recs)
        for (int d = 0; d < c->count; ++d) {
            recs[d].vstar = vstar[d];
            recs[d].move = moves[d];
            recs[d].lambda = c->h_sc[d].lam;
            recs[d].ms_total = std::chrono::duration<double, std::milli>(t3 - t0).count();
            recs[d].ms_solve = std::chrono::duration<double, std::milli>(t2 - t1).count();
            recs[d].stop = c->gov[d].flat >= c->go.stall_iters ? 1 : 0;
        }
    c->t_ms[0] = std::chrono::duration<double, std::milli>(t1 - t0).count();
    c->t_ms[1] = std::chrono::duration<double, std::milli>(t2 - t1).count();
    c->t_ms[2] = std::chrono::duration<double, std::milli>(t3 - t2).count();
    c->t_ms[3] = std::chrono::duration<double, std::milli>(t3 - t0).count();
    c->iter += 1;
    return conv ? OTM_OK : OTM_NOT_CONVERGED;
}

// ---- checkpoint / resume -----------------------------------------------------
// A batch run's state, in one little-endian binary file written here:
//   "OTMBATCH" | u32 version 1 | i32 count | u32 flags (bit 0: solutions
//   present) | i32 design iterations done | per design: i32 n | u32 0 |
//   f64 problem[11] (k0, kmin, penal, filter radius, target[6], objective) |
//   f64 governor[8] (V*, Df, stalls, gap, previous objective, flat count,
//   OC step, the objective's last change) | then the density arena (every
//   design's rho[n^3] in order) | the solution arena (3 n^3 per design) if
//   bit 0 | u64 FNV-1a hash of every preceding byte.
// Written under path.tmp and renamed over path, so a crash while saving
// leaves any earlier checkpoint whole.
namespace {
const char kBatchMagic[8] = {'O', 'T', 'M', 'B', 'A', 'T', 'C', 'H'};
constexpr uint32_t kBatchVersion = 1;

void governor_out(const VolumeBound& v, double g[8]) {
    g[0] = v.vstar;
    g[1] = v.df;
    g[2] = (double)v.stalls;
    g[3] = v.gap;
    g[4] = v.g_prev;
    g[5] = (double)v.flat;
    g[6] = v.move;
    g[7] = v.dg_prev;
}

void governor_in(const double g[8], VolumeBound& v) {
    v.vstar = g[0];
    v.df = g[1];
    v.stalls = (int)g[2];
    v.gap = g[3];
    v.g_prev = g[4];
    v.flat = (int)g[5];
    v.move = g[6] > 0.0 ? g[6] : 0.0;
    v.dg_prev = g[7];
}
}  // namespace

int otm_batch_save_state(otm_batch* c, const char* path) {
    if (!c || !path || !path[0]) return OTM_EINVAL;
    for (int d = 0; d < c->count; ++d)
        if (!c->have_density[d]) return bfail(c, OTM_ESTATE, "every design needs a density to save");
    std::vector<double> rho((size_t)c->total), chi;
    BCHK(c, hipMemcpyAsync(rho.data(), c->rho, rho.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (c->have_solution) {
        chi.resize(3 * (size_t)c->total);
        BCHK(c, hipMemcpyAsync(chi.data(), c->x, chi.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    BCHK(c, hipStreamSynchronize(c->stream));
    const uint32_t version = kBatchVersion, flags = c->have_solution ? 1u : 0u, zero = 0u;
    const int32_t count = c->count, iter = c->iter;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return bfail(c, OTM_EIO, "cannot open " + tmp + " for writing");
    Fnv1a h;
    bool ok = true;
    auto put = [&](const void* p, size_t len) {
        if (!ok || len == 0) return;
        h.add(p, len);
        ok = std::fwrite(p, 1, len, f) == len;
    };
    put(kBatchMagic, 8);
    put(&version, 4);
    put(&count, 4);
    put(&flags, 4);
    put(&iter, 4);
    for (int d = 0; d < c->count; ++d) {
        const int32_t n = c->prob[d].n;
        double sig[11], gov[8];
        problem_signature(c->prob[d], sig);
        governor_out(c->gov[d], gov);
        put(&n, 4);
        put(&zero, 4);
        put(sig, sizeof(sig));
        put(gov, sizeof(gov));
    }
    put(rho.data(), rho.size() * sizeof(double));
    put(chi.data(), chi.size() * sizeof(double));
    const uint64_t digest = h.h;
    ok = ok && std::fwrite(&digest, 1, 8, f) == 8;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return bfail(c, OTM_EIO, std::string("cannot write ") + path);
    }
    return OTM_OK;
}

int otm_batch_load_state(otm_batch* c, const char* path) {
    if (!c || !path || !path[0]) return OTM_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (!f) return bfail(c, OTM_EIO, std::string("cannot open ") + path);
    std::vector<unsigned char> buf;
    unsigned char chunk[1 << 16];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) buf.insert(buf.end(), chunk, chunk + got);
    const bool read_err = std::ferror(f) != 0;
    std::fclose(f);
    if (read_err) return bfail(c, OTM_EIO, std::string("cannot read ") + path);
    const size_t top = 8 + 4 * 4, per = 8 + 11 * 8 + 8 * 8;
    if (buf.size() < top + 8 || std::memcmp(buf.data(), kBatchMagic, 8) != 0)
        return bfail(c, OTM_EIO, std::string(path) + " is not a batch state file");
    uint32_t version, flags;
    int32_t count, iter;
    std::memcpy(&version, &buf[8], 4);
    std::memcpy(&count, &buf[12], 4);
    std::memcpy(&flags, &buf[16], 4);
    std::memcpy(&iter, &buf[20], 4);
    if (version != kBatchVersion) return bfail(c, OTM_EIO, "unsupported batch state file version");
    if (count != c->count) return bfail(c, OTM_EINVAL, "batch state file holds another number of designs");
    const size_t head = top + (size_t)count * per;
    if (buf.size() < head + 8) return bfail(c, OTM_EIO, "batch state file is shorter than its header");
    // The body's size follows from the file's own per-design n, so a whole
    // file written for other grid sizes is told apart from a damaged one.
    size_t cells = 0;
    for (int d = 0; d < count; ++d) {
        int32_t n;
        std::memcpy(&n, &buf[top + (size_t)d * per], 4);
        if (n < 4 || n > 1024) return bfail(c, OTM_EIO, "batch state file holds an invalid grid size");
        cells += (size_t)n * n * n;
    }
    const size_t body = cells * sizeof(double) * ((flags & 1u) ? 4 : 1);
    if (buf.size() != head + body + 8) return bfail(c, OTM_EIO, "batch state file size does not match its header");
    Fnv1a h;
    h.add(buf.data(), head + body);
    uint64_t digest;
    std::memcpy(&digest, &buf[head + body], 8);
    if (digest != h.h) return bfail(c, OTM_EIO, "batch state file checksum mismatch");
    std::vector<VolumeBound> gov(c->count);
    for (int d = 0; d < c->count; ++d) {
        const unsigned char* q = &buf[top + (size_t)d * per];
        int32_t n;
        double sig[11], mine[11], g[8];
        std::memcpy(&n, q, 4);
        std::memcpy(sig, q + 8, sizeof(sig));
        std::memcpy(g, q + 8 + sizeof(sig), sizeof(g));
        problem_signature(c->prob[d], mine);
        if (n != c->prob[d].n || std::memcmp(sig, mine, sizeof(sig)) != 0)
            return bfail(c, OTM_EINVAL, "batch state file was written for other problems (n, constants, target or "
                                        "objective of design " + std::to_string(d) + ")");
        for (double v : g)
            if (!std::isfinite(v)) return bfail(c, OTM_ENONFINITE, "non-finite governor state in batch state file");
        governor_in(g, gov[d]);
    }
    if (cells != (size_t)c->total) return bfail(c, OTM_EINVAL, "batch state file was written for other grid sizes");
    std::vector<double> vals(body / sizeof(double));
    std::memcpy(vals.data(), &buf[head], body);
    for (double v : vals)
        if (!std::isfinite(v)) return bfail(c, OTM_ENONFINITE, "non-finite value in batch state file");
    BCHK(c, hipMemcpyAsync(c->rho, vals.data(), (size_t)c->total * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (flags & 1u)
        BCHK(c, hipMemcpyAsync(c->x, vals.data() + c->total, 3 * (size_t)c->total * sizeof(double),
                               hipMemcpyHostToDevice, c->stream));
    BCHK(c, hipStreamSynchronize(c->stream));  // vals may go
    c->gov = gov;
    c->iter = iter;
    c->have_density.assign(c->count, 1);
    c->have_solution = (flags & 1u) != 0;
    return OTM_OK;
}

int otm_batch_get_governor(const otm_batch* c, int32_t d, double s[8]) {
    if (!c || !s || d < 0 || d >= c->count) return OTM_EINVAL;
    const VolumeBound& v = c->gov[d];
    s[0] = v.vstar;
    s[1] = v.df;
    s[2] = (double)v.stalls;
    s[3] = v.gap;
    s[4] = v.g_prev;
    s[5] = (double)v.flat;
    s[6] = (double)c->iter;
    s[7] = v.move;
    return OTM_OK;
}

int otm_batch_device_bytes(const otm_batch* c, int64_t* bytes) {
    if (!c || !bytes) return OTM_EINVAL;
    *bytes = c->dev_bytes;
    return OTM_OK;
}

int otm_batch_info(const otm_batch* c, double info8[10]) {
    if (!c || !info8) return OTM_EINVAL;
    info8[0] = (double)c->count;
    info8[1] = (double)c->total;
    info8[2] = (double)c->tab.mb_total;
    info8[3] = (double)(2 * c->wx);
    info8[4] = c->hdesc.empty() ? 0.0 : (double)c->hdesc[0].tz;
    info8[5] = c->tune_us;
    info8[6] = c->t_ms[1];
    info8[7] = c->t_ms[3];
    info8[8] = c->fused ? 1.0 : 0.0;
    info8[9] = (double)c->refreshes;
    return OTM_OK;
}

const char* otm_batch_last_error(const otm_batch* c) { return c ? c->err.c_str() : "null batch"; }

}  // extern "C"
