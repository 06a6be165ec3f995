// Internal declarations shared by the kernel and engine translation units.
// Not part of the public ABI (include/opentm_amd.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "opentm_amd.h"

namespace otm {

constexpr int kBlock = 256;          // threads per block for node/element sweeps
constexpr int kMaxReduce = 32;       // widest multi-value block reduction
constexpr int kMaxBlocks = 4096;     // producer blocks per reduction (workspace rows)
constexpr int kFusedSums = 15;       // partial sums per block of a fused PCG pass, per load l: [l] p.q,
                                     // [3+l] q.z, [6+l] q.D^-1 q, [9+l] r.z, [12+l] r.r
constexpr int kFinThreads = 1024;    // fused-pass finalize: one wave per partial sum
constexpr int kOcLevels = 5;         // bisection levels resolved per OC pass
constexpr int kOcCands = (1 << kOcLevels) - 1;
// passes that reach the bisection's 200-halving cap, plus the first and a spare
constexpr int kOcMaxPasses = 200 / kOcLevels + 2;
// partial sums of a fused pass: value-major (value v of slot b at v * kMaxBlocks + b),
// one such region per pass parity
constexpr int64_t kFusedStride = (int64_t)kFusedSums * kMaxBlocks;

// State of the fused PCG iteration between passes (per load): the step and
// direction weight a pass used, the last reduced dots, and the constants the
// convergence test needs.  Two copies, by pass parity, live in Scalars: a pass
// reads its predecessor's copy and writes its own.
struct FusedState {
    double alpha[3], beta[3];
    double rz[3], pq[3], qdq[3], rr[3];
    double bb[3];
    double tol2;
    int32_t active[3];
    int32_t iters[3];
};

// Device-resident scalars of the solver and the OC search.  One instance per
// context, written only by "last block" epilogues or by host copies between
// kernels.
struct Scalars {
    // PCG, per load
    double rz[3];       // r . D^-1 r of the current residual
    double rz_prev[3];  // previous value (reliable-update beta)
    double pq[3];
    double qdq[3];      // q . D^-1 q of the last pass (fused iteration)
    double alpha[3];
    double beta[3];
    double rr[3];       // recursive ||r||^2
    double bb[3];       // ||b||^2
    double rr_true[3];  // ||b - A x||^2 from the last residual refresh
    double tol2;        // tol^2
    int32_t active[3];  // load still iterating
    int32_t iters[3];
    // reductions over the design field
    double sum_rho;      // sum rho
    double sum_rhofp;    // sum rho~^p
    double bsum[3];      // sum of macro loads (projection)
    double xsum[3];      // sum of chi (projection)
    double kappa_sum[6]; // sum k_e E_e,c
    double gscale[3];    // energy-minimising factor of the start guess, per load
    // OC bisection state
    double l1, l2;
    double vstar_n;      // V* * n^3
    double lam;
    int32_t oc_steps;
    int32_t oc_done;
    double cand[kOcCands];    // lambda candidates of the current pass (bisection tree, BFS order)
    double cpow[kOcCands];    // candidate^-eta
    FusedState fs[2];         // fused iteration, by pass parity
};

// Separable periodic hat-filter weights (1-D, normalized), reach R <= 4.
struct FilterW {
    int R;
    double w[9];
};
FilterW filter_weights(double r);

struct W6 {
    double w[6];
};

// ---- batched designs -------------------------------------------------------
// Each design d owns the slice [off, off + n^3) of every n^3-sized arena and
// [3 off, 3 off + 3 n^3) of every three-load arena.  Kernels over the batch
// map work items to designs through the *_design tables; the items of a
// design are contiguous so its per-item partial sums form one range.
struct BatchDesc {
    int n;
    int64_t off;
    int eb_start, eb_count;  // element/node sweep items
    int mb_start, mb_count;  // z-march items
    int ntx, nty, tz;        // z-march tiling of this design
    double k0, kmin, penal;
    FilterW fw;
};
struct BatchTab {
    const BatchDesc* desc;
    const int* eb_design;
    const int* mb_design;
    int count, eb_total, mb_total;
};

// Launch helpers (otm_kernels.hip).  All are asynchronous on `s`.
// `partials`/`counter` are the shared reduction workspace; `sc` the device scalars.
struct Workspace {
    double* partials;   // >= max_blocks * kMaxReduce doubles
    unsigned* counter;  // one zero-initialised counter per reduction slot
    Scalars* sc;
    int max_blocks;
};

// Finalize step after a reduction kernel: one block sums the producer's
// per-block partials and updates the device scalars.
enum FinOp {
    FIN_FILTER_SIMP = 0,
    FIN_SETUP,
    FIN_RES_START,
    FIN_RES_REFRESH,
    FIN_PQ,
    FIN_UPDATE,
    FIN_SUM3_X,
    FIN_SUM3_B,
    FIN_ENERGY,
    FIN_OC,
    FIN_F_START,    // fused iteration: residual at the start of a solve
    FIN_F_REFRESH,  // fused iteration: float64 residual replaces the recursive one
    FIN_GUESS,      // scale factors of a start guess
    FIN_MG_RZ0,     // multigrid PCG: r.z after the V-cycle, (re)start with beta = 0
    FIN_MG_RZ,      // multigrid PCG: r.z after the V-cycle -> beta
    FIN_MG_UPDATE   // multigrid PCG: r.r after the update -> convergence
};
void launch_finalize(int op, int nblocks, const Workspace& ws, hipStream_t s, int64_t nn = 0, double eta = 0.5);

void launch_filter_simp(int n, double r, const double* rho, double* rhof, double* k, float* k32, double k0,
                        double kmin, double p, const Workspace& ws, hipStream_t s);
void launch_filter(int n, double r, const double* in, double* out, hipStream_t s);
void launch_setup_nodes(int n, const double* k, double* b, double* dinv, float* dinv32, const Workspace& ws,
                        hipStream_t s);

// PCG building blocks.  T = double (FP64 path) or float (mixed path); b and
// the accumulated solution are float64 in both paths.
enum { RES_START = 0, RES_REFRESH = 1 };
template <typename T>
void launch_dir(int n, const T* r, const T* dinv, const T* p_old, T* p_new, const Workspace& ws, hipStream_t s);
template <typename T>
void launch_apply_pq(int n, const T* k, const T* p, T* q, const Workspace& ws, hipStream_t s);
template <typename T>
void launch_update(int n, T* x, T* r, const T* p, const T* q, const T* dinv, const Workspace& ws, hipStream_t s);
// r = b - A x with the float64 operator (x_zero: skip the operator), stored as TR.
template <typename TR>
void launch_residual(int n, const double* k, const double* b, const double* x, TR* r, TR* p_old, const TR* dinv,
                     int mode, int x_zero, const Workspace& ws, hipStream_t s);
void launch_accumulate(int n, double* x, float* x32, hipStream_t s);
// Scales each load of the start guess x by s = b.x / x.A x (float64 operator),
// the factor that minimises the quadratic energy along x (0 if b.x <= 0).
void launch_guess_scale(int n, const double* k, const double* b, double* x, const Workspace& ws, hipStream_t s);
// slot 0: sums into sc->xsum, slot 1: into sc->bsum
void launch_sum3(int n, const double* x, int slot, const Workspace& ws, hipStream_t s);
void launch_sub_mean3(int n, double* x, int slot, const Workspace& ws, hipStream_t s);

void launch_energy(int n, const double* k, const double* chi, const Workspace& ws, hipStream_t s);
void launch_sens(int n, const double* rhof, const double* chi, const double* w6, double k0, double kmin, double p,
                 double* st, hipStream_t s);

// q_e and the bisection's upper bound per block (into ws.partials; their count in *nblocks_out)
void launch_oc_prepare(int n, const double* rho, const double* sens, double eta, double move, double rho_min,
                       double* q, const Workspace& ws, hipStream_t s, int* nblocks_out);
void launch_oc_init(double vstar, int n, double eta, int prep_blocks, const Workspace& ws, hipStream_t s);
void launch_oc_pass(int n, const double* rho, const double* q, double move, double rho_min, double eta,
                    const Workspace& ws, hipStream_t s);
void launch_oc_apply(int n, double* rho, const double* q, double eta, double move, double rho_min,
                     const Workspace& ws, hipStream_t s);
// The whole OC update with q recomputed from (rho, sens) instead of stored:
// prepare, bracket, kOcMaxPasses bisection passes (those after the stop return
// at once) and the update into rho_out, all asynchronous on `s` with no host
// round trip.  The same grids as the stored-q path, so the same lambda and
// rho_out.  Scratch: ws.sc and 1024 x 2 / 512 x kOcCands doubles of ws.partials.
void launch_oc_from_sens(int n, const double* rho, const double* sens, double* rho_out, double* lambda_out,
                         double vstar, double eta, double move, double rho_min, const Workspace& ws,
                         hipStream_t s);
void launch_clamp(int n, double* rho, double lo, double hi, hipStream_t s);
// Persistent tuning choices (otm_tunecache.hip): keyed by the current
// device's architecture and `key`, in the file named by OTM_TUNE_CACHE (no
// file: lookups miss, stores do nothing).  lookup fills vals (its size is the
// expected count) from the last matching line.
std::string device_arch();
bool tune_cache_lookup(const std::string& key, std::vector<double>& vals);
void tune_cache_store(const std::string& key, const std::vector<double>& vals);

// The objective over the six tensor components and dg/dkappa (Sec. 4.4):
// squared error, relative squared error, or l1 with d|a|/da = 0 at a = 0.
inline void objective_grad(int kind, const double* kappa, const double* target, double* g, double* w6) {
    double s = 0.0;
    for (int q = 0; q < 6; ++q) {
        if (kind == OTM_OBJ_REL) {
            const double d = kappa[q] / target[q] - 1.0;
            s += d * d;
            w6[q] = 2.0 * d / target[q];
        } else if (kind == OTM_OBJ_L1) {
            const double d = kappa[q] - target[q];
            s += d < 0.0 ? -d : d;
            w6[q] = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
        } else {
            const double d = kappa[q] - target[q];
            s += d * d;
            w6[q] = 2.0 * d;
        }
    }
    *g = s;
}

// Adaptive volume bound V* of the moving-constraint model (Sec. 2.3, model 3;
// Algorithm 1), kept between design iterations of one design.  Single
// contexts and batches hold one each and advance it with advance_volume_bound.
// Host helpers of the checkpoint files (contexts and batches): the FNV-1a
// 64-bit hash over the bytes written, and the problem constants a file must
// match to be loaded.
struct Fnv1a {
    uint64_t h = 1469598103934665603ull;
    void add(const void* p, size_t len) {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < len; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    }
};

inline void problem_signature(const otm_problem& p, double out[11]) {
    out[0] = p.k0;
    out[1] = p.kmin;
    out[2] = p.penal;
    out[3] = p.filter_radius;
    for (int q = 0; q < 6; ++q) out[4 + q] = p.target[q];
    out[10] = (double)p.objective;
}

struct VolumeBound {
    double vstar = 1.0;   // the bound V* the next OC update enforces
    double df = 1.0;      // decrease factor: the fraction of the gap removed by a shrink
    double gap = 0.0;     // V* - lowBound as measured at the last shrink (sizes a rebound)
    double g_prev = 1.0;  // objective of the previous design iteration (1 before the first)
    int stalls = 0;       // consecutive iterations that made no headway against the bound
    int flat = 0;         // consecutive iterations whose objective changed by less than g_tol
    double move = 0.0;    // OC move limit of the next update (0: not yet set, take oc.move)
    double dg_prev = 0.0; // g_prev - (the objective before it): the last change of the objective
};

// The OC move limit of the next update.  With oc.move_min = 0 it is oc.move
// (a fixed step, as the paper's OC optimizer takes it).  With oc.move_min > 0
// the step adapts to the objective's course: it halves after a design
// iteration whose change of the objective reversed the previous change (a
// zig-zag) and grows by a tenth after one that continued it, within
// [move_min, move].  A fixed step that the volume bound cannot absorb moves
// every element by the full step (a sign-of-gradient step), which circles the
// optimum at the step's own scale, visible as an objective that alternately
// rises and falls; the halving shrinks that circle.  A steady rise (the
// bound taking material away) or fall leaves the step growing.  Call before
// advance_volume_bound (which replaces g_prev).
inline double next_move(const otm_oc_opts& oc, VolumeBound& s, double g) {
    const double dg = g - s.g_prev;
    if (oc.move_min <= 0.0 || s.move <= 0.0) {
        s.move = oc.move;
    } else if (dg * s.dg_prev < 0.0) {
        s.move = 0.5 * s.move > oc.move_min ? 0.5 * s.move : oc.move_min;
    } else {
        s.move = 1.1 * s.move < oc.move ? 1.1 * s.move : oc.move;
    }
    s.dg_prev = dg;
    return s.move;
}

// One design iteration's transition, given its objective g, the
// solid-equivalent volume low = mean(rho~^p) and the volume vol = mean(rho).
// The rules of the adaptive bound:
//  * shrink: an objective at or below the tolerable value means material can
//    go; V* moves the fraction Df of the way down to `low`, and Df decays;
//  * stall: an objective above that value that barely moved while the volume
//    sits on V* means the bound is what holds the design back; such
//    iterations are counted while consecutive (a shrink or any other
//    iteration resets the count);
//  * grow: the patience-th consecutive stall raises V* by rebound * gap * Df
//    and starts the count again.
// V* stays in [rho_min, 1].  `flat` feeds the termination test (the objective
// changing little for several consecutive iterations).
inline void advance_volume_bound(const otm_governor_opts& o, double rho_min, VolumeBound& s, double g, double low,
                                 double vol) {
    const double dg = g > s.g_prev ? g - s.g_prev : s.g_prev - g;
    if (g <= o.bound) {
        s.gap = s.vstar - low;
        s.vstar = s.vstar - s.gap * s.df;
        s.df = o.decay * s.df;
        s.stalls = 0;
    } else {
        const double off = vol > s.vstar ? vol - s.vstar : s.vstar - vol;
        s.stalls = (dg < o.dg_small && off < o.dv_small) ? s.stalls + 1 : 0;
    }
    if (s.stalls >= o.patience) {
        s.vstar = s.vstar + o.rebound * s.gap * s.df;
        s.stalls = 0;
    }
    s.vstar = s.vstar > 1.0 ? 1.0 : (s.vstar < rho_min ? rho_min : s.vstar);
    s.flat = dg < o.g_tol ? s.flat + 1 : 0;
    s.g_prev = g;
}

// Governor options are usable: finite, non-negative thresholds, decay in
// [0, 1], patience and stall_iters >= 1.
inline bool governor_opts_valid(const otm_governor_opts& o) {
    auto fin = [](double v) { return v - v == 0.0; };
    return fin(o.bound) && fin(o.dg_small) && fin(o.dv_small) && fin(o.decay) && fin(o.rebound) && fin(o.g_tol) &&
           o.bound >= 0.0 && o.dg_small >= 0.0 && o.dv_small >= 0.0 && o.decay >= 0.0 && o.decay <= 1.0 &&
           o.rebound >= 0.0 && o.g_tol >= 0.0 && o.patience >= 1 && o.stall_iters >= 1;
}

// f_e = f_{n^3-1-e} = (f_e + f_{n^3-1-e}) / 2: central symmetry of an element field
void launch_sym_central(int n, double* f, hipStream_t s);

// Tiled fused direction + operator pass and vectorized update (otm_stencil.hip).
struct TileShape {
    int tx = 32, ty = 8, tz = 8;  // nodes per block in x, y; planes per z-march
    int blocks = 0;
};
TileShape choose_tile(int n, int max_blocks, int tz_override, int tx_override = 0);
template <typename T>
void launch_dir_apply(int n, const TileShape& t, const T* r, const T* dinv, const T* p_old, T* p_new, const T* k,
                      T* q, const Workspace& ws, hipStream_t s);
template <typename T>
void launch_dir_march(int n, const TileShape& t, const T* r, const T* dinv, const T* p_old, T* p_new, const T* k,
                      T* q, const Workspace& ws, hipStream_t s);
template <typename T>
void launch_apply_march(int n, const TileShape& t, const T* k, const T* x, T* y, hipStream_t s);
// Pair kernel (otm_march2.hip): two x-adjacent nodes per thread, even n only.
TileShape choose_tile2(int n, int max_blocks, int tz_override, int tx_override);
template <typename T>
void launch_dir_march2(int n, const TileShape& t, bool all_active, const T* r, const T* dinv, const T* p_old,
                       T* p_new, const T* k, T* q, const Workspace& ws, hipStream_t s, bool fin = true,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename T>
void launch_apply_march2(int n, const TileShape& t, const T* k, const T* x, T* y, hipStream_t s);
// Fused single-pass PCG iteration (otm_fused.hip): even n, pair tiles of
// choose_tile2.  r, q, p are read from *_in and written to *_out (ping-pong);
// x is updated in place.  par: parity of the pass (its partial sums and state
// copy).  chained = false: the pass takes its step from the device scalars
// (after a residual or a finalize); chained = true: every block first reduces
// the previous pass's partial sums itself (same fixed order in every block).
// fin: close the chain with a finalize that writes the device scalars.
template <typename T>
void launch_fused(int n, const TileShape& t, bool all_active, const T* r_in, const T* q_in, const T* p_in, T* r_out,
                  T* q_out, T* p_out, T* x, const T* dinv, const T* k, const Workspace& ws, hipStream_t s, int par,
                  bool chained, bool fin, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Multigrid V-cycle preconditioner (otm_mg.hip), float32.
constexpr int kMgMaxLevels = 10;
constexpr float kMgOmega = 0.9f;  // damped Jacobi weight of the relaxation
enum MgMarch { MG_NONE = 0, MG_RELAX = 1, MG_RESID = 2 };
constexpr int kMgCoarseMax = 64;  // nodes of the coarsest level (direct solve)
struct MgLevel {
    int n = 0;
    const float* k = nullptr;  // level conductivities (level 0: the solver's)
    const float* dinv = nullptr;
    float* kc = nullptr;       // owned (levels >= 1)
    float* dinvc = nullptr;
    float* x[2] = {nullptr, nullptr};
    float* f = nullptr;        // level right-hand side (level 0: the residual, not owned)
    float* t = nullptr;        // A x scratch
    TileShape tile;
};
struct MgHierarchy {
    int levels = 0;
    int sweeps = 2;          // damped Jacobi steps before and after the coarse correction (finest level)
    int coarse_sweeps = 2;   // the same on the coarser levels
    bool gs = false;         // 8-colour Gauss-Seidel sweeps instead of damped Jacobi steps
    float* minv = nullptr;   // inverse of the coarsest operator (at most 64 x 64)
    MgLevel lv[kMgMaxLevels];
};
void launch_mg_coarsen(int nc, const float* kf, float* kc, float* dinv_c, hipStream_t s);
// One z-march pass of a level (n even): out = x + w D^-1 (f - A x) (MG_RELAX)
// or f - A x (MG_RESID), with x = in, or x = w D^-1 f when from_f; MG_RELAX
// with partials writes the per-block sums f . out (t.blocks of them).
void launch_mg_march(int n, const TileShape& t, bool from_f, int mode, const float* in, const float* dinv,
                     const float* f, const float* k, float* out, double* partials, hipStream_t s);
void launch_mg_restrict(int nc, const float* r, float* fc, hipStream_t s);
// x_f += P x_c, or x_f = w D^-1 f + P x_c when f0 is given
void launch_mg_prolong(int nc, const float* xc, float* xf, const float* f0, const float* dinv0, hipStream_t s);
void launch_mg_coarse_setup(int n, const float* k, float* minv, hipStream_t s);
void launch_mg_coarse_solve(int n, const float* minv, const float* f, float* x, hipStream_t s);
// The second-coarsest level (n <= 8, even) and the coarsest below it in one
// block: x = V(f) with nu relaxation steps per leg, written to x (3 n^3).
void launch_mg_tail(int n, int nu, const float* f, const float* k, const float* dinv, const float* minv, float* x,
                    bool gs, hipStream_t s);
// z = V(r) for the three loads, r = lv[0].f; *z_out receives the level-0
// buffer that holds z.  The last relaxation writes the per-block sums r.z
// into partials; returns their block count.
int mg_vcycle(const MgHierarchy& H, double* partials, int max_blocks, hipStream_t s, const float** z_out);

// Deterministic pseudo-random fill in [-0.5, 0.5) (timing inputs), and a constant fill.
template <typename T>
void launch_fill_hash(T* p, int64_t count, uint32_t seed, hipStream_t s);
template <typename T>
void launch_fill_const(T* p, int64_t count, T v, hipStream_t s);
// r = b - A x (float64 operator) for the fused iteration; start: begin a solve
// (q unused, may be null), else refresh the recursive residual keeping the
// pending step (q = the last pass's A p).
template <typename TR>
void launch_residual_f(int n, const double* k, const double* b, const double* x, TR* r, const TR* q, const TR* dinv,
                       bool start, int x_zero, const Workspace& ws, hipStream_t s);
template <typename T>
void launch_apply_tiled(int n, const TileShape& t, const T* k, const T* x, T* y, hipStream_t s);
// launch_dir_march2<double> with a float32 z (the multigrid cycle's output);
// finalize (FIN_PQ) included.
void launch_dir_march2_zf(int n, const TileShape& t, bool all_active, const float* z, const double* dinv,
                          const double* p_old, double* p_new, const double* k, double* q, const Workspace& ws,
                          hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename T>
void launch_update_vec(int n, T* x, T* r, const T* p, const T* q, const T* dinv, const Workspace& ws, hipStream_t s,
                       bool fin = true, int fin_op = FIN_UPDATE, float* r32 = nullptr);

// Batched launches (one launch covers every design).
void launch_b_reset_solver(Scalars* sc, int count, double tol2, hipStream_t s);
void launch_b_clamp(const BatchTab& t, double* rho, double lo, double hi, hipStream_t s);
void launch_b_filter_simp(const BatchTab& t, const double* rho, double* rhof, double* k, double* partials,
                          Scalars* sc, hipStream_t s);
void launch_b_setup_nodes(const BatchTab& t, const double* k, double* b, double* dinv, double* partials, Scalars* sc,
                          hipStream_t s);
void launch_b_sum3(const BatchTab& t, const double* x, int slot, double* partials, Scalars* sc, hipStream_t s);
void launch_b_sub_mean3(const BatchTab& t, double* x, int slot, Scalars* sc, hipStream_t s);
void launch_b_residual(const BatchTab& t, const double* k, const double* b, const double* x, double* r, double* p_old,
                       const double* dinv, int mode, int x_zero, double* partials, Scalars* sc, hipStream_t s);
void launch_b_energy(const BatchTab& t, const double* k, const double* chi, double* partials, Scalars* sc,
                     hipStream_t s);
void launch_b_sens(const BatchTab& t, const double* rhof, const double* chi, const W6* w6, double* st, hipStream_t s);
void launch_b_filter(const BatchTab& t, const double* in, double* out, hipStream_t s);
void launch_b_oc_prepare(const BatchTab& t, const double* rho, const double* sens, double eta, double* q,
                         hipStream_t s);
void launch_b_oc_init(const BatchTab& t, Scalars* sc, const double* vstar, double eta, hipStream_t s);
// Batched fused PCG pass (float64, or float32 vectors and operator), followed
// by its per-design finalize when fin is set (a pass without it leaves every
// design's state as it was: the autotuner times passes that way); the
// partials need 2 kFusedStride doubles and the batch at most kMaxBlocks work
// items.  Designs whose loads have all stopped are skipped.
template <typename T>
void launch_b_fused(const BatchTab& t, int wx, int grid, const T* r_in, const T* q_in, const T* p_in, T* r_out,
                    T* q_out, T* p_out, T* x, const T* dinv, const T* k, double* partials, Scalars* sc, int par,
                    bool fin, hipStream_t s);
// r = b - A x per design (float64 operator and x; r stored as TR) with the
// sums the fused iteration (re)starts from (start: FIN_F_START, else
// FIN_F_REFRESH with the pending q).
template <typename TR>
void launch_b_residual_f(const BatchTab& t, const double* k, const double* b, const double* x, TR* r, const TR* q,
                         const TR* dinv, bool start, int x_zero, double* partials, Scalars* sc, hipStream_t s);
// x += x32, x32 = 0 per design
void launch_b_accumulate(const BatchTab& t, double* x, float* x32, hipStream_t s);
// k32 = (float)k, dinv32 = (float)dinv per design
void launch_b_to_f32(const BatchTab& t, const double* k, const double* dinv, float* k32, float* dinv32,
                     hipStream_t s);
void launch_b_oc_pass(const BatchTab& t, const double* rho, const double* q, const double* moves, double rho_min,
                      double eta, double* partials, Scalars* sc, hipStream_t s);
void launch_b_oc_apply(const BatchTab& t, double* rho, const double* q, double eta, const double* moves,
                       double rho_min, Scalars* sc, hipStream_t s);
void launch_b_finalize(const BatchTab& t, int op, int which_mb, double* partials, Scalars* sc, double eta,
                       hipStream_t s);
// z-march work-list launch (persistent blocks) and vector update, float64,
// each followed by its per-design finalize when fin is set (without it every
// design's state stays as it was: the autotuner times passes that way)
template <int WX, int TY>
void launch_b_dir_march2(const BatchTab& t, int grid, const double* r, const double* dinv, const double* p_old,
                         double* p_new, const double* k, double* q, double* partials, const Scalars* sc, bool fin,
                         hipStream_t s);
void launch_b_update_vec(const BatchTab& t, int grid, double* x, double* r, const double* p, const double* q,
                         const double* dinv, double* partials, const Scalars* sc, bool fin, hipStream_t s);

// Stateless operator y = A x (three loads)
template <typename T>
void launch_apply(int n, const T* k, const T* x, T* y, hipStream_t s);

void launch_fill_u32(unsigned* p, int count, unsigned v, hipStream_t s);
void launch_cast_f64_f32(int64_t count, const double* in, float* out, hipStream_t s);
void launch_cast_f32_f64(int64_t count, const float* in, double* out, hipStream_t s);

// The stream a network's kernels run on (a context orders its solve after
// the network's forward pass with an event on it).
hipStream_t nn_stream(const otm_nn* net);

}  // namespace otm
