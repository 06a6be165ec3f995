// Fused Jacobi-PCG iteration: one streaming pass and one reduction per
// iteration (gfx950).
//
// Plain PCG reduces twice per iteration (p.Ap for alpha, then r.D^-1 r for
// beta), so it needs two passes over the vectors.  Here the updates of
// iteration m-1 and the direction and operator of iteration m share one
// z-march:
//
//   r_m = r_{m-1} - a q_{m-1},   x += a p_{m-1},
//   z_m = D^-1 r_m,   p_m = z_m + b p_{m-1},   q_m = A p_m,
//
// where a = rz_{m-1} / pq_{m-1} and b = rz_m / rz_{m-1}.  rz_m is needed before
// r_m exists; it follows from the expansion
//   (r - a q)^T D^-1 (r - a q) = r^T D^-1 r - 2a q^T D^-1 r + a^2 q^T D^-1 q,
// whose terms the previous pass reduced next to p.q.  The same pass also
// reduces the exact r_m^T z_m and r_m^T r_m, so alpha and the convergence test
// use exact values and the expansion only bridges one step (no drift).  In exact
// arithmetic the iterates are those of plain Jacobi-PCG.
//
// Halo nodes of p_m are recomputed from r_{m-1}, q_{m-1}, p_{m-1}: r, q and p are
// double-buffered so no pass overwrites what a neighbouring block still reads.
// x is updated in place (own nodes only).  Two x-adjacent nodes per thread with
// 8-byte accesses, as the pair operator; even n only.
#include <hip/hip_ext.h>
#include <type_traits>

#include "otm_device.h"

namespace otm {

template <typename T>
struct FV2 {
    typedef T type __attribute__((ext_vector_type(2)));
};

template <typename T>
struct PreF {
    typename FV2<T>::type r[3], q[3], p[3], x[3], dv, k;  // own pair
    T hr[3], hq[3], hp[3], hdv, kh;                      // one halo node / element
};

// CHAIN: the block first reduces the previous pass's partial sums (parity
// par ^ 1, nslots of them) and advances the state itself; else it takes the
// state from the scalar block.  The design's first tile records the state it
// ran with as fs[par].  tile: the tile (x, then y, then z) this call
// computes; slot: where its partial sums go.
template <typename T, int WX, int TY, bool ALL, bool CHAIN>
__device__ __forceinline__ void fused_body(int tile, int slot, int nslots, bool first, int n, int tz, int ntx, int nty,
                                           const T* __restrict__ r_in,
                                           const T* __restrict__ q_in, const T* __restrict__ p_in,
                                           T* __restrict__ r_out, T* __restrict__ q_out, T* __restrict__ p_out,
                                           T* __restrict__ x, const T* __restrict__ dinv, const T* __restrict__ k,
                                           double* __restrict__ partials, Scalars* __restrict__ sc, int par) {
    typedef typename FV2<T>::type T2;
    static_assert(WX * TY == kBlock, "block size");
    constexpr int TX = 2 * WX;
    constexpr int PX = TX + 2, PY = TY + 2;
    constexpr int PXP = TX + 4;
    constexpr int NH = 2 * PX + 2 * (PY - 2);
    constexpr int KX = TX + 1, KY = TY + 1;
    constexpr int KXP = TX + 2;
    constexpr int NKH = KX + KY - 1;
    static_assert(NH <= kBlock && NKH <= kBlock, "halo");
    __shared__ __attribute__((aligned(16))) T sp[2][3][PY * PXP];
    __shared__ __attribute__((aligned(16))) T sk[2][KY * KXP];

    const int tid = threadIdx.x;
    const int tx = tid % WX, ty = tid / WX;
    int bid = tile;  // tiles in x, then y, then z
    const int bx = bid % ntx;
    bid /= ntx;
    const int by = bid % nty;
    const int bz = bid / nty;
    const int i0 = bx * TX, j0 = by * TY, z0 = bz * tz;
    const int z1 = min(z0 + tz, n);
    const int64_t nn = (int64_t)n * n * n;
    const int64_t n2 = (int64_t)n * n;

    // per-load uniforms: activity, step a (alpha), direction weight b (beta);
    // a chained pass with every load active prefetches its first planes with
    // every field before its state is known (fields it then does not need
    // are simply not used)
    bool act[3], ua[3], up[3];
    T al[3], be[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        act[l] = true;
        ua[l] = true;
        up[l] = true;
        al[l] = (T)0;
        be[l] = (T)0;
    }
    const int i = i0 + 2 * tx, j = j0 + ty;
    const bool own = (i < n) && (j < n);  // n even: i < n implies i + 1 < n
    const uint32_t xy_own = (uint32_t)(i % n) + (uint32_t)n * (uint32_t)(j % n);
    const int lp = (ty + 1) * PXP + (2 * tx + 1) + 1;
    const int lk = (ty + 1) * KXP + (2 * tx + 1) + 1;
    const bool has_h = tid < NH;
    uint32_t xy_h = 0;
    int lph = 0;
    if (has_h) {
        int px, py;
        if (tid < PX) {
            px = tid;
            py = 0;
        } else if (tid < 2 * PX) {
            px = tid - PX;
            py = PY - 1;
        } else if (tid < 2 * PX + (PY - 2)) {
            px = 0;
            py = 1 + (tid - 2 * PX);
        } else {
            px = PX - 1;
            py = 1 + (tid - 2 * PX - (PY - 2));
        }
        const int gi = (i0 - 1 + px + n) % n, gj = (j0 - 1 + py + n) % n;
        xy_h = (uint32_t)gi + (uint32_t)n * (uint32_t)gj;
        lph = py * PXP + px + 1;
    }
    const bool has_kh = tid < NKH;
    uint32_t xy_kh = 0;
    int lkh = 0;
    if (has_kh) {
        int kx, ky;
        if (tid < KX) {
            kx = tid;
            ky = 0;
        } else {
            kx = 0;
            ky = 1 + (tid - KX);
        }
        const int gi = (i0 - 1 + kx + n) % n, gj = (j0 - 1 + ky + n) % n;
        xy_kh = (uint32_t)gi + (uint32_t)n * (uint32_t)gj;
        lkh = ky * KXP + kx + 1;
    }

    auto plane_off = [&](int P) -> int64_t {
        const int pw = P < 0 ? P + n : (P >= n ? P - n : P);
        return (int64_t)pw * n2;
    };

    const uint32_t bo = xy_own * (uint32_t)sizeof(T);   // own pair
    const uint32_t bh = xy_h * (uint32_t)sizeof(T);     // halo node
    const uint32_t bkh = xy_kh * (uint32_t)sizeof(T);   // halo element

    // own pair loads first, then every halo load under one branch (one exec
    // mask change per plane instead of one per field)
    auto load_plane = [&](int P, PreF<T>& f) {
        const int64_t zoff = plane_off(P);
        const bool inr = P >= z0 && P < z1;
        const T* dp = dinv + zoff;
        const T* kp = k + zoff;
        f.dv = ld_at<T2>(dp, bo);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            const int64_t o = l * nn + zoff;
            f.r[l] = ld_at<T2>(r_in + o, bo);
            if (ua[l]) {
                f.q[l] = ld_at<T2>(q_in + o, bo);
                if (inr) f.x[l] = ld_at<T2>(x + o, bo);
            }
            if (up[l]) f.p[l] = ld_at<T2>(p_in + o, bo);
        }
        f.k = ld_at<T2>(kp, bo);
        if (has_h) {
            f.hdv = ld_at<T>(dp, bh);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                if (!act[l]) continue;
                const int64_t o = l * nn + zoff;
                f.hr[l] = ld_at<T>(r_in + o, bh);
                if (ua[l]) f.hq[l] = ld_at<T>(q_in + o, bh);
                if (up[l]) f.hp[l] = ld_at<T>(p_in + o, bh);
            }
        }
        if (has_kh) f.kh = ld_at<T>(kp, bkh);
    };

    // per-thread partials in T (at most 2 tz terms each), block and grid sums in float64
    T acc[kFusedSums];
#pragma unroll
    for (int q = 0; q < kFusedSums; ++q) acc[q] = (T)0;
    T2 pP[3], zP[3], dvP;

    auto store_plane = [&](int P, const PreF<T>& f) {
        const int slot = P & 1;
        const bool inr = P >= z0 && P < z1;
        const int64_t zoff = plane_off(P);
        T2 rnv[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            T2 rn = f.r[l];
            if (ua[l]) rn -= al[l] * f.q[l];
            const T2 z = f.dv * rn;
            T2 pn = z;
            if (up[l]) pn += be[l] * f.p[l];
            *reinterpret_cast<T2*>(&sp[slot][l][lp]) = pn;
            rnv[l] = rn;
            pP[l] = pn;
            zP[l] = z;
        }
        if (inr && own) {
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                if (!act[l]) continue;
                const int64_t o = l * nn + zoff;
                st_at<T2>(r_out + o, bo, rnv[l]);
                st_at<T2>(p_out + o, bo, pP[l]);
                if (ua[l]) st_at<T2>(x + o, bo, f.x[l] + al[l] * f.p[l]);
                acc[9 + l] += rnv[l].x * zP[l].x + rnv[l].y * zP[l].y;
                acc[12 + l] += rnv[l].x * rnv[l].x + rnv[l].y * rnv[l].y;
            }
        }
        dvP = f.dv;
        *reinterpret_cast<T2*>(&sk[slot][lk]) = f.k;
        if (has_h) {
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                if (!act[l]) continue;
                T hrn = f.hr[l];
                if (ua[l]) hrn -= al[l] * f.hq[l];
                T hpn = f.hdv * hrn;
                if (up[l]) hpn += be[l] * f.hp[l];
                sp[slot][l][lph] = hpn;
            }
        }
        if (has_kh) sk[slot][lkh] = f.kh;
    };

    const T w = (T)(1.0 / 12.0);
    const T third = (T)(1.0 / 3.0);
    T2 yA[3], yB[3], pB[3], zB[3], dvB = (T2)((T)0);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        yA[l] = (T2)((T)0);
        yB[l] = (T2)((T)0);
        pB[l] = (T2)((T)0);
        zB[l] = (T2)((T)0);
    }
    T kpm0 = 0, kpm1 = 0, kpm2 = 0, kpc0 = 0, kpc1 = 0, kpc2 = 0;

    // Node plane P arrives: finish node P-1 (its dz = +1 taps), add the
    // in-plane taps of node P, start node P+1 (dz = -1 taps).
    auto compute = [&](int P) {
        const int slot = P & 1;
        const T* K = sk[slot];
        const T km0 = K[lk - KXP - 1];
        const T2 km12 = *reinterpret_cast<const T2*>(&K[lk - KXP]);
        const T kc0 = K[lk - 1];
        const T2 kc12 = *reinterpret_cast<const T2*>(&K[lk]);
        const T km1 = km12.x, km2 = km12.y, kc1 = kc12.x, kc2 = kc12.y;
        const T pa_xm = kpm0 + kpc0, pa_xp = kpm1 + kpc1, pa_ym = kpm0 + kpm1, pa_yp = kpc0 + kpc1;
        const T pb_xm = kpm1 + kpc1, pb_xp = kpm2 + kpc2, pb_ym = kpm1 + kpm2, pb_yp = kpc1 + kpc2;
        const T ca_xm = km0 + kc0, ca_xp = km1 + kc1, ca_ym = km0 + km1, ca_yp = kc0 + kc1;
        const T cb_xm = km1 + kc1, cb_xp = km2 + kc2, cb_ym = km1 + km2, cb_yp = kc1 + kc2;
        const T ea0 = kpm0 + km0, ea1 = kpm1 + km1, ea2 = kpc0 + kc0, ea3 = kpc1 + kc1;
        const T eb0 = kpm1 + km1, eb1 = kpm2 + km2, eb2 = kpc1 + kc1, eb3 = kpc2 + kc2;
        const T c0a = (ea0 + ea1 + ea2 + ea3) * third;
        const T c0b = (eb0 + eb1 + eb2 + eb3) * third;
        const bool done = (P - 1 >= z0) && own;
        T2 qd[3];
        const int64_t zdone = (int64_t)(P - 1 < 0 ? 0 : (P - 1)) * n2;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            const T* L = sp[slot][l];
            const T m0 = L[lp - PXP - 1];
            const T2 m12 = *reinterpret_cast<const T2*>(&L[lp - PXP]);
            const T m3 = L[lp - PXP + 2];
            const T c0v = L[lp - 1];
            const T2 c12 = *reinterpret_cast<const T2*>(&L[lp]);
            const T c3 = L[lp + 2];
            const T p0 = L[lp + PXP - 1];
            const T2 p12 = *reinterpret_cast<const T2*>(&L[lp + PXP]);
            const T p3 = L[lp + PXP + 2];
            const T m1 = m12.x, m2 = m12.y, c1 = c12.x, c2 = c12.y, p1 = p12.x, p2 = p12.y;
            const T opa = pa_xm * c0v + pa_xp * c2 + pa_ym * m1 + pa_yp * p1 + kpm0 * m0 + kpm1 * m2 + kpc0 * p0 +
                          kpc1 * p2;
            const T oca = ca_xm * c0v + ca_xp * c2 + ca_ym * m1 + ca_yp * p1 + km0 * m0 + km1 * m2 + kc0 * p0 +
                          kc1 * p2;
            const T ina = c0a * c1 - w * (ea0 * m0 + ea1 * m2 + ea2 * p0 + ea3 * p2);
            const T opb = pb_xm * c1 + pb_xp * c3 + pb_ym * m2 + pb_yp * p2 + kpm1 * m1 + kpm2 * m3 + kpc1 * p1 +
                          kpc2 * p3;
            const T ocb = cb_xm * c1 + cb_xp * c3 + cb_ym * m2 + cb_yp * p2 + km1 * m1 + km2 * m3 + kc1 * p1 +
                          kc2 * p3;
            const T inb = c0b * c2 - w * (eb0 * m1 + eb1 * m3 + eb2 * p1 + eb3 * p3);
            T2 qv;
            qv.x = yA[l].x - w * opa;
            qv.y = yA[l].y - w * opb;
            qd[l] = qv;
            T2 yb;
            yb.x = yB[l].x + ina;
            yb.y = yB[l].y + inb;
            yA[l] = yb;
            yB[l].x = -w * oca;
            yB[l].y = -w * ocb;
        }
        if (done) {
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                if (!act[l]) continue;
                const T2 qv = qd[l];
                st_at<T2>(q_out + l * nn + zdone, bo, qv);
                acc[l] += pB[l].x * qv.x + pB[l].y * qv.y;
                acc[3 + l] += zB[l].x * qv.x + zB[l].y * qv.y;
                acc[6 + l] += dvB.x * qv.x * qv.x + dvB.y * qv.y * qv.y;
            }
        }
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            pB[l] = pP[l];
            zB[l] = zP[l];
        }
        dvB = dvP;
        kpm0 = km0;
        kpm1 = km1;
        kpm2 = km2;
        kpc0 = kc0;
        kpc1 = kc1;
        kpc2 = kc2;
    };

    __shared__ FusedState st_sh;
    __shared__ double tot[kFusedSums];
    auto take_state = [&]() {
        if (CHAIN) {
            final_sums_vm<kFusedSums>(partials + (par ^ 1) * kFusedStride, nslots, tot);
            if (tid == 0) {
                FusedState s;
                fused_advance(sc->fs[par ^ 1], tot, s);
                st_sh = s;
                if (first) sc->fs[par] = s;
            }
        } else if (tid == 0) {
            FusedState s;
            fused_state_of(sc, s);
            st_sh = s;
            if (first) sc->fs[par] = s;
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            act[l] = ALL ? true : (st_sh.active[l] != 0);
            al[l] = (T)st_sh.alpha[l];
            be[l] = (T)st_sh.beta[l];
            ua[l] = act[l] && al[l] != (T)0;
            up[l] = ua[l] || (act[l] && be[l] != (T)0);
        }
    };

    // With every load active the first two planes' loads do not depend on the
    // state (the flags gating them start true; what the state then switches
    // off is loaded but not used), so they go out before the state read and
    // its barrier, and the two latencies overlap.
    PreF<T> fa, fb;
    if (ALL) {
        load_plane(z0 - 1, fa);
        load_plane(z0, fb);
        take_state();
        // every load stopped inside the chunk: nothing left to step until the
        // host sees it (the finalize ignores inactive loads' sums; a restart
        // recomputes r from x and keeps the last consistent p, q = A p pair)
        if (!st_sh.active[0] && !st_sh.active[1] && !st_sh.active[2]) return;
    } else {
        take_state();
        load_plane(z0 - 1, fa);
        load_plane(z0, fb);
    }
    int P = z0 - 1;
    for (; P + 1 <= z1; P += 2) {
        store_plane(P, fa);
        if (P + 2 <= z1) load_plane(P + 2, fa);
        __syncthreads();
        compute(P);
        store_plane(P + 1, fb);
        if (P + 3 <= z1) load_plane(P + 3, fb);
        __syncthreads();
        compute(P + 1);
    }
    if (P <= z1) {
        store_plane(P, fa);
        __syncthreads();
        compute(P);
    }
    double accd[kFusedSums];
#pragma unroll
    for (int q = 0; q < kFusedSums; ++q) accd[q] = (double)acc[q];
    block_partials_vm<kFusedSums>(accd, partials + par * kFusedStride, slot);
}

// Closes a chain of passes: reduces the last pass's partial sums, advances the
// state and writes it to the scalar block (host-visible).  The last wave has
// no sum of its own (15 sums, 16 waves): its first lane loads the state the
// pass ran with while the other waves' partial loads are in flight, and
// advances it.
__global__ void __launch_bounds__(kFinThreads) k_fused_fin(int nblocks, const double* __restrict__ partials,
                                                      Scalars* __restrict__ sc, int par) {
    __shared__ double tot[kFusedSums];
    const bool lead = threadIdx.x == blockDim.x - 64;
    FusedState in;
    if (lead) in = sc->fs[par];
    final_sums_vm<kFusedSums>(partials + par * kFusedStride, nblocks, tot);
    if (!lead) return;
    FusedState s;
    fused_advance(in, tot, s);
    for (int l = 0; l < 3; ++l) {
        sc->alpha[l] = s.alpha[l];
        sc->beta[l] = s.beta[l];
        sc->rz[l] = s.rz[l];
        sc->pq[l] = s.pq[l];
        sc->qdq[l] = s.qdq[l];
        sc->rr[l] = s.rr[l];
        sc->active[l] = s.active[l];
        sc->iters[l] = s.iters[l];
    }
}

// float32: two waves per SIMD (two blocks per CU) must fit, i.e. at most 256
// registers per lane; float64 state does not fit that and runs one wave per SIMD.
template <int WX, int TY, bool ALL, bool CHAIN>
__global__ void __launch_bounds__(WX* TY) __attribute__((amdgpu_waves_per_eu(2)))
    k_fused_f32(int n, int tz, int ntx, int nty, const float* __restrict__ r_in, const float* __restrict__ q_in,
                const float* __restrict__ p_in, float* __restrict__ r_out, float* __restrict__ q_out,
                float* __restrict__ p_out, float* __restrict__ x, const float* __restrict__ dinv,
                const float* __restrict__ k, double* __restrict__ partials, Scalars* __restrict__ sc, int par) {
    fused_body<float, WX, TY, ALL, CHAIN>(xcd_tile(blockIdx.x, gridDim.x), blockIdx.x, gridDim.x, blockIdx.x == 0, n, tz,
                                          ntx, nty, r_in, q_in, p_in, r_out, q_out, p_out, x, dinv, k, partials, sc,
                                          par);
}

template <int WX, int TY, bool ALL, bool CHAIN>
__global__ void __launch_bounds__(WX* TY)
    k_fused_f64(int n, int tz, int ntx, int nty, const double* __restrict__ r_in, const double* __restrict__ q_in,
                const double* __restrict__ p_in, double* __restrict__ r_out, double* __restrict__ q_out,
                double* __restrict__ p_out, double* __restrict__ x, const double* __restrict__ dinv,
                const double* __restrict__ k, double* __restrict__ partials, Scalars* __restrict__ sc, int par) {
    fused_body<double, WX, TY, ALL, CHAIN>(xcd_tile(blockIdx.x, gridDim.x), blockIdx.x, gridDim.x, blockIdx.x == 0, n,
                                           tz, ntx, nty, r_in, q_in, p_in, r_out, q_out, p_out, x, dinv, k, partials,
                                           sc, par);
}

template <typename T, int WX, int TY, bool ALL, bool CHAIN>
struct FusedKernel;
template <int WX, int TY, bool ALL, bool CHAIN>
struct FusedKernel<float, WX, TY, ALL, CHAIN> {
    static constexpr auto fn = k_fused_f32<WX, TY, ALL, CHAIN>;
};
template <int WX, int TY, bool ALL, bool CHAIN>
struct FusedKernel<double, WX, TY, ALL, CHAIN> {
    static constexpr auto fn = k_fused_f64<WX, TY, ALL, CHAIN>;
};

// ev0/ev1 (optional): HIP events recorded at the kernel's start and end.
template <typename T, bool ALL, bool CHAIN>
static void launch_f(int n, const TileShape& t, const T* r_in, const T* q_in, const T* p_in, T* r_out, T* q_out,
                     T* p_out, T* x, const T* dinv, const T* k, double* partials, Scalars* sc, int par, hipStream_t s,
                     hipEvent_t ev0, hipEvent_t ev1) {
    const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
    if (t.tx == 32)
        hipExtLaunchKernelGGL((FusedKernel<T, 16, 16, ALL, CHAIN>::fn), dim3(t.blocks), dim3(kBlock), 0, s, ev0, ev1,
                              0, n, t.tz, ntx, nty, r_in, q_in, p_in, r_out, q_out, p_out, x, dinv, k, partials, sc,
                              par);
    else
        hipExtLaunchKernelGGL((FusedKernel<T, 32, 8, ALL, CHAIN>::fn), dim3(t.blocks), dim3(kBlock), 0, s, ev0, ev1, 0,
                              n, t.tz, ntx, nty, r_in, q_in, p_in, r_out, q_out, p_out, x, dinv, k, partials, sc, par);
}

template <typename T>
void launch_fused(int n, const TileShape& t, bool all_active, const T* r_in, const T* q_in, const T* p_in, T* r_out,
                  T* q_out, T* p_out, T* x, const T* dinv, const T* k, const Workspace& ws, hipStream_t s, int par,
                  bool chained, bool fin, hipEvent_t ev0, hipEvent_t ev1) {
    if (all_active) {
        if (chained)
            launch_f<T, true, true>(n, t, r_in, q_in, p_in, r_out, q_out, p_out, x, dinv, k, ws.partials, ws.sc, par,
                                    s, ev0, ev1);
        else
            launch_f<T, true, false>(n, t, r_in, q_in, p_in, r_out, q_out, p_out, x, dinv, k, ws.partials, ws.sc, par,
                                     s, ev0, ev1);
    } else {
        if (chained)
            launch_f<T, false, true>(n, t, r_in, q_in, p_in, r_out, q_out, p_out, x, dinv, k, ws.partials, ws.sc, par,
                                     s, ev0, ev1);
        else
            launch_f<T, false, false>(n, t, r_in, q_in, p_in, r_out, q_out, p_out, x, dinv, k, ws.partials, ws.sc,
                                      par, s, ev0, ev1);
    }
    if (fin) hipLaunchKernelGGL(k_fused_fin, dim3(1), dim3(kFinThreads), 0, s, t.blocks, ws.partials, ws.sc, par);
}

template void launch_fused<float>(int, const TileShape&, bool, const float*, const float*, const float*, float*,
                                  float*, float*, float*, const float*, const float*, const Workspace&, hipStream_t,
                                  int, bool, bool, hipEvent_t, hipEvent_t);
template void launch_fused<double>(int, const TileShape&, bool, const double*, const double*, const double*, double*,
                                   double*, double*, double*, const double*, const double*, const Workspace&,
                                   hipStream_t, int, bool, bool, hipEvent_t, hipEvent_t);

// Deterministic fills for timing inputs: a 32-bit integer hash of the index
// mapped to [-0.5, 0.5), and a constant.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill_hash(T* __restrict__ p, int64_t count, uint32_t seed) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    uint32_t h = (uint32_t)i * 2654435761u ^ seed;
    h ^= h >> 16;
    h *= 2246822519u;
    h ^= h >> 13;
    h *= 3266489917u;
    h ^= h >> 16;
    p[i] = (T)((double)h * (1.0 / 4294967296.0) - 0.5);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill_const(T* __restrict__ p, int64_t count, T v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) p[i] = v;
}

template <typename T>
void launch_fill_hash(T* p, int64_t count, uint32_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_hash<T>, dim3(nblocks_for(count)), dim3(kBlock), 0, s, p, count, seed);
}
template <typename T>
void launch_fill_const(T* p, int64_t count, T v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_const<T>, dim3(nblocks_for(count)), dim3(kBlock), 0, s, p, count, v);
}
template void launch_fill_hash<float>(float*, int64_t, uint32_t, hipStream_t);
template void launch_fill_hash<double>(double*, int64_t, uint32_t, hipStream_t);
template void launch_fill_const<float>(float*, int64_t, float, hipStream_t);
template void launch_fill_const<double>(double*, int64_t, double, hipStream_t);

// r = b - A x with the float64 operator, stored as TR, with the sums the fused
// iteration restarts from: per load [l] r.r (float64 r), [3+l] r.D^-1 r and
// [9+l] q.D^-1 r (stored r), [6+l] b.b.  q may be null (start: no pending step).
// (bid, nblk: this block's index and the block count of its design;
// partials: slot bid of the design's range.)
template <typename TR>
__device__ __forceinline__ void b_residual_f(int bid, int nblk, int n, const double* __restrict__ k,
                                             const double* __restrict__ b, const double* __restrict__ x,
                                             TR* __restrict__ r, const TR* __restrict__ q,
                                             const TR* __restrict__ dinv, int x_zero, double* __restrict__ partials) {
    const int64_t nn = (int64_t)n * n * n;
    double acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = 0.0;
    for (int64_t v = (int64_t)bid * kBlock + threadIdx.x; v < nn; v += (int64_t)nblk * kBlock) {
        double ax[3] = {0.0, 0.0, 0.0};
        if (!x_zero) {
            int i, j, kk;
            node_ijk(v, n, i, j, kk);
            const Nbr o = nbr_of(i, j, kk, n);
            double ko[8];
            load_k8(k, o, ko);
            NodeCoef<double> c;
            node_coefs(ko, c);
#pragma unroll
            for (int l = 0; l < 3; ++l) ax[l] = stencil_node<double, double>(c, o, x + l * nn);
        }
        const double dv = (double)dinv[v];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const double bv = b[l * nn + v];
            const double rv = bv - ax[l];
            const TR rs = (TR)rv;
            r[l * nn + v] = rs;
            const double zs = dv * (double)rs;
            acc[l] += rv * rv;
            acc[3 + l] += zs * (double)rs;
            acc[6 + l] += bv * bv;
            if (q) acc[9 + l] += (double)q[l * nn + v] * zs;
        }
    }
    block_partials_at<12>(acc, partials, bid);
}

template <typename TR>
__global__ void __launch_bounds__(kBlock)
    k_residual_f(int n, const double* __restrict__ k, const double* __restrict__ b, const double* __restrict__ x,
                 TR* __restrict__ r, const TR* __restrict__ q, const TR* __restrict__ dinv, int x_zero,
                 double* __restrict__ partials) {
    b_residual_f<TR>(blockIdx.x, gridDim.x, n, k, b, x, r, q, dinv, x_zero, partials);
}

// ---- batches of designs ---------------------------------------------------
// The fused pass over a batch's work list of (design, tile) items: each block
// walks items (contiguous ranges per XCD), the design's first tile records
// its state, and item i's partial sums go to slot i (value-major, so the
// batch needs at most kMaxBlocks items).  Every design and load may be
// inactive (per-design state); the items of a design whose three loads have
// all stopped are skipped, and so is its finalize (a stopped design's state
// is a fixed point of the pass and the finalize).
__device__ __forceinline__ bool design_live(const Scalars* s) {
    return (s->active[0] | s->active[1] | s->active[2]) != 0;
}

template <typename T, int WX, int TY>
__device__ __forceinline__ void b_fused_items(const BatchTab& t, const T* __restrict__ r_in,
                                              const T* __restrict__ q_in, const T* __restrict__ p_in,
                                              T* __restrict__ r_out, T* __restrict__ q_out, T* __restrict__ p_out,
                                              T* __restrict__ x, const T* __restrict__ dinv, const T* __restrict__ k,
                                              double* __restrict__ partials, Scalars* __restrict__ sc, int par) {
    for (int v = blockIdx.x; v < t.mb_total; v += gridDim.x) {
        const int item = xcd_tile(v, t.mb_total);
        const int d = t.mb_design[item];
        if (!design_live(sc + d)) continue;  // uniform over the block
        const BatchDesc D = t.desc[d];
        const int64_t o1 = D.off, o3 = 3 * D.off;
        __syncthreads();  // the previous item's LDS rings are no longer read
        fused_body<T, WX, TY, false, false>(item - D.mb_start, item, 0, item == D.mb_start, D.n, D.tz, D.ntx, D.nty,
                                            r_in + o3, q_in + o3, p_in + o3, r_out + o3, q_out + o3, p_out + o3,
                                            x + o3, dinv + o1, k + o1, partials, sc + d, par);
    }
}

template <int WX, int TY>
__global__ void __launch_bounds__(WX* TY) __attribute__((amdgpu_waves_per_eu(2)))
    kb_fused_f32(BatchTab t, const float* __restrict__ r_in, const float* __restrict__ q_in,
                 const float* __restrict__ p_in, float* __restrict__ r_out, float* __restrict__ q_out,
                 float* __restrict__ p_out, float* __restrict__ x, const float* __restrict__ dinv,
                 const float* __restrict__ k, double* __restrict__ partials, Scalars* __restrict__ sc, int par) {
    b_fused_items<float, WX, TY>(t, r_in, q_in, p_in, r_out, q_out, p_out, x, dinv, k, partials, sc, par);
}

template <int WX, int TY>
__global__ void __launch_bounds__(WX* TY)
    kb_fused_f64(BatchTab t, const double* __restrict__ r_in, const double* __restrict__ q_in,
                 const double* __restrict__ p_in, double* __restrict__ r_out, double* __restrict__ q_out,
                 double* __restrict__ p_out, double* __restrict__ x, const double* __restrict__ dinv,
                 const double* __restrict__ k, double* __restrict__ partials, Scalars* __restrict__ sc, int par) {
    b_fused_items<double, WX, TY>(t, r_in, q_in, p_in, r_out, q_out, p_out, x, dinv, k, partials, sc, par);
}

// Per design (one block each): reduce the pass's partial sums of the design's
// items and advance its state (the batch form of k_fused_fin).
__global__ void __launch_bounds__(kFinThreads) kb_fused_fin(BatchTab t, const double* __restrict__ partials,
                                                       Scalars* __restrict__ sc, int par) {
    const int d = blockIdx.x;
    Scalars* s = sc + d;
    if (!design_live(s)) return;  // uniform over the block
    const BatchDesc D = t.desc[d];
    __shared__ double tot[kFusedSums];
    const bool lead = threadIdx.x == blockDim.x - 64;  // the wave without a sum (as in k_fused_fin)
    FusedState in;
    if (lead) in = s->fs[par];
    final_sums_vm<kFusedSums>(partials + par * kFusedStride + D.mb_start, D.mb_count, tot);
    if (!lead) return;
    FusedState st;
    fused_advance(in, tot, st);
    for (int l = 0; l < 3; ++l) {
        s->alpha[l] = st.alpha[l];
        s->beta[l] = st.beta[l];
        s->rz[l] = st.rz[l];
        s->pq[l] = st.pq[l];
        s->qdq[l] = st.qdq[l];
        s->rr[l] = st.rr[l];
        s->active[l] = st.active[l];
        s->iters[l] = st.iters[l];
    }
}

template <typename TR>
__global__ void __launch_bounds__(kBlock) kb_residual_f(BatchTab t, const double* __restrict__ k,
                                                        const double* __restrict__ b, const double* __restrict__ x,
                                                        TR* __restrict__ r, const TR* __restrict__ q,
                                                        const TR* __restrict__ dinv, int x_zero,
                                                        double* __restrict__ partials) {
    const int g = blockIdx.x;
    const int d = t.eb_design[g];
    const BatchDesc D = t.desc[d];
    const int64_t o1 = D.off, o3 = 3 * D.off;
    b_residual_f<TR>(g - D.eb_start, D.eb_count, D.n, k + o1, b + o3, x + o3, r + o3, q ? q + o3 : nullptr,
                     dinv + o1, x_zero, partials + (size_t)D.eb_start * 12);
}

// x += x32, x32 = 0 for every design (the float32 iterate folded into the
// float64 solution)
__global__ void __launch_bounds__(kBlock) kb_accumulate(BatchTab t, double* __restrict__ x, float* __restrict__ x32) {
    const int g = blockIdx.x;
    const int d = t.eb_design[g];
    const BatchDesc D = t.desc[d];
    const int64_t o3 = 3 * D.off, cnt = 3 * (int64_t)D.n * D.n * D.n;
    for (int64_t v = (int64_t)(g - D.eb_start) * kBlock + threadIdx.x; v < cnt; v += (int64_t)D.eb_count * kBlock) {
        x[o3 + v] += (double)x32[o3 + v];
        x32[o3 + v] = 0.0f;
    }
}

// float32 copies of the element conductivities and the inverse diagonal
__global__ void __launch_bounds__(kBlock) kb_to_f32(BatchTab t, const double* __restrict__ k,
                                                    const double* __restrict__ dinv, float* __restrict__ k32,
                                                    float* __restrict__ dinv32) {
    const int g = blockIdx.x;
    const int d = t.eb_design[g];
    const BatchDesc D = t.desc[d];
    const int64_t o1 = D.off, nn = (int64_t)D.n * D.n * D.n;
    for (int64_t v = (int64_t)(g - D.eb_start) * kBlock + threadIdx.x; v < nn; v += (int64_t)D.eb_count * kBlock) {
        k32[o1 + v] = (float)k[o1 + v];
        dinv32[o1 + v] = (float)dinv[o1 + v];
    }
}

template <typename T>
void launch_b_fused(const BatchTab& t, int wx, int grid, const T* r_in, const T* q_in, const T* p_in, T* r_out,
                    T* q_out, T* p_out, T* x, const T* dinv, const T* k, double* partials, Scalars* sc, int par,
                    bool fin, hipStream_t s) {
    if constexpr (std::is_same<T, float>::value) {
        if (wx == 32)
            hipLaunchKernelGGL((kb_fused_f32<32, 8>), dim3(grid), dim3(kBlock), 0, s, t, r_in, q_in, p_in, r_out,
                               q_out, p_out, x, dinv, k, partials, sc, par);
        else
            hipLaunchKernelGGL((kb_fused_f32<16, 16>), dim3(grid), dim3(kBlock), 0, s, t, r_in, q_in, p_in, r_out,
                               q_out, p_out, x, dinv, k, partials, sc, par);
    } else {
        if (wx == 32)
            hipLaunchKernelGGL((kb_fused_f64<32, 8>), dim3(grid), dim3(kBlock), 0, s, t, r_in, q_in, p_in, r_out,
                               q_out, p_out, x, dinv, k, partials, sc, par);
        else
            hipLaunchKernelGGL((kb_fused_f64<16, 16>), dim3(grid), dim3(kBlock), 0, s, t, r_in, q_in, p_in, r_out,
                               q_out, p_out, x, dinv, k, partials, sc, par);
    }
    if (fin) hipLaunchKernelGGL(kb_fused_fin, dim3(t.count), dim3(kFinThreads), 0, s, t, partials, sc, par);
}

template void launch_b_fused<float>(const BatchTab&, int, int, const float*, const float*, const float*, float*,
                                    float*, float*, float*, const float*, const float*, double*, Scalars*, int, bool,
                                    hipStream_t);
template void launch_b_fused<double>(const BatchTab&, int, int, const double*, const double*, const double*,
                                     double*, double*, double*, double*, const double*, const double*, double*,
                                     Scalars*, int, bool, hipStream_t);

template <typename TR>
void launch_b_residual_f(const BatchTab& t, const double* k, const double* b, const double* x, TR* r, const TR* q,
                         const TR* dinv, bool start, int x_zero, double* partials, Scalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(kb_residual_f<TR>, dim3(t.eb_total), dim3(kBlock), 0, s, t, k, b, x, r, q, dinv, x_zero,
                       partials);
    launch_b_finalize(t, start ? FIN_F_START : FIN_F_REFRESH, 0, partials, sc, 0.5, s);
}

template void launch_b_residual_f<float>(const BatchTab&, const double*, const double*, const double*, float*,
                                         const float*, const float*, bool, int, double*, Scalars*, hipStream_t);
template void launch_b_residual_f<double>(const BatchTab&, const double*, const double*, const double*, double*,
                                          const double*, const double*, bool, int, double*, Scalars*, hipStream_t);

void launch_b_accumulate(const BatchTab& t, double* x, float* x32, hipStream_t s) {
    hipLaunchKernelGGL(kb_accumulate, dim3(t.eb_total), dim3(kBlock), 0, s, t, x, x32);
}

void launch_b_to_f32(const BatchTab& t, const double* k, const double* dinv, float* k32, float* dinv32,
                     hipStream_t s) {
    hipLaunchKernelGGL(kb_to_f32, dim3(t.eb_total), dim3(kBlock), 0, s, t, k, dinv, k32, dinv32);
}

template <typename TR>
void launch_residual_f(int n, const double* k, const double* b, const double* x, TR* r, const TR* q, const TR* dinv,
                       bool start, int x_zero, const Workspace& ws, hipStream_t s) {
    const int64_t nn = (int64_t)n * n * n;
    const int g = grid_for(nn, ws.max_blocks);
    hipLaunchKernelGGL(k_residual_f<TR>, dim3(g), dim3(kBlock), 0, s, n, k, b, x, r, q, dinv, x_zero, ws.partials);
    launch_finalize(start ? FIN_F_START : FIN_F_REFRESH, g, ws, s);
}

template void launch_residual_f<float>(int, const double*, const double*, const double*, float*, const float*,
                                       const float*, bool, int, const Workspace&, hipStream_t);
template void launch_residual_f<double>(int, const double*, const double*, const double*, double*, const double*,
                                        const double*, bool, int, const Workspace&, hipStream_t);

}  // namespace otm
