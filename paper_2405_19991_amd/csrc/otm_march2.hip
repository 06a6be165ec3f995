// Streaming z-march operator, two nodes per thread (gfx950).
//
// Same arithmetic as k_march (otm_stencil.hip): each incoming node plane P
// finishes node P-1 (its dz=+1 taps), adds the in-plane taps of node P and
// starts node P+1 (dz=-1 taps), using the conductivities of element planes
// P-1 and P.  Here every thread owns the x-adjacent node pair (i, i+1), i even,
// so global and LDS traffic use 8-byte (float2 / double2) accesses and each
// LDS row of the 3x4 neighbourhood costs three reads instead of six.
// Requires an even n (a pair never straddles the periodic wrap).
//
// The march is unrolled by two planes so that the two-plane register
// prefetch alternates between two register sets without copies.
#include <hip/hip_ext.h>

#include <type_traits>

#include "otm_device.h"

namespace otm {

// Streaming store (nontemporal hint): the stand-alone operator's result is
// not re-read by this launch, so it should not displace the inputs in cache.
template <typename V>
__device__ __forceinline__ void st_stream(void* base, uint32_t boff, V v) {
    asm volatile("" : "+v"(boff));
    __builtin_nontemporal_store(v, reinterpret_cast<V*>(reinterpret_cast<char*>(base) + boff));
}

template <typename T>
struct V2 {
    typedef T type __attribute__((ext_vector_type(2)));
};

template <typename T, bool DIR>
struct Pre2 {
    typename V2<T>::type r[3], po[3], dv;  // own pair
    T hr[3], hpo[3], hdv;                  // one halo node
    typename V2<T>::type k;                // own element pair
    T kh;                                  // one halo element
};

// ALL: every load is active (DIR) -- removes the per-load branches.
// MG (multigrid relaxation, float32 V-cycle): the operator's result at a
// finished node feeds an epilogue instead of being stored: MG_RELAX writes
// x + w D^-1 (f - A x), MG_RESID writes f - A x.  The input is x (DIR false;
// f comes in through p_old and D^-1 through dinv, own nodes only) or
// w D^-1 f (DIR true, r = f: the Jacobi step from zero), all loads active.
// MG_RELAX with partials also sums f . x_new per load (r.z of the cycle).
// TR: element type of r (float with T = double: a float32 preconditioner's
// output read directly by the float64 direction pass).
template <typename T, int WX, int TY, bool DIR, bool ALL, int MG = MG_NONE, typename TR = T>
__device__ __forceinline__ void march2_body(int bid_, int slot_, int n, int tz, int ntx, int nty,
                                            const TR* __restrict__ r, const T* __restrict__ dinv,
                                            const T* __restrict__ p_old, T* __restrict__ p_new,
                                            const T* __restrict__ k, T* __restrict__ q, double* __restrict__ partials,
                                            const Scalars* __restrict__ sc) {
    typedef typename V2<T>::type T2;
    static_assert(WX * TY == kBlock, "block size");
    constexpr int TX = 2 * WX;                   // nodes per tile row
    constexpr int PX = TX + 2, PY = TY + 2;       // padded plane (halo 1)
    constexpr int PXP = TX + 4;                   // row pitch, even; element px lives at px + 1
    constexpr int NH = 2 * PX + 2 * (PY - 2);     // halo nodes
    constexpr int KX = TX + 1, KY = TY + 1;       // element plane, low-side halo
    constexpr int KXP = TX + 2;                   // even pitch; element kx lives at kx + 1
    constexpr int NKH = KX + KY - 1;
    static_assert(NH <= kBlock && NKH <= kBlock, "halo");
    __shared__ __attribute__((aligned(16))) T sp[2][3][PY * PXP];
    __shared__ __attribute__((aligned(16))) T sk[2][KY * KXP];

    const int tid = threadIdx.x;
    const int tx = tid % WX, ty = tid / WX;
    int bid = bid_;
    const int bx = bid % ntx;
    bid /= ntx;
    const int by = bid % nty;
    const int bz = bid / nty;
    const int i0 = bx * TX, j0 = by * TY, z0 = bz * tz;
    const int z1 = min(z0 + tz, n);
    const int64_t nn = (int64_t)n * n * n;
    const int64_t n2 = (int64_t)n * n;

    bool act[3] = {true, true, true};
    T beta[3] = {(T)0, (T)0, (T)0};
    if (DIR && MG == MG_NONE) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            act[l] = ALL ? true : (sc->active[l] != 0);
            beta[l] = (T)sc->beta[l];
        }
    }
    const int i = i0 + 2 * tx, j = j0 + ty;
    const bool own = (i < n) && (j < n);  // n even: i < n implies i + 1 < n
    const uint32_t xy_own = (uint32_t)(i % n) + (uint32_t)n * (uint32_t)(j % n);  // even
    const int lp = (ty + 1) * PXP + (2 * tx + 1) + 1;  // LDS index of node a (even)
    const int lk = (ty + 1) * KXP + (2 * tx + 1) + 1;  // LDS index of element a (even)
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

    const uint32_t bo = xy_own * (uint32_t)sizeof(T);
    const uint32_t bh = xy_h * (uint32_t)sizeof(T);
    const uint32_t bor = xy_own * (uint32_t)sizeof(TR);  // the same nodes in r
    const uint32_t bhr = xy_h * (uint32_t)sizeof(TR);
    typedef typename V2<TR>::type TR2;
    const uint32_t bkh = xy_kh * (uint32_t)sizeof(T);

    // own pair loads first, then every halo load under one branch (one exec
    // mask change per plane instead of one per field)
    auto load_plane = [&](int P, Pre2<T, DIR>& f) {
        const int64_t zoff = plane_off(P);
        const T* dp = dinv + zoff;
        const T* kp = k + zoff;
        if (DIR || MG == MG_RELAX) f.dv = ld_at<T2>(dp, bo);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            f.r[l] = __builtin_convertvector(ld_at<TR2>(r + l * nn + zoff, bor), T2);
            if (DIR && MG == MG_NONE && beta[l] != (T)0) f.po[l] = ld_at<T2>(p_old + l * nn + zoff, bo);
            if (!DIR && MG != MG_NONE) f.po[l] = ld_at<T2>(p_old + l * nn + zoff, bo);  // own f
        }
        f.k = ld_at<T2>(kp, bo);
        if (has_h) {
            if (DIR) f.hdv = ld_at<T>(dp, bh);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                if (!act[l]) continue;
                f.hr[l] = (T)ld_at<TR>(r + l * nn + zoff, bhr);
                if (DIR && beta[l] != (T)0) f.hpo[l] = ld_at<T>(p_old + l * nn + zoff, bh);
            }
        }
        if (has_kh) f.kh = ld_at<T>(kp, bkh);
    };

    T2 pP[3];
    T2 fP[3], dP;  // MG: own f and D^-1 of the stored plane
    auto store_plane = [&](int P, const Pre2<T, DIR>& f) {
        const int slot = P & 1;
        const bool in_range = P >= z0 && P < z1;
        const int64_t zoff = plane_off(P);
        T hv[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            T2 val = f.r[l];
            hv[l] = f.hr[l];
            if (DIR && MG != MG_NONE) {
                val = ((T)kMgOmega * f.dv) * f.r[l];
                hv[l] = ((T)kMgOmega * f.hdv) * f.hr[l];
            } else if (DIR) {
                val = f.dv * f.r[l];
                hv[l] = f.hdv * f.hr[l];
                if (beta[l] != (T)0) {
                    val += beta[l] * f.po[l];
                    hv[l] += beta[l] * f.hpo[l];
                }
            }
            *reinterpret_cast<T2*>(&sp[slot][l][lp]) = val;
            pP[l] = val;
            if (MG != MG_NONE) fP[l] = DIR ? f.r[l] : f.po[l];
        }
        if (MG == MG_RELAX) dP = f.dv;
        if (DIR && MG == MG_NONE && in_range && own) {
#pragma unroll
            for (int l = 0; l < 3; ++l)
                if (act[l]) st_at<T2>(p_new + l * nn + zoff, bo, pP[l]);
        }
        *reinterpret_cast<T2*>(&sk[slot][lk]) = f.k;
        if (has_h) {
#pragma unroll
            for (int l = 0; l < 3; ++l)
                if (act[l]) sp[slot][l][lph] = hv[l];
        }
        if (has_kh) sk[slot][lkh] = f.kh;
    };

    const T w = (T)(1.0 / 12.0);
    const T third = (T)(1.0 / 3.0);
    T2 yA[3], yB[3], pB[3], fB[3], dB = (T2)((T)0);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        yA[l] = (T2)((T)0);
        yB[l] = (T2)((T)0);
        pB[l] = (T2)((T)0);
        fB[l] = (T2)((T)0);
    }
    // conductivities of the previous element plane around nodes a and b:
    // kp = elements (i-1, i, i+1) at rows j-1 (m) and j (c)
    T kpm0 = 0, kpm1 = 0, kpm2 = 0, kpc0 = 0, kpc1 = 0, kpc2 = 0;
    double acc[3] = {0.0, 0.0, 0.0};

    auto compute = [&](int P) {
        const int slot = P & 1;
        const T* K = sk[slot];
        // element plane P: rows j-1 and j, columns i-1, i, i+1
        const T km0 = K[lk - KXP - 1];
        const T2 km12 = *reinterpret_cast<const T2*>(&K[lk - KXP]);
        const T kc0 = K[lk - 1];
        const T2 kc12 = *reinterpret_cast<const T2*>(&K[lk]);
        const T km1 = km12.x, km2 = km12.y, kc1 = kc12.x, kc2 = kc12.y;
        // node a uses columns (0,1), node b columns (1,2); K order (i-1,j-1),(i,j-1),(i-1,j),(i,j)
        // previous plane pair sums / in-plane sums, per node
        const T pa_xm = kpm0 + kpc0, pa_xp = kpm1 + kpc1, pa_ym = kpm0 + kpm1, pa_yp = kpc0 + kpc1;
        const T pb_xm = kpm1 + kpc1, pb_xp = kpm2 + kpc2, pb_ym = kpm1 + kpm2, pb_yp = kpc1 + kpc2;
        const T ca_xm = km0 + kc0, ca_xp = km1 + kc1, ca_ym = km0 + km1, ca_yp = kc0 + kc1;
        const T cb_xm = km1 + kc1, cb_xp = km2 + kc2, cb_ym = km1 + km2, cb_yp = kc1 + kc2;
        const T ea0 = kpm0 + km0, ea1 = kpm1 + km1, ea2 = kpc0 + kc0, ea3 = kpc1 + kc1;
        const T eb0 = kpm1 + km1, eb1 = kpm2 + km2, eb2 = kpc1 + kc1, eb3 = kpc2 + kc2;
        const T c0a = (ea0 + ea1 + ea2 + ea3) * third;
        const T c0b = (eb0 + eb1 + eb2 + eb3) * third;
        const bool done = P - 1 >= z0;
        T2 qd[3];
        const int64_t zdone = (int64_t)(P - 1 < 0 ? 0 : (P - 1)) * n2;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            const T* L = sp[slot][l];
            // rows j-1 (m), j (c), j+1 (p); columns i-1 | i, i+1 | i+2
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
            // node a: xm=c0v xc=c1 xp=c2, ym=m1 yp=p1, diagonals m0 m2 p0 p2
            const T opa = pa_xm * c0v + pa_xp * c2 + pa_ym * m1 + pa_yp * p1 + kpm0 * m0 + kpm1 * m2 + kpc0 * p0 +
                          kpc1 * p2;
            const T oca = ca_xm * c0v + ca_xp * c2 + ca_ym * m1 + ca_yp * p1 + km0 * m0 + km1 * m2 + kc0 * p0 +
                          kc1 * p2;
            const T ina = c0a * c1 - w * (ea0 * m0 + ea1 * m2 + ea2 * p0 + ea3 * p2);
            // node b: xm=c1 xc=c2 xp=c3, ym=m2 yp=p2, diagonals m1 m3 p1 p3
            const T opb = pb_xm * c1 + pb_xp * c3 + pb_ym * m2 + pb_yp * p2 + kpm1 * m1 + kpm2 * m3 + kpc1 * p1 +
                          kpc2 * p3;
            const T ocb = cb_xm * c1 + cb_xp * c3 + cb_ym * m2 + cb_yp * p2 + km1 * m1 + km2 * m3 + kc1 * p1 +
                          kc2 * p3;
            const T inb = c0b * c2 - w * (eb0 * m1 + eb1 * m3 + eb2 * p1 + eb3 * p3);
            T2 ya;
            ya.x = yA[l].x - w * opa;
            ya.y = yA[l].y - w * opb;
            qd[l] = ya;
            T2 yb;
            yb.x = yB[l].x + ina;
            yb.y = yB[l].y + inb;
            yA[l] = yb;
            yB[l].x = -w * oca;
            yB[l].y = -w * ocb;
        }
        if (MG != MG_NONE) {
            if (done && own) {
                const T2 wd = (T)kMgOmega * dB;
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    const T2 res = fB[l] - qd[l];
                    if (MG == MG_RELAX) {
                        const T2 xn = pB[l] + wd * res;
                        st_at<T2>(q + l * nn + zdone, bo, xn);
                        acc[l] += (double)fB[l].x * (double)xn.x + (double)fB[l].y * (double)xn.y;
                    } else {
                        st_at<T2>(q + l * nn + zdone, bo, res);
                    }
                }
            }
#pragma unroll
            for (int l = 0; l < 3; ++l) fB[l] = fP[l];
            dB = dP;
        } else if (done && own) {
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                if (!act[l]) continue;
                if (DIR)
                    st_at<T2>(q + l * nn + zdone, bo, qd[l]);
                else
                    st_stream<T2>(q + l * nn + zdone, bo, qd[l]);
                if (DIR) acc[l] += (double)pB[l].x * (double)qd[l].x + (double)pB[l].y * (double)qd[l].y;
            }
        }
#pragma unroll
        for (int l = 0; l < 3; ++l) pB[l] = pP[l];
        kpm0 = km0;
        kpm1 = km1;
        kpm2 = km2;
        kpc0 = kc0;
        kpc1 = kc1;
        kpc2 = kc2;
    };

    Pre2<T, DIR> fa, fb;
    load_plane(z0 - 1, fa);
    load_plane(z0, fb);
    int P = z0 - 1;
    // two planes per trip: (fa holds P, fb holds P+1) -> (fb holds P+1, fa holds P+2)
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
    if (P <= z1) {  // odd number of planes: the last one sits in fa
        store_plane(P, fa);
        __syncthreads();
        compute(P);
    }
    if (MG == MG_RELAX) {
        if (partials) block_partials_at<3>(acc, partials, slot_);
        return;
    }
    if (!DIR || MG != MG_NONE) return;
    block_partials_at<3>(acc, partials, slot_);
}

template <typename T, int WX, int TY, bool DIR, bool ALL>
__global__ void __launch_bounds__(WX* TY) k_march2(int n, int tz, int ntx, int nty, const T* __restrict__ r,
                                                   const T* __restrict__ dinv, const T* __restrict__ p_old,
                                                   T* __restrict__ p_new, const T* __restrict__ k,
                                                   T* __restrict__ q, double* __restrict__ partials,
                                                   const Scalars* __restrict__ sc) {
    march2_body<T, WX, TY, DIR, ALL>(xcd_tile(blockIdx.x, gridDim.x), blockIdx.x, n, tz, ntx, nty, r, dinv, p_old,
                                     p_new, k, q, partials, sc);
}

// Direction + operator pass of float64 CG whose preconditioned residual z is
// float32 (the multigrid cycle's output): p = z + beta p, q = A p, p.q.
template <int WX, int TY, bool ALL>
__global__ void __launch_bounds__(WX* TY) k_march2_zf(int n, int tz, int ntx, int nty, const float* __restrict__ z,
                                                      const double* __restrict__ dinv,
                                                      const double* __restrict__ p_old, double* __restrict__ p_new,
                                                      const double* __restrict__ k, double* __restrict__ q,
                                                      double* __restrict__ partials, const Scalars* __restrict__ sc) {
    march2_body<double, WX, TY, true, ALL, MG_NONE, float>(xcd_tile(blockIdx.x, gridDim.x), blockIdx.x, n, tz, ntx,
                                                           nty, z, dinv, p_old, p_new, k, q, partials, sc);
}

// Stand-alone float32 operator (no direction, no dots): its register state
// fits three waves per SIMD (float64 would spill there and keeps k_march2).
template <int WX, int TY>
__global__ void __launch_bounds__(WX* TY) __attribute__((amdgpu_waves_per_eu(3)))
    k_apply2_f32(int n, int tz, int ntx, int nty, const float* __restrict__ x, const float* __restrict__ k,
                 float* __restrict__ y) {
    march2_body<float, WX, TY, false, true>(xcd_tile(blockIdx.x, gridDim.x), blockIdx.x, n, tz, ntx, nty, x, nullptr,
                                            nullptr, nullptr, k, y, nullptr, nullptr);
}

// Multigrid relaxation / residual pass (float32), see march2_body.
template <int WX, int TY, bool FROM_F, int MG>
__global__ void __launch_bounds__(WX* TY) __attribute__((amdgpu_waves_per_eu(2)))
    k_mg_march(int n, int tz, int ntx, int nty, const float* __restrict__ in, const float* __restrict__ dinv,
               const float* __restrict__ f, const float* __restrict__ k, float* __restrict__ out,
               double* __restrict__ partials) {
    march2_body<float, WX, TY, FROM_F, true, MG>(xcd_tile(blockIdx.x, gridDim.x), blockIdx.x, n, tz, ntx, nty,
                                                 FROM_F ? f : in, dinv, f, nullptr, k, out, partials, nullptr);
}

template <int WX, int TY>
static void launch_mg_march_t(int n, const TileShape& t, bool from_f, int mode, const float* in, const float* dinv,
                              const float* f, const float* k, float* out, double* partials, hipStream_t s) {
    const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
    const dim3 g(t.blocks), b(kBlock);
    if (from_f && mode == MG_RELAX)
        hipLaunchKernelGGL((k_mg_march<WX, TY, true, MG_RELAX>), g, b, 0, s, n, t.tz, ntx, nty, in, dinv, f, k, out,
                           partials);
    else if (from_f)
        hipLaunchKernelGGL((k_mg_march<WX, TY, true, MG_RESID>), g, b, 0, s, n, t.tz, ntx, nty, in, dinv, f, k, out,
                           partials);
    else if (mode == MG_RELAX)
        hipLaunchKernelGGL((k_mg_march<WX, TY, false, MG_RELAX>), g, b, 0, s, n, t.tz, ntx, nty, in, dinv, f, k, out,
                           partials);
    else
        hipLaunchKernelGGL((k_mg_march<WX, TY, false, MG_RESID>), g, b, 0, s, n, t.tz, ntx, nty, in, dinv, f, k, out,
                           partials);
}

void launch_mg_march(int n, const TileShape& t, bool from_f, int mode, const float* in, const float* dinv,
                     const float* f, const float* k, float* out, double* partials, hipStream_t s) {
    if (t.tx == 32)
        launch_mg_march_t<16, 16>(n, t, from_f, mode, in, dinv, f, k, out, partials, s);
    else
        launch_mg_march_t<32, 8>(n, t, from_f, mode, in, dinv, f, k, out, partials, s);
}

// ev0/ev1 (optional): HIP events recorded at the kernel's start and end.
template <typename T, bool DIR, bool ALL>
static void launch_m2(int n, const TileShape& t, const T* r, const T* dinv, const T* p_old, T* p_new, const T* k,
                      T* q, double* partials, const Scalars* sc, hipStream_t s, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr) {
    const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
    if (t.tx == 32)
        hipExtLaunchKernelGGL((k_march2<T, 16, 16, DIR, ALL>), dim3(t.blocks), dim3(kBlock), 0, s, ev0, ev1, 0, n,
                              t.tz, ntx, nty, r, dinv, p_old, p_new, k, q, partials, sc);
    else
        hipExtLaunchKernelGGL((k_march2<T, 32, 8, DIR, ALL>), dim3(t.blocks), dim3(kBlock), 0, s, ev0, ev1, 0, n,
                              t.tz, ntx, nty, r, dinv, p_old, p_new, k, q, partials, sc);
}

// Tile shapes of the pair kernel: tx in {32, 64} nodes (16 or 32 threads wide).
TileShape choose_tile2(int n, int max_blocks, int tz_override, int tx_override) {
    TileShape t;
    if (tx_override == 32 || tx_override == 64)
        t.tx = tx_override;
    else
        t.tx = n <= 40 ? 32 : 64;
    t.ty = kBlock / (t.tx / 2);
    const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
    int tz = tz_override;
    if (tz <= 0) {
        const int64_t cols = (int64_t)ntx * nty;
        tz = (int)((cols * n + 1023) / 1024);
        if (tz < 2) tz = 2;
    }
    if (tz > n) tz = n;
    while ((int64_t)ntx * nty * ((n + tz - 1) / tz) > max_blocks && tz < n) ++tz;
    t.tz = tz;
    t.blocks = ntx * nty * ((n + tz - 1) / tz);
    return t;
}

template <typename T>
void launch_dir_march2(int n, const TileShape& t, bool all_active, const T* r, const T* dinv, const T* p_old,
                       T* p_new, const T* k, T* q, const Workspace& ws, hipStream_t s, bool fin, hipEvent_t ev0,
                       hipEvent_t ev1) {
    if (all_active)
        launch_m2<T, true, true>(n, t, r, dinv, p_old, p_new, k, q, ws.partials, ws.sc, s, ev0, ev1);
    else
        launch_m2<T, true, false>(n, t, r, dinv, p_old, p_new, k, q, ws.partials, ws.sc, s, ev0, ev1);
    if (fin) launch_finalize(FIN_PQ, t.blocks, ws, s);
}

void launch_dir_march2_zf(int n, const TileShape& t, bool all_active, const float* z, const double* dinv,
                          const double* p_old, double* p_new, const double* k, double* q, const Workspace& ws,
                          hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
    const dim3 g(t.blocks), b(kBlock);
    if (t.tx == 32) {
        if (all_active)
            hipExtLaunchKernelGGL((k_march2_zf<16, 16, true>), g, b, 0, s, ev0, ev1, 0, n, t.tz, ntx, nty, z, dinv,
                                  p_old, p_new, k, q, ws.partials, ws.sc);
        else
            hipExtLaunchKernelGGL((k_march2_zf<16, 16, false>), g, b, 0, s, ev0, ev1, 0, n, t.tz, ntx, nty, z, dinv,
                                  p_old, p_new, k, q, ws.partials, ws.sc);
    } else {
        if (all_active)
            hipExtLaunchKernelGGL((k_march2_zf<32, 8, true>), g, b, 0, s, ev0, ev1, 0, n, t.tz, ntx, nty, z, dinv,
                                  p_old, p_new, k, q, ws.partials, ws.sc);
        else
            hipExtLaunchKernelGGL((k_march2_zf<32, 8, false>), g, b, 0, s, ev0, ev1, 0, n, t.tz, ntx, nty, z, dinv,
                                  p_old, p_new, k, q, ws.partials, ws.sc);
    }
    launch_finalize(FIN_PQ, t.blocks, ws, s);
}

template <typename T>
void launch_apply_march2(int n, const TileShape& t, const T* k, const T* x, T* y, hipStream_t s) {
    if constexpr (std::is_same<T, float>::value) {
        const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
        if (t.tx == 32)
            hipLaunchKernelGGL((k_apply2_f32<16, 16>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, x, k, y);
        else
            hipLaunchKernelGGL((k_apply2_f32<32, 8>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, x, k, y);
    } else {
        launch_m2<T, false, true>(n, t, x, nullptr, nullptr, nullptr, k, y, nullptr, nullptr, s);
    }
}

template void launch_dir_march2<double>(int, const TileShape&, bool, const double*, const double*, const double*,
                                        double*, const double*, double*, const Workspace&, hipStream_t, bool,
                                        hipEvent_t, hipEvent_t);
template void launch_dir_march2<float>(int, const TileShape&, bool, const float*, const float*, const float*, float*,
                                       const float*, float*, const Workspace&, hipStream_t, bool, hipEvent_t,
                                       hipEvent_t);
template void launch_apply_march2<double>(int, const TileShape&, const double*, const double*, double*, hipStream_t);
template void launch_apply_march2<float>(int, const TileShape&, const float*, const float*, float*, hipStream_t);

}  // namespace otm

namespace otm {

// Batched direction + operator pass: persistent blocks walk the work list of
// (design, tile) items; an item of an inactive or converged design still runs
// (its loads' activity flags are read per design), which keeps the per-item
// partial slots of every design filled for its finalize.
template <int WX, int TY>
__global__ void __launch_bounds__(WX* TY) kb_dir_march2(BatchTab t, const double* __restrict__ r,
                                                        const double* __restrict__ dinv,
                                                        const double* __restrict__ p_old, double* __restrict__ p_new,
                                                        const double* __restrict__ k, double* __restrict__ q,
                                                        double* __restrict__ partials, const Scalars* __restrict__ sc) {
    for (int v = blockIdx.x; v < t.mb_total; v += gridDim.x) {
        // contiguous item ranges per XCD (the grid is a multiple of 8 or covers every item)
        const int item = xcd_tile(v, t.mb_total);
        const int d = t.mb_design[item];
        const BatchDesc D = t.desc[d];
        const int64_t o1 = D.off, o3 = 3 * D.off;
        __syncthreads();
        march2_body<double, WX, TY, true, false>(item - D.mb_start, item, D.n, D.tz, D.ntx, D.nty, r + o3, dinv + o1,
                                                 p_old + o3, p_new + o3, k + o1, q + o3, partials, sc + d);
    }
}

template <int WX, int TY>
void launch_b_dir_march2(const BatchTab& t, int grid, const double* r, const double* dinv, const double* p_old,
                         double* p_new, const double* k, double* q, double* partials, const Scalars* sc, bool fin,
                         hipStream_t s) {
    hipLaunchKernelGGL((kb_dir_march2<WX, TY>), dim3(grid), dim3(kBlock), 0, s, t, r, dinv, p_old, p_new, k, q,
                       partials, sc);
    if (fin) launch_b_finalize(t, FIN_PQ, 1, partials, const_cast<Scalars*>(sc), 0.5, s);
}

template void launch_b_dir_march2<32, 8>(const BatchTab&, int, const double*, const double*, const double*, double*,
                                         const double*, double*, double*, const Scalars*, bool, hipStream_t);
template void launch_b_dir_march2<16, 16>(const BatchTab&, int, const double*, const double*, const double*, double*,
                                          const double*, double*, double*, const Scalars*, bool, hipStream_t);

}  // namespace otm
