// Tiled solver kernels for the PCG iteration (gfx950).
//
// k_tiled (DIR = true): one pass that forms the new search direction
//   p_new = D^-1 r + beta p_old
// and applies the operator q = A p_new for the three loads, with the dot
// products p.q reduced in float64 and alpha = rz / pq set by the last block.
//
// Layout of the pass: a block owns a TX x TY column of nodes and marches in z
// over tz planes.  p_new of the planes z-1, z, z+1 (with a one-node halo in x
// and y) lives in a 3-slot LDS ring; k of the element planes z-1 and z in a
// 2-slot ring.  Each node of plane z then reads its 20 non-zero neighbours
// and 8 incident conductivities from LDS, so every HBM value is fetched by
// one block (halo values are re-read from L2 by the neighbouring block).
//
// k_update_vec: x += alpha p, r -= alpha q and the dots r.D^-1 r, r.r, with
// 16-byte vector accesses (float4 / double2).
#include <type_traits>

#include "otm_device.h"

namespace otm {

// y at one node from the three LDS planes (pm: z-1, p0: z, pp: z+1); pc is the
// node's position in the padded plane, PX its row pitch.
template <typename T>
__device__ __forceinline__ T stencil_lds(const NodeCoef<T>& c, const T* pm, const T* p0, const T* pp, int pc,
                                         int PX) {
    T y = c.c0 * p0[pc];
    // edge-diagonal neighbours in the xy plane: (2a-1, 2b-1, 0)
    y += c.ce[0] * p0[pc - PX - 1];
    y += c.ce[1] * p0[pc - PX + 1];
    y += c.ce[2] * p0[pc + PX - 1];
    y += c.ce[3] * p0[pc + PX + 1];
    // xz plane: (2a-1, 0, 2c-1)
    y += c.ce[4] * pm[pc - 1];
    y += c.ce[5] * pm[pc + 1];
    y += c.ce[6] * pp[pc - 1];
    y += c.ce[7] * pp[pc + 1];
    // yz plane: (0, 2b-1, 2c-1)
    y += c.ce[8] * pm[pc - PX];
    y += c.ce[9] * pm[pc + PX];
    y += c.ce[10] * pp[pc - PX];
    y += c.ce[11] * pp[pc + PX];
    // corners (2a-1, 2b-1, 2c-1), index a + 2b + 4c
    y += c.cc[0] * pm[pc - PX - 1];
    y += c.cc[1] * pm[pc - PX + 1];
    y += c.cc[2] * pm[pc + PX - 1];
    y += c.cc[3] * pm[pc + PX + 1];
    y += c.cc[4] * pp[pc - PX - 1];
    y += c.cc[5] * pp[pc - PX + 1];
    y += c.cc[6] * pp[pc + PX - 1];
    y += c.cc[7] * pp[pc + PX + 1];
    return y;
}

// DIR = true : p_new = D^-1 r + beta p_old, q = A p_new, dots p.q (PCG pass)
// DIR = false: q = A r (plain operator; dinv, p_old, p_new, the scalars and the
//              reduction workspace are unused and may be null)
template <typename T, int TX, int TY, bool DIR>
__global__ void __launch_bounds__(TX* TY) k_tiled(int n, int tz, int ntx, int nty, const T* __restrict__ r,
                                                      const T* __restrict__ dinv, const T* __restrict__ p_old,
                                                      T* __restrict__ p_new, const T* __restrict__ k,
                                                      T* __restrict__ q, double* partials, unsigned* counter,
                                                      Scalars* sc) {
    static_assert(TX * TY == kBlock, "block size");
    constexpr int PX = TX + 2, PY = TY + 2, PA = PX * PY;
    constexpr int KX = TX + 1, KY = TY + 1, KA = KX * KY;
    __shared__ T sp[3][3][PA];
    __shared__ T sk[2][KA];

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    int bid = xcd_tile(blockIdx.x, gridDim.x);  // tiles in x, then y, then z
    const int bx = bid % ntx;
    bid /= ntx;
    const int by = bid % nty;
    const int bz = bid / nty;
    const int i0 = bx * TX, j0 = by * TY, z0 = bz * tz;
    const int z1 = min(z0 + tz, n);
    const int64_t nn = (int64_t)n * n * n;
    const int64_t n2 = (int64_t)n * n;
    int act[3] = {1, 1, 1};
    T beta[3] = {(T)0, (T)0, (T)0};
    if (DIR) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            act[l] = sc->active[l];
            beta[l] = (T)sc->beta[l];
        }
    }
    const int i = i0 + tx, j = j0 + ty;
    const bool own = (i < n) && (j < n);
    double acc[3] = {0.0, 0.0, 0.0};

    // p_new of plane zz (zz in [z0-1, z1]) into its ring slot; owned nodes of
    // planes [z0, z1) are also written to global memory (exactly once overall).
    auto fill_p = [&](int zz) {
        const int slot = (zz - z0 + 1) % 3;
        const int64_t zoff = (int64_t)((zz + n) % n) * n2;
        const bool plane_owned = (zz >= z0) && (zz < z1);
        for (int t = tid; t < PA; t += kBlock) {
            const int px = t % PX, py = t / PX;
            const int gi0 = i0 - 1 + px, gj0 = j0 - 1 + py;
            const bool interior = plane_owned && px >= 1 && px <= TX && py >= 1 && py <= TY && gi0 < n && gj0 < n;
            const int gi = (gi0 + n) % n, gj = (gj0 + n) % n;
            const int64_t v = gi + (int64_t)n * gj + zoff;
            if (DIR) {
                const T dv = dinv[v];
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    if (!act[l]) continue;
                    const T z = dv * r[l * nn + v];
                    const T pn = (beta[l] == (T)0) ? z : z + beta[l] * p_old[l * nn + v];
                    sp[slot][l][t] = pn;
                    if (interior) p_new[l * nn + v] = pn;
                }
            } else {
                (void)interior;
#pragma unroll
                for (int l = 0; l < 3; ++l) sp[slot][l][t] = r[l * nn + v];
            }
        }
    };
    auto fill_k = [&](int ze) {
        const int slot = (ze - z0 + 1) & 1;
        const int64_t zoff = (int64_t)((ze + n) % n) * n2;
        for (int t = tid; t < KA; t += kBlock) {
            const int kx = t % KX, ky = t / KX;
            const int gi = (i0 - 1 + kx + n) % n, gj = (j0 - 1 + ky + n) % n;
            sk[slot][t] = k[gi + (int64_t)n * gj + zoff];
        }
    };

    fill_p(z0 - 1);
    fill_p(z0);
    fill_k(z0 - 1);
    for (int z = z0; z < z1; ++z) {
        fill_p(z + 1);
        fill_k(z);
        __syncthreads();
        if (own) {
            const int sm = (z - z0) % 3, s0 = (z - z0 + 1) % 3, s1 = (z - z0 + 2) % 3;
            const int km = (z - z0) & 1, k0 = (z - z0 + 1) & 1;
            T ko[8];
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int a = o & 1, b = (o >> 1) & 1, c = o >> 2;
                ko[o] = sk[c ? k0 : km][(ty + b) * KX + tx + a];
            }
            NodeCoef<T> cf;
            node_coefs(ko, cf);
            const int pc = (ty + 1) * PX + (tx + 1);
            const int64_t v = i + (int64_t)n * j + (int64_t)z * n2;
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                if (!act[l]) continue;
                const T y = stencil_lds<T>(cf, sp[sm][l], sp[s0][l], sp[s1][l], pc, PX);
                q[l * nn + v] = y;
                if (DIR) acc[l] += (double)sp[s0][l][pc] * (double)y;
            }
        }
        __syncthreads();
    }
    if (!DIR) return;
    block_partials<3>(acc, partials);
}


// ---------------------------------------------------------------- k_march
// Streaming z-march.  The contribution of node plane P to the operator at a
// node (i,j,z) depends only on the element planes between z and P, so each
// thread keeps three running sums: node P-1 (receives its last, dz=+1 taps
// and is finished), node P (dz=0 taps) and node P+1 (first, dz=-1 taps).
// With K = the 4 conductivities of an element plane around (i,j) in the order
// (i-1,j-1), (i,j-1), (i-1,j), (i,j), the off-plane taps of a neighbour plane
// are -(1/12) O(K, nb) with
//   O(K, nb) = (K0+K2) nb(-1,0) + (K1+K3) nb(1,0) + (K0+K1) nb(0,-1) + (K2+K3) nb(0,1)
//            + K0 nb(-1,-1) + K1 nb(1,-1) + K2 nb(-1,1) + K3 nb(1,1)
// and the in-plane taps are (1/3) sum(Kprev+Kcur) nb(0,0) - (1/12) sum_q (Kprev+Kcur)_q nb(diag q).
// One plane of values (with a one-node halo) and one element plane (with a
// low-side halo) sit in a 2-slot LDS ring; global loads run two planes ahead
// in registers.
template <typename T, bool DIR>
struct PlaneRegs {
    T r[3];   // DIR: residual; else the operand x
    T po[3];  // DIR: previous direction
    T dv;     // DIR: D^-1
    T hr[3];
    T hpo[3];
    T hdv;
    T k_own, k_h;
};

template <typename T, int TX, int TY, bool DIR>
__global__ void __launch_bounds__(TX* TY) k_march(int n, int tz, int ntx, int nty, const T* __restrict__ r,
                                                  const T* __restrict__ dinv, const T* __restrict__ p_old,
                                                  T* __restrict__ p_new, const T* __restrict__ k, T* __restrict__ q,
                                                  double* __restrict__ partials, const Scalars* __restrict__ sc) {
    static_assert(TX * TY == kBlock, "block size");
    constexpr int PX = TX + 2, PY = TY + 2, PA = PX * PY, NH = 2 * PX + 2 * (PY - 2);
    constexpr int KX = TX + 1, KY = TY + 1, KA = KX * KY, NKH = KX + KY - 1;
    static_assert(NH <= kBlock && NKH <= kBlock, "halo");
    __shared__ T sp[2][3][PA];
    __shared__ T sk[2][KA];

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    int bid = xcd_tile(blockIdx.x, gridDim.x);  // tiles in x, then y, then z
    const int bx = bid % ntx;
    bid /= ntx;
    const int by = bid % nty;
    const int bz = bid / nty;
    const int i0 = bx * TX, j0 = by * TY, z0 = bz * tz;
    const int z1 = min(z0 + tz, n);
    const int64_t nn = (int64_t)n * n * n;
    const int64_t n2 = (int64_t)n * n;

    int act[3] = {1, 1, 1};
    T beta[3] = {(T)0, (T)0, (T)0};
    if (DIR) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            act[l] = sc->active[l];
            beta[l] = (T)sc->beta[l];
        }
    }
    // own column (wrapped so that masked columns of partial tiles load valid data)
    const int i = i0 + tx, j = j0 + ty;
    const bool own = (i < n) && (j < n);
    const int64_t xy_own = (int64_t)(i % n) + (int64_t)n * (j % n);
    const int lp = (ty + 1) * PX + (tx + 1);
    const int lk = (ty + 1) * KX + (tx + 1);
    // this thread's halo node (ring around the tile) and halo element (low side)
    const bool has_h = tid < NH;
    int64_t xy_h = 0;
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
        xy_h = gi + (int64_t)n * gj;
        lph = py * PX + px;
    }
    const bool has_kh = tid < NKH;
    int64_t xy_kh = 0;
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
        xy_kh = gi + (int64_t)n * gj;
        lkh = ky * KX + kx;
    }

    auto load_plane = [&](int P, PlaneRegs<T, DIR>& f) {
        const int pw = P < 0 ? P + n : (P >= n ? P - n : P);
        const int64_t zoff = (int64_t)pw * n2;
        const int64_t vo = xy_own + zoff;
        if (DIR) f.dv = dinv[vo];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            f.r[l] = r[l * nn + vo];
            if (DIR && beta[l] != (T)0) f.po[l] = p_old[l * nn + vo];
        }
        if (has_h) {
            const int64_t vh = xy_h + zoff;
            if (DIR) f.hdv = dinv[vh];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                if (!act[l]) continue;
                f.hr[l] = r[l * nn + vh];
                if (DIR && beta[l] != (T)0) f.hpo[l] = p_old[l * nn + vh];
            }
        }
        f.k_own = k[xy_own + zoff];
        if (has_kh) f.k_h = k[xy_kh + zoff];
    };

    T pP[3] = {(T)0, (T)0, (T)0};
    auto store_plane = [&](int P, const PlaneRegs<T, DIR>& f) {
        const int slot = P & 1;
        const bool write_p = DIR && own && P >= z0 && P < z1;
        const int pw = P < 0 ? P + n : (P >= n ? P - n : P);
        const int64_t vo = xy_own + (int64_t)pw * n2;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            T val = f.r[l];
            if (DIR) {
                val = f.dv * f.r[l];
                if (beta[l] != (T)0) val += beta[l] * f.po[l];
            }
            sp[slot][l][lp] = val;
            pP[l] = val;
            if (write_p) p_new[l * nn + vo] = val;
            if (has_h) {
                T hv = f.hr[l];
                if (DIR) {
                    hv = f.hdv * f.hr[l];
                    if (beta[l] != (T)0) hv += beta[l] * f.hpo[l];
                }
                sp[slot][l][lph] = hv;
            }
        }
        sk[slot][lk] = f.k_own;
        if (has_kh) sk[slot][lkh] = f.k_h;
    };

    const T w = (T)(1.0 / 12.0);
    const T third = (T)(1.0 / 3.0);
    T yA[3] = {(T)0, (T)0, (T)0}, yB[3] = {(T)0, (T)0, (T)0};
    T pB[3] = {(T)0, (T)0, (T)0};
    T kp[4] = {(T)0, (T)0, (T)0, (T)0};
    double acc[3] = {0.0, 0.0, 0.0};

    PlaneRegs<T, DIR> fa, fb;
    load_plane(z0 - 1, fa);
    load_plane(z0, fb);
    for (int P = z0 - 1; P <= z1; ++P) {
        store_plane(P, fa);
        fa = fb;
        if (P + 2 <= z1) load_plane(P + 2, fb);
        __syncthreads();
        const int slot = P & 1;
        const T* K = sk[slot];
        T kc[4];
        kc[0] = K[lk - KX - 1];
        kc[1] = K[lk - KX];
        kc[2] = K[lk - 1];
        kc[3] = K[lk];
        const T pxm = kp[0] + kp[2], pxp = kp[1] + kp[3], pym = kp[0] + kp[1], pyp = kp[2] + kp[3];
        const T cxm = kc[0] + kc[2], cxp = kc[1] + kc[3], cym = kc[0] + kc[1], cyp = kc[2] + kc[3];
        const T e0 = kp[0] + kc[0], e1 = kp[1] + kc[1], e2 = kp[2] + kc[2], e3 = kp[3] + kc[3];
        const T c0 = (e0 + e1 + e2 + e3) * third;
        const bool done_node = own && (P - 1 >= z0);
        const int64_t vdone = xy_own + (int64_t)(P - 1 < 0 ? 0 : P - 1) * n2;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            const T* L = sp[slot][l];
            const T xc = L[lp];
            const T xm = L[lp - 1], xp = L[lp + 1], ym = L[lp - PX], yp = L[lp + PX];
            const T d00 = L[lp - PX - 1], d10 = L[lp - PX + 1], d01 = L[lp + PX - 1], d11 = L[lp + PX + 1];
            const T op = pxm * xm + pxp * xp + pym * ym + pyp * yp + kp[0] * d00 + kp[1] * d10 + kp[2] * d01 +
                         kp[3] * d11;
            const T oc = cxm * xm + cxp * xp + cym * ym + cyp * yp + kc[0] * d00 + kc[1] * d10 + kc[2] * d01 +
                         kc[3] * d11;
            const T ya = yA[l] - w * op;
            const T yb = yB[l] + c0 * xc - w * (e0 * d00 + e1 * d10 + e2 * d01 + e3 * d11);
            const T yc = -w * oc;
            if (done_node) {
                q[l * nn + vdone] = ya;
                if (DIR) acc[l] += (double)pB[l] * (double)ya;
            }
            yA[l] = yb;
            yB[l] = yc;
            pB[l] = pP[l];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) kp[t] = kc[t];
    }
    if (!DIR) return;
    block_partials<3>(acc, partials);
}

// r32 (optional): a float32 copy of the updated r of the active loads, the
// input of a float32 preconditioner.
template <typename T, int V>
__device__ __forceinline__ void update_vec_body(int bid_, int nblk_, int slot_, int64_t nn, T* __restrict__ x,
                                                T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
                                                const T* __restrict__ dinv, double* partials, const Scalars* sc,
                                                float* __restrict__ r32 = nullptr) {
    typedef T VT __attribute__((ext_vector_type(V)));
    typedef float VF __attribute__((ext_vector_type(V)));
    const int64_t nv = nn / V;
    const int act[3] = {sc->active[0], sc->active[1], sc->active[2]};
    const T alpha[3] = {(T)sc->alpha[0], (T)sc->alpha[1], (T)sc->alpha[2]};
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const VT* dv4 = reinterpret_cast<const VT*>(dinv);
    for (int64_t t = (int64_t)bid_ * kBlock + threadIdx.x; t < nv; t += (int64_t)nblk_ * kBlock) {
        const VT dv = dv4[t];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            VT* xv = reinterpret_cast<VT*>(x + l * nn);
            VT* rv = reinterpret_cast<VT*>(r + l * nn);
            const VT pv = reinterpret_cast<const VT*>(p + l * nn)[t];
            const VT qv = reinterpret_cast<const VT*>(q + l * nn)[t];
            VT xx = xv[t];
            VT rr = rv[t];
            xx += alpha[l] * pv;
            rr -= alpha[l] * qv;
            xv[t] = xx;
            rv[t] = rr;
            if (r32) {
                VF f;
#pragma unroll
                for (int c = 0; c < V; ++c) f[c] = (float)rr[c];
                reinterpret_cast<VF*>(r32 + l * nn)[t] = f;
            }
#pragma unroll
            for (int c = 0; c < V; ++c) {
                const double rd = (double)rr[c];
                acc[l] += (double)dv[c] * rd * rd;
                acc[3 + l] += rd * rd;
            }
        }
    }
    block_partials_at<6>(acc, partials, slot_);
}

template <typename T, int V>
__global__ void __launch_bounds__(kBlock) k_update_vec(int64_t nn, T* __restrict__ x, T* __restrict__ r,
                                                       const T* __restrict__ p, const T* __restrict__ q,
                                                       const T* __restrict__ dinv, double* partials,
                                                       unsigned* counter, Scalars* sc, float* __restrict__ r32) {
    update_vec_body<T, V>(blockIdx.x, gridDim.x, blockIdx.x, nn, x, r, p, q, dinv, partials, sc, r32);
}

// ---------------------------------------------------------------- launchers

static inline int64_t cube(int n) { return (int64_t)n * n * n; }

TileShape choose_tile(int n, int max_blocks, int tz_override, int tx_override) {
    TileShape t;
    if (tx_override == 16 || tx_override == 32 || tx_override == 64) {
        t.tx = tx_override;
        t.ty = kBlock / tx_override;
    } else if (n <= 24) {
        t.tx = 16;
        t.ty = 16;
    } else {
        t.tx = 32;
        t.ty = 8;
    }
    const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
    int tz = tz_override;
    if (tz <= 0) {
        // aim at ~1024 blocks (4 per CU) with at least 2 planes per march
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
void launch_dir_apply(int n, const TileShape& t, const T* r, const T* dinv, const T* p_old, T* p_new, const T* k,
                      T* q, const Workspace& ws, hipStream_t s) {
    const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
    if (t.tx == 16)
        hipLaunchKernelGGL((k_tiled<T, 16, 16, true>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, r,
                           dinv, p_old, p_new, k, q, ws.partials, ws.counter, ws.sc);
    else if (t.tx == 64)
        hipLaunchKernelGGL((k_tiled<T, 64, 4, true>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, r,
                           dinv, p_old, p_new, k, q, ws.partials, ws.counter, ws.sc);
    else
        hipLaunchKernelGGL((k_tiled<T, 32, 8, true>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, r,
                           dinv, p_old, p_new, k, q, ws.partials, ws.counter, ws.sc);
    launch_finalize(FIN_PQ, t.blocks, ws, s);
}

template <typename T>
void launch_dir_march(int n, const TileShape& t, const T* r, const T* dinv, const T* p_old, T* p_new, const T* k,
                      T* q, const Workspace& ws, hipStream_t s) {
    const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
    if (t.tx == 16)
        hipLaunchKernelGGL((k_march<T, 16, 16, true>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, r, dinv,
                           p_old, p_new, k, q, ws.partials, ws.sc);
    else if (t.tx == 64)
        hipLaunchKernelGGL((k_march<T, 64, 4, true>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, r, dinv,
                           p_old, p_new, k, q, ws.partials, ws.sc);
    else
        hipLaunchKernelGGL((k_march<T, 32, 8, true>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, r, dinv,
                           p_old, p_new, k, q, ws.partials, ws.sc);
    launch_finalize(FIN_PQ, t.blocks, ws, s);
}

template <typename T>
void launch_apply_march(int n, const TileShape& t, const T* k, const T* x, T* y, hipStream_t s) {
    const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
    const T* nul = nullptr;
    if (t.tx == 16)
        hipLaunchKernelGGL((k_march<T, 16, 16, false>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, x, nul,
                           nul, (T*)nullptr, k, y, (double*)nullptr, (const Scalars*)nullptr);
    else if (t.tx == 64)
        hipLaunchKernelGGL((k_march<T, 64, 4, false>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, x, nul,
                           nul, (T*)nullptr, k, y, (double*)nullptr, (const Scalars*)nullptr);
    else
        hipLaunchKernelGGL((k_march<T, 32, 8, false>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, x, nul,
                           nul, (T*)nullptr, k, y, (double*)nullptr, (const Scalars*)nullptr);
}

template <typename T>
void launch_apply_tiled(int n, const TileShape& t, const T* k, const T* x, T* y, hipStream_t s) {
    const int ntx = (n + t.tx - 1) / t.tx, nty = (n + t.ty - 1) / t.ty;
    if (t.tx == 16)
        hipLaunchKernelGGL((k_tiled<T, 16, 16, false>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, x,
                           (const T*)nullptr, (const T*)nullptr, (T*)nullptr, k, y, (double*)nullptr,
                           (unsigned*)nullptr, (Scalars*)nullptr);
    else if (t.tx == 64)
        hipLaunchKernelGGL((k_tiled<T, 64, 4, false>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, x,
                           (const T*)nullptr, (const T*)nullptr, (T*)nullptr, k, y, (double*)nullptr,
                           (unsigned*)nullptr, (Scalars*)nullptr);
    else
        hipLaunchKernelGGL((k_tiled<T, 32, 8, false>), dim3(t.blocks), dim3(kBlock), 0, s, n, t.tz, ntx, nty, x,
                           (const T*)nullptr, (const T*)nullptr, (T*)nullptr, k, y, (double*)nullptr,
                           (unsigned*)nullptr, (Scalars*)nullptr);
}

template <typename T>
void launch_update_vec(int n, T* x, T* r, const T* p, const T* q, const T* dinv, const Workspace& ws, hipStream_t s,
                       bool fin, int fin_op, float* r32) {
    constexpr int V = 16 / sizeof(T);
    const int64_t nn = cube(n);
    if (nn % V != 0) {
        launch_update<T>(n, x, r, p, q, dinv, ws, s);
        if constexpr (std::is_same<T, double>::value) {
            if (r32) launch_cast_f64_f32(3 * nn, r, r32, s);
        }
        return;
    }
    const int g = grid_for(nn / V, ws.max_blocks);
    hipLaunchKernelGGL((k_update_vec<T, V>), dim3(g), dim3(kBlock), 0, s, nn, x, r, p, q, dinv, ws.partials,
                       ws.counter, ws.sc, r32);
    if (fin) launch_finalize(fin_op, g, ws, s);
}

template void launch_dir_apply<double>(int, const TileShape&, const double*, const double*, const double*, double*,
                                       const double*, double*, const Workspace&, hipStream_t);
template void launch_dir_apply<float>(int, const TileShape&, const float*, const float*, const float*, float*,
                                      const float*, float*, const Workspace&, hipStream_t);
template void launch_dir_march<double>(int, const TileShape&, const double*, const double*, const double*, double*,
                                       const double*, double*, const Workspace&, hipStream_t);
template void launch_dir_march<float>(int, const TileShape&, const float*, const float*, const float*, float*,
                                      const float*, float*, const Workspace&, hipStream_t);
template void launch_apply_march<double>(int, const TileShape&, const double*, const double*, double*, hipStream_t);
template void launch_apply_march<float>(int, const TileShape&, const float*, const float*, float*, hipStream_t);
template void launch_apply_tiled<double>(int, const TileShape&, const double*, const double*, double*, hipStream_t);
template void launch_apply_tiled<float>(int, const TileShape&, const float*, const float*, float*, hipStream_t);
template void launch_update_vec<double>(int, double*, double*, const double*, const double*, const double*,
                                        const Workspace&, hipStream_t, bool, int, float*);
template void launch_update_vec<float>(int, float*, float*, const float*, const float*, const float*,
                                       const Workspace&, hipStream_t, bool, int, float*);

}  // namespace otm

namespace otm {

// Batched x/r update over the element-sweep work list (persistent blocks).
__global__ void __launch_bounds__(kBlock) kb_update_vec(BatchTab t, double* __restrict__ x, double* __restrict__ r,
                                                        const double* __restrict__ p, const double* __restrict__ q,
                                                        const double* __restrict__ dinv, double* partials,
                                                        const Scalars* sc) {
    for (int item = blockIdx.x; item < t.eb_total; item += gridDim.x) {
        const int d = t.eb_design[item];
        const BatchDesc D = t.desc[d];
        const int64_t o1 = D.off, o3 = 3 * D.off;
        const int64_t nn = (int64_t)D.n * D.n * D.n;
        __syncthreads();
        update_vec_body<double, 2>(item - D.eb_start, D.eb_count, item, nn, x + o3, r + o3, p + o3, q + o3, dinv + o1,
                                   partials, sc + d);
    }
}

void launch_b_update_vec(const BatchTab& t, int grid, double* x, double* r, const double* p, const double* q,
                         const double* dinv, double* partials, const Scalars* sc, bool fin, hipStream_t s) {
    hipLaunchKernelGGL(kb_update_vec, dim3(grid), dim3(kBlock), 0, s, t, x, r, p, q, dinv, partials, sc);
    if (fin) launch_b_finalize(t, FIN_UPDATE, 0, partials, const_cast<Scalars*>(sc), 0.5, s);
}

}  // namespace otm
