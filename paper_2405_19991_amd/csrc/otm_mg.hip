// Geometric multigrid V-cycle as the PCG preconditioner (float32), after the
// paper's multigrid solver (Algorithm 3, Sec. 2.4: relax, restrict the
// residual, solve the coarsest level, interpolate and correct, relax).
//
// Level l has n_l = n / 2^l nodes per side.  Coarse element E covers the 2x2x2
// fine elements below it; its conductivity is twice their mean (the element
// stiffness of a cube of edge h is h times the unit-cube matrix), so the
// coarse operator is the same hex-8 stencil on the coarse conductivities.
// Interpolation P is trilinear and restriction R = P^T.  Relaxation is damped
// Jacobi (weight 0.9; by Gershgorin every eigenvalue of D^-1 A lies in [0, 2]
// for any conductivity field), the same number of steps in both legs, so the
// V-cycle is a symmetric positive definite operator and a valid PCG
// preconditioner; or the paper's 8-colour Gauss-Seidel (Sec. 2.4: S_v T_v =
// f_v - M_v, the nodes of one parity class (i mod 2, j mod 2, k mod 2) at a
// time, which share no element), colours 0..7 before the coarse correction
// and 7..0 after it, which makes the cycle symmetric as well.  Each relaxation step (and the residual before a
// restriction) is one z-march pass of the operator kernel with a relaxation
// epilogue (otm_march2.hip); the coarsest level (at most 4^3 nodes) is solved
// directly.
#include <hip/hip_runtime.h>

#include "otm_device.h"

namespace otm {

// k_c(E) = 2 * mean of the 8 fine elements of coarse element E (x fastest).
__global__ void __launch_bounds__(kBlock) k_mg_coarsen(int nc, const float* __restrict__ kf, float* __restrict__ kc) {
    const uint32_t ncc = (uint32_t)nc * nc * nc;
    const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= ncc) return;
    const uint32_t nf = 2 * nc;
    const uint32_t I = e % nc, J = (e / nc) % nc, K = e / ((uint32_t)nc * nc);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint32_t i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = 2 * K + (c >> 2);
        s += kf[i + nf * (j + nf * k)];
    }
    kc[e] = 0.25f * s;  // 2 * s / 8
}

// D^-1 of the level operator: D_v = (1/3) * sum of the 8 incident element conductivities.
__global__ void __launch_bounds__(kBlock) k_mg_dinv(int n, const float* __restrict__ k, float* __restrict__ dinv) {
    const uint32_t nn = (uint32_t)n * n * n;
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= nn) return;
    int i, j, kk;
    node_ijk(v, n, i, j, kk);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int a = wrapi(i - 1 + (c & 1), n), b = wrapi(j - 1 + ((c >> 1) & 1), n), z = wrapi(kk - 1 + (c >> 2), n);
        s += k[(uint32_t)a + (uint32_t)n * ((uint32_t)b + (uint32_t)n * (uint32_t)z)];
    }
    dinv[v] = 3.f / s;
}

// f_c = P^T r: each coarse node gathers the 27 fine nodes around its fine
// image with weights prod_d (1 at offset 0, 1/2 at offset +-1).
__global__ void __launch_bounds__(kBlock) k_mg_restrict(int nc, const float* __restrict__ r, float* __restrict__ fc) {
    const uint32_t ncc = (uint32_t)nc * nc * nc;
    const uint32_t V = blockIdx.x * kBlock + threadIdx.x;
    if (V >= ncc) return;
    const int nf = 2 * nc;
    const uint32_t nnf = (uint32_t)nf * nf * nf;
    const int I = (int)(V % nc), J = (int)((V / nc) % nc), K = (int)(V / ((uint32_t)nc * nc));
    uint32_t xs[3], ys[3], zs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        xs[d] = (uint32_t)wrapi(2 * I + d - 1, nf);
        ys[d] = (uint32_t)wrapi(2 * J + d - 1, nf) * (uint32_t)nf;
        zs[d] = (uint32_t)wrapi(2 * K + d - 1, nf) * (uint32_t)nf * (uint32_t)nf;
    }
    float s[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const float w = (dx != 1 ? 0.5f : 1.f) * (dy != 1 ? 0.5f : 1.f) * (dz != 1 ? 0.5f : 1.f);
                const uint32_t u = xs[dx] + ys[dy] + zs[dz];
#pragma unroll
                for (int l = 0; l < 3; ++l) s[l] += w * r[l * nnf + u];
            }
#pragma unroll
    for (int l = 0; l < 3; ++l) fc[l * ncc + V] = s[l];
}

// x_f += P x_c (trilinear interpolation of the coarse correction), or, with
// f0 given, x_f = w D^-1 f0 + P x_c (the fine level's Jacobi step from zero
// recomputed instead of stored).
__global__ void __launch_bounds__(kBlock) k_mg_prolong(int nc, const float* __restrict__ xc, float* __restrict__ xf,
                                                      const float* __restrict__ f0, const float* __restrict__ dinv0) {
    const uint32_t nf = 2 * nc;
    const uint32_t nnf = nf * nf * nf, ncc = (uint32_t)nc * nc * nc;
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= nnf) return;
    const uint32_t i = v % nf, j = (v / nf) % nf, k = v / (nf * nf);
    // per axis: even -> one coarse node (weight 1), odd -> two (1/2 each); an
    // even index takes its one node twice with weight 1/2
    const uint32_t i0 = i >> 1, j0 = j >> 1, k0 = k >> 1;
    const uint32_t i1 = (i & 1) ? (i0 + 1 == (uint32_t)nc ? 0 : i0 + 1) : i0;
    const uint32_t j1 = (j & 1) ? (j0 + 1 == (uint32_t)nc ? 0 : j0 + 1) : j0;
    const uint32_t k1 = (k & 1) ? (k0 + 1 == (uint32_t)nc ? 0 : k0 + 1) : k0;
    const uint32_t ncs = (uint32_t)nc, nc2 = ncs * ncs;
    const uint32_t a00 = i0 + ncs * j0, a01 = i1 + ncs * j0, a10 = i0 + ncs * j1, a11 = i1 + ncs * j1;
    const uint32_t z0 = nc2 * k0, z1 = nc2 * k1;
    const float wd = f0 ? kMgOmega * dinv0[v] : 0.f;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const float* c = xc + l * ncc;
        const float s = (c[a00 + z0] + c[a01 + z0] + c[a10 + z0] + c[a11 + z0]) +
                        (c[a00 + z1] + c[a01 + z1] + c[a10 + z1] + c[a11 + z1]);
        const float base = f0 ? wd * f0[l * nnf + v] : xf[l * nnf + v];
        xf[l * nnf + v] = base + 0.125f * s;
    }
}

// Coarsest level, solved directly (at most 4^3 nodes).  The periodic
// operator A is singular with the constants as its null space; the
// right-hand sides have zero sum, so x = (A + s 1 1^T)^-1 f is the zero-mean
// solution of A x = f for any s > 0 (1^T of the system gives s N 1^T x = 0).
// One block assembles A + s 1 1^T in float64 in LDS (s N = mean diagonal),
// inverts it by Gauss-Jordan elimination (symmetric positive definite: no
// pivoting), and stores the symmetrised inverse in float32.
// Rows and columns at pitch kMgCoarseMax (64): element (r, c) at r * 64 + c.
static_assert(kMgCoarseMax == 64, "pitch 64 indexing");
constexpr int kMgSetupThreads = 1024;
__global__ void __launch_bounds__(kMgSetupThreads) k_mg_coarse_setup(int n, const float* __restrict__ k,
                                                                    float* __restrict__ minv) {
    constexpr int P = kMgCoarseMax;
    __shared__ double M[P * P];
    __shared__ double col[P];
    __shared__ double row[P];
    __shared__ double diag_sum;
    const int N = n * n * n;
    const int tid = threadIdx.x;
    for (int e = tid; e < P * P; e += kMgSetupThreads) M[e] = 0.0;
    __syncthreads();
    if (tid < N) {
        const int v = tid;
        const int i = v % n, j = (v / n) % n, kk = v / (n * n);
        // the 8 elements incident to v; v is vertex (1-ex, 1-ey, 1-ez) of
        // the element with lower corner (i-1+ex, j-1+ey, k-1+ez)
        for (int e = 0; e < 8; ++e) {
            const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
            const int ei = (i - 1 + ex + n) % n, ej = (j - 1 + ey + n) % n, ek = (kk - 1 + ez + n) % n;
            const double ke = (double)k[ei + n * (ej + n * ek)] / 12.0;
            for (int q = 0; q < 8; ++q) {
                const int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
                const int d = (qa != 1 - ex) + (qb != 1 - ey) + (qc != 1 - ez);
                if (d == 1) continue;
                const int u = (ei + qa) % n + n * ((ej + qb) % n + n * ((ek + qc) % n));
                M[v * P + u] += ke * (d == 0 ? 4.0 : -1.0);
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int v = 0; v < N; ++v) t += M[v * P + v];
        diag_sum = t;
    }
    __syncthreads();
    const double sreg = diag_sum / ((double)N * N);
    for (int e = tid; e < P * P; e += kMgSetupThreads)
        if ((e >> 6) < N && (e & 63) < N) M[e] += sreg;
    __syncthreads();
    // in-place Gauss-Jordan inversion
    for (int p = 0; p < N; ++p) {
        const double piv = 1.0 / M[p * P + p];
        if (tid < N) {
            col[tid] = M[tid * P + p];
            row[tid] = (tid == p ? 1.0 : M[p * P + tid]) * piv;
        }
        __syncthreads();
        for (int e = tid; e < P * P; e += kMgSetupThreads) {
            const int r = e >> 6, c = e & 63;
            if (r >= N || c >= N) continue;
            if (r == p)
                M[e] = row[c];
            else
                M[e] = (c == p ? 0.0 : M[e]) - col[r] * row[c];
        }
        __syncthreads();
    }
    for (int e = tid; e < N * N; e += kMgSetupThreads) {
        const int r = e / N, c = e % N;
        minv[e] = (float)(0.5 * (M[r * P + c] + M[c * P + r]));
    }
}

// x = M^-1 f on the coarsest level, three loads (thread = (load, node)); the
// inverse and the right-hand sides are staged in LDS first.
__global__ void __launch_bounds__(kBlock) k_mg_coarse_solve(int N, const float* __restrict__ minv,
                                                           const float* __restrict__ f, float* __restrict__ x) {
    __shared__ float sm[kMgCoarseMax * kMgCoarseMax];
    __shared__ float sf[3 * kMgCoarseMax];
    for (int e = threadIdx.x; e < N * N; e += kBlock) sm[e] = minv[e];
    for (int e = threadIdx.x; e < 3 * N; e += kBlock) sf[e] = f[e];
    __syncthreads();
    const int l = threadIdx.x / kMgCoarseMax, v = threadIdx.x % kMgCoarseMax;
    if (l >= 3 || v >= N) return;
    float s0 = 0.f, s1 = 0.f;
    int u = 0;
    for (; u + 1 < N; u += 2) {
        s0 += sm[u * N + v] * sf[l * N + u];
        s1 += sm[(u + 1) * N + v] * sf[l * N + u + 1];
    }
    if (u < N) s0 += sm[u * N + v] * sf[l * N + u];
    x[l * N + v] = s0 + s1;
}

// One colour of the 8-colour Gauss-Seidel relaxation on a level (n even): a
// thread per 2x2x2 cell updates the cell's node of colour `color` (bits:
// i mod 2, j mod 2, k mod 2) in place, x_v += D^-1_v (f_v - (A x)_v), i.e.
// S_v x_v = f_v - M_v with M_v the off-diagonal part of [KT]_v.  Its 26
// neighbours all have other colours, so no thread reads a value another
// thread of the pass writes.  FIRST: the first pass of a cycle's first sweep,
// from x = 0: x_v = D^-1_v f_v and the cell's other seven nodes are set to 0
// (x needs no clearing).  DOT: every node of the cell is final after this
// pass (the last colour of the last sweep): the block sums of f . x per load
// go to partials[block * 3 + load] (r.z of the cycle on the finest level).
template <bool FIRST, bool DOT>
__global__ void __launch_bounds__(kBlock) k_mg_gs(int n, int color, const float* __restrict__ dinv,
                                                 const float* __restrict__ f, const float* __restrict__ k,
                                                 float* __restrict__ x, double* __restrict__ partials) {
    const int h = n >> 1;
    const uint32_t cells = (uint32_t)h * h * h;
    const uint32_t nn = (uint32_t)n * n * n;
    double acc[3] = {0.0, 0.0, 0.0};
    for (uint32_t cidx = blockIdx.x * kBlock + threadIdx.x; cidx < cells; cidx += gridDim.x * kBlock) {
        const int a = (int)(cidx % h), b = (int)((cidx / h) % h), cz = (int)(cidx / ((uint32_t)h * h));
        const int i = 2 * a + (color & 1), j = 2 * b + ((color >> 1) & 1), kk = 2 * cz + (color >> 2);
        const uint32_t v = (uint32_t)i + (uint32_t)n * ((uint32_t)j + (uint32_t)n * (uint32_t)kk);
        const float dv = dinv[v];
        if (FIRST) {
#pragma unroll
            for (int l = 0; l < 3; ++l) x[l * nn + v] = dv * f[l * nn + v];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (q == color) continue;
                const uint32_t u = (uint32_t)(2 * a + (q & 1)) +
                                   (uint32_t)n * ((uint32_t)(2 * b + ((q >> 1) & 1)) + (uint32_t)n * (uint32_t)(2 * cz + (q >> 2)));
#pragma unroll
                for (int l = 0; l < 3; ++l) x[l * nn + u] = 0.f;
            }
        } else {
            const Nbr o = nbr_of(i, j, kk, n);
            float ko[8];
            load_k8(k, o, ko);
            NodeCoef<float> cf;
            node_coefs(ko, cf);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const float ax = stencil_node<float, float>(cf, o, x + l * nn);
                x[l * nn + v] += dv * (f[l * nn + v] - ax);
            }
        }
        if (DOT) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t u = (uint32_t)(2 * a + (q & 1)) +
                                   (uint32_t)n * ((uint32_t)(2 * b + ((q >> 1) & 1)) + (uint32_t)n * (uint32_t)(2 * cz + (q >> 2)));
#pragma unroll
                for (int l = 0; l < 3; ++l) acc[l] += (double)f[l * nn + u] * (double)x[l * nn + u];
            }
        }
    }
    if (DOT) block_partials_at<3>(acc, partials, blockIdx.x);
}

// nu sweeps of 8-colour Gauss-Seidel on a level, forward (colours 0..7) or
// backward (7..0); from_zero: x starts at 0 (forward only).  With partials the
// last pass also sums f . x per block (at most kMaxBlocks blocks, each
// striding over the cells); returns that pass's block count.
int launch_mg_gs(int n, int nu, bool forward, bool from_zero, const float* dinv, const float* f, const float* k,
                 float* x, double* partials, hipStream_t s) {
    const int h = n / 2;
    const int grid = grid_for((int64_t)h * h * h, kMaxBlocks);
    for (int sw = 0; sw < nu; ++sw)
        for (int q = 0; q < 8; ++q) {
            const int color = forward ? q : 7 - q;
            const bool first = from_zero && sw == 0 && q == 0;
            const bool dot = partials && sw == nu - 1 && q == 7;
            if (first)
                hipLaunchKernelGGL((k_mg_gs<true, false>), dim3(grid), dim3(kBlock), 0, s, n, color, dinv, f, k, x,
                                   (double*)nullptr);
            else if (dot)
                hipLaunchKernelGGL((k_mg_gs<false, true>), dim3(grid), dim3(kBlock), 0, s, n, color, dinv, f, k, x,
                                   partials);
            else
                hipLaunchKernelGGL((k_mg_gs<false, false>), dim3(grid), dim3(kBlock), 0, s, n, color, dinv, f, k, x,
                                   (double*)nullptr);
        }
    return grid;
}

// The last two levels in one block (the second-coarsest level has at most
// 8^3 = 512 nodes, one thread each, everything in LDS): the same steps as the
// level kernels -- nu damped Jacobi steps from zero, the residual, its
// restriction, the direct coarse solve, interpolation and correction, nu
// steps -- without a launch per step.  A x at a node is the 21-point form of
// the hex-8 operator: (1/3) sum_8 k_e on the node, -(k_a + k_b)/12 for the 12
// edge-diagonal neighbours (the two elements they share with the node),
// -k_e/12 for the 8 corners, 0 for the 6 axis neighbours.
constexpr int kMgTailMax = 512;

template <int PITCH>
__device__ __forceinline__ void tail_apply(int n, int i, int j, int kk, const float* __restrict__ sk,
                                           const float (*__restrict__ x)[PITCH], float y[3]) {
    int ci[3], cj[3], ck[3];  // wrapped coordinates of offsets -1, 0, +1
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ci[d] = (i + d - 1 + n) % n;
        cj[d] = (j + d - 1 + n) % n;
        ck[d] = (kk + d - 1 + n) % n;
    }
    // conductivities of the 8 incident elements: ke[ez][ey][ex], ex = 1 is the
    // element whose lower corner is the node, ex = 0 the one below it in x
    float ke[2][2][2];
    float ksum = 0.f;
#pragma unroll
    for (int ez = 0; ez < 2; ++ez)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                ke[ez][ey][ex] = sk[ci[ex] + n * (cj[ey] + n * ck[ez])];
                ksum += ke[ez][ey][ex];
            }
    const int v = ci[1] + n * (cj[1] + n * ck[1]);
#pragma unroll
    for (int l = 0; l < 3; ++l) y[l] = (ksum * (1.f / 3.f)) * x[l][v];
    const float w = 1.f / 12.f;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int nz = (dx != 1) + (dy != 1) + (dz != 1);
                if (nz < 2) continue;  // the node itself and its axis neighbours
                float c = 0.f;         // sum of the elements shared with this neighbour
#pragma unroll
                for (int ez = 0; ez < 2; ++ez)
#pragma unroll
                    for (int ey = 0; ey < 2; ++ey)
#pragma unroll
                        for (int ex = 0; ex < 2; ++ex) {
                            const bool sx = dx == 1 || ex == (dx == 2 ? 1 : 0);
                            const bool sy = dy == 1 || ey == (dy == 2 ? 1 : 0);
                            const bool sz = dz == 1 || ez == (dz == 2 ? 1 : 0);
                            if (sx && sy && sz) c += ke[ez][ey][ex];
                        }
                const int u = ci[dx] + n * (cj[dy] + n * ck[dz]);
#pragma unroll
                for (int l = 0; l < 3; ++l) y[l] -= w * c * x[l][u];
            }
}

// One V-cycle over the second-coarsest level (n <= 8, one thread per node;
// every thread of the block takes part in the barriers) and the coarsest
// level below it, all in LDS: nu damped Jacobi steps from zero, the residual,
// its restriction, the direct coarse solve, interpolation and correction, nu
// steps.  f has pitch fp (global memory or LDS); k and D^-1 come from global
// memory.  The result is left in sx[return value].
// gs: 8-colour Gauss-Seidel sweeps in place (colours 0..7 before the coarse
// correction, 7..0 after it) instead of damped Jacobi steps.
__device__ __forceinline__ int mid_cycle(int n, int nu, const float* f, int fp, const float* __restrict__ k,
                         const float* __restrict__ dinv, const float* __restrict__ minv, float* sk,
                         float (*sx)[3][kMgTailMax], float (*sc)[3][kMgCoarseMax], bool gs) {
    const int N = n * n * n, nc = n / 2, Nc = nc * nc * nc;
    const int v = threadIdx.x;
    const bool own = v < N;
    int i = 0, j = 0, kk = 0;
    float fv[3] = {0.f, 0.f, 0.f}, wd = 0.f;
    if (own) {
        i = v % n;
        j = (v / n) % n;
        kk = v / (n * n);
        sk[v] = k[v];
        wd = kMgOmega * dinv[v];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            fv[l] = f[l * fp + v];
            sx[0][l][v] = wd * fv[l];  // first step from zero
        }
    }
    __syncthreads();
    int cur = 0;
    float y[3];
    const int colour = own ? (i & 1) + 2 * (j & 1) + 4 * (kk & 1) : -1;
    const float dv = own ? dinv[v] : 0.f;
    // one colour of Gauss-Seidel in place on sx[0]
    auto gs_colour = [&](int q) {
        if (colour == q) {
            tail_apply<kMgTailMax>(n, i, j, kk, sk, sx[0], y);
#pragma unroll
            for (int l = 0; l < 3; ++l) sx[0][l][v] += dv * (fv[l] - y[l]);
        }
        __syncthreads();
    };
    if (gs) {
        if (own) {
#pragma unroll
            for (int l = 0; l < 3; ++l) sx[0][l][v] = 0.f;
        }
        __syncthreads();
        for (int it = 0; it < nu; ++it)
            for (int q = 0; q < 8; ++q) gs_colour(q);
    } else {
        for (int it = 1; it < nu; ++it) {
            if (own) {
                tail_apply<kMgTailMax>(n, i, j, kk, sk, sx[cur], y);
#pragma unroll
                for (int l = 0; l < 3; ++l) sx[cur ^ 1][l][v] = sx[cur][l][v] + wd * (fv[l] - y[l]);
            }
            __syncthreads();
            cur ^= 1;
        }
    }
    // residual into the other buffer, then its restriction to the coarsest level
    if (own) {
        tail_apply<kMgTailMax>(n, i, j, kk, sk, sx[cur], y);
#pragma unroll
        for (int l = 0; l < 3; ++l) sx[cur ^ 1][l][v] = fv[l] - y[l];
    }
    __syncthreads();
    if (v < Nc) {
        const int I = v % nc, J = (v / nc) % nc, K = v / (nc * nc);
        float r[3] = {0.f, 0.f, 0.f};
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const float w = (dx ? 0.5f : 1.f) * (dy ? 0.5f : 1.f) * (dz ? 0.5f : 1.f);
                    const int u = (2 * I + dx + n) % n + n * ((2 * J + dy + n) % n + n * ((2 * K + dz + n) % n));
#pragma unroll
                    for (int l = 0; l < 3; ++l) r[l] += w * sx[cur ^ 1][l][u];
                }
#pragma unroll
        for (int l = 0; l < 3; ++l) sc[0][l][v] = r[l];
    }
    __syncthreads();
    if (v < 3 * kMgCoarseMax) {
        const int l = v / kMgCoarseMax, V = v % kMgCoarseMax;
        if (V < Nc) {
            float t = 0.f;
            for (int u = 0; u < Nc; ++u) t += minv[u * Nc + V] * sc[0][l][u];
            sc[1][l][V] = t;
        }
    }
    __syncthreads();
    if (own) {  // x += P x_c
        const int i0 = i >> 1, j0 = j >> 1, k0 = kk >> 1;
        const int i1 = (i & 1) ? (i0 + 1) % nc : i0, j1 = (j & 1) ? (j0 + 1) % nc : j0,
                  k1 = (kk & 1) ? (k0 + 1) % nc : k0;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const float* c = sc[1][l];
            const float t = (c[i0 + nc * (j0 + nc * k0)] + c[i1 + nc * (j0 + nc * k0)] + c[i0 + nc * (j1 + nc * k0)] +
                             c[i1 + nc * (j1 + nc * k0)]) +
                            (c[i0 + nc * (j0 + nc * k1)] + c[i1 + nc * (j0 + nc * k1)] + c[i0 + nc * (j1 + nc * k1)] +
                             c[i1 + nc * (j1 + nc * k1)]);
            sx[cur][l][v] += 0.125f * t;
        }
    }
    __syncthreads();
    if (gs) {
        for (int it = 0; it < nu; ++it)
            for (int q = 7; q >= 0; --q) gs_colour(q);
        return 0;
    }
    for (int it = 0; it < nu; ++it) {
        if (own) {
            tail_apply<kMgTailMax>(n, i, j, kk, sk, sx[cur], y);
#pragma unroll
            for (int l = 0; l < 3; ++l) sx[cur ^ 1][l][v] = sx[cur][l][v] + wd * (fv[l] - y[l]);
        }
        __syncthreads();
        cur ^= 1;
    }
    return cur;
}

__global__ void __launch_bounds__(kMgTailMax) k_mg_tail(int n, int nu, const float* __restrict__ f,
                                                       const float* __restrict__ k, const float* __restrict__ dinv,
                                                       const float* __restrict__ minv, float* __restrict__ xout,
                                                       int gs) {
    __shared__ float sk[kMgTailMax];
    __shared__ float sx[2][3][kMgTailMax];
    __shared__ float sc[2][3][kMgCoarseMax];
    const int N = n * n * n;
    const int cur = mid_cycle(n, nu, f, N, k, dinv, minv, sk, sx, sc, gs != 0);
    const int v = threadIdx.x;
    if (v < N) {
#pragma unroll
        for (int l = 0; l < 3; ++l) xout[l * N + v] = sx[cur][l][v];
    }
}

void launch_mg_tail(int n, int nu, const float* f, const float* k, const float* dinv, const float* minv, float* x,
                    bool gs, hipStream_t s) {
    hipLaunchKernelGGL(k_mg_tail, dim3(1), dim3(kMgTailMax), 0, s, n, nu, f, k, dinv, minv, x, gs ? 1 : 0);
}

void launch_mg_coarsen(int nc, const float* kf, float* kc, float* dinv_c, hipStream_t s) {
    const int64_t ncc = (int64_t)nc * nc * nc;
    hipLaunchKernelGGL(k_mg_coarsen, dim3(nblocks_for(ncc)), dim3(kBlock), 0, s, nc, kf, kc);
    hipLaunchKernelGGL(k_mg_dinv, dim3(nblocks_for(ncc)), dim3(kBlock), 0, s, nc, kc, dinv_c);
}

void launch_mg_restrict(int nc, const float* r, float* fc, hipStream_t s) {
    const int64_t ncc = (int64_t)nc * nc * nc;
    hipLaunchKernelGGL(k_mg_restrict, dim3(nblocks_for(ncc)), dim3(kBlock), 0, s, nc, r, fc);
}

void launch_mg_prolong(int nc, const float* xc, float* xf, const float* f0, const float* dinv0, hipStream_t s) {
    const int64_t nnf = (int64_t)8 * nc * nc * nc;
    hipLaunchKernelGGL(k_mg_prolong, dim3(nblocks_for(nnf)), dim3(kBlock), 0, s, nc, xc, xf, f0, dinv0);
}

void launch_mg_coarse_setup(int n, const float* k, float* minv, hipStream_t s) {
    hipLaunchKernelGGL(k_mg_coarse_setup, dim3(1), dim3(kMgSetupThreads), 0, s, n, k, minv);
}

void launch_mg_coarse_solve(int n, const float* minv, const float* f, float* x, hipStream_t s) {
    hipLaunchKernelGGL(k_mg_coarse_solve, dim3(1), dim3(kBlock), 0, s, n * n * n, minv, f, x);
}

int mg_vcycle(const MgHierarchy& H, double* partials, int max_blocks, hipStream_t s, const float** z_out) {
    (void)max_blocks;
    const int L = H.levels;
    int cur[kMgMaxLevels] = {};
    // the last two levels run in one block when there is a level above them
    // (one CU relaxes an 8^3 level faster than the launches would take; a
    // 16^3 level is already slower there than as grid-wide passes)
    const bool tail = L >= 3;
    const int Ldown = tail ? L - 2 : L - 1;
    // down: nu relaxation steps from zero, the last one replaced by the
    // residual; restrict the residual (a.t)
    for (int l = 0; l < Ldown; ++l) {
        const MgLevel& a = H.lv[l];
        const int nu = l == 0 ? H.sweeps : H.coarse_sweeps;
        int c = 0;
        if (H.gs) {  // nu forward sweeps in place on x[0], then the residual
            launch_mg_gs(a.n, nu, true, true, a.dinv, a.f, a.k, a.x[0], nullptr, s);
            launch_mg_march(a.n, a.tile, false, MG_RESID, a.x[0], a.dinv, a.f, a.k, a.t, nullptr, s);
        } else if (nu == 1) {
            launch_mg_march(a.n, a.tile, true, MG_RESID, nullptr, a.dinv, a.f, a.k, a.t, nullptr, s);
        } else {
            launch_mg_march(a.n, a.tile, true, MG_RELAX, nullptr, a.dinv, a.f, a.k, a.x[0], nullptr, s);
            for (int it = 2; it < nu; ++it) {
                launch_mg_march(a.n, a.tile, false, MG_RELAX, a.x[c], a.dinv, a.f, a.k, a.x[c ^ 1], nullptr, s);
                c ^= 1;
            }
            launch_mg_march(a.n, a.tile, false, MG_RESID, a.x[c], a.dinv, a.f, a.k, a.t, nullptr, s);
        }
        launch_mg_restrict(H.lv[l + 1].n, a.t, H.lv[l + 1].f, s);
        cur[l] = c;
    }
    if (tail) {
        const MgLevel& t = H.lv[L - 2];
        launch_mg_tail(t.n, H.coarse_sweeps, t.f, t.k, t.dinv, H.minv, t.x[0], H.gs, s);
        cur[L - 2] = 0;
    } else {
        const MgLevel& cl = H.lv[L - 1];
        launch_mg_coarse_solve(cl.n, H.minv, cl.f, cl.x[0], s);
        cur[L - 1] = 0;
    }
    // up: interpolate and correct, nu relaxation steps (the adjoint of the
    // way down, so the cycle is a symmetric operator)
    int nb = 0;
    for (int l = Ldown - 1; l >= 0; --l) {
        const MgLevel& a = H.lv[l];
        const int nu = l == 0 ? H.sweeps : H.coarse_sweeps;
        int c = cur[l];
        if (H.gs) {  // x += P x_c, then nu backward sweeps (the adjoint of the way down)
            launch_mg_prolong(H.lv[l + 1].n, H.lv[l + 1].x[cur[l + 1]], a.x[0], nullptr, nullptr, s);
            const int g = launch_mg_gs(a.n, nu, false, false, a.dinv, a.f, a.k, a.x[0], l == 0 ? partials : nullptr, s);
            if (l == 0) nb = g;
            cur[l] = 0;
            continue;
        }
        launch_mg_prolong(H.lv[l + 1].n, H.lv[l + 1].x[cur[l + 1]], a.x[c], nu == 1 ? a.f : nullptr,
                          nu == 1 ? a.dinv : nullptr, s);
        for (int it = 0; it < nu; ++it) {
            const bool last = (l == 0 && it == nu - 1);
            launch_mg_march(a.n, a.tile, false, MG_RELAX, a.x[c], a.dinv, a.f, a.k, a.x[c ^ 1],
                            last ? partials : nullptr, s);
            if (last) nb = a.tile.blocks;
            c ^= 1;
        }
        cur[l] = c;
    }
    if (z_out) *z_out = H.lv[0].x[cur[0]];
    return nb;
}

}  // namespace otm
