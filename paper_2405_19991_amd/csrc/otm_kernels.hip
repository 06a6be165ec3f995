// HIP kernels for the periodic thermal homogenization step (gfx950).
//
// Grid convention: n^3 elements and n^3 nodes, periodic; node (i,j,k) is the
// lower corner of element (i,j,k); flat index i + n*(j + n*k).  Element e with
// origin o has local vertex l = a + 2b + 4c at node o + (a,b,c).
//
// Operator (hex-8 trilinear conduction, unit voxel): per element the 8x8
// matrix is (1/12) * [4 on the diagonal, 0 between vertices one edge apart,
// -1 between face-diagonal and body-diagonal vertices].  Gathered per node
// (the node-centric [KT]_v of Sec. 2.4), with k_o the conductivity of the
// incident element whose origin is v + (a'-1, b'-1, c'-1):
//   centre          : (1/3) sum_o k_o
//   face neighbour  : 0
//   edge-diagonal   : -(1/12)(k_o1 + k_o2) over the two elements sharing it
//   corner          : -(1/12) k_o of the one element sharing it.
#include "otm_device.h"

namespace otm {

// ---------------------------------------------------------------- filter
// Separable periodic hat weights w(d) = max(0, r - |d|), normalized per axis;
// the 3D weight is the product, so its normalization is the product of the
// 1D normalizations.  Reach R < 4.
FilterW filter_weights(double r) {
    FilterW f{};
    if (!(r > 0.0)) {
        f.R = 0;
        f.w[0] = 1.0;
        return f;
    }
    int R = 0;
    while (r - (double)(R + 1) > 0.0 && R < 4) ++R;
    f.R = R;
    double s = 0.0;
    for (int d = -R; d <= R; ++d) s += r - fabs((double)d);
    for (int d = -R; d <= R; ++d) f.w[d + R] = (r - fabs((double)d)) / s;
    return f;
}

__device__ __forceinline__ double filter_at(const double* in, int n, int i, int j, int k, const FilterW& f) {
    double acc = 0.0;
    for (int dz = -f.R; dz <= f.R; ++dz) {
        const int zk = wrapi(k + dz, n) * n;
        double accy = 0.0;
        for (int dy = -f.R; dy <= f.R; ++dy) {
            const int row = (wrapi(j + dy, n) + zk) * n;
            double accx = 0.0;
            for (int dx = -f.R; dx <= f.R; ++dx) accx += f.w[dx + f.R] * in[row + wrapi(i + dx, n)];
            accy += f.w[dy + f.R] * accx;
        }
        acc += f.w[dz + f.R] * accy;
    }
    return acc;
}

__device__ __forceinline__ void b_filter(int bid_, int nblk_, int n, const FilterW& f, const double* __restrict__ in,
                                                   double* __restrict__ out) {
    const int64_t nn = (int64_t)n * n * n;
    for (int64_t e = (int64_t)bid_ * kBlock + threadIdx.x; e < nn; e += (int64_t)nblk_ * kBlock) {
        int i, j, k;
        node_ijk(e, n, i, j, k);
        out[e] = filter_at(in, n, i, j, k, f);
    }
}

__global__ void __launch_bounds__(kBlock) k_filter(int n, FilterW f, const double* __restrict__ in,
                                                   double* __restrict__ out) { b_filter(blockIdx.x, gridDim.x, n, f, in, out); }

// rho -> rho~ -> k (SIMP), plus the sums of rho and rho~^p.
__device__ __forceinline__ void b_filter_simp(int bid_, int nblk_, int n, const FilterW& f, const double* __restrict__ rho,
                                                        double* __restrict__ rhof, double* __restrict__ k,
                                                        float* __restrict__ k32, double k0, double kmin, double p,
                                                        double* partials, unsigned* counter, Scalars* sc) {
    const int64_t nn = (int64_t)n * n * n;
    double acc[2] = {0.0, 0.0};
    for (int64_t e = (int64_t)bid_ * kBlock + threadIdx.x; e < nn; e += (int64_t)nblk_ * kBlock) {
        int i, j, kk;
        node_ijk(e, n, i, j, kk);
        const double rf = filter_at(rho, n, i, j, kk, f);
        const double rp = (p == 3.0) ? rf * rf * rf : pow(rf, p);  // the paper's p = 3 without pow
        const double ke = kmin + rp * (k0 - kmin);
        rhof[e] = rf;
        k[e] = ke;
        if (k32) k32[e] = (float)ke;
        acc[0] += rho[e];
        acc[1] += rp;
    }
    block_partials<2>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_filter_simp(int n, FilterW f, const double* __restrict__ rho,
                                                        double* __restrict__ rhof, double* __restrict__ k,
                                                        float* __restrict__ k32, double k0, double kmin, double p,
                                                        double* partials, unsigned* counter, Scalars* sc) { b_filter_simp(blockIdx.x, gridDim.x, n, f, rho, rhof, k, k32, k0, kmin, p, partials, counter, sc); }

// ---------------------------------------------------------------- node setup
// Macro load b^i_v = (1/4)(sum of k over the 4 incident elements on the -i side
// of v  -  sum over the 4 on the +i side); Jacobi diagonal d_v = (1/3) sum of
// the 8 incident k.  Also the sums of b^i (they vanish up to rounding; the
// engine projects b to zero mean).
__device__ __forceinline__ void b_setup_nodes(int bid_, int nblk_, int n, const double* __restrict__ k, double* __restrict__ b,
                                                        double* __restrict__ dinv, float* __restrict__ dinv32,
                                                        double* partials, unsigned* counter, Scalars* sc) {
    const int64_t nn = (int64_t)n * n * n;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t v = (int64_t)bid_ * kBlock + threadIdx.x; v < nn; v += (int64_t)nblk_ * kBlock) {
        int i, j, kk;
        node_ijk(v, n, i, j, kk);
        const int xi[2] = {wrapi(i - 1, n), i};
        const int yj[2] = {wrapi(j - 1, n) * n, j * n};
        const int zk[2] = {wrapi(kk - 1, n) * n * n, kk * n * n};
        double ko[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) ko[o] = k[xi[o & 1] + yj[(o >> 1) & 1] + zk[(o >> 2) & 1]];
        double tot = 0.0, side[3][2] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            tot += ko[o];
            side[0][o & 1] += ko[o];
            side[1][(o >> 1) & 1] += ko[o];
            side[2][(o >> 2) & 1] += ko[o];
        }
        // element with a' = 0 lies on the -x side of v
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double bv = 0.25 * (side[a][0] - side[a][1]);
            b[a * nn + v] = bv;
            acc[a] += bv;
        }
        const double d = tot / 3.0;
        dinv[v] = 1.0 / d;
        if (dinv32) dinv32[v] = (float)(1.0 / d);
    }
    block_partials<3>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_setup_nodes(int n, const double* __restrict__ k, double* __restrict__ b,
                                                        double* __restrict__ dinv, float* __restrict__ dinv32,
                                                        double* partials, unsigned* counter, Scalars* sc) { b_setup_nodes(blockIdx.x, gridDim.x, n, k, b, dinv, dinv32, partials, counter, sc); }

// ---------------------------------------------------------------- operator
template <typename T>
__global__ void __launch_bounds__(kBlock) k_apply(int n, const T* __restrict__ k, const T* __restrict__ x,
                                                  T* __restrict__ y) {
    const int64_t nn = (int64_t)n * n * n;
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nn) return;
    int i, j, kk;
    node_ijk(v, n, i, j, kk);
    const Nbr o = nbr_of(i, j, kk, n);
    T ko[8];
    load_k8(k, o, ko);
    NodeCoef<T> c;
    node_coefs(ko, c);
#pragma unroll
    for (int l = 0; l < 3; ++l) y[l * nn + v] = stencil_node<T, T>(c, o, x + l * nn);
}

// ---------------------------------------------------------------- PCG pieces
// r = b - A x (float64 operator) stored as TR; p_old zeroed (START) or kept
// (REFRESH); sums ||r||^2, r.D^-1 r, ||b||^2 -> epilogue per mode.

template <typename TR>
__device__ __forceinline__ void b_residual(int bid_, int nblk_, int n, const double* __restrict__ k, const double* __restrict__ b,
                                                     const double* __restrict__ x, TR* __restrict__ r,
                                                     TR* __restrict__ p_old, const TR* __restrict__ dinv, int mode,
                                                     int x_zero, double* partials, unsigned* counter, Scalars* sc) {
    const int64_t nn = (int64_t)n * n * n;
    double acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.0;
    for (int64_t v = (int64_t)bid_ * kBlock + threadIdx.x; v < nn; v += (int64_t)nblk_ * kBlock) {
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
            if (mode == RES_START) p_old[l * nn + v] = (TR)0;
            acc[l] += rv * rv;
            acc[3 + l] += dv * (double)rs * (double)rs;
            acc[6 + l] += bv * bv;
        }
    }
    block_partials<9>(acc, partials);
}

template <typename TR>
__global__ void __launch_bounds__(kBlock) k_residual(int n, const double* __restrict__ k, const double* __restrict__ b,
                                                     const double* __restrict__ x, TR* __restrict__ r,
                                                     TR* __restrict__ p_old, const TR* __restrict__ dinv, int mode,
                                                     int x_zero, double* partials, unsigned* counter, Scalars* sc) { b_residual<TR>(blockIdx.x, gridDim.x, n, k, b, x, r, p_old, dinv, mode, x_zero, partials, counter, sc); }

// p_new = D^-1 r + beta p_old (beta == 0 -> p_new = D^-1 r) for active loads.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dir(int n, const T* __restrict__ r, const T* __restrict__ dinv,
                                                const T* __restrict__ p_old, T* __restrict__ p_new,
                                                const Scalars* __restrict__ sc) {
    const int64_t nn = (int64_t)n * n * n;
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nn) return;
    const T dv = dinv[v];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (!sc->active[l]) continue;
        const T beta = (T)sc->beta[l];
        const T z = dv * r[l * nn + v];
        p_new[l * nn + v] = (beta == (T)0) ? z : z + beta * p_old[l * nn + v];
    }
}

// q = A p for active loads; sums p.q -> alpha = rz / pq.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_apply_pq(int n, const T* __restrict__ k, const T* __restrict__ p,
                                                     T* __restrict__ q, double* partials, unsigned* counter,
                                                     Scalars* sc) {
    const int64_t nn = (int64_t)n * n * n;
    const int act[3] = {sc->active[0], sc->active[1], sc->active[2]};
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < nn; v += (int64_t)gridDim.x * kBlock) {
        int i, j, kk;
        node_ijk(v, n, i, j, kk);
        const Nbr o = nbr_of(i, j, kk, n);
        T ko[8];
        load_k8(k, o, ko);
        NodeCoef<T> c;
        node_coefs(ko, c);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            const T y = stencil_node<T, T>(c, o, p + l * nn);
            q[l * nn + v] = y;
            acc[l] += (double)p[l * nn + v] * (double)y;
        }
    }
    block_partials<3>(acc, partials);
}

// x += alpha p; r -= alpha q; sums r.D^-1 r and ||r||^2 -> beta, stop test.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_update(int n, T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                                   const T* __restrict__ q, const T* __restrict__ dinv,
                                                   double* partials, unsigned* counter, Scalars* sc) {
    const int64_t nn = (int64_t)n * n * n;
    const int act[3] = {sc->active[0], sc->active[1], sc->active[2]};
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < nn; v += (int64_t)gridDim.x * kBlock) {
        const T dv = dinv[v];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (!act[l]) continue;
            const T a = (T)sc->alpha[l];
            x[l * nn + v] += a * p[l * nn + v];
            const T rv = r[l * nn + v] - a * q[l * nn + v];
            r[l * nn + v] = rv;
            acc[l] += (double)dv * (double)rv * (double)rv;
            acc[3 + l] += (double)rv * (double)rv;
        }
    }
    block_partials<6>(acc, partials);
}

// x64 += x32; x32 = 0 (mixed-precision solution accumulation).
__global__ void __launch_bounds__(kBlock) k_accumulate(int64_t count, double* __restrict__ x, float* __restrict__ x32) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= count) return;
    x[v] += (double)x32[v];
    x32[v] = 0.0f;
}

// sums of the three loads of x -> sc->xsum (slot 0) or sc->bsum (slot 1)
__device__ __forceinline__ void b_sum3(int bid_, int nblk_, int n, const double* __restrict__ x, int slot, double* partials,
                                                 unsigned* counter, Scalars* sc) {
    const int64_t nn = (int64_t)n * n * n;
    double acc[3] = {0, 0, 0};
    for (int64_t v = (int64_t)bid_ * kBlock + threadIdx.x; v < nn; v += (int64_t)nblk_ * kBlock) {
#pragma unroll
        for (int l = 0; l < 3; ++l) acc[l] += x[l * nn + v];
    }
    block_partials<3>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_sum3(int n, const double* __restrict__ x, int slot, double* partials,
                                                 unsigned* counter, Scalars* sc) { b_sum3(blockIdx.x, gridDim.x, n, x, slot, partials, counter, sc); }

// x^l -= sum^l / n^3 with the sum taken from slot 0 (xsum) or 1 (bsum)
__device__ __forceinline__ void b_sub_mean3(int bid_, int nblk_, int n, double* __restrict__ x, int slot, const Scalars* sc) {
    const int64_t nn = (int64_t)n * n * n;
    for (int64_t v = (int64_t)bid_ * kBlock + threadIdx.x; v < nn; v += (int64_t)nblk_ * kBlock) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const double m = (slot == 0 ? sc->xsum[l] : sc->bsum[l]) / (double)nn;
            x[l * nn + v] -= m;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_sub_mean3(int n, double* __restrict__ x, int slot, const Scalars* sc) { b_sub_mean3(blockIdx.x, gridDim.x, n, x, slot, sc); }

// ---------------------------------------------------------------- tensor
// u^i_l = X_{l,i} - chi^i(vertex l);  E_c = u^i . K u^j for the six pairs.
// K u at vertex l = (1/12)(4 u_l - sum of u over vertices differing in 2 or 3
// coordinates) = (1/12)(5 u_l + sum over the 3 edge neighbours - sum of all 8).
__device__ __forceinline__ void element_energies(const double* __restrict__ chi, int64_t nn, int n, int i, int j,
                                                 int k, double (&E)[6]) {
    const int xi[2] = {i, wrapi(i + 1, n)};
    const int yj[2] = {j * n, wrapi(j + 1, n) * n};
    const int zk[2] = {k * n * n, wrapi(k + 1, n) * n * n};
    double u[3][8];
#pragma unroll
    for (int l = 0; l < 8; ++l) {
        const int v = xi[l & 1] + yj[(l >> 1) & 1] + zk[(l >> 2) & 1];
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a][l] = (double)((l >> a) & 1) - chi[a * nn + v];
    }
    double Ku[3][8];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double tot = 0.0;
#pragma unroll
        for (int l = 0; l < 8; ++l) tot += u[a][l];
#pragma unroll
        for (int l = 0; l < 8; ++l)
            Ku[a][l] = (5.0 * u[a][l] + u[a][l ^ 1] + u[a][l ^ 2] + u[a][l ^ 4] - tot) * (1.0 / 12.0);
    }
    const int I[6] = {0, 1, 2, 0, 1, 0};
    const int J[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < 8; ++l) s += u[I[c]][l] * Ku[J[c]][l];
        E[c] = s;
    }
}

__device__ __forceinline__ void b_energy(int bid_, int nblk_, int n, const double* __restrict__ k, const double* __restrict__ chi,
                                                   double* partials, unsigned* counter, Scalars* sc) {
    const int64_t nn = (int64_t)n * n * n;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t e = (int64_t)bid_ * kBlock + threadIdx.x; e < nn; e += (int64_t)nblk_ * kBlock) {
        int i, j, kk;
        node_ijk(e, n, i, j, kk);
        double E[6];
        element_energies(chi, nn, n, i, j, kk, E);
        const double ke = k[e];
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += ke * E[c];
    }
    block_partials<6>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_energy(int n, const double* __restrict__ k, const double* __restrict__ chi,
                                                   double* partials, unsigned* counter, Scalars* sc) { b_energy(blockIdx.x, gridDim.x, n, k, chi, partials, counter, sc); }

// s~_e = n^-3 p rho~^(p-1) (k0 - kmin) sum_c w_c E_e,c
__device__ __forceinline__ void b_sens(int bid_, int nblk_, int n, const double* __restrict__ rhof, const double* __restrict__ chi,
                                                 W6 w, double k0, double kmin, double p, double* __restrict__ st) {
    const int64_t nn = (int64_t)n * n * n;
    for (int64_t e = (int64_t)bid_ * kBlock + threadIdx.x; e < nn; e += (int64_t)nblk_ * kBlock) {
    int i, j, kk;
    node_ijk(e, n, i, j, kk);
    double E[6];
    element_energies(chi, nn, n, i, j, kk, E);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) s += w.w[c] * E[c];
    const double rf = rhof[e];
    st[e] = p * ((p == 3.0) ? rf * rf : pow(rf, p - 1.0)) * (k0 - kmin) * s / (double)nn;
    }
}

__global__ void __launch_bounds__(kBlock) k_sens(int n, const double* __restrict__ rhof, const double* __restrict__ chi,
                                                 W6 w, double k0, double kmin, double p, double* __restrict__ st) { b_sens(blockIdx.x, gridDim.x, n, rhof, chi, w, k0, kmin, p, st); }

// ---------------------------------------------------------------- OC
// q_e = rho_e (max(0, -s_e) n^3)^eta ; rho_new(lam) = clamp(q lam^-eta, lo, hi)
// Every kernel that needs q_e (stored or recomputed from rho and s) evaluates
// this one expression, so a recomputed q is bit-identical to a stored one.
__device__ __forceinline__ double oc_q(double rho_e, double s_e, int64_t nn, double eta) {
    const double B = fmax(0.0, -s_e) * (double)nn;
    return rho_e * (eta == 0.5 ? sqrt(B) : pow(B, eta));
}

__device__ __forceinline__ void b_oc_prepare(int bid_, int nblk_, int64_t nn, const double* __restrict__ rho,
                                                       const double* __restrict__ s, double eta,
                                                       double* __restrict__ q) {
    for (int64_t e = (int64_t)bid_ * kBlock + threadIdx.x; e < nn; e += (int64_t)nblk_ * kBlock) {
    q[e] = oc_q(rho[e], s[e], nn, eta);
    }
}

__global__ void __launch_bounds__(kBlock) k_oc_prepare(int64_t nn, const double* __restrict__ rho,
                                                       const double* __restrict__ s, double eta,
                                                       double* __restrict__ q) { b_oc_prepare(blockIdx.x, gridDim.x, nn, rho, s, eta, q); }

// q as above (stored when q is not null), plus per block the largest
// (q_e / lo_e)^(1/eta) -- at or above that lambda every element of the block
// sits at its lower move limit lo_e = max(rho_min, rho_e - m) -- and the sum of
// lo_e (partials[2b], [2b+1]).
__global__ void __launch_bounds__(kBlock) k_oc_prepare_max(int64_t nn, const double* __restrict__ rho,
                                                           const double* __restrict__ s, double eta, double move,
                                                           double rho_min, double* __restrict__ q,
                                                           double* __restrict__ partials) {
    double tmax = 0.0, losum = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nn; e += (int64_t)gridDim.x * kBlock) {
        const double r = rho[e];
        const double qe = oc_q(r, s[e], nn, eta);
        if (q) q[e] = qe;
        const double lo = fmax(rho_min, r - move);
        const double ratio = qe / lo;
        tmax = fmax(tmax, eta == 0.5 ? ratio * ratio : pow(ratio, 1.0 / eta));
        losum += lo;
    }
    __shared__ double sh[2][kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        tmax = fmax(tmax, __shfl_xor(tmax, off, 64));
        losum += __shfl_xor(losum, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = tmax;
        sh[1][threadIdx.x >> 6] = losum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh[0][0], t = sh[1][0];
        for (int w = 1; w < kBlock / 64; ++w) {
            m = fmax(m, sh[0][w]);
            t += sh[1][w];
        }
        partials[2 * blockIdx.x] = m;
        partials[2 * blockIdx.x + 1] = t;
    }
}

// Candidates of the next kOcLevels bisection levels below [l1, l2], in
// breadth-first order of the midpoint tree, each computed exactly as the
// sequential bisection would: mid = 0.5 (lo + hi) of its parent interval.
// The bisection tree's candidates below [l1, l2], node t at lane t (t <
// kOcCands): the lane walks from the root to its node, halving the interval
// with the same mid-point arithmetic as step-by-step bisection, so each
// candidate equals the mid-point that sequential bisection would reach there.
__device__ void oc_candidates_lane(Scalars* sc, double l1, double l2, double eta) {
    const int t = threadIdx.x;
    if (t >= kOcCands) return;
    int path[kOcLevels];
    int depth = 0;
    for (int u = t; u > 0; u = (u - 1) / 2) path[depth++] = u & 1;  // 1: left child
    double lo = l1, hi = l2;
    for (int d = depth - 1; d >= 0; --d) {
        const double mid = 0.5 * (lo + hi);
        if (path[d])
            hi = mid;
        else
            lo = mid;
    }
    const double mid = 0.5 * (lo + hi);
    sc->cand[t] = mid;
    sc->cpow[t] = (eta == 0.5) ? 1.0 / sqrt(mid) : pow(mid, -eta);
}

// Bisection bracket [0, l2]: l2 = 1e9, lowered to just above the largest
// block bound of k_oc_prepare_max when that is smaller and the volume there
// (every element at its lower move limit, the smallest volume any lambda
// gives) is below V*: then no larger lambda can be the root, and the
// bisection reaches its stopping width in fewer halvings.  Otherwise (no
// positive bound, or a V* at or below that smallest volume, where the
// bisection runs to the top of the bracket) the bracket stays [0, 1e9].
// nblocks = 0 keeps 1e9.
__global__ void __launch_bounds__(kBlock) k_oc_init(Scalars* sc, double vstar_n, double eta,
                                                    const double* __restrict__ partials, int nblocks) {
    __shared__ double sl2;
    __shared__ double sh[2][kBlock / 64];
    double t = 0.0, lo_sum = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) {
        t = fmax(t, partials[2 * b]);
        lo_sum += partials[2 * b + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        t = fmax(t, __shfl_xor(t, off, 64));
        lo_sum += __shfl_xor(lo_sum, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = t;
        sh[1][threadIdx.x >> 6] = lo_sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            t = fmax(t, sh[0][w]);
            lo_sum += sh[1][w];
        }
        const double up = t * (1.0 + 1e-12);
        const bool lower = nblocks > 0 && t > 0.0 && up < 1e9 && lo_sum < vstar_n * (1.0 - 1e-12);
        sl2 = lower ? up : 1e9;
        sc->l1 = 0.0;
        sc->l2 = sl2;
        sc->vstar_n = vstar_n;
        sc->oc_steps = 0;
        sc->oc_done = 0;
    }
    __syncthreads();
    oc_candidates_lane(sc, 0.0, sl2, eta);
}

// One pass: sum clamp(q c_m, lo, hi) for every candidate, then walk the tree
// with the sequential stopping rule (width <= 1e-13 (l1 + l2), 200 halvings).
// kFromSens: `q` holds the sensitivities s and q_e is recomputed from them.
template <bool kFromSens = false>
__device__ __forceinline__ void b_oc_pass(int bid_, int nblk_, int64_t nn, const double* __restrict__ rho,
                                                    const double* __restrict__ q, double move, double rho_min,
                                                    double eta, double* partials, unsigned* counter, Scalars* sc) {
    if (sc->oc_done) return;
    double cp[kOcCands];
#pragma unroll
    for (int t = 0; t < kOcCands; ++t) cp[t] = sc->cpow[t];
    double acc[kOcCands];
#pragma unroll
    for (int t = 0; t < kOcCands; ++t) acc[t] = 0.0;
#pragma unroll 2
    for (int64_t e = (int64_t)bid_ * kBlock + threadIdx.x; e < nn; e += (int64_t)nblk_ * kBlock) {
        const double r = rho[e], qe = kFromSens ? oc_q(r, q[e], nn, eta) : q[e];
        const double lo = fmax(rho_min, r - move), hi = fmin(1.0, r + move);
#pragma unroll
        for (int t = 0; t < kOcCands; ++t) acc[t] += fmin(hi, fmax(lo, qe * cp[t]));
    }
    block_partials<kOcCands>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_oc_pass(int64_t nn, const double* __restrict__ rho,
                                                    const double* __restrict__ q, double move, double rho_min,
                                                    double eta, double* partials, unsigned* counter, Scalars* sc) { b_oc_pass(blockIdx.x, gridDim.x, nn, rho, q, move, rho_min, eta, partials, counter, sc); }

__device__ __forceinline__ void b_oc_apply(int bid_, int nblk_, int64_t nn, double* __restrict__ rho, const double* __restrict__ q,
                                                     double eta, double move, double rho_min, const Scalars* sc) {
    for (int64_t e = (int64_t)bid_ * kBlock + threadIdx.x; e < nn; e += (int64_t)nblk_ * kBlock) {
    const double lam = sc->lam;
    const double c = (eta == 0.5) ? 1.0 / sqrt(lam) : pow(lam, -eta);
    const double r = rho[e];
    const double lo = fmax(rho_min, r - move), hi = fmin(1.0, r + move);
    rho[e] = fmin(hi, fmax(lo, q[e] * c));
    }
}

__global__ void __launch_bounds__(kBlock) k_oc_apply(int64_t nn, double* __restrict__ rho, const double* __restrict__ q,
                                                     double eta, double move, double rho_min, const Scalars* sc) { b_oc_apply(blockIdx.x, gridDim.x, nn, rho, q, eta, move, rho_min, sc); }

// Pass and update with q recomputed from the sensitivities (no q buffer):
// the same sums over the same grid as k_oc_pass, so the same lambda.
__global__ void __launch_bounds__(kBlock) k_oc_pass_s(int64_t nn, const double* __restrict__ rho,
                                                      const double* __restrict__ s, double move, double rho_min,
                                                      double eta, double* partials, Scalars* sc) {
    b_oc_pass<true>(blockIdx.x, gridDim.x, nn, rho, s, move, rho_min, eta, partials, nullptr, sc);
}

// rho_out may be rho itself (each element is read and written by one thread).
// lambda_out (device, may be null) receives the multiplier.
__global__ void __launch_bounds__(kBlock) k_oc_apply_s(int64_t nn, const double* rho, const double* __restrict__ s,
                                                       double* rho_out, double* __restrict__ lambda_out, double eta,
                                                       double move, double rho_min, const Scalars* sc) {
    const double lam = sc->lam;
    const double c = (eta == 0.5) ? 1.0 / sqrt(lam) : pow(lam, -eta);
    if (lambda_out && blockIdx.x == 0 && threadIdx.x == 0) *lambda_out = lam;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nn; e += (int64_t)gridDim.x * kBlock) {
        const double r = rho[e];
        const double lo = fmax(rho_min, r - move), hi = fmin(1.0, r + move);
        rho_out[e] = fmin(hi, fmax(lo, oc_q(r, s[e], nn, eta) * c));
    }
}

__device__ __forceinline__ void b_clamp(int bid_, int nblk_, int64_t nn, double* __restrict__ rho, double lo, double hi) {
    for (int64_t e = (int64_t)bid_ * kBlock + threadIdx.x; e < nn; e += (int64_t)nblk_ * kBlock) {
    rho[e] = fmin(hi, fmax(lo, rho[e]));
    }
}

__global__ void __launch_bounds__(kBlock) k_clamp(int64_t nn, double* __restrict__ rho, double lo, double hi) { b_clamp(blockIdx.x, gridDim.x, nn, rho, lo, hi); }

// Element e and its image under the point reflection through the cell
// centre, (i,j,k) -> (n-1-i, n-1-j, n-1-k), which is flat index n^3 - 1 - e,
// both take their mean (an odd n leaves the centre element as it is).
__global__ void __launch_bounds__(kBlock) k_sym_central(int64_t nn, double* __restrict__ f) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= nn / 2) return;
    const int64_t p = nn - 1 - e;
    const double v = 0.5 * (f[e] + f[p]);
    f[e] = v;
    f[p] = v;
}

__global__ void k_fill_u32(unsigned* p, int count, unsigned v) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = v;
}


// ---------------------------------------------------------------- finalize
// One block: sums the per-block partials of the kernel just before it (fixed
// order, so results are reproducible for a fixed launch shape) and updates
// the device scalars.  The kernel boundary makes the producer's partial
// stores visible, so producers need no device-scope fences.
template <int NV>
__device__ __forceinline__ void fin_sums(const double* partials, int nblocks, double* tot) {
    final_sums<NV, 4>(partials, nblocks, tot);
}

// The OC candidates' sums (31 per block, slot-major): lane i of each 32-lane
// group reads value i, so a wave reads two blocks' rows contiguously; the
// groups' results are added in group order (fixed order).
__device__ __forceinline__ void fin_sums_oc(const double* partials, int nblocks, double* tot) {
    static_assert(kOcCands <= 32, "one lane per candidate");
    constexpr int G = kBlock / 32;
    __shared__ double sh[G][32];
    const int g = threadIdx.x / 32, i = threadIdx.x % 32;
    double v = 0.0;
    if (i < kOcCands) {
        // four blocks' loads in flight before their additions (in block order)
        for (int b0 = g; b0 < nblocks; b0 += 4 * G) {
            double t[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int b = b0 + u * G;
                t[u] = b < nblocks ? partials[(size_t)b * kOcCands + i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) v += t[u];
        }
    }
    sh[g][i] = v;
    __syncthreads();
    if (threadIdx.x < kOcCands) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) s += sh[q][threadIdx.x];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
}

// Step of the fused iteration from the current residual's r.z (rz) and the
// pending direction's p.q, q.D^-1 q (stored) and q.z (qz):
// alpha = rz / pq; the next r.z follows from expanding (r - alpha q)^T D^-1 (r - alpha q).
__device__ __forceinline__ void fused_step(Scalars* sc, int l, double rz, double qz) {
    const double pq = sc->pq[l];
    const double a = (pq > 0.0) ? rz / pq : 0.0;
    const double rz_next = rz - 2.0 * a * qz + a * a * sc->qdq[l];
    sc->rz[l] = rz;
    sc->alpha[l] = a;
    sc->beta[l] = (rz > 0.0 && rz_next > 0.0) ? rz_next / rz : 0.0;
}

__device__ __forceinline__ void b_finalize(int op, int nblocks, const double* __restrict__ partials, Scalars* sc,
                                           int64_t nn, double eta) {
    __shared__ double tot[kMaxReduce];
    if (op == FIN_OC && sc->oc_done) return;  // passes after convergence are empty
    switch (op) {
        case FIN_FILTER_SIMP: fin_sums<2>(partials, nblocks, tot); break;
        case FIN_SETUP:
        case FIN_PQ:
        case FIN_SUM3_X:
        case FIN_SUM3_B: fin_sums<3>(partials, nblocks, tot); break;
        case FIN_RES_START:
        case FIN_RES_REFRESH: fin_sums<9>(partials, nblocks, tot); break;
        case FIN_UPDATE:
        case FIN_ENERGY: fin_sums<6>(partials, nblocks, tot); break;
        case FIN_OC: fin_sums_oc(partials, nblocks, tot); break;
        case FIN_F_START:
        case FIN_F_REFRESH: fin_sums<12>(partials, nblocks, tot); break;
        case FIN_GUESS: fin_sums<6>(partials, nblocks, tot); break;
        case FIN_MG_RZ0:
        case FIN_MG_RZ: fin_sums<3>(partials, nblocks, tot); break;
        case FIN_MG_UPDATE: fin_sums<6>(partials, nblocks, tot); break;
        default: return;
    }
    if (op == FIN_OC) {
        // walk the candidate tree with the sequential stopping rule (width
        // <= 1e-13 (l1 + l2), 200 halvings), then the next pass's candidates
        __shared__ double sl[2];
        __shared__ int sdone;
        if (threadIdx.x == 0) {
            double l1 = sc->l1, l2 = sc->l2;
            int steps = sc->oc_steps;
            int node = 0;
            int done = 0;
            for (int lev = 0; lev < kOcLevels; ++lev) {
                if (steps >= 200 || (l2 - l1) <= 1e-13 * (l1 + l2)) {
                    done = 1;
                    break;
                }
                const double mid = sc->cand[node];
                const double vol = tot[node] / (double)nn;
                if (vol > sc->vstar_n / (double)nn) {
                    l1 = mid;
                    node = 2 * node + 2;
                } else {
                    l2 = mid;
                    node = 2 * node + 1;
                }
                ++steps;
            }
            if (!done && (steps >= 200 || (l2 - l1) <= 1e-13 * (l1 + l2))) done = 1;
            sc->l1 = l1;
            sc->l2 = l2;
            sc->oc_steps = steps;
            sc->lam = 0.5 * (l1 + l2);
            if (done) sc->oc_done = 1;
            sl[0] = l1;
            sl[1] = l2;
            sdone = done;
        }
        __syncthreads();
        if (!sdone) oc_candidates_lane(sc, sl[0], sl[1], eta);
        return;
    }
    if (threadIdx.x != 0) return;
    switch (op) {
        case FIN_FILTER_SIMP:
            sc->sum_rho = tot[0];
            sc->sum_rhofp = tot[1];
            break;
        case FIN_SETUP:
        case FIN_SUM3_B:
            for (int l = 0; l < 3; ++l) sc->bsum[l] = tot[l];
            break;
        case FIN_SUM3_X:
            for (int l = 0; l < 3; ++l) sc->xsum[l] = tot[l];
            break;
        case FIN_RES_START:
        case FIN_RES_REFRESH:
            for (int l = 0; l < 3; ++l) {
                const double rr = tot[l], rz = tot[3 + l], bb = tot[6 + l];
                sc->rr_true[l] = rr;
                sc->rr[l] = rr;
                sc->bb[l] = bb;
                const bool need = (bb > 0.0) && (rr > sc->tol2 * bb);
                if (op == FIN_RES_START) {
                    sc->active[l] = need ? 1 : 0;
                    sc->beta[l] = 0.0;
                    sc->rz[l] = rz;
                    sc->rz_prev[l] = rz;
                } else if (sc->active[l]) {
                    sc->beta[l] = (sc->rz_prev[l] > 0.0) ? rz / sc->rz_prev[l] : 0.0;
                    sc->rz[l] = rz;
                } else if (need) {
                    sc->active[l] = 1;
                    sc->beta[l] = 0.0;
                    sc->rz[l] = rz;
                    sc->rz_prev[l] = rz;
                }
            }
            break;
        case FIN_PQ:
            for (int l = 0; l < 3; ++l) {
                if (!sc->active[l]) continue;
                sc->pq[l] = tot[l];
                sc->alpha[l] = (tot[l] > 0.0) ? sc->rz[l] / tot[l] : 0.0;
            }
            break;
        case FIN_UPDATE:
            for (int l = 0; l < 3; ++l) {
                if (!sc->active[l]) continue;
                const double rz_new = tot[l], rr = tot[3 + l];
                sc->rz_prev[l] = sc->rz[l];
                sc->beta[l] = (sc->rz[l] > 0.0) ? rz_new / sc->rz[l] : 0.0;
                sc->rz[l] = rz_new;
                sc->rr[l] = rr;
                sc->iters[l] += 1;
                if (!(rr > sc->tol2 * sc->bb[l])) sc->active[l] = 0;
            }
            break;
        case FIN_ENERGY:
            for (int c = 0; c < 6; ++c) sc->kappa_sum[c] = tot[c];
            break;
        case FIN_F_START:
        case FIN_F_REFRESH:
            // sums: [l] r.r (float64), [3+l] r.D^-1 r, [6+l] b.b, [9+l] q.D^-1 r
            for (int l = 0; l < 3; ++l) {
                const double rr = tot[l], rz = tot[3 + l], bb = tot[6 + l], qz = tot[9 + l];
                sc->rr_true[l] = rr;
                sc->rr[l] = rr;
                sc->bb[l] = bb;
                const bool need = (bb > 0.0) && (rr > sc->tol2 * bb);
                if (!need) {
                    sc->active[l] = 0;
                    sc->alpha[l] = 0.0;
                    sc->beta[l] = 0.0;
                } else if (op == FIN_F_REFRESH && sc->active[l] && sc->alpha[l] != 0.0) {
                    // keep the pending step p, q; re-derive it from the new residual
                    fused_step(sc, l, rz, qz);
                } else {
                    // (re)start: the next pass takes p = D^-1 r and no step
                    sc->active[l] = 1;
                    sc->alpha[l] = 0.0;
                    sc->beta[l] = 0.0;
                    sc->rz[l] = rz;
                }
            }
            break;
        case FIN_MG_RZ0:
        case FIN_MG_RZ:
            // z = M^-1 r from the V-cycle; rz_prev holds the previous r.z of
            // this preconditioner only (the residual kernels' r.D^-1 r goes to rz)
            for (int l = 0; l < 3; ++l) {
                if (!sc->active[l]) continue;
                const double rz = tot[l];
                sc->beta[l] = (op == FIN_MG_RZ && sc->rz_prev[l] > 0.0) ? rz / sc->rz_prev[l] : 0.0;
                sc->rz_prev[l] = rz;
                sc->rz[l] = rz;
            }
            break;
        case FIN_MG_UPDATE:
            // update with D^-1 := 1: sums [l] r.r, [3+l] r.r
            for (int l = 0; l < 3; ++l) {
                if (!sc->active[l]) continue;
                sc->rr[l] = tot[3 + l];
                sc->iters[l] += 1;
                if (!(tot[3 + l] > sc->tol2 * sc->bb[l])) sc->active[l] = 0;
            }
            break;
        case FIN_GUESS:
            for (int l = 0; l < 3; ++l) {
                const double bx = tot[l], xax = tot[3 + l];
                const double g = (bx > 0.0 && xax > 0.0) ? bx / xax : 0.0;
                sc->gscale[l] = (isfinite(g) && g > 0.0) ? g : 0.0;
            }
            break;
        default: break;
    }
}

__global__ void __launch_bounds__(kBlock) k_finalize(int op, int nblocks, const double* __restrict__ partials,
                                                     Scalars* sc, int64_t nn, double eta) {
    b_finalize(op, nblocks, partials, sc, nn, eta);
}

void launch_finalize(int op, int nblocks, const Workspace& ws, hipStream_t s, int64_t nn, double eta) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, op, nblocks, ws.partials, ws.sc, nn, eta);
}

// Start guess along its own direction, per load: b.x and x.A x with the
// float64 operator.  The energy 1/2 (s x)^T A (s x) - b^T (s x) is minimal at
// s = b.x / x.A x, where it is -(b.x)^2 / (2 x.A x) < 0, the energy of x = 0:
// the scaled guess is never farther from the solution in the A-norm than zero.
__global__ void __launch_bounds__(kBlock) k_guess_dots(int n, const double* __restrict__ k,
                                                       const double* __restrict__ b, const double* __restrict__ x,
                                                       double* partials) {
    const int64_t nn = (int64_t)n * n * n;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < nn; v += (int64_t)gridDim.x * kBlock) {
        int i, j, kk;
        node_ijk(v, n, i, j, kk);
        const Nbr o = nbr_of(i, j, kk, n);
        double ko[8];
        load_k8(k, o, ko);
        NodeCoef<double> c;
        node_coefs(ko, c);
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const double xv = x[l * nn + v];
            acc[l] += b[l * nn + v] * xv;
            acc[3 + l] += xv * stencil_node<double, double>(c, o, x + l * nn);
        }
    }
    block_partials<6>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_scale3(int64_t nn, double* __restrict__ x, const Scalars* __restrict__ sc) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= nn) return;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        // a load whose guess is unusable (factor 0) starts from zero, also
        // where the guess holds non-finite values
        const double g = sc->gscale[l];
        x[l * nn + v] = (g != 0.0) ? x[l * nn + v] * g : 0.0;
    }
}

// ---------------------------------------------------------------- launchers

static inline int64_t cube(int n) { return (int64_t)n * n * n; }

// Z-march form of the filter for reach 1 (radius in (1, 2], the default 1.5):
// a block owns a column of 32 x 8 elements and marches tz planes in z.  Each
// incoming plane (with a one-element periodic halo in x and y) goes to a
// two-slot LDS ring; the thread filters it in x then y (the same order and
// weights as filter_at), keeps the last three such values in registers, and
// finishes element plane P-1 from planes P-2, P-1, P.  SIMP: also k, k32 and
// the sums of rho and rho~^p.
constexpr int kFzX = 32, kFzY = 8, kFzPX = kFzX + 2, kFzPY = kFzY + 2;
constexpr int kFzHalo = 2 * kFzPX + 2 * kFzY;

struct FzShape {
    int ntx, nty, tz, blocks;
};

static FzShape fz_shape(int n, int max_blocks) {
    FzShape f;
    f.ntx = (n + kFzX - 1) / kFzX;
    f.nty = (n + kFzY - 1) / kFzY;
    const int cols = f.ntx * f.nty;
    int nz = (n + 7) / 8;
    if ((int64_t)cols * nz > max_blocks) nz = max_blocks / cols > 0 ? max_blocks / cols : 1;
    f.tz = (n + nz - 1) / nz;
    f.blocks = cols * ((n + f.tz - 1) / f.tz);
    return f;
}

template <bool SIMP>
__global__ void __launch_bounds__(kBlock) k_filter_zm(int n, int tz, int ntx, int nty, double w0, double w1,
                                                      double w2, const double* __restrict__ in,
                                                      double* __restrict__ out, double* __restrict__ kout,
                                                      float* __restrict__ k32, double k0, double kmin, double p,
                                                      double* __restrict__ partials) {
    static_assert(kFzX * kFzY == kBlock && kFzHalo <= kBlock, "tile");
    __shared__ double sp[2][kFzPY * kFzPX];
    int bid = xcd_tile(blockIdx.x, gridDim.x);
    const int bx = bid % ntx;
    bid /= ntx;
    const int by = bid % nty;
    const int bz = bid / nty;
    const int i0 = bx * kFzX, j0 = by * kFzY, z0 = bz * tz, z1 = min(z0 + tz, n);
    const int tx = threadIdx.x % kFzX, ty = threadIdx.x / kFzX;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = i < n && j < n;
    const int64_t n2 = (int64_t)n * n;
    // every interior cell is loaded (periodically wrapped) so that the own
    // elements next to a partial tile's edge read correct neighbours
    const int64_t xy_in = (int64_t)(i % n) + (int64_t)n * (j % n);
    const int l_in = (ty + 1) * kFzPX + tx + 1;
    const int tid = threadIdx.x;
    const bool has_h = tid < kFzHalo;
    int64_t xy_h = 0;
    int l_h = 0;
    if (has_h) {
        int px, py;
        if (tid < kFzPX) {
            px = tid;
            py = 0;
        } else if (tid < 2 * kFzPX) {
            px = tid - kFzPX;
            py = kFzPY - 1;
        } else if (tid < 2 * kFzPX + kFzY) {
            px = 0;
            py = 1 + tid - 2 * kFzPX;
        } else {
            px = kFzPX - 1;
            py = 1 + tid - 2 * kFzPX - kFzY;
        }
        const int gi = ((i0 - 1 + px) % n + n) % n, gj = ((j0 - 1 + py) % n + n) % n;
        xy_h = (int64_t)gi + (int64_t)n * gj;
        l_h = py * kFzPX + px;
    }
    double f_m2 = 0.0, f_m1 = 0.0, own_m1 = 0.0;
    double acc[2] = {0.0, 0.0};
    for (int P = z0 - 1; P <= z1; ++P) {
        const int pw = P < 0 ? P + n : (P >= n ? P - n : P);
        const double* pl = in + (int64_t)pw * n2;
        const int slot = P & 1;
        const double vin = pl[xy_in];
        sp[slot][l_in] = vin;
        if (has_h) sp[slot][l_h] = pl[xy_h];
        __syncthreads();
        const double* L = sp[slot];
        double fy = 0.0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const double* row = L + l_in + dy * kFzPX;
            double fx = 0.0;
            fx += w0 * row[-1];
            fx += w1 * row[0];
            fx += w2 * row[1];
            fy += (dy < 0 ? w0 : (dy == 0 ? w1 : w2)) * fx;
        }
        if (P - 1 >= z0 && own) {
            double v = 0.0;
            v += w0 * f_m2;
            v += w1 * f_m1;
            v += w2 * fy;
            const int64_t e = (int64_t)(P - 1) * n2 + xy_in;
            out[e] = v;
            if (SIMP) {
                const double rp = (p == 3.0) ? v * v * v : pow(v, p);
                const double ke = kmin + rp * (k0 - kmin);
                kout[e] = ke;
                if (k32) k32[e] = (float)ke;
                acc[0] += own_m1;
                acc[1] += rp;
            }
        }
        f_m2 = f_m1;
        f_m1 = fy;
        own_m1 = vin;
    }
    if (SIMP) block_partials<2>(acc, partials);
}

void launch_filter_simp(int n, double r, const double* rho, double* rhof, double* k, float* k32, double k0,
                        double kmin, double p, const Workspace& ws, hipStream_t s) {
    const FilterW fw = filter_weights(r);
    if (fw.R == 1) {
        const FzShape z = fz_shape(n, ws.max_blocks);
        hipLaunchKernelGGL(k_filter_zm<true>, dim3(z.blocks), dim3(kBlock), 0, s, n, z.tz, z.ntx, z.nty, fw.w[0],
                           fw.w[1], fw.w[2], rho, rhof, k, k32, k0, kmin, p, ws.partials);
        launch_finalize(FIN_FILTER_SIMP, z.blocks, ws, s);
        return;
    }
    const int g = grid_for(cube(n), ws.max_blocks);
    hipLaunchKernelGGL(k_filter_simp, dim3(g), dim3(kBlock), 0, s, n, filter_weights(r), rho, rhof, k, k32, k0, kmin,
                       p, ws.partials, ws.counter, ws.sc);
    launch_finalize(FIN_FILTER_SIMP, g, ws, s);
}

void launch_filter(int n, double r, const double* in, double* out, hipStream_t s) {
    const FilterW fw = filter_weights(r);
    if (fw.R == 1) {
        const FzShape z = fz_shape(n, kMaxBlocks);
        hipLaunchKernelGGL(k_filter_zm<false>, dim3(z.blocks), dim3(kBlock), 0, s, n, z.tz, z.ntx, z.nty, fw.w[0],
                           fw.w[1], fw.w[2], in, out, nullptr, nullptr, 0.0, 0.0, 0.0, nullptr);
        return;
    }
    hipLaunchKernelGGL(k_filter, dim3(nblocks_for(cube(n))), dim3(kBlock), 0, s, n, fw, in, out);
}

void launch_setup_nodes(int n, const double* k, double* b, double* dinv, float* dinv32, const Workspace& ws,
                        hipStream_t s) {
    const int g = grid_for(cube(n), ws.max_blocks);
    hipLaunchKernelGGL(k_setup_nodes, dim3(g), dim3(kBlock), 0, s, n, k, b, dinv, dinv32, ws.partials, ws.counter,
                       ws.sc);
    launch_finalize(FIN_SETUP, g, ws, s);
}

template <typename T>
void launch_dir(int n, const T* r, const T* dinv, const T* p_old, T* p_new, const Workspace& ws, hipStream_t s) {
    hipLaunchKernelGGL(k_dir<T>, dim3(nblocks_for(cube(n))), dim3(kBlock), 0, s, n, r, dinv, p_old, p_new, ws.sc);
}

template <typename T>
void launch_apply_pq(int n, const T* k, const T* p, T* q, const Workspace& ws, hipStream_t s) {
    const int g = grid_for(cube(n), ws.max_blocks);
    hipLaunchKernelGGL(k_apply_pq<T>, dim3(g), dim3(kBlock), 0, s, n, k, p, q, ws.partials, ws.counter, ws.sc);
    launch_finalize(FIN_PQ, g, ws, s);
}

template <typename T>
void launch_update(int n, T* x, T* r, const T* p, const T* q, const T* dinv, const Workspace& ws, hipStream_t s) {
    const int g = grid_for(cube(n), ws.max_blocks);
    hipLaunchKernelGGL(k_update<T>, dim3(g), dim3(kBlock), 0, s, n, x, r, p, q, dinv, ws.partials, ws.counter, ws.sc);
    launch_finalize(FIN_UPDATE, g, ws, s);
}

template <typename TR>
void launch_residual(int n, const double* k, const double* b, const double* x, TR* r, TR* p_old, const TR* dinv,
                          int mode, int x_zero, const Workspace& ws, hipStream_t s) {
    const int g = grid_for(cube(n), ws.max_blocks);
    hipLaunchKernelGGL(k_residual<TR>, dim3(g), dim3(kBlock), 0, s, n, k, b, x, r, p_old, dinv, mode, x_zero,
                       ws.partials, ws.counter, ws.sc);
    launch_finalize(mode == RES_START ? FIN_RES_START : FIN_RES_REFRESH, g, ws, s);
}

void launch_accumulate(int n, double* x, float* x32, hipStream_t s) {
    const int64_t cnt = 3 * cube(n);
    hipLaunchKernelGGL(k_accumulate, dim3(nblocks_for(cnt)), dim3(kBlock), 0, s, cnt, x, x32);
}

void launch_sum3(int n, const double* x, int slot, const Workspace& ws, hipStream_t s) {
    const int g = grid_for(cube(n), ws.max_blocks);
    hipLaunchKernelGGL(k_sum3, dim3(g), dim3(kBlock), 0, s, n, x, slot, ws.partials, ws.counter, ws.sc);
    launch_finalize(slot == 0 ? FIN_SUM3_X : FIN_SUM3_B, g, ws, s);
}

void launch_sub_mean3(int n, double* x, int slot, const Workspace& ws, hipStream_t s) {
    hipLaunchKernelGGL(k_sub_mean3, dim3(nblocks_for(cube(n))), dim3(kBlock), 0, s, n, x, slot, ws.sc);
}

void launch_guess_scale(int n, const double* k, const double* b, double* x, const Workspace& ws, hipStream_t s) {
    const int64_t nn = cube(n);
    const int g = grid_for(nn, ws.max_blocks);
    hipLaunchKernelGGL(k_guess_dots, dim3(g), dim3(kBlock), 0, s, n, k, b, x, ws.partials);
    launch_finalize(FIN_GUESS, g, ws, s);
    hipLaunchKernelGGL(k_scale3, dim3(nblocks_for(nn)), dim3(kBlock), 0, s, nn, x, ws.sc);
}

void launch_energy(int n, const double* k, const double* chi, const Workspace& ws, hipStream_t s) {
    const int g = grid_for(cube(n), ws.max_blocks);
    hipLaunchKernelGGL(k_energy, dim3(g), dim3(kBlock), 0, s, n, k, chi, ws.partials, ws.counter, ws.sc);
    launch_finalize(FIN_ENERGY, g, ws, s);
}

void launch_sens(int n, const double* rhof, const double* chi, const double* w6, double k0, double kmin, double p,
                 double* st, hipStream_t s) {
    W6 w;
    for (int c = 0; c < 6; ++c) w.w[c] = w6[c];
    hipLaunchKernelGGL(k_sens, dim3(nblocks_for(cube(n))), dim3(kBlock), 0, s, n, rhof, chi, w, k0, kmin, p, st);
}

void launch_oc_prepare(int n, const double* rho, const double* sens, double eta, double move, double rho_min,
                       double* q, const Workspace& ws, hipStream_t s, int* nblocks_out) {
    const int g = grid_for(cube(n), ws.max_blocks < 1024 ? ws.max_blocks : 1024);
    hipLaunchKernelGGL(k_oc_prepare_max, dim3(g), dim3(kBlock), 0, s, cube(n), rho, sens, eta, move, rho_min, q,
                       ws.partials);
    *nblocks_out = g;
}

void launch_oc_init(double vstar, int n, double eta, int prep_blocks, const Workspace& ws, hipStream_t s) {
    hipLaunchKernelGGL(k_oc_init, dim3(1), dim3(kBlock), 0, s, ws.sc, vstar * (double)cube(n), eta, ws.partials,
                       prep_blocks);
}

void launch_oc_pass(int n, const double* rho, const double* q, double move, double rho_min, double eta,
                        const Workspace& ws, hipStream_t s) {
    // 512 blocks: a short 31 x 512 reduction in the finalize
    const int g = grid_for(cube(n), ws.max_blocks < 512 ? ws.max_blocks : 512);
    hipLaunchKernelGGL(k_oc_pass, dim3(g), dim3(kBlock), 0, s, cube(n), rho, q, move, rho_min, eta, ws.partials,
                       ws.counter, ws.sc);
    launch_finalize(FIN_OC, g, ws, s, cube(n), eta);
}

void launch_oc_apply(int n, double* rho, const double* q, double eta, double move, double rho_min,
                     const Workspace& ws, hipStream_t s) {
    hipLaunchKernelGGL(k_oc_apply, dim3(nblocks_for(cube(n))), dim3(kBlock), 0, s, cube(n), rho, q, eta, move,
                       rho_min, ws.sc);
}

void launch_oc_from_sens(int n, const double* rho, const double* sens, double* rho_out, double* lambda_out,
                         double vstar, double eta, double move, double rho_min, const Workspace& ws,
                         hipStream_t s) {
    int prep_blocks = 0;
    launch_oc_prepare(n, rho, sens, eta, move, rho_min, nullptr, ws, s, &prep_blocks);
    launch_oc_init(vstar, n, eta, prep_blocks, ws, s);
    const int g = grid_for(cube(n), ws.max_blocks < 512 ? ws.max_blocks : 512);
    // every pass the bisection could need; passes after it has stopped return at once
    for (int pass = 0; pass < kOcMaxPasses; ++pass) {
        hipLaunchKernelGGL(k_oc_pass_s, dim3(g), dim3(kBlock), 0, s, cube(n), rho, sens, move, rho_min, eta,
                           ws.partials, ws.sc);
        launch_finalize(FIN_OC, g, ws, s, cube(n), eta);
    }
    hipLaunchKernelGGL(k_oc_apply_s, dim3(grid_for(cube(n), 2048)), dim3(kBlock), 0, s, cube(n), rho, sens, rho_out,
                       lambda_out, eta, move, rho_min, (const Scalars*)ws.sc);
}

void launch_sym_central(int n, double* f, hipStream_t s) {
    const int64_t nn = cube(n);
    if (nn < 2) return;
    hipLaunchKernelGGL(k_sym_central, dim3(nblocks_for(nn / 2)), dim3(kBlock), 0, s, nn, f);
}

void launch_clamp(int n, double* rho, double lo, double hi, hipStream_t s) {
    hipLaunchKernelGGL(k_clamp, dim3(nblocks_for(cube(n))), dim3(kBlock), 0, s, cube(n), rho, lo, hi);
}

template <typename T>
void launch_apply(int n, const T* k, const T* x, T* y, hipStream_t s) {
    hipLaunchKernelGGL(k_apply<T>, dim3(nblocks_for(cube(n))), dim3(kBlock), 0, s, n, k, x, y);
}

void launch_fill_u32(unsigned* p, int count, unsigned v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3((count + 255) / 256), dim3(256), 0, s, p, count, v);
}

template void launch_dir<double>(int, const double*, const double*, const double*, double*, const Workspace&,
                                 hipStream_t);
template void launch_dir<float>(int, const float*, const float*, const float*, float*, const Workspace&, hipStream_t);
template void launch_apply_pq<double>(int, const double*, const double*, double*, const Workspace&, hipStream_t);
template void launch_apply_pq<float>(int, const float*, const float*, float*, const Workspace&, hipStream_t);
template void launch_update<double>(int, double*, double*, const double*, const double*, const double*,
                                    const Workspace&, hipStream_t);
template void launch_update<float>(int, float*, float*, const float*, const float*, const float*, const Workspace&,
                                   hipStream_t);
template void launch_residual<double>(int, const double*, const double*, const double*, double*, double*,
                                           const double*, int, int, const Workspace&, hipStream_t);
template void launch_residual<float>(int, const double*, const double*, const double*, float*, float*,
                                          const float*, int, int, const Workspace&, hipStream_t);
template void launch_apply<double>(int, const double*, const double*, double*, hipStream_t);
template void launch_apply<float>(int, const float*, const float*, float*, hipStream_t);

}  // namespace otm

namespace otm {

__global__ void k_cast_f64_f32(int64_t count, const double* __restrict__ in, float* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < count) out[t] = (float)in[t];
}
__global__ void k_cast_f32_f64(int64_t count, const float* __restrict__ in, double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < count) out[t] = (double)in[t];
}

void launch_cast_f64_f32(int64_t count, const double* in, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_f64_f32, dim3(nblocks_for(count)), dim3(kBlock), 0, s, count, in, out);
}
void launch_cast_f32_f64(int64_t count, const float* in, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_f32_f64, dim3(nblocks_for(count)), dim3(kBlock), 0, s, count, in, out);
}

}  // namespace otm

// ====================================================================== batch
// One launch covers every design of a batch: work item (block) g belongs to
// design t.eb_design[g] and runs the single-design body on that design's
// slices with the design-local block index.  Partial sums land in slot g, so
// the items of design d occupy the contiguous range of its descriptor.
namespace otm {

#define OTM_BATCH_ITEM                                        \
    const int g_ = blockIdx.x;                                \
    const int d_ = t.eb_design[g_];                           \
    const BatchDesc D = t.desc[d_];                           \
    const int lb_ = g_ - D.eb_start;                          \
    const int nb_ = D.eb_count;                               \
    const int64_t o1 = D.off, o3 = 3 * D.off;                 \
    (void)o1;                                                 \
    (void)o3;

// Every design's solver scalars (the fields before sum_rho) cleared and tol^2
// set, in one launch; the reductions stored after them are kept.
constexpr int kSolverWords = (int)(offsetof(Scalars, sum_rho) / sizeof(double));
static_assert(offsetof(Scalars, sum_rho) % sizeof(double) == 0, "solver scalars are whole doubles");
static_assert(offsetof(Scalars, tol2) % sizeof(double) == 0, "tol2 is a double slot");
__global__ void __launch_bounds__(kBlock) kb_reset_solver(Scalars* __restrict__ sc, int count, double tol2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= count * kSolverWords) return;
    const int d = i / kSolverWords, w = i - d * kSolverWords;
    double* p = reinterpret_cast<double*>(sc + d);
    p[w] = (w == (int)(offsetof(Scalars, tol2) / sizeof(double))) ? tol2 : 0.0;
}

__global__ void __launch_bounds__(kBlock) kb_clamp(BatchTab t, double* rho, double lo, double hi) {
    OTM_BATCH_ITEM
    b_clamp(lb_, nb_, (int64_t)D.n * D.n * D.n, rho + o1, lo, hi);
}

__global__ void __launch_bounds__(kBlock) kb_filter_simp(BatchTab t, const double* rho, double* rhof, double* k,
                                                         double* partials, Scalars* sc) {
    OTM_BATCH_ITEM
    // the weights are read from the device table: a local copy indexed with
    // the runtime radius would be placed in scratch memory
    b_filter_simp(lb_, nb_, D.n, t.desc[d_].fw, rho + o1, rhof + o1, k + o1, nullptr, D.k0, D.kmin, D.penal, partials,
                  nullptr, sc + d_);
}

__global__ void __launch_bounds__(kBlock) kb_setup_nodes(BatchTab t, const double* k, double* b, double* dinv,
                                                         double* partials, Scalars* sc) {
    OTM_BATCH_ITEM
    b_setup_nodes(lb_, nb_, D.n, k + o1, b + o3, dinv + o1, nullptr, partials, nullptr, sc + d_);
}

__global__ void __launch_bounds__(kBlock) kb_sum3(BatchTab t, const double* x, int slot, double* partials,
                                                  Scalars* sc) {
    OTM_BATCH_ITEM
    b_sum3(lb_, nb_, D.n, x + o3, slot, partials, nullptr, sc + d_);
}

__global__ void __launch_bounds__(kBlock) kb_sub_mean3(BatchTab t, double* x, int slot, Scalars* sc) {
    OTM_BATCH_ITEM
    b_sub_mean3(lb_, nb_, D.n, x + o3, slot, sc + d_);
}

__global__ void __launch_bounds__(kBlock) kb_residual(BatchTab t, const double* k, const double* b, const double* x,
                                                      double* r, double* p_old, const double* dinv, int mode,
                                                      int x_zero, double* partials, Scalars* sc) {
    OTM_BATCH_ITEM
    b_residual<double>(lb_, nb_, D.n, k + o1, b + o3, x + o3, r + o3, p_old + o3, dinv + o1, mode, x_zero, partials,
                       nullptr, sc + d_);
}

__global__ void __launch_bounds__(kBlock) kb_energy(BatchTab t, const double* k, const double* chi, double* partials,
                                                    Scalars* sc) {
    OTM_BATCH_ITEM
    b_energy(lb_, nb_, D.n, k + o1, chi + o3, partials, nullptr, sc + d_);
}

__global__ void __launch_bounds__(kBlock) kb_sens(BatchTab t, const double* rhof, const double* chi, const W6* w6,
                                                  double* st) {
    OTM_BATCH_ITEM
    b_sens(lb_, nb_, D.n, rhof + o1, chi + o3, w6[d_], D.k0, D.kmin, D.penal, st + o1);
}

__global__ void __launch_bounds__(kBlock) kb_filter(BatchTab t, const double* in, double* out) {
    OTM_BATCH_ITEM
    b_filter(lb_, nb_, D.n, t.desc[d_].fw, in + o1, out + o1);
}

__global__ void __launch_bounds__(kBlock) kb_oc_prepare(BatchTab t, const double* rho, const double* sens, double eta,
                                                        double* q) {
    OTM_BATCH_ITEM
    b_oc_prepare(lb_, nb_, (int64_t)D.n * D.n * D.n, rho + o1, sens + o1, eta, q + o1);
}

__global__ void kb_oc_init(BatchTab t, Scalars* sc, const double* vstar, double eta) {
    const int d = blockIdx.x;
    if (d >= t.count) return;
    const int n = t.desc[d].n;
    Scalars* s = sc + d;
    if (threadIdx.x == 0) {
        s->l1 = 0.0;
        s->l2 = 1e9;
        s->vstar_n = vstar[d] * (double)n * n * n;
        s->oc_steps = 0;
        s->oc_done = 0;
    }
    oc_candidates_lane(s, 0.0, 1e9, eta);
}

// moves[d]: the OC move limit of design d
__global__ void __launch_bounds__(kBlock) kb_oc_pass(BatchTab t, const double* rho, const double* q,
                                                     const double* __restrict__ moves, double rho_min, double eta,
                                                     double* partials, Scalars* sc) {
    OTM_BATCH_ITEM
    b_oc_pass(lb_, nb_, (int64_t)D.n * D.n * D.n, rho + o1, q + o1, moves[d_], rho_min, eta, partials, nullptr,
              sc + d_);
}

__global__ void __launch_bounds__(kBlock) kb_oc_apply(BatchTab t, double* rho, const double* q, double eta,
                                                      const double* __restrict__ moves, double rho_min,
                                                      const Scalars* sc) {
    OTM_BATCH_ITEM
    b_oc_apply(lb_, nb_, (int64_t)D.n * D.n * D.n, rho + o1, q + o1, eta, moves[d_], rho_min, sc + d_);
}

static int fin_width(int op) {
    switch (op) {
        case FIN_FILTER_SIMP: return 2;
        case FIN_RES_START:
        case FIN_RES_REFRESH: return 9;
        case FIN_UPDATE:
        case FIN_ENERGY: return 6;
        case FIN_OC: return kOcCands;
        case FIN_F_START:
        case FIN_F_REFRESH: return 12;
        case FIN_GUESS:
        case FIN_MG_UPDATE: return 6;
        default: return 3;
    }
}

__global__ void __launch_bounds__(kBlock) kb_finalize(BatchTab t, int op, int which_mb, int width,
                                                      const double* partials, Scalars* sc, double eta) {
    const int d = blockIdx.x;
    const BatchDesc D = t.desc[d];
    const int start = which_mb ? D.mb_start : D.eb_start;
    const int cnt = which_mb ? D.mb_count : D.eb_count;
    b_finalize(op, cnt, partials + (size_t)start * width, sc + d, (int64_t)D.n * D.n * D.n, eta);
}

void launch_b_reset_solver(Scalars* sc, int count, double tol2, hipStream_t s) {
    const int threads = count * kSolverWords;
    hipLaunchKernelGGL(kb_reset_solver, dim3((threads + kBlock - 1) / kBlock), dim3(kBlock), 0, s, sc, count, tol2);
}
void launch_b_clamp(const BatchTab& t, double* rho, double lo, double hi, hipStream_t s) {
    hipLaunchKernelGGL(kb_clamp, dim3(t.eb_total), dim3(kBlock), 0, s, t, rho, lo, hi);
}
void launch_b_filter_simp(const BatchTab& t, const double* rho, double* rhof, double* k, double* partials,
                          Scalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(kb_filter_simp, dim3(t.eb_total), dim3(kBlock), 0, s, t, rho, rhof, k, partials, sc);
    launch_b_finalize(t, FIN_FILTER_SIMP, 0, partials, sc, 0.5, s);
}
void launch_b_setup_nodes(const BatchTab& t, const double* k, double* b, double* dinv, double* partials, Scalars* sc,
                          hipStream_t s) {
    hipLaunchKernelGGL(kb_setup_nodes, dim3(t.eb_total), dim3(kBlock), 0, s, t, k, b, dinv, partials, sc);
    launch_b_finalize(t, FIN_SETUP, 0, partials, sc, 0.5, s);
}
void launch_b_sum3(const BatchTab& t, const double* x, int slot, double* partials, Scalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(kb_sum3, dim3(t.eb_total), dim3(kBlock), 0, s, t, x, slot, partials, sc);
    launch_b_finalize(t, slot == 0 ? FIN_SUM3_X : FIN_SUM3_B, 0, partials, sc, 0.5, s);
}
void launch_b_sub_mean3(const BatchTab& t, double* x, int slot, Scalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(kb_sub_mean3, dim3(t.eb_total), dim3(kBlock), 0, s, t, x, slot, sc);
}
void launch_b_residual(const BatchTab& t, const double* k, const double* b, const double* x, double* r, double* p_old,
                       const double* dinv, int mode, int x_zero, double* partials, Scalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(kb_residual, dim3(t.eb_total), dim3(kBlock), 0, s, t, k, b, x, r, p_old, dinv, mode, x_zero,
                       partials, sc);
    launch_b_finalize(t, mode == RES_START ? FIN_RES_START : FIN_RES_REFRESH, 0, partials, sc, 0.5, s);
}
void launch_b_energy(const BatchTab& t, const double* k, const double* chi, double* partials, Scalars* sc,
                     hipStream_t s) {
    hipLaunchKernelGGL(kb_energy, dim3(t.eb_total), dim3(kBlock), 0, s, t, k, chi, partials, sc);
    launch_b_finalize(t, FIN_ENERGY, 0, partials, sc, 0.5, s);
}
void launch_b_sens(const BatchTab& t, const double* rhof, const double* chi, const W6* w6, double* st, hipStream_t s) {
    hipLaunchKernelGGL(kb_sens, dim3(t.eb_total), dim3(kBlock), 0, s, t, rhof, chi, w6, st);
}
void launch_b_filter(const BatchTab& t, const double* in, double* out, hipStream_t s) {
    hipLaunchKernelGGL(kb_filter, dim3(t.eb_total), dim3(kBlock), 0, s, t, in, out);
}
void launch_b_oc_prepare(const BatchTab& t, const double* rho, const double* sens, double eta, double* q,
                         hipStream_t s) {
    hipLaunchKernelGGL(kb_oc_prepare, dim3(t.eb_total), dim3(kBlock), 0, s, t, rho, sens, eta, q);
}
void launch_b_oc_init(const BatchTab& t, Scalars* sc, const double* vstar, double eta, hipStream_t s) {
    hipLaunchKernelGGL(kb_oc_init, dim3(t.count), dim3(64), 0, s, t, sc, vstar, eta);
}
void launch_b_oc_pass(const BatchTab& t, const double* rho, const double* q, const double* moves, double rho_min,
                      double eta, double* partials, Scalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(kb_oc_pass, dim3(t.eb_total), dim3(kBlock), 0, s, t, rho, q, moves, rho_min, eta, partials, sc);
    launch_b_finalize(t, FIN_OC, 0, partials, sc, eta, s);
}
void launch_b_oc_apply(const BatchTab& t, double* rho, const double* q, double eta, const double* moves,
                       double rho_min, Scalars* sc, hipStream_t s) {
    hipLaunchKernelGGL(kb_oc_apply, dim3(t.eb_total), dim3(kBlock), 0, s, t, rho, q, eta, moves, rho_min, sc);
}
void launch_b_finalize(const BatchTab& t, int op, int which_mb, double* partials, Scalars* sc, double eta,
                       hipStream_t s) {
    hipLaunchKernelGGL(kb_finalize, dim3(t.count), dim3(kBlock), 0, s, t, op, which_mb, fin_width(op), partials, sc,
                       eta);
}

}  // namespace otm
