// Device-side helpers shared by the kernel translation units: periodic
// wrap, deterministic block reductions with a last-block epilogue, and the
// node-centric hex-8 conduction stencil.
#pragma once

#include "otm_internal.h"

namespace otm {

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

template <int NV>
__device__ __forceinline__ void wave_reduce(double (&v)[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
    }
}

constexpr int pow2_up(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// One step of the transposed wave reduction: lanes whose bit O is set keep
// the upper half of the C values and send the lower half to their partner
// (lane ^ O), which keeps the lower half; both add what they receive.  idx
// collects the kept halves' bits.  With one value left, plain butterfly steps
// finish the sum over the remaining lane bits.
template <int C, int O>
__device__ __forceinline__ void spread_step(double* a, int lane, int& idx) {
    if constexpr (C > 1 && O > 0) {
        constexpr int H = C / 2;
        const bool hi = (lane & O) != 0;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const double send = hi ? a[j] : a[j + H];
            const double keep = hi ? a[j + H] : a[j];
            a[j] = keep + __shfl_xor(send, O, 64);
        }
        idx = 2 * idx + (hi ? 1 : 0);
        spread_step<H, O / 2>(a, lane, idx);
    } else if constexpr (O > 0) {
        a[0] += __shfl_xor(a[0], O, 64);
        spread_step<C, O / 2>(a, lane, idx);
    }
}

// Wave sums of NV values at about NV cross-lane moves instead of 6 NV: on
// return every lane holds in a[0] the wave total of value idx (lanes that
// differ only in their low log2(64 / P) bits hold the same one; P = NV rounded
// up to a power of two).  Fixed order: deterministic.
template <int NV>
__device__ __forceinline__ double wave_reduce_spread(const double (&v)[NV], int& idx) {
    constexpr int P = pow2_up(NV);
    static_assert(P <= 64, "at most 64 values");
    double a[P];
#pragma unroll
    for (int i = 0; i < P; ++i) a[i] = i < NV ? v[i] : 0.0;
    idx = 0;
    spread_step<P, 32>(a, threadIdx.x & 63, idx);
    return a[0];
}

// Block-level sum of NV values; threads 0..NV-1 write partials[slot*NV + t]
// (slot = blockIdx.x unless a persistent block processes several work items).
// Uses a fixed reduction order (deterministic for a fixed launch shape).
template <int NV>
__device__ __forceinline__ void block_partials_at(double (&v)[NV], double* partials, int slot) {
    __shared__ double sh[NV][kBlock / 64];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    int idx;
    const double t = wave_reduce_spread<NV>(v, idx);
    if ((lane & (64 / pow2_up(NV) - 1)) == 0 && idx < NV) sh[idx][w] = t;
    __syncthreads();
    if (tid < NV) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < kBlock / 64; ++j) s += sh[tid][j];
        partials[(size_t)slot * NV + tid] = s;
    }
    __syncthreads();
}

template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* partials) {
    block_partials_at<NV>(v, partials, blockIdx.x);
}

// Value-major variant: value i of slot b at partials[i * kMaxBlocks + b], so
// the one-block sum below reads each value with coalesced loads.
template <int NV>
__device__ __forceinline__ void block_partials_vm(double (&v)[NV], double* partials, int slot) {
    __shared__ double sh[NV][kBlock / 64];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    int idx;
    const double t = wave_reduce_spread<NV>(v, idx);
    if ((lane & (64 / pow2_up(NV) - 1)) == 0 && idx < NV) sh[idx][w] = t;
    __syncthreads();
    if (tid < NV) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < kBlock / 64; ++j) s += sh[tid][j];
        partials[(size_t)tid * kMaxBlocks + slot] = s;
    }
    __syncthreads();
}

// Sum the value-major partials of nblocks blocks (value i of block b at
// partials[i * kMaxBlocks + b]) -> out[NV] in shared memory.  Wave w takes
// values w, w + nwaves, ...: lane j adds blocks j, j + 64, j + 128, ... in
// that order (eight loads in flight before their additions), then the 64
// lane sums meet in a fixed xor butterfly.  The order depends on nblocks
// only, so every block size gives the same bits; with at least NV waves
// (the finalize kernels run 16) each value costs one round of loads.  The
// loop body runs only for lane < nblocks, so nblocks - 1 is a valid index.
template <int NV>
__device__ __forceinline__ void final_sums_vm(const double* partials, int nblocks, double* out /* shared */) {
    const int lane = threadIdx.x & 63, nw = (int)blockDim.x >> 6;
    for (int i = (int)threadIdx.x >> 6; i < NV; i += nw) {
        const double* src = partials + (size_t)i * kMaxBlocks;
        double s = 0.0;
        for (int b0 = lane; b0 < nblocks; b0 += 8 * 64) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {  // unconditional loads (clamped index), then a select
                const int b = b0 + 64 * u;
                const double x = src[b < nblocks ? b : nblocks - 1];
                t[u] = b < nblocks ? x : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) s += t[u];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) out[i] = s;
    }
    __syncthreads();
}

// Sum the partial arrays of all blocks (fixed order) -> out[NV] in shared memory.
// U: slots per thread whose loads are all issued before the first addition
// (the additions keep the slot order b = tid, tid + blockDim, ...).
template <int NV, int U = 1>
__device__ __forceinline__ void final_sums(const double* partials, int nblocks, double* out /* shared */) {
    double v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = 0.0;
    for (int b0 = threadIdx.x; b0 < nblocks; b0 += U * blockDim.x) {
        double t[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * (int)blockDim.x;
#pragma unroll
            for (int i = 0; i < NV; ++i) t[u][i] = b < nblocks ? partials[(size_t)b * NV + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < NV; ++i) v[i] += t[u][i];
    }
    __shared__ double sh[NV][kBlock / 64];
    wave_reduce<NV>(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[i][w] = v[i];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < kBlock / 64; ++j) s += sh[threadIdx.x][j];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Global access at a block-uniform base plus a per-thread 32-bit byte offset:
// the base stays in scalar registers and the address needs no 64-bit vector
// arithmetic (the offsets of one plane stay far below 4 GiB).
// (The empty asm keeps the offset a 32-bit value at the access, so the
// compiler does not hoist its widening out of the march loop.)
template <typename V>
__device__ __forceinline__ V ld_at(const void* base, uint32_t boff) {
    asm volatile("" : "+v"(boff));
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + boff);
}
template <typename V>
__device__ __forceinline__ void st_at(void* base, uint32_t boff, V v) {
    asm volatile("" : "+v"(boff));
    *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + boff) = v;
}

// Workgroups of a launch are dispatched round-robin over the 8 XCDs, each
// with its own L2.  This bijection gives every XCD a contiguous range of tile
// ids, so neighbouring tiles (whose halos overlap) share one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    const int q = nb / kXcds, r = nb % kXcds;
    const int x = bid % kXcds, k = bid / kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Bookkeeping of the fused iteration after a pass.  in: the state the pass
// ran with; tot: its reduced sums, per load [l] p.q, [3+l] q.z, [6+l] q.D^-1 q,
// [9+l] r.z, [12+l] r.r.  out: the state of the next pass.  alpha = r.z / p.q;
// beta = (next r.z) / r.z with the next r.z expanded as
// r.z - 2 alpha q.z + alpha^2 q.D^-1 q.  A load whose r.r meets tol^2 b.b stops.
__device__ inline void fused_advance(const FusedState& in, const double* tot, FusedState& out) {
    out = in;
    for (int l = 0; l < 3; ++l) {
        if (!in.active[l]) {
            out.alpha[l] = 0.0;
            out.beta[l] = 0.0;
            continue;
        }
        if (in.alpha[l] != 0.0) out.iters[l] += 1;
        const double rr = tot[12 + l];
        out.rr[l] = rr;
        if (!(rr > in.tol2 * in.bb[l])) {
            out.active[l] = 0;
            out.alpha[l] = 0.0;
            out.beta[l] = 0.0;
            continue;
        }
        const double pq = tot[l], qz = tot[3 + l], qdq = tot[6 + l], rz = tot[9 + l];
        const double a = (pq > 0.0) ? rz / pq : 0.0;
        const double rz_next = rz - 2.0 * a * qz + a * a * qdq;
        out.rz[l] = rz;
        out.pq[l] = pq;
        out.qdq[l] = qdq;
        out.alpha[l] = a;
        out.beta[l] = (rz > 0.0 && rz_next > 0.0) ? rz_next / rz : 0.0;
    }
}

// The fused state held in the scalar block (after a residual or a finalize).
__device__ inline void fused_state_of(const Scalars* sc, FusedState& s) {
    for (int l = 0; l < 3; ++l) {
        s.alpha[l] = sc->alpha[l];
        s.beta[l] = sc->beta[l];
        s.rz[l] = sc->rz[l];
        s.pq[l] = sc->pq[l];
        s.qdq[l] = sc->qdq[l];
        s.rr[l] = sc->rr[l];
        s.bb[l] = sc->bb[l];
        s.active[l] = sc->active[l];
        s.iters[l] = sc->iters[l];
    }
    s.tol2 = sc->tol2;
}

// (i, j, k) of flat index v = i + n (j + n k) with 32-bit arithmetic (n^3 < 2^31
// for n <= 1024): a 64-bit division is a long emulated sequence on the GPU.
__device__ __forceinline__ void node_ijk(int64_t v, int n, int& i, int& j, int& k) {
    const uint32_t u = (uint32_t)v, un = (uint32_t)n;
    const uint32_t q = u / un;
    i = (int)(u - q * un);
    const uint32_t q2 = q / un;
    j = (int)(q - q2 * un);
    k = (int)q2;
}

static inline int nblocks_for(int64_t count) { return (int)((count + kBlock - 1) / kBlock); }

// Clamp grid size for grid-stride reductions so partial arrays stay small.
static inline int grid_for(int64_t count, int max_blocks) {
    int g = nblocks_for(count);
    return g > max_blocks ? max_blocks : g;
}

// ---------------------------------------------------------------- stencil
// Gather the 8 incident element conductivities of node (i,j,k) and the
// 21 non-zero stencil coefficients, then y = sum coef * x for each load.
template <typename T>
struct NodeCoef {
    T c0;       // centre
    T ce[12];   // edge-diagonal neighbours
    T cc[8];    // corners
};

template <typename T>
__device__ __forceinline__ void node_coefs(const T (&ko)[8], NodeCoef<T>& c) {
    const T w = (T)(1.0 / 12.0);
    T tot = 0;
#pragma unroll
    for (int o = 0; o < 8; ++o) tot += ko[o];
    c.c0 = tot * (T)(1.0 / 3.0);
    // edges in the xy plane: (dx,dy) in {-,+}^2, shared elements c' = 0,1
    int q = 0;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) c.ce[q++] = -w * (ko[a + 2 * b] + ko[a + 2 * b + 4]);
    // edges in the xz plane: (dx,dz), shared b' = 0,1
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int a = 0; a < 2; ++a) c.ce[q++] = -w * (ko[a + 4 * cz] + ko[a + 2 + 4 * cz]);
    // edges in the yz plane: (dy,dz), shared a' = 0,1
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int b = 0; b < 2; ++b) c.ce[q++] = -w * (ko[2 * b + 4 * cz] + ko[1 + 2 * b + 4 * cz]);
#pragma unroll
    for (int o = 0; o < 8; ++o) c.cc[o] = -w * ko[o];
}

// Offsets of the 3x3x3 neighbourhood of node (i,j,k).
struct Nbr {
    int x[3], y[3], z[3];
};

__device__ __forceinline__ Nbr nbr_of(int i, int j, int k, int n) {
    Nbr o;
    o.x[0] = wrapi(i - 1, n);
    o.x[1] = i;
    o.x[2] = wrapi(i + 1, n);
    o.y[0] = wrapi(j - 1, n) * n;
    o.y[1] = j * n;
    o.y[2] = wrapi(j + 1, n) * n;
    const int nn2 = n * n;
    o.z[0] = wrapi(k - 1, n) * nn2;
    o.z[1] = k * nn2;
    o.z[2] = wrapi(k + 1, n) * nn2;
    return o;
}

template <typename T>
__device__ __forceinline__ void load_k8(const T* __restrict__ k, const Nbr& o, T (&ko)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) ko[q] = k[o.x[q & 1] + o.y[(q >> 1) & 1] + o.z[(q >> 2) & 1]];
}

// y = A x at one node for one load (x is the load's base pointer).
template <typename T, typename TX>
__device__ __forceinline__ T stencil_node(const NodeCoef<T>& c, const Nbr& o, const TX* __restrict__ x) {
    // a' index (0 or 1) maps to offset -1 / +1 -> Nbr index 0 / 2
    T y = c.c0 * (T)x[o.x[1] + o.y[1] + o.z[1]];
    int q = 0;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) y += c.ce[q++] * (T)x[o.x[2 * a] + o.y[2 * b] + o.z[1]];
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int a = 0; a < 2; ++a) y += c.ce[q++] * (T)x[o.x[2 * a] + o.y[1] + o.z[2 * cz]];
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int b = 0; b < 2; ++b) y += c.ce[q++] * (T)x[o.x[1] + o.y[2 * b] + o.z[2 * cz]];
#pragma unroll
    for (int q2 = 0; q2 < 8; ++q2) y += c.cc[q2] * (T)x[o.x[2 * (q2 & 1)] + o.y[2 * ((q2 >> 1) & 1)] + o.z[2 * ((q2 >> 2) & 1)]];
    return y;
}

}  // namespace otm
