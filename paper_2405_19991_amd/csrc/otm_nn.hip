// Learned PCG warm start: a 5-layer periodic 3x3x3 convolutional network
// (channels 1 -> 16 -> 16 -> 16 -> 16 -> 3, ReLU after layers 1-4, output mean
// removed per channel) that maps the filtered density to the three
// fluctuation fields.  Forward, input-gradient and weight-gradient
// convolutions run on bf16 MFMA (v_mfma_f32_16x16x16_bf16) with float32
// accumulation; Adam keeps float32 master weights.
//
// Layout: activations are channels-last bf16 [voxel][16] (padded channels are
// zero), voxel index x + n (y + n z), n a multiple of 16.  A convolution is an
// implicit GEMM per tap t: out^T (16 out-channels x 16 voxels) +=
// W_t (16 out x 16 in) * in^T (16 in x 16 voxels shifted by tap t).  With the
// MFMA lane layout (lane l: A row l%16, k = 4(l/16)+i; B column l%16, same k;
// D column l%16, rows 4(l/16)+i) every lane loads 4 consecutive channels of
// one voxel and stores 4 consecutive output channels of one voxel.
// Tap t = 9 (dz+1) + 3 (dy+1) + (dx+1); the convolution is the correlation
// y[v] = b + sum_t W_t x[v + d_t] with periodic wrap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "opentm_amd.h"
#include "otm_device.h"

namespace otm {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));  // 16-byte chunk (a native vector: stays in registers)
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8b __attribute__((ext_vector_type(8)));

// D += A B on gfx950's 16x16x32 bf16 MFMA with K = two 16-deep halves: lane
// group g of A and of B holds elements k = 8 g .. 8 g + 7, the first four
// taken from (a0, b0) and the last four from (a1, b1); whatever order the
// unit sums k in, A's and B's element j of a lane group meet, so the result
// is a0 b0 + a1 b1 summed over the two 16x16x16 operand pairs.
__device__ __forceinline__ v4f mfma_pair(v4s a0, v4s a1, v4s b0, v4s b1, v4f d) {
    const v8s a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
    const v8s b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8b, a), __builtin_bit_cast(v8b, b), d, 0, 0, 0);
}

constexpr int kNNLayers = 5;
constexpr int kNNCh[kNNLayers + 1] = {1, 16, 16, 16, 16, 3};
constexpr int kNNW = 16 * 16 * 27;  // padded weights per layer [co][ci][t]

__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

enum { NN_FWD_RELU = 0, NN_FWD_LAST = 1, NN_DGRAD_MASK = 2, NN_DGRAD = 3 };

// One convolution layer: forward with bias and ReLU, the last layer in FP32,
// or the input gradient masked by the forward activation.  A block computes a
// 16x4x4 brick of voxels.  The brick and its one-voxel periodic halo (18x6x6
// voxels, 16 bf16 channels each, 25.9 KB at a 40-byte voxel stride) are staged in LDS once and read by
// all 27 taps, instead of every tap re-reading its shifted voxels from global
// memory.  Wave w computes the four 16-voxel rows (y = 0..3) of brick plane
// z = w as four independent chains of 27 MFMAs.
constexpr int kBX = 16, kBY = 4, kBZ = 4;
constexpr int kHX = kBX + 2, kHY = kBY + 2, kHZ = kBZ + 2;
constexpr int kHVox = kHX * kHY * kHZ;
constexpr int kCS = 20;  // LDS voxel stride of the convolution tile (bf16 elements)

template <int MODE>
__global__ void __launch_bounds__(256) k_nn_conv_b(int n, const uint16_t* __restrict__ in,
                                                   const uint16_t* __restrict__ wl, const float* __restrict__ bias,
                                                   void* __restrict__ out, const uint16_t* __restrict__ mask) {
    // voxel stride 20 channels (40 bytes): the 16 voxels of a row read by one
    // lane group then fall on 16 distinct bank pairs (a 32-byte stride would
    // put every fourth voxel on the same banks)
    __shared__ __attribute__((aligned(16))) uint16_t tile[kHVox * kCS];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int nbx = n / kBX, nby = n / kBY;
    const int nbricks = nbx * nby * (n / kBZ);
    // weights of the 27 taps in lane order, wl[(t*64 + lane)*4 + i]: loaded once
    // per block, which then walks its share of the bricks
    v4s w[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const uint2 raw = *reinterpret_cast<const uint2*>(wl + ((size_t)t * 64 + lane) * 4);
        w[t] = *reinterpret_cast<const v4s*>(&raw);
    }
    const int m = lane & 15;         // voxel within the row (B column / D column)
    const int cg = (lane >> 4) * 4;  // channel quad (B rows k / D rows)
    float bq[4] = {0.f, 0.f, 0.f, 0.f};
    if (MODE == NN_FWD_RELU || MODE == NN_FWD_LAST) {
#pragma unroll
        for (int i = 0; i < 4; ++i) bq[i] = bias[cg + i];
    }
    constexpr int kChunks = kHVox * 2;
    constexpr int kPer = (kChunks + 255) / 256;
    // bricks in x, then y, then z; contiguous ranges per XCD (the grid is a
    // multiple of 8 or covers every brick)
    for (int vb = blockIdx.x; vb < nbricks; vb += gridDim.x) {
        int b = xcd_tile(vb, nbricks);
        const int bx = b % nbx;
        b /= nbx;
        const int by = b % nby;
        const int bz = b / nby;
        const int x0 = bx * kBX, y0 = by * kBY, z0 = bz * kBZ;
        // stage the halo brick: two 16-byte chunks per voxel, a thread's loads
        // all issued before its first LDS store
        v4u buf[kPer];
#pragma unroll
        for (int it = 0; it < kPer; ++it) {
            const int c = threadIdx.x + it * 256;
            if (c < kChunks) {
                const int vox = c >> 1, half = c & 1;
                const int hx = vox % kHX, hy = (vox / kHX) % kHY, hz = vox / (kHX * kHY);
                int xs = x0 - 1 + hx, ys = y0 - 1 + hy, zs = z0 - 1 + hz;
                xs = xs < 0 ? xs + n : (xs >= n ? xs - n : xs);
                ys = ys < 0 ? ys + n : (ys >= n ? ys - n : ys);
                zs = zs < 0 ? zs + n : (zs >= n ? zs - n : zs);
                const size_t vs = (size_t)xs + (size_t)n * ((size_t)ys + (size_t)n * zs);
                buf[it] = *reinterpret_cast<const v4u*>(in + vs * 16 + half * 8);
            }
        }
        __syncthreads();  // the previous brick's reads of the tile are done
#pragma unroll
        for (int it = 0; it < kPer; ++it) {
            const int c = threadIdx.x + it * 256;
            if (c < kChunks) {
                uint16_t* dst = &tile[(c >> 1) * kCS + (c & 1) * 8];  // 8-byte aligned
                reinterpret_cast<uint2*>(dst)[0] = make_uint2(buf[it].x, buf[it].y);
                reinterpret_cast<uint2*>(dst)[1] = make_uint2(buf[it].z, buf[it].w);
            }
        }
        __syncthreads();
        // the wave's four rows (y = 0..3 of brick plane z = wv) as four
        // independent accumulator chains, tap by tap
        const int zz = wv;
        v4f acc[kBY];
#pragma unroll
        for (int yy = 0; yy < kBY; ++yy) acc[yy] = (v4f){0.f, 0.f, 0.f, 0.f};
        // taps in pairs (2p, 2p + 1) on the 16x16x32 MFMA, tap 26 on the 16x16x16 one
        auto rows = [&](int t, v4s (&bb)[kBY]) {
            const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
#pragma unroll
            for (int yy = 0; yy < kBY; ++yy) {
                const int hv = ((zz + 1 + dz) * kHY + (yy + 1 + dy)) * kHX + (m + 1 + dx);
                const uint2 raw = *reinterpret_cast<const uint2*>(&tile[hv * kCS + cg]);
                bb[yy] = *reinterpret_cast<const v4s*>(&raw);
            }
        };
#pragma unroll
        for (int pr = 0; pr < 13; ++pr) {
            v4s b0[kBY], b1[kBY];
            rows(2 * pr, b0);
            rows(2 * pr + 1, b1);
#pragma unroll
            for (int yy = 0; yy < kBY; ++yy) acc[yy] = mfma_pair(w[2 * pr], w[2 * pr + 1], b0[yy], b1[yy], acc[yy]);
        }
        {
            v4s b0[kBY];
            rows(26, b0);
#pragma unroll
            for (int yy = 0; yy < kBY; ++yy)
                acc[yy] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[26], b0[yy], acc[yy], 0, 0, 0);
        }
#pragma unroll
        for (int yy = 0; yy < kBY; ++yy) {
            const size_t v = (size_t)(x0 + m) + (size_t)n * ((size_t)(y0 + yy) + (size_t)n * (z0 + zz));
            if (MODE == NN_FWD_LAST) {
                float4 o = make_float4(acc[yy][0] + bq[0], acc[yy][1] + bq[1], acc[yy][2] + bq[2], acc[yy][3] + bq[3]);
                reinterpret_cast<float4*>(out)[v * 4 + (cg >> 2)] = o;
            } else {
                float o[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    o[i] = acc[yy][i] + bq[i];
                    if (MODE == NN_FWD_RELU) o[i] = fmaxf(o[i], 0.f);
                }
                if (MODE == NN_DGRAD_MASK) {
                    const uint2 mr = *reinterpret_cast<const uint2*>(mask + v * 16 + cg);
                    const uint16_t* mh = reinterpret_cast<const uint16_t*>(&mr);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (!(bf2f(mh[i]) > 0.f)) o[i] = 0.f;
                }
                uint2 pk;
                pk.x = (uint32_t)f2bf(o[0]) | ((uint32_t)f2bf(o[1]) << 16);
                pk.y = (uint32_t)f2bf(o[2]) | ((uint32_t)f2bf(o[3]) << 16);
                *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(out) + v * 16 + cg) = pk;
            }
        }
    }
}

// Weight and bias gradients of one layer: dW[t][ci][co] = sum_v x[v + d_t][ci] dy[v][co],
// db[co] = sum_v dy[v][co].  A block stages a 16x4x4 brick of dy and the
// brick of x with its one-voxel periodic halo in LDS, with a voxel stride of
// kWS = 20 channels so that the four lane groups' 2-byte reads of one channel
// (voxels 4 apart) fall in different banks; wave w accumulates the taps
// w, w + 4, ... over the brick's 16 rows of 16 voxels (MFMA with the voxels as
// the reduction dimension: A = x shifted by the tap, 16 ci x 16 voxels; B =
// dy, 16 voxels x 16 co) and walks its share of the bricks; the block then
// writes its 27 tiles and (wave 0) its bias sums to its own partial slot.
constexpr int kWS = 20;
constexpr int kWSlot = 27 * 256 + 16;  // floats per partial slot
constexpr int kWSlots = 512;           // partial slots (blocks of the weight gradient)

__global__ void __launch_bounds__(256) k_nn_wgrad(int n, const uint16_t* __restrict__ x, const uint16_t* __restrict__ dy,
                                                  float* __restrict__ partials /* [blocks][kWSlot] */) {
    __shared__ __attribute__((aligned(16))) uint16_t xt[kHVox * kWS];
    __shared__ __attribute__((aligned(16))) uint16_t dt[kBX * kBY * kBZ * kWS];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int c = lane & 15;         // A row = ci ; B column = co
    const int kq = (lane >> 4) * 4;  // the lane's 4 voxels of a 16-voxel row (the reduction index)
    const int nbx = n / kBX, nby = n / kBY;
    const int nbricks = nbx * nby * (n / kBZ);
    constexpr int kT = 7;  // taps per wave (wave 3 has 6)
    v4f acc[kT];
#pragma unroll
    for (int j = 0; j < kT; ++j) acc[j] = (v4f){0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    constexpr int kChunks = kHVox * 2;
    constexpr int kPer = (kChunks + 255) / 256;
    constexpr int kDPer = kBX * kBY * kBZ * 2 / 256;  // dy chunks per thread (2)
    for (int vb = blockIdx.x; vb < nbricks; vb += gridDim.x) {
        int b = xcd_tile(vb, nbricks);
        const int bx = b % nbx;
        b /= nbx;
        const int by = b % nby;
        const int bz = b / nby;
        const int x0 = bx * kBX, y0 = by * kBY, z0 = bz * kBZ;
        v4u buf[kPer], dbuf[kDPer];
#pragma unroll
        for (int it = 0; it < kPer; ++it) {
            const int ch = threadIdx.x + it * 256;
            if (ch < kChunks) {
                const int vox = ch >> 1, half = ch & 1;
                const int hx = vox % kHX, hy = (vox / kHX) % kHY, hz = vox / (kHX * kHY);
                int xs = x0 - 1 + hx, ys = y0 - 1 + hy, zs = z0 - 1 + hz;
                xs = xs < 0 ? xs + n : (xs >= n ? xs - n : xs);
                ys = ys < 0 ? ys + n : (ys >= n ? ys - n : ys);
                zs = zs < 0 ? zs + n : (zs >= n ? zs - n : zs);
                const size_t vs = (size_t)xs + (size_t)n * ((size_t)ys + (size_t)n * zs);
                buf[it] = *reinterpret_cast<const v4u*>(x + vs * 16 + half * 8);
            }
        }
#pragma unroll
        for (int it = 0; it < kDPer; ++it) {
            const int ch = threadIdx.x + it * 256;
            const int vox = ch >> 1, half = ch & 1;
            const int ix = vox % kBX, iy = (vox / kBX) % kBY, iz = vox / (kBX * kBY);
            const size_t vs = (size_t)(x0 + ix) + (size_t)n * ((size_t)(y0 + iy) + (size_t)n * (z0 + iz));
            dbuf[it] = *reinterpret_cast<const v4u*>(dy + vs * 16 + half * 8);
        }
        __syncthreads();  // the previous brick's reads of the tiles are done
        // 16-byte chunks at 8-byte aligned LDS offsets (voxel stride 40 bytes)
#pragma unroll
        for (int it = 0; it < kPer; ++it) {
            const int ch = threadIdx.x + it * 256;
            if (ch < kChunks) {
                uint16_t* dst = &xt[(ch >> 1) * kWS + (ch & 1) * 8];
                reinterpret_cast<uint2*>(dst)[0] = make_uint2(buf[it].x, buf[it].y);
                reinterpret_cast<uint2*>(dst)[1] = make_uint2(buf[it].z, buf[it].w);
            }
        }
#pragma unroll
        for (int it = 0; it < kDPer; ++it) {
            const int ch = threadIdx.x + it * 256;
            uint16_t* dst = &dt[(ch >> 1) * kWS + (ch & 1) * 8];
            reinterpret_cast<uint2*>(dst)[0] = make_uint2(dbuf[it].x, dbuf[it].y);
            reinterpret_cast<uint2*>(dst)[1] = make_uint2(dbuf[it].z, dbuf[it].w);
        }
        __syncthreads();
        // rows in pairs (K = 32 voxels per 16x16x32 MFMA)
#pragma unroll 2
        for (int rp = 0; rp < kBY * kBZ / 2; ++rp) {
            v4s bv[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int row = 2 * rp + h;
                const int yk = row % kBY, zk = row / kBY;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint16_t v = dt[((zk * kBY + yk) * kBX + kq + i) * kWS + c];
                    bv[h][i] = (short)v;
                    if (wv == 0) bsum += bf2f(v);
                }
            }
#pragma unroll
            for (int j = 0; j < kT; ++j) {
                const int t = wv + 4 * j;
                if (t < 27) {
                    const int dz = t / 9 - 1, dyy = (t / 3) % 3 - 1, dx = t % 3 - 1;
                    v4s av[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int row = 2 * rp + h;
                        const int yk = row % kBY, zk = row / kBY;
                        const int hrow = ((zk + 1 + dz) * kHY + (yk + 1 + dyy)) * kHX + 1 + dx;
#pragma unroll
                        for (int i = 0; i < 4; ++i) av[h][i] = (short)xt[(hrow + kq + i) * kWS + c];
                    }
                    acc[j] = mfma_pair(av[0], av[1], bv[0], bv[1], acc[j]);
                }
            }
        }
    }
    // D[ci][co]: lane holds co = lane%16, ci = 4(lane/16)+i
    float* dst = partials + (size_t)blockIdx.x * kWSlot;
#pragma unroll
    for (int j = 0; j < kT; ++j) {
        const int t = wv + 4 * j;
        if (t < 27)
#pragma unroll
            for (int i = 0; i < 4; ++i) dst[t * 256 + (kq + i) * 16 + c] = acc[j][i];
    }
    // bias (wave 0): lanes with the same co (lane%16) hold disjoint voxel quads
    bsum += __shfl_xor(bsum, 16, 64);
    bsum += __shfl_xor(bsum, 32, 64);
    if (wv == 0 && lane < 16) dst[27 * 256 + lane] = bsum;
}

// grad[t][ci][co] (+ bias) += the sum over the slots, in a fixed order: a
// block takes 64 consecutive entries, each of its four waves a quarter of the
// slots (in order), and the quarters are added in order.
__global__ void __launch_bounds__(256) k_nn_wgrad_reduce(int nslots, const float* __restrict__ partials,
                                                         float* __restrict__ gw /* [co][ci][27] padded */,
                                                         float* __restrict__ gb) {
    __shared__ float sh[4][64];
    const int j = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + j;
    const int per = (nslots + 3) / 4;
    float s = 0.f;
    if (e < kWSlot) {
        const int w0 = q * per, w1 = min(nslots, w0 + per);
#pragma unroll 8
        for (int w = w0; w < w1; ++w) s += partials[(size_t)w * kWSlot + e];
    }
    sh[q][j] = s;
    __syncthreads();
    if (q != 0 || e >= kWSlot) return;
    const float tot = ((sh[0][j] + sh[1][j]) + sh[2][j]) + sh[3][j];
    if (e < 27 * 256) {
        const int t = e / 256, ci = (e / 16) % 16, co = e % 16;
        gw[(co * 16 + ci) * 27 + t] += tot;
    } else {
        gb[e - 27 * 256] += tot;
    }
}

// Lane-ordered bf16 weights for the forward pass (A = W_t[co][ci]) and for
// the input gradient (A = W_{26-t}[co][ci] transposed: rows ci, columns co).
__global__ void k_nn_prep(const float* __restrict__ W /* [co][ci][27] */, int cout, int cin,
                          uint16_t* __restrict__ wf, uint16_t* __restrict__ wd) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;  // (t, lane, i)
    if (e >= 27 * 64 * 4) return;
    const int t = e / 256, lane = (e / 4) % 64, i = e % 4;
    const int row = lane % 16, k = 4 * (lane / 16) + i;
    // forward: row = co, k = ci
    float vf = (row < cout && k < cin) ? W[(row * 16 + k) * 27 + t] : 0.f;
    wf[e] = f2bf(vf);
    // input gradient: row = ci, k = co, tap mirrored
    float vd = (k < cout && row < cin) ? W[(k * 16 + row) * 27 + (26 - t)] : 0.f;
    wd[e] = f2bf(vd);
}

__global__ void k_nn_pack_input(int64_t nn, const double* __restrict__ rhof, uint16_t* __restrict__ act) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nn) return;
    uint4 z0 = make_uint4(0, 0, 0, 0);
    z0.x = f2bf((float)rhof[v]);
    reinterpret_cast<uint4*>(act + v * 16)[0] = z0;
    reinterpret_cast<uint4*>(act + v * 16)[1] = make_uint4(0, 0, 0, 0);
}

// sums of out[v][c] (c < 3) and, when chi != null, of chi[c][v]
__global__ void __launch_bounds__(kBlock) k_nn_sums(int64_t nn, const float* __restrict__ out,
                                                    const double* __restrict__ chi, double* partials) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < nn; v += (int64_t)gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[c] += out[v * 16 + c];
            if (chi) acc[3 + c] += chi[c * nn + v];
        }
    }
    block_partials<6>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_nn_reduce(int nblocks, int nv, const double* __restrict__ partials,
                                                      double* __restrict__ dst) {
    __shared__ double sh[kBlock];
    for (int q = 0; q < nv; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partials[(size_t)b * nv + q];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) dst[q] = sh[0];
        __syncthreads();
    }
}

// d = (out - mean out) - (chi - mean chi); loss partial sum d^2; dout = 2 d / (3 nn) as bf16
__global__ void __launch_bounds__(kBlock) k_nn_loss(int64_t nn, const float* __restrict__ out,
                                                    const double* __restrict__ chi, const double* __restrict__ sums,
                                                    uint16_t* __restrict__ dout, double* partials) {
    double acc[1] = {0.0};
    const double inv = 1.0 / (double)nn;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < nn; v += (int64_t)gridDim.x * kBlock) {
        uint16_t g[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) g[c] = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double d = ((double)out[v * 16 + c] - sums[c] * inv) - (chi[c * nn + v] - sums[3 + c] * inv);
            acc[0] += d * d;
            g[c] = f2bf((float)(2.0 * d / (3.0 * (double)nn)));
        }
        uint4* dst = reinterpret_cast<uint4*>(dout + v * 16);
        dst[0] = make_uint4(g[0] | (g[1] << 16), g[2] | (g[3] << 16), g[4] | (g[5] << 16), g[6] | (g[7] << 16));
        dst[1] = make_uint4(g[8] | (g[9] << 16), g[10] | (g[11] << 16), g[12] | (g[13] << 16), g[14] | (g[15] << 16));
    }
    block_partials<1>(acc, partials);
}

// chi0[c][v] = out[v][c] - mean(out[.][c]) as float64
__global__ void k_nn_extract(int64_t nn, const float* __restrict__ out, const double* __restrict__ sums,
                             double* __restrict__ chi0) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nn) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) chi0[c * nn + v] = (double)out[v * 16 + c] - sums[c] / (double)nn;
}

__global__ void k_nn_adam(int count, float* __restrict__ p, float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, const float* __restrict__ live, float lr, float b1, float b2,
                          float eps, float c1, float c2, float scale) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const float gr = g[e] * scale;
    g[e] = 0.f;
    if (live[e] == 0.f) return;  // padded entries stay zero
    const float mm = b1 * m[e] + (1.f - b1) * gr;
    const float vv = b2 * v[e] + (1.f - b2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

}  // namespace otm

using namespace otm;

// ---------------------------------------------------------------- network
struct otm_nn {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n_max = 0;
    // float32 master parameters, padded per layer: W [16][16][27], b [16]
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *live = nullptr;
    uint16_t *wf = nullptr, *wd = nullptr;  // lane-ordered bf16, per layer 27*64*4
    uint16_t* act[kNNLayers] = {};          // inputs of each layer [voxel][16]
    uint16_t *gA = nullptr, *gB = nullptr;  // gradient ping-pong
    float* out = nullptr;                   // last layer [voxel][16] float32
    float* wpart = nullptr;
    double* partials = nullptr;
    double* sums = nullptr;                 // 6 means + loss
    int adam_t = 0;

    std::string err;
};

hipStream_t otm::nn_stream(const otm_nn* net) { return net->stream; }

namespace {

constexpr int kLayerParams = kNNW + 16;

int nn_fail(otm_nn* c, int code, const std::string& m) {
    if (c) c->err = m;
    return code;
}

#define NNCHK(c, call)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return nn_fail((c), OTM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int compact_count() {
    int s = 0;
    for (int l = 0; l < kNNLayers; ++l) s += kNNCh[l + 1] * kNNCh[l] * 27 + kNNCh[l + 1];
    return s;
}

void prep_all(otm_nn* c) {
    for (int l = 0; l < kNNLayers; ++l)
        hipLaunchKernelGGL(k_nn_prep, dim3((27 * 256 + 255) / 256), dim3(256), 0, c->stream,
                           c->p + (size_t)l * kLayerParams, kNNCh[l + 1], kNNCh[l], c->wf + (size_t)l * 27 * 256,
                           c->wd + (size_t)l * 27 * 256);
}

// blocks of the convolution: persistent over the 16x4x4 bricks (n is a
// multiple of 16), at most 4 per CU
int conv_bricks(int n) {
    const int bricks = (n / kBX) * (n / kBY) * (n / kBZ);
    return bricks < 1024 ? bricks : 1024;
}


int forward(otm_nn* c, int n, const double* rhof) {
    const int64_t nn = (int64_t)n * n * n;
    hipLaunchKernelGGL(k_nn_pack_input, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, c->stream, nn, rhof,
                       c->act[0]);
    const int bricks = conv_bricks(n);
    for (int l = 0; l < kNNLayers; ++l) {
        const uint16_t* wl = c->wf + (size_t)l * 27 * 256;
        const float* b = c->p + (size_t)l * kLayerParams + kNNW;
        if (l < kNNLayers - 1)
            hipLaunchKernelGGL(k_nn_conv_b<NN_FWD_RELU>, dim3(bricks), dim3(256), 0, c->stream, n, c->act[l], wl, b,
                               (void*)c->act[l + 1], (const uint16_t*)nullptr);
        else
            hipLaunchKernelGGL(k_nn_conv_b<NN_FWD_LAST>, dim3(bricks), dim3(256), 0, c->stream, n, c->act[l], wl, b,
                               (void*)c->out, (const uint16_t*)nullptr);
    }
    return hipGetLastError() == hipSuccess ? OTM_OK : nn_fail(c, OTM_EDEVICE, "nn forward launch");
}

int out_means(otm_nn* c, int n, const double* chi) {
    const int64_t nn = (int64_t)n * n * n;
    int blocks = (int)std::min<int64_t>((nn + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(k_nn_sums, dim3(blocks), dim3(kBlock), 0, c->stream, nn, (const float*)c->out, chi,
                       c->partials);
    hipLaunchKernelGGL(k_nn_reduce, dim3(1), dim3(kBlock), 0, c->stream, blocks, 6, (const double*)c->partials,
                       c->sums);
    return OTM_OK;
}

}  // namespace

extern "C" {

int otm_nn_create(int32_t n_max, uint64_t seed, void* stream, otm_nn** out) {
    if (!out || n_max < 16 || n_max > 512 || n_max % 16) return OTM_EINVAL;
    *out = nullptr;
    otm_nn* c = new (std::nothrow) otm_nn();
    if (!c) return OTM_ENOMEM;
    c->n_max = n_max;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return OTM_EDEVICE;
    } else {
        c->own_stream = true;
    }
    const int64_t nn = (int64_t)n_max * n_max * n_max;
    const size_t np = (size_t)kNNLayers * kLayerParams;
    bool ok = true;
    auto al = [&](void** p, size_t bytes) {
        if (ok && hipMalloc(p, bytes) != hipSuccess) ok = false;
    };
    al((void**)&c->p, np * 4);
    al((void**)&c->g, np * 4);
    al((void**)&c->m, np * 4);
    al((void**)&c->v, np * 4);
    al((void**)&c->live, np * 4);
    al((void**)&c->wf, (size_t)kNNLayers * 27 * 256 * 2);
    al((void**)&c->wd, (size_t)kNNLayers * 27 * 256 * 2);
    for (int l = 0; l < kNNLayers; ++l) al((void**)&c->act[l], (size_t)nn * 16 * 2);
    al((void**)&c->gA, (size_t)nn * 16 * 2);
    al((void**)&c->gB, (size_t)nn * 16 * 2);
    al((void**)&c->out, (size_t)nn * 16 * 4);
    al((void**)&c->wpart, (size_t)kWSlots * kWSlot * 4);
    al((void**)&c->partials, (size_t)1024 * 8 * 8);
    al((void**)&c->sums, 16 * 8);
    if (!ok) {
        (void)hipGetLastError();
        otm_nn_destroy(c);
        return OTM_ENOMEM;
    }
    // He-uniform initialization (fan-in 27 cin) with a 64-bit LCG, zero biases
    std::vector<float> hp(np, 0.f), hl(np, 0.f);
    uint64_t s = seed * 6364136223846793005ull + 1442695040888963407ull;
    for (int l = 0; l < kNNLayers; ++l) {
        const int cin = kNNCh[l], cout = kNNCh[l + 1];
        const float lim = std::sqrt(6.0f / (27.0f * cin));
        float* W = hp.data() + (size_t)l * kLayerParams;
        float* L = hl.data() + (size_t)l * kLayerParams;
        for (int co = 0; co < cout; ++co)
            for (int ci = 0; ci < cin; ++ci)
                for (int t = 0; t < 27; ++t) {
                    s = s * 6364136223846793005ull + 1442695040888963407ull;
                    const double u = (double)(s >> 11) / 9007199254740992.0;
                    W[(co * 16 + ci) * 27 + t] = (float)((2.0 * u - 1.0) * lim);
                    L[(co * 16 + ci) * 27 + t] = 1.f;
                }
        for (int co = 0; co < cout; ++co) L[kNNW + co] = 1.f;
    }
    (void)hipMemcpyAsync(c->p, hp.data(), np * 4, hipMemcpyHostToDevice, c->stream);
    (void)hipMemcpyAsync(c->live, hl.data(), np * 4, hipMemcpyHostToDevice, c->stream);
    (void)hipMemsetAsync(c->g, 0, np * 4, c->stream);
    (void)hipMemsetAsync(c->m, 0, np * 4, c->stream);
    (void)hipMemsetAsync(c->v, 0, np * 4, c->stream);
    prep_all(c);
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        otm_nn_destroy(c);
        return OTM_EDEVICE;
    }
    *out = c;
    return OTM_OK;
}

void otm_nn_destroy(otm_nn* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    void* bufs[] = {c->p, c->g, c->m, c->v, c->live, c->wf, c->wd, c->gA, c->gB, c->out, c->wpart, c->partials, c->sums};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (auto* a : c->act)
        if (a) (void)hipFree(a);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int32_t otm_nn_param_count(void) { return compact_count(); }

// compact layout: per layer W[cout][cin][27] then b[cout]
static int nn_copy_params(otm_nn* c, float* host, bool get, const float* src_dev) {
    const size_t np = (size_t)kNNLayers * kLayerParams;
    std::vector<float> pad(np);
    if (get) {
        NNCHK(c, hipMemcpyAsync(pad.data(), src_dev, np * 4, hipMemcpyDeviceToHost, c->stream));
        NNCHK(c, hipStreamSynchronize(c->stream));
    }
    size_t q = 0;
    for (int l = 0; l < kNNLayers; ++l) {
        const int cin = kNNCh[l], cout = kNNCh[l + 1];
        float* W = pad.data() + (size_t)l * kLayerParams;
        for (int co = 0; co < cout; ++co)
            for (int ci = 0; ci < cin; ++ci)
                for (int t = 0; t < 27; ++t, ++q) {
                    if (get)
                        host[q] = W[(co * 16 + ci) * 27 + t];
                    else
                        W[(co * 16 + ci) * 27 + t] = host[q];
                }
        for (int co = 0; co < cout; ++co, ++q) {
            if (get)
                host[q] = W[kNNW + co];
            else
                W[kNNW + co] = host[q];
        }
    }
    if (!get) {
        NNCHK(c, hipMemcpyAsync(c->p, pad.data(), np * 4, hipMemcpyHostToDevice, c->stream));
        prep_all(c);
        NNCHK(c, hipStreamSynchronize(c->stream));
    }
    return OTM_OK;
}

int otm_nn_get_params(otm_nn* c, float* host, int64_t count) {
    if (!c || !host || count != compact_count()) return OTM_EINVAL;
    return nn_copy_params(c, host, true, c->p);
}

int otm_nn_set_params(otm_nn* c, const float* host, int64_t count) {
    if (!c || !host || count != compact_count()) return OTM_EINVAL;
    for (int64_t q = 0; q < count; ++q)
        if (!std::isfinite(host[q])) return nn_fail(c, OTM_ENONFINITE, "non-finite parameter");
    c->adam_t = 0;
    return nn_copy_params(c, const_cast<float*>(host), false, nullptr);
}

int otm_nn_get_grads(otm_nn* c, float* host, int64_t count) {
    if (!c || !host || count != compact_count()) return OTM_EINVAL;
    return nn_copy_params(c, host, true, c->g);
}

int otm_nn_forward(otm_nn* c, int32_t n, const void* rhof_dev, void* chi0_dev) {
    if (!c || !rhof_dev || !chi0_dev || n < 16 || n > c->n_max || n % 16) return OTM_EINVAL;
    int rc = forward(c, n, (const double*)rhof_dev);
    if (rc) return rc;
    out_means(c, n, nullptr);
    const int64_t nn = (int64_t)n * n * n;
    hipLaunchKernelGGL(k_nn_extract, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, c->stream, nn,
                       (const float*)c->out, (const double*)c->sums, (double*)chi0_dev);
    return hipGetLastError() == hipSuccess ? OTM_OK : nn_fail(c, OTM_EDEVICE, "nn extract");
}

int otm_nn_accumulate(otm_nn* c, int32_t n, const void* rhof_dev, const void* chi_dev, double* loss_out) {
    if (!c || !rhof_dev || !chi_dev || n < 16 || n > c->n_max || n % 16) return OTM_EINVAL;
    const int64_t nn = (int64_t)n * n * n;
    int rc = forward(c, n, (const double*)rhof_dev);
    if (rc) return rc;
    out_means(c, n, (const double*)chi_dev);
    int blocks = (int)std::min<int64_t>((nn + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(k_nn_loss, dim3(blocks), dim3(kBlock), 0, c->stream, nn, (const float*)c->out,
                       (const double*)chi_dev, (const double*)c->sums, c->gA, c->partials);
    hipLaunchKernelGGL(k_nn_reduce, dim3(1), dim3(kBlock), 0, c->stream, blocks, 1, (const double*)c->partials,
                       c->sums + 8);
    // backward: gA holds dL/d(out of layer l); the mean removal needs no
    // correction because the loss gradient already has zero mean per channel
    uint16_t* gcur = c->gA;
    uint16_t* gnext = c->gB;
    for (int l = kNNLayers - 1; l >= 0; --l) {
        const int wblocks = std::min((n / kBX) * (n / kBY) * (n / kBZ), kWSlots);
        hipLaunchKernelGGL(k_nn_wgrad, dim3(wblocks), dim3(256), 0, c->stream, n, (const uint16_t*)c->act[l],
                           (const uint16_t*)gcur, c->wpart);
        hipLaunchKernelGGL(k_nn_wgrad_reduce, dim3((kWSlot + 63) / 64), dim3(256), 0, c->stream, wblocks,
                           (const float*)c->wpart, c->g + (size_t)l * kLayerParams,
                           c->g + (size_t)l * kLayerParams + kNNW);
        if (l > 0) {
            hipLaunchKernelGGL(k_nn_conv_b<NN_DGRAD_MASK>, dim3(conv_bricks(n)), dim3(256), 0, c->stream, n,
                               (const uint16_t*)gcur, (const uint16_t*)(c->wd + (size_t)l * 27 * 256),
                               (const float*)nullptr, (void*)gnext, (const uint16_t*)c->act[l]);
            uint16_t* tmp = gcur;
            gcur = gnext;
            gnext = tmp;
        }
    }
    if (hipGetLastError() != hipSuccess) return nn_fail(c, OTM_EDEVICE, "nn backward launch");
    if (loss_out) {
        double h[16];
        NNCHK(c, hipMemcpyAsync(h, c->sums, 16 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        NNCHK(c, hipStreamSynchronize(c->stream));
        *loss_out = h[8] / (3.0 * (double)nn);
    }
    return OTM_OK;
}

int otm_nn_adam(otm_nn* c, double lr, int32_t batch) {
    if (!c || !(lr > 0.0) || batch < 1) return OTM_EINVAL;
    c->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)c->adam_t), c2 = 1.f - std::pow(b2, (float)c->adam_t);
    const int np = kNNLayers * kLayerParams;
    hipLaunchKernelGGL(k_nn_adam, dim3((np + 255) / 256), dim3(256), 0, c->stream, np, c->p, c->g, c->m, c->v,
                       (const float*)c->live, (float)lr, b1, b2, 1e-8f, c1, c2, 1.f / (float)batch);
    prep_all(c);
    NNCHK(c, hipStreamSynchronize(c->stream));
    return OTM_OK;
}

int otm_nn_zero_grads(otm_nn* c) {
    if (!c) return OTM_EINVAL;
    NNCHK(c, hipMemsetAsync(c->g, 0, (size_t)kNNLayers * kLayerParams * 4, c->stream));
    NNCHK(c, hipStreamSynchronize(c->stream));
    return OTM_OK;
}

const char* otm_nn_last_error(const otm_nn* c) { return c ? c->err.c_str() : "null network"; }

// Weights file: the compact parameter vector as a NumPy .npy array (format
// 1.0: magic, version, header length, a Python-literal header dict, then the
// raw little-endian float32 values), so that numpy.load reads it too.
int otm_nn_save(otm_nn* c, const char* path) {
    if (!c || !path || !path[0]) return OTM_EINVAL;
    const int64_t count = compact_count();
    std::vector<float> w((size_t)count);
    int rc = otm_nn_get_params(c, w.data(), count);
    if (rc) return rc;
    std::string hdr = "{'descr': '<f4', 'fortran_order': False, 'shape': (" + std::to_string(count) + ",), }";
    const size_t pre = 6 + 2 + 2;  // magic, version, header length
    while ((pre + hdr.size() + 1) % 64 != 0) hdr += ' ';
    hdr += '\n';
    const unsigned char magic[8] = {0x93, 'N', 'U', 'M', 'P', 'Y', 1, 0};
    const uint16_t hlen = (uint16_t)hdr.size();
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return nn_fail(c, OTM_EIO, "cannot open " + tmp + " for writing");
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&hlen, 1, 2, f) == 2 &&
              std::fwrite(hdr.data(), 1, hdr.size(), f) == hdr.size() &&
              std::fwrite(w.data(), sizeof(float), w.size(), f) == w.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return nn_fail(c, OTM_EIO, std::string("cannot write ") + path);
    }
    return OTM_OK;
}

int otm_nn_load(otm_nn* c, const char* path) {
    if (!c || !path || !path[0]) return OTM_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (!f) return nn_fail(c, OTM_EIO, std::string("cannot open ") + path);
    std::vector<unsigned char> buf;
    unsigned char chunk[1 << 16];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) buf.insert(buf.end(), chunk, chunk + got);
    const bool read_err = std::ferror(f) != 0;
    std::fclose(f);
    if (read_err) return nn_fail(c, OTM_EIO, std::string("cannot read ") + path);
    static const unsigned char magic[6] = {0x93, 'N', 'U', 'M', 'P', 'Y'};
    if (buf.size() < 10 || std::memcmp(buf.data(), magic, 6) != 0)
        return nn_fail(c, OTM_EIO, std::string(path) + " is not a .npy file");
    size_t hlen, hoff;
    if (buf[6] == 1) {
        hlen = (size_t)buf[8] | ((size_t)buf[9] << 8);
        hoff = 10;
    } else if ((buf[6] == 2 || buf[6] == 3) && buf.size() >= 12) {
        hlen = (size_t)buf[8] | ((size_t)buf[9] << 8) | ((size_t)buf[10] << 16) | ((size_t)buf[11] << 24);
        hoff = 12;
    } else {
        return nn_fail(c, OTM_EIO, "unsupported .npy version");
    }
    if (buf.size() < hoff + hlen) return nn_fail(c, OTM_EIO, "truncated .npy header");
    std::string hdr(buf.begin() + hoff, buf.begin() + hoff + hlen);
    std::string compact;
    for (char ch : hdr)
        if (ch != ' ') compact += ch;
    const int64_t count = compact_count();
    if (compact.find("'descr':'<f4'") == std::string::npos)
        return nn_fail(c, OTM_EIO, "weights must be little-endian float32 ('<f4')");
    if (compact.find("'fortran_order':False") == std::string::npos)
        return nn_fail(c, OTM_EIO, "weights must be in C order");
    const std::string shape1 = "'shape':(" + std::to_string(count) + ",)";
    if (compact.find(shape1) == std::string::npos)
        return nn_fail(c, OTM_EIO, "weights must be a 1-D array of " + std::to_string(count) + " values");
    const size_t data = hoff + hlen;
    if (buf.size() != data + (size_t)count * sizeof(float))
        return nn_fail(c, OTM_EIO, "weights file size does not match its header");
    std::vector<float> w((size_t)count);
    std::memcpy(w.data(), &buf[data], (size_t)count * sizeof(float));
    return otm_nn_set_params(c, w.data(), count);
}

}  // extern "C"
