// Learned warm start: a small MLP (16 inputs -> 4 x 256 ReLU -> 1) that predicts
// activation times from per-vertex features, trained and evaluated with BF16
// matrix-core kernels (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// Precision policy:
//   features X and the hidden-layer weights W1..W4 are rounded to bf16;
//   Z_l = H_{l-1} W_l^T + b_l accumulates in fp32, H_l = bf16(relu(Z_l));
//   y = H_4 . w5 + b5 in fp32 (w5, b5 fp32);
//   backward: dy = 2 (y - t) / m; dZ_4 = bf16(dy w5 [H_4 > 0]);
//   dW_l = dZ_l^T H_{l-1} and db_l = sum_i dZ_l accumulate in fp32;
//   dZ_{l-1} = bf16((dZ_l W_l) [H_{l-1} > 0]);  Adam on fp32 master weights.
#include <math.h>

#include <algorithm>

#include <cstring>
#include <random>
#include <vector>

#include "gbp_internal.h"

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

constexpr int IN = 16;      // 15 features + 1 zero pad
constexpr int HID = 256;
constexpr int NLAYER = 4;   // hidden layers

// flat parameter layout: W1 [256x16], b1, W2 [256x256], b2, W3, b3, W4, b4, w5 [256], b5 [1]
__host__ __device__ constexpr int off_W_dev(int l) {   // l = 1..4
    return l == 1 ? 0 : HID * IN + HID + (l - 2) * (HID * HID + HID);
}
__host__ __device__ constexpr int off_b_dev(int l) { return off_W_dev(l) + (l == 1 ? HID * IN : HID * HID); }
__host__ __device__ constexpr int off_w5_dev() { return off_W_dev(4) + HID * HID + HID; }

__device__ __forceinline__ bf16 to_bf16(float x) {
    const unsigned u = __float_as_uint(x);
    return (bf16)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(bf16 h) { return __uint_as_float((unsigned)h << 16); }

// ---------------------------------------------------------------- loss
__global__ void k_sum_parts(const float* __restrict__ part, int n, float scale, float* __restrict__ out) {
    __shared__ float sh[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0] * scale;
}

// ---------------------------------------------------------------- fused row-tile kernels
// A block of 4 waves owns a tile of 16 TR rows and runs the network's 256-wide layers
// on it with the tile in LDS (16 TR x 256 bf16 per layer).  Wave w
// computes the output columns [64 w, 64 w + 64) of a layer for all the tile's rows as
// the transposed product A S^T: TR x 4 tiles of v_mfma_f32_16x16x32_bf16 per K step of
// 32, the A operand (a row of a 256 x 256 weight matrix, 8 consecutive K values per
// lane) loaded straight from global memory (the matrix stays in L2; each fragment
// serves 16 TR rows), the B operand (a tile row's 8 K values) read from LDS, the next
// step's weight fragments in flight while the current step multiplies.  A lane's 4
// results are 4 consecutive columns of one row, stored with one 8-byte write.  Where a
// layer's output overwrites its input, it does so only after every wave has finished
// reading it.
//   forward:  H_l = bf16(relu(W_l H_{l-1} + b_l)), then y = H_4 . w5 + b5 in fp32;
//   backward: dZ_{l-1} = bf16((W_l^T dZ_l) [H_{l-1} > 0]) with A = W_l^T (a bf16
//             copy kept transposed).
// Inference runs the forward alone; training runs forward, misfit and backward
// chain in one kernel with H1..H3 kept in LDS for the backward's masks.
constexpr int HP = HID + 8;   // LDS row pitch (bf16): 528 bytes, 16-byte aligned rows

__device__ __forceinline__ bf16x8_t ld8(const bf16* p) {
    return *reinterpret_cast<const bf16x8_t*>(p);
}
__device__ __forceinline__ bool relu_on(bf16 h) { return h != 0 && !(h & 0x8000); }

// acc[t][c][r] = sum_k A[j][k] S[16 t + lr][k] with j = j0 + 16 c + 4 lq + r.  The
// weight fragments run D K steps ahead of the multiplies (a ring of D + 1 steps): 3
// for the small tiles, whose few multiplies per step would otherwise wait on the
// loads, 1 for the 128-row tile (registers).
template <int TR>
__device__ __forceinline__ void tile_layer(const bf16* __restrict__ A, bf16 (*S)[HP],
                                           floatx4 (&acc)[TR][4], int j0, int lr, int lq) {
    constexpr int NS = HID / 32;   // K steps
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[t][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bf16* a0 = A + (size_t)(j0 + lr) * HID + 8 * lq;
    if constexpr (TR >= 8) {
        bf16x8_t bw[4], bn[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bw[c] = ld8(a0 + (size_t)c * 16 * HID);
#pragma unroll 2
        for (int ks = 0; ks < NS; ++ks) {
            if (ks + 1 < NS) {
#pragma unroll
                for (int c = 0; c < 4; ++c) bn[c] = ld8(a0 + (size_t)c * 16 * HID + (ks + 1) * 32);
            }
#pragma unroll
            for (int t = 0; t < TR; ++t) {
                const bf16x8_t af = *reinterpret_cast<const bf16x8_t*>(&S[t * 16 + lr][ks * 32 + 8 * lq]);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[c], af, acc[t][c], 0, 0, 0);
            }
            if (ks + 1 < NS) {
#pragma unroll
                for (int c = 0; c < 4; ++c) bw[c] = bn[c];
            }
        }
    } else {
        constexpr int D = 3;
        bf16x8_t ring[D + 1][4];
#pragma unroll
        for (int d = 0; d < D; ++d)
#pragma unroll
            for (int c = 0; c < 4; ++c) ring[d][c] = ld8(a0 + (size_t)c * 16 * HID + d * 32);
#pragma unroll
        for (int ks = 0; ks < NS; ++ks) {
            if (ks + D < NS) {
#pragma unroll
                for (int c = 0; c < 4; ++c) ring[(ks + D) % (D + 1)][c] = ld8(a0 + (size_t)c * 16 * HID + (ks + D) * 32);
            }
#pragma unroll
            for (int t = 0; t < TR; ++t) {
                const bf16x8_t af = *reinterpret_cast<const bf16x8_t*>(&S[t * 16 + lr][ks * 32 + 8 * lq]);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ring[ks % (D + 1)][c], af, acc[t][c], 0, 0, 0);
            }
        }
    }
}

// forward epilogue: S = bf16(relu(acc + b)) in the wave's 64 columns
template <int TR>
__device__ __forceinline__ void relu_store(bf16 (*S)[HP], const floatx4 (&acc)[TR][4],
                                           const float* __restrict__ bias, int j0, int lr, int lq) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int j = j0 + c * 16 + 4 * lq;
        const float b0 = bias[j], b1 = bias[j + 1], b2 = bias[j + 2], b3 = bias[j + 3];
#pragma unroll
        for (int t = 0; t < TR; ++t) {
            const unsigned lo = to_bf16(fmaxf(acc[t][c][0] + b0, 0.f)) |
                                ((unsigned)to_bf16(fmaxf(acc[t][c][1] + b1, 0.f)) << 16);
            const unsigned hi = to_bf16(fmaxf(acc[t][c][2] + b2, 0.f)) |
                                ((unsigned)to_bf16(fmaxf(acc[t][c][3] + b3, 0.f)) << 16);
            *reinterpret_cast<uint2*>(&S[t * 16 + lr][j]) = make_uint2(lo, hi);
        }
    }
}

// backward epilogue: S = bf16(acc) where the forward activation in Hp (the same
// tile's H_{l-1}, in LDS) is positive, else 0; rows at or past m are zero
template <int TR>
__device__ __forceinline__ void mask_store(bf16 (*S)[HP], const floatx4 (&acc)[TR][4], bf16 (*Hp)[HP],
                                           int i0, int m, int j0, int lr, int lq) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int j = j0 + c * 16 + 4 * lq;
#pragma unroll
        for (int t = 0; t < TR; ++t) {
            const int r = t * 16 + lr;
            const uint2 h = i0 + r < m ? *reinterpret_cast<const uint2*>(&Hp[r][j]) : make_uint2(0u, 0u);
            const unsigned z0 = relu_on((bf16)(h.x & 0xffffu)) ? to_bf16(acc[t][c][0]) : 0u;
            const unsigned z1 = relu_on((bf16)(h.x >> 16)) ? to_bf16(acc[t][c][1]) : 0u;
            const unsigned z2 = relu_on((bf16)(h.y & 0xffffu)) ? to_bf16(acc[t][c][2]) : 0u;
            const unsigned z3 = relu_on((bf16)(h.y >> 16)) ? to_bf16(acc[t][c][3]) : 0u;
            *reinterpret_cast<uint2*>(&S[r][j]) = make_uint2(z0 | (z1 << 16), z2 | (z3 << 16));
        }
    }
}

// the tile transposed into dst ([256][mp]): dst[c][i0 + r] = S[r][c], zero for rows at
// or past m; thread c (one per column) also returns the column's sum over the tile's
// rows, in row order, in fp32
template <int IB>
__device__ __forceinline__ float tile_store_T(bf16 (*S)[HP], bf16* __restrict__ dst, int mp, int i0, int m) {
    const int c = threadIdx.x;
    bf16* d = dst + (size_t)c * mp + i0;
    float s = 0.f;
#pragma unroll 2
    for (int g = 0; g < IB / 8; ++g) {
        unsigned w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 8 * g + 2 * q;
            const bf16 a = i0 + r < m ? S[r][c] : (bf16)0;
            const bf16 b = i0 + r + 1 < m ? S[r + 1][c] : (bf16)0;
            s += from_bf16(a);
            s += from_bf16(b);
            w[q] = a | ((unsigned)b << 16);
        }
        *reinterpret_cast<uint4*>(d + 8 * g) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    return s;
}

// layer 1 (K = 16 features; quarters 2 and 3 of the 32-wide K step are zero) on the
// tile's rows of X into acc
template <int TR>
__device__ __forceinline__ void tile_layer1(const bf16* __restrict__ X, int i0, int m,
                                            const bf16* __restrict__ W1, floatx4 (&acc)[TR][4], int j0,
                                            int lr, int lq) {
    bf16x8_t zero8;
#pragma unroll
    for (int q = 0; q < 8; ++q) zero8[q] = (__bf16)0.f;
    bf16x8_t bw[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) bw[c] = lq < 2 ? ld8(W1 + (size_t)(j0 + c * 16 + lr) * IN + 8 * lq) : zero8;
#pragma unroll
    for (int t = 0; t < TR; ++t) {
        const int i = i0 + t * 16 + lr;
        const bf16x8_t af = (lq < 2 && i < m) ? ld8(X + (size_t)i * IN + 8 * lq) : zero8;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[c], af, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
}

// y for the tile's row `row` = H4 . w5 + b5 in fp32, 256 / IB threads per row (the
// result is valid in every thread of the row)
template <int IB>
__device__ __forceinline__ float tile_head(bf16 (*S)[HP], const float* __restrict__ w5, int row, int part) {
    constexpr int TPR = 256 / IB;              // threads per row
    constexpr int CPT = HID / TPR;             // columns per thread
    float sum = 0.f;
#pragma unroll 4
    for (int j = part * CPT; j < part * CPT + CPT; j += 8) {
        const uint4 u = *reinterpret_cast<const uint4*>(&S[row][j]);
        const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            sum += __uint_as_float(w[q] << 16) * w5[j + 2 * q];
            sum += __uint_as_float(w[q] & 0xffff0000u) * w5[j + 2 * q + 1];
        }
    }
#pragma unroll
    for (int o = 1; o < TPR; o <<= 1) sum += __shfl_xor(sum, o);
    return sum + w5[HID];
}

// Inference on a tile of 16 TR rows of X [m][16] (16-byte aligned rows):
// y = out_scale * (H4 . w5 + b5), non-finite values as +inf.
template <int TR>
__global__ void __launch_bounds__(256, 2)
    k_mlp_fwd(const bf16* __restrict__ X, int m, const bf16* __restrict__ W1, const bf16* __restrict__ W2,
              const bf16* __restrict__ W3, const bf16* __restrict__ W4, const float* __restrict__ params,
              float out_scale, float* __restrict__ y) {
    constexpr int IB = 16 * TR;                // rows per block
    __shared__ __align__(16) bf16 S[IB][HP];
    const int i0 = blockIdx.x * IB;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j0 = wave * 64;                  // this wave's output columns
    const int lr = lane & 15, lq = lane >> 4;  // row in a 16-tile, K quarter
    floatx4 acc[TR][4];
    tile_layer1<TR>(X, i0, m, W1, acc, j0, lr, lq);
    relu_store<TR>(S, acc, params + off_b_dev(1), j0, lr, lq);
    __syncthreads();
    // layers 2..4: the output overwrites the input once every wave has read it
#pragma unroll 1
    for (int l = 2; l <= NLAYER; ++l) {
        tile_layer<TR>(l == 2 ? W2 : l == 3 ? W3 : W4, S, acc, j0, lr, lq);
        __syncthreads();
        relu_store<TR>(S, acc, params + off_b_dev(l), j0, lr, lq);
        __syncthreads();
    }
    const int row = threadIdx.x / (256 / IB), part = threadIdx.x % (256 / IB);
    const float v = out_scale * tile_head<IB>(S, params + off_w5_dev(), row, part);
    const int i = i0 + row;
    if (part == 0 && i < m) y[i] = isfinite(v) ? v : __builtin_huge_valf();
}

// Per-block partial sums a training block leaves for the reduction: db1..db4
// (column sums of dZ_l), dw5 (sum of dy_i H4_i), db5 (sum of dy_i).
constexpr int kBwdPart = NLAYER * HID + HID + 1;

struct MlpTrain {
    const bf16* X;              // [m][16]
    const float* target;        // [m]
    const bf16* W[NLAYER];      // W1..W4 (bf16)
    const bf16* WT[NLAYER - 1]; // W2^T, W3^T, W4^T (bf16 [256][256])
    const float* params;        // fp32: biases, w5, b5
    bf16* T[NLAYER];            // the layers' inputs transposed: X^T [16][mp], H1^T..H3^T [256][mp]
    bf16* dZT[NLAYER];          // dZ1^T..dZ4^T [256][mp]
    float* part;                // [blocks][kBwdPart]
    float* loss_part;           // [blocks]: sum of (y - t)^2 over the block's rows
    int m, mp;
};

// One training pass on a tile of 16 TR rows: the forward (H1..H3 kept in LDS, the
// layers' inputs written transposed for the weight gradients), y and the misfit,
// dy = 2 (y - t) / m, then the backward chain dZ4 -> dZ1 with the ReLU masks read
// from LDS, each dZ written transposed, and the block's bias and head partial sums
// (fixed order).
template <int TR>
__global__ void __launch_bounds__(256) k_mlp_train(MlpTrain a) {
    constexpr int IB = 16 * TR;
    __shared__ __align__(16) bf16 S[IB][HP];                // H4, then dZ4 .. dZ1
    __shared__ __align__(16) bf16 Hs[NLAYER - 1][IB][HP];   // H1..H3
    __shared__ float dys[IB], sq[IB];
    __shared__ float red[8][HID + 1];
    const int i0 = blockIdx.x * IB, m = a.m;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j0 = wave * 64;
    const int lr = lane & 15, lq = lane >> 4;
    float* part = a.part + (size_t)blockIdx.x * kBwdPart;
    // X^T for the first layer's weight gradient
    for (int e = threadIdx.x; e < IN * (IB / 8); e += 256) {
        const int c = e % IN, g = e / IN;
        unsigned w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + 8 * g + 2 * q;
            const unsigned lo = i < m ? a.X[(size_t)i * IN + c] : 0u;
            const unsigned hi = i + 1 < m ? a.X[(size_t)(i + 1) * IN + c] : 0u;
            w[q] = lo | (hi << 16);
        }
        *reinterpret_cast<uint4*>(a.T[0] + (size_t)c * a.mp + i0 + 8 * g) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    // forward: H1..H3 into their own buffers (no overwrite, no barrier before the
    // epilogue), H4 into S
    floatx4 acc[TR][4];
    tile_layer1<TR>(a.X, i0, m, a.W[0], acc, j0, lr, lq);
    relu_store<TR>(Hs[0], acc, a.params + off_b_dev(1), j0, lr, lq);
    __syncthreads();
    tile_store_T<IB>(Hs[0], a.T[1], a.mp, i0, m);
#pragma unroll 1
    for (int l = 2; l <= NLAYER; ++l) {
        tile_layer<TR>(a.W[l - 1], Hs[l - 2], acc, j0, lr, lq);
        relu_store<TR>(l < NLAYER ? Hs[l - 1] : S, acc, a.params + off_b_dev(l), j0, lr, lq);
        __syncthreads();
        if (l < NLAYER) tile_store_T<IB>(Hs[l - 1], a.T[l], a.mp, i0, m);
    }
    // head, misfit, dy
    {
        const int row = threadIdx.x / (256 / IB), pt = threadIdx.x % (256 / IB);
        const float yv = tile_head<IB>(S, a.params + off_w5_dev(), row, pt);
        const int i = i0 + row;
        if (pt == 0) {
            const float d = i < m ? yv - a.target[i] : 0.f;
            dys[row] = 2.f * d / (float)m;
            sq[row] = d * d;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int r = 0; r < IB; ++r) t += sq[r];
        a.loss_part[blockIdx.x] = t;
    }
    {
        // dZ4 = bf16(dy_i w5_j [H4 > 0]) in place; dw5 and db5 partials (thread: 8
        // columns, rows ph, ph + 8, ... in order; then the 8 row phases in order)
        const int cc = threadIdx.x & 31, ph = threadIdx.x >> 5;
        const float* w5 = a.params + off_w5_dev();
        float w5v[8], sw[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            w5v[q] = w5[8 * cc + q];
            sw[q] = 0.f;
        }
        float sd = 0.f;
        for (int r = ph; r < IB; r += 8) {
            const float d = dys[r];
            const uint4 h = *reinterpret_cast<const uint4*>(&S[r][8 * cc]);
            const unsigned hw[4] = {h.x, h.y, h.z, h.w};
            unsigned o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bf16 h0 = (bf16)(hw[q] & 0xffffu), h1 = (bf16)(hw[q] >> 16);
                sw[2 * q] += d * from_bf16(h0);
                sw[2 * q + 1] += d * from_bf16(h1);
                const unsigned z0 = relu_on(h0) ? to_bf16(d * w5v[2 * q]) : 0u;
                const unsigned z1 = relu_on(h1) ? to_bf16(d * w5v[2 * q + 1]) : 0u;
                o[q] = z0 | (z1 << 16);
            }
            sd += d;
            *reinterpret_cast<uint4*>(&S[r][8 * cc]) = make_uint4(o[0], o[1], o[2], o[3]);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) red[ph][8 * cc + q] = sw[q];
        if (cc == 0) red[ph][HID] = sd;
    }
    __syncthreads();
    {
        const int c = threadIdx.x;
        float sum = 0.f;
#pragma unroll
        for (int ph = 0; ph < 8; ++ph) sum += red[ph][c];
        part[NLAYER * HID + c] = sum;
        if (c == 0) {
            float t = 0.f;
#pragma unroll
            for (int ph = 0; ph < 8; ++ph) t += red[ph][HID];
            part[NLAYER * HID + HID] = t;
        }
    }
    part[(NLAYER - 1) * HID + threadIdx.x] = tile_store_T<IB>(S, a.dZT[NLAYER - 1], a.mp, i0, m);
    // backward chain: dZ_{l-1} = bf16((W_l^T dZ_l) [H_{l-1} > 0])
#pragma unroll 1
    for (int l = NLAYER; l >= 2; --l) {
        tile_layer<TR>(a.WT[l - 2], S, acc, j0, lr, lq);
        __syncthreads();                       // every wave has read dZ_l
        mask_store<TR>(S, acc, Hs[l - 2], i0, m, j0, lr, lq);
        __syncthreads();
        part[(l - 2) * HID + threadIdx.x] = tile_store_T<IB>(S, a.dZT[l - 2], a.mp, i0, m);
    }
}

// ---------------------------------------------------------------- weight gradients
// dW_l[j][n] = sum_i dZ_l[i][j] H_{l-1}[i][n] (H_0 = X) over the rows [kb, ke) of a
// split, from the transposed copies (both operands K-contiguous): a block computes 128
// (j) x NB (n) of one layer, K steps of 64 staged through LDS in two buffers (the next
// step's global loads in flight while the current one multiplies); waves 2 x 2 of 64 x 64
// (NB = 128, layers 2..4: block x = 4 (l - 2) + 2 j-tile + n-tile) or 4 x 1 of 32 x 16
// (NB = 16, layer 1: block x = j-tile).  Fixed-order fp32 partials per split.
constexpr int KW = 64;         // K per staged step of the weight gradients
constexpr int KP = KW + 8;     // LDS row pitch (bf16): 144 bytes, conflict-free 16-byte reads

struct MlpWgrad {
    const bf16* dZT[NLAYER];   // [256][mp]
    const bf16* T[NLAYER];     // X^T [16][mp], H1^T, H2^T, H3^T [256][mp]
    float* part;               // [splits][n_params]
    int mp, kend, kchunk;      // kend: m rounded up to 32 (the transposed rows are zero there)
    int n_params;
};

template <int NB>
__device__ __forceinline__ void wgrad_tile(const MlpWgrad& a, int tile, bf16 (*As)[128][KP], bf16 (*Bs)[NB][KP]) {
    constexpr int TJ = NB == 128 ? 4 : 2, TN = NB == 128 ? 4 : 1;
    constexpr int in = NB == 128 ? HID : IN;
    const int l = NB == 128 ? 2 + tile / 4 : 1;
    const int jt = NB == 128 ? (tile >> 1) & 1 : tile, nt = NB == 128 ? tile & 1 : 0;
    const bf16* A = (l == 1 ? a.dZT[0] : l == 2 ? a.dZT[1] : l == 3 ? a.dZT[2] : a.dZT[3]) +
                    (size_t)(jt * 128) * a.mp;
    const bf16* Bm = (l == 1 ? a.T[0] : l == 2 ? a.T[1] : l == 3 ? a.T[2] : a.T[3]) + (size_t)(nt * NB) * a.mp;
    const int kb = blockIdx.y * a.kchunk, ke = min(a.kend, kb + a.kchunk);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lq = lane >> 4;
    const int wj = NB == 128 ? (wave >> 1) * 64 : wave * 32, wn = NB == 128 ? (wave & 1) * 64 : 0;
    floatx4 acc[TJ][TN];
#pragma unroll
    for (int x = 0; x < TJ; ++x)
#pragma unroll
        for (int z = 0; z < TN; ++z) acc[x][z] = floatx4{0.f, 0.f, 0.f, 0.f};
    // staging: A 128 rows x 8 chunks of 16 bytes (4 per thread), B NB rows x 8 chunks;
    // chunks at or past ke (a multiple of 32) are zero
    uint4 ra[4], rb[4];
    auto gload = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = threadIdx.x + 256 * u, row = e >> 3, q = e & 7;
            const bool in_k = k0 + 8 * q < ke;
            ra[u] = in_k ? *reinterpret_cast<const uint4*>(A + (size_t)row * a.mp + k0 + 8 * q) : make_uint4(0u, 0u, 0u, 0u);
            if (e < NB * 8)
                rb[u] = in_k ? *reinterpret_cast<const uint4*>(Bm + (size_t)row * a.mp + k0 + 8 * q)
                             : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = threadIdx.x + 256 * u, row = e >> 3, q = e & 7;
            *reinterpret_cast<uint4*>(&As[buf][row][8 * q]) = ra[u];
            if (e < NB * 8) *reinterpret_cast<uint4*>(&Bs[buf][row][8 * q]) = rb[u];
        }
    };
    if (kb < ke) {
        gload(kb);
        lstore(0);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = kb; k0 < ke; k0 += KW) {
        const bool more = k0 + KW < ke;
        if (more) gload(k0 + KW);
#pragma unroll
        for (int kk = 0; kk < KW; kk += 32) {
            bf16x8_t af[TJ], bfr[TN];
#pragma unroll
            for (int x = 0; x < TJ; ++x)
                af[x] = *reinterpret_cast<const bf16x8_t*>(&As[buf][wj + x * 16 + lr][kk + 8 * lq]);
#pragma unroll
            for (int z = 0; z < TN; ++z)
                bfr[z] = *reinterpret_cast<const bf16x8_t*>(&Bs[buf][wn + z * 16 + lr][kk + 8 * lq]);
#pragma unroll
            for (int x = 0; x < TJ; ++x)
#pragma unroll
                for (int z = 0; z < TN; ++z)
                    acc[x][z] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[x], bfr[z], acc[x][z], 0, 0, 0);
        }
        if (more) lstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // lane holds D[j = wj + 16 x + 4 lq + r][n = wn + 16 z + lr]
    float* out = a.part + (size_t)blockIdx.y * a.n_params + off_W_dev(l);
#pragma unroll
    for (int x = 0; x < TJ; ++x)
#pragma unroll
        for (int z = 0; z < TN; ++z)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = jt * 128 + wj + x * 16 + 4 * lq + r, n = nt * NB + wn + z * 16 + lr;
                out[(size_t)j * in + n] = acc[x][z][r];
            }
}

// blocks x < 12: layers 2..4 (NB = 128); x = 12, 13: layer 1 (NB = 16); y: the split
constexpr int kWgradTiles = 4 * (NLAYER - 1) + HID / 128;
__global__ void __launch_bounds__(256) k_mlp_wgrad(MlpWgrad a) {
    __shared__ __align__(16) bf16 As[2][128][KP];
    __shared__ __align__(16) bf16 Bs[2][128][KP];
    if (blockIdx.x < 4 * (NLAYER - 1))
        wgrad_tile<128>(a, blockIdx.x, As, Bs);
    else
        wgrad_tile<16>(a, blockIdx.x - 4 * (NLAYER - 1), As, reinterpret_cast<bf16(*)[16][KP]>(&Bs[0][0][0]));
}

// weight gradients: the splits' partials of each W1..W4 entry, summed in split order
__global__ void k_mlp_reduce_w(const float* __restrict__ pw, int splits, int n_params, float* __restrict__ g) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_params) return;
    bool weight = false;
    for (int l = 1; l <= NLAYER; ++l) weight |= e >= off_W_dev(l) && e < off_b_dev(l);
    if (!weight) return;
    float s = 0.f;
#pragma unroll 8
    for (int z = 0; z < splits; ++z) s += pw[(size_t)z * n_params + e];
    g[e] = s;
}

// b1..b4, w5, b5: one wave per entry; lane k sums the backward blocks k, k + 64, ... in
// order, then a fixed butterfly adds the lanes (the same order on every call)
__global__ void k_mlp_reduce_b(const float* __restrict__ pb, int blocks, float* __restrict__ g) {
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (col >= kBwdPart) return;
    float s = 0.f;
    for (int b = lane; b < blocks; b += 64) s += pb[(size_t)b * kBwdPart + col];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0)
        g[col < NLAYER * HID ? off_b_dev(col / HID + 1) + col % HID : off_w5_dev() + (col - NLAYER * HID)] = s;
}

// Rows per block (16 TR) of the row-tile kernels: a larger tile fetches the weights
// fewer times per row, more blocks hide more latency; the steps are where the
// measured forward and training times cross (128 rows from 65536 rows, 64 from
// 16384, else 32).
__host__ int tile_rows(int m) { return m >= 65536 ? 128 : m >= 16384 ? 64 : 32; }
// Rows per block of the training pass (H1..H3 stay in LDS: 32 rows take 76 KB, two
// blocks per CU; 64 rows 144 KB, one)
__host__ int train_rows(int m) { return m >= 65536 ? 64 : 32; }
// inference keeps nothing per row on the device: any batch up to 2^27 rows
constexpr int kInferRowsMax = 1 << 27;

// The bf16 copies of the hidden weights the kernels read: W1..W4 as stored and
// W2^T..W4^T (WT[n][j] = W[j][n]) for the backward chain.
struct MlpCopies {
    bf16* w[NLAYER];
    bf16* wT;   // [3][256][256]
};

__device__ __forceinline__ void write_copies(const MlpCopies& c, int e, float v) {
#pragma unroll
    for (int l = 1; l <= NLAYER; ++l)
        if (e >= off_W_dev(l) && e < off_b_dev(l)) {
            const int k = e - off_W_dev(l);
            const bf16 h = to_bf16(v);
            c.w[l - 1][k] = h;
            if (l > 1) c.wT[(size_t)(l - 2) * HID * HID + (k % HID) * HID + k / HID] = h;
        }
}

__global__ void k_refresh_copies(const float* __restrict__ p, int n, MlpCopies c) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) write_copies(c, t, p[t]);
}

// one Adam step on the fp32 masters, refreshing their bf16 copies
__global__ void k_adam_flat(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float c1, float c2, MlpCopies c) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gi = g[t];
    const float mi = 0.9f * m[t] + 0.1f * gi;
    const float vi = 0.999f * v[t] + 0.001f * gi * gi;
    m[t] = mi;
    v[t] = vi;
    const float pi = p[t] - lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
    p[t] = pi;
    write_copies(c, t, pi);
}

// ---------------------------------------------------------------- features
// Per row (15 used + 1 zero pad): position relative to the centre / len_scale (3),
// fibre direction (3), the eight root features
//     a_r = |x - x_r| / len_scale + t_r / time_scale
// sorted ascending (so the set of roots enters symmetrically and the first one
// is the nearest-root guess; fewer than 8 roots repeat root 0), velocity scale.
// With T given, the row's training target T[i] / time_scale is written as well.
__global__ void k_features(const float* __restrict__ xyz, const float* __restrict__ fibre,
                           const float* __restrict__ vscale, int n_v, const int* __restrict__ rows,
                           int n_rows, const float* __restrict__ root_xyz,
                           const float* __restrict__ root_t, int n_roots, float cx, float cy,
                           float cz, float len_scale, float time_scale, const float* __restrict__ T,
                           bf16* __restrict__ X, float* __restrict__ target) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int i = rows ? rows[r] : r;
    bf16* o = X + (size_t)r * IN;
    if (i < 0 || i >= n_v) {   // invalid row id: zero features, NaN target
        for (int k = 0; k < IN; ++k) o[k] = 0;
        if (target) target[r] = __builtin_nanf("");
        return;
    }
    const float x = xyz[3 * (size_t)i], y = xyz[3 * (size_t)i + 1], z = xyz[3 * (size_t)i + 2];
    const float il = 1.f / len_scale, it = 1.f / time_scale;
    float a[8];
    for (int k = 0; k < 8; ++k) {
        const int q = k < n_roots ? k : 0;
        const float dx = x - root_xyz[3 * q], dy = y - root_xyz[3 * q + 1], dz = z - root_xyz[3 * q + 2];
        a[k] = sqrtf(dx * dx + dy * dy + dz * dz) * il + root_t[q] * it;
    }
    for (int k = 1; k < 8; ++k) {   // insertion sort, 8 values
        const float v = a[k];
        int j = k - 1;
        while (j >= 0 && a[j] > v) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = v;
    }
    o[0] = to_bf16((x - cx) * il);
    o[1] = to_bf16((y - cy) * il);
    o[2] = to_bf16((z - cz) * il);
    o[3] = to_bf16(fibre[3 * (size_t)i]);
    o[4] = to_bf16(fibre[3 * (size_t)i + 1]);
    o[5] = to_bf16(fibre[3 * (size_t)i + 2]);
    for (int k = 0; k < 8; ++k) o[6 + k] = to_bf16(a[k]);
    o[14] = to_bf16(vscale ? vscale[i] : 1.f);
    o[15] = 0;
    if (T && target) target[r] = T[i] * it;
}

}  // namespace

// ====================================================================== host
struct gbp_mlp_s {
    int device = 0;
    int max_rows = 0;
    int mp = 0;                // row pitch of the transposed training buffers
    int n_params = 0;
    int step = 0;
    float* params = nullptr;   // fp32 masters, flat
    float* grads = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    bf16* wbf[NLAYER] = {};    // bf16 copies of W1..W4
    bf16* wT = nullptr;        // bf16 W2^T, W3^T, W4^T [3][256][256]
    bf16* T = nullptr;         // X^T [16][mp], H1^T..H3^T [3][256][mp]
    bf16* dZT = nullptr;       // dZ1^T..dZ4^T [4][256][mp]
    float* part = nullptr;     // loss partials, one per training block
    float* part_w = nullptr;   // weight-gradient partials [kMaxSplits][n_params]
    float* part_b = nullptr;   // backward-chain partials [blocks][kBwdPart]
    float* loss = nullptr;     // [1]
};

namespace {
// flat layout: W1 [256x16], b1, W2 [256x256], b2, W3, b3, W4, b4, w5 [256], b5 [1]
int off_W(int l) { return off_W_dev(l); }   // l = 1..4
int off_b(int l) { return off_b_dev(l); }
int off_w5() { return off_w5_dev(); }
int n_params_total() { return off_w5() + HID + 1; }
int in_dim(int l) { return l == 1 ? IN : HID; }

// Row chunks of the weight-gradient splits: at most kMaxSplits chunks of a multiple of
// the staged K step, at least 256 rows.
constexpr int kMaxSplits = 32;
int wgrad_chunk(int kend) { return std::max(256, ((kend + kMaxSplits - 1) / kMaxSplits + KW - 1) / KW * KW); }

void free_mlp(gbp_mlp p) {
    if (!p) return;
    void* ptrs[] = {p->params, p->grads, p->m, p->v, p->wT, p->T, p->dZT, p->part, p->part_w, p->part_b,
                    p->loss};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    for (int l = 0; l < NLAYER; ++l)
        if (p->wbf[l]) (void)hipFree(p->wbf[l]);
    delete p;
}

MlpCopies copies_of(gbp_mlp p) {
    MlpCopies c{};
    for (int l = 0; l < NLAYER; ++l) c.w[l] = p->wbf[l];
    c.wT = p->wT;
    return c;
}

int refresh_bf16(gbp_mlp p, hipStream_t s) {
    k_refresh_copies<<<gbp_blocks(p->n_params, 256), 256, 0, s>>>(p->params, p->n_params, copies_of(p));
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

// the network on m rows of X, y = out_scale * prediction
void launch_infer(gbp_mlp p, const bf16* X, int m, float out_scale, float* y, hipStream_t s) {
    const int ib = tile_rows(m), blocks = (m + ib - 1) / ib;
    if (ib == 128)
        k_mlp_fwd<8><<<blocks, 256, 0, s>>>(X, m, p->wbf[0], p->wbf[1], p->wbf[2], p->wbf[3], p->params, out_scale, y);
    else if (ib == 64)
        k_mlp_fwd<4><<<blocks, 256, 0, s>>>(X, m, p->wbf[0], p->wbf[1], p->wbf[2], p->wbf[3], p->params, out_scale, y);
    else
        k_mlp_fwd<2><<<blocks, 256, 0, s>>>(X, m, p->wbf[0], p->wbf[1], p->wbf[2], p->wbf[3], p->params, out_scale, y);
}

// training pass (forward, misfit, backward chain), weight gradients, reductions into
// p->grads and p->loss
void launch_train(gbp_mlp p, const bf16* X, int m, const float* target, hipStream_t s) {
    MlpTrain a{};
    a.X = X;
    a.target = target;
    for (int l = 0; l < NLAYER; ++l) a.W[l] = p->wbf[l];
    for (int l = 0; l < NLAYER - 1; ++l) a.WT[l] = p->wT + (size_t)l * HID * HID;
    a.params = p->params;
    a.T[0] = p->T;
    for (int l = 1; l < NLAYER; ++l) a.T[l] = p->T + (size_t)(IN + (l - 1) * HID) * p->mp;
    for (int l = 0; l < NLAYER; ++l) a.dZT[l] = p->dZT + (size_t)l * HID * p->mp;
    a.part = p->part_b;
    a.loss_part = p->part;
    a.m = m;
    a.mp = p->mp;
    const int ib = train_rows(m), blocks = (m + ib - 1) / ib;
    if (ib == 64) k_mlp_train<4><<<blocks, 256, 0, s>>>(a);
    else k_mlp_train<2><<<blocks, 256, 0, s>>>(a);
    k_sum_parts<<<1, 256, 0, s>>>(p->part, blocks, 1.f / (float)m, p->loss);
    MlpWgrad w{};
    for (int l = 0; l < NLAYER; ++l) {
        w.dZT[l] = a.dZT[l];
        w.T[l] = a.T[l];
    }
    w.part = p->part_w;
    w.mp = p->mp;
    w.kend = (m + 31) / 32 * 32;
    w.kchunk = wgrad_chunk(w.kend);
    w.n_params = p->n_params;
    const int splits = (w.kend + w.kchunk - 1) / w.kchunk;
    k_mlp_wgrad<<<dim3(kWgradTiles, splits), 256, 0, s>>>(w);
    k_mlp_reduce_w<<<gbp_blocks(p->n_params, 256), 256, 0, s>>>(p->part_w, splits, p->n_params, p->grads);
    k_mlp_reduce_b<<<(kBwdPart + 3) / 4, 256, 0, s>>>(p->part_b, blocks, p->grads);
}

int check_rows(gbp_mlp p, int m) {
    if (!p || m < 1 || m > p->max_rows) {
        gbp_set_error("mlp: rows must be in [1, max_rows=%d]", p ? p->max_rows : 0);
        return GBP_ERR_ARG;
    }
    return GBP_OK;
}
}  // namespace

extern "C" int gbp_mlp_create(int max_rows, uint64_t seed, gbp_mlp* out) {
    if (!out || max_rows < 1 || max_rows > (1 << 21)) {
        gbp_set_error("mlp: need 1 <= max_rows <= 2097152");
        return GBP_ERR_ARG;
    }
    *out = nullptr;
    gbp_mlp p = new gbp_mlp_s();
    (void)hipGetDevice(&p->device);
    p->max_rows = max_rows;
    p->n_params = n_params_total();
    p->mp = (max_rows + 127) / 128 * 128;
    const size_t mr = (size_t)max_rows, mp = (size_t)p->mp;
    bool ok = hipMalloc((void**)&p->params, sizeof(float) * p->n_params) == hipSuccess &&
              hipMalloc((void**)&p->grads, sizeof(float) * p->n_params) == hipSuccess &&
              hipMalloc((void**)&p->m, sizeof(float) * p->n_params) == hipSuccess &&
              hipMalloc((void**)&p->v, sizeof(float) * p->n_params) == hipSuccess &&
              hipMalloc((void**)&p->wT, sizeof(bf16) * (NLAYER - 1) * HID * HID) == hipSuccess &&
              hipMalloc((void**)&p->T, sizeof(bf16) * (IN + (NLAYER - 1) * HID) * mp) == hipSuccess &&
              hipMalloc((void**)&p->dZT, sizeof(bf16) * NLAYER * HID * mp) == hipSuccess &&
              hipMalloc((void**)&p->part, sizeof(float) * ((mr + 31) / 32)) == hipSuccess &&
              hipMalloc((void**)&p->part_w, sizeof(float) * kMaxSplits * p->n_params) == hipSuccess &&
              hipMalloc((void**)&p->part_b, sizeof(float) * ((mr + 31) / 32) * kBwdPart) == hipSuccess &&
              hipMalloc((void**)&p->loss, sizeof(float)) == hipSuccess;
    for (int l = 1; ok && l <= NLAYER; ++l)
        ok = hipMalloc((void**)&p->wbf[l - 1], sizeof(bf16) * HID * in_dim(l)) == hipSuccess;
    if (!ok) {
        gbp_set_error("mlp: allocation failed");
        free_mlp(p);
        return GBP_ERR_NOMEM;
    }
    // He-normal initialisation of the weights, zero biases
    std::vector<float> h(p->n_params, 0.f);
    std::mt19937_64 rng(seed);
    for (int l = 1; l <= NLAYER; ++l) {
        std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (l == 1 ? 15.f : (float)HID)));
        for (int k = 0; k < HID * in_dim(l); ++k) h[off_W(l) + k] = nd(rng);
        if (l == 1)
            for (int j = 0; j < HID; ++j) h[off_W(1) + j * IN + (IN - 1)] = 0.f;   // pad input
    }
    std::normal_distribution<float> nd5(0.f, std::sqrt(1.f / HID));
    for (int j = 0; j < HID; ++j) h[off_w5() + j] = nd5(rng);
    if (hipMemcpy(p->params, h.data(), sizeof(float) * p->n_params, hipMemcpyHostToDevice) ||
        hipMemset(p->m, 0, sizeof(float) * p->n_params) || hipMemset(p->v, 0, sizeof(float) * p->n_params) ||
        refresh_bf16(p, nullptr) || hipDeviceSynchronize()) {
        gbp_set_error("mlp: initialisation failed");
        free_mlp(p);
        return GBP_ERR_HIP;
    }
    *out = p;
    return GBP_OK;
}

extern "C" void gbp_mlp_destroy(gbp_mlp p) { free_mlp(p); }

extern "C" int gbp_mlp_num_params(gbp_mlp p) { return p ? p->n_params : 0; }

extern "C" int gbp_mlp_set_params(gbp_mlp p, const float* host, void* stream) {
    if (!p || !host) {
        gbp_set_error("mlp: NULL argument");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    GBP_HIP(hipMemcpyAsync(p->params, host, sizeof(float) * p->n_params, hipMemcpyHostToDevice, s));
    GBP_HIP(hipStreamSynchronize(s));
    return refresh_bf16(p, s);
}

extern "C" int gbp_mlp_get_params(gbp_mlp p, float* host, float* grads_host, void* stream) {
    if (!p || (!host && !grads_host)) {
        gbp_set_error("mlp: NULL argument");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    if (host)
        GBP_HIP(hipMemcpyAsync(host, p->params, sizeof(float) * p->n_params, hipMemcpyDeviceToHost, s));
    if (grads_host)
        GBP_HIP(hipMemcpyAsync(grads_host, p->grads, sizeof(float) * p->n_params,
                               hipMemcpyDeviceToHost, s));
    GBP_HIP(hipStreamSynchronize(s));
    return GBP_OK;
}

extern "C" int gbp_mlp_get_state(gbp_mlp p, float* m_host, float* v_host, int* step, void* stream) {
    if (!p || !m_host || !v_host || !step) {
        gbp_set_error("mlp_get_state: NULL argument");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    GBP_HIP(hipMemcpyAsync(m_host, p->m, sizeof(float) * p->n_params, hipMemcpyDeviceToHost, s));
    GBP_HIP(hipMemcpyAsync(v_host, p->v, sizeof(float) * p->n_params, hipMemcpyDeviceToHost, s));
    GBP_HIP(hipStreamSynchronize(s));
    *step = p->step;
    return GBP_OK;
}

extern "C" int gbp_mlp_set_state(gbp_mlp p, const float* m_host, const float* v_host, int step,
                                 void* stream) {
    if (!p || !m_host || !v_host || step < 0) {
        gbp_set_error("mlp_set_state: NULL argument or step < 0");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    GBP_HIP(hipMemcpyAsync(p->m, m_host, sizeof(float) * p->n_params, hipMemcpyHostToDevice, s));
    GBP_HIP(hipMemcpyAsync(p->v, v_host, sizeof(float) * p->n_params, hipMemcpyHostToDevice, s));
    GBP_HIP(hipStreamSynchronize(s));
    p->step = step;
    return GBP_OK;
}

extern "C" int gbp_mlp_features(const float* xyz, const float* fibre, const float* vscale, int n_v,
                                const int32_t* rows, int n_rows, const float* root_xyz,
                                const float* root_t, int n_roots, const float* norm,
                                const float* T, uint16_t* X, float* target, void* stream) {
    if (!xyz || !fibre || !root_xyz || !root_t || !norm || !X || n_v < 1 || n_rows < 1 ||
        (!rows && n_rows > n_v) || n_roots < 1 ||
        n_roots > 8 || !(norm[3] > 0.f) || !(norm[4] > 0.f) || (!T != !target)) {
        gbp_set_error("mlp_features: bad arguments (1 <= n_roots <= 8, scales > 0, T and target together)");
        return GBP_ERR_ARG;
    }
    k_features<<<gbp_blocks(n_rows, 256), 256, 0, (hipStream_t)stream>>>(
        xyz, fibre, vscale, n_v, rows, n_rows, root_xyz, root_t, n_roots, norm[0], norm[1], norm[2],
        norm[3], norm[4], T, (bf16*)X, target);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_mlp_forward(gbp_mlp p, const uint16_t* X, int m, float out_scale, float* y,
                               void* stream) {
    if (!p || m < 1 || m > kInferRowsMax) {
        gbp_set_error("mlp_forward: rows must be in [1, %d]", kInferRowsMax);
        return GBP_ERR_ARG;
    }
    if (!X || !y) {
        gbp_set_error("mlp_forward: NULL argument");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    if (reinterpret_cast<uintptr_t>(X) & 15) {
        gbp_set_error("mlp_forward: X must be 16-byte aligned");
        return GBP_ERR_ARG;
    }
    launch_infer(p, (const bf16*)X, m, out_scale, y, s);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_mlp_gradient(gbp_mlp p, const uint16_t* X, int m, const float* target,
                                float* loss, void* stream) {
    int rc = check_rows(p, m);
    if (rc) return rc;
    if (!X || !target) {
        gbp_set_error("mlp_gradient: NULL argument");
        return GBP_ERR_ARG;
    }
    if (reinterpret_cast<uintptr_t>(X) & 15) {
        gbp_set_error("mlp_gradient: X must be 16-byte aligned");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    launch_train(p, (const bf16*)X, m, target, s);
    GBP_LAUNCH_CHECK();
    if (loss) GBP_HIP(hipMemcpyAsync(loss, p->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
    return GBP_OK;
}

extern "C" int gbp_mlp_train_step(gbp_mlp p, const uint16_t* X, int m, const float* target,
                                  float lr, float* loss, void* stream) {
    int rc = gbp_mlp_gradient(p, X, m, target, loss, stream);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    p->step += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, p->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, p->step)));
    k_adam_flat<<<gbp_blocks(p->n_params, 256), 256, 0, s>>>(p->params, p->grads, p->m, p->v,
                                                             p->n_params, lr, c1, c2, copies_of(p));
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}
