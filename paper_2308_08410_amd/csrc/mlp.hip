// Learned warm start: a small MLP (16 inputs -> 4 x 256 ReLU -> 1) that predicts
// activation times from per-vertex features, trained and evaluated with BF16
// matrix-core kernels (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// Precision policy (mirrored by the reference):
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

// ---------------------------------------------------------------- GEMM
// C[i][j] = sum_k A(i,k) B(k,j) with A(i,k) = A[i*ar + k*ac], B(k,j) = B[k*br + j*bc]
// (bf16), 64x64 tile per block of 4 waves, each wave 32x32 = 2x2 tiles of
// v_mfma_f32_16x16x32_bf16, K in steps of 32 staged through LDS (B stored
// transposed so that a lane's 8 consecutive K values are one 16-byte read).
// MFMA 16x16x32 lane layout: lane l holds A[l % 16][8 (l / 16) + q] and
// B[8 (l / 16) + q][l % 16], q = 0..7, and returns D[4 (l / 16) + r][l % 16].
enum { EPI_BIAS_RELU = 0, EPI_MASK = 1, EPI_PARTIAL = 2 };
constexpr int KS = 32;          // K per staged step
constexpr int KP = KS + 8;      // LDS row pitch (bf16): 80 bytes, 16-byte aligned rows

template <int EPI>
__global__ void __launch_bounds__(256)
    k_gemm(const bf16* __restrict__ A, int ar, int ac, const bf16* __restrict__ Bm, int br, int bc,
           int M, int N, int K, int kchunk, const float* __restrict__ bias,
           const bf16* __restrict__ mask, bf16* __restrict__ out, float* __restrict__ part) {
    __shared__ __align__(16) bf16 As[64][KP];
    __shared__ __align__(16) bf16 Bt[64][KP];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    floatx4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += KS) {
        for (int e = threadIdx.x; e < 64 * KS; e += 256) {
            const int r = e / KS, kk = e % KS;
            const int gi = i0 + r, gk = k0 + kk;
            As[r][kk] = (gi < M && gk < ke) ? A[(size_t)gi * ar + (size_t)gk * ac] : (bf16)0;
            const int gj = j0 + r;
            Bt[r][kk] = (gj < N && gk < ke) ? Bm[(size_t)gk * br + (size_t)gj * bc] : (bf16)0;
        }
        __syncthreads();
        bf16x8_t af[2], bfv[2];
        const int kq = (lane >> 4) * 8;
        for (int t = 0; t < 2; ++t) {
            const int ra = wi + t * 16 + (lane & 15), rb = wj + t * 16 + (lane & 15);
            af[t] = *reinterpret_cast<const bf16x8_t*>(&As[ra][kq]);
            bfv[t] = *reinterpret_cast<const bf16x8_t*>(&Bt[rb][kq]);
        }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfv[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + a * 16 + (lane >> 4) * 4 + r;
                const int j = j0 + wj + b * 16 + (lane & 15);
                if (i >= M || j >= N) continue;
                const float v = acc[a][b][r];
                if (EPI == EPI_BIAS_RELU) {
                    out[(size_t)i * N + j] = to_bf16(fmaxf(v + bias[j], 0.f));
                } else if (EPI == EPI_MASK) {
                    const bf16 h = mask[(size_t)i * N + j];
                    out[(size_t)i * N + j] = to_bf16((h != 0 && !(h & 0x8000)) ? v : 0.f);
                } else {
                    part[(size_t)blockIdx.z * M * N + (size_t)i * N + j] = v;
                }
            }
}

// sum of split-K partials (fixed order)
__global__ void k_reduce_parts(const float* __restrict__ part, int splits, int n,
                               float* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[(size_t)z * n + t];
    out[t] = s;
}

// column sums of a bf16 [m x n] matrix (bias gradients), fixed order per column
// Column sums (bias gradients) in two fixed-order passes: block (g, r) sums, for 64
// columns of group g, the rows [r R, (r+1) R) (4 row phases, then the phases in
// order) into part[r][c]; k_reduce_parts then adds the row blocks in order.
// WEIGHTED: sum_i w_i X[i][c], and column n (one past the last) gives sum_i w_i.
template <bool WEIGHTED>
__global__ void k_colsum_part(const bf16* __restrict__ X, const float* __restrict__ w, int m, int n,
                              int R, float* __restrict__ part) {
    __shared__ float red[4][64];
    const int cl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cl;
    const int ncol = WEIGHTED ? n + 1 : n;
    const int r0 = blockIdx.y * R, r1 = min(m, r0 + R);
    float acc = 0.f;
    if (c < ncol)
        for (int i = r0 + q; i < r1; i += 4) {
            const float x = c < n ? from_bf16(X[(size_t)i * n + c]) : 1.f;
            acc += WEIGHTED ? w[i] * x : x;
        }
    red[q][cl] = acc;
    __syncthreads();
    if (q == 0 && c < ncol)
        part[(size_t)blockIdx.y * ncol + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

// ---------------------------------------------------------------- head, loss
// y_i = H4_i . w5 + b5 (16 lanes per row, fp32)
__global__ void k_head(const bf16* __restrict__ H, int m, const float* __restrict__ w5,
                       const float* __restrict__ b5, float* __restrict__ y) {
    const int lane = threadIdx.x & 15;
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    if (i >= m) return;
    float s = 0.f;
    for (int j = lane; j < HID; j += 16) s += from_bf16(H[(size_t)i * HID + j]) * w5[j];
    for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) y[i] = s + b5[0];
}

// dy = 2 (y - t) / m, squared error partial sums per block
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t, int m,
                      float* __restrict__ dy, float* __restrict__ part) {
    __shared__ float sh[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float e = 0.f;
    if (i < m) {
        const float d = y[i] - t[i];
        dy[i] = 2.f * d / (float)m;
        e = d * d;
    }
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

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

// dZ4 = bf16(dy_i w5_j [H4 > 0])
__global__ void k_head_bwd(const float* __restrict__ dy, const bf16* __restrict__ H, int m,
                           const float* __restrict__ w5, bf16* __restrict__ dZ) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)m * HID) return;
    const int i = (int)(t / HID), j = (int)(t % HID);
    const bf16 h = H[t];
    dZ[t] = to_bf16((h != 0 && !(h & 0x8000)) ? dy[i] * w5[j] : 0.f);
}

// ---------------------------------------------------------------- fused inference
// The whole network for a tile of 16 TR rows in one block of 4 waves: the
// activations stay in LDS (16 TR x 256 bf16, overwritten layer by layer), only
// the features come in and the predictions go out.  Wave w computes the output
// columns [64 w, 64 w + 64) of a layer for all the tile's rows as the transposed
// product W H^T: TR x 4 tiles of v_mfma_f32_16x16x32_bf16 per K step of 32, the
// A operand (a weight row's 8 consecutive K values) loaded straight from global
// memory (a layer's 128 KB of weights stay in L2; each fragment serves 16 TR
// rows), the B operand (an activation row's 8 K values) read from LDS, the next
// step's weight fragments in flight while the current step multiplies.  A
// layer's output overwrites its input only after every wave has finished
// reading it.  Rounding as in the layered kernels: H = bf16(relu(fp32 acc + b)),
// the head in fp32.
constexpr int HP = HID + 8;   // LDS row pitch (bf16): 528 bytes, 16-byte aligned rows

__device__ __forceinline__ bf16x8_t ld8(const bf16* p) {
    return *reinterpret_cast<const bf16x8_t*>(p);
}

// layer output bf16(relu(acc + b)) into the wave's 64 columns of H.  The tiles
// hold the layer's output transposed (column j of the layer = row of the tile),
// so a lane's 4 values are 4 consecutive columns of one row: one 8-byte store.
template <int TR>
__device__ __forceinline__ void infer_store(bf16 (*H)[HP], const floatx4 (&acc)[TR][4],
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
            *reinterpret_cast<uint2*>(&H[t * 16 + lr][j]) = make_uint2(lo, hi);
        }
    }
}

template <int TR>
__global__ void __launch_bounds__(256, 2)
    k_mlp_infer(const bf16* __restrict__ X, int m, const bf16* __restrict__ W1,
                const bf16* __restrict__ W2, const bf16* __restrict__ W3, const bf16* __restrict__ W4,
                const float* __restrict__ params, float out_scale, float* __restrict__ y) {
    constexpr int IB = 16 * TR;                // rows per block
    __shared__ __align__(16) bf16 H[IB][HP];
    const int i0 = blockIdx.x * IB;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j0 = wave * 64;                  // this wave's output columns
    const int lr = lane & 15, lq = lane >> 4;  // row (A) / column (B) in a 16-tile, K quarter
    floatx4 acc[TR][4];
    bf16x8_t zero8;
#pragma unroll
    for (int q = 0; q < 8; ++q) zero8[q] = (__bf16)0.f;
    // layer 1: K = 16 features; quarters 2 and 3 of the 32-wide K step are zero
    {
        bf16x8_t bw[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bw[c] = lq < 2 ? ld8(W1 + (size_t)(j0 + c * 16 + lr) * IN + 8 * lq) : zero8;
#pragma unroll
        for (int t = 0; t < TR; ++t) {
            const int i = i0 + t * 16 + lr;
            const bf16x8_t af = (lq < 2 && i < m) ? ld8(X + (size_t)i * IN + 8 * lq) : zero8;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[c], af, floatx4{0.f, 0.f, 0.f, 0.f},
                                                                    0, 0, 0);
        }
        infer_store<TR>(H, acc, params + off_b_dev(1), j0, lr, lq);
        __syncthreads();
    }
    // layers 2..4: K = 256 in 8 steps
#pragma unroll 1
    for (int l = 2; l <= NLAYER; ++l) {
        const bf16* W = l == 2 ? W2 : l == 3 ? W3 : W4;
#pragma unroll
        for (int t = 0; t < TR; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[t][c] = floatx4{0.f, 0.f, 0.f, 0.f};
        bf16x8_t bw[4], bn[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bw[c] = ld8(W + (size_t)(j0 + c * 16 + lr) * HID + 8 * lq);
#pragma unroll 2
        for (int ks = 0; ks < HID / 32; ++ks) {
            if (ks + 1 < HID / 32) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    bn[c] = ld8(W + (size_t)(j0 + c * 16 + lr) * HID + (ks + 1) * 32 + 8 * lq);
            }
#pragma unroll
            for (int t = 0; t < TR; ++t) {
                const bf16x8_t af = *reinterpret_cast<const bf16x8_t*>(&H[t * 16 + lr][ks * 32 + 8 * lq]);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[c], af, acc[t][c], 0, 0, 0);
            }
            if (ks + 1 < HID / 32) {
#pragma unroll
                for (int c = 0; c < 4; ++c) bw[c] = bn[c];
            }
        }
        __syncthreads();                       // every wave has read this layer's input
        infer_store<TR>(H, acc, params + off_b_dev(l), j0, lr, lq);
        __syncthreads();
    }
    // head: y = H4 . w5 + b5 in fp32, 256 / IB threads per row
    constexpr int TPR = 256 / IB;              // threads per row
    constexpr int CPT = HID / TPR;             // columns per thread
    const float* w5 = params + off_w5_dev();
    const int row = threadIdx.x / TPR, part = threadIdx.x % TPR;
    float sum = 0.f;
#pragma unroll 4
    for (int j = part * CPT; j < part * CPT + CPT; j += 8) {
        const uint4 u = *reinterpret_cast<const uint4*>(&H[row][j]);
        const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            sum += __uint_as_float(w[q] << 16) * w5[j + 2 * q];
            sum += __uint_as_float(w[q] & 0xffff0000u) * w5[j + 2 * q + 1];
        }
    }
#pragma unroll
    for (int o = 1; o < TPR; o <<= 1) sum += __shfl_xor(sum, o);
    const int i = i0 + row;
    if (part == 0 && i < m) {
        const float v = out_scale * (sum + w5[HID]);
        y[i] = isfinite(v) ? v : __builtin_huge_valf();
    }
}
// rows per block 16 TR: 128 once there are enough rows to give every CU a block
// (fewer weight fetches per row), else 64 (more blocks for small batches)
constexpr int kInferRowsLarge = 32768;
// inference keeps nothing per row on the device: any batch up to 2^27 rows
constexpr int kInferRowsMax = 1 << 27;

// prediction out: scale * y, non-finite values as +inf (no information)
__global__ void k_scale_out(const float* __restrict__ y, int m, float scale, float* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const float v = scale * y[t];
    out[t] = isfinite(v) ? v : __builtin_huge_valf();
}

__global__ void k_cast_bf16(const float* __restrict__ x, int n, bf16* __restrict__ y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = to_bf16(x[t]);
}

__global__ void k_adam_flat(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gi = g[t];
    const float mi = 0.9f * m[t] + 0.1f * gi;
    const float vi = 0.999f * v[t] + 0.001f * gi * gi;
    m[t] = mi;
    v[t] = vi;
    p[t] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
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
    int n_params = 0;
    int step = 0;
    float* params = nullptr;   // fp32 masters, flat
    float* grads = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    bf16* wbf[NLAYER] = {};    // bf16 copies of W1..W4
    bf16* H[NLAYER + 1] = {};  // H[0] unused (X is the input), H[1..4] activations [rows x 256]
    bf16* dZ[2] = {};          // ping-pong [rows x 256]
    float* y = nullptr;
    float* dy = nullptr;
    float* part = nullptr;     // split-K partials / loss partials
    size_t part_n = 0;
    float* loss = nullptr;     // [1]
};

namespace {
// flat layout: W1 [256x16], b1, W2 [256x256], b2, W3, b3, W4, b4, w5 [256], b5 [1]
int off_W(int l) {   // l = 1..4
    if (l == 1) return 0;
    return HID * IN + HID + (l - 2) * (HID * HID + HID);
}
int off_b(int l) { return off_W(l) + (l == 1 ? HID * IN : HID * HID); }
int off_w5() { return off_W(4) + HID * HID + HID; }
int n_params_total() { return off_w5() + HID + 1; }
int in_dim(int l) { return l == 1 ? IN : HID; }

void free_mlp(gbp_mlp p) {
    if (!p) return;
    void* ptrs[] = {p->params, p->grads, p->m, p->v, p->y, p->dy, p->part, p->loss,
                    p->dZ[0], p->dZ[1]};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    for (int l = 0; l < NLAYER; ++l)
        if (p->wbf[l]) (void)hipFree(p->wbf[l]);
    for (int l = 0; l <= NLAYER; ++l)
        if (p->H[l]) (void)hipFree(p->H[l]);
    delete p;
}

int refresh_bf16(gbp_mlp p, hipStream_t s) {
    for (int l = 1; l <= NLAYER; ++l) {
        const int n = HID * in_dim(l);
        k_cast_bf16<<<gbp_blocks(n, 256), 256, 0, s>>>(p->params + off_W(l), n, p->wbf[l - 1]);
    }
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

void gemm_fwd(const bf16* Hin, int m, int in, const bf16* W, const float* bias, bf16* out,
              hipStream_t s) {
    // out[m x 256] = relu(Hin[m x in] W^T + b): A(i,k) = Hin[i*in + k], B(k,j) = W[j*in + k]
    dim3 grid((HID + 63) / 64, (m + 63) / 64, 1);
    k_gemm<EPI_BIAS_RELU><<<grid, 256, 0, s>>>(Hin, in, 1, W, 1, in, m, HID, in, in, bias, nullptr,
                                                out, nullptr);
}

// Rows per K chunk of the split-K weight-gradient GEMMs: at most kSplits chunks,
// each a multiple of the GEMM's K step.
constexpr int kSplits = 64;
int split_chunk(int m) { return std::max(512, ((m + kSplits - 1) / kSplits + 31) / 32 * 32); }

// out[c] = sum over the m rows of X[:, c] (w == nullptr) or of w_i X[i][c] with
// out[n] = sum w_i; deterministic (fixed-order partials in p->part)
void colsum(gbp_mlp p, const bf16* X, const float* w, int m, int n, float* out, hipStream_t s) {
    const int R = 256;
    const int ncol = w ? n + 1 : n;
    const dim3 g((ncol + 63) / 64, (m + R - 1) / R);
    if (w) k_colsum_part<true><<<g, 256, 0, s>>>(X, w, m, n, R, p->part);
    else k_colsum_part<false><<<g, 256, 0, s>>>(X, nullptr, m, n, R, p->part);
    k_reduce_parts<<<gbp_blocks(ncol, 256), 256, 0, s>>>(p->part, (int)g.y, ncol, out);
}

int forward_all(gbp_mlp p, const bf16* X, int m, hipStream_t s) {
    const bf16* hin = X;
    for (int l = 1; l <= NLAYER; ++l) {
        gemm_fwd(hin, m, in_dim(l), p->wbf[l - 1], p->params + off_b(l), p->H[l], s);
        hin = p->H[l];
    }
    k_head<<<gbp_blocks(16LL * m, 256), 256, 0, s>>>(p->H[NLAYER], m, p->params + off_w5(),
                                                     p->params + off_w5() + HID, p->y);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

int backward_all(gbp_mlp p, const bf16* X, int m, const float* target, hipStream_t s) {
    const int nb = gbp_blocks(m, 256);
    k_mse<<<nb, 256, 0, s>>>(p->y, target, m, p->dy, p->part);
    k_sum_parts<<<1, 256, 0, s>>>(p->part, nb, 1.f / (float)m, p->loss);
    // dw5 = H4^T dy and db5 = sum dy (parameter order: w5 then b5, adjacent)
    colsum(p, p->H[NLAYER], p->dy, m, HID, p->grads + off_w5(), s);
    k_head_bwd<<<gbp_blocks((long long)m * HID, 256), 256, 0, s>>>(p->dy, p->H[NLAYER], m,
                                                                    p->params + off_w5(), p->dZ[0]);
    int cur = 0;
    for (int l = NLAYER; l >= 1; --l) {
        const int in = in_dim(l);
        const bf16* hprev = l > 1 ? p->H[l - 1] : X;
        // dW_l [256 x in] = dZ^T Hprev: A(i,k) = dZ[k*256 + i], B(k,j) = Hprev[k*in + j], split K
        const int kchunk = split_chunk(m);
        const int splits = (m + kchunk - 1) / kchunk;
        dim3 g1((in + 63) / 64, (HID + 63) / 64, splits);
        k_gemm<EPI_PARTIAL><<<g1, 256, 0, s>>>(p->dZ[cur], 1, HID, hprev, in, 1, HID, in, m, kchunk,
                                               nullptr, nullptr, nullptr, p->part);
        k_reduce_parts<<<gbp_blocks(HID * in, 256), 256, 0, s>>>(p->part, splits, HID * in,
                                                                 p->grads + off_W(l));
        colsum(p, p->dZ[cur], nullptr, m, HID, p->grads + off_b(l), s);
        if (l > 1) {
            // dZ_{l-1} [m x in] = (dZ W_l) masked: A(i,k) = dZ[i*256 + k], B(k,j) = W[k*in + j]
            dim3 g2((in + 63) / 64, (m + 63) / 64, 1);
            k_gemm<EPI_MASK><<<g2, 256, 0, s>>>(p->dZ[cur], HID, 1, p->wbf[l - 1], in, 1, m, in, HID,
                                                HID, nullptr, hprev, p->dZ[1 - cur], nullptr);
            cur = 1 - cur;
        }
    }
    GBP_LAUNCH_CHECK();
    return GBP_OK;
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
    // split-K partials of a weight gradient, column-sum partials, loss partials
    p->part_n = std::max({(size_t)kSplits * HID * HID, (size_t)((max_rows + 255) / 256) * (HID + 1),
                          (size_t)gbp_blocks(max_rows, 256)});
    bool ok = hipMalloc((void**)&p->params, sizeof(float) * p->n_params) == hipSuccess &&
              hipMalloc((void**)&p->grads, sizeof(float) * p->n_params) == hipSuccess &&
              hipMalloc((void**)&p->m, sizeof(float) * p->n_params) == hipSuccess &&
              hipMalloc((void**)&p->v, sizeof(float) * p->n_params) == hipSuccess &&
              hipMalloc((void**)&p->y, sizeof(float) * max_rows) == hipSuccess &&
              hipMalloc((void**)&p->dy, sizeof(float) * max_rows) == hipSuccess &&
              hipMalloc((void**)&p->part, sizeof(float) * p->part_n) == hipSuccess &&
              hipMalloc((void**)&p->loss, sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&p->dZ[0], sizeof(bf16) * max_rows * HID) == hipSuccess &&
              hipMalloc((void**)&p->dZ[1], sizeof(bf16) * max_rows * HID) == hipSuccess;
    for (int l = 1; ok && l <= NLAYER; ++l)
        ok = hipMalloc((void**)&p->wbf[l - 1], sizeof(bf16) * HID * in_dim(l)) == hipSuccess &&
             hipMalloc((void**)&p->H[l], sizeof(bf16) * max_rows * HID) == hipSuccess;
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
    if (m >= kInferRowsLarge)
        k_mlp_infer<8><<<(m + 127) / 128, 256, 0, s>>>((const bf16*)X, m, p->wbf[0], p->wbf[1], p->wbf[2],
                                                      p->wbf[3], p->params, out_scale, y);
    else
        k_mlp_infer<4><<<(m + 63) / 64, 256, 0, s>>>((const bf16*)X, m, p->wbf[0], p->wbf[1], p->wbf[2],
                                                    p->wbf[3], p->params, out_scale, y);
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
    hipStream_t s = (hipStream_t)stream;
    if ((rc = forward_all(p, (const bf16*)X, m, s))) return rc;
    if ((rc = backward_all(p, (const bf16*)X, m, target, s))) return rc;
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
                                                             p->n_params, lr, c1, c2);
    GBP_LAUNCH_CHECK();
    return refresh_bf16(p, s);
}
