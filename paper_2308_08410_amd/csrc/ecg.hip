// Lead-field ECG (Sec. 2.4) and its backward pass on gfx950 matrix cores.
//
//   ecg[s,l] = sum_n W[n,l] U(t_s - T_n),   U(xi) = K0 + (K1-K0) sigma(4 xi / tau)
//
// The template saturates: for |4 xi / tau| >= 24, sigma equals 1 to FP32
// precision on the upper side (1 - sigma < 4e-11) and is below 4e-11 on the lower
// side.  A wavefront owns 64 consecutive vertices; their finite activation times
// span [Tmin, Tmax], so for t_s < Tmin - 6 tau every term is at rest and for
// t_s > Tmax + 6 tau every term is at K1.  Only the window in between needs the
// template; there the contraction (time x vertices) . (vertices x leads) runs on
// v_mfma_f32_16x16x16_bf16 tiles whose A operand is generated in registers from T.
// (The K = 32 shape of gfx950 halves the matrix instructions but made both kernels
// slower, 74 -> 106 us and 63 -> 67 us at 500k: they are bound by the template's
// vector-ALU work and latency, and the wider operands raised register use.)
// Both operands are split into bf16 hi + lo parts (three products, FP32
// accumulation), since the lead weights sum to ~0 and the ECG is a cancellation.
// The saturated part is a step function: the window's weight sum is added once at
// the first saturated step and prefix-summed over time at the end.
//
// Backward:  dT_n = -sum_s U'(t_s - T_n) sum_l G[s,l] W[n,l], with U' zero outside
// the same window; R = U' G runs on MFMA (vertices x time) . (time x leads) and the
// row-wise dot with W finishes in registers.  No atomics: deterministic.
//
// One launch covers a tile of at most 16 leads and a chunk of at most kMaxChunk
// time steps (the window and G tiles live in LDS); the host walks the tiles and
// chunks.  A chunk is an independent ECG on its own time grid; the backward adds
// the contributions of later tiles and chunks to dT in launch order.
//
// MFMA 16x16x16 lane layout: lane l holds A[l % 16][4 (l / 16) + q] and
// B[4 (l / 16) + q][l % 16], q = 0..3, and returns D[4 (l / 16) + r][l % 16], r = 0..3.
#include <math.h>
#include <mutex>

#include "gbp_internal.h"
#include "profile.h"

namespace {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr float kSat = 24.f;          // |4 xi / tau| beyond which sigma is saturated
constexpr float kLog2e = 1.4426950408889634f;
constexpr int kMaxChunk = 992;        // time steps per launch: keeps the LDS of both kernels within 64 KB
constexpr int kMaxSteps = 1 << 20;    // time steps per call
constexpr int kMaxLeads = 256;

__device__ __forceinline__ unsigned bf16_rne(float x) {
    const unsigned u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void split_bf16(float x, short& hi, short& lo) {
    const unsigned h = bf16_rne(x);
    hi = (short)h;
    lo = (short)bf16_rne(x - __uint_as_float(h << 16));
}

__device__ __forceinline__ floatx4 mfma3(bf16x4_t ah, bf16x4_t al, bf16x4_t bh, bf16x4_t bl,
                                         floatx4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    return acc;
}

__device__ __forceinline__ float wave_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

struct ApDev {
    float K0, amp, c4, dudx, t0, dt, halfw;  // c4 = 4 log2(e)/tau, dudx = amp*4/tau, halfw = 6 tau
    int S;                                    // time steps of this chunk
};

// Tile of the lead and time axes a launch works on: columns [0, Lt) of arrays
// whose rows are Ls floats long (W, and ecg / G per time step), the latter
// `istride` floats apart from one instance to the next.
struct LeadTile {
    int Ls, Lt;
    long long istride;
};

// window [s_lo, s_hi) of a wave's finite activation times; empty if none finite
__device__ __forceinline__ void wave_window(float Tv, const ApDev& ap, int& s_lo, int& s_hi,
                                            bool& any) {
    const bool fin = Tv < __builtin_huge_valf();
    const float tmin = wave_min(fin ? Tv : __builtin_huge_valf());
    const float tmax = wave_max(fin ? Tv : -__builtin_huge_valf());
    any = tmin < __builtin_huge_valf();
    if (!any) {
        s_lo = s_hi = ap.S;
        return;
    }
    const float lo = ceilf((tmin - ap.halfw - ap.t0) / ap.dt);
    const float hi = floorf((tmax + ap.halfw - ap.t0) / ap.dt) + 1.f;
    s_lo = (int)fminf(fmaxf(lo, 0.f), (float)ap.S);
    s_hi = (int)fminf(fmaxf(hi, 0.f), (float)ap.S);
    if (s_hi < s_lo) s_hi = s_lo;
}

// ------------------------------------------------------------------ forward
// Block: 4 waves; each wave takes 64-vertex groups of the block's range (two
// K-steps of 32 vertices: lane (col, kq) holds vertices 8 kq .. 8 kq + 7).
// Dynamic LDS: win[S_pad*16] floats.  The step histogram goes to global memory
// directly (one 16-wide add per 64-vertex group).
// Grid (blocks per instance, instances); instance i owns vertices
// [off[i], off[i+1]) (off == nullptr: one instance of n_v vertices).
__global__ void __launch_bounds__(256)
    k_ecg_fwd(const float* __restrict__ T, const float* __restrict__ W, int n_v, LeadTile lt,
              ApDev ap, int S_pad, int groups_per_block, const int* __restrict__ off,
              float* __restrict__ g_win_all, float* __restrict__ g_hist_all,
              float* __restrict__ g_wsum_all) {
    extern __shared__ float win[];
    const int inst = blockIdx.y;
    const int vbeg = off ? off[inst] : 0, vend = off ? off[inst + 1] : n_v;
    const int Ls = lt.Ls, Lt = lt.Lt;
    float* g_win = g_win_all + (size_t)inst * S_pad * 16;
    float* g_hist = g_hist_all + (size_t)inst * S_pad * 16;
    float* g_wsum = g_wsum_all + (size_t)inst * 16;
    __shared__ int blo, bhi;
    __shared__ float wsum_sh[4][16];
    for (int x = threadIdx.x; x < S_pad * 16; x += blockDim.x) win[x] = 0.f;
    if (threadIdx.x == 0) {
        blo = ap.S;
        bhi = 0;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, kq = lane >> 4;
    float wsum_all = 0.f;   // lane: lead col, vertices 4kq+r of each K-step
    for (int gi = wave; gi < groups_per_block; gi += 4) {
        const int g0 = vbeg + (blockIdx.x * groups_per_block + gi) * 64;
        if (g0 >= vend) break;
        const int nl = g0 + lane;
        const float Tl = nl < vend ? T[nl] : __builtin_huge_valf();
        int s_lo, s_hi;
        bool any;
        wave_window(Tl, ap, s_lo, s_hi, any);
        float wsum_fin = 0.f;
        // W fragments and sums (4 K-steps of 16 vertices)
        for (int ks = 0; ks < 4; ++ks) {
            for (int r = 0; r < 4; ++r) {
                const int n = g0 + ks * 16 + kq * 4 + r;
                const float w = (n < vend && col < Lt) ? W[(size_t)n * Ls + col] : 0.f;
                const float t = n < vend ? T[n] : __builtin_huge_valf();
                wsum_all += w;
                if (t < __builtin_huge_valf()) wsum_fin += w;
            }
        }
        if (!any) continue;
        // window contraction, up to 4 time tiles per pass
        for (int s0 = s_lo; s0 < s_hi; s0 += 64) {
            floatx4 acc[4];
            for (int m = 0; m < 4; ++m) acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
            const int ntile = min(4, (s_hi - s0 + 15) / 16);
            for (int ks = 0; ks < 4; ++ks) {
                float tv[4];
                bf16x4_t bh, bl;
                for (int r = 0; r < 4; ++r) {
                    const int n = g0 + ks * 16 + kq * 4 + r;
                    const float w = (n < vend && col < Lt) ? W[(size_t)n * Ls + col] : 0.f;
                    tv[r] = n < vend ? T[n] : __builtin_huge_valf();
                    short h, l;
                    split_bf16(w, h, l);
                    bh[r] = h;
                    bl[r] = l;
                }
                for (int m = 0; m < 4; ++m) {
                    if (m >= ntile) break;
                    const float t = ap.t0 + (float)(s0 + 16 * m + col) * ap.dt;
                    bf16x4_t ah, al;
                    for (int r = 0; r < 4; ++r) {
                        const float e = __builtin_amdgcn_exp2f((tv[r] - t) * ap.c4);
                        const float a = ap.amp * __builtin_amdgcn_rcpf(1.f + e);
                        short h, l;
                        split_bf16(a, h, l);
                        ah[r] = h;
                        al[r] = l;
                    }
                    acc[m] = mfma3(ah, al, bh, bl, acc[m]);
                }
            }
            for (int m = 0; m < ntile; ++m)
                for (int r = 0; r < 4; ++r) {
                    const int s = s0 + 16 * m + kq * 4 + r;
                    if (s < s_hi && col < Lt) atomicAdd(&win[s * 16 + col], acc[m][r]);
                }
        }
        // saturated part: step at s_hi
        float hsum = wsum_fin;
        hsum += __shfl_xor(hsum, 16);
        hsum += __shfl_xor(hsum, 32);
        if (s_hi < ap.S && kq == 0 && col < Lt) atomicAdd(&g_hist[s_hi * 16 + col], ap.amp * hsum);
        if (lane == 0) {
            atomicMin(&blo, s_lo);
            atomicMax(&bhi, s_hi);
        }
    }
    wsum_all += __shfl_xor(wsum_all, 16);
    wsum_all += __shfl_xor(wsum_all, 32);
    if (kq == 0) wsum_sh[wave][col] = wsum_all;
    __syncthreads();
    if (threadIdx.x < 16 && (int)threadIdx.x < Lt) {
        const float v = wsum_sh[0][threadIdx.x] + wsum_sh[1][threadIdx.x] +
                        wsum_sh[2][threadIdx.x] + wsum_sh[3][threadIdx.x];
        atomicAdd(&g_wsum[threadIdx.x], v);
    }
    const int lo = blo, hi = min(bhi, ap.S);
    for (int x = lo * 16 + threadIdx.x; x < hi * 16; x += blockDim.x) {
        if ((x & 15) >= Lt) continue;
        const float a = win[x];
        if (a != 0.f) atomicAdd(&g_win[x], a);
    }
}

__global__ void k_ecg_zero(float* __restrict__ p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// ecg[s,l] = K0 * sum W + prefix_s(hist) + win.  One block of 1024 threads:
// thread (c, l) owns lead l and the c-th of 64 contiguous chunks of time steps.
__global__ void __launch_bounds__(1024)
    k_ecg_finish(const float* __restrict__ g_win_all, const float* __restrict__ g_hist_all,
                 const float* __restrict__ g_wsum_all, int S, int S_pad, LeadTile lt, float K0,
                 float* __restrict__ ecg_all) {
    __shared__ float part[64][17];
    const int inst = blockIdx.x;
    const float* g_win = g_win_all + (size_t)inst * S_pad * 16;
    const float* g_hist = g_hist_all + (size_t)inst * S_pad * 16;
    const float* g_wsum = g_wsum_all + (size_t)inst * 16;
    float* ecg = ecg_all + (size_t)inst * lt.istride;
    const int l = threadIdx.x & 15, c = threadIdx.x >> 4;
    const int len = (S + 63) / 64;
    const int s0 = c * len, s1 = min(S, s0 + len);
    float run = 0.f;
    for (int s = s0; s < s1; ++s) run += g_hist[s * 16 + l];
    part[c][l] = run;
    __syncthreads();
    float off = 0.f;
    for (int k = 0; k < c; ++k) off += part[k][l];
    if (l < lt.Lt) {
        const float base = K0 * g_wsum[l];
        float r = off;
        for (int s = s0; s < s1; ++s) {
            r += g_hist[s * 16 + l];
            ecg[(size_t)s * lt.Ls + l] = base + r + g_win[s * 16 + l];
        }
    }
}

// ------------------------------------------------------------------ backward
// accumulate: add this tile's / chunk's contribution to dT instead of writing it.
__global__ void __launch_bounds__(256)
    k_ecg_bwd(const float* __restrict__ T, const float* __restrict__ W,
              const float* __restrict__ G_all, int n_v, LeadTile lt, ApDev ap, int S_pad,
              const int* __restrict__ off, int accumulate, float* __restrict__ dT) {
    extern __shared__ short gl[];  // [S_pad*16] hi, then [S_pad*16] lo
    const int inst = blockIdx.y;
    const int vbeg = off ? off[inst] : 0, vend = off ? off[inst + 1] : n_v;
    const int Ls = lt.Ls, Lt = lt.Lt;
    const float* G = G_all + (size_t)inst * lt.istride;
    short* gh = gl;
    short* glo = gl + S_pad * 16;
    for (int x = threadIdx.x; x < S_pad * 16; x += blockDim.x) {
        const int s = x >> 4, l = x & 15;
        const float v = (s < ap.S && l < Lt) ? G[(size_t)s * Ls + l] : 0.f;
        short h, lo;
        split_bf16(v, h, lo);
        gh[x] = h;
        glo[x] = lo;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, kq = lane >> 4;
    const int nwaves = gridDim.x * 4;
    for (int grp = blockIdx.x * 4 + wave; vbeg + grp * 64 < vend; grp += nwaves) {
        const int g0 = vbeg + grp * 64;
        const int nl = g0 + lane;
        const float Tl = nl < vend ? T[nl] : __builtin_huge_valf();
        int s_lo, s_hi;
        bool any;
        wave_window(Tl, ap, s_lo, s_hi, any);
        // 4 vertex tiles of 16
        for (int mt = 0; mt < 4; ++mt) {
            const int nrow = g0 + mt * 16 + col;   // A row: vertex
            const float tn = nrow < vend ? T[nrow] : __builtin_huge_valf();
            floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
            if (any) {
                for (int s0 = s_lo; s0 < s_hi; s0 += 16) {
                    bf16x4_t ah, al, bh, bl;
                    for (int r = 0; r < 4; ++r) {
                        const int s = s0 + kq * 4 + r;
                        const float t = ap.t0 + (float)s * ap.dt;
                        const float e = __builtin_amdgcn_exp2f((tn - t) * ap.c4);
                        const float q = __builtin_amdgcn_rcpf(1.f + e);
                        const float omq = e < 1.f ? e * q : 1.f - q;
                        const float a = (s < ap.S) ? ap.dudx * q * omq : 0.f;
                        short h, l;
                        split_bf16(a, h, l);
                        ah[r] = h;
                        al[r] = l;
                        const int sc = s < S_pad ? s : S_pad - 1;
                        bh[r] = (s < ap.S) ? gh[sc * 16 + col] : (short)0;
                        bl[r] = (s < ap.S) ? glo[sc * 16 + col] : (short)0;
                    }
                    acc = mfma3(ah, al, bh, bl, acc);
                }
            }
            // acc[r]: R[vertex g0+mt*16+kq*4+r][lead col]
            float out[4];
            for (int r = 0; r < 4; ++r) {
                const int n = g0 + mt * 16 + kq * 4 + r;
                const float w = (n < vend && col < Lt) ? W[(size_t)n * Ls + col] : 0.f;
                float v = acc[r] * w;
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 4);
                v += __shfl_xor(v, 8);
                out[r] = v;
            }
            if (col == 0)
                for (int r = 0; r < 4; ++r) {
                    const int n = g0 + mt * 16 + kq * 4 + r;
                    if (n < vend) dT[n] = accumulate ? dT[n] - out[r] : -out[r];
                }
        }
    }
}

// ------------------------------------------------------------------ workspace
// Scratch of gbp_ecg_forward_noalloc: one chunk's window, histogram and weight
// sums for one instance (every chunk and lead tile reuses it in stream order),
// file-scope device memory that each GPU holds until the process ends.
constexpr int kNoAllocFloats = 2 * ((kMaxChunk + 15) / 16 * 16 + 16) * 16 + 16;
__device__ __align__(256) float scratch[kNoAllocFloats];

// The array's device address on the current device, looked up once per device
// (in host code the symbol's name is a host-side stand-in, not this address).
int noalloc_scratch(float** out) {
    static std::mutex mu;
    static float* addr[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        gbp_set_error("no HIP device");
        return GBP_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            gbp_set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return GBP_ERR_HIP;
        }
        addr[dev] = (float*)p;
    }
    *out = addr[dev];
    return GBP_OK;
}

struct EcgWork {
    float* buf = nullptr;
    size_t cap = 0;
};
std::mutex g_mu;
EcgWork g_work[64];

int ecg_workspace(size_t nfloat, float** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        gbp_set_error("no HIP device");
        return GBP_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    EcgWork& w = g_work[dev];
    if (w.cap < nfloat) {
        if (w.buf) (void)hipFree(w.buf);
        w.buf = nullptr;
        w.cap = 0;
        if (hipMalloc((void**)&w.buf, nfloat * sizeof(float)) != hipSuccess) {
            gbp_set_error("ECG workspace allocation failed");
            return GBP_ERR_NOMEM;
        }
        w.cap = nfloat;
    }
    *out = w.buf;
    return GBP_OK;
}

int check_ap(const float* T, int n_v, const float* W, int L, const gbp_ap* ap) {
    if (!T || !W || !ap || n_v <= 0 || L < 1 || L > kMaxLeads) {
        gbp_set_error("ECG: need T, W, ap, n_v > 0 and 1 <= L <= %d (L=%d)", kMaxLeads, L);
        return GBP_ERR_ARG;
    }
    if (ap->n_steps < 1 || ap->n_steps > kMaxSteps || !(ap->dt > 0.f) || !(ap->tau > 0.f) ||
        !std::isfinite(ap->K0) || !std::isfinite(ap->K1) || !std::isfinite(ap->t0)) {
        gbp_set_error("ECG: bad template/time grid (n_steps in [1,%d], dt > 0, tau > 0)", kMaxSteps);
        return GBP_ERR_ARG;
    }
    return GBP_OK;
}

// the template constants for the chunk of `len` steps starting at step s0
ApDev make_ap(const gbp_ap* a, int s0, int len) {
    ApDev d;
    d.K0 = a->K0;
    d.amp = a->K1 - a->K0;
    d.c4 = 4.f * kLog2e / a->tau;
    d.dudx = (a->K1 - a->K0) * 4.f / a->tau;
    d.t0 = a->t0 + (float)s0 * a->dt;
    d.dt = a->dt;
    d.halfw = kSat * a->tau / 4.f;
    d.S = len;
    return d;
}

int chunk_pad(int len) { return (len + 15) / 16 * 16 + 16; }

// floats of forward scratch per instance: window and histogram of one chunk, weight sums
size_t ecg_work_floats(int n_steps) {
    const int S_pad = chunk_pad(std::min(n_steps, kMaxChunk));
    return (size_t)2 * S_pad * 16 + 16;
}

struct EcgLaunch {
    const int* off;       // device offsets or nullptr
    int n_inst;
    int max_verts;        // largest instance
    float* work;          // n_inst * ecg_work_floats(n_steps) floats
};

// Every (lead tile, time chunk) of the call: a forward chunk is an ECG on its own
// time grid (the instance's rows of ecg are n_steps * L floats apart).
int ecg_forward_launch(const EcgLaunch& el, const float* T, int n_v, const float* W, int L,
                       const gbp_ap* ap, float* ecg, hipStream_t s) {
    const int S = ap->n_steps;
    for (int c0 = 0; c0 < L; c0 += 16) {
        for (int s0 = 0; s0 < S; s0 += kMaxChunk) {
            const int len = std::min(kMaxChunk, S - s0);
            const ApDev d = make_ap(ap, s0, len);
            const LeadTile lt{L, std::min(16, L - c0), (long long)S * L};
            const int S_pad = chunk_pad(len);
            float* g_win = el.work;
            float* g_hist = el.work + (size_t)el.n_inst * S_pad * 16;
            float* g_wsum = el.work + (size_t)2 * el.n_inst * S_pad * 16;
            const int total = el.n_inst * (2 * S_pad * 16 + 16);
            k_ecg_zero<<<std::min((total + 255) / 256, 1024), 256, 0, s>>>(el.work, total);
            const int groups = (el.max_verts + 63) / 64;
            const int gpb = 8;    // 64-vertex groups per block (2 per wave; 16 measured slower: fewer resident waves)
            const dim3 grid((groups + gpb - 1) / gpb, el.n_inst);
            const size_t lds = (size_t)S_pad * 16 * sizeof(float);
            {
                ProfScope ps(GBP_PROF_ECG_FWD, s);
                k_ecg_fwd<<<grid, 256, lds, s>>>(T, W + c0, n_v, lt, d, S_pad, gpb, el.off, g_win,
                                                 g_hist, g_wsum);
            }
            k_ecg_finish<<<el.n_inst, 1024, 0, s>>>(g_win, g_hist, g_wsum, len, S_pad, lt, d.K0,
                                                    ecg + (size_t)s0 * L + c0);
            GBP_LAUNCH_CHECK();
        }
    }
    return GBP_OK;
}

int ecg_backward_launch(const EcgLaunch& el, const float* T, int n_v, const float* W, int L,
                        const gbp_ap* ap, const float* G, float* dT, hipStream_t s) {
    const int S = ap->n_steps;
    int first = 1;
    for (int c0 = 0; c0 < L; c0 += 16) {
        for (int s0 = 0; s0 < S; s0 += kMaxChunk) {
            const int len = std::min(kMaxChunk, S - s0);
            const ApDev d = make_ap(ap, s0, len);
            const LeadTile lt{L, std::min(16, L - c0), (long long)S * L};
            const int S_pad = chunk_pad(len);
            const int groups = (el.max_verts + 63) / 64;
            const dim3 grid(std::max(1, std::min((groups + 3) / 4, 2048 / std::max(1, el.n_inst) + 1)),
                            el.n_inst);
            const size_t lds = (size_t)2 * S_pad * 16 * sizeof(short);
            ProfScope ps(GBP_PROF_ECG_BWD, s);
            k_ecg_bwd<<<grid, 256, lds, s>>>(T, W + c0, G + (size_t)s0 * L + c0, n_v, lt, d, S_pad,
                                             el.off, first ? 0 : 1, dT);
            GBP_LAUNCH_CHECK();
            first = 0;
        }
    }
    return GBP_OK;
}

}  // namespace

struct gbp_batch_s {
    int device = 0;
    int n_inst = 0, max_verts = 0, total = 0, max_steps = 0;
    int* off = nullptr;
    float* work = nullptr;
};

extern "C" int gbp_batch_create(const int32_t* offsets, int n_inst, int max_steps, gbp_batch* out) {
    if (!out || !offsets || n_inst < 1 || max_steps < 1 || max_steps > kMaxSteps) {
        gbp_set_error("batch: need offsets, n_inst >= 1, 1 <= max_steps <= %d", kMaxSteps);
        return GBP_ERR_ARG;
    }
    *out = nullptr;
    if (offsets[0] != 0) {
        gbp_set_error("batch: offsets[0] must be 0");
        return GBP_ERR_ARG;
    }
    int mx = 0;
    for (int i = 0; i < n_inst; ++i) {
        if (offsets[i + 1] < offsets[i]) {
            gbp_set_error("batch: offsets must be non-decreasing");
            return GBP_ERR_ARG;
        }
        mx = std::max(mx, offsets[i + 1] - offsets[i]);
    }
    gbp_batch b = new gbp_batch_s();
    (void)hipGetDevice(&b->device);
    b->n_inst = n_inst;
    b->max_verts = std::max(mx, 1);
    b->total = offsets[n_inst];
    b->max_steps = max_steps;
    const size_t nwork = (size_t)n_inst * ecg_work_floats(max_steps);
    if (hipMalloc((void**)&b->off, sizeof(int) * (n_inst + 1)) != hipSuccess ||
        hipMalloc((void**)&b->work, sizeof(float) * nwork) != hipSuccess) {
        gbp_set_error("batch: allocation failed");
        gbp_batch_destroy(b);
        return GBP_ERR_NOMEM;
    }
    if (hipMemcpy(b->off, offsets, sizeof(int) * (n_inst + 1), hipMemcpyHostToDevice) != hipSuccess) {
        gbp_set_error("batch: copy failed");
        gbp_batch_destroy(b);
        return GBP_ERR_HIP;
    }
    *out = b;
    return GBP_OK;
}

extern "C" int gbp_batch_sizes(gbp_batch b, int* n_inst, int* n_total) {
    if (!b) {
        gbp_set_error("batch is NULL");
        return GBP_ERR_ARG;
    }
    if (n_inst) *n_inst = b->n_inst;
    if (n_total) *n_total = b->total;
    return GBP_OK;
}

extern "C" void gbp_batch_destroy(gbp_batch b) {
    if (!b) return;
    if (b->off) (void)hipFree(b->off);
    if (b->work) (void)hipFree(b->work);
    delete b;
}

static int check_batch(gbp_batch b, const gbp_ap* ap) {
    if (!b) {
        gbp_set_error("batch is NULL");
        return GBP_ERR_ARG;
    }
    if (ap && ap->n_steps > b->max_steps) {
        gbp_set_error("n_steps %d exceeds the batch's max_steps %d", ap->n_steps, b->max_steps);
        return GBP_ERR_ARG;
    }
    return GBP_OK;
}

extern "C" int gbp_ecg_forward(const float* T, int n_v, const float* W, int L, const gbp_ap* ap,
                               float* ecg, void* stream) {
    int rc = check_ap(T, n_v, W, L, ap);
    if (rc) return rc;
    if (!ecg) {
        gbp_set_error("ecg is NULL");
        return GBP_ERR_ARG;
    }
    float* work;
    if ((rc = ecg_workspace(ecg_work_floats(ap->n_steps), &work))) return rc;
    return ecg_forward_launch(EcgLaunch{nullptr, 1, n_v, work}, T, n_v, W, L, ap, ecg,
                              (hipStream_t)stream);
}

extern "C" int gbp_ecg_forward_noalloc(const float* T, int n_v, const float* W, int L,
                                       const gbp_ap* ap, float* ecg, void* stream) {
    int rc = check_ap(T, n_v, W, L, ap);
    if (rc) return rc;
    if (!ecg) {
        gbp_set_error("ecg is NULL");
        return GBP_ERR_ARG;
    }
    const size_t need = ecg_work_floats(ap->n_steps);
    if (need > (size_t)kNoAllocFloats) {
        gbp_set_error("ECG (no allocation): needs %zu scratch floats, the library holds %d", need,
                      kNoAllocFloats);
        return GBP_ERR_ARG;
    }
    float* work;
    if ((rc = noalloc_scratch(&work))) return rc;
    return ecg_forward_launch(EcgLaunch{nullptr, 1, n_v, work}, T, n_v, W, L, ap, ecg,
                              (hipStream_t)stream);
}

extern "C" int gbp_ecg_backward(const float* T, int n_v, const float* W, int L, const gbp_ap* ap,
                                const float* dL_decg, float* dL_dT, void* stream) {
    int rc = check_ap(T, n_v, W, L, ap);
    if (rc) return rc;
    if (!dL_decg || !dL_dT) {
        gbp_set_error("dL_decg and dL_dT are required");
        return GBP_ERR_ARG;
    }
    return ecg_backward_launch(EcgLaunch{nullptr, 1, n_v, nullptr}, T, n_v, W, L, ap, dL_decg, dL_dT,
                               (hipStream_t)stream);
}

extern "C" int gbp_ecg_forward_batched(gbp_batch b, const float* T, const float* W, int L,
                                       const gbp_ap* ap, float* ecg, void* stream) {
    int rc = check_batch(b, ap);
    if (rc) return rc;
    if ((rc = check_ap(T, b->total, W, L, ap))) return rc;
    if (!ecg) {
        gbp_set_error("ecg is NULL");
        return GBP_ERR_ARG;
    }
    return ecg_forward_launch(EcgLaunch{b->off, b->n_inst, b->max_verts, b->work}, T, b->total, W,
                              L, ap, ecg, (hipStream_t)stream);
}

extern "C" int gbp_ecg_backward_batched(gbp_batch b, const float* T, const float* W, int L,
                                        const gbp_ap* ap, const float* dL_decg, float* dL_dT,
                                        void* stream) {
    int rc = check_batch(b, ap);
    if (rc) return rc;
    if ((rc = check_ap(T, b->total, W, L, ap))) return rc;
    if (!dL_decg || !dL_dT) {
        gbp_set_error("dL_decg and dL_dT are required");
        return GBP_ERR_ARG;
    }
    return ecg_backward_launch(EcgLaunch{b->off, b->n_inst, b->max_verts, nullptr}, T, b->total, W,
                               L, ap, dL_decg, dL_dT, (hipStream_t)stream);
}
