// Eikonal forward (Alg. 2 as an active-list relaxation) and its adjoint
// (Sec. 2.3: back-propagation along the frozen geodesic parents) for gfx950.
//
// Forward.  Each sweep processes a work queue of vertices; a vertex takes the
// minimum over the local problems of its patch (Eq. (hopflax_global)), every
// local problem solved in closed form (local_solve.h).  A vertex whose value
// drops by more than eps_rel*max(1,|T|) pushes its unique neighbours into the
// next queue (deduplicated with per-vertex stamps).  This is the change mask of
// Alg. 2 applied at vertex granularity; updates are in place (chaotic
// relaxation), which reaches the same fixed point because every value read is an
// upper bound of the solution and the update is monotone.
//
// Adjoint.  lambda = g + P^T lambda with P the parent weights.  The parent graph
// is walked leaves-first in levels (Kahn order): a vertex is finished once all of
// its children are, and then pulls their contributions in a fixed order, so the
// result is deterministic.  Vertices left over by a cycle in the (non-causal)
// anisotropic parent graph are finished with in-place (Gauss-Seidel) sweeps.
#include <math.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include <vector>

#include "gbp_internal.h"
#include "local_solve.h"
#include "fista.h"
#include "profile.h"

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ bool finitef(float x) { return x == x && fabsf(x) < GBP_INF; }

// Sum over the block (fixed order); result valid in thread 0.
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v) {
    __shared__ unsigned long long red[TPB / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < TPB / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Sums of two values over the block (fixed order); results valid in thread 0.
__device__ __forceinline__ void block_sum2_u64(unsigned long long& a, unsigned long long& b) {
    __shared__ unsigned long long red2[2][TPB / 64];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red2[0][threadIdx.x >> 6] = a;
        red2[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = b = 0;
        for (int w = 0; w < TPB / 64; ++w) {
            a += red2[0][w];
            b += red2[1][w];
        }
    }
}

__device__ __forceinline__ float block_max_f(float v) {
    __shared__ float red[TPB / 64];
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float t = 0.f;
    if (threadIdx.x == 0)
        for (int w = 0; w < TPB / 64; ++w) t = fmaxf(t, red[w]);
    __syncthreads();
    return t;
}

// Capacity of a block's LDS push buffer (entries, all sub-queue sections): cold
// rounds' fronts fit 4096; a two-sided (warm) round queues every vertex, so its
// blocks get 8192 (32 KB, still within four resident blocks' share of the LDS).
constexpr int kPushCap = 4096;
constexpr int kPushCapWide = 8192;

__device__ __forceinline__ int xcd_of(int i, int R) { return (i / R) & 7; }
// position of vertex i inside its sub-queue when every vertex is queued
__device__ __forceinline__ int xcd_rank(int i, int R) {
    const int r = i / R;
    return (r >> 3) * R + (i - r * R);
}

// Block-level push buffer: pushes land in LDS (any sub-queue); at flush time the
// entries are counted per sub-queue, one atomic per non-empty sub-queue reserves
// room, and the entries are scattered to their sub-queues (overflow goes
// straight to global).
struct XPushBuf {
    int* q;      // LDS [cap]
    int* n;      // LDS counter
    int cap;
};

// Overflow of the LDS buffer: the overflowing lanes of a wave reserve global room
// together, one atomic per sub-queue present among them (a per-lane atomic on one
// counter serialises the whole wave at L2; fronts of millions of vertices
// overflow every block).
// The loop runs over the sub-queues (a wave-uniform bound), one ballot each: a
// loop that peels lanes by readfirstlane until none is left is not safe here,
// since the compiler may hoist the readfirstlane and then take the loop to run
// once for every lane.
__device__ __forceinline__ void xpush_global(int v, const XcdQueues& xq, int* __restrict__ qout,
                                             int* cnt_next) {
    const int x = xq.nq == 1 ? 0 : xcd_of(v, xq.R);
    const unsigned long long below = (1ull << __lane_id()) - 1ull;
    for (int xs = 0; xs < xq.nq; ++xs) {
        const bool mine = x == xs;
        const unsigned long long grp = __ballot(mine);   // overflowing lanes of sub-queue xs
        if (grp == 0ull) continue;
        if (mine) {
            const int rank = __popcll(grp & below);
            int base = 0;
            if (rank == 0) base = atomicAdd(&cnt_next[xs], __popcll(grp));
            base = __shfl(base, __ffsll((unsigned long long)grp) - 1);
            qout[xq.off[xs] + base + rank] = v;
        }
    }
}

// WIDE: fronts that overflow the LDS buffer wholesale (a warm start queues every
// vertex) take the wave-aggregated reservation; cold fronts overflow rarely and
// keep the plain per-lane atomic, which needs fewer registers in the round's
// main loop.
template <bool WIDE>
__device__ __forceinline__ void xpush_node(XPushBuf b, int v, const XcdQueues& xq,
                                           int* __restrict__ qout, int* cnt_next) {
    const int pos = atomicAdd(b.n, 1);
    if (pos < b.cap) {
        b.q[pos] = v;
    } else if constexpr (WIDE) {
        xpush_global(v, xq, qout, cnt_next);
    } else {
        const int x = xcd_of(v, xq.R);
        qout[xq.off[x] + atomicAdd(&cnt_next[x], 1)] = v;
    }
}

// cnt_sh, base_sh: LDS [8] scratch
__device__ __forceinline__ void xpush_flush(XPushBuf b, const XcdQueues& xq, int* __restrict__ qout,
                                            int* cnt_next, int* cnt_sh, int* base_sh) {
    __syncthreads();
    const int n = min(*b.n, b.cap);
    if (xq.nq == 1) {   // one queue: a single reservation, entries in push order
        if (threadIdx.x == 0) base_sh[0] = n > 0 ? atomicAdd(&cnt_next[0], n) : 0;
        __syncthreads();
        for (int k = threadIdx.x; k < n; k += blockDim.x) qout[base_sh[0] + k] = b.q[k];
        return;
    }
    if (threadIdx.x < 8) cnt_sh[threadIdx.x] = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) atomicAdd(&cnt_sh[xcd_of(b.q[k], xq.R)], 1);
    __syncthreads();
    if (threadIdx.x < 8) {
        const int m = cnt_sh[threadIdx.x];
        base_sh[threadIdx.x] = m > 0 ? xq.off[threadIdx.x] + atomicAdd(&cnt_next[threadIdx.x], m) : 0;
        cnt_sh[threadIdx.x] = 0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const int v = b.q[k];
        const int x = xcd_of(v, xq.R);
        qout[base_sh[x] + atomicAdd(&cnt_sh[x], 1)] = v;
    }
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Sum the per-block counters of the relaxation rounds into the control block.
__global__ void k_reduce_stats(const unsigned long long* __restrict__ blk, GbpCtl* ctl) {
    unsigned long long a = 0, b = 0;
    for (int i = threadIdx.x; i < kStatBlocks; i += blockDim.x) {
        a += blk[2 * i];
        b += blk[2 * i + 1];
    }
    a = block_sum_u64(a);
    b = block_sum_u64(b);
    if (threadIdx.x == 0) {
        ctl->solves = a;
        ctl->updates = b;
    }
}

// ------------------------------------------------------------------ preparation
// Per-vertex inputs of a call, internal order: the velocity scale (1 without
// one; a scale that is not finite and > 0 flags an error), the onsets reset to
// +inf, and T: +inf (T_init null, a cold start) or T_init (NaN read as +inf);
// the queue marks are cleared when the control reset restarted the stamps.
// only_T: T alone (the scales and onsets of the last preparation are kept).
// G_init non-null: copied (NaN read as +inf) into guess, the hold-back's ordering key.
__global__ void k_vertex_in(const float* __restrict__ vs_user, const float* __restrict__ T_init,
                            const int* __restrict__ node_user, float* __restrict__ vs,
                            float* __restrict__ troot, float* __restrict__ T,
                            int* __restrict__ mark, int n_v, int only_T, GbpCtl* ctl,
                            int* __restrict__ hold, const float* __restrict__ G_init,
                            float* __restrict__ guess) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_v) return;
    if (ctl->marks_stale) mark[i] = 0;   // the stamps restarted from 1
    if (hold) hold[i] = INT_MIN;          // held in no bucket
    const int u = node_user[i];
    if (!only_T) {
        float s = 1.f;
        if (vs_user) {
            s = vs_user[u];
            if (!(s > 0.f) || !finitef(s)) {
                atomicOr(&ctl->err, ERRBIT_VSCALE);
                s = 1.f;
            }
        }
        vs[i] = s;
        troot[i] = GBP_INF;
    }
    float t = GBP_INF;
    if (T_init) {
        t = T_init[u];
        if (t != t) t = GBP_INF;
    }
    T[i] = t;
    if (G_init) {
        const float gv = G_init[u];
        guess[i] = gv == gv ? gv : GBP_INF;
    }
}

// Per element: M = D_eff^{-1} = D^{-1} / sbar^2 and G = F^T M F (F: edges from v0).
__global__ void k_metric(const float* __restrict__ D, const int* __restrict__ tet_user,
                         const int4* __restrict__ tetv, const float4* __restrict__ xyz,
                         const float* __restrict__ vs, float4* __restrict__ tetg, int n_e,
                         GbpCtl* ctl) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_e) return;
    const int u = tet_user[j];
    const float2* d2 = reinterpret_cast<const float2*>(D + 6 * (size_t)u);
    const float2 da = d2[0], db = d2[1], dc = d2[2];
    const float a = da.x, b = da.y, c = db.x, d = db.y, e = dc.x, f = dc.y;  // xx yy zz xy xz yz
    const int4 v = tetv[j];
    const float sbar = 0.25f * (vs[v.x] + vs[v.y] + vs[v.z] + vs[v.w]);
    const float A00 = b * c - f * f, A11 = a * c - e * e, A22 = a * b - d * d;
    const float A01 = e * f - d * c, A02 = d * f - e * b, A12 = d * e - a * f;
    const float det = a * A00 + d * A01 + e * A02;
    const bool fin = finitef(a) && finitef(b) && finitef(c) && finitef(d) && finitef(e) && finitef(f);
    if (!fin) atomicOr(&ctl->err, ERRBIT_D_NONFINITE);
    else if (!(a > 0.f && A22 > 0.f && det > 0.f)) atomicOr(&ctl->err, ERRBIT_D_NOT_SPD);
    const float s = 1.f / (det * sbar * sbar);
    const float m00 = A00 * s, m11 = A11 * s, m22 = A22 * s, m01 = A01 * s, m02 = A02 * s, m12 = A12 * s;
    const float4 x0 = xyz[v.x], x1 = xyz[v.y], x2 = xyz[v.z], x3 = xyz[v.w];
    const float F1x = x1.x - x0.x, F1y = x1.y - x0.y, F1z = x1.z - x0.z;
    const float F2x = x2.x - x0.x, F2y = x2.y - x0.y, F2z = x2.z - x0.z;
    const float F3x = x3.x - x0.x, F3y = x3.y - x0.y, F3z = x3.z - x0.z;
    // M F_a
    const float M1x = m00 * F1x + m01 * F1y + m02 * F1z, M1y = m01 * F1x + m11 * F1y + m12 * F1z,
                M1z = m02 * F1x + m12 * F1y + m22 * F1z;
    const float M2x = m00 * F2x + m01 * F2y + m02 * F2z, M2y = m01 * F2x + m11 * F2y + m12 * F2z,
                M2z = m02 * F2x + m12 * F2y + m22 * F2z;
    const float M3x = m00 * F3x + m01 * F3y + m02 * F3z, M3y = m01 * F3x + m11 * F3y + m12 * F3z,
                M3z = m02 * F3x + m12 * F3y + m22 * F3z;
    const float G11 = F1x * M1x + F1y * M1y + F1z * M1z;
    const float G22 = F2x * M2x + F2y * M2y + F2z * M2z;
    const float G33 = F3x * M3x + F3y * M3y + F3z * M3z;
    const float G12 = F1x * M2x + F1y * M2y + F1z * M2z;
    const float G13 = F1x * M3x + F1y * M3y + F1z * M3z;
    const float G23 = F2x * M3x + F2y * M3y + F2z * M3z;
    tetg[2 * (size_t)j] = make_float4(G11, G22, G33, G12);
    tetg[2 * (size_t)j + 1] = make_float4(G13, G23, sbar, 0.f);
}

__global__ void k_scatter_out(const float* __restrict__ src, const int* __restrict__ node_int,
                              float* __restrict__ dst_user, int n_v) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n_v) dst_user[u] = src[node_int[u]];
}

// min(*a, v) for a finite v, as one atomic: floats with the sign bit clear order
// like their bits as signed ints, those with it set (-0 included) in reverse like
// their bits as unsigned ints, and every sign-set pattern is above every
// sign-clear one as unsigned, below it as signed.
__device__ __forceinline__ void atomic_min_float(float* a, float v) {
    if (__float_as_int(v) >= 0) atomicMin(reinterpret_cast<int*>(a), __float_as_int(v));
    else atomicMax(reinterpret_cast<unsigned*>(a), __float_as_uint(v));
}

// Roots: the smallest onset per vertex (a minimum, so duplicates resolve the same
// in any order), then (cold start) push the neighbours of every root into the
// first queue.  16 lanes per root: the first applies the onset, all of them push
// the root's neighbours.
constexpr int kRootLanes = 16;

__global__ void k_roots(const int* __restrict__ root_node, const float* __restrict__ root_t,
                        int n_roots, const int* __restrict__ node_int, int n_v,
                        float* __restrict__ troot, float* __restrict__ T, int cold,
                        const int* __restrict__ adj_ptr, const int* __restrict__ adj,
                        int* __restrict__ qout, int* __restrict__ mark, GbpCtl* ctl,
                        XcdQueues xq) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = gid / kRootLanes, lane = gid % kRootLanes;
    if (r >= n_roots) return;
    const int u = root_node[r];
    const float t = root_t[r];
    if (u < 0 || u >= n_v) {
        if (lane == 0) atomicOr(&ctl->err, ERRBIT_ROOT_RANGE);
        return;
    }
    const int i = node_int[u];
    if (lane == 0) {
        if (!finitef(t)) {
            atomicOr(&ctl->err, ERRBIT_ROOT_NONFINITE);
        } else {
            atomic_min_float(&troot[i], t);
            if (cold) {
                atomic_min_float(&T[i], t);
                atomic_min_float(&ctl->tmin, t);
            }
        }
    }
    if (!cold) return;
    const int stamp = ctl->stamp;
    for (int a = adj_ptr[i] + lane; a < adj_ptr[i + 1]; a += kRootLanes) {
        const int nb = adj[a];
        if (atomicMax(&mark[nb], stamp) < stamp) {
            const int x = xcd_of(nb, xq.R);
            qout[xq.off[x] + atomicAdd(&ctl->qcnt[0][x], 1)] = nb;
        }
    }
}

// Two-sided warm start: a connected component without a root has no finite fixed
// point to reach (each round would raise its values by at least an edge cost), so
// its guess is dropped to +inf.  Components holding a root vertex (finite onset)
// are flagged, then the others cleared.
__global__ void k_comp_flag(const float* __restrict__ troot, const int* __restrict__ comp, int n_v,
                            int* __restrict__ comp_root) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_v && troot[i] < GBP_INF) comp_root[comp[i]] = 1;
}

__global__ void k_comp_clear(const int* __restrict__ comp, const int* __restrict__ comp_root, int n_v,
                             float* __restrict__ T) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_v && !comp_root[comp[i]]) T[i] = GBP_INF;
}

__global__ void k_fill_int(int* __restrict__ p, int v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_queue_all(int* __restrict__ q, int* __restrict__ mark, int n_v, GbpCtl* ctl,
                            XcdQueues xq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 8) ctl->qcnt[0][i] = xq.off[i + 1] - xq.off[i];
    if (i < n_v) {
        q[xq.off[xcd_of(i, xq.R)] + xcd_rank(i, xq.R)] = i;
        mark[i] = ctl->stamp;
    }
}

// Control-block reset at the start of a call.  The queue stamp base survives;
// so does the forward's status bit when a backward starts (keep_fwd), so that one
// status read after a captured iteration reports both passes.
__global__ void k_ctl_reset(GbpCtl* ctl, int keep_fwd) {
    if (threadIdx.x == 0) {
        const int stamp = ctl->stamp;
        const int st = keep_fwd ? (ctl->status & 1) : 0;
        const int err = keep_fwd == 2 ? ctl->err : 0;   // 2: mid-call reset, keep input errors
        GbpCtl z{};
        z.tmin = GBP_INF;
        z.marks_stale = stamp > (1 << 30) ? 1 : 0;
        z.stamp = z.marks_stale ? 1 : stamp;
        z.status = st;
        z.err = err;
        *ctl = z;
    }
}

// After `launched` relaxation rounds: advance the stamp base past every stamp
// used, and flag non-convergence if the next queue is not empty.
__global__ void k_forward_end(GbpCtl* ctl, int launched) {
    if (threadIdx.x == 0) {
        ctl->stamp += launched + 2;
        int left = 0;
        for (int x = 0; x < 8; ++x) left += ctl->qcnt[launched % 3][x];
        // vertices still held in buckets beyond the current one (hold-back)
        const int bc = ctl->bcur[launched % 3];
        for (int k = 1; k < kHoldBuckets; ++k) left += ctl->bcnt[(bc + k) & (kHoldBuckets - 1)];
        if (left != 0) ctl->status |= 1;
    }
}

// Step constant of Alg. 1 for every face (4 per element, face K of element t at 4t + K).
__global__ void k_fista_lip(const float4* __restrict__ tetg, int n_e, int mode,
                            float* __restrict__ lip) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4LL * n_e) return;
    const long long t = i >> 2;
    lip[i] = fista_lipschitz(face_q_rt(tetg[2 * t], tetg[2 * t + 1], (int)(i & 3)), mode);
}

// ------------------------------------------------------------------ relaxation
template <int K>
__device__ __forceinline__ void relax_slot(int& e, int cnt, const int* __restrict__ nent,
                                           const int4* __restrict__ tetv,
                                           const float4* __restrict__ tetg, const float* T,
                                           float& best) {
    for (int c = 0; c < cnt; ++c) {
        const int t = nent[e + c];
        const int4 v = tetv[t];
        const float4 g0 = tetg[2 * (size_t)t], g1 = tetg[2 * (size_t)t + 1];
        int a, b, cc;
        face_nodes<K>(v, a, b, cc);
        const float pa = T[a], pb = T[b], pc = T[cc];
        best = fminf(best, local_min<false>(face_q<K>(g0, g1), pa, pb, pc));
    }
    e += cnt;
}

// One relaxation round.  Each vertex of the queue is handled by L lanes (8, 16 or
// 32, autotuned); lane c evaluates local problems c and c+L of the vertex's patch (slot picked at run
// time, both problems' loads in flight together), a 16-lane min-reduction forms
// the Hopf-Lax minimum, and on a change the lanes push the unique neighbours.
// SOLVER 0: the exact predicated solve; 1: Alg. 1 with the face's step constant
// lip[4 t + K], n_f iterations (tau = 0) or the face's count for tolerance tau.
template <int SOLVER>
__device__ __forceinline__ float face_value(const int* __restrict__ nent,
                                            const int4* __restrict__ tetv,
                                            const float4* __restrict__ tetg, const float* T,
                                            int e, int K, const float* __restrict__ lip, int n_f,
                                            float tau) {
    const int t = nent[e];
    const int4 v = tetv[t];
    const float4 g0 = tetg[2 * (size_t)t], g1 = tetg[2 * (size_t)t + 1];
    int a, b, cc;
    face_nodes_sel(v, K, a, b, cc);
    if constexpr (SOLVER == 0) return local_min<false>(face_q_rt(g0, g1, K), T[a], T[b], T[cc]);
    else {
        const float L = lip[4 * (size_t)t + K];
        return local_fista<false>(face_q_rt(g0, g1, K), T[a], T[b], T[cc], L, fista_iters(L, tau, n_f));
    }
}

// Hold-back (HOLD, cold rounds only): Delta-stepping on the active list.  Bucket b
// holds values in [tmin + b Delta, tmin + (b+1) Delta).  A vertex whose value drops
// into a bucket beyond the current one does not push its neighbours yet: it is
// appended to that bucket's list (once per bucket) and waits.  A round that finds
// the queue shorter than open_below (the rest of the current bucket's tail, too
// short to fill the grid) also opens the next non-empty bucket: every listed vertex
// whose value has not dropped below that bucket pushes its neighbours (values
// beyond the ring's last bucket wait there).  With a guess of the solution
// (guess non-null) the evaluation waits instead: a changed vertex pushes its
// neighbours at once, but a neighbour whose guess lies beyond the window goes to
// its guess's bucket list, not the queue, and is queued once that bucket opens,
// when its upwind neighbours (smaller guesses) have had their turn; with a good
// guess most vertices are evaluated about once.  Only the order of the
// relaxation changes (every held vertex is released before the solve ends), so
// the fixed point is the same for any guess; a vertex that finds its bucket's
// list full is pushed (or queued) at once.
struct HoldArgs {
    int* hold;          // [n_v] bucket a vertex was last appended to
    int* blist;         // [kHoldBuckets * bcap]
    int bcap;
    float inv_delta;
    int open_below;     // open the next bucket once the queue is shorter than this
    int window;         // buckets past the current one that propagate at once (>= 0)
    const float* guess; // [n_v] ordering guess (internal order) or null
};

__device__ __forceinline__ int bucket_of(float t, float tmin, float inv_delta) {
    return (int)fminf(floorf((t - tmin) * inv_delta), (float)(1 << 30));
}

constexpr int kHoldStage = 1024;   // held vertices staged per block in LDS

// List vertex v in bucket b (once: a vertex already listed there is left alone).
// Staged in the block's LDS (the block reserves list room per ring slot at its
// end: one global atomic per slot, not per vertex), else appended directly.
// False: the list is full (the caller pushes at once).
__device__ __forceinline__ bool hold_list(int v, int b, const HoldArgs& ha, GbpCtl* ctl,
                                          int* hold_v, unsigned char* hold_s, int* hold_n) {
    if (ha.hold[v] == b) return true;
    const int slot = b & (kHoldBuckets - 1);
    const int hp = atomicAdd(hold_n, 1);
    if (hp < kHoldStage) {
        hold_v[hp] = v;
        hold_s[hp] = (unsigned char)slot;
        ha.hold[v] = b;
        return true;
    }
    const int pos = atomicAdd(&ctl->bcnt[slot], 1);
    if (pos < ha.bcap) {
        ha.blist[(size_t)slot * ha.bcap + pos] = v;
        ha.hold[v] = b;
        return true;
    }
    return false;
}

template <bool TWO_SIDED, int L, int SOLVER, bool HOLD>
__global__ void __launch_bounds__(TPB)
    k_sweep(const int2* __restrict__ nptr, const int* __restrict__ nent,
            const int4* __restrict__ tetv, const float4* __restrict__ tetg,
            const float* __restrict__ troot, float* T, const int* __restrict__ qin,
            int* __restrict__ qout, const int* __restrict__ adj_ptr, const int* __restrict__ adj,
            int* __restrict__ mark, GbpCtl* ctl, unsigned long long* __restrict__ blk, int s,
            float eps_rel, int n_v, XcdQueues xq, const float* __restrict__ lip, int n_f,
            float tau, int* __restrict__ st, HoldArgs ha) {
    static_assert(!(HOLD && TWO_SIDED), "hold-back is a cold-start ordering");
    constexpr int PER_BLOCK = TPB / L;
    // blocks are placed on the 8 XCDs round-robin: with the split layout block b
    // serves sub-queue b % 8, else every block serves the one queue
    const bool split = xq.nq == 8;
    const int x = split ? (blockIdx.x & 7) : 0;
    const int lb = split ? (blockIdx.x >> 3) : blockIdx.x;
    const int nbx = split ? (gridDim.x + 7 - x) >> 3 : gridDim.x;
    const int* qx = qin + xq.off[x];
    // the first queue entry of this lane group is loaded before the queue length
    // is known (both loads in flight together); it is used only if it is in the
    // queue, and clamped so that a stale entry never indexes out of range
    const int qi0 = lb * PER_BLOCK + threadIdx.x / L;
    const int pre = qi0 < xq.off[x + 1] - xq.off[x] ? qx[qi0] : 0;
    const int n = ctl->qcnt[s % 3][x];
    const int stamp_next = ctl->stamp + s + 1;
    // hold-back: the current bucket, and whether this round opens the next one
    int bc = 0, bopen = -1, nopen = 0;
    float tmin = 0.f;
    if constexpr (HOLD) {
        bc = ctl->bcur[s % 3];
        tmin = ctl->tmin;
        int tot = 0;
        for (int xs = 0; xs < 8; ++xs) tot += ctl->qcnt[s % 3][xs];
        if (tot == 0) {
            // nothing is evaluated, so no list grows: skip to the next non-empty bucket
            // (lane k of each wave reads bucket bc + 1 + k, a ballot finds the first)
            const int k = threadIdx.x & 63;
            const int c = k < kHoldBuckets - 1 ? ctl->bcnt[(bc + 1 + k) & (kHoldBuckets - 1)] : 0;
            const unsigned long long nz = __ballot(c > 0);
            if (nz) {
                const int first = __ffsll(nz) - 1;
                bopen = bc + 1 + first;
                nopen = min(__shfl(c, first), ha.bcap);
            }
        } else if (tot < ha.open_below) {
            // the tail of the current bucket: open the next one beside it; this
            // round holds nothing in it (its list stays as counted here)
            bopen = bc + 1;
            nopen = min(ctl->bcnt[bopen & (kHoldBuckets - 1)], ha.bcap);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            // the bucket the last round opened has been consumed: its slot is free
            if (bc != ctl->bcur[(s + 2) % 3]) ctl->bcnt[bc & (kHoldBuckets - 1)] = 0;
            ctl->bcur[(s + 1) % 3] = bopen >= 0 ? bopen : bc;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < 8) {
        int left = ctl->qcnt[s % 3][threadIdx.x];
        ctl->qcnt[(s + 2) % 3][threadIdx.x] = 0;
        if (HOLD && threadIdx.x == 0 && nopen > 0) left = max(left, 1);
        if (left > 0) atomicMax(&ctl->rounds, s + 1);
        if (st) {   // status for the host: this round's work, error bits, round index
            st[threadIdx.x] = left;
            if (threadIdx.x == 0) {
                st[8] = ctl->err;
                st[9] = s;
            }
        }
    }
    int* cnt_next = ctl->qcnt[(s + 1) % 3];
    constexpr int CAP = TWO_SIDED ? kPushCapWide : kPushCap;
    __shared__ int push_q[CAP];
    __shared__ int push_n, push_cnt[8], push_base[8];
    // held vertices staged per block (HOLD): vertex, ring slot
    __shared__ int hold_v[HOLD ? kHoldStage : 1];
    __shared__ unsigned char hold_s[HOLD ? kHoldStage : 1];
    __shared__ int hold_n, hold_cnt[HOLD ? kHoldBuckets : 1], hold_base[HOLD ? kHoldBuckets : 1];
    // an opening takes one lane group per listed vertex (its neighbours are pushed),
    // or one thread (ordered: the vertex itself is queued)
    const int open_per_block = HOLD && ha.guess ? TPB : PER_BLOCK;
    const bool have_open = HOLD && bopen >= 0 && (int)blockIdx.x * open_per_block < nopen;
    if (lb * PER_BLOCK >= n && !have_open) return;   // no vertex for this block
    if (threadIdx.x == 0) {
        push_n = 0;
        hold_n = 0;
    }
    __syncthreads();
    const XPushBuf pb{push_q, &push_n, CAP};
    const int lane = threadIdx.x & (L - 1);
    const int sub = threadIdx.x / L;                // vertex slot of this lane group
    unsigned long long solves = 0, upd = 0;
    // software pipeline over the lane group's passes (hold-back rounds): the queue
    // entry two passes ahead and the vertex record (patch pointer, value, neighbour
    // range) one pass ahead are in flight while the current vertex is relaxed (T[i]
    // has one writer, the group that holds i, and i is queued at most once per round).
    // Measured: it pays on the hold-back's short rounds and costs on long plain ones
    // (many passes per block, where the extra loads in flight compete for the memory
    // pipeline), so plain and two-sided rounds load each vertex when they reach it.
    constexpr bool PIPE = HOLD;
    const int stride = nbx * PER_BLOCK;
    int f_iq = 0;                                   // entry of the next pass
    int2 c_p = make_int2(0, 0);                     // record of the current pass
    float c_t = 0.f, c_tr = 0.f;
    int c_a0 = 0, c_a1 = 0, c_i = 0;
    if constexpr (PIPE) {
        const int q0 = lb * PER_BLOCK + sub, q1 = q0 + stride;
        const int iq0 = q0 < n ? pre : 0;
        c_i = min(max(iq0, 0), n_v - 1);
        c_p = q0 < n ? nptr[c_i] : make_int2(0, 0);
        c_t = T[c_i];
        c_tr = TWO_SIDED ? troot[c_i] : 0.f;
        c_a0 = adj_ptr[c_i];
        c_a1 = adj_ptr[c_i + 1];
        f_iq = q1 < n ? qx[q1] : 0;
    }
    for (int base = lb * PER_BLOCK; base < n; base += stride) {
        const int qi = base + sub;
        const bool act = qi < n;                    // uniform over the lane group
        if constexpr (!PIPE) {
            const int iq = act ? (qi == qi0 ? pre : qx[qi]) : 0;
            c_i = min(max(iq, 0), n_v - 1);
            c_p = act ? nptr[c_i] : make_int2(0, 0);
            c_t = T[c_i];
            c_tr = TWO_SIDED ? troot[c_i] : 0.f;
            c_a0 = adj_ptr[c_i];
            c_a1 = adj_ptr[c_i + 1];
        }
        const int i = c_i;
        const int2 p = c_p;
        const float told = c_t;
        const float tr = c_tr;
        const int adj0 = c_a0, adj1 = c_a1;
        if constexpr (PIPE) {
            const int q1 = qi + stride, q2 = qi + 2 * stride;
            c_i = min(max(f_iq, 0), n_v - 1);
            c_p = q1 < n ? nptr[c_i] : make_int2(0, 0);
            c_t = T[c_i];
            c_tr = TWO_SIDED ? troot[c_i] : 0.f;
            c_a0 = adj_ptr[c_i];
            c_a1 = adj_ptr[c_i + 1];
            f_iq = q2 < n ? qx[q2] : 0;
        }
        const int c0 = p.y & 255, c1 = (p.y >> 8) & 255, c2 = (p.y >> 16) & 255,
                  c3 = (p.y >> 24) & 255;
        const int e01 = c0 + c1, e012 = e01 + c2;
        const int tot = e012 + c3;
        float best = GBP_INF;
        if constexpr (SOLVER == 1 && L == 8) {
            // FISTA rounds are bound by arithmetic: at 8 lanes each lane takes local
            // problems c, c + 8 and c + 16, so a 24-element patch fills three
            // passes with no idle slot (two passes of 16 lanes leave 8 of 32 idle)
            for (int c = lane; c < tot; c += 3 * L) {
                float v3[3];
                bool ok3[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int d = c + k * L;
                    ok3[k] = k == 0 || d < tot;
                    const int dd = ok3[k] ? d : c;
                    const int Kd = (dd < c0) ? 0 : (dd < e01) ? 1 : (dd < e012) ? 2 : 3;
                    v3[k] = face_value<SOLVER>(nent, tetv, tetg, T, p.x + dd, Kd, lip, n_f, tau);
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    best = fminf(best, ok3[k] ? v3[k] : GBP_INF);
                    solves += ok3[k] ? 1 : 0;
                }
            }
        } else {
            for (int c = lane; c < tot; c += 2 * L) {
                const int d = c + L;       // second local problem of this lane
                const bool okd = d < tot;
                const int Kc = (c < c0) ? 0 : (c < e01) ? 1 : (c < e012) ? 2 : 3;
                const int Kd = (d < c0) ? 0 : (d < e01) ? 1 : (d < e012) ? 2 : 3;
                const float vc = face_value<SOLVER>(nent, tetv, tetg, T, p.x + c, Kc, lip, n_f, tau);
                const float vd = face_value<SOLVER>(nent, tetv, tetg, T, p.x + (okd ? d : c),
                                                    okd ? Kd : Kc, lip, n_f, tau);
                best = fminf(best, okd ? fminf(vc, vd) : vc);
                solves += okd ? 2 : 1;
            }
        }
        for (int o = L / 2; o > 0; o >>= 1) best = fminf(best, __shfl_xor(best, o));
        if (!act) continue;
        bool changed;
        if (TWO_SIDED) {
            best = fminf(best, tr);
            if (lane == 0 && best != told) T[i] = best;
            const bool bf = best < GBP_INF, tf = told < GBP_INF;
            changed = (bf != tf) ||
                      (bf && fabsf(best - told) > eps_rel * fmaxf(1.f, fabsf(told)));
        } else {
            if (lane == 0 && best < told) T[i] = best;   // the only writer of T[i]
            changed = (told < GBP_INF) ? (best < told - eps_rel * fmaxf(1.f, fabsf(told)))
                                       : (best < GBP_INF);
        }
        if (changed) {
            if (lane == 0) ++upd;
            // hold-back: the bucket opened by this round, if any, counts as current;
            // lists go to buckets after it, up to the ring's last (blast)
            int bce = 0, blast = 0;
            bool can_hold = false;
            if constexpr (HOLD) {
                bce = (bopen >= 0 ? bopen : bc) + ha.window;
                blast = bc + kHoldBuckets - 1;
                can_hold = max(bopen, bc) < blast;
            }
            if (HOLD && !ha.guess) {
                int b = bucket_of(best, tmin, ha.inv_delta);
                if (b > bce && can_hold) {   // beyond the window: wait in b's list
                    b = min(b, blast);
                    int ok = 0;
                    if (lane == 0) ok = hold_list(i, b, ha, ctl, hold_v, hold_s, &hold_n) ? 1 : 0;
                    if (__shfl(ok, (threadIdx.x & 63) & ~(L - 1))) continue;
                }
            }
            for (int a = adj0 + lane; a < adj1; a += L) {
                const int nb = adj[a];
                if (HOLD && ha.guess) {
                    // ordered: a neighbour whose guess is beyond the window waits
                    const float gn = ha.guess[nb];
                    if (atomicMax(&mark[nb], stamp_next) < stamp_next) {
                        const int b = bucket_of(gn, tmin, ha.inv_delta);
                        if (b <= bce || !can_hold ||
                            !hold_list(nb, min(b, blast), ha, ctl, hold_v, hold_s, &hold_n))
                            xpush_node<false>(pb, nb, xq, qout, cnt_next);
                    }
                    continue;
                }
                if (atomicMax(&mark[nb], stamp_next) < stamp_next)
                    xpush_node<TWO_SIDED>(pb, nb, xq, qout, cnt_next);
            }
        }
    }
    if constexpr (HOLD) {
        if (have_open && ha.guess) {
            // ordered: open bucket bopen by queueing every vertex still listed in it
            const int* lst = ha.blist + (size_t)(bopen & (kHoldBuckets - 1)) * ha.bcap;
            for (int qi = blockIdx.x * TPB + threadIdx.x; qi < nopen; qi += gridDim.x * TPB) {
                const int v = lst[qi];
                if (ha.hold[v] == bopen && atomicMax(&mark[v], stamp_next) < stamp_next)
                    xpush_node<true>(pb, v, xq, qout, cnt_next);
            }
        } else if (have_open) {
            // open bucket bopen: every listed vertex not below it pushes its neighbours
            const int* lst = ha.blist + (size_t)(bopen & (kHoldBuckets - 1)) * ha.bcap;
            for (int qi = blockIdx.x * PER_BLOCK + sub; qi < nopen; qi += gridDim.x * PER_BLOCK) {
                const int v = lst[qi];
                // stale: re-held in a lower bucket, or pushed already from the current
                // one; a value beyond bopen was clamped into the ring's last bucket
                if (ha.hold[v] != bopen || bucket_of(T[v], tmin, ha.inv_delta) < bopen) continue;
                for (int a = adj_ptr[v] + lane; a < adj_ptr[v + 1]; a += L) {
                    const int nb = adj[a];
                    if (atomicMax(&mark[nb], stamp_next) < stamp_next)
                        xpush_node<false>(pb, nb, xq, qout, cnt_next);
                }
            }
        }
    }
    if constexpr (HOLD) {
        // the staged holds and the pushed vertices together: count per ring slot and
        // per sub-queue, reserve room with one atomic per non-empty slot or sub-queue
        // (all in one pass), scatter; a vertex that finds its list full pushes its
        // neighbours straight to the global queue
        __syncthreads();
        const int nh = min(hold_n, kHoldStage);
        const int np = min(push_n, CAP);
        if (threadIdx.x < kHoldBuckets) hold_cnt[threadIdx.x] = 0;
        if (threadIdx.x < 8) push_cnt[threadIdx.x] = 0;
        __syncthreads();
        for (int k = threadIdx.x; k < nh; k += blockDim.x) atomicAdd(&hold_cnt[hold_s[k]], 1);
        if (split)
            for (int k = threadIdx.x; k < np; k += blockDim.x) atomicAdd(&push_cnt[xcd_of(push_q[k], xq.R)], 1);
        else if (threadIdx.x == 0)
            push_cnt[0] = np;
        __syncthreads();
        if (threadIdx.x < kHoldBuckets) {
            const int m = hold_cnt[threadIdx.x];
            hold_base[threadIdx.x] = m > 0 ? atomicAdd(&ctl->bcnt[threadIdx.x], m) : 0;
            hold_cnt[threadIdx.x] = 0;
        } else if (threadIdx.x < kHoldBuckets + 8) {
            const int xs = threadIdx.x - kHoldBuckets;
            const int m = push_cnt[xs];
            push_base[xs] = m > 0 ? xq.off[xs] + atomicAdd(&cnt_next[xs], m) : 0;
            push_cnt[xs] = 0;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nh; k += blockDim.x) {
            const int v = hold_v[k], sl = hold_s[k];
            const int pos = hold_base[sl] + atomicAdd(&hold_cnt[sl], 1);
            if (pos < ha.bcap) {
                ha.blist[(size_t)sl * ha.bcap + pos] = v;
            } else if (ha.guess) {
                ha.hold[v] = INT_MIN;   // its list is full: queued now (claimed this round)
                const int x2 = split ? xcd_of(v, xq.R) : 0;
                qout[xq.off[x2] + atomicAdd(&cnt_next[x2], 1)] = v;
            } else {
                ha.hold[v] = INT_MIN;
                for (int a = adj_ptr[v]; a < adj_ptr[v + 1]; ++a) {
                    const int nb = adj[a];
                    if (atomicMax(&mark[nb], stamp_next) < stamp_next) {
                        const int x2 = split ? xcd_of(nb, xq.R) : 0;
                        qout[xq.off[x2] + atomicAdd(&cnt_next[x2], 1)] = nb;
                    }
                }
            }
        }
        if (split) {
            for (int k = threadIdx.x; k < np; k += blockDim.x) {
                const int v = push_q[k];
                const int x2 = xcd_of(v, xq.R);
                qout[push_base[x2] + atomicAdd(&push_cnt[x2], 1)] = v;
            }
        } else {
            for (int k = threadIdx.x; k < np; k += blockDim.x) qout[push_base[0] + k] = push_q[k];
        }
    } else {
        xpush_flush(pb, xq, qout, cnt_next, push_cnt, push_base);
    }
    // per-block counters: one writer per slot, no contended atomics
    block_sum2_u64(solves, upd);
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&blk[2 * blockIdx.x], solves, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&blk[2 * blockIdx.x + 1], upd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_count_inf(const float* __restrict__ T, int n_v, GbpCtl* ctl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long c = (i < n_v && !(T[i] < GBP_INF)) ? 1ull : 0ull;
    const unsigned long long t = block_sum_u64(c);
    if (threadIdx.x == 0 && t) atomicAdd(&ctl->unreached, (int)t);
}

// ------------------------------------------------------------------ parents
// The parent of a vertex is an argmin over its local problems: a decision taken
// by floating point.  It is taken here in FP64 from the raw inputs (coordinates,
// velocity tensor, nodal scales, activation times), the precision of the
// reference, so that near-ties resolve the same way on both sides.
struct Sym64 {
    double xx, yy, zz, xy, xz, yz;
};

__device__ __forceinline__ Sym64 inv_metric64(const float* __restrict__ D6, double sbar) {
    const double a = D6[0], b = D6[1], c = D6[2], d = D6[3], e = D6[4], f = D6[5];
    const double A00 = b * c - f * f, A11 = a * c - e * e, A22 = a * b - d * d;
    const double A01 = e * f - d * c, A02 = d * f - e * b, A12 = d * e - a * f;
    const double s = 1.0 / ((a * A00 + d * A01 + e * A02) * sbar * sbar);
    return Sym64{A00 * s, A11 * s, A22 * s, A01 * s, A02 * s, A12 * s};
}

__device__ __forceinline__ double quad64(const Sym64& M, double x0, double x1, double x2, double y0,
                                         double y1, double y2) {
    return x0 * (M.xx * y0 + M.xy * y1 + M.xz * y2) + x1 * (M.xy * y0 + M.yy * y1 + M.yz * y2) +
           x2 * (M.xz * y0 + M.yz * y1 + M.zz * y2);
}

// FP64 value and weights of the local problem of entry `e` (slot K) of vertex i,
// from the raw inputs (coordinates, velocity tensor, nodal scales, T).
__device__ __forceinline__ double parent_face64(int t, int K, int self, const int4* __restrict__ tetv,
                                                const int* __restrict__ tet_user,
                                                const float* __restrict__ D,
                                                const float* __restrict__ vs,
                                                const float4* __restrict__ xyz,
                                                const float* __restrict__ T, double& a0,
                                                double& a1, double& a2) {
    const float4 xi = xyz[self];
    const int4 v = tetv[t];
    const double sbar = 0.25 * ((double)vs[v.x] + (double)vs[v.y] + (double)vs[v.z] + (double)vs[v.w]);
    const Sym64 M = inv_metric64(D + 6 * (size_t)tet_user[t], sbar);
    int n0, n1, n2;
    face_nodes_sel(v, K, n0, n1, n2);
    const float4 x0 = xyz[n0], x1 = xyz[n1], x2 = xyz[n2];
    const double e0x = (double)x0.x - xi.x, e0y = (double)x0.y - xi.y, e0z = (double)x0.z - xi.z;
    const double e1x = (double)x1.x - xi.x, e1y = (double)x1.y - xi.y, e1z = (double)x1.z - xi.z;
    const double e2x = (double)x2.x - xi.x, e2y = (double)x2.y - xi.y, e2z = (double)x2.z - xi.z;
    LocalQT<double> q;
    q.q00 = quad64(M, e0x, e0y, e0z, e0x, e0y, e0z);
    q.q11 = quad64(M, e1x, e1y, e1z, e1x, e1y, e1z);
    q.q22 = quad64(M, e2x, e2y, e2z, e2x, e2y, e2z);
    q.q01 = quad64(M, e0x, e0y, e0z, e1x, e1y, e1z);
    q.q02 = quad64(M, e0x, e0y, e0z, e2x, e2y, e2z);
    q.q12 = quad64(M, e1x, e1y, e1z, e2x, e2y, e2z);
    return local_min<true, double>(q, (double)T[n0], (double)T[n1], (double)T[n2], &a0, &a1, &a2);
}

// Parents: L lanes per vertex.  Every local problem of the patch is first solved
// in FP32 (from the element Gram records); only those within 1e-4*max(1,|T|) of
// the FP32 minimum -- a margin about a hundred times the FP32 error -- are
// solved again in FP64, and the FP64 values decide the argmin (ties: first
// entry in (slot, element) order).
// The FP64 candidates are few per vertex (the minimum and its near-ties), so they
// are gathered per block in LDS and solved densely, one per thread: solved in the
// lane that found them, one candidate anywhere in a wave would hold all 64 lanes
// for the whole FP64 solve.  A candidate that finds the list full is solved in
// its own lane.  Same values, same tie rule: the result does not depend on where
// a candidate was solved.
constexpr int kParCands = 512;   // FP64 candidates per block held in LDS
constexpr int kParLanes = 8;     // lanes per vertex: 3 passes cover a 24-element patch

template <int L>
__global__ void __launch_bounds__(TPB)
    k_parent(const int2* __restrict__ nptr, const int* __restrict__ nent,
             const int4* __restrict__ tetv, const float4* __restrict__ tetg,
             const int* __restrict__ tet_user, const float* __restrict__ D,
             const float* __restrict__ vs, const float4* __restrict__ xyz,
             const float* __restrict__ T, const float* __restrict__ troot, int n_v,
             int* __restrict__ par, float4* __restrict__ pa) {
    constexpr int VPB = TPB / L;                    // vertices per block
    __shared__ int cand_key[kParCands];             // vertex slot << 16 | entry position
    __shared__ double cand_val[kParCands];
    __shared__ float cand_w[kParCands][3];
    __shared__ int n_cand;
    if (threadIdx.x == 0) n_cand = 0;
    __syncthreads();
    const int lane = threadIdx.x & (L - 1);
    const int slot = threadIdx.x / L;
    const int i0 = blockIdx.x * VPB + slot;
    const bool act = i0 < n_v;                      // uniform over the lane group
    const int i = act ? i0 : 0;
    const bool reached = act && T[i] < GBP_INF;
    const int2 p = reached ? nptr[i] : make_int2(0, 0);
    const int c0 = p.y & 255, c1 = (p.y >> 8) & 255, c2 = (p.y >> 16) & 255, c3 = (p.y >> 24) & 255;
    const int e01 = c0 + c1, e012 = e01 + c2, tot = e012 + c3;
    // FP32 screen.  The lane's first kKeep entries (c = lane, lane + L, ...) are
    // solved together -- their loads in flight at once, an entry past the patch
    // repeating entry 0 and discarded -- and kept for the second pass.
    constexpr int kKeep = 3;
    auto screen = [&](int c) {
        const int K = (c < c0) ? 0 : (c < e01) ? 1 : (c < e012) ? 2 : 3;
        const int t = nent[p.x + c];
        const int4 v = tetv[t];
        int a, b, cc;
        face_nodes_sel(v, K, a, b, cc);
        return local_min<false>(face_q_rt(tetg[2 * (size_t)t], tetg[2 * (size_t)t + 1], K), T[a], T[b],
                                T[cc]);
    };
    float keep[kKeep];
    float b32 = GBP_INF;
    if (tot > 0) {
        float v3[kKeep];
#pragma unroll
        for (int h = 0; h < kKeep; ++h) v3[h] = screen(lane + h * L < tot ? lane + h * L : 0);
#pragma unroll
        for (int h = 0; h < kKeep; ++h) {
            keep[h] = lane + h * L < tot ? v3[h] : GBP_INF;
            b32 = fminf(b32, keep[h]);
        }
    }
    for (int c = lane + kKeep * L; c < tot; c += L) b32 = fminf(b32, screen(c));
    for (int o = L / 2; o > 0; o >>= 1) b32 = fminf(b32, __shfl_xor(b32, o));
    const float cut = b32 + 1e-4f * fmaxf(1.f, fabsf(b32));
    // candidates of the FP64 decision: into the block's list, or (list full) solved here
    double best = __builtin_huge_val(), b0 = 0, b1 = 0, b2 = 0;
    int bpos = 0x7fffffff;
    for (int c = lane, k = 0; c < tot && b32 < GBP_INF; c += L, ++k) {
        float v32;
        if (k < kKeep) {
            v32 = k == 0 ? keep[0] : k == 1 ? keep[1] : keep[2];
        } else {
            v32 = screen(c);
        }
        if (!(v32 <= cut)) continue;
        const int q = atomicAdd(&n_cand, 1);
        if (q < kParCands) {
            cand_key[q] = (slot << 16) | c;
            continue;
        }
        const int K = (c < c0) ? 0 : (c < e01) ? 1 : (c < e012) ? 2 : 3;
        double x0, x1, x2;
        const double val = parent_face64(nent[p.x + c], K, i, tetv, tet_user, D, vs, xyz, T, x0, x1, x2);
        if (val < best) {
            best = val;
            bpos = c;
            b0 = (float)x0;
            b1 = (float)x1;
            b2 = (float)x2;
        }
    }
    __syncthreads();
    const int nc = min(n_cand, kParCands);
    // dense FP64 solves of the listed candidates
    for (int q = threadIdx.x; q < nc; q += blockDim.x) {
        const int key = cand_key[q];
        const int vi = blockIdx.x * VPB + (key >> 16), c = key & 0xffff;
        const int2 pq = nptr[vi];
        const int q0 = pq.y & 255, q01 = q0 + ((pq.y >> 8) & 255), q012 = q01 + ((pq.y >> 16) & 255);
        const int K = (c < q0) ? 0 : (c < q01) ? 1 : (c < q012) ? 2 : 3;
        double x0, x1, x2;
        cand_val[q] = parent_face64(nent[pq.x + c], K, vi, tetv, tet_user, D, vs, xyz, T, x0, x1, x2);
        cand_w[q][0] = (float)x0;
        cand_w[q][1] = (float)x1;
        cand_w[q][2] = (float)x2;
    }
    __syncthreads();
    // each lane group takes its own vertex's listed candidates
    for (int q = lane; q < nc; q += L) {
        const int key = cand_key[q];
        if ((key >> 16) != slot) continue;
        const int c = key & 0xffff;
        const double val = cand_val[q];
        if (val < best || (val == best && c < bpos)) {
            best = val;
            bpos = c;
            b0 = cand_w[q][0];
            b1 = cand_w[q][1];
            b2 = cand_w[q][2];
        }
    }
    // group argmin of (value, entry position)
    for (int o = L / 2; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int op = __shfl_xor(bpos, o);
        const double o0 = __shfl_xor(b0, o), o1 = __shfl_xor(b1, o), o2 = __shfl_xor(b2, o);
        if (ob < best || (ob == best && op < bpos)) {
            best = ob;
            bpos = op;
            b0 = o0;
            b1 = o1;
            b2 = o2;
        }
    }
    if (!act || lane != 0) return;
    int bpar = -1;
    if (bpos != 0x7fffffff) {
        const int K = (bpos < c0) ? 0 : (bpos < e01) ? 1 : (bpos < e012) ? 2 : 3;
        bpar = (nent[p.x + bpos] << 2) | K;
        if ((double)troot[i] <= best) bpar = -1;   // an active root keeps its onset
    }
    par[i] = bpar;
    pa[i] = make_float4((float)b0, (float)b1, (float)b2, (float)best);
}

__device__ __forceinline__ void face_nodes_rt(const int4 v, int K, int& a, int& b, int& c) {
    switch (K) {
        case 0: a = v.y; b = v.z; c = v.w; break;
        case 1: a = v.x; b = v.z; c = v.w; break;
        case 2: a = v.x; b = v.y; c = v.w; break;
        default: a = v.x; b = v.y; c = v.z; break;
    }
}

// ------------------------------------------------------------------ adjoint
// Parent face vertices carrying weight, and two-cycle detection: a and c are
// partners when each is a weighted parent of the other (the anisotropic scheme
// is not causal).  The mutual edges are left out of the readiness counts; the
// pair is solved jointly once both members' other children are finished.
// (Also clears the child counters and fill cursors the next kernels accumulate into,
// and the entry slots k_child_sort fills.)
__global__ void k_pnodes(const int* __restrict__ par, const float4* __restrict__ pa,
                         const int4* __restrict__ tetv, int n_v, int4* __restrict__ pnode,
                         int* __restrict__ cnt, int* __restrict__ cfill, int4* __restrict__ cslot) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_v) return;
    cnt[c] = 0;
    cfill[c] = 0;
    cslot[c] = make_int4(-1, -1, -1, -1);
    const int pr = par[c];
    int4 out = make_int4(-1, -1, -1, -1);
    if (pr >= 0) {
        int f[3];
        face_nodes_rt(tetv[pr >> 2], pr & 3, f[0], f[1], f[2]);
        const float4 w = pa[c];
        out.x = w.x > 0.f ? f[0] : -1;
        out.y = w.y > 0.f ? f[1] : -1;
        out.z = w.z > 0.f ? f[2] : -1;
    }
    pnode[c] = out;
}

__device__ __forceinline__ bool has_parent(int4 pn, int x) {
    return pn.x == x || pn.y == x || pn.z == x;
}

__global__ void k_partner(const int4* __restrict__ pnode, int n_v, int* __restrict__ partner) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_v) return;
    const int4 pn = pnode[a];
    const int cand[3] = {pn.x, pn.y, pn.z};
    int best = -1;
    for (int k = 0; k < 3; ++k)
        if (cand[k] >= 0 && has_parent(pnode[cand[k]], a) && (best < 0 || cand[k] < best))
            best = cand[k];
    partner[a] = best;
}

// keep a pair only if both members chose each other; prime the pair counter
// (pairrem: 2 at the smaller member of a pair, -1 at the larger, 0 elsewhere)
__global__ void k_partner_sym(const int* __restrict__ partner, int n_v, int* __restrict__ pairrem) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_v) return;
    const int c = partner[a];
    const bool ok = c >= 0 && partner[c] == a;
    pairrem[a] = ok ? (a < c ? 2 : -1) : 0;
}

__global__ void k_partner_fix(int* __restrict__ partner, int* __restrict__ pairrem, int n_v) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_v) return;
    const int r = pairrem[a];
    if (r == 0) partner[a] = -1;
    if (r < 0) pairrem[a] = 0;
}

// Children per vertex.  (A vertex waits for all of them but its two-cycle
// partner, which is always among them: see k_adj_init.)
__global__ void k_child_count(const int4* __restrict__ pnode, int n_v, int* __restrict__ cnt) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_v) return;
    const int4 pn = pnode[c];
    const int f[3] = {pn.x, pn.y, pn.z};
    for (int k = 0; k < 3; ++k)
        if (f[k] >= 0) atomicAdd(&cnt[f[k]], 1);
}

__global__ void k_child_fill(const int4* __restrict__ pnode, const float4* __restrict__ pa,
                             int n_v, const int* __restrict__ cptr, int* __restrict__ cfill,
                             int* __restrict__ cchild, float* __restrict__ calpha) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_v) return;
    const int4 pn = pnode[c];
    const int f[3] = {pn.x, pn.y, pn.z};
    const float4 w = pa[c];
    const float al[3] = {w.x, w.y, w.z};
    for (int k = 0; k < 3; ++k)
        if (f[k] >= 0) {
            const int pos = cptr[f[k]] + atomicAdd(&cfill[f[k]], 1);
            cchild[pos] = (c << 2) | k;     // unpacked by k_child_sort
            calpha[pos] = al[k];
        }
}

// Position of entry k (rank r in x's sorted child list) in the entry array.
__device__ __forceinline__ int centry(int x, int r, int k, int n_v) {
    return r < kChildSlots ? x * kChildSlots + r : n_v * kChildSlots + k;
}

// Sort each child list by child id (fixed summation order -> deterministic), then
// tell each child where its entry sits (the component of its cslot for this
// parent).  The entries arrive as (child << 2 | which of the child's parents this
// is) from k_child_fill; child ids are distinct within a list, so the packed keys
// sort in child order, and the ids are written back unpacked.
constexpr int kSortRegs = 16;   // child lists up to this long are sorted in registers

__global__ void __launch_bounds__(TPB) k_child_sort(const int* __restrict__ cptr, int* __restrict__ cchild,
                                                    float* __restrict__ calpha, int n_v,
                                                    int4* __restrict__ cslot) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_v) return;
    const int b = cptr[p], e = cptr[p + 1];
    if (e - b <= kSortRegs) {
        // the list in registers (padded with INT_MAX) through a bitonic network
        int ch[kSortRegs];
        float al[kSortRegs];
#pragma unroll
        for (int k = 0; k < kSortRegs; ++k) {
            ch[k] = b + k < e ? cchild[b + k] : INT_MAX;
            al[k] = b + k < e ? calpha[b + k] : 0.f;
        }
#pragma unroll
        for (int k = 2; k <= kSortRegs; k <<= 1)
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
                for (int i = 0; i < kSortRegs; ++i) {
                    const int l = i ^ j;
                    if (l > i) {
                        const int u = ch[i], v = ch[l];
                        const float fu = al[i], fv = al[l];
                        const bool sw = (u > v) == ((i & k) == 0);
                        ch[i] = sw ? v : u;
                        ch[l] = sw ? u : v;
                        al[i] = sw ? fv : fu;
                        al[l] = sw ? fu : fv;
                    }
                }
#pragma unroll
        for (int k = 0; k < kSortRegs; ++k)
            if (b + k < e) {
                const int c = ch[k] >> 2;
                cchild[b + k] = c;
                calpha[b + k] = al[k];
                reinterpret_cast<int*>(&cslot[c])[ch[k] & 3] = centry(p, k, b + k, n_v);
            }
        return;
    }
    for (int x = b + 1; x < e; ++x) {
        const int kc = cchild[x];
        const float ka = calpha[x];
        int y = x - 1;
        while (y >= b && cchild[y] > kc) {
            cchild[y + 1] = cchild[y];
            calpha[y + 1] = calpha[y];
            --y;
        }
        cchild[y + 1] = kc;
        calpha[y + 1] = ka;
    }
    for (int x = b; x < e; ++x) {
        const int v = cchild[x];
        const int c = v >> 2;
        cchild[x] = c;
        reinterpret_cast<int*>(&cslot[c])[v & 3] = centry(p, x - b, x, n_v);
    }
}

// Readiness stamps of the level walk: the launch from which a vertex may be
// finished (0 for leaves), or one of the markers below.
constexpr int kRdyNever = 0x7fffffff;   // waiting for children (or unreached)
constexpr int kRdyWait = 0x7ffffffe;    // first member of a two-cycle, partner not ready
constexpr int kRdyDone = 0x7ffffffd;    // finished
constexpr int kLevelPer = 8;            // vertices per thread in a level scan (grid >= n_v / (8 TPB))

// rem: the children a vertex waits for, all of them (the CSR range) but its
// two-cycle partner, which is one of them (partners are parents of each other).
__global__ void k_adj_init(const float* __restrict__ dLdT_user, const int* __restrict__ node_user,
                           const float* __restrict__ T, const int* __restrict__ cptr,
                           const int* __restrict__ partner, int* __restrict__ rem, int n_v,
                           float* __restrict__ g, float* __restrict__ lam, int* __restrict__ done,
                           int* __restrict__ rdy, float* __restrict__ contrib, GbpCtl* ctl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_v) return;
    // fixed entry slots start at zero: a vertex sums all of them, used or not
    float4* z = reinterpret_cast<float4*>(contrib + (size_t)i * kChildSlots);
#pragma unroll
    for (int k = 0; k < kChildSlots / 4; ++k) z[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    const bool reached = T[i] < GBP_INF;
    float gi = reached ? dLdT_user[node_user[i]] : 0.f;
    if (gi != gi) gi = 0.f;
    g[i] = gi;
    lam[i] = gi;
    done[i] = reached ? 0 : 1;
    const int wait = cptr[i + 1] - cptr[i] - (partner[i] >= 0 ? 1 : 0);
    rem[i] = wait;
    const bool leaf = reached && wait == 0;
    rdy[i] = leaf ? 0 : kRdyNever;
    if (leaf) ctl->count[0] = 1;   // flag: the first launch has work
}

// Fixed entry slot r (0..7) of a vertex from its two loaded float4s.
__device__ __forceinline__ float slot_of(float4 s0, float4 s1, int r) {
    const float4 h = r < 4 ? s0 : s1;
    const int k = r & 3;
    return k == 0 ? h.x : k == 1 ? h.y : k == 2 ? h.z : h.w;
}

// A finished vertex hands alpha * lambda to its entries in its parents' child
// lists (read only in later launches, after this one has ended).
__device__ __forceinline__ void publish_to(float l, int4 cs, float4 w, float* __restrict__ contrib) {
    if (cs.x >= 0) contrib[cs.x] = w.x * l;
    if (cs.y >= 0) contrib[cs.y] = w.y * l;
    if (cs.z >= 0) contrib[cs.z] = w.z * l;
}

__device__ __forceinline__ void publish(int x, float l, const float4* __restrict__ pa,
                                        const int4* __restrict__ cslot, float* __restrict__ contrib) {
    publish_to(l, cslot[x], pa[x], contrib);
}

// A finished vertex releases its parents; a parent whose last child this was
// becomes ready for the next launch (stamped with a plain store: it is only
// read after this launch ends).
__device__ __forceinline__ bool release_from(int4 pn, int skip, int self, int* __restrict__ rem,
                                             int* __restrict__ rdy, int next) {
    const int f[3] = {pn.x, pn.y, pn.z};
    // the three releases in flight together, with no branch between them: a slot
    // without a parent subtracts 0 from the finished vertex's own count (no longer
    // read by anyone), and its result is ignored
    bool v[3];
    int r[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = f[k] >= 0 && f[k] != skip;
        r[k] = atomicSub(&rem[v[k] ? f[k] : self], v[k] ? 1 : 0);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) r[k] = v[k] ? r[k] : 0;
    bool any = false;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (r[k] == 1) {
            rdy[f[k]] = next;
            any = true;
        }
    return any;
}

__device__ __forceinline__ bool release_parents(int x, int skip, const int4* __restrict__ pnode,
                                                int* __restrict__ rem, int* __restrict__ rdy,
                                                int next) {
    return release_from(pnode[x], skip, x, rem, rdy, next);
}

// One leaves-first level, as a scan over all vertices (one thread per vertex):
// every vertex stamped ready for this launch has all (non-partner) children
// finished in earlier launches, so their contributions are visible.  It sums
// lambda = g + sum alpha_c lambda_c over its child entries in a fixed order
// (deterministic; each child wrote its alpha_c lambda_c there), then writes its
// own contributions to its parents' entries; the second
// member of a two-cycle to become ready solves the pair
//   lam_a = S_a + w_ca lam_c,  lam_c = S_c + w_ac lam_a.
__global__ void __launch_bounds__(TPB)
    k_adj_level(int* __restrict__ rdy, const int* __restrict__ cptr,
                const int* __restrict__ cchild, const float* __restrict__ calpha,
                const float* __restrict__ g, float* lam, int* __restrict__ done,
                const int4* __restrict__ pnode, const float4* __restrict__ pa,
                const int4* __restrict__ cslot, float* __restrict__ contrib,
                const int* __restrict__ partner, int* __restrict__ pairrem, int* __restrict__ rem,
                int n_v, GbpCtl* ctl, int s, int* __restrict__ st) {
    // up to kLevelPer vertices per thread: their stamps are loaded together, and
    // before the work flag, so that all these loads are in flight at once
    const int stride = gridDim.x * blockDim.x;
    const int xb = blockIdx.x * blockDim.x + threadIdx.x;
    int rv[kLevelPer];
#pragma unroll
    for (int k = 0; k < kLevelPer; ++k) {
        const int x = xb + k * stride;
        rv[k] = x < n_v ? rdy[x] : kRdyNever;
    }
    const int flag = ctl->count[s % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->count[(s + 2) % 3] = 0;
        if (flag != 0) atomicMax(&ctl->levels, s + 1);
        if (st) {   // status for the host: this level's work flag, error bits, level index
            st[0] = flag;
            st[8] = ctl->err;
            st[9] = s;
        }
    }
    if (flag == 0) return;
    __shared__ int any_sh;
    if (threadIdx.x == 0) any_sh = 0;
    __syncthreads();
    bool any = false;
#pragma unroll
    for (int k = 0; k < kLevelPer; ++k) {
        if (rv[k] > s) continue;                    // not ready yet, waiting or finished
        const int x = xb + k * stride;
        // everything this vertex needs, its first child entries included, loaded together:
        // one memory round trip instead of a chain (partner, entry range, entries)
        const int q = partner[x];
        const float gx = g[x];
        const int cb = cptr[x], ce = cptr[x + 1];
        const int4 csx = cslot[x];
        const float4 wx = pa[x];
        const int4 pnx = pnode[x];
        const float4* sl = reinterpret_cast<const float4*>(contrib + (size_t)x * kChildSlots);
        const float4 s0 = sl[0], s1 = sl[1];
        static_assert(kChildSlots == 8, "two float4 slot loads");
        if (q < 0) {
            // entries in child order: the fixed slots (zero where unused), then the rest
            float l = gx;
            l += s0.x; l += s0.y; l += s0.z; l += s0.w;
            l += s1.x; l += s1.y; l += s1.z; l += s1.w;
            for (int k = cb + kChildSlots; k < ce; ++k) l += contrib[n_v * kChildSlots + k];
            lam[x] = l;
            done[x] = 1;
            rdy[x] = kRdyDone;
            publish_to(l, csx, wx, contrib);
            any |= release_from(pnx, -1, x, rem, rdy, s + 1);
            continue;
        }
        if (atomicSub(&pairrem[min(x, q)], 1) != 1) {   // partner not ready yet
            rdy[x] = kRdyWait;
            continue;
        }
        // x's own g, entry range and fixed slots come from the registers loaded above
        // (no child of x other than q finishes in this launch, and q's entry is
        // skipped); using them on this path too keeps the compiler from moving those
        // loads behind the partner test, which would add a round trip to every level
        float S[2], w[2];
        const int pr[2] = {x, q};
        for (int m = 0; m < 2; ++m) {
            const int a = pr[m], o = pr[1 - m];
            float l = m == 0 ? gx : g[a], wo = 0.f;
            const int b = m == 0 ? cb : cptr[a];
            const int e = m == 0 ? ce : cptr[a + 1];
            for (int k = b; k < e; ++k) {
                const int ch = cchild[k];
                if (ch == o) {
                    wo = calpha[k];
                } else {
                    const int r = k - b;
                    l += (m == 0 && r < kChildSlots) ? slot_of(s0, s1, r) : contrib[centry(a, r, k, n_v)];
                }
            }
            S[m] = l;
            w[m] = wo;     // weight of a in o's parent face
        }
        const float lx = (S[0] + w[0] * S[1]) / (1.f - w[0] * w[1]);
        const float lq = S[1] + w[1] * lx;
        lam[x] = lx;
        lam[q] = lq;
        done[x] = 1;
        done[q] = 1;
        rdy[x] = kRdyDone;
        rdy[q] = kRdyDone;
        publish_to(lx, csx, wx, contrib);
        publish(q, lq, pa, cslot, contrib);
        any |= release_from(pnx, q, x, rem, rdy, s + 1);
        any |= release_parents(q, x, pnode, rem, rdy, s + 1);
    }
    if (any) any_sh = 1;
    __syncthreads();
    if (threadIdx.x == 0 && any_sh) ctl->count[(s + 1) % 3] = 1;
}

__global__ void k_adj_remaining(const int* __restrict__ done, int n_v, int* __restrict__ list,
                                GbpCtl* ctl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_v && !done[i]) list[atomicAdd(&ctl->remaining, 1)] = i;
}

// Gauss-Seidel sweep (in place) over the vertices the level walk could not
// finish because of a cycle in the parent graph.  Every cycle leaks weight to
// parents outside it, so the sweeps contract to the unique solution.  Records
// the largest |change| and the largest |lambda| of the sweep (as float bits).
__global__ void k_adj_gs(const int* __restrict__ list, const int* __restrict__ cptr,
                         const int* __restrict__ cchild, const float* __restrict__ calpha,
                         const float* __restrict__ g, float* lam, GbpCtl* ctl, int slot) {
    // change of this sweep goes to slot (slot&1); the other slot is cleared for the next
    int* md = reinterpret_cast<int*>(slot & 1 ? &ctl->maxdiff2 : &ctl->maxdiff);
    int* md_next = reinterpret_cast<int*>(slot & 1 ? &ctl->maxdiff : &ctl->maxdiff2);
    if (blockIdx.x == 0 && threadIdx.x == 0) *md_next = 0;
    const int n_list = ctl->remaining;
    // a block with no listed vertex has nothing to add (in a budgeted backward most
    // sweeps find the list empty: they must cost a launch, not 2 contended atomics
    // per block)
    if ((int)(blockIdx.x * blockDim.x) >= n_list) return;
    float d = 0.f, a = 0.f;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_list; q += gridDim.x * blockDim.x) {
        const int i = list[q];
        float l = g[i];
        for (int x = cptr[i]; x < cptr[i + 1]; ++x) l += calpha[x] * lam[cchild[x]];
        d = fmaxf(d, fabsf(l - lam[i]));
        a = fmaxf(a, fabsf(l));
        lam[i] = l;
    }
    d = block_max_f(d);
    a = block_max_f(a);
    if (threadIdx.x == 0) {   // both are >= 0 and start at 0: a zero changes no maximum
        if (d > 0.f) atomicMax(md, __float_as_int(d));
        if (a > 0.f) atomicMax(&ctl->lmax_bits, __float_as_int(a));
    }
}

// Adjoint status after `sweeps` Gauss-Seidel sweeps: unsettled if the last
// sweep still moved lambda by more than 1e-6 of its largest magnitude.
__global__ void k_backward_end(GbpCtl* ctl, int sweeps) {
    if (threadIdx.x != 0 || ctl->remaining == 0) return;
    const float md = ((sweeps - 1) & 1) ? ctl->maxdiff2 : ctl->maxdiff;
    const float lmax = __int_as_float(ctl->lmax_bits);
    if (sweeps == 0 || !(md <= 1e-6f * lmax)) ctl->status |= 2;
}

// ------------------------------------------------------------------ gradients
__global__ void k_grad_tet(const int4* __restrict__ tetv, const float4* __restrict__ tetg,
                           const float4* __restrict__ xyz, const float* __restrict__ D,
                           const int* __restrict__ tet_user, const int* __restrict__ par,
                           const float4* __restrict__ pa, const float* __restrict__ lam,
                           int n_e, float* __restrict__ dD_user, float* __restrict__ dsbar) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_e) return;
    const int4 v = tetv[j];
    const int vv[4] = {v.x, v.y, v.z, v.w};
    // most elements are no vertex's parent element: those write zeros without
    // reading the tensor, the metric or their user id (unless dL/dD is wanted)
    int pk[4];
#pragma unroll
    for (int K = 0; K < 4; ++K) pk[K] = par[vv[K]];
    bool any = false;
#pragma unroll
    for (int K = 0; K < 4; ++K) any |= pk[K] == ((j << 2) | K);
    if (!any && !dD_user) {
        dsbar[j] = 0.f;
        return;
    }
    const float sbar = tetg[2 * (size_t)j + 1].z;
    const int u = tet_user[j];
    const float* d6 = D + 6 * (size_t)u;
    const float a = d6[0], b = d6[1], c = d6[2], d = d6[3], e = d6[4], f = d6[5];
    const float A00 = b * c - f * f, A11 = a * c - e * e, A22 = a * b - d * d;
    const float A01 = e * f - d * c, A02 = d * f - e * b, A12 = d * e - a * f;
    const float idet = 1.f / (a * A00 + d * A01 + e * A02);
    float g00 = 0, g11 = 0, g22 = 0, g01 = 0, g02 = 0, g12 = 0, gs = 0;
    for (int K = 0; K < 4; ++K) {
        const int i = vv[K];
        if (pk[K] != ((j << 2) | K)) continue;
        const float l = lam[i];
        if (l == 0.f) continue;
        int f3[3];
        face_nodes_rt(v, K, f3[0], f3[1], f3[2]);
        const float4 w = pa[i];
        const float al[3] = {w.x, w.y, w.z};
        const float4 xi = xyz[i];
        float ex = 0, ey = 0, ez = 0;
        for (int k = 0; k < 3; ++k) {
            const float4 xk = xyz[f3[k]];
            ex += al[k] * (xk.x - xi.x);
            ey += al[k] * (xk.y - xi.y);
            ez += al[k] * (xk.z - xi.z);
        }
        // u = D^{-1} e
        const float ux = (A00 * ex + A01 * ey + A02 * ez) * idet;
        const float uy = (A01 * ex + A11 * ey + A12 * ez) * idet;
        const float uz = (A02 * ex + A12 * ey + A22 * ez) * idet;
        const float h = sqrtf(fmaxf(ex * ux + ey * uy + ez * uz, 0.f)) / sbar;
        if (!(h > 0.f)) continue;
        const float cf = -l / (2.f * h * sbar * sbar);
        g00 += cf * ux * ux;
        g11 += cf * uy * uy;
        g22 += cf * uz * uz;
        g01 += cf * ux * uy;
        g02 += cf * ux * uz;
        g12 += cf * uy * uz;
        gs += l * (-h / sbar);
    }
    if (dD_user) {
        float* o = dD_user + 6 * (size_t)u;
        o[0] = g00;
        o[1] = g11;
        o[2] = g22;
        o[3] = 2.f * g01;
        o[4] = 2.f * g02;
        o[5] = 2.f * g12;
    }
    dsbar[j] = gs;
}

// dL/ds_n = 1/4 sum over the elements of n of dL/dsbar_j; L lanes per vertex (8: three
// passes over a 24-element patch), fixed reduction order.
template <int L>
__global__ void k_grad_node(const int2* __restrict__ nptr, const int* __restrict__ nent,
                            const float* __restrict__ dsbar, const int* __restrict__ node_user,
                            int n_v, float* __restrict__ dvs_user) {
    const int lane = threadIdx.x & (L - 1);
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) / L;
    if (i >= n_v) return;                           // uniform over the L-lane group
    const int2 p = nptr[i];
    const int tot = (p.y & 255) + ((p.y >> 8) & 255) + ((p.y >> 16) & 255) + ((p.y >> 24) & 255);
    // three entries per lane at a time (their loads in flight together), added in
    // entry order
    float s = 0.f;
    for (int c = lane; c < tot; c += 3 * L) {
        float v[3];
#pragma unroll
        for (int h = 0; h < 3; ++h) v[h] = dsbar[nent[p.x + (c + h * L < tot ? c + h * L : c)]];
#pragma unroll
        for (int h = 0; h < 3; ++h)
            if (c + h * L < tot) s += v[h];
    }
    for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) dvs_user[node_user[i]] = 0.25f * s;
}

__global__ void k_grad_root(const int* __restrict__ root_node, const float* __restrict__ root_t,
                            int n_roots, const int* __restrict__ node_int, int n_v,
                            const int* __restrict__ par, const float* __restrict__ troot,
                            const float* __restrict__ T, const float* __restrict__ lam,
                            float* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_roots) return;
    const int u = root_node[r];
    float val = 0.f;
    if (u >= 0 && u < n_v) {
        const int i = node_int[u];
        bool active = par[i] < 0 && T[i] < GBP_INF && root_t[r] == troot[i];
        for (int q = 0; q < r && active; ++q)
            if (root_node[q] == u && root_t[q] == root_t[r]) active = false;
        if (active) val = lam[i];
    }
    out[r] = val;
}

__global__ void k_parent_out(const int* __restrict__ par, const float4* __restrict__ pa,
                             const int4* __restrict__ tetv, const int* __restrict__ tet_user,
                             const int* __restrict__ node_user, const int* __restrict__ node_int,
                             int n_v, int* __restrict__ par_tet, int* __restrict__ par_node,
                             float* __restrict__ par_alpha, float* __restrict__ best) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_v) return;
    const int i = node_int[u];
    const int pr = par[i];
    const float4 w = pa[i];
    if (best) best[u] = w.w;
    if (pr < 0) {
        par_tet[u] = -1;
        for (int k = 0; k < 3; ++k) {
            par_node[3 * u + k] = -1;
            par_alpha[3 * u + k] = 0.f;
        }
        return;
    }
    int f[3];
    face_nodes_rt(tetv[pr >> 2], pr & 3, f[0], f[1], f[2]);
    par_tet[u] = tet_user[pr >> 2];
    const float al[3] = {w.x, w.y, w.z};
    for (int k = 0; k < 3; ++k) {
        par_node[3 * u + k] = node_user[f[k]];
        par_alpha[3 * u + k] = al[k];
    }
}

// ------------------------------------------------------------------ scan
__global__ void k_scan_block(const int* __restrict__ in, int* __restrict__ out, int n,
                             int* __restrict__ bsum) {
    __shared__ int sh[1024];
    const int base = blockIdx.x * 1024;
    int v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        const int idx = base + threadIdx.x * 4 + k;
        v[k] = idx < n ? in[idx] : 0;
        s += v[k];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int run = sh[threadIdx.x] - s;  // exclusive prefix of this thread
    for (int k = 0; k < 4; ++k) {
        const int idx = base + threadIdx.x * 4 + k;
        if (idx < n) out[idx] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) bsum[blockIdx.x] = sh[255];
}

// Exclusive scan of the block sums by one block of 1024 threads (chunks of 1024).
__global__ void __launch_bounds__(1024) k_scan_top(int* __restrict__ bsum, int nb,
                                                   int* __restrict__ total_out) {
    __shared__ int sh[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int idx = base + threadIdx.x;
        const int v = idx < nb ? bsum[idx] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (idx < nb) bsum[idx] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_add(int* __restrict__ out, int n, const int* __restrict__ bsum) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] += bsum[idx / 1024];
}

}  // namespace

int gbp_scan_exclusive(const int* in, int* out, int n, int* tmp, hipStream_t s) {
    const int nb = (n + 1023) / 1024;
    k_scan_block<<<nb, 256, 0, s>>>(in, out, n, tmp);
    k_scan_top<<<1, 1024, 0, s>>>(tmp, nb, out + n);
    k_scan_add<<<gbp_blocks(n, TPB), TPB, 0, s>>>(out, n, tmp);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

// ====================================================================== host
static int read_ctl(gbp_plan p, hipStream_t s) {
    GBP_HIP(hipMemcpyAsync(p->ctl_host, p->ctl, sizeof(GbpCtl), hipMemcpyDeviceToHost, s));
    GBP_HIP(hipStreamSynchronize(s));
    return GBP_OK;
}

// Pipelined convergence checks of the synchronous loops: the host waits for
// batch k's status only after batch k+1 is queued, so the device never idles on
// the check.  A finished loop costs at most one batch of empty launches (each
// returns at once).  The status comes from the first launch of the next batch
// (no copy in the stream); status_post, an asynchronous copy of the control block
// into pinned slot 1 or 2 with an event, serves when no launch is left.
static int status_post(gbp_plan p, int slot, hipStream_t s) {
    GBP_HIP(hipMemcpyAsync(p->ctl_host + 1 + slot, p->ctl, sizeof(GbpCtl), hipMemcpyDeviceToHost, s));
    GBP_HIP(hipEventRecord(p->ev[slot], s));
    return GBP_OK;
}

static int status_wait(gbp_plan p, int slot) {
    GBP_HIP(hipEventSynchronize(p->ev[slot]));
    return GBP_OK;
}

// Runs launch(k, st) for k = 0, 1, ... in growing batches until the status
// after a batch ending at k_end shows no work left, or `cap` launches.  The
// first launch of the next batch (launch k_end) writes that status into the
// pinned words st (the work it finds, the error bits, its index) and an event
// follows it; the host waits for that event while the rest of the batch is
// queued.  Only when no launch is left (cap) is the control block copied.
// fwd: the status counts are the 8 sub-queue lengths (forward), else one work
// flag (adjoint level).  Returns GBP_OK, or the device error bits' code;
// `launched` and `finished` out.
template <class Launch>
static int run_pipelined(gbp_plan p, hipStream_t s, int cap, bool fwd, Launch launch,
                         int& launched, bool& finished) {
    int r = 0, slot = 0, batch = 4, rc;
    finished = false;
    const int nb = std::min(batch, cap);
    for (int b = 0; b < nb; ++b, ++r) launch(r, nullptr);
    launched = r;
    GBP_LAUNCH_CHECK();
    while (true) {
        const int k_end = r;                      // status wanted: after k_end launches
        batch = std::min(batch * 2, p->sync_batch);
        const int nb2 = std::min(batch, cap - r);
        if (nb2 > 0) {
            launch(r, p->st_dev + slot * kStWords);
            GBP_HIP(hipEventRecord(p->ev[slot], s));
            ++r;
            for (int b = 1; b < nb2; ++b, ++r) launch(r, nullptr);
            launched = r;
            GBP_LAUNCH_CHECK();
        } else if ((rc = status_post(p, slot, s))) {
            return rc;
        }
        if ((rc = status_wait(p, slot))) return rc;
        int left = 0, err;
        if (nb2 > 0) {
            const volatile int* w = p->st_host + slot * kStWords;
            if (w[9] != k_end) {
                gbp_set_error("loop status out of order (launch %d reported, %d expected)", w[9], k_end);
                return GBP_ERR_HIP;
            }
            for (int x = 0; x < (fwd ? 8 : 1); ++x) left += w[x];
            err = w[8];
        } else {
            const GbpCtl& c = p->ctl_host[1 + slot];
            if (fwd)
                for (int x = 0; x < 8; ++x) left += c.qcnt[k_end % 3][x];
            else
                left = c.count[k_end % 3];
            err = c.err;
        }
        if (err) return gbp_err_from_bits(err);
        if (left == 0) {
            finished = true;
            return GBP_OK;
        }
        if (nb2 <= 0) return GBP_OK;              // cap reached
        slot ^= 1;
    }
}

int gbp_err_from_bits(int bits) {
    if (bits & ERRBIT_ROOT_RANGE) {
        gbp_set_error("root vertex id out of range");
        return GBP_ERR_ARG;
    }
    if (bits & ERRBIT_ROOT_NONFINITE) {
        gbp_set_error("non-finite root onset time");
        return GBP_ERR_NONFINITE;
    }
    if (bits & ERRBIT_D_NONFINITE) {
        gbp_set_error("non-finite velocity tensor entry");
        return GBP_ERR_NONFINITE;
    }
    if (bits & ERRBIT_D_NOT_SPD) {
        gbp_set_error("velocity tensor not positive definite");
        return GBP_ERR_NOT_SPD;
    }
    if (bits & ERRBIT_VSCALE) {
        gbp_set_error("velocity scale must be finite and > 0");
        return GBP_ERR_NONFINITE;
    }
    gbp_set_error("device error bits 0x%x", bits);
    return GBP_ERR_HIP;
}

static int check_roots(const float* D, const int32_t* root_node, const float* root_t, int n_roots) {
    if (!D) {
        gbp_set_error("D is NULL");
        return GBP_ERR_ARG;
    }
    if (n_roots < 0 || (n_roots > 0 && (!root_node || !root_t))) {
        gbp_set_error("bad roots (n_roots=%d)", n_roots);
        return GBP_ERR_ARG;
    }
    return GBP_OK;
}

// Control reset, metric, onsets and (cold == 1) +inf start with the roots' neighbours
// queued, (cold == 0) T from T_init.  G_init (cold == 1 only): the hold-back's
// ordering guess.  Enqueue only; no synchronisation.
static int prepare(gbp_plan p, const float* D, const float* vscale, const int32_t* root_node,
                   const float* root_t, int n_roots, int cold, const float* T_init,
                   hipStream_t s, const float* G_init = nullptr) {
    const int n_v = p->n_v, n_e = p->n_e;
    // A backward (cold == 2) may keep the element metric, scales and onsets of the
    // last full preparation when the caller allows it (gbp_plan_set_input_reuse)
    // and passes the same arrays; the control reset then keeps the error bits that
    // preparation raised.
    const bool keep = cold == 2 && p->reuse_inputs && p->prep_valid && p->prep_D == D &&
                      p->prep_vs == vscale && p->prep_rn == root_node && p->prep_rt == root_t &&
                      p->prep_nroots == n_roots;
    k_ctl_reset<<<1, 64, 0, s>>>(p->ctl, keep ? 2 : (cold == 2 ? 1 : 0));
    k_vertex_in<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(vscale, cold == 1 ? nullptr : T_init,
                                                     p->node_user, p->vs, p->troot, p->T, p->mark,
                                                     n_v, keep ? 1 : 0, p->ctl,
                                                     cold == 1 && p->hold_delta > 0.f ? p->hold
                                                                                      : nullptr,
                                                     G_init, p->guess);
    if (keep) {
        GBP_LAUNCH_CHECK();
        return GBP_OK;
    }
    {
        ProfScope ps(GBP_PROF_METRIC, s);
        k_metric<<<gbp_blocks(n_e, TPB), TPB, 0, s>>>(D, p->tet_user, p->tetv, p->xyz, p->vs,
                                                      p->tetg, n_e, p->ctl);
        if (p->solver == 1 && cold != 2)   // step constants of Alg. 1, per face
            k_fista_lip<<<gbp_blocks(4LL * n_e, TPB), TPB, 0, s>>>(p->tetg, n_e, p->fista_lmode,
                                                                   p->lip);
    }
    k_roots<<<std::max(1, gbp_blocks((long long)kRootLanes * n_roots, TPB)), TPB, 0, s>>>(
        root_node, root_t, n_roots, p->node_int, n_v, p->troot, p->T, cold == 1 ? 1 : 0, p->adj_ptr,
        p->adj, p->q[0], p->mark, p->ctl, p->xq);
    GBP_LAUNCH_CHECK();
    p->prep_valid = true;
    p->prep_D = D;
    p->prep_vs = vscale;
    p->prep_rn = root_node;
    p->prep_rt = root_t;
    p->prep_nroots = n_roots;
    return GBP_OK;
}

static void launch_round(gbp_plan p, bool cold, bool ordered, int r, hipStream_t s,
                         int* st = nullptr) {
    const int* qin = p->q[r & 1];
    int* qout = p->q[(r + 1) & 1];
    const int grid = std::min(p->sweep_blocks, kStatBlocks);
    ProfScope ps(GBP_PROF_FIM_SWEEP, s);
    const int open_below = p->hold_open > 0 ? p->hold_open : grid * (TPB / p->lanes) / 2;
    const HoldArgs ha{p->hold, p->blist, p->bcap, p->hold_delta > 0.f ? 1.f / p->hold_delta : 0.f,
                      open_below, p->hold_window, ordered ? p->guess : nullptr};
    const bool hold = cold && p->hold_delta > 0.f;
#define GBP_SWEEP(TS, LN, SV, HD)                                                                  \
    k_sweep<TS, LN, SV, HD><<<grid, TPB, 0, s>>>(p->nptr, p->nent, p->tetv, p->tetg, p->troot,    \
                                                 p->T, qin, qout, p->adj_ptr, p->adj, p->mark,    \
                                                 p->ctl, p->blk, r, p->eps_rel, p->n_v, p->xq,    \
                                                 p->lip, p->fista_iters, p->fista_tau, st, ha)
#define GBP_SWEEP_LANES(TS, SV, HD)                         \
    do {                                                    \
        if (p->lanes == 8) GBP_SWEEP(TS, 8, SV, HD);        \
        else if (p->lanes == 32) GBP_SWEEP(TS, 32, SV, HD); \
        else GBP_SWEEP(TS, 16, SV, HD);                     \
    } while (0)
    if (p->solver == 1) {
        if (hold) GBP_SWEEP_LANES(false, 1, true);
        else if (cold) GBP_SWEEP_LANES(false, 1, false);
        else GBP_SWEEP_LANES(true, 1, false);
    } else {
        if (hold) GBP_SWEEP_LANES(false, 0, true);
        else if (cold) GBP_SWEEP_LANES(false, 0, false);
        else GBP_SWEEP_LANES(true, 0, false);
    }
#undef GBP_SWEEP_LANES
#undef GBP_SWEEP
}

// Forward.  budget <= 0: synchronous, rounds until the queue empties (checked every
// sync_batch rounds).  budget > 0: exactly `budget` rounds, no host synchronisation
// (graph-capturable); empty rounds return at once and status bit 0 reports a queue
// left non-empty.
int gbp_forward_impl(gbp_plan p, const float* D, const float* vscale, const int32_t* root_node,
                     const float* root_t, int n_roots, const float* T_init, float* T_out,
                     gbp_stats* stats, hipStream_t s, int budget) {
    int rc = check_roots(D, root_node, root_t, n_roots);
    if (rc) return rc;
    const int n_v = p->n_v;
    // ordered warm start: T_init orders the hold-back of a cold solve
    const bool ordered = T_init && p->warm_order && p->hold_delta > 0.f;
    const bool cold = !T_init || p->warm_order;
    if ((rc = prepare(p, D, vscale, root_node, root_t, n_roots, cold ? 1 : 0, cold ? nullptr : T_init,
                      s, ordered ? T_init : nullptr)))
        return rc;
    k_zero_u64<<<gbp_blocks(2 * kStatBlocks, TPB), TPB, 0, s>>>(p->blk, 2 * kStatBlocks);
    if (!cold) {
        k_fill_int<<<gbp_blocks(p->n_comp, TPB), TPB, 0, s>>>(p->comp_root, 0, p->n_comp);
        k_comp_flag<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(p->troot, p->comp, n_v, p->comp_root);
        k_comp_clear<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(p->comp, p->comp_root, n_v, p->T);
        k_queue_all<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(p->q[0], p->mark, n_v, p->ctl, p->xq);
    }
    GBP_LAUNCH_CHECK();
    int r = 0;
    bool converged = true;
    if (budget > 0) {
        for (; r < budget; ++r) launch_round(p, cold, ordered, r, s);
    } else {
        rc = run_pipelined(
            p, s, p->max_rounds, true, [&](int k, int* st) { launch_round(p, cold, ordered, k, s, st); },
            r, converged);
        if (rc) {
            k_forward_end<<<1, 64, 0, s>>>(p->ctl, r);   // stamps used so far stay retired
            return rc;
        }
    }
    k_forward_end<<<1, 64, 0, s>>>(p->ctl, r);
    k_reduce_stats<<<1, TPB, 0, s>>>(p->blk, p->ctl);
    k_count_inf<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(p->T, n_v, p->ctl);
    k_scatter_out<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(p->T, p->node_int, T_out, n_v);
    GBP_LAUNCH_CHECK();
    if (budget > 0) return GBP_OK;
    if ((rc = read_ctl(p, s))) return rc;
    p->last_rounds = p->ctl_host->rounds;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->rounds = p->ctl_host->rounds;
        stats->converged = converged ? 1 : 0;
        stats->face_solves = (int64_t)p->ctl_host->solves;
        stats->node_updates = (int64_t)p->ctl_host->updates;
        stats->unreached = p->ctl_host->unreached;
    }
    if (!converged) {
        gbp_set_error("eikonal forward: no convergence after %d rounds", r);
        return GBP_ERR_NOT_CONVERGED;
    }
    return GBP_OK;
}

extern "C" int gbp_eikonal_forward(gbp_plan p, const float* D, const float* vscale,
                                   const int32_t* root_node, const float* root_t, int n_roots,
                                   const float* T_init, float* T_out, gbp_stats* stats,
                                   void* stream) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (!T_out) {
        gbp_set_error("T_out is NULL");
        return GBP_ERR_ARG;
    }
    return gbp_forward_impl(p, D, vscale, root_node, root_t, n_roots, T_init, T_out, stats,
                            (hipStream_t)stream, 0);
}

// parents at the converged T (internal order); T must already be in p->T
static int run_parents(gbp_plan p, const float* D_in, hipStream_t s) {
    const int n_v = p->n_v;
    ProfScope ps(GBP_PROF_PARENT, s);
    k_parent<kParLanes><<<gbp_blocks((long long)kParLanes * n_v, TPB), TPB, 0, s>>>(
        p->nptr, p->nent, p->tetv, p->tetg, p->tet_user, D_in, p->vs, p->xyz, p->T, p->troot, n_v,
        p->par, p->pa);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_parent_map(gbp_plan p, const float* D, const float* vscale,
                              const int32_t* root_node, const float* root_t, int n_roots,
                              const float* T, int32_t* par_tet, int32_t* par_node,
                              float* par_alpha, float* best, void* stream) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (!T || !par_tet || !par_node || !par_alpha) {
        gbp_set_error("NULL output or T");
        return GBP_ERR_ARG;
    }
    if ((rc = check_roots(D, root_node, root_t, n_roots))) return rc;
    if ((rc = gbp_alloc_backward(p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = prepare(p, D, vscale, root_node, root_t, n_roots, 2, T, s))) return rc;
    if ((rc = read_ctl(p, s))) return rc;
    if (p->ctl_host->err) return gbp_err_from_bits(p->ctl_host->err);
    if ((rc = run_parents(p, D, s))) return rc;
    k_parent_out<<<gbp_blocks(p->n_v, TPB), TPB, 0, s>>>(p->par, p->pa, p->tetv, p->tet_user,
                                                         p->node_user, p->node_int, p->n_v,
                                                         par_tet, par_node, par_alpha, best);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_backward_info(gbp_plan p, int* levels, int* cyclic, int* gs_sweeps) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (levels) *levels = p->bwd_levels;
    if (cyclic) *cyclic = p->bwd_cyclic;
    if (gs_sweeps) *gs_sweeps = p->bwd_gs_sweeps;
    return GBP_OK;
}

static void launch_level(gbp_plan p, int level, hipStream_t s, int* st = nullptr) {
    ProfScope ps(GBP_PROF_ADJ_LEVEL, s);
    const int need = gbp_blocks(p->n_v, TPB);
    const int grid = std::max(std::max(1, gbp_blocks(p->n_v, (long long)TPB * kLevelPer)),
                              std::min(need, p->level_blocks));
    k_adj_level<<<grid, TPB, 0, s>>>(
        p->rdy, p->ccnt, p->cchild, p->calpha, p->g, p->lam, p->done, p->pnode, p->pa, p->cslot,
        p->contrib, p->partner, p->pairrem, p->rem, p->n_v, p->ctl, level, st);
}

static void launch_gs(gbp_plan p, int it, hipStream_t s) {
    ProfScope ps(GBP_PROF_AUX, s);
    k_adj_gs<<<std::max(1, std::min(gbp_blocks(p->n_v, TPB), 1024)), TPB, 0, s>>>(
        p->cfill, p->ccnt, p->cchild, p->calpha, p->g, p->lam, p->ctl, it);
}

// Backward.  level_budget <= 0: synchronous (levels until the frontier empties,
// Gauss-Seidel on what cycles leave until settled).  level_budget > 0: exactly
// that many levels then gs_budget sweeps, no host synchronisation; status bit 1
// reports an unsettled remainder.
int gbp_backward_impl(gbp_plan p, const float* D, const float* vscale, const int32_t* root_node,
                      const float* root_t, int n_roots, const float* T, const float* dL_dT,
                      float* dL_dD, float* dL_dvscale, float* dL_droot_t, hipStream_t s,
                      int level_budget, int gs_budget) {
    int rc = check_roots(D, root_node, root_t, n_roots);
    if (rc) return rc;
    if ((rc = gbp_alloc_backward(p))) return rc;
    const int n_v = p->n_v, n_e = p->n_e;
    const bool sync = level_budget <= 0;
    if ((rc = prepare(p, D, vscale, root_node, root_t, n_roots, 2, T, s))) return rc;
    if ((rc = run_parents(p, D, s))) return rc;   // input errors surface at the first status read
    // parent lists, two-cycle partners, children lists
    {
        ProfScope ps_child(GBP_PROF_CHILD, s);
        const int nb = gbp_blocks(n_v, TPB);
        // p->done holds the child counts until the scan
        k_pnodes<<<nb, TPB, 0, s>>>(p->par, p->pa, p->tetv, n_v, p->pnode, p->done, p->cfill,
                                    p->cslot);
        k_partner<<<nb, TPB, 0, s>>>(p->pnode, n_v, p->partner);
        k_partner_sym<<<nb, TPB, 0, s>>>(p->partner, n_v, p->pairrem);
        k_partner_fix<<<nb, TPB, 0, s>>>(p->partner, p->pairrem, n_v);
        k_child_count<<<nb, TPB, 0, s>>>(p->pnode, n_v, p->done);
        GBP_LAUNCH_CHECK();
        if ((rc = gbp_scan_exclusive(p->done, p->ccnt, n_v, p->scan_tmp, s))) return rc;
        k_child_fill<<<nb, TPB, 0, s>>>(p->pnode, p->pa, n_v, p->ccnt, p->cfill, p->cchild,
                                        p->calpha);
        k_child_sort<<<nb, TPB, 0, s>>>(p->ccnt, p->cchild, p->calpha, n_v, p->cslot);
        GBP_LAUNCH_CHECK();
    }
    // leaves-first level walk
    k_ctl_reset<<<1, 64, 0, s>>>(p->ctl, 2);
    k_adj_init<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(dL_dT, p->node_user, p->T, p->ccnt, p->partner,
                                                    p->rem, n_v, p->g, p->lam, p->done, p->rdy,
                                                    p->contrib, p->ctl);
    GBP_LAUNCH_CHECK();
    int level = 0;
    if (!sync) {
        for (; level < level_budget; ++level) launch_level(p, level, s);
    } else {
        bool empty = false;
        rc = run_pipelined(
            p, s, p->max_rounds + n_v, false, [&](int k, int* st) { launch_level(p, k, s, st); },
            level, empty);
        if (rc) return rc;
    }
    // vertices on or above cycles longer than two: Gauss-Seidel on the remainder
    k_adj_remaining<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(p->done, n_v, p->cfill, p->ctl);
    GBP_LAUNCH_CHECK();
    int it = 0;
    if (!sync) {
        for (; it < gs_budget; ++it) launch_gs(p, it, s);
        k_backward_end<<<1, 64, 0, s>>>(p->ctl, it);
    } else {
        if ((rc = read_ctl(p, s))) return rc;
        p->bwd_levels = p->ctl_host->levels;
        p->last_levels = p->ctl_host->levels;
        p->bwd_cyclic = p->ctl_host->remaining;
        if (p->ctl_host->remaining > 0) {
            bool ok = false;
            const int cap = 4 * p->max_rounds + 1000;
            while (!ok && it < cap) {
                for (int b = 0; b < 16; ++b, ++it) launch_gs(p, it, s);
                GBP_LAUNCH_CHECK();
                if ((rc = read_ctl(p, s))) return rc;
                const float lmax = __builtin_bit_cast(float, p->ctl_host->lmax_bits);
                const float md = ((it - 1) & 1) ? p->ctl_host->maxdiff2 : p->ctl_host->maxdiff;
                ok = md <= 1e-6f * lmax;
            }
            if (!ok) {
                gbp_set_error("adjoint did not settle on %d vertices left by parent-graph cycles",
                              p->bwd_cyclic);
                return GBP_ERR_NOT_CONVERGED;
            }
        }
        p->bwd_gs_sweeps = it;
    }
    // gradients
    ProfScope ps_grad(GBP_PROF_GRAD, s);
    k_grad_tet<<<gbp_blocks(n_e, TPB), TPB, 0, s>>>(p->tetv, p->tetg, p->xyz, D, p->tet_user,
                                                    p->par, p->pa, p->lam, n_e, dL_dD, p->dsbar);
    if (dL_dvscale)
        k_grad_node<8><<<gbp_blocks(8LL * n_v, TPB), TPB, 0, s>>>(p->nptr, p->nent, p->dsbar,
                                                                  p->node_user, n_v, dL_dvscale);
    if (dL_droot_t && n_roots > 0)
        k_grad_root<<<gbp_blocks(n_roots, TPB), TPB, 0, s>>>(root_node, root_t, n_roots,
                                                             p->node_int, n_v, p->par, p->troot,
                                                             p->T, p->lam, dL_droot_t);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_eikonal_backward(gbp_plan p, const float* D, const float* vscale,
                                    const int32_t* root_node, const float* root_t, int n_roots,
                                    const float* T, const float* dL_dT, float* dL_dD,
                                    float* dL_dvscale, float* dL_droot_t, void* stream) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (!T || !dL_dT) {
        gbp_set_error("T and dL_dT are required");
        return GBP_ERR_ARG;
    }
    return gbp_backward_impl(p, D, vscale, root_node, root_t, n_roots, T, dL_dT, dL_dD, dL_dvscale,
                             dL_droot_t, (hipStream_t)stream, 0, 0);
}

extern "C" int gbp_eikonal_forward_async(gbp_plan p, const float* D, const float* vscale,
                                         const int32_t* root_node, const float* root_t,
                                         int n_roots, const float* T_init, float* T_out,
                                         int round_budget, void* stream) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (!T_out || round_budget < 1) {
        gbp_set_error("forward_async: T_out is required and round_budget >= 1 (%d)", round_budget);
        return GBP_ERR_ARG;
    }
    return gbp_forward_impl(p, D, vscale, root_node, root_t, n_roots, T_init, T_out, nullptr,
                            (hipStream_t)stream, round_budget);
}

extern "C" int gbp_eikonal_backward_async(gbp_plan p, const float* D, const float* vscale,
                                          const int32_t* root_node, const float* root_t,
                                          int n_roots, const float* T, const float* dL_dT,
                                          float* dL_dD, float* dL_dvscale, float* dL_droot_t,
                                          int level_budget, int gs_budget, void* stream) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (!T || !dL_dT || level_budget < 1 || gs_budget < 0) {
        gbp_set_error("backward_async: T and dL_dT are required, level_budget >= 1, gs_budget >= 0");
        return GBP_ERR_ARG;
    }
    return gbp_backward_impl(p, D, vscale, root_node, root_t, n_roots, T, dL_dT, dL_dD, dL_dvscale,
                             dL_droot_t, (hipStream_t)stream, level_budget, gs_budget);
}

extern "C" int gbp_plan_forward_work(gbp_plan p, int64_t* face_solves, int64_t* node_updates,
                                     void* stream) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    std::vector<unsigned long long> b(2 * (size_t)kStatBlocks);
    hipStream_t s = (hipStream_t)stream;
    GBP_HIP(hipMemcpyAsync(b.data(), p->blk, b.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    GBP_HIP(hipStreamSynchronize(s));
    unsigned long long a = 0, u = 0;
    for (int i = 0; i < kStatBlocks; ++i) {
        a += b[2 * i];
        u += b[2 * i + 1];
    }
    if (face_solves) *face_solves = (int64_t)a;
    if (node_updates) *node_updates = (int64_t)u;
    return GBP_OK;
}

extern "C" int gbp_plan_status(gbp_plan p, int* err_code, int* forward_converged,
                               int* backward_settled, int* rounds, int* levels, void* stream) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if ((rc = read_ctl(p, (hipStream_t)stream))) return rc;
    const GbpCtl& c = *p->ctl_host;
    if (err_code) *err_code = c.err ? gbp_err_from_bits(c.err) : GBP_OK;
    if (forward_converged) *forward_converged = (c.status & 1) ? 0 : 1;
    if (backward_settled) *backward_settled = (c.status & 2) ? 0 : 1;
    if (rounds) *rounds = c.rounds;
    if (levels) *levels = c.levels;
    return GBP_OK;
}
