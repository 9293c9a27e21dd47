// Geodesic-BP on triangle meshes (d = 2), the setting of the paper's 2-D study
// (Sec. 3.1): the same three steps as on tetrahedra with a segment as the local
// simplex.
//
// * forward: Alg. 2 as an active queue of vertices, a group of lanes per queued
//   vertex evaluating the local problems of its triangles (Sec. 2.2 Eq. (upwind_eq_lsqr)
//   with d = 2: two vertex candidates and one interior candidate, predicated);
// * backward: geodesic parents in FP64 (the argmin is a decision taken by
//   floating point: same precision as the reference), the adjoint
//   lambda = g + P^T lambda (Sec. 2.3 Eq. (dto_grad)) as a leaves-first walk
//   over device-built child lists in a fixed order (a vertex finished once all
//   its children are, two-cycles solved as pairs; the whole walk in one
//   work-group, since these parent graphs are deep and narrow), Gauss-Seidel
//   sweeps over just the vertices that longer cycles leave unfinished (geometric
//   convergence there), and the gradients w.r.t. the triangle tensors, nodal
//   velocity scales and root onsets.
//
// Meshes of the 2-D study are small (thousands of vertices); the kernels keep
// the tetrahedral path's structure (queue, level walk, block-aggregated
// counters) without its XCD and LDS-gather refinements.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "gbp_internal.h"
#include "local_solve.h"

struct TriCtl {
    int count[3];
    int err;
    unsigned long long solves, updates;
    int unreached;
    int diff_bits[2];    // adjoint sweeps: largest |change| (float bits), by parity
    int lmax_bits[2];    // ... and largest |lambda|
    int levels;          // adjoint: last level with work + 1
    int remaining;       // adjoint: reached vertices the level walk has not finished
    int nlist;           // adjoint: length of the list of those vertices
    int rounds;          // forward: last round with work + 1
};

struct gbp_tri_plan_s {
    int device = 0;
    int n_v = 0, n_t = 0;
    float2* xy = nullptr;
    int4* tri = nullptr;          // vertex ids (w unused)
    int* vptr = nullptr;          // [n_v+1] incidence: entries (tri << 2 | slot) sorted by tri
    int* vent = nullptr;
    int* nbp = nullptr;           // [n_v+1] unique neighbours
    int* nb = nullptr;
    float4* minv = nullptr;       // [n_t] D_eff^-1 (xx, yy, xy) and sbar
    float* T = nullptr;
    float* troot = nullptr;
    int* q[2] = {nullptr, nullptr};
    int* mark = nullptr;
    TriCtl* ctl = nullptr;
    TriCtl* ctl_host = nullptr;
    TriCtl* ctl_pipe = nullptr;   // pinned [2]: control block after each batch of rounds
    hipEvent_t ev[2] = {nullptr, nullptr};
    int* par = nullptr;
    int2* pnode = nullptr;
    float4* pa = nullptr;         // alpha_a, alpha_b, best, root_self
    int* ccnt = nullptr;          // [n_v+1]
    int* cfill = nullptr;         // child fill cursors, then the level walk's remaining-children counts
    int* rdy = nullptr;           // [n_v] adjoint walk: finished flags
    int* partner = nullptr;       // [n_v] two-cycle partner or -1
    int* pairrem = nullptr;       // [n_v] members of a two-cycle not yet ready (at the smaller one)
    int* cchild = nullptr;        // [2 n_v]
    float* calpha = nullptr;
    float* lam[2] = {nullptr, nullptr};
    float* g = nullptr;
    float* dsbar = nullptr;
    int* scan_tmp = nullptr;
    int stamp = 1;
    int last_levels = 0, last_cyclic = 0, last_sweeps = 0;   // of the last backward
    int max_rounds = 20000;
    float eps_rel = 1.0f / (1 << 20);
};

namespace {

constexpr int TPB = 256;

template <typename T>
int tri_alloc(T** p, size_t n) {
    if (n == 0) n = 1;
    if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) {
        gbp_set_error("hipMalloc of %zu bytes failed", n * sizeof(T));
        return GBP_ERR_NOMEM;
    }
    return GBP_OK;
}

void tri_free(gbp_tri_plan p) {
    if (!p) return;
    void* ptrs[] = {p->xy,    p->tri,   p->vptr,   p->vent,   p->nbp,    p->nb,     p->minv,
                    p->T,     p->troot, p->q[0],   p->q[1],   p->mark,   p->ctl,    p->par,
                    p->pnode, p->pa,    p->ccnt,   p->cfill,  p->cchild, p->calpha, p->lam[0],
                    p->lam[1], p->g,    p->dsbar,  p->scan_tmp, p->rdy, p->partner, p->pairrem};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (p->ctl_host) (void)hipHostFree(p->ctl_host);
    if (p->ctl_pipe) (void)hipHostFree(p->ctl_pipe);
    for (hipEvent_t e : p->ev)
        if (e) (void)hipEventDestroy(e);
    delete p;
}

__device__ __forceinline__ bool fin(float x) { return x - x == 0.f; }

// block reductions (one atomic per block instead of one per thread)
__device__ __forceinline__ unsigned long long tri_block_sum(unsigned long long v) {
    __shared__ unsigned long long part[TPB / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long t = 0;
    for (int w = 0; w < TPB / 64; ++w) t += part[w];
    return t;
}

__device__ __forceinline__ float tri_block_max(float v) {
    __shared__ float part[TPB / 64];
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    float t = 0.f;
    for (int w = 0; w < TPB / 64; ++w) t = fmaxf(t, part[w]);
    return t;
}

// face (a, b) of the triangle seen from its local vertex k: the other two
// vertices in increasing local order
__device__ __forceinline__ void tri_face(int4 t, int k, int& i, int& a, int& b) {
    i = k == 0 ? t.x : k == 1 ? t.y : t.z;
    a = k == 0 ? t.y : t.x;
    b = k == 2 ? t.y : t.z;
}

// d = 2 local solve in precision R: vertex a, vertex b, interior (first wins on
// ties); unreached vertices leave the other vertex's candidate.
template <typename R>
__device__ __forceinline__ R tri_local(R qaa, R qbb, R qab, R pa, R pb, R* alpha_a = nullptr) {
    const R INF = gbp_inf<R>();
    const bool fa = pa < INF, fb = pb < INF;
    R best = fa ? pa + gbp_sqrt(qaa) : INF;
    R al = fa ? R(1) : R(0);
    const R vb = fb ? pb + gbp_sqrt(qbb) : INF;
    if (vb < best) { best = vb; al = R(0); }
    if (fa && fb) {
        const R m = fmin(pa, pb);
        R v, ua, ub;
        edge_candidate<R>(qaa, qbb, qab, pa - m, pb - m, true, v, ua, ub);
        if (m + v < best) { best = m + v; al = ua / (ua + ub); }
    }
    if (alpha_a) *alpha_a = al;
    return best;
}

__global__ void k_tri_metric(const float* __restrict__ D, const float* __restrict__ vscale,
                             const int4* __restrict__ tri, int n_t, float4* __restrict__ minv,
                             TriCtl* ctl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_t) return;
    const int4 v = tri[t];
    float sbar = 1.f;
    if (vscale) {
        const float s0 = vscale[v.x], s1 = vscale[v.y], s2 = vscale[v.z];
        if (!(s0 > 0.f && s1 > 0.f && s2 > 0.f && fin(s0) && fin(s1) && fin(s2)))
            atomicOr(&ctl->err, ERRBIT_VSCALE);
        sbar = (s0 + s1 + s2) * (1.f / 3.f);
    }
    const float xx = D[3 * (size_t)t], yy = D[3 * (size_t)t + 1], xy = D[3 * (size_t)t + 2];
    const float det = xx * yy - xy * xy;
    if (!(fin(xx) && fin(yy) && fin(xy))) atomicOr(&ctl->err, ERRBIT_D_NONFINITE);
    else if (!(xx > 0.f && det > 0.f)) atomicOr(&ctl->err, ERRBIT_D_NOT_SPD);
    const float s = 1.f / (det * sbar * sbar);
    minv[t] = make_float4(yy * s, xx * s, -xy * s, sbar);
}

__global__ void k_tri_roots(const int* __restrict__ root_node, const float* __restrict__ root_t,
                            int n_roots, int n_v, float* __restrict__ troot, float* __restrict__ T,
                            int cold, const int* __restrict__ nbp, const int* __restrict__ nb,
                            int* __restrict__ q0, int* __restrict__ mark, int stamp, TriCtl* ctl) {
    if (threadIdx.x == 0) {
        for (int r = 0; r < n_roots; ++r) {
            const int u = root_node[r];
            const float t = root_t[r];
            if (u < 0 || u >= n_v) { atomicOr(&ctl->err, ERRBIT_ROOT_RANGE); continue; }
            if (!fin(t)) { atomicOr(&ctl->err, ERRBIT_ROOT_NONFINITE); continue; }
            troot[u] = fminf(troot[u], t);
            if (cold) T[u] = fminf(T[u], t);
        }
    }
    __syncthreads();
    if (!cold) return;
    for (int r = threadIdx.x; r < n_roots; r += blockDim.x) {
        const int u = root_node[r];
        if (u < 0 || u >= n_v) continue;
        for (int a = nbp[u]; a < nbp[u + 1]; ++a) {
            const int w = nb[a];
            if (atomicMax(&mark[w], stamp) < stamp) q0[atomicAdd(&ctl->count[0], 1)] = w;
        }
    }
}

// Lanes per queued vertex in a relaxation round: the lanes of a group take the
// vertex's triangles (and then its neighbours) in turn, so a round's chain of
// dependent loads is one triangle's, not the sum over the vertex's triangles.
// Narrow fronts (at most kNarrowFront queued vertices) take 8 lanes per vertex,
// wider ones 4: the round is latency-bound when the front is narrow and bound by
// the waves it issues when it is wide.
constexpr int kNarrowFront = 1024;

template <int L>
__device__ __forceinline__ void tri_relax(const float2* __restrict__ xy, const int4* __restrict__ tri,
                                          const float4* __restrict__ minv, const int* __restrict__ vptr,
                                          const int* __restrict__ vent, const int* __restrict__ nbp,
                                          const int* __restrict__ nb, float* T, const int* __restrict__ qin,
                                          int n, int* __restrict__ qout, int* __restrict__ mark,
                                          int* cnt_next, int stamp_next, float eps_rel, int* pbuf,
                                          int* pn, int cap, unsigned long long& solves,
                                          unsigned long long& upd) {
    const int lane = threadIdx.x & (L - 1);
    // k is the same in every lane of a group, so a group runs its passes together
    for (int k = (blockIdx.x * TPB + threadIdx.x) / L; k < n; k += gridDim.x * (TPB / L)) {
        const int i = qin[k];
        const float told = T[i];
        float best = told;
        const float2 xi = xy[i];
        for (int e = vptr[i] + lane; e < vptr[i + 1]; e += L) {
            const int code = vent[e];
            const int t = code >> 2;
            int ii, a, b;
            tri_face(tri[t], code & 3, ii, a, b);
            const float4 m = minv[t];
            const float2 xa = xy[a], xb = xy[b];
            const float ax = xa.x - xi.x, ay = xa.y - xi.y, bx = xb.x - xi.x, by = xb.y - xi.y;
            const float qaa = ax * (m.x * ax + m.z * ay) + ay * (m.z * ax + m.y * ay);
            const float qbb = bx * (m.x * bx + m.z * by) + by * (m.z * bx + m.y * by);
            const float qab = ax * (m.x * bx + m.z * by) + ay * (m.z * bx + m.y * by);
            best = fminf(best, tri_local<float>(qaa, qbb, qab, T[a], T[b]));
            ++solves;
        }
#pragma unroll
        for (int o = 1; o < L; o <<= 1) best = fminf(best, __shfl_xor(best, o));
        const bool changed = (told < GBP_INF) ? (best < told - eps_rel * fmaxf(1.f, fabsf(told)))
                                              : (best < GBP_INF);
        if (lane == 0 && best < told) T[i] = best;
        if (changed) {
            if (lane == 0) ++upd;
            for (int a = nbp[i] + lane; a < nbp[i + 1]; a += L) {
                const int w = nb[a];
                if (atomicMax(&mark[w], stamp_next) < stamp_next) {
                    const int pos = atomicAdd(pn, 1);
                    if (pos < cap) pbuf[pos] = w;
                    else qout[atomicAdd(cnt_next, 1)] = w;     // buffer full: straight to the queue
                }
            }
        }
    }
}

// one relaxation round over the queue qin; the grid covers kNarrowFront vertices
// at 8 lanes each or the mesh, whichever is less
__global__ void __launch_bounds__(TPB)
    k_tri_sweep(const float2* __restrict__ xy, const int4* __restrict__ tri,
                const float4* __restrict__ minv, const int* __restrict__ vptr,
                const int* __restrict__ vent, const int* __restrict__ nbp,
                const int* __restrict__ nb, float* T, const int* __restrict__ qin,
                int* __restrict__ qout, int* __restrict__ mark, TriCtl* ctl, int s, int stamp_next,
                float eps_rel) {
    const int n = ctl->count[s % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->count[(s + 2) % 3] = 0;
        if (n > 0) atomicMax(&ctl->rounds, s + 1);
    }
    const bool narrow = n <= kNarrowFront;
    if ((int)(blockIdx.x * (narrow ? TPB / 8 : TPB / 4)) >= n) return;   // uniform over the block
    // pushes collect in LDS; one atomic per block reserves their room in the queue
    constexpr int kCap = 4096;
    __shared__ int pbuf[kCap];
    __shared__ int pn, pbase;
    int* cnt_next = &ctl->count[(s + 1) % 3];
    if (threadIdx.x == 0) pn = 0;
    __syncthreads();
    unsigned long long solves = 0, upd = 0;
    if (narrow)
        tri_relax<8>(xy, tri, minv, vptr, vent, nbp, nb, T, qin, n, qout, mark, cnt_next, stamp_next, eps_rel,
                     pbuf, &pn, kCap, solves, upd);
    else
        tri_relax<4>(xy, tri, minv, vptr, vent, nbp, nb, T, qin, n, qout, mark, cnt_next, stamp_next, eps_rel,
                     pbuf, &pn, kCap, solves, upd);
    __syncthreads();
    const int m = min(pn, kCap);
    if (threadIdx.x == 0) pbase = m > 0 ? atomicAdd(cnt_next, m) : 0;
    __syncthreads();
    for (int k = threadIdx.x; k < m; k += blockDim.x) qout[pbase + k] = pbuf[k];
    solves = tri_block_sum(solves);
    upd = tri_block_sum(upd);
    if (threadIdx.x == 0) {
        if (solves) atomicAdd(&ctl->solves, solves);
        if (upd) atomicAdd(&ctl->updates, upd);
    }
}

__global__ void k_tri_ctl_reset(TriCtl* ctl) {
    if (threadIdx.x == 0) *ctl = TriCtl{};
}

__global__ void k_tri_fill(float* __restrict__ x, float v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void k_tri_fill_i(int* __restrict__ x, int v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void k_tri_count_inf(const float* __restrict__ T, int n_v, TriCtl* ctl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_v && !(T[i] < GBP_INF)) atomicAdd(&ctl->unreached, 1);
}

// FP64 geodesic parent of every vertex: lowest triangle among local values
// within 1e-12 max(1, |T|) of the minimum; a vertex whose smallest onset does
// not exceed that minimum is a root (its own parent).
__global__ void k_tri_parent(const float2* __restrict__ xy, const int4* __restrict__ tri,
                             const float* __restrict__ D, const float* __restrict__ vscale,
                             const int* __restrict__ vptr, const int* __restrict__ vent,
                             const float* __restrict__ T, const float* __restrict__ troot, int n_v,
                             int* __restrict__ par, int2* __restrict__ pnode,
                             float4* __restrict__ pa) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_v) return;
    par[i] = -1;
    pnode[i] = make_int2(-1, -1);
    pa[i] = make_float4(0.f, 0.f, GBP_INF, 0.f);
    const double Ti = T[i];
    if (!(T[i] < GBP_INF)) return;
    const double xi = xy[i].x, yi = xy[i].y;
    double best = gbp_inf<double>();
    for (int pass = 0; pass < 2; ++pass) {
        const double tol = 1e-12 * fmax(1.0, fabs(Ti));
        for (int e = vptr[i]; e < vptr[i + 1]; ++e) {
            const int code = vent[e];
            const int t = code >> 2;
            const int4 tv = tri[t];
            int ii, a, b;
            tri_face(tv, code & 3, ii, a, b);
            double sbar = 1.0;
            if (vscale) sbar = ((double)vscale[tv.x] + vscale[tv.y] + vscale[tv.z]) / 3.0;
            const double dxx = D[3 * (size_t)t], dyy = D[3 * (size_t)t + 1], dxy = D[3 * (size_t)t + 2];
            const double s = 1.0 / ((dxx * dyy - dxy * dxy) * sbar * sbar);
            const double mxx = dyy * s, myy = dxx * s, mxy = -dxy * s;
            const double ax = xy[a].x - xi, ay = xy[a].y - yi, bx = xy[b].x - xi, by = xy[b].y - yi;
            const double qaa = ax * (mxx * ax + mxy * ay) + ay * (mxy * ax + myy * ay);
            const double qbb = bx * (mxx * bx + mxy * by) + by * (mxy * bx + myy * by);
            const double qab = ax * (mxx * bx + mxy * by) + ay * (mxy * bx + myy * by);
            const double ta = T[a] < GBP_INF ? (double)T[a] : gbp_inf<double>();
            const double tb = T[b] < GBP_INF ? (double)T[b] : gbp_inf<double>();
            double al;
            const double v = tri_local<double>(qaa, qbb, qab, ta, tb, &al);
            if (pass == 0) {
                best = fmin(best, v);
            } else if (v <= best + tol && v < gbp_inf<double>()) {
                if (troot[i] < GBP_INF && (double)troot[i] <= best) {   // a root: its own parent
                    pa[i] = make_float4(0.f, 0.f, (float)best, 1.f);
                } else {
                    par[i] = t;
                    pnode[i] = make_int2(a, b);
                    pa[i] = make_float4((float)al, (float)(1.0 - al), (float)best, 0.f);
                }
                return;
            }
        }
        if (pass == 0 && !(best < gbp_inf<double>())) break;
    }
    if (troot[i] < GBP_INF) pa[i] = make_float4(0.f, 0.f, (float)best, 1.f);   // root
}

__global__ void k_tri_child_count(const int* __restrict__ par, const int2* __restrict__ pnode,
                                  const float4* __restrict__ pa, int n_v, int* __restrict__ cnt) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_v || par[c] < 0) return;
    const int2 p = pnode[c];
    const float4 w = pa[c];
    if (w.x > 0.f) atomicAdd(&cnt[p.x], 1);
    if (w.y > 0.f) atomicAdd(&cnt[p.y], 1);
}

__global__ void k_tri_child_fill(const int* __restrict__ par, const int2* __restrict__ pnode,
                                 const float4* __restrict__ pa, int n_v, const int* __restrict__ cptr,
                                 int* __restrict__ cfill, int* __restrict__ cchild,
                                 float* __restrict__ calpha) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_v || par[c] < 0) return;
    const int2 p = pnode[c];
    const float4 w = pa[c];
    if (w.x > 0.f) {
        const int k = cptr[p.x] + atomicAdd(&cfill[p.x], 1);
        cchild[k] = c;
        calpha[k] = w.x;
    }
    if (w.y > 0.f) {
        const int k = cptr[p.y] + atomicAdd(&cfill[p.y], 1);
        cchild[k] = c;
        calpha[k] = w.y;
    }
}

// child lists sorted by child id: a fixed summation order (deterministic)
__global__ void k_tri_child_sort(const int* __restrict__ cptr, int* __restrict__ cchild,
                                 float* __restrict__ calpha, int n_v) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_v) return;
    const int b = cptr[p], e = cptr[p + 1];
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
}

__global__ void k_tri_adj_init(const float* __restrict__ dLdT, const float* __restrict__ T, int n_v,
                               float* __restrict__ g, float* __restrict__ lam) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_v) return;
    float v = T[i] < GBP_INF ? dLdT[i] : 0.f;
    if (v != v) v = 0.f;
    g[i] = v;
    lam[i] = v;
}

// Gauss-Seidel sweep (in place) over the vertices the level walk left unfinished
// (on or above parent-graph cycles; every cycle leaks weight to parents outside
// it, so the sweeps contract); records the largest |change| and |lambda|.
__global__ void k_tri_adj_gs(const int* __restrict__ list, const int* __restrict__ cptr,
                             const int* __restrict__ cchild, const float* __restrict__ calpha,
                             const float* __restrict__ g, float* lam, TriCtl* ctl, int it) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->diff_bits[(it + 1) & 1] = 0;
        ctl->lmax_bits[(it + 1) & 1] = 0;
    }
    const int n = ctl->nlist;
    float d = 0.f, a = 0.f;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const int i = list[q];
        float l = g[i];
        for (int k = cptr[i]; k < cptr[i + 1]; ++k) l += calpha[k] * lam[cchild[k]];
        d = fmaxf(d, fabsf(l - lam[i]));
        a = fmaxf(a, fabsf(l));
        lam[i] = l;
    }
    d = tri_block_max(d);
    a = tri_block_max(a);
    if (threadIdx.x == 0) {
        if (d > 0.f) atomicMax(&ctl->diff_bits[it & 1], __float_as_int(d));
        if (a > 0.f) atomicMax(&ctl->lmax_bits[it & 1], __float_as_int(a));
    }
}

// Two-cycles of the parent graph: a and c are partners when each is a weighted
// parent of the other (the anisotropic scheme is not causal).  The walk leaves the
// mutual edge out of both readiness counts and solves the pair jointly once both
// members' other children are finished.  A vertex picks its smallest mutual
// parent; a pair is kept only if both picked each other (pairrem: 2 at the
// smaller member, -1 at the larger until k_tri_partner_fix, 0 elsewhere).
__device__ __forceinline__ bool tri_weighted_parent(int2 pn, float4 w, int x) {
    return (pn.x == x && w.x > 0.f) || (pn.y == x && w.y > 0.f);
}

__global__ void k_tri_partner(const int* __restrict__ par, const int2* __restrict__ pnode,
                              const float4* __restrict__ pa, int n_v, int* __restrict__ partner) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_v) return;
    int best = -1;
    if (par[a] >= 0) {
        const int2 pn = pnode[a];
        const float4 w = pa[a];
        const int cand[2] = {w.x > 0.f ? pn.x : -1, w.y > 0.f ? pn.y : -1};
        for (int k = 0; k < 2; ++k) {
            const int c = cand[k];
            if (c >= 0 && par[c] >= 0 && tri_weighted_parent(pnode[c], pa[c], a) && (best < 0 || c < best))
                best = c;
        }
    }
    partner[a] = best;
}

__global__ void k_tri_partner_sym(const int* __restrict__ partner, int n_v, int* __restrict__ pairrem) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_v) return;
    const int c = partner[a];
    const bool ok = c >= 0 && partner[c] == a;
    pairrem[a] = ok ? (a < c ? 2 : -1) : 0;
}

__global__ void k_tri_partner_fix(int* __restrict__ partner, int* __restrict__ pairrem, int n_v) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_v) return;
    const int r = pairrem[a];
    if (r == 0) partner[a] = -1;
    if (r < 0) pairrem[a] = 0;
}

// rem: the children a vertex waits for (its sorted CSR range but its partner);
// done: 1 for unreached vertices; ctl->remaining: the reached vertices (the walk
// subtracts those it finishes)
__global__ void k_tri_walk_init(const int* __restrict__ cptr, const int* __restrict__ partner,
                                const float* __restrict__ T, int n_v, int* __restrict__ rem,
                                int* __restrict__ done, TriCtl* ctl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool reached = false;
    if (i < n_v) {
        rem[i] = cptr[i + 1] - cptr[i] - (partner[i] >= 0 ? 1 : 0);
        reached = T[i] < GBP_INF;
        done[i] = reached ? 0 : 1;
    }
    const unsigned long long r = tri_block_sum(reached ? 1ull : 0ull);
    if (threadIdx.x == 0 && r) atomicAdd(&ctl->remaining, (int)r);
}

constexpr int kWalkThreads = 1024;

// A finished vertex releases its weighted parents (but `skip`); a parent whose
// last awaited child this was joins the next frontier.
__device__ __forceinline__ void tri_release(int px, int2 pn, float4 w, int skip, int self,
                                            int* __restrict__ rem, int* __restrict__ next, int* n_next) {
    if (px < 0) return;
    // both releases in flight together, with no branch between them: a parent that
    // is not released takes 0 off the finished vertex's own count instead (no
    // longer read by anyone), and its result is ignored
    const bool va = w.x > 0.f && pn.x != skip, vb = w.y > 0.f && pn.y != skip;
    const int ra = atomicSub(&rem[va ? pn.x : self], va ? 1 : 0);
    const int rb = atomicSub(&rem[vb ? pn.y : self], vb ? 1 : 0);
    if (va && ra == 1) next[atomicAdd(n_next, 1)] = pn.x;
    if (vb && rb == 1) next[atomicAdd(n_next, 1)] = pn.y;
}

// The whole leaves-first walk in one work-group: the 2-D study's parent graphs are
// deep and narrow (~2,000 levels of ~100 vertices at 250k vertices), so a launch
// (and a convergence read) per level would cost more than the level's work.
// Each level's frontier lives in global memory (qa / qb, each vertex enters once);
// block barriers order the levels, which makes every earlier level's lambdas
// visible to the next.  A vertex sums lambda = g + sum alpha_c lambda_c over its
// children in child order (the value a sweep of lambda = g + P^T lambda gives);
// the second member of a two-cycle to become ready solves the pair
//   lam_a = S_a + w_ca lam_c,  lam_c = S_c + w_ac lam_a.
// Ends when a frontier is empty (each vertex enters at most once, so after at
// most n_v levels).
__global__ void __launch_bounds__(kWalkThreads)
    k_tri_walk(const int* __restrict__ cptr, const int* __restrict__ cchild,
               const float* __restrict__ calpha, const float* __restrict__ g, float* lam,
               const int* __restrict__ par, const int2* __restrict__ pnode,
               const float4* __restrict__ pa, const int* __restrict__ partner,
               int* __restrict__ rem, int* __restrict__ pairrem, int* __restrict__ done,
               const float* __restrict__ T, int* qa, int* qb, int n_v, TriCtl* ctl) {
    __shared__ int n_cur, n_next, n_fin;
    if (threadIdx.x == 0) {
        n_cur = 0;
        n_fin = 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_v; i += blockDim.x)
        if (T[i] < GBP_INF && rem[i] == 0) qa[atomicAdd(&n_cur, 1)] = i;
    __syncthreads();
    int* cur = qa;
    int* nxt = qb;
    int level = 0;
    while (n_cur > 0) {
        const int n = n_cur;
        __syncthreads();                    // everyone has read n_cur
        if (threadIdx.x == 0) n_next = 0;
        __syncthreads();
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const int x = cur[k];
            // what depends on x alone, in one round trip
            const int q = partner[x];
            const int e0 = cptr[x], e1 = cptr[x + 1];
            const float gx = g[x];
            const int px = par[x];
            const int2 pn = pnode[x];
            const float4 pw = pa[x];
            if (q < 0) {
                // children four at a time: their ids and weights, then their lambdas,
                // summed in child order
                float l = gx;
                for (int e = e0; e < e1; e += 4) {
                    int c[4];
                    float a[4], lc[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        c[j] = e + j < e1 ? cchild[e + j] : -1;
                        a[j] = e + j < e1 ? calpha[e + j] : 0.f;
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) lc[j] = c[j] >= 0 ? lam[c[j]] : 0.f;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (e + j < e1) l += a[j] * lc[j];
                }
                lam[x] = l;
                done[x] = 1;
                atomicAdd(&n_fin, 1);
                tri_release(px, pn, pw, -1, x, rem, nxt, &n_next);
                continue;
            }
            if (atomicSub(&pairrem[min(x, q)], 1) != 1) continue;   // partner not ready yet
            float S[2], w[2];
            const int pr[2] = {x, q};
            for (int m = 0; m < 2; ++m) {
                const int a = pr[m], o = pr[1 - m];
                float l = g[a], wo = 0.f;
                for (int e = cptr[a]; e < cptr[a + 1]; ++e) {
                    const int c = cchild[e];
                    if (c == o) wo = calpha[e];
                    else l += calpha[e] * lam[c];
                }
                S[m] = l;
                w[m] = wo;                  // weight of a in o's parent face
            }
            const float lx = (S[0] + w[0] * S[1]) / (1.f - w[0] * w[1]);
            lam[x] = lx;
            lam[q] = S[1] + w[1] * lx;
            done[x] = 1;
            done[q] = 1;
            atomicAdd(&n_fin, 2);
            tri_release(px, pn, pw, q, x, rem, nxt, &n_next);
            tri_release(par[q], pnode[q], pa[q], x, q, rem, nxt, &n_next);
        }
        __syncthreads();                    // the level's lambdas, releases and n_next
        if (threadIdx.x == 0) n_cur = n_next;
        int* t = cur;
        cur = nxt;
        nxt = t;
        ++level;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ctl->levels = level;
        atomicSub(&ctl->remaining, n_fin);
    }
}

// the reached vertices the walk left unfinished (on or above longer cycles), as a list
__global__ void k_tri_walk_list(const int* __restrict__ done, int n_v, int* __restrict__ list,
                                TriCtl* ctl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_v && !done[i]) list[atomicAdd(&ctl->nlist, 1)] = i;
}

__global__ void k_tri_grad_tri(const float2* __restrict__ xy, const int4* __restrict__ tri,
                               const float* __restrict__ D, const float* __restrict__ vscale,
                               const int* __restrict__ par, const int2* __restrict__ pnode,
                               const float4* __restrict__ pa, const float* __restrict__ lam, int n_v,
                               float* __restrict__ dD, float* __restrict__ dsbar) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_v) return;
    const int t = par[i];
    const float l = lam[i];
    if (t < 0 || l == 0.f) return;
    const int2 p = pnode[i];
    const float4 w = pa[i];
    const int4 tv = tri[t];
    double sbar = 1.0;
    if (vscale) sbar = ((double)vscale[tv.x] + vscale[tv.y] + vscale[tv.z]) / 3.0;
    const double dxx = D[3 * (size_t)t], dyy = D[3 * (size_t)t + 1], dxy = D[3 * (size_t)t + 2];
    const double idet = 1.0 / (dxx * dyy - dxy * dxy);
    const double ex = w.x * ((double)xy[p.x].x - xy[i].x) + w.y * ((double)xy[p.y].x - xy[i].x);
    const double ey = w.x * ((double)xy[p.x].y - xy[i].y) + w.y * ((double)xy[p.y].y - xy[i].y);
    const double ux = (dyy * ex - dxy * ey) * idet, uy = (dxx * ey - dxy * ex) * idet;   // D^-1 e
    const double h = sqrt((ex * ux + ey * uy) / (sbar * sbar));
    if (!(h > 0.0)) return;
    if (dD) {
        const double cf = -(double)l / (2.0 * sbar * sbar * h);
        atomicAdd(&dD[3 * (size_t)t], (float)(cf * ux * ux));
        atomicAdd(&dD[3 * (size_t)t + 1], (float)(cf * uy * uy));
        atomicAdd(&dD[3 * (size_t)t + 2], (float)(2.0 * cf * ux * uy));
    }
    atomicAdd(&dsbar[t], (float)((double)l * (-h / sbar)));
}

__global__ void k_tri_grad_node(const int* __restrict__ vptr, const int* __restrict__ vent,
                                const float* __restrict__ dsbar, int n_v, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_v) return;
    float s = 0.f;
    for (int e = vptr[i]; e < vptr[i + 1]; ++e) s += dsbar[vent[e] >> 2];
    out[i] = s * (1.f / 3.f);
}

__global__ void k_tri_grad_root(const int* __restrict__ root_node, const float* __restrict__ root_t,
                                int n_roots, int n_v, const float4* __restrict__ pa,
                                const float* __restrict__ troot, const float* __restrict__ lam,
                                float* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_roots) return;
    const int u = root_node[r];
    float v = 0.f;
    if (u >= 0 && u < n_v) {
        bool active = pa[u].w > 0.5f && root_t[r] == troot[u];
        for (int q = 0; q < r && active; ++q)
            if (root_node[q] == u && root_t[q] == root_t[r]) active = false;
        if (active) v = lam[u];
    }
    out[r] = v;
}

int tri_check(gbp_tri_plan p, const float* D, const int32_t* root_node, const float* root_t,
              int n_roots) {
    if (!p) {
        gbp_set_error("null triangle plan");
        return GBP_ERR_ARG;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev != p->device) {
        gbp_set_error("triangle plan belongs to device %d, current device is %d", p->device, dev);
        return GBP_ERR_ARG;
    }
    if (!D || n_roots < 0 || (n_roots > 0 && (!root_node || !root_t))) {
        gbp_set_error("D is required, n_roots >= 0 with root arrays");
        return GBP_ERR_ARG;
    }
    return GBP_OK;
}

int tri_read(gbp_tri_plan p, hipStream_t s) {
    GBP_HIP(hipMemcpyAsync(p->ctl_host, p->ctl, sizeof(TriCtl), hipMemcpyDeviceToHost, s));
    GBP_HIP(hipStreamSynchronize(s));
    return GBP_OK;
}

// metric, onsets and (cold) the first queue; cold = 0 leaves T alone
int tri_prepare(gbp_tri_plan p, const float* D, const float* vscale, const int32_t* root_node,
                const float* root_t, int n_roots, bool cold, hipStream_t s) {
    const int n_v = p->n_v;
    k_tri_ctl_reset<<<1, 64, 0, s>>>(p->ctl);
    if (p->stamp > (1 << 30)) {
        k_tri_fill_i<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(p->mark, 0, n_v);
        p->stamp = 1;
    }
    k_tri_metric<<<gbp_blocks(p->n_t, TPB), TPB, 0, s>>>(D, vscale, p->tri, p->n_t, p->minv, p->ctl);
    k_tri_fill<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(p->troot, GBP_INF, n_v);
    if (cold) k_tri_fill<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(p->T, GBP_INF, n_v);
    k_tri_roots<<<1, TPB, 0, s>>>(root_node, root_t, n_roots, n_v, p->troot, p->T, cold ? 1 : 0,
                                  p->nbp, p->nb, p->q[0], p->mark, p->stamp, p->ctl);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

}  // namespace

extern "C" int gbp_tri_plan_create(const float* xy, int n_v, const int32_t* tris, int n_t,
                                   gbp_tri_plan* out) {
    if (!out || !xy || !tris || n_v < 1 || n_t < 1) {
        gbp_set_error("tri_plan_create: xy, tris, out required; n_v, n_t >= 1");
        return GBP_ERR_ARG;
    }
    *out = nullptr;
    for (int i = 0; i < 2 * n_v; ++i)
        if (!std::isfinite(xy[i])) {
            gbp_set_error("non-finite coordinate at vertex %d", i / 2);
            return GBP_ERR_NONFINITE;
        }
    for (int t = 0; t < n_t; ++t) {
        const int32_t* v = tris + 3 * (size_t)t;
        for (int k = 0; k < 3; ++k)
            if (v[k] < 0 || v[k] >= n_v) {
                gbp_set_error("triangle %d: vertex id out of range", t);
                return GBP_ERR_ARG;
            }
        if (v[0] == v[1] || v[0] == v[2] || v[1] == v[2]) {
            gbp_set_error("triangle %d repeats a vertex", t);
            return GBP_ERR_ARG;
        }
        const double ax = xy[2 * v[1]] - xy[2 * v[0]], ay = xy[2 * v[1] + 1] - xy[2 * v[0] + 1];
        const double bx = xy[2 * v[2]] - xy[2 * v[0]], by = xy[2 * v[2] + 1] - xy[2 * v[0] + 1];
        const double cx = bx - ax, cy = by - ay;
        const double l2 = std::max(std::max(ax * ax + ay * ay, bx * bx + by * by), cx * cx + cy * cy);
        if (!(std::fabs(ax * by - ay * bx) > 1e-7 * l2)) {
            gbp_set_error("triangle %d is degenerate", t);
            return GBP_ERR_DEGENERATE_TET;
        }
    }
    // incidence (sorted by triangle within a vertex) and unique neighbours
    std::vector<int> vptr(n_v + 1, 0), vent((size_t)3 * n_t);
    for (int t = 0; t < n_t; ++t)
        for (int k = 0; k < 3; ++k) vptr[tris[3 * (size_t)t + k] + 1]++;
    for (int i = 0; i < n_v; ++i) vptr[i + 1] += vptr[i];
    {
        std::vector<int> cur(vptr.begin(), vptr.end() - 1);
        for (int t = 0; t < n_t; ++t)
            for (int k = 0; k < 3; ++k) vent[cur[tris[3 * (size_t)t + k]]++] = (t << 2) | k;
    }
    std::vector<int> nbp(n_v + 1, 0), nb;
    nb.reserve((size_t)6 * n_v);
    std::vector<int> tmp;
    for (int i = 0; i < n_v; ++i) {
        tmp.clear();
        for (int e = vptr[i]; e < vptr[i + 1]; ++e) {
            const int t = vent[e] >> 2;
            for (int k = 0; k < 3; ++k)
                if (tris[3 * (size_t)t + k] != i) tmp.push_back(tris[3 * (size_t)t + k]);
        }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        nb.insert(nb.end(), tmp.begin(), tmp.end());
        nbp[i + 1] = (int)nb.size();
    }
    std::vector<float2> xy2(n_v);
    for (int i = 0; i < n_v; ++i) xy2[i] = make_float2(xy[2 * i], xy[2 * i + 1]);
    std::vector<int4> t4(n_t);
    for (int t = 0; t < n_t; ++t)
        t4[t] = make_int4(tris[3 * (size_t)t], tris[3 * (size_t)t + 1], tris[3 * (size_t)t + 2], 0);

    gbp_tri_plan p = new gbp_tri_plan_s();
    (void)hipGetDevice(&p->device);
    p->n_v = n_v;
    p->n_t = n_t;
    int rc = GBP_OK;
#define TRI_TRY(x)                  \
    if ((rc = (x)) != GBP_OK) {     \
        tri_free(p);                \
        return rc;                  \
    }
#define TRI_UP(dst, src, n)                                                                  \
    TRI_TRY(tri_alloc(&(dst), (n)));                                                        \
    if (hipMemcpy((dst), (src), (n) * sizeof(*(src)), hipMemcpyHostToDevice) != hipSuccess) { \
        gbp_set_error("upload failed");                                                      \
        tri_free(p);                                                                         \
        return GBP_ERR_HIP;                                                                  \
    }
    TRI_UP(p->xy, xy2.data(), (size_t)n_v);
    TRI_UP(p->tri, t4.data(), (size_t)n_t);
    TRI_UP(p->vptr, vptr.data(), (size_t)n_v + 1);
    TRI_UP(p->vent, vent.data(), (size_t)3 * n_t);
    TRI_UP(p->nbp, nbp.data(), (size_t)n_v + 1);
    TRI_UP(p->nb, nb.data(), nb.size());
    TRI_TRY(tri_alloc(&p->minv, n_t));
    TRI_TRY(tri_alloc(&p->T, n_v));
    TRI_TRY(tri_alloc(&p->troot, n_v));
    TRI_TRY(tri_alloc(&p->q[0], n_v));
    TRI_TRY(tri_alloc(&p->q[1], n_v));
    TRI_TRY(tri_alloc(&p->mark, n_v));
    TRI_TRY(tri_alloc(&p->ctl, 1));
    TRI_TRY(tri_alloc(&p->par, n_v));
    TRI_TRY(tri_alloc(&p->pnode, n_v));
    TRI_TRY(tri_alloc(&p->pa, n_v));
    TRI_TRY(tri_alloc(&p->ccnt, (size_t)n_v + 1));
    TRI_TRY(tri_alloc(&p->cfill, n_v));
    TRI_TRY(tri_alloc(&p->rdy, n_v));
    TRI_TRY(tri_alloc(&p->partner, n_v));
    TRI_TRY(tri_alloc(&p->pairrem, n_v));
    TRI_TRY(tri_alloc(&p->cchild, (size_t)2 * n_v));
    TRI_TRY(tri_alloc(&p->calpha, (size_t)2 * n_v));
    TRI_TRY(tri_alloc(&p->lam[0], n_v));
    TRI_TRY(tri_alloc(&p->g, n_v));
    TRI_TRY(tri_alloc(&p->dsbar, n_t));
    TRI_TRY(tri_alloc(&p->scan_tmp, (size_t)(n_v / 256 + 2)));
#undef TRI_UP
#undef TRI_TRY
    if (hipHostMalloc((void**)&p->ctl_host, sizeof(TriCtl)) != hipSuccess ||
        hipHostMalloc((void**)&p->ctl_pipe, 2 * sizeof(TriCtl)) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev[1], hipEventDisableTiming) != hipSuccess ||
        hipMemset(p->mark, 0, (size_t)n_v * sizeof(int)) != hipSuccess) {
        gbp_set_error("pinned control block or mark reset failed");
        tri_free(p);
        return GBP_ERR_HIP;
    }
    *out = p;
    return GBP_OK;
}

extern "C" void gbp_tri_plan_destroy(gbp_tri_plan p) { tri_free(p); }

extern "C" int gbp_tri_backward_info(gbp_tri_plan p, int* levels, int* cyclic, int* sweeps) {
    if (!p) {
        gbp_set_error("null triangle plan");
        return GBP_ERR_ARG;
    }
    if (levels) *levels = p->last_levels;
    if (cyclic) *cyclic = p->last_cyclic;
    if (sweeps) *sweeps = p->last_sweeps;
    return GBP_OK;
}

extern "C" int gbp_tri_forward(gbp_tri_plan p, const float* D, const float* vscale,
                               const int32_t* root_node, const float* root_t, int n_roots,
                               float* T_out, gbp_stats* stats, void* stream) {
    int rc = tri_check(p, D, root_node, root_t, n_roots);
    if (rc) return rc;
    if (!T_out) {
        gbp_set_error("T_out is required");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const int n_v = p->n_v;
    if ((rc = tri_prepare(p, D, vscale, root_node, root_t, n_roots, true, s))) return rc;
    // enough blocks for the widest narrow front at 8 lanes or for a wide front at 4
    const size_t lanes_max = std::max<size_t>((size_t)std::min(n_v, kNarrowFront) * 8, (size_t)n_v * 4);
    const int grid = (int)std::max<size_t>(1, std::min<size_t>((lanes_max + TPB - 1) / TPB, 1024));
    // batches of 8 rounds; the host checks batch k's queue length (copied into
    // pinned memory behind it, with an event) only once batch k + 1 is queued, so
    // the device never waits for the check; a finished solve costs one batch of
    // empty rounds (each returns at once)
    int r = 0, batch = 0, r_prev = 0;
    bool converged = false;
    while (r < p->max_rounds) {
        for (int b = 0; b < 8; ++b, ++r)
            k_tri_sweep<<<grid, TPB, 0, s>>>(p->xy, p->tri, p->minv, p->vptr, p->vent, p->nbp, p->nb,
                                              p->T, p->q[r & 1], p->q[(r + 1) & 1], p->mark, p->ctl, r,
                                              p->stamp + r + 1, p->eps_rel);
        GBP_LAUNCH_CHECK();
        GBP_HIP(hipMemcpyAsync(p->ctl_pipe + (batch & 1), p->ctl, sizeof(TriCtl), hipMemcpyDeviceToHost, s));
        GBP_HIP(hipEventRecord(p->ev[batch & 1], s));
        if (batch > 0) {
            GBP_HIP(hipEventSynchronize(p->ev[(batch - 1) & 1]));
            const TriCtl& c = p->ctl_pipe[(batch - 1) & 1];
            if (c.err) break;
            if (c.count[r_prev % 3] == 0) {
                converged = true;
                break;
            }
        }
        r_prev = r;
        ++batch;
    }
    p->stamp += r + 2;
    k_tri_count_inf<<<gbp_blocks(n_v, TPB), TPB, 0, s>>>(p->T, n_v, p->ctl);
    GBP_HIP(hipMemcpyAsync(T_out, p->T, (size_t)n_v * sizeof(float), hipMemcpyDeviceToDevice, s));
    if ((rc = tri_read(p, s))) return rc;
    const TriCtl& c = *p->ctl_host;
    if (!converged && !c.err && c.count[r % 3] == 0) converged = true;   // the cap's last batch finished it
    if (stats) {
        stats->rounds = c.rounds;
        stats->converged = converged ? 1 : 0;
        stats->face_solves = (int64_t)c.solves;
        stats->node_updates = (int64_t)c.updates;
        stats->unreached = c.unreached;
    }
    if (c.err) return gbp_err_from_bits(c.err);
    if (!converged) {
        gbp_set_error("triangle forward did not converge in %d rounds", r);
        return GBP_ERR_NOT_CONVERGED;
    }
    return GBP_OK;
}

extern "C" int gbp_tri_backward(gbp_tri_plan p, const float* D, const float* vscale,
                                const int32_t* root_node, const float* root_t, int n_roots,
                                const float* T, const float* dL_dT, float* dL_dD,
                                float* dL_dvscale, float* dL_droot_t, void* stream) {
    int rc = tri_check(p, D, root_node, root_t, n_roots);
    if (rc) return rc;
    if (!T || !dL_dT) {
        gbp_set_error("T and dL_dT are required");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const int n_v = p->n_v, n_t = p->n_t;
    const int nb = gbp_blocks(n_v, TPB);
    GBP_HIP(hipMemcpyAsync(p->T, T, (size_t)n_v * sizeof(float), hipMemcpyDeviceToDevice, s));
    if ((rc = tri_prepare(p, D, vscale, root_node, root_t, n_roots, false, s))) return rc;
    k_tri_parent<<<nb, TPB, 0, s>>>(p->xy, p->tri, D, vscale, p->vptr, p->vent, p->T, p->troot, n_v,
                                    p->par, p->pnode, p->pa);
    // child lists in a fixed order
    k_tri_fill_i<<<gbp_blocks(n_v + 1, TPB), TPB, 0, s>>>(p->cfill, 0, n_v);
    k_tri_child_count<<<nb, TPB, 0, s>>>(p->par, p->pnode, p->pa, n_v, p->cfill);
    GBP_LAUNCH_CHECK();
    if ((rc = gbp_scan_exclusive(p->cfill, p->ccnt, n_v, p->scan_tmp, s))) return rc;
    k_tri_fill_i<<<nb, TPB, 0, s>>>(p->cfill, 0, n_v);
    k_tri_child_fill<<<nb, TPB, 0, s>>>(p->par, p->pnode, p->pa, n_v, p->ccnt, p->cfill, p->cchild,
                                        p->calpha);
    k_tri_child_sort<<<nb, TPB, 0, s>>>(p->ccnt, p->cchild, p->calpha, n_v);
    k_tri_adj_init<<<nb, TPB, 0, s>>>(dL_dT, p->T, n_v, p->g, p->lam[0]);
    // two-cycles, then the leaves-first walk in one work-group (cfill: the children
    // each vertex still waits for; rdy: finished flags; the forward's queues hold
    // the frontiers)
    k_tri_partner<<<nb, TPB, 0, s>>>(p->par, p->pnode, p->pa, n_v, p->partner);
    k_tri_partner_sym<<<nb, TPB, 0, s>>>(p->partner, n_v, p->pairrem);
    k_tri_partner_fix<<<nb, TPB, 0, s>>>(p->partner, p->pairrem, n_v);
    k_tri_walk_init<<<nb, TPB, 0, s>>>(p->ccnt, p->partner, p->T, n_v, p->cfill, p->rdy, p->ctl);
    k_tri_walk<<<1, kWalkThreads, 0, s>>>(p->ccnt, p->cchild, p->calpha, p->g, p->lam[0], p->par, p->pnode,
                                          p->pa, p->partner, p->cfill, p->pairrem, p->rdy, p->T, p->q[0],
                                          p->q[1], n_v, p->ctl);
    GBP_LAUNCH_CHECK();
    if ((rc = tri_read(p, s))) return rc;
    if (p->ctl_host->err) return gbp_err_from_bits(p->ctl_host->err);
    p->last_levels = p->ctl_host->levels;
    p->last_cyclic = p->ctl_host->remaining;
    // vertices on or above parent-graph cycles: Gauss-Seidel sweeps over just
    // those (their children outside the list are final), checked every 16
    int it = 0;
    if (p->ctl_host->remaining > 0) {
        k_tri_walk_list<<<nb, TPB, 0, s>>>(p->rdy, n_v, p->cfill, p->ctl);   // rem is no longer needed
        const int gs_grid = std::max(1, std::min(gbp_blocks(p->ctl_host->remaining, TPB), 1024));
        const int cap = 8 * n_v + 64;
        bool settled = false;
        while (it < cap) {
            for (int b = 0; b < 16; ++b, ++it)
                k_tri_adj_gs<<<gs_grid, TPB, 0, s>>>(p->cfill, p->ccnt, p->cchild, p->calpha, p->g,
                                                     p->lam[0], p->ctl, it);
            GBP_LAUNCH_CHECK();
            if ((rc = tri_read(p, s))) return rc;
            const float d = __builtin_bit_cast(float, p->ctl_host->diff_bits[(it - 1) & 1]);
            const float a = __builtin_bit_cast(float, p->ctl_host->lmax_bits[(it - 1) & 1]);
            if (d <= 1e-7f * a) {
                settled = true;
                break;
            }
        }
        if (!settled) {
            gbp_set_error("triangle adjoint did not settle in %d sweeps", it);
            return GBP_ERR_NOT_CONVERGED;
        }
    }
    p->last_sweeps = it;
    const float* lam = p->lam[0];
    k_tri_fill<<<gbp_blocks(n_t, TPB), TPB, 0, s>>>(p->dsbar, 0.f, n_t);
    if (dL_dD) k_tri_fill<<<gbp_blocks(3LL * n_t, TPB), TPB, 0, s>>>(dL_dD, 0.f, 3 * n_t);
    k_tri_grad_tri<<<nb, TPB, 0, s>>>(p->xy, p->tri, D, vscale, p->par, p->pnode, p->pa, lam, n_v,
                                      dL_dD, p->dsbar);
    if (dL_dvscale)
        k_tri_grad_node<<<nb, TPB, 0, s>>>(p->vptr, p->vent, p->dsbar, n_v, dL_dvscale);
    if (dL_droot_t && n_roots > 0)
        k_tri_grad_root<<<gbp_blocks(n_roots, TPB), TPB, 0, s>>>(root_node, root_t, n_roots, n_v,
                                                                 p->pa, p->troot, lam, dL_droot_t);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}
