// Mesh plan: validation, locality reordering, node->element incidence (CSR by
// local vertex slot), unique-neighbour lists and device workspace.
//
// The patch omega_i of Sec. 2.1 (the elements that contain v_i) is stored as a
// node-sorted CSR of element ids, split by the local slot of v_i inside each
// element so that a kernel can unroll over the slot with compile-time face
// algebra.  Nodes are renumbered along a Morton curve of their coordinates and
// elements are sorted by their smallest internal vertex, so that neighbouring
// vertices and their elements sit close in memory.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstdlib>
#include <numeric>
#include <vector>

#include <climits>
#include <cstddef>
#include <cmath>

#include "gbp_internal.h"
#include "gbp_test_hooks.h"

static thread_local std::string g_last_error;

void gbp_set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

extern "C" const char* gbp_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* gbp_version(void) { return "gbp 0.1 (gfx950)"; }

static uint64_t spread3(uint64_t x) {
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

template <typename T>
static int upload(T** dst, const T* src, size_t n) {
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
    if (e != hipSuccess) {
        gbp_set_error("hipMalloc of %zu bytes failed: %s", n * sizeof(T), hipGetErrorString(e));
        return GBP_ERR_NOMEM;
    }
    if (src) {
        e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            gbp_set_error("hipMemcpy failed: %s", hipGetErrorString(e));
            return GBP_ERR_HIP;
        }
    }
    return GBP_OK;
}

template <typename T>
static int dalloc(T** dst, size_t n) {
    return upload<T>(dst, nullptr, n);
}

static void plan_free(gbp_plan p) {
    if (!p) return;
    void* ptrs[] = {p->xyz, p->tetv, p->tet_user, p->tet_int, p->node_user, p->node_int, p->nptr, p->nent,
                    p->adj_ptr, p->adj, p->tetg, p->vs, p->T, p->troot, p->q[0], p->q[1],
                    p->mark, p->ctl, p->blk, p->par, p->pa, p->ccnt, p->cfill, p->rem, p->cchild,
                    p->calpha, p->lam, p->contrib, p->cslot, p->g, p->dsbar, p->done, p->rdy, p->scan_tmp, p->lip,
                    p->pnode, p->partner, p->pairrem, p->hold, p->blist, p->guess, p->comp,
                    p->comp_root};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (p->ctl_host) (void)hipHostFree(p->ctl_host);
    if (p->st_host) (void)hipHostFree(p->st_host);
    for (hipEvent_t e : p->ev)
        if (e) (void)hipEventDestroy(e);
    delete p;
}

extern "C" void gbp_plan_destroy(gbp_plan p) { plan_free(p); }

extern "C" int gbp_plan_sizes(gbp_plan p, int* n_v, int* n_e) {
    if (!p) {
        gbp_set_error("null plan");
        return GBP_ERR_ARG;
    }
    if (n_v) *n_v = p->n_v;
    if (n_e) *n_e = p->n_e;
    return GBP_OK;
}

int gbp_plan_check(gbp_plan p) {
    if (!p || p->n_v <= 0) {
        gbp_set_error("invalid plan");
        return GBP_ERR_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
        gbp_set_error("plan was created on device %d but the current device is %d", p->device, dev);
        return GBP_ERR_ARG;
    }
    return GBP_OK;
}

extern "C" int gbp_plan_create(const float* xyz, int n_v, const int32_t* tets, int n_e,
                               const gbp_options* opt, gbp_plan* out) {
    if (!out) {
        gbp_set_error("out is NULL");
        return GBP_ERR_ARG;
    }
    *out = nullptr;
    if (!xyz || !tets || n_v <= 0 || n_e <= 0) {
        gbp_set_error("need xyz, tets, n_v > 0, n_e > 0 (got n_v=%d n_e=%d)", n_v, n_e);
        return GBP_ERR_ARG;
    }
    if ((long long)n_e * 4 >= (1LL << 31)) {
        gbp_set_error("too many elements (%d)", n_e);
        return GBP_ERR_ARG;
    }
    gbp_options o{};
    if (opt) o = *opt;
    for (int k = 0; k < 5; ++k)
        if (o.reserved[k] != 0) {
            gbp_set_error("gbp_options.reserved must be zero");
            return GBP_ERR_ARG;
        }
    for (long long i = 0; i < 3LL * n_v; ++i)
        if (!std::isfinite(xyz[i])) {
            gbp_set_error("non-finite coordinate at node %lld", i / 3);
            return GBP_ERR_NONFINITE;
        }
    for (int j = 0; j < n_e; ++j) {
        const int32_t* t = tets + 4 * (size_t)j;
        for (int a = 0; a < 4; ++a) {
            if (t[a] < 0 || t[a] >= n_v) {
                gbp_set_error("element %d has vertex id %d out of range [0,%d)", j, t[a], n_v);
                return GBP_ERR_ARG;
            }
            for (int b = 0; b < a; ++b)
                if (t[a] == t[b]) {
                    gbp_set_error("element %d repeats vertex %d", j, t[a]);
                    return GBP_ERR_ARG;
                }
        }
        double F[3][3], lmax = 0;
        for (int a = 1; a < 4; ++a)
            for (int d = 0; d < 3; ++d) F[a - 1][d] = (double)xyz[3 * t[a] + d] - xyz[3 * t[0] + d];
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b) {
                double s = 0;
                for (int d = 0; d < 3; ++d) {
                    double e = (double)xyz[3 * t[b] + d] - xyz[3 * t[a] + d];
                    s += e * e;
                }
                lmax = std::max(lmax, s);
            }
        double det = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                     F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                     F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
        double l3 = lmax * sqrt(lmax);
        if (!(fabs(det) / 6.0 >= 1e-7 * l3)) {
            gbp_set_error("element %d is degenerate (volume %g, longest edge %g)", j, det / 6.0,
                          sqrt(lmax));
            return GBP_ERR_DEGENERATE_TET;
        }
    }

    // ---- node order (internal -> caller)
    std::vector<int> node_user(n_v);
    std::iota(node_user.begin(), node_user.end(), 0);
    if (o.reorder >= 0) {
        float lo[3] = {xyz[0], xyz[1], xyz[2]}, hi[3] = {xyz[0], xyz[1], xyz[2]};
        for (int i = 0; i < n_v; ++i)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], xyz[3 * i + d]);
                hi[d] = std::max(hi[d], xyz[3 * i + d]);
            }
        float span = std::max(std::max(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
        if (span <= 0) span = 1;
        std::vector<uint64_t> key(n_v);
        for (int i = 0; i < n_v; ++i) {
            uint64_t c[3];
            for (int d = 0; d < 3; ++d)
                c[d] = (uint64_t)((xyz[3 * i + d] - lo[d]) / span * 2097151.0);
            key[i] = spread3(c[0]) | spread3(c[1]) << 1 | spread3(c[2]) << 2;
        }
        std::stable_sort(node_user.begin(), node_user.end(),
                         [&](int a, int b) { return key[a] < key[b]; });
    }
    std::vector<int> node_int(n_v);
    for (int i = 0; i < n_v; ++i) node_int[node_user[i]] = i;

    // ---- elements in internal numbering, sorted by smallest vertex
    std::vector<int4> tv(n_e);
    std::vector<int> tmin(n_e);
    for (int j = 0; j < n_e; ++j) {
        const int32_t* t = tets + 4 * (size_t)j;
        tv[j] = make_int4(node_int[t[0]], node_int[t[1]], node_int[t[2]], node_int[t[3]]);
        tmin[j] = std::min(std::min(tv[j].x, tv[j].y), std::min(tv[j].z, tv[j].w));
    }
    std::vector<int> tet_user(n_e);
    std::iota(tet_user.begin(), tet_user.end(), 0);
    std::stable_sort(tet_user.begin(), tet_user.end(),
                     [&](int a, int b) { return tmin[a] < tmin[b]; });
    std::vector<int4> tvs(n_e);
    for (int j = 0; j < n_e; ++j) tvs[j] = tv[tet_user[j]];
    std::vector<int> tet_int(n_e);
    for (int j = 0; j < n_e; ++j) tet_int[tet_user[j]] = j;

    // ---- incidence CSR by (node, slot, element)
    std::vector<int> cnt((size_t)n_v * 4, 0);
    for (int j = 0; j < n_e; ++j) {
        const int* v = &tvs[j].x;
        for (int k = 0; k < 4; ++k) cnt[(size_t)v[k] * 4 + k]++;
    }
    std::vector<int2> nptr(n_v);
    std::vector<int> start((size_t)n_v * 4);
    int run = 0;
    for (int i = 0; i < n_v; ++i) {
        int packed = 0;
        nptr[i].x = run;
        for (int k = 0; k < 4; ++k) {
            int c = cnt[(size_t)i * 4 + k];
            if (c > 255) {
                gbp_set_error("node %d belongs to %d elements in one local slot (max 255)",
                              node_user[i], c);
                return GBP_ERR_ARG;
            }
            start[(size_t)i * 4 + k] = run;
            run += c;
            packed |= c << (8 * k);
        }
        nptr[i].y = packed;
    }
    std::vector<int> nent((size_t)n_e * 4);
    for (int j = 0; j < n_e; ++j) {
        const int* v = &tvs[j].x;
        for (int k = 0; k < 4; ++k) nent[start[(size_t)v[k] * 4 + k]++] = j;
    }

    // ---- unique neighbours per node
    std::vector<int> adj_ptr(n_v + 1, 0);
    std::vector<int> adj;
    adj.reserve((size_t)n_v * 16);
    std::vector<int> tmp;
    for (int i = 0; i < n_v; ++i) {
        tmp.clear();
        int e = nptr[i].x;
        int tot = 0;
        for (int k = 0; k < 4; ++k) tot += (nptr[i].y >> (8 * k)) & 255;
        for (int c = 0; c < tot; ++c) {
            const int* v = &tvs[nent[e + c]].x;
            for (int k = 0; k < 4; ++k)
                if (v[k] != i) tmp.push_back(v[k]);
        }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        adj.insert(adj.end(), tmp.begin(), tmp.end());
        adj_ptr[i + 1] = (int)adj.size();
    }

    // ---- connected components (internal numbering): a two-sided warm start sets
    // the guess of every component without a root to +inf
    std::vector<int> comp(n_v);
    std::iota(comp.begin(), comp.end(), 0);
    auto find = [&comp](int x) {
        while (comp[x] != x) x = comp[x] = comp[comp[x]];
        return x;
    };
    for (int j = 0; j < n_e; ++j) {
        const int* v = &tvs[j].x;
        for (int k = 1; k < 4; ++k) {
            const int a = find(v[0]), r = find(v[k]);
            if (r != a) comp[std::max(r, a)] = std::min(r, a);   // roots link to the smaller root
        }
    }
    int n_comp = 0;
    {
        std::vector<int> root(n_v), label(n_v, -1);
        for (int i = 0; i < n_v; ++i) root[i] = find(i);   // before relabelling in place
        for (int i = 0; i < n_v; ++i) {
            if (label[root[i]] < 0) label[root[i]] = n_comp++;
            comp[i] = label[root[i]];
        }
    }

    std::vector<float4> x4(n_v);
    for (int i = 0; i < n_v; ++i) {
        int u = node_user[i];
        x4[i] = make_float4(xyz[3 * u], xyz[3 * u + 1], xyz[3 * u + 2], 0.f);
    }

    gbp_plan p = new gbp_plan_s();
    (void)hipGetDevice(&p->device);
    p->n_v = n_v;
    p->n_e = n_e;
    p->n_adj = (int)adj.size();
    p->eps_rel = o.eps_rel > 0 ? o.eps_rel : 1.0f / (1 << 20);
    p->max_rounds = o.max_rounds > 0 ? o.max_rounds : 20000;
    int rc = GBP_OK;
#define TRY(x)                 \
    if ((rc = (x)) != GBP_OK) { \
        plan_free(p);          \
        return rc;             \
    }
    TRY(upload(&p->xyz, x4.data(), n_v));
    TRY(upload(&p->tetv, tvs.data(), n_e));
    TRY(upload(&p->tet_user, tet_user.data(), n_e));
    TRY(upload(&p->tet_int, tet_int.data(), n_e));
    TRY(upload(&p->node_user, node_user.data(), n_v));
    TRY(upload(&p->node_int, node_int.data(), n_v));
    TRY(upload(&p->nptr, nptr.data(), n_v));
    TRY(upload(&p->nent, nent.data(), (size_t)n_e * 4));
    TRY(upload(&p->adj_ptr, adj_ptr.data(), n_v + 1));
    TRY(upload(&p->adj, adj.data(), adj.size()));
    TRY(upload(&p->comp, comp.data(), n_v));
    TRY(dalloc(&p->comp_root, (size_t)n_comp));
    p->n_comp = n_comp;
    TRY(dalloc(&p->tetg, (size_t)n_e * 2));
    TRY(dalloc(&p->vs, n_v));
    TRY(dalloc(&p->T, n_v));
    TRY(dalloc(&p->troot, n_v));
    gbp_set_queue_layout(p, 1);
    TRY(dalloc(&p->q[0], n_v));
    TRY(dalloc(&p->q[1], n_v));
    TRY(dalloc(&p->mark, n_v));
    TRY(dalloc(&p->ctl, 1));
    TRY(dalloc(&p->blk, 2 * (size_t)kStatBlocks));
#undef TRY
    GbpCtl c0{};
    c0.stamp = 1;
    if (hipMemset(p->mark, 0, sizeof(int) * n_v) != hipSuccess ||
        hipMemcpy(p->ctl, &c0, sizeof(GbpCtl), hipMemcpyHostToDevice) != hipSuccess) {
        gbp_set_error("hipMemset failed");
        plan_free(p);
        return GBP_ERR_HIP;
    }
    if (hipHostMalloc((void**)&p->ctl_host, 3 * sizeof(GbpCtl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&p->st_host, 2 * kStWords * sizeof(int),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev[1], hipEventDisableTiming) != hipSuccess) {
        gbp_set_error("hipHostMalloc failed");
        plan_free(p);
        return GBP_ERR_NOMEM;
    }
    if (hipHostGetDevicePointer((void**)&p->st_dev, p->st_host, 0) != hipSuccess || !p->st_dev) {
        gbp_set_error("hipHostGetDevicePointer failed");
        plan_free(p);
        return GBP_ERR_HIP;
    }
    memset(p->ctl_host, 0, 3 * sizeof(GbpCtl));
    memset(p->st_host, 0xff, 2 * kStWords * sizeof(int));
    *out = p;
    return GBP_OK;
}

int gbp_alloc_backward(gbp_plan p) {
    if (p->bwd_ready) return GBP_OK;
    const int n_v = p->n_v, n_e = p->n_e;
    if ((long long)(kChildSlots + 3) * n_v > INT_MAX) {
        gbp_set_error("adjoint: %d vertices exceed the entry layout (at most %d)", n_v,
                      INT_MAX / (kChildSlots + 3));
        return GBP_ERR_ARG;
    }
    int rc;
    if ((rc = dalloc(&p->par, n_v)) || (rc = dalloc(&p->pa, n_v)) ||
        (rc = dalloc(&p->ccnt, n_v + 1)) || (rc = dalloc(&p->cfill, n_v)) ||
        (rc = dalloc(&p->rem, n_v)) || (rc = dalloc(&p->cchild, (size_t)3 * n_v)) ||
        (rc = dalloc(&p->calpha, (size_t)3 * n_v)) || (rc = dalloc(&p->lam, n_v)) ||
        (rc = dalloc(&p->contrib, (size_t)(kChildSlots + 3) * n_v)) || (rc = dalloc(&p->cslot, n_v)) ||
        (rc = dalloc(&p->g, n_v)) ||
        (rc = dalloc(&p->dsbar, n_e)) || (rc = dalloc(&p->done, n_v)) || (rc = dalloc(&p->rdy, n_v)) ||
        (rc = dalloc(&p->pnode, n_v)) || (rc = dalloc(&p->partner, n_v)) ||
        (rc = dalloc(&p->pairrem, n_v)) ||
        (rc = dalloc(&p->scan_tmp, (size_t)(n_v / 256 + 2))))
        return rc;
    p->bwd_ready = true;
    return GBP_OK;
}

extern "C" int gbp_plan_set_launch(gbp_plan p, int lanes, int sweep_blocks, int level_blocks,
                                   int sync_batch) {
    if (!p || !(lanes == 8 || lanes == 16 || lanes == 32) || sweep_blocks < 64 ||
        sweep_blocks > kStatBlocks || level_blocks < 16 || level_blocks > 2048 || sync_batch < 1 ||
        sync_batch > 64) {
        gbp_set_error("set_launch: lanes in {8,16,32}, sweep_blocks 64..%d, level_blocks 16..2048, "
                      "sync_batch 1..64", kStatBlocks);
        return GBP_ERR_ARG;
    }
    p->lanes = lanes;
    p->sweep_blocks = sweep_blocks;
    p->level_blocks = level_blocks;
    p->sync_batch = sync_batch;
    return GBP_OK;
}

// Sub-queue layout of the relaxation queues: split (region r of R vertices
// belongs to sub-queue r % 8) or a single queue.
void gbp_set_queue_layout(gbp_plan p, int split) {
    const int n_v = p->n_v;
    const int R = split ? std::max(1, (n_v + kXcdRegions - 1) / kXcdRegions) : std::max(1, n_v);
    int cap[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int r = 0; (long long)r * R < n_v; ++r) cap[r & 7] += std::min(R, n_v - r * R);
    p->xq.R = R;
    p->xq.nq = split ? 8 : 1;
    p->xq.off[0] = 0;
    for (int x = 0; x < 8; ++x) p->xq.off[x + 1] = p->xq.off[x] + cap[x];
}

extern "C" int gbp_plan_set_queue_split(gbp_plan p, int split) {
    if (!p || (split != 0 && split != 1)) {
        gbp_set_error("set_queue_split: split must be 0 or 1");
        return GBP_ERR_ARG;
    }
    gbp_set_queue_layout(p, split);
    return GBP_OK;
}

extern "C" int gbp_plan_set_local_solver(gbp_plan p, int solver, int n_f, int lipschitz_mode) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if ((solver != 0 && solver != 1) || n_f < 1 || n_f > 100000 ||
        (lipschitz_mode != 0 && lipschitz_mode != 1)) {
        gbp_set_error("set_local_solver: solver 0 or 1, n_f 1..100000, lipschitz_mode 0 or 1");
        return GBP_ERR_ARG;
    }
    if (solver == 1 && !p->lip && (rc = dalloc(&p->lip, (size_t)4 * p->n_e))) return rc;
    p->solver = solver;
    p->fista_iters = n_f;
    p->fista_lmode = lipschitz_mode;
    return GBP_OK;
}

extern "C" int gbp_plan_get_local_solver(gbp_plan p, int* solver, int* n_f, int* lipschitz_mode) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (solver) *solver = p->solver;
    if (n_f) *n_f = p->fista_iters;
    if (lipschitz_mode) *lipschitz_mode = p->fista_lmode;
    return GBP_OK;
}

extern "C" int gbp_plan_set_fista_tolerance(gbp_plan p, float tau) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (!(tau >= 0.f) || !std::isfinite(tau)) {
        gbp_set_error("set_fista_tolerance: tau must be finite and >= 0");
        return GBP_ERR_ARG;
    }
    p->fista_tau = tau;
    return GBP_OK;
}

extern "C" int gbp_plan_set_hold(gbp_plan p, float delta, int window, int open_below) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (!(delta >= 0.f) || !std::isfinite(delta) || open_below < 0 || window < 0 ||
        window > kHoldBuckets / 2) {
        gbp_set_error("set_hold: delta finite and >= 0, window 0..%d, open_below >= 0",
                      kHoldBuckets / 2);
        return GBP_ERR_ARG;
    }
    p->hold_open = open_below;
    p->hold_window = window;
    if (delta > 0.f && !p->hold) {
        p->bcap = std::max(4096, p->n_v / 16);
        if ((rc = dalloc(&p->hold, (size_t)p->n_v)) ||
            (rc = dalloc(&p->blist, (size_t)kHoldBuckets * p->bcap)))
            return rc;
    }
    p->hold_delta = delta;
    return GBP_OK;
}

extern "C" int gbp_plan_set_warm_order(gbp_plan p, int on) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (on != 0 && on != 1) {
        gbp_set_error("set_warm_order: on must be 0 or 1 (got %d)", on);
        return GBP_ERR_ARG;
    }
    if (on && !p->guess && (rc = dalloc(&p->guess, (size_t)p->n_v))) return rc;
    p->warm_order = on;
    return GBP_OK;
}

extern "C" int gbp_plan_get_warm_order(gbp_plan p, int* on) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (on) *on = p->warm_order;
    return GBP_OK;
}

extern "C" int gbp_plan_get_hold(gbp_plan p, float* delta, int* window, int* open_below) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (delta) *delta = p->hold_delta;
    if (window) *window = p->hold_window;
    if (open_below) *open_below = p->hold_open;
    return GBP_OK;
}

extern "C" int gbp_plan_get_fista_tolerance(gbp_plan p, float* tau) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (!tau) {
        gbp_set_error("get_fista_tolerance: NULL argument");
        return GBP_ERR_ARG;
    }
    *tau = p->fista_tau;
    return GBP_OK;
}

extern "C" int gbp_plan_set_input_reuse(gbp_plan p, int on) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (on != 0 && on != 1) {
        gbp_set_error("set_input_reuse: on must be 0 or 1");
        return GBP_ERR_ARG;
    }
    p->reuse_inputs = on;
    return GBP_OK;
}

extern "C" int gbp_plan_set_stamp_base(gbp_plan p, int stamp) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (stamp < 1) {
        gbp_set_error("set_stamp_base: stamp must be >= 1");
        return GBP_ERR_ARG;
    }
    GBP_HIP(hipDeviceSynchronize());
    GBP_HIP(hipMemcpy(reinterpret_cast<char*>(p->ctl) + offsetof(GbpCtl, stamp), &stamp, sizeof(int),
                      hipMemcpyHostToDevice));
    return GBP_OK;
}

extern "C" int gbp_plan_get_queue_split(gbp_plan p, int* split) {
    if (!p || !split) {
        gbp_set_error("get_queue_split: NULL argument");
        return GBP_ERR_ARG;
    }
    *split = p->xq.nq == 8 ? 1 : 0;
    return GBP_OK;
}

extern "C" int gbp_plan_get_launch(gbp_plan p, int* lanes, int* sweep_blocks, int* level_blocks,
                                   int* sync_batch) {
    if (!p) {
        gbp_set_error("null plan");
        return GBP_ERR_ARG;
    }
    if (lanes) *lanes = p->lanes;
    if (sweep_blocks) *sweep_blocks = p->sweep_blocks;
    if (level_blocks) *level_blocks = p->level_blocks;
    if (sync_batch) *sync_batch = p->sync_batch;
    return GBP_OK;
}

extern "C" int gbp_plan_last_counts(gbp_plan p, int* rounds, int* levels) {
    if (!p) {
        gbp_set_error("null plan");
        return GBP_ERR_ARG;
    }
    if (rounds) *rounds = p->last_rounds;
    if (levels) *levels = p->last_levels;
    return GBP_OK;
}
