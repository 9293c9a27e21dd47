// Internal declarations shared by the translation units of libgbp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "gbp.h"

// ---------------------------------------------------------------- errors
void gbp_set_error(const char* fmt, ...);

#define GBP_HIP(call)                                                           \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) {                                                 \
            gbp_set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                          __FILE__, __LINE__);                                  \
            return GBP_ERR_HIP;                                                 \
        }                                                                       \
    } while (0)

#define GBP_LAUNCH_CHECK()                                                   \
    do {                                                                     \
        hipError_t e_ = hipGetLastError();                                   \
        if (e_ != hipSuccess) {                                              \
            gbp_set_error("kernel launch failed: %s (%s:%d)",                \
                          hipGetErrorString(e_), __FILE__, __LINE__);        \
            return GBP_ERR_HIP;                                              \
        }                                                                    \
    } while (0)

// Device-side error bits (set by kernels, read back at synchronisation points).
enum : int {
    ERRBIT_ROOT_RANGE = 1,
    ERRBIT_ROOT_NONFINITE = 2,
    ERRBIT_D_NONFINITE = 4,
    ERRBIT_D_NOT_SPD = 8,
    ERRBIT_VSCALE = 16,
    ERRBIT_SPIN = 32,
};

// Control block of the relaxation loops (device memory, mirrored to pinned host).
struct GbpCtl {
    int count[3];                  // rotating queue lengths
    int err;                       // ERRBIT_* flags
    unsigned long long solves;     // local problems evaluated
    unsigned long long updates;    // nodes that changed
    int unreached;
    int remaining;                 // adjoint: vertices the level walk did not finish
    float maxdiff;                 // adjoint fallback: largest change of an even sweep
    float maxdiff2;                // ... of an odd sweep
    int rounds;                    // forward: last round with work + 1
    int lmax_bits;                 // adjoint fallback: largest |lambda| (float bits)
    int stamp;                     // queue stamp base, kept across calls
    int status;                    // bit 0: forward not converged, bit 1: adjoint not settled
    int levels;                    // adjoint: last level with work + 1
    int marks_stale;               // set by a reset that restarted the stamps: clear the marks
    int qcnt[3][8];                // forward: rotating lengths of the 8 sub-queues
    // bucketed hold-back of the cold forward (Delta-stepping): changed vertices whose
    // value lies beyond the current bucket wait in per-bucket lists (a ring)
    float tmin;                    // smallest root onset: bucket 0 starts there
    int bcur[3];                   // rotating current bucket
    int bcnt[64];                  // entries per ring slot (slot = bucket % 64)
};
constexpr int kHoldBuckets = 64;   // ring size (bcnt)

// The forward's work queue is split into 8 sub-queues, one per XCD: the vertex
// range (Morton order) is cut into kXcdRegions contiguous regions, region r
// belongs to sub-queue r % 8, and the blocks of a relaxation round that the
// hardware places on XCD x (blockIdx % 8 == x) work on sub-queue x.  Each XCD's
// L2 then caches a fixed eighth of the mesh.
constexpr int kXcdRegions = 512;
struct XcdQueues {
    int off[9];                    // segment of sub-queue x: [off[x], off[x+1])
    int R;                         // vertices per region
    int nq;                        // 8 (split) or 1 (one queue: R = n_v, every block serves it)
};
void gbp_set_queue_layout(gbp_plan p, int split);

struct gbp_plan_s {
    int device = 0;
    int n_v = 0, n_e = 0;
    int n_adj = 0;
    int max_rounds = 0;
    float eps_rel = 0.f;

    // mesh, internal numbering (device)
    float4* xyz = nullptr;        // [n_v]  (x, y, z, 0)
    int4* tetv = nullptr;         // [n_e]  internal vertex ids
    int* tet_user = nullptr;      // [n_e]  internal element -> caller element id
    int* tet_int = nullptr;       // [n_e]  caller element id -> internal element
    int* node_user = nullptr;     // [n_v]  internal node -> caller node id
    int* node_int = nullptr;      // [n_v]  caller node id -> internal node
    int2* nptr = nullptr;         // [n_v]  (first entry, 4 packed 8-bit counts per local slot)
    int* nent = nullptr;          // [4 n_e] element ids sorted by (node, local slot, element)
    int* adj_ptr = nullptr;       // [n_v+1] unique neighbour lists
    int* adj = nullptr;           // [n_adj]
    int* comp = nullptr;          // [n_v] connected component of each vertex
    int* comp_root = nullptr;     // [n_comp] per call: the component holds a root
    int n_comp = 0;

    // per-call workspace (device)
    float4* tetg = nullptr;       // [2 n_e]: (G11,G22,G33,G12), (G13,G23,sbar,0)
    float* vs = nullptr;          // [n_v] nodal velocity scale (internal order)
    float* T = nullptr;           // [n_v] activation times (internal order)
    float* troot = nullptr;       // [n_v] min onset per node (+inf elsewhere)
    int* q[2] = {nullptr, nullptr};  // work queues
    int* mark = nullptr;          // [n_v] queue stamps
    XcdQueues xq{};               // sub-queue layout of q[0], q[1]
    // launch configuration (autotunable)
    int lanes = 16;               // lanes per vertex in a relaxation round (8, 16 or 32)
    int sweep_blocks = 2048;      // grid of a relaxation round (<= kStatBlocks)
    int solver = 0;               // local solver: 0 exact (predicated KKT), 1 FISTA (Alg. 1)
    int fista_iters = 32;         // FISTA iterations per local problem
    int fista_lmode = 1;          // FISTA step constant: 0 Eq. (lipschitz_est), 1 tightened
    float fista_tau = 0.f;        // > 0: per-face iterations from the rate bound, capped by fista_iters
    float hold_delta = 0.f;       // bucket width of the cold forward's hold-back (0: off)
    int hold_open = 0;            // queue length below which a round opens the next bucket (0: half the grid)
    int hold_window = 0;          // buckets past the current one that propagate at once
    int* hold = nullptr;          // [n_v] bucket a vertex was last held in (allocated on use)
    int* blist = nullptr;         // [kHoldBuckets * bcap] held vertices per ring slot
    int bcap = 0;                 // entries per ring slot
    int warm_order = 0;           // 1: a forward's T_init only orders the hold-back of a cold solve
    float* guess = nullptr;       // [n_v] that ordering guess (internal order, allocated on use)
    // inputs of the last full preparation (element metric, scales, onsets): a
    // backward may reuse them when the caller allows it and passes the same arrays
    int reuse_inputs = 0;
    bool prep_valid = false;
    const void *prep_D = nullptr, *prep_vs = nullptr, *prep_rn = nullptr, *prep_rt = nullptr;
    int prep_nroots = 0;
    float* lip = nullptr;         // [4 n_e] FISTA step constant per face (allocated on use)
    int level_blocks = 2048;      // grid of an adjoint level (scan; at least n_v / (8 * 256))
    int sync_batch = 16;          // launches between convergence checks (synchronous mode)
    int last_rounds = 0, last_levels = 0;   // of the last synchronous calls
    GbpCtl* ctl = nullptr;        // device control block
    unsigned long long* blk = nullptr;  // [2 * kStatBlocks] per-block (solves, updates)
    GbpCtl* ctl_host = nullptr;   // pinned mirror [3]: [0] status reads, [1..2] pipelined checks
    int* st_host = nullptr;       // pinned, device-mapped [2][kStWords]: loop status written by
    int* st_dev = nullptr;        //   the first launch of a batch (st_dev: its device address)
    hipEvent_t ev[2] = {nullptr, nullptr};   // completion of the pipelined status copies

    // backward workspace (allocated on first use)
    bool bwd_ready = false;
    int bwd_levels = 0, bwd_cyclic = 0, bwd_gs_sweeps = 0;   // last backward
    int* par = nullptr;           // [n_v] (element << 2 | local slot) or -1
    float4* pa = nullptr;         // [n_v] (alpha0, alpha1, alpha2, best)
    int* ccnt = nullptr;          // [n_v+1] children per node, then exclusive scan
    int* cfill = nullptr;         // [n_v]
    int* rem = nullptr;           // [n_v]
    int* cchild = nullptr;        // [3 n_v]
    float* calpha = nullptr;      // [3 n_v]
    float* lam = nullptr;         // [n_v]
    float* contrib = nullptr;     // [(kChildSlots + 3) n_v] alpha * lambda of each child entry, written by the child
    int4* cslot = nullptr;        // [n_v] position of a vertex in each weighted parent's child list
    float* g = nullptr;           // [n_v]
    float* dsbar = nullptr;       // [n_e]
    int* done = nullptr;          // [n_v] adjoint finished flag
    int* rdy = nullptr;           // [n_v] adjoint readiness stamp (launch index or marker)
    int4* pnode = nullptr;        // [n_v] parent face vertices with alpha > 0 (-1 otherwise)
    int* partner = nullptr;       // [n_v] mutual parent (two-cycle partner) or -1
    int* pairrem = nullptr;       // [n_v] members of a two-cycle not yet ready (at min id)
    int* scan_tmp = nullptr;      // block sums
};

constexpr int kStatBlocks = 2048;   // max grid of the relaxation kernels
// Loop status words a relaxation round or adjoint level writes for the host when
// asked: [0..7] work left (the round's sub-queue lengths; a level: [0] its work
// flag), [8] device error bits, [9] the launch index that wrote them.  They live
// in coherent pinned host memory: the host reads them after an event that follows
// the writing launch, when the launch's writes have completed.
constexpr int kStWords = 16;
// Adjoint entries: the first kChildSlots children of vertex x hand over their
// alpha * lambda in fixed slots contrib[x * kChildSlots + r] (rank r in the
// sorted child list), further ones at contrib[n_v * kChildSlots + k] (k = the
// CSR index), so a finished vertex reads its first entries without its CSR range.
constexpr int kChildSlots = 8;

int gbp_plan_check(gbp_plan p);
int gbp_err_from_bits(int bits);
// budget <= 0: synchronous; > 0: fixed launch counts, graph-capturable
int gbp_forward_impl(gbp_plan p, const float* D, const float* vscale, const int32_t* root_node,
                     const float* root_t, int n_roots, const float* T_init, float* T_out,
                     gbp_stats* stats, hipStream_t s, int budget);
int gbp_backward_impl(gbp_plan p, const float* D, const float* vscale, const int32_t* root_node,
                      const float* root_t, int n_roots, const float* T, const float* dL_dT,
                      float* dL_dD, float* dL_dvscale, float* dL_droot_t, hipStream_t s,
                      int level_budget, int gs_budget);
int gbp_alloc_backward(gbp_plan p);

// exclusive scan of n ints in place into out[0..n] (out[n] = total); device
int gbp_scan_exclusive(const int* in, int* out, int n, int* tmp, hipStream_t s);

static inline int gbp_blocks(long long n, int threads) {
    long long b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    return (int)b;
}
