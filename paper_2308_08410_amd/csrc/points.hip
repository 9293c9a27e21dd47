// Roots at points inside elements (Sec. 2.3 Eq. (upwind_xi)).
//
// A root at a point x of element E_k with onset t gives the four vertices of E_k
// the values t + ||v - x|| in the metric of E_k (D_eff^-1, the step cost of the
// forward).  These are handed to the forward as ordinary vertex roots; its
// adjoint returns dL/d(onset) for them, and the chain rule below carries that
// to the point, the onset, the element's tensor and its nodes' velocity scales.
// Per-root work is a handful of flops: computed in FP64 from the FP32 inputs.
#include <climits>

#include "gbp_internal.h"

namespace {

constexpr int TPB = 256;

struct Sym3 {
    double xx, yy, zz, xy, xz, yz;
};

// inverse of a packed symmetric 3x3 (xx, yy, zz, xy, xz, yz) by cofactors
__device__ Sym3 sym_inverse(const float* __restrict__ d) {
    const double a = d[0], b = d[1], c = d[2], e = d[3], f = d[4], g = d[5];
    const double c00 = b * c - g * g, c11 = a * c - f * f, c22 = a * b - e * e;
    const double c01 = f * g - e * c, c02 = e * g - f * b, c12 = e * f - a * g;
    const double inv = 1.0 / (a * c00 + e * c01 + f * c02);
    return Sym3{c00 * inv, c11 * inv, c22 * inv, c01 * inv, c02 * inv, c12 * inv};
}

__device__ void sym_apply(const Sym3& M, const double* v, double* out) {
    out[0] = M.xx * v[0] + M.xy * v[1] + M.xz * v[2];
    out[1] = M.xy * v[0] + M.yy * v[1] + M.yz * v[2];
    out[2] = M.xz * v[0] + M.yz * v[1] + M.zz * v[2];
}

// The element of root r in internal numbering and the mean velocity scale of its
// nodes; false for an element id out of range.
__device__ bool root_element(int k, int n_e, const int* __restrict__ tet_int,
                             const int4* __restrict__ tetv, const int* __restrict__ node_user,
                             const float* __restrict__ vscale, int v[4], double& sbar) {
    if (k < 0 || k >= n_e) return false;
    const int4 t = tetv[tet_int[k]];
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
    sbar = 1.0;
    if (vscale) {
        double s = 0.0;
        for (int n = 0; n < 4; ++n) s += vscale[node_user[v[n]]];
        sbar = 0.25 * s;
    }
    return true;
}

__global__ void k_point_roots(const int* __restrict__ root_tet, const float* __restrict__ root_xyz,
                              const float* __restrict__ root_t, int n_roots,
                              const int* __restrict__ tet_int, const int4* __restrict__ tetv,
                              const float4* __restrict__ xyz, const int* __restrict__ node_user,
                              const float* __restrict__ D, const float* __restrict__ vscale, int n_e,
                              int* __restrict__ node_out, float* __restrict__ t_out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_roots) return;
    int v[4];
    double sbar;
    if (!root_element(root_tet[r], n_e, tet_int, tetv, node_user, vscale, v, sbar)) {
        for (int n = 0; n < 4; ++n) {   // the forward reports ids out of range
            node_out[4 * r + n] = -1;
            t_out[4 * r + n] = 0.f;
        }
        return;
    }
    const Sym3 Di = sym_inverse(D + 6 * (size_t)root_tet[r]);
    const double s2 = 1.0 / (sbar * sbar);
    const Sym3 M{Di.xx * s2, Di.yy * s2, Di.zz * s2, Di.xy * s2, Di.xz * s2, Di.yz * s2};
    const double px = root_xyz[3 * r], py = root_xyz[3 * r + 1], pz = root_xyz[3 * r + 2];
    const double t = root_t[r];
    for (int n = 0; n < 4; ++n) {
        const float4 q = xyz[v[n]];
        const double e[3] = {q.x - px, q.y - py, q.z - pz};
        double Me[3];
        sym_apply(M, e, Me);
        node_out[4 * r + n] = node_user[v[n]];
        t_out[4 * r + n] = (float)(t + sqrt(e[0] * Me[0] + e[1] * Me[1] + e[2] * Me[2]));
    }
}

// Chain rule of the point-root values; with e = v - x, h = |e|_M, M = D_eff^-1:
//   dt = sum_n g_n,  dx = -sum_n g_n M e / h,
//   dD_k += g_n (-sbar^-2 D^-1 e e^T D^-1 / (2h)),  dsbar += g_n (-h / sbar).
// A vertex at the point (h = 0) contributes to dt only.  dD and dvscale are
// accumulated with atomics (roots sharing an element or a node add in any order).
__global__ void k_point_roots_bwd(const int* __restrict__ root_tet, const float* __restrict__ root_xyz,
                                  int n_roots, const int* __restrict__ tet_int,
                                  const int4* __restrict__ tetv, const float4* __restrict__ xyz,
                                  const int* __restrict__ node_user, const float* __restrict__ D,
                                  const float* __restrict__ vscale, int n_e,
                                  const float* __restrict__ g_onset, float* __restrict__ dt,
                                  float* __restrict__ dx, float* __restrict__ dD,
                                  float* __restrict__ dvs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_roots) return;
    int v[4];
    double sbar;
    const bool ok = root_element(root_tet[r], n_e, tet_int, tetv, node_user, vscale, v, sbar);
    double gt = 0.0, gx[3] = {0.0, 0.0, 0.0}, gD[6] = {0, 0, 0, 0, 0, 0}, gs = 0.0;
    if (ok) {
        const int k = root_tet[r];
        const Sym3 Di = sym_inverse(D + 6 * (size_t)k);
        const double s2 = 1.0 / (sbar * sbar);
        const double px = root_xyz[3 * r], py = root_xyz[3 * r + 1], pz = root_xyz[3 * r + 2];
        for (int n = 0; n < 4; ++n) {
            const double g = g_onset[4 * r + n];
            gt += g;
            const float4 q = xyz[v[n]];
            const double e[3] = {q.x - px, q.y - py, q.z - pz};
            double u[3];   // D^-1 e
            sym_apply(Di, e, u);
            const double h = sqrt(s2 * (e[0] * u[0] + e[1] * u[1] + e[2] * u[2]));
            if (!(h > 0.0) || g == 0.0) continue;
            for (int c = 0; c < 3; ++c) gx[c] -= g * s2 * u[c] / h;
            const double cf = -g * s2 / (2.0 * h);
            gD[0] += cf * u[0] * u[0];
            gD[1] += cf * u[1] * u[1];
            gD[2] += cf * u[2] * u[2];
            gD[3] += 2.0 * cf * u[0] * u[1];   // off-diagonals doubled
            gD[4] += 2.0 * cf * u[0] * u[2];
            gD[5] += 2.0 * cf * u[1] * u[2];
            gs += g * (-h / sbar);
        }
        if (dD)
            for (int c = 0; c < 6; ++c) atomicAdd(&dD[6 * (size_t)k + c], (float)gD[c]);
        if (dvs)
            for (int n = 0; n < 4; ++n) atomicAdd(&dvs[node_user[v[n]]], (float)(0.25 * gs));
    }
    if (dt) dt[r] = (float)gt;
    if (dx)
        for (int c = 0; c < 3; ++c) dx[3 * r + c] = (float)gx[c];
}

// Point location: each thread owns one element and tests the points of the
// current chunk (staged in LDS) against its barycentric coordinates; a hit
// lowers the point's answer to the element's caller id (the lowest containing
// id wins).
constexpr int kLocChunk = 1024;

__global__ void k_locate(const int4* __restrict__ tetv, const float4* __restrict__ xyz,
                         const int* __restrict__ tet_user, int n_e, const float* __restrict__ pts,
                         int n_pts, float tol, int* __restrict__ out) {
    __shared__ float sp[3 * kLocChunk];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const bool own = j < n_e;
    float v0x = 0.f, v0y = 0.f, v0z = 0.f;
    float a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // inverse of [v1-v0, v2-v0, v3-v0]
    bool valid = false;
    if (own) {
        const int4 t = tetv[j];
        const float4 p0 = xyz[t.x], p1 = xyz[t.y], p2 = xyz[t.z], p3 = xyz[t.w];
        v0x = p0.x;
        v0y = p0.y;
        v0z = p0.z;
        const float e00 = p1.x - p0.x, e10 = p1.y - p0.y, e20 = p1.z - p0.z;
        const float e01 = p2.x - p0.x, e11 = p2.y - p0.y, e21 = p2.z - p0.z;
        const float e02 = p3.x - p0.x, e12 = p3.y - p0.y, e22 = p3.z - p0.z;
        const float c00 = e11 * e22 - e12 * e21, c01 = e02 * e21 - e01 * e22,
                    c02 = e01 * e12 - e02 * e11;
        const float c10 = e12 * e20 - e10 * e22, c11 = e00 * e22 - e02 * e20,
                    c12 = e02 * e10 - e00 * e12;
        const float c20 = e10 * e21 - e11 * e20, c21 = e01 * e20 - e00 * e21,
                    c22 = e00 * e11 - e01 * e10;
        const float det = e00 * c00 + e01 * c10 + e02 * c20;
        valid = det != 0.f;
        const float id = valid ? 1.f / det : 0.f;
        a[0] = c00 * id; a[1] = c01 * id; a[2] = c02 * id;
        a[3] = c10 * id; a[4] = c11 * id; a[5] = c12 * id;
        a[6] = c20 * id; a[7] = c21 * id; a[8] = c22 * id;
    }
    const int me = own ? tet_user[j] : INT_MAX;
    for (int base = 0; base < n_pts; base += kLocChunk) {
        const int m = min(kLocChunk, n_pts - base);
        __syncthreads();
        for (int q = threadIdx.x; q < 3 * m; q += blockDim.x) sp[q] = pts[3 * (size_t)base + q];
        __syncthreads();
        if (!valid) continue;
        for (int q = 0; q < m; ++q) {
            const float dx = sp[3 * q] - v0x, dy = sp[3 * q + 1] - v0y, dz = sp[3 * q + 2] - v0z;
            const float l1 = a[0] * dx + a[1] * dy + a[2] * dz;
            const float l2 = a[3] * dx + a[4] * dy + a[5] * dz;
            const float l3 = a[6] * dx + a[7] * dy + a[8] * dz;
            const float l0 = 1.f - l1 - l2 - l3;
            if (l0 >= -tol && l1 >= -tol && l2 >= -tol && l3 >= -tol) atomicMin(&out[base + q], me);
        }
    }
}

__global__ void k_fill_int(int* __restrict__ p, int v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_unfound(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && p[i] == INT_MAX) p[i] = -1;
}

int check_points(gbp_plan p, const float* D, const int32_t* root_tet, const float* root_xyz,
                 int n_roots) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (n_roots < 0) {
        gbp_set_error("n_roots must be >= 0");
        return GBP_ERR_ARG;
    }
    if (n_roots > 0 && (!D || !root_tet || !root_xyz)) {
        gbp_set_error("D, root_tet and root_xyz are required");
        return GBP_ERR_ARG;
    }
    return GBP_OK;
}

}  // namespace

extern "C" int gbp_point_roots(gbp_plan p, const float* D, const float* vscale,
                               const int32_t* root_tet, const float* root_xyz, const float* root_t,
                               int n_roots, int32_t* node_out, float* t_out, void* stream) {
    int rc = check_points(p, D, root_tet, root_xyz, n_roots);
    if (rc) return rc;
    if (n_roots == 0) return GBP_OK;
    if (!root_t || !node_out || !t_out) {
        gbp_set_error("root_t, node_out and t_out are required");
        return GBP_ERR_ARG;
    }
    k_point_roots<<<gbp_blocks(n_roots, TPB), TPB, 0, (hipStream_t)stream>>>(
        root_tet, root_xyz, root_t, n_roots, p->tet_int, p->tetv, p->xyz, p->node_user, D, vscale,
        p->n_e, node_out, t_out);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_point_roots_backward(gbp_plan p, const float* D, const float* vscale,
                                        const int32_t* root_tet, const float* root_xyz,
                                        int n_roots, const float* dL_donset, float* dL_droot_t,
                                        float* dL_droot_xyz, float* dL_dD, float* dL_dvscale,
                                        void* stream) {
    int rc = check_points(p, D, root_tet, root_xyz, n_roots);
    if (rc) return rc;
    if (n_roots == 0) return GBP_OK;
    if (!dL_donset) {
        gbp_set_error("dL_donset is required");
        return GBP_ERR_ARG;
    }
    k_point_roots_bwd<<<gbp_blocks(n_roots, TPB), TPB, 0, (hipStream_t)stream>>>(
        root_tet, root_xyz, n_roots, p->tet_int, p->tetv, p->xyz, p->node_user, D, vscale, p->n_e,
        dL_donset, dL_droot_t, dL_droot_xyz, dL_dD, dL_dvscale);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_locate_points(gbp_plan p, const float* points, int n_points, float tol,
                                 int32_t* tet_out, void* stream) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (n_points < 0 || !(tol >= 0.f)) {
        gbp_set_error("n_points must be >= 0 and tol >= 0");
        return GBP_ERR_ARG;
    }
    if (n_points == 0) return GBP_OK;
    if (!points || !tet_out) {
        gbp_set_error("points and tet_out are required");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    k_fill_int<<<gbp_blocks(n_points, TPB), TPB, 0, s>>>(tet_out, INT_MAX, n_points);
    k_locate<<<gbp_blocks(p->n_e, TPB), TPB, 0, s>>>(p->tetv, p->xyz, p->tet_user, p->n_e, points,
                                                      n_points, tol, tet_out);
    k_unfound<<<gbp_blocks(n_points, TPB), TPB, 0, s>>>(tet_out, n_points);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}
