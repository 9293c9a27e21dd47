// Lead weights on the device (Sec. 2.4): B = K Z with K the P1 stiffness of the
// plan's mesh (unit conductivity) and Z[n, l] = 1 / |x_n - e_l| the lead field of
// a point electrode, so that electrodes can move without a host assembly.
//
// One thread per vertex gathers its row of K Z over the elements around it (the
// incidence lists of the plan): for each element it forms the barycentric
// gradients (inverse of the edge matrix), its row of the element stiffness
// |E| grad l_k . grad l_m, and adds K_km Z_l(x_m) for a chunk of leads.  FP64
// throughout: B is a sum of terms of both signs that nearly cancel away from the
// boundary.  Deterministic (fixed order, no atomics).
#include "gbp_internal.h"

namespace {

constexpr int TPB = 256;
constexpr int kChunk = 8;          // leads per pass over a vertex's elements
constexpr int kMaxLeads = 256;

__global__ void __launch_bounds__(TPB)
    k_lead_field(const int2* __restrict__ nptr, const int* __restrict__ nent,
                 const int4* __restrict__ tetv, const float4* __restrict__ xyz,
                 const int* __restrict__ node_user, int n_v, const float* __restrict__ elec,
                 int L, float* __restrict__ W) {
    __shared__ double se[3 * kMaxLeads];
    for (int q = threadIdx.x; q < 3 * L; q += blockDim.x) se[q] = elec[q];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_v) return;
    const int2 p = nptr[i];
    const int cnt[4] = {p.y & 255, (p.y >> 8) & 255, (p.y >> 16) & 255, (p.y >> 24) & 255};
    const int u = node_user[i];
    for (int l0 = 0; l0 < L; l0 += kChunk) {
        double acc[kChunk];
#pragma unroll
        for (int c = 0; c < kChunk; ++c) acc[c] = 0.0;
        int e = p.x;
        for (int k = 0; k < 4; ++k) {              // this vertex is local vertex k
            for (int c = 0; c < cnt[k]; ++c, ++e) {
                const int4 v = tetv[nent[e]];
                const int vid[4] = {v.x, v.y, v.z, v.w};
                double X[4][3];
                for (int m = 0; m < 4; ++m) {
                    const float4 q = xyz[vid[m]];
                    X[m][0] = q.x;
                    X[m][1] = q.y;
                    X[m][2] = q.z;
                }
                // edge matrix rows E_a = X_a - X_0 (a = 1..3); gradients of l_1..l_3
                // are the columns of E^-1, grad l_0 = -(sum of the others)
                const double a = X[1][0] - X[0][0], b = X[1][1] - X[0][1], cc = X[1][2] - X[0][2];
                const double d = X[2][0] - X[0][0], f = X[2][1] - X[0][1], g = X[2][2] - X[0][2];
                const double h = X[3][0] - X[0][0], s = X[3][1] - X[0][1], t = X[3][2] - X[0][2];
                const double A00 = f * t - g * s, A01 = cc * s - b * t, A02 = b * g - cc * f;
                const double A10 = g * h - d * t, A11 = a * t - cc * h, A12 = cc * d - a * g;
                const double A20 = d * s - f * h, A21 = b * h - a * s, A22 = a * f - b * d;
                const double det = a * A00 + b * A10 + cc * A20;
                const double id = 1.0 / det;
                double G[4][3];
                G[1][0] = A00 * id; G[1][1] = A10 * id; G[1][2] = A20 * id;   // column 0 of E^-1
                G[2][0] = A01 * id; G[2][1] = A11 * id; G[2][2] = A21 * id;
                G[3][0] = A02 * id; G[3][1] = A12 * id; G[3][2] = A22 * id;
                for (int z = 0; z < 3; ++z) G[0][z] = -(G[1][z] + G[2][z] + G[3][z]);
                const double vol = fabs(det) / 6.0;
                for (int m = 0; m < 4; ++m) {
                    const double km = vol * (G[k][0] * G[m][0] + G[k][1] * G[m][1] + G[k][2] * G[m][2]);
#pragma unroll
                    for (int c = 0; c < kChunk; ++c) {
                        const int l = l0 + c;
                        if (l < L) {
                            const double dx = X[m][0] - se[3 * l], dy = X[m][1] - se[3 * l + 1],
                                         dz = X[m][2] - se[3 * l + 2];
                            acc[c] += km / sqrt(dx * dx + dy * dy + dz * dz);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kChunk; ++c)
            if (l0 + c < L) W[(size_t)u * L + l0 + c] = (float)acc[c];
    }
}

}  // namespace

extern "C" int gbp_lead_field(gbp_plan p, const float* electrodes, int n_leads, float* W,
                              void* stream) {
    int rc = gbp_plan_check(p);
    if (rc) return rc;
    if (n_leads < 1 || n_leads > kMaxLeads || !electrodes || !W) {
        gbp_set_error("lead_field: 1 <= n_leads <= %d, electrodes and W required", kMaxLeads);
        return GBP_ERR_ARG;
    }
    k_lead_field<<<gbp_blocks(p->n_v, TPB), TPB, 0, (hipStream_t)stream>>>(
        p->nptr, p->nent, p->tetv, p->xyz, p->node_user, p->n_v, electrodes, n_leads, W);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}
