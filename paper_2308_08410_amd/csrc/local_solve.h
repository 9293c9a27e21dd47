// FP32 device solver of the local Hopf-Lax problem (Sec. 2.2, Eq. (upwind_eq_lsqr)):
//
//   phi*_{j\i} = min over alpha >= 0, sum(alpha) = 1 of  <alpha, Phi> + sqrt(alpha^T Q alpha)
//
// with Q = E^T M E, E = [v_n - v_i] the three edges from the target vertex v_i to
// the face vertices and M = D_eff^{-1} the element's inverse velocity tensor.
//
// The paper solves this with FISTA (Alg. 1) and names the closed form as the
// alternative (Sec. 2.5), rejecting it because of branching.  Here the closed form
// is evaluated branch-free: all seven KKT candidates (three vertices, three
// edges, the interior) are computed with predication and the smallest feasible
// one is selected, so a wavefront never diverges.
//
// Closed form on a support S with adjugate A = adj(Q_S), w = A 1, a~ = 1^T w:
//   Pbar = w.P / a~              (weighted mean; the problem is shift-equivariant)
//   Pc   = P - Pbar
//   r    = sqrt((det Q_S - Pc^T A Pc) / a~)        (exists iff the radicand > 0)
//   value = Pbar + r,   alpha ~ r w - A Pc          (feasible iff every entry >= 0)
// Phi is shifted by its finite minimum first; faces with +inf vertices use the
// finite vertices only.
#pragma once

#include <hip/hip_runtime.h>

#define GBP_INF __builtin_huge_valf()

struct LocalQ {
    float q00, q11, q22, q01, q02, q12;
};

// Element data: G = F^T M F with F_a = v_a - v_0 (a = 1..3), packed as
// g0 = (G11, G22, G33, G12), g1 = (G13, G23, sbar, 0).  Q of the face opposite
// local vertex K follows by linearity: edges from v_K are F_a - F_K.
template <int K>
__device__ __forceinline__ LocalQ face_q(const float4 g0, const float4 g1) {
    const float G11 = g0.x, G22 = g0.y, G33 = g0.z, G12 = g0.w, G13 = g1.x, G23 = g1.y;
    LocalQ q;
    if constexpr (K == 0) {          // face (v1, v2, v3)
        q.q00 = G11; q.q11 = G22; q.q22 = G33;
        q.q01 = G12; q.q02 = G13; q.q12 = G23;
    } else if constexpr (K == 1) {   // face (v0, v2, v3): edges -F1, F2-F1, F3-F1
        q.q00 = G11;
        q.q11 = G22 - 2.f * G12 + G11;
        q.q22 = G33 - 2.f * G13 + G11;
        q.q01 = G11 - G12;
        q.q02 = G11 - G13;
        q.q12 = G23 - G12 - G13 + G11;
    } else if constexpr (K == 2) {   // face (v0, v1, v3): edges -F2, F1-F2, F3-F2
        q.q00 = G22;
        q.q11 = G11 - 2.f * G12 + G22;
        q.q22 = G33 - 2.f * G23 + G22;
        q.q01 = G22 - G12;
        q.q02 = G22 - G23;
        q.q12 = G13 - G12 - G23 + G22;
    } else {                         // face (v0, v1, v2): edges -F3, F1-F3, F2-F3
        q.q00 = G33;
        q.q11 = G11 - 2.f * G13 + G33;
        q.q22 = G22 - 2.f * G23 + G33;
        q.q01 = G33 - G13;
        q.q02 = G33 - G23;
        q.q12 = G12 - G13 - G23 + G33;
    }
    return q;
}

// Face vertices of the face opposite local vertex K (in increasing local order).
template <int K>
__device__ __forceinline__ void face_nodes(const int4 v, int& a, int& b, int& c) {
    if constexpr (K == 0) { a = v.y; b = v.z; c = v.w; }
    else if constexpr (K == 1) { a = v.x; b = v.z; c = v.w; }
    else if constexpr (K == 2) { a = v.x; b = v.y; c = v.w; }
    else { a = v.x; b = v.y; c = v.z; }
}

template <int K>
__device__ __forceinline__ int face_target(const int4 v) {
    if constexpr (K == 0) return v.x;
    else if constexpr (K == 1) return v.y;
    else if constexpr (K == 2) return v.z;
    else return v.w;
}

// Two-vertex candidate on the edge (a, b) of the face.
__device__ __forceinline__ void edge_candidate(float qaa, float qbb, float qab, float Pa, float Pb,
                                               bool ok, float& val, float& ua, float& ub) {
    const float wa = qbb - qab, wb = qaa - qab;
    const float at = wa + wb;                       // |e_b - e_a|^2_M > 0
    const float inv = __builtin_amdgcn_rcpf(at);
    const float pbar = (wa * Pa + wb * Pb) * inv;
    const float d = Pb - Pa;
    const float det = qaa * qbb - qab * qab;
    const float rad = det * (at - d * d) * inv * inv;
    const float r = __builtin_sqrtf(fmaxf(rad, 0.f));
    const float pca = Pa - pbar, pcb = Pb - pbar;
    ua = r * wa - (qbb * pca - qab * pcb);
    ub = r * wb - (qaa * pcb - qab * pca);
    const bool feas = ok && (rad > 0.f) && (ua >= 0.f) && (ub >= 0.f);
    val = feas ? pbar + r : GBP_INF;
}

// Full local solve.  Returns the minimum (GBP_INF if all three vertices are
// unreached).  With WANT_ALPHA also the minimiser's barycentric weights.
template <bool WANT_ALPHA>
__device__ __forceinline__ float local_min(const LocalQ q, float p0, float p1, float p2,
                                           float* a0 = nullptr, float* a1 = nullptr,
                                           float* a2 = nullptr) {
    const bool f0 = p0 < GBP_INF, f1 = p1 < GBP_INF, f2 = p2 < GBP_INF;
    const float m = fminf(fminf(p0, p1), p2);
    const float P0 = f0 ? p0 - m : 0.f;
    const float P1 = f1 ? p1 - m : 0.f;
    const float P2 = f2 ? p2 - m : 0.f;

    // vertex candidates
    float best = f0 ? P0 + __builtin_sqrtf(q.q00) : GBP_INF;
    float b0 = 1.f, b1 = 0.f, b2 = 0.f;
    {
        const float v = f1 ? P1 + __builtin_sqrtf(q.q11) : GBP_INF;
        if (v < best) { best = v; if (WANT_ALPHA) { b0 = 0.f; b1 = 1.f; b2 = 0.f; } }
    }
    {
        const float v = f2 ? P2 + __builtin_sqrtf(q.q22) : GBP_INF;
        if (v < best) { best = v; if (WANT_ALPHA) { b0 = 0.f; b1 = 0.f; b2 = 1.f; } }
    }
    // edge candidates
    {
        float v, ua, ub;
        edge_candidate(q.q00, q.q11, q.q01, P0, P1, f0 && f1, v, ua, ub);
        if (v < best) {
            best = v;
            if (WANT_ALPHA) { const float s = 1.f / (ua + ub); b0 = ua * s; b1 = ub * s; b2 = 0.f; }
        }
    }
    {
        float v, ua, ub;
        edge_candidate(q.q00, q.q22, q.q02, P0, P2, f0 && f2, v, ua, ub);
        if (v < best) {
            best = v;
            if (WANT_ALPHA) { const float s = 1.f / (ua + ub); b0 = ua * s; b1 = 0.f; b2 = ub * s; }
        }
    }
    {
        float v, ua, ub;
        edge_candidate(q.q11, q.q22, q.q12, P1, P2, f1 && f2, v, ua, ub);
        if (v < best) {
            best = v;
            if (WANT_ALPHA) { const float s = 1.f / (ua + ub); b0 = 0.f; b1 = ua * s; b2 = ub * s; }
        }
    }
    // interior candidate
    {
        const float A00 = q.q11 * q.q22 - q.q12 * q.q12;
        const float A11 = q.q00 * q.q22 - q.q02 * q.q02;
        const float A22 = q.q00 * q.q11 - q.q01 * q.q01;
        const float A01 = q.q02 * q.q12 - q.q01 * q.q22;
        const float A02 = q.q01 * q.q12 - q.q02 * q.q11;
        const float A12 = q.q01 * q.q02 - q.q00 * q.q12;
        const float det = q.q00 * A00 + q.q01 * A01 + q.q02 * A02;
        const float w0 = A00 + A01 + A02, w1 = A01 + A11 + A12, w2 = A02 + A12 + A22;
        const float at = w0 + w1 + w2;
        const float inv = __builtin_amdgcn_rcpf(at);
        const float pbar = (w0 * P0 + w1 * P1 + w2 * P2) * inv;
        const float c0 = P0 - pbar, c1 = P1 - pbar, c2 = P2 - pbar;
        const float y0 = A00 * c0 + A01 * c1 + A02 * c2;
        const float y1 = A01 * c0 + A11 * c1 + A12 * c2;
        const float y2 = A02 * c0 + A12 * c1 + A22 * c2;
        const float s = c0 * y0 + c1 * y1 + c2 * y2;
        const float rad = (det - s) * inv;
        const float r = __builtin_sqrtf(fmaxf(rad, 0.f));
        const float u0 = r * w0 - y0, u1 = r * w1 - y1, u2 = r * w2 - y2;
        const bool feas = f0 && f1 && f2 && (rad > 0.f) && (u0 >= 0.f) && (u1 >= 0.f) && (u2 >= 0.f);
        const float v = feas ? pbar + r : GBP_INF;
        if (v < best) {
            best = v;
            if (WANT_ALPHA) { const float sc = 1.f / (u0 + u1 + u2); b0 = u0 * sc; b1 = u1 * sc; b2 = u2 * sc; }
        }
    }
    if (WANT_ALPHA) { *a0 = b0; *a1 = b1; *a2 = b2; }
    return (best < GBP_INF) ? m + best : GBP_INF;
}
