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

template <typename R>
struct LocalQT {
    R q00, q11, q22, q01, q02, q12;
};
using LocalQ = LocalQT<float>;

__device__ __forceinline__ float gbp_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double gbp_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float gbp_sqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double gbp_sqrt(double x) { return __builtin_sqrt(x); }
template <typename R>
__device__ __forceinline__ R gbp_inf() { return (R)__builtin_huge_val(); }

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

// Same, with the slot known only at run time (selects, no divergence).  With
// G4 the 4x4 Gram of (0, F1, F2, F3), the face opposite K uses the other three
// indices o0 < o1 < o2 and Q_ab = G4[oa][ob] - G4[oa][K] - G4[K][ob] + G4[K][K];
// column K of G4 vanishes at row 0, which removes most terms.
__device__ __forceinline__ LocalQ face_q_rt(const float4 g0, const float4 g1, int K) {
    const float G11 = g0.x, G22 = g0.y, G33 = g0.z, G12 = g0.w, G13 = g1.x, G23 = g1.y;
    const bool k0 = K == 0, k1 = K == 1, k2 = K == 2;
    const float d = k0 ? 0.f : k1 ? G11 : k2 ? G22 : G33;        // G4[K][K]
    const float c1 = k0 ? 0.f : k1 ? G12 : k2 ? G12 : G13;       // G4[o1][K]
    const float c2 = k0 ? 0.f : k1 ? G13 : k2 ? G23 : G23;       // G4[o2][K]
    const float g00 = k0 ? G11 : 0.f;                            // G4[o0][o0]
    const float g11 = (k0 || k1) ? G22 : G11;                    // G4[o1][o1]
    const float g22 = (K <= 2) ? G33 : G22;                      // G4[o2][o2]
    const float g01 = k0 ? G12 : 0.f;                            // G4[o0][o1]
    const float g02 = k0 ? G13 : 0.f;                            // G4[o0][o2]
    const float g12 = (k0 || k1) ? G23 : k2 ? G13 : G12;         // G4[o1][o2]
    LocalQ q;
    q.q00 = g00 + d;
    q.q11 = g11 - 2.f * c1 + d;
    q.q22 = g22 - 2.f * c2 + d;
    q.q01 = g01 - c1 + d;
    q.q02 = g02 - c2 + d;
    q.q12 = g12 - c1 - c2 + d;
    return q;
}

__device__ __forceinline__ void face_nodes_sel(const int4 v, int K, int& a, int& b, int& c) {
    a = (K == 0) ? v.y : v.x;
    b = (K <= 1) ? v.z : v.y;
    c = (K <= 2) ? v.w : v.z;
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
template <typename R>
__device__ __forceinline__ void edge_candidate(R qaa, R qbb, R qab, R Pa, R Pb, bool ok, R& val,
                                               R& ua, R& ub) {
    const R wa = qbb - qab, wb = qaa - qab;
    const R at = wa + wb;                           // |e_b - e_a|^2_M > 0
    const R inv = gbp_rcp(at);
    const R pbar = (wa * Pa + wb * Pb) * inv;
    const R d = Pb - Pa;
    const R det = qaa * qbb - qab * qab;
    const R rad = det * (at - d * d) * inv * inv;
    const R r = gbp_sqrt(rad > R(0) ? rad : R(0));
    const R pca = Pa - pbar, pcb = Pb - pbar;
    ua = r * wa - (qbb * pca - qab * pcb);
    ub = r * wb - (qaa * pcb - qab * pca);
    const bool feas = ok && (rad > R(0)) && (ua >= R(0)) && (ub >= R(0));
    val = feas ? pbar + r : gbp_inf<R>();
}

// Full local solve in precision R.  Returns the minimum (+inf if all three
// vertices are unreached).  With WANT_ALPHA also the minimiser's barycentric
// weights.  Candidate order (first wins on ties): vertices 0,1,2, edges 01,02,12,
// interior.
template <bool WANT_ALPHA, typename R = float>
__device__ __forceinline__ R local_min(const LocalQT<R> q, R p0, R p1, R p2, R* a0 = nullptr,
                                       R* a1 = nullptr, R* a2 = nullptr) {
    const R INF = gbp_inf<R>();
    const bool f0 = p0 < INF, f1 = p1 < INF, f2 = p2 < INF;
    const R m = fmin(fmin(p0, p1), p2);
    const R P0 = f0 ? p0 - m : R(0);
    const R P1 = f1 ? p1 - m : R(0);
    const R P2 = f2 ? p2 - m : R(0);

    // vertex candidates
    R best = f0 ? P0 + gbp_sqrt(q.q00) : INF;
    R b0 = 1, b1 = 0, b2 = 0;
    {
        const R v = f1 ? P1 + gbp_sqrt(q.q11) : INF;
        if (v < best) { best = v; if (WANT_ALPHA) { b0 = 0; b1 = 1; b2 = 0; } }
    }
    {
        const R v = f2 ? P2 + gbp_sqrt(q.q22) : INF;
        if (v < best) { best = v; if (WANT_ALPHA) { b0 = 0; b1 = 0; b2 = 1; } }
    }
    // edge candidates
    {
        R v, ua, ub;
        edge_candidate<R>(q.q00, q.q11, q.q01, P0, P1, f0 && f1, v, ua, ub);
        if (v < best) {
            best = v;
            if (WANT_ALPHA) { const R s = R(1) / (ua + ub); b0 = ua * s; b1 = ub * s; b2 = 0; }
        }
    }
    {
        R v, ua, ub;
        edge_candidate<R>(q.q00, q.q22, q.q02, P0, P2, f0 && f2, v, ua, ub);
        if (v < best) {
            best = v;
            if (WANT_ALPHA) { const R s = R(1) / (ua + ub); b0 = ua * s; b1 = 0; b2 = ub * s; }
        }
    }
    {
        R v, ua, ub;
        edge_candidate<R>(q.q11, q.q22, q.q12, P1, P2, f1 && f2, v, ua, ub);
        if (v < best) {
            best = v;
            if (WANT_ALPHA) { const R s = R(1) / (ua + ub); b0 = 0; b1 = ua * s; b2 = ub * s; }
        }
    }
    // interior candidate
    {
        const R A00 = q.q11 * q.q22 - q.q12 * q.q12;
        const R A11 = q.q00 * q.q22 - q.q02 * q.q02;
        const R A22 = q.q00 * q.q11 - q.q01 * q.q01;
        const R A01 = q.q02 * q.q12 - q.q01 * q.q22;
        const R A02 = q.q01 * q.q12 - q.q02 * q.q11;
        const R A12 = q.q01 * q.q02 - q.q00 * q.q12;
        const R det = q.q00 * A00 + q.q01 * A01 + q.q02 * A02;
        const R w0 = A00 + A01 + A02, w1 = A01 + A11 + A12, w2 = A02 + A12 + A22;
        const R at = w0 + w1 + w2;
        const R inv = gbp_rcp(at);
        const R pbar = (w0 * P0 + w1 * P1 + w2 * P2) * inv;
        const R c0 = P0 - pbar, c1 = P1 - pbar, c2 = P2 - pbar;
        const R y0 = A00 * c0 + A01 * c1 + A02 * c2;
        const R y1 = A01 * c0 + A11 * c1 + A12 * c2;
        const R y2 = A02 * c0 + A12 * c1 + A22 * c2;
        const R s = c0 * y0 + c1 * y1 + c2 * y2;
        const R rad = (det - s) * inv;
        const R r = gbp_sqrt(rad > R(0) ? rad : R(0));
        const R u0 = r * w0 - y0, u1 = r * w1 - y1, u2 = r * w2 - y2;
        const bool feas = f0 && f1 && f2 && (rad > R(0)) && (u0 >= R(0)) && (u1 >= R(0)) && (u2 >= R(0));
        const R v = feas ? pbar + r : INF;
        if (v < best) {
            best = v;
            if (WANT_ALPHA) { const R sc = R(1) / (u0 + u1 + u2); b0 = u0 * sc; b1 = u1 * sc; b2 = u2 * sc; }
        }
    }
    if (WANT_ALPHA) { *a0 = b0; *a1 = b1; *a2 = b2; }
    return (best < INF) ? m + best : INF;
}
