// FISTA on the local problem (Alg. 1, Sec. 2.2) -- the paper's own local solver,
// kept beside the exact predicated one of local_solve.h:
//
//   min over the simplex of  F(alpha) = <alpha, Phi> + h(alpha),  h = sqrt(alpha^T Q alpha)
//
// with step 1/L, L a Lipschitz constant of grad h on the simplex (Eq.
// (lipschitz_est)): L = lmax / h_ (1 + sqrt(lmax) / h_), lmax the largest
// eigenvalue of Q = A^T A and h_ a lower bound of h on the simplex -- either
// sigma_min(A) / (d sqrt d) (the bound of the equation) or the tightened
// h(alpha*_0) / 1.1 of Sec. 2.5, alpha*_0 the minimiser of h alone.
// Iteration k: alpha_k = proj(a_hat - (grad h(a_hat) + Phi) / L),
// a_hat <- alpha_k + (k-1)/(k+1) (alpha_k - alpha_{k-1}), from a_hat = 1/d.
// Unreached face vertices (+inf) get weight zero (the projection sends them to 0)
// and Phi is shifted by its finite minimum, which leaves every iterate unchanged
// (the projection commutes with adding a multiple of the ones vector).
#pragma once

#include "local_solve.h"

// Euclidean projection of y onto {a >= 0, sum a = 1} (sort of three values;
// entries at -inf end at 0).
__device__ __forceinline__ void simplex_proj3(float y0, float y1, float y2, float& a0, float& a1,
                                              float& a2) {
    float u0 = fmaxf(y0, y1), u1 = fminf(y0, y1);
    const float u2 = fminf(u1, y2);
    u1 = fmaxf(u1, y2);
    const float t = fmaxf(u0, u1);
    u1 = fminf(u0, u1);
    u0 = t;                                        // u0 >= u1 >= u2
    const float t1 = u0 - 1.f;
    const float t2 = 0.5f * (u0 + u1 - 1.f);
    const float t3 = (u0 + u1 + u2 - 1.f) * (1.f / 3.f);
    float theta = t1;
    if (u1 - t2 > 0.f) theta = t2;                 // false for u1 = -inf (NaN compares false)
    if (u1 - t2 > 0.f && u2 - t3 > 0.f) theta = t3;
    a0 = fmaxf(y0 - theta, 0.f);
    a1 = fmaxf(y1 - theta, 0.f);
    a2 = fmaxf(y2 - theta, 0.f);
}

// Iterations for a face with step constant L and value tolerance tau, from the
// rate Eq. (fista_convergence): 2 L ||alpha_0 - alpha*||^2 / (k+1)^2 <= tau with
// ||alpha_0 - alpha*||^2 <= 2/3 on the simplex (alpha_0 = 1/3), i.e. the least
// k with k + 1 >= sqrt(4 L / (3 tau)); at least 1, at most n_max (also for
// tau <= 0 or a non-finite bound).  Guaranteed with the bound of Eq.
// (lipschitz_est); with the tightened constant it is the same rule on a
// heuristic L.  FP32, rounded product then quotient then root.
__device__ __forceinline__ int fista_iters(float L, float tau, int n_max) {
    if (!(tau > 0.f)) return n_max;
    const float x = sqrtf(((4.0f / 3.0f) * L) / tau);
    if (!(x < (float)(n_max + 1))) return n_max;
    const int k = (int)ceilf(x) - 1;
    return k < 1 ? 1 : k;
}

// n_f FISTA iterations; returns F(alpha_{n_f}) (+inf if no vertex is reached),
// optionally alpha_{n_f}.
template <bool WANT_ALPHA>
__device__ __forceinline__ float local_fista(const LocalQ q, float p0, float p1, float p2, float L,
                                             int n_f, float* a0 = nullptr, float* a1 = nullptr,
                                             float* a2 = nullptr) {
    const float INF = GBP_INF;
    const bool f0 = p0 < INF, f1 = p1 < INF, f2 = p2 < INF;
    if (!(f0 || f1 || f2)) {
        if (WANT_ALPHA) { *a0 = 0.f; *a1 = 0.f; *a2 = 0.f; }
        return INF;
    }
    const float m = fminf(fminf(p0, p1), p2);
    const float il = 1.f / L;
    // Phi / L, +inf for unreached vertices: their gradient step lands at -inf
    // and the projection gives them weight zero
    const float s0 = f0 ? (p0 - m) * il : INF, s1 = f1 ? (p1 - m) * il : INF,
                s2 = f2 ? (p2 - m) * il : INF;
    float h0 = 1.f / 3.f, h1 = 1.f / 3.f, h2 = 1.f / 3.f;    // a_hat
    float k0 = h0, k1 = h1, k2 = h2;                          // alpha_{k-1}
    for (int k = 1; k <= n_f; ++k) {
        const float g0 = q.q00 * h0 + q.q01 * h1 + q.q02 * h2;
        const float g1 = q.q01 * h0 + q.q11 * h1 + q.q12 * h2;
        const float g2 = q.q02 * h0 + q.q12 * h1 + q.q22 * h2;
        const float ih = il * rsqrtf(h0 * g0 + h1 * g1 + h2 * g2);   // 1 / (L h)
        float n0, n1, n2;
        simplex_proj3(h0 - g0 * ih - s0, h1 - g1 * ih - s1, h2 - g2 * ih - s2, n0, n1, n2);
        const float beta = (float)(k - 1) / (float)(k + 1);
        h0 = n0 + beta * (n0 - k0);
        h1 = n1 + beta * (n1 - k1);
        h2 = n2 + beta * (n2 - k2);
        k0 = n0;
        k1 = n1;
        k2 = n2;
    }
    const float Qa0 = q.q00 * k0 + q.q01 * k1 + q.q02 * k2;
    const float Qa1 = q.q01 * k0 + q.q11 * k1 + q.q12 * k2;
    const float Qa2 = q.q02 * k0 + q.q12 * k1 + q.q22 * k2;
    const float lin = (f0 ? k0 * (p0 - m) : 0.f) + (f1 ? k1 * (p1 - m) : 0.f) +
                      (f2 ? k2 * (p2 - m) : 0.f);
    if (WANT_ALPHA) { *a0 = k0; *a1 = k1; *a2 = k2; }
    return m + lin + sqrtf(k0 * Qa0 + k1 * Qa1 + k2 * Qa2);
}

// Smallest and largest eigenvalue of a symmetric 3x3 (trigonometric closed form,
// FP64).
__device__ __forceinline__ void sym3_eig_minmax(double a, double b, double c, double d, double e,
                                                double f, double& lmin, double& lmax) {
    // matrix [[a d e] [d b f] [e f c]]
    const double p1 = d * d + e * e + f * f;
    const double tr = (a + b + c) / 3.0;
    const double p2 = (a - tr) * (a - tr) + (b - tr) * (b - tr) + (c - tr) * (c - tr) + 2.0 * p1;
    if (p2 <= 0.0) {
        lmin = lmax = tr;
        return;
    }
    const double p = sqrt(p2 / 6.0);
    const double ip = 1.0 / p;
    const double B00 = (a - tr) * ip, B11 = (b - tr) * ip, B22 = (c - tr) * ip;
    const double B01 = d * ip, B02 = e * ip, B12 = f * ip;
    const double detB = B00 * (B11 * B22 - B12 * B12) - B01 * (B01 * B22 - B12 * B02) +
                        B02 * (B01 * B12 - B11 * B02);
    double r = 0.5 * detB;
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    const double phi = acos(r) / 3.0;
    lmax = tr + 2.0 * p * cos(phi);
    lmin = tr + 2.0 * p * cos(phi + 2.0943951023931954923);   // + 2 pi / 3
}

// Step constant of Alg. 1 for one face.  mode 0: h_ = sqrt(lmin) / (3 sqrt 3)
// (Eq. (lipschitz_est), d = 3); mode 1: h_ = h(alpha*_0) / 1.1 (Sec. 2.5).
__device__ __forceinline__ float fista_lipschitz(const LocalQ q, int mode) {
    double lmin, lmax;
    sym3_eig_minmax(q.q00, q.q11, q.q22, q.q01, q.q02, q.q12, lmin, lmax);
    double hl;
    if (mode == 0) {
        hl = sqrt(lmin > 0.0 ? lmin : 0.0) / (3.0 * sqrt(3.0));
    } else {
        const LocalQT<double> qd{q.q00, q.q11, q.q22, q.q01, q.q02, q.q12};
        hl = local_min<false, double>(qd, 0.0, 0.0, 0.0) / 1.1;   // min of h over the simplex
    }
    return (float)(lmax / hl * (1.0 + sqrt(lmax) / hl));
}
