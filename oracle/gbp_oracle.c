/*
 * FP64 reference ("oracle") for the Geodesic-BP eikonal path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source, header, table or helper with the
 * HIP implementation.
 *
 * Contents (paper: Grandits et al., "Geodesic-BP", arXiv 2308.08410):
 *   orc_local_solve   exact minimum of the local Hopf-Lax problem over the face
 *                     simplex, Sec. 2.2 Eq. (upwind_eq_lsqr), by enumeration of
 *                     the KKT points of every face of the simplex;
 *   orc_fim           the global iteration of Alg. 2 (Jacobi over all
 *                     (element, vertex) pairs, optional change mask, scatter-min,
 *                     epsilon stop), plus a Gauss-Seidel variant and a two-sided
 *                     warm-start variant;
 *   orc_parent_map    the minimising element, barycentric weights and support of
 *                     every node at a fixed point (the geodesic "parents" along
 *                     which Sec. 2.3 back-propagates).
 *
 * Readings of the paper taken here (the paper is silent or garbled):
 *   - nodes whose first-sweep mask would be empty: the roots count as changed
 *     at k = 1 (phi_{-1} = +inf everywhere);
 *   - inf - inf in the mask / stop test: a value counts as changed iff
 *     new < old - eps(old), eps(x) = eps_abs + eps_rel*|x| (inf counts as old);
 *   - the vertex update keeps the old value: phi_k = min(phi_{k-1}, updates);
 *   - faces with infinite vertex values: the minimum is taken over the finite
 *     vertices only (alpha = 0 on the others); all-infinite faces give +inf;
 *   - parents: argmin over all incident (element, vertex) problems; among
 *     candidates within 1e-12*max(1,|T|) of the minimum the smallest element
 *     index wins; a root is its own parent when its onset time does not exceed
 *     the best upwind value.
 * Metric input: per element the packed inverse velocity tensor
 *   Minv = D_eff^{-1} as (xx, yy, zz, xy, xz, yz); the step cost is
 *   sqrt(e^T Minv e) (the paper's ||e||_D with its D = M^{-1}).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_INF (1.0 / 0.0)

/* Threads for the loops below that are independent per element or per node (1
 * unless a caller asks for more, e.g. to time the oracle on every host core).
 * Results do not depend on the count: the only shared update is the scatter-min
 * of Alg. 2, and a minimum does not depend on the order of its operands. */
static int orc_threads = 1;

int orc_set_threads(int n) {
#ifdef _OPENMP
    orc_threads = n < 1 ? 1 : n;
#else
    (void)n;
    orc_threads = 1;
#endif
    return orc_threads;
}

/* *addr = min(*addr, val), safe when several threads update one node */
static void orc_min_update(double *addr, double val) {
    unsigned long long *a = (unsigned long long *)addr;
    unsigned long long old = __atomic_load_n(a, __ATOMIC_RELAXED);
    for (;;) {
        double cur;
        memcpy(&cur, &old, sizeof cur);
        if (!(val < cur)) return;
        unsigned long long nv;
        memcpy(&nv, &val, sizeof nv);
        if (__atomic_compare_exchange_n(a, &old, nv, 0, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) return;
    }
}

/* ---- small dense linear algebra (Gaussian elimination, partial pivoting) */
static int orc_solve(int m, const double *A_in, const double *b_in, double *x) {
    double A[3][4];
    for (int r = 0; r < m; ++r) {
        for (int c = 0; c < m; ++c) A[r][c] = A_in[r * m + c];
        A[r][m] = b_in[r];
    }
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int c = 0; c <= m; ++c) {
                double t = A[col][c];
                A[col][c] = A[piv][c];
                A[piv][c] = t;
            }
        for (int r = 0; r < m; ++r) {
            if (r == col) continue;
            double f = A[r][col] / A[col][col];
            for (int c = col; c <= m; ++c) A[r][c] -= f * A[col][c];
        }
    }
    for (int r = 0; r < m; ++r) x[r] = A[r][m] / A[r][r];
    return 0;
}

/*
 * Local problem (Sec. 2.2, Eq. (upwind_eq_lsqr)) for one face with three
 * vertices:   min over alpha >= 0, sum(alpha) = 1  of  <alpha,Phi> + sqrt(alpha^T Q alpha)
 * with Q = E^T Minv E, E = [v_n - v_i] (the paper's A^T A).
 *
 * The problem is convex (Sec. 2.2), so its minimum is the smallest objective
 * value over the KKT points that are feasible.  On the face of the simplex
 * spanned by a support S (alpha_n = 0 off S), stationarity on the affine hull
 * reads Phi_S + Q_S alpha / h = mu 1 with h = sqrt(alpha^T Q_S alpha), which
 * gives (with a = 1^T Q_S^-1 1, b = 1^T Q_S^-1 Phi_S, c = Phi_S^T Q_S^-1 Phi_S)
 *     mu^2 a - 2 mu b + c = 1,  h = 1/(mu a - b) > 0,
 * hence mu = (b + sqrt(b^2 - a (c - 1))) / a, alpha_S = Q_S^-1 (mu 1 - Phi_S) h,
 * and the objective value at that point equals mu.  Support size 1 is the
 * edge path Phi_n + sqrt(Q_nn).  Phi is shifted by its minimum first (the
 * problem is shift-equivariant).  Ties: first candidate in the order
 * {0},{1},{2},{0,1},{0,2},{1,2},{0,1,2} wins.
 *
 * Returns the support bit mask (0 if every Phi is infinite: value = +inf).
 */
int orc_local_solve(const double *Q /*3x3 row-major*/, const double *Phi /*3*/,
                    double *value, double *alpha /*3*/) {
    static const int order[7] = {1, 2, 4, 3, 5, 6, 7};
    double shift = ORC_INF;
    for (int n = 0; n < 3; ++n)
        if (isfinite(Phi[n]) && Phi[n] < shift) shift = Phi[n];
    alpha[0] = alpha[1] = alpha[2] = 0.0;
    if (!isfinite(shift)) {
        *value = ORC_INF;
        return 0;
    }
    double P[3];
    for (int n = 0; n < 3; ++n) P[n] = Phi[n] - shift;

    double best = ORC_INF;
    int best_mask = 0;
    double best_alpha[3] = {0, 0, 0};
    for (int o = 0; o < 7; ++o) {
        int mask = order[o];
        int S[3], m = 0, ok = 1;
        for (int n = 0; n < 3; ++n)
            if (mask & (1 << n)) {
                if (!isfinite(Phi[n])) ok = 0;
                S[m++] = n;
            }
        if (!ok) continue;
        double cand, a_s[3] = {0, 0, 0};
        if (m == 1) {
            cand = P[S[0]] + sqrt(Q[S[0] * 3 + S[0]]);
            a_s[0] = 1.0;
        } else {
            double Qs[9], ones[3], Ps[3], y1[3], yP[3];
            for (int r = 0; r < m; ++r) {
                for (int c = 0; c < m; ++c) Qs[r * m + c] = Q[S[r] * 3 + S[c]];
                ones[r] = 1.0;
                Ps[r] = P[S[r]];
            }
            if (orc_solve(m, Qs, ones, y1) != 0 || orc_solve(m, Qs, Ps, yP) != 0) continue;
            double a = 0, b = 0, c = 0;
            for (int r = 0; r < m; ++r) {
                a += y1[r];
                b += yP[r];
                c += Ps[r] * yP[r];
            }
            double disc = b * b - a * (c - 1.0);
            if (!(disc > 0.0) || !(a > 0.0)) continue;
            double sd = sqrt(disc);
            double mu = (b + sd) / a;
            int feas = 1;
            for (int r = 0; r < m; ++r) {
                a_s[r] = (mu * y1[r] - yP[r]) / sd;
                if (a_s[r] < 0.0) feas = 0;
            }
            if (!feas) continue;
            cand = mu;
        }
        if (cand < best) {
            best = cand;
            best_mask = mask;
            best_alpha[0] = best_alpha[1] = best_alpha[2] = 0.0;
            for (int r = 0; r < m; ++r) best_alpha[S[r]] = a_s[r];
        }
    }
    if (best_mask == 0) {
        *value = ORC_INF;
        return 0;
    }
    /* renormalise the weights (they sum to one up to rounding) */
    double s = best_alpha[0] + best_alpha[1] + best_alpha[2];
    for (int n = 0; n < 3; ++n) alpha[n] = best_alpha[n] / s;
    *value = shift + best;
    return best_mask;
}

/* Q of the face opposite local vertex k of element j; the face vertices are
 * the other three local vertices in increasing local order.                */
static void orc_face(const double *xyz, const int *tet, const double *Minv6, int k,
                     double *Q, int *fv) {
    double M[3][3] = {{Minv6[0], Minv6[3], Minv6[4]},
                      {Minv6[3], Minv6[1], Minv6[5]},
                      {Minv6[4], Minv6[5], Minv6[2]}};
    double e[3][3];
    int m = 0;
    for (int n = 0; n < 4; ++n) {
        if (n == k) continue;
        fv[m] = tet[n];
        for (int d = 0; d < 3; ++d) e[m][d] = xyz[3 * tet[n] + d] - xyz[3 * tet[k] + d];
        ++m;
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) s += e[r][p] * M[p][q] * e[c][q];
            Q[r * 3 + c] = s;
        }
}

static double orc_eps(double x, double eps_abs, double eps_rel) {
    return eps_abs + eps_rel * (isfinite(x) ? fabs(x) : 0.0);
}

/* new < old - eps(old), NaN-free for infinite old values */
static int orc_changed(double newv, double oldv, double eps_abs, double eps_rel) {
    if (!isfinite(newv)) return 0;
    if (!isfinite(oldv)) return 1;
    return newv < oldv - orc_eps(oldv, eps_abs, eps_rel);
}

/*
 * Alg. 2: global Jacobi iteration over all (element, vertex) pairs.
 *   mode 0: Jacobi as written (Phi read from phi_{k-1}), with the change mask;
 *   mode 1: Gauss-Seidel (Phi read from the array being updated), with mask;
 *   mode 2: two-sided warm start from T (in/out): every node takes the min over
 *           all its faces (no min with its old value), roots also min with
 *           their onset; all nodes recomputed each sweep; stop when no node
 *           moves by more than eps.
 * T: in/out [n_v] (ignored on input for modes 0/1).
 * stats[0] sweeps, [1] local solves, [2] node value decreases,
 * [3] converged (1) or not (0), [4] node value increases (modes 0/1: 0).
 * Returns 0 on convergence, 1 if max_sweeps was reached.
 */
int orc_fim(int n_v, const double *xyz, int n_e, const int *tets, const double *Minv,
            int n_roots, const int *root_node, const double *root_t, double eps_abs,
            double eps_rel, int max_sweeps, int mode, double *T, long long *stats) {
    double *km2 = (double *)malloc(sizeof(double) * n_v); /* phi_{k-2} */
    double *km1 = (double *)malloc(sizeof(double) * n_v); /* phi_{k-1} */
    double *k0 = (double *)malloc(sizeof(double) * n_v);  /* phi_k     */
    double *troot = (double *)malloc(sizeof(double) * n_v);
    for (int i = 0; i < n_v; ++i) troot[i] = ORC_INF;
    for (int r = 0; r < n_roots; ++r)
        if (root_t[r] < troot[root_node[r]]) troot[root_node[r]] = root_t[r];
    long long solves = 0, decreases = 0, increases = 0;
    if (mode == 2) {
        for (int i = 0; i < n_v; ++i) {
            km1[i] = T[i];
            if (troot[i] < km1[i]) km1[i] = troot[i];
        }
    } else {
        for (int i = 0; i < n_v; ++i) {
            km2[i] = ORC_INF;
            km1[i] = troot[i];
        }
    }
    int k, converged = 0;
    for (k = 1; k <= max_sweeps; ++k) {
        if (mode == 2) {
            for (int i = 0; i < n_v; ++i) k0[i] = troot[i];
        } else {
            memcpy(k0, km1, sizeof(double) * n_v);
        }
        const double *src = (mode == 1) ? k0 : km1;
        /* Gauss-Seidel (mode 1) reads the array it writes: sequential */
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : solves) \
    num_threads(mode == 1 ? 1 : orc_threads)
        for (int j = 0; j < n_e; ++j) {
            const int *tet = tets + 4 * j;
            for (int kk = 0; kk < 4; ++kk) {
                double Q[9], Phi[3], a[3], val;
                int fv[3];
                int need = 1;
                if (mode != 2) {
                    need = 0;
                    for (int n = 0; n < 4; ++n)
                        if (n != kk && orc_changed(km1[tet[n]], km2[tet[n]], eps_abs, eps_rel))
                            need = 1;
                }
                if (!need) continue;
                orc_face(xyz, tet, Minv + 6 * j, kk, Q, fv);
                for (int n = 0; n < 3; ++n) Phi[n] = src[fv[n]];
                orc_local_solve(Q, Phi, &val, a);
                ++solves;
                orc_min_update(&k0[tet[kk]], val);
            }
        }
        int any = 0;
        for (int i = 0; i < n_v; ++i) {
            if (mode == 2) {
                double d = k0[i] - km1[i];
                int moved;
                if (isfinite(k0[i]) && isfinite(km1[i]))
                    moved = fabs(d) > orc_eps(km1[i], eps_abs, eps_rel);
                else
                    moved = (isfinite(k0[i]) != isfinite(km1[i]));
                if (moved) {
                    any = 1;
                    if (k0[i] < km1[i]) ++decreases; else ++increases;
                }
            } else {
                if (orc_changed(k0[i], km1[i], eps_abs, eps_rel)) any = 1;
                if (k0[i] < km1[i]) ++decreases;
            }
        }
        double *t = km2;
        km2 = km1;
        km1 = k0;
        k0 = t;
        if (!any) {
            converged = 1;
            break;
        }
    }
    memcpy(T, km1, sizeof(double) * n_v);
    if (stats) {
        stats[0] = converged ? k : max_sweeps;
        stats[1] = solves;
        stats[2] = decreases;
        stats[3] = converged;
        stats[4] = increases;
    }
    free(km2);
    free(km1);
    free(k0);
    free(troot);
    return converged ? 0 : 1;
}

/*
 * Geodesic parents at a fixed point T.  For every node i:
 *   best[i]    min over incident (element j, vertex i) problems,
 *   par_tet[i] minimising element (smallest index within 1e-12*max(1,|best|)),
 *              -1 for a root that is its own parent or an unreached node,
 *   par_node[3i..3i+2] the three face vertices of that element,
 *   par_alpha[3i..]    their barycentric weights (0 off the support),
 *   gap[i]     (second best value with a different weighted support) - best,
 *              +inf if no such candidate,
 *   root_self[i] 1 if i is a root whose onset <= best (own parent).
 */
int orc_parent_map(int n_v, const double *xyz, int n_e, const int *tets, const double *Minv,
                   int n_roots, const int *root_node, const double *root_t, const double *T,
                   int *par_tet, int *par_node, double *par_alpha, double *best, double *gap,
                   int *root_self) {
    double *troot = (double *)malloc(sizeof(double) * n_v);
    for (int i = 0; i < n_v; ++i) troot[i] = ORC_INF;
    for (int r = 0; r < n_roots; ++r)
        if (root_t[r] < troot[root_node[r]]) troot[root_node[r]] = root_t[r];
    /* incidence lists node -> (element, local vertex) */
    int *cnt = (int *)calloc(n_v + 1, sizeof(int));
    for (int j = 0; j < n_e; ++j)
        for (int k = 0; k < 4; ++k) cnt[tets[4 * j + k] + 1]++;
    for (int i = 0; i < n_v; ++i) cnt[i + 1] += cnt[i];
    int *fill = (int *)malloc(sizeof(int) * n_v);
    memcpy(fill, cnt, sizeof(int) * n_v);
    int *inc = (int *)malloc(sizeof(int) * 4 * (size_t)n_e);
    for (int j = 0; j < n_e; ++j)
        for (int k = 0; k < 4; ++k) inc[fill[tets[4 * j + k]]++] = 4 * j + k;

#pragma omp parallel for schedule(dynamic, 256) num_threads(orc_threads)
    for (int i = 0; i < n_v; ++i) {
        int nc = cnt[i + 1] - cnt[i];
        double *vals = (double *)malloc(sizeof(double) * (nc > 0 ? nc : 1));
        double *alps = (double *)malloc(sizeof(double) * 3 * (nc > 0 ? nc : 1));
        int *fvs = (int *)malloc(sizeof(int) * 3 * (nc > 0 ? nc : 1));
        int *tj = (int *)malloc(sizeof(int) * (nc > 0 ? nc : 1));
        double vmin = ORC_INF;
        for (int c = 0; c < nc; ++c) {
            int e = inc[cnt[i] + c];
            int j = e >> 2, k = e & 3;
            double Q[9], Phi[3];
            orc_face(xyz, tets + 4 * j, Minv + 6 * j, k, Q, fvs + 3 * c);
            for (int n = 0; n < 3; ++n) Phi[n] = T[fvs[3 * c + n]];
            orc_local_solve(Q, Phi, vals + c, alps + 3 * c);
            tj[c] = j;
            if (vals[c] < vmin) vmin = vals[c];
        }
        int bc = -1;
        double tol = 1e-12 * fmax(1.0, isfinite(vmin) ? fabs(vmin) : 0.0);
        for (int c = 0; c < nc; ++c)
            if (isfinite(vals[c]) && vals[c] <= vmin + tol && (bc < 0 || tj[c] < tj[bc])) bc = c;
        best[i] = vmin;
        gap[i] = ORC_INF;
        par_node[3 * i] = par_node[3 * i + 1] = par_node[3 * i + 2] = -1;
        par_alpha[3 * i] = par_alpha[3 * i + 1] = par_alpha[3 * i + 2] = 0.0;
        par_tet[i] = -1;
        root_self[i] = 0;
        if (isfinite(troot[i]) && troot[i] <= vmin) {
            root_self[i] = 1;
            /* gap: distance of the onset to the best upwind value */
            gap[i] = vmin - troot[i];
        } else if (bc >= 0) {
            par_tet[i] = tj[bc];
            for (int n = 0; n < 3; ++n) {
                par_node[3 * i + n] = fvs[3 * bc + n];
                par_alpha[3 * i + n] = alps[3 * bc + n];
            }
            /* second best among candidates whose weighted support differs */
            for (int c = 0; c < nc; ++c) {
                if (!isfinite(vals[c])) continue;
                int same = 1;
                for (int n = 0; n < 3 && same; ++n) {
                    /* weight on node fvs[3bc+n] in candidate c */
                    double wb = alps[3 * bc + n], wc = 0.0;
                    for (int q = 0; q < 3; ++q)
                        if (fvs[3 * c + q] == fvs[3 * bc + n]) wc = alps[3 * c + q];
                    if (fabs(wb - wc) > 1e-9) same = 0;
                }
                /* weights of c on nodes outside bc's face */
                for (int q = 0; q < 3 && same; ++q) {
                    int inface = 0;
                    for (int n = 0; n < 3; ++n)
                        if (fvs[3 * c + q] == fvs[3 * bc + n]) inface = 1;
                    if (!inface && alps[3 * c + q] > 1e-9) same = 0;
                }
                if (!same && vals[c] - vmin < gap[i]) gap[i] = vals[c] - vmin;
            }
            if (isfinite(troot[i]) && troot[i] - vmin < gap[i]) gap[i] = troot[i] - vmin;
        }
        free(vals);
        free(alps);
        free(fvs);
        free(tj);
    }
    free(troot);
    free(cnt);
    free(fill);
    free(inc);
    return 0;
}
