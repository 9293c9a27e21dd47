// Independent local problems (Sec. 2.2, Eq. (upwind_eq_lsqr)) solved in a batch
// with either local solver: the exact predicated KKT solve or n_f iterations of
// FISTA (Alg. 1).  Used to compare the two solvers face by face and to time them
// per local problem.
#include <cmath>

#include "fista.h"
#include "gbp_internal.h"

namespace {

constexpr int TPB = 256;

__global__ void k_local_batch(const float* __restrict__ Q6, const float* __restrict__ Phi, int n,
                              int solver, int n_f, const float* __restrict__ lip_in, int lmode,
                              float* __restrict__ value, float* __restrict__ alpha,
                              float* __restrict__ lip_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* q6 = Q6 + 6 * (size_t)i;
    const LocalQ q{q6[0], q6[1], q6[2], q6[3], q6[4], q6[5]};
    const float p0 = Phi[3 * (size_t)i], p1 = Phi[3 * (size_t)i + 1], p2 = Phi[3 * (size_t)i + 2];
    float a0, a1, a2, v;
    if (solver == 0) {
        v = local_min<true>(q, p0, p1, p2, &a0, &a1, &a2);
    } else {
        const float L = lip_in ? lip_in[i] : fista_lipschitz(q, lmode);
        if (lip_out) lip_out[i] = L;
        v = local_fista<true>(q, p0, p1, p2, L, n_f, &a0, &a1, &a2);
    }
    value[i] = v;
    if (alpha) {
        alpha[3 * (size_t)i] = a0;
        alpha[3 * (size_t)i + 1] = a1;
        alpha[3 * (size_t)i + 2] = a2;
    }
}

__global__ void k_fista_iters(const float* __restrict__ lip, int n, float tau, int n_max,
                              int* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = fista_iters(lip[i], tau, n_max);
}

}  // namespace

extern "C" int gbp_fista_iterations(const float* lip, int n, float tau, int n_max, int* n_f,
                                    void* stream) {
    if (n < 0 || n_max < 1 || n_max > 100000 || !(tau >= 0.f) || !std::isfinite(tau)) {
        gbp_set_error("fista_iterations: n >= 0, n_max 1..100000, tau finite and >= 0");
        return GBP_ERR_ARG;
    }
    if (n == 0) return GBP_OK;
    if (!lip || !n_f) {
        gbp_set_error("fista_iterations: lip and n_f are required");
        return GBP_ERR_ARG;
    }
    k_fista_iters<<<gbp_blocks(n, TPB), TPB, 0, (hipStream_t)stream>>>(lip, n, tau, n_max, n_f);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_local_solve(const float* Q6, const float* Phi, int n, int solver, int n_f,
                               const float* lip, int lipschitz_mode, float* value, float* alpha,
                               float* lip_out, void* stream) {
    if (n < 0 || (solver != 0 && solver != 1) || (solver == 1 && (n_f < 1 || n_f > 100000)) ||
        (lipschitz_mode != 0 && lipschitz_mode != 1)) {
        gbp_set_error("local_solve: n >= 0, solver 0 or 1, n_f 1..100000, lipschitz_mode 0 or 1");
        return GBP_ERR_ARG;
    }
    if (n == 0) return GBP_OK;
    if (!Q6 || !Phi || !value) {
        gbp_set_error("local_solve: Q6, Phi and value are required");
        return GBP_ERR_ARG;
    }
    k_local_batch<<<gbp_blocks(n, TPB), TPB, 0, (hipStream_t)stream>>>(
        Q6, Phi, n, solver, n_f, lip, lipschitz_mode, value, alpha, lip_out);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}
