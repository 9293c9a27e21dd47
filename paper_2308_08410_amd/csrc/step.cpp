// One Geodesic-BP iteration recorded into a HIP graph and replayed.
//
// The forward and adjoint run with fixed launch budgets (empty rounds and levels
// return at once), every clear is a kernel (no memset nodes), the queue stamp
// base and the Adam step counter live in device memory, and all scratch is
// allocated before capture; so the graph is static and replays are independent.
#include <cstring>

#include "gbp_internal.h"

struct gbp_step_s {
    gbp_step_desc d{};
    int n_v = 0, n_inst = 0, S = 0;
    float *G = nullptr, *gT = nullptr, *dvs = nullptr, *drt = nullptr;
    float *m_vs = nullptr, *v_vs = nullptr, *m_rt = nullptr, *v_rt = nullptr;
    int* counter = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void step_free(gbp_step st) {
    if (!st) return;
    if (st->exec) (void)hipGraphExecDestroy(st->exec);
    if (st->graph) (void)hipGraphDestroy(st->graph);
    if (st->cap) (void)hipStreamDestroy(st->cap);
    void* ptrs[] = {st->G, st->gT, st->dvs, st->drt, st->m_vs, st->v_vs, st->m_rt, st->v_rt,
                    st->counter};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete st;
}

extern "C" void gbp_step_destroy(gbp_step st) { step_free(st); }

static int record(gbp_step st) {
    const gbp_step_desc& d = st->d;
    hipStream_t s = st->cap;
    int rc;
    if ((rc = gbp_forward_impl(d.plan, d.D, d.vscale, d.root_node, d.root_t, d.n_roots,
                               d.warm ? d.T : nullptr, d.T, nullptr, s, d.round_budget)))
        return rc;
    if ((rc = gbp_ecg_forward_batched(d.batch, d.T, d.W, d.L, &d.ap, d.ecg, s))) return rc;
    if ((rc = gbp_ecg_loss_batched(d.ecg, d.target, st->n_inst, st->S * d.L, d.loss, st->G, s)))
        return rc;
    if ((rc = gbp_ecg_backward_batched(d.batch, d.T, d.W, d.L, &d.ap, st->G, st->gT, s))) return rc;
    if ((rc = gbp_backward_impl(d.plan, d.D, d.vscale, d.root_node, d.root_t, d.n_roots, d.T, st->gT,
                                nullptr, st->dvs, st->drt, s, d.level_budget, d.gs_budget)))
        return rc;
    if ((rc = gbp_adam_step_dev(d.vscale, st->dvs, st->m_vs, st->v_vs, st->n_v, d.lr_vscale, 0.9f,
                                0.999f, 1e-8f, st->counter, d.vscale_lo, d.vscale_hi, s)))
        return rc;
    if (d.n_roots > 0 &&
        (rc = gbp_adam_step_dev(d.root_t, st->drt, st->m_rt, st->v_rt, d.n_roots, d.lr_root_t, 0.9f,
                                0.999f, 1e-8f, st->counter, 0.f, 0.f, s)))
        return rc;
    return gbp_counter_add(st->counter, 1, s);
}

extern "C" int gbp_step_create(const gbp_step_desc* desc, gbp_step* out) {
    if (!desc || !out) {
        gbp_set_error("step: NULL argument");
        return GBP_ERR_ARG;
    }
    *out = nullptr;
    const gbp_step_desc& d = *desc;
    int rc = gbp_plan_check(d.plan);
    if (rc) return rc;
    for (int k = 0; k < 4; ++k)
        if (d.reserved[k]) {
            gbp_set_error("step: reserved fields must be zero");
            return GBP_ERR_ARG;
        }
    int n_v = 0, n_inst = 0;
    gbp_plan_sizes(d.plan, &n_v, nullptr);
    if (!d.batch || !d.D || !d.vscale || !d.W || !d.target || !d.T || !d.ecg || !d.loss ||
        d.n_roots < 0 || (d.n_roots > 0 && (!d.root_node || !d.root_t)) || d.round_budget < 1 ||
        d.level_budget < 1 || d.gs_budget < 0 || d.L < 1 || d.L > 256) {
        gbp_set_error("step: missing buffer or bad budget/size");
        return GBP_ERR_ARG;
    }
    if ((rc = gbp_batch_sizes(d.batch, &n_inst, nullptr))) return rc;
    gbp_step st = new gbp_step_s();
    st->d = d;
    st->n_v = n_v;
    st->n_inst = n_inst;
    st->S = d.ap.n_steps;
    const size_t ne = (size_t)n_inst * st->S * d.L;
    const int R = std::max(d.n_roots, 1);
    if (hipMalloc((void**)&st->G, ne * sizeof(float)) || hipMalloc((void**)&st->gT, n_v * sizeof(float)) ||
        hipMalloc((void**)&st->dvs, n_v * sizeof(float)) || hipMalloc((void**)&st->drt, R * sizeof(float)) ||
        hipMalloc((void**)&st->m_vs, n_v * sizeof(float)) || hipMalloc((void**)&st->v_vs, n_v * sizeof(float)) ||
        hipMalloc((void**)&st->m_rt, R * sizeof(float)) || hipMalloc((void**)&st->v_rt, R * sizeof(float)) ||
        hipMalloc((void**)&st->counter, sizeof(int))) {
        gbp_set_error("step: allocation failed");
        step_free(st);
        return GBP_ERR_NOMEM;
    }
    const int one = 1;
    if (hipMemset(st->m_vs, 0, n_v * sizeof(float)) || hipMemset(st->v_vs, 0, n_v * sizeof(float)) ||
        hipMemset(st->m_rt, 0, R * sizeof(float)) || hipMemset(st->v_rt, 0, R * sizeof(float)) ||
        hipMemcpy(st->counter, &one, sizeof(int), hipMemcpyHostToDevice)) {
        gbp_set_error("step: initialisation failed");
        step_free(st);
        return GBP_ERR_HIP;
    }
    if ((rc = gbp_alloc_backward(d.plan))) {
        step_free(st);
        return rc;
    }
    if (hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking) != hipSuccess) {
        gbp_set_error("step: stream creation failed");
        step_free(st);
        return GBP_ERR_HIP;
    }
    if (hipStreamBeginCapture(st->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        gbp_set_error("step: hipStreamBeginCapture failed");
        step_free(st);
        return GBP_ERR_HIP;
    }
    rc = record(st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st->cap, &g);
    st->graph = g;
    if (rc) {
        step_free(st);
        return rc;
    }
    if (e != hipSuccess || !g) {
        gbp_set_error("step: capture failed: %s", hipGetErrorString(e));
        step_free(st);
        return GBP_ERR_HIP;
    }
    if (hipGraphInstantiate(&st->exec, st->graph, nullptr, nullptr, 0) != hipSuccess) {
        gbp_set_error("step: hipGraphInstantiate failed");
        step_free(st);
        return GBP_ERR_HIP;
    }
    *out = st;
    return GBP_OK;
}

extern "C" int gbp_step_gradients(gbp_step st, float* dL_dT, float* dL_dvscale, float* dL_droot_t,
                                  void* stream) {
    if (!st || !st->exec) {
        gbp_set_error("step: not created");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    if (dL_dT) GBP_HIP(hipMemcpyAsync(dL_dT, st->gT, st->n_v * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (dL_dvscale)
        GBP_HIP(hipMemcpyAsync(dL_dvscale, st->dvs, st->n_v * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (dL_droot_t && st->d.n_roots > 0)
        GBP_HIP(hipMemcpyAsync(dL_droot_t, st->drt, st->d.n_roots * sizeof(float), hipMemcpyDeviceToDevice,
                               s));
    return GBP_OK;
}

extern "C" int gbp_step_get_state(gbp_step st, float* m_vscale, float* v_vscale, float* m_root_t,
                                  float* v_root_t, int* counter, void* stream) {
    if (!st || !st->exec || !m_vscale || !v_vscale || !counter ||
        (st->d.n_roots > 0 && (!m_root_t || !v_root_t))) {
        gbp_set_error("step_get_state: NULL argument");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t nv = st->n_v * sizeof(float), nr = st->d.n_roots * sizeof(float);
    GBP_HIP(hipMemcpyAsync(m_vscale, st->m_vs, nv, hipMemcpyDeviceToDevice, s));
    GBP_HIP(hipMemcpyAsync(v_vscale, st->v_vs, nv, hipMemcpyDeviceToDevice, s));
    if (nr) {
        GBP_HIP(hipMemcpyAsync(m_root_t, st->m_rt, nr, hipMemcpyDeviceToDevice, s));
        GBP_HIP(hipMemcpyAsync(v_root_t, st->v_rt, nr, hipMemcpyDeviceToDevice, s));
    }
    GBP_HIP(hipMemcpyAsync(counter, st->counter, sizeof(int), hipMemcpyDeviceToHost, s));
    GBP_HIP(hipStreamSynchronize(s));
    return GBP_OK;
}

extern "C" int gbp_step_set_state(gbp_step st, const float* m_vscale, const float* v_vscale,
                                  const float* m_root_t, const float* v_root_t, int counter,
                                  void* stream) {
    if (!st || !st->exec || !m_vscale || !v_vscale || counter < 1 ||
        (st->d.n_roots > 0 && (!m_root_t || !v_root_t))) {
        gbp_set_error("step_set_state: NULL argument or counter < 1");
        return GBP_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t nv = st->n_v * sizeof(float), nr = st->d.n_roots * sizeof(float);
    GBP_HIP(hipMemcpyAsync(st->m_vs, m_vscale, nv, hipMemcpyDeviceToDevice, s));
    GBP_HIP(hipMemcpyAsync(st->v_vs, v_vscale, nv, hipMemcpyDeviceToDevice, s));
    if (nr) {
        GBP_HIP(hipMemcpyAsync(st->m_rt, m_root_t, nr, hipMemcpyDeviceToDevice, s));
        GBP_HIP(hipMemcpyAsync(st->v_rt, v_root_t, nr, hipMemcpyDeviceToDevice, s));
    }
    GBP_HIP(hipMemcpyAsync(st->counter, &counter, sizeof(int), hipMemcpyHostToDevice, s));
    GBP_HIP(hipStreamSynchronize(s));
    return GBP_OK;
}

extern "C" int gbp_step_launch(gbp_step st, void* stream) {
    if (!st || !st->exec) {
        gbp_set_error("step: not created");
        return GBP_ERR_ARG;
    }
    GBP_HIP(hipGraphLaunch(st->exec, (hipStream_t)stream));
    return GBP_OK;
}
