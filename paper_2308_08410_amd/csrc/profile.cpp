// Optional per-kernel timing with HIP events recorded on the launching stream.
#include <mutex>
#include <vector>

#include "gbp_internal.h"
#include "profile.h"

namespace {
struct Rec {
    int id;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_pending;
std::vector<hipEvent_t> g_pool;
double g_ms[GBP_PROF_NKERNELS];
long long g_n[GBP_PROF_NKERNELS];
const char* g_names[GBP_PROF_NKERNELS] = {"metric", "fim_sweep", "parent", "child_lists",
                                          "adj_level", "grad", "ecg_fwd", "ecg_bwd", "aux"};

hipEvent_t take() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void drain_locked() {
    for (Rec& r : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_ms[r.id] += ms;
            g_n[r.id] += 1;
        }
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_pending.clear();
}
}  // namespace

ProfScope::ProfScope(int id, hipStream_t s) : id_(id), s_(s) {
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    a_ = take();
    if (a_) (void)hipEventRecord((hipEvent_t)a_, s_);
}

ProfScope::~ProfScope() {
    if (!a_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take();
    if (!b) return;
    (void)hipEventRecord(b, s_);
    g_pending.push_back(Rec{id_, (hipEvent_t)a_, b});
    if (g_pending.size() > 4096) drain_locked();
}

extern "C" int gbp_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return GBP_OK;
}

extern "C" void gbp_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    drain_locked();
    for (int k = 0; k < GBP_PROF_NKERNELS; ++k) {
        g_ms[k] = 0;
        g_n[k] = 0;
    }
}

extern "C" int gbp_profile_read(const char* kernel, int64_t* launches, double* total_ms) {
    std::lock_guard<std::mutex> lk(g_mu);
    drain_locked();
    for (int k = 0; k < GBP_PROF_NKERNELS; ++k)
        if (kernel && std::string(kernel) == g_names[k]) {
            if (launches) *launches = g_n[k];
            if (total_ms) *total_ms = g_ms[k];
            return GBP_OK;
        }
    gbp_set_error("unknown kernel name for profiling");
    return GBP_ERR_ARG;
}
