// Kernel timing scopes (see gbp_profile_enable in gbp.h).
#pragma once
#include <hip/hip_runtime.h>

enum {
    GBP_PROF_METRIC = 0,
    GBP_PROF_FIM_SWEEP,
    GBP_PROF_PARENT,
    GBP_PROF_CHILD,
    GBP_PROF_ADJ_LEVEL,
    GBP_PROF_GRAD,
    GBP_PROF_ECG_FWD,
    GBP_PROF_ECG_BWD,
    GBP_PROF_AUX,
    GBP_PROF_NKERNELS
};

// Records HIP events around the enclosed launches when profiling is on.
class ProfScope {
  public:
    ProfScope(int id, hipStream_t s);
    ~ProfScope();

  private:
    int id_;
    hipStream_t s_;
    void* a_ = nullptr;
};
