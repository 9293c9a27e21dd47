/*
 * gbp_test_hooks.h -- entry points of libgbp that exist for tests only.  They
 * reach states that ordinary use meets rarely or never, so that the code paths
 * for those states can be tested.  Not part of the solver interface (gbp.h).
 */
#ifndef GBP_TEST_HOOKS_H
#define GBP_TEST_HOOKS_H

#include "gbp.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * gbp_plan_set_stamp_base -- sets the base of the forward's queue stamps (each
 * relaxation round marks queued vertices with the base plus its round index; the
 * base restarts from 1, clearing every mark, once it exceeds 2^30).  The restart
 * otherwise comes after some ten million solves on one plan.  Synchronises the
 * device.  Errors: GBP_ERR_ARG for stamp < 1, GBP_ERR_HIP.
 */
int gbp_plan_set_stamp_base(gbp_plan plan, int stamp);

#ifdef __cplusplus
}
#endif
#endif /* GBP_TEST_HOOKS_H */
