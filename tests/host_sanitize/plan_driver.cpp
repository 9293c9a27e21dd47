// Drives the plan builder's host code (argument checks, element validation,
// Morton reordering, incidence and neighbour lists, settings and their bounds,
// clean-up after every allocation failure) under the sanitizers.  Prints one
// line per case and exits non-zero on the first unexpected return code; the
// sanitizers abort on a memory or undefined-behaviour error, and the leak checker
// reports anything a failed or destroyed plan did not free.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "gbp.h"
#include "gbp_internal.h"   // the plan's arrays are host memory under the stand-ins

extern "C" void stub_fail_after(int n);
extern "C" int stub_allocations(void);

namespace {
int failures = 0;

void expect(const char* what, int got, int want) {
    std::printf("%-58s rc %3d (want %3d)%s\n", what, got, want, got == want ? "" : "  <-- FAIL");
    if (got != want) ++failures;
}

// Kuhn subdivision of an n^3 grid of unit cubes: 6 elements per cube.
void kuhn_cube(int n, std::vector<float>& xyz, std::vector<int32_t>& tets) {
    const int m = n + 1;
    auto id = [m](int i, int j, int k) { return i + m * (j + m * k); };
    for (int k = 0; k < m; ++k)
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) {
                xyz.push_back((float)i / n);
                xyz.push_back((float)j / n);
                xyz.push_back((float)k / n);
            }
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                for (const auto& p : perm) {
                    int c[3] = {i, j, k};
                    tets.push_back(id(c[0], c[1], c[2]));
                    for (int s = 0; s < 3; ++s) {
                        ++c[p[s]];
                        tets.push_back(id(c[0], c[1], c[2]));
                    }
                }
}
}  // namespace

int main() {
    std::vector<float> xyz;
    std::vector<int32_t> tets;
    kuhn_cube(5, xyz, tets);
    const int n_v = (int)xyz.size() / 3, n_e = (int)tets.size() / 4;
    gbp_plan p = nullptr;

    // a valid plan and its settings
    expect("valid Kuhn cube", gbp_plan_create(xyz.data(), n_v, tets.data(), n_e, nullptr, &p), GBP_OK);
    if (!p) return 1;
    int a = 0, b = 0, c = 0, d = 0;
    float f = 0.f;
    expect("sizes", gbp_plan_sizes(p, &a, &b), GBP_OK);
    expect("sizes match", (a == n_v && b == n_e) ? 0 : 1, 0);
    expect("launch 16/1024/2048/16", gbp_plan_set_launch(p, 16, 1024, 2048, 16), GBP_OK);
    expect("launch lanes 12 refused", gbp_plan_set_launch(p, 12, 1024, 2048, 16), GBP_ERR_ARG);
    expect("launch blocks 0 refused", gbp_plan_set_launch(p, 16, 0, 2048, 16), GBP_ERR_ARG);
    expect("get launch", gbp_plan_get_launch(p, &a, &b, &c, &d), GBP_OK);
    expect("hold 1.0/2/0", gbp_plan_set_hold(p, 1.0f, 2, 0), GBP_OK);
    expect("hold again (lists kept)", gbp_plan_set_hold(p, 0.5f, 0, 100), GBP_OK);
    expect("hold negative refused", gbp_plan_set_hold(p, -1.0f, 0, 0), GBP_ERR_ARG);
    expect("hold NaN refused", gbp_plan_set_hold(p, NAN, 0, 0), GBP_ERR_ARG);
    expect("hold window 33 refused", gbp_plan_set_hold(p, 1.0f, 33, 0), GBP_ERR_ARG);
    expect("get hold", gbp_plan_get_hold(p, &f, &a, &b), GBP_OK);
    expect("warm order on", gbp_plan_set_warm_order(p, 1), GBP_OK);
    expect("warm order 2 refused", gbp_plan_set_warm_order(p, 2), GBP_ERR_ARG);
    expect("get warm order", gbp_plan_get_warm_order(p, &a), GBP_OK);
    expect("queue split off", gbp_plan_set_queue_split(p, 0), GBP_OK);
    expect("get queue split", gbp_plan_get_queue_split(p, &a), GBP_OK);
    expect("local solver FISTA 32", gbp_plan_set_local_solver(p, 1, 32, 1), GBP_OK);
    expect("local solver 3 refused", gbp_plan_set_local_solver(p, 3, 32, 1), GBP_ERR_ARG);
    expect("fista tolerance", gbp_plan_set_fista_tolerance(p, 1e-3f), GBP_OK);
    expect("fista tolerance NaN refused", gbp_plan_set_fista_tolerance(p, NAN), GBP_ERR_ARG);
    expect("input reuse", gbp_plan_set_input_reuse(p, 1), GBP_OK);
    expect("last counts", gbp_plan_last_counts(p, &a, &b), GBP_OK);
    gbp_plan_destroy(p);
    p = nullptr;
    gbp_plan_destroy(nullptr);

    // caller order kept, and a plan with options
    gbp_options o{};
    o.reorder = -1;
    o.eps_rel = 1e-6f;
    expect("reorder off", gbp_plan_create(xyz.data(), n_v, tets.data(), n_e, &o, &p), GBP_OK);
    gbp_plan_destroy(p);
    p = nullptr;

    // argument and element checks
    expect("out NULL", gbp_plan_create(xyz.data(), n_v, tets.data(), n_e, nullptr, nullptr), GBP_ERR_ARG);
    expect("xyz NULL", gbp_plan_create(nullptr, n_v, tets.data(), n_e, nullptr, &p), GBP_ERR_ARG);
    expect("n_v 0", gbp_plan_create(xyz.data(), 0, tets.data(), n_e, nullptr, &p), GBP_ERR_ARG);
    expect("element count overflow", gbp_plan_create(xyz.data(), n_v, tets.data(), 1 << 29, nullptr, &p),
           GBP_ERR_ARG);
    o = gbp_options{};
    o.reserved[2] = 1;
    expect("reserved option set", gbp_plan_create(xyz.data(), n_v, tets.data(), n_e, &o, &p), GBP_ERR_ARG);
    {
        auto x = xyz;
        x[3 * 7 + 1] = NAN;
        expect("NaN coordinate", gbp_plan_create(x.data(), n_v, tets.data(), n_e, nullptr, &p),
               GBP_ERR_NONFINITE);
        x[3 * 7 + 1] = INFINITY;
        expect("Inf coordinate", gbp_plan_create(x.data(), n_v, tets.data(), n_e, nullptr, &p),
               GBP_ERR_NONFINITE);
    }
    {
        auto t = tets;
        t[4 * 3 + 2] = n_v;
        expect("vertex id n_v", gbp_plan_create(xyz.data(), n_v, t.data(), n_e, nullptr, &p), GBP_ERR_ARG);
        t[4 * 3 + 2] = -1;
        expect("vertex id -1", gbp_plan_create(xyz.data(), n_v, t.data(), n_e, nullptr, &p), GBP_ERR_ARG);
        t = tets;
        t[4 * 5 + 3] = t[4 * 5 + 1];
        expect("repeated vertex", gbp_plan_create(xyz.data(), n_v, t.data(), n_e, nullptr, &p), GBP_ERR_ARG);
    }
    {
        // four coplanar points
        const float q[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 1, 1, 0};
        const int32_t t[4] = {0, 1, 2, 3};
        expect("flat element", gbp_plan_create(q, 4, t, 1, nullptr, &p), GBP_ERR_DEGENERATE_TET);
    }
    {
        // vertex 0 in local slot 0 of 256 elements: beyond the 8-bit count
        std::vector<float> q = {0, 0, 0};
        std::vector<int32_t> t;
        for (int k = 0; k < 256; ++k) {
            const float z = 1.0f + k;
            const int b = (int)q.size() / 3;
            q.insert(q.end(), {1, 0, z, 0, 1, z, 1, 1, z + 0.5f});
            t.insert(t.end(), {0, b, b + 1, b + 2});
        }
        expect("256 elements in one slot", gbp_plan_create(q.data(), (int)q.size() / 3, t.data(), 256, nullptr, &p),
               GBP_ERR_ARG);
        t.resize(4 * 255);
        expect("255 elements in one slot", gbp_plan_create(q.data(), (int)q.size() / 3, t.data(), 255, nullptr, &p),
               GBP_OK);
        gbp_plan_destroy(p);
        p = nullptr;
    }

    {
        // connected components (a two-sided warm start drops the guess on the
        // components without a root): the cube plus a separate element, in an
        // order where the far element's vertices are linked after the cube's
        std::vector<float> q = xyz;
        std::vector<int32_t> t = tets;
        const float far[12] = {10, 10, 10, 11, 10, 10, 10, 11, 10, 10, 10, 11};
        q.insert(q.end(), far, far + 12);
        t.insert(t.end(), {n_v + 3, n_v + 1, n_v, n_v + 2});
        expect("two components", gbp_plan_create(q.data(), n_v + 4, t.data(), n_e + 1, nullptr, &p), GBP_OK);
        int bad = p->n_comp == 2 ? 0 : 1;
        for (int i = 0; i < n_v + 4; ++i) {
            const int u = p->node_user[i];
            bad += p->comp[i] != (u < n_v ? p->comp[p->node_int[0]] : p->comp[p->node_int[n_v]]);
        }
        bad += p->comp[p->node_int[0]] == p->comp[p->node_int[n_v]];
        expect("component labels", bad, 0);
        gbp_plan_destroy(p);
        p = nullptr;
    }

    // every allocation of a plan made to fail in turn: an error, no plan, no leak
    stub_fail_after(-1);
    expect("count allocations", gbp_plan_create(xyz.data(), n_v, tets.data(), n_e, nullptr, &p), GBP_OK);
    const int n_alloc = stub_allocations();
    gbp_plan_destroy(p);
    for (int k = 0; k < n_alloc; ++k) {
        p = nullptr;
        stub_fail_after(k);
        const int rc = gbp_plan_create(xyz.data(), n_v, tets.data(), n_e, nullptr, &p);
        char what[64];
        std::snprintf(what, sizeof what, "allocation %d of %d fails", k + 1, n_alloc);
        expect(what, (rc == GBP_ERR_NOMEM || rc == GBP_ERR_HIP) && p == nullptr ? 0 : 1, 0);
    }
    stub_fail_after(-1);
    {
        // the hold-back's lists and the warm order's guess, allocated on use
        expect("plan for settings", gbp_plan_create(xyz.data(), n_v, tets.data(), n_e, nullptr, &p), GBP_OK);
        stub_fail_after(0);
        expect("hold lists fail", gbp_plan_set_hold(p, 1.0f, 0, 0) < 0 ? 0 : 1, 0);
        expect("guess fails", gbp_plan_set_warm_order(p, 1) < 0 ? 0 : 1, 0);
        stub_fail_after(-1);
        gbp_plan_destroy(p);
    }
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "OK", failures);
    return failures ? 1 : 0;
}
