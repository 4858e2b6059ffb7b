// Host-side checks of the C ABI (include/lbm.h) for a sanitizer build: the
// argument validation and workspace layout of every lbm_params variant the
// library accepts or rejects, init's early rejections, and every context
// call given a NULL context.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer on its host side only (no kernel is ever
// launched) by tests/test_host_sanitizers.py; prints each failed expectation
// and exits non-zero if there was one.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "lbm.h"

static int failures = 0;

#define EXPECT(cond)                                                    \
    do {                                                                \
        if (!(cond)) {                                                  \
            fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #cond);   \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static lbm_params base(int nx, int ny, int nz) {
    lbm_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.precision = LBM_FP32;
    p.tau[0] = p.tau[1] = 1.0;
    p.G = 3.6;
    p.rho_maj = 0.7;
    p.rho_min = 0.04;
    p.mass_tol = 1e-3;
    p.wet_scale = 1.0;
    p.rep_d0 = 1.25;
    p.node_mass = 5.0;
    p.mass_c0 = 2500.0;
    return p;
}

static int ws(const lbm_params& p, int64_t nodes, int64_t faces, int64_t* out) {
    return lbm_workspace_bytes(&p, nodes, faces, out);
}

int main() {
    int64_t n = 0, n0 = 0, n1 = 0;
    // accepted parameter sets give a positive size that grows with the membrane
    {
        lbm_params p = base(32, 32, 32);
        EXPECT(ws(p, 0, 0, &n0) == LBM_OK && n0 > 0);
        EXPECT(ws(p, 642, 1280, &n1) == LBM_OK && n1 > n0);
        p.n_slots = 3;
        EXPECT(ws(p, 642, 1280, &n) == LBM_OK && n > n1);
        p = base(48, 24, 24);
        p.ring_len = 10;
        EXPECT(ws(p, 162, 320, &n) == LBM_OK && n > 0);
        p = base(16, 16, 16);
        p.precision = LBM_FP16;
        EXPECT(ws(p, 162, 320, &n) == LBM_OK);
        p = base(16, 16, 16);
        p.deterministic = 1;
        EXPECT(ws(p, 162, 320, &n) == LBM_OK);
        p = base(16, 16, 16);
        p.mass_fix = 1;
        p.check_every = 10;
        EXPECT(ws(p, 162, 320, &n) == LBM_OK);
        p = base(16, 16, 16);
        p.coupling = 1;
        int64_t nbb = 0;
        EXPECT(ws(p, 162, 320, &nbb) == LBM_OK);
        p.coupling = 0;
        EXPECT(ws(p, 162, 320, &n) == LBM_OK && nbb > n);
        // the largest lattice that 32-bit offsets address, and beyond it
        p = base(1024, 1024, 1024);
        EXPECT(ws(p, 0, 0, &n) == LBM_OK && n > (int64_t)1 << 30);
        p = base(1024, 1024, 1025);
        EXPECT(ws(p, 0, 0, &n) == LBM_EINVAL);
        p = base(1 << 20, 1 << 20, 4);
        EXPECT(ws(p, 0, 0, &n) == LBM_EINVAL);
        p = base(-8, 16, 16);
        EXPECT(ws(p, 0, 0, &n) == LBM_EINVAL);
        p = base(16, 16, 16);
        EXPECT(ws(p, -1, 0, &n) == LBM_EINVAL);
        EXPECT(ws(p, (int64_t)1 << 40, (int64_t)1 << 40, &n) == LBM_EINVAL);
        EXPECT(ws(p, ((int64_t)1 << 29) + 1, 0, &n) == LBM_EINVAL);
        EXPECT(ws(p, 0, ((int64_t)1 << 29) + 1, &n) == LBM_EINVAL);
        EXPECT(ws(p, (int64_t)1 << 29, (int64_t)1 << 29, &n) == LBM_OK && n > 0);
    }
    // rejected parameter values, one at a time
    {
        std::vector<lbm_params> bad;
        lbm_params p = base(16, 16, 16);
        p.tau[0] = 0.5; bad.push_back(p);
        p = base(16, 16, 16); p.tau[1] = NAN; bad.push_back(p);
        p = base(16, 16, 16); p.G = -1.0; bad.push_back(p);
        p = base(16, 16, 16); p.walls = 3; bad.push_back(p);
        p = base(16, 16, 16); p.precision = 7; bad.push_back(p);
        p = base(16, 16, 16); p.stream_policy = 3; bad.push_back(p);
        p = base(16, 16, 16); p.zchunk = 12; bad.push_back(p);
        p = base(16, 16, 16); p.ring_len = 4; p.precision = LBM_FP16; bad.push_back(p);
        p = base(16, 16, 16); p.rep_eps = NAN; bad.push_back(p);
        p = base(16, 16, 16); p.rep_eps = 0.5; p.rep_d0 = 2.5; bad.push_back(p);
        p = base(16, 16, 16); p.psi_kind = 2; bad.push_back(p);
        p = base(16, 16, 16); p.coupling = 2; bad.push_back(p);
        p = base(16, 16, 16); p.coupling = 1; p.precision = LBM_FP16; bad.push_back(p);
        p = base(16, 16, 16); p.coupling = 1; p.walls = 1; bad.push_back(p);
        p = base(16, 16, 16); p.coupling = 1; p.n_slots = 1; bad.push_back(p);
        p = base(16, 16, 16); p.coupling = 1; p.node_mass = INFINITY; bad.push_back(p);
        p = base(16, 16, 16); p.coupling = 1; p.mass_c0 = -1.0; bad.push_back(p);
        p = base(16, 16, 16); p.deterministic = 2; bad.push_back(p);
        p = base(16, 16, 16); p.mass_fix = 2; p.check_every = 10; bad.push_back(p);
        p = base(16, 16, 16); p.mass_fix = 1; bad.push_back(p);                       // no mass check
        p = base(16, 16, 16); p.mass_fix = 1; p.check_every = 10; p.precision = LBM_FP16; bad.push_back(p);
        p = base(16, 16, 16); p.mass_fix = 1; p.check_every = 10; p.walls = 2; bad.push_back(p);
        p = base(16, 16, 16); p.deterministic = 1; p.coupling = 1; bad.push_back(p);
        p = base(3, 16, 16); bad.push_back(p);
        for (size_t k = 0; k < bad.size(); ++k) {
            const int r = ws(bad[k], 0, 0, &n);
            if (r != LBM_EINVAL) fprintf(stderr, "parameter set %zu accepted\n", k);
            EXPECT(r == LBM_EINVAL);
            EXPECT(lbm_last_error(NULL) != NULL && strlen(lbm_last_error(NULL)) > 0);
        }
        EXPECT(lbm_workspace_bytes(NULL, 0, 0, &n) == LBM_EINVAL);
        lbm_params ok = base(16, 16, 16);
        EXPECT(lbm_workspace_bytes(&ok, 0, 0, NULL) == LBM_EINVAL);
    }
    // init rejects before any device work
    {
        std::vector<float> r(16 * 16 * 16, 1.0f), neg(r);
        neg[7] = -1.0f;
        lbm_ctx* ctx = (lbm_ctx*)0x1;
        lbm_params p = base(16, 16, 16);
        p.tau[0] = 0.4;
        EXPECT(lbm_init(&p, r.data(), r.data(), (void*)256, (int64_t)1 << 30, 0, 0, NULL, &ctx) == LBM_EINVAL);
        EXPECT(ctx == NULL);
        p = base(16, 16, 16);
        EXPECT(lbm_init(&p, neg.data(), r.data(), (void*)256, (int64_t)1 << 40, 0, 0, NULL, &ctx) == LBM_EINVAL);
        EXPECT(lbm_init(&p, r.data(), r.data(), (void*)256, 1024, 0, 0, NULL, &ctx) == LBM_ENOMEM);
        EXPECT(lbm_init(&p, NULL, r.data(), (void*)256, (int64_t)1 << 40, 0, 0, NULL, &ctx) == LBM_EINVAL);
        EXPECT(lbm_init(&p, r.data(), r.data(), NULL, (int64_t)1 << 40, 0, 0, NULL, &ctx) == LBM_EINVAL);
        EXPECT(lbm_init(NULL, r.data(), r.data(), (void*)256, (int64_t)1 << 40, 0, 0, NULL, &ctx) == LBM_EINVAL);
        EXPECT(lbm_init(&p, r.data(), r.data(), (void*)256, (int64_t)1 << 40, 0, 0, NULL, NULL) == LBM_EINVAL);
    }
    // every context call rejects a NULL context; destroying NULL is a no-op
    {
        double d[8] = {0};
        float f[8] = {0};
        int32_t i[8] = {0};
        lbm_obs o;
        lbm_capsule_obs co;
        EXPECT(lbm_capsules_add(NULL, 0, i, i, d, i, d, d, d, d, i) == LBM_EINVAL);
        EXPECT(lbm_capsules_bending(NULL, 0, 0, d) == LBM_EINVAL);
        EXPECT(lbm_capsules_velocity(NULL, 0, 0, d, 0) == LBM_EINVAL);
        EXPECT(lbm_reference_relax(NULL, 1, 0.01, 1.0, 0.0, 0.05) == LBM_EINVAL);
        EXPECT(lbm_step(NULL, 1) == LBM_EINVAL);
        EXPECT(lbm_step_timed(NULL, 1, d) == LBM_EINVAL);
        EXPECT(lbm_observables(NULL, &o, &co) == LBM_EINVAL);
        EXPECT(lbm_observables_noalloc(NULL, &o, &co) == LBM_EINVAL);
        EXPECT(lbm_get_fields(NULL, f, f, f) == LBM_EINVAL);
        EXPECT(lbm_get_nodes(NULL, d) == LBM_EINVAL);
        EXPECT(lbm_get_node_forces(NULL, f) == LBM_EINVAL);
        EXPECT(lbm_get_node_velocities(NULL, f) == LBM_EINVAL);
        EXPECT(lbm_get_spread(NULL, f, f) == LBM_EINVAL);
        EXPECT(lbm_debug_bins(NULL, i, i) == LBM_EINVAL);
        EXPECT(lbm_debug_labels(NULL, i) == LBM_EINVAL);
        EXPECT(lbm_state_save(NULL, 0) == LBM_EINVAL);
        EXPECT(lbm_state_load(NULL, 0) == LBM_EINVAL);
        EXPECT(lbm_adjoint_forward(NULL, 1, 1, 0, 0, d) == LBM_EINVAL);
        EXPECT(lbm_adjoint_backward(NULL, d) == LBM_EINVAL);
        EXPECT(lbm_adjoint_seed(NULL, 0, 0) == LBM_EINVAL);
        EXPECT(lbm_adjoint_record(NULL, 1) == LBM_EINVAL);
        EXPECT(lbm_adjoint_step(NULL, 0) == LBM_EINVAL);
        EXPECT(lbm_adjoint_grads(NULL, d) == LBM_EINVAL);
        lbm_destroy(NULL);
        EXPECT(lbm_last_error(NULL) != NULL);
    }
    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("host checks passed\n");
    return 0;
}
