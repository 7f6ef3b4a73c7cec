/* Host-only walk through the C ABI for the sanitizer build: defaults,
 * version, workspace queries of valid and invalid configurations, handle
 * creation that must fail before touching a device, and calls on a NULL
 * handle.  Nothing here needs a GPU.  Prints "host driver ok" and returns 0
 * when every check holds. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "mirve.h"

static int failures = 0;

#define CHECK(cond)                                                     \
    do {                                                                \
        if (!(cond)) {                                                  \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static rve_config base(int nx, int ny, int nz) {
    rve_config c;
    memset(&c, 0xA5, sizeof(c));   /* every field must be set by the defaults */
    CHECK(rve_default_config(&c) == RVE_OK);
    c.dim = nz > 1 ? 3 : 2;
    c.n[0] = nx;
    c.n[1] = ny;
    c.n[2] = nz;
    c.f[0] = c.f[1] = c.f[2] = c.f[3] = c.f[4] = c.f[5] = 0.0;
    c.f[c.dim == 3 ? 2 : 1] = 1.0;
    return c;
}

static int query(const rve_config* c, size_t* bytes) {
    *bytes = 0;
    return rve_query_workspace(c, bytes);
}

int main(void) {
    const char* v = rve_version();
    CHECK(v != NULL && strlen(v) > 0);

    /* valid shapes: power-of-two, 3/5/7-smooth, 3D, batches, both precisions */
    const int shapes[][3] = {{64, 64, 1}, {256, 256, 1}, {512, 64, 1}, {96, 80, 1},
                             {98, 70, 1}, {32, 32, 32}, {16, 128, 16}, {2, 2, 1}};
    size_t last = 0;
    for (unsigned i = 0; i < sizeof(shapes) / sizeof(shapes[0]); ++i) {
        for (int prec = RVE_PREC_FP64; prec <= RVE_PREC_MIXED; ++prec) {
            for (int batch = 1; batch <= 9; batch += 8) {
                rve_config c = base(shapes[i][0], shapes[i][1], shapes[i][2]);
                c.precision = prec;
                c.batch = batch;
                size_t b = 0;
                CHECK(query(&c, &b) == RVE_OK);
                CHECK(b > 0);
                if (batch == 9) CHECK(b > last);
                last = b;
            }
        }
    }

    /* invalid configurations: each rejected with a message */
    for (int k = 0; k < 20; ++k) {
        rve_config c = base(64, 64, 1);
        switch (k) {
            case 0: c.dim = 4; break;
            case 1: c.n[0] = 1; break;
            case 2: c.n[1] = 2048; break;
            case 3: c.h = 0.0; break;
            case 4: c.ell = -1.0; break;
            case 5: c.tol_cg = -1e-8; break;
            case 6: c.tol = NAN; break;
            case 7: c.max_cg = 0; break;
            case 8: c.max_halvings = 13; break;
            case 9: c.max_halvings = -1; break;
            case 10: c.stall_window = -1; break;
            case 11: c.batch = 0; break;
            case 12: c.batch = 5000; break;
            case 13: c.anderson_depth = 9; break;
            case 14: memset(c.f, 0, sizeof(c.f)); break;
            case 15: c.n[0] = 97; break;
            case 16: c.streaming = 2; break;
            case 17: c.graphs = 2; break;
            case 18: c.k_res = INFINITY; break;
            case 19: c.ell = NAN; break;
        }
        size_t b = 0;
        if (query(&c, &b) != RVE_EINVAL) {
            fprintf(stderr, "invalid configuration %d accepted\n", k);
            ++failures;
        }
        const char* msg = rve_last_error(NULL);
        CHECK(msg != NULL && strlen(msg) > 3);
    }
    CHECK(rve_query_workspace(NULL, &last) == RVE_EINVAL);

    /* creation fails before any device work: no workspace, too small, misaligned */
    {
        rve_config c = base(64, 64, 1);
        rve_handle h = NULL;
        CHECK(rve_create(&c, NULL, 0, NULL, &h) == RVE_EINVAL && h == NULL);
        CHECK(rve_create(&c, (void*)256, 16, NULL, &h) == RVE_ENOSPC && h == NULL);
        CHECK(rve_create(&c, (void*)(4096 + 8), (size_t)1 << 40, NULL, &h) == RVE_EINVAL && h == NULL);
        CHECK(rve_create(NULL, (void*)256, 16, NULL, &h) == RVE_EINVAL);
    }

    /* NULL handles are refused, not dereferenced */
    {
        rve_step_info info;
        double g = 0.0, buf[8] = {0};
        size_t n = 0;
        int shape[4] = {0};
        (void)rve_destroy(NULL);
        CHECK(rve_step_dissipation(NULL, 1.0, &info) != RVE_OK);
        CHECK(rve_effective_toughness(NULL, &g) != RVE_OK);
        CHECK(rve_get_field(NULL, RVE_FIELD_PHI, buf, 8) != RVE_OK);
        CHECK(rve_set_field(NULL, RVE_FIELD_PHI, buf, 8) != RVE_OK);
        CHECK(rve_get_scalars(NULL, buf) != RVE_OK);
        CHECK(rve_state_bytes(NULL, &n) != RVE_OK);
        CHECK(rve_autotune(NULL, 1, shape) != RVE_OK);
        CHECK(rve_batch_size(NULL) <= 0);
        CHECK(rve_last_error(NULL) != NULL);
    }

    /* Newton options: defaults filled in */
    {
        rve_newton_opts o;
        memset(&o, 0, sizeof(o));
        rve_newton_default_opts(&o);
        rve_newton_opts z;
        memset(&z, 0, sizeof(z));
        CHECK(memcmp(&o, &z, sizeof(o)) != 0);
    }

    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host driver ok\n");
    return 0;
}
