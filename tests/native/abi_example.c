/* Use of libmi355_sincos.so from plain C through include/sincos.h and the HIP
 * runtime's C API, with no Python: the plain form, argument errors, a ragged
 * plan replayed as a graph, the interleaved layout and the request server.
 * Checks each result against the C library's double-precision sin/cos within
 * the method's accuracy (about 5e-7 for angles of moderate size) and prints
 * "abi_example: ok" on success.                                            */
#define __HIP_PLATFORM_AMD__ 1
#include <hip/hip_runtime_api.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/sincos.h"

#define CHECK(cond, ...)                                        \
    do {                                                        \
        if (!(cond)) {                                          \
            fprintf(stderr, "abi_example: FAILED: " __VA_ARGS__); \
            fprintf(stderr, "\n");                              \
            exit(1);                                            \
        }                                                       \
    } while (0)

static double max_err(const float *x, const float *s, const float *c, long n)
{
    double m = 0.0;
    for (long i = 0; i < n; i++) {
        double e = hypot((double)s[i] - sin((double)x[i]), (double)c[i] - cos((double)x[i]));
        if (e > m)
            m = e;
    }
    return m;
}

int main(void)
{
    int ndev = 0;
    CHECK(hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0, "no HIP device");
    const long n = 1000003;
    float *hx = malloc(sizeof(float) * n), *hs = malloc(sizeof(float) * n),
          *hc = malloc(sizeof(float) * n);
    for (long i = 0; i < n; i++)
        hx[i] = (float)(-20.0 + 40.0 * (double)i / (double)n);
    float *x, *s, *c, *cs;
    CHECK(hipMalloc((void **)&x, sizeof(float) * n) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void **)&s, sizeof(float) * n) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void **)&c, sizeof(float) * n) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void **)&cs, sizeof(float) * 2 * n) == hipSuccess, "hipMalloc");
    CHECK(hipMemcpy(x, hx, sizeof(float) * n, hipMemcpyHostToDevice) == hipSuccess, "copy");

    /* plain form on the null stream */
    CHECK(sincos_f32(x, s, c, n, NULL) == SINCOS_OK, "sincos_f32: %s", sincos_last_error());
    CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
    CHECK(hipMemcpy(hs, s, sizeof(float) * n, hipMemcpyDeviceToHost) == hipSuccess, "copy");
    CHECK(hipMemcpy(hc, c, sizeof(float) * n, hipMemcpyDeviceToHost) == hipSuccess, "copy");
    double e = max_err(hx, hs, hc, n);
    CHECK(e < 2e-6, "plain form error %g", e);

    /* argument errors come back as status codes with a message */
    CHECK(sincos_f32(x, s, s, n, NULL) == SINCOS_EOVERLAP, "s == c not rejected");
    CHECK(strlen(sincos_last_error()) > 0, "no error message");
    CHECK(sincos_f32(x, s, c, -1, NULL) == SINCOS_EINVAL, "n < 0 not rejected");

    /* ragged plan over three pieces of the same arrays, replayed as a graph */
    CHECK(hipMemset(s, 0, sizeof(float) * n) == hipSuccess, "memset");
    CHECK(hipMemset(c, 0, sizeof(float) * n) == hipSuccess, "memset");
    sincos_seg_t segs[3] = {{x, s, c}, {x + 1000, s + 1000, c + 1000}, {x + 500000, s + 500000, c + 500000}};
    int64_t lens[3] = {1000, 499000, n - 500000};
    sincos_ragged_plan_t *plan = NULL;
    CHECK(sincos_ragged_plan_create(segs, lens, 3, SINCOS_ARITH_FUSED, SINCOS_METHOD_NORMALIZED,
                                    NULL, &plan) == SINCOS_OK,
          "plan: %s", sincos_last_error());
    for (int r = 0; r < 3; r++)
        CHECK(sincos_ragged_plan_graph_launch(plan, NULL) == SINCOS_OK, "graph launch: %s",
              sincos_last_error());
    CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
    float *hs2 = malloc(sizeof(float) * n), *hc2 = malloc(sizeof(float) * n);
    CHECK(hipMemcpy(hs2, s, sizeof(float) * n, hipMemcpyDeviceToHost) == hipSuccess, "copy");
    CHECK(hipMemcpy(hc2, c, sizeof(float) * n, hipMemcpyDeviceToHost) == hipSuccess, "copy");
    CHECK(memcmp(hs, hs2, sizeof(float) * n) == 0 && memcmp(hc, hc2, sizeof(float) * n) == 0,
          "ragged plan differs from the plain form");
    CHECK(sincos_ragged_plan_destroy(plan) == SINCOS_OK, "plan destroy");

    /* complex64 output: (cos, sin) pairs, the same bits */
    CHECK(sincos_f32_interleaved(x, cs, n, 0, NULL) == SINCOS_OK, "interleaved: %s",
          sincos_last_error());
    CHECK(hipDeviceSynchronize() == hipSuccess, "sync");
    float *hcs = malloc(sizeof(float) * 2 * n);
    CHECK(hipMemcpy(hcs, cs, sizeof(float) * 2 * n, hipMemcpyDeviceToHost) == hipSuccess, "copy");
    for (long i = 0; i < n; i++)
        CHECK(memcmp(&hcs[2 * i], &hc[i], 4) == 0 && memcmp(&hcs[2 * i + 1], &hs[i], 4) == 0,
              "complex output differs at %ld", i);

    /* request server: two requests, completions, release */
    sincos_server_config_t cfg;
    memset(&cfg, 0, sizeof cfg);
    sincos_server_t *srv = NULL;
    CHECK(sincos_server_create(&cfg, &srv) == SINCOS_OK, "server: %s", sincos_last_error());
    int64_t id1, id2;
    CHECK(sincos_server_submit(srv, x, 4096, 1, &id1) == SINCOS_OK, "submit");
    CHECK(sincos_server_submit(srv, x + 4096, n - 4096, 2, &id2) == SINCOS_OK, "submit");
    int done = 0;
    sincos_completion_t comp[4];
    while (done < 2) {
        int32_t k = 0;
        CHECK(sincos_server_poll(srv, comp, 4, &k, 1000000000) == SINCOS_OK, "poll");
        for (int i = 0; i < k; i++) {
            CHECK(comp[i].status == SINCOS_OK, "request failed");
            const long off = comp[i].tag == 1 ? 0 : 4096;
            float *ts = malloc(sizeof(float) * comp[i].n);
            CHECK(hipMemcpy(ts, comp[i].s, sizeof(float) * comp[i].n, hipMemcpyDeviceToHost) ==
                      hipSuccess, "copy");
            CHECK(memcmp(ts, hs + off, sizeof(float) * comp[i].n) == 0, "served result differs");
            free(ts);
            CHECK(sincos_server_release(srv, comp[i].id) == SINCOS_OK, "release");
            done++;
        }
    }
    CHECK(sincos_server_destroy(srv) == SINCOS_OK, "server destroy");

    hipFree(x);
    hipFree(s);
    hipFree(c);
    hipFree(cs);
    free(hx);
    free(hs);
    free(hc);
    free(hs2);
    free(hc2);
    free(hcs);
    printf("abi_example: ok (%s, max error %.3g)\n", sincos_version(), e);
    return 0;
}
