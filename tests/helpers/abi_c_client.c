/* A plain C client of the library: it owns the device workspace and the
 * stream, builds one simple-cubic system (periodic x, y; open z; no grains),
 * sets a uniform temperature and write field, runs Heun steps and writes
 * the spins and the FP64 magnetisation.  Used by the tests to show the
 * C ABI is usable without Python.
 *
 * usage: abi_c_client nx ny nz a J mu_s alpha gamma dt k_u Bz T seed steps out.bin
 * out.bin: [3][n] doubles (spins after the steps), then 4 doubles (Mx, My, Mz, N). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "asd.h"

#define CHECK(x)                                                               \
    do {                                                                       \
        int rc_ = (x);                                                         \
        if (rc_ != ASD_OK) {                                                   \
            fprintf(stderr, "%s failed: %s (%s)\n", #x, asd_strerror(rc_),     \
                    asd_last_error(h));                                        \
            return 1;                                                          \
        }                                                                      \
    } while (0)

int main(int argc, char **argv)
{
    if (argc != 16) {
        fprintf(stderr, "usage: %s nx ny nz a J mu_s alpha gamma dt k_u Bz T seed steps out\n", argv[0]);
        return 2;
    }
    asd_t *h = NULL;
    asd_params p = {0};
    p.lattice = ASD_SC;
    p.precision = ASD_FP64;
    p.a = p.c = strtod(argv[4], NULL);
    p.n_shells = 1;
    p.J[0] = strtod(argv[5], NULL);
    p.mu_s = strtod(argv[6], NULL);
    p.alpha = strtod(argv[7], NULL);
    p.gamma = strtod(argv[8], NULL);
    p.dt = strtod(argv[9], NULL);
    p.k_u = strtod(argv[10], NULL);
    p.seed = strtoull(argv[13], NULL, 10);
    p.philox_rounds = 10;
    p.kernel = ASD_KERNEL_AUTO;
    p.graph_steps = 10;

    asd_system_desc d = {0};
    d.nx = atoi(argv[1]);
    d.ny = atoi(argv[2]);
    d.nz = atoi(argv[3]);
    d.bc_x = ASD_BC_PERIODIC;
    d.bc_y = ASD_BC_PERIODIC;
    d.bc_z = ASD_BC_OPEN;
    d.T_system = -1.0;

    size_t bytes = 0;
    CHECK(asd_workspace_bytes(&p, &d, 1, &bytes));
    void *ws = NULL;
    hipStream_t stream = NULL;
    if (hipMalloc(&ws, bytes) != hipSuccess || hipStreamCreate(&stream) != hipSuccess) {
        fprintf(stderr, "hip allocation failed\n");
        return 1;
    }
    CHECK(asd_create(&p, &d, 1, ws, bytes, stream, &h));

    asd_drive drv = {0};
    drv.B[2] = strtod(argv[11], NULL);
    drv.spot_mode = ASD_SPOT_NONE;
    drv.T_amb = strtod(argv[12], NULL);
    CHECK(asd_set_field_temperature(h, &drv));
    CHECK(asd_prepare(h));
    CHECK(asd_step(h, atoll(argv[14])));

    int64_t n = 0;
    CHECK(asd_stored_sites(h, 0, &n));
    double *S = (double *)malloc(sizeof(double) * (size_t)(3 * n + 4));
    CHECK(asd_get_spins(h, 0, S, 0));
    double M[4];
    CHECK(asd_reduce_magnetization(h, NULL, M));
    for (int k = 0; k < 4; ++k) S[3 * n + k] = M[k];
    FILE *f = fopen(argv[15], "wb");
    if (!f || fwrite(S, sizeof(double), (size_t)(3 * n + 4), f) != (size_t)(3 * n + 4)) {
        fprintf(stderr, "cannot write %s\n", argv[15]);
        return 1;
    }
    fclose(f);
    printf("sites %lld M %.17g %.17g %.17g N %.0f\n", (long long)n, M[0], M[1], M[2], M[3]);
    free(S);
    CHECK(asd_destroy(h));
    (void)hipStreamDestroy(stream);
    (void)hipFree(ws);
    return 0;
}
