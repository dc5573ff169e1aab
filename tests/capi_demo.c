/* A plain C program that drives the solver through include/lbcg.h alone: it allocates the device
 * workspace and the stream itself with the HIP runtime (the library never allocates), creates a
 * solver from parameters given on the command line, steps it, and prints the diagnostics and the
 * crystal extents along four directions. tests/test_gpu_capi_demo.py checks them against the
 * oracle.
 *
 *   capi_demo dim nx ny nz flow xbc precision W0 tau0 lambda D eps nu h_drag u_in U0 U_in
 *             cx cy cz R collision omega_bulk steps
 */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "lbcg.h"

#define CHECK(call)                                                                          \
    do {                                                                                     \
        lbcg_status st_ = (call);                                                            \
        if (st_ != LBCG_OK) {                                                                \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, lbcg_last_error());     \
            return 1;                                                                        \
        }                                                                                    \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 25) {
        fprintf(stderr, "usage: capi_demo dim nx ny nz flow xbc precision W0 tau0 lambda D eps nu h_drag "
                        "u_in U0 U_in cx cy cz R collision omega_bulk steps\n");
        return 2;
    }
    lbcg_params p = {0};
    p.dim = atoi(argv[1]);
    p.nx = atoi(argv[2]);
    p.ny = atoi(argv[3]);
    p.nz = atoi(argv[4]);
    p.flow = atoi(argv[5]);
    p.xbc = atoi(argv[6]);
    p.precision = atoi(argv[7]);
    p.W0 = atof(argv[8]);
    p.tau0 = atof(argv[9]);
    p.lambda = atof(argv[10]);
    p.D = atof(argv[11]);
    p.eps_aniso = atof(argv[12]);
    p.nu = atof(argv[13]);
    p.h_drag = atof(argv[14]);
    p.u_inlet = atof(argv[15]);
    p.U0 = atof(argv[16]);
    p.U_inlet = atof(argv[17]);
    p.seed_center[0] = atof(argv[18]);
    p.seed_center[1] = atof(argv[19]);
    p.seed_center[2] = atof(argv[20]);
    p.seed_radius = atof(argv[21]);
    p.grad_eps2 = 1e-12;
    p.collision = atoi(argv[22]);
    p.omega_bulk = atof(argv[23]);
    long long steps = atoll(argv[24]);

    size_t bytes = lbcg_workspace_bytes(&p);
    if (bytes == 0) {
        fprintf(stderr, "invalid parameters\n");
        return 1;
    }
    void* ws = NULL;
    hipStream_t stream;
    if (hipMalloc(&ws, bytes) != hipSuccess || hipStreamCreate(&stream) != hipSuccess) {
        fprintf(stderr, "HIP allocation failed\n");
        return 1;
    }
    lbcg_handle* h = NULL;
    CHECK(lbcg_create(&p, ws, bytes, (void*)stream, &h));
    CHECK(lbcg_step(h, steps));
    const double dirs[12] = {1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0};
    double L[4], mass[6];
    CHECK(lbcg_measure(h, 4, dirs, L, mass));
    printf("steps %lld\n", (long long)lbcg_step_count(h));
    printf("L %.17g %.17g %.17g %.17g\n", L[0], L[1], L[2], L[3]);
    printf("mass %.17g %.17g %.17g %.17g %.17g %.17g\n", mass[0], mass[1], mass[2], mass[3], mass[4], mass[5]);
    CHECK(lbcg_destroy(h));
    hipStreamDestroy(stream);
    hipFree(ws);
    return 0;
}
