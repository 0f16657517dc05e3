/*
 * The C ABI of libwrls used from plain C99, with no Python and no torch.
 *
 *   abi_demo host             host-side calls only (no GPU needed): defaults,
 *                             validation, sizes and error text; prints them
 *   abi_demo gpu W H T out    one d = 8 stream of W x H FP32 pixels on device 0:
 *                             T frames of a fixed hashed pattern (see
 *                             frame_value); writes every frame's inputs to
 *                             `out`.inputs (float32 [T][13][H][W]: colour,
 *                             7 features, variance, motion) and the last
 *                             frame's output to `out` (float32 [3][H][W])
 *
 * Test infrastructure: tests/test_c_abi.py builds and runs it and checks
 * the GPU output against the FP64 oracle.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "wrls.h"

/* The HIP runtime's C entry points used here (libamdhip64). */
typedef int hipError_t;
extern hipError_t hipMalloc(void **ptr, size_t size);
extern hipError_t hipFree(void *ptr);
extern hipError_t hipMemcpy(void *dst, const void *src, size_t size, int kind);
extern hipError_t hipDeviceSynchronize(void);
enum { kHostToDevice = 1, kDeviceToHost = 2 };

/* Plane k of frame t at pixel j: a hashed value in [0.05, 1]. */
static float frame_value(int t, int plane, long j)
{
    uint32_t h = (uint32_t)(j * 2654435761u) ^ (uint32_t)(plane * 40503u + t * 97u);
    h ^= h >> 13;
    h *= 0x5bd1e995u;
    h ^= h >> 15;
    return 0.05f + 0.95f * (float)(h & 0xffffu) / 65535.0f;
}

static int host_checks(void)
{
    wrls_params p;
    wrls_params_default(&p, 1920, 1080, 8);
    printf("version %s\n", wrls_version());
    printf("state_floats %d\n", wrls_state_floats(8));
    printf("state_bytes %zu\n", wrls_state_bytes(&p));
    printf("validate_ok %d\n", (int)wrls_params_validate(&p));
    p.d = 11;
    printf("validate_d11 %d\n", (int)wrls_params_validate(&p));
    printf("error_d11 %s\n", wrls_last_error());
    printf("step_null %d\n", (int)wrls_step(NULL, NULL, NULL, NULL, NULL, NULL));
    return 0;
}

static int gpu_run(int W, int H, int T, const char *path)
{
    const int d = 8;
    const size_t n = (size_t)W * H;
    char ipath[4096];
    snprintf(ipath, sizeof ipath, "%s.inputs", path);
    wrls_params p;
    wrls_params_default(&p, W, H, d);
    wrls_stream *s = NULL;
    if (wrls_create_stream(&p, NULL, &s) != WRLS_OK) {
        fprintf(stderr, "create: %s\n", wrls_last_error());
        return 1;
    }
    /* planes: colour [0, 3), features [3, 10), variance 10, motion [11, 13) */
    float *host = (float *)malloc(sizeof(float) * n * 13);
    float *dev = NULL, *dout = NULL;
    FILE *fin = fopen(ipath, "wb");
    if (!host || !fin || hipMalloc((void **)&dev, sizeof(float) * n * 13) != 0 ||
        hipMalloc((void **)&dout, sizeof(float) * n * 3) != 0)
        return 1;
    for (int t = 0; t < T; t++) {
        for (int k = 0; k < 10; k++)
            for (size_t j = 0; j < n; j++) host[k * n + j] = frame_value(t, k, (long)j);
        for (size_t j = 0; j < n; j++) {
            host[10 * n + j] = 0.01f + 0.19f * frame_value(t, 10, (long)j);
            host[11 * n + j] = 1.25f;
            host[12 * n + j] = -0.5f;
        }
        if (fwrite(host, sizeof(float), n * 13, fin) != n * 13) return 1;
        if (hipMemcpy(dev, host, sizeof(float) * n * 13, kHostToDevice) != 0) return 1;
        if (wrls_step(s, dev, dev + 3 * n, dev + 10 * n, dev + 11 * n, dout) != WRLS_OK) {
            fprintf(stderr, "step: %s\n", wrls_last_error());
            return 1;
        }
    }
    fclose(fin);
    if (hipDeviceSynchronize() != 0) return 1;
    if (hipMemcpy(host, dout, sizeof(float) * n * 3, kDeviceToHost) != 0) return 1;
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(host, sizeof(float), n * 3, f) != n * 3) return 1;
    fclose(f);
    printf("frames %lld\n", (long long)wrls_frames(s));
    wrls_destroy(s);
    hipFree(dout);
    hipFree(dev);
    free(host);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc >= 2 && strcmp(argv[1], "host") == 0) return host_checks();
    if (argc >= 6 && strcmp(argv[1], "gpu") == 0)
        return gpu_run(atoi(argv[2]), atoi(argv[3]), atoi(argv[4]), argv[5]);
    fprintf(stderr, "usage: abi_demo host | abi_demo gpu W H T out\n");
    return 2;
}
