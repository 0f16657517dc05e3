/* The host-side paths of the C ABI that need no GPU -- parameter defaults
 * and validation, size queries, NULL handles and arguments, the size limit
 * of the allocation-free batched step, error text -- driven from plain C99
 * so that a build of libwrls with AddressSanitizer and
 * UndefinedBehaviorSanitizer on its host code can check them.  Exits
 * non-zero when a call returns other than documented. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "wrls.h"

static int bad = 0;
#define EXPECT(cond)                                              \
    do {                                                          \
        if (!(cond)) {                                            \
            printf("line %d: %s\n", __LINE__, #cond);             \
            bad++;                                                \
        }                                                         \
    } while (0)

int main(void)
{
    wrls_params p;
    wrls_params_default(NULL, 1, 1, 1);
    for (int d = 0; d <= WRLS_MAX_D + 1; d++) {
        wrls_params_default(&p, 1920, 1080, d);
        int ok = d >= 1 && d <= WRLS_MAX_D;
        EXPECT((wrls_params_validate(&p) == WRLS_OK) == ok);
        EXPECT((wrls_state_floats(d) > 0) == ok);
        EXPECT((wrls_state_bytes(&p) > 0) == ok);
        EXPECT(wrls_stream_device_bytes(&p) >= 2 * wrls_state_bytes(&p));
    }
    wrls_params_default(&p, 3840, 2160, 10);
    EXPECT(wrls_state_bytes(&p) == (size_t)85 * 4 * 3840 * 2160);
    struct { float *field; float value; } bad_floats[] = {
        {&p.lambda, 0.0f}, {&p.lambda, 1.5f}, {&p.lambda, NAN}, {&p.delta, 0.0f},
        {&p.delta, INFINITY}, {&p.var_floor, -1.0f}, {&p.sigma0, -2.0f}, {&p.sigma0, NAN}};
    for (size_t i = 0; i < sizeof bad_floats / sizeof bad_floats[0]; i++) {
        wrls_params_default(&p, 64, 48, 8);
        *bad_floats[i].field = bad_floats[i].value;
        EXPECT(wrls_params_validate(&p) == WRLS_EINVAL);
        EXPECT(strlen(wrls_last_error()) > 0);
    }
    wrls_params_default(&p, 64, 48, 8);
    p.sigma0 = 30.0f;
    p.lambda_min = 0.99f;
    EXPECT(wrls_params_validate(&p) == WRLS_EINVAL);
    p.lambda_min = 0.5f;
    EXPECT(wrls_params_validate(&p) == WRLS_OK);
    wrls_params_default(&p, 16385, 8, 8);
    EXPECT(wrls_params_validate(&p) == WRLS_EINVAL);
    wrls_params_default(&p, 16384, 16384, 10);
    EXPECT(wrls_params_validate(&p) == WRLS_EUNSUPPORTED);   /* state copy above 4 GiB */
    wrls_params_default(&p, 64, 48, 8);
    p.weight_mode = WRLS_W_PAPER;
    EXPECT(wrls_params_validate(&p) == WRLS_EINVAL);          /* paper mode needs d = 4 */
    EXPECT(wrls_params_validate(NULL) == WRLS_EINVAL);

    wrls_stream *s = NULL;
    EXPECT(wrls_create_stream(&p, NULL, NULL) == WRLS_EINVAL);
    EXPECT(wrls_create_stream(NULL, NULL, &s) == WRLS_EINVAL && s == NULL);
    EXPECT(wrls_create_stream_in(&p, NULL, 0, NULL, &s) == WRLS_EINVAL);
    EXPECT(wrls_destroy(NULL) == WRLS_OK);
    EXPECT(wrls_reset(NULL) == WRLS_EINVAL);
    EXPECT(wrls_frames(NULL) == -1);
    EXPECT(wrls_step(NULL, NULL, NULL, NULL, NULL, NULL) == WRLS_EINVAL);
    EXPECT(wrls_get_state(NULL, NULL, NULL) == WRLS_EINVAL);
    EXPECT(wrls_set_state(NULL, NULL, NULL, 0) == WRLS_EINVAL);
    EXPECT(wrls_blend(NULL, NULL, NULL, 1.0f, 1.0f, NULL) == WRLS_EINVAL);
    EXPECT(wrls_get_history(NULL, NULL) == WRLS_EINVAL);
    EXPECT(wrls_set_history(NULL, NULL) == WRLS_EINVAL);
    EXPECT(wrls_set_tile(NULL, 7, 128, 0) == WRLS_EINVAL);
    int32_t a, b, c;
    EXPECT(wrls_get_tile(NULL, &a, &b, &c) == WRLS_EINVAL);
    EXPECT(wrls_set_hip_stream(NULL, NULL) == WRLS_EINVAL);
    wrls_batch *bt = NULL;
    EXPECT(wrls_batch_create(0, 8, WRLS_F16, NULL, &bt) == WRLS_EINVAL);
    EXPECT(wrls_batch_create(WRLS_MAX_BATCH + 1, 8, WRLS_F16, NULL, &bt) == WRLS_EINVAL);
    EXPECT(wrls_batch_create(4, 11, WRLS_F16, NULL, &bt) == WRLS_EUNSUPPORTED);
    EXPECT(wrls_batch_destroy(NULL) == WRLS_OK);
    EXPECT(wrls_batch_hip_stream(NULL) == NULL);
    EXPECT(wrls_batch_set_tile(NULL, 7, 128, 0) == WRLS_EINVAL);
    EXPECT(wrls_batch_use_graph(NULL, 1) == WRLS_EINVAL);
    EXPECT(wrls_batch_step(NULL, 0, NULL, NULL) == WRLS_EINVAL);
    wrls_stream *none[1] = {NULL};
    wrls_frame fr[1];
    memset(fr, 0, sizeof fr);
    EXPECT(wrls_batch_step_noalloc(WRLS_NOALLOC_MAX_STREAMS + 1, none, fr, 7, 128, NULL) == WRLS_EINVAL);
    EXPECT(strstr(wrls_last_error(), "65") != NULL);
    EXPECT(wrls_batch_step_noalloc(-1, none, fr, 7, 128, NULL) == WRLS_EINVAL);
    EXPECT(wrls_batch_step_noalloc(0, NULL, NULL, 7, 128, NULL) == WRLS_OK);
    EXPECT(wrls_batch_step_noalloc(1, none, fr, 7, 128, NULL) == WRLS_EINVAL);
    EXPECT(wrls_batch_step_noalloc(1, none, fr, 9, 256, NULL) == WRLS_EINVAL);
    char buf[64];
    EXPECT(wrls_device_copy(buf, buf + 32, 0, NULL) == WRLS_OK);
    EXPECT(wrls_device_copy(NULL, buf, 16, NULL) == WRLS_EINVAL);
    EXPECT(wrls_device_copy(buf + 1, buf + 33, 16, NULL) == WRLS_EINVAL);   /* misaligned */
    EXPECT(wrls_traffic_probe(NULL, NULL, NULL, NULL, NULL, NULL) == WRLS_EINVAL);
    EXPECT(wrls_checked_build() == 0);
    uint32_t flags = 7u;
    EXPECT(wrls_checked_failures(&flags) == WRLS_EUNSUPPORTED && flags == 7u);
    EXPECT(wrls_checked_raise(1u, NULL) == WRLS_EUNSUPPORTED);
    EXPECT(strncmp(wrls_version(), "libwrls", 7) == 0);
    printf("abi validate: %s\n", bad ? "FAILED" : "ok");
    return bad != 0;
}
