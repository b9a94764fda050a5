/* Host-side calls of libtmd that need no GPU (tables, messages, argument
 * checks), linked against a build of the library whose host code carries
 * AddressSanitizer and UndefinedBehaviorSanitizer instrumentation.  Prints
 * "ok" and exits 0 if every call returned what include/tmd.h documents. */
#include <stdio.h>
#include <string.h>

#include "tmd.h"

static int fails = 0;
#define EXPECT(c)                                                 \
    do {                                                          \
        if (!(c)) {                                               \
            fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__); \
            fails++;                                              \
        }                                                         \
    } while (0)

int main(void)
{
    float t[2048];
    EXPECT(tmd_tables(0.5f, t, 2048) == 7 * 152 + 2 * 18 + 4);
    EXPECT(tmd_tables(0.5f, t, 10) < 0);
    EXPECT(tmd_tables(0.5f, NULL, 2048) < 0);
    for (int c = 0; c >= -7; c--) EXPECT(tmd_strerror(c) != NULL && strlen(tmd_strerror(c)) > 0);
    EXPECT(strncmp(tmd_version(), "tmd", 3) == 0);
    tmd_frame_shape sh = {10, 100, 50};
    tmd_params p = {0.5f, 0u};
    tmd_plan_t *plan = NULL;
    size_t ws = 0;
    EXPECT(tmd_plan(NULL, 1, &p, &plan, &ws) == TMD_E_ARG);
    EXPECT(tmd_plan(&sh, 0, &p, &plan, &ws) == TMD_E_ARG);
    tmd_frame_shape big = {TMD_MAX_TRACKS + 1u, 0, 0};
    EXPECT(tmd_plan(&big, 1, &p, &plan, &ws) == TMD_E_ARG);
    /* with no GPU: an error code, never a crash */
    int rc = tmd_plan(&sh, 1, &p, &plan, &ws);
    EXPECT(rc == TMD_OK || rc == TMD_E_HIP);
    if (rc == TMD_OK) tmd_free(plan);
    tmd_frame_in in;
    tmd_frame_out out;
    memset(&in, 0, sizeof(in));
    memset(&out, 0, sizeof(out));
    EXPECT(tmd_decode(NULL, &in, &out, NULL, NULL) == TMD_E_ARG);
    EXPECT(tmd_decode_shapes(NULL, &sh, &in, &out, NULL, NULL) == TMD_E_ARG);
    EXPECT(tmd_decode_static(NULL, &sh, &in, &out, NULL) == TMD_E_ARG);
    uint32_t fl = 0;
    EXPECT(tmd_status(NULL, 0, &fl) == TMD_E_ARG);
    tmd_free(NULL);
    tmd_pipe_t *pipe = NULL;
    EXPECT(tmd_pipe_create(NULL, 1, &p, &pipe) == TMD_E_ARG);
    EXPECT(tmd_pipe_create(&sh, 0, &p, &pipe) == TMD_E_ARG);
    EXPECT(tmd_pipe_create(&sh, TMD_PIPE_MAX_DEPTH + 1u, &p, &pipe) == TMD_E_ARG);
    EXPECT(tmd_pipe_run(NULL, 1, &sh, &in, &out, &fl) == TMD_E_ARG);
    EXPECT(tmd_pipe_run_rans(NULL, 1, &sh, NULL, NULL, &out, &fl) == TMD_E_ARG);
    tmd_pipe_free(NULL);
    size_t eb = 0;
    EXPECT(tmd_encode_workspace(10, 100, 50, &eb) == TMD_OK && eb > 0);
    EXPECT(tmd_encode_workspace(10, 100, 50, NULL) == TMD_E_ARG);
    tmd_enc_in ein;
    tmd_enc_out eout;
    memset(&ein, 0, sizeof(ein));
    memset(&eout, 0, sizeof(eout));
    EXPECT(tmd_encode(NULL, &ein, &eout, NULL, 0, NULL) == TMD_E_ARG);
    size_t rb = 0;
    EXPECT(tmd_rans_workspace(&sh, 1, &rb) == TMD_OK && rb > 0);
    EXPECT(tmd_rans_workspace(NULL, 1, &rb) == TMD_E_ARG);
    EXPECT(tmd_rans_workspace(&sh, 0, &rb) == TMD_E_ARG);
    EXPECT(tmd_decode_rans(NULL, &sh, NULL, NULL, &out, NULL, NULL, NULL) == TMD_E_ARG);
    uint64_t bound = 0;
    EXPECT(tmd_rans_encode_workspace(&sh, &rb, &bound) == TMD_OK && rb > 0 && bound > 376);
    EXPECT(tmd_rans_encode_workspace(&sh, NULL, &bound) == TMD_E_ARG);
    tmd_frame_shape huge = {10, (1u << 30) + 1u, 0};
    EXPECT(tmd_rans_encode_workspace(&huge, &rb, &bound) == TMD_E_ARG);
    static uint64_t word;
    static unsigned char area[512] __attribute__((aligned(256)));
    EXPECT(tmd_encode_rans(NULL, &in, area, 512, &word, area, NULL) == TMD_E_ARG);
    EXPECT(tmd_encode_rans(&sh, &in, area, 512, &word, area, NULL) == TMD_E_CAPACITY);
    EXPECT(tmd_set_schedule(NULL, 64, 0) == TMD_E_ARG);
    EXPECT(tmd_set_profiling(NULL, 1u) == TMD_E_ARG);
    EXPECT(tmd_stage_times(NULL, NULL, 0, NULL) == TMD_E_ARG);
    EXPECT(strcmp(tmd_stage_name(0), "tilesum") == 0 && strcmp(tmd_stage_name(99), "") == 0);
    EXPECT(tmd_selftest_fp(NULL, NULL, NULL, 1, NULL) == TMD_E_ARG);
    EXPECT(tmd_selftest_math(NULL, NULL, 1, NULL) == TMD_E_ARG);
    EXPECT(tmd_selftest_sqrt(2, 1, NULL, NULL) == TMD_E_ARG);
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
