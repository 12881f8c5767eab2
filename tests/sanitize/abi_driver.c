/* Host-side paths of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_sanitizers_cpu.py): argument validation, error statuses and the
 * thread-local error message, on a machine without a GPU (calls that need the device
 * report DEVICE).  Exit status 0 when every call returns the documented status. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/vdmc.h"

static int fails = 0;
#define EXPECT(call, want)                                                                  \
    do {                                                                                    \
        vdmc_status st_ = (call);                                                           \
        if (st_ != (want)) {                                                                \
            fprintf(stderr, "%s: got %d, want %d (%s)\n", #call, st_, want, vdmc_last_error()); \
            fails++;                                                                        \
        }                                                                                   \
    } while (0)

int main(void) {
    if (vdmc_num_classes(3) != 13 || vdmc_num_classes(4) != 199 || vdmc_num_classes(5) != 9364 ||
        vdmc_num_classes(6) != -1)
        fails++;
    if (vdmc_num_classes_undirected(3) != 2 || vdmc_num_classes_undirected(4) != 6) fails++;
    uint16_t codes[199];
    uint64_t u64[16];
    int32_t i32[8];
    EXPECT(vdmc_class_codes(5, codes), VDMC_ERR_UNSUPPORTED);
    EXPECT(vdmc_class_codes(2, codes), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_class_codes(4, NULL), VDMC_ERR_INVALID_ARG);
    if (strlen(vdmc_last_error()) == 0) fails++;
    vdmc_graph g = NULL;
    int32_t s[2] = {0, 1}, d[2] = {1, 2};
    EXPECT(vdmc_build_graph(-1, 2, s, d, 0, NULL, &g), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_build_graph(4, 2, NULL, d, 0, NULL, &g), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_build_graph((int64_t)1 << 31, 2, s, d, 0, NULL, &g), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_count(NULL, 4, NULL, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_count34(NULL, NULL, NULL, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_count_range(NULL, 4, NULL, 0, 1, 0, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_shape_counts(NULL, u64), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_set_hub_threshold(NULL, 4), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_free_graph(NULL), VDMC_OK);
    EXPECT(vdmc_count_batch(NULL, 1, 4, NULL, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_count_batch(NULL, 0, 5, NULL, NULL), VDMC_OK);
    EXPECT(vdmc_count_batch(NULL, 0, 6, NULL, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_count(NULL, 5, NULL, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_count_supported(NULL, 5), -1);
    EXPECT(vdmc_class_codes_u32(5, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_class_table_u16(7, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_count_batch_noalloc(NULL, 9000, 4, NULL, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_count_batch_noalloc(NULL, 0, 4, NULL, NULL), VDMC_OK);
    EXPECT(vdmc_tune(NULL, 0, 4, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_tuned_choice(NULL, 0, 4, i32), VDMC_ERR_INVALID_ARG);
    vdmc_serve_config cfg = {0, 4};
    vdmc_server srv = NULL;
    EXPECT(vdmc_serve_create(&cfg, &srv), VDMC_ERR_INVALID_ARG);
    cfg.mem_budget_bytes = 1 << 20;
    cfg.max_inflight = 0;
    EXPECT(vdmc_serve_create(&cfg, &srv), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_serve_create(NULL, &srv), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_serve_submit(NULL, NULL, 4, NULL, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_serve_counters(NULL, u64, 10), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_serve_destroy(NULL), VDMC_OK);
    EXPECT(vdmc_edge_list(NULL, NULL, NULL), VDMC_ERR_INVALID_ARG);
    EXPECT(vdmc_count_undirected(NULL, 4, NULL, NULL), VDMC_ERR_INVALID_ARG);
    if (fails) return 1;
    printf("ABI sanitizer run ok\n");
    return 0;
}
