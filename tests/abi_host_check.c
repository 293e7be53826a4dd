/* Host-side checks of the C ABI from plain C, with no GPU: every argument
 * validation path of include/cellgraph.h that returns before a launch, the
 * size queries, the error text and the status strings.  Built and run by
 * tests/test_sanitizers.py under AddressSanitizer + UndefinedBehaviorSanitizer
 * (host code only).  Prints "ok" and exits 0 when every check holds. */
#include <stdio.h>
#include <string.h>

#include "cellgraph.h"

static int fails = 0;

#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++fails;                                                         \
        }                                                                    \
    } while (0)

int main(void) {
    char buf[512];
    cg_layout lay;
    size_t bytes = 0;

    CHECK((cg_version() >> 16) == 1);
    CHECK(strcmp(cg_status_string(CG_OK), "ok") == 0);
    for (int st = -8; st <= 2; ++st) CHECK(cg_status_string(st) != NULL);

    /* layouts */
    CHECK(cg_make_layout(1024, 64, &lay) == CG_OK && lay.words == 16);
    CHECK(cg_make_layout(130, 32, &lay) == CG_OK && lay.words == 5);
    CHECK(cg_make_layout(0, 64, &lay) == CG_EINVAL);
    CHECK(cg_make_layout(65536, 64, &lay) == CG_EINVAL);
    CHECK(cg_make_layout(10, 16, &lay) == CG_EINVAL);
    CHECK(cg_make_layout(10, 64, NULL) == CG_EINVAL);
    CHECK(cg_last_error(buf, sizeof buf) == CG_EINVAL && strlen(buf) > 0);
    CHECK(cg_last_error(buf, 1) == CG_EINVAL && buf[0] == 0);

    /* workspace and size queries, including every bad argument */
    CHECK(cg_make_layout(300, 64, &lay) == CG_OK);
    CHECK(cg_dedup_workspace(100000, lay, &bytes) == CG_OK && bytes > 0);
    CHECK(cg_dedup_workspace(0, lay, &bytes) == CG_OK);
    CHECK(cg_dedup_workspace(-1, lay, &bytes) == CG_EINVAL);
    CHECK(cg_dedup_workspace((int64_t)1 << 32, lay, &bytes) == CG_EINVAL);
    CHECK(cg_dedup_workspace(10, lay, NULL) == CG_EINVAL);
    CHECK(cg_dedup_dict_workspace(100000, lay, &bytes) == CG_OK && bytes > 0);

    cg_dict_params p;
    CHECK(cg_dict_params_default(&p) == CG_OK);
    CHECK(p.dir_bits == -1 && p.split_bit == -1 && p.group_max == -1 && p.path == CG_PATH_LOOKUP);
    CHECK(cg_dict_params_default(NULL) == CG_EINVAL);
    CHECK(cg_dict_size(100000, lay, &p, &bytes) == CG_OK && bytes > 0);
    CHECK(cg_dict_size(100000, lay, NULL, &bytes) == CG_OK);
    p.dir_bits = 25;
    CHECK(cg_dict_size(1000, lay, &p, &bytes) == CG_EINVAL);
    cg_dict_params_default(&p);
    p.split_bit = 301;
    CHECK(cg_dict_size(1000, lay, &p, &bytes) == CG_EINVAL);
    cg_dict_params_default(&p);
    p.kind = 9;
    CHECK(cg_dict_size(1000, lay, &p, &bytes) != CG_OK);
    cg_dict_params_default(&p);
    p.fanout_bits = 3;  /* the sorted kind has no tree */
    CHECK(cg_dict_size(1000, lay, &p, &bytes) == CG_EINVAL);
    p.kind = CG_DICT_TREE;
    CHECK(cg_dict_size(1000, lay, &p, &bytes) == CG_OK);
    p.fanout_bits = 9;
    CHECK(cg_dict_size(1000, lay, &p, &bytes) == CG_EINVAL);
    cg_dict_params_default(&p);
    p.key_bits = 40;
    CHECK(cg_dict_size(1000, lay, &p, &bytes) == CG_EINVAL);
    p.key_bits = 32;
    CHECK(cg_dict_size(1000, lay, &p, &bytes) == CG_OK);
    cg_dict_params_default(&p);
    CHECK(cg_edges_workspace_size(100000, lay, &p, 1000, &bytes) == CG_OK && bytes > 0);
    CHECK(cg_edges_workspace_size(100000, lay, NULL, -1, &bytes) == CG_EINVAL);
    CHECK(cg_edges_workspace_size(-5, lay, NULL, 10, &bytes) == CG_EINVAL);
    p.path = CG_PATH_ALLPAIRS;
    CHECK(cg_edges_workspace_size(100000, lay, &p, 1000, &bytes) == CG_OK && bytes > 0);

    /* calls refused before any launch: bad handles, NULL buffers, small workspaces */
    cg_dict d;
    memset(&d, 0, sizeof d);
    CHECK(cg_edges_workspace(&d, 10, &bytes) == CG_EINVAL);
    CHECK(cg_edges(&d, NULL, NULL, 0, NULL, NULL, NULL, 0, NULL, NULL) == CG_EINVAL);
    CHECK(cg_neighbors_d1(&d, NULL, 0, NULL, NULL, NULL, NULL) == CG_EINVAL);
    CHECK(cg_neighbors_d1(NULL, NULL, 0, NULL, NULL, NULL, NULL) == CG_EINVAL);
    CHECK(cg_pack((const uint8_t *)16, 10, 100, lay, (void *)32, NULL) == CG_EINVAL); /* stride < l */
    CHECK(cg_pack(NULL, 10, 300, lay, (void *)32, NULL) == CG_EINVAL);
    CHECK(cg_pack(NULL, -1, 300, lay, NULL, NULL) == CG_EINVAL);
    CHECK(cg_dedup_workspace(1000, lay, &bytes) == CG_OK);
    CHECK(cg_dedup((void *)16, 1000, lay, (void *)32, NULL, (int64_t *)64, (void *)128, bytes - 1, NULL) ==
          CG_EWORKSPACE);
    CHECK(cg_dedup((void *)16, 1000, lay, (void *)32, NULL, NULL, (void *)128, bytes, NULL) == CG_EINVAL);
    CHECK(cg_dict_build(NULL, NULL, 10, lay, NULL, NULL, 0, &d, NULL) != CG_OK);
    CHECK(cg_batch_layout(0, &lay) == CG_EINVAL);
    CHECK(cg_batch_layout(512, &lay) == CG_OK && lay.word_bits == 32 && lay.words == 17);
    CHECK(cg_graph_csr_workspace(-1, 10, &bytes) == CG_EINVAL);
    CHECK(cg_graph_csr_workspace(1000, 4000, &bytes) == CG_OK && bytes > 0);
    CHECK(cg_bfs_workspace(1000, &bytes) == CG_OK && bytes > 0);
    CHECK(cg_bfs_workspace(-1, &bytes) == CG_EINVAL);
    double box[6] = {0, 0, 0, -1, 1, 1}; /* lo > hi */
    CHECK(cg_make_layout(64, 64, &lay) == CG_OK);
    CHECK(cg_sample_pack((const double *)16, 10, 1, 2, box, lay, (void *)32, NULL) == CG_EINVAL);
    /* the last error text is always NUL-terminated */
    memset(buf, 'x', sizeof buf);
    cg_last_error(buf, sizeof buf);
    CHECK(memchr(buf, 0, sizeof buf) != NULL);

    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("ok\n");
    return 0;
}
