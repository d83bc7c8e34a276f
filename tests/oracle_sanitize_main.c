/* Driver for the sanitizer check of the oracle (tests/test_oracle_sanitize.py):
 * links oracle.c built with -fsanitize=address,undefined and runs every
 * entry point on small ragged shapes. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t rc[30][12];
    uint64_t mds[12][12];
} oracle_params;

void oracle_permute(const oracle_params *prm, uint64_t *states, size_t n, int threads);
void oracle_merkle_build(const oracle_params *prm, const uint64_t *leaves, size_t n_rows, size_t n_cols,
                         uint64_t *nodes_out, int threads);
size_t oracle_merkle_num_nodes(size_t n);
void oracle_field_array(int op, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t n);

int main(void) {
    static oracle_params prm;
    for (int r = 0; r < 30; r++)
        for (int i = 0; i < 12; i++) prm.rc[r][i] = 0x9E3779B97F4A7C15ull * (uint64_t)(r * 12 + i + 1) % 0xFFFFFFFF00000001ull;
    for (int i = 0; i < 12; i++)
        for (int j = 0; j < 12; j++) prm.mds[i][j] = 1 + (uint64_t)((j - i + 12) % 12);
    uint64_t st[5 * 12];
    for (int i = 0; i < 60; i++) st[i] = (uint64_t)i * 0x1234567ull;
    oracle_permute(&prm, st, 5, 3);
    const size_t shapes[][2] = {{1, 1}, {3, 9}, {37, 17}, {64, 8}};
    for (size_t s = 0; s < 4; s++) {
        size_t n = shapes[s][0], w = shapes[s][1];
        uint64_t *lv = (uint64_t *)malloc(n * w * sizeof(uint64_t));
        for (size_t i = 0; i < n * w; i++) lv[i] = i * 0x9E3779B97F4A7C15ull % 0xFFFFFFFF00000001ull;
        size_t nn = oracle_merkle_num_nodes(n);
        uint64_t *nodes = (uint64_t *)malloc(nn * 4 * sizeof(uint64_t));
        oracle_merkle_build(&prm, lv, n, w, nodes, 4);
        free(lv);
        free(nodes);
    }
    uint64_t a[7] = {0, 1, 2, 0xFFFFFFFF, 0xFFFFFFFF00000000ull, 0xFFFFFFFF00000000ull, 5}, out[7];
    for (int op = 0; op < 7; op++) oracle_field_array(op, a, a, out, 7);
    printf("sanitized oracle ok\n");
    return 0;
}
