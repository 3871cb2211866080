/* Drives the C oracle over many small seeded graphs (every option combination, self-loops,
 * repeated rows, unknown labels, empty graphs and classes, isolated nodes, signed weights,
 * invalid arguments) so that an AddressSanitizer / UndefinedBehaviorSanitizer build reports
 * any out-of-bounds access, leak or undefined operation. Exit status 0 when every call
 * returned what its arguments call for. Test infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int gee_oracle_class_counts(const int32_t *labels, int64_t N, int32_t K, int64_t *counts);
int gee_oracle_degrees(const int32_t *src, const int32_t *dst, const double *w, int64_t E, int64_t N,
                       uint32_t flags, double *deg);
int gee_oracle_in_degrees(const int32_t *src, const int32_t *dst, const double *w, int64_t E, int64_t N,
                          uint32_t flags, double *deg);
int gee_oracle_embed(const int32_t *src, const int32_t *dst, const double *w, int64_t E, int64_t N,
                     const int32_t *labels, int32_t K, uint32_t flags, double *Z);

static uint64_t state = 0x2406037260000001ull;
static uint32_t next(void) { /* xorshift64* */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (uint32_t)((state * 0x2545F4914F6CDD1Dull) >> 32);
}

int main(void) {
    int bad = 0;
    for (int trial = 0; trial < 400; ++trial) {
        const int64_t N = (trial % 17 == 0) ? 0 : 1 + next() % 40;
        const int64_t E = (N == 0 || trial % 11 == 0) ? 0 : next() % 120;
        const int32_t K = 1 + (int32_t)(next() % 9);
        int32_t *src = malloc(sizeof(int32_t) * (size_t)(E ? E : 1));
        int32_t *dst = malloc(sizeof(int32_t) * (size_t)(E ? E : 1));
        double *w = malloc(sizeof(double) * (size_t)(E ? E : 1));
        int32_t *lab = malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
        for (int64_t e = 0; e < E; ++e) {
            src[e] = (int32_t)(next() % (uint32_t)N);
            dst[e] = (trial % 5 == 0) ? src[e] : (int32_t)(next() % (uint32_t)N); /* self-loops */
            w[e] = (trial % 7 == 0) ? ((double)(next() % 200) - 100.0) / 37.0 : 1.0 - (next() % 1000) / 1000.0;
        }
        for (int64_t i = 0; i < N; ++i) lab[i] = (int32_t)(next() % (uint32_t)(K + 1)) - 1; /* -1 = unknown */
        int64_t *cnt = malloc(sizeof(int64_t) * (size_t)K);
        if (gee_oracle_class_counts(lab, N, K, cnt) != 0) bad |= 1;
        double *deg = malloc(sizeof(double) * (size_t)(N ? N : 1));
        double *Z = malloc(sizeof(double) * (size_t)((N ? N : 1) * K));
        for (uint32_t flags = 0; flags < 32; ++flags) {
            const double *wp = (flags & 1) ? w : NULL; /* weighted or not, beside the option bits */
            if (gee_oracle_degrees(src, dst, wp, E, N, flags & ~1u, deg) != 0) bad |= 2;
            if (gee_oracle_in_degrees(src, dst, wp, E, N, flags & ~1u, deg) != 0) bad |= 4;
            if (gee_oracle_embed(src, dst, wp, E, N, lab, K, flags, Z) != 0) bad |= 8;
            for (int64_t q = 0; q < N * K; ++q)
                if (!isfinite(Z[q])) bad |= 16;
        }
        /* invalid arguments are refused */
        if (N > 0) {
            lab[0] = K; /* label out of range */
            if (gee_oracle_embed(src, dst, w, E, N, lab, K, 0, Z) == 0) bad |= 32;
            lab[0] = -1;
            if (E > 0) {
                const int32_t keep = src[0];
                src[0] = (int32_t)N; /* index out of range */
                if (gee_oracle_embed(src, dst, w, E, N, lab, K, 8, Z) == 0) bad |= 64;
                src[0] = keep;
            }
        }
        if (gee_oracle_embed(src, dst, w, -1, N, lab, K, 0, Z) == 0) bad |= 128;
        if (gee_oracle_embed(src, dst, w, E, N, lab, 0, 0, Z) == 0) bad |= 256;
        if (gee_oracle_embed(src, dst, w, E, N, lab, K, 1u << 20, Z) == 0) bad |= 512;
        free(src);
        free(dst);
        free(w);
        free(lab);
        free(cnt);
        free(deg);
        free(Z);
    }
    if (bad) fprintf(stderr, "oracle driver: unexpected return codes (mask %#x)\n", bad);
    return bad ? 1 : 0;
}
