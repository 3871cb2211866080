/* Drives the library's host-side planning (launch plans, workspace carve-up, batch
 * chunking, schedule checks) through the size queries and the argument checks of the C ABI,
 * none of which touches a device, so that an AddressSanitizer / UndefinedBehaviorSanitizer
 * build of the host code reports any out-of-bounds access or undefined operation on a
 * machine without a GPU. Exit status 0 when every answer is consistent. Test
 * infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "gee.h"

static uint64_t state = 0x2406037260000002ull;
static uint32_t next(void) { /* xorshift64* */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (uint32_t)((state * 0x2545F4914F6CDD1Dull) >> 32);
}

static int64_t pick_E(void) {
    switch (next() % 5) {
    case 0: return 0;
    case 1: return next() % 100;
    case 2: return next() % 100000;
    case 3: return (int64_t)(next() % 20000000);
    default: return (int64_t)(next() % 1000000000);
    }
}

int main(void) {
    int bad = 0;
    const uint32_t opts[] = {0, GEE_SYMMETRIZE, GEE_DIAG | GEE_LAPLACIAN | GEE_CORRELATION | GEE_SYMMETRIZE,
                             GEE_LAPLACIAN | GEE_DIRECTED_DEGREES, GEE_NO_VALIDATE | GEE_SYMMETRIZE};
    for (int trial = 0; trial < 3000; ++trial) {
        const int64_t E = pick_E();
        const int32_t N = (int32_t)((trial % 13 == 0) ? next() % 3 : 1 + next() % (1u << (next() % 25)));
        const int32_t K = (int32_t)(1 + next() % 140); /* beyond 128 is refused */
        const uint32_t flags = opts[next() % 5];
        gee_schedule sc = {0, 0, 0, 0};
        if (next() % 2) {
            sc.wave_entries = (int32_t)(1u << (7 + next() % 8));
            sc.waves_per_block = (int32_t)(next() % 5);
            sc.bucket_rows_log2 = (int32_t)(next() % 13);
        }
        const size_t a = gee_embed_workspace_bytes(E, N, K, flags, (int)(next() % 2), &sc);
        const size_t b = gee_embed_workspace_bytes(E, N, K, flags, 1, NULL);
        const size_t c = gee_build_csr_workspace_bytes(E, N, flags, &sc);
        const size_t d = gee_embed_csr_workspace_bytes(E, N, K, flags, &sc);
        const size_t e = gee_embed_sparse_workspace_bytes(E, N, K, flags, 1, NULL);
        const size_t f = gee_embed_atomic_workspace_bytes(N, K, flags);
        (void)a;
        (void)c;
        (void)d;
        (void)f;
        if (K > GEE_MAX_CLASSES && b != 0) bad |= 1;
        if (e != 0 && b == 0) bad |= 2;
        gee_schedule out;
        const int rc = gee_default_schedule(E, N, K, flags, &out);
        if (rc == GEE_OK && (out.wave_entries <= 0 || out.tile_entries <= 0)) bad |= 4;
        if (gee_csr_capacity(E, flags) != ((flags & GEE_SYMMETRIZE) ? 2 * E : E)) bad |= 8;
    }
    /* batches: sizes only (pointers may be NULL in the size query) */
    for (int trial = 0; trial < 300; ++trial) {
        const int G = 1 + (int)(next() % 300);
        gee_graph *gs = calloc((size_t)G, sizeof(gee_graph));
        for (int g = 0; g < G; ++g) {
            gs[g].N = (int32_t)(1 + next() % 60000);
            gs[g].E = (int64_t)(next() % 300000);
            gs[g].K = (int32_t)(1 + next() % 128);
            gs[g].flags = opts[next() % 5];
            gs[g].w = (next() % 2) ? (const float *)16 : NULL;
            if (next() % 3 == 0) gs[g].sched.wave_entries = (int32_t)(1u << (11 + next() % 4));
            if (next() % 3 == 0) gs[g].sched.bucket_rows_log2 = (int32_t)(5 + next() % 2);
        }
        const size_t bytes = gee_embed_batch_workspace_bytes(gs, G);
        if (bytes == 0) bad |= 16;
        /* one graph alone never needs more than the whole batch */
        const size_t one = gee_embed_batch_workspace_bytes(gs, 1);
        if (one == 0 || one > bytes) bad |= 32;
        free(gs);
    }
    /* argument errors answer before any device work */
    if (gee_embed(NULL, NULL, NULL, -1, 10, NULL, 3, 0, NULL, NULL) != GEE_ERR_ARG) bad |= 64;
    if (gee_embed(NULL, NULL, NULL, 0, 10, NULL, 0, 0, NULL, NULL) != GEE_ERR_ARG) bad |= 128;
    if (gee_embed(NULL, NULL, NULL, 0, 10, NULL, 3, 1u << 30, NULL, NULL) != GEE_ERR_ARG) bad |= 256;
    if (gee_embed(NULL, NULL, NULL, 0, 10, NULL, 200, 0, NULL, NULL) != GEE_ERR_UNSUPPORTED) bad |= 512;
    if (gee_embed_batch_workspace_bytes(NULL, 3) != 0) bad |= 1024;
    for (int st = -12; st <= 1; ++st)
        if (!gee_status_string(st)) bad |= 2048;
    if (bad) fprintf(stderr, "planning driver: inconsistent answers (mask %#x)\n", bad);
    return bad ? 1 : 0;
}
