/*
 * gee_oracle.c - plain, slow FP64 reference of the sparse Graph Encoder Embedding.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code, header, table or constant with the HIP implementation.
 *
 * What it computes (Qin & Shen, "Efficient Graph Encoder Embedding for Large Sparse
 * Graphs in Python"):
 *   - Section 2: W is the N x K normalized one-hot label matrix, row j holding 1/n_k in
 *     column k = y_j, with n_k the number of nodes of class k; the embedding is
 *     Z = A W (Eq. 1), i.e. Z_i^k = sum over neighbours j of i with label k of
 *     e_ij * W_j^k, evaluated as one pass over the edge list (the original GEE form).
 *   - Section 2 options / Table 1: diagonal augmentation replaces A by A + I;
 *     Laplacian normalization replaces A by D^-1/2 A D^-1/2 with D the degree matrix;
 *     correlation divides every row of Z by its 2-norm.
 *
 * Readings taken where the paper is silent (each is listed in the design notes):
 *   - SYMMETRIZE: an input row (s, d, w) stands for A[s,d] and A[d,s]; a self-loop
 *     (s == d) contributes A[s,s] = w once.  Without it each row is the single
 *     directed entry A[s,d].
 *   - repeated rows add up (A[s,d] is the sum of its rows).
 *   - label -1 means unknown: W row is zero, the node is not counted in any n_k, but it
 *     still has a degree and its own Z row is computed.
 *   - a class with n_k = 0 gives an all-zero column.
 *   - diagonal augmentation is applied first and the Laplacian then uses the degrees of
 *     A + I (row sums, weighted).
 *   - "D the degree matrix" names no side for a directed graph. By default both factors
 *     take the row sums (out-degrees). With the directed-degree option the left factor
 *     takes each node's out-degree (row sum) and the right factor its in-degree (column
 *     sum): D_out^-1/2 A D_in^-1/2, both with A + I under augmentation. For a symmetric A
 *     the two coincide.
 *   - a node with degree <= 0 gets D^-1/2 = 0.
 *   - correlation is a plain row 2-norm division (no centering); zero rows stay zero.
 *
 * Return codes: 0 ok, -1 bad argument, -2 label outside [-1, K), -3 node index outside
 * [0, N), -4 non-finite weight, -6 out of host memory.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_DIAG 1u
#define OR_LAPLACIAN 2u
#define OR_CORRELATION 4u
#define OR_SYMMETRIZE 8u
#define OR_DIRECTED_DEGREES 16u

/* Class sizes n_k = #{j : y_j = k} (Section 2). Also checks the label range. */
int gee_oracle_class_counts(const int32_t *labels, int64_t N, int32_t K, int64_t *counts)
{
    if (N < 0 || K < 1 || (N > 0 && !labels) || !counts)
        return -1;
    for (int32_t k = 0; k < K; ++k)
        counts[k] = 0;
    for (int64_t j = 0; j < N; ++j) {
        int32_t y = labels[j];
        if (y < -1 || y >= K)
            return -2;
        if (y >= 0)
            counts[y] += 1;
    }
    return 0;
}

/* The list of adjacency entries (row i, column j, value v) that A (or A + I) is made of. */
typedef struct {
    int64_t *i;
    int64_t *j;
    double *v;
    int64_t n;
} entry_list;

static int build_entries(const int32_t *src, const int32_t *dst, const double *w, int64_t E,
                         int64_t N, uint32_t flags, entry_list *L)
{
    int64_t cap = 2 * E + N + 1;
    L->i = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    L->j = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    L->v = (double *)malloc(sizeof(double) * (size_t)cap);
    L->n = 0;
    if (!L->i || !L->j || !L->v)
        return -6;
    for (int64_t e = 0; e < E; ++e) {
        int64_t s = src[e], d = dst[e];
        double val = w ? w[e] : 1.0;
        if (s < 0 || s >= N || d < 0 || d >= N)
            return -3;
        if (!isfinite(val))
            return -4;
        /* the row itself: A[s, d] */
        L->i[L->n] = s;
        L->j[L->n] = d;
        L->v[L->n] = val;
        L->n++;
        /* undirected input: the mirror entry A[d, s], once for a self-loop */
        if ((flags & OR_SYMMETRIZE) && s != d) {
            L->i[L->n] = d;
            L->j[L->n] = s;
            L->v[L->n] = val;
            L->n++;
        }
    }
    /* diagonal augmentation: A + I */
    if (flags & OR_DIAG) {
        for (int64_t i = 0; i < N; ++i) {
            L->i[L->n] = i;
            L->j[L->n] = i;
            L->v[L->n] = 1.0;
            L->n++;
        }
    }
    return 0;
}

static void free_entries(entry_list *L)
{
    free(L->i);
    free(L->j);
    free(L->v);
}

/*
 * Degrees of the (possibly augmented) adjacency: d_i = sum of the values in row i.
 * Exposed for tests. `deg` has N slots.
 */
int gee_oracle_degrees(const int32_t *src, const int32_t *dst, const double *w, int64_t E,
                       int64_t N, uint32_t flags, double *deg)
{
    if (E < 0 || N < 0 || (E > 0 && (!src || !dst)) || (N > 0 && !deg))
        return -1;
    entry_list L;
    int rc = build_entries(src, dst, w, E, N, flags, &L);
    if (rc == 0) {
        for (int64_t i = 0; i < N; ++i)
            deg[i] = 0.0;
        for (int64_t t = 0; t < L.n; ++t)
            deg[L.i[t]] += L.v[t];
    }
    free_entries(&L);
    return rc;
}

/*
 * In-degrees of the (possibly augmented) adjacency: the column sums, din_j = sum of the
 * values in column j. Exposed for tests. `deg` has N slots.
 */
int gee_oracle_in_degrees(const int32_t *src, const int32_t *dst, const double *w, int64_t E,
                          int64_t N, uint32_t flags, double *deg)
{
    if (E < 0 || N < 0 || (E > 0 && (!src || !dst)) || (N > 0 && !deg))
        return -1;
    entry_list L;
    int rc = build_entries(src, dst, w, E, N, flags, &L);
    if (rc == 0) {
        for (int64_t j = 0; j < N; ++j)
            deg[j] = 0.0;
        for (int64_t t = 0; t < L.n; ++t)
            deg[L.j[t]] += L.v[t];
    }
    free_entries(&L);
    return rc;
}

/*
 * The embedding Z (row-major N x K, float64), with the options of Section 2 / Table 1.
 */
int gee_oracle_embed(const int32_t *src, const int32_t *dst, const double *w, int64_t E,
                     int64_t N, const int32_t *labels, int32_t K, uint32_t flags, double *Z)
{
    if (E < 0 || N < 0 || K < 1 || (E > 0 && (!src || !dst)) || (N > 0 && (!labels || !Z)))
        return -1;
    if (flags & ~(OR_DIAG | OR_LAPLACIAN | OR_CORRELATION | OR_SYMMETRIZE | OR_DIRECTED_DEGREES))
        return -1;

    /* n_k and the non-zero value of each W row (Section 2). */
    int64_t *nk = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    if (!nk)
        return -6;
    int rc = gee_oracle_class_counts(labels, N, K, nk);
    if (rc != 0) {
        free(nk);
        return rc;
    }

    entry_list L;
    rc = build_entries(src, dst, w, E, N, flags, &L);
    if (rc != 0) {
        free_entries(&L);
        free(nk);
        return rc;
    }

    /* Laplacian normalization: v_ij <- v_ij * d_i^-1/2 * d_j^-1/2 with d the row sums;
       with directed degrees the column factor takes the in-degree (column sum) of j:
       v_ij <- v_ij * dout_i^-1/2 * din_j^-1/2. */
    if (flags & OR_LAPLACIAN) {
        size_t n1 = (size_t)(N > 0 ? N : 1);
        double *deg = (double *)calloc(n1, sizeof(double));
        double *dinv = (double *)calloc(n1, sizeof(double));
        double *degc = (double *)calloc(n1, sizeof(double));
        double *dinvc = (double *)calloc(n1, sizeof(double));
        if (!deg || !dinv || !degc || !dinvc) {
            free(deg);
            free(dinv);
            free(degc);
            free(dinvc);
            free_entries(&L);
            free(nk);
            return -6;
        }
        for (int64_t t = 0; t < L.n; ++t)
            deg[L.i[t]] += L.v[t];
        for (int64_t t = 0; t < L.n; ++t)
            degc[L.j[t]] += L.v[t];
        for (int64_t i = 0; i < N; ++i)
            dinv[i] = deg[i] > 0.0 ? 1.0 / sqrt(deg[i]) : 0.0;
        for (int64_t j = 0; j < N; ++j) {
            if (flags & OR_DIRECTED_DEGREES)
                dinvc[j] = degc[j] > 0.0 ? 1.0 / sqrt(degc[j]) : 0.0;
            else
                dinvc[j] = dinv[j];
        }
        for (int64_t t = 0; t < L.n; ++t)
            L.v[t] = L.v[t] * dinv[L.i[t]] * dinvc[L.j[t]];
        free(deg);
        free(dinv);
        free(degc);
        free(dinvc);
    }

    /* Z = A W, one pass over the entries: Z[i, y_j] += v_ij * (1 / n_{y_j}). */
    for (int64_t t = 0; t < N * (int64_t)K; ++t)
        Z[t] = 0.0;
    for (int64_t t = 0; t < L.n; ++t) {
        int64_t i = L.i[t], j = L.j[t];
        int32_t k = labels[j];
        if (k < 0)
            continue; /* unknown label: zero row of W */
        Z[i * K + k] += L.v[t] * (1.0 / (double)nk[k]);
    }

    /* Correlation: each row divided by its 2-norm. */
    if (flags & OR_CORRELATION) {
        for (int64_t i = 0; i < N; ++i) {
            double ss = 0.0;
            for (int32_t k = 0; k < K; ++k)
                ss += Z[i * K + k] * Z[i * K + k];
            if (ss > 0.0) {
                double r = sqrt(ss);
                for (int32_t k = 0; k < K; ++k)
                    Z[i * K + k] /= r;
            }
        }
    }

    free_entries(&L);
    free(nk);
    return 0;
}
