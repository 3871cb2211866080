/*
 * gee.h - C ABI of the MI355X (gfx950) sparse Graph Encoder Embedding library.
 *
 * The library computes the embedding of Qin & Shen, "Efficient Graph Encoder
 * Embedding for Large Sparse Graphs in Python":
 *   Section 2: W is the N x K normalized one-hot label matrix (row j holds 1/n_k in
 *   column k = y_j, with n_k the number of nodes labelled k) and Z = A W (Eq. 1),
 *   Z_i^k = sum over neighbours j of i with label k of e_ij / n_k.
 *   Section 2 options, Table 1: diagonal augmentation (A + I), Laplacian
 *   normalization (D^-1/2 A D^-1/2) and correlation (each row of Z divided by its
 *   2-norm).
 *   Section 3: the adjacency is held in CSR (index_pointers of N + 1 entries, then
 *   col_indices and data row by row).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer on the current HIP device, owned by
 *     the caller. The library never frees, retains or reads caller memory after the
 *     call's work on `stream` has completed.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). All
 *     work is enqueued asynchronously on it; inputs must stay valid and outputs must
 *     not be read until the stream reaches that point.
 *   - Node ids, labels and CSR indices are int32; E and M (entry counts) are int64.
 *     Weights and Z are float32; Z is row-major N x K and is fully overwritten.
 *   - Label -1 means "unknown": the node contributes a zero W row and is counted in
 *     no class, but it keeps its degree and gets its own Z row.
 *   - Return value: GEE_OK or a negative gee_status. An argument error is detected
 *     on the host before anything is enqueued. A data error found on the device
 *     (a label outside [-1, K), a node index outside [0, N), a non-finite weight, a
 *     malformed CSR) never makes a kernel read or write out of bounds: the offending
 *     item is skipped, Z is then unspecified, and a sticky bit is raised in the data-error
 *     word of the call's stream, which gee_get_data_errors(stream) reads and clears.
 *     Each stream of a device has a word of its own (up to 1023 streams per device; any
 *     further streams share one more word), so an error is reported on the stream whose
 *     call found it and on no other. A call recorded into a graph by stream capture
 *     reports to the word of the stream it was captured on.
 *   - Results are deterministic: the same inputs give bitwise identical Z, CSR and
 *     class counts on every call. No floating-point global atomics are used. The one
 *     exception is gee_embed_atomic (the original, edge-list form of the method), whose Z
 *     may differ from call to call in the last bits.
 *   - Calls on different streams may run concurrently.
 */
#ifndef GEE_H
#define GEE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GEE_ABI_VERSION 1

/* Option bits (Section 2 options; Table 1 rows). */
#define GEE_DIAG (1u << 0)        /* A -> A + I */
#define GEE_LAPLACIAN (1u << 1)   /* A -> D^-1/2 A D^-1/2, D = row sums of A (+ I) */
#define GEE_CORRELATION (1u << 2) /* each row of Z divided by its 2-norm (zero rows stay 0) */
#define GEE_SYMMETRIZE (1u << 3)  /* each input row (s, d, w) is an undirected edge:
                                     A[s,d] and A[d,s] (a self-loop once) */
#define GEE_DIRECTED_DEGREES (1u << 4) /* with GEE_LAPLACIAN on directed input: the left factor
                                     takes each node's out-degree (row sum of A, + 1 with
                                     GEE_DIAG) and the right factor its in-degree (column sum):
                                     D_out^-1/2 A D_in^-1/2 (Section 2 options, Table 1: the
                                     paper's "degree matrix" names no side for a directed
                                     graph). Without it both sides take the row sums. No effect
                                     with GEE_SYMMETRIZE (A is symmetric) or without the
                                     Laplacian. The edge-list entry points compute the column
                                     sums from one more partition pass over the transposed
                                     entries; gee_embed_csr returns GEE_ERR_UNSUPPORTED for it
                                     (a resident CSR has no column sums), and so do graphs past
                                     the bucket path's limit (2^22 rows) */
#define GEE_NO_VALIDATE (1u << 8) /* skip the checks that only report (non-finite weights)
                                     and raise no data-error bits; items that would address
                                     memory out of bounds (indices, labels) are still skipped,
                                     silently, and Z is then unspecified */

/* Status codes. */
typedef enum {
    GEE_OK = 0,
    GEE_ERR_ARG = -1,         /* bad argument (NULL, negative size, unknown flag bit, ...) */
    GEE_ERR_LABEL = -2,       /* (data error bit) label outside [-1, K) */
    GEE_ERR_INDEX = -3,       /* (data error bit) node index outside [0, N) */
    GEE_ERR_WEIGHT = -4,      /* (data error bit) non-finite weight */
    GEE_ERR_TOO_LARGE = -5,   /* sizes beyond what the library supports (see below) */
    GEE_ERR_OOM = -6,         /* device allocation failed */
    GEE_ERR_HIP = -7,         /* a HIP runtime call failed */
    GEE_ERR_UNSUPPORTED = -8, /* valid request the library does not implement */
    GEE_ERR_WORKSPACE = -9,   /* caller workspace too small */
    GEE_ERR_SCRATCH = -10     /* gee_embed_noalloc: the request's workspace exceeds the
                                 library's fixed scratch (gee_scratch_bytes) */
} gee_status;

/* Device data-error bits returned by gee_get_data_errors. */
#define GEE_DATA_LABEL (1u << 0)
#define GEE_DATA_INDEX (1u << 1)
#define GEE_DATA_WEIGHT (1u << 2)
#define GEE_DATA_CSR (1u << 3)
/* Raised only by builds with GEE_DEBUG=1 (internal-consistency checks of the kernels' own
   index arithmetic): a computed LDS slot or staging/output position outside its array was
   skipped. Never raised by a release build. */
#define GEE_DATA_INTERNAL (1u << 30)

/* Limits of the library: N <= 2^24, K <= 128, CSR entries M < 2^31 - 2^16.
   (M = 2E minus self-loops under GEE_SYMMETRIZE, else E.) */
#define GEE_MAX_NODES (1 << 24)
#define GEE_MAX_CLASSES 128

/* Launch schedule of the embedding kernels. A zero field takes the library's
   default for the graph's size. Schedules change speed, never results except for
   floating-point rounding order (a schedule is chosen from the graph's own sizes, so
   a graph embedded alone or inside a batch with the same schedule is bit-identical). */
typedef struct {
    int32_t wave_entries;   /* entries per wavefront in the embed kernel (power of 2, 256..16384);
                               on the bucket path (below) the entries of a bucket part, at least
                               2048 (0: the largest power of two up to 8192 that leaves at
                               least 2048 parts of the graph's CSR entries) */
    int32_t waves_per_block;/* wavefronts per workgroup in the embed kernel (1, 2 or 4) */
    int32_t tile_entries;   /* entries per workgroup tile of the CSR partition passes; this
                               library supports only 4096 (0 = default) */
    int32_t bucket_rows_log2; /* rows per CSR sort bucket = 2^this (0 = automatic, else 1..12;
                                 raised to what keeps the bucket count <= 65536); on the
                                 bucket path 5 or 6 chooses 32- or 64-row buckets (raised to
                                 64 when 32 would need more than 65536), other values leave
                                 the choice to the class-count rule */
} gee_schedule;
/* Paths. gee_embed, gee_embed_ws and batches take the bucket path whenever the launch's
   rows fit 65536 buckets of 64 rows (2^22 rows, batch graphs each rounded up to the
   bucket size): the entries are partitioned into buckets of 64 consecutive rows (32 when a
   graph has K > 64 and 32 rows suffice) and every bucket's class sums are accumulated
   whole, without building the CSR. Larger launches, and gee_embed_csr, take the CSR path.
   Batches run as chunks that give every graph the path and bucket size it gets alone, so a
   graph's Z is bitwise the same alone and in any batch. */

int gee_abi_version(void);
const char *gee_status_string(int status);
/* Text of the HIP runtime error behind the last GEE_ERR_HIP (or GEE_ERR_OOM) returned on
   the calling thread; "" if there was none. The string is static (owned by HIP). */
const char *gee_last_hip_error(void);

/* Per-device set-up: finds the device addresses of the library's data-error words and
   fixed scratch on the current device. Allocates nothing. Called lazily by every entry
   point; call it once up front on each device when later calls run under stream capture. */
int gee_init(void);

/* Takes (reads and clears, atomically and in stream order) the sticky data-error bits
   (GEE_DATA_*) of `stream` on the current device and waits for `stream` to reach that point.
   Bits raised by calls on other streams are not seen and not cleared. */
int gee_get_data_errors(void *stream, uint32_t *bits);
/* The same take without waiting: enqueues on `stream` a kernel that moves the stream's
   data-error bits into *dst and clears the word. dst must be device-writable at the same
   address (device memory, or pinned host memory from hipHostMalloc); *dst holds the bits of
   the calls enqueued on `stream` before this one once the stream has passed this point
   (for example once an event recorded after it has completed). For serving loops that
   read the bits of each batch without a stream synchronization. */
int gee_take_data_errors_async(void *stream, uint32_t *dst);

/* Profiling hook (for benchmarks and tests). From this call on, every launch of the named
   kernel records hipEvent `start_event` on its stream right before the launch and
   `stop_event` right after (both hipEvent_t passed as void*; both NULL removes the hook).
   Kernel names:
     class counts: "class_count_partial", "class_count_final";
     partition passes: "a_hist", "digit_scan", "a_scatter", "b_hist", "b_scan", "b_scatter",
       "c_tiles", "c_hist", "c_scan", "c_scatter", "bucket_sort";
     CSR path: "graph_meta", "zero_steps", "node_rows", "degree_rows", "degree_fixup",
       "node_coef", "fill_empty", "embed_rows", "embed_fixup";
     bucket path (gee_embed and batches): "bucket_part_count", "bucket_part_fill",
       "bucket_degree", "bucket_degree_fix", "bucket_embed", "bucket_embed_fix";
     resident CSR on the bucket kernels (gee_embed_csr): "csr_prep";
     original GEE form (gee_embed_atomic): "edge_init", "edge_prep", "edge_coef",
       "edge_scatter", "edge_finish";
     sparse Z (gee_embed_sparse): "zs_count" or "zs_tile_sum" (the row counts' tile sums),
       "zs_write" (the compaction, or the placement of the staged pairs).
   Launches recorded into a batch plan's hipGraph are not hooked. The caller owns the
   events and keeps them alive while the hook is set. Returns GEE_ERR_ARG for an unknown
   name. Process-wide; not meant for concurrent use from several threads. */
int gee_profile_kernel(const char *kernel, void *start_event, void *stop_event);

/* Default schedule for a graph of these sizes. */
int gee_default_schedule(int64_t E, int32_t N, int32_t K, uint32_t flags, gee_schedule *out);

/* ---------------------------------------------------------------------------------
 * gee_class_counts - n_k = #{j : labels[j] = k} for k in [0, K) (Section 2).
 *   labels : int32[N] device, values in [-1, K)
 *   counts : int32[K] device, output (exact integers)
 * Out-of-range labels are counted nowhere and raise GEE_DATA_LABEL. */
int gee_class_counts(const int32_t *labels, int32_t N, int32_t K, int32_t *counts, void *stream);

/* ---------------------------------------------------------------------------------
 * gee_build_csr - edge list -> CSR (Section 3 layout), built on the device by a stable
 * sort on the row index (two partition passes, then a sort inside buckets of rows).
 *   src, dst : int32[E] device, node ids in [0, N)
 *   w        : float32[E] device weights, or NULL (every weight is 1)
 *   flags    : only GEE_SYMMETRIZE is meaningful here
 *   row_ptr  : int32[N + 1] device output; row_ptr[N] = M, the number of entries
 *   col      : int32[capacity] device output, capacity = gee_csr_capacity(E, flags)
 *   val      : float32[capacity] device output, or NULL when w is NULL
 * Canonical order: row i lists, in increasing input row index e, the other endpoint of
 * every input row with src = i (and, under GEE_SYMMETRIZE, with dst = i); for one e the
 * (src,dst) entry precedes its mirror; a self-loop appears once; val holds the input
 * weight bits unchanged. Rows with an out-of-range endpoint are dropped (GEE_DATA_INDEX).
 * gee_build_csr allocates its scratch with hipMallocAsync on `stream`; the _ws variant
 * uses caller scratch of gee_build_csr_workspace_bytes() bytes instead. */
int64_t gee_csr_capacity(int64_t E, uint32_t flags);
size_t gee_build_csr_workspace_bytes(int64_t E, int32_t N, uint32_t flags, const gee_schedule *sched);
int gee_build_csr(const int32_t *src, const int32_t *dst, const float *w, int64_t E, int32_t N,
                  uint32_t flags, int32_t *row_ptr, int32_t *col, float *val, void *stream);
int gee_build_csr_ws(const int32_t *src, const int32_t *dst, const float *w, int64_t E, int32_t N,
                     uint32_t flags, int32_t *row_ptr, int32_t *col, float *val,
                     const gee_schedule *sched, void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * gee_embed - the whole path, edge list -> Z (Eq. 1 with the Table 1 options).
 *   src, dst : int32[E] device edge list, node ids in [0, N)
 *   w        : float32[E] device weights, or NULL (every weight is 1)
 *   labels   : int32[N] device, values in [-1, K)
 *   flags    : GEE_DIAG | GEE_LAPLACIAN | GEE_CORRELATION | GEE_SYMMETRIZE
 *   Z        : float32[N * K] device output, row-major
 * Steps, all on the device: class counts, CSR build, degrees (Laplacian), the
 * per-row class scatter with the rescale and diagonal term fused, correlation.
 * Diagonal augmentation is applied before the Laplacian (degrees are those of A + I).
 * gee_embed allocates its scratch with hipMallocAsync/hipFreeAsync on `stream`; the
 * _ws variant takes caller scratch of gee_embed_workspace_bytes() bytes and a schedule
 * (NULL = default) and allocates nothing. */
size_t gee_embed_workspace_bytes(int64_t E, int32_t N, int32_t K, uint32_t flags, int weighted,
                                 const gee_schedule *sched);
int gee_embed(const int32_t *src, const int32_t *dst, const float *w, int64_t E, int32_t N,
              const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *stream);
int gee_embed_ws(const int32_t *src, const int32_t *dst, const float *w, int64_t E, int32_t N,
                 const int32_t *labels, int32_t K, uint32_t flags, float *Z,
                 const gee_schedule *sched, void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * gee_embed_noalloc - gee_embed for callers that cannot allocate device memory: code under
 * stream capture (HIP graphs), tight serving loops, harnesses that forbid allocation.
 *   Arguments, results, determinism and data errors: exactly those of gee_embed (the same
 *   kernels; Z is bitwise the Z of gee_embed_ws with the default schedule).
 *   Workspace: the library's fixed scratch, a file-scope device array of gee_scratch_bytes()
 *   bytes (256 MiB) that every device the library runs on holds until the process ends. The
 *   call allocates nothing. A request whose gee_embed_workspace_bytes() (default schedule)
 *   exceeds it returns GEE_ERR_SCRATCH and enqueues nothing: up to about 12.8M CSR entries
 *   unweighted or 7.6M weighted fit at K = 50 (M = 2E under GEE_SYMMETRIZE; the 10,000-node
 *   SBM graph of 5.57M edges needs 92 MiB).
 *   Concurrency: every call on one device uses the same scratch, so calls whose work
 *   overlaps on one device (different streams, or host threads) race and give wrong
 *   results; order them on one stream or synchronize between them. Nothing in the scratch
 *   needs to start at zero, so the contents a previous call left do not matter.
 * Call gee_init() once on the device before capturing a call into a graph. */
size_t gee_scratch_bytes(void);
int gee_embed_noalloc(const int32_t *src, const int32_t *dst, const float *w, int64_t E, int32_t N,
                      const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *stream);

/* ---------------------------------------------------------------------------------
 * gee_embed_csr - Z from a resident CSR (for example one built by gee_build_csr).
 *   row_ptr : int32[N + 1] device, non-decreasing, row_ptr[0] = 0, row_ptr[N] = M
 *   col     : int32[M] device, column indices in [0, N)
 *   val     : float32[M] device, or NULL (every value is 1)
 *   M       : number of entries (must equal row_ptr[N])
 *   labels, K, flags, Z : as for gee_embed (GEE_SYMMETRIZE is ignored: the CSR
 *             already holds both directions when wanted)
 * Columns outside [0, N) are skipped and raise GEE_DATA_CSR. */
size_t gee_embed_csr_workspace_bytes(int64_t M, int32_t N, int32_t K, uint32_t flags,
                                     const gee_schedule *sched);
int gee_embed_csr(const int32_t *row_ptr, const int32_t *col, const float *val, int64_t M, int32_t N,
                  const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *stream);
int gee_embed_csr_ws(const int32_t *row_ptr, const int32_t *col, const float *val, int64_t M,
                     int32_t N, const int32_t *labels, int32_t K, uint32_t flags, float *Z,
                     const gee_schedule *sched, void *workspace, size_t workspace_bytes,
                     void *stream);

/* ---------------------------------------------------------------------------------
 * gee_embed_sparse - gee_embed with Z returned in sparse storage, as the paper keeps the
 * embedding matrix (Section 3: a CSR of index pointers, column indices and data; most
 * entries of Z are zero, since W is one-hot).
 *   src, dst, w, E, N, labels, K, flags : as for gee_embed (N * K must be below 2^31)
 *   row_ptr  : int32[N + 1] device output; row i's non-zero entries of Z are entries
 *              row_ptr[i] .. row_ptr[i+1]-1; row_ptr[N] = nnz, the number of non-zero entries
 *   col      : int32[capacity] device output, the class k of each entry, increasing in a row
 *   val      : float32[capacity] device output, Z[i, k] (exactly the values gee_embed writes)
 *   capacity : entries col and val can hold. Only the first min(nnz, capacity) entries are
 *              written; row_ptr is always complete, so a caller that finds row_ptr[N] >
 *              capacity can call again with larger arrays (capacity N * K always suffices).
 *              capacity 0 with col and val NULL computes row_ptr alone.
 * An entry is stored when its float32 value is not zero (a -0.0 is not stored).
 * gee_embed_sparse allocates its scratch (which includes room for twice a dense Z's bytes:
 * the class-scatter kernels stage each bucket's non-zero (class, value) pairs there, or write
 * a dense Z for graphs above 2^22 rows) with hipMallocAsync / hipFreeAsync on `stream`; the
 * _ws variant takes caller scratch of gee_embed_sparse_workspace_bytes() bytes (0 for
 * invalid sizes) and a schedule. */
size_t gee_embed_sparse_workspace_bytes(int64_t E, int32_t N, int32_t K, uint32_t flags, int weighted,
                                        const gee_schedule *sched);
int gee_embed_sparse(const int32_t *src, const int32_t *dst, const float *w, int64_t E, int32_t N,
                     const int32_t *labels, int32_t K, uint32_t flags, int32_t *row_ptr, int32_t *col,
                     float *val, int64_t capacity, void *stream);
int gee_embed_sparse_ws(const int32_t *src, const int32_t *dst, const float *w, int64_t E, int32_t N,
                        const int32_t *labels, int32_t K, uint32_t flags, int32_t *row_ptr, int32_t *col,
                        float *val, int64_t capacity, const gee_schedule *sched, void *workspace,
                        size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * gee_embed_atomic - the original GEE form (Section 2): Z computed straight from the edge
 * list in one pass over its rows, with no CSR and no sort, the form the paper compares
 * sparse GEE against (Section 4, Tables 3-4, Figure 3). Same result as gee_embed (Eq. 1
 * with the Table 1 options, diagonal augmentation before the Laplacian) up to float32
 * rounding, but NOT deterministic: every row adds its term to Z with a float atomic, so
 * the summation order, and the last bits of Z, may change from call to call.
 *   src, dst, w, E, N, labels, K, flags, Z : as for gee_embed
 * Steps, all on the device: Z = 0; class counts; under the Laplacian, weighted degrees by
 * float atomics (d_i = 1 + row sum under diagonal augmentation); per node s_j = d_j^-1/2
 * (0 for d_j <= 0) and c_j = s_j / n_{y_j}; per edge row Z[src, y_dst] += w c_dst (and,
 * under GEE_SYMMETRIZE, Z[dst, y_src] += w c_src, a self-loop once); per Z row the
 * diagonal term, the factor s_i and the correlation 2-norm.
 * Data errors as for gee_embed: offending rows or labels are skipped and flagged.
 * gee_embed_atomic allocates its scratch with hipMallocAsync/hipFreeAsync on `stream`; the
 * _ws variant takes caller scratch of gee_embed_atomic_workspace_bytes() bytes (0 for
 * invalid sizes) and allocates nothing. Limits as for gee_embed except that E has no
 * upper bound beyond int64 (no CSR is formed). */
size_t gee_embed_atomic_workspace_bytes(int32_t N, int32_t K, uint32_t flags);
int gee_embed_atomic(const int32_t *src, const int32_t *dst, const float *w, int64_t E, int32_t N,
                     const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *stream);
int gee_embed_atomic_ws(const int32_t *src, const int32_t *dst, const float *w, int64_t E, int32_t N,
                        const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *workspace,
                        size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * Batches: gee_embed of G independent graphs in one launch sequence. The graphs are
 * embedded as the disjoint union of their edge lists (one CSR sort, one pass of each
 * kernel over all graphs); each graph keeps its own sizes, labels, options, output and
 * schedule. Every Z of a batch is bitwise identical to that graph's gee_embed_ws with
 * the same schedule (its schedule is chosen from its own sizes, never from the batch).
 *   src, dst, w, E, N, labels, K, flags, Z : as for gee_embed, per graph
 *   sched : zero fields take the graph's defaults; waves_per_block and the CSR path's
 *           bucket_rows_log2 are taken from graph 0 for the whole batch (the bucket
 *           path's 32/64-row choice is per graph)
 * Limits: at most 2^20 graphs, 2^28 nodes and 2^31 - 2^16 CSR entries in total; each
 * graph within the single-graph limits. */
typedef struct {
    const int32_t *src, *dst;
    const float *w;
    int64_t E;
    int32_t N;
    const int32_t *labels;
    int32_t K;
    uint32_t flags;
    float *Z;
    gee_schedule sched;
} gee_graph;

/* Caller-workspace form: the graph table is copied to the device (stream-ordered) and the
 * kernels are enqueued on `stream`. The size query reads only sizes, flags, weights-or-not
 * and schedules (pointers may be NULL there); it returns 0 bytes for invalid arguments. */
size_t gee_embed_batch_workspace_bytes(const gee_graph *graphs, int32_t G);
int gee_embed_batch_ws(const gee_graph *graphs, int32_t G, void *workspace, size_t workspace_bytes,
                       void *stream);

/* Batch plan: allocates its workspace (hipMalloc) and uploads the graph table once, then
 * captures the whole launch sequence in a hipGraph. Each gee_batch_plan_launch replays it
 * on `stream` (one graph launch) and recomputes every Z from the current contents of the
 * input arrays named at creation (or at the last gee_batch_plan_update). The arrays must
 * stay allocated while the plan holds them;
 * launches of one plan must not overlap (they share the workspace). Create and destroy
 * on the device the arrays live on. Data errors found by a launch are reported on the
 * launch's stream (gee_get_data_errors). */
typedef struct gee_batch_plan gee_batch_plan;
int gee_batch_plan_create(const gee_graph *graphs, int32_t G, gee_batch_plan **plan);
/* As gee_batch_plan_create, with a workspace of at least min_workspace_bytes (room for
 * later, larger graph sets given to gee_batch_plan_update); 0 sizes it for `graphs`. */
int gee_batch_plan_create_ws(const gee_graph *graphs, int32_t G, size_t min_workspace_bytes,
                             gee_batch_plan **plan);
/* Bytes of the plan's workspace (what gee_embed_batch_workspace_bytes of a new graph set
 * may be at most for gee_batch_plan_update); 0 for NULL. */
size_t gee_batch_plan_workspace_bytes(const gee_batch_plan *plan);
/* Replaces the plan's graphs with `graphs` (any sizes, classes, options and schedules
 * within the batch limits) without allocating: the new tables are written into the plan's
 * workspace (completed before returning) and the launch sequence is captured again; the
 * executable graph takes the new kernel arguments in place when the sequence has the same
 * kernels (hipGraphExecUpdate), else it is instantiated again. Every later launch embeds
 * the new graphs, with Z bitwise equal to gee_embed_batch_ws on them. The caller must not
 * update a plan while a launch of it may still run (synchronize its stream first).
 * Returns GEE_ERR_WORKSPACE, leaving the plan unchanged, when the new set needs more than
 * gee_batch_plan_workspace_bytes; argument errors also leave it unchanged. After
 * GEE_ERR_HIP or GEE_ERR_OOM the plan cannot be launched any more and must be destroyed.
 * Call on the device the plan was created on. */
int gee_batch_plan_update(gee_batch_plan *plan, const gee_graph *graphs, int32_t G);
int gee_batch_plan_launch(gee_batch_plan *plan, void *stream);
int gee_batch_plan_destroy(gee_batch_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* GEE_H */
