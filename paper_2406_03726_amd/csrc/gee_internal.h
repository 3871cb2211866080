// gee_internal.h - shared by the HIP translation units of libgee (never installed).
//
// Device helpers for 64-wide wavefronts on gfx950, the launch plan computed on the
// host from (E, N, K, flags, schedule), and the host-side launchers each .hip file
// exports.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gee {

// Option bits (same values as the public GEE_* flags).
constexpr unsigned kDiag = 1u, kLap = 2u, kCor = 4u, kSym = 8u, kDirDeg = 16u;
// A graph whose Laplacian takes in-degrees on the right (directed input with the
// directed-degree option): its column sums come from a pass over the transposed entries.
__host__ __device__ constexpr bool in_degree_pass(unsigned f) {
    return (f & kLap) && (f & kDirDeg) && !(f & kSym);
}
// Device data-error bits (same values as the public GEE_DATA_* bits).
constexpr unsigned kErrLabel = 1u, kErrIndex = 2u, kErrWeight = 4u, kErrCsr = 8u;
// GEE_NO_VALIDATE: the graph's checks raise nothing (memory-safety guards stay).
constexpr unsigned kNoValidate = 1u << 8;

constexpr int kWave = 64;
constexpr int kMaxBuckets = 65536;     // CSR buckets: 256 high digits x 256 low digits
constexpr int kMaxBucketRowsLog2 = 12; // rows per bucket (the last sort pass ranks by row)
constexpr int kMaxClasses = 128;
// Bucket path after a pass B: each entry's row inside its bucket rides in its column word
// above this many bits; the keys themselves are written only with GEE_PASSB_KEYS.
constexpr int kBucketPackShift = 22;
#ifndef GEE_PASSB_KEYS
#define GEE_PASSB_KEYS 0
#endif
#ifndef GEE_PART_TILE
#define GEE_PART_TILE 4096
#endif
constexpr int kPartTile = GEE_PART_TILE;  // entries per CSR partition tile (4 wavefronts)

// ----------------------------------------------------------------------------- wave ops

__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// Number of set bits of `mask` strictly below this lane.
__device__ __forceinline__ int count_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p ? 1 : 0); }

// Orders LDS accesses of one wavefront (LDS instructions of a wave execute in order;
// this keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// DPP lane moves (GFX9 encodings: row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143). A lane with no source (or masked off) gets `old`.
template <int CTRL, int ROWS = 0xF, bool BC = false>
__device__ __forceinline__ int dpp_i(int x, int old) {
    return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWS, 0xF, BC);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_f(float x, float old) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, ROWS,
                                                       0xF, false));
}
__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Inclusive prefix sums over the 64 lanes with DPP (no LDS round trips): shifts of
// 1, 2, 4, 8 inside each row of 16 lanes, then lane 15 of rows 0/2 into rows 1/3 and
// lane 31 into rows 2/3. Fixed combination order.
__device__ __forceinline__ int wave_scan_add(int x) {
    x += dpp_i<0x111>(x, 0);
    x += dpp_i<0x112>(x, 0);
    x += dpp_i<0x114>(x, 0);
    x += dpp_i<0x118>(x, 0);
    x += dpp_i<0x142, 0xA>(x, 0);
    x += dpp_i<0x143, 0xC>(x, 0);
    return x;
}
__device__ __forceinline__ float wave_scan_addf(float x) {
    x += dpp_f<0x111>(x, 0.0f);
    x += dpp_f<0x112>(x, 0.0f);
    x += dpp_f<0x114>(x, 0.0f);
    x += dpp_f<0x118>(x, 0.0f);
    x += dpp_f<0x142, 0xA>(x, 0.0f);
    x += dpp_f<0x143, 0xC>(x, 0.0f);
    return x;
}
// Inclusive prefix sums restarted wherever the key changes (keys non-decreasing).
__device__ __forceinline__ float wave_seg_scan_addf(float x, int key) {
#define GEE_SEG_STEP(CTRL, ROWS)                                   \
    {                                                              \
        const float xs = dpp_f<CTRL, ROWS>(x, 0.0f);               \
        const int ks = dpp_i<CTRL, ROWS>(key, INT32_MIN);          \
        x += (ks == key) ? xs : 0.0f;                              \
    }
    GEE_SEG_STEP(0x111, 0xF)
    GEE_SEG_STEP(0x112, 0xF)
    GEE_SEG_STEP(0x114, 0xF)
    GEE_SEG_STEP(0x118, 0xF)
    GEE_SEG_STEP(0x142, 0xA)
    GEE_SEG_STEP(0x143, 0xC)
#undef GEE_SEG_STEP
    return x;
}
// Sum over the whole wavefront, the same value on every lane.
__device__ __forceinline__ float wave_sum(float v) { return readlane_f(wave_scan_addf(v), 63); }
// Exclusive scan of one int per thread over a workgroup of NT threads (DPP inside each
// wavefront, then the wavefront totals); `total` is the sum. wsum needs NT/64 ints.
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int *wsum, int &total) {
    constexpr int NWV = NT / 64;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int x = wave_scan_add(v);
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NWV; ++i) {
        const int t = wsum[i];
        base += i < wv ? t : 0;
        tot += t;
    }
    total = tot;
    __syncthreads();
    return base + x - v;
}

// Workgroups of a launch are dealt to the 8 XCDs in turn (workgroup i runs on XCD i mod 8),
// and every XCD has an L2 of its own. xcd_order(i, n) renumbers the first n workgroups so
// that each XCD takes one contiguous range of tiles, in order: neighbouring tiles, whose
// output runs end and start inside the same cache lines, then meet in one L2, which merges
// those partial lines before they are written back. Workgroups i >= n keep their number.
#ifndef GEE_XCD_REMAP
#define GEE_XCD_REMAP 1
#endif
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_order(int64_t i, int64_t n) {
#if GEE_XCD_REMAP
    if (i >= n) return i;
    const int64_t x = i % kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + i / kXcds;
#else
    (void)n;
    return i;
#endif
}

__device__ __forceinline__ void raise_error(unsigned *status, unsigned bit) {
    if (status) atomicOr(status, bit);
}

// Internal-consistency checks of GEE_DEBUG=1 builds: before an LDS slot, a staging position
// or an output position that the kernels compute themselves is used, it is checked against
// its array; a violation skips the access and raises kErrInternal (GEE_DATA_INTERNAL) in the
// call's data-error word. Release builds compile the checks away (dbg_ok is true).
#ifndef GEE_DEBUG
#define GEE_DEBUG 0
#endif
constexpr unsigned kErrInternal = 1u << 30;
__device__ __forceinline__ bool dbg_ok(bool cond, unsigned *status) {
#if GEE_DEBUG
    if (!cond) raise_error(status, kErrInternal);
    return cond;
#else
    (void)cond;
    (void)status;
    return true;
#endif
}

// ----------------------------------------------------------------------------- shared by the embed paths

// Floats per slot of the embed ring: K rounded up to a multiple of 4 (16-byte rows).
__host__ __device__ constexpr int ring_stride(int K) { return (K + 3) & ~3; }
// Per-node table entry {c_i, y_i}. A node without a known label has c_i = 0 and is filed
// under class 0, so every class index read from the table lies in [0, K) and adding c_i
// there changes nothing.
__device__ __forceinline__ float2 node_info(float c, int y) {
    return make_float2(c, __int_as_float(y >= 0 ? y : 0));
}

// Buffer resource over `bytes` bytes at p (gfx9 layout: raw, stride 0). Loads past the
// end return 0 instead of touching memory; offsets are 32-bit.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *p, int64_t bytes) {
    const int64_t n = bytes < 0 ? 0 : (bytes > 0xFFFFFFFFll ? 0xFFFFFFFFll : bytes);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)(uint32_t)n, 0x00020000);
}
__device__ __forceinline__ int4 buf_i4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(int4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ float4 buf_f4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ float2 buf_f2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ unsigned buf_u32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
__device__ __forceinline__ unsigned buf_u8(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
}

// Adds xv[j] into acc[ad[j]] for the N entries of every lane of one wavefront (N <= 4)
// without LDS float atomics for most of them (those run at a small fraction of the plain
// LDS rate on gfx950): every entry with a non-zero term writes its id (N * lane + j) into
// the byte tag of its word; exactly one entry per word reads its own id back, and those
// entries (all at distinct words) add with plain reads and writes; the others then add
// with atomics. Zero terms are skipped: the sums start at +0 and never hold -0, so adding
// a zero changes nothing. The order in which a word receives its terms is fixed by the
// entries' places, so the sums are reproducible. With tmask, the tags are a hash table of
// tmask + 1 bytes indexed by word & tmask: entries of two words that share a tag can only
// lose, and losing costs an atomic, never a wrong sum.
template <int N>
__device__ __forceinline__ void lds_tag_add(float *acc, unsigned char *tag, const int (&ad)[N],
                                            const float (&xv0)[N], int lane, int tmask = -1,
                                            int limit = 0x7FFFFFFF, unsigned *status = nullptr) {
    static_assert(N <= 4, "entry ids must fit a byte");
    float xv[N];
#pragma unroll
    for (int j = 0; j < N; ++j)  // (GEE_DEBUG: words outside acc[0, limit) are dropped and reported)
        xv[j] = (xv0[j] != 0.0f && !dbg_ok(ad[j] >= 0 && ad[j] < limit, status)) ? 0.0f : xv0[j];
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (xv[j] != 0.0f) tag[ad[j] & tmask] = (unsigned char)(N * lane + j);
    wave_lds_fence();
    bool win[N];
    float old[N];
#pragma unroll
    for (int j = 0; j < N; ++j) win[j] = xv[j] != 0.0f && tag[ad[j] & tmask] == (unsigned char)(N * lane + j);
#pragma unroll
    for (int j = 0; j < N; ++j) old[j] = win[j] ? acc[ad[j]] : 0.0f;
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (win[j]) acc[ad[j]] = old[j] + xv[j];
    wave_lds_fence();
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (xv[j] != 0.0f && !win[j]) atomicAdd(&acc[ad[j]], xv[j]);
}

// s_i from a weighted degree d (plus 1 with augmentation); 0 for d <= 0.
__device__ __forceinline__ void finish_degree(int r, float d, bool diag, float *__restrict__ srow) {
    const float dd = d + (diag ? 1.0f : 0.0f);
    srow[r] = dd > 0.0f ? 1.0f / sqrtf(dd) : 0.0f;
}

// Factor that turns a row's sums u (diagonal term included) into its Z row: s_i without
// correlation; with it u/|u|, since D^-1/2 scales the whole row by s_i > 0 and the 2-norm
// removes it (a row with s_i = 0 or u = 0 stays zero).
__device__ __forceinline__ float row_factor(float s, float ss, bool cor) {
    if (!cor) return s;
    return (s > 0.0f && ss > 0.0f) ? 1.0f / sqrtf(ss) : 0.0f;
}

// ----------------------------------------------------------------------------- graphs

// One graph of a launch. A plain call is a batch of one graph; a batch is the disjoint
// union of its graphs: graph g owns rows [node_off, node_off + N) of one CSR, the virtual
// entries [voff, voff + Mcap) of its edge list (2E under symmetrization, else E), the
// classes [class_off, class_off + K) of one count array and the embed wavefronts
// [wave_off, wave_off + NWcap). Every kernel finds a work item's graph by binary search
// over the offsets and reads the graph's own sizes, options and schedule from here.
struct GDesc {
    const int *src = nullptr, *dst = nullptr;  // edge list (device)
    const float *w = nullptr;                  // weights or nullptr (every e = 1)
    const int *labels = nullptr;               // [N]
    float *Z = nullptr;                        // [N * K] row-major
    int64_t voff = 0, E = 0, Mcap = 0;
    int N = 0, node_off = 0;
    int K = 1, kp = 1, class_off = 0;  // kp: lanes per row when finishing (pow2 >= K, <= 64)
    unsigned flags = 0;                // option bits incl. symmetrize
    int weighted = 0;
    int WE = 1024, wave_off = 0, NWcap = 1;
    int64_t part_off = 0;              // first float of the graph's head/tail partial rows
    int cnt_off = 0, cnt_blocks = 1;   // class-count partial workgroups
    int64_t cpart_off = 0;             // first int of the graph's class-count partials
};

// Set on the device once the CSR exists: first entry, entry count, embed wavefronts.
struct GMeta {
    int ent_off, M, NW, pad;
};

// Kernel-side view of a launch: the descriptor table and the offset arrays (device), or,
// for a single graph, the descriptor itself (tab == nullptr, offset arrays unused).
struct Batch {
    int G = 1;
    const GDesc *tab = nullptr;
    GDesc one;
    const int *node_offs = nullptr;     // [G + 1]
    const int64_t *voffs = nullptr;     // [G + 1]
    const int *wave_offs = nullptr;     // [G + 1]
    const int *cnt_offs = nullptr;      // [G + 1]
    const int *class_offs = nullptr;    // [G + 1]
    GMeta *gm = nullptr;                // [G]
    unsigned *status = nullptr;         // the call's data-error word (kernels without their own)
};

__device__ __forceinline__ bool validates(const GDesc &d) { return !(d.flags & kNoValidate); }

// A wave-uniform 64-bit value as a scalar (its first active lane's).
__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint64_t u = (uint64_t)x;
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Last g with offs[g] <= x (offs non-decreasing, offs[0] <= x).
template <typename T>
__device__ __forceinline__ int find_graph(const T *__restrict__ offs, int G, T x) {
    if (G <= 1) return 0;
    int lo = 0, hi = G;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offs[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ GDesc load_desc(const Batch &b, int g) { return b.tab ? b.tab[g] : b.one; }

// ----------------------------------------------------------------------------- plan

// Host-side plan of a launch over the union of its graphs.
struct Plan {
    int G = 1;
    int64_t Vtot = 0;    // virtual entries (CSR capacity) over all graphs
    int64_t Ntot = 0;    // rows over all graphs
    int Kmax = 1, Kmin = 1 << 30, Ktot = 0;
    bool weighted = false;  // some graph has weights (the CSR then carries val)
    bool any_lap_w = false; // some weighted graph uses the Laplacian
    // partition (CSR build)
    int sb = 0;          // rows per bucket = 1 << sb
    int32_t B = 1;       // buckets
    int s2 = 0;          // low digit bits (pass B digits = 1 << s2; 0: no pass B)
    int DA = 1;          // pass A digits (high digit = bucket >> s2), <= 256
    int tile = kPartTile;  // entries per partition tile
    int64_t TA = 1;      // pass A tiles
    int64_t TBcap = 1;   // pass B tiles (upper bound)
    int64_t TCcap = 1;   // pass C tiles (upper bound; buckets above the staging capacity)
    // embed
    int wpb = 1;         // wavefronts per embed workgroup
    int64_t NWtot = 1;   // embed wavefronts launched (upper bound, all graphs)
    int64_t parts = 0;   // floats of head/tail partial rows (all graphs)
    int cnt_blocks = 1;  // class-count partial workgroups (all graphs)
    int64_t cparts = 0;  // ints of class-count partials (all graphs)
    // bucket path (edge lists straight to Z, gee_bucket.hip): every graph's first row is
    // aligned to the 2^sb-row buckets; bparts / bslots bound the wavefront parts and the
    // partial slots of buckets cut into several parts
    bool bucket = false;
    int64_t bparts = 0, bslots = 0;
    // every graph of the launch needs in-degrees (in_degree_pass): the partition and the
    // degree kernels run first over the transposed entries
    bool io = false;
};

// Workspace carve-up; every member is a device pointer into one caller buffer.
struct Work {
    // batch tables (G > 1); tabT: the descriptors with src and dst swapped (Plan::io)
    GDesc *tab = nullptr, *tabT = nullptr;
    int *node_offs = nullptr, *wave_offs = nullptr, *cnt_offs = nullptr, *class_offs = nullptr;
    int64_t *voffs = nullptr;
    GMeta *gm = nullptr;       // [G]
    int *counts = nullptr;     // [Ktot]
    float *inv_n = nullptr;    // [Ktot]
    int *cpart = nullptr;      // [cparts]
    int *meta = nullptr;       // [4]: M (all graphs)
    int *ghA = nullptr;        // [DA * TA] pass A tile histograms (scanned in place)
    int *totA = nullptr;       // [DA]
    int *segA = nullptr;       // [DA + 1] pass A segment starts
    int *tileB = nullptr;      // [DA + 1] first pass-B tile of each segment
    int *ghB = nullptr;        // [(1 << s2) * TBcap] pass B tile histograms
    int *segB = nullptr;       // [TBcap] segment of each pass-B tile
    int *bstart = nullptr;     // [B + 1]
    int *tileC = nullptr;      // [B + 1] first pass-C tile of each bucket
    int *ghC = nullptr;        // [TCcap << sb] pass C tile histograms
    int *akey = nullptr;       // [Vtot] pass A output: row
    uint16_t *tkey = nullptr;  // [Vtot] pass B output: row within bucket
    int *tcol = nullptr;       // [Vtot]
    float *tval = nullptr;     // [Vtot] (weighted only)
    int *rp = nullptr;         // [Ntot + 1]
    int *col = nullptr;        // [Vtot]
    float *val = nullptr;      // [Vtot] (weighted only)
    float2 *info = nullptr;    // [Ntot] {c_i, y_i bits}; y_i = 0 (and c_i = 0) without a known label
    float *srow = nullptr;     // [Ntot] D^-1/2 (Laplacian)
    int *wrow = nullptr;       // [NWtot] row holding each embed wavefront's first entry
    uint8_t *rstep = nullptr;  // [Vtot] row step from the previous CSR entry (see gee_embed.hip)
    int *split = nullptr;      // [NWtot]
    float *headp = nullptr;    // [parts]
    float *tailp = nullptr;    // [parts]
    float *headd = nullptr;    // [NWtot] degree partials (weighted Laplacian)
    float *taild = nullptr;    // [NWtot]
    int *dsplit = nullptr;     // [NWtot]
    // bucket path
    int4 *part = nullptr;      // [bparts] {bucket, first entry, end entry, partial slot or -1}
    int4 *multi = nullptr;     // [bslots / 2] {bucket, first slot, parts} of buckets of several parts
    int *ptot = nullptr;       // [4 * 64] per-workgroup totals of the part count
    int *bmeta = nullptr;      // [4]: parts, buckets of several parts
    float *dpart = nullptr;    // [bslots * 64] partial degrees
    float *zpart = nullptr;    // [bslots << sb * Kmax] partial class sums
    int *rcnt = nullptr;       // [N] non-zero entries of each Z row (sparse Z of one graph), or nullptr
    // sparse Z of one graph on the bucket path: each bucket's non-zero (class, value bits)
    // pairs in row-major order from its first row's place in a dense Z, r0 K (no dense Z is
    // written), or nullptr
    int2 *zs_pairs = nullptr;
};

// ----------------------------------------------------------------------------- class counts
// (Section 2: W row j holds 1/n_{y_j}). No global atomics on the counts: workgroup j of the
// label slices histograms a contiguous slice of one graph's labels in LDS and writes its K
// partial counts; then one wavefront per class adds the partials (integers, so the order
// cannot change the result) and forms 1/n_k in float32 (0 for an empty class).

// The whole workgroup: label slice j (hist: LDS of at least kMaxClasses ints).
__device__ __forceinline__ void class_count_slice(const Batch &b, int j, int *__restrict__ part,
                                                  unsigned *status, int *hist) {
    const int g = find_graph(b.cnt_offs, b.G, j);
    const GDesc d = load_desc(b, g);
    const int jb = j - d.cnt_off;
    const int K = d.K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    const int64_t per = ((int64_t)d.N + d.cnt_blocks - 1) / d.cnt_blocks;
    const int64_t lo = (int64_t)jb * per;
    const int64_t hi = min((int64_t)d.N, lo + per);
    bool bad = false;
    // 8 labels per thread in flight together (positions past the slice read as unknown)
    constexpr int U = 8;
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (int64_t)U * blockDim.x) {
        int y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x;
            y[u] = i < hi ? d.labels[i] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (y[u] >= 0 && y[u] < K)
                atomicAdd(&hist[y[u]], 1);
            else if (y[u] != -1 && validates(d))
                bad = true;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) raise_error(status, kErrLabel);
    for (int k = threadIdx.x; k < K; k += blockDim.x) part[d.cpart_off + (int64_t)jb * K + k] = hist[k];
}

// Parts of a bucket of n entries with part size P, and whether it is a one-part bucket of
// more than P/4 entries (listed before the short ones in the part table).
__device__ __forceinline__ int parts_of(int n, int P) { return n > P ? (n + P - 1) / P : 1; }
__device__ __forceinline__ bool large_single(int n, int k, int P) { return k == 1 && 4 * n > P; }

// One block of 1024 buckets of the bucket path's part table, by a workgroup of 256 threads
// (four consecutive buckets each): bucket bk of n entries gets k = parts_of(n, P) parts
// {bucket, first entry, end entry, slot} (slot -1 for one part, else the bucket's first slot
// + part index), listed as: the parts of split buckets first (at their slots), then the
// one-part buckets of more than P/4 entries, then the rest, each group in bucket order; a
// split bucket also gets {bucket, first slot, parts} in `multi`. ptot holds the four
// totals of every block (parts, slots, split buckets, large one-part buckets); the last
// block writes bmeta = {parts, split buckets}.
// With `bad` set (a resident CSR that failed its checks) every bucket counts as empty.
// Without ptot (a single block: nblk = 1) the block's own scan totals are the totals.
__device__ __forceinline__ void part_fill_block(const Batch &b, const int *__restrict__ bstart, int B, int sb,
                                                const int *__restrict__ ptot, int nblk, int blk,
                                                int4 *__restrict__ part, int4 *__restrict__ multi,
                                                int *__restrict__ bmeta, const int *__restrict__ bad = nullptr) {
    const bool none = bad && *bad;
    __shared__ int pf_wsum[4];
    // before this block: parts, slots, split buckets, large one-part buckets, small
    // one-part buckets; over all blocks: slots, large one-part buckets
    __shared__ int pf_base[7];
    if (threadIdx.x < 64) {
        int v[7] = {0, 0, 0, 0, 0, 0, 0};
        if (ptot && (int)threadIdx.x < nblk) {
            const int q0 = ptot[4 * threadIdx.x], q1 = ptot[4 * threadIdx.x + 1];
            const int q2 = ptot[4 * threadIdx.x + 2], q3 = ptot[4 * threadIdx.x + 3];
            v[5] = q1;
            v[6] = q3;
            if ((int)threadIdx.x < blk) {
                v[0] = q0;
                v[1] = q1;
                v[2] = q2;
                v[3] = q3;
                v[4] = q0 - q1 - q3;  // one-part buckets that are not large
            }
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] = readlane(wave_scan_add(v[c]), 63);
        if (threadIdx.x == 0)
            for (int c = 0; c < 7; ++c) pf_base[c] = v[c];
    }
    __syncthreads();
    int k[4], s0[4], s1[4], P[4];
    int nk = 0, nslot = 0, nsplit = 0, nlarge = 0, nsmall = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int bk = blk * 1024 + 4 * (int)threadIdx.x + u;
        k[u] = 0;
        P[u] = 1;
        s0[u] = s1[u] = 0;
        if (bk < B) {
            P[u] = load_desc(b, find_graph(b.node_offs, b.G, bk << sb)).WE;
            s0[u] = bstart[bk];
            s1[u] = none ? s0[u] : bstart[bk + 1];
            k[u] = parts_of(s1[u] - s0[u], P[u]);
        }
        const bool large = large_single(s1[u] - s0[u], k[u], P[u]);
        nk += k[u];
        nslot += k[u] > 1 ? k[u] : 0;
        nsplit += k[u] > 1 ? 1 : 0;
        nlarge += large ? 1 : 0;
        nsmall += (k[u] == 1 && !large) ? 1 : 0;
    }
    int t0, t1, t2, t3, t4;
    (void)block_excl_scan<256>(nk, pf_wsum, t0);
    int ss = pf_base[1] + block_excl_scan<256>(nslot, pf_wsum, t1);
    int mm = pf_base[2] + block_excl_scan<256>(nsplit, pf_wsum, t2);
    int ll = pf_base[3] + block_excl_scan<256>(nlarge, pf_wsum, t3);
    int sm = pf_base[4] + block_excl_scan<256>(nsmall, pf_wsum, t4);
    // the one-part buckets follow every split bucket's parts, the small ones every large one
    const int all_slots = ptot ? pf_base[5] : t1, all_large = ptot ? pf_base[6] : t3;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int bk = blk * 1024 + 4 * (int)threadIdx.x + u;
        if (bk >= B) break;
        if (k[u] > 1) {
            for (int q = 0; q < k[u]; ++q)
                part[ss + q] = make_int4(bk, s0[u] + q * P[u], min(s0[u] + (q + 1) * P[u], s1[u]), ss + q);
            multi[mm] = make_int4(bk, ss, k[u], 0);
            ss += k[u];
            ++mm;
        } else if (large_single(s1[u] - s0[u], k[u], P[u])) {
            part[all_slots + ll] = make_int4(bk, s0[u], s1[u], -1);
            ++ll;
        } else {
            part[all_slots + all_large + sm] = make_int4(bk, s0[u], s1[u], -1);
            ++sm;
        }
    }
    if (blk == nblk - 1 && threadIdx.x == 0) {
        bmeta[0] = pf_base[0] + t0;
        bmeta[1] = pf_base[2] + t2;
    }
}

// The part table's inputs and outputs, for the launch that fills it (the pass-B scatter
// takes its blocks as extra workgroups; nblk = 0: none).
struct PartFill {
    const int *bstart = nullptr;
    const int *ptot = nullptr;
    int4 *part = nullptr;
    int4 *multi = nullptr;
    int *bmeta = nullptr;
    int B = 0, sb = 0, nblk = 0;
};

// One wavefront: class c of the launch (all graphs' classes in order).
__device__ __forceinline__ void class_count_total(const Batch &b, int c, const int *__restrict__ part,
                                                  int *__restrict__ counts, float *__restrict__ inv_n) {
    const int lane = lane_id();
    const int g = find_graph(b.class_offs, b.G, c);
    const GDesc d = load_desc(b, g);
    const int k = c - d.class_off;
    const int *pp = part + d.cpart_off + k;
    int n = 0;
    for (int j = lane; j < d.cnt_blocks; j += 64) n += pp[(int64_t)j * d.K];
    n = readlane(wave_scan_add(n), 63);
    if (lane == 0) {
        counts[c] = n;
        if (inv_n) inv_n[c] = n > 0 ? 1.0f / (float)n : 0.0f;
    }
}

// Class counts run inside the first partition launches (a_hist takes the label slices as
// extra workgroups, digit_scan the class totals): both are independent of the partition.
struct CountJob {
    int *part = nullptr;
    int *counts = nullptr;
    float *inv_n = nullptr;
    int slices = 0;  // label-slice workgroups (Plan::cnt_blocks)
    int classes = 0; // Plan::Ktot
};

// ----------------------------------------------------------------------------- profiling
// Kernel ids for the optional event hook (gee_profile_kernel). The hook records a
// caller's hipEvents on the launch stream right before / after a kernel launch.
enum KernelId : int {
    kKCountPartial = 0, kKCountFinal, kKAHist, kKAScan, kKAScatter, kKBHist, kKBScan,
    kKBScatter, kKCTiles, kKCHist, kKCScan, kKCScatter, kKBucketSort, kKGraphMeta, kKZeroSteps, kKNodeRows, kKDegreeRows, kKDegreeFixup,
    kKNodeCoef, kKFillEmpty, kKEmbedRows, kKEmbedFixup, kKBucketPartCount, kKBucketPartFill, kKBucketDegree,
    kKBucketDegreeFix, kKBucketEmbed, kKBucketEmbedFix, kKEdgeInit, kKEdgePrep, kKEdgeCoef, kKEdgeScatter,
    kKEdgeFinish, kKZsCount, kKZsWrite, kKZsTileSum, kKCsrPrep, kKNumKernels
};
extern const char *const kKernelNames[kKNumKernels];
void prof_begin(int kid, hipStream_t s);
void prof_end(int kid, hipStream_t s);

// ----------------------------------------------------------------------------- launchers
// gee_count.hip: host bytes -> device memory, stream-ordered, in kernel-argument chunks.
constexpr int kUploadChunk = 2048;
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s);
// gee_count.hip: counts[class_off + k] and inv_n (inv_n may be nullptr); zero_word (if
// given) is set to 0 first, in stream order before every later launch of the call. Without
// totals only the per-slice partial counts are formed (a later launch adds them up).
hipError_t launch_class_counts(const Batch &b, const Plan &p, int *part, int *counts, float *inv_n,
                               unsigned *status, hipStream_t s, int *zero_word = nullptr, bool totals = true);
// gee_csr.hip: edge lists -> CSR of the union (rows and columns offset by node_off).
// With job, the class counts of the launch run in the same launches.
hipError_t launch_csr_build(const Batch &b, const Plan &p, const Work &wk, unsigned *status, hipStream_t s,
                            const CountJob *job = nullptr);
hipError_t launch_csr_pass2(const Plan &p, const Work &wk, unsigned *status, hipStream_t s);
size_t bucket_sort_lds(int sb);
int bucket_stage_cap(int sb);
// gee_embed.hip
// Per-graph entry ranges and wavefront counts from row_ptr (after a CSR build), or
// from the given entry count M (a single resident CSR, rp_of_union == nullptr).
hipError_t launch_graph_meta(const Batch &b, const int *rp_of_union, int M, hipStream_t s);
// Per-node data (ownership, degrees, s_i, c_i).
hipError_t launch_node_prep(const Batch &b, const Plan &p, const int *rp, const float *val, int64_t n_entries,
                            const Work &wk, unsigned *status, hipStream_t s);
size_t embed_lds_per_wave(int K);
// Z from the CSR; n_entries = length of the col/val arrays (entries past it are never read).
hipError_t launch_embed(const Batch &b, const Plan &p, const int *rp, const int *col, const float *val,
                        int64_t n_entries, const Work &wk, unsigned *status, hipStream_t s);
// gee_bucket.hip: Z straight from the row buckets of the first two sort passes
// (launch_csr_build), for plans with p.bucket.
// A resident CSR through the bucket kernels (plans made with csr_bucket): its checks and
// bucket starts (csr_prep, whose extra workgroups add up the class counts' partials in
// wk.cpart), the part table, degrees and class sums, rows from row_ptr.
hipError_t launch_bucket_embed_csr(const Batch &b, const Plan &p, const Work &wk, const int *rp, const int *col,
                                   const float *val, int64_t M, unsigned *status, hipStream_t s);
#ifndef GEE_BUCKET_MIN_PART
#define GEE_BUCKET_MIN_PART 2048
#endif
constexpr int kBucketMinPart = GEE_BUCKET_MIN_PART;  // entries of a bucket part, at least
// Default part size of a graph of `entries` CSR entries: the largest power of two in
// [kBucketMinPart, 8192] that still leaves at least 2048 parts, so a small graph's buckets
// still spread over the chip (2048 on a 2,000-node SBM graph of 446k entries, 4096 at 11M
// entries, 8192 from 16.8M).
inline int default_bucket_part(int64_t entries) {
    int p = kBucketMinPart;
    while (p < 8192 && (int64_t)p * 2 * 2048 <= entries) p *= 2;
    return p;
}
constexpr int kBucketWindowPad = 256;  // entries allocated past the bucketed arrays' end
// Degree kernels' outputs: s_i into srow and c_i = s_i / n_{y_i} into info (both), c_i alone
// from the in-degrees of a transposed pass (in), s_i alone from the out-degrees (out).
enum DegreeMode : int { kDegBoth = 0, kDegIn = 1, kDegOut = 2 };
// sums = false: the part table and the degrees only (the transposed pass).
hipError_t launch_bucket_embed(const Batch &b, const Plan &p, const Work &wk, hipStream_t s, int mode = kDegBoth,
                               bool sums = true);
// Original GEE form (edge-list scatter with float atomics; gee_edge.hip): workspace bytes
// and the whole launch sequence for one graph.
size_t edge_workspace_bytes(int N, int K, unsigned flags);  // (+ N floats of in-degrees for in_degree_pass)
hipError_t launch_edge_embed(const int *src, const int *dst, const float *w, int64_t E, int N, const int *labels,
                             int K, unsigned flags, float *Z, void *ws, unsigned *status, hipStream_t s);
// Sparse storage of a dense Z (gee_zsparse.hip): scratch of one int per tile of rows and
// one per row, then row_ptr[N + 1] and at most `cap` (class, value) pairs.
int zsparse_tiles(int N);
// counts_given: rcnt already holds every row's non-zero count (written by the class-scatter
// kernels), so the count pass over Z is skipped.
// Staged sparse Z (Work::zs_pairs after the bucket kernels; rcnt given): row_ptr from
// the row counts, then each bucket's staged run (buckets of 2^sb <= 256 rows, the run of the
// bucket of first row r0 starting at r0 K) copied to its place.
#ifndef GEE_ZS_STAGED
#define GEE_ZS_STAGED 1
#endif
hipError_t launch_zsparse_staged(int N, int K, int sb, const int2 *zs_pairs, int *tile, int *rcnt, int *row_ptr,
                                 int *col, float *val, int64_t cap, hipStream_t s);
hipError_t launch_zsparse(const float *Z, int N, int K, int *tile, int *rcnt, int *row_ptr, int *col, float *val,
                          int64_t cap, bool counts_given, hipStream_t s);

}  // namespace gee
