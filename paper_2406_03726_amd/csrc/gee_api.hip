// gee_api.hip - the C ABI declared in include/gee.h: argument checks, the launch plan,
// workspace carve-up, the per-device data-error word and the entry points.
#include <atomic>
#include <cstring>
#include <mutex>

#include "gee.h"
#include "gee_internal.h"

using namespace gee;

namespace {

constexpr size_t kAlign = 256;
constexpr unsigned kKnownFlags = GEE_DIAG | GEE_LAPLACIAN | GEE_CORRELATION | GEE_SYMMETRIZE;
constexpr int64_t kMaxEntries = (int64_t)INT32_MAX - 65536;

int ilog2_ceil(int64_t x) {
    int b = 0;
    while (((int64_t)1 << b) < x) ++b;
    return b;
}
bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int hip_status(hipError_t e) {
    if (e == hipSuccess) return GEE_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return GEE_ERR_OOM;
    return GEE_ERR_HIP;
}

// ------------------------------------------------------------------------- data-error word

std::mutex g_status_mu;
unsigned *g_status[64] = {nullptr};

int device_status(unsigned **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GEE_ERR_HIP;
    if (dev < 0 || dev >= 64) return GEE_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_status_mu);
    if (!g_status[dev]) {
        unsigned *p = nullptr;
        hipError_t e = hipMalloc(&p, 256);
        if (e != hipSuccess) return hip_status(e);
        e = hipMemset(p, 0, 256);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            (void)hipFree(p);
            return hip_status(e);
        }
        g_status[dev] = p;
    }
    *out = g_status[dev];
    return GEE_OK;
}

// ------------------------------------------------------------------------- profiling hook

struct ProfSlot {
    hipEvent_t start = nullptr, stop = nullptr;
};
std::mutex g_prof_mu;
ProfSlot g_prof[kKNumKernels];
std::atomic<int> g_prof_active{0};

// ------------------------------------------------------------------------- plan

int make_plan(int64_t E, int32_t N, int32_t K, uint32_t flags, bool weighted, const gee_schedule *sc,
              Plan &p) {
    p.E = E;
    p.N = N;
    p.K = K;
    p.flags = flags;
    p.weighted = weighted;
    p.Mcap = (flags & GEE_SYMMETRIZE) ? 2 * E : E;
    if (p.Mcap > kMaxEntries) return GEE_ERR_TOO_LARGE;
    // buckets of 2^sb rows, about 3000 entries each on average; at most 65536 buckets
    const int sb_min = ilog2_ceil(N > 0 ? N : 1) > 16 ? ilog2_ceil(N) - 16 : 0;
    if (sb_min > kMaxBucketRowsLog2) return GEE_ERR_TOO_LARGE;
    int sb = 0;
    if (p.Mcap > 0) {
        const double rows = 3000.0 * (double)(N > 0 ? N : 1) / (double)p.Mcap;
        while (sb < kMaxBucketRowsLog2 && (double)(2 << sb) <= rows) ++sb;
    } else {
        sb = kMaxBucketRowsLog2;
    }
    if (sc && sc->bucket_rows_log2 > 0) sb = sc->bucket_rows_log2;
    if (sb < sb_min) sb = sb_min;
    if (sb > kMaxBucketRowsLog2) sb = kMaxBucketRowsLog2;
    p.sb = sb;
    p.B = (int32_t)(((int64_t)(N > 0 ? N : 1) + (1 << sb) - 1) >> sb);
    const int nbB = ilog2_ceil(p.B);
    p.s2 = nbB <= 8 ? 0 : (nbB - 8 > nbB / 2 ? nbB - 8 : nbB / 2);
    p.DA = (int)(((int64_t)p.B + (1 << p.s2) - 1) >> p.s2);
    p.tile = 4096;
    if (sc && sc->tile_entries && sc->tile_entries != p.tile) return GEE_ERR_ARG;
    p.TA = (p.Mcap + p.tile - 1) / p.tile;
    if (p.TA < 1) p.TA = 1;
    p.TBcap = p.s2 > 0 ? p.TA + p.DA : 1;
    // embed: entries per wavefront
    int we = p.Mcap >= (1 << 20) ? 1024 : 512;
    if (sc && sc->wave_entries) {
        if (!is_pow2(sc->wave_entries) || sc->wave_entries < 256 || sc->wave_entries > 16384)
            return GEE_ERR_ARG;
        we = sc->wave_entries;
    }
    p.WE = we;
    // one wavefront per workgroup by default: the LDS ring of each wavefront then limits
    // residency least (more wavefronts in flight per CU)
    const size_t per_wave = embed_lds_per_wave(K);
    int wpb = 1;
    if (sc && sc->waves_per_block) {
        if (sc->waves_per_block < 1 || sc->waves_per_block > 4) return GEE_ERR_ARG;
        if ((size_t)sc->waves_per_block * per_wave <= 65536) wpb = sc->waves_per_block;
    }
    p.wpb = wpb;
    p.NWcap = p.Mcap > 0 ? (p.Mcap + p.WE - 1) / p.WE : 1;
    int64_t cb = ((int64_t)N + 4095) / 4096;
    p.cnt_blocks = (int)(cb < 1 ? 1 : (cb > 512 ? 512 : cb));
    return GEE_OK;
}

enum Parts : unsigned { kPCount = 1, kPPart = 2, kPCsrOut = 4, kPEmbed = 8 };

// Carves the workspace; with base == nullptr only the size is computed.
size_t carve(const Plan &p, unsigned parts, char *base, Work &w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *r = base ? base + off : nullptr;
        off += (bytes + kAlign - 1) / kAlign * kAlign;
        return r;
    };
    w.meta = (int *)take(4 * sizeof(int));
    if (parts & kPCount) {
        w.counts = (int *)take((size_t)p.K * sizeof(int));
        w.inv_n = (float *)take((size_t)p.K * sizeof(float));
        w.cpart = (int *)take((size_t)p.cnt_blocks * p.K * sizeof(int));
    }
    if (parts & kPPart) {
        w.ghA = (int *)take((size_t)p.DA * p.TA * sizeof(int));
        w.totA = (int *)take((size_t)p.DA * sizeof(int));
        w.segA = (int *)take((size_t)(p.DA + 1) * sizeof(int));
        w.tileB = (int *)take((size_t)(p.DA + 1) * sizeof(int));
        if (p.s2 > 0) w.ghB = (int *)take(((size_t)p.TBcap << p.s2) * sizeof(int));
        w.bstart = (int *)take((size_t)(p.B + 1) * sizeof(int));
        w.akey = (int *)take((size_t)p.Mcap * sizeof(int));
        if (p.s2 > 0) w.tkey = (uint16_t *)take((size_t)p.Mcap * sizeof(uint16_t));
        w.tcol = (int *)take((size_t)p.Mcap * sizeof(int));
        if (p.weighted) w.tval = (float *)take((size_t)p.Mcap * sizeof(float));
    }
    if (parts & kPCsrOut) {
        w.rp = (int *)take((size_t)(p.N + 1) * sizeof(int));
        w.col = (int *)take((size_t)p.Mcap * sizeof(int));
        if (p.weighted) w.val = (float *)take((size_t)p.Mcap * sizeof(float));
    }
    if (parts & kPEmbed) {
        w.info = (float2 *)take((size_t)p.N * sizeof(float2));
        w.srow = (float *)take((size_t)p.N * sizeof(float));
        w.wrow = (int *)take((size_t)p.NWcap * sizeof(int));
        w.rstep = (uint8_t *)take((size_t)(p.Mcap > 0 ? p.Mcap : 1));
        w.split = (int *)take((size_t)p.NWcap * sizeof(int));
        w.headp = (float *)take((size_t)p.NWcap * p.K * sizeof(float));
        w.tailp = (float *)take((size_t)p.NWcap * p.K * sizeof(float));
        w.headd = (float *)take((size_t)p.NWcap * sizeof(float));
        w.taild = (float *)take((size_t)p.NWcap * sizeof(float));
        w.dsplit = (int *)take((size_t)p.NWcap * sizeof(int));
    }
    return off;
}

int check_common(int32_t N, int32_t K, uint32_t flags) {
    if (N < 0 || K < 1) return GEE_ERR_ARG;
    if (flags & ~kKnownFlags) return GEE_ERR_ARG;
    if (N > GEE_MAX_NODES) return GEE_ERR_TOO_LARGE;
    if (K > GEE_MAX_CLASSES) return GEE_ERR_UNSUPPORTED;
    return GEE_OK;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

namespace gee {

const char *const kKernelNames[kKNumKernels] = {
    "class_count_partial", "class_count_final", "a_hist", "digit_scan", "a_totals", "a_scatter",
    "b_hist", "b_scan", "b_scatter", "bucket_sort", "zero_steps", "node_rows", "degree_rows", "degree_fixup", "fill_empty",
    "embed_rows", "embed_fixup", "set_meta"};

void prof_begin(int kid, hipStream_t s) {
    if (!g_prof_active.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof[kid].start) (void)hipEventRecord(g_prof[kid].start, s);
}

void prof_end(int kid, hipStream_t s) {
    if (!g_prof_active.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof[kid].stop) (void)hipEventRecord(g_prof[kid].stop, s);
}

}  // namespace gee

// =========================================================================== C ABI

extern "C" {

int gee_abi_version(void) { return GEE_ABI_VERSION; }

const char *gee_status_string(int st) {
    switch (st) {
    case GEE_OK: return "ok";
    case GEE_ERR_ARG: return "invalid argument";
    case GEE_ERR_LABEL: return "label outside [-1, K)";
    case GEE_ERR_INDEX: return "node index outside [0, N)";
    case GEE_ERR_WEIGHT: return "non-finite edge weight";
    case GEE_ERR_TOO_LARGE: return "sizes beyond this build's limits";
    case GEE_ERR_OOM: return "device out of memory";
    case GEE_ERR_HIP: return "HIP runtime error";
    case GEE_ERR_UNSUPPORTED: return "unsupported request";
    case GEE_ERR_WORKSPACE: return "workspace too small";
    default: return "unknown status";
    }
}

int gee_profile_kernel(const char *kernel, void *start_event, void *stop_event) {
    if (!kernel) return GEE_ERR_ARG;
    int kid = -1;
    for (int i = 0; i < kKNumKernels; ++i)
        if (std::strcmp(kernel, kKernelNames[i]) == 0) kid = i;
    if (kid < 0 || (start_event == nullptr) != (stop_event == nullptr)) return GEE_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[kid].start = reinterpret_cast<hipEvent_t>(start_event);
    g_prof[kid].stop = reinterpret_cast<hipEvent_t>(stop_event);
    int active = 0;
    for (int i = 0; i < kKNumKernels; ++i) active |= g_prof[i].start != nullptr;
    g_prof_active.store(active, std::memory_order_relaxed);
    return GEE_OK;
}

int gee_init(void) {
    unsigned *st = nullptr;
    return device_status(&st);
}

int gee_get_data_errors(void *stream, uint32_t *bits) {
    if (!bits) return GEE_ERR_ARG;
    unsigned *st = nullptr;
    int rc = device_status(&st);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(as_stream(stream));
    if (e != hipSuccess) return hip_status(e);
    unsigned h = 0;
    e = hipMemcpy(&h, st, sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_status(e);
    e = hipMemset(st, 0, sizeof(unsigned));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_status(e);
    *bits = h;
    return GEE_OK;
}

int gee_default_schedule(int64_t E, int32_t N, int32_t K, uint32_t flags, gee_schedule *out) {
    if (!out || E < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    Plan p;
    rc = make_plan(E, N, K, flags, true, nullptr, p);
    if (rc) return rc;
    out->wave_entries = p.WE;
    out->waves_per_block = p.wpb;
    out->tile_entries = p.tile;
    out->bucket_rows_log2 = p.sb;
    return GEE_OK;
}

int64_t gee_csr_capacity(int64_t E, uint32_t flags) {
    if (E < 0) return -1;
    return (flags & GEE_SYMMETRIZE) ? 2 * E : E;
}

// --------------------------------------------------------------------------- class counts

int gee_class_counts(const int32_t *labels, int32_t N, int32_t K, int32_t *counts, void *stream) {
    int rc = check_common(N, K, 0);
    if (rc) return rc;
    if (!counts || (N > 0 && !labels)) return GEE_ERR_ARG;
    unsigned *st = nullptr;
    if ((rc = device_status(&st))) return rc;
    Plan p;
    if ((rc = make_plan(0, N, K, 0, false, nullptr, p))) return rc;
    hipStream_t s = as_stream(stream);
    int *part = nullptr;
    hipError_t e = hipMallocAsync((void **)&part, (size_t)p.cnt_blocks * K * sizeof(int), s);
    if (e != hipSuccess) return hip_status(e);
    e = launch_class_counts(labels, N, K, p.cnt_blocks, part, counts, nullptr, st, s);
    hipError_t e2 = hipFreeAsync(part, s);
    return hip_status(e != hipSuccess ? e : e2);
}

// --------------------------------------------------------------------------- CSR build

size_t gee_build_csr_workspace_bytes(int64_t E, int32_t N, uint32_t flags, const gee_schedule *sched) {
    Plan p;
    if (E < 0 || check_common(N, 1, flags) || make_plan(E, N, 1, flags, true, sched, p)) return 0;
    Work w;
    return carve(p, kPPart, nullptr, w);
}

int gee_build_csr_ws(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
                     uint32_t flags, int32_t *row_ptr, int32_t *col, float *val,
                     const gee_schedule *sched, void *workspace, size_t workspace_bytes,
                     void *stream) {
    if (E < 0) return GEE_ERR_ARG;
    int rc = check_common(N, 1, flags);
    if (rc) return rc;
    if (!row_ptr || (E > 0 && (!src || !dst || !col)) || (wgt && E > 0 && !val)) return GEE_ERR_ARG;
    if (N == 0 && E > 0) return GEE_ERR_ARG;
    unsigned *st = nullptr;
    if ((rc = device_status(&st))) return rc;
    Plan p;
    if ((rc = make_plan(E, N, 1, flags, wgt != nullptr, sched, p))) return rc;
    // size with weights present so one workspace size serves both cases
    Plan pw = p;
    pw.weighted = true;
    Work wk;
    if (!workspace || workspace_bytes < carve(pw, kPPart, nullptr, wk)) return GEE_ERR_WORKSPACE;
    carve(p, kPPart, (char *)workspace, wk);
    hipStream_t s = as_stream(stream);
    if (N == 0) {
        hipError_t e = hipMemsetAsync(row_ptr, 0, sizeof(int32_t), s);
        return hip_status(e);
    }
    wk.rp = row_ptr;
    wk.col = col;
    wk.val = wgt ? val : nullptr;
    hipError_t e = launch_csr_build(src, dst, wgt, p, wk, st, s);
    if (e == hipSuccess) e = launch_csr_pass2(p, wk, st, s);
    return hip_status(e);
}

int gee_build_csr(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
                  uint32_t flags, int32_t *row_ptr, int32_t *col, float *val, void *stream) {
    size_t bytes = gee_build_csr_workspace_bytes(E, N, flags, nullptr);
    if (bytes == 0) return E < 0 ? GEE_ERR_ARG : check_common(N, 1, flags) ? check_common(N, 1, flags) : GEE_ERR_TOO_LARGE;
    hipStream_t s = as_stream(stream);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, bytes, s);
    if (e != hipSuccess) return hip_status(e);
    int rc = gee_build_csr_ws(src, dst, wgt, E, N, flags, row_ptr, col, val, nullptr, ws, bytes, stream);
    e = hipFreeAsync(ws, s);
    return rc ? rc : hip_status(e);
}

// --------------------------------------------------------------------------- embed

size_t gee_embed_workspace_bytes(int64_t E, int32_t N, int32_t K, uint32_t flags, int weighted,
                                 const gee_schedule *sched) {
    Plan p;
    if (E < 0 || check_common(N, K, flags) || make_plan(E, N, K, flags, weighted != 0, sched, p)) return 0;
    Work w;
    return carve(p, kPCount | kPPart | kPCsrOut | kPEmbed, nullptr, w);
}

int gee_embed_ws(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
                 const int32_t *labels, int32_t K, uint32_t flags, float *Z, const gee_schedule *sched,
                 void *workspace, size_t workspace_bytes, void *stream) {
    if (E < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    if ((E > 0 && (!src || !dst)) || (N > 0 && (!labels || !Z))) return GEE_ERR_ARG;
    if (N == 0) return E > 0 ? GEE_ERR_ARG : GEE_OK;
    unsigned *st = nullptr;
    if ((rc = device_status(&st))) return rc;
    Plan p;
    if ((rc = make_plan(E, N, K, flags, wgt != nullptr, sched, p))) return rc;
    Work wk;
    const unsigned parts = kPCount | kPPart | kPCsrOut | kPEmbed;
    if (!workspace || workspace_bytes < carve(p, parts, nullptr, wk)) return GEE_ERR_WORKSPACE;
    carve(p, parts, (char *)workspace, wk);
    hipStream_t s = as_stream(stream);
    hipError_t e = launch_class_counts(labels, N, K, p.cnt_blocks, wk.cpart, wk.counts, wk.inv_n, st, s);
    if (e == hipSuccess) e = launch_csr_build(src, dst, wgt, p, wk, st, s);
    if (e == hipSuccess) e = launch_csr_pass2(p, wk, st, s);
    const float *val = p.weighted ? wk.val : nullptr;
    if (e == hipSuccess) e = launch_node_prep(wk.rp, val, labels, p, wk, st, s);
    if (e == hipSuccess) e = launch_embed(wk.rp, wk.col, val, p, wk, Z, st, s);
    return hip_status(e);
}

int gee_embed(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
              const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *stream) {
    if (E < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    if (N == 0) return E > 0 ? GEE_ERR_ARG : GEE_OK;
    size_t bytes = gee_embed_workspace_bytes(E, N, K, flags, wgt != nullptr, nullptr);
    if (bytes == 0) return GEE_ERR_TOO_LARGE;
    hipStream_t s = as_stream(stream);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, bytes, s);
    if (e != hipSuccess) return hip_status(e);
    rc = gee_embed_ws(src, dst, wgt, E, N, labels, K, flags, Z, nullptr, ws, bytes, stream);
    e = hipFreeAsync(ws, s);
    return rc ? rc : hip_status(e);
}

// --------------------------------------------------------------------------- embed from CSR

size_t gee_embed_csr_workspace_bytes(int64_t M, int32_t N, int32_t K, uint32_t flags,
                                     const gee_schedule *sched) {
    Plan p;
    if (M < 0 || check_common(N, K, flags) || make_plan(M, N, K, flags & ~GEE_SYMMETRIZE, true, sched, p))
        return 0;
    Work w;
    return carve(p, kPCount | kPEmbed, nullptr, w);
}

int gee_embed_csr_ws(const int32_t *row_ptr, const int32_t *col, const float *val, int64_t M, int32_t N,
                     const int32_t *labels, int32_t K, uint32_t flags, float *Z,
                     const gee_schedule *sched, void *workspace, size_t workspace_bytes, void *stream) {
    if (M < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    if (N == 0) return M > 0 ? GEE_ERR_ARG : GEE_OK;
    if (!row_ptr || !labels || !Z || (M > 0 && !col)) return GEE_ERR_ARG;
    unsigned *st = nullptr;
    if ((rc = device_status(&st))) return rc;
    Plan p;
    if ((rc = make_plan(M, N, K, flags & ~GEE_SYMMETRIZE, val != nullptr, sched, p))) return rc;
    Work wk;
    const unsigned parts = kPCount | kPEmbed;
    if (!workspace || workspace_bytes < carve(p, parts, nullptr, wk)) return GEE_ERR_WORKSPACE;
    carve(p, parts, (char *)workspace, wk);
    hipStream_t s = as_stream(stream);
    const int NW = M > 0 ? (int)((M + p.WE - 1) / p.WE) : 1;
    hipError_t e = launch_class_counts(labels, N, K, p.cnt_blocks, wk.cpart, wk.counts, wk.inv_n, st, s);
    if (e == hipSuccess) e = launch_set_meta(wk.meta, (int)M, NW, s);
    if (e == hipSuccess) e = launch_node_prep(row_ptr, val, labels, p, wk, st, s);
    if (e == hipSuccess) e = launch_embed(row_ptr, col, val, p, wk, Z, st, s);
    return hip_status(e);
}

int gee_embed_csr(const int32_t *row_ptr, const int32_t *col, const float *val, int64_t M, int32_t N,
                  const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *stream) {
    if (M < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    if (N == 0) return M > 0 ? GEE_ERR_ARG : GEE_OK;
    size_t bytes = gee_embed_csr_workspace_bytes(M, N, K, flags, nullptr);
    if (bytes == 0) return GEE_ERR_TOO_LARGE;
    hipStream_t s = as_stream(stream);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, bytes, s);
    if (e != hipSuccess) return hip_status(e);
    rc = gee_embed_csr_ws(row_ptr, col, val, M, N, labels, K, flags, Z, nullptr, ws, bytes, stream);
    e = hipFreeAsync(ws, s);
    return rc ? rc : hip_status(e);
}

}  // extern "C"
