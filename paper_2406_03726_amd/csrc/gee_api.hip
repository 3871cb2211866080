// gee_api.hip - the C ABI declared in include/gee.h: argument checks, the launch plan,
// workspace carve-up, the per-device data-error word, the entry points, and batch
// plans (one hipGraph per batch).
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "gee.h"
#include "gee_internal.h"

using namespace gee;

namespace {

constexpr size_t kAlign = 256;
constexpr unsigned kKnownFlags =
    GEE_DIAG | GEE_LAPLACIAN | GEE_CORRELATION | GEE_SYMMETRIZE | GEE_DIRECTED_DEGREES | GEE_NO_VALIDATE;
constexpr int64_t kMaxEntries = (int64_t)INT32_MAX - 65536;
constexpr int64_t kMaxBatchNodes = (int64_t)1 << 28;
constexpr int kMaxBatchGraphs = 1 << 20;

int ilog2_ceil(int64_t x) {
    int b = 0;
    while (((int64_t)1 << b) < x) ++b;
    return b;
}
bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

thread_local hipError_t t_last_hip = hipSuccess;  // the last failed HIP call on this thread

int hip_status(hipError_t e) {
    if (e == hipSuccess) return GEE_OK;
    t_last_hip = e;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return GEE_ERR_OOM;
    return GEE_ERR_HIP;
}

// ------------------------------------------------------------------------- data-error words

// One data-error word per (device, stream): calls on one stream raise bits in that stream's
// word, so a bad request on one stream is never reported on another. The words live in a
// file-scope device array (no allocation, so every entry point can run under stream capture
// once gee_init has run on the device); a stream gets a slot the first time a call uses it,
// by a hash of its handle with linear probing. Past kStatusSlots - 1 distinct streams on a
// device the rest share the last slot. A slot is 64 bytes: the word and, beside it, the
// value gee_get_data_errors took from it.
constexpr int kStatusSlots = 1024;
constexpr int kStatusStride = 16;  // unsigned per slot
static __device__ __align__(256) unsigned status_words[kStatusSlots * kStatusStride];

// Fixed-size scratch of gee_embed_noalloc (device memory the library owns for the life of
// the process, one copy per device): the workspace of requests up to kScratchBytes.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DevState {
    bool ready = false;
    unsigned *words = nullptr;   // device address of status_words on this device
    void *scratch = nullptr;     // device address of scratch on this device
    const void *key[kStatusSlots];
    bool used[kStatusSlots];
};
std::mutex g_status_mu;
DevState g_dev[64];

// Device addresses of the file-scope arrays for the current device (once per device; the
// names of the arrays are host-side stand-ins that kernels must never be given).
int device_state(DevState **out) {
    int dev = 0;
    hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return hip_status(ge);
    if (dev < 0 || dev >= 64) return GEE_ERR_UNSUPPORTED;
    DevState &ds = g_dev[dev];
    if (!ds.ready) {
        void *w = nullptr, *sc = nullptr;
        hipError_t e = hipGetSymbolAddress(&w, HIP_SYMBOL(status_words));
        if (e == hipSuccess) e = hipGetSymbolAddress(&sc, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e);
        ds.words = static_cast<unsigned *>(w);
        ds.scratch = sc;
        for (int i = 0; i < kStatusSlots; ++i) {
            ds.key[i] = nullptr;
            ds.used[i] = false;
        }
        ds.ready = true;
    }
    *out = &ds;
    return GEE_OK;
}

// The data-error word of `stream` on the current device.
int stream_status(hipStream_t stream, unsigned **out) {
    std::lock_guard<std::mutex> lk(g_status_mu);
    DevState *ds = nullptr;
    int rc = device_state(&ds);
    if (rc) return rc;
    const void *key = reinterpret_cast<const void *>(stream);
    const uint64_t h = (uint64_t)reinterpret_cast<uintptr_t>(key) * 0x9E3779B97F4A7C15ull;
    int slot = kStatusSlots - 1;  // shared once the table is full
    for (int i = 0; i < kStatusSlots - 1; ++i) {
        const int j = (int)((h >> 40) + (uint64_t)i) % (kStatusSlots - 1);
        if (ds->used[j] && ds->key[j] == key) {
            slot = j;
            break;
        }
        if (!ds->used[j]) {
            ds->used[j] = true;
            ds->key[j] = key;
            slot = j;
            break;
        }
    }
    *out = ds->words + (size_t)slot * kStatusStride;
    return GEE_OK;
}

__global__ void status_take(unsigned *word) { word[1] = atomicExch(word, 0u); }
__global__ void status_take_to(unsigned *word, unsigned *dst) { *dst = atomicExch(word, 0u); }
__global__ void status_fold(unsigned *from, unsigned *to) {
    const unsigned v = atomicExch(from, 0u);
    if (v) atomicOr(to, v);
}

// ------------------------------------------------------------------------- profiling hook

struct ProfSlot {
    hipEvent_t start = nullptr, stop = nullptr;
};
std::mutex g_prof_mu;
ProfSlot g_prof[kKNumKernels];
std::atomic<int> g_prof_active{0};
thread_local bool t_capturing = false;  // no event records while a batch plan is captured

// ------------------------------------------------------------------------- plan

// One graph as the caller describes it. For a resident CSR, E is the entry count M.
struct GraphIn {
    const int *src = nullptr, *dst = nullptr;
    const float *w = nullptr;
    int64_t E = 0;
    int N = 0;
    const int *labels = nullptr;
    int K = 1;
    unsigned flags = 0;
    float *Z = nullptr;
    gee_schedule sc{0, 0, 0, 0};
};

int check_common(int32_t N, int32_t K, uint32_t flags) {
    if (N < 0 || K < 1) return GEE_ERR_ARG;
    if (flags & ~kKnownFlags) return GEE_ERR_ARG;
    if (N > GEE_MAX_NODES) return GEE_ERR_TOO_LARGE;
    if (K > GEE_MAX_CLASSES) return GEE_ERR_UNSUPPORTED;
    return GEE_OK;
}

int check_schedule(const gee_schedule &sc) {
    if (sc.wave_entries && (!is_pow2(sc.wave_entries) || sc.wave_entries < 256 || sc.wave_entries > 16384))
        return GEE_ERR_ARG;
    if (sc.waves_per_block && (sc.waves_per_block < 1 || sc.waves_per_block > 4)) return GEE_ERR_ARG;
    if (sc.tile_entries && sc.tile_entries != kPartTile) return GEE_ERR_ARG;
    if (sc.bucket_rows_log2 < 0 || sc.bucket_rows_log2 > kMaxBucketRowsLog2) return GEE_ERR_ARG;
    return GEE_OK;
}

// Default CSR entries per embed wavefront for a graph with this many entries.
int default_wave_entries(int64_t Mcap) { return Mcap >= (1 << 20) ? 1024 : 512; }

// Bucket path rows per bucket (log2) for a launch of these graphs: 64-row buckets when
// every graph's class sums fit 64 floats a row (the wavefront's LDS block stays at most
// 16 KiB), else 32-row buckets, raised to 64 when 32 would need more than kMaxBuckets; -1
// when 64 rows are not enough either. Graph offsets are then aligned to the bucket size,
// so a graph's buckets are its own.
#ifndef GEE_BUCKET_SB_MIN
#define GEE_BUCKET_SB_MIN 5
#endif
// A schedule's bucket_rows_log2 of 5 or 6 chooses the graph's bucket size on this path
// (32 or 64 rows); other values leave it to the class-count rule.
int preferred_bucket_sb(const GraphIn &x) {
    if (x.sc.bucket_rows_log2 == 5 || x.sc.bucket_rows_log2 == 6) return x.sc.bucket_rows_log2;
    return ring_stride(x.K) <= 64 ? 6 : GEE_BUCKET_SB_MIN;
}
int bucket_path_sb(const GraphIn *gs, int G) {
    int sb0 = 6;
    for (int g = 0; g < G; ++g) sb0 = preferred_bucket_sb(gs[g]) < sb0 ? preferred_bucket_sb(gs[g]) : sb0;
    for (int sb = sb0; sb <= 6; ++sb) {
        int64_t n = 0;
        for (int g = 0; g < G; ++g) n = ((n + (1 << sb) - 1) >> sb << sb) + gs[g].N;
        if (n <= kMaxBatchNodes && ((n + (1 << sb) - 1) >> sb) <= kMaxBuckets) return sb;
    }
    return -1;
}

// Plan of a launch over G graphs. `resident`: the graphs are given as CSRs (E = M).
// `edge_embed`: the launch embeds edge lists (gee_embed and batches), which take the
// bucket path whenever its buckets can hold the launch's rows.
// `csr_bucket`: a resident CSR embedded by the bucket kernels (rows from row_ptr).
int make_plan(const GraphIn *gs, int G, bool resident, Plan &p, std::vector<GDesc> &d, bool edge_embed = false,
              bool csr_bucket = false) {
    if (G < 1 || G > kMaxBatchGraphs) return GEE_ERR_ARG;
    p = Plan();
    p.G = G;
    d.assign(G, GDesc());
    int64_t voff = 0, noff = 0, woff = 0, parts = 0, coff = 0, cpo = 0, ktot = 0;
    int wpb = 0, sb_req = 0;
    const int sb_bucket = (edge_embed && !resident) || (resident && csr_bucket) ? bucket_path_sb(gs, G) : -1;
    p.bucket = sb_bucket >= 0;
    int64_t bparts = 0;
    for (int g = 0; g < G; ++g) {
        const GraphIn &x = gs[g];
        int rc = check_common(x.N, x.K, x.flags);
        if (rc) return rc;
        if (x.E < 0) return GEE_ERR_ARG;
        if ((rc = check_schedule(x.sc))) return rc;
        const bool sym = !resident && (x.flags & GEE_SYMMETRIZE);
        const int64_t mcap = sym ? 2 * x.E : x.E;
        if (mcap > kMaxEntries) return GEE_ERR_TOO_LARGE;
        GDesc &o = d[g];
        o.src = x.src;
        o.dst = x.dst;
        o.w = x.w;
        o.labels = x.labels;
        o.Z = x.Z;
        o.voff = voff;
        o.E = x.E;
        o.Mcap = mcap;
        o.N = x.N;
        if (p.bucket) noff = (noff + (1 << sb_bucket) - 1) >> sb_bucket << sb_bucket;
        o.node_off = (int)noff;
        o.K = x.K;
        int kp = 1;
        while (kp < x.K && kp < 64) kp <<= 1;
        o.kp = kp;
        o.class_off = (int)ktot;
        o.flags = resident ? (x.flags & ~GEE_SYMMETRIZE) : x.flags;
        o.weighted = x.w != nullptr;
        if (p.bucket) {
            // entries of a bucket part (one wavefront of the bucket path)
            o.WE = x.sc.wave_entries > kBucketMinPart ? x.sc.wave_entries
                   : x.sc.wave_entries ? kBucketMinPart : default_bucket_part(mcap);
            bparts += mcap / o.WE;
        } else {
            o.WE = x.sc.wave_entries ? x.sc.wave_entries : default_wave_entries(mcap);
        }
        o.NWcap = mcap > 0 ? (int)((mcap + o.WE - 1) / o.WE) : 1;
        o.wave_off = (int)woff;
        o.part_off = parts;
        int64_t cb = ((int64_t)x.N + 4095) / 4096;
        o.cnt_blocks = (int)(cb < 1 ? 1 : (cb > 512 ? 512 : cb));
        o.cnt_off = (int)coff;
        o.cpart_off = cpo;
        voff += mcap;
        noff += x.N;
        woff += o.NWcap;
        parts += (int64_t)o.NWcap * x.K;
        coff += o.cnt_blocks;
        cpo += (int64_t)o.cnt_blocks * x.K;
        ktot += x.K;
        if (voff > kMaxEntries || noff > kMaxBatchNodes || woff > INT32_MAX / 2 || coff > INT32_MAX / 2 ||
            ktot > INT32_MAX / 2)
            return GEE_ERR_TOO_LARGE;
        p.Kmax = x.K > p.Kmax ? x.K : p.Kmax;
        p.Kmin = x.K < p.Kmin ? x.K : p.Kmin;
        p.weighted = p.weighted || o.weighted;
        p.any_lap_w = p.any_lap_w || (o.weighted && (x.flags & GEE_LAPLACIAN));
        if (g == 0) {
            wpb = x.sc.waves_per_block;
            sb_req = x.sc.bucket_rows_log2;
        }
    }
    p.io = edge_embed && !resident;
    for (int g = 0; g < G && p.io; ++g) p.io = in_degree_pass(gs[g].flags);
    p.Vtot = voff;
    p.Ntot = noff;
    p.Ktot = (int)ktot;
    p.NWtot = woff;
    p.parts = parts;
    p.cnt_blocks = (int)coff;
    p.cparts = cpo;
    // CSR sort buckets of 2^sb rows (at most 65536 buckets). Dense graphs, whose 256-row
    // buckets average at least twice the staging capacity, take 256-row buckets: nearly
    // all of them go to the pass-C partition, which costs the same per entry whatever the
    // bucket size. Otherwise about 3000 entries a bucket, so most fit one workgroup's LDS.
    const int64_t n1 = p.Ntot > 0 ? p.Ntot : 1;
    const int sb_min = ilog2_ceil(n1) > 16 ? ilog2_ceil(n1) - 16 : 0;
    if (sb_min > kMaxBucketRowsLog2) return GEE_ERR_TOO_LARGE;
    int sb = 0;
    if (p.Vtot > 0) {
        const double per_row = (double)p.Vtot / (double)n1;
        if (256.0 * per_row >= 2.0 * bucket_stage_cap(8)) {
            sb = 8;
        } else {
            const double rows = 3000.0 / per_row;
            while (sb < kMaxBucketRowsLog2 && (double)(2 << sb) <= rows) ++sb;
        }
    } else {
        sb = kMaxBucketRowsLog2;
    }
    if (sb_req > 0) sb = sb_req;
    if (sb < sb_min) sb = sb_min;
    if (sb > kMaxBucketRowsLog2) sb = kMaxBucketRowsLog2;
    if (p.bucket) sb = sb_bucket;
    p.sb = sb;
    p.B = (int32_t)((n1 + (1 << sb) - 1) >> sb);
    const int nbB = ilog2_ceil(p.B);
#ifndef GEE_A_BITS_MAX
#define GEE_A_BITS_MAX 8
#endif
    p.s2 = nbB <= 8 ? 0 : (nbB - GEE_A_BITS_MAX > nbB / 2 ? nbB - GEE_A_BITS_MAX : nbB / 2);
    if (p.s2 > 8) p.s2 = 8;
    p.DA = (int)(((int64_t)p.B + (1 << p.s2) - 1) >> p.s2);
    p.tile = kPartTile;
    p.TA = (p.Vtot + p.tile - 1) / p.tile;
    if (p.TA < 1) p.TA = 1;
    p.TBcap = p.s2 > 0 ? p.TA + p.DA : 1;
    // pass C: every bucket above the staging capacity holds more than cap entries
    p.TCcap = p.sb <= 8 && !p.bucket ? p.TA + p.Vtot / bucket_stage_cap(p.sb) + 1 : 1;
    // bucket path: a bucket of n entries has max(1, ceil(n / P)) <= 1 + floor(n / P) parts;
    // one of several parts has ceil(n / P) <= 2 floor(n / P) partial slots
    p.bparts = p.bucket ? p.B + bparts : 0;
    p.bslots = p.bucket ? 2 * bparts : 0;
    // One wavefront per embed workgroup by default: the LDS ring of each wavefront then
    // limits residency least. Larger workgroups must stay within 64 KiB of LDS.
    const size_t per_wave = embed_lds_per_wave(p.Kmax);
    p.wpb = 1;
    if (wpb > 1 && (size_t)wpb * per_wave <= 65536) p.wpb = wpb;
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
    w = Work();
    w.meta = (int *)take(4 * sizeof(int));
    w.gm = (GMeta *)take((size_t)p.G * sizeof(GMeta));
    if (p.G > 1) {
        w.tab = (GDesc *)take((size_t)p.G * sizeof(GDesc));
        if (p.io) w.tabT = (GDesc *)take((size_t)p.G * sizeof(GDesc));
        w.node_offs = (int *)take((size_t)(p.G + 1) * sizeof(int));
        w.wave_offs = (int *)take((size_t)(p.G + 1) * sizeof(int));
        w.cnt_offs = (int *)take((size_t)(p.G + 1) * sizeof(int));
        w.class_offs = (int *)take((size_t)(p.G + 1) * sizeof(int));
        w.voffs = (int64_t *)take((size_t)(p.G + 1) * sizeof(int64_t));
    }
    if (parts & kPCount) {
        w.counts = (int *)take((size_t)p.Ktot * sizeof(int));
        w.inv_n = (float *)take((size_t)p.Ktot * sizeof(float));
        w.cpart = (int *)take((size_t)p.cparts * sizeof(int));
    }
    if (parts & kPPart) {
        w.ghA = (int *)take((size_t)p.DA * p.TA * sizeof(int));
        w.totA = (int *)take((size_t)p.DA * sizeof(int));
        w.segA = (int *)take((size_t)(p.DA + 1) * sizeof(int));
        w.tileB = (int *)take((size_t)(p.DA + 1) * sizeof(int));
        if (p.s2 > 0) w.ghB = (int *)take(((size_t)p.TBcap << p.s2) * sizeof(int));
        if (p.s2 > 0) w.segB = (int *)take((size_t)p.TBcap * sizeof(int));
        w.bstart = (int *)take((size_t)(p.B + 1) * sizeof(int));
        w.tileC = (int *)take((size_t)(p.B + 1) * sizeof(int));
        w.ghC = (int *)take(((size_t)p.TCcap << p.sb) * sizeof(int));
        // one window of entries past the end: the bucket path reads whole windows
        const size_t vp = (size_t)p.Vtot + kBucketWindowPad;
        w.akey = (int *)take(vp * sizeof(int));
        if (p.s2 > 0) w.tkey = (uint16_t *)take(vp * sizeof(uint16_t));
        w.tcol = (int *)take(vp * sizeof(int));
        if (p.weighted) w.tval = (float *)take(vp * sizeof(float));
    }
    if ((parts & kPCsrOut) && p.bucket) {
        // no CSR: col / val only hold pass A's output when a pass B follows
        if (p.s2 > 0) {
            w.col = (int *)take((size_t)p.Vtot * sizeof(int));
            if (p.weighted) w.val = (float *)take((size_t)p.Vtot * sizeof(float));
        }
    } else if (parts & kPCsrOut) {
        w.rp = (int *)take((size_t)(p.Ntot + 1) * sizeof(int));
        w.col = (int *)take((size_t)p.Vtot * sizeof(int));
        if (p.weighted) w.val = (float *)take((size_t)p.Vtot * sizeof(float));
    }
    if ((parts & kPEmbed) && p.bucket) {
        // (a resident CSR: the bucket starts come from row_ptr, no partition)
        if (!(parts & kPPart)) w.bstart = (int *)take((size_t)(p.B + 1) * sizeof(int));
        w.info = (float2 *)take((size_t)p.Ntot * sizeof(float2));
        w.srow = (float *)take((size_t)p.Ntot * sizeof(float));
        w.part = (int4 *)take((size_t)p.bparts * sizeof(int4));
        w.multi = (int4 *)take((size_t)(p.bslots / 2 + 1) * sizeof(int4));
        w.ptot = (int *)take(4 * 64 * sizeof(int));
        w.bmeta = (int *)take(4 * sizeof(int));
        w.dpart = (float *)take((size_t)p.bslots * 64 * sizeof(float));
        w.zpart = (float *)take(((size_t)p.bslots << p.sb) * (size_t)p.Kmax * sizeof(float));
    } else if (parts & kPEmbed) {
        w.info = (float2 *)take((size_t)p.Ntot * sizeof(float2));
        w.srow = (float *)take((size_t)p.Ntot * sizeof(float));
        w.wrow = (int *)take((size_t)p.NWtot * sizeof(int));
        w.rstep = (uint8_t *)take((size_t)(p.Vtot > 0 ? p.Vtot : 1));
        w.split = (int *)take((size_t)p.NWtot * sizeof(int));
        w.headp = (float *)take((size_t)p.parts * sizeof(float));
        w.tailp = (float *)take((size_t)p.parts * sizeof(float));
        w.headd = (float *)take((size_t)p.NWtot * sizeof(float));
        w.taild = (float *)take((size_t)p.NWtot * sizeof(float));
        w.dsplit = (int *)take((size_t)p.NWtot * sizeof(int));
    }
    return off;
}

// Host images of the batch tables, in the carve order of the device copies.
struct Tables {
    std::vector<int> node_offs, wave_offs, cnt_offs, class_offs;
    std::vector<int64_t> voffs;
};
Tables make_tables(const std::vector<GDesc> &d) {
    Tables t;
    const int G = (int)d.size();
    t.node_offs.resize(G + 1);
    t.wave_offs.resize(G + 1);
    t.cnt_offs.resize(G + 1);
    t.class_offs.resize(G + 1);
    t.voffs.resize(G + 1);
    for (int g = 0; g < G; ++g) {
        t.node_offs[g] = d[g].node_off;
        t.wave_offs[g] = d[g].wave_off;
        t.cnt_offs[g] = d[g].cnt_off;
        t.class_offs[g] = d[g].class_off;
        t.voffs[g] = d[g].voff;
    }
    const GDesc &l = d[G - 1];
    t.node_offs[G] = l.node_off + l.N;
    t.wave_offs[G] = l.wave_off + l.NWcap;
    t.cnt_offs[G] = l.cnt_off + l.cnt_blocks;
    t.class_offs[G] = l.class_off + l.K;
    t.voffs[G] = l.voff + l.Mcap;
    return t;
}

// The descriptors with src and dst swapped: the transposed entries, whose row sums are the
// column sums (in-degrees) of the graphs.
std::vector<GDesc> transposed(const std::vector<GDesc> &d) {
    std::vector<GDesc> t = d;
    for (GDesc &x : t) std::swap(x.src, x.dst);
    return t;
}

// Kernel view of the launch; for G > 1 also writes the tables into the workspace
// (stream-ordered kernels carrying the bytes as arguments, so no host buffer has to
// outlive the call; with sync = true they complete before returning). With bT (plans with
// Plan::io) also the view of the transposed entries.
hipError_t make_batch(const Plan &p, const std::vector<GDesc> &d, const Work &w, hipStream_t s, bool sync,
                      Batch &b, Batch *bT = nullptr) {
    b = Batch();
    b.G = p.G;
    b.gm = w.gm;
    const std::vector<GDesc> dt = p.io ? transposed(d) : std::vector<GDesc>();
    if (p.G == 1) {
        b.one = d[0];
        if (bT) {
            *bT = b;
            if (p.io) bT->one = dt[0];
        }
        return hipSuccess;
    }
    const Tables t = make_tables(d);
    const size_t n = (size_t)(p.G + 1);
    struct Copy {
        void *dst;
        const void *src;
        size_t bytes;
    } copies[] = {{w.tab, d.data(), sizeof(GDesc) * p.G},
                  {w.tabT, p.io ? dt.data() : nullptr, p.io ? sizeof(GDesc) * p.G : 0},
                  {w.node_offs, t.node_offs.data(), sizeof(int) * n},
                  {w.wave_offs, t.wave_offs.data(), sizeof(int) * n},
                  {w.cnt_offs, t.cnt_offs.data(), sizeof(int) * n},
                  {w.class_offs, t.class_offs.data(), sizeof(int) * n},
                  {w.voffs, t.voffs.data(), sizeof(int64_t) * n}};
    for (const Copy &c : copies) {
        if (!c.bytes) continue;
        hipError_t e = launch_upload(c.dst, c.src, c.bytes, s);
        if (e != hipSuccess) return e;
    }
    if (sync) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
    }
    b.tab = w.tab;
    b.node_offs = w.node_offs;
    b.wave_offs = w.wave_offs;
    b.cnt_offs = w.cnt_offs;
    b.class_offs = w.class_offs;
    b.voffs = w.voffs;
    if (bT) {
        *bT = b;
        if (p.io) bT->tab = w.tabT;
    }
    return hipSuccess;
}

// Kernel sequence of gee_embed over a batch (edge lists -> Z). bT: the view of the
// transposed entries (used when p.io).
hipError_t enqueue_embed(const Batch &b, const Batch &bT, const Plan &p, const Work &wk, unsigned *st,
                         hipStream_t s) {
    CountJob job;
    job.part = wk.cpart;
    job.counts = wk.counts;
    job.inv_n = wk.inv_n;
    job.slices = p.cnt_blocks;
    job.classes = p.Ktot;
    if (p.io) {
        // in-degrees: the transposed entries partitioned by their rows (the columns), c_j from
        // their sums; then the entries themselves, s_i from the out-degrees, and the class sums
        if (!p.bucket) return hipErrorNotSupported;  // excluded on the host (plan_chunks)
        hipError_t e = launch_csr_build(bT, p, wk, st, s, &job);
        if (e == hipSuccess) e = launch_bucket_embed(bT, p, wk, s, kDegIn, false);
        if (e == hipSuccess) e = launch_csr_build(b, p, wk, st, s, nullptr);
        if (e == hipSuccess) e = launch_bucket_embed(b, p, wk, s, kDegOut, true);
        return e;
    }
    hipError_t e = launch_csr_build(b, p, wk, st, s, &job);
    if (p.bucket) return e == hipSuccess ? launch_bucket_embed(b, p, wk, s) : e;
    if (e == hipSuccess) e = launch_csr_pass2(p, wk, st, s);
    if (e == hipSuccess) e = launch_graph_meta(b, wk.rp, 0, s);
    const float *val = p.weighted ? wk.val : nullptr;
    if (e == hipSuccess) e = launch_node_prep(b, p, wk.rp, val, p.Vtot, wk, st, s);
    if (e == hipSuccess) e = launch_embed(b, p, wk.rp, wk.col, val, p.Vtot, wk, st, s);
    return e;
}

// `sizing`: only sizes are read (workspace queries), device pointers are not checked.
int graphs_from_api(const gee_graph *graphs, int32_t G, std::vector<GraphIn> &out, bool sizing = false) {
    if (!graphs || G < 1 || G > kMaxBatchGraphs) return GEE_ERR_ARG;
    out.resize(G);
    for (int g = 0; g < G; ++g) {
        const gee_graph &x = graphs[g];
        GraphIn &o = out[g];
        o.src = x.src;
        o.dst = x.dst;
        o.w = x.w;
        o.E = x.E;
        o.N = x.N;
        o.labels = x.labels;
        o.K = x.K;
        o.flags = x.flags;
        o.Z = x.Z;
        o.sc = x.sched;
        if (x.E < 0 || x.N < 0) return GEE_ERR_ARG;
        if (!sizing && ((x.E > 0 && (!x.src || !x.dst)) || (x.N > 0 && (!x.labels || !x.Z)))) return GEE_ERR_ARG;
        if (x.N == 0 && x.E > 0) return GEE_ERR_ARG;
    }
    return GEE_OK;
}

// A batch as chunks, each launched on its own (one after the other on the stream) so that
// every graph takes the path and bucket size it takes alone: graphs are grouped by their
// preferred bucket size (64 rows for K <= 64, else 32) and packed in order while their
// rows, each graph rounded up to that bucket size, total at most kMaxBuckets buckets; a
// graph of more rows forms a chunk of its own. The summation order, and so every bit of Z,
// depends on the bucket size, so this keeps batched and plain results identical.
struct Chunk {
    std::vector<GraphIn> gs;
    Plan p;
    std::vector<GDesc> d;
    size_t off = 0;  // workspace offset
};
constexpr unsigned kEmbedParts = kPCount | kPPart | kPCsrOut | kPEmbed;
// Rows of a chunk of several graphs, at most (a larger graph takes a chunk of its own): fewer
// rows per launch mean fewer pass-A digits, hence longer runs per tile in the pass-A scatter.
#ifndef GEE_CHUNK_ROWS_LOG2
#define GEE_CHUNK_ROWS_LOG2 22
#endif
int plan_chunks(const std::vector<GraphIn> &gs, std::vector<Chunk> &out, size_t &total) {
    out.clear();
    for (int sbp : {6, GEE_BUCKET_SB_MIN}) {
        const int64_t cap = std::min((int64_t)kMaxBuckets << sbp, (int64_t)1 << GEE_CHUNK_ROWS_LOG2);
        std::vector<GraphIn> cur;
        int64_t rows = 0;
        auto flush = [&]() {
            if (!cur.empty()) {
                out.emplace_back();
                out.back().gs.swap(cur);
            }
            cur.clear();
            rows = 0;
        };
        // graphs that need the transposed pass (in-degrees) form chunks of their own
        for (int io = 0; io < 2; ++io) {
            for (const GraphIn &x : gs) {
                if (preferred_bucket_sb(x) != sbp || (int)in_degree_pass(x.flags) != io) continue;
                const int64_t n = x.N;
                if (n > cap) {
                    flush();
                    cur.push_back(x);
                    flush();
                    continue;
                }
                const int64_t next = ((rows + (1 << sbp) - 1) >> sbp << sbp) + n;
                if (!cur.empty() && next > cap) {
                    flush();
                    rows = n;
                } else {
                    rows = next;
                }
                cur.push_back(x);
            }
            flush();
        }
        if (sbp == GEE_BUCKET_SB_MIN) break;
    }
    total = 0;
    for (Chunk &c : out) {
        int rc = make_plan(c.gs.data(), (int)c.gs.size(), false, c.p, c.d, true);
        if (rc) return rc;
        // in-degrees come from the bucket path's transposed pass only
        if (c.p.io && !c.p.bucket) return GEE_ERR_UNSUPPORTED;
        Work w;
        c.off = total;
        total += (carve(c.p, kEmbedParts, nullptr, w) + kAlign - 1) / kAlign * kAlign;
    }
    return GEE_OK;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }
int embed_batch(const gee_graph *graphs, int32_t G, void *workspace, size_t workspace_bytes, void *stream,
                int *rcnt = nullptr, bool *counts_given = nullptr, int2 *zs_pairs = nullptr,
                int *zs_sb = nullptr);
// Stream of a call about to enqueue kernels. HIP keeps a thread's last error until it is
// read; one left by the application's own earlier calls is consumed here, so the checks
// after this call's launches see only this call's launches.
hipStream_t launch_stream(void *s) {
    (void)hipGetLastError();
    return as_stream(s);
}

}  // namespace

namespace gee {

const char *const kKernelNames[kKNumKernels] = {
    "class_count_partial", "class_count_final", "a_hist", "digit_scan", "a_scatter",
    "b_hist", "b_scan", "b_scatter", "c_tiles", "c_hist", "c_scan", "c_scatter", "bucket_sort", "graph_meta", "zero_steps", "node_rows",
    "degree_rows", "degree_fixup", "node_coef", "fill_empty", "embed_rows", "embed_fixup", "bucket_part_count",
    "bucket_part_fill", "bucket_degree", "bucket_degree_fix", "bucket_embed", "bucket_embed_fix",
    "edge_init", "edge_prep", "edge_coef", "edge_scatter", "edge_finish", "zs_count", "zs_write", "zs_tile_sum", "csr_prep"};

void prof_begin(int kid, hipStream_t s) {
    if (!g_prof_active.load(std::memory_order_relaxed) || t_capturing) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof[kid].start) (void)hipEventRecord(g_prof[kid].start, s);
}

void prof_end(int kid, hipStream_t s) {
    if (!g_prof_active.load(std::memory_order_relaxed) || t_capturing) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof[kid].stop) (void)hipEventRecord(g_prof[kid].stop, s);
}

}  // namespace gee

// Batch plan: a workspace, the uploaded tables and the captured launch sequence.
struct gee_batch_plan {
    int device = 0;
    unsigned *status = nullptr;  // the plan's data-error word (in ws)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int G = 0;
};

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
    case GEE_ERR_TOO_LARGE: return "sizes beyond the library's limits";
    case GEE_ERR_OOM: return "device out of memory";
    case GEE_ERR_HIP: return "HIP runtime error";
    case GEE_ERR_UNSUPPORTED: return "unsupported request";
    case GEE_ERR_WORKSPACE: return "workspace too small";
    case GEE_ERR_SCRATCH: return "request needs more than the library's fixed scratch (gee_scratch_bytes)";
    default: return "unknown status";
    }
}

const char *gee_last_hip_error(void) {
    return t_last_hip == hipSuccess ? "" : hipGetErrorString(t_last_hip);
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
    std::lock_guard<std::mutex> lk(g_status_mu);
    DevState *ds = nullptr;
    return device_state(&ds);
}

int gee_get_data_errors(void *stream, uint32_t *bits) {
    if (!bits) return GEE_ERR_ARG;
    unsigned *st = nullptr;
    int rc = stream_status(as_stream(stream), &st);
    if (rc) return rc;
    // take the word (atomically, in stream order), then copy what was taken
    hipStream_t s = launch_stream(stream);
    hipLaunchKernelGGL(status_take, dim3(1), dim3(1), 0, s, st);
    hipError_t e = hipGetLastError();
    unsigned h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, st + 1, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e);
    *bits = h;
    return GEE_OK;
}

int gee_take_data_errors_async(void *stream, uint32_t *dst) {
    if (!dst) return GEE_ERR_ARG;
    unsigned *st = nullptr;
    int rc = stream_status(as_stream(stream), &st);
    if (rc) return rc;
    hipStream_t s = launch_stream(stream);
    hipLaunchKernelGGL(status_take_to, dim3(1), dim3(1), 0, s, st, dst);
    return hip_status(hipGetLastError());
}

size_t gee_scratch_bytes(void) { return kScratchBytes; }

int gee_default_schedule(int64_t E, int32_t N, int32_t K, uint32_t flags, gee_schedule *out) {
    if (!out || E < 0) return GEE_ERR_ARG;
    GraphIn x;
    x.E = E;
    x.N = N;
    x.K = K;
    x.flags = flags;
    Plan p;
    std::vector<GDesc> d;
    int rc = make_plan(&x, 1, false, p, d, true);
    if (rc) return rc;
    out->wave_entries = d[0].WE;
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
    if ((rc = stream_status(as_stream(stream), &st))) return rc;
    GraphIn x;
    x.N = N;
    x.K = K;
    x.labels = labels;
    Plan p;
    std::vector<GDesc> d;
    if ((rc = make_plan(&x, 1, false, p, d))) return rc;
    Batch b;
    b.one = d[0];
    b.status = st;
    hipStream_t s = launch_stream(stream);
    int *part = nullptr;
    hipError_t e = hipMallocAsync((void **)&part, (size_t)p.cparts * sizeof(int), s);
    if (e != hipSuccess) return hip_status(e);
    e = launch_class_counts(b, p, part, counts, nullptr, st, s);
    hipError_t e2 = hipFreeAsync(part, s);
    return hip_status(e != hipSuccess ? e : e2);
}

// --------------------------------------------------------------------------- CSR build

size_t gee_build_csr_workspace_bytes(int64_t E, int32_t N, uint32_t flags, const gee_schedule *sched) {
    GraphIn x;
    x.E = E;
    x.N = N;
    x.flags = flags;
    x.w = reinterpret_cast<const float *>(16);  // sized with weights, so one size serves both
    if (sched) x.sc = *sched;
    Plan p;
    std::vector<GDesc> d;
    if (E < 0 || make_plan(&x, 1, false, p, d)) return 0;
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
    if ((rc = stream_status(as_stream(stream), &st))) return rc;
    GraphIn x;
    x.src = src;
    x.dst = dst;
    x.w = wgt;
    x.E = E;
    x.N = N;
    x.flags = flags;
    if (sched) x.sc = *sched;
    Plan p;
    std::vector<GDesc> d;
    if ((rc = make_plan(&x, 1, false, p, d))) return rc;
    if (!workspace || workspace_bytes < gee_build_csr_workspace_bytes(E, N, flags, sched)) return GEE_ERR_WORKSPACE;
    Work wk;
    carve(p, kPPart, (char *)workspace, wk);
    hipStream_t s = launch_stream(stream);
    if (N == 0) return hip_status(hipMemsetAsync(row_ptr, 0, sizeof(int32_t), s));
    wk.rp = row_ptr;
    wk.col = col;
    wk.val = wgt ? val : nullptr;
    Batch b;
    b.one = d[0];
    b.status = st;
    hipError_t e = launch_csr_build(b, p, wk, st, s);
    if (e == hipSuccess) e = launch_csr_pass2(p, wk, st, s);
    return hip_status(e);
}

int gee_build_csr(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
                  uint32_t flags, int32_t *row_ptr, int32_t *col, float *val, void *stream) {
    size_t bytes = gee_build_csr_workspace_bytes(E, N, flags, nullptr);
    if (bytes == 0) {
        if (E < 0) return GEE_ERR_ARG;
        const int rc = check_common(N, 1, flags);
        return rc ? rc : GEE_ERR_TOO_LARGE;
    }
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
    GraphIn x;
    x.E = E;
    x.N = N;
    x.K = K;
    x.flags = flags;
    x.w = weighted ? reinterpret_cast<const float *>(16) : nullptr;
    if (sched) x.sc = *sched;
    Plan p;
    std::vector<GDesc> d;
    if (E < 0 || make_plan(&x, 1, false, p, d, true)) return 0;
    Work w;
    return carve(p, kPCount | kPPart | kPCsrOut | kPEmbed, nullptr, w);
}

int gee_embed_ws(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
                 const int32_t *labels, int32_t K, uint32_t flags, float *Z, const gee_schedule *sched,
                 void *workspace, size_t workspace_bytes, void *stream) {
    gee_graph g;
    g.src = src;
    g.dst = dst;
    g.w = wgt;
    g.E = E;
    g.N = N;
    g.labels = labels;
    g.K = K;
    g.flags = flags;
    g.Z = Z;
    g.sched = sched ? *sched : gee_schedule{0, 0, 0, 0};
    return gee_embed_batch_ws(&g, 1, workspace, workspace_bytes, stream);
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

// --------------------------------------------------------------------------- without allocation

int gee_embed_noalloc(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
                      const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *stream) {
    if (E < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    if (N == 0) return E > 0 ? GEE_ERR_ARG : GEE_OK;
    const size_t need = gee_embed_workspace_bytes(E, N, K, flags, wgt != nullptr, nullptr);
    if (need == 0) return GEE_ERR_TOO_LARGE;
    if (need > kScratchBytes) return GEE_ERR_SCRATCH;
    void *sc = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_status_mu);
        DevState *ds = nullptr;
        if ((rc = device_state(&ds))) return rc;
        sc = ds->scratch;
    }
    return gee_embed_ws(src, dst, wgt, E, N, labels, K, flags, Z, nullptr, sc, kScratchBytes, stream);
}

// --------------------------------------------------------------------------- sparse Z

// Staged sparse Z: on the bucket path the class scatter writes only the non-zero pairs, each
// bucket's from the place of its first row in a dense Z (r0 K: a bucket never holds more
// pairs than its rows have classes, whatever the values), into N K staging pairs (class,
// value bits): twice a dense Z's bytes, of which only the non-zero pairs are touched.
// The region also holds a dense Z (the CSR path).
static size_t zs_region_bytes(int32_t N, int32_t K) {
    return (size_t)N * K * sizeof(float) * (GEE_ZS_STAGED ? 2 : 1);
}

size_t gee_embed_sparse_workspace_bytes(int64_t E, int32_t N, int32_t K, uint32_t flags, int weighted,
                                        const gee_schedule *sched) {
    if (E < 0 || check_common(N, K, flags) || (int64_t)N * K > INT32_MAX) return 0;
    if (N == 0) return kAlign;
    const size_t eb = gee_embed_workspace_bytes(E, N, K, flags, weighted, sched);
    if (eb == 0) return 0;
    auto up = [](size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); };
    return up(eb) + up(zs_region_bytes(N, K)) + up((size_t)zsparse_tiles(N) * sizeof(int)) +
           up((size_t)N * sizeof(int));
}

int gee_embed_sparse_ws(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
                        const int32_t *labels, int32_t K, uint32_t flags, int32_t *row_ptr, int32_t *col,
                        float *val, int64_t capacity, const gee_schedule *sched, void *workspace,
                        size_t workspace_bytes, void *stream) {
    if (E < 0 || capacity < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    if ((int64_t)N * K > INT32_MAX) return GEE_ERR_TOO_LARGE;
    if (!row_ptr || (capacity > 0 && (!col || !val))) return GEE_ERR_ARG;
    if (N == 0) {
        if (E > 0) return GEE_ERR_ARG;
        return hip_status(hipMemsetAsync(row_ptr, 0, sizeof(int32_t), launch_stream(stream)));
    }
    const size_t need = gee_embed_sparse_workspace_bytes(E, N, K, flags, wgt != nullptr, sched);
    if (need == 0) return GEE_ERR_TOO_LARGE;
    if (!workspace || workspace_bytes < need) return GEE_ERR_WORKSPACE;
    auto up = [](size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); };
    const size_t eb = up(gee_embed_workspace_bytes(E, N, K, flags, wgt != nullptr, sched));
    char *base = static_cast<char *>(workspace);
    float *Zd = reinterpret_cast<float *>(base + eb);
    int *tile = reinterpret_cast<int *>(base + eb + up(zs_region_bytes(N, K)));
    int *rcnt = tile + up((size_t)zsparse_tiles(N) * sizeof(int)) / sizeof(int);
    int2 *zpairs = GEE_ZS_STAGED ? reinterpret_cast<int2 *>(Zd) : nullptr;
    // the class-scatter kernels count each row's non-zero entries as they write it (bucket
    // path), so the compaction reads Z once
    gee_graph g;
    g.src = src;
    g.dst = dst;
    g.w = wgt;
    g.E = E;
    g.N = N;
    g.labels = labels;
    g.K = K;
    g.flags = flags;
    g.Z = Zd;
    g.sched = sched ? *sched : gee_schedule{0, 0, 0, 0};
    bool counts_given = false;
    int sb = -1;
    rc = embed_batch(&g, 1, workspace, eb, stream, rcnt, &counts_given, zpairs, &sb);
    if (rc) return rc;
    if (sb >= 0)  // the bucket kernels staged the non-zero pairs: no dense Z was written
        return hip_status(launch_zsparse_staged(N, K, sb, zpairs, tile, rcnt, row_ptr, col, val, capacity,
                                                as_stream(stream)));
    return hip_status(launch_zsparse(Zd, N, K, tile, rcnt, row_ptr, col, val, capacity, counts_given,
                                     as_stream(stream)));
}

int gee_embed_sparse(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
                     const int32_t *labels, int32_t K, uint32_t flags, int32_t *row_ptr, int32_t *col,
                     float *val, int64_t capacity, void *stream) {
    if (E < 0 || capacity < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    const size_t bytes = gee_embed_sparse_workspace_bytes(E, N, K, flags, wgt != nullptr, nullptr);
    if (bytes == 0) return GEE_ERR_TOO_LARGE;
    hipStream_t s = as_stream(stream);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, bytes, s);
    if (e != hipSuccess) return hip_status(e);
    rc = gee_embed_sparse_ws(src, dst, wgt, E, N, labels, K, flags, row_ptr, col, val, capacity, nullptr, ws,
                             bytes, stream);
    e = hipFreeAsync(ws, s);
    return rc ? rc : hip_status(e);
}

// --------------------------------------------------------------------------- original GEE form

size_t gee_embed_atomic_workspace_bytes(int32_t N, int32_t K, uint32_t flags) {
    if (check_common(N, K, flags)) return 0;
    return edge_workspace_bytes(N, K, flags);
}

int gee_embed_atomic_ws(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
                        const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *workspace,
                        size_t workspace_bytes, void *stream) {
    if (E < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    if (N == 0) return E > 0 ? GEE_ERR_ARG : GEE_OK;
    if (!labels || !Z || (E > 0 && (!src || !dst))) return GEE_ERR_ARG;
    if (!workspace || workspace_bytes < edge_workspace_bytes(N, K, flags)) return GEE_ERR_WORKSPACE;
    unsigned *st = nullptr;
    if ((rc = stream_status(as_stream(stream), &st))) return rc;
    hipStream_t s = launch_stream(stream);
    return hip_status(launch_edge_embed(src, dst, wgt, E, N, labels, K, flags, Z, workspace, st, s));
}

int gee_embed_atomic(const int32_t *src, const int32_t *dst, const float *wgt, int64_t E, int32_t N,
                     const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *stream) {
    if (E < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    if (N == 0) return E > 0 ? GEE_ERR_ARG : GEE_OK;
    const size_t bytes = edge_workspace_bytes(N, K, flags);
    hipStream_t s = as_stream(stream);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, bytes, s);
    if (e != hipSuccess) return hip_status(e);
    rc = gee_embed_atomic_ws(src, dst, wgt, E, N, labels, K, flags, Z, ws, bytes, stream);
    e = hipFreeAsync(ws, s);
    return rc ? rc : hip_status(e);
}

// --------------------------------------------------------------------------- batches

size_t gee_embed_batch_workspace_bytes(const gee_graph *graphs, int32_t G) {
    std::vector<GraphIn> gs;
    if (graphs_from_api(graphs, G, gs, true)) return 0;
    std::vector<Chunk> ch;
    size_t total = 0;
    if (plan_chunks(gs, ch, total)) return 0;
    return total;
}

}  // extern "C"

namespace {

// gee_embed_batch_ws; with rcnt (a single graph), the class-scatter kernels also write each Z
// row's number of non-zero entries there when the graph takes the bucket path, and
// *counts_given says whether they did. With zs_pairs (N K pairs) as well they write the
// non-zero (class, value bits) pairs there instead of a dense Z (staged sparse Z; each
// bucket's from its first row's place in a dense Z), and *zs_sb gives the bucket size (log2
// rows, at most 8; -1 when no staging took place).
int embed_batch(const gee_graph *graphs, int32_t G, void *workspace, size_t workspace_bytes, void *stream,
                int *rcnt, bool *counts_given, int2 *zs_pairs, int *zs_sb) {
    if (counts_given) *counts_given = false;
    if (zs_sb) *zs_sb = -1;
    std::vector<GraphIn> gs;
    int rc = graphs_from_api(graphs, G, gs);
    if (rc) return rc;
    std::vector<Chunk> ch;
    size_t total = 0;
    if ((rc = plan_chunks(gs, ch, total))) return rc;
    int64_t rows = 0;
    for (const Chunk &c : ch) rows += c.p.Ntot;
    if (rows == 0) return GEE_OK;
    unsigned *st = nullptr;
    if ((rc = stream_status(as_stream(stream), &st))) return rc;
    if (!workspace || workspace_bytes < total) return GEE_ERR_WORKSPACE;
    hipStream_t s = launch_stream(stream);
    hipError_t e = hipSuccess;
    for (const Chunk &c : ch) {
        if (c.p.Ntot == 0) continue;
        Work wk;
        carve(c.p, kEmbedParts, (char *)workspace + c.off, wk);
        if (rcnt && G == 1 && c.p.bucket) {
            wk.rcnt = rcnt;
            *counts_given = true;
            if (zs_pairs && zs_sb && c.p.sb <= 8) {
                wk.zs_pairs = zs_pairs;
                *zs_sb = c.p.sb;
            }
        }
        Batch b;
        Batch bT;
        e = make_batch(c.p, c.d, wk, s, false, b, &bT);
        b.status = bT.status = st;
        if (e == hipSuccess) e = enqueue_embed(b, bT, c.p, wk, st, s);
        if (e != hipSuccess) break;
    }
    return hip_status(e);
}

}  // namespace

extern "C" {

int gee_embed_batch_ws(const gee_graph *graphs, int32_t G, void *workspace, size_t workspace_bytes,
                       void *stream) {
    return embed_batch(graphs, G, workspace, workspace_bytes, stream);
}

}  // extern "C"

namespace {

// Lays the chunks of `graphs` out in the plan's workspace (after its data-error word),
// uploads their tables (completed before returning) and captures their launch sequence in
// a new hipGraph. The plan's workspace must hold them (GEE_ERR_WORKSPACE otherwise, with
// nothing changed).
int plan_capture(gee_batch_plan *pl, const gee_graph *graphs, int32_t G, hipGraph_t *out) {
    *out = nullptr;
    std::vector<GraphIn> gs;
    int rc = graphs_from_api(graphs, G, gs);
    if (rc) return rc;
    std::vector<Chunk> ch;
    size_t total = 0;
    if ((rc = plan_chunks(gs, ch, total))) return rc;
    int64_t rows = 0;
    for (const Chunk &c : ch) rows += c.p.Ntot;
    if (rows == 0) return GEE_ERR_ARG;
    if (kAlign + total > pl->ws_bytes) return GEE_ERR_WORKSPACE;
    unsigned *st = pl->status;
    char *wsb = static_cast<char *>(pl->ws) + kAlign;
    // every chunk has its own workspace region, so all tables are written before capture
    std::vector<Batch> bs(ch.size()), bTs(ch.size());
    std::vector<Work> wks(ch.size());
    (void)hipGetLastError();  // see launch_stream
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < ch.size() && e == hipSuccess; ++i) {
        if (ch[i].p.Ntot == 0) continue;
        carve(ch[i].p, kEmbedParts, wsb + ch[i].off, wks[i]);
        e = make_batch(ch[i].p, ch[i].d, wks[i], nullptr, true, bs[i], &bTs[i]);
        bs[i].status = bTs[i].status = st;
    }
    hipStream_t cs = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        t_capturing = true;
        hipError_t e1 = hipSuccess;
        for (size_t i = 0; i < ch.size() && e1 == hipSuccess; ++i)
            if (ch[i].p.Ntot > 0) e1 = enqueue_embed(bs[i], bTs[i], ch[i].p, wks[i], st, cs);
        t_capturing = false;
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        e = e1 != hipSuccess ? e1 : e2;
        if (e == hipSuccess) *out = g;
        else if (g) (void)hipGraphDestroy(g);
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (e == hipSuccess) pl->G = G;
    return hip_status(e);
}

}  // namespace

extern "C" {

int gee_batch_plan_create_ws(const gee_graph *graphs, int32_t G, size_t min_workspace_bytes,
                             gee_batch_plan **out) {
    if (!out) return GEE_ERR_ARG;
    *out = nullptr;
    std::vector<GraphIn> gs;
    int rc = graphs_from_api(graphs, G, gs);
    if (rc) return rc;
    std::vector<Chunk> ch;
    size_t total = 0;
    if ((rc = plan_chunks(gs, ch, total))) return rc;
    int64_t rows = 0;
    for (const Chunk &c : ch) rows += c.p.Ntot;
    if (rows == 0) return GEE_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(g_status_mu);
        DevState *ds = nullptr;
        if ((rc = device_state(&ds))) return rc;
    }
    gee_batch_plan *pl = new (std::nothrow) gee_batch_plan();
    if (!pl) return GEE_ERR_OOM;
    (void)hipGetDevice(&pl->device);
    // the plan's own data-error word (first kAlign bytes), then the chunks' workspaces
    pl->ws_bytes = kAlign + (total > min_workspace_bytes ? total : min_workspace_bytes);
    hipError_t e = hipMalloc(&pl->ws, pl->ws_bytes);
    if (e != hipSuccess) {
        gee_batch_plan_destroy(pl);
        return hip_status(e);
    }
    pl->status = static_cast<unsigned *>(pl->ws);
    (void)hipGetLastError();  // see launch_stream
    hipLaunchKernelGGL(status_take, dim3(1), dim3(1), 0, nullptr, pl->status);  // word = 0
    e = hipGetLastError();
    if (e != hipSuccess) {
        gee_batch_plan_destroy(pl);
        return hip_status(e);
    }
    hipGraph_t g = nullptr;
    rc = plan_capture(pl, graphs, G, &g);
    if (rc == GEE_OK) {
        pl->graph = g;
        rc = hip_status(hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0));
    }
    if (rc != GEE_OK) {
        gee_batch_plan_destroy(pl);
        return rc;
    }
    *out = pl;
    return GEE_OK;
}

int gee_batch_plan_create(const gee_graph *graphs, int32_t G, gee_batch_plan **out) {
    return gee_batch_plan_create_ws(graphs, G, 0, out);
}

size_t gee_batch_plan_workspace_bytes(const gee_batch_plan *plan) { return plan ? plan->ws_bytes - kAlign : 0; }

int gee_batch_plan_update(gee_batch_plan *plan, const gee_graph *graphs, int32_t G) {
    if (!plan || !plan->exec) return GEE_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return GEE_ERR_ARG;
    hipGraph_t g = nullptr;
    int rc = plan_capture(plan, graphs, G, &g);
    if (rc == GEE_ERR_HIP || rc == GEE_ERR_OOM) {
        // the tables in the workspace may be half rewritten: the plan cannot run any more
        (void)hipGraphExecDestroy(plan->exec);
        plan->exec = nullptr;
    }
    if (rc != GEE_OK) return rc;
    // same launch sequence (the same chunks, paths and kernels): the executable graph takes
    // the new kernel arguments and grids in place; otherwise it is instantiated again
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    hipError_t e = hipGraphExecUpdate(plan->exec, g, &bad, &res);
    if (e != hipSuccess || res != hipGraphExecUpdateSuccess) {
        (void)hipGetLastError();  // the failed in-place update is not the caller's error
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_status(e);
        }
        (void)hipGraphExecDestroy(plan->exec);
        plan->exec = x;
    }
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    plan->graph = g;
    return GEE_OK;
}

int gee_batch_plan_launch(gee_batch_plan *plan, void *stream) {
    if (!plan || !plan->exec) return GEE_ERR_ARG;
    unsigned *st = nullptr;
    int rc = stream_status(as_stream(stream), &st);
    if (rc) return rc;
    hipStream_t s = launch_stream(stream);
    hipError_t e = hipGraphLaunch(plan->exec, s);
    // the plan's data errors move to the launch stream's word
    if (e == hipSuccess) {
        hipLaunchKernelGGL(status_fold, dim3(1), dim3(1), 0, s, plan->status, st);
        e = hipGetLastError();
    }
    return hip_status(e);
}

int gee_batch_plan_destroy(gee_batch_plan *plan) {
    if (!plan) return GEE_OK;
    hipError_t e = hipSuccess;
    if (plan->exec) e = hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->ws) {
        hipError_t e2 = hipFree(plan->ws);
        if (e == hipSuccess) e = e2;
    }
    delete plan;
    return hip_status(e);
}

// --------------------------------------------------------------------------- embed from CSR

// gee_embed_csr runs the bucket kernels (rows from row_ptr) unless its schedule asks for the
// CSR path's kernels: wave_entries or waves_per_block set with no 32- or 64-row bucket size.
// Past the bucket kernels' row limit it takes the CSR path's kernels in any case.
bool resident_bucket_mode(const GraphIn &x) {
    if (x.sc.bucket_rows_log2 == 5 || x.sc.bucket_rows_log2 == 6) return true;
    return x.sc.wave_entries == 0 && x.sc.waves_per_block == 0 && x.sc.bucket_rows_log2 == 0;
}

size_t gee_embed_csr_workspace_bytes(int64_t M, int32_t N, int32_t K, uint32_t flags,
                                     const gee_schedule *sched) {
    GraphIn x;
    x.E = M;
    x.N = N;
    x.K = K;
    x.flags = flags;
    x.w = reinterpret_cast<const float *>(16);
    if (sched) x.sc = *sched;
    Plan p;
    std::vector<GDesc> d;
    if (M < 0 || make_plan(&x, 1, true, p, d, false, resident_bucket_mode(x))) return 0;
    Work w;
    return carve(p, kPCount | kPEmbed, nullptr, w);
}

// A resident CSR carries no column sums: the directed-degree Laplacian needs the edge list.
bool csr_unsupported(uint32_t flags) { return (flags & GEE_DIRECTED_DEGREES) && (flags & GEE_LAPLACIAN); }

int gee_embed_csr_ws(const int32_t *row_ptr, const int32_t *col, const float *val, int64_t M, int32_t N,
                     const int32_t *labels, int32_t K, uint32_t flags, float *Z,
                     const gee_schedule *sched, void *workspace, size_t workspace_bytes, void *stream) {
    if (M < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    if (csr_unsupported(flags)) return GEE_ERR_UNSUPPORTED;
    if (N == 0) return M > 0 ? GEE_ERR_ARG : GEE_OK;
    if (!row_ptr || !labels || !Z || (M > 0 && !col)) return GEE_ERR_ARG;
    unsigned *st = nullptr;
    if ((rc = stream_status(as_stream(stream), &st))) return rc;
    GraphIn x;
    x.E = M;
    x.N = N;
    x.K = K;
    x.flags = flags;
    x.w = val;
    x.labels = labels;
    x.Z = Z;
    if (sched) x.sc = *sched;
    Plan p;
    std::vector<GDesc> d;
    if ((rc = make_plan(&x, 1, true, p, d, false, resident_bucket_mode(x)))) return rc;
    Work wk;
    const unsigned parts = kPCount | kPEmbed;
    if (!workspace || workspace_bytes < gee_embed_csr_workspace_bytes(M, N, K, flags, sched))
        return GEE_ERR_WORKSPACE;
    carve(p, parts, (char *)workspace, wk);
    hipStream_t s = launch_stream(stream);
    Batch b;
    b.one = d[0];
    b.status = st;
    b.gm = wk.gm;
    if (p.bucket) {  // the bucket kernels, rows from row_ptr; meta[1] holds the CSR's check
        // (the class totals are added up by extra workgroups of the CSR checks' launch)
        hipError_t e = launch_class_counts(b, p, wk.cpart, wk.counts, wk.inv_n, st, s, wk.meta + 1, false);
        if (e == hipSuccess) e = launch_bucket_embed_csr(b, p, wk, row_ptr, col, val, M, st, s);
        return hip_status(e);
    }
    hipError_t e = launch_class_counts(b, p, wk.cpart, wk.counts, wk.inv_n, st, s);
    if (e == hipSuccess) e = launch_graph_meta(b, nullptr, (int)M, s);
    if (e == hipSuccess) e = launch_node_prep(b, p, row_ptr, val, M, wk, st, s);
    if (e == hipSuccess) e = launch_embed(b, p, row_ptr, col, val, M, wk, st, s);
    return hip_status(e);
}

int gee_embed_csr(const int32_t *row_ptr, const int32_t *col, const float *val, int64_t M, int32_t N,
                  const int32_t *labels, int32_t K, uint32_t flags, float *Z, void *stream) {
    if (M < 0) return GEE_ERR_ARG;
    int rc = check_common(N, K, flags);
    if (rc) return rc;
    if (csr_unsupported(flags)) return GEE_ERR_UNSUPPORTED;
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
