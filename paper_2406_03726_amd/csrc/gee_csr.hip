// gee_csr.hip - edge list -> CSR on the device (Section 3 layout), deterministic.
//
// The adjacency entries of an edge list are the rows themselves and, under
// symmetrization, their mirrors: virtual entry 2e is (src_e -> dst_e) and 2e+1 is
// (dst_e -> src_e), the latter absent for a self-loop. The CSR is a stable sort of
// that sequence by row index. A batch sorts the concatenation of its graphs' sequences
// with every graph's rows and columns offset by its first node, so each graph's slice of
// the result is its own CSR. Rows are grouped in buckets of 2^sb consecutive rows
// (a few thousand entries each); the bucket id is split into a high digit (at most 256
// values) and a low digit (2^s2 values), and the sort is three stable passes:
//
//   pass A  partition the virtual entries by high digit      (a_hist, digit_scan,
//                                                              a_scatter)
//   pass B  partition each high-digit segment by low digit    (seg_hist, seg_scan,
//                                                              seg_scatter)
//   pass C  buckets within the staging capacity (bucket_stage_cap): one workgroup per
//           bucket, row counts -> row_ptr, then the entries in row order (bucket_sort)
//           larger buckets (they hold hub rows): the segment partition once more with
//           the row inside the bucket as the digit, over many workgroups (c_tiles,
//           seg_hist, seg_scan, seg_scatter)
//
// With few buckets (s2 = 0) pass A partitions by bucket and pass B is skipped. The bucket
// path (gee_bucket.hip) stops after pass B: it needs each bucket's entries together, not
// the rows in order.
//
// Tiles are numbered so that each XCD takes one contiguous range of them (xcd_order): the
// runs that neighbouring tiles write end and start in the same cache lines, which one L2
// then merges. Every partition pass works on tiles of kPartTile entries: the tile's entries are ranked
// by digit (stable) and staged in LDS in digit order, then written out so that
// consecutive threads write consecutive addresses of each digit's run; no pass writes
// scattered single words. Stable ranks never use global atomics: each wavefront owns a
// contiguous part of the tile and ranks its items against its own per-digit running
// positions in LDS (see wave_rank), so equal digits keep the input order. Tile offsets
// come from per-tile histograms scanned on the device, digit-major, so pass outputs are
// the same for every launch.
#include "gee_internal.h"

namespace gee {

constexpr int kTile = kPartTile;  // entries per partition tile
constexpr int kRounds = kTile / 256;
#ifndef GEE_PART_WAVES
#define GEE_PART_WAVES 4
#endif
constexpr int kWaves = GEE_PART_WAVES;    // wavefronts per partition workgroup
constexpr int kThreads = kWaves * 64;
constexpr int kQuarter = kTile / kWaves;  // items per wavefront per tile
constexpr int kRoundsW = kQuarter / 64;   // rounds of one wavefront
#ifndef GEE_QUARTER_BUF
#define GEE_QUARTER_BUF 1
#endif
#ifndef GEE_OUT_UNROLL
#define GEE_OUT_UNROLL 4
#endif
constexpr int kOutUnroll = GEE_OUT_UNROLL;  // staged items per thread in flight in a tile's write-out
static_assert(kTile % (kWaves * 64) == 0 && kRoundsW <= 16 && kThreads >= 256, "partition tile shape");
// bucket_sort's wave-split path: 4 wavefronts of at most 16 rounds (kSortCap entries)
constexpr int kSortWaves = 4, kSortRoundsW = 16, kSortCap = kSortWaves * kSortRoundsW * 64;

// ----------------------------------------------------------------------------- helpers

// Stable rank of this thread's item among the items with the same digit in the tile
// processed so far by this 256-thread workgroup. `run[d]` holds the running base of
// digit d; `tab` is a zeroed u8[4][ndig] scratch. All threads must call it together.
__device__ __forceinline__ int block_rank4(int digit, bool valid, int nbits, unsigned char *tab,
                                           int *run, int ndig) {
    const int wv = threadIdx.x >> 6;
    uint64_t peers = ballot(valid);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (digit >> b) & 1;
        const uint64_t m = ballot(valid && bit);
        peers &= bit ? m : ~m;
    }
    const int below = count_below(peers);
    const int cnt = __popcll(peers);
    const bool leader = valid && (below == cnt - 1);
    if (leader) tab[wv * ndig + digit] = (unsigned char)cnt;
    __syncthreads();
    int r = 0;
    if (valid) {
        r = run[digit] + below;
        for (int w2 = 0; w2 < wv; ++w2) r += tab[w2 * ndig + digit];
    }
    __syncthreads();
    if (leader) {
        tab[wv * ndig + digit] = 0;
        atomicAdd(&run[digit], cnt);
    }
    return r;
}

// Exclusive scan of one int per thread over a 256-thread workgroup.
__device__ __forceinline__ int block_excl_scan256(int v, int *wsum, int &total) {
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int base = 0;
    for (int i = 0; i < wv; ++i) base += wsum[i];
    total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return base + x - v;
}

// In-place exclusive scan of a[0..n) in LDS (n <= 4096), 256 threads; returns total.
__device__ int block_excl_scan_lds(int *a, int n, int *wsum) {
    const int per = (n + 255) / 256;
    const int lo = threadIdx.x * per;
    int s = 0;
    for (int i = 0; i < per; ++i)
        if (lo + i < n) s += a[lo + i];
    int total;
    int base = block_excl_scan256(s, wsum, total);
    for (int i = 0; i < per; ++i)
        if (lo + i < n) {
            int t = a[lo + i];
            a[lo + i] = base;
            base += t;
        }
    __syncthreads();
    return total;
}

// ----------------------------------------------------------------------------- pass A

// Virtual entry v of the batch: its graph, then (row, column[, weight]) with the graph's
// node offset added. Invalid: index out of range (sets badi), or the mirror of a
// self-loop under symmetrization. `gd`/`g` cache the graph of the previous call (g < 0:
// none); any v outside the cached graph's range looks its graph up again.
template <bool VAL>
__device__ __forceinline__ bool load_virtual(const Batch &b, int64_t v, int64_t V, int &g, GDesc &gd,
                                             int &key, int &cl, float &val, bool &badi, bool &badw) {
    if (v >= V) return false;
    if (g < 0 || v < gd.voff || v >= gd.voff + gd.Mcap) {  // not in the cached graph
        g = find_graph(b.voffs, b.G, v);
        gd = load_desc(b, g);
    }
    const int64_t lv = v - gd.voff;
    const bool sym = gd.flags & kSym;
    const int64_t e = sym ? (lv >> 1) : lv;
    const int side = sym ? (int)(lv & 1) : 0;
    const int s = gd.src[e], d = gd.dst[e];
    key = (side ? d : s) + gd.node_off;
    cl = (side ? s : d) + gd.node_off;
    if (VAL) {
        val = 1.0f;
        if (gd.w) {
            val = gd.w[e];
            if (side == 0 && validates(gd) && !isfinite(val)) badw = true;
        }
    }
    const bool inr = (unsigned)s < (unsigned)gd.N && (unsigned)d < (unsigned)gd.N;
    if (!inr && validates(gd)) badi = true;
    return inr && (side == 0 || s != d);
}

// A wavefront's quarter of a tile (kRoundsW rounds of 64 virtual entries), loaded into
// registers with every load issued before any is used. Entry r of this lane is virtual
// entry vw + 64 r + lane.
template <bool VAL>
struct Quarter {
    int key[kRoundsW], col[kRoundsW];
    float val[kRoundsW];
    unsigned valid;  // bit r: entry r is a real adjacency entry
};

// load_quarter for a quarter inside one graph whose edge arrays fit 32-bit buffer offsets
// (and, under symmetrization, whose virtual entries start at an even place of the launch):
// the same entries in the same order, read with buffer loads whose per-round part of the
// offset is the same for the whole wavefront (a scalar offset) and whose per-lane part is
// fixed, so the rounds cost no address arithmetic; entries at or past V are invalid (loads
// past the arrays' end return 0).
template <bool VAL>
__device__ __forceinline__ void load_quarter_buf(const GDesc &gd, int64_t vw, int64_t V, Quarter<VAL> &q, bool &badi,
                                                 bool &badw) {
    const int lane = lane_id();
    q.valid = 0;
    if (vw >= V) return;
    const bool sym = gd.flags & kSym;
    const bool chk = validates(gd);
    const int64_t lv0 = vw - gd.voff;  // (even: quarters start at multiples of kQuarter)
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(gd.src, gd.E * 4), rd = buffer_rsrc(gd.dst, gd.E * 4);
    const __amdgpu_buffer_rsrc_t rw = buffer_rsrc(gd.w, gd.w ? gd.E * 4 : 0);
    // entry lv0 + 64 r + lane is edge (lv0 + 64 r + lane) / 2 under symmetrization
    const uint32_t lo = (uint32_t)(sym ? (lane >> 1) : lane) * 4u;
    const int64_t e0 = sym ? (lv0 >> 1) : lv0;
    const int step = sym ? 32 : 64;
    int sv[kRoundsW], dv[kRoundsW];
    float wv[kRoundsW];
#pragma unroll
    for (int r = 0; r < kRoundsW; ++r) {
        const int so = __builtin_amdgcn_readfirstlane((int)((e0 + (int64_t)r * step) * 4));
        sv[r] = (int)__builtin_amdgcn_raw_buffer_load_b32(rs, lo, so, 0);
        dv[r] = (int)__builtin_amdgcn_raw_buffer_load_b32(rd, lo, so, 0);
        if (VAL) wv[r] = gd.w ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rw, lo, so, 0)) : 1.0f;
    }
#pragma unroll
    for (int r = 0; r < kRoundsW; ++r) {
        const int64_t v = vw + r * 64 + lane;
        const int side = sym ? (lane & 1) : 0;
        const bool inb = v < V;
        const bool inr = (unsigned)sv[r] < (unsigned)gd.N && (unsigned)dv[r] < (unsigned)gd.N;
        if (chk && inb && !inr) badi = true;
        if (VAL && chk && inb && gd.w && side == 0 && !isfinite(wv[r])) badw = true;
        q.key[r] = (side ? dv[r] : sv[r]) + gd.node_off;
        q.col[r] = (side ? sv[r] : dv[r]) + gd.node_off;
        if (VAL) q.val[r] = wv[r];
        q.valid |= (inb && inr && (side == 0 || sv[r] != dv[r])) ? (1u << r) : 0u;
    }
}

template <bool VAL>
__device__ __forceinline__ void load_quarter(const Batch &b, int64_t vw, int64_t V, Quarter<VAL> &q, bool &badi,
                                             bool &badw) {
    static_assert(kRoundsW <= 16, "Quarter holds at most 16 rounds");
    const int lane = lane_id();
    q.valid = 0;
    vw = uniform64(vw);  // (the wavefront's quarter: the graph search and descriptor loads are scalar)
    if (vw >= V) return;
    const int64_t vhi = min(vw + (int64_t)kQuarter, V) - 1;
    const int g0 = find_graph(b.voffs, b.G, vw), g1 = find_graph(b.voffs, b.G, vhi);
    if (g0 == g1) {
        const GDesc gd = load_desc(b, g0);
        if (GEE_QUARTER_BUF && gd.E * 4 <= (int64_t)INT32_MAX && (!(gd.flags & kSym) || ((vw - gd.voff) & 1) == 0)) {
            load_quarter_buf<VAL>(gd, vw, vhi + 1, q, badi, badw);
            return;
        }
        // one graph: clamped unconditional loads, then the checks
        const bool sym = gd.flags & kSym;
        const bool chk = validates(gd);
        int sv[kRoundsW], dv[kRoundsW];
        float wv[kRoundsW];
#pragma unroll
        for (int r = 0; r < kRoundsW; ++r) {
            const int64_t lv = min(vw + r * 64 + lane, vhi) - gd.voff;
            const int64_t e = sym ? (lv >> 1) : lv;
            sv[r] = gd.src[e];
            dv[r] = gd.dst[e];
            if (VAL) wv[r] = gd.w ? gd.w[e] : 1.0f;
        }
#pragma unroll
        for (int r = 0; r < kRoundsW; ++r) {
            const int64_t v = vw + r * 64 + lane;
            const int side = sym ? (int)((v - gd.voff) & 1) : 0;
            const bool inb = v <= vhi;
            const bool inr = (unsigned)sv[r] < (unsigned)gd.N && (unsigned)dv[r] < (unsigned)gd.N;
            if (chk && inb && !inr) badi = true;
            if (VAL && chk && inb && gd.w && side == 0 && !isfinite(wv[r])) badw = true;
            q.key[r] = (side ? dv[r] : sv[r]) + gd.node_off;
            q.col[r] = (side ? sv[r] : dv[r]) + gd.node_off;
            if (VAL) q.val[r] = wv[r];
            q.valid |= (inb && inr && (side == 0 || sv[r] != dv[r])) ? (1u << r) : 0u;
        }
    } else {
        // the quarter spans graphs (small graphs of a batch): entry by entry
        int g = -1;
        GDesc gd;
#pragma unroll
        for (int r = 0; r < kRoundsW; ++r) {
            float val = 1.0f;
            const bool ok = load_virtual<VAL>(b, vw + r * 64 + lane, V, g, gd, q.key[r], q.col[r], val, badi, badw);
            if (VAL) q.val[r] = val;
            q.valid |= ok ? (1u << r) : 0u;
        }
    }
}

// Per tile of virtual entries: histogram of the high digit (row >> shift), written
// digit-major; index checks.
// The first gridDim.x - T workgroups are label slices of the class counts (first, so that
// their longer loops overlap the tiles instead of ending the launch).
// With vec (one graph whose src and dst are 16-byte aligned and fit 32-bit buffer offsets)
// each thread reads 4 edges per 16-byte load instead of one virtual entry per lane: the
// tile's edges are the same (virtual entries 2e and 2e+1 are edge e under symmetrization),
// so are its counts.
#ifndef GEE_AHIST_EDGES
#define GEE_AHIST_EDGES 1
#endif
static_assert(kTile % (kThreads * 8) == 0 && kTile / kThreads <= 16, "a_hist: whole 16-byte loads of edges per thread");
// The tile histograms (a_hist, seg_hist) count into kHistCopies interleaved copies of each
// digit's counter (word digit * kHistCopies + lane mod kHistCopies), summed at the end: lanes
// of one instruction that hit the same digit then mostly hit different words, which the LDS
// serves in one pass instead of one lane after another.
#ifndef GEE_HIST_COPIES
#define GEE_HIST_COPIES 4
#endif
constexpr int kHistCopies = GEE_HIST_COPIES;
static_assert(kHistCopies >= 1 && kHistCopies <= 16 && (kHistCopies & (kHistCopies - 1)) == 0, "histogram copies");
__device__ __forceinline__ int hist_sum(const int *hist, int d) {
    int s = 0;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) s += hist[d * kHistCopies + c];
    return s;
}
__global__ __launch_bounds__(kThreads) void a_hist(Batch b, int64_t V, int shift, int D, int64_t T,
                                                   int *__restrict__ gh, unsigned *status, int *__restrict__ cpart,
                                                   int vec) {
    __shared__ int hist_all[256 * kHistCopies];
    const int64_t nslices = (int64_t)gridDim.x - T;
    if ((int64_t)blockIdx.x < nslices) {
        class_count_slice(b, (int)blockIdx.x, cpart, status, hist_all);
        return;
    }
    for (int i = threadIdx.x; i < 256 * kHistCopies; i += kThreads) hist_all[i] = 0;
    __syncthreads();
    int *hist = hist_all + (threadIdx.x & (kHistCopies - 1));  // digit d at hist[d * kHistCopies]
    const int64_t t = xcd_order((int64_t)blockIdx.x - nslices, T);
    bool badi = false;
    if (GEE_AHIST_EDGES && vec) {
        const GDesc &gd = b.one;
        const bool sym = gd.flags & kSym;
        const bool chk = validates(gd);
        const unsigned N = (unsigned)gd.N;
        const int per = sym ? kTile / kThreads / 2 : kTile / kThreads;  // edges per thread (8 or 16)
        const int64_t e0 = t * (sym ? kTile / 2 : kTile) + (int64_t)threadIdx.x * per;
        const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(gd.src, gd.E * 4), rd = buffer_rsrc(gd.dst, gd.E * 4);
        int4 sv[4], dv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (4 * k < per) {
                sv[k] = buf_i4(rs, (uint32_t)((e0 + 4 * k) * 4));
                dv[k] = buf_i4(rd, (uint32_t)((e0 + 4 * k) * 4));
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (4 * k >= per) break;
            const int ss[4] = {sv[k].x, sv[k].y, sv[k].z, sv[k].w};
            const int dd[4] = {dv[k].x, dv[k].y, dv[k].z, dv[k].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (e0 + 4 * k + j >= gd.E) continue;
                const bool inr = (unsigned)ss[j] < N && (unsigned)dd[j] < N;
                if (!inr) {
                    badi |= chk;
                    continue;
                }
                atomicAdd(&hist[((ss[j] + gd.node_off) >> shift) * kHistCopies], 1);
                if (sym && ss[j] != dd[j]) atomicAdd(&hist[((dd[j] + gd.node_off) >> shift) * kHistCopies], 1);
            }
        }
    } else {
        const int wv = threadIdx.x >> 6;
        bool badw = false;
        Quarter<false> q;
        load_quarter<false>(b, t * kTile + (int64_t)wv * kQuarter, V, q, badi, badw);
#pragma unroll
        for (int r = 0; r < kRoundsW; ++r)
            if (q.valid >> r & 1u) atomicAdd(&hist[(q.key[r] >> shift) * kHistCopies], 1);
    }
    if (__syncthreads_or(badi) && threadIdx.x == 0) raise_error(status, kErrIndex);
    if (threadIdx.x < D) gh[(int64_t)threadIdx.x * T + t] = hist_sum(hist_all, threadIdx.x);
}

// One workgroup per digit d: exclusive scan of the row gh[d*T .. d*T+T) in place;
// tot[d] = its sum.
// Workgroups past the D digits take 16 classes of the class totals each.
__global__ __launch_bounds__(1024) void digit_scan(int *__restrict__ gh, int64_t T, int *__restrict__ tot, int D,
                                                   Batch b, int Ktot, const int *__restrict__ cpart,
                                                   int *__restrict__ counts, float *__restrict__ inv_n) {
    if ((int)blockIdx.x >= D) {
        const int c = ((int)blockIdx.x - D) * 16 + (int)(threadIdx.x >> 6);
        if (c < Ktot) class_count_total(b, c, cpart, counts, inv_n);
        return;
    }
    __shared__ int wsum[16];
    int *row = gh + (int64_t)blockIdx.x * T;
    int carry = 0;
    constexpr int IPT = 8;
    for (int64_t c = 0; c < T; c += 1024 * IPT) {
        int vals[IPT];
        int s = 0;
        const int64_t lo = c + (int64_t)threadIdx.x * IPT;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            vals[i] = (lo + i < T) ? row[lo + i] : 0;
            s += vals[i];
        }
        int total;
        int base = block_excl_scan<1024>(s, wsum, total) + carry;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if (lo + i < T) row[lo + i] = base;
            base += vals[i];
        }
        carry += total;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// ----------------------------------------------------------------------------- wave-split ranking
//
// A tile is sorted by digit in LDS without a workgroup barrier per round: each of the 4
// wavefronts owns a contiguous quarter of the tile. The wavefronts first count their
// items per digit (LDS atomics on their own row of counters), one scan over
// (digit, wavefront) turns the counts into the first position of every (wavefront,
// digit) pair, then each wavefront ranks its items in round and lane order against the
// per-digit running positions of its row (wave_rank).


template <typename KS>
struct PartLds {
    int cnt[kWaves][256];  // per-wavefront digit counts, then running positions
    int gdelta[256], wsum[kWaves];  // gdelta[d]: global position of the tile's digit-d run minus its tile position
    KS key[kTile];            // the key as written out
    unsigned char dig[kTile]; // its digit (at most 256 digits)
    int col[kTile];
    float val[kTile];
    // kRankMask ranking: each wavefront's 256 peer masks, in the column staging area (not
    // in use until the ranks are known)
    __device__ __forceinline__ unsigned long long *masks(int wv) {
        return reinterpret_cast<unsigned long long *>(col) + wv * 256;
    }
    __device__ __forceinline__ void zero_masks() {
        for (int i = threadIdx.x; i < kWaves * 256; i += blockDim.x) masks(0)[i] = 0ull;
    }
};
static_assert(kTile * sizeof(int) >= kWaves * 256 * sizeof(unsigned long long), "peer masks fit the column staging");
static_assert(offsetof(PartLds<uint16_t>, col) % 8 == 0 && offsetof(PartLds<int>, col) % 8 == 0,
              "peer masks are 8-byte aligned");

// Thread d: the offset from a tile position of digit d to its global position (gdelta =
// the run's global base minus the tile's first position of d), and the first position of
// every wavefront's run of digit d (in cnt). Returns the tile's item count.
__device__ __forceinline__ int wave_split_layout(int (*cnt)[256], int *gdelta, int *wsum, int D, int gbase_d) {
    const int d = threadIdx.x;
    int c[kWaves], csum = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        c[w] = d < D ? cnt[w][d] : 0;
        csum += c[w];
    }
    int total;
    const int ls = block_excl_scan<kThreads>(csum, wsum, total);
    if (d < D) {
        gdelta[d] = gbase_d - ls;
        int run = ls;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            cnt[w][d] = run;
            run += c[w];
        }
    }
    __syncthreads();
    return total;
}

// Stable position of this lane's item among the wavefront's items of the same digit (in
// round and lane order), from the digit's running position in LDS. One LDS atomic add
// with return per item: the LDS serves the lanes of one instruction that hit the same
// word in ascending lane order (measured on gfx950, and the CSR parity tests compare the
// result bit for bit with a stable sort), and the instructions of one wavefront in
// program order.
__device__ __forceinline__ int wave_rank(int *run, int digit, bool valid) {
    return valid ? atomicAdd(&run[digit], 1) : 0;
}

// Positions of a wavefront's R rounds of items (round r: digit[r], valid bit r), in round
// and lane order. Without bal, wave_rank per item. With bal, the same stable positions
// without relying on the order in which the LDS serves the lanes of one atomic instruction
// that hit one word: the lanes of a round with the same digit find each other (their peer
// mask); the last of them alone adds their count to the digit's running position (so no
// two lanes of an instruction touch one word), and each peer takes the returned base, read
// from that lane, plus the number of peers below it. The LDS operations of one wavefront
// take effect in program order, so each round sees the additions of the rounds before it;
// all rounds' adds are issued before any base is read, so no round waits for the previous
// one's LDS round trip. Peer masks: with bal = 1 by ballots over the digit's nbits bits;
// with bal = 2 (kRankMask) each lane sets its bit in its digit's 64-bit word of `mask` with
// an LDS atomic OR (the result does not depend on the order in which the lanes are
// served), reads the word back and clears it — three LDS operations per round instead of
// one ballot per digit bit (the wavefront's words must be zero on entry and are zero again
// on return). The CSR build (its bit-exact contract) ranks with kRankMask; the bucket
// path, whose entry order only sets the floating-point summation order, takes wave_rank,
// which is faster still.
constexpr int kRankMask = 2;
#ifndef GEE_CSR_RANK_BALLOT
#define GEE_CSR_RANK_BALLOT kRankMask
#endif
#ifndef GEE_BUCKET_RANK
#define GEE_BUCKET_RANK 0
#endif
template <int R>
__device__ __forceinline__ void wave_ranks(int *run, const int (&digit)[R], unsigned valid, int nbits, int bal,
                                           int (&pos)[R], unsigned long long *mask = nullptr) {
    if (!bal) {
#pragma unroll
        for (int r = 0; r < R; ++r) pos[r] = wave_rank(run, digit[r], valid >> r & 1u);
        return;
    }
    int below[R], last[R], b0[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool v = valid >> r & 1u;
        uint64_t peers;
        if (bal == kRankMask) {
            unsigned long long *w = mask + digit[r];
            if (v) __hip_atomic_fetch_or(w, 1ull << lane_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            peers = v ? __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) : 0ull;
            if (v) __hip_atomic_store(w, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        } else {
            peers = ballot(v);
            for (int b = 0; b < nbits; ++b) {
                const bool bit = (digit[r] >> b) & 1;
                const uint64_t m = ballot(v && bit);
                peers &= bit ? m : ~m;
            }
        }
        below[r] = count_below(peers);
        const int cnt = __popcll(peers);
        last[r] = v ? 63 - __clzll(peers) : lane_id();
        b0[r] = 0;
        if (v && below[r] == cnt - 1) b0[r] = atomicAdd(&run[digit[r]], cnt);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) pos[r] = __shfl(b0[r], last[r], 64) + below[r];
}

// Tiles whose items share few digits (entries of one small graph of a batch) would serialize
// LDS atomics on a few words, one lane after another. When the
// digits of a wavefront's R rounds span at most 2^kNarrowBits values, the lanes of each round
// with the same digit find each other by one ballot per bit of the digit's offset from the
// smallest, and one lane per group adds the group's count: the same stable positions (the
// groups' adds in round order), from a few ballots and at most one LDS atomic per digit and
// round. Per round, packed: peers below the lane (bits 0-6), group size (7-13), the group's
// last lane (14-19).
#ifndef GEE_RANK_NARROW
#define GEE_RANK_NARROW 1
#endif
#ifndef GEE_NARROW_BITS
#define GEE_NARROW_BITS 2
#endif
constexpr int kNarrowBits = GEE_NARROW_BITS;
// Minimum / maximum over the wavefront by the DPP moves of wave_scan_add (lane 63 of the
// inclusive scan), the same value on every lane.
__device__ __forceinline__ int wave_min_i(int x) {
    x = min(x, dpp_i<0x111>(x, INT_MAX));
    x = min(x, dpp_i<0x112>(x, INT_MAX));
    x = min(x, dpp_i<0x114>(x, INT_MAX));
    x = min(x, dpp_i<0x118>(x, INT_MAX));
    x = min(x, dpp_i<0x142, 0xA>(x, INT_MAX));
    x = min(x, dpp_i<0x143, 0xC>(x, INT_MAX));
    return readlane(x, 63);
}
__device__ __forceinline__ int wave_max_i(int x) {
    x = max(x, dpp_i<0x111>(x, INT_MIN));
    x = max(x, dpp_i<0x112>(x, INT_MIN));
    x = max(x, dpp_i<0x114>(x, INT_MIN));
    x = max(x, dpp_i<0x118>(x, INT_MIN));
    x = max(x, dpp_i<0x142, 0xA>(x, INT_MIN));
    x = max(x, dpp_i<0x143, 0xC>(x, INT_MIN));
    return readlane(x, 63);
}
// The smallest digit (lo) and the bits of the span (nb) of the valid items of a wavefront's
// R rounds; false when the span needs more than kNarrowBits bits.
template <int R>
__device__ __forceinline__ bool narrow_span(const int (&key)[R], int shift, unsigned valid, int &lo, int &nb) {
    int a = INT_MAX, z = -1;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (valid >> r & 1u) {
            a = min(a, key[r] >> shift);
            z = max(z, key[r] >> shift);
        }
    lo = wave_min_i(a);
    z = wave_max_i(z);
    const int span = z >= lo ? z - lo : 0;
    nb = span == 0 ? 0 : 32 - __clz(span);
    return nb <= kNarrowBits;
}
// One round's peers (lanes with the same digit) by nb ballots over the digit's offset from lo,
// packed as below.
__device__ __forceinline__ int narrow_round(int digit, bool v, int lo, int nb) {
    uint64_t peers = ballot(v);
    const int off = digit - lo;
    for (int b = 0; b < nb; ++b) {
        const bool bit = (off >> b) & 1;
        const uint64_t m = ballot(v && bit);
        peers &= bit ? m : ~m;
    }
    const int last = v ? 63 - __clzll(peers) : lane_id();
    return count_below(peers) | (__popcll(peers) << 7) | (last << 14);
}
__device__ __forceinline__ int pk_below(int p) { return p & 0x7F; }
__device__ __forceinline__ int pk_count(int p) { return (p >> 7) & 0x7F; }
__device__ __forceinline__ int pk_last(int p) { return p >> 14; }

// Pass A scatter: tile t of the virtual entries, sorted by high digit in LDS (wave-split
// ranking over the wavefront's registers) and written to seg_start[d] + (scanned tile
// offset) in runs. The key written keeps only the bits the later passes read (amask): the
// high digit is implied by the segment, so with at most 16 bits left it fits a u16.
template <typename AK>
__global__ __launch_bounds__(kThreads) void a_scatter(Batch b, int64_t V, int shift, int D, int nbits, int64_t T,
                                                      const int *__restrict__ gh, const int *__restrict__ tot,
                                                      AK *__restrict__ okey, int amask, int *__restrict__ ocol,
                                                      float *__restrict__ oval, unsigned *status, int with_b, int B,
                                                      int *__restrict__ seg_start, int *__restrict__ tile_off,
                                                      int *__restrict__ bstart, int *__restrict__ meta, int bal,
                                                      int *__restrict__ ptot, int *__restrict__ tile_seg,
                                                      int qbuf) {
    __shared__ PartLds<AK> L;
    const int wv = threadIdx.x >> 6;
    const int64_t t = xcd_order(blockIdx.x, T);
    // the digit totals and this tile's scanned offsets, loaded before the entries (they do
    // not depend on them)
    const int dn = (int)threadIdx.x < D ? tot[threadIdx.x] : 0;
    const int gtile = (int)threadIdx.x < D ? gh[(int64_t)threadIdx.x * T + t] : 0;
    bool badi = false, badw = false;
    Quarter<true> q;
    if (qbuf) load_quarter_buf<true>(b.one, t * kTile + (int64_t)wv * kQuarter, V, q, badi, badw);
    else load_quarter<true>(b, t * kTile + (int64_t)wv * kQuarter, V, q, badi, badw);
    for (int i = threadIdx.x; i < kWaves * 256; i += blockDim.x) (&L.cnt[0][0])[i] = 0;
    if (bal == kRankMask) L.zero_masks();
    int nlo = 0, nnb = 0;
    // (launches of several graphs only: a single graph's tiles spread their rows over the
    // graph's digits, where the per-item LDS atomics were measured faster)
    const bool narrow = GEE_RANK_NARROW && b.G > 1 && narrow_span<kRoundsW>(q.key, shift, q.valid, nlo, nnb);
    __syncthreads();
    if (narrow) {
#pragma unroll
        for (int r = 0; r < kRoundsW; ++r) {
            const bool v = q.valid >> r & 1u;
            const int pk = narrow_round(q.key[r] >> shift, v, nlo, nnb);
            if (v && pk_below(pk) == pk_count(pk) - 1) atomicAdd(&L.cnt[wv][q.key[r] >> shift], pk_count(pk));
        }
    } else {
#pragma unroll
        for (int r = 0; r < kRoundsW; ++r)
            if (q.valid >> r & 1u) atomicAdd(&L.cnt[wv][q.key[r] >> shift], 1);
    }
    __syncthreads();
    // segment starts: exclusive scan of the digit totals, in every workgroup (workgroup 0
    // also writes them, the entry count M, the pass-B tiles of every segment and, without
    // a pass B, the bucket starts, for the later launches)
    int total;
    const int st = block_excl_scan<kThreads>(dn, L.wsum, total);
    if (blockIdx.x == 0) {
        int ttot;
        const int to = block_excl_scan<kThreads>(with_b ? (dn + kTile - 1) / kTile : 0, L.wsum, ttot);
        const int d = threadIdx.x;
        if (d < D) {
            seg_start[d] = st;
            if (with_b) tile_off[d] = to;
            if (!with_b && d < B) bstart[d] = st;
            if (with_b && tile_seg)
                for (int j = 0, nt = (dn + kTile - 1) / kTile; j < nt; ++j) tile_seg[to + j] = d;
        }
        if (d == 0) {
            seg_start[D] = total;
            if (with_b) tile_off[D] = ttot;
            bstart[B] = total;
            meta[0] = total;
        }
        if (ptot) ptot[d] = 0;  // 64 blocks x 4 totals, formed by the pass-B scan
    }
    const int gb = (int)threadIdx.x < D ? st + gtile : 0;
    const int n = wave_split_layout(L.cnt, L.gdelta, L.wsum, D, gb);
    int dg[kRoundsW], pos[kRoundsW];
#pragma unroll
    for (int r = 0; r < kRoundsW; ++r) dg[r] = (q.valid >> r & 1u) ? (q.key[r] >> shift) : 0;
    if (narrow) {
        // (each round's base is read right after its add: issuing all adds first would need
        // the peers formed twice, which measured slower)
#pragma unroll
        for (int r = 0; r < kRoundsW; ++r) {
            const bool v = q.valid >> r & 1u;
            const int pk = narrow_round(dg[r], v, nlo, nnb);
            int b0 = 0;
            if (v && pk_below(pk) == pk_count(pk) - 1) b0 = atomicAdd(&L.cnt[wv][dg[r]], pk_count(pk));
            pos[r] = __shfl(b0, pk_last(pk), 64) + pk_below(pk);
        }
    } else {
        wave_ranks<kRoundsW>(L.cnt[wv], dg, q.valid, nbits, bal, pos, L.masks(wv));
    }
    if (bal == kRankMask) __syncthreads();  // (the masks share the staging area)
#pragma unroll
    for (int r = 0; r < kRoundsW; ++r) {
        if ((q.valid >> r & 1u) && dbg_ok(pos[r] >= 0 && pos[r] < kTile, status)) {
            L.key[pos[r]] = (AK)(q.key[r] & amask);
            L.dig[pos[r]] = (unsigned char)dg[r];
            L.col[pos[r]] = q.col[r];
            if (oval) L.val[pos[r]] = q.val[r];
        }
    }
    if (__syncthreads_or(badw) && threadIdx.x == 0) raise_error(status, kErrWeight);
    // kOutUnroll items per thread at a time, so their LDS reads overlap
    for (int i0 = threadIdx.x; i0 < n; i0 += kOutUnroll * kThreads) {
        int dd[kOutUnroll];
#pragma unroll
        for (int u = 0; u < kOutUnroll; ++u) dd[u] = L.dig[min(i0 + u * kThreads, n - 1)];
#pragma unroll
        for (int u = 0; u < kOutUnroll; ++u) {
            const int i = i0 + u * kThreads;
            if (i >= n) break;
            const int64_t g2 = (int64_t)L.gdelta[dd[u]] + i;
            if (!dbg_ok(g2 >= 0 && g2 < V, status)) continue;
            okey[g2] = L.key[i];
            ocol[g2] = L.col[i];
            if (oval) oval[g2] = L.val[i];
        }
    }
}

// ----------------------------------------------------------------------------- pass B

// Pass-B tile j -> (segment d, tile within segment); returns false past the last tile.
// With tile_seg (pass B: the segment of every tile, written by the pass-A scatter) one
// lookup, else a binary search over the segments' first tiles (pass C).
__device__ __forceinline__ bool b_tile(const int *__restrict__ tile_off, const int *__restrict__ tile_seg, int D,
                                       int j, int &d, int &jt, int &ntd) {
    if (tile_seg) {
        const int tb = tile_off[D], dj = tile_seg[j];  // (j < the grid's tile capacity: in bounds)
        if (j >= tb) return false;
        d = dj;
    } else {
        if (j >= tile_off[D]) return false;
        int lo = 0, hi = D;  // last d with tile_off[d] <= j
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tile_off[mid] <= j) lo = mid;
            else hi = mid;
        }
        d = lo;
    }
    jt = j - tile_off[d];
    ntd = tile_off[d + 1] - tile_off[d];
    return true;
}

// Segment partitions (pass B, and pass C for buckets too large for one workgroup): the
// items of segment d (seg_start[d] .. seg_start[d+1]) are split into tiles of kTile;
// tile_off[d] is the segment's first tile. The digit of a key is
// (key >> dshift) & (2^dbits - 1).

// Per tile: digit histogram; segment d's counts are stored tile-major at
// gh + tile_off[d] * 2^dbits, [tile][digit], so each tile writes (and later reads) one
// contiguous row.
template <typename KT>
__global__ __launch_bounds__(256) void seg_hist(const KT *__restrict__ key, int dshift, int dbits,
                                                const int *__restrict__ seg_start, const int *__restrict__ tile_off,
                                                int D, int *__restrict__ gh, const int *__restrict__ tile_seg) {
    __shared__ int hist_all[256 * kHistCopies];
    int d, jt, ntd;
    if (!b_tile(tile_off, tile_seg, D, blockIdx.x, d, jt, ntd)) return;
    const int L = 1 << dbits;
    for (int i = threadIdx.x; i < 256 * kHistCopies; i += 256) hist_all[i] = 0;
    __syncthreads();
    int *hist = hist_all + (threadIdx.x & (kHistCopies - 1));
    const int e0 = seg_start[d] + jt * kTile;
    const int e1 = min(e0 + kTile, seg_start[d + 1]);
    int k[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) k[r] = (int)key[min(e0 + r * 256 + (int)threadIdx.x, e1 - 1)];
#pragma unroll
    for (int r = 0; r < kRounds; ++r)
        if (e0 + r * 256 + (int)threadIdx.x < e1) atomicAdd(&hist[((k[r] >> dshift) & (L - 1)) * kHistCopies], 1);
    __syncthreads();
    if ((int)threadIdx.x < L) gh[(((int64_t)tile_off[d] + jt) << dbits) + threadIdx.x] = hist_sum(hist_all, threadIdx.x);
}

// One workgroup per segment d: every (tile, digit) count becomes the position of that
// run inside the segment (digits in order, and within a digit the tiles in order), and
// starts[(d << dbits) + digit] = the first position of each digit (for indices below
// `limit`). A thread per digit walks the tile rows (coalesced across the digits); four
// groups of threads take a quarter of the tiles each. With skip_untiled, segments
// without tiles are left alone (pass C: those buckets are sorted whole by bucket_sort).
//
// With ptot (pass B of the bucket path), the segment's buckets (2^dbits of them, inside one
// block of 1024 buckets) also add their part-table totals to that block's four counters
// (parts, partial slots, split buckets, large one-part buckets; integer atomics, so the sums
// do not depend on the order); ptot was cleared by the pass-A scatter.
__global__ __launch_bounds__(1024) void seg_scan(int *__restrict__ gh, int dbits, const int *__restrict__ seg_start,
                                                 const int *__restrict__ tile_off, int limit,
                                                 int *__restrict__ starts, int skip_untiled, Batch b, int sb,
                                                 int *__restrict__ ptot) {
    __shared__ int part[4][256];
    __shared__ int dstart[256];
    __shared__ int wsum[16];
    const int d = blockIdx.x;
    const int ntd = tile_off[d + 1] - tile_off[d];
    if (skip_untiled && ntd == 0) return;
    const int L = 1 << dbits;
    int *seg = gh + ((int64_t)tile_off[d] << dbits);  // [ntd][L]
    const int dig = threadIdx.x & 255, grp = threadIdx.x >> 8;
    const int per = (ntd + 3) >> 2;
    const int t0 = min(ntd, grp * per), t1 = min(ntd, t0 + per);
    int tot = 0;
    if (dig < L) {
        int t = t0;
        for (; t + 4 <= t1; t += 4) {
            const int a0 = seg[((int64_t)t << dbits) + dig], a1 = seg[((int64_t)(t + 1) << dbits) + dig];
            const int a2 = seg[((int64_t)(t + 2) << dbits) + dig], a3 = seg[((int64_t)(t + 3) << dbits) + dig];
            tot += a0 + a1 + a2 + a3;
        }
        for (; t < t1; ++t) tot += seg[((int64_t)t << dbits) + dig];
    }
    part[grp][dig] = tot;
    __syncthreads();
    const int dsum = (threadIdx.x < 256) ? part[0][dig] + part[1][dig] + part[2][dig] + part[3][dig] : 0;
    int total;
    const int ds = block_excl_scan<1024>(dsum, wsum, total);
    if (threadIdx.x < 256) dstart[dig] = ds;
    __syncthreads();
    if (dig < L) {
        int run = dstart[dig];
        for (int g = 0; g < grp; ++g) run += part[g][dig];
        int t = t0;
        for (; t + 4 <= t1; t += 4) {
            int *q0 = seg + ((int64_t)t << dbits) + dig;
            const int a0 = q0[0], a1 = q0[L], a2 = q0[2 * L], a3 = q0[3 * L];
            q0[0] = run;
            q0[L] = run + a0;
            q0[2 * L] = run + a0 + a1;
            q0[3 * L] = run + a0 + a1 + a2;
            run += a0 + a1 + a2 + a3;
        }
        for (; t < t1; ++t) {
            int *q0 = seg + ((int64_t)t << dbits) + dig;
            const int a0 = q0[0];
            q0[0] = run;
            run += a0;
        }
    }
    const int s0 = seg_start[d];
    if ((int)threadIdx.x < L) {
        const int64_t bk = ((int64_t)d << dbits) + threadIdx.x;
        if (bk < limit) starts[bk] = s0 + dstart[threadIdx.x];
    }
    if (ptot && threadIdx.x < 256) {
        const int bk = (d << dbits) + dig;
        int k = 0, n = 0, P = 1;
        if (dig < L && bk < limit) {
            n = dsum;
            P = load_desc(b, find_graph(b.node_offs, b.G, bk << sb)).WE;
            k = parts_of(n, P);
        }
        const int v0 = readlane(wave_scan_add(k), 63), v1 = readlane(wave_scan_add(k > 1 ? k : 0), 63);
        const int v2 = readlane(wave_scan_add(k > 1 ? 1 : 0), 63);
        const int v3 = readlane(wave_scan_add(large_single(n, k, P) ? 1 : 0), 63);
        if (lane_id() == 0 && (v0 | v1 | v2 | v3)) {
            int *q = ptot + 4 * ((d << dbits) >> 10);
            atomicAdd(q, v0);
            atomicAdd(q + 1, v1);
            atomicAdd(q + 2, v2);
            atomicAdd(q + 3, v3);
        }
    }
}

// Per tile: sorted by digit in LDS (wave-split ranking over registers), written in runs.
// FINAL = false (pass B): key, column and value go to the next pass, the key reduced to
// the row inside its bucket (key & kmask) — for the bucket path (pack) packed into the
// column word above kBucketPackShift instead, with no key array (okey null). FINAL = true
// (pass C): column and value go to their CSR slots. With pf.nblk > 0 the first workgroups
// fill the bucket path's part table instead (part_fill_block).
template <typename KT, bool FINAL>
__global__ __launch_bounds__(kThreads) void seg_scatter(const KT *__restrict__ key, const int *__restrict__ col,
                                                   const float *__restrict__ val, int dshift, int dbits, int kmask,
                                                   const int *__restrict__ gh, const int *__restrict__ seg_start,
                                                   const int *__restrict__ tile_off, int D,
                                                   uint16_t *__restrict__ okey, int *__restrict__ ocol,
                                                   float *__restrict__ oval, unsigned *status, int bal,
                                                   const int *__restrict__ tile_seg, int pack, Batch b,
                                                   PartFill pf) {
    __shared__ PartLds<uint16_t> L;
    // the first pf.nblk workgroups fill the bucket path's part table (its inputs, the bucket
    // starts and the block totals, are complete once the pass-B scan has run)
    if ((int)blockIdx.x < pf.nblk) {
        part_fill_block(b, pf.bstart, pf.B, pf.sb, pf.ptot, pf.nblk, (int)blockIdx.x, pf.part, pf.multi, pf.bmeta);
        return;
    }
    const int jb = (int)blockIdx.x - pf.nblk;
    int d, jt, ntd;
    // (with the tile map, tiles are ordered over the grid's capacity, which spares a load)
    const int64_t jn = tile_seg ? (int64_t)gridDim.x - pf.nblk : (int64_t)tile_off[D];
    if (!b_tile(tile_off, tile_seg, D, (int)xcd_order(jb, jn), d, jt, ntd)) return;
    const int wv = threadIdx.x >> 6, lane = lane_id();
    const int ND = 1 << dbits;
    const int s0 = seg_start[d];
    const int nseg = seg_start[d + 1] - s0;
    const int *seg = gh + ((int64_t)tile_off[d] << dbits);
    // this tile's scanned run offsets, loaded before the entries (they do not depend on them)
    const int gtile = (int)threadIdx.x < ND ? seg[((int64_t)jt << dbits) + threadIdx.x] : 0;
    for (int i = threadIdx.x; i < kWaves * 256; i += blockDim.x) (&L.cnt[0][0])[i] = 0;
    if (bal == kRankMask) L.zero_masks();
    __syncthreads();
    const int e0 = s0 + jt * kTile;
    const int e1 = min(e0 + kTile, s0 + nseg);
    const int ew = e0 + wv * kQuarter;
    int kr[kRoundsW], cr[kRoundsW];
    float vr[kRoundsW];
#pragma unroll
    for (int r = 0; r < kRoundsW; ++r) {
        const int ec = min(ew + r * 64 + lane, e1 - 1);
        kr[r] = (int)key[ec];
        cr[r] = col[ec];
        vr[r] = oval ? val[ec] : 1.0f;
    }
#pragma unroll
    for (int r = 0; r < kRoundsW; ++r)
        if (ew + r * 64 + lane < e1) atomicAdd(&L.cnt[wv][(kr[r] >> dshift) & (ND - 1)], 1);
    __syncthreads();
    const int gb = (int)threadIdx.x < ND ? s0 + gtile : 0;
    const int n = wave_split_layout(L.cnt, L.gdelta, L.wsum, ND, gb);
    int dg[kRoundsW], pos[kRoundsW];
    unsigned vmask = 0;
#pragma unroll
    for (int r = 0; r < kRoundsW; ++r) {
        const bool valid = ew + r * 64 + lane < e1;
        vmask |= valid ? (1u << r) : 0u;
        dg[r] = valid ? ((kr[r] >> dshift) & (ND - 1)) : 0;
    }
    wave_ranks<kRoundsW>(L.cnt[wv], dg, vmask, dbits, bal, pos, L.masks(wv));
    if (bal == kRankMask) __syncthreads();  // (the masks share the staging area)
#pragma unroll
    for (int r = 0; r < kRoundsW; ++r) {
        if ((vmask >> r & 1u) && dbg_ok(pos[r] >= 0 && pos[r] < kTile, status)) {
            if (!FINAL && okey) L.key[pos[r]] = (uint16_t)(kr[r] & kmask);
            L.dig[pos[r]] = (unsigned char)dg[r];
            // (pack: the bucket path's kernels read the row from the column word)
            L.col[pos[r]] = pack ? (cr[r] | ((kr[r] & kmask) << kBucketPackShift)) : cr[r];
            if (oval) L.val[pos[r]] = vr[r];
        }
    }
    __syncthreads();
    for (int i0 = threadIdx.x; i0 < n; i0 += kOutUnroll * kThreads) {
        int dd[kOutUnroll];
#pragma unroll
        for (int u = 0; u < kOutUnroll; ++u) dd[u] = L.dig[min(i0 + u * kThreads, n - 1)];
#pragma unroll
        for (int u = 0; u < kOutUnroll; ++u) {
            const int i = i0 + u * kThreads;
            if (i >= n) break;
            const int64_t g = (int64_t)L.gdelta[dd[u]] + i;
            if (!dbg_ok(g >= s0 && g < (int64_t)s0 + nseg, status)) continue;
            if (!FINAL && okey) okey[g] = L.key[i];
            ocol[g] = L.col[i];
            if (oval) oval[g] = L.val[i];
        }
    }
}

// Single workgroup: pass-C tiles of every bucket (buckets above `cap` entries only).
__global__ __launch_bounds__(1024) void c_tiles(const int *__restrict__ bstart, int B, int cap,
                                                int *__restrict__ tile_off) {
    __shared__ int wsum[16];
    const int per = (B + 1023) / 1024;
    const int lo = threadIdx.x * per;
    int s = 0;
    for (int i = 0; i < per; ++i) {
        const int b = lo + i;
        if (b < B) {
            const int n = bstart[b + 1] - bstart[b];
            s += n > cap ? (n + kTile - 1) / kTile : 0;
        }
    }
    int total;
    int base = block_excl_scan<1024>(s, wsum, total);
    for (int i = 0; i < per; ++i) {
        const int b = lo + i;
        if (b < B) {
            tile_off[b] = base;
            const int n = bstart[b + 1] - bstart[b];
            base += n > cap ? (n + kTile - 1) / kTile : 0;
        }
    }
    if (threadIdx.x == 0) tile_off[B] = total;
}

// ----------------------------------------------------------------------------- pass C

// One workgroup per bucket b (rows [b << sb, (b+1) << sb)): row counts in LDS, their
// scan -> row_ptr, then a stable rank by row. A bucket of at most `cap` entries is
// staged in LDS and written out contiguously; a larger one (it holds long rows) is
// written at its ranks directly.
template <typename KT>
__global__ __launch_bounds__(256) void bucket_sort(const KT *__restrict__ tkey, const int *__restrict__ tcol,
                                                   const float *__restrict__ tval,
                                                   const int *__restrict__ bstart, int B, int sb, int N,
                                                   int *__restrict__ rp, int *__restrict__ col,
                                                   float *__restrict__ val, int cap, int pass_c, unsigned *status,
                                                   int bal) {
    extern __shared__ int smem_i[];
    __shared__ int wsum[4];
    const int R = 1 << sb;
    int *run = smem_i;                                                 // [R]
    unsigned char *tab = reinterpret_cast<unsigned char *>(run + R);  // [4][R]
    int *scol = reinterpret_cast<int *>(tab + 4 * R);                 // [cap]
    float *sval = reinterpret_cast<float *>(scol + cap);              // [cap]
    const int b = blockIdx.x;
    const int r0 = b << sb;
    const int Rb = min(R, N - r0);
    const int e0 = bstart[b], e1 = bstart[b + 1];
    const int rmask = R - 1;
    if (pass_c && e1 - e0 > cap) {  // sorted by the pass-C tiles
        if (b == B - 1 && threadIdx.x == 0) rp[N] = e1;
        return;
    }
    if (R <= 1024 && e1 - e0 <= cap) {
        // Wave-split ranking: each wavefront counts and ranks a contiguous quarter.
        const int wv = threadIdx.x >> 6, lane = lane_id();
        int *cnt = smem_i;                                              // [4][R]
        int *scol2 = cnt + kSortWaves * R;                              // [cap]
        float *sval2 = reinterpret_cast<float *>(scol2 + cap);          // [cap]
        // kRankMask ranking when the wavefronts' R peer masks fit the column staging area
        const int rbal = bal == kRankMask ? (8 * R <= cap ? kRankMask : 1) : bal;
        unsigned long long *masks = reinterpret_cast<unsigned long long *>(scol2);
        for (int i = threadIdx.x; i < kSortWaves * R; i += blockDim.x) cnt[i] = 0;
        if (rbal == kRankMask)
            for (int i = threadIdx.x; i < kSortWaves * R; i += blockDim.x) masks[i] = 0ull;
        __syncthreads();
        const int n = e1 - e0;
        // <= kSortCap / kSortWaves: kSortRoundsW rounds
        const int q = (((n + kSortWaves - 1) / kSortWaves) + 63) & ~63;
        const int ew = e0 + min(n, wv * q), ee = e0 + min(n, (wv + 1) * q);
        int kr[kSortRoundsW] = {0}, cr[kSortRoundsW] = {0};
        float vr[kSortRoundsW] = {0.0f};
        if (ee > ew) {  // this wavefront has entries: clamped loads stay inside [ew, ee)
#pragma unroll
            for (int r = 0; r < kSortRoundsW; ++r) {
                const int ec = min(ew + r * 64 + lane, ee - 1);
                kr[r] = (int)tkey[ec] & rmask;
                cr[r] = tcol[ec];
                vr[r] = val ? tval[ec] : 0.0f;
            }
        }
#pragma unroll
        for (int r = 0; r < kSortRoundsW; ++r)
            if (ew + r * 64 + lane < ee) atomicAdd(&cnt[wv * R + kr[r]], 1);
        __syncthreads();
        // thread t owns rows [t * rpt, (t + 1) * rpt): their counts, one scan, then each
        // (wavefront, row) pair's first position
        const int rpt = (R + 255) >> 8;  // at most 4
        const int rb0 = threadIdx.x * rpt;
        int csum = 0;
        for (int i = 0; i < rpt; ++i) {
            const int r = rb0 + i;
            if (r < R) csum += cnt[r] + cnt[R + r] + cnt[2 * R + r] + cnt[3 * R + r];
        }
        int total;
        int run2 = block_excl_scan256(csum, wsum, total);
        for (int i = 0; i < rpt; ++i) {
            const int r = rb0 + i;
            if (r >= R) break;
            if (r < Rb) rp[r0 + r] = e0 + run2;
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) {
                const int c = cnt[w * R + r];
                cnt[w * R + r] = run2;
                run2 += c;
            }
        }
        if (b == B - 1 && threadIdx.x == 0) rp[N] = e1;
        __syncthreads();
        int dg[kSortRoundsW], pos[kSortRoundsW];
        unsigned vmask = 0;
#pragma unroll
        for (int r = 0; r < kSortRoundsW; ++r) {
            const bool valid = ew + r * 64 + lane < ee;
            vmask |= valid ? (1u << r) : 0u;
            dg[r] = valid ? kr[r] : 0;
        }
        wave_ranks<kSortRoundsW>(cnt + wv * R, dg, vmask, sb, rbal, pos, masks + wv * R);
        if (rbal == kRankMask) __syncthreads();  // (the masks share the staging area)
#pragma unroll
        for (int r = 0; r < kSortRoundsW; ++r) {
            if ((vmask >> r & 1u) && dbg_ok(pos[r] >= 0 && pos[r] < n, status)) {
                scol2[pos[r]] = cr[r];
                if (val) sval2[pos[r]] = vr[r];
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            col[e0 + i] = scol2[i];
            if (val) val[e0 + i] = sval2[i];
        }
        return;
    }
    for (int i = threadIdx.x; i < R; i += blockDim.x) run[i] = 0;
    for (int i = threadIdx.x; i < 4 * R; i += blockDim.x) tab[i] = 0;
    __syncthreads();
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) atomicAdd(&run[(int)tkey[e] & rmask], 1);
    __syncthreads();
    block_excl_scan_lds(run, R, wsum);
    for (int i = threadIdx.x; i < Rb; i += blockDim.x) rp[r0 + i] = e0 + run[i];
    if (b == B - 1 && threadIdx.x == 0) rp[N] = e1;
    __syncthreads();
    const bool staged = e1 - e0 <= cap;
    for (int eb = e0; eb < e1; eb += 256) {
        const int e = eb + threadIdx.x;
        const bool valid = e < e1;
        const int ec = valid ? e : e0;
        const int digit = valid ? ((int)tkey[ec] & rmask) : 0;
        const int cl = tcol[ec];
        const float vv = val ? tval[ec] : 0.0f;
        const int pos = block_rank4(digit, valid, sb, tab, run, R);
        if (valid && dbg_ok(pos >= 0 && pos < e1 - e0, status)) {
            if (staged) {
                scol[pos] = cl;
                if (val) sval[pos] = vv;
            } else {
                col[e0 + pos] = cl;
                if (val) val[e0 + pos] = vv;
            }
        }
    }
    if (staged) {
        __syncthreads();
        for (int i = threadIdx.x; i < e1 - e0; i += blockDim.x) {
            col[e0 + i] = scol[i];
            if (val) val[e0 + i] = sval[i];
        }
    }
}

// ----------------------------------------------------------------------------- launch

// Staging capacity of bucket_sort: the whole workgroup stays within 64 KiB of LDS.
int bucket_stage_cap(int sb) { return sb >= 12 ? 2048 : (kTile < kSortCap ? kTile : kSortCap); }
size_t bucket_sort_lds(int sb) {
    const size_t R = (size_t)1 << sb;
    const size_t counters = R <= 1024 ? kSortWaves * R * 4 : 8 * R;  // wave-split path : block-rank path
    return (counters > 8 * R ? counters : 8 * R) + (size_t)bucket_stage_cap(sb) * 8;
}

hipError_t launch_csr_build(const Batch &b, const Plan &p, const Work &wk, unsigned *status, hipStream_t s,
                            const CountJob *job) {
    const unsigned xslices = job ? (unsigned)job->slices : 0u;
    const unsigned xclass = job ? (unsigned)((job->classes + 15) / 16) : 0u;
    const bool with_b = p.s2 > 0;
    const int shift = p.sb + p.s2;
    int nbits = 0;
    while ((1 << nbits) < p.DA) ++nbits;
    // pass A output: final col/val buffers as scratch when a pass B follows
    int *acol = with_b ? wk.col : wk.tcol;
    float *aval = p.weighted ? (with_b ? wk.val : wk.tval) : nullptr;
    hipError_t e;
    prof_begin(kKAHist, s);
    // one graph with 16-byte aligned src and dst: a_hist reads 4 edges per load
    const bool vec = b.tab == nullptr && ((reinterpret_cast<uintptr_t>(b.one.src) | reinterpret_cast<uintptr_t>(b.one.dst)) & 15) == 0 &&
                     b.one.E * 4 + 64 < (int64_t)0xFFFFFFFF;
    hipLaunchKernelGGL(a_hist, dim3((unsigned)p.TA + xslices), dim3(kThreads), 0, s, b, p.Vtot, shift, p.DA, p.TA,
                       wk.ghA, status, job ? job->part : nullptr, vec ? 1 : 0);
    prof_end(kKAHist, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKAScan, s);
    hipLaunchKernelGGL(digit_scan, dim3((unsigned)p.DA + xclass), dim3(1024), 0, s, wk.ghA, p.TA, wk.totA, p.DA, b,
                       job ? job->classes : 0, job ? job->part : nullptr, job ? job->counts : nullptr,
                       job ? job->inv_n : nullptr);
    prof_end(kKAScan, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // pass A keys: the row's low sb + s2 bits, as u16 when they fit
    const bool k16 = p.sb + p.s2 <= 16;
    // ranks: the CSR build keeps its bit-exact stable order without relying on the LDS's
    // lane order (wave_ranks with peer masks); the bucket path takes the faster wave_rank
    const int bal = p.bucket ? GEE_BUCKET_RANK : GEE_CSR_RANK_BALLOT;
    uint16_t *akey16 = reinterpret_cast<uint16_t *>(wk.akey);
    // the bucket path's part-table block totals, formed by the pass-B scan
    int *ptot = (p.bucket && with_b) ? wk.ptot : nullptr;
    // one graph whose edge arrays fit 32-bit offsets: buffer loads with scalar round offsets
    const int qbuf = (GEE_QUARTER_BUF && b.tab == nullptr && b.one.E * 4 + 256 < (int64_t)0x7FFFFFFF) ? 1 : 0;
    prof_begin(kKAScatter, s);
    const int wb = with_b ? 1 : 0;
    if (k16) {
        hipLaunchKernelGGL(a_scatter<uint16_t>, dim3((unsigned)p.TA), dim3(kThreads), 0, s, b, p.Vtot, shift, p.DA, nbits,
                           p.TA, wk.ghA, wk.totA, akey16, (1 << (p.sb + p.s2)) - 1, acol, aval, status, wb, p.B,
                           wk.segA, wk.tileB, wk.bstart, wk.meta, bal, ptot, wk.segB, qbuf);
    } else {
        hipLaunchKernelGGL(a_scatter<int>, dim3((unsigned)p.TA), dim3(kThreads), 0, s, b, p.Vtot, shift, p.DA, nbits,
                           p.TA, wk.ghA, wk.totA, wk.akey, -1, acol, aval, status, wb, p.B, wk.segA, wk.tileB,
                           wk.bstart, wk.meta, bal, ptot, wk.segB, qbuf);
    }
    prof_end(kKAScatter, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!with_b) return hipSuccess;
    prof_begin(kKBHist, s);
    if (k16) {
        hipLaunchKernelGGL(seg_hist<uint16_t>, dim3((unsigned)p.TBcap), dim3(256), 0, s, akey16, p.sb, p.s2,
                           wk.segA, wk.tileB, p.DA, wk.ghB, wk.segB);
    } else {
        hipLaunchKernelGGL(seg_hist<int>, dim3((unsigned)p.TBcap), dim3(256), 0, s, wk.akey, p.sb, p.s2, wk.segA,
                           wk.tileB, p.DA, wk.ghB, wk.segB);
    }
    prof_end(kKBHist, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKBScan, s);
    hipLaunchKernelGGL(seg_scan, dim3(p.DA), dim3(1024), 0, s, wk.ghB, p.s2, wk.segA, wk.tileB, p.B, wk.bstart, 0, b,
                       p.sb, ptot);
    prof_end(kKBScan, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKBScatter, s);
    // the bucket path reads its rows from the packed column words: no keys
    uint16_t *bkeys = (p.bucket && !GEE_PASSB_KEYS) ? nullptr : wk.tkey;
    // the bucket path's part table, in extra workgroups of this launch
    PartFill pf;
    if (p.bucket && wk.part && wk.ptot) {
        pf.bstart = wk.bstart;
        pf.ptot = wk.ptot;
        pf.part = wk.part;
        pf.multi = wk.multi;
        pf.bmeta = wk.bmeta;
        pf.B = (int)p.B;
        pf.sb = p.sb;
        pf.nblk = (int)((p.B + 1023) / 1024);
    }
    const unsigned gB = (unsigned)(p.TBcap + pf.nblk);
    if (k16) {
        hipLaunchKernelGGL((seg_scatter<uint16_t, false>), dim3(gB), dim3(kThreads), 0, s, akey16, acol, aval, p.sb, p.s2,
                           (1 << p.sb) - 1, wk.ghB, wk.segA, wk.tileB, p.DA, bkeys, wk.tcol,
                           p.weighted ? wk.tval : nullptr, status, bal, wk.segB, p.bucket ? 1 : 0, b, pf);
    } else {
        hipLaunchKernelGGL((seg_scatter<int, false>), dim3(gB), dim3(kThreads), 0, s, wk.akey, acol, aval, p.sb, p.s2,
                           (1 << p.sb) - 1, wk.ghB, wk.segA, wk.tileB, p.DA, bkeys, wk.tcol,
                           p.weighted ? wk.tval : nullptr, status, bal, wk.segB, p.bucket ? 1 : 0, b, pf);
    }
    prof_end(kKBScatter, s);
    return hipGetLastError();
}

// Pass C for buckets above the staging capacity (their hub rows would serialize one
// workgroup): the same segment partition with the row inside the bucket as the digit,
// straight into the CSR; then bucket_sort for all other buckets.
template <typename KT>
static hipError_t launch_pass_c(const KT *key, const Plan &p, const Work &wk, int cap, unsigned *status,
                                hipStream_t s) {
    const float *tv = p.weighted ? wk.tval : nullptr;
    float *ov = p.weighted ? wk.val : nullptr;
    prof_begin(kKCTiles, s);
    hipLaunchKernelGGL(c_tiles, dim3(1), dim3(1024), 0, s, wk.bstart, p.B, cap, wk.tileC);
    prof_end(kKCTiles, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    prof_begin(kKCHist, s);
    hipLaunchKernelGGL(seg_hist<KT>, dim3((unsigned)p.TCcap), dim3(256), 0, s, key, 0, p.sb, wk.bstart, wk.tileC,
                       p.B, wk.ghC, nullptr);
    prof_end(kKCHist, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKCScan, s);
    hipLaunchKernelGGL(seg_scan, dim3(p.B), dim3(1024), 0, s, wk.ghC, p.sb, wk.bstart, wk.tileC, (int)p.Ntot, wk.rp,
                       1, Batch{}, 0, nullptr);
    prof_end(kKCScan, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKCScatter, s);
    hipLaunchKernelGGL((seg_scatter<KT, true>), dim3((unsigned)p.TCcap), dim3(kThreads), 0, s, key, wk.tcol, tv, 0, p.sb,
                       0, wk.ghC, wk.bstart, wk.tileC, p.B, nullptr, wk.col, ov, status, GEE_CSR_RANK_BALLOT, nullptr, 0, Batch{},
                       PartFill{});
    prof_end(kKCScatter, s);
    return hipGetLastError();
}

hipError_t launch_csr_pass2(const Plan &p, const Work &wk, unsigned *status, hipStream_t s) {
    const size_t lds = bucket_sort_lds(p.sb);
    const int cap = bucket_stage_cap(p.sb);
    const float *tv = p.weighted ? wk.tval : nullptr;
    float *ov = p.weighted ? wk.val : nullptr;
    const int pass_c = p.sb <= 8 ? 1 : 0;  // pass C ranks rows as digits of at most 8 bits
    const bool k16 = p.sb + p.s2 <= 16;    // pass A wrote u16 keys (see launch_csr_build)
    const uint16_t *akey16 = reinterpret_cast<const uint16_t *>(wk.akey);
    hipError_t e = hipSuccess;
    if (pass_c) {
        e = (p.s2 > 0 || k16) ? launch_pass_c<uint16_t>(p.s2 > 0 ? wk.tkey : akey16, p, wk, cap, status, s)
                              : launch_pass_c<int>(wk.akey, p, wk, cap, status, s);
        if (e != hipSuccess) return e;
    }
    prof_begin(kKBucketSort, s);
    if (p.s2 > 0 || k16) {
        hipLaunchKernelGGL(bucket_sort<uint16_t>, dim3(p.B), dim3(256), lds, s, p.s2 > 0 ? wk.tkey : akey16, wk.tcol,
                           tv, wk.bstart, p.B, p.sb, (int)p.Ntot, wk.rp, wk.col, ov, cap, pass_c, status, GEE_CSR_RANK_BALLOT);
    } else {
        hipLaunchKernelGGL(bucket_sort<int>, dim3(p.B), dim3(256), lds, s, wk.akey, wk.tcol, tv, wk.bstart, p.B,
                           p.sb, (int)p.Ntot, wk.rp, wk.col, ov, cap, pass_c, status, GEE_CSR_RANK_BALLOT);
    }
    prof_end(kKBucketSort, s);
    return hipGetLastError();
}

}  // namespace gee
