// gee_bucket.hip - Z = A W straight from the row buckets of the CSR sort (Eq. 1, Table 1).
//
// The edge-list entry points need every row's sums, not the CSR itself. After the first
// two partition passes of the sort (gee_csr.hip) the entries of each bucket of R
// consecutive rows (R = 64; 32 when a graph of the launch has K > 64 and 32-row buckets
// hold the launch's rows) lie together, in input order; after a pass B each entry's row
// inside its bucket rides in its column word (above bit kPackShift), and no key array is
// written. A resident CSR's buckets are contiguous already: its rows come from row_ptr
// (CsrRows, csr_prep). Each bucket is cut into parts of at most P entries (P = the graph's
// wave_entries, at least kBucketMinPart), one wavefront per part:
//
//   * bucket_part_count / bucket_part_fill  the part table {bucket, entries, partial slot}
//                    and the list of buckets of several parts (two passes of prefix sums
//                    over the buckets; after a pass B the first runs in its scan and the
//                    second in extra workgroups of its scatter, part_fill_block).
//   * bucket_degree  (Laplacian) each part's weighted degrees (entry counts without weights)
//                    of the bucket's rows, summed in private LDS copies; a one-part bucket
//                    then sets s_i and c_i = s_i / n_{y_i} of its rows, a longer one leaves
//                    partial sums. Without the Laplacian, c_i = 1 / n_{y_i}.
//   * bucket_degree_fix  adds the partial degrees of split buckets in part order.
//   * bucket_embed   the class sums: the wavefront holds acc[R rows][class] in LDS and adds
//                    every entry's val * c_j into acc[row][y_j] (4 consecutive entries per
//                    lane, 16-byte loads, the loads of window k+2 and the gathers of window
//                    k+1 in flight while window k is added; most entries add without
//                    LDS float atomics, see the tag rule below). A one-part bucket then
//                    finishes its rows (diagonal term c_i, factor s_i or the 2-norm) and
//                    writes them as one contiguous block of Z; a longer one leaves its sums.
//   * bucket_embed_fix  adds the partial sums of split buckets in part order and finishes
//                    their rows.
//
// A wavefront adds its entries in a fixed order (windows in order; within a window the tag
// rule and the LDS's lane order for atomics on one word are fixed) and parts are combined
// in part order, so Z is bitwise reproducible. Buckets never straddle graphs (each graph's
// first row is aligned to R), and a graph's buckets and parts depend on that graph alone,
// so its Z is the same alone and in a batch with the same R. The diagonal term is added
// after the entries of its row.
#include <algorithm>

#include "gee_internal.h"

namespace gee {

constexpr int BEPL = 4;          // consecutive entries per lane in a window
constexpr int BWIN = 64 * BEPL;  // entries per window
// Threads per split bucket when combining class sums: 1024 (one pass over a bucket's sums)
// when the launch can hold few split buckets, 256 (four workgroups per CU more, four passes
// per bucket) when it can hold more than kFixManyBuckets, on grids of kFixGrid / kFixGridMany.
constexpr int kFixThreads = 1024;
constexpr int kFixThreadsMany = 256;
constexpr int kFixGrid = 1024, kFixGridMany = 8192;
constexpr int64_t kFixManyBuckets = 4096;
constexpr int kFixUnroll = 4;      // class sums per thread in flight together (R * K <= 4096)
// After a pass B on the bucket path each column word carries the entry's row inside its
// bucket above bit kPackShift (bucket-path launches hold at most 2^22 rows).
constexpr int kPackShift = kBucketPackShift;
static_assert(((int64_t)kMaxBuckets << 6) <= ((int64_t)1 << kPackShift), "packed bucket columns");
#ifndef GEE_EMBED_SCHED_BARRIER
#define GEE_EMBED_SCHED_BARRIER 1
#endif

// LDS of one class-sum workgroup: R rows of ring_stride(K) floats, 64 row factors and
// (bucket_embed) a 1 KB hash table of entry tags (lds_tag_add), which leaves room for more
// resident wavefronts than a tag per class sum.
constexpr int kTagBytes = 1024;
static size_t bucket_lds(int sb, int Kmax) {
    return ((size_t)ring_stride(Kmax) << sb) * sizeof(float) + 64 * sizeof(float) + kTagBytes;
}

// ----------------------------------------------------------------------------- part table

// Part table order: the parts of split buckets first (at the index of their partial slot),
// then the one-part buckets of more than P/4 entries (large_single), then the rest, each
// group in bucket order, so the longest wavefronts start first.

// One thread per bucket: per-workgroup totals of parts, partial slots, split buckets and
// large one-part buckets (the ptot of part_fill_block). After a pass B the pass-B scan has
// formed them already (seg_scan) and this launch is skipped.
__global__ __launch_bounds__(1024) void bucket_part_count(Batch b, const int *__restrict__ bstart, int B, int sb,
                                                          int *__restrict__ ptot, const int *__restrict__ bad) {
    __shared__ int wsum[16];
    const int bk = blockIdx.x * 1024 + threadIdx.x;
    int k = 0, n = 0, P = 1;
    if (bk < B) {
        n = (bad && *bad) ? 0 : bstart[bk + 1] - bstart[bk];  // (a failed resident CSR: empty buckets)
        P = load_desc(b, find_graph(b.node_offs, b.G, bk << sb)).WE;
        k = parts_of(n, P);
    }
    int t0, t1, t2, t3;
    (void)block_excl_scan<1024>(k, wsum, t0);
    (void)block_excl_scan<1024>(k > 1 ? k : 0, wsum, t1);
    (void)block_excl_scan<1024>(k > 1 ? 1 : 0, wsum, t2);
    (void)block_excl_scan<1024>(large_single(n, k, P) ? 1 : 0, wsum, t3);
    if (threadIdx.x == 0) {
        ptot[4 * blockIdx.x] = t0;
        ptot[4 * blockIdx.x + 1] = t1;
        ptot[4 * blockIdx.x + 2] = t2;
        ptot[4 * blockIdx.x + 3] = t3;
    }
}

// The part table, one workgroup per block of 1024 buckets (part_fill_block). After a pass B
// the pass-B scatter fills it in extra workgroups instead and this launch is skipped.
__global__ __launch_bounds__(256) void bucket_part_fill(Batch b, const int *__restrict__ bstart, int B, int sb,
                                                        const int *__restrict__ ptot, int4 *__restrict__ part,
                                                        int4 *__restrict__ multi, int *__restrict__ bmeta,
                                                        const int *__restrict__ bad) {
    part_fill_block(b, bstart, B, sb, ptot, (int)gridDim.x, (int)blockIdx.x, part, multi, bmeta, bad);
}

// The bucket path's per-node record {c_i, y_i}: 5 bytes (c_i, then y_i as one byte; y_i = 0
// when unknown, with c_i = 0), so the gathered table of N records is 5N bytes (plus 3 bytes
// of padding read by the last record's 8-byte load, which takes the next record's first
// bytes with it); with GEE_INFO_BYTES = 8, float2 records.
#ifndef GEE_INFO_BYTES
#define GEE_INFO_BYTES 5
#endif
constexpr int kInfoBytes = GEE_INFO_BYTES;
static_assert(kInfoBytes == 5 || kInfoBytes == 8, "5- or 8-byte node records");
static_assert(kMaxClasses <= 256, "a class index fits one byte");
__device__ __forceinline__ void put_info(float2 *info, int r, float c, int y) {
    if (kInfoBytes == 5) {
        unsigned char *q = reinterpret_cast<unsigned char *>(info) + 5 * (int64_t)r;
        const unsigned cb = __float_as_uint(c);
        q[0] = (unsigned char)(cb & 0xFFu);
        q[1] = (unsigned char)((cb >> 8) & 0xFFu);
        q[2] = (unsigned char)((cb >> 16) & 0xFFu);
        q[3] = (unsigned char)(cb >> 24);
        q[4] = (unsigned char)(y >= 0 ? y : 0);
    } else {
        info[r] = node_info(c, y);
    }
}
// {c_i, y_i as int bits} from a record read as 8 bytes
__device__ __forceinline__ float2 info_of(float2 raw) {
    return kInfoBytes == 5 ? make_float2(raw.x, __int_as_float(__float_as_int(raw.y) & 0xFF)) : raw;
}
__device__ __forceinline__ float2 get_info(const float2 *info, int r) {
    if (kInfoBytes == 5) {
        const unsigned char *q = reinterpret_cast<const unsigned char *>(info) + 5 * (int64_t)r;
        const unsigned cb = (unsigned)q[0] | ((unsigned)q[1] << 8) | ((unsigned)q[2] << 16) | ((unsigned)q[3] << 24);
        return make_float2(__uint_as_float(cb), __int_as_float((int)q[4]));
    }
    return info[r];
}

// s_i and c_i of row r of graph gd from its degree d (entries' weight sum, or count); the
// mode says which of them this pass owns (kDegIn: d is an in-degree, from the transposed
// entries, and sets c_i only; kDegOut: d is an out-degree and sets s_i only).
__device__ __forceinline__ void set_row_coef(const GDesc &gd, const float *__restrict__ inv_n, int r, float d,
                                             float *__restrict__ srow, float2 *__restrict__ info, int mode) {
    float s = 1.0f;
    if (gd.flags & kLap) {
        const float dd = d + ((gd.flags & kDiag) ? 1.0f : 0.0f);
        s = dd > 0.0f ? 1.0f / sqrtf(dd) : 0.0f;
    }
    if (mode != kDegIn) srow[r] = s;
    if (mode == kDegOut) return;
    int y = gd.labels[r - gd.node_off];
    if (y < 0 || y >= gd.K) y = -1;
    put_info(info, r, y >= 0 ? s * inv_n[gd.class_off + y] : 0.0f, y);
}

// ----------------------------------------------------------------------------- windows

// Entries [a, a + nwin*BWIN) of the bucketed arrays in windows of BWIN: lane l holds
// entries a + i*BWIN + 4l .. +3 of window i, read with one 8- or 16-byte load per array.
// The arrays are allocated kBucketWindowPad entries past their end, so every window of a
// part lies inside them; the buffer range ends with the part's last window, so windows
// past it read as 0 without touching memory. Entries past the part's end are masked by
// the caller. Every load is unconditional, which keeps the compiler's counter waits exact
// in the pipelined loops. Without KEYS the key array is not read (packed columns carry the
// row, see bucket_embed).
template <typename KT, bool WEIGHTED, bool COLS, bool KEYS = true>
struct Windows {
    __amdgpu_buffer_rsrc_t rk, rc, rv;
    struct Raw {
        int4 k, c;
        float4 v;
    };
    // limit: entries readable from a (the end of caller arrays that carry no padding)
    __device__ __forceinline__ Windows(const KT *key, const int *col, const float *val, int a, int nwin,
                                       int64_t limit = INT64_MAX) {
        int64_t n = (int64_t)nwin * BWIN;
        n = n < limit ? n : limit;
        n = n > 0 ? n : 0;
        rk = buffer_rsrc(key + a, n * (int64_t)sizeof(KT));
        rc = buffer_rsrc(COLS ? (const void *)(col + a) : (const void *)key, COLS ? n * 4 : 0);
        rv = buffer_rsrc(WEIGHTED ? (const void *)(val + a) : (const void *)key, WEIGHTED ? n * 4 : 0);
    }
    __device__ __forceinline__ void load(int i, int lane, Raw &r) const {
        const uint32_t o = (uint32_t)(i * BWIN + BEPL * lane);
        if (!KEYS) {
            r.k = make_int4(0, 0, 0, 0);
        } else if (sizeof(KT) == 2) {
            const uint2 q = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(rk, 2 * o, 0, 0));
            r.k = make_int4((int)(q.x & 0xFFFFu), (int)(q.x >> 16), (int)(q.y & 0xFFFFu), (int)(q.y >> 16));
        } else {
            r.k = buf_i4(rk, 4 * o);
        }
        if (COLS) r.c = buf_i4(rc, 4 * o);
        r.v = WEIGHTED ? buf_f4(rv, 4 * o) : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
    }
};

// Rows of a resident CSR's entries inside one bucket, from row_ptr alone (no key array):
// lane r holds s = the first entry of the bucket's row r; the row of entry e is the number of
// rows r with s_r <= e, less one. For a window of BWIN entries starting at w0 that is the
// rows started before w0 (one ballot) plus the rows starting inside the window up to e: each
// lane adds one to the 8-bit counter of its row's start position (four to a word in `cw`,
// 64 words of LDS), each lane reads the word of its own four entries, and a wave scan adds
// the counts of the lanes before it. Rows are clamped into the bucket (a malformed CSR has
// been refused by csr_prep before any part is listed).
struct CsrRows {
    int s;
    unsigned *cw;
    __device__ __forceinline__ void init(const int *__restrict__ rp, int N, int64_t M, int row0, int R, int lane,
                                         unsigned *words) {
        cw = words;
        s = INT_MAX;
        if (lane < R) {
            const int64_t v = rp[min(row0 + lane, N)];  // rows past N start at rp[N] = M
            s = (int)(v < 0 ? 0 : (v > M ? M : v));
        }
    }
    __device__ __forceinline__ void rows(int w0, int lane, int R, int (&row)[BEPL]) const {
        const int before = __popcll(ballot(s < w0));
        cw[lane] = 0u;
        wave_lds_fence();
        const int d = s - w0;  // (s = INT_MAX on lanes past the rows: no overflow, d >= BWIN)
        if (d >= 0 && d < BWIN) atomicAdd(&cw[d >> 2], 1u << (8 * (d & 3)));
        wave_lds_fence();
        const unsigned q = cw[lane];
        const int c0 = (int)(q & 0xFFu), c1 = c0 + (int)((q >> 8) & 0xFFu);
        const int c2 = c1 + (int)((q >> 16) & 0xFFu), c3 = c2 + (int)(q >> 24);
        const int base = before + wave_scan_add(c3) - c3 - 1;
        const int cc[BEPL] = {c0, c1, c2, c3};
#pragma unroll
        for (int j = 0; j < BEPL; ++j) row[j] = min(max(base + cc[j], 0), R - 1);
        wave_lds_fence();
    }
};

// The part a wavefront works on (false past the last part) and its graph. The entry is
// loaded together with the part count (from an index clamped to the table's capacity).
__device__ __forceinline__ bool part_view(const Batch &b, int j, const int4 *__restrict__ part, int cap,
                                          const int *__restrict__ bmeta, int sb, int4 &pt, GDesc &gd) {
    const int n = bmeta[0];
    pt = part[min(j, cap - 1)];
    if (j >= n) return false;
    gd = load_desc(b, find_graph(b.node_offs, b.G, pt.x << sb));
    return true;
}

// ----------------------------------------------------------------------------- degrees

// Four independent wavefronts per workgroup, one part each. The R row sums are kept in
// kDegCopies = 32 private copies per wavefront (rows padded to R + 1 so the copies of a
// row sit in different banks): lanes l and l + 32 own copy l, the low half of the
// wavefront adds its entries with plain LDS read-modify-writes, then the high half. A
// window's 256 entries fall on only R rows, and LDS float atomics on shared sums run at a
// small fraction of the plain LDS rate. The copies are added in copy order at the end.
// With PACKED the rows come from the packed column words (see bucket_embed), read in
// place of the keys.
constexpr int kDegCopies = 32;
// With CSRM (a resident CSR: no keys, no packed words) the rows come from row_ptr
// (CsrRows) and the entry arrays are the caller's, of M entries.
template <typename KT, bool WEIGHTED, bool PACKED, bool CSRM = false>
__global__ __launch_bounds__(256) void bucket_degree(Batch b, const KT *__restrict__ key, const int *__restrict__ pcol,
                                                     const float *__restrict__ val,
                                                     const int4 *__restrict__ part, int cap,
                                                     const int *__restrict__ bmeta, int sb,
                                                     const float *__restrict__ inv_n,
                                                     float *__restrict__ dpart, float *__restrict__ srow,
                                                     float2 *__restrict__ info, int mode,
                                                     const int *__restrict__ rp = nullptr, int64_t M = 0) {
    extern __shared__ float dsum_all[];  // [4][kDegCopies][R + 1], then (CSRM) [4][64] row-start counters
    const int lane = lane_id();
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int4 pt;
    GDesc gd;
    if (!part_view(b, blockIdx.x * 4 + wib, part, cap, bmeta, sb, pt, gd)) return;
    const bool lap = gd.flags & kLap;
    const int R = 1 << sb, r = (pt.x << sb) + lane;
    const bool own = lane < R && r >= gd.node_off && r < gd.node_off + gd.N;
    if (!lap) {
        // c_i = 1 / n_{y_i}; a split bucket's rows are set by bucket_degree_fix
        if (pt.w < 0 && own) set_row_coef(gd, inv_n, r, 0.0f, srow, info, mode);
        return;
    }
    const int RS = R + 1;
    float *dsum = dsum_all + wib * kDegCopies * RS;
    for (int i = lane; i < kDegCopies * RS; i += 64) dsum[i] = 0.0f;
    wave_lds_fence();
    float *mine = dsum + (lane & (kDegCopies - 1)) * RS;
    const bool wt = WEIGHTED && gd.weighted;
    const int rmask = R - 1;
    using W = Windows<KT, WEIGHTED, PACKED, !PACKED && !CSRM>;
    const int nwin = (pt.z - pt.y + BWIN - 1) / BWIN;
    const W win(key, pcol, val, pt.y, nwin, CSRM ? M - pt.y : INT64_MAX);
    CsrRows cr;
    if (CSRM)
        cr.init(rp, gd.N, M, (pt.x << sb) - gd.node_off, R, lane,
                reinterpret_cast<unsigned *>(dsum_all + 4 * kDegCopies * RS) + 64 * wib);
    // window i: entries masked past the part's end add 0
    auto add = [&](int i, const typename W::Raw &q) {
        const int nv = min(BEPL, max(0, pt.z - (pt.y + i * BWIN + BEPL * lane)));
        int4 k4 = PACKED ? make_int4(q.c.x >> kPackShift, q.c.y >> kPackShift, q.c.z >> kPackShift,
                                     q.c.w >> kPackShift)
                         : q.k;
        if (CSRM) {
            int rr[BEPL];
            cr.rows(pt.y + i * BWIN, lane, R, rr);
            k4 = make_int4(rr[0], rr[1], rr[2], rr[3]);
        }
        const int kk[BEPL] = {k4.x, k4.y, k4.z, k4.w};
        const float vv[BEPL] = {q.v.x, q.v.y, q.v.z, q.v.w};
        float x[BEPL];
        int rw[BEPL];
#pragma unroll
        for (int j = 0; j < BEPL; ++j) {
            x[j] = j < nv ? (wt ? vv[j] : 1.0f) : 0.0f;
            rw[j] = kk[j] & rmask;
        }
        if (lane < 32) {
#pragma unroll
            for (int j = 0; j < BEPL; ++j) mine[rw[j]] += x[j];
        }
        wave_lds_fence();
        if (lane >= 32) {
#pragma unroll
            for (int j = 0; j < BEPL; ++j) mine[rw[j]] += x[j];
        }
        wave_lds_fence();
    };
    // two register sets with fixed roles (no copies that would wait for loads in flight):
    // the loads of window i+1 are in flight while window i is added
    typename W::Raw A, Bw;
    win.load(0, lane, A);
    // (scheduling barriers keep each window's loads issued before the previous window's
    // adds, which wait for their own loads only)
    for (int i = 0; i < nwin; i += 2) {
        win.load(i + 1, lane, Bw);
        __builtin_amdgcn_sched_barrier(0);
        add(i, A);
        __builtin_amdgcn_sched_barrier(0);
        win.load(i + 2, lane, A);
        __builtin_amdgcn_sched_barrier(0);
        add(i + 1, Bw);  // past the last window every entry is masked (adds 0)
        __builtin_amdgcn_sched_barrier(0);
    }
    wave_lds_fence();
    float d = 0.0f;
    if (lane < R)
        for (int c = 0; c < kDegCopies; ++c) d += dsum[c * RS + lane];
    if (pt.w >= 0) {
        dpart[(int64_t)pt.w * 64 + lane] = d;
        return;
    }
    if (own) set_row_coef(gd, inv_n, r, d, srow, info, mode);
}

// Wavefronts take the split buckets in turn: degrees = the parts' partial sums in part
// order (the Laplacian), then s_i and c_i of the bucket's rows.
__global__ __launch_bounds__(256) void bucket_degree_fix(Batch b, const int4 *__restrict__ multi,
                                                         const int *__restrict__ bmeta, int sb,
                                                         const float *__restrict__ inv_n,
                                                         const float *__restrict__ dpart, float *__restrict__ srow,
                                                         float2 *__restrict__ info, int mode) {
    const int lane = lane_id();
    const int nmulti = bmeta[1];
    for (int i = blockIdx.x * 4 + (threadIdx.x >> 6); i < nmulti; i += gridDim.x * 4) {
        const int4 m = multi[i];
        const int r0 = m.x << sb;
        const GDesc gd = load_desc(b, find_graph(b.node_offs, b.G, r0));
        float d = 0.0f;
        if (gd.flags & kLap) {
            const float *dp = dpart + (int64_t)m.y * 64 + lane;
            int k = 0;
            for (; k + 4 <= m.z; k += 4) {
                const float x0 = dp[(int64_t)k * 64], x1 = dp[(int64_t)(k + 1) * 64];
                const float x2 = dp[(int64_t)(k + 2) * 64], x3 = dp[(int64_t)(k + 3) * 64];
                d += x0;
                d += x1;
                d += x2;
                d += x3;
            }
            for (; k < m.z; ++k) d += dp[(int64_t)k * 64];
        }
        const int r = r0 + lane;
        if (lane < (1 << sb) && r >= gd.node_off && r < gd.node_off + gd.N)
            set_row_coef(gd, inv_n, r, d, srow, info, mode);
    }
}

// ----------------------------------------------------------------------------- class sums

// Lane-per-row finish of bucket rows r0 .. r0+R-1 held in acc[R][KP]: diagonal term, then
// fac[row] = s_i, or 1/|row| under correlation (class columns K .. KP-1 are zero).
// q = {c_i, y_i} and s of the lane's row, loaded by the caller. With rcnt (sparse Z of one
// graph), also the row's number of non-zero entries of Z, acc * fac exactly as written.
__device__ __forceinline__ void finish_rows(const GDesc &gd, int r0, int R, int KP, float *acc, float *fac,
                                            float2 q, float s, int lane, unsigned *status, int *rcnt,
                                            int *nzl = nullptr) {
    const int r = r0 + lane;
    if (lane < R && r >= gd.node_off && r < gd.node_off + gd.N) {
        float *row = acc + lane * KP;
        const int y = __float_as_int(q.y);
        if ((gd.flags & kDiag) && dbg_ok(y >= 0 && y < KP, status)) row[y] += q.x;
        float ss = 0.0f;
        const bool cor = gd.flags & kCor;
        if (cor) {
            const float4 *a4 = reinterpret_cast<const float4 *>(row);
            for (int q = 0; q < (KP >> 2); ++q) {
                const float4 t = a4[q];
                ss += t.x * t.x + t.y * t.y + t.z * t.z + t.w * t.w;
            }
        }
        const float f = row_factor((gd.flags & kLap) ? s : 1.0f, ss, cor);
        fac[lane] = f;
        if (rcnt) {
            int nz = 0;
            const float4 *a4 = reinterpret_cast<const float4 *>(row);
            for (int q4 = 0; q4 < (KP >> 2); ++q4) {  // columns K .. KP-1 hold 0
                const float4 t = a4[q4];
                nz += (t.x * f != 0.0f) + (t.y * f != 0.0f) + (t.z * f != 0.0f) + (t.w * f != 0.0f);
            }
            rcnt[r - gd.node_off] = nz;
            if (nzl) nzl[lane] = nz;
        }
    }
}

// Z rows r0 .. of the bucket (those of the graph) as one flat run of floats, written by
// threads t of nt with non-temporal stores (Z is not read again here): when the run starts
// on a 16-byte boundary (Z's base permitting: the run starts at a multiple of R rows),
// thread t writes floats 4t .. 4t+3, 4(t+nt) .., one 16-byte store each, and the last
// F mod 4 floats one by one; otherwise every float one by one.
__device__ __forceinline__ void write_rows(const GDesc &gd, int r0, int R, int KP, const float *acc,
                                           const float *fac, int t, int nt) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const int K = gd.K;
    const int nv = max(0, min(R, gd.node_off + gd.N - r0));
    const int F = nv * K;
    float *z = gd.Z + (int64_t)(r0 - gd.node_off) * K;
    int f0 = 0;
    if ((reinterpret_cast<uintptr_t>(z) & 15) == 0) {
        const int F4 = F & ~3, step = 4 * nt;
        const int qn = step / K, rn = step - qn * K;
        int jj = (4 * t) / K, kk = 4 * t - ((4 * t) / K) * K;
        const bool whole = (K & 3) == 0;  // every group of 4 lies in one row, 16-byte aligned in LDS
        for (int f = 4 * t; f < F4; f += step) {
            v4 v;
            if (whole) {
                const float4 a = *reinterpret_cast<const float4 *>(acc + jj * KP + kk);
                const float g = fac[jj];
                v[0] = a.x * g;
                v[1] = a.y * g;
                v[2] = a.z * g;
                v[3] = a.w * g;
            } else {
                int j2 = jj, k2 = kk;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = acc[j2 * KP + k2] * fac[j2];
                    if (++k2 == K) {
                        k2 = 0;
                        ++j2;
                    }
                }
            }
            __builtin_nontemporal_store(v, reinterpret_cast<v4 *>(z + f));
            kk += rn;
            jj += qn;
            if (kk >= K) {
                kk -= K;
                ++jj;
            }
        }
        f0 = F4;
    }
    const int qn = nt / K, rn = nt - qn * K;
    int jj = (f0 + t) / K, kk = f0 + t - ((f0 + t) / K) * K;
    for (int f = f0 + t; f < F; f += nt) {
        __builtin_nontemporal_store(acc[jj * KP + kk] * fac[jj], z + f);
        kk += rn;
        jj += qn;
        if (kk >= K) {
            kk -= K;
            ++jj;
        }
    }
}

// Rows as write_rows writes them (nv rows from acc / fac, K classes, row stride KP), but only
// their non-zero values, each as a (class, value bits) pair, in row-major order from place
// `off` of the staging pairs (sparse Z): one wavefront, four consecutive floats per lane per
// step, each non-zero placed by the non-zeros before it (four ballots), one 8-byte
// non-temporal store per pair. The same values, bit for bit, as the dense rows.
__device__ __forceinline__ void write_rows_sparse(int K, int KP, int nv, const float *acc, const float *fac,
                                                  int lane, int2 *__restrict__ zp, int64_t off) {
    typedef int v2i __attribute__((ext_vector_type(2)));
    const int F = max(nv, 0) * K;
    const uint64_t below = (1ull << lane) - 1;
    const int qn = 256 / K, rn = 256 - qn * K;
    int jj = (4 * lane) / K, kk = 4 * lane - ((4 * lane) / K) * K;
    for (int f = 4 * lane, c0 = 0; c0 < F; c0 += 256, f += 256) {
        float v[4];
        int cls[4];
        int j2 = jj, k2 = kk;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[e] = f + e < F ? acc[j2 * KP + k2] * fac[j2] : 0.0f;
            cls[e] = k2;
            if (++k2 == K) {
                k2 = 0;
                ++j2;
            }
        }
        uint64_t m[4];
        int before = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            m[e] = ballot(v[e] != 0.0f);
            before += __popcll(m[e] & below);
        }
        int mine = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (v[e] != 0.0f) {
                v2i pr;
                pr.x = cls[e];
                pr.y = __float_as_int(v[e]);
                __builtin_nontemporal_store(pr, reinterpret_cast<v2i *>(zp + off + before + mine));
                ++mine;
            }
        }
        off += __popcll(m[0]) + __popcll(m[1]) + __popcll(m[2]) + __popcll(m[3]);
        kk += rn;
        jj += qn;
        if (kk >= K) {
            kk -= K;
            ++jj;
        }
    }
}

// With PACKED (after a pass B) each column word carries its row inside the bucket above
// its kPackShift bits, so the keys are not read.
// With CSRM (a resident CSR) the rows come from row_ptr (CsrRows), the entry arrays are the
// caller's, of M entries, and columns outside [0, N) are skipped and raise GEE_DATA_CSR.
template <typename KT, bool WEIGHTED, bool PACKED, bool CSRM = false>
__global__ __launch_bounds__(64) void bucket_embed(Batch b, const KT *__restrict__ key, const int *__restrict__ col,
                                                   const float *__restrict__ val,
                                                   const int4 *__restrict__ part, int cap,
                                                   const int *__restrict__ bmeta, int sb,
                                                   const float2 *__restrict__ info,
                                                   const float *__restrict__ srow, float *__restrict__ zpart, int zs,
                                                   int *__restrict__ rcnt, int2 *__restrict__ zsp,
                                                   const int *__restrict__ rp = nullptr,
                                                   int64_t M = 0) {
    extern __shared__ float smem_b[];
    const int lane = lane_id();
    int4 pt;
    GDesc gd;
    if (!part_view(b, blockIdx.x, part, cap, bmeta, sb, pt, gd)) return;
    const int K = gd.K, KP = ring_stride(K), node_off = gd.node_off;
    const int R = 1 << sb, rmask = R - 1;
    float *acc = smem_b;           // [R][KP]
    float *fac = smem_b + R * KP;  // [64] row factors
    unsigned char *tag = reinterpret_cast<unsigned char *>(fac + 64);  // [kTagBytes] entry ids
    // the lane's row {c_i, y_i} and s_i, needed at the end, loaded now
    const int r0 = pt.x << sb, rl = r0 + lane;
    const bool own = lane < R && rl >= node_off && rl < node_off + gd.N;
    const float2 q_own = own ? get_info(info, rl) : make_float2(0.0f, 0.0f);
    const float s_own = own ? srow[rl] : 0.0f;
    {
        float4 *a4 = reinterpret_cast<float4 *>(acc);
        for (int i = lane; i < ((R * KP) >> 2); i += 64) a4[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    wave_lds_fence();

    using W = Windows<KT, WEIGHTED, true, !PACKED && !CSRM>;
    const int nwin = (pt.z - pt.y + BWIN - 1) / BWIN;
    const W win(key, col, val, pt.y, nwin, CSRM ? M - pt.y : INT64_MAX);
    CsrRows cr;
    if (CSRM)
        cr.init(rp, gd.N, M, r0 - node_off, R, lane, reinterpret_cast<unsigned *>(tag + kTagBytes));
    const bool chk = CSRM && validates(gd);
    bool badc = false;
    const __amdgpu_buffer_rsrc_t r_inf =
        buffer_rsrc(reinterpret_cast<const char *>(info) + (int64_t)node_off * kInfoBytes,
                    (int64_t)gd.N * kInfoBytes + (8 - kInfoBytes));
    struct Prep {
        int row[BEPL];
        float x[BEPL];   // val, 0 when masked
        float2 f[BEPL];  // {c_j, y_j}; masked entries read past the table: {0, class 0}
    };
    auto prep = [&](int i, const typename W::Raw &q, Prep &P) {
        const int nv = min(BEPL, max(0, pt.z - (pt.y + i * BWIN + BEPL * lane)));
        int kk[BEPL] = {q.k.x, q.k.y, q.k.z, q.k.w};
        const int cc[BEPL] = {q.c.x, q.c.y, q.c.z, q.c.w};
        const float vv[BEPL] = {q.v.x, q.v.y, q.v.z, q.v.w};
        if (CSRM) cr.rows(pt.y + i * BWIN, lane, R, kk);
#pragma unroll
        for (int j = 0; j < BEPL; ++j) {
            const int cj = PACKED ? (cc[j] & ((1 << kPackShift) - 1)) : cc[j];
            bool use = j < nv;
            if (CSRM && use && (unsigned)(cj - node_off) >= (unsigned)gd.N) {
                badc = true;  // a column outside the graph: skipped
                use = false;
            }
            const unsigned u = use ? (unsigned)(cj - node_off) : 0xFFFFFFFFu;
            P.row[j] = (PACKED ? (cc[j] >> kPackShift) : kk[j]) & rmask;
            P.x[j] = use ? vv[j] : 0.0f;
            P.f[j] = info_of(buf_f2(r_inf, u * (unsigned)kInfoBytes));
        }
    };
    // window update: see lds_tag_add
    auto add = [&](const Prep &P) {
        int ad[BEPL];
        float xv[BEPL];
#pragma unroll
        for (int j = 0; j < BEPL; ++j) {
            ad[j] = P.row[j] * KP + __float_as_int(P.f[j].y);
            xv[j] = P.x[j] * P.f[j].x;
        }
        lds_tag_add<BEPL>(acc, tag, ad, xv, lane, kTagBytes - 1, R * KP, b.status);
    };
    // Three stages, two register sets each with fixed roles (no copies that would wait for
    // loads in flight): the loads of window i+2 are issued first, then the gathers of
    // window i+1 (which wait only for its loads, issued one step earlier), then window i
    // is added (its gathers were issued one step earlier). The counter retires in issue
    // order, so every wait leaves the younger loads in flight.
    typename W::Raw R0, R1;
    Prep P0, P1;
    win.load(0, lane, R0);
    win.load(1, lane, R1);
    prep(0, R0, P0);
    // (scheduling barriers keep that issue order)
#if GEE_EMBED_SCHED_BARRIER
#define EMB_SB() __builtin_amdgcn_sched_barrier(0)
#else
#define EMB_SB() (void)0
#endif
    for (int i = 0; i < nwin; i += 2) {
        win.load(i + 2, lane, R0);
        EMB_SB();
        prep(i + 1, R1, P1);
        EMB_SB();
        add(P0);
        EMB_SB();
        win.load(i + 3, lane, R1);
        EMB_SB();
        prep(i + 2, R0, P0);
        EMB_SB();
        add(P1);  // past the last window every entry is masked (adds 0)
        EMB_SB();
    }
#undef EMB_SB
    wave_lds_fence();
    if (CSRM && chk && __ballot(badc ? 1 : 0) != 0 && lane == 0) raise_error(b.status, kErrCsr);
    if (pt.w < 0) {
        finish_rows(gd, r0, R, KP, acc, fac, q_own, s_own, lane, b.status, rcnt);
        wave_lds_fence();
        if (zsp)
            write_rows_sparse(K, KP, min(R, gd.node_off + gd.N - r0), acc, fac, lane, zsp,
                              (int64_t)(r0 - gd.node_off) * K);
        else
            write_rows(gd, r0, R, KP, acc, fac, lane, 64);
        return;
    }
    // a part of a split bucket: its raw sums of the R rows, flat [R][K]
    float *zp = zpart + (int64_t)pt.w * zs;
    const int q64 = 64 / K, r64 = 64 - q64 * K;
    int jj = lane / K, kk = lane - (lane / K) * K;
    for (int f = lane; f < R * K; f += 64) {
        zp[f] = acc[jj * KP + kk];
        kk += r64;
        jj += q64;
        if (kk >= K) {
            kk -= K;
            ++jj;
        }
    }
}

// Workgroups of kFixThreads take the split buckets in turn (the grid is sized for the
// largest possible count; far fewer are split): the parts' raw sums added in part order (the
// same order, so the same bits, whatever the thread count), then the rows
// finished as in bucket_embed. A thread takes kFixUnroll class sums of the bucket, and the
// loads of four parts of all of them are in flight together; the finishing lanes load their
// rows' coefficients first, so a bucket costs few dependent memory round trips.
template <int kFixThreads>
__global__ __launch_bounds__(kFixThreads) void bucket_embed_fix(Batch b, const int4 *__restrict__ multi,
                                                                const int *__restrict__ bmeta, int sb,
                                                                const float2 *__restrict__ info,
                                                                const float *__restrict__ srow,
                                                                const float *__restrict__ zpart, int zs,
                                                                int *__restrict__ rcnt, int2 *__restrict__ zsp) {
    extern __shared__ float smem_b[];
    const int nmulti = bmeta[1];
    for (int i = blockIdx.x; i < nmulti; i += gridDim.x) {
        const int4 m = multi[i];
        const int r0 = m.x << sb;
        const GDesc gd = load_desc(b, find_graph(b.node_offs, b.G, r0));
        const int K = gd.K, KP = ring_stride(K), R = 1 << sb;
        const int t = threadIdx.x;
        const int rl = r0 + t;
        const bool own = t < R && rl >= gd.node_off && rl < gd.node_off + gd.N;
        const float2 q_own = own ? get_info(info, rl) : make_float2(0.0f, 0.0f);
        const float s_own = own ? srow[rl] : 0.0f;
        float *acc = smem_b;
        float *fac = smem_b + R * KP;
        __syncthreads();  // the previous bucket's rows are written
        {
            // class columns K .. KP-1 stay zero (the norm reads whole 16-byte groups)
            float4 *a4 = reinterpret_cast<float4 *>(acc);
            for (int q = t; q < ((R * KP) >> 2); q += kFixThreads) a4[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        __syncthreads();
        const float *zp = zpart + (int64_t)m.y * zs;
        const int n = R * K;
        for (int f0 = t; f0 < n; f0 += kFixUnroll * kFixThreads) {
            float sum[kFixUnroll];
#pragma unroll
            for (int u = 0; u < kFixUnroll; ++u) sum[u] = 0.0f;
            int k = 0;
            for (; k + 4 <= m.z; k += 4) {
                float x[kFixUnroll][4];
#pragma unroll
                for (int u = 0; u < kFixUnroll; ++u) {
                    const int f = min(f0 + u * kFixThreads, n - 1);  // (past n: a sum that is not kept)
#pragma unroll
                    for (int j = 0; j < 4; ++j) x[u][j] = zp[(int64_t)(k + j) * zs + f];
                }
#pragma unroll
                for (int u = 0; u < kFixUnroll; ++u)
#pragma unroll
                    for (int j = 0; j < 4; ++j) sum[u] += x[u][j];
            }
            for (; k < m.z; ++k) {
                float x[kFixUnroll];
#pragma unroll
                for (int u = 0; u < kFixUnroll; ++u) x[u] = zp[(int64_t)k * zs + min(f0 + u * kFixThreads, n - 1)];
#pragma unroll
                for (int u = 0; u < kFixUnroll; ++u) sum[u] += x[u];
            }
#pragma unroll
            for (int u = 0; u < kFixUnroll; ++u) {
                const int f = f0 + u * kFixThreads;
                if (f < n) acc[(f / K) * KP + f % K] = sum[u];
            }
        }
        __syncthreads();
        int *nzl = reinterpret_cast<int *>(fac + 64);  // [64] rows' non-zero counts (staged sparse Z)
        if (t < 64) {
            if (zsp) nzl[t] = 0;
            finish_rows(gd, r0, R, KP, acc, fac, q_own, s_own, t, b.status, rcnt, zsp ? nzl : nullptr);
        }
        __syncthreads();
        if (!zsp) {
            write_rows(gd, r0, R, KP, acc, fac, t, kFixThreads);
        } else {
            // wavefront w writes rows [w rpw, (w + 1) rpw) from the place after the rows before
            constexpr int kW = kFixThreads / 64;
            const int rpw = R / kW, w = t >> 6, ra = w * rpw;
            const int nv = min(ra + rpw, gd.node_off + gd.N - r0) - ra;
            int64_t off = (int64_t)(r0 - gd.node_off) * K;
            for (int j = 0; j < ra; ++j) off += nzl[j];
            write_rows_sparse(K, KP, nv, acc + ra * KP, fac + ra, t & 63, zsp, off);
        }
    }
}

// ----------------------------------------------------------------------------- resident CSR

// Thread per row pointer of a resident CSR: the checks (row_ptr[0] = 0, non-decreasing,
// within [0, M], row_ptr[N] = M; a failure sets *bad, which empties every bucket, and raises
// GEE_DATA_CSR unless the graph skips validation) and the bucket starts bstart[b] =
// row_ptr[b R] (clamped into [0, M]; bstart[B] = row_ptr[N]).
// Workgroups past the row pointers' take the class totals, one wavefront per class.
__global__ __launch_bounds__(256) void csr_prep(const int *__restrict__ rp, int N, int64_t M, int sb,
                                                int *__restrict__ bstart, int *__restrict__ bad, unsigned *status,
                                                int chk, int nprep, Batch b, int Ktot, const int *__restrict__ cpart,
                                                int *__restrict__ counts, float *__restrict__ inv_n) {
    if ((int)blockIdx.x >= nprep) {
        const int c = ((int)blockIdx.x - nprep) * 4 + (int)(threadIdx.x >> 6);
        if (c < Ktot) class_count_total(b, c, cpart, counts, inv_n);
        return;
    }
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i > N) return;
    const int64_t v = rp[i];
    bool wrong = v < 0 || v > M || (i == 0 && v != 0) || (i == N && v != M);
    if (i < N) wrong = wrong || rp[i + 1] < v;
    if (wrong) {
        *bad = 1;
        if (chk) raise_error(status, kErrCsr);
    }
    const int R = 1 << sb;
    if ((i & (R - 1)) == 0 || i == N) bstart[(i + R - 1) >> sb] = (int)(v < 0 ? 0 : (v > M ? M : v));
}

template <bool WEIGHTED>
static hipError_t launch_bucket_sums_csr(const Batch &b, const Plan &p, const Work &wk, const int *rp, const int *col,
                                         const float *val, int64_t M, hipStream_t s) {
    const unsigned nbp = (unsigned)p.bparts;
    const int mode = kDegBoth;
    prof_begin(kKBucketDegree, s);
    const size_t dlds = (size_t)4 * kDegCopies * ((1 << p.sb) + 1) * sizeof(float) + 4 * 64 * sizeof(unsigned);
    hipLaunchKernelGGL((bucket_degree<int, WEIGHTED, false, true>), dim3((nbp + 3) / 4), dim3(256), dlds, s, b,
                       (const int *)nullptr, col, val, wk.part, (int)nbp, wk.bmeta, p.sb, wk.inv_n, wk.dpart, wk.srow,
                       wk.info, mode, rp, M);
    prof_end(kKBucketDegree, s);
    const bool many = p.bslots / 2 > kFixManyBuckets;  // (split buckets the launch can hold, at most)
    const unsigned nm = (unsigned)std::min<int64_t>(p.bslots / 2 + 1, many ? kFixGridMany : kFixGrid);
    prof_begin(kKBucketDegreeFix, s);
    hipLaunchKernelGGL(bucket_degree_fix, dim3((nm + 3) / 4), dim3(256), 0, s, b, wk.multi, wk.bmeta, p.sb, wk.inv_n,
                       wk.dpart, wk.srow, wk.info, mode);
    prof_end(kKBucketDegreeFix, s);
    const size_t lds = bucket_lds(p.sb, p.Kmax) + 64 * sizeof(unsigned);
    const int zs = p.Kmax << p.sb;
    prof_begin(kKBucketEmbed, s);
    hipLaunchKernelGGL((bucket_embed<int, WEIGHTED, false, true>), dim3(nbp), dim3(64), lds, s, b, (const int *)nullptr,
                       col, val, wk.part, (int)nbp, wk.bmeta, p.sb, wk.info, wk.srow, wk.zpart, zs,
                       (int *)nullptr, (int2 *)nullptr, rp, M);
    prof_end(kKBucketEmbed, s);
    prof_begin(kKBucketEmbedFix, s);
    if (many)
        hipLaunchKernelGGL(bucket_embed_fix<kFixThreadsMany>, dim3(nm), dim3(kFixThreadsMany), lds, s, b, wk.multi,
                           wk.bmeta, p.sb, wk.info, wk.srow, wk.zpart, zs, (int *)nullptr, (int2 *)nullptr);
    else
        hipLaunchKernelGGL(bucket_embed_fix<kFixThreads>, dim3(nm), dim3(kFixThreads), lds, s, b, wk.multi, wk.bmeta,
                           p.sb, wk.info, wk.srow, wk.zpart, zs, (int *)nullptr, (int2 *)nullptr);
    prof_end(kKBucketEmbedFix, s);
    return hipGetLastError();
}

hipError_t launch_bucket_embed_csr(const Batch &b, const Plan &p, const Work &wk, const int *rp, const int *col,
                                   const float *val, int64_t M, unsigned *status, hipStream_t s) {
    const int N = (int)p.Ntot;
    int *bad = wk.meta + 1;  // cleared by the class-count launch before this one
    const int nprep = (N + 1 + 255) / 256;
    prof_begin(kKCsrPrep, s);
    hipLaunchKernelGGL(csr_prep, dim3((unsigned)(nprep + (p.Ktot + 3) / 4)), dim3(256), 0, s, rp, N, M, p.sb,
                       wk.bstart, bad, status, (b.one.flags & kNoValidate) ? 0 : 1, nprep, b, p.Ktot,
                       (const int *)wk.cpart, wk.counts, wk.inv_n);
    prof_end(kKCsrPrep, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nblk = (unsigned)((p.B + 1023) / 1024);
    if (nblk > 1) {  // (one block of buckets forms its own totals)
        prof_begin(kKBucketPartCount, s);
        hipLaunchKernelGGL(bucket_part_count, dim3(nblk), dim3(1024), 0, s, b, wk.bstart, p.B, p.sb, wk.ptot,
                           (const int *)bad);
        prof_end(kKBucketPartCount, s);
    }
    prof_begin(kKBucketPartFill, s);
    hipLaunchKernelGGL(bucket_part_fill, dim3(nblk), dim3(256), 0, s, b, wk.bstart, p.B, p.sb,
                       nblk > 1 ? (const int *)wk.ptot : nullptr, wk.part, wk.multi, wk.bmeta, (const int *)bad);
    prof_end(kKBucketPartFill, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return val ? launch_bucket_sums_csr<true>(b, p, wk, rp, col, val, M, s)
               : launch_bucket_sums_csr<false>(b, p, wk, rp, col, val, M, s);
}

// ----------------------------------------------------------------------------- launch

template <typename KT, bool WEIGHTED>
static void launch_bucket_sums(const Batch &b, const Plan &p, const Work &wk, const KT *key, hipStream_t s, int mode,
                               bool sums) {
    const unsigned nbp = (unsigned)p.bparts;
    const float *val = WEIGHTED ? wk.tval : nullptr;
    prof_begin(kKBucketDegree, s);
    const size_t dlds = (size_t)4 * kDegCopies * ((1 << p.sb) + 1) * sizeof(float);
    if (p.s2 > 0 && !GEE_PASSB_KEYS)  // rows from the packed column words
        hipLaunchKernelGGL((bucket_degree<KT, WEIGHTED, true>), dim3((nbp + 3) / 4), dim3(256), dlds, s, b, key,
                           wk.tcol, val, wk.part, (int)nbp, wk.bmeta, p.sb, wk.inv_n, wk.dpart, wk.srow, wk.info,
                           mode);
    else
        hipLaunchKernelGGL((bucket_degree<KT, WEIGHTED, false>), dim3((nbp + 3) / 4), dim3(256), dlds, s, b, key,
                           wk.tcol, val, wk.part, (int)nbp, wk.bmeta, p.sb, wk.inv_n, wk.dpart, wk.srow, wk.info,
                           mode);
    prof_end(kKBucketDegree, s);
    // split buckets, at most (the grids of the two fix kernels loop over the actual count)
    const bool many = p.bslots / 2 > kFixManyBuckets;  // (split buckets the launch can hold, at most)
    const unsigned nm = (unsigned)std::min<int64_t>(p.bslots / 2 + 1, many ? kFixGridMany : kFixGrid);
    prof_begin(kKBucketDegreeFix, s);
    hipLaunchKernelGGL(bucket_degree_fix, dim3((nm + 3) / 4), dim3(256), 0, s, b, wk.multi, wk.bmeta, p.sb, wk.inv_n,
                       wk.dpart, wk.srow, wk.info, mode);
    prof_end(kKBucketDegreeFix, s);
    if (!sums) return;
    const size_t lds = bucket_lds(p.sb, p.Kmax);
    const int zs = p.Kmax << p.sb;  // floats per partial slot
    prof_begin(kKBucketEmbed, s);
    if (p.s2 > 0)  // pass B packed the rows into the column words
        hipLaunchKernelGGL((bucket_embed<KT, WEIGHTED, true>), dim3(nbp), dim3(64), lds, s, b, key, wk.tcol, val,
                           wk.part, (int)nbp, wk.bmeta, p.sb, wk.info, wk.srow, wk.zpart, zs, wk.rcnt, wk.zs_pairs);
    else
        hipLaunchKernelGGL((bucket_embed<KT, WEIGHTED, false>), dim3(nbp), dim3(64), lds, s, b, key, wk.tcol, val,
                           wk.part, (int)nbp, wk.bmeta, p.sb, wk.info, wk.srow, wk.zpart, zs, wk.rcnt, wk.zs_pairs);
    prof_end(kKBucketEmbed, s);
    prof_begin(kKBucketEmbedFix, s);
    if (many)
        hipLaunchKernelGGL(bucket_embed_fix<kFixThreadsMany>, dim3(nm), dim3(kFixThreadsMany), lds, s, b, wk.multi,
                           wk.bmeta, p.sb, wk.info, wk.srow, wk.zpart, zs, wk.rcnt, wk.zs_pairs);
    else
        hipLaunchKernelGGL(bucket_embed_fix<kFixThreads>, dim3(nm), dim3(kFixThreads), lds, s, b, wk.multi, wk.bmeta,
                           p.sb, wk.info, wk.srow, wk.zpart, zs, wk.rcnt, wk.zs_pairs);
    prof_end(kKBucketEmbedFix, s);
}

hipError_t launch_bucket_embed(const Batch &b, const Plan &p, const Work &wk, hipStream_t s, int mode, bool sums) {
    // rows of the bucketed entries: after a pass B packed into the column words, else pass
    // A's key (u16 when the row's low bits fit, else the whole row)
    const bool with_b = p.s2 > 0;
    const bool key16 = with_b || p.sb + p.s2 <= 16;
    const void *key = with_b ? (const void *)wk.tkey : (const void *)wk.akey;
    const unsigned nblk = (unsigned)((p.B + 1023) / 1024);
    if (!with_b) {  // (after a pass B its scan has formed the block totals and its scatter the table)
        if (nblk > 1) {  // (one block of buckets forms its own totals)
            prof_begin(kKBucketPartCount, s);
            hipLaunchKernelGGL(bucket_part_count, dim3(nblk), dim3(1024), 0, s, b, wk.bstart, p.B, p.sb, wk.ptot,
                               (const int *)nullptr);
            prof_end(kKBucketPartCount, s);
        }
        prof_begin(kKBucketPartFill, s);
        hipLaunchKernelGGL(bucket_part_fill, dim3(nblk), dim3(256), 0, s, b, wk.bstart, p.B, p.sb,
                           nblk > 1 ? (const int *)wk.ptot : nullptr, wk.part, wk.multi, wk.bmeta,
                           (const int *)nullptr);
        prof_end(kKBucketPartFill, s);
    }
    if (key16 && p.weighted) launch_bucket_sums<uint16_t, true>(b, p, wk, (const uint16_t *)key, s, mode, sums);
    else if (key16) launch_bucket_sums<uint16_t, false>(b, p, wk, (const uint16_t *)key, s, mode, sums);
    else if (p.weighted) launch_bucket_sums<int, true>(b, p, wk, (const int *)key, s, mode, sums);
    else launch_bucket_sums<int, false>(b, p, wk, (const int *)key, s, mode, sums);
    return hipGetLastError();
}

}  // namespace gee
