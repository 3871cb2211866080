// gee_csr.hip - edge list -> CSR on the device (Section 3 layout), deterministic.
//
// The adjacency entries of an edge list are the rows themselves and, under
// symmetrization, their mirrors: virtual entry 2e is (src_e -> dst_e) and 2e+1 is
// (dst_e -> src_e), the latter absent for a self-loop. The CSR is a stable sort of
// that sequence by row index, done as a two-level most-significant-digit partition:
//
//   pass 1  partition by bucket = row >> sb (at most 4096 buckets):
//           p1_hist       per-tile bucket histograms (LDS), written bucket-major
//           p1_scan       exclusive scan of each bucket's tile counts
//           p1_totals     exclusive scan of bucket totals -> bucket starts, M
//           p1_scatter    stable in-tile rank per bucket -> partitioned entries
//   pass 2  one workgroup per bucket: count rows (LDS), scan -> row_ptr, stable rank by
//           row within the bucket -> col/val at their final CSR slots. When the
//           embedding follows, the same workgroup also reads back its rows to form the
//           degrees, the per-node coefficients and the embed wavefront ownership.
//
// Stable ranking never uses global atomics: within a 64-wide wavefront, lanes with
// the same digit are found by ballots over the digit bits; across the wavefronts of
// a round a small per-wave count table in LDS gives the offset; the running counts per
// digit live in LDS for the whole tile/bucket, so the order of equal digits is the
// input order.
#include "gee_internal.h"

namespace gee {

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

// ----------------------------------------------------------------------------- pass 1

__global__ __launch_bounds__(256) void p1_hist(const int *__restrict__ src, const int *__restrict__ dst,
                                               int64_t E, int N, int sym, int sb, int B, int tile,
                                               int64_t T1, int *__restrict__ ghist, unsigned *status) {
    extern __shared__ int hist[];
    for (int b = threadIdx.x; b < B; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    const int64_t t = blockIdx.x;
    const int64_t V = sym ? 2 * E : E;
    const int64_t v0 = t * tile;
    const int64_t v1 = min(v0 + tile, V);
    bool bad = false;
    const int64_t e0 = sym ? v0 / 2 : v0;
    const int64_t e1 = sym ? (v1 + 1) / 2 : v1;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const int s = src[e], d = dst[e];
        if ((unsigned)s < (unsigned)N && (unsigned)d < (unsigned)N) {
            atomicAdd(&hist[s >> sb], 1);
            if (sym && s != d) atomicAdd(&hist[d >> sb], 1);
        } else {
            bad = true;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) raise_error(status, kErrIndex);
    for (int b = threadIdx.x; b < B; b += blockDim.x) ghist[(int64_t)b * T1 + t] = hist[b];
}

// One workgroup per bucket: exclusive scan over the bucket's tile counts.
__global__ __launch_bounds__(256) void p1_scan(int *__restrict__ ghist, int64_t T1,
                                               int *__restrict__ btot) {
    __shared__ int wsum[4];
    int *row = ghist + (int64_t)blockIdx.x * T1;
    int carry = 0;
    constexpr int IPT = 8;
    for (int64_t c = 0; c < T1; c += 256 * IPT) {
        int vals[IPT];
        int s = 0;
        const int64_t lo = c + (int64_t)threadIdx.x * IPT;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            vals[i] = (lo + i < T1) ? row[lo + i] : 0;
            s += vals[i];
        }
        int total;
        int base = block_excl_scan256(s, wsum, total) + carry;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if (lo + i < T1) row[lo + i] = base;
            base += vals[i];
        }
        carry += total;
    }
    if (threadIdx.x == 0) btot[blockIdx.x] = carry;
}

// Single workgroup: bucket starts, total entry count M and the embed wavefront count.
__global__ __launch_bounds__(256) void p1_totals(const int *__restrict__ btot, int B,
                                                 int *__restrict__ bstart, int *__restrict__ meta,
                                                 int WE) {
    __shared__ int wsum[4];
    const int per = (B + 255) / 256;
    const int lo = threadIdx.x * per;
    int s = 0;
    for (int i = 0; i < per; ++i)
        if (lo + i < B) s += btot[lo + i];
    int total;
    int base = block_excl_scan256(s, wsum, total);
    for (int i = 0; i < per; ++i)
        if (lo + i < B) {
            bstart[lo + i] = base;
            base += btot[lo + i];
        }
    if (threadIdx.x == 0) {
        bstart[B] = total;
        meta[0] = total;
        meta[1] = total > 0 ? (int)(((int64_t)total + WE - 1) / WE) : 1;
    }
}

__global__ __launch_bounds__(256) void p1_scatter(const int *__restrict__ src, const int *__restrict__ dst,
                                                  const float *__restrict__ w, int64_t E, int N, int sym,
                                                  int sb, int B, int nbits, int tile, int64_t T1,
                                                  const int *__restrict__ ghist,
                                                  const int *__restrict__ bstart,
                                                  uint16_t *__restrict__ tkey, int *__restrict__ tcol,
                                                  float *__restrict__ tval, unsigned *status) {
    extern __shared__ int smem_i[];
    int *run = smem_i;                                        // [B]
    unsigned char *tab = reinterpret_cast<unsigned char *>(run + B);  // [4][B]
    const int64_t t = blockIdx.x;
    for (int b = threadIdx.x; b < B; b += blockDim.x) run[b] = bstart[b] + ghist[(int64_t)b * T1 + t];
    for (int i = threadIdx.x; i < 4 * B; i += blockDim.x) tab[i] = 0;
    __syncthreads();
    const int64_t V = sym ? 2 * E : E;
    const int64_t v0 = t * tile;
    const int64_t v1 = min(v0 + tile, V);
    const int lowmask = (1 << sb) - 1;
    bool badw = false;
    for (int64_t vb = v0; vb < v1; vb += 256) {
        const int64_t v = vb + threadIdx.x;
        bool valid = false;
        int key = 0, cl = 0;
        float val = 1.0f;
        if (v < v1) {
            const int64_t e = sym ? (v >> 1) : v;
            const int side = sym ? (int)(v & 1) : 0;
            const int s = src[e], d = dst[e];
            valid = (unsigned)s < (unsigned)N && (unsigned)d < (unsigned)N && (side == 0 || s != d);
            key = side ? d : s;
            cl = side ? s : d;
            if (w) {
                val = w[e];
                if (side == 0 && !isfinite(val)) badw = true;
            }
        }
        const int digit = valid ? (key >> sb) : 0;
        const int pos = block_rank4(digit, valid, nbits, tab, run, B);
        if (valid) {
            tkey[pos] = (uint16_t)(key & lowmask);
            tcol[pos] = cl;
            if (tval) tval[pos] = val;
        }
    }
    if (__syncthreads_or(badw) && threadIdx.x == 0) raise_error(status, kErrWeight);
}

// ----------------------------------------------------------------------------- pass 2

__global__ __launch_bounds__(256) void p2_bucket(const uint16_t *__restrict__ tkey,
                                                 const int *__restrict__ tcol,
                                                 const float *__restrict__ tval,
                                                 const int *__restrict__ bstart, int B, int sb, int N,
                                                 int *__restrict__ rp, int *__restrict__ col,
                                                 float *__restrict__ val) {
    extern __shared__ int smem_i[];
    __shared__ int wsum[4];
    const int R = 1 << sb;
    int *run = smem_i;                                        // [R]
    unsigned char *tab = reinterpret_cast<unsigned char *>(run + R);  // [4][R]
    const int b = blockIdx.x;
    const int r0 = b << sb;
    const int Rb = min(R, N - r0);
    const int e0 = bstart[b], e1 = bstart[b + 1];
    // A: rows' entry counts
    for (int i = threadIdx.x; i < R; i += blockDim.x) run[i] = 0;
    for (int i = threadIdx.x; i < 4 * R; i += blockDim.x) tab[i] = 0;
    __syncthreads();
    for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) atomicAdd(&run[tkey[e]], 1);
    __syncthreads();
    // B: row offsets -> row_ptr
    block_excl_scan_lds(run, R, wsum);
    for (int i = threadIdx.x; i < Rb; i += blockDim.x) rp[r0 + i] = e0 + run[i];
    if (b == B - 1 && threadIdx.x == 0) rp[N] = e1;
    __syncthreads();
    // C: stable placement by row within the bucket
    for (int eb = e0; eb < e1; eb += 256) {
        const int e = eb + threadIdx.x;
        const bool valid = e < e1;
        const int digit = valid ? (int)tkey[e] : 0;
        const int pos = block_rank4(digit, valid, sb, tab, run, R);
        if (valid) {
            col[e0 + pos] = tcol[e];
            if (val) val[e0 + pos] = tval[e];
        }
    }
}

// ----------------------------------------------------------------------------- launch

hipError_t launch_csr_build(const int *src, const int *dst, const float *w, const Plan &p,
                            const Work &wk, unsigned *status, hipStream_t s) {
    const int sym = (p.flags & kSym) ? 1 : 0;
    int nbits = 0;
    while ((1 << nbits) < p.B) ++nbits;
    prof_begin(kKP1Hist, s);
    hipLaunchKernelGGL(p1_hist, dim3((unsigned)p.T1), dim3(256), p.B * sizeof(int), s, src, dst, p.E,
                       p.N, sym, p.sb, p.B, p.tile, p.T1, wk.ghist, status);
    prof_end(kKP1Hist, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    prof_begin(kKP1Scan, s);
    hipLaunchKernelGGL(p1_scan, dim3(p.B), dim3(256), 0, s, wk.ghist, p.T1, wk.btot);
    prof_end(kKP1Scan, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKP1Totals, s);
    hipLaunchKernelGGL(p1_totals, dim3(1), dim3(256), 0, s, wk.btot, p.B, wk.bstart, wk.meta, p.WE);
    prof_end(kKP1Totals, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKP1Scatter, s);
    hipLaunchKernelGGL(p1_scatter, dim3((unsigned)p.T1), dim3(256), p.B * 8, s, src, dst,
                       p.weighted ? w : nullptr, p.E, p.N, sym, p.sb, p.B, nbits, p.tile, p.T1,
                       wk.ghist, wk.bstart, wk.tkey, wk.tcol, p.weighted ? wk.tval : nullptr, status);
    prof_end(kKP1Scatter, s);
    return hipGetLastError();
}

hipError_t launch_csr_pass2(const Plan &p, const Work &wk, unsigned *status, hipStream_t s) {
    (void)status;
    const int R = 1 << p.sb;
    prof_begin(kKP2Bucket, s);
    hipLaunchKernelGGL(p2_bucket, dim3(p.B), dim3(256), R * 8, s, wk.tkey, wk.tcol,
                       p.weighted ? wk.tval : nullptr, wk.bstart, p.B, p.sb, p.N, wk.rp, wk.col,
                       p.weighted ? wk.val : nullptr);
    prof_end(kKP2Bucket, s);
    return hipGetLastError();
}

}  // namespace gee
