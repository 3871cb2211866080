// gee_zsparse.hip - the embedding in sparse storage: Z's non-zero entries kept row by row in
// the CSR layout of Section 3 (index pointers of N + 1 entries, then the class index and the
// value of each non-zero entry, row after row, classes increasing), as the paper stores the
// embedding matrix. On the bucket path (a single graph of at most 2^22 rows) the class-scatter
// kernels stage each bucket's non-zero (class, value) pairs, row-major, from its first row's
// place in a dense Z, and each row's count; zs_tile_sum, zs_scan and zs_place then form
// row_ptr and copy each bucket's run to its place. Otherwise Z is dense float32 N x K on
// entry and is compacted as below.
//
// Rows are taken in tiles of kZT; inside a tile, groups of L lanes (the power of two at or
// above min(K, 64)) take one row each, a lane the columns sub and sub + L.
//   zs_count  per tile: each row's number of non-zero entries (kept), and the tile's total
//   zs_scan   one workgroup: exclusive scan of the tile counts, total into row_ptr[N]
//   zs_write  per tile: the rows' counts scanned in LDS, then row_ptr and the compacted
//             (class, value) pairs at each lane's rank within its row (one pass over Z);
//             zs_flat does the same over Z as a flat stream when K >= 4
#include "gee_internal.h"

namespace gee {
namespace {

constexpr int kZT = 256;   // rows per tile
constexpr int kZB = 256;   // threads per workgroup of the tile kernels
#ifndef GEE_ZS_FLAT
#define GEE_ZS_FLAT 1
#endif

// Bits of `m` that belong to this lane's group of L lanes, shifted down to bit 0.
template <int L>
__device__ __forceinline__ uint64_t group_bits(uint64_t m, int lane) {
    if constexpr (L == 64) {
        return m;
    } else {
        return (m >> (lane & ~(L - 1))) & ((1ull << L) - 1);
    }
}

// Loads the lane's two columns of row i (zero past K or for i >= N) and returns the row's
// non-zero masks over its group (bit sub: column sub, and column sub + L).
template <int L>
__device__ __forceinline__ void row_nonzeros(const float *__restrict__ Z, int64_t i, int N, int K, int sub,
                                            int lane, float &z0, float &z1, uint64_t &m0, uint64_t &m1) {
    z0 = 0.0f;
    z1 = 0.0f;
    if (i < N) {
        const float *row = Z + i * K;
        if (sub < K) z0 = row[sub];
        if (sub + L < K) z1 = row[sub + L];
    }
    m0 = group_bits<L>(ballot(z0 != 0.0f), lane);
    m1 = group_bits<L>(ballot(z1 != 0.0f), lane);
}

template <int L>
__global__ __launch_bounds__(kZB) void zs_count(const float *__restrict__ Z, int N, int K, int *__restrict__ row_cnt,
                                              int *__restrict__ tile_tot) {
    __shared__ int wsum[kZB / 64];
    const int lane = lane_id(), sub = threadIdx.x % L, grp = threadIdx.x / L;
    constexpr int G = kZB / L;
    const int64_t base = (int64_t)blockIdx.x * kZT;
    int n = 0;
#pragma unroll 4
    for (int r = grp; r < kZT; r += G) {  // the same trip count for every group of a wavefront
        float z0, z1;
        uint64_t m0, m1;
        row_nonzeros<L>(Z, base + r, N, K, sub, lane, z0, z1, m0, m1);
        const int c = __popcll(m0) + __popcll(m1);
        if (sub == 0) {
            n += c;
            if (base + r < N) row_cnt[base + r] = c;
        }
    }
    int tot = 0;
    (void)block_excl_scan<kZB>(n, wsum, tot);
    if (threadIdx.x == 0) tile_tot[blockIdx.x] = tot;
}

// Per tile, with the row counts already known (written by the class-scatter kernels): the
// tile's total alone (4 bytes a row instead of a pass over Z).
__global__ __launch_bounds__(kZB) void zs_tile_sum(const int *__restrict__ row_cnt, int N, int *__restrict__ tile_tot) {
    __shared__ int wsum[kZB / 64];
    const int64_t base = (int64_t)blockIdx.x * kZT;
    int n = 0;
    for (int r = threadIdx.x; r < kZT; r += kZB) n += base + r < N ? row_cnt[base + r] : 0;
    int tot = 0;
    (void)block_excl_scan<kZB>(n, wsum, tot);
    if (threadIdx.x == 0) tile_tot[blockIdx.x] = tot;
}

// One workgroup of 1024 threads: tile_tot becomes exclusive offsets; the total is row_ptr[N].
__global__ __launch_bounds__(1024) void zs_scan(int *__restrict__ tile_tot, int T, int *__restrict__ row_ptr, int N) {
    __shared__ int wsum[1024 / 64];
    int carry = 0;
    for (int b0 = 0; b0 < T; b0 += 1024) {
        const int b = b0 + (int)threadIdx.x;
        const int v = b < T ? tile_tot[b] : 0;
        int tot = 0;
        const int x = block_excl_scan<1024>(v, wsum, tot);
        if (b < T) tile_tot[b] = carry + x;
        carry += tot;
    }
    if (threadIdx.x == 0) row_ptr[N] = carry;
}

template <int L>
__global__ __launch_bounds__(kZB) void zs_write(const float *__restrict__ Z, int N, int K,
                                              const int *__restrict__ row_cnt, const int *__restrict__ tile_off,
                                              int *__restrict__ row_ptr, int *__restrict__ col,
                                              float *__restrict__ val, int64_t cap) {
    __shared__ int cnt[kZT];
    __shared__ int wsum[kZB / 64];
    const int lane = lane_id(), sub = threadIdx.x % L, grp = threadIdx.x / L;
    constexpr int G = kZB / L;
    const int64_t base = (int64_t)blockIdx.x * kZT;
    for (int r = threadIdx.x; r < kZT; r += kZB) cnt[r] = base + r < N ? row_cnt[base + r] : 0;
    __syncthreads();
    // exclusive scan of the tile's kZT row counts: kZT / kZB consecutive rows per thread
    constexpr int PER = kZT / kZB;
    int c[PER], s = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        c[q] = cnt[threadIdx.x * PER + q];
        s += c[q];
    }
    int tot = 0;
    int x = block_excl_scan<kZB>(s, wsum, tot);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        cnt[threadIdx.x * PER + q] = x;
        x += c[q];
    }
    __syncthreads();
    const int64_t off = tile_off[blockIdx.x];
#pragma unroll 4
    for (int r = grp; r < kZT; r += G) {
        const int64_t i = base + r;
        float z0, z1;
        uint64_t m0, m1;
        row_nonzeros<L>(Z, i, N, K, sub, lane, z0, z1, m0, m1);
        if (i >= N) continue;
        const int64_t start = off + cnt[r];
        if (sub == 0) row_ptr[i] = (int)start;
        const uint64_t below = (1ull << sub) - 1;  // sub < L <= 64; sub = 63 gives 2^63 - 1
        if (z0 != 0.0f) {
            const int64_t p = start + __popcll(m0 & below);
            if (p < cap) {
                col[p] = sub;
                val[p] = z0;
            }
        }
        if (z1 != 0.0f) {
            const int64_t p = start + __popcll(m0) + __popcll(m1 & below);
            if (p < cap) {
                col[p] = sub + L;
                val[p] = z1;
            }
        }
    }
}

// zs_write over Z as one flat row-major stream (K >= 4, Z 16-byte aligned): the output is Z's
// non-zero values in row-major order, so an entry's place is the tile's offset plus the
// number of non-zeros before it in the tile. Wavefront w takes the tile's rows 64w ..
// 64w + 63 (a contiguous range of floats, whose first place comes from the scanned row
// counts), four consecutive floats per lane per 16-byte load, and ranks each non-zero by
// four ballots; its class is its index within the row. Same output as zs_write.
__global__ __launch_bounds__(kZB) void zs_flat(const float *__restrict__ Z, int N, int K,
                                             const int *__restrict__ row_cnt, const int *__restrict__ tile_off,
                                             int *__restrict__ row_ptr, int *__restrict__ col,
                                             float *__restrict__ val, int64_t cap) {
    static_assert(kZT == kZB && kZB == 256, "one thread per row of the tile, four wavefronts of 64 rows");
    __shared__ int cnt[kZT];
    __shared__ int wsum[kZB / 64];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kZT;
    const int r = threadIdx.x;
    const int c = base + r < N ? row_cnt[base + r] : 0;
    int tot = 0;
    const int x = block_excl_scan<kZB>(c, wsum, tot);
    cnt[r] = x;
    const int64_t off = tile_off[blockIdx.x];
    if (base + r < N) row_ptr[base + r] = (int)(off + x);
    __syncthreads();
    const int64_t r0 = base + 64 * wv;
    const int nrows = (int)min((int64_t)64, (int64_t)N - r0);
    if (nrows <= 0) return;
    const int64_t f0 = r0 * K;                  // the wavefront's first float
    const int nf = nrows * K;                   // its floats
    const __amdgpu_buffer_rsrc_t rz = buffer_rsrc(Z + f0, (int64_t)nf * 4);
    int64_t p = off + cnt[64 * wv];             // place of its first non-zero
    const uint64_t below = (1ull << lane) - 1;  // lane < 64: lane 63 gives 2^63 - 1
    for (int lf = 4 * lane, c0 = 0; c0 < nf; c0 += 256, lf += 256) {
        float zz[4];
        if (lf + 4 <= nf) {
            const float4 z4 = buf_f4(rz, (uint32_t)lf * 4u);
            zz[0] = z4.x;
            zz[1] = z4.y;
            zz[2] = z4.z;
            zz[3] = z4.w;
        } else {  // the range's last floats, one by one (0 past it)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                zz[j] = lf + j < nf ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rz, (uint32_t)(lf + j) * 4u, 0, 0))
                                    : 0.0f;
        }
        uint64_t m[4];
        int before = 0, mine = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            m[j] = ballot(zz[j] != 0.0f);
            before += __popcll(m[j] & below);
        }
        int cls = lf % K;  // the class of the lane's first float
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (zz[j] != 0.0f) {
                const int64_t q = p + before + mine;
                if (q < cap) {
                    col[q] = cls;
                    val[q] = zz[j];
                }
                ++mine;
            }
            if (++cls == K) cls = 0;
        }
        p += __popcll(m[0]) + __popcll(m[1]) + __popcll(m[2]) + __popcll(m[3]);
    }
}

// Staged sparse Z: the class scatter has left each bucket's non-zero pairs, row-major, from
// its first row r0's place r0 K of the (class, value bits) pairs zp, and each row's count in
// row_cnt. Per tile of
// kZT rows (whole buckets: R divides kZT): the rows' counts scanned into row_ptr, then
// wavefront w copies the runs of the tile's buckets w, w + 4, ... to their places, 64 pairs
// per step.
__global__ __launch_bounds__(kZB) void zs_place(int N, int K, int sb, const int2 *__restrict__ zp,
                                              const int *__restrict__ row_cnt, const int *__restrict__ tile_off,
                                              int *__restrict__ row_ptr, int *__restrict__ col,
                                              float *__restrict__ val, int64_t cap) {
    static_assert(kZT == kZB, "one thread per row of the tile");
    __shared__ int cnt[kZT + 1];
    __shared__ int wsum[kZB / 64];
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kZT;
    const int r = threadIdx.x;
    const int c = base + r < N ? row_cnt[base + r] : 0;
    int tot = 0;
    const int x = block_excl_scan<kZB>(c, wsum, tot);
    cnt[r] = x;
    if (r == 0) cnt[kZT] = tot;
    const int64_t off = tile_off[blockIdx.x];
    if (base + r < N) row_ptr[base + r] = (int)(off + x);
    __syncthreads();
    const int R = 1 << sb;
    const int nb = (int)((min((int64_t)kZT, (int64_t)N - base) + R - 1) >> sb);  // the tile's buckets
    for (int j = wv; j < nb; j += kZB / 64) {
        const int bk = (int)(base >> sb) + j;
        const int n = cnt[min((j + 1) << sb, kZT)] - cnt[j << sb];
        const int64_t src = ((int64_t)bk << sb) * K;
        const int64_t dst = off + cnt[j << sb];
        for (int i = lane; i < n; i += 64) {
            const int64_t q = dst + i;
            if (q < cap) {
                const int2 pr = zp[src + i];
                col[q] = pr.x;
                val[q] = __int_as_float(pr.y);
            }
        }
    }
}

template <int L>
hipError_t launch_zs(const float *Z, int N, int K, int T, int *tile, int *rcnt, int *row_ptr, int *col, float *val,
                     int64_t cap, bool counts_given, hipStream_t s) {
    const int kid = counts_given ? kKZsTileSum : kKZsCount;
    prof_begin(kid, s);
    if (counts_given)
        hipLaunchKernelGGL(zs_tile_sum, dim3((unsigned)T), dim3(kZB), 0, s, rcnt, N, tile);
    else
        hipLaunchKernelGGL(zs_count<L>, dim3((unsigned)T), dim3(kZB), 0, s, Z, N, K, rcnt, tile);
    prof_end(kid, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(zs_scan, dim3(1), dim3(1024), 0, s, tile, T, row_ptr, N);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKZsWrite, s);
    if (GEE_ZS_FLAT && K >= 4 && (reinterpret_cast<uintptr_t>(Z) & 15) == 0)
        hipLaunchKernelGGL(zs_flat, dim3((unsigned)T), dim3(kZB), 0, s, Z, N, K, rcnt, tile, row_ptr, col, val, cap);
    else
        hipLaunchKernelGGL(zs_write<L>, dim3((unsigned)T), dim3(kZB), 0, s, Z, N, K, rcnt, tile, row_ptr, col, val,
                           cap);
    prof_end(kKZsWrite, s);
    return hipGetLastError();
}

}  // namespace

int zsparse_tiles(int N) { return (N + kZT - 1) / kZT; }

hipError_t launch_zsparse_staged(int N, int K, int sb, const int2 *zs_pairs, int *tile, int *rcnt, int *row_ptr,
                                 int *col, float *val, int64_t cap, hipStream_t s) {
    if (sb < 0 || (1 << sb) > kZT) return hipErrorInvalidValue;  // (bucket-path buckets have 32 or 64 rows)
    const int T = zsparse_tiles(N);
    prof_begin(kKZsTileSum, s);
    hipLaunchKernelGGL(zs_tile_sum, dim3((unsigned)T), dim3(kZB), 0, s, rcnt, N, tile);
    prof_end(kKZsTileSum, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(zs_scan, dim3(1), dim3(1024), 0, s, tile, T, row_ptr, N);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKZsWrite, s);
    hipLaunchKernelGGL(zs_place, dim3((unsigned)T), dim3(kZB), 0, s, N, K, sb, zs_pairs, rcnt, tile, row_ptr, col,
                       val, cap);
    prof_end(kKZsWrite, s);
    return hipGetLastError();
}

hipError_t launch_zsparse(const float *Z, int N, int K, int *tile, int *rcnt, int *row_ptr, int *col, float *val,
                          int64_t cap, bool counts_given, hipStream_t s) {
    const int T = zsparse_tiles(N);
    const int L = K > 32 ? 64 : K > 16 ? 32 : K > 8 ? 16 : K > 4 ? 8 : K > 2 ? 4 : K > 1 ? 2 : 1;
    switch (L) {
        case 64: return launch_zs<64>(Z, N, K, T, tile, rcnt, row_ptr, col, val, cap, counts_given, s);
        case 32: return launch_zs<32>(Z, N, K, T, tile, rcnt, row_ptr, col, val, cap, counts_given, s);
        case 16: return launch_zs<16>(Z, N, K, T, tile, rcnt, row_ptr, col, val, cap, counts_given, s);
        case 8: return launch_zs<8>(Z, N, K, T, tile, rcnt, row_ptr, col, val, cap, counts_given, s);
        case 4: return launch_zs<4>(Z, N, K, T, tile, rcnt, row_ptr, col, val, cap, counts_given, s);
        case 2: return launch_zs<2>(Z, N, K, T, tile, rcnt, row_ptr, col, val, cap, counts_given, s);
        default: return launch_zs<1>(Z, N, K, T, tile, rcnt, row_ptr, col, val, cap, counts_given, s);
    }
}

}  // namespace gee
