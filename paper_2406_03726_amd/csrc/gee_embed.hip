// gee_embed.hip - Z = A W with the Table 1 options, from a CSR (Eq. 1, Section 2).
//
// For row i with D^-1/2 factor s_i (1 without the Laplacian) and per-node
// coefficient c_j = s_j / n_{y_j} (0 for an unknown label):
//     Z[i, k] = s_i * ( sum_{e in row i, y_col(e) = k} val_e * c_col(e)  +  [diag, k = y_i] c_i )
// then, with correlation, row i is divided by its 2-norm. This is Eq. 1 with A
// replaced by D^-1/2 (A + I) D^-1/2: the rescale e_ij s_i s_j is split into the
// gathered c_j and the per-row s_i, and the identity's entry is the c_i term.
//
// Work split (MI355X, 64-wide wavefronts, HBM-bound, no MFMA since W is one-hot):
//   * embed_rows: wavefront w processes the CSR entries [w*WE, (w+1)*WE) in windows
//     of 64 (coalesced col/val loads, one 8-byte gather of {c_j, y_j} per entry), so
//     every wavefront does the same work whatever the degree distribution.
//     Rows get slots of an LDS ring acc[k][slot] (64 slots x K classes per wave).
//     Lanes adding to the same (slot, class) are found by ballots over the key bits
//     and take turns in lane order, so each LDS add instruction touches distinct
//     addresses and the summation order is fixed: results are bitwise reproducible.
//     A row that ends inside the wavefront is finished there (diagonal term, s_i,
//     correlation) and written with coalesced stores; a row cut by wavefront
//     boundaries leaves raw partial sums (head/tail) for embed_fixup.
//   * embed_fixup: adds the partials of each cut row in wavefront order and finishes it.
//   * fill_empty: rows without entries (zero, or the diagonal term alone).
#include "gee_internal.h"

#include <climits>

namespace gee {

// ----------------------------------------------------------------------------- prep

// Degrees, coefficients and wavefront ownership for a caller-provided CSR.
// One 256-thread workgroup per 256 rows.
__global__ __launch_bounds__(256) void prep_from_csr(const int *__restrict__ rp,
                                                     const float *__restrict__ val, int N,
                                                     const int *__restrict__ labels, int K,
                                                     const float *__restrict__ inv_n, unsigned flags,
                                                     float2 *__restrict__ info, float *__restrict__ srow,
                                                     int *__restrict__ fown, int M, int NW, int WE,
                                                     unsigned *status) {
    __shared__ float degs[256];
    const int r0 = blockIdx.x * 256;
    const int lane = lane_id();
    const bool lap = flags & kLap, diag = flags & kDiag;
    bool bad = false;
    if (lap) {
        if (val) {
            for (int i = threadIdx.x >> 6; i < 256; i += 4) {
                const int r = r0 + i;
                float s = 0.0f;
                if (r < N) {
                    const int lo = max(0, min(rp[r], M)), hi = max(lo, min(rp[r + 1], M));
                    for (int e = lo + lane; e < hi; e += 64) s += val[e];
                }
                s = wave_sum(s);
                if (lane == 0) degs[i] = s;
            }
        } else {
            const int r = r0 + threadIdx.x;
            if (r < N) degs[threadIdx.x] = (float)(rp[r + 1] - rp[r]);
        }
    }
    __syncthreads();
    const int r = r0 + threadIdx.x;
    if (r < N) {
        const int lo = rp[r], hi = rp[r + 1];
        if (lo > hi || lo < 0 || hi > M) bad = true;
        if (r == 0 && lo != 0) bad = true;
        if (r == N - 1 && hi != M) bad = true;
        int y = labels[r];
        if (y < 0 || y >= K) y = -1;
        float s = 1.0f;
        if (lap) {
            const float d = degs[threadIdx.x] + (diag ? 1.0f : 0.0f);
            s = d > 0.0f ? 1.0f / sqrtf(d) : 0.0f;
            srow[r] = s;
        }
        info[r] = make_float2(y >= 0 ? s * inv_n[y] : 0.0f, __int_as_float(y));
        // wavefronts w with rp[r] < w*WE <= rp[r+1] start owning at row r+1
        const int64_t wa = (int64_t)max(lo, 0) / WE + 1;
        const int64_t wb = min((int64_t)min(max(hi, 0), M) / WE, (int64_t)NW - 1);
        for (int64_t ww = wa; ww <= wb; ++ww) fown[ww] = r + 1;
        if (r == 0) {
            fown[0] = 0;
            fown[NW] = N;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) raise_error(status, kErrCsr);
}

// ----------------------------------------------------------------------------- empty rows

__global__ __launch_bounds__(256) void fill_empty(const int *__restrict__ rp, int N, int K,
                                                  unsigned flags, const float2 *__restrict__ info,
                                                  const float *__restrict__ srow,
                                                  float *__restrict__ Z) {
    __shared__ int emp[256];
    __shared__ float dv[256];
    __shared__ int yy[256];
    const int r0 = blockIdx.x * 256;
    const int r = r0 + threadIdx.x;
    const bool lap = flags & kLap, diag = flags & kDiag, cor = flags & kCor;
    int e = 0;
    float d = 0.0f;
    int y = -1;
    if (r < N) {
        e = rp[r] == rp[r + 1];
        if (e && diag) {
            const float2 inf = info[r];
            y = __float_as_int(inf.y);
            d = inf.x * (lap ? srow[r] : 1.0f);
            if (cor) d = d != 0.0f ? 1.0f : 0.0f;
        }
    }
    emp[threadIdx.x] = e;
    dv[threadIdx.x] = d;
    yy[threadIdx.x] = y;
    if (!__syncthreads_or(e)) return;
    const int nr = min(256, N - r0);
    const int64_t base = (int64_t)r0 * K;
    for (int idx = threadIdx.x; idx < nr * K; idx += 256) {
        const int i = idx / K, k = idx - i * K;
        if (emp[i]) Z[base + idx] = (k == yy[i]) ? dv[i] : 0.0f;
    }
}

// ----------------------------------------------------------------------------- finish a row

// Finish row r from raw class sums held one class per lane (K <= 64) and store it.
__device__ __forceinline__ void finish_store_64(float v, int lane, int r, int K, bool diag, bool lap,
                                                bool cor, const float2 *__restrict__ info,
                                                const float *__restrict__ srow, float *__restrict__ Z) {
    const float2 inf = info[r];
    const int y = __float_as_int(inf.y);
    if (diag && lane == y) v += inf.x;
    if (lap) v *= srow[r];
    if (cor) {
        const float ss = wave_sum(v * v);
        if (ss > 0.0f) v *= 1.0f / sqrtf(ss);
    }
    if (lane < K) Z[(int64_t)r * K + lane] = v;
}

// K in (64, 128]: two classes per lane (lane and lane + 64).
__device__ __forceinline__ void finish_store_128(float v0, float v1, int lane, int r, int K, bool diag,
                                                 bool lap, bool cor, const float2 *__restrict__ info,
                                                 const float *__restrict__ srow,
                                                 float *__restrict__ Z) {
    const float2 inf = info[r];
    const int y = __float_as_int(inf.y);
    if (diag && lane == y) v0 += inf.x;
    if (diag && lane + 64 == y) v1 += inf.x;
    if (lap) {
        const float s = srow[r];
        v0 *= s;
        v1 *= s;
    }
    if (cor) {
        const float ss = wave_sum(v0 * v0 + v1 * v1);
        if (ss > 0.0f) {
            const float sc = 1.0f / sqrtf(ss);
            v0 *= sc;
            v1 *= sc;
        }
    }
    Z[(int64_t)r * K + lane] = v0;
    if (lane + 64 < K) Z[(int64_t)r * K + lane + 64] = v1;
}

// ----------------------------------------------------------------------------- main kernel

template <bool WEIGHTED, bool WIDE>
__global__ __launch_bounds__(256) void embed_rows(const int *__restrict__ rp, const int *__restrict__ col,
                                                  const float *__restrict__ val,
                                                  const float2 *__restrict__ info,
                                                  const float *__restrict__ srow,
                                                  const int *__restrict__ fown,
                                                  const int *__restrict__ meta, int N, int K, int kbits,
                                                  int WE, unsigned flags, float *__restrict__ Z,
                                                  float *__restrict__ headp, float *__restrict__ tailp,
                                                  int *__restrict__ split, unsigned *status) {
    extern __shared__ float smem_f[];
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int M = meta[0], NW = meta[1];
    const int w = blockIdx.x * wpb + wib;
    if (w >= NW) return;  // whole wavefront leaves; no workgroup barrier is used below
    const bool diag = flags & kDiag, lap = flags & kLap, cor = flags & kCor;

    float *acc = smem_f + (size_t)wib * (K * 64 + 128);  // [K][64]
    int *own = reinterpret_cast<int *>(acc + K * 64);    // [64]
    int *slot_row = own + 64;                            // [64]
    for (int k = 0; k < K; ++k) acc[k * 64 + lane] = 0.0f;
    own[lane] = -1;

    const int a = w * WE;
    const int b = min(a + WE, M);
    const int r_lo = min(max(fown[w], 0), N);
    const int head_row = (rp[r_lo] > a) ? r_lo - 1 : -1;
    int cur_row = r_lo - 1;
    int next_row = r_lo;
    int cur_slot = 63;
    slot_row[63] = cur_row;
    bool cont = false;
    int row_last = cur_row, slot_last = cur_slot;
    wave_lds_fence();

    for (int p = a; p < b; p += 64) {
        const int nvalid = min(64, b - p);
        const bool valid = lane < nvalid;
        const int e = p + lane;
        const int j = valid ? col[e] : 0;
        float v = 1.0f;
        if (WEIGHTED && valid) v = val[e];

        // Rows starting inside this window: lane q of `own` receives the last row whose
        // first entry is p + q (empty rows share a start with the next row).
        int next_start;
        for (;;) {
            const int r = next_row + lane;
            const int st = (r <= N) ? rp[r] : INT_MAX;
            // (r < N and st >= p always hold for a well-formed CSR; they keep a
            // malformed caller CSR from producing rows or LDS slots out of range)
            const bool fl = r < N && st >= p && st < p + nvalid;
            const uint64_t fm = ballot(fl);
            if (fl) atomicMax(&own[st - p], r);
            const int cnt = __popcll(fm);
            if (cnt < 64) {
                next_start = __shfl(st, cnt, 64);
                next_row += cnt;
                break;
            }
            next_row += 64;
        }
        wave_lds_fence();
        int row = own[lane];
        wave_lds_fence();
        own[lane] = -1;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(row, o, 64);
            if (lane >= o) row = max(row, y);
        }
        row = max(row, cur_row);

        // Segments of equal rows get consecutive ring slots.
        int prev = __shfl_up(row, 1, 64);
        if (lane == 0) prev = cur_row;
        const bool start = valid && row != prev;
        const uint64_t sm = ballot(start);
        const int slot = (cur_slot + count_below(sm) + (start ? 1 : 0)) & 63;
        if (start) slot_row[slot] = row;

        // Gather {c_j, y_j} and add val * c_j into acc[y_j][slot].
        const bool okj = valid && (unsigned)j < (unsigned)N;
        if (ballot(valid && !okj) && lane == 0) raise_error(status, kErrCsr);
        float2 inf = make_float2(0.0f, __int_as_float(-1));
        if (okj) inf = info[j];
        const int y = __float_as_int(inf.y);
        const bool contrib = okj && y >= 0;
        const float x = v * inf.x;
        const int key = slot * K + y;
        uint64_t peers = ballot(contrib);
        for (int bit = 0; bit < kbits; ++bit) {
            const bool bb = (key >> bit) & 1;
            const uint64_t m = ballot(contrib && bb);
            peers &= bb ? m : ~m;
        }
        const int rank = count_below(peers);
        for (int pass = 0;; ++pass) {
            if (!ballot(contrib && rank >= pass)) break;
            if (contrib && rank == pass) atomicAdd(&acc[y * 64 + slot], x);
            wave_lds_fence();
        }

        // Rows that end in this window are finished now.
        row_last = __shfl(row, nvalid - 1, 64);
        slot_last = __shfl(slot, nvalid - 1, 64);
        const int first_slot = __shfl(slot, 0, 64);
        cont = next_start > p + nvalid;
        const int nseg = ((slot_last - first_slot) & 63) + 1;
        const int nend = cont ? nseg - 1 : nseg;
        for (int si = 0; si < nend; ++si) {
            const int sl = (first_slot + si) & 63;
            const int r = slot_row[sl];
            if (r < 0 || r >= N) {  // only reachable with a malformed caller CSR
                for (int k = lane; k < K; k += 64) acc[k * 64 + sl] = 0.0f;
                continue;
            }
            if (!WIDE) {
                float s0 = lane < K ? acc[lane * 64 + sl] : 0.0f;
                if (lane < K) acc[lane * 64 + sl] = 0.0f;
                if (r == head_row) {
                    if (lane < K) headp[(int64_t)w * K + lane] = s0;
                } else {
                    finish_store_64(s0, lane, r, K, diag, lap, cor, info, srow, Z);
                }
            } else {
                float s0 = acc[lane * 64 + sl];
                float s1 = lane + 64 < K ? acc[(lane + 64) * 64 + sl] : 0.0f;
                acc[lane * 64 + sl] = 0.0f;
                if (lane + 64 < K) acc[(lane + 64) * 64 + sl] = 0.0f;
                if (r == head_row) {
                    headp[(int64_t)w * K + lane] = s0;
                    if (lane + 64 < K) headp[(int64_t)w * K + lane + 64] = s1;
                } else {
                    finish_store_128(s0, s1, lane, r, K, diag, lap, cor, info, srow, Z);
                }
            }
        }
        wave_lds_fence();
        cur_row = row_last;
        cur_slot = slot_last;
    }

    // The last row continues past this wavefront: leave its raw partial sums.
    int my_split = -1;
    if (cont) {
        float *dstp = (row_last == head_row) ? headp : tailp;
        if (row_last != head_row) my_split = row_last;
        for (int k = lane; k < K; k += 64) dstp[(int64_t)w * K + k] = acc[k * 64 + slot_last];
    }
    if (lane == 0) split[w] = my_split;
}

// One wavefront per embed wavefront w: finish the row that starts in w and continues.
__global__ __launch_bounds__(256) void embed_fixup(const int *__restrict__ rp,
                                                   const float2 *__restrict__ info,
                                                   const float *__restrict__ srow,
                                                   const int *__restrict__ meta, int K, int WE,
                                                   unsigned flags, const float *__restrict__ headp,
                                                   const float *__restrict__ tailp,
                                                   const int *__restrict__ split, float *__restrict__ Z) {
    const int lane = lane_id();
    const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int NW = meta[1];
    if (w >= NW) return;
    const int r = split[w];
    if (r < 0) return;
    const bool diag = flags & kDiag, lap = flags & kLap, cor = flags & kCor;
    const int end = rp[r + 1];
    const int we = (int)min((int64_t)NW - 1, max((int64_t)w, ((int64_t)end - 1) / WE));
    float v0 = 0.0f, v1 = 0.0f;
    if (lane < K) v0 = tailp[(int64_t)w * K + lane];
    if (lane + 64 < K) v1 = tailp[(int64_t)w * K + lane + 64];
    for (int w2 = w + 1; w2 <= we; ++w2) {
        if (lane < K) v0 += headp[(int64_t)w2 * K + lane];
        if (lane + 64 < K) v1 += headp[(int64_t)w2 * K + lane + 64];
    }
    if (K <= 64)
        finish_store_64(v0, lane, r, K, diag, lap, cor, info, srow, Z);
    else
        finish_store_128(v0, v1, lane, r, K, diag, lap, cor, info, srow, Z);
}

// ----------------------------------------------------------------------------- launch

size_t embed_lds_per_wave(int K) { return (size_t)(K * 64 + 128) * sizeof(float); }

hipError_t launch_embed_prep_from_csr(const int *rp, const float *val, const int *labels, int64_t M,
                                      const Plan &p, const Work &wk, unsigned *status, hipStream_t s) {
    const int NW = M > 0 ? (int)((M + p.WE - 1) / p.WE) : 1;
    prof_begin(kKPrepCsr, s);
    hipLaunchKernelGGL(prep_from_csr, dim3((p.N + 255) / 256), dim3(256), 0, s, rp, val, p.N, labels,
                       p.K, wk.inv_n, p.flags, wk.info, wk.srow, wk.fown, (int)M, NW, p.WE, status);
    prof_end(kKPrepCsr, s);
    return hipGetLastError();
}

__global__ void set_meta(int *meta, int M, int NW) {
    meta[0] = M;
    meta[1] = NW;
}

hipError_t launch_embed(const int *rp, const int *col, const float *val, const Plan &p,
                        const Work &wk, float *Z, unsigned *status, hipStream_t s) {
    const int K = p.K;
    int kbits = 0;
    while ((1 << kbits) < 64 * K) ++kbits;
    const int wpb = p.wpb;
    const unsigned grid = (unsigned)((p.NWcap + wpb - 1) / wpb);
    const size_t lds = embed_lds_per_wave(K) * wpb;
    const bool wide = K > 64;
    const bool weighted = val != nullptr;
    prof_begin(kKFillEmpty, s);
    hipLaunchKernelGGL(fill_empty, dim3((p.N + 255) / 256), dim3(256), 0, s, rp, p.N, K, p.flags,
                       wk.info, wk.srow, Z);
    prof_end(kKFillEmpty, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define GEE_EMBED_LAUNCH(WT, WD)                                                                   \
    hipLaunchKernelGGL((embed_rows<WT, WD>), dim3(grid), dim3(64 * wpb), lds, s, rp, col, val,     \
                       wk.info, wk.srow, wk.fown, wk.meta, p.N, K, kbits, p.WE, p.flags, Z,        \
                       wk.headp, wk.tailp, wk.split, status)
    prof_begin(kKEmbedRows, s);
    if (weighted) {
        if (wide) GEE_EMBED_LAUNCH(true, true); else GEE_EMBED_LAUNCH(true, false);
    } else {
        if (wide) GEE_EMBED_LAUNCH(false, true); else GEE_EMBED_LAUNCH(false, false);
    }
    prof_end(kKEmbedRows, s);
#undef GEE_EMBED_LAUNCH
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKEmbedFixup, s);
    hipLaunchKernelGGL(embed_fixup, dim3((unsigned)((p.NWcap + 3) / 4)), dim3(256), 0, s, rp, wk.info,
                       wk.srow, wk.meta, K, p.WE, p.flags, wk.headp, wk.tailp, wk.split, Z);
    prof_end(kKEmbedFixup, s);
    return hipGetLastError();
}

hipError_t launch_set_meta(int *meta, int M, int NW, hipStream_t s) {
    prof_begin(kKSetMeta, s);
    hipLaunchKernelGGL(set_meta, dim3(1), dim3(1), 0, s, meta, M, NW);
    prof_end(kKSetMeta, s);
    return hipGetLastError();
}

}  // namespace gee
