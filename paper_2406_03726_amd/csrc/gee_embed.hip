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
//   * node_rows    thread per row: the first row of every wavefront, the row step of
//                  each row's first entry (see below), and the coefficients c_i, s_i
//                  wherever the degree is a row count or not needed.
//   * degree_rows  (weighted Laplacian) degrees as segmented sums over entry-balanced
//                  wavefronts, then c_i and s_i; degree_fixup finishes cut rows.
//   * fill_empty   rows without entries (zero, or the diagonal term alone).
//   * embed_rows   wavefront w processes the CSR entries [w*WE, (w+1)*WE) in windows
//                  of 64, so every wavefront does the same work whatever the degree
//                  distribution. Rows are found without row_ptr lookups: a byte per
//                  entry holds the row step from the previous entry (0 inside a row;
//                  an escape value for steps >= 255), and a wave prefix sum turns the
//                  steps into row ids. The wavefront works in batches of 4 windows; the
//                  col/val/step loads of batch k+2 and the gathers of batch k+1 ({c_j,
//                  y_j} by column, {c_i, y_i, s_i} by row) are in flight while batch k
//                  is processed, and nothing loaded is consumed in the batch that loads
//                  it, so the memory pipeline never drains inside a batch.
//                  Rows get slots of an LDS ring acc[class][slot]. A window inside one
//                  row adds into per-lane columns (no conflicts, no matching);
//                  otherwise lanes of one row with the same class are found by ballots
//                  and take turns in lane order. The summation order is fixed, so
//                  results are bitwise reproducible. Rows ending in the wavefront are
//                  finished there (diagonal term, s_i, correlation) and stored with
//                  coalesced writes; rows cut by wavefront boundaries leave raw partials.
//   * embed_fixup  adds the partials of each cut row in wavefront order and finishes it.
#include "gee_internal.h"

#include <climits>

namespace gee {

constexpr int KS = 65;        // padded LDS stride of one class row of the slot ring
constexpr int kStepEsc = 255;  // row-step byte meaning "look the row up in row_ptr"
constexpr int BW = 4;          // windows per pipeline batch

// LDS floats of one embed wavefront: a 64-entry slot table of float4 and the slot ring
// [K][65], rounded to 16 bytes.
__host__ __device__ constexpr int embed_lds_floats(int K) { return 4 * 64 + ((K * KS + 3) & ~3); }

// ----------------------------------------------------------------------------- row steps

__global__ __launch_bounds__(256) void zero_bytes(uint8_t *__restrict__ p, int64_t n) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    if (i + 16 <= n) {
        *reinterpret_cast<uint4 *>(p + i) = make_uint4(0, 0, 0, 0);
    } else {
        for (int64_t j = i; j < n; ++j) p[j] = 0;
    }
}

// Thread per row: the first row of every embed wavefront (wrow), the step byte of each
// non-empty row's first entry (rows since the previous non-empty row, capped at the
// escape value), ownership checks, and the per-node data needing no weighted degree
// (with `skip_nonempty`, a weighted Laplacian, degree_rows fills non-empty rows).
__global__ __launch_bounds__(256) void node_rows(const int *__restrict__ rp, int N, const int *__restrict__ meta,
                                                 int WE, const int *__restrict__ labels, int K,
                                                 const float *__restrict__ inv_n, unsigned flags,
                                                 int skip_nonempty, float2 *__restrict__ info,
                                                 float *__restrict__ srow, int *__restrict__ wrow,
                                                 uint8_t *__restrict__ rstep, unsigned *status) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int M = meta[0], NW = meta[1];
    bool bad = false;
    if (r < N) {
        const int lo = rp[r], hi = rp[r + 1];
        if (lo > hi || lo < 0 || hi > M || (r == 0 && lo != 0) || (r == N - 1 && hi != M)) bad = true;
        const bool lap = flags & kLap, diag = flags & kDiag;
        if (!(skip_nonempty && hi > lo)) {
            int y = labels[r];
            if (y < 0 || y >= K) y = -1;
            float s = 1.0f;
            if (lap) {
                const float d = (float)max(hi - lo, 0) + (diag ? 1.0f : 0.0f);
                s = d > 0.0f ? 1.0f / sqrtf(d) : 0.0f;
                srow[r] = s;
            }
            info[r] = make_float2(y >= 0 ? s * inv_n[y] : 0.0f, __int_as_float(y));
        }
        if (hi > lo && lo >= 0 && hi <= M) {
            // rows back to the previous non-empty row (row -1 before row 0)
            int gap = 1;
            while (gap < kStepEsc && r - gap >= 0 && rp[r - gap] == rp[r - gap + 1]) ++gap;
            rstep[lo] = (uint8_t)min(gap, kStepEsc);
            // wavefronts whose first entry lies in this row
            const int64_t wa = ((int64_t)lo + WE - 1) / WE;
            const int64_t wb = min(((int64_t)hi - 1) / WE, (int64_t)NW - 1);
            for (int64_t ww = wa; ww <= wb; ++ww) wrow[ww] = r;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) raise_error(status, kErrCsr);
}

// The row holding entry q (last r with rp[r] <= q), by binary search.
__device__ __forceinline__ int row_of_entry(const int *__restrict__ rp, int N, int q) {
    int lo = 0, hi = N;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rp[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Rows of the 64 lanes of a window from their step bytes: row = base + inclusive sum of
// the steps; an escape lane looks its row up and the sum restarts there. `d` must be 0 on
// lanes past the end. With `force_lane0`, lane 0's step is taken as 0 (its row is `base`).
__device__ __forceinline__ int window_rows(int d, int base, bool force_lane0, int p,
                                           const int *__restrict__ rp, int N) {
    const int lane = lane_id();
    if (force_lane0 && lane == 0) d = 0;
    const bool esc = d == kStepEsc;
    const int S = wave_scan_add(esc ? 0 : d);
    const uint64_t em = ballot(esc);
    if (em == 0) return base + S;
    // rare: a run of >= 254 empty rows before some row of this window
    const int ar = esc ? row_of_entry(rp, N, p + lane) : 0;
    const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
    const uint64_t eb = em & le;
    const int e = eb ? 63 - __clzll(eb) : 0;
    const int are = __shfl(ar, e, 64), Se = __shfl(S, e, 64);
    return eb ? are + (S - Se) : base + S;
}

// ----------------------------------------------------------------------------- degrees

__device__ __forceinline__ void finish_node(int r, float d, int y, const float *inv_n_lds, bool diag,
                                            float2 *__restrict__ info, float *__restrict__ srow) {
    const float dd = d + (diag ? 1.0f : 0.0f);
    const float s = dd > 0.0f ? 1.0f / sqrtf(dd) : 0.0f;
    srow[r] = s;
    info[r] = make_float2(y >= 0 ? s * inv_n_lds[y] : 0.0f, __int_as_float(y));
}

// Weighted degrees d_i = sum of the row's values, as segmented sums over the same
// entry-balanced wavefronts and batches as embed_rows (fixed summation order; the open
// row's running sum is compensated). Then s_i and c_i.
__global__ __launch_bounds__(256) void degree_rows(const int *__restrict__ rp, const float *__restrict__ val,
                                                   const uint8_t *__restrict__ rstep,
                                                   const int *__restrict__ wrow, const int *__restrict__ meta,
                                                   int N, int WE, const int *__restrict__ labels, int K,
                                                   const float *__restrict__ inv_n, unsigned flags,
                                                   float2 *__restrict__ info, float *__restrict__ srow,
                                                   float *__restrict__ headd, float *__restrict__ taild,
                                                   int *__restrict__ dsplit) {
    __shared__ float invn_s[kMaxClasses];
    for (int k = threadIdx.x; k < K; k += blockDim.x) invn_s[k] = inv_n[k];
    __syncthreads();
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int M = meta[0], NW = meta[1];
    const int w = blockIdx.x * (blockDim.x >> 6) + wib;
    if (w >= NW) return;
    const bool diag = flags & kDiag;
    const int a = w * WE, b = min(a + WE, M), last = b - 1;
    const int row_a = min(max(wrow[w], 0), N - 1);
    const bool head = rstep[a] == 0;
    const int head_row = head ? row_a : -1;
    const bool cont_end = b < M && rstep[min(b, M - 1)] == 0;
    int cur_row = head ? row_a : -1;
    float carry = 0.0f, comp = 0.0f;  // running sum of the open row and its compensation
    bool cont = false;
    const int nwin = (b - a + 63) >> 6;
    auto ld_val = [&](int e) { const float v = val[min(e, last)]; return e < b ? v : 0.0f; };
    auto ld_step = [&](int e) { const int v = rstep[min(e, last)]; return e < b ? v : 0; };
    auto ld_lab = [&](int r) { const int y = labels[min(max(r, 0), N - 1)]; return (y >= 0 && y < K) ? y : -1; };
    float vc[BW], vn1[BW], vn2[BW];
    int dc[BW], dn1[BW], dn2[BW], rc[BW], rn1[BW], yc[BW], yn1[BW];
    int base;
#pragma unroll
    for (int u = 0; u < BW; ++u) {
        vc[u] = ld_val(a + u * 64 + lane);
        dc[u] = ld_step(a + u * 64 + lane);
        vn1[u] = ld_val(a + (BW + u) * 64 + lane);
        dn1[u] = ld_step(a + (BW + u) * 64 + lane);
    }
    base = row_a;
#pragma unroll
    for (int u = 0; u < BW; ++u) {
        rc[u] = window_rows(dc[u], base, u == 0, a + u * 64, rp, N);
        base = readlane(rc[u], 63);
        yc[u] = ld_lab(rc[u]);
    }
    for (int i0 = 0; i0 < nwin; i0 += BW) {
#pragma unroll
        for (int u = 0; u < BW; ++u) {
            rn1[u] = window_rows(dn1[u], base, false, a + (i0 + BW + u) * 64, rp, N);
            base = readlane(rn1[u], 63);
            yn1[u] = ld_lab(rn1[u]);
            vn2[u] = ld_val(a + (i0 + 2 * BW + u) * 64 + lane);
            dn2[u] = ld_step(a + (i0 + 2 * BW + u) * 64 + lane);
        }
#pragma unroll
        for (int u = 0; u < BW; ++u) {
            const int i = i0 + u;
            if (i >= nwin) break;
            const int p = a + (i << 6);
            const int nvalid = min(64, b - p);
            const float v = vc[u];
            const int row = rc[u];
            const int nxt = (u + 1 < BW) ? readlane(dc[u + 1], 0) : readlane(dn1[0], 0);
            cont = (p + nvalid < b) ? (nxt == 0) : cont_end;
            const uint64_t sm = ballot(lane < nvalid && dc[u] != 0);
            if (sm == 0) {  // the window lies inside the open row
                const float t = wave_sum(v) - comp;
                const float s = carry + t;
                comp = (s - carry) - t;
                carry = s;
                if (!cont) {
                    if (lane == 0) {  // every lane holds the open row and its label
                        if (cur_row == head_row) headd[w] = carry;
                        else if (cur_row >= 0 && cur_row < N)
                            finish_node(cur_row, carry, yc[u], invn_s, diag, info, srow);
                    }
                    carry = comp = 0.0f;
                }
                continue;
            }
            // inclusive segmented scan of the values over lanes of equal rows
            const float x = wave_seg_scan_addf(v, row);
            const int nxt_row = dpp_i<0x130>(row, INT32_MIN);  // wave_shl:1, lane l gets lane l+1
            const bool last_of_seg = lane < nvalid && (lane == nvalid - 1 || nxt_row != row);
            const int row_last = readlane(row, nvalid - 1);
            if (last_of_seg) {
                float d = x;
                if (row == cur_row) d = carry + (x - comp);  // the open row's earlier windows first
                const bool ends = !(row == row_last && cont);
                if (ends) {
                    if (row == head_row) headd[w] = d;
                    else if (row >= 0 && row < N) finish_node(row, d, yc[u], invn_s, diag, info, srow);
                }
            }
            const float tail = readlane_f(x, nvalid - 1);
            if (cont) {
                carry = (row_last == cur_row) ? carry + (tail - comp) : tail;
                comp = 0.0f;
            } else {
                carry = comp = 0.0f;
            }
            cur_row = row_last;
        }
#pragma unroll
        for (int u = 0; u < BW; ++u) {
            vc[u] = vn1[u];
            dc[u] = dn1[u];
            rc[u] = rn1[u];
            yc[u] = yn1[u];
            vn1[u] = vn2[u];
            dn1[u] = dn2[u];
        }
    }
    int my_split = -1;
    if (cont && lane == 0) {
        if (cur_row == head_row) {
            headd[w] = carry;
        } else {
            taild[w] = carry;
            my_split = cur_row;
        }
    }
    if (lane == 0) dsplit[w] = my_split;
}

__global__ __launch_bounds__(256) void degree_fixup(const int *__restrict__ rp, const int *__restrict__ meta,
                                                    int N, int WE, const int *__restrict__ labels, int K,
                                                    const float *__restrict__ inv_n, unsigned flags,
                                                    const float *__restrict__ headd,
                                                    const float *__restrict__ taild,
                                                    const int *__restrict__ dsplit,
                                                    float2 *__restrict__ info, float *__restrict__ srow) {
    const int NW = meta[1];
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= NW) return;
    const int r = dsplit[w];
    if (r < 0 || r >= N) return;
    const int end = rp[r + 1];
    const int we = (int)min((int64_t)NW - 1, max((int64_t)w, ((int64_t)end - 1) / WE));
    float d = taild[w];
    for (int w2 = w + 1; w2 <= we; ++w2) d += headd[w2];
    int y = labels[r];
    if (y < 0 || y >= K) y = -1;
    const float dd = d + ((flags & kDiag) ? 1.0f : 0.0f);
    const float s = dd > 0.0f ? 1.0f / sqrtf(dd) : 0.0f;
    srow[r] = s;
    info[r] = make_float2(y >= 0 ? s * inv_n[y] : 0.0f, __int_as_float(y));
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

// Sum of v over aligned groups of kp lanes (kp a power of two <= 64), returned on every
// lane of the group. DPP lane moves only; every lane of the wavefront must take part.
__device__ __forceinline__ float group_sum(float v, int kp) {
    if (kp == 64) return wave_sum(v);
    if (kp == 32) {
        // prefix sums inside each half (no carry from lane 31 into the upper half, so
        // neither half's sum is formed as a difference)
        v += dpp_f<0x111>(v, 0.0f);
        v += dpp_f<0x112>(v, 0.0f);
        v += dpp_f<0x114>(v, 0.0f);
        v += dpp_f<0x118>(v, 0.0f);
        v += dpp_f<0x142, 0xA>(v, 0.0f);
        const float s31 = readlane_f(v, 31), s63 = readlane_f(v, 63);
        return lane_id() < 32 ? s31 : s63;
    }
    if (kp >= 2) v += dpp_f<0xB1>(v, 0.0f);   // quad_perm [1,0,3,2]
    if (kp >= 4) v += dpp_f<0x4E>(v, 0.0f);   // quad_perm [2,3,0,1]
    if (kp >= 8) v += dpp_f<0x141>(v, 0.0f);  // row_half_mirror: the other quad of 8
    if (kp >= 16) v += dpp_f<0x140>(v, 0.0f); // row_mirror: the other half of 16
    return v;
}

// ----------------------------------------------------------------------------- main kernel

template <bool WEIGHTED, bool WIDE>
__global__ __launch_bounds__(256) void embed_rows(const int *__restrict__ rp, const int *__restrict__ col,
                                                  const float *__restrict__ val,
                                                  const uint8_t *__restrict__ rstep,
                                                  const float2 *__restrict__ info,
                                                  const float *__restrict__ srow,
                                                  const int *__restrict__ wrow,
                                                  const int *__restrict__ meta, int N, int K, int kp,
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

    // per wavefront: slot table [64] {row, c_i, y_i, s_i}, then the ring acc[K][KS]
    float4 *slot_meta = reinterpret_cast<float4 *>(smem_f + (size_t)wib * embed_lds_floats(K));
    float *acc = reinterpret_cast<float *>(slot_meta + 64);
    for (int k = 0; k < K; ++k) acc[k * KS + lane] = 0.0f;
    // Finished rows stay in their ring slots ("pending") until drain() stores them:
    // slots [pend_first, pend_first + npend) in ring order, just behind the open row.
    int npend = 0, pend_first = 0;

    const int a = w * WE;
    const int b = min(a + WE, M);
    const int last = b - 1;
    const int row_a = min(max(wrow[w], 0), N - 1);
    // entry a continues a row begun before the wavefront / entry b continues the last row
    const bool head = __builtin_amdgcn_readfirstlane(rstep[a]) == 0;
    const int head_row = head ? row_a : -1;
    const bool cont_end = b < M && __builtin_amdgcn_readfirstlane(rstep[min(b, M - 1)]) == 0;
    int cur_row = head ? row_a : -1;
    int cur_slot = 63;
    if (lane == 0) slot_meta[63] = make_float4(__int_as_float(cur_row), 0.0f, __int_as_float(-1), 0.0f);
    bool cont = false;

    // Finish the pending rows (diagonal term, s_i, correlation; the head row goes out
    // raw) and store them. kp lanes per row (WIDE: one row, two classes per lane). This
    // loop holds the only global stores and reads nothing loaded from global memory, so
    // it never waits for the loads in flight.
    auto drain = [&]() {
        wave_lds_fence();
        const int grp = WIDE ? 1 : 64 / kp;  // rows per pass
        const int g = WIDE ? 0 : lane / kp;
        const int k = WIDE ? lane : lane & (kp - 1);
        const int kk = min(k, K - 1);
        for (int j = 0; j < npend; j += grp) {
            const bool has = j + g < npend;
            const int sl = (pend_first + j + g) & 63;
            const float4 m = slot_meta[sl];
            const int r = __float_as_int(m.x);
            const int lab = __float_as_int(m.z);
            const bool live = has && r >= 0 && r < N;
            float v0 = acc[kk * KS + sl];
            float v1 = 0.0f;
            if (WIDE) v1 = acc[min(k + 64, K - 1) * KS + sl];
            if (has) {
                acc[kk * KS + sl] = 0.0f;
                if (WIDE && k + 64 < K) acc[(k + 64) * KS + sl] = 0.0f;
            }
            v0 = k < K ? v0 : 0.0f;
            v1 = (WIDE && k + 64 < K) ? v1 : 0.0f;
            float z0 = v0, z1 = v1;
            if (diag && k == lab) z0 += m.y;
            if (WIDE && diag && k + 64 == lab) z1 += m.y;
            if (lap) {
                z0 *= m.w;
                z1 *= m.w;
            }
            if (cor) {
                const float ss = WIDE ? wave_sum(z0 * z0 + z1 * z1) : group_sum(z0 * z0, kp);
                const float sc = ss > 0.0f ? 1.0f / sqrtf(ss) : 1.0f;
                z0 *= sc;
                z1 *= sc;
            }
            if (r == head_row) {
                z0 = v0;
                z1 = v1;
            }
            if (live) {
                float *dst = r == head_row ? headp + (int64_t)w * K : Z + (int64_t)r * K;
                if (k < K) dst[k] = z0;
                if (WIDE && k + 64 < K) dst[k + 64] = z1;
            }
        }
        npend = 0;
        wave_lds_fence();
    };

    // Loads are unconditional (clamped address, value masked afterwards) and are only
    // consumed in a later batch.
    const int nwin = (b - a + 63) >> 6;
    auto ld_col = [&](int e) { const int v = col[min(e, last)]; return e < b ? v : -1; };
    auto ld_val = [&](int e) { return WEIGHTED ? val[min(e, last)] : 1.0f; };
    auto ld_step = [&](int e) { const int v = rstep[min(e, last)]; return e < b ? v : 0; };
    auto gather_col = [&](int j) {
        const float2 f = info[min(max(j, 0), N - 1)];
        return (unsigned)j < (unsigned)N ? f : make_float2(0.0f, __int_as_float(-1));
    };
    int cn1[BW], cn2[BW], dc[BW], dn1[BW], dn2[BW], rc[BW], rn1[BW];
    float vc[BW], vn1[BW], vn2[BW], sc[BW], sn1[BW];
    float2 fc[BW], fn1[BW], qc[BW], qn1[BW];  // f: {c_j, y_j} by column; q: {c_i, y_i} by row
    bool bad = false;
    int base;
#pragma unroll
    for (int u = 0; u < BW; ++u) {
        const int e0 = a + u * 64 + lane, e1 = a + (BW + u) * 64 + lane;
        const int c0 = ld_col(e0);
        vc[u] = ld_val(e0);
        dc[u] = ld_step(e0);
        cn1[u] = ld_col(e1);
        vn1[u] = ld_val(e1);
        dn1[u] = ld_step(e1);
        bad |= e0 < b && (unsigned)c0 >= (unsigned)N;
        fc[u] = gather_col(c0);
    }
    base = row_a;
#pragma unroll
    for (int u = 0; u < BW; ++u) {
        rc[u] = window_rows(dc[u], base, u == 0, a + u * 64, rp, N);
        base = readlane(rc[u], 63);
        const int rr = min(max(rc[u], 0), N - 1);
        qc[u] = info[rr];
        sc[u] = lap ? srow[rr] : 1.0f;
    }
    const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1);  // lanes <= this one

    for (int i0 = 0; i0 < nwin; i0 += BW) {
        // issue: rows and gathers of batch k+1, col/val/steps of batch k+2
#pragma unroll
        for (int u = 0; u < BW; ++u) {
            const int e1 = a + (i0 + BW + u) * 64 + lane, e2 = a + (i0 + 2 * BW + u) * 64 + lane;
            rn1[u] = window_rows(dn1[u], base, false, a + (i0 + BW + u) * 64, rp, N);
            base = readlane(rn1[u], 63);
            const int rr = min(max(rn1[u], 0), N - 1);
            bad |= e1 < b && (unsigned)cn1[u] >= (unsigned)N;
            fn1[u] = gather_col(cn1[u]);
            qn1[u] = info[rr];
            sn1[u] = lap ? srow[rr] : 1.0f;
            cn2[u] = ld_col(e2);
            vn2[u] = ld_val(e2);
            dn2[u] = ld_step(e2);
        }
        // process batch k
#pragma unroll
        for (int u = 0; u < BW; ++u) {
            const int i = i0 + u;
            if (i >= nwin) break;
            const int p = a + (i << 6);
            const int nvalid = min(64, b - p);
            const bool valid = lane < nvalid;
            const int y = __float_as_int(fc[u].y);
            const float x = vc[u] * fc[u].x;
            const int nxt = (u + 1 < BW) ? readlane(dc[u + 1], 0) : readlane(dn1[0], 0);
            cont = (p + nvalid < b) ? (nxt == 0) : cont_end;
            const bool start = valid && dc[u] != 0;
            const uint64_t sm = ballot(start);
            const int nnew = __popcll(sm);
            // the open row and the new rows need ring slots next to the pending ones
            if (npend + 1 + nnew > 64) drain();
            const int slot = (cur_slot + __popcll(sm & le)) & 63;
            // Lanes with equal (row, class) add to the same LDS word; the LDS applies
            // them one after another in a fixed order, so the sums are reproducible.
            if (valid && y >= 0) atomicAdd(&acc[y * KS + slot], x);
            if (start) slot_meta[slot] = make_float4(__int_as_float(rc[u]), qc[u].x, qc[u].y, sc[u]);
            // rows ended in this window: from lane 0's row to the last lane's row, the
            // latter only if the next entry starts a new row
            const int first_slot = (sm & 1ull) ? (cur_slot + 1) & 63 : cur_slot;
            const int slot_last = (cur_slot + nnew) & 63;
            const int nseg = ((slot_last - first_slot) & 63) + 1;
            const int nend = cont ? nseg - 1 : nseg;
            if (nend > 0) {
                if (npend == 0) pend_first = first_slot;
                npend += nend;
            }
            cur_row = nnew ? readlane(rc[u], 63 - __clzll(sm)) : cur_row;
            cur_slot = slot_last;
        }
        drain();
#pragma unroll
        for (int u = 0; u < BW; ++u) {
            vc[u] = vn1[u];
            dc[u] = dn1[u];
            rc[u] = rn1[u];
            fc[u] = fn1[u];
            qc[u] = qn1[u];
            sc[u] = sn1[u];
            cn1[u] = cn2[u];
            vn1[u] = vn2[u];
            dn1[u] = dn2[u];
        }
    }
    if (ballot(bad) && lane == 0) raise_error(status, kErrCsr);

    // The last row continues past this wavefront: leave its raw partial sums.
    if (npend > 0) drain();
    int my_split = -1;
    if (cont) {
        float *dstp = (cur_row == head_row) ? headp : tailp;
        if (cur_row != head_row) my_split = cur_row;
        for (int k = lane; k < K; k += 64) dstp[(int64_t)w * K + k] = acc[k * KS + cur_slot];
    }
    if (lane == 0) split[w] = my_split;
}

// One wavefront per embed wavefront w: finish the row that starts in w and continues.
__global__ __launch_bounds__(256) void embed_fixup(const int *__restrict__ rp,
                                                   const float2 *__restrict__ info,
                                                   const float *__restrict__ srow,
                                                   const int *__restrict__ meta, int N, int K, int WE,
                                                   unsigned flags, const float *__restrict__ headp,
                                                   const float *__restrict__ tailp,
                                                   const int *__restrict__ split, float *__restrict__ Z) {
    const int lane = lane_id();
    const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int NW = meta[1];
    if (w >= NW) return;
    const int r = split[w];
    if (r < 0 || r >= N) return;
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
    const float2 inf = info[r];
    const int lab = __float_as_int(inf.y);
    const float s = lap ? srow[r] : 1.0f;
    if (diag && lane == lab) v0 += inf.x;
    if (diag && lane + 64 == lab) v1 += inf.x;
    if (lap) {
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
    if (lane < K) Z[(int64_t)r * K + lane] = v0;
    if (lane + 64 < K) Z[(int64_t)r * K + lane + 64] = v1;
}

// ----------------------------------------------------------------------------- launch

size_t embed_lds_per_wave(int K) { return (size_t)embed_lds_floats(K) * sizeof(float); }

__global__ void set_meta(int *meta, int M, int NW) {
    meta[0] = M;
    meta[1] = NW;
}

hipError_t launch_set_meta(int *meta, int M, int NW, hipStream_t s) {
    prof_begin(kKSetMeta, s);
    hipLaunchKernelGGL(set_meta, dim3(1), dim3(1), 0, s, meta, M, NW);
    prof_end(kKSetMeta, s);
    return hipGetLastError();
}

// Per-node data for the embedding of a CSR: first rows of the wavefronts, row steps,
// degrees, s_i and c_i. meta[0..1] (M and the wavefront count) must be set beforehand.
hipError_t launch_node_prep(const int *rp, const float *val, const int *labels, const Plan &p,
                            const Work &wk, unsigned *status, hipStream_t s) {
    const bool weighted_lap = val != nullptr && (p.flags & kLap);
    const int64_t nz = (p.Mcap + 16 * 256 - 1) / (16 * 256);
    prof_begin(kKZeroSteps, s);
    hipLaunchKernelGGL(zero_bytes, dim3((unsigned)(nz > 0 ? nz : 1)), dim3(256), 0, s, wk.rstep, p.Mcap);
    prof_end(kKZeroSteps, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    prof_begin(kKNodeRows, s);
    hipLaunchKernelGGL(node_rows, dim3((p.N + 255) / 256), dim3(256), 0, s, rp, p.N, wk.meta, p.WE, labels,
                       p.K, wk.inv_n, p.flags, weighted_lap ? 1 : 0, wk.info, wk.srow, wk.wrow, wk.rstep,
                       status);
    prof_end(kKNodeRows, s);
    if ((e = hipGetLastError()) != hipSuccess || !weighted_lap) return e;
    prof_begin(kKDegreeRows, s);
    hipLaunchKernelGGL(degree_rows, dim3((unsigned)((p.NWcap + 3) / 4)), dim3(256), 0, s, rp, val, wk.rstep,
                       wk.wrow, wk.meta, p.N, p.WE, labels, p.K, wk.inv_n, p.flags, wk.info, wk.srow, wk.headd,
                       wk.taild, wk.dsplit);
    prof_end(kKDegreeRows, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKDegreeFixup, s);
    hipLaunchKernelGGL(degree_fixup, dim3((unsigned)((p.NWcap + 255) / 256)), dim3(256), 0, s, rp, wk.meta,
                       p.N, p.WE, labels, p.K, wk.inv_n, p.flags, wk.headd, wk.taild, wk.dsplit, wk.info,
                       wk.srow);
    prof_end(kKDegreeFixup, s);
    return hipGetLastError();
}

hipError_t launch_embed(const int *rp, const int *col, const float *val, const Plan &p,
                        const Work &wk, float *Z, unsigned *status, hipStream_t s) {
    const int K = p.K;
    int kp = 1;
    while (kp < K && kp < 64) kp <<= 1;
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
                       wk.rstep, wk.info, wk.srow, wk.wrow, wk.meta, p.N, K, kp, p.WE,       \
                       p.flags, Z,                                                                 \
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
                       wk.srow, wk.meta, p.N, K, p.WE, p.flags, wk.headp, wk.tailp, wk.split, Z);
    prof_end(kKEmbedFixup, s);
    return hipGetLastError();
}

}  // namespace gee
