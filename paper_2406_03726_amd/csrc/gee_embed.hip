// gee_embed.hip - Z = A W with the Table 1 options, from a CSR (Eq. 1, Section 2).
//
// For row i with D^-1/2 factor s_i (1 without the Laplacian) and per-node
// coefficient c_j = s_j / n_{y_j} (0 for an unknown label):
//     Z[i, k] = s_i * ( sum_{e in row i, y_col(e) = k} val_e * c_col(e)  +  [diag, k = y_i] c_i )
// then, with correlation, row i is divided by its 2-norm. This is Eq. 1 with A
// replaced by D^-1/2 (A + I) D^-1/2: the rescale e_ij s_i s_j is split into the
// gathered c_j and the per-row s_i, and the identity's entry is the c_i term.
//
// Every kernel serves a batch of graphs (a plain call is a batch of one): rows and CSR
// entries are those of the union, and each work item reads its graph's sizes, options
// and schedule from the graph descriptor (gee_internal.h). A graph's work is split
// exactly as when it is embedded alone, so its Z is bit-identical either way.
//
// Work split (MI355X, 64-wide wavefronts, HBM-bound, no MFMA since W is one-hot):
//   * graph_meta   per graph: first CSR entry, entry count, embed wavefront count.
//   * node_rows    thread per row: the first row of every wavefront, the row step of
//                  each row's first entry (see below), and the coefficients c_i, s_i
//                  wherever the degree is a row count or not needed.
//   * degree_rows  (weighted Laplacian) degrees as segmented sums over entry-balanced
//                  wavefronts, then c_i and s_i; degree_fixup finishes cut rows.
//   * fill_empty   rows without entries (zero, or the diagonal term alone).
//   * embed_rows   wavefront w of a graph processes that graph's CSR entries
//                  [w*WE, (w+1)*WE) in windows of 64, so every wavefront does the same
//                  work whatever the degree distribution. Rows are found without
//                  row_ptr lookups: a byte per entry holds the row step from the previous
//                  entry (0 inside a row; an escape value for steps >= 255), and a wave
//                  prefix sum turns the steps into row ids. The wavefront works in
//                  batches of 2 windows; the col/val/step loads of batch k+2 and the
//                  gathers of batch k+1 ({c_j, y_j} by column, {c_i, y_i, s_i} by row)
//                  are in flight while batch k is processed, and nothing loaded is
//                  consumed in the batch that loads it, so the memory pipeline never
//                  drains inside a batch. Rows get slots of an LDS ring acc[slot][class];
//                  a starting row first receives its diagonal term, then every lane adds
//                  its entry into acc[slot(row)][y_j] with an LDS float atomic, and the
//                  LDS applies lanes that hit the same word one after another in a fixed
//                  order, so results are bitwise reproducible. Rows ending in the
//                  wavefront are finished there (s_i, correlation) and stored with
//                  coalesced writes; rows cut by wavefront boundaries leave raw partials.
//   * embed_fixup  adds the partials of each cut row in wavefront order and finishes it.
#include "gee_internal.h"

#include <climits>

namespace gee {

constexpr int kStepEsc = 255;  // row-step byte meaning "look the row up in row_ptr"
constexpr int BW = 4;          // windows per pipeline batch (degree_rows)
constexpr int EBW = 2;         // windows per pipeline batch (embed_rows)

// Floats per slot of the embed ring: K rounded up to a multiple of 4 (16-byte rows).
__host__ __device__ constexpr int ring_stride(int K) { return (K + 3) & ~3; }
// LDS floats of one embed wavefront: the ring [64][ring_stride(K)] and three 64-entry
// slot tables.
__host__ __device__ constexpr int embed_lds_floats(int K) { return 64 * ring_stride(K) + 3 * 64; }

// Graph and local index of embed wavefront w; false if w has no work.
__device__ __forceinline__ bool wave_graph(const Batch &b, int w, GDesc &d, GMeta &m, int &lw) {
    const int g = find_graph(b.wave_offs, b.G, w);
    d = load_desc(b, g);
    lw = w - d.wave_off;
    if (lw < 0 || lw >= d.NWcap) return false;
    m = b.gm[g];
    return lw < m.NW;
}

// ----------------------------------------------------------------------------- per graph

__global__ __launch_bounds__(256) void zero_bytes(uint8_t *__restrict__ p, int64_t n) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    if (i + 16 <= n) {
        *reinterpret_cast<uint4 *>(p + i) = make_uint4(0, 0, 0, 0);
    } else {
        for (int64_t j = i; j < n; ++j) p[j] = 0;
    }
}

// Thread per graph: entry range and wavefront count, from the union's row_ptr or, for a
// single resident CSR, from its entry count.
__global__ __launch_bounds__(256) void graph_meta(Batch b, const int *__restrict__ rp, int M1) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= b.G) return;
    const GDesc d = load_desc(b, g);
    GMeta m;
    if (rp) {
        m.ent_off = rp[d.node_off];
        m.M = rp[d.node_off + d.N] - m.ent_off;
    } else {
        m.ent_off = 0;
        m.M = M1;
    }
    m.NW = m.M > 0 ? (int)min((int64_t)d.NWcap, ((int64_t)m.M + d.WE - 1) / d.WE) : 0;
    m.pad = 0;
    b.gm[g] = m;
}

// ----------------------------------------------------------------------------- row steps

// Thread per row: the first row of every embed wavefront (wrow), the step byte of each
// non-empty row's first entry (rows since the previous non-empty row of the graph,
// capped at the escape value), ownership checks, and the per-node data needing no
// weighted degree (a weighted graph with the Laplacian gets them from degree_rows).
__global__ __launch_bounds__(256) void node_rows(Batch b, int Ntot, const int *__restrict__ rp,
                                                 const float *__restrict__ inv_n, float2 *__restrict__ info,
                                                 float *__restrict__ srow, int *__restrict__ wrow,
                                                 uint8_t *__restrict__ rstep, unsigned *status) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (r < Ntot) {
        const int g = find_graph(b.node_offs, b.G, r);
        const GDesc d = load_desc(b, g);
        const GMeta m = b.gm[g];
        const int rl = r - d.node_off;
        const int lo = rp[r], hi = rp[r + 1];
        const int e_lo = m.ent_off, e_hi = m.ent_off + m.M;
        if (lo > hi || lo < e_lo || hi > e_hi || (rl == 0 && lo != e_lo) || (rl == d.N - 1 && hi != e_hi))
            bad = true;
        const bool lap = d.flags & kLap, diag = d.flags & kDiag;
        const bool skip = d.weighted && lap && hi > lo;
        if (!skip) {
            int y = d.labels[rl];
            if (y < 0 || y >= d.K) y = -1;
            float s = 1.0f;
            if (lap) {
                const float dg = (float)max(hi - lo, 0) + (diag ? 1.0f : 0.0f);
                s = dg > 0.0f ? 1.0f / sqrtf(dg) : 0.0f;
                srow[r] = s;
            }
            info[r] = make_float2(y >= 0 ? s * inv_n[d.class_off + y] : 0.0f, __int_as_float(y));
        }
        if (hi > lo && !bad) {
            // rows back to the previous non-empty row of the graph (row -1 before row 0)
            int gap = 1;
            while (gap < kStepEsc && rl - gap >= 0 && rp[r - gap] == rp[r - gap + 1]) ++gap;
            rstep[lo] = (uint8_t)min(gap, kStepEsc);
            // wavefronts of the graph whose first entry lies in this row
            const int64_t wa = ((int64_t)(lo - e_lo) + d.WE - 1) / d.WE;
            const int64_t wb = min(((int64_t)(hi - e_lo) - 1) / d.WE, (int64_t)m.NW - 1);
            for (int64_t ww = wa; ww <= wb; ++ww) wrow[d.wave_off + ww] = r;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) raise_error(status, kErrCsr);
}

// The row holding entry q among the graph's rows rp[0..N] (last r with rp[r] <= q).
__device__ __forceinline__ int row_of_entry(const int *__restrict__ rpg, int N, int q) {
    int lo = 0, hi = N;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rpg[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Rows of the 64 lanes of a window from their step bytes: row = base + inclusive sum of
// the steps; an escape lane looks its row up and the sum restarts there. `d` must be 0 on
// lanes past the end. With `force_lane0`, lane 0's step is taken as 0 (its row is `base`).
// rpg/N/node_off: the graph's rows.
__device__ __forceinline__ int window_rows(int d, int base, bool force_lane0, int p,
                                           const int *__restrict__ rpg, int N, int node_off) {
    const int lane = lane_id();
    if (force_lane0 && lane == 0) d = 0;
    const bool esc = d == kStepEsc;
    const int S = wave_scan_add(esc ? 0 : d);
    const uint64_t em = ballot(esc);
    if (em == 0) return base + S;
    // rare: a run of >= 254 empty rows before some row of this window
    const int ar = esc ? row_of_entry(rpg, N, p + lane) + node_off : 0;
    const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
    const uint64_t eb = em & le;
    const int e = eb ? 63 - __clzll(eb) : 0;
    const int are = __shfl(ar, e, 64), Se = __shfl(S, e, 64);
    return eb ? are + (S - Se) : base + S;
}

// ----------------------------------------------------------------------------- degrees

__device__ __forceinline__ void finish_node(int r, float d, int y, float inv_n_y, bool diag,
                                            float2 *__restrict__ info, float *__restrict__ srow) {
    const float dd = d + (diag ? 1.0f : 0.0f);
    const float s = dd > 0.0f ? 1.0f / sqrtf(dd) : 0.0f;
    srow[r] = s;
    info[r] = make_float2(y >= 0 ? s * inv_n_y : 0.0f, __int_as_float(y));
}

// Weighted degrees d_i = sum of the row's values, as segmented sums over the same
// entry-balanced wavefronts and batches as embed_rows (fixed summation order; the open
// row's running sum is compensated). Then s_i and c_i. Wavefronts of graphs without
// weights or without the Laplacian leave at once.
__global__ __launch_bounds__(256) void degree_rows(Batch b, const int *__restrict__ rp,
                                                   const float *__restrict__ val,
                                                   const uint8_t *__restrict__ rstep,
                                                   const int *__restrict__ wrow,
                                                   const float *__restrict__ inv_n, float2 *__restrict__ info,
                                                   float *__restrict__ srow, float *__restrict__ headd,
                                                   float *__restrict__ taild, int *__restrict__ dsplit) {
    const int lane = lane_id();
    const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    GDesc gd;
    GMeta gm;
    int lw;
    if (!wave_graph(b, w, gd, gm, lw)) return;
    if (!(gd.weighted && (gd.flags & kLap))) return;
    const bool diag = gd.flags & kDiag;
    const int N = gd.N, K = gd.K, node_off = gd.node_off;
    const int *rpg = rp + node_off;
    const float *invn = inv_n + gd.class_off;
    const int a = gm.ent_off + lw * gd.WE, b_ = min(a + gd.WE, gm.ent_off + gm.M), last = b_ - 1;
    const int E_end = gm.ent_off + gm.M;
    const int row_a = min(max(wrow[w], node_off), node_off + N - 1);
    const bool head = __builtin_amdgcn_readfirstlane(rstep[a]) == 0;
    const int head_row = head ? row_a : -1;
    const bool cont_end = b_ < E_end && __builtin_amdgcn_readfirstlane(rstep[min(b_, E_end - 1)]) == 0;
    int cur_row = head ? row_a : -1;
    float carry = 0.0f, comp = 0.0f;  // running sum of the open row and its compensation
    bool cont = false;
    const int nwin = (b_ - a + 63) >> 6;
    auto ld_val = [&](int e) { const float v = val[min(e, last)]; return e < b_ ? v : 0.0f; };
    auto ld_step = [&](int e) { const int v = rstep[min(e, last)]; return e < b_ ? v : 0; };
    auto ld_lab = [&](int r) {
        const int y = gd.labels[min(max(r - node_off, 0), N - 1)];
        return (y >= 0 && y < K) ? y : -1;
    };
    auto inv_of = [&](int y) { return y >= 0 ? invn[y] : 0.0f; };
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
        rc[u] = window_rows(dc[u], base, u == 0, a + u * 64, rpg, N, node_off);
        base = readlane(rc[u], 63);
        yc[u] = ld_lab(rc[u]);
    }
    for (int i0 = 0; i0 < nwin; i0 += BW) {
#pragma unroll
        for (int u = 0; u < BW; ++u) {
            rn1[u] = window_rows(dn1[u], base, false, a + (i0 + BW + u) * 64, rpg, N, node_off);
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
            const int nvalid = min(64, b_ - p);
            const float v = vc[u];
            const int row = rc[u];
            const int nxt = (u + 1 < BW) ? readlane(dc[u + 1], 0) : readlane(dn1[0], 0);
            cont = (p + nvalid < b_) ? (nxt == 0) : cont_end;
            const uint64_t sm = ballot(lane < nvalid && dc[u] != 0);
            if (sm == 0) {  // the window lies inside the open row
                const float t = wave_sum(v) - comp;
                const float s = carry + t;
                comp = (s - carry) - t;
                carry = s;
                if (!cont) {
                    if (lane == 0) {  // every lane holds the open row and its label
                        if (cur_row == head_row) headd[w] = carry;
                        else if (cur_row >= node_off && cur_row < node_off + N)
                            finish_node(cur_row, carry, yc[u], inv_of(yc[u]), diag, info, srow);
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
                float dsum = x;
                if (row == cur_row) dsum = carry + (x - comp);  // the open row's earlier windows first
                const bool ends = !(row == row_last && cont);
                if (ends) {
                    if (row == head_row) headd[w] = dsum;
                    else if (row >= node_off && row < node_off + N)
                        finish_node(row, dsum, yc[u], inv_of(yc[u]), diag, info, srow);
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

// Thread per wavefront: the degree of a row cut by wavefront boundaries, in wavefront order.
__global__ __launch_bounds__(256) void degree_fixup(Batch b, int NWtot, const int *__restrict__ rp,
                                                    const float *__restrict__ inv_n,
                                                    const float *__restrict__ headd,
                                                    const float *__restrict__ taild,
                                                    const int *__restrict__ dsplit, float2 *__restrict__ info,
                                                    float *__restrict__ srow) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= NWtot) return;
    GDesc gd;
    GMeta gm;
    int lw;
    if (!wave_graph(b, w, gd, gm, lw)) return;
    if (!(gd.weighted && (gd.flags & kLap))) return;
    const int r = dsplit[w];
    if (r < gd.node_off || r >= gd.node_off + gd.N) return;
    const int end = rp[r + 1];
    const int wl = (int)min((int64_t)gm.NW - 1, max((int64_t)lw, ((int64_t)(end - gm.ent_off) - 1) / gd.WE));
    float d = taild[w];
    for (int w2 = lw + 1; w2 <= wl; ++w2) d += headd[gd.wave_off + w2];
    int y = gd.labels[r - gd.node_off];
    if (y < 0 || y >= gd.K) y = -1;
    finish_node(r, d, y, y >= 0 ? inv_n[gd.class_off + y] : 0.0f, gd.flags & kDiag, info, srow);
}

// ----------------------------------------------------------------------------- empty rows

// Thread per row: a row without entries is zero, or holds the diagonal term alone
// (c_i s_i at its own class; 1 under correlation).
__global__ __launch_bounds__(256) void fill_empty(Batch b, int Ntot, const int *__restrict__ rp,
                                                  const float2 *__restrict__ info,
                                                  const float *__restrict__ srow) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= Ntot || rp[r] != rp[r + 1]) return;
    const int g = find_graph(b.node_offs, b.G, r);
    const GDesc d = load_desc(b, g);
    const bool lap = d.flags & kLap, diag = d.flags & kDiag, cor = d.flags & kCor;
    int y = -1;
    float v = 0.0f;
    if (diag) {
        const float2 inf = info[r];
        y = __float_as_int(inf.y);
        v = inf.x * (lap ? srow[r] : 1.0f);
        if (cor) v = v != 0.0f ? 1.0f : 0.0f;
    }
    float *z = d.Z + (int64_t)(r - d.node_off) * d.K;
    for (int k = 0; k < d.K; ++k) z[k] = (k == y) ? v : 0.0f;
}

// ----------------------------------------------------------------------------- finish a row

// Factor that turns a row's sums u (diagonal term included) into its Z row: s_i without
// correlation; with it u/|u|, since D^-1/2 scales the whole row by s_i > 0 and the 2-norm
// removes it (a row with s_i = 0 or u = 0 stays zero).
__device__ __forceinline__ float row_factor(float s, float ss, bool cor) {
    if (!cor) return s;
    return (s > 0.0f && ss > 0.0f) ? 1.0f / sqrtf(ss) : 0.0f;
}

// ----------------------------------------------------------------------------- main kernel

template <bool WEIGHTED>
__global__ __launch_bounds__(256) void embed_rows(Batch b, const int *__restrict__ rp, const int *__restrict__ col,
                                                  const float *__restrict__ val,
                                                  const uint8_t *__restrict__ rstep,
                                                  const float2 *__restrict__ info,
                                                  const float *__restrict__ srow,
                                                  const int *__restrict__ wrow, int lds_floats,
                                                  float *__restrict__ headp, float *__restrict__ tailp,
                                                  int *__restrict__ split, unsigned *status) {
    extern __shared__ float smem_f[];
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int w = blockIdx.x * wpb + wib;
    GDesc gd;
    GMeta gm;
    int lw;
    if (!wave_graph(b, w, gd, gm, lw)) return;  // whole wavefront leaves; no workgroup barrier below
    const unsigned flags = gd.flags;
    const bool diag = flags & kDiag, lap = flags & kLap, cor = flags & kCor;
    const int N = gd.N, K = gd.K, node_off = gd.node_off;
    const int KP = ring_stride(K);
    const int *rpg = rp + node_off;
    float *Z = gd.Z;
    float *headw = headp + gd.part_off + (int64_t)lw * K;
    float *tailw = tailp + gd.part_off + (int64_t)lw * K;

    // per wavefront: the ring acc[64 slots][KP] and per-slot row, s_i and finishing factor
    float *acc = smem_f + (size_t)wib * lds_floats;
    int *slot_row = reinterpret_cast<int *>(acc + 64 * KP);
    float *slot_s = reinterpret_cast<float *>(slot_row + 64);
    float *slot_f = slot_s + 64;
    for (int k = 0; k < KP; ++k) acc[lane * KP + k] = 0.0f;
    // Finished rows stay in their ring slots ("pending") until drain() stores them:
    // slots [pend_first, pend_first + npend) in ring order, just behind the open row.
    int npend = 0, pend_first = 0;

    const int E_end = gm.ent_off + gm.M;
    const int a = gm.ent_off + lw * gd.WE;
    const int b_ = min(a + gd.WE, E_end);
    const int last = b_ - 1;
    const int row_a = min(max(wrow[w], node_off), node_off + N - 1);
    // entry a continues a row begun before the wavefront / entry b continues the last row
    const bool head = __builtin_amdgcn_readfirstlane(rstep[a]) == 0;
    const int head_row = head ? row_a : -1;
    const bool cont_end = b_ < E_end && __builtin_amdgcn_readfirstlane(rstep[min(b_, E_end - 1)]) == 0;
    int cur_row = head ? row_a : -1;
    int cur_slot = 63;
    if (lane == 0) slot_row[63] = cur_row;
    bool cont = false;
    // this lane's (row, class) offset in the flat finishing pass, and its step per pass
    const int j0 = lane / K, k0 = lane - j0 * K;
    const int q64 = 64 / K, r64 = 64 - q64 * K;

    // Finish the pending rows and store them. First the factor of every pending row (one
    // lane per row: its sums read back with 16-byte LDS loads for the 2-norm), then a flat
    // pass over (row, class) in which consecutive lanes write consecutive words of Z. The
    // head row goes out raw. This code holds the only global stores and reads nothing
    // loaded from global memory, so it never waits for the loads in flight.
    auto drain = [&]() {
        wave_lds_fence();
        if (lane < npend) {
            const int sl = (pend_first + lane) & 63;
            float ss = 0.0f;
            if (cor) {
                const float4 *a4 = reinterpret_cast<const float4 *>(acc + sl * KP);
                for (int q = 0; q < (KP >> 2); ++q) {
                    const float4 t = a4[q];
                    ss += t.x * t.x + t.y * t.y + t.z * t.z + t.w * t.w;
                }
            }
            const float f = row_factor(lap ? slot_s[sl] : 1.0f, ss, cor);
            slot_f[sl] = slot_row[sl] == head_row ? 1.0f : f;
        }
        wave_lds_fence();
        const int F = npend * K;
        int jj = j0, kk = k0;
        for (int f0 = 0; f0 < F; f0 += 64) {
            const bool has = f0 + lane < F;
            const int sl = (pend_first + jj) & 63;
            const int ai = sl * KP + kk;
            const float v = acc[ai];
            const int r = slot_row[sl];
            const float fac = slot_f[sl];
            if (has) {
                acc[ai] = 0.0f;
                if (r >= node_off && r < node_off + N) {
                    float *dst = r == head_row ? headw + kk : Z + (int64_t)(r - node_off) * K + kk;
                    *dst = v * fac;
                }
            }
            kk += r64;
            jj += q64;
            if (kk >= K) {
                kk -= K;
                ++jj;
            }
        }
        npend = 0;
        wave_lds_fence();
    };

    // Loads are unconditional (clamped address, value masked afterwards) and are only
    // consumed in a later batch.
    const int nwin = (b_ - a + 63) >> 6;
    auto ld_col = [&](int e) { const int v = col[min(e, last)]; return e < b_ ? v : -1; };
    auto ld_val = [&](int e) { return WEIGHTED ? val[min(e, last)] : 1.0f; };
    auto ld_step = [&](int e) { const int v = rstep[min(e, last)]; return e < b_ ? v : 0; };
    auto gather_col = [&](int j) {
        const float2 f = info[min(max(j, node_off), node_off + N - 1)];
        return (unsigned)(j - node_off) < (unsigned)N ? f : make_float2(0.0f, __int_as_float(-1));
    };
    auto gather_row = [&](int r, float2 &q, float &sv) {
        const int rr = min(max(r, node_off), node_off + N - 1);
        q = info[rr];
        sv = lap ? srow[rr] : 1.0f;
    };
    int cn1[EBW], cn2[EBW], dc[EBW], dn1[EBW], dn2[EBW], rc[EBW], rn1[EBW];
    float vc[EBW], vn1[EBW], vn2[EBW], sc[EBW], sn1[EBW];
    float2 fc[EBW], fn1[EBW], qc[EBW], qn1[EBW];  // f: {c_j, y_j} by column; q: {c_i, y_i} by row
    bool bad = false;
    int base;
    int c0[EBW];
#pragma unroll
    for (int u = 0; u < EBW; ++u) {
        const int e0 = a + u * 64 + lane;
        c0[u] = ld_col(e0);
        vc[u] = ld_val(e0);
        dc[u] = ld_step(e0);
    }
#pragma unroll
    for (int u = 0; u < EBW; ++u) {
        const int e1 = a + (EBW + u) * 64 + lane;
        cn1[u] = ld_col(e1);
        vn1[u] = ld_val(e1);
        dn1[u] = ld_step(e1);
    }
#pragma unroll
    for (int u = 0; u < EBW; ++u) {
        bad |= a + u * 64 + lane < b_ && (unsigned)(c0[u] - node_off) >= (unsigned)N;
        fc[u] = gather_col(c0[u]);
    }
    base = row_a;
#pragma unroll
    for (int u = 0; u < EBW; ++u) {
        rc[u] = window_rows(dc[u], base, u == 0, a + u * 64, rpg, N, node_off);
        base = readlane(rc[u], 63);
        gather_row(rc[u], qc[u], sc[u]);
    }
    const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1);  // lanes <= this one

    for (int i0 = 0; i0 < nwin; i0 += EBW) {
        // Issue col/val/steps of batch k+2 first, then the rows and gathers of batch k+1
        // (which need the col/steps of batch k+1, loaded one iteration earlier). The
        // memory counter retires in issue order, so waiting for those col/steps here
        // leaves the gathers of batch k, issued after them, in flight.
#pragma unroll
        for (int u = 0; u < EBW; ++u) {
            const int e2 = a + (i0 + 2 * EBW + u) * 64 + lane;
            cn2[u] = ld_col(e2);
            vn2[u] = ld_val(e2);
            dn2[u] = ld_step(e2);
        }
#pragma unroll
        for (int u = 0; u < EBW; ++u) {
            const int e1 = a + (i0 + EBW + u) * 64 + lane;
            rn1[u] = window_rows(dn1[u], base, false, a + (i0 + EBW + u) * 64, rpg, N, node_off);
            base = readlane(rn1[u], 63);
            bad |= e1 < b_ && (unsigned)(cn1[u] - node_off) >= (unsigned)N;
            fn1[u] = gather_col(cn1[u]);
            gather_row(rn1[u], qn1[u], sn1[u]);
        }
        // process batch k
#pragma unroll
        for (int u = 0; u < EBW; ++u) {
            const int i = i0 + u;
            if (i >= nwin) break;
            const int p = a + (i << 6);
            const int nvalid = min(64, b_ - p);
            const bool valid = lane < nvalid;
            const int y = __float_as_int(fc[u].y);
            const float x = vc[u] * fc[u].x;
            const int nxt = (u + 1 < EBW) ? readlane(dc[u + 1], 0) : readlane(dn1[0], 0);
            cont = (p + nvalid < b_) ? (nxt == 0) : cont_end;
            const bool start = valid && dc[u] != 0;
            const uint64_t sm = ballot(start);
            const int nnew = __popcll(sm);
            // the open row and the new rows need ring slots next to the pending ones
            if (npend + 1 + nnew > 64) drain();
            const int slot = (cur_slot + __popcll(sm & le)) & 63;
            // A starting row gets its slot and, with augmentation, its diagonal term c_i
            // before any entry. Lanes with equal (row, class) add to the same LDS word;
            // the LDS applies them one after another in a fixed order, so the sums are
            // reproducible.
            if (start) {
                slot_row[slot] = rc[u];
                slot_s[slot] = sc[u];
                const int yi = __float_as_int(qc[u].y);
                if (diag && yi >= 0) atomicAdd(&acc[slot * KP + yi], qc[u].x);
            }
            if (valid && y >= 0) atomicAdd(&acc[slot * KP + y], x);
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
        for (int u = 0; u < EBW; ++u) {
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
        wave_lds_fence();
        float *dstp = (cur_row == head_row) ? headw : tailw;
        if (cur_row != head_row) my_split = cur_row;
        for (int k = lane; k < K; k += 64) dstp[k] = acc[cur_slot * KP + k];
    }
    if (lane == 0) split[w] = my_split;
}

// One wavefront per embed wavefront w: finish the row that starts in w and continues
// (its diagonal term is already in the tail partial).
__global__ __launch_bounds__(256) void embed_fixup(Batch b, int NWtot, const int *__restrict__ rp,
                                                   const float *__restrict__ srow,
                                                   const float *__restrict__ headp,
                                                   const float *__restrict__ tailp,
                                                   const int *__restrict__ split) {
    const int lane = lane_id();
    const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= NWtot) return;
    GDesc gd;
    GMeta gm;
    int lw;
    if (!wave_graph(b, w, gd, gm, lw)) return;
    const int r = split[w];
    if (r < gd.node_off || r >= gd.node_off + gd.N) return;
    const bool lap = gd.flags & kLap, cor = gd.flags & kCor;
    const int K = gd.K;
    const int end = rp[r + 1];
    const int wl = (int)min((int64_t)gm.NW - 1, max((int64_t)lw, ((int64_t)(end - gm.ent_off) - 1) / gd.WE));
    const float *part = tailp + gd.part_off;
    const float *heads = headp + gd.part_off;
    float v0 = 0.0f, v1 = 0.0f;
    if (lane < K) v0 = part[(int64_t)lw * K + lane];
    if (lane + 64 < K) v1 = part[(int64_t)lw * K + lane + 64];
    for (int w2 = lw + 1; w2 <= wl; ++w2) {
        if (lane < K) v0 += heads[(int64_t)w2 * K + lane];
        if (lane + 64 < K) v1 += heads[(int64_t)w2 * K + lane + 64];
    }
    const float s = lap ? srow[r] : 1.0f;
    const float ss = cor ? wave_sum(v0 * v0 + v1 * v1) : 0.0f;
    const float f = row_factor(s, ss, cor);
    float *z = gd.Z + (int64_t)(r - gd.node_off) * K;
    if (lane < K) z[lane] = v0 * f;
    if (lane + 64 < K) z[lane + 64] = v1 * f;
}

// ----------------------------------------------------------------------------- launch

size_t embed_lds_per_wave(int K) { return (size_t)embed_lds_floats(K) * sizeof(float); }

hipError_t launch_graph_meta(const Batch &b, const int *rp_of_union, int M, hipStream_t s) {
    prof_begin(kKGraphMeta, s);
    hipLaunchKernelGGL(graph_meta, dim3((unsigned)((b.G + 255) / 256)), dim3(256), 0, s, b, rp_of_union, M);
    prof_end(kKGraphMeta, s);
    return hipGetLastError();
}

// Per-node data for the embedding of a CSR: first rows of the wavefronts, row steps,
// degrees, s_i and c_i. The graph metadata must be set beforehand.
hipError_t launch_node_prep(const Batch &b, const Plan &p, const int *rp, const float *val, const Work &wk,
                            unsigned *status, hipStream_t s) {
    const int64_t nz = (p.Vtot + 16 * 256 - 1) / (16 * 256);
    prof_begin(kKZeroSteps, s);
    hipLaunchKernelGGL(zero_bytes, dim3((unsigned)(nz > 0 ? nz : 1)), dim3(256), 0, s, wk.rstep, p.Vtot);
    prof_end(kKZeroSteps, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nblk = (unsigned)((p.Ntot + 255) / 256);
    prof_begin(kKNodeRows, s);
    hipLaunchKernelGGL(node_rows, dim3(nblk > 0 ? nblk : 1), dim3(256), 0, s, b, (int)p.Ntot, rp, wk.inv_n,
                       wk.info, wk.srow, wk.wrow, wk.rstep, status);
    prof_end(kKNodeRows, s);
    if ((e = hipGetLastError()) != hipSuccess || !(val && p.any_lap_w)) return e;
    prof_begin(kKDegreeRows, s);
    hipLaunchKernelGGL(degree_rows, dim3((unsigned)((p.NWtot + 3) / 4)), dim3(256), 0, s, b, rp, val, wk.rstep,
                       wk.wrow, wk.inv_n, wk.info, wk.srow, wk.headd, wk.taild, wk.dsplit);
    prof_end(kKDegreeRows, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKDegreeFixup, s);
    hipLaunchKernelGGL(degree_fixup, dim3((unsigned)((p.NWtot + 255) / 256)), dim3(256), 0, s, b, (int)p.NWtot, rp,
                       wk.inv_n, wk.headd, wk.taild, wk.dsplit, wk.info, wk.srow);
    prof_end(kKDegreeFixup, s);
    return hipGetLastError();
}

hipError_t launch_embed(const Batch &b, const Plan &p, const int *rp, const int *col, const float *val,
                        const Work &wk, unsigned *status, hipStream_t s) {
    const int wpb = p.wpb;
    const unsigned grid = (unsigned)((p.NWtot + wpb - 1) / wpb);
    const int lds_floats = embed_lds_floats(p.Kmax);
    const size_t lds = (size_t)lds_floats * sizeof(float) * wpb;
    const unsigned nblk = (unsigned)((p.Ntot + 255) / 256);
    prof_begin(kKFillEmpty, s);
    hipLaunchKernelGGL(fill_empty, dim3(nblk > 0 ? nblk : 1), dim3(256), 0, s, b, (int)p.Ntot, rp, wk.info,
                       wk.srow);
    prof_end(kKFillEmpty, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    prof_begin(kKEmbedRows, s);
    if (val) {
        hipLaunchKernelGGL(embed_rows<true>, dim3(grid), dim3(64 * wpb), lds, s, b, rp, col, val, wk.rstep, wk.info,
                           wk.srow, wk.wrow, lds_floats, wk.headp, wk.tailp, wk.split, status);
    } else {
        hipLaunchKernelGGL(embed_rows<false>, dim3(grid), dim3(64 * wpb), lds, s, b, rp, col, val, wk.rstep,
                           wk.info, wk.srow, wk.wrow, lds_floats, wk.headp, wk.tailp, wk.split, status);
    }
    prof_end(kKEmbedRows, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKEmbedFixup, s);
    hipLaunchKernelGGL(embed_fixup, dim3((unsigned)((p.NWtot + 3) / 4)), dim3(256), 0, s, b, (int)p.NWtot, rp,
                       wk.srow, wk.headp, wk.tailp, wk.split);
    prof_end(kKEmbedFixup, s);
    return hipGetLastError();
}

}  // namespace gee
