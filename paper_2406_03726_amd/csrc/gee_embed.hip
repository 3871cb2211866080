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
//   * degree_rows  (weighted Laplacian) degrees as segmented sums over the same
//                  entry-balanced wavefronts and windows, then s_i; degree_fixup
//                  finishes cut rows and node_coef sets c_i from s_i.
//   * fill_empty   rows without entries (zero, or the diagonal term alone).
//   * embed_rows   wavefront w of a graph processes that graph's CSR entries
//                  [w*WE, (w+1)*WE) in windows of 256: lane l holds 4 consecutive
//                  entries, read with 16-byte loads. Every wavefront does the same work
//                  whatever the degree distribution. Rows are found without row_ptr
//                  lookups: a byte per entry holds the row step from the previous entry
//                  (0 inside a row; an escape value for steps >= 255), and one wave prefix
//                  sum per window turns the steps into row ids and counts the row starts.
//                  The loads of window k+2 and the gathers of window k+1 ({c_j, y_j} by
//                  column; {c_i, y_i}, s_i by row for entries that start a row) are in
//                  flight while window k is added, and nothing loaded is consumed in the
//                  window that loads it, so the memory pipeline never drains. Rows get
//                  slots of an LDS ring acc[slot][class] in the order they start; a
//                  starting row first receives its diagonal term, then every entry adds
//                  into acc[slot(row)][y_j] with an LDS float atomic, and the LDS applies
//                  lanes that hit the same word one after another in a fixed order, so
//                  results are bitwise reproducible. Rows ending in the wavefront are
//                  finished there (s_i, correlation) when the ring fills or the wavefront
//                  ends, and stored with coalesced writes; rows cut by wavefront
//                  boundaries leave raw partials.
//   * embed_fixup  adds the partials of each cut row in wavefront order and finishes it.
#include "gee_internal.h"

#include <climits>

namespace gee {

constexpr int kStepEsc = 255;  // row-step byte meaning "look the row up in row_ptr"
constexpr int EPL = 4;          // consecutive CSR entries per lane (embed_rows)
constexpr int EWIN = 64 * EPL;  // entries per embed window
#ifndef GEE_RING_SLOTS
#define GEE_RING_SLOTS 32
#endif
constexpr int RS = GEE_RING_SLOTS;  // row slots of an embed wavefront's LDS ring (16..64)
static_assert(RS >= 16 && RS <= 64 && (RS & (RS - 1)) == 0, "ring slots: power of two in [16, 64]");

// LDS floats of one embed wavefront: the ring [RS][ring_stride(K)] and per slot its row
// and s_i (later its finishing factor), with room to spare.
// The ring acc[RS][KP], its slot metadata (3 RS words) and a byte tag per ring word.
__host__ __device__ constexpr int embed_lds_floats(int K) {
    return RS * ring_stride(K) + 3 * RS + (RS * ring_stride(K) + 3) / 4;
}

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
            bad = true;  // (the row is skipped either way; only the report depends on validation)
        const bool lap = d.flags & kLap, diag = d.flags & kDiag;
        const bool skip = d.weighted && lap && hi > lo;
        int y = d.labels[rl];
        if (y < 0 || y >= d.K) y = -1;
        if (!skip) {
            float s = 1.0f;
            if (lap) {
                const float dg = (float)max(hi - lo, 0) + (diag ? 1.0f : 0.0f);
                s = dg > 0.0f ? 1.0f / sqrtf(dg) : 0.0f;
                srow[r] = s;
            }
            info[r] = node_info(y >= 0 ? s * inv_n[d.class_off + y] : 0.0f, y);
        } else {
            info[r] = node_info(0.0f, y);  // c_i follows from the weighted degree
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
    const bool report = bad && validates(load_desc(b, find_graph(b.node_offs, b.G, min(r, Ntot - 1))));
    if (__syncthreads_or(report) && threadIdx.x == 0) raise_error(status, kErrCsr);
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

// Rows of this lane's EPL consecutive entries e0 .. e0+3 of a window, from their step
// bytes d (byte j for entry e0 + j; 0 past the wavefront's entries): row = base + the
// inclusive sum of the steps over the window. In the wavefront's first window
// (`first_win`) lane 0's first entry keeps row `base` whatever its step says. An escape
// step's row is looked up in row_ptr and the later entries of the window follow from it.
// Also the inclusive count of row starts (non-zero steps) in the window, per entry, and
// stm (bit j: entry j starts a row). Returns the packed inclusive scan of the lane (steps
// in bits 0..19, starts above), so lane 63 holds the window's totals.
__device__ __forceinline__ int window_rows4(unsigned d, bool first_win, int base, int e0,
                                            const int *__restrict__ rpg, int N, int node_off,
                                            int (&r)[EPL], int (&n)[EPL], int &stm) {
    const int lane = lane_id();
    int sp[EPL], stp[EPL];
    int escm = 0;
    stm = 0;
#pragma unroll
    for (int j = 0; j < EPL; ++j) {
        const int dj = (int)((d >> (8 * j)) & 0xFFu);
        const bool first = (j == 0) && first_win && lane == 0;
        stm |= (dj != 0) << j;
        const bool esc = dj == kStepEsc && !first;
        escm |= esc << j;
        sp[j] = (esc || first) ? 0 : dj;
    }
    int rs = 0, cs = 0;
#pragma unroll
    for (int j = 0; j < EPL; ++j) {
        rs += sp[j];
        cs += (stm >> j) & 1;
        sp[j] = rs;
        stp[j] = cs;
    }
    // one scan for both: row steps in the low 20 bits (at most 64 * EPL * 254), starts above
    const int T = rs | (cs << 20);
    const int X = wave_scan_add(T);
    const int Xe = X - T;
    const int rb = base + (Xe & 0xFFFFF), nb0 = Xe >> 20;
#pragma unroll
    for (int j = 0; j < EPL; ++j) {
        r[j] = rb + sp[j];
        n[j] = nb0 + stp[j];
    }
    uint64_t em = ballot(escm != 0);
    if (em) {
        // rare: a run of >= 254 empty rows. Each escaped entry's row comes from row_ptr,
        // then every later entry of the window moves by the difference, in entry order.
        int ar[EPL];
#pragma unroll
        for (int j = 0; j < EPL; ++j) ar[j] = ((escm >> j) & 1) ? row_of_entry(rpg, N, e0 + j) + node_off : 0;
        while (em) {
            const int L = __builtin_ctzll(em);
            em &= em - 1;
            const int mL = readlane(escm, L);
#pragma unroll
            for (int j = 0; j < EPL; ++j) {
                if (!((mL >> j) & 1)) continue;
                const int delta = readlane(ar[j], L) - readlane(r[j], L);
#pragma unroll
                for (int jj = 0; jj < EPL; ++jj)
                    if (lane > L || (lane == L && jj >= j)) r[jj] += delta;
            }
        }
    }
    return X;
}

// ----------------------------------------------------------------------------- degrees

// Weighted degrees d_i = sum of the row's values over the same entry-balanced wavefronts
// and 256-entry windows as embed_rows (lane l holds 4 consecutive entries). In a window,
// each lane sums its entries row by row, a segmented wave scan (keyed by row) carries the
// sums across lanes, and the last entry of every row holds the row's sum over the window;
// a row open across windows keeps a compensated running sum. Summation order is fixed.
// Rows ending in the wavefront get s_i; a row cut by the wavefront's ends leaves its
// partial sums for degree_fixup. Wavefronts of graphs without weights or without the
// Laplacian leave at once.
__global__ __launch_bounds__(256) void degree_rows(Batch b, const int *__restrict__ rp,
                                                   const float *__restrict__ val, int64_t n_entries,
                                                   const uint8_t *__restrict__ rstep,
                                                   const int *__restrict__ wrow, float *__restrict__ srow,
                                                   float *__restrict__ headd, float *__restrict__ taild,
                                                   int *__restrict__ dsplit) {
    const int lane = lane_id();
    const int w = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    GDesc gd;
    GMeta gm;
    int lw;
    if (!wave_graph(b, w, gd, gm, lw)) return;
    if (!(gd.weighted && (gd.flags & kLap))) return;
    const bool diag = gd.flags & kDiag;
    const int N = gd.N, node_off = gd.node_off;
    const int *rpg = rp + node_off;
    const int E_end = gm.ent_off + gm.M;
    const int a = gm.ent_off + lw * gd.WE, b_ = min(a + gd.WE, E_end);
    const int row_a = min(max(wrow[w], node_off), node_off + N - 1);
    const bool head = __builtin_amdgcn_readfirstlane(rstep[a]) == 0;
    const int head_row = head ? row_a : -1;
    const bool cont_end = b_ < E_end && __builtin_amdgcn_readfirstlane(rstep[min(b_, E_end - 1)]) == 0;
    int cur_row = head ? row_a : -1;
    float carry = 0.0f, comp = 0.0f;  // running sum of the open row and its compensation
    bool cont = false;
    const int nwin = (b_ - a + EWIN - 1) / EWIN;
    const __amdgpu_buffer_rsrc_t r_val = buffer_rsrc(val + a, (n_entries - a) * 4);
    const __amdgpu_buffer_rsrc_t r_stp = buffer_rsrc(rstep + a, n_entries - a);
    auto load_win = [&](int i, float4 &v, unsigned &d) {
        const uint32_t o = (uint32_t)(i * EWIN + EPL * lane);
        if ((int64_t)a + (int64_t)(i + 1) * EWIN <= n_entries) {
            v = buf_f4(r_val, 4 * o);
            d = buf_u32(r_stp, o);
        } else {
            v = make_float4(__uint_as_float(buf_u32(r_val, 4 * o)), __uint_as_float(buf_u32(r_val, 4 * o + 4)),
                            __uint_as_float(buf_u32(r_val, 4 * o + 8)), __uint_as_float(buf_u32(r_val, 4 * o + 12)));
            d = buf_u8(r_stp, o) | (buf_u8(r_stp, o + 1) << 8) | (buf_u8(r_stp, o + 2) << 16) |
                (buf_u8(r_stp, o + 3) << 24);
        }
    };
    float4 v0, v1, v2;
    unsigned d0, d1 = 0, d2;
    load_win(0, v0, d0);
    if (nwin > 1) load_win(1, v1, d1);
    int base = row_a;
    for (int i = 0; i < nwin; ++i) {
        if (i + 2 < nwin) load_win(i + 2, v2, d2);
        const int p = a + i * EWIN;
        const int e0 = p + EPL * lane;
        float v[EPL] = {v0.x, v0.y, v0.z, v0.w};
        unsigned d = d0;
        if (p + EWIN > b_) {  // entries past b add nothing and start nothing
            const int nb = min(max(b_ - e0, 0), EPL);
            d = nb >= EPL ? d : (d & ((1u << (8 * nb)) - 1u));
#pragma unroll
            for (int j = 0; j < EPL; ++j)
                if (j >= nb) v[j] = 0.0f;
        }
        int r[EPL], n[EPL], stm;
        window_rows4(d, i == 0, base, e0, rpg, N, node_off, r, n, stm);
        base = readlane(r[EPL - 1], 63);
        // this lane's sums row by row, then across lanes for the row of its last entry
        float x[EPL];
        x[0] = v[0];
#pragma unroll
        for (int j = 1; j < EPL; ++j) x[j] = (r[j] == r[j - 1]) ? x[j - 1] + v[j] : v[j];
        const float S = wave_seg_scan_addf(x[EPL - 1], r[EPL - 1]);
        const float Sp = dpp_f<0x138>(S, 0.0f);         // wave_shr:1, lane l gets lane l-1
        const int rp3 = dpp_i<0x138>(r[EPL - 1], INT32_MIN);
        const int rn0 = dpp_i<0x130>(r[0], INT32_MAX);  // wave_shl:1, lane l gets lane l+1
        const bool last_win = p + EWIN >= b_;
        const bool cw = last_win ? cont_end : ((readlane((int)d1, 0) & 0xFF) == 0);
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
            // the sum of row r[j] from the window's start through entry j
            const float t = (r[j] == rp3 && r[j] == r[0]) ? Sp + x[j] : x[j];
            const bool ends = (j + 1 < EPL) ? r[j + 1] != r[j] : (lane < 63 ? rn0 != r[j] : !cw);
            if (ends) {
                const float dsum = (r[j] == cur_row) ? carry + (t - comp) : t;
                if (r[j] == head_row) headd[w] = dsum;
                else if (r[j] >= node_off && r[j] < node_off + N) finish_degree(r[j], dsum, diag, srow);
            }
        }
        // the row of the window's last entry, when it continues into the next window
        const float tail = readlane_f(S, 63);
        const int rl = base;
        if (cw) {
            if (rl == cur_row) {
                const float y = tail - comp;
                const float tt = carry + y;
                comp = (tt - carry) - y;
                carry = tt;
            } else {
                carry = tail;
                comp = 0.0f;
            }
        } else {
            carry = comp = 0.0f;
        }
        cur_row = rl;
        cont = cw;
        v0 = v1;
        d0 = d1;
        v1 = v2;
        d1 = d2;
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
                                                    const float *__restrict__ headd,
                                                    const float *__restrict__ taild,
                                                    const int *__restrict__ dsplit, float *__restrict__ srow) {
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
    finish_degree(r, d, gd.flags & kDiag, srow);
}

// Thread per row of a weighted graph with the Laplacian: c_i = s_i / n_{y_i} once the
// weighted degrees are known (other rows got theirs in node_rows).
__global__ __launch_bounds__(256) void node_coef(Batch b, int Ntot, const int *__restrict__ rp,
                                                 const float *__restrict__ inv_n, const float *__restrict__ srow,
                                                 float2 *__restrict__ info) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= Ntot) return;
    const int g = find_graph(b.node_offs, b.G, r);
    const GDesc d = load_desc(b, g);
    if (!(d.weighted && (d.flags & kLap)) || rp[r] == rp[r + 1]) return;
    int y = d.labels[r - d.node_off];
    if (y < 0 || y >= d.K) y = -1;
    info[r] = node_info(y >= 0 ? srow[r] * inv_n[d.class_off + y] : 0.0f, y);
}

// ----------------------------------------------------------------------------- empty rows

// Rows without entries: zero, or the diagonal term alone (c_i s_i at its own class; 1
// under correlation). A workgroup takes 256 consecutive rows; when they belong to one
// graph (their Z rows are then contiguous) the empty ones are written in one flat pass
// over (row, class), consecutive threads on consecutive words; else a thread per row.
__global__ __launch_bounds__(256) void fill_empty(Batch b, int Ntot, const int *__restrict__ rp,
                                                  const float2 *__restrict__ info,
                                                  const float *__restrict__ srow) {
    __shared__ int s_y[256];
    __shared__ float s_v[256];
    const int t = threadIdx.x;
    const int r0 = blockIdx.x * 256;
    const int r = r0 + t;
    const int nrows = min(256, Ntot - r0);
    const bool empty = r < Ntot && rp[r] == rp[r + 1];
    int y = -2;  // -2: not empty (nothing to write)
    float v = 0.0f;
    GDesc d;
    if (empty) {
        d = load_desc(b, find_graph(b.node_offs, b.G, r));
        const bool lap = d.flags & kLap, diag = d.flags & kDiag, cor = d.flags & kCor;
        y = -1;
        if (diag) {
            const float2 inf = info[r];
            y = __float_as_int(inf.y);
            v = inf.x * (lap ? srow[r] : 1.0f);
            if (cor) v = v != 0.0f ? 1.0f : 0.0f;
        }
    }
    s_y[t] = y;
    s_v[t] = v;
    const int g0 = find_graph(b.node_offs, b.G, r0);
    const bool one_graph = find_graph(b.node_offs, b.G, r0 + nrows - 1) == g0;
    if (!__syncthreads_or(empty)) return;
    if (!one_graph) {
        if (empty) {
            float *z = d.Z + (int64_t)(r - d.node_off) * d.K;
            for (int k = 0; k < d.K; ++k) z[k] = (k == y) ? v : 0.0f;
        }
        return;
    }
    const GDesc dg = load_desc(b, g0);
    const int K = dg.K;
    float *z0 = dg.Z + (int64_t)(r0 - dg.node_off) * K;
    const int F = nrows * K;
    const int q = 256 / K, rq = 256 - q * K;
    int j = t / K, k = t - (t / K) * K;
    for (int f = t; f < F; f += 256) {
        const int yj = s_y[j];
        if (yj != -2) __builtin_nontemporal_store(k == yj ? s_v[j] : 0.0f, z0 + f);
        k += rq;
        j += q;
        if (k >= K) {
            k -= K;
            ++j;
        }
    }
}

// ----------------------------------------------------------------------------- finish a row


// ----------------------------------------------------------------------------- main kernel

// One window of a wavefront as loaded: lane l holds entries p + 4l .. p + 4l + 3.
struct WinRaw {
    int4 c;
    float4 v;
    unsigned d;  // the four step bytes
};
// A window ready to be added: weights, gathered {c_j, y_j} by column, rows, the running
// count of row starts, and for starting entries {c_i, y_i} and s_i of their row.
struct WinPrep {
    float v[EPL];
    float2 f[EPL];
    int r[EPL], n[EPL];
    int stm;  // bit j: entry j starts a row
    float2 q[EPL];
    float s[EPL];
    int nnew;   // row starts in the window
    int rlast;  // row of the window's last entry
};

#ifndef GEE_EMBED_MIN_WAVES
#define GEE_EMBED_MIN_WAVES 1
#endif
template <bool WEIGHTED>
__global__ __launch_bounds__(256, GEE_EMBED_MIN_WAVES) void embed_rows(Batch b, const int *__restrict__ rp, const int *__restrict__ col,
                                                  const float *__restrict__ val, int64_t n_entries,
                                                  const uint8_t *__restrict__ rstep,
                                                  const float2 *__restrict__ info,
                                                  const float *__restrict__ srow,
                                                  const int *__restrict__ wrow, int lds_floats,
                                                  float *__restrict__ headp, float *__restrict__ tailp,
                                                  int *__restrict__ split, unsigned *status) {
    extern __shared__ float smem_f[];
    const int lane = lane_id();
    // wavefront-uniform (so descriptors, sizes and buffer resources live in SGPRs)
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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

    // per wavefront: the ring acc[RS slots][KP] and per slot its row and s_i
    float *acc = smem_f + (size_t)wib * lds_floats;
    int2 *slot_meta = reinterpret_cast<int2 *>(acc + RS * KP);  // {row, s_i}, then {row, factor}
    unsigned char *tag = reinterpret_cast<unsigned char *>(acc + RS * KP + 3 * RS);  // [RS * KP]
    {
        float4 *acc4 = reinterpret_cast<float4 *>(acc);
        for (int i = lane; i < ((RS * KP) >> 2); i += 64) acc4[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    // Finished rows stay in their ring slots ("pending") until drain() stores them:
    // slots [pend_first, pend_first + npend) in ring order, just behind the open row.
    // Draining only when the ring is full, and at the end, lets one drain serve many rows
    // (its fixed cost, the lane-per-row norm pass, is paid per drain, not per row).
    int npend = 0, pend_first = 0;

    const int E_end = gm.ent_off + gm.M;
    const int a = gm.ent_off + lw * gd.WE;
    const int b_ = min(a + gd.WE, E_end);
    const int row_a = min(max(wrow[w], node_off), node_off + N - 1);
    // entry a continues a row begun before the wavefront / entry b continues the last row
    const bool head = __builtin_amdgcn_readfirstlane(rstep[a]) == 0;
    const int head_row = head ? row_a : -1;
    const bool cont_end = b_ < E_end && __builtin_amdgcn_readfirstlane(rstep[min(b_, E_end - 1)]) == 0;
    int cur_row = head ? row_a : -1;
    int cur_slot = RS - 1;
    if (lane == 0) slot_meta[RS - 1] = make_int2(cur_row, __float_as_int(1.0f));
    bool cont = false;
    // this lane's (row, class) offset in the flat finishing pass, and its step per pass
    const int j0 = lane / K, k0 = lane - j0 * K;
    const int q64 = 64 / K, r64 = 64 - q64 * K;

    // Finish the pending rows and store them. First the factor of every pending row (one
    // lane per row: its sums read back with 16-byte LDS loads for the 2-norm), then a flat
    // pass over (row, class) in which consecutive lanes read consecutive classes and write
    // consecutive words of Z, then the drained slots are cleared. The head row goes out
    // raw. This code holds the only global stores and reads nothing loaded from global
    // memory, so it never waits for the loads in flight. Z is written with non-temporal
    // stores: it is not read again here, and keeping it out of the L2 leaves room for the
    // gathered per-node table.
    auto drain = [&]() {
        wave_lds_fence();
        float fac = 0.0f;
        int rrow = -1;
        if (lane < npend) {
            const int sl = (pend_first + lane) & (RS - 1);
            const int2 m = slot_meta[sl];
            float ss = 0.0f;
            if (cor) {
                const float4 *a4 = reinterpret_cast<const float4 *>(acc + sl * KP);
                for (int q = 0; q < (KP >> 2); ++q) {
                    const float4 t = a4[q];
                    ss += t.x * t.x + t.y * t.y + t.z * t.z + t.w * t.w;
                }
            }
            rrow = m.x;
            fac = rrow == head_row ? 1.0f : row_factor(lap ? __int_as_float(m.y) : 1.0f, ss, cor);
        }
        // flat pass over (row, class): consecutive lanes write consecutive words of Z; each
        // lane reads its row and factor as one pair
        if (lane < npend) slot_meta[(pend_first + lane) & (RS - 1)].y = __float_as_int(fac);
        wave_lds_fence();
        const int F = npend * K;
        int jj = j0, kk = k0;
        for (int f0 = 0; f0 < F; f0 += 64) {
            const bool has = f0 + lane < F;
            const int sl = (pend_first + jj) & (RS - 1);
            const float v = acc[sl * KP + kk];
            const int2 m = slot_meta[sl];
            if (has && m.x >= node_off && m.x < node_off + N) {
                float *dst = m.x == head_row ? headw + kk : Z + (int64_t)(m.x - node_off) * K + kk;
                __builtin_nontemporal_store(v * __int_as_float(m.y), dst);
            }
            kk += r64;
            jj += q64;
            if (kk >= K) {
                kk -= K;
                ++jj;
            }
        }
        // clear the drained slots (one or two contiguous runs of the ring) with 16-byte writes
        {
            const int KQ = KP >> 2;
            float4 *acc4 = reinterpret_cast<float4 *>(acc);
            const int n1 = min(npend, RS - pend_first) * KQ, n2 = npend * KQ - n1;
            const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            for (int q = lane; q < n1; q += 64) acc4[pend_first * KQ + q] = z4;
            for (int q = lane; q < n2; q += 64) acc4[q] = z4;
        }
        npend = 0;
        wave_lds_fence();
    };

    // Streams over the wavefront's entries and the gathered per-node tables. Offsets are
    // relative to entry a; a window wholly inside the arrays is read with 16-byte loads,
    // the others entry by entry (past the end the loads return 0).
    const __amdgpu_buffer_rsrc_t r_col = buffer_rsrc(col + a, (n_entries - a) * 4);
    const __amdgpu_buffer_rsrc_t r_val = buffer_rsrc(WEIGHTED ? (const void *)(val + a) : (const void *)(col + a), (n_entries - a) * 4);
    const __amdgpu_buffer_rsrc_t r_stp = buffer_rsrc(rstep + a, n_entries - a);
    const __amdgpu_buffer_rsrc_t r_inf = buffer_rsrc(info + node_off, (int64_t)N * 8);
    const __amdgpu_buffer_rsrc_t r_srw = buffer_rsrc(srow + node_off, (int64_t)N * 4);
    const int nwin = (b_ - a + EWIN - 1) / EWIN;

    auto load_win = [&](int i, WinRaw &R) {
        const uint32_t o = (uint32_t)(i * EWIN + EPL * lane);
        if ((int64_t)a + (int64_t)(i + 1) * EWIN <= n_entries) {
            R.c = buf_i4(r_col, 4 * o);
            if (WEIGHTED) R.v = buf_f4(r_val, 4 * o);
            R.d = buf_u32(r_stp, o);
        } else {
            R.c = make_int4((int)buf_u32(r_col, 4 * o), (int)buf_u32(r_col, 4 * o + 4),
                            (int)buf_u32(r_col, 4 * o + 8), (int)buf_u32(r_col, 4 * o + 12));
            if (WEIGHTED)
                R.v = make_float4(__uint_as_float(buf_u32(r_val, 4 * o)), __uint_as_float(buf_u32(r_val, 4 * o + 4)),
                                  __uint_as_float(buf_u32(r_val, 4 * o + 8)),
                                  __uint_as_float(buf_u32(r_val, 4 * o + 12)));
            R.d = buf_u8(r_stp, o) | (buf_u8(r_stp, o + 1) << 8) | (buf_u8(r_stp, o + 2) << 16) |
                  (buf_u8(r_stp, o + 3) << 24);
        }
    };

    bool bad = false;
    int base = row_a;  // row of the last entry of the windows prepared so far

    // Rows, row-start counts and gathers of window i. Entries past b are masked: no step,
    // no start, a column whose gather returns 0 and a weight of 0, so they add nothing.
    auto prep_win = [&](int i, const WinRaw &R, WinPrep &P) {
        const int p = a + i * EWIN;
        const int e0 = p + EPL * lane;
        int c[EPL] = {R.c.x, R.c.y, R.c.z, R.c.w};
        float v[EPL] = {R.v.x, R.v.y, R.v.z, R.v.w};
        unsigned d = R.d;
        unsigned u[EPL];
#pragma unroll
        for (int j = 0; j < EPL; ++j) u[j] = (unsigned)(c[j] - node_off);
        if (p + EWIN <= b_) {
#pragma unroll
            for (int j = 0; j < EPL; ++j) bad |= u[j] >= (unsigned)N;
        } else {
            const int nb = min(max(b_ - e0, 0), EPL);
            d = nb >= EPL ? d : (d & ((1u << (8 * nb)) - 1u));
#pragma unroll
            for (int j = 0; j < EPL; ++j) {
                if (j < nb) {
                    bad |= u[j] >= (unsigned)N;
                } else {
                    u[j] = 0xFFFFFFFFu;
                    v[j] = 0.0f;
                }
            }
        }
        int stm;
        const int X = window_rows4(d, i == 0, base, e0, rpg, N, node_off, P.r, P.n, stm);
        P.stm = stm;
        P.nnew = readlane(X, 63) >> 20;
        P.rlast = readlane(P.r[EPL - 1], 63);
        base = P.rlast;
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
            P.v[j] = v[j];
            P.f[j] = buf_f2(r_inf, u[j] << 3);
        }
        if (diag || lap) {
#pragma unroll
            for (int j = 0; j < EPL; ++j) {
                if ((stm >> j) & 1) {
                    const uint32_t ri = (uint32_t)(P.r[j] - node_off);
                    if (diag) P.q[j] = buf_f2(r_inf, ri << 3);
                    if (lap) P.s[j] = __uint_as_float(buf_u32(r_srw, ri << 2));
                }
            }
        }
    };

    // Adds the entries of lanes [lo, hi) of a prepared window; n0 = row starts before
    // lane lo. A starting row first gets its slot, s_i and diagonal term c_i (a plain
    // write: LDS operations of a wavefront take effect in order), then every entry adds
    // into acc[slot(row)][y_j] (lds_tag_add: a fixed order per word, so the sums are
    // reproducible). Then the rows that ended become pending.
    auto add_lanes = [&](const WinPrep &P, int lo, int hi, int n0, int nn, bool st0, bool cnt) {
        if (npend + 1 + nn > RS) drain();
        const bool act = lane >= lo && lane < hi;
        int sl[EPL];
#pragma unroll
        for (int j = 0; j < EPL; ++j) sl[j] = (cur_slot + P.n[j] - n0) & (RS - 1);
        if (act) {
#pragma unroll
            for (int j = 0; j < EPL; ++j) {
                if ((P.stm >> j) & 1) {
                    slot_meta[sl[j]] = make_int2(P.r[j], __float_as_int(lap ? P.s[j] : 1.0f));
                    // the slot is clear and no entry of the row has been added yet
                    const int ya = sl[j] * KP + __float_as_int(P.q[j].y);
                    if (diag && dbg_ok(ya >= 0 && ya < RS * KP, status)) acc[ya] = P.q[j].x;
                }
            }
        }
        {
            int ad[EPL];
            float xv[EPL];
#pragma unroll
            for (int j = 0; j < EPL; ++j) {
                ad[j] = sl[j] * KP + __float_as_int(P.f[j].y);
                xv[j] = act ? (WEIGHTED ? P.v[j] * P.f[j].x : P.f[j].x) : 0.0f;
            }
            lds_tag_add<EPL>(acc, tag, ad, xv, lane, -1, RS * KP, status);
        }
        // segments of this range: the open row unless the range starts a row, then the
        // new rows; all but the last end here, the last unless the next entry continues it
        const int first_slot = st0 ? (cur_slot + 1) & (RS - 1) : cur_slot;
        const int nseg = nn + (st0 ? 0 : 1);
        const int nend = cnt ? nseg - 1 : nseg;
        if (nend > 0) {
            if (npend == 0) pend_first = first_slot;
            npend += nend;
        }
        cur_slot = (cur_slot + nn) & (RS - 1);
    };

    // Whether the entry at index e (first entry of lane L of the prepared window P, or
    // b or later) continues the row of the entry before it.
    auto continues = [&](int e, const WinPrep &P, int L) {
        return e >= b_ ? cont_end : !(readlane(P.stm, L) & 1);
    };

    auto process = [&](int i, const WinPrep &P, const WinPrep &Pn) {
        const int p = a + i * EWIN;
        const bool st0 = readlane(P.stm, 0) & 1;
        const bool cw = continues(p + EWIN, Pn, 0);
        if (P.nnew + (st0 ? 0 : 1) <= RS) {
            add_lanes(P, 0, 64, 0, P.nnew, st0, cw);
            cur_row = P.rlast;
            cont = cw;
            return;
        }
        // more row starts than ring slots: ranges of RS / EPL lanes (at most RS entries, so
        // at most RS starts each), draining in between
        constexpr int GL = RS / EPL, NG = 64 / GL;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int lo = GL * g, hi = lo + GL;
            if (p + EPL * lo >= b_) break;
            const int n0 = g ? readlane(P.n[EPL - 1], lo - 1) : 0;
            const int nn = readlane(P.n[EPL - 1], hi - 1) - n0;
            const bool s0 = readlane(P.stm, lo) & 1;
            const bool cg = (g < NG - 1) ? continues(p + EPL * hi, P, hi) : cw;
            add_lanes(P, lo, hi, n0, nn, s0, cg);
            cur_row = readlane(P.r[EPL - 1], hi - 1);
            cont = cg;
        }
    };

    WinRaw R1, R2;
    WinPrep P0, P1;
    R1.v = R2.v = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
    load_win(0, R2);
    if (nwin > 1) load_win(1, R1);
    prep_win(0, R2, P0);
    for (int i = 0; i < nwin; ++i) {
        // Issue the loads of window i+2 first, then the rows and gathers of window i+1
        // (which need the loads of window i+1, issued one iteration earlier). The memory
        // counter retires in issue order, so waiting for those leaves the gathers of
        // window i, issued after them, in flight.
        if (i + 2 < nwin) load_win(i + 2, R2);
        if (i + 1 < nwin) {
            prep_win(i + 1, R1, P1);
        } else {
            P1.stm = 0;
        }
        process(i, P0, P1);
        P0 = P1;
        R1 = R2;
    }
    if (ballot(bad) && lane == 0 && validates(gd)) raise_error(status, kErrCsr);

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
hipError_t launch_node_prep(const Batch &b, const Plan &p, const int *rp, const float *val, int64_t n_entries,
                            const Work &wk, unsigned *status, hipStream_t s) {
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
    hipLaunchKernelGGL(degree_rows, dim3((unsigned)((p.NWtot + 3) / 4)), dim3(256), 0, s, b, rp, val, n_entries,
                       wk.rstep, wk.wrow, wk.srow, wk.headd, wk.taild, wk.dsplit);
    prof_end(kKDegreeRows, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKDegreeFixup, s);
    hipLaunchKernelGGL(degree_fixup, dim3((unsigned)((p.NWtot + 255) / 256)), dim3(256), 0, s, b, (int)p.NWtot, rp,
                       wk.headd, wk.taild, wk.dsplit, wk.srow);
    prof_end(kKDegreeFixup, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prof_begin(kKNodeCoef, s);
    hipLaunchKernelGGL(node_coef, dim3(nblk > 0 ? nblk : 1), dim3(256), 0, s, b, (int)p.Ntot, rp, wk.inv_n, wk.srow,
                       wk.info);
    prof_end(kKNodeCoef, s);
    return hipGetLastError();
}

hipError_t launch_embed(const Batch &b, const Plan &p, const int *rp, const int *col, const float *val,
                        int64_t n_entries, const Work &wk, unsigned *status, hipStream_t s) {
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
        hipLaunchKernelGGL(embed_rows<true>, dim3(grid), dim3(64 * wpb), lds, s, b, rp, col, val, n_entries, wk.rstep, wk.info,
                           wk.srow, wk.wrow, lds_floats, wk.headp, wk.tailp, wk.split, status);
    } else {
        hipLaunchKernelGGL(embed_rows<false>, dim3(grid), dim3(64 * wpb), lds, s, b, rp, col, val, n_entries, wk.rstep,
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
