// gee_edge.hip - the original GEE form (Section 2: the embedding computed straight from the
// edge list, one pass over its rows, without a CSR). Every row (i, j, e_ij) adds e_ij / n_{y_j}
// to Z[i, y_j] with a float atomic, so the summation order, and with it the last bits of Z,
// changes from call to call; the sparse (CSR / bucket) paths are the deterministic ones.
//
// Launches (all grid-stride, 256 threads):
//   edge_init     Z = 0, degrees = 1 under diagonal augmentation (else 0), class counts = 0
//   edge_prep     class counts (label range check) in the first workgroups; under the
//                 Laplacian, weighted degrees d_i = sum_j (A [+ I])_ij by float atomics (and,
//                 with directed degrees, the in-degrees sum_i (A [+ I])_ij as well)
//   edge_coef     per node: s_j = d_j^-1/2 (0 for d_j <= 0; 1 without the Laplacian) and
//                 c_j = s_j / n_{y_j} (0 for an unknown label or an empty class); with
//                 directed degrees c_j takes the in-degree's inverse square root instead
//   edge_scatter  per edge row: Z[s, y_d] += e c_d and, for undirected input, Z[d, y_s] += e c_s
//   edge_finish   per Z row: the diagonal term c_i at k = y_i, the row factor s_i (Table 1,
//                 Laplacian row) and the row 2-norm (correlation)
#include "gee.h"
#include "gee_internal.h"

#include <cstring>

namespace gee {
namespace {

constexpr int kEB = 256;  // threads per workgroup of every launch here

__device__ __forceinline__ bool finite_f(float x) { return (__float_as_uint(x) & 0x7f800000u) != 0x7f800000u; }

// Z = 0 (16-byte stores on the aligned body), degrees = d0, class counts = 0.
__global__ __launch_bounds__(kEB) void edge_init(float *__restrict__ Z, int64_t nz, float *__restrict__ deg,
                                               float *__restrict__ degin, int N, float d0, int *__restrict__ counts,
                                               int K) {
    const int64_t tid = (int64_t)blockIdx.x * kEB + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * kEB;
    const int64_t head = (int64_t)((16u - ((unsigned)(uintptr_t)Z & 15u)) & 15u) / 4;  // Z is 4-byte aligned
    const int64_t h = head < nz ? head : nz;
    const int64_t n4 = (nz - h) / 4;
    float4 *Z4 = reinterpret_cast<float4 *>(Z + h);
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t i = tid; i < n4; i += nth) Z4[i] = z4;
    if (tid < h) Z[tid] = 0.f;
    const int64_t t0 = h + 4 * n4;
    if (tid < nz - t0) Z[t0 + tid] = 0.f;
    if (deg)
        for (int64_t i = tid; i < N; i += nth) deg[i] = d0;
    if (degin)
        for (int64_t i = tid; i < N; i += nth) degin[i] = d0;
    if (tid < K) counts[tid] = 0;
}

// Workgroups [0, cblocks): class counts of contiguous label slices (LDS histogram, then one
// integer atomic per class and workgroup). Workgroups [cblocks, ...): under the Laplacian,
// the weighted degree of both endpoints of every edge row (one of a self-loop). Rows with
// an endpoint out of range or a non-finite weight are skipped here; edge_scatter reports them.
__global__ __launch_bounds__(kEB) void edge_prep(const int *__restrict__ labels, int N, int K, int cblocks,
                                               int *__restrict__ counts, const int *__restrict__ src,
                                               const int *__restrict__ dst, const float *__restrict__ w,
                                               int64_t E, bool sym, float *__restrict__ deg,
                                               float *__restrict__ degin, unsigned *status) {
    __shared__ int hist[kMaxClasses];
    if ((int)blockIdx.x < cblocks) {
        for (int k = threadIdx.x; k < K; k += kEB) hist[k] = 0;
        __syncthreads();
        const int64_t per = ((int64_t)N + cblocks - 1) / cblocks;
        const int64_t lo = (int64_t)blockIdx.x * per;
        const int64_t hi = lo + per < N ? lo + per : N;
        bool bad = false;
        for (int64_t i = lo + threadIdx.x; i < hi; i += kEB) {
            const int y = labels[i];
            if (y >= 0 && y < K)
                atomicAdd(&hist[y], 1);
            else if (y != -1)
                bad = true;
        }
        if (ballot(bad) && lane_id() == 0) raise_error(status, kErrLabel);
        __syncthreads();
        for (int k = threadIdx.x; k < K; k += kEB)
            if (hist[k]) atomicAdd(&counts[k], hist[k]);
        return;
    }
    const int64_t nth = (int64_t)(gridDim.x - cblocks) * kEB;
    for (int64_t e = (int64_t)(blockIdx.x - cblocks) * kEB + threadIdx.x; e < E; e += nth) {
        const int s = src[e], d = dst[e];
        const float x = w ? w[e] : 1.0f;
        if ((unsigned)s >= (unsigned)N || (unsigned)d >= (unsigned)N || !finite_f(x)) continue;
        unsafeAtomicAdd(&deg[s], x);
        if (sym && s != d) unsafeAtomicAdd(&deg[d], x);
        if (degin) unsafeAtomicAdd(&degin[d], x);
    }
}

// Per node: info[j] = {c_j, y_j (-1 when unknown or out of range)}, and the row factor s_j
// written over the degree in place.
__global__ __launch_bounds__(kEB) void edge_coef(const int *__restrict__ labels, int N, int K,
                                               const int *__restrict__ counts, float *__restrict__ deg_s,
                                               const float *__restrict__ degin, float2 *__restrict__ info) {
    const int64_t nth = (int64_t)gridDim.x * kEB;
    for (int64_t j = (int64_t)blockIdx.x * kEB + threadIdx.x; j < N; j += nth) {
        const int y = labels[j];
        const bool known = y >= 0 && y < K;
        const int n = known ? counts[y] : 0;
        float s = 1.0f;
        if (deg_s) {
            const float d = deg_s[j];
            s = d > 0.0f ? 1.0f / sqrtf(d) : 0.0f;
            deg_s[j] = s;
        }
        if (degin) {
            const float d = degin[j];
            s = d > 0.0f ? 1.0f / sqrtf(d) : 0.0f;  // the column factor (in-degree)
        }
        const float c = n > 0 ? s / (float)n : 0.0f;
        info[j] = make_float2(c, __int_as_float(known && c != 0.0f ? y : -1));
    }
}

// Per edge row: the gathered coefficient of the other endpoint, times the weight, added to
// the endpoint's Z entry of that neighbour's class. Four rows per thread and iteration, so
// the loads of four rows are in flight before their atomics issue.
__global__ __launch_bounds__(kEB) void edge_scatter(const int *__restrict__ src, const int *__restrict__ dst,
                                                  const float *__restrict__ w, int64_t E, int N, int K, bool sym,
                                                  const float2 *__restrict__ info, float *__restrict__ Z,
                                                  unsigned *status) {
    constexpr int U = 4;
    const int64_t nth = (int64_t)gridDim.x * kEB;
    bool bad_i = false, bad_w = false;
    for (int64_t e0 = (int64_t)blockIdx.x * kEB + threadIdx.x; e0 < E; e0 += U * nth) {
        int s[U], d[U];
        float x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * nth;
            const bool in = e < E;
            s[u] = in ? src[e] : -1;
            d[u] = in ? dst[e] : -1;
            x[u] = in ? (w ? w[e] : 1.0f) : 0.0f;
            if (!in) continue;
            if ((unsigned)s[u] >= (unsigned)N || (unsigned)d[u] >= (unsigned)N) {
                bad_i = true;
                s[u] = -1;
            } else if (status && !finite_f(x[u])) {
                bad_w = true;
                s[u] = -1;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (s[u] < 0) continue;
            const float2 id = info[d[u]];
            const int yd = __float_as_int(id.y);
            if (yd >= 0) unsafeAtomicAdd(&Z[(int64_t)s[u] * K + yd], x[u] * id.x);
            if (sym && s[u] != d[u]) {
                const float2 is = info[s[u]];
                const int ys = __float_as_int(is.y);
                if (ys >= 0) unsafeAtomicAdd(&Z[(int64_t)d[u] * K + ys], x[u] * is.x);
            }
        }
    }
    if (ballot(bad_i) && lane_id() == 0) raise_error(status, kErrIndex);
    if (ballot(bad_w) && lane_id() == 0) raise_error(status, kErrWeight);
}

// One group of L lanes per Z row (L = the power of two at or above min(K, 64), so a
// wavefront covers 64 / L rows and each lane at most two columns of its row).
template <int L>
__global__ __launch_bounds__(kEB) void edge_finish(float *__restrict__ Z, int N, int K, const float *__restrict__ s_of,
                                                 const float2 *__restrict__ info, bool diag, bool cor) {
    constexpr int RPW = kEB / L;  // rows per workgroup and iteration
    const int sub = threadIdx.x % L;
    for (int64_t i = (int64_t)blockIdx.x * RPW + threadIdx.x / L; i < N; i += (int64_t)gridDim.x * RPW) {
        const float s = s_of ? s_of[i] : 1.0f;
        const float2 ii = info[i];
        const int yi = diag ? __float_as_int(ii.y) : -1;
        float *row = Z + i * K;
        const int k0 = sub, k1 = sub + L;
        float z0 = 0.0f, z1 = 0.0f;
        if (k0 < K) z0 = (row[k0] + (k0 == yi ? ii.x : 0.0f)) * s;
        if (k1 < K) z1 = (row[k1] + (k1 == yi ? ii.x : 0.0f)) * s;
        if (cor) {
            float ss = z0 * z0 + z1 * z1;
#pragma unroll
            for (int o = L / 2; o > 0; o >>= 1) ss += __shfl_xor(ss, o, L);
            if (ss > 0.0f) {
                const float r = sqrtf(ss);
                z0 /= r;
                z1 /= r;
            }
        }
        if (k0 < K) row[k0] = z0;
        if (k1 < K) row[k1] = z1;
    }
}

int grid_for(int64_t items, int per_thread, int cap) {
    const int64_t b = (items + (int64_t)kEB * per_thread - 1) / ((int64_t)kEB * per_thread);
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

template <int L>
void launch_finish(int blocks, hipStream_t s, float *Z, int N, int K, const float *sv, const float2 *info,
                   bool diag, bool cor) {
    hipLaunchKernelGGL(edge_finish<L>, dim3((unsigned)blocks), dim3(kEB), 0, s, Z, N, K, sv, info, diag, cor);
}

}  // namespace

size_t edge_workspace_bytes(int N, int K, unsigned flags) {
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return up((size_t)K * 4) + up((size_t)N * 8) + ((flags & kLap) ? up((size_t)N * 4) : 0) +
           (in_degree_pass(flags) ? up((size_t)N * 4) : 0);
}

hipError_t launch_edge_embed(const int *src, const int *dst, const float *w, int64_t E, int N, const int *labels,
                             int K, unsigned flags, float *Z, void *ws, unsigned *status, hipStream_t s) {
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *p = static_cast<char *>(ws);
    int *counts = reinterpret_cast<int *>(p);
    p += up((size_t)K * 4);
    float2 *info = reinterpret_cast<float2 *>(p);
    p += up((size_t)N * 8);
    float *deg = (flags & kLap) ? reinterpret_cast<float *>(p) : nullptr;
    if (deg) p += up((size_t)N * 4);
    float *degin = in_degree_pass(flags) ? reinterpret_cast<float *>(p) : nullptr;
    const bool sym = flags & kSym, diag = flags & kDiag, cor = flags & kCor;
    const int64_t nz = (int64_t)N * K;
    if (flags & kNoValidate) status = nullptr;  // no checks that only report, no bits raised

    prof_begin(kKEdgeInit, s);
    hipLaunchKernelGGL(edge_init, dim3((unsigned)grid_for(nz / 4 + 1, 4, 16384)), dim3(kEB), 0, s, Z, nz, deg, degin,
                       N, diag ? 1.0f : 0.0f, counts, K);
    prof_end(kKEdgeInit, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    const int cblocks = grid_for(N, 16, 1024);
    const int dblocks = deg && E > 0 ? grid_for(E, 4, 16384) : 0;
    prof_begin(kKEdgePrep, s);
    hipLaunchKernelGGL(edge_prep, dim3((unsigned)(cblocks + dblocks)), dim3(kEB), 0, s, labels, N, K, cblocks,
                       counts, src, dst, w, E, sym, deg, degin, status);
    prof_end(kKEdgePrep, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    prof_begin(kKEdgeCoef, s);
    hipLaunchKernelGGL(edge_coef, dim3((unsigned)grid_for(N, 4, 16384)), dim3(kEB), 0, s, labels, N, K, counts, deg,
                       degin, info);
    prof_end(kKEdgeCoef, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    if (E > 0) {
        prof_begin(kKEdgeScatter, s);
        hipLaunchKernelGGL(edge_scatter, dim3((unsigned)grid_for(E, 8, 8192)), dim3(kEB), 0, s, src, dst, w, E, N,
                           K, sym, info, Z, status);
        prof_end(kKEdgeScatter, s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }

    if (diag || deg || cor) {
        const int L = K > 32 ? 64 : K > 16 ? 32 : K > 8 ? 16 : K > 4 ? 8 : K > 2 ? 4 : K > 1 ? 2 : 1;
        const int blocks = grid_for((int64_t)N * L, 4, 16384);
        prof_begin(kKEdgeFinish, s);
        switch (L) {
            case 64: launch_finish<64>(blocks, s, Z, N, K, deg, info, diag, cor); break;
            case 32: launch_finish<32>(blocks, s, Z, N, K, deg, info, diag, cor); break;
            case 16: launch_finish<16>(blocks, s, Z, N, K, deg, info, diag, cor); break;
            case 8: launch_finish<8>(blocks, s, Z, N, K, deg, info, diag, cor); break;
            case 4: launch_finish<4>(blocks, s, Z, N, K, deg, info, diag, cor); break;
            case 2: launch_finish<2>(blocks, s, Z, N, K, deg, info, diag, cor); break;
            default: launch_finish<1>(blocks, s, Z, N, K, deg, info, diag, cor); break;
        }
        prof_end(kKEdgeFinish, s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace gee
