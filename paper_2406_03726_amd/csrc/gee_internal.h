// gee_internal.h - shared by the HIP translation units of libgee (never installed).
//
// Device helpers for 64-wide wavefronts on gfx950, the launch plan computed on the
// host from (E, N, K, flags, schedule), and the host-side launchers each .hip file
// exports.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gee {

// Option bits (same values as the public GEE_* flags).
constexpr unsigned kDiag = 1u, kLap = 2u, kCor = 4u, kSym = 8u;
// Device data-error bits (same values as the public GEE_DATA_* bits).
constexpr unsigned kErrLabel = 1u, kErrIndex = 2u, kErrWeight = 4u, kErrCsr = 8u;

constexpr int kWave = 64;
constexpr int kMaxBuckets = 4096;      // partition buckets (pass 1 digits)
constexpr int kMaxBucketRowsLog2 = 12; // rows per bucket (pass 2 digits)
constexpr int kMaxClasses = 128;

// ----------------------------------------------------------------------------- wave ops

__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// Number of set bits of `mask` strictly below this lane.
__device__ __forceinline__ int count_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p ? 1 : 0); }

// Orders LDS accesses of one wavefront (LDS instructions of a wave execute in order;
// this keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ void raise_error(unsigned *status, unsigned bit) {
    atomicOr(status, bit);
}

// ----------------------------------------------------------------------------- plan

struct Plan {
    int64_t E = 0;       // input rows
    int32_t N = 0, K = 0;
    unsigned flags = 0;
    bool weighted = false;
    int64_t Mcap = 0;    // upper bound of CSR entries (2E under symmetrization, else E)
    // partition (CSR build)
    int sb = 0;          // rows per bucket = 1 << sb
    int32_t B = 1;       // buckets
    int tile = 16384;    // virtual entries per pass-1 tile
    int64_t T1 = 1;      // pass-1 tiles
    // embed
    int WE = 2048;       // CSR entries per embed wavefront
    int wpb = 4;         // wavefronts per embed workgroup
    int64_t NWcap = 1;   // embed wavefronts launched (upper bound)
    int cnt_blocks = 1;  // class-count partial blocks
};

// Workspace carve-up; every member is a device pointer into one caller buffer.
struct Work {
    int *counts = nullptr;     // [K]
    float *inv_n = nullptr;    // [K]
    int *cpart = nullptr;      // [cnt_blocks * K]
    int *meta = nullptr;       // [4]: M, NW, ...
    int *ghist = nullptr;      // [B * T1]
    int *btot = nullptr;       // [B]
    int *bstart = nullptr;     // [B + 1]
    uint16_t *tkey = nullptr;  // [Mcap] row within bucket
    int *tcol = nullptr;       // [Mcap]
    float *tval = nullptr;     // [Mcap] (weighted only)
    int *rp = nullptr;         // [N + 1]
    int *col = nullptr;        // [Mcap]
    float *val = nullptr;      // [Mcap] (weighted only)
    float2 *info = nullptr;    // [N] {coefficient, label bits}
    float *srow = nullptr;     // [N] D^-1/2 (Laplacian)
    int *fown = nullptr;       // [NWcap + 1] first row owned by each embed wavefront
    int *split = nullptr;      // [NWcap]
    float *headp = nullptr;    // [NWcap * K]
    float *tailp = nullptr;    // [NWcap * K]
};

// ----------------------------------------------------------------------------- profiling
// Kernel ids for the optional event hook (gee_profile_kernel). The hook records a
// caller's hipEvents on the launch stream right before / after a kernel launch.
enum KernelId : int {
    kKCountPartial = 0, kKCountFinal, kKP1Hist, kKP1Scan, kKP1Totals, kKP1Scatter, kKP2Bucket,
    kKPrepCsr, kKFillEmpty, kKEmbedRows, kKEmbedFixup, kKSetMeta, kKBatchEmbed, kKBatchFixup,
    kKNumKernels
};
extern const char *const kKernelNames[kKNumKernels];
void prof_begin(int kid, hipStream_t s);
void prof_end(int kid, hipStream_t s);

// ----------------------------------------------------------------------------- launchers
// gee_count.hip
hipError_t launch_class_counts(const int *labels, int N, int K, int nblocks, int *part, int *counts,
                               float *inv_n, unsigned *status, hipStream_t s);
// gee_csr.hip
hipError_t launch_csr_build(const int *src, const int *dst, const float *w, const Plan &p,
                            const Work &wk, unsigned *status, hipStream_t s);
// Pass 2 also prepares the embedding's per-node data when `embed_prep` is set.
hipError_t launch_csr_pass2(const Plan &p, const Work &wk, const int *labels, bool embed_prep,
                            unsigned *status, hipStream_t s);
// gee_embed.hip
hipError_t launch_embed_prep_from_csr(const int *rp, const float *val, const int *labels, int64_t M,
                                      const Plan &p, const Work &wk, unsigned *status, hipStream_t s);
hipError_t launch_embed(const int *rp, const int *col, const float *val, const Plan &p,
                        const Work &wk, float *Z, unsigned *status, hipStream_t s);

}  // namespace gee
