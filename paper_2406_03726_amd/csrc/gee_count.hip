// gee_count.hip - class sizes n_k and 1/n_k (Section 2: W row j holds 1/n_{y_j}).
//
// Two launches, no global atomics on the counts: every workgroup histograms a
// contiguous slice of one graph's labels in LDS and writes its K partial counts; a
// second launch adds each class's partials in workgroup order (integers, so the order
// cannot change the result) and forms 1/n_k in float32 (0 for an empty class).
#include "gee_internal.h"

#include <cstring>

namespace gee {

__global__ __launch_bounds__(256) void class_count_partial(Batch b, int *__restrict__ part,
                                                           unsigned *status) {
    __shared__ int hist[kMaxClasses];
    const int g = find_graph(b.cnt_offs, b.G, (int)blockIdx.x);
    const GDesc d = load_desc(b, g);
    const int jb = blockIdx.x - d.cnt_off;
    const int K = d.K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    const int64_t per = ((int64_t)d.N + d.cnt_blocks - 1) / d.cnt_blocks;
    const int64_t lo = (int64_t)jb * per;
    const int64_t hi = min((int64_t)d.N, lo + per);
    bool bad = false;
    for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
        const int y = d.labels[j];
        if (y >= 0 && y < K)
            atomicAdd(&hist[y], 1);
        else if (y != -1)
            bad = true;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) raise_error(status, kErrLabel);
    for (int k = threadIdx.x; k < K; k += blockDim.x) part[d.cpart_off + (int64_t)jb * K + k] = hist[k];
}

// Wavefront per class (all graphs): the lanes add the graph's partials (integers, so the
// order does not matter), then 1/n_k.
__global__ __launch_bounds__(256) void class_count_final(Batch b, int Ktot, const int *__restrict__ part,
                                                         int *__restrict__ counts, float *__restrict__ inv_n) {
    const int c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (c >= Ktot) return;
    const int lane = lane_id();
    const int g = find_graph(b.class_offs, b.G, c);
    const GDesc d = load_desc(b, g);
    const int k = c - d.class_off;
    const int *pp = part + d.cpart_off + k;
    int n = 0;
    for (int j = lane; j < d.cnt_blocks; j += 64) n += pp[(int64_t)j * d.K];
    n = readlane(wave_scan_add(n), 63);
    if (lane == 0) {
        counts[c] = n;
        if (inv_n) inv_n[c] = n > 0 ? 1.0f / (float)n : 0.0f;
    }
}

// Host bytes to device memory through kernel arguments: each launch carries one chunk.
struct UploadChunk {
    unsigned char b[kUploadChunk];
};
__global__ __launch_bounds__(256) void upload_chunk(unsigned char *__restrict__ dst, UploadChunk c, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.b[i];
}

hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
    const unsigned char *p = static_cast<const unsigned char *>(src);
    unsigned char *q = static_cast<unsigned char *>(dst);
    for (size_t off = 0; off < bytes; off += kUploadChunk) {
        const int n = (int)(bytes - off < (size_t)kUploadChunk ? bytes - off : (size_t)kUploadChunk);
        UploadChunk c;
        std::memcpy(c.b, p + off, (size_t)n);
        hipLaunchKernelGGL(upload_chunk, dim3(1), dim3(256), 0, s, q + off, c, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_class_counts(const Batch &b, const Plan &p, int *part, int *counts, float *inv_n,
                               unsigned *status, hipStream_t s) {
    prof_begin(kKCountPartial, s);
    hipLaunchKernelGGL(class_count_partial, dim3((unsigned)p.cnt_blocks), dim3(256), 0, s, b, part, status);
    prof_end(kKCountPartial, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    prof_begin(kKCountFinal, s);
    hipLaunchKernelGGL(class_count_final, dim3((unsigned)((p.Ktot + 3) / 4)), dim3(256), 0, s, b, p.Ktot, part,
                       counts, inv_n);
    prof_end(kKCountFinal, s);
    return hipGetLastError();
}

}  // namespace gee
