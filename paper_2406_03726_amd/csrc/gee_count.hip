// gee_count.hip - class sizes n_k and 1/n_k (Section 2: W row j holds 1/n_{y_j}) as two
// launches of their own (class_count_slice, class_count_total), for gee_class_counts and
// the resident-CSR path; the edge-list paths run them inside the partition launches.
#include "gee_internal.h"

#include <cstring>

namespace gee {

__global__ __launch_bounds__(256) void class_count_partial(Batch b, int *__restrict__ part,
                                                           unsigned *status, int *__restrict__ zero_word) {
    __shared__ int hist[kMaxClasses];
    if (zero_word && blockIdx.x == 0 && threadIdx.x == 0) *zero_word = 0;
    class_count_slice(b, blockIdx.x, part, status, hist);
}

// Wavefront per class (all graphs).
__global__ __launch_bounds__(256) void class_count_final(Batch b, int Ktot, const int *__restrict__ part,
                                                         int *__restrict__ counts, float *__restrict__ inv_n) {
    const int c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (c >= Ktot) return;
    class_count_total(b, c, part, counts, inv_n);
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
                               unsigned *status, hipStream_t s, int *zero_word, bool totals) {
    prof_begin(kKCountPartial, s);
    hipLaunchKernelGGL(class_count_partial, dim3((unsigned)p.cnt_blocks), dim3(256), 0, s, b, part, status,
                       zero_word);
    prof_end(kKCountPartial, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !totals) return e;
    prof_begin(kKCountFinal, s);
    hipLaunchKernelGGL(class_count_final, dim3((unsigned)((p.Ktot + 3) / 4)), dim3(256), 0, s, b, p.Ktot, part,
                       counts, inv_n);
    prof_end(kKCountFinal, s);
    return hipGetLastError();
}

}  // namespace gee
