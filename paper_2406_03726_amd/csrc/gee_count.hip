// gee_count.hip - class sizes n_k and 1/n_k (Section 2: W row j holds 1/n_{y_j}).
//
// Two launches, no global atomics on the counts: every workgroup histograms a
// contiguous slice of the labels in LDS and writes its K partial counts; a second
// launch adds the partials in workgroup order (integers, so the order cannot change
// the result) and forms 1/n_k in float32 (0 for an empty class).
#include "gee_internal.h"

namespace gee {

__global__ __launch_bounds__(256) void class_count_partial(const int *__restrict__ labels, int N,
                                                           int K, int *__restrict__ part,
                                                           unsigned *status) {
    extern __shared__ int hist[];
    for (int k = threadIdx.x; k < K; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    const int64_t per = ((int64_t)N + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = min((int64_t)N, lo + per);
    bool bad = false;
    for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
        int y = labels[j];
        if (y >= 0 && y < K)
            atomicAdd(&hist[y], 1);
        else if (y != -1)
            bad = true;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) raise_error(status, kErrLabel);
    for (int k = threadIdx.x; k < K; k += blockDim.x) part[(int64_t)blockIdx.x * K + k] = hist[k];
}

__global__ __launch_bounds__(256) void class_count_final(const int *__restrict__ part, int nblocks,
                                                         int K, int *__restrict__ counts,
                                                         float *__restrict__ inv_n) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    int n = 0;
    for (int b = 0; b < nblocks; ++b) n += part[(int64_t)b * K + k];
    counts[k] = n;
    if (inv_n) inv_n[k] = n > 0 ? 1.0f / (float)n : 0.0f;
}

hipError_t launch_class_counts(const int *labels, int N, int K, int nblocks, int *part, int *counts,
                               float *inv_n, unsigned *status, hipStream_t s) {
    if (nblocks < 1) nblocks = 1;
    prof_begin(kKCountPartial, s);
    hipLaunchKernelGGL(class_count_partial, dim3(nblocks), dim3(256), K * sizeof(int), s, labels, N,
                       K, part, status);
    prof_end(kKCountPartial, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    prof_begin(kKCountFinal, s);
    hipLaunchKernelGGL(class_count_final, dim3((K + 255) / 256), dim3(256), 0, s, part, nblocks, K,
                       counts, inv_n);
    prof_end(kKCountFinal, s);
    return hipGetLastError();
}

}  // namespace gee
