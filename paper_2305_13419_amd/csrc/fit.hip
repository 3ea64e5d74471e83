// FP64 normal equations of the linear-prediction ringdown fit.
#include "tfl_internal.h"

namespace tfl {
namespace {

constexpr int kGramThreads = 256;

// One block per pair (j, k), j <= k: a deterministic block reduction.
__global__ __launch_bounds__(kGramThreads) void gram_kernel(const double *x, long long start, long long count,
                                                            long long decim, int order, double *out)
{
    int pair = blockIdx.x, j = 0;
    while (pair >= order + 1 - j) {
        pair -= order + 1 - j;
        ++j;
    }
    const int k = j + pair;
    double acc = 0.0;
    for (long long m = order + threadIdx.x; m < count; m += kGramThreads)
        acc += x[start + (m - j) * decim] * x[start + (m - k) * decim];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double part[kGramThreads / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kGramThreads / 64; ++w) s += part[w];
        out[blockIdx.x] = s;
    }
}

// One block per lag j: the correction A^T (b - A a) formed from the data
// itself, without the cancellation of the normal equations.
__global__ __launch_bounds__(kGramThreads) void lp_residual_kernel(const double *x, long long start, long long count,
                                                                   long long decim, int order, const double *a,
                                                                   double *out)
{
    const int j = blockIdx.x + 1;
    double acc = 0.0;
    for (long long m = order + threadIdx.x; m < count; m += kGramThreads) {
        double e = x[start + m * decim];
        for (int k = 1; k <= order; ++k) e -= a[k - 1] * x[start + (m - k) * decim];
        acc += x[start + (m - j) * decim] * e;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double part[kGramThreads / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kGramThreads / 64; ++w) s += part[w];
        out[blockIdx.x] = s;
    }
}

}  // namespace

hipError_t launch_lp_residual(const double *series, long long start, long long count, long long decim, int order,
                              const double *a, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(lp_residual_kernel, dim3(order), dim3(kGramThreads), 0, s, series, start, count, decim, order,
                       a, out);
    return hipGetLastError();
}

hipError_t launch_gram(const double *series, long long start, long long count, long long decim, int order,
                       double *out, hipStream_t s)
{
    const int npairs = (order + 1) * (order + 2) / 2;
    hipLaunchKernelGGL(gram_kernel, dim3(npairs), dim3(kGramThreads), 0, s, series, start, count, decim, order, out);
    return hipGetLastError();
}

}  // namespace tfl
