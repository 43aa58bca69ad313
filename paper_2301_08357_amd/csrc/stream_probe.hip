// Memory-bandwidth probe of the GPU, used by the benchmark to state the
// practical HBM ceiling beside the 8 TB/s specification and to scale the
// rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes: a plain copy (every
// byte of src read once, every byte of dst written once) and a plain read
// (every byte read once, one reduction value per block kept only so that
// the loads are not removed).  Not part of the solver.

#include <hip/hip_runtime.h>

#include <cstddef>

namespace {

__global__ void __launch_bounds__(256) k_copy(const double *__restrict__ src, double *__restrict__ dst, size_t n)
{
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

__global__ void __launch_bounds__(256) k_read(const double *__restrict__ src, size_t n, double *__restrict__ sink)
{
    double s = 0.0;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        s += src[i];
    // never true for the finite data the probe reads; keeps the sum (and the loads) alive
    if (s == -1.0e300) sink[blockIdx.x] = s;
}

}  // namespace

extern "C" {

// kind 0: copy n doubles src -> dst; kind 1: read n doubles of src (dst
// receives nothing unless the data sum to -1e300; it must hold `grid`
// doubles).  grid blocks of 256 threads, asynchronous on stream.  Returns
// 0, or -1 for invalid arguments, -5 for a HIP error.
int stream_probe(int kind, const double *src, double *dst, size_t n, int grid, void *stream)
{
    if (!src || !dst || grid < 1 || (kind != 0 && kind != 1)) return -1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (kind == 0)
        hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, s, src, dst, n);
    else
        hipLaunchKernelGGL(k_read, dim3(grid), dim3(256), 0, s, src, n, dst);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"
