// cm_probe.hip -- microbenchmarks that give the roofline denominators of the
// CM loss kernels on the running GPU: achievable HBM stream bandwidth and the
// throughput of global and LDS floating-point atomic adds.  Measurement only;
// nothing here is on the loss path.
//
// Every entry point enqueues `reps` launches on `stream` and returns at once;
// the caller times the stream (HIP events) and synchronises.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src,
                                                   float4* __restrict__ dst, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__device__ __forceinline__ uint32_t mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// ops_per_thread atomic adds per thread into arr[0..n).  pattern 0: random
// addresses; pattern 1: lane-contiguous (a wave covers consecutive elements).
template <typename T>
__global__ __launch_bounds__(256) void global_atomic_kernel(T* __restrict__ arr, uint32_t n,
                                                            int ops_per_thread, int pattern)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nthreads = gridDim.x * blockDim.x;
    for (int k = 0; k < ops_per_thread; ++k) {
        uint32_t idx;
        if (pattern == 0) idx = mix(gid * 0x9E3779B9u + (uint32_t)k * 0x85EBCA6Bu) % n;
        else idx = (uint32_t)(((uint64_t)k * nthreads + gid) % n);
        unsafeAtomicAdd(arr + idx, (T)1);
    }
}

// LDS atomic adds into a per-workgroup array of n_lds elements.
template <typename T>
__global__ __launch_bounds__(256) void lds_atomic_kernel(T* __restrict__ out, uint32_t n_lds,
                                                         int ops_per_thread)
{
    extern __shared__ unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    for (uint32_t i = threadIdx.x; i < n_lds; i += blockDim.x) lds[i] = (T)0;
    __syncthreads();
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int k = 0; k < ops_per_thread; ++k) {
        const uint32_t idx = mix(gid * 0x9E3779B9u + (uint32_t)k * 0x85EBCA6Bu) % n_lds;
        atomicAdd(lds + idx, (T)1);
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = lds[0];
}

// Random 16-byte stores / loads (record scatter and gather patterns).
__global__ __launch_bounds__(256) void random_store_kernel(double2* __restrict__ arr, uint32_t n,
                                                           int ops_per_thread)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int k = 0; k < ops_per_thread; ++k) {
        const uint32_t idx = mix(gid * 0x9E3779B9u + (uint32_t)k * 0x85EBCA6Bu) % n;
        arr[idx] = make_double2((double)gid, (double)k);
    }
}

__global__ __launch_bounds__(256) void random_load_kernel(const double2* __restrict__ arr,
                                                          uint32_t n, int ops_per_thread,
                                                          double* __restrict__ sink)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    for (int k = 0; k < ops_per_thread; ++k) {
        const uint32_t idx = mix(gid * 0x9E3779B9u + (uint32_t)k * 0x85EBCA6Bu) % n;
        const double2 v = arr[idx];
        acc += v.x + v.y;
    }
    if (acc == 12345.678) sink[0] = acc;   // keeps the loads alive
}

}  // namespace

extern "C" {

// Random 16-byte stores (store != 0) or loads into an array of n_elems double2.
int cmprobe_random_access(void* arr, size_t n_elems, int store, int blocks, int ops_per_thread,
                          int reps, void* sink, void* stream)
{
    if (n_elems == 0 || n_elems > 0xffffffffu) return -1;
    for (int r = 0; r < reps; ++r) {
        if (store)
            random_store_kernel<<<blocks, 256, 0, (hipStream_t)stream>>>(
                (double2*)arr, (uint32_t)n_elems, ops_per_thread);
        else
            random_load_kernel<<<blocks, 256, 0, (hipStream_t)stream>>>(
                (const double2*)arr, (uint32_t)n_elems, ops_per_thread, (double*)sink);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}


int cmprobe_copy(const void* src, void* dst, size_t bytes, int reps, void* stream)
{
    const size_t n = bytes / 16;
    const int grid = 256 * 8 * 4;
    for (int r = 0; r < reps; ++r)
        copy_kernel<<<grid, 256, 0, (hipStream_t)stream>>>((const float4*)src, (float4*)dst, n);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// elem_bytes 4 or 8; returns 0 on success.
int cmprobe_global_atomic(void* arr, size_t n_elems, int elem_bytes, int blocks,
                          int ops_per_thread, int pattern, int reps, void* stream)
{
    if (n_elems == 0 || n_elems > 0xffffffffu) return -1;
    for (int r = 0; r < reps; ++r) {
        if (elem_bytes == 8)
            global_atomic_kernel<double><<<blocks, 256, 0, (hipStream_t)stream>>>(
                (double*)arr, (uint32_t)n_elems, ops_per_thread, pattern);
        else
            global_atomic_kernel<float><<<blocks, 256, 0, (hipStream_t)stream>>>(
                (float*)arr, (uint32_t)n_elems, ops_per_thread, pattern);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int cmprobe_lds_atomic(void* out, size_t lds_elems, int elem_bytes, int blocks,
                       int ops_per_thread, int reps, void* stream)
{
    const size_t lds_bytes = lds_elems * (size_t)elem_bytes;
    if (lds_elems == 0 || lds_bytes > 65536) return -1;
    for (int r = 0; r < reps; ++r) {
        if (elem_bytes == 8)
            lds_atomic_kernel<double><<<blocks, 256, lds_bytes, (hipStream_t)stream>>>(
                (double*)out, (uint32_t)lds_elems, ops_per_thread);
        else
            lds_atomic_kernel<float><<<blocks, 256, lds_bytes, (hipStream_t)stream>>>(
                (float*)out, (uint32_t)lds_elems, ops_per_thread);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
