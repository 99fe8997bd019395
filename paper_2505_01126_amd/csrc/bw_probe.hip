// Memory-bandwidth probe: what streaming kernels reach on this GPU, the scale
// against which the fused step's HBM rate is read.  Standalone program (not
// part of liblbm.so): 2 GiB buffers, HIP-event timing of 10 launches after 3
// warm-ups, one line per kernel with the bytes each launch moves.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                              \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);        \
            std::exit(1);                                                                     \
        }                                                                                     \
    } while (0)

__global__ void k_copy4(const float4 *__restrict__ a, float4 *__restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ void k_read4(const float4 *__restrict__ a, float *__restrict__ out, size_t n)
{
    float s = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float4 v = a[i];
        s += (v.x + v.y) + (v.z + v.w);
    }
    if (s == 1234.5f) out[0] = s;  // keeps the loads live
}

__global__ void k_write4(float4 *__restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = make_float4(1.f, 2.f, 3.f, 4.f);
}

// 27 rows in, 27 rows out, one element per row per site and thread: the
// population stream of a lattice update without the shifts and the arithmetic
template <class T>
__global__ void k_rows27(const T *__restrict__ a, T *__restrict__ b, unsigned n)
{
    const unsigned s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    T v[27];
#pragma unroll
    for (int q = 0; q < 27; q++) v[q] = a[(size_t)q * n + s];
#pragma unroll
    for (int q = 0; q < 27; q++) b[(size_t)q * n + s] = v[q];
}

int main()
{
    const size_t bytes = (size_t)2 << 30;
    void *a = nullptr, *b = nullptr;
    float *o = nullptr;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&b, bytes));
    CHECK(hipMalloc(&o, 64));
    CHECK(hipMemset(a, 0, bytes));
    CHECK(hipMemset(b, 0, bytes));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    auto timeit = [&](const char *name, int blocks, double moved, auto launch) {
        for (int w = 0; w < 3; w++) launch();
        CHECK(hipDeviceSynchronize());
        CHECK(hipEventRecord(e0));
        for (int r = 0; r < 10; r++) launch();
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        ms /= 10.f;
        std::printf("%-10s blocks %7d  %8.3f ms  %7.1f GB/s\n", name, blocks, ms, moved / ms / 1e6);
        std::fflush(stdout);
    };
    const size_t n4 = bytes / 16;
    for (int blocks : {1024, 4096, 16384, 65536}) {
        timeit("copy", blocks, 2.0 * bytes, [&] { k_copy4<<<blocks, 256>>>((const float4 *)a, (float4 *)b, n4); });
        timeit("read", blocks, 1.0 * bytes, [&] { k_read4<<<blocks, 256>>>((const float4 *)a, o, n4); });
        timeit("write", blocks, 1.0 * bytes, [&] { k_write4<<<blocks, 256>>>((float4 *)b, n4); });
    }
    const unsigned n32 = (unsigned)(bytes / 4 / 27), n16 = (unsigned)(bytes / 2 / 27);
    timeit("rows27_f32", (n32 + 255) / 256, 2.0 * 27 * 4.0 * n32,
           [&] { k_rows27<float><<<(n32 + 255) / 256, 256>>>((const float *)a, (float *)b, n32); });
    timeit("rows27_f16", (n16 + 255) / 256, 2.0 * 27 * 2.0 * n16,
           [&] { k_rows27<_Float16><<<(n16 + 255) / 256, 256>>>((const _Float16 *)a, (_Float16 *)b, n16); });
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(o));
    return 0;
}
