// Calibration program for HBM traffic counters: a plain device-to-device
// copy of a known size.  The FETCH_SIZE / WRITE_SIZE that a counter run
// reports for k_copy, divided by the bytes it must read / write, gives the
// factor by which the same counters over- or under-count for any kernel.
//
// Measurement tooling for the benchmark's traffic figures, not part of the
// library.  Build and run (on the GPU host):
//   hipcc --offload-arch=gfx950 -O3 -o _build/hbm_copy hbm_copy.hip
//   _build/hbm_copy [MiB]   (default 256; copies that many MiB three times)
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src,
                                              uint4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

#define CHECK(x)                                                                  \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));        \
            return 1;                                                             \
        }                                                                         \
    } while (0)

int main(int argc, char** argv) {
    const size_t mib = argc > 1 ? (size_t)atol(argv[1]) : 256;
    if (mib < 1 || mib > 16384) {
        fprintf(stderr, "size must be 1..16384 MiB\n");
        return 1;
    }
    const size_t bytes = mib << 20;
    const size_t n = bytes / sizeof(uint4);
    void *a = nullptr, *b = nullptr;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&b, bytes));
    CHECK(hipMemset(a, 1, bytes));
    CHECK(hipMemset(b, 0, bytes));
    CHECK(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (int rep = 0; rep < 3; rep++) {
        CHECK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL(k_copy, dim3(8192), dim3(256), 0, 0, (const uint4*)a, (uint4*)b, n);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        printf("k_copy %zu MiB: read %zu B, write %zu B, %.3f ms, %.1f GB/s\n", mib, bytes, bytes,
               ms, 2.0 * bytes / (ms * 1e-3) / 1e9);
    }
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    return 0;
}
