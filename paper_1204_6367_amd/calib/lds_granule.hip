// LDS allocation granule on the device: how many 512-thread workgroups with a
// given amount of dynamic LDS share a compute unit at once.  Every workgroup of
// a grid of three per compute unit spins a fixed 2 ms of wall clock and
// exits; the launch takes 2 ms when all three are resident and 4 ms when only
// two are.  Output: one line per LDS size with the runtime's occupancy answer
// beside the measured one.
#include <hip/hip_runtime.h>

#include <cstdio>

#define CHECK(x)                                                                            \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) {                                                             \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                       \
        }                                                                                   \
    } while (0)

namespace {

__global__ __launch_bounds__(512) void spin(long long ticks, int* out) {
    extern __shared__ int s[];
    if (threadIdx.x == 0) s[0] = (int)blockIdx.x;
    __syncthreads();
    const long long t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) {
    }
    if (threadIdx.x == 0) out[blockIdx.x] = s[0];          // one word per workgroup (grid entries)
}

}  // namespace

int main() {
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, 0));
    int rate_khz = 0;
    CHECK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, 0));
    std::printf("compute units %d, LDS per workgroup %zu, per compute unit %zu bytes\n", p.multiProcessorCount,
                p.sharedMemPerBlock, p.maxSharedMemoryPerMultiProcessor);
    const long long ticks = 2LL * rate_khz;                   // 2 ms
    const int grid = p.multiProcessorCount * 3;
    int* out = nullptr;
    CHECK(hipMalloc(&out, grid * sizeof(int)));
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    for (int bytes = 40960; bytes <= 57344; bytes += 256) {
        int query = 0;
        CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&query, spin, 512, bytes));
        float best = 1e30f;
        for (int r = 0; r < 3; ++r) {
            CHECK(hipEventRecord(a));
            hipLaunchKernelGGL(spin, dim3(grid), dim3(512), bytes, 0, ticks, out);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(b));
            CHECK(hipEventSynchronize(b));
            float ms = 0.0f;
            CHECK(hipEventElapsedTime(&ms, a, b));
            best = ms < best ? ms : best;
        }
        std::printf("lds %6d bytes: occupancy query %d; three workgroups per compute unit %s (%.2f ms)\n", bytes,
                    query, best < 3.0f ? "resident at once" : "NOT resident at once", best);
    }
    CHECK(hipFree(out));
    return 0;
}
