// Random-gather throughput on the device: the memory-side peak that the
// transport's gathers (32-byte cell records, 8-byte cube records, 4-byte
// words) can reach at a given working-set size -- L2 (4 MB per XCD), the
// 256 MB last-level cache, or HBM.
//
// Each lane reads `kIters` records at pseudo-random positions (a hash of its
// index and the iteration, masked to a power-of-two record count, so every
// index is in bounds) and xors them into one word it writes out.  Output: one
// line per (record size, working set) with the useful bytes per second.
#include <hip/hip_runtime.h>

#include <cstdint>
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

constexpr int kIters = 256;
constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t mix(uint32_t x) {      // a 32-bit integer hash (xorshift-multiply)
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

template <int WORDS>    // record size in 4-byte words: 1, 2 or 8
__global__ __launch_bounds__(kBlock) void gather(const uint32_t* __restrict__ buf, uint32_t mask,
                                                 uint32_t* __restrict__ out, uint32_t salt) {
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    uint32_t acc = 0;
    for (int i = 0; i < kIters; ++i) {
        const uint32_t r = mix(gid * kIters + (uint32_t)i + salt) & mask;
        const uint32_t* p = buf + (size_t)r * WORDS;
        if (WORDS == 8) {
            const uint4 a = reinterpret_cast<const uint4*>(p)[0];
            const uint4 b = reinterpret_cast<const uint4*>(p)[1];
            acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w;
        } else if (WORDS == 2) {
            const uint2 a = reinterpret_cast<const uint2*>(p)[0];
            acc ^= a.x ^ a.y;
        } else {
            acc ^= p[0];
        }
    }
    out[gid] = acc;
}

__global__ void fill(uint32_t* buf, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        buf[i] = (uint32_t)i * 2654435761u;
}

}  // namespace

int main() {
    int cus = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const int blocks = cus * 8;
    const size_t lanes = (size_t)blocks * kBlock;
    const size_t max_bytes = (size_t)4 << 30;                // 4 GiB
    uint32_t* buf = nullptr;
    uint32_t* out = nullptr;
    CHECK(hipMalloc(&buf, max_bytes));
    CHECK(hipMalloc(&out, lanes * sizeof(uint32_t)));
    hipLaunchKernelGGL(fill, dim3(4096), dim3(256), 0, nullptr, buf, max_bytes / 4);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const size_t sets[] = {(size_t)2 << 20, (size_t)32 << 20, (size_t)128 << 20, (size_t)1 << 30, max_bytes};
    const int words[] = {8, 2, 1};
    std::printf("%8s %12s %10s %12s\n", "record_B", "working_set", "ms", "GB/s");
    for (const int w : words) {
        for (const size_t bytes : sets) {
            const size_t records = bytes / (4u * w);         // a power of two
            const uint32_t mask = (uint32_t)(records - 1);
            float best = 1e30f;
            for (int rep = 0; rep < 5; ++rep) {
                CHECK(hipEventRecord(e0, nullptr));
                if (w == 8)
                    hipLaunchKernelGGL(gather<8>, dim3(blocks), dim3(kBlock), 0, nullptr, buf, mask, out, 977u * rep);
                else if (w == 2)
                    hipLaunchKernelGGL(gather<2>, dim3(blocks), dim3(kBlock), 0, nullptr, buf, mask, out, 977u * rep);
                else
                    hipLaunchKernelGGL(gather<1>, dim3(blocks), dim3(kBlock), 0, nullptr, buf, mask, out, 977u * rep);
                CHECK(hipGetLastError());
                CHECK(hipEventRecord(e1, nullptr));
                CHECK(hipEventSynchronize(e1));
                float ms = 0.0f;
                CHECK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) best = ms;
            }
            const double useful = (double)lanes * kIters * 4.0 * w;
            std::printf("%8d %9zu MiB %10.4f %12.1f\n", 4 * w, bytes >> 20, best, useful / (best * 1e-3) / 1e9);
            std::fflush(stdout);
        }
    }
    CHECK(hipFree(out));
    CHECK(hipFree(buf));
    return 0;
}
