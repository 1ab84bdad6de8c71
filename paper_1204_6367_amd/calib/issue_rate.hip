// Issue cost of the VALU instruction kinds that the benchmark's work model
// prices (integer 32x32 products, transcendentals, float64 FMA), measured on
// the device against a chain of full-rate float32 FMAs.
//
// Each kernel runs, per lane, 8 independent dependency chains (so latency is
// hidden by the other chains and by 8 wavefronts per SIMD); a chain step is
// the instruction under test plus at most a few companions that keep the
// compiler from folding the chain.  Printed: the time of a chain step in units
// of a float32 FMA step, t(step) / t(FMA step), which does not depend on the
// clock; an instruction's own cost is that less its companions' costs, read
// from the rows that measure them.  Output: one line per kind.
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

constexpr int kIters = 4096;
constexpr int kChains = 8;
constexpr int kBlock = 256;

// out[gid] receives a value depending on every chain (nothing is dead code)
#define RATE_KERNEL_F(name, T, init, step)                                            \
    __global__ __launch_bounds__(kBlock) void name(uint32_t* out, float s) {          \
        T a[kChains];                                                                 \
        _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = (T)(init);         \
        for (int i = 0; i < kIters; ++i) {                                            \
            _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = (step);        \
        }                                                                             \
        T r = 0;                                                                      \
        _Pragma("unroll") for (int c = 0; c < kChains; ++c) r += a[c];                \
        out[blockIdx.x * kBlock + threadIdx.x] = (uint32_t)(float)r;                  \
    }

#define RATE_KERNEL_U(name, init, step)                                               \
    __global__ __launch_bounds__(kBlock) void name(uint32_t* out, float s) {          \
        uint32_t a[kChains];                                                          \
        const uint32_t k = __float_as_uint(s) | 1u;                                   \
        _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = (init);            \
        for (int i = 0; i < kIters; ++i) {                                            \
            _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = (step);        \
        }                                                                             \
        uint32_t r = 0;                                                               \
        _Pragma("unroll") for (int c = 0; c < kChains; ++c) r ^= a[c];                \
        out[blockIdx.x * kBlock + threadIdx.x] = r;                                   \
    }

const float kInitScale = 1e-7f;
#define F_INIT (1.25f + (float)(threadIdx.x * kChains + c) * kInitScale)

RATE_KERNEL_F(k_fma, float, F_INIT, __builtin_fmaf(a[c], 0.999f, s))
RATE_KERNEL_F(k_add, float, F_INIT, a[c] + s)
// the same with a per-lane (vector register) operand instead of the scalar s
RATE_KERNEL_F(k_addv, float, F_INIT, a[c] + (s + (float)threadIdx.x * 1e-30f))
RATE_KERNEL_F(k_fmas, float, F_INIT, __builtin_fmaf(a[c], s, 0.25f))
RATE_KERNEL_F(k_mul, float, F_INIT, a[c] * s)
RATE_KERNEL_F(k_min, float, F_INIT, __builtin_fminf(a[c] + s, 3.0f))
RATE_KERNEL_F(k_floor, float, F_INIT, __builtin_floorf(a[c]) + s)
RATE_KERNEL_F(k_sel, float, F_INIT, (a[c] > 2.0f ? a[c] * 0.5f : a[c]) + s)
RATE_KERNEL_F(k_log, float, F_INIT, __builtin_amdgcn_logf(a[c]) + 2.0f)
RATE_KERNEL_F(k_exp, float, F_INIT, __builtin_amdgcn_exp2f(-a[c]) + 0.5f)
RATE_KERNEL_F(k_rcp, float, F_INIT, __builtin_amdgcn_rcpf(a[c]) + 1.5f)
RATE_KERNEL_F(k_rsq, float, F_INIT, __builtin_amdgcn_rsqf(a[c]) + 0.5f)
RATE_KERNEL_F(k_sqrt, float, F_INIT, __builtin_amdgcn_sqrtf(a[c]) + 0.5f)
RATE_KERNEL_F(k_sin, float, F_INIT, __builtin_amdgcn_sinf(a[c]) + 0.25f)
RATE_KERNEL_F(k_fma64, double, F_INIT, __builtin_fma(a[c], 0.999, (double)s))
RATE_KERNEL_U(k_xor, threadIdx.x * kChains + c + k, (a[c] ^ (uint32_t)i) + k)
RATE_KERNEL_U(k_mullo, threadIdx.x * kChains + c + k, (a[c] * k) ^ (uint32_t)i)
RATE_KERNEL_U(k_cvt, threadIdx.x * kChains + c + k, (uint32_t)((float)a[c] * 0.75f))
RATE_KERNEL_U(k_mulhi, threadIdx.x * kChains + c + k, __umulhi(a[c], 0xD2511F53u) ^ k)
RATE_KERNEL_U(k_mad64, threadIdx.x * kChains + c + k,
              (uint32_t)(((uint64_t)a[c] * 0xD2511F53ull) >> 32) ^ (uint32_t)((uint64_t)a[c] * 0xD2511F53ull))


// integer chains with per-lane (vector register) operands read from memory
__global__ __launch_bounds__(kBlock) void k_xadv(uint32_t* out, float s) {
    uint32_t a[kChains];
    const uint32_t kv = out[blockIdx.x * kBlock + threadIdx.x] | 1u;
    const uint32_t kw = kv * 3u;
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = threadIdx.x * kChains + c + __float_as_uint(s);
    for (int i = 0; i < kIters; ++i) {
        _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = (a[c] ^ kv) + kw;   // one v_xad_u32
    }
    uint32_t r = 0;
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) r ^= a[c];
    out[blockIdx.x * kBlock + threadIdx.x] = r;
}

// three-input xor (gfx950 v_bitop3_b32, truth table 0x96) then an add, vector operands
__global__ __launch_bounds__(kBlock) void k_bitop3v(uint32_t* out, float s) {
    uint32_t a[kChains];
    const uint32_t kv = out[blockIdx.x * kBlock + threadIdx.x] | 1u;
    const uint32_t kw = kv * 3u;
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = threadIdx.x * kChains + c + __float_as_uint(s);
    for (int i = 0; i < kIters; ++i) {
        _Pragma("unroll") for (int c = 0; c < kChains; ++c)
            a[c] = __builtin_amdgcn_bitop3_b32(a[c], kv, (uint32_t)i, 0x96) + kw;
    }
    uint32_t r = 0;
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) r ^= a[c];
    out[blockIdx.x * kBlock + threadIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_mad64v(uint32_t* out, float s) {
    uint32_t a[kChains];
    const uint32_t kv = out[blockIdx.x * kBlock + threadIdx.x] | 1u;
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) a[c] = threadIdx.x * kChains + c + __float_as_uint(s);
    for (int i = 0; i < kIters; ++i) {
        _Pragma("unroll") for (int c = 0; c < kChains; ++c) {
            const uint64_t p = (uint64_t)a[c] * kv;
            a[c] = (uint32_t)(p >> 32) ^ (uint32_t)p;
        }
    }
    uint32_t r = 0;
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) r ^= a[c];
    out[blockIdx.x * kBlock + threadIdx.x] = r;
}

struct Kind {
    const char* name;
    void (*fn)(uint32_t*, float);
    const char* what;   // the instructions of one chain step
};

}  // namespace

int main() {
    int cus = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const int blocks = cus * 8;                // 8 workgroups of 4 wavefronts per CU
    uint32_t* d = nullptr;
    CHECK(hipMalloc(&d, (size_t)blocks * kBlock * sizeof(uint32_t)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const Kind kinds[] = {
        {"fma_f32", k_fma, "v_fma_f32 (vector operands and a literal; the unit)"},
        {"add_f32", k_add, "v_add_f32 (scalar-register operand)"},
        {"add_f32_v", k_addv, "v_add_f32 (vector operands)"},
        {"fma_f32_s", k_fmas, "v_fma_f32 (scalar-register operand)"},
        {"mul_f32", k_mul, "v_mul_f32 (scalar-register operand)"},
        {"min_f32", k_min, "v_min_f32 + v_add_f32"},
        {"floor_f32", k_floor, "v_floor_f32 + v_add_f32"},
        {"cmp_cnd_f32", k_sel, "v_cmp_f32 + v_cndmask_b32 + v_mul_f32 + v_add_f32"},
        {"xor_add_u32", k_xor, "v_xor_b32 + v_add_u32"},
        {"mul_lo_u32", k_mullo, "v_mul_lo_u32 + v_xor_b32"},
        {"cvt_f32_u32", k_cvt, "v_cvt_f32_u32 + v_mul_f32 + v_cvt_u32_f32"},
        {"xad_u32_v", k_xadv, "v_xad_u32 (vector operands)"},
        {"bitop3_add_v", k_bitop3v, "v_bitop3_b32 (a ^ b ^ c) + v_add_u32 (vector operands)"},
        {"mul_hi_u32", k_mulhi, "v_mul_hi_u32 + v_xor_b32"},
        {"mad_u64_u32", k_mad64, "v_mad_u64_u32 (32x32->64 product) + v_xor_b32"},
        {"mad_u64_u32_v", k_mad64v, "v_mad_u64_u32 (vector multiplier) + v_xor_b32"},
        {"log_f32", k_log, "v_log_f32 + v_add_f32"},
        {"exp_f32", k_exp, "v_exp_f32 + v_add_f32"},
        {"rcp_f32", k_rcp, "v_rcp_f32 + v_add_f32"},
        {"rsq_f32", k_rsq, "v_rsq_f32 + v_add_f32"},
        {"sqrt_f32", k_sqrt, "v_sqrt_f32 + v_add_f32"},
        {"sin_f32", k_sin, "v_sin_f32 + v_add_f32"},
        {"fma_f64", k_fma64, "v_fma_f64"},
    };
    float ref = 0.0f;
    std::printf("%-12s %10s %10s  %s\n", "kind", "ms", "FMA steps", "chain step");
    for (const Kind& k : kinds) {
        float best = 1e30f;
        for (int rep = 0; rep < 5; ++rep) {
            CHECK(hipEventRecord(e0, nullptr));
            hipLaunchKernelGGL(k.fn, dim3(blocks), dim3(kBlock), 0, nullptr, d, 1.0f + 0.001f * rep);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1, nullptr));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.0f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) best = ms;
        }
        if (ref == 0.0f) ref = best;
        std::printf("%-12s %10.4f %10.2f  %s\n", k.name, best, best / ref, k.what);
        std::fflush(stdout);
    }
    CHECK(hipFree(d));
    return 0;
}
