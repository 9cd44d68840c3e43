// valu_probe.hip -- issue cost of the VALU instructions the search kernel is
// made of, on the device at hand (a measurement aid for the kernel's VALU
// slot model; not part of the library).  Each kernel runs 8 independent
// register chains of one instruction per thread, 4,096 times, over a grid of
// 32 blocks of 256 threads per CU; one in-bounds store per thread keeps the
// result live.  Prints cycles per wave64 instruction per SIMD at 2.4 GHz.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <vector>

#define CHECK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s line %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

constexpr int ITERS = 4096;

#define CHAINS8(OP) OP(a0) OP(a1) OP(a2) OP(a3) OP(a4) OP(a5) OP(a6) OP(a7)

__global__ void k_fma_f32(float *out, float b, float c) {
    float a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    for (int i = 0; i < ITERS; ++i) {
#define OPF(x) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(x) : "v"(b), "v"(c));
        CHAINS8(OPF)
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;
}
__global__ void k_fract_f32(float *out, float b, float c) {
    float a0 = threadIdx.x * 0.1f, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    for (int i = 0; i < ITERS; ++i) {
#define OPR(x) asm volatile("v_fract_f32 %0, %0" : "+v"(x));
        CHAINS8(OPR)
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7 + b + c;
}
__global__ void k_fma_f64(float *out, double b, double c) {
    double a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    for (int i = 0; i < ITERS; ++i) {
#define OPD(x) asm volatile("v_fma_f64 %0, %1, %2, %0" : "+v"(x) : "v"(b), "v"(c));
        CHAINS8(OPD)
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = (float)(a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7);
}
__global__ void k_fract_f64(float *out, double b, double c) {
    double a0 = threadIdx.x * 0.1, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    for (int i = 0; i < ITERS; ++i) {
#define OPDR(x) asm volatile("v_fract_f64 %0, %0" : "+v"(x));
        CHAINS8(OPDR)
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = (float)(a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7 + b + c);
}
__global__ void k_cvt_i32_f64(float *out, double b, double c) {
    double d = threadIdx.x * 0.37 + b;
    int a0 = 0, a1 = 1, a2 = 2, a3 = 3, a4 = 4, a5 = 5, a6 = 6, a7 = 7;
    for (int i = 0; i < ITERS; ++i) {
#define OPC(x) asm volatile("v_cvt_i32_f64 %0, %1" : "+v"(x) : "v"(d));
        CHAINS8(OPC)
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = (float)(a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7) + (float)c;
}
__global__ void k_lshl_add(float *out, float b, float c) {
    uint32_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    uint32_t s = (uint32_t)b;
    for (int i = 0; i < ITERS; ++i) {
#define OPI(x) asm volatile("v_lshl_add_u32 %0, %0, 1, %1" : "+v"(x) : "v"(s));
        CHAINS8(OPI)
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = (float)(a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7) + c;
}
__global__ void k_add_f64(float *out, double b, double c) {
    double a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    for (int i = 0; i < ITERS; ++i) {
#define OPA(x) asm volatile("v_add_f64 %0, %0, %1" : "+v"(x) : "v"(b));
        CHAINS8(OPA)
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = (float)(a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7 + c);
}

int main() {
    int dev = 0; hipDeviceProp_t p; CHECK(hipGetDeviceProperties(&p, dev));
    int clk_khz = 0; CHECK(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeClockRate, dev));
    const int blocks = p.multiProcessorCount * 32, threads = 256;
    const size_t n = (size_t)blocks * threads;
    float *out = nullptr; CHECK(hipMalloc(&out, n * sizeof(float)));
    hipEvent_t e0, e1; CHECK(hipEventCreate(&e0)); CHECK(hipEventCreate(&e1));
    printf("CUs %d, clock attribute %.0f MHz, grid %d x %d\n", p.multiProcessorCount, clk_khz / 1e3, blocks, threads);
    struct K { const char *name; void (*f32)(float *, float, float); void (*f64)(float *, double, double); };
    K ks[] = {{"v_fma_f32", k_fma_f32, nullptr}, {"v_fract_f32", k_fract_f32, nullptr},
              {"v_lshl_add_u32", k_lshl_add, nullptr}, {"v_fma_f64", nullptr, k_fma_f64},
              {"v_add_f64", nullptr, k_add_f64}, {"v_fract_f64", nullptr, k_fract_f64},
              {"v_cvt_i32_f64", nullptr, k_cvt_i32_f64}};
    for (const K &k : ks) {
        float best = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
            CHECK(hipEventRecord(e0));
            if (k.f32) hipLaunchKernelGGL(k.f32, dim3(blocks), dim3(threads), 0, 0, out, 1.0000001f, 1e-7f);
            else hipLaunchKernelGGL(k.f64, dim3(blocks), dim3(threads), 0, 0, out, 1.0000001, 1e-7);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1)); CHECK(hipEventSynchronize(e1));
            float ms = 0; CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0 && ms < best) best = ms;
        }
        const double wave_instr = (double)n / 64 * ITERS * 8;
        const double simds = p.multiProcessorCount * 4.0;
        // wave-instructions per SIMD per microsecond and cycles per instruction at 2.4 GHz
        const double per_simd_per_s = wave_instr / simds / (best * 1e-3);
        printf("%-16s %8.3f ms  %.3f wave-instr/SIMD/ns  -> %.2f cycles each at 2.4 GHz\n",
               k.name, best, per_simd_per_s * 1e-9, 2.4e9 / per_simd_per_s);
    }
    CHECK(hipFree(out));
    return 0;
}
