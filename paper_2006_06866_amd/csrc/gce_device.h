// gce_device.h -- device helpers shared by the search, prepass, epilogue
// and debug kernels (Katz et al. 2020, Sec. 2.3).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "gce_internal.h"

// Tuning of the search kernel's epoch loop (measured on MI355X).
#ifndef GCE_UNROLL_SMALL_TQ
#define GCE_UNROLL_SMALL_TQ 8   // epochs per iteration, trials_per_lane <= 4
#endif
#ifndef GCE_UNROLL_LARGE_TQ
#define GCE_UNROLL_LARGE_TQ 4   // epochs per iteration, trials_per_lane = 8
#endif
#ifndef GCE_PREFETCH
#define GCE_PREFETCH 0          // load the next epochs during the current ones
#endif
#ifndef GCE_RD_GROUP
#define GCE_RD_GROUP 8          // FP64 bin fmas per rounding-mode switch
#endif
#ifndef GCE_FLUSH_ACC
#define GCE_FLUSH_ACC 4         // partial entropy sums per trial (trials_per_lane <= 2)
#endif
#ifndef GCE_FLUSH_WORDS
#define GCE_FLUSH_WORDS 8       // histogram words per scheduling group of the flush
#endif
#ifndef GCE_SCALAR_EPOCHS
#define GCE_SCALAR_EPOCHS 1     // read epoch offsets with scalar loads
#endif
#ifndef GCE_CUM_GROUP
#define GCE_CUM_GROUP 12        // phase bins per group of the cumulative flush (one trial pair)
#endif
#ifndef GCE_WAVES_PER_EU
#define GCE_WAVES_PER_EU 0      // occupancy hint for the search kernel (0: none)
#endif
#if GCE_WAVES_PER_EU > 0
#define GCE_SEARCH_ATTR __attribute__((amdgpu_waves_per_eu(GCE_WAVES_PER_EU)))
#else
#define GCE_SEARCH_ATTR
#endif
namespace gce {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Read-only, wave-uniform arrays (a curve's epoch offsets and segment
// starts) are read through the constant address space, so the loads become
// scalar loads into SGPRs that the vector instructions take as operands.
#if GCE_SCALAR_EPOCHS
typedef __attribute__((address_space(4))) const double uniform_f64;
typedef __attribute__((address_space(4))) const float uniform_f32;
typedef __attribute__((address_space(4))) const int32_t uniform_i32;
#else
typedef const double uniform_f64;
typedef const float uniform_f32;
typedef const int32_t uniform_i32;
#endif

__device__ __forceinline__ uint32_t lds_add(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// The same for a cell that the other waves of the block add into too.
__device__ __forceinline__ uint32_t lds_add_block(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Eq. (3) phase bins in binary64, bit-identical to the documented sequence
// y = fma(-Pdot/2, x^2, x); phi = y - floor(y); bin = floor(phi * n_phase),
// the floor taken of the exact product.
//  - v_fract_f64 returns y - floor(y) clamped to 1 - 2^-53: a phase that
//    rounds up to 1 lands in the last bin, as floor((1 - 2^-53) n) = n - 1.
//  - floor(phi * n) exactly: one fma phi * n + 2^52 rounded toward minus
//    infinity.  Doubles in [2^52, 2^53) are the integers, so the result is
//    2^52 + floor(phi * n) and its low word is the bin (phi * n < 128).  The
//    MODE register's FP64 rounding field (bits 3:2; 2 = toward -inf, 0 =
//    nearest even) is switched around these fmas only, inside one asm block
//    so that no other floating-point instruction runs in that mode.
constexpr uint64_t kTwo52Bits = 0x4330000000000000ull;

template <int T>
__device__ __forceinline__ void fp64_floor_products(double (&phi)[T], double n,
                                                    uint32_t (&bin)[T]);

// The FP_ROUND field is written twice per block; two writes of one hardware
// register need two wait states between them, which the fmas (or, for a
// single fma, an s_nop) provide.  Vector instructions need none after it.
#define GCE_RD_BEGIN "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2\n\t"
#define GCE_RD_END "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0"

template <>
__device__ __forceinline__ void fp64_floor_products<1>(double (&phi)[1], double n,
                                                       uint32_t (&bin)[1])
{
    const double m = __longlong_as_double((long long)kTwo52Bits);
    asm volatile(GCE_RD_BEGIN
                 "v_fma_f64 %0, %0, %1, %2\n\t"
                 "s_nop 1\n\t"
                 GCE_RD_END
                 : "+v"(phi[0])
                 : "s"(n), "v"(m));
#pragma unroll
    for (int t = 0; t < 1; ++t) bin[t] = (uint32_t)__double2loint(phi[t]);
}

template <>
__device__ __forceinline__ void fp64_floor_products<2>(double (&phi)[2], double n,
                                                       uint32_t (&bin)[2])
{
    const double m = __longlong_as_double((long long)kTwo52Bits);
    asm volatile(GCE_RD_BEGIN
                 "v_fma_f64 %0, %0, %2, %3\n\t"
                 "v_fma_f64 %1, %1, %2, %3\n\t"
                 GCE_RD_END
                 : "+v"(phi[0]), "+v"(phi[1])
                 : "s"(n), "v"(m));
#pragma unroll
    for (int t = 0; t < 2; ++t) bin[t] = (uint32_t)__double2loint(phi[t]);
}

template <>
__device__ __forceinline__ void fp64_floor_products<4>(double (&phi)[4], double n,
                                                       uint32_t (&bin)[4])
{
    const double m = __longlong_as_double((long long)kTwo52Bits);
    asm volatile(GCE_RD_BEGIN
                 "v_fma_f64 %0, %0, %4, %5\n\t"
                 "v_fma_f64 %1, %1, %4, %5\n\t"
                 "v_fma_f64 %2, %2, %4, %5\n\t"
                 "v_fma_f64 %3, %3, %4, %5\n\t"
                 GCE_RD_END
                 : "+v"(phi[0]), "+v"(phi[1]), "+v"(phi[2]), "+v"(phi[3])
                 : "s"(n), "v"(m));
#pragma unroll
    for (int t = 0; t < 4; ++t) bin[t] = (uint32_t)__double2loint(phi[t]);
}

template <>
__device__ __forceinline__ void fp64_floor_products<8>(double (&phi)[8], double n,
                                                       uint32_t (&bin)[8])
{
    const double m = __longlong_as_double((long long)kTwo52Bits);
    asm volatile(GCE_RD_BEGIN
                 "v_fma_f64 %0, %0, %8, %9\n\t"
                 "v_fma_f64 %1, %1, %8, %9\n\t"
                 "v_fma_f64 %2, %2, %8, %9\n\t"
                 "v_fma_f64 %3, %3, %8, %9\n\t"
                 "v_fma_f64 %4, %4, %8, %9\n\t"
                 "v_fma_f64 %5, %5, %8, %9\n\t"
                 "v_fma_f64 %6, %6, %8, %9\n\t"
                 "v_fma_f64 %7, %7, %8, %9\n\t"
                 GCE_RD_END
                 : "+v"(phi[0]), "+v"(phi[1]), "+v"(phi[2]), "+v"(phi[3]), "+v"(phi[4]), "+v"(phi[5]), "+v"(phi[6]), "+v"(phi[7])
                 : "s"(n), "v"(m));
#pragma unroll
    for (int t = 0; t < 8; ++t) bin[t] = (uint32_t)__double2loint(phi[t]);
}

template <>
__device__ __forceinline__ void fp64_floor_products<16>(double (&phi)[16], double n,
                                                       uint32_t (&bin)[16])
{
    const double m = __longlong_as_double((long long)kTwo52Bits);
    asm volatile(GCE_RD_BEGIN
                 "v_fma_f64 %0, %0, %16, %17\n\t"
                 "v_fma_f64 %1, %1, %16, %17\n\t"
                 "v_fma_f64 %2, %2, %16, %17\n\t"
                 "v_fma_f64 %3, %3, %16, %17\n\t"
                 "v_fma_f64 %4, %4, %16, %17\n\t"
                 "v_fma_f64 %5, %5, %16, %17\n\t"
                 "v_fma_f64 %6, %6, %16, %17\n\t"
                 "v_fma_f64 %7, %7, %16, %17\n\t"
                 "v_fma_f64 %8, %8, %16, %17\n\t"
                 "v_fma_f64 %9, %9, %16, %17\n\t"
                 "v_fma_f64 %10, %10, %16, %17\n\t"
                 "v_fma_f64 %11, %11, %16, %17\n\t"
                 "v_fma_f64 %12, %12, %16, %17\n\t"
                 "v_fma_f64 %13, %13, %16, %17\n\t"
                 "v_fma_f64 %14, %14, %16, %17\n\t"
                 "v_fma_f64 %15, %15, %16, %17\n\t"
                 GCE_RD_END
                 : "+v"(phi[0]), "+v"(phi[1]), "+v"(phi[2]), "+v"(phi[3]), "+v"(phi[4]), "+v"(phi[5]), "+v"(phi[6]), "+v"(phi[7]), "+v"(phi[8]), "+v"(phi[9]), "+v"(phi[10]), "+v"(phi[11]), "+v"(phi[12]), "+v"(phi[13]), "+v"(phi[14]), "+v"(phi[15])
                 : "s"(n), "v"(m));
#pragma unroll
    for (int t = 0; t < 16; ++t) bin[t] = (uint32_t)__double2loint(phi[t]);
}

#undef GCE_RD_BEGIN
#undef GCE_RD_END

// Bins of G epochs under T Pdot trials each (x = dt / P, x2 = x^2 per
// epoch): bin[g * T + t].  All G * T round-down fmas share one mode switch.
template <int G, int T>
__device__ __forceinline__ void fp64_phase_bins(const double (&x)[G], const double (&x2)[G],
                                                const double (&half_pdot)[T], double nph,
                                                uint32_t (&bin)[G * T])
{
    double phi[G * T];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int t = 0; t < T; ++t)
            phi[g * T + t] = __builtin_amdgcn_fract(__builtin_fma(-half_pdot[t], x2[g], x[g]));
    fp64_floor_products<G * T>(phi, nph, bin);
}

// Sums of the low (high) 16-bit halves of two words in one instruction: an
// SDWA add selecting the same half of both operands.
__device__ __forceinline__ uint32_t add_low_halves(uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD "
        "src0_sel:WORD_0 src1_sel:WORD_0"
        : "=v"(r)
        : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ uint32_t add_high_halves(uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD "
        "src0_sel:WORD_1 src1_sel:WORD_1"
        : "=v"(r)
        : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ bool lex_less(double h1, int64_t f1, double h2,
                                         int64_t f2)
{
    // NaN never wins; among equal values the lower flat index wins.
    if (f2 < 0) return f1 >= 0;
    if (f1 < 0) return false;
    return (h1 < h2) || (h1 == h2 && f1 < f2);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Chan et al. pairwise update of (count, mean, M2) with another part.
__device__ __forceinline__ void moments_merge(double &n, double &mean, double &m2,
                                              double nb, double mb, double m2b)
{
    if (nb == 0.0) return;
    if (n == 0.0) {
        n = nb;
        mean = mb;
        m2 = m2b;
        return;
    }
    const double nn = n + nb;
    const double d = mb - mean;
    mean += d * (nb / nn);
    m2 += m2b + d * d * (n * nb / nn);
    n = nn;
}

__device__ __forceinline__ void wave_argmin(double &h, int64_t &f)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ho = __shfl_xor(h, off, kWave);
        const int64_t fo = __shfl_xor(f, off, kWave);
        if (lex_less(ho, fo, h, f)) {
            h = ho;
            f = fo;
        }
    }
}

// ---------------------------------------------------------------------------
// split-precision binning
// ---------------------------------------------------------------------------
// Split-precision bin.  FP64 forms x = dt / P and frac(x) (the step whose
// magnitude needs it); FP32 converts frac(x) to float, forms x^2 as the
// product of dt^2 and (1/P)^2 (each rounded to float once, to nearest: dt^2
// by the prepass, (1/P)^2 by the grid set-up), applies each trial's Pdot
// term with one fma, reduces mod 1 (v_fract_f32, exact) and floors
// n * phase by adding 1.5 * 2^23 in one fma: with the FP32 rounding mode set
// toward minus infinity (split_round_down), the sum rounds to 1.5 * 2^23 +
// floor(n * phase) of the exact product, and the float's low mantissa bits
// hold that integer.  The phase is below 1, so the slot is in [0, n).  Every
// FP32 instruction between split_round_down and split_round_nearest rounds
// down: the conversion of frac(x), the product x^2 and the Pdot fma err by
// under one ulp each (frac(x): 2^-24 cycle; the Pdot term: under 2.5 * 2^-23
// of its size with the roundings of its factors), always in the same
// direction.
constexpr float kRoundMagic = 12582912.0f;           // 1.5 * 2^23
constexpr uint32_t kRoundMagicBits = 0x4B400000u;    // its bit pattern

// MODE register, FP_ROUND field bits 1:0 (FP32): 2 = toward -inf, 0 = nearest
// even; the FP64 field (bits 3:2) is left alone.  The builtin (rather than
// inline asm) tells the compiler that the write defines the mode register
// that every FP32 instruction reads, so none is scheduled across it.  The
// optimiser above that level still assumes the default rounding, so no FP32
// value computed before split_round_down may be one that the binning also
// computes (it could be reused): there is none.
constexpr int kHwregModeFp32Round = 1 | (0 << 6) | ((2 - 1) << 11);   // hwreg(MODE, 0, 2)
__device__ __forceinline__ void split_round_down()
{
    __builtin_amdgcn_s_setreg(kHwregModeFp32Round, 2);
}
__device__ __forceinline__ void split_round_nearest()
{
    __builtin_amdgcn_s_setreg(kHwregModeFp32Round, 0);
}

struct SplitPoint {
    float xf;    // frac(x)
    float x2f;   // x^2
};

// dt2f: dt^2 rounded to float (by the prepass); invp2f: (1/P)^2 rounded to
// float (by the grid set-up)
__device__ __forceinline__ SplitPoint split_point(double dt, double invp, float dt2f,
                                                  float invp2f)
{
    const double x = dt * invp;
    SplitPoint sp;
    // FP64 only where the magnitude of x demands it (x and its fraction),
    // the square as dt^2 (1/P)^2 in FP32 (a half-slot instruction)
    sp.xf = (float)__builtin_amdgcn_fract(x);
    sp.x2f = dt2f * invp2f;
    return sp;
}

// Bit pattern kRoundMagicBits + slot, slot = floor(n * phase) in [0, n),
// under split_round_down.
__device__ __forceinline__ uint32_t split_slot_bits(SplitPoint sp, float half_pdot,
                                                    float nph)
{
    const float y = __builtin_fmaf(-half_pdot, sp.x2f, sp.xf);
    const float fr = __builtin_amdgcn_fractf(y);
    return __float_as_uint(__builtin_fmaf(fr, nph, kRoundMagic));
}

constexpr int kPrecFp64 = GCE_PRECISION_FP64;
constexpr int kPrecSplit = GCE_PRECISION_SPLIT_FP32;

}  // namespace gce
