// gce_kernels.hip -- CDNA4 (gfx950) kernels of the conditional-entropy
// (P, Pdot) search of Katz et al. 2020, Sec. 2.3.
//
// Pipeline of one execution (all on the caller's stream):
//   k_grid_setup  1/P and Pdot/2 per grid value, grid validity      (trial setup)
//   k_prepass     per curve: t0, magnitude bins, points grouped by
//                 magnitude bin (stable counting sort)               (prepass)
//   k_search_*    the fold of Eq. (3), 2-D histogram, Eq. (4)        (hot loop)
//   k_epilogue    per-curve minimum over the work units              (argmin)
//
// Search-kernel layout (one wave = one work unit):
//   lane l          <-> period index p = 64 * tile + l
//   trial t < TQ    <-> Pdot index q = TQ * group + t (same for the wave)
//   epoch k         <-> uniform across the wave: dt_k is read with scalar
//                       loads and enters the VALU as an SGPR operand.
// Epochs are pre-grouped by magnitude bin, so each lane only keeps a 1-D
// phase histogram per trial (the paper's Sec. 2.3 GPU observation that one
// magnitude value's phase counts suffice); at the end of each magnitude
// segment the histogram is folded into the entropy sums and cleared.
// Histograms live in LDS as [trial pair][phase bin][lane] 32-bit words: the
// low and high 16 bits count trials 2r and 2r+1, so one ds_add_u32 with
// value 1 or 0x10000 bins one point-trial, and lanes always hit distinct
// banks.  The marginal phase counts accumulate in registers.
//
// Entropy: N * H = sum_b c_b ln c_b - sum_{j,b} c_jb ln c_jb, which equals
// Eq. (4) multiplied by N; c ln c comes from a table built on the device.
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
__device__ __forceinline__ uint32_t lds_add(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Eq. (3) phase bin in binary64, bit-identical to the documented sequence
// y = fma(-Pdot/2, x^2, x); phi = y - floor(y); bin = (int)(phi * n_phase).
// v_fract_f64 returns y - floor(y) clamped to 1 - 2^-53; the clamp maps a
// phase that rounds up to 1 into the last bin, as the reference clamp does,
// and (1 - 2^-53) * n < n for every bin count n, so no clamp is needed.
__device__ __forceinline__ int fp64_phase_bin(double x, double x2,
                                              double half_pdot, double nph)
{
    const double y = __builtin_fma(-half_pdot, x2, x);
    const double fr = __builtin_amdgcn_fract(y);
    return (int)(fr * nph);
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
// c ln c table
// ---------------------------------------------------------------------------
__global__ void k_lut(double *lut, float *lut32, int32_t max_n)
{
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > max_n) return;
    const double v = (c == 0) ? 0.0 : (double)c * log((double)c);
    lut[c] = v;
    lut32[c] = (float)v;
}

hipError_t launch_lut(const DevPlan &dp, hipStream_t s)
{
    const int n = dp.max_n + 1;
    hipLaunchKernelGGL(k_lut, dim3((n + 255) / 256), dim3(256), 0, s,
                       const_cast<double *>(dp.lut),
                       const_cast<float *>(dp.lut32), dp.max_n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// trial setup: 1/P (correctly rounded division), Pdot/2 (exact), validity
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_grid_setup(DevPlan dp,
                                                    const double *periods,
                                                    const double *pdots)
{
    __shared__ int bad_sh;
    if (threadIdx.x == 0) bad_sh = 0;
    __syncthreads();
    int bad = 0;
    for (int64_t p = threadIdx.x; p < dp.n_p; p += blockDim.x) {
        const double P = periods[p];
        const bool ok = P >= kMinPeriod && P <= kMaxPeriod;  // false for NaN
        bad |= !ok;
        dp.inv_p[p] = ok ? 1.0 / P : 1.0;
    }
    for (int64_t q = threadIdx.x; q < dp.n_pd; q += blockDim.x) {
        const double Pd = pdots[q];
        const bool ok = fabs(Pd) <= kMaxAbsPdot;             // false for NaN
        bad |= !ok;
        dp.half_pd[q] = ok ? 0.5 * Pd : 0.0;
        dp.half_pd32[q] = ok ? (float)(0.5 * Pd) : 0.0f;
    }
    if (bad) atomicOr(&bad_sh, 1);
    __syncthreads();
    if (threadIdx.x == 0) *dp.grid_ok = bad_sh ? 0 : 1;
}

hipError_t launch_grid_setup(const DevPlan &dp, const double *periods,
                             const double *pdots, hipStream_t s)
{
    hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(256), 0, s, dp, periods,
                       pdots);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// prepass: one block per curve
// ---------------------------------------------------------------------------
constexpr int kPrepBlock = 256;
constexpr int kPrepChunk = 16384;   // epochs staged in LDS per scatter round

__device__ __forceinline__ double block_reduce(double v, bool is_min,
                                               double *sh)
{
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(v, off, kWave);
        v = is_min ? fmin(v, o) : fmax(v, o);
    }
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < kPrepBlock / kWave; ++i)
        r = is_min ? fmin(r, sh[i]) : fmax(r, sh[i]);
    return r;
}

__global__ __launch_bounds__(kPrepBlock) void k_prepass(
    DevPlan dp, const double *__restrict__ times, const double *__restrict__ mags)
{
    __shared__ uint8_t jb[kPrepChunk];
    __shared__ int32_t cnt[kMaxMagBins + 1];
    __shared__ int32_t cur[kMaxMagBins + 1];
    __shared__ double red[kPrepBlock / kWave];
    __shared__ int bad_sh;

    const int64_t c = blockIdx.x;
    const int64_t base = dp.off[c];
    const int32_t n = (int32_t)(dp.off[c + 1] - base);
    const int32_t n_mag = dp.n_mag;
    const double *t = times + base;
    const double *m = mags + base;

    if (threadIdx.x == 0) bad_sh = 0;
    for (int j = threadIdx.x; j <= kMaxMagBins; j += kPrepBlock) cnt[j] = 0;
    __syncthreads();

    // reductions: t0 = min t, t_max, magnitude range, finiteness
    double tmin = INFINITY, tmax = -INFINITY, mlo = INFINITY, mhi = -INFINITY;
    int bad = 0;
    for (int32_t k = threadIdx.x; k < n; k += kPrepBlock) {
        const double tk = t[k], mk = m[k];
        bad |= !(isfinite(tk) && isfinite(mk));
        tmin = fmin(tmin, tk);
        tmax = fmax(tmax, tk);
        mlo = fmin(mlo, mk);
        mhi = fmax(mhi, mk);
    }
    if (bad) atomicOr(&bad_sh, 1);
    tmin = block_reduce(tmin, true, red);
    tmax = block_reduce(tmax, false, red);
    mlo = block_reduce(mlo, true, red);
    mhi = block_reduce(mhi, false, red);
    __syncthreads();
    const bool ok = !bad_sh && (tmax - tmin) <= kMaxSpanDays;
    const double t0 = tmin;
    const bool flat_mag = !(mhi > mlo);

    // magnitude bin of every epoch; counts per bin
    for (int32_t k = threadIdx.x; k < n; k += kPrepBlock) {
        int32_t j = 0;
        if (ok && !flat_mag) {
            const double u = (m[k] - mlo) / (mhi - mlo);
            j = (int32_t)(u * (double)n_mag);
            if (j >= n_mag) j = n_mag - 1;
        }
        atomicAdd(&cnt[j], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t *seg = dp.seg + c * (int64_t)(n_mag + 1);
        int32_t acc = 0;
        for (int j = 0; j < n_mag; ++j) {
            seg[j] = acc;
            cur[j] = acc;
            acc += cnt[j];
        }
        seg[n_mag] = acc;
        dp.curve_ok[c] = ok ? 1 : 0;
    }
    __syncthreads();

    // stable scatter of dt = t - t0 into magnitude-bin order, in chunks
    double *dst = dp.dt_sorted + base;
    for (int32_t k0 = 0; k0 < n; k0 += kPrepChunk) {
        const int32_t k1 = min(n, k0 + kPrepChunk);
        for (int32_t k = k0 + threadIdx.x; k < k1; k += kPrepBlock) {
            int32_t j = 0;
            if (ok && !flat_mag) {
                const double u = (m[k] - mlo) / (mhi - mlo);
                j = (int32_t)(u * (double)n_mag);
                if (j >= n_mag) j = n_mag - 1;
            }
            jb[k - k0] = (uint8_t)j;
        }
        __syncthreads();
        const int j = threadIdx.x;
        if (j < n_mag) {
            int32_t pos = cur[j];
            for (int32_t k = k0; k < k1; ++k) {
                if (jb[k - k0] == j) {
                    dst[pos] = ok ? t[k] - t0 : 0.0;
                    ++pos;
                }
            }
            cur[j] = pos;
        }
        __syncthreads();
    }
}

hipError_t launch_prepass(const DevPlan &dp, const double *times,
                          const double *mags, hipStream_t s)
{
    hipLaunchKernelGGL(k_prepass, dim3((unsigned)dp.n_curves), dim3(kPrepBlock),
                       0, s, dp, times, mags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// search kernel (FP64 and split precision)
// ---------------------------------------------------------------------------
// Split-precision bin.  FP64 forms the point-period part x = dt / P, x^2 and
// frac(x) - 1/(2n) (the phase shifted down by half a bin); FP32 applies each
// trial's Pdot term, reduces mod 1 and rounds n * phase to the nearest
// integer by adding 1.5 * 2^23 (the float's low mantissa bits then hold the
// integer).  round(n * frac(y - 1/(2n))) equals floor(n * frac(y)), except
// that the upper half of bin 0 rounds to n: slot n is a wrap slot folded into
// bin 0 at each flush.  The shift is 2^-23 cycle short of half a bin: a phase
// exactly on a bin edge (every curve's first epoch has phase 0 for every
// trial) would otherwise be an exact rounding tie decided by the float
// rounding of 1/(2n); with the margin exact edges fall in the right bin, and
// only phases within 2^-23 cycle below an edge move up.  Accuracy is that of
// the FP32 Pdot term (~1e-7 of its size) and of frac(x) rounded to float
// (2^-25 cycle).
constexpr float kRoundMagic = 12582912.0f;           // 1.5 * 2^23
constexpr uint32_t kRoundMagicBits = 0x4B400000u;    // its bit pattern

__device__ __forceinline__ double split_shift(int nph)
{
    return 0.5 / (double)nph - 0x1p-23;
}

struct SplitPoint {
    float xf;    // frac(x) - 1/(2n)
    float x2f;   // x^2
};

__device__ __forceinline__ SplitPoint split_point(double dt, double invp,
                                                  double half_bin)
{
    const double x = dt * invp;
    SplitPoint sp;
    sp.xf = (float)(__builtin_amdgcn_fract(x) - half_bin);
    sp.x2f = (float)(x * x);
    return sp;
}

// Bit pattern kRoundMagicBits + slot, slot in [0, n] (n = wrap slot).
__device__ __forceinline__ uint32_t split_slot_bits(SplitPoint sp, float half_pdot,
                                                    float nph)
{
    const float y = __builtin_fmaf(-half_pdot, sp.x2f, sp.xf);
    const float fr = __builtin_amdgcn_fractf(y);
    return __float_as_uint(__builtin_fmaf(fr, nph, kRoundMagic));
}

constexpr int kPrecFp64 = GCE_PRECISION_FP64;
constexpr int kPrecSplit = GCE_PRECISION_SPLIT_FP32;

// NPH > 0: phase-bin count fixed at compile time, marginals in VGPRs.
// NPH = 0: runtime phase-bin count, marginals in LDS behind the histograms.
template <int PREC, int NPH, int TQ>
struct SearchShape {
    static constexpr int kRegions = (TQ + 1) / 2;
    static constexpr bool kLdsMarg = (NPH == 0);
    static constexpr int kWrap = (PREC == kPrecSplit) ? 1 : 0;   // extra slot
    // phase bins per scheduling group of the segment flush: ~8 words,
    // i.e. ~16 table loads, in flight at a time
    static constexpr int kFlushGroup = kRegions >= 8 ? 1 : 8 / kRegions;
};

template <int PREC, int NPH, int TQ>
__global__ __launch_bounds__(kWave) GCE_SEARCH_ATTR void k_search(DevPlan dp,
                                                                  void *out_ce_v)
{
    using S = SearchShape<PREC, NPH, TQ>;
    using OutT = typename std::conditional<PREC == kPrecFp64, double, float>::type;
    constexpr int R = S::kRegions;
    extern __shared__ uint32_t lds[];
    OutT *__restrict__ out_ce = static_cast<OutT *>(out_ce_v);

    const int lane = threadIdx.x;
    const int nph = NPH > 0 ? NPH : dp.n_phase;
    const int nslot = nph + S::kWrap;                   // LDS words per region
    // 2-D launch (a dispatch's grid size counts work-items in 32 bits):
    // unit = y * gridDim.x + x, in dispatch order
    const int64_t u = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (u >= dp.n_units) return;
    const int64_t rank = u / dp.units_per_curve;
    const int64_t rem = u - rank * dp.units_per_curve;
    const int32_t g = (int32_t)(rem / dp.n_ptiles);
    const int64_t tile = rem - (int64_t)g * dp.n_ptiles;
    const int32_t c = dp.order[rank];
    const int64_t base = dp.off[c];
    const int32_t n = (int32_t)(dp.off[c + 1] - base);
    const int64_t p = tile * kWave + lane;
    const bool p_ok = p < dp.n_p;
    const int32_t q0 = g * TQ;

    if (!(dp.curve_ok[c] && *dp.grid_ok)) {
        if (out_ce && p_ok) {
#pragma unroll
            for (int t = 0; t < TQ; ++t)
                if (q0 + t < dp.n_pd)
                    out_ce[((int64_t)c * dp.n_pd + q0 + t) * dp.n_p + p] = (OutT)NAN;
        }
        if (lane == 0) {
            dp.partials[u] = Partial{NAN, -1};
            dp.stats[u] = UnitStats{0.0, 0.0, 0.0};
        }
        return;
    }

    const double invp = dp.inv_p[p_ok ? p : dp.n_p - 1];
    double ha[TQ];
    float ha32[TQ];
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
        const int32_t q = min(q0 + t, (int32_t)dp.n_pd - 1);
        if constexpr (PREC == kPrecFp64) ha[t] = dp.half_pd[q];
        else ha32[t] = dp.half_pd32[q];
    }

    uint32_t *hist = lds;                                  // [R][nslot][64]
    uint32_t *lmarg = lds + (size_t)R * nslot * kWave;     // [R][nph][64] (NPH == 0)
    for (int i = 0; i < R * nslot; ++i) hist[i * kWave + lane] = 0;
    if (S::kLdsMarg)
        for (int i = 0; i < R * nph; ++i) lmarg[i * kWave + lane] = 0;
    uint32_t vmarg[R][NPH > 0 ? NPH : 1];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int b = 0; b < (NPH > 0 ? NPH : 1); ++b) vmarg[r][b] = 0;

    double s1[TQ];
#pragma unroll
    for (int t = 0; t < TQ; ++t) s1[t] = 0.0;

    const double nphd = (double)nph;
    const float nphf = (float)nph;
    const double half_bin = split_shift(nph);
    // split path: (bits << 8) of slot s is 0x40000000 + 256 s (mod 2^32)
    const uint32_t split_base = (uint32_t)lane * 4u - (kRoundMagicBits << 8);
    const double *__restrict__ dts = dp.dt_sorted + base;
    const int32_t *segc = dp.seg + (int64_t)c * (dp.n_mag + 1);
    const double *__restrict__ lut = dp.lut;
    uint32_t *hcol = hist + lane;
    char *lbytes = reinterpret_cast<char *>(lds);

    auto fold_point = [&](double dt) {
        if constexpr (PREC == kPrecFp64) {
            const double x = dt * invp;
            const double x2 = x * x;
#pragma unroll
            for (int t = 0; t < TQ; ++t) {
                const int b = fp64_phase_bin(x, x2, ha[t], nphd);
                lds_add(hcol + ((t >> 1) * nslot + b) * kWave,
                        (t & 1) ? 0x10000u : 1u);
            }
        } else {
            const SplitPoint sp = split_point(dt, invp, half_bin);
#pragma unroll
            for (int t = 0; t < TQ; ++t) {
                const uint32_t bits = split_slot_bits(sp, ha32[t], nphf);
                const uint32_t addr = (bits << 8) + split_base +
                                      (uint32_t)((t >> 1) * nslot * kWave * 4);
                lds_add(reinterpret_cast<uint32_t *>(lbytes + addr),
                        (t & 1) ? 0x10000u : 1u);
            }
        }
    };

    // end of a magnitude segment: sum c ln c, add to marginals, clear
    auto cell = [&](int r, int b) -> uint32_t * { return hcol + (r * nslot + b) * kWave; };
    auto add_lut = [&](int r, uint32_t w) {
        s1[2 * r] += lut[w & 0xffffu];
        if (2 * r + 1 < TQ) s1[2 * r + 1] += lut[w >> 16];
    };
    // One branch-free pass over the phase bins.  With 50%-overlapping bins,
    // bin b spans disjoint bins b and b + 1 (mod n): its count is the sum of
    // the two words (packed halves cannot overflow: together they hold at
    // most the curve's N epochs); with disjoint bins the neighbour is masked
    // to zero.  Bin 0's word (wrap slot merged) is kept in a register for
    // the last bin, so every cell is cleared as soon as it is read.
    const bool ovl = dp.overlap != 0;
    const uint32_t nb_mask = ovl ? 0xffffffffu : 0u;
    auto flush_segment = [&]() {
        uint32_t w0[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            w0[r] = *cell(r, 0);
            if (S::kWrap) {   // the wrap slot belongs to bin 0
                w0[r] += *cell(r, nph);
                *cell(r, nph) = 0;
            }
        }
        if constexpr (NPH > 0) {
#pragma unroll
            for (int b = 0; b < NPH; ++b) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t w = (b == 0) ? w0[r] : *cell(r, b);
                    const uint32_t wn = ((b + 1 < NPH) ? *cell(r, b + 1) : w0[r]) & nb_mask;
                    *cell(r, b) = 0;
                    vmarg[r][b] += w;
                    add_lut(r, w + wn);
                }
                // bound the table loads in flight (register pressure): no
                // memory access may move across this point
                if ((b + 1) % S::kFlushGroup == 0) asm volatile("" ::: "memory");
            }
        } else {
            for (int b = 0; b < nph; ++b) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t w = (b == 0) ? w0[r] : *cell(r, b);
                    const uint32_t wn = ((b + 1 < nph) ? *cell(r, b + 1) : w0[r]) & nb_mask;
                    *cell(r, b) = 0;
                    lmarg[(r * nph + b) * kWave + lane] += w;
                    add_lut(r, w + wn);
                }
            }
        }
    };

    for (int32_t j = 0; j < dp.n_mag; ++j) {
        const int32_t k0 = segc[j], k1 = segc[j + 1];
        if (k0 == k1) continue;
        // U epochs per iteration; optionally the next U epoch offsets are
        // loaded while the current ones are binned.
        constexpr int U = (TQ >= 8) ? GCE_UNROLL_LARGE_TQ : GCE_UNROLL_SMALL_TQ;
        int32_t k = k0;
        if (k + U <= k1) {
            double cur[U], nxt[U];
#pragma unroll
            for (int uu = 0; uu < U; ++uu) cur[uu] = dts[k + uu];
            while (true) {
                const int32_t kn = k + U;
                const bool more = kn + U <= k1;
                if (GCE_PREFETCH && more) {
#pragma unroll
                    for (int uu = 0; uu < U; ++uu) nxt[uu] = dts[kn + uu];
                }
#pragma unroll
                for (int uu = 0; uu < U; ++uu) fold_point(cur[uu]);
                k = kn;
                if (!more) break;
#pragma unroll
                for (int uu = 0; uu < U; ++uu)
                    cur[uu] = GCE_PREFETCH ? nxt[uu] : dts[k + uu];
            }
        }
        for (; k < k1; ++k) fold_point(dts[k]);

        flush_segment();
    }

    double s2[TQ];
#pragma unroll
    for (int t = 0; t < TQ; ++t) s2[t] = 0.0;
    auto marg_word = [&](int r, uint32_t w) {
        s2[2 * r] += lut[w & 0xffffu];
        if (2 * r + 1 < TQ) s2[2 * r + 1] += lut[w >> 16];
    };
    if constexpr (NPH > 0) {
        // the histograms are empty now: park the register marginals there and
        // sum them in a rolled loop (an unrolled one keeps every table load
        // in flight at once)
#pragma unroll
        for (int b = 0; b < NPH; ++b)
#pragma unroll
            for (int r = 0; r < R; ++r) hcol[(r * nslot + b) * kWave] = vmarg[r][b];
#pragma unroll 1
        for (int b = 0; b < NPH; ++b) {
            const int bn = (b + 1 == NPH) ? 0 : b + 1;
#pragma unroll
            for (int r = 0; r < R; ++r)
                marg_word(r, hcol[(r * nslot + b) * kWave] +
                                 (hcol[(r * nslot + bn) * kWave] & nb_mask));
        }
    } else {
        for (int b = 0; b < nph; ++b) {
            const int bn = (b + 1 == nph) ? 0 : b + 1;
#pragma unroll
            for (int r = 0; r < R; ++r)
                marg_word(r, lmarg[(r * nph + b) * kWave + lane] +
                                 (lmarg[(r * nph + bn) * kWave + lane] & nb_mask));
        }
    }

    // probabilities are counts / N, or counts / (2N) with overlapping bins
    const double nd = ovl ? 2.0 * (double)n : (double)n;
    double best_h = NAN;
    int64_t best_f = -1;
    double hv[TQ];
    double lsum = 0.0, lcnt = 0.0;
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
        const OutT h = (OutT)((s2[t] - s1[t]) / nd);
        hv[t] = (double)h;
        const int32_t q = q0 + t;
        if (p_ok && q < dp.n_pd) {
            const int64_t flat = (int64_t)q * dp.n_p + p;
            if (out_ce) out_ce[((int64_t)c * dp.n_pd + q) * dp.n_p + p] = h;
            if (lex_less(hv[t], flat, best_h, best_f)) {
                best_h = hv[t];
                best_f = flat;
            }
            lsum += hv[t];
            lcnt += 1.0;
        }
    }
    wave_argmin(best_h, best_f);
    // moments of this unit's CE values (two passes over registers)
    const double wcnt = wave_sum(lcnt);
    const double wmean = wave_sum(lsum) / wcnt;
    double lm2 = 0.0;
#pragma unroll
    for (int t = 0; t < TQ; ++t)
        if (p_ok && q0 + t < dp.n_pd) {
            const double d = hv[t] - wmean;
            lm2 += d * d;
        }
    const double wm2 = wave_sum(lm2);
    if (lane == 0) {
        dp.partials[u] = Partial{best_h, best_f};
        dp.stats[u] = UnitStats{wcnt, wmean, wm2};
    }
}

// ---------------------------------------------------------------------------
// variant table
// ---------------------------------------------------------------------------
using SearchFn = void (*)(DevPlan, void *);

struct Variant {
    int prec;
    int nph;   // 0 = generic
    int tq;
    SearchFn fn;
};

#define GCE_V(P, N, T) Variant{P, N, T, &k_search<P, N, T>}
static const Variant kVariants[] = {
    GCE_V(kPrecFp64, 10, 1), GCE_V(kPrecFp64, 10, 2), GCE_V(kPrecFp64, 10, 4),
    GCE_V(kPrecFp64, 10, 8),
    GCE_V(kPrecFp64, 15, 1), GCE_V(kPrecFp64, 15, 2), GCE_V(kPrecFp64, 15, 4),
    GCE_V(kPrecFp64, 15, 8),
    GCE_V(kPrecFp64, 20, 1), GCE_V(kPrecFp64, 20, 2), GCE_V(kPrecFp64, 20, 4),
    GCE_V(kPrecFp64, 20, 8),
    GCE_V(kPrecFp64, 50, 1), GCE_V(kPrecFp64, 50, 2), GCE_V(kPrecFp64, 50, 4),
    GCE_V(kPrecFp64, 0, 1),  GCE_V(kPrecFp64, 0, 2),  GCE_V(kPrecFp64, 0, 4),
    GCE_V(kPrecFp64, 0, 8),
    GCE_V(kPrecSplit, 10, 1), GCE_V(kPrecSplit, 10, 2), GCE_V(kPrecSplit, 10, 4),
    GCE_V(kPrecSplit, 10, 8),
    GCE_V(kPrecSplit, 15, 1), GCE_V(kPrecSplit, 15, 2), GCE_V(kPrecSplit, 15, 4),
    GCE_V(kPrecSplit, 15, 8),
    GCE_V(kPrecSplit, 20, 1), GCE_V(kPrecSplit, 20, 2), GCE_V(kPrecSplit, 20, 4),
    GCE_V(kPrecSplit, 20, 8),
    GCE_V(kPrecSplit, 50, 1), GCE_V(kPrecSplit, 50, 2), GCE_V(kPrecSplit, 50, 4),
    GCE_V(kPrecSplit, 0, 1),  GCE_V(kPrecSplit, 0, 2),  GCE_V(kPrecSplit, 0, 4),
    GCE_V(kPrecSplit, 0, 8),
};
#undef GCE_V

static const Variant *find_variant(int prec, int n_phase, int tq)
{
    for (const Variant &v : kVariants)
        if (v.prec == prec && v.nph == n_phase && v.tq == tq) return &v;
    for (const Variant &v : kVariants)
        if (v.prec == prec && v.nph == 0 && v.tq == tq) return &v;
    return nullptr;
}

bool search_variant_exists(int precision, int n_phase, int tq)
{
    return find_variant(precision, n_phase, tq) != nullptr;
}

size_t search_lds_bytes(int precision, int n_phase, int tq)
{
    const Variant *v = find_variant(precision, n_phase, tq);
    const size_t regions = (size_t)(tq + 1) / 2;
    const size_t slots = (size_t)n_phase + (precision == kPrecSplit ? 1 : 0);
    const size_t hist = regions * slots * kWave * sizeof(uint32_t);
    const size_t marg = regions * (size_t)n_phase * kWave * sizeof(uint32_t);
    return (v && v->nph == 0) ? hist + marg : hist;
}

hipError_t launch_search(const DevPlan &dp, void *out_ce, hipStream_t s)
{
    const Variant *v = find_variant(dp.precision, dp.n_phase, dp.tq);
    if (!v) return hipErrorInvalidValue;
    const size_t lds = search_lds_bytes(dp.precision, dp.n_phase, dp.tq);
    const int64_t gx = dp.n_units < kSearchGridX ? dp.n_units : kSearchGridX;
    const int64_t gy = (dp.n_units + gx - 1) / gx;
    hipLaunchKernelGGL(v->fn, dim3((unsigned)gx, (unsigned)gy), dim3(kWave), lds, s,
                       dp, out_ce);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// epilogue: per-curve minimum over the curve's work units
// ---------------------------------------------------------------------------
constexpr int kEpiBlock = 256;

__global__ __launch_bounds__(kEpiBlock) void k_epilogue(DevPlan dp,
                                                        gce_best_t *out_best)
{
    __shared__ double sh_h[kEpiBlock / kWave];
    __shared__ int64_t sh_f[kEpiBlock / kWave];
    __shared__ double sh_n[kEpiBlock], sh_mean[kEpiBlock], sh_m2[kEpiBlock];
    const int64_t rank = blockIdx.x;
    const int32_t c = dp.order[rank];
    const Partial *pp = dp.partials + rank * dp.units_per_curve;
    const UnitStats *ps = dp.stats + rank * dp.units_per_curve;
    double h = NAN;
    int64_t f = -1;
    double n = 0.0, mean = 0.0, m2 = 0.0;
    for (int64_t i = threadIdx.x; i < dp.units_per_curve; i += kEpiBlock) {
        const Partial v = pp[i];
        if (lex_less(v.h, v.flat, h, f)) {
            h = v.h;
            f = v.flat;
        }
        const UnitStats st = ps[i];
        moments_merge(n, mean, m2, st.n, st.mean, st.m2);
    }
    // moments: fixed-order tree over the block (deterministic)
    sh_n[threadIdx.x] = n;
    sh_mean[threadIdx.x] = mean;
    sh_m2[threadIdx.x] = m2;
    __syncthreads();
    for (int half = kEpiBlock / 2; half >= 1; half >>= 1) {
        if (threadIdx.x < half) {
            double a = sh_n[threadIdx.x], b = sh_mean[threadIdx.x], d = sh_m2[threadIdx.x];
            moments_merge(a, b, d, sh_n[threadIdx.x + half], sh_mean[threadIdx.x + half],
                          sh_m2[threadIdx.x + half]);
            sh_n[threadIdx.x] = a;
            sh_mean[threadIdx.x] = b;
            sh_m2[threadIdx.x] = d;
        }
        __syncthreads();
    }
    wave_argmin(h, f);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sh_h[w] = h;
        sh_f[w] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kEpiBlock / kWave; ++i)
            if (lex_less(sh_h[i], sh_f[i], h, f)) {
                h = sh_h[i];
                f = sh_f[i];
            }
        gce_best_t b;
        const bool ok = dp.curve_ok[c] && *dp.grid_ok && f >= 0 && sh_n[0] > 0.0;
        b.flat_index = ok ? f : -1;
        b.period_index = ok ? (int32_t)(f % dp.n_p) : -1;
        b.pdot_index = ok ? (int32_t)(f / dp.n_p) : -1;
        b.ce_min = ok ? h : NAN;
        const double sd = sqrt(sh_m2[0] / sh_n[0]);
        b.ce_mean = ok ? sh_mean[0] : NAN;
        b.ce_std = ok ? sd : NAN;
        b.significance = ok ? (sd > 0.0 ? (sh_mean[0] - h) / sd : 0.0) : NAN;
        out_best[c] = b;
    }
}

hipError_t launch_epilogue(const DevPlan &dp, gce_best_t *out_best,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_epilogue, dim3((unsigned)dp.n_curves), dim3(kEpiBlock),
                       0, s, dp, out_best);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// debug counts: one thread per requested trial, same binning as the search
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_debug_counts(
    DevPlan dp, const int64_t *__restrict__ trial_curve,
    const int64_t *__restrict__ trial_flat, int64_t n_trials,
    uint32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_trials) return;
    const int32_t nph = dp.n_phase, nmag = dp.n_mag;
    uint32_t *o = out + i * (int64_t)nph * nmag;
    for (int64_t e = 0; e < (int64_t)nph * nmag; ++e) o[e] = 0;
    const int64_t c = trial_curve[i], f = trial_flat[i];
    if (c < 0 || c >= dp.n_curves || f < 0 || f >= dp.n_p * dp.n_pd) return;
    if (!(dp.curve_ok[c] && *dp.grid_ok)) return;
    const int64_t q = f / dp.n_p, p = f % dp.n_p;
    const double invp = dp.inv_p[p], ha = dp.half_pd[q];
    const float ha32 = dp.half_pd32[q];
    const double half_bin = split_shift(nph);
    const int64_t base = dp.off[c];
    const int32_t *segc = dp.seg + c * (int64_t)(nmag + 1);
    for (int32_t j = 0; j < nmag; ++j) {
        for (int32_t k = segc[j]; k < segc[j + 1]; ++k) {
            const double dt = dp.dt_sorted[base + k];
            int b;
            if (dp.precision == kPrecFp64) {
                const double x = dt * invp;
                const double x2 = x * x;
                b = fp64_phase_bin(x, x2, ha, (double)nph);
            } else {
                const SplitPoint sp = split_point(dt, invp, half_bin);
                b = (int)(split_slot_bits(sp, ha32, (float)nph) - kRoundMagicBits);
                if (b == nph) b = 0;   // wrap slot
            }
            b = b < 0 ? 0 : (b >= nph ? nph - 1 : b);
            o[(int64_t)j * nph + b] += 1;
        }
        if (dp.overlap) {   // bin b spans disjoint bins b and b + 1 (mod n)
            uint32_t *row = o + (int64_t)j * nph;
            const uint32_t first = row[0];
            for (int32_t b = 0; b < nph; ++b)
                row[b] += (b + 1 < nph) ? row[b + 1] : first;
        }
    }
}

hipError_t launch_debug_counts(const DevPlan &dp, const int64_t *trial_curve,
                               const int64_t *trial_flat, int64_t n_trials,
                               uint32_t *out_counts, hipStream_t s)
{
    if (n_trials == 0) return hipSuccess;
    hipLaunchKernelGGL(k_debug_counts, dim3((unsigned)((n_trials + 63) / 64)),
                       dim3(64), 0, s, dp, trial_curve, trial_flat, n_trials,
                       out_counts);
    return hipGetLastError();
}

}  // namespace gce
