// gce_kernels.hip -- CDNA4 (gfx950) kernels of the conditional-entropy
// (P, Pdot) search of Katz et al. 2020, Sec. 2.3.
//
// Pipeline of one execution (all on the caller's stream):
//   k_prepass     per curve: t0, magnitude bins, points grouped by
//                 magnitude bin (stable counting sort)               (prepass)
//   k_grid_setup  1/P and Pdot/2 per grid value, grid validity      (trial setup)
//   k_search      the fold of Eq. (3), 2-D histogram, Eq. (4)        (hot loop,
//                 gce_search.h, instantiated by gce_search_*.hip)
//   k_epilogue    per-curve minimum over the work units              (argmin)
#include <mutex>
#include <unordered_map>

#include "gce_device.h"

namespace gce {

// ---------------------------------------------------------------------------
// c ln c table
// ---------------------------------------------------------------------------
__global__ void k_lut(double *lut, int32_t max_count)
{
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > max_count) return;
    lut[c] = (c == 0) ? 0.0 : (double)c * log((double)c);
}

hipError_t launch_lut(const DevPlan &dp, hipStream_t s)
{
    const int n = dp.max_count + 1;
    hipLaunchKernelGGL(k_lut, dim3((n + 255) / 256), dim3(256), 0, s,
                       const_cast<double *>(dp.lut), dp.max_count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// trial setup: 1/P (correctly rounded division), Pdot/2 (exact), validity;
// for the split path also (1/P)^2 and Pdot/2 rounded to float here, in the
// default rounding, so that every kernel reading them sees the same values.
// Grid-stride over the period and Pdot axes.  The prepass (launched first)
// sets grid_ok to 1; any thread that meets an invalid value stores 0 (all
// writers store the same value, so no atomics are needed).
// ---------------------------------------------------------------------------
constexpr int kGridBlock = 256;

__global__ __launch_bounds__(kGridBlock) void k_grid_setup(DevPlan dp,
                                                          const double *periods,
                                                          const double *pdots)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double p_min = dp.precision == kPrecSplit ? kSplitMinPeriod : kMinPeriod;
    bool bad = false;
    for (int64_t p = i0; p < dp.n_p; p += stride) {
        const double P = periods[p];
        const bool ok = P >= p_min && P <= kMaxPeriod;       // false for NaN
        bad |= !ok;
        const double ip = ok ? 1.0 / P : 1.0;
        dp.inv_p[p] = ip;
        if (dp.inv_p2f) dp.inv_p2f[p] = (float)(ip * ip);
    }
    for (int64_t q = i0; q < dp.n_pd; q += stride) {
        const double Pd = pdots[q];
        const bool ok = fabs(Pd) <= kMaxAbsPdot;             // false for NaN
        bad |= !ok;
        dp.half_pd[q] = ok ? 0.5 * Pd : 0.0;
        dp.half_pd32[q] = ok ? (float)(0.5 * Pd) : 0.0f;
    }
    if (bad) *dp.grid_ok = 0;
}

hipError_t launch_grid_setup(const DevPlan &dp, const double *periods,
                             const double *pdots, hipStream_t s)
{
    const int64_t n = dp.n_p > dp.n_pd ? dp.n_p : dp.n_pd;
    int64_t blocks = (n + kGridBlock - 1) / kGridBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_grid_setup, dim3((unsigned)blocks), dim3(kGridBlock), 0, s, dp,
                       periods, pdots);
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

// Magnitude bins of one epoch from its normalised magnitude u in [0, 1]
// (Sec. 2.3).  Disjoint bins: bin j is [j, j + 1) / n_mag.  50%-overlapping
// bins: bin j is [j, j + 2) / (n_mag + 1), so the sub-interval
// s = floor(u (n_mag + 1)) belongs to bins s - 1 and s where they exist.  The
// top edge u = 1 belongs to the last bin.  `second` is kNoBin unless the
// epoch lies in two bins.
constexpr uint8_t kNoBin = 255;   // n_mag <= 255: bins are 0..254
struct MagBins {
    int32_t first, second;
};

// floor(u * n) of the exact product, at most n - 1: the rounded product is
// right unless it rounded up onto an integer, which the sign of the exact
// remainder u * n - p (one fma) tells.
__device__ __forceinline__ int32_t floor_product_bin(double u, int32_t n)
{
    const double nd = (double)n;
    const double p = u * nd;
    int32_t b = (int32_t)p;   // u >= 0: truncation is the floor of p
    if ((double)b == p && __builtin_fma(u, nd, -p) < 0.0) --b;
    return b < n ? b : n - 1;
}

__device__ __forceinline__ MagBins magnitude_bins(double u, int32_t n_mag, bool overlap)
{
    if (!overlap) return MagBins{floor_product_bin(u, n_mag), kNoBin};
    const int32_t s = floor_product_bin(u, n_mag + 1);
    if (s == 0) return MagBins{0, kNoBin};
    if (s == n_mag) return MagBins{n_mag - 1, kNoBin};
    return MagBins{s - 1, s};
}

__global__ __launch_bounds__(kPrepBlock) void k_prepass(
    DevPlan dp, const double *__restrict__ times, const double *__restrict__ mags)
{
    __shared__ uint8_t jb[kPrepChunk];
    __shared__ uint8_t jb2[kPrepChunk];   // second bin (overlapping bins)
    __shared__ int32_t cnt[kMaxMagBins + 1];
    __shared__ int32_t cur[kMaxMagBins + 1];
    __shared__ double red[kPrepBlock / kWave];
    __shared__ int bad_sh;

    const int64_t c = blockIdx.x;
    if (c == 0 && threadIdx.x == 0) *dp.grid_ok = 1;   // the grid set-up may clear it
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
    const double max_span = dp.precision == kPrecSplit ? kSplitMaxSpanDays : kMaxSpanDays;
    const bool ok = !bad_sh && (tmax - tmin) <= max_span;
    const double t0 = tmin;
    const bool flat_mag = !(mhi > mlo);

    // magnitude bins of every epoch (a constant or invalid curve has one
    // bin); entries per bin
    const bool movl = dp.mag_overlap != 0;
    auto bins_of = [&](int32_t k) -> MagBins {
        if (!ok || flat_mag) return MagBins{0, kNoBin};
        return magnitude_bins((m[k] - mlo) / (mhi - mlo), n_mag, movl);
    };
    for (int32_t k = threadIdx.x; k < n; k += kPrepBlock) {
        const MagBins mb = bins_of(k);
        atomicAdd(&cnt[mb.first], 1);
        if (mb.second != kNoBin) atomicAdd(&cnt[mb.second], 1);
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

    // stable scatter of dt = t - t0 (and, for the split path, of dt^2
    // rounded to float) into magnitude-bin order, in chunks; an epoch in two
    // bins is written into both segments
    const int64_t dbase = movl ? 2 * base : base;
    double *dst = dp.dt_sorted + dbase;
    float *dst2 = dp.dt2f_sorted ? dp.dt2f_sorted + dbase : nullptr;
    for (int32_t k0 = 0; k0 < n; k0 += kPrepChunk) {
        const int32_t k1 = min(n, k0 + kPrepChunk);
        for (int32_t k = k0 + threadIdx.x; k < k1; k += kPrepBlock) {
            const MagBins mb = bins_of(k);
            jb[k - k0] = (uint8_t)mb.first;
            jb2[k - k0] = (uint8_t)mb.second;
        }
        __syncthreads();
        const int j = threadIdx.x;
        if (j < n_mag) {
            int32_t pos = cur[j];
            for (int32_t k = k0; k < k1; ++k) {
                if (jb[k - k0] == j || jb2[k - k0] == j) {
                    const double dt = ok ? t[k] - t0 : 0.0;
                    dst[pos] = dt;
                    if (dst2) dst2[pos] = (float)(dt * dt);
                    ++pos;
                }
            }
            cur[j] = pos;
        }
        __syncthreads();
    }
}

// identity schedule: rank r searches curve r
__global__ void k_iota_order(int32_t *order, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) order[i] = (int32_t)i;
}

hipError_t launch_iota_order(const DevPlan &dp, hipStream_t s)
{
    hipLaunchKernelGGL(k_iota_order, dim3((unsigned)((dp.n_curves + 255) / 256)), dim3(256),
                       0, s, const_cast<int32_t *>(dp.order), dp.n_curves);
    return hipGetLastError();
}

hipError_t launch_prepass(const DevPlan &dp, const double *times,
                          const double *mags, hipStream_t s)
{
    hipLaunchKernelGGL(k_prepass, dim3((unsigned)dp.n_curves), dim3(kPrepBlock),
                       0, s, dp, times, mags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// search-kernel dispatch
// ---------------------------------------------------------------------------
static SearchTable search_table(int precision, int overlap)
{
    if (precision == kPrecFp64) return overlap ? search_table_fp64_overlap() : search_table_fp64();
    return overlap ? search_table_split_overlap() : search_table_split();
}

// Two-wave variants exist only for their own phase-bin count; one-wave
// variants fall back on the runtime-count kernel.
static const SearchVariant *find_variant(int prec, int overlap, int n_phase, int tq, int ll,
                                         int co = 1)
{
    const SearchTable t = search_table(prec, overlap);
    for (int32_t i = 0; i < t.n; ++i)
        if (t.v[i].nph == n_phase && t.v[i].tq == tq && t.v[i].ll == ll && t.v[i].co == co)
            return &t.v[i];
    if (co != 1) return nullptr;
    for (int32_t i = 0; i < t.n; ++i)
        if (t.v[i].nph == 0 && t.v[i].tq == tq && t.v[i].ll == ll && t.v[i].co == 1)
            return &t.v[i];
    return nullptr;
}

bool search_variant_exists(int precision, int n_phase, int tq, int co)
{
    return find_variant(precision, 0, n_phase, tq, 0, co) != nullptr;
}

size_t search_lds_bytes(int precision, int n_phase, int tq, int lut_lds, int max_count, int co)
{
    const SearchVariant *v = find_variant(precision, 0, n_phase, tq, 0);
    const size_t regions = (size_t)(tq + 1) / 2;
    const size_t slots = (size_t)n_phase;
    const size_t hist = regions * slots * kWave * sizeof(uint32_t);
    const size_t marg = regions * (size_t)n_phase * kWave * sizeof(uint32_t);
    // two waves per unit keep one copy of the unit's histograms
    size_t bytes = co == 2 ? hist
                           : ((v && v->nph == 0) ? hist + marg : hist) * search_waves_per_block(lut_lds);
    if (lut_lds) bytes += sizeof(double) * (size_t)(max_count + 1);
    return bytes;
}

// A variant with the c ln c table in LDS reads the table by LDS address,
// taking the table to open the kernel's dynamic LDS at address 0; that holds
// when the kernel has no static LDS, which is checked once per variant here.
static bool table_at_lds_zero(const SearchVariant *v)
{
    static std::mutex mu;
    static std::unordered_map<const void *, bool> known;
    const void *fn = reinterpret_cast<const void *>(v->fn);
    std::lock_guard<std::mutex> lock(mu);
    auto it = known.find(fn);
    if (it != known.end()) return it->second;
    hipFuncAttributes a;
    const bool ok = hipFuncGetAttributes(&a, fn) == hipSuccess && a.sharedSizeBytes == 0;
    known.emplace(fn, ok);
    return ok;
}

bool search_table_in_lds_ok(int precision, int overlap, int n_phase, int tq, int co)
{
    const SearchVariant *v = find_variant(precision, overlap, n_phase, tq, 1, co);
    return v && table_at_lds_zero(v);
}

hipError_t launch_search(const DevPlan &dp, void *out_ce, hipStream_t s)
{
    const SearchVariant *v =
        find_variant(dp.precision, dp.overlap, dp.n_phase, dp.tq, dp.lut_lds, dp.co);
    if (!v) return hipErrorInvalidValue;
    if (v->ll && !table_at_lds_zero(v)) return hipErrorInvalidDeviceFunction;
    const size_t lds =
        search_lds_bytes(dp.precision, dp.n_phase, dp.tq, dp.lut_lds, dp.max_count, dp.co);
    const int wpb = search_waves_per_block(dp.lut_lds, dp.co);
    const int upb = dp.co == 2 ? 1 : wpb;   // work units per block
    const int64_t blocks = (dp.n_units - dp.unit0 + upb - 1) / upb;
    const int64_t gx = blocks < kSearchGridX ? blocks : kSearchGridX;
    const int64_t gy = (blocks + gx - 1) / gx;
    hipLaunchKernelGGL(v->fn, dim3((unsigned)gx, (unsigned)gy), dim3(kWave * wpb), lds, s,
                       dp, out_ce);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// epilogue: per-curve minimum over the curve's work units
// ---------------------------------------------------------------------------
// One block per curve reads all the curve's work units (1.3 M of them per
// curve on the paper-scale grid): 1024 threads keep more loads in flight.
constexpr int kEpiBlock = 1024;

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
// FP64 confirmation of a split search's minima (gce_opts.refine_units)
// ---------------------------------------------------------------------------
// One block per curve (schedule rank): the k work units with the smallest
// (minimum CE, flat index) among the curve's units, in k rounds of a block
// minimum over the units above the previous round's choice.  A curve with
// fewer valid units than k repeats its last choice.
__global__ __launch_bounds__(kEpiBlock) void k_refine_select(DevPlan dp, int32_t k,
                                                             int64_t *list)
{
    __shared__ double sh_h[kEpiBlock / kWave];
    __shared__ int64_t sh_f[kEpiBlock / kWave];
    __shared__ int64_t sh_i[kEpiBlock / kWave];
    const int64_t rank = blockIdx.x;
    const int64_t base = rank * dp.units_per_curve;
    const Partial *pp = dp.partials + base;
    double prev_h = NAN;
    int64_t prev_f = -1, prev_i = 0;
    for (int32_t r = 0; r < k; ++r) {
        double h = NAN;
        int64_t f = -1, idx = -1;
        for (int64_t i = threadIdx.x; i < dp.units_per_curve; i += kEpiBlock) {
            const Partial v = pp[i];
            if (r > 0 && !lex_less(prev_h, prev_f, v.h, v.flat)) continue;
            if (lex_less(v.h, v.flat, h, f)) {
                h = v.h;
                f = v.flat;
                idx = i;
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double ho = __shfl_xor(h, off, kWave);
            const int64_t fo = __shfl_xor(f, off, kWave);
            const int64_t io = __shfl_xor(idx, off, kWave);
            if (lex_less(ho, fo, h, f)) {
                h = ho;
                f = fo;
                idx = io;
            }
        }
        const int w = threadIdx.x / kWave;
        if ((threadIdx.x & (kWave - 1)) == 0) {
            sh_h[w] = h;
            sh_f[w] = f;
            sh_i[w] = idx;
        }
        __syncthreads();
        h = sh_h[0];
        f = sh_f[0];
        idx = sh_i[0];
        for (int i = 1; i < kEpiBlock / kWave; ++i)
            if (lex_less(sh_h[i], sh_f[i], h, f)) {
                h = sh_h[i];
                f = sh_f[i];
                idx = sh_i[i];
            }
        __syncthreads();   // every thread has read this round's candidates
        if (f >= 0) {
            prev_h = h;
            prev_f = f;
            prev_i = idx;
        }
        if (threadIdx.x == 0) list[rank * k + r] = base + prev_i;
    }
}

hipError_t launch_refine_select(const DevPlan &dp, int32_t k, int64_t *list, hipStream_t s)
{
    hipLaunchKernelGGL(k_refine_select, dim3((unsigned)dp.n_curves), dim3(kEpiBlock), 0, s, dp,
                       k, list);
    return hipGetLastError();
}

// One thread per curve: the FP64 minimum over the curve's k confirmed units
// replaces the reported minimum; the moments stay those of the split values.
__global__ void k_refine_merge(DevPlan dp, int32_t k, const Partial *ref,
                               gce_best_t *out_best)
{
    const int64_t rank = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (rank >= dp.n_curves) return;
    const int32_t c = dp.order[rank];
    double h = NAN;
    int64_t f = -1;
    for (int32_t i = 0; i < k; ++i) {
        const Partial v = ref[rank * k + i];
        if (lex_less(v.h, v.flat, h, f)) {
            h = v.h;
            f = v.flat;
        }
    }
    gce_best_t b = out_best[c];
    if (b.flat_index < 0 || f < 0) return;   // an invalid curve stays as reported
    b.flat_index = f;
    b.period_index = (int32_t)(f % dp.n_p);
    b.pdot_index = (int32_t)(f / dp.n_p);
    b.ce_min = h;
    b.significance = b.ce_std > 0.0 ? (b.ce_mean - h) / b.ce_std : 0.0;
    out_best[c] = b;
}

hipError_t launch_refine_merge(const DevPlan &dp, int32_t k, const Partial *ref,
                               gce_best_t *out_best, hipStream_t s)
{
    constexpr int kMergeBlock = 256;
    const int64_t blocks = (dp.n_curves + kMergeBlock - 1) / kMergeBlock;
    hipLaunchKernelGGL(k_refine_merge, dim3((unsigned)blocks), dim3(kMergeBlock), 0, s, dp, k, ref,
                       out_best);
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
    const int64_t base = dp.mag_overlap ? 2 * dp.off[c] : dp.off[c];
    const int32_t *segc = dp.seg + c * (int64_t)(nmag + 1);
    for (int32_t j = 0; j < nmag; ++j) {
        for (int32_t k = segc[j]; k < segc[j + 1]; ++k) {
            const double dt = dp.dt_sorted[base + k];
            int b;
            if (dp.precision == kPrecFp64) {
                const double x = dt * invp;
                const double x2 = x * x;
                const double hpd[1] = {ha}, xs[1] = {x}, x2s[1] = {x2};
                uint32_t bb[1];
                fp64_phase_bins<1, 1>(xs, x2s, hpd, (double)nph, bb);
                b = (int)bb[0];
            } else {
                const float ip2 = dp.inv_p2f[p];
                const float d2f = dp.dt2f_sorted[base + k];
                split_round_down();
                const SplitPoint sp = split_point(dt, invp, d2f, ip2);
                const uint32_t bits = split_slot_bits(sp, ha32, (float)nph);
                // the bin leaves through an asm operand before the mode is
                // reset, so that its instructions all round down
                asm volatile("" : : "v"(bits));
                split_round_nearest();
                b = (int)(bits - kRoundMagicBits);
            }
            // a slot outside [0, n_phase) is not counted, so that the row
            // totals show it
            if (b >= 0 && b < nph) o[(int64_t)j * nph + b] += 1;
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
