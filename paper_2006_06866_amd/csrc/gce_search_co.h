// gce_search_co.h -- the search kernel with two waves per work unit: the fold
// of Eq. (3), the 2-D histogram and the entropy of Eq. (4) (Katz et al. 2020,
// Sec. 2.3), for shapes whose histograms, one per wave, would cap the waves
// a CU can hold.
//
// A block of two waves takes one work unit (64 periods x TQ Pdot trials x
// one curve, as in k_search) and keeps ONE copy of its histograms in LDS:
//   - each magnitude segment's epochs are split in two halves, one per wave;
//     both waves add into the same cells (LDS atomics), lane l of either wave
//     counting for period l;
//   - after a barrier each wave folds half of the phase bins into the entropy
//     sums; cells are cumulative (never cleared: a segment's count is the
//     cell minus its value at the previous flush), so a wave may read its
//     neighbour's cell (overlapping bins) while the other wave flushes;
//   - a second barrier keeps the next segment's adds behind the flush;
//   - at the end each wave sums its bins' marginal terms, and the two partial
//     sums of each trial meet in LDS.
// Per wave this halves the histogram LDS (the table in LDS, when used, is
// shared as before), at the cost of two barriers per magnitude segment.
#pragma once

#include "gce_device.h"

namespace gce {

constexpr int kCoWaves = 2;   // waves per work unit

template <int PREC, int NPH, int TQ, int LL, int OVL>
__global__ __launch_bounds__(kWave * kCoWaves) GCE_SEARCH_ATTR
void k_search_co(DevPlan dp, void *out_ce_v)
{
    static_assert(NPH > 1 && NPH % kCoWaves == 0,
                  "two-wave units need an even compile-time phase-bin count");
    using OutT = typename std::conditional<PREC == kPrecFp64, double, float>::type;
    constexpr int R = (TQ + 1) / 2;                    // trial pairs
    constexpr int BH = NPH / kCoWaves;                 // bins flushed per wave
    // bins per flush group: as in k_search's cumulative flush, about
    // GCE_CUM_GROUP words with one trial pair, else GCE_FLUSH_WORDS
    constexpr int G0 = R == 1 ? GCE_CUM_GROUP : (R >= GCE_FLUSH_WORDS ? 1 : GCE_FLUSH_WORDS / R);
    constexpr int G = BH < G0 ? BH : G0;
    constexpr int KA = (TQ <= 2) ? GCE_FLUSH_ACC : 1;  // partial sums per trial
    extern __shared__ uint32_t lds[];
    OutT *__restrict__ out_ce = static_cast<OutT *>(out_ce_v);

    const int lane = (int)(threadIdx.x % kWave);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // LDS: [c ln c table (LL)] [R][NPH][64] histogram words of the unit
    const size_t table_words = LL ? (size_t)2 * (dp.max_count + 1) : 0;
    double *lut_lds = reinterpret_cast<double *>(lds);
    uint32_t *hist = lds + table_words;
    uint32_t *hcol = hist + lane;
    auto cell = [&](int r, int b) -> uint32_t * { return hcol + (r * NPH + b) * kWave; };
    // this wave's phase bins: [b0, b0 + BH), and the bin after them
    const int b0 = wave * BH;
    const int bnext = (b0 + BH == NPH) ? 0 : b0 + BH;
    if (LL)
        for (int i = threadIdx.x; i <= dp.max_count; i += kWave * kCoWaves) lut_lds[i] = dp.lut[i];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < BH; ++i) *cell(r, b0 + i) = 0;
    __syncthreads();   // table and cleared cells, before any wave adds or leaves

    // one unit per block (2-D launch: a dispatch counts work-items in 32 bits)
    // (or, with a unit list, entry unit0 + ... of the list)
    const int64_t ui = dp.unit0 + (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (ui >= dp.n_units) return;   // the same for both waves
    const int64_t u = dp.unit_list ? dp.unit_list[ui] : ui;
    const int64_t rank = u / dp.units_per_curve;
    const int64_t rem = u - rank * dp.units_per_curve;
    const int32_t g = (int32_t)(rem / dp.n_ptiles);
    const int64_t tile = rem - (int64_t)g * dp.n_ptiles;
    const int32_t c = dp.order[rank];
    const int64_t base = dp.off[c] << dp.mag_overlap;
    const int64_t p = tile * kWave + lane;
    const bool p_ok = p < dp.n_p;
    const int32_t q0 = g * TQ;

    if (!(dp.curve_ok[c] && *dp.grid_ok)) {   // the same for both waves
        if (wave == 0) {
            if (out_ce && p_ok) {
#pragma unroll
                for (int t = 0; t < TQ; ++t)
                    if (q0 + t < dp.n_pd)
                        out_ce[((int64_t)c * dp.n_pd + q0 + t) * dp.n_p + p] = (OutT)NAN;
            }
            if (lane == 0) {
                dp.partials[ui] = Partial{NAN, -1};
                dp.stats[ui] = UnitStats{0.0, 0.0, 0.0};
            }
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

    const double nphd = (double)NPH;
    const float nphf = (float)NPH;
    const uint32_t split_base = (uint32_t)lane * 4u - (kRoundMagicBits << 8);
    uniform_f64 *dts = (uniform_f64 *)(dp.dt_sorted + base);
    // split path: dt^2 and (1/P)^2 in float, their product is x^2
    uniform_f32 *d2s = (uniform_f32 *)(PREC == kPrecSplit ? dp.dt2f_sorted + base : nullptr);
    const float invp2f = PREC == kPrecSplit ? dp.inv_p2f[p_ok ? p : dp.n_p - 1] : 0.0f;
    uniform_i32 *segc = (uniform_i32 *)(dp.seg + (int64_t)c * (dp.n_mag + 1));
    const double *__restrict__ lut = LL ? lut_lds : dp.lut;
    char *lbytes = reinterpret_cast<char *>(hist);
    constexpr uint32_t kUnit = LL ? 8u : 1u;   // table in LDS: counts in units of 8
    const uint32_t inc_lo = kUnit, inc_hi = kUnit << 16;

    // the fold and binning of G epochs for the lane's TQ trials (as in
    // k_search): FP64 round-down bins, or the split path's float bins
    auto fold_points = [&](const double *dt, const float *d2, auto g_tag) {
        constexpr int GE = decltype(g_tag)::value;
        if constexpr (PREC == kPrecFp64) {
            double x[GE], x2[GE];
#pragma unroll
            for (int e = 0; e < GE; ++e) {
                x[e] = dt[e] * invp;
                x2[e] = x[e] * x[e];
            }
            uint32_t b[GE * TQ];
            fp64_phase_bins<GE, TQ>(x, x2, ha, nphd, b);
#pragma unroll
            for (int e = 0; e < GE; ++e)
#pragma unroll
                for (int t = 0; t < TQ; ++t)
                    lds_add_block(hcol + ((t >> 1) * NPH + b[e * TQ + t]) * kWave,
                            (t & 1) ? inc_hi : inc_lo);
        } else {
#pragma unroll
            for (int e = 0; e < GE; ++e) {
                const SplitPoint sp = split_point(dt[e], invp, d2[e], invp2f);
#pragma unroll
                for (int t = 0; t < TQ; ++t) {
                    const uint32_t bits = split_slot_bits(sp, ha32[t], nphf);
                    const uint32_t addr = (bits << 8) + split_base +
                                          (uint32_t)((t >> 1) * NPH * kWave * 4);
                    lds_add_block(reinterpret_cast<uint32_t *>(lbytes + addr),
                            (t & 1) ? inc_hi : inc_lo);
                }
            }
        }
    };

    auto lut_lo = [&](uint32_t w) -> double {
        if constexpr (LL)
            return *reinterpret_cast<const double *>(
                reinterpret_cast<const char *>(lut) + (w & 0xffffu));
        else
            return lut[w & 0xffffu];
    };
    auto lut_hi = [&](uint32_t w) -> double {
        if constexpr (LL)
            return *reinterpret_cast<const double *>(
                reinterpret_cast<const char *>(lut) + (w >> 16));
        else
            return lut[w >> 16];
    };

    // the table entry at byte offset o, read through its LDS address (the
    // table opens the kernel's dynamic LDS at address 0, which the host
    // checks before launching a variant with the table in LDS)
    auto lut_at = [&](uint32_t o) -> double {
        return *reinterpret_cast<const __attribute__((address_space(3))) double *>(
            static_cast<size_t>(o));
    };

    // cumulative cells: the previous flush's values of this wave's bins, and
    // of the bin after them (overlapping bins read it as a neighbour)
    uint32_t vprev[R][BH], vnext[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        vnext[r] = 0;
#pragma unroll
        for (int i = 0; i < BH; ++i) vprev[r][i] = 0;
    }
    double s1[KA][TQ], s2[KA][TQ];
#pragma unroll
    for (int a = 0; a < KA; ++a)
#pragma unroll
        for (int t = 0; t < TQ; ++t) s1[a][t] = s2[a][t] = 0.0;

    auto seg_word = [&](int r, int i) -> uint32_t {   // this wave's bin b0 + i
        const uint32_t cv = *cell(r, b0 + i);
        const uint32_t w = cv - vprev[r][i];
        vprev[r][i] = cv;
        return w;
    };
    auto next_word = [&](int r) -> uint32_t {          // the bin after them
        const uint32_t cv = *cell(r, bnext);
        const uint32_t w = cv - vnext[r];
        vnext[r] = cv;
        return w;
    };
    // Eq. (4) terms of this wave's bins for one segment (or, at the end, of
    // the marginals): words in groups of G bins, all cell reads, then all
    // table loads, then the adds, as in k_search's cumulative flush
    auto flush_bins = [&](auto word_of, auto next_of, double (&acc)[KA][TQ]) {
        uint32_t cur[R];
#pragma unroll
        for (int r = 0; r < R; ++r) cur[r] = word_of(r, 0);
#pragma unroll
        for (int i0 = 0; i0 < BH; i0 += G) {
            uint32_t wv[G + 1][R];
#pragma unroll
            for (int r = 0; r < R; ++r) wv[0][r] = cur[r];
#pragma unroll
            for (int i = 1; i <= G; ++i)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int idx = i0 + i;
                    wv[i][r] = idx < BH ? word_of(r, idx) : (OVL && idx == BH) ? next_of(r) : 0u;
                }
            asm volatile("" ::: "memory");
            double lo[G][R], hi[G][R];
#pragma unroll
            for (int i = 0; i < G; ++i)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    lo[i][r] = hi[i][r] = 0.0;
                    if (i0 + i >= BH) continue;
                    if constexpr (OVL && LL && PREC == kPrecFp64) {
                        const uint32_t a = wv[i][r], nbr = wv[i + 1][r];
                        lo[i][r] = lut_at(add_low_halves(a, nbr));
                        hi[i][r] = (2 * r + 1 < TQ) ? lut_at(add_high_halves(a, nbr)) : 0.0;
                    } else {
                        const uint32_t w = OVL ? wv[i][r] + wv[i + 1][r] : wv[i][r];
                        lo[i][r] = lut_lo(w);
                        hi[i][r] = (2 * r + 1 < TQ) ? lut_hi(w) : 0.0;
                    }
                }
            asm volatile("" ::: "memory");
#pragma unroll
            for (int i = 0; i < G; ++i)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (i0 + i >= BH) continue;
                    acc[(i0 + i) % KA][2 * r] += lo[i][r];
                    if (2 * r + 1 < TQ) acc[(i0 + i) % KA][2 * r + 1] += hi[i][r];
                }
#pragma unroll
            for (int r = 0; r < R; ++r) cur[r] = wv[G][r];
        }
    };

    if constexpr (PREC == kPrecSplit) split_round_down();
    for (int32_t j = 0; j < dp.n_mag; ++j) {
        const int32_t k0 = segc[j], k1 = segc[j + 1];
        if (k0 == k1) continue;   // the same for both waves
        // this wave's half of the segment's epochs
        const int32_t half = (k1 - k0 + 1) >> 1;
        const int32_t ka = wave ? k0 + half : k0;
        const int32_t kb = wave ? k1 : k0 + half;
        constexpr int U = (TQ >= 8) ? GCE_UNROLL_LARGE_TQ : GCE_UNROLL_SMALL_TQ;
        constexpr int GF0 = GCE_RD_GROUP / TQ < 1 ? 1 : GCE_RD_GROUP / TQ;
        constexpr int GF = GF0 < U ? GF0 : U;
        int32_t k = ka;
        if (k + U <= kb) {
            double cur[U];
            float cur2[U];
#pragma unroll
            for (int uu = 0; uu < U; ++uu) {
                cur[uu] = dts[k + uu];
                if constexpr (PREC == kPrecSplit) cur2[uu] = d2s[k + uu];
            }
            while (true) {
                const int32_t kn = k + U;
                const bool more = kn + U <= kb;
#pragma unroll
                for (int uu = 0; uu < U; uu += GF)
                    fold_points(&cur[uu], &cur2[uu], std::integral_constant<int, GF>{});
                k = kn;
                if (!more) break;
#pragma unroll
                for (int uu = 0; uu < U; ++uu) {
                    cur[uu] = dts[k + uu];
                    if constexpr (PREC == kPrecSplit) cur2[uu] = d2s[k + uu];
                }
            }
        }
        for (; k < kb; ++k) {
            const double d1[1] = {dts[k]};
            float e1[1] = {0.0f};
            if constexpr (PREC == kPrecSplit) e1[0] = d2s[k];
            fold_points(d1, e1, std::integral_constant<int, 1>{});
        }
        __syncthreads();   // the segment's adds of both waves are in
        flush_bins(seg_word, next_word, s1);
        __syncthreads();   // its cells read before the next segment's adds
    }
    if constexpr (PREC == kPrecSplit) split_round_nearest();

    // marginal terms of this wave's bins: the cells now hold the marginals
    auto marg_word = [&](int r, int i) -> uint32_t { return *cell(r, b0 + i); };
    auto marg_next = [&](int r) -> uint32_t { return *cell(r, bnext); };
    flush_bins(marg_word, marg_next, s2);

    // the two waves' partial sums of each trial meet in LDS (the histogram
    // words are free once both waves have read them)
    double part[TQ];
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
        double a2 = s2[0][t], a1 = s1[0][t];
#pragma unroll
        for (int a = 1; a < KA; ++a) {
            a2 += s2[a][t];
            a1 += s1[a][t];
        }
        part[t] = a2 - a1;
    }
    double *xch = reinterpret_cast<double *>(hist);   // [TQ][64]
    static_assert(2 * TQ <= R * NPH, "exchange fits in the histogram words");
    __syncthreads();
    if (wave == 1) {
#pragma unroll
        for (int t = 0; t < TQ; ++t) xch[t * kWave + lane] = part[t];
    }
    __syncthreads();
    if (wave == 1) return;
#pragma unroll
    for (int t = 0; t < TQ; ++t) part[t] += xch[t * kWave + lane];

    const double entries = (double)segc[dp.n_mag];
    const double nd = OVL ? 2.0 * entries : entries;
    double best_h = NAN;
    int64_t best_f = -1;
    double hv[TQ];
    double lsum = 0.0, lcnt = 0.0;
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
        const OutT h = (OutT)(part[t] / nd);
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
        dp.partials[ui] = Partial{best_h, best_f};
        dp.stats[ui] = UnitStats{wcnt, wmean, wm2};
    }
}

}  // namespace gce
