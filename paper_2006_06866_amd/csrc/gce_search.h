// gce_search.h -- the search kernel template: the fold of Eq. (3), the
// per-lane phase histograms and the entropy of Eq. (4) (Katz et al. 2020,
// Sec. 2.3).  Instantiated by the gce_search_*.hip files, one per precision
// and phase-bin kind, so the variants compile in parallel.
//
// Search-kernel layout (one wave = one work unit; a block holds one wave, or
// two sharing an LDS copy of the c ln c table; k_search_co in
// gce_search_co.h runs one unit on two waves instead):
//   lane l          <-> period index p = 64 * tile + l
//   trial t < TQ    <-> Pdot index q = TQ * group + t (same for the wave)
//   epoch k         <-> uniform across the wave: dt_k is read with scalar
//                       loads and enters the VALU as an SGPR operand.
// Epochs are pre-grouped by magnitude bin, so each lane only keeps a 1-D
// phase histogram per trial (the paper's Sec. 2.3 GPU observation that one
// magnitude value's phase counts suffice); at the end of each magnitude
// segment the histogram is folded into the entropy sums (and cleared, or,
// with the table in LDS, left to accumulate).  Histograms live in LDS as
// [trial pair][phase bin][lane] 32-bit words: the low and high 16 bits count
// trials 2r and 2r+1, so one ds_add_u32 bins one point-trial, and lanes
// always hit distinct banks.  The marginal phase counts accumulate in
// registers.  The FP64 bin is one round-down fma (fp64_phase_bins).
//
// Entropy: N * H = sum_b c_b ln c_b - sum_{j,b} c_jb ln c_jb, which equals
// Eq. (4) multiplied by N; c ln c comes from a table built on the device.
#pragma once

#include "gce_device.h"
#include "gce_search_co.h"

namespace gce {

// NPH > 0: phase-bin count fixed at compile time, marginals in VGPRs.
// NPH = 0: runtime phase-bin count, marginals in LDS behind the histograms.
template <int PREC, int NPH, int TQ>
struct SearchShape {
    static constexpr int kRegions = (TQ + 1) / 2;
    static constexpr bool kLdsMarg = (NPH == 0);
    // phase bins per scheduling group of the segment flush: about
    // GCE_FLUSH_WORDS words, i.e. twice that many table loads, in flight
    static constexpr int kFlushGroup =
        kRegions >= GCE_FLUSH_WORDS ? 1 : GCE_FLUSH_WORDS / kRegions;
    // the same for the cumulative flush (table in LDS): 12 bins with one
    // trial pair (24 table loads), else as above (more cost registers)
    static constexpr int kCumGroup = kRegions == 1 ? GCE_CUM_GROUP : kFlushGroup;
};

// LL = 1: the c ln c table is copied into LDS, shared by the block's
// search_waves_per_block(1) waves (for shapes with many cells per epoch,
// where the segment flush dominates).
// OVL = 1: 50%-overlapping phase bins (each epoch counts in two bins).
template <int PREC, int NPH, int TQ, int LL, int OVL>
__global__ __launch_bounds__(kWave * (LL ? kLutWaves : 1)) GCE_SEARCH_ATTR
void k_search(DevPlan dp, void *out_ce_v)
{
    using S = SearchShape<PREC, NPH, TQ>;
    using OutT = typename std::conditional<PREC == kPrecFp64, double, float>::type;
    constexpr int R = S::kRegions;
    constexpr int WPB = LL ? kLutWaves : 1;             // waves per block
    extern __shared__ uint32_t lds[];
    OutT *__restrict__ out_ce = static_cast<OutT *>(out_ce_v);

    const int lane = WPB > 1 ? (int)(threadIdx.x % kWave) : (int)threadIdx.x;
    // the wave's index in the block is uniform across its lanes: say so, so
    // that everything derived from the work unit stays in scalar registers
    const int wave = WPB > 1 ? __builtin_amdgcn_readfirstlane(threadIdx.x / kWave) : 0;
    const int nph = NPH > 0 ? NPH : dp.n_phase;
    const int nslot = nph;                              // LDS words per region
    // LDS: [c ln c table (LL)] then one region per wave:
    // [R][nslot][64] histogram words, then [R][nph][64] marginals (NPH == 0)
    const size_t table_words = LL ? (size_t)2 * (dp.max_count + 1) : 0;
    const size_t wave_words = (size_t)R * (nslot + (S::kLdsMarg ? nph : 0)) * kWave;
    double *lut_lds = reinterpret_cast<double *>(lds);
    if (LL) {   // before any wave of the block may leave
        for (int c = threadIdx.x; c <= dp.max_count; c += kWave * WPB) lut_lds[c] = dp.lut[c];
        __syncthreads();
    }
    // 2-D launch (a dispatch's grid size counts work-items in 32 bits):
    // unit = unit0 + (y * gridDim.x + x) * WPB + wave, in dispatch order
    // (or, with a unit list, entry unit0 + ... of the list)
    const int64_t ui = dp.unit0 + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * WPB + wave;
    if (ui >= dp.n_units) return;
    const int64_t u = dp.unit_list ? dp.unit_list[ui] : ui;
    const int64_t rank = u / dp.units_per_curve;
    const int64_t rem = u - rank * dp.units_per_curve;
    const int32_t g = (int32_t)(rem / dp.n_ptiles);
    const int64_t tile = rem - (int64_t)g * dp.n_ptiles;
    const int32_t c = dp.order[rank];
    // the curve's sorted epochs start at off[c], or 2 off[c] with overlapping
    // magnitude bins (mag_overlap is 0 or 1; a shift keeps this scalar, where
    // a select cost 18 VGPRs in the 10-bin, 4-trial kernel)
    const int64_t base = dp.off[c] << dp.mag_overlap;
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
            dp.partials[ui] = Partial{NAN, -1};
            dp.stats[ui] = UnitStats{0.0, 0.0, 0.0};
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

    uint32_t *hist = lds + table_words + wave * wave_words;  // [R][nslot][64]
    uint32_t *lmarg = hist + (size_t)R * nslot * kWave;      // [R][nph][64] (NPH == 0)
    for (int i = 0; i < R * nslot; ++i) hist[i * kWave + lane] = 0;
    if (S::kLdsMarg)
        for (int i = 0; i < R * nph; ++i) lmarg[i * kWave + lane] = 0;
    uint32_t vmarg[R][NPH > 0 ? NPH : 1];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int b = 0; b < (NPH > 0 ? NPH : 1); ++b) vmarg[r][b] = 0;

    // conditional-entropy sums: KA partial sums per trial (independent
    // add chains in the segment flush when there are few trials per lane)
    constexpr int KA = (TQ <= 2) ? GCE_FLUSH_ACC : 1;
    double s1[KA][TQ];
#pragma unroll
    for (int a = 0; a < KA; ++a)
#pragma unroll
        for (int t = 0; t < TQ; ++t) s1[a][t] = 0.0;

    const double nphd = (double)nph;
    const float nphf = (float)nph;
    // split path: (bits << 8) of slot s is 0x40000000 + 256 s (mod 2^32)
    const uint32_t split_base = (uint32_t)lane * 4u - (kRoundMagicBits << 8);
    uniform_f64 *dts = (uniform_f64 *)(dp.dt_sorted + base);
    // split path: dt^2 and (1/P)^2 in float, their product is x^2
    uniform_f32 *d2s = (uniform_f32 *)(PREC == kPrecSplit ? dp.dt2f_sorted + base : nullptr);
    const float invp2f = PREC == kPrecSplit ? dp.inv_p2f[p_ok ? p : dp.n_p - 1] : 0.0f;
    uniform_i32 *segc = (uniform_i32 *)(dp.seg + (int64_t)c * (dp.n_mag + 1));
    const double *__restrict__ lut = LL ? lut_lds : dp.lut;
    uint32_t *hcol = hist + lane;
    char *lbytes = reinterpret_cast<char *>(hist);     // this wave's histogram words

    // With the table in LDS (LL), counts are kept in units of 8 (at most
    // 8 * 8191 per 16-bit half), so a half is directly the byte offset of
    // its c ln c entry: no shift before each table load.
    constexpr uint32_t kUnit = LL ? 8u : 1u;
    const uint32_t inc_lo = kUnit, inc_hi = kUnit << 16;
    // G epochs at a time: on the FP64 path their G * TQ round-down fmas
    // share one rounding-mode switch
    auto fold_points = [&](const double *dt, const float *d2, auto g_tag) {
        constexpr int G = decltype(g_tag)::value;
        if constexpr (PREC == kPrecFp64) {
            double x[G], x2[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                x[g] = dt[g] * invp;
                x2[g] = x[g] * x[g];
            }
            uint32_t b[G * TQ];
            fp64_phase_bins<G, TQ>(x, x2, ha, nphd, b);
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int t = 0; t < TQ; ++t)
                    lds_add(hcol + ((t >> 1) * nslot + b[g * TQ + t]) * kWave,
                            (t & 1) ? inc_hi : inc_lo);
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const SplitPoint sp = split_point(dt[g], invp, d2[g], invp2f);
#pragma unroll
                for (int t = 0; t < TQ; ++t) {
                    const uint32_t bits = split_slot_bits(sp, ha32[t], nphf);
                    const uint32_t addr = (bits << 8) + split_base +
                                          (uint32_t)((t >> 1) * nslot * kWave * 4);
                    lds_add(reinterpret_cast<uint32_t *>(lbytes + addr),
                            (t & 1) ? inc_hi : inc_lo);
                }
            }
        }
    };

    // c ln c of the two counts packed in a word
    auto lut_lo = [&](uint32_t w) -> double {
        if constexpr (LL)
            return *reinterpret_cast<const double *>(
                reinterpret_cast<const char *>(lut) + (w & 0xffffu));
        else
            return lut[w & 0xffffu];
    };
    // the table entry at byte offset o (table in LDS: counts in units of 8).
    // The FP64 kernels read the LDS copy through its LDS address, which is o
    // itself: the table opens the kernel's dynamic LDS, which starts at LDS
    // address 0 because the search kernels have no static LDS (the host
    // checks that before launching a variant with the table in LDS).
    // Addressing it off the array's symbol instead costs an add of that
    // (link-time) address per table load.  Measured on 32 curves of the
    // 50 x 10 overlapping-bin workload: FP64 search 896 -> 863 ms, split
    // 867 -> 882 ms (same register count), so the split kernels keep the
    // symbol-relative form.
    auto lut_at = [&](uint32_t o) -> double {
        if constexpr (LL && PREC == kPrecFp64)
            return *reinterpret_cast<const __attribute__((address_space(3))) double *>(
                static_cast<size_t>(o));
        else
            return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(lut) + o);
    };
    auto lut_hi = [&](uint32_t w) -> double {
        if constexpr (LL)
            return *reinterpret_cast<const double *>(
                reinterpret_cast<const char *>(lut) + (w >> 16));
        else
            return lut[w >> 16];
    };

    // end of a magnitude segment: sum c ln c, add to marginals, clear
    auto cell = [&](int r, int b) -> uint32_t * { return hcol + (r * nslot + b) * kWave; };
    auto add_lut = [&](int r, uint32_t w, int a) {
        s1[a][2 * r] += lut_lo(w);
        if (2 * r + 1 < TQ) s1[a][2 * r + 1] += lut_hi(w);
    };
    // One pass over the phase bins.  With 50%-overlapping bins, bin b
    // spans disjoint bins b and b + 1 (mod n): its count is the sum of the
    // two words (packed halves cannot overflow: together they hold at most
    // the segment's entries, or twice that for a single phase bin, within
    // the plan's count bound).  Bin 0's word is kept in a
    // register for the last bin, so every cell is cleared as soon as it is
    // read.
    // With the table in LDS (and NPH > 0) cells are never cleared.  They hold
    // counts accumulated over the segments so far; vmarg holds the same at
    // the previous flush, so a segment's count is their difference (packed
    // halves never borrow: each half only grows), and at the end the cells
    // are the marginal counts.  One LDS write per cell and segment fewer;
    // measured faster only where the flush dominates (2.4% on 50 x 10
    // overlapping bins at N = 500, 3% slower on 10 x 5 bins at N = 600).
    constexpr bool kCum = NPH > 0 && LL;
    auto seg_word = [&](int r, int b) -> uint32_t {
        const uint32_t c = *cell(r, b);
        const uint32_t w = c - vmarg[r][b];
        vmarg[r][b] = c;
        return w;
    };
    auto flush_segment = [&]() {
        if constexpr (kCum) {
            // groups of G bins in three phases kept apart by compiler
            // barriers: all cell reads, then all table loads, then the
            // adds, so a group's table loads are in flight together (the
            // compiler's own schedule kept 3 or 4; 2.5% faster on 50 x 10
            // overlapping bins at N = 500)
            constexpr int G = S::kCumGroup;
            uint32_t w0[R], cur[R];
#pragma unroll
            for (int r = 0; r < R; ++r) cur[r] = w0[r] = seg_word(r, 0);
#pragma unroll
            for (int b0 = 0; b0 < NPH; b0 += G) {
                uint32_t wv[G + 1][R];
#pragma unroll
                for (int r = 0; r < R; ++r) wv[0][r] = cur[r];
#pragma unroll
                for (int i = 1; i <= G; ++i)
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        wv[i][r] = (b0 + i < NPH) ? seg_word(r, b0 + i)
                                                  : (b0 + i == NPH ? w0[r] : 0u);
                asm volatile("" ::: "memory");
                double lo[G][R], hi[G][R];
#pragma unroll
                for (int i = 0; i < G; ++i)
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if (b0 + i >= NPH) continue;
                        if constexpr (OVL && PREC == kPrecFp64) {
                            // the two halves summed apart, one instruction
                            // each: the low and high trial's table offsets
                            const uint32_t a = wv[i][r], nb = wv[i + 1][r];
                            lo[i][r] = lut_at(add_low_halves(a, nb));
                            hi[i][r] = (2 * r + 1 < TQ) ? lut_at(add_high_halves(a, nb)) : 0.0;
                        } else {
                            // the packed sum (halves cannot carry: together
                            // they hold at most the plan's count bound)
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
                        if (b0 + i >= NPH) continue;
                        s1[(b0 + i) % KA][2 * r] += lo[i][r];
                        if (2 * r + 1 < TQ) s1[(b0 + i) % KA][2 * r + 1] += hi[i][r];
                    }
#pragma unroll
                for (int r = 0; r < R; ++r) cur[r] = wv[G][r];
            }
            return;
        }
        uint32_t w0[R];
#pragma unroll
        for (int r = 0; r < R; ++r) w0[r] = *cell(r, 0);
        if constexpr (NPH > 0) {
#pragma unroll
            for (int b = 0; b < NPH; ++b) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t w = (b == 0) ? w0[r] : *cell(r, b);
                    uint32_t wo = w;
                    if constexpr (OVL) wo += (b + 1 < NPH) ? *cell(r, b + 1) : w0[r];
                    *cell(r, b) = 0;
                    vmarg[r][b] += w;
                    add_lut(r, wo, b % KA);
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
                    uint32_t wo = w;
                    if constexpr (OVL) wo += (b + 1 < nph) ? *cell(r, b + 1) : w0[r];
                    *cell(r, b) = 0;
                    lmarg[(r * nph + b) * kWave + lane] += w;
                    add_lut(r, wo, 0);
                }
            }
        }
    };

    // split path: FP32 rounds toward minus infinity while the epochs are
    // binned (the bin fma floors n * phase), and to nearest again after
    if constexpr (PREC == kPrecSplit) split_round_down();
    for (int32_t j = 0; j < dp.n_mag; ++j) {
        const int32_t k0 = segc[j], k1 = segc[j + 1];
        if (k0 == k1) continue;
        // U epochs per iteration; optionally the next U epoch offsets are
        // loaded while the current ones are binned.
        constexpr int U = (TQ >= 8) ? GCE_UNROLL_LARGE_TQ : GCE_UNROLL_SMALL_TQ;
        // epochs per rounding-mode switch: up to GCE_RD_GROUP fmas, dividing U
        constexpr int GF0 = GCE_RD_GROUP / TQ < 1 ? 1 : GCE_RD_GROUP / TQ;
        constexpr int GF = GF0 < U ? GF0 : U;
        static_assert(U % GF == 0, "epoch groups must divide the unroll");
        int32_t k = k0;
        if (k + U <= k1) {
            double cur[U], nxt[U];
            float cur2[U], nxt2[U];
#pragma unroll
            for (int uu = 0; uu < U; ++uu) {
                cur[uu] = dts[k + uu];
                if constexpr (PREC == kPrecSplit) cur2[uu] = d2s[k + uu];
            }
            while (true) {
                const int32_t kn = k + U;
                const bool more = kn + U <= k1;
                if (GCE_PREFETCH && more) {
#pragma unroll
                    for (int uu = 0; uu < U; ++uu) {
                        nxt[uu] = dts[kn + uu];
                        if constexpr (PREC == kPrecSplit) nxt2[uu] = d2s[kn + uu];
                    }
                }
#pragma unroll
                for (int uu = 0; uu < U; uu += GF)
                    fold_points(&cur[uu], &cur2[uu], std::integral_constant<int, GF>{});
                k = kn;
                if (!more) break;
#pragma unroll
                for (int uu = 0; uu < U; ++uu) {
                    cur[uu] = GCE_PREFETCH ? nxt[uu] : dts[k + uu];
                    if constexpr (PREC == kPrecSplit)
                        cur2[uu] = GCE_PREFETCH ? nxt2[uu] : d2s[k + uu];
                }
            }
        }
        for (; k < k1; ++k) {
            const double d1[1] = {dts[k]};
            float e1[1] = {0.0f};
            if constexpr (PREC == kPrecSplit) e1[0] = d2s[k];
            fold_points(d1, e1, std::integral_constant<int, 1>{});
        }

        flush_segment();
    }
    if constexpr (PREC == kPrecSplit) split_round_nearest();

    double s2[TQ];
#pragma unroll
    for (int t = 0; t < TQ; ++t) s2[t] = 0.0;
    auto marg_word = [&](int r, uint32_t w) {
        s2[2 * r] += lut_lo(w);
        if (2 * r + 1 < TQ) s2[2 * r + 1] += lut_hi(w);
    };
    constexpr uint32_t nb_mask = OVL ? 0xffffffffu : 0u;
    if constexpr (NPH > 0) {
        if constexpr (!kCum) {
            // the histograms are empty now: park the register marginals there
#pragma unroll
            for (int b = 0; b < NPH; ++b)
#pragma unroll
                for (int r = 0; r < R; ++r) hcol[(r * nslot + b) * kWave] = vmarg[r][b];
        }
        // summed in a rolled loop (an unrolled one keeps every table load
        // in flight at once)
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

    // probabilities are counts over the histogram total: the curve's
    // entries (N, or up to 2N with overlapping magnitude bins), twice that
    // with overlapping phase bins
    const double entries = (double)segc[dp.n_mag];
    const double nd = OVL ? 2.0 * entries : entries;
    double best_h = NAN;
    int64_t best_f = -1;
    double hv[TQ];
    double lsum = 0.0, lcnt = 0.0;
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
        double s1t = s1[0][t];
#pragma unroll
        for (int a = 1; a < KA; ++a) s1t += s1[a][t];
        const OutT h = (OutT)((s2[t] - s1t) / nd);
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
        dp.partials[ui] = Partial{best_h, best_f};
        dp.stats[ui] = UnitStats{wcnt, wmean, wm2};
    }
}

// Table of the variants of one precision and phase-bin kind: every
// compiled phase-bin count (0 = any count), trials per lane and table
// placement.  Expanded once in each gce_search_*.hip file.
#define GCE_SV(P, O, N, T)                                                      \
    SearchVariant{N, T, 0, 1, &k_search<P, N, T, 0, O>},                        \
        SearchVariant{N, T, 1, 1, &k_search<P, N, T, 1, O>}
// the same shape also with two waves per work unit
#define GCE_SV2(P, O, N, T)                                                     \
    GCE_SV(P, O, N, T), SearchVariant{N, T, 0, 2, &k_search_co<P, N, T, 0, O>}, \
        SearchVariant{N, T, 1, 2, &k_search_co<P, N, T, 1, O>}
#define GCE_SEARCH_TABLE(P, O, FN)                                              \
    namespace gce {                                                             \
    static const SearchVariant kSearchTable[] = {                               \
        GCE_SV(P, O, 10, 1), GCE_SV(P, O, 10, 2), GCE_SV2(P, O, 10, 4),         \
        GCE_SV2(P, O, 10, 8), GCE_SV(P, O, 15, 1), GCE_SV(P, O, 15, 2),         \
        GCE_SV(P, O, 15, 4), GCE_SV(P, O, 15, 8), GCE_SV(P, O, 20, 1),          \
        GCE_SV2(P, O, 20, 2), GCE_SV2(P, O, 20, 4), GCE_SV2(P, O, 20, 8),       \
        GCE_SV2(P, O, 50, 1), GCE_SV2(P, O, 50, 2), GCE_SV2(P, O, 50, 4),       \
        GCE_SV(P, O, 0, 1),  GCE_SV(P, O, 0, 2),  GCE_SV(P, O, 0, 4),           \
        GCE_SV(P, O, 0, 8)};                                                    \
    SearchTable FN()                                                            \
    {                                                                           \
        return SearchTable{kSearchTable,                                        \
                           (int32_t)(sizeof(kSearchTable) / sizeof(kSearchTable[0]))}; \
    }                                                                           \
    }

}  // namespace gce
