// gce_internal.h -- shapes, workspace views and kernel launchers shared by
// the host API (gce_api.cpp) and the HIP kernels (gce_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "gce.h"

namespace gce {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kMaxPoints = 65535;    // 16-bit histogram counters
constexpr int kMaxMagBins = 255;
constexpr int kMaxRefineUnits = 64;  // work units per curve of an FP64 confirmation
constexpr int kMaxPhaseBins = 128;   // LDS budget of the generic kernel
constexpr double kMaxSpanDays = 1e12;
constexpr double kMinPeriod = 1e-12;
constexpr double kMaxPeriod = 1e12;
constexpr double kMaxAbsPdot = 1.0;
// The split path forms x^2 = (t - t0)^2 (1/P)^2 in FP32: its plans keep x
// below 1e16 cycles (x^2 < 1e32, (t - t0)^2 <= 1e20 and (1/P)^2 <= 1e12, far
// inside the float range) by accepting periods of at least 1e-6 days and
// curves spanning at most 1e10 days.
constexpr double kSplitMinPeriod = 1e-6;
constexpr double kSplitMaxSpanDays = 1e10;
// Largest count with the c ln c table in LDS: counts are kept in units of 8
// in 16-bit halves.
constexpr int32_t kMaxLdsTableCount = 8191;
constexpr size_t kMaxLdsBytes = 64 * 1024;   // LDS of one search block
// Search launches are 2-D: at most this many one-wave blocks along x (the
// dispatch grid size counts work-items in 32 bits), up to 65,535 rows.
constexpr int64_t kSearchGridX = 65536;
constexpr int64_t kMaxUnits = kSearchGridX * 65535;

// Minimum of one work unit: smallest H_c and its flat index (-1: none).
struct Partial {
    double h;
    int64_t flat;
};

// Moments of one work unit's CE values: count, mean, sum of squared
// deviations from the mean (merged per curve for Eq. (5)).
struct UnitStats {
    double n;
    double mean;
    double m2;
};

// Everything a kernel needs: the shape, the schedule and views into the
// plan's device workspace.  Passed to kernels by value.
struct DevPlan {
    int64_t n_curves;
    int64_t n_p;
    int64_t n_pd;
    int32_t n_phase;
    int32_t n_mag;
    int32_t tq;               // Pdot trials per lane
    int32_t n_qgroups;        // ceil(n_pd / tq)
    int64_t n_ptiles;         // ceil(n_p / 64)
    int64_t units_per_curve;  // n_qgroups * n_ptiles
    int64_t n_units;          // n_curves * units_per_curve; for one search
                              // launch: the end of its unit range
    int64_t unit0;            // first work unit of a search launch (0 unless
                              // the batch is searched in two launches)
    const int64_t *unit_list; // null, or the work units a search launch takes
                              // (entries unit0 .. n_units - 1 of the list;
                              // unit i's minimum and moments go to
                              // partials[i], stats[i])
    int32_t max_count;        // largest count of a histogram cell, a marginal
                              // or a pair of phase slots: the longest curve,
                              // doubled with overlapping magnitude bins and
                              // again for one overlapping phase bin
    int32_t precision;
    int32_t overlap;          // 50%-overlapping phase bins
    int32_t mag_overlap;      // 50%-overlapping magnitude bins: each curve's
                              // sorted-epoch region has room for 2N entries
    int32_t lut_lds;          // c ln c table copied into LDS by each wave
    int32_t co;               // waves per work unit: 1, or 2 sharing one
                              // copy of the unit's histograms

    // plan-time metadata
    const int64_t *off;       // [n_curves + 1] curve offsets
    const int32_t *order;     // [n_curves] schedule rank -> curve
    const double *lut;        // [max_count + 1] c * ln(c)

    // per-execution scratch
    double *dt_sorted;        // [total] t - t0, grouped by magnitude bin; curve
                              // c at off[c] (2 off[c] with mag_overlap)
    float *dt2f_sorted;       // [total] (t - t0)^2 rounded to float, same order
                              // (split path only; null for FP64 plans)
    int32_t *seg;             // [n_curves][n_mag + 1] segment starts
    int32_t *curve_ok;        // [n_curves]
    int32_t *grid_ok;         // [1]
    double *inv_p;            // [n_p] 1 / P
    float *inv_p2f;           // [n_p] (1 / P)^2 rounded to float (split path
                              // only; null for FP64 plans)
    double *half_pd;          // [n_pd] Pdot / 2
    float *half_pd32;         // [n_pd] Pdot / 2 rounded to float (split path)
    Partial *partials;        // [n_units]
    UnitStats *stats;         // [n_units]
};

// Kernel launchers (gce_kernels.hip).  Each returns the launch status.
hipError_t launch_lut(const DevPlan &dp, hipStream_t s);
hipError_t launch_grid_setup(const DevPlan &dp, const double *periods,
                             const double *pdots, hipStream_t s);
hipError_t launch_prepass(const DevPlan &dp, const double *times,
                          const double *mags, hipStream_t s);
hipError_t launch_search(const DevPlan &dp, void *out_ce, hipStream_t s);
hipError_t launch_epilogue(const DevPlan &dp, gce_best_t *out_best,
                           hipStream_t s);
// FP64 confirmation of a split search's minima: per curve the k work units
// with the smallest split minima (into `list`, k per curve in schedule
// order), then, after the FP64 search over them has written `ref` (k
// partials per curve), each curve's FP64 minimum over those units into
// out_best (gce_opts.refine_units).
hipError_t launch_refine_select(const DevPlan &dp, int32_t k, int64_t *list, hipStream_t s);
hipError_t launch_refine_merge(const DevPlan &dp, int32_t k, const Partial *ref,
                               gce_best_t *out_best, hipStream_t s);
hipError_t launch_debug_counts(const DevPlan &dp, const int64_t *trial_curve,
                               const int64_t *trial_flat, int64_t n_trials,
                               uint32_t *out_counts, hipStream_t s);

// Search-kernel variants of one precision and phase-bin kind, each table
// compiled in its own translation unit (gce_search_*.hip).
using SearchFn = void (*)(DevPlan, void *);
struct SearchVariant {
    int32_t nph;   // phase bins fixed at compile time; 0 = any count
    int32_t tq;    // Pdot trials per lane
    int32_t ll;    // c ln c table in LDS
    int32_t co;    // waves per work unit (2: one histogram shared by both)
    SearchFn fn;
};
struct SearchTable {
    const SearchVariant *v;
    int32_t n;
};
SearchTable search_table_fp64();
SearchTable search_table_fp64_overlap();
SearchTable search_table_split();
SearchTable search_table_split_overlap();

// Search-kernel variants compiled into the library.
bool search_variant_exists(int precision, int n_phase, int tq, int co = 1);
// Whether the table-in-LDS variant of a shape can run (its kernel has no
// static LDS, so the table it copies opens LDS at address 0).  Checked at
// plan creation, which also keeps the answer for later launches (so a
// captured launch makes no HIP query).
bool search_table_in_lds_ok(int precision, int overlap, int n_phase, int tq, int co = 1);
// Waves per search block: the waves of a block share the LDS copy of the
// c ln c table; with two waves per work unit (co = 2) they also share the
// unit's histograms.
constexpr int kLutWaves = 2;
inline int search_waves_per_block(int lut_lds, int co = 1)
{
    return co == 2 ? 2 : lut_lds ? kLutWaves : 1;
}
// Bytes of LDS one search block uses (lut_lds: the c ln c table of
// max_count + 1 entries is kept in LDS too, once per block).
size_t search_lds_bytes(int precision, int n_phase, int tq, int lut_lds, int max_count,
                        int co = 1);
// Fill dp.order[rank] = rank (the identity schedule) on `s`.
hipError_t launch_iota_order(const DevPlan &dp, hipStream_t s);

// ---------------------------------------------------------------------------
// host-side plan construction (gce_api.cpp), shared by the entry points
// ---------------------------------------------------------------------------
// Byte offsets of the parts of a plan's device workspace (one block).
struct WorkspaceLayout {
    size_t off, order, lut, dt, dt2f, seg, curve_ok, grid_ok, inv_p, inv_p2f, half_pd,
        half_pd32, partials, stats, refine_list, refine_partials, refine_stats, total;
};

// Record `msg` as the calling thread's last error text; returns `code`.
int set_error(int code, const char *msg);
// GCE_OK if `dev` is a gfx950 device, else GCE_ENODEV (with the reason).
int check_device(int dev);
// Host checks of a shape: offsets, counts, bin counts, grid sizes.  On
// success *max_n receives the longest curve's length.
int validate_shape(const int64_t *off, int64_t n_curves, int64_t n_p, int64_t n_pd,
                   int32_t n_phase, int32_t n_mag, int32_t *max_n);
// Largest count of a histogram cell, a marginal or a pair of phase slots.
int count_bound(int32_t max_n, int32_t n_phase, int32_t phase_overlap, int32_t mag_overlap,
                int32_t *max_count);
// Waves per work unit chosen by the measured heuristic (1 or 2).
int heuristic_co(int precision, int n_phase, int tq, int lut_lds, int32_t max_count);
// Pdot trials per lane chosen by the measured heuristic; waves_per_unit is
// the requested count (0 automatic).
int heuristic_tq(int precision, int n_phase, int64_t n_pd, int32_t max_count,
                 int waves_per_unit = 0);
// Whether a tiling has a kernel and fits the LDS and count limits.
bool tiling_fits(int precision, int n_phase, int tq, int lut_lds, int32_t max_count);
// Fill the shape fields of dp (pointers untouched).
void fill_shape(DevPlan &dp, int64_t n_curves, int64_t n_p, int64_t n_pd, int32_t n_phase,
                int32_t n_mag, int32_t tq, int32_t max_count, const gce_opts &o, int32_t lut_lds);
// Workspace layout of a filled shape holding total_points epochs (and the
// lists of refine_units work units per curve of an FP64 confirmation).
WorkspaceLayout workspace_layout(const DevPlan &dp, int64_t total_points,
                                 int32_t refine_units = 0);
// Point dp's workspace views into the block at `base`.
void bind_workspace(DevPlan &dp, char *base, const WorkspaceLayout &lay);

}  // namespace gce
