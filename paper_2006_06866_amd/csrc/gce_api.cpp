// gce_api.cpp -- host side of the C ABI declared in include/gce.h:
// argument validation, scheduling, workspace, plan cache and error text.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cinttypes>
#include <cstdlib>
#include <fstream>
#include <map>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <list>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "gce.h"
#include "gce_internal.h"

using gce::DevPlan;

namespace {

thread_local std::string g_last_error;
thread_local char g_status_buf[512];

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int fail_hip(hipError_t e, const char *what)
{
    return fail(GCE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Failure injection for tests of the out-of-memory paths: with the
// environment variable GCE_FAIL_ALLOC set to 1, every entry point that would
// allocate device memory fails with GCE_ENOMEM after validating its
// arguments and before touching the device.
bool alloc_failure_injected()
{
    const char *v = std::getenv("GCE_FAIL_ALLOC");
    return v && std::strcmp(v, "1") == 0;
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

int gce::check_device(int dev)
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(GCE_ENODEV, "no HIP device available");
    if (dev < 0 || dev >= count)
        return fail(GCE_ENODEV, "device ordinal out of range");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(GCE_ENODEV, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GCE_ENODEV, std::string("device is ") + prop.gcnArchName +
                                    ", the library is built for gfx950 only");
    return GCE_OK;
}

namespace {

using gce::check_device;

// ---------------------------------------------------------------------------
// tiling choice: autotuned per shape class, else a measured heuristic
// ---------------------------------------------------------------------------
// prec, overlap bits (1 phase, 2 magnitude), nph, nmag, pd class, N class
using TuneKey = std::tuple<int, int, int, int, int, int>;

struct Tiling {
    int tq;        // Pdot trials per lane
    int lut_lds;   // c ln c table in LDS
};

std::mutex g_tune_mu;
std::map<TuneKey, Tiling> g_tuned;
bool g_tune_file_read = false;

int pdot_class(int64_t n_pd)
{
    return n_pd <= 1 ? 0 : n_pd <= 2 ? 1 : n_pd <= 4 ? 2 : n_pd <= 8 ? 3 : 4;
}

int64_t median_length(const int64_t *off, int64_t n_curves)
{
    std::vector<int64_t> len((size_t)n_curves);
    for (int64_t c = 0; c < n_curves; ++c) len[(size_t)c] = off[c + 1] - off[c];
    std::nth_element(len.begin(), len.begin() + n_curves / 2, len.end());
    return len[(size_t)(n_curves / 2)];
}

int length_class(const int64_t *off, int64_t n_curves)
{
    const int64_t med = median_length(off, n_curves);
    return med < 128 ? 0 : med < 512 ? 1 : med < 2048 ? 2 : 3;
}

TuneKey tune_key(int precision, int overlap, int n_phase, int n_mag, int64_t n_pd,
                 const int64_t *off, int64_t n_curves)
{
    return TuneKey{precision, overlap, n_phase, n_mag, pdot_class(n_pd),
                   length_class(off, n_curves)};
}

// GCE_TUNE_CACHE file: one "prec overlap nph nmag pdclass nclass tq lut_lds"
// line per choice.
void read_tune_file_locked()
{
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char *path = std::getenv("GCE_TUNE_CACHE");
    if (!path || !*path) return;
    std::ifstream in(path);
    int a, b, c, d, e, f, tq, ll;
    while (in >> a >> b >> c >> d >> e >> f >> tq >> ll)
        if ((tq == 1 || tq == 2 || tq == 4 || tq == 8) && (ll == 0 || ll == 1))
            g_tuned[TuneKey{a, b, c, d, e, f}] = Tiling{tq, ll};
}

// The table in LDS costs every wave one pass over max_count + 1 doubles and
// LDS space, and saves a global gather per histogram cell at every
// magnitude-segment flush: it pays when the table is small, the cells are
// many per epoch, and the wave's LDS stays small enough for 8 or more
// waves per CU.  Measured on MI355X: 50 x 10 overlapping bins, N = 500,
// 2 trials: 4.9 s with the table in LDS vs 6.5 s; 10 x 5 bins, N = 600:
// 75 vs 61 ms; N up to 3,000: 485 vs 209 ms.
int heuristic_lut_lds(int precision, int n_phase, int n_mag, int tq, int32_t max_count,
                      int64_t median_n)
{
    return max_count <= 1023 && 4 * (int64_t)n_phase * n_mag >= median_n &&
           gce::search_lds_bytes(precision, n_phase, tq, 1, max_count) <=
               (size_t)gce::search_waves_per_block(1) * 20 * 1024;
}

}  // namespace

int gce::set_error(int code, const char *msg) { return fail(code, msg); }

#ifndef GCE_CO_MIN_BYTES
#define GCE_CO_MIN_BYTES 8192   // one-wave histogram bytes from which two waves share a unit
#endif
// Waves per work unit: two share one copy of the unit's histograms where a
// wave's own copy would be large.  Measured on MI355X (kernel ms, one / two
// waves per unit): 50 x 10 overlapping bins, 32 curves of the paper-scale
// grid, 2 trials: 860 / 712; 20 x 10 bins, 64 x 5,000 epochs, 4 trials:
// 1114 / 1057; split path, 10 x 5 bins, 8 trials: 46.1 / 44.6; but FP64,
// 10 x 5 bins, 4 trials (5 KiB): 52.4 / 53.9.
int gce::heuristic_co(int precision, int n_phase, int tq, int lut_lds, int32_t max_count)
{
    const size_t hist = (size_t)((tq + 1) / 2) * n_phase * gce::kWave * sizeof(uint32_t);
    return GCE_CO_MIN_BYTES > 0 && hist >= (size_t)GCE_CO_MIN_BYTES &&
                   gce::search_variant_exists(precision, n_phase, tq, 2) &&
                   gce::search_lds_bytes(precision, n_phase, tq, lut_lds, max_count, 2) <=
                       gce::kMaxLdsBytes
               ? 2
               : 1;
}

int gce::heuristic_tq(int precision, int n_phase, int64_t n_pd, int32_t max_count,
                      int waves_per_unit)
{
    // Pdot trials per lane: more trials share each epoch's x and x^2, but
    // every trial pair adds a histogram region of LDS and registers.
    // Measured on MI355X (kernel ms at 1 / 2 / 4 / 8 trials, one wave per
    // work unit):
    //   FP64, 10 x 5 bins, 512 x 600 x 20,000 x 64:     - / 59.4 / 53.1 / 54.4
    //   FP64, 20 x 10 bins, 64 x 5,000 x 100,000 x 256: - / 1165 / 1121 / 1563
    //   split, 10 x 5 bins, 512 x 600 x 20,000 x 64:    - / 63.6 / 50.9 / 48.3
    //   split, 20 x 10 bins, 64 x 5,000 x ...:          - / 1213 / 1022 / 1539
    // so FP64 starts from 4 and the split path from 8, and a wave's
    // histograms stay within ~13 KiB (at 20 KiB the CU holds too few waves).
    // With two waves per unit, FP64 at 10 x 5 bins and 8 trials keeps 5 KiB
    // per wave, as 4 trials on one wave do, and was faster: 52.6 against
    // 53.8 ms (one box); at 20 x 10 bins (10 KiB per wave) it was not, 1072
    // against 1062 ms.  So FP64 starts from 8 where two waves hold eight
    // trials in at most 5 KiB per wave.
    int tq = precision == GCE_PRECISION_FP64 ? 4 : 8;
    const size_t hist8 = (size_t)4 * n_phase * kWave * sizeof(uint32_t);
    if (precision == GCE_PRECISION_FP64 && waves_per_unit != 1 && hist8 / 2 <= 5 * 1024 &&
        heuristic_co(precision, n_phase, 8, 0, max_count) == 2)
        tq = 8;
    while (tq > 1 &&
           (tq >= 2 * n_pd || !gce::search_variant_exists(precision, n_phase, tq) ||
            gce::search_lds_bytes(precision, n_phase, tq, 0, max_count) > 13 * 1024))
        tq /= 2;
    return tq;
}

bool gce::tiling_fits(int precision, int n_phase, int tq, int lut_lds, int32_t max_count)
{
    return gce::search_variant_exists(precision, n_phase, tq) &&
           (!lut_lds || max_count <= gce::kMaxLdsTableCount) &&
           gce::search_lds_bytes(precision, n_phase, tq, lut_lds, max_count) <= gce::kMaxLdsBytes;
}

namespace {

// Tiling of a plan: an autotuned choice for the shape class when neither
// trials per lane nor the table placement is requested (and the choice fits
// this batch: a class is keyed by the median curve length, so a batch of the
// same class may hold a curve too long for a tuned table in LDS), else the
// request and the heuristics for what was left open.
Tiling choose_tiling(int precision, int overlap, int n_phase, int n_mag, int64_t n_pd,
                     const int64_t *off, int64_t n_curves, int32_t max_count,
                     int requested_tq, int requested_placement, int requested_co)
{
    if (requested_tq == 0 && requested_placement == GCE_TABLE_AUTO) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        read_tune_file_locked();
        auto it = g_tuned.find(tune_key(precision, overlap, n_phase, n_mag, n_pd, off,
                                        n_curves));
        if (it != g_tuned.end() &&
            gce::tiling_fits(precision, n_phase, it->second.tq, it->second.lut_lds, max_count))
            return it->second;
    }
    Tiling t{0, 0};
    t.tq = requested_tq > 0 ? requested_tq
                            : gce::heuristic_tq(precision, n_phase, n_pd, max_count,
                                                requested_co);
    if (requested_placement == GCE_TABLE_GLOBAL) t.lut_lds = 0;
    else if (requested_placement == GCE_TABLE_LDS) t.lut_lds = 1;
    else t.lut_lds = heuristic_lut_lds(precision, n_phase, n_mag, t.tq, max_count,
                                       median_length(off, n_curves));
    return t;
}

}  // namespace

struct gce_plan_s {
    int device = 0;
    gce_opts opts{};
    DevPlan dp{};
    int64_t total_points = 0;
    // a second search launch over the shortest curves with the table in
    // LDS: its first unit (0 = one launch) and count bound
    int64_t split_unit = 0;
    int32_t split_max_count = 0;
    std::vector<int64_t> off_host;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    uint64_t key_hash = 0;
    // FP64 confirmation of a split search's minima (gce_opts.refine_units):
    // work units per curve and the device lists and results
    int32_t refine_k = 0;
    int64_t *refine_list = nullptr;
    gce::Partial *refine_partials = nullptr;
    gce::UnitStats *refine_stats = nullptr;
    // search-kernel timing ring (gce_plan_set_timing)
    std::vector<hipEvent_t> ev_start, ev_stop;
    int64_t n_timed = 0;
};

namespace {

uint64_t hash_offsets(const int64_t *off, int64_t n)
{
    uint64_t h = 1469598103934665603ull;   // FNV-1a over the offset words
    for (int64_t i = 0; i <= n; ++i) {
        uint64_t v = (uint64_t)off[i];
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xffu;
            h *= 1099511628211ull;
        }
    }
    return h;
}

}  // namespace

int gce::validate_shape(const int64_t *off, int64_t n_curves, int64_t n_p,
                        int64_t n_pd, int32_t n_phase, int32_t n_mag,
                        int32_t *max_n_out)
{
    if (!off) return fail(GCE_EINVAL, "curve_offsets is NULL");
    if (n_curves < 1) return fail(GCE_EINVAL, "n_curves must be >= 1");
    // one 256-thread block per curve in the per-curve kernels: the dispatch
    // grid (work-items) must stay below 2^32
    if (n_curves > 16000000) return fail(GCE_EINVAL, "more than 16,000,000 curves");
    if (n_p < 1 || n_pd < 1) return fail(GCE_EINVAL, "grid sizes must be >= 1");
    if (n_phase < 1 || n_phase > gce::kMaxPhaseBins)
        return fail(GCE_EINVAL, "n_phase_bins out of range [1, 128]");
    if (n_mag < 1 || n_mag > gce::kMaxMagBins)
        return fail(GCE_EINVAL, "n_mag_bins out of range [1, 255]");
    if (off[0] != 0) return fail(GCE_EINVAL, "curve_offsets[0] must be 0");
    int64_t max_n = 0;
    for (int64_t c = 0; c < n_curves; ++c) {
        const int64_t n = off[c + 1] - off[c];
        if (n < 1) return fail(GCE_EINVAL, "curve with no epochs (offsets not increasing)");
        if (n > gce::kMaxPoints) return fail(GCE_EINVAL, "curve longer than 65535 epochs");
        max_n = std::max(max_n, n);
    }
    // index arithmetic in the kernels keeps tiles and Pdot groups in 32 bits
    const int64_t n_ptiles = (n_p + gce::kWave - 1) / gce::kWave;
    if (n_ptiles > (int64_t)1 << 30 || n_pd > (int64_t)1 << 30)
        return fail(GCE_EINVAL, "grid too large");
    *max_n_out = (int32_t)max_n;
    return GCE_OK;
}

// Largest count a histogram cell, a marginal or a pair of phase slots can
// reach: every entry of a curve lands in one cell per phase slot, a curve has
// up to 2N entries with overlapping magnitude bins, and a single overlapping
// phase bin adds its one slot to itself.  Counts are 16-bit, so the bound must
// stay at or below 65535.
int gce::count_bound(int32_t max_n, int32_t n_phase, int32_t phase_overlap,
                     int32_t mag_overlap, int32_t *max_count_out)
{
    int64_t m = max_n;
    if (mag_overlap) m *= 2;
    if (phase_overlap && n_phase == 1) m *= 2;
    if (m > gce::kMaxPoints)
        return fail(GCE_EUNSUPPORTED,
                    "overlapping bins count an epoch more than once: the counts of "
                    "the longest curve would exceed 65535");
    *max_count_out = (int32_t)m;
    return GCE_OK;
}

void gce::fill_shape(DevPlan &dp, int64_t n_curves, int64_t n_p, int64_t n_pd,
                     int32_t n_phase, int32_t n_mag, int32_t tq, int32_t max_count,
                     const gce_opts &o, int32_t lut_lds)
{
    dp.n_curves = n_curves;
    dp.n_p = n_p;
    dp.n_pd = n_pd;
    dp.n_phase = n_phase;
    dp.n_mag = n_mag;
    dp.tq = tq;
    dp.n_qgroups = (int32_t)((n_pd + tq - 1) / tq);
    dp.n_ptiles = (n_p + kWave - 1) / kWave;
    dp.units_per_curve = (int64_t)dp.n_qgroups * dp.n_ptiles;
    dp.n_units = n_curves * dp.units_per_curve;
    dp.unit0 = 0;
    dp.max_count = max_count;
    dp.precision = o.precision;
    dp.overlap = o.phase_overlap;
    dp.mag_overlap = o.mag_overlap;
    dp.lut_lds = lut_lds;
    dp.co = 1;
}

gce::WorkspaceLayout gce::workspace_layout(const DevPlan &dp, int64_t total_points,
                                           int32_t refine_units)
{
    const size_t A = 256;
    size_t sz = 0;
    auto take = [&](size_t bytes) {
        size_t at = sz;
        sz = align_up(sz + bytes, A);
        return at;
    };
    WorkspaceLayout L{};
    L.off = take(sizeof(int64_t) * (size_t)(dp.n_curves + 1));
    L.order = take(sizeof(int32_t) * (size_t)dp.n_curves);
    L.lut = take(sizeof(double) * (size_t)(dp.max_count + 1));
    const size_t entries = (size_t)total_points * (dp.mag_overlap ? 2 : 1);
    L.dt = take(sizeof(double) * entries);
    L.dt2f = take(dp.precision == GCE_PRECISION_SPLIT_FP32 ? sizeof(float) * entries : 0);
    L.seg = take(sizeof(int32_t) * (size_t)dp.n_curves * (size_t)(dp.n_mag + 1));
    L.curve_ok = take(sizeof(int32_t) * (size_t)dp.n_curves);
    L.grid_ok = take(sizeof(int32_t));
    L.inv_p = take(sizeof(double) * (size_t)dp.n_p);
    L.inv_p2f = take(dp.precision == GCE_PRECISION_SPLIT_FP32 ? sizeof(float) * (size_t)dp.n_p : 0);
    L.half_pd = take(sizeof(double) * (size_t)dp.n_pd);
    L.half_pd32 = take(sizeof(float) * (size_t)dp.n_pd);
    L.partials = take(sizeof(Partial) * (size_t)dp.n_units);
    L.stats = take(sizeof(UnitStats) * (size_t)dp.n_units);
    const size_t nref = (size_t)refine_units * (size_t)dp.n_curves;
    L.refine_list = take(sizeof(int64_t) * nref);
    L.refine_partials = take(sizeof(Partial) * nref);
    L.refine_stats = take(sizeof(UnitStats) * nref);
    L.total = sz;
    return L;
}

void gce::bind_workspace(DevPlan &dp, char *w, const WorkspaceLayout &L)
{
    dp.off = reinterpret_cast<const int64_t *>(w + L.off);
    dp.order = reinterpret_cast<const int32_t *>(w + L.order);
    dp.lut = reinterpret_cast<const double *>(w + L.lut);
    dp.dt_sorted = reinterpret_cast<double *>(w + L.dt);
    dp.dt2f_sorted =
        dp.precision == GCE_PRECISION_SPLIT_FP32 ? reinterpret_cast<float *>(w + L.dt2f) : nullptr;
    dp.seg = reinterpret_cast<int32_t *>(w + L.seg);
    dp.curve_ok = reinterpret_cast<int32_t *>(w + L.curve_ok);
    dp.grid_ok = reinterpret_cast<int32_t *>(w + L.grid_ok);
    dp.inv_p = reinterpret_cast<double *>(w + L.inv_p);
    dp.inv_p2f =
        dp.precision == GCE_PRECISION_SPLIT_FP32 ? reinterpret_cast<float *>(w + L.inv_p2f) : nullptr;
    dp.half_pd = reinterpret_cast<double *>(w + L.half_pd);
    dp.half_pd32 = reinterpret_cast<float *>(w + L.half_pd32);
    dp.partials = reinterpret_cast<Partial *>(w + L.partials);
    dp.stats = reinterpret_cast<UnitStats *>(w + L.stats);
}

namespace {

int overlap_bits(int32_t phase_overlap, int32_t mag_overlap)
{
    return (phase_overlap ? 1 : 0) | (mag_overlap ? 2 : 0);
}

// Ragged batches: the curves with many histogram cells per epoch (N at most
// 4 n_phase n_mag, the automatic placement's own criterion) take a second
// search launch with the table in LDS, sized for the longest of them, when
// the placement is automatic and the batch as a whole keeps the table in
// global memory.  Measured on MI355X, 8,192 curves of 50-3,000 epochs,
// 10 x 5 bins, 4 trials per lane (kernel ms, global / LDS table):
// N <= 150: 16.4 / 11.8; 150 < N <= 600: 63.5 / 68.9; N > 600: 100.6 / 157.1.
// Returns the number of curves of the first launch (the longest ones; the
// schedule is longest first), or 0 for one launch; *short_max_count receives
// the second launch's count bound (below the whole plan's, which passed).
int64_t split_by_length(int precision, int n_phase, int n_mag, int tq, int phase_overlap,
                        int mag_overlap, const int64_t *off, int64_t n_curves,
                        int32_t *short_max_count)
{
    const int64_t limit = 4 * (int64_t)n_phase * n_mag;
    int64_t n_long = 0, short_max = 0;
    for (int64_t c = 0; c < n_curves; ++c) {
        const int64_t n = off[c + 1] - off[c];
        if (n > limit) ++n_long;
        else short_max = std::max(short_max, n);
    }
    if (n_long == 0 || n_long == n_curves) return 0;
    int32_t mc = 0;
    if (gce::count_bound((int32_t)short_max, n_phase, phase_overlap, mag_overlap, &mc) != GCE_OK)
        return 0;
    if (mc > 1023 ||
        gce::search_lds_bytes(precision, n_phase, tq, 1, mc) >
            (size_t)gce::search_waves_per_block(1) * 20 * 1024)
        return 0;
    *short_max_count = mc;
    return n_long;
}

}  // namespace

extern "C" {

const char *gce_version(void) { return "gce-mi355x 0.4.0 (gfx950)"; }

const char *gce_status_string(int status)
{
    const char *base = "unknown status";
    switch (status) {
    case GCE_OK: base = "success"; break;
    case GCE_EINVAL: base = "invalid argument"; break;
    case GCE_ENOMEM: base = "out of memory"; break;
    case GCE_EHIP: base = "HIP runtime error"; break;
    case GCE_EWORKSPACE: base = "workspace too small"; break;
    case GCE_ENODEV: base = "no usable gfx950 device"; break;
    case GCE_EUNSUPPORTED: base = "unsupported option"; break;
    default: break;
    }
    if (status != GCE_OK && !g_last_error.empty())
        std::snprintf(g_status_buf, sizeof(g_status_buf), "%s: %s", base,
                      g_last_error.c_str());
    else
        std::snprintf(g_status_buf, sizeof(g_status_buf), "%s", base);
    return g_status_buf;
}

int gce_plan_create(gce_plan_t *plan_out, const int64_t *curve_offsets,
                    int64_t n_curves, int64_t n_periods, int64_t n_pdots,
                    int32_t n_phase_bins, int32_t n_mag_bins,
                    const gce_opts *opts, int32_t device)
{
    if (!plan_out) return fail(GCE_EINVAL, "plan pointer is NULL");
    *plan_out = nullptr;
    int32_t max_n = 0;
    int rc = gce::validate_shape(curve_offsets, n_curves, n_periods, n_pdots,
                                 n_phase_bins, n_mag_bins, &max_n);
    if (rc != GCE_OK) return rc;
    gce_opts o{};
    if (opts) o = *opts;
    if (o.precision != GCE_PRECISION_FP64 && o.precision != GCE_PRECISION_SPLIT_FP32)
        return fail(GCE_EINVAL, "unknown precision");
    if (o.trials_per_lane != 0 && o.trials_per_lane != 1 && o.trials_per_lane != 2 &&
        o.trials_per_lane != 4 && o.trials_per_lane != 8)
        return fail(GCE_EINVAL, "trials_per_lane must be 0, 1, 2, 4 or 8");
    if (o.phase_overlap != 0 && o.phase_overlap != 1)
        return fail(GCE_EINVAL, "phase_overlap must be 0 or 1");
    if (o.mag_overlap != 0 && o.mag_overlap != 1)
        return fail(GCE_EINVAL, "mag_overlap must be 0 or 1");
    if (o.table_placement != GCE_TABLE_AUTO && o.table_placement != GCE_TABLE_GLOBAL &&
        o.table_placement != GCE_TABLE_LDS)
        return fail(GCE_EINVAL, "table_placement must be 0, 1 or 2");
    if (o.waves_per_unit != 0 && o.waves_per_unit != 1 && o.waves_per_unit != 2)
        return fail(GCE_EINVAL, "waves_per_unit must be 0, 1 or 2");
    if (o.refine_units < 0 || o.refine_units > gce::kMaxRefineUnits)
        return fail(GCE_EINVAL, "refine_units must be in [0, 64]");
    int32_t max_count = 0;
    rc = gce::count_bound(max_n, n_phase_bins, o.phase_overlap, o.mag_overlap, &max_count);
    if (rc != GCE_OK) return rc;
    const Tiling tl = choose_tiling(o.precision, overlap_bits(o.phase_overlap, o.mag_overlap),
                                    n_phase_bins, n_mag_bins, n_pdots, curve_offsets,
                                    n_curves, max_count, o.trials_per_lane,
                                    o.table_placement, o.waves_per_unit);
    const int tq = tl.tq;
    if (!gce::search_variant_exists(o.precision, n_phase_bins, tq))
        return fail(GCE_EUNSUPPORTED, "no search kernel for this phase-bin count and trials_per_lane");
    if (tl.lut_lds && max_count > gce::kMaxLdsTableCount)   // counts in units of 8
        return fail(GCE_EUNSUPPORTED,
                    "the table in LDS needs counts of at most 8191 (curves of at most "
                    "8191 epochs, half that with overlapping magnitude bins)");
    const int co = o.waves_per_unit != 0
                       ? o.waves_per_unit
                       : gce::heuristic_co(o.precision, n_phase_bins, tq, tl.lut_lds, max_count);
    if (co == 2 && !gce::search_variant_exists(o.precision, n_phase_bins, tq, 2))
        return fail(GCE_EUNSUPPORTED,
                    "no two-wave search kernel for this phase-bin count and trials_per_lane");
    if (gce::search_lds_bytes(o.precision, n_phase_bins, tq, tl.lut_lds, max_count, co) >
        gce::kMaxLdsBytes)
        return fail(GCE_EUNSUPPORTED,
                    "a block's LDS would exceed 64 KiB: lower trials_per_lane or keep the "
                    "table in global memory");
    // the FP64 confirmation runs the FP64 kernel of the same tiling, with the
    // table in global memory, over the chosen work units
    const int32_t refine_k = o.precision == GCE_PRECISION_SPLIT_FP32 ? o.refine_units : 0;
    if (refine_k > 0 &&
        (!gce::search_variant_exists(GCE_PRECISION_FP64, n_phase_bins, tq, co) ||
         gce::search_lds_bytes(GCE_PRECISION_FP64, n_phase_bins, tq, 0, max_count, co) >
             gce::kMaxLdsBytes))
        return fail(GCE_EUNSUPPORTED, "no FP64 search kernel of this tiling for refine_units");

    DevPlan shape{};
    gce::fill_shape(shape, n_curves, n_periods, n_pdots, n_phase_bins, n_mag_bins, tq,
                    max_count, o, tl.lut_lds);
    if (shape.n_units > gce::kMaxUnits)
        return fail(GCE_EINVAL, "too many work units for one launch");
    if (alloc_failure_injected())
        return fail(GCE_ENOMEM, "device allocation failure injected (GCE_FAIL_ALLOC=1)");

    rc = check_device(device);
    if (rc != GCE_OK) return rc;
    DeviceGuard guard(device);
    if (!guard.ok) return fail(GCE_ENODEV, "hipSetDevice failed");

    gce_plan_s *pl = new (std::nothrow) gce_plan_s();
    if (!pl) return fail(GCE_ENOMEM, "host allocation failed");
    pl->device = device;
    pl->opts = o;
    pl->off_host.assign(curve_offsets, curve_offsets + n_curves + 1);
    pl->total_points = curve_offsets[n_curves];
    pl->key_hash = hash_offsets(curve_offsets, n_curves);

    DevPlan &dp = pl->dp;
    dp = shape;
    dp.co = co;
    // whenever the placement is automatic and the batch keeps the table in
    // global memory (chosen by the heuristics or by tuning)
    if (o.table_placement == GCE_TABLE_AUTO && !tl.lut_lds) {
        const int64_t n_long = split_by_length(o.precision, n_phase_bins, n_mag_bins, tq,
                                               o.phase_overlap, o.mag_overlap, curve_offsets,
                                               n_curves, &pl->split_max_count);
        pl->split_unit = n_long * dp.units_per_curve;
    }

    if ((dp.lut_lds || pl->split_unit > 0) &&
        !gce::search_table_in_lds_ok(o.precision, dp.overlap, n_phase_bins, tq, dp.co)) {
        delete pl;
        return fail(GCE_EUNSUPPORTED, "search kernel with the table in LDS has static LDS");
    }

    // schedule: longest curves first (stable), so ragged batches drain evenly
    std::vector<int32_t> order((size_t)n_curves);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return (curve_offsets[a + 1] - curve_offsets[a]) >
               (curve_offsets[b + 1] - curve_offsets[b]);
    });

    pl->refine_k = refine_k;
    const gce::WorkspaceLayout lay = gce::workspace_layout(dp, pl->total_points, refine_k);
    pl->ws_bytes = lay.total;
    hipError_t e = hipMalloc(&pl->ws, lay.total);
    if (e != hipSuccess) {
        delete pl;
        (void)hipGetLastError();
        return fail(GCE_ENOMEM, "hipMalloc of the workspace failed");
    }
    gce::bind_workspace(dp, static_cast<char *>(pl->ws), lay);
    if (refine_k > 0) {
        char *w = static_cast<char *>(pl->ws);
        pl->refine_list = reinterpret_cast<int64_t *>(w + lay.refine_list);
        pl->refine_partials = reinterpret_cast<gce::Partial *>(w + lay.refine_partials);
        pl->refine_stats = reinterpret_cast<gce::UnitStats *>(w + lay.refine_stats);
    }

    e = hipMemcpy(const_cast<int64_t *>(dp.off), curve_offsets,
                  sizeof(int64_t) * (size_t)(n_curves + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(const_cast<int32_t *>(dp.order), order.data(),
                      sizeof(int32_t) * (size_t)n_curves, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = gce::launch_lut(dp, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        int r = fail_hip(e, "plan set-up");
        (void)hipFree(pl->ws);
        delete pl;
        return r;
    }
    *plan_out = pl;
    return GCE_OK;
}

// The search over the plan's work units: one launch, or with a length split
// the longest curves (table as chosen) then the shortest (table in LDS).
static hipError_t search_launches(const gce_plan_s *pl, void *out_ce, hipStream_t s)
{
    if (pl->split_unit <= 0) return gce::launch_search(pl->dp, out_ce, s);
    DevPlan a = pl->dp;
    a.n_units = pl->split_unit;
    hipError_t e = gce::launch_search(a, out_ce, s);
    if (e != hipSuccess) return e;
    DevPlan b = pl->dp;
    b.unit0 = pl->split_unit;
    b.lut_lds = 1;
    b.max_count = pl->split_max_count;
    return gce::launch_search(b, out_ce, s);
}

int gce_plan_execute(gce_plan_t pl, const double *times, const double *mags,
                     const double *periods, const double *pdots, void *out_ce,
                     gce_best_t *out_best, void *stream)
{
    if (!pl) return fail(GCE_EINVAL, "plan is NULL");
    if (!times || !mags || !periods || !pdots || !out_best)
        return fail(GCE_EINVAL, "NULL input or output pointer");
    DeviceGuard guard(pl->device);
    if (!guard.ok) return fail(GCE_ENODEV, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const DevPlan &dp = pl->dp;
    // the prepass sets the grid-validity flag that the grid set-up may clear
    hipError_t e = gce::launch_prepass(dp, times, mags, s);
    if (e != hipSuccess) return fail_hip(e, "prepass launch");
    e = gce::launch_grid_setup(dp, periods, pdots, s);
    if (e != hipSuccess) return fail_hip(e, "grid set-up launch");
    const bool timed = !pl->ev_start.empty();
    const size_t slot = timed ? (size_t)(pl->n_timed % (int64_t)pl->ev_start.size()) : 0;
    if (timed && (e = hipEventRecord(pl->ev_start[slot], s)) != hipSuccess)
        return fail_hip(e, "timing event");
    e = search_launches(pl, out_ce, s);
    if (e != hipSuccess) return fail_hip(e, "search launch");
    if (timed) {
        if ((e = hipEventRecord(pl->ev_stop[slot], s)) != hipSuccess)
            return fail_hip(e, "timing event");
        ++pl->n_timed;
    }
    e = gce::launch_epilogue(dp, out_best, s);
    if (e != hipSuccess) return fail_hip(e, "epilogue launch");
    if (pl->refine_k > 0) {
        // the FP64 kernel of the same tiling over each curve's refine_k best
        // split work units, then their FP64 minimum into out_best
        e = gce::launch_refine_select(dp, pl->refine_k, pl->refine_list, s);
        if (e != hipSuccess) return fail_hip(e, "refine selection launch");
        DevPlan r = dp;
        r.precision = GCE_PRECISION_FP64;
        r.lut_lds = 0;
        r.unit_list = pl->refine_list;
        r.unit0 = 0;
        r.n_units = (int64_t)pl->refine_k * dp.n_curves;
        r.partials = pl->refine_partials;
        r.stats = pl->refine_stats;
        e = gce::launch_search(r, nullptr, s);
        if (e != hipSuccess) return fail_hip(e, "refine search launch");
        e = gce::launch_refine_merge(dp, pl->refine_k, pl->refine_partials, out_best, s);
        if (e != hipSuccess) return fail_hip(e, "refine merge launch");
    }
    return GCE_OK;
}

int gce_plan_debug_counts(gce_plan_t pl, const double *times,
                          const double *mags, const double *periods,
                          const double *pdots, const int64_t *trial_curve,
                          const int64_t *trial_flat, int64_t n_trials,
                          uint32_t *out_counts, void *stream)
{
    if (!pl) return fail(GCE_EINVAL, "plan is NULL");
    if (n_trials < 0) return fail(GCE_EINVAL, "n_trials < 0");
    if (!times || !mags || !periods || !pdots ||
        (n_trials > 0 && (!trial_curve || !trial_flat || !out_counts)))
        return fail(GCE_EINVAL, "NULL pointer");
    if (n_trials > ((int64_t)1 << 31) - 64) return fail(GCE_EINVAL, "too many trials");
    DeviceGuard guard(pl->device);
    if (!guard.ok) return fail(GCE_ENODEV, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const DevPlan &dp = pl->dp;
    hipError_t e = gce::launch_prepass(dp, times, mags, s);
    if (e == hipSuccess) e = gce::launch_grid_setup(dp, periods, pdots, s);
    if (e == hipSuccess)
        e = gce::launch_debug_counts(dp, trial_curve, trial_flat, n_trials, out_counts, s);
    if (e != hipSuccess) return fail_hip(e, "debug counts launch");
    return GCE_OK;
}

size_t gce_plan_workspace_bytes(gce_plan_t pl) { return pl ? pl->ws_bytes : 0; }

int gce_merge_results(gce_best_t *acc, int64_t acc_trials, const gce_best_t *part,
                      int64_t n_curves, int64_t n_periods, int64_t part_p_offset,
                      int64_t part_n_periods, int64_t part_q_offset,
                      int64_t part_n_pdots)
{
    if (!acc || !part || n_curves < 1 || acc_trials < 0 || n_periods < 1 ||
        part_p_offset < 0 || part_n_periods < 1 || part_q_offset < 0 ||
        part_n_pdots < 1 || part_p_offset + part_n_periods > n_periods)
        return fail(GCE_EINVAL, "bad merge arguments");
    const double nb = (double)part_n_periods * (double)part_n_pdots;
    const double na = (double)acc_trials;
    for (int64_t c = 0; c < n_curves; ++c) {
        gce_best_t in = part[c];
        if (in.flat_index >= 0) {   // to full-grid indices
            const int64_t q = in.flat_index / part_n_periods + part_q_offset;
            const int64_t p = in.flat_index % part_n_periods + part_p_offset;
            in.flat_index = q * n_periods + p;
            in.period_index = (int32_t)p;
            in.pdot_index = (int32_t)q;
        }
        gce_best_t &a = acc[c];
        if (acc_trials == 0) {
            a = in;
            continue;
        }
        if (a.flat_index < 0 || in.flat_index < 0) {   // invalid stays invalid
            a.flat_index = -1;
            a.period_index = a.pdot_index = -1;
            a.ce_min = a.ce_mean = a.ce_std = a.significance = NAN;
            continue;
        }
        if (in.ce_min < a.ce_min || (in.ce_min == a.ce_min && in.flat_index < a.flat_index)) {
            a.flat_index = in.flat_index;
            a.period_index = in.period_index;
            a.pdot_index = in.pdot_index;
            a.ce_min = in.ce_min;
        }
        const double n = na + nb;
        const double d = in.ce_mean - a.ce_mean;
        const double m2 = a.ce_std * a.ce_std * na + in.ce_std * in.ce_std * nb +
                          d * d * (na * nb / n);
        a.ce_mean = a.ce_mean + d * (nb / n);
        a.ce_std = std::sqrt(m2 / n);
        a.significance = a.ce_std > 0.0 ? (a.ce_mean - a.ce_min) / a.ce_std : 0.0;
    }
    return GCE_OK;
}

int gce_plan_get_info(gce_plan_t pl, gce_plan_info_t *info)
{
    if (!pl || !info) return fail(GCE_EINVAL, "NULL argument");
    info->precision = pl->dp.precision;
    info->trials_per_lane = pl->dp.tq;
    info->lds_bytes_per_wave = (int32_t)(
        gce::search_lds_bytes(pl->dp.precision, pl->dp.n_phase, pl->dp.tq, pl->dp.lut_lds,
                              pl->dp.max_count, pl->dp.co) /
        gce::search_waves_per_block(pl->dp.lut_lds, pl->dp.co));
    info->table_in_lds = pl->split_unit > 0 ? 2 : pl->dp.lut_lds;
    info->work_units = pl->dp.n_units;
    info->workspace_bytes = (int64_t)pl->ws_bytes;
    info->waves_per_unit = pl->dp.co;
    info->refine_units = pl->refine_k;
    return GCE_OK;
}

static void free_timing(gce_plan_s *pl)
{
    for (hipEvent_t ev : pl->ev_start) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : pl->ev_stop) (void)hipEventDestroy(ev);
    pl->ev_start.clear();
    pl->ev_stop.clear();
    pl->n_timed = 0;
}

int gce_plan_set_timing(gce_plan_t pl, int32_t capacity)
{
    if (!pl) return fail(GCE_EINVAL, "plan is NULL");
    if (capacity < 0 || capacity > 65536) return fail(GCE_EINVAL, "capacity out of range");
    DeviceGuard guard(pl->device);
    if (!guard.ok) return fail(GCE_ENODEV, "hipSetDevice failed");
    (void)hipDeviceSynchronize();
    free_timing(pl);
    for (int32_t i = 0; i < capacity; ++i) {
        hipEvent_t a = nullptr, b = nullptr;
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e != hipSuccess) {
            if (a) (void)hipEventDestroy(a);
            free_timing(pl);
            return fail_hip(e, "hipEventCreate");
        }
        pl->ev_start.push_back(a);
        pl->ev_stop.push_back(b);
    }
    return GCE_OK;
}

int gce_plan_search_times(gce_plan_t pl, float *out_ms, int32_t max, int32_t *n_out)
{
    if (!pl || !n_out || max < 0 || (max > 0 && !out_ms))
        return fail(GCE_EINVAL, "bad argument");
    *n_out = 0;
    const int64_t cap = (int64_t)pl->ev_start.size();
    if (cap == 0) return GCE_OK;
    const int64_t avail = std::min<int64_t>(pl->n_timed, cap);
    const int64_t n = std::min<int64_t>(avail, max);
    DeviceGuard guard(pl->device);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t k = pl->n_timed - n + i;   // oldest of the last n first
        const size_t slot = (size_t)(k % cap);
        hipError_t e = hipEventSynchronize(pl->ev_stop[slot]);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, pl->ev_start[slot], pl->ev_stop[slot]);
        if (e != hipSuccess) return fail_hip(e, "timing read-out");
        out_ms[i] = ms;
    }
    *n_out = (int32_t)n;
    return GCE_OK;
}

int gce_plan_destroy(gce_plan_t pl)
{
    if (!pl) return GCE_OK;
    int rc = GCE_OK;
    {
        DeviceGuard guard(pl->device);
        hipError_t e = hipDeviceSynchronize();
        free_timing(pl);
        if (e == hipSuccess) e = hipFree(pl->ws);
        if (e != hipSuccess) rc = fail_hip(e, "plan destroy");
    }
    delete pl;
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// gce_search: a small cache of plans keyed by device and shape
// ---------------------------------------------------------------------------
namespace {

// Keyed by stream too: calls on different streams never share a workspace
// (overlapping searches on two streams would race on it), while calls on one
// stream are ordered by the stream itself.
struct CacheEntry {
    int device;
    void *stream;
    int64_t n_curves, n_p, n_pd;
    int32_t n_phase, n_mag;
    uint64_t hash;
    gce_plan_t plan;
};

std::mutex g_cache_mu;
std::list<CacheEntry> g_cache;   // most recent first
constexpr size_t kCacheMax = 4;

}  // namespace

extern "C" int gce_search(const double *times, const double *mags,
                          const int64_t *curve_offsets, int64_t n_curves,
                          const double *periods, int64_t n_periods,
                          const double *pdots, int64_t n_pdots,
                          int32_t n_phase_bins, int32_t n_mag_bins,
                          double *out_ce, gce_best_t *out_best, void *stream)
{
    int32_t max_n = 0;
    int rc = gce::validate_shape(curve_offsets, n_curves, n_periods, n_pdots,
                                 n_phase_bins, n_mag_bins, &max_n);
    if (rc != GCE_OK) return rc;
    if (!times || !mags || !periods || !pdots || !out_best)
        return fail(GCE_EINVAL, "NULL input or output pointer");
    if (alloc_failure_injected())
        return fail(GCE_ENOMEM, "device allocation failure injected (GCE_FAIL_ALLOC=1)");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(GCE_ENODEV, "hipGetDevice failed");
    const uint64_t h = hash_offsets(curve_offsets, n_curves);

    std::lock_guard<std::mutex> lock(g_cache_mu);
    gce_plan_t plan = nullptr;
    for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
        if (it->device == dev && it->stream == stream && it->n_curves == n_curves &&
            it->n_p == n_periods &&
            it->n_pd == n_pdots && it->n_phase == n_phase_bins &&
            it->n_mag == n_mag_bins && it->hash == h &&
            std::equal(curve_offsets, curve_offsets + n_curves + 1,
                       it->plan->off_host.begin())) {
            plan = it->plan;
            g_cache.splice(g_cache.begin(), g_cache, it);
            break;
        }
    }
    if (!plan) {
        rc = gce_plan_create(&plan, curve_offsets, n_curves, n_periods, n_pdots,
                             n_phase_bins, n_mag_bins, nullptr, dev);
        if (rc != GCE_OK) return rc;
        g_cache.push_front(CacheEntry{dev, stream, n_curves, n_periods, n_pdots,
                                      n_phase_bins, n_mag_bins, h, plan});
        while (g_cache.size() > kCacheMax) {
            gce_plan_destroy(g_cache.back().plan);
            g_cache.pop_back();
        }
    }
    return gce_plan_execute(plan, times, mags, periods, pdots, out_ce, out_best,
                            stream);
}

extern "C" int gce_autotune(const double *times, const double *mags,
                            const int64_t *curve_offsets, int64_t n_curves,
                            const double *periods, int64_t n_periods,
                            const double *pdots, int64_t n_pdots,
                            int32_t n_phase_bins, int32_t n_mag_bins,
                            int32_t precision, int32_t phase_overlap,
                            int32_t mag_overlap, int32_t device, void *stream,
                            int32_t *best_tq, int32_t *best_placement, float *ms)
{
    int32_t max_n = 0;
    int rc = gce::validate_shape(curve_offsets, n_curves, n_periods, n_pdots, n_phase_bins,
                                 n_mag_bins, &max_n);
    if (rc != GCE_OK) return rc;
    if (!times || !mags || !periods || !pdots || !best_tq)
        return fail(GCE_EINVAL, "NULL pointer");
    if (precision != GCE_PRECISION_FP64 && precision != GCE_PRECISION_SPLIT_FP32)
        return fail(GCE_EINVAL, "unknown precision");
    if (phase_overlap != 0 && phase_overlap != 1)
        return fail(GCE_EINVAL, "phase_overlap must be 0 or 1");
    if (mag_overlap != 0 && mag_overlap != 1)
        return fail(GCE_EINVAL, "mag_overlap must be 0 or 1");
    int32_t max_count = 0;
    rc = gce::count_bound(max_n, n_phase_bins, phase_overlap, mag_overlap, &max_count);
    if (rc != GCE_OK) return rc;
    if (alloc_failure_injected())
        return fail(GCE_ENOMEM, "device allocation failure injected (GCE_FAIL_ALLOC=1)");
    rc = check_device(device);
    if (rc != GCE_OK) return rc;
    DeviceGuard guard(device);
    if (!guard.ok) return fail(GCE_ENODEV, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);

    // slice: up to 128 curves spread evenly over the length-sorted curves,
    // gathered into one contiguous device buffer
    std::vector<int64_t> idx((size_t)n_curves);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        return (curve_offsets[a + 1] - curve_offsets[a]) <
               (curve_offsets[b + 1] - curve_offsets[b]);
    });
    const int64_t k = std::min<int64_t>(n_curves, 128);
    std::vector<int64_t> pick((size_t)k), off((size_t)k + 1, 0);
    for (int64_t i = 0; i < k; ++i) {
        pick[(size_t)i] = idx[(size_t)((i * n_curves + n_curves / 2) / k)];
        off[(size_t)i + 1] = off[(size_t)i] + curve_offsets[pick[(size_t)i] + 1] -
                             curve_offsets[pick[(size_t)i]];
    }
    const int64_t np_slice = std::min<int64_t>(n_periods, 8192);
    const int64_t tot = off[(size_t)k];
    double *buf = nullptr;
    gce_best_t *best = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&buf, sizeof(double) * (size_t)(2 * tot));
    if (e == hipSuccess) e = hipMalloc(&best, sizeof(gce_best_t) * (size_t)k);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int64_t i = 0; i < k && e == hipSuccess; ++i) {
        const int64_t a = curve_offsets[pick[(size_t)i]];
        const size_t n = (size_t)(off[(size_t)i + 1] - off[(size_t)i]);
        e = hipMemcpyAsync(buf + off[(size_t)i], times + a, n * sizeof(double),
                           hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(buf + tot + off[(size_t)i], mags + a, n * sizeof(double),
                               hipMemcpyDeviceToDevice, s);
    }
    const int cands[4] = {1, 2, 4, 8};
    float best_ms = -1.f;
    Tiling chosen{0, 0};
    for (int ci = 0; ci < 8 && e == hipSuccess; ++ci) {
        if (ms) ms[ci] = -1.f;
        const int tq = cands[ci % 4], ll = ci / 4;
        if (tq > 1 && tq >= 2 * n_pdots) continue;
        if (!gce::search_variant_exists(precision, n_phase_bins, tq) ||
            gce::search_lds_bytes(precision, n_phase_bins, tq, ll, max_count) > 40 * 1024)
            continue;
        gce_opts o{};
        o.precision = precision;
        o.trials_per_lane = tq;
        o.phase_overlap = phase_overlap;
        o.mag_overlap = mag_overlap;
        o.table_placement = ll ? GCE_TABLE_LDS : GCE_TABLE_GLOBAL;
        gce_plan_t pl = nullptr;
        rc = gce_plan_create(&pl, off.data(), k, np_slice, n_pdots, n_phase_bins,
                             n_mag_bins, &o, device);
        if (rc != GCE_OK) continue;
        float t_sum = 0.f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            // first execute warms up; the next two are timed
            if (rep > 0) e = hipEventRecord(e0, s);
            if (e == hipSuccess && gce_plan_execute(pl, buf, buf + tot, periods, pdots,
                                                    nullptr, best, s) != GCE_OK)
                e = hipErrorLaunchFailure;
            if (rep > 0 && e == hipSuccess) e = hipEventRecord(e1, s);
            if (rep > 0 && e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.f;
            if (rep > 0 && e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            t_sum += t;
        }
        gce_plan_destroy(pl);
        if (e != hipSuccess) break;
        const float t = t_sum / 2.f;
        if (ms) ms[ci] = t;
        if (best_ms < 0.f || t < best_ms) {
            best_ms = t;
            chosen = Tiling{tq, ll};
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (buf) (void)hipFree(buf);
    if (best) (void)hipFree(best);
    if (e != hipSuccess) return fail_hip(e, "autotune");
    if (chosen.tq == 0) return fail(GCE_EUNSUPPORTED, "no tiling fits this shape");
    *best_tq = chosen.tq;
    if (best_placement) *best_placement = chosen.lut_lds ? GCE_TABLE_LDS : GCE_TABLE_GLOBAL;
    const int ovl = overlap_bits(phase_overlap, mag_overlap);
    const TuneKey key = tune_key(precision, ovl, n_phase_bins, n_mag_bins, n_pdots,
                                 curve_offsets, n_curves);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    read_tune_file_locked();
    g_tuned[key] = chosen;
    if (const char *path = std::getenv("GCE_TUNE_CACHE")) {
        if (*path) {
            std::ofstream out(path, std::ios::app);
            out << precision << ' ' << ovl << ' ' << n_phase_bins << ' '
                << n_mag_bins << ' ' << pdot_class(n_pdots) << ' '
                << length_class(curve_offsets, n_curves) << ' ' << chosen.tq << ' '
                << chosen.lut_lds << '\n';
        }
    }
    return GCE_OK;
}
