// gce_noalloc.hip -- gce_search_noalloc: the one-call FP64 search with its
// workspace in a device array owned by the library, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Same kernels as every other entry point.
#include <mutex>

#include "gce_internal.h"

namespace {

constexpr size_t kScratchBytes = GCE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The workspace of every gce_search_noalloc call on a device.  Each device
// holds its own copy; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in there, not a device address).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];   // device address of `scratch`, per device

// The device address of this device's `scratch`, looked up (and the device
// checked) on the first call with that device current.
int scratch_address(int dev, char **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return gce::set_error(GCE_ENODEV, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int rc = gce::check_device(dev);
        if (rc != GCE_OK) return rc;
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return gce::set_error(GCE_EHIP, "hipGetSymbolAddress of the scratch array failed");
        }
        g_scratch_dev[dev] = p;
    }
    *out = static_cast<char *>(g_scratch_dev[dev]);
    return GCE_OK;
}

int hip_failed(hipError_t e, const char *what)
{
    (void)hipGetLastError();
    return gce::set_error(GCE_EHIP, what);
}

}  // namespace

extern "C" int gce_search_noalloc(const double *times, const double *mags,
                                  const int64_t *curve_offsets, int64_t n_curves,
                                  const double *periods, int64_t n_periods,
                                  const double *pdots, int64_t n_pdots,
                                  int32_t n_phase_bins, int32_t n_mag_bins,
                                  double *out_ce, gce_best_t *out_best, void *stream)
{
    using gce::DevPlan;
    int32_t max_n = 0;
    int rc = gce::validate_shape(curve_offsets, n_curves, n_periods, n_pdots, n_phase_bins,
                                 n_mag_bins, &max_n);
    if (rc != GCE_OK) return rc;
    if (!times || !mags || !periods || !pdots || !out_best)
        return gce::set_error(GCE_EINVAL, "NULL input or output pointer");
    int32_t max_count = 0;
    rc = gce::count_bound(max_n, n_phase_bins, 0, 0, &max_count);
    if (rc != GCE_OK) return rc;
    // FP64, the heuristic trials and waves per work unit, the c ln c table
    // in global memory, curves in their given order (no schedule to upload)
    const gce_opts o{};
    const int tq = gce::heuristic_tq(GCE_PRECISION_FP64, n_phase_bins, n_pdots, max_count);
    if (!gce::tiling_fits(GCE_PRECISION_FP64, n_phase_bins, tq, 0, max_count))
        return gce::set_error(GCE_EUNSUPPORTED, "no search kernel fits this shape");
    DevPlan dp{};
    gce::fill_shape(dp, n_curves, n_periods, n_pdots, n_phase_bins, n_mag_bins, tq, max_count,
                    o, 0);
    dp.co = gce::heuristic_co(GCE_PRECISION_FP64, n_phase_bins, tq, 0, max_count);
    if (dp.n_units > gce::kMaxUnits)
        return gce::set_error(GCE_EINVAL, "too many work units for one launch");
    const gce::WorkspaceLayout lay = gce::workspace_layout(dp, curve_offsets[n_curves]);
    if (lay.total > kScratchBytes)
        return gce::set_error(GCE_EWORKSPACE,
                              "the shape needs more workspace than the scratch array holds "
                              "(GCE_NOALLOC_SCRATCH_BYTES); use gce_search or a plan");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_failed(hipErrorNoDevice, "hipGetDevice failed");
    char *base = nullptr;
    rc = scratch_address(dev, &base);
    if (rc != GCE_OK) return rc;
    gce::bind_workspace(dp, base, lay);

    hipStream_t s = static_cast<hipStream_t>(stream);
    // every part of the workspace is written before it is read in each
    // call: the offsets and the schedule here, the c ln c table, then the
    // per-curve, per-grid and per-unit parts by the pipeline's kernels
    hipError_t e = hipMemcpyAsync(const_cast<int64_t *>(dp.off), curve_offsets,
                                  sizeof(int64_t) * (size_t)(n_curves + 1),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_failed(e, "offsets upload");
    if ((e = gce::launch_iota_order(dp, s)) != hipSuccess) return hip_failed(e, "schedule launch");
    if ((e = gce::launch_lut(dp, s)) != hipSuccess) return hip_failed(e, "table launch");
    if ((e = gce::launch_prepass(dp, times, mags, s)) != hipSuccess)
        return hip_failed(e, "prepass launch");
    if ((e = gce::launch_grid_setup(dp, periods, pdots, s)) != hipSuccess)
        return hip_failed(e, "grid set-up launch");
    if ((e = gce::launch_search(dp, out_ce, s)) != hipSuccess) return hip_failed(e, "search launch");
    if ((e = gce::launch_epilogue(dp, out_best, s)) != hipSuccess)
        return hip_failed(e, "epilogue launch");
    return GCE_OK;
}
