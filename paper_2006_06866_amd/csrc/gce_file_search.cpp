// gce_file_search -- run the CE (P, Pdot) search on inputs stored as raw
// files, through the C ABI of libgce.so alone (no Python).
//
//   gce_file_search DIR N_PHASE N_MAG [--split] [--phase-overlap]
//                   [--mag-overlap] [--cube] [--table global|lds]
//                   [--trials-per-lane T] [--waves-per-unit W] [--device D]
//
// Reads, from DIR, little-endian raw arrays:
//   times.f64, mags.f64   [sum N] epochs (days) and magnitudes, curve-major
//   offsets.i64           [n_curves + 1] curve offsets (offsets[0] = 0)
//   periods.f64           [n_periods] trial periods (days)
//   pdots.f64             [n_pdots] trial period derivatives
// Writes best.bin ([n_curves] gce_best_t, see gce.h) and, with --cube,
// cube.f64 (FP64) or cube.f32 (split path), row-major [curve][pdot][period].
// Prints one JSON line with the sizes and the search time.  Exit status 0 on
// success, 1 on a library or I/O error (message on stderr), 2 on bad usage.
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "gce.h"

namespace {

int usage()
{
    std::fprintf(stderr,
                 "usage: gce_file_search DIR N_PHASE N_MAG [--split] [--phase-overlap] "
                 "[--mag-overlap] [--cube] [--table global|lds] [--trials-per-lane T] "
                 "[--waves-per-unit W] [--refine-units K] [--device D]\n");
    return 2;
}

template <typename T>
bool read_array(const std::string &path, std::vector<T> &out)
{
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) {
        std::fprintf(stderr, "cannot open %s\n", path.c_str());
        return false;
    }
    std::fseek(f, 0, SEEK_END);
    const long bytes = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    if (bytes < 0 || bytes % (long)sizeof(T) != 0) {
        std::fprintf(stderr, "%s: size %ld is not a multiple of %zu\n", path.c_str(), bytes,
                     sizeof(T));
        std::fclose(f);
        return false;
    }
    out.resize((size_t)bytes / sizeof(T));
    const size_t got = out.empty() ? 0 : std::fread(out.data(), sizeof(T), out.size(), f);
    std::fclose(f);
    if (got != out.size()) {
        std::fprintf(stderr, "%s: short read\n", path.c_str());
        return false;
    }
    return true;
}

bool write_bytes(const std::string &path, const void *data, size_t bytes)
{
    FILE *f = std::fopen(path.c_str(), "wb");
    if (!f) {
        std::fprintf(stderr, "cannot create %s\n", path.c_str());
        return false;
    }
    const bool ok = std::fwrite(data, 1, bytes, f) == bytes;
    std::fclose(f);
    if (!ok) std::fprintf(stderr, "%s: short write\n", path.c_str());
    return ok;
}

// device buffers released on every exit path
struct DeviceBuffers {
    std::vector<void *> ptrs;
    bool alloc(void **p, size_t bytes)
    {
        if (hipMalloc(p, bytes ? bytes : 1) != hipSuccess) return false;
        ptrs.push_back(*p);
        return true;
    }
    ~DeviceBuffers()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

}  // namespace

int main(int argc, char **argv)
{
    if (argc < 4) return usage();
    const std::string dir = argv[1];
    const int n_phase = std::atoi(argv[2]);
    const int n_mag = std::atoi(argv[3]);
    gce_opts opts;
    std::memset(&opts, 0, sizeof(opts));
    bool want_cube = false;
    int device = 0;
    for (int i = 4; i < argc; ++i) {
        const std::string a = argv[i];
        if (a == "--split") opts.precision = GCE_PRECISION_SPLIT_FP32;
        else if (a == "--phase-overlap") opts.phase_overlap = 1;
        else if (a == "--mag-overlap") opts.mag_overlap = 1;
        else if (a == "--cube") want_cube = true;
        else if (a == "--table" && i + 1 < argc) {
            const std::string v = argv[++i];
            if (v == "global") opts.table_placement = GCE_TABLE_GLOBAL;
            else if (v == "lds") opts.table_placement = GCE_TABLE_LDS;
            else return usage();
        } else if (a == "--trials-per-lane" && i + 1 < argc) opts.trials_per_lane = std::atoi(argv[++i]);
        else if (a == "--waves-per-unit" && i + 1 < argc) opts.waves_per_unit = std::atoi(argv[++i]);
        else if (a == "--refine-units" && i + 1 < argc) opts.refine_units = std::atoi(argv[++i]);
        else if (a == "--device" && i + 1 < argc) device = std::atoi(argv[++i]);
        else return usage();
    }

    std::vector<double> times, mags, periods, pdots;
    std::vector<int64_t> offsets;
    if (!read_array(dir + "/times.f64", times) || !read_array(dir + "/mags.f64", mags) ||
        !read_array(dir + "/offsets.i64", offsets) ||
        !read_array(dir + "/periods.f64", periods) || !read_array(dir + "/pdots.f64", pdots))
        return 1;
    if (offsets.size() < 2 || times.size() != mags.size() ||
        (int64_t)times.size() != offsets.back()) {
        std::fprintf(stderr, "inconsistent inputs: %zu epochs, %zu magnitudes, offsets end %lld\n",
                     times.size(), mags.size(),
                     offsets.empty() ? -1LL : (long long)offsets.back());
        return 1;
    }
    const int64_t n_curves = (int64_t)offsets.size() - 1;
    const int64_t n_p = (int64_t)periods.size(), n_pd = (int64_t)pdots.size();

    // the plan validates the shape on the host before anything touches the GPU
    gce_plan_t plan = nullptr;
    int rc = gce_plan_create(&plan, offsets.data(), n_curves, n_p, n_pd, n_phase, n_mag, &opts,
                             device);
    if (rc != GCE_OK) {
        std::fprintf(stderr, "gce_plan_create: %s\n", gce_status_string(rc));
        return 1;
    }
    const size_t cube_elems = want_cube ? (size_t)(n_curves * n_pd * n_p) : 0;
    const size_t cube_elem_bytes = opts.precision == GCE_PRECISION_FP64 ? 8 : 4;
    int status = 1;
    {
        DeviceBuffers buf;
        void *d_t = nullptr, *d_m = nullptr, *d_p = nullptr, *d_pd = nullptr;
        void *d_cube = nullptr, *d_best = nullptr;
        bool ok = buf.alloc(&d_t, times.size() * 8) && buf.alloc(&d_m, mags.size() * 8) &&
                  buf.alloc(&d_p, periods.size() * 8) && buf.alloc(&d_pd, pdots.size() * 8) &&
                  buf.alloc(&d_best, (size_t)n_curves * sizeof(gce_best_t)) &&
                  (!want_cube || buf.alloc(&d_cube, cube_elems * cube_elem_bytes));
        ok = ok && hipMemcpy(d_t, times.data(), times.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(d_m, mags.data(), mags.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(d_p, periods.data(), periods.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(d_pd, pdots.data(), pdots.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
        if (!ok) {
            std::fprintf(stderr, "device allocation or upload failed\n");
        } else {
            const auto t0 = std::chrono::steady_clock::now();
            rc = gce_plan_execute(plan, (const double *)d_t, (const double *)d_m,
                                  (const double *)d_p, (const double *)d_pd, d_cube,
                                  (gce_best_t *)d_best, nullptr);
            const hipError_t se = hipDeviceSynchronize();
            const double ms = std::chrono::duration<double, std::milli>(
                                  std::chrono::steady_clock::now() - t0).count();
            if (rc != GCE_OK || se != hipSuccess) {
                std::fprintf(stderr, "gce_plan_execute: %s\n",
                             rc != GCE_OK ? gce_status_string(rc) : hipGetErrorString(se));
            } else {
                std::vector<gce_best_t> best((size_t)n_curves);
                std::vector<char> cube(cube_elems * cube_elem_bytes);
                ok = hipMemcpy(best.data(), d_best, best.size() * sizeof(gce_best_t),
                               hipMemcpyDeviceToHost) == hipSuccess &&
                     (!want_cube || hipMemcpy(cube.data(), d_cube, cube.size(),
                                              hipMemcpyDeviceToHost) == hipSuccess);
                ok = ok && write_bytes(dir + "/best.bin", best.data(),
                                       best.size() * sizeof(gce_best_t));
                if (ok && want_cube)
                    ok = write_bytes(dir + (cube_elem_bytes == 8 ? "/cube.f64" : "/cube.f32"),
                                     cube.data(), cube.size());
                if (ok) {
                    std::printf("{\"n_curves\": %lld, \"points\": %lld, \"n_periods\": %lld, "
                                "\"n_pdots\": %lld, \"search_ms\": %.3f, \"version\": \"%s\"}\n",
                                (long long)n_curves, (long long)offsets.back(),
                                (long long)n_p, (long long)n_pd, ms, gce_version());
                    status = 0;
                } else {
                    std::fprintf(stderr, "download or file write failed\n");
                }
            }
        }
    }
    gce_plan_destroy(plan);
    return status;
}
