// Host-side memory check of the runtime (test infrastructure): linked by
// tests/test_host_asan.py against the library's objects built with the
// address sanitizer on the host code only, and run without a GPU.  It
// drives every entry point along the paths that end on the host: workspace
// and layout arithmetic for single blocks, cones and SCS settings, argument
// validation, and the error paths of calls whose first device call fails
// (plan creation, timing).  Prints "ok" when every status is the expected one.
#include <cstdio>
#include <vector>

#include "psdproj.h"

static int bad = 0;
static void expect(bool ok, const char *what) {
    if (!ok) {
        std::printf("unexpected: %s\n", what);
        ++bad;
    }
}

int main() {
    size_t b = 0;
    for (int mode = 0; mode < 4; ++mode)
        for (int n : {1, 2, 16, 32, 33, 64, 65, 120, 121, 625, 1296, 2401, 4096, 4200}) {
            expect(psd_workspace_size(1, &n, (psd_mode)mode, 0, &b) == PSD_OK, "workspace");
            expect(psd_workspace_size(1, &n, (psd_mode)mode, PSD_FLAG_SAVE, &b) == PSD_OK, "workspace save");
            expect(psd_workspace_size(1, &n, (psd_mode)mode, PSD_FLAG_WARM, &b) == (mode == 0 ? PSD_OK : PSD_EINVAL),
                   "workspace warm");
        }
    for (int d = 2; d <= 8; ++d) {
        std::vector<int> cone;
        for (int i = 0; i < 32; ++i) {
            cone.push_back(d * d * d * d);
            for (int k = 0; k < 8; ++k) cone.push_back(d * d);
        }
        for (int mode = 0; mode < 4; ++mode)
            expect(psd_workspace_size((int)cone.size(), cone.data(), (psd_mode)mode, 0, &b) == PSD_OK, "cone");
        int64_t nx = 0, ny = 0;
        expect(psd_affine_dims(d, &nx, &ny) == PSD_OK, "affine dims");
        expect(psd_affine_workspace_size(d, &b) == PSD_OK, "affine workspace");
        for (int aa : {0, 5, 16})
            for (int warm : {0, 1}) {
                psd_scs_settings s{};
                s.d = d; s.max_iters = 10; s.check_every = 1; s.mixed_iters = 0; s.mixed_mode = 2;
                s.normalize = 1; s.warm_start = 0; s.anderson = aa; s.eps = 1e-5; s.alpha = 1.5;
                s.mixed_switch = 0.0; s.warm_proj = warm;
                expect(psd_scs_workspace_size(&s, &b) == PSD_OK, "scs workspace");
                expect(psd_scs_workspace_size_batched(&s, 3, &b) == (warm ? PSD_EINVAL : PSD_OK), "scs batched");
            }
    }
    // validation before any device call
    double *fx = reinterpret_cast<double *>(0x10000), *fy = reinterpret_cast<double *>(0x10000 + 8 * 256);
    void *ws = reinterpret_cast<void *>(0x100000);
    expect(psd_project(0, fx, fy, PSD_FP64_EIG, ws, 1 << 20, nullptr, nullptr, nullptr) == PSD_EINVAL, "n = 0");
    expect(psd_project(16, fx, fy, PSD_FP64_EIG, ws, 0, nullptr, nullptr, nullptr) == PSD_EWORKSPACE, "ws");
    int sizes[3] = {4, 0, 9};
    expect(psd_project_batched(3, sizes, fx, fy, PSD_FP64_EIG, ws, 1 << 20, nullptr, nullptr) == PSD_EINVAL,
           "batched");
    double *sp = reinterpret_cast<double *>(0x200000), *so = reinterpret_cast<double *>(0x400000);
    expect(psd_project_warm(16, fx, fy, sp, so, ws, 0, nullptr, nullptr) == PSD_EWORKSPACE, "warm ws");
    expect(psd_project_warm(16, fx, fy, nullptr, so, ws, 1 << 30, nullptr, nullptr) == PSD_EINVAL, "warm null");
    expect(psd_project_vjp(16, nullptr, nullptr, fx, fy, PSD_FP64_EIG, ws, 1 << 20, nullptr) == PSD_EINVAL, "vjp");
    expect(psd_set_ns_iterations(-1, 0) == PSD_EINVAL && psd_set_mixed_fallback(-1.0) == PSD_EINVAL, "setters");
    for (int st = 0; st < 8; ++st) expect(psd_status_string((psd_status)st) != nullptr, "status string");
    // calls whose first device call fails without a GPU: their cleanup paths
    std::vector<int> cone;
    for (int i = 0; i < 4; ++i) {
        cone.push_back(625);
        for (int k = 0; k < 8; ++k) cone.push_back(25);
    }
    psd_plan plan = nullptr;
    const psd_status pc = psd_plan_create((int)cone.size(), cone.data(), PSD_FP64_EIG, 0, &plan);
    if (pc == PSD_OK) psd_plan_destroy(plan);
    expect(pc == PSD_OK || pc == PSD_EDEVICE, "plan create");
    if (psd_timing_start(1, 16) == PSD_OK) {
        double ms = 0.0, work = 0.0;
        int32_t launches = 0;
        psd_timing_stop(&ms, &launches, &work);
    }
    if (bad) {
        std::printf("%d unexpected statuses\n", bad);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
