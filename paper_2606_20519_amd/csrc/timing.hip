// HIP-event timing of one kernel family (see psd_timing_start in psdproj.h).
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/psdproj.h"
#include "timing.h"

namespace psd {

namespace {
struct TimingState {
    int family = 0;
    int max = 0;
    int used = 0;
    std::vector<hipEvent_t> ev;
    std::vector<double> work;
};
TimingState g_timing;
}  // namespace

int timing_begin(int family, hipStream_t st) {
    TimingState &T = g_timing;
    if (T.family != family || T.used >= T.max) return -1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
    const int slot = T.used++;
    if (hipEventRecord(T.ev[2 * slot], st) != hipSuccess) return -1;
    return slot;
}

void timing_end(int slot, hipStream_t st, double work) {
    if (slot < 0) return;
    TimingState &T = g_timing;
    (void)hipEventRecord(T.ev[2 * slot + 1], st);
    T.work[slot] = work;
}

}  // namespace psd

extern "C" {

psd_status psd_timing_start(int32_t family, int32_t max_launches) {
    using namespace psd;
    TimingState &T = g_timing;
    if (family < KF_HEMV || family > KF_WSTEP || max_launches < 1 || T.family != 0)
        return PSD_EINVAL;
    T.ev.assign(2 * (size_t)max_launches, nullptr);
    for (auto &e : T.ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return PSD_EDEVICE;
    T.work.assign(max_launches, 0.0);
    T.max = max_launches;
    T.used = 0;
    T.family = family;
    return PSD_OK;
}

psd_status psd_timing_stop(double *ms, int32_t *launches, double *work) {
    using namespace psd;
    TimingState &T = g_timing;
    if (T.family == 0) return PSD_EINVAL;
    double total = 0.0, wk = 0.0;
    psd_status st = PSD_OK;
    for (int i = 0; i < T.used; ++i) {
        float t = 0.f;
        if (hipEventSynchronize(T.ev[2 * i + 1]) != hipSuccess ||
            hipEventElapsedTime(&t, T.ev[2 * i], T.ev[2 * i + 1]) != hipSuccess) {
            st = PSD_EDEVICE;
            continue;
        }
        total += t;
        wk += T.work[i];
    }
    if (ms) *ms = total;
    if (launches) *launches = T.used;
    if (work) *work = wk;
    for (auto &e : T.ev) (void)hipEventDestroy(e);
    T.ev.clear();
    T.work.clear();
    T.family = 0;
    T.used = T.max = 0;
    return st;
}

}  // extern "C"
