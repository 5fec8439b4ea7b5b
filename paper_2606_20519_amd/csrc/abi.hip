// Host runtime behind the C ABI declared in include/psdproj.h: argument
// validation, workspace layout and kernel dispatch.  No call allocates or
// prints; all device work goes on the caller's stream, and only a mixed
// psd_project with the FP64 fallback enabled and psd_project_warm (which
// reads whether its refinement was accepted) synchronise it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/psdproj.h"
#include "kernels.h"
#include "large.h"
#include "mixed.h"
#include "warm.h"

using namespace psd;

static_assert(sizeof(psd_info) == sizeof(psd_dev_info), "psd_info layout");

// Workspace of psd_project_noalloc: a fixed device array, one copy on every
// device the library runs on, held until the process ends.  Host code never
// passes `scratch` itself (its host-side name is not a device address): the
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[PSD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

bool valid_mode(int m) {
    return m == PSD_FP64_EIG || m == PSD_MIXED_BF16 || m == PSD_MIXED_FP32 || m == PSD_MIXED_BF16X3;
}

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

// Partial overlap of [a, a+na) and [b, b+nb) (identical ranges are allowed).
bool partial_overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    if (pa == pb && na == nb) return false;
    return pa < pb + nb && pb < pa + na;
}

// Bump allocator over the caller's workspace.
struct Carve {
    char *base;
    size_t used = 0;
    explicit Carve(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used = align_up(used + count * sizeof(T));
        return p;
    }
};

// Workspace of one large-block computation of order n.  Mixed modes also
// reserve, after the larger of the two paths' layouts, an svec copy of the
// input and one info record for the FP64 fallback (psd_set_mixed_fallback).
size_t large_ws_bytes(int n, int mode, int flags) {
    size_t b = large_layout(n, flags, nullptr, nullptr);
    if ((mode == PSD_MIXED_BF16 || mode == PSD_MIXED_FP32 || mode == PSD_MIXED_BF16X3) && !(flags & PSD_FLAG_SAVE)) {
        b = align_up(std::max(b, mixed_layout(n, mode, nullptr, nullptr)));
        b += align_up(sizeof(double) * (size_t)n * (size_t)n) + align_up(sizeof(psd_info));
    }
    return b;
}

bool is_mixed(int mode) { return mode == PSD_MIXED_BF16 || mode == PSD_MIXED_FP32 || mode == PSD_MIXED_BF16X3; }

int g_ns_iters = 0;  // automatic
int g_ns_corr = -1;  // automatic: 1 for BF16, 0 for FP32 and split BF16
double g_fallback_bound = 0.0;  // 0: no FP64 fallback of the mixed modes

// Marks a record written by the FP64 path as the fallback of a mixed call.
__global__ void mark_fallback_kernel(psd_dev_info *info) { info->fallback = 1; }

// Host tables reach the device as kernel arguments, copied by value at the
// launch: no staging buffer outlives the call, and a captured graph holds
// its own copy of the values.
constexpr int kArgWords = 512;
struct ArgChunk {
    uint32_t w[kArgWords];
};
__global__ void __launch_bounds__(256) upload_kernel(ArgChunk c, int nwords, uint32_t *dst) {
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = c.w[i];
}
hipError_t upload_table(void *dst, const void *src, size_t bytes, hipStream_t s) {
    const size_t words = (bytes + 3) / 4;
    const uint32_t *sw = static_cast<const uint32_t *>(src);
    for (size_t off = 0; off < words; off += kArgWords) {
        ArgChunk c;
        const int nw = (int)std::min<size_t>(kArgWords, words - off);
        std::memcpy(c.w, sw + off, sizeof(uint32_t) * nw);
        hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, s, c, nw, static_cast<uint32_t *>(dst) + off);
    }
    return hipGetLastError();
}

// Lockstep groups: blocks of one order n > 64 go through the path (FP64 or
// mixed) together, at most group_cap(n, mode) at a time (128, fewer where 128
// workspace slots would pass 4 GiB).
constexpr int kMaxGroup = 128;
constexpr size_t kGroupBytes = size_t(4) << 30;

// Workspace slot of one group member.
size_t member_bytes(int n, int mode) {
    return is_mixed(mode) ? mixed_layout(n, mode, nullptr, nullptr) : large_layout(n, 0, nullptr, nullptr);
}

int group_cap(int n, int mode) {
    return (int)std::max<size_t>(1, std::min<size_t>(kMaxGroup, kGroupBytes / member_bytes(n, mode)));
}

// The large blocks of a call split into groups (same order, in order of
// first appearance, each at most group_cap members).
std::vector<psd::GroupChunk> make_chunks(int nblocks, const int32_t *n, int mode, int max_group = 0) {
    std::vector<psd::GroupChunk> out;
    std::vector<int> done(nblocks, 0);
    for (int b = 0; b < nblocks; ++b) {
        if (n[b] <= 64 || done[b]) continue;
        const int cap = max_group > 0 ? std::min(max_group, group_cap(n[b], mode)) : group_cap(n[b], mode);
        psd::GroupChunk cur{n[b], {}};
        for (int c = b; c < nblocks; ++c) {
            if (n[c] != n[b] || done[c]) continue;
            done[c] = 1;
            cur.blocks.push_back(c);
            if ((int)cur.blocks.size() == cap) {
                out.push_back(cur);
                cur.blocks.clear();
            }
        }
        if (!cur.blocks.empty()) out.push_back(cur);
    }
    return out;
}

size_t chunk_ws_bytes(const psd::GroupChunk &c, int mode) { return c.blocks.size() * member_bytes(c.n, mode); }

// Full FP64 eigen pipeline on one block: unpack, tridiagonalise, block
// reflectors, divide and conquer.  Leaves w.lam / w.Zfinal set.
hipError_t large_eigen(LargeWs &w, const double *x, hipStream_t s) {
    hipError_t e;
    if ((e = large_init(w, s)) != hipSuccess) return e;
    if ((e = large_unpack(w, x, s)) != hipSuccess) return e;
    if ((e = large_tridiag(w, s)) != hipSuccess) return e;
    if ((e = large_compute_T(w, s)) != hipSuccess) return e;
    return large_dc(w, s);
}

// y = Pi(x) for one block of order n through the large-block path.
hipError_t large_project(int n, const double *x, double *y, void *ws, hipStream_t s, psd_dev_info *info,
                         double *saved) {
    LargeWs w;
    large_layout(n, saved ? PSD_FLAG_SAVE : 0, ws, &w);
    hipError_t e = large_eigen(w, x, s);
    if (e != hipSuccess) return e;
    if (saved) {
        if ((e = large_select(w, info, s, true)) != hipSuccess) return e;
        if ((e = large_backtransform(w, n, s)) != hipSuccess) return e;
        if ((e = large_save(w, saved, s)) != hipSuccess) return e;
        return large_reconstruct(w, x, y, n, s);
    }
    if ((e = large_select(w, info, s, false)) != hipSuccess) return e;
    if ((e = large_backtransform(w, w.kmax, s)) != hipSuccess) return e;
    return large_reconstruct(w, x, y, w.kmax, s);
}

// Lockstep group: nmem FP64 blocks of order n, member b reading x + ioff[b]
// and writing y + ioff[b] (device table), info record infos[infoidx[b]],
// workspace slot b at ws + b * slot bytes.  Every launch of the path covers
// all members, so one group costs the launches of one block.
hipError_t large_project_group(int n, int nmem, const double *x, double *y, const int64_t *ioff, const int *infoidx,
                               psd_dev_info *infos, void *ws, hipStream_t s) {
    LargeWs w;
    const size_t slot = large_layout(n, 0, ws, &w);
    w.nmem = nmem;
    w.zs = (int64_t)slot;
    w.ioff = ioff;
    w.infoidx = infoidx;
    hipError_t e = large_eigen(w, x, s);
    if (e != hipSuccess) return e;
    if ((e = large_select(w, infos, s, false)) != hipSuccess) return e;
    if ((e = large_backtransform(w, w.kmax, s)) != hipSuccess) return e;
    return large_reconstruct(w, x, y, w.kmax, s);
}

// A lockstep group in either precision form.
hipError_t project_group(int n, int nmem, psd_mode mode, const double *x, double *y, const int64_t *ioff,
                         const int *infoidx, psd_dev_info *infos, void *ws, hipStream_t s,
                         int ns_big = NS_BIG_DEFAULT) {
    if (!is_mixed(mode)) return large_project_group(n, nmem, x, y, ioff, infoidx, infos, ws, s);
    MixedWs w;
    const size_t slot = mixed_layout(n, mode, ws, &w);
    w.ns_big = ns_big;
    w.nmem = nmem;
    w.zs = (int64_t)slot;
    w.ioff = ioff;
    w.infoidx = infoidx;
    return mixed_project(w, mode, x, y, infos, g_ns_iters, g_ns_corr, s);
}

psd_status status_of(hipError_t e) { return e == hipSuccess ? PSD_OK : PSD_EDEVICE; }

// Device address of `scratch` on the current device (looked up on the first
// call made with that device current, then cached).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}


// Mixed projection of one block with the FP64 fallback: the record of the
// mixed run goes to the workspace, the stream is synchronised, and when the
// run reports a failed status or an error estimate above the bound (or not a
// number) the block is projected again by the FP64 path, whose record is
// marked fallback = 1.  A non-finite input is not retried (FP64 would fail
// the same way).  The input is copied first when the call is in place.
hipError_t mixed_with_fallback(int n, const double *x, double *y, psd_mode mode, void *ws, hipStream_t s,
                               psd_dev_info *info) {
    MixedWs w;
    const size_t base = align_up(std::max(large_layout(n, 0, nullptr, nullptr), mixed_layout(n, mode, nullptr, nullptr)));
    mixed_layout(n, mode, ws, &w);
    const size_t nb = sizeof(double) * (size_t)n * (size_t)n;
    double *xcopy = reinterpret_cast<double *>(static_cast<char *>(ws) + base);
    psd_dev_info *winfo = reinterpret_cast<psd_dev_info *>(static_cast<char *>(ws) + base + align_up(nb));
    hipError_t e;
    const double *xin = x;
    if (x == y) {
        if ((e = hipMemcpyAsync(xcopy, x, nb, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
        xin = xcopy;
    }
    if ((e = mixed_project(w, mode, x, y, winfo, g_ns_iters, g_ns_corr, s)) != hipSuccess) return e;
    psd_dev_info h{};
    if ((e = hipMemcpyAsync(&h, winfo, sizeof(h), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const bool accept = h.status == PSD_ENONFINITE || (h.status == PSD_OK && h.est_rel_err <= g_fallback_bound);
    if (accept) return info ? hipMemcpyAsync(info, winfo, sizeof(h), hipMemcpyDefault, s) : hipSuccess;
    if ((e = large_project(n, xin, y, ws, s, info, nullptr)) != hipSuccess) return e;
    if (info) hipLaunchKernelGGL(mark_fallback_kernel, dim3(1), dim3(1), 0, s, info);
    return hipGetLastError();
}

// One block of order n > 64: the mixed path for mixed modes, else FP64.
hipError_t project_block(int n, const double *x, double *y, psd_mode mode, void *ws, hipStream_t s,
                         psd_dev_info *info, double *saved, bool allow_fallback = false) {
    if (is_mixed(mode) && !saved) {
        if (allow_fallback && g_fallback_bound > 0.0) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
                return mixed_with_fallback(n, x, y, mode, ws, s, info);
        }
        MixedWs w;
        mixed_layout(n, mode, ws, &w);
        return mixed_project(w, mode, x, y, info, g_ns_iters, g_ns_corr, s);
    }
    return large_project(n, x, y, ws, s, info, saved);
}

}  // namespace

namespace psd {

std::vector<GroupChunk> group_chunks(int nblocks, const int32_t *n, int mode, int max_group) {
    return make_chunks(nblocks, n, mode, max_group);
}
size_t group_ws_bytes(const GroupChunk &c, int mode) { return chunk_ws_bytes(c, mode); }
hipError_t project_group_ext(int n, int nmem, psd_mode mode, const double *x, double *y, const int64_t *ioff,
                             const int *infoidx, psd_dev_info *infos, void *ws, hipStream_t s, int ns_big) {
    return project_group(n, nmem, mode, x, y, ioff, infoidx, infos, ws, s, ns_big);
}

hipError_t prepare_kernel_attributes() {
    hipError_t e = small_prepare();
    if (e != hipSuccess) return e;
    return dc_prepare();
}

}  // namespace psd

extern "C" {

const char *psd_version(void) { return "psdproj 0.1 (gfx950)"; }

psd_status psd_set_ns_iterations(int32_t iters, int32_t corrections) {
    if (iters < 0 || iters > 200 || corrections < -1 || corrections > 8) return PSD_EINVAL;
    g_ns_iters = iters;
    g_ns_corr = corrections;
    return PSD_OK;
}

psd_status psd_set_mixed_fallback(double max_rel_err) {
    if (!(max_rel_err >= 0.0)) return PSD_EINVAL;
    g_fallback_bound = max_rel_err;
    return PSD_OK;
}

const char *psd_status_string(psd_status s) {
    switch (s) {
        case PSD_OK: return "ok";
        case PSD_EINVAL: return "invalid argument";
        case PSD_EWORKSPACE: return "workspace too small";
        case PSD_ENOMEM: return "out of memory";
        case PSD_ENONFINITE: return "non-finite input";
        case PSD_ENOCONV: return "iteration did not converge";
        case PSD_EDEVICE: return "HIP runtime error";
        case PSD_EUNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

size_t psd_saved_size(int32_t n) {
    if (n < 1) return 0;
    return sizeof(double) * ((size_t)n + 2 * (size_t)n * (size_t)n);
}

psd_status psd_workspace_size(int32_t nblocks, const int32_t *n, psd_mode mode, int32_t flags,
                              size_t *bytes) {
    if (nblocks < 1 || !n || !bytes || !valid_mode(mode)) return PSD_EINVAL;
    if ((flags & PSD_FLAG_WARM) && (nblocks != 1 || mode != PSD_FP64_EIG)) return PSD_EINVAL;
    size_t small = 0, large = 0;
    for (int b = 0; b < nblocks; ++b) {
        if (n[b] < 1) return PSD_EINVAL;
        if (n[b] <= 64 && !(flags & (PSD_FLAG_SAVE | PSD_FLAG_WARM))) ++small;
        else large = std::max(large, large_ws_bytes(n[b], mode, flags | (flags & PSD_FLAG_WARM ? PSD_FLAG_SAVE : 0)));
        // the refinement and, when it is not accepted, the cold path with
        // the saved pair share the workspace one after the other
        if (flags & PSD_FLAG_WARM) large = std::max(large, warm_layout(n[b], nullptr, nullptr));
    }
    size_t tables = 0;
    if (nblocks > 1 && !(flags & PSD_FLAG_SAVE)) {
        // lockstep groups: member slots side by side, plus the offset and
        // info-index tables
        for (const auto &c : make_chunks(nblocks, n, mode)) large = std::max(large, chunk_ws_bytes(c, mode));
        tables = align_up(sizeof(int64_t) * nblocks) + align_up(sizeof(int) * nblocks);
    }
    *bytes = align_up(small * sizeof(SmallJob)) + tables + large + kAlign;
    return PSD_OK;
}

psd_status psd_project(int32_t n, const double *x, double *y, psd_mode mode, void *ws,
                       size_t ws_bytes, void *stream, psd_info *info, double *saved) {
    if (n < 1 || !x || !y || !valid_mode(mode)) return PSD_EINVAL;
    if (!aligned8(x) || !aligned8(y) || (saved && !aligned8(saved))) return PSD_EINVAL;
    const size_t nb = sizeof(double) * (size_t)n * (size_t)n;
    if (partial_overlap(x, nb, y, nb)) return PSD_EINVAL;
    size_t need = 0;
    psd_status st = psd_workspace_size(1, &n, mode, saved ? PSD_FLAG_SAVE : 0, &need);
    if (st != PSD_OK) return st;
    if (ws_bytes < need || (need && !ws)) return PSD_EWORKSPACE;
    if (ws && (reinterpret_cast<uintptr_t>(ws) % kAlign)) return PSD_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    psd_dev_info *dinfo = reinterpret_cast<psd_dev_info *>(info);
    if (n <= 64) {
        SmallJob job{0, 0, n, 0};
        return status_of(launch_small_one(job, x, y, dinfo, saved, s));
    }
    return status_of(project_block(n, x, y, mode, ws, s, dinfo, saved, true));
}

psd_status psd_project_warm(int32_t n, const double *x, double *y, const double *saved_prev,
                            double *saved_out, void *ws, size_t ws_bytes, void *stream, psd_info *info) {
    if (n < 1 || !x || !y || !saved_prev || !saved_out) return PSD_EINVAL;
    if (!aligned8(x) || !aligned8(y) || !aligned8(saved_prev) || !aligned8(saved_out)) return PSD_EINVAL;
    const size_t nb = sizeof(double) * (size_t)n * (size_t)n;
    const size_t sb = psd_saved_size(n);
    if (partial_overlap(x, nb, y, nb) || partial_overlap(saved_prev, sb, saved_out, sb)) return PSD_EINVAL;
    if (partial_overlap(x, nb, saved_out, sb) || partial_overlap(x, nb, saved_prev, sb) ||
        partial_overlap(y, nb, saved_out, sb) || partial_overlap(y, nb, saved_prev, sb))
        return PSD_EINVAL;
    size_t need = 0;
    psd_status st = psd_workspace_size(1, &n, PSD_FP64_EIG, PSD_FLAG_WARM, &need);
    if (st != PSD_OK) return st;
    if (ws_bytes < need || !ws) return PSD_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return PSD_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return PSD_EDEVICE;
    if (cs != hipStreamCaptureStatusNone) return PSD_EUNSUPPORTED;  // the host reads the outcome
    psd_dev_info *dinfo = reinterpret_cast<psd_dev_info *>(info);
    WarmWs w;
    warm_layout(n, ws, &w);
    if (warm_refine(w, x, saved_prev, y, saved_out, dinfo, s) != hipSuccess) return PSD_EDEVICE;
    int reject = 1;
    if (hipMemcpyAsync(&reject, w.flags + WF_REJECT, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        return PSD_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return PSD_EDEVICE;
    if (!reject) return PSD_OK;
    // not accepted: the cold FP64 path (x is intact: y and saved_out were not written)
    hipError_t e;
    if (n <= 64) {
        SmallJob job{0, 0, n, 0};
        e = launch_small_one(job, x, y, dinfo, saved_out, s);
    } else {
        e = large_project(n, x, y, ws, s, dinfo, saved_out);
    }
    if (e != hipSuccess) return PSD_EDEVICE;
    if (dinfo) hipLaunchKernelGGL(mark_fallback_kernel, dim3(1), dim3(1), 0, s, dinfo);
    return status_of(hipGetLastError());
}

psd_status psd_project_noalloc(int32_t n, const double *x, double *y, psd_mode mode, void *stream,
                               psd_info *info) {
    if (n < 1 || !x || !y || !valid_mode(mode)) return PSD_EINVAL;
    if (!aligned8(x) || !aligned8(y)) return PSD_EINVAL;
    const size_t nb = sizeof(double) * (size_t)n * (size_t)n;
    if (partial_overlap(x, nb, y, nb)) return PSD_EINVAL;
    size_t need = 0;
    psd_status st = psd_workspace_size(1, &n, mode, 0, &need);
    if (st != PSD_OK) return st;
    if (need > PSD_NOALLOC_SCRATCH_BYTES) return PSD_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    psd_dev_info *dinfo = reinterpret_cast<psd_dev_info *>(info);
    if (n <= 64) {
        SmallJob job{0, 0, n, 0};
        return status_of(launch_small_one(job, x, y, dinfo, nullptr, s));
    }
    void *ws = nullptr;
    if (scratch_address(&ws) != hipSuccess) return PSD_EDEVICE;
    return status_of(project_block(n, x, y, mode, ws, s, dinfo, nullptr, false));
}

psd_status psd_project_batched(int32_t nblocks, const int32_t *n, const double *x, double *y,
                               psd_mode mode, void *ws, size_t ws_bytes, void *stream,
                               psd_info *infos) {
    if (nblocks < 1 || !n || !x || !y || !valid_mode(mode)) return PSD_EINVAL;
    if (!aligned8(x) || !aligned8(y)) return PSD_EINVAL;
    size_t total = 0;
    for (int b = 0; b < nblocks; ++b) {
        if (n[b] < 1) return PSD_EINVAL;
        total += (size_t)n[b] * (size_t)n[b];
    }
    if (partial_overlap(x, total * sizeof(double), y, total * sizeof(double))) return PSD_EINVAL;
    size_t need = 0;
    psd_status st = psd_workspace_size(nblocks, n, mode, 0, &need);
    if (st != PSD_OK) return st;
    if (ws_bytes < need || !ws) return PSD_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return PSD_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);

    std::vector<SmallJob> small, small64;  // orders <= 32 first, then 33 .. 64
    std::vector<int> large;
    std::vector<int64_t> boff(nblocks);
    int64_t off = 0;
    for (int b = 0; b < nblocks; ++b) {
        boff[b] = off;
        if (n[b] <= 32) small.push_back(SmallJob{off, 0, n[b], b});
        else if (n[b] <= 64) small64.push_back(SmallJob{off, 0, n[b], b});
        else large.push_back(b);
        off += (int64_t)n[b] * n[b];
    }
    const int n32 = (int)small.size();
    int nt32 = 0;
    for (const SmallJob &j : small) nt32 = std::max(nt32, small32_threads(j.n));
    small.insert(small.end(), small64.begin(), small64.end());
    psd_dev_info *dinfos = reinterpret_cast<psd_dev_info *>(infos);
    const bool grouped = nblocks > 1;
    Carve cv(ws);
    SmallJob *djobs = cv.take<SmallJob>(small.size());
    const size_t ioff_at = cv.used;
    int64_t *dioff = grouped ? cv.take<int64_t>(nblocks) : nullptr;
    const size_t idx_at = cv.used;
    int *didx = grouped ? cv.take<int>(nblocks) : nullptr;
    void *lws = cv.base + cv.used;
    std::vector<GroupChunk> chunks;
    if (grouped) chunks = make_chunks(nblocks, n, mode);
    // The job and group tables, uploaded as kernel arguments.
    if (cv.used > 0 && (!small.empty() || grouped)) {
        std::vector<char> host((cv.used + 3) / 4 * 4, 0);
        if (!small.empty()) std::memcpy(host.data(), small.data(), small.size() * sizeof(SmallJob));
        if (grouped) {
            int64_t *hoff = reinterpret_cast<int64_t *>(host.data() + ioff_at);
            int *hidx = reinterpret_cast<int *>(host.data() + idx_at);
            int pos = 0;
            for (const auto &c : chunks)
                for (int b : c.blocks) {
                    hoff[pos] = boff[b];
                    hidx[pos] = b;
                    ++pos;
                }
        }
        hipError_t e = upload_table(ws, host.data(), cv.used, s);
        if (e != hipSuccess) return PSD_EDEVICE;
    }
    if (grouped) {
        int pos = 0;
        for (const auto &c : chunks) {
            const int cnt = (int)c.blocks.size();
            hipError_t e = project_group(c.n, cnt, mode, x, y, dioff + pos, didx + pos, dinfos, lws, s);
            if (e != hipSuccess) return PSD_EDEVICE;
            pos += cnt;
        }
    } else {
        // large blocks one after another on the stream, sharing one workspace
        for (int b : large) {
            psd_dev_info *inf = dinfos ? dinfos + b : nullptr;
            hipError_t e = project_block(n[b], x + boff[b], y + boff[b], mode, lws, s, inf, nullptr);
            if (e != hipSuccess) return PSD_EDEVICE;
        }
    }
    if (!small.empty()) {
        hipError_t e = launch_small(djobs, (int)small.size(), n32, nt32, x, y, dinfos, nullptr, s);
        if (e != hipSuccess) return PSD_EDEVICE;
    }
    return PSD_OK;
}

psd_status psd_project_vjp(int32_t n, const double *x, const double *saved, const double *gy,
                           double *gx, psd_mode mode, void *ws, size_t ws_bytes, void *stream) {
    if (n < 1 || (!x && !saved) || !gy || !gx || !valid_mode(mode)) return PSD_EINVAL;
    if ((x && !aligned8(x)) || (saved && !aligned8(saved)) || !aligned8(gy) || !aligned8(gx)) return PSD_EINVAL;
    const size_t nb = sizeof(double) * (size_t)n * (size_t)n;
    if (partial_overlap(gy, nb, gx, nb)) return PSD_EINVAL;
    size_t need = 0;
    psd_status st = psd_workspace_size(1, &n, mode, PSD_FLAG_SAVE, &need);
    if (st != PSD_OK) return st;
    if (ws_bytes < need || !ws) return PSD_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return PSD_EINVAL;
    // The derivative is the Daleckii-Krein formula on the FP64 eigen-pair in
    // every mode (the Newton-Schulz form yields no eigenvectors).
    hipStream_t s = static_cast<hipStream_t>(stream);
    LargeWs w;
    large_layout(n, PSD_FLAG_SAVE, ws, &w);
    hipError_t e;
    if (saved) {
        if ((e = large_init(w, s)) != hipSuccess) return PSD_EDEVICE;
        if ((e = large_load_saved(w, saved, s)) != hipSuccess) return PSD_EDEVICE;
        w.lam = w.D0;
    } else {
        if ((e = large_eigen(w, x, s)) != hipSuccess) return PSD_EDEVICE;
        if ((e = large_select(w, nullptr, s, true)) != hipSuccess) return PSD_EDEVICE;
        if ((e = large_backtransform(w, n, s)) != hipSuccess) return PSD_EDEVICE;
    }
    return status_of(large_vjp_from_v(w, gy, gx, s));
}

}  // extern "C"
