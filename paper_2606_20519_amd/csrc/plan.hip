// Plans: the blocks of one SCS cone (App. D.1: the cone is a product of PSD
// blocks; for the see-saw's process step, the d^4 x d^4 W blocks, and for the
// batched workload also the d^2 x d^2 instrument Choi blocks) projected by a
// single hipGraph launch.
//
// The graph is captured on a stream the plan owns: a fork event, the
// whole-block LDS kernel for every block of order <= 64 (one workgroup per
// block), the large-block jobs spread round-robin over K side streams (each
// with its own workspace slot, so K jobs are in flight at once), and a join.
// A job is a lockstep group of same-order blocks (every launch covers all its
// members), in FP64 or mixed mode.  Executing a plan whose buffers were already captured is one
// hipGraphLaunch on the caller's stream.  K, the group size and, for BF16
// plans with blocks of padded order 1024..2047, the tile form of the
// Newton-Schulz product (64x64, or 128x128 from padded order 1024 on) are
// chosen by psd_plan_tune: it replays the graph for each candidate, keeps the
// fastest and records it in a small JSON-lines cache (PSD_TUNE_CACHE, default
// ./psdproj_tune.jsonl) keyed by the device architecture, the mode and the
// block sizes; psd_plan_create reads that cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/psdproj.h"
#include "kernels.h"
#include "large.h"
#include "mixed.h"

namespace psd {
// defined in abi.hip
hipError_t prepare_kernel_attributes();
}  // namespace psd

using namespace psd;

namespace {

constexpr int kMaxConcurrency = 32;
constexpr int kMaxGraphs = 8;  // captured (x, y, ws, infos) sets kept per plan
// Longest run of captured launches one stream of a plan may carry.  The
// longest captures known to run carry about 18 000 launches per stream (the
// FP64 d = 8 cone at concurrency 4: two lockstep groups of order 4096 a
// stream; the d = 7 cone at concurrency 1: 16 000); a tune of the d = 8 cone
// that also tried concurrency 2 and 1 (36 000 and 72 000 launches on one
// stream) ended the process with a segmentation fault whose cause was not
// established, so longer chains are not captured.
constexpr long kMaxChain = 20000;

struct GraphEntry {
    const double *x;
    double *y;
    void *ws;
    psd_info *infos;
    int K;
    int group;
    int ns_big;
    hipGraphExec_t exec;
};

std::string tune_key(const std::vector<int> &n, int mode) {
    std::string k = "gfx950:mode" + std::to_string(mode) + ":";
    for (size_t i = 0; i < n.size(); ++i) k += (i ? "," : "") + std::to_string(n[i]);
    return k;
}

const char *tune_path() {
    const char *p = std::getenv("PSD_TUNE_CACHE");
    return (p && *p) ? p : "psdproj_tune.jsonl";
}

// Last recorded concurrency, group size and Newton-Schulz tile threshold
// for `key` (0 where none).
void tune_lookup(const std::string &key, int *K, int *group, int *ns_big) {
    *K = 0;
    *group = 0;
    *ns_big = 0;
    FILE *f = std::fopen(tune_path(), "r");
    if (!f) return;
    char line[1 << 14];
    const std::string pat = "\"key\": \"" + key + "\"";
    while (std::fgets(line, sizeof line, f)) {
        if (!std::strstr(line, pat.c_str())) continue;
        const char *c = std::strstr(line, "\"concurrency\": ");
        const char *g = std::strstr(line, "\"group\": ");
        const char *b = std::strstr(line, "\"ns_big\": ");
        *K = c ? std::atoi(c + 15) : 0;
        *group = g ? std::atoi(g + 9) : 0;
        *ns_big = b ? std::atoi(b + 10) : 0;
    }
    std::fclose(f);
}

void tune_record(const std::string &key, int K, int group, int ns_big, double ms) {
    FILE *f = std::fopen(tune_path(), "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"concurrency\": %d, \"group\": %d, \"ns_big\": %d, \"ms\": %.6f}\n",
                 key.c_str(), K, group, ns_big, ms);
    std::fclose(f);
}

}  // namespace

struct psd_plan_s {
    std::vector<int> n;
    std::vector<int64_t> off;
    psd_mode mode;
    int K = 1;
    int nlarge = 0;
    size_t slot_bytes = 0;
    std::vector<SmallJob> small;     // orders <= 32 first (n32 of them), then 33 .. 64
    int n32 = 0, nt32 = 0;
    SmallJob *dsmall = nullptr;
    std::vector<GroupChunk> chunks;  // jobs: lockstep groups
    int group = 0;                   // members per group at most (0: the memory-derived limit)
    int ns_big = NS_BIG_DEFAULT;     // padded order from which BF16 products use 128x128 tiles
    int64_t *dioff = nullptr;        // member svec offsets, chunk after chunk
    int *didx = nullptr;             // member block indices
    hipStream_t cap = nullptr;
    hipStream_t side[kMaxConcurrency] = {};
    hipEvent_t fork = nullptr, join[kMaxConcurrency] = {};
    std::vector<GraphEntry> graphs;
};

namespace {

hipError_t capture(psd_plan_s *p, const double *x, double *y, void *ws, psd_info *infos, int K,
                   hipGraphExec_t *out) {
    hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t err = hipSuccess;
    auto chk = [&](hipError_t r) { if (err == hipSuccess && r != hipSuccess) err = r; };
    const bool fork = !p->chunks.empty();  // only small blocks: one kernel node, no fork/join
    if (fork) {
        chk(hipEventRecord(p->fork, p->cap));
        for (int i = 0; i < K; ++i) chk(hipStreamWaitEvent(p->side[i], p->fork, 0));
    }
    psd_dev_info *di = reinterpret_cast<psd_dev_info *>(infos);
    if (!p->small.empty()) chk(launch_small(p->dsmall, (int)p->small.size(), p->n32, p->nt32, x, y, di, nullptr, p->cap));
    int pos = 0;
    for (size_t ci = 0; ci < p->chunks.size(); ++ci) {
        const int slot = (int)(ci % K), cnt = (int)p->chunks[ci].blocks.size();
        char *wsl = static_cast<char *>(ws) + (size_t)slot * p->slot_bytes;
        chk(project_group_ext(p->chunks[ci].n, cnt, p->mode, x, y, p->dioff + pos, p->didx + pos, di, wsl,
                              p->side[slot], p->ns_big));
        pos += cnt;
    }
    for (int i = 0; fork && i < K; ++i) {
        chk(hipEventRecord(p->join[i], p->side[i]));
        chk(hipStreamWaitEvent(p->cap, p->join[i], 0));
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap, &g);
    if (err == hipSuccess) err = e;
    if (err == hipSuccess) err = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return err;
}

hipGraphExec_t find_graph(psd_plan_s *p, const double *x, double *y, void *ws, psd_info *infos, int K) {
    for (auto &g : p->graphs)
        if (g.x == x && g.y == y && g.ws == ws && g.infos == infos && g.K == K && g.group == p->group &&
            g.ns_big == p->ns_big)
            return g.exec;
    return nullptr;
}

// (Re)split the large blocks into lockstep groups of at most `group`
// members (0: the memory-derived limit) and refill the device tables, whose
// size (one entry per large block) does not depend on the split.
bool set_jobs(psd_plan_s *p, int group) {
    p->group = group;
    p->chunks = group_chunks((int)p->n.size(), p->n.data(), p->mode, group);
    p->nlarge = (int)p->chunks.size();
    p->slot_bytes = 0;
    for (const auto &c : p->chunks) p->slot_bytes = std::max(p->slot_bytes, group_ws_bytes(c, p->mode));
    p->slot_bytes = (p->slot_bytes + 255) / 256 * 256;
    if (p->chunks.empty()) return true;
    std::vector<int64_t> hoff;
    std::vector<int> hidx;
    for (const auto &c : p->chunks)
        for (int b : c.blocks) {
            hoff.push_back(p->off[b]);
            hidx.push_back(b);
        }
    if (!p->dioff &&
        (hipMalloc(&p->dioff, hoff.size() * sizeof(int64_t)) != hipSuccess ||
         hipMalloc(&p->didx, hidx.size() * sizeof(int)) != hipSuccess))
        return false;
    return hipMemcpy(p->dioff, hoff.data(), hoff.size() * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(p->didx, hidx.data(), hidx.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
}

// Launches of one lockstep group of order n (captured graph nodes): the FP64
// path launches two kernels per column of the reduction, one GEMM and one
// norm per panel, and a few hundred for the rest; the mixed forms a few
// hundred in all.
long group_launches(int n, int mode) {
    if (n <= 64) return 0;
    return mode == PSD_FP64_EIG ? 2L * n + n / 8 + 300 : 400;
}

// Launches on the busiest stream when the jobs go round-robin over K streams.
long longest_chain(const psd_plan_s *p, int K) {
    std::vector<long> per(std::max(1, K), 0);
    for (size_t ci = 0; ci < p->chunks.size(); ++ci)
        per[ci % per.size()] += group_launches(p->chunks[ci].n, p->mode);
    return *std::max_element(per.begin(), per.end());
}

// Largest group of the current split.
int max_members(const psd_plan_s *p) {
    size_t m = 0;
    for (const auto &c : p->chunks) m = std::max(m, c.blocks.size());
    return (int)m;
}

}  // namespace

extern "C" {

psd_status psd_plan_create(int32_t nblocks, const int32_t *n, psd_mode mode, int32_t concurrency,
                           psd_plan *plan) {
    if (nblocks < 1 || !n || !plan || concurrency < 0 || concurrency > kMaxConcurrency) return PSD_EINVAL;
    if (mode != PSD_FP64_EIG && mode != PSD_MIXED_BF16 && mode != PSD_MIXED_FP32 && mode != PSD_MIXED_BF16X3)
        return PSD_EINVAL;
    psd_plan_s *p = new (std::nothrow) psd_plan_s();
    if (!p) return PSD_ENOMEM;
    p->mode = mode;
    int64_t off = 0;
    std::vector<SmallJob> small64;
    for (int b = 0; b < nblocks; ++b) {
        if (n[b] < 1) { delete p; return PSD_EINVAL; }
        p->n.push_back(n[b]);
        p->off.push_back(off);
        if (n[b] <= 32) p->small.push_back(SmallJob{off, 0, n[b], b});
        else if (n[b] <= 64) small64.push_back(SmallJob{off, 0, n[b], b});
        off += (int64_t)n[b] * n[b];
    }
    p->n32 = (int)p->small.size();
    for (const SmallJob &j : p->small) p->nt32 = std::max(p->nt32, small32_threads(j.n));
    p->small.insert(p->small.end(), small64.begin(), small64.end());
    // jobs are lockstep groups; concurrency and group size from the cache
    int K = concurrency, group = 0;
    {
        int Kc = 0, gc = 0, bc = 0;
        tune_lookup(tune_key(p->n, mode), &Kc, &gc, &bc);
        if (K == 0) K = Kc;
        group = gc;
        if (bc == NS_BIG_MIN || bc == NS_BIG_DEFAULT) p->ns_big = bc;
    }
    if (K == 0) K = 4;
    bool ok = set_jobs(p, group);
    p->K = std::max(1, std::min(K, std::max(1, p->nlarge)));
    // enough streams that no stream carries more than kMaxChain launches
    while (p->K < std::min(kMaxConcurrency, p->nlarge) && longest_chain(p, p->K) > kMaxChain) ++p->K;
    ok = ok && prepare_kernel_attributes() == hipSuccess &&
              hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < kMaxConcurrency; ++i)
        ok = hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming) == hipSuccess;
    if (ok && !p->small.empty()) {
        ok = hipMalloc(&p->dsmall, p->small.size() * sizeof(SmallJob)) == hipSuccess &&
             hipMemcpy(p->dsmall, p->small.data(), p->small.size() * sizeof(SmallJob), hipMemcpyHostToDevice) ==
                 hipSuccess;
    }
    if (!ok) {
        psd_plan_destroy(p);
        return PSD_EDEVICE;
    }
    *plan = p;
    return PSD_OK;
}

psd_status psd_plan_workspace_size(psd_plan p, int32_t concurrency, size_t *bytes) {
    if (!p || !bytes || concurrency < 0 || concurrency > kMaxConcurrency) return PSD_EINVAL;
    const int K = concurrency ? concurrency : p->K;
    *bytes = (size_t)K * p->slot_bytes + 256;
    return PSD_OK;
}

int32_t psd_plan_concurrency(psd_plan p) { return p ? p->K : 0; }

int32_t psd_plan_group_size(psd_plan p) { return p ? max_members(p) : 0; }

int32_t psd_plan_ns_tile_threshold(psd_plan p) { return p ? p->ns_big : 0; }

psd_status psd_plan_execute(psd_plan p, const double *x, double *y, void *ws, size_t ws_bytes, void *stream,
                            psd_info *infos) {
    if (!p || !x || !y) return PSD_EINVAL;
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 7u) return PSD_EINVAL;
    const size_t need = (size_t)p->K * p->slot_bytes;
    if (p->nlarge && (!ws || ws_bytes < need)) return PSD_EWORKSPACE;
    if (ws && (reinterpret_cast<uintptr_t>(ws) % 256)) return PSD_EINVAL;
    hipGraphExec_t ex = find_graph(p, x, y, ws, infos, p->K);
    if (!ex && longest_chain(p, p->K) > kMaxChain) return PSD_EUNSUPPORTED;
    if (!ex) {
        // at most kMaxGraphs captured buffer sets; the oldest is dropped once
        // the work already queued on the stream (which may replay it) is done
        if ((int)p->graphs.size() >= kMaxGraphs) {
            if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return PSD_EDEVICE;
            (void)hipGraphExecDestroy(p->graphs.front().exec);
            p->graphs.erase(p->graphs.begin());
        }
        if (capture(p, x, y, ws, infos, p->K, &ex) != hipSuccess) return PSD_EDEVICE;
        p->graphs.push_back(GraphEntry{x, y, ws, infos, p->K, p->group, p->ns_big, ex});
    }
    return hipGraphLaunch(ex, static_cast<hipStream_t>(stream)) == hipSuccess ? PSD_OK : PSD_EDEVICE;
}

psd_status psd_plan_tune(psd_plan p, const double *x, double *y, void *ws, size_t ws_bytes, void *stream,
                         int32_t reps, int32_t *best_out) {
    if (!p || !x || !y || reps < 1) return PSD_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) return PSD_EDEVICE;
    int bestK = p->K, bestG = p->group, bestB = p->ns_big;
    double best_ms = 1e300;
    // tile forms of the BF16 Newton-Schulz product: the default, and 128x128
    // tiles from padded order 1024 when a block falls in 1024..2047
    std::vector<int> forms{NS_BIG_DEFAULT};
    if (p->mode == PSD_MIXED_BF16)
        for (int m : p->n) {
            const int npad = (m + 63) / 64 * 64;
            if (m > 64 && npad >= NS_BIG_MIN && npad < NS_BIG_DEFAULT) {
                forms.push_back(NS_BIG_MIN);
                break;
            }
        }
    // group sizes: the memory-derived limit (up to 128), then 16 and 8 where
    // they split differently; for each, concurrency 1, 2, 4, ... and the
    // number of jobs.  Each candidate is captured and replayed once untimed,
    // then scored by its fastest of `reps` timed replays (the minimum is not
    // moved by other work on the device); two replays of the plan as it
    // stands come first so that the first candidate is not timed cold.
    for (int r = 0; r < 2; ++r)
        if (psd_plan_execute(p, x, y, ws, ws_bytes, stream, nullptr) != PSD_OK) break;
    for (int form : forms) {
    p->ns_big = form;
    std::vector<int> tried;
    for (int g : {0, 16, 8}) {
        if (!set_jobs(p, g)) break;
        const int mm = max_members(p);
        if (std::find(tried.begin(), tried.end(), mm) != tried.end()) continue;
        tried.push_back(mm);
        const int maxK = std::max(1, std::min(p->nlarge, kMaxConcurrency));
        std::vector<int> cand;
        for (int K = 1; K < maxK; K *= 2) cand.push_back(K);
        cand.push_back(maxK);
        for (int K : cand) {
            if ((size_t)K * p->slot_bytes > ws_bytes) break;
            if (longest_chain(p, K) > kMaxChain) continue;   // not captured (kMaxChain)
            p->K = K;
            psd_status st = psd_plan_execute(p, x, y, ws, ws_bytes, stream, nullptr);  // capture + warm up
            if (st != PSD_OK) continue;
            double cand_ms = 1e300;
            for (int r = 0; r < reps && st == PSD_OK; ++r) {
                (void)hipEventRecord(t0, s);
                st = psd_plan_execute(p, x, y, ws, ws_bytes, stream, nullptr);
                (void)hipEventRecord(t1, s);
                (void)hipEventSynchronize(t1);  // also: nothing in flight reads the tables set_jobs rewrites
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, t0, t1);
                cand_ms = std::min(cand_ms, (double)ms);
            }
            if (st == PSD_OK && cand_ms < best_ms) {
                best_ms = cand_ms;
                bestK = K;
                bestG = g;
                bestB = form;
            }
        }
    }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (!set_jobs(p, bestG)) return PSD_EDEVICE;
    p->ns_big = bestB;
    p->K = std::max(1, std::min(bestK, std::max(1, p->nlarge)));
    while (p->K < std::min(kMaxConcurrency, p->nlarge) && longest_chain(p, p->K) > kMaxChain) ++p->K;
    tune_record(tune_key(p->n, p->mode), p->K, bestG, bestB, best_ms);
    if (best_out) *best_out = p->K;
    return PSD_OK;
}

psd_status psd_plan_destroy(psd_plan p) {
    if (!p) return PSD_EINVAL;
    for (auto &g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    if (p->dsmall) (void)hipFree(p->dsmall);
    if (p->dioff) (void)hipFree(p->dioff);
    if (p->didx) (void)hipFree(p->didx);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->fork) (void)hipEventDestroy(p->fork);
    for (int i = 0; i < kMaxConcurrency; ++i) {
        if (p->side[i]) (void)hipStreamDestroy(p->side[i]);
        if (p->join[i]) (void)hipEventDestroy(p->join[i]);
    }
    delete p;
    return PSD_OK;
}

}  // extern "C"
