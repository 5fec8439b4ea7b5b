// Workspace layout and stage launchers of the large-block FP64 path
// (order n > 64): unpack -> blocked Householder tridiagonalisation ->
// divide-and-conquer tridiagonal eigensolver -> back-transform of the
// smaller sign side -> fused clamp + reconstruction + svec pack.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/psdproj.h"
#include "gemm.h"
#include "kernels.h"

namespace psd {

constexpr int LG_NB = 32;      // panel width of the tridiagonalisation
constexpr int LG_TILE = 64;    // HEMV tile
constexpr int LG_TAIL = 120;   // largest trailing order reduced by one workgroup in LDS
constexpr int DC_LEAF = 16;    // largest leaf of the divide and conquer

struct LargeWs {
    int n;
    int64_t lda;        // leading dimension of M, Zc (elements)
    int mb;             // ceil(n / 64)
    int npanel;         // panels of reflectors
    int kmax;           // max columns of the selected side (= n)
    // tridiagonalisation
    double2 *M;         // lda x n: Hermitian input, then reflectors
    double2 *W;         // lda x NB: panel w vectors
    double2 *vbuf;      // lda: current reflector
    double2 *tau;       // n
    double *d, *e;      // n, n
    double2 *P;         // mb*mb*64 HEMV partials
    double *tdot;       // mb*(mb+1)/2 partial v^H A v
    double2 *pq;        // mb * 2 * NB
    double *npart;      // mb sigma partials of the next column
    double2 *T;         // npanel * NB * NB block-reflector factors
    // divide and conquer
    double *Q0, *Q1;    // n x n (ld n) eigenvector ping-pong
    double *D0, *D1;    // n eigenvalue ping-pong
    double *U;          // n x n merge matrices (block diagonal, ld n)
    double *dcd;        // 16 * n per-merge vectors (see dc.hip)
    int *dci;           // 8 * n per-merge index vectors
    int *dcs;           // per-merge scalars (4 * n)
    GemmDesc *gdesc;    // 2 * (n/2 + 1) merge GEMM descriptors
    // back-transform and reconstruction
    double2 *Zc;        // lda x kmax selected eigenvectors (complex)
    double *lamsel;     // kmax selected eigenvalues
    double *wpart;      // split-K partials of V^H Z: nchunk * 128 * kmax complex
    double2 *W2;        // 128 x kmax
    double2 *Sg;        // 128 x 128: V^H V of a group of four panels
    double2 *spart;     // split-K partials of V^H V of a group: nchunk * 128 * 128
    int *ksel;          // [0] = k, [1] = n_pos, [2] = status
    double *sgn;        // reconstruction sign
    double *lam;        // n final eigenvalues (ascending)
    double *Zfinal;     // n x n real eigenvectors of T (points at Q0 or Q1)
    int nchunk;         // split-K chunks for V^H Z
    int kchunk;         // rows per chunk
    double2 *B1;        // n x n (ld n) derivative scratch (full layouts only)
    // lockstep group (every launch covers nmem blocks of this order; member b
    // uses the workspace slot b * zs bytes on, svec offset ioff[b] and info
    // record infoidx[b]); a single block: nmem = 1, zs = 0, null tables
    int nmem;
    int64_t zs;
    const int64_t *ioff;
    const int *infoidx;
};

// Bytes of a LargeWs for order n; carves it from `base` when non-null.
size_t large_layout(int n, int flags, void *base, LargeWs *ws);

hipError_t large_init(const LargeWs &w, hipStream_t st);
hipError_t large_unpack(const LargeWs &w, const double *x, hipStream_t st);
hipError_t large_tridiag(const LargeWs &w, hipStream_t st);
hipError_t large_compute_T(const LargeWs &w, hipStream_t st);
hipError_t large_dc(LargeWs &w, hipStream_t st);
hipError_t large_select(const LargeWs &w, psd_dev_info *info, hipStream_t st, bool all_columns);
hipError_t large_backtransform(const LargeWs &w, int ncols_max, hipStream_t st);
hipError_t large_reconstruct(const LargeWs &w, const double *x, double *y, int kmax, hipStream_t st);
hipError_t large_save(const LargeWs &w, double *saved, hipStream_t st);
hipError_t large_load_saved(const LargeWs &w, const double *saved, hipStream_t st);
hipError_t large_vjp_from_v(const LargeWs &w, const double *gy, double *gx, hipStream_t st);

// Lockstep groups of same-order blocks (abi.hip): the large blocks of a call
// split into groups; a group of c.blocks.size() members needs
// group_ws_bytes(c, mode) of workspace.
struct GroupChunk {
    int n;
    std::vector<int> blocks;  // block indices, in member order
};
// max_group > 0 caps the members per group below the memory-derived limit.
std::vector<GroupChunk> group_chunks(int nblocks, const int32_t *n, int mode, int max_group = 0);
size_t group_ws_bytes(const GroupChunk &c, int mode);
// ns_big: npad from which the BF16 Newton-Schulz product uses 128x128 tiles.
hipError_t project_group_ext(int n, int nmem, psd_mode mode, const double *x, double *y, const int64_t *ioff,
                             const int *infoidx, psd_dev_info *infos, void *ws, hipStream_t s, int ns_big);

}  // namespace psd
