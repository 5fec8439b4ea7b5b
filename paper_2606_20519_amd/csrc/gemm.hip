// FP64 MFMA GEMM (see gemm.h).  Block tile 64x64x16, 256 threads = 4 waves
// in a 2x2 arrangement, each wave owning a 32x32 sub-tile made of 2x2
// v_mfma_f64_16x16x4 blocks.  Complex products use four real MFMAs per block
// (re*re - im*im, re*im + im*re) on interleaved {re, im} operands.
//
// MFMA f64 16x16x4 operand layout (lane l of the wave):
//   A[i][k]: i = l % 16, k = l / 16;  B[k][j]: j = l % 16, k = l / 16;
//   D[i][j] (4 values per lane): j = l % 16, i = l / 16 + 4 * v
// (checked on gfx950 with one-hot inputs; the f32/bf16 forms differ).
#include <algorithm>

#include "common.h"
#include "gemm.h"
#include "gemm_tile.h"
#include "timing.h"

namespace psd {

namespace {

using namespace gemmdev;

template <typename T, int OPA, int OPB, int EPI>
__global__ void __launch_bounds__(NT, 3) gemm_kernel(GemmDesc d) {
    __shared__ GemmLds<T> L;
    if (d.skip && *d.skip) return;
    int tz = blockIdx.z, b = 0;
    if (d.nmem > 1) {
        const int ks = gemm_kslices(d);
        b = tz / ks;
        tz -= b * ks;
        d.A.p0 = member_ptr(d.A.p0, d.zs, b);
        d.A.p1 = member_ptr(d.A.p1, d.zs, b);
        d.A.kscale = member_ptr(d.A.kscale, d.zs, b);
        d.B.p0 = member_ptr(d.B.p0, d.zs, b);
        d.B.p1 = member_ptr(d.B.p1, d.zs, b);
        d.B.kscale = member_ptr(d.B.kscale, d.zs, b);
        d.C = member_ptr(d.C, d.zs, b);
        d.lam = member_ptr(d.lam, d.zs, b);
        d.dN = member_ptr(d.dN, d.zs, b);
        d.dK = member_ptr(d.dK, d.zs, b);
        d.dsign = member_ptr(d.dsign, d.zs, b);
        d.dstatus = member_ptr(d.dstatus, d.zs, b);
    }
    if (d.ioff) {  // also for a group of one: its svec need not start at offset 0
        const int64_t o = d.ioff[b];
        if (d.y) d.y += o;
        if (d.xbase) d.xbase += o;
    }
    int ti = blockIdx.x, tj = blockIdx.y;
    if (d.lower_only) {
        // compact grid over the lower tiles only (M == N): column by column,
        // longest column first, rows consecutive within a column (the order
        // of the full grid, without the workgroups that would exit at once)
        const int mt = (d.M + BM - 1) / BM;
        const int t = mt * (mt + 1) / 2 - 1 - (int)blockIdx.x;
        int u = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((u + 1) * (u + 2) / 2 <= t) ++u;
        while (u * (u + 1) / 2 > t) --u;
        tj = mt - 1 - u;
        ti = mt - 1 - (t - u * (u + 1) / 2);
    }
    gemm_tile<T, OPA, OPB, EPI>(d, ti, tj, tz, L);
}

template <typename T, int OPA, int OPB>
__global__ void __launch_bounds__(NT) gemm_kernel_batched(const GemmDesc *ds, int count, int64_t zs) {
    __shared__ GemmLds<T> L;
    const int b = blockIdx.z / count;
    const GemmDesc d = member_ptr(ds, zs, b)[blockIdx.z - b * count];
    gemm_tile<T, OPA, OPB, EPI_STORE>(d, blockIdx.x, blockIdx.y, 0, L);
}

template <typename T, int EPI>
hipError_t launch_ops(const GemmDesc &d, hipStream_t st) {
    dim3 grid((d.M + BM - 1) / BM, (d.N + BN - 1) / BN, gemm_kslices(d) * std::max(1, d.nmem));
    if (d.lower_only) {
        const int mt = (d.M + BM - 1) / BM;
        grid.x = mt * (mt + 1) / 2;
        grid.y = 1;
    }
    const int key = d.A.op * 2 + d.B.op;
    switch (key) {
        case 0: hipLaunchKernelGGL((gemm_kernel<T, OP_N, OP_N, EPI>), grid, dim3(NT), 0, st, d); break;
        case 1: hipLaunchKernelGGL((gemm_kernel<T, OP_N, OP_C, EPI>), grid, dim3(NT), 0, st, d); break;
        case 2: hipLaunchKernelGGL((gemm_kernel<T, OP_C, OP_N, EPI>), grid, dim3(NT), 0, st, d); break;
        default: hipLaunchKernelGGL((gemm_kernel<T, OP_C, OP_C, EPI>), grid, dim3(NT), 0, st, d); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t gemm_launch(const GemmDesc &d, bool complex_data, int epilogue, hipStream_t st) {
    if (d.M <= 0 || d.N <= 0) return hipSuccess;
    if (d.lower_only && d.M != d.N) return hipErrorInvalidValue;  // the lower-tile grid assumes a square output
    const int slot = timing_begin(KF_GEMM, st);
    hipError_t e;
    if (complex_data) {
        switch (epilogue) {
            case EPI_SVEC: e = launch_ops<cd, EPI_SVEC>(d, st); break;
            case EPI_GAMMA: e = launch_ops<cd, EPI_GAMMA>(d, st); break;
            default: e = launch_ops<cd, EPI_STORE>(d, st); break;
        }
    } else {
        e = launch_ops<double, EPI_STORE>(d, st);
    }
    // algorithmic flops (upper bound when N or K is only known on the device)
    double f = (complex_data ? 8.0 : 2.0) * (double)d.M * (double)d.N * (double)d.K * std::max(1, d.nmem);
    if (d.lower_only) f *= 0.5;
    timing_end(slot, st, f);
    return e;
}

hipError_t gemm_launch_batched(const GemmDesc *ddesc, int count, int maxM, int maxN, bool complex_data,
                               hipStream_t st, int nmem, int64_t zs) {
    if (count <= 0 || maxM <= 0 || maxN <= 0) return hipSuccess;
    dim3 grid((maxM + BM - 1) / BM, (maxN + BN - 1) / BN, count * std::max(1, nmem));
    // Batched problems use op(A) = N and op(B) = C (the divide-and-conquer
    // merge products Q_child * U^T with U stored row-major).
    if (complex_data)
        hipLaunchKernelGGL((gemm_kernel_batched<cd, OP_N, OP_C>), grid, dim3(NT), 0, st, ddesc, count, zs);
    else
        hipLaunchKernelGGL((gemm_kernel_batched<double, OP_N, OP_C>), grid, dim3(NT), 0, st, ddesc, count, zs);
    return hipGetLastError();
}

}  // namespace psd
