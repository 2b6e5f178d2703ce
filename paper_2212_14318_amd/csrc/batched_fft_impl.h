// Persistent tube FFT of the batched path: one launch walks a heterogeneous
// list of (job, CD part, 256-position block) items; every job has its own
// p, shape, twiddle table and radix-order policy (picked by the autotuner).
#pragma once
#include "batched.h"
#include "fft_impl.h"

namespace qt {
namespace detail {

template <bool INV>
__global__ void __launch_bounds__(256)
batched_fft_kernel(const BatchFftJob* __restrict__ jobs, const BatchFftItem* __restrict__ items,
                   int nitems) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BatchFftItem item = items[it];
        const BatchFftJob bj = jobs[item.job];
        const long e = (long)item.e0 + threadIdx.x;
        if (e >= (long)bj.rows * bj.cols) continue;
        const FftJob<float> jb{bj.src, bj.dst, bj.rows, bj.cols, bj.src_ld, bj.dst_ld, bj.pack};
        switch (2 * bj.p + bj.pol) {
#define QT_BCASE(P)                                                                \
    case 2 * P: tube_fft_one<P, INV, float, 0>(jb, item.part, e, bj.tw); break;   \
    case 2 * P + 1: tube_fft_one<P, INV, float, 1>(jb, item.part, e, bj.tw); break;
            QT_FFT_SIZES_F64(QT_BCASE)
#undef QT_BCASE
            default: break;
        }
    }
}

template <bool INV>
hipError_t launch_batched_fft_impl(const BatchFftJob* jobs, const BatchFftItem* items, int nitems,
                                   int grid, hipStream_t stream) {
    hipLaunchKernelGGL((batched_fft_kernel<INV>), dim3(grid), dim3(256), 0, stream, jobs, items, nitems);
    return hipGetLastError();
}

}  // namespace detail
}  // namespace qt
