// Tube FFT of the batched path.  The work list holds (job, CD part,
// 256-position block) items sorted by tube length; the host launches one
// kernel instance per run of equal length, so every launch has the register
// budget (and occupancy) of its own p instead of that of the longest p.
// Every job keeps its own shape, strides and twiddle table; the radix-order
// policy is the one the autotuner picked for that p.
#pragma once
#include "batched.h"
#include "fft_impl.h"

namespace qt {
namespace detail {

// one workgroup = one item
template <int P, int POL, bool INV>
__global__ void __launch_bounds__(256)
batched_fft_kernel(const BatchFftJob* __restrict__ jobs, const BatchFftItem* __restrict__ items) {
    const BatchFftItem item = items[xcd_contiguous(blockIdx.x, gridDim.x)];
    const BatchFftJob bj = jobs[item.job];
    const bool fill = !INV && bj.fill;              // (inverse jobs never fill)
    const int w = fill ? bj.dst_ld : bj.cols;       // positions per row
    const long e = (long)item.e0 + threadIdx.x;
    if (e >= (long)bj.rows * w) return;
    const FftJob<float> jb{bj.src, bj.dst, bj.rows, bj.cols, bj.src_ld, bj.dst_ld, bj.pack};
    if constexpr (!INV) {
        if (fill) {
            const int i = (int)(e / w);
            tube_fft_rc<P, false, float, POL, true>(jb, item.part, i, (int)(e - (long)i * w), bj.tw);
            return;
        }
    }
    tube_fft_one<P, INV, float, POL>(jb, item.part, e, bj.tw);
}

template <bool INV>
hipError_t launch_batched_fft_impl(int p, int pol, const BatchFftJob* jobs, const BatchFftItem* items,
                                   int nitems, hipStream_t stream) {
    if (nitems <= 0) return hipSuccess;
    const dim3 grid((unsigned)nitems), block(256);
    switch (2 * p + (pol ? 1 : 0)) {
#define QT_BCASE(P)                                                                                   \
    case 2 * P:                                                                                       \
        hipLaunchKernelGGL((batched_fft_kernel<P, 0, INV>), grid, block, 0, stream, jobs, items);     \
        break;                                                                                        \
    case 2 * P + 1:                                                                                   \
        hipLaunchKernelGGL((batched_fft_kernel<P, 1, INV>), grid, block, 0, stream, jobs, items);     \
        break;
        QT_FFT_SIZES_F64(QT_BCASE)
#undef QT_BCASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace detail
}  // namespace qt
