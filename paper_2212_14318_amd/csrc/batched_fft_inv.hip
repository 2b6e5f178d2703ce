// Persistent inverse tube FFT of the batched path.
#include "batched_fft_impl.h"

namespace qt {
hipError_t launch_batched_fft_inv(const BatchFftJob* jobs, const BatchFftItem* items, int nitems,
                                  int grid, hipStream_t stream) {
    return detail::launch_batched_fft_impl<true>(jobs, items, nitems, grid, stream);
}
int batched_fft_inv_blocks_per_cu() {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, detail::batched_fft_kernel<true>, 256, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}
}  // namespace qt
