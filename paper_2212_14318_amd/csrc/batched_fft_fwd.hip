// Persistent forward tube FFT of the batched path.
#include "batched_fft_impl.h"

namespace qt {
bool batched_fft_supported(int p) {
    switch (p) {
#define QT_CASE(P) case P:
        QT_FFT_SIZES_F64(QT_CASE) return true;
#undef QT_CASE
        default: return false;
    }
}

hipError_t launch_batched_fft_fwd(const BatchFftJob* jobs, const BatchFftItem* items, int nitems,
                                  int grid, hipStream_t stream) {
    return detail::launch_batched_fft_impl<false>(jobs, items, nitems, grid, stream);
}
int batched_fft_fwd_blocks_per_cu() {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, detail::batched_fft_kernel<false>, 256, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}
}  // namespace qt
