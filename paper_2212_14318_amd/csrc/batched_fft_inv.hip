// Inverse tube FFT of the batched path (one instance per tube length).
#include "batched_fft_impl.h"

namespace qt {
hipError_t launch_batched_fft_inv(int p, int pol, const BatchFftJob* jobs, const BatchFftItem* items,
                                  int nitems, hipStream_t stream) {
    return detail::launch_batched_fft_impl<true>(p, pol, jobs, items, nitems, stream);
}
}  // namespace qt
