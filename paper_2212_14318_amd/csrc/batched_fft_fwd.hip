// Forward tube FFT of the batched path (one instance per tube length).
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

hipError_t launch_batched_fft_fwd(int p, int pol, const BatchFftJob* jobs, const BatchFftItem* items,
                                  int nitems, hipStream_t stream) {
    return detail::launch_batched_fft_impl<false>(p, pol, jobs, items, nitems, stream);
}
}  // namespace qt
