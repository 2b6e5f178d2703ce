// Register-resident FP32 tube-FFT kernels, length group 0.
#include "fft_impl.h"
QT_FFT_SIZES_G0(QT_FFT_INST_F32)
