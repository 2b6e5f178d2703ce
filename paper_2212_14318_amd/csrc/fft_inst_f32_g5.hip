// Register-resident FP32 tube-FFT kernels, length group 5.
#include "fft_impl.h"
QT_FFT_SIZES_G5(QT_FFT_INST_F32)
