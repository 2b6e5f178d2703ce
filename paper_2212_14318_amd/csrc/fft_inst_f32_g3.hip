// Register-resident FP32 tube-FFT kernels, length group 3.
#include "fft_impl.h"
QT_FFT_SIZES_G3(QT_FFT_INST_F32)
