// Register-resident FP32 tube-FFT kernels, length group 4.
#include "fft_impl.h"
QT_FFT_SIZES_G4(QT_FFT_INST_F32)
