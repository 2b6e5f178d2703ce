// Tube-FFT dispatch (register-resident kernels are instantiated in
// fft_inst_*.hip) and the FP64 twiddle-table kernel.
#include "fft_impl.h"

QT_FFT_SIZES_F32(QT_FFT_EXTERN_F32)
QT_FFT_SIZES_F64(QT_FFT_EXTERN_F64)

namespace qt {
namespace {

// FP64 twiddle table: w^k = exp(-2 pi i k / p) from sincospi of 2k/p in
// double, rounded once to float for the FP32 table.
__global__ void twiddle_kernel(int p, float2* __restrict__ t32, double2* __restrict__ t64) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)p, &s, &c);
    t64[k] = double2{c, -s};
    t32[k] = float2{(float)c, (float)-s};
}

}  // namespace

template <>
bool tube_fft_supported<float>(int p) {
    switch (p) {
#define QT_CASE(P) case P:
        QT_FFT_SIZES_F32(QT_CASE) return true;
#undef QT_CASE
        default: return false;
    }
}

template <>
bool tube_fft_supported<double>(int p) {
    switch (p) {
#define QT_CASE(P) case P:
        QT_FFT_SIZES_F64(QT_CASE) return true;
#undef QT_CASE
        default: return false;
    }
}

template <>
hipError_t launch_tube_fft<float>(int p, bool inverse, const FftJob<float>* jobs, int njobs,
                                  const Twiddles& tw, hipStream_t stream) {
    if (njobs < 1 || njobs > 2) return hipErrorInvalidValue;
    if (!tube_fft_supported<float>(p)) {
        if (tw.blue.M == 0) return hipErrorNotSupported;
        return launch_bluestein<float>(p, inverse, jobs, njobs, tw.blue, stream);
    }
    switch (p) {
#define QT_CASE(P)                                                                           \
    case P:                                                                                  \
        return inverse ? detail::launch_p<P, true, float>(jobs, njobs, tw, stream)           \
                       : detail::launch_p<P, false, float>(jobs, njobs, tw, stream);
        QT_FFT_SIZES_F32(QT_CASE)
#undef QT_CASE
        default: return hipErrorNotSupported;
    }
}

template <>
hipError_t launch_tube_fft<double>(int p, bool inverse, const FftJob<double>* jobs, int njobs,
                                   const Twiddles& tw, hipStream_t stream) {
    if (njobs < 1 || njobs > 2) return hipErrorInvalidValue;
    if (!tube_fft_supported<double>(p)) {
        if (tw.blue.M == 0) return hipErrorNotSupported;
        return launch_bluestein<double>(p, inverse, jobs, njobs, tw.blue, stream);
    }
    switch (p) {
#define QT_CASE(P)                                                                           \
    case P:                                                                                  \
        return inverse ? detail::launch_p<P, true, double>(jobs, njobs, tw, stream)          \
                       : detail::launch_p<P, false, double>(jobs, njobs, tw, stream);
        QT_FFT_SIZES_F64(QT_CASE)
#undef QT_CASE
        default: return hipErrorNotSupported;
    }
}

hipError_t launch_twiddles(int p, Twiddles tw, hipStream_t stream) {
    hipLaunchKernelGGL(twiddle_kernel, dim3((p + 255) / 256), dim3(256), 0, stream, p, tw.f32, tw.f64);
    return hipGetLastError();
}

}  // namespace qt
