// Conversion of a Fourier-domain FP32 tensor into the split-bf16 operand
// format, in place: every real x becomes the word hi | lo << 16 with
// hi = rn_bf16(x), lo = rn_bf16(x - hi) -- the words the forward tube FFT
// writes for QT_SPLIT_BF16.  It lets the FP32 output of one coupled product
// (qt_fourier_tprod) feed the next split-bf16 product without leaving the
// Fourier domain: bcirc(A * B) = bcirc(A) bcirc(B) (proof of Theorem 5.1), so
// products of block-diagonalised tensors chain frequency by frequency.
#include "fft_impl.h"

namespace qt {
namespace {

// grid-stride over (face, row, 4-column group); ld is a multiple of 4, so a
// group is one aligned 16-byte access
__global__ void __launch_bounds__(256)
split_words_kernel(float* __restrict__ X, long faces, long rows, long cols, long ld) {
    const long groups = (cols + 3) / 4;
    const long total = faces * rows * groups;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long g = e % groups;
        const long fr = e / groups;                      // face * rows + row
        float* row = X + fr * ld + 4 * g;
        const int n = (int)(cols - 4 * g < 4 ? cols - 4 * g : 4);
        if (n == 4) {
            float4 v = *reinterpret_cast<const float4*>(row);
            uint4 w;
            w.x = detail::split_bf16_word(v.x);
            w.y = detail::split_bf16_word(v.y);
            w.z = detail::split_bf16_word(v.z);
            w.w = detail::split_bf16_word(v.w);
            *reinterpret_cast<uint4*>(row) = w;
        } else {
            for (int j = 0; j < n; ++j)
                reinterpret_cast<unsigned*>(row)[j] = detail::split_bf16_word(row[j]);
        }
    }
}

// fp16 words of a Fourier-domain tensor [planes][p][rows][ld] scaled per
// frequency: x -> hi | lo << 16 with hi = rn_fp16(x s_f), lo = rn_fp16(x s_f
// - hi); s_f = scale[f] is a power of two, so the scaling is exact.
__global__ void __launch_bounds__(256)
fp16_words_kernel(float* __restrict__ X, long p, long rows, long cols, long ld, const float* __restrict__ scale,
                  int planes) {
    const long groups = (cols + 3) / 4;
    const long total = planes * p * rows * groups;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const long g = e % groups;
        const long fr = e / groups;                      // (plane * p + face) * rows + row
        const float sc = scale[(fr / rows) % p];
        float* row = X + fr * ld + 4 * g;
        const int n = (int)(cols - 4 * g < 4 ? cols - 4 * g : 4);
        auto word = [sc](float x) { return detail::split_fp16_word(x, sc); };
        if (n == 4) {
            const float4 v = *reinterpret_cast<const float4*>(row);
            *reinterpret_cast<uint4*>(row) = uint4{word(v.x), word(v.y), word(v.z), word(v.w)};
        } else {
            for (int j = 0; j < n; ++j) reinterpret_cast<unsigned*>(row)[j] = word(row[j]);
        }
    }
}

}  // namespace

hipError_t launch_fp16_words(float* X, long p, long rows, long cols, long ld, const float* scale,
                             hipStream_t stream, int planes) {
    const long total = planes * p * rows * ((cols + 3) / 4);
    if (total <= 0) return hipSuccess;
    long blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fp16_words_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X, p, rows, cols, ld,
                       scale, planes);
    return hipGetLastError();
}

hipError_t launch_split_words(float* X, long faces, long rows, long cols, long ld, hipStream_t stream) {
    const long total = faces * rows * ((cols + 3) / 4);
    if (total <= 0) return hipSuccess;
    long blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(split_words_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, X, faces, rows, cols,
                       ld);
    return hipGetLastError();
}

}  // namespace qt
