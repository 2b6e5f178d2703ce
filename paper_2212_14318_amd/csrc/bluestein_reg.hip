// Bluestein tube FFT with the whole convolution in registers: one thread owns
// one tube, for convolution lengths M = 32, 64 (FP32) and 32 (FP64), i.e.
// every length p <= 32 (p <= 16 in FP64) that has no register-resident
// mixed-radix kernel of its own (11, 13, 17, 19, 22, 23, 26, 29, 31, ...).
// Longer convolutions would spill (M = 128 needs more than 256 VGPRs) and go
// to the LDS kernel.
//
// Same arithmetic as the LDS kernel in bluestein.hip (chirp c_k =
// exp(i pi (k^2 mod 2p) / p), a = x conj(c) zero-padded to M, FFT_M,
// pointwise product with the chirp spectrum, inverse FFT_M, conj(c_f) / M;
// conj c and 1 / (M p) for the inverse transform), with the length-M
// transforms done by the compile-time mixed-radix DFT of the register tube
// FFT (natural order in and out, so the spectra are the natural-order ones).
// Consecutive threads own consecutive (i, j) positions: every face is read
// and written as 64 consecutive reals per wave and plane.
#include "fft_impl.h"

namespace qt {
namespace {

template <typename T, bool INV, int M>
__global__ void __launch_bounds__(256)
bluestein_reg_kernel(detail::FftJobs2<T> jobs, int p, const typename detail::Vec2<T>::type* __restrict__ chirp,
                     const typename detail::Vec2<T>::type* __restrict__ hat,
                     const typename detail::Vec2<T>::type* __restrict__ twf) {
    using V = typename detail::Vec2<T>::type;
    const unsigned b = detail::xcd_contiguous(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const unsigned bx = b % gridDim.x, by = b / gridDim.x;
    const int part = by & 1;
    const FftJob<T> jb = jobs.j[by >> 1];
    const long e = (long)bx * blockDim.x + threadIdx.x;
    if (e >= (long)jb.rows * jb.cols || part >= jb.parts) return;
    const long i = e / jb.cols, c = e - i * jb.cols;
    const size_t sface = (size_t)jb.rows * jb.src_ld;
    const size_t dface = (size_t)jb.rows * jb.dst_ld;
    const int H = p / 2 + 1;                       // Hermitian half spectrum (real tubes)
    const bool half = jb.half != 0;
    const size_t splane = (size_t)(half && INV ? H : p) * sface;
    const size_t dplane = (size_t)(half && !INV ? H : p) * dface;
    const T* src = jb.src + (size_t)(half ? 0 : 2 * part) * splane + (size_t)i * jb.src_ld + c;
    T* dst = jb.dst + (size_t)(half && INV ? 0 : 2 * part) * dplane + (size_t)i * jb.dst_ld + c;

    V x[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        V v{0, 0};
        if (k < p) {
            if (!half) {
                v = V{src[k * sface], src[k * sface + splane]};
            } else if (!INV) {
                v = V{src[k * sface], T(0)};
            } else {
                const int kk = k < H ? k : p - k;   // X^[k] = conj(X^[p - k]) for k >= H
                v = V{src[kk * sface], k < H ? src[kk * sface + splane] : -src[kk * sface + splane]};
            }
            const V ck = chirp[k];
            v = detail::cmul(v, INV ? ck : V{ck.x, -ck.y});
        }
        x[k] = v;
    }
    detail::Dft<M, M, false, V>::run(x, twf);
#pragma unroll
    for (int f = 0; f < M; ++f) x[f] = detail::cmul(x[f], hat[f]);
    detail::Dft<M, M, true, V>::run(x, twf);
    const T scale = INV ? T(1) / (T(M) * T(p)) : T(1) / T(M);
    const int nout = half && !INV ? H : p;
#pragma unroll
    for (int f = 0; f < M; ++f) {
        if (f < nout) {
            const V cf = chirp[f];
            const V y = detail::cmul(x[f], INV ? cf : V{cf.x, -cf.y});
            const T yr = y.x * scale, yi = y.y * scale;
            if (half && INV) {                    // real output: one plane
                dst[f * dface] = yr;
            } else if (!INV && sizeof(T) == 4 && jb.pack) {
                reinterpret_cast<unsigned*>(dst)[f * dface] = detail::split_bf16_word((float)yr);
                reinterpret_cast<unsigned*>(dst)[f * dface + dplane] = detail::split_bf16_word((float)yi);
            } else {
                dst[f * dface] = yr;
                dst[f * dface + dplane] = yi;
            }
        }
    }
}

template <typename T, int M>
hipError_t launch_m(int p, bool inverse, const detail::FftJobs2<T>& pk, dim3 grid, const BluesteinTables& bt,
                    hipStream_t stream) {
    using V = typename detail::Vec2<T>::type;
    const V *chirp, *hat, *twf;
    if constexpr (sizeof(T) == 4) {
        chirp = bt.chirp32; hat = inverse ? bt.hatn_inv32 : bt.hatn_fwd32; twf = bt.twf32;
    } else {
        chirp = bt.chirp64; hat = inverse ? bt.hatn_inv64 : bt.hatn_fwd64; twf = bt.twf64;
    }
    if (inverse)
        hipLaunchKernelGGL((bluestein_reg_kernel<T, true, M>), grid, dim3(256), 0, stream, pk, p, chirp, hat, twf);
    else
        hipLaunchKernelGGL((bluestein_reg_kernel<T, false, M>), grid, dim3(256), 0, stream, pk, p, chirp, hat, twf);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_bluestein_reg(int p, bool inverse, const FftJob<T>* jobs, int njobs, const BluesteinTables& bt,
                                hipStream_t stream) {
    constexpr int MMAX = sizeof(T) == 4 ? 64 : 32;
    if (bt.M > MMAX || bt.M < 32) return hipErrorNotSupported;
    detail::FftJobs2<T> pk{};
    long maxc = 0;
    for (int q = 0; q < njobs; ++q) {
        pk.j[q] = jobs[q];
        const long cnt = (long)jobs[q].rows * jobs[q].cols;
        maxc = cnt > maxc ? cnt : maxc;
    }
    const dim3 grid((unsigned)((maxc + 255) / 256), 2 * njobs);
    if (bt.M == 32) return launch_m<T, 32>(p, inverse, pk, grid, bt, stream);
    if constexpr (sizeof(T) == 4) return launch_m<T, 64>(p, inverse, pk, grid, bt, stream);
    return hipErrorNotSupported;
}

template hipError_t launch_bluestein_reg<float>(int, bool, const FftJob<float>*, int, const BluesteinTables&,
                                                hipStream_t);
template hipError_t launch_bluestein_reg<double>(int, bool, const FftJob<double>*, int, const BluesteinTables&,
                                                 hipStream_t);

}  // namespace qt
