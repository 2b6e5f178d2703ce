// Tube FFTs along the third mode of a quaternion tensor (gfx950).
//
// Theorem 4.4 turns the block diagonalisation of bcirc(Q) into a length-p DFT
// of every tube Q(i, j, :); Remark 4.3 (iv) gives the inverse.  Both
// Cayley-Dickson parts Q1 = a + b i and Q2 = c + d i are transformed with the
// plain DFT  X^[f] = sum_k X[k] w^(f k),  w = exp(-2 pi i / p), and the
// inverse carries 1/p.  (The paper transforms conj(Q); with the coupling
// written for the plain transform the product C is the same.)
//
// Design: one thread owns one complex tube (p values of one CD part at one
// (i, j) position) and keeps it in registers.  Consecutive threads own
// consecutive (i, j), so for every face each wave reads and writes 64
// consecutive reals per plane: fully coalesced and each element read once
// and written once (32 bytes per quaternion per direction in FP32, the HBM
// minimum).  The transform is a mixed-radix decimation-in-time FFT whose
// length P is a template parameter, so every index is a compile-time
// constant and the data never leaves VGPRs.  Twiddles come from a table
// generated in FP64 on the device (uniform addresses -> scalar loads).
#pragma once
#include "qt_internal.h"

namespace qt {
namespace detail {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

template <typename V>
__device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V>
__device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
    return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename V>
__device__ __forceinline__ V mul_mi(V a) { return INV ? V{-a.y, a.x} : V{a.y, -a.x}; }

// w_N^e for a length-N sub-transform of a length-P table, conjugated for INV.
template <int P, int N, bool INV, typename V>
__device__ __forceinline__ V twiddle(int e, const V* __restrict__ tw) {
    V w = tw[(e % N) * (P / N)];
    if (INV) w.y = -w.y;
    return w;
}

// Radix order of the decimation (the "radix plan"):
//   POL = 0: powers of two first (4, then 2), then 3, 5, 7;
//   POL = 1: odd primes first (7, 5, 3), then 4, 2.
// Both give the same transform; they differ in the number and position of
// twiddle multiplications.  The batched path lets its autotuner pick one per p.
template <int POL>
constexpr int pick_radix(int n) {
    if constexpr (POL == 0) {
        return (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : (n % 5 == 0) ? 5
             : (n % 7 == 0) ? 7 : n;
    } else {
        return (n % 7 == 0) ? 7 : (n % 5 == 0) ? 5 : (n % 3 == 0) ? 3 : (n % 4 == 0) ? 4
             : (n % 2 == 0) ? 2 : n;
    }
}

// In-register DFT of length R (the butterfly of one radix stage).
template <int P, int R, bool INV, typename V>
__device__ __forceinline__ void small_dft(V (&t)[R], const V* __restrict__ tw) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        V a = t[0], b = t[1];
        t[0] = cadd(a, b);
        t[1] = csub(a, b);
    } else if constexpr (R == 4) {
        V a = t[0], b = t[1], c = t[2], d = t[3];
        V s0 = cadd(a, c), d0 = csub(a, c);
        V s1 = cadd(b, d), d1 = mul_mi<INV>(csub(b, d));
        t[0] = cadd(s0, s1);
        t[2] = csub(s0, s1);
        t[1] = cadd(d0, d1);
        t[3] = csub(d0, d1);
    } else {
        // odd prime radix: X[u] = sum_v t[v] w_R^(u v), pairing v and R - v
        // (w^(u(R-v)) = conj(w^(uv))) to halve the multiplications.
        V x[R];
#pragma unroll
        for (int u = 0; u < R; ++u) x[u] = t[u];
        V sum = x[0];
#pragma unroll
        for (int v = 1; v < R; ++v) sum = cadd(sum, x[v]);
        t[0] = sum;
#pragma unroll
        for (int u = 1; u < R; ++u) {
            V acc = x[0];
#pragma unroll
            for (int v = 1; v <= R / 2; ++v) {
                const V w = twiddle<P, R, INV>(u * v, tw);
                const V sp = cadd(x[v], x[R - v]);
                const V sm = csub(x[v], x[R - v]);
                // x[v] w + x[R-v] conj(w) = (sp wr) + i (sm wi) componentwise
                acc.x += sp.x * w.x - sm.y * w.y;
                acc.y += sp.y * w.x + sm.x * w.y;
            }
            t[u] = acc;
        }
    }
}

// Decimation in time: N = R M.  Sub-transforms of the R decimated sequences
// x[j R + r], then X[q + M u] = sum_r w_R^(r u) (w_N^(r q) Y_r[q]).
template <int P, int N, bool INV, typename V, int POL = 0>
struct Dft {
    static __device__ __forceinline__ void run(V (&x)[N], const V* __restrict__ tw) {
        constexpr int R = pick_radix<POL>(N);
        constexpr int M = N / R;
        if constexpr (M == 1) {
            small_dft<P, R, INV>(x, tw);
        } else {
            V sub[R][M];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = 0; j < M; ++j) sub[r][j] = x[j * R + r];
#pragma unroll
            for (int r = 0; r < R; ++r) Dft<P, M, INV, V, POL>::run(sub[r], tw);
#pragma unroll
            for (int q = 0; q < M; ++q) {
                V t[R];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    t[r] = (r * q == 0) ? sub[r][q] : cmul(sub[r][q], twiddle<P, N, INV>(r * q, tw));
                small_dft<P, R, INV>(t, tw);
#pragma unroll
                for (int u = 0; u < R; ++u) x[q + M * u] = t[u];
            }
        }
    }
};

template <typename T>
struct FftJobs2 {
    FftJob<T> j[2];
};

// bf16 split of one real in one word: low half hi = rn(x), high half
// lo = rn(x - hi), both round-to-nearest-even (hardware conversion).
__device__ __forceinline__ unsigned split_bf16_word(float x) {
    const __bf16 hi = (__bf16)x;
    const __bf16 lo = (__bf16)(x - (float)hi);
    return (unsigned)__builtin_bit_cast(unsigned short, hi) |
           ((unsigned)__builtin_bit_cast(unsigned short, lo) << 16);
}

// fp16 split of one real scaled by a power of two sc (exact): low half
// hi = rn_fp16(x sc), high half lo = rn_fp16(x sc - hi).
__device__ __forceinline__ unsigned split_fp16_word(float x, float sc) {
    const float y = x * sc;
    const _Float16 hi = (_Float16)y;
    const _Float16 lo = (_Float16)(y - (float)hi);
    return (unsigned)__builtin_bit_cast(unsigned short, hi) |
           ((unsigned)__builtin_bit_cast(unsigned short, lo) << 16);
}

// Real tubes (the DFT of a real sequence is Hermitian, X^[p - f] =
// conj(X^[f])): forward from one real plane to faces 0..p/2 of the (Re, Im)
// planes, inverse from those faces back to the real plane.  sre / dre point
// at position (i, c) of plane 0; the half-spectrum planes hold H = p/2 + 1
// faces.
template <int P, bool INV, typename T, int POL>
__device__ __forceinline__ void tube_fft_half(const FftJob<T>& jb, const T* __restrict__ sre,
                                              T* __restrict__ dre, size_t sface, size_t dface,
                                              const typename Vec2<T>::type* __restrict__ tw) {
    using V = typename Vec2<T>::type;
    constexpr int H = P / 2 + 1;
    V x[P];
    if constexpr (!INV) {
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = V{sre[k * sface], T(0)};
    } else {
        const T* __restrict__ sim = sre + (size_t)H * sface;
#pragma unroll
        for (int k = 0; k < H; ++k) x[k] = V{sre[k * sface], sim[k * sface]};
#pragma unroll
        for (int k = H; k < P; ++k) x[k] = V{x[P - k].x, -x[P - k].y};
    }
    Dft<P, P, INV, V, POL>::run(x, tw);
    if constexpr (!INV) {
        T* __restrict__ dim = dre + (size_t)H * dface;
        if constexpr (sizeof(T) == 4) {
            if (jb.pack) {
                unsigned* ure = reinterpret_cast<unsigned*>(dre);
                unsigned* uim = reinterpret_cast<unsigned*>(dim);
#pragma unroll
                for (int k = 0; k < H; ++k) {
                    ure[k * dface] = split_bf16_word(x[k].x);
                    uim[k * dface] = split_bf16_word(x[k].y);
                }
                return;
            }
        }
#pragma unroll
        for (int k = 0; k < H; ++k) {
            dre[k * dface] = x[k].x;
            dim[k * dface] = x[k].y;
        }
    } else {
        const T scale = T(1) / T(P);
#pragma unroll
        for (int k = 0; k < P; ++k) dre[k * dface] = x[k].x * scale;
    }
}

// Transform one complex tube: part 0 = X1 (planes 0, 1), part 1 = X2
// (planes 2, 3) at row i, column c of job jb.  FILL (forward): c runs over
// the destination's padded rows, and a column c >= cols is transformed as a
// zero tube (its loads read column cols - 1 and are discarded), so that the
// padding columns are written in the same store instructions as the others.
template <int P, bool INV, typename T, int POL = 0, bool FILL = false>
__device__ __forceinline__ void tube_fft_rc(const FftJob<T>& jb, int part, int i, int c,
                                            const typename Vec2<T>::type* __restrict__ tw) {
    using V = typename Vec2<T>::type;
    static_assert(!(FILL && INV), "padding columns are filled by the forward transform");
    const bool zero = FILL && c >= jb.cols;
    const int cs = zero ? jb.cols - 1 : c;
    const size_t sface = (size_t)jb.rows * jb.src_ld;
    const size_t dface = (size_t)jb.rows * jb.dst_ld;
    const T* __restrict__ sre = jb.src + (size_t)(2 * part) * P * sface + (size_t)i * jb.src_ld + cs;
    const T* __restrict__ sim = sre + (size_t)P * sface;
    T* __restrict__ dre = jb.dst + (size_t)(2 * part) * P * dface + (size_t)i * jb.dst_ld + c;
    T* __restrict__ dim = dre + (size_t)P * dface;

    if constexpr (!FILL) {
        if (jb.half) {
            tube_fft_half<P, INV, T, POL>(jb, sre, dre, sface, dface, tw);
            return;
        }
    }
    V x[P];
#pragma unroll
    for (int k = 0; k < P; ++k) x[k] = V{sre[k * sface], sim[k * sface]};
    if constexpr (FILL) {
        if (zero) {
#pragma unroll
            for (int k = 0; k < P; ++k) x[k] = V{T(0), T(0)};
        }
    }
    Dft<P, P, INV, V, POL>::run(x, tw);
    if constexpr (!INV && sizeof(T) == 4) {
        if (jb.pack) {   // bf16 split of every real: hi | lo << 16
            unsigned* ure = reinterpret_cast<unsigned*>(dre);
            unsigned* uim = reinterpret_cast<unsigned*>(dim);
#pragma unroll
            for (int k = 0; k < P; ++k) {
                ure[k * dface] = split_bf16_word(x[k].x);
                uim[k * dface] = split_bf16_word(x[k].y);
            }
            return;
        }
    }
    const T scale = INV ? T(1) / T(P) : T(1);
#pragma unroll
    for (int k = 0; k < P; ++k) {
        dre[k * dface] = x[k].x * scale;
        dim[k * dface] = x[k].y * scale;
    }
}

// The same at flattened position e = i * cols + c.
template <int P, bool INV, typename T, int POL = 0>
__device__ __forceinline__ void tube_fft_one(const FftJob<T>& jb, int part, long e,
                                             const typename Vec2<T>::type* __restrict__ tw) {
    const int i = (int)(e / jb.cols);
    tube_fft_rc<P, INV, T, POL>(jb, part, i, (int)(e - (long)i * jb.cols), tw);
}

// Workgroups go to the eight XCDs in turn (workgroup w to XCD w mod 8).  This
// maps w to a block index such that every XCD takes one contiguous run of
// blocks: a face is in general not aligned to 128-byte lines, so two
// neighbouring blocks share a line in every face they read or write, and that
// line then meets in one L2 instead of being fetched (or partly written back)
// by two.
__device__ __forceinline__ unsigned xcd_contiguous(unsigned w, unsigned n) {
    const unsigned q = n / 8, r = n % 8, x = w % 8;
    return x * q + (x < r ? x : r) + w / 8;
}

// Positions a transform of job jb runs over: rows x cols, or rows x dst_ld
// when a forward transform fills the padding columns.
template <bool INV, typename T>
__host__ __device__ inline long fft_positions(const FftJob<T>& jb) {
    return (long)jb.rows * (!INV && jb.fill && !jb.half ? jb.dst_ld : jb.cols);
}

// grid: x covers the positions of the largest job, y = 2 * njobs (job, CD part).
template <int P, bool INV, typename T>
__global__ void __launch_bounds__(256)
tube_fft_kernel(FftJobs2<T> jobs, const typename Vec2<T>::type* __restrict__ tw) {
    const unsigned b = xcd_contiguous(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const unsigned bx = b % gridDim.x, by = b / gridDim.x;
    const int job = by >> 1;
    const int part = by & 1;                         // 0: X1 (planes 0,1), 1: X2 (planes 2,3)
    const FftJob<T> jb = jobs.j[job];
    const long e = (long)bx * blockDim.x + threadIdx.x;
    if (e >= fft_positions<INV>(jb) || part >= jb.parts) return;
    if constexpr (!INV) {
        if (jb.fill && !jb.half) {
            const int i = (int)(e / jb.dst_ld);
            tube_fft_rc<P, false, T, 0, true>(jb, part, i, (int)(e - (long)i * jb.dst_ld), tw);
            return;
        }
    }
    tube_fft_one<P, INV, T>(jb, part, e, tw);
}

template <int P, bool INV, typename T>
hipError_t launch_p(const FftJob<T>* jobs, int njobs, const Twiddles& tw, hipStream_t stream) {
    FftJobs2<T> pk{};
    long maxc = 0;
    for (int q = 0; q < njobs; ++q) {
        pk.j[q] = jobs[q];
        maxc = fft_positions<INV>(jobs[q]) > maxc ? fft_positions<INV>(jobs[q]) : maxc;
    }
    const dim3 block(256);
    const dim3 grid((unsigned)((maxc + 255) / 256), 2 * njobs);
    const typename Vec2<T>::type* t;
    if constexpr (sizeof(T) == 4) t = tw.f32; else t = tw.f64;
    hipLaunchKernelGGL((tube_fft_kernel<P, INV, T>), grid, block, 0, stream, pk, t);
    return hipGetLastError();
}

}  // namespace detail
}  // namespace qt

// Register-resident lengths, split into groups that compile in separate
// translation units (fft_inst_*.hip): 7-smooth p, FP32 up to 128 and FP64 up
// to 64 (bounded by the VGPR budget of one tube per thread).
#define QT_FFT_SIZES_G0(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(12) X(14) X(15) \
    X(16) X(18) X(20) X(21) X(24) X(25) X(27) X(28) X(30) X(32)
#define QT_FFT_SIZES_G1(X) X(35) X(36) X(40) X(42) X(45) X(48) X(49) X(50)
#define QT_FFT_SIZES_G2(X) X(54) X(56) X(60) X(63) X(64)
#define QT_FFT_SIZES_G3(X) X(70) X(72) X(75) X(80) X(81) X(84) X(90)
#define QT_FFT_SIZES_G4(X) X(96) X(98) X(100) X(105)
#define QT_FFT_SIZES_G5(X) X(108) X(112) X(120) X(125) X(126) X(128)

#define QT_FFT_SIZES_F64(X) QT_FFT_SIZES_G0(X) QT_FFT_SIZES_G1(X) QT_FFT_SIZES_G2(X)
#define QT_FFT_SIZES_F32(X) QT_FFT_SIZES_F64(X) QT_FFT_SIZES_G3(X) QT_FFT_SIZES_G4(X) \
    QT_FFT_SIZES_G5(X)

#define QT_FFT_EXTERN_F32(P)                                                              \
    extern template hipError_t qt::detail::launch_p<P, false, float>(                    \
        const qt::FftJob<float>*, int, const qt::Twiddles&, hipStream_t);               \
    extern template hipError_t qt::detail::launch_p<P, true, float>(                     \
        const qt::FftJob<float>*, int, const qt::Twiddles&, hipStream_t);
#define QT_FFT_EXTERN_F64(P)                                                              \
    extern template hipError_t qt::detail::launch_p<P, false, double>(                   \
        const qt::FftJob<double>*, int, const qt::Twiddles&, hipStream_t);              \
    extern template hipError_t qt::detail::launch_p<P, true, double>(                    \
        const qt::FftJob<double>*, int, const qt::Twiddles&, hipStream_t);
#define QT_FFT_INST_F32(P)                                                                \
    template hipError_t qt::detail::launch_p<P, false, float>(                           \
        const qt::FftJob<float>*, int, const qt::Twiddles&, hipStream_t);               \
    template hipError_t qt::detail::launch_p<P, true, float>(                            \
        const qt::FftJob<float>*, int, const qt::Twiddles&, hipStream_t);
#define QT_FFT_INST_F64(P)                                                                \
    template hipError_t qt::detail::launch_p<P, false, double>(                          \
        const qt::FftJob<double>*, int, const qt::Twiddles&, hipStream_t);              \
    template hipError_t qt::detail::launch_p<P, true, double>(                           \
        const qt::FftJob<double>*, int, const qt::Twiddles&, hipStream_t);
