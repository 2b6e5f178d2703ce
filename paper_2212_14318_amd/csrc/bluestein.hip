// Tube FFT of any length p by Bluestein's algorithm (lengths without a
// register-resident kernel: primes and other non-7-smooth p, and p beyond the
// register budget).
//
// With c_k = exp(i pi k^2 / p) and f k = (f^2 + k^2 - (f - k)^2) / 2,
//   X[f] = sum_k x[k] w^(f k) = conj(c_f) sum_k (x[k] conj(c_k)) c_(f - k),
// a circular convolution of length M >= 2p - 1 (M a power of two) done as
// FFT_M, a pointwise product with the FFT of the chirp, and an inverse FFT_M.
// The inverse transform uses conj(c) and the factor 1/p.  The chirp
// (with k^2 reduced mod 2p in integers), its length-M spectra and the length-M
// twiddles are computed in FP64 on the device when the plan for p is created.
//
// Kernel: a workgroup takes T consecutive (i, j) positions of one CD part, so
// that each face is read and written as T contiguous reals; the T tubes, zero-
// padded to M, live in LDS (row stride M + 1 to spread banks) and go through
// radix-2 decimation-in-time passes in place (bit-reversed loading).
#include "qt_internal.h"

namespace qt {
namespace {

template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };

template <typename V>
__device__ __forceinline__ V cmulv(V a, V b) { return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename V>
__device__ __forceinline__ V conjv(V a) { return V{a.x, -a.y}; }

__device__ __forceinline__ unsigned bitrev(unsigned x, int bits) { return __brev(x) >> (32 - bits); }

// FP64 tables: chirp c_k (k < p), spectra of the forward and inverse chirp
// sequences b (length M), and the length-M twiddles exp(-2 pi i j / M), j < M/2.
__global__ void bluestein_tables_kernel(int p, int M, double2* chirp, double2* hat_fwd,
                                        double2* hat_inv, double2* twm, float2* chirp32,
                                        float2* hat_fwd32, float2* hat_inv32, float2* twm32) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < p) {
        const long long k = t;
        const long long r = (k * k) % (2LL * p);
        double s, c;
        sincospi((double)r / (double)p, &s, &c);
        chirp[t] = double2{c, s};
        chirp32[t] = float2{(float)c, (float)s};
    }
    if (t < M / 2) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)M, &s, &c);
        twm[t] = double2{c, s};
        twm32[t] = float2{(float)c, (float)s};
    }
    if (t < M) {
        // spectrum at frequency t of b: b_j = c_j (j < p), b_(M-j) = c_j (0 < j < p)
        double fr = 0, fi = 0, ir = 0, ii = 0;
        for (int j = 0; j < M; ++j) {
            int src = -1;
            if (j < p) src = j;
            else if (j > M - p) src = M - j;
            if (src < 0) continue;
            const long long kk = src;
            const long long r = (kk * kk) % (2LL * p);
            double cs, cc;
            sincospi((double)r / (double)p, &cs, &cc);            // c_src
            const long long e = ((long long)t * j) % M;
            double ws, wc;
            sincospi(-2.0 * (double)e / (double)M, &ws, &wc);     // exp(-2 pi i t j / M)
            fr += cc * wc - cs * ws;                               // c * w
            fi += cc * ws + cs * wc;
            ir += cc * wc + cs * ws;                               // conj(c) * w
            ii += cc * ws - cs * wc;
        }
        hat_fwd[t] = double2{fr, fi};
        hat_inv[t] = double2{ir, ii};
        hat_fwd32[t] = float2{(float)fr, (float)fi};
        hat_inv32[t] = float2{(float)ir, (float)ii};
    }
}

// In-place radix-2 DIT over `ntubes` rows of length M (row stride M + 1) in
// LDS; input in bit-reversed order, output in natural order.  conj_tw selects
// the inverse transform (unnormalised).
template <typename V>
__device__ void lds_fft(V* buf, int ntubes, int M, int logM, const V* __restrict__ twm, bool conj_tw) {
    const int half_total = ntubes * (M >> 1);
    for (int s = 1; s <= logM; ++s) {
        const int half = 1 << (s - 1);
        const int stride = M >> s;           // twiddle index step
        for (int b = threadIdx.x; b < half_total; b += blockDim.x) {
            const int t = b / (M >> 1), j = b - t * (M >> 1);
            const int group = j >> (s - 1), pos = j & (half - 1);
            const int i0 = group * 2 * half + pos, i1 = i0 + half;
            V w = twm[pos * stride];
            if (conj_tw) w.y = -w.y;
            V* row = buf + (size_t)t * (M + 1);
            const V u = row[i0];
            const V v = cmulv(row[i1], w);
            row[i0] = V{u.x + v.x, u.y + v.y};
            row[i1] = V{u.x - v.x, u.y - v.y};
        }
        __syncthreads();
    }
}

template <typename T, bool INV>
__global__ void __launch_bounds__(256)
bluestein_kernel(FftJob<T> j0, FftJob<T> j1, int p, int M, int logM, int ntubes,
                 const typename V2<T>::type* __restrict__ chirp,
                 const typename V2<T>::type* __restrict__ hat,
                 const typename V2<T>::type* __restrict__ twm) {
    using V = typename V2<T>::type;
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    V* buf = reinterpret_cast<V*>(smem_raw);
    const FftJob<T> jb = (blockIdx.y >> 1) ? j1 : j0;
    const int part = blockIdx.y & 1;
    const long count = (long)jb.rows * jb.cols;
    const long e0 = (long)blockIdx.x * ntubes;
    if (e0 >= count || part >= jb.parts) return;      // whole workgroup
    const int nt = (int)((count - e0) < ntubes ? (count - e0) : ntubes);
    const size_t sface = (size_t)jb.rows * jb.src_ld;
    const size_t dface = (size_t)jb.rows * jb.dst_ld;
    // Hermitian half spectrum (real tubes): H faces per plane on the Fourier side
    const int H = p / 2 + 1;
    const bool half = jb.half != 0;
    const size_t splane = (size_t)(half && INV ? H : p) * sface;
    const size_t dplane = (size_t)(half && !INV ? H : p) * dface;

    // zero the padded tubes, then load a_k = x_k conj(c_k) (c_k for INV) at rev(k)
    for (int idx = threadIdx.x; idx < ntubes * (M + 1); idx += blockDim.x) buf[idx] = V{0, 0};
    __syncthreads();
    for (int idx = threadIdx.x; idx < p * nt; idx += blockDim.x) {
        const int k = idx / nt, t = idx - k * nt;
        const long e = e0 + t;
        const int i = (int)(e / jb.cols), c = (int)(e - (long)i * jb.cols);
        V x;
        if (!half) {
            const T* sre = jb.src + (size_t)(2 * part) * splane + (size_t)k * sface + (size_t)i * jb.src_ld + c;
            x = V{sre[0], sre[splane]};
        } else if (!INV) {
            x = V{jb.src[(size_t)k * sface + (size_t)i * jb.src_ld + c], T(0)};
        } else {
            const int kk = k < H ? k : p - k;           // X^[k] = conj(X^[p - k]) for k >= H
            const T* sre = jb.src + (size_t)kk * sface + (size_t)i * jb.src_ld + c;
            x = V{sre[0], k < H ? sre[splane] : -sre[splane]};
        }
        const V ck = INV ? chirp[k] : conjv(chirp[k]);
        buf[(size_t)t * (M + 1) + bitrev((unsigned)k, logM)] = cmulv(x, ck);
    }
    __syncthreads();
    lds_fft(buf, nt, M, logM, twm, false);
    // pointwise product with the chirp spectrum, then back to bit-reversed order
    for (int idx = threadIdx.x; idx < nt * M; idx += blockDim.x) {
        const int t = idx / M, f = idx - t * M;
        V* row = buf + (size_t)t * (M + 1);
        row[f] = cmulv(row[f], hat[f]);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nt * M; idx += blockDim.x) {
        const int t = idx / M, f = idx - t * M;
        const int r = (int)bitrev((unsigned)f, logM);
        if (f < r) {
            V* row = buf + (size_t)t * (M + 1);
            const V a = row[f];
            row[f] = row[r];
            row[r] = a;
        }
    }
    __syncthreads();
    lds_fft(buf, nt, M, logM, twm, true);
    // X_f = conj(c_f) y_f / M  (c_f y_f / (M p) for the inverse)
    const T scale = INV ? T(1) / (T(M) * T(p)) : T(1) / T(M);
    const int nout = half && !INV ? H : p;
    for (int idx = threadIdx.x; idx < nout * nt; idx += blockDim.x) {
        const int f = idx / nt, t = idx - f * nt;
        const long e = e0 + t;
        const int i = (int)(e / jb.cols), c = (int)(e - (long)i * jb.cols);
        const V cf = INV ? chirp[f] : conjv(chirp[f]);
        const V y = cmulv(buf[(size_t)t * (M + 1) + f], cf);
        T* dre = jb.dst + (size_t)(2 * part) * dplane + (size_t)f * dface + (size_t)i * jb.dst_ld + c;
        const T yr = y.x * scale, yi = y.y * scale;
        if (half && INV) {                              // real output: one plane
            dre[0] = yr;
            continue;
        }
        if constexpr (!INV && sizeof(T) == 4) {
            if (jb.pack) {
                auto word = [](float x) {
                    const __bf16 hi = (__bf16)x;
                    const __bf16 lo = (__bf16)(x - (float)hi);
                    return (unsigned)__builtin_bit_cast(unsigned short, hi) |
                           ((unsigned)__builtin_bit_cast(unsigned short, lo) << 16);
                };
                reinterpret_cast<unsigned*>(dre)[0] = word(yr);
                reinterpret_cast<unsigned*>(dre)[dplane] = word(yi);
                continue;
            }
        }
        dre[0] = yr;
        dre[dplane] = yi;
    }
}

}  // namespace

int bluestein_length(int p) {
    int M = 1;
    while (M < 2 * p - 1) M <<= 1;
    return M;
}

size_t bluestein_tables_bytes(int p) {
    if (tube_fft_supported<double>(p)) return 0;   // FP64 covers fewer lengths than FP32
    const size_t M = (size_t)bluestein_length(p);
    // chirp (p), two spectra (M each), half-length twiddles (M / 2), in FP64 and FP32
    return (2 * M + (size_t)p + M / 2) * (sizeof(double2) + sizeof(float2));
}

void carve_bluestein_tables(int p, char* mem, BluesteinTables* bt) {
    bt->M = bluestein_length(p);
    double2* d = reinterpret_cast<double2*>(mem);
    bt->chirp64 = d; d += p;
    bt->hat_fwd64 = d; d += bt->M;
    bt->hat_inv64 = d; d += bt->M;
    bt->twm64 = d; d += bt->M / 2;
    float2* f = reinterpret_cast<float2*>(d);
    bt->chirp32 = f; f += p;
    bt->hat_fwd32 = f; f += bt->M;
    bt->hat_inv32 = f; f += bt->M;
    bt->twm32 = f;
}

hipError_t launch_bluestein_tables(int p, const BluesteinTables& bt, hipStream_t stream) {
    const int n = bt.M > p ? bt.M : p;
    hipLaunchKernelGGL(bluestein_tables_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, bt.M,
                       bt.chirp64, bt.hat_fwd64, bt.hat_inv64, bt.twm64, bt.chirp32, bt.hat_fwd32,
                       bt.hat_inv32, bt.twm32);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bluestein(int p, bool inverse, const FftJob<T>* jobs, int njobs,
                            const BluesteinTables& bt, hipStream_t stream) {
    using V = typename V2<T>::type;
    if (njobs < 1 || njobs > 2) return hipErrorInvalidValue;
    const int M = bt.M;
    int logM = 0;
    while ((1 << logM) < M) ++logM;
    // tubes per workgroup: fill ~48 KB of LDS, at most 64
    int ntubes = (int)((48 * 1024) / (sizeof(V) * (size_t)(M + 1)));
    if (ntubes > 64) ntubes = 64;
    if (ntubes < 1) ntubes = 1;
    const size_t smem = sizeof(V) * (size_t)ntubes * (M + 1);
    long maxc = 0;
    for (int q = 0; q < njobs; ++q) {
        const long c = (long)jobs[q].rows * jobs[q].cols;
        maxc = c > maxc ? c : maxc;
    }
    const FftJob<T> j0 = jobs[0], j1 = njobs == 2 ? jobs[1] : jobs[0];
    const dim3 grid((unsigned)((maxc + ntubes - 1) / ntubes), 2 * njobs);
    const V* chirp;
    const V* hat;
    const V* twm;
    if constexpr (sizeof(T) == 4) {
        chirp = bt.chirp32; hat = inverse ? bt.hat_inv32 : bt.hat_fwd32; twm = bt.twm32;
    } else {
        chirp = bt.chirp64; hat = inverse ? bt.hat_inv64 : bt.hat_fwd64; twm = bt.twm64;
    }
    if (smem > 64 * 1024) {
        hipError_t e = inverse
            ? hipFuncSetAttribute((const void*)bluestein_kernel<T, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)
            : hipFuncSetAttribute((const void*)bluestein_kernel<T, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    if (inverse)
        hipLaunchKernelGGL((bluestein_kernel<T, true>), grid, dim3(256), smem, stream, j0, j1, p, M, logM,
                           ntubes, chirp, hat, twm);
    else
        hipLaunchKernelGGL((bluestein_kernel<T, false>), grid, dim3(256), smem, stream, j0, j1, p, M, logM,
                           ntubes, chirp, hat, twm);
    return hipGetLastError();
}

template hipError_t launch_bluestein<float>(int, bool, const FftJob<float>*, int, const BluesteinTables&,
                                            hipStream_t);
template hipError_t launch_bluestein<double>(int, bool, const FftJob<double>*, int, const BluesteinTables&,
                                             hipStream_t);

}  // namespace qt
