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
// that each face is read and written as T contiguous reals; the T tubes,
// zero-padded to M, live in LDS.  The length-M transforms run as a few
// passes of radix 16 (then 4 and 2 for the remaining factor): each thread
// takes R elements of a tube from LDS into registers, does the radix-R
// butterfly there, and writes them back, one barrier per pass.  The forward
// FFT_M is decimation in frequency (natural order in, digit-reversed order
// out); the chirp spectra are stored in that same digit-reversed order, so the
// pointwise product needs no reordering; the inverse FFT_M runs the mirrored
// decimation-in-time passes (digit-reversed in, natural order out).
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

// Radix plan of the length-M transforms (M = 2^logM): radix 16 while four or
// more factors of two remain, then 4 and 2.  Returns the number of passes.
__host__ __device__ __forceinline__ int radix_plan(int logM, int (&rs)[8]) {
    int n = 0, L = logM;
    while (L >= 4) { rs[n++] = 16; L -= 4; }
    if (L == 3) { rs[n++] = 4; rs[n++] = 2; }
    else if (L == 2) rs[n++] = 4;
    else if (L == 1) rs[n++] = 2;
    return n;
}

// Position at which the decimation-in-frequency passes leave frequency k:
// with k = sum_s r_s R_0 ... R_(s-1) (digits r_s < R_s), the position is
// sum_s r_s M / (R_0 ... R_s).
__device__ __forceinline__ int dif_position(int k, int logM) {
    int rs[8];
    const int np = radix_plan(logM, rs);
    int N = 1 << logM, base = 1, pos = 0;
    for (int s = 0; s < np; ++s) {
        N /= rs[s];
        const int r = (k / base) % rs[s];
        pos += r * N;
        base *= rs[s];
    }
    return pos;
}

// FP64 tables: chirp c_k (k < p); spectra of the forward and inverse chirp
// sequences b (length M) in natural order and in the order of the LDS
// kernel's passes; the twiddles exp(-2 pi i j / M) for j < M (and j < M/2).
struct TablePtrs {
    double2 *chirp, *hat_fwd, *hat_inv, *twm, *hatn_fwd, *hatn_inv, *twf;
    float2 *chirp32, *hat_fwd32, *hat_inv32, *twm32, *hatn_fwd32, *hatn_inv32, *twf32;
};

__global__ void bluestein_tables_kernel(int p, int M, TablePtrs tp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < p) {
        const long long k = t;
        const long long r = (k * k) % (2LL * p);
        double s, c;
        sincospi((double)r / (double)p, &s, &c);
        tp.chirp[t] = double2{c, s};
        tp.chirp32[t] = float2{(float)c, (float)s};
    }
    if (t < M) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)M, &s, &c);
        tp.twf[t] = double2{c, s};
        tp.twf32[t] = float2{(float)c, (float)s};
        if (t < M / 2) {
            tp.twm[t] = double2{c, s};
            tp.twm32[t] = float2{(float)c, (float)s};
        }
        // spectrum of b at frequency t: b_j = c_j (j < p), b_(M-j) = c_j (0 < j < p)
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
        int logM = 0;
        while ((1 << logM) < M) ++logM;
        const int pos = dif_position(t, logM);
        tp.hatn_fwd[t] = double2{fr, fi};
        tp.hatn_inv[t] = double2{ir, ii};
        tp.hatn_fwd32[t] = float2{(float)fr, (float)fi};
        tp.hatn_inv32[t] = float2{(float)ir, (float)ii};
        tp.hat_fwd[pos] = double2{fr, fi};
        tp.hat_inv[pos] = double2{ir, ii};
        tp.hat_fwd32[pos] = float2{(float)fr, (float)fi};
        tp.hat_inv32[pos] = float2{(float)ir, (float)ii};
    }
}

// DFT of 4 points in natural order, w = exp(-2 pi i / 4) (conjugate roots when INV).
template <bool INV, typename V>
__device__ __forceinline__ void dft4(V& x0, V& x1, V& x2, V& x3) {
    const V a{x0.x + x2.x, x0.y + x2.y}, b{x0.x - x2.x, x0.y - x2.y};
    const V c{x1.x + x3.x, x1.y + x3.y}, d{x1.x - x3.x, x1.y - x3.y};
    // -i d (forward) or +i d (inverse)
    const V e = INV ? V{-d.y, d.x} : V{d.y, -d.x};
    x0 = V{a.x + c.x, a.y + c.y};
    x2 = V{a.x - c.x, a.y - c.y};
    x1 = V{b.x + e.x, b.y + e.y};
    x3 = V{b.x - e.x, b.y - e.y};
}

// DFT of R = 2, 4 or 16 points in registers, natural order in and out.  The
// 16-point one is 4 x 4: DFTs over n2 of x[n1 + 4 n2], twiddles w16^(n1 k2),
// DFTs over n1, output X[k2 + 4 k1].
template <int R, bool INV, typename V>
__device__ __forceinline__ void dft_r(V (&x)[16], const V (&w16)[16]) {
    if constexpr (R == 2) {
        const V a = x[0], b = x[1];
        x[0] = V{a.x + b.x, a.y + b.y};
        x[1] = V{a.x - b.x, a.y - b.y};
    } else if constexpr (R == 4) {
        dft4<INV>(x[0], x[1], x[2], x[3]);
    } else {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) dft4<INV>(x[n1], x[n1 + 4], x[n1 + 8], x[n1 + 12]);
        // element n1 + 4 k2 now holds Y[n1][k2]; twiddle by w16^(n1 k2)
#pragma unroll
        for (int n1 = 1; n1 < 4; ++n1)
#pragma unroll
            for (int k2 = 1; k2 < 4; ++k2) {
                const V w = w16[n1 * k2];
                const V y = x[n1 + 4 * k2];
                const V wc = INV ? V{w.x, -w.y} : w;
                x[n1 + 4 * k2] = cmulv(y, wc);
            }
        V z[16];
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            V a = x[4 * k2], b = x[4 * k2 + 1], c = x[4 * k2 + 2], d = x[4 * k2 + 3];
            dft4<INV>(a, b, c, d);
            z[k2] = a;           // X[k2 + 4 k1] for k1 = 0..3
            z[k2 + 4] = b;
            z[k2 + 8] = c;
            z[k2 + 12] = d;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) x[q] = z[q];
    }
}

// One pass over every tube in LDS.  DIF (forward): butterfly, then twiddle
// w_N^(j r), stored at j + r N/R.  DIT (inverse): conj twiddle, inverse
// butterfly, stored at j + q N/R.  Span N of the pass, radix R.
template <int R, bool DIF, typename V>
__device__ __forceinline__ void fft_pass(V* buf, int row, int nt, int tpt, int logM, int logN,
                                         const V* __restrict__ tw, const V (&w16)[16]) {
    const int M = 1 << logM, N = 1 << logN, S = N / R;         // S = N / R: stride of a butterfly
    const int logS = logN - (R == 16 ? 4 : R == 4 ? 2 : 1);
    // consecutive threads take consecutive tubes (rows M + 1 apart): the
    // butterflies of one pass then hit distinct LDS banks across a wave
    const int nta = blockDim.x / tpt;
    const int t = threadIdx.x % nta, lt = threadIdx.x / nta;
    if (t >= nt) return;
    V* rowp = buf + (size_t)t * row;
    const int shift = logM - logN;                              // w_N^e = w_M^(e M/N)
    for (int bf = lt; bf < M / R; bf += tpt) {
        const int b = bf >> logS, j = bf & (S - 1);
        V* base = rowp + b * N + j;
        V x[16];
#pragma unroll
        for (int q = 0; q < R; ++q) x[q] = base[q * S];
        if constexpr (DIF) {
            dft_r<R, false>(x, w16);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int e = ((j * r) << shift) & (M - 1);
                const V w = e < M / 2 ? tw[e] : V{-tw[e - M / 2].x, -tw[e - M / 2].y};
                x[r] = cmulv(x[r], w);
            }
        } else {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int e = ((j * r) << shift) & (M - 1);
                const V w = e < M / 2 ? tw[e] : V{-tw[e - M / 2].x, -tw[e - M / 2].y};
                x[r] = cmulv(x[r], V{w.x, -w.y});
            }
            dft_r<R, true>(x, w16);
        }
#pragma unroll
        for (int q = 0; q < R; ++q) base[q * S] = x[q];
    }
}

template <bool DIF, typename V>
__device__ void fft_passes(V* buf, int row, int nt, int tpt, int logM, const V* __restrict__ tw,
                           const V (&w16)[16]) {
    int rs[8];
    const int np = radix_plan(logM, rs);
    for (int i = 0; i < np; ++i) {
        const int s = DIF ? i : np - 1 - i;
        int logN = logM;
        for (int u = 0; u < s; ++u) logN -= rs[u] == 16 ? 4 : rs[u] == 4 ? 2 : 1;
        if (rs[s] == 16) fft_pass<16, DIF>(buf, row, nt, tpt, logM, logN, tw, w16);
        else if (rs[s] == 4) fft_pass<4, DIF>(buf, row, nt, tpt, logM, logN, tw, w16);
        else fft_pass<2, DIF>(buf, row, nt, tpt, logM, logN, tw, w16);
        __syncthreads();
    }
}

// Layout of the dynamic LDS: ntubes rows of M + 1 complex values, then the
// M / 2 twiddles when they fit (twl = 1; else they are read from global
// memory), then the source and destination offsets of the ntubes tubes.
template <typename T, bool INV>
__global__ void __launch_bounds__(256)
bluestein_kernel(FftJob<T> j0, FftJob<T> j1, int p, int M, int logM, int ntubes, int tpt, int twl,
                 const typename V2<T>::type* __restrict__ chirp,
                 const typename V2<T>::type* __restrict__ hat,
                 const typename V2<T>::type* __restrict__ twm) {
    using V = typename V2<T>::type;
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    V* buf = reinterpret_cast<V*>(smem_raw);
    const int row = M + 1;
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

    V* tws = twl ? buf + (size_t)ntubes * row : nullptr;
    if (twl)
        for (int i = threadIdx.x; i < M / 2; i += blockDim.x) tws[i] = twm[i];
    const V* tw = twl ? tws : twm;
    // w16^k for the inner twiddles of the radix-16 butterfly: w_M^(k M / 16)
    V w16[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int e = (k * (M >> 4)) & (M - 1);
        w16[k] = M >= 16 ? (e < M / 2 ? twm[e] : V{-twm[e - M / 2].x, -twm[e - M / 2].y}) : V{1, 0};
    }

    // element offsets of the workgroup's tubes within a face, source and
    // destination (the one 64-bit division per tube happens here)
    long* soff = reinterpret_cast<long*>(buf + (size_t)ntubes * row + (twl ? M / 2 : 0));
    long* doff = soff + ntubes;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        const long e = e0 + t;
        const long i = e / jb.cols, c = e - i * jb.cols;
        soff[t] = i * jb.src_ld + c;
        doff[t] = i * jb.dst_ld + c;
    }
    // zeros from p up to M
    for (int idx = threadIdx.x; idx < nt * (M - p); idx += blockDim.x) {
        const int t = idx / (M - p), k = p + (idx - t * (M - p));
        buf[(size_t)t * row + k] = V{0, 0};
    }
    __syncthreads();
    // a_k = x_k conj(c_k) (c_k for INV) at natural index k: eight independent
    // loads per thread in flight before any is used
    constexpr int U = 8;
    const int total = p * nt;
    for (int base = 0; base < total; base += U * (int)blockDim.x) {
        V xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * (int)blockDim.x + threadIdx.x;
            xv[u] = V{0, 0};
            if (idx < total) {
                const int k = idx / nt, t = idx - k * nt;
                const long o = soff[t];
                if (!half) {
                    const T* sre = jb.src + (size_t)(2 * part) * splane + (size_t)k * sface + o;
                    xv[u] = V{sre[0], sre[splane]};
                } else if (!INV) {
                    xv[u] = V{jb.src[(size_t)k * sface + o], T(0)};
                } else {
                    const int kk = k < H ? k : p - k;       // X^[k] = conj(X^[p - k]) for k >= H
                    const T* sre = jb.src + (size_t)kk * sface + o;
                    xv[u] = V{sre[0], k < H ? sre[splane] : -sre[splane]};
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * (int)blockDim.x + threadIdx.x;
            if (idx < total) {
                const int k = idx / nt, t = idx - k * nt;
                const V ck = INV ? chirp[k] : conjv(chirp[k]);
                buf[(size_t)t * row + k] = cmulv(xv[u], ck);
            }
        }
    }
    __syncthreads();
    fft_passes<true>(buf, row, nt, tpt, logM, tw, w16);
    // pointwise product with the chirp spectrum (stored in the same order)
    for (int idx = threadIdx.x; idx < nt * M; idx += blockDim.x) {
        const int t = idx >> logM, f = idx & (M - 1);
        V* r = buf + (size_t)t * row;
        r[f] = cmulv(r[f], hat[f]);
    }
    __syncthreads();
    fft_passes<false>(buf, row, nt, tpt, logM, tw, w16);
    // X_f = conj(c_f) y_f / M  (c_f y_f / (M p) for the inverse)
    const T scale = INV ? T(1) / (T(M) * T(p)) : T(1) / T(M);
    const int nout = half && !INV ? H : p;
    for (int idx = threadIdx.x; idx < nout * nt; idx += blockDim.x) {
        const int f = idx / nt, t = idx - f * nt;
        const V cf = INV ? chirp[f] : conjv(chirp[f]);
        const V y = cmulv(buf[(size_t)t * row + f], cf);
        T* dre = jb.dst + (size_t)(2 * part) * dplane + (size_t)f * dface + doff[t];
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
    // chirp (p), four spectra (M each), twiddles (M / 2 and M), in FP64 and FP32
    return (4 * M + (size_t)p + M / 2 + M) * (sizeof(double2) + sizeof(float2));
}

void carve_bluestein_tables(int p, char* mem, BluesteinTables* bt) {
    bt->M = bluestein_length(p);
    double2* d = reinterpret_cast<double2*>(mem);
    bt->chirp64 = d; d += p;
    bt->hat_fwd64 = d; d += bt->M;
    bt->hat_inv64 = d; d += bt->M;
    bt->twm64 = d; d += bt->M / 2;
    bt->hatn_fwd64 = d; d += bt->M;
    bt->hatn_inv64 = d; d += bt->M;
    bt->twf64 = d; d += bt->M;
    float2* f = reinterpret_cast<float2*>(d);
    bt->chirp32 = f; f += p;
    bt->hat_fwd32 = f; f += bt->M;
    bt->hat_inv32 = f; f += bt->M;
    bt->twm32 = f; f += bt->M / 2;
    bt->hatn_fwd32 = f; f += bt->M;
    bt->hatn_inv32 = f; f += bt->M;
    bt->twf32 = f;
}

hipError_t launch_bluestein_tables(int p, const BluesteinTables& bt, hipStream_t stream) {
    const int n = bt.M > p ? bt.M : p;
    const TablePtrs tp{bt.chirp64, bt.hat_fwd64, bt.hat_inv64, bt.twm64, bt.hatn_fwd64, bt.hatn_inv64, bt.twf64,
                       bt.chirp32, bt.hat_fwd32, bt.hat_inv32, bt.twm32, bt.hatn_fwd32, bt.hatn_inv32, bt.twf32};
    hipLaunchKernelGGL(bluestein_tables_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, bt.M, tp);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bluestein(int p, bool inverse, const FftJob<T>* jobs, int njobs,
                            const BluesteinTables& bt, hipStream_t stream) {
    using V = typename V2<T>::type;
    if (njobs < 1 || njobs > 2) return hipErrorInvalidValue;
    {
        const hipError_t e = launch_bluestein_reg<T>(p, inverse, jobs, njobs, bt, stream);
        if (e != hipErrorNotSupported) return e;
    }
    const int M = bt.M;
    int logM = 0;
    while ((1 << logM) < M) ++logM;
    // tubes per workgroup: a power of two, up to 256, whose rows (M + 1
    // complex values each) fill at most 64 KB; threads per tube = 256 / tubes
    const size_t row_bytes = sizeof(V) * (size_t)(M + 1);
    int ntubes = 256;
    while (ntubes > 1 && (size_t)ntubes * row_bytes > 64 * 1024) ntubes >>= 1;
    const int tpt = 256 / ntubes;
    // the twiddle table goes to LDS beside the rows when the total fits
    const size_t tw_bytes = sizeof(V) * (size_t)(M / 2);
    const int twl = (size_t)ntubes * row_bytes + tw_bytes <= 128 * 1024 ? 1 : 0;
    const size_t smem = (size_t)ntubes * row_bytes + (twl ? tw_bytes : 0) + 2 * sizeof(long) * (size_t)ntubes;
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
                           ntubes, tpt, twl, chirp, hat, twm);
    else
        hipLaunchKernelGGL((bluestein_kernel<T, false>), grid, dim3(256), smem, stream, j0, j1, p, M, logM,
                           ntubes, tpt, twl, chirp, hat, twm);
    return hipGetLastError();
}

template hipError_t launch_bluestein<float>(int, bool, const FftJob<float>*, int, const BluesteinTables&,
                                            hipStream_t);
template hipError_t launch_bluestein<double>(int, bool, const FftJob<double>*, int, const BluesteinTables&,
                                             hipStream_t);

}  // namespace qt
