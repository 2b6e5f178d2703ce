// Coupled facewise products in the Fourier domain (gfx950).
//
// Theorem 5.1 / Remark 5.1: after the tube FFT every frequency f is an
// independent complex product, except that j c = conj(c) j pairs f with
// g = -f mod p.  Written for the plain DFT:
//   C1^[f] = A1^[f] B1^[f] - A2^[f] conj(B2^[g])
//   C2^[f] = A1^[f] B2^[f] + A2^[f] conj(B1^[g])
// In real planes (r = real, i = imaginary part) each output plane is a sum of
// four real m x n by n x s products:
//   Re C1 = Ar1 Br1f - Ai1 Bi1f - Ar2 Br2g - Ai2 Bi2g
//   Im C1 = Ar1 Bi1f + Ai1 Br1f + Ar2 Bi2g - Ai2 Br2g
//   Re C2 = Ar1 Br2f - Ai1 Bi2f + Ar2 Br1g + Ai2 Bi1g
//   Im C2 = Ar1 Bi2f + Ai1 Br2f + Ai2 Br1g - Ar2 Bi1g
// i.e. 16 real products = 32 m n s flops per frequency (the count of the
// proof of Theorem 5.2, additions included).  Each workgroup keeps the four
// A planes and the eight B planes (f and g) of one k-chunk in LDS, so B is
// read once per output tile instead of once per output plane.
// Coupled facewise products in the Fourier domain: single-problem kernels.
// The tile routines (and the derivation of the coupled real products) live in
// facewise_impl.h, shared with the persistent batched kernel.
#include "facewise_impl.h"


namespace qt {
namespace {

using namespace detail;


// Workgroup -> (frequency, tile row, tile column) over a 1-D grid.
struct TileGrid {
    int tiles_m, tiles_n, p;
};

__device__ __forceinline__ bool tile_of_block(const TileGrid& t, int& f, int& tm, int& tn) {
    const int L = blockIdx.x;
    const int per = t.tiles_m * t.tiles_n;
    f = L / per;
    tm = (L - f * per) / t.tiles_n;
    tn = L - f * per - tm * t.tiles_n;
    return f < t.p;
}

template <int CFG>
__global__ void __launch_bounds__(64 * tile_waves(0, CFG))
facewise_f32_kernel(FacewiseArgs<float> a, TileGrid tg) {
    constexpr int MT = tile_mt(CFG), NT = tile_nt(CFG);
    __shared__ __attribute__((aligned(16))) V2Smem<MT, NT> sm;
    int f, tm, tn;
    if (!tile_of_block(tg, f, tm, tn)) return;
    tile_v2<0, MT, NT, tile_waves(0, CFG)>(a, f, tm * MT, tn * NT, 1.f, 1.f, sm);
}

template <typename H, int CFG>
__global__ void __launch_bounds__(64 * tile_waves(std::is_same<H, _Float16>::value ? 2 : 1, CFG))
facewise_split_kernel(FacewiseArgs<float> a, TileGrid tg, const float* __restrict__ scales) {
    constexpr int MT = tile_mt(CFG), NT = tile_nt(CFG);
    constexpr int MODE = std::is_same<H, _Float16>::value ? 2 : 1;
    __shared__ __attribute__((aligned(16))) V2Smem<MT, NT> sm;
    int f, tm, tn;
    if (!tile_of_block(tg, f, tm, tn)) return;
    float sa = 1.f, sb = 1.f;
    if (scales) {   // fp16: scales[f] for A^ at f, scales[p + f] for the B^ pair {f, -f}
        sa = scales[f];
        sb = scales[a.p + f];
    }
    tile_v2<MODE, MT, NT, tile_waves(MODE, CFG), plane_groups(MODE, CFG)>(a, f, tm * MT, tn * NT, sa, sb, sm);
}

// ---------------------------------------------------------------- FP64 MFMA
// 64 x 64 tile of all four output planes per workgroup on
// v_mfma_f64_16x16x4_f64 (4 waves in a 2 x 2 grid, each wave 32 x 32 as 2 x 2
// blocks of 16 x 16).  Operand layout of that instruction (checked on the
// device): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; register r of
// the accumulator holds D[4 r + l / 16][l % 16].  Each output plane is the
// signed sum of four real products (the expansion above), so a 4-deep k-step
// issues 16 MFMAs per 16 x 16 block; the signs are taken from negated A
// fragments.  Chunks of 8 k of the four A planes and the eight B planes (f and
// -f) go through LDS with out-of-range entries stored as zero (any lda, ldb:
// the Fourier rows of an FP64 product need no alignment).
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kF64T = 64, kF64K = 8;
constexpr int kF64ALd = kF64K + 1;          // A chunk row stride (doubles): 16 lanes, 16 distinct bank pairs
constexpr int kF64BLd = kF64T + 2;          // B chunk row stride (doubles)

__global__ void __launch_bounds__(256, 2) facewise_f64_kernel(FacewiseArgs<double> a) {
    __shared__ double sA[4][kF64T * kF64ALd];
    __shared__ double sB[8][kF64K * kF64BLd];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int n0 = blockIdx.x * kF64T, m0 = blockIdx.y * kF64T;
    const int f = blockIdx.z;
    const int g = (a.p - f) % a.p;
    const size_t pa = (size_t)a.p * a.m * a.lda;
    const size_t pb = (size_t)a.p * a.n * a.ldb;
    const size_t pc = (size_t)a.p * a.m * a.ldc;
    const double* Af = a.Ah + (size_t)f * a.m * a.lda;
    const double* Bf = a.Bh + (size_t)f * a.n * a.ldb;
    const double* Bg = a.Bh + (size_t)g * a.n * a.ldb;
    const int li = lane & 15, lk = lane >> 4;

    v4d acc[4][2][2];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[c][mb][nb] = v4d{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < a.n; k0 += kF64K) {
        __syncthreads();                     // the previous chunk is consumed
        // A: 64 rows x 8 k per plane (two entries per thread and plane)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int idx = tid + 256 * j;
            const int r = idx >> 3, k = idx & 7;
            const bool ok = (m0 + r < a.m) && (k0 + k < a.n);
            const size_t off = (size_t)(m0 + r) * a.lda + k0 + k;
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) sA[pl][r * kF64ALd + k] = ok ? Af[pl * pa + off] : 0.0;
        }
        // B: 8 k x 64 columns per plane, staged at f (planes 0..3) and at -f (4..7)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int idx = tid + 256 * j;
            const int k = idx >> 6, c = idx & 63;
            const bool ok = (k0 + k < a.n) && (n0 + c < a.s);
            const size_t off = (size_t)(k0 + k) * a.ldb + n0 + c;
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) {
                sB[pl][k * kF64BLd + c] = ok ? Bf[pl * pb + off] : 0.0;
                sB[4 + pl][k * kF64BLd + c] = ok ? Bg[pl * pb + off] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int ks = 0; ks < kF64K / 4; ++ks) {
            const int k = 4 * ks + lk;
            double ar1[2], ai1[2], ar2[2], ai2[2];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                const int r = wm * 32 + mb * 16 + li;
                ar1[mb] = sA[0][r * kF64ALd + k];
                ai1[mb] = sA[1][r * kF64ALd + k];
                ar2[mb] = sA[2][r * kF64ALd + k];
                ai2[mb] = sA[3][r * kF64ALd + k];
            }
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const int c = wn * 32 + nb * 16 + li;
                double b[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) b[q] = sB[q][k * kF64BLd + c];
                // b: B1r, B1i, B2r, B2i at f, then the same planes at -f
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) {
                    const double x1 = ar1[mb], y1 = ai1[mb], x2 = ar2[mb], y2 = ai2[mb];
                    // Re C1 = Ar1 B1r - Ai1 B1i - Ar2 B2r(-f) - Ai2 B2i(-f)
                    acc[0][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, b[0], acc[0][mb][nb], 0, 0, 0);
                    acc[0][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y1, b[1], acc[0][mb][nb], 0, 0, 0);
                    acc[0][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x2, b[6], acc[0][mb][nb], 0, 0, 0);
                    acc[0][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y2, b[7], acc[0][mb][nb], 0, 0, 0);
                    // Im C1 = Ar1 B1i + Ai1 B1r + Ar2 B2i(-f) - Ai2 B2r(-f)
                    acc[1][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, b[1], acc[1][mb][nb], 0, 0, 0);
                    acc[1][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(y1, b[0], acc[1][mb][nb], 0, 0, 0);
                    acc[1][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(x2, b[7], acc[1][mb][nb], 0, 0, 0);
                    acc[1][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y2, b[6], acc[1][mb][nb], 0, 0, 0);
                    // Re C2 = Ar1 B2r - Ai1 B2i + Ar2 B1r(-f) + Ai2 B1i(-f)
                    acc[2][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, b[2], acc[2][mb][nb], 0, 0, 0);
                    acc[2][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y1, b[3], acc[2][mb][nb], 0, 0, 0);
                    acc[2][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(x2, b[4], acc[2][mb][nb], 0, 0, 0);
                    acc[2][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(y2, b[5], acc[2][mb][nb], 0, 0, 0);
                    // Im C2 = Ar1 B2i + Ai1 B2r + Ai2 B1r(-f) - Ar2 B1i(-f)
                    acc[3][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, b[3], acc[3][mb][nb], 0, 0, 0);
                    acc[3][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(y1, b[2], acc[3][mb][nb], 0, 0, 0);
                    acc[3][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(y2, b[4], acc[3][mb][nb], 0, 0, 0);
                    acc[3][mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x2, b[5], acc[3][mb][nb], 0, 0, 0);
                }
            }
        }
    }
    double* Cf = a.Ch + (size_t)f * a.m * a.ldc;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int col = n0 + wn * 32 + nb * 16 + li;
            if (col >= a.s) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + mb * 16 + 4 * r + lk;
                if (row >= a.m) continue;
#pragma unroll
                for (int c = 0; c < 4; ++c) Cf[c * pc + (size_t)row * a.ldc + col] = acc[c][mb][nb][r];
            }
        }
}

// ------------------------------------------------------ complex products
// A2 = B2 = 0 (complex tensors, the paper's Algorithm 2.1 / Proposition 2.1
// case): C^[f] = A^[f] B^[f] with no coupling, two A planes and two B planes
// per chunk.  8 waves (4 x 2).  256 x 128 (96 KB of LDS, each wave 64 x 64)
// holds as many products per chunk and barrier as the quaternion tile;
// 128 x 128 (64 KB, two workgroups per CU) is used when the large tiles
// would fill the chip fewer than kCxWaves times.
constexpr int kCxWaves = 3;

// The split-bf16 128 x 128 instance is held to 128 VGPRs (4 waves per SIMD,
// so two workgroups share a CU and cover each other's barrier waits; a few
// values spill to scratch): 5% faster on the 17-frequency real product.
template <int MODE, int MT, int NT>
__global__ void __launch_bounds__(512, (MODE != 0 && MT == 128 ? 4 : 2))
facewise_cx_kernel(FacewiseArgs<float> a, TileGrid tg, const float* __restrict__ scales) {
    __shared__ __attribute__((aligned(16))) V2Smem<MT, NT, true> sm;
    int f, tm, tn;
    if (!tile_of_block(tg, f, tm, tn)) return;
    float sa = 1.f, sb = 1.f;
    if (MODE == 2) {     // fp16: scales[f] for A^, scales[p + f] for B^ at f
        sa = scales[f];
        sb = scales[a.p + f];
    }
    tile_v2<MODE, MT, NT, 8, false, true>(a, f, tm * MT, tn * NT, sa, sb, sm);
}

// ---------------------------------------------------- narrow products (s <= 4)
// A block-circulant quaternion matrix times a few tube vectors (s <= 4; the
// circulant mat-vec of Theorems 4.2 / 4.3 when m = n = s = 1): the coupled
// product is then bound by reading A^ once from HBM, which a 64-column MFMA
// tile would do with ~1/64 of its work useful.  FP32 VALU: a block owns 16
// output rows of one frequency (4 waves x 4 rows), stages B^[f] and B^[-f]
// for k-tiles of 256 in LDS, and reads A^ coalesced along k; lanes own k,
// and the 64 partial sums of every output meet in a wave reduction.  Split-
// bf16 operand words are decoded to hi + lo (exact in FP32).
constexpr int kNarrowRows = 16, kNarrowK = 256;

template <bool WORDS>
__device__ __forceinline__ float operand(float x) {
    if constexpr (WORDS) {
        const unsigned w = __builtin_bit_cast(unsigned, x);
        return __builtin_bit_cast(float, w << 16) + __builtin_bit_cast(float, w & 0xFFFF0000u);
    } else {
        return x;
    }
}

template <int S, bool WORDS>
__global__ void __launch_bounds__(256) facewise_narrow_kernel(FacewiseArgs<float> a) {
    __shared__ float sb[8][S][kNarrowK];          // planes 0..3 = B^[f], 4..7 = B^[-f]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int f = blockIdx.y, g = (a.p - f) % a.p;
    const int row0 = blockIdx.x * kNarrowRows + wave * 4;
    const size_t pa = (size_t)a.p * a.m * a.lda, pb = (size_t)a.p * a.n * a.ldb;
    const size_t pc = (size_t)a.p * a.m * a.ldc;
    const float* Af = a.Ah + (size_t)f * a.m * a.lda;
    const float* Bf = a.Bh + (size_t)f * a.n * a.ldb;
    const float* Bg = a.Bh + (size_t)g * a.n * a.ldb;
    float c[4][4][S];                              // [row][plane][column]
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < S; ++j) c[r][q][j] = 0.f;
    for (int k0 = 0; k0 < a.n; k0 += kNarrowK) {
        __syncthreads();                           // previous tile consumed
        for (int e = threadIdx.x; e < 8 * S * kNarrowK; e += 256) {
            const int kk = e % kNarrowK, j = (e / kNarrowK) % S, q = e / (kNarrowK * S);
            const int k = k0 + kk;
            float v = 0.f;
            if (k < a.n) v = operand<WORDS>((q < 4 ? Bf : Bg)[(q & 3) * pb + (size_t)k * a.ldb + j]);
            sb[q][j][kk] = v;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kNarrowK / 64; ++u) {
            const int kk = u * 64 + lane, k = k0 + kk;
            if (k >= a.n) break;                   // k >= n only in the last tile
            float b[8][S];
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int j = 0; j < S; ++j) b[q][j] = sb[q][j][kk];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = row0 + r;
                if (i >= a.m) break;
                const float* Ai = Af + (size_t)i * a.lda + k;
                const float ar1 = operand<WORDS>(Ai[0]), ai1 = operand<WORDS>(Ai[pa]);
                const float ar2 = operand<WORDS>(Ai[2 * pa]), ai2 = operand<WORDS>(Ai[3 * pa]);
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    // C1 = A1 B1^[f] - A2 conj(B2^[g]),  C2 = A1 B2^[f] + A2 conj(B1^[g])
                    c[r][0][j] += ar1 * b[0][j] - ai1 * b[1][j] - ar2 * b[6][j] - ai2 * b[7][j];
                    c[r][1][j] += ar1 * b[1][j] + ai1 * b[0][j] + ar2 * b[7][j] - ai2 * b[6][j];
                    c[r][2][j] += ar1 * b[2][j] - ai1 * b[3][j] + ar2 * b[4][j] + ai2 * b[5][j];
                    c[r][3][j] += ar1 * b[3][j] + ai1 * b[2][j] + ai2 * b[4][j] - ar2 * b[5][j];
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < S; ++j) {
                float v = c[r][q][j];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                c[r][q][j] = v;
            }
    if (lane == 0) {
        float* Cf = a.Ch + (size_t)f * a.m * a.ldc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = row0 + r;
            if (i >= a.m) break;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int j = 0; j < S; ++j) Cf[q * pc + (size_t)i * a.ldc + j] = c[r][q][j];
        }
    }
}

// ------------------------------------------------ fp16 power-of-two scales
// fp16 has a 5-bit exponent, so the split operands are scaled by a power of
// two before the split: per frequency f, sa[f] for the four planes of A^[f],
// and sb[f] for the eight B planes of the pair {f, -f}, chosen so that the
// largest magnitude lands in [2^14, 2^15) (hi <= 65504 with room, lo keeps
// 11 more bits).  Powers of two make the scaling exact; the product is
// multiplied back by 1 / sa and then by 1 / sb.  Max-abs is a deterministic two-pass
// reduction (per-block partials, then one thread per frequency).
__global__ void __launch_bounds__(256)
absmax_partial_kernel(const float* __restrict__ X, int rows, int cols, int ld, int p, int nblk,
                      float* __restrict__ partial, int planes) {
    __shared__ float red[256];
    const int f = blockIdx.y;
    const size_t face = (size_t)rows * ld, plane = (size_t)p * face;
    const float* Xf = X + (size_t)f * face;
    float mx = 0.f;
    const long count = (long)rows * cols;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < count; e += (long)nblk * 256) {
        const int i = (int)(e / cols), j = (int)(e - (long)i * cols);
        const size_t off = (size_t)i * ld + j;
        for (int c = 0; c < planes; ++c) mx = fmaxf(mx, fabsf(Xf[c * plane + off]));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)f * nblk + blockIdx.x] = red[0];
}

// paired: the B^ scale covers the pair {f, -f} that the coupled product
// stages together; complex products take B^[f] alone.
__global__ void fp16_scales_kernel(const float* __restrict__ pa, int nba, const float* __restrict__ pb,
                                   int nbb, int p, float* __restrict__ scales, int paired) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= p) return;
    const int g = paired ? (p - f) % p : f;
    float ma = 0.f, mb = 0.f;
    for (int b = 0; b < nba; ++b) ma = fmaxf(ma, pa[(size_t)f * nba + b]);
    for (int b = 0; b < nbb; ++b) mb = fmaxf(mb, fmaxf(pb[(size_t)f * nbb + b], pb[(size_t)g * nbb + b]));
    scales[f] = pow2_scale(ma);
    scales[p + f] = pow2_scale(mb);
}

}  // namespace

int fp16_partial_blocks(long rows, long cols) {
    const long b = (rows * cols + 255) / 256;
    return (int)(b < 64 ? b : 64);
}

hipError_t launch_fp16_scales(const FacewiseArgs<float>& a, float* partials, float* scales,
                              hipStream_t stream, int planes) {
    const int nba = fp16_partial_blocks(a.m, a.n), nbb = fp16_partial_blocks(a.n, a.s);
    float* pa = partials;
    float* pb = partials + (size_t)a.p * nba;
    hipLaunchKernelGGL(absmax_partial_kernel, dim3(nba, a.p), dim3(256), 0, stream, a.Ah, a.m, a.n, a.lda,
                       a.p, nba, pa, planes);
    hipLaunchKernelGGL(absmax_partial_kernel, dim3(nbb, a.p), dim3(256), 0, stream, a.Bh, a.n, a.s, a.ldb,
                       a.p, nbb, pb, planes);
    hipLaunchKernelGGL(fp16_scales_kernel, dim3((a.p + 255) / 256), dim3(256), 0, stream, pa, nba, pb, nbb,
                       a.p, scales, planes == 4 ? 1 : 0);
    return hipGetLastError();
}

template <int CFG>
static hipError_t launch_cfg(const FacewiseArgs<float>& a, int precision, const float* scales,
                             hipStream_t stream) {
    constexpr int MT = tile_mt(CFG), NT = tile_nt(CFG);
    const int tiles_m = (a.m + MT - 1) / MT;
    const int tiles_n = (a.s + NT - 1) / NT;
    const TileGrid tg{tiles_m, tiles_n, a.p};
    const dim3 grid((unsigned)(tiles_m * tiles_n * a.p)), block(64 * tile_waves(precision, CFG));
    if (precision == 0) {
        hipLaunchKernelGGL((facewise_f32_kernel<CFG>), grid, block, 0, stream, a, tg);
    } else if (precision == 1) {
        hipLaunchKernelGGL((facewise_split_kernel<__bf16, CFG>), grid, block, 0, stream, a,
                           tg, (const float*)nullptr);
    } else if (precision == 2) {
        if (!scales) return hipErrorInvalidValue;
        hipLaunchKernelGGL((facewise_split_kernel<_Float16, CFG>), grid, block, 0, stream, a,
                           tg, scales);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template <int S>
static hipError_t launch_narrow(const FacewiseArgs<float>& a, bool words, hipStream_t stream) {
    const dim3 grid((unsigned)((a.m + kNarrowRows - 1) / kNarrowRows), (unsigned)a.p), block(256);
    if (words) hipLaunchKernelGGL((facewise_narrow_kernel<S, true>), grid, block, 0, stream, a);
    else hipLaunchKernelGGL((facewise_narrow_kernel<S, false>), grid, block, 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_facewise_f32(const FacewiseArgs<float>& a, int precision, hipStream_t stream,
                               int tile_cfg, const float* scales) {
    if (precision < 0 || precision > 2) return hipErrorNotSupported;
    if (a.s <= kNarrowMaxS) {
        // HBM-bound shape: FP32 VALU on the (decoded) operands, any precision
        const bool words = precision == 1;
        switch (a.s) {
            case 1: return launch_narrow<1>(a, words, stream);
            case 2: return launch_narrow<2>(a, words, stream);
            case 3: return launch_narrow<3>(a, words, stream);
            default: return launch_narrow<4>(a, words, stream);
        }
    }
    switch (tile_cfg) {
        case TILE_128x64: return launch_cfg<TILE_128x64>(a, precision, scales, stream);
        case TILE_64x128: return launch_cfg<TILE_64x128>(a, precision, scales, stream);
        case TILE_64x64: return launch_cfg<TILE_64x64>(a, precision, scales, stream);
        case TILE_32x64: return launch_cfg<TILE_32x64>(a, precision, scales, stream);
        default: return hipErrorInvalidValue;
    }
}

template <int MT, int NT>
hipError_t launch_cx(const FacewiseArgs<float>& a, int precision, hipStream_t stream, const float* scales) {
    const int tiles_m = (a.m + MT - 1) / MT, tiles_n = (a.s + NT - 1) / NT;
    const TileGrid tg{tiles_m, tiles_n, a.p};
    const dim3 grid((unsigned)(tiles_m * tiles_n * a.p)), block(512);
    if (precision == 0) hipLaunchKernelGGL((facewise_cx_kernel<0, MT, NT>), grid, block, 0, stream, a, tg, scales);
    else if (precision == 1) hipLaunchKernelGGL((facewise_cx_kernel<1, MT, NT>), grid, block, 0, stream, a, tg, scales);
    else hipLaunchKernelGGL((facewise_cx_kernel<2, MT, NT>), grid, block, 0, stream, a, tg, scales);
    return hipGetLastError();
}

static int cx_big_tile(int m, int s, int p, int cus) {
    const long big = (long)((m + 255) / 256) * ((s + 127) / 128) * p;
    return big >= (long)kCxWaves * cus ? 1 : 0;
}

hipError_t launch_facewise_cx(const FacewiseArgs<float>& a, int precision, hipStream_t stream,
                              const float* scales) {
    if (precision < 0 || precision > 2) return hipErrorNotSupported;
    if (precision == 2 && !scales) return hipErrorInvalidValue;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    return cx_big_tile(a.m, a.s, a.p, cus) ? launch_cx<256, 128>(a, precision, stream, scales)
                                           : launch_cx<128, 128>(a, precision, stream, scales);
}

hipError_t launch_facewise_f64(const FacewiseArgs<double>& a, hipStream_t stream) {
    hipLaunchKernelGGL(facewise_f64_kernel, dim3((a.s + kF64T - 1) / kF64T, (a.m + kF64T - 1) / kF64T, a.p),
                       dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace qt
