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
#include "qt_internal.h"

namespace qt {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- FP32 MFMA
// Workgroup tile MT x NT of all four output planes; 4 waves in a 2 x 2 grid,
// each wave 64 x 32 = two 32x32 MFMA blocks (v_mfma_f32_32x32x2_f32).
constexpr int MT = 128, NT = 64, KT = 16;
constexpr int APAD = 4;

__global__ void __launch_bounds__(256)
facewise_f32_mfma(FacewiseArgs<float> a, int tiles_n) {
    __shared__ float sA[4][KT][MT + APAD];   // k-major A chunk (4 planes)
    __shared__ float sB[8][KT][NT];          // B chunk: 4 planes at f, 4 at g

    const int tid = threadIdx.x;
    const int f = blockIdx.y;
    const int g = (a.p - f) % a.p;
    const int tm = blockIdx.x / tiles_n;
    const int tn = blockIdx.x - tm * tiles_n;
    const int m0 = tm * MT, n0 = tn * NT;

    const size_t pa = (size_t)a.p * a.m * a.lda;
    const size_t pb = (size_t)a.p * a.n * a.ldb;
    const size_t pc = (size_t)a.p * a.m * a.ldc;
    const float* Af = a.Ah + (size_t)f * a.m * a.lda;
    const float* Bf = a.Bh + (size_t)f * a.n * a.ldb;
    const float* Bg = a.Bh + (size_t)g * a.n * a.ldb;

    float4 ra[8], rb[8];

    auto load_global = [&](int k0) {
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int idx = tid + 256 * it;
            const int pl = idx >> 9, rem = idx & 511;
            const int row = rem >> 2, kq = rem & 3;
            const int grow = m0 + row, gk = k0 + 4 * kq;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (grow < a.m && gk < a.n) {
                v = *reinterpret_cast<const float4*>(Af + pl * pa + (size_t)grow * a.lda + gk);
                if (gk + 1 >= a.n) v.y = 0.f;
                if (gk + 2 >= a.n) v.z = 0.f;
                if (gk + 3 >= a.n) v.w = 0.f;
            }
            ra[it] = v;
        }
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int idx = tid + 256 * it;
            const int pl = idx >> 8, rem = idx & 255;
            const int kr = rem >> 4, nq = rem & 15;
            const int gk = k0 + kr, gc = n0 + 4 * nq;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gk < a.n && gc < a.s) {
                const float* src = (pl < 4 ? Bf + pl * pb : Bg + (pl - 4) * pb);
                v = *reinterpret_cast<const float4*>(src + (size_t)gk * a.ldb + gc);
                if (gc + 1 >= a.s) v.y = 0.f;
                if (gc + 2 >= a.s) v.z = 0.f;
                if (gc + 3 >= a.s) v.w = 0.f;
            }
            rb[it] = v;
        }
    };
    auto store_lds = [&]() {
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int idx = tid + 256 * it;
            const int pl = idx >> 9, rem = idx & 511;
            const int row = rem >> 2, kq = rem & 3;
            sA[pl][4 * kq + 0][row] = ra[it].x;
            sA[pl][4 * kq + 1][row] = ra[it].y;
            sA[pl][4 * kq + 2][row] = ra[it].z;
            sA[pl][4 * kq + 3][row] = ra[it].w;
        }
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int idx = tid + 256 * it;
            const int pl = idx >> 8, rem = idx & 255;
            const int kr = rem >> 4, nq = rem & 15;
            *reinterpret_cast<float4*>(&sB[pl][kr][4 * nq]) = rb[it];
        }
    };

    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int lr = lane & 31, lk = lane >> 5;

    v16f acc[4][2];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[c][mb][r] = 0.f;

    load_global(0);
    store_lds();
    __syncthreads();
    for (int k0 = 0; k0 < a.n; k0 += KT) {
        const bool more = k0 + KT < a.n;
        if (more) load_global(k0 + KT);
#pragma unroll
        for (int kk = 0; kk < KT / 2; ++kk) {
            const int k = 2 * kk + lk;
            float bf[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) bf[c] = sB[c][k][wn * 32 + lr];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                const int r = wm * 64 + mb * 32 + lr;
                const float ar1 = sA[0][k][r], ai1 = sA[1][k][r];
                const float ar2 = sA[2][k][r], ai2 = sA[3][k][r];
                v16f c0 = acc[0][mb], c1 = acc[1][mb], c2 = acc[2][mb], c3 = acc[3][mb];
                c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar1, bf[0], c0, 0, 0, 0);
                c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai1, bf[1], c0, 0, 0, 0);
                c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(-ar2, bf[6], c0, 0, 0, 0);
                c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai2, bf[7], c0, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar1, bf[1], c1, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai1, bf[0], c1, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar2, bf[7], c1, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai2, bf[6], c1, 0, 0, 0);
                c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar1, bf[2], c2, 0, 0, 0);
                c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai1, bf[3], c2, 0, 0, 0);
                c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar2, bf[4], c2, 0, 0, 0);
                c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai2, bf[5], c2, 0, 0, 0);
                c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar1, bf[3], c3, 0, 0, 0);
                c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai1, bf[2], c3, 0, 0, 0);
                c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai2, bf[4], c3, 0, 0, 0);
                c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(-ar2, bf[5], c3, 0, 0, 0);
                acc[0][mb] = c0; acc[1][mb] = c1; acc[2][mb] = c2; acc[3][mb] = c3;
            }
        }
        __syncthreads();
        if (more) {
            store_lds();
            __syncthreads();
        }
    }

    // 32x32 f32 accumulator layout: register r of lane l holds
    // row 8 (r / 4) + 4 (l / 32) + (r % 4), column l % 32.
    float* Cf = a.Ch + (size_t)f * a.m * a.ldc;
    const int col = n0 + wn * 32 + lr;
    if (col < a.s) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * 64 + mb * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
                if (row < a.m) {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        Cf[c * pc + (size_t)row * a.ldc + col] = acc[c][mb][r];
                }
            }
    }
}

// ------------------------------------------------------ split bf16 / fp16
// x = hi + lo with hi = rn(x), lo = rn(x - hi) in a 16-bit format; a real
// product X Y is taken as Xhi Yhi + Xhi Ylo + Xlo Yhi (the dropped Xlo Ylo is
// ~2^-16 relative for bf16), each on v_mfma_f32_32x32x16_{bf16,f16} with FP32
// accumulation.  The split happens while a chunk is staged into LDS, so the
// Fourier-domain tensors stay FP32 in HBM (same bytes as the FP32 path).
//
// The coupled products are rewritten as two plain complex products,
//   C1^ = A1^ B1^[f] + A2^ D,  D = -conj(B2^[g]),
//   C2^ = A1^ B2^[f] + A2^ E,  E =  conj(B1^[g]),
// whose signs are applied to the B chunk when it is staged, so that every real
// term adds: Re = Xr Yr + (-Xi) Yi, Im = Xr Yi + Xi Yr.
//
// LDS holds both operands k-contiguous (a row of A, a column of B): 16 hi
// values, 16 lo values and 8 padding values per row/column, so one lane reads
// its 8 consecutive k of hi (or lo) with a single 16-byte load.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));

template <typename H> struct SplitTypes;
template <> struct SplitTypes<__bf16> { using v8 = v8bf; using v4 = v4bf; };
template <> struct SplitTypes<_Float16> { using v8 = v8h; using v4 = v4h; };

template <typename H>
__device__ __forceinline__ v16f mfma16(typename SplitTypes<H>::v8 a, typename SplitTypes<H>::v8 b, v16f c);
template <>
__device__ __forceinline__ v16f mfma16<__bf16>(v8bf a, v8bf b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ v16f mfma16<_Float16>(v8h a, v8h b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

template <typename V8>
__device__ __forceinline__ V8 neg8(V8 x) {
    // flip the sign bit of all eight 16-bit lanes (exact negation)
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    u4 b = __builtin_bit_cast(u4, x);
    b ^= 0x80008000u;
    return __builtin_bit_cast(V8, b);
}

constexpr int SRS = 40;   // LDS row stride of the split kernel, in 16-bit values

// scale: power-of-two scale applied before the split (1 for bf16, whose range
// equals FP32's; per-frequency for fp16, see launch_facewise_f32).
template <typename H>
__global__ void __launch_bounds__(256)
facewise_split_mfma(FacewiseArgs<float> a, int tiles_n, const float* __restrict__ scales) {
    using V8 = typename SplitTypes<H>::v8;
    using V4 = typename SplitTypes<H>::v4;
    __shared__ __attribute__((aligned(16))) H sA[4][MT][SRS];
    __shared__ __attribute__((aligned(16))) H sB[8][NT][SRS];

    const int tid = threadIdx.x;
    const int f = blockIdx.y;
    const int g = (a.p - f) % a.p;
    const int tm = blockIdx.x / tiles_n;
    const int tn = blockIdx.x - tm * tiles_n;
    const int m0 = tm * MT, n0 = tn * NT;
    float sa = 1.f, sb = 1.f, out_scale = 1.f;
    if (scales) {   // fp16: scales[f] for A^ at f, scales[p + f] for the B^ pair {f, g}
        sa = scales[f];
        sb = scales[a.p + f];
        out_scale = 1.f / (sa * sb);
    }

    const size_t pa = (size_t)a.p * a.m * a.lda;
    const size_t pb = (size_t)a.p * a.n * a.ldb;
    const size_t pc = (size_t)a.p * a.m * a.ldc;
    const float* Af = a.Ah + (size_t)f * a.m * a.lda;
    const float* Bf = a.Bh + (size_t)f * a.n * a.ldb;
    const float* Bg = a.Bh + (size_t)g * a.n * a.ldb;

    // A chunk: plane = tid / 64; 4 lanes cover the 16 k of one row
    const int a_pl = tid >> 6, a_kq = tid & 3, a_r0 = (tid & 63) >> 2;
    // B chunk: plane = tid / 32; 16 lanes cover 64 columns, 2 halves of 8 k rows
    const int b_pl = tid >> 5, b_cq = tid & 15, b_kh = (tid & 31) >> 4;
    // source plane and sign of the staged B plane (0..3: B^[f]; 4..7: D, E from B^[g])
    const int b_src = b_pl < 4 ? b_pl : (b_pl == 4 ? 2 : b_pl == 5 ? 3 : b_pl == 6 ? 0 : 1);
    const float b_sign = (b_pl == 4 || b_pl == 7) ? -1.f : 1.f;
    const float* b_base = (b_pl < 4 ? Bf : Bg) + b_src * pb;

    float4 ra[8], rb[8];
    auto load_global = [&](int k0) {
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int grow = m0 + a_r0 + 16 * h, gk = k0 + 4 * a_kq;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (grow < a.m && gk < a.n) {
                v = *reinterpret_cast<const float4*>(Af + a_pl * pa + (size_t)grow * a.lda + gk);
                if (gk + 1 >= a.n) v.y = 0.f;
                if (gk + 2 >= a.n) v.z = 0.f;
                if (gk + 3 >= a.n) v.w = 0.f;
            }
            ra[h] = v;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int gk = k0 + 8 * b_kh + j, gc = n0 + 4 * b_cq;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gk < a.n && gc < a.s) {
                v = *reinterpret_cast<const float4*>(b_base + (size_t)gk * a.ldb + gc);
                if (gc + 1 >= a.s) v.y = 0.f;
                if (gc + 2 >= a.s) v.z = 0.f;
                if (gc + 3 >= a.s) v.w = 0.f;
            }
            rb[j] = v;
        }
    };
    auto store_lds = [&]() {
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const float x[4] = {ra[h].x * sa, ra[h].y * sa, ra[h].z * sa, ra[h].w * sa};
            V4 hi, lo;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                hi[q] = (H)x[q];
                lo[q] = (H)(x[q] - (float)hi[q]);
            }
            H* row = &sA[a_pl][a_r0 + 16 * h][0];
            *reinterpret_cast<V4*>(row + 4 * a_kq) = hi;
            *reinterpret_cast<V4*>(row + 16 + 4 * a_kq) = lo;
        }
        const float bs = b_sign * sb;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            V8 hi, lo;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float x = (c == 0 ? rb[j].x : c == 1 ? rb[j].y : c == 2 ? rb[j].z : rb[j].w) * bs;
                hi[j] = (H)x;
                lo[j] = (H)(x - (float)hi[j]);
            }
            H* col = &sB[b_pl][4 * b_cq + c][0];
            *reinterpret_cast<V8*>(col + 8 * b_kh) = hi;
            *reinterpret_cast<V8*>(col + 16 + 8 * b_kh) = lo;
        }
    };

    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int lr = lane & 31, lk = lane >> 5;

    v16f acc[4][2];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[c][mb][r] = 0.f;

    load_global(0);
    store_lds();
    __syncthreads();
    for (int k0 = 0; k0 < a.n; k0 += KT) {
        const bool more = k0 + KT < a.n;
        if (more) load_global(k0 + KT);
        V8 bh[8], bl[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const H* col = &sB[c][wn * 32 + lr][0];
            bh[c] = *reinterpret_cast<const V8*>(col + 8 * lk);
            bl[c] = *reinterpret_cast<const V8*>(col + 16 + 8 * lk);
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const H* row0 = &sA[0][wm * 64 + mb * 32 + lr][0];
            V8 ah[4], al[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const H* row = row0 + (size_t)c * MT * SRS;
                ah[c] = *reinterpret_cast<const V8*>(row + 8 * lk);
                al[c] = *reinterpret_cast<const V8*>(row + 16 + 8 * lk);
            }
            const V8 nh1 = neg8(ah[1]), nl1 = neg8(al[1]);   // -Ai1
            const V8 nh3 = neg8(ah[3]), nl3 = neg8(al[3]);   // -Ai2
            v16f c0 = acc[0][mb], c1 = acc[1][mb], c2 = acc[2][mb], c3 = acc[3][mb];
#define QT_SPLIT3(ACC, XH, XL, YI)                      \
    ACC = mfma16<H>(XL, bh[YI], ACC);                   \
    ACC = mfma16<H>(XH, bl[YI], ACC);                   \
    ACC = mfma16<H>(XH, bh[YI], ACC);
            // Re C1 = Ar1 B1r + (-Ai1) B1i + Ar2 Dr + (-Ai2) Di
            QT_SPLIT3(c0, ah[0], al[0], 0) QT_SPLIT3(c0, nh1, nl1, 1)
            QT_SPLIT3(c0, ah[2], al[2], 4) QT_SPLIT3(c0, nh3, nl3, 5)
            // Im C1 = Ar1 B1i + Ai1 B1r + Ar2 Di + Ai2 Dr
            QT_SPLIT3(c1, ah[0], al[0], 1) QT_SPLIT3(c1, ah[1], al[1], 0)
            QT_SPLIT3(c1, ah[2], al[2], 5) QT_SPLIT3(c1, ah[3], al[3], 4)
            // Re C2 = Ar1 B2r + (-Ai1) B2i + Ar2 Er + (-Ai2) Ei
            QT_SPLIT3(c2, ah[0], al[0], 2) QT_SPLIT3(c2, nh1, nl1, 3)
            QT_SPLIT3(c2, ah[2], al[2], 6) QT_SPLIT3(c2, nh3, nl3, 7)
            // Im C2 = Ar1 B2i + Ai1 B2r + Ar2 Ei + Ai2 Er
            QT_SPLIT3(c3, ah[0], al[0], 3) QT_SPLIT3(c3, ah[1], al[1], 2)
            QT_SPLIT3(c3, ah[2], al[2], 7) QT_SPLIT3(c3, ah[3], al[3], 6)
#undef QT_SPLIT3
            acc[0][mb] = c0; acc[1][mb] = c1; acc[2][mb] = c2; acc[3][mb] = c3;
        }
        __syncthreads();
        if (more) {
            store_lds();
            __syncthreads();
        }
    }

    float* Cf = a.Ch + (size_t)f * a.m * a.ldc;
    const int col = n0 + wn * 32 + lr;
    if (col < a.s) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * 64 + mb * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
                if (row < a.m) {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        Cf[c * pc + (size_t)row * a.ldc + col] = acc[c][mb][r] * out_scale;
                }
            }
    }
}

// ---------------------------------------------------------------- FP64 VALU
// Plain 16 x 16 tiled kernel: one output element (all four planes) per thread.
__global__ void __launch_bounds__(256) facewise_f64_valu(FacewiseArgs<double> a) {
    __shared__ double sA[4][16][17];
    __shared__ double sB[8][16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row = blockIdx.y * 16 + ty;
    const int col = blockIdx.x * 16 + tx;
    const int f = blockIdx.z;
    const int g = (a.p - f) % a.p;
    const size_t pa = (size_t)a.p * a.m * a.lda;
    const size_t pb = (size_t)a.p * a.n * a.ldb;
    const size_t pc = (size_t)a.p * a.m * a.ldc;
    const double* Af = a.Ah + (size_t)f * a.m * a.lda;
    const double* Bf = a.Bh + (size_t)f * a.n * a.ldb;
    const double* Bg = a.Bh + (size_t)g * a.n * a.ldb;
    double c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    for (int k0 = 0; k0 < a.n; k0 += 16) {
        const int ka = k0 + tx, kb = k0 + ty;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            sA[c][ty][tx] = (row < a.m && ka < a.n) ? Af[c * pa + (size_t)row * a.lda + ka] : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            sB[c][ty][tx] = (kb < a.n && col < a.s) ? Bf[c * pb + (size_t)kb * a.ldb + col] : 0.0;
            sB[4 + c][ty][tx] = (kb < a.n && col < a.s) ? Bg[c * pb + (size_t)kb * a.ldb + col] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const double ar1 = sA[0][ty][k], ai1 = sA[1][ty][k];
            const double ar2 = sA[2][ty][k], ai2 = sA[3][ty][k];
            const double br1f = sB[0][k][tx], bi1f = sB[1][k][tx];
            const double br2f = sB[2][k][tx], bi2f = sB[3][k][tx];
            const double br1g = sB[4][k][tx], bi1g = sB[5][k][tx];
            const double br2g = sB[6][k][tx], bi2g = sB[7][k][tx];
            c0 += ar1 * br1f - ai1 * bi1f - ar2 * br2g - ai2 * bi2g;
            c1 += ar1 * bi1f + ai1 * br1f + ar2 * bi2g - ai2 * br2g;
            c2 += ar1 * br2f - ai1 * bi2f + ar2 * br1g + ai2 * bi1g;
            c3 += ar1 * bi2f + ai1 * br2f + ai2 * br1g - ar2 * bi1g;
        }
        __syncthreads();
    }
    if (row < a.m && col < a.s) {
        double* Cf = a.Ch + (size_t)f * a.m * a.ldc + (size_t)row * a.ldc + col;
        Cf[0] = c0;
        Cf[pc] = c1;
        Cf[2 * pc] = c2;
        Cf[3 * pc] = c3;
    }
}

}  // namespace

hipError_t launch_facewise_f32(const FacewiseArgs<float>& a, int precision, hipStream_t stream) {
    const int tiles_m = (a.m + MT - 1) / MT;
    const int tiles_n = (a.s + NT - 1) / NT;
    const dim3 grid(tiles_m * tiles_n, a.p);
    if (precision == 0) {
        hipLaunchKernelGGL(facewise_f32_mfma, grid, dim3(256), 0, stream, a, tiles_n);
    } else if (precision == 1) {
        hipLaunchKernelGGL(facewise_split_mfma<__bf16>, grid, dim3(256), 0, stream, a, tiles_n,
                           (const float*)nullptr);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

hipError_t launch_facewise_f64(const FacewiseArgs<double>& a, hipStream_t stream) {
    hipLaunchKernelGGL(facewise_f64_valu, dim3((a.s + 15) / 16, (a.m + 15) / 16, a.p), dim3(256), 0,
                       stream, a);
    return hipGetLastError();
}

}  // namespace qt
