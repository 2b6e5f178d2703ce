// Quaternion t-SVD A = U * S * V^H (A m x n x p, U m x m x p and V n x n x p
// unitary tensors, S f-diagonal), built on the block diagonalisation of
// Theorem 4.4 and the coupled products of Theorem 5.1 / Remark 5.1.
//
// With X^1, X^2 the tube DFTs of the complex parts of X = X1 + X2 j, the
// matrices
//     chi_f(X) = [[ X^1[f], X^2[f] ], [ -conj X^2[-f], conj X^1[-f] ]]
// multiply as chi_f(A * B) = chi_f(A) chi_f(B) (that is what the coupled
// products TC / TC2 say) and chi_f(X^H) = chi_f(X)^*.  chi_-f(X) is J conj(
// chi_f(X)) J^T, so one SVD per frequency pair {f, -f} gives the factors at
// both frequencies:
//   * f != -f: a complex SVD of chi_f(A) (2m x 2n).  Singular value 2i (in
//     descending order) goes to diagonal entry i of S^1[f], value 2i + 1 to
//     entry i of S^1[-f]; singular vectors to columns i and half + i.
//   * f == -f (f = 0, and p/2 for even p): chi_f(A) is the complex adjoint of
//     the quaternion matrix A^1[f] + A^2[f] j, and the factors must be too.
//     A quaternion column is stored as its first complex column (x; y); the
//     second is its partner (-conj y; conj x).
//
// Steps: the forward tube FFT of A (the kernels of the T-product), one
// workgroup per frequency pair running a one-sided (Hestenes) Jacobi SVD on
// the columns of chi_f(A) (or of chi_f(A)^* when m < n, so that columns are
// the long side), an orthonormal completion of the left vectors where the
// matrix is not square or singular, and inverse tube FFTs of U^, S^ and V^.
// For quaternion columns a Jacobi step first turns the quaternion inner
// product of the two columns real by right-multiplying one column by a unit
// quaternion, then applies a real plane rotation; partners follow implicitly,
// so the factors keep their quaternion structure.
#include <math.h>

#include "qt_internal.h"
#include "workspace.h"
#include "../../include/qtprod.h"

namespace qt {
namespace {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxMin = 512;      // min(m, n) served
constexpr int kMaxMax = 1024;     // max(m, n) served
constexpr int kMaxSweeps = 60;

template <typename T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
    return V{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return V{a.x, -a.y}; }
template <typename V, typename T> __device__ __forceinline__ V cscale(V a, T s) { return V{a.x * s, a.y * s}; }
template <typename V> __device__ __forceinline__ V cneg(V a) { return V{-a.x, -a.y}; }

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}


// Accumulator type of the inner products: double for both precisions, so
// that the cosine between two FP32 columns is known far below the stopping
// threshold (a float sum over 2 max(m, n) terms carries rounding errors of
// about that threshold, and the sweeps would keep rotating on noise).
using Acc = double;

template <typename T>
struct TsvdArgs {
    const T* Ah;            // Fourier-domain A, [4][p][m][lda]
    T* Uh;                  // U^, [4][p][m][ldu]
    T* Vh;                  // V^, [4][p][n][ldv]
    T* sigma;               // [p][min(m, n)]: diagonal of S^1[f]
    char* pairs;            // per-pair scratch, pair_bytes each
    size_t pair_bytes;
    int m, n, p, lda, ldu, ldv;
};

// State of one frequency pair between the kernels of the block sweeps.
struct PairHdr {
    double scale;           // power of two applied to the pair's matrix
    double negl2;           // squared column norm below which a column is rounding noise
    int done;               // a whole sweep applied no rotation
    int rot[2];             // sweep s applied a rotation (slot s & 1)
    int pad;
};
constexpr size_t kHdrBytes = 256;

// Per-pair scratch layout, for r = max(m, n), c = min(m, n): the header,
// then (complex entries)
//   X   2c columns of 2r   (columns of chi_f(A) or chi_f(A)^*)
//   Q   2c columns of 2c   (accumulated rotations)
//   L   2r columns of 2r   (left vectors in rank order, then completed)
//   W   2r + r coefficients of the completion
template <typename T>
size_t pair_scratch_bytes(int m, int n) {
    const size_t r = m > n ? m : n, c = m > n ? n : m;
    const size_t e = 2 * c * 2 * r + 2 * c * 2 * c + 2 * r * 2 * r + 3 * r;
    return kHdrBytes + ((e * sizeof(typename Cx<T>::type) + 255) & ~(size_t)255);
}

// Position of player q in round t of the circle method over nup players
// (nup even): every pair of players meets once in nup - 1 rounds.
__device__ __forceinline__ int circle(int q, int t, int nup) {
    return q == 0 ? 0 : ((q - 1 + t) % (nup - 1)) + 1;
}

// Sum over the 64 lanes of a wave (all lanes active), returned in every lane:
// DPP adds within rows of 16 lanes (two quad permutations, the half-row and
// row mirrors), the row broadcasts of lanes 15 and 31, and the total read
// from lane 63.  Register moves only, no LDS round trips.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_shift(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double wave_total(double v) {
    v += dpp_shift<0xB1, 0xF>(v);      // quad_perm [1, 0, 3, 2]
    v += dpp_shift<0x4E, 0xF>(v);      // quad_perm [2, 3, 0, 1]
    v += dpp_shift<0x141, 0xF>(v);     // row_half_mirror
    v += dpp_shift<0x140, 0xF>(v);     // row_mirror
    v += dpp_shift<0x142, 0xA>(v);     // row_bcast:15 into rows 1 and 3
    v += dpp_shift<0x143, 0xC>(v);     // row_bcast:31 into rows 2 and 3
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Parameters of a Jacobi step from the wave-summed inner products (gn2 =
// |gamma|^2 > 0): the phase e = gamma / |gamma| (applied as x_j conj(e)) and
// the plane rotation (cs, sn) that then zeroes the real inner product, formed
// in double (reciprocal square roots and a refined reciprocal, no division)
// and rounded once to T.
template <typename T, typename V>
__device__ __forceinline__ void rotation(Acc al, Acc be, Acc g1r, Acc g1i, Acc g2r, Acc g2i, Acc gn2, V& e1c,
                                         V& e2c, T& cs, T& sn) {
    const Acc ign = rsqrt(gn2);
    e1c = V{T(g1r * ign), T(-g1i * ign)};
    e2c = V{T(g2r * ign), T(-g2i * ign)};
    const Acc zeta = (be - al) * (Acc(0.5) * ign);
    const Acc az = fabs(zeta);
    // |t| = 1 / (|zeta| + sqrt(1 + zeta^2)) = (sqrt(1 + zeta^2) - |zeta|);
    // sqrt(y) = y rsqrt(y), and for |zeta| > 1 the reciprocal of d = |zeta| +
    // w >= 2 is the hardware estimate refined by two Newton steps (each one
    // doubles the correct bits), without the scaling of a general division
    const Acc y = Acc(1) + az * az;
    const Acc w = y * rsqrt(y);
    Acc at;
    if (az > Acc(1)) {
        const Acc d = az + w;
        Acc r = __builtin_amdgcn_rcp(d);
        r = fma(r, fma(-d, r, Acc(1)), r);
        r = fma(r, fma(-d, r, Acc(1)), r);
        at = r;
    } else {
        at = w - az;
    }
    const Acc csd = rsqrt(Acc(1) + at * at);
    cs = T(csd);
    sn = T(csd * (zeta >= 0 ? at : -at));
}

// Partner component k of a quaternion column x of 2h entries.
template <typename V>
__device__ __forceinline__ V partner_at(const V* x, int k, int h) {
    return k < h ? cneg(cconj(x[k + h])) : cconj(x[k - h]);
}

// One Jacobi step on columns xi, xj (2h entries each) and their rotation
// columns qi, qj (2hq entries), executed by one wave.  Returns true if a
// rotation was applied.
template <typename T, typename V>
__device__ __forceinline__ bool jacobi_pair(V* xi, V* xj, V* qi, V* qj, int h, int hq, bool quat, T tol, Acc negl2, int lane) {
    Acc al = 0, be = 0, g1r = 0, g1i = 0, g2r = 0, g2i = 0;
#pragma unroll 4
    for (int k = lane; k < h; k += 64) {
        const V a0 = xi[k], a1 = xi[k + h], b0 = xj[k], b1 = xj[k + h];
        const Acc a0x = a0.x, a0y = a0.y, a1x = a1.x, a1y = a1.y;
        const Acc b0x = b0.x, b0y = b0.y, b1x = b1.x, b1y = b1.y;
        al += a0x * a0x + a0y * a0y + a1x * a1x + a1y * a1y;
        be += b0x * b0x + b0y * b0y + b1x * b1x + b1y * b1y;
        // x_i^* x_j
        g1r += a0x * b0x + a0y * b0y + a1x * b1x + a1y * b1y;
        g1i += a0x * b0y - a0y * b0x + a1x * b1y - a1y * b1x;
        if (quat) {   // x_i^* partner(x_j), partner(x_j) = (-conj b1; conj b0)
            g2r += -(a0x * b1x - a0y * b1y) + (a1x * b0x - a1y * b0y);
            g2i += (a0x * b1y + a0y * b1x) - (a1x * b0y + a1y * b0x);
        }
    }
    al = wave_total(al);
    be = wave_total(be);
    g1r = wave_total(g1r);
    g1i = wave_total(g1i);
    if (quat) {
        g2r = wave_total(g2r);
        g2i = wave_total(g2i);
    }
    // a column at rounding level of the whole matrix belongs to the null
    // space: rotating it only stirs rounding errors (and never converges)
    if (al <= negl2 || be <= negl2) return false;
    // |gamma| > tol sqrt(al be), compared in squares (no square roots on the
    // path of a pair that does not rotate)
    const Acc gn2 = g1r * g1r + g1i * g1i + g2r * g2r + g2i * g2i;
    if (!(gn2 > (Acc)tol * (Acc)tol * (al * be))) return false;
    // x_j <- x_j conj(e), e = gamma / |gamma| (a unit quaternion, or a complex
    // phase when g2 = 0): afterwards x_i^* x_j = |gamma| is real
    V e1c, e2c;
    T cs, sn;
    rotation<T, V>(al, be, g1r, g1i, g2r, g2i, gn2, e1c, e2c, cs, sn);
    auto apply = [&](V* ci, V* cj, int hh) {
#pragma unroll 4
        for (int k = lane; k < hh; k += 64) {
            const V a0 = ci[k], a1 = ci[k + hh], b0 = cj[k], b1 = cj[k + hh];
            V c0 = cmul(e1c, b0), c1 = cmul(e1c, b1);
            if (quat) {
                c0 = cadd(c0, cmul(e2c, cneg(cconj(b1))));
                c1 = cadd(c1, cmul(e2c, cconj(b0)));
            }
            ci[k] = csub(cscale(a0, cs), cscale(c0, sn));
            ci[k + hh] = csub(cscale(a1, cs), cscale(c1, sn));
            cj[k] = cadd(cscale(a0, sn), cscale(c0, cs));
            cj[k + hh] = cadd(cscale(a1, sn), cscale(c1, cs));
        }
    };
    apply(xi, xj, h);
    apply(qi, qj, hq);
    return true;
}

// The same step with both columns held in registers between the inner
// products and the update (K loads per lane and column half issued together):
// for h <= 64 K and hq <= 64 KQ.
template <typename T, typename V, int K, int KQ = K>
__device__ __forceinline__ bool jacobi_pair_reg(V* xi, V* xj, V* qi, V* qj, int h, int hq, bool quat, T tol, Acc negl2, int lane) {
    // the rotation columns are loaded with the data columns (one memory
    // round trip per pair); they are only written back if a rotation happens
    V a0[K], a1[K], b0[K], b1[K], c0[KQ], c1[KQ], d0[KQ], d1[KQ];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int k = lane + 64 * t;
        const bool in = k < h;
        a0[t] = in ? xi[k] : V{0, 0};
        a1[t] = in ? xi[k + h] : V{0, 0};
        b0[t] = in ? xj[k] : V{0, 0};
        b1[t] = in ? xj[k + h] : V{0, 0};
    }
#pragma unroll
    for (int t = 0; t < KQ; ++t) {
        const int k = lane + 64 * t;
        const bool inq = k < hq;
        c0[t] = inq ? qi[k] : V{0, 0};
        c1[t] = inq ? qi[k + hq] : V{0, 0};
        d0[t] = inq ? qj[k] : V{0, 0};
        d1[t] = inq ? qj[k + hq] : V{0, 0};
    }
    Acc al = 0, be = 0, g1r = 0, g1i = 0, g2r = 0, g2i = 0;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const Acc a0x = a0[t].x, a0y = a0[t].y, a1x = a1[t].x, a1y = a1[t].y;
        const Acc b0x = b0[t].x, b0y = b0[t].y, b1x = b1[t].x, b1y = b1[t].y;
        al += a0x * a0x + a0y * a0y + a1x * a1x + a1y * a1y;
        be += b0x * b0x + b0y * b0y + b1x * b1x + b1y * b1y;
        g1r += a0x * b0x + a0y * b0y + a1x * b1x + a1y * b1y;
        g1i += a0x * b0y - a0y * b0x + a1x * b1y - a1y * b1x;
        if (quat) {
            g2r += -(a0x * b1x - a0y * b1y) + (a1x * b0x - a1y * b0y);
            g2i += (a0x * b1y + a0y * b1x) - (a1x * b0y + a1y * b0x);
        }
    }
    al = wave_total(al);
    be = wave_total(be);
    g1r = wave_total(g1r);
    g1i = wave_total(g1i);
    if (quat) {
        g2r = wave_total(g2r);
        g2i = wave_total(g2i);
    }
    if (al <= negl2 || be <= negl2) return false;
    // |gamma| > tol sqrt(al be), compared in squares (no square roots on the
    // path of a pair that does not rotate)
    const Acc gn2 = g1r * g1r + g1i * g1i + g2r * g2r + g2i * g2i;
    if (!(gn2 > (Acc)tol * (Acc)tol * (al * be))) return false;
    V e1c, e2c;
    T cs, sn;
    rotation<T, V>(al, be, g1r, g1i, g2r, g2i, gn2, e1c, e2c, cs, sn);
    auto rot = [&](V& u0, V& u1, V& w0, V& w1) {
        V r0 = cmul(e1c, w0), r1 = cmul(e1c, w1);
        if (quat) {
            r0 = cadd(r0, cmul(e2c, cneg(cconj(w1))));
            r1 = cadd(r1, cmul(e2c, cconj(w0)));
        }
        const V n0 = csub(cscale(u0, cs), cscale(r0, sn)), n1 = csub(cscale(u1, cs), cscale(r1, sn));
        w0 = cadd(cscale(u0, sn), cscale(r0, cs));
        w1 = cadd(cscale(u1, sn), cscale(r1, cs));
        u0 = n0;
        u1 = n1;
    };
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int k = lane + 64 * t;
        if (k < h) {
            rot(a0[t], a1[t], b0[t], b1[t]);
            xi[k] = a0[t];
            xi[k + h] = a1[t];
            xj[k] = b0[t];
            xj[k + h] = b1[t];
        }
    }
#pragma unroll
    for (int t = 0; t < KQ; ++t) {
        const int k = lane + 64 * t;
        if (k < hq) {
            rot(c0[t], c1[t], d0[t], d1[t]);
            qi[k] = c0[t];
            qi[k + hq] = c1[t];
            qj[k] = d0[t];
            qj[k + hq] = d1[t];
        }
    }
    return true;
}

// Write column vector u (2*half entries, the slot-th column of chi_f(Y) for an
// half x half quaternion tensor Y) into Y^ at frequencies f and g = -f:
//   slot j <  half: Y^1[f](:, j) = top,        Y^2[g](:, j) = -conj(bottom)
//   slot j >= half: Y^2[f](:, j - half) = top, Y^1[g](:, j - half) = conj(bottom)
template <typename T, typename V>
__device__ void write_slot(T* Yh, int ld, int p, int half, int f, int g, int slot, const V* u, int tid,
                           int nthreads) {
    const size_t plane = (size_t)p * half * ld;
    const bool second = slot >= half;
    const int j = second ? slot - half : slot;
    for (int i = tid; i < half; i += nthreads) {
        const V top = u[i], bot = u[i + half];
        const V tf = top;
        const V bg = second ? cconj(bot) : cneg(cconj(bot));
        const int pf = second ? 2 : 0, pg = second ? 0 : 2;
        const size_t rf = ((size_t)f * half + i) * ld + j, rg = ((size_t)g * half + i) * ld + j;
        Yh[pf * plane + rf] = tf.x;
        Yh[(pf + 1) * plane + rf] = tf.y;
        Yh[pg * plane + rg] = bg.x;
        Yh[(pg + 1) * plane + rg] = bg.y;
    }
}

// Entry i (0 <= i < 2 half) of the column vector of slot `slot`, placed as
// write_slot places it.
template <typename T, typename V>
__device__ __forceinline__ void place_entry(T* Yh, int ld, int p, int half, int f, int g, int slot, int i, V v) {
    const size_t plane = (size_t)p * half * ld;
    const bool second = slot >= half;
    const int j = second ? slot - half : slot;
    if (i < half) {
        const int pf = second ? 2 : 0;
        const size_t rf = ((size_t)f * half + i) * ld + j;
        Yh[pf * plane + rf] = v.x;
        Yh[(pf + 1) * plane + rf] = v.y;
    } else {
        const V bg = second ? cconj(v) : cneg(cconj(v));
        const int pg = second ? 0 : 2;
        const size_t rg = ((size_t)g * half + (i - half)) * ld + j;
        Yh[pg * plane + rg] = bg.x;
        Yh[(pg + 1) * plane + rg] = bg.y;
    }
}

// Geometry of frequency pair f: which matrix is orthogonalised and where its
// scratch lives.
template <typename T>
struct PairView {
    using V = typename Cx<T>::type;
    int f, g;
    bool quat, tall;
    int r, c, nu, nL, R, Rq;
    PairHdr* hdr;
    V *X, *Q, *L, *coef, *coef2;
};

template <typename T>
__device__ __forceinline__ PairView<T> pair_view(const TsvdArgs<T>& a, int f) {
    using V = typename Cx<T>::type;
    PairView<T> v;
    v.f = f;
    v.g = (a.p - f) % a.p;
    v.quat = f == v.g;
    v.tall = a.m >= a.n;
    v.r = v.tall ? a.m : a.n;
    v.c = v.tall ? a.n : a.m;
    v.nu = v.quat ? v.c : 2 * v.c;        // Jacobi units (columns, or quaternion columns)
    v.nL = v.quat ? v.r : 2 * v.r;        // left-side slots
    v.R = 2 * v.r;
    v.Rq = 2 * v.c;
    char* base = a.pairs + (size_t)f * a.pair_bytes;
    v.hdr = reinterpret_cast<PairHdr*>(base);
    v.X = reinterpret_cast<V*>(base + kHdrBytes);
    v.Q = v.X + (size_t)2 * v.c * v.R;
    v.L = v.Q + (size_t)2 * v.c * v.Rq;
    v.coef = v.L + (size_t)2 * v.r * v.R;
    v.coef2 = v.coef + (size_t)2 * v.r;
    return v;
}

// Stopping threshold: the largest cosine left between two columns.
template <typename T>
__device__ __forceinline__ T jacobi_tol(int R) {
    const T eps = sizeof(T) == 4 ? T(5.9604645e-8) : T(1.1102230246251565e-16);
    return eps * sqrt((T)R);
}

// X <- the pair's matrix scaled by a power of two so that its largest entry
// is in [0.5, 1) (the squared norms of the Jacobi steps then neither overflow
// nor underflow), Q <- identity; the header gets the scale and the noise
// level negl2 (tol^2 times the squared Frobenius norm: a column below it is
// rounding noise of the whole matrix).  Whole workgroup.
template <typename T>
__device__ void pair_prep(const TsvdArgs<T>& a, const PairView<T>& pv, Acc* s_red, T& scale, Acc& negl2) {
    using V = typename Cx<T>::type;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = a.m, n = a.n, f = pv.f, g = pv.g;
    const size_t pl = (size_t)a.p * m * a.lda;
    auto A1 = [&](int fr, int i, int j) {
        const size_t o = ((size_t)fr * m + i) * a.lda + j;
        return V{a.Ah[o], a.Ah[pl + o]};
    };
    auto A2 = [&](int fr, int i, int j) {
        const size_t o = ((size_t)fr * m + i) * a.lda + j;
        return V{a.Ah[2 * pl + o], a.Ah[3 * pl + o]};
    };
    // entry k of unit u of the matrix whose columns are orthogonalised
    auto entry = [&](int u, int k) -> V {
        if (pv.tall) {   // column u of chi_f(A)
            if (u < n) return k < m ? A1(f, k, u) : cneg(cconj(A2(g, k - m, u)));
            return k < m ? A2(f, k, u - n) : cconj(A1(g, k - m, u - n));
        }
        // column u of chi_f(A)^*: the conjugate of row u of chi_f(A)
        if (u < m) return k < n ? cconj(A1(f, u, k)) : cconj(A2(f, u, k - n));
        return k < n ? cneg(A2(g, u - m, k)) : A1(g, u - m, k - n);
    };
    const int R = pv.R, Rq = pv.Rq, nu = pv.nu;
    T mx = 0;
    for (int e = tid; e < nu * R; e += kThreads) {
        const V v = entry(e / R, e % R);
        mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) s_red[wave] = mx;
    __syncthreads();
    mx = 0;
    for (int w = 0; w < kWaves; ++w) mx = fmax(mx, (T)s_red[w]);
    const int ex = (mx > 0 && isfinite(mx)) ? ilogb(mx) + 1 : 0;
    scale = ldexp(T(1), -ex);
    Acc fro = 0;
    for (int e = tid; e < nu * R; e += kThreads) {
        const V v = cscale(entry(e / R, e % R), scale);
        pv.X[e] = v;
        fro += (Acc)v.x * v.x + (Acc)v.y * v.y;
    }
    for (int e = tid; e < nu * Rq; e += kThreads) pv.Q[e] = V{(e % Rq) == (e / Rq) ? T(1) : T(0), T(0)};
    fro = wave_sum(fro);
    __syncthreads();
    if (lane == 0) s_red[wave] = fro;
    __syncthreads();
    fro = 0;
    for (int w = 0; w < kWaves; ++w) fro += s_red[w];
    const T tol = jacobi_tol<T>(R);
    negl2 = (Acc)tol * tol * fro;
    if (tid == 0) {
        pv.hdr->scale = (double)scale;
        pv.hdr->negl2 = negl2;
        pv.hdr->done = 0;
        pv.hdr->rot[0] = 0;
        pv.hdr->rot[1] = 0;
    }
}

// One-sided Jacobi sweeps of one workgroup over all unit pairs, round-robin
// over disjoint pairs, until a sweep applies no rotation.
template <typename T>
__device__ void pair_sweeps(const PairView<T>& pv, Acc negl2, int* s_flag) {
    using V = typename Cx<T>::type;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nu = pv.nu, R = pv.R, Rq = pv.Rq, r = pv.r, c = pv.c;
    const T tol = jacobi_tol<T>(R);
    const int nup = nu + (nu & 1);
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        __syncthreads();
        if (tid == 0) *s_flag = 0;
        __syncthreads();
        for (int t = 0; t < nup - 1; ++t) {
            for (int q = wave; q < nup / 2; q += kWaves) {
                const int i = circle(q, t, nup), j = circle(nup - 1 - q, t, nup);
                if (i >= nu || j >= nu) continue;
                V *xi = pv.X + (size_t)i * R, *xj = pv.X + (size_t)j * R;
                V *qi = pv.Q + (size_t)i * Rq, *qj = pv.Q + (size_t)j * Rq;
                const bool rotated =
                    (r <= 64 && c <= 64)     ? jacobi_pair_reg<T, V, 1>(xi, xj, qi, qj, r, c, pv.quat, tol, negl2, lane)
                    : (r <= 256 && c <= 256) ? jacobi_pair_reg<T, V, 4>(xi, xj, qi, qj, r, c, pv.quat, tol, negl2, lane)
                                             : jacobi_pair<T, V>(xi, xj, qi, qj, r, c, pv.quat, tol, negl2, lane);
                if (rotated && lane == 0) *s_flag = 1;
            }
            __syncthreads();
        }
        if (*s_flag == 0) break;
    }
}

// Shared arrays of the last step.
template <typename T>
struct FinishSmem {
    using V = typename Cx<T>::type;
    T sig[2 * kMaxMin];
    int perm[2 * kMaxMin];
    unsigned char ok[2 * kMaxMax];
    V w[2 * kMaxMax];
    Acc red[kWaves];
};

// From the orthogonalised columns: singular values in descending order,
// normalised left vectors (completed to an orthonormal basis), and both
// vector sets placed at f and -f.  Whole workgroup.
template <typename T>
__device__ void pair_finish(const TsvdArgs<T>& a, const PairView<T>& pv, T scale, Acc negl2, FinishSmem<T>& sm,
                            bool place = true) {
    using V = typename Cx<T>::type;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int p = a.p, f = pv.f, g = pv.g, r = pv.r, c = pv.c, nu = pv.nu, nL = pv.nL, R = pv.R, Rq = pv.Rq;
    const bool quat = pv.quat, tall = pv.tall;
    V *X = pv.X, *Q = pv.Q, *L = pv.L, *coef = pv.coef, *coef2 = pv.coef2;
    T* s_sig = sm.sig;
    int* s_perm = sm.perm;
    unsigned char* s_ok = sm.ok;
    V* s_w = sm.w;
    Acc* s_red = sm.red;

    // singular values (column norms) and their descending order
    for (int u = wave; u < nu; u += kWaves) {
        Acc s = 0;
        for (int k = lane; k < R; k += 64) {
            const V v = X[(size_t)u * R + k];
            s += (Acc)v.x * v.x + (Acc)v.y * v.y;
        }
        s = wave_sum(s);
        if (lane == 0) s_sig[u] = (T)sqrt(s);
    }
    __syncthreads();
    for (int u = tid; u < nu; u += kThreads) {
        const T su = s_sig[u];
        int rank = 0;
        for (int v = 0; v < nu; ++v) {
            const T sv = s_sig[v];
            rank += (sv > su) || (sv == su && v < u);
        }
        s_perm[rank] = u;
    }
    for (int k = tid; k < nL; k += kThreads) s_ok[k] = 0;
    __syncthreads();

    // sigma, and the normalised left vectors in rank order; a column at the
    // noise level leaves its slot to the completion below
    const T tiny = (T)sqrt(negl2);
    for (int rho = tid; rho < nu; rho += kThreads) {
        const T sv = s_sig[s_perm[rho]] / scale;
        const int k = quat ? rho : rho / 2;
        const int fr = (quat || !(rho & 1)) ? f : g;
        a.sigma[(size_t)fr * c + k] = sv;
    }
    for (int rho = wave; rho < nu; rho += kWaves) {
        const int u = s_perm[rho];
        const T su = s_sig[u];
        if (su > tiny) {
            const T inv = T(1) / su;
            for (int k = lane; k < R; k += 64) L[(size_t)rho * R + k] = cscale(X[(size_t)u * R + k], inv);
            if (lane == 0) s_ok[rho] = 1;
        }
    }
    __syncthreads();

    // complete the left vectors to an orthonormal basis: Gram-Schmidt
    // (twice) of unit vectors against the accepted columns (and, for
    // quaternion columns, their partners).  A candidate is accepted when its
    // residual exceeds half the average that must remain, which some
    // candidate always does.
    const T accept = T(0.5) / (T)R;
    int cand = 0;
    for (int rho = 0; rho < nL; ++rho) {
        if (s_ok[rho]) continue;
        while (cand < R) {
            for (int k = tid; k < R; k += kThreads) s_w[k] = V{k == cand ? T(1) : T(0), T(0)};
            __syncthreads();
            for (int pass = 0; pass < 2; ++pass) {
                for (int b = tid; b < nL; b += kThreads) {
                    if (!s_ok[b]) continue;
                    const V* lb = L + (size_t)b * R;
                    V d1 = V{0, 0}, d2 = V{0, 0};
                    for (int k = 0; k < R; ++k) {
                        const V w = s_w[k];
                        d1 = cadd(d1, cmulc(lb[k], w));
                        if (quat) d2 = cadd(d2, cmulc(partner_at(lb, k, r), w));
                    }
                    coef[b] = d1;
                    if (quat) coef2[b] = d2;
                }
                __syncthreads();
                for (int k = tid; k < R; k += kThreads) {
                    V w = s_w[k];
                    for (int b = 0; b < nL; ++b) {
                        if (!s_ok[b]) continue;
                        const V* lb = L + (size_t)b * R;
                        w = csub(w, cmul(lb[k], coef[b]));
                        if (quat) w = csub(w, cmul(partner_at(lb, k, r), coef2[b]));
                    }
                    s_w[k] = w;
                }
                __syncthreads();
            }
            Acc s = 0;
            for (int k = tid; k < R; k += kThreads) s += (Acc)s_w[k].x * s_w[k].x + (Acc)s_w[k].y * s_w[k].y;
            s = wave_sum(s);
            if (lane == 0) s_red[wave] = s;
            __syncthreads();
            s = 0;
            for (int w = 0; w < kWaves; ++w) s += s_red[w];
            ++cand;
            if (s > accept) {
                const T inv = T(1 / sqrt(s));
                for (int k = tid; k < R; k += kThreads) L[(size_t)rho * R + k] = cscale(s_w[k], inv);
                __syncthreads();
                if (tid == 0) s_ok[rho] = 1;
                __syncthreads();
                break;
            }
            __syncthreads();
        }
    }
    __syncthreads();

    if (!place) {
        // the placement runs as a kernel of its own: it needs the rank order
        // of the rotation columns, kept where the completion's coefficients were
        int* gperm = reinterpret_cast<int*>(coef);
        for (int rho = tid; rho < nu; rho += kThreads) gperm[rho] = s_perm[rho];
        return;
    }
    // place the vectors: rank rho goes to slot rho (quaternion columns) or
    // to slot rho / 2 (+ half for odd rho) -- the interleaving of f and -f
    T* Lh = tall ? a.Uh : a.Vh;
    T* Qh = tall ? a.Vh : a.Uh;
    const int ldl = tall ? a.ldu : a.ldv, ldq = tall ? a.ldv : a.ldu;
    auto slot = [&](int rho, int half) { return quat ? rho : rho / 2 + ((rho & 1) ? half : 0); };
    for (int rho = 0; rho < nL; ++rho)
        write_slot<T, V>(Lh, ldl, p, r, f, g, slot(rho, r), L + (size_t)rho * R, tid, kThreads);
    for (int rho = 0; rho < nu; ++rho)
        write_slot<T, V>(Qh, ldq, p, c, f, g, slot(rho, c), Q + (size_t)s_perm[rho] * Rq, tid, kThreads);
}

// One workgroup per frequency pair, every step in one launch.
template <typename T>
__global__ void __launch_bounds__(kThreads) tsvd_pair_kernel(TsvdArgs<T> a) {
    __shared__ FinishSmem<T> sm;
    __shared__ int s_flag;
    const PairView<T> pv = pair_view(a, blockIdx.x);
    T scale;
    Acc negl2;
    pair_prep(a, pv, sm.red, scale, negl2);
    __syncthreads();
    pair_sweeps(pv, negl2, &s_flag);
    __syncthreads();
    pair_finish(a, pv, scale, negl2, sm);
}

// ------------------------------------------------------------ block sweeps
// For larger matrices the sweeps are spread over many workgroups per pair.
// The units are cut into blocks of bs; in round t of a sweep, block pair q
// of the circle schedule over the blocks goes to one workgroup, which stages
// the data columns of its two blocks in LDS, applies the rotations of every
// unit pair across the two blocks (and, in round 0, the pairs within each
// block), and writes the columns back.  Every unit pair is visited once per
// sweep, as in the single-workgroup order, with one global read and write of
// a column per block pair instead of one per unit pair.
// The rotation columns are not staged: the workgroup accumulates the product
// W of its rotations over its nk units in LDS and applies it once at the end,
// Q_j <- sum_i Q_i A_ij + partner(Q_i) B_ij.
// A Jacobi step maps unit columns to combinations of this form, and since
// partner is conjugate-linear with partner(partner(x)) = -x, the coefficient
// column (A_j; B_j) of unit j transforms under a step exactly as a
// quaternion column (top; bottom) does, so the same step code updates it
// (B stays zero for complex pairs).  Only the data columns take LDS, which
// lets two workgroups share a CU when they fit in half of it.
// A sweep is one launch per round plus a check: a pair whose sweep applied no
// rotation is done, and its workgroups return at once in later launches.
constexpr size_t kBlockLds = 144 << 10;   // LDS of one workgroup per CU
constexpr size_t kBlockLdsHalf = 72 << 10; // two workgroups per CU
constexpr int kBlockMaxBs = 8;            // units per block (one cross pair per wave and round)
constexpr int kBlockMinUnits = 128;       // smaller matrices stay in one workgroup
constexpr int kBlockMaxSweeps = 32;

// LDS of a block pair: 2 bs data columns of R entries and 2 bs coefficient
// columns of 4 bs entries.
template <typename T>
size_t block_lds_bytes(int bs, int R) {
    return ((size_t)2 * bs * R + (size_t)2 * bs * 4 * bs) * sizeof(typename Cx<T>::type);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) tsvd_prep_kernel(TsvdArgs<T> a) {
    __shared__ Acc s_red[kWaves];
    const PairView<T> pv = pair_view(a, blockIdx.x);
    T scale;
    Acc negl2;
    pair_prep(a, pv, s_red, scale, negl2);
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Copy bytes (a multiple of 16, both ends 16-byte aligned) from global memory
// to LDS by DMA: global_load_lds_dwordx4 moves 64 x 16 B per wave
// instruction into 1 KB of LDS (lane L at byte 16 L), without registers;
// lanes past the end are masked off.  The caller waits (s_waitcnt, barrier).
template <typename V>
__device__ __forceinline__ void dma_copy(const V* src, V* dst, size_t bytes, int wave, int lane) {
    const char* s = reinterpret_cast<const char*>(src);
    char* d = reinterpret_cast<char*>(dst);
    for (size_t off = (size_t)wave * 1024; off < bytes; off += (size_t)kWaves * 1024) {
        const size_t mine = off + 16 * (size_t)lane;
        if (mine < bytes) __builtin_amdgcn_global_load_lds((const void*)(s + mine), (lds_void_t*)(d + off), 16, 0, 0);
    }
}

// Q <- Q W for the nk staged units of a block pair (units u < nI at QI + u Rq,
// the others at QJ + u Rq), W in LDS as coefficient columns wc + j 2nk (A
// part, then B part): Q_j = sum_u Q_u A_uj + partner(Q_u) B_uj, where
// partner(q) = (-conj(bottom half); conj(top half)) and B = 0 for a complex
// pair (QUAT false).  A thread holds row k of every unit (rows k and k + hq of
// a quaternion column) in registers and overwrites them column by column.
// With two threads per row (quaternion pairs of up to kThreads / 2 rows) the
// threads of a row split the output columns and read the row before either
// writes.  FULL: nk is the largest block pair, known at compile time, so the
// coefficient reads of one output column issue together.
template <bool FULL, bool QUAT, typename V>
__device__ __forceinline__ void apply_coefficients(V* QI, V* QJ, int nI, int nk, int Rq, const V* wc, int tid) {
    constexpr int MU = 2 * kBlockMaxBs;
    const int hq = Rq / 2, rows = QUAT ? hq : Rq, w2 = 2 * nk;
    const int per_row = QUAT && 2 * rows <= kThreads ? 2 : 1;
    const int kend = per_row * rows;
    for (int base = 0; base < kend; base += kThreads) {
        const int id = base + tid, k = id % rows, j0 = id / rows;
        const bool act = id < kend;
        V top[MU], bot[MU];
#pragma unroll
        for (int u = 0; u < MU; ++u) {
            top[u] = bot[u] = V{0, 0};
            if (act && (FULL || u < nk)) {
                const V* qu = (u < nI ? QI : QJ) + (size_t)u * Rq;
                top[u] = qu[k];
                if (QUAT) bot[u] = qu[k + hq];
            }
        }
        if (per_row == 2) __syncthreads();
        if (!act) continue;
#pragma unroll 1
        for (int j = j0; j < nk; j += per_row) {
            const V* cj = wc + (size_t)j * w2;
            V o0{0, 0}, o1{0, 0};
#pragma unroll
            for (int u = 0; u < MU; ++u) {
                if (FULL || u < nk) {
                    const V aa = cj[u];
                    o0 = cadd(o0, cmul(top[u], aa));
                    if (QUAT) {
                        const V bb = cj[nk + u];
                        o0 = csub(o0, cmul(cconj(bot[u]), bb));
                        o1 = cadd(o1, cadd(cmul(bot[u], aa), cmul(cconj(top[u]), bb)));
                    }
                }
            }
            V* qj = (j < nI ? QI : QJ) + (size_t)j * Rq;
            qj[k] = o0;
            if (QUAT) qj[k + hq] = o1;
        }
    }
}

// grid: (block pairs of the longest schedule, frequency pairs).  LDS bytes
// of staging (kBlockLds or kBlockLdsHalf); with the half, the register
// budget allows two workgroups of 8 waves per CU.  KR: data-column entries
// per lane and column half held in registers by a Jacobi step (1 for
// max(m, n) <= 64, 4 for <= 256), 0 for the looping step of longer columns.
template <typename T, size_t LDS, int KR>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(LDS == kBlockLdsHalf ? 4 : 2)))
tsvd_round_kernel(TsvdArgs<T> a, int bs_c, int t, int sweep) {
    using V = typename Cx<T>::type;
    __shared__ __attribute__((aligned(16))) char s_cols[LDS];
    __shared__ int s_rot;
    // the self-paired frequencies (f = 0, and p / 2 for even p) first: their
    // quaternion steps and updates take longest, and dispatched last they
    // would set the end of every round
    const int y = blockIdx.y;
    const int f = (a.p % 2 == 0 && a.p > 1) ? (y == 0 ? 0 : y == 1 ? a.p / 2 : y - 1) : y;
    const PairView<T> pv = pair_view(a, f);
    if (pv.hdr->done) return;
    // a quaternion pair has half as many units, each step and update costs
    // about twice as much: blocks of half the size give it the same number
    // of block pairs and rounds per sweep as the complex pairs, and
    // workgroups that finish with theirs (ceil(bs / 2) units never needs
    // more rounds than bs units of the complex pairs)
    const int bs = pv.quat ? (bs_c + 1) / 2 : bs_c;
    const int nu = pv.nu, nb = (nu + bs - 1) / bs, nbp = nb + (nb & 1);
    const int q = blockIdx.x;
    if (t >= nbp - 1 || q >= nbp / 2) return;      // a shorter schedule (quaternion pair)
    const int I = circle(q, t, nbp), J = circle(nbp - 1 - q, t, nbp);
    const int nI = I < nb ? min(bs, nu - I * bs) : 0;
    const int nJ = J < nb ? min(bs, nu - J * bs) : 0;
    if (t > 0 && (nI == 0 || nJ == 0)) return;      // within-block pairs go in round 0 only
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int R = pv.R, Rq = pv.Rq, nk = nI + nJ, w2 = 2 * nk;
    V* xs = reinterpret_cast<V*>(s_cols);            // staged unit k: xs + k R
    V* wc = xs + (size_t)nk * R;                     // its coefficient column: wc + k 2nk (A, then B)
    // each block's columns are contiguous in X: two DMA copies
    dma_copy(pv.X + (size_t)I * bs * R, xs, (size_t)nI * R * sizeof(V), wave, lane);
    dma_copy(pv.X + (size_t)J * bs * R, xs + (size_t)nI * R, (size_t)nJ * R * sizeof(V), wave, lane);
    for (int e = tid; e < nk * w2; e += kThreads) wc[e] = V{e % w2 == e / w2 ? T(1) : T(0), T(0)};
    __builtin_amdgcn_s_waitcnt(0);                   // this wave's copies have landed
    if (tid == 0) s_rot = 0;
    __syncthreads();
    const T tol = jacobi_tol<T>(R);
    const Acc negl2 = pv.hdr->negl2;
    bool rot = false;
    const int r = pv.r;
    auto step = [&](int i, int j) {
        V *xi = xs + (size_t)i * R, *xj = xs + (size_t)j * R, *wi = wc + (size_t)i * w2, *wj = wc + (size_t)j * w2;
        if constexpr (KR > 0)
            rot |= jacobi_pair_reg<T, V, KR, 1>(xi, xj, wi, wj, r, nk, pv.quat, tol, negl2, lane);
        else
            rot |= jacobi_pair<T, V>(xi, xj, wi, wj, r, nk, pv.quat, tol, negl2, lane);
    };
    if (t == 0) {
        // pairs within block I (staged 0 .. nI - 1) and within block J
        // (nI .. nk - 1), both on the circle schedule, in the same rounds
        const int pI = nI + (nI & 1), pJ = nJ + (nJ & 1);
        const int rounds = (pI > pJ ? pI : pJ) - 1;
        for (int tt = 0; tt < rounds; ++tt) {
            const int hI = tt < pI - 1 ? pI / 2 : 0, hJ = tt < pJ - 1 ? pJ / 2 : 0;
            for (int w = wave; w < hI + hJ; w += kWaves) {
                int i, j;
                if (w < hI) {
                    i = circle(w, tt, pI);
                    j = circle(pI - 1 - w, tt, pI);
                    if (i >= nI || j >= nI) continue;
                } else {
                    const int v = w - hI;
                    i = circle(v, tt, pJ);
                    j = circle(pJ - 1 - v, tt, pJ);
                    if (i >= nJ || j >= nJ) continue;
                    i += nI;
                    j += nI;
                }
                step(i, j);
            }
            __syncthreads();
        }
    }
    // pairs across the blocks: in round tt, unit k of I meets unit
    // (k + tt) mod bmax of J (disjoint within a round, all pairs over bmax rounds)
    const int bmax = nI > nJ ? nI : nJ;
    if (nI > 0 && nJ > 0) {
        for (int tt = 0; tt < bmax; ++tt) {
            for (int k = wave; k < bmax; k += kWaves) {
                const int l = (k + tt) % bmax;
                if (k < nI && l < nJ) step(k, nI + l);
            }
            __syncthreads();
        }
    }
    if (rot && lane == 0) s_rot = 1;
    __syncthreads();
    if (!s_rot) return;
    // write the data columns back in 16-byte words, four LDS reads in flight
    // per thread before the stores
    auto copy_out = [&](V* g, const V* sh, size_t bytes) {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        u4* gd = reinterpret_cast<u4*>(g);
        const u4* sd = reinterpret_cast<const u4*>(sh);
        const size_t n16 = bytes / 16;
        for (size_t i = tid; i < n16; i += 4 * kThreads) {
            u4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const size_t j = i + (size_t)u * kThreads;
                v[u] = j < n16 ? sd[j] : u4{0, 0, 0, 0};
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const size_t j = i + (size_t)u * kThreads;
                if (j < n16) gd[j] = v[u];
            }
        }
    };
    copy_out(pv.X + (size_t)I * bs * R, xs, (size_t)nI * R * sizeof(V));
    copy_out(pv.X + (size_t)J * bs * R, xs + (size_t)nI * R, (size_t)nJ * R * sizeof(V));
    V* QI = pv.Q + (size_t)I * bs * Rq;
    V* QJ = pv.Q + (size_t)J * bs * Rq - (size_t)nI * Rq;   // staged unit u >= nI: QJ + u Rq
    constexpr int MU = 2 * kBlockMaxBs;
    if (nk == MU) {
        if (pv.quat) apply_coefficients<true, true, V>(QI, QJ, nI, nk, Rq, wc, tid);
        else apply_coefficients<true, false, V>(QI, QJ, nI, nk, Rq, wc, tid);
    } else {
        if (pv.quat) apply_coefficients<false, true, V>(QI, QJ, nI, nk, Rq, wc, tid);
        else apply_coefficients<false, false, V>(QI, QJ, nI, nk, Rq, wc, tid);
    }
    if (tid == 0) pv.hdr->rot[sweep & 1] = 1;
}

// After sweep s: a pair whose sweep applied no rotation is done; the slot of
// sweep s is cleared for sweep s + 2.
template <typename T>
__global__ void __launch_bounds__(256) tsvd_check_kernel(TsvdArgs<T> a, int npairs, int sweep) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= npairs) return;
    PairHdr* h = reinterpret_cast<PairHdr*>(a.pairs + (size_t)f * a.pair_bytes);
    if (!h->done && !h->rot[sweep & 1]) h->done = 1;
    h->rot[sweep & 1] = 0;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) tsvd_finish_kernel(TsvdArgs<T> a) {
    __shared__ FinishSmem<T> sm;
    const PairView<T> pv = pair_view(a, blockIdx.x);
    pair_finish(a, pv, (T)pv.hdr->scale, pv.hdr->negl2, sm, false);
}

// Placement of the block path's vectors, spread over many workgroups: grid
// (tiles of 32 ranks, frequency pairs, 2), z = 0 the left vectors L, z = 1
// the rotation columns Q in rank order.  A tile of 32 columns x 64 entries is
// read along the columns into LDS and written along the slots, so that
// consecutive lanes store consecutive columns of a row.
template <typename T>
__global__ void __launch_bounds__(256) tsvd_place_kernel(TsvdArgs<T> a) {
    using V = typename Cx<T>::type;
    constexpr int TC = 32, TI = 64;
    __shared__ V tile[TC][TI + 1];
    const PairView<T> pv = pair_view(a, blockIdx.y);
    const bool left = blockIdx.z == 0;
    const int count = left ? pv.nL : pv.nu;
    const int rho0 = blockIdx.x * TC;
    if (rho0 >= count) return;
    const int half = left ? pv.r : pv.c, R = 2 * half, tid = threadIdx.x;
    const V* src = left ? pv.L : pv.Q;
    const int* perm = reinterpret_cast<const int*>(pv.coef);
    T* Yh = left == pv.tall ? a.Uh : a.Vh;
    const int ld = left == pv.tall ? a.ldu : a.ldv;
    for (int i0 = 0; i0 < R; i0 += TI) {
        for (int e = tid; e < TC * TI; e += 256) {
            const int cl = e / TI, il = e % TI, rho = rho0 + cl, i = i0 + il;
            if (rho < count && i < R) tile[cl][il] = src[(size_t)(left ? rho : perm[rho]) * R + i];
        }
        __syncthreads();
        for (int e = tid; e < TC * TI; e += 256) {
            const int cl = e % TC, il = e / TC, rho = rho0 + cl, i = i0 + il;
            if (rho < count && i < R) {
                const int slot = pv.quat ? rho : rho / 2 + ((rho & 1) ? half : 0);
                place_entry<T, V>(Yh, ld, a.p, half, pv.f, pv.g, slot, i, tile[cl][il]);
            }
        }
        __syncthreads();
    }
}

// S^ from sigma: S^1[f](i, i) = sigma[f][i], every other entry zero.
template <typename T>
__global__ void __launch_bounds__(256) tsvd_sigma_kernel(const T* __restrict__ sigma, T* __restrict__ Sh, int m, int n,
                                                         int p, int ld) {
    const int k = m < n ? m : n;
    const long total = 4L * p * m * ld;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int j = (int)(e % ld);
        const long rest = e / ld;
        const int i = (int)(rest % m);
        const long pf = rest / m;          // plane * p + face
        const int f = (int)(pf % p), plane = (int)(pf / p);
        Sh[e] = (plane == 0 && i == j && i < k) ? sigma[(size_t)f * k + i] : T(0);
    }
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
    if (!a || !b) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

struct TsvdLayout {
    size_t ah, uh, vh, sh, sig, pairs, pair_bytes, total;
};

TsvdLayout tsvd_layout(int m, int n, int p, int prec) {
    const size_t es = prec == QT_FP64 ? 8 : 4;
    TsvdLayout L{};
    size_t off = 0;
    auto take = [&](size_t b) { const size_t o = off; off += align_up(b); return o; };
    L.ah = take(4 * (size_t)p * m * fourier_ld(n) * es);
    L.uh = take(4 * (size_t)p * m * fourier_ld(m) * es);
    L.vh = take(4 * (size_t)p * n * fourier_ld(n) * es);
    L.sh = take(4 * (size_t)p * m * fourier_ld(n) * es);
    L.sig = take((size_t)p * (m < n ? m : n) * es);
    L.pair_bytes = prec == QT_FP64 ? pair_scratch_bytes<double>(m, n) : pair_scratch_bytes<float>(m, n);
    L.pairs = take((size_t)(p / 2 + 1) * L.pair_bytes);
    L.total = off;
    return L;
}

bool tsvd_dims_ok(int m, int n, int p) {
    return m >= 1 && n >= 1 && p >= 1 && p <= QT_MAX_P && (m < n ? m : n) <= kMaxMin &&
           (m > n ? m : n) <= kMaxMax;
}

// Staged units per block of the block sweeps for an m x n pair matrix (0:
// the single-workgroup kernel serves this size), and whether a block pair
// fits in half the LDS (two workgroups per CU).
template <typename T>
int tsvd_block_size(int m, int n, bool* half_lds) {
    const int r = m > n ? m : n, c = m > n ? n : m;
    int bs = kBlockMaxBs < c ? kBlockMaxBs : c;   // at least two blocks
    while (bs >= 4 && block_lds_bytes<T>(bs, 2 * r) > kBlockLds) --bs;
    // (FP32 only: the FP64 round kernel does not fit the register budget of
    // two workgroups per CU)
    *half_lds = sizeof(T) == 4 && block_lds_bytes<T>(bs, 2 * r) <= kBlockLdsHalf;
    return (bs >= 4 && 2 * c >= kBlockMinUnits) ? bs : 0;
}

// The pair kernels on a transformed A^: U^, V^ and sigma.
template <typename T>
hipError_t launch_tsvd_pairs(int m, int n, int p, const T* Ah, int lda, T* Uh, int ldu, T* Vh, int ldv, T* sigma,
                             char* pairs, hipStream_t stream) {
    const size_t pb = pair_scratch_bytes<T>(m, n);
    TsvdArgs<T> args{Ah, Uh, Vh, sigma, pairs, pb, m, n, p, lda, ldu, ldv};
    const int npairs = p / 2 + 1;
    bool half = false;
    const int bs = tsvd_block_size<T>(m, n, &half);
    if (!bs) {
        hipLaunchKernelGGL(tsvd_pair_kernel<T>, dim3(npairs), dim3(kThreads), 0, stream, args);
        return hipGetLastError();
    }
    const int c = m > n ? n : m;
    const int nb = (2 * c + bs - 1) / bs, nbp = nb + (nb & 1);
    hipLaunchKernelGGL(tsvd_prep_kernel<T>, dim3(npairs), dim3(kThreads), 0, stream, args);
    const int r = m > n ? m : n;
    auto round = [&](int t, int sweep) {
        const dim3 grid(nbp / 2, npairs), block(kThreads);
#define QT_ROUND(LDS, KR) hipLaunchKernelGGL((tsvd_round_kernel<T, LDS, KR>), grid, block, 0, stream, args, bs, t, sweep)
        if constexpr (sizeof(T) == 4) {
            // half: max(m, n) <= 272 (KR = 4 exceeds the register budget of
            // two workgroups per CU); otherwise the columns are longer than 256
            if (!half) QT_ROUND(kBlockLds, 0);
            else if (r <= 64) QT_ROUND(kBlockLdsHalf, 1);
            else QT_ROUND(kBlockLdsHalf, 0);
        } else {
            if (r <= 64) QT_ROUND(kBlockLds, 1);
            else if (r <= 256) QT_ROUND(kBlockLds, 4);
            else QT_ROUND(kBlockLds, 0);
        }
#undef QT_ROUND
    };
    for (int sweep = 0; sweep < kBlockMaxSweeps; ++sweep) {
        for (int t = 0; t < nbp - 1; ++t) round(t, sweep);
        hipLaunchKernelGGL(tsvd_check_kernel<T>, dim3((npairs + 255) / 256), dim3(256), 0, stream, args, npairs,
                           sweep);
    }
    hipLaunchKernelGGL(tsvd_finish_kernel<T>, dim3(npairs), dim3(kThreads), 0, stream, args);
    hipLaunchKernelGGL(tsvd_place_kernel<T>, dim3((2 * r + 31) / 32, npairs, 2), dim3(256), 0, stream, args);
    return hipGetLastError();
}

template <typename T>
int run_tsvd(int m, int n, int p, const T* A, T* U, T* S, T* V, T* sigma_out, int prec, char* ws,
             hipStream_t stream) {
    Twiddles tw;
    int st = get_twiddles(p, stream, &tw);
    if (st != QT_OK) return st;
    const TsvdLayout L = tsvd_layout(m, n, p, prec);
    T* Ah = reinterpret_cast<T*>(ws + L.ah);
    T* Uh = reinterpret_cast<T*>(ws + L.uh);
    T* Vh = reinterpret_cast<T*>(ws + L.vh);
    T* Sh = reinterpret_cast<T*>(ws + L.sh);
    T* sig = sigma_out ? sigma_out : reinterpret_cast<T*>(ws + L.sig);
    const int lda = (int)fourier_ld(n), ldu = (int)fourier_ld(m), ldv = (int)fourier_ld(n);

    FftJob<T> fwd[1] = {{A, Ah, m, n, n, lda, 0, 2, 0, 1}};
    if (launch_tube_fft<T>(p, false, fwd, 1, tw, stream) != hipSuccess) return QT_ERR_HIP;
    if (launch_tsvd_pairs<T>(m, n, p, Ah, lda, Uh, ldu, Vh, ldv, sig, ws + L.pairs, stream) != hipSuccess)
        return QT_ERR_HIP;
    if (S) {
        const long total = 4L * p * m * lda;
        const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
        hipLaunchKernelGGL(tsvd_sigma_kernel<T>, dim3(blocks), dim3(256), 0, stream, sig, Sh, m, n, p, lda);
        if (hipGetLastError() != hipSuccess) return QT_ERR_HIP;
    }
    FftJob<T> inv[3];
    int ninv = 0;
    if (U) inv[ninv++] = FftJob<T>{Uh, U, m, m, ldu, m};
    if (V) inv[ninv++] = FftJob<T>{Vh, V, n, n, ldv, n};
    if (S) inv[ninv++] = FftJob<T>{Sh, S, m, n, lda, n};
    for (int q = 0; q < ninv; q += 2) {
        if (launch_tube_fft<T>(p, true, inv + q, ninv - q < 2 ? ninv - q : 2, tw, stream) != hipSuccess)
            return QT_ERR_HIP;
    }
    return QT_OK;
}

int tsvd_ws(int m, int n, int p, const void* A, void* U, void* S, void* V, void* sigma, qt_precision prec,
            void* ws, size_t ws_bytes, hipStream_t stream) {
    if (prec != QT_FP32 && prec != QT_FP64 && prec != QT_SPLIT_BF16 && prec != QT_SPLIT_FP16)
        return QT_ERR_INVALID_ARG;
    if (m < 1 || n < 1 || p < 1 || !A || !aligned16(A)) return QT_ERR_INVALID_ARG;
    const size_t es = prec == QT_FP64 ? 8 : 4;
    const void* outs[4] = {U, S, V, sigma};
    const size_t k = m < n ? m : n;
    const size_t osz[4] = {4 * (size_t)p * m * m * es, 4 * (size_t)p * m * n * es, 4 * (size_t)p * n * n * es,
                           (size_t)p * k * es};
    const size_t abytes = 4 * (size_t)p * m * n * es;
    for (int q = 0; q < 4; ++q) {
        if (outs[q] && !aligned16(outs[q])) return QT_ERR_INVALID_ARG;
        if (overlaps(outs[q], osz[q], A, abytes)) return QT_ERR_INVALID_ARG;
        for (int o = 0; o < q; ++o)
            if (overlaps(outs[q], osz[q], outs[o], osz[o])) return QT_ERR_INVALID_ARG;
    }
    if (prec != QT_FP32 && prec != QT_FP64) return QT_ERR_UNSUPPORTED;
    if (!tsvd_dims_ok(m, n, p)) return QT_ERR_UNSUPPORTED;
    const TsvdLayout L = tsvd_layout(m, n, p, prec);
    if (!ws || !aligned16(ws) || ws_bytes < L.total) return QT_ERR_INVALID_ARG;
    for (int q = 0; q < 4; ++q)
        if (overlaps(outs[q], osz[q], ws, L.total)) return QT_ERR_INVALID_ARG;
    if (overlaps(A, abytes, ws, L.total)) return QT_ERR_INVALID_ARG;
    if (!U && !S && !V && !sigma) return QT_OK;
    if (prec == QT_FP64)
        return run_tsvd<double>(m, n, p, (const double*)A, (double*)U, (double*)S, (double*)V, (double*)sigma,
                                prec, (char*)ws, stream);
    return run_tsvd<float>(m, n, p, (const float*)A, (float*)U, (float*)S, (float*)V, (float*)sigma, prec,
                           (char*)ws, stream);
}

}  // namespace
}  // namespace qt

extern "C" {

size_t qt_tsvd_workspace_size(int m, int n, int p, qt_precision precision) {
    if ((precision != QT_FP32 && precision != QT_FP64) || !qt::tsvd_dims_ok(m, n, p)) return 0;
    return qt::tsvd_layout(m, n, p, precision).total;
}

size_t qt_fourier_tsvd_workspace_size(int m, int n, int p, qt_precision precision) {
    if ((precision != QT_FP32 && precision != QT_FP64) || !qt::tsvd_dims_ok(m, n, p)) return 0;
    const size_t pb = precision == QT_FP64 ? qt::pair_scratch_bytes<double>(m, n)
                                           : qt::pair_scratch_bytes<float>(m, n);
    return (size_t)(p / 2 + 1) * pb;
}

qt_status qt_fourier_tsvd(int m, int n, int p, const void* Ah, int lda, void* Uh, int ldu, void* Vh, int ldv,
                          void* sigma, qt_precision precision, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (precision != QT_FP32 && precision != QT_FP64 && precision != QT_SPLIT_BF16 && precision != QT_SPLIT_FP16)
        return QT_ERR_INVALID_ARG;
    if (m < 1 || n < 1 || p < 1 || !Ah || !Uh || !Vh || !sigma || !ws) return QT_ERR_INVALID_ARG;
    if (lda < n || ldu < m || ldv < n) return QT_ERR_INVALID_ARG;
    if (!qt::aligned16(Ah) || !qt::aligned16(Uh) || !qt::aligned16(Vh) || !qt::aligned16(sigma) ||
        !qt::aligned16(ws))
        return QT_ERR_INVALID_ARG;
    if (precision != QT_FP32 && precision != QT_FP64) return QT_ERR_UNSUPPORTED;
    if (!qt::tsvd_dims_ok(m, n, p)) return QT_ERR_UNSUPPORTED;
    const size_t es = precision == QT_FP64 ? 8 : 4;
    const size_t need = qt_fourier_tsvd_workspace_size(m, n, p, precision);
    if (ws_bytes < need) return QT_ERR_INVALID_ARG;
    const size_t k = m < n ? m : n;
    const void* bufs[5] = {Ah, Uh, Vh, sigma, ws};
    const size_t sz[5] = {4 * (size_t)p * m * lda * es, 4 * (size_t)p * m * ldu * es, 4 * (size_t)p * n * ldv * es,
                          (size_t)p * k * es, need};
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < a; ++b)
            if (qt::overlaps(bufs[a], sz[a], bufs[b], sz[b])) return QT_ERR_INVALID_ARG;
    hipError_t e;
    if (precision == QT_FP64)
        e = qt::launch_tsvd_pairs<double>(m, n, p, (const double*)Ah, lda, (double*)Uh, ldu, (double*)Vh, ldv,
                                          (double*)sigma, (char*)ws, stream);
    else
        e = qt::launch_tsvd_pairs<float>(m, n, p, (const float*)Ah, lda, (float*)Uh, ldu, (float*)Vh, ldv,
                                         (float*)sigma, (char*)ws, stream);
    return e == hipSuccess ? QT_OK : QT_ERR_HIP;
}

qt_status qt_tsvd(int m, int n, int p, const void* A, void* U, void* S, void* V, void* sigma,
                  qt_precision precision, void* ws, size_t ws_bytes, hipStream_t stream) {
    return qt::with_workspace(ws, ws_bytes, qt_tsvd_workspace_size(m, n, p, precision), stream,
                              [&](void* w, size_t wb) {
                                  return qt::tsvd_ws(m, n, p, A, U, S, V, sigma, precision, w, wb, stream);
                              });
}

}  // extern "C"
