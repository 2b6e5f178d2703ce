// C-ABI entry points of libqtprod (declared in include/qtprod.h).
//
// Host side only: argument validation, the per-(device, p) plan cache
// (twiddle tables), workspace carving and kernel launches.  Every step of the
// T-product itself runs in the HIP kernels of fft.hip and facewise.hip.
#include <mutex>
#include <unordered_map>

#include "qt_internal.h"
#include "workspace.h"
#include "../../include/qtprod.h"

namespace {

using qt::FftJob;
using qt::FacewiseArgs;
using qt::Twiddles;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool valid_precision(int prec) {
    return prec == QT_FP32 || prec == QT_SPLIT_BF16 || prec == QT_SPLIT_FP16 || prec == QT_FP64;
}

size_t real_bytes(int prec) { return prec == QT_FP64 ? 8 : 4; }

bool dims_ok(long rows, long cols, long p) {
    if (rows < 1 || cols < 1 || p < 1) return false;
    // element counts must stay far from 64-bit overflow and within 2^40
    const double elems = 4.0 * (double)p * (double)rows * (double)qt::fourier_ld(cols);
    return elems < (double)(1LL << 40);
}

bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

size_t tensor_bytes(long rows, long cols, long p, int prec) {
    return 4 * (size_t)p * (size_t)rows * (size_t)cols * real_bytes(prec);
}

size_t fourier_bytes(long rows, long cols, long p, int prec) {
    return align_up(4 * (size_t)p * (size_t)rows * (size_t)qt::fourier_ld(cols) * real_bytes(prec));
}

// Every p up to QT_MAX_P: register-resident kernels for the 7-smooth lengths
// they cover, Bluestein for all others.
bool p_supported(int p, int prec) {
    (void)prec;
    return p >= 1 && p <= QT_MAX_P;
}

// ------------------------------------------------------------- plan cache
struct PlanKey {
    int device, p;
    bool operator==(const PlanKey& o) const { return device == o.device && p == o.p; }
};
struct PlanKeyHash {
    size_t operator()(const PlanKey& k) const { return ((size_t)k.device << 32) ^ (size_t)k.p; }
};

std::mutex g_plan_mutex;
std::unordered_map<PlanKey, Twiddles, PlanKeyHash> g_plans;

}  // namespace

namespace qt {
bool find_twiddles(int p, Twiddles* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lock(g_plan_mutex);
    auto it = g_plans.find(PlanKey{dev, p});
    if (it == g_plans.end()) return false;
    *out = it->second;
    return true;
}

int get_twiddles(int p, hipStream_t stream, Twiddles* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return QT_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_plan_mutex);
    auto it = g_plans.find(PlanKey{dev, p});
    if (it != g_plans.end()) {
        *out = it->second;
        return QT_OK;
    }
    Twiddles tw{};
    if (hipMalloc((void**)&tw.f32, sizeof(float2) * (size_t)p) != hipSuccess) return QT_ERR_ALLOC;
    if (hipMalloc((void**)&tw.f64, sizeof(double2) * (size_t)p) != hipSuccess) {
        (void)hipFree(tw.f32);
        return QT_ERR_ALLOC;
    }
    bool ok = qt::launch_twiddles(p, tw, stream) == hipSuccess;
    const size_t tb = qt::bluestein_tables_bytes(p);
    if (ok && tb) {
        char* mem = nullptr;
        if (hipMalloc((void**)&mem, tb) != hipSuccess) {
            (void)hipFree(tw.f32);
            (void)hipFree(tw.f64);
            return QT_ERR_ALLOC;
        }
        qt::carve_bluestein_tables(p, mem, &tw.blue);
        ok = qt::launch_bluestein_tables(p, tw.blue, stream) == hipSuccess;
    }
    if (!ok || hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipFree(tw.f32);
        (void)hipFree(tw.f64);
        if (tw.blue.M) (void)hipFree(tw.blue.chirp64);
        return QT_ERR_HIP;
    }
    g_plans.emplace(PlanKey{dev, p}, tw);
    *out = tw;
    return QT_OK;
}
}  // namespace qt

namespace {
using qt::get_twiddles;
int get_plan(int p, hipStream_t stream, Twiddles* out) { return get_twiddles(p, stream, out); }

// ------------------------------------------------------------- forward path
template <typename T>
hipError_t facewise(const FacewiseArgs<T>& fa, int prec, hipStream_t stream) {
    if constexpr (sizeof(T) == 8) return qt::launch_facewise_f64(fa, stream);
    else return qt::launch_facewise_f32(fa, prec, stream, qt::choose_tile(fa.m, fa.n, fa.s, prec));
}

int hip_status(hipError_t e) {
    if (e == hipSuccess) return QT_OK;
    return e == hipErrorNotSupported ? QT_ERR_UNSUPPORTED : QT_ERR_HIP;
}

// given: a ready plan for p (the allocation-free entry point), else the
// plan cache is used.
template <typename T>
int run_tprod(int m, int n, int s, int p, const T* A, const T* B, T* C, int prec, char* ws,
              hipStream_t stream, const Twiddles* given = nullptr) {
    Twiddles tw;
    int st = QT_OK;
    if (given) tw = *given;
    else st = get_plan(p, stream, &tw);
    if (st != QT_OK) return st;
    const int lda = (int)qt::fourier_ld(n), ldb = (int)qt::fourier_ld(s), ldc = ldb;
    T* Ah = reinterpret_cast<T*>(ws);
    T* Bh = reinterpret_cast<T*>(ws + fourier_bytes(m, n, p, prec));
    T* Ch = reinterpret_cast<T*>(ws + fourier_bytes(m, n, p, prec) + fourier_bytes(n, s, p, prec));

    // step 1: tube FFT of A and B (one launch); split-bf16 operands leave the
    // FFT already split into hi/lo words
    const int pack = prec == QT_SPLIT_BF16 ? 1 : 0;
    FftJob<T> fwd[2] = {{A, Ah, m, n, n, lda, pack, 2, 0, 1}, {B, Bh, n, s, s, ldb, pack, 2, 0, 1}};
    if (qt::launch_tube_fft<T>(p, false, fwd, 2, tw, stream) != hipSuccess) return QT_ERR_HIP;

    // step 2: coupled facewise products
    FacewiseArgs<T> fa{Ah, Bh, Ch, m, n, s, p, lda, ldb, ldc};
    if constexpr (sizeof(T) == 4) {
        if (prec == QT_SPLIT_FP16) {
            char* sc = ws + fourier_bytes(m, n, p, prec) + fourier_bytes(n, s, p, prec) +
                       fourier_bytes(m, s, p, prec);
            float* scales = reinterpret_cast<float*>(sc);
            float* partials = scales + 2 * (size_t)p;
            st = hip_status(qt::launch_fp16_scales(fa, partials, scales, stream));
            if (st != QT_OK) return st;
            if (s > qt::kNarrowMaxS) {
                // scaled fp16 words in place (narrow products read the FP32 values)
                st = hip_status(qt::launch_fp16_words(Ah, p, m, n, lda, scales, stream));
                if (st != QT_OK) return st;
                st = hip_status(qt::launch_fp16_words(Bh, p, n, s, ldb, scales + p, stream));
                if (st != QT_OK) return st;
            }
            st = hip_status(qt::launch_facewise_f32(fa, prec, stream, qt::choose_tile(m, n, s, prec), scales));
            if (st != QT_OK) return st;
            FftJob<T> inv16[1] = {{Ch, C, m, s, ldc, s}};
            return hip_status(qt::launch_tube_fft<T>(p, true, inv16, 1, tw, stream));
        }
    }
    st = hip_status(facewise<T>(fa, prec, stream));
    if (st != QT_OK) return st;

    // step 3: inverse tube FFT of C^ into C
    FftJob<T> inv[1] = {{Ch, C, m, s, ldc, s}};
    if (qt::launch_tube_fft<T>(p, true, inv, 1, tw, stream) != hipSuccess) return QT_ERR_HIP;
    return QT_OK;
}

// ------------------------------------------------------------ backward path
// Workspace regions of the backward pass (each 256-byte aligned):
//   Y  = B^H (s x n x p, dense)      Z  = A^H (n x m x p, dense)
//   G^ (m x s, row stride ld(s))     Y^ (s x n, ld(n))     Z^ (n x m, ld(m))
//   dA^ (m x n, ld(n))               dB^ (n x s, ld(s))
// Split-fp16 adds a second transform of G (each product scales and rewrites
// its operands in place, and G^ is an operand of both) and the scales and
// max-abs partials of the two products.
struct BackwardLayout {
    size_t y, z, gh, yh, zh, dah, dbh, gh2, sc1, sc2, total;
};

size_t fp16_scale_floats(long rows, long k, long cols, long p) {
    return (size_t)p * (2 + qt::fp16_partial_blocks(rows, k) + qt::fp16_partial_blocks(k, cols));
}

BackwardLayout backward_layout(long m, long n, long s, long p, int prec) {
    BackwardLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    L.y = take(tensor_bytes(s, n, p, prec));
    L.z = take(tensor_bytes(n, m, p, prec));
    L.gh = take(fourier_bytes(m, s, p, prec));
    L.yh = take(fourier_bytes(s, n, p, prec));
    L.zh = take(fourier_bytes(n, m, p, prec));
    L.dah = take(fourier_bytes(m, n, p, prec));
    L.dbh = take(fourier_bytes(n, s, p, prec));
    if (prec == QT_SPLIT_FP16) {
        L.gh2 = take(fourier_bytes(m, s, p, prec));
        L.sc1 = take(sizeof(float) * fp16_scale_floats(m, s, n, p));   // dA = G * B^H
        L.sc2 = take(sizeof(float) * fp16_scale_floats(n, m, s, p));   // dB = A^H * G
    }
    L.total = off;
    return L;
}

// One split-fp16 product on FP32 Fourier operands: per-frequency scales,
// scaled fp16 words written over both operands (narrow products read the
// FP32 values), the product, scales undone at the store.
int fp16_product(const FacewiseArgs<float>& fa, float* sc, hipStream_t stream) {
    float* scales = sc;
    float* partials = sc + 2 * (size_t)fa.p;
    int st = hip_status(qt::launch_fp16_scales(fa, partials, scales, stream));
    if (st != QT_OK) return st;
    if (fa.s > qt::kNarrowMaxS) {
        st = hip_status(qt::launch_fp16_words(const_cast<float*>(fa.Ah), fa.p, fa.m, fa.n, fa.lda, scales, stream));
        if (st != QT_OK) return st;
        st = hip_status(qt::launch_fp16_words(const_cast<float*>(fa.Bh), fa.p, fa.n, fa.s, fa.ldb, scales + fa.p,
                                              stream));
        if (st != QT_OK) return st;
    }
    return hip_status(qt::launch_facewise_f32(fa, QT_SPLIT_FP16, stream,
                                              qt::choose_tile(fa.m, fa.n, fa.s, QT_SPLIT_FP16), scales));
}

// dA = G * B^H and dB = A^H * G: transpose-conjugate B and A, one FFT of G
// shared by both products (it is the left operand of the first and the right
// operand of the second, with the same Fourier layout), two coupled facewise
// products, one inverse FFT launch for both results.
template <typename T>
int run_backward(int m, int n, int s, int p, const T* A, const T* B, const T* G, T* dA, T* dB,
                 int prec, char* ws, hipStream_t stream) {
    Twiddles tw;
    int st = get_plan(p, stream, &tw);
    if (st != QT_OK) return st;
    const BackwardLayout L = backward_layout(m, n, s, p, prec);
    const int ldm = (int)qt::fourier_ld(m), ldn = (int)qt::fourier_ld(n), lds = (int)qt::fourier_ld(s);
    T* Y = reinterpret_cast<T*>(ws + L.y);
    T* Z = reinterpret_cast<T*>(ws + L.z);
    T* Gh = reinterpret_cast<T*>(ws + L.gh);
    T* Yh = reinterpret_cast<T*>(ws + L.yh);
    T* Zh = reinterpret_cast<T*>(ws + L.zh);
    T* dAh = reinterpret_cast<T*>(ws + L.dah);
    T* dBh = reinterpret_cast<T*>(ws + L.dbh);

    qt::ConjTJob<T> cj[2];
    int ncj = 0;
    if (dA) cj[ncj++] = qt::ConjTJob<T>{B, Y, n, s, p, 0};
    if (dB) cj[ncj++] = qt::ConjTJob<T>{A, Z, m, n, p, 0};
    st = hip_status(qt::launch_conj_transpose<T>(cj, ncj, stream));
    if (st != QT_OK) return st;

    const int pack = prec == QT_SPLIT_BF16 ? 1 : 0;
    FftJob<T> f1[2] = {{G, Gh, m, s, s, lds, pack, 2, 0, 1}, {Y, Yh, s, n, n, ldn, pack, 2, 0, 1}};
    st = hip_status(qt::launch_tube_fft<T>(p, false, f1, dA ? 2 : 1, tw, stream));
    if (st != QT_OK) return st;
    if (dB) {
        FftJob<T> f2[1] = {{Z, Zh, n, m, m, ldm, pack, 2, 0, 1}};
        st = hip_status(qt::launch_tube_fft<T>(p, false, f2, 1, tw, stream));
        if (st != QT_OK) return st;
    }
    if constexpr (sizeof(T) == 4) {
        if (prec == QT_SPLIT_FP16) {
            // G^ is the left operand of dA and the right one of dB, each
            // rewritten in place with its own scales: dB gets a second copy
            T* Gb = Gh;
            if (dA && dB) {
                Gb = reinterpret_cast<T*>(ws + L.gh2);
                FftJob<T> f3[1] = {{G, Gb, m, s, s, lds, 0, 2, 0, 1}};
                st = hip_status(qt::launch_tube_fft<T>(p, false, f3, 1, tw, stream));
                if (st != QT_OK) return st;
            }
            if (dA) {
                st = fp16_product(FacewiseArgs<T>{Gh, Yh, dAh, m, s, n, p, lds, ldn, ldn},
                                  reinterpret_cast<float*>(ws + L.sc1), stream);
                if (st != QT_OK) return st;
            }
            if (dB) {
                st = fp16_product(FacewiseArgs<T>{Zh, Gb, dBh, n, m, s, p, ldm, lds, lds},
                                  reinterpret_cast<float*>(ws + L.sc2), stream);
                if (st != QT_OK) return st;
            }
            FftJob<T> inv16[2];
            int n16 = 0;
            if (dA) inv16[n16++] = FftJob<T>{dAh, dA, m, n, ldn, n};
            if (dB) inv16[n16++] = FftJob<T>{dBh, dB, n, s, lds, s};
            return hip_status(qt::launch_tube_fft<T>(p, true, inv16, n16, tw, stream));
        }
    }
    if (dA) {
        FacewiseArgs<T> fa{Gh, Yh, dAh, m, s, n, p, lds, ldn, ldn};
        st = hip_status(facewise<T>(fa, prec, stream));
        if (st != QT_OK) return st;
    }
    if (dB) {
        FacewiseArgs<T> fb{Zh, Gh, dBh, n, m, s, p, ldm, lds, lds};
        st = hip_status(facewise<T>(fb, prec, stream));
        if (st != QT_OK) return st;
    }
    FftJob<T> inv[2];
    int ninv = 0;
    if (dA) inv[ninv++] = FftJob<T>{dAh, dA, m, n, ldn, n};
    if (dB) inv[ninv++] = FftJob<T>{dBh, dB, n, s, lds, s};
    return hip_status(qt::launch_tube_fft<T>(p, true, inv, ninv, tw, stream));
}

}  // namespace

extern "C" {

int qt_version(void) { return 100; }

const char* qt_status_string(qt_status status) {
    switch ((int)status) {
        case QT_OK: return "QT_OK";
        case QT_ERR_INVALID_ARG: return "QT_ERR_INVALID_ARG: invalid size, pointer, alignment, aliasing or workspace";
        case QT_ERR_UNSUPPORTED: return "QT_ERR_UNSUPPORTED: request not supported by this build";
        case QT_ERR_ALLOC: return "QT_ERR_ALLOC: device allocation failed";
        case QT_ERR_HIP: return "QT_ERR_HIP: HIP runtime or launch error";
        case QT_ERR_TOO_LARGE: return "QT_ERR_TOO_LARGE: problem exceeds the allocation-free scratch";
        default: return "unknown qt_status";
    }
}

qt_status qt_prepare(int p, hipStream_t stream) {
    if (p < 1) return QT_ERR_INVALID_ARG;
    if (p > QT_MAX_P) return QT_ERR_UNSUPPORTED;
    Twiddles tw;
    return qt::to_status(get_plan(p, stream, &tw));
}

int qt_fourier_ld(int cols) { return cols < 1 ? 0 : (int)qt::fourier_ld(cols); }

qt_status qt_tube_fft(int rows, int cols, int p, const void* X, int ldx, void* Xh, int ldh, int inverse,
                qt_precision precision, hipStream_t stream) {
    if (!valid_precision(precision)) return QT_ERR_INVALID_ARG;
    if (!dims_ok(rows, cols, p) || !X || !Xh || !aligned16(X) || !aligned16(Xh))
        return QT_ERR_INVALID_ARG;
    if (ldx < cols || ldh < cols || !dims_ok(rows, ldx, p) || !dims_ok(rows, ldh, p))
        return QT_ERR_INVALID_ARG;
    if (inverse != 0 && inverse != 1) return QT_ERR_INVALID_ARG;
    if (overlaps(X, tensor_bytes(rows, ldx, p, precision), Xh, tensor_bytes(rows, ldh, p, precision)))
        return QT_ERR_INVALID_ARG;
    if (!p_supported(p, precision)) return QT_ERR_UNSUPPORTED;
    Twiddles tw;
    int st = get_plan(p, stream, &tw);
    if (st != QT_OK) return qt::to_status(st);
    hipError_t e;
    if (precision == QT_FP64) {
        FftJob<double> j{(const double*)X, (double*)Xh, rows, cols, ldx, ldh};
        e = qt::launch_tube_fft<double>(p, inverse != 0, &j, 1, tw, stream);
    } else {
        const int pack = (precision == QT_SPLIT_BF16 && !inverse) ? 1 : 0;
        FftJob<float> j{(const float*)X, (float*)Xh, rows, cols, ldx, ldh, pack};
        e = qt::launch_tube_fft<float>(p, inverse != 0, &j, 1, tw, stream);
    }
    return qt::to_status(e == hipSuccess ? QT_OK : QT_ERR_HIP);
}

qt_status qt_fourier_tprod(int m, int n, int s, int p, const void* Ah, int lda, const void* Bh, int ldb,
                     void* Ch, int ldc, qt_precision precision, hipStream_t stream) {
    if (!valid_precision(precision)) return QT_ERR_INVALID_ARG;
    if (!dims_ok(m, n, p) || !dims_ok(n, s, p) || !dims_ok(m, s, p)) return QT_ERR_INVALID_ARG;
    if (!Ah || !Bh || !Ch || !aligned16(Ah) || !aligned16(Bh) || !aligned16(Ch))
        return QT_ERR_INVALID_ARG;
    if (lda < n || ldb < s || ldc < s) return QT_ERR_INVALID_ARG;
    if (precision != QT_FP64 && ((lda | ldb | ldc) & 3)) return QT_ERR_INVALID_ARG;
    if (precision == QT_SPLIT_FP16) return QT_ERR_UNSUPPORTED;   // needs scales: use qt_tprod
    if (!dims_ok(m, lda, p) || !dims_ok(n, ldb, p) || !dims_ok(m, ldc, p)) return QT_ERR_INVALID_ARG;
    const size_t cb = tensor_bytes(m, ldc, p, precision);
    if (overlaps(Ch, cb, Ah, tensor_bytes(m, lda, p, precision)) ||
        overlaps(Ch, cb, Bh, tensor_bytes(n, ldb, p, precision)))
        return QT_ERR_INVALID_ARG;
    hipError_t e;
    if (precision == QT_FP64) {
        FacewiseArgs<double> fa{(const double*)Ah, (const double*)Bh, (double*)Ch, m, n, s, p,
                                lda, ldb, ldc};
        e = qt::launch_facewise_f64(fa, stream);
    } else {
        FacewiseArgs<float> fa{(const float*)Ah, (const float*)Bh, (float*)Ch, m, n, s, p,
                               lda, ldb, ldc};
        e = qt::launch_facewise_f32(fa, precision, stream);
    }
    if (e == hipErrorNotSupported) return QT_ERR_UNSUPPORTED;
    return qt::to_status(e == hipSuccess ? QT_OK : QT_ERR_HIP);
}

qt_status qt_split_words(int rows, int cols, int p, void* Xh, int ld, hipStream_t stream) {
    if (!dims_ok(rows, cols, p) || !Xh || !aligned16(Xh)) return QT_ERR_INVALID_ARG;
    if (ld < cols || (ld & 3) || !dims_ok(rows, ld, p)) return QT_ERR_INVALID_ARG;
    return qt::to_status(hip_status(qt::launch_split_words((float*)Xh, 4L * p, rows, cols, ld, stream)));
}

size_t qt_workspace_size(int m, int n, int s, int p, qt_precision precision) {
    if (!valid_precision(precision) || !dims_ok(m, n, p) || !dims_ok(n, s, p) || !dims_ok(m, s, p))
        return 0;
    size_t total = fourier_bytes(m, n, p, precision) + fourier_bytes(n, s, p, precision) +
                   fourier_bytes(m, s, p, precision);
    if (precision == QT_SPLIT_FP16)    // scales (2p floats) and max-abs partials
        total += align_up(sizeof(float) * (size_t)p *
                          (2 + qt::fp16_partial_blocks(m, n) + qt::fp16_partial_blocks(n, s)));
    return total;
}

}  // extern "C"

namespace qt {
// Arguments of qt_tprod other than the workspace.
int check_tprod(int m, int n, int s, int p, const void* A, const void* B, const void* C,
                int precision) {
    if (!valid_precision(precision)) return QT_ERR_INVALID_ARG;
    if (!dims_ok(m, n, p) || !dims_ok(n, s, p) || !dims_ok(m, s, p)) return QT_ERR_INVALID_ARG;
    if (!A || !B || !C) return QT_ERR_INVALID_ARG;
    if (!aligned16(A) || !aligned16(B) || !aligned16(C)) return QT_ERR_INVALID_ARG;
    const size_t cb = tensor_bytes(m, s, p, precision);
    if (overlaps(C, cb, A, tensor_bytes(m, n, p, precision)) ||
        overlaps(C, cb, B, tensor_bytes(n, s, p, precision)))
        return QT_ERR_INVALID_ARG;
    return QT_OK;
}

int dispatch_tprod(int m, int n, int s, int p, const void* A, const void* B, void* C,
                   int precision, char* ws, hipStream_t stream, const Twiddles* given) {
    if (precision == QT_FP64)
        return run_tprod<double>(m, n, s, p, (const double*)A, (const double*)B, (double*)C, precision,
                                 ws, stream, given);
    return run_tprod<float>(m, n, s, p, (const float*)A, (const float*)B, (float*)C, precision, ws,
                            stream, given);
}
}  // namespace qt

namespace {
int tprod_ws(int m, int n, int s, int p, const void* A, const void* B, void* C, qt_precision precision,
             void* ws, size_t ws_bytes, hipStream_t stream) {
    int st = qt::check_tprod(m, n, s, p, A, B, C, precision);
    if (st != QT_OK) return st;
    if (!ws || !aligned16(ws)) return QT_ERR_INVALID_ARG;
    const size_t need = qt_workspace_size(m, n, s, p, precision);
    if (ws_bytes < need) return QT_ERR_INVALID_ARG;
    if (overlaps(ws, need, A, tensor_bytes(m, n, p, precision)) ||
        overlaps(ws, need, B, tensor_bytes(n, s, p, precision)) ||
        overlaps(ws, need, C, tensor_bytes(m, s, p, precision)))
        return QT_ERR_INVALID_ARG;
    if (!p_supported(p, precision)) return QT_ERR_UNSUPPORTED;
    return qt::dispatch_tprod(m, n, s, p, A, B, C, precision, (char*)ws, stream, nullptr);
}

}  // namespace

extern "C" {

qt_status qt_tprod(int m, int n, int s, int p, const void* A, const void* B, void* C, qt_precision precision,
             void* ws, size_t ws_bytes, hipStream_t stream) {
    return qt::with_workspace(ws, ws_bytes, qt_workspace_size(m, n, s, p, precision), stream,
                              [&](void* w, size_t wb) { return tprod_ws(m, n, s, p, A, B, C, precision, w, wb, stream); });
}

// ------------------------------------------- complex and real T-products
namespace {

// Fourier-side faces: p for complex tensors, p / 2 + 1 for real ones (the
// spectrum of a real tube is Hermitian).
int cx_faces(int p, bool real) { return real ? p / 2 + 1 : p; }

size_t cx_workspace(int m, int n, int s, int p, qt_precision precision, bool real) {
    if ((precision != QT_FP32 && precision != QT_SPLIT_BF16 && precision != QT_SPLIT_FP16) || !dims_ok(m, n, p) ||
        !dims_ok(n, s, p) || !dims_ok(m, s, p))
        return 0;
    const long h = cx_faces(p, real);
    // two planes (Re, Im) of h faces per tensor
    auto part = [h](long rows, long cols) {
        return align_up(2 * (size_t)h * (size_t)rows * (size_t)qt::fourier_ld(cols) * sizeof(float));
    };
    size_t total = part(m, n) + part(n, s) + part(m, s);
    if (precision == QT_SPLIT_FP16)    // scales (2h floats) and max-abs partials
        total += align_up(sizeof(float) * (size_t)h *
                          (2 + qt::fp16_partial_blocks(m, n) + qt::fp16_partial_blocks(n, s)));
    return total;
}

// Forward transforms of A and B (two planes, or one real plane to a half
// spectrum), the uncoupled per-frequency complex products, and the inverse.
int run_cx(int m, int n, int s, int p, const void* A, const void* B, void* C, qt_precision precision, void* ws,
           size_t ws_bytes, bool real, hipStream_t stream) {
    if (precision != QT_FP32 && precision != QT_SPLIT_BF16 && precision != QT_SPLIT_FP16) {
        return valid_precision(precision) ? QT_ERR_UNSUPPORTED : QT_ERR_INVALID_ARG;
    }
    if (!dims_ok(m, n, p) || !dims_ok(n, s, p) || !dims_ok(m, s, p)) return QT_ERR_INVALID_ARG;
    if (!A || !B || !C || !ws) return QT_ERR_INVALID_ARG;
    if (!aligned16(A) || !aligned16(B) || !aligned16(C) || !aligned16(ws)) return QT_ERR_INVALID_ARG;
    const size_t need = cx_workspace(m, n, s, p, precision, real);
    if (ws_bytes < need) return QT_ERR_INVALID_ARG;
    const int planes = real ? 1 : 2;
    const size_t ab = tensor_bytes(m, n, p, precision) / 4 * planes;
    const size_t bb = tensor_bytes(n, s, p, precision) / 4 * planes;
    const size_t cb = tensor_bytes(m, s, p, precision) / 4 * planes;
    if (overlaps(C, cb, A, ab) || overlaps(C, cb, B, bb) || overlaps(ws, need, A, ab) ||
        overlaps(ws, need, B, bb) || overlaps(ws, need, C, cb))
        return QT_ERR_INVALID_ARG;
    if (!p_supported(p, precision)) return QT_ERR_UNSUPPORTED;
    Twiddles tw;
    int st = get_plan(p, stream, &tw);
    if (st != QT_OK) return qt::to_status(st);
    const int h = cx_faces(p, real);
    const int lda = (int)qt::fourier_ld(n), ldb = (int)qt::fourier_ld(s), ldc = ldb;
    char* w = (char*)ws;
    const size_t a_bytes = align_up(2 * (size_t)h * m * lda * sizeof(float));
    const size_t b_bytes = align_up(2 * (size_t)h * n * ldb * sizeof(float));
    float* Ah = reinterpret_cast<float*>(w);
    float* Bh = reinterpret_cast<float*>(w + a_bytes);
    float* Ch = reinterpret_cast<float*>(w + a_bytes + b_bytes);
    const int pack = precision == QT_SPLIT_BF16 ? 1 : 0;
    const int hf = real ? 1 : 0;
    // one CD part (planes 0, 1) per tensor
    FftJob<float> fwd[2] = {{(const float*)A, Ah, m, n, n, lda, pack, 1, hf, 1},
                            {(const float*)B, Bh, n, s, s, ldb, pack, 1, hf, 1}};
    if (qt::launch_tube_fft<float>(p, false, fwd, 2, tw, stream) != hipSuccess) return QT_ERR_HIP;
    FacewiseArgs<float> fa{Ah, Bh, Ch, m, n, s, h, lda, ldb, ldc};
    const float* scales = nullptr;
    if (precision == QT_SPLIT_FP16) {
        // per-frequency scales of A^ and B^ (no -f coupling), then the scaled
        // fp16 words written over both operands
        const size_t c_bytes = align_up(2 * (size_t)h * m * ldc * sizeof(float));
        float* sc = reinterpret_cast<float*>(w + a_bytes + b_bytes + c_bytes);
        st = hip_status(qt::launch_fp16_scales(fa, sc + 2 * (size_t)h, sc, stream, 2));
        if (st == QT_OK) st = hip_status(qt::launch_fp16_words(Ah, h, m, n, lda, sc, stream, 2));
        if (st == QT_OK) st = hip_status(qt::launch_fp16_words(Bh, h, n, s, ldb, sc + h, stream, 2));
        if (st != QT_OK) return qt::to_status(st);
        scales = sc;
    }
    const int mode = precision == QT_SPLIT_BF16 ? 1 : precision == QT_SPLIT_FP16 ? 2 : 0;
    st = hip_status(qt::launch_facewise_cx(fa, mode, stream, scales));
    if (st != QT_OK) return qt::to_status(st);
    FftJob<float> inv[1] = {{Ch, (float*)C, m, s, ldc, s, 0, 1, hf}};
    return hip_status(qt::launch_tube_fft<float>(p, true, inv, 1, tw, stream));
}

}  // namespace

size_t qt_complex_workspace_size(int m, int n, int s, int p, qt_precision precision) {
    return cx_workspace(m, n, s, p, precision, false);
}

qt_status qt_tprod_complex(int m, int n, int s, int p, const void* A, const void* B, void* C, qt_precision precision,
                     void* ws, size_t ws_bytes, hipStream_t stream) {
    return qt::with_workspace(ws, ws_bytes, cx_workspace(m, n, s, p, precision, false), stream,
                              [&](void* w, size_t wb) { return run_cx(m, n, s, p, A, B, C, precision, w, wb, false, stream); });
}

size_t qt_real_workspace_size(int m, int n, int s, int p, qt_precision precision) {
    return cx_workspace(m, n, s, p, precision, true);
}

qt_status qt_tprod_real(int m, int n, int s, int p, const void* A, const void* B, void* C, qt_precision precision,
                  void* ws, size_t ws_bytes, hipStream_t stream) {
    return qt::with_workspace(ws, ws_bytes, cx_workspace(m, n, s, p, precision, true), stream,
                              [&](void* w, size_t wb) { return run_cx(m, n, s, p, A, B, C, precision, w, wb, true, stream); });
}

size_t qt_backward_workspace_size(int m, int n, int s, int p, qt_precision precision) {
    if (!valid_precision(precision) || !dims_ok(m, n, p) || !dims_ok(n, s, p) || !dims_ok(m, s, p))
        return 0;
    return backward_layout(m, n, s, p, precision).total;
}

namespace {
int backward_ws(int m, int n, int s, int p, const void* A, const void* B, const void* G,
                void* dA, void* dB, qt_precision precision, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!valid_precision(precision)) return QT_ERR_INVALID_ARG;
    if (!dims_ok(m, n, p) || !dims_ok(n, s, p) || !dims_ok(m, s, p)) return QT_ERR_INVALID_ARG;
    if (!A || !B || !G || !ws) return QT_ERR_INVALID_ARG;
    if (!aligned16(A) || !aligned16(B) || !aligned16(G) || !aligned16(ws) ||
        (dA && !aligned16(dA)) || (dB && !aligned16(dB)))
        return QT_ERR_INVALID_ARG;
    const size_t need = qt_backward_workspace_size(m, n, s, p, precision);
    if (ws_bytes < need) return QT_ERR_INVALID_ARG;
    const size_t ab = tensor_bytes(m, n, p, precision), bb = tensor_bytes(n, s, p, precision);
    const size_t gb = tensor_bytes(m, s, p, precision);
    const void* ins[4] = {A, B, G, ws};
    const size_t insz[4] = {ab, bb, gb, need};
    for (int q = 0; q < 4; ++q) {
        if (dA && overlaps(dA, ab, ins[q], insz[q])) return QT_ERR_INVALID_ARG;
        if (dB && overlaps(dB, bb, ins[q], insz[q])) return QT_ERR_INVALID_ARG;
    }
    if (dA && dB && overlaps(dA, ab, dB, bb)) return QT_ERR_INVALID_ARG;
    if (!p_supported(p, precision)) return QT_ERR_UNSUPPORTED;
    if (!dA && !dB) return QT_OK;
    if (precision == QT_FP64)
        return run_backward<double>(m, n, s, p, (const double*)A, (const double*)B, (const double*)G,
                                    (double*)dA, (double*)dB, precision, (char*)ws, stream);
    return run_backward<float>(m, n, s, p, (const float*)A, (const float*)B, (const float*)G,
                               (float*)dA, (float*)dB, precision, (char*)ws, stream);
}
}  // namespace

qt_status qt_tprod_backward(int m, int n, int s, int p, const void* A, const void* B, const void* G,
                      void* dA, void* dB, qt_precision precision, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
    return qt::with_workspace(ws, ws_bytes, qt_backward_workspace_size(m, n, s, p, precision), stream,
                              [&](void* w, size_t wb) {
                                  return qt::to_status(backward_ws(m, n, s, p, A, B, G, dA, dB, precision, w, wb, stream));
                              });
}

}  // extern "C"
