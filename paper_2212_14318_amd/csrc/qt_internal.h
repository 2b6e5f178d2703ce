// Internal declarations shared by the HIP translation units of libqtprod.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qt {

// Row stride (in reals) of a Fourier-domain matrix: columns rounded up to a
// multiple of 4 so that every row starts 16-byte aligned for vector loads.
inline long fourier_ld(long cols) { return (cols + 3) & ~3L; }

// Plane stride of a tensor stored as [4][p][rows][ld].
inline size_t plane_elems(long p, long rows, long ld) { return (size_t)p * (size_t)rows * (size_t)ld; }

// One tube-FFT job: a quaternion tensor of rows x cols x p, read from `src`
// with row stride src_ld and written to `dst` with row stride dst_ld.  Both
// buffers are [4][p][rows][ld].  Planes (0,1) form the complex part X1,
// planes (2,3) the part X2 of the Cayley-Dickson form.
// pack = 1 (float forward transforms only): every output real x is stored as
// the 32-bit word hi | lo << 16 of its bf16 split, hi = rn(x), lo = rn(x - hi)
// -- the operand format of the split-bf16 facewise products.
template <typename T>
struct FftJob {
    const T* src;
    T* dst;
    int rows, cols, src_ld, dst_ld;
    int pack;
    int parts = 2;            // CD parts to transform: 2 (quaternion) or 1 (complex, planes 0 and 1)
    // Hermitian half spectrum (real tensors, parts = 1): forward reads one
    // real plane of p faces and writes faces 0..p/2 of two planes; inverse
    // reads those p/2 + 1 faces (the rest are conj(X^[p - f])) and writes
    // the real plane of p faces.
    int half = 0;
    // fill = 1 (forward, dst_ld > cols, a library workspace as destination):
    // the register-resident kernels also write the padding columns of the
    // destination rows, as zero tubes, so that no line is written in part
    int fill = 0;
};

// Bluestein tables of one p (lengths without a register-resident kernel):
// M = smallest power of two >= 2p - 1; chirp c_k = exp(i pi (k^2 mod 2p) / p)
// (k < p); hat_fwd / hat_inv = length-M DFTs of the chirp sequence and of its
// conjugate; twm = exp(-2 pi i j / M), j < M/2.  All made in FP64 on the
// device, stored in both precisions.  M = 0 when p does not need them.
// The spectra are kept in two orders: hat_* in the order that the LDS
// kernel's decimation-in-frequency passes leave the frequencies in, hatn_* in
// natural order (register-resident kernels); twf = exp(-2 pi i j / M), j < M.
struct BluesteinTables {
    int M;
    double2 *chirp64, *hat_fwd64, *hat_inv64, *twm64, *hatn_fwd64, *hatn_inv64, *twf64;
    float2 *chirp32, *hat_fwd32, *hat_inv32, *twm32, *hatn_fwd32, *hatn_inv32, *twf32;
};

// Twiddle tables of one p: tw[k] = exp(-2 pi i k / p), k in [0, p), made in
// FP64 on the device and stored in both precisions, plus the Bluestein tables
// when some precision has no register-resident kernel for p.
struct Twiddles {
    float2* f32;
    double2* f64;
    BluesteinTables blue;
};

int bluestein_length(int p);
// Bytes of the Bluestein tables of p in one buffer (0 when every precision
// has a register-resident kernel for p), and the carving of such a buffer
// into the tables of `bt` (M set from p).
size_t bluestein_tables_bytes(int p);
void carve_bluestein_tables(int p, char* mem, BluesteinTables* bt);
hipError_t launch_bluestein_tables(int p, const BluesteinTables& bt, hipStream_t stream);
template <typename T>
hipError_t launch_bluestein(int p, bool inverse, const FftJob<T>* jobs, int njobs,
                            const BluesteinTables& bt, hipStream_t stream);
// The register-resident variant (one tube per thread) for convolution lengths
// M <= 64 (FP32) / 32 (FP64); hipErrorNotSupported for longer ones.
template <typename T>
hipError_t launch_bluestein_reg(int p, bool inverse, const FftJob<T>* jobs, int njobs,
                                const BluesteinTables& bt, hipStream_t stream);

// Forward (inverse = false) or inverse (inverse = true, with the 1/p scale)
// tube FFT of up to two jobs in one launch.  Returns hipSuccess or the launch
// error; hipErrorNotSupported if p has no kernel in this build.
template <typename T>
hipError_t launch_tube_fft(int p, bool inverse, const FftJob<T>* jobs, int njobs,
                           const Twiddles& tw, hipStream_t stream);

// True if launch_tube_fft has a kernel for this p and element type.
template <typename T>
bool tube_fft_supported(int p);

// Generate the twiddle table of p on `stream` (FP64 sincos on the device).
hipError_t launch_twiddles(int p, Twiddles tw, hipStream_t stream);

// Operands of the coupled facewise products for one problem, all in the
// Fourier domain, [4][p][rows][ld] layout:
//   A^: m x n (row stride lda), B^: n x s (ldb), C^: m x s (ldc).
template <typename T>
struct FacewiseArgs {
    const T* Ah;
    const T* Bh;
    T* Ch;
    int m, n, s, p;
    int lda, ldb, ldc;
};

// Products with at most this many columns (s) run the narrow FP32 VALU kernel
// in every float precision (they are bound by reading A^, not by MFMA).
constexpr int kNarrowMaxS = 4;

// C^[f] = A^[f] B^[f] coupled with -f (see qtprod.h) for every f.
// precision: 0 = FP32 MFMA, 1 = split bf16, 2 = split fp16 (float only; needs
// `scales`: 2p power-of-two scales, [f] for A^ and [p + f] for B^).
// tile_cfg: detail::TileCfg (0 = 128x64, 1 = 64x128, 2 = 64x64).
hipError_t launch_facewise_f32(const FacewiseArgs<float>& a, int precision, hipStream_t stream,
                               int tile_cfg = 0, const float* scales = nullptr);
hipError_t launch_facewise_f64(const FacewiseArgs<double>& a, hipStream_t stream);
// Complex products C^[f] = A^[f] B^[f] (planes 0, 1 of each tensor; no -f
// coupling).  precision: 0 = FP32 MFMA, 1 = split bf16 (operand words),
// 2 = split fp16 (operand words scaled by scales[f] for A^, scales[p + f]
// for B^).
hipError_t launch_facewise_cx(const FacewiseArgs<float>& a, int precision, hipStream_t stream,
                              const float* scales = nullptr);

// fp16 split: per-frequency power-of-two scales of A^ and of the B^ pairs
// {f, -f} into scales[0 .. 2p); partials needs p * (fp16_partial_blocks(m, n) +
// fp16_partial_blocks(n, s)) floats.  Complex operands (planes = 2, no -f
// coupling): the scale of B^ is per frequency, not per pair.
int fp16_partial_blocks(long rows, long cols);
hipError_t launch_fp16_scales(const FacewiseArgs<float>& a, float* partials, float* scales,
                              hipStream_t stream, int planes = 4);

// Tensor conjugate transpose job: src is rows x cols x p ([4][p][rows][cols]),
// dst is cols x rows x p.  planes_faces is filled in by the launcher.
template <typename T>
struct ConjTJob {
    const T* src;
    T* dst;
    int rows, cols, p;
    int planes_faces;
};

// dst = src^H for one or two jobs in one launch.
template <typename T>
hipError_t launch_conj_transpose(const ConjTJob<T>* jobs, int njobs, hipStream_t stream);

// Twiddle table of p on the current device from the plan cache (created on
// first use on `stream`, which is then synchronised once).  Returns a qt_status.
int get_twiddles(int p, hipStream_t stream, Twiddles* out);
// The cached plan of p on the current device, if there is one (no allocation).
bool find_twiddles(int p, Twiddles* out);

// qt_tprod's checks of everything but the workspace (a qt_status), and its
// three steps on a workspace of qt_workspace_size() bytes with the plan
// `given` (nullptr: the plan cache).
int check_tprod(int m, int n, int s, int p, const void* A, const void* B, const void* C,
                int precision);
int dispatch_tprod(int m, int n, int s, int p, const void* A, const void* B, void* C,
                   int precision, char* ws, hipStream_t stream, const Twiddles* given);

// In-place FP32 -> split-bf16 words of `faces` faces of rows x cols (row
// stride ld, a multiple of 4).
hipError_t launch_split_words(float* X, long faces, long rows, long cols, long ld, hipStream_t stream);
// In place: the Fourier-domain tensor [planes][p][rows][ld] (cols valid
// columns; 4 planes, or 2 for complex tensors) becomes fp16 words
// hi | lo << 16 of x * scale[f] (the split-fp16 operands).
hipError_t launch_fp16_words(float* X, long p, long rows, long cols, long ld, const float* scale,
                             hipStream_t stream, int planes = 4);

// Tile shape (detail::TileCfg) for one facewise product: from the autotuner's
// cost model when it has run on this device for this precision, else the
// shape with the least padded area (ties go to 128x64).
int choose_tile(int m, int n, int s, int precision);

}  // namespace qt
