/*
 * qtprod.h -- C-ABI of libqtprod.so: the fast T-product of third-order
 * quaternion tensors on AMD Instinct MI355X (gfx950).
 *
 * Method (Zheng & Ni, "Block diagonalization of block circulant quaternion
 * matrices and the fast calculation for T-product of quaternion tensors"):
 * the T-product C = A * B := fold(bcirc(A) . unfold(B)) (Section 2.4,
 * Definition of the T-product) of A (m x n x p) and B (n x s x p) is computed
 * in three device steps, all hand-written HIP kernels:
 *   1. a tube FFT along the third mode of the Cayley-Dickson parts A1, A2,
 *      B1, B2 (Theorem 4.4: the block diagonalisation of bcirc is a DFT of the
 *      tubes);
 *   2. facewise complex products in the Fourier domain, where frequency f is
 *      coupled with frequency -f mod p because j c = conj(c) j
 *      (Theorem 5.1, Remark 5.1):
 *        C1^[f] = A1^[f] B1^[f] - A2^[f] conj(B2^[-f])
 *        C2^[f] = A1^[f] B2^[f] + A2^[f] conj(B1^[-f])
 *   3. the inverse tube FFT (Remark 4.3 (iv), Remark 5.1).
 * Steps 1-3 are Algorithm 5.1 written with a plain forward DFT
 * (omega = exp(-2 pi i / p), unnormalised) and 1/p in the inverse; the
 * paper's conj-FFT convention gives the same C.
 *
 * ---------------------------------------------------------------- layout --
 * A quaternion tensor X of size rows x cols x p is ONE device buffer of
 * 4 * p * rows * cols reals, planar, C order [4][p][rows][cols]:
 *   plane 0 = a, plane 1 = b, plane 2 = c, plane 3 = d of a + b i + c j + d k,
 * which in Cayley-Dickson form X = X1 + X2 j (Section 2.2) is
 *   plane 0 = Re X1, plane 1 = Im X1, plane 2 = Re X2, plane 3 = Im X2.
 * Face k (0-based; face k + 1 of the paper) of plane c starts at element
 * (c * p + k) * rows * cols.  Reals are float (QT_FP32, QT_SPLIT_BF16) or
 * double (QT_FP64).
 *
 * ------------------------------------------------------------ ownership --
 * The caller owns every input, output and workspace buffer; the library never
 * frees them.  The library owns only its plan cache: one small twiddle table
 * per (device, p), generated in FP64 on the GPU on first use (that first call
 * allocates it with hipMalloc and synchronises the stream once), kept until
 * the library is unloaded.  Call qt_prepare(p) before capturing a HIP graph.
 *
 * ------------------------------------------------------------ semantics --
 * Every compute call is asynchronous on `stream` (NULL = the null stream)
 * and never synchronises with the host except the one-time plan creation.
 * Argument errors are detected on the host before any launch and returned
 * synchronously; a HIP launch error is returned as QT_ERR_HIP.  Faults inside
 * kernels surface at the caller's next synchronisation.
 *
 * Preconditions checked (QT_ERR_INVALID_ARG otherwise): m, n, s, p >= 1;
 * every pointer non-NULL and 16-byte aligned; outputs do not overlap inputs;
 * ws_bytes >= the matching *_workspace_size(); 4 * p * rows * cols < 2^40.
 *
 * Workspace.  The one-shot products (qt_tprod, qt_tprod_complex,
 * qt_tprod_real, qt_tprod_backward, qt_tprod_batched) also accept ws == NULL
 * with ws_bytes == 0: the call then takes its workspace from the
 * stream-ordered allocator (hipMallocAsync on `stream`) and returns it
 * (hipFreeAsync on `stream`) after its kernels, with no host synchronisation;
 * an allocation failure returns QT_ERR_ALLOC.  Callers that capture graphs or
 * must not allocate pass their own buffer.  ws == NULL with ws_bytes != 0 is
 * QT_ERR_INVALID_ARG.  Plans (qt_batched_plan_create) always need a caller
 * buffer.
 */
#ifndef QTPROD_H
#define QTPROD_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QT_OK = 0,
    QT_ERR_INVALID_ARG = -1,  /* bad size, pointer, alignment, aliasing, workspace */
    QT_ERR_UNSUPPORTED = -2,  /* valid request this build cannot serve (e.g. p too large) */
    QT_ERR_ALLOC = -3,        /* device allocation failed (plan cache, or a workspace requested with ws == NULL) */
    QT_ERR_HIP = -4,          /* a HIP runtime call or kernel launch failed */
    QT_ERR_TOO_LARGE = -5,    /* the problem does not fit the fixed scratch of qt_tprod_noalloc */
    QT_STATUS_INT_RANGE = 0x7fffffff  /* not a status: gives the enum the full int range, so
                                         that any int a caller passes is a valid value */
} qt_status;

typedef enum {
    QT_FP32 = 0,        /* FP32 FFTs; facewise products on FP32 MFMA, FP32 accumulate */
    QT_SPLIT_BF16 = 1,  /* FP32 FFTs; facewise products as bf16 hi+lo split:
                           x = hi + lo, product ~ hi*hi + hi*lo + lo*hi on bf16 MFMA,
                           FP32 accumulate */
    QT_SPLIT_FP16 = 2,  /* as QT_SPLIT_BF16 with fp16 hi+lo; operands scaled by a
                           power of two per frequency (A^[f]) and per frequency
                           pair (B^[f], B^[-f]) computed on the device.  Served
                           by qt_tprod, qt_tprod_noalloc, qt_tprod_backward,
                           the batched calls, qt_tprod_complex and
                           qt_tprod_real (each product computes the scales of
                           its own operands); qt_fourier_tprod (its operands
                           are the caller's) returns QT_ERR_UNSUPPORTED */
    QT_FP64 = 3,        /* every step in double (small problems, validation) */
    QT_PRECISION_INT_RANGE = 0x7fffffff  /* not a precision: full int range (checked values
                                            outside 0..3 are rejected, not undefined) */
} qt_precision;

/* Largest p served (QT_ERR_UNSUPPORTED above it).  Every p in [1, QT_MAX_P]
 * is supported by the single-problem entry points: 7-smooth p (prime factors
 * 2, 3, 5, 7) up to 128 (64 for QT_FP64) have register-resident tube FFTs,
 * every other p goes through Bluestein's algorithm (chirp tables in FP64 on
 * the device), whose length-M convolution (M the power of two >= 2p - 1) is
 * held in one workgroup's LDS.  The batched path serves every p as well: its
 * own batched tube-FFT launches cover 7-smooth p <= 64, and problems of any
 * other length get tube-FFT launches of their own inside the same call or
 * plan (their products still share the persistent product launches). */
#define QT_MAX_P 4096

/* Library ABI version (major * 100 + minor). */
int qt_version(void);

/* Human-readable name of a status code (static string, never NULL). */
const char* qt_status_string(qt_status status);

/* Create the plan (twiddle table, and Bluestein chirp spectrum when p needs
 * one) for p on the current device, on `stream`, and wait for it.  Optional:
 * compute calls do this lazily.  Returns QT_OK, QT_ERR_INVALID_ARG,
 * QT_ERR_UNSUPPORTED, QT_ERR_ALLOC or QT_ERR_HIP. */
qt_status qt_prepare(int p, hipStream_t stream);

/* Row stride (in reals) that qt_tprod uses for its Fourier-domain tensors:
 * cols rounded up to a multiple of 4.  Any ld >= cols that is a multiple of 4
 * is accepted by qt_fourier_tprod. */
int qt_fourier_ld(int cols);

/* Tube FFT of one quaternion tensor X (rows x cols x p) -- the block
 * diagonalisation of bcirc(X) of Theorem 4.4, in the plain-DFT convention:
 *   inverse = 0:  Xh[c][f] = sum_k X[c][k] w^(f k), w = exp(-2 pi i / p), applied
 *                 to the complex parts X1 = (plane 0, plane 1) and
 *                 X2 = (plane 2, plane 3) separately;
 *   inverse = 1:  the inverse transform, with the factor 1/p.
 * X is read as [4][p][rows][ldx] and Xh written as [4][p][rows][ldh]
 * (ldx, ldh >= cols; entries beyond cols are neither read nor written);
 * Xh planes are (Re X1^, Im X1^, Re X2^, Im X2^).  The paper's transform of
 * Theorem 4.4 is fft(conj X) = conj(X1^[-f]) - X2^[f] j in these terms.
 * X and Xh must not overlap.  precision: QT_FP32 (float) or QT_FP64 (double).
 * QT_SPLIT_BF16 with inverse = 0 writes the operand format of the split-bf16
 * facewise products instead of floats: every real x becomes the 32-bit word
 * hi | lo << 16 with hi = rn_bf16(x), lo = rn_bf16(x - hi) (same layout and
 * size); QT_SPLIT_FP16, and any split precision with inverse = 1, transform
 * floats like QT_FP32. */
qt_status qt_tube_fft(int rows, int cols, int p, const void* X, int ldx, void* Xh, int ldh,
                int inverse, qt_precision precision, hipStream_t stream);

/* Step 2 alone, for Fourier-domain-resident chains: for every frequency f,
 *   C1^[f] = A1^[f] B1^[f] - A2^[f] conj(B2^[-f]),
 *   C2^[f] = A1^[f] B2^[f] + A2^[f] conj(B1^[-f])   (Theorem 5.1, Remark 5.1),
 * on tensors produced by qt_tube_fft with the same precision (QT_SPLIT_BF16:
 * split words): Ah [4][p][m][lda], Bh [4][p][n][ldb], Ch [4][p][m][ldc] (floats;
 * ldc >= s, entries beyond s untouched).  For the float precisions lda, ldb,
 * ldc must be multiples of 4 (16-byte rows).  qt_tube_fft(inverse = 1) of Ch
 * is then A * B.  No workspace.  QT_SPLIT_FP16 needs per-call scales and is
 * served by qt_tprod only (QT_ERR_UNSUPPORTED here). */
qt_status qt_fourier_tprod(int m, int n, int s, int p, const void* Ah, int lda, const void* Bh,
                     int ldb, void* Ch, int ldc, qt_precision precision, hipStream_t stream);

/* In place: turn a Fourier-domain FP32 tensor Xh [4][p][rows][ld] (e.g. the
 * C^ written by qt_fourier_tprod) into the QT_SPLIT_BF16 operand format, the
 * word hi | lo << 16 per real (hi = rn_bf16(x), lo = rn_bf16(x - hi)), which
 * is what qt_tube_fft writes for QT_SPLIT_BF16.  This keeps chains
 * A * B * C ... in the Fourier domain for the split-bf16 products: since
 * bcirc(A * B) = bcirc(A) bcirc(B) (proof of Theorem 5.1), the product of two
 * transformed tensors is the transform of A * B, ready to be multiplied
 * again.  Columns beyond cols are untouched.  ld >= cols, a multiple of 4;
 * Xh 16-byte aligned.  Returns QT_OK, QT_ERR_INVALID_ARG or QT_ERR_HIP. */
qt_status qt_split_words(int rows, int cols, int p, void* Xh, int ld, hipStream_t stream);

/* Workspace bytes needed by qt_tprod for these sizes and precision
 * (0 if an argument is invalid).  Holds the Fourier-domain tensors
 * A^, B^ and C^ (row strides rounded up to a multiple of 4 reals). */
size_t qt_workspace_size(int m, int n, int s, int p, qt_precision precision);

/* C = A * B.  A: m x n x p, B: n x s x p, C: m x s x p (layout above; all
 * device pointers).  ws: device workspace of ws_bytes >= qt_workspace_size().
 * C is fully overwritten.  Definition: Section 2.4; algorithm: Algorithm 5.1
 * with Theorem 5.1. */
qt_status qt_tprod(int m, int n, int s, int p,
             const void* A, const void* B, void* C,
             qt_precision precision, void* ws, size_t ws_bytes, hipStream_t stream);

/* One problem of a batch: sizes and device pointers, same layout as above. */
typedef struct {
    int m, n, s, p;
    const void* A;
    const void* B;
    void* C;
} qt_problem;

/* Workspace bytes for qt_tprod_batched over `count` problems (host array). */
size_t qt_batched_workspace_size(int count, const qt_problem* probs, qt_precision precision);

/* C_i = A_i * B_i for count independent problems of any sizes (Section 2.4
 * definition of each product), each by Algorithm 5.1 with the coupled
 * facewise products of Theorem 5.1 / Remark 5.1, in three
 * phases: the forward tube FFT of every A_i, B_i (one launch per distinct p,
 * one workgroup per 256 tubes); the coupled facewise products of every
 * frequency and output tile (one persistent launch per tile shape, walking a
 * cost-sorted work list); the inverse tube FFT of every C_i^ (one launch per
 * distinct p).  A small descriptor upload into ws comes first, from pageable
 * memory, so the call returns once it is staged.
 * probs is a HOST array read before the call returns.  Each problem obeys the
 * single-call preconditions; outputs must not overlap any input or output.
 * precision: QT_FP32, QT_SPLIT_BF16 or QT_SPLIT_FP16 (QT_FP64 returns
 * QT_ERR_UNSUPPORTED); any p <= QT_MAX_P (problems whose p is not 7-smooth or
 * exceeds 64 get tube-FFT launches of their own).  QT_SPLIT_FP16 adds three
 * launches between the phases: the largest magnitude of every face of every
 * A_i^, B_i^, each problem's power-of-two scales (A_i^ per frequency, B_i^ per
 * pair {f, -f}, as qt_tprod computes them), and the scaled fp16 words written
 * over the Fourier operands in the workspace.
 * The first call per device and precision runs the autotuner (allocates and
 * synchronises once).  Same arithmetic as qt_tprod per problem (tile shapes
 * may differ, hence rounding order).  For graph replays use the plan API. */
qt_status qt_tprod_batched(int count, const qt_problem* probs, qt_precision precision,
                     void* ws, size_t ws_bytes, hipStream_t stream);

/* Size of the device array that qt_tprod_noalloc uses as its workspace:
 * 256 MiB, held on every device the library runs on until the process ends. */
#define QT_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* qt_tprod without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments (minus the workspace), arithmetic, kernels and
 * results as qt_tprod: the workspace is a library-owned device array of
 * QT_NOALLOC_SCRATCH_BYTES per device instead of a caller buffer.  If the
 * plan of p was created before (qt_prepare, or any earlier call with this p
 * on this device), it is used; otherwise the twiddle (and Bluestein) tables
 * are generated into the array behind the workspace on this call (for a
 * Bluestein length that is an O(M^2) kernel: call qt_prepare first).
 * Returns QT_ERR_TOO_LARGE, before any launch, when qt_workspace_size() plus
 * those tables exceeds QT_NOALLOC_SCRATCH_BYTES; the other statuses as
 * qt_tprod.  Every call on one device shares that device's array, which keeps
 * the last call's contents: calls that overlap in time on one device (other
 * streams, other host threads) race and give wrong results; calls on one
 * stream are ordered and safe.  The first call on a device resolves the
 * array's device address (a host-side lookup, no allocation). */
qt_status qt_tprod_noalloc(int m, int n, int s, int p, const void* A, const void* B, void* C,
                     qt_precision precision, hipStream_t stream);

/* Batched plan: the work lists of one batch, built once, with all launches of
 * the three phases captured into one hipGraph.  The plan refers to the
 * problems' buffers and to `ws`, which must stay allocated (and untouched by
 * other work while a replay runs) until qt_batched_plan_destroy. */
typedef struct qt_batched_plan_s* qt_batched_plan;

/* Build a plan for count problems (host array, read during the call): run the
 * autotuner if it has not run for this device and precision, create missing
 * twiddle tables, upload the work lists into ws, synchronise `stream`, and
 * capture + instantiate the graph.  Not capture-safe itself.  precision:
 * QT_FP32 or QT_SPLIT_BF16; any p <= QT_MAX_P (else
 * QT_ERR_UNSUPPORTED). */
qt_status qt_batched_plan_create(int count, const qt_problem* probs, qt_precision precision, void* ws,
                           size_t ws_bytes, hipStream_t stream, qt_batched_plan* plan);

/* Replay the plan on `stream` (one hipGraphLaunch): recomputes every C_i from
 * the current contents of A_i and B_i. */
qt_status qt_batched_plan_launch(qt_batched_plan plan, hipStream_t stream);

/* Release the plan's graph (the caller's buffers are untouched). */
qt_status qt_batched_plan_destroy(qt_batched_plan plan);

/* Run (or load from the file named by the environment variable
 * QT_TUNE_CACHE) the autotuner for `precision` on the current device: it times
 * every facewise tile shape on a calibration problem to fit the per-tile cost
 * model t = alpha + beta * ceil(n / 16), and times both radix orders of the
 * batched tube FFT for every batched p.  Allocates scratch memory and
 * synchronises `stream`.  Single-problem calls then use the cost model for
 * their tile shape too.  precision: QT_FP32, QT_SPLIT_BF16 or QT_SPLIT_FP16
 * (the split-fp16 tiles share the split-bf16 cost model: same instruction
 * mix at the same rate); QT_FP64 returns QT_ERR_UNSUPPORTED. */
qt_status qt_autotune(qt_precision precision, hipStream_t stream);

/* Workspace bytes needed by qt_tprod_complex (0 if an argument is invalid or
 * the precision is QT_FP64). */
size_t qt_complex_workspace_size(int m, int n, int s, int p, qt_precision precision);

/* T-product of complex tensors, the special case A2 = B2 = 0 of the
 * quaternion product (Algorithm 2.1 and Proposition 2.1 of the paper, the
 * complex case that the quaternion method extends): C^[f] = A^[f] B^[f] for
 * every frequency, with no coupling to -f, i.e. one complex product per face
 * instead of four coupled ones, and one complex tube FFT per tensor.  Layout:
 * TWO planes per tensor, [2][p][rows][cols] = (Re, Im); A: m x n x p,
 * B: n x s x p, C: m x s x p (device pointers, C fully overwritten).
 * precision: QT_FP32 (FP32 MFMA), QT_SPLIT_BF16 (bf16 hi+lo products, as
 * for qt_tprod) or QT_SPLIT_FP16 (fp16 hi+lo with a power-of-two scale per
 * frequency for A^[f] and for B^[f], there being no -f coupling); QT_FP64
 * returns QT_ERR_UNSUPPORTED.  A real tensor is a complex one with a zero
 * imaginary plane.  Same preconditions, ownership and error behaviour as
 * qt_tprod. */
qt_status qt_tprod_complex(int m, int n, int s, int p, const void* A, const void* B, void* C,
                     qt_precision precision, void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes needed by qt_tprod_real (0 if an argument is invalid or the
 * precision is QT_FP64). */
size_t qt_real_workspace_size(int m, int n, int s, int p, qt_precision precision);

/* T-product of real tensors (Algorithm 2.1 of the paper on real input, the
 * T-product of Kilmer and Martin).  The DFT of a real tube is Hermitian,
 * X^[p - f] = conj(X^[f]), so only frequencies f = 0 .. p/2 are transformed,
 * multiplied (one complex product C^[f] = A^[f] B^[f] each) and inverted:
 * p/2 + 1 complex products instead of p.  Layout: ONE plane per tensor,
 * [p][rows][cols] row-major faces; A: m x n x p, B: n x s x p, C: m x s x p
 * (device pointers, C fully overwritten).  precision: QT_FP32, QT_SPLIT_BF16
 * or QT_SPLIT_FP16 (as for qt_tprod_complex, on the p/2 + 1 faces); QT_FP64
 * returns QT_ERR_UNSUPPORTED.  Same preconditions, ownership and error
 * behaviour as qt_tprod. */
qt_status qt_tprod_real(int m, int n, int s, int p, const void* A, const void* B, void* C,
                  qt_precision precision, void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes needed by qt_tprod_backward. */
size_t qt_backward_workspace_size(int m, int n, int s, int p, qt_precision precision);

/* Adjoints of C = A * B for an output gradient G (m x s x p):
 *   dA = G * B^H   (m x n x p),   dB = A^H * G   (n x s x p),
 * where X^H is the tensor conjugate transpose (face 0 -> (X_0)^*, face k ->
 * (X_{p-k})^*; bcirc(X^H) = bcirc(X)^*).  For L = 1/2 ||A * B - T||_F^2 and
 * G = A * B - T these are dL/dA and dL/dB of the real components.  Either of
 * dA, dB may be NULL to skip it.  Computed in the Fourier domain with the
 * same frequency coupling as the forward product (bcirc(A * B) =
 * bcirc(A) bcirc(B), proof of Theorem 5.1).  All four precisions; with
 * QT_SPLIT_FP16 each of the two products scales its own operands (G is
 * transformed twice when both adjoints are asked for). */
qt_status qt_tprod_backward(int m, int n, int s, int p,
                      const void* A, const void* B, const void* G,
                      void* dA, void* dB,
                      qt_precision precision, void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes needed by qt_tsvd (0 if an argument is invalid, a size is
 * beyond the limits below, or the precision is not QT_FP32 / QT_FP64). */
size_t qt_tsvd_workspace_size(int m, int n, int p, qt_precision precision);

/* Quaternion t-SVD A = U * S * V^H of A (m x n x p): U (m x m x p) and
 * V (n x n x p) unitary tensors (U^H * U = U * U^H = identity), S (m x n x p)
 * f-diagonal (every face diagonal; its entries have no j part).  The paper
 * names T-product factorisations as the use of its block diagonalisation
 * (Section 6); this one follows from Theorem 5.1 / Remark 5.1: the matrices
 *   chi_f(X) = [[X1^[f], X2^[f]], [-conj X2^[-f], conj X1^[-f]]]
 * (X1^, X2^ the tube DFTs of the complex parts) satisfy chi_f(A * B) =
 * chi_f(A) chi_f(B) and chi_f(X^H) = chi_f(X)^*, and chi_-f follows from
 * chi_f, so one SVD per frequency pair {f, -f} (f = 0 .. p/2) gives the
 * factors.  For f != -f the singular values of chi_f(A) in descending order
 * are placed alternately on f and -f (value 2i on entry i of S1^[f], value
 * 2i + 1 on entry i of S1^[-f]); for f = -f (f = 0, p/2) chi_f(A) is the
 * complex adjoint of a quaternion matrix and the factors keep that structure.
 * Truncating S to its first r diagonal tubes then keeps the 2r largest
 * singular values of every chi_f.  The singular values of bcirc(A) are the
 * p * min(m, n) values of sigma.
 * Layout: A, U, S, V as in the T-product ([4][p][rows][cols]); sigma (may be
 * NULL): p x min(m, n) reals, sigma[f][i] = entry (i, i) of S1^[f], the tube
 * DFT of S's diagonal.  U, S and V may each be NULL (not written).  All device
 * pointers; outputs must not overlap A, each other or the workspace.
 * precision: QT_FP32 or QT_FP64 (one-sided Jacobi in that precision; split
 * precisions return QT_ERR_UNSUPPORTED).  Limits: min(m, n) <= 512,
 * max(m, n) <= 1024, p <= QT_MAX_P (QT_ERR_UNSUPPORTED beyond).  U and V are
 * not unique (phases, bases of repeated singular values and of null spaces);
 * S is.  One workgroup per frequency pair; workspace as qt_tprod (ws == NULL
 * allocates on the stream). */
qt_status qt_tsvd(int m, int n, int p, const void* A, void* U, void* S, void* V, void* sigma,
                  qt_precision precision, void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of qt_fourier_tsvd (0 if invalid or beyond the limits). */
size_t qt_fourier_tsvd_workspace_size(int m, int n, int p, qt_precision precision);

/* The middle step of qt_tsvd alone, for tensors kept in the Fourier domain:
 * from Ah = the tube FFT of A ([4][p][m][lda], as written by qt_tube_fft in
 * QT_FP32 / QT_FP64) it writes Uh = the tube FFT of U ([4][p][m][ldu]),
 * Vh = that of V ([4][p][n][ldv]) and sigma (p x min(m, n)); S^ is the
 * f-diagonal tensor with S1^[f](i, i) = sigma[f][i] and no other non-zero
 * entry.  Columns beyond m (Uh) and n (Vh) are not written.  ws: device
 * scratch of at least qt_fourier_tsvd_workspace_size() bytes (required, no
 * NULL form).  Same precisions, limits and error behaviour as qt_tsvd; no
 * buffer may overlap another. */
qt_status qt_fourier_tsvd(int m, int n, int p, const void* Ah, int lda, void* Uh, int ldu, void* Vh, int ldv,
                          void* sigma, qt_precision precision, void* ws, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* QTPROD_H */
