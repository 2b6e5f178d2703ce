// Batched T-products: the persistent product kernel and the dispatch of the
// batched tube FFT.
//
// A batch of independent problems C_i = A_i * B_i (any m, n, s, p per
// problem) runs in three phases: forward tube FFT of every A_i and B_i (one
// launch per distinct tube length), coupled facewise products of every
// (problem, frequency, tile) in one persistent launch whose fixed grid strides
// a heterogeneous work list sorted by estimated cost (longest first), and the
// inverse tube FFT of every C_i^.  The phases are ordered by the launch
// boundaries, so no workgroup ever waits on another.  A plan captures all
// launches into one hipGraph, so a replay is a single hipGraphLaunch.
#include "batched.h"
#include "facewise_impl.h"
#include "fft_impl.h"
#include "../../include/qtprod.h"

namespace qt {

hipError_t launch_batched_fft_fwd(int, int, const BatchFftJob*, const BatchFftItem*, int, hipStream_t);
hipError_t launch_batched_fft_inv(int, int, const BatchFftJob*, const BatchFftItem*, int, hipStream_t);

namespace {

using namespace detail;

// Persistent product kernel of one tile shape: the grid strides its own
// item list (all items of the launch have tile shape CFG).  Workgroups are
// dispatched to the 8 XCDs in turn (workgroup w on XCD w % 8), so in each
// stride the workgroups of one XCD take a run of consecutive items: the tiles
// of one (problem, frequency), adjacent in the list, then share that XCD's L2
// for their A rows and B columns instead of each fetching them from beyond it.
constexpr int kXcds = 8;

template <int PREC, int CFG>
__global__ void __launch_bounds__(64 * tile_waves(PREC, CFG))
batched_gemm_kernel(const BatchGemmProb* __restrict__ probs, const BatchGemmItem* __restrict__ items,
                    int nitems) {
    constexpr int MT = tile_mt(CFG), NT = tile_nt(CFG);
    __shared__ __attribute__((aligned(16))) V2Smem<MT, NT> sm;
    const int grid = gridDim.x;
    const int slot = grid % kXcds == 0 ? (blockIdx.x % kXcds) * (grid / kXcds) + blockIdx.x / kXcds
                                       : blockIdx.x;
    for (int it = slot; it < nitems; it += grid) {
        const BatchGemmItem item = items[it];
        const BatchGemmProb pr = probs[item.prob];
        float sa = 1.f, sb = 1.f;
        if constexpr (PREC == 2) {
            sa = pr.scales[item.f];
            sb = pr.scales[pr.a.p + item.f];
        }
        tile_v2<PREC, MT, NT, tile_waves(PREC, CFG), plane_groups(PREC, CFG)>(pr.a, item.f, item.tm * MT,
                                                                         item.tn * NT, sa, sb, sm);
    }
}

// ------------------------------------------------------- split fp16 prep
// Largest magnitude over the four planes of one face of one operand.
__global__ void __launch_bounds__(256)
batched_facemax_kernel(const BatchFp16Job* __restrict__ jobs, const BatchFp16Item* __restrict__ items) {
    __shared__ float red[256];
    const BatchFp16Item it = items[blockIdx.x];
    const BatchFp16Job j = jobs[it.job];
    const size_t face = (size_t)j.rows * j.ld, plane = (size_t)j.p * face;
    const float* Xf = j.X + (size_t)it.face * face;
    const long count = (long)j.rows * j.cols;
    float mx = 0.f;
    for (long e = threadIdx.x; e < count; e += 256) {
        const int r = (int)(e / j.cols), c = (int)(e - (long)r * j.cols);
        const size_t off = (size_t)r * j.ld + c;
#pragma unroll
        for (int q = 0; q < 4; ++q) mx = fmaxf(mx, fabsf(Xf[q * plane + off]));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) j.facemax[it.face] = red[0];
}

// Scales of problem i from its operands' face maxima (jobs 2 i: A^, 2 i + 1:
// B^): A^ at f alone, B^ over the pair {f, -f} that the product stages together.
__global__ void __launch_bounds__(256)
batched_fp16_scales_kernel(const BatchGemmProb* __restrict__ probs, const BatchFp16Job* __restrict__ jobs,
                           int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int p = probs[i].a.p;
    float* scales = const_cast<float*>(probs[i].scales);
    const float* ma = jobs[2 * i].facemax;
    const float* mb = jobs[2 * i + 1].facemax;
    for (int f = 0; f < p; ++f) {
        const int g = (p - f) % p;
        scales[f] = pow2_scale(ma[f]);
        scales[p + f] = pow2_scale(fmaxf(mb[f], mb[g]));
    }
}

// Scaled fp16 words over one face of one operand, in place.
__global__ void __launch_bounds__(256)
batched_fp16_words_kernel(const BatchFp16Job* __restrict__ jobs, const BatchFp16Item* __restrict__ items) {
    const BatchFp16Item it = items[blockIdx.x];
    const BatchFp16Job j = jobs[it.job];
    const size_t face = (size_t)j.rows * j.ld, plane = (size_t)j.p * face;
    float* Xf = j.X + (size_t)it.face * face;
    const float sc = j.scale[it.face];
    const long count = (long)j.rows * j.cols;
    for (long e = threadIdx.x; e < count; e += 256) {
        const int r = (int)(e / j.cols), c = (int)(e - (long)r * j.cols);
        const size_t off = (size_t)r * j.ld + c;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float* x = Xf + q * plane + off;
            *reinterpret_cast<unsigned*>(x) = split_fp16_word(*x, sc);
        }
    }
}

template <int PREC, int CFG>
const void* gemm_fn() { return reinterpret_cast<const void*>(&batched_gemm_kernel<PREC, CFG>); }

const void* gemm_kernel(int precision, int cfg) {
    if (precision < 0 || precision > 2) return nullptr;
    switch (3 * cfg + precision) {
#define QT_GEMM_FN(CFG)                                      \
    case 3 * CFG: return gemm_fn<0, CFG>();                  \
    case 3 * CFG + 1: return gemm_fn<1, CFG>();              \
    case 3 * CFG + 2: return gemm_fn<2, CFG>();
        QT_GEMM_FN(TILE_128x64)
        QT_GEMM_FN(TILE_64x128)
        QT_GEMM_FN(TILE_64x64)
        QT_GEMM_FN(TILE_32x64)
#undef QT_GEMM_FN
        default: return nullptr;
    }
}

}  // namespace

hipError_t launch_batched_fft(bool inverse, int p, int pol, const BatchFftJob* jobs,
                              const BatchFftItem* items, int nitems, hipStream_t stream) {
    if (nitems <= 0) return hipSuccess;
    return inverse ? launch_batched_fft_inv(p, pol, jobs, items, nitems, stream)
                   : launch_batched_fft_fwd(p, pol, jobs, items, nitems, stream);
}

int batched_gemm_blocks_per_cu(int precision, int cfg) {
    const void* fn = gemm_kernel(precision, cfg);
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 64 * tile_waves(precision, cfg), 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

hipError_t launch_batched_fp16_prep(const BatchFp16Job* jobs, const BatchFp16Item* items, int nitems,
                                    const BatchGemmProb* probs, int count, hipStream_t stream) {
    if (nitems <= 0 || count <= 0) return hipSuccess;
    hipLaunchKernelGGL(batched_facemax_kernel, dim3((unsigned)nitems), dim3(256), 0, stream, jobs, items);
    hipLaunchKernelGGL(batched_fp16_scales_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                       probs, jobs, count);
    hipLaunchKernelGGL(batched_fp16_words_kernel, dim3((unsigned)nitems), dim3(256), 0, stream, jobs, items);
    return hipGetLastError();
}

hipError_t launch_batched_gemm(int precision, int cfg, const BatchGemmProb* probs,
                               const BatchGemmItem* items, int nitems, int grid, hipStream_t stream) {
    if (nitems <= 0) return hipSuccess;
    if (precision < 0 || precision > 2) return hipErrorNotSupported;
    const dim3 g((unsigned)grid), b(64 * tile_waves(precision, cfg));
#define QT_GEMM_LAUNCH(PREC, CFG) \
    hipLaunchKernelGGL((batched_gemm_kernel<PREC, CFG>), g, b, 0, stream, probs, items, nitems)
#define QT_GEMM_CASES(CFG)                                   \
    case 3 * CFG: QT_GEMM_LAUNCH(0, CFG); break;             \
    case 3 * CFG + 1: QT_GEMM_LAUNCH(1, CFG); break;         \
    case 3 * CFG + 2: QT_GEMM_LAUNCH(2, CFG); break;
    switch (3 * cfg + precision) {
        QT_GEMM_CASES(TILE_128x64)
        QT_GEMM_CASES(TILE_64x128)
        QT_GEMM_CASES(TILE_64x64)
        QT_GEMM_CASES(TILE_32x64)
        default: return hipErrorInvalidValue;
    }
#undef QT_GEMM_CASES
#undef QT_GEMM_LAUNCH
    return hipGetLastError();
}

}  // namespace qt
