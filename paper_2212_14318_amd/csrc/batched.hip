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
        tile_v2<PREC, MT, NT, tile_waves(PREC, CFG), plane_groups(PREC, CFG)>(pr.a, item.f, item.tm * MT,
                                                                         item.tn * NT, 1.f, 1.f, sm);
    }
}

template <int PREC, int CFG>
const void* gemm_fn() { return reinterpret_cast<const void*>(&batched_gemm_kernel<PREC, CFG>); }

const void* gemm_kernel(int precision, int cfg) {
    switch (2 * cfg + (precision == 0 ? 0 : 1)) {
        case 2 * TILE_128x64: return gemm_fn<0, TILE_128x64>();
        case 2 * TILE_128x64 + 1: return gemm_fn<1, TILE_128x64>();
        case 2 * TILE_64x128: return gemm_fn<0, TILE_64x128>();
        case 2 * TILE_64x128 + 1: return gemm_fn<1, TILE_64x128>();
        case 2 * TILE_64x64: return gemm_fn<0, TILE_64x64>();
        case 2 * TILE_64x64 + 1: return gemm_fn<1, TILE_64x64>();
        case 2 * TILE_32x64: return gemm_fn<0, TILE_32x64>();
        case 2 * TILE_32x64 + 1: return gemm_fn<1, TILE_32x64>();
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
    const void* fn = (precision == 0 || precision == 1) ? gemm_kernel(precision, cfg) : nullptr;
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 64 * tile_waves(precision, cfg), 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

hipError_t launch_batched_gemm(int precision, int cfg, const BatchGemmProb* probs,
                               const BatchGemmItem* items, int nitems, int grid, hipStream_t stream) {
    if (nitems <= 0) return hipSuccess;
    if (precision != 0 && precision != 1) return hipErrorNotSupported;
    const dim3 g((unsigned)grid), b(64 * tile_waves(precision, cfg));
#define QT_GEMM_LAUNCH(PREC, CFG) \
    hipLaunchKernelGGL((batched_gemm_kernel<PREC, CFG>), g, b, 0, stream, probs, items, nitems)
    switch (2 * cfg + precision) {
        case 2 * TILE_128x64: QT_GEMM_LAUNCH(0, TILE_128x64); break;
        case 2 * TILE_128x64 + 1: QT_GEMM_LAUNCH(1, TILE_128x64); break;
        case 2 * TILE_64x128: QT_GEMM_LAUNCH(0, TILE_64x128); break;
        case 2 * TILE_64x128 + 1: QT_GEMM_LAUNCH(1, TILE_64x128); break;
        case 2 * TILE_64x64: QT_GEMM_LAUNCH(0, TILE_64x64); break;
        case 2 * TILE_64x64 + 1: QT_GEMM_LAUNCH(1, TILE_64x64); break;
        case 2 * TILE_32x64: QT_GEMM_LAUNCH(0, TILE_32x64); break;
        case 2 * TILE_32x64 + 1: QT_GEMM_LAUNCH(1, TILE_32x64); break;
        default: return hipErrorInvalidValue;
    }
#undef QT_GEMM_LAUNCH
    return hipGetLastError();
}

}  // namespace qt
