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
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "batched.h"
#include "facewise_impl.h"
#include "../../include/qtprod.h"

namespace qt {

hipError_t launch_batched_fft_fwd(int, int, const BatchFftJob*, const BatchFftItem*, int, hipStream_t);
hipError_t launch_batched_fft_inv(int, int, const BatchFftJob*, const BatchFftItem*, int, hipStream_t);

namespace {

using namespace detail;

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kSmem = cmax(sizeof(V2Smem<128, 64>), sizeof(V2Smem<64, 64>));
constexpr size_t kF32Smem = kSmem, kSplitSmem = kSmem;

template <int PREC, int MT, int NT>
__device__ __forceinline__ void run_tile(const FacewiseArgs<float>& a, int f, int tm, int tn, char* smem) {
    tile_v2<PREC, MT, NT>(a, f, tm * MT, tn * NT, 1.f, 1.f, *reinterpret_cast<V2Smem<MT, NT>*>(smem));
}

template <int PREC>
__global__ void __launch_bounds__(256)
batched_gemm_kernel(const BatchGemmProb* __restrict__ probs, const BatchGemmItem* __restrict__ items,
                    int nitems) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BatchGemmItem item = items[it];
        const BatchGemmProb pr = probs[item.prob];
        switch (pr.cfg) {
            // (the batched kernel carries two tile shapes; more raise its
            // register pressure into scratch spills)
            case TILE_128x64: run_tile<PREC, 128, 64>(pr.a, item.f, item.tm, item.tn, smem); break;
            default: run_tile<PREC, 64, 64>(pr.a, item.f, item.tm, item.tn, smem); break;
        }
    }
}

}  // namespace

hipError_t launch_batched_fft(bool inverse, int p, int pol, const BatchFftJob* jobs,
                              const BatchFftItem* items, int nitems, hipStream_t stream) {
    if (nitems <= 0) return hipSuccess;
    return inverse ? launch_batched_fft_inv(p, pol, jobs, items, nitems, stream)
                   : launch_batched_fft_fwd(p, pol, jobs, items, nitems, stream);
}

size_t batched_gemm_smem_bytes(int precision) { return precision == 0 ? kF32Smem : kSplitSmem; }

int batched_gemm_blocks_per_cu(int precision) {
    int n = 0;
    const hipError_t e = precision == 0
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batched_gemm_kernel<0>, 256, kF32Smem)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batched_gemm_kernel<1>, 256, kSplitSmem);
    return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_batched_gemm(int precision, const BatchGemmProb* probs, const BatchGemmItem* items,
                               int nitems, int grid, hipStream_t stream) {
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [] {
        hipError_t e0 = hipFuncSetAttribute((const void*)batched_gemm_kernel<0>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kF32Smem);
        hipError_t e1 = hipFuncSetAttribute((const void*)batched_gemm_kernel<1>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSplitSmem);
        attr_err = e0 != hipSuccess ? e0 : e1;
    });
    if (attr_err != hipSuccess) return attr_err;
    if (nitems <= 0) return hipSuccess;   // (a zero-item call only sets the attributes)
    if (precision == 0)
        hipLaunchKernelGGL(batched_gemm_kernel<0>, dim3(grid), dim3(256), kF32Smem, stream, probs, items, nitems);
    else if (precision == 1)
        hipLaunchKernelGGL(batched_gemm_kernel<1>, dim3(grid), dim3(256), kSplitSmem, stream, probs, items, nitems);
    else
        return hipErrorNotSupported;
    return hipGetLastError();
}

}  // namespace qt
