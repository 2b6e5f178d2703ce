// Descriptors and launchers of the batched (many problems, one launch per
// phase) T-product.
#pragma once
#include "qt_internal.h"

namespace qt {

// One tube-FFT job of the batch (one quaternion tensor), FP32.
struct BatchFftJob {
    const float* src;
    float* dst;
    const float2* tw;          // twiddle table of p
    int rows, cols, src_ld, dst_ld;
    int p, pol;                // length and radix-order policy (0 or 1)
    int pack, pad;             // 1: forward output as split-bf16 words (FftJob::pack)
};

// 256 consecutive positions of one CD part of one job.
struct BatchFftItem {
    int job, part, e0, pad;
};

// One problem of the facewise phase and its tile shape (detail::TileCfg).
struct BatchGemmProb {
    FacewiseArgs<float> a;
    int cfg, pad0, pad1, pad2;
};

// One output tile (tm, tn) at frequency f of problem prob.
struct BatchGemmItem {
    int prob, f, tm, tn;
};

// True if the persistent FFT kernel has a case for p (7-smooth, p <= 64).
bool batched_fft_supported(int p);

// Tube FFT of nitems items that all have tube length p and radix-order
// policy pol (one workgroup per item).  Descriptor arrays are device pointers.
hipError_t launch_batched_fft(bool inverse, int p, int pol, const BatchFftJob* jobs,
                              const BatchFftItem* items, int nitems, hipStream_t stream);

// Persistent coupled facewise products over a list of tiles that all have
// tile shape cfg (detail::TileCfg).  precision: 0 = FP32, 1 = split bf16.
hipError_t launch_batched_gemm(int precision, int cfg, const BatchGemmProb* probs,
                               const BatchGemmItem* items, int nitems, int grid, hipStream_t stream);

// Resident workgroups per CU of the persistent product kernel of a shape.
int batched_gemm_blocks_per_cu(int precision, int cfg);

}  // namespace qt
