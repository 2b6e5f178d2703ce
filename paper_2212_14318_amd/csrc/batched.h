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
    int pack;                  // 1: forward output as split-bf16 words (FftJob::pack)
    // 1 (forward, dst_ld > cols): the positions run over rows x dst_ld and
    // the padding columns of the destination rows are written as zeros, so
    // that every destination line is written whole (a partly written line
    // costs a read-modify-write beyond L2)
    int fill;
};

// 256 consecutive positions of one CD part of one job.
struct BatchFftItem {
    int job, part, e0, pad;
};

// One problem of the facewise phase and its tile shape (detail::TileCfg).
// Split fp16: scales[f] is the power-of-two scale of A^ at f and
// scales[p + f] that of the B^ pair {f, -f} (NULL otherwise).
struct BatchGemmProb {
    FacewiseArgs<float> a;
    const float* scales;
    int cfg, pad;
};

// Split fp16: one operand of one problem (A^ or B^, FP32 Fourier planes
// [4][p][rows][ld] written by the forward FFT), the largest magnitude of each
// of its faces, and the per-face scales its words are written with.
struct BatchFp16Job {
    float* X;
    float* facemax;            // [p]
    const float* scale;        // [p]
    int rows, cols, ld, p;
};

// One face of one such operand.
struct BatchFp16Item {
    int job, face;
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

// Split fp16, between the forward FFTs and the products: the largest
// magnitude of every face of every operand (one workgroup per item), the
// per-frequency scales of every problem (from its two jobs, 2 i and 2 i + 1),
// and the scaled fp16 words written over the operands in place.
hipError_t launch_batched_fp16_prep(const BatchFp16Job* jobs, const BatchFp16Item* items, int nitems,
                                    const BatchGemmProb* probs, int count, hipStream_t stream);

// Persistent coupled facewise products over a list of tiles that all have
// tile shape cfg (detail::TileCfg).  precision: 0 = FP32, 1 = split bf16,
// 2 = split fp16 (scales from each problem's BatchGemmProb).
hipError_t launch_batched_gemm(int precision, int cfg, const BatchGemmProb* probs,
                               const BatchGemmItem* items, int nitems, int grid, hipStream_t stream);

// Resident workgroups per CU of the persistent product kernel of a shape.
int batched_gemm_blocks_per_cu(int precision, int cfg);

}  // namespace qt
