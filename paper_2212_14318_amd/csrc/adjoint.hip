// Tensor conjugate transpose X^H of a quaternion tensor (gfx950).
//
// X^H is the tensor whose block circulant matrix is bcirc(X)^*: face 0 of
// X^H is (face 0 of X)^*, face k >= 1 is (face p - k of X)^*, where ^* is the
// quaternion conjugate transpose (conjugate every entry, Section 2.2, and
// transpose).  The adjoints of the T-product are dL/dA = G * B^H and
// dL/dB = A^H * G (bcirc(A * B) = bcirc(A) bcirc(B), proof of Theorem 5.1).
//
// Kernel: 32 x 32 tiles staged through LDS so that both the read (along the
// columns of X) and the write (along the columns of X^H) are coalesced; the
// conjugate flips the sign of planes 1..3 (b, c, d).
#include "qt_internal.h"

namespace qt {
namespace {

template <typename T>
__global__ void __launch_bounds__(256)
conj_transpose_kernel(ConjTJob<T> j0, ConjTJob<T> j1, int njobs) {
    __shared__ T tile[32][33];
    // grid z enumerates (plane, output face) of job 0, then of job 1
    const bool second = blockIdx.z >= (unsigned)j0.planes_faces;
    if (second && njobs < 2) return;
    const ConjTJob<T> jb = second ? j1 : j0;
    const int pf = second ? (int)blockIdx.z - j0.planes_faces : (int)blockIdx.z;
    const int c = pf / jb.p;              // component plane
    const int k = pf - c * jb.p;          // output face
    const int ksrc = k == 0 ? 0 : jb.p - k;
    const int tiles_c = (jb.cols + 31) / 32;
    const int tr = blockIdx.x / tiles_c, tc = blockIdx.x - tr * tiles_c;
    if (tr * 32 >= jb.rows) return;
    const size_t face = (size_t)jb.rows * jb.cols;
    const T* src = jb.src + ((size_t)c * jb.p + ksrc) * face;
    T* dst = jb.dst + ((size_t)c * jb.p + k) * face;    // dst is cols x rows
    const T sign = c == 0 ? T(1) : T(-1);
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int i = tr * 32 + ty + r, jj = tc * 32 + tx;
        if (i < jb.rows && jj < jb.cols) tile[ty + r][tx] = src[(size_t)i * jb.cols + jj];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        const int jj = tc * 32 + ty + r, i = tr * 32 + tx;     // dst row jj, column i
        if (jj < jb.cols && i < jb.rows) dst[(size_t)jj * jb.rows + i] = sign * tile[tx][ty + r];
    }
}

}  // namespace

template <typename T>
hipError_t launch_conj_transpose(const ConjTJob<T>* jobs, int njobs, hipStream_t stream) {
    if (njobs < 1 || njobs > 2) return hipErrorInvalidValue;
    ConjTJob<T> j0 = jobs[0];
    ConjTJob<T> j1 = njobs == 2 ? jobs[1] : jobs[0];
    j0.planes_faces = 4 * j0.p;
    j1.planes_faces = njobs == 2 ? 4 * j1.p : 0;
    long tiles = 0;
    for (int q = 0; q < njobs; ++q) {
        const long t = (long)((jobs[q].rows + 31) / 32) * ((jobs[q].cols + 31) / 32);
        tiles = t > tiles ? t : tiles;
    }
    const dim3 grid((unsigned)tiles, 1, (unsigned)(j0.planes_faces + j1.planes_faces));
    hipLaunchKernelGGL((conj_transpose_kernel<T>), grid, dim3(256), 0, stream, j0, j1, njobs);
    return hipGetLastError();
}

template hipError_t launch_conj_transpose<float>(const ConjTJob<float>*, int, hipStream_t);
template hipError_t launch_conj_transpose<double>(const ConjTJob<double>*, int, hipStream_t);

}  // namespace qt
