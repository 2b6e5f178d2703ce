// Tile routines of the coupled facewise products in the Fourier domain
// (gfx950), shared by the single-problem kernels (facewise.hip) and the
// persistent batched kernel (batched.hip).
//
// Theorem 5.1 / Remark 5.1: after the tube FFT every frequency f is an
// independent complex product, except that j c = conj(c) j pairs f with
// g = -f mod p.  Written for the plain DFT:
//   C1^[f] = A1^[f] B1^[f] - A2^[f] conj(B2^[g])
//   C2^[f] = A1^[f] B2^[f] + A2^[f] conj(B1^[g])
// In real planes (r = real, i = imaginary part) each output plane is a sum of
// four real m x n by n x s products:
//   Re C1 = Ar1 Br1f - Ai1 Bi1f - Ar2 Br2g - Ai2 Bi2g
//   Im C1 = Ar1 Bi1f + Ai1 Br1f + Ar2 Bi2g - Ai2 Br2g
//   Re C2 = Ar1 Br2f - Ai1 Bi2f + Ar2 Br1g + Ai2 Bi1g
//   Im C2 = Ar1 Bi2f + Ai1 Br2f + Ai2 Br1g - Ar2 Bi1g
// i.e. 16 real products = 32 m n s flops per frequency (the count of the
// proof of Theorem 5.2, additions included).  A workgroup (NW waves in an
// (NW / 2) x 2 grid) owns an MT x NT tile of all four output planes and stages
// the four A planes and the eight B planes (f and g) of one 16-deep k-chunk in
// LDS, so each B value is read once per output tile rather than once per
// output plane.
#pragma once
#include <type_traits>

#include "qt_internal.h"


namespace qt {
namespace detail {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int KT = 16;     // k-chunk depth

// 32x32 f32 accumulator layout of v_mfma_f32_32x32x*: register r of lane l
// holds row 8 (r / 4) + 4 (l / 32) + (r % 4), column l % 32.
template <int MB, int NB, int C0 = 0, int NC = 4>
__device__ __forceinline__ void store_tile(const FacewiseArgs<float>& a, int f, int row0, int col0,
                                           const v16f (&acc)[4][MB][NB], float scale, float scale2,
                                           int lane) {
    const size_t pc = (size_t)a.p * a.m * a.ldc;
    float* Cf = a.Ch + (size_t)f * a.m * a.ldc;
    const int lr = lane & 31, lk = lane >> 5;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int col = col0 + nb * 32 + lr;
        if (col >= a.s) continue;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = row0 + mb * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
                if (row < a.m) {
#pragma unroll
                    for (int c = C0; c < C0 + NC; ++c)
                        Cf[c * pc + (size_t)row * a.ldc + col] = (acc[c][mb][nb][r] * scale) * scale2;
                }
            }
    }
}

// ------------------------------------------------------ split bf16 / fp16
// x = hi + lo with hi = rn(x), lo = rn(x - hi) in a 16-bit format; a real
// product X Y is taken as Xhi Yhi + Xhi Ylo + Xlo Yhi (the dropped Xlo Ylo is
// ~2^-16 relative for bf16), each on v_mfma_f32_32x32x16_{bf16,f16} with FP32
// accumulation.  The split operands take the same bytes in HBM as FP32 ones:
// every real is one word hi | lo << 16, unpacked into fragments with byte
// permutes.  For bf16 the forward tube FFT writes the words; for fp16 a pass
// after the per-frequency power-of-two scales writes them in place (the scale
// depends on the whole frequency), and the product undoes the scales.
//
// The coupled products are rewritten as two plain complex products,
//   C1^ = A1^ B1^[f] + A2^ D,  D = -conj(B2^[g]),
//   C2^ = A1^ B2^[f] + A2^ E,  E =  conj(B1^[g]),
// whose signs are applied to the B fragments, so that every real term adds:
// Re = Xr Yr + (-Xi) Yi, Im = Xr Yi + Xi Yr.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));

template <typename H> struct SplitTypes;
template <> struct SplitTypes<__bf16> { using v8 = v8bf; using v4 = v4bf; };
template <> struct SplitTypes<_Float16> { using v8 = v8h; using v4 = v4h; };

template <typename H>
__device__ __forceinline__ v16f mfma16(typename SplitTypes<H>::v8 a, typename SplitTypes<H>::v8 b, v16f c);
template <>
__device__ __forceinline__ v16f mfma16<__bf16>(v8bf a, v8bf b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ v16f mfma16<_Float16>(v8h a, v8h b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

template <typename V8>
__device__ __forceinline__ V8 neg8(V8 x) {
    // flip the sign bit of all eight 16-bit lanes (exact negation)
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    u4 b = __builtin_bit_cast(u4, x);
    b ^= 0x80008000u;
    return __builtin_bit_cast(V8, b);
}

// Power-of-two scale of a split-fp16 operand block whose largest magnitude
// is mx: mx * scale < 2^15 (the hi halves stay below the fp16 maximum with
// room for the products' sums).  The exponent is capped at 126 so that the
// scale and its reciprocal are normal floats (only inputs below 2^-111 hit
// the cap, and they then land below 2^15 instead of in [2^14, 2^15)).
__device__ __forceinline__ float pow2_scale(float mx) {
    if (!(mx > 0.f) || !isfinite(mx)) return 1.f;
    int e;
    (void)frexpf(mx, &e);                 // mx < 2^e, e in [-148, 128]
    const int k = 15 - e < 126 ? 15 - e : 126;
    return ldexpf(1.f, k);
}

// Tile shapes (MT x NT) compiled for both kernels; the id is what the
// autotuner stores and what a batched work item carries.
// 32x64 cuts the row padding of small problems (m <= 32, or m just above a
// multiple of 64); its FP32 form has two waves, its split forms four.
enum TileCfg { TILE_128x64 = 0, TILE_64x128 = 1, TILE_64x64 = 2, TILE_32x64 = 3, NUM_TILE_CFGS = 4 };
__host__ __device__ constexpr int tile_mt(int cfg) {
    return cfg == TILE_128x64 ? 128 : cfg == TILE_32x64 ? 32 : 64;
}
__host__ __device__ constexpr int tile_nt(int cfg) { return cfg == TILE_64x128 ? 128 : 64; }
// The split tiles (bf16 or fp16 words) split 8 waves into two plane groups
// (tile_v2's PG): each wave reads half the staged planes per chunk, which cuts
// LDS fragment reads and unpacking by a third.  Not the 64 x 128 split tile:
// with two waves per SIMD its 128 accumulator registers plus the group's
// fragments and DMA addresses exceed 256 VGPRs and spill, so it runs 4 waves
// of 512 registers each.
__host__ __device__ constexpr bool plane_groups(int mode, int cfg) { return mode != 0 && cfg != TILE_64x128; }
// Waves per workgroup of a tile shape and mode (0 FP32, 1 split bf16, 2 split
// fp16): 8 waves for the 128 x 64 tile (4 x 2, each 32 x 32) and for the
// plane-group split tiles (two groups of 2 x 2), so that two waves share a
// SIMD and hide each other's LDS and VALU latency; the other 64-wide tiles run
// 4 waves (2 x 2).  (A 64-wide tile stages 96 or 160 KB per workgroup, so one
// workgroup fills a CU's LDS.)
__host__ __device__ constexpr int tile_waves(int mode, int cfg) {
    return cfg == TILE_32x64 ? (plane_groups(mode, cfg) ? 4 : 2)
                             : (cfg == TILE_128x64 || plane_groups(mode, cfg)) ? 8 : 4;
}


// ======================================================== pipelined tile
// Tile routine shared by the FP32 and split paths:
//  * k-chunks of 16 go global -> LDS by DMA (global_load_lds_dwordx4: each
//    wave instruction moves 64 x 16 B into 1 KB of LDS, lane L at byte 16 L),
//    so no prefetch registers are live across the MFMA loop;
//  * two LDS buffers, one barrier per chunk: the DMA of chunk c + 1 goes out
//    in slices between the plane steps of chunk c (with plane groups, whole,
//    from group 1 before its fragment reads);
//  * B planes are consumed in pairs (q, q + 2) feeding C1 and C2, which gives
//    4 MB independent accumulator chains per split product;
//  * within a chunk, lane group g = lane / 32 owns logical k = 8 g .. 8 g + 7
//    of both operands (any assignment works as long as A and B agree), so an
//    A fragment is 8 contiguous floats (two 16-byte LDS reads) and a B
//    fragment is 8 floats of one column (eight 4-byte reads, conflict-free);
//  * the A chunk is stored row-major with its four 16-byte k-pieces XOR-
//    swizzled by row group (piece q of row i sits at slot 4 i + (q ^ (i/4 % 4))
//    of its 16-row block), which makes the 16-byte fragment reads conflict-free;
//  * rows/columns/k beyond the problem are read from clamped (valid)
//    addresses and zeroed before use; interior chunks skip the masks.
// MODE 0: FP32 operands on v_mfma_f32_32x32x2_f32 (8 k-steps per chunk);
// MODE 1: operands already split by the tube FFT into bf16 words hi | lo << 16
//         (FftJob::pack), unpacked with byte permutes, 3 products per term on
//         v_mfma_f32_32x32x16_bf16 (one k-step per chunk);
// MODE 2: the same with fp16 words of operands scaled by powers of two per
//         frequency (undone at the store), on v_mfma_f32_32x32x16_f16.
typedef __attribute__((address_space(3))) void lds_void_t;

// CX: complex products (two A planes, two B planes) instead of the coupled
// quaternion ones (four A planes, eight staged B planes).
template <int MT, int NT, bool CX = false>
struct V2Smem {
    float A[2][CX ? 2 : 4][MT / 16][256];      // [buffer][plane][16-row block][1 KB]
    float B[2][CX ? 2 : 8][NT / 16][256];      // [buffer][plane][block of 256/NT k-rows][1 KB]
};

__device__ __forceinline__ void dma16(const float* g, float* lds_block) {
    __builtin_amdgcn_global_load_lds((const void*)g, (lds_void_t*)lds_block, 16, 0, 0);
}

// Split operand words (hi | lo << 16, bf16 or fp16) -> the hi and lo
// fragments of 8 consecutive k (one v_perm_b32 per pair).
template <typename V8>
__device__ __forceinline__ void unpack8(const unsigned (&w)[8], V8& hi, V8& lo) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    u4 h, l;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        h[j] = __builtin_amdgcn_perm(w[2 * j + 1], w[2 * j], 0x05040100u);
        l[j] = __builtin_amdgcn_perm(w[2 * j + 1], w[2 * j], 0x07060302u);
    }
    hi = __builtin_bit_cast(V8, h);
    lo = __builtin_bit_cast(V8, l);
}

template <int MODE, int MT, int NT, int NW = 4, bool PG = false, bool CX = false>
__device__ __forceinline__ void tile_v2(const FacewiseArgs<float>& a, int f, int m0, int n0,
                                        float sa, float sb, V2Smem<MT, NT, CX>& sm) {
    using H = typename std::conditional<MODE == 2, _Float16, __bf16>::type;
    using V8 = typename SplitTypes<H>::v8;
    // NW waves as a (NW / 2) x 2 grid; each wave owns MB x NB 32 x 32 blocks.
    // PG (split bf16): two plane groups of NW / 2 waves, each a (NW / 4) x 2
    // grid over the whole tile; group 0 takes the B^[f] planes with A1, group
    // 1 the D, E planes with A2, and the partial sums meet once per tile.
    // CX: the complex product C^[f] = A^[f] B^[f] (A2 = B2 = 0: no coupling
    // with -f), two A planes, two B planes, output planes 0 and 1.
    static_assert(!PG || (MODE != 0 && !CX), "plane groups are built for the split quaternion paths");
    constexpr int NPA = CX ? 2 : 4, NPB = CX ? 2 : 8;
    constexpr int WG = PG ? NW / 2 : NW;
    constexpr int WM = WG / 2;
    constexpr int MB = MT / (32 * WM), NB = NT / 64;
    static_assert(MB >= 1 && MT == 32 * WM * MB && (NPA * (MT / 16)) % NW == 0 && (NPB * (NT / 16)) % NW == 0,
                  "tile shape does not fit the wave grid");
    constexpr int ABLK = MT / 16, BBLK = NT / 16;       // 1 KB blocks per plane
    constexpr int RB = 256 / NT, CQ = NT / 4;           // B block: RB k-rows of CQ 16-byte pieces
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform (SGPR)
    const int grp = PG ? wave / WG : 0;                  // plane group (wave-uniform)
    const int tw = PG ? wave % WG : wave;
    const int g = (a.p - f) % a.p;
    const size_t pa = (size_t)a.p * a.m * a.lda;
    const size_t pb = (size_t)a.p * a.n * a.ldb;
    const float* Af = a.Ah + (size_t)f * a.m * a.lda;
    const float* Bf = a.Bh + (size_t)f * a.n * a.ldb;
    const float* Bg = a.Bh + (size_t)g * a.n * a.ldb;
    const int nchunks = (a.n + KT - 1) / KT;
    const bool edge_tile = (m0 + MT > a.m) || (n0 + NT > a.s);

    // ---- staging of chunk c: DTOT copy slots of 1 KB per wave (64 lanes x
    // 16 B, lane L at byte 16 L of its LDS block); slot d < DA is an A block,
    // the rest B blocks.  Interior chunks ("fast") use a wave-uniform base plus
    // a per-lane offset fixed for the tile; other chunks clamp rows, columns
    // and k to valid addresses (the compute masks those entries).
    constexpr int DA = NPA * ABLK / NW, DB = NPB * BBLK / NW, DTOT = DA + DB;   // slots per wave per chunk
    const int a_i = lane >> 2;
    const int a_lane_off = a_i * a.lda + 4 * ((lane & 3) ^ ((a_i >> 2) & 3));
    const int b_lane_off = (lane / CQ) * a.ldb + 4 * (lane % CQ);
    // Block q (0 <= q < 4 * ABLK) of the A chunk or block q (0 <= q < 8 *
    // BBLK) of the B chunk.
    auto block_src = [&](int c, bool isA, int q, bool fast) -> const float* {
        const int k0 = c * KT;
        if (isA) {
            const int pl = q / ABLK, blk = q % ABLK;
            if (fast) return Af + pl * pa + (size_t)(m0 + blk * 16) * a.lda + k0 + a_lane_off;
            const int i = lane >> 2;
            const int kq = (lane & 3) ^ ((i >> 2) & 3);
            int grow = m0 + blk * 16 + i;
            grow = grow < a.m ? grow : a.m - 1;
            int gk = k0 + 4 * kq;
            gk = gk <= a.lda - 4 ? gk : a.lda - 4;
            return Af + pl * pa + (size_t)grow * a.lda + gk;
        }
        const int pl = q / BBLK, blk = q % BBLK;
        // staged planes: 0..3 = B^[f] (B1r, B1i, B2r, B2i); 4..7 = D, E from
        // B^[g]: Dr = -B2r, Di = B2i, Er = B1r, Ei = -B1i (signs applied later)
        const int src = pl < 4 ? pl : (pl == 4 ? 2 : pl == 5 ? 3 : pl == 6 ? 0 : 1);
        const float* base = (pl < 4 ? Bf : Bg) + src * pb;
        if (fast) return base + (size_t)(k0 + blk * RB) * a.ldb + n0 + b_lane_off;
        int gk = k0 + blk * RB + lane / CQ;
        gk = gk < a.n ? gk : a.n - 1;
        int gc = n0 + 4 * (lane % CQ);
        gc = gc <= a.ldb - 4 ? gc : a.ldb - 4;
        return base + (size_t)gk * a.ldb + gc;
    };
    auto block_dst = [&](int b, bool isA, int q) -> float* {
        return isA ? &sm.A[b][q / ABLK][q % ABLK][0] : &sm.B[b][q / BBLK][q % BBLK][0];
    };
    // slot d of this wave (d is a compile-time constant at every call)
    auto slot_src = [&](int c, int d, bool fast) -> const float* {
        return d < DA ? block_src(c, true, NW * d + wave, fast) : block_src(c, false, NW * (d - DA) + wave, fast);
    };
    auto slot_dst = [&](int b, int d) -> float* {
        return d < DA ? block_dst(b, true, NW * d + wave) : block_dst(b, false, NW * (d - DA) + wave);
    };
    // whole interior chunk c issued by the NW / 2 waves of plane group 1 alone
    auto issue_fast_g1 = [&](int c) {
        constexpr int NG = NW / 2;
#pragma unroll
        for (int d = 0; d < NPA * ABLK / NG; ++d)
            dma16(block_src(c, true, NG * d + tw, true), block_dst(c & 1, true, NG * d + tw));
#pragma unroll
        for (int d = 0; d < NPB * BBLK / NG; ++d)
            dma16(block_src(c, false, NG * d + tw, true), block_dst(c & 1, false, NG * d + tw));
        __builtin_amdgcn_sched_barrier(0);
    };

    // DMA of chunk c into buffer b
    auto issue = [&](int c, int b) {
#pragma unroll
        for (int d = 0; d < DTOT; ++d) dma16(slot_src(c, d, false), slot_dst(b, d));
    };
    auto issue_fast_one = [&](int c, int b, int d) { dma16(slot_src(c, d, true), slot_dst(b, d)); };
    auto issue_fast = [&](int c, int b) {
#pragma unroll
        for (int d = 0; d < DTOT; ++d) issue_fast_one(c, b, d);
    };
    // the share of plane step q (of 8) of the DMA of interior chunk c
    auto issue_slice = [&](int c, int q) {
#pragma unroll
        for (int d = q * DTOT / 8; d < (q + 1) * DTOT / 8; ++d) issue_fast_one(c, c & 1, d);
        // keep the slice here: the scheduler would otherwise sink the DMA to
        // the end of the chunk, where its latency is no longer hidden
        __builtin_amdgcn_sched_barrier(0);
    };
    auto chunk_inside = [&](int c) { return !edge_tile && (c * KT + KT <= a.n); };

    const int wm = tw % WM, wn = tw / WM;
    const int lr = lane & 31, lg = lane >> 5;

    // FP32 tiles form each complex product with three real products (KARA):
    // P1 = Re A Re Y, P2 = Im A Im Y, P3 = (Re A + Im A)(Re Y + Im Y),
    // accumulated per output (C1, C2; C alone for CX) over its coupled terms,
    // and Re C = P1 - P2, Im C = P3 - P1 - P2 at the end: 12 real products per
    // quaternion output pair and k instead of 16 (3 instead of 4 for CX).
    constexpr bool KARA = MODE == 0;
    constexpr int NOUT = CX ? 1 : 2;                  // complex outputs per tile
    constexpr int NACC = KARA ? 3 * NOUT : 4;
    v16f acc[NACC][MB][NB];
#pragma unroll
    for (int c = 0; c < NACC; ++c)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[c][mb][nb][r] = 0.f;

    // ---- fragments of chunk c from buffer b; MASK zeroes out-of-range entries
    auto load_a = [&](int b, int mb, int c, bool mask, float (&x)[4][8]) {
        const int rl = wm * (MT / WM) + mb * 32 + lr;
        const int blk = rl >> 4, i = rl & 15;
        const int s0 = 4 * i + ((2 * lg) ^ ((i >> 2) & 3));
        const int s1 = 4 * i + ((2 * lg + 1) ^ ((i >> 2) & 3));
        const bool row_ok = !mask || (m0 + rl < a.m);
#pragma unroll
        for (int pl = 0; pl < NPA; ++pl) {
            const float4 u = *reinterpret_cast<const float4*>(&sm.A[b][pl][blk][4 * s0]);
            const float4 w = *reinterpret_cast<const float4*>(&sm.A[b][pl][blk][4 * s1]);
            const float v[8] = {u.x, u.y, u.z, u.w, w.x, w.y, w.z, w.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bool ok = row_ok && (!mask || (c * KT + 8 * lg + j < a.n));
                x[pl][j] = ok ? v[j] : 0.f;
            }
        }
    };

    // MODE 1 A fragments: raw split words, zeroed where masked
    auto load_a_words = [&](int b, int mb, int c, bool mask, unsigned (&w)[4][8]) {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        const int rl = wm * (MT / WM) + mb * 32 + lr;
        const int blk = rl >> 4, i = rl & 15;
        const int s0 = 4 * i + ((2 * lg) ^ ((i >> 2) & 3));
        const int s1 = 4 * i + ((2 * lg + 1) ^ ((i >> 2) & 3));
        const bool row_ok = !mask || (m0 + rl < a.m);
#pragma unroll
        for (int pl = 0; pl < NPA; ++pl) {
            const u4 u = *reinterpret_cast<const u4*>(&sm.A[b][pl][blk][4 * s0]);
            const u4 v = *reinterpret_cast<const u4*>(&sm.A[b][pl][blk][4 * s1]);
            const unsigned x[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bool ok = row_ok && (!mask || (c * KT + 8 * lg + j < a.n));
                w[pl][j] = ok ? x[j] : 0u;
            }
        }
    };

    // One chunk, B plane by B plane: the A fragments of the chunk stay live,
    // each B plane is loaded, (split,) negated where a term needs -Im A, and
    // used at once by the two terms that contain it, on both M blocks:
    //   plane 0 B1r: ReC1 += Ar1 B1r   ImC1 += Ai1 B1r
    //   plane 1 B1i: ReC1 -= Ai1 B1i   ImC1 += Ar1 B1i
    //   plane 2 B2r: ReC2 += Ar1 B2r   ImC2 += Ai1 B2r
    //   plane 3 B2i: ReC2 -= Ai1 B2i   ImC2 += Ar1 B2i
    //   plane 4 Dr : ReC1 += Ar2 Dr    ImC1 += Ai2 Dr
    //   plane 5 Di : ReC1 -= Ai2 Di    ImC1 += Ar2 Di
    //   plane 6 Er : ReC2 += Ar2 Er    ImC2 += Ai2 Er
    //   plane 7 Ei : ReC2 -= Ai2 Ei    ImC2 += Ar2 Ei
    // i.e. plane q feeds accumulators (q & 2 ? C2 : C1), real part from
    // A-plane (q & 1 ? Im : Re) and imaginary part from the other one.
    // inter: the DMA of interior chunk c + 1 is issued in slices between the
    // plane steps (mask and inter are literals at every call)
    auto compute = [&](int c, int b, bool mask, bool inter) {
        // A fragments of the chunk, read and formed once for all NB column blocks
        float xa[MODE == 0 ? MB : 1][4][8];
        V8 ah[MB][4], al[MB][4];
        if constexpr (MODE == 0) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) load_a(b, mb, c, mask, xa[mb]);
        } else {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                unsigned wa[4][8];
                load_a_words(b, mb, c, mask, wa);
#pragma unroll
                for (int pl = 0; pl < NPA; ++pl) unpack8(wa[pl], ah[mb][pl], al[mb][pl]);
            }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int cl = wn * (NT / 2) + nb * 32 + lr;
            const bool col_ok = !mask || (n0 + cl < a.s);
            // the DMA slices of chunk c + 1 go out once, with the first column block
            const bool dma = inter && nb == 0;
            if constexpr (MODE == 0) {
                // A sums Re + Im of A1 and A2 (exact inputs, one FP32 rounding)
                float xs[MB][NPA / 2][8];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int h = 0; h < NPA / 2; ++h)
#pragma unroll
                        for (int t = 0; t < 8; ++t) xs[mb][h][t] = xa[mb][2 * h][t] + xa[mb][2 * h + 1][t];
                // staged B planes in (real, imaginary) pairs: (B1r, B1i) and (B2r, B2i)
                // with A1, (Dr, Di) and (Er, Ei) with A2; the first and third
                // feed C1, the second and fourth C2 (CX: the one pair (Br, Bi))
                constexpr int NPP = NPB / 2;
#pragma unroll
                for (int pp = 0; pp < NPP; ++pp) {
                    if (dma) {
#pragma unroll
                        for (int sl = pp * 8 / NPP; sl < (pp + 1) * 8 / NPP; ++sl) issue_slice(c + 1, sl);
                    }
                    float yr[8], yi[8], ys[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int k = 8 * lg + j;
                        const bool ok = col_ok && (!mask || (c * KT + k < a.n));
                        const float vr = sm.B[b][2 * pp][k / RB][(k % RB) * NT + cl];
                        const float vi = sm.B[b][2 * pp + 1][k / RB][(k % RB) * NT + cl];
                        // D = (-B2r, B2i), E = (B1r, -B1i) at -f
                        yr[j] = ok ? (pp == 2 ? -vr : vr) : 0.f;
                        yi[j] = ok ? (pp == 3 ? -vi : vi) : 0.f;
                        ys[j] = yr[j] + yi[j];
                    }
                    const int ca = (pp & 1) ? 3 : 0;          // P1, P2, P3 of C1 or C2
                    const int apl = (pp & 2) ? 2 : 0;         // A1 or A2
#pragma unroll
                    for (int t = 0; t < 8; ++t)
#pragma unroll
                        for (int mb = 0; mb < MB; ++mb) {
                            acc[ca][mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[mb][apl][t], yr[t], acc[ca][mb][nb], 0, 0, 0);
                            acc[ca + 1][mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[mb][apl + 1][t], yi[t], acc[ca + 1][mb][nb], 0, 0, 0);
                            acc[ca + 2][mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[mb][apl / 2][t], ys[t], acc[ca + 2][mb][nb], 0, 0, 0);
                        }
                }
            } else {
                // all B words of the chunk are read up front, so that their LDS
                // latency overlaps the products of the earlier planes
                unsigned wb[8][8];
#pragma unroll
                for (int q = 0; q < NPB; ++q)
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int k = 8 * lg + j;
                        wb[q][j] = __builtin_bit_cast(unsigned, sm.B[b][q][k / RB][(k % RB) * NT + cl]);
                    }
                // B fragment (hi, lo) of staged plane q, D/E signs applied
                auto bfrag = [&](int q, V8& yh, V8& yl) {
                    const unsigned flip = (q == 4 || q == 7) ? 0x80008000u : 0u;
                    unsigned w[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const bool ok = col_ok && (!mask || (c * KT + 8 * lg + j < a.n));
                        w[j] = ok ? (wb[q][j] ^ flip) : 0u;
                    }
                    unpack8(w, yh, yl);
                };
                if constexpr (CX) {
                    // complex: plane 0 (Re B) and plane 1 (Im B) of C1 alone
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        if (dma) {
#pragma unroll
                            for (int sl = 4 * q; sl < 4 * q + 4; ++sl) issue_slice(c + 1, sl);
                        }
                        V8 yh, yl, nyh, nyl;
                        bfrag(q, yh, yl);
                        if (q == 1) {
                            nyh = neg8(yh);
                            nyl = neg8(yl);
                        }
#pragma unroll
                        for (int step = 0; step < 3; ++step)
#pragma unroll
                            for (int mb = 0; mb < MB; ++mb) {
                                const V8 xr = step == 0 ? al[mb][0] : ah[mb][0];
                                const V8 xi = step == 0 ? al[mb][1] : ah[mb][1];
                                const V8 y = step == 1 ? yl : yh;
                                if (q == 0) {          // Re += Ar Br, Im += Ai Br
                                    acc[0][mb][nb] = mfma16<H>(xr, y, acc[0][mb][nb]);
                                    acc[1][mb][nb] = mfma16<H>(xi, y, acc[1][mb][nb]);
                                } else {               // Re -= Ai Bi, Im += Ar Bi
                                    const V8 ny = step == 1 ? nyl : nyh;
                                    acc[0][mb][nb] = mfma16<H>(xi, ny, acc[0][mb][nb]);
                                    acc[1][mb][nb] = mfma16<H>(xr, y, acc[1][mb][nb]);
                                }
                            }
                    }
                } else {
                // Planes are taken in pairs (q, q + 2) = (0, 2), (1, 3), (4, 6),
                // (5, 7): the first feeds C1, the second C2, so each of the three
                // split products runs over 4 MB independent accumulator chains.
#pragma unroll
                for (int qp = 0; qp < 4; ++qp) {
                    const int qa = (qp & 1) | ((qp & 2) << 1), qb = qa + 2;
                    if (dma) {
                        issue_slice(c + 1, 2 * qp);
                        issue_slice(c + 1, 2 * qp + 1);
                    }
                    V8 yh[2], yl[2], nyh[2], nyl[2];
                    bfrag(qa, yh[0], yl[0]);
                    bfrag(qb, yh[1], yl[1]);
                    const bool odd = (qa & 1) != 0;          // imaginary B part: Re -= Ai Y, Im += Ar Y
                    const int apl = (qa & 4) ? 2 : 0;        // A1 or A2
                    if (odd) {
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            nyh[t] = neg8(yh[t]);
                            nyl[t] = neg8(yl[t]);
                        }
                    }
                    // lo x hi, hi x lo, then hi x hi (small terms first)
#pragma unroll
                    for (int step = 0; step < 3; ++step)
#pragma unroll
                        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                            for (int t = 0; t < 2; ++t) {
                                const int cre = 2 * t;
                                const V8 xr = step == 0 ? al[mb][apl] : ah[mb][apl];
                                const V8 xi = step == 0 ? al[mb][apl + 1] : ah[mb][apl + 1];
                                const V8 y = step == 1 ? yl[t] : yh[t];
                                if (!odd) {
                                    acc[cre][mb][nb] = mfma16<H>(xr, y, acc[cre][mb][nb]);
                                    acc[cre + 1][mb][nb] = mfma16<H>(xi, y, acc[cre + 1][mb][nb]);
                                } else {
                                    const V8 ny = step == 1 ? nyl[t] : nyh[t];
                                    acc[cre][mb][nb] = mfma16<H>(xi, ny, acc[cre][mb][nb]);
                                    acc[cre + 1][mb][nb] = mfma16<H>(xr, y, acc[cre + 1][mb][nb]);
                                }
                            }
                }
                }   // !CX
            }
        }
    };

    // PG: chunk c for plane group G, i.e. staged B planes 4 G .. 4 G + 3 and
    // A planes 2 G, 2 G + 1; pairs (q, q + 2) feed C1 and C2 as in compute.
    auto compute_pg = [&](auto G, int c, int b, bool mask, bool inter) {
        constexpr int g0 = decltype(G)::value;
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        // The DMA of chunk c + 1 is issued by group 1 alone, before its
        // fragment reads: group 0's reads then meet an idle LDS and its
        // products start sooner after the barrier (group 0 also wins the
        // MFMA arbitration, so the pipe fills from the start of the chunk).
        if constexpr (g0 == 1) {
            if (inter) issue_fast_g1(c + 1);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int cl = wn * (NT / 2) + nb * 32 + lr;
            const bool col_ok = !mask || (n0 + cl < a.s);
            V8 ah[MB][2], al[MB][2];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int rl = wm * (MT / WM) + mb * 32 + lr;
                const int blk = rl >> 4, i = rl & 15;
                const int s0 = 4 * i + ((2 * lg) ^ ((i >> 2) & 3));
                const int s1 = 4 * i + ((2 * lg + 1) ^ ((i >> 2) & 3));
                const bool row_ok = !mask || (m0 + rl < a.m);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int pl = 2 * g0 + t;
                    const u4 u = *reinterpret_cast<const u4*>(&sm.A[b][pl][blk][4 * s0]);
                    const u4 v = *reinterpret_cast<const u4*>(&sm.A[b][pl][blk][4 * s1]);
                    const unsigned x[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
                    unsigned w[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const bool ok = row_ok && (!mask || (c * KT + 8 * lg + j < a.n));
                        w[j] = ok ? x[j] : 0u;
                    }
                    unpack8(w, ah[mb][t], al[mb][t]);
                }
            }
            unsigned wb[4][8];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = 8 * lg + j;
                    wb[q][j] = __builtin_bit_cast(unsigned, sm.B[b][4 * g0 + q][k / RB][(k % RB) * NT + cl]);
                }
            auto bfrag = [&](int q, V8& yh, V8& yl) {
                const unsigned flip = (q == 4 || q == 7) ? 0x80008000u : 0u;
                unsigned w[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bool ok = col_ok && (!mask || (c * KT + 8 * lg + j < a.n));
                    w[j] = ok ? (wb[q - 4 * g0][j] ^ flip) : 0u;
                }
                unpack8(w, yh, yl);
            };
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int qa = 4 * g0 + k, qb = qa + 2;
                V8 yh[2], yl[2], nyh[2], nyl[2];
                bfrag(qa, yh[0], yl[0]);
                bfrag(qb, yh[1], yl[1]);
                const bool odd = k == 1;                 // imaginary B part: Re -= Ai Y, Im += Ar Y
                if (odd) {
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        nyh[t] = neg8(yh[t]);
                        nyl[t] = neg8(yl[t]);
                    }
                }
#pragma unroll
                for (int step = 0; step < 3; ++step)
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            const int cre = 2 * t;
                            const V8 xr = step == 0 ? al[mb][0] : ah[mb][0];
                            const V8 xi = step == 0 ? al[mb][1] : ah[mb][1];
                            const V8 y = step == 1 ? yl[t] : yh[t];
                            if (!odd) {
                                acc[cre][mb][nb] = mfma16<H>(xr, y, acc[cre][mb][nb]);
                                acc[cre + 1][mb][nb] = mfma16<H>(xi, y, acc[cre + 1][mb][nb]);
                            } else {
                                const V8 ny = step == 1 ? nyl[t] : nyh[t];
                                acc[cre][mb][nb] = mfma16<H>(xi, ny, acc[cre][mb][nb]);
                                acc[cre + 1][mb][nb] = mfma16<H>(xr, y, acc[cre + 1][mb][nb]);
                            }
                        }
            }
        }
    };

    auto sync = [&]() {
        __builtin_amdgcn_s_waitcnt(0);       // this wave's DMA of the chunk has landed
        __syncthreads();                     // ... and every wave's; the previous chunk is consumed
    };
    if (chunk_inside(0)) issue_fast(0, 0);
    else issue(0, 0);
    const int nfull = edge_tile ? 0 : a.n / KT;
    // undo the fp16 scales one at a time: each reciprocal is a normal power
    // of two, while 1 / (sa sb) could leave the float range
    const float ra = (MODE == 0) ? 1.f : 1.f / sa, rb = (MODE == 0) ? 1.f : 1.f / sb;
    // The k loop and the epilogue, for plane group G (a compile-time constant,
    // so register arrays are indexed statically; both groups run the same
    // sequence of barriers).
    auto run = [&](auto G) {
        auto comp = [&](int c, int b, bool mask, bool inter) {
            if constexpr (PG) compute_pg(G, c, b, mask, inter);
            else compute(c, b, mask, inter);
        };
        // Unmasked chunks first, then the masked ones (a k tail, or every
        // chunk of an edge tile): one compute variant per loop, so that the
        // accumulators are defined in one place per loop and stay in AGPRs
        // across iterations.  While chunk c is multiplied, the DMA of chunk
        // c + 1 goes out in slices between its plane steps.
        int c = 0;
        for (; c + 1 < nfull; ++c) {         // chunk c + 1 is interior as well
            sync();
            comp(c, c & 1, false, true);
        }
        for (; c < nfull; ++c) {
            sync();
            if (c + 1 < nchunks) {
                if (chunk_inside(c + 1)) issue_fast(c + 1, (c + 1) & 1);
                else issue(c + 1, (c + 1) & 1);
            }
            comp(c, c & 1, false, false);
        }
        for (; c < nchunks; ++c) {
            sync();
            if (c + 1 < nchunks) issue(c + 1, (c + 1) & 1);
            comp(c, c & 1, true, false);
        }
        __syncthreads();                     // the staging buffers are free
        const int row0 = m0 + wm * (MT / WM), col0 = n0 + wn * (NT / 2);
        if constexpr (PG) {
            // group 0 stores C1 (planes 0, 1), group 1 stores C2 (planes 2, 3);
            // each hands the other its partial sums of the other's planes
            constexpr int g0 = decltype(G)::value;
            constexpr int send = g0 == 0 ? 2 : 0, keep = g0 == 0 ? 0 : 2;
            constexpr int NREG = 2 * MB * NB * 16, LANES = 64 * WG;
            static_assert(2 * NREG * LANES * sizeof(float) <= sizeof(V2Smem<MT, NT>),
                          "reduction does not fit the staging buffers");
            float* red = reinterpret_cast<float*>(&sm);
            float* mine = red + (size_t)g0 * NREG * LANES;
            const float* theirs = red + (size_t)(1 - g0) * NREG * LANES;
            const int slot = tw * 64 + lane;
            int idx = 0;
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int r = 0; r < 16; ++r) mine[(size_t)(idx++) * LANES + slot] = acc[send + c2][mb][nb][r];
            __syncthreads();
            idx = 0;
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int r = 0; r < 16; ++r) acc[keep + c2][mb][nb][r] += theirs[(size_t)(idx++) * LANES + slot];
            __syncthreads();                 // LDS may be reused by the next tile
            store_tile<MB, NB, keep, 2>(a, f, row0, col0, acc, ra, rb, lane);
        } else if constexpr (KARA) {
            v16f out[4][MB][NB];
#pragma unroll
            for (int h = 0; h < NOUT; ++h)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const float p1 = acc[3 * h][mb][nb][r], p2 = acc[3 * h + 1][mb][nb][r];
                            out[2 * h][mb][nb][r] = p1 - p2;
                            out[2 * h + 1][mb][nb][r] = acc[3 * h + 2][mb][nb][r] - p1 - p2;
                        }
            store_tile<MB, NB, 0, 2 * NOUT>(a, f, row0, col0, out, ra, rb, lane);
        } else {
            store_tile<MB, NB, 0, CX ? 2 : 4>(a, f, row0, col0, acc, ra, rb, lane);
        }
    };
    if constexpr (PG) {
        if (grp == 0) run(std::integral_constant<int, 0>{});
        else run(std::integral_constant<int, 1>{});
    } else {
        run(std::integral_constant<int, 0>{});
    }
}

}  // namespace detail
}  // namespace qt
