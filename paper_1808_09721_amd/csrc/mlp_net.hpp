// mlp_net.hpp -- the learned starting guess's 19-64-64-7 tanh network as one wavefront
// evaluates it on the matrix cores (bfloat16 operands, FP32 accumulation): operand layout,
// weight and bias registers, one 16-sample tile, the features of a stage's right-hand side and
// the starting point formed from the outputs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/rmhd_mlp.h"

namespace rmhd {
namespace mlp {

constexpr int NIN = RMHD_MLP_NIN, NH = RMHD_MLP_NHID, NOUT = RMHD_MLP_NOUT, NPAR = RMHD_MLP_NPARAMS;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NOUT * NH;
static_assert(OB3 + NOUT == NPAR, "parameter layout");
// normalisation vector
constexpr int NFM = 0, NFS = NIN, NTM = 2 * NIN, NTS = 2 * NIN + NOUT;

// Matrix-core operand tiles for v_mfma_f32_16x16x32_bf16 (16 rows x 32 columns of a weight
// matrix, 64 lanes x 8 bfloat16 each): W1 as 4 row blocks (19 columns padded to 32), W2 as
// 4 x 2, W3 as 1 x 2 (7 rows padded to 16).
constexpr int TILES = 4 + 8 + 2;
constexpr int PACKED = TILES * 64 * 8;   // bfloat16 values

typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// The K index a lane's operand element stands for.  A product sums over K, so any
// permutation of K applied to both operands gives the same sum; this one is chosen so that
// the accumulator rows one product leaves in a lane (rows 4q .. 4q+3 of each 16-row block,
// q = lane / 16) are, two blocks side by side, exactly the B operand the next product needs
// from that lane.  Element e of lane group q in the tile over columns 32 kb .. 32 kb + 31:
//   e < 4:  column 32 kb + 4 q + e        (first 16-column half)
//   e >= 4: column 32 kb + 16 + 4 q + e-4 (second half)
__host__ __device__ constexpr int operand_col(int kb, int q, int e)
{
    return 32 * kb + (e < 4 ? 4 * q + e : 16 + 4 * q + (e - 4));
}

__host__ __device__ inline unsigned short bf16_bits(float f)
{
    unsigned u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__host__ __device__ inline float bf16_float(float f)
{
    const unsigned u = (unsigned)bf16_bits(f) << 16;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

__device__ inline float fast_tanh(float z)
{
    // 1 - 2 / (1 + e^{2z}) = 1 - 2 / (1 + 2^{2 z log2 e}) with the hardware base-2 exponential
    // and reciprocal (about 1 ulp each, far below the bfloat16 rounding that follows);
    // saturates to +-1.  The constant is 2 log2 e, so the product is twice z log2 e exactly.
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * 2.8853900817779268f));
}

// Four values rounded to bfloat16 (nearest, ties to even: gfx950's packed conversion, two
// values per instruction, the same rounding as bf16_bits for finite values).
__device__ inline bf4 pack4(float a, float b, float c, float d)
{
    const f4 x = {a, b, c, d};
    return __builtin_convertvector(x, bf4);
}
__device__ inline bf8 cat8(bf4 lo, bf4 hi) { return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7); }

// The network as one wavefront holds it: the 14 weight tiles in the A-operand layout and the
// biases of the accumulator rows of this lane (rows 4q + e).
struct NetRegs {
    bf8 w1[4], w2[4][2], w3[2];
    float b1[4][4], b2[4][4], b3[4];
};

__device__ inline void load_net(const bf8 *packed, const float *wq, int lane, NetRegs &N)
{
    const int q = lane >> 4;
#pragma unroll
    for (int m = 0; m < 4; ++m) N.w1[m] = packed[m * 64 + lane];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) N.w2[m][kb] = packed[(4 + m * 2 + kb) * 64 + lane];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) N.w3[kb] = packed[(12 + kb) * 64 + lane];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            N.b1[m][e] = wq[OB1 + 16 * m + 4 * q + e];
            N.b2[m][e] = wq[OB2 + 16 * m + 4 * q + e];
        }
#pragma unroll
    for (int e = 0; e < 4; ++e) N.b3[e] = (4 * q + e < NOUT) ? wq[OB3 + 4 * q + e] : 0.0f;
}

// One tile of 16 samples through the network, evaluated transposed (H^T = W U^T) so that
// activations never leave registers.  x: the standardised inputs operand_col(0, q, e) of
// sample lane % 16 (B-operand layout).  Returns the output rows 4q + e of that sample,
// biases included, in standardised target units.  Each product accumulates onto its biases.
__device__ inline f4 net_tile(const NetRegs &N, bf8 x)
{
    bf4 h1[4], h2[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        f4 acc = {N.b1[m][0], N.b1[m][1], N.b1[m][2], N.b1[m][3]};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.w1[m], x, acc, 0, 0, 0);
        h1[m] = pack4(fast_tanh(acc[0]), fast_tanh(acc[1]), fast_tanh(acc[2]), fast_tanh(acc[3]));
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        f4 acc = {N.b2[m][0], N.b2[m][1], N.b2[m][2], N.b2[m][3]};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.w2[m][kb], cat8(h1[2 * kb], h1[2 * kb + 1]), acc, 0, 0, 0);
        h2[m] = pack4(fast_tanh(acc[0]), fast_tanh(acc[1]), fast_tanh(acc[2]), fast_tanh(acc[3]));
    }
    f4 acc = {N.b3[0], N.b3[1], N.b3[2], N.b3[3]};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.w3[kb], cat8(h2[2 * kb], h2[2 * kb + 1]), acc, 0, 0, 0);
    return acc;
}

// Reciprocal standard deviations of the inputs (0 where a std is not positive): the
// standardised value is rounded to bfloat16 next, far coarser than the multiply's rounding.
__device__ inline float inv_std(float s) { return s > 0.0f ? 1.0f / s : 0.0f; }

constexpr int UROW = 40;   // bfloat16 per LDS feature row (32 used): 80-byte rows spread the
                           // B-operand reads of 16 consecutive cells over the banks

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The 19 standardised features of a two-fluid right-hand side R (18 conserved values) with
// stage coefficient a, conductivity sig and amu = a mu1^2, rounded to bfloat16 into an LDS
// row (32 values, zero past the 19th; all zero where live is false).  fm, fsi: means and
// reciprocal standard deviations of the features.
//   f0 = log10(a mu1^2 D), fk = R_k / D (k = 1..17), f18 = log10(a sig)
__device__ inline void guess_features(const double (&R)[18], double sig, double amu, double a, bool live,
                                      const float *fm, const float *fsi, unsigned short *row)
{
    const float iD = __builtin_amdgcn_rcpf((float)R[0]);
    float f[32];
    f[0] = __log10f((float)(amu * R[0]));
#pragma unroll
    for (int k = 1; k < 18; ++k) f[k] = (float)R[k] * iD;
    f[18] = __log10f((float)(a * sig));
#pragma unroll
    for (int k = 0; k < NIN; ++k) f[k] = live ? (f[k] - fm[k]) * fsi[k] : 0.0f;
#pragma unroll
    for (int k = NIN; k < 32; ++k) f[k] = 0.0f;
    bf4 *r = (bf4 *)row;
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = pack4(f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]);
}

// B operand of the cells 16 t .. 16 t + 15 of a wave's LDS feature rows, for this lane.
__device__ inline bf8 guess_operand(const unsigned short (*rows)[UROW], int t, int lane)
{
    const bf4 *src = (const bf4 *)&rows[16 * t + (lane & 15)][0];
    const int q = lane >> 4;
    return cat8(src[q], src[4 + q]);
}


// Learned starting unknowns of the two-fluid stage from the network's outputs y (standardised
// target units; norm: the normalisation vector) for right-hand side R (18 conserved values):
// x0 = R_x + D (tm + ts y) on the seven source-carrying components Sbar, taubar, E, in
// conserved units (the momentum and energy parts times sc = |mu1|).
__device__ inline void guess_start(const double (&R)[18], const float *y, const float *norm, double sc,
                                   double (&x0)[NOUT])
{
    constexpr int px[NOUT] = {6, 7, 8, 9, 13, 14, 15};   // Sbx, Sby, Sbz, taubar, Ex, Ey, Ez
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
        const float t = norm[NTM + k] + norm[NTS + k] * y[k];
        const double scale = k < 4 ? sc : 1.0;
        x0[k] = R[px[k]] + R[0] * scale * (double)t;
    }
}

}  // namespace mlp
}  // namespace rmhd
