// mlp.hip -- learned starting guess of the two-fluid implicit stage (include/rmhd_mlp.h):
// a 19-64-64-7 tanh network with FP32 master weights used in bfloat16.
//
//   k_quantize   master weights -> bfloat16-rounded FP32 copy and matrix-core operand tiles
//   k_infer      inference on the matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulate)
//                of raw feature rows
//   k_guess      the same network on the features of a stage's right-hand side R, writing
//                the starting point x0 = R_x + D y (coalesced: one cell per lane)
//   k_fwd32      FP32-activation forward, one sample per thread
//   k_grad       forward + backward of 32 samples per block through LDS, per-block gradient
//   k_adam       fixed-order sum of the block gradients, Adam update, re-rounding
//   k_moments    column sums for the normalisation (two passes, FP64, ordered)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/rmhd_mlp.h"
#include "kernels.hpp"
#include "mlp.hpp"
#include "mlp_net.hpp"

namespace rmhd {
namespace mlp {

// ---------------------------------------------------------------------------------------
// re-rounding of the master weights
// ---------------------------------------------------------------------------------------
// Tile t, lane l, element e holds the weight of row 16 m + (l % 16) and column
// operand_col(kb, l / 16, e) of its matrix: the A-operand layout of the 16x16x32 matrix
// instruction with the K order the network's B operands use.
__global__ void k_quantize(const float *master, float *wq, unsigned short *packed)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < NPAR) wq[t] = bf16_float(master[t]);
    if (t >= PACKED) return;
    const int tile = t >> 9, lane = (t >> 3) & 63, e = t & 7;
    const int r16 = lane & 15, q = lane >> 4;
    float v = 0.0f;
    if (tile < 4) {
        const int row = 16 * tile + r16, col = operand_col(0, q, e);
        if (col < NIN) v = master[OW1 + row * NIN + col];
    } else if (tile < 12) {
        const int m = (tile - 4) >> 1, kb = (tile - 4) & 1;
        v = master[OW2 + (16 * m + r16) * NH + operand_col(kb, q, e)];
    } else {
        const int kb = tile - 12;
        if (r16 < NOUT) v = master[OW3 + r16 * NH + operand_col(kb, q, e)];
    }
    packed[t] = bf16_bits(v);
}

// ---------------------------------------------------------------------------------------
// inference on the matrix cores (net_tile, mlp_net.hpp)
// ---------------------------------------------------------------------------------------
// Raw feature rows X[n][19] -> outputs Y[n][7] (target units), one 16-sample tile per wave
// and step; the next tile's inputs are fetched before the current tile's products.
struct InferArgs {
    const bf8 *packed;
    const float *wq;     // biases
    const float *norm;
    const float *X;
    float *Y;
    long n;
};

__global__ __launch_bounds__(256) void k_infer(InferArgs A)
{
    const int lane = threadIdx.x & 63, col = lane & 15, q = lane >> 4;
    NetRegs N;
    load_net(A.packed, A.wq, lane, N);
    // this lane's inputs: 4q + e (first K block) and 16 + 4q + e (second, q = 0 only)
    float fm[8], fsi[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int f = (e < 4 ? 0 : 16) + 4 * q + (e & 3);
        fm[e] = f < NIN ? A.norm[NFM + f] : 0.0f;
        fsi[e] = f < NIN ? inv_std(A.norm[NFS + f]) : 0.0f;
    }
    const long ntiles = (A.n + 15) / 16;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
    auto fetch = [&](long tile, float (&v)[8]) {
        const long s = tile * 16 + col;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = 0.0f;
        if (tile >= ntiles || s >= A.n) return;
        const float *x = A.X + s * NIN;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int fi = (e < 4 ? 0 : 16) + 4 * q + (e & 3);
            if (fi < NIN) v[e] = x[fi];
        }
    };
    float cur[8], nxt[8];
    fetch(wave, cur);
    for (long tile = wave; tile < ntiles; tile += nwaves) {
        fetch(tile + nwaves, nxt);
        const long s = tile * 16 + col;
        float u[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) u[e] = (cur[e] - fm[e]) * fsi[e];
        if (q > 0) u[4] = u[5] = u[6] = u[7] = 0.0f;   // padded columns 20..31
        const f4 acc = net_tile(N, cat8(pack4(u[0], u[1], u[2], u[3]), pack4(u[4], u[5], u[6], u[7])));
        if (s < A.n && q <= 1) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = 4 * q + e;
                if (k < NOUT) A.Y[s * NOUT + k] = A.norm[NTM + k] + A.norm[NTS + k] * acc[e];
            }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) cur[e] = nxt[e];
    }
}

// Learned starting point of a two-fluid stage with right-hand side R: x0 = R_x + D y on the
// seven source-carrying planes, for every cell of the padded grid.  One wavefront takes 64
// consecutive cells, one per lane, so that every plane is read and written in whole
// 512-byte rows; the standardised features go to the matrix-core layout (16 cells per
// product) through LDS, and the outputs come back to their cells the same way.  The LDS
// rows are private to the wavefront, so a wave-level fence orders them (no block barrier).
struct GuessArgs {
    const bf8 *packed;
    const float *wq, *norm;
    CPlanes R;
    Planes guess;
    Geo g;
    Phys P;
    double a;
};
// Bounded to three wavefronts per SIMD (168 registers), which the kernel fits without spills.
__global__ __launch_bounds__(256, 3) void k_guess(GuessArgs A)
{
    __shared__ __attribute__((aligned(16))) unsigned short s_u[4][64][UROW];
    __shared__ float s_y[4][64][8];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, col = lane & 15, q = lane >> 4;
    // standardisation of the features (means, reciprocal standard deviations), read from LDS
    // as broadcasts
    __shared__ float s_fm[NIN], s_fsi[NIN];
    if (threadIdx.x < NIN) {
        s_fm[threadIdx.x] = A.norm[NFM + threadIdx.x];
        s_fsi[threadIdx.x] = inv_std(A.norm[NFS + threadIdx.x]);
    }
    __syncthreads();
    NetRegs N;
    load_net(A.packed, A.wq, lane, N);
    const Geo &g = A.g;
    const double sc = fabs(A.P.mu1), amu = A.a * A.P.mu1 * A.P.mu1;
    const long nchunks = (g.plane + 63) / 64;
    for (long c = (long)blockIdx.x * 4 + wv; c < nchunks; c += (long)gridDim.x * 4) {
        const long s = c * 64 + lane;
        const long r = s / g.pitch;
        const bool live = s < g.plane && s - r * g.pitch < g.nxg && r < g.rows;
        // every lane loads (a lane past the end from the last cell), so the loads need no
        // branches; dead lanes' values are replaced below
        const long sl = s < g.plane ? s : g.plane - 1;
        double Rv[18];
#pragma unroll
        for (int v = 0; v < 18; ++v) Rv[v] = A.R.p[v][sl];
        const double sig = cell_sigma(A.P, sl);
        // features in FP32 (rounded to bfloat16 before the first product), standardised
        guess_features(Rv, sig, amu, A.a, live, s_fm, s_fsi, &s_u[wv][lane][0]);
        wave_lds_sync();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const f4 acc = net_tile(N, guess_operand(s_u[wv], t, lane));
            if (q <= 1) {
#pragma unroll
                for (int e = 0; e < 4; ++e) s_y[wv][16 * t + col][4 * q + e] = acc[e];
            }
        }
        wave_lds_sync();
        if (live) {
            // x0 = R_x + D y in conserved units, as the stage reads its starting point
            const int px[NOUT] = {tf::SBX, tf::SBY, tf::SBZ, tf::TAUB, tf::EX, tf::EY, tf::EZ};
            double x0[NOUT];
            guess_start(Rv, s_y[wv][lane], A.norm, sc, x0);
#pragma unroll
            for (int k = 0; k < NOUT; ++k) A.guess.p[px[k]][s] = x0[k];
        }
        wave_lds_sync();   // this chunk's LDS reads before the next chunk's writes
    }
}

// ---------------------------------------------------------------------------------------
// FP32 forward, one sample per thread
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fwd32(const float *X, long n, const float *wq, const float *norm, float *Y)
{
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float u[NIN], h1[NH], h2[NH];
#pragma unroll
    for (int f = 0; f < NIN; ++f) u[f] = (X[s * NIN + f] - norm[NFM + f]) / norm[NFS + f];
    for (int i = 0; i < NH; ++i) {
        float z = wq[OB1 + i];
#pragma unroll
        for (int f = 0; f < NIN; ++f) z = fmaf(wq[OW1 + i * NIN + f], u[f], z);
        h1[i] = tanhf(z);
    }
    for (int i = 0; i < NH; ++i) {
        float z = wq[OB2 + i];
#pragma unroll
        for (int k = 0; k < NH; ++k) z = fmaf(wq[OW2 + i * NH + k], h1[k], z);
        h2[i] = tanhf(z);
    }
    for (int o = 0; o < NOUT; ++o) {
        float z = wq[OB3 + o];
#pragma unroll
        for (int k = 0; k < NH; ++k) z = fmaf(wq[OW3 + o * NH + k], h2[k], z);
        Y[s * NOUT + o] = norm[NTM + o] + norm[NTS + o] * z;
    }
}

// ---------------------------------------------------------------------------------------
// training: forward + backward of GS samples per block
// ---------------------------------------------------------------------------------------
constexpr int GS = 32;          // samples per block: 64 blocks for a 2048-sample batch (measured
                                // 1.5x faster steps than 64 samples, half the partials of 16)
constexpr int HP = NH + 1;      // padded row of the 64-wide LDS arrays
struct GradArgs {
    const float *X, *T;
    long n, first, stride;
    int batch;
    float inv_batch;            // 1 / batch
    const float *wq, *norm;
    float *partial;             // [blocks][NPAR + 1]: gradients, then the sum of squared errors
};

__global__ __launch_bounds__(256) void k_grad(GradArgs A)
{
    __shared__ float sW1[NH * NIN], sB1[NH], sW2[NH * HP], sB2[NH], sW3[NOUT * HP], sB3[8];
    __shared__ float sU[GS][NIN + 1], sT[GS][8], sDY[GS][8];
    __shared__ float sH1[GS][HP], sH2[GS][HP], sD2[GS][HP], sD1[GS][HP];
    __shared__ float sLoss[4];
    const int tid = threadIdx.x;
    const long blk = blockIdx.x;
    for (int p = tid; p < NH * NIN; p += 256) sW1[p] = A.wq[OW1 + p];
    for (int p = tid; p < NH * NH; p += 256) sW2[(p / NH) * HP + p % NH] = A.wq[OW2 + p];
    for (int p = tid; p < NOUT * NH; p += 256) sW3[(p / NH) * HP + p % NH] = A.wq[OW3 + p];
    if (tid < NH) {
        sB1[tid] = A.wq[OB1 + tid];
        sB2[tid] = A.wq[OB2 + tid];
    }
    if (tid < NOUT) sB3[tid] = A.wq[OB3 + tid];
    // samples: standardised inputs and targets; rows past the batch contribute nothing
    for (int e = tid; e < GS * (NIN + NOUT); e += 256) {
        const int s = e / (NIN + NOUT), c = e % (NIN + NOUT);
        const long r = blk * GS + s;
        float v = 0.0f;
        if (r < A.batch) {
            const long row = (A.first + r * A.stride) % A.n;
            v = c < NIN ? (A.X[row * NIN + c] - A.norm[NFM + c]) / A.norm[NFS + c]
                        : (A.T[row * NOUT + c - NIN] - A.norm[NTM + c - NIN]) / A.norm[NTS + c - NIN];
        }
        if (c < NIN) sU[s][c] = v;
        else sT[s][c - NIN] = v;
    }
    __syncthreads();
    const int i = tid & 63, s0 = tid >> 6;
    // layer 1
    for (int s = s0; s < GS; s += 4) {
        float z = sB1[i];
#pragma unroll
        for (int f = 0; f < NIN; ++f) z = fmaf(sW1[i * NIN + f], sU[s][f], z);
        sH1[s][i] = tanhf(z);
    }
    __syncthreads();
    // layer 2
    for (int s = s0; s < GS; s += 4) {
        float z = sB2[i];
#pragma unroll 16
        for (int k = 0; k < NH; ++k) z = fmaf(sW2[i * HP + k], sH1[s][k], z);
        sH2[s][i] = tanhf(z);
    }
    __syncthreads();
    // output, residual and dL/dv = 2 (v - t) / batch
    float se = 0.0f;
    for (int e = tid; e < GS * NOUT; e += 256) {
        const int s = e / NOUT, o = e % NOUT;
        float z = sB3[o];
#pragma unroll 16
        for (int k = 0; k < NH; ++k) z = fmaf(sW3[o * HP + k], sH2[s][k], z);
        const float r = (blk * GS + s < A.batch) ? z - sT[s][o] : 0.0f;
        se = fmaf(r, r, se);
        sDY[s][o] = 2.0f * r * A.inv_batch;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) se += __shfl_xor(se, o);
    if ((tid & 63) == 0) sLoss[tid >> 6] = se;
    __syncthreads();
    // dZ2 = (W3^T dv) (1 - H2^2)
    for (int s = s0; s < GS; s += 4) {
        float z = 0.0f;
#pragma unroll
        for (int o = 0; o < NOUT; ++o) z = fmaf(sDY[s][o], sW3[o * HP + i], z);
        const float h = sH2[s][i];
        sD2[s][i] = z * (1.0f - h * h);
    }
    __syncthreads();
    // dZ1 = (W2^T dZ2) (1 - H1^2)
    for (int s = s0; s < GS; s += 4) {
        float z = 0.0f;
#pragma unroll 16
        for (int k = 0; k < NH; ++k) z = fmaf(sD2[s][k], sW2[k * HP + i], z);
        const float h = sH1[s][i];
        sD1[s][i] = z * (1.0f - h * h);
    }
    __syncthreads();
    float *out = A.partial + blk * (NPAR + 1);
    // dW2[r][k] = sum_s dZ2[s][r] H1[s][k]
    for (int r = s0; r < NH; r += 4) {
        float z = 0.0f;
        for (int s = 0; s < GS; ++s) z = fmaf(sD2[s][r], sH1[s][i], z);
        out[OW2 + r * NH + i] = z;
    }
    // dW1[r][f] = sum_s dZ1[s][r] U[s][f]
    for (int e = tid; e < NH * NIN; e += 256) {
        const int r = e / NIN, f = e % NIN;
        float z = 0.0f;
        for (int s = 0; s < GS; ++s) z = fmaf(sD1[s][r], sU[s][f], z);
        out[OW1 + e] = z;
    }
    // dW3[o][k] = sum_s dv[s][o] H2[s][k]
    for (int e = tid; e < NOUT * NH; e += 256) {
        const int o = e / NH, k = e % NH;
        float z = 0.0f;
        for (int s = 0; s < GS; ++s) z = fmaf(sDY[s][o], sH2[s][k], z);
        out[OW3 + e] = z;
    }
    // biases
    if (tid < NH) {
        float z1 = 0.0f, z2 = 0.0f;
        for (int s = 0; s < GS; ++s) {
            z1 += sD1[s][tid];
            z2 += sD2[s][tid];
        }
        out[OB1 + tid] = z1;
        out[OB2 + tid] = z2;
    } else if (tid < NH + NOUT) {
        const int o = tid - NH;
        float z = 0.0f;
        for (int s = 0; s < GS; ++s) z += sDY[s][o];
        out[OB3 + o] = z;
    } else if (tid == NH + NOUT) {
        out[NPAR] = sLoss[0] + sLoss[1] + sLoss[2] + sLoss[3];
    }
}

struct AdamArgs {
    const float *partial;
    int nblk;
    float inv_batch;
    float *grad_out;   // optional
    float *loss_out;   // optional
    int update;
    float lr, bc1, bc2;   // bias corrections 1 - beta^t
    float *master, *m1, *m2, *wq;
};

// 32 parameters per block: the 8 thread groups of 32 each add a fixed contiguous range of
// the block partials in block order, and the 8 range sums are added in group order, so the
// sum is the same in every run (eight memory latencies in flight per parameter instead of
// one).
constexpr int ADAM_P = 32, ADAM_G = 8;
__global__ __launch_bounds__(256) void k_adam(AdamArgs A)
{
    __shared__ float part[ADAM_G][ADAM_P];
    const int lp = threadIdx.x % ADAM_P, grp = threadIdx.x / ADAM_P;
    const int p = blockIdx.x * ADAM_P + lp;
    const int per = (A.nblk + ADAM_G - 1) / ADAM_G, b0 = grp * per, b1 = min(A.nblk, b0 + per);
    float g = 0.0f;
    if (p <= NPAR) {
#pragma unroll 4
        for (int b = b0; b < b1; ++b) g += A.partial[(long)b * (NPAR + 1) + p];
    }
    part[grp][lp] = g;
    __syncthreads();
    if (grp != 0 || p > NPAR) return;
    g = part[0][lp];
#pragma unroll
    for (int k = 1; k < ADAM_G; ++k) g += part[k][lp];
    if (p == NPAR) {
        if (A.loss_out) *A.loss_out = g * A.inv_batch;
        return;
    }
    if (A.grad_out) A.grad_out[p] = g;
    if (!A.update) return;
    const float m = 0.9f * A.m1[p] + 0.1f * g;
    const float v = 0.999f * A.m2[p] + 0.001f * g * g;
    A.m1[p] = m;
    A.m2[p] = v;
    const float w = A.master[p] - A.lr * (m / A.bc1) / (sqrtf(v / A.bc2) + 1e-8f);
    A.master[p] = w;
    A.wq[p] = bf16_float(w);
}

// ---------------------------------------------------------------------------------------
// normalisation: column sums (pass 0) and centred sums of squares (pass 1), FP64, ordered
// ---------------------------------------------------------------------------------------
constexpr int NCOL = NIN + NOUT;
constexpr int MOM_BLOCKS = 256;

__global__ __launch_bounds__(256) void k_moments(const float *X, const float *T, long n, const double *mean,
                                                 double *partial)
{
    __shared__ double red[256];
    for (int c = 0; c < NCOL; ++c) {
        double acc = 0.0;
        const double mu = mean ? mean[c] : 0.0;
        for (long r = (long)blockIdx.x * 256 + threadIdx.x; r < n; r += (long)gridDim.x * 256) {
            const double v = (c < NIN ? X[r * NIN + c] : T[r * NOUT + c - NIN]) - mu;
            acc += mean ? v * v : v;
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[blockIdx.x * NCOL + c] = red[0];
        __syncthreads();
    }
}

__global__ void k_moments_final(const double *partial, int nblk, long n, double *mean, float *norm, int pass)
{
    const int c = threadIdx.x;
    if (c >= NCOL) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[b * NCOL + c];
    if (pass == 0) {
        mean[c] = s / (double)n;
        norm[c < NIN ? NFM + c : NTM + c - NIN] = (float)mean[c];
    } else {
        double sd = sqrt(s / (double)n);
        if (!(sd > 1e-12 * (1.0 + fabs(mean[c])))) sd = 1.0;
        norm[c < NIN ? NFS + c : NTS + c - NIN] = (float)sd;
    }
}

}  // namespace mlp
}  // namespace rmhd

// =======================================================================================
// host side
// =======================================================================================
using namespace rmhd;
using namespace rmhd::mlp;

struct rmhd_mlp {
    hipStream_t stream;
    float *master, *m1, *m2, *wq, *norm, *partial, *scratch;
    unsigned short *packed;
    double *mom;      // MOM_BLOCKS x NCOL partials + NCOL means
    long steps;
    int cus;
    std::string err;
};

static std::string g_mlp_err;

static int mfail(rmhd_mlp *m, int code, const std::string &msg)
{
    if (m) m->err = msg;
    else g_mlp_err = msg;
    return code;
}
static int mcheck(rmhd_mlp *m, hipError_t e, const char *what)
{
    if (e == hipSuccess) return RMHD_OK;
    return mfail(m, RMHD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

static int quantize(rmhd_mlp *m)
{
    const int n = PACKED > NPAR ? PACKED : NPAR;
    hipLaunchKernelGGL(k_quantize, dim3((n + 255) / 256), dim3(256), 0, m->stream, m->master, m->wq, m->packed);
    return mcheck(m, hipGetLastError(), "k_quantize launch");
}

extern "C" int rmhd_mlp_create(const float *params, void *stream, rmhd_mlp **out)
{
    if (!out) return mfail(nullptr, RMHD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params) return mfail(nullptr, RMHD_EINVAL, "params is NULL");
    for (int p = 0; p < NPAR; ++p)
        if (!std::isfinite(params[p])) return mfail(nullptr, RMHD_EINVAL, "params must be finite");
    rmhd_mlp *m = new (std::nothrow) rmhd_mlp();
    if (!m) return mfail(nullptr, RMHD_ENOMEM, "host allocation failed");
    m->stream = (hipStream_t)stream;
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&m->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (m->cus < 1) m->cus = 256;
    const size_t nblk = (RMHD_MLP_MAX_BATCH + GS - 1) / GS;
    const size_t bytes = sizeof(float) * (4 * (size_t)NPAR + RMHD_MLP_NNORM + nblk * (NPAR + 1)) +
                         sizeof(unsigned short) * PACKED + sizeof(double) * (MOM_BLOCKS + 1) * NCOL + 16;
    char *base = nullptr;
    if (hipMalloc(&base, bytes) != hipSuccess) {
        delete m;
        return mfail(nullptr, RMHD_ENOMEM, "device allocation failed");
    }
    m->scratch = (float *)base;
    float *f = m->scratch;
    m->master = f; f += NPAR;
    m->m1 = f; f += NPAR;
    m->m2 = f; f += NPAR;
    m->wq = f; f += NPAR;
    m->norm = f; f += RMHD_MLP_NNORM;
    m->partial = f; f += nblk * (NPAR + 1);
    m->mom = (double *)(((uintptr_t)f + 7) & ~(uintptr_t)7);
    m->packed = (unsigned short *)(m->mom + (MOM_BLOCKS + 1) * NCOL);
    std::vector<float> norm(RMHD_MLP_NNORM, 0.0f);
    for (int k = 0; k < NIN; ++k) norm[NFS + k] = 1.0f;
    for (int k = 0; k < NOUT; ++k) norm[NTS + k] = 1.0f;
    int rc = mcheck(m, hipMemcpyAsync(m->master, params, sizeof(float) * NPAR, hipMemcpyHostToDevice, m->stream),
                    "copy params");
    if (!rc) rc = mcheck(m, hipMemsetAsync(m->m1, 0, sizeof(float) * 2 * NPAR, m->stream), "clear moments");
    if (!rc)
        rc = mcheck(m, hipMemcpyAsync(m->norm, norm.data(), sizeof(float) * RMHD_MLP_NNORM, hipMemcpyHostToDevice,
                                      m->stream), "copy norm");
    if (!rc) rc = quantize(m);
    if (!rc) rc = mcheck(m, hipStreamSynchronize(m->stream), "create sync");
    if (rc) {
        g_mlp_err = m->err;
        hipFree(m->scratch);
        delete m;
        return rc;
    }
    *out = m;
    return RMHD_OK;
}

extern "C" void rmhd_mlp_destroy(rmhd_mlp *m)
{
    if (!m) return;
    hipStreamSynchronize(m->stream);
    hipFree(m->scratch);
    delete m;
}

extern "C" int rmhd_mlp_get_params(rmhd_mlp *m, float *params)
{
    if (!m || !params) return mfail(m, RMHD_EINVAL, "rmhd_mlp_get_params: NULL argument");
    int rc = mcheck(m, hipMemcpyAsync(params, m->master, sizeof(float) * NPAR, hipMemcpyDeviceToHost, m->stream),
                    "copy params");
    return rc ? rc : mcheck(m, hipStreamSynchronize(m->stream), "sync");
}

extern "C" int rmhd_mlp_get_norm(rmhd_mlp *m, float *norm)
{
    if (!m || !norm) return mfail(m, RMHD_EINVAL, "rmhd_mlp_get_norm: NULL argument");
    int rc = mcheck(m, hipMemcpyAsync(norm, m->norm, sizeof(float) * RMHD_MLP_NNORM, hipMemcpyDeviceToHost, m->stream),
                    "copy norm");
    return rc ? rc : mcheck(m, hipStreamSynchronize(m->stream), "sync");
}

extern "C" int rmhd_mlp_set_norm(rmhd_mlp *m, const float *norm)
{
    if (!m || !norm) return mfail(m, RMHD_EINVAL, "rmhd_mlp_set_norm: NULL argument");
    for (int k = 0; k < RMHD_MLP_NNORM; ++k) {
        if (!std::isfinite(norm[k])) return mfail(m, RMHD_EINVAL, "rmhd_mlp_set_norm: values must be finite");
        const bool is_std = (k >= NFS && k < NTM) || k >= NTS;
        if (is_std && !(norm[k] > 0.0f)) return mfail(m, RMHD_EINVAL, "rmhd_mlp_set_norm: std must be > 0");
    }
    int rc = mcheck(m, hipMemcpyAsync(m->norm, norm, sizeof(float) * RMHD_MLP_NNORM, hipMemcpyHostToDevice, m->stream),
                    "copy norm");
    return rc ? rc : mcheck(m, hipStreamSynchronize(m->stream), "sync");
}

extern "C" int rmhd_mlp_fit_norm(rmhd_mlp *m, const float *X, const float *T, long n)
{
    if (!m || !X || !T) return mfail(m, RMHD_EINVAL, "rmhd_mlp_fit_norm: NULL argument");
    if (n < 1) return mfail(m, RMHD_EINVAL, "rmhd_mlp_fit_norm: n must be >= 1");
    double *partial = m->mom, *mean = m->mom + MOM_BLOCKS * NCOL;
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_moments, dim3(MOM_BLOCKS), dim3(256), 0, m->stream, X, T, n,
                           (const double *)(pass ? mean : nullptr), partial);
        hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(64), 0, m->stream, (const double *)partial, MOM_BLOCKS, n,
                           mean, m->norm, pass);
    }
    return mcheck(m, hipGetLastError(), "k_moments launch");
}

extern "C" int rmhd_mlp_forward(rmhd_mlp *m, const float *X, long n, float *Y, int precision)
{
    if (!m || !X || !Y) return mfail(m, RMHD_EINVAL, "rmhd_mlp_forward: NULL argument");
    if (n < 0) return mfail(m, RMHD_EINVAL, "rmhd_mlp_forward: n must be >= 0");
    if (precision != 0 && precision != 1) return mfail(m, RMHD_EINVAL, "rmhd_mlp_forward: precision must be 0 or 1");
    if (n == 0) return RMHD_OK;
    if (precision == 0) {
        hipLaunchKernelGGL(k_fwd32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m->stream, X, n,
                           (const float *)m->wq, (const float *)m->norm, Y);
        return mcheck(m, hipGetLastError(), "k_fwd32 launch");
    }
    InferArgs A{};
    A.packed = (const bf8 *)m->packed;
    A.wq = m->wq;
    A.norm = m->norm;
    A.X = X;
    A.Y = Y;
    A.n = n;
    const long tiles = (n + 15) / 16;
    long blocks = (tiles + 3) / 4;
    if (blocks > 8L * m->cus) blocks = 8L * m->cus;
    hipLaunchKernelGGL(k_infer, dim3((unsigned)blocks), dim3(256), 0, m->stream, A);
    return mcheck(m, hipGetLastError(), "k_infer launch");
}

static int grad_step(rmhd_mlp *m, const float *X, const float *T, long n, long first, long stride, int batch,
                     float *grad, float *loss, int update, float lr)
{
    GradArgs G{};
    G.X = X;
    G.T = T;
    G.n = n;
    G.first = first;
    G.stride = stride;
    G.batch = batch;
    G.inv_batch = 1.0f / (float)batch;
    G.wq = m->wq;
    G.norm = m->norm;
    G.partial = m->partial;
    const int nblk = (batch + GS - 1) / GS;
    hipLaunchKernelGGL(k_grad, dim3(nblk), dim3(256), 0, m->stream, G);
    AdamArgs A{};
    A.partial = m->partial;
    A.nblk = nblk;
    A.inv_batch = G.inv_batch;
    A.grad_out = grad;
    A.loss_out = loss;
    A.update = update;
    if (update) {
        m->steps += 1;
        A.lr = lr;
        A.bc1 = (float)(1.0 - pow(0.9, (double)m->steps));
        A.bc2 = (float)(1.0 - pow(0.999, (double)m->steps));
    }
    A.master = m->master;
    A.m1 = m->m1;
    A.m2 = m->m2;
    A.wq = m->wq;
    hipLaunchKernelGGL(k_adam, dim3((NPAR + 1 + ADAM_P - 1) / ADAM_P), dim3(ADAM_P * ADAM_G), 0, m->stream, A);
    int rc = mcheck(m, hipGetLastError(), "k_grad/k_adam launch");
    if (!rc && update) rc = quantize(m);
    return rc;
}

extern "C" int rmhd_mlp_loss_grad(rmhd_mlp *m, const float *X, const float *T, long n, float *grad, float *loss)
{
    if (!m || !X || !T) return mfail(m, RMHD_EINVAL, "rmhd_mlp_loss_grad: NULL argument");
    if (n < 1 || n > RMHD_MLP_MAX_BATCH) return mfail(m, RMHD_EINVAL, "rmhd_mlp_loss_grad: need 1 <= n <= max batch");
    return grad_step(m, X, T, n, 0, 1, (int)n, grad, loss, 0, 0.0f);
}

extern "C" int rmhd_mlp_train_step(rmhd_mlp *m, const float *X, const float *T, long n, long first, long stride,
                                   int batch, float lr, float *loss)
{
    if (!m || !X || !T) return mfail(m, RMHD_EINVAL, "rmhd_mlp_train_step: NULL argument");
    if (n < 1 || batch < 1 || batch > RMHD_MLP_MAX_BATCH)
        return mfail(m, RMHD_EINVAL, "rmhd_mlp_train_step: need n >= 1 and 1 <= batch <= max batch");
    if (first < 0 || stride < 1) return mfail(m, RMHD_EINVAL, "rmhd_mlp_train_step: need first >= 0, stride >= 1");
    if (!(lr > 0.0f)) return mfail(m, RMHD_EINVAL, "rmhd_mlp_train_step: lr must be > 0");
    return grad_step(m, X, T, n, first % n, stride % n == 0 ? 1 : stride % n, batch, nullptr, loss, 1, lr);
}

static unsigned long long splitmix(unsigned long long &s)
{
    unsigned long long z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static long gcdl(long a, long b)
{
    while (b) {
        const long t = a % b;
        a = b;
        b = t;
    }
    return a;
}

extern "C" int rmhd_mlp_train(rmhd_mlp *m, const float *X, const float *T, long n, int batch, int epochs, float lr0,
                              float lr1, unsigned long long seed, float *loss_hist)
{
    if (!m || !X || !T) return mfail(m, RMHD_EINVAL, "rmhd_mlp_train: NULL argument");
    if (n < 1 || batch < 1 || batch > RMHD_MLP_MAX_BATCH || epochs < 1)
        return mfail(m, RMHD_EINVAL, "rmhd_mlp_train: need n >= 1, 1 <= batch <= max batch, epochs >= 1");
    if (!(lr0 > 0.0f) || !(lr1 > 0.0f)) return mfail(m, RMHD_EINVAL, "rmhd_mlp_train: learning rates must be > 0");
    const long per_epoch = (n + batch - 1) / batch;
    const long total = per_epoch * epochs;
    float *losses = nullptr;   // per-step losses of one epoch, in the partial buffer's tail
    std::vector<float> host(per_epoch);
    if (loss_hist) {
        if (hipMalloc(&losses, sizeof(float) * per_epoch) != hipSuccess)
            return mfail(m, RMHD_ENOMEM, "rmhd_mlp_train: loss buffer");
    }
    unsigned long long st = seed;
    long k = 0;
    int rc = RMHD_OK;
    for (int ep = 0; ep < epochs && !rc; ++ep) {
        long stride = 1 + (long)(splitmix(st) % (unsigned long long)n);
        while (gcdl(stride, n) != 1) stride = stride % n + 1;
        const long first = (long)(splitmix(st) % (unsigned long long)n);
        for (long b = 0; b < per_epoch && !rc; ++b, ++k) {
            const int rows = (int)(b + 1 < per_epoch ? batch : n - b * (long)batch);
            const float lr = lr0 + (lr1 - lr0) * (float)((double)k / (double)(total > 1 ? total - 1 : 1));
            rc = grad_step(m, X, T, n, (first + b * (long)batch * stride) % n, stride, rows, nullptr,
                           losses ? losses + b : nullptr, 1, lr);
        }
        if (!rc && loss_hist) {
            rc = mcheck(m, hipMemcpyAsync(host.data(), losses, sizeof(float) * per_epoch, hipMemcpyDeviceToHost,
                                          m->stream), "copy losses");
            if (!rc) rc = mcheck(m, hipStreamSynchronize(m->stream), "sync");
            double s = 0.0;
            for (long b = 0; b < per_epoch; ++b) s += host[b];
            loss_hist[ep] = (float)(s / (double)per_epoch);
        }
    }
    if (losses) {
        hipStreamSynchronize(m->stream);
        hipFree(losses);
    }
    return rc;
}

extern "C" long rmhd_mlp_steps(const rmhd_mlp *m) { return m ? m->steps : 0; }

extern "C" const char *rmhd_mlp_last_error(const rmhd_mlp *m) { return m ? m->err.c_str() : g_mlp_err.c_str(); }

// ---- internal interface for the solver context -----------------------------------------
namespace rmhd {

int mlp_launch_guess(const rmhd_mlp *m, hipStream_t stream, const CPlanes &R, const Planes &guess, const Geo &g,
                     const Phys &P, double a)
{
    GuessArgs A{};
    A.packed = (const bf8 *)m->packed;
    A.wq = m->wq;
    A.norm = m->norm;
    A.R = R;
    A.guess = guess;
    A.g = g;
    A.P = P;
    A.a = a;
    // four 64-cell chunks per block and round; a few blocks per CU, each wave loading the
    // weight tiles once
    long blocks = (g.plane + 255) / 256;
    if (blocks > 4L * m->cus) blocks = 4L * m->cus;
    hipLaunchKernelGGL(k_guess, dim3((unsigned)blocks), dim3(256), 0, stream, A);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
}  // namespace rmhd
