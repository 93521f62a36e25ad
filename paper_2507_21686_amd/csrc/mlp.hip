// Learned surrogate of the per-pair integrals: training-side kernels.
//
// The network maps 8 canonical pair features to 4 outputs (standardised
// I, h Gx, h Gy in the rotated frame, and an error indicator) through three
// hidden layers of 128 units:  8 -> 128 -> 128 -> 128 -> 4.
//
// Arithmetic: layer inputs and weights are rounded to bfloat16 and multiplied
// on the matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation); the
// features enter as bfloat16 pairs hi + lo (about 16 significant bits) in the
// otherwise empty half of the first layer's 16-wide k step; biases,
// activations and their derivatives are FP32; master weights, gradients and
// Adam moments are FP32.  In the backward pass the pre-activation gradients
// are rounded to bfloat16 before they enter the matrix cores.
//
// Training uses one generic GEMM kernel (one wavefront per 32x32 output
// tile) with fused epilogues, a loss kernel, deterministic split reductions
// for the weight and bias gradients, and an Adam kernel.  Batches are padded
// to a multiple of 32 rows; padded rows carry zero features and zero loss
// gradient.

#include <math.h>

#include "internal.h"
#include "surrogate.h"

namespace sphbi {
namespace {

using namespace mlp;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ----------------------------------------------------------------------------
// generic 32x32-tile GEMM with fused epilogues
// ----------------------------------------------------------------------------
enum Epi { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_BWD = 2, EPI_PART = 3 };

struct GemmArgs {
    int M, N, K;                    // multiples of 32, 32 and 16
    const bf16 *A;                  // A(m, k) = A[m * a_m + k * a_k]
    int64_t a_m, a_k;
    const bf16 *B;                  // B(k, n) = B[k * b_k + n * b_n]
    int64_t b_k, b_n;
    int k_chunk;                    // split-K: blockIdx.z covers [z k_chunk, (z+1) k_chunk)
    const float *bias;              // EPI_HIDDEN / EPI_OUT: [N]
    float *zout;                    // EPI_HIDDEN: pre-activations [M][N]
    bf16 *aout;                     // EPI_HIDDEN: activations [M][N]
    const float *zin;               // EPI_BWD: pre-activations of the layer below [M][N]
    bf16 *dzout;                    // EPI_BWD: [M][N]
    float *out;                     // EPI_OUT: [M][N]; EPI_PART: [splits][M][N]
};

// AKC / BKC: the k index of A / B is contiguous (a_k == 1 / b_k == 1), so a
// lane's eight consecutive k values are one 16-byte load.
template <bool AKC, bool BKC, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    const int lane = threadIdx.x & 63;
    const int tn = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (tn * 32 >= g.N) return;                     // whole wavefront
    const int64_t m0 = (int64_t)blockIdx.x * 32;
    const int n0 = tn * 32;
    const int kb = blockIdx.z * g.k_chunk;
    const int ke = min(g.K, kb + g.k_chunk);
    const int64_t mi = m0 + (lane & 31), ni = n0 + (lane & 31);
    const int kh = (lane >> 5) * 8;
    f32x16 acc = {};
    for (int k0 = kb; k0 < ke; k0 += 16) {
        bf16x8 a, b;
        if (AKC) {
            a = *reinterpret_cast<const bf16x8 *>(g.A + mi * g.a_m + (k0 + kh));
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = g.A[mi * g.a_m + (int64_t)(k0 + kh + j) * g.a_k];
        }
        if (BKC) {
            b = *reinterpret_cast<const bf16x8 *>(g.B + ni * g.b_n + (k0 + kh));
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) b[j] = g.B[(int64_t)(k0 + kh + j) * g.b_k + ni * g.b_n];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    // acc[r] holds C[m0 + 8 (r / 4) + 4 (lane / 32) + r % 4][n0 + lane % 32]
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t m = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t o = m * g.N + ni;
        const float v = acc[r];
        if (EPI == EPI_HIDDEN) {
            const float z = v + g.bias[ni];
            g.zout[o] = z;
            g.aout[o] = (bf16)act(z);
        } else if (EPI == EPI_OUT) {
            g.out[o] = v + g.bias[ni];
        } else if (EPI == EPI_BWD) {
            g.dzout[o] = (bf16)(v * act_grad(g.zin[o]));
        } else {
            g.out[(int64_t)blockIdx.z * g.M * g.N + o] = v;
        }
    }
}

template <bool AKC, bool BKC, int EPI>
void gemm(const GemmArgs &g, int splits, hipStream_t s) {
    dim3 grid((unsigned)(g.M / 32), (unsigned)((g.N / 32 + 3) / 4), (unsigned)splits);
    hipLaunchKernelGGL((gemm_kernel<AKC, BKC, EPI>), grid, dim3(256), 0, s, g);
}

// ----------------------------------------------------------------------------
// weights: FP32 master vector -> bfloat16 operand layouts
// ----------------------------------------------------------------------------
// wt1 [128][16]  wt1[n][k] = W1[k % 8][n] (inputs 0-7 are the bfloat16 high
//                parts of the features, 8-15 the low parts: both see W1)
// wt2, wt3 [128][128]  wt[n][k] = W[k][n]
// wt4 [32][128]  wt4[n][k] = W4[k][n] (n < 4), 0 otherwise
// wn2, wn3 [128][128]  = W (row-major [in][out]), for the backward products
// wn4 [128][32]  wn4[k][n] = W4[k][n] (n < 4), 0 otherwise
// bias [128 | 128 | 128 | 32] FP32, zero padded
__global__ void pack_kernel(const float *__restrict__ p, TrainWeights w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 128 * 16) {
        const int n = i / 16, k = i % 16;
        w.wt1[i] = (bf16)p[kOffW1 + (k % kIn) * kHid + n];
    }
    if (i < 128 * 128) {
        const int n = i / 128, k = i % 128;
        w.wt2[i] = (bf16)p[kOffW2 + k * kHid + n];
        w.wt3[i] = (bf16)p[kOffW3 + k * kHid + n];
        w.wn2[i] = (bf16)p[kOffW2 + i];
        w.wn3[i] = (bf16)p[kOffW3 + i];
    }
    if (i < 32 * 128) {
        const int n = i / 128, k = i % 128;
        w.wt4[i] = (bf16)(n < kOut ? p[kOffW4 + k * kOut + n] : 0.0f);
        const int k2 = i / 32, n2 = i % 32;
        w.wn4[i] = (bf16)(n2 < kOut ? p[kOffW4 + k2 * kOut + n2] : 0.0f);
    }
    if (i < 3 * 128 + 32) {
        float v = 0.0f;
        if (i < 128) v = p[kOffB1 + i];
        else if (i < 256) v = p[kOffB2 + i - 128];
        else if (i < 384) v = p[kOffB3 + i - 256];
        else if (i - 384 < kOut) v = p[kOffB4 + i - 384];
        w.bias[i] = v;
    }
}

// features [B][8] FP32 -> bfloat16 [Bp][32]: columns 0-7 the high parts
// hi = bf16(f), 8-15 the low parts bf16(f - hi) (f - hi is exact in FP32),
// the rest zero (the forward product reads 16 columns, the weight gradient a
// 32-row tile)
__global__ void feats_kernel(const float *__restrict__ f, int64_t B, int64_t Bp, bf16 *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Bp * 32) return;
    const int64_t b = i / 32;
    const int k = (int)(i % 32);
    bf16 v = (bf16)0.0f;
    if (b < B && k < 2 * kIn) {
        const float fv = f[b * kIn + (k % kIn)];
        const bf16 hi = (bf16)fv;
        v = k < kIn ? hi : (bf16)(fv - (float)hi);
    }
    x[i] = v;
}

// ----------------------------------------------------------------------------
// loss: mean squared error of the standardised targets plus the indicator term
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void loss_kernel(const float *__restrict__ Y, const float *__restrict__ T,
                                                   int64_t B, int64_t Bp, float s0, float s1, float s2,
                                                   float lam, bf16 *__restrict__ dz, float *__restrict__ part) {
    __shared__ float red[256];
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float l = 0.0f;
    if (b < Bp) {
        float g[kOutPad];
#pragma unroll
        for (int k = 0; k < kOutPad; ++k) g[k] = 0.0f;
        if (b < B) {
            const float *y = Y + b * kOutPad;
            const float d0 = y[0] - T[b * 3 + 0], d1 = y[1] - T[b * 3 + 1], d2 = y[2] - T[b * 3 + 2];
            const float e = log10f(fmaxf(fmaxf(fabsf(d0) * s0, fabsf(d1) * s1), fabsf(d2) * s2) + kErrFloor);
            const float de = y[3] - e;
            const float iB = 1.0f / (float)B;
            l = (d0 * d0 + d1 * d1 + d2 * d2) * (iB / 3.0f) + lam * de * de * iB;
            g[0] = 2.0f * d0 * (iB / 3.0f);
            g[1] = 2.0f * d1 * (iB / 3.0f);
            g[2] = 2.0f * d2 * (iB / 3.0f);
            g[3] = 2.0f * lam * de * iB;
        }
#pragma unroll
        for (int k = 0; k < kOutPad; ++k) dz[b * kOutPad + k] = (bf16)g[k];
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// sum of n partials in index order (one block)
__global__ __launch_bounds__(256) void sum_kernel(const float *__restrict__ part, int n, float *__restrict__ out) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// column sums of dz [M][N] over chunks of kColRows rows: part[z][n].  A block
// covers 64 columns; its four waves take every fourth row of the chunk and
// are combined in a fixed order (deterministic).
constexpr int kColRows = 256;
__global__ __launch_bounds__(256) void colsum_kernel(const bf16 *__restrict__ dz, int64_t M, int N,
                                                     float *__restrict__ part) {
    __shared__ float red[4][64];
    const int l = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int n = blockIdx.y * 64 + l;
    const int64_t r0 = (int64_t)blockIdx.x * kColRows, r1 = min(M, r0 + kColRows);
    float s = 0.0f;
    if (n < N)
        for (int64_t m = r0 + ph; m < r1; m += 4) s += (float)dz[m * N + n];
    red[ph][l] = s;
    __syncthreads();
    if (ph == 0 && n < N) part[(int64_t)blockIdx.x * N + n] = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
}

// grad[off + k n_real + n] = sum_z part[z][k][n] (+ part[z][k + fold][n]) for
// k < k_real, n < n_real (tile [M][N]); fold adds the rows of the low parts
// of the layer-1 inputs, which share the weights of the high parts
__global__ void reduce_w_kernel(const float *__restrict__ part, int splits, int M, int N, int k_real, int n_real,
                                int fold, float *__restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k_real * n_real) return;
    const int k = i / n_real, n = i % n_real;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) {
        s += part[((int64_t)z * M + k) * N + n];
        if (fold) s += part[((int64_t)z * M + k + fold) * N + n];
    }
    grad[i] = s;
}

__global__ void reduce_b_kernel(const float *__restrict__ part, int splits, int N, int n_real, float *__restrict__ grad) {
    const int n = threadIdx.x;
    if (n >= n_real) return;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * N + n];
    grad[n] = s;
}

// Adam (Kingma & Ba 2015, Algorithm 1) with bias correction
// (1 - beta) is formed in FP64 on the host: 1 - 0.999f in FP32 is off by 1.3e-5
__global__ void adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int64_t n, float lr, float b1, float omb1, float b2,
                            float omb2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ----------------------------------------------------------------------------
// workspace layout
// ----------------------------------------------------------------------------
constexpr int kRowsPerSplit = 512;

struct TrainWs {
    TrainWeights w;
    bf16 *x0;                   // [Bp][32]
    float *z[3];                // [Bp][128]
    bf16 *a[3];                 // [Bp][128]
    float *y;                   // [Bp][32]
    bf16 *dz4;                  // [Bp][32]
    bf16 *dz[3];                // [Bp][128]  (dz of hidden layers 1..3)
    float *wpart;               // [splits][128][128]
    float *bpart;               // [Bp / kColRows + 1][128]
    float *lpart;               // [Bp / 256 + 1]
    size_t bytes;
};

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

TrainWs carve(void *base, int64_t B) {
    const int64_t Bp = (B + 31) / 32 * 32;
    const int64_t splits = (Bp + kRowsPerSplit - 1) / kRowsPerSplit;
    TrainWs t;
    char *p = (char *)base;
    size_t o = 0;
    auto take = [&](size_t bytes) { char *r = p ? p + o : nullptr; o += al(bytes); return r; };
    t.w.wt1 = (bf16 *)take(128 * 16 * 2);
    t.w.wt2 = (bf16 *)take(128 * 128 * 2);
    t.w.wt3 = (bf16 *)take(128 * 128 * 2);
    t.w.wt4 = (bf16 *)take(32 * 128 * 2);
    t.w.wn2 = (bf16 *)take(128 * 128 * 2);
    t.w.wn3 = (bf16 *)take(128 * 128 * 2);
    t.w.wn4 = (bf16 *)take(128 * 32 * 2);
    t.w.bias = (float *)take((3 * 128 + 32) * 4);
    t.x0 = (bf16 *)take(Bp * 32 * 2);
    for (int l = 0; l < 3; ++l) t.z[l] = (float *)take(Bp * 128 * 4);
    for (int l = 0; l < 3; ++l) t.a[l] = (bf16 *)take(Bp * 128 * 2);
    t.y = (float *)take(Bp * 32 * 4);
    t.dz4 = (bf16 *)take(Bp * 32 * 2);
    for (int l = 0; l < 3; ++l) t.dz[l] = (bf16 *)take(Bp * 128 * 2);
    t.wpart = (float *)take(splits * 128 * 128 * 4);
    t.bpart = (float *)take((Bp / kColRows + 1) * 128 * 4);
    t.lpart = (float *)take((Bp / 256 + 1) * 4);
    t.bytes = o;
    return t;
}

// forward through the four layers (weights already packed, features in x0)
void forward_layers(const TrainWs &t, int64_t Bp, hipStream_t s) {
    const float *bias = t.w.bias;
    GemmArgs g{};
    g.M = (int)Bp;
    // layer 1: [Bp][16 of 32] x wt1^T
    g.N = 128; g.K = 16; g.k_chunk = 16;
    g.A = t.x0; g.a_m = 32; g.a_k = 1;
    g.B = t.w.wt1; g.b_k = 1; g.b_n = 16;
    g.bias = bias; g.zout = t.z[0]; g.aout = t.a[0];
    gemm<true, true, EPI_HIDDEN>(g, 1, s);
    // layers 2, 3
    const bf16 *wt[2] = {t.w.wt2, t.w.wt3};
    for (int l = 1; l < 3; ++l) {
        g.K = 128; g.k_chunk = 128;
        g.A = t.a[l - 1]; g.a_m = 128;
        g.B = wt[l - 1]; g.b_n = 128;
        g.bias = bias + 128 * l; g.zout = t.z[l]; g.aout = t.a[l];
        gemm<true, true, EPI_HIDDEN>(g, 1, s);
    }
    // layer 4 (output, padded to 32 columns)
    g.N = 32; g.K = 128; g.k_chunk = 128;
    g.A = t.a[2]; g.a_m = 128;
    g.B = t.w.wt4; g.b_n = 128;
    g.bias = bias + 384; g.out = t.y;
    gemm<true, true, EPI_OUT>(g, 1, s);
}

}  // namespace

size_t mlp_workspace(int64_t B) { return carve(nullptr, B).bytes; }

int mlp_forward(const float *params, int64_t B, const float *feats, float *out, void *ws, hipStream_t s) {
    if (B == 0) return SPHBI_OK;
    const int64_t Bp = (B + 31) / 32 * 32;
    TrainWs t = carve(ws, B);
    hipLaunchKernelGGL(pack_kernel, dim3(64), dim3(256), 0, s, params, t.w);
    hipLaunchKernelGGL(feats_kernel, dim3((unsigned)((Bp * 32 + 255) / 256)), dim3(256), 0, s, feats, B, Bp, t.x0);
    forward_layers(t, Bp, s);
    hipError_t e = hipMemcpy2DAsync(out, kOut * sizeof(float), t.y, 32 * sizeof(float), kOut * sizeof(float),
                                    (size_t)B, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) { set_error("mlp forward copy: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    e = hipGetLastError();
    if (e != hipSuccess) { set_error("mlp forward launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

int mlp_loss_grad(const float *params, int64_t B, const float *feats, const float *targets, const float *scale,
                  float lam, float *loss, float *grad, void *ws, hipStream_t s) {
    const int64_t Bp = (B + 31) / 32 * 32;
    const int splits = (int)((Bp + kRowsPerSplit - 1) / kRowsPerSplit);
    TrainWs t = carve(ws, B);
    hipLaunchKernelGGL(pack_kernel, dim3(64), dim3(256), 0, s, params, t.w);
    hipLaunchKernelGGL(feats_kernel, dim3((unsigned)((Bp * 32 + 255) / 256)), dim3(256), 0, s, feats, B, Bp, t.x0);
    forward_layers(t, Bp, s);
    const int lblocks = (int)((Bp + 255) / 256);
    hipLaunchKernelGGL(loss_kernel, dim3(lblocks), dim3(256), 0, s, t.y, targets, B, Bp, scale[0], scale[1], scale[2],
                       lam, t.dz4, t.lpart);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, t.lpart, lblocks, loss);

    // backward, layer 4 -> 1
    const bf16 *dz_top[4] = {t.dz[0], t.dz[1], t.dz[2], t.dz4};
    const int n_of[4] = {128, 128, 128, 32}, nreal[4] = {128, 128, 128, kOut};
    const int k_of[4] = {32, 128, 128, 128}, kreal[4] = {kIn, 128, 128, 128};   // x0 rows are 32 wide
    const bf16 *act_in[4] = {t.x0, t.a[0], t.a[1], t.a[2]};
    const int64_t offw[4] = {kOffW1, kOffW2, kOffW3, kOffW4}, offb[4] = {kOffB1, kOffB2, kOffB3, kOffB4};
    const bf16 *wn[4] = {nullptr, t.w.wn2, t.w.wn3, t.w.wn4};
    for (int l = 3; l >= 0; --l) {
        const int N = n_of[l], K = k_of[l];
        // weight gradient: dW[k][n] = sum_b act_in[b][k] dz[b][n]  (split over the batch)
        GemmArgs g{};
        g.M = K; g.N = N; g.K = (int)Bp; g.k_chunk = kRowsPerSplit;
        g.A = act_in[l]; g.a_m = 1; g.a_k = K;
        g.B = dz_top[l]; g.b_k = N; g.b_n = 1;
        g.out = t.wpart;
        gemm<false, false, EPI_PART>(g, splits, s);
        hipLaunchKernelGGL(reduce_w_kernel, dim3((unsigned)((kreal[l] * nreal[l] + 255) / 256)), dim3(256), 0, s,
                           t.wpart, splits, K, N, kreal[l], nreal[l], l == 0 ? kIn : 0, grad + offw[l]);
        const int csplits = (int)((Bp + kColRows - 1) / kColRows);
        hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)csplits, (unsigned)((N + 63) / 64)), dim3(256), 0, s,
                           dz_top[l], Bp, N, t.bpart);
        hipLaunchKernelGGL(reduce_b_kernel, dim3(1), dim3(128), 0, s, t.bpart, csplits, N, nreal[l], grad + offb[l]);
        if (l == 0) break;
        // input gradient of this layer -> pre-activation gradient of the layer below
        GemmArgs d{};
        d.M = (int)Bp; d.N = 128; d.K = N; d.k_chunk = N;
        d.A = dz_top[l]; d.a_m = N; d.a_k = 1;
        d.B = wn[l]; d.b_k = 1; d.b_n = N;
        d.zin = t.z[l - 1]; d.dzout = t.dz[l - 1];
        gemm<true, true, EPI_BWD>(d, 1, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("mlp backward launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

int adam_step(float *p, float *m, float *v, const float *g, int64_t n, double lr, double b1, double b2, double eps,
              int64_t step, hipStream_t s) {
    if (n == 0) return SPHBI_OK;
    const float c1 = (float)(1.0 - pow(b1, (double)step));
    const float c2 = (float)(1.0 - pow(b2, (double)step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, m, v, g, n, (float)lr,
                       (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("adam launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
