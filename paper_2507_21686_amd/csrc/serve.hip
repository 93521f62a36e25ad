// Learned surrogate of the per-pair integrals: feature extraction, the fused
// serving kernel, the router and the analytic fallback.
//
// Serving path for a P0 field (constant value A per triangle) and the kernel
// the network was trained on:
//   1. serve_kernel: a wavefront owns 64 consecutive particles and sweeps
//      their CSR pair range 64 pairs at a time (one pair per lane).  Each
//      lane builds its pair's canonical features; the wavefront then runs
//      the network on the matrix cores for its 64 pairs (two blocks of 32
//      pairs, v_mfma_f32_32x32x16_bf16 with the weights resident in LDS).
//      The output of one layer is the B operand of the next without any
//      transpose: the k index of every layer is permuted (in the packed
//      weights) to the order in which the accumulator lanes hold the
//      previous layer's outputs.  A pair is flagged when its indicator
//      output exceeds the threshold or a feature lies outside the trained
//      range; unflagged pairs are rotated back, scaled by A and 1/h, and
//      summed per particle by a segmented wave scan.
//   2. the flagged pairs are compacted in pair order;
//   3. fallback_kernel evaluates them with the closed form (FP64);
//   4. merge_kernel adds each particle's fallback pairs, in pair order, to
//      its sums (one thread per run of a particle, so the result is
//      deterministic without atomics).

#include <rocprim/device/device_select.hpp>
#include <math.h>

#include "features.h"
#include "internal.h"
#include "pairmath.h"
#include "surrogate.h"

namespace sphbi {
namespace {

using namespace mlp;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ----------------------------------------------------------------------------
// packed model (device memory, written by pack_model_kernel)
// ----------------------------------------------------------------------------
// k order of the B operand of layers 2-4: at k-step s (16 inputs), lane l
// holds the eight inputs f(s, l / 32, j), j = 0..7, which are the outputs
// the previous layer's accumulator tile (s / 2) holds in lane l at register
// 8 (s % 2) + j.
__host__ __device__ constexpr int kperm(int s, int hl, int j) {
    return 32 * (s >> 1) + 16 * (s & 1) + 8 * (j >> 2) + 4 * hl + (j & 3);
}

struct Model {
    bf16 w1[4][64][8];           // layer 1: [out tile][lane][j]
    bf16 w2[4][8][64][8];        // layer 2: [out tile][k-step][lane][j]
    bf16 w3[4][8][64][8];
    bf16 w4[8][64][8];           // layer 4: one out tile (4 of 32 rows used)
    float b1[128], b2[128], b3[128], b4[4];
    float mean[3], stdev[3];
    float fmax;                  // |features 0-5| beyond this are outside the trained range
    float pad[5];
};
static_assert(sizeof(Model) % 16 == 0, "model size");

__global__ void pack_model_kernel(const float *__restrict__ p, SurrogateStats st, Model *__restrict__ m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;     // one (tile, k-step, lane) per thread
    if (i < 4 * 64) {       // lanes 32-63 carry the low parts of the features: same weights
        const int ob = i / 64, l = i % 64;
        for (int j = 0; j < 8; ++j) m->w1[ob][l][j] = (bf16)p[kOffW1 + j * kHid + 32 * ob + (l & 31)];
    }
    if (i < 4 * 8 * 64) {
        const int ob = i / 512, s = (i / 64) % 8, l = i % 64;
        for (int j = 0; j < 8; ++j) {
            const int k = kperm(s, l >> 5, j), n = 32 * ob + (l & 31);
            m->w2[ob][s][l][j] = (bf16)p[kOffW2 + k * kHid + n];
            m->w3[ob][s][l][j] = (bf16)p[kOffW3 + k * kHid + n];
        }
    }
    if (i < 8 * 64) {
        const int s = i / 64, l = i % 64;
        for (int j = 0; j < 8; ++j) {
            const int k = kperm(s, l >> 5, j), n = l & 31;
            m->w4[s][l][j] = (bf16)(n < kOut ? p[kOffW4 + k * kOut + n] : 0.0f);
        }
    }
    if (i < 128) {
        m->b1[i] = p[kOffB1 + i];
        m->b2[i] = p[kOffB2 + i];
        m->b3[i] = p[kOffB3 + i];
    }
    if (i < kOut) m->b4[i] = p[kOffB4 + i];
    if (i < 3) {
        m->mean[i] = st.mean[i];
        m->stdev[i] = st.stdev[i];
    }
    if (i == 0) {
        m->fmax = st.fmax;
        for (int k = 0; k < 5; ++k) m->pad[k] = 0.0f;
    }
}

// ----------------------------------------------------------------------------
// features of every pair (training data and tests)
// ----------------------------------------------------------------------------
__global__ void features_kernel(int64_t N, const double *__restrict__ px, const double *__restrict__ py,
                                int64_t T, const double *__restrict__ tri, const int64_t *__restrict__ off,
                                const int32_t *__restrict__ tri_idx, int64_t P, double invh, float *__restrict__ feats,
                                float *__restrict__ rot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t q0 = min(max(off[i], (int64_t)0), P), q1 = min(max(off[i + 1], q0), P);
    for (int64_t q = q0; q < q1; ++q) {
        const int32_t t = tri_idx[q];
        float f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        double c = 1.0, s = 0.0;
        if (t >= 0 && t < T) {
            double v[6];
            for (int k = 0; k < 6; ++k) v[k] = tri[k * T + t];
            pair_features(px[i], py[i], v, invh, f, c, s);
        }
        for (int k = 0; k < 8; ++k) feats[q * 8 + k] = f[k];
        rot[q * 2] = (float)c;
        rot[q * 2 + 1] = (float)s;
    }
}

// closed-form per-pair values [3][P] -> standardised targets [P][3] of the
// rotated frame: (I, h Gx', h Gy') with (Gx', Gy') = R(-theta) (Gx, Gy)
__global__ void targets_kernel(int64_t P, double h, const double *__restrict__ pp, const float *__restrict__ rot,
                               SurrogateStats st, float *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    const double c = rot[2 * q], s = rot[2 * q + 1];
    const double gx = pp[P + q] * h, gy = pp[2 * P + q] * h;
    const double v[3] = {pp[q], c * gx + s * gy, c * gy - s * gx};
    for (int k = 0; k < 3; ++k) out[3 * q + k] = (float)((v[k] - st.mean[k]) / st.stdev[k]);
}

// ----------------------------------------------------------------------------
// fused serving kernel
// ----------------------------------------------------------------------------
// 256 threads, two waves per SIMD: the model (79 KB of LDS) fits twice in a
// CU's 160 KB and the kernel in 256 registers without spilling
constexpr int kServeThreads = 256;

__device__ inline bf16x8 pack8(const f32x16 &a, int half) {
    bf16x8 r;
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = (bf16)act(a[8 * half + j]);
    return r;
}

// acc[r] <- bias of output 32 ob + 8 (r / 4) + 4 (lane / 32) + r % 4
__device__ inline f32x16 bias_tile(const float *b, int ob, int lane) {
    f32x16 a;
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = b[32 * ob + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)];
    return a;
}

// one hidden 128 -> 128 layer: B operands in, B operands of the next layer out
__device__ inline void hidden_layer(const bf16 (*w)[8][64][8], const float *b, const bf16x8 (&in)[8][2],
                                    bf16x8 (&out)[8][2], int lane) {
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x16 acc0 = bias_tile(b, ob, lane), acc1 = acc0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&w[ob][s][lane][0]);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, in[s][0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, in[s][1], acc1, 0, 0, 0);
            if (s == 3) __builtin_amdgcn_sched_barrier(0);
        }
        out[2 * ob][0] = pack8(acc0, 0);
        out[2 * ob + 1][0] = pack8(acc0, 1);
        out[2 * ob][1] = pack8(acc1, 0);
        out[2 * ob + 1][1] = pack8(acc1, 1);
        // keep the next tile's weight loads from being hoisted here (they
        // would hold 32 more registers each)
        __builtin_amdgcn_sched_barrier(0);
    }
}

__global__ __launch_bounds__(kServeThreads, 2) void serve_kernel(
    const Model *__restrict__ model, double invh, float threshold, int64_t N, const double *__restrict__ px,
    const double *__restrict__ py, int64_t T, const double *__restrict__ tri, const double *__restrict__ nodal,
    const int64_t *__restrict__ off, const int32_t *__restrict__ tri_idx, int64_t P, double *__restrict__ I,
    double *__restrict__ Gx, double *__restrict__ Gy, double *__restrict__ per_pair, uint8_t *__restrict__ flags) {
    __shared__ Model sm;
    {   // stage the packed model in LDS (16-byte copies)
        const uint4 *src = reinterpret_cast<const uint4 *>(model);
        uint4 *dst = reinterpret_cast<uint4 *>(&sm);
        for (int i = threadIdx.x; i < (int)(sizeof(Model) / 16); i += kServeThreads) dst[i] = src[i];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int64_t n_waves = (N + 63) / 64;
    const int64_t waves_per_grid = (int64_t)gridDim.x * (kServeThreads / 64);
    for (int64_t wv = (int64_t)blockIdx.x * (kServeThreads / 64) + (threadIdx.x >> 6); wv < n_waves;
         wv += waves_per_grid) {
        const int64_t p0 = wv * 64;
        const int64_t pid = p0 + lane;
        const int64_t plast = p0 + 64 < N ? p0 + 64 : N;
        const int64_t q_end = min(max(off[plast], (int64_t)0), P);
        const int64_t my_off = pid < N ? min(max(off[pid], (int64_t)0), q_end) : q_end;
        const int64_t my_end = pid < N ? min(max(off[pid + 1], my_off), q_end) : q_end;
        const int64_t q_begin = __shfl(my_off, 0);
        double accI = 0.0, accX = 0.0, accY = 0.0;        // per-particle sums in FP64
        for (int64_t base = q_begin; base < q_end; base += 64) {
            const int64_t q = base + lane;
            const int64_t qq = q < q_end ? q : q_end - 1;
            int lo = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int64_t om = __shfl(my_off, lo + step < 64 ? lo + step : 63);
                if (lo + step < 64 && om <= qq) lo += step;
            }
            const int owner = lo;
            const int64_t ip = p0 + owner < N ? p0 + owner : N - 1;
            // features of this lane's pair; the rotation and the field value are
            // kept in FP32, which is ample at the network's accuracy
            float f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            float cf = 1.0f, sf = 0.0f, Af = 0.0f;
            bool valid = false;
            if (q < q_end) {
                const int32_t t = tri_idx[q];
                if (t >= 0 && t < T) {
                    double v[6], c, s;
#pragma unroll
                    for (int k = 0; k < 6; ++k) v[k] = tri[k * T + t];
                    pair_features(px[ip], py[ip], v, invh, f, c, s);
                    cf = (float)c;
                    sf = (float)s;
                    Af = (float)nodal[t];
                    valid = true;
                }
            }
            bool inrange = valid;
#pragma unroll
            for (int k = 0; k < 6; ++k) inrange = inrange && fabsf(f[k]) <= sm.fmax;
            // layer 1 operands: pair block 0 = the pairs of lanes 0-31, block 1 =
            // those of lanes 32-63; k slots 0-7 (lanes 0-31) take the bfloat16
            // high parts of the features, slots 8-15 (lanes 32-63) the low parts
            bf16x8 x0, x1;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float other = __shfl_xor(f[j], 32);
                const float v0 = lane < 32 ? f[j] : other;      // feature of the block-0 pair
                const float v1 = lane < 32 ? other : f[j];      // feature of the block-1 pair
                const bf16 h0 = (bf16)v0, h1 = (bf16)v1;
                x0[j] = lane < 32 ? h0 : (bf16)(v0 - (float)h0);
                x1[j] = lane < 32 ? h1 : (bf16)(v1 - (float)h1);
            }
            bf16x8 h1[8][2], h2[8][2];
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&sm.w1[ob][lane][0]);
                f32x16 acc0 = bias_tile(sm.b1, ob, lane), acc1 = acc0;
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, x0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, x1, acc1, 0, 0, 0);
                h1[2 * ob][0] = pack8(acc0, 0);
                h1[2 * ob + 1][0] = pack8(acc0, 1);
                h1[2 * ob][1] = pack8(acc1, 0);
                h1[2 * ob + 1][1] = pack8(acc1, 1);
            }
            hidden_layer(sm.w2, sm.b2, h1, h2, lane);
            hidden_layer(sm.w3, sm.b3, h2, h1, lane);
            // output layer: rows 0-3 of one tile; lanes 0-31 hold the four outputs of pair (block, lane)
            f32x16 o0 = {}, o1 = {};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float bb = lane < 32 ? sm.b4[r] : 0.0f;
                o0[r] = bb;
                o1[r] = bb;
            }
#pragma unroll
            for (int st = 0; st < 8; ++st) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&sm.w4[st][lane][0]);
                o0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, h1[st][0], o0, 0, 0, 0);
                o1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, h1[st][1], o1, 0, 0, 0);
            }
            float y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float from_low = __shfl(o1[r], lane & 31);    // block 1 results live in lanes 0-31
                y[r] = lane < 32 ? o0[r] : from_low;
            }
            // router and de-standardisation
            const bool ok = inrange && y[3] <= threshold;
            double vI = 0.0, vX = 0.0, vY = 0.0;           // the pair's values: FP32 network outputs, summed in FP64
            if (ok) {
                const float i0 = y[0] * sm.stdev[0] + sm.mean[0];
                const float g1 = y[1] * sm.stdev[1] + sm.mean[1];
                const float g2 = y[2] * sm.stdev[2] + sm.mean[2];
                const float ah = Af * (float)invh;
                vI = (double)(Af * i0);
                vX = (double)(ah * (cf * g1 - sf * g2));
                vY = (double)(ah * (sf * g1 + cf * g2));
            }
            if (q < q_end) {
                flags[q] = (uint8_t)(valid && !ok);
                if (per_pair) {
                    per_pair[q] = vI;
                    per_pair[P + q] = vX;
                    per_pair[2 * P + q] = vY;
                }
            }
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const double uI = __shfl_up(vI, d), uX = __shfl_up(vX, d), uY = __shfl_up(vY, d);
                const int uo = __shfl_up(owner, d);
                if (lane >= d && uo == owner) {
                    vI += uI;
                    vX += uX;
                    vY += uY;
                }
            }
            const int64_t s0 = my_off > base ? my_off : base;
            const int64_t s1 = my_end < base + 64 ? my_end : base + 64;
            const int src = s1 > s0 ? (int)(s1 - 1 - base) : 0;
            const double rI = __shfl(vI, src), rX = __shfl(vX, src), rY = __shfl(vY, src);
            if (s1 > s0) {
                accI += rI;
                accX += rX;
                accY += rY;
            }
        }
        if (pid < N) {
            I[pid] = accI;
            Gx[pid] = accX;
            Gy[pid] = accY;
        }
    }
}

// ----------------------------------------------------------------------------
// analytic fallback for the flagged pairs
// ----------------------------------------------------------------------------
__device__ inline int64_t owner_of(const int64_t *off, int64_t N, int64_t q) {
    int64_t lo = 0, hi = N;          // largest i with off[i] <= q
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (off[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int DEG>
__global__ void fallback_kernel(const KArgs K, double invh, int64_t N, const double *__restrict__ px,
                                const double *__restrict__ py, int64_t T, const double *__restrict__ rec,
                                const int64_t *__restrict__ off, const int32_t *__restrict__ tri_idx,
                                const int64_t *__restrict__ list, const int64_t *__restrict__ count,
                                int64_t *__restrict__ owner, double *__restrict__ res, double *__restrict__ per_pair,
                                int64_t P) {
    const int64_t n = *count;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = list[j];
        const int64_t i = owner_of(off, N, q);
        const int32_t t = tri_idx[q];
        double vI = 0.0, vX = 0.0, vY = 0.0;
        if (t >= 0 && t < T)
            pair_fwd<DEG, 0, double>(K, ExactMath(), 0.0, px[i], py[i], invh, rec + (int64_t)t * kRecDoubles, vI,
                                     vX, vY);
        owner[j] = i;
        res[j] = vI;
        res[P + j] = vX;
        res[2 * P + j] = vY;
        if (per_pair) {
            per_pair[q] = vI;
            per_pair[P + q] = vX;
            per_pair[2 * P + q] = vY;
        }
    }
}

// first entry of each particle's run adds the run, in list order
__global__ void merge_kernel(const int64_t *__restrict__ count, const int64_t *__restrict__ owner,
                             const double *__restrict__ res, int64_t P, double *__restrict__ I,
                             double *__restrict__ Gx, double *__restrict__ Gy) {
    const int64_t n = *count;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = owner[j];
        if (j > 0 && owner[j - 1] == i) continue;
        double sI = 0.0, sX = 0.0, sY = 0.0;
        for (int64_t k = j; k < n && owner[k] == i; ++k) {
            sI += res[k];
            sX += res[P + k];
            sY += res[2 * P + k];
        }
        I[i] += sI;
        Gx[i] += sX;
        Gy[i] += sY;
    }
}

__global__ void iota64_kernel(int64_t n, int64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = i;
}

// Clears the routing flags (the serving kernel writes only the pairs of the
// particles' CSR range [offsets[0], offsets[N]); the rest must read as "not
// flagged") and the flagged count.  A kernel rather than a memset, so that a
// captured graph replays it like any other node.
__global__ void clear_flags_kernel(int64_t n, uint8_t *__restrict__ flags, int64_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = 0;
    if (i == 0 && count) *count = 0;
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct ServeWs {
    double *rec;            // [T][16] field records
    int64_t *iota;          // [P]
    int64_t *list;          // [P] flagged pair indices
    int64_t *count;         // [1]
    int64_t *owner;         // [P]
    double *res;            // [3][P]
    void *cub;
    size_t cub_bytes;
    size_t bytes;
};

ServeWs carve_serve(void *base, int64_t T, int64_t P) {
    ServeWs w;
    size_t cub_bytes = 0;
    // size query only (no device work); a failure leaves cub_bytes at 0 and
    // the compaction call reports it
    (void)rocprim::select(nullptr, cub_bytes, (int64_t *)nullptr, (uint8_t *)nullptr, (int64_t *)nullptr,
                          (int64_t *)nullptr, (size_t)(P > 0 ? P : 1));
    char *p = (char *)base;
    size_t o = 0;
    auto take = [&](size_t bytes) { char *r = p ? p + o : nullptr; o += al(bytes); return r; };
    w.rec = (double *)take((size_t)T * kRecDoubles * 8);
    w.iota = (int64_t *)take((size_t)P * 8);
    w.list = (int64_t *)take((size_t)P * 8);
    w.count = (int64_t *)take(8);
    w.owner = (int64_t *)take((size_t)P * 8);
    w.res = (double *)take((size_t)P * 3 * 8);
    w.cub = take(cub_bytes);
    w.cub_bytes = cub_bytes;
    w.bytes = o;
    return w;
}

}  // namespace

size_t surrogate_model_bytes() { return sizeof(Model); }

size_t surrogate_workspace(int64_t T, int64_t P) { return carve_serve(nullptr, T, P).bytes; }

int surrogate_pack(const float *params, const SurrogateStats &st, void *model, hipStream_t s) {
    hipLaunchKernelGGL(pack_model_kernel, dim3(8), dim3(256), 0, s, params, st, (Model *)model);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("surrogate pack launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

int surrogate_features(double h, int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                       const int64_t *off, const int32_t *tri_idx, int64_t P, float *feats, float *rot,
                       hipStream_t s) {
    if (N == 0) return SPHBI_OK;
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, px, py, T, tri, off,
                       tri_idx, P, 1.0 / h, feats, rot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("features launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

int surrogate_targets(int64_t P, double h, const double *pp, const float *rot, const SurrogateStats &st, float *out,
                      hipStream_t s) {
    if (P == 0) return SPHBI_OK;
    hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, P, h, pp, rot, st, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("targets launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

int surrogate_integrate(const KArgs &K, int deg, double h, int64_t N, const double *px, const double *py, int64_t T,
                        const double *tri, const double *nodal, const int64_t *off, const int32_t *tri_idx, int64_t P,
                        const void *model, float threshold, double *I, double *Gx, double *Gy, double *per_pair,
                        uint8_t *flags, int64_t *n_flagged, void *ws, hipStream_t s) {
    if (N == 0) return SPHBI_OK;
    ServeWs w = carve_serve(ws, T, P);
    const double invh = 1.0 / h;
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
        n_cu = 256;
    const int64_t n_waves = (N + 63) / 64;
    const int64_t want = (n_waves + kServeThreads / 64 - 1) / (kServeThreads / 64);
    const unsigned grid = (unsigned)(want < (int64_t)n_cu * 2 ? want : (int64_t)n_cu * 2);
    hipLaunchKernelGGL(clear_flags_kernel, dim3((unsigned)((P + 255) / 256 > 0 ? (P + 255) / 256 : 1)), dim3(256), 0,
                       s, P, flags, n_flagged);
    hipLaunchKernelGGL(serve_kernel, dim3(grid), dim3(kServeThreads), 0, s, (const Model *)model, invh, threshold, N,
                       px, py, T, tri, nodal, off, tri_idx, P, I, Gx, Gy, per_pair, flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("serve launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    if (P == 0) return SPHBI_OK;
    // compact the flagged pairs (pair order)
    hipLaunchKernelGGL(iota64_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, P, w.iota);
    size_t cb = w.cub_bytes;
    e = rocprim::select(w.cub, cb, w.iota, flags, w.list, w.count, (size_t)P, s);
    if (e != hipSuccess) { set_error("flag compaction: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    // field records for the fallback (P0: vertices + value)
    int rc = launch_prepare(0, T, tri, nodal, h, w.rec, s);
    if (rc) return rc;
    const int64_t fb_want = (P + 255) / 256;
    const unsigned fb_grid = (unsigned)(fb_want < (int64_t)n_cu * 8 ? fb_want : (int64_t)n_cu * 8);
    if (deg <= 3)
        hipLaunchKernelGGL(fallback_kernel<3>, dim3(fb_grid), dim3(256), 0, s, K, invh, N, px, py, T, w.rec, off,
                           tri_idx, w.list, w.count, w.owner, w.res, per_pair, P);
    else if (deg <= 5)
        hipLaunchKernelGGL(fallback_kernel<5>, dim3(fb_grid), dim3(256), 0, s, K, invh, N, px, py, T, w.rec, off,
                           tri_idx, w.list, w.count, w.owner, w.res, per_pair, P);
    else if (deg <= 8)
        hipLaunchKernelGGL(fallback_kernel<8>, dim3(fb_grid), dim3(256), 0, s, K, invh, N, px, py, T, w.rec, off,
                           tri_idx, w.list, w.count, w.owner, w.res, per_pair, P);
    else
        hipLaunchKernelGGL(fallback_kernel<11>, dim3(fb_grid), dim3(256), 0, s, K, invh, N, px, py, T, w.rec, off,
                           tri_idx, w.list, w.count, w.owner, w.res, per_pair, P);
    hipLaunchKernelGGL(merge_kernel, dim3(fb_grid), dim3(256), 0, s, w.count, w.owner, w.res, P, I, Gx, Gy);
    e = hipMemcpyAsync(n_flagged, w.count, sizeof(int64_t), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) { set_error("fallback launch: %s", hipGetErrorString(e)); return SPHBI_EDEVICE; }
    return SPHBI_OK;
}

}  // namespace sphbi
