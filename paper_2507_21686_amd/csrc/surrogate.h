// Learned surrogate of the per-pair integrals: shared constants and
// declarations (training kernels in mlp.hip, serving kernel in serve.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sphbi {

typedef __bf16 bf16;

namespace mlp {

constexpr int kIn = 8, kHid = 128, kOut = 4, kOutPad = 32;
// flat FP32 parameter vector: W1[8][128] b1 W2[128][128] b2 W3[128][128] b3 W4[128][4] b4
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + kIn * kHid;
constexpr int64_t kOffW2 = kOffB1 + kHid;
constexpr int64_t kOffB2 = kOffW2 + kHid * kHid;
constexpr int64_t kOffW3 = kOffB2 + kHid;
constexpr int64_t kOffB3 = kOffW3 + kHid * kHid;
constexpr int64_t kOffW4 = kOffB3 + kHid;
constexpr int64_t kOffB4 = kOffW4 + kHid * kOut;
constexpr int64_t kParams = kOffB4 + kOut;
static_assert(kParams == SPHBI_MLP_PARAMS, "parameter count");

// floor of the indicator target log10(err + floor)
constexpr float kErrFloor = 1e-7f;

// activation between layers: a piecewise quadratic stand-in for z sigmoid(z),
//   act(z) = z s(u),  s(u) = 1/2 + u/4 - u|u|/32,  u = clamp(z, -4, 4),
// continuously differentiable (s rises from 0 to 1 with zero slope at both
// ends); four FP32 operations and no transcendental.  The clamp is the
// hardware median of three: fminf/fmaxf would first quiet signalling NaNs
// with one more instruction per value (the network never produces them).
__device__ inline float act(float z) {
    const float u = __builtin_amdgcn_fmed3f(z, -4.0f, 4.0f);
    return z * fmaf(u, fmaf(fabsf(u), -0.03125f, 0.25f), 0.5f);
}
__device__ inline float act_grad(float z) {
    if (z >= 4.0f) return 1.0f;
    if (z <= -4.0f) return 0.0f;
    return fmaf(z, fmaf(fabsf(z), -0.09375f, 0.5f), 0.5f);
}

// bfloat16 operand copies of the weights for the training products
struct TrainWeights {
    bf16 *wt1, *wt2, *wt3, *wt4;    // transposed [out][in] (input padded to 16 / output padded to 32)
    bf16 *wn2, *wn3, *wn4;          // [in][out] (output of layer 4 padded to 32)
    float *bias;                    // [128 | 128 | 128 | 32]
};

}  // namespace mlp

// standardisation of the outputs and range of the trained features
struct SurrogateStats {
    float mean[3], stdev[3];
    float fmax;
};

struct KArgs;

size_t mlp_workspace(int64_t B);
int mlp_forward(const float *params, int64_t B, const float *feats, float *out, void *ws, hipStream_t s);
int mlp_loss_grad(const float *params, int64_t B, const float *feats, const float *targets, const float *scale,
                  float lam, float *loss, float *grad, void *ws, hipStream_t s);
int adam_step(float *p, float *m, float *v, const float *g, int64_t n, double lr, double b1, double b2, double eps,
              int64_t step, hipStream_t s);

size_t surrogate_model_bytes();
size_t surrogate_workspace(int64_t T, int64_t P);
int surrogate_pack(const float *params, const SurrogateStats &st, void *model, hipStream_t s);
int surrogate_features(double h, int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                       const int64_t *off, const int32_t *tri_idx, int64_t P, float *feats, float *rot,
                       hipStream_t s);
int surrogate_targets(int64_t P, double h, const double *pp, const float *rot, const SurrogateStats &st, float *out,
                      hipStream_t s);
int surrogate_integrate(const KArgs &K, int deg, double h, int64_t N, const double *px, const double *py, int64_t T,
                        const double *tri, const double *nodal, const int64_t *off, const int32_t *tri_idx, int64_t P,
                        const void *model, float threshold, double *I, double *Gx, double *Gy, double *per_pair,
                        uint8_t *flags, int64_t *n_flagged, void *ws, hipStream_t s);

}  // namespace sphbi
