// Fused Adam step over all parameter groups of the Gaussian set in one
// launch: the gradient-descent optimisation of Sec. III-B with the default
// 3DGS optimiser configuration adopted in Sec. IV-A.  The step is purely
// HBM-bound (read p, g, m, v; write p, m, v: 28 bytes per scalar), so each
// thread streams float4 vectors and the bias corrections are formed once per
// workgroup from the device-resident step counter.
#include <cmath>
#include <string>

#include "gs_internal.h"

namespace gs {

constexpr int kAdamThreads = 256;
constexpr int kAdamVec = 4;

struct AdamTable {
  float* p[GS_MAX_ADAM_GROUPS];
  float* g[GS_MAX_ADAM_GROUPS];
  float* m[GS_MAX_ADAM_GROUPS];
  float* v[GS_MAX_ADAM_GROUPS];
  int64_t n[GS_MAX_ADAM_GROUPS];
  float lr[GS_MAX_ADAM_GROUPS];
  int64_t blk_off[GS_MAX_ADAM_GROUPS + 1];
  int32_t n_groups;
};


__global__ __launch_bounds__(kAdamThreads) void k_adam(AdamTable t, AdamCoef c, const int32_t* __restrict__ d_step,
                                                       int zero_grad) {
  __shared__ float s_k[2];
  if (threadIdx.x == 0) adam_bias_factors(c, *d_step, s_k[0], s_k[1]);
  __syncthreads();
  const int64_t b = blockIdx.x;
  int gi = 0;
#pragma unroll 1
  for (int k = 1; k < t.n_groups; ++k)
    if (t.blk_off[k] <= b) gi = k;
  const int64_t n = t.n[gi];
  const int64_t e0 = ((b - t.blk_off[gi]) * kAdamThreads + threadIdx.x) * kAdamVec;
  if (e0 >= n) return;
  float* P = t.p[gi];
  float* G = t.g[gi];
  float* M = t.m[gi];
  float* V = t.v[gi];
  const float step_size = t.lr[gi] * s_k[0];
  const float isb = s_k[1];
  const bool vec = e0 + kAdamVec <= n && ((reinterpret_cast<uintptr_t>(P) | reinterpret_cast<uintptr_t>(G) |
                                           reinterpret_cast<uintptr_t>(M) | reinterpret_cast<uintptr_t>(V)) &
                                          15) == 0;
  if (vec) {
    float4 p = *reinterpret_cast<float4*>(P + e0);
    float4 g = *reinterpret_cast<float4*>(G + e0);
    float4 m = *reinterpret_cast<float4*>(M + e0);
    float4 v = *reinterpret_cast<float4*>(V + e0);
    adam_update(p.x, g.x, m.x, v.x, c, step_size, isb);
    adam_update(p.y, g.y, m.y, v.y, c, step_size, isb);
    adam_update(p.z, g.z, m.z, v.z, c, step_size, isb);
    adam_update(p.w, g.w, m.w, v.w, c, step_size, isb);
    *reinterpret_cast<float4*>(P + e0) = p;
    *reinterpret_cast<float4*>(M + e0) = m;
    *reinterpret_cast<float4*>(V + e0) = v;
    if (zero_grad) *reinterpret_cast<float4*>(G + e0) = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    for (int64_t e = e0; e < n && e < e0 + kAdamVec; ++e) {
      float p = P[e], g = G[e], m = M[e], v = V[e];
      adam_update(p, g, m, v, c, step_size, isb);
      P[e] = p;
      M[e] = m;
      V[e] = v;
      if (zero_grad) G[e] = 0.0f;
    }
  }
}

__global__ void k_step_increment(int32_t* d_step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *d_step += 1;
}

void launch_step_increment(int32_t* d_step, hipStream_t st) {
  hipLaunchKernelGGL(k_step_increment, dim3(1), dim3(64), 0, st, d_step);
}

AdamCoef make_adam_coef(double beta1, double beta2, double eps) {
  return AdamCoef{beta1, beta2, (float)beta1, (float)beta2, (float)(1.0 - beta1), (float)(1.0 - beta2), (float)eps};
}

gs_status validate_adam_hyper(double beta1, double beta2, double eps, const int32_t* d_step) {
  if (!d_step) return fail(GS_ERR_INVALID_VALUE, "d_step is NULL");
  if (!(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps >= 0) || !std::isfinite(eps))
    return fail(GS_ERR_INVALID_VALUE, "need 0 <= beta < 1 and eps >= 0");
  return GS_OK;
}

}  // namespace gs

extern "C" gs_status gs_adam_step(const gs_adam_group* groups, int32_t n_groups, double beta1, double beta2,
                                  double eps, int32_t* d_step, int32_t zero_grad, void* stream) {
  using namespace gs;
  if (!groups || n_groups < 1 || n_groups > GS_MAX_ADAM_GROUPS)
    return fail(GS_ERR_INVALID_VALUE, "n_groups must be in [1, " + std::to_string(GS_MAX_ADAM_GROUPS) + "]");
  gs_status s;
  if ((s = validate_adam_hyper(beta1, beta2, eps, d_step)) != GS_OK) return s;
  AdamTable t{};
  t.n_groups = n_groups;
  int64_t blocks = 0;
  for (int k = 0; k < n_groups; ++k) {
    const gs_adam_group& g = groups[k];
    if (g.numel < 0) return fail(GS_ERR_INVALID_VALUE, "group " + std::to_string(k) + ": numel < 0");
    if (g.numel > 0 && (!g.param || !g.grad || !g.exp_avg || !g.exp_avg_sq))
      return fail(GS_ERR_INVALID_VALUE, "group " + std::to_string(k) + ": NULL pointer");
    if (!std::isfinite(g.lr)) return fail(GS_ERR_INVALID_VALUE, "group " + std::to_string(k) + ": lr not finite");
    t.p[k] = g.param;
    t.g[k] = g.grad;
    t.m[k] = g.exp_avg;
    t.v[k] = g.exp_avg_sq;
    t.n[k] = g.numel;
    t.lr[k] = g.lr;
    t.blk_off[k] = blocks;
    blocks += (g.numel + (int64_t)kAdamThreads * kAdamVec - 1) / ((int64_t)kAdamThreads * kAdamVec);
  }
  t.blk_off[n_groups] = blocks;
  const AdamCoef c = make_adam_coef(beta1, beta2, eps);
  hipStream_t st = as_stream(stream);
  if (blocks > 0)
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(kAdamThreads), 0, st, t, c, d_step, zero_grad);
  launch_step_increment(d_step, st);
  return check_launch("adam");
}
