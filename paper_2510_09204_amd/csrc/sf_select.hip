// Candidate selection around the SF (the trajectory-planning pipeline of the
// paper's "Validation and Benchmarking" section, the three-stage figure and
// "Qualitative Validation"): sampled candidates are ranked by their primal
// residual (eq. primal_residual), the best few are refined by the SF, and the
// refined candidate chosen is the feasible one with the least smoothness cost
// (the squared acceleration norm summed over time steps, averaged over
// robots: the "Smoothness Cost" metric of "Implementation Details").
//
// Kernels: the smoothness cost of every problem of a plan (one workgroup per
// problem, acceleration basis from the workspace), the k smallest residuals
// (exact ranks by counting), the best candidate (a lexicographic arg-min) and
// a gather of equal-size coefficient blocks.  Every reduction is in a fixed
// order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "sf_internal.h"

namespace sf {
namespace {

constexpr int kSelThreads = 1024;
constexpr int kSmoothThreads = 256;

// Ranking key of a residual row (||r_1||, ||r_2||, ., status): ||r||^2 with
// each operation rounded separately (no contraction), +inf for a flagged or
// non-finite row.
__device__ __forceinline__ float residual_key(const float* __restrict__ row) {
  const float r1 = row[0], r2 = row[1];
  const float k = __fadd_rn(__fmul_rn(r1, r1), __fmul_rn(r2, r2));
  return (row[3] != 0.f || !(k <= 3.40282347e+38f)) ? __builtin_inff() : k;
}

// (key_a, a) before (key_b, b): smaller key, then smaller index.
__device__ __forceinline__ bool key_before(float ka, int a, float kb, int b) {
  return ka < kb || (ka == kb && a < b);
}

__global__ __launch_bounds__(kSelThreads) void topk_kernel(const float* __restrict__ residual,
                                                           int B, int k,
                                                           int32_t* __restrict__ idx) {
  extern __shared__ float keys[];
  for (int b = threadIdx.x; b < B; b += kSelThreads) keys[b] = residual_key(residual + 4 * b);
  __syncthreads();
  for (int b = threadIdx.x; b < B; b += kSelThreads) {
    const float kb = keys[b];
    int rank = 0;
    for (int j = 0; j < B; ++j) rank += key_before(keys[j], j, kb, b) ? 1 : 0;
    if (rank < k) idx[rank] = b;
  }
}

// Best candidate: feasible (key <= tol^2) first; among feasible the least
// cost, then the least key; otherwise the least key; then the least index.
struct Cand {
  int infeasible;
  float primary, key;
  int index;
};
__device__ __forceinline__ bool cand_before(const Cand& a, const Cand& b) {
  if (a.infeasible != b.infeasible) return a.infeasible < b.infeasible;
  if (a.primary != b.primary) return a.primary < b.primary;
  if (a.key != b.key) return a.key < b.key;
  return a.index < b.index;
}

__global__ __launch_bounds__(kSelThreads) void best_kernel(const float* __restrict__ residual,
                                                           const float* __restrict__ cost, int B,
                                                           float tol, int32_t* __restrict__ idx) {
  __shared__ Cand red[kSelThreads];
  const float tol2 = __fmul_rn(tol, tol);
  Cand best{2, __builtin_inff(), __builtin_inff(), 0x7fffffff};
  for (int b = threadIdx.x; b < B; b += kSelThreads) {
    const float key = residual_key(residual + 4 * b);
    const float c = cost[b];
    Cand x;
    x.infeasible = key <= tol2 ? 0 : 1;
    x.primary = x.infeasible ? key : ((c <= 3.40282347e+38f) ? c : __builtin_inff());
    x.key = key;
    x.index = b;
    if (cand_before(x, best)) best = x;
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = kSelThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w && cand_before(red[threadIdx.x + w], red[threadIdx.x]))
      red[threadIdx.x] = red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) idx[0] = red[0].index;
}

// Smoothness cost of problem blockIdx.x: (1/n) sum_i sum_k |Wdd_k xi_i|^2
// scaled by inv_tf4 (Wdd is the second tau-derivative of the basis; the time
// derivative is 1/t_f^2 of it).  Thread t takes the (row, k) items t, t + NT,
// ... of the 2n x T products, so every sum has a fixed order.
__global__ __launch_bounds__(kSmoothThreads) void smoothness_kernel(
    const ProbDesc* __restrict__ probs, const float* __restrict__ Wdd,
    const float* __restrict__ xi, int nc, int T, float inv_tf4, float* __restrict__ cost) {
  __shared__ float red[kSmoothThreads];
  const ProbDesc P = probs[blockIdx.x];
  const int rows = 2 * P.n;
  const float* x = xi + P.coef_off;
  float s = 0.f;
  for (int it = threadIdx.x; it < rows * T; it += kSmoothThreads) {
    const int r = it / T, k = it - r * T;
    const float* wk = Wdd + (size_t)k * nc;
    const float* xr = x + (size_t)r * nc;
    float acc = 0.f;
    for (int c = 0; c < nc; ++c) acc = fmaf(wk[c], xr[c], acc);
    s = fmaf(acc, acc, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kSmoothThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) cost[blockIdx.x] = red[0] / (float)P.n * inv_tf4;
}

// dst[q] = src[idx[q]] for blocks of S floats; an index outside [0, B) gives a
// block of NaN (the caller's error shows in every result derived from it).
__global__ void gather_kernel(const float* __restrict__ src, const int32_t* __restrict__ idx,
                              int k, int S, int B, float* __restrict__ dst) {
  const int q = blockIdx.y;
  const int j = idx[q];
  const bool ok = j >= 0 && j < B;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x)
    dst[(size_t)q * S + s] = ok ? src[(size_t)j * S + s] : __builtin_nanf("");
}

}  // namespace

hipError_t launch_topk(const float* residual, int B, int k, int32_t* idx, hipStream_t s) {
  hipLaunchKernelGGL(topk_kernel, dim3(1), dim3(kSelThreads), sizeof(float) * B, s, residual, B,
                     k, idx);
  return hipGetLastError();
}

hipError_t launch_best(const float* residual, const float* cost, int B, float tol, int32_t* idx,
                       hipStream_t s) {
  hipLaunchKernelGGL(best_kernel, dim3(1), dim3(kSelThreads), 0, s, residual, cost, B, tol, idx);
  return hipGetLastError();
}

hipError_t launch_smoothness(const ProbDesc* probs, int B, const float* Wdd, const float* xi,
                             int nc, int T, float inv_tf4, float* cost, hipStream_t s) {
  hipLaunchKernelGGL(smoothness_kernel, dim3(B), dim3(kSmoothThreads), 0, s, probs, Wdd, xi, nc,
                     T, inv_tf4, cost);
  return hipGetLastError();
}

hipError_t launch_gather(const float* src, const int32_t* idx, int k, int S, int B, float* dst,
                         hipStream_t s) {
  int gx = (S + 255) / 256;
  gx = gx < 1 ? 1 : (gx > 64 ? 64 : gx);
  hipLaunchKernelGGL(gather_kernel, dim3(gx, k), dim3(256), 0, s, src, idx, k, S, B, dst);
  return hipGetLastError();
}

}  // namespace sf
