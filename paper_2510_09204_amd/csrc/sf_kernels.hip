// HIP kernels of the safety-filter (SF) iteration for gfx950.
//
// One iteration of the fixed-point operator T (Appendix, eqs. alpha_step ..
// xi_step) is computed in the reduced form below, which is algebraically the
// paper's update:
//
//   X    = W xi_bar                         positions, per robot and axis (eq. poly)
//   V_i  = sum_{j != i} r(X_i - X_j) + sum_m r_o(X_i - c_m) + r_box(X_i)
//          with r(D) = D - e(D): e is the alpha/d step result, so
//          r(D) = (1 - a/|D|) D when |D| < a and 0 otherwise (eqs. alpha_step,
//          d_step in 2D, inter_robot_polar, workspace_polar); r_box is the
//          workspace residual G xi_bar - h + s with the s step folded in
//   R    = W^T V                            = F^T r_1 + G^T r_2
//   lambda' = lambda - rho R                (eq. lambda_step)
//   xi_bar' = c_xi + S(lambda - 2 rho R) + SH xi_bar   (eq. xi_step)
//
// S, SH and the constant c_xi = S xi + N b come from the KKT matrix, which
// splits into a robot-mean mode and n-1 identical deviation modes because
// F^T F + G^T G = ((n + M + 2) I - 1 1^T) (x) W^T W: a problem's operator is
// P_perp Y_i + (P_par - P_perp) mean_i(Y) per axis with nc x nc matrices.
//
// Constraint evaluation is exact but culled: time is cut into windows of 16
// steps (one 16-lane DPP row of a wave each); the coefficient->time map also
// reduces each robot's bounding box per window, a wave per (robot, window)
// turns box overlaps into 64-bit candidate masks with a ballot, and the
// pair/obstacle loop visits only candidates.  A skipped pair is farther apart
// than a (plus a rounding margin) at every step of the window, so it is
// inactive and contributes exactly 0: the result equals the full loop's.
//
// The coefficient<->time maps are dense contractions and run on MFMA (16x16x4
// FP32 tiles); the constraint stages are VALU work over LDS.
//
// Data layout: coefficient arrays [axis][robot][coef]; positions and
// constraint sums [robot][time] as float2 (x, y) with an odd row stride
// (window multiple + 1) to spread robots over LDS banks; W as [T][nc].
#include <hip/hip_runtime.h>

#include "sf_internal.h"

namespace sf {

namespace {

constexpr int kRed = 64;   // floats of LDS reduction scratch
constexpr int kWin = 16;   // time steps per culling window (one DPP row)
constexpr int kMeans = 4 * kMaxCoef + 8;

typedef unsigned long long u64;

__device__ __forceinline__ int round4(int x) { return (x + 3) & ~3; }
__device__ __forceinline__ int round16(int x) { return (x + 15) & ~15; }

// Row stride (in steps) of the position/sum buffers: a window multiple plus
// one, so that the 2*stride-float rows of different robots start in different
// LDS banks.
__host__ __device__ __forceinline__ int tstride(int Tc) { return ((Tc + 15) & ~15) + 1; }

typedef float floatx4 __attribute__((ext_vector_type(4)));

// D += A B for a 16x4 by 4x16 FP32 tile: lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[4(l/16)+v][l%16] in element v.
__device__ __forceinline__ floatx4 mfma_16x16x4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// DPP move of v (rows outside row_mask keep `old`); all lanes must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL,
                                                    ROW_MASK, 0xF, false));
}

// Wave sum through DPP in a fixed order: pairs, quads, half rows, rows, then
// row broadcasts; the total lands in lane 63 and is returned to all lanes.
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v += dpp_f<0xB1, 0xF>(0.f, v);    // quad_perm [1,0,3,2]
  v += dpp_f<0x4E, 0xF>(0.f, v);    // quad_perm [2,3,0,1]
  v += dpp_f<0x141, 0xF>(0.f, v);   // row_half_mirror
  v += dpp_f<0x140, 0xF>(0.f, v);   // row_mirror
  v += dpp_f<0x142, 0xA>(0.f, v);   // row_bcast:15 -> rows 1, 3
  v += dpp_f<0x143, 0xC>(0.f, v);   // row_bcast:31 -> rows 2, 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// OR over each quad of lanes (DPP quad permutations); all lanes active.
__device__ __forceinline__ unsigned quad_or(unsigned v) {
  v |= (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
  v |= (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);
  return v;
}

// floor(x / d) for 0 <= x < 2^16 and 16 <= d <= 4096 through a multiply-high
// by m = floor((2^32 - 1)/d) + 1 (exact in that range).
__device__ __forceinline__ unsigned div_magic(unsigned d) { return 0xFFFFFFFFu / d + 1u; }
__device__ __forceinline__ int fast_div(int x, unsigned m) { return (int)__umulhi((unsigned)x, m); }

// Deterministic block sum of up to 4 values: wave shuffles, then a fixed-order
// pass over the per-wave partials.  All threads get the totals.
template <int K>
__device__ void block_sum(float (&v)[K], float* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < K; ++q) v[q] = wave_sum(v[q]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < K; ++q) scratch[q * 16 + wid] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < K; ++q) {
    float t = 0.f;
    for (int w = 0; w < nw; ++w) t += scratch[q * 16 + w];
    v[q] = t;
  }
  __syncthreads();
}

__device__ __forceinline__ u64 readlane64(u64 v, int lane) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), lane);
  return ((u64)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// Stages used by the plain (unfused, global-memory) path.
// ---------------------------------------------------------------------------

// Pair/obstacle/box residual sums for one (robot, step): every other robot
// and every obstacle is visited.
__device__ __forceinline__ void stage_constraints(
    const float2* __restrict__ X, float2* __restrict__ V, int n, int Tce, int Tcs,
    const float* __restrict__ obs, int M, float a, float pmin0, float pmin1, float pmax0,
    float pmax1, bool accum, float& r1sq, float& r2sq, int tid, int nthr) {
  const float a2 = a * a;
  const int items = n * Tce;
  for (int idx = tid; idx < items; idx += nthr) {
    const int i = idx / Tce;
    const int kk = idx - i * Tce;
    const float2 p = X[i * Tcs + kk];
    float vx = 0.f, vy = 0.f;
    for (int j = 0; j < n; ++j) {
      const float2 q = X[j * Tcs + kk];
      const float dx = p.x - q.x;
      const float dy = p.y - q.y;
      const float d2 = fmaf(dy, dy, dx * dx);
      if (d2 < a2 && j != i) {
        float rx, ry;
        if (d2 > 0.f) {
          const float f = 1.f - a * rsqrtf(d2);
          rx = f * dx;
          ry = f * dy;
        } else {  // coincident: alpha = atan2(0, 0) = 0 for the row (min, max)
          rx = (i < j) ? -a : a;
          ry = 0.f;
        }
        vx += rx;
        vy += ry;
        if (accum && j > i) r1sq = fmaf(rx, rx, fmaf(ry, ry, r1sq));
      }
    }
    for (int m = 0; m < M; ++m) {
      const float cx = obs[3 * m], cy = obs[3 * m + 1], ao = obs[3 * m + 2];
      const float dx = p.x - cx;
      const float dy = p.y - cy;
      const float d2 = fmaf(dy, dy, dx * dx);
      if (d2 < ao * ao) {
        float rx, ry;
        if (d2 > 0.f) {
          const float f = 1.f - ao * rsqrtf(d2);
          rx = f * dx;
          ry = f * dy;
        } else {
          rx = -ao;
          ry = 0.f;
        }
        vx += rx;
        vy += ry;
        if (accum) r1sq = fmaf(rx, rx, fmaf(ry, ry, r1sq));
      }
    }
    const float hx = fmaxf(p.x - pmax0, 0.f), lx = fmaxf(pmin0 - p.x, 0.f);
    const float hy = fmaxf(p.y - pmax1, 0.f), ly = fmaxf(pmin1 - p.y, 0.f);
    vx = fmaf(1.f, hx - lx, vx);
    vy = fmaf(1.f, hy - ly, vy);
    if (accum) r2sq += hx * hx + lx * lx + hy * hy + ly * ly;
    V[i * Tcs + kk] = make_float2(vx, vy);
  }
}

// ---------------------------------------------------------------------------
// Coefficient-space helpers shared by both paths.
// ---------------------------------------------------------------------------

// Mode operator: out_i = P_perp y_i + D ybar (rows of P are contiguous).
__device__ __forceinline__ float mode_row(const float* __restrict__ Pp,
                                          const float* __restrict__ D,
                                          const float* __restrict__ y,
                                          const float* __restrict__ ym, int nc, int c,
                                          float acc) {
  const float* pr = Pp + c * nc;
  const float* dr = D + c * nc;
  for (int q = 0; q < nc; ++q) acc = fmaf(pr[q], y[q], fmaf(dr[q], ym[q], acc));
  return acc;
}

// Transposed mode operator: out_i = P_perp^T y_i + D^T ybar.
__device__ __forceinline__ float mode_row_t(const float* __restrict__ Pp,
                                            const float* __restrict__ D,
                                            const float* __restrict__ y,
                                            const float* __restrict__ ym, int nc, int c,
                                            float acc) {
  for (int q = 0; q < nc; ++q)
    acc = fmaf(Pp[q * nc + c], y[q], fmaf(D[q * nc + c], ym[q], acc));
  return acc;
}

// Robot means of every (axis, coef) column of up to two coefficient arrays:
// out[axis*nc + c] for src0 and out[2nc + axis*nc + c] for src1.  One wave per
// column; lane i holds robots i, i+64, ...; fixed reduction tree.
__device__ __forceinline__ void robot_means(const float* __restrict__ src0,
                                            const float* __restrict__ src1, int n, int nc,
                                            float* __restrict__ out, int tid, int nthr) {
  const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
  const float inv = 1.f / (float)n;
  const int cols = (src1 ? 4 : 2) * nc;
  for (int col = wave; col < cols; col += nwaves) {
    const float* src = col < 2 * nc ? src0 : src1;
    const int cc = col < 2 * nc ? col : col - 2 * nc;
    const int ax = cc / nc, c = cc - ax * nc;
    const float* base = src + ax * n * nc + c;
    float s = 0.f;
    for (int i = lane; i < n; i += 64) s += base[i * nc];
    s = wave_sum_dpp(s);
    if (lane == 0) out[col] = s * inv;
  }
}

// Constant term c_xi = S xi + N b, mode form (first block of K^{-1} applied to
// the xi and b parts of eta).  tgt: target xi (coefficient layout), xm/bm:
// robot means of xi ([2][nc]) and of b ([2 axes][2 ends] as bm[ax*2+q]).
__device__ __forceinline__ float cxi_entry(const float* __restrict__ fac, int nc,
                                           const float* __restrict__ tgt,
                                           const float* __restrict__ xm,
                                           const float* __restrict__ bnd_i,
                                           const float* __restrict__ bm, int n, int ax, int i,
                                           int c) {
  const int nc2 = nc * nc;
  const float* Sp = fac;
  const float* DS = fac + nc2;
  const float* Np = fac + 4 * nc2;
  const float* DN = Np + 2 * nc;
  float out = mode_row(Sp, DS, tgt + ax * n * nc + i * nc, xm + ax * nc, nc, c, 0.f);
  for (int q = 0; q < 2; ++q) {
    out = fmaf(Np[c * 2 + q], bnd_i[q * 2 + ax], out);
    out = fmaf(DN[c * 2 + q], bm[ax * 2 + q], out);
  }
  return out;
}

// Robot means of the boundary positions into bm[ax*2 + q].
__device__ __forceinline__ void boundary_means(const float* __restrict__ bnd, int n,
                                               float* __restrict__ bm, int tid, int nthr) {
  for (int t = tid; t < 4; t += nthr) {
    const int ax = t >> 1, q = t & 1;
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += bnd[i * 4 + q * 2 + ax];
    bm[t] = s / (float)n;
  }
}

// ---------------------------------------------------------------------------
// The two dense contractions on MFMA (16x16x4 FP32 tiles), one tile per wave.
// Columns are (robot, axis) pairs col = 2 i + axis, padded to a multiple of 16.
// Positions/sums are float views of [robot][step] float2 arrays with row
// stride Ts steps.
// ---------------------------------------------------------------------------

// Coefficient -> time map X[i][kk].axis = sum_c W[kk][c] xb[axis][i][c] for kk <
// Tce (rows = steps, 16 per tile = one culling window; K = coefficients padded
// to 4).  Padding rows repeat the chunk's last step.  With `box`, each robot's
// per-window bounding box (xmin, xmax, ymin, ymax) is reduced from the tile.
__device__ __forceinline__ void stage_xmap_mfma(const float* __restrict__ W, int nc,
                                                const float* __restrict__ xb, int n,
                                                float* __restrict__ Xf, int Tce, int Ts,
                                                float* __restrict__ boxf, int nws, int wave,
                                                int nwaves, int lane) {
  const int nwin = (Tce + 15) >> 4;
  const int ncol = (2 * n + 15) >> 4;
  const int ks = (nc + 3) >> 2;
  const int m = lane & 15, kq = lane >> 4;
  for (int tile = wave; tile < nwin * ncol; tile += nwaves) {
    const int mt = tile / ncol, nt = tile - mt * ncol;
    const int row = min(mt * 16 + m, Tce - 1);
    const int col = nt * 16 + m;
    const int i = col >> 1, ax = col & 1;
    const bool colok = i < n;
    const float* wrow = W + row * nc;
    const float* brow = xb + ax * n * nc + i * nc;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < ks; ++s) {
      const int c = 4 * s + kq;
      const float a = c < nc ? wrow[c] : 0.f;
      const float b = (c < nc && colok) ? brow[c] : 0.f;
      acc = mfma_16x16x4(a, b, acc);
    }
    const int k0 = mt * 16 + 4 * kq;
    if (colok) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (k0 + v < Tce) Xf[((size_t)i * Ts + k0 + v) * 2 + ax] = acc[v];
    }
    if (boxf) {
      float lo = fminf(fminf(acc[0], acc[1]), fminf(acc[2], acc[3]));
      float hi = fmaxf(fmaxf(acc[0], acc[1]), fmaxf(acc[2], acc[3]));
      lo = fminf(lo, __shfl_xor(lo, 16, 64));
      hi = fmaxf(hi, __shfl_xor(hi, 16, 64));
      lo = fminf(lo, __shfl_xor(lo, 32, 64));
      hi = fmaxf(hi, __shfl_xor(hi, 32, 64));
      if (lane < 16 && colok) {
        float* bx = boxf + ((size_t)i * nws + mt) * 4 + 2 * ax;
        bx[0] = lo;
        bx[1] = hi;
      }
    }
  }
}

// Time -> coefficient map R[axis][i][c] (+)= sum_kk W[kk][c] V[i][kk].axis over
// kk < Tce (rows = coefficients, K = steps padded to 16).  With `lam`, the
// lambda step runs on the finished R: lambda' = lambda - rho R and R becomes
// u = lambda - 2 rho R.
__device__ __forceinline__ void stage_wtmap_mfma(const float* __restrict__ W, int nc,
                                                 const float* __restrict__ Vf, int n, int Tce,
                                                 int Ts, float* __restrict__ R, bool accumulate,
                                                 float* __restrict__ lam, float rho,
                                                 bool want_dz, float& dzsq, int wave, int nwaves,
                                                 int lane) {
  const int nct = (nc + 15) >> 4;
  const int ncol = (2 * n + 15) >> 4;
  const int ks = ((Tce + 15) >> 4) * 4;
  const int m = lane & 15, kq = lane >> 4;
  for (int tile = wave; tile < nct * ncol; tile += nwaves) {
    const int ct = tile / ncol, nt = tile - ct * ncol;
    const int ca = ct * 16 + m;
    const int col = nt * 16 + m;
    const int i = col >> 1, ax = col & 1;
    const bool colok = i < n;
    const float* vrow = Vf + (size_t)(colok ? i : 0) * Ts * 2 + ax;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int st = 0; st < ks; st += 4) {
      float av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = 4 * (st + u) + kq;
        const bool kok = kk < Tce;
        av[u] = (kok && ca < nc) ? W[kk * nc + ca] : 0.f;
        bv[u] = (kok && colok) ? vrow[2 * kk] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = mfma_16x16x4(av[u], bv[u], acc);
    }
    if (colok) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = ct * 16 + 4 * kq + v;
        if (c >= nc) continue;
        const int sidx = ax * n * nc + i * nc + c;
        const float r = accumulate ? R[sidx] + acc[v] : acc[v];
        if (lam) {
          const float lm = lam[sidx];
          lam[sidx] = fmaf(-rho, r, lm);
          R[sidx] = fmaf(-2.f * rho, r, lm);
          if (want_dz) dzsq = fmaf(rho * r, rho * r, dzsq);
        } else {
          R[sidx] = r;
        }
      }
    }
  }
}

// Number of K splits of the time->coefficient map for a problem: enough
// (tile, split) work items for 16 waves, at most kSplitMax; depends only on
// the problem's shape, so every launch configuration sums in the same order.
constexpr int kSplitMax = 4;
__host__ __device__ __forceinline__ int wt_splits(int n, int nc) {
  const int tiles = ((nc + 15) >> 4) * ((2 * n + 15) >> 4);
  const int ks = 16 / tiles;
  return ks < 1 ? 1 : (ks > kSplitMax ? kSplitMax : ks);
}

// K-split time->coefficient map: split sp of tile t adds sum over its share of
// the steps of W[kk][c] V[i][kk].axis into part[sp*S + s] (or stores it).
// Loads of four K steps are issued ahead of their MFMAs; zero-padded steps
// add exact zeros.
__device__ __forceinline__ void stage_wtmap_part(const float* __restrict__ W, int nc,
                                                 const float* __restrict__ Vf, int n, int Tce,
                                                 int Ts, float* __restrict__ part, int S,
                                                 bool accumulate, int wave, int nwaves,
                                                 int lane) {
  const int nct = (nc + 15) >> 4;
  const int ncol = (2 * n + 15) >> 4;
  const int tiles = nct * ncol;
  const int KS = wt_splits(n, nc);
  const int ks = ((Tce + 15) >> 4) * 4;
  const int kps = (((ks + KS - 1) / KS) + 3) & ~3;
  const int m = lane & 15, kq = lane >> 4;
  for (int wi = wave; wi < tiles * KS; wi += nwaves) {
    const int sp = wi / tiles, tile = wi - sp * tiles;
    const int ct = tile / ncol, nt = tile - ct * ncol;
    const int ca = ct * 16 + m;
    const int col = nt * 16 + m;
    const int i = col >> 1, ax = col & 1;
    const bool colok = i < n;
    const float* vrow = Vf + (size_t)(colok ? i : 0) * Ts * 2 + ax;
    const int s0 = sp * kps, s1 = min(ks, s0 + kps);
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int st = s0; st < s1; st += 4) {
      float av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = 4 * (st + u) + kq;
        const bool kok = (st + u < s1) && kk < Tce;
        av[u] = (kok && ca < nc) ? W[kk * nc + ca] : 0.f;
        bv[u] = (kok && colok) ? vrow[2 * kk] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = mfma_16x16x4(av[u], bv[u], acc);
    }
    if (colok) {
      float* dst = part + (size_t)sp * S;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = ct * 16 + 4 * kq + v;
        if (c >= nc) continue;
        const int sidx = ax * n * nc + i * nc + c;
        dst[sidx] = accumulate ? dst[sidx] + acc[v] : acc[v];
      }
    }
  }
}

// R = the K-split partials summed in split order; lambda step lambda' =
// lambda - rho R; u = lambda - 2 rho R into Ru; robot means of u
// (means[axis*nc + c]) and of xb (means[2nc + axis*nc + c]).  One wave per
// column, lanes over robots.
__device__ __forceinline__ void combine_lambda_means(const float* __restrict__ part, int S,
                                                     float* __restrict__ lam,
                                                     float* __restrict__ Ru,
                                                     const float* __restrict__ xb, int n, int nc,
                                                     float rho, bool want_dz, float& dzsq,
                                                     float* __restrict__ means, int tid,
                                                     int nthr) {
  const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
  const int KS = wt_splits(n, nc);
  const float inv = 1.f / (float)n;
  for (int col = wave; col < 4 * nc; col += nwaves) {
    const bool ucol = col < 2 * nc;
    const int cc = ucol ? col : col - 2 * nc;
    const int ax = cc / nc, c = cc - ax * nc;
    float acc = 0.f;
    for (int i = lane; i < n; i += 64) {
      const int sidx = ax * n * nc + i * nc + c;
      if (ucol) {
        float r = part[sidx];
        for (int k = 1; k < KS; ++k) r += part[(size_t)k * S + sidx];
        const float lm = lam[sidx];
        lam[sidx] = fmaf(-rho, r, lm);
        const float u = fmaf(-2.f * rho, r, lm);
        Ru[sidx] = u;
        acc += u;
        if (want_dz) dzsq = fmaf(rho * r, rho * r, dzsq);
      } else {
        acc += xb[sidx];
      }
    }
    acc = wave_sum_dpp(acc);
    if (lane == 0) means[col] = acc * inv;
  }
}

// ---------------------------------------------------------------------------
// Stages of the fused kernels (LDS-resident state, culled constraints).
// Loops over (robot, step) items advance a whole wave at a time so that a
// 16-lane row always holds one (robot, window) and shuffles see whole rows.
// ---------------------------------------------------------------------------

// Copy rows k0 .. k0+Tce-1 of W (global, [T][nc]) into the LDS table W.
__device__ __forceinline__ void load_wchunk(const float* __restrict__ Wg, float* __restrict__ W,
                                            int nc, int k0, int Tce, int tid, int nthr) {
  for (int t = tid; t < Tce * nc; t += nthr) W[t] = Wg[k0 * nc + t];
}

// Culling geometry of one chunk: padded step count, window count and strides.
struct Geo {
  int Tce;   // steps in this chunk
  int Tcp;   // Tce rounded up to a window multiple
  int Tcs;   // row stride of X/V buffers (>= Tcp)
  int nws;   // row stride (in windows) of the box and mask arrays
  int pw;    // 64-bit mask words for robots
  int ow;    // 64-bit mask words for obstacles
};

// Candidate masks per (robot, window): bit j of word q set when robot 64q+j
// (j != i) has a box within a (plus margin) of robot i's box in both axes;
// bit m of the obstacle words when obstacle m's disc (plus margin) meets robot
// i's box.  Four lanes (a DPP quad) share a (robot, window) and split the
// candidates.  The margin covers rounding of the box comparison and of the
// exact test at coordinates of magnitude up to the box's plus the threshold.
__device__ __forceinline__ void stage_masks(const float4* __restrict__ box, int n,
                                            const float4* __restrict__ obs, int M, float a,
                                            u64* __restrict__ masks, const Geo& g, int tid,
                                            int nthr) {
  const int lane = tid & 63;
  const int nwin = g.Tcp >> 4;
  const int tasks = n * nwin;
  const int mw = g.pw + g.ow;
  for (int base = tid & ~63; base < tasks * 4; base += nthr) {
    const int idx = base + lane;
    const bool live = idx < tasks * 4;
    const int task = live ? idx >> 2 : 0;
    const int q = idx & 3;
    const int i = task / nwin, w = task - i * nwin;
    const float4 bi = box[i * g.nws + w];
    const float si = fmaxf(fmaxf(fabsf(bi.x), fabsf(bi.y)), fmaxf(fabsf(bi.z), fabsf(bi.w)));
    const float am = a * 1.0001f + 4e-6f * (1.f + si + 2.f * a);
    u64* out = masks + (size_t)(i * g.nws + w) * mw;
    for (int wd = 0; wd < g.pw; ++wd) {
      unsigned lo = 0u, hi = 0u;
      const int jend = min(n - wd * 64, 64);
      for (int jj = q; jj < jend; jj += 4) {
        const int j = wd * 64 + jj;
        const float4 bj = box[j * g.nws + w];
        const bool c = (j != i) && (bi.x < bj.y + am) && (bj.x < bi.y + am) &&
                       (bi.z < bj.w + am) && (bj.z < bi.w + am);
        const unsigned bit = c ? (1u << (jj & 31)) : 0u;
        if (jj < 32) lo |= bit; else hi |= bit;
      }
      lo = quad_or(lo);
      hi = quad_or(hi);
      if (live && q == 0) out[wd] = ((u64)hi << 32) | lo;
    }
    for (int wd = 0; wd < g.ow; ++wd) {
      unsigned lo = 0u, hi = 0u;
      const int mend = min(M - wd * 64, 64);
      for (int mm = q; mm < mend; mm += 4) {
        const float4 o = obs[wd * 64 + mm];
        const float r = o.z * 1.0001f + 4e-6f * (1.f + si + 2.f * o.z);
        const bool c = (o.x - r < bi.y) && (bi.x < o.x + r) && (o.y - r < bi.w) && (bi.z < o.y + r);
        const unsigned bit = c ? (1u << (mm & 31)) : 0u;
        if (mm < 32) lo |= bit; else hi |= bit;
      }
      lo = quad_or(lo);
      hi = quad_or(hi);
      if (live && q == 0) out[g.pw + wd] = ((u64)hi << 32) | lo;
    }
  }
}

// Union over the wave's four rows of the rows' candidate words.
__device__ __forceinline__ u64 wave_union(u64 m) {
  return readlane64(m, 0) | readlane64(m, 16) | readlane64(m, 32) | readlane64(m, 48);
}

// Culled constraint stage: V = w_pair (pair + obstacle sums) + w_box (box
// residual), pairs visited in increasing robot index, then obstacles, then the
// box (the order of the full loop).  With `accum`, ||r_1||^2 (each unordered
// pair once) and ||r_2||^2.
__device__ __forceinline__ void stage_constraints_culled(
    const float2* __restrict__ X, float2* __restrict__ V, int n,
    const float4* __restrict__ obs, const u64* __restrict__ masks, float a, float pmin0,
    float pmin1, float pmax0, float pmax1, bool accum, float& r1sq, float& r2sq,
    const Geo& g, int tid, int nthr, float w_pair = 1.f, float w_box = 1.f) {
  const float a2 = a * a;
  const int items = n * g.Tcp;
  const int mw = g.pw + g.ow;
  const unsigned dm = div_magic((unsigned)g.Tcp);
  for (int base = tid & ~63; base < items; base += nthr) {
    const int idx = base + (tid & 63);
    const bool live = idx < items;
    const int i = live ? fast_div(idx, dm) : 0;
    const int kk = live ? idx - i * g.Tcp : 0;
    const bool valid = live && kk < g.Tce;
    const int kq = min(kk, g.Tce - 1);
    const u64* my = masks + (size_t)(i * g.nws + (kk >> 4)) * mw;
    const float2 p = X[i * g.Tcs + kq];
    float vx = 0.f, vy = 0.f, s1 = 0.f;
    for (int q = 0; q < g.pw; ++q) {
      u64 u = wave_union(live ? my[q] : 0ull);
      while (u) {
        const int j = q * 64 + __builtin_ctzll(u);
        u &= u - 1;
        const float2 o = X[j * g.Tcs + kq];
        const float dx = p.x - o.x;
        const float dy = p.y - o.y;
        const float d2 = fmaf(dy, dy, dx * dx);
        if (d2 < a2 && j != i) {
          float rx, ry;
          if (d2 > 0.f) {
            const float f = 1.f - a * rsqrtf(d2);
            rx = f * dx;
            ry = f * dy;
          } else {  // coincident: alpha = atan2(0, 0) = 0 for the row (min, max)
            rx = (i < j) ? -a : a;
            ry = 0.f;
          }
          vx += rx;
          vy += ry;
          if (j > i) s1 = fmaf(rx, rx, fmaf(ry, ry, s1));
        }
      }
    }
    for (int q = 0; q < g.ow; ++q) {
      u64 u = wave_union(live ? my[g.pw + q] : 0ull);
      while (u) {
        const int m = q * 64 + __builtin_ctzll(u);
        u &= u - 1;
        const float4 ob = obs[m];
        const float dx = p.x - ob.x;
        const float dy = p.y - ob.y;
        const float d2 = fmaf(dy, dy, dx * dx);
        if (d2 < ob.w) {
          float rx, ry;
          if (d2 > 0.f) {
            const float f = 1.f - ob.z * rsqrtf(d2);
            rx = f * dx;
            ry = f * dy;
          } else {
            rx = -ob.z;
            ry = 0.f;
          }
          vx += rx;
          vy += ry;
          s1 = fmaf(rx, rx, fmaf(ry, ry, s1));
        }
      }
    }
    const float hx = fmaxf(p.x - pmax0, 0.f), lx = fmaxf(pmin0 - p.x, 0.f);
    const float hy = fmaxf(p.y - pmax1, 0.f), ly = fmaxf(pmin1 - p.y, 0.f);
    vx = fmaf(w_box, hx - lx, w_pair * vx);
    vy = fmaf(w_box, hy - ly, w_pair * vy);
    if (valid) {
      V[i * g.Tcs + kk] = make_float2(vx, vy);
      if (accum) {
        r1sq += s1;
        r2sq += hx * hx + lx * lx + hy * hy + ly * ly;
      }
    }
  }
}

// Culled vector-Jacobian product of the constraint stage: given the cotangent
// G of V at positions X,
//   H_i = sum_{j != i} J(X_i - X_j) (G_i - G_j) + sum_m J_o(X_i - c_m) G_i
//         + box'(X_i) G_i,
// where J(D) = (1 - f) I + f u u^T, f = a/|D|, u = D/|D| is the Jacobian of
// r(D) = D - e(D) for an active pair (|D| < a) and 0 otherwise; at D = 0 the
// e of the alpha/d steps is locally constant, so J = I.
__device__ __forceinline__ void stage_vjp_culled(
    const float2* __restrict__ X, const float2* __restrict__ G, float2* __restrict__ H, int n,
    const float4* __restrict__ obs, const u64* __restrict__ masks, float a, float pmin0,
    float pmin1, float pmax0, float pmax1, const Geo& g, int tid, int nthr) {
  const float a2 = a * a;
  const int items = n * g.Tcp;
  const int mw = g.pw + g.ow;
  const unsigned dm = div_magic((unsigned)g.Tcp);
  for (int base = tid & ~63; base < items; base += nthr) {
    const int idx = base + (tid & 63);
    const bool live = idx < items;
    const int i = live ? fast_div(idx, dm) : 0;
    const int kk = live ? idx - i * g.Tcp : 0;
    const int kq = min(kk, g.Tce - 1);
    const u64* my = masks + (size_t)(i * g.nws + (kk >> 4)) * mw;
    const float2 p = X[i * g.Tcs + kq];
    const float2 gi = G[i * g.Tcs + kq];
    float hx = 0.f, hy = 0.f;
    for (int q = 0; q < g.pw; ++q) {
      u64 u = wave_union(live ? my[q] : 0ull);
      while (u) {
        const int j = q * 64 + __builtin_ctzll(u);
        u &= u - 1;
        const float2 o = X[j * g.Tcs + kq];
        const float dx = p.x - o.x;
        const float dy = p.y - o.y;
        const float d2 = fmaf(dy, dy, dx * dx);
        if (d2 < a2 && j != i) {
          const float2 gj = G[j * g.Tcs + kq];
          const float wx = gi.x - gj.x, wy = gi.y - gj.y;
          if (d2 > 0.f) {
            const float inv = rsqrtf(d2);
            const float f = a * inv;
            const float ux = dx * inv, uy = dy * inv;
            const float dot = fmaf(ux, wx, uy * wy);
            hx += fmaf(1.f - f, wx, f * ux * dot);
            hy += fmaf(1.f - f, wy, f * uy * dot);
          } else {
            hx += wx;
            hy += wy;
          }
        }
      }
    }
    for (int q = 0; q < g.ow; ++q) {
      u64 u = wave_union(live ? my[g.pw + q] : 0ull);
      while (u) {
        const int m = q * 64 + __builtin_ctzll(u);
        u &= u - 1;
        const float4 ob = obs[m];
        const float dx = p.x - ob.x;
        const float dy = p.y - ob.y;
        const float d2 = fmaf(dy, dy, dx * dx);
        if (d2 < ob.w) {
          if (d2 > 0.f) {
            const float inv = rsqrtf(d2);
            const float f = ob.z * inv;
            const float ux = dx * inv, uy = dy * inv;
            const float dot = fmaf(ux, gi.x, uy * gi.y);
            hx += fmaf(1.f - f, gi.x, f * ux * dot);
            hy += fmaf(1.f - f, gi.y, f * uy * dot);
          } else {
            hx += gi.x;
            hy += gi.y;
          }
        }
      }
    }
    if (p.x > pmax0 || p.x < pmin0) hx += gi.x;
    if (p.y > pmax1 || p.y < pmin1) hy += gi.y;
    if (live && kk < g.Tce) H[i * g.Tcs + kk] = make_float2(hx, hy);
  }
}

// Per-problem constants of the fused kernels, with LDS-resident tables.
struct Ctx {
  int n, M, nc, T, Tc, S, tid;
  float rho, a, pmin0, pmin1, pmax0, pmax1;
  float* W;
  const float *fac, *Wg;
  const float4* obs;
  float4* box;
  u64* masks;
  int n_max, M_max;
  bool chunked;  // T > Tc: the LDS W tables hold one time chunk at a time

  __device__ __forceinline__ Geo geo(int k0) const {
    Geo g;
    g.Tce = min(Tc, T - k0);
    g.Tcp = round16(g.Tce);
    g.Tcs = tstride(Tc);
    g.nws = g.Tcs / kWin;
    g.pw = (n + 63) >> 6;
    g.ow = (M + 63) >> 6;
    return g;
  }

  // Make the LDS W tables hold rows k0 .. k0+Tce-1 (block-wide; no-op when
  // the whole horizon is resident).
  template <int NT>
  __device__ __forceinline__ void wchunk(int k0, int Tce) const {
    if (!chunked) return;
    __syncthreads();
    load_wchunk(Wg, W, nc, k0, Tce, tid, NT);
    __syncthreads();
  }

  // X map, boxes and masks of one chunk into X (block-synchronised on return).
  template <int NT>
  __device__ __forceinline__ void positions(const float* xb, float2* X, const Geo& g) const {
    stage_xmap_mfma(W, nc, xb, n, reinterpret_cast<float*>(X), g.Tce, g.Tcs,
                    reinterpret_cast<float*>(box), g.nws, tid >> 6, NT >> 6, tid & 63);
    __syncthreads();
    stage_masks(box, n, obs, M, a, masks, g, tid, NT);
    __syncthreads();
  }
};

// Floats of the box and mask regions shared by both fused kernels.
__host__ __device__ inline int box_floats(int Tc, int n_max) {
  return 4 * n_max * (((Tc + 15) & ~15) / 16);
}
__host__ __device__ inline int mask_floats(int Tc, int n_max, int M_max) {
  const int nws = ((Tc + 15) & ~15) / 16;
  return 2 * n_max * nws * ((n_max + 63) / 64 + (M_max + 63) / 64);
}

// One application of T on the LDS state (xb, lam) -> (xn, lam).  Ru, X, V and
// means are scratch.  Entered and left with the block synchronised.
template <int NT>
__device__ __forceinline__ void sf_iteration(const Ctx& C, const float* xb, float* xn, float* lam, float* Ru,
                             float* means, float2* X, float2* V, const float* cx, bool last,
                             float& dzsq, float* part) {
  const int n = C.n, nc = C.nc, T = C.T, S = C.S, tid = C.tid;
  float d1 = 0.f, d2 = 0.f;
  for (int k0 = 0; k0 < T; k0 += C.Tc) {
    const Geo g = C.geo(k0);
    C.wchunk<NT>(k0, g.Tce);
    C.positions<NT>(xb, X, g);
    stage_constraints_culled(X, V, n, C.obs, C.masks, C.a, C.pmin0, C.pmin1, C.pmax0, C.pmax1,
                             false, d1, d2, g, tid, NT);
    __syncthreads();
    stage_wtmap_part(C.W, nc, reinterpret_cast<const float*>(V), n, g.Tce, g.Tcs, part, S,
                     k0 > 0, tid >> 6, NT >> 6, tid & 63);
  }
  __syncthreads();
  combine_lambda_means(part, S, lam, Ru, xb, n, nc, C.rho, last, dzsq, means, tid, NT);
  __syncthreads();
  const int nc2 = nc * nc;
  for (int s = tid; s < S; s += NT) {
    const int ax = s / (n * nc), rem = s - ax * n * nc, i = rem / nc, c = rem - i * nc;
    const int row = ax * n * nc + i * nc;
    float v = mode_row(C.fac, C.fac + nc2, Ru + row, means + ax * nc, nc, c, cx[s]);
    v = mode_row(C.fac + 2 * nc2, C.fac + 3 * nc2, xb + row, means + 2 * nc + ax * nc, nc, c,
                 v);
    xn[s] = v;
    if (last) {
      const float d = v - xb[s];
      dzsq = fmaf(d, d, dzsq);
    }
  }
  __syncthreads();
}

// ||r_1||^2 and ||r_2||^2 partials of the iterate xb (block-synchronised on
// return); V is scratch.
template <int NT>
__device__ __forceinline__ void residual_norms(const Ctx& C, const float* xb, float2* X, float2* V, float& r1sq,
                               float& r2sq) {
  for (int k0 = 0; k0 < C.T; k0 += C.Tc) {
    const Geo g = C.geo(k0);
    C.wchunk<NT>(k0, g.Tce);
    C.positions<NT>(xb, X, g);
    stage_constraints_culled(X, V, C.n, C.obs, C.masks, C.a, C.pmin0, C.pmin1, C.pmax0,
                             C.pmax1, true, r1sq, r2sq, g, C.tid, NT);
    __syncthreads();
  }
}

struct FwdLds {
  float *W, *fac, *xbA, *xbB, *lam, *cx, *Ru, *means, *red, *part;
  float4* obs;
  float4* box;
  u64* masks;
  float2 *X, *V;
};

__device__ __forceinline__ FwdLds carve_fwd(float* sm, int nc, int Tc, int n_max, int M_max,
                                            int S_max) {
  FwdLds L;
  float* p = sm;
  L.W = p; p += round4(nc * Tc);
  L.fac = p; p += round4(fac_stride(nc));
  L.xbA = p; p += round4(S_max);
  L.xbB = p; p += round4(S_max);
  L.lam = p; p += round4(S_max);
  L.cx = p; p += round4(S_max);
  L.Ru = p; p += round4(S_max);
  L.part = p; p += kSplitMax * round4(S_max);
  L.means = p; p += kMeans;
  L.red = p; p += kRed;
  L.obs = reinterpret_cast<float4*>(p); p += 4 * M_max;
  L.box = reinterpret_cast<float4*>(p); p += box_floats(Tc, n_max);
  L.masks = reinterpret_cast<u64*>(p); p += mask_floats(Tc, n_max, M_max);
  L.X = reinterpret_cast<float2*>(p); p += 2 * n_max * tstride(Tc);
  L.V = reinterpret_cast<float2*>(p);
  return L;
}

}  // namespace

size_t fwd_lds_bytes(int nc, int T, int Tc, int n_max, int M_max, int S_max, int) {
  auto r4 = [](int x) { return (size_t)((x + 3) & ~3); };
  const size_t Tcs = tstride(Tc);
  size_t f = r4(nc * Tc) + r4(fac_stride(nc)) + (5 + kSplitMax) * r4(S_max) + kMeans + kRed +
             4 * (size_t)M_max + box_floats(Tc, n_max) + mask_floats(Tc, n_max, M_max) +
             4 * (size_t)n_max * Tcs;
  return f * sizeof(float);
}

// ---------------------------------------------------------------------------
// Fused forward: one workgroup runs all L iterations of one problem with the
// whole state in LDS.  Launch slot -> problem through `order` (longest first).
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void fwd_fused_kernel(FwdArgs A) {
  extern __shared__ float4 sm4[];
  float* sm = reinterpret_cast<float*>(sm4);
  const int tid = threadIdx.x;
  const int b = A.order[blockIdx.x];
  const ProbDesc P = A.probs[b];
  const int n = P.n, M = P.M, nc = A.nc, T = A.T;
  const int S = 2 * n * nc;
  const int fs = fac_stride(nc);
  FwdLds L = carve_fwd(sm, nc, A.Tc, A.n_max, A.M_max, A.S_max);
  Ctx C{n,         M,         nc,        T,         A.Tc, S,   tid,   A.rho, P.a,
        P.pmin[0], P.pmin[1], P.pmax[0], P.pmax[1], L.W, L.fac, A.W,   L.obs,
        L.box,     L.masks,   A.n_max,   A.M_max,   A.Tc < T};
  if (!C.chunked) load_wchunk(A.W, L.W, nc, 0, T, tid, NT);
  for (int t = tid; t < fs; t += NT) L.fac[t] = A.fac[(size_t)P.fac * fs + t];
  for (int m = tid; m < M; m += NT) {
    const float* o = A.obstacles + ((size_t)P.obs_off + m) * 3;
    L.obs[m] = make_float4(o[0], o[1], o[2], o[2] * o[2]);
    if (A.save) {
      float* d = A.ws_obs + ((size_t)P.obs_off + m) * 3;
      d[0] = o[0];
      d[1] = o[1];
      d[2] = o[2];
    }
  }
  for (int s = tid; s < S; s += NT) {
    L.xbA[s] = A.xi0[P.coef_off + s];
    L.lam[s] = A.lam0[P.coef_off + s];
    L.Ru[s] = A.xi[P.coef_off + s];
  }
  __syncthreads();
  const float* bnd = A.boundary + (size_t)P.rob_off * 4;
  robot_means(L.Ru, nullptr, n, nc, L.means, tid, NT);
  boundary_means(bnd, n, L.means + 2 * nc, tid, NT);
  __syncthreads();
  for (int s = tid; s < S; s += NT) {
    const int ax = s / (n * nc), rem = s - ax * n * nc, i = rem / nc, c = rem - i * nc;
    const float v = cxi_entry(L.fac, nc, L.Ru, L.means, bnd + i * 4, L.means + 2 * nc, n,
                              ax, i, c);
    L.cx[s] = v;
    if (A.save) A.ws_cxi[P.coef_off + s] = v;
  }
  __syncthreads();

  float* xb = L.xbA;
  float* xn = L.xbB;
  float dzsq = 0.f;
  for (int l = 0; l < A.L; ++l) {
    if (A.save && (l % A.ckpt_every) == 0) {
      float* ck = A.ws_ckpt + (size_t)(l / A.ckpt_every) * 2 * A.S_total + P.coef_off;
      for (int s = tid; s < S; s += NT) {
        ck[s] = xb[s];
        ck[A.S_total + s] = L.lam[s];
      }
    }
    sf_iteration<NT>(C, xb, xn, L.lam, L.Ru, L.means, L.X, L.V, L.cx, l == A.L - 1, dzsq,
                     L.part);
    float* t = xb;
    xb = xn;
    xn = t;
  }

  float bad = 0.f;
  for (int s = tid; s < S; s += NT) {
    const float x = xb[s], lm = L.lam[s];
    if (A.save) {
      A.ws_final[P.coef_off + s] = x;
      A.ws_final[A.S_total + P.coef_off + s] = lm;
    }
    A.xi_out[P.coef_off + s] = x;
    A.lam_out[P.coef_off + s] = lm;
    if (!isfinite(x) || !isfinite(lm)) bad = 1.f;
  }
  // residual of the returned iterate
  float r1sq = 0.f, r2sq = 0.f;
  residual_norms<NT>(C, xb, L.X, L.V, r1sq, r2sq);
  float v[4] = {r1sq, r2sq, dzsq, bad};
  block_sum(v, L.red);
  if (tid == 0) {
    float* res = A.residual + (size_t)b * 4;
    res[0] = sqrtf(v[0]);
    res[1] = sqrtf(v[1]);
    res[2] = sqrtf(v[2]);
    res[3] = (v[3] > 0.f || !isfinite(v[0]) || !isfinite(v[1])) ? 1.f : 0.f;
  }
}

hipError_t launch_fwd_fused(const FwdArgs& a, int threads, size_t lds, hipStream_t s) {
  dim3 grid(a.B);
  switch (threads) {
    case 256:
      hipLaunchKernelGGL(fwd_fused_kernel<256>, grid, dim3(256), lds, s, a);
      break;
    case 512:
      hipLaunchKernelGGL(fwd_fused_kernel<512>, grid, dim3(512), lds, s, a);
      break;
    case 1024:
      hipLaunchKernelGGL(fwd_fused_kernel<1024>, grid, dim3(1024), lds, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused adjoint: one workgroup per problem walks the checkpoint segments in
// reverse; each segment's iterates are recomputed from its checkpoint into a
// global scratch area, then the reverse sweep applies, per iteration,
//   g_u = S^T g_xi_bar'          (also the cotangent of the target xi)
//   g_R = -2 rho g_u - rho g_lambda'
//   g_xi_bar = SH^T g_xi_bar' + W^T VJP(W g_R),  g_lambda = g_lambda' + g_u.
// ---------------------------------------------------------------------------
namespace {

struct BwdLds {
  float *W, *fac, *red, *means, *gA, *gB, *glam, *gxi, *cx, *b0, *b1, *b2, *b3, *part;
  float4* obs;
  float4* box;
  u64* masks;
  float2 *X, *G, *H;
};

__device__ __forceinline__ BwdLds carve_bwd(float* sm, int nc, int Tc, int n_max, int M_max,
                                            int S_max) {
  BwdLds L;
  float* p = sm;
  L.W = p; p += round4(nc * Tc);
  L.fac = p; p += round4(fac_stride(nc));
  L.red = p; p += kRed;
  L.means = p; p += kMeans;
  float** bufs[9] = {&L.gA, &L.gB, &L.glam, &L.gxi, &L.cx, &L.b0, &L.b1, &L.b2, &L.b3};
  for (int q = 0; q < 9; ++q) {
    *bufs[q] = p;
    p += round4(S_max);
  }
  L.part = p; p += kSplitMax * round4(S_max);
  L.obs = reinterpret_cast<float4*>(p); p += 4 * M_max;
  L.box = reinterpret_cast<float4*>(p); p += box_floats(Tc, n_max);
  L.masks = reinterpret_cast<u64*>(p); p += mask_floats(Tc, n_max, M_max);
  L.X = reinterpret_cast<float2*>(p); p += 2 * n_max * tstride(Tc);
  L.G = reinterpret_cast<float2*>(p); p += 2 * n_max * tstride(Tc);
  L.H = reinterpret_cast<float2*>(p);
  return L;
}

template <int NT>
__global__ __launch_bounds__(NT) void bwd_fused_kernel(BwdArgs A) {
  extern __shared__ float4 sm4[];
  float* sm = reinterpret_cast<float*>(sm4);
  const int tid = threadIdx.x;
  const int b = A.order[blockIdx.x];
  const ProbDesc P = A.probs[b];
  const int n = P.n, M = P.M, nc = A.nc, T = A.T, Tc = A.Tc;
  const int S = 2 * n * nc;
  const int fs = fac_stride(nc);
  const int nc2 = nc * nc;
  const float rho = A.rho, w = A.fp_weight;
  const size_t St = (size_t)A.S_total;
  BwdLds L = carve_bwd(sm, nc, Tc, A.n_max, A.M_max, A.S_max);
  Ctx C{n,         M,         nc,        T,         Tc,   S,   tid,   rho, P.a,
        P.pmin[0], P.pmin[1], P.pmax[0], P.pmax[1], L.W, L.fac, A.W, L.obs,
        L.box,     L.masks,   A.n_max,   A.M_max,   Tc < T};
  if (!C.chunked) load_wchunk(A.W, L.W, nc, 0, T, tid, NT);
  for (int t = tid; t < fs; t += NT) L.fac[t] = A.fac[(size_t)P.fac * fs + t];
  for (int m = tid; m < M; m += NT) {
    const float* o = A.obs + ((size_t)P.obs_off + m) * 3;
    L.obs[m] = make_float4(o[0], o[1], o[2], o[2] * o[2]);
  }
  for (int s = tid; s < S; s += NT) {
    L.cx[s] = A.cxi[P.coef_off + s];
    L.gA[s] = A.g_xi_out ? A.g_xi_out[P.coef_off + s] : 0.f;
    L.glam[s] = A.g_lam_out ? A.g_lam_out[P.coef_off + s] : 0.f;
    L.gxi[s] = 0.f;
  }
  __syncthreads();
  float* gx = L.gA;
  float* gn = L.gB;

  // cotangents of ||r_1|| and ||r_2|| of the returned iterate: d(0.5||r_1||^2)/dX
  // is the pair/obstacle part of V and d(0.5||r_2||^2)/dX its box part.
  const float gr1 = A.g_res ? A.g_res[(size_t)b * 4] : 0.f;
  const float gr2 = A.g_res ? A.g_res[(size_t)b * 4 + 1] : 0.f;
  if (gr1 != 0.f || gr2 != 0.f) {
    for (int s = tid; s < S; s += NT) L.b0[s] = A.fin[P.coef_off + s];
    __syncthreads();
    float r1sq = 0.f, r2sq = 0.f;
    residual_norms<NT>(C, L.b0, L.X, L.G, r1sq, r2sq);
    float v[2] = {r1sq, r2sq};
    block_sum(v, L.red);
    const float c1 = v[0] > 0.f ? gr1 / sqrtf(v[0]) : 0.f;
    const float c2 = v[1] > 0.f ? gr2 / sqrtf(v[1]) : 0.f;
    float d1 = 0.f, d2 = 0.f, dz = 0.f;
    for (int k0 = 0; k0 < T; k0 += Tc) {
      const Geo g = C.geo(k0);
      C.wchunk<NT>(k0, g.Tce);
      C.positions<NT>(L.b0, L.X, g);
      stage_constraints_culled(L.X, L.H, n, L.obs, L.masks, P.a, P.pmin[0], P.pmin[1],
                               P.pmax[0], P.pmax[1], false, d1, d2, g, tid, NT, c1, c2);
      __syncthreads();
      stage_wtmap_mfma(L.W, nc, reinterpret_cast<const float*>(L.H), n, g.Tce, g.Tcs, gx, true,
                       nullptr, 0.f, false, dz, tid >> 6, NT >> 6, tid & 63);
    }
    __syncthreads();
  }

  const int L_ = A.L, k = A.ckpt_every;
  const int nseg = (L_ + k - 1) / k;
  float dz = 0.f;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int l0 = seg * k;
    const int l1 = min(L_, l0 + k);
    // recompute iterates l0 .. l1-1 into the segment scratch
    {
      float* xr = L.b0;
      float* xq = L.b1;
      const float* ck = A.ckpt + (size_t)seg * 2 * St + P.coef_off;
      float* sg = A.seg + P.coef_off;
      for (int s = tid; s < S; s += NT) {
        const float x = ck[s], lm = ck[St + s];
        xr[s] = x;
        L.b2[s] = lm;
        sg[s] = x;
        sg[St + s] = lm;
      }
      __syncthreads();
      for (int l = l0; l < l1 - 1; ++l) {
        sf_iteration<NT>(C, xr, xq, L.b2, L.b3, L.means, L.X, L.G, L.cx, false, dz, L.part);
        float* t = xr;
        xr = xq;
        xq = t;
        float* dst = A.seg + (size_t)(l + 1 - l0) * 2 * St + P.coef_off;
        for (int s = tid; s < S; s += NT) {
          dst[s] = xr[s];
          dst[St + s] = L.b2[s];
        }
      }
      __syncthreads();
    }
    for (int l = l1 - 1; l >= l0; --l) {
      const float* cur = A.seg + (size_t)(l - l0) * 2 * St + P.coef_off;
      const float* nxt = (l + 1 < l1) ? A.seg + (size_t)(l + 1 - l0) * 2 * St + P.coef_off
                         : (l1 == L_) ? A.fin + P.coef_off
                                      : A.ckpt + (size_t)(seg + 1) * 2 * St + P.coef_off;
      float* xbl = L.b0;
      float* gR = L.b2;
      float* fpx = L.b3;
      for (int s = tid; s < S; s += NT) {
        const float xl = cur[s];
        xbl[s] = xl;
        if (w != 0.f) {
          const float dxi = nxt[s] - xl;
          const float dla = nxt[St + s] - cur[St + s];
          gx[s] = fmaf(2.f * w, dxi, gx[s]);
          fpx[s] = -2.f * w * dxi;
          gR[s] = -2.f * rho * w * dla;
        } else {
          fpx[s] = 0.f;
          gR[s] = 0.f;
        }
      }
      __syncthreads();
      robot_means(gx, nullptr, n, nc, L.means, tid, NT);
      __syncthreads();
      for (int s = tid; s < S; s += NT) {
        const int ax = s / (n * nc), rem = s - ax * n * nc, i = rem / nc, c = rem - i * nc;
        const int row = ax * n * nc + i * nc;
        const float gu =
            mode_row_t(L.fac, L.fac + nc2, gx + row, L.means + ax * nc, nc, c, 0.f);
        gn[s] = mode_row_t(L.fac + 2 * nc2, L.fac + 3 * nc2, gx + row, L.means + ax * nc, nc,
                           c, fpx[s]);
        gR[s] = fmaf(-2.f * rho, gu, fmaf(-rho, L.glam[s], gR[s]));
        L.glam[s] += gu;
        L.gxi[s] += gu;
      }
      __syncthreads();
      for (int k0 = 0; k0 < T; k0 += Tc) {
        const Geo g = C.geo(k0);
        C.wchunk<NT>(k0, g.Tce);
        stage_xmap_mfma(L.W, nc, gR, n, reinterpret_cast<float*>(L.G), g.Tce, g.Tcs, nullptr, 0,
                        tid >> 6, NT >> 6, tid & 63);
        C.positions<NT>(xbl, L.X, g);
        stage_vjp_culled(L.X, L.G, L.H, n, L.obs, L.masks, P.a, P.pmin[0], P.pmin[1],
                         P.pmax[0], P.pmax[1], g, tid, NT);
        __syncthreads();
        stage_wtmap_mfma(L.W, nc, reinterpret_cast<const float*>(L.H), n, g.Tce, g.Tcs, gn,
                         true, nullptr, 0.f, false, dz, tid >> 6, NT >> 6, tid & 63);
      }
      __syncthreads();
      float* t = gx;
      gx = gn;
      gn = t;
    }
  }
  for (int s = tid; s < S; s += NT) {
    if (A.g_xi0) A.g_xi0[P.coef_off + s] = gx[s];
    if (A.g_lam0) A.g_lam0[P.coef_off + s] = L.glam[s];
    if (A.g_xi) A.g_xi[P.coef_off + s] = L.gxi[s];
  }
}

}  // namespace

size_t bwd_lds_bytes(int nc, int T, int Tc, int n_max, int M_max, int S_max, int) {
  auto r4 = [](int x) { return (size_t)((x + 3) & ~3); };
  const size_t Tcs = tstride(Tc);
  size_t f = r4(nc * Tc) + r4(fac_stride(nc)) + kRed + kMeans + (9 + kSplitMax) * r4(S_max) +
             4 * (size_t)M_max + box_floats(Tc, n_max) + mask_floats(Tc, n_max, M_max) +
             6 * (size_t)n_max * Tcs;
  return f * sizeof(float);
}

hipError_t launch_bwd_fused(const BwdArgs& a, int threads, size_t lds, hipStream_t s) {
  dim3 grid(a.B);
  switch (threads) {
    case 256:
      hipLaunchKernelGGL(bwd_fused_kernel<256>, grid, dim3(256), lds, s, a);
      break;
    case 512:
      hipLaunchKernelGGL(bwd_fused_kernel<512>, grid, dim3(512), lds, s, a);
      break;
    case 1024:
      hipLaunchKernelGGL(bwd_fused_kernel<1024>, grid, dim3(1024), lds, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t prepare_kernels(size_t lds) {
  const void* fns[] = {
      reinterpret_cast<const void*>(&fwd_fused_kernel<256>),
      reinterpret_cast<const void*>(&fwd_fused_kernel<512>),
      reinterpret_cast<const void*>(&fwd_fused_kernel<1024>),
      reinterpret_cast<const void*>(&bwd_fused_kernel<256>),
      reinterpret_cast<const void*>(&bwd_fused_kernel<512>),
      reinterpret_cast<const void*>(&bwd_fused_kernel<1024>)};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Plain path: the same steps as separate kernels over global memory, one
// problem per launch and every pair visited (the per-problem baseline the
// fused launch is compared with).
// ---------------------------------------------------------------------------
namespace {

__global__ __launch_bounds__(256) void plain_prep_kernel(FwdArgs A, PlainBufs Bf, int b) {
  __shared__ float means[kMeans];
  const ProbDesc P = A.probs[b];
  const int n = P.n, nc = A.nc, S = 2 * n * nc, tid = threadIdx.x;
  const float* fac = A.fac + (size_t)P.fac * fac_stride(nc);
  const float* tgt = A.xi + P.coef_off;
  const float* bnd = A.boundary + (size_t)P.rob_off * 4;
  robot_means(tgt, nullptr, n, nc, means, tid, 256);
  boundary_means(bnd, n, means + 2 * nc, tid, 256);
  __syncthreads();
  for (int s = tid; s < S; s += 256) {
    const int ax = s / (n * nc), rem = s - ax * n * nc, i = rem / nc, c = rem - i * nc;
    Bf.cxi[P.coef_off + s] =
        cxi_entry(fac, nc, tgt, means, bnd + i * 4, means + 2 * nc, n, ax, i, c);
    Bf.xb[0][P.coef_off + s] = A.xi0[P.coef_off + s];
    Bf.lam[P.coef_off + s] = A.lam0[P.coef_off + s];
  }
}

__global__ __launch_bounds__(256) void plain_xmap_kernel(FwdArgs A, PlainBufs Bf, int b,
                                                         int pp) {
  const ProbDesc P = A.probs[b];
  stage_xmap_mfma(A.W, A.nc, Bf.xb[pp] + P.coef_off, P.n, Bf.X + (size_t)P.pos_off * 2, A.T,
                  A.T, nullptr, 0, blockIdx.x * 4 + (threadIdx.x >> 6), gridDim.x * 4,
                  threadIdx.x & 63);
}

__global__ __launch_bounds__(256) void plain_constraint_kernel(FwdArgs A, PlainBufs Bf,
                                                               int b) {
  const ProbDesc P = A.probs[b];
  const int tid = blockIdx.x * 256 + threadIdx.x;
  float d1 = 0.f, d2 = 0.f;
  stage_constraints(reinterpret_cast<const float2*>(Bf.X) + P.pos_off,
                    reinterpret_cast<float2*>(Bf.V) + P.pos_off, P.n, A.T, A.T,
                    A.obstacles + (size_t)P.obs_off * 3, P.M, P.a, P.pmin[0], P.pmin[1],
                    P.pmax[0], P.pmax[1], false, d1, d2, tid, gridDim.x * 256);
}

__global__ __launch_bounds__(256) void plain_wtmap_kernel(FwdArgs A, PlainBufs Bf, int b) {
  const ProbDesc P = A.probs[b];
  const int S = 2 * P.n * A.nc;
  stage_wtmap_part(A.W, A.nc, Bf.V + (size_t)P.pos_off * 2, P.n, A.T, A.T,
                   Bf.part + (size_t)kSplitMax * P.coef_off, S, false,
                   blockIdx.x * 4 + (threadIdx.x >> 6), gridDim.x * 4, threadIdx.x & 63);
}

__global__ __launch_bounds__(256) void plain_update_kernel(FwdArgs A, PlainBufs Bf, int b,
                                                           int pp, int last) {
  __shared__ float means[kMeans];
  __shared__ float red[kRed];
  const ProbDesc P = A.probs[b];
  const int n = P.n, nc = A.nc, S = 2 * n * nc, tid = threadIdx.x, nc2 = nc * nc;
  const float rho = A.rho;
  const float* fac = A.fac + (size_t)P.fac * fac_stride(nc);
  float* R = Bf.R + P.coef_off;
  float* lam = Bf.lam + P.coef_off;
  float* xb = Bf.xb[pp] + P.coef_off;
  float* xn = Bf.xb[pp ^ 1] + P.coef_off;
  const float* cx = Bf.cxi + P.coef_off;
  float dzsq = 0.f;
  combine_lambda_means(Bf.part + (size_t)kSplitMax * P.coef_off, S, lam, R, xb, n, nc, rho,
                       last, dzsq, means, tid, 256);
  __syncthreads();
  for (int s = tid; s < S; s += 256) {
    const int ax = s / (n * nc), rem = s - ax * n * nc, i = rem / nc, c = rem - i * nc;
    const int row = ax * n * nc + i * nc;
    float v = mode_row(fac, fac + nc2, R + row, means + ax * nc, nc, c, cx[s]);
    v = mode_row(fac + 2 * nc2, fac + 3 * nc2, xb + row, means + 2 * nc + ax * nc, nc, c, v);
    xn[s] = v;
    if (last) {
      const float d = v - xb[s];
      dzsq = fmaf(d, d, dzsq);
    }
  }
  if (last) {
    float v[1] = {dzsq};
    block_sum(v, red);
    if (tid == 0) Bf.red[b * 4 + 2] = v[0];
  }
}

__global__ __launch_bounds__(256) void plain_final_kernel(FwdArgs A, PlainBufs Bf, int b,
                                                          int pp) {
  __shared__ float red[kRed];
  const ProbDesc P = A.probs[b];
  const int n = P.n, nc = A.nc, S = 2 * n * nc, tid = threadIdx.x;
  float r1sq = 0.f, r2sq = 0.f, bad = 0.f;
  stage_constraints(reinterpret_cast<const float2*>(Bf.X) + P.pos_off,
                    reinterpret_cast<float2*>(Bf.V) + P.pos_off, n, A.T, A.T,
                    A.obstacles + (size_t)P.obs_off * 3, P.M, P.a, P.pmin[0], P.pmin[1],
                    P.pmax[0], P.pmax[1], true, r1sq, r2sq, tid, 256);
  for (int s = tid; s < S; s += 256) {
    const float x = Bf.xb[pp][P.coef_off + s], lm = Bf.lam[P.coef_off + s];
    A.xi_out[P.coef_off + s] = x;
    A.lam_out[P.coef_off + s] = lm;
    if (!isfinite(x) || !isfinite(lm)) bad = 1.f;
  }
  float v[3] = {r1sq, r2sq, bad};
  block_sum(v, red);
  if (tid == 0) {
    float* res = A.residual + (size_t)b * 4;
    res[0] = sqrtf(v[0]);
    res[1] = sqrtf(v[1]);
    res[2] = A.L > 0 ? sqrtf(Bf.red[b * 4 + 2]) : 0.f;
    res[3] = (v[2] > 0.f || !isfinite(v[0]) || !isfinite(v[1])) ? 1.f : 0.f;
  }
}

__global__ void fill_kernel(float* p, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_plain_problem(const FwdArgs& a, const PlainBufs& pb, int b, hipStream_t s) {
  // grids sized for the batch's largest problem; the kernels stride over the
  // items of problem b
  const int tiles_x = ((a.T + 15) / 16) * ((2 * a.n_max + 15) / 16);
  const int tiles_w = ((a.nc + 15) / 16) * ((2 * a.n_max + 15) / 16) * kSplitMax;
  const int gx = (tiles_x + 3) / 4;             // four waves per block, a tile per wave
  const int gw = (tiles_w + 3) / 4;
  const int gc = (a.n_max * a.T + 255) / 256;
  hipLaunchKernelGGL(plain_prep_kernel, dim3(1), dim3(256), 0, s, a, pb, b);
  int pp = 0;
  for (int l = 0; l < a.L; ++l) {
    hipLaunchKernelGGL(plain_xmap_kernel, dim3(gx), dim3(256), 0, s, a, pb, b, pp);
    hipLaunchKernelGGL(plain_constraint_kernel, dim3(gc), dim3(256), 0, s, a, pb, b);
    hipLaunchKernelGGL(plain_wtmap_kernel, dim3(gw), dim3(256), 0, s, a, pb, b);
    hipLaunchKernelGGL(plain_update_kernel, dim3(1), dim3(256), 0, s, a, pb, b, pp,
                       (int)(l == a.L - 1));
    pp ^= 1;
  }
  hipLaunchKernelGGL(plain_xmap_kernel, dim3(gx), dim3(256), 0, s, a, pb, b, pp);
  hipLaunchKernelGGL(plain_final_kernel, dim3(1), dim3(256), 0, s, a, pb, b, pp);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace sf
