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
// Work decomposition.  Time is cut into windows of 16 steps.  A map phase
// computes the coefficient->time map of every window on MFMA (16x16x4 FP32
// tiles, one (window, column tile) job per wave in turn; on a list rebuild the
// per-window bounding box of every robot falls out of the tile).  After a
// block barrier, a wave owns a (window, robot part) unit and runs it end to
// end: candidate masks for its robots on a rebuild (a pair or obstacle is a
// candidate when the boxes come within the constraint distance plus a
// rounding margin; lane j tests robot j and a ballot forms the mask), the
// exact pair/obstacle/box stage over candidates (four lanes of four steps per
// robot, each robot walking its own list), and the window's share of the
// time->coefficient map R = W^T V on MFMA into a per-window partial.  Skipped
// pairs are inactive at every step of the window and contribute exactly 0.
// The partials are summed in window order, so every launch shape gives the
// same bits.
//
// The coefficient update is a set of MFMA tiles (axis x 16 robots x 16
// coefficients), one per wave: the wave forms its A operand u = lambda -
// 2 rho R straight from the partials, multiplies by the mode blocks, and gets
// the robot-mean term as column sums of a second accumulator (lane swaps),
// exchanged between row tiles through LDS.  Four block barriers per
// iteration: after the map phase, after the window units, after the column
// sums, after the update.
//
// Data layout: coefficient arrays [axis][robot][coef]; positions and
// constraint sums [robot][time] as float2 (x, y) with an odd row stride
// (window multiple + 1) to spread robots over LDS banks; W as [T][nc].
#include <hip/hip_runtime.h>

#include <mutex>

#include "sf_internal.h"

namespace sf {

namespace {

constexpr int kRed = 64;      // floats of LDS reduction scratch
constexpr int kMeans = 4 * kMaxCoef + 8;
constexpr int kMaxParts = 4;  // waves sharing one window
constexpr int kMaxWaves = 16; // waves of the largest workgroup

typedef unsigned long long u64;
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int round4(int x) { return (x + 3) & ~3; }

// Row stride (in steps) of the position/sum buffers: a window multiple plus
// one, so that the 2*stride-float rows of different robots start in different
// LDS banks.
__host__ __device__ __forceinline__ int tstride(int Tc) { return ((Tc + 15) & ~15) + 1; }
__host__ __device__ __forceinline__ int nwindows(int Tc) { return (Tc + 15) >> 4; }

// D += A B for a 16x4 by 4x16 FP32 tile: lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[4(l/16)+v][l%16] in element v.
__device__ __forceinline__ floatx4 mfma_16x16x4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// The lane index through an empty asm statement: values derived from it are
// recomputed where used instead of being hoisted out of the iteration loop
// and kept live (and spilled) across it.
__device__ __forceinline__ int lane_here(int tid) {
  int l = tid & 63;
  asm volatile("" : "+v"(l));
  return l;
}

// The wave's index in the block as a wave-uniform (scalar) value, so that
// everything derived from it (unit, window, part, tile, robot ranges) is
// scalar code and uniform control flow.
__device__ __forceinline__ int wave_id(int tid) {
  return __builtin_amdgcn_readfirstlane(tid >> 6);
}

// Orders the LDS accesses of one wave (its stores before its later loads).
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
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

// Combine the four 16-lane rows of a wave column-wise (lanes m, m+16, m+32,
// m+48): lanes l and l^32 first, then l and l^16, through the gfx950 lane-swap
// instructions (VALU, no LDS trip).  Every lane gets the result; the order of
// the operations is the same in every lane (op is commutative).
template <typename Op>
__device__ __forceinline__ float rows_reduce(float v, Op op) {
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  v = op(__uint_as_float(p[0]), __uint_as_float(p[1]));
  const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  return op(__uint_as_float(q[0]), __uint_as_float(q[1]));
}
struct OpAdd {
  __device__ float operator()(float a, float b) const { return a + b; }
};
// Min/max as compare-and-select (no NaN canonicalisation; a non-finite box
// only has to fail its tests, which it does either way).
__device__ __forceinline__ float min_sel(float a, float b) { return b < a ? b : a; }
__device__ __forceinline__ float max_sel(float a, float b) { return b > a ? b : a; }
struct OpMin {
  __device__ float operator()(float a, float b) const { return min_sel(a, b); }
};
struct OpMax {
  __device__ float operator()(float a, float b) const { return max_sel(a, b); }
};

// Deterministic block sum of up to 4 values: wave sums, then a fixed-order
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

// ---------------------------------------------------------------------------
// Window stages.  Xf/Vf are float views of [robot][step] float2 arrays with
// row stride Ts steps; steps are chunk-local.  Columns of the map tiles are
// (robot, axis) pairs col = 2 i + axis, 16 per tile (8 robots).
// ---------------------------------------------------------------------------

// t-th robot of part h when 8-robot groups are dealt round-robin to H parts.
__device__ __forceinline__ int part_robot(int t, int h, int H) {
  return ((t >> 3) * H + h) * 8 + (t & 7);
}

// Robots in part h (h < number of 8-robot groups).
__device__ __forceinline__ int part_count(int n, int h, int H) {
  const int ng = (n + 7) >> 3;
  const int mine = (ng - h + H - 1) / H;
  int cnt = 8 * mine;
  if ((ng - 1) % H == h) cnt -= 8 * ng - n;
  return cnt;
}

// Rounding margins of the candidate tests for a robot whose window box has
// largest coordinate magnitude s: pairs use a(1 + 1e-4) + 4e-6 (1 + s + 2a),
// obstacles r_o(1 + 1e-4) + 8e-6 r_o (on the obstacle's side) plus
// 4e-6 (1 + s) (on the robot's side).  They exceed the distance threshold by
// far more than the float rounding of the exact tests and of the box sums, so
// a pair or obstacle outside them is inactive at every step of the window.
//
// Candidate lists are kept across iterations with a skin d (neighbour lists
// in the molecular-dynamics sense): they are built with the pair margin
// widened by 2d and the robot-side obstacle margin by d, together with a
// reference copy of every robot's box.  As long as no robot's box has grown
// by more than d beyond its reference in any direction, every pair or
// obstacle that can be active is still on the lists; the first iteration in
// which one has, rebuilds the window's lists.  Culling stays exact.
__device__ __forceinline__ float pair_margin(float a, float s) {
  return fmaf(4e-6f, 1.f + s + 2.f * a, a * 1.0001f);
}
__device__ __forceinline__ float robot_obs_margin(float s) { return 4e-6f * (1.f + s); }
__device__ __forceinline__ float obs_margin(float ao) { return fmaf(8e-6f, ao, ao * 1.0001f); }

// Coefficient -> time map of window w for all robots: X[i][16w + r].axis =
// sum_c W[16w + r][c] xb[axis][i][c] for steps < Tce (padding rows repeat the
// last step).  With BOX, each robot's window box (xmin, xmax, ymin, ymax) goes
// to box[i nws + w].  PADDED: rows have room for the padding steps, which are
// then stored too (no per-row guard).  Column tiles are taken four at a time
// with all their operand loads issued before the MFMA chains.
template <int KS, bool BOX, bool PADDED>
__device__ __forceinline__ void xmap_window(const float* __restrict__ W, int nc,
                                            const float* __restrict__ xb, int n,
                                            float* __restrict__ Xf, int Ts, int w, int Tce,
                                            float* __restrict__ box, int nws, int lane) {
  const int ncol = (2 * n + 15) >> 4;
  const int m = lane & 15, kq = lane >> 4;
  const int row = min(w * 16 + m, Tce - 1);
  float av[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int c = 4 * s + kq;
    const float v = W[__umul24(row, nc) + min(c, nc - 1)];
    av[s] = c < nc ? v : 0.f;
  }
  const int k0 = w * 16 + 4 * kq;
  for (int nt0 = 0; nt0 < ncol; nt0 += 4) {
    // B at clamped entries: A is zero past nc, padded columns are not stored
    float bv[4][KS];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int col = (nt0 + g) * 16 + m;
      const int i = min(col >> 1, n - 1), ax = col & 1;
      const float* brow = xb + __umul24(ax * n + i, nc);
#pragma unroll
      for (int s = 0; s < KS; ++s) bv[g][s] = brow[min(4 * s + kq, nc - 1)];
    }
    floatx4 acc[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      acc[g] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s) acc[g] = mfma_16x16x4(av[s], bv[g][s], acc[g]);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      if (nt0 + g >= ncol) break;
      const int col = (nt0 + g) * 16 + m;
      const int i = col >> 1, ax = col & 1;
      const bool colok = i < n;
      if (colok) {
        float* xr = Xf + (__umul24(i, Ts) + k0) * 2 + ax;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (PADDED || k0 + v < Tce) xr[2 * v] = acc[g][v];
      }
      if (BOX) {
        float lo = min_sel(min_sel(acc[g][0], acc[g][1]), min_sel(acc[g][2], acc[g][3]));
        float hi = max_sel(max_sel(acc[g][0], acc[g][1]), max_sel(acc[g][2], acc[g][3]));
        lo = rows_reduce(lo, OpMin());
        hi = rows_reduce(hi, OpMax());
        if (lane < 16 && colok)
          *reinterpret_cast<float2*>(box + (__umul24(i, nws) + w) * 4 + 2 * ax) =
              make_float2(lo, hi);
      }
    }
  }
}

// One job of the fused kernels' map phase: column tile nt (8 robots x 2 axes)
// of window w, X[i][16w + r].axis = sum_c W[16w + r][c] xb[axis][i][c], the
// padding rows stored too (rows have room for them); with BOX the tile's
// window boxes go to box[i nws + w].  Same MFMA chain, hence the same bits, as
// the tile in xmap_window.
template <int KS, bool BOX>
__device__ __forceinline__ void xmap_tile(const float* __restrict__ W, int nc,
                                          const float* __restrict__ xb, int n,
                                          float* __restrict__ Xf, int Ts, int w, int nt, int Tce,
                                          float* __restrict__ box, int nws, int lane) {
  const int m = lane & 15, kq = lane >> 4;
  const int row = min(w * 16 + m, Tce - 1);
  const int col = nt * 16 + m;
  const int i = min(col >> 1, n - 1), ax = col & 1;
  const float* brow = xb + __umul24(ax * n + i, nc);
  float av[KS], bv[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int c = 4 * s + kq;
    const float v = W[__umul24(row, nc) + min(c, nc - 1)];
    av[s] = c < nc ? v : 0.f;
    bv[s] = brow[min(c, nc - 1)];
  }
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < KS; ++s) acc = mfma_16x16x4(av[s], bv[s], acc);
  const bool colok = (col >> 1) < n;
  if (colok) {
    float* xr = Xf + (__umul24(i, Ts) + w * 16 + 4 * kq) * 2 + ax;
#pragma unroll
    for (int v = 0; v < 4; ++v) xr[2 * v] = acc[v];
  }
  if (BOX) {
    float lo = min_sel(min_sel(acc[0], acc[1]), min_sel(acc[2], acc[3]));
    float hi = max_sel(max_sel(acc[0], acc[1]), max_sel(acc[2], acc[3]));
    lo = rows_reduce(lo, OpMin());
    hi = rows_reduce(hi, OpMax());
    if (lane < 16 && colok)
      *reinterpret_cast<float2*>(box + (__umul24(i, nws) + w) * 4 + 2 * ax) = make_float2(lo, hi);
  }
}

// Map phase of a chunk: the (window, column tile) jobs dealt to the block's
// waves round-robin, so each window's positions are computed once rather than
// by every unit of the window.
template <int NT, int KS, bool BOX>
__device__ __forceinline__ void map_chunk(const float* __restrict__ W, int nc,
                                          const float* __restrict__ src, int n,
                                          float* __restrict__ dst, int Ts, int Tce,
                                          float* __restrict__ box, int nws, int wave, int lane) {
  constexpr int nwaves = NT >> 6;
  const int nwin = nwindows(Tce), ncol = (2 * n + 15) >> 4;
  int w = wave / ncol, nt = wave - w * ncol;
  for (; w < nwin;) {
    xmap_tile<KS, BOX>(W, nc, src, n, dst, Ts, w, nt, Tce, box, nws, lane);
    nt += nwaves;
    while (nt >= ncol) {
      nt -= ncol;
      ++w;
    }
  }
}

// Candidate masks (32-bit words) of window w for the robots of part h.  Word q
// of robot i's pair mask (at mw[q * mrow + i]) has bit jj set when robot
// j = 32 q + jj (j != i) has a window box meeting robot i's box widened by the
// pair margin plus twice the skin; obstacle word q (at mw[(mpw + q) * mrow + i])
// likewise for obstacle 32 q + jj, whose box is already widened by its own
// margin, against robot i's box widened by the robot-side margin plus the
// skin.  A ballot tests two robots at once (lane = 32 slot + jj) and one 64-bit
// store writes both words: robots t0 and t0 + 1 of a part are adjacent rows.
__device__ __forceinline__ float4 widened(float4 b, float d) {
  return make_float4(b.x - d, b.y + d, b.z - d, b.w + d);
}
__device__ __forceinline__ float box_magnitude(float4 b) {
  return fmaxf(fmaxf(fabsf(b.x), fabsf(b.y)), fmaxf(fabsf(b.z), fabsf(b.w)));
}

__device__ __forceinline__ void masks_window(const float4* __restrict__ box, int n,
                                             const float4* __restrict__ obox, int M, float a,
                                             float skin, unsigned* __restrict__ mw, int mrow,
                                             int mpw, int nws, int w, int h, int H, int lane) {
  const int cnt = part_count(n, h, H);
  const int slot = lane >> 5, jj = lane & 31;
  for (int q = 0; q < ((n + 31) >> 5); ++q) {
    const int j = q * 32 + jj;
    const float4 bj = box[__umul24(min(j, n - 1), nws) + w];
    const bool jl = j < n;
    for (int t0 = 0; t0 < cnt; t0 += 2) {
      const bool tl = t0 + slot < cnt;
      const int i = part_robot(tl ? t0 + slot : t0, h, H);
      const float4 bi = box[__umul24(i, nws) + w];
      const float4 ei = widened(bi, fmaf(2.f, skin, pair_margin(a, box_magnitude(bi))));
      const bool c = tl && jl && (j != i) && (ei.x < bj.y) && (bj.x < ei.y) && (ei.z < bj.w) &&
                     (bj.z < ei.w);
      const u64 b = __builtin_amdgcn_ballot_w64(c);
      if (lane == 0)
        *reinterpret_cast<u64*>(mw + q * mrow + part_robot(t0, h, H)) = b;
    }
  }
  for (int q = 0; q < ((M + 31) >> 5); ++q) {
    const int mo = q * 32 + jj;
    const float4 ob = obox[min(mo, M - 1)];
    const bool ml = mo < M;
    for (int t0 = 0; t0 < cnt; t0 += 2) {
      const bool tl = t0 + slot < cnt;
      const int i = part_robot(tl ? t0 + slot : t0, h, H);
      const float4 bi = box[__umul24(i, nws) + w];
      const float4 ei = widened(bi, robot_obs_margin(box_magnitude(bi)) + skin);
      const bool c = tl && ml && (ob.x < ei.y) && (ei.x < ob.y) && (ob.z < ei.w) && (ei.z < ob.w);
      const u64 b = __builtin_amdgcn_ballot_w64(c);
      if (lane == 0)
        *reinterpret_cast<u64*>(mw + (mpw + q) * mrow + part_robot(t0, h, H)) = b;
    }
  }
}

// Validity of the candidate lists, checked on coefficients.  A robot's
// position is a convex combination of its coefficients (Bernstein basis of eq.
// poly: non-negative weights summing to one), so on each axis no position moves
// further than the largest change of that axis's coefficients.  The lists stay
// valid while no coefficient differs from its value at the last rebuild by more
// than the skin.  Each wave records in its slot whether a coefficient it
// compared moved further; the units rebuild when any slot is set.
__device__ __forceinline__ void note_moved(bool moved, int* __restrict__ slots, int wave,
                                           int lane) {
  const bool any = __builtin_amdgcn_ballot_w64(moved) != 0ull;
  if (lane == 0) slots[wave] = any ? 1 : 0;
}
__device__ __forceinline__ bool lists_moved(const int* __restrict__ slots, int nwaves,
                                            int lane) {
  const int v = lane < nwaves ? slots[lane] : 0;
  return __builtin_amdgcn_ballot_w64(v != 0) != 0ull;
}
// Block-wide check of the iterate x against the reference coefficients; a
// thread compares the entries it wrote itself, so no barrier is needed before.
template <int NT>
__device__ __forceinline__ void check_lists(const float* __restrict__ x,
                                            const float* __restrict__ ref, int S, float skin,
                                            int* __restrict__ slots, int tid) {
  bool moved = false;
  for (int s = tid; s < S; s += NT) moved |= !(fabsf(x[s] - ref[s]) <= skin);
  note_moved(moved, slots, wave_id(tid), tid & 63);
}

// Next candidate of a lane's mask word (lowest set bit) plus base (a multiple
// of 32), or -1 when the word is empty (find-first-bit gives -1 there).
__device__ __forceinline__ int pop_candidate(unsigned& u, int base) {
  const int b = __ffs(u) - 1;
  u &= u - 1u;
  return b | base;
}

// 1/sqrt(d2) by the hardware reciprocal square root (1 ulp) on an input held
// at or above the smallest normal float (a median-of-three clamp), so that no
// input is flushed; only the coincident case d2 = 0 reaches the clamp.
__device__ __forceinline__ float rsqrt_clamped(float d2) {
  return __builtin_amdgcn_rsqf(__builtin_amdgcn_fmed3f(d2, 1.17549435e-38f, 3.40282347e+38f));
}

// Residual vector of a pair at difference (dx, dy) with d2 = |D|^2 < a^2:
// (1 - a/|D|) D, and (-a, 0) from robot i's side of a coincident pair with
// i < j (alpha = atan2(0, 0) = 0), (a, 0) from the other side.  Branch-free:
// at D = 0 the products f D are zero (f is finite there) and the tie adds
// its (-+a, 0).
__device__ __forceinline__ void pair_residual(float dx, float dy, float d2, float a, bool lower,
                                              float& rx, float& ry) {
  const float f = fmaf(-a, rsqrt_clamped(d2), 1.f);
  const float tie = d2 > 0.f ? 0.f : (lower ? -a : a);
  rx = fmaf(f, dx, tie);
  ry = f * dy;
}

// Exact constraint stage of window w for the robots of part h: 16 robots per
// pass, four lanes per robot and four consecutive steps per lane, so that a
// popped candidate serves 4 steps of each lane and the pass overhead is shared
// by 16 robots.  V = w_pair (pair + obstacle sums) + w_box (box residual).
// Each robot walks its own candidates in increasing index (pairs, then
// obstacles), two per round so their loads overlap; skipped pairs are
// inactive and would add exactly 0.  Every step's sums are formed in candidate
// order.  Position rows hold finite values up to the window's last padding
// step, so the reads need no clamp.  With ACCUM, ||r_1||^2 (each unordered
// pair once) and ||r_2||^2.
constexpr int kStepsPerLane = 4;

template <bool ACCUM, bool MOVING>
__device__ __forceinline__ void constraints_window(
    const float2* __restrict__ X, float2* __restrict__ V, int n, int Ts,
    const float4* __restrict__ obs, const float2* __restrict__ ovel, int kg, float inv_Tm1,
    int M, const unsigned* __restrict__ mw, int mrow, int mpw,
    float a, float pmin0, float pmin1, float pmax0, float pmax1, int w, int Tce, int h, int H,
    float& r1sq, float& r2sq, float w_pair, float w_box, int lane) {
  constexpr int E = kStepsPerLane, LPR = 16 / E;
  const float a2 = a * a;
  const int k0 = w * 16 + E * (lane & (LPR - 1));
  // tau of this lane's steps (global step kg + k0 + e), for moving obstacles
  float tau[E];
#pragma unroll
  for (int e = 0; e < E; ++e) tau[e] = MOVING ? (float)(kg + k0 + e) * inv_Tm1 : 0.f;
  const int cnt = part_count(n, h, H);
  for (int t0 = 0; t0 < cnt; t0 += 64 / LPR) {
    const int t = t0 + lane / LPR;
    const bool live = t < cnt;
    const int i = part_robot(live ? t : t0, h, H);
    const float2* xi = X + __umul24(i, Ts) + k0;
    float2 p[E];
    float vx[E], vy[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      p[e] = xi[e];
      vx[e] = 0.f;
      vy[e] = 0.f;
    }
    float s1 = 0.f;
    for (int wq = 0; wq < ((n + 31) >> 5); ++wq) {
      unsigned u = live ? mw[wq * mrow + i] : 0u;
      while (u != 0u) {
        int j[2];
        float2 o[2][E];
#pragma unroll
        for (int q = 0; q < 2; ++q) j[q] = pop_candidate(u, wq * 32);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float2* xj = X + __umul24(max(j[q], 0), Ts) + k0;
#pragma unroll
          for (int e = 0; e < E; ++e) o[q][e] = xj[e];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const float dx = p[e].x - o[q][e].x;
            const float dy = p[e].y - o[q][e].y;
            const float d2 = fmaf(dy, dy, dx * dx);
            if (j[q] >= 0 && d2 < a2) {
              float rx, ry;
              pair_residual(dx, dy, d2, a, i < j[q], rx, ry);
              vx[e] += rx;
              vy[e] += ry;
              if (ACCUM && j[q] > i && k0 + e < Tce) s1 = fmaf(rx, rx, fmaf(ry, ry, s1));
            }
          }
        }
      }
    }
    for (int wd = 0; wd < ((M + 31) >> 5); ++wd) {
      unsigned u = live ? mw[(mpw + wd) * mrow + i] : 0u;
      while (u != 0u) {
        int mq[2];
        float4 ob[2];
        float2 ov[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) mq[q] = pop_candidate(u, wd * 32);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          ob[q] = obs[max(mq[q], 0)];
          if (MOVING) ov[q] = ovel[max(mq[q], 0)];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const float cx = MOVING ? fmaf(ov[q].x, tau[e], ob[q].x) : ob[q].x;
            const float cy = MOVING ? fmaf(ov[q].y, tau[e], ob[q].y) : ob[q].y;
            const float dx = p[e].x - cx;
            const float dy = p[e].y - cy;
            const float d2 = fmaf(dy, dy, dx * dx);
            if (mq[q] >= 0 && d2 < ob[q].w) {
              float rx, ry;
              pair_residual(dx, dy, d2, ob[q].z, true, rx, ry);
              vx[e] += rx;
              vy[e] += ry;
              if (ACCUM && k0 + e < Tce) s1 = fmaf(rx, rx, fmaf(ry, ry, s1));
            }
          }
        }
      }
    }
    if (!live) continue;
    float2* vi = V + __umul24(i, Ts) + k0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (k0 + e >= Tce) break;
      const float hx = fmaxf(p[e].x - pmax0, 0.f), lx = fmaxf(pmin0 - p[e].x, 0.f);
      const float hy = fmaxf(p[e].y - pmax1, 0.f), ly = fmaxf(pmin1 - p[e].y, 0.f);
      vi[e] = make_float2(fmaf(w_box, hx - lx, w_pair * vx[e]),
                          fmaf(w_box, hy - ly, w_pair * vy[e]));
      if (ACCUM) r2sq += hx * hx + lx * lx + hy * hy + ly * ly;
    }
    if (ACCUM) r1sq += s1;
  }
}

// Contribution of one active pair or obstacle to the vector-Jacobian product:
// J(D) w with J(D) = (1 - f) I + f u u^T, f = a/|D|, u = D/|D|; at D = 0 the
// e of the alpha/d steps is locally constant, so J = I.
// Branch-free: at D = 0, f is set to 0 (J = I) and u = 0; a zero w adds
// exactly nothing, which is how inactive tests are masked.
__device__ __forceinline__ void vjp_term(float dx, float dy, float d2, float a, float wx,
                                         float wy, float& hx, float& hy) {
  const float inv = rsqrt_clamped(d2);
  const float f = d2 > 0.f ? a * inv : 0.f;
  const float ux = dx * inv, uy = dy * inv;
  const float c = f * fmaf(ux, wx, uy * wy);
  const float omf = 1.f - f;
  hx = fmaf(c, ux, fmaf(omf, wx, hx));
  hy = fmaf(c, uy, fmaf(omf, wy, hy));
}

// Vector-Jacobian product of the constraint stage over window w for the robots
// of part h: given the cotangent G of V at positions X,
//   H_i = sum_{j != i} J(X_i - X_j) (G_i - G_j) + sum_m J_o(X_i - c_m) G_i
//         + box'(X_i) G_i,
// J the Jacobian of r(D) = D - e(D) on active pairs (|D| < a), 0 otherwise.
// Same walk over candidates as the constraint stage.
template <bool MOVING>
__device__ __forceinline__ void vjp_window(const float2* __restrict__ X,
                                           const float2* __restrict__ G, float2* __restrict__ Hb,
                                           int n, int Ts, const float4* __restrict__ obs,
                                           const float2* __restrict__ ovel, int kg,
                                           float inv_Tm1, int M,
                                           const unsigned* __restrict__ mw, int mrow,
                                           int mpw, float a, float pmin0, float pmin1,
                                           float pmax0, float pmax1, int w, int Tce, int h, int H,
                                           int lane) {
  constexpr int E = kStepsPerLane, LPR = 16 / E;
  const float a2 = a * a;
  const int k0 = w * 16 + E * (lane & (LPR - 1));
  float tau[E];
#pragma unroll
  for (int e = 0; e < E; ++e) tau[e] = MOVING ? (float)(kg + k0 + e) * inv_Tm1 : 0.f;
  const int cnt = part_count(n, h, H);
  for (int t0 = 0; t0 < cnt; t0 += 64 / LPR) {
    const int t = t0 + lane / LPR;
    const bool live = t < cnt;
    const int i = part_robot(live ? t : t0, h, H);
    const float2* xi = X + __umul24(i, Ts) + k0;
    const float2* gip = G + __umul24(i, Ts) + k0;
    float2 p[E], gi[E];
    float hx[E], hy[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      p[e] = xi[e];
      gi[e] = gip[e];
      hx[e] = 0.f;
      hy[e] = 0.f;
    }
    for (int wq = 0; wq < ((n + 31) >> 5); ++wq) {
      unsigned u = live ? mw[wq * mrow + i] : 0u;
      while (u != 0u) {
        int j[2], row[2];
        float2 o[2][E];
#pragma unroll
        for (int q = 0; q < 2; ++q) j[q] = pop_candidate(u, wq * 32);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          row[q] = __umul24(max(j[q], 0), Ts) + k0;
#pragma unroll
          for (int e = 0; e < E; ++e) o[q][e] = X[row[q] + e];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          float dx[E], dy[E], d2[E];
          bool act[E], any = false;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            dx[e] = p[e].x - o[q][e].x;
            dy[e] = p[e].y - o[q][e].y;
            d2[e] = fmaf(dy[e], dy[e], dx[e] * dx[e]);
            act[e] = j[q] >= 0 && d2[e] < a2;
            any |= act[e];
          }
          // the candidate's cotangents are read only when one of its tests
          // is active; then all four steps are formed, inactive ones with a
          // zero cotangent
          if (any) {
            float2 gj[E];
#pragma unroll
            for (int e = 0; e < E; ++e) gj[e] = G[row[q] + e];
#pragma unroll
            for (int e = 0; e < E; ++e) {
              const float wx = act[e] ? gi[e].x - gj[e].x : 0.f;
              const float wy = act[e] ? gi[e].y - gj[e].y : 0.f;
              vjp_term(dx[e], dy[e], d2[e], a, wx, wy, hx[e], hy[e]);
            }
          }
        }
      }
    }
    for (int wd = 0; wd < ((M + 31) >> 5); ++wd) {
      unsigned u = live ? mw[(mpw + wd) * mrow + i] : 0u;
      while (u != 0u) {
        int mq[2];
        float4 ob[2];
        float2 ov[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) mq[q] = pop_candidate(u, wd * 32);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          ob[q] = obs[max(mq[q], 0)];
          if (MOVING) ov[q] = ovel[max(mq[q], 0)];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const float cx = MOVING ? fmaf(ov[q].x, tau[e], ob[q].x) : ob[q].x;
            const float cy = MOVING ? fmaf(ov[q].y, tau[e], ob[q].y) : ob[q].y;
            const float dx = p[e].x - cx;
            const float dy = p[e].y - cy;
            const float d2 = fmaf(dy, dy, dx * dx);
            if (mq[q] >= 0 && d2 < ob[q].w)
              vjp_term(dx, dy, d2, ob[q].z, gi[e].x, gi[e].y, hx[e], hy[e]);
          }
        }
      }
    }
    if (!live) continue;
    float2* hi = Hb + __umul24(i, Ts) + k0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (k0 + e >= Tce) break;
      float ox = hx[e], oy = hy[e];
      if (p[e].x > pmax0 || p[e].x < pmin0) ox += gi[e].x;
      if (p[e].y > pmax1 || p[e].y < pmin1) oy += gi[e].y;
      hi[e] = make_float2(ox, oy);
    }
  }
}

// Window w's share of the time->coefficient map for the column tiles of part
// h (tiles nt = h, h+H, ...): part_w[axis][i][c] (+)= sum over the window's
// steps of W[k][c] V[i][k].axis.  The W^T operands of the window stay in
// registers across the column tiles.
template <int KS>
__device__ __forceinline__ void wtmap_window(const float* __restrict__ W, int nc,
                                             const float* __restrict__ Vf, int n, int Ts, int w,
                                             int Tce, int h, int H, float* __restrict__ part_w,
                                             bool accumulate, int lane) {
  constexpr int NCT = (KS + 3) / 4;   // coefficient tiles of 16
  const int nct = (nc + 15) >> 4;
  const int ncol = (2 * n + 15) >> 4;
  const int m = lane & 15, kq = lane >> 4;
  float av[NCT][4];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    const int ca = ct * 16 + m;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = w * 16 + 4 * s + kq;
      const float v = W[__umul24(min(kk, Tce - 1), nc) + min(ca, nc - 1)];
      av[ct][s] = (kk < Tce && ca < nc) ? v : 0.f;
    }
  }
  for (int nt = h; nt < ncol; nt += H) {
    const int col = nt * 16 + m;
    const int i = col >> 1, ax = col & 1;
    const bool colok = i < n;
    const float* vrow = Vf + __umul24(min(i, n - 1), Ts) * 2 + ax;
    // V at clamped steps: the W^T operand is zero past Tce, padded columns
    // are not stored
    float bv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) bv[s] = vrow[2 * min(w * 16 + 4 * s + kq, Tce - 1)];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      if (ct >= nct) break;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = mfma_16x16x4(av[ct][s], bv[s], acc);
      if (colok) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = ct * 16 + 4 * kq + v;
          if (c >= nc) continue;
          const int sidx = __umul24(ax * n + i, nc) + c;
          part_w[sidx] = accumulate ? part_w[sidx] + acc[v] : acc[v];
        }
      }
    }
  }
}

// Waves per window: enough (window, part) units for the block's waves, at most
// kMaxParts and at most one part per 8-robot group.
__device__ __forceinline__ int parts_per_window(int n, int nwin, int nwaves) {
  int H = nwaves / max(nwin, 1);
  H = min(H, kMaxParts);
  H = min(H, (n + 7) >> 3);
  return max(H, 1);
}

// ---------------------------------------------------------------------------
// Coefficient-space stages.
// ---------------------------------------------------------------------------

// Robot means of the columns of one coefficient array into out[axis*nc + c].
__device__ __forceinline__ void robot_means(const float* __restrict__ src, int n, int nc,
                                            float* __restrict__ out, int wave, int nwaves,
                                            int lane) {
  const float inv = 1.f / (float)n;
  for (int col = wave; col < 2 * nc; col += nwaves) {
    const int ax = col / nc, c = col - ax * nc;
    const float* base = src + ax * n * nc + c;
    float s = 0.f;
    for (int i = lane; i < n; i += 64) s += base[i * nc];
    s = wave_sum_dpp(s);
    if (lane == 0) out[col] = s * inv;
  }
}

// Mode products on MFMA tiles.  A problem's operator acts on a coefficient
// array Y (rows = robots) as
//   (S Y)_i = P_perp Y_i + (P_par - P_perp) mean_j(Y_j)
// (S^T: transposed blocks).  A tile covers one axis, 16 robots (row tile rt)
// and 16 output coefficients (column tile ct); lanes supply A[m][k] =
// Y[16 rt + m][4 s + kq] (m = lane % 16, kq = lane / 16) for s < KS, and hold
// outputs [16 rt + 4 kq + v][16 ct + m].  The mean term is formed as the
// column sums of D Y over the block's robots (rows past n are zero), summed
// over row tiles through LDS between two block-synchronised phases.
constexpr int kTilesMax = 16;    // 2 axes x 4 row tiles x 2 column tiles
constexpr int kColSums = 2 * 2 * 4 * 16;

__host__ __device__ constexpr int tiles_per_wave(int NT) {
  return (kTilesMax + (NT >> 6) - 1) / (NT >> 6);
}

struct Tile {
  int ax, rt, ct;
};
// Tile slots: ax | rt << 1 | ct << 3 (16 slots for up to 4 row tiles and 2
// column tiles); slots beyond the problem's tiles are empty.  The active
// slots of small problems are the first ones, so they land on different SIMDs.
__device__ __forceinline__ bool mode_tile_of(int tile, int n, int nc, Tile& t) {
  t.ax = tile & 1;
  t.rt = (tile >> 1) & 3;
  t.ct = tile >> 3;
  return t.rt < ((n + 15) >> 4) && t.ct < ((nc + 15) >> 4);
}
__device__ __forceinline__ int colsum_slot(const Tile& t, int rt) {
  return ((t.ax * 2 + t.ct) * 4 + rt) * 16;
}

// B operands of the block (P, D) at fac + fo (transposed with `trans`) for
// output column cb.  B is read at clamped (finite) entries: A is zero at
// padded k, and padded output columns are never used.
template <int KS>
__device__ __forceinline__ void mode_operands(const float* __restrict__ fac, int nc, int fo,
                                              bool trans, int cb, float (&bp)[KS],
                                              float (&bd)[KS], int lane) {
  const int kq = lane >> 4;
  const int nc2 = nc * nc;
  const int cbc = min(cb, nc - 1);
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int kc = min(4 * s + kq, nc - 1);
    const int idx = trans ? __umul24(kc, nc) + cbc : __umul24(cbc, nc) + kc;
    bp[s] = fac[fo + idx];
    bd[s] = fac[fo + nc2 + idx];
  }
}

// accP += Y P^(T) and accD += Y D^(T) from the operands of mode_operands.
template <int KS>
__device__ __forceinline__ void mode_mfma(const float (&a)[KS], const float (&bp)[KS],
                                          const float (&bd)[KS], floatx4& accP, floatx4& accD) {
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    accP = mfma_16x16x4(a[s], bp[s], accP);
    accD = mfma_16x16x4(a[s], bd[s], accD);
  }
}

// R entries of a tile's lanes: the per-window partials summed in window order
// (r = part_0 + part_1 + ...), the reads of G windows issued together (reads
// past the last window are clamped and unused).
template <int KS, int G>
__device__ __forceinline__ void window_sum(const float* __restrict__ part, int nwin, int S,
                                           const int (&sidx)[KS], float (&r)[KS]) {
#pragma unroll
  for (int s = 0; s < KS; ++s) r[s] = 0.f;   // replaced by window 0, not added to
  for (int w0 = 0; w0 < nwin; w0 += G) {
    float pv[G][KS];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const float* pw = part + min(w0 + g, nwin - 1) * S;
#pragma unroll
      for (int s = 0; s < KS; ++s) pv[g][s] = pw[sidx[s]];
    }
    // selects, not branches, so that every read above stays ahead of the adds
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const bool first = w0 + g == 0, live = w0 + g < nwin;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const float sum = r[s] + pv[g][s];
        r[s] = first ? pv[g][s] : (live ? sum : r[s]);
      }
    }
  }
}

// Column sum of a D accumulator over the tile's 16 robots, written for the
// later mean.
__device__ __forceinline__ void put_colsum(const floatx4& accD, float* __restrict__ csum,
                                           const Tile& t, int lane) {
  const float cs = rows_reduce((accD[0] + accD[1]) + (accD[2] + accD[3]), OpAdd());
  if (lane < 16) csum[colsum_slot(t, t.rt) + lane] = cs;
}
__device__ __forceinline__ float get_mean(const float* __restrict__ csum, const Tile& t, int n,
                                          int lane) {
  // all four row-tile slots are read at once; those past the problem's row
  // tiles (stale contents) are not added
  const int nrt = (n + 15) >> 4;
  float v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = csum[colsum_slot(t, r) + (lane & 15)];
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < 4; ++r) s = r < nrt ? s + v[r] : s;
  return s * (1.f / (float)n);
}

// Forward update, phase 1 (tiles of this wave): R = sum of the per-window
// partials in window order; lambda' = lambda - rho R into lam_n; u = lambda -
// 2 rho R; accP = c_xi + P_S u + P_SH xb; column sums of D_S u + D_SH xb.
// With `last`, dzsq gets ||rho R||^2.
template <int NT, int KS>
__device__ __forceinline__ void update_fwd_p1(const float* __restrict__ fac, int nc, int n,
                                              const float* __restrict__ part, int nwin, int S,
                                              const float* __restrict__ lam,
                                              float* __restrict__ lam_n,
                                              const float* __restrict__ xb,
                                              const float* __restrict__ cx, float rho, bool last,
                                              float& dzsq, float* __restrict__ csum,
                                              floatx4 (&accP)[tiles_per_wave(NT)], int wave,
                                              int lane) {
  constexpr int TPW = tiles_per_wave(NT);
  const int m = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    Tile t;
    if (!mode_tile_of(wave + q * (NT >> 6), n, nc, t)) continue;
    const int i = t.rt * 16 + m;
    const int ic = min(i, n - 1);
    const int cb = t.ct * 16 + m;
    // every read of the tile is issued before its arithmetic
    float bS[KS], dS[KS], bH[KS], dH[KS];
    mode_operands<KS>(fac, nc, 0, false, cb, bS, dS, lane);
    mode_operands<KS>(fac, nc, 2 * nc * nc, false, cb, bH, dH, lane);
    int sidx[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) sidx[s] = __umul24(t.ax * n + ic, nc) + min(4 * s + kq, nc - 1);
    float r[KS];
    window_sum<KS, KS == 4 ? 8 : 2>(part, nwin, S, sidx, r);
    float au[KS], axb[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const bool ok = i < n && 4 * s + kq < nc;
      const float lm = lam[sidx[s]];
      const float xv = xb[sidx[s]];
      au[s] = ok ? fmaf(-2.f * rho, r[s], lm) : 0.f;
      axb[s] = ok ? xv : 0.f;
      if (ok && t.ct == 0) {
        lam_n[sidx[s]] = fmaf(-rho, r[s], lm);
        if (last) dzsq = fmaf(rho * r[s], rho * r[s], dzsq);
      }
    }
    // rows past n and columns past nc of the tile are never stored: their
    // accumulators may start from any finite value
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int io = t.rt * 16 + 4 * kq + v;
      accP[q][v] = cx[__umul24(t.ax * n + min(io, n - 1), nc) + min(cb, nc - 1)];
    }
    floatx4 accD = {0.f, 0.f, 0.f, 0.f};
    mode_mfma<KS>(au, bS, dS, accP[q], accD);
    mode_mfma<KS>(axb, bH, dH, accP[q], accD);
    put_colsum(accD, csum, t, lane);
  }
}

// Forward update, phase 2: xn = accP + mean term.  With `last`, dzsq gets
// ||xn - xb||^2.
template <int NT>
__device__ __forceinline__ void update_fwd_p2(int nc, int n, const float* __restrict__ csum,
                                              const floatx4 (&accP)[tiles_per_wave(NT)],
                                              const float* __restrict__ xb,
                                              float* __restrict__ xn, bool last, float& dzsq,
                                              const float* __restrict__ refc,
                                              int* __restrict__ lslot, float skin, int wave,
                                              int lane) {
  constexpr int TPW = tiles_per_wave(NT);
  const int m = lane & 15, kq = lane >> 4;
  bool moved = false;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    Tile t;
    if (!mode_tile_of(wave + q * (NT >> 6), n, nc, t)) continue;
    const float mean = get_mean(csum, t, n, lane);
    const int cb = t.ct * 16 + m;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int io = t.rt * 16 + 4 * kq + v;
      if (io < n && cb < nc) {
        const int s = __umul24(t.ax * n + io, nc) + cb;
        const float val = accP[q][v] + mean;
        xn[s] = val;
        if (lslot) moved |= !(fabsf(val - refc[s]) <= skin);
        if (last) {
          const float d = val - xb[s];
          dzsq = fmaf(d, d, dzsq);
        }
      }
    }
  }
  if (lslot) note_moved(moved, lslot, wave, lane);
}

// Constant term c_xi = S xi + N b, mode form (first block of K^{-1} applied to
// the xi and b parts of eta), one entry.  tgt: target xi, xm/bm: robot means of
// xi ([2][nc]) and of b (bm[ax*2 + q]).
__device__ __forceinline__ float cxi_entry(const float* __restrict__ fac, int nc,
                                           const float* __restrict__ tgt,
                                           const float* __restrict__ xm,
                                           const float* __restrict__ bnd_i,
                                           const float* __restrict__ bm, int n, int ax, int i,
                                           int c) {
  const int nc2 = nc * nc;
  const float* Sp = fac + c * nc;
  const float* DS = fac + nc2 + c * nc;
  const float* Np = fac + 4 * nc2;
  const float* DN = Np + 2 * nc;
  const float* y = tgt + ax * n * nc + i * nc;
  const float* ym = xm + ax * nc;
  float out = 0.f;
  for (int q = 0; q < nc; ++q) out = fmaf(Sp[q], y[q], fmaf(DS[q], ym[q], out));
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

// Pair/obstacle/box residual sums with every pair visited (plain path; global
// memory, one thread per (robot, step)), in the culled stage's order.
__device__ __forceinline__ void constraints_full(
    const float2* __restrict__ X, float2* __restrict__ V, int n, int T,
    const float* __restrict__ obs, const float* __restrict__ ovel, int M, float a, float pmin0,
    float pmin1, float pmax0, float pmax1, bool accum, float& r1sq, float& r2sq, int tid,
    int nthr) {
  const float inv_Tm1 = 1.f / (float)(T - 1);
  const float a2 = a * a;
  for (int idx = tid; idx < n * T; idx += nthr) {
    const int i = idx / T;
    const int kk = idx - i * T;
    const float2 p = X[i * T + kk];
    float vx = 0.f, vy = 0.f, s1 = 0.f;
    for (int j = 0; j < n; ++j) {
      const float2 q = X[j * T + kk];
      const float dx = p.x - q.x;
      const float dy = p.y - q.y;
      const float d2 = fmaf(dy, dy, dx * dx);
      if (d2 < a2 && j != i) {
        float rx, ry;
        pair_residual(dx, dy, d2, a, i < j, rx, ry);
        vx += rx;
        vy += ry;
        if (j > i) s1 = fmaf(rx, rx, fmaf(ry, ry, s1));
      }
    }
    const float tau = (float)kk * inv_Tm1;
    for (int m = 0; m < M; ++m) {
      const float ao = obs[3 * m + 2];
      const float cx = ovel ? fmaf(ovel[2 * m], tau, obs[3 * m]) : obs[3 * m];
      const float cy = ovel ? fmaf(ovel[2 * m + 1], tau, obs[3 * m + 1]) : obs[3 * m + 1];
      const float dx = p.x - cx;
      const float dy = p.y - cy;
      const float d2 = fmaf(dy, dy, dx * dx);
      if (d2 < ao * ao) {
        float rx, ry;
        pair_residual(dx, dy, d2, ao, true, rx, ry);
        vx += rx;
        vy += ry;
        s1 = fmaf(rx, rx, fmaf(ry, ry, s1));
      }
    }
    const float hx = fmaxf(p.x - pmax0, 0.f), lx = fmaxf(pmin0 - p.x, 0.f);
    const float hy = fmaxf(p.y - pmax1, 0.f), ly = fmaxf(pmin1 - p.y, 0.f);
    vx = fmaf(1.f, hx - lx, 1.f * vx);
    vy = fmaf(1.f, hy - ly, 1.f * vy);
    if (accum) {
      r1sq += s1;
      r2sq += hx * hx + lx * lx + hy * hy + ly * ly;
    }
    V[i * T + kk] = make_float2(vx, vy);
  }
}

// ---------------------------------------------------------------------------
// Fused kernels: per-problem context and the block-level steps.
// ---------------------------------------------------------------------------

// Copy rows k0 .. k0+Tce-1 of W (global, [T][nc]) into the LDS table W.
__device__ __forceinline__ void load_wchunk(const float* __restrict__ Wg, float* __restrict__ W,
                                            int nc, int k0, int Tce, int tid, int nthr) {
  for (int t = tid; t < Tce * nc; t += nthr) W[t] = Wg[k0 * nc + t];
}

// Rows of the mask arrays (robots, padded so that a ballot's two robots and
// its 64-bit store stay inside) and 32-bit words per window.
__host__ __device__ inline int mask_rows(int n_max) { return (n_max + 7) & ~7; }
__host__ __device__ inline int mask_words(int n_max, int M_max) {
  return (((n_max + 31) >> 5) + ((M_max + 31) >> 5)) * mask_rows(n_max);
}

struct Ctx {
  int n, M, nc, T, Tc, S, tid;
  float rho, a, pmin0, pmin1, pmax0, pmax1;
  float* W;
  const float *fac, *Wg;
  const float4* obs;    // (cx, cy, a_o, a_o^2) at tau = 0
  float4* obox;         // obstacle window boxes [window][M_max], widened by their margin
  float* box3;          // window boxes [robot][window] (xmin, xmax, ymin, ymax)
  unsigned* masks;      // [window][word][row]
  float* refc;          // coefficients at the last list rebuild
  int* lslot;           // per-wave "moved" flags of the list check
  int mrow, mpw, mstride;
  float skin;
  bool chunked;  // T > Tc: the LDS W table holds one time chunk at a time
  const float2* ovel;   // obstacle displacement over the horizon (centre at tau: c + d tau)
  int ostride;          // M_max: window stride of obox
  float inv_Tm1;        // 1 / (T - 1): tau of global step k is k * inv_Tm1
  bool moving;          // some obstacle moves (displacements were set)
  unsigned* gmask;      // chunked: this problem's lists of every chunk (global memory)

  __device__ __forceinline__ int Ts() const { return tstride(Tc); }
  __device__ __forceinline__ int nws() const { return nwindows(Tc); }
  __device__ __forceinline__ unsigned* mwin(int w) const { return masks + w * mstride; }

  // After a rebuild of window 0's lists: this part's robots' coefficients
  // become the reference of the list check.
  __device__ __forceinline__ void set_reference(const float* __restrict__ xb, int h, int H,
                                                int lane) const {
    const int cnt = part_count(n, h, H), per = 2 * nc;
    for (int e = lane; e < cnt * per; e += 64) {
      const int t = e / per, r = e - t * per;
      const int ax = r >= nc, c = r - ax * nc;
      const int s = __umul24(ax * n + part_robot(t, h, H), nc) + c;
      refc[s] = xb[s];
    }
  }

  // Chunked horizons keep the lists of every chunk between passes in global
  // memory: after a rebuild the chunk's LDS window slots are stored (out),
  // otherwise they are loaded before the chunk's units use them.  Block-wide;
  // the caller orders it with barriers.
  template <int NT>
  __device__ __forceinline__ void chunk_lists(int chunk, bool out) const {
    const int words = nws() * mstride;
    unsigned* g = gmask + (size_t)chunk * words;
    for (int t = tid; t < words; t += NT) {
      if (out)
        g[t] = masks[t];
      else
        masks[t] = g[t];
    }
  }

  // Make the LDS W table hold rows k0 .. k0+Tce-1 (block-wide; no-op when
  // the whole horizon is resident).
  template <int NT>
  __device__ __forceinline__ void wchunk(int k0, int Tce) const {
    if (!chunked) return;
    __syncthreads();
    load_wchunk(Wg, W, nc, k0, Tce, tid, NT);
    __syncthreads();
  }
};

// Window boxes of the obstacles for the windows of the chunk that starts at
// global step kg (Tce steps): a centre moves linearly in tau (c + d tau), so
// its extent over a window is that of the window's first and last steps (the
// centres the walks form with the same rounded operations are monotone in
// the step); widened by the obstacle-side margin.  Static obstacles (d = 0)
// get the same box in every window.
__device__ __forceinline__ void obstacle_boxes(const Ctx& C, int kg, int Tce, int tid,
                                               int nthr) {
  const int nwin = nwindows(Tce);
  for (int e = tid; e < nwin * C.M; e += nthr) {
    const int w = e / C.M, m = e - w * C.M;
    const float4 o = C.obs[m];
    const float2 d = C.ovel[m];
    const float f = obs_margin(o.z);
    const float t0 = (float)(kg + w * 16) * C.inv_Tm1;
    const float t1 = (float)(kg + min(w * 16 + 15, Tce - 1)) * C.inv_Tm1;
    const float x0 = fmaf(d.x, t0, o.x), x1 = fmaf(d.x, t1, o.x);
    const float y0 = fmaf(d.y, t0, o.y), y1 = fmaf(d.y, t1, o.y);
    C.obox[w * C.ostride + m] = make_float4(fminf(x0, x1) - f, fmaxf(x0, x1) + f,
                                            fminf(y0, y1) - f, fmaxf(y0, y1) + f);
  }
}

// One chunk of window units: positions, masks and the constraint stage of
// every window (V = w_pair (pairs + obstacles) + w_box box), and with `part`
// the windows' shares of W^T V into part[w][S] (added when `accumulate`).
// Leaves the block synchronised.
template <int NT, int KS>
__device__ __forceinline__ void chunk_units(const Ctx& C, int chunk, int Tce, const float* xb,
                                            float2* X, float2* V, float* part, bool accumulate,
                                            bool accum, float& r1sq, float& r2sq, float w_pair,
                                            float w_box) {
  const int lane = lane_here(C.tid), wave = wave_id(C.tid), nwaves = NT >> 6;
  const bool rebuild = lists_moved(C.lslot, nwaves, lane);
  const int nwin = nwindows(Tce);
  const int H = parts_per_window(C.n, nwin, nwaves);
  const int Ts = C.Ts(), nws = C.nws();
  const int kg = chunk * C.Tc;   // global step of the chunk's first step
  if (rebuild) {
    obstacle_boxes(C, kg, Tce, C.tid, NT);
    map_chunk<NT, KS, true>(C.W, C.nc, xb, C.n, reinterpret_cast<float*>(X), Ts, Tce, C.box3,
                            nws, wave, lane);
  } else {
    map_chunk<NT, KS, false>(C.W, C.nc, xb, C.n, reinterpret_cast<float*>(X), Ts, Tce, nullptr,
                             nws, wave, lane);
    if (C.chunked) C.chunk_lists<NT>(chunk, false);
  }
  __syncthreads();
  for (int u = wave; u < nwin * H; u += nwaves) {
    const int w = u / H, h = u - w * H;
    if (rebuild) {
      masks_window(reinterpret_cast<const float4*>(C.box3), C.n, C.obox + w * C.ostride, C.M,
                   C.a, C.skin, C.mwin(w), C.mrow, C.mpw, nws, w, h, H, lane);
      if (w == 0 && chunk == 0) C.set_reference(xb, h, H, lane);
      wave_fence();
    }
#define SF_CONSTRAINTS(ACC, MOV)                                                               \
  constraints_window<ACC, MOV>(X, V, C.n, Ts, C.obs, C.ovel, kg, C.inv_Tm1, C.M,              \
                               C.mwin(w),                                                 \
                               C.mrow, C.mpw, C.a, C.pmin0, C.pmin1, C.pmax0, C.pmax1, w, Tce, \
                               h, H, r1sq, r2sq, w_pair, w_box, lane)
    if (C.moving) {
      if (accum) SF_CONSTRAINTS(true, true);
      else SF_CONSTRAINTS(false, true);
    } else {
      if (accum) SF_CONSTRAINTS(true, false);
      else SF_CONSTRAINTS(false, false);
    }
#undef SF_CONSTRAINTS
    if (part) {
      wave_fence();
      wtmap_window<KS>(C.W, C.nc, reinterpret_cast<const float*>(V), C.n, Ts, w, Tce, h, H,
                       part + w * C.S, accumulate, lane);
    }
  }
  __syncthreads();
  if (rebuild && C.chunked) C.chunk_lists<NT>(chunk, true);
}

// One application of T on the LDS state: (xb, lam) -> (xn, lam_n).  X, V,
// part and csum are scratch.  With want_dz, dzsq gets this thread's share of
// ||z' - z||^2.  With check, the residual of xb is formed on the way (wave
// sums through red) and the return value says whether it is <= tol; the
// update is completed either way.  Entered and left with the block
// synchronised.
template <int NT, int KS>
__device__ __forceinline__ bool sf_iteration(const Ctx& C, const float* xb, float* xn,
                                             const float* lam, float* lam_n, float* csum,
                                             float2* X, float2* V, float* part, const float* cx,
                                             bool want_dz, float& dzsq,
                                             bool check = false, float tol = 0.f,
                                             float* red = nullptr) {
  const int wave = wave_id(C.tid);
  float d1 = 0.f, d2 = 0.f;
  for (int k0 = 0, ch = 0; k0 < C.T; k0 += C.Tc, ++ch) {
    const int Tce = min(C.Tc, C.T - k0);
    C.wchunk<NT>(k0, Tce);
    chunk_units<NT, KS>(C, ch, Tce, xb, X, V, part, k0 > 0, check, d1, d2, 1.f, 1.f);
  }
  if (check) {
    d1 = wave_sum_dpp(d1);
    d2 = wave_sum_dpp(d2);
    if ((C.tid & 63) == 0) {
      red[2 * wave] = d1;
      red[2 * wave + 1] = d2;
    }
  }
  floatx4 accP[tiles_per_wave(NT)];
  int lane = lane_here(C.tid);
  update_fwd_p1<NT, KS>(C.fac, C.nc, C.n, part, nwindows(min(C.Tc, C.T)), C.S, lam, lam_n, xb,
                        cx, C.rho, want_dz, dzsq, csum, accP, wave, lane);
  __syncthreads();
  bool stop = false;
  if (check) {
    float r1 = 0.f, r2 = 0.f;
    for (int q = 0; q < (NT >> 6); ++q) {
      r1 += red[2 * q];
      r2 += red[2 * q + 1];
    }
    stop = sqrtf(r1 + r2) <= tol;
  }
  lane = lane_here(C.tid);
  update_fwd_p2<NT>(C.nc, C.n, csum, accP, xb, xn, want_dz, dzsq, C.refc,
                    C.lslot, C.skin, wave, lane);
  __syncthreads();
  return stop;
}

// ||r_1||^2 and ||r_2||^2 partials of the iterate xb (block-synchronised on
// return); V is scratch.
template <int NT, int KS>
__device__ __forceinline__ void residual_norms(const Ctx& C, const float* xb, float2* X,
                                               float2* V, float& r1sq, float& r2sq) {
  for (int k0 = 0, ch = 0; k0 < C.T; k0 += C.Tc, ++ch) {
    const int Tce = min(C.Tc, C.T - k0);
    C.wchunk<NT>(k0, Tce);
    chunk_units<NT, KS>(C, ch, Tce, xb, X, V, nullptr, false, true, r1sq, r2sq, 1.f, 1.f);
  }
}

// LDS floats of the obstacle data: centres and sizes, window boxes of a
// chunk, displacements.
__host__ __device__ inline size_t obstacle_floats(int Tc, int M_max) {
  return 4 * (size_t)M_max * (1 + nwindows(Tc)) + (size_t)((2 * M_max + 3) & ~3);
}

// LDS floats of the box and mask regions.
__host__ __device__ inline int box_floats(int Tc, int n_max) {
  return 4 * n_max * nwindows(Tc);
}
// Windows whose candidate lists are held in LDS: all windows of the horizon
// when it is LDS-resident, else those of one time chunk (the lists of every
// chunk then live in global memory between passes, see chunk_lists).
__host__ __device__ inline int horizon_windows(int T, int Tc) {
  return nwindows(min(T, Tc));
}
__host__ __device__ inline int mask_floats(int T, int Tc, int n_max, int M_max) {
  return horizon_windows(T, Tc) * mask_words(n_max, M_max);
}
// 32-bit words of one problem's global copy of the lists of every chunk (0
// when the horizon is LDS-resident).
__host__ __device__ inline size_t list_words(int T, int Tc, int n_max, int M_max) {
  if (Tc >= T) return 0;
  return (size_t)((T + Tc - 1) / Tc) * nwindows(Tc) * mask_words(n_max, M_max);
}
// Reference coefficients of the list check and the per-wave flags.
__host__ __device__ inline int list_floats(int S_max) { return ((S_max + 3) & ~3) + kMaxWaves; }

// Skin of the candidate lists: a quarter of the robot size.
__device__ __forceinline__ float list_skin(float a) { return 0.25f * a; }

// Every wave flags "moved": the first pass builds all lists.
__device__ __forceinline__ void force_rebuild(int* __restrict__ lslot, int tid) {
  if (tid < kMaxWaves) lslot[tid] = 1;
}

struct FwdLds {
  float *W, *fac, *xbA, *xbB, *lamA, *lamB, *cx, *part, *means, *red, *csum, *box3;
  float4 *obs, *obox;
  float* refc;
  int* lslot;
  unsigned* masks;
  float2* ovel;
  float2 *X, *V;
};

__device__ __forceinline__ FwdLds carve_fwd(float* sm, int nc, int T, int Tc, int n_max,
                                            int M_max, int S_max) {
  FwdLds L;
  float* p = sm;
  L.W = p; p += round4(nc * Tc);
  L.fac = p; p += round4(fac_stride(nc));
  L.xbA = p; p += round4(S_max);
  L.xbB = p; p += round4(S_max);
  L.lamA = p; p += round4(S_max);
  L.lamB = p; p += round4(S_max);
  L.cx = p; p += round4(S_max);
  L.part = p; p += nwindows(Tc) * round4(S_max);
  L.means = p; p += kMeans;
  L.red = p; p += kRed;
  L.csum = p; p += kColSums;
  L.obs = reinterpret_cast<float4*>(p); p += 4 * M_max;
  L.obox = reinterpret_cast<float4*>(p); p += 4 * M_max * nwindows(Tc);
  L.ovel = reinterpret_cast<float2*>(p); p += round4(2 * M_max);
  L.box3 = p; p += box_floats(Tc, n_max);
  L.masks = reinterpret_cast<unsigned*>(p); p += mask_floats(T, Tc, n_max, M_max);
  L.refc = p;
  L.lslot = reinterpret_cast<int*>(p + ((S_max + 3) & ~3));
  p += list_floats(S_max);
  L.X = reinterpret_cast<float2*>(p); p += 2 * n_max * tstride(Tc);
  L.V = reinterpret_cast<float2*>(p);
  return L;
}

}  // namespace

size_t chunk_list_bytes(int T, int Tc, int n_max, int M_max) {
  return sizeof(unsigned) * list_words(T, Tc, n_max, M_max);
}

size_t fwd_lds_bytes(int nc, int T, int Tc, int n_max, int M_max, int S_max, int) {
  auto r4 = [](int x) { return (size_t)((x + 3) & ~3); };
  size_t f = r4(nc * Tc) + r4(fac_stride(nc)) + (5 + nwindows(Tc)) * r4(S_max) + kMeans + kRed +
             kColSums + obstacle_floats(Tc, M_max) + box_floats(Tc, n_max) + mask_floats(T, Tc, n_max, M_max) + list_floats(S_max) +
             4 * (size_t)n_max * tstride(Tc);
  return f * sizeof(float);
}

// ---------------------------------------------------------------------------
// Fused forward: one workgroup runs all L iterations of one problem with the
// whole state in LDS.  Launch slot -> problem through `order` (longest first).
// ---------------------------------------------------------------------------
template <int NT, int KS>
__global__ __launch_bounds__(NT) void fwd_fused_kernel(FwdArgs A) {
  extern __shared__ float4 sm4[];
  float* sm = reinterpret_cast<float*>(sm4);
  const int tid = threadIdx.x;
  const int b = A.order[blockIdx.x];
  const ProbDesc P = A.probs[b];
  const int n = P.n, M = P.M, nc = A.nc, T = A.T;
  const int S = 2 * n * nc;
  const int fs = fac_stride(nc);
  FwdLds L = carve_fwd(sm, nc, T, A.Tc, A.n_max, A.M_max, A.S_max);
  Ctx C{n,      M,         nc,        T,         A.Tc,      S,
        tid,    A.rho,     P.a,       P.pmin[0], P.pmin[1], P.pmax[0],
        P.pmax[1], L.W,    L.fac,     A.W,       L.obs,     L.obox,
        L.box3, L.masks,   L.refc,    L.lslot,   mask_rows(A.n_max), (A.n_max + 31) >> 5,
        mask_words(A.n_max, A.M_max), list_skin(P.a), A.Tc < T,
        L.ovel, A.M_max, 1.f / (float)(T - 1), A.ovel != nullptr,
        A.gmask + (size_t)b * list_words(T, A.Tc, A.n_max, A.M_max)};
  force_rebuild(L.lslot, tid);
  if (!C.chunked) load_wchunk(A.W, L.W, nc, 0, T, tid, NT);
  for (int t = tid; t < fs; t += NT) L.fac[t] = A.fac[(size_t)P.fac * fs + t];
  for (int m = tid; m < M; m += NT) {
    const float* o = A.obstacles + ((size_t)P.obs_off + m) * 3;
    L.obs[m] = make_float4(o[0], o[1], o[2], o[2] * o[2]);
    L.ovel[m] = A.ovel ? make_float2(A.ovel[((size_t)P.obs_off + m) * 2],
                                     A.ovel[((size_t)P.obs_off + m) * 2 + 1])
                       : make_float2(0.f, 0.f);
    if (A.save) {
      float* d = A.ws_obs + ((size_t)P.obs_off + m) * 3;
      d[0] = o[0];
      d[1] = o[1];
      d[2] = o[2];
    }
  }
  for (int s = tid; s < S; s += NT) {
    L.xbA[s] = A.xi0[P.coef_off + s];
    L.lamA[s] = A.lam0[P.coef_off + s];
    L.lamB[s] = A.xi[P.coef_off + s];   // target xi, staged for c_xi
  }
  __syncthreads();
  const float* bnd = A.boundary + (size_t)P.rob_off * 4;
  robot_means(L.lamB, n, nc, L.means, wave_id(tid), NT >> 6, tid & 63);
  boundary_means(bnd, n, L.means + 2 * nc, tid, NT);
  __syncthreads();
  for (int s = tid; s < S; s += NT) {
    const int ax = s / (n * nc), rem = s - ax * n * nc, i = rem / nc, c = rem - i * nc;
    const float v = cxi_entry(L.fac, nc, L.lamB, L.means, bnd + i * 4, L.means + 2 * nc, n,
                              ax, i, c);
    L.cx[s] = v;
    if (A.save) A.ws_cxi[P.coef_off + s] = v;
  }
  __syncthreads();

  float* xb = L.xbA;
  float* xn = L.xbB;
  float* lam = L.lamA;
  float* lamn = L.lamB;
  float dzsq = 0.f;
  int ran = A.L;
  for (int l = 0; l < A.L; ++l) {
    if (A.save && (l % A.ckpt_every) == 0) {
      float* ck = A.ws_ckpt + (size_t)(l / A.ckpt_every) * 2 * A.S_total + P.coef_off;
      for (int s = tid; s < S; s += NT) {
        ck[s] = xb[s];
        ck[A.S_total + s] = lam[s];
      }
    }
    const bool check = A.check_every > 0 && (l % A.check_every) == 0;
    const bool want_dz = check || l == A.L - 1;
    if (want_dz) dzsq = 0.f;   // the reported ||dz|| is that of the last update
    const bool stop = sf_iteration<NT, KS>(C, xb, xn, lam, lamn, L.csum, L.X, L.V, L.part, L.cx,
                                           want_dz, dzsq, check, A.tol, L.red);
    float* t = xb;
    xb = xn;
    xn = t;
    t = lam;
    lam = lamn;
    lamn = t;
    if (stop) {
      ran = l + 1;
      break;
    }
  }
  if (tid == 0) A.ws_iters[b] = ran;

  float bad = 0.f;
  for (int s = tid; s < S; s += NT) {
    const float x = xb[s], lm = lam[s];
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
  residual_norms<NT, KS>(C, xb, L.X, L.V, r1sq, r2sq);
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

// MFMA K steps of 4 coefficients: 4 covers n_coef <= 16, 8 covers <= 32.
__host__ __device__ inline int ks_class(int nc) { return nc <= 16 ? 4 : 8; }

template <int KS>
hipError_t launch_fwd_ks(const FwdArgs& a, int threads, size_t lds, hipStream_t s) {
  dim3 grid(a.B);
  switch (threads) {
    case 256:
      hipLaunchKernelGGL((fwd_fused_kernel<256, KS>), grid, dim3(256), lds, s, a);
      break;
    case 512:
      hipLaunchKernelGGL((fwd_fused_kernel<512, KS>), grid, dim3(512), lds, s, a);
      break;
    case 1024:
      hipLaunchKernelGGL((fwd_fused_kernel<1024, KS>), grid, dim3(1024), lds, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fwd_fused(const FwdArgs& a, int threads, size_t lds, hipStream_t s) {
  return ks_class(a.nc) == 4 ? launch_fwd_ks<4>(a, threads, lds, s)
                             : launch_fwd_ks<8>(a, threads, lds, s);
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
  float *W, *fac, *red, *csum, *gA, *gB, *glam, *gxi, *cx, *b0, *b1, *b2, *b3, *part, *box3;
  float4 *obs, *obox;
  float* refc;
  int* lslot;
  unsigned* masks;
  float2* ovel;
  float2 *X, *G, *H;
};

__device__ __forceinline__ BwdLds carve_bwd(float* sm, int nc, int T, int Tc, int n_max,
                                            int M_max, int S_max) {
  BwdLds L;
  float* p = sm;
  L.W = p; p += round4(nc * Tc);
  L.fac = p; p += round4(fac_stride(nc));
  L.red = p; p += kRed;
  L.csum = p; p += 2 * kColSums;
  float** bufs[9] = {&L.gA, &L.gB, &L.glam, &L.gxi, &L.cx, &L.b0, &L.b1, &L.b2, &L.b3};
  for (int q = 0; q < 9; ++q) {
    *bufs[q] = p;
    p += round4(S_max);
  }
  L.part = p; p += nwindows(Tc) * round4(S_max);
  L.obs = reinterpret_cast<float4*>(p); p += 4 * M_max;
  L.obox = reinterpret_cast<float4*>(p); p += 4 * M_max * nwindows(Tc);
  L.ovel = reinterpret_cast<float2*>(p); p += round4(2 * M_max);
  L.box3 = p; p += box_floats(Tc, n_max);
  L.masks = reinterpret_cast<unsigned*>(p); p += mask_floats(T, Tc, n_max, M_max);
  L.refc = p;
  L.lslot = reinterpret_cast<int*>(p + ((S_max + 3) & ~3));
  p += list_floats(S_max);
  L.X = reinterpret_cast<float2*>(p); p += 2 * n_max * tstride(Tc);
  L.G = reinterpret_cast<float2*>(p); p += 2 * n_max * tstride(Tc);
  L.H = reinterpret_cast<float2*>(p);
  return L;
}

// g[s] += sum of the per-window partials part[w][s] (w < nwin, window order).
__device__ __forceinline__ void add_partials(float* __restrict__ g, const float* __restrict__ part,
                                             int nwin, int S, int tid, int nthr) {
  for (int s = tid; s < S; s += nthr) {
    float r = part[s];
    for (int w = 1; w < nwin; ++w) r += part[w * S + s];
    g[s] += r;
  }
}

// Adjoint update, phase 1 (tiles of this wave): the A operand is the
// cotangent g of xi_bar^{l+1}, plus the pending W^T VJP partials (part, when
// not null) and, with a fixed-point weight fw, 2 fw (xi_bar^{l+1} - xi_bar^l);
// accU = S^T g, accN = SH^T g - 2 fw (xi_bar^{l+1} - xi_bar^l); column sums of
// the D^T blocks into csU / csN.  cur and nxt are the iterates l and l+1
// ([2][S_total] slices: xi_bar, then lambda at +St).
template <int NT, int KS>
__device__ __forceinline__ void update_bwd_p1(const float* __restrict__ fac, int nc, int n,
                                              const float* __restrict__ gx,
                                              const float* __restrict__ part, int nwin, int S,
                                              const float* __restrict__ cur,
                                              const float* __restrict__ nxt, float fw,
                                              float* __restrict__ csU, float* __restrict__ csN,
                                              floatx4 (&accU)[tiles_per_wave(NT)],
                                              floatx4 (&accN)[tiles_per_wave(NT)], int wave,
                                              int lane) {
  constexpr int TPW = tiles_per_wave(NT);
  const int m = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    Tile t;
    if (!mode_tile_of(wave + q * (NT >> 6), n, nc, t)) continue;
    const int i = t.rt * 16 + m;
    const int ic = min(i, n - 1);
    const int cb = t.ct * 16 + m;
    // every read of the tile is issued before its arithmetic
    float bU[KS], dU_[KS], bN[KS], dN_[KS];
    mode_operands<KS>(fac, nc, 0, true, cb, bU, dU_, lane);
    mode_operands<KS>(fac, nc, 2 * nc * nc, true, cb, bN, dN_, lane);
    int sidx[KS];
    float g[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      sidx[s] = __umul24(t.ax * n + ic, nc) + min(4 * s + kq, nc - 1);
      g[s] = gx[sidx[s]];
    }
    if (part) {
      float r[KS];
      window_sum<KS, KS == 4 ? 4 : 2>(part, nwin, S, sidx, r);
#pragma unroll
      for (int s = 0; s < KS; ++s) g[s] += r[s];
    }
    if (fw != 0.f) {
#pragma unroll
      for (int s = 0; s < KS; ++s) g[s] = fmaf(2.f * fw, nxt[sidx[s]] - cur[sidx[s]], g[s]);
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const bool ok = i < n && 4 * s + kq < nc;
      g[s] = ok ? g[s] : 0.f;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int io = t.rt * 16 + 4 * kq + v;
      float f0 = 0.f;
      if (fw != 0.f && io < n && cb < nc) {
        const int s = __umul24(t.ax * n + io, nc) + cb;
        f0 = -2.f * fw * (nxt[s] - cur[s]);
      }
      accU[q][v] = 0.f;
      accN[q][v] = f0;
    }
    floatx4 dU = {0.f, 0.f, 0.f, 0.f}, dN = {0.f, 0.f, 0.f, 0.f};
    mode_mfma<KS>(g, bU, dU_, accU[q], dU);
    mode_mfma<KS>(g, bN, dN_, accN[q], dN);
    put_colsum(dU, csU, t, lane);
    put_colsum(dN, csN, t, lane);
  }
}

// Adjoint update, phase 2: g_u = accU + mean term (the cotangent reaching u =
// lambda - 2 rho R, hence also the target xi and lambda); g_R = -2 rho g_u -
// rho g_lambda' (- 2 rho fw (lambda^{l+1} - lambda^l)); g_lambda += g_u;
// g_xi += g_u; the new g_xi_bar (before its W^T VJP part) = accN + mean term.
template <int NT>
__device__ __forceinline__ void update_bwd_p2(int nc, int n, const float* __restrict__ csU,
                                              const float* __restrict__ csN,
                                              const floatx4 (&accU)[tiles_per_wave(NT)],
                                              const floatx4 (&accN)[tiles_per_wave(NT)],
                                              float rho, float fw, const float* __restrict__ cur,
                                              const float* __restrict__ nxt, size_t St,
                                              float* __restrict__ glam, float* __restrict__ gxi,
                                              float* __restrict__ gR, float* __restrict__ gn,
                                              int wave, int lane) {
  constexpr int TPW = tiles_per_wave(NT);
  const int m = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    Tile t;
    if (!mode_tile_of(wave + q * (NT >> 6), n, nc, t)) continue;
    const float mu = get_mean(csU, t, n, lane);
    const float mn = get_mean(csN, t, n, lane);
    const int cb = t.ct * 16 + m;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int io = t.rt * 16 + 4 * kq + v;
      if (io < n && cb < nc) {
        const int s = __umul24(t.ax * n + io, nc) + cb;
        const float gu = accU[q][v] + mu;
        const float gfp = fw != 0.f ? -2.f * rho * fw * (nxt[St + s] - cur[St + s]) : 0.f;
        const float gl = glam[s];
        gR[s] = fmaf(-2.f * rho, gu, fmaf(-rho, gl, gfp));
        glam[s] = gl + gu;
        gxi[s] += gu;
        gn[s] = accN[q][v] + mn;
      }
    }
  }
}

// Window units of one reverse iteration: positions X = W xb (with boxes) and
// G = W g_R, masks, the VJP H and its W^T share into part.
template <int NT, int KS>
__device__ __forceinline__ void adjoint_units(const Ctx& C, int chunk, int Tce, const float* xb,
                                              const float* gR, float2* X, float2* G, float2* Hb,
                                              float* part, bool accumulate) {
  const int lane = lane_here(C.tid), wave = wave_id(C.tid), nwaves = NT >> 6;
  const bool rebuild = lists_moved(C.lslot, nwaves, lane);
  const int nwin = nwindows(Tce);
  const int H = parts_per_window(C.n, nwin, nwaves);
  const int Ts = C.Ts(), nws = C.nws();
  const int kg = chunk * C.Tc;
  if (rebuild) {
    obstacle_boxes(C, kg, Tce, C.tid, NT);
    map_chunk<NT, KS, true>(C.W, C.nc, xb, C.n, reinterpret_cast<float*>(X), Ts, Tce, C.box3,
                            nws, wave, lane);
  } else {
    map_chunk<NT, KS, false>(C.W, C.nc, xb, C.n, reinterpret_cast<float*>(X), Ts, Tce, nullptr,
                             nws, wave, lane);
    if (C.chunked) C.chunk_lists<NT>(chunk, false);
  }
  map_chunk<NT, KS, false>(C.W, C.nc, gR, C.n, reinterpret_cast<float*>(G), Ts, Tce, nullptr,
                           nws, wave, lane);
  __syncthreads();
  for (int u = wave; u < nwin * H; u += nwaves) {
    const int w = u / H, h = u - w * H;
    if (rebuild) {
      masks_window(reinterpret_cast<const float4*>(C.box3), C.n, C.obox + w * C.ostride, C.M,
                   C.a, C.skin, C.mwin(w), C.mrow, C.mpw, nws, w, h, H, lane);
      if (w == 0 && chunk == 0) C.set_reference(xb, h, H, lane);
      wave_fence();
    }
    if (C.moving)
      vjp_window<true>(X, G, Hb, C.n, Ts, C.obs, C.ovel, kg, C.inv_Tm1, C.M, C.mwin(w),
                       C.mrow,
                       C.mpw, C.a, C.pmin0, C.pmin1, C.pmax0, C.pmax1, w, Tce, h, H, lane);
    else
      vjp_window<false>(X, G, Hb, C.n, Ts, C.obs, C.ovel, kg, C.inv_Tm1, C.M, C.mwin(w),
                        C.mrow,
                        C.mpw, C.a, C.pmin0, C.pmin1, C.pmax0, C.pmax1, w, Tce, h, H, lane);
    wave_fence();
    wtmap_window<KS>(C.W, C.nc, reinterpret_cast<const float*>(Hb), C.n, Ts, w, Tce, h, H,
                     part + w * C.S, accumulate, lane);
  }
  __syncthreads();
  if (rebuild && C.chunked) C.chunk_lists<NT>(chunk, true);
}

template <int NT, int KS>
__global__ __launch_bounds__(NT) void bwd_fused_kernel(BwdArgs A) {
  extern __shared__ float4 sm4[];
  float* sm = reinterpret_cast<float*>(sm4);
  const int tid = threadIdx.x;
  const int wave = wave_id(tid);
  const int b = A.order[blockIdx.x];
  const ProbDesc P = A.probs[b];
  const int n = P.n, M = P.M, nc = A.nc, T = A.T, Tc = A.Tc;
  const int S = 2 * n * nc;
  const int fs = fac_stride(nc);
  const float rho = A.rho, fw = A.fp_weight;
  const size_t St = (size_t)A.S_total;
  BwdLds L = carve_bwd(sm, nc, T, Tc, A.n_max, A.M_max, A.S_max);
  Ctx C{n,      M,         nc,        T,         Tc,        S,
        tid,    rho,       P.a,       P.pmin[0], P.pmin[1], P.pmax[0],
        P.pmax[1], L.W,    L.fac,     A.W,       L.obs,     L.obox,
        L.box3, L.masks,   L.refc,    L.lslot,   mask_rows(A.n_max), (A.n_max + 31) >> 5,
        mask_words(A.n_max, A.M_max), list_skin(P.a), Tc < T,
        L.ovel, A.M_max, 1.f / (float)(T - 1), A.ovel != nullptr,
        A.gmask + (size_t)b * list_words(T, Tc, A.n_max, A.M_max)};
  force_rebuild(L.lslot, tid);
  const int nwin0 = nwindows(min(Tc, T));
  if (!C.chunked) load_wchunk(A.W, L.W, nc, 0, T, tid, NT);
  for (int t = tid; t < fs; t += NT) L.fac[t] = A.fac[(size_t)P.fac * fs + t];
  for (int m = tid; m < M; m += NT) {
    const float* o = A.obs + ((size_t)P.obs_off + m) * 3;
    L.obs[m] = make_float4(o[0], o[1], o[2], o[2] * o[2]);
    L.ovel[m] = A.ovel ? make_float2(A.ovel[((size_t)P.obs_off + m) * 2],
                                     A.ovel[((size_t)P.obs_off + m) * 2 + 1])
                       : make_float2(0.f, 0.f);
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
    residual_norms<NT, KS>(C, L.b0, L.X, L.G, r1sq, r2sq);
    float v[2] = {r1sq, r2sq};
    block_sum(v, L.red);
    const float c1 = v[0] > 0.f ? gr1 / sqrtf(v[0]) : 0.f;
    const float c2 = v[1] > 0.f ? gr2 / sqrtf(v[1]) : 0.f;
    float d1 = 0.f, d2 = 0.f;
    for (int k0 = 0, ch = 0; k0 < T; k0 += Tc, ++ch) {
      const int Tce = min(Tc, T - k0);
      C.wchunk<NT>(k0, Tce);
      chunk_units<NT, KS>(C, ch, Tce, L.b0, L.X, L.H, L.part, k0 > 0, false, d1, d2, c1, c2);
    }
    add_partials(gx, L.part, nwin0, S, tid, NT);
    __syncthreads();
  }

  const int L_ = A.iters ? min(A.L, A.iters[b]) : A.L, k = A.ckpt_every;
  const int nseg = (L_ + k - 1) / k;
  float dz = 0.f;
  bool pending = false;   // L.part holds W^T VJP partials not yet added to gx
  // positions of the current reverse step (xbl) and a staging buffer (xalt)
  // for the next one, read ahead from global memory while this step's update
  // runs whenever that iterate needs no recompute
  float* xbl = L.b0;
  float* xalt = L.b1;
  bool staged = false;
  floatx4 accU[tiles_per_wave(NT)], accN[tiles_per_wave(NT)];
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int l0 = seg * k;
    const int l1 = min(L_, l0 + k);
    // the segment's first iterate is its checkpoint; recompute iterates
    // l0+1 .. l1-1 into the segment scratch (slot l - l0)
    const float* ck = A.ckpt + (size_t)seg * 2 * St + P.coef_off;
    if (l1 - 1 > l0) {
      float* xr = L.b0;
      float* xq = L.b1;
      float* lr = L.b2;
      float* lq = L.b3;
      staged = false;
      for (int s = tid; s < S; s += NT) {
        xr[s] = ck[s];
        lr[s] = ck[St + s];
      }
      check_lists<NT>(xr, L.refc, S, C.skin, L.lslot, tid);
      if (pending) {
        // the recompute reuses the partial buffer: fold it into gx first
        add_partials(gx, L.part, nwin0, S, tid, NT);
        pending = false;
      }
      __syncthreads();
      for (int l = l0; l < l1 - 1; ++l) {
        sf_iteration<NT, KS>(C, xr, xq, lr, lq, L.csum, L.X, L.G, L.part, L.cx, false, dz);
        float* t = xr;
        xr = xq;
        xq = t;
        t = lr;
        lr = lq;
        lq = t;
        float* dst = A.seg + (size_t)(l + 1 - l0) * 2 * St + P.coef_off;
        for (int s = tid; s < S; s += NT) {
          dst[s] = xr[s];
          dst[St + s] = lr[s];
        }
      }
      __syncthreads();
    }
    for (int l = l1 - 1; l >= l0; --l) {
      const float* cur = l == l0 ? ck : A.seg + (size_t)(l - l0) * 2 * St + P.coef_off;
      const float* nxt = (l + 1 < l1) ? A.seg + (size_t)(l + 1 - l0) * 2 * St + P.coef_off
                         : (l1 == L_) ? A.fin + P.coef_off
                                      : A.ckpt + (size_t)(seg + 1) * 2 * St + P.coef_off;
      float* gR = L.b2;
      if (!staged)
        for (int s = tid; s < S; s += NT) xbl[s] = cur[s];
      staged = false;
      check_lists<NT>(xbl, L.refc, S, C.skin, L.lslot, tid);
      const float* ahead = l > l0                ? (l - 1 == l0 ? ck : cur - 2 * St)
                           : (k == 1 && seg > 0) ? ck - 2 * St
                                                 : nullptr;
      const bool read_ahead = ahead != nullptr && S <= 2 * NT;
      float pv0 = 0.f, pv1 = 0.f;
      if (read_ahead) {
        if (tid < S) pv0 = ahead[tid];
        if (tid + NT < S) pv1 = ahead[tid + NT];
      }
      int lane = lane_here(tid);
      update_bwd_p1<NT, KS>(L.fac, nc, n, gx, pending ? L.part : nullptr, nwin0, S, cur, nxt, fw,
                            L.csum, L.csum + kColSums, accU, accN, wave, lane);
      pending = false;
      __syncthreads();
      lane = lane_here(tid);
      update_bwd_p2<NT>(nc, n, L.csum, L.csum + kColSums, accU, accN, rho, fw, cur, nxt, St,
                        L.glam, L.gxi, gR, gn, wave, lane);
      __syncthreads();
      if (read_ahead) {
        if (tid < S) xalt[tid] = pv0;
        if (tid + NT < S) xalt[tid + NT] = pv1;
      }
      for (int k0 = 0, ch = 0; k0 < T; k0 += Tc, ++ch) {
        const int Tce = min(Tc, T - k0);
        C.wchunk<NT>(k0, Tce);
        adjoint_units<NT, KS>(C, ch, Tce, xbl, gR, L.X, L.G, L.H, L.part, k0 > 0);
      }
      if (read_ahead) {
        float* t = xbl;
        xbl = xalt;
        xalt = t;
        staged = true;
      }
      pending = true;
      float* t = gx;
      gx = gn;
      gn = t;
    }
  }
  if (pending) {
    add_partials(gx, L.part, nwin0, S, tid, NT);
    __syncthreads();
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
  size_t f = r4(nc * Tc) + r4(fac_stride(nc)) + kRed + 2 * kColSums + (9 + nwindows(Tc)) * r4(S_max) +
             obstacle_floats(Tc, M_max) + box_floats(Tc, n_max) + mask_floats(T, Tc, n_max, M_max) + list_floats(S_max) +
             6 * (size_t)n_max * tstride(Tc);
  return f * sizeof(float);
}

template <int KS>
hipError_t launch_bwd_ks(const BwdArgs& a, int threads, size_t lds, hipStream_t s) {
  dim3 grid(a.B);
  switch (threads) {
    case 256:
      hipLaunchKernelGGL((bwd_fused_kernel<256, KS>), grid, dim3(256), lds, s, a);
      break;
    case 512:
      hipLaunchKernelGGL((bwd_fused_kernel<512, KS>), grid, dim3(512), lds, s, a);
      break;
    case 1024:
      hipLaunchKernelGGL((bwd_fused_kernel<1024, KS>), grid, dim3(1024), lds, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bwd_fused(const BwdArgs& a, int threads, size_t lds, hipStream_t s) {
  return ks_class(a.nc) == 4 ? launch_bwd_ks<4>(a, threads, lds, s)
                             : launch_bwd_ks<8>(a, threads, lds, s);
}

// Recompute area of the adjoint for callers that cannot allocate device
// memory (sf_project_backward_static): a file-scope device array, one copy per
// GPU, that lives until the process ends.  In host code `scratch` names a
// host-side stand-in, so host code only ever uses the device address that
// hipGetSymbolAddress returns for the current device.  The reverse sweep
// writes every slot before it reads it, so nothing has to be cleared between
// calls; calls that overlap on one GPU share the array and race.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t prepare_kernels(size_t lds) {
  const void* fns[] = {
      reinterpret_cast<const void*>(&fwd_fused_kernel<256, 4>),
      reinterpret_cast<const void*>(&fwd_fused_kernel<512, 4>),
      reinterpret_cast<const void*>(&fwd_fused_kernel<1024, 4>),
      reinterpret_cast<const void*>(&fwd_fused_kernel<256, 8>),
      reinterpret_cast<const void*>(&fwd_fused_kernel<512, 8>),
      reinterpret_cast<const void*>(&fwd_fused_kernel<1024, 8>),
      reinterpret_cast<const void*>(&bwd_fused_kernel<256, 4>),
      reinterpret_cast<const void*>(&bwd_fused_kernel<512, 4>),
      reinterpret_cast<const void*>(&bwd_fused_kernel<1024, 4>),
      reinterpret_cast<const void*>(&bwd_fused_kernel<256, 8>),
      reinterpret_cast<const void*>(&bwd_fused_kernel<512, 8>),
      reinterpret_cast<const void*>(&bwd_fused_kernel<1024, 8>)};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Plain path: the same steps as separate kernels over global memory, one
// problem per launch and every pair visited (the per-problem baseline the
// fused launch is compared with).  Blocks of 256 threads; map kernels give one
// window per wave.
// ---------------------------------------------------------------------------
namespace {

// Problem of a plain-path block: b itself, or with b < 0 (a launch over the
// whole batch) the problem of grid row blockIdx.y.
__device__ __forceinline__ int plain_problem(const FwdArgs& A, int b) {
  return b >= 0 ? b : A.order[blockIdx.y];
}

__global__ __launch_bounds__(256) void plain_prep_kernel(FwdArgs A, PlainBufs Bf, int b) {
  __shared__ float means[kMeans];
  b = plain_problem(A, b);
  const ProbDesc P = A.probs[b];
  const int n = P.n, nc = A.nc, S = 2 * n * nc, tid = threadIdx.x;
  const float* fac = A.fac + (size_t)P.fac * fac_stride(nc);
  const float* tgt = A.xi + P.coef_off;
  const float* bnd = A.boundary + (size_t)P.rob_off * 4;
  robot_means(tgt, n, nc, means, wave_id(tid), 4, tid & 63);
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

// Positions of every window (one window per wave).
template <int KS>
__global__ __launch_bounds__(256) void plain_xmap_kernel(FwdArgs A, PlainBufs Bf, int b,
                                                         int pp) {
  b = plain_problem(A, b);
  const ProbDesc P = A.probs[b];
  const int w = blockIdx.x * 4 + wave_id(threadIdx.x);
  if (w >= nwindows(A.T)) return;
  xmap_window<KS, false, false>(A.W, A.nc, Bf.xb[pp] + P.coef_off, P.n,
                                Bf.X + (size_t)P.pos_off * 2, A.T, w, A.T, nullptr, 0,
                                threadIdx.x & 63);
}

__global__ __launch_bounds__(256) void plain_constraint_kernel(FwdArgs A, PlainBufs Bf,
                                                               int b) {
  b = plain_problem(A, b);
  const ProbDesc P = A.probs[b];
  const int tid = blockIdx.x * 256 + threadIdx.x;
  float d1 = 0.f, d2 = 0.f;
  constraints_full(reinterpret_cast<const float2*>(Bf.X) + P.pos_off,
                   reinterpret_cast<float2*>(Bf.V) + P.pos_off, P.n, A.T,
                   A.obstacles + (size_t)P.obs_off * 3,
                   A.ovel ? A.ovel + (size_t)P.obs_off * 2 : nullptr, P.M, P.a, P.pmin[0],
                   P.pmin[1], P.pmax[0], P.pmax[1], false, d1, d2, tid, gridDim.x * 256);
}

// Per-window partials of W^T V (one window per wave, all column tiles), with
// the fused kernels' window boundaries: 16-step windows local to each time
// chunk of Tc steps, chunk contributions added in chunk order.
template <int KS>
__global__ __launch_bounds__(256) void plain_wtmap_kernel(FwdArgs A, PlainBufs Bf, int b) {
  b = plain_problem(A, b);
  const ProbDesc P = A.probs[b];
  const int w = blockIdx.x * 4 + wave_id(threadIdx.x);
  if (w >= nwindows(min(A.Tc, A.T))) return;
  const int S = 2 * P.n * A.nc;
  const float* V = Bf.V + (size_t)P.pos_off * 2;
  float* part = Bf.part + (size_t)nwindows(A.T) * P.coef_off + (size_t)w * S;
  for (int k0 = 0; k0 < A.T; k0 += A.Tc) {
    const int Tce = min(A.Tc, A.T - k0);
    if (w < nwindows(Tce))
      wtmap_window<KS>(A.W + (size_t)k0 * A.nc, A.nc, V + (size_t)k0 * 2, P.n, A.T, w, Tce, 0,
                       1, part, k0 > 0, threadIdx.x & 63);
  }
}

// lambda buffer of ping-pong parity pp (the plain path alternates lam and R).
__device__ __forceinline__ float* plain_lam(const PlainBufs& Bf, int pp) {
  return pp ? Bf.R : Bf.lam;
}

// Combine, lambda step and the xi_bar step (one block, the fused update).
template <int KS>
__global__ __launch_bounds__(256) void plain_update_kernel(FwdArgs A, PlainBufs Bf, int b,
                                                           int pp, int last) {
  __shared__ float csum[kColSums];
  __shared__ float red[kRed];
  b = plain_problem(A, b);
  const ProbDesc P = A.probs[b];
  const int n = P.n, nc = A.nc, S = 2 * n * nc, tid = threadIdx.x;
  const int lane = tid & 63, wave = wave_id(tid);
  const float* fac = A.fac + (size_t)P.fac * fac_stride(nc);
  const float* xb = Bf.xb[pp] + P.coef_off;
  float* xn = Bf.xb[pp ^ 1] + P.coef_off;
  const float* cx = Bf.cxi + P.coef_off;
  float dzsq = 0.f;
  floatx4 accP[tiles_per_wave(256)];
  update_fwd_p1<256, KS>(fac, nc, n, Bf.part + (size_t)nwindows(A.T) * P.coef_off,
                         nwindows(min(A.Tc, A.T)), S, plain_lam(Bf, pp) + P.coef_off,
                         plain_lam(Bf, pp ^ 1) + P.coef_off, xb, cx, A.rho, last, dzsq, csum,
                         accP, wave, lane);
  __syncthreads();
  update_fwd_p2<256>(nc, n, csum, accP, xb, xn, last, dzsq, nullptr, nullptr, 0.f, wave, lane);
  if (last) {
    float v[1] = {dzsq};
    block_sum(v, red);
    if (tid == 0) Bf.red[b * 4 + 2] = v[0];
  }
}

__global__ __launch_bounds__(256) void plain_final_kernel(FwdArgs A, PlainBufs Bf, int b,
                                                          int pp) {
  __shared__ float red[kRed];
  b = plain_problem(A, b);
  const ProbDesc P = A.probs[b];
  const int n = P.n, nc = A.nc, S = 2 * n * nc, tid = threadIdx.x;
  float r1sq = 0.f, r2sq = 0.f, bad = 0.f;
  constraints_full(reinterpret_cast<const float2*>(Bf.X) + P.pos_off,
                   reinterpret_cast<float2*>(Bf.V) + P.pos_off, n, A.T,
                   A.obstacles + (size_t)P.obs_off * 3,
                   A.ovel ? A.ovel + (size_t)P.obs_off * 2 : nullptr, P.M, P.a, P.pmin[0],
                   P.pmin[1], P.pmax[0], P.pmax[1], true, r1sq, r2sq, tid, 256);
  for (int s = tid; s < S; s += 256) {
    const float x = Bf.xb[pp][P.coef_off + s], lm = plain_lam(Bf, pp)[P.coef_off + s];
    A.xi_out[P.coef_off + s] = x;
    A.lam_out[P.coef_off + s] = lm;
    if (!isfinite(x) || !isfinite(lm)) bad = 1.f;
  }
  float v[3] = {r1sq, r2sq, bad};
  block_sum(v, red);
  if (tid == 0) {
    A.ws_iters[b] = A.L;
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

size_t plain_part_floats(int T, int64_t coef) { return (size_t)nwindows(T) * (size_t)coef; }

hipError_t launch_plain_problem(const FwdArgs& a, const PlainBufs& pb, int b, hipStream_t s) {
  // b >= 0: one problem per launch; b < 0: every launch covers the batch
  // (grid y = problem).  Grids are sized for the batch's largest problem; the
  // kernels stride over the items of their problem.
  const unsigned gy = b >= 0 ? 1u : (unsigned)a.B;
  const int gw = (nwindows(a.T) + 3) / 4;     // four waves per block, a window per wave
  const int gp = (nwindows(std::min(a.Tc, a.T)) + 3) / 4;
  const int gc = (a.n_max * a.T + 255) / 256;
  hipLaunchKernelGGL(plain_prep_kernel, dim3(1, gy), dim3(256), 0, s, a, pb, b);
  const bool k4 = ks_class(a.nc) == 4;
  auto xmap = k4 ? plain_xmap_kernel<4> : plain_xmap_kernel<8>;
  auto wtmap = k4 ? plain_wtmap_kernel<4> : plain_wtmap_kernel<8>;
  auto update = k4 ? plain_update_kernel<4> : plain_update_kernel<8>;
  int pp = 0;
  for (int l = 0; l < a.L; ++l) {
    hipLaunchKernelGGL(xmap, dim3(gw, gy), dim3(256), 0, s, a, pb, b, pp);
    hipLaunchKernelGGL(plain_constraint_kernel, dim3(gc, gy), dim3(256), 0, s, a, pb, b);
    hipLaunchKernelGGL(wtmap, dim3(gp, gy), dim3(256), 0, s, a, pb, b);
    hipLaunchKernelGGL(update, dim3(1, gy), dim3(256), 0, s, a, pb, b, pp, (int)(l == a.L - 1));
    pp ^= 1;
  }
  hipLaunchKernelGGL(xmap, dim3(gw, gy), dim3(256), 0, s, a, pb, b, pp);
  hipLaunchKernelGGL(plain_final_kernel, dim3(1, gy), dim3(256), 0, s, a, pb, b, pp);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace sf
