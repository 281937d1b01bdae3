// 3D (spheroid) SF: the forward (fwd3_kernel), its adjoint (bwd3_kernel) and
// the per-stage plain path (plain3_kernel); one workgroup per problem, the
// problem's state in LDS for all L iterations.
//
// Robots are axis-aligned spheroids (a/2, a/2, b/2) and obstacles spheroids
// (a_o, a_o, b_o) inflated by the robot (problem formulation; Appendix eqs.
// inter_robot_polar, workspace_polar).  The paper gives the alpha step's
// closed form only; the beta step (eq. beta_step) is read here as the polar
// angle of Delta in the spheroid's scaled coordinates, beta = atan2(rho_xy / a,
// dz / b) with rho_xy = dx cos(alpha) + dy sin(alpha) (for a != b not the
// Euclidean argmin with d held fixed), and d (eq. d_step) as the least-squares
// minimiser over d >= 1.  Together they put e on the ray of Delta: with
// s^2 = (dx^2 + dy^2)/a^2 + dz^2/b^2, e = Delta for s >= 1 and e = Delta / s
// inside, so r_1 = (1 - 1/s) Delta there (and at Delta = 0, alpha = beta = 0
// gives e = (0, 0, b)).  The xi_bar step is the
// planar one applied per axis: F, G and A are block diagonal over the three
// axes with identical blocks, so the planar (n, M) factor block serves each
// axis.
//
// One iteration, in time chunks of Tc steps held in LDS:
//   positions X = W xi_bar (MFMA tiles), stored as x/a, y/a, z/b   [3][n][Tc]
//   V = F^T r_1 + G^T r_2 per (robot, step), over each robot's     [3][n][Tc]
//       candidate partners and obstacles (or all of them)
//   R += W^T V (MFMA tiles)
// then lambda' = lambda - rho R, u = lambda - 2 rho R and the mode-form
// xi_bar' = c_xi + S u + SH xi_bar (S, SH: perpendicular block per robot plus
// the parallel-minus-perpendicular block on the robot mean).
#include <hip/hip_runtime.h>

#include <cfloat>

#include "sf_internal.h"

namespace sf {
namespace {

constexpr int kRed3 = 64;          // block-reduction scratch (3 values x 16 waves)
constexpr int kPlainThreads3 = 256;   // threads of the plain path's stage kernels
constexpr int kObsFloats = 12;     // obstacle table entry (10 used, see the set-up)

__host__ __device__ inline int r4(int x) { return (x + 3) & ~3; }

typedef float floatx4 __attribute__((ext_vector_type(4)));

// threadIdx.x passed through an empty asm: the per-lane addresses of each
// phase are then formed inside the iteration loop instead of being hoisted
// out of it by the compiler and held in registers for the whole loop (which
// exceeds the 128 VGPRs of a 1024-thread block and spills).
__device__ __forceinline__ int phase_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// The wave's index as a scalar: job and tile indices derived from it stay in
// scalar registers (divisions by tile counts run on the scalar unit).
__device__ __forceinline__ int wave_id3(int tid) { return __builtin_amdgcn_readfirstlane(tid >> 6); }

// Scheduling fence between a group of LDS operand reads and the MFMA chain
// that consumes them: the reads are all issued before the first MFMA (one
// wait for the group instead of one LDS round trip per MFMA step).
__device__ __forceinline__ void reads_first() { __builtin_amdgcn_sched_barrier(0); }

// C += A B on a 16x16x4 FP32 MFMA tile (A[m][k] and B[k][m] from lane
// m + 16 k; C[4 k + v][m] in accumulator v of lane m + 16 k).
__device__ __forceinline__ floatx4 mfma_16x16x4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float wave_sum3(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums of v[0..2] over the block, returned to every thread.
template <int NT>
__device__ __forceinline__ void block_sum3(float (&v)[3], float* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = NT >> 6;
#pragma unroll
  for (int q = 0; q < 3; ++q) v[q] = wave_sum3(v[q]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 3; ++q) red[q * NW + wave] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    float s = 0.f;
    for (int w = 0; w < NW; ++w) s += red[q * NW + w];
    v[q] = s;
  }
  __syncthreads();
}

// r_1 of one spheroid row from its scaled offset (ex, ey, ez) = (dx/sa,
// dy/sa, dz/sb), (sa, sb) the spheroid's semi-axes pair (a, b) or (a_o, b_o):
// s^2 = ex^2 + ey^2 + ez^2 and r_1 = (1 - 1/s) Delta for s < 1.  `tie` is the z
// value of r_1 at Delta = 0 (-b for the row's own orientation); rows with
// `live` false (a robot against itself) add nothing.  Adds r_1 to (vx, vy, vz)
// and, with SQ, |r_1|^2 to sq.  Active rows are rare, so the residual sits
// behind a branch that a wave skips when none of its lanes has one (the test
// alone is the common cost).  At Delta = 0 the clamped reciprocal square root
// is finite, so f * 0 = 0 and the tie term alone remains.
template <bool SQ>
__device__ __forceinline__ void spheroid_residual(float ex, float ey, float ez, float sa,
                                                  float sb, float tie, bool live, float& vx,
                                                  float& vy, float& vz, float& sq) {
  const float s2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
  if (live && s2 < 1.f) {
    const float f = 1.f - __builtin_amdgcn_rsqf(fmaxf(s2, FLT_MIN));
    const float rx = f * (sa * ex);
    const float ry = f * (sa * ey);
    const float rz = fmaf(f, sb * ez, s2 == 0.f ? tie : 0.f);
    vx += rx;
    vy += ry;
    vz += rz;
    if (SQ) sq = fmaf(rx, rx, fmaf(ry, ry, fmaf(rz, rz, sq)));
  }
}

// J^T w for the residual of one spheroid row, J = dr_1/dDelta of r_1 = (1 -
// 1/s) Delta (s < 1): J^T w = (1 - 1/s) w + (ex/sa, ey/sa, ez/sb) <Delta, w> / s^3
// with Delta = (sa ex, sa ey, sb ez).  At Delta = 0 e is locally constant, so J = I.
// Inactive rows (s >= 1 or `live` false) add nothing.  Added to (hx, hy, hz).
__device__ __forceinline__ void spheroid_vjp(float ex, float ey, float ez, float sa, float sb,
                                             float wx, float wy, float wz, bool live,
                                             float& hx, float& hy, float& hz) {
  const float s2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
  if (live && s2 < 1.f) {
    const float is = __builtin_amdgcn_rsqf(fmaxf(s2, FLT_MIN));
    const float f = s2 > 0.f ? 1.f - is : 1.f;
    const float c = s2 > 0.f ? is * is * is * fmaf(sb * ez, wz, sa * fmaf(ex, wx, ey * wy))
                             : 0.f;
    const float isa = 1.f / sa, isb = 1.f / sb;
    hx = fmaf(f, wx, fmaf(c * isa, ex, hx));
    hy = fmaf(f, wy, fmaf(c * isa, ey, hy));
    hz = fmaf(f, wz, fmaf(c * isb, ez, hz));
  }
}

// J^T r_1 of one spheroid row (the gradient of 1/2 |r_1|^2 with respect to
// Delta), from its scaled offset; at Delta = 0, r_1 itself (J = I there).
__device__ __forceinline__ void spheroid_resgrad(float ex, float ey, float ez, float sa,
                                                 float sb, float tie, bool live, float& vx,
                                                 float& vy, float& vz) {
  const float s2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
  if (live && s2 < 1.f) {
    const float f = 1.f - __builtin_amdgcn_rsqf(fmaxf(s2, FLT_MIN));
    const float rx = f * (sa * ex), ry = f * (sa * ey);
    const float rz = fmaf(f, sb * ez, s2 == 0.f ? tie : 0.f);
    spheroid_vjp(ex, ey, ez, sa, sb, rx, ry, rz, true, vx, vy, vz);
  }
}

// Robots per thread in the constraint stage: more robots share each LDS read,
// fewer threads have work; four from 24 robots, two from 8.
__device__ __forceinline__ int robots_per_thread(int n) { return n >= 24 ? 4 : (n >= 8 ? 2 : 1); }

// Candidate lists.  Each robot keeps, per window of kWin3 steps of the horizon,
// a bit mask of the partners and obstacles whose rows can be active in that
// window, built from window boxes of the positions (scaled coordinates) widened
// by a skin d.  A row with a scaled offset of magnitude >= 1 on some axis is
// inactive (its s^2 >= 1 in float too, the rounding being monotone), and a
// robot's positions are convex combinations of its coefficients (Bernstein
// weights, eq. poly), so the lists stay complete while no coefficient differs
// from its value at the last rebuild by more than d a (x, y) or d b (z); the
// first iteration in which one does, rebuilds them.  The sweep then walks the
// lists in increasing index: the rows it skips add exact zeros in the full
// sweep, so both give the same bits.
//
// The skin only trades rebuilds against longer walks, so it follows the
// iterates: d = 1/2 while the lists last few passes (early iterates move by
// more than a quarter of a semi-axis per iteration), 1/4 once they served
// sixteen passes or more, and back to 1/2 when the lists of a 1/4 skin serve a
// single pass (measured on 32 robots: a fixed 1/2 is 11 % faster than 1/4 over
// the first 100 iterations and 2 % slower over 1000; larger skins are slower).
// Every thread keeps its own copy and updates it at the same block-uniform
// points, so all agree; the lists always match the skin they were built with.
constexpr int kSlots3 = 16;        // per-wave flags of the list check (waves of 1024 threads)
constexpr float kSkinInit3 = 0.5f, kSkinMin3 = 0.25f, kSkinMax3 = 0.5f;
struct Skin3 {
  float d = kSkinInit3;   // skin in scaled units
  int age = 2;            // passes served by the current lists
  // one pass over the horizon, rebuilding or not
  __device__ __forceinline__ void pass(bool rebuild) {
    if (rebuild) {
      if (age <= 1)
        d = fminf(2.f * d, kSkinMax3);
      else if (age >= 16)
        d = fmaxf(0.5f * d, kSkinMin3);
      age = 0;
    }
    ++age;
  }
};
constexpr int kWinShift3 = 4;      // list window of 2^kWinShift3 steps
constexpr int kWin3 = 1 << kWinShift3;
constexpr int kListRob3 = 1;       // robots per thread of the list walk
static_assert(kWin3 >= 4, "window boxes of a chunk must fit in the V area");

// 32-bit mask words per (window, robot): partner words, then obstacle words.
__host__ __device__ inline int mask_words3(int n, int M) {
  return ((n + 31) >> 5) + ((M + 31) >> 5);
}
// LDS floats of the lists: reference coefficients, flags, masks of every
// window of a T-step horizon.
__host__ __device__ inline size_t list3_floats(int T, int n_max, int M_max, int S_max) {
  return (size_t)r4(S_max) + kSlots3 +
         (size_t)((T + kWin3 - 1) >> kWinShift3) * n_max * mask_words3(n_max, M_max);
}

struct Lds3 {
  float *W, *fac, *xb[2], *lam, *cxi, *R, *means, *obs, *X, *V, *red;
  float* refc;       // coefficients at the last list rebuild
  int* lslot;        // per-wave "moved" flags
  unsigned* mask;    // [window][n][mask_words3]
};

__device__ __forceinline__ Lds3 carve3(float* p, int nc, int Tc, int n_max, int M_max,
                                       int S_max) {
  Lds3 L;
  L.W = p; p += r4(Tc * nc);
  L.fac = p; p += r4(fac_stride(nc));
  L.xb[0] = p; p += r4(S_max);
  L.xb[1] = p; p += r4(S_max);
  L.lam = p; p += r4(S_max);
  L.cxi = p; p += r4(S_max);
  L.R = p; p += r4(S_max);
  L.means = p; p += 6 * kMaxCoef + 8;
  L.obs = p; p += kObsFloats * M_max;
  L.red = p; p += kRed3;
  L.X = p; p += r4(3 * n_max * (Tc | 1));
  L.V = p; p += r4(3 * n_max * (Tc | 1));
  // list area (used only when the lists are on)
  L.refc = p; p += r4(S_max);
  L.lslot = reinterpret_cast<int*>(p); p += kSlots3;
  L.mask = reinterpret_cast<unsigned*>(p);
  return L;
}

// The adjoint's arrangement of the same arrays (same total): xi_bar's
// ping-pong partner, lambda and c_xi last, after the list area (present only
// with the lists), so that the VJP chunk's G can lie over them during a
// reverse step (they are reloaded before a segment is recomputed).
__device__ __forceinline__ Lds3 carve3_adj(float* p, int nc, int T, int Tc, int n_max,
                                           int M_max, int S_max, bool lists) {
  Lds3 L;
  L.W = p; p += r4(Tc * nc);
  L.fac = p; p += r4(fac_stride(nc));
  L.xb[0] = p; p += r4(S_max);
  L.R = p; p += r4(S_max);
  L.means = p; p += 6 * kMaxCoef + 8;
  L.obs = p; p += kObsFloats * M_max;
  L.red = p; p += kRed3;
  L.X = p; p += r4(3 * n_max * (Tc | 1));
  L.V = p; p += r4(3 * n_max * (Tc | 1));
  L.refc = p;
  L.lslot = reinterpret_cast<int*>(p + r4(S_max));
  L.mask = reinterpret_cast<unsigned*>(p + r4(S_max) + kSlots3);
  if (lists) p += r4(list3_floats(T, n_max, M_max, S_max));
  L.xb[1] = p; p += r4(S_max);
  L.lam = p; p += r4(S_max);
  L.cxi = p;
  return L;
}

// LDS floats of the forward's layout (carve3), with or without the lists.
__host__ __device__ inline size_t lds3_floats(int nc, int T, int Tc, int n_max, int M_max,
                                              int S_max, bool lists) {
  return (size_t)r4(Tc * nc) + r4(fac_stride(nc)) + 5 * (size_t)r4(S_max) + 6 * kMaxCoef + 8 +
         (size_t)kObsFloats * M_max + kRed3 + 2 * (size_t)r4(3 * n_max * (Tc | 1)) +
         (lists ? r4(list3_floats(T, n_max, M_max, S_max)) : 0);
}

// List check: every wave records whether a coefficient it compared moved
// further than the skin; all waves read the flags at the next sweep.
__device__ __forceinline__ void note_moved3(bool moved, int* lslot) {
  const bool any = __builtin_amdgcn_ballot_w64(moved) != 0ull;
  if ((threadIdx.x & 63) == 0) lslot[threadIdx.x >> 6] = any ? 1 : 0;
}
__device__ __forceinline__ bool lists_moved3(const int* lslot, int nwaves) {
  const int lane = threadIdx.x & 63;
  const int v = lane < nwaves ? lslot[lane] : 0;
  return __builtin_amdgcn_ballot_w64(v != 0) != 0ull;
}
// Before the first sweep: every flag set and a NaN reference, so that a check
// made before the first rebuild still reports a move.
template <int NT>
__device__ __forceinline__ void reset_lists3(float* refc, int* lslot, int S) {
  for (int t = threadIdx.x; t < S; t += NT) refc[t] = __builtin_nanf("");
  if (threadIdx.x < kSlots3) lslot[threadIdx.x] = 1;
}
// Whether coefficient t of x (layout [3][n][nc], nn = n nc) left the skin.
__device__ __forceinline__ bool coef_moved3(const float* x, const float* ref, int t, int nn,
                                            float ska, float skb) {
  return !(fabsf(x[t] - ref[t]) <= (t < 2 * nn ? ska : skb));
}

// Lists of the windows of a chunk of Tce steps starting at step k0 (a
// multiple of kWin3), from the scaled positions in L.X: list_boxes3 writes
// the window boxes to L.V (written again only after the lists), over threads
// t0, t0 + nt, ...; list_masks3 then ballots the masks.
// Margins: a pair is kept when its boxes come within 1 + 2 d (both robots may
// move by d), an obstacle when the box of the offset in the obstacle's scaling
// comes within 1 + d (r_a, r_b) of the origin; 1e-4 (1 + magnitudes) more on
// each covers the float rounding of the positions and of the tests, which is
// orders of magnitude smaller.  A ballot tests two robots against 32
// candidates at once (lane = 32 slot + jj).
__device__ __forceinline__ void list_boxes3(const ProbDesc& P, const Lds3& L, int Tce, int Ts,
                                            int t0, int nt) {
  const int n = P.n, nwc = (Tce + kWin3 - 1) >> kWinShift3;
  float* box = L.V;   // [3 n][nwc] (lo, hi)
  for (int t = t0; t < 3 * n * nwc; t += nt) {
    const int row = t / nwc, wl = t - row * nwc;
    const float* x = L.X + row * Ts + wl * kWin3;
    const int cnt = min(kWin3, Tce - wl * kWin3);
    float lo = x[0], hi = x[0];
    for (int s = 1; s < cnt; ++s) {
      lo = fminf(lo, x[s]);
      hi = fmaxf(hi, x[s]);
    }
    box[2 * t] = lo;
    box[2 * t + 1] = hi;
  }
}

// The masks of list_boxes3's windows.  A job is (window, mask word, range of
// robot pairs): a lane holds its candidate (partner j = 32 word + jj, or
// obstacle 32 (word - pw) + jj) and that candidate's part of the test, and
// each robot pair of the range takes one ballot (lane = 32 slot + jj: robots
// 2 ip and 2 ip + 1), reading only the two robots' boxes.
__device__ __forceinline__ void list_masks3(const ProbDesc& P, const Lds3& L, int k0, int Tce,
                                            float inv_Tm1, bool moving, float d, int w0,
                                            int nw) {
  const int n = P.n, M = P.M, lane = phase_tid() & 63;
  const int nwc = (Tce + kWin3 - 1) >> kWinShift3;
  const float* box = L.V;
  const int pw = (n + 31) >> 5, mw = mask_words3(n, M), np = (n + 1) >> 1;
  const int slot = lane >> 5, jj = lane & 31;
  // ranges of robot pairs per (window, word): enough jobs for the waves
  const int split = min(max((nw + nwc * mw - 1) / (nwc * mw), 1), np);
  const int per = (np + split - 1) / split, jobs = nwc * mw * split;
  for (int q = w0; q < jobs; q += nw) {
    const int wl = q / (mw * split), rem = q - wl * (mw * split);
    const int word = rem / split, ip0 = (rem - word * split) * per, ip1 = min(np, ip0 + per);
    unsigned* mk = L.mask + (size_t)((k0 >> kWinShift3) + wl) * n * mw + word;
    if (word < pw) {
      const int j = 32 * word + jj, jc = min(j, n - 1);
      float jlo[3], jhi[3], jmag[3];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const float* bj = box + ((ax * n + jc) * nwc + wl) * 2;
        jlo[ax] = bj[0];
        jhi[ax] = bj[1];
        jmag[ax] = fmaxf(fabsf(bj[0]), fabsf(bj[1]));
      }
      for (int ip = ip0; ip < ip1; ++ip) {
        const int i = 2 * ip + slot, ic = min(i, n - 1);
        bool c = i < n && j < n && j != i;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const float* bi = box + ((ax * n + ic) * nwc + wl) * 2;
          const float mag = fmaxf(fmaxf(fabsf(bi[0]), fabsf(bi[1])), jmag[ax]);
          const float thr = 1.f + 2.f * d + 1e-4f * (1.f + mag);
          c = c && (bi[0] - jhi[ax] < thr) && (jlo[ax] - bi[1] < thr);
        }
        const unsigned long long bal = __builtin_amdgcn_ballot_w64(c);
        if (lane == 0) {
          mk[(size_t)2 * ip * mw] = (unsigned)bal;
          if (2 * ip + 1 < n) mk[(size_t)(2 * ip + 1) * mw] = (unsigned)(bal >> 32);
        }
      }
    } else {
      const int mo = 32 * (word - pw) + jj;
      const float* o = L.obs + min(mo, M - 1) * kObsFloats;
      // the obstacle's centre term is monotone in the step, so its range over
      // the window is that of the window's first and last steps
      const float ta = (float)(k0 + wl * kWin3) * inv_Tm1;
      const float tb = (float)(k0 + min(wl * kWin3 + kWin3 - 1, Tce - 1)) * inv_Tm1;
      float clo[3], chi[3], rr[3];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const float ca = moving ? fmaf(o[7 + ax], ta, o[2 + ax]) : o[2 + ax];
        const float cb = moving ? fmaf(o[7 + ax], tb, o[2 + ax]) : o[2 + ax];
        clo[ax] = fminf(ca, cb);
        chi[ax] = fmaxf(ca, cb);
        rr[ax] = ax < 2 ? o[0] : o[1];
      }
      for (int ip = ip0; ip < ip1; ++ip) {
        const int i = 2 * ip + slot, ic = min(i, n - 1);
        bool c = i < n && mo < M;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const float* bi = box + ((ax * n + ic) * nwc + wl) * 2;
          const float r = rr[ax];
          const float elo = fmaf(bi[0], r, clo[ax]), ehi = fmaf(bi[1], r, chi[ax]);
          const float sl = fmaf(r, d, 1e-4f * (1.f + fabsf(elo) + fabsf(ehi) +
                                               r * (fabsf(bi[0]) + fabsf(bi[1]))));
          c = c && (elo - sl < 1.f) && (ehi + sl > -1.f);
        }
        const unsigned long long bal = __builtin_amdgcn_ballot_w64(c);
        if (lane == 0) {
          mk[(size_t)2 * ip * mw] = (unsigned)bal;
          if (2 * ip + 1 < n) mk[(size_t)(2 * ip + 1) * mw] = (unsigned)(bal >> 32);
        }
      }
    }
  }
}

// Both passes over the block, each ending at a barrier.
template <int NT>
__device__ __forceinline__ void build_lists3(const ProbDesc& P, const Lds3& L, int k0, int Tce,
                                             int Ts, float inv_Tm1, bool moving, float d) {
  const int tid = phase_tid();
  list_boxes3(P, L, Tce, Ts, tid, NT);
  __syncthreads();
  list_masks3(P, L, k0, Tce, inv_Tm1, moving, d, wave_id3(tid), NT >> 6);
  __syncthreads();
}

// Passes over the horizon at xi_bar = xb (MODE): kForward gives positions X,
// constraint sums V and R = W^T V; kFinal the residual sums ||r_1||^2 and
// ||r_2||^2 instead; kResGrad R = W^T V with V = w1 sum J^T r_1 + w2 (box
// overshoot), the gradient of w1 ||r_1||^2 / 2 + w2 ||r_2||^2 / 2.
constexpr int kForward = 0, kFinal = 1, kResGrad = 2;

// Position tiles: dst[col][step] = scale(col) sum_c W[step][c] Y[col][c]
// (col < rows; scale s_lo for col < rows_lo, else s_hi) on MFMA 16x16x4 tiles
// of 16 steps x 16 columns.  A lane supplies A[m][k] = W[16 wt + m][4 s + k']
// and B[k][m] = Y[16 ct + m][4 s + k'] (m = lane % 16, k' = lane / 16) and
// holds dst[16 ct + m][16 wt + 4 k' + v]; coefficients past nc enter as 0.
// Every operand read of a tile is issued before its chain of KS = ceil(nc/4)
// MFMA steps.  Tiles q0, q0 + qs, ... of nsrc sources (Y0 -> D0 scaled, Y1 ->
// D1 unscaled) are this wave's.
template <int KS>
__device__ __forceinline__ void map_tiles3(const float* Wc, int nc, int rows, int Ts, int Tce,
                                           const float* Y0, float* D0, float s_lo, float s_hi,
                                           int rows_lo, const float* Y1, float* D1, int nsrc,
                                           int q0, int qs) {
  const int lane = phase_tid() & 63, m = lane & 15, kq = lane >> 4;
  const int nwt = (Tce + 15) >> 4, nct = (rows + 15) >> 4, per = nwt * nct;
  for (int q = q0; q < nsrc * per; q += qs) {
    const int src = q >= per, qq = q - src * per;
    const int wt = qq / nct, ct = qq - wt * nct;
    const float* Y = src ? Y1 : Y0;
    const int stepA = min(wt * 16 + m, Tce - 1), colB = min(ct * 16 + m, rows - 1);
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    if (KS > 0) {
      constexpr int K = KS > 0 ? KS : 1;
      float a[K], b[K];
#pragma unroll
      for (int s4 = 0; s4 < K; ++s4) {
        const int c = 4 * s4 + kq, cc = min(c, nc - 1);
        const float w = Wc[stepA * nc + cc];
        a[s4] = c < nc ? w : 0.f;
        b[s4] = Y[colB * nc + cc];
      }
      reads_first();
#pragma unroll
      for (int s4 = 0; s4 < K; ++s4) acc = mfma_16x16x4(a[s4], b[s4], acc);
    } else {
      for (int s4 = 0; s4 < ((nc + 3) >> 2); ++s4) {
        const int c = 4 * s4 + kq, cc = min(c, nc - 1);
        const float w = Wc[stepA * nc + cc];
        acc = mfma_16x16x4(c < nc ? w : 0.f, Y[colB * nc + cc], acc);
      }
    }
    // stores without branches: a padding step's value is that of step Tce - 1
    // and a padding column's that of column rows - 1 (the same operands give
    // the same bits), so their clamped stores repeat those values
    const int col = min(ct * 16 + m, rows - 1);
    const float sc = src ? 1.f : (col < rows_lo ? s_lo : s_hi);
    float* d = (src ? D1 : D0) + col * Ts;
    const int k = wt * 16 + 4 * kq;
#pragma unroll
    for (int v = 0; v < 4; ++v) d[min(k + v, Tce - 1)] = acc[v] * sc;
  }
}

// map_tiles3 for nc coefficients: three or four MFMA steps with their
// operands read first up to 16 coefficients (steps past nc add exact zeros),
// a plain loop above.
__device__ __forceinline__ void map_tiles3_any(const float* Wc, int nc, int rows, int Ts,
                                               int Tce, const float* Y0, float* D0, float s_lo,
                                               float s_hi, int rows_lo, const float* Y1,
                                               float* D1, int nsrc, int q0, int qs) {
  if (nc <= 12)
    map_tiles3<3>(Wc, nc, rows, Ts, Tce, Y0, D0, s_lo, s_hi, rows_lo, Y1, D1, nsrc, q0, qs);
  else if (nc <= 16)
    map_tiles3<4>(Wc, nc, rows, Ts, Tce, Y0, D0, s_lo, s_hi, rows_lo, Y1, D1, nsrc, q0, qs);
  else
    map_tiles3<0>(Wc, nc, rows, Ts, Tce, Y0, D0, s_lo, s_hi, rows_lo, Y1, D1, nsrc, q0, qs);
}

// R (+)= W^T V over a chunk of Tce steps: MFMA 16x16x4 tiles of 16 rows x 16
// coefficients, A[m][k] = V[16 rt + m][4 s + k'], B[k][m] = W[4 s + k'][16 ct
// + m]; steps past Tce enter as 0.  Even and odd s go to two accumulators,
// added at the end; the operands of eight steps are read before their MFMAs.
template <int NT>
__device__ __forceinline__ void wtv_tiles3(const float* V, int Ts, const float* Wc, int nc,
                                           int Tce, int rows, float* R, bool first) {
  const int tid = phase_tid(), lane = tid & 63, wave = wave_id3(tid), m = lane & 15, kq = lane >> 4;
  const int nrt = (rows + 15) >> 4, nct = (nc + 15) >> 4, nk = (Tce + 3) >> 2;
  for (int q = wave; q < nrt * nct; q += NT >> 6) {
    const int rt = q / nct, ct = q - rt * nct;
    const int rowA = min(rt * 16 + m, rows - 1), cB = min(ct * 16 + m, nc - 1);
    const float* vrow = V + rowA * Ts;
    floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    int s0 = 0;
    for (; s0 + 8 <= nk; s0 += 8) {
      float a[8], b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = 4 * (s0 + u) + kq, kc = min(k, Tce - 1);
        const float v = vrow[kc];
        a[u] = k < Tce ? v : 0.f;
        b[u] = Wc[kc * nc + cB];
      }
      reads_first();
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        acc0 = mfma_16x16x4(a[u], b[u], acc0);
        acc1 = mfma_16x16x4(a[u + 1], b[u + 1], acc1);
      }
    }
    for (; s0 < nk; ++s0) {
      const int k = 4 * s0 + kq, kc = min(k, Tce - 1);
      const float v = vrow[kc];
      const float a = k < Tce ? v : 0.f, b = Wc[kc * nc + cB];
      if (s0 & 1)
        acc1 = mfma_16x16x4(a, b, acc1);
      else
        acc0 = mfma_16x16x4(a, b, acc0);
    }
    const int c = ct * 16 + m;
    if (c < nc) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rt * 16 + 4 * kq + v;
        if (row < rows) {
          const float sum = acc0[v] + acc1[v];
          R[row * nc + c] = first ? sum : R[row * nc + c] + sum;
        }
      }
    }
  }
}

// The rows of kRob robots (indices ir, scaled positions p) against partner
// j at scaled position q: r_1 (kForward, and |r_1|^2 for each unordered pair
// once in kFinal) or J^T r_1 (kResGrad) added to v.
template <int MODE, int kRob>
__device__ __forceinline__ void pair_rows3(const ProbDesc& P, const int (&ir)[kRob], int j,
                                           const float (&px)[kRob], const float (&py)[kRob],
                                           const float (&pz)[kRob], float qx, float qy,
                                           float qz, float (&vx)[kRob], float (&vy)[kRob],
                                           float (&vz)[kRob], float (&sq)[kRob]) {
  constexpr bool FINAL = MODE == kFinal;
#pragma unroll
  for (int r = 0; r < kRob; ++r) {
    float s1 = 0.f;
    if (MODE == kResGrad)
      spheroid_resgrad(px[r] - qx, py[r] - qy, pz[r] - qz, P.a, P.b, ir[r] < j ? -P.b : P.b,
                       j != ir[r], vx[r], vy[r], vz[r]);
    else
      spheroid_residual<FINAL>(px[r] - qx, py[r] - qy, pz[r] - qz, P.a, P.b,
                               ir[r] < j ? -P.b : P.b, j != ir[r], vx[r], vy[r], vz[r], s1);
    if (FINAL) sq[r] += j > ir[r] ? s1 : 0.f;   // each unordered pair once
  }
}

// The rows of kRob robots against obstacle entry o (see setup3) at time tau.
template <int MODE, int kRob>
__device__ __forceinline__ void obstacle_rows3(const float* o, float tau, bool moving,
                                               const float (&px)[kRob], const float (&py)[kRob],
                                               const float (&pz)[kRob], float (&vx)[kRob],
                                               float (&vy)[kRob], float (&vz)[kRob],
                                               float (&sq)[kRob]) {
  const float cx = moving ? fmaf(o[7], tau, o[2]) : o[2];
  const float cy = moving ? fmaf(o[8], tau, o[3]) : o[3];
  const float cz = moving ? fmaf(o[9], tau, o[4]) : o[4];
  const float ra = o[0], rb = o[1], oa = o[5], ob = o[6];
#pragma unroll
  for (int r = 0; r < kRob; ++r) {
    if (MODE == kResGrad)
      spheroid_resgrad(fmaf(px[r], ra, cx), fmaf(py[r], ra, cy), fmaf(pz[r], rb, cz), oa, ob,
                       -ob, true, vx[r], vy[r], vz[r]);
    else
      spheroid_residual<MODE == kFinal>(fmaf(px[r], ra, cx), fmaf(py[r], ra, cy),
                                        fmaf(pz[r], rb, cz), oa, ob, -ob, true, vx[r], vy[r],
                                        vz[r], sq[r]);
  }
}

template <int NT, int MODE, int kRob, typename Args>
__device__ __forceinline__ void sweep3(const Args& A, const ProbDesc& P, const Lds3& L,
                                       const float* xb, float& r1sq, float& r2sq, Skin3& sk,
                                       float w1 = 1.f, float w2 = 1.f) {
  constexpr bool FINAL = MODE == kFinal;
  const int n = P.n, M = P.M, nc = A.nc, T = A.T, Tc = A.Tc, tid = phase_tid();
  const bool chunked = Tc < T;
  const float inv_a = 1.f / P.a, inv_b = 1.f / P.b;
  const float inv_Tm1 = 1.f / (float)(T - 1);
  const bool moving = A.ovel != nullptr;
  // candidate lists: rebuilt in this pass when a wave flagged a move (every
  // thread reads the flags here; they are cleared after the first map), with
  // xb as the new reference
  const bool lists = A.lists3 != 0;
  const bool rebuild = lists && lists_moved3(L.lslot, NT >> 6);
  if (lists) sk.pass(rebuild);
  if (rebuild)
    for (int t = tid; t < 3 * n * nc; t += NT) L.refc[t] = xb[t];
  for (int k0 = 0; k0 < T; k0 += Tc) {
    const int Tce = min(Tc, T - k0);
    const int Ts = Tce | 1;   // odd row stride of X and V: column reads without bank conflicts
    if (chunked) {
      for (int t = tid; t < Tce * nc; t += NT) L.W[t] = A.W[k0 * nc + t];
      __syncthreads();
    }
    const float* Wc = chunked ? L.W : L.W + k0 * nc;
    // positions X[row][kk] = sum_c W[kk][c] xb[row][c] (row = axis * n +
    // robot), stored scaled by the robot's semi-axes: x/a, y/a, z/b
    map_tiles3_any(Wc, nc, 3 * n, Ts, Tce, xb, L.X, inv_a, inv_b, 2 * n, nullptr, nullptr, 1,
                   wave_id3(tid), NT >> 6);
    __syncthreads();
    if (lists && rebuild) {
      if (k0 == 0 && tid < kSlots3) L.lslot[tid] = 0;   // every thread has read the flags
      build_lists3<NT>(P, L, k0, Tce, Ts, inv_Tm1, moving, sk.d);
    }
    // constraint rows (robot pairs, obstacles, the box).  A thread takes kRob
    // robots at one step, so each partner position and obstacle read from LDS
    // serves kRob rows; every row still sums its terms in the same order
    // (partners j = 0..n-1, then obstacles), over all of them or, with the
    // lists, over the union of its robots' lists.  kRob depends on the
    // problem's robot count only (robots_per_thread), not on the block size.
    const int plane = n * Ts;
    const int ngrp = (n + kRob - 1) / kRob;
    const int pw = (n + 31) >> 5, mw = mask_words3(n, M);
    for (int t = tid; t < ngrp * Tce; t += NT) {
      const int g = t / Tce, kk = t - g * Tce;
      float px[kRob], py[kRob], pz[kRob], vx[kRob], vy[kRob], vz[kRob], sq[kRob];
      int ir[kRob];
#pragma unroll
      for (int r = 0; r < kRob; ++r) {
        ir[r] = g * kRob + r;
        const int u = min(ir[r], n - 1) * Ts + kk;
        px[r] = L.X[u];
        py[r] = L.X[plane + u];
        pz[r] = L.X[2 * plane + u];
        vx[r] = vy[r] = vz[r] = sq[r] = 0.f;
      }
      // obstacle offsets in the obstacle's scaling: (a x' - c - d tau) / a_o
      // (x' the stored x / a), i.e. x' (a / a_o) - c / a_o - (d / a_o) tau
      const float tau = (float)(k0 + kk) * inv_Tm1;
      if (lists) {
        const unsigned* mk = L.mask + ((size_t)((k0 + kk) >> kWinShift3) * n + g * kRob) * mw;
        for (int q = 0; q < pw; ++q) {
          unsigned u = 0u;
#pragma unroll
          for (int r = 0; r < kRob; ++r)
            if (ir[r] < n) u |= mk[r * mw + q];
          while (u) {
            const int j = (__ffs(u) - 1) + 32 * q;
            u &= u - 1u;
            const int v = j * Ts + kk;
            pair_rows3<MODE, kRob>(P, ir, j, px, py, pz, L.X[v], L.X[plane + v],
                                   L.X[2 * plane + v], vx, vy, vz, sq);
          }
        }
        for (int q = 0; q < mw - pw; ++q) {
          unsigned u = 0u;
#pragma unroll
          for (int r = 0; r < kRob; ++r)
            if (ir[r] < n) u |= mk[r * mw + pw + q];
          while (u) {
            const int mo = (__ffs(u) - 1) + 32 * q;
            u &= u - 1u;
            obstacle_rows3<MODE, kRob>(L.obs + mo * kObsFloats, tau, moving, px, py, pz, vx,
                                       vy, vz, sq);
          }
        }
      } else {
        // partners in groups of four, every read of a group issued first
        int j0 = 0;
        for (; j0 + 4 <= n; j0 += 4) {
          float qx[4], qy[4], qz[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int u = (j0 + e) * Ts + kk;
            qx[e] = L.X[u];
            qy[e] = L.X[plane + u];
            qz[e] = L.X[2 * plane + u];
          }
#pragma unroll
          for (int e = 0; e < 4; ++e)
            pair_rows3<MODE, kRob>(P, ir, j0 + e, px, py, pz, qx[e], qy[e], qz[e], vx, vy, vz,
                                   sq);
        }
        for (int j = j0; j < n; ++j) {
          const int u = j * Ts + kk;
          pair_rows3<MODE, kRob>(P, ir, j, px, py, pz, L.X[u], L.X[plane + u],
                                 L.X[2 * plane + u], vx, vy, vz, sq);
        }
        for (int mo = 0; mo < M; ++mo)
          obstacle_rows3<MODE, kRob>(L.obs + mo * kObsFloats, tau, moving, px, py, pz, vx, vy,
                                     vz, sq);
      }
#pragma unroll
      for (int r = 0; r < kRob; ++r) {
        if (ir[r] >= n) continue;
        const int u = ir[r] * Ts + kk;
        const float x = P.a * px[r], y = P.a * py[r], z = P.b * pz[r];
        const float hx = fmaxf(x - P.pmax[0], 0.f), lx = fmaxf(P.pmin[0] - x, 0.f);
        const float hy = fmaxf(y - P.pmax[1], 0.f), ly = fmaxf(P.pmin[1] - y, 0.f);
        const float hz = fmaxf(z - P.pmax[2], 0.f), lz = fmaxf(P.pmin[2] - z, 0.f);
        if (FINAL) {   // the row's shares, summed below in a fixed order
          L.V[u] = sq[r];
          L.V[plane + u] = hx * hx + lx * lx + hy * hy + ly * ly + hz * hz + lz * lz;
        } else if (MODE == kResGrad) {
          L.V[u] = fmaf(w2, hx - lx, w1 * vx[r]);
          L.V[plane + u] = fmaf(w2, hy - ly, w1 * vy[r]);
          L.V[2 * plane + u] = fmaf(w2, hz - lz, w1 * vz[r]);
        } else {
          L.V[u] = vx[r] + (hx - lx);
          L.V[plane + u] = vy[r] + (hy - ly);
          L.V[2 * plane + u] = vz[r] + (hz - lz);
        }
      }
    }
    __syncthreads();
    if (FINAL) {
      // ||r_1||^2 and ||r_2||^2 of the chunk: 256 partial sums over rows e =
      // p (mod 256) in increasing order, the same whatever the block size and
      // the robots per thread (the caller then adds the partials per wave and
      // the waves in order)
      if (tid < 256)
        for (int e = tid; e < n * Tce; e += 256) {
          const int i = e / Tce, kk = e - i * Tce;
          r1sq += L.V[i * Ts + kk];
          r2sq += L.V[plane + i * Ts + kk];
        }
      __syncthreads();
    } else {
      wtv_tiles3<NT>(L.V, Ts, Wc, nc, Tce, 3 * n, L.R, k0 == 0);
      __syncthreads();
    }
  }
}

// Sweep dispatch on the problem's robots per thread.
template <int NT, int MODE, typename Args>
__device__ __forceinline__ void sweep3_any(const Args& A, const ProbDesc& P, const Lds3& L,
                                           const float* xb, float& r1sq, float& r2sq, Skin3& sk,
                                           float w1 = 1.f, float w2 = 1.f) {
  const int rpt = robots_per_thread(P.n);
  if (A.lists3)
    sweep3<NT, MODE, kListRob3>(A, P, L, xb, r1sq, r2sq, sk, w1, w2);
  else if (rpt == 4)
    sweep3<NT, MODE, 4>(A, P, L, xb, r1sq, r2sq, sk, w1, w2);
  else if (rpt == 2)
    sweep3<NT, MODE, 2>(A, P, L, xb, r1sq, r2sq, sk, w1, w2);
  else
    sweep3<NT, MODE, 1>(A, P, L, xb, r1sq, r2sq, sk, w1, w2);
}

// Set-up shared by the forward and the adjoint: factor block, W (whole table
// when unchunked) and the obstacle table from obstacles [M][5] (x, y, z, a_o,
// b_o) and optional displacements [M][3].
template <int NT, typename Args>
__device__ __forceinline__ void setup3(const Args& A, const ProbDesc& P, const Lds3& L,
                                       const float* obstacles) {
  const int M = P.M, nc = A.nc, T = A.T, tid = threadIdx.x;
  const float* facg = A.fac + (size_t)P.fac * fac_stride(nc);
  for (int t = tid; t < fac_stride(nc); t += NT) L.fac[t] = facg[t];
  if (A.Tc >= T)
    for (int t = tid; t < T * nc; t += NT) L.W[t] = A.W[t];
  for (int m = tid; m < M; m += NT) {
    const float* o = obstacles + (size_t)(P.obs_off + m) * 5;
    float* d = L.obs + m * kObsFloats;
    // the offset from a robot in the obstacle's scaling (a_o, a_o, b_o), from
    // the robot's stored scaled position: a / a_o, b / b_o, -c / (a_o, a_o,
    // b_o), the semi-axes, -d / (a_o, a_o, b_o) for moving obstacles
    const float ia = 1.f / o[3], ib = 1.f / o[4];
    d[0] = P.a * ia;
    d[1] = P.b * ib;
    d[2] = -o[0] * ia;
    d[3] = -o[1] * ia;
    d[4] = -o[2] * ib;
    d[5] = o[3];
    d[6] = o[4];
    const float* v = A.ovel ? A.ovel + (size_t)(P.obs_off + m) * 3 : nullptr;
    d[7] = v ? -v[0] * ia : 0.f;
    d[8] = v ? -v[1] * ia : 0.f;
    d[9] = v ? -v[2] * ib : 0.f;
  }
}

// Robot means per (axis, coefficient) of u = lambda - 2 rho R (into
// L.means[ax nc + q]) and of x (into L.means[3 nc + ax nc + q]), one (axis,
// quantity) job per wave: lane q + QW p sums the robots i = p (mod 64 / QW) in
// two chains, then a butterfly over p.
template <int NT>
__device__ __forceinline__ void mean_field3(const ProbDesc& P, const Lds3& L, int nc, float rho,
                                            const float* x) {
  const int n = P.n, nn = n * nc, tid = phase_tid(), lane = tid & 63;
  const int QW = nc <= 16 ? 16 : 32, Pw = 64 / QW;
  const int q = lane % QW, p = lane / QW, qq = min(q, nc - 1);
  for (int job = wave_id3(tid); job < 6; job += NT >> 6) {
    const int ax = job >> 1, which = job & 1;
    const float* lam = L.lam + ax * nn + qq;
    const float* R = L.R + ax * nn + qq;
    const float* xa = x + ax * nn + qq;
    float s0 = 0.f, s1 = 0.f;
    int i = p;
    for (; i + Pw < n; i += 2 * Pw) {
      const int i1 = i + Pw;
      s0 += which ? xa[i * nc] : fmaf(-2.f * rho, R[i * nc], lam[i * nc]);
      s1 += which ? xa[i1 * nc] : fmaf(-2.f * rho, R[i1 * nc], lam[i1 * nc]);
    }
    if (i < n) s0 += which ? xa[i * nc] : fmaf(-2.f * rho, R[i * nc], lam[i * nc]);
    float sm = s0 + s1;
    for (int o = QW; o < 64; o <<= 1) sm += __shfl_xor(sm, o, 64);
    if (p == 0 && q < nc) L.means[which * 3 * nc + ax * nc + q] = sm / (float)n;
  }
}

// The xi_bar step on MFMA 16x16x4 tiles, one wave per tile of 16 rows (row =
// axis * n + robot) and every coefficient column tile:
//   xi_bar'[row][c] = c_xi + sum_q (u[row][q] S[c][q] + um[axis][q] DS[c][q])
//                           + sum_q (x[row][q] SH[c][q] + xm[axis][q] DSH[c][q])
// with u = lambda - 2 rho R formed as the A operand is read (A[m][k] =
// u[16 rt + m][4 s + k'], B[k][m] = S[16 ct + m][4 s + k'], KS >= nc/4
// steps in groups of four whose operand reads are issued first; steps past
// nc add exact zeros).  The tile's lanes then write lambda'
// = lambda - rho R of their own entries (no other wave reads these rows),
// check the candidate lists and, with `last`, add ||z' - z||^2.
template <int NT, int KS>
__device__ __forceinline__ void xi_step3(const ProbDesc& P, const Lds3& L, int nc, float rho,
                                         const float* xcur, float* xnext, bool last,
                                         bool lists, float d, float& dzsq) {
  const int n = P.n, nc2 = nc * nc, rows = 3 * n;
  const int tid = phase_tid(), lane = tid & 63, wave = wave_id3(tid), m = lane & 15, kq = lane >> 4;
  const int nrt = (rows + 15) >> 4, nct = (nc + 15) >> 4;
  const float ska = d * P.a, skb = d * P.b;
  bool moved = false;
  for (int rt = wave; rt < nrt; rt += NT >> 6) {
    const int rowA = min(rt * 16 + m, rows - 1), axA = rowA / n;
    floatx4 acc[2][2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[ct][0] = acc[ct][1] = floatx4{0.f, 0.f, 0.f, 0.f};
    // KS > 0: groups of up to four MFMA steps, every operand of a group read
    // first; KS = 0: one step at a time over ceil(nc / 4) steps
    const int ksteps = KS > 0 ? KS : (nc + 3) >> 2;
#pragma unroll
    for (int g0 = 0; g0 < ksteps; g0 += (KS > 0 ? 4 : 1)) {
      constexpr int KG = KS == 0 ? 1 : (KS < 4 ? KS : 4);
      float au[KG], aum[KG], ax[KG], axm[KG];
#pragma unroll
      for (int e = 0; e < KG; ++e) {
        const int q = 4 * (g0 + e) + kq, qq = min(q, nc - 1);
        const bool ok = g0 + e < ksteps && q < nc;
        const float u = fmaf(-2.f * rho, L.R[rowA * nc + qq], L.lam[rowA * nc + qq]);
        const float um = L.means[axA * nc + qq], xv = xcur[rowA * nc + qq];
        const float xm = L.means[3 * nc + axA * nc + qq];
        au[e] = ok ? u : 0.f;
        aum[e] = ok ? um : 0.f;
        ax[e] = ok ? xv : 0.f;
        axm[e] = ok ? xm : 0.f;
      }
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        if (ct >= nct) continue;
        const float* Sr = L.fac + min(ct * 16 + m, nc - 1) * nc;
        float bs[KG], bds[KG], bsh[KG], bdsh[KG];
#pragma unroll
        for (int e = 0; e < KG; ++e) {
          const int qq = min(4 * (g0 + e) + kq, nc - 1);
          bs[e] = Sr[qq];
          bds[e] = Sr[nc2 + qq];
          bsh[e] = Sr[2 * nc2 + qq];
          bdsh[e] = Sr[3 * nc2 + qq];
        }
        reads_first();
#pragma unroll
        for (int e = 0; e < KG; ++e) {
          acc[ct][0] = mfma_16x16x4(au[e], bs[e], acc[ct][0]);
          acc[ct][1] = mfma_16x16x4(ax[e], bsh[e], acc[ct][1]);
        }
#pragma unroll
        for (int e = 0; e < KG; ++e) {
          acc[ct][0] = mfma_16x16x4(aum[e], bds[e], acc[ct][0]);
          acc[ct][1] = mfma_16x16x4(axm[e], bdsh[e], acc[ct][1]);
        }
      }
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int c = ct * 16 + m;
      if (ct >= nct || c >= nc) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rt * 16 + 4 * kq + v;
        if (row >= rows) continue;
        const int e = row * nc + c;
        const float val = L.cxi[e] + (acc[ct][0][v] + acc[ct][1][v]);
        xnext[e] = val;
        const float r = L.R[e];
        L.lam[e] = fmaf(-rho, r, L.lam[e]);
        if (lists) moved |= !(fabsf(val - L.refc[e]) <= (row < 2 * n ? ska : skb));
        if (last) {
          const float d = val - xcur[e];
          dzsq = fmaf(rho * r, rho * r, fmaf(d, d, dzsq));
        }
      }
    }
  }
  if (lists) note_moved3(moved, L.lslot);
}

// One application of T on the LDS state (xcur, L.lam) -> (xnext, L.lam): the
// constraint sweep (R = W^T V), the mean-field term, the xi_bar and lambda
// steps.  With `last`, dzsq gets this thread's share of ||z' - z||^2.
// Entered and left block-synchronised.
template <int NT, typename Args>
__device__ __forceinline__ void iterate3(const Args& A, const ProbDesc& P, const Lds3& L,
                                         const float* xcur, float* xnext, bool last,
                                         float& dzsq, Skin3& sk) {
  float z0 = 0.f, z1 = 0.f;
  sweep3_any<NT, kForward>(A, P, L, xcur, z0, z1, sk);
  mean_field3<NT>(P, L, A.nc, A.rho, xcur);
  __syncthreads();
  const bool lists = A.lists3 != 0;
  if (A.nc <= 16)
    xi_step3<NT, 4>(P, L, A.nc, A.rho, xcur, xnext, last, lists, sk.d, dzsq);
  else
    xi_step3<NT, 0>(P, L, A.nc, A.rho, xcur, xnext, last, lists, sk.d, dzsq);
  __syncthreads();
}

// The constant term c_xi = S xi + DS mean(xi) + N b + DN mean(b) per axis
// (mode form) into L.cxi, from the target staged in L.R and the boundary
// [n][2][3]; L.means is scratch.  Entered and left block-synchronised.
template <int NT>
__device__ __forceinline__ void form_cxi3(const ProbDesc& P, const Lds3& L, int nc,
                                          const float* bnd) {
  const int n = P.n, tid = threadIdx.x;
  const int nn = n * nc, S = 3 * nn, nc2 = nc * nc;
  // robot means of the target ([3][nc]) and of the boundary ([3][2])
  for (int t = tid; t < 3 * nc + 6; t += NT) {
    float s = 0.f;
    if (t < 3 * nc) {
      const int ax = t / nc, c = t - ax * nc;
      for (int i = 0; i < n; ++i) s += L.R[ax * nn + i * nc + c];
    } else {
      const int q = t - 3 * nc, ax = q >> 1, e = q & 1;
      for (int i = 0; i < n; ++i) s += bnd[i * 6 + e * 3 + ax];
    }
    L.means[t] = s / (float)n;
  }
  __syncthreads();
  const float* Np = L.fac + 4 * nc2;
  const float* DN = Np + 2 * nc;
  const float* bm = L.means + 3 * nc;
  for (int t = tid; t < S; t += NT) {
    const int ax = t / nn, rem = t - ax * nn, i = rem / nc, c = rem - i * nc;
    const float* Sp = L.fac + c * nc;
    const float* DS = L.fac + nc2 + c * nc;
    const float* y = L.R + ax * nn + i * nc;
    const float* ym = L.means + ax * nc;
    float out = 0.f;
    for (int q = 0; q < nc; ++q) out = fmaf(Sp[q], y[q], fmaf(DS[q], ym[q], out));
    for (int e = 0; e < 2; ++e) {
      out = fmaf(Np[c * 2 + e], bnd[i * 6 + e * 3 + ax], out);
      out = fmaf(DN[c * 2 + e], bm[ax * 2 + e], out);
    }
    L.cxi[t] = out;
  }
  __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT) void fwd3_kernel(FwdArgs A) {
  extern __shared__ float lds3[];
  const int b = A.order[blockIdx.x];
  const ProbDesc P = A.probs[b];
  const int n = P.n, M = P.M, nc = A.nc, tid = threadIdx.x;
  const int nn = n * nc, S = 3 * nn;
  const Lds3 L = carve3(lds3, nc, A.Tc, A.n_max, A.M_max, A.S_max);
  const float* bnd = A.boundary + (size_t)P.rob_off * 6;
  const size_t St = (size_t)A.S_total;

  Skin3 sk;
  setup3<NT>(A, P, L, A.obstacles);
  if (A.lists3) reset_lists3<NT>(L.refc, L.lslot, S);   // the first sweep builds every list
  if (A.save)   // the adjoint reads the obstacles from the workspace
    for (int t = tid; t < 5 * M; t += NT)
      A.ws_obs[(size_t)P.obs_off * 5 + t] = A.obstacles[(size_t)P.obs_off * 5 + t];
  for (int t = tid; t < S; t += NT) {
    L.xb[0][t] = A.xi0[P.coef_off + t];
    L.lam[t] = A.lam0[P.coef_off + t];
    L.R[t] = A.xi[P.coef_off + t];      // the target, until c_xi is formed
  }
  __syncthreads();
  form_cxi3<NT>(P, L, nc, bnd);
  if (A.save)
    for (int t = tid; t < S; t += NT) A.ws_cxi[P.coef_off + t] = L.cxi[t];

  // ping-pong by pointer swap (an index into L.xb would put L in scratch)
  float* xcur = L.xb[0];
  float* xnext = L.xb[1];
  float dzsq = 0.f;
  int ran = A.L;
  for (int l = 0; l < A.L; ++l) {
    if (A.save && (l % A.ckpt_every) == 0) {
      float* ck = A.ws_ckpt + (size_t)(l / A.ckpt_every) * 2 * St + P.coef_off;
      for (int t = tid; t < S; t += NT) {
        ck[t] = xcur[t];
        ck[St + t] = L.lam[t];
      }
    }
    // early exit: at a check iteration, the residual of xi_bar^l decides
    // whether this iteration is the problem's last (sums in a fixed order,
    // the same value in every thread)
    bool stop = false;
    if (A.check_every > 0 && (l % A.check_every) == 0) {
      float v[3] = {0.f, 0.f, 0.f};
      sweep3_any<NT, kFinal>(A, P, L, xcur, v[0], v[1], sk);
      block_sum3<NT>(v, L.red);
      stop = sqrtf(v[0] + v[1]) <= A.tol;
    }
    iterate3<NT>(A, P, L, xcur, xnext, stop || l == A.L - 1, dzsq, sk);
    float* tmp = xcur;
    xcur = xnext;
    xnext = tmp;
    if (stop) {
      ran = l + 1;
      break;
    }
  }

  // residual of the returned iterate, outputs, status
  float v[3] = {0.f, 0.f, 0.f};
  sweep3_any<NT, kFinal>(A, P, L, xcur, v[0], v[1], sk);
  float bad = 0.f;
  for (int t = tid; t < S; t += NT) {
    const float x = xcur[t], lm = L.lam[t];
    A.xi_out[P.coef_off + t] = x;
    A.lam_out[P.coef_off + t] = lm;
    if (A.save) {
      A.ws_final[P.coef_off + t] = x;
      A.ws_final[St + P.coef_off + t] = lm;
    }
    if (!isfinite(x) || !isfinite(lm)) bad = 1.f;
  }
  v[2] = bad;
  block_sum3<NT>(v, L.red);
  float dz[3] = {dzsq, 0.f, 0.f};
  block_sum3<NT>(dz, L.red);
  if (tid == 0) {
    A.ws_iters[b] = ran;
    float* res = A.residual + (size_t)b * 4;
    res[0] = sqrtf(v[0]);
    res[1] = sqrtf(v[1]);
    res[2] = ran > 0 ? sqrtf(dz[0]) : 0.f;
    res[3] = (v[2] > 0.f || !isfinite(v[0]) || !isfinite(v[1])) ? 1.f : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Plain 3D path (SF_PLAIN, SF_UNFUSED): the forward's stages as separate
// launches with the state in the workspace between them — prep (the state and
// c_xi), per iteration the constraint sweep (positions, rows, W^T V into R)
// and the update (mean field, xi_bar and lambda steps), then the final pass
// (residual of the returned iterate, outputs).  One workgroup per problem,
// problem b0 alone (b0 >= 0) or the batch (b0 < 0, grid = B).  Each stage
// runs the fused kernel's own code on the same LDS layout (the full sweep,
// without candidate lists, whose rows give the same sums), so the outputs
// carry the fused kernel's bits.
// ---------------------------------------------------------------------------
constexpr int kPlainPrep = 0, kPlainSweep = 1, kPlainUpdate = 2, kPlainFinal = 3;

template <int NT>
__global__ __launch_bounds__(NT) void plain3_kernel(FwdArgs A, PlainBufs pb, int b0, int stage,
                                                    int cur, int last) {
  extern __shared__ float lds3[];
  const int b = b0 >= 0 ? b0 : A.order[blockIdx.x];
  const ProbDesc P = A.probs[b];
  const int n = P.n, nc = A.nc, tid = threadIdx.x;
  const int S = 3 * n * nc;
  const Lds3 L = carve3(lds3, nc, A.Tc, A.n_max, A.M_max, A.S_max);
  const size_t off = P.coef_off;
  float* gcur = pb.xb[cur] + off;
  float* gnext = pb.xb[cur ^ 1] + off;
  float* glam = pb.lam + off;
  setup3<NT>(A, P, L, A.obstacles);
  if (stage == kPlainPrep) {
    for (int t = tid; t < S; t += NT) {
      gcur[t] = A.xi0[off + t];
      glam[t] = A.lam0[off + t];
      L.R[t] = A.xi[off + t];   // the target, until c_xi is formed
    }
    __syncthreads();
    form_cxi3<NT>(P, L, nc, A.boundary + (size_t)P.rob_off * 6);
    for (int t = tid; t < S; t += NT) pb.cxi[off + t] = L.cxi[t];
    if (tid == 0) pb.red[(size_t)b * 4 + 2] = 0.f;
  } else if (stage == kPlainSweep) {
    for (int t = tid; t < S; t += NT) L.xb[0][t] = gcur[t];
    __syncthreads();
    float z0 = 0.f, z1 = 0.f;
    Skin3 sk;   // the plain path runs without lists
    sweep3_any<NT, kForward>(A, P, L, L.xb[0], z0, z1, sk);
    for (int t = tid; t < S; t += NT) pb.R[off + t] = L.R[t];
  } else if (stage == kPlainUpdate) {
    for (int t = tid; t < S; t += NT) {
      L.xb[0][t] = gcur[t];
      L.lam[t] = glam[t];
      L.R[t] = pb.R[off + t];
      L.cxi[t] = pb.cxi[off + t];
    }
    __syncthreads();
    mean_field3<NT>(P, L, nc, A.rho, L.xb[0]);
    __syncthreads();
    float dzsq = 0.f;
    if (nc <= 16)
      xi_step3<NT, 4>(P, L, nc, A.rho, L.xb[0], L.xb[1], last != 0, false, 0.f, dzsq);
    else
      xi_step3<NT, 0>(P, L, nc, A.rho, L.xb[0], L.xb[1], last != 0, false, 0.f, dzsq);
    __syncthreads();
    for (int t = tid; t < S; t += NT) {
      gnext[t] = L.xb[1][t];
      glam[t] = L.lam[t];
    }
    if (last) {
      float dz[3] = {dzsq, 0.f, 0.f};
      block_sum3<NT>(dz, L.red);
      if (tid == 0) pb.red[(size_t)b * 4 + 2] = dz[0];
    }
  } else {
    for (int t = tid; t < S; t += NT) L.xb[0][t] = gcur[t];
    __syncthreads();
    float v[3] = {0.f, 0.f, 0.f};
    Skin3 sk;
    sweep3_any<NT, kFinal>(A, P, L, L.xb[0], v[0], v[1], sk);
    float bad = 0.f;
    for (int t = tid; t < S; t += NT) {
      const float x = gcur[t], lm = glam[t];
      A.xi_out[off + t] = x;
      A.lam_out[off + t] = lm;
      if (!isfinite(x) || !isfinite(lm)) bad = 1.f;
    }
    v[2] = bad;
    block_sum3<NT>(v, L.red);
    if (tid == 0) {
      A.ws_iters[b] = A.L;
      float* res = A.residual + (size_t)b * 4;
      res[0] = sqrtf(v[0]);
      res[1] = sqrtf(v[1]);
      res[2] = A.L > 0 ? sqrtf(pb.red[(size_t)b * 4 + 2]) : 0.f;
      res[3] = (v[2] > 0.f || !isfinite(v[0]) || !isfinite(v[1])) ? 1.f : 0.f;
    }
  }
}

// ---------------------------------------------------------------------------
// 3D adjoint: one workgroup per problem walks the checkpoint segments in
// reverse, recomputing a segment's iterates from its checkpoint with the
// forward's own iteration (same code, same time chunks, hence the same bits)
// into the global segment area, then per iteration l, for the cotangent g of
// xi_bar^{l+1} (plus 2 fw (xi_bar^{l+1} - xi_bar^l) with a fixed-point weight):
//   g_u      = S^T g          (also the cotangent of the target xi)
//   g_lambda += g_u,  g_R = -2 rho g_u - rho g_lambda' - 2 rho fw (lambda^{l+1} - lambda^l)
//   g_xi_bar = SH^T g - 2 fw (xi_bar^{l+1} - xi_bar^l) + W^T VJP(W g_R)
// S^T and SH^T in mode form: the transposed perpendicular block per robot plus
// the transposed parallel-minus-perpendicular block on the robot mean of g.
// The VJP of the constraint sums at X = W xi_bar^l: H_i = sum_j J_ij^T (G_i -
// G_j) + sum_m J_im^T G_i + box'(X_i) G_i (J the spheroid residual's Jacobian,
// I at Delta = 0, 0 on inactive rows), over time chunks of Tv steps.
// ---------------------------------------------------------------------------

// LDS of the adjoint beyond the forward's arrays (carve3_adj): G = W g_R over
// a VJP chunk [3][n][Tv], laid from xi_bar's ping-pong partner on (over lambda
// and c_xi, which a reverse step does not use), then the cotangents g (two,
// ping-pong), g_lambda, g_xi and g_R.
struct Lds3b {
  float *gA, *gB, *glam, *gxi, *gR, *G;
};

__host__ __device__ inline size_t g_area3(int n_max, int Tv, int S_max) {
  const size_t g = r4(3 * n_max * (Tv | 1)), tail = 3 * (size_t)r4(S_max);
  return g > tail ? g : tail;
}

__device__ __forceinline__ Lds3b carve3b(const Lds3& L, int n_max, int Tv, int S_max) {
  Lds3b B;
  float* p = L.xb[1];
  B.G = p; p += g_area3(n_max, Tv, S_max);
  B.gA = p; p += r4(S_max);
  B.gB = p; p += r4(S_max);
  B.glam = p; p += r4(S_max);
  B.gxi = p; p += r4(S_max);
  B.gR = p;
  return B;
}

// VJP rows of kRob robots against partner j (its position and G at u, u +
// plane, u + 2 plane): J^T (G_i - G_j) added to h.
template <int kRob>
__device__ __forceinline__ void pair_vjp3(const ProbDesc& P, const int (&ir)[kRob], int j, int u,
                                          int plane, const float* X, const float* G,
                                          const float (&px)[kRob], const float (&py)[kRob],
                                          const float (&pz)[kRob], const float (&gx)[kRob],
                                          const float (&gy)[kRob], const float (&gz)[kRob],
                                          float (&hx)[kRob], float (&hy)[kRob],
                                          float (&hz)[kRob]) {
  const float qx = X[u], qy = X[plane + u], qz = X[2 * plane + u];
  const float wx = G[u], wy = G[plane + u], wz = G[2 * plane + u];
#pragma unroll
  for (int r = 0; r < kRob; ++r)
    spheroid_vjp(px[r] - qx, py[r] - qy, pz[r] - qz, P.a, P.b, gx[r] - wx, gy[r] - wy,
                 gz[r] - wz, j != ir[r], hx[r], hy[r], hz[r]);
}

// VJP rows of kRob robots against obstacle entry o at time tau: J^T G_i.
template <int kRob>
__device__ __forceinline__ void obstacle_vjp3(const float* o, float tau, bool moving,
                                              const float (&px)[kRob], const float (&py)[kRob],
                                              const float (&pz)[kRob], const float (&gx)[kRob],
                                              const float (&gy)[kRob], const float (&gz)[kRob],
                                              float (&hx)[kRob], float (&hy)[kRob],
                                              float (&hz)[kRob]) {
  const float cx = moving ? fmaf(o[7], tau, o[2]) : o[2];
  const float cy = moving ? fmaf(o[8], tau, o[3]) : o[3];
  const float cz = moving ? fmaf(o[9], tau, o[4]) : o[4];
  const float ra = o[0], rb = o[1], oa = o[5], ob = o[6];
#pragma unroll
  for (int r = 0; r < kRob; ++r)
    spheroid_vjp(fmaf(px[r], ra, cx), fmaf(py[r], ra, cy), fmaf(pz[r], rb, cz), oa, ob, gx[r],
                 gy[r], gz[r], true, hx[r], hy[r], hz[r]);
}

// VJP sweep over the horizon in chunks of Tv steps: X = W xb (scaled), G = W
// gR, H = VJP (stored in L.V as [3][n][Tv]), R = W^T H (into L.R).  With
// `premapped` (one chunk, Tv >= T) the caller has mapped X and, for a list
// rebuild, written the window boxes already.
template <int NT, int kRob>
__device__ __forceinline__ void vjp3(const BwdArgs& A, const ProbDesc& P, const Lds3& L,
                                     const Lds3b& B, const float* xb, int Tv, bool rebuild,
                                     bool premapped, float d) {
  const int n = P.n, M = P.M, nc = A.nc, T = A.T, Tc = A.Tc, tid = phase_tid();
  const bool chunked = Tc < T;
  const float inv_a = 1.f / P.a, inv_b = 1.f / P.b;
  const float inv_Tm1 = 1.f / (float)(T - 1);
  const bool moving = A.ovel != nullptr;
  const int wave = wave_id3(tid);
  const bool lists = A.lists3 != 0;
  if (rebuild)
    for (int t = tid; t < 3 * n * nc; t += NT) L.refc[t] = xb[t];
  const int pw = (n + 31) >> 5, mw = mask_words3(n, M);
  for (int k0 = 0; k0 < T; k0 += Tv) {
    const int Tce = min(Tv, T - k0);
    const int Ts = Tce | 1;   // odd row stride of X, G and H
    if (chunked) {
      __syncthreads();
      for (int t = tid; t < Tce * nc; t += NT) L.W[t] = A.W[k0 * nc + t];
      __syncthreads();
    }
    const float* Wc = chunked ? L.W : L.W + k0 * nc;
    if (premapped) {
      // G = W g_R, then the list masks from the boxes
      map_tiles3_any(Wc, nc, 3 * n, Ts, Tce, B.gR, B.G, 1.f, 1.f, 0, nullptr, nullptr, 1, wave,
                     NT >> 6);
      if (rebuild) {
        if (tid < kSlots3) L.lslot[tid] = 0;   // every thread has read the flags
        list_masks3(P, L, k0, Tce, inv_Tm1, moving, d, wave, NT >> 6);
      }
      __syncthreads();
    } else {
      // X (scaled as in the forward) and G = W g_R, the forward's position tiles
      map_tiles3_any(Wc, nc, 3 * n, Ts, Tce, xb, L.X, inv_a, inv_b, 2 * n, B.gR, B.G, 2, wave,
                     NT >> 6);
      __syncthreads();
      if (rebuild) {
        if (k0 == 0 && tid < kSlots3) L.lslot[tid] = 0;   // every thread has read the flags
        build_lists3<NT>(P, L, k0, Tce, Ts, inv_Tm1, moving, d);
      }
    }
    const int plane = n * Ts;
    const int ngrp = (n + kRob - 1) / kRob;
    for (int t = tid; t < ngrp * Tce; t += NT) {
      const int g = t / Tce, kk = t - g * Tce;
      float px[kRob], py[kRob], pz[kRob], gx[kRob], gy[kRob], gz[kRob];
      float hx[kRob], hy[kRob], hz[kRob];
      int ir[kRob];
#pragma unroll
      for (int r = 0; r < kRob; ++r) {
        ir[r] = g * kRob + r;
        const int u = min(ir[r], n - 1) * Ts + kk;
        px[r] = L.X[u];
        py[r] = L.X[plane + u];
        pz[r] = L.X[2 * plane + u];
        gx[r] = B.G[u];
        gy[r] = B.G[plane + u];
        gz[r] = B.G[2 * plane + u];
        hx[r] = hy[r] = hz[r] = 0.f;
      }
      const float tau = (float)(k0 + kk) * inv_Tm1;
      if (lists) {
        // the union of the thread's robots' lists, in increasing index
        const unsigned* mk = L.mask + ((size_t)((k0 + kk) >> kWinShift3) * n + g * kRob) * mw;
        for (int q = 0; q < pw; ++q) {
          unsigned u = 0u;
#pragma unroll
          for (int r = 0; r < kRob; ++r)
            if (ir[r] < n) u |= mk[r * mw + q];
          while (u) {
            const int j = (__ffs(u) - 1) + 32 * q;
            u &= u - 1u;
            pair_vjp3<kRob>(P, ir, j, j * Ts + kk, plane, L.X, B.G, px, py, pz, gx, gy, gz,
                            hx, hy, hz);
          }
        }
        for (int q = 0; q < mw - pw; ++q) {
          unsigned u = 0u;
#pragma unroll
          for (int r = 0; r < kRob; ++r)
            if (ir[r] < n) u |= mk[r * mw + pw + q];
          while (u) {
            const int mo = (__ffs(u) - 1) + 32 * q;
            u &= u - 1u;
            obstacle_vjp3<kRob>(L.obs + mo * kObsFloats, tau, moving, px, py, pz, gx, gy, gz,
                                hx, hy, hz);
          }
        }
      } else {
        for (int j = 0; j < n; ++j)
          pair_vjp3<kRob>(P, ir, j, j * Ts + kk, plane, L.X, B.G, px, py, pz, gx, gy, gz, hx,
                          hy, hz);
        for (int mo = 0; mo < M; ++mo)
          obstacle_vjp3<kRob>(L.obs + mo * kObsFloats, tau, moving, px, py, pz, gx, gy, gz, hx,
                              hy, hz);
      }
#pragma unroll
      for (int r = 0; r < kRob; ++r) {
        if (ir[r] >= n) continue;
        const int u = ir[r] * Ts + kk;
        const float x = P.a * px[r], y = P.a * py[r], z = P.b * pz[r];
        float ox = hx[r], oy = hy[r], oz = hz[r];
        if (x > P.pmax[0] || x < P.pmin[0]) ox += gx[r];
        if (y > P.pmax[1] || y < P.pmin[1]) oy += gy[r];
        if (z > P.pmax[2] || z < P.pmin[2]) oz += gz[r];
        L.V[u] = ox;
        L.V[plane + u] = oy;
        L.V[2 * plane + u] = oz;
      }
    }
    __syncthreads();
    // R (+)= W^T H, the forward's W^T tiles
    wtv_tiles3<NT>(L.V, Ts, Wc, nc, Tce, 3 * n, L.R, k0 == 0);
    __syncthreads();
  }
}

// Robot means per (axis, coefficient) of the coefficient array g (into
// L.means[ax nc + q]), one axis per wave, lanes as in mean_field3.
// Axes w0, w0 + nw, ... of this wave.
__device__ __forceinline__ void robot_means3(const ProbDesc& P, const Lds3& L, int nc,
                                             const float* g, int w0, int nw) {
  const int n = P.n, nn = n * nc, lane = phase_tid() & 63;
  const int QW = nc <= 16 ? 16 : 32, Pw = 64 / QW;
  const int q = lane % QW, p = lane / QW, qq = min(q, nc - 1);
  for (int ax = w0; ax < 3; ax += nw) {
    const float* ga = g + ax * nn + qq;
    float s0 = 0.f, s1 = 0.f;
    int i = p;
    for (; i + Pw < n; i += 2 * Pw) {
      s0 += ga[i * nc];
      s1 += ga[(i + Pw) * nc];
    }
    if (i < n) s0 += ga[i * nc];
    float sm = s0 + s1;
    for (int o = QW; o < 64; o <<= 1) sm += __shfl_xor(sm, o, 64);
    if (p == 0 && q < nc) L.means[ax * nc + q] = sm / (float)n;
  }
}

// The transposed xi_bar step of the adjoint on MFMA 16x16x4 tiles, one wave
// per tile of 16 rows (row = axis * n + robot; tiles w0, w0 + nw, ...) and
// every coefficient column tile: for the cotangent g of xi_bar^{l+1} with robot means gm (L.means),
//   g_u[row][q] = sum_c (g[row][c] S[c][q]  + gm[axis][c] DS[c][q])
//   g_x[row][q] = sum_c (g[row][c] SH[c][q] + gm[axis][c] DSH[c][q])
// (A[m][k] = g[16 rt + m][4 s + k'], B[k][m] = S[4 s + k'][16 ct + m]; steps
// past nc add exact zeros).  The tile's lanes then form, for their own
// entries, the cotangent of R (through u = lambda - 2 rho R and lambda' =
// lambda - rho R), of lambda^l and of the target, and g_x into gn, with the
// fixed-point terms of weight fw (xi_bar and lambda of steps l, l + 1 at cur
// and nxt, lambda St floats after xi_bar).
template <int KS>
__device__ __forceinline__ void adj_step3(const ProbDesc& P, const Lds3& L, const Lds3b& B,
                                          int nc, float rho, float fw, const float* g, float* gn,
                                          const float* cur, const float* nxt, size_t St, int w0,
                                          int nw) {
  const int n = P.n, nc2 = nc * nc, rows = 3 * n;
  const int lane = phase_tid() & 63, m = lane & 15, kq = lane >> 4;
  const int nrt = (rows + 15) >> 4, nct = (nc + 15) >> 4;
  for (int rt = w0; rt < nrt; rt += nw) {
    const int rowA = min(rt * 16 + m, rows - 1), axA = rowA / n;
    floatx4 acc[2][2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[ct][0] = acc[ct][1] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int ksteps = KS > 0 ? KS : (nc + 3) >> 2;
#pragma unroll
    for (int g0 = 0; g0 < ksteps; g0 += (KS > 0 ? 4 : 1)) {
      constexpr int KG = KS == 0 ? 1 : (KS < 4 ? KS : 4);
      float ag[KG], agm[KG];
#pragma unroll
      for (int e = 0; e < KG; ++e) {
        const int q = 4 * (g0 + e) + kq, qq = min(q, nc - 1);
        const bool ok = g0 + e < ksteps && q < nc;
        const float gv = g[rowA * nc + qq], gmv = L.means[axA * nc + qq];
        ag[e] = ok ? gv : 0.f;
        agm[e] = ok ? gmv : 0.f;
      }
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        if (ct >= nct) continue;
        const int col = min(ct * 16 + m, nc - 1);
        float bs[KG], bds[KG], bsh[KG], bdsh[KG];
#pragma unroll
        for (int e = 0; e < KG; ++e) {
          const float* Sc = L.fac + min(4 * (g0 + e) + kq, nc - 1) * nc + col;
          bs[e] = Sc[0];
          bds[e] = Sc[nc2];
          bsh[e] = Sc[2 * nc2];
          bdsh[e] = Sc[3 * nc2];
        }
        reads_first();
#pragma unroll
        for (int e = 0; e < KG; ++e) {
          acc[ct][0] = mfma_16x16x4(ag[e], bs[e], acc[ct][0]);
          acc[ct][1] = mfma_16x16x4(ag[e], bsh[e], acc[ct][1]);
        }
#pragma unroll
        for (int e = 0; e < KG; ++e) {
          acc[ct][0] = mfma_16x16x4(agm[e], bds[e], acc[ct][0]);
          acc[ct][1] = mfma_16x16x4(agm[e], bdsh[e], acc[ct][1]);
        }
      }
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int c = ct * 16 + m;
      if (ct >= nct || c >= nc) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rt * 16 + 4 * kq + v;
        if (row >= rows) continue;
        const int e = row * nc + c;
        const float gu = acc[ct][0][v];
        const float dxi = fw != 0.f ? nxt[e] - cur[e] : 0.f;
        const float dla = fw != 0.f ? nxt[St + e] - cur[St + e] : 0.f;
        const float gl = B.glam[e];
        B.gR[e] = fmaf(-2.f * rho, gu, fmaf(-rho, gl, -2.f * rho * fw * dla));
        B.glam[e] = gl + gu;
        B.gxi[e] += gu;
        gn[e] = fmaf(-2.f * fw, dxi, acc[ct][1][v]);
      }
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void bwd3_kernel(BwdArgs A, int Tv) {
  extern __shared__ float lds3[];
  const int b = A.order[blockIdx.x];
  const ProbDesc P = A.probs[b];
  const int n = P.n, nc = A.nc, tid = threadIdx.x;
  const int nn = n * nc, S = 3 * nn;
  const Lds3 L = carve3_adj(lds3, nc, A.T, A.Tc, A.n_max, A.M_max, A.S_max, A.lists3 != 0);
  const Lds3b B = carve3b(L, A.n_max, Tv, A.S_max);
  const float rho = A.rho, fw = A.fp_weight;
  const size_t St = (size_t)A.S_total;
  const int rpt = robots_per_thread(n);
  const bool lists = A.lists3 != 0;
  Skin3 sk;
  const int T = A.T, NW = NT >> 6, wave = wave_id3(tid);
  const bool whole = Tv >= T;   // one VJP chunk

  setup3<NT>(A, P, L, A.obs);
  if (lists) reset_lists3<NT>(L.refc, L.lslot, S);
  for (int t = tid; t < S; t += NT) {
    B.gA[t] = A.g_xi_out ? A.g_xi_out[P.coef_off + t] : 0.f;
    B.glam[t] = A.g_lam_out ? A.g_lam_out[P.coef_off + t] : 0.f;
    B.gxi[t] = 0.f;
  }
  __syncthreads();
  float* gx = B.gA;
  float* gn = B.gB;

  // cotangents of ||r_1|| and ||r_2|| of the returned iterate
  const float gr1 = A.g_res ? A.g_res[(size_t)b * 4] : 0.f;
  const float gr2 = A.g_res ? A.g_res[(size_t)b * 4 + 1] : 0.f;
  if (gr1 != 0.f || gr2 != 0.f) {
    float* xf = L.xb[0];
    for (int t = tid; t < S; t += NT) xf[t] = A.fin[P.coef_off + t];
    __syncthreads();
    float v[3] = {0.f, 0.f, 0.f};
    sweep3_any<NT, kFinal>(A, P, L, xf, v[0], v[1], sk);
    block_sum3<NT>(v, L.red);
    const float c1 = v[0] > 0.f ? gr1 / sqrtf(v[0]) : 0.f;
    const float c2 = v[1] > 0.f ? gr2 / sqrtf(v[1]) : 0.f;
    float d0 = 0.f, d1 = 0.f;
    sweep3_any<NT, kResGrad>(A, P, L, xf, d0, d1, sk, c1, c2);
    for (int t = tid; t < S; t += NT) gx[t] += L.R[t];
    __syncthreads();
  }

  const int L_ = A.iters ? A.iters[b] : A.L, k = A.ckpt_every;   // each problem's own chain
  const int nseg = (L_ + k - 1) / k;
  float dz = 0.f;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int l0 = seg * k;
    const int l1 = min(L_, l0 + k);
    const float* ck = A.ckpt + (size_t)seg * 2 * St + P.coef_off;
    if (l1 - 1 > l0) {
      // recompute iterates l0+1 .. l1-1 into the segment area (slot l - l0)
      float* xc = L.xb[0];
      float* xq = L.xb[1];
      bool moved = false;
      for (int t = tid; t < S; t += NT) {
        xc[t] = ck[t];
        L.lam[t] = ck[St + t];
        L.cxi[t] = A.cxi[P.coef_off + t];
        if (lists) moved |= coef_moved3(xc, L.refc, t, nn, sk.d * P.a, sk.d * P.b);
      }
      if (lists) note_moved3(moved, L.lslot);
      __syncthreads();
      for (int l = l0; l < l1 - 1; ++l) {
        iterate3<NT>(A, P, L, xc, xq, false, dz, sk);
        float* tmp = xc;
        xc = xq;
        xq = tmp;
        float* dst = A.seg + (size_t)(l + 1 - l0) * 2 * St + P.coef_off;
        for (int t = tid; t < S; t += NT) {
          dst[t] = xc[t];
          dst[St + t] = L.lam[t];
        }
      }
      __syncthreads();
    }
    for (int l = l1 - 1; l >= l0; --l) {
      const float* cur = l == l0 ? ck : A.seg + (size_t)(l - l0) * 2 * St + P.coef_off;
      const float* nxt = (l + 1 < l1) ? A.seg + (size_t)(l + 1 - l0) * 2 * St + P.coef_off
                         : (l1 == L_) ? A.fin + P.coef_off
                                      : A.ckpt + (size_t)(seg + 1) * 2 * St + P.coef_off;
      float* xl = L.xb[0];
      // the cotangent entering the step: g + 2 fw (xi_bar^{l+1} - xi_bar^l)
      bool moved = false;
      for (int t = tid; t < S; t += NT) {
        xl[t] = cur[t];
        if (fw != 0.f) gx[t] = fmaf(2.f * fw, nxt[t] - cur[t], gx[t]);
        if (lists) moved |= coef_moved3(xl, L.refc, t, nn, sk.d * P.a, sk.d * P.b);
      }
      if (lists) note_moved3(moved, L.lslot);
      __syncthreads();
      const bool rebuild = lists && lists_moved3(L.lslot, NW);
      if (lists) sk.pass(rebuild);
      const int nrt = (3 * n + 15) >> 4;
      if (whole) {
        // the robot means of g (waves 0-2) beside the positions X = W xi_bar^l
        // (the other waves), then the g step beside the window boxes of a
        // list rebuild
        if (wave < 3)
          robot_means3(P, L, nc, gx, wave, 3);
        else
          map_tiles3_any(L.W, nc, 3 * n, T | 1, T, xl, L.X, 1.f / P.a, 1.f / P.b, 2 * n, nullptr,
                         nullptr, 1, wave - 3, NW - 3);
        __syncthreads();
        const int wa = rebuild ? min(nrt, NW - 1) : NW;
        if (wave < wa) {
          if (nc <= 16)
            adj_step3<4>(P, L, B, nc, rho, fw, gx, gn, cur, nxt, St, wave, wa);
          else
            adj_step3<0>(P, L, B, nc, rho, fw, gx, gn, cur, nxt, St, wave, wa);
        } else {
          list_boxes3(P, L, T, T | 1, tid - 64 * wa, NT - 64 * wa);
        }
      } else {
        robot_means3(P, L, nc, gx, wave, NW);
        __syncthreads();
        if (nc <= 16)
          adj_step3<4>(P, L, B, nc, rho, fw, gx, gn, cur, nxt, St, wave, NW);
        else
          adj_step3<0>(P, L, B, nc, rho, fw, gx, gn, cur, nxt, St, wave, NW);
      }
      __syncthreads();
      if (lists)
        vjp3<NT, kListRob3>(A, P, L, B, xl, Tv, rebuild, whole, sk.d);
      else if (rpt == 4)
        vjp3<NT, 4>(A, P, L, B, xl, Tv, false, whole, 0.f);
      else if (rpt == 2)
        vjp3<NT, 2>(A, P, L, B, xl, Tv, false, whole, 0.f);
      else
        vjp3<NT, 1>(A, P, L, B, xl, Tv, false, whole, 0.f);
      for (int t = tid; t < S; t += NT) gn[t] += L.R[t];
      __syncthreads();
      float* tmp = gx;
      gx = gn;
      gn = tmp;
    }
  }
  for (int t = tid; t < S; t += NT) {
    if (A.g_xi0) A.g_xi0[P.coef_off + t] = gx[t];
    if (A.g_lam0) A.g_lam0[P.coef_off + t] = B.glam[t];
    if (A.g_xi) A.g_xi[P.coef_off + t] = B.gxi[t];
  }
}

}  // namespace

int list_window3() { return kWin3; }

size_t fwd3_lds_bytes(int nc, int T, int Tc, int n_max, int M_max, int S_max, bool lists) {
  return lds3_floats(nc, T, Tc, n_max, M_max, S_max, lists) * sizeof(float);
}

size_t bwd3_lds_bytes(int nc, int T, int Tc, int Tv, int n_max, int M_max, int S_max,
                      bool lists) {
  // the forward's layout up to its last three arrays, G over them, five more
  return (lds3_floats(nc, T, Tc, n_max, M_max, S_max, lists) - 3 * (size_t)r4(S_max) +
          g_area3(n_max, Tv, S_max) + 5 * (size_t)r4(S_max)) * sizeof(float);
}

hipError_t prepare_kernels3(size_t lds) {
  const void* fns[] = {reinterpret_cast<const void*>(&fwd3_kernel<256>),
                       reinterpret_cast<const void*>(&fwd3_kernel<512>),
                       reinterpret_cast<const void*>(&fwd3_kernel<1024>),
                       reinterpret_cast<const void*>(&bwd3_kernel<256>),
                       reinterpret_cast<const void*>(&bwd3_kernel<512>),
                       reinterpret_cast<const void*>(&bwd3_kernel<1024>),
                       reinterpret_cast<const void*>(&plain3_kernel<kPlainThreads3>)};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fwd3(const FwdArgs& a, int threads, size_t lds, hipStream_t s) {
  dim3 grid(a.B);
  switch (threads) {
    case 256:
      hipLaunchKernelGGL(fwd3_kernel<256>, grid, dim3(256), lds, s, a);
      break;
    case 512:
      hipLaunchKernelGGL(fwd3_kernel<512>, grid, dim3(512), lds, s, a);
      break;
    case 1024:
      hipLaunchKernelGGL(fwd3_kernel<1024>, grid, dim3(1024), lds, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_plain3(const FwdArgs& a, const PlainBufs& pb, int b, size_t lds,
                         hipStream_t s) {
  FwdArgs ap = a;
  ap.lists3 = 0;   // the full sweep (same sums as the lists)
  const dim3 grid(b >= 0 ? 1 : a.B), block(kPlainThreads3);
  hipLaunchKernelGGL(plain3_kernel<kPlainThreads3>, grid, block, lds, s, ap, pb, b, kPlainPrep,
                     0, 0);
  int cur = 0;
  for (int l = 0; l < a.L; ++l) {
    hipLaunchKernelGGL(plain3_kernel<kPlainThreads3>, grid, block, lds, s, ap, pb, b,
                       kPlainSweep, cur, 0);
    hipLaunchKernelGGL(plain3_kernel<kPlainThreads3>, grid, block, lds, s, ap, pb, b,
                       kPlainUpdate, cur, (int)(l == a.L - 1));
    cur ^= 1;
  }
  hipLaunchKernelGGL(plain3_kernel<kPlainThreads3>, grid, block, lds, s, ap, pb, b, kPlainFinal,
                     cur, 0);
  return hipGetLastError();
}

hipError_t launch_bwd3(const BwdArgs& a, int threads, size_t lds, int Tv, hipStream_t s) {
  dim3 grid(a.B);
  switch (threads) {
    case 256:
      hipLaunchKernelGGL(bwd3_kernel<256>, grid, dim3(256), lds, s, a, Tv);
      break;
    case 512:
      hipLaunchKernelGGL(bwd3_kernel<512>, grid, dim3(512), lds, s, a, Tv);
      break;
    case 1024:
      hipLaunchKernelGGL(bwd3_kernel<1024>, grid, dim3(1024), lds, s, a, Tv);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sf
