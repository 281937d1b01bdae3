// 3D (spheroid) SF forward: one workgroup per problem, the problem's state in
// LDS for all L iterations.
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
//   V = F^T r_1 + G^T r_2 per (robot, step), every pair visited    [3][n][Tc]
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
constexpr int kObsFloats = 12;     // obstacle table entry (10 used, see the set-up)

__host__ __device__ inline int r4(int x) { return (x + 3) & ~3; }

typedef float floatx4 __attribute__((ext_vector_type(4)));

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

// Robots per thread in the constraint stage: more robots share each LDS read,
// fewer threads have work; four from 24 robots, two from 8.
__device__ __forceinline__ int robots_per_thread(int n) { return n >= 24 ? 4 : (n >= 8 ? 2 : 1); }

struct Lds3 {
  float *W, *fac, *xb[2], *lam, *cxi, *R, *means, *obs, *X, *V, *red;
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
  L.X = p; p += 3 * n_max * Tc;
  L.V = p;
  return L;
}

// One pass over the horizon at xi_bar = xb: positions X, constraint sums V
// and (unless FINAL) R = W^T V; with FINAL the residual sums instead.
template <int NT, bool FINAL, int kRob>
__device__ __forceinline__ void sweep3(const FwdArgs& A, const ProbDesc& P, const Lds3& L,
                                       const float* xb, float& r1sq, float& r2sq) {
  const int n = P.n, M = P.M, nc = A.nc, T = A.T, Tc = A.Tc, tid = threadIdx.x;
  const bool chunked = Tc < T;
  const float inv_a = 1.f / P.a, inv_b = 1.f / P.b;
  const float inv_Tm1 = 1.f / (float)(T - 1);
  const bool moving = A.ovel != nullptr;
  for (int k0 = 0; k0 < T; k0 += Tc) {
    const int Tce = min(Tc, T - k0);
    if (chunked) {
      for (int t = tid; t < Tce * nc; t += NT) L.W[t] = A.W[k0 * nc + t];
      __syncthreads();
    }
    const float* Wc = chunked ? L.W : L.W + k0 * nc;
    // positions X[row][kk] = sum_c W[kk][c] xb[row][c] on MFMA 16x16x4 tiles
    // of 16 steps x 16 rows (row = axis * n + robot), the wave's tiles dealt
    // round-robin.  A lane supplies A[m][k] = W[16 wt + m][4 s + k'] and
    // B[k][m] = xb[16 ct + m][4 s + k'] (m = lane % 16, k' = lane / 16) and
    // holds X[16 ct + m][16 wt + 4 k' + v]; coefficients past nc enter as 0.
    {
      const int lane = tid & 63, wave = tid >> 6, m = lane & 15, kq = lane >> 4;
      const int nwt = (Tce + 15) >> 4, nct = (3 * n + 15) >> 4, ks = (nc + 3) >> 2;
      for (int q = wave; q < nwt * nct; q += NT >> 6) {
        const int wt = q / nct, ct = q - wt * nct;
        const int stepA = min(wt * 16 + m, Tce - 1), colB = min(ct * 16 + m, 3 * n - 1);
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int s4 = 0; s4 < ks; ++s4) {
          const int c = 4 * s4 + kq, cc = min(c, nc - 1);
          const float a = c < nc ? Wc[stepA * nc + cc] : 0.f;
          acc = mfma_16x16x4(a, xb[colB * nc + cc], acc);
        }
        // stored scaled by the robot's semi-axes: x/a, y/a, z/b
        const int col = ct * 16 + m;
        const float sc = col < 2 * n ? inv_a : inv_b;
        if (col < 3 * n) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int step = wt * 16 + 4 * kq + v;
            if (step < Tce) L.X[col * Tce + step] = acc[v] * sc;
          }
        }
      }
    }
    __syncthreads();
    // constraint rows (every robot pair, every obstacle, the box).  A thread
    // takes kRob robots at one step, so each partner position and obstacle
    // read from LDS serves kRob rows; every row still sums its terms in the
    // same order (partners j = 0..n-1, then obstacles).  kRob depends on the
    // problem's robot count only (robots_per_thread), not on the block size.
    const int plane = n * Tce;
    const int ngrp = (n + kRob - 1) / kRob;
    for (int t = tid; t < ngrp * Tce; t += NT) {
      const int g = t / Tce, kk = t - g * Tce;
      float px[kRob], py[kRob], pz[kRob], vx[kRob], vy[kRob], vz[kRob], sq[kRob];
      int ir[kRob];
#pragma unroll
      for (int r = 0; r < kRob; ++r) {
        ir[r] = g * kRob + r;
        const int u = min(ir[r], n - 1) * Tce + kk;
        px[r] = L.X[u];
        py[r] = L.X[plane + u];
        pz[r] = L.X[2 * plane + u];
        vx[r] = vy[r] = vz[r] = sq[r] = 0.f;
      }
      // partners in groups of four, every read of a group issued first
      int j0 = 0;
      for (; j0 + 4 <= n; j0 += 4) {
        float qx[4], qy[4], qz[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int u = (j0 + e) * Tce + kk;
          qx[e] = L.X[u];
          qy[e] = L.X[plane + u];
          qz[e] = L.X[2 * plane + u];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = j0 + e;
#pragma unroll
          for (int r = 0; r < kRob; ++r) {
            float s1 = 0.f;
            spheroid_residual<FINAL>(px[r] - qx[e], py[r] - qy[e], pz[r] - qz[e], P.a, P.b,
                                     ir[r] < j ? -P.b : P.b, j != ir[r], vx[r], vy[r], vz[r],
                                     s1);
            if (FINAL) sq[r] += j > ir[r] ? s1 : 0.f;   // each unordered pair once
          }
        }
      }
      for (int j = j0; j < n; ++j) {
        const int u = j * Tce + kk;
        const float qx = L.X[u], qy = L.X[plane + u], qz = L.X[2 * plane + u];
#pragma unroll
        for (int r = 0; r < kRob; ++r) {
          float s1 = 0.f;
          spheroid_residual<FINAL>(px[r] - qx, py[r] - qy, pz[r] - qz, P.a, P.b,
                                   ir[r] < j ? -P.b : P.b, j != ir[r], vx[r], vy[r], vz[r], s1);
          if (FINAL) sq[r] += j > ir[r] ? s1 : 0.f;
        }
      }
      // obstacle offsets in the obstacle's scaling: (a x' - c - d tau) / a_o
      // (x' the stored x / a), i.e. x' (a / a_o) - c / a_o - (d / a_o) tau
      const float tau = (float)(k0 + kk) * inv_Tm1;
      for (int m = 0; m < M; ++m) {
        const float* o = L.obs + m * kObsFloats;
        const float cx = moving ? fmaf(o[7], tau, o[2]) : o[2];
        const float cy = moving ? fmaf(o[8], tau, o[3]) : o[3];
        const float cz = moving ? fmaf(o[9], tau, o[4]) : o[4];
        const float ra = o[0], rb = o[1], oa = o[5], ob = o[6];
#pragma unroll
        for (int r = 0; r < kRob; ++r)
          spheroid_residual<FINAL>(fmaf(px[r], ra, cx), fmaf(py[r], ra, cy), fmaf(pz[r], rb, cz),
                                   oa, ob, -ob, true, vx[r], vy[r], vz[r], sq[r]);
      }
#pragma unroll
      for (int r = 0; r < kRob; ++r) {
        if (ir[r] >= n) continue;
        const int u = ir[r] * Tce + kk;
        const float x = P.a * px[r], y = P.a * py[r], z = P.b * pz[r];
        const float hx = fmaxf(x - P.pmax[0], 0.f), lx = fmaxf(P.pmin[0] - x, 0.f);
        const float hy = fmaxf(y - P.pmax[1], 0.f), ly = fmaxf(P.pmin[1] - y, 0.f);
        const float hz = fmaxf(z - P.pmax[2], 0.f), lz = fmaxf(P.pmin[2] - z, 0.f);
        if (FINAL) {
          r1sq += sq[r];
          r2sq += hx * hx + lx * lx + hy * hy + ly * ly + hz * hz + lz * lz;
        } else {
          L.V[u] = vx[r] + (hx - lx);
          L.V[plane + u] = vy[r] + (hy - ly);
          L.V[2 * plane + u] = vz[r] + (hz - lz);
        }
      }
    }
    __syncthreads();
    if (!FINAL) {
      // R (+)= W^T V over this chunk's steps on MFMA 16x16x4 tiles of 16 rows
      // x 16 coefficients: A[m][k] = V[16 rt + m][4 s + k'], B[k][m] =
      // W[4 s + k'][16 ct + m]; steps past Tce enter as 0.  Two accumulators
      // (even and odd s) added at the end.
      const int lane = tid & 63, wave = tid >> 6, m = lane & 15, kq = lane >> 4;
      const int nrt = (3 * n + 15) >> 4, nct = (nc + 15) >> 4, nk = (Tce + 3) >> 2;
      for (int q = wave; q < nrt * nct; q += NT >> 6) {
        const int rt = q / nct, ct = q - rt * nct;
        const int rowA = min(rt * 16 + m, 3 * n - 1), cB = min(ct * 16 + m, nc - 1);
        const float* vrow = L.V + rowA * Tce;
        floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        int s4 = 0;
        for (; s4 + 2 <= nk; s4 += 2) {
          const int k0s = 4 * s4 + kq, k1s = k0s + 4;
          const float a0 = k0s < Tce ? vrow[min(k0s, Tce - 1)] : 0.f;
          const float a1 = k1s < Tce ? vrow[min(k1s, Tce - 1)] : 0.f;
          const float b0 = Wc[min(k0s, Tce - 1) * nc + cB];
          const float b1 = Wc[min(k1s, Tce - 1) * nc + cB];
          acc0 = mfma_16x16x4(a0, b0, acc0);
          acc1 = mfma_16x16x4(a1, b1, acc1);
        }
        if (s4 < nk) {
          const int k0s = 4 * s4 + kq;
          const float a0 = k0s < Tce ? vrow[min(k0s, Tce - 1)] : 0.f;
          acc0 = mfma_16x16x4(a0, Wc[min(k0s, Tce - 1) * nc + cB], acc0);
        }
        const int c = ct * 16 + m;
        if (c < nc) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = rt * 16 + 4 * kq + v;
            if (row < 3 * n) {
              const float sum = acc0[v] + acc1[v];
              L.R[row * nc + c] = k0 == 0 ? sum : L.R[row * nc + c] + sum;
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void fwd3_kernel(FwdArgs A) {
  extern __shared__ float lds3[];
  const int b = A.order[blockIdx.x];
  const ProbDesc P = A.probs[b];
  const int n = P.n, M = P.M, nc = A.nc, T = A.T, Tc = A.Tc, tid = threadIdx.x;
  const int nn = n * nc, S = 3 * nn, nc2 = nc * nc;
  const Lds3 L = carve3(lds3, nc, Tc, A.n_max, A.M_max, A.S_max);
  const float rho = A.rho;
  const float* bnd = A.boundary + (size_t)P.rob_off * 6;
  const bool chunked = Tc < T;
  const int rpt = robots_per_thread(n);

  // --- set-up: factor block, W (whole table when unchunked), obstacles, state
  const float* facg = A.fac + (size_t)P.fac * fac_stride(nc);
  for (int t = tid; t < fac_stride(nc); t += NT) L.fac[t] = facg[t];
  if (!chunked)
    for (int t = tid; t < T * nc; t += NT) L.W[t] = A.W[t];
  for (int m = tid; m < M; m += NT) {
    const float* o = A.obstacles + (size_t)(P.obs_off + m) * 5;
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
  for (int t = tid; t < S; t += NT) {
    L.xb[0][t] = A.xi0[P.coef_off + t];
    L.lam[t] = A.lam0[P.coef_off + t];
    L.R[t] = A.xi[P.coef_off + t];      // the target, until c_xi is formed
  }
  __syncthreads();
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
  {
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
  }
  __syncthreads();

  // ping-pong by pointer swap (an index into L.xb would put L in scratch)
  float* xcur = L.xb[0];
  float* xnext = L.xb[1];
  float dzsq = 0.f;
  for (int l = 0; l < A.L; ++l) {
    const bool last = l == A.L - 1;
    float z0 = 0.f, z1 = 0.f;
    if (rpt == 4)
      sweep3<NT, false, 4>(A, P, L, xcur, z0, z1);
    else if (rpt == 2)
      sweep3<NT, false, 2>(A, P, L, xcur, z0, z1);
    else
      sweep3<NT, false, 1>(A, P, L, xcur, z0, z1);
    // lambda step and u = lambda - 2 rho R (u replaces R)
    for (int t = tid; t < S; t += NT) {
      const float r = L.R[t], lm = L.lam[t];
      L.lam[t] = fmaf(-rho, r, lm);
      L.R[t] = fmaf(-2.f * rho, r, lm);
      if (last) dzsq = fmaf(rho * r, rho * r, dzsq);
    }
    __syncthreads();
    // robot means of u and xb: means[0..3nc) and means[3nc..6nc)
    for (int t = tid; t < 6 * nc; t += NT) {
      const int which = t / (3 * nc), q = t - which * 3 * nc, ax = q / nc, c = q - ax * nc;
      const float* src = (which ? xcur : L.R) + ax * nn + c;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;   // four chains in flight
      int i = 0;
      for (; i + 4 <= n; i += 4) {
        s0 += src[i * nc];
        s1 += src[(i + 1) * nc];
        s2 += src[(i + 2) * nc];
        s3 += src[(i + 3) * nc];
      }
      for (; i < n; ++i) s0 += src[i * nc];
      L.means[t] = ((s0 + s1) + (s2 + s3)) / (float)n;
    }
    __syncthreads();
    // xi_bar step
    {
      const float* xb = xcur;
      float* xn = xnext;
      for (int t = tid; t < S; t += NT) {
        const int ax = t / nn, rem = t - ax * nn, i = rem / nc, c = rem - i * nc;
        const float* Sp = L.fac + c * nc;
        const float* DS = Sp + nc2;
        const float* SH = Sp + 2 * nc2;
        const float* DSH = Sp + 3 * nc2;
        const float* u = L.R + ax * nn + i * nc;
        const float* x = xb + ax * nn + i * nc;
        const float* um = L.means + ax * nc;
        const float* xm = L.means + 3 * nc + ax * nc;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;   // one chain per block
        for (int q = 0; q < nc; ++q) {
          a0 = fmaf(Sp[q], u[q], a0);
          a1 = fmaf(DS[q], um[q], a1);
          a2 = fmaf(SH[q], x[q], a2);
          a3 = fmaf(DSH[q], xm[q], a3);
        }
        const float v = L.cxi[t] + ((a0 + a1) + (a2 + a3));
        xn[t] = v;
        if (last) {
          const float d = v - xb[t];
          dzsq = fmaf(d, d, dzsq);
        }
      }
    }
    __syncthreads();
    float* tmp = xcur;
    xcur = xnext;
    xnext = tmp;
  }

  // residual of the returned iterate, outputs, status
  float v[3] = {0.f, 0.f, 0.f};
  if (rpt == 4)
    sweep3<NT, true, 4>(A, P, L, xcur, v[0], v[1]);
  else if (rpt == 2)
    sweep3<NT, true, 2>(A, P, L, xcur, v[0], v[1]);
  else
    sweep3<NT, true, 1>(A, P, L, xcur, v[0], v[1]);
  float bad = 0.f;
  for (int t = tid; t < S; t += NT) {
    const float x = xcur[t], lm = L.lam[t];
    A.xi_out[P.coef_off + t] = x;
    A.lam_out[P.coef_off + t] = lm;
    if (!isfinite(x) || !isfinite(lm)) bad = 1.f;
  }
  v[2] = bad;
  block_sum3<NT>(v, L.red);
  float dz[3] = {dzsq, 0.f, 0.f};
  block_sum3<NT>(dz, L.red);
  if (tid == 0) {
    A.ws_iters[b] = A.L;
    float* res = A.residual + (size_t)b * 4;
    res[0] = sqrtf(v[0]);
    res[1] = sqrtf(v[1]);
    res[2] = A.L > 0 ? sqrtf(dz[0]) : 0.f;
    res[3] = (v[2] > 0.f || !isfinite(v[0]) || !isfinite(v[1])) ? 1.f : 0.f;
  }
}

}  // namespace

size_t fwd3_lds_bytes(int nc, int T, int Tc, int n_max, int M_max, int S_max) {
  (void)T;
  const size_t f = (size_t)r4(Tc * nc) + r4(fac_stride(nc)) + 5 * (size_t)r4(S_max) +
                   6 * kMaxCoef + 8 + (size_t)kObsFloats * M_max + kRed3 +
                   6 * (size_t)n_max * Tc;
  return f * sizeof(float);
}

hipError_t prepare_kernels3(size_t lds) {
  const void* fns[] = {reinterpret_cast<const void*>(&fwd3_kernel<256>),
                       reinterpret_cast<const void*>(&fwd3_kernel<512>),
                       reinterpret_cast<const void*>(&fwd3_kernel<1024>)};
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

}  // namespace sf
