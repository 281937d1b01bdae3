// Internal declarations shared by the host runtime (sf_host.cpp) and the HIP
// kernels (sf_kernels.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sf {

constexpr int kDim = 2;
constexpr int kMaxCoef = 32;

// Per-problem descriptor, resident in the workspace.
struct ProbDesc {
  int32_t n;         // robots
  int32_t M;         // obstacles
  int32_t coef_off;  // first float of this problem in coefficient arrays
  int32_t rob_off;   // first robot (boundary rows)
  int32_t obs_off;   // first obstacle (obstacle rows)
  int32_t fac;       // index of this problem's factor block
  int32_t pos_off;   // first (robot, step) slot in the plain-path position buffers
  int32_t pad0;
  float a;           // minimum robot centre distance (horizontal in 3D)
  float pmin[3];     // box per axis (the planar SF reads the first two)
  float pmax[3];
  float b;           // 3D: minimum centre distance along z
};
static_assert(sizeof(ProbDesc) == 64, "descriptor layout");

// Factor block of one (n, M) class, float32, each matrix row-major [n_coef][.]:
//   S_perp, DS = S_par - S_perp, SH_perp, DSH = SH_par - SH_perp   [nc][nc]
//   N_perp, DN = N_par - N_perp                                    [nc][2]
__host__ __device__ inline int fac_stride(int nc) { return 4 * nc * nc + 4 * nc; }

struct FwdArgs {
  const ProbDesc* probs;
  const int32_t* order;   // launch slot -> problem (longest first)
  const float* W;         // [T][nc]
  const float* fac;       // factor blocks
  const float* xi;
  const float* xi0;
  const float* lam0;
  const float* boundary;
  const float* obstacles;
  const float* ovel;      // obstacle displacements [sum M][n_dim] over the horizon, or null (static)
  float* xi_out;
  float* lam_out;
  float* residual;        // [B][4]
  float* ws_cxi;          // saved constant term, coefficient layout
  float* ws_obs;          // saved obstacles
  float* ws_ckpt;         // [n_ckpt][2][S_total]
  float* ws_final;        // [2][S_total]
  int32_t* ws_iters;      // [B] iterations each problem ran
  unsigned* gmask;        // chunked horizons: [B][chunk_list_bytes / 4] candidate lists
  int64_t S_total;        // floats in one coefficient array
  int32_t B;
  int32_t nc;
  int32_t T;
  int32_t Tc;             // time-chunk length held in LDS
  int32_t n_max, M_max, S_max;
  int32_t L;
  int32_t ckpt_every;
  int32_t save;
  int32_t check_every;    // early exit: test the residual every this many iterations (0 = off)
  int32_t lists3;         // 3D: candidate lists on
  float tol;              // early exit threshold on sqrt(||r_1||^2 + ||r_2||^2)
  float rho;
};

struct BwdArgs {
  const ProbDesc* probs;
  const int32_t* order;
  const float* W;
  const float* fac;
  const float* cxi;       // saved constant term
  const float* obs;       // saved obstacles
  const float* ovel;      // obstacle displacements, or null (static)
  const float* ckpt;      // [n_ckpt][2][S_total]
  const float* fin;       // [2][S_total]
  float* seg;             // recompute scratch [ckpt_every][2][S_total]
  const float* g_xi_out;  // nullable
  const float* g_lam_out; // nullable
  const float* g_res;     // nullable [B][4]
  float* g_xi;            // nullable
  float* g_xi0;           // nullable
  float* g_lam0;          // nullable
  const int32_t* iters;   // nullable [B]: iterations each problem ran (early exit)
  unsigned* gmask;        // chunked horizons: [B][chunk_list_bytes / 4] candidate lists
  int64_t S_total;
  int32_t B;
  int32_t nc;
  int32_t T;
  int32_t Tc;
  int32_t n_max, M_max, S_max;
  int32_t L;
  int32_t ckpt_every;
  int32_t lists3;         // 3D: candidate lists on
  float rho;
  float fp_weight;
};

// Bytes per problem of the global copy of the candidate lists that a chunked
// horizon (Tc < T) keeps between passes; 0 when the horizon is LDS-resident.
size_t chunk_list_bytes(int T, int Tc, int n_max, int M_max);

// Dynamic LDS bytes of the fused kernels for given batch maxima.
size_t fwd_lds_bytes(int nc, int T, int Tc, int n_max, int M_max, int S_max, int threads);
size_t bwd_lds_bytes(int nc, int T, int Tc, int n_max, int M_max, int S_max, int threads);

hipError_t launch_fwd_fused(const FwdArgs& a, int threads, size_t lds, hipStream_t s);
hipError_t launch_bwd_fused(const BwdArgs& a, int threads, size_t lds, hipStream_t s);

// Plain path: one problem, one iteration per launch group.
struct PlainBufs {
  float* X;      // [sum n][T][2] positions
  float* V;      // [sum n][T][2] constraint sums
  float* R;      // coefficient layout: lambda of odd iterations (ping-pong with lam)
  float* xb[2];  // ping-pong xi_bar, coefficient layout
  float* lam;    // coefficient layout
  float* cxi;    // coefficient layout
  float* red;    // [B][4] residual partials
  float* part;   // per-problem per-window partial sums [windows][coefficient layout]
};
// Problem b (b >= 0), or with b < 0 the whole batch in every launch.
hipError_t launch_plain_problem(const FwdArgs& a, const PlainBufs& pb, int b,
                                hipStream_t s);

hipError_t launch_fill(float* p, float v, int64_t n, hipStream_t s);

// Floats of the plain path's per-window partial buffer for `coef` coefficients.
size_t plain_part_floats(int T, int64_t coef);

// Device address, on the current device, of the library's static recompute
// area of kStaticScratchBytes bytes (looked up once per device).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
hipError_t static_scratch(void** ptr);

// Raise the dynamic-LDS limit of the fused kernels to `lds` bytes.
hipError_t prepare_kernels(size_t lds);

// 3D (spheroid) forward (sf_kernels3d.hip): one workgroup per problem; the
// coefficient arrays hold [3][n][nc] per problem, boundary [n][2][3],
// obstacles [M][5] = x, y, z, a_o, b_o.  Tc: time steps held in LDS at once.
// With `lists`, room for the candidate lists of the whole horizon (time chunks
// Tc, Tv then a multiple of list_window3() steps unless they cover the
// horizon).
int list_window3();
size_t fwd3_lds_bytes(int nc, int T, int Tc, int n_max, int M_max, int S_max, bool lists);
hipError_t prepare_kernels3(size_t lds);
hipError_t launch_fwd3(const FwdArgs& a, int threads, size_t lds, hipStream_t s);
// 3D adjoint: the forward's layout for time chunks of Tc plus its own buffers
// for VJP chunks of Tv <= Tc steps.
size_t bwd3_lds_bytes(int nc, int T, int Tc, int Tv, int n_max, int M_max, int S_max,
                      bool lists);
hipError_t launch_bwd3(const BwdArgs& a, int threads, size_t lds, int Tv, hipStream_t s);
// 3D plain path: the forward's stages as separate launches (state in pb:
// xb[2], lam, cxi, R, red), problem b alone (b >= 0) or the batch (b < 0).
hipError_t launch_plain3(const FwdArgs& a, const PlainBufs& pb, int b, size_t lds,
                         hipStream_t s);

// Candidate selection (sf_select.hip).  Batches of at most kSelectMaxBatch
// candidates (the ranking keys live in LDS).
constexpr int kSelectMaxBatch = 8192;
hipError_t launch_topk(const float* residual, int B, int k, int32_t* idx, hipStream_t s);
hipError_t launch_best(const float* residual, const float* cost, int B, float tol, int32_t* idx,
                       hipStream_t s);
hipError_t launch_smoothness(const ProbDesc* probs, int B, const float* Wdd, const float* xi,
                             int nc, int T, float inv_tf4, float* cost, hipStream_t s);
hipError_t launch_gather(const float* src, const int32_t* idx, int k, int S, int B, float* dst,
                         hipStream_t s);

}  // namespace sf
