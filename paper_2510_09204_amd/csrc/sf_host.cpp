// Host runtime of the SF library: argument validation, the FP64 KKT factors,
// the workspace layout, launch dispatch, the graph cache and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sf.h"
#include "sf_internal.h"

namespace {

thread_local std::string g_detail;

int fail(int code, const std::string& msg) {
  g_detail = msg;
  return code;
}

#define SF_HIP_CHECK(expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(SF_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_) + " (" + \
                                  std::to_string((int)e_) + ")");                       \
  } while (0)

constexpr size_t kLdsBudget = 160 * 1024;  // gfx950 LDS per workgroup
constexpr int kMaxRobots = 1024;
// The planar update tiles cover 2 axes x 4 row tiles of 16 robots (x 2
// coefficient tiles), so a planar problem holds at most 64 robots.
constexpr int kMaxRobots2d = 64;
constexpr int kMaxObs = 4096;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// FP64 factors.  The xi_bar step solves [I + rho H, A^T; A, 0] [xi; nu] =
// [eta; b] with H = F^T F + G^T G = ((n + M + 2) I - 1 1^T) (x) W^T W per axis
// and A = I_n (x) A1.  In the robot-mean mode H acts as (M + 2) W^T W and in
// each deviation mode as (n + M + 2) W^T W, so the inverse reduces to two
// (nc + 2)-sized KKT matrices K(c) = [I + rho c W^T W, A1^T; A1, 0].
// ---------------------------------------------------------------------------
std::vector<double> bernstein(int nc, int T) {
  std::vector<double> W((size_t)T * nc);
  const int deg = nc - 1;
  std::vector<double> binom(nc);
  for (int c = 0; c < nc; ++c) {
    double v = 1.0;
    for (int q = 1; q <= c; ++q) v = v * (deg - c + q) / q;
    binom[c] = v;
  }
  for (int k = 0; k < T; ++k) {
    const double tau = (double)k / (double)(T - 1);
    for (int c = 0; c < nc; ++c)
      W[(size_t)k * nc + c] = binom[c] * std::pow(tau, c) * std::pow(1.0 - tau, deg - c);
  }
  return W;
}

// Second derivative in tau of the Bernstein basis, [T][nc]: for degree N,
// B''_{c,N} = N (N - 1) (B_{c-2,N-2} - 2 B_{c-1,N-2} + B_{c,N-2}) (terms with
// an index outside 0..N-2 vanish); all zero for N < 2.
std::vector<double> bernstein_dd(int nc, int T) {
  std::vector<double> D((size_t)T * nc, 0.0);
  const int N = nc - 1;
  if (N < 2) return D;
  const std::vector<double> low = bernstein(N - 1, T);  // degree N - 2: N - 1 functions
  for (int k = 0; k < T; ++k)
    for (int c = 0; c < nc; ++c) {
      auto b = [&](int j) { return (j < 0 || j > N - 2) ? 0.0 : low[(size_t)k * (N - 1) + j]; };
      D[(size_t)k * nc + c] = (double)N * (N - 1) * (b(c - 2) - 2.0 * b(c - 1) + b(c));
    }
  return D;
}

// In-place Gauss-Jordan inverse with partial pivoting; false if singular.
bool invert(std::vector<double>& A, int m) {
  std::vector<double> I((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) I[(size_t)i * m + i] = 1.0;
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (std::fabs(A[(size_t)r * m + col]) > std::fabs(A[(size_t)piv * m + col])) piv = r;
    if (std::fabs(A[(size_t)piv * m + col]) < 1e-300) return false;
    if (piv != col)
      for (int q = 0; q < m; ++q) {
        std::swap(A[(size_t)piv * m + q], A[(size_t)col * m + q]);
        std::swap(I[(size_t)piv * m + q], I[(size_t)col * m + q]);
      }
    const double d = 1.0 / A[(size_t)col * m + col];
    for (int q = 0; q < m; ++q) {
      A[(size_t)col * m + q] *= d;
      I[(size_t)col * m + q] *= d;
    }
    for (int r = 0; r < m; ++r) {
      if (r == col) continue;
      const double f = A[(size_t)r * m + col];
      if (f == 0.0) continue;
      for (int q = 0; q < m; ++q) {
        A[(size_t)r * m + q] -= f * A[(size_t)col * m + q];
        I[(size_t)r * m + q] -= f * I[(size_t)col * m + q];
      }
    }
  }
  A.swap(I);
  return true;
}

struct ModeFactors {
  std::vector<double> S, SH, N;  // [nc][nc], [nc][nc], [nc][2]
};

// Q0: the objective's block per robot and axis ([nc][nc]; the identity for
// the projection, Wdd^T Wdd for the acceleration objective).
bool mode_factors(const std::vector<double>& W, const std::vector<double>& Q0, int nc, int T,
                  double rho, double c, ModeFactors& out) {
  std::vector<double> WtW((size_t)nc * nc, 0.0);
  for (int p = 0; p < nc; ++p)
    for (int q = 0; q < nc; ++q) {
      double s = 0.0;
      for (int k = 0; k < T; ++k) s += W[(size_t)k * nc + p] * W[(size_t)k * nc + q];
      WtW[(size_t)p * nc + q] = s;
    }
  const int m = nc + 2;
  std::vector<double> K((size_t)m * m, 0.0);
  for (int p = 0; p < nc; ++p) {
    for (int q = 0; q < nc; ++q)
      K[(size_t)p * m + q] = Q0[(size_t)p * nc + q] + rho * c * WtW[(size_t)p * nc + q];
    K[(size_t)p * m + nc] = W[p];                          // A1 row 0: position at k = 0
    K[(size_t)p * m + nc + 1] = W[(size_t)(T - 1) * nc + p];  // A1 row 1: k = K
    K[(size_t)nc * m + p] = W[p];
    K[(size_t)(nc + 1) * m + p] = W[(size_t)(T - 1) * nc + p];
  }
  if (!invert(K, m)) return false;
  out.S.assign((size_t)nc * nc, 0.0);
  out.SH.assign((size_t)nc * nc, 0.0);
  out.N.assign((size_t)nc * 2, 0.0);
  for (int p = 0; p < nc; ++p) {
    for (int q = 0; q < nc; ++q) out.S[(size_t)p * nc + q] = K[(size_t)p * m + q];
    out.N[p * 2 + 0] = K[(size_t)p * m + nc];
    out.N[p * 2 + 1] = K[(size_t)p * m + nc + 1];
  }
  for (int p = 0; p < nc; ++p)
    for (int q = 0; q < nc; ++q) {
      double s = 0.0;
      for (int r = 0; r < nc; ++r) s += out.S[(size_t)p * nc + r] * WtW[(size_t)r * nc + q];
      out.SH[(size_t)p * nc + q] = rho * c * s;
    }
  return true;
}

uint32_t float_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, sizeof(u));
  return u;
}

int choose_tc(int nc, int T, int n_max, int M_max, int S_max, int threads, bool bwd) {
  auto bytes = [&](int tc) {
    return bwd ? sf::bwd_lds_bytes(nc, T, tc, n_max, M_max, S_max, threads)
               : sf::fwd_lds_bytes(nc, T, tc, n_max, M_max, S_max, threads);
  };
  int best = 0;
  for (int tc = T; tc >= 1; --tc)
    if (bytes(tc) <= kLdsBudget) {
      best = tc;
      break;
    }
  if (best == 0) return 0;
  const int chunks = (T + best - 1) / best;
  return (T + chunks - 1) / chunks;  // balanced chunks
}

struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct sf_plan {
  sf_config_t cfg{};
  int B = 0;
  std::vector<sf::ProbDesc> desc;
  std::vector<int32_t> order;
  std::vector<float> W, Wdd, fac;
  int nfac = 0;
  int n_max = 0, M_max = 0, S_max = 0;
  int64_t S_total = 0, pos_total = 0, obs_total = 0, rob_total = 0;
  int n_ckpt = 0;
  int threads = 512;      // fused forward
  int threads_bwd = 512;  // fused adjoint
  bool tune_fwd = false;  // pick threads on first use (cfg.threads == 0)
  bool tune_bwd = false;
  int Tc_fwd = 0, Tc_bwd = 0;
  int Tv3 = 0;            // 3D adjoint: VJP time chunk (<= Tc_bwd)
  bool lists3 = false;    // 3D: the candidate lists fit (the kernels' LDS has room)
  bool lists3_on = true;  // 3D: sf_set_candidate_lists
  size_t lds_fwd = 0, lds_bwd = 0;
  // workspace layout (byte offsets)
  size_t off_desc = 0, off_order = 0, off_W = 0, off_Wdd = 0, off_fac = 0, off_cxi = 0,
         off_obs = 0, off_ckpt = 0, off_final = 0, off_seg = 0, off_X = 0, off_V = 0,
         off_R = 0, off_xb0 = 0, off_xb1 = 0, off_lam = 0, off_pcxi = 0, off_red = 0, off_part = 0,
         off_iters = 0, off_zero = 0, off_ovel = 0, off_gmask = 0, total = 0;
  bool moving = false;        // obstacle displacements set (sf_set_obstacle_motion)
  char* ws = nullptr;
  bool saved = false;
  int64_t generation = 0;     // sf_project / sf_set_obstacle_motion calls so far
  int saved_L = 0;
  bool saved_early = false;   // the saved forward ran with early exit
  float exit_tol = 0.f;       // early exit (sf_set_early_exit); check_every 0 = off
  int exit_every = 0;
  std::vector<GraphEntry> graphs;

  ~sf_plan() {
    for (auto& g : graphs) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
    }
  }
  template <typename Tp>
  Tp* at(size_t off) const {
    return reinterpret_cast<Tp*>(ws + off);
  }
};

namespace {

int validate_cfg(const sf_config_t* cfg) {
  if (!cfg) return fail(SF_ERR_INVALID_ARG, "cfg is NULL");
  if (cfg->n_dim != 2 && cfg->n_dim != 3) return fail(SF_ERR_SHAPE, "n_dim must be 2 or 3");
  if (cfg->n_coef < 2 || cfg->n_coef > sf::kMaxCoef)
    return fail(SF_ERR_SHAPE, "n_coef must be in [2, 32]");
  if (cfg->n_steps < 2 || cfg->n_steps > 4096)
    return fail(SF_ERR_SHAPE, "n_steps must be in [2, 4096]");
  if (cfg->checkpoint_every < 1) return fail(SF_ERR_INVALID_ARG, "checkpoint_every < 1");
  if (cfg->max_iters < 0) return fail(SF_ERR_INVALID_ARG, "max_iters < 0");
  if (!(cfg->rho > 0.0) || !std::isfinite(cfg->rho))
    return fail(SF_ERR_INVALID_ARG, "rho must be finite and > 0");
  if (cfg->threads != 0 && cfg->threads != 256 && cfg->threads != 512 &&
      cfg->threads != 1024)
    return fail(SF_ERR_INVALID_ARG, "threads must be 0, 256, 512 or 1024");
  if (cfg->objective != SF_OBJECTIVE_PROJECTION && cfg->objective != SF_OBJECTIVE_ACCEL)
    return fail(SF_ERR_INVALID_ARG, "objective must be SF_OBJECTIVE_PROJECTION or _ACCEL");
  return SF_OK;
}

int build_plan(const sf_config_t* cfg, int B, const int32_t* n_robots, const int32_t* n_obs,
               const float* robot_a, const float* box, std::unique_ptr<sf_plan>& out) {
  int rc = validate_cfg(cfg);
  if (rc) return rc;
  if (B < 1) return fail(SF_ERR_INVALID_ARG, "n_problems < 1");
  if (!n_robots || !n_obs || !robot_a || !box)
    return fail(SF_ERR_INVALID_ARG, "n_robots, n_obs, robot_a and box must be non-NULL");
  auto p = std::make_unique<sf_plan>();
  p->cfg = *cfg;
  p->B = B;
  const int nc = cfg->n_coef, T = cfg->n_steps;
  const std::vector<double> W = bernstein(nc, T);
  p->W.resize((size_t)T * nc);
  for (size_t q = 0; q < p->W.size(); ++q) p->W[q] = (float)W[q];
  const std::vector<double> Wdd = bernstein_dd(nc, T);
  p->Wdd.resize(Wdd.size());
  for (size_t q = 0; q < Wdd.size(); ++q) p->Wdd[q] = (float)Wdd[q];
  std::vector<double> Q0((size_t)nc * nc, 0.0);
  if (cfg->objective == SF_OBJECTIVE_ACCEL) {
    for (int a = 0; a < nc; ++a)
      for (int c = 0; c < nc; ++c) {
        double s = 0.0;
        for (int k = 0; k < T; ++k) s += Wdd[(size_t)k * nc + a] * Wdd[(size_t)k * nc + c];
        Q0[(size_t)a * nc + c] = s;
      }
  } else {
    for (int a = 0; a < nc; ++a) Q0[(size_t)a * nc + a] = 1.0;
  }
  const int D = cfg->n_dim;
  std::map<std::pair<int, int>, int> fac_index;
  const int fs = sf::fac_stride(nc);
  int64_t coef = 0, rob = 0, obs = 0, pos = 0;
  std::vector<double> cost(B);
  for (int b = 0; b < B; ++b) {
    const int n = n_robots[b], M = n_obs[b];
    const int n_limit = D == 2 ? kMaxRobots2d : kMaxRobots;
    if (n < 1 || n > n_limit)
      return fail(SF_ERR_SHAPE, "problem " + std::to_string(b) + ": n_robots out of [1, " +
                                    std::to_string(n_limit) + "]");
    if (M < 0 || M > kMaxObs)
      return fail(SF_ERR_SHAPE, "problem " + std::to_string(b) + ": n_obs out of [0, 4096]");
    const float a = robot_a[(size_t)b * (D - 1)];
    const float rb = D == 3 ? robot_a[(size_t)b * 2 + 1] : a;
    if (!(a > 0.f) || !std::isfinite(a) || !(rb > 0.f) || !std::isfinite(rb))
      return fail(SF_ERR_INVALID_ARG, "problem " + std::to_string(b) + ": robot sizes must be > 0");
    const float* bx = box + (size_t)b * 2 * D;
    for (int q = 0; q < 2 * D; ++q)
      if (!std::isfinite(bx[q]))
        return fail(SF_ERR_NONFINITE, "problem " + std::to_string(b) + ": box not finite");
    for (int q = 0; q < D; ++q)
      if (!(bx[q] < bx[D + q]))
        return fail(SF_ERR_INVALID_ARG, "problem " + std::to_string(b) + ": p_min >= p_max");
    auto key = std::make_pair(n, M);
    auto it = fac_index.find(key);
    int fi;
    if (it == fac_index.end()) {
      ModeFactors perp, par;
      if (!mode_factors(W, Q0, nc, T, cfg->rho, (double)(n + M + 2), perp) ||
          !mode_factors(W, Q0, nc, T, cfg->rho, (double)(M + 2), par))
        return fail(SF_ERR_SHAPE, "singular KKT matrix");
      fi = p->nfac++;
      fac_index[key] = fi;
      const size_t base = p->fac.size();
      p->fac.resize(base + fs);
      float* f = p->fac.data() + base;
      const int nc2 = nc * nc;
      for (int q = 0; q < nc2; ++q) {
        f[q] = (float)perp.S[q];
        f[nc2 + q] = (float)(par.S[q] - perp.S[q]);
        f[2 * nc2 + q] = (float)perp.SH[q];
        f[3 * nc2 + q] = (float)(par.SH[q] - perp.SH[q]);
      }
      for (int q = 0; q < 2 * nc; ++q) {
        f[4 * nc2 + q] = (float)perp.N[q];
        f[4 * nc2 + 2 * nc + q] = (float)(par.N[q] - perp.N[q]);
      }
    } else {
      fi = it->second;
    }
    sf::ProbDesc d{};
    d.n = n;
    d.M = M;
    d.coef_off = (int32_t)coef;
    d.rob_off = (int32_t)rob;
    d.obs_off = (int32_t)obs;
    d.fac = fi;
    d.pos_off = (int32_t)pos;
    d.a = a;
    d.b = rb;
    for (int q = 0; q < D; ++q) {
      d.pmin[q] = bx[q];
      d.pmax[q] = bx[D + q];
    }
    p->desc.push_back(d);
    coef += (int64_t)D * n * nc;
    rob += n;
    obs += M;
    pos += (int64_t)n * T;
    p->n_max = std::max(p->n_max, n);
    p->M_max = std::max(p->M_max, M);
    p->S_max = std::max(p->S_max, D * n * nc);
    cost[b] = (double)T * (0.5 * n * (n - 1) + (double)n * M + n) + 4.0 * n * nc * nc;
  }
  if (coef > (int64_t)1 << 30 || pos > (int64_t)1 << 30)
    return fail(SF_ERR_SHAPE, "batch too large for 32-bit offsets");
  p->S_total = coef;
  p->rob_total = rob;
  p->obs_total = obs;
  p->pos_total = pos;
  // longest problems first (LPT order of the launch slots)
  p->order.resize(B);
  for (int b = 0; b < B; ++b) p->order[b] = b;
  std::stable_sort(p->order.begin(), p->order.end(),
                   [&](int x, int y) { return cost[x] > cost[y]; });
  p->threads = cfg->threads ? cfg->threads : 512;
  p->threads_bwd = p->threads;
  p->tune_fwd = p->tune_bwd = (cfg->threads == 0);
  if (D == 3) {
    // 3D: the forward kernel of sf_kernels3d.hip, the longest time chunk that
    // fits in LDS (balanced); 1024 threads unless set (measured fastest on
    // 16 and 32 robots: 15 / 40 us per iteration against 20 / 50 at 512)
    p->tune_fwd = p->tune_bwd = false;
    if (cfg->threads == 0) p->threads = p->threads_bwd = 1024;
    // The adjoint recomputes forward iterates with the forward's time chunks
    // (same sums, same bits) and runs its VJP in chunks of Tv <= Tc steps; a
    // plan that can save a forward takes the longest Tc for which some Tv fits.
    // With the candidate lists (when they fit; their LDS covers the whole
    // horizon) chunks shorter than the horizon are multiples of the list
    // window.
    auto pick = [&](bool lists) -> bool {
      const int win = sf::list_window3();
      auto len_ok = [&](int len) { return !lists || len >= T || len % win == 0; };
      auto round_win = [&](int len) { return lists && len < T ? (len + win - 1) / win * win : len; };
      // longest VJP chunk that fits beside forward chunks of tc
      auto tv_for = [&](int tc) {
        int tv = tc;
        while (tv > 0 &&
               sf::bwd3_lds_bytes(nc, T, tc, tv, p->n_max, p->M_max, p->S_max, lists) >
                   kLdsBudget)
          --tv;
        if (lists && tv < T) tv = tv / win * win;
        return tv;
      };
      int best = 0;
      for (int tc = T; tc >= 1 && best == 0; --tc)
        if (len_ok(tc) &&
            sf::fwd3_lds_bytes(nc, T, tc, p->n_max, p->M_max, p->S_max, lists) <= kLdsBudget)
          best = tc;
      if (best == 0) return false;
      int tc = best, tv = 0;
      if (cfg->max_iters > 0) {
        // fewest chunk passes per adjoint iteration (recompute plus VJP)
        int score = INT_MAX;
        for (int c = best; c >= 1; --c) {
          const int v = len_ok(c) ? tv_for(c) : 0;
          if (v == 0) continue;
          const int sc = (T + c - 1) / c + (T + v - 1) / v;
          if (sc < score) {
            score = sc;
            tc = c;
            tv = v;
          }
        }
        if (tv == 0) return false;
      }
      const int chunks = (T + tc - 1) / tc;
      p->Tc_fwd = p->Tc_bwd = round_win((T + chunks - 1) / chunks);
      p->Tv3 = 0;
      if (tv > 0) {
        const int vchunks = (T + tv - 1) / tv;
        p->Tv3 = std::min(p->Tc_bwd, round_win((T + vchunks - 1) / vchunks));
      }
      p->lists3 = lists;
      p->lds_fwd = sf::fwd3_lds_bytes(nc, T, p->Tc_fwd, p->n_max, p->M_max, p->S_max, lists);
      p->lds_bwd = p->Tv3 > 0 ? sf::bwd3_lds_bytes(nc, T, p->Tc_bwd, p->Tv3, p->n_max,
                                                   p->M_max, p->S_max, lists)
                              : 0;
      return true;
    };
    if (!pick(true) && !pick(false))
      return fail(SF_ERR_SHAPE, cfg->max_iters > 0
                                    ? "problem or adjoint state does not fit the LDS of one "
                                      "workgroup"
                                    : "problem state does not fit the LDS of one workgroup");
  }
  // One time-chunk length for both kernels: the adjoint recomputes forward
  // iterates and must sum in the same order to reproduce them bitwise.
  if (D == 2) {
    p->Tc_fwd = choose_tc(nc, T, p->n_max, p->M_max, p->S_max, p->threads, false);
    p->Tc_bwd = choose_tc(nc, T, p->n_max, p->M_max, p->S_max, p->threads, true);
    if (p->Tc_fwd == 0 || p->Tc_bwd == 0)
      return fail(SF_ERR_SHAPE, "problem state does not fit the LDS of one workgroup");
    p->Tc_fwd = p->Tc_bwd = std::min(p->Tc_fwd, p->Tc_bwd);
    p->lds_fwd = sf::fwd_lds_bytes(nc, T, p->Tc_fwd, p->n_max, p->M_max, p->S_max, p->threads);
    p->lds_bwd = sf::bwd_lds_bytes(nc, T, p->Tc_bwd, p->n_max, p->M_max, p->S_max, p->threads);
  }
  const int L = cfg->max_iters, k = cfg->checkpoint_every;
  p->n_ckpt = L > 0 ? (L + k - 1) / k : 0;
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + std::max<size_t>(bytes, 1));
    return o;
  };
  const size_t F = sizeof(float);
  p->off_desc = take(sizeof(sf::ProbDesc) * B);
  p->off_order = take(sizeof(int32_t) * B);
  p->off_W = take(F * T * nc);
  p->off_Wdd = take(F * T * nc);
  p->off_fac = take(F * p->fac.size());
  p->off_cxi = take(F * coef);
  p->off_obs = take(F * (2 * D - 1) * obs);
  p->off_ckpt = take(F * 2 * coef * (size_t)p->n_ckpt);
  p->off_final = take(F * 2 * coef);
  p->off_seg = take(F * 2 * coef * (size_t)k);
  p->off_X = take(F * 2 * pos);
  p->off_V = take(F * 2 * pos);
  p->off_R = take(F * coef);
  p->off_xb0 = take(F * coef);
  p->off_xb1 = take(F * coef);
  p->off_lam = take(F * coef);
  p->off_pcxi = take(F * coef);
  p->off_red = take(F * 4 * B);
  p->off_part = take(F * sf::plain_part_floats(T, coef));
  p->off_iters = take(sizeof(int32_t) * B);
  p->off_zero = take(F * coef);   // the target read by the acceleration objective
  p->off_ovel = take(F * D * obs);  // obstacle displacements
  if (D == 2)                        // candidate lists of chunked horizons
    p->off_gmask = take(sf::chunk_list_bytes(T, p->Tc_fwd, p->n_max, p->M_max) * (size_t)B);
  p->total = off;
  out = std::move(p);
  return SF_OK;
}

sf::FwdArgs fwd_args(const sf_plan* p, const float* xi, const float* xi0, const float* lam0,
                     const float* boundary, const float* obstacles, int L, bool save,
                     float* xi_out, float* lam_out, float* residual) {
  sf::FwdArgs a{};
  a.probs = p->at<sf::ProbDesc>(p->off_desc);
  a.order = p->at<int32_t>(p->off_order);
  a.W = p->at<float>(p->off_W);
  a.fac = p->at<float>(p->off_fac);
  // the acceleration objective has no target: its linear term is zero
  a.xi = p->cfg.objective == SF_OBJECTIVE_ACCEL ? p->at<float>(p->off_zero) : xi;
  a.ovel = p->moving ? p->at<float>(p->off_ovel) : nullptr;
  a.xi0 = xi0;
  a.lam0 = lam0;
  a.boundary = boundary;
  a.obstacles = obstacles;
  a.xi_out = xi_out;
  a.lam_out = lam_out;
  a.residual = residual;
  a.ws_cxi = p->at<float>(p->off_cxi);
  a.ws_obs = p->at<float>(p->off_obs);
  a.ws_ckpt = p->at<float>(p->off_ckpt);
  a.ws_final = p->at<float>(p->off_final);
  a.ws_iters = p->at<int32_t>(p->off_iters);
  a.gmask = p->at<unsigned>(p->off_gmask);
  a.S_total = p->S_total;
  a.B = p->B;
  a.nc = p->cfg.n_coef;
  a.T = p->cfg.n_steps;
  a.Tc = p->Tc_fwd;
  a.n_max = p->n_max;
  a.M_max = p->M_max;
  a.S_max = p->S_max;
  a.L = L;
  a.ckpt_every = p->cfg.checkpoint_every;
  a.save = save ? 1 : 0;
  a.check_every = p->exit_every;
  a.lists3 = p->lists3 && p->lists3_on ? 1 : 0;
  a.tol = p->exit_tol;
  a.rho = (float)p->cfg.rho;
  return a;
}

// ---------------------------------------------------------------------------
// Autotuner: threads per workgroup of the fused kernels, chosen by timing the
// candidates on the device at the first call of a plan and cached per size
// bucket (gfx arch, n_coef, n_steps, robot/obstacle/batch buckets, kernel).
// With SF_AUTOTUNE_CACHE=<file> the choices persist as JSON lines.
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

int bucket_up(int v, const int* edges, int ne) {
  for (int q = 0; q < ne; ++q)
    if (v <= edges[q]) return edges[q];
  return ((v + 63) / 64) * 64;
}

std::string tune_key(const sf_plan* p, bool bwd) {
  static const int nb[] = {8, 16, 32, 48, 64};
  static const int mb[] = {0, 15, 30, 60};
  static const int bb[] = {16, 64, 128, 256};
  int dev = 0;
  char arch[64] = "unknown";
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c)
      if (*c == ':' || *c == '"' || *c == ' ') *c = '_';
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s/%s/nc%d/T%d/n%d/M%d/B%d/k%d", bwd ? "bwd" : "fwd", arch,
                p->cfg.n_coef, p->cfg.n_steps, bucket_up(p->n_max, nb, 5),
                bucket_up(p->M_max, mb, 4), bucket_up(p->B, bb, 4),
                bwd ? p->cfg.checkpoint_every : 0);
  return buf;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("SF_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t k0 = line.find("\"key\": \"");
    const size_t t0 = line.find("\"threads\": ");
    if (k0 == std::string::npos || t0 == std::string::npos) continue;
    const size_t ks = k0 + 8, ke = line.find('"', ks);
    if (ke == std::string::npos) continue;
    const int t = std::atoi(line.c_str() + t0 + 11);
    if (t == 256 || t == 512 || t == 1024) g_tune[line.substr(ks, ke - ks)] = t;
  }
}

bool tune_lookup(const std::string& key, int& threads) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  threads = it->second;
  return true;
}

void tune_store(const std::string& key, int threads, const float* ms) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_load_locked();
  g_tune[key] = threads;
  const char* path = std::getenv("SF_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream out(path, std::ios::app);
  out << "{\"key\": \"" << key << "\", \"threads\": " << threads << ", \"ms\": [" << ms[0]
      << ", " << ms[1] << ", " << ms[2] << "]}\n";
}

// Time `launch(threads)` for each candidate (one warm-up, then the mean of two
// timed launches) and return the fastest.  Synchronises the stream.
template <typename F>
int time_candidates(hipStream_t s, F launch, float* ms_out, hipError_t& err) {
  static const int cand[3] = {256, 512, 1024};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  int best = 512;
  float best_ms = 1e30f;
  for (int q = 0; q < 3 && err == hipSuccess; ++q) {
    err = launch(cand[q]);
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int r = 0; r < 2 && err == hipSuccess; ++r) err = launch(cand[q]);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    ms_out[q] = ms / 2.f;
    if (err == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = cand[q];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return best;
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

}  // namespace

extern "C" {

int sf_setup(const sf_config_t* cfg, int32_t n_problems, const int32_t* n_robots,
             const int32_t* n_obs, const float* robot_a, const float* box, void* workspace,
             size_t* workspace_bytes, void* stream, sf_plan_t** plan) {
  g_detail.clear();
  if (!workspace_bytes) return fail(SF_ERR_INVALID_ARG, "workspace_bytes is NULL");
  std::unique_ptr<sf_plan> p;
  int rc = build_plan(cfg, n_problems, n_robots, n_obs, robot_a, box, p);
  if (rc) return rc;
  if (!workspace) {
    *workspace_bytes = p->total;
    return SF_OK;
  }
  if (!plan) return fail(SF_ERR_INVALID_ARG, "plan is NULL");
  if (*workspace_bytes < p->total)
    return fail(SF_ERR_WORKSPACE_SMALL, "workspace has " + std::to_string(*workspace_bytes) +
                                            " bytes, plan needs " + std::to_string(p->total));
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(SF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  int dev = 0, lds_max = 0;
  SF_HIP_CHECK(hipGetDevice(&dev));
  SF_HIP_CHECK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if ((size_t)lds_max < std::max(p->lds_fwd, p->lds_bwd))
    return fail(SF_ERR_SHAPE, "device LDS per workgroup (" + std::to_string(lds_max) +
                                  ") below the plan's need");
  if (p->cfg.n_dim == 3)
    SF_HIP_CHECK(sf::prepare_kernels3(std::max(p->lds_fwd, p->lds_bwd)));
  else
    SF_HIP_CHECK(sf::prepare_kernels(std::max(p->lds_fwd, p->lds_bwd)));
  {
    void* area = nullptr;   // look up the static recompute area on this device once
    SF_HIP_CHECK(sf::static_scratch(&area));
  }
  p->ws = static_cast<char*>(workspace);
  hipStream_t s = static_cast<hipStream_t>(stream);
  SF_HIP_CHECK(hipMemcpyAsync(p->ws + p->off_desc, p->desc.data(),
                              sizeof(sf::ProbDesc) * p->B, hipMemcpyHostToDevice, s));
  SF_HIP_CHECK(hipMemcpyAsync(p->ws + p->off_order, p->order.data(), sizeof(int32_t) * p->B,
                              hipMemcpyHostToDevice, s));
  SF_HIP_CHECK(hipMemcpyAsync(p->ws + p->off_W, p->W.data(), sizeof(float) * p->W.size(),
                              hipMemcpyHostToDevice, s));
  SF_HIP_CHECK(hipMemcpyAsync(p->ws + p->off_Wdd, p->Wdd.data(), sizeof(float) * p->Wdd.size(),
                              hipMemcpyHostToDevice, s));
  SF_HIP_CHECK(hipMemcpyAsync(p->ws + p->off_fac, p->fac.data(), sizeof(float) * p->fac.size(),
                              hipMemcpyHostToDevice, s));
  SF_HIP_CHECK(sf::launch_fill(reinterpret_cast<float*>(p->ws + p->off_zero), 0.f,
                               (int64_t)p->S_total, s));
  SF_HIP_CHECK(hipStreamSynchronize(s));
  *workspace_bytes = p->total;
  *plan = p.release();
  return SF_OK;
}

int sf_project(sf_plan_t* plan, void* workspace, const float* xi, const float* xi0,
               const float* lam0, const float* boundary, const float* obstacles,
               int32_t n_iters, int32_t flags, float* xi_out, float* lam_out, float* residual,
               void* stream) {
  g_detail.clear();
  if (!plan) return fail(SF_ERR_INVALID_ARG, "plan is NULL");
  if (workspace != plan->ws)
    return fail(SF_ERR_INVALID_ARG, "workspace differs from the one bound at sf_setup");
  const bool accel = plan->cfg.objective == SF_OBJECTIVE_ACCEL;
  if ((!xi && !accel) || !xi0 || !lam0 || !boundary || !xi_out || !lam_out || !residual)
    return fail(SF_ERR_INVALID_ARG, "NULL input or output pointer");
  if (plan->obs_total > 0 && !obstacles)
    return fail(SF_ERR_INVALID_ARG, "obstacles is NULL but the plan has obstacles");
  if (n_iters < 0) return fail(SF_ERR_INVALID_ARG, "n_iters < 0");
  if (flags & ~(SF_SAVE_FOR_BACKWARD | SF_PLAIN | SF_GRAPH | SF_UNFUSED))
    return fail(SF_ERR_INVALID_ARG, "unknown flag bits");
  const bool save = flags & SF_SAVE_FOR_BACKWARD;
  const bool unfused = flags & SF_UNFUSED;
  const bool plain = (flags & SF_PLAIN) || unfused;
  if ((flags & SF_PLAIN) && unfused)
    return fail(SF_ERR_INVALID_ARG, "SF_PLAIN and SF_UNFUSED together");
  if (save && plain)
    return fail(SF_ERR_INVALID_ARG, "SF_SAVE_FOR_BACKWARD with SF_PLAIN or SF_UNFUSED");
  if (plain && plan->exit_every > 0)
    return fail(SF_ERR_INVALID_ARG, "early exit is not available with SF_PLAIN or SF_UNFUSED");
  if (save && n_iters > plan->cfg.max_iters)
    return fail(SF_ERR_INVALID_ARG, "n_iters exceeds cfg.max_iters for a saved forward");
  if (xi_out == xi || xi_out == xi0 || lam_out == lam0 || xi_out == lam_out)
    return fail(SF_ERR_INVALID_ARG, "outputs must not alias inputs");
  const bool dim3 = plan->cfg.n_dim == 3;
  hipStream_t s = static_cast<hipStream_t>(stream);
  plan->saved = false;
  ++plan->generation;
  sf::FwdArgs a = fwd_args(plan, xi, xi0, lam0, boundary, obstacles, n_iters, save, xi_out,
                           lam_out, residual);
  auto launch_fused = [&](const sf::FwdArgs& args, int th) {
    return dim3 ? sf::launch_fwd3(args, th, plan->lds_fwd, s)
                : sf::launch_fwd_fused(args, th, plan->lds_fwd, s);
  };
  if (plain) {
    sf::PlainBufs pb{};
    pb.X = plan->at<float>(plan->off_X);
    pb.V = plan->at<float>(plan->off_V);
    pb.R = plan->at<float>(plan->off_R);
    pb.xb[0] = plan->at<float>(plan->off_xb0);
    pb.xb[1] = plan->at<float>(plan->off_xb1);
    pb.lam = plan->at<float>(plan->off_lam);
    pb.cxi = plan->at<float>(plan->off_pcxi);
    pb.red = plan->at<float>(plan->off_red);
    pb.part = plan->at<float>(plan->off_part);
    if (dim3) {
      if (unfused) {
        SF_HIP_CHECK(sf::launch_plain3(a, pb, -1, plan->lds_fwd, s));
      } else {
        for (int b = 0; b < plan->B; ++b)
          SF_HIP_CHECK(sf::launch_plain3(a, pb, b, plan->lds_fwd, s));
      }
    } else if (unfused) {
      SF_HIP_CHECK(sf::launch_plain_problem(a, pb, -1, s));
    } else {
      for (int b = 0; b < plan->B; ++b) SF_HIP_CHECK(sf::launch_plain_problem(a, pb, b, s));
    }
    return SF_OK;
  }
  if ((flags & SF_GRAPH) && s == nullptr)
    return fail(SF_ERR_INVALID_ARG, "SF_GRAPH needs a non-default stream (capture)");
  if (plan->tune_fwd && n_iters > 0 && !stream_capturing(s)) {
    const std::string key = tune_key(plan, false);
    int t = 0;
    if (!tune_lookup(key, t)) {
      // trials of a few dozen iterations: the first iterations of a launch
      // (set-up, the forced list build) are not representative
      sf::FwdArgs trial = a;
      trial.L = std::min<int>(n_iters, 24);
      trial.save = 0;
      float ms[3] = {0.f, 0.f, 0.f};
      hipError_t err = hipSuccess;
      t = time_candidates(
          s, [&](int th) { return sf::launch_fwd_fused(trial, th, plan->lds_fwd, s); }, ms,
          err);
      SF_HIP_CHECK(err);
      tune_store(key, t, ms);
    }
    plan->threads = t;
    plan->tune_fwd = false;
  }
  if (flags & SF_GRAPH) {
    std::vector<uint64_t> key = {(uint64_t)xi,      (uint64_t)xi0,     (uint64_t)lam0,
                                 (uint64_t)boundary, (uint64_t)obstacles, (uint64_t)xi_out,
                                 (uint64_t)lam_out, (uint64_t)residual, (uint64_t)n_iters,
                                 (uint64_t)save,    (uint64_t)plan->threads, (uint64_t)s,
                                 (uint64_t)plan->exit_every, (uint64_t)float_bits(plan->exit_tol),
                                 (uint64_t)plan->moving, (uint64_t)a.lists3};
    GraphEntry* hit = nullptr;
    for (auto& g : plan->graphs)
      if (g.key == key) hit = &g;
    if (!hit) {
      GraphEntry g;
      g.key = key;
      SF_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipError_t le = launch_fused(a, plan->threads);
      hipError_t ce = hipStreamEndCapture(s, &g.graph);
      SF_HIP_CHECK(le);
      SF_HIP_CHECK(ce);
      SF_HIP_CHECK(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
      if (plan->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(plan->graphs.front().exec);
        (void)hipGraphDestroy(plan->graphs.front().graph);
        plan->graphs.erase(plan->graphs.begin());
      }
      plan->graphs.push_back(g);
      hit = &plan->graphs.back();
    }
    SF_HIP_CHECK(hipGraphLaunch(hit->exec, s));
  } else {
    SF_HIP_CHECK(launch_fused(a, plan->threads));
  }
  plan->saved = save;
  plan->saved_L = n_iters;
  plan->saved_early = plan->exit_every > 0;
  return SF_OK;
}

}  // extern "C"

namespace {

// sf_project_backward and its variant without a workspace recompute area:
// with `static_area` the segment recompute goes to the library's static device
// array, and the call neither autotunes (that creates events) nor allocates.
int backward_impl(sf_plan_t* plan, void* workspace, const float* g_xi_out,
                  const float* g_lam_out, const float* g_residual, float fp_weight,
                  float* g_xi, float* g_xi0, float* g_lam0, void* stream, bool static_area) {
  g_detail.clear();
  if (!plan) return fail(SF_ERR_INVALID_ARG, "plan is NULL");
  if (workspace != plan->ws)
    return fail(SF_ERR_INVALID_ARG, "workspace differs from the one bound at sf_setup");
  if (!plan->saved) return fail(SF_ERR_NOT_SAVED, "no saved forward on this plan");
  if (!std::isfinite(fp_weight)) return fail(SF_ERR_NONFINITE, "fp_weight not finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  sf::BwdArgs a{};
  a.probs = plan->at<sf::ProbDesc>(plan->off_desc);
  a.order = plan->at<int32_t>(plan->off_order);
  a.W = plan->at<float>(plan->off_W);
  a.fac = plan->at<float>(plan->off_fac);
  a.cxi = plan->at<float>(plan->off_cxi);
  a.obs = plan->at<float>(plan->off_obs);
  a.ovel = plan->moving ? plan->at<float>(plan->off_ovel) : nullptr;
  a.ckpt = plan->at<float>(plan->off_ckpt);
  a.fin = plan->at<float>(plan->off_final);
  if (static_area) {
    const size_t need = sizeof(float) * 2 * (size_t)plan->S_total *
                        (size_t)plan->cfg.checkpoint_every;
    if (need > sf::kStaticScratchBytes)
      return fail(SF_ERR_SHAPE, "recompute area of " + std::to_string(need) +
                                    " bytes exceeds the static area of " +
                                    std::to_string(sf::kStaticScratchBytes) + " bytes");
    void* area = nullptr;
    SF_HIP_CHECK(sf::static_scratch(&area));
    a.seg = static_cast<float*>(area);
  } else {
    a.seg = plan->at<float>(plan->off_seg);
  }
  a.g_xi_out = g_xi_out;
  a.g_lam_out = g_lam_out;
  a.g_res = g_residual;
  a.g_xi = g_xi;
  a.g_xi0 = g_xi0;
  a.g_lam0 = g_lam0;
  a.iters = plan->saved_early ? plan->at<int32_t>(plan->off_iters) : nullptr;
  a.gmask = plan->at<unsigned>(plan->off_gmask);
  a.S_total = plan->S_total;
  a.B = plan->B;
  a.nc = plan->cfg.n_coef;
  a.T = plan->cfg.n_steps;
  a.Tc = plan->Tc_bwd;
  a.n_max = plan->n_max;
  a.M_max = plan->M_max;
  a.S_max = plan->S_max;
  a.L = plan->saved_L;
  a.ckpt_every = plan->cfg.checkpoint_every;
  a.lists3 = plan->lists3 && plan->lists3_on ? 1 : 0;
  a.rho = (float)plan->cfg.rho;
  a.fp_weight = fp_weight;
  if (!static_area && plan->tune_bwd && a.L > 0 && !stream_capturing(s)) {
    const std::string key = tune_key(plan, true);
    int t = 0;
    if (!tune_lookup(key, t)) {
      sf::BwdArgs trial = a;
      trial.L = std::min<int>(a.L, std::max(2, a.ckpt_every));
      float ms[3] = {0.f, 0.f, 0.f};
      hipError_t err = hipSuccess;
      t = time_candidates(
          s, [&](int th) { return sf::launch_bwd_fused(trial, th, plan->lds_bwd, s); }, ms,
          err);
      SF_HIP_CHECK(err);
      tune_store(key, t, ms);
    }
    plan->threads_bwd = t;
    plan->tune_bwd = false;
  }
  if (plan->cfg.n_dim == 3) {
    if (plan->Tv3 == 0)
      return fail(SF_ERR_SHAPE, "the plan has no adjoint layout (max_iters was 0)");
    SF_HIP_CHECK(sf::launch_bwd3(a, plan->threads_bwd, plan->lds_bwd, plan->Tv3, s));
  } else {
    SF_HIP_CHECK(sf::launch_bwd_fused(a, plan->threads_bwd, plan->lds_bwd, s));
  }
  if (g_xi && plan->cfg.objective == SF_OBJECTIVE_ACCEL)
    SF_HIP_CHECK(sf::launch_fill(g_xi, 0.f, plan->S_total, s));   // xi is not an input there
  return SF_OK;
}

}  // namespace

extern "C" {

int sf_project_backward(sf_plan_t* plan, void* workspace, const float* g_xi_out,
                        const float* g_lam_out, const float* g_residual, float fp_weight,
                        float* g_xi, float* g_xi0, float* g_lam0, void* stream) {
  return backward_impl(plan, workspace, g_xi_out, g_lam_out, g_residual, fp_weight, g_xi,
                       g_xi0, g_lam0, stream, false);
}

int sf_project_backward_static(sf_plan_t* plan, void* workspace, const float* g_xi_out,
                               const float* g_lam_out, const float* g_residual,
                               float fp_weight, float* g_xi, float* g_xi0, float* g_lam0,
                               void* stream) {
  return backward_impl(plan, workspace, g_xi_out, g_lam_out, g_residual, fp_weight, g_xi,
                       g_xi0, g_lam0, stream, true);
}

void sf_destroy(sf_plan_t* plan) { delete plan; }

const char* sf_error_string(int code) {
  switch (code) {
    case SF_OK: return "success";
    case SF_ERR_INVALID_ARG: return "invalid argument";
    case SF_ERR_SHAPE: return "unsupported shape";
    case SF_ERR_WORKSPACE_SMALL: return "workspace too small";
    case SF_ERR_NOT_SAVED: return "no saved forward for the backward";
    case SF_ERR_HIP: return "HIP runtime error";
    case SF_ERR_NONFINITE: return "non-finite input";
    default: return "unknown error code";
  }
}

const char* sf_last_error_detail(void) { return g_detail.c_str(); }

int sf_plan_threads(const sf_plan_t* plan) { return plan ? plan->threads : 0; }

int64_t sf_forward_generation(const sf_plan_t* plan) { return plan ? plan->generation : -1; }

int sf_set_early_exit(sf_plan_t* plan, float tol, int32_t check_every) {
  g_detail.clear();
  if (!plan) return fail(SF_ERR_INVALID_ARG, "plan is NULL");
  if (check_every < 0) return fail(SF_ERR_INVALID_ARG, "check_every < 0");
  if (!std::isfinite(tol) || tol < 0.f) return fail(SF_ERR_INVALID_ARG, "tol must be finite, >= 0");
  plan->exit_every = check_every;
  plan->exit_tol = tol;
  return SF_OK;
}

int sf_set_candidate_lists(sf_plan_t* plan, int32_t enable) {
  g_detail.clear();
  if (!plan) return fail(SF_ERR_INVALID_ARG, "plan is NULL");
  if (plan->cfg.n_dim != 3)
    return fail(SF_ERR_INVALID_ARG, "candidate lists are switchable for n_dim = 3 only");
  plan->lists3_on = enable != 0;
  return plan->lists3 && plan->lists3_on ? 1 : 0;
}

int sf_project_iterations(const sf_plan_t* plan, const void* workspace, int32_t* iters,
                          void* stream) {
  g_detail.clear();
  if (!plan) return fail(SF_ERR_INVALID_ARG, "plan is NULL");
  if (workspace != plan->ws)
    return fail(SF_ERR_INVALID_ARG, "workspace differs from the one bound at sf_setup");
  if (!iters) return fail(SF_ERR_INVALID_ARG, "iters is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  SF_HIP_CHECK(hipMemcpyAsync(iters, plan->ws + plan->off_iters, sizeof(int32_t) * plan->B,
                              hipMemcpyDeviceToDevice, s));
  return SF_OK;
}

int sf_set_obstacle_motion(sf_plan_t* plan, void* workspace, const float* displacement,
                           void* stream) {
  g_detail.clear();
  if (!plan) return fail(SF_ERR_INVALID_ARG, "plan is NULL");
  if (workspace != plan->ws)
    return fail(SF_ERR_INVALID_ARG, "workspace differs from the one bound at sf_setup");
  plan->saved = false;   // a saved forward no longer matches the obstacles
  ++plan->generation;
  if (!displacement) {
    plan->moving = false;
    return SF_OK;
  }
  if (plan->obs_total > 0)
    SF_HIP_CHECK(hipMemcpyAsync(plan->ws + plan->off_ovel, displacement,
                                sizeof(float) * plan->cfg.n_dim * (size_t)plan->obs_total,
                                hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  plan->moving = plan->obs_total > 0;
  return SF_OK;
}

int sf_smoothness(const sf_plan_t* plan, const void* workspace, const float* xi,
                  float t_final, float* cost, void* stream) {
  g_detail.clear();
  if (!plan) return fail(SF_ERR_INVALID_ARG, "plan is NULL");
  if (workspace != plan->ws)
    return fail(SF_ERR_INVALID_ARG, "workspace differs from the one bound at sf_setup");
  if (plan->cfg.n_dim == 3) return fail(SF_ERR_INVALID_ARG, "sf_smoothness covers n_dim = 2");
  if (!xi || !cost) return fail(SF_ERR_INVALID_ARG, "xi or cost is NULL");
  if (!(t_final > 0.f) || !std::isfinite(t_final))
    return fail(SF_ERR_INVALID_ARG, "t_final must be positive and finite");
  const double tf2 = (double)t_final * (double)t_final;
  const float inv_tf4 = (float)(1.0 / (tf2 * tf2));
  hipStream_t s = static_cast<hipStream_t>(stream);
  SF_HIP_CHECK(sf::launch_smoothness(plan->at<sf::ProbDesc>(plan->off_desc), plan->B,
                                     plan->at<float>(plan->off_Wdd), xi, plan->cfg.n_coef,
                                     plan->cfg.n_steps, inv_tf4, cost, s));
  return SF_OK;
}

int sf_rank_residual(const float* residual, int32_t n_candidates, int32_t k, int32_t* idx,
                     void* stream) {
  g_detail.clear();
  if (!residual || !idx) return fail(SF_ERR_INVALID_ARG, "residual or idx is NULL");
  if (n_candidates < 1 || n_candidates > sf::kSelectMaxBatch)
    return fail(SF_ERR_SHAPE, "n_candidates must be in 1.." + std::to_string(sf::kSelectMaxBatch));
  if (k < 1 || k > n_candidates) return fail(SF_ERR_INVALID_ARG, "k must be in 1..n_candidates");
  SF_HIP_CHECK(sf::launch_topk(residual, n_candidates, k, idx, static_cast<hipStream_t>(stream)));
  return SF_OK;
}

int sf_select_best(const float* residual, const float* cost, int32_t n_candidates, float tol,
                   int32_t* idx, void* stream) {
  g_detail.clear();
  if (!residual || !cost || !idx) return fail(SF_ERR_INVALID_ARG, "residual, cost or idx is NULL");
  if (n_candidates < 1 || n_candidates > sf::kSelectMaxBatch)
    return fail(SF_ERR_SHAPE, "n_candidates must be in 1.." + std::to_string(sf::kSelectMaxBatch));
  if (!(tol >= 0.f) || !std::isfinite(tol))
    return fail(SF_ERR_INVALID_ARG, "tol must be finite and non-negative");
  SF_HIP_CHECK(sf::launch_best(residual, cost, n_candidates, tol, idx,
                               static_cast<hipStream_t>(stream)));
  return SF_OK;
}

int sf_gather_blocks(const float* src, int32_t n_blocks, const int32_t* idx, int32_t k,
                     int32_t block_floats, float* dst, void* stream) {
  g_detail.clear();
  if (!src || !idx || !dst) return fail(SF_ERR_INVALID_ARG, "src, idx or dst is NULL");
  if (n_blocks < 1 || k < 1 || block_floats < 1 || k > 65535)
    return fail(SF_ERR_INVALID_ARG, "n_blocks, k and block_floats must be positive (k <= 65535)");
  SF_HIP_CHECK(sf::launch_gather(src, idx, k, block_floats, n_blocks, dst,
                                 static_cast<hipStream_t>(stream)));
  return SF_OK;
}

}  // extern "C"
