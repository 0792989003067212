// Host side of the C ABI declared in include/mppi_jump.h: configuration
// validation, workspace layout, kernel dispatch.  See the header for the
// contract of every entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <utility>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/mppi_jump.h"
#include "kernels.hpp"

using namespace mppi;

namespace {

// detail of the calling thread's last failure (a fixed buffer: reporting an
// error allocates nothing)
thread_local char g_last_error[512];

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
  return code;
}

int ok() {
  g_last_error[0] = '\0';
  return MPPI_OK;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(MPPI_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_CHECK(name)                                                                   \
  do {                                                                                       \
    hipError_t e_ = hipGetLastError();                                                       \
    if (e_ != hipSuccess) return fail(MPPI_EDEVICE, "launch of %s: %s", name, hipGetErrorString(e_)); \
  } while (0)

constexpr uint64_t kTwo32 = 1ull << 32;

bool dims_of(int32_t dyn, int& n, int& m, int& q) {
  switch (dyn) {
    case MPPI_DYN_LINEAR: n = 2; m = 1; q = 1; return true;
    case MPPI_DYN_CARTPOLE: n = 4; m = 1; q = 1; return true;
    case MPPI_DYN_QUADROTOR: n = 12; m = 4; q = 3; return true;
    default: return false;
  }
}

// Count-law table of at most MPPI_JUMP_MAX_LEVELS entries, held in place
// (no heap allocation, so that an entry point can run without allocating).
struct Thresholds {
  uint64_t v[MPPI_JUMP_MAX_LEVELS];
  int n = 0;
  void clear() { n = 0; }
  void push_back(uint64_t x) {
    if (n < MPPI_JUMP_MAX_LEVELS) v[n++] = x;
  }
  size_t size() const { return (size_t)n; }
  uint64_t operator[](size_t i) const { return v[i]; }
};

// Inversion thresholds of the count law with mean a = nu * dt, computed in
// fp64: Poisson CDF by the recurrence p_j = p_{j-1} a / j, or the zero-one
// law F(0) = 1 - a.  theta_j = floor(F(j) 2^32); the first level reaching
// 2^32 - 1 closes the table at 2^32.  Returns false if the law needs more
// than MPPI_JUMP_MAX_LEVELS levels.
bool count_thresholds(double a, int law, Thresholds& th) {
  th.clear();
  if (law == MPPI_COUNT_ZERO_ONE) {
    if (a > 1.0) return false;
    double f = std::floor((1.0 - a) * (double)kTwo32);
    uint64_t t0 = f >= (double)kTwo32 ? kTwo32 : (uint64_t)f;
    if (t0 < kTwo32) th.push_back(t0);
    th.push_back(kTwo32);
    return true;
  }
  double p = std::exp(-a), F = p;
  for (int j = 0; j < MPPI_JUMP_MAX_LEVELS; ++j) {
    if (j > 0) {
      p = p * a / j;
      F = F + p;
    }
    const double f = std::floor(F * (double)kTwo32);
    if (f >= (double)(kTwo32 - 1)) {
      th.push_back(kTwo32);
      return true;
    }
    th.push_back((uint64_t)f);
  }
  return false;
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.f; }

int validate(const mppi_jump_config* c, int& n, int& m, int& q, Thresholds& th) {
  if (!c) return fail(MPPI_EINVAL, "config is NULL");
  if (c->abi_version != MPPI_JUMP_ABI_VERSION)
    return fail(MPPI_EINVAL, "abi_version %d != %d", c->abi_version, MPPI_JUMP_ABI_VERSION);
  if (!dims_of(c->dynamics, n, m, q)) return fail(MPPI_EINVAL, "unknown dynamics %d", c->dynamics);
  if (c->K < 1 || c->K > MPPI_JUMP_MAX_K) return fail(MPPI_EINVAL, "K=%d out of [1, 2^24]", c->K);
  if (c->T < 1 || c->T > MPPI_JUMP_MAX_T) return fail(MPPI_EINVAL, "T=%d out of [1, 4096]", c->T);
  if (!finite_pos(c->dt)) return fail(MPPI_EINVAL, "dt must be finite and > 0");
  if (!finite_pos(c->lambda)) return fail(MPPI_EINVAL, "lambda must be finite and > 0");
  if (!finite_pos(c->c)) return fail(MPPI_EINVAL, "c must be finite and > 0");
  if (!std::isfinite(c->alpha)) return fail(MPPI_EINVAL, "alpha must be finite");
  if (!(std::isfinite(c->nu) && c->nu >= 0.f)) return fail(MPPI_EINVAL, "nu must be finite and >= 0");
  if (c->count_law != MPPI_COUNT_POISSON && c->count_law != MPPI_COUNT_ZERO_ONE)
    return fail(MPPI_EINVAL, "unknown count_law %d", c->count_law);
  if (c->mark_law != MPPI_MARK_NORMAL) return fail(MPPI_EINVAL, "unknown mark_law %d", c->mark_law);
  if (c->cost_form != MPPI_COST_IT && c->cost_form != MPPI_COST_SO)
    return fail(MPPI_EINVAL, "unknown cost_form %d", c->cost_form);
  if (c->debug_dump != 0 && c->debug_dump != 1) return fail(MPPI_EINVAL, "debug_dump must be 0 or 1");
  if (c->schedule < MPPI_SCHED_AUTO || c->schedule > MPPI_SCHED_WAVE_SPECIALISED)
    return fail(MPPI_EINVAL, "unknown schedule %d", c->schedule);
  if (c->full_sigma != 0 && c->full_sigma != 1) return fail(MPPI_EINVAL, "full_sigma must be 0 or 1");
  if (c->sample_offset < 0 || (int64_t)c->sample_offset + c->K > (int64_t)1 << 31)
    return fail(MPPI_EINVAL, "sample_offset must be >= 0 with sample_offset + K <= 2^31");
  if (c->full_sigma) {
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        const float v = c->sigma_L[4 * i + j];
        if (!std::isfinite(v)) return fail(MPPI_EINVAL, "sigma_L[%d][%d] must be finite", i, j);
        if (j > i && v != 0.f) return fail(MPPI_EINVAL, "sigma_L must be lower triangular");
        if (j == i && !(v > 0.f)) return fail(MPPI_EINVAL, "sigma_L[%d][%d] must be > 0", i, i);
      }
  } else {
    for (int j = 0; j < m; ++j)
      if (!(std::isfinite(c->sigma[j]) && c->sigma[j] >= 0.f))
        return fail(MPPI_EINVAL, "sigma[%d] must be finite and >= 0", j);
  }
  for (int i = 0; i < q; ++i)
    if (!(std::isfinite(c->sigma_J[i]) && c->sigma_J[i] >= 0.f))
      return fail(MPPI_EINVAL, "sigma_J[%d] must be finite and >= 0", i);
  for (int j = 0; j < m; ++j)
    if (!std::isfinite(c->u_init[j]) || !std::isfinite(c->R[j]))
      return fail(MPPI_EINVAL, "u_init / R must be finite");
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(c->Q[i]) || !std::isfinite(c->Qf[i]) || !std::isfinite(c->x_goal[i]))
      return fail(MPPI_EINVAL, "Q / Qf / x_goal must be finite");
  if (!std::isfinite(c->crash_penalty)) return fail(MPPI_EINVAL, "crash_penalty must be finite");
  if (c->controller_id >= (1ull << 24)) return fail(MPPI_EINVAL, "controller_id must be < 2^24");
  if (c->start_iteration >= kTwo32) return fail(MPPI_EINVAL, "start_iteration must be < 2^32");
  const float* P = c->params;
  if (c->dynamics == MPPI_DYN_CARTPOLE) {
    if (!finite_pos(P[0]) || !finite_pos(P[1]) || !finite_pos(P[2]) || !std::isfinite(P[3]))
      return fail(MPPI_EINVAL, "cartpole params need m_cart, m_pole, half_length > 0, finite g");
  } else if (c->dynamics == MPPI_DYN_QUADROTOR) {
    for (int i = 0; i < 5; ++i)
      if (!finite_pos(P[i])) return fail(MPPI_EINVAL, "quadrotor mass, J, arm must be > 0");
    if (!std::isfinite(P[5]) || !std::isfinite(P[6]) || !std::isfinite(P[8]))
      return fail(MPPI_EINVAL, "quadrotor k_yaw, g, z_min must be finite");
    if (!(P[7] > 0.f && P[7] < 1.5f)) return fail(MPPI_EINVAL, "quadrotor tilt_max must be in (0, 1.5)");
  }
  const double a = (double)c->nu * (double)c->dt;
  if (!count_thresholds(a, c->count_law, th))
    return fail(MPPI_EINVAL, "jump mean nu*dt=%g does not fit the count law table", a);
  return MPPI_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  int R, Ks, nwg, nch, chunk;
  bool ws;     // wave-specialised schedule (64 samples per workgroup)
  int spw;     // samples per rollout workgroup
  bool fused;     // the update in the rollout's epilogue (kFusedWgWs / kFusedWgLane)
  // beyond that (no debug dumps): tile sums published, the update by
  // partial_update_kernel
  bool deferred;
  bool eps_lds;  // wave-specialised iterations keep the perturbations on chip
  size_t U, eps, S, E, part, scale, upart, wpart, stats, counters, W, zD, N, zJ, total;
};

Layout make_layout(const mppi_jump_config* c, int m, int q) {
  Layout L{};
  const size_t K = (size_t)c->K, T = (size_t)c->T;
  L.R = (int)(T * m);
  // AUTO: the wave-specialised schedule up to the measured crossover (T=100,
  // us per iteration, lane against wave-specialised: quadrotor K=98304
  // 189.1 / 182.4, K=114688 193.5 / 216.4; cartpole K=131072 99.0 / 92.9)
  const int ws_max_k = m > 1 ? MPPI_JUMP_WS_MAX_K_MULTI : MPPI_JUMP_WS_MAX_K;
  L.ws = c->schedule == MPPI_SCHED_WAVE_SPECIALISED ||
         (c->schedule == MPPI_SCHED_AUTO && c->K <= ws_max_k);
  L.spw = L.ws ? kWsSamples : kBlock;
  L.Ks = (int)align_up(K, kBlock);  // rows padded to whole rollout workgroups
  L.nwg = (int)((K + L.spw - 1) / L.spw);
  int nch = (int)((K + 1023) / 1024);
  if (nch > 64) nch = 64;
  L.chunk = (int)align_up((K + nch - 1) / nch, kBlock);
  L.nch = (int)((K + L.chunk - 1) / L.chunk);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  L.U = take((size_t)L.R * 4);
  L.eps = take((size_t)L.R * L.Ks * 4);
  L.S = take(K * 8);
  L.E = take(K * 8);
  L.part = take((size_t)L.nwg * sizeof(WgPartial));
  L.scale = take((size_t)L.nwg * 8);
  L.upart = take((size_t)L.R * L.nch * 8);
  L.fused = L.nwg <= (L.ws ? kFusedWgWs : kFusedWgLane);
  L.deferred = !L.fused && !c->debug_dump;
  const int per_cu = L.fused ? 1 : 2;
  bool fits = false;
  switch (c->dynamics) {
    case MPPI_DYN_LINEAR: fits = ws_eps_fits<MPPI_DYN_LINEAR>(L.R, per_cu); break;
    case MPPI_DYN_CARTPOLE: fits = ws_eps_fits<MPPI_DYN_CARTPOLE>(L.R, per_cu); break;
    default: fits = ws_eps_fits<MPPI_DYN_QUADROTOR>(L.R, per_cu); break;
  }
  L.eps_lds = L.ws && (L.fused || L.deferred) && !c->debug_dump && fits;
  L.wpart = take(L.fused || L.deferred ? (size_t)L.nwg * L.R * 8 : 0);
  L.stats = take(sizeof(mppi_jump_stats));
  L.counters = take((size_t)counter_count(L.R) * sizeof(uint32_t));
  L.W = take(K * 8);
  if (c->debug_dump) {
    L.zD = take(K * T * m * 4);
    L.N = take(K * T * 4);
    L.zJ = take(K * T * q * 4);
  }
  L.total = off;
  return L;
}

DevParams make_params(const mppi_jump_config* c, int n, int m, int q, const Layout& L,
                      const Thresholds& th) {
  DevParams p;
  std::memset(&p, 0, sizeof p);
  p.K = c->K;
  p.T = c->T;
  p.Ks = L.Ks;
  p.wg_shift = L.ws ? 6 : 8;
  p.k0 = (uint32_t)c->sample_offset;
  p.key0 = (uint32_t)(c->seed & 0xFFFFFFFFull);
  p.key1 = (uint32_t)(c->seed >> 32);
  p.ctr3 = (uint32_t)(c->controller_id << 8);
  p.cost_form = c->cost_form;
  p.dt = c->dt;
  p.lam = c->lambda;
  p.lam_d = (double)c->lambda;
  p.alpha = c->alpha;
  p.pen = c->crash_penalty;
  const double lam = c->lambda, cc = c->c;
  // a one-channel covariance L L^T is the diagonal form with sigma = L00
  float sig_in[4] = {c->sigma[0], c->sigma[1], c->sigma[2], c->sigma[3]};
  if (c->full_sigma && m == 1) sig_in[0] = c->sigma_L[0];
  if (c->full_sigma && m > 1) {
    // Sigma_D = L L^T: eps_D = L z, and the IS terms take Sigma_D^-1 =
    // L^-T L^-1 (forward substitution in fp64), pre-scaled by lambda c and
    // lambda (c - 1) / 2
    double Li[4][4] = {};
    for (int i = 0; i < m; ++i) {
      Li[i][i] = 1.0 / (double)c->sigma_L[4 * i + i];
      for (int j = 0; j < i; ++j) {
        double acc = 0.0;
        for (int k = j; k < i; ++k) acc += (double)c->sigma_L[4 * i + k] * Li[k][j];
        Li[i][j] = -acc / (double)c->sigma_L[4 * i + i];
      }
    }
    p.full = 1;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double P = 0.0;
        for (int k = 0; k < m; ++k) P += Li[k][i] * Li[k][j];
        p.L[4 * i + j] = c->sigma_L[4 * i + j];
        p.Pc[4 * i + j] = (float)(lam * cc * P);
        p.Pv[4 * i + j] = (float)(0.5 * lam * (cc - 1.0) * P);
      }
  }
  for (int j = 0; j < m; ++j) {
    p.sigma[j] = sig_in[j];
    const double s2 = (double)sig_in[j] * (double)sig_in[j];
    p.isc[j] = s2 > 0 ? (float)(lam * cc / s2) : 0.f;
    p.isv[j] = s2 > 0 ? (float)(0.5 * lam * (cc - 1.0) / s2) : 0.f;
    p.halfR[j] = 0.5f * c->R[j];
  }
  for (int i = 0; i < q; ++i) p.sigJ[i] = c->sigma_J[i];
  for (int i = 0; i < n; ++i) {
    p.Q[i] = c->Q[i];
    p.Qf[i] = c->Qf[i];
    p.goal[i] = c->x_goal[i];
  }
  const float* P = c->params;
  if (c->dynamics == MPPI_DYN_CARTPOLE) {
    const double mc = P[0], mp = P[1], l = P[2], g = P[3];
    p.mc.c[0] = (float)g;
    p.mc.c[1] = (float)(1.0 / (mc + mp));
    p.mc.c[2] = (float)(mp * l);
    p.mc.c[3] = (float)(mp * l / (mc + mp));
    p.mc.c[4] = (float)(4.0 / 3.0 * l);
  } else if (c->dynamics == MPPI_DYN_QUADROTOR) {
    const double mass = P[0], Jx = P[1], Jy = P[2], Jz = P[3];
    p.mc.c[0] = (float)(1.0 / mass);
    p.mc.c[1] = (float)(1.0 / Jx);
    p.mc.c[2] = (float)(1.0 / Jy);
    p.mc.c[3] = (float)(1.0 / Jz);
    p.mc.c[4] = (float)(Jz - Jy);
    p.mc.c[5] = (float)(Jx - Jz);
    p.mc.c[6] = (float)(Jy - Jx);
    p.mc.c[7] = P[4];
    p.mc.c[8] = P[5];
    p.mc.c[9] = P[6];
    p.mc.c[10] = P[7];
    p.mc.c[11] = P[8];
  }
  p.n_th = 0;
  for (size_t j = 0; j < th.size() && j < MPPI_JUMP_MAX_LEVELS; ++j)
    if (th[j] < kTwo32) p.th[p.n_th++] = (uint32_t)th[j];
  return p;
}

}  // namespace

struct mppi_jump_ctx {
  mppi_jump_config cfg;
  int n, m, q;
  Layout L;
  DevParams p;
  Buffers b;
  double* W;
  uint64_t th64[MPPI_JUMP_MAX_LEVELS];
  uint64_t host_iteration;  // iterations enqueued so far (range check only)
  bool eps_stored = true;   // the last rollout enqueued stored its perturbations
  bool profiling = false;
  struct Bracket {
    hipEvent_t e0, e1;
    int launches, iterations;
  };
  std::vector<Bracket> events;  // one pair per bracketed span of rollout launches
  size_t events_used = 0;
};

namespace {

// Context fields of a validated configuration over a workspace at `base`
// (laid out by L).
void bind_context(mppi_jump_ctx* ctx, const mppi_jump_config* cfg, int n, int m, int q,
                  const Layout& L, const Thresholds& th, char* base) {
  ctx->cfg = *cfg;
  ctx->n = n;
  ctx->m = m;
  ctx->q = q;
  ctx->L = L;
  ctx->p = make_params(cfg, n, m, q, L, th);
  for (int j = 0; j < MPPI_JUMP_MAX_LEVELS; ++j) ctx->th64[j] = j < (int)th.size() ? th[j] : kTwo32;
  Buffers& b = ctx->b;
  b.U = reinterpret_cast<float*>(base + L.U);
  b.eps = reinterpret_cast<float*>(base + L.eps);
  b.S = reinterpret_cast<double*>(base + L.S);
  b.E = reinterpret_cast<double*>(base + L.E);
  b.part = reinterpret_cast<WgPartial*>(base + L.part);
  b.scale = reinterpret_cast<double*>(base + L.scale);
  b.upart = reinterpret_cast<double*>(base + L.upart);
  b.wpart = L.fused || L.deferred ? reinterpret_cast<double*>(base + L.wpart) : nullptr;
  b.stats = reinterpret_cast<mppi_jump_stats*>(base + L.stats);
  b.counters = reinterpret_cast<uint32_t*>(base + L.counters);
  ctx->W = reinterpret_cast<double*>(base + L.W);
  b.dbg_zD = cfg->debug_dump ? reinterpret_cast<float*>(base + L.zD) : nullptr;
  b.dbg_N = cfg->debug_dump ? reinterpret_cast<int32_t*>(base + L.N) : nullptr;
  b.dbg_zJ = cfg->debug_dump ? reinterpret_cast<float*>(base + L.zJ) : nullptr;
  ctx->host_iteration = cfg->start_iteration;
}

// A wave-specialised kernel's dynamic LDS (ring, the perturbation tile when
// on chip, U) can exceed the default launch limit, so each kernel's limit is
// raised once, to the compute unit's LDS less the static part bounded by
// kWsStaticLds; that bound is checked then too.
int raise_ws_lds_limit(const void* kern) {
  const hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(kLdsBytes - kWsStaticLds));
  if (e != hipSuccess)
    return fail(MPPI_EDEVICE, "raising the LDS limit of rollout_ws_kernel: %s",
                hipGetErrorString(e));
  hipFuncAttributes a{};
  HIP_TRY(hipFuncGetAttributes(&a, kern));
  if (a.sharedSizeBytes > kWsStaticLds)
    return fail(MPPI_EDEVICE, "rollout_ws_kernel holds %zu bytes of static LDS, above %zu",
                a.sharedSizeBytes, kWsStaticLds);
  return MPPI_OK;
}

template <int DYN, bool JUMPS, bool DEBUG, int FORM, bool FUSED, bool FULL, bool EPS_LDS,
          bool DEFER = false>
int launch_ws(mppi_jump_ctx* ctx, const float* x0, hipStream_t s, const ShiftArgs& sh) {
  const auto kern = rollout_ws_kernel<DYN, JUMPS, DEBUG, FORM, FUSED, FULL, EPS_LDS, DEFER>;
  static const int raised = raise_ws_lds_limit(reinterpret_cast<const void*>(kern));
  if (raised != MPPI_OK) return fail(raised, "%s", "the LDS limit of rollout_ws_kernel");
  const size_t lds = EPS_LDS ? ws_eps_lds_bytes<DYN>(ctx->L.R) : ws_lds_bytes<DYN>(ctx->L.R);
  kern<<<dim3(ctx->L.nwg), dim3(64 * WsWaves<DYN>::W), lds, s>>>(ctx->p, ctx->b, x0, ctx->b.U,
                                                                 ctx->L.R, sh);
  LAUNCH_CHECK("rollout_ws_kernel");
  return MPPI_OK;
}

template <int DYN, bool JUMPS, bool DEBUG, int FORM, bool FUSED, bool FULL>
int launch_rollout_t(mppi_jump_ctx* ctx, const float* x0, hipStream_t s, const ShiftArgs& sh) {
  ctx->eps_stored = !(FUSED && !DEBUG && ctx->L.eps_lds);
  if constexpr (FUSED && !DEBUG) {
    if (ctx->L.deferred && ctx->L.ws) {
      if (ctx->L.eps_lds)
        return launch_ws<DYN, JUMPS, DEBUG, FORM, FUSED, FULL, true, true>(ctx, x0, s, sh);
      return launch_ws<DYN, JUMPS, DEBUG, FORM, FUSED, FULL, false, true>(ctx, x0, s, sh);
    }
    if (ctx->L.eps_lds) return launch_ws<DYN, JUMPS, DEBUG, FORM, FUSED, FULL, true>(ctx, x0, s, sh);
    if (ctx->L.deferred) {
      rollout_kernel<DYN, JUMPS, DEBUG, FORM, FUSED, FULL, true>
          <<<dim3(ctx->L.nwg), dim3(kBlock), 0, s>>>(ctx->p, ctx->b, x0, ctx->b.U, ctx->L.R, sh);
      LAUNCH_CHECK("rollout_kernel");
      return MPPI_OK;
    }
  }
  if (ctx->L.ws) {
    return launch_ws<DYN, JUMPS, DEBUG, FORM, FUSED, FULL, false>(ctx, x0, s, sh);
  } else {
    rollout_kernel<DYN, JUMPS, DEBUG, FORM, FUSED, FULL>
        <<<dim3(ctx->L.nwg), dim3(kBlock), 0, s>>>(ctx->p, ctx->b, x0, ctx->b.U, ctx->L.R, sh);
    LAUNCH_CHECK("rollout_kernel");
  }
  return MPPI_OK;
}

template <int DYN, bool JUMPS, bool DEBUG, bool FULL>
int launch_rollout_form(mppi_jump_ctx* ctx, const float* x0, hipStream_t s, bool fused,
                        const ShiftArgs& sh) {
  const bool it = ctx->cfg.cost_form == MPPI_COST_IT;
  if (fused)
    return it ? launch_rollout_t<DYN, JUMPS, DEBUG, MPPI_COST_IT, true, FULL>(ctx, x0, s, sh)
              : launch_rollout_t<DYN, JUMPS, DEBUG, MPPI_COST_SO, true, FULL>(ctx, x0, s, sh);
  return it ? launch_rollout_t<DYN, JUMPS, DEBUG, MPPI_COST_IT, false, FULL>(ctx, x0, s, sh)
            : launch_rollout_t<DYN, JUMPS, DEBUG, MPPI_COST_SO, false, FULL>(ctx, x0, s, sh);
}

template <int DYN, bool FULL>
int launch_rollout_full(mppi_jump_ctx* ctx, const float* x0, hipStream_t s, bool fused,
                        const ShiftArgs& sh) {
  const bool jumps = ctx->p.n_th > 0, dbg = ctx->cfg.debug_dump != 0;
  if (jumps)
    return dbg ? launch_rollout_form<DYN, true, true, FULL>(ctx, x0, s, fused, sh)
               : launch_rollout_form<DYN, true, false, FULL>(ctx, x0, s, fused, sh);
  return dbg ? launch_rollout_form<DYN, false, true, FULL>(ctx, x0, s, fused, sh)
             : launch_rollout_form<DYN, false, false, FULL>(ctx, x0, s, fused, sh);
}

// The full-covariance variants exist for the multi-channel model only (a
// one-channel covariance is passed as its diagonal form).
template <int DYN>
int launch_rollout_dyn(mppi_jump_ctx* ctx, const float* x0, hipStream_t s, bool fused,
                       const ShiftArgs& sh) {
  if constexpr (Model<DYN>::M > 1) {
    if (ctx->p.full) return launch_rollout_full<DYN, true>(ctx, x0, s, fused, sh);
  }
  return launch_rollout_full<DYN, false>(ctx, x0, s, fused, sh);
}

// Timing brackets: an event pair around a span of back-to-back rollout
// launches (one launch, or all fused launches of one entry-point call).
int bracket_begin(mppi_jump_ctx* ctx, hipStream_t s) {
  if (!ctx->profiling) return MPPI_OK;
  if (ctx->events_used >= 4096) return fail(MPPI_EINVAL, "profiling buffer full (4096 spans)");
  if (ctx->events_used == ctx->events.size()) {
    mppi_jump_ctx::Bracket br{nullptr, nullptr, 0};
    HIP_TRY(hipEventCreate(&br.e0));
    HIP_TRY(hipEventCreate(&br.e1));
    ctx->events.push_back(br);
  }
  HIP_TRY(hipEventRecord(ctx->events[ctx->events_used].e0, s));
  return MPPI_OK;
}

int bracket_end(mppi_jump_ctx* ctx, hipStream_t s, int launches, int iterations) {
  if (!ctx->profiling) return MPPI_OK;
  HIP_TRY(hipEventRecord(ctx->events[ctx->events_used].e1, s));
  ctx->events[ctx->events_used].launches = launches;
  ctx->events[ctx->events_used].iterations = iterations;
  ctx->events_used++;
  return MPPI_OK;
}

// own_bracket: time this launch on its own (else the caller brackets a span)
int launch_rollout(mppi_jump_ctx* ctx, const float* x0, hipStream_t s, bool fused,
                   const ShiftArgs& sh = ShiftArgs{}, bool own_bracket = true) {
  if (own_bracket) {
    const int rb = bracket_begin(ctx, s);
    if (rb != MPPI_OK) return rb;
  }
  int rc;
  switch (ctx->cfg.dynamics) {
    case MPPI_DYN_LINEAR: rc = launch_rollout_dyn<MPPI_DYN_LINEAR>(ctx, x0, s, fused, sh); break;
    case MPPI_DYN_CARTPOLE: rc = launch_rollout_dyn<MPPI_DYN_CARTPOLE>(ctx, x0, s, fused, sh); break;
    default: rc = launch_rollout_dyn<MPPI_DYN_QUADROTOR>(ctx, x0, s, fused, sh); break;
  }
  if (rc != MPPI_OK) return rc;
  return own_bracket ? bracket_end(ctx, s, 1, 1) : MPPI_OK;
}

int launch_update(mppi_jump_ctx* ctx, hipStream_t s) {
  const dim3 grid((ctx->L.R + kRowsPerWg - 1) / kRowsPerWg, ctx->L.nch), block(kBlock);
  update_kernel<<<grid, block, 0, s>>>(ctx->p, ctx->b, ctx->L.R, ctx->L.nch, ctx->L.chunk);
  LAUNCH_CHECK("update_kernel");
  return MPPI_OK;
}

// The update after a deferred-form rollout: the L.nch chunks of workgroup
// partials (upart holds R x L.nch chunk sums) over row blocks of kPartRows.
int launch_partial_update(mppi_jump_ctx* ctx, hipStream_t s) {
  const int nch = ctx->L.nch, nwg = ctx->L.nwg;
  if (nch < 1 || nch > kPartMaxChunks)
    return fail(MPPI_EDEVICE, "deferred update over %d chunks (1..%d)", nch, kPartMaxChunks);
  const dim3 grid((ctx->L.R + kPartRows - 1) / kPartRows, nch), block(kBlock);
  partial_update_kernel<<<grid, block, 0, s>>>(ctx->p, ctx->b, ctx->L.R, nwg, nch,
                                               (nwg + nch - 1) / nch);
  LAUNCH_CHECK("partial_update_kernel");
  return MPPI_OK;
}

float4 u_init4(const mppi_jump_config& c) {
  return make_float4(c.u_init[0], c.u_init[1], c.u_init[2], c.u_init[3]);
}

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(MPPI_EDEVICE, "host allocation failed");
  } catch (...) {
    return fail(MPPI_EDEVICE, "unexpected exception");
  }
}

}  // namespace

extern "C" {

int mppi_jump_abi_version(void) { return MPPI_JUMP_ABI_VERSION; }

int mppi_jump_dims(int32_t dynamics, int32_t* n, int32_t* m, int32_t* q) {
  int nn, mm, qq;
  if (!n || !m || !q) return fail(MPPI_EINVAL, "NULL output");
  if (!dims_of(dynamics, nn, mm, qq)) return fail(MPPI_EINVAL, "unknown dynamics %d", dynamics);
  *n = nn;
  *m = mm;
  *q = qq;
  return ok();
}

int mppi_jump_workspace_bytes(const mppi_jump_config* cfg, size_t* bytes) {
  return guarded([&]() -> int {
    if (!bytes) return fail(MPPI_EINVAL, "bytes is NULL");
    int n, m, q;
    Thresholds th;
    const int rc = validate(cfg, n, m, q, th);
    if (rc != MPPI_OK) return rc;
    *bytes = make_layout(cfg, m, q).total;
    return ok();
  });
}

int mppi_jump_count_thresholds(const mppi_jump_config* cfg, uint64_t* out) {
  return guarded([&]() -> int {
    if (!out) return fail(MPPI_EINVAL, "out is NULL");
    int n, m, q;
    Thresholds th;
    const int rc = validate(cfg, n, m, q, th);
    if (rc != MPPI_OK) return rc;
    for (int j = 0; j < MPPI_JUMP_MAX_LEVELS; ++j) out[j] = j < (int)th.size() ? th[j] : kTwo32;
    return ok();
  });
}

int mppi_jump_init(const mppi_jump_config* cfg, void* d_workspace, size_t ws_bytes,
                   const float* d_U0, void* stream, mppi_jump_ctx** out) {
  return guarded([&]() -> int {
    if (!out) return fail(MPPI_EINVAL, "out is NULL");
    *out = nullptr;
    int n, m, q;
    Thresholds th;
    int rc = validate(cfg, n, m, q, th);
    if (rc != MPPI_OK) return rc;
    const Layout L = make_layout(cfg, m, q);
    if (!d_workspace || ((uintptr_t)d_workspace & 255u))
      return fail(MPPI_EWORKSPACE, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < L.total)
      return fail(MPPI_EWORKSPACE, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
    auto* ctx = new mppi_jump_ctx();
    bind_context(ctx, cfg, n, m, q, L, th, static_cast<char*>(d_workspace));
    const Buffers& b = ctx->b;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int threads = 256, blocks = (L.R + threads - 1) / threads;
    init_kernel<<<blocks, threads, 0, s>>>(b, d_U0, L.R, m, u_init4(*cfg), cfg->start_iteration);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      delete ctx;
      return fail(MPPI_EDEVICE, "launch of init_kernel: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return ok();
  });
}

int mppi_jump_rollout(mppi_jump_ctx* ctx, const float* d_x0, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !d_x0) return fail(MPPI_EINVAL, "NULL context or state");
    const int rc = launch_rollout(ctx, d_x0, static_cast<hipStream_t>(stream), false);
    return rc == MPPI_OK ? ok() : rc;
  });
}

int mppi_jump_update(mppi_jump_ctx* ctx, void* stream) {
  return guarded([&]() -> int {
    if (!ctx) return fail(MPPI_EINVAL, "NULL context");
    if (ctx->host_iteration + 1 > kTwo32) return fail(MPPI_EINVAL, "iteration counter exhausted");
    const int rc = launch_update(ctx, static_cast<hipStream_t>(stream));
    if (rc != MPPI_OK) return rc;
    ctx->host_iteration += 1;
    return ok();
  });
}

int mppi_jump_step(mppi_jump_ctx* ctx, const float* d_x0, int32_t iters, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !d_x0) return fail(MPPI_EINVAL, "NULL context or state");
    if (iters < 1) return fail(MPPI_EINVAL, "iters=%d < 1", iters);
    if (ctx->host_iteration + (uint64_t)iters > kTwo32)
      return fail(MPPI_EINVAL, "iteration counter would pass 2^32");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const bool span = ctx->L.fused;  // fused launches run back to back: one bracket
    if (span) {
      const int rb = bracket_begin(ctx, s);
      if (rb != MPPI_OK) return rb;
    }
    for (int i = 0; i < iters; ++i) {
      int rc = launch_rollout(ctx, d_x0, s, ctx->L.fused || ctx->L.deferred, ShiftArgs{}, !span);
      if (rc != MPPI_OK) return rc;
      if (!ctx->L.fused) {
        rc = ctx->L.deferred ? launch_partial_update(ctx, s) : launch_update(ctx, s);
        if (rc != MPPI_OK) return rc;
      }
      ctx->host_iteration += 1;
    }
    if (span) {
      const int rb = bracket_end(ctx, s, iters, iters);
      if (rb != MPPI_OK) return rb;
    }
    return ok();
  });
}

}  // extern "C"

namespace {

// Body of mppi_jump_control_step on a checked context.
int enqueue_control_step(mppi_jump_ctx* ctx, const float* d_x0, int32_t iters, float* d_u0_out,
                         void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (!ctx->L.fused) {
    int rc = mppi_jump_step(ctx, d_x0, iters, stream);
    if (rc != MPPI_OK) return rc;
    return mppi_jump_shift(ctx, d_u0_out, stream);
  }
  int rc = bracket_begin(ctx, s);
  if (rc != MPPI_OK) return rc;
  for (int i = 0; i < iters; ++i) {
    ShiftArgs sh{};
    if (i == iters - 1) {
      sh.on = 1;
      sh.u0_out = d_u0_out;
      sh.m = ctx->m;
      sh.u_init = u_init4(ctx->cfg);
    }
    rc = launch_rollout(ctx, d_x0, s, true, sh, false);
    if (rc != MPPI_OK) return rc;
    ctx->host_iteration += 1;
  }
  rc = bracket_end(ctx, s, iters, iters);
  return rc == MPPI_OK ? ok() : rc;
}

// Scratch of mppi_jump_control_step_static: a library-owned device array,
// one copy per GPU, held until the process ends.  In host code its name
// stands for the host-side shadow, not a device address: the device address
// is resolved once per device by hipGetSymbolAddress and only that address
// is used.
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[MPPI_JUMP_STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved on the first
// call per device, with that device current).
int static_scratch(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MPPI_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255u)) return fail(MPPI_EDEVICE, "static scratch address unusable");
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return MPPI_OK;
}

}  // namespace

extern "C" {

int mppi_jump_control_step(mppi_jump_ctx* ctx, const float* d_x0, int32_t iters, float* d_u0_out,
                           void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !d_x0) return fail(MPPI_EINVAL, "NULL context or state");
    if (iters < 1) return fail(MPPI_EINVAL, "iters=%d < 1", iters);
    if (ctx->host_iteration + (uint64_t)iters > kTwo32)
      return fail(MPPI_EINVAL, "iteration counter would pass 2^32");
    return enqueue_control_step(ctx, d_x0, iters, d_u0_out, stream);
  });
}

int mppi_jump_control_step_static(const mppi_jump_config* cfg, float* d_U, const float* d_x0,
                                  int32_t iters, float* d_u0_out, void* stream) {
  return guarded([&]() -> int {
    if (!d_U || !d_x0) return fail(MPPI_EINVAL, "NULL control sequence or state");
    if (iters < 1) return fail(MPPI_EINVAL, "iters=%d < 1", iters);
    int n, m, q;
    Thresholds th;
    int rc = validate(cfg, n, m, q, th);
    if (rc != MPPI_OK) return rc;
    if (cfg->debug_dump) return fail(MPPI_EUNSUPPORTED, "debug_dump needs a context and its workspace");
    if (cfg->start_iteration + (uint64_t)iters > kTwo32)
      return fail(MPPI_EINVAL, "iteration counter would pass 2^32");
    const Layout L = make_layout(cfg, m, q);
    if (L.total > (size_t)MPPI_JUMP_STATIC_SCRATCH_BYTES)
      return fail(MPPI_EWORKSPACE, "K=%d, T=%d needs %zu bytes of scratch, above the static "
                  "maximum of %zu", cfg->K, cfg->T, L.total, (size_t)MPPI_JUMP_STATIC_SCRATCH_BYTES);
    void* base = nullptr;
    rc = static_scratch(&base);
    if (rc != MPPI_OK) return rc;
    // a context on the stack over the static scratch; the sequence is the
    // caller's (its region of the layout stays unused)
    mppi_jump_ctx ctx;
    bind_context(&ctx, cfg, n, m, q, L, th, static_cast<char*>(base));
    ctx.b.U = d_U;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // statistics, iteration counter and arrival counters start afresh (a fill
    // kernel, not a memset node, so that the call can be captured)
    stats_init_kernel<<<1, 64, 0, s>>>(ctx.b, L.R, cfg->start_iteration);
    LAUNCH_CHECK("stats_init_kernel");
    return enqueue_control_step(&ctx, d_x0, iters, d_u0_out, stream);
  });
}

int mppi_jump_shift(mppi_jump_ctx* ctx, float* u0_out, void* stream) {
  return guarded([&]() -> int {
    if (!ctx) return fail(MPPI_EINVAL, "NULL context");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // u_0 leaves by a stream-ordered copy (device or host destination)
    if (u0_out) HIP_TRY(hipMemcpyAsync(u0_out, ctx->b.U, (size_t)ctx->m * 4, hipMemcpyDefault, s));
    shift_kernel<<<1, 1024, 0, s>>>(ctx->b.U, ctx->L.R, ctx->m, u_init4(ctx->cfg));
    LAUNCH_CHECK("shift_kernel");
    return ok();
  });
}

int mppi_jump_get(mppi_jump_ctx* ctx, int32_t what, void* dst, size_t dst_bytes, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !dst) return fail(MPPI_EINVAL, "NULL context or destination");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t K = (size_t)ctx->cfg.K, T = (size_t)ctx->cfg.T;
    auto need = [&](size_t bytes) -> int {
      if (dst_bytes < bytes) return fail(MPPI_EINVAL, "destination of %zu bytes < %zu", dst_bytes, bytes);
      return MPPI_OK;
    };
    const void* src = nullptr;
    size_t bytes = 0;
    switch (what) {
      case MPPI_ITEM_U: src = ctx->b.U; bytes = (size_t)ctx->L.R * 4; break;
      case MPPI_ITEM_S: src = ctx->b.S; bytes = K * 8; break;
      case MPPI_ITEM_STATS: src = ctx->b.stats; bytes = sizeof(mppi_jump_stats); break;
      case MPPI_ITEM_W: {
        if (need(K * 8) != MPPI_OK) return MPPI_EINVAL;
        weights_kernel<<<(unsigned)((K + 255) / 256), 256, 0, s>>>(ctx->p, ctx->b, ctx->W);
        LAUNCH_CHECK("weights_kernel");
        src = ctx->W;
        bytes = K * 8;
        break;
      }
      case MPPI_ITEM_EPS: {
        if (!ctx->eps_stored)
          return fail(MPPI_EUNSUPPORTED, "the last iteration kept its perturbations on chip "
                      "(fused wave-specialised form); a staged rollout stores them");
        if (need((size_t)ctx->L.R * K * 4) != MPPI_OK) return MPPI_EINVAL;
        HIP_TRY(hipMemcpy2DAsync(dst, K * 4, ctx->b.eps, (size_t)ctx->L.Ks * 4, K * 4,
                                 (size_t)ctx->L.R, hipMemcpyDefault, s));
        return ok();
      }
      case MPPI_ITEM_DBG_ZD:
      case MPPI_ITEM_DBG_N:
      case MPPI_ITEM_DBG_ZJ:
        if (!ctx->cfg.debug_dump) return fail(MPPI_EUNSUPPORTED, "context was created without debug_dump");
        if (what == MPPI_ITEM_DBG_ZD) { src = ctx->b.dbg_zD; bytes = K * T * ctx->m * 4; }
        if (what == MPPI_ITEM_DBG_N) { src = ctx->b.dbg_N; bytes = K * T * 4; }
        if (what == MPPI_ITEM_DBG_ZJ) { src = ctx->b.dbg_zJ; bytes = K * T * ctx->q * 4; }
        break;
      case MPPI_ITEM_THRESH: src = ctx->th64; bytes = sizeof(ctx->th64); break;
      default: return fail(MPPI_EINVAL, "unknown item %d", what);
    }
    if (need(bytes) != MPPI_OK) return MPPI_EINVAL;
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, s));
    return ok();
  });
}

int mppi_jump_set(mppi_jump_ctx* ctx, int32_t what, const void* src, size_t src_bytes, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !src) return fail(MPPI_EINVAL, "NULL context or source");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (what == MPPI_ITEM_U) {
      const size_t bytes = (size_t)ctx->L.R * 4;
      if (src_bytes != bytes) return fail(MPPI_EINVAL, "U needs %zu bytes, got %zu", bytes, src_bytes);
      HIP_TRY(hipMemcpyAsync(ctx->b.U, src, bytes, hipMemcpyDefault, s));
      return ok();
    }
    if (what == MPPI_ITEM_S) {
      const size_t bytes = (size_t)ctx->cfg.K * 8;
      if (src_bytes != bytes) return fail(MPPI_EINVAL, "S needs %zu bytes, got %zu", bytes, src_bytes);
      HIP_TRY(hipMemcpyAsync(ctx->b.S, src, bytes, hipMemcpyDefault, s));
      if (ctx->L.ws)
        restats_kernel<kWsSamples><<<ctx->L.nwg, kBlock, 0, s>>>(ctx->p, ctx->b);
      else
        restats_kernel<kBlock><<<ctx->L.nwg, kBlock, 0, s>>>(ctx->p, ctx->b);
      LAUNCH_CHECK("restats_kernel");
      return ok();
    }
    return fail(MPPI_EINVAL, "item %d cannot be set", what);
  });
}

// ------------------------------------------------------------------ batch
}  // extern "C"

struct mppi_jump_batch {
  std::vector<mppi_jump_ctx*> ctxs;
  std::vector<BatchDesc> h_desc;
  std::vector<BatchTile> h_tiles;
  BatchDesc* d_desc = nullptr;
  BatchTile* d_tiles = nullptr;
  float* d_u0 = nullptr;
  BatchQueue* d_queue = nullptr;
  bool ws = false;
  int mask = kMaskAll;          // dynamics ids of the batch's kernel
  int launch = MPPI_BATCH_GRID;
  int slots = 0;                // workgroups of the persistent launch
  size_t dyn_lds = 0;
};

namespace {

struct BatchLayout {
  size_t desc, tiles, u0, queue, total;
  int ntiles;
};

int batch_check(mppi_jump_ctx* const* ctxs, int32_t n, BatchLayout& BL, bool& ws) {
  if (!ctxs || n < 1) return fail(MPPI_EINVAL, "batch needs at least one context");
  int ntiles = 0;
  for (int i = 0; i < n; ++i) {
    const mppi_jump_ctx* c = ctxs[i];
    if (!c) return fail(MPPI_EINVAL, "context %d is NULL", i);
    // only controllers whose own iteration is fused: a batched iteration
    // then runs the same epilogue and gives the same results bitwise
    if (!c->L.fused)
      return fail(MPPI_EUNSUPPORTED, "context %d: K=%d needs more than %d rollout workgroups", i,
                  c->cfg.K, c->L.ws ? kFusedWgWs : kFusedWgLane);
    if (c->cfg.debug_dump) return fail(MPPI_EUNSUPPORTED, "context %d has debug_dump set", i);
    if (c->p.full) return fail(MPPI_EUNSUPPORTED, "context %d has a full noise covariance", i);
    if (i == 0) ws = c->L.ws;
    if (c->L.ws != ws) return fail(MPPI_EINVAL, "contexts of one batch must share a rollout schedule");
    ntiles += c->L.nwg;
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  BL.desc = take((size_t)n * sizeof(BatchDesc));
  BL.tiles = take((size_t)ntiles * sizeof(BatchTile));
  BL.u0 = take((size_t)n * 4 * sizeof(float));
  BL.queue = take(sizeof(BatchQueue));
  BL.total = off;
  BL.ntiles = ntiles;
  return MPPI_OK;
}

// Tile cost estimate for the longest-first order: time steps times the
// issue slots of one sample-step of the model.
double tile_cost(const mppi_jump_ctx* c) {
  const double per_step = c->cfg.dynamics == MPPI_DYN_QUADROTOR ? 534.0
                          : c->cfg.dynamics == MPPI_DYN_CARTPOLE ? 216.0 : 184.0;
  return per_step * c->cfg.T;
}

// The batch kernel instantiations: grid launch of either schedule over all
// models, and of the lane schedule per model; persistent launch of the lane
// schedule (all models, or one) and of the wave-specialised schedule.
template <bool WS, int MASK>
int launch_batch_t(mppi_jump_batch* bt, int shift, hipStream_t s) {
  const size_t lds = WS ? bt->dyn_lds : 0;
  if (bt->launch == MPPI_BATCH_PERSISTENT) {
    batch_persistent_kernel<WS, MASK><<<bt->slots, kBlock, lds, s>>>(
        bt->d_desc, bt->d_tiles, (int)bt->h_tiles.size(), shift, bt->d_queue);
    LAUNCH_CHECK("batch_persistent_kernel");
  } else {
    batch_rollout_kernel<WS, MASK><<<(unsigned)bt->h_tiles.size(), kBlock, lds, s>>>(
        bt->d_desc, bt->d_tiles, shift);
    LAUNCH_CHECK("batch_rollout_kernel");
  }
  return MPPI_OK;
}

int launch_batch(mppi_jump_batch* bt, int shift, hipStream_t s) {
  if (bt->ws) return launch_batch_t<true, kMaskAll>(bt, shift, s);
  if (bt->mask == kMaskCartpole) return launch_batch_t<false, kMaskCartpole>(bt, shift, s);
  if (bt->mask == kMaskQuadrotor) return launch_batch_t<false, kMaskQuadrotor>(bt, shift, s);
  return launch_batch_t<false, kMaskAll>(bt, shift, s);
}

// Workgroups of the persistent launch: as many as the GPU holds at once
// (occupancy of the batch's persistent kernel times the compute units), at
// most one per tile.
template <bool WS, int MASK>
int occupancy_of(mppi_jump_batch* bt, int* per_cu) {
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      per_cu, batch_persistent_kernel<WS, MASK>, kBlock, WS ? bt->dyn_lds : 0));
  return MPPI_OK;
}

int persistent_slots(mppi_jump_batch* bt) {
  int dev = 0, cus = 0, per_cu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  int rc;
  if (bt->ws)
    rc = occupancy_of<true, kMaskAll>(bt, &per_cu);
  else if (bt->mask == kMaskCartpole)
    rc = occupancy_of<false, kMaskCartpole>(bt, &per_cu);
  else if (bt->mask == kMaskQuadrotor)
    rc = occupancy_of<false, kMaskQuadrotor>(bt, &per_cu);
  else
    rc = occupancy_of<false, kMaskAll>(bt, &per_cu);
  if (rc != MPPI_OK) return rc;
  if (per_cu < 1 || cus < 1) return fail(MPPI_EDEVICE, "no resident workgroup for the batch kernel");
  bt->slots = std::min(per_cu * cus, (int)bt->h_tiles.size());
  return MPPI_OK;
}

}  // namespace

extern "C" {

int mppi_jump_batch_scratch_bytes(mppi_jump_ctx* const* ctxs, int32_t n, size_t* bytes) {
  return guarded([&]() -> int {
    if (!bytes) return fail(MPPI_EINVAL, "bytes is NULL");
    BatchLayout BL;
    bool ws;
    const int rc = batch_check(ctxs, n, BL, ws);
    if (rc != MPPI_OK) return rc;
    *bytes = BL.total;
    return ok();
  });
}

int mppi_jump_batch_create(mppi_jump_ctx* const* ctxs, const float* const* d_x0, int32_t n,
                           void* d_scratch, size_t scratch_bytes, void* stream,
                           mppi_jump_batch** out) {
  return guarded([&]() -> int {
    if (!out) return fail(MPPI_EINVAL, "out is NULL");
    *out = nullptr;
    BatchLayout BL;
    bool ws = false;
    int rc = batch_check(ctxs, n, BL, ws);
    if (rc != MPPI_OK) return rc;
    if (!d_x0) return fail(MPPI_EINVAL, "state pointer array is NULL");
    for (int i = 0; i < n; ++i)
      if (!d_x0[i]) return fail(MPPI_EINVAL, "state pointer %d is NULL", i);
    if (!d_scratch || ((uintptr_t)d_scratch & 255u))
      return fail(MPPI_EWORKSPACE, "scratch must be a 256-byte aligned device pointer");
    if (scratch_bytes < BL.total)
      return fail(MPPI_EWORKSPACE, "scratch of %zu bytes < %zu needed", scratch_bytes, BL.total);
    auto* bt = new mppi_jump_batch();
    bt->ws = ws;
    int models = 0;
    bt->ctxs.assign(ctxs, ctxs + n);
    char* base = static_cast<char*>(d_scratch);
    bt->d_desc = reinterpret_cast<BatchDesc*>(base + BL.desc);
    bt->d_tiles = reinterpret_cast<BatchTile*>(base + BL.tiles);
    bt->d_u0 = reinterpret_cast<float*>(base + BL.u0);
    bt->d_queue = reinterpret_cast<BatchQueue*>(base + BL.queue);
    bt->h_desc.resize(n);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) {
      const mppi_jump_ctx* c = ctxs[i];
      BatchDesc& d = bt->h_desc[i];
      std::memset(&d, 0, sizeof d);
      d.p = c->p;
      d.b = c->b;
      d.x0 = d_x0[i];
      d.u0_out = bt->d_u0 + 4 * i;
      d.u_init = u_init4(c->cfg);
      d.R = c->L.R;
      d.nwg = c->L.nwg;
      d.dyn = c->cfg.dynamics;
      d.jumps = c->p.n_th > 0 ? 1 : 0;
      d.form = c->cfg.cost_form;
      d.m = c->m;
      order[i] = i;
      models |= 1 << c->cfg.dynamics;
      if (ws) {
        const size_t lds = c->cfg.dynamics == MPPI_DYN_QUADROTOR ? ws_ring_bytes<MPPI_DYN_QUADROTOR>()
                           : c->cfg.dynamics == MPPI_DYN_CARTPOLE ? ws_ring_bytes<MPPI_DYN_CARTPOLE>()
                                                                  : ws_ring_bytes<MPPI_DYN_LINEAR>();
        if (lds > bt->dyn_lds) bt->dyn_lds = lds;
      }
    }
    // one-model batches of the lane schedule run a kernel of that model's
    // variants only
    if (!ws && (models == kMaskCartpole || models == kMaskQuadrotor)) bt->mask = models;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return tile_cost(ctxs[a]) > tile_cost(ctxs[b]); });
    bt->h_tiles.reserve(BL.ntiles);
    for (int i : order)
      for (int w = 0; w < ctxs[i]->L.nwg; ++w) bt->h_tiles.push_back(BatchTile{i, w});
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(bt->d_desc, bt->h_desc.data(), (size_t)n * sizeof(BatchDesc),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(bt->d_tiles, bt->h_tiles.data(), bt->h_tiles.size() * sizeof(BatchTile),
                         hipMemcpyHostToDevice, s);
    const std::vector<float> zeros((size_t)n * 4, 0.f);  // unused u_0 slots read as 0
    if (e == hipSuccess)
      e = hipMemcpyAsync(bt->d_u0, zeros.data(), zeros.size() * sizeof(float),
                         hipMemcpyHostToDevice, s);
    const BatchQueue q0{0u, 0u};  // the persistent launch's queue starts empty
    if (e == hipSuccess)
      e = hipMemcpyAsync(bt->d_queue, &q0, sizeof q0, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      delete bt;
      return fail(MPPI_EDEVICE, "batch table upload: %s", hipGetErrorString(e));
    }
    *out = bt;
    return ok();
  });
}

int mppi_jump_batch_step(mppi_jump_batch* bt, int32_t iters, int32_t shift, void* stream) {
  return guarded([&]() -> int {
    if (!bt) return fail(MPPI_EINVAL, "NULL batch");
    if (iters < 1) return fail(MPPI_EINVAL, "iters=%d < 1", iters);
    for (auto* c : bt->ctxs)
      if (c->host_iteration + (uint64_t)iters > kTwo32)
        return fail(MPPI_EINVAL, "iteration counter would pass 2^32");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < iters; ++i) {
      const int sh = (shift && i == iters - 1) ? 1 : 0;
      const int rc = launch_batch(bt, sh, s);
      if (rc != MPPI_OK) return rc;
    }
    for (auto* c : bt->ctxs) {
      c->host_iteration += (uint64_t)iters;
      c->eps_stored = true;  // batched tiles store their perturbations
    }
    return ok();
  });
}

int mppi_jump_batch_set_launch(mppi_jump_batch* bt, int32_t launch) {
  return guarded([&]() -> int {
    if (!bt) return fail(MPPI_EINVAL, "NULL batch");
    if (launch != MPPI_BATCH_GRID && launch != MPPI_BATCH_PERSISTENT)
      return fail(MPPI_EINVAL, "unknown batch launch %d", launch);
    if (launch == MPPI_BATCH_PERSISTENT) {
      const int rc = persistent_slots(bt);
      if (rc != MPPI_OK) return rc;
    }
    bt->launch = launch;
    return ok();
  });
}

int mppi_jump_batch_u0(mppi_jump_batch* bt, float** d_u0) {
  if (!bt || !d_u0) return fail(MPPI_EINVAL, "NULL argument");
  *d_u0 = bt->d_u0;
  return ok();
}

int mppi_jump_batch_destroy(mppi_jump_batch* bt) {
  delete bt;
  return ok();
}

// ------------------------------------------------------------------ pool
}  // extern "C"

namespace {

// Request record of one slot: ids [n], prefix [n + 1], states [n][12],
// disturbances [n][8], outputs [n][16] (4-byte words; parts 256-byte aligned).
struct SlotLayout {
  size_t ids, prefix, states, dist, out, total;
};

SlotLayout slot_layout(int n) {
  SlotLayout S{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  S.ids = take((size_t)n * 4);
  S.prefix = take((size_t)(n + 1) * 4);
  S.states = take((size_t)n * 12 * 4);
  S.dist = take((size_t)n * kPoolDist * 4);
  S.out = take((size_t)n * kPoolOut * 4);
  S.total = off;
  return S;
}

struct PoolSlot {
  hipEvent_t done = nullptr;
  bool pending = false;       // a tick was enqueued and its results not yet taken
  bool plant = false;         // that tick stepped the plant
  std::vector<int> order;     // record position j holds the caller's request order[j]
  std::vector<int> ids;       // the caller's ids, in the caller's order
  int count = 0;
};

}  // namespace

struct mppi_jump_pool {
  std::vector<mppi_jump_ctx*> ctxs;
  std::vector<double> cost;
  std::vector<int> busy;      // slot whose tick holds the controller, or -1
  std::vector<PoolSlot> slots;
  BatchDesc* d_desc = nullptr;
  char* d_slots = nullptr;
  char* h_slots = nullptr;
  SlotLayout S{};
  int n = 0;
  bool ws = false;
  size_t dyn_lds = 0;
  ~mppi_jump_pool() {
    for (auto& sl : slots)
      if (sl.done) (void)hipEventDestroy(sl.done);
  }
};

extern "C" {

int mppi_jump_pool_bytes(mppi_jump_ctx* const* ctxs, int32_t n, int32_t max_inflight,
                         size_t* device_bytes, size_t* pinned_host_bytes) {
  return guarded([&]() -> int {
    if (!device_bytes || !pinned_host_bytes) return fail(MPPI_EINVAL, "NULL output");
    if (max_inflight < 1 || max_inflight > MPPI_JUMP_POOL_MAX_INFLIGHT)
      return fail(MPPI_EINVAL, "max_inflight=%d out of [1, %d]", max_inflight,
                  MPPI_JUMP_POOL_MAX_INFLIGHT);
    BatchLayout BL;
    bool ws;
    const int rc = batch_check(ctxs, n, BL, ws);
    if (rc != MPPI_OK) return rc;
    const SlotLayout S = slot_layout(n);
    *device_bytes = align_up((size_t)n * sizeof(BatchDesc), 256) + S.total * max_inflight;
    *pinned_host_bytes = S.total * max_inflight;
    return ok();
  });
}

int mppi_jump_pool_create(mppi_jump_ctx* const* ctxs, int32_t n, int32_t max_inflight,
                          void* d_scratch, size_t device_bytes, void* h_pinned,
                          size_t pinned_bytes, void* stream, mppi_jump_pool** out) {
  return guarded([&]() -> int {
    if (!out) return fail(MPPI_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need_d = 0, need_h = 0;
    const int rc = mppi_jump_pool_bytes(ctxs, n, max_inflight, &need_d, &need_h);
    if (rc != MPPI_OK) return rc;
    if (!d_scratch || ((uintptr_t)d_scratch & 255u) || device_bytes < need_d)
      return fail(MPPI_EWORKSPACE, "device scratch missing, misaligned or below %zu bytes", need_d);
    if (!h_pinned || ((uintptr_t)h_pinned & 255u) || pinned_bytes < need_h)
      return fail(MPPI_EWORKSPACE, "pinned staging missing, misaligned or below %zu bytes", need_h);
    std::unique_ptr<mppi_jump_pool> pl(new mppi_jump_pool());
    pl->ctxs.assign(ctxs, ctxs + n);
    pl->n = n;
    pl->ws = ctxs[0]->L.ws;
    pl->S = slot_layout(n);
    pl->busy.assign(n, -1);
    pl->slots.resize(max_inflight);
    for (auto& sl : pl->slots) HIP_TRY(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    char* base = static_cast<char*>(d_scratch);
    pl->d_desc = reinterpret_cast<BatchDesc*>(base);
    pl->d_slots = base + align_up((size_t)n * sizeof(BatchDesc), 256);
    pl->h_slots = static_cast<char*>(h_pinned);
    std::vector<BatchDesc> h_desc(n);
    pl->cost.resize(n);
    for (int i = 0; i < n; ++i) {
      const mppi_jump_ctx* c = ctxs[i];
      BatchDesc& d = h_desc[i];
      std::memset(&d, 0, sizeof d);
      d.p = c->p;
      d.b = c->b;
      d.u_init = u_init4(c->cfg);
      d.R = c->L.R;
      d.nwg = c->L.nwg;
      d.dyn = c->cfg.dynamics;
      d.jumps = c->p.n_th > 0 ? 1 : 0;
      d.form = c->cfg.cost_form;
      d.m = c->m;
      pl->cost[i] = tile_cost(c);
    }
    // a wave-specialised pool launches with the largest ring of any model, so
    // that a position can take a context of any model (mppi_jump_pool_replace)
    if (pl->ws)
      pl->dyn_lds = std::max({ws_ring_bytes<MPPI_DYN_QUADROTOR>(), ws_ring_bytes<MPPI_DYN_CARTPOLE>(),
                              ws_ring_bytes<MPPI_DYN_LINEAR>()});
    // the staging is zeroed once so that unused state / disturbance words
    // of a request are defined
    std::memset(pl->h_slots, 0, need_h);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(pl->d_desc, h_desc.data(), (size_t)n * sizeof(BatchDesc),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = pl.release();
    return ok();
  });
}

namespace {

// Whether the tick last enqueued on a slot has finished on the device.
int slot_finished(mppi_jump_pool* pl, int slot, bool* finished) {
  PoolSlot& sl = pl->slots[slot];
  if (!sl.pending) {
    *finished = true;
    return MPPI_OK;
  }
  const hipError_t e = hipEventQuery(sl.done);
  if (e == hipErrorNotReady) {
    *finished = false;
    return MPPI_OK;
  }
  if (e != hipSuccess) return fail(MPPI_EDEVICE, "slot %d: %s", slot, hipGetErrorString(e));
  *finished = true;
  return MPPI_OK;
}

}  // namespace

int mppi_jump_pool_tick(mppi_jump_pool* pl, const int32_t* ids, const float* states,
                        const float* dist, int32_t count, int32_t iters, int32_t slot,
                        void* stream) {
  return guarded([&]() -> int {
    if (!pl || !ids || !states) return fail(MPPI_EINVAL, "NULL argument");
    if (count < 1 || count > pl->n) return fail(MPPI_EINVAL, "count=%d out of [1, %d]", count, pl->n);
    if (iters < 1) return fail(MPPI_EINVAL, "iters=%d < 1", iters);
    if (slot < 0 || slot >= (int)pl->slots.size()) return fail(MPPI_EINVAL, "slot %d out of range", slot);
    PoolSlot& sl = pl->slots[slot];
    if (sl.pending) return fail(MPPI_EINVAL, "slot %d holds results not yet taken", slot);
    std::vector<int> order(count);
    std::vector<char> seen(pl->n, 0);
    for (int i = 0; i < count; ++i) {
      const int c = ids[i];
      if (c < 0 || c >= pl->n) return fail(MPPI_EINVAL, "controller id %d out of range", c);
      if (seen[c]) return fail(MPPI_EINVAL, "controller %d requested twice in one tick", c);
      if (pl->busy[c] >= 0) return fail(MPPI_EINVAL, "controller %d is in a tick in flight", c);
      if (pl->ctxs[c]->host_iteration + (uint64_t)iters > kTwo32)
        return fail(MPPI_EINVAL, "iteration counter of controller %d would pass 2^32", c);
      seen[c] = 1;
      order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return pl->cost[ids[a]] > pl->cost[ids[b]]; });
    const SlotLayout& S = pl->S;
    char* h = pl->h_slots + (size_t)slot * S.total;
    char* d = pl->d_slots + (size_t)slot * S.total;
    int32_t* h_ids = reinterpret_cast<int32_t*>(h + S.ids);
    int32_t* h_pre = reinterpret_cast<int32_t*>(h + S.prefix);
    float* h_st = reinterpret_cast<float*>(h + S.states);
    float* h_di = reinterpret_cast<float*>(h + S.dist);
    int tiles = 0;
    for (int j = 0; j < count; ++j) {
      const int i = order[j];
      const mppi_jump_ctx* c = pl->ctxs[ids[i]];
      h_ids[j] = ids[i];
      h_pre[j] = tiles;
      tiles += c->L.nwg;
      std::memcpy(h_st + 12 * j, states + 12 * i, sizeof(float) * c->n);
      if (dist) std::memcpy(h_di + kPoolDist * j, dist + kPoolDist * i, sizeof(float) * kPoolDist);
    }
    h_pre[count] = tiles;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // one upload of ids, prefix, states and disturbances
    HIP_TRY(hipMemcpyAsync(d, h, S.out, hipMemcpyHostToDevice, s));
    PoolTick tk;
    tk.ids = reinterpret_cast<const int*>(d + S.ids);
    tk.prefix = reinterpret_cast<const int*>(d + S.prefix);
    tk.states = reinterpret_cast<const float*>(d + S.states);
    tk.dist = reinterpret_cast<const float*>(d + S.dist);
    tk.out = reinterpret_cast<float*>(d + S.out);
    tk.count = count;
    for (int it = 0; it < iters; ++it) {
      tk.shift = it == iters - 1 ? 1 : 0;
      if (pl->ws)
        pool_rollout_kernel<true><<<tiles, kBlock, pl->dyn_lds, s>>>(pl->d_desc, tk);
      else
        pool_rollout_kernel<false><<<tiles, kBlock, 0, s>>>(pl->d_desc, tk);
      LAUNCH_CHECK("pool_rollout_kernel");
    }
    if (dist) {
      pool_plant_kernel<<<(count + 63) / 64, 64, 0, s>>>(pl->d_desc, tk);
      LAUNCH_CHECK("pool_plant_kernel");
    }
    HIP_TRY(hipMemcpyAsync(h + S.out, d + S.out, (size_t)count * kPoolOut * 4,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(sl.done, s));
    sl.pending = true;
    sl.plant = dist != nullptr;
    sl.order = std::move(order);
    sl.ids.assign(ids, ids + count);
    sl.count = count;
    for (int i = 0; i < count; ++i) {
      pl->busy[ids[i]] = slot;
      pl->ctxs[ids[i]]->host_iteration += (uint64_t)iters;
      pl->ctxs[ids[i]]->eps_stored = true;  // pooled tiles store their perturbations
    }
    return ok();
  });
}

int mppi_jump_pool_replace(mppi_jump_pool* pl, int32_t index, mppi_jump_ctx* ctx, void* stream) {
  return guarded([&]() -> int {
    if (!pl || !ctx) return fail(MPPI_EINVAL, "NULL argument");
    if (index < 0 || index >= pl->n) return fail(MPPI_EINVAL, "index %d out of [0, %d)", index, pl->n);
    if (pl->busy[index] >= 0) return fail(MPPI_EINVAL, "position %d is in a tick in flight", index);
    BatchLayout BL;
    bool ws = false;
    mppi_jump_ctx* one[1] = {ctx};
    const int rc = batch_check(one, 1, BL, ws);
    if (rc != MPPI_OK) return rc;
    if (ws != pl->ws) return fail(MPPI_EINVAL, "the context's rollout schedule differs from the pool's");
    BatchDesc d;
    std::memset(&d, 0, sizeof d);
    d.p = ctx->p;
    d.b = ctx->b;
    d.u_init = u_init4(ctx->cfg);
    d.R = ctx->L.R;
    d.nwg = ctx->L.nwg;
    d.dyn = ctx->cfg.dynamics;
    d.jumps = ctx->p.n_th > 0 ? 1 : 0;
    d.form = ctx->cfg.cost_form;
    d.m = ctx->m;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(pl->d_desc + index, &d, sizeof d, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    pl->ctxs[index] = ctx;
    pl->cost[index] = tile_cost(ctx);
    return ok();
  });
}

int mppi_jump_pool_query(mppi_jump_pool* pl, int32_t slot, int32_t* finished) {
  return guarded([&]() -> int {
    if (!pl || !finished) return fail(MPPI_EINVAL, "NULL argument");
    if (slot < 0 || slot >= (int)pl->slots.size()) return fail(MPPI_EINVAL, "slot %d out of range", slot);
    bool f = false;
    const int rc = slot_finished(pl, slot, &f);
    if (rc != MPPI_OK) return rc;
    *finished = f ? 1 : 0;
    return ok();
  });
}

int mppi_jump_pool_results(mppi_jump_pool* pl, int32_t slot, int32_t* ids, float* u0,
                           float* x_next, int32_t* count) {
  return guarded([&]() -> int {
    if (!pl || !count) return fail(MPPI_EINVAL, "NULL argument");
    if (slot < 0 || slot >= (int)pl->slots.size()) return fail(MPPI_EINVAL, "slot %d out of range", slot);
    PoolSlot& sl = pl->slots[slot];
    if (!sl.pending) return fail(MPPI_EINVAL, "slot %d has no tick", slot);
    bool f = false;
    int rc = slot_finished(pl, slot, &f);
    if (rc != MPPI_OK) return rc;
    if (!f) return fail(MPPI_EINVAL, "the tick of slot %d has not finished", slot);
    if (x_next && !sl.plant) return fail(MPPI_EINVAL, "the tick of slot %d ran no plant step", slot);
    const float* h_out = reinterpret_cast<const float*>(pl->h_slots + (size_t)slot * pl->S.total +
                                                        pl->S.out);
    // a record position keeps words of earlier, larger requests beyond this
    // request's m and n: copy only the live words and zero the rest
    for (int j = 0; j < sl.count; ++j) {
      const int i = sl.order[j];
      const mppi_jump_ctx* c = pl->ctxs[sl.ids[i]];
      if (ids) ids[i] = sl.ids[i];
      if (u0)
        for (int k = 0; k < 4; ++k) u0[4 * i + k] = k < c->m ? h_out[kPoolOut * j + k] : 0.f;
      if (x_next)
        for (int k = 0; k < 12; ++k) x_next[12 * i + k] = k < c->n ? h_out[kPoolOut * j + 4 + k] : 0.f;
    }
    *count = sl.count;
    for (int c : sl.ids) pl->busy[c] = -1;
    sl.pending = false;
    return ok();
  });
}

int mppi_jump_pool_destroy(mppi_jump_pool* pl) {
  delete pl;
  return ok();
}

int mppi_jump_destroy(mppi_jump_ctx* ctx) {
  if (!ctx) return ok();
  for (auto& e : ctx->events) {
    (void)hipEventDestroy(e.e0);
    (void)hipEventDestroy(e.e1);
  }
  delete ctx;
  return ok();
}

const char* mppi_jump_strerror(int code) {
  switch (code) {
    case MPPI_OK: return "ok";
    case MPPI_EINVAL: return "invalid argument";
    case MPPI_EWORKSPACE: return "workspace too small or misaligned";
    case MPPI_EDEVICE: return "HIP runtime error";
    case MPPI_ENONFINITE: return "all path costs non-finite";
    case MPPI_EUNSUPPORTED: return "unsupported";
    default: return "unknown status code";
  }
}

const char* mppi_jump_last_error(void) { return g_last_error; }

int mppi_jump_plant_step_force(mppi_jump_ctx* ctx, float* d_x, const float* d_u,
                               const float* d_dist, const float* d_force, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !d_x || !d_u || !d_dist) return fail(MPPI_EINVAL, "NULL argument");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    switch (ctx->cfg.dynamics) {
      case MPPI_DYN_LINEAR:
        plant_kernel<MPPI_DYN_LINEAR><<<1, 64, 0, s>>>(ctx->p, d_x, d_u, d_dist, d_force);
        break;
      case MPPI_DYN_CARTPOLE:
        plant_kernel<MPPI_DYN_CARTPOLE><<<1, 64, 0, s>>>(ctx->p, d_x, d_u, d_dist, d_force);
        break;
      default:
        plant_kernel<MPPI_DYN_QUADROTOR><<<1, 64, 0, s>>>(ctx->p, d_x, d_u, d_dist, d_force);
        break;
    }
    LAUNCH_CHECK("plant_kernel");
    return ok();
  });
}

int mppi_jump_plant_step(mppi_jump_ctx* ctx, float* d_x, const float* d_u, const float* d_dist,
                         void* stream) {
  return mppi_jump_plant_step_force(ctx, d_x, d_u, d_dist, nullptr, stream);
}

int mppi_jump_philox(const uint32_t* d_counters, uint32_t key0, uint32_t key1, uint32_t* d_out,
                     int64_t n, void* stream) {
  return guarded([&]() -> int {
    if (n < 0 || (n > 0 && (!d_counters || !d_out))) return fail(MPPI_EINVAL, "bad arguments");
    if (n == 0) return ok();
    if (n > (1ll << 30)) return fail(MPPI_EINVAL, "n too large");
    philox_kernel<<<(unsigned)((n + 255) / 256), 256, 0, static_cast<hipStream_t>(stream)>>>(
        d_counters, key0, key1, d_out, n);
    LAUNCH_CHECK("philox_kernel");
    return ok();
  });
}

int mppi_jump_profile(mppi_jump_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(MPPI_EINVAL, "NULL context");
  ctx->profiling = enable != 0;
  return ok();
}

int mppi_jump_profile_read(mppi_jump_ctx* ctx, double* total_ms, int64_t* launches,
                           int64_t* iterations) {
  return guarded([&]() -> int {
    if (!ctx || !total_ms || !launches || !iterations) return fail(MPPI_EINVAL, "NULL argument");
    double tot = 0.0;
    int64_t n = 0, ni = 0;
    for (size_t i = 0; i < ctx->events_used; ++i) {
      HIP_TRY(hipEventSynchronize(ctx->events[i].e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ctx->events[i].e0, ctx->events[i].e1));
      tot += ms;
      n += ctx->events[i].launches;
      ni += ctx->events[i].iterations;
    }
    *total_ms = tot;
    *launches = n;
    *iterations = ni;
    ctx->events_used = 0;
    return ok();
  });
}

}  // extern "C"

#ifdef MPPI_PHASE_STAMPS
#include "../../include/mppi_jump_phases.h"
static_assert(mppi::kPhaseLaunches == MPPI_PHASE_LAUNCHES && mppi::kPhaseMaxWg == MPPI_PHASE_MAX_WG &&
                  mppi::kPhaseSlots == MPPI_PHASE_SLOTS && mppi::kPhaseTiles == MPPI_PHASE_TILES,
              "record layout of the phase hook");
extern "C" int mppi_phase_read(unsigned long long* out, size_t count) {
  const size_t n = sizeof(mppi::g_phase) / sizeof(mppi::g_phase[0]);
  if (!out || count < n) return MPPI_EINVAL;
  return hipMemcpyFromSymbol(out, HIP_SYMBOL(mppi::g_phase), sizeof(mppi::g_phase)) == hipSuccess
             ? MPPI_OK
             : MPPI_EDEVICE;
}
extern "C" int mppi_phase_read_tiles(unsigned long long* out, size_t count) {
  const size_t n = sizeof(mppi::g_phase_tiles) / sizeof(mppi::g_phase_tiles[0]);
  if (!out || count < n) return MPPI_EINVAL;
  return hipMemcpyFromSymbol(out, HIP_SYMBOL(mppi::g_phase_tiles), sizeof(mppi::g_phase_tiles)) ==
                 hipSuccess
             ? MPPI_OK
             : MPPI_EDEVICE;
}
#endif
