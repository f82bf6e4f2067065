// C ABI of libnisqtol (declared in include/nisqtol.h).  Every entry point
// validates its arguments, converts internal errors into nt_status codes and
// records a thread-local message; no exception crosses the boundary.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "engine.hpp"
#include "gnn_model.hpp"

struct nt_ctx {
  nt::Ctx *impl;
};
struct nt_circuit {
  nt::Circuit *impl;
};
struct nt_gnn {
  nt_ctx *ctx;
  gnn::Model *impl;
};

namespace {

thread_local std::string g_last_error;

nt_status fail(nt_status s, const std::string &m) {
  g_last_error = m;
  return s;
}

template <typename F>
nt_status guard(F &&f) {
  try {
    f();
    g_last_error.clear();
    return NT_OK;
  } catch (const nt::Error &e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc &) {
    return fail(NT_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(NT_ERR_DEVICE, e.what());
  } catch (...) {
    return fail(NT_ERR_DEVICE, "unknown error");
  }
}

bool valid_prob(double p) { return std::isfinite(p) && p >= 0.0 && p <= 1.0; }

void check_hip_entry(nt_ctx *ctx) { nt::check_hip(hipSetDevice(ctx->impl->device), "hipSetDevice"); }

}  // namespace

extern "C" {

const char *nt_last_error(void) { return g_last_error.c_str(); }

const char *nt_version(void) { return "nisqtol 0.1 (gfx950)"; }

nt_status nt_create(nt_ctx **out, int device, void *hip_stream) {
  if (!out) return fail(NT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  return guard([&] {
    nt::Ctx *c = new nt::Ctx(device, hip_stream);
    *out = new nt_ctx{c};
  });
}

void nt_destroy(nt_ctx *ctx) {
  if (!ctx) return;
  try {
    delete ctx->impl;
  } catch (...) {
  }
  delete ctx;
}

nt_status nt_set_error_model(nt_ctx *ctx, double px, double py, double pz) {
  if (!ctx) return fail(NT_ERR_INVALID_ARG, "ctx is NULL");
  if (!valid_prob(px) || !valid_prob(py) || !valid_prob(pz))
    return fail(NT_ERR_INVALID_ARG, "each Pauli probability must be finite and in [0, 1]");
  if (px + py + pz > 1.0) return fail(NT_ERR_INVALID_ARG, "p_x + p_y + p_z must be <= 1");
  ctx->impl->px = px;
  ctx->impl->py = py;
  ctx->impl->pz = pz;
  g_last_error.clear();
  return NT_OK;
}

nt_status nt_set_precision(nt_ctx *ctx, int prec) {
  if (!ctx) return fail(NT_ERR_INVALID_ARG, "ctx is NULL");
  if (prec != NT_C64 && prec != NT_C128) return fail(NT_ERR_INVALID_ARG, "precision must be NT_C64 or NT_C128");
  ctx->impl->prec = prec;
  g_last_error.clear();
  return NT_OK;
}

nt_status nt_set_max_batch(nt_ctx *ctx, uint64_t max_batch) {
  if (!ctx) return fail(NT_ERR_INVALID_ARG, "ctx is NULL");
  if (max_batch > (1ull << 31)) return fail(NT_ERR_INVALID_ARG, "max_batch too large");
  ctx->impl->max_batch = max_batch;
  g_last_error.clear();
  return NT_OK;
}

nt_status nt_circuit_load(nt_ctx *ctx, int n_qubits, const nt_gate *gates, int64_t n_gates, nt_circuit **out) {
  (void)ctx;
  if (!out) return fail(NT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  return guard([&] { *out = new nt_circuit{nt::load_circuit(n_qubits, gates, n_gates)}; });
}

nt_status nt_circuit_load_text(nt_ctx *ctx, const char *path, nt_circuit **out) {
  (void)ctx;
  if (!out) return fail(NT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  return guard([&] { *out = new nt_circuit{nt::load_circuit_text(path)}; });
}

void nt_circuit_free(nt_circuit *c) {
  if (!c) return;
  delete c->impl;
  delete c;
}

nt_status nt_circuit_info(const nt_circuit *c, int *n, int64_t *G, int64_t *S) {
  if (!c) return fail(NT_ERR_INVALID_ARG, "circuit is NULL");
  if (n) *n = c->impl->n;
  if (G) *G = (int64_t)c->impl->gates.size();
  if (S) *S = c->impl->S;
  g_last_error.clear();
  return NT_OK;
}

nt_status nt_circuit_set_id(nt_circuit *c, uint64_t cid) {
  if (!c) return fail(NT_ERR_INVALID_ARG, "circuit is NULL");
  c->impl->cid = cid;
  g_last_error.clear();
  return NT_OK;
}

static nt_status check_run_args(nt_ctx *ctx, const nt_circuit *c, double tau);

nt_status nt_circuit_set_tile(nt_circuit *c, int prec, int tile_qubits) {
  if (!c) return fail(NT_ERR_INVALID_ARG, "circuit is NULL");
  if (prec != NT_C64 && prec != NT_C128) return fail(NT_ERR_INVALID_ARG, "precision must be NT_C64 or NT_C128");
  int lo = 0, hi = 0;
  nt::tile_range(*c->impl, prec, &lo, &hi);
  if (tile_qubits != 0 && (tile_qubits < lo || tile_qubits > hi))
    return fail(NT_ERR_INVALID_ARG, "tile width outside [" + std::to_string(lo) + ", " + std::to_string(hi) + "]");
  c->impl->tile_override[prec == NT_C64 ? 1 : 2] = tile_qubits;
  g_last_error.clear();
  return NT_OK;
}

nt_status nt_circuit_set_fusion(nt_circuit *c, int prec, int width) {
  if (!c) return fail(NT_ERR_INVALID_ARG, "circuit is NULL");
  if (prec != NT_C64 && prec != NT_C128) return fail(NT_ERR_INVALID_ARG, "precision must be NT_C64 or NT_C128");
  if (width < 0 || width > 4) return fail(NT_ERR_INVALID_ARG, "fusion width must be in 0..4");
  c->impl->fuse_width[prec == NT_C64 ? 1 : 2] = width;
  g_last_error.clear();
  return NT_OK;
}

nt_status nt_autotune(nt_ctx *ctx, nt_circuit *c, uint64_t seed, uint64_t n_traj, int *tile_out, double *ms_out) {
  nt_status s = check_run_args(ctx, c, 0.9);
  if (s) return s;
  if (n_traj == 0) return fail(NT_ERR_INVALID_ARG, "n_traj must be > 0");
  const int slot = ctx->impl->prec == NT_C64 ? 1 : 2;
  const int saved = c->impl->tile_override[slot];
  int best = 0;
  nt_status st = guard([&] {
    nt::Ctx &cx = *ctx->impl;
    int lo = 0, hi = 0;
    nt::tile_range(*c->impl, cx.prec, &lo, &hi);
    double best_ms = 0;
    int k = 0;
    for (int L = hi; L >= std::max(lo, hi - 2); --L, ++k) {
      c->impl->tile_override[slot] = L;
      cx.run(*c->impl, seed, 0, std::min<uint64_t>(n_traj, 4), 0.9, nullptr, nullptr);   // plan, reference, warm-up
      const auto t0 = std::chrono::steady_clock::now();
      cx.run(*c->impl, seed, 0, n_traj, 0.9, nullptr, nullptr);
      const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (ms_out) ms_out[k] = ms;
      if (best == 0 || ms < best_ms) {
        best = L;
        best_ms = ms;
      }
    }
    c->impl->tile_override[slot] = best;
  });
  if (st) {
    c->impl->tile_override[slot] = saved;
    return st;
  }
  if (tile_out) *tile_out = best;
  return NT_OK;
}

nt_status nt_autotune_plan(nt_ctx *ctx, nt_circuit *c, uint64_t seed, uint64_t n_traj, int *tile_out,
                           int *fusion_out, double *ms_out, int ms_cap) {
  nt_status s = check_run_args(ctx, c, 0.9);
  if (s) return s;
  if (n_traj == 0) return fail(NT_ERR_INVALID_ARG, "n_traj must be > 0");
  if (ms_out && ms_cap < 0) return fail(NT_ERR_INVALID_ARG, "ms_cap must be >= 0");
  const int slot = ctx->impl->prec == NT_C64 ? 1 : 2;
  const int saved_tile = c->impl->tile_override[slot], saved_fuse = c->impl->fuse_width[slot];
  int best_tile = 0, best_fuse = 0;
  nt_status st = guard([&] {
    nt::Ctx &cx = *ctx->impl;
    int lo = 0, hi = 0;
    nt::tile_range(*c->impl, cx.prec, &lo, &hi);
    double best_ms = 0;
    int k = 0;
    for (int L = hi; L >= std::max(lo, hi - 2); --L)
      for (int fw : {2, 3, 4, 1}) {
        c->impl->tile_override[slot] = L;
        c->impl->fuse_width[slot] = fw;
        cx.run(*c->impl, seed, 0, std::min<uint64_t>(n_traj, 4), 0.9, nullptr, nullptr);   // plan, reference, warm-up
        const auto t0 = std::chrono::steady_clock::now();
        cx.run(*c->impl, seed, 0, n_traj, 0.9, nullptr, nullptr);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (ms_out && k < ms_cap) ms_out[k] = ms;
        ++k;
        if (best_tile == 0 || ms < best_ms) {
          best_tile = L;
          best_fuse = fw;
          best_ms = ms;
        }
      }
    c->impl->tile_override[slot] = best_tile;
    c->impl->fuse_width[slot] = best_fuse;
  });
  if (st) {
    c->impl->tile_override[slot] = saved_tile;
    c->impl->fuse_width[slot] = saved_fuse;
    return st;
  }
  if (tile_out) *tile_out = best_tile;
  if (fusion_out) *fusion_out = best_fuse;
  return NT_OK;
}

nt_status nt_plan_info(const nt_circuit *c, int prec, int *n_passes, int *n_segments, int *tile_qubits) {
  if (!c) return fail(NT_ERR_INVALID_ARG, "circuit is NULL");
  if (prec != NT_C64 && prec != NT_C128) return fail(NT_ERR_INVALID_ARG, "precision must be NT_C64 or NT_C128");
  return guard([&] {
    nt::Plan P = nt::choose_plan(*c->impl, prec);
    if (n_passes) *n_passes = (int)P.passes.size();
    if (n_segments) *n_segments = (int)P.segs.size();
    if (tile_qubits) *tile_qubits = P.L;
  });
}

nt_status nt_plan_ops(const nt_circuit *c, int prec, int64_t *n_ops, int64_t *n_fused) {
  if (!c) return fail(NT_ERR_INVALID_ARG, "circuit is NULL");
  if (prec != NT_C64 && prec != NT_C128) return fail(NT_ERR_INVALID_ARG, "precision must be NT_C64 or NT_C128");
  return guard([&] {
    nt::Plan P = nt::choose_plan(*c->impl, prec);
    if (n_ops) *n_ops = (int64_t)P.ops.size();
    if (n_fused) *n_fused = P.n_fused + P.n_diag + P.n_layer;
  });
}

nt_status nt_plan_export(const nt_circuit *c, int prec, int32_t *op_gate, int32_t *op_pass, int32_t *op_segment,
                         uint64_t *pass_local_mask, uint64_t *segment_reg_mask) {
  if (!c) return fail(NT_ERR_INVALID_ARG, "circuit is NULL");
  if (prec != NT_C64 && prec != NT_C128) return fail(NT_ERR_INVALID_ARG, "precision must be NT_C64 or NT_C128");
  return guard([&] {
    nt::Plan P = nt::choose_plan(*c->impl, prec);
    size_t k = 0;   // gates in application order
    for (size_t p = 0; p < P.passes.size(); ++p) {
      const nt::Pass &ps = P.passes[p];
      if (pass_local_mask) pass_local_mask[p] = ps.local_mask;
      for (int s = ps.seg_begin; s < ps.seg_end; ++s) {
        const nt::Segment &sg = P.segs[s];
        uint64_t m = 0;
        for (int q : sg.reg_q) m |= 1ull << q;
        if (segment_reg_mask) segment_reg_mask[s] = m;
        for (int o = sg.op_begin; o < sg.op_end; ++o) {
          const nt::HostOp &h = P.ops[o];
          for (int g : h.gates()) {   // a fused block: its gates in order
            if (op_gate) op_gate[k] = g;
            if (op_pass) op_pass[k] = (int32_t)p;
            if (op_segment) op_segment[k] = s;
            ++k;
          }
        }
      }
    }
  });
}

static nt_status check_run_args(nt_ctx *ctx, const nt_circuit *c, double tau) {
  if (!ctx) return fail(NT_ERR_INVALID_ARG, "ctx is NULL");
  if (!c) return fail(NT_ERR_INVALID_ARG, "circuit is NULL");
  if (!std::isfinite(tau)) return fail(NT_ERR_INVALID_ARG, "tau must be finite");
  return NT_OK;
}

nt_status nt_run(nt_ctx *ctx, const nt_circuit *c, uint64_t seed, uint64_t traj_begin, uint64_t n_traj,
                 double tau, double *fid_out, uint64_t *count_out, double *p_out) {
  nt_status s = check_run_args(ctx, c, tau);
  if (s) return s;
  if (n_traj == 0) return fail(NT_ERR_INVALID_ARG, "n_traj must be > 0");
  return guard([&] {
    nt::Ctx &cx = *ctx->impl;
    uint64_t cnt = 0;
    double sum = 0;
    const bool fidc = cx.crit == NT_CRIT_FIDELITY;
    cx.run(*c->impl, seed, traj_begin, n_traj, tau, fid_out, &cnt, (p_out && !fidc) ? &sum : nullptr);
    if (count_out) *count_out = cnt;
    if (p_out) *p_out = fidc ? (double)cnt / (double)n_traj : sum / (double)n_traj;
  });
}

nt_status nt_run_noalloc(nt_ctx *ctx, const nt_circuit *c, uint64_t seed, uint64_t traj_begin, uint64_t n_traj,
                         double tau, double *fid_out, uint64_t *count_out, double *p_out) {
  nt_status s = check_run_args(ctx, c, tau);
  if (s) return s;
  if (n_traj == 0) return fail(NT_ERR_INVALID_ARG, "n_traj must be > 0");
  return guard([&] {
    nt::Ctx &cx = *ctx->impl;
    uint64_t cnt = 0;
    double sum = 0;
    const bool fidc = cx.crit == NT_CRIT_FIDELITY;
    cx.run_noalloc(*c->impl, seed, traj_begin, n_traj, tau, fid_out, &cnt, (p_out && !fidc) ? &sum : nullptr);
    if (count_out) *count_out = cnt;
    if (p_out) *p_out = fidc ? (double)cnt / (double)n_traj : sum / (double)n_traj;
  });
}

nt_status nt_run_batch(nt_ctx *ctx, const nt_circuit *const *circuits, int n_circ, uint64_t seed,
                       uint64_t traj_begin, uint64_t n_traj, double tau, double *vals_out, uint64_t *count_out,
                       double *p_out) {
  if (!ctx) return fail(NT_ERR_INVALID_ARG, "ctx is NULL");
  if (n_circ <= 0 || !circuits) return fail(NT_ERR_INVALID_ARG, "need n_circ > 0 circuits");
  for (int i = 0; i < n_circ; ++i) {
    nt_status s = check_run_args(ctx, circuits[i], tau);
    if (s) return s;
  }
  if (n_traj == 0) return fail(NT_ERR_INVALID_ARG, "n_traj must be > 0");
  if ((uint64_t)n_circ * n_traj > ((uint64_t)1 << 32)) return fail(NT_ERR_INVALID_ARG, "n_circ * n_traj too large");
  return guard([&] {
    nt::Ctx &cx = *ctx->impl;
    std::vector<const nt::Circuit *> cs(n_circ);
    for (int i = 0; i < n_circ; ++i) cs[i] = circuits[i]->impl;
    std::vector<uint64_t> cnt(n_circ);
    std::vector<double> sum(n_circ);
    const bool fidc = cx.crit == NT_CRIT_FIDELITY;
    cx.run_batch(cs, seed, traj_begin, n_traj, tau, vals_out, cnt.data(), (p_out && !fidc) ? sum.data() : nullptr);
    if (count_out) std::memcpy(count_out, cnt.data(), n_circ * sizeof(uint64_t));
    if (p_out)
      for (int i = 0; i < n_circ; ++i) p_out[i] = fidc ? (double)cnt[i] / (double)n_traj : sum[i] / (double)n_traj;
  });
}

nt_status nt_sweep(nt_ctx *ctx, const nt_circuit *c, const double *rates, int R, uint64_t seed, uint64_t n_traj,
                   double tau, double *p_out) {
  nt_status s = check_run_args(ctx, c, tau);
  if (s) return s;
  if (R < 0 || (R > 0 && (!rates || !p_out))) return fail(NT_ERR_INVALID_ARG, "bad rates / p_out");
  if (n_traj == 0) return fail(NT_ERR_INVALID_ARG, "n_traj must be > 0");
  for (int r = 0; r < R; ++r)
    if (!valid_prob(rates[r])) return fail(NT_ERR_INVALID_ARG, "rates must be in [0, 1]");
  return guard([&] {
    nt::Ctx &cx = *ctx->impl;
    const double spx = cx.px, spy = cx.py, spz = cx.pz;
    try {
      for (int r = 0; r < R; ++r) {
        const double p3 = rates[r] / 3.0;
        cx.px = cx.py = cx.pz = p3;
        p_out[r] = cx.success(*c->impl, seed, 0, n_traj, tau);
      }
    } catch (...) {
      cx.px = spx; cx.py = spy; cx.pz = spz;
      throw;
    }
    cx.px = spx; cx.py = spy; cx.pz = spz;
  });
}

nt_status nt_sweep_crossing(nt_ctx *ctx, const nt_circuit *c, const double *rates, int R, uint64_t seed,
                           uint64_t n_traj, double tau, double P_target, double *p_out, double *p_star) {
  if (R < 1 || !rates || !p_star) return fail(NT_ERR_INVALID_ARG, "need R >= 1 rates and p_star");
  for (int r = 1; r < R; ++r)
    if (!(rates[r] > rates[r - 1])) return fail(NT_ERR_INVALID_ARG, "rates must be ascending");
  if (!(rates[0] > 0)) return fail(NT_ERR_INVALID_ARG, "rates must be > 0");
  std::vector<double> P(R, 0.0);
  nt_status s = nt_sweep(ctx, c, rates, R, seed, n_traj, tau, P.data());
  if (s) return s;
  if (p_out) std::copy(P.begin(), P.end(), p_out);
  // the rate where the curve, linear in log10 p between grid points, first
  // falls below the target
  *p_star = P[0] < P_target ? rates[0] : rates[R - 1];
  for (int k = 0; k + 1 < R; ++k) {
    if (P[k] >= P_target && P_target > P[k + 1]) {
      const double x0 = std::log10(rates[k]), x1 = std::log10(rates[k + 1]);
      const double t = (P[k] - P_target) / (P[k] - P[k + 1]);
      *p_star = std::pow(10.0, x0 + t * (x1 - x0));
      break;
    }
  }
  return NT_OK;
}

nt_status nt_tolerable_rate(nt_ctx *ctx, const nt_circuit *c, double P_target, double tol, double p_lo,
                            double p_hi, uint64_t seed, uint64_t n_traj, double tau, double *p_star,
                            int *n_probes) {
  nt_status s = check_run_args(ctx, c, tau);
  if (s) return s;
  if (!p_star) return fail(NT_ERR_INVALID_ARG, "p_star is NULL");
  if (!(P_target >= 0 && P_target <= 1) || !(tol >= 0)) return fail(NT_ERR_INVALID_ARG, "bad P_target / tol");
  if (!(p_lo > 0) || !(p_hi <= 1) || !(p_lo < p_hi)) return fail(NT_ERR_INVALID_ARG, "need 0 < p_lo < p_hi <= 1");
  if (n_traj == 0) return fail(NT_ERR_INVALID_ARG, "n_traj must be > 0");
  int probes = 0;
  bool bracketed = true;
  nt_status st = guard([&] {
    nt::Ctx &cx = *ctx->impl;
    const double spx = cx.px, spy = cx.py, spz = cx.pz;
    auto P_at = [&](double p) {
      cx.px = cx.py = cx.pz = p / 3.0;
      ++probes;
      return cx.success(*c->impl, seed, 0, n_traj, tau);
    };
    try {
      // Safeguarded regula falsi (Illinois) in x = log10 p on
      // f(x) = P(10^x) - P_target, same trajectories at every probe.
      double a = std::log10(p_lo), b = std::log10(p_hi);
      double fa = P_at(p_lo) - P_target;
      double fb = P_at(p_hi) - P_target;
      if (fa < 0 || fb > 0) {
        bracketed = false;
      } else {
        int side = 0;
        for (;;) {
          if (std::pow(10.0, b - a) <= 1.001) { *p_star = std::pow(10.0, 0.5 * (a + b)); break; }
          double x = (fa == fb) ? 0.5 * (a + b) : (a * fb - b * fa) / (fb - fa);
          if (!(x > a && x < b)) x = 0.5 * (a + b);
          const double px = std::pow(10.0, x);
          const double fx = P_at(px) - P_target;
          if (std::fabs(fx) <= tol) { *p_star = px; break; }
          if (fx > 0) {
            a = x; fa = fx;
            if (side == 1) fb *= 0.5;
            side = 1;
          } else {
            b = x; fb = fx;
            if (side == -1) fa *= 0.5;
            side = -1;
          }
        }
      }
    } catch (...) {
      cx.px = spx; cx.py = spy; cx.pz = spz;
      throw;
    }
    cx.px = spx; cx.py = spy; cx.pz = spz;
  });
  if (n_probes) *n_probes = probes;
  if (st) return st;
  if (!bracketed) return fail(NT_ERR_NOT_BRACKETED, "target success probability not bracketed by [p_lo, p_hi]");
  return NT_OK;
}

nt_status nt_tolerable_rate_auto(nt_ctx *ctx, const nt_circuit *c, double P_target, double tol, uint64_t seed,
                                 uint64_t n_traj, double tau, double *p_star, int *n_coarse, int *n_full,
                                 double bracket_out[2]) {
  nt_status s = check_run_args(ctx, c, tau);
  if (s) return s;
  if (!p_star) return fail(NT_ERR_INVALID_ARG, "p_star is NULL");
  if (!(P_target > 0 && P_target < 1) || !(tol >= 0)) return fail(NT_ERR_INVALID_ARG, "need 0 < P_target < 1, tol >= 0");
  if (n_traj == 0) return fail(NT_ERR_INVALID_ARG, "n_traj must be > 0");
  const double S = (double)std::max<int64_t>(c->impl->S, 1), G = (double)std::max<size_t>(c->impl->gates.size(), 1);
  const double p0 = 1.0 - std::pow(P_target, 1.0 / S);
  const double lo0 = std::max(1e-6, 0.5 * p0), pmax = 0.5;
  const double wide[4][2] = {{lo0, std::min(2.0 * p0, 1.0 / G)}, {lo0, 1.0 / G}, {1e-6, 1.0 / G}, {1e-6, pmax}};
  int kc = 0, kf = 0;
  double br[2] = {0.0, 0.0};
  auto finish = [&](nt_status st) {
    if (n_coarse) *n_coarse = kc;
    if (n_full) *n_full = kf;
    if (bracket_out) {
      bracket_out[0] = br[0];
      bracket_out[1] = br[1];
    }
    return st;
  };
  // nt_tolerable_rate over a list of brackets until one holds the target
  auto search = [&](const double (*tries)[2], int nt, uint64_t n, int *k) -> nt_status {
    nt_status st = NT_ERR_NOT_BRACKETED;
    for (int i = 0; i < nt && st == NT_ERR_NOT_BRACKETED; ++i) {
      if (!(tries[i][0] > 0 && tries[i][0] < tries[i][1] && tries[i][1] <= 1)) continue;
      br[0] = tries[i][0];
      br[1] = tries[i][1];
      int pr = 0;
      st = nt_tolerable_rate(ctx, c, P_target, tol, br[0], br[1], seed, n, tau, p_star, &pr);
      *k += pr;
    }
    return st;
  };
  const uint64_t nc = std::max<uint64_t>(1, n_traj / 5);
  s = search(wide, 4, nc, &kc);
  if (s) return finish(s);
  const double pc = *p_star, bc0 = br[0], bc1 = br[1];
  double Pc = 0.0;
  s = nt_sweep(ctx, c, &pc, 1, seed, n_traj, tau, &Pc);
  if (s) return finish(s);
  ++kf;
  if (std::fabs(Pc - P_target) <= tol) {
    *p_star = pc;
    br[0] = br[1] = pc;
    return finish(NT_OK);
  }
  double side[1][2] = {{0.0, 0.0}};
  bool have_side = false;
  double Pb[2] = {0.0, 0.0};
  const double bce[2] = {bc0, bc1};
  s = nt_sweep(ctx, c, bce, 2, seed, nc, tau, Pb);
  if (s) return finish(s);
  kc += 2;
  const double slope = (Pb[0] - Pb[1]) / (std::log10(bc1) - std::log10(bc0));
  if (slope > 0) {
    const double p1 = std::min(pmax, std::max(1e-6, pc * std::pow(10.0, (Pc - P_target) / slope)));
    double P1 = 0.0;
    s = nt_sweep(ctx, c, &p1, 1, seed, n_traj, tau, &P1);
    if (s) return finish(s);
    ++kf;
    if (std::fabs(P1 - P_target) <= tol) {
      *p_star = p1;
      br[0] = br[1] = p1;
      return finish(NT_OK);
    }
    if ((P1 - P_target) * (Pc - P_target) < 0) {
      side[0][0] = std::min(pc, p1);
      side[0][1] = std::max(pc, p1);
      have_side = true;
    }
  }
  if (!have_side) {
    const double f = std::pow(10.0, 0.1);
    side[0][0] = Pc > P_target ? pc : std::max(1e-6, pc / f);
    side[0][1] = Pc > P_target ? std::min(pmax, pc * f) : pc;
  }
  s = search(side, 1, n_traj, &kf);
  if (s == NT_ERR_NOT_BRACKETED) s = search(wide, 4, n_traj, &kf);
  return finish(s);
}

nt_status nt_tolerable_rate_fig3(nt_ctx *ctx, const nt_circuit *c, double P_target, double tol, uint64_t seed,
                                 uint64_t n_traj, double tau, double *p_star, int *method, int *n_probes,
                                 double P_single[4]) {
  nt_status s = check_run_args(ctx, c, tau);
  if (s) return s;
  if (!p_star) return fail(NT_ERR_INVALID_ARG, "p_star is NULL");
  if (!(P_target > 0 && P_target < 1) || !(tol >= 0)) return fail(NT_ERR_INVALID_ARG, "need 0 < P_target < 1, tol >= 0");
  if (n_traj == 0) return fail(NT_ERR_INVALID_ARG, "n_traj must be > 0");
  if (ctx->impl->crit != NT_CRIT_FIDELITY)
    return fail(NT_ERR_UNSUPPORTED, "the tolerable-rate steps use the fidelity criterion");
  int probes = 0, meth = -1;
  if (n_probes) *n_probes = 0;
  if (c->impl->S == 0) return fail(NT_ERR_NOT_BRACKETED, "a circuit without error sites has no tolerable rate");
  // 1. exhaustive single-error simulation (Sec. IV-B.1)
  double P_e[3] = {0, 0, 0}, P_R = 0;
  s = guard([&] { ctx->impl->exhaustive(*c->impl, tau, nullptr, P_e, &P_R); });
  if (s) return s;
  if (P_single) {
    P_single[0] = P_e[0]; P_single[1] = P_e[1]; P_single[2] = P_e[2]; P_single[3] = P_R;
  }
  if (method) *method = -1;
  if (P_R < P_target) return fail(NT_ERR_NOT_BRACKETED, "the error-free state misses the target");
  const double S = (double)c->impl->S;
  // 2. success at one average error: Eq. 4 with E(N_e) = 1/3 per type
  const double P1 = (P_e[0] + P_e[1] + P_e[2]) / 3.0;
  if (P1 <= P_target && P1 != P_R) {
    // 3. at most one error is tolerable: Eq. 5 over the S error locations
    s = nt_eq5(P_target, P_e, P_R, S, p_star);
    if (s) return s;
    if (method) *method = 0;
    return NT_OK;
  }
  // 4. Monte Carlo at increasing rates 2^k / S while the success stays at or
  // above the target (decreasing by halves when it is already below at 1/S),
  // then the search between the last two rates
  meth = 1;
  if (method) *method = meth;
  auto P_at = [&](double p, double *P) {
    ++probes;
    return nt_sweep(ctx, c, &p, 1, seed, n_traj, tau, P);
  };
  auto done = [&](nt_status st) {
    if (n_probes) *n_probes = probes;
    return st;
  };
  double p = 1.0 / S, P = 0.0, lo = 0.0, hi = 0.0;
  s = P_at(p, &P);
  if (s) return done(s);
  if (std::fabs(P - P_target) <= tol) {
    *p_star = p;
    return done(NT_OK);
  }
  if (P >= P_target) {
    for (;;) {
      lo = p;
      p *= 2.0;
      if (p > 0.5) return done(fail(NT_ERR_NOT_BRACKETED, "success stays above the target up to p = 0.5"));
      s = P_at(p, &P);
      if (s) return done(s);
      if (std::fabs(P - P_target) <= tol) {
        *p_star = p;
        return done(NT_OK);
      }
      if (P < P_target) {
        hi = p;
        break;
      }
    }
  } else {
    for (;;) {
      hi = p;
      p *= 0.5;
      if (p < 1e-9) return done(fail(NT_ERR_NOT_BRACKETED, "success stays below the target down to p = 1e-9"));
      s = P_at(p, &P);
      if (s) return done(s);
      if (std::fabs(P - P_target) <= tol) {
        *p_star = p;
        return done(NT_OK);
      }
      if (P >= P_target) {
        lo = p;
        break;
      }
    }
  }
  int k = 0;
  s = nt_tolerable_rate(ctx, c, P_target, tol, lo, hi, seed, n_traj, tau, p_star, &k);
  probes += k;
  return done(s);
}

nt_status nt_set_shortcuts(nt_ctx *ctx, int flags) {
  if (!ctx) return fail(NT_ERR_INVALID_ARG, "ctx is NULL");
  if (flags & ~(NT_SHORTCUT_ZERO_FIRED | NT_SHORTCUT_CHECKPOINT | NT_SHORTCUT_LAST_ERROR | NT_SHORTCUT_REUSE))
    return fail(NT_ERR_INVALID_ARG, "unknown shortcut flag");
  ctx->impl->shortcuts = flags;
  // every call empties the reuse store
  ctx->impl->reuse.clear();
  ctx->impl->reuse_values = 0;
  ctx->impl->reuse_valid = false;
  g_last_error.clear();
  return NT_OK;
}

nt_status nt_set_criterion(nt_ctx *ctx, int criterion, uint64_t target) {
  if (!ctx) return fail(NT_ERR_INVALID_ARG, "ctx is NULL");
  if (criterion != NT_CRIT_FIDELITY && criterion != NT_CRIT_TARGET_PROB && criterion != NT_CRIT_HEAVY)
    return fail(NT_ERR_INVALID_ARG, "unknown criterion");
  if (criterion == NT_CRIT_TARGET_PROB && (target >> 32) != 0)
    return fail(NT_ERR_INVALID_ARG, "target basis state beyond 32 qubits");
  ctx->impl->crit = criterion;
  ctx->impl->target = criterion == NT_CRIT_TARGET_PROB ? target : 0;
  g_last_error.clear();
  return NT_OK;
}

nt_status nt_exhaustive(nt_ctx *ctx, const nt_circuit *c, double tau, double *fid_out, double P_e[3],
                        double *P_R) {
  nt_status s = check_run_args(ctx, c, tau);
  if (s) return s;
  if (!P_e || !P_R) return fail(NT_ERR_INVALID_ARG, "P_e / P_R is NULL");
  return guard([&] { ctx->impl->exhaustive(*c->impl, tau, fid_out, P_e, P_R); });
}

nt_status nt_eq4(const double P_e[3], double P_R, const double E_e[3], double *P) {
  if (!P_e || !E_e || !P) return fail(NT_ERR_INVALID_ARG, "NULL argument");
  double sum = 0, se = 0;
  for (int e = 0; e < 3; ++e) {
    sum += P_e[e] * E_e[e];
    se += E_e[e];
  }
  *P = sum + P_R * (1.0 - se);
  g_last_error.clear();
  return NT_OK;
}

nt_status nt_eq5(double P_target, const double P_e[3], double P_R, double units, double *p) {
  if (!P_e || !p) return fail(NT_ERR_INVALID_ARG, "NULL argument");
  if (!(units > 0)) return fail(NT_ERR_INVALID_ARG, "units must be > 0");
  const double avg = (P_e[0] + P_e[1] + P_e[2]) / 3.0;
  if (avg == P_R) return fail(NT_ERR_INVALID_ARG, "single errors do not change the success probability");
  *p = (P_target - P_R) / (avg - P_R) / units;
  g_last_error.clear();
  return NT_OK;
}

nt_status nt_success_probability(nt_ctx *ctx, const nt_circuit *c, uint64_t seed, uint64_t n_traj, double tau,
                                 double *P, int *method) {
  nt_status s = check_run_args(ctx, c, tau);
  if (s) return s;
  if (!P) return fail(NT_ERR_INVALID_ARG, "P is NULL");
  return guard([&] {
    nt::Ctx &cx = *ctx->impl;
    const double S = (double)c->impl->S;
    const double EN = S * (cx.px + cx.py + cx.pz);
    if (EN <= 1.0) {
      double P_e[3], P_R;
      cx.exhaustive(*c->impl, tau, nullptr, P_e, &P_R);
      // Pauli types in the order X, Y, Z
      const double E_e[3] = {S * cx.px, S * cx.py, S * cx.pz};
      double sum = 0, se = 0;
      for (int e = 0; e < 3; ++e) {
        sum += P_e[e] * E_e[e];
        se += E_e[e];
      }
      *P = sum + P_R * (1.0 - se);
      if (method) *method = 0;
    } else {
      if (n_traj == 0) throw nt::Error(NT_ERR_INVALID_ARG, "n_traj must be > 0 for the Monte Carlo branch");
      *P = cx.success(*c->impl, seed, 0, n_traj, tau);
      if (method) *method = 1;
    }
  });
}

nt_status nt_sample_sites(nt_ctx *ctx, const nt_circuit *c, uint64_t seed, uint64_t traj_begin, uint64_t n_traj,
                          uint64_t *offsets, int32_t *sites, uint8_t *paulis, int64_t cap, int64_t *n_out) {
  if (!ctx || !c) return fail(NT_ERR_INVALID_ARG, "ctx / circuit is NULL");
  if (!offsets || !n_out || cap < 0 || (cap > 0 && (!sites || !paulis)))
    return fail(NT_ERR_INVALID_ARG, "bad output buffers");
  return guard([&] { ctx->impl->sample_sites(*c->impl, seed, traj_begin, n_traj, offsets, sites, paulis, cap, n_out); });
}

nt_status nt_final_state(nt_ctx *ctx, const nt_circuit *c, uint64_t seed, uint64_t traj, void *amps_out,
                         int64_t len) {
  if (!ctx || !c) return fail(NT_ERR_INVALID_ARG, "ctx / circuit is NULL");
  if (!amps_out) return fail(NT_ERR_INVALID_ARG, "amps_out is NULL");
  return guard([&] { ctx->impl->final_state(*c->impl, seed, traj, amps_out, len); });
}

nt_status nt_reference_state(nt_ctx *ctx, const nt_circuit *c, void *amps_out, int64_t len) {
  if (!ctx || !c) return fail(NT_ERR_INVALID_ARG, "ctx / circuit is NULL");
  if (!amps_out) return fail(NT_ERR_INVALID_ARG, "amps_out is NULL");
  return guard([&] { ctx->impl->reference_state(*c->impl, amps_out, len); });
}

nt_status nt_timing_enable(nt_ctx *ctx, int enable) {
  if (!ctx) return fail(NT_ERR_INVALID_ARG, "ctx is NULL");
  return guard([&] {
    if (!enable) ctx->impl->timing_flush();
    ctx->impl->timing = enable != 0;
  });
}

nt_status nt_timing_reset(nt_ctx *ctx) {
  if (!ctx) return fail(NT_ERR_INVALID_ARG, "ctx is NULL");
  return guard([&] {
    nt::Ctx &cx = *ctx->impl;
    cx.timing_flush();
    cx.t_launches = 0;
    cx.t_ms = cx.t_bytes = cx.t_updates = cx.t_flops = 0;
  });
}

nt_status nt_timing_read(nt_ctx *ctx, int64_t *n_launches, double *ms_total, double *bytes_total,
                         double *updates_total, double *flops_total) {
  if (!ctx) return fail(NT_ERR_INVALID_ARG, "ctx is NULL");
  return guard([&] {
    nt::Ctx &cx = *ctx->impl;
    cx.timing_flush();
    if (n_launches) *n_launches = cx.t_launches;
    if (ms_total) *ms_total = cx.t_ms;
    if (bytes_total) *bytes_total = cx.t_bytes;
    if (updates_total) *updates_total = cx.t_updates;
    if (flops_total) *flops_total = cx.t_flops;
  });
}


nt_status nt_gnn_create(nt_ctx *ctx, uint64_t seed, nt_gnn **out) {
  if (!ctx || !out) return fail(NT_ERR_INVALID_ARG, "ctx / out is NULL");
  *out = nullptr;
  return guard([&] {
    check_hip_entry(ctx);
    auto *m = new nt_gnn{ctx, new gnn::Model(ctx->impl, seed)};
    *out = m;
  });
}

void nt_gnn_destroy(nt_gnn *m) {
  if (!m) return;
  (void)hipSetDevice(m->ctx->impl->device);
  delete m->impl;
  delete m;
}

nt_status nt_gnn_graph(const nt_circuit *c, float *x, int32_t *row_ptr, int32_t *col, float *glob, int64_t *n_nodes,
                       int64_t *n_edges) {
  if (!c || !n_nodes || !n_edges) return fail(NT_ERR_INVALID_ARG, "NULL argument");
  return guard([&] {
    const gnn::Graph g = gnn::build_graph(*c->impl);
    *n_nodes = g.n_nodes;
    *n_edges = (int64_t)g.col.size();
    if (x) std::memcpy(x, g.x.data(), g.x.size() * sizeof(float));
    if (row_ptr) std::memcpy(row_ptr, g.row_ptr.data(), g.row_ptr.size() * sizeof(int32_t));
    if (col && !g.col.empty()) std::memcpy(col, g.col.data(), g.col.size() * sizeof(int32_t));
    if (glob) std::memcpy(glob, g.glob, sizeof g.glob);
  });
}

nt_status nt_gnn_params(nt_gnn *m, float *out, int64_t *len) {
  if (!m || !len) return fail(NT_ERR_INVALID_ARG, "NULL argument");
  return guard([&] {
    *len = (int64_t)m->impl->lay.total;
    if (out) {
      check_hip_entry(m->ctx);
      nt::check_hip(hipMemcpy(out, m->impl->params.p, m->impl->lay.total * 4, hipMemcpyDeviceToHost), "copy params");
    }
  });
}

nt_status nt_gnn_set_params(nt_gnn *m, const float *in, int64_t len) {
  if (!m || !in) return fail(NT_ERR_INVALID_ARG, "NULL argument");
  if (len != (int64_t)m->impl->lay.total) return fail(NT_ERR_INVALID_ARG, "parameter vector has the wrong length");
  return guard([&] {
    check_hip_entry(m->ctx);
    nt::check_hip(hipMemcpy(m->impl->params.p, in, (size_t)len * 4, hipMemcpyHostToDevice), "copy params");
  });
}

static std::vector<gnn::Graph> graphs_of(const nt_circuit *const *cs, int n) {
  std::vector<gnn::Graph> gs;
  gs.reserve(n);
  for (int i = 0; i < n; ++i) {
    if (!cs[i]) throw nt::Error(NT_ERR_INVALID_ARG, "circuit is NULL");
    gs.push_back(gnn::build_graph(*cs[i]->impl));
    if (gs.back().n_nodes == 0) throw nt::Error(NT_ERR_INVALID_ARG, "circuit without gates");
  }
  return gs;
}

nt_status nt_gnn_set_data(nt_gnn *m, const nt_circuit *const *circuits, int n, const float *labels) {
  if (!m || !circuits || n <= 0) return fail(NT_ERR_INVALID_ARG, "need n > 0 circuits");
  return guard([&] {
    check_hip_entry(m->ctx);
    const std::vector<gnn::Graph> gs = graphs_of(circuits, n);
    m->impl->data.upload(gs, labels, m->ctx->impl->stream);
  });
}

nt_status nt_gnn_loss_grad(nt_gnn *m, int g0, int g1, int exact, double *loss, float *grad) {
  if (!m) return fail(NT_ERR_INVALID_ARG, "model is NULL");
  if (g0 < 0 || g1 <= g0 || g1 > m->impl->data.n_graphs) return fail(NT_ERR_INVALID_ARG, "bad graph range");
  return guard([&] {
    check_hip_entry(m->ctx);
    const double l = m->impl->loss_backward(m->impl->data, g0, g1, exact == 0);
    if (loss) *loss = l;
    if (grad)
      nt::check_hip(hipMemcpy(grad, m->impl->grads.p, m->impl->lay.total * 4, hipMemcpyDeviceToHost), "copy grads");
  });
}

nt_status nt_gnn_train(nt_gnn *m, int epochs, int batch_graphs, double lr, uint64_t seed, double *loss_out) {
  if (!m) return fail(NT_ERR_INVALID_ARG, "model is NULL");
  if (epochs < 0 || batch_graphs <= 0 || !(lr > 0)) return fail(NT_ERR_INVALID_ARG, "bad training settings");
  if (m->impl->data.n_graphs == 0 || !m->impl->data.has_labels) return fail(NT_ERR_INVALID_ARG, "no labelled data");
  return guard([&] {
    check_hip_entry(m->ctx);
    for (int e = 0; e < epochs; ++e) {
      const double l = m->impl->train_epoch(batch_graphs, lr, seed + (uint64_t)e * 0x9E3779B97F4A7C15ull);
      if (loss_out) loss_out[e] = l;
    }
  });
}

nt_status nt_gnn_predict(nt_gnn *m, const nt_circuit *const *circuits, int n, int exact, float *out) {
  if (!m || !circuits || n <= 0 || !out) return fail(NT_ERR_INVALID_ARG, "NULL argument or n <= 0");
  return guard([&] {
    check_hip_entry(m->ctx);
    gnn::Dataset ds;
    ds.upload(graphs_of(circuits, n), nullptr, m->ctx->impl->stream);
    const int chunk = 256;
    for (int g0 = 0; g0 < n; g0 += chunk) {
      const int g1 = std::min(n, g0 + chunk);
      m->impl->forward(ds, g0, g1, exact == 0);
      nt::check_hip(hipMemcpyAsync(out + (size_t)g0 * gnn::OUT, m->impl->v.p, (size_t)(g1 - g0) * gnn::OUT * 4,
                                   hipMemcpyDeviceToHost, m->ctx->impl->stream), "copy predictions");
      nt::check_hip(hipStreamSynchronize(m->ctx->impl->stream), "hipStreamSynchronize");
    }
  });
}

nt_status nt_tolerable_rate_guided(nt_ctx *ctx, const nt_circuit *c, nt_gnn *m, double P_target, double tol,
                                   uint64_t seed, uint64_t n_traj, double tau, double *p_star, int *n_probes,
                                   double bracket_out[2]) {
  nt_status s = check_run_args(ctx, c, tau);
  if (s) return s;
  if (!m || !p_star) return fail(NT_ERR_INVALID_ARG, "model / p_star is NULL");
  float pred[gnn::OUT];
  s = nt_gnn_predict(m, &c, 1, 0, pred);
  if (s) return s;
  const double grid_lo = gnn::output_rate(0), grid_hi = gnn::output_rate(gnn::OUT - 1);
  // first grid interval [j, j + 1] where the predicted curve falls through P_target
  int j = -1;
  for (int k = 0; k + 1 < gnn::OUT; ++k)
    if (pred[k] >= P_target && pred[k + 1] < P_target) {
      j = k;
      break;
    }
  int probes = 0, pr = 0;
  double lo = grid_lo, hi = grid_hi;
  if (j < 0) {
    s = nt_tolerable_rate(ctx, c, P_target, tol, lo, hi, seed, n_traj, tau, p_star, &pr);
    probes += pr;
  } else {
    // 1. One Monte Carlo probe at the predicted crossing (linear in log10 p
    //    between the two grid points); done if it meets the tolerance.
    const double x0 = std::log10(gnn::output_rate(j)), x1 = std::log10(gnn::output_rate(j + 1));
    const double t = ((double)pred[j] - P_target) / ((double)pred[j] - (double)pred[j + 1]);
    const double ph = std::pow(10.0, x0 + t * (x1 - x0));
    double Ph = 0.0;
    s = nt_sweep(ctx, c, &ph, 1, seed, n_traj, tau, &Ph);
    if (s) {
      if (n_probes) *n_probes = 0;
      return s;
    }
    probes = 1;
    lo = hi = ph;
    if (std::fabs(Ph - P_target) <= tol) {
      *p_star = ph;
      s = NT_OK;
    } else {
      // 2. Half a grid step from the probe, on the side its value points
      //    to; 3. the grid interval widened by one step per side; 4. the
      //    whole grid.  Rates probed before are evaluated again (from the
      //    stored trajectory values when NT_SHORTCUT_REUSE is on).
      const double half = std::pow(10.0, 0.125);
      double tries[3][2] = {{Ph > P_target ? ph : std::max(grid_lo, ph / half),
                             Ph > P_target ? std::min(grid_hi, ph * half) : ph},
                            {gnn::output_rate(std::max(0, j - 1)), gnn::output_rate(std::min(gnn::OUT - 1, j + 2))},
                            {grid_lo, grid_hi}};
      s = NT_ERR_NOT_BRACKETED;
      for (int k = 0; k < 3 && s == NT_ERR_NOT_BRACKETED; ++k) {
        if (!(tries[k][0] < tries[k][1])) continue;
        lo = tries[k][0];
        hi = tries[k][1];
        pr = 0;
        s = nt_tolerable_rate(ctx, c, P_target, tol, lo, hi, seed, n_traj, tau, p_star, &pr);
        probes += pr;
      }
    }
  }
  if (n_probes) *n_probes = probes;
  if (bracket_out) {
    bracket_out[0] = lo;
    bracket_out[1] = hi;
  }
  return s;
}

}  // extern "C"
