// Host engine of libnisqtol: owns device buffers, uploads plans, sequences
// kernel launches on the context stream.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <unordered_map>
#include <memory>
#include <vector>

#include "kernels.hpp"
#include "nt_internal.hpp"

namespace nt {

// A bump allocator over caller-provided device memory (the static scratch
// array of the allocation-free entry point): regions are 256-byte aligned and
// only handed out, never freed; running out is an error, not an allocation.
struct Arena {
  char *base = nullptr;
  size_t cap = 0, off = 0;
  void *take(size_t n);
};

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  Arena *arena = nullptr;      // when set, space comes from the arena (no hipMalloc)
  ~DevBuf();
  void ensure(size_t n);       // grows (never shrinks); contents not kept
  void release();
  template <typename X> X *as() const { return static_cast<X *>(p); }
};

// Device copy of a plan for one precision, plus the cached reference state.
struct DevPlan {
  int prec = 0;
  Plan plan;
  int nthreads = 0;            // threads per work-group = 2^(L - R)
  DevBuf ops, aux, segs, passes, app_order, app_tag, site_order, site_tag;
  DevBuf ref, nref, ref_partials;
  bool ref_ready = false;
  DevBuf ckpt;                 // error-free state before passes 1..np-1
  DevBuf ckpt_partials, nref_pass;   // norms of the error-free state after each pass
  bool ckpt_ready = false;
  double nref_host = 0;        // <R|R>, copied once the reference is built
  double heavy_med = 0;        // median of the error-free probabilities (heavy criterion)
  bool med_ready = false;
  // criterion value of the error-free state, keyed by (criterion, target)
  std::map<std::pair<int, uint64_t>, double> ref_value;
  std::vector<int> pass_of_op;
  std::vector<double> pass_flops_per_amp;   // algorithmic flops per amplitude, per pass
  std::vector<int> pass_gates;              // circuit gates applied by each pass
  uint64_t last_use = 0;       // plan cache: least recently used goes first
  int pins = 0;                // > 0 while a batched run holds it
  size_t footprint() const { return ref.bytes + ckpt.bytes + ckpt_partials.bytes + ref_partials.bytes; }
};

// Arguments of one run of all passes over a batch (engine.cpp).
struct PassRun {
  int B = 0;
  int last_flags = 0;
  const uint32_t *events = nullptr;
  const int32_t *ev_count = nullptr;
  int ev_stride = 1;
  double *partials = nullptr;
  uint32_t *frames = nullptr;
  const int32_t *start = nullptr;            // device: first pass per entry (sorted), or NULL
  const std::vector<int> *active = nullptr;  // per pass: entries with start <= p
  const int32_t *end = nullptr;              // device: pass after which each entry is scored, or NULL
  bool capture = false;                      // copy the state into the checkpoints after each pass
  int crit = 0;                              // success criterion of the scoring pass
  uint32_t target = 0;
  double heavy_med = 0;
};

// Shortcut flags (nt_set_shortcuts).
enum : int { SC_ZERO_FIRED = 1, SC_CHECKPOINT = 2, SC_LAST_ERROR = 4, SC_REUSE = 8 };

// Identity of the runs whose trajectory values may be reused
// (NT_SHORTCUT_REUSE): everything a value depends on except the rate.
struct ReuseKey {
  uint64_t serial = 0, cid = 0, seed = 0, target = 0, c_x = 0, c_xy = 0;
  uint32_t always_types = 0;
  int prec = 0, crit = 0, flags = 0, tile = 0;   // tile: the plan's tile-width and fusion overrides (set the reduction order)
  bool operator==(const ReuseKey &o) const {
    return serial == o.serial && cid == o.cid && seed == o.seed && target == o.target && c_x == o.c_x &&
           c_xy == o.c_xy && always_types == o.always_types && prec == o.prec && crit == o.crit &&
           flags == o.flags && tile == o.tile;
  }
};

struct Ctx {
  int device = 0;
  void *scratch = nullptr;     // device address of this device's scratch array
  hipStream_t stream = nullptr;
  bool own_stream = false;
  double px = 0, py = 0, pz = 0;
  int prec = NT_C128;
  uint64_t max_batch = 0;
  int shortcuts = 0;
  // NT_SHORTCUT_REUSE store: trajectory -> (fired-site count, value) pairs
  ReuseKey reuse_key;
  bool reuse_valid = false;
  std::unordered_map<uint64_t, std::vector<std::pair<int32_t, double>>> reuse;
  size_t reuse_values = 0;
  int crit = 0;                // NT_CRIT_*
  uint64_t target = 0;         // basis state of NT_CRIT_TARGET_PROB
  std::map<std::pair<uint64_t, int>, std::unique_ptr<DevPlan>> plans;
  uint64_t use_clock = 0;
  size_t plan_budget = (size_t)24 << 30;   // device bytes held by cached plans
  size_t max_plans = 4096;
  void evict_plans();
  // batched runs: per-launch descriptor tables and per-circuit results
  DevBuf multi_items, sample_items, item_map, multi_nref, bvals, bcounts;
  DevBuf states, events, ev_count, partials, fid, count, frames, tmp, tlist, start, end, firstlast, hist;
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  std::vector<double> ev_bytes, ev_updates, ev_flops;
  std::vector<hipEvent_t> ev_pool;
  int64_t t_launches = 0;
  double t_ms = 0, t_bytes = 0, t_updates = 0, t_flops = 0;

  Ctx(int dev, void *stream);
  ~Ctx();

  DevPlan &plan_for(const Circuit &c, int prec);
  void upload_plan(const Circuit &c, DevPlan &dp);
  void ensure_reference(const Circuit &c, DevPlan &dp);
  uint64_t batch_size(const Circuit &c, const DevPlan &dp, uint64_t n_traj);

  // Simulate trajectories [t0, t0 + B) and leave results on the device:
  //   mode 0: score -> fid_dev[0..B), count_dev += successes
  //   mode 1: store final states (frames in `frames`)
  void simulate_batch(const Circuit &c, DevPlan &dp, uint64_t seed, uint64_t t0, int B, int mode,
                      double tau, double *fid_dev, uint64_t *count_dev, const Thresholds &th);

  // Per-trajectory criterion values to fid_out (host or device, may be
  // NULL), the number of values >= tau to count_out, their sum (in
  // trajectory order) to sum_out when given.
  void run(const Circuit &c, uint64_t seed, uint64_t t0, uint64_t n, double tau, double *fid_out,
           uint64_t *count_out, double *sum_out = nullptr);
  void run_shortcut(const Circuit &c, uint64_t seed, uint64_t t0, uint64_t n, double tau, double *fid_out,
                    uint64_t *count_out, double *sum_out);
  // run() without device allocation: every device buffer of the call lives
  // in this device's static scratch array (no short-cuts)
  void run_noalloc(const Circuit &c, uint64_t seed, uint64_t t0, uint64_t n, double tau, double *fid_out,
                   uint64_t *count_out, double *sum_out);
  // Success probability of n trajectories: the fraction with F >= tau for
  // the fidelity criterion, the mean measurement probability otherwise.
  double success(const Circuit &c, uint64_t seed, uint64_t t0, uint64_t n, double tau);
  // Many circuits, trajectories [t0, t0 + n) of each: values [n_circ][n]
  // (host or device, may be NULL), success counts and value sums per
  // circuit (host, may be NULL).  Single-pass circuits of one tile shape
  // share launches; the values equal those of run() on each circuit.
  void run_batch(const std::vector<const Circuit *> &cs, uint64_t seed, uint64_t t0, uint64_t n, double tau,
                 double *vals_out, uint64_t *counts_out, double *sums_out);
  // Criterion fields of a scoring run (computes the heavy-set median once).
  void criterion_args(const Circuit &c, DevPlan &dp, PassRun &r);
  double heavy_median(const Circuit &c, DevPlan &dp);
  void check_target(const Circuit &c) const;
  // Criterion value of the error-free state (1 for the fidelity).
  double reference_value(const Circuit &c, DevPlan &dp, double tau);
  bool ensure_checkpoints(const Circuit &c, DevPlan &dp);
  // Score batch entries with explicit event lists (ev_stride words each, counts
  // given) and first passes `start` (sorted); fids to host.
  void score_entries(const Circuit &c, DevPlan &dp, int B, const std::vector<uint32_t> &ev, int ev_stride,
                     const std::vector<int32_t> &cnt, const std::vector<int32_t> &start, double tau,
                     double *fid_host);
  void exhaustive(const Circuit &c, double tau, double *fid_out, double P_e[3], double *P_R);
  void sample_sites(const Circuit &c, uint64_t seed, uint64_t t0, uint64_t n, uint64_t *offsets,
                    int32_t *sites, uint8_t *paulis, int64_t cap, int64_t *n_out);
  void final_state(const Circuit &c, uint64_t seed, uint64_t traj, void *out, int64_t len);
  void reference_state(const Circuit &c, void *out, int64_t len);

  void timing_flush();
  void sync();
};

void check_hip(hipError_t e, const char *what);
bool is_device_pointer(const void *p);

}  // namespace nt
