// Gate-pass planner.
//
// The Monte Carlo branch simulates every trajectory gate by gate (Sec. IV-B,
// IV-B.2); its cost is one sweep over the 2^n amplitudes per gate.  On the GPU
// a sweep over HBM is the expensive unit, so gates are grouped:
//
//   pass     one read + one write of the state in HBM.  A work-group holds a
//            tile of 2^L amplitudes whose indices differ only in L "local"
//            qubits (always including the lowest `cfix`, so that each tile is
//            made of contiguous 128-byte runs).  A pass applies every gate it
//            can reach whose non-diagonal qubits are local.  Diagonal gates
//            (Z, S, T, RZ, CZ, CP, RZZ) and the control of a CNOT only read
//            index bits, so they never need their qubits local.
//   segment  inside a pass, each thread holds 2^R amplitudes in registers,
//            whose indices differ in R "register" qubits; gates whose dense
//            qubits are register qubits are applied without LDS traffic.
//            Between segments the tile is exchanged through LDS.
//
// Gates keep their order on every qubit, so any schedule produced here is
// the circuit's product of unitaries; errors stay attached to their gate.
// The plan is the same for every trajectory.
#include <algorithm>
#include <numeric>

#include "nt_internal.hpp"

namespace nt {

namespace {

struct Sched {
  const std::vector<HostOp> *ops;
  int n;
  std::vector<std::vector<int>> queue;   // per qubit: op indices in order
  std::vector<int> head;
  std::vector<char> done;

  Sched(const std::vector<HostOp> &o, int nq, const std::vector<int> &subset) : ops(&o), n(nq) {
    queue.assign(n, {});
    head.assign(n, 0);
    done.assign(o.size(), 0);
    for (int i : subset) {
      const HostOp &op = o[i];
      queue[op.qa].push_back(i);
      if (op.qb >= 0) queue[op.qb].push_back(i);
    }
  }

  bool finished() const {
    for (int q = 0; q < n; ++q)
      if (head[q] < (int)queue[q].size()) return false;
    return true;
  }

  // Schedule every ready op whose needed qubits are in `allowed`.  With
  // out != nullptr the schedule is committed and the ops appended in order;
  // otherwise heads are restored and only the count is returned.
  // mode 0: any op; mode 1: no dense two-qubit ops (register segments).
  int drain(uint64_t allowed, std::vector<int> *out, int mode = 0) {
    std::vector<int> saved;
    if (!out) saved = head;
    int cnt = 0;
    std::vector<int> stack(n);
    std::iota(stack.begin(), stack.end(), 0);
    std::vector<char> instack(n, 1);
    while (!stack.empty()) {
      int q = stack.back();
      stack.pop_back();
      instack[q] = 0;
      while (head[q] < (int)queue[q].size()) {
        int i = queue[q][head[q]];
        const HostOp &op = (*ops)[i];
        int other = (op.qa == q) ? op.qb : op.qa;
        if (other >= 0 && (head[other] >= (int)queue[other].size() || queue[other][head[other]] != i)) break;
        if ((uint64_t)op.need_mask() & ~allowed) break;
        if (mode == 1 && op.cls == OPC_G2) break;
        head[q]++;
        if (other >= 0) {
          head[other]++;
          if (!instack[other]) { stack.push_back(other); instack[other] = 1; }
        }
        ++cnt;
        if (out) out->push_back(i);
      }
    }
    if (!out) head = saved;
    return cnt;
  }

  // A ready dense two-qubit op, or -1.
  int ready_g2() const {
    for (int q = 0; q < n; ++q) {
      if (head[q] >= (int)queue[q].size()) continue;
      int i = queue[q][head[q]];
      const HostOp &op = (*ops)[i];
      if (op.cls != OPC_G2) continue;
      int other = (op.qa == q) ? op.qb : op.qa;
      if (head[other] < (int)queue[other].size() && queue[other][head[other]] == i) return i;
    }
    return -1;
  }

  void commit(int i) {
    const HostOp &op = (*ops)[i];
    head[op.qa]++;
    if (op.qb >= 0) head[op.qb]++;
  }

  // Op index at the head of qubit q's queue (or a large value).
  int head_op(int q) const { return head[q] < (int)queue[q].size() ? queue[q][head[q]] : (1 << 30); }
};

// Greedy choice of a qubit set of size k within `pool`, starting from
// `base`: add one qubit at a time, taking the one that lets the most ops be
// scheduled; ties go to the qubit whose next op comes first.
uint64_t choose_set(Sched &s, uint64_t base, uint64_t pool, int k, int mode = 0) {
  uint64_t set = base;
  int have = __builtin_popcountll(base);
  while (have < k) {
    int best = -1, best_cnt = -1, best_head = 1 << 30;
    for (int q = 0; q < s.n; ++q) {
      if (!((pool >> q) & 1) || ((set >> q) & 1)) continue;
      int c = s.drain(set | (1ull << q), nullptr, mode);
      int h = s.head_op(q);
      if (c > best_cnt || (c == best_cnt && h < best_head)) {
        best = q; best_cnt = c; best_head = h;
      }
    }
    if (best < 0) break;
    set |= 1ull << best;
    ++have;
  }
  return set;
}

// Local improvement of a pass's local set: exchange one chosen qubit (not
// in `fixed`) for one outside the set while that lets more ops be scheduled.
uint64_t improve_set(Sched &s, uint64_t set, uint64_t fixed, uint64_t pool, int mode = 0) {
  int cur = s.drain(set, nullptr, mode);
  for (int round = 0; round < 64; ++round) {
    int best = cur;
    uint64_t best_set = set;
    for (int qi = 0; qi < s.n; ++qi) {
      if (!((set >> qi) & 1) || ((fixed >> qi) & 1)) continue;
      for (int qo = 0; qo < s.n; ++qo) {
        if (!((pool >> qo) & 1) || ((set >> qo) & 1)) continue;
        const uint64_t t = (set & ~(1ull << qi)) | (1ull << qo);
        const int c = s.drain(t, nullptr, mode);
        if (c > best) {
          best = c;
          best_set = t;
        }
      }
    }
    if (best_set == set) break;
    set = best_set;
    cur = best;
  }
  return set;
}

// Fusion into two-qubit blocks, among the ops of one pass (so the passes stay
// those of the unfused schedule; the segments are then planned over the
// blocks).  A CNOT whose target and control were each last touched, in the
// pass's order, by a one-qubit gate of the same pass takes both gates into
// one block: U_t on the target and U_c on the control, then the CNOT.
// Moving U_t and U_c to the CNOT keeps the gate order on every qubit (each is
// the gate right before the CNOT on its qubit, and they act on different
// qubits), so the block is the circuit's product of unitaries.
std::vector<HostOp> fuse_pass(const std::vector<HostOp> &ops, const std::vector<int> &order, int n, int *n_fused) {
  const int K = (int)order.size();
  std::vector<int> last(n, -1), into(K, -1), jt(K, -1), jc(K, -1);
  auto one_qubit = [&](int k) {
    const HostOp &h = ops[order[k]];
    return k >= 0 && (h.cls == OPC_G1 || h.cls == OPC_D1) && into[k] < 0;
  };
  for (int k = 0; k < K; ++k) {
    const HostOp &op = ops[order[k]];
    if (op.cls == OPC_C1 && last[op.qa] >= 0 && last[op.qb] >= 0 && one_qubit(last[op.qa]) &&
        one_qubit(last[op.qb])) {
      jt[k] = last[op.qa];
      jc[k] = last[op.qb];
      into[jt[k]] = into[jc[k]] = k;
    }
    last[op.qa] = k;
    if (op.qb >= 0) last[op.qb] = k;
  }
  auto as_2x2 = [](const HostOp &h, cd *m) {
    if (h.cls == OPC_D1) {
      m[0] = h.m[0]; m[1] = 0; m[2] = 0; m[3] = h.m[1];
    } else {
      for (int t = 0; t < 4; ++t) m[t] = h.m[t];
    }
  };
  std::vector<HostOp> units;
  for (int k = 0; k < K; ++k) {
    if (into[k] >= 0) continue;          // moved into its CNOT's block
    const HostOp &op = ops[order[k]];
    if (jt[k] < 0) {
      units.push_back(op);
      continue;
    }
    HostOp b;
    b.cls = OPC_UCX;
    b.qa = op.qa;
    b.qb = op.qb;
    b.gate = op.gate;
    b.pre[0] = ops[order[jt[k]]].gate;
    b.pre[1] = ops[order[jc[k]]].gate;
    for (int t = 0; t < 16; ++t) b.m[t] = 0;
    as_2x2(ops[order[jt[k]]], b.m);
    as_2x2(ops[order[jc[k]]], b.m + 4);
    units.push_back(b);
    ++*n_fused;
  }
  return units;
}

}  // namespace

void plan_for_precision(const Circuit &c, int prec, int *L, int *R, int *cfix) {
  int n = c.n;
  int lmax = prec == NT_C64 ? 13 : 12;      // 64 KiB of LDS per tile
  int cf = prec == NT_C64 ? 4 : 3;          // 128-byte contiguous runs
  *L = std::min(n, lmax);
  *cfix = std::min(n, cf);
  int r = std::max(2, std::min(4, *L - 6)); // >= 64 threads where possible
  *R = std::min(r, *L);
}

// Tile shape.  A complex64 pass over 2^12-amplitude tiles (32 KiB of LDS,
// four work-groups per CU) costs about 0.74 of one over 2^13-amplitude tiles
// (64 KiB, two per CU): with more independent work-groups per CU the load
// and store phases of one overlap the arithmetic of the others.  The smaller
// tile has fewer local qubits, so it can need more passes; it is taken when
// its predicted pass cost is at least 5% lower.  Deterministic (a function of
// the circuit), so results stay a function of the inputs.
void tile_range(const Circuit &c, int prec, int *lo, int *hi) {
  int L, R, cfix;
  plan_for_precision(c, prec, &L, &R, &cfix);
  *hi = L;
  *lo = std::min(L, 10);   // 2^(L - 4) >= 64 threads per work-group
}

Plan choose_plan(const Circuit &c, int prec) {
  int L, R, cfix;
  plan_for_precision(c, prec, &L, &R, &cfix);
  const int ov = c.tile_override[prec == NT_C64 ? 1 : 2];
  const bool fuse = c.fuse_width[prec == NT_C64 ? 1 : 2] != 1;
  if (ov > 0) {
    const int Lo = std::min(ov, L);
    const int Ro = std::max(2, std::min(4, Lo - 6));
    return make_plan(c, Lo, std::min(Ro, Lo), cfix, fuse);
  }
  Plan p = make_plan(c, L, R, cfix, fuse);
  if (prec == NT_C64 && L == 13 && p.passes.size() > 1) {
    const int L2 = 12, R2 = std::max(2, std::min(4, L2 - 6));
    Plan q = make_plan(c, L2, R2, cfix, fuse);
    if ((double)q.passes.size() * 0.74 < (double)p.passes.size() * 0.95) return q;
  }
  return p;
}

Plan make_plan(const Circuit &c, int L, int R, int cfix, bool fuse) {
  Plan P;
  P.n = c.n;
  P.L = L;
  P.R = R;
  P.cfix = cfix;
  const int n = c.n;
  const std::vector<HostOp> ops = classify(c);
  const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1);
  for (const HostOp &op : ops)
    if (op.cls != OPC_G2 && __builtin_popcount(op.need_mask()) > R)
      throw Error(NT_ERR_UNSUPPORTED, "internal: op needs more register qubits than the plan has");

  std::vector<int> all_ops(ops.size());
  std::iota(all_ops.begin(), all_ops.end(), 0);
  Sched top(ops, n, all_ops);
  const uint64_t fixed = (1ull << cfix) - 1;

  std::vector<std::vector<int>> pass_ops;
  std::vector<uint64_t> pass_mask;
  if (ops.empty()) {
    pass_ops.push_back({});
    pass_mask.push_back(all & ((1ull << L) - 1));
  }
  while (!top.finished()) {
    uint64_t lset = (L >= n) ? all : improve_set(top, choose_set(top, fixed, all, L), fixed, all);
    std::vector<int> sched;
    top.drain(lset, &sched);
    if (sched.empty()) throw Error(NT_ERR_UNSUPPORTED, "planner made no progress");
    pass_ops.push_back(sched);
    pass_mask.push_back(lset);
  }

  // Segments inside each pass.
  for (size_t p = 0; p < pass_ops.size(); ++p) {
    Pass ps;
    ps.local_mask = pass_mask[p];
    ps.seg_begin = (int)P.segs.size();
    ps.op_begin = (int)P.ops.size();
    // the pass's ops, with two-qubit blocks formed among them
    // (in circuit order, a valid order of any subset, which also keeps the
    // segment planner's ties as they are without fusion)
    std::vector<int> sorted_ops = pass_ops[p];
    std::sort(sorted_ops.begin(), sorted_ops.end());
    std::vector<HostOp> pu;
    if (fuse) {
      pu = fuse_pass(ops, sorted_ops, n, &P.n_fused);
    } else {
      for (int i : sorted_ops) pu.push_back(ops[i]);
    }
    std::vector<int> pall(pu.size());
    std::iota(pall.begin(), pall.end(), 0);
    Sched in(pu, n, pall);
    auto emit = [&](int i) { P.ops.push_back(pu[i]); };
    if (pass_ops[p].empty()) {
      Segment sg;
      sg.op_begin = sg.op_end = (int)P.ops.size();
      for (int q = 0; q < n && (int)sg.reg_q.size() < R; ++q)
        if ((ps.local_mask >> q) & 1) sg.reg_q.push_back(q);
      P.segs.push_back(sg);
    }
    while (!in.finished()) {
      // dense two-qubit ops go to quad segments as soon as they are ready
      int g2 = in.ready_g2();
      if (g2 >= 0) {
        Segment sg;
        sg.kind = SEG_QUAD;
        sg.op_begin = (int)P.ops.size();
        emit(g2);
        sg.op_end = (int)P.ops.size();
        for (int q = 0; q < n && (int)sg.reg_q.size() < R; ++q)
          if ((ps.local_mask >> q) & 1) sg.reg_q.push_back(q);
        in.commit(g2);
        P.segs.push_back(sg);
        continue;
      }
      uint64_t rset = improve_set(in, choose_set(in, 0, ps.local_mask, R, 1), 0, ps.local_mask, 1);
      std::vector<int> sched;
      in.drain(rset, &sched, 1);
      if (sched.empty()) throw Error(NT_ERR_UNSUPPORTED, "segment planner made no progress");
      Segment sg;
      sg.op_begin = (int)P.ops.size();
      for (int i : sched) emit(i);
      sg.op_end = (int)P.ops.size();
      for (int q = 0; q < n; ++q)
        if ((rset >> q) & 1) sg.reg_q.push_back(q);
      // pad to exactly R register qubits with other local qubits
      for (int q = 0; q < n && (int)sg.reg_q.size() < R; ++q)
        if (((ps.local_mask >> q) & 1) && !((rset >> q) & 1)) sg.reg_q.push_back(q);
      std::sort(sg.reg_q.begin(), sg.reg_q.end());
      P.segs.push_back(sg);
    }
    ps.seg_end = (int)P.segs.size();
    ps.op_end = (int)P.ops.size();
    P.passes.push_back(ps);
  }

  // Sites in application order.
  std::vector<int64_t> site_base(c.gates.size());
  int64_t s = 0;
  for (size_t g = 0; g < c.gates.size(); ++g) {
    site_base[g] = s;
    s += c.gates[g].nq;
  }
  P.op_of_gate.assign(c.gates.size(), -1);
  for (size_t o = 0; o < P.ops.size(); ++o) {
    const HostOp &op = P.ops[o];
    // a fused block's one-qubit gates first (interior sites), then its CNOT
    for (int k = 0; k < 2; ++k) {
      const int g = op.pre[k];
      if (g < 0) continue;
      P.op_of_gate[g] = (int)o;
      P.app_site.push_back((int32_t)site_base[g]);
      P.app_tag.push_back(((uint32_t)o << 8) | ((uint32_t)c.gates[g].q[0] << 2) | SITE_INTERIOR);
    }
    const int g = op.gate;
    P.op_of_gate[g] = (int)o;
    const HostGate &hg = c.gates[g];
    for (int j = 0; j < hg.nq; ++j) {
      P.app_site.push_back((int32_t)(site_base[g] + j));
      P.app_tag.push_back(((uint32_t)o << 8) | ((uint32_t)hg.q[j] << 2));
    }
  }
  return P;
}

}  // namespace nt
