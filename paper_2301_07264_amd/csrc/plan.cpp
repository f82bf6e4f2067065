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
#include <tuple>

#include "nt_internal.hpp"

namespace nt {

// 4x4 matrix (local index b_qa + 2 b_qb) of gate g acting within {qa, qb}.
void embed_gate(const HostGate &g, int qa, int qb, cd *e) {
  for (int i = 0; i < 16; ++i) e[i] = 0.0;
  if (g.nq == 1) {
    const bool on_a = g.q[0] == qa;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        const int ia = i & 1, ib = i >> 1, ja = j & 1, jb = j >> 1;
        if (on_a) e[4 * i + j] = ib == jb ? g.m[2 * ia + ja] : cd(0.0);
        else e[4 * i + j] = ia == ja ? g.m[2 * ib + jb] : cd(0.0);
      }
    return;
  }
  // the gate's matrix acts on local index b_q0 + 2 b_q1
  const bool same = g.q[0] == qa;
  auto sw = [](int i) { return ((i & 1) << 1) | (i >> 1); };
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) e[4 * i + j] = same ? g.m[4 * i + j] : g.m[4 * sw(i) + sw(j)];
}

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
    // register segments: the fused blocks' qubit pairs must be disjoint (the
    // gate kernel applies a block on register bits 0,1 or 2,3)
    std::vector<int> pair;
    if (mode == 1) pair.assign(n, -1);
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
        if (mode == 1 && op.cls == OPC_G4) {
          const bool fresh = pair[op.qa] < 0 && pair[op.qb] < 0;
          if (!fresh && pair[op.qa] != op.qb) break;
          pair[op.qa] = op.qb;
          pair[op.qb] = op.qa;
        }
        head[q]++;
        if (other >= 0) {
          head[other]++;
          if (!instack[other]) { stack.push_back(other); instack[other] = 1; }
        }
        cnt += op.sub.empty() ? 1 : (int)op.sub.size();   // gates applied
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

// Rough cost of an op in SIMD cycles per wave (a wave applies an op to
// 64 x 16 amplitudes): the larger of its vector work (about 2.3 cycles per
// FP32 instruction) and a floor of about 230 cycles, the scalar work every op
// costs (descriptor load, frame conjugation, dispatch), as measured per op
// kind on the pass kernel.
double op_cost(const HostOp &h) {
  constexpr double FLOOR = 230.0, CYC = 2.3;
  auto re = [](cd v) { return v.imag() == 0.0; };
  double v = 0.0;
  switch (h.cls) {
    case OPC_G1: {
      const bool real = re(h.m[0]) && re(h.m[1]) && re(h.m[2]) && re(h.m[3]);
      const bool rx = h.m[0] == h.m[3] && re(h.m[0]) && h.m[1] == h.m[2] && h.m[1].real() == 0.0;
      v = (real || rx ? 64.0 : 128.0) * CYC;
      break;
    }
    case OPC_D1: case OPC_D2: v = 64.0 * CYC; break;
    case OPC_C1: case OPC_SW: v = 32.0 * CYC; break;
    case OPC_G2: v = 256.0 * CYC + 2.0 * FLOOR; break;   // and an LDS round trip of its own
    case OPC_G4: v = 288.0 * CYC; break;                 // 256 FMA, 32 moves of matrix entries
    default: break;
  }
  return std::max(v, FLOOR);
}

// Fusion into two-qubit blocks among the ops of one pass (the passes stay
// those of the unfused schedule; segments are then planned over the units).
// A two-qubit gate on {a, b} takes the runs of one-qubit gates right before
// it on a and on b that no earlier block took and, when it took any, also
// the runs right after it; the block is applied as one dense 4x4.  On every
// qubit the gates of a block are consecutive, so the block applied at its
// two-qubit gate's place is the circuit's product of unitaries.  Taking the
// runs after the gate only together with runs before it makes alternate
// layers of one-qubit gates and entangling gates form blocks of four
// one-qubit gates (half the arithmetic of applying them one by one) instead
// of blocks of two (the same arithmetic).  A block is formed only when the
// cost model above prices it below its parts.
std::vector<HostOp> fuse_blocks(const Circuit &c, const std::vector<HostOp> &ops, const std::vector<int> &order,
                                int n, uint64_t local, int *n_fused) {
  const int K = (int)order.size();
  std::vector<std::vector<int>> line(n);
  std::vector<int> pa(K, -1), pb(K, -1);
  for (int k = 0; k < K; ++k) {
    const HostOp &op = ops[order[k]];
    pa[k] = (int)line[op.qa].size();
    line[op.qa].push_back(k);
    if (op.qb >= 0) {
      pb[k] = (int)line[op.qb].size();
      line[op.qb].push_back(k);
    }
  }
  std::vector<int> claim(K, -1);
  std::vector<std::vector<int>> members(K);
  auto one_qubit = [&](int k) { return ops[order[k]].qb < 0; };
  HostOp g4proto;
  g4proto.cls = OPC_G4;
  const double c4 = op_cost(g4proto);
  for (int k = 0; k < K; ++k) {
    const HostOp &op = ops[order[k]];
    // both qubits must be in the pass's tile (a CNOT's control need not be)
    if (op.qb < 0 || !((local >> op.qa) & 1) || !((local >> op.qb) & 1)) continue;
    std::vector<int> pre, post;
    for (int side = 0; side < 2; ++side) {
      const int q = side ? op.qb : op.qa, p0 = side ? pb[k] : pa[k];
      for (int i = p0 - 1; i >= 0; --i) {
        const int j = line[q][i];
        if (!one_qubit(j) || claim[j] >= 0) break;
        pre.push_back(j);
      }
      for (int i = p0 + 1; i < (int)line[q].size(); ++i) {
        const int j = line[q][i];
        if (!one_qubit(j)) break;
        post.push_back(j);
      }
    }
    // a dense two-qubit gate forms a block even alone: as a block it runs
    // on two register qubits instead of an LDS pass of its own
    if ((pre.empty() && op.cls != OPC_G2) || (int)pre.size() + 1 > MAX_BLOCK_GATES) continue;
    std::vector<int> mem = pre;
    mem.push_back(k);
    // the runs after the gate only when the block still has room for them
    if ((int)(mem.size() + post.size()) <= MAX_BLOCK_GATES) mem.insert(mem.end(), post.begin(), post.end());
    std::sort(mem.begin(), mem.end());
    double parts = 0.0;
    for (int j : mem) parts += op_cost(ops[order[j]]);
    if (parts <= 1.1 * c4) continue;
    for (int j : mem) claim[j] = k;
    members[k] = mem;
  }
  std::vector<HostOp> units;
  for (int k = 0; k < K; ++k) {
    if (claim[k] >= 0 && claim[k] != k) continue;   // applied by its block
    const HostOp &op = ops[order[k]];
    if (claim[k] != k) {
      units.push_back(op);
      continue;
    }
    HostOp b;
    b.cls = OPC_G4;
    b.qa = op.qa;
    b.qb = op.qb;
    b.gate = op.gate;
    cd M[16], E[16], T[16];
    for (int i = 0; i < 16; ++i) M[i] = (i % 5 == 0) ? cd(1.0) : cd(0.0);
    for (int j : members[k]) {
      const int g = ops[order[j]].gate;
      b.sub.push_back(g);
      embed_gate(c.gates[(size_t)g], b.qa, b.qb, E);
      for (int r = 0; r < 4; ++r)
        for (int s2 = 0; s2 < 4; ++s2) {
          cd acc = 0.0;
          for (int t = 0; t < 4; ++t) acc += E[4 * r + t] * M[4 * t + s2];
          T[4 * r + s2] = acc;
        }
      for (int i = 0; i < 16; ++i) M[i] = T[i];
    }
    for (int i = 0; i < 16; ++i) b.m[i] = M[i];
    units.push_back(b);
    ++*n_fused;
  }
  return units;
}

// Qubits an op acts on.
uint64_t op_qubits(const Circuit &c, const HostOp &h) {
  uint64_t m = 0;
  if (h.cls == OPC_NOP) return 0;
  for (int g : h.gates()) {
    const HostGate &hg = c.gates[(size_t)g];
    m |= 1ull << hg.q[0];
    if (hg.nq == 2) m |= 1ull << hg.q[1];
  }
  return m;
}

// Whether two ops of one segment may trade places: only ops on disjoint
// qubits (two diagonal gates on a shared qubit commute, but an error after
// the first of them does not commute with the second).
bool commute(const Circuit &c, const HostOp &x, const HostOp &y) { return (op_qubits(c, x) & op_qubits(c, y)) == 0; }

// Fused diagonal runs.  A diagonal op of a segment may move back to the
// previous diagonal op past ops on other qubits.  Runs of at
// least three diagonal gates with at most one qubit in the registers then
// become one op (OPC_DF, up to MAX_BLOCK_GATES gates) that multiplies each
// amplitude once by the product of the gates' phases, instead of once per
// gate.  Errors inside a run (a later gate of the run acts on the qubit)
// still act right after their gate: the kernel evaluates each gate's phase
// under the frame as the errors before it left it.
std::vector<int> fuse_diagonals(const Circuit &c, std::vector<HostOp> &pu, const std::vector<int> &sched,
                                const std::vector<int> &reg_q, int *n_diag) {
  auto in_reg = [&](int q) { return q >= 0 && std::find(reg_q.begin(), reg_q.end(), q) != reg_q.end(); };
  auto eligible = [&](const HostOp &h) {
    if (h.cls == OPC_D1) return true;
    if (h.cls == OPC_D2) return !(in_reg(h.qa) && in_reg(h.qb));
    return false;
  };
  // move each eligible diagonal right after the previous one when it commutes
  // with everything in between
  std::vector<int> seq(sched);
  for (size_t i = 1; i < seq.size(); ++i) {
    if (!eligible(pu[seq[i]])) continue;
    size_t j = i;
    while (j > 0 && !eligible(pu[seq[j - 1]]) && commute(c, pu[seq[i]], pu[seq[j - 1]])) --j;
    if (j > 0 && j < i && eligible(pu[seq[j - 1]])) {
      const int v = seq[i];
      seq.erase(seq.begin() + (long)i);
      seq.insert(seq.begin() + (long)j, v);
    }
  }
  std::vector<int> out;
  for (size_t i = 0; i < seq.size();) {
    size_t j = i;
    while (j < seq.size() && eligible(pu[seq[j]]) && (int)(j - i) < MAX_BLOCK_GATES) ++j;
    if (j - i >= 3) {
      HostOp d;
      d.cls = OPC_DF;
      d.qa = pu[seq[i]].qa;
      d.qb = -1;
      d.gate = pu[seq[i]].gate;
      for (size_t k = i; k < j; ++k) d.sub.push_back(pu[seq[k]].gate);
      pu.push_back(d);
      out.push_back((int)pu.size() - 1);
      ++*n_diag;
      i = j;
    } else {
      out.push_back(seq[i]);
      ++i;
    }
  }
  return out;
}

// Shape of a one-qubit gate's body in the gate kernel: general, real, or
// [[c, -i s], [-i s, c]].
int g1_shape(const HostOp &h) {
  auto real = [](cd v) { return v.imag() == 0.0; };
  auto imag = [](cd v) { return v.real() == 0.0; };
  if (real(h.m[0]) && real(h.m[1]) && real(h.m[2]) && real(h.m[3])) return 1;
  if (h.m[0] == h.m[3] && real(h.m[0]) && h.m[1] == h.m[2] && imag(h.m[1])) return 2;
  return 0;
}

// One-qubit layers.  In a segment with four register qubits, one-qubit ops
// of RX type ([[c, -i s], [-i s, c]]) on all four register qubits become
// one op when the later ones can move back to the first past everything in
// between (ops on other qubits).  The four gates act on different qubits, so their order is free
// and an error after any of them commutes with the others: the errors all
// act after the op.
std::vector<int> fuse_layers(const Circuit &c, std::vector<HostOp> &pu, const std::vector<int> &sched,
                             const std::vector<int> &reg_q, int *n_layer) {
  if (reg_q.size() != 4) return sched;
  auto rbit = [&](int q) {
    for (int b = 0; b < 4; ++b)
      if (reg_q[(size_t)b] == q) return b;
    return -1;
  };
  const size_t L = sched.size();
  std::vector<char> used(L, 0);
  std::vector<int> out;
  for (size_t i = 0; i < L; ++i) {
    if (used[i]) continue;
    const HostOp &h = pu[(size_t)sched[i]];
    if (h.cls != OPC_G1 || rbit(h.qa) < 0) {
      out.push_back(sched[i]);
      continue;
    }
    const int shape = g1_shape(h);
    if (shape != 2) {
      out.push_back(sched[i]);
      continue;
    }
    std::vector<size_t> grp = {i};
    int have = 1 << rbit(h.qa);
    for (size_t j = i + 1; j < L && grp.size() < 4; ++j) {
      if (used[j]) continue;
      const HostOp &g = pu[(size_t)sched[j]];
      const int b = g.cls == OPC_G1 ? rbit(g.qa) : -1;
      if (b < 0 || (have >> b) & 1 || g1_shape(g) != shape) continue;
      bool ok = true;
      for (size_t k = i + 1; k < j && ok; ++k)
        if (!used[k] && std::find(grp.begin(), grp.end(), k) == grp.end()) ok = commute(c, g, pu[(size_t)sched[k]]);
      if (!ok) continue;
      grp.push_back(j);
      have |= 1 << b;
    }
    if (grp.size() < 4) {
      out.push_back(sched[i]);
      continue;
    }
    HostOp l;
    l.cls = OPC_L4;
    l.qa = reg_q[0];
    l.qb = -1;
    l.gate = h.gate;
    l.sub.assign(4, -1);
    for (size_t k : grp) {
      const HostOp &g = pu[(size_t)sched[k]];
      const int b = rbit(g.qa);
      l.sub[(size_t)b] = g.gate;
      for (int e = 0; e < 4; ++e) l.m[4 * b + e] = g.m[e];
      used[k] = 1;
    }
    pu.push_back(l);
    out.push_back((int)pu.size() - 1);
    ++*n_layer;
  }
  return out;
}

}  // namespace

int fusion_mode(int width) {
  switch (width) {
    case 1: return 0;
    case 3: return FUSE_BLOCKS;
    case 4: return FUSE_DIAG;
    default: return FUSE_BLOCKS | FUSE_DIAG;   // 0 (automatic) and 2
  }
}

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
  int fuse = fusion_mode(c.fuse_width[prec == NT_C64 ? 1 : 2]);
  // one-qubit layers go with the blocks, at complex64 (their descriptor
  // points at single-precision matrices)
  if (prec == NT_C64 && (fuse & FUSE_BLOCKS)) fuse |= FUSE_LAYERS;
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

Plan make_plan(const Circuit &c, int L, int R, int cfix, int fuse) {
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
    if (fuse & FUSE_BLOCKS) {
      pu = fuse_blocks(c, ops, sorted_ops, n, ps.local_mask, &P.n_fused);
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
      // register qubits: the blocks' pairs on bits (0, 1) and (2, 3), the
      // first block on a pair putting its qa on the lower bit, then the
      // segment's other qubits, then padding with other local qubits
      for (int i : sched)
        if (pu[i].cls == OPC_G4 && std::find(sg.reg_q.begin(), sg.reg_q.end(), pu[i].qa) == sg.reg_q.end()) {
          sg.reg_q.push_back(pu[i].qa);
          sg.reg_q.push_back(pu[i].qb);
        }
      for (int q = 0; q < n; ++q)
        if (((rset >> q) & 1) && std::find(sg.reg_q.begin(), sg.reg_q.end(), q) == sg.reg_q.end())
          sg.reg_q.push_back(q);
      for (int q = 0; q < n && (int)sg.reg_q.size() < R; ++q)
        if (((ps.local_mask >> q) & 1) && std::find(sg.reg_q.begin(), sg.reg_q.end(), q) == sg.reg_q.end())
          sg.reg_q.push_back(q);
      if ((int)sg.reg_q.size() != R) throw Error(NT_ERR_UNSUPPORTED, "internal: register set size");
      if (fuse & FUSE_DIAG) sched = fuse_diagonals(c, pu, sched, sg.reg_q, &P.n_diag);
      if (fuse & FUSE_LAYERS) sched = fuse_layers(c, pu, sched, sg.reg_q, &P.n_layer);
      // Offsets in the segment: the gate kernel applies ops in pairs and
      // holds the block body for register bits (0, 1) and the diagonal-run
      // body in the first slot of a pair, the block body for bits (2, 3) in
      // the second.  A later op that commutes with everything it passes
      // moves in front of a fused op that would land on the wrong parity,
      // else a no-op fills the place.
      auto align = [&](const std::vector<int> &rq) {
        auto parity = [&](int i) -> int {
          if (pu[i].cls == OPC_DF) return 0;
          if (pu[i].cls == OPC_L4) return 0;
          if (pu[i].cls != OPC_G4) return -1;
          return (int)(std::find(rq.begin(), rq.end(), pu[i].qa) - rq.begin()) / 2;
        };
        std::vector<int> pend(sched.begin(), sched.end()), out;
        while (!pend.empty()) {
          const int i = pend.front();
          const int want = parity(i);
          if (want >= 0 && (int)(out.size() & 1) != want) {
            int found = -1;
            for (size_t x = 1; x < pend.size() && found < 0; ++x) {
              const HostOp &cand = pu[pend[x]];
              if (parity(pend[x]) >= 0) continue;
              bool ok = true;
              for (size_t y = 0; y < x && ok; ++y) ok = commute(c, cand, pu[pend[y]]);
              if (ok) found = (int)x;
            }
            if (found >= 0) {
              out.push_back(pend[(size_t)found]);
              pend.erase(pend.begin() + found);
            } else {
              out.push_back(-1);
            }
            continue;
          }
          out.push_back(i);
          pend.erase(pend.begin());
        }
        return out;
      };
      std::vector<int> seq = align(sg.reg_q);
      if (R == 4) {
        // the two register pairs the other way round, if that needs fewer
        // no-ops
        std::vector<int> rq2 = {sg.reg_q[2], sg.reg_q[3], sg.reg_q[0], sg.reg_q[1]};
        std::vector<int> seq2 = align(rq2);
        auto nops = [](const std::vector<int> &v) { return std::count(v.begin(), v.end(), -1); };
        if (nops(seq2) < nops(seq)) {
          seq = seq2;
          sg.reg_q = rq2;
        }
      }
      sg.op_begin = (int)P.ops.size();
      for (int i : seq) {
        if (i >= 0) {
          emit(i);
        } else {
          HostOp nop;
          nop.cls = OPC_NOP;
          nop.gate = -1;
          nop.qa = sg.reg_q[0];
          P.ops.push_back(nop);
        }
      }
      sg.op_end = (int)P.ops.size();
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
  if (P.ops.size() >= ((size_t)1 << (32 - SITE_OP_SHIFT)))
    throw Error(NT_ERR_UNSUPPORTED, "plan has more ops than the event words can index");
  P.op_of_gate.assign(c.gates.size(), -1);
  for (size_t o = 0; o < P.ops.size(); ++o) {
    const HostOp &op = P.ops[o];
    const std::vector<int32_t> gs = op.gates();
    // (stage or SITE_STAGE_END, qubit, site): a site is interior when a
    // later gate of the op acts on its qubit
    std::vector<std::tuple<uint32_t, int, int64_t>> in, end;
    for (size_t k = 0; k < gs.size(); ++k) {
      const int g = gs[k];
      P.op_of_gate[g] = (int)o;
      const HostGate &hg = c.gates[g];
      for (int j = 0; j < hg.nq; ++j) {
        bool later = false;
        for (size_t k2 = k + 1; k2 < gs.size() && !later; ++k2) {
          const HostGate &h2 = c.gates[gs[k2]];
          later = h2.q[0] == hg.q[j] || (h2.nq == 2 && h2.q[1] == hg.q[j]);
        }
        (later ? in : end).emplace_back(later ? (uint32_t)k : SITE_STAGE_END, hg.q[j], site_base[g] + j);
      }
    }
    for (auto *v : {&in, &end})
      for (const auto &t : *v) {
        P.app_site.push_back((int32_t)std::get<2>(t));
        P.app_tag.push_back(((uint32_t)o << SITE_OP_SHIFT) | (std::get<0>(t) << SITE_STAGE_SHIFT) | ((uint32_t)std::get<1>(t) << 2));
      }
  }
  return P;
}

}  // namespace nt
