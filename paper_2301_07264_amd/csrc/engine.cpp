// Host engine: plan upload, reference state, batched trajectory runs.
//
// Per batch of B trajectories (Sec. IV-B.2 Monte Carlo runs):
//   1. k_sample draws every error site of every trajectory (Philox) and
//      writes the fired ones in plan order;
//   2. one k_pass launch per pass of the plan (the first synthesizes |0...0>,
//      the last fuses the fidelity partials against the resident reference);
//   3. k_finalize turns partials into F per trajectory and the success count.
// The error-free reference state (Sec. IV-B.1: the reference state psi_R) is
// computed once per circuit and precision with the same kernels and kept in
// device memory.
#include "engine.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <tuple>

namespace nt {

static_assert(SITE_OP_SHIFT == ntk::EV_OP_SHIFT && SITE_STAGE_SHIFT == ntk::EV_STAGE_SHIFT &&
                  SITE_STAGE_END == ntk::EV_STAGE_END,
              "event word layout of the planner and the gate kernel");

void check_hip(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      throw Error(NT_ERR_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
    throw Error(NT_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}

bool is_device_pointer(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof attr);
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice;
}

DevBuf::~DevBuf() { release(); }

void *Arena::take(size_t n) {
  const size_t at = (off + 255) & ~(size_t)255;
  if (at > cap || n > cap - at)
    throw Error(NT_ERR_UNSUPPORTED, "this call needs more than the " + std::to_string(cap >> 20) +
                                        " MiB scratch array of the allocation-free entry point");
  off = at + n;
  return base + at;
}

void DevBuf::release() {
  if (arena) {              // arena space is never freed
    p = nullptr;
    bytes = 0;
    return;
  }
  // queued work may still read the buffer
  if (p) (void)hipDeviceSynchronize();
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

void DevBuf::ensure(size_t n) {
  if (n == 0) n = 16;
  if (n <= bytes) return;
  if (arena) {
    p = arena->take(n);
    bytes = n;
    return;
  }
  release();
  check_hip(hipMalloc(&p, n), "hipMalloc");
  bytes = n;
}

Ctx::Ctx(int dev, void *s) : device(dev) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) {
    (void)hipGetLastError();
    throw Error(NT_ERR_DEVICE, "no HIP device present");
  }
  if (dev < 0 || dev >= count) throw Error(NT_ERR_INVALID_ARG, "device index out of range");
  check_hip(hipSetDevice(dev), "hipSetDevice");
  // device address of this device's scratch array (allocation-free runs)
  check_hip(ntk::scratch_address(dev, &scratch), "hipGetSymbolAddress(scratch)");
  if (s) {
    stream = static_cast<hipStream_t>(s);
  } else {
    check_hip(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking), "hipStreamCreate");
    own_stream = true;
  }
}

Ctx::~Ctx() {
  (void)hipSetDevice(device);
  if (stream) (void)hipStreamSynchronize(stream);
  for (auto &pr : ev_pending) {
    ev_pool.push_back(pr.first);
    ev_pool.push_back(pr.second);
  }
  for (hipEvent_t ev : ev_pool) (void)hipEventDestroy(ev);
  plans.clear();
  states.release(); events.release(); ev_count.release(); partials.release();
  fid.release(); count.release(); frames.release(); tmp.release();
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

void Ctx::sync() { check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize"); }

static size_t amp_bytes(int prec) { return prec == NT_C64 ? 8 : 16; }

// LDS address swizzle of the gate kernels (complex64: SW = 4, complex128:
// SW = 3): the low SW bits of a tile index are XORed with every higher SW-bit
// chunk.  The kernels apply the same map to the thread part of a slot's index;
// the register part is precomputed here per segment.
static uint32_t lds_swizzle(uint32_t j, int SW) {
  const uint32_t M = (1u << SW) - 1u;
  uint32_t r = j;
  for (int c = SW; c < 32; c += SW) r ^= (j >> c) & M;
  return r;
}

// Order of a segment's thread-id bits: lanes 0..2^SW-1 take local positions
// with distinct residues mod SW (conflict-free under the LDS swizzle), the
// rest follow in ascending order.
static std::vector<int> thread_bit_order(const std::vector<int> &tpos, int SW) {
  std::vector<int> first, rest;
  std::vector<char> used_res(SW, 0), used(tpos.size(), 0);
  for (size_t i = 0; i < tpos.size() && (int)first.size() < SW; ++i) {
    int r = tpos[i] % SW;
    if (!used_res[r]) {
      used_res[r] = 1;
      used[i] = 1;
      first.push_back(tpos[i]);
    }
  }
  if ((int)first.size() < SW) return tpos;   // cannot do better
  for (size_t i = 0; i < tpos.size(); ++i)
    if (!used[i]) rest.push_back(tpos[i]);
  first.insert(first.end(), rest.begin(), rest.end());
  return first;
}

// Dispatch code of a register-segment op (kind * 4 + register bit of the
// target) or of a quad op; rbit: the target's register bit (or 0).
static int32_t op_code(const HostOp &h, int rbit) {
  auto real = [](cd v) { return v.imag() == 0.0; };
  auto imag = [](cd v) { return v.real() == 0.0; };
  switch (h.cls) {
    case OPC_G1:
      if (real(h.m[0]) && real(h.m[1]) && real(h.m[2]) && real(h.m[3])) return ntk::OPK_G1R * 4 + rbit;
      if (h.m[0] == h.m[3] && real(h.m[0]) && h.m[1] == h.m[2] && imag(h.m[1])) return ntk::OPK_G1X * 4 + rbit;
      return ntk::OPK_G1 * 4 + rbit;
    case OPC_C1:
      if (!(h.m[0] == cd(0) && h.m[1] == cd(1) && h.m[2] == cd(1) && h.m[3] == cd(0)))
        throw Error(NT_ERR_UNSUPPORTED, "internal: controlled op other than CNOT");
      return ntk::OPK_CX * 4 + rbit;
    case OPC_D1: return ntk::OPK_D1 * 4;
    case OPC_D2: return ntk::OPK_D2 * 4;
    case OPC_NOP: return ntk::OPK_NOP * 4;
    default: return ntk::OPK_G2 * 4;
  }
}

// Rounded entries of the 16 frame variants of a 4x4 (local index b_qa +
// 2 b_qb): conjugated by X^x Z^z on the two qubits, entry (i, j) is
// (-1)^popcount(z & (i ^ j)) M[i ^ x][j ^ x]; variant x + 4 z, 16 entries
// each (rounded once, then permuted and negated exactly).
template <typename T>
static void push_variants(const cd *M, bool swap_ab, std::vector<ntk::cx<T>> &out) {
  auto sw = [](int i) { return ((i & 1) << 1) | (i >> 1); };
  for (int z = 0; z < 4; ++z)
    for (int x = 0; x < 4; ++x)
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          const int si = swap_ab ? sw(i ^ x) : (i ^ x), sj = swap_ab ? sw(j ^ x) : (j ^ x);
          ntk::cx<T> e{(T)M[4 * si + sj].real(), (T)M[4 * si + sj].imag()};
          if (__builtin_popcount((unsigned)(z & (i ^ j))) & 1) e = ntk::cx<T>{-e.x, -e.y};
          out.push_back(e);
        }
}

// rsel / code per op are computed with the pass layouts (register bit of the
// dense qubit for register-segment ops, tile-local positions for quad ops).
// Fused blocks keep their matrices in the plan's aux table: the block's
// product, then one 4x4 per gate (the stages its interior errors split it
// into), each as its 16 frame variants; rsel holds the block's first matrix
// index and its stage count.
// Fused diagonal runs keep one DfRec per gate in the aux table (16-byte
// aligned).
template <typename T>
static void push_diag_record(const HostGate &g, int rb0, int rb1, std::vector<ntk::cx<T>> &out) {
  cd d[4];
  if (g.nq == 1) {
    d[0] = g.m[0];
    d[1] = g.m[3];
  } else {
    for (int i = 0; i < 4; ++i) d[i] = g.m[5 * i];
  }
  ntk::DfRec<T> r;
  std::memset(&r, 0, sizeof r);
  cd e[4];
  if (g.nq == 1 && rb0 < 0) {
    r.sa = r.sb = (uint32_t)g.q[0];
    e[0] = e[1] = d[0];
    e[2] = e[3] = d[1];     // b_a + 2 b_a is 0 or 3
  } else if (g.nq == 2 && rb0 < 0 && rb1 < 0) {
    r.sa = (uint32_t)g.q[0];
    r.sb = (uint32_t)g.q[1];
    for (int i = 0; i < 4; ++i) e[i] = d[i];
  } else {
    // register qubit on bit rb, the other qubit a (a one-qubit gate: none;
    // its bit is then read from the register qubit's frame word, and both
    // entries are equal)
    const bool r_is_1 = g.nq == 2 && rb1 >= 0;
    const int rb = r_is_1 ? rb1 : rb0;
    r.kr = 1u | ((uint32_t)rb << 4);
    r.rq = (uint32_t)(r_is_1 ? g.q[1] : g.q[0]);
    r.sa = r.sb = (uint32_t)(g.nq == 1 ? g.q[0] : (r_is_1 ? g.q[0] : g.q[1]));
    for (int ba = 0; ba < 2; ++ba) {
      cd lo, hi;   // register bit 0 / 1
      if (g.nq == 1) {
        lo = d[0];
        hi = d[1];
      } else if (r_is_1) {
        lo = d[ba];
        hi = d[ba + 2];
      } else {
        lo = d[2 * ba];
        hi = d[1 + 2 * ba];
      }
      e[ba] = lo;
      e[2 + ba] = hi / lo;
    }
  }
  for (int i = 0; i < 4; ++i) {
    r.p[2 * i] = (T)e[i].real();
    r.p[2 * i + 1] = (T)e[i].imag();
  }
  static_assert(sizeof(ntk::DfRec<T>) % sizeof(ntk::cx<T>) == 0, "record size");
  ntk::cx<T> w[sizeof(ntk::DfRec<T>) / sizeof(ntk::cx<T>)];
  std::memcpy(w, &r, sizeof r);
  for (const auto &x : w) out.push_back(x);
}

// Fixed-point form of a diagonal run (complex64), after its DfRecs: each
// gate's phase arg d(b) split into a constant per group and terms over the
// bits outside the registers (the gate kernel sums the terms whose bits are
// set, mod 2^32, then takes one sine and cosine per group).  local: the
// qubits held in the pass's tile; a term whose bits are both outside it is
// the same for the whole work-group.  Not formed (header 0) when a gate's
// entries are not unit complex numbers or the run has too many terms.
static void push_diag_fast(const Circuit &c, const HostOp &h, const std::vector<int> &rb, uint64_t local,
                           std::vector<ntk::cx<float>> &aux) {
  auto turns = [](double rad) {
    double t = rad / (2.0 * M_PI);
    t -= std::floor(t);
    return (uint32_t)(uint64_t)std::nearbyint(t * 4294967296.0);
  };
  std::vector<ntk::DfTerm> lane[5], uni[5];
  ntk::DfFast f;
  std::memset(&f, 0, sizeof f);
  uint32_t used = 0;
  bool ok = true;
  auto term = [&](int g, int qa, int qb, double ph0, double ph1) {
    const uint32_t a = turns(ph0), b = g < 4 ? turns(ph1) : 0u;
    if (a == 0 && b == 0) return;
    const bool u = ((local >> qa) & 1u) == 0 && ((local >> qb) & 1u) == 0;
    (u ? uni : lane)[g].push_back(ntk::DfTerm{(uint32_t)qa | ((uint32_t)qb << 8), a, b, 0u});
  };
  for (int gi : h.sub) {
    const HostGate &g = c.gates[(size_t)gi];
    cd d[4];
    const int nd = g.nq == 1 ? 2 : 4;
    if (g.nq == 1) {
      d[0] = g.m[0];
      d[1] = g.m[3];
    } else {
      for (int i = 0; i < 4; ++i) d[i] = g.m[5 * i];
    }
    double ph[4] = {0, 0, 0, 0};
    for (int i = 0; i < nd; ++i) {
      if (std::abs(std::abs(d[i]) - 1.0) > 1e-12) ok = false;
      ph[i] = std::arg(d[i]);
    }
    if (g.nq == 1) {
      const int q = g.q[0], r = rb[(size_t)q];
      if (r >= 0) {
        f.c0[r] += turns(ph[0]);
        f.c1[r] += turns(ph[1]);
        used |= 1u << r;
        f.rq |= (uint32_t)q << (8 * r);
      } else {
        f.c0[4] += turns(ph[0]);
        term(4, q, q, ph[1] - ph[0], 0);
      }
      continue;
    }
    // phase of (b_q0, b_q1) is ph[b_q0 + 2 b_q1]
    const int q0 = g.q[0], q1 = g.q[1], r0 = rb[(size_t)q0], r1 = rb[(size_t)q1];
    if (r0 >= 0 && r1 >= 0) {
      ok = false;   // the planner keeps such gates out of runs
    } else if (r0 < 0 && r1 < 0) {
      f.c0[4] += turns(ph[0]);
      term(4, q0, q0, ph[1] - ph[0], 0);
      term(4, q1, q1, ph[2] - ph[0], 0);
      term(4, q0, q1, ph[3] - ph[1] - ph[2] + ph[0], 0);
    } else {
      const bool reg1 = r1 >= 0;
      const int r = reg1 ? r1 : r0, qr = reg1 ? q1 : q0, qo = reg1 ? q0 : q1;
      auto phi = [&](int bo, int br) { return reg1 ? ph[bo + 2 * br] : ph[br + 2 * bo]; };
      f.c0[r] += turns(phi(0, 0));
      f.c1[r] += turns(phi(0, 1));
      used |= 1u << r;
      f.rq = (f.rq & ~(255u << (8 * r))) | ((uint32_t)qr << (8 * r));
      term(r, qo, qo, phi(1, 0) - phi(0, 0), phi(1, 1) - phi(0, 1));
    }
  }
  for (int g = 0; g < 5; ++g) {
    if (lane[g].size() > (size_t)ntk::DF_MAX_TERMS || uni[g].size() > (size_t)ntk::DF_MAX_TERMS) ok = false;
    f.nlane |= (uint32_t)std::min<size_t>(lane[g].size(), 63) << (6 * g);
    f.nuni |= (uint32_t)std::min<size_t>(uni[g].size(), 63) << (6 * g);
  }
  f.hdr = ok ? 1u | (used << 1) : 0u;
  std::vector<uint32_t> wds(sizeof f / 4);
  std::memcpy(wds.data(), &f, sizeof f);
  if (ok)
    for (int g = 0; g < 5; ++g)
      for (const auto *v : {&lane[g], &uni[g]})
        for (const ntk::DfTerm &t : *v) wds.insert(wds.end(), {t.sab, t.q0, t.q1, t.pad});
  for (size_t i = 0; i < wds.size(); i += 2) {
    ntk::cx<float> x;
    std::memcpy(&x, &wds[i], sizeof x);
    aux.push_back(x);
  }
}

template <typename T>
static void upload_ops(const Circuit &c, DevPlan &dp, const std::vector<int32_t> &code,
                       const std::vector<int32_t> &rsel, const std::vector<char> &swap_ab,
                       const std::vector<std::vector<int>> &reg_of_op, hipStream_t s) {
  const Plan &P = dp.plan;
  // two zero padding entries: the gate kernel loads the descriptor one past
  // a segment's last op
  std::vector<ntk::DevOp<T>> ops(P.ops.size() + 2);
  std::memset(ops.data(), 0, ops.size() * sizeof(ntk::DevOp<T>));
  std::vector<ntk::cx<T>> aux;
  std::vector<uint64_t> local_of_op(P.ops.size(), 0);
  for (const Pass &ps : P.passes)
    for (int o = ps.op_begin; o < ps.op_end; ++o) local_of_op[(size_t)o] = ps.local_mask;
  for (size_t o = 0; o < P.ops.size(); ++o) {
    const HostOp &h = P.ops[o];
    ntk::DevOp<T> &d = ops[o];
    d.cls = code[o];
    d.qa = h.qa;
    d.qb = h.qb;
    d.rsel = rsel[o];
    int nent = 0;
    switch (h.cls) {
      case OPC_G1: case OPC_C1: case OPC_D2: nent = 4; break;
      case OPC_D1: nent = 2; break;
      case OPC_G2: nent = 16; break;
      default: break;
    }
    for (int i = 0; i < nent; ++i) {
      d.m[2 * i] = (T)h.m[i].real();
      d.m[2 * i + 1] = (T)h.m[i].imag();
    }
    if (h.cls == OPC_L4) {
      // c and Im m01 of each RX-type gate, register bit 0 first
      for (int b = 0; b < 4; ++b) {
        d.m[2 * b] = (T)h.m[4 * b].real();
        d.m[2 * b + 1] = (T)h.m[4 * b + 1].imag();
      }
      continue;
    }
    if (h.cls == OPC_G4) {
      // matrix sets are addressed in units of 256 entries
      while (aux.size() % 256) aux.push_back(ntk::cx<T>{0, 0});
      const size_t first = aux.size() / 256;
      if (first + h.sub.size() + 1 >= ((size_t)1 << 24) || h.sub.size() > (size_t)MAX_BLOCK_GATES)
        throw Error(NT_ERR_UNSUPPORTED, "internal: fused-block table too large");
      push_variants<T>(h.m, swap_ab[o] != 0, aux);
      for (int g : h.sub) {
        cd E[16];
        embed_gate(c.gates[(size_t)g], h.qa, h.qb, E);
        push_variants<T>(E, swap_ab[o] != 0, aux);
      }
      d.rsel = (int32_t)((uint32_t)first | ((uint32_t)h.sub.size() << 24));
      if (swap_ab[o]) {
        d.qa = h.qb;
        d.qb = h.qa;
      }
      continue;
    }
    if (h.cls == OPC_DF) {
      while ((aux.size() * sizeof(ntk::cx<T>)) % 16) aux.push_back(ntk::cx<T>{0, 0});
      const size_t first = aux.size() * sizeof(ntk::cx<T>) / 16;
      if (first >= ((size_t)1 << 24) || h.sub.size() > (size_t)MAX_BLOCK_GATES)
        throw Error(NT_ERR_UNSUPPORTED, "internal: diagonal-run table too large");
      const std::vector<int> &rb = reg_of_op[o];   // register bit per qubit id (-1: none)
      for (int g : h.sub) {
        const HostGate &hg = c.gates[(size_t)g];
        push_diag_record<T>(hg, rb[hg.q[0]], hg.nq == 2 ? rb[hg.q[1]] : -1, aux);
      }
      if constexpr (sizeof(T) == 4) push_diag_fast(c, h, rb, local_of_op[o], aux);
      d.rsel = (int32_t)((uint32_t)first | ((uint32_t)h.sub.size() << 24));
      continue;
    }
    if (swap_ab[o]) {
      // two-qubit diagonal with qa on the higher register bit: the qubits
      // trade roles, so the entries of local index b_qa + 2 b_qb = 1 and 2
      // trade places
      d.qa = h.qb;
      d.qb = h.qa;
      std::swap(d.m[2], d.m[4]);
      std::swap(d.m[3], d.m[5]);
    }
  }
  dp.ops.ensure(ops.size() * sizeof(ntk::DevOp<T>));
  check_hip(hipMemcpyAsync(dp.ops.p, ops.data(), ops.size() * sizeof(ntk::DevOp<T>), hipMemcpyHostToDevice, s),
            "upload ops");
  dp.aux.ensure(std::max<size_t>(aux.size(), 1) * sizeof(ntk::cx<T>));
  if (!aux.empty())
    check_hip(hipMemcpyAsync(dp.aux.p, aux.data(), aux.size() * sizeof(ntk::cx<T>), hipMemcpyHostToDevice, s),
              "upload block matrices");
}

// Device tables of a plan (ops, segments, passes, site order and tags), in
// dp's buffers, and its per-pass bookkeeping; dp.plan and dp.prec are set.
void Ctx::upload_plan(const Circuit &c, DevPlan &dp) {
  const int pr = dp.prec;
  const Plan &P = dp.plan;
  const int L = P.L, R = P.R;
  dp.nthreads = 1 << (L - R);
  const int SW = pr == NT_C64 ? 4 : 3;
  // Algorithmic flops per amplitude of each pass: the sum over its gates of
  // each gate's own count (gate_flops), whatever ops the plan made of them.
  for (const Pass &ps : P.passes) {
    double f = 0;
    int ng = 0;
    for (int o = ps.op_begin; o < ps.op_end; ++o) {
      const HostOp &h = P.ops[o];
      for (int g : h.gates()) {
        f += gate_flops(c.gates[(size_t)g]);
        ++ng;
      }
    }
    dp.pass_flops_per_amp.push_back(f);
    dp.pass_gates.push_back(ng);
  }
  dp.pass_of_op.assign(P.ops.size(), 0);
  for (size_t p = 0; p < P.passes.size(); ++p)
    for (int o = P.passes[p].op_begin; o < P.passes[p].op_end; ++o) dp.pass_of_op[o] = (int)p;

  std::vector<ntk::DevSeg> segs(std::max<size_t>(P.segs.size(), 1));
  std::memset(segs.data(), 0, segs.size() * sizeof(ntk::DevSeg));
  std::vector<ntk::DevPass> dpass(P.passes.size());
  std::memset(dpass.data(), 0, dpass.size() * sizeof(ntk::DevPass));
  std::vector<int32_t> rsel(P.ops.size(), 0), code(P.ops.size(), 0);
  std::vector<char> swap_ab(P.ops.size(), 0);
  std::vector<std::vector<int>> reg_of_op(P.ops.size());
  for (size_t p = 0; p < P.passes.size(); ++p) {
    const Pass &ps = P.passes[p];
    std::vector<int> loc, nl;
    for (int q = 0; q < c.n; ++q) ((ps.local_mask >> q) & 1 ? loc : nl).push_back(q);
    if ((int)loc.size() != L) throw Error(NT_ERR_UNSUPPORTED, "internal: tile size mismatch");
    for (int q = 0; q < P.cfix; ++q)
      if (loc[q] != q) throw Error(NT_ERR_UNSUPPORTED, "internal: low qubits not local");
    for (size_t i = 0; i < loc.size(); ++i) dpass[p].locq[i] = (uint8_t)loc[i];
    for (int bb = 0; bb < P.R && P.L - P.R + bb < (int)loc.size(); ++bb) dpass[p].hq[bb] = (uint8_t)loc[P.L - P.R + bb];
    for (size_t i = 0; i < nl.size(); ++i) dpass[p].nlq[i] = (uint8_t)nl[i];
    for (int s = ps.seg_begin; s < ps.seg_end; ++s) {
      const Segment &sg = P.segs[s];
      ntk::DevSeg &d = segs[s];
      d.kind = sg.kind == SEG_QUAD ? ntk::SEG_KIND_QUAD : ntk::SEG_KIND_REG;
      d.op_begin = sg.op_begin;
      d.op_end = sg.op_end;
      auto local_pos = [&](int q) { return (int)(std::find(loc.begin(), loc.end(), q) - loc.begin()); };
      for (int o = sg.op_begin; o < sg.op_end; ++o) {
        const HostOp &h = P.ops[o];
        if (sg.kind == SEG_QUAD) {
          if (h.cls != OPC_G2) throw Error(NT_ERR_UNSUPPORTED, "internal: quad segment without a dense 2q op");
          const int pa = local_pos(h.qa), pb = local_pos(h.qb);
          if (pa >= L || pb >= L) throw Error(NT_ERR_UNSUPPORTED, "internal: quad op qubit not local");
          rsel[o] = pa | (pb << 4);
          code[o] = op_code(h, 0);
        } else if (h.cls == OPC_G4) {
          // fused block: its qubits on register bits (0, 1) or (2, 3); the
          // kernel takes qa on the lower bit
          auto rbit = [&](int q) {
            auto it = std::find(sg.reg_q.begin(), sg.reg_q.end(), q);
            if (it == sg.reg_q.end()) throw Error(NT_ERR_UNSUPPORTED, "internal: fused block outside the registers");
            return (int)(it - sg.reg_q.begin());
          };
          const int ba = rbit(h.qa), bb = rbit(h.qb);
          const int lo = std::min(ba, bb), hi = std::max(ba, bb);
          if (!(hi == lo + 1 && (lo & 1) == 0)) throw Error(NT_ERR_UNSUPPORTED, "internal: fused block off its register pair");
          if (((o - sg.op_begin) & 1) != (lo >> 1))
            throw Error(NT_ERR_UNSUPPORTED, "internal: fused block at the wrong segment offset parity");
          swap_ab[o] = ba > bb;
          code[o] = ntk::OPK_G4 * 4 + (lo >> 1);
        } else if (h.cls == OPC_NOP) {
          code[o] = ntk::OPK_NOP * 4;
        } else if (h.cls == OPC_L4) {
          if ((o - sg.op_begin) & 1) throw Error(NT_ERR_UNSUPPORTED, "internal: one-qubit layer at an odd segment offset");
          if (pr != NT_C64 || R != 4) throw Error(NT_ERR_UNSUPPORTED, "internal: one-qubit layer outside a complex64 plan");
          uint32_t qw = 0;
          for (int b = 0; b < 4; ++b) {
            const HostGate &hg = c.gates[(size_t)h.sub[(size_t)b]];
            if (hg.q[0] != sg.reg_q[(size_t)b]) throw Error(NT_ERR_UNSUPPORTED, "internal: one-qubit layer off its register bits");
            qw |= (uint32_t)hg.q[0] << (8 * b);
          }
          rsel[o] = (int32_t)qw;
          code[o] = ntk::OPK_L4 * 4;
        } else if (h.cls == OPC_SW) {
          // register permutation of the bit pair holding qa and qb
          auto rbit = [&](int q) {
            auto it = std::find(sg.reg_q.begin(), sg.reg_q.end(), q);
            if (it == sg.reg_q.end()) throw Error(NT_ERR_UNSUPPORTED, "internal: SWAP outside the registers");
            return (int)(it - sg.reg_q.begin());
          };
          const int ba = rbit(h.qa), bb = rbit(h.qb);
          const int lo = std::min(ba, bb), hi = std::max(ba, bb);
          int k = 0;
          while (k < 6 && !(ntk::D2RR_PAIRS[k][0] == lo && ntk::D2RR_PAIRS[k][1] == hi)) ++k;
          if (k == 6 || lo == hi) throw Error(NT_ERR_UNSUPPORTED, "internal: register-bit pair out of range");
          code[o] = ntk::OPK_SW * 4 + k;
        } else if (h.cls == OPC_DF) {
          if ((o - sg.op_begin) & 1) throw Error(NT_ERR_UNSUPPORTED, "internal: diagonal run at an odd segment offset");
          code[o] = ntk::OPK_DF * 4;
          reg_of_op[o].assign((size_t)c.n, -1);
          for (int b = 0; b < R; ++b) reg_of_op[o][(size_t)sg.reg_q[b]] = b;
          for (int g : h.sub) {
            const HostGate &hg = c.gates[(size_t)g];
            if (hg.nq == 2 && reg_of_op[o][(size_t)hg.q[0]] >= 0 && reg_of_op[o][(size_t)hg.q[1]] >= 0)
              throw Error(NT_ERR_UNSUPPORTED, "internal: diagonal run gate with both qubits in the registers");
          }
        } else if (h.cls == OPC_G1 || h.cls == OPC_C1 || h.cls == OPC_D1 || h.cls == OPC_D2) {
          auto rmask = [&](int q) -> int32_t {
            if (q < 0) return 0;
            auto it = std::find(sg.reg_q.begin(), sg.reg_q.end(), q);
            return it == sg.reg_q.end() ? 0 : (int32_t)(1u << (it - sg.reg_q.begin()));
          };
          const int32_t am = rmask(h.qa), bm = rmask(h.qb);
          rsel[o] = am | (bm << 4);
          int rb = 0;
          if (h.cls == OPC_G1 || h.cls == OPC_C1) {
            if (!am) throw Error(NT_ERR_UNSUPPORTED, "internal: dense op outside its segment's registers");
            rb = __builtin_ctz((unsigned)am);
          }
          code[o] = op_code(h, rb);
          // diagonal ops with exactly one register qubit: body specialized on its bit
          if (h.cls == OPC_D1 && am) code[o] = ntk::OPK_D1R * 4 + __builtin_ctz((unsigned)am);
          if (h.cls == OPC_D2 && am && !bm) code[o] = ntk::OPK_D2A * 4 + __builtin_ctz((unsigned)am);
          if (h.cls == OPC_D2 && bm && !am) code[o] = ntk::OPK_D2B * 4 + __builtin_ctz((unsigned)bm);
          if (h.cls == OPC_D2 && am && bm) {
            const int lo = __builtin_ctz((unsigned)(am < bm ? am : bm)), hi = __builtin_ctz((unsigned)(am < bm ? bm : am));
            // the kernel takes qa on the lower register bit
            if (am > bm) {
              swap_ab[o] = 1;
              rsel[o] = bm | (am << 4);
            }
            int k = 0;
            while (k < 6 && !(ntk::D2RR_PAIRS[k][0] == lo && ntk::D2RR_PAIRS[k][1] == hi)) ++k;
            if (k == 6) throw Error(NT_ERR_UNSUPPORTED, "internal: register-bit pair out of range");
            code[o] = ntk::OPK_D2RR * 4 + k;
          }
        } else {
          throw Error(NT_ERR_UNSUPPORTED, "internal: dense 2q op in a register segment");
        }
      }
      std::vector<int> is_reg(L, 0);
      for (int b = 0; b < R; ++b) {
        int lp = (int)(std::find(loc.begin(), loc.end(), sg.reg_q[b]) - loc.begin());
        if (lp >= L) throw Error(NT_ERR_UNSUPPORTED, "internal: register qubit not local");
        d.rpos[b] = (uint8_t)lp;
        d.rq[b] = (uint8_t)sg.reg_q[b];
        is_reg[lp] = 1;
      }
      std::vector<int> tpos;
      for (int lp = 0; lp < L; ++lp)
        if (!is_reg[lp]) tpos.push_back(lp);
      tpos = thread_bit_order(tpos, SW);
      for (size_t i = 0; i < tpos.size(); ++i) {
        d.tpos[i] = (uint8_t)tpos[i];
        d.tq[i] = (uint8_t)loc[tpos[i]];
        d.tpos_w[i] = (uint32_t)tpos[i];
        d.tq_w[i] = (uint32_t)loc[tpos[i]];
      }
      const uint32_t amp_bytes = pr == NT_C64 ? 8u : 16u;
      for (int r = 0; r < (1 << R); ++r) {
        uint32_t off = 0;
        for (int b = 0; b < R; ++b)
          if ((r >> b) & 1) off ^= lds_swizzle(1u << d.rpos[b], SW) * amp_bytes;
        d.slot_off[r] = off;
      }
    }
  }
  dp.passes.ensure(dpass.size() * sizeof(ntk::DevPass));
  check_hip(hipMemcpyAsync(dp.passes.p, dpass.data(), dpass.size() * sizeof(ntk::DevPass), hipMemcpyHostToDevice,
                           stream), "upload passes");
  dp.segs.ensure(segs.size() * sizeof(ntk::DevSeg));
  check_hip(hipMemcpyAsync(dp.segs.p, segs.data(), segs.size() * sizeof(ntk::DevSeg), hipMemcpyHostToDevice, stream),
            "upload segments");
  if (pr == NT_C64) upload_ops<float>(c, dp, code, rsel, swap_ab, reg_of_op, stream);
  else upload_ops<double>(c, dp, code, rsel, swap_ab, reg_of_op, stream);

  const size_t S = std::max<size_t>(P.app_site.size(), 1);
  std::vector<int32_t> ident(S);
  std::vector<uint32_t> itag(S);
  for (size_t k = 0; k < S; ++k) {
    ident[k] = (int32_t)k;
    itag[k] = (uint32_t)k << 8;
  }
  dp.app_order.ensure(S * 4);
  dp.app_tag.ensure(S * 4);
  dp.site_order.ensure(S * 4);
  dp.site_tag.ensure(S * 4);
  if (!P.app_site.empty()) {
    check_hip(hipMemcpyAsync(dp.app_order.p, P.app_site.data(), P.app_site.size() * 4, hipMemcpyHostToDevice, stream), "upload");
    check_hip(hipMemcpyAsync(dp.app_tag.p, P.app_tag.data(), P.app_tag.size() * 4, hipMemcpyHostToDevice, stream), "upload");
  }
  check_hip(hipMemcpyAsync(dp.site_order.p, ident.data(), S * 4, hipMemcpyHostToDevice, stream), "upload");
  check_hip(hipMemcpyAsync(dp.site_tag.p, itag.data(), S * 4, hipMemcpyHostToDevice, stream), "upload");
  sync();   // host vectors go out of scope
}

DevPlan &Ctx::plan_for(const Circuit &c, int pr) {
  // the tile and fusion overrides are part of the key: changing them builds a new plan
  const int slot = pr == NT_C64 ? 1 : 2;
  auto key = std::make_pair(c.serial, pr + 16 * c.tile_override[slot] + 1024 * c.fuse_width[slot]);
  auto it = plans.find(key);
  if (it != plans.end()) {
    it->second->last_use = ++use_clock;
    return *it->second;
  }
  evict_plans();
  auto dp = std::make_unique<DevPlan>();
  dp->last_use = ++use_clock;
  dp->prec = pr;
  dp->plan = choose_plan(c, pr);
  upload_plan(c, *dp);
  DevPlan &ref = *dp;
  plans.emplace(key, std::move(dp));
  return ref;
}

// Drop least-recently-used plans (and their reference states and
// checkpoints) until one more fits under the count and byte budgets; plans
// pinned by a batched run stay.
void Ctx::evict_plans() {
  for (;;) {
    size_t bytes = 0;
    auto victim = plans.end();
    for (auto it = plans.begin(); it != plans.end(); ++it) {
      bytes += it->second->footprint();
      if (it->second->pins == 0 && (victim == plans.end() || it->second->last_use < victim->second->last_use))
        victim = it;
    }
    if (plans.size() < max_plans && bytes <= plan_budget) return;
    if (victim == plans.end()) return;
    sync();   // its buffers may still be read by queued work
    plans.erase(victim);
  }
}

uint64_t Ctx::batch_size(const Circuit &c, const DevPlan &dp, uint64_t n_traj) {
  const size_t state = ((size_t)1 << c.n) * amp_bytes(dp.prec);
  uint64_t cap = max_batch ? max_batch : 65536;
  if (dp.plan.passes.size() > 1) {
    size_t freeb = 0, total = 0;
    check_hip(hipMemGetInfo(&freeb, &total), "hipMemGetInfo");
    size_t held = states.bytes;             // reusable
    size_t avail = freeb + held;
    size_t margin = (size_t)1 << 30;
    if (avail < state + margin / 4)
      throw Error(NT_ERR_OUT_OF_MEMORY, "not enough device memory for one state vector");
    size_t budget = std::min(avail > margin ? avail - margin : avail / 2, (size_t)32 << 30);
    uint64_t by_mem = std::max<uint64_t>(1, budget / state);
    if (!max_batch) cap = std::min<uint64_t>(cap, by_mem);
    else if (cap > by_mem) throw Error(NT_ERR_OUT_OF_MEMORY, "max_batch state vectors do not fit in device memory");
  }
  return std::max<uint64_t>(1, std::min<uint64_t>(cap, std::max<uint64_t>(n_traj, 1)));
}

static hipEvent_t take_event(std::vector<hipEvent_t> &pool) {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  check_hip(hipEventCreate(&e), "hipEventCreate");
  return e;
}

void Ctx::timing_flush() {
  if (ev_pending.empty()) return;
  sync();
  for (size_t i = 0; i < ev_pending.size(); ++i) {
    float ms = 0;
    check_hip(hipEventElapsedTime(&ms, ev_pending[i].first, ev_pending[i].second), "hipEventElapsedTime");
    t_ms += ms;
    t_bytes += ev_bytes[i];
    t_updates += ev_updates[i];
    t_flops += ev_flops[i];
    ++t_launches;
    ev_pool.push_back(ev_pending[i].first);
    ev_pool.push_back(ev_pending[i].second);
  }
  ev_pending.clear();
  ev_bytes.clear();
  ev_updates.clear();
  ev_flops.clear();
}

// Gate-kernel instance a plan needs (the fused ops it holds).
static int plan_features(const Plan &P) {
  return (P.n_fused > 0 ? ntk::FEAT_G4 : 0) | (P.n_diag > 0 ? ntk::FEAT_DF : 0) | (P.n_layer > 0 ? ntk::FEAT_L4 : 0);
}

// One launch of every pass of the plan over a batch.  With `start`, batch
// entries are sorted by their first pass and pass p runs the prefix
// active[p] of them; entries starting at p > 0 load the error-free checkpoint
// taken before pass p.  With `capture`, the state of entry 0 is copied into
// the checkpoint slots after each pass (error-free reference run).
template <typename T>
static void run_passes(Ctx &cx, const Circuit &c, DevPlan &dp, ntk::cx<T> *state, const PassRun &r) {
  const Plan &P = dp.plan;
  const int np = (int)P.passes.size();
  const size_t dim = (size_t)1 << c.n;
  const size_t bytes = dim * sizeof(ntk::cx<T>);
  for (int p = 0; p < np; ++p) {
    const int Bp = r.active ? (*r.active)[p] : r.B;
    if (Bp <= 0) continue;
    const Pass &ps = P.passes[p];
    ntk::PassArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.state = state;
    a.ref = static_cast<const ntk::cx<T> *>(dp.ref.p);
    a.ops = static_cast<const ntk::DevOp<T> *>(dp.ops.p);
    a.aux = static_cast<const ntk::cx<T> *>(dp.aux.p);
    a.segs = static_cast<const ntk::DevSeg *>(dp.segs.p);
    a.events = r.events;
    a.ev_count = r.ev_count;
    a.partials = r.partials;
    // frames double-buffered by pass parity
    a.frame_out = r.frames ? r.frames + (size_t)(p & 1) * 4 * r.B : nullptr;
    a.frame_in = (r.frames && p > 0) ? r.frames + (size_t)((p - 1) & 1) * 4 * r.B : nullptr;
    a.state_stride = dim;
    a.ev_stride = r.ev_stride;
    a.B = Bp;
    a.L = P.L;
    a.ntile_bits = c.n - P.L;
    a.seg_begin = ps.seg_begin;
    a.seg_end = ps.seg_end;
    a.op_begin = ps.op_begin;
    a.flags = (p == np - 1 ? r.last_flags : ntk::PF_STORE);
    if (r.capture) {
      a.flags = ntk::PF_STORE | ntk::PF_NORM;
      a.partials = dp.ckpt_partials.as<double>() + (size_t)p * ((size_t)1 << (c.n - P.L)) * ntk::NPART;
    }
    a.init_index = 0;
    a.pass = static_cast<const ntk::DevPass *>(dp.passes.p) + p;
    a.start = r.start;
    a.ckpt = (r.start && p > 0) ? dp.ckpt.as<ntk::cx<T>>() + (size_t)(p - 1) * dim : nullptr;
    a.pass_index = p;
    a.end = r.end;
    a.ref_here = r.end ? (p == np - 1 ? static_cast<const ntk::cx<T> *>(dp.ref.p)
                                      : dp.ckpt.as<ntk::cx<T>>() + (size_t)p * dim)
                       : nullptr;
    a.crit = r.crit;
    a.target = r.target;
    a.heavy_med = r.heavy_med;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (cx.timing) {
      e0 = take_event(cx.ev_pool);
      e1 = take_event(cx.ev_pool);
      check_hip(hipEventRecord(e0, cx.stream), "hipEventRecord");
    }
    check_hip(ntk::launch_pass<T>(a, P.R, dp.nthreads, plan_features(P), cx.stream), "k_pass launch");
    if (cx.timing) {
      check_hip(hipEventRecord(e1, cx.stream), "hipEventRecord");
      // algorithmic HBM bytes: every pass reads and writes each state once,
      // except that pass 0 does not read and a scoring pass reads the
      // reference instead of writing.
      double per_state = (double)bytes;
      double reads = p == 0 ? 0.0 : 1.0;
      double writes = (a.flags & ntk::PF_SCORE) ? 0.0 : 1.0;
      double refr = (a.flags & ntk::PF_SCORE) ? 1.0 : 0.0;
      cx.ev_pending.emplace_back(e0, e1);
      cx.ev_bytes.push_back(per_state * Bp * (reads + writes + refr));
      cx.ev_updates.push_back((double)dim * Bp * dp.pass_gates[p]);
      double fl = dp.pass_flops_per_amp[p] + ((a.flags & ntk::PF_SCORE) ? 8.0 : 0.0);
      cx.ev_flops.push_back((double)dim * Bp * fl);
      if (cx.ev_pending.size() >= 2048) cx.timing_flush();
    }
    if (r.capture && p + 1 < np)
      check_hip(hipMemcpyAsync(dp.ckpt.as<char>() + (size_t)p * bytes, state, bytes, hipMemcpyDeviceToDevice,
                               cx.stream), "checkpoint copy");
  }
}

void Ctx::ensure_reference(const Circuit &c, DevPlan &dp) {
  if (dp.ref_ready) return;
  const size_t dim = (size_t)1 << c.n;
  const size_t ntiles = (size_t)1 << (c.n - dp.plan.L);
  size_t freeb = 0, total = 0;
  check_hip(hipMemGetInfo(&freeb, &total), "hipMemGetInfo");
  if (dim * amp_bytes(dp.prec) + (64u << 20) > freeb)
    throw Error(NT_ERR_OUT_OF_MEMORY, "not enough device memory for the reference state");
  dp.ref.ensure(dim * amp_bytes(dp.prec));
  dp.nref.ensure(sizeof(double));
  dp.ref_partials.ensure(ntiles * ntk::NPART * sizeof(double));
  ev_count.ensure(sizeof(int32_t) * 4);
  events.ensure(16);
  check_hip(ntk::launch_zero_words(ev_count.as<uint32_t>(), 1, stream), "k_zero_words launch");
  bool was = timing;
  timing = false;
  PassRun r;
  r.B = 1;
  r.last_flags = ntk::PF_STORE | ntk::PF_NORM;
  r.events = events.as<uint32_t>();
  r.ev_count = ev_count.as<int32_t>();
  r.ev_stride = 1;
  r.partials = dp.ref_partials.as<double>();
  if (dp.prec == NT_C64) run_passes<float>(*this, c, dp, dp.ref.as<ntk::cx<float>>(), r);
  else run_passes<double>(*this, c, dp, dp.ref.as<ntk::cx<double>>(), r);
  timing = was;
  check_hip(ntk::launch_norm_final(dp.ref_partials.as<double>(), (int)ntiles, dp.nref.as<double>(), stream),
            "k_norm_final launch");
  check_hip(hipMemcpyAsync(&dp.nref_host, dp.nref.p, sizeof(double), hipMemcpyDeviceToHost, stream), "copy norm");
  sync();
  dp.ref_ready = true;
}

void Ctx::simulate_batch(const Circuit &c, DevPlan &dp, uint64_t seed, uint64_t t0, int B, int mode, double tau,
                         double *fid_dev, uint64_t *count_dev, const Thresholds &th) {
  const Plan &P = dp.plan;
  const size_t dim = (size_t)1 << c.n;
  const size_t ntiles = (size_t)1 << (c.n - P.L);
  const int S = (int)std::max<int64_t>(c.S, 1);
  events.ensure((size_t)B * S * 4);
  ev_count.ensure((size_t)B * 4);
  partials.ensure((size_t)B * ntiles * ntk::NPART * sizeof(double));
  frames.ensure((size_t)2 * B * 4 * sizeof(uint32_t));
  const bool need_states = P.passes.size() > 1 || mode == 1;
  if (need_states) states.ensure((size_t)B * dim * amp_bytes(dp.prec));

  ntk::SampleArgs sa;
  std::memset(&sa, 0, sizeof sa);
  sa.seed = seed;
  sa.cid = c.cid;
  sa.t0 = t0;
  sa.t_fire = th.t_fire;
  sa.c_x = th.c_x;
  sa.c_xy = th.c_xy;
  sa.always = th.always;
  sa.B = B;
  sa.S = (int)c.S;
  sa.ev_stride = S;
  sa.order = dp.app_order.as<int32_t>();
  sa.tag = dp.app_tag.as<uint32_t>();
  sa.events = events.as<uint32_t>();
  sa.ev_count = ev_count.as<int32_t>();
  check_hip(ntk::launch_sample(sa, stream), "k_sample launch");

  PassRun r;
  r.B = B;
  r.last_flags = mode == 0 ? ntk::PF_SCORE : ntk::PF_STORE;
  r.events = events.as<uint32_t>();
  r.ev_count = ev_count.as<int32_t>();
  r.ev_stride = S;
  r.partials = partials.as<double>();
  r.frames = frames.as<uint32_t>();
  if (mode == 0) criterion_args(c, dp, r);
  if (dp.prec == NT_C64) run_passes<float>(*this, c, dp, need_states ? states.as<ntk::cx<float>>() : nullptr, r);
  else run_passes<double>(*this, c, dp, need_states ? states.as<ntk::cx<double>>() : nullptr, r);
  if (mode == 0)
    check_hip(ntk::launch_finalize(partials.as<double>(), (int)ntiles, B, dp.nref.as<double>(), nullptr, r.crit, tau,
                                   fid_dev, count_dev, stream),
              "k_finalize launch");
}

void Ctx::run(const Circuit &c, uint64_t seed, uint64_t t0, uint64_t n, double tau, double *fid_out,
              uint64_t *count_out, double *sum_out) {
  check_hip(hipSetDevice(device), "hipSetDevice");
  check_target(c);
  if (shortcuts) {
    run_shortcut(c, seed, t0, n, tau, fid_out, count_out, sum_out);
    return;
  }
  DevPlan &dp = plan_for(c, prec);
  ensure_reference(c, dp);
  const Thresholds th = make_thresholds(px, py, pz);
  const uint64_t bs = batch_size(c, dp, n);
  const bool dev_out = is_device_pointer(fid_out);
  count.ensure(sizeof(uint64_t));
  check_hip(ntk::launch_zero_words(count.as<uint32_t>(), 2, stream), "k_zero_words launch");
  if (!dev_out) fid.ensure((size_t)bs * sizeof(double));
  // host copy of the values when their sum is asked for and fid_out is not on the host
  std::vector<double> hv(sum_out && (!fid_out || dev_out) ? n : 0);
  double *host_vals = sum_out ? (fid_out && !dev_out ? fid_out : hv.data()) : (dev_out ? nullptr : fid_out);
  for (uint64_t off = 0; off < n; off += bs) {
    const int B = (int)std::min<uint64_t>(bs, n - off);
    double *fd = dev_out ? fid_out + off : fid.as<double>();
    simulate_batch(c, dp, seed, t0 + off, B, 0, tau, fd, count.as<uint64_t>(), th);
    if (host_vals)
      check_hip(hipMemcpyAsync(host_vals + off, fd, (size_t)B * sizeof(double), hipMemcpyDeviceToHost, stream),
                "copy fidelities");
  }
  uint64_t cnt = 0;
  check_hip(hipMemcpyAsync(&cnt, count.p, sizeof cnt, hipMemcpyDeviceToHost, stream), "copy count");
  sync();
  if (count_out) *count_out = cnt;
  if (sum_out) {
    double sum = 0;
    for (uint64_t i = 0; i < n; ++i) sum += host_vals[i];
    *sum_out = sum;
  }
}

// nt_run without device allocation: the plan tables, the reference state and
// every per-trajectory buffer of the call are carved out of this device's
// static scratch array (ntk::SCRATCH_BYTES), rebuilt on every call.  The
// short-cuts are not used (every trajectory is simulated in full); values are
// those of nt_run with the short-cuts off.
void Ctx::run_noalloc(const Circuit &c, uint64_t seed, uint64_t t0, uint64_t n, double tau, double *fid_out,
                      uint64_t *count_out, double *sum_out) {
  check_hip(hipSetDevice(device), "hipSetDevice");
  check_target(c);
  if (!scratch) throw Error(NT_ERR_DEVICE, "no scratch array address for this device");
  Arena ar;
  ar.base = static_cast<char *>(scratch);
  ar.cap = ntk::SCRATCH_BYTES;
  // the context's working buffers point into the arena for the call
  DevBuf *work[] = {&events, &ev_count, &partials, &frames, &states, &fid, &count, &hist, &tmp};
  struct Held {
    DevBuf *b;
    void *p;
    size_t bytes;
    Arena *arena;
  };
  std::vector<Held> held;
  for (DevBuf *b : work) {
    held.push_back({b, b->p, b->bytes, b->arena});
    b->p = nullptr;
    b->bytes = 0;
    b->arena = &ar;
  }
  const bool was_timing = timing;
  timing = false;
  struct Restore {
    std::vector<Held> &h;
    bool &timing;
    bool was;
    ~Restore() {
      for (Held &x : h) {
        x.b->p = x.p;
        x.b->bytes = x.bytes;
        x.b->arena = x.arena;
      }
      timing = was;
    }
  } restore{held, timing, was_timing};

  DevPlan dp;
  for (DevBuf *b : {&dp.ops, &dp.aux, &dp.segs, &dp.passes, &dp.app_order, &dp.app_tag, &dp.site_order, &dp.site_tag, &dp.ref,
                    &dp.nref, &dp.ref_partials, &dp.ckpt, &dp.ckpt_partials, &dp.nref_pass})
    b->arena = &ar;
  dp.prec = prec;
  dp.plan = choose_plan(c, prec);
  upload_plan(c, dp);
  ensure_reference(c, dp);
  PassRun probe;
  if (crit != NT_CRIT_FIDELITY) criterion_args(c, dp, probe);   // heavy-set median before the chunks
  const Thresholds th = make_thresholds(px, py, pz);
  const Plan &P = dp.plan;
  const size_t dim = (size_t)1 << c.n;
  const size_t ntiles = (size_t)1 << (c.n - P.L);
  const size_t S = (size_t)std::max<int64_t>(c.S, 1);
  const bool dev_out = is_device_pointer(fid_out);
  count.ensure(sizeof(uint64_t));
  // bytes per trajectory of a chunk, 256-byte alignment of each buffer included
  const size_t per = S * 4 + 4 + ntiles * ntk::NPART * sizeof(double) + 2 * 4 * sizeof(uint32_t) +
                     (P.passes.size() > 1 ? dim * amp_bytes(prec) : 0) + (dev_out ? 0 : sizeof(double));
  const size_t slack = 8 * 256;
  const size_t left = ar.cap - std::min(ar.cap, ((ar.off + 255) & ~(size_t)255) + slack);
  const uint64_t bs = std::min<uint64_t>(n, left / per);
  if (bs == 0)
    throw Error(NT_ERR_UNSUPPORTED, "one trajectory of this circuit does not fit in the " +
                                        std::to_string(ntk::SCRATCH_BYTES >> 20) +
                                        " MiB scratch array of the allocation-free entry point");
  check_hip(ntk::launch_zero_words(count.as<uint32_t>(), 2, stream), "k_zero_words launch");
  if (!dev_out) fid.ensure((size_t)bs * sizeof(double));
  std::vector<double> hv(sum_out && (!fid_out || dev_out) ? n : 0);
  double *host_vals = sum_out ? (fid_out && !dev_out ? fid_out : hv.data()) : (dev_out ? nullptr : fid_out);
  for (uint64_t off = 0; off < n; off += bs) {
    const int B = (int)std::min<uint64_t>(bs, n - off);
    double *fd = dev_out ? fid_out + off : fid.as<double>();
    simulate_batch(c, dp, seed, t0 + off, B, 0, tau, fd, count.as<uint64_t>(), th);
    if (host_vals)
      check_hip(hipMemcpyAsync(host_vals + off, fd, (size_t)B * sizeof(double), hipMemcpyDeviceToHost, stream),
                "copy fidelities");
  }
  uint64_t cnt = 0;
  check_hip(hipMemcpyAsync(&cnt, count.p, sizeof cnt, hipMemcpyDeviceToHost, stream), "copy count");
  sync();
  if (count_out) *count_out = cnt;
  if (sum_out) {
    double sum = 0;
    for (uint64_t i = 0; i < n; ++i) sum += host_vals[i];
    *sum_out = sum;
  }
}

void Ctx::check_target(const Circuit &c) const {
  if (crit == NT_CRIT_TARGET_PROB && (target >> c.n) != 0)
    throw Error(NT_ERR_INVALID_ARG, "target basis state out of range for this circuit");
}

double Ctx::success(const Circuit &c, uint64_t seed, uint64_t t0, uint64_t n, double tau) {
  uint64_t cnt = 0;
  double sum = 0;
  run(c, seed, t0, n, tau, nullptr, &cnt, crit == NT_CRIT_FIDELITY ? nullptr : &sum);
  return crit == NT_CRIT_FIDELITY ? (double)cnt / (double)n : sum / (double)n;
}

// Exact median of the error-free probabilities |a_k|^2 (FP64, computed as in
// the scoring epilogue) by radix selection over their bit patterns: four
// 16-bit digits, integer histograms on the device, the scan on the host.
double Ctx::heavy_median(const Circuit &c, DevPlan &dp) {
  if (dp.med_ready) return dp.heavy_med;
  ensure_reference(c, dp);
  const uint64_t dim = (uint64_t)1 << c.n;
  hist.ensure(65536 * sizeof(uint32_t));
  std::vector<uint32_t> h(65536);
  auto select = [&](uint64_t k) {
    uint64_t prefix = 0;
    for (int shift = 48; shift >= 0; shift -= 16) {
      check_hip(ntk::launch_zero_words(hist.as<uint32_t>(), 65536, stream), "k_zero_words launch");
      if (dp.prec == NT_C64)
        check_hip(ntk::launch_prob_hist<float>(dp.ref.as<ntk::cx<float>>(), dim, shift, prefix, hist.as<uint32_t>(),
                                               stream), "k_prob_hist launch");
      else
        check_hip(ntk::launch_prob_hist<double>(dp.ref.as<ntk::cx<double>>(), dim, shift, prefix,
                                                hist.as<uint32_t>(), stream), "k_prob_hist launch");
      check_hip(hipMemcpyAsync(h.data(), hist.p, 65536 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream),
                "copy histogram");
      sync();
      uint64_t d = 0;
      for (; d < 65536; ++d) {
        if (k < h[d]) break;
        k -= h[d];
      }
      if (d == 65536) throw Error(NT_ERR_DEVICE, "median selection lost its rank");
      prefix = (prefix << 16) | d;
    }
    double v;
    std::memcpy(&v, &prefix, sizeof v);
    return v;
  };
  double med;
  if (dim & 1) med = select(dim / 2);
  else med = 0.5 * (select(dim / 2 - 1) + select(dim / 2));
  dp.heavy_med = med;
  dp.med_ready = true;
  return med;
}

double Ctx::reference_value(const Circuit &c, DevPlan &dp, double tau) {
  if (crit == NT_CRIT_FIDELITY) return 1.0;   // F of the error-free state is exactly 1
  const auto key = std::make_pair(crit, crit == NT_CRIT_TARGET_PROB ? target : (uint64_t)0);
  auto it = dp.ref_value.find(key);
  if (it != dp.ref_value.end()) return it->second;
  // one entry without events, from the last checkpoint when there is one:
  // bit-identical to an error-free trajectory run from pass 0
  const int np = (int)dp.plan.passes.size();
  const std::vector<uint32_t> ev(1, 0u);
  const std::vector<int32_t> cnt(1, 0), st(1, (dp.ckpt_ready && np > 1) ? np - 1 : 0);
  double v = 0;
  score_entries(c, dp, 1, ev, 1, cnt, st, tau, &v);
  dp.ref_value[key] = v;
  return v;
}

void Ctx::criterion_args(const Circuit &c, DevPlan &dp, PassRun &r) {
  r.crit = crit;
  r.target = (uint32_t)target;
  r.heavy_med = crit == NT_CRIT_HEAVY ? heavy_median(c, dp) : 0.0;
}

// Error-free checkpoints: the reference run repeated with the state copied
// out after every pass.  Returns false (and stores nothing) when they do not
// fit in device memory; callers then start every trajectory at pass 0.
bool Ctx::ensure_checkpoints(const Circuit &c, DevPlan &dp) {
  if (dp.ckpt_ready) return true;
  ensure_reference(c, dp);
  const int np = (int)dp.plan.passes.size();
  if (np <= 1) {
    // no checkpoints; the per-pass reference norm of the single pass is <R|R>
    dp.nref_pass.ensure(sizeof(double));
    check_hip(hipMemcpyAsync(dp.nref_pass.p, dp.nref.p, sizeof(double), hipMemcpyDeviceToDevice, stream),
              "copy norm");
    sync();
    dp.ckpt_ready = true;
    return true;
  }
  const size_t bytes = (size_t)(np - 1) * ((size_t)1 << c.n) * amp_bytes(dp.prec);
  size_t freeb = 0, total = 0;
  check_hip(hipMemGetInfo(&freeb, &total), "hipMemGetInfo");
  if (bytes + states.bytes + ((size_t)4 << 30) > freeb + states.bytes) return false;
  dp.ckpt.ensure(bytes);
  const size_t ntiles = (size_t)1 << (c.n - dp.plan.L);
  dp.ckpt_partials.ensure((size_t)np * ntiles * ntk::NPART * sizeof(double));
  dp.nref_pass.ensure((size_t)np * sizeof(double));
  bool was = timing;
  timing = false;
  PassRun r;
  r.B = 1;
  r.last_flags = ntk::PF_STORE | ntk::PF_NORM;
  ev_count.ensure(sizeof(int32_t) * 4);
  events.ensure(16);
  check_hip(ntk::launch_zero_words(ev_count.as<uint32_t>(), 1, stream), "k_zero_words launch");
  r.events = events.as<uint32_t>();
  r.ev_count = ev_count.as<int32_t>();
  r.partials = dp.ref_partials.as<double>();
  r.capture = true;
  if (dp.prec == NT_C64) run_passes<float>(*this, c, dp, dp.ref.as<ntk::cx<float>>(), r);
  else run_passes<double>(*this, c, dp, dp.ref.as<ntk::cx<double>>(), r);
  for (int p = 0; p < np; ++p)
    check_hip(ntk::launch_norm_final(dp.ckpt_partials.as<double>() + (size_t)p * ntiles * ntk::NPART, (int)ntiles,
                                     dp.nref_pass.as<double>() + p, stream), "k_norm_final launch");
  timing = was;
  sync();
  dp.ckpt_ready = true;
  return true;
}

// Run batch entries whose events and counts are already in `events` /
// `ev_count` (ev_stride words each); start: first pass per entry, sorted
// ascending.  Fidelities go to fid_host[0..B).
static void run_entries(Ctx &cx, const Circuit &c, DevPlan &dp, int B, int ev_stride,
                        const std::vector<int32_t> &start, double tau, double *fid_host,
                        const std::vector<int32_t> *end = nullptr) {
  const Plan &P = dp.plan;
  const int np = (int)P.passes.size();
  const size_t dim = (size_t)1 << c.n;
  const size_t ntiles = (size_t)1 << (c.n - P.L);
  cx.partials.ensure((size_t)B * ntiles * ntk::NPART * sizeof(double));
  cx.frames.ensure((size_t)2 * B * 4 * sizeof(uint32_t));
  cx.fid.ensure((size_t)B * sizeof(double));
  cx.count.ensure(sizeof(uint64_t));
  cx.start.ensure((size_t)B * sizeof(int32_t));
  if (np > 1) cx.states.ensure((size_t)B * dim * amp_bytes(dp.prec));
  std::vector<int> active(np, 0);
  for (int p = 0; p < np; ++p)
    active[p] = (int)(std::upper_bound(start.begin(), start.end(), p) - start.begin());
  check_hip(hipMemcpyAsync(cx.start.p, start.data(), (size_t)B * sizeof(int32_t), hipMemcpyHostToDevice, cx.stream),
            "upload start passes");
  PassRun r;
  r.B = B;
  r.last_flags = ntk::PF_SCORE;
  r.events = cx.events.as<uint32_t>();
  r.ev_count = cx.ev_count.as<int32_t>();
  r.ev_stride = ev_stride;
  r.partials = cx.partials.as<double>();
  r.frames = cx.frames.as<uint32_t>();
  r.start = cx.start.as<int32_t>();
  r.active = &active;
  cx.criterion_args(c, dp, r);
  if (end) {
    cx.end.ensure((size_t)B * sizeof(int32_t));
    check_hip(hipMemcpyAsync(cx.end.p, end->data(), (size_t)B * sizeof(int32_t), hipMemcpyHostToDevice, cx.stream),
              "upload end passes");
    r.end = cx.end.as<int32_t>();
  }
  if (dp.prec == NT_C64) run_passes<float>(cx, c, dp, np > 1 ? cx.states.as<ntk::cx<float>>() : nullptr, r);
  else run_passes<double>(cx, c, dp, np > 1 ? cx.states.as<ntk::cx<double>>() : nullptr, r);
  if (end) {
    // k_finalize reads the reference norm after pass end[b] from nref_pass:
    // each end pass must be a pass of the plan whose norm is there
    for (int32_t e : *end)
      if (e < 0 || e >= np || (size_t)(e + 1) * sizeof(double) > dp.nref_pass.bytes)
        throw Error(NT_ERR_UNSUPPORTED, "internal: end pass without a reference norm");
  }
  check_hip(ntk::launch_finalize(cx.partials.as<double>(), (int)ntiles, B,
                                 end ? dp.nref_pass.as<double>() : dp.nref.as<double>(), r.end, r.crit, tau,
                                 cx.fid.as<double>(), cx.count.as<uint64_t>(), cx.stream),
            "k_finalize launch");
  check_hip(hipMemcpyAsync(fid_host, cx.fid.p, (size_t)B * sizeof(double), hipMemcpyDeviceToHost, cx.stream),
            "copy fidelities");
  cx.sync();
}

void Ctx::score_entries(const Circuit &c, DevPlan &dp, int B, const std::vector<uint32_t> &ev, int ev_stride,
                        const std::vector<int32_t> &cnt, const std::vector<int32_t> &st, double tau,
                        double *fid_host) {
  events.ensure((size_t)B * ev_stride * 4);
  ev_count.ensure((size_t)B * 4);
  check_hip(hipMemcpyAsync(events.p, ev.data(), (size_t)B * ev_stride * 4, hipMemcpyHostToDevice, stream),
            "upload events");
  check_hip(hipMemcpyAsync(ev_count.p, cnt.data(), (size_t)B * 4, hipMemcpyHostToDevice, stream), "upload counts");
  run_entries(*this, c, dp, B, ev_stride, st, tau, fid_host);
}

// Monte Carlo run with the short-cuts: a trajectory with no fired site has
// the reference state itself (F = 1 exactly, not simulated), a trajectory
// starts from the error-free checkpoint before the pass holding its first
// error, and values of fired sets already simulated are reused; with these
// the results are bit-identical to the plain run.  The last-error short-cut
// (scoring right after the pass of the last error) is exact in arithmetic
// only: its fidelities differ from the plain run's by rounding.
void Ctx::run_shortcut(const Circuit &c, uint64_t seed, uint64_t t0, uint64_t n, double tau, double *fid_out,
                       uint64_t *count_out, double *sum_out) {
  DevPlan &dp = plan_for(c, prec);
  ensure_reference(c, dp);
  const bool have_ckpt = (shortcuts & (SC_CHECKPOINT | SC_LAST_ERROR)) && ensure_checkpoints(c, dp);
  // The measurement-probability criteria are not invariant under the
  // error-free suffix of the circuit: no early scoring for them.
  const bool early_end = have_ckpt && (shortcuts & SC_LAST_ERROR) && crit == NT_CRIT_FIDELITY &&
                         dp.plan.passes.size() > 1;
  const double v_ref = (shortcuts & SC_ZERO_FIRED) ? reference_value(c, dp, tau) : 0.0;
  const Thresholds th = make_thresholds(px, py, pz);
  const int S = (int)std::max<int64_t>(c.S, 1);
  const int np = (int)dp.plan.passes.size();
  std::vector<double> fh(n, 0.0);
  const bool reuse_on = (shortcuts & SC_REUSE) != 0;
  if (reuse_on) {
    ReuseKey k;
    k.serial = c.serial;
    k.cid = c.cid;
    k.tile = c.tile_override[dp.prec == NT_C64 ? 1 : 2] + 64 * c.fuse_width[dp.prec == NT_C64 ? 1 : 2];
    k.seed = seed;
    k.target = target;
    k.c_x = th.c_x;
    k.c_xy = th.c_xy;
    k.always_types = th.always & 6u;
    k.prec = dp.prec;
    k.crit = crit;
    k.flags = shortcuts & ~SC_REUSE;
    if (!reuse_valid || !(k == reuse_key) || reuse_values > ((size_t)1 << 24)) {
      reuse.clear();
      reuse_values = 0;
    }
    reuse_key = k;
    reuse_valid = true;
  }
  const uint64_t chunk = std::max<uint64_t>(1, std::min<uint64_t>(n, (256u << 20) / ((uint64_t)S * 4)));
  const uint64_t bs = batch_size(c, dp, n);
  std::vector<int32_t> hcnt;
  std::vector<uint32_t> hfirst;
  for (uint64_t off = 0; off < n; off += chunk) {
    const int Bc = (int)std::min<uint64_t>(chunk, n - off);
    events.ensure((size_t)Bc * S * 4);
    ev_count.ensure((size_t)Bc * 4);
    ntk::SampleArgs sa;
    std::memset(&sa, 0, sizeof sa);
    sa.seed = seed; sa.cid = c.cid; sa.t0 = t0 + off;
    sa.t_fire = th.t_fire; sa.c_x = th.c_x; sa.c_xy = th.c_xy; sa.always = th.always;
    sa.B = Bc; sa.S = (int)c.S; sa.ev_stride = S;
    sa.order = dp.app_order.as<int32_t>();
    sa.tag = dp.app_tag.as<uint32_t>();
    sa.events = events.as<uint32_t>();
    sa.ev_count = ev_count.as<int32_t>();
    check_hip(ntk::launch_sample(sa, stream), "k_sample launch");
    hcnt.resize(Bc);
    hfirst.resize(2 * (size_t)Bc);
    firstlast.ensure((size_t)Bc * 8);
    check_hip(ntk::launch_first_last(events.as<uint32_t>(), ev_count.as<int32_t>(), S, Bc, firstlast.as<uint32_t>(),
                                     stream), "k_first_last launch");
    check_hip(hipMemcpyAsync(hcnt.data(), ev_count.p, (size_t)Bc * 4, hipMemcpyDeviceToHost, stream), "copy counts");
    check_hip(hipMemcpyAsync(hfirst.data(), firstlast.p, (size_t)Bc * 8, hipMemcpyDeviceToHost, stream),
              "copy first/last events");
    sync();
    // (first pass, index within the chunk, last pass) of the trajectories to simulate
    std::vector<std::tuple<int32_t, int32_t, int32_t>> act;
    for (int b = 0; b < Bc; ++b) {
      if (hcnt[b] == 0 && (shortcuts & SC_ZERO_FIRED)) {
        fh[off + b] = v_ref;
        continue;
      }
      if (reuse_on) {
        // same count at the same Pauli-type proportions: the same fired set
        auto it = reuse.find(t0 + off + (uint64_t)b);
        bool hit = false;
        if (it != reuse.end())
          for (const auto &e : it->second)
            if (e.first == hcnt[b]) {
              fh[off + b] = e.second;
              hit = true;
              break;
            }
        if (hit) continue;
      }
      int32_t sp = 0, ep = np - 1;
      if (have_ckpt) sp = hcnt[b] ? dp.pass_of_op[hfirst[2 * b] >> ntk::EV_OP_SHIFT] : np - 1;
      if (early_end) ep = hcnt[b] ? dp.pass_of_op[hfirst[2 * b + 1] >> ntk::EV_OP_SHIFT] : np - 1;
      act.emplace_back(sp, b, ep);
    }
    std::stable_sort(act.begin(), act.end());
    std::vector<uint64_t> tl;
    std::vector<int32_t> st, en;
    std::vector<double> fsub;
    for (size_t a0 = 0; a0 < act.size(); a0 += bs) {
      const int B = (int)std::min<size_t>(bs, act.size() - a0);
      tl.resize(B);
      st.resize(B);
      en.resize(B);
      fsub.resize(B);
      for (int j = 0; j < B; ++j) {
        tl[j] = t0 + off + (uint64_t)std::get<1>(act[a0 + j]);
        st[j] = std::get<0>(act[a0 + j]);
        en[j] = std::get<2>(act[a0 + j]);
      }
      this->tlist.ensure((size_t)B * 8);
      check_hip(hipMemcpyAsync(this->tlist.p, tl.data(), (size_t)B * 8, hipMemcpyHostToDevice, stream), "upload ids");
      events.ensure((size_t)B * S * 4);
      ev_count.ensure((size_t)B * 4);
      sa.B = B;
      sa.events = events.as<uint32_t>();     // (re)allocated above
      sa.ev_count = ev_count.as<int32_t>();
      sa.tlist = this->tlist.as<uint64_t>();
      check_hip(ntk::launch_sample(sa, stream), "k_sample launch");
      sa.tlist = nullptr;
      run_entries(*this, c, dp, B, S, st, tau, fsub.data(), early_end ? &en : nullptr);
      for (int j = 0; j < B; ++j) {
        const int b = std::get<1>(act[a0 + j]);
        fh[off + b] = fsub[j];
        if (reuse_on) {
          reuse[t0 + off + (uint64_t)b].emplace_back(hcnt[b], fsub[j]);
          ++reuse_values;
        }
      }
    }
  }
  uint64_t cnt = 0;
  double sum = 0;
  for (uint64_t i = 0; i < n; ++i) {
    cnt += fh[i] >= tau ? 1 : 0;
    sum += fh[i];
  }
  if (count_out) *count_out = cnt;
  if (sum_out) *sum_out = sum;
  if (fid_out) {
    if (is_device_pointer(fid_out))
      check_hip(hipMemcpy(fid_out, fh.data(), n * sizeof(double), hipMemcpyHostToDevice), "copy fidelities");
    else
      std::memcpy(fid_out, fh.data(), n * sizeof(double));
  }
}

// Exhaustive single-error simulation (Sec. IV-B.1, Eq. 3): every site, every
// Pauli, one error each; entries in plan order start at their error's pass.
void Ctx::exhaustive(const Circuit &c, double tau, double *fid_out, double P_e[3], double *P_R) {
  check_hip(hipSetDevice(device), "hipSetDevice");
  check_target(c);
  DevPlan &dp = plan_for(c, prec);
  ensure_reference(c, dp);
  const bool have_ckpt = ensure_checkpoints(c, dp);
  const Plan &P = dp.plan;
  const int64_t S = c.S;
  const int64_t total = 3 * S;
  std::vector<double> fall((size_t)std::max<int64_t>(total, 1), 0.0);
  const uint64_t bs = batch_size(c, dp, (uint64_t)std::max<int64_t>(total, 1));
  std::vector<uint32_t> ev;
  std::vector<int32_t> cnt, st;
  std::vector<double> fsub;
  for (int64_t off = 0; off < total; off += (int64_t)bs) {
    const int B = (int)std::min<int64_t>((int64_t)bs, total - off);
    ev.resize(B);
    cnt.assign(B, 1);
    st.resize(B);
    fsub.resize(B);
    for (int j = 0; j < B; ++j) {
      const int64_t i = off + j, k = i / 3;
      ev[j] = P.app_tag[(size_t)k] | (uint32_t)(i % 3 + 1);
      st[j] = have_ckpt ? dp.pass_of_op[P.app_tag[(size_t)k] >> ntk::EV_OP_SHIFT] : 0;
    }
    score_entries(c, dp, B, ev, 1, cnt, st, tau, fsub.data());
    for (int j = 0; j < B; ++j) {
      const int64_t i = off + j, k = i / 3;
      fall[(size_t)P.app_site[(size_t)k] * 3 + (size_t)(i % 3)] = fsub[j];
    }
  }
  // success of one state: F >= tau for the fidelity, the measurement
  // probability itself for the other criteria
  const bool fidc = crit == NT_CRIT_FIDELITY;
  for (int e = 0; e < 3; ++e) {
    double s = 0;
    for (int64_t site = 0; site < S; ++site) {
      const double v = fall[(size_t)site * 3 + e];
      s += fidc ? (v >= tau ? 1.0 : 0.0) : v;
    }
    P_e[e] = S ? s / (double)S : 0.0;
  }
  *P_R = fidc ? (1.0 >= tau ? 1.0 : 0.0) : reference_value(c, dp, tau);
  if (fid_out) std::memcpy(fid_out, fall.data(), (size_t)total * sizeof(double));
}

void Ctx::sample_sites(const Circuit &c, uint64_t seed, uint64_t t0, uint64_t n, uint64_t *offsets, int32_t *sites,
                       uint8_t *paulis, int64_t cap, int64_t *n_out) {
  check_hip(hipSetDevice(device), "hipSetDevice");
  DevPlan &dp = plan_for(c, prec);
  const Thresholds th = make_thresholds(px, py, pz);
  const int S = (int)std::max<int64_t>(c.S, 1);
  const uint64_t chunk = std::max<uint64_t>(1, std::min<uint64_t>(n, (256u << 20) / ((uint64_t)S * 4)));
  events.ensure((size_t)chunk * S * 4);
  ev_count.ensure((size_t)chunk * 4);
  std::vector<uint32_t> hev((size_t)chunk * S);
  std::vector<int32_t> hcnt(chunk);
  int64_t total = 0;
  offsets[0] = 0;
  for (uint64_t off = 0; off < n; off += chunk) {
    const int B = (int)std::min<uint64_t>(chunk, n - off);
    ntk::SampleArgs sa;
    std::memset(&sa, 0, sizeof sa);
    sa.seed = seed; sa.cid = c.cid; sa.t0 = t0 + off;
    sa.t_fire = th.t_fire; sa.c_x = th.c_x; sa.c_xy = th.c_xy; sa.always = th.always;
    sa.B = B; sa.S = (int)c.S; sa.ev_stride = S;
    sa.order = dp.site_order.as<int32_t>();
    sa.tag = dp.site_tag.as<uint32_t>();
    sa.events = events.as<uint32_t>();
    sa.ev_count = ev_count.as<int32_t>();
    check_hip(ntk::launch_sample(sa, stream), "k_sample launch");
    check_hip(hipMemcpyAsync(hcnt.data(), ev_count.p, (size_t)B * 4, hipMemcpyDeviceToHost, stream), "copy counts");
    check_hip(hipMemcpyAsync(hev.data(), events.p, (size_t)B * S * 4, hipMemcpyDeviceToHost, stream), "copy events");
    sync();
    for (int b = 0; b < B; ++b) {
      for (int k = 0; k < hcnt[b]; ++k) {
        if (total + k < cap) {
          const uint32_t e = hev[(size_t)b * S + k];
          sites[total + k] = (int32_t)(e >> 8);
          paulis[total + k] = (uint8_t)(e & 3u);
        }
      }
      total += hcnt[b];
      offsets[off + b + 1] = (uint64_t)total;
    }
  }
  *n_out = total;
  if (total > cap) throw Error(NT_ERR_BUFFER_TOO_SMALL, "site buffers too small; required size in *n_out");
}

void Ctx::final_state(const Circuit &c, uint64_t seed, uint64_t traj, void *out, int64_t len) {
  check_hip(hipSetDevice(device), "hipSetDevice");
  const size_t dim = (size_t)1 << c.n;
  if (len < (int64_t)dim) throw Error(NT_ERR_BUFFER_TOO_SMALL, "amps_out shorter than 2^n");
  DevPlan &dp = plan_for(c, prec);
  ensure_reference(c, dp);
  const Thresholds th = make_thresholds(px, py, pz);
  simulate_batch(c, dp, seed, traj, 1, 1, 0.0, nullptr, nullptr, th);
  // frames of a batch of one, double-buffered by pass parity
  const uint32_t *last_frame = frames.as<uint32_t>() + (size_t)((dp.plan.passes.size() - 1) & 1) * 4;
  const size_t bytes = dim * amp_bytes(prec);
  const bool dev_out = is_device_pointer(out);
  void *dst = out;
  if (!dev_out) {
    tmp.ensure(bytes);
    dst = tmp.p;
  }
  if (prec == NT_C64)
    check_hip(ntk::launch_unframe<float>(states.as<ntk::cx<float>>(), static_cast<ntk::cx<float> *>(dst), dim,
                                         last_frame, stream), "k_unframe launch");
  else
    check_hip(ntk::launch_unframe<double>(states.as<ntk::cx<double>>(), static_cast<ntk::cx<double> *>(dst), dim,
                                          last_frame, stream), "k_unframe launch");
  if (!dev_out) check_hip(hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, stream), "copy state");
  sync();
}

void Ctx::reference_state(const Circuit &c, void *out, int64_t len) {
  check_hip(hipSetDevice(device), "hipSetDevice");
  const size_t dim = (size_t)1 << c.n;
  if (len < (int64_t)dim) throw Error(NT_ERR_BUFFER_TOO_SMALL, "amps_out shorter than 2^n");
  DevPlan &dp = plan_for(c, prec);
  ensure_reference(c, dp);
  const size_t bytes = dim * amp_bytes(prec);
  check_hip(hipMemcpyAsync(out, dp.ref.p, bytes, is_device_pointer(out) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           stream), "copy reference");
  sync();
}

}  // namespace nt

namespace nt {

// Batched Monte Carlo over many circuits.  Circuits whose plan is one pass
// over one tile (n <= tile width) are grouped by tile shape; each group runs
// as one sampling launch, one gate-pass launch and one finalize launch per
// trajectory chunk, with per-circuit plan pointers in a descriptor table.
// Larger circuits run their usual pass sequence back to back on the stream,
// with no host synchronization between circuits.
void Ctx::run_batch(const std::vector<const Circuit *> &cs, uint64_t seed, uint64_t t0, uint64_t n, double tau,
                    double *vals_out, uint64_t *counts_out, double *sums_out) {
  check_hip(hipSetDevice(device), "hipSetDevice");
  const size_t nc = cs.size();
  for (const Circuit *c : cs) check_target(*c);
  const Thresholds th = make_thresholds(px, py, pz);
  const bool dev_out = is_device_pointer(vals_out);
  bvals.ensure(nc * n * sizeof(double));
  bcounts.ensure(nc * sizeof(uint64_t));
  check_hip(ntk::launch_zero_words(bcounts.as<uint32_t>(), 2 * (uint64_t)nc, stream), "k_zero_words launch");
  double *vals_dev = dev_out ? vals_out : bvals.as<double>();
  const bool c64 = prec == NT_C64;
  // zero-fired trajectories of one-tile circuits are not simulated (fidelity
  // criterion: F = 1 exactly either way)
  const int skip0 = ((shortcuts & SC_ZERO_FIRED) && crit == NT_CRIT_FIDELITY) ? ntk::PF_SKIP0 : 0;
  std::vector<uint64_t> host_counts(nc, 0);

  size_t i0 = 0;
  while (i0 < nc) {
    // a window of circuits whose plans and reference states are held together
    std::vector<DevPlan *> dps;
    size_t bytes = 0, i1 = i0;
    while (i1 < nc) {
      DevPlan &dp = plan_for(*cs[i1], prec);
      ++dp.pins;
      dps.push_back(&dp);
      ensure_reference(*cs[i1], dp);
      if (crit == NT_CRIT_HEAVY) heavy_median(*cs[i1], dp);
      bytes += dp.footprint();
      ++i1;
      if (bytes > plan_budget / 2) break;
    }
    struct Unpin {
      std::vector<DevPlan *> &v;
      ~Unpin() { for (DevPlan *d : v) --d->pins; }
    } unpin{dps};

    // group the one-pass, one-tile circuits by tile shape
    std::map<std::pair<int, int>, std::vector<size_t>> groups;   // (L, R) -> window slots
    std::vector<size_t> big;
    for (size_t k = 0; k < dps.size(); ++k) {
      const Plan &P = dps[k]->plan;
      if (P.passes.size() == 1 && P.L == cs[i0 + k]->n) groups[{P.L, P.R}].push_back(k);
      else big.push_back(k);
    }
    // descriptor tables of every group, uploaded once for the window
    std::vector<ntk::MultiItem<float>> mf;
    std::vector<ntk::MultiItem<double>> md;
    std::vector<ntk::SampleItem> si;
    std::vector<int32_t> imap;
    std::vector<double> nref;
    std::vector<size_t> gbase;
    for (auto &g : groups) {
      gbase.push_back(si.size());
      for (size_t k : g.second) {
        DevPlan &dp = *dps[k];
        const Circuit &c = *cs[i0 + k];
        const Pass &ps = dp.plan.passes[0];
        ntk::MultiItem<float> a;
        ntk::MultiItem<double> b;
        std::memset(&a, 0, sizeof a);
        std::memset(&b, 0, sizeof b);
        a.ops = static_cast<const ntk::DevOp<float> *>(dp.ops.p);
        b.ops = static_cast<const ntk::DevOp<double> *>(dp.ops.p);
        a.aux = static_cast<const ntk::cx<float> *>(dp.aux.p);
        b.aux = static_cast<const ntk::cx<double> *>(dp.aux.p);
        a.segs = b.segs = static_cast<const ntk::DevSeg *>(dp.segs.p);
        a.pass = b.pass = static_cast<const ntk::DevPass *>(dp.passes.p);
        a.ref = static_cast<const ntk::cx<float> *>(dp.ref.p);
        b.ref = static_cast<const ntk::cx<double> *>(dp.ref.p);
        a.seg_begin = b.seg_begin = ps.seg_begin;
        a.seg_end = b.seg_end = ps.seg_end;
        a.op_begin = b.op_begin = ps.op_begin;
        a.heavy_med = b.heavy_med = dp.heavy_med;
        a.nref = b.nref = dp.nref_host;
        mf.push_back(a);
        md.push_back(b);
        ntk::SampleItem s;
        std::memset(&s, 0, sizeof s);
        s.cid = c.cid;
        s.order = dp.app_order.as<int32_t>();
        s.tag = dp.app_tag.as<uint32_t>();
        s.S = (int32_t)c.S;
        si.push_back(s);
        imap.push_back((int32_t)(i0 + k));
        nref.push_back(dp.nref_host);
      }
    }
    if (!si.empty()) {
      const size_t ni = si.size();
      multi_items.ensure(ni * (c64 ? sizeof(ntk::MultiItem<float>) : sizeof(ntk::MultiItem<double>)));
      sample_items.ensure(ni * sizeof(ntk::SampleItem));
      item_map.ensure(ni * sizeof(int32_t));
      multi_nref.ensure(ni * sizeof(double));
      if (c64)
        check_hip(hipMemcpyAsync(multi_items.p, mf.data(), ni * sizeof(ntk::MultiItem<float>), hipMemcpyHostToDevice,
                                 stream), "upload batch tables");
      else
        check_hip(hipMemcpyAsync(multi_items.p, md.data(), ni * sizeof(ntk::MultiItem<double>),
                                 hipMemcpyHostToDevice, stream), "upload batch tables");
      check_hip(hipMemcpyAsync(sample_items.p, si.data(), ni * sizeof(ntk::SampleItem), hipMemcpyHostToDevice, stream),
                "upload batch tables");
      check_hip(hipMemcpyAsync(item_map.p, imap.data(), ni * sizeof(int32_t), hipMemcpyHostToDevice, stream),
                "upload batch tables");
      check_hip(hipMemcpyAsync(multi_nref.p, nref.data(), ni * sizeof(double), hipMemcpyHostToDevice, stream),
                "upload batch tables");
    }
    size_t gi = 0;
    for (auto &g : groups) {
      const int L = g.first.first, R = g.first.second;
      const size_t base = gbase[gi++];
      const size_t ng = g.second.size();
      int64_t smax = 1;
      int feat = 0;
      for (size_t k : g.second) {
        smax = std::max<int64_t>(smax, cs[i0 + k]->S);
        feat |= plan_features(dps[k]->plan);
      }
      // trajectories per circuit per launch: bounded work-group count and event memory
      uint64_t bc = std::min<uint64_t>(n, std::max<uint64_t>(1, ((uint64_t)1 << 20) / ng));
      bc = std::min<uint64_t>(bc, std::max<uint64_t>(1, (((uint64_t)512 << 20) / (4 * (uint64_t)smax)) / ng));
      for (uint64_t off = 0; off < n; off += bc) {
        const int per = (int)std::min<uint64_t>(bc, n - off);
        const int items = (int)(ng * (size_t)per);
        events.ensure((size_t)items * smax * 4);
        ev_count.ensure((size_t)items * 4);
        partials.ensure((size_t)items * ntk::NPART * sizeof(double));
        ntk::SampleArgs sa;
        std::memset(&sa, 0, sizeof sa);
        sa.seed = seed;
        sa.t0 = t0 + off;
        sa.t_fire = th.t_fire;
        sa.c_x = th.c_x;
        sa.c_xy = th.c_xy;
        sa.always = th.always;
        sa.B = items;
        sa.ev_stride = (int)smax;
        sa.events = events.as<uint32_t>();
        sa.ev_count = ev_count.as<int32_t>();
        sa.multi = sample_items.as<ntk::SampleItem>() + base;
        sa.per_item = per;
        check_hip(ntk::launch_sample(sa, stream), "k_sample launch");
        const int nthreads = 1 << (L - R);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
          e0 = take_event(ev_pool);
          e1 = take_event(ev_pool);
          check_hip(hipEventRecord(e0, stream), "hipEventRecord");
        }
        if (c64) {
          ntk::PassArgs<float> a;
          std::memset(&a, 0, sizeof a);
          a.events = events.as<uint32_t>();
          a.ev_count = ev_count.as<int32_t>();
          a.partials = partials.as<double>();
          a.ev_stride = (int)smax;
          a.B = items;
          a.L = L;
          a.flags = ntk::PF_SCORE | skip0;
          a.crit = crit;
          a.target = (uint32_t)target;
          a.multi = multi_items.as<ntk::MultiItem<float>>() + base;
          a.per_item = per;
          check_hip(ntk::launch_pass<float>(a, R, nthreads, feat, stream), "k_pass launch");
        } else {
          ntk::PassArgs<double> a;
          std::memset(&a, 0, sizeof a);
          a.events = events.as<uint32_t>();
          a.ev_count = ev_count.as<int32_t>();
          a.partials = partials.as<double>();
          a.ev_stride = (int)smax;
          a.B = items;
          a.L = L;
          a.flags = ntk::PF_SCORE | skip0;
          a.crit = crit;
          a.target = (uint32_t)target;
          a.multi = multi_items.as<ntk::MultiItem<double>>() + base;
          a.per_item = per;
          check_hip(ntk::launch_pass<double>(a, R, nthreads, feat, stream), "k_pass launch");
        }
        if (timing) {
          // a scoring pass over one tile reads the reference once per trajectory
          check_hip(hipEventRecord(e1, stream), "hipEventRecord");
          double by = 0, up = 0, fl = 0;
          for (size_t k : g.second) {
            const double dim = (double)((uint64_t)1 << cs[i0 + k]->n);
            by += dim * (double)amp_bytes(prec);
            up += dim * (double)cs[i0 + k]->gates.size();
            fl += dim * (dps[k]->pass_flops_per_amp[0] + 8.0);
          }
          ev_pending.emplace_back(e0, e1);
          ev_bytes.push_back(by * per);
          ev_updates.push_back(up * per);
          ev_flops.push_back(fl * per);
          if (ev_pending.size() >= 2048) timing_flush();
        }
        check_hip(ntk::launch_finalize_multi(partials.as<double>(), 1, items, multi_nref.as<double>() + base, per,
                                             item_map.as<int32_t>() + base, (int64_t)n, (int64_t)off, crit, tau,
                                             vals_dev, bcounts.as<uint64_t>(), stream),
                  "k_finalize launch");
      }
    }
    for (size_t k : big) {
      const Circuit &c = *cs[i0 + k];
      DevPlan &dp = *dps[k];
      if (shortcuts) {
        // the short-cut path of a single run (synchronizes per chunk)
        uint64_t cnt = 0;
        run_shortcut(c, seed, t0, n, tau, vals_dev + (i0 + k) * n, &cnt, nullptr);
        host_counts[i0 + k] = cnt;
        continue;
      }
      const uint64_t bs = batch_size(c, dp, n);
      for (uint64_t off = 0; off < n; off += bs) {
        const int B = (int)std::min<uint64_t>(bs, n - off);
        simulate_batch(c, dp, seed, t0 + off, B, 0, tau, vals_dev + (i0 + k) * n + off,
                       bcounts.as<uint64_t>() + (i0 + k), th);
      }
    }
    sync();   // host tables of this window go out of scope
    i0 = i1;
  }
  std::vector<double> hv;
  double *host_vals = nullptr;
  if (vals_out && !dev_out) host_vals = vals_out;
  else if (sums_out) {
    hv.resize(nc * n);
    host_vals = hv.data();
  }
  if (host_vals)
    check_hip(hipMemcpyAsync(host_vals, vals_dev, nc * n * sizeof(double), hipMemcpyDeviceToHost, stream),
              "copy values");
  std::vector<uint64_t> hc(nc);
  check_hip(hipMemcpyAsync(hc.data(), bcounts.p, nc * sizeof(uint64_t), hipMemcpyDeviceToHost, stream), "copy counts");
  sync();
  for (size_t i = 0; i < nc; ++i) hc[i] += host_counts[i];
  if (counts_out) std::memcpy(counts_out, hc.data(), nc * sizeof(uint64_t));
  if (sums_out)
    for (size_t i = 0; i < nc; ++i) {
      double s = 0;
      for (uint64_t j = 0; j < n; ++j) s += host_vals[i * n + j];
      sums_out[i] = s;
    }
}

}  // namespace nt
