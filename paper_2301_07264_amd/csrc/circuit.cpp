// Circuit ingest: validation, gate matrices (FP64), text format, and the
// classification of gates into the simulator's op classes.
//
// Gate definitions follow the conventions stated in nisqtol.h: R_P(theta) =
// exp(-i theta P / 2), U(a,b,c) = Rz(a) Ry(b) Rz(c), CNOT lists (control,
// target), CP phases |11>, RZZ = exp(-i g Z(x)Z / 2); two-qubit matrices act on
// local index b_q0 + 2 b_q1.  The Pauli gates are those of Eq. 2.
#include <atomic>
#include <cmath>
#include <cstring>
#include <fstream>
#include <sstream>

#include "nt_internal.hpp"

namespace nt {

static const char *KIND_NAMES[NT_NUM_GATE_KINDS] = {
    "H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "U", "U1Q",
    "CNOT", "CZ", "CP", "SWAP", "RZZ", "U2Q"};

int kind_arity(int kind) { return kind >= NT_CNOT ? 2 : 1; }
const char *kind_name(int kind) { return (kind >= 0 && kind < NT_NUM_GATE_KINDS) ? KIND_NAMES[kind] : "?"; }
int kind_from_name(const std::string &s) {
  for (int k = 0; k < NT_NUM_GATE_KINDS; ++k)
    if (s == KIND_NAMES[k]) return k;
  return -1;
}

int kind_nparam(int kind) {
  switch (kind) {
    case NT_RX: case NT_RY: case NT_RZ: case NT_CP: case NT_RZZ: return 1;
    case NT_U: return 3;
    default: return 0;
  }
}

// 2x2 rotation factors.
static void rz2(double t, cd *m) { m[0] = std::polar(1.0, -t / 2); m[1] = 0; m[2] = 0; m[3] = std::polar(1.0, t / 2); }
static void ry2(double t, cd *m) {
  double c = std::cos(t / 2), s = std::sin(t / 2);
  m[0] = c; m[1] = -s; m[2] = s; m[3] = c;
}
static void mul2(const cd *a, const cd *b, cd *o) {
  cd r0 = a[0] * b[0] + a[1] * b[2], r1 = a[0] * b[1] + a[1] * b[3];
  cd r2 = a[2] * b[0] + a[3] * b[2], r3 = a[2] * b[1] + a[3] * b[3];
  o[0] = r0; o[1] = r1; o[2] = r2; o[3] = r3;
}

void gate_matrix(int kind, const double *p, const double *umat, cd *m) {
  for (int i = 0; i < 16; ++i) m[i] = 0;
  const cd I(0, 1);
  const double h = 1.0 / std::sqrt(2.0);
  switch (kind) {
    case NT_H: m[0] = h; m[1] = h; m[2] = h; m[3] = -h; break;
    case NT_X: m[1] = 1; m[2] = 1; break;
    case NT_Y: m[1] = -I; m[2] = I; break;
    case NT_Z: m[0] = 1; m[3] = -1; break;
    case NT_S: m[0] = 1; m[3] = I; break;
    case NT_T: m[0] = 1; m[3] = std::polar(1.0, M_PI / 4); break;
    case NT_RX: {
      double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
      m[0] = c; m[1] = -I * s; m[2] = -I * s; m[3] = c;
      break;
    }
    case NT_RY: ry2(p[0], m); break;
    case NT_RZ: rz2(p[0], m); break;
    case NT_U: {
      cd a[4], b[4], c[4], t[4];
      rz2(p[0], a); ry2(p[1], b); rz2(p[2], c);
      mul2(a, b, t);
      mul2(t, c, m);
      break;
    }
    case NT_U1Q:
      for (int i = 0; i < 4; ++i) m[i] = cd(umat[2 * i], umat[2 * i + 1]);
      break;
    case NT_CNOT:  // control = local bit 0, target = local bit 1
      m[0 * 4 + 0] = 1; m[2 * 4 + 2] = 1; m[1 * 4 + 3] = 1; m[3 * 4 + 1] = 1;
      break;
    case NT_CZ: m[0] = 1; m[5] = 1; m[10] = 1; m[15] = -1; break;
    case NT_CP: m[0] = 1; m[5] = 1; m[10] = 1; m[15] = std::polar(1.0, p[0]); break;
    case NT_SWAP: m[0] = 1; m[1 * 4 + 2] = 1; m[2 * 4 + 1] = 1; m[15] = 1; break;
    case NT_RZZ: {
      cd e = std::polar(1.0, -p[0] / 2), f = std::polar(1.0, p[0] / 2);
      m[0] = e; m[5] = f; m[10] = f; m[15] = e;
      break;
    }
    case NT_U2Q:
      for (int i = 0; i < 16; ++i) m[i] = cd(umat[2 * i], umat[2 * i + 1]);
      break;
    default: throw Error(NT_ERR_INVALID_ARG, "unknown gate kind");
  }
}

static std::atomic<uint64_t> g_serial{1};

static void validate_and_fill(Circuit *c, int n, const nt_gate *gates, int64_t G) {
  if (n < 1 || n > 32) throw Error(NT_ERR_INVALID_ARG, "n_qubits must be in [1, 32]");
  if (G < 0) throw Error(NT_ERR_INVALID_ARG, "n_gates must be >= 0");
  if (G > 0 && !gates) throw Error(NT_ERR_INVALID_ARG, "gates is NULL");
  if (G > (int64_t(1) << 19)) throw Error(NT_ERR_UNSUPPORTED, "more than 2^19 gates");
  c->n = n;
  c->gates.resize((size_t)G);
  c->S = 0;
  for (int64_t g = 0; g < G; ++g) {
    const nt_gate &in = gates[g];
    HostGate &hg = c->gates[(size_t)g];
    if (in.kind >= NT_NUM_GATE_KINDS)
      throw Error(NT_ERR_INVALID_ARG, "gate " + std::to_string(g) + ": unknown kind " + std::to_string(in.kind));
    int ar = kind_arity(in.kind);
    if (in.nq != ar)
      throw Error(NT_ERR_INVALID_ARG, "gate " + std::to_string(g) + ": nq does not match kind " + kind_name(in.kind));
    for (int j = 0; j < ar; ++j)
      if (in.q[j] < 0 || in.q[j] >= n)
        throw Error(NT_ERR_INVALID_ARG, "gate " + std::to_string(g) + ": qubit out of range");
    if (ar == 2 && in.q[0] == in.q[1])
      throw Error(NT_ERR_INVALID_ARG, "gate " + std::to_string(g) + ": duplicate qubits");
    if ((in.kind == NT_U1Q || in.kind == NT_U2Q) && !in.matrix)
      throw Error(NT_ERR_INVALID_ARG, "gate " + std::to_string(g) + ": matrix required");
    for (int j = 0; j < kind_nparam(in.kind); ++j)
      if (!std::isfinite(in.param[j]))
        throw Error(NT_ERR_INVALID_ARG, "gate " + std::to_string(g) + ": non-finite angle");
    hg.kind = in.kind;
    hg.nq = ar;
    hg.q[0] = in.q[0];
    hg.q[1] = ar == 2 ? in.q[1] : -1;
    for (int j = 0; j < 3; ++j) hg.param[j] = in.param[j];
    gate_matrix(in.kind, in.param, in.matrix, hg.m);
    if (in.kind == NT_U1Q || in.kind == NT_U2Q) {
      int d = ar == 1 ? 2 : 4;
      for (int i = 0; i < d * d; ++i)
        if (!std::isfinite(hg.m[i].real()) || !std::isfinite(hg.m[i].imag()))
          throw Error(NT_ERR_INVALID_ARG, "gate " + std::to_string(g) + ": non-finite matrix");
      // Must be unitary to within 1e-9 (the fidelity criterion assumes it).
      for (int r = 0; r < d; ++r)
        for (int s = 0; s < d; ++s) {
          cd acc = 0;
          for (int k = 0; k < d; ++k) acc += std::conj(hg.m[k * d + r]) * hg.m[k * d + s];
          if (std::abs(acc - cd(r == s ? 1.0 : 0.0)) > 1e-9)
            throw Error(NT_ERR_INVALID_ARG, "gate " + std::to_string(g) + ": matrix is not unitary");
        }
    }
    c->S += ar;
  }
  c->serial = g_serial.fetch_add(1);
}

Circuit *load_circuit(int n, const nt_gate *gates, int64_t G) {
  Circuit *c = new Circuit();
  try {
    validate_and_fill(c, n, gates, G);
  } catch (...) {
    delete c;
    throw;
  }
  return c;
}

Circuit *load_circuit_text(const char *path) {
  if (!path) throw Error(NT_ERR_INVALID_ARG, "path is NULL");
  std::ifstream f(path);
  if (!f) throw Error(NT_ERR_INVALID_ARG, std::string("cannot open ") + path);
  int n = -1;
  std::vector<nt_gate> gates;
  std::vector<std::vector<double>> mats;
  std::string line;
  int64_t lineno = 0;
  while (std::getline(f, line)) {
    ++lineno;
    size_t p = line.find_first_not_of(" \t\r");
    if (p == std::string::npos || line[p] == '#') continue;
    std::istringstream ss(line);
    std::string tok;
    ss >> tok;
    if (tok == "qubits") {
      if (!(ss >> n)) throw Error(NT_ERR_INVALID_ARG, "line " + std::to_string(lineno) + ": bad qubits line");
      continue;
    }
    int kind = kind_from_name(tok);
    if (kind < 0) throw Error(NT_ERR_INVALID_ARG, "line " + std::to_string(lineno) + ": unknown gate " + tok);
    nt_gate g;
    std::memset(&g, 0, sizeof g);
    g.kind = (uint16_t)kind;
    g.nq = (uint8_t)kind_arity(kind);
    for (int j = 0; j < g.nq; ++j)
      if (!(ss >> g.q[j])) throw Error(NT_ERR_INVALID_ARG, "line " + std::to_string(lineno) + ": missing qubit");
    std::vector<double> rest;
    std::string v;
    while (ss >> v) {
      char *end = nullptr;
      double d = std::strtod(v.c_str(), &end);
      if (!end || *end) throw Error(NT_ERR_INVALID_ARG, "line " + std::to_string(lineno) + ": bad number " + v);
      rest.push_back(d);
    }
    if (kind == NT_U1Q || kind == NT_U2Q) {
      size_t want = kind == NT_U1Q ? 8 : 32;
      if (rest.size() != want) throw Error(NT_ERR_INVALID_ARG, "line " + std::to_string(lineno) + ": bad matrix size");
      mats.push_back(rest);
    } else {
      if ((int)rest.size() != kind_nparam(kind))
        throw Error(NT_ERR_INVALID_ARG, "line " + std::to_string(lineno) + ": wrong number of angles");
      for (size_t j = 0; j < rest.size(); ++j) g.param[j] = rest[j];
      mats.emplace_back();
    }
    gates.push_back(g);
  }
  if (n < 0) throw Error(NT_ERR_INVALID_ARG, "missing 'qubits' line");
  for (size_t i = 0; i < gates.size(); ++i)
    if (!mats[i].empty()) gates[i].matrix = mats[i].data();
  return load_circuit(n, gates.data(), (int64_t)gates.size());
}

// A matrix entry is treated as zero only when it is exactly zero, so the
// class decision never changes the arithmetic.
static bool is_zero(cd v) { return v.real() == 0.0 && v.imag() == 0.0; }

std::vector<HostOp> classify(const Circuit &c) {
  std::vector<HostOp> ops(c.gates.size());
  for (size_t g = 0; g < c.gates.size(); ++g) {
    const HostGate &hg = c.gates[g];
    HostOp &op = ops[g];
    op.gate = (int32_t)g;
    for (int i = 0; i < 16; ++i) op.m[i] = 0;
    if (hg.nq == 1) {
      op.qa = hg.q[0];
      op.qb = -1;
      if (is_zero(hg.m[1]) && is_zero(hg.m[2])) {
        op.cls = OPC_D1;
        op.m[0] = hg.m[0];
        op.m[1] = hg.m[3];
      } else {
        op.cls = OPC_G1;
        for (int i = 0; i < 4; ++i) op.m[i] = hg.m[i];
      }
      continue;
    }
    op.qa = hg.q[0];
    op.qb = hg.q[1];
    bool diag = true;
    for (int r = 0; r < 4; ++r)
      for (int s = 0; s < 4; ++s)
        if (r != s && !is_zero(hg.m[r * 4 + s])) diag = false;
    if (diag) {
      op.cls = OPC_D2;
      for (int i = 0; i < 4; ++i) op.m[i] = hg.m[i * 4 + i];
      continue;
    }
    if (hg.kind == NT_CNOT) {
      // controlled X: target = second listed qubit, control = first
      op.cls = OPC_C1;
      op.qa = hg.q[1];
      op.qb = hg.q[0];
      op.m[0] = 0; op.m[1] = 1; op.m[2] = 1; op.m[3] = 0;
      continue;
    }
    if (hg.kind == NT_SWAP) {
      op.cls = OPC_SW;
      continue;
    }
    op.cls = OPC_G2;
    for (int i = 0; i < 16; ++i) op.m[i] = hg.m[i];
  }
  return ops;
}

// Algorithmic flops per amplitude of one gate, from its own matrix (a
// complex multiply is 6 flops, a complex add 2):
//   a permutation whose entries are 1, -1, i or -i (X, Y, CNOT, SWAP): 0;
//   a diagonal: 6 for each entry other than 1, averaged over the amplitudes
//     (RZ and RZZ 6, Z, S and T 3, CZ and CP 1.5: only |11> changes);
//   any other one-qubit gate: 2 complex multiplies and 1 add per amplitude,
//     14; any other two-qubit gate: 4 multiplies and 3 adds, 30.
double gate_flops(const HostGate &g) {
  const int d = g.nq == 1 ? 2 : 4;
  bool diag = true, perm = true;
  int nonunit = 0;
  for (int r = 0; r < d; ++r) {
    int nz = 0;
    for (int s = 0; s < d; ++s) {
      const cd v = g.m[r * d + s];
      if (is_zero(v)) continue;
      ++nz;
      if (r != s) diag = false;
      const bool unit_phase = (v == cd(1, 0) || v == cd(-1, 0) || v == cd(0, 1) || v == cd(0, -1));
      if (!unit_phase) perm = false;
    }
    if (nz != 1) perm = false;
    if (!(g.m[r * d + r] == cd(1, 0))) ++nonunit;
  }
  if (diag) return 6.0 * nonunit / d;
  if (perm) return 0.0;
  return g.nq == 1 ? 14.0 : 30.0;
}

uint32_t HostOp::need_mask() const {
  switch (cls) {
    case OPC_G1: case OPC_C1: return 1u << qa;
    case OPC_G2: case OPC_G4: case OPC_SW: return (1u << qa) | (1u << qb);
    default: return 0u;
  }
}

Thresholds make_thresholds(double px, double py, double pz) {
  Thresholds t;
  auto thr = [](double x, bool *always) -> uint64_t {
    *always = false;
    if (!(x > 0)) return 0;
    if (x >= 1.0) { *always = true; return UINT64_MAX; }
    return (uint64_t)std::floor(std::ldexp(x, 64));
  };
  double sum = px + py + pz;
  bool a0, a1 = false, a2 = false;
  t.t_fire = thr(sum, &a0);
  if (sum > 0 && px == py && py == pz) {
    // uniform model: exactly one third each, whatever the rate (px / sum
    // rounds differently from rate to rate, and the type draws must be the
    // same at every rate for the fired sets to be nested with equal types)
    t.c_x = thr(1.0 / 3.0, &a1);
    t.c_xy = thr(2.0 / 3.0, &a2);
  } else if (sum > 0) {
    t.c_x = thr(px / sum, &a1);
    t.c_xy = thr((px + py) / sum, &a2);
  }
  t.always = (a0 ? 1u : 0u) | (a1 ? 2u : 0u) | (a2 ? 4u : 0u);
  return t;
}

}  // namespace nt
