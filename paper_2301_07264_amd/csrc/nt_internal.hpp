// Internal declarations of libnisqtol (host side).
#pragma once

#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "nisqtol.h"

namespace nt {

using cd = std::complex<double>;

// Status-carrying exception used inside the library; converted to an
// nt_status at the C ABI.
struct Error : std::runtime_error {
  nt_status code;
  Error(nt_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// How a gate acts on the amplitude array.  Diagonal ops never need their
// qubits in a work-group's tile; dense ops need every listed qubit there; a
// controlled op needs only its target.
enum OpClass : int32_t {
  OPC_G1 = 0,  // dense 2x2 on qa
  OPC_D1 = 1,  // diagonal (d0, d1) on qa
  OPC_C1 = 2,  // 2x2 on target qa when control qb equals the control value
  OPC_D2 = 3,  // diagonal (d00, d10, d01, d11) on local index b_qa + 2 b_qb
  OPC_G2 = 4,  // dense 4x4 on local index b_qa + 2 b_qb
  // Fused two-qubit block: several gates on the qubits qa, qb (a two-qubit
  // gate with one-qubit gates before and after it on either qubit) applied
  // as one dense 4x4, m = their product on local index b_qa + 2 b_qb; both
  // qubits in the registers.  HostOp::sub lists the gates in order.
  OPC_G4 = 5,
  // No operation: keeps a fused block at an even position in its segment
  // (the gate kernel's op loop applies ops in pairs and compiles the block
  // body into the first of the two slots only).  No gate, no sites.
  OPC_NOP = 6,
  // Fused run of diagonal gates (HostOp::sub, in order), each with at most
  // one qubit in the segment's registers: one multiply per amplitude by the
  // product of their phases.
  OPC_DF = 7,
  // SWAP with both qubits in the registers: a register permutation, the
  // frame's bits on the two qubits trade places.
  OPC_SW = 8,
  // Four one-qubit gates of RX type, one on each register qubit
  // (HostOp::sub in register-bit order, m: their 2x2s), applied in one op
  // (complex64, four register qubits).
  OPC_L4 = 9,
};

struct HostGate {
  int kind = 0;
  int nq = 1;
  int q[2] = {0, -1};
  double param[3] = {0, 0, 0};
  cd m[16];          // full local matrix (2x2 or 4x4 row-major), FP64
};

// One gate as an op of the simulator: class, qubits and the class's matrix
// data (FP64; rounded once to FP32 for complex64 amplitudes).
struct HostOp {
  int32_t cls = OPC_G1;
  int32_t qa = 0, qb = -1;
  int32_t gate = 0;        // index in the circuit (a fused block: its two-qubit gate)
  std::vector<int32_t> sub;    // fused block: its gates in application order (empty otherwise)
  cd m[16];                // G1/C1: 4 entries; D1: 2; D2: 4; G2, G4: 16
  // qubits that must be in the work-group tile / in registers
  uint32_t need_mask() const;
  // the circuit gates the op applies, in order
  std::vector<int32_t> gates() const {
    if (!sub.empty()) return sub;
    if (gate >= 0) return {gate};
    return {};
  }
};

// Segment kinds: a register segment applies one-qubit, controlled-X and
// diagonal ops to amplitudes held in registers; a quad segment applies one
// dense two-qubit op directly to the tile in LDS.
enum SegKind : int { SEG_REG = 0, SEG_QUAD = 1 };

struct Segment {
  int kind = SEG_REG;
  int op_begin = 0, op_end = 0;       // into Plan::ops (application order)
  std::vector<int> reg_q;             // register qubits (global ids), size R
};

struct Pass {
  uint64_t local_mask = 0;            // qubits held in the tile
  int seg_begin = 0, seg_end = 0;
  int op_begin = 0, op_end = 0;
};

// A plan's op list holds, in application order, ops of one gate each and
// fused blocks (Plan::ops[o].sub).  The error site of a block's gate g on
// qubit q is tagged with g's stage in the block when a later gate of the
// block acts on q (an interior site: the error must act between the two
// gates), else with SITE_STAGE_END (the error commutes with the rest of the
// block and acts after it).  Sites of an op are listed interior first, in
// stage order, then the others.
constexpr int SITE_OP_SHIFT = 12;       // tag = (op << 12) | (stage << 7) | (qubit << 2)
constexpr int SITE_STAGE_SHIFT = 7;
constexpr uint32_t SITE_STAGE_END = 31u;
constexpr int MAX_BLOCK_GATES = 31;     // stages 0..30
struct Plan {
  int n = 0;
  int L = 0;          // tile qubits (<= n)
  int R = 0;          // register qubits per thread
  int cfix = 0;       // low qubits always in the tile (coalescing)
  std::vector<HostOp> ops;              // application order
  std::vector<Pass> passes;
  std::vector<Segment> segs;
  // sites in application order: Philox site index and kernel tag
  std::vector<int32_t> app_site;
  std::vector<uint32_t> app_tag;        // (op << 12) | (stage << 7) | (qubit << 2)
  std::vector<int> op_of_gate;          // gate -> application position
  int n_fused = 0;                      // fused blocks
  int n_diag = 0;                       // fused diagonal runs
  int n_layer = 0;                      // fused one-qubit layers (OPC_L4)
};

struct Circuit {
  int n = 0;
  std::vector<HostGate> gates;
  int64_t S = 0;
  uint64_t cid = 0;
  uint64_t serial = 0;                  // unique per loaded circuit
  int tile_override[3] = {0, 0, 0};     // per precision (NT_C64, NT_C128): tile qubits, 0 = automatic
  int fuse_width[3] = {0, 0, 0};        // per precision: nt_circuit_set_fusion's width (0 = automatic)
};

// circuit.cpp
void gate_matrix(int kind, const double *param, const double *umat, cd *m);
int kind_arity(int kind);
int kind_nparam(int kind);   // number of angles the kind takes
const char *kind_name(int kind);
int kind_from_name(const std::string &s);
Circuit *load_circuit(int n, const nt_gate *gates, int64_t G);
Circuit *load_circuit_text(const char *path);
std::vector<HostOp> classify(const Circuit &c);
double gate_flops(const HostGate &g);   // algorithmic flops per amplitude

// plan.cpp
// 4x4 matrix (local index b_qa + 2 b_qb) of gate g, which acts within {qa, qb}.
void embed_gate(const HostGate &g, int qa, int qb, cd *e);
// Fusion of a plan: two-qubit blocks, diagonal runs, one-qubit layers (bit
// set; layers at complex64 only).
enum : int { FUSE_BLOCKS = 1, FUSE_DIAG = 2, FUSE_LAYERS = 4 };
int fusion_mode(int width);   // nt_circuit_set_fusion width -> FUSE_* bits
Plan make_plan(const Circuit &c, int max_tile_qubits, int max_reg, int cfix, int fuse = FUSE_BLOCKS | FUSE_DIAG);
void plan_for_precision(const Circuit &c, int prec, int *L, int *R, int *cfix);
// The plan the library runs for a precision (tile shape chosen per circuit,
// or the circuit's override).
Plan choose_plan(const Circuit &c, int prec);
// Range of tile widths a precision allows for a circuit: [lo, hi].
void tile_range(const Circuit &c, int prec, int *lo, int *hi);

// sampling thresholds (host, FP64)
struct Thresholds {
  uint64_t t_fire = 0, c_x = 0, c_xy = 0;
  uint32_t always = 0;                  // bit0 fire, bit1 x, bit2 xy
};
Thresholds make_thresholds(double px, double py, double pz);

}  // namespace nt
