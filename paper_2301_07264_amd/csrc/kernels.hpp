// Device data layouts shared by the host engine and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ntk {

// Interleaved complex amplitude.
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

// One gate of the plan, as the kernels read it (uniform per work-group).
//   cls  : dispatch code (OPK_* kind * 4 + register bit of the target)
//   qa,qb: qubits (C1: qa = target, qb = control)
//   rsel : register-segment ops: register-bit masks of qa (bits 0..3) and qb
//          (bits 4..7) in the op's segment, 0 for a non-register qubit;
//          G2: tile-local bit positions of qa (bits 0..3) and qb (bits 4..7)
//   m    : matrix data, (re, im) interleaved; G1/C1 2x2 row-major, D1 (d0,d1),
//          D2 (d0..d3) on local index b_qa + 2 b_qb, G2 4x4 row-major.
//   G4 (fused block, qa on the lower register bit): rsel = index of the
//          block's first matrix in the plan's aux table | (stages << 24);
//          the table holds the block's product, then one 4x4 per gate, each
//          as its 16 frame variants (x + 4 z) of 16 entries.
template <typename T>
struct DevOp {
  int32_t cls, qa, qb, rsel;
  T m[40];
  // padding to a power of two (256 bytes for complex64 tables, 512 for
  // complex128): the gate kernel addresses op o as base + (o << 8) with one
  // shift instead of a 64-bit multiply
  int32_t pad[sizeof(T) == 4 ? 20 : 44];
};
static_assert(sizeof(DevOp<float>) == 256 && sizeof(DevOp<double>) == 512, "op table stride");

// Op dispatch codes: kind * 4 + register bit (kinds with a register
// qubit) or kind * 4 (diagonal kinds without one).  G2 ops live in quad
// segments.
enum : int32_t {
  OPK_G1 = 0,   // general complex 2x2, m = 4 entries
  OPK_G1R = 1,  // real 2x2 (imaginary parts zero)
  OPK_G1X = 2,  // [[c, -i s], [-i s, c]]: m00 = c, m01 = -i s
  OPK_CX = 3,   // controlled X: qa target, qb control
  OPK_D1 = 4,   // diagonal (d0, d1) on qa, qa not a register qubit
  OPK_D2 = 5,   // diagonal (d0..d3) on local index b_qa + 2 b_qb, neither qubit in the registers
  OPK_G2 = 6,   // dense 4x4 (quad segment)
  OPK_D2A = 7,  // diagonal on two qubits, qa in register bit b, qb not
  OPK_D2B = 8,  // diagonal on two qubits, qb in register bit b, qa not
  OPK_D1R = 9,  // diagonal on one qubit, qa in register bit b
  // Diagonal on two qubits, both in the registers: code OPK_D2RR * 4 + k
  // for the register-bit pair D2RR_PAIRS[k] (lower bit first), k = 0..5.
  OPK_D2RR = 10,
  // Fused two-qubit block, dense 4x4 on register bits (0, 1) (code
  // OPK_G4 * 4, at even offsets of its segment) or (2, 3) (code
  // OPK_G4 * 4 + 1, at odd offsets).
  OPK_G4 = 12,
  OPK_NOP = 13,  // no operation (pads a segment so fused ops sit at their offset parity)
  // Fused run of diagonal gates: rsel = byte offset / 16 of its first record
  // (DfRec) in the aux table | (gates << 24).
  OPK_DF = 14,
  // SWAP of two register qubits: code OPK_SW * 4 + k, the pair
  // D2RR_PAIRS[k] of register bits (codes up to OPK_SW * 4 + 5)
  OPK_SW = 15,
  // Four RX-type one-qubit gates, one per register bit (complex64, R = 4):
  // m[2i] = c, m[2i + 1] = Im m01 of the gate on register bit i, rsel = the
  // four qubits (8 bits each, bit 0 first).  Code OPK_L4 * 4.
  OPK_L4 = 17,
};

// One gate of a fused diagonal run.  kind 0 (no qubit in the registers):
// p[b_a + 2 b_b] are the gate's phases by the bits of qubits sa, sb (a
// one-qubit gate has sa = sb and uses p[0], p[3]).  kind 1 (qubit rq on
// register bit rbit, the other qubit sa outside the registers, or none):
// p[b_a] is the phase with the register qubit's bit 0 and p[2 + b_a] the
// ratio of the phase with bit 1 to it.  kr = kind | rbit << 4.
template <typename T>
struct DfRec {
  uint32_t sa, sb, kr, rq;
  T p[8];
};

// The same run as phase angles in fixed point (turns x 2^32, sums mod 2^32
// are exact mod 2 pi), complex64 only, stored after the run's DfRecs.  Every
// gate's phase is split into a constant and terms "add q when bits sa and sb
// of the global index (XOR the frame's X) are both 1".  Group rho < 4 holds
// the gates whose register qubit sits on register bit rho, with a pair of
// angles for that bit's two values; group 4 the gates with no register
// qubit.  Valid only when no error falls inside the run (the frame is then
// constant over it).
struct DfFast {
  uint32_t hdr;        // bit 0: form present; bit 1 + rho: group rho used
  uint32_t nlane;      // per group (6 bits each): terms whose bits vary per lane
  uint32_t nuni;       // per group: terms whose bits are uniform over the work-group
  uint32_t rq;         // qubit on register bit rho (8 bits each)
  uint32_t c0[5], c1[4];
  uint32_t pad[3];
};
struct DfTerm {
  uint32_t sab;        // sa | sb << 8
  uint32_t q0, q1, pad;
};
static_assert(sizeof(DfFast) == 64 && sizeof(DfTerm) == 16, "fixed-point run layout");
constexpr int DF_MAX_TERMS = 63;


// Event words: (op << EV_OP_SHIFT) | (stage << EV_STAGE_SHIFT) | (qubit << 2) | pauli
// (qubit < 32).
// stage: for an error inside a fused block, the block gate it follows (the
// next gate of the block on its qubit comes after it); EV_STAGE_END for an
// error that acts after the whole op.
constexpr int EV_OP_SHIFT = 12;
constexpr int EV_STAGE_SHIFT = 7;
constexpr uint32_t EV_STAGE_END = 31u;
constexpr int D2RR_PAIRS[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

// One register segment: which local bits / global qubits the thread's
// register slots and thread-id bits map to.
// kind: SEG_KIND_REG (ops on amplitudes held in registers) or SEG_KIND_QUAD
// (one dense two-qubit op applied directly to the tile in LDS).
enum : int32_t { SEG_KIND_REG = 0, SEG_KIND_QUAD = 1 };

struct DevSeg {
  int32_t kind;
  int32_t op_begin, op_end;
  uint8_t rpos[4];   // local bit position of register bit b
  uint8_t rq[4];     // global qubit of register bit b
  uint8_t tpos[16];  // local bit position of thread-id bit i
  uint8_t tq[16];    // global qubit of thread-id bit i
  // Read by the gate kernel with scalar loads, precomputed on the host so a
  // segment change costs no scalar arithmetic: the swizzled LDS byte offset
  // term of register slot r (XOR of the swizzled offsets of the register
  // bits set in r), and tpos / tq widened to one dword each.
  uint32_t slot_off[16];
  uint32_t tpos_w[16];
  uint32_t tq_w[16];
};

// Tile layout of one pass.
struct DevPass {
  uint8_t locq[16];        // global qubit of tile-local bit i (ascending)
  uint8_t nlq[32];         // global qubit of tile-id bit i (ascending)
  uint8_t hq[4];           // locq[L - R + b]: qubit of the coalesced layout's register bit b
};
static_assert(sizeof(DevPass) == 52, "the pass table is read as 13 dwords");

// Components of a per-tile scoring partial: overlap re, overlap im, norm of
// the trajectory's state, criterion mass (probability of the target basis
// state, or of the heavy set).
constexpr int NPART = 4;

// Success criteria (Sec. II): fidelity against the error-free state, the
// probability of measuring one target basis state, the probability of the
// heavy set (basis states whose error-free probability exceeds the median).
enum : int32_t { CRIT_FIDELITY = 0, CRIT_TARGET = 1, CRIT_HEAVY = 2 };

enum : int32_t {
  PF_SCORE = 2,   // overlap with the reference + norm (FP64 partials); no store
  PF_STORE = 4,   // write the tile back (always unless PF_SCORE)
  PF_NORM = 8,    // norm partials only (reference run)
  PF_SKIP0 = 16,  // batched fidelity scoring: a trajectory without errors is
                  // the reference itself; its partials are (<R|R>, 0, <R|R>, 0)
};

// One circuit of a batched launch over many circuits that share a tile
// shape: its plan, reference state and heavy-set median.
template <typename T>
struct MultiItem {
  const DevOp<T> *ops;
  const DevSeg *segs;
  const DevPass *pass;
  const cx<T> *ref;
  const cx<T> *aux;        // fused-block matrices
  int32_t seg_begin, seg_end, op_begin, pad;
  double heavy_med;
  double nref;             // <R|R>
};

template <typename T>
struct PassArgs {
  const DevPass *pass;     // this pass's tile layout (device memory)
  cx<T> *state;            // B state vectors, state_stride amplitudes apart
  const cx<T> *ref;        // reference state (PF_SCORE)
  const DevOp<T> *ops;
  const cx<T> *aux;        // fused-block matrices (see DevOp)
  const DevSeg *segs;
  const uint32_t *events;  // per trajectory, in plan order: event words (EV_OP_SHIFT)
  const int32_t *ev_count;
  double *partials;        // [B][ntiles][NPART]
  // Pauli frame (x-mask, z-mask, phase) per trajectory, [B][4]: written at
  // the end of the pass, read at the start of the next one.  The frame is
  // not a function of the errors alone (a CNOT moves a frame Z from its
  // target to its control), so it is carried from pass to pass.
  uint32_t *frame_out;
  const uint32_t *frame_in;
  uint64_t state_stride;
  int32_t ev_stride;
  int32_t B;
  int32_t L;
  int32_t ntile_bits;
  int32_t seg_begin, seg_end, op_begin;
  int32_t flags;
  uint32_t init_index;
  // Trajectories may start late: start[b] is the first pass trajectory b
  // runs (NULL: all start at pass 0).  A trajectory starting at this pass
  // synthesizes the initial state (pass 0) or loads `ckpt`, the error-free
  // state before this pass; one that started earlier loads its own state.
  const int32_t *start;
  const cx<T> *ckpt;
  int32_t pass_index;
  // With `end`, trajectory b is scored at the end of pass end[b] against
  // `ref_here` (the error-free state after this pass) and skips later passes.
  const int32_t *end;
  const cx<T> *ref_here;
  int32_t crit;            // CRIT_*
  uint32_t target;         // CRIT_TARGET: basis state
  double heavy_med;        // CRIT_HEAVY: median of the error-free probabilities
  // Batched circuits (single-pass plans only): work-group b belongs to
  // circuit slot b / per_item, whose ops / segs / pass / ref / seg range /
  // median replace the fields above.  NULL: one circuit.
  const MultiItem<T> *multi;
  int32_t per_item;
};

// One circuit of a batched sampling launch.
struct SampleItem {
  uint64_t cid;
  const int32_t *order;
  const uint32_t *tag;
  int32_t S, pad;
};

struct SampleArgs {
  uint64_t seed, cid, t0;
  const uint64_t *tlist;   // trajectory ids (NULL: t0 + b)
  uint64_t t_fire, c_x, c_xy;
  uint32_t always;
  int32_t B, S, ev_stride;
  const int32_t *order;    // Philox site index per position
  const uint32_t *tag;     // event code without the Pauli bits, per position
  uint32_t *events;
  int32_t *ev_count;
  // Batched circuits: trajectory slot b is trajectory t0 + b % per_item of
  // circuit slot b / per_item, whose key, site count and tables replace
  // cid / S / order / tag.  NULL: one circuit.
  const SampleItem *multi;
  int32_t per_item;
};

// Size of the static scratch array of the allocation-free entry point (one
// per device).
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
// Device address of that array on `device`, which must be the current
// device; looked up once per device (hipGetSymbolAddress), then cached.
hipError_t scratch_address(int device, void **out);
// p[0..n) = 0 with a kernel (no memset node, so it also records in graphs).
hipError_t launch_zero_words(uint32_t *p, uint64_t n, hipStream_t s);

// Launch wrappers (kernels.hip).
hipError_t launch_sample(const SampleArgs &a, hipStream_t s);
// Fused ops a plan holds; the gate kernel has an instance per combination.
enum : int { FEAT_G4 = 1, FEAT_DF = 2, FEAT_L4 = 4 };
template <typename T>
hipError_t launch_pass(const PassArgs<T> &a, int R, int nthreads, int feat, hipStream_t s);
// nref: reference norm (end == NULL) or per-pass reference norms indexed by
// end[b].
hipError_t launch_finalize(const double *partials, int ntiles, int B, const double *nref, const int32_t *end,
                           int crit, double tau, double *fid, uint64_t *count, hipStream_t s);
// Batched circuits: entry b is trajectory j = b % per_item of circuit slot
// k = b / per_item, batch circuit item_map[k]: reference norm nref[k], value
// to fid[item_map[k] * out_stride + out_off + j], success counted in
// count[item_map[k]].
hipError_t launch_finalize_multi(const double *partials, int ntiles, int B, const double *nref, int per_item,
                                 const int32_t *item_map, int64_t out_stride, int64_t out_off, int crit, double tau,
                                 double *fid, uint64_t *count, hipStream_t s);
// Histogram (65536 bins) of bits [shift, shift+16) of the FP64 probability
// |a_k|^2 of every amplitude whose bits above shift+16 equal `prefix`.
template <typename T>
hipError_t launch_prob_hist(const cx<T> *a, uint64_t dim, int shift, uint64_t prefix, uint32_t *hist,
                            hipStream_t s);
// First and last event word of each trajectory (0 when it has none).
hipError_t launch_first_last(const uint32_t *events, const int32_t *ev_count, int ev_stride, int B,
                             uint32_t *out, hipStream_t s);
hipError_t launch_norm_final(const double *partials, int ntiles, double *nref, hipStream_t s);
template <typename T>
hipError_t launch_unframe(const cx<T> *st, cx<T> *out, uint64_t dim, const uint32_t *frame,
                          hipStream_t s);

}  // namespace ntk
