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
//   cls  : op class (G1 dense 2x2, D1 diagonal 1q, C1 controlled 2x2,
//          D2 diagonal 2q, G2 dense 4x4)
//   qa,qb: qubits (C1: qa = target, qb = control)
//   rsel : G1 / C1: register bit of qa in the segment that applies the op;
//          G2: tile-local bit positions of qa (bits 0..3) and qb (bits 4..7);
//          RSEL_CX marks a controlled X (the only C1 the host emits)
//   m    : matrix data, (re, im) interleaved; G1/C1 2x2 row-major, D1 (d0,d1),
//          D2 (d0..d3) on local index b_qa + 2 b_qb, G2 4x4 row-major
template <typename T>
struct DevOp {
  int32_t cls, qa, qb, rsel;
  T m[32];
};

enum : int32_t { OP_G1 = 0, OP_D1 = 1, OP_C1 = 2, OP_D2 = 3, OP_G2 = 4 };
// rsel flag: the C1 op's target matrix is exactly X (a CNOT).
enum : int32_t { RSEL_CX = 0x100 };

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
};

// Tile layout of one pass.
struct DevPass {
  uint8_t locq[16];        // global qubit of tile-local bit i (ascending)
  uint8_t nlq[32];         // global qubit of tile-id bit i (ascending)
};

enum : int32_t {
  PF_FIRST = 1,   // synthesize the initial basis state instead of loading
  PF_SCORE = 2,   // overlap with the reference + norm (FP64 partials); no store
  PF_STORE = 4,   // write the tile back (always unless PF_SCORE)
  PF_NORM = 8,    // norm partials only (reference run)
};

template <typename T>
struct PassArgs {
  const DevPass *pass;     // this pass's tile layout (device memory)
  cx<T> *state;            // B state vectors, state_stride amplitudes apart
  const cx<T> *ref;        // reference state (PF_SCORE)
  const DevOp<T> *ops;
  const DevSeg *segs;
  const uint32_t *events;  // per trajectory, sorted by op: (op << 8) | (qubit << 2) | pauli
  const int32_t *ev_count;
  double *partials;        // [B][ntiles][3]: overlap re, overlap im, norm
  uint32_t *frame_out;     // [B][4]: final Pauli frame x-mask, z-mask, phase
  uint64_t state_stride;
  int32_t ev_stride;
  int32_t B;
  int32_t L;
  int32_t ntile_bits;
  int32_t seg_begin, seg_end, op_begin;
  int32_t flags;
  uint32_t init_index;
};

struct SampleArgs {
  uint64_t seed, cid, t0;
  uint64_t t_fire, c_x, c_xy;
  uint32_t always;
  int32_t B, S, ev_stride;
  const int32_t *order;    // Philox site index per position
  const uint32_t *tag;     // event code without the Pauli bits, per position
  uint32_t *events;
  int32_t *ev_count;
};

// Launch wrappers (kernels.hip).
hipError_t launch_sample(const SampleArgs &a, hipStream_t s);
template <typename T>
hipError_t launch_pass(const PassArgs<T> &a, int R, int nthreads, hipStream_t s);
hipError_t launch_finalize(const double *partials, int ntiles, int B, const double *nref, double tau,
                           double *fid, uint64_t *count, hipStream_t s);
hipError_t launch_norm_final(const double *partials, int ntiles, double *nref, hipStream_t s);
template <typename T>
hipError_t launch_unframe(const cx<T> *st, cx<T> *out, uint64_t dim, const uint32_t *frame,
                          hipStream_t s);

}  // namespace ntk
