// HIP kernels for gfx950 (MI355X): Monte Carlo Pauli-error state-vector
// simulation (ArsoNISQ, arXiv 2301.07264, Sec. IV-B.2 and IV-C).
//
//   k_sample    error-site sampling: one Philox4x64-10 block per (site,
//               trajectory); a site fires iff word0 < thr(p); the Pauli comes
//               from word1 (Sec. IV-B.2).  One wavefront per trajectory
//               compacts its fired sites in plan order with a ballot.
//   k_pass      one HBM pass of the gate plan over a tile of 2^L amplitudes
//               per work-group: load (coalesced; or synthesize |0..0>, or
//               start from an error-free checkpoint) -> LDS -> register
//               segments / LDS quads -> store, or -> fused FP64 scoring.
//   k_finalize  fixed-order FP64 sums of the per-tile partials, fidelity and
//               success indicator per trajectory, integer success count
//               (Sec. IV-C: success probability = mean over the states).
//
// Errors (Sec. IV-B: an error gate appended after the gate) are carried as a
// per-trajectory Pauli frame F = i^c X^x Z^z: the stored vector s satisfies
// psi = F s.  A gate U is applied to s as F^dag U F, which is U with rows and
// columns permuted and signs flipped (exact in floating point), and an error
// P after the gate updates F <- P F.  This keeps every trajectory on the same
// pass plan and keeps diagonal gates diagonal.  The overlap is then
// <R|psi> = i^c sum_j conj(R[j ^ x]) (-1)^{popcount(z & j)} s[j].
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace ntk {

#define DEV __device__ __forceinline__

// Plan tables, error events and the previous pass's frames are never written
// while a pass kernel runs.  Reading them through the constant address space
// lets the compiler turn uniform loads into scalar loads, so op headers,
// matrix entries and frame bits stay in SGPRs and the frame conjugation of an
// op is scalar work instead of vector selects.
#define NT_CONST __attribute__((address_space(4)))
template <typename X>
DEV const NT_CONST X *cptr(const X *p) {
  return (const NT_CONST X *)p;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).

DEV void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                       uint64_t k1, uint64_t &w0, uint64_t &w1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  w0 = c0;
  w1 = c1;
}

__global__ void __launch_bounds__(256) k_sample(const SampleArgs a) {
  const int lane = threadIdx.x & 63;
  const int b = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (b >= a.B) return;                       // whole wavefront leaves together
  uint64_t t = a.tlist ? a.tlist[b] : a.t0 + (uint64_t)b;
  uint64_t cid = a.cid;
  int S = a.S;
  const int32_t *order = a.order;
  const uint32_t *tag = a.tag;
  if (a.multi) {
    const SampleItem &m = a.multi[b / a.per_item];
    t = a.t0 + (uint64_t)(b % a.per_item);
    cid = m.cid;
    S = m.S;
    order = m.order;
    tag = m.tag;
  }
  uint32_t *ev = a.events + (size_t)b * a.ev_stride;
  int base = 0;
  for (int k0 = 0; k0 < S; k0 += 64) {
    const int k = k0 + lane;
    bool fire = false;
    uint32_t code = 0;
    if (k < S) {
      uint64_t w0, w1;
      philox4x64_10((uint64_t)(uint32_t)order[k], t, 0, 0, a.seed, cid, w0, w1);
      fire = (a.always & 1u) || (w0 < a.t_fire);
      uint32_t pa = ((a.always & 2u) || w1 < a.c_x) ? 1u : (((a.always & 4u) || w1 < a.c_xy) ? 2u : 3u);
      code = tag[k] | pa;
    }
    const uint64_t mask = __ballot(fire);
    const int pos = base + (int)__popcll(mask & ((1ull << lane) - 1ull));
    if (fire) ev[pos] = code;
    base += (int)__popcll(mask);
  }
  if (lane == 0) a.ev_count[b] = base;
}

hipError_t launch_sample(const SampleArgs &a, hipStream_t s) {
  if (a.B <= 0) return hipSuccess;
  const int waves_per_block = 4;
  const int blocks = (a.B + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(k_sample, dim3(blocks), dim3(64 * waves_per_block), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Complex helpers.

template <typename T> DEV T fmat(T a, T b, T c);
template <> DEV float fmat<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> DEV double fmat<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// m0 * x + m1 * y
template <typename T>
DEV cx<T> mac2(cx<T> m0, cx<T> x, cx<T> m1, cx<T> y) {
  cx<T> r;
  r.x = m0.x * x.x;
  r.x = fmat(-m0.y, x.y, r.x);
  r.x = fmat(m1.x, y.x, r.x);
  r.x = fmat(-m1.y, y.y, r.x);
  r.y = m0.x * x.y;
  r.y = fmat(m0.y, x.x, r.y);
  r.y = fmat(m1.x, y.y, r.y);
  r.y = fmat(m1.y, y.x, r.y);
  return r;
}

template <typename T>
DEV cx<T> cmul(cx<T> m, cx<T> x) {
  cx<T> r;
  r.x = m.x * x.x;
  r.x = fmat(-m.y, x.y, r.x);
  r.y = m.x * x.y;
  r.y = fmat(m.y, x.x, r.y);
  return r;
}

template <typename T>
DEV cx<T> cneg(cx<T> v) {
  return cx<T>{-v.x, -v.y};
}

// Copy a uniform value into a VGPR.  On gfx950 a VALU instruction that reads
// an SGPR operand issues at most every 4 cycles per SIMD, while FP32
// arithmetic on VGPR operands alone can issue about twice as fast; a gate
// body's 64-128 FMAs all read the same few matrix entries, so one move per
// entry pays for itself many times over.
template <typename T>
DEV T vpin(T x) {
  asm volatile("" : "+v"(x));
  return x;
}
template <typename T>
DEV cx<T> vpin(cx<T> x) {
  return cx<T>{vpin(x.x), vpin(x.y)};
}

// Matrix entry i of an op (uniform address).
template <typename T>
DEV cx<T> ment(const NT_CONST DevOp<T> &op, uint32_t i) {
  return cx<T>{op.m[2 * i], op.m[2 * i + 1]};
}

// LDS address swizzle: the low SW bits of a tile index are XORed with every
// higher SW-bit chunk, so that 2^SW lanes whose indices differ in bits with
// distinct residues mod SW hit distinct banks (SW = 4 for 8-byte, 3 for
// 16-byte amplitudes).
template <typename T>
DEV uint32_t swz(uint32_t j) {
  constexpr int SW = sizeof(T) == 4 ? 4 : 3;
  constexpr uint32_t M = (1u << SW) - 1u;
  return j ^ ((j >> SW) & M) ^ ((j >> (2 * SW)) & M) ^ ((j >> (3 * SW)) & M) ^ ((j >> (4 * SW)) & M);
}

// A uniform table read as dwords with wide scalar loads (scalar loads have
// no byte form: a byte field read directly becomes a vector load whose
// latency every use then waits for), and byte i of it.
template <typename S, int NW>
DEV void cwords(const S *p, uint32_t (&w)[NW]) {
  static_assert(sizeof(S) == 4 * NW, "whole table");
  const NT_CONST uint32_t *q = reinterpret_cast<const NT_CONST uint32_t *>(cptr(p));
#pragma unroll
  for (int i = 0; i < NW; ++i) w[i] = q[i];
}
template <int NW>
DEV uint32_t wbyte(const uint32_t (&w)[NW], int i) {
  return (w[i >> 2] >> (8 * (i & 3))) & 0xffu;
}
constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

// out[k] = XOR of base[b] over the set bits b of k, one XOR per entry
// (each entry extends the one with k's lowest set bit cleared).  Used for the
// uniform address terms of a thread's 2^R register slots: the global index
// bits and the swizzled LDS offsets are both linear over GF(2) in k.
template <int N>
DEV void xor_span(const uint32_t (&base)[N], uint32_t (&out)[1 << N]) {
  out[0] = 0u;
#pragma unroll
  for (int k = 1; k < (1 << N); ++k) out[k] = out[k & (k - 1)] ^ base[__builtin_ctz((unsigned)k)];
}

// Pauli frame update F <- P_q F for F = i^c X^x Z^z (P = X: x ^= q;
// P = Z: c += 2 x_q, z ^= q; P = Y = iXZ: c += 1 + 2 x_q, x ^= q, z ^= q).
// Written without branches so the frame stays in scalar registers.
// The frame is the same for the whole work-group (one trajectory); the
// readfirstlane keeps it, and all conjugations derived from it, scalar.
DEV void frame_apply(uint32_t e, uint32_t &fx, uint32_t &fz, uint32_t &fc) {
  const uint32_t q = (e >> 2) & 31u, p = e & 3u, bit = 1u << q;
  const uint32_t xq = (fx >> q) & 1u;
  const uint32_t has_x = (p == 1u || p == 2u) ? 1u : 0u;
  const uint32_t has_z = (p >= 2u) ? 1u : 0u;
  const uint32_t dc = (p == 2u ? 1u : 0u) + has_z * 2u * xq;
  fx = __builtin_amdgcn_readfirstlane(fx ^ (has_x * bit));
  fz = __builtin_amdgcn_readfirstlane(fz ^ (has_z * bit));
  fc = __builtin_amdgcn_readfirstlane(fc + dc);
}

// ---------------------------------------------------------------------------
// Register-slot gate application.  v[r] holds the amplitude whose register
// bits are r; a dense op acts on the pairs (r, r | 1 << B).  Every body is
// specialized at compile time on B; the host picks the body through a flat
// dispatch code (OpCode), so that each op is one jump.

// general complex 2x2: 16 FMA per pair
template <int B, int R, typename T>
DEV void g1_apply(const cx<T> (&v)[1 << R], cx<T> (&w)[1 << R], cx<T> m00, cx<T> m01, cx<T> m10, cx<T> m11) {
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    if (r & (1 << B)) continue;
    const cx<T> x = v[r], y = v[r | (1 << B)];
    w[r] = mac2(m00, x, m01, y);
    w[r | (1 << B)] = mac2(m10, x, m11, y);
  }
}

// real 2x2 (H, RY, X, and their frame conjugates): 8 FMA per pair
template <int B, int R, typename T>
DEV void g1r_apply(const cx<T> (&v)[1 << R], cx<T> (&w)[1 << R], T m00, T m01, T m10, T m11) {
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    if (r & (1 << B)) continue;
    const cx<T> x = v[r], y = v[r | (1 << B)];
    w[r] = cx<T>{fmat(m01, y.x, m00 * x.x), fmat(m01, y.y, m00 * x.y)};
    w[r | (1 << B)] = cx<T>{fmat(m11, y.x, m10 * x.x), fmat(m11, y.y, m10 * x.y)};
  }
}

// [[c, i w], [i w, c]] with c, w real (RX(t): c = cos t/2, w = -sin t/2; a
// Z in the frame flips w, an X leaves it): 8 FMA per pair
template <int B, int R, typename T>
DEV void g1x_apply(const cx<T> (&v)[1 << R], cx<T> (&o)[1 << R], T c, T w) {
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    if (r & (1 << B)) continue;
    const cx<T> x = v[r], y = v[r | (1 << B)];
    o[r] = cx<T>{fmat(-w, y.y, c * x.x), fmat(w, y.x, c * x.y)};
    o[r | (1 << B)] = cx<T>{fmat(-w, x.y, c * y.x), fmat(w, x.x, c * y.y)};
  }
}

// Controlled X on register bit B, control value 1 (the caller moves the
// frame's effect on the control value into the frame): a swap of each
// register pair whose control bit is set.  With the control in the
// registers (register bit C) the swap pattern is known at compile time and
// the op is a plain register permutation; with the control outside them
// the swap is a per-lane select.
template <int B, int C, int R, typename T>
DEV void cx_perm(const cx<T> (&v)[1 << R], cx<T> (&w)[1 << R]) {
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) w[r] = ((r >> C) & 1) ? v[r ^ (1 << B)] : v[r];
}

template <int B, int R, typename T>
DEV void cx_apply(const cx<T> (&v)[1 << R], cx<T> (&w)[1 << R], bool take_lane, uint32_t cmask) {
  switch (cmask) {
    case 1u:
      if constexpr (B != 0) { cx_perm<B, 0, R>(v, w); return; }
      break;
    case 2u:
      if constexpr (B != 1 && R > 1) { cx_perm<B, 1, R>(v, w); return; }
      break;
    case 4u:
      if constexpr (B != 2 && R > 2) { cx_perm<B, 2, R>(v, w); return; }
      break;
    case 8u:
      if constexpr (B != 3 && R > 3) { cx_perm<B, 3, R>(v, w); return; }
      break;
    default:
      break;
  }
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    if (r & (1 << B)) continue;
    const cx<T> x = v[r], y = v[r | (1 << B)];
    w[r] = take_lane ? y : x;
    w[r | (1 << B)] = take_lane ? x : y;
  }
}

// Dense 4x4 on register bits LO and LO + 1 (local index b_LO + 2 b_LO+1):
// each slot group holds x0..x3 at r, r | 1 << LO, r | 2 << LO, r | 3 << LO;
// 16 FMA per output amplitude.  Group by group, so each group's inputs die
// as its outputs are formed (the two register banks together hold about one
// bank's worth next to the 16 matrix entries).
template <int LO, int R, typename T>
DEV void g4_apply(const cx<T> (&v)[1 << R], cx<T> (&w)[1 << R], const cx<T> (&m)[16]) {
  constexpr int A = 1 << LO, B = 2 << LO;
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    if (r & (A | B)) continue;
    const cx<T> x[4] = {v[r], v[r | A], v[r | B], v[r | A | B]};
    const int at[4] = {r, r | A, r | B, r | A | B};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      T re = m[4 * i].x * x[0].x, im = m[4 * i].x * x[0].y;
      re = fmat(-m[4 * i].y, x[0].y, re);
      im = fmat(m[4 * i].y, x[0].x, im);
#pragma unroll
      for (int j = 1; j < 4; ++j) {
        re = fmat(m[4 * i + j].x, x[j].x, re);
        re = fmat(-m[4 * i + j].y, x[j].y, re);
        im = fmat(m[4 * i + j].x, x[j].y, im);
        im = fmat(m[4 * i + j].y, x[j].x, im);
      }
      w[at[i]] = cx<T>{re, im};
    }
  }
}

// Header and the first four complex matrix entries of an op: what a
// register-segment op needs (a fused block reads its matrix from the aux
// table), read with scalar loads one op ahead (NM = 8 reals).
template <typename T, int NM = 8>
struct OpLite {
  int32_t code, qa, qb, rsel;
  T m[NM];
};

template <typename T, int NM>
DEV OpLite<T, NM> load_lite(const DevOp<T> *ops, int o) {
  OpLite<T, NM> h;
  if constexpr (sizeof(T) == 4) {
    // header and the entries: the first 4 + NM dwords of the descriptor
    struct Wn {
      uint32_t w[4 + NM];
    };
    const NT_CONST Wn &q = *reinterpret_cast<const NT_CONST Wn *>(
        reinterpret_cast<const NT_CONST char *>(cptr(ops)) + ((uint32_t)o << 8));
    uint32_t w[4 + NM];
#pragma unroll
    for (int i = 0; i < 4 + NM; ++i) w[i] = q.w[i];
    h.code = (int32_t)w[0];
    h.qa = (int32_t)w[1];
    h.qb = (int32_t)w[2];
    h.rsel = (int32_t)w[3];
#pragma unroll
    for (int i = 0; i < NM; ++i) h.m[i] = __builtin_bit_cast(T, w[4 + i]);
  } else {
    const NT_CONST DevOp<T> &op = cptr(ops)[o];
    h.code = op.cls;
    h.qa = op.qa;
    h.qb = op.qb;
    h.rsel = op.rsel;
#pragma unroll
    for (int i = 0; i < NM; ++i) h.m[i] = op.m[i];
  }
  return h;
}

// Descriptor of op o, loaded only after the descriptor `prev` has arrived.
// Scalar loads complete out of order, so a wait for any of them is a wait for
// all: tying the index to `prev` through an empty asm makes the wait for the
// op about to run come before this load is issued, which then has a whole op
// to arrive.  The opaque index also keeps loop strength reduction from
// splitting the load into one pointer per field.
template <typename T, int NM, int NP>
DEV OpLite<T, NM> load_lite_after(const DevOp<T> *ops, int o, const OpLite<T, NP> &prev) {
  asm volatile("" : "+s"(o) : "s"(prev.code));
  return load_lite<T, NM>(ops, o);
}

template <typename T, int NM>
DEV cx<T> lent(const OpLite<T, NM> &h, int i) {
  return cx<T>{h.m[2 * i], h.m[2 * i + 1]};
}

// Entries e[i] = entry i ^ xm of a 4-entry list, xm uniform in 0..3: two
// rounds of conditional swaps (bit 0 of xm swaps within pairs, bit 1 swaps
// the pairs), eight scalar selects instead of a select chain per entry.
template <typename T, int NM>
DEV void perm4(const OpLite<T, NM> &h, uint32_t xm, cx<T> &e0, cx<T> &e1, cx<T> &e2, cx<T> &e3) {
  const cx<T> a0 = lent(h, 0), a1 = lent(h, 1), a2 = lent(h, 2), a3 = lent(h, 3);
  const bool s0 = (xm & 1u) != 0u, s1 = (xm & 2u) != 0u;
  const cx<T> b0 = s0 ? a1 : a0, b1 = s0 ? a0 : a1, b2 = s0 ? a3 : a2, b3 = s0 ? a2 : a3;
  e0 = s1 ? b2 : b0;
  e1 = s1 ? b3 : b1;
  e2 = s1 ? b0 : b2;
  e3 = s1 ? b1 : b3;
}

// Diagonal whose phase is p1 on the slots with register bit B set and p0
// on the others (B known at compile time: no per-slot selects).
// cos + i sin of the angle t / 2^32 turns, single precision.  The nearest
// quarter turn k comes from the top bits (exact), the rest is an angle x in
// [-pi/4, pi/4), where the Taylor series of sin to x^9 and of cos to x^10
// are accurate to 2e-9; then e^{i(x + k pi/2)} = i^k e^{ix}.
DEV cx<float> phase_turns(uint32_t t) {
  const uint32_t k = (t + (1u << 29)) >> 30;
  const float x = (float)(int32_t)(t - (k << 30)) * 1.46291807926715968e-9f;   // 2 pi / 2^32
  const float x2 = x * x;
  const float s = x * (1.f + x2 * (-1.f / 6 + x2 * (1.f / 120 + x2 * (-1.f / 5040 + x2 * (1.f / 362880)))));
  const float c = 1.f + x2 * (-0.5f + x2 * (1.f / 24 + x2 * (-1.f / 720 + x2 * (1.f / 40320 + x2 * (-1.f / 3628800)))));
  const float re = (k & 1u) ? -s : c, im = (k & 1u) ? c : s;
  return (k & 2u) ? cx<float>{-re, -im} : cx<float>{re, im};
}

template <int B, int R, typename T>
DEV void diag_bit(const cx<T> (&v)[1 << R], cx<T> (&w)[1 << R], cx<T> p0, cx<T> p1) {
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) w[r] = cmul(((r >> B) & 1) ? p1 : p0, v[r]);
}

// Diagonal on one qubit outside the registers: one phase per lane.
template <int R, typename T>
DEV void d1_apply(const cx<T> (&v)[1 << R], cx<T> (&w)[1 << R], cx<T> d0, cx<T> d1, uint32_t lane) {
  const cx<T> d = lane ? d1 : d0;
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) w[r] = cmul(d, v[r]);
}

// Diagonal on two qubits outside the registers: one phase per lane, entries
// d[b_a + 2 b_b].
template <int R, typename T>
DEV void d2_apply(const cx<T> (&v)[1 << R], cx<T> (&w)[1 << R], cx<T> d0, cx<T> d1, cx<T> d2, cx<T> d3, uint32_t la,
                  uint32_t lb) {
  const cx<T> d = lb ? (la ? d3 : d2) : (la ? d1 : d0);
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) w[r] = cmul(d, v[r]);
}

// Diagonal on register bits LO < HI: slot r takes p[b_LO + 2 b_HI] (known at
// compile time, so no per-slot selects).
template <int LO, int HI, int R, typename T>
DEV void diag2(const cx<T> (&v)[1 << R], cx<T> (&w)[1 << R], cx<T> p0, cx<T> p1, cx<T> p2, cx<T> p3) {
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    const int i = ((r >> LO) & 1) | (((r >> HI) & 1) << 1);
    w[r] = cmul(i == 0 ? p0 : (i == 1 ? p1 : (i == 2 ? p2 : p3)), v[r]);
  }
}

// Register permutation of a SWAP on register bits A and B: slot r takes the
// slot with those two bits exchanged.
template <int A, int B, int R, typename T>
DEV void swap_perm(const cx<T> (&v)[1 << R], cx<T> (&w)[1 << R]) {
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    const int ba = (r >> A) & 1, bb = (r >> B) & 1;
    w[r] = v[ba == bb ? r : (r ^ (1 << A) ^ (1 << B))];
  }
}

// Frame after a SWAP of qubits a and b: the X and Z bits of the two qubits
// trade places (the phase is unchanged).
DEV void swap_frame(uint32_t a, uint32_t b, uint32_t &fx, uint32_t &fz) {
  const uint32_t m = (1u << a) | (1u << b);
  const uint32_t dx = ((fx >> a) ^ (fx >> b)) & 1u, dz = ((fz >> a) ^ (fz >> b)) & 1u;
  fx = __builtin_amdgcn_readfirstlane(fx ^ (dx ? m : 0u));
  fz = __builtin_amdgcn_readfirstlane(fz ^ (dz ? m : 0u));
}

// Frame update of a CNOT (control qc, target qt).  Conjugated by the frame,
// the CNOT becomes (+-Z_c)^{z_t} CX_cv: the frame's X on the control sets the
// control value cv, its Z on the target turns X into -X = (+-Z_c) X (sign +
// for cv = 1).  The register work is always CX_1, since CX_0 = X_t CX_1, and
// both factors around it move into the frame: F <- F (+-Z_c)^{z_t} X_t^{1-cv}.
// Working out the products: z_c ^= z_t, x_t ^= 1 - cv, and the phase is
// unchanged (the -1 of -Z_c is cancelled by commuting X_t past Z_t).
DEV void cx_frame(uint32_t zt, uint32_t qc, uint32_t qt, uint32_t cv, uint32_t &fx, uint32_t &fz) {
  fz = __builtin_amdgcn_readfirstlane(fz ^ (zt << qc));
  fx = __builtin_amdgcn_readfirstlane(fx ^ ((cv ^ 1u) << qt));
}

// A 2x2 conjugated by the frame's X^x Z^z on its qubit: rows and columns
// permuted by x, the off-diagonal entries negated by z.
template <typename T>
DEV void conj2(cx<T> m00, cx<T> m01, cx<T> m10, cx<T> m11, uint32_t x, uint32_t z, cx<T> &c00, cx<T> &c01,
               cx<T> &c10, cx<T> &c11) {
  if constexpr (sizeof(T) == 4) {
    // complex64 entries as 64-bit words: one scalar select per entry, one
    // XOR of both sign bits per negated entry
    auto u = [](cx<T> c) { return __builtin_bit_cast(uint64_t, c); };
    auto f = [](uint64_t q) { return __builtin_bit_cast(cx<T>, q); };
    const uint64_t sgn = z ? 0x8000000080000000ull : 0ull;
    c00 = f(x ? u(m11) : u(m00));
    c01 = f((x ? u(m10) : u(m01)) ^ sgn);
    c10 = f((x ? u(m01) : u(m10)) ^ sgn);
    c11 = f(x ? u(m00) : u(m11));
  } else {
    c00 = x ? m11 : m00;
    c01 = x ? m10 : m01;
    c10 = x ? m01 : m10;
    c11 = x ? m00 : m11;
    if (z) {
      c01 = cneg(c01);
      c10 = cneg(c10);
    }
  }
}

// Apply one register-segment op, conjugated by the current Pauli frame, to
// the register slots.  gb: the thread's global index with all register bits
// zero.  Index bit q of slot r is ((gb >> q) & 1) | (r & mask(q) != 0), where
// mask(q) is the register bit holding q (0 if none).  Conjugation by X^x Z^z of a 2x2
// M gives entries (i, j) = (-1)^{z(i+j)} M[i^x][j^x].
template <int R, int SLOT, int FEAT, typename T, int NM, typename TI, typename TS>
DEV void apply_reg_op(const OpLite<T, NM> &op, const cx<T> *aux, cx<T> (&v)[1 << R], cx<T> (&w)[1 << R],
                      uint32_t gb, uint32_t &fx, uint32_t &fz, uint32_t &fc, TI &&interior, TS &&take_stage) {
  const int code = op.code;
  const uint32_t qa = (uint32_t)op.qa;
  const uint32_t xa = (fx >> qa) & 1u, za = (fz >> qa) & 1u;
  // rsel: register-bit masks of qa (bits 0..3) and qb (bits 4..7) in this
  // op's segment (0 when the qubit is not a register qubit), from the host.
  const uint32_t bm = ((uint32_t)op.rsel >> 4) & 15u;
  const cx<T> m00 = lent(op, 0), m01 = lent(op, 1), m10 = lent(op, 2), m11 = lent(op, 3);
  // the frame-conjugated dense 2x2 on qa
  auto conj = [&](cx<T> &c00, cx<T> &c01, cx<T> &c10, cx<T> &c11) { conj2(m00, m01, m10, m11, xa, za, c00, c01, c10, c11); };
  // controlled X (control qb)
  const uint32_t qc = (uint32_t)op.qb;
  const uint32_t xc = (fx >> qc) & 1u;   // frame X on qb
  const uint32_t cv = 1u ^ xc;
  // Fused ops, then the dense one-qubit and controlled-X kinds, are tested
  // first, each followed by a branch on the register bits; everything else
  // goes through one switch on the full code.  The op loop applies ops in
  // pairs; the host puts blocks on register bits (0, 1) and diagonal runs at
  // even offsets of their segment (SLOT 1) and blocks on bits (2, 3) at odd
  // ones (SLOT 2), so each slot holds one block body (two bodies in one slot
  // need more registers than the kernel's budget).
  if constexpr (FEAT != 0) {
    if ((FEAT & FEAT_G4) && code == OPK_G4 * 4 + (SLOT - 1)) {
      // F^dag B F for the frame F = X^x Z^z at the block's start is the
      // table's variant x + 4 z of B (exact permutation and signs), and F
      // stays the frame after the block.  An error inside the block (a
      // later gate of the block acts on its qubit) splits it: its gates are
      // applied one by one, each conjugated by the frame as the errors
      // before it left it.
      const uint32_t rs = (uint32_t)op.rsel;
      const uint32_t first = rs & 0xffffffu, nst = rs >> 24;
      const bool split = interior();
      const uint32_t kend = split ? nst : 1u;
      for (uint32_t k = 0;;) {
        const uint32_t xm = ((fx >> qa) & 1u) | (((fx >> qc) & 1u) << 1);
        const uint32_t zm = ((fz >> qa) & 1u) | (((fz >> qc) & 1u) << 1);
        const uint32_t mi = ((first + (split ? 1u + k : 0u)) << 4) + xm + 4u * zm;
        const NT_CONST cx<T> *mp = cptr(aux) + ((size_t)mi << 4);
        cx<T> m[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) m[i] = vpin(cx<T>{mp[i].x, mp[i].y});
        if constexpr (SLOT == 1) g4_apply<0, R>(v, w, m);
        if constexpr (SLOT == 2 && R > 3) g4_apply<2, R>(v, w, m);
        if (++k >= kend) break;
        take_stage(k - 1u);
#pragma unroll
        for (int r = 0; r < (1 << R); ++r) v[r] = w[r];
      }
      return;
    }
    if constexpr ((FEAT & FEAT_L4) && SLOT == 1 && R == 4 && sizeof(T) == 4) {
      if (code == OPK_L4 * 4) {
        // four RX-type gates, one per register bit; a Z of the frame on a
        // gate's qubit flips its w, an X leaves it (the gates act on
        // different qubits, so the frame is the op's own for all four)
        const uint32_t qw = (uint32_t)op.rsel;
        auto wz = [&](int i) {
          const T w0 = op.m[2 * i + 1];
          return ((fz >> ((qw >> (8 * i)) & 255u)) & 1u) ? -w0 : w0;
        };
        cx<T> t[1 << R], u[1 << R];
        g1x_apply<0, R>(v, t, vpin(op.m[0]), vpin(wz(0)));
        g1x_apply<1, R>(t, u, vpin(op.m[2]), vpin(wz(1)));
        g1x_apply<2, R>(u, t, vpin(op.m[4]), vpin(wz(2)));
        g1x_apply<3, R>(t, w, vpin(op.m[6]), vpin(wz(3)));
        return;
      }
    }
    if ((FEAT & FEAT_DF) && SLOT == 1 && code == OPK_DF * 4) {
      // Run of diagonal gates: each gate's phase is taken under the frame as
      // the errors before it left it (F^dag D F = D(j ^ x)), per lane for
      // its qubits outside the registers and as a factor per register bit
      // for a register qubit; the product multiplies each amplitude once.
      // Gate records are read one ahead of the gate being evaluated.
      const uint32_t rs = (uint32_t)op.rsel;
      const uint32_t ng = rs >> 24;
      const DfRec<T> *recs = reinterpret_cast<const DfRec<T> *>(reinterpret_cast<const char *>(aux) +
                                                                 ((size_t)(rs & 0xffffffu) << 4));
      if constexpr (sizeof(T) == 4) {
        // With no error inside the run the frame is the same for all its
        // gates, and the run is one phase per amplitude: per group, a sum of
        // fixed-point angles over the terms whose bits are set (integer adds,
        // exact mod 2 pi), then one sine and cosine per group.
        const NT_CONST DfFast &f = *reinterpret_cast<const NT_CONST DfFast *>(cptr(recs) + ng);
        const uint32_t hdr = f.hdr;
        if ((hdr & 1u) && !interior()) {
          const uint32_t nl = f.nlane, nu = f.nuni, rqw = f.rq;
          const uint32_t gx = gb ^ fx;
          const uint32_t ux = __builtin_amdgcn_readfirstlane(gb) ^ fx;   // bits outside the tile
          const NT_CONST DfTerm *tm = reinterpret_cast<const NT_CONST DfTerm *>(&f + 1);
          uint32_t a0[5], a1[4];
#pragma unroll
          for (int g = 0; g < 5; ++g) {
            uint32_t s0 = 0, s1 = 0, u0 = f.c0[g], u1 = g < 4 ? f.c1[g] : 0u;
            const uint32_t cl = (nl >> (6 * g)) & 63u, cu = (nu >> (6 * g)) & 63u;
            for (uint32_t i = 0; i < cl; ++i, ++tm) {
              const uint32_t sab = tm->sab, q0 = tm->q0, q1 = tm->q1;
              const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int32_t)gx, sab & 255u, 1) &
                                 (uint32_t)__builtin_amdgcn_sbfe((int32_t)gx, sab >> 8, 1);
              s0 += m & q0;
              if (g < 4) s1 += m & q1;
            }
            for (uint32_t i = 0; i < cu; ++i, ++tm) {
              const uint32_t sab = tm->sab, q0 = tm->q0, q1 = tm->q1;
              const uint32_t m = 0u - ((ux >> (sab & 255u)) & (ux >> (sab >> 8)) & 1u);
              u0 += m & q0;
              if (g < 4) u1 += m & q1;
            }
            a0[g] = s0 + u0;
            if (g < 4) a1[g] = s1 + u1;
          }
          // slot with all register bits 0: bit rho takes the frame's X on
          // its qubit; the factor for a set register bit is the phase
          // difference of the two values, negated under that X
          uint32_t tb = a0[4];
          uint32_t td[4];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const bool xr = ((fx >> ((rqw >> (8 * g)) & 255u)) & 1u) != 0u;
            tb += xr ? a1[g] : a0[g];
            td[g] = xr ? a0[g] - a1[g] : a1[g] - a0[g];
          }
          auto phase = [](uint32_t t) { return phase_turns(t); };
          const cx<T> pb = phase(tb);
          const uint32_t used = (hdr >> 1) & 15u;
          if (used == 0u) {
#pragma unroll
            for (int r = 0; r < (1 << R); ++r) w[r] = cmul(pb, v[r]);
          } else if ((used & (used - 1u)) == 0u) {
            const int g = __builtin_ctz(used);
            const cx<T> p1 = cmul(phase(td[g]), pb);
            switch (g) {
              case 0: diag_bit<0, R>(v, w, pb, p1); break;
              case 1: if constexpr (R > 1) diag_bit<1, R>(v, w, pb, p1); break;
              case 2: if constexpr (R > 2) diag_bit<2, R>(v, w, pb, p1); break;
              default: if constexpr (R > 3) diag_bit<3, R>(v, w, pb, p1); break;
            }
          } else {
            cx<T> rt[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) rt[g] = ((used >> g) & 1u) ? phase(td[g]) : cx<T>{T(1), T(0)};
            cx<T> ph[1 << R];
#pragma unroll
            for (int r = 0; r < (1 << R); ++r) {
              ph[r] = r == 0 ? pb : cmul(rt[__builtin_ctz((unsigned)r)], ph[r & (r - 1)]);
              w[r] = cmul(ph[r], v[r]);
            }
          }
          return;
        }
      }
      cx<T> base{T(1), T(0)}, rt0{T(1), T(0)}, rt1{T(1), T(0)}, rt2{T(1), T(0)}, rt3{T(1), T(0)};
      auto load = [&](uint32_t k) {
        const NT_CONST DfRec<T> &q = cptr(recs)[k];
        DfRec<T> r;
        r.sa = q.sa;
        r.sb = q.sb;
        r.kr = q.kr;
        r.rq = q.rq;
#pragma unroll
        for (int i = 0; i < 8; ++i) r.p[i] = q.p[i];
        return r;
      };
      DfRec<T> cur = load(0u), nxt;
      for (uint32_t k = 0; k < ng; ++k) {
        uint32_t kn = k + 1u < ng ? k + 1u : k;
        asm volatile("" : "+s"(kn) : "s"(cur.kr));
        nxt = load(kn);
        const uint32_t gx = gb ^ fx;
        const uint32_t ia = (gx >> cur.sa) & 1u;
        const cx<T> e0{cur.p[0], cur.p[1]}, e1{cur.p[2], cur.p[3]}, e2{cur.p[4], cur.p[5]}, e3{cur.p[6], cur.p[7]};
        if ((cur.kr & 15u) == 0u) {
          const uint32_t ib = (gx >> cur.sb) & 1u;
          base = cmul(ib ? (ia ? e3 : e2) : (ia ? e1 : e0), base);
        } else {
          // the frame's X on the register qubit swaps the phases of its two
          // values: base * ratio for bit 0, 1 / ratio = conj(ratio) for bit 1
          const bool xr = ((fx >> cur.rq) & 1u) != 0u;
          const cx<T> q = ia ? e1 : e0, r = ia ? e3 : e2;
          base = cmul(xr ? cmul(r, q) : q, base);
          const cx<T> rr{r.x, xr ? -r.y : r.y};
          switch ((cur.kr >> 4) & 3u) {
            case 0: rt0 = cmul(rr, rt0); break;
            case 1: rt1 = cmul(rr, rt1); break;
            case 2: rt2 = cmul(rr, rt2); break;
            default: rt3 = cmul(rr, rt3); break;
          }
        }
        take_stage(k);
        cur = nxt;
      }
      // phase of slot r: base times the factors of its set register bits,
      // each slot's phase used as soon as it is formed (few live at once)
      const cx<T> rt[4] = {rt0, rt1, rt2, rt3};
      cx<T> ph[1 << R];
#pragma unroll
      for (int r = 0; r < (1 << R); ++r) {
        ph[r] = r == 0 ? base : cmul(rt[__builtin_ctz((unsigned)r)], ph[r & (r - 1)]);
        w[r] = cmul(ph[r], v[r]);
      }
      return;
    }
  }
  const int kind = code >> 2;
  if (kind == OPK_G1) {
    cx<T> c00, c01, c10, c11;
    conj(c00, c01, c10, c11);
    c00 = vpin(c00);
    c01 = vpin(c01);
    c10 = vpin(c10);
    c11 = vpin(c11);
    switch (code & 3) {
      case 0: g1_apply<0, R>(v, w, c00, c01, c10, c11); break;
      case 1: if constexpr (R > 1) g1_apply<1, R>(v, w, c00, c01, c10, c11); break;
      case 2: if constexpr (R > 2) g1_apply<2, R>(v, w, c00, c01, c10, c11); break;
      default: if constexpr (R > 3) g1_apply<3, R>(v, w, c00, c01, c10, c11); break;
    }
    return;
  }
  if (kind == OPK_CX) {
    const bool take = ((gb >> qc) & 1u) != 0u;
    switch (code & 3) {
      case 0: cx_apply<0, R>(v, w, take, bm); break;
      case 1: if constexpr (R > 1) cx_apply<1, R>(v, w, take, bm); break;
      case 2: if constexpr (R > 2) cx_apply<2, R>(v, w, take, bm); break;
      default: if constexpr (R > 3) cx_apply<3, R>(v, w, take, bm); break;
    }
    cx_frame(za, qc, qa, cv, fx, fz);
    return;
  }
  // Diagonal on two register qubits (qa on the lower register bit, the host
  // orders them): the phase of slot group (b_qa, b_qb) is D[(b_qa, b_qb) ^
  // (x_qa, x_qb)] under the frame.
  // SWAP of two register qubits: the slots trade along the bit pair, and
  // SWAP F SWAP^dag is F with the two qubits' frame bits exchanged
  const uint32_t swk = (uint32_t)(code - OPK_SW * 4);
  if (swk < 6u) {
    switch (swk) {
#define NT_SW(k)                                                                \
  case k:                                                                       \
    if constexpr (D2RR_PAIRS[k][1] < R) swap_perm<D2RR_PAIRS[k][0], D2RR_PAIRS[k][1], R>(v, w); \
    break;
      NT_SW(0)
      NT_SW(1)
      NT_SW(2)
      NT_SW(3)
      NT_SW(4)
      default:
        if constexpr (D2RR_PAIRS[5][1] < R) swap_perm<D2RR_PAIRS[5][0], D2RR_PAIRS[5][1], R>(v, w);
        break;
#undef NT_SW
    }
    swap_frame(qa, qc, fx, fz);
    return;
  }
  const uint32_t d2k = (uint32_t)(code - OPK_D2RR * 4);
  if (d2k < 6u) {
    cx<T> e0, e1, e2, e3;
    perm4(op, xa | (xc << 1), e0, e1, e2, e3);
    switch (d2k) {
#define NT_D2RR(k)                                                                               \
  case k:                                                                                        \
    if constexpr (D2RR_PAIRS[k][1] < R)                                                          \
      diag2<D2RR_PAIRS[k][0], D2RR_PAIRS[k][1], R>(v, w, vpin(e0), vpin(e1), vpin(e2), vpin(e3)); \
    break;
      NT_D2RR(0)
      NT_D2RR(1)
      NT_D2RR(2)
      NT_D2RR(3)
      NT_D2RR(4)
      default:
        if constexpr (D2RR_PAIRS[5][1] < R)
          diag2<D2RR_PAIRS[5][0], D2RR_PAIRS[5][1], R>(v, w, vpin(e0), vpin(e1), vpin(e2), vpin(e3));
        break;
#undef NT_D2RR
    }
    return;
  }
  switch (code) {
#define NT_G1(b)                                                                          \
  case OPK_G1R * 4 + b:                                                                   \
    if constexpr (b < R) {                                                                \
      cx<T> c00, c01, c10, c11;                                                           \
      conj(c00, c01, c10, c11);                                                           \
      g1r_apply<b, R>(v, w, vpin(c00.x), vpin(c01.x), vpin(c10.x), vpin(c11.x));          \
    }                                                                                     \
    break;                                                                                \
  case OPK_G1X * 4 + b:                                                                   \
    if constexpr (b < R) g1x_apply<b, R>(v, w, vpin(m00.x), vpin(za ? -m01.y : m01.y));   \
    break;
    NT_G1(0)
    NT_G1(1)
    NT_G1(2)
    NT_G1(3)
#undef NT_G1
    // Diagonal ops with one register qubit at bit b.  Under the frame the
    // phase of index g is D(g ^ x): the frame's X flips index bits, so it
    // swaps the two phases of a slot group instead of permuting entries.
#define NT_D(b)                                                                           \
  case OPK_D1R * 4 + b:                                                                   \
    if constexpr (b < R) diag_bit<b, R>(v, w, vpin(xa ? m01 : m00), vpin(xa ? m00 : m01));\
    break;                                                                                \
  case OPK_D2A * 4 + b:                                                                   \
    if constexpr (b < R) {                                                                \
      const uint32_t t = ((gb >> qc) & 1u) ^ xc;                                          \
      const cx<T> lo = t ? m10 : m00, hi = t ? m11 : m01;                                 \
      diag_bit<b, R>(v, w, xa ? hi : lo, xa ? lo : hi);                                   \
    }                                                                                     \
    break;                                                                                \
  case OPK_D2B * 4 + b:                                                                   \
    if constexpr (b < R) {                                                                \
      const uint32_t t = ((gb >> qa) & 1u) ^ xa;                                          \
      const uint32_t xb = xc;                                                             \
      const cx<T> lo = t ? m01 : m00, hi = t ? m11 : m10;                                 \
      diag_bit<b, R>(v, w, xb ? hi : lo, xb ? lo : hi);                                   \
    }                                                                                     \
    break;
    NT_D(0)
    NT_D(1)
    NT_D(2)
    NT_D(3)
#undef NT_D
    case OPK_D1 * 4: {
      d1_apply<R>(v, w, xa ? m01 : m00, xa ? m00 : m01, (gb >> qa) & 1u);
      break;
    }
    case OPK_D2 * 4: {
      cx<T> e0, e1, e2, e3;
      perm4(op, xa | (xc << 1), e0, e1, e2, e3);
      d2_apply<R>(v, w, e0, e1, e2, e3, (gb >> qa) & 1u, (gb >> qc) & 1u);
      break;
    }
    case OPK_NOP * 4: {
#pragma unroll
      for (int r = 0; r < (1 << R); ++r) w[r] = v[r];
      break;
    }
    default:
      // the host only emits the codes above (it rejects anything else when
      // it builds the plan); no identity copy here, which the compiler would
      // otherwise hoist into the shared branches of the dispatch tree
      __builtin_unreachable();
  }
}

// Dense two-qubit op applied directly to the tile in LDS (quad segment).
// rsel holds the tile-local bit positions of qa (bits 0..3) and qb (4..7).
template <typename T>
DEV void apply_quad_lds(const NT_CONST DevOp<T> &op, cx<T> *lds, int L, uint32_t fx, uint32_t fz) {
  const uint32_t qa = (uint32_t)op.qa, qb = (uint32_t)op.qb;
  const uint32_t pa = (uint32_t)op.rsel & 15u, pb = ((uint32_t)op.rsel >> 4) & 15u;
  const uint32_t xm = ((fx >> qa) & 1u) | (((fx >> qb) & 1u) << 1);
  const uint32_t zm = ((fz >> qa) & 1u) | (((fz >> qb) & 1u) << 1);
  cx<T> m[16];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cx<T> e = ment(op, ((uint32_t)i ^ xm) * 4u + ((uint32_t)j ^ xm));
      const uint32_t neg = (__popc(zm & (uint32_t)i) + __popc(zm & (uint32_t)j)) & 1u;
      m[4 * i + j] = neg ? cneg(e) : e;
    }
  const uint32_t lo = pa < pb ? pa : pb, hi = pa < pb ? pb : pa;
  const uint32_t nq = 1u << (L - 2);
  for (uint32_t qi = threadIdx.x; qi < nq; qi += blockDim.x) {
    uint32_t j = ((qi >> lo) << (lo + 1)) | (qi & ((1u << lo) - 1u));
    j = ((j >> hi) << (hi + 1)) | (j & ((1u << hi) - 1u));
    const uint32_t i0 = swz<T>(j), i1 = swz<T>(j | (1u << pa)), i2 = swz<T>(j | (1u << pb)),
                   i3 = swz<T>(j | (1u << pa) | (1u << pb));
    const cx<T> a0 = lds[i0], a1 = lds[i1], a2 = lds[i2], a3 = lds[i3];
    cx<T> o[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const cx<T> s = mac2(m[4 * i + 0], a0, m[4 * i + 1], a1);
      const cx<T> t = mac2(m[4 * i + 2], a2, m[4 * i + 3], a3);
      o[i] = cx<T>{s.x + t.x, s.y + t.y};
    }
    lds[i0] = o[0];
    lds[i1] = o[1];
    lds[i2] = o[2];
    lds[i3] = o[3];
  }
}

// Deterministic block reduction of NPART doubles into out[0..NPART).
DEV void block_reduce(double (&v)[NPART], double *out, unsigned char *smem) {
  const int NT = blockDim.x;
  const int tid = threadIdx.x;
  const int width = NT < 64 ? NT : 64;
  for (int off = width >> 1; off > 0; off >>= 1) {
#pragma unroll
    for (int c = 0; c < NPART; ++c) v[c] = __dadd_rn(v[c], __shfl_xor(v[c], off, 64));
  }
  __syncthreads();                       // tile reads done; reuse LDS
  double *red = reinterpret_cast<double *>(smem);
  const int nw = (NT + 63) >> 6;
  if ((tid & 63) == 0) {
#pragma unroll
    for (int c = 0; c < NPART; ++c) red[NPART * (tid >> 6) + c] = v[c];
  }
  __syncthreads();
  if (tid == 0) {
    double s[NPART] = {0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < nw; ++w)
#pragma unroll
      for (int c = 0; c < NPART; ++c) s[c] = __dadd_rn(s[c], red[NPART * w + c]);
#pragma unroll
    for (int c = 0; c < NPART; ++c) out[c] = s[c];
  }
}

// MAXT: largest work-group this instantiation serves; WPE: waves per SIMD
// it must fit (bounds the register budget so two work-groups share a CU);
// SLDS: the work-group is exactly MAXT threads and its tile is static LDS.
// FEAT: the fused ops the plan holds (FEAT_G4 blocks, FEAT_DF diagonal
// runs; their bodies are compiled only into these instances: each body in the
// op loop costs registers and instructions on every other op's path too)
template <typename T, int R, int MAXT, int WPE, bool SLDS, int FEAT>
__global__ void __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(WPE))) k_pass(const PassArgs<T> a) {
  constexpr int NS = 1 << R;
  // SLDS: the tile of exactly MAXT threads (MAXT * 2^R amplitudes) as a
  // static array, whose LDS address is known when the kernel is compiled, so
  // slot addresses need no base added; 0: the tile in dynamic LDS sized at
  // launch (kernels whose work-groups vary in size).
  constexpr size_t SLDS_BYTES = SLDS ? (size_t)MAXT * NS * sizeof(cx<T>) : 16;
  __shared__ __align__(16) unsigned char smem_static[SLDS_BYTES];
  extern __shared__ __align__(16) unsigned char smem_dyn[];
  unsigned char *const smem_raw = SLDS ? smem_static : smem_dyn;
  cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
  const uint32_t NT = blockDim.x;
  const uint32_t tid = threadIdx.x;
  const int b = (int)(blockIdx.x % (uint32_t)a.B);
  const uint32_t tile = blockIdx.x / (uint32_t)a.B;
  // trajectories already scored at an earlier pass have nothing to do
  if (a.end && a.pass_index > cptr(a.end)[b]) return;
  const bool score_here = a.end ? (cptr(a.end)[b] == a.pass_index) : ((a.flags & PF_SCORE) != 0);
  const cx<T> *refp = a.end ? a.ref_here : a.ref;
  const DevOp<T> *ops = a.ops;
  const cx<T> *aux = a.aux;
  const DevSeg *segs = a.segs;
  const DevPass *passp = a.pass;
  int seg_begin = a.seg_begin, seg_end = a.seg_end, op_begin = a.op_begin;
  double heavy_med = a.heavy_med;
  if (a.multi) {
    const NT_CONST MultiItem<T> &m = cptr(a.multi)[b / a.per_item];
    if ((a.flags & PF_SKIP0) && cptr(a.ev_count)[b] == 0) {
      // F = <R|R>^2 / (<R|R> <R|R>) = 1 exactly, as for the simulated state
      if (threadIdx.x == 0) {
        double *pt = a.partials + (size_t)b * NPART;
        pt[0] = m.nref;
        pt[1] = 0.0;
        pt[2] = m.nref;
        pt[3] = 0.0;
      }
      return;
    }
    ops = m.ops;
    aux = m.aux;
    segs = m.segs;
    passp = m.pass;
    refp = m.ref;
    seg_begin = m.seg_begin;
    seg_end = m.seg_end;
    op_begin = m.op_begin;
    heavy_med = m.heavy_med;
  }
  // The table pointers become values of their own: loaded from the kernel
  // arguments they belong to one wide scalar register group, which the
  // register allocator would otherwise spill and reload whole in the op loop.
  // (measured on the instruction listings: it removes the op loop's spills
  // of every variant but the complex128 one without fused blocks, which has
  // fewer spills without it)
  if constexpr (sizeof(T) == 4 || FEAT != 0) asm volatile("" : "+s"(ops), "+s"(segs));

  // Pass layout as dwords.  Thread-id bits at and above lt = L - R are zero
  // (NT = 2^lt <= MAXT), and so are tile-id bits at and above ntile_bits;
  // unused entries of the tables are zero, so the loops below run to
  // compile-time bounds (tile bits in groups of four, the rest skipped).
  constexpr int LTMAX = ilog2c(MAXT);
  uint32_t pw[13];
  cwords(passp, pw);
  uint32_t tilebase = 0;
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    if (4 * g >= a.ntile_bits) break;
#pragma unroll
    for (int u = 0; u < 4; ++u) tilebase |= ((tile >> (4 * g + u)) & 1u) << wbyte(pw, 16 + 4 * g + u);
  }
  cx<T> *st = a.state + (uint64_t)b * a.state_stride;
  uint32_t dlo = 0;
#pragma unroll
  for (int i = 0; i < LTMAX; ++i) dlo |= ((tid >> i) & 1u) << wbyte(pw, i);
  // Coalesced layout: slot k of thread tid holds tile index tid + k * NT.
  // Its global-index bits are tilebase | dlo | dk[k], dk[k] the XOR of
  // hbit[b] over the set bits b of k; the swizzle is linear over GF(2), so its
  // LDS byte offset is swz(tid) ^ lk[k] with lk[k] the XOR of swz(NT << b).
  // Both tables are uniform; they are rebuilt where needed instead of being
  // kept live across the segment loop.
  uint32_t hbit[R], lbit[R];
#pragma unroll
  for (int bb = 0; bb < R; ++bb) {
    hbit[bb] = 1u << wbyte(pw, 48 + bb);
    lbit[bb] = swz<T>(NT << bb) * (uint32_t)sizeof(cx<T>);
  }
  const uint32_t lds_tid = swz<T>(tid) * (uint32_t)sizeof(cx<T>);
  const cx<T> *sp = st + (tilebase | dlo);   // the dk bits are disjoint from tilebase | dlo

  // Load the tile (coalesced: thread-id bits are the low local bits).
  const int my_start = a.start ? cptr(a.start)[b] : 0;
  {
    uint32_t dk[NS], lk[NS];
    xor_span(hbit, dk);
    xor_span(lbit, lk);
    auto lds_k = [&](int k) -> cx<T> & { return *reinterpret_cast<cx<T> *>(smem_raw + (lds_tid ^ lk[k])); };
    if (my_start == a.pass_index && a.pass_index == 0) {
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const uint32_t g = tilebase | dlo | dk[k];
        lds_k(k) = cx<T>{g == a.init_index ? T(1) : T(0), T(0)};
      }
    } else {
      const cx<T> *src = (my_start == a.pass_index) ? a.ckpt + (tilebase | dlo) : sp;
      cx<T> v[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) v[k] = src[dk[k]];
#pragma unroll
      for (int k = 0; k < NS; ++k) lds_k(k) = v[k];
    }
  }
  __syncthreads();

  // Pauli frame at the start of this pass: carried from the previous pass,
  // or (first pass of the trajectory) the identity with every earlier error
  // applied.  next_op is the op index of the trajectory's next error event
  // (~0 when there is none).
  const NT_CONST uint32_t *ev = cptr(a.events + (size_t)b * a.ev_stride);
  const int ne = __builtin_amdgcn_readfirstlane(cptr(a.ev_count)[b]);
  const bool carried = a.frame_in != nullptr && my_start < a.pass_index;
  int ep = 0;
  uint32_t fx = 0, fz = 0, fc = 0;
  uint32_t next_e = 0, next_op = 0xffffffffu;
  while (ep < ne) {
    next_e = __builtin_amdgcn_readfirstlane(ev[ep]);
    if ((int)(next_e >> EV_OP_SHIFT) >= op_begin) break;
    if (!carried) frame_apply(next_e, fx, fz, fc);
    ++ep;
  }
  if (carried) {
    const NT_CONST uint32_t *fin = cptr(a.frame_in + 4 * b);
    fx = __builtin_amdgcn_readfirstlane(fin[0]);
    fz = __builtin_amdgcn_readfirstlane(fin[1]);
    fc = __builtin_amdgcn_readfirstlane(fin[2]);
  }
  if (ep < ne) next_op = next_e >> EV_OP_SHIFT;
  auto advance = [&]() {
    frame_apply(next_e, fx, fz, fc);
    ++ep;
    if (ep < ne) {
      next_e = __builtin_amdgcn_readfirstlane(ev[ep]);
      next_op = next_e >> EV_OP_SHIFT;
    } else {
      next_op = 0xffffffffu;
    }
  };
  auto take_events = [&](int o) {
    while (next_op == (uint32_t)o) advance();
  };
  // A fused block's interior errors come first among its events, in stage
  // order: whether op o has any, and those that follow its stage k.
  auto stage_of = [&]() { return (next_e >> EV_STAGE_SHIFT) & 31u; };
  auto has_interior = [&](int o) { return next_op == (uint32_t)o && stage_of() != EV_STAGE_END; };
  auto take_stage = [&](int o, uint32_t k) {
    while (next_op == (uint32_t)o && stage_of() == k) advance();
  };

  for (int s = seg_begin; s < seg_end; ++s) {
    // segment table: scalar loads of whole dwords only (header, the widened
    // thread-bit tables, the precomputed slot offsets)
    const NT_CONST DevSeg &sg = cptr(segs)[s];
    const int sg_kind = sg.kind, sg_op_begin = sg.op_begin, sg_op_end = sg.op_end;
    if (sg_kind == SEG_KIND_QUAD) {
      apply_quad_lds<T>(cptr(ops)[sg_op_begin], lds, a.L, fx, fz);
      take_events(sg_op_begin);
      __syncthreads();
      continue;
    }
    uint32_t jb = 0, gb = tilebase;
#pragma unroll
    for (int i = 0; i < LTMAX; ++i) {
      const uint32_t bit = (tid >> i) & 1u;
      jb |= bit << sg.tpos_w[i];
      gb |= bit << sg.tq_w[i];
    }
    // LDS byte offset of slot r: swz(jb) ^ slot_off[r] (the swizzle is linear
    // over GF(2); the register part is uniform and comes from the host).
    const uint32_t sjb = swz<T>(jb) * (uint32_t)sizeof(cx<T>);
    auto slot = [&](int r) -> cx<T> & { return *reinterpret_cast<cx<T> *>(smem_raw + (sjb ^ sg.slot_off[r])); };
    // Two register banks, ops alternating between them (v -> w -> v), so no
    // op has to copy its results back into the registers it read.
    cx<T> v[NS], w[NS];
#pragma unroll
    for (int r = 0; r < NS; ++r) v[r] = slot(r);
    // Descriptors are double-buffered: a_op holds the op at an even offset,
    // b_op the one after it; each is loaded while the other's op runs.  The
    // op table carries padding entries after its last op, so the loads one
    // past a segment's end stay inside it.
    int o = sg_op_begin;
    const int oe = sg_op_end;
    if (o < oe) {
      constexpr int NMA = 8;
      OpLite<T, NMA> a_op = load_lite<T, NMA>(ops, o);
      OpLite<T, 8> b_op;
      for (; o < oe; o += 2) {
        b_op = load_lite_after<T, 8>(ops, o + 1, a_op);
        apply_reg_op<R, 1, FEAT, T>(a_op, aux, v, w, gb, fx, fz, fc, [&] { return has_interior(o); },
                                          [&](uint32_t k) { take_stage(o, k); });
        take_events(o);
        if (o + 1 < oe) {
          a_op = load_lite_after<T, NMA>(ops, o + 2, b_op);
          apply_reg_op<R, 2, FEAT, T>(b_op, aux, w, v, gb, fx, fz, fc, [&] { return has_interior(o + 1); },
                                            [&](uint32_t k) { take_stage(o + 1, k); });
          take_events(o + 1);
        } else {
          // odd op count: the last result is in w
#pragma unroll
          for (int r = 0; r < NS; ++r) v[r] = w[r];
        }
      }
    }
    // the slot offsets are read again from the segment table (scalar cache)
    // instead of being kept in 2^R scalar registers across the op loop
    const DevSeg *sg_again = segs + s;
    asm volatile("" : "+s"(sg_again));
    const NT_CONST DevSeg &sg2 = *cptr(sg_again);
#pragma unroll
    for (int r = 0; r < NS; ++r) *reinterpret_cast<cx<T> *>(smem_raw + (sjb ^ sg2.slot_off[r])) = v[r];
    __syncthreads();
  }

  // The epilogue recomputes its addresses instead of keeping 2^R of them
  // live across the segment loop, and reads the register-bit words of the
  // pass table again rather than holding them in scalar registers.
  asm volatile("" : "+v"(dlo));
  {
    const DevPass *pp = passp;
    asm volatile("" : "+s"(pp));
    uint32_t pw2[13];
    cwords(pp, pw2);
#pragma unroll
    for (int bb = 0; bb < R; ++bb) {
      hbit[bb] = 1u << wbyte(pw2, 48 + bb);
      lbit[bb] = swz<T>(NT << bb) * (uint32_t)sizeof(cx<T>);
    }
  }
  uint32_t dk[NS], lk[NS];
  xor_span(hbit, dk);
  xor_span(lbit, lk);
  auto lds_k = [&](int k) -> cx<T> & { return *reinterpret_cast<cx<T> *>(smem_raw + (lds_tid ^ lk[k])); };
  const size_t ntiles = (size_t)1 << a.ntile_bits;
  if (score_here) {
    double ovr = 0.0, ovi = 0.0, nrm = 0.0, mass = 0.0;
    const uint32_t tgt = a.target ^ fx;   // psi[target] = +-s[target ^ x]
    const bool want_t = a.crit == CRIT_TARGET, want_h = a.crit == CRIT_HEAVY;
    // all reference loads in flight before the first use
    cx<T> rv[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) rv[k] = refp[(tilebase | dlo | dk[k]) ^ fx];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const uint32_t g = tilebase | dlo | dk[k];
      const cx<T> s = lds_k(k);
      const cx<T> r = rv[k];
      double sr = (double)s.x, si = (double)s.y;
      if (__popc(fz & g) & 1u) {
        sr = -sr;
        si = -si;
      }
      const double rr = (double)r.x, ri = (double)r.y;
      ovr = __dadd_rn(ovr, __fma_rn(ri, si, __dmul_rn(rr, sr)));
      ovi = __dadd_rn(ovi, __fma_rn(-ri, sr, __dmul_rn(rr, si)));
      const double ps = __fma_rn(si, si, __dmul_rn(sr, sr));
      nrm = __dadd_rn(nrm, ps);
      // heavy iff the error-free probability of index g ^ x exceeds the median
      const bool in = want_t ? (g == tgt) : (want_h && __fma_rn(ri, ri, __dmul_rn(rr, rr)) > heavy_med);
      mass = __dadd_rn(mass, in ? ps : 0.0);
    }
    double part[NPART] = {ovr, ovi, nrm, mass};
    block_reduce(part, a.partials + ((size_t)b * ntiles + tile) * NPART, smem_raw);
  } else {
    double nrm = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const uint32_t g = tilebase | dlo | dk[k];
      const cx<T> s = lds_k(k);
      st[g] = s;
      const double sr = (double)s.x, si = (double)s.y;
      nrm = __dadd_rn(nrm, __fma_rn(si, si, __dmul_rn(sr, sr)));
    }
    if (a.flags & PF_NORM) {
      double part[NPART] = {nrm, 0.0, nrm, 0.0};
      block_reduce(part, a.partials + ((size_t)b * ntiles + tile) * NPART, smem_raw);
    }
  }
  if (a.frame_out && tile == 0 && tid == 0) {
    a.frame_out[4 * b + 0] = fx;
    a.frame_out[4 * b + 1] = fz;
    a.frame_out[4 * b + 2] = fc & 3u;
  }
}

template <typename T, int FEAT>
static hipError_t launch_pass_k(const PassArgs<T> &a, int R, int nthreads, hipStream_t s) {
  const size_t ntiles = (size_t)1 << a.ntile_bits;
  const size_t blocks = ntiles * (size_t)a.B;
  size_t lds = ((size_t)1 << a.L) * sizeof(cx<T>);
  if (lds < 16 * NPART * sizeof(double)) lds = 16 * NPART * sizeof(double);
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
  // R = 4 work-groups are 2^(L-4) threads: 512 or 256 for complex64
  // (L = 13 or 12), 256 for complex128 (L = 12).  The two complex64 sizes
  // have kernels with the tile in static LDS (measured faster); everything
  // else uses dynamic LDS (for complex128 the static form measured slower).
  constexpr int MAXT4 = sizeof(T) == 4 ? 512 : 256;
  constexpr int WPE4 = sizeof(T) == 4 ? 4 : 2;
  if (nthreads > (R == 4 ? MAXT4 : 1024)) return hipErrorInvalidValue;
  const dim3 grid((uint32_t)blocks), blk(nthreads);
  switch (R) {
    case 1: hipLaunchKernelGGL((k_pass<T, 1, 1024, 1, false, FEAT>), grid, blk, lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_pass<T, 2, 1024, 1, false, FEAT>), grid, blk, lds, s, a); break;
    case 3: hipLaunchKernelGGL((k_pass<T, 3, 1024, 1, false, FEAT>), grid, blk, lds, s, a); break;
    case 4:
      if constexpr (sizeof(T) == 4) {
        if (nthreads == 512 && a.L == 13) {
          hipLaunchKernelGGL((k_pass<T, 4, 512, WPE4, true, FEAT>), grid, blk, 0, s, a);
          break;
        }
        if (nthreads == 256 && a.L == 12) {
          hipLaunchKernelGGL((k_pass<T, 4, 256, WPE4, true, FEAT>), grid, blk, 0, s, a);
          break;
        }
      }
      hipLaunchKernelGGL((k_pass<T, 4, MAXT4, WPE4, false, FEAT>), grid, blk, lds, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pass(const PassArgs<T> &a, int R, int nthreads, int feat, hipStream_t s) {
  // the tables and buffers every launch reads (per-circuit tables come with
  // the batch items instead), the fused-op table when the instance reads it,
  // and what the scoring epilogue and the partials need
  if (!a.multi && (!a.ops || !a.segs || !a.pass)) return hipErrorInvalidValue;
  if (!a.multi && feat != 0 && !a.aux) return hipErrorInvalidValue;
  if (!a.events || !a.ev_count) return hipErrorInvalidValue;
  if ((a.flags & PF_SCORE) && !a.multi && !(a.end ? a.ref_here : a.ref)) return hipErrorInvalidValue;
  if ((a.flags & (PF_SCORE | PF_NORM)) && !a.partials) return hipErrorInvalidValue;
  if (a.end && !a.ref_here) return hipErrorInvalidValue;
  switch (feat) {
    case 0: return launch_pass_k<T, 0>(a, R, nthreads, s);
    case FEAT_G4: return launch_pass_k<T, FEAT_G4>(a, R, nthreads, s);
    case FEAT_DF: return launch_pass_k<T, FEAT_DF>(a, R, nthreads, s);
    case FEAT_G4 | FEAT_DF: return launch_pass_k<T, FEAT_G4 | FEAT_DF>(a, R, nthreads, s);
    default: break;
  }
  // one-qubit layers: complex64 plans only
  if constexpr (sizeof(T) == 4) {
    switch (feat) {
      case FEAT_L4: return launch_pass_k<T, FEAT_L4>(a, R, nthreads, s);
      case FEAT_L4 | FEAT_G4: return launch_pass_k<T, FEAT_L4 | FEAT_G4>(a, R, nthreads, s);
      case FEAT_L4 | FEAT_DF: return launch_pass_k<T, FEAT_L4 | FEAT_DF>(a, R, nthreads, s);
      case FEAT_L4 | FEAT_G4 | FEAT_DF: return launch_pass_k<T, FEAT_L4 | FEAT_G4 | FEAT_DF>(a, R, nthreads, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_pass<float>(const PassArgs<float> &, int, int, int, hipStream_t);
template hipError_t launch_pass<double>(const PassArgs<double> &, int, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Fixed-order FP64 sum over tiles of component `comp` of the partials of
// trajectory b (block-wide; every thread returns the same value in tid 0).
DEV double sum_partials(const double *p, int ntiles, int comp, double *red) {
  const int tid = threadIdx.x, NT = blockDim.x;
  double acc = 0.0;
  for (int t = tid; t < ntiles; t += NT) acc = __dadd_rn(acc, p[(size_t)t * NPART + comp]);
  for (int off = 32; off > 0; off >>= 1) acc = __dadd_rn(acc, __shfl_xor(acc, off, 64));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  double s = 0.0;
  if (tid == 0)
    for (int w = 0; w < (NT >> 6); ++w) s = __dadd_rn(s, red[w]);
  return s;
}

// Entry b of a batched launch (per_item > 0) is trajectory b % per_item of
// circuit slot b / per_item.
__global__ void __launch_bounds__(256) k_finalize(const double *partials, int ntiles, const double *nref,
                                                  const int32_t *end, int per_item, const int32_t *item_map,
                                                  int64_t out_stride, int64_t out_off, int crit, double tau,
                                                  double *fid, uint64_t *count) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  const double *p = partials + (size_t)b * ntiles * NPART;
  const double ovr = sum_partials(p, ntiles, 0, red);
  const double ovi = sum_partials(p, ntiles, 1, red);
  const double nrm = sum_partials(p, ntiles, 2, red);
  const double mass = sum_partials(p, ntiles, 3, red);
  if (threadIdx.x == 0) {
    int slot = 0;
    int64_t out = b;
    uint64_t *cnt = count;
    if (per_item > 0) {
      slot = b / per_item;
      const int64_t ci = item_map[slot];
      out = ci * out_stride + out_off + (b % per_item);
      cnt = count + ci;
    }
    double v;
    if (crit == CRIT_FIDELITY) {
      const double num = __fma_rn(ovi, ovi, __dmul_rn(ovr, ovr));
      const double nr = per_item > 0 ? nref[slot] : (end ? nref[end[b]] : nref[0]);
      v = __ddiv_rn(num, __dmul_rn(nr, nrm));
    } else {
      v = __ddiv_rn(mass, nrm);
    }
    fid[out] = v;
    if (v >= tau) atomicAdd((unsigned long long *)cnt, 1ull);
  }
}

hipError_t launch_finalize(const double *partials, int ntiles, int B, const double *nref, const int32_t *end,
                           int crit, double tau, double *fid, uint64_t *count, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  // every buffer the kernel reads or writes must exist (end may be NULL)
  if (!partials || !nref || !fid || !count || ntiles <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finalize, dim3(B), dim3(256), 0, s, partials, ntiles, nref, end, 0, (const int32_t *)nullptr,
                     (int64_t)0, (int64_t)0, crit, tau, fid, count);
  return hipGetLastError();
}

hipError_t launch_finalize_multi(const double *partials, int ntiles, int B, const double *nref, int per_item,
                                 const int32_t *item_map, int64_t out_stride, int64_t out_off, int crit, double tau,
                                 double *fid, uint64_t *count, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (per_item <= 0 || !partials || !nref || !item_map || !fid || !count || ntiles <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finalize, dim3(B), dim3(256), 0, s, partials, ntiles, nref, (const int32_t *)nullptr,
                     per_item, item_map, out_stride, out_off, crit, tau, fid, count);
  return hipGetLastError();
}

// Radix-select step for the median of the error-free probabilities: the
// probabilities are non-negative doubles, whose bit patterns order like the
// values.  Integer atomics only, so the counts are exact.
template <typename T>
__global__ void __launch_bounds__(256) k_prob_hist(const cx<T> *a, uint64_t dim, int shift, uint64_t prefix,
                                                   uint32_t *hist) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < dim; k += stride) {
    const double re = (double)a[k].x, im = (double)a[k].y;
    const uint64_t bits = (uint64_t)__double_as_longlong(__fma_rn(im, im, __dmul_rn(re, re)));
    const uint64_t hi = (shift + 16 >= 64) ? 0 : (bits >> (shift + 16));
    if (hi == prefix) atomicAdd(&hist[(bits >> shift) & 0xffffu], 1u);
  }
}

template <typename T>
hipError_t launch_prob_hist(const cx<T> *a, uint64_t dim, int shift, uint64_t prefix, uint32_t *hist,
                            hipStream_t s) {
  uint64_t blocks = (dim + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((k_prob_hist<T>), dim3((uint32_t)blocks), dim3(256), 0, s, a, dim, shift, prefix, hist);
  return hipGetLastError();
}

template hipError_t launch_prob_hist<float>(const cx<float> *, uint64_t, int, uint64_t, uint32_t *, hipStream_t);
template hipError_t launch_prob_hist<double>(const cx<double> *, uint64_t, int, uint64_t, uint32_t *, hipStream_t);

__global__ void __launch_bounds__(256) k_first_last(const uint32_t *events, const int32_t *ev_count, int ev_stride,
                                                    int B, uint32_t *out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int n = ev_count[b];
  const uint32_t *e = events + (size_t)b * ev_stride;
  out[2 * b] = n > 0 ? e[0] : 0u;
  out[2 * b + 1] = n > 0 ? e[n - 1] : 0u;
}

hipError_t launch_first_last(const uint32_t *events, const int32_t *ev_count, int ev_stride, int B, uint32_t *out,
                             hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_first_last, dim3((B + 255) / 256), dim3(256), 0, s, events, ev_count, ev_stride, B, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_norm_final(const double *partials, int ntiles, double *nref) {
  __shared__ double red[4];
  const double nrm = sum_partials(partials, ntiles, 2, red);
  if (threadIdx.x == 0) nref[0] = nrm;
}

hipError_t launch_norm_final(const double *partials, int ntiles, double *nref, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, s, partials, ntiles, nref);
  return hipGetLastError();
}

// psi[k] = i^c (-1)^{popcount(z & (k ^ x))} s[k ^ x]
template <typename T>
__global__ void __launch_bounds__(256) k_unframe(const cx<T> *st, cx<T> *out, uint64_t dim,
                                                 const uint32_t *frame) {
  const uint32_t x = frame[0], z = frame[1], c = frame[2] & 3u;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < dim; k += stride) {
    const uint64_t src = k ^ (uint64_t)x;
    cx<T> v = st[src];
    if (__popc(z & (uint32_t)src) & 1u) v = cneg(v);
    cx<T> o = v;
    if (c == 1u) o = cx<T>{-v.y, v.x};
    else if (c == 2u) o = cneg(v);
    else if (c == 3u) o = cx<T>{v.y, -v.x};
    out[k] = o;
  }
}

template <typename T>
hipError_t launch_unframe(const cx<T> *st, cx<T> *out, uint64_t dim, const uint32_t *frame, hipStream_t s) {
  // grid-stride: a dispatch holds fewer than 2^32 work-items, and 2^32
  // amplitudes (32 qubits) would reach that
  const uint64_t blocks = std::min<uint64_t>((dim + 255) / 256, (uint64_t)1 << 16);
  hipLaunchKernelGGL((k_unframe<T>), dim3((uint32_t)blocks), dim3(256), 0, s, st, out, dim, frame);
  return hipGetLastError();
}

template hipError_t launch_unframe<float>(const cx<float> *, cx<float> *, uint64_t, const uint32_t *, hipStream_t);
template hipError_t launch_unframe<double>(const cx<double> *, cx<double> *, uint64_t, const uint32_t *,
                                           hipStream_t);

// ---------------------------------------------------------------------------
// Scratch memory of the allocation-free entry point: one static array per
// device, held until the process ends.  Host code never uses the array's
// name as an address; it uses the device address looked up once per device
// (scratch_address), with that device current.

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

hipError_t scratch_address(int device, void **out) {
  static std::mutex mu;
  static void *addr[64] = {};
  static bool have[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!have[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = ptr;
    have[device] = true;
  }
  *out = addr[device];
  return hipSuccess;
}

__global__ void __launch_bounds__(256) k_zero_words(uint32_t *p, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t launch_zero_words(uint32_t *p, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n > ((uint64_t)1 << 30)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zero_words, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace ntk
