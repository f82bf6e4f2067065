// HIP kernels for gfx950 (MI355X): Monte Carlo Pauli-error state-vector
// simulation (ArsoNISQ, arXiv 2301.07264, Sec. IV-B.2 and IV-C).
//
//   k_sample    error-site sampling: one Philox4x64-10 block per (site,
//               trajectory); a site fires iff word0 < thr(p); the Pauli comes
//               from word1 (Sec. IV-B.2).  One wavefront per trajectory
//               compacts its fired sites in plan order with a ballot.
//   k_pass      one HBM pass of the gate plan over a tile of 2^L amplitudes
//               per work-group: load (coalesced) -> LDS -> register segments
//               -> store, or -> fused FP64 scoring against the reference.
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

#include "kernels.hpp"

namespace ntk {

#define DEV __device__ __forceinline__

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
  const uint64_t t = a.t0 + (uint64_t)b;
  uint32_t *ev = a.events + (size_t)b * a.ev_stride;
  int base = 0;
  for (int k0 = 0; k0 < a.S; k0 += 64) {
    const int k = k0 + lane;
    bool fire = false;
    uint32_t code = 0;
    if (k < a.S) {
      uint64_t w0, w1;
      philox4x64_10((uint64_t)(uint32_t)a.order[k], t, 0, 0, a.seed, a.cid, w0, w1);
      fire = (a.always & 1u) || (w0 < a.t_fire);
      uint32_t pa = ((a.always & 2u) || w1 < a.c_x) ? 1u : (((a.always & 4u) || w1 < a.c_xy) ? 2u : 3u);
      code = a.tag[k] | pa;
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

// Matrix entry i of an op (uniform address).
template <typename T>
DEV cx<T> ment(const DevOp<T> &op, uint32_t i) {
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

// Pauli frame update F <- P_q F for F = i^c X^x Z^z (P = X: x ^= q;
// P = Z: c += 2 x_q, z ^= q; P = Y = iXZ: c += 1 + 2 x_q, x ^= q, z ^= q).
// Written without branches so the frame stays in scalar registers.
DEV void frame_apply(uint32_t e, uint32_t &fx, uint32_t &fz, uint32_t &fc) {
  const uint32_t q = (e >> 2) & 31u, p = e & 3u, bit = 1u << q;
  const uint32_t xq = (fx >> q) & 1u;
  const uint32_t has_x = (p == 1u || p == 2u) ? 1u : 0u;
  const uint32_t has_z = (p >= 2u) ? 1u : 0u;
  const uint32_t dc = (p == 2u ? 1u : 0u) + has_z * 2u * xq;
  fx = fx ^ (has_x * bit);
  fz = fz ^ (has_z * bit);
  fc = fc + dc;
}

// ---------------------------------------------------------------------------
// Register-slot gate application.  v[r] holds the amplitude whose register
// bits are r; a dense op acts on register bit B (and B1).

template <int B, int R, typename T>
DEV void g1_apply(cx<T> (&v)[1 << R], cx<T> m00, cx<T> m01, cx<T> m10, cx<T> m11) {
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    if (r & (1 << B)) continue;
    const cx<T> x = v[r], y = v[r | (1 << B)];
    v[r] = mac2(m00, x, m01, y);
    v[r | (1 << B)] = mac2(m10, x, m11, y);
    __builtin_amdgcn_sched_barrier(0);   // one pair at a time: bounded register use
  }
}

// Control bit of slot r = lane bit (thread / tile part of the index) or the
// slot's own bit when the control is a register qubit (cmask: its register
// bit, uniform).
template <int B, int R, typename T>
DEV void c1_apply(cx<T> (&v)[1 << R], cx<T> m00, cx<T> m01, cx<T> m10, cx<T> m11, uint32_t clane,
                  uint32_t cmask, uint32_t cv) {
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    if (r & (1 << B)) continue;
    const cx<T> x = v[r], y = v[r | (1 << B)];
    const bool take = (clane | (((uint32_t)r & cmask) ? 1u : 0u)) == cv;
    const cx<T> n0 = mac2(m00, x, m01, y), n1 = mac2(m10, x, m11, y);
    v[r] = take ? n0 : x;
    v[r | (1 << B)] = take ? n1 : y;
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int B0, int B1, int R, typename T>
DEV void g2_apply(cx<T> (&v)[1 << R], const cx<T> (&m)[16]) {
#pragma unroll
  for (int r = 0; r < (1 << R); ++r) {
    if (r & ((1 << B0) | (1 << B1))) continue;
    const int i0 = r, i1 = r | (1 << B0), i2 = r | (1 << B1), i3 = r | (1 << B0) | (1 << B1);
    const cx<T> a0 = v[i0], a1 = v[i1], a2 = v[i2], a3 = v[i3];
    cx<T> o[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      cx<T> s = mac2(m[4 * i + 0], a0, m[4 * i + 1], a1);
      cx<T> t = mac2(m[4 * i + 2], a2, m[4 * i + 3], a3);
      o[i] = cx<T>{s.x + t.x, s.y + t.y};
    }
    v[i0] = o[0];
    v[i1] = o[1];
    v[i2] = o[2];
    v[i3] = o[3];
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int R, typename T>
DEV void dispatch_g1(int B, cx<T> (&v)[1 << R], cx<T> m00, cx<T> m01, cx<T> m10, cx<T> m11) {
  switch (B) {
    case 0: g1_apply<0, R>(v, m00, m01, m10, m11); break;
    case 1: if constexpr (R > 1) g1_apply<1, R>(v, m00, m01, m10, m11); break;
    case 2: if constexpr (R > 2) g1_apply<2, R>(v, m00, m01, m10, m11); break;
    case 3: if constexpr (R > 3) g1_apply<3, R>(v, m00, m01, m10, m11); break;
    default: break;
  }
}

template <int R, typename T>
DEV void dispatch_c1(int B, cx<T> (&v)[1 << R], cx<T> m00, cx<T> m01, cx<T> m10, cx<T> m11,
                     uint32_t clane, uint32_t cmask, uint32_t cv) {
  switch (B) {
    case 0: c1_apply<0, R>(v, m00, m01, m10, m11, clane, cmask, cv); break;
    case 1: if constexpr (R > 1) c1_apply<1, R>(v, m00, m01, m10, m11, clane, cmask, cv); break;
    case 2: if constexpr (R > 2) c1_apply<2, R>(v, m00, m01, m10, m11, clane, cmask, cv); break;
    case 3: if constexpr (R > 3) c1_apply<3, R>(v, m00, m01, m10, m11, clane, cmask, cv); break;
    default: break;
  }
}

template <int B0, int B1, int R, typename T>
DEV void g2_if(cx<T> (&v)[1 << R], const cx<T> (&m)[16]) {
  if constexpr (B0 != B1 && B0 < R && B1 < R) g2_apply<B0, B1, R>(v, m);
}

template <int R, typename T>
DEV void dispatch_g2(int sel, cx<T> (&v)[1 << R], const cx<T> (&m)[16]) {
  switch (sel) {
    case 0x10: g2_if<0, 1, R>(v, m); break;
    case 0x20: g2_if<0, 2, R>(v, m); break;
    case 0x30: g2_if<0, 3, R>(v, m); break;
    case 0x01: g2_if<1, 0, R>(v, m); break;
    case 0x21: g2_if<1, 2, R>(v, m); break;
    case 0x31: g2_if<1, 3, R>(v, m); break;
    case 0x02: g2_if<2, 0, R>(v, m); break;
    case 0x12: g2_if<2, 1, R>(v, m); break;
    case 0x32: g2_if<2, 3, R>(v, m); break;
    case 0x03: g2_if<3, 0, R>(v, m); break;
    case 0x13: g2_if<3, 1, R>(v, m); break;
    case 0x23: g2_if<3, 2, R>(v, m); break;
    default: break;
  }
}

// Register bits of the segment that hold qubit q (0 or one bit), uniform.
template <int R>
DEV uint32_t reg_mask(const uint32_t (&rq)[R], uint32_t q) {
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < R; ++b) m |= (rq[b] == q ? 1u : 0u) << b;
  return m;
}

// Apply one op, conjugated by the current Pauli frame, to the register slots.
// gb: the thread's global index with all register bits zero; rq: global
// qubit of each register bit.  Index bit q of slot r is
// ((gb >> q) & 1) | (r & reg_mask(q) != 0).
template <int R, typename T>
DEV void apply_op(const DevOp<T> &op, cx<T> (&v)[1 << R], uint32_t gb, const uint32_t (&rq)[R],
                  uint32_t fx, uint32_t fz) {
  constexpr int NS = 1 << R;
  const int cls = op.cls;
  const uint32_t qa = (uint32_t)op.qa;
  const uint32_t xa = (fx >> qa) & 1u, za = (fz >> qa) & 1u;
  if (cls == OP_G1 || cls == OP_C1) {
    // (Z^z X^x) M (X^x Z^z): entry (i, j) = (-1)^{z(i+j)} M[i^x][j^x]
    cx<T> m00 = ment(op, (0u ^ xa) * 2u + (0u ^ xa)), m01 = ment(op, (0u ^ xa) * 2u + (1u ^ xa));
    cx<T> m10 = ment(op, (1u ^ xa) * 2u + (0u ^ xa)), m11 = ment(op, (1u ^ xa) * 2u + (1u ^ xa));
    if (za) {
      m01 = cneg(m01);
      m10 = cneg(m10);
    }
    if (cls == OP_G1) {
      dispatch_g1<R>(op.rsel & 15, v, m00, m01, m10, m11);
    } else {
      const uint32_t qc = (uint32_t)op.qb;
      const uint32_t cv = 1u ^ ((fx >> qc) & 1u);
      dispatch_c1<R>(op.rsel & 15, v, m00, m01, m10, m11, (gb >> qc) & 1u, reg_mask<R>(rq, qc), cv);
    }
  } else if (cls == OP_D1) {
    const cx<T> d0 = ment(op, 0u ^ xa), d1 = ment(op, 1u ^ xa);
    const uint32_t lane = (gb >> qa) & 1u, am = reg_mask<R>(rq, qa);
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const bool hi = lane | (((uint32_t)r & am) ? 1u : 0u);
      v[r] = cmul(hi ? d1 : d0, v[r]);
    }
  } else if (cls == OP_D2) {
    const uint32_t qb = (uint32_t)op.qb;
    const uint32_t xm = xa | (((fx >> qb) & 1u) << 1);
    const cx<T> d0 = ment(op, 0u ^ xm), d1 = ment(op, 1u ^ xm), d2 = ment(op, 2u ^ xm), d3 = ment(op, 3u ^ xm);
    const uint32_t la = (gb >> qa) & 1u, lb = (gb >> qb) & 1u;
    const uint32_t am = reg_mask<R>(rq, qa), bm = reg_mask<R>(rq, qb);
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const bool ba = la | (((uint32_t)r & am) ? 1u : 0u);
      const bool bb = lb | (((uint32_t)r & bm) ? 1u : 0u);
      const cx<T> d = bb ? (ba ? d3 : d2) : (ba ? d1 : d0);
      v[r] = cmul(d, v[r]);
    }
  } else if (cls == OP_G2) {
    const uint32_t qb = (uint32_t)op.qb;
    const uint32_t xm = xa | (((fx >> qb) & 1u) << 1);
    const uint32_t zm = za | (((fz >> qb) & 1u) << 1);
    cx<T> m[16];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cx<T> e = ment(op, ((uint32_t)i ^ xm) * 4u + ((uint32_t)j ^ xm));
        const uint32_t neg = (__popc(zm & (uint32_t)i) + __popc(zm & (uint32_t)j)) & 1u;
        m[4 * i + j] = neg ? cneg(e) : e;
      }
    dispatch_g2<R>(op.rsel & 0xff, v, m);
  }
}

// Deterministic block reduction of three doubles into out[0..2].
DEV void block_reduce3(double v0, double v1, double v2, double *out, unsigned char *smem) {
  const int NT = blockDim.x;
  const int tid = threadIdx.x;
  const int width = NT < 64 ? NT : 64;
  for (int off = width >> 1; off > 0; off >>= 1) {
    v0 = __dadd_rn(v0, __shfl_xor(v0, off, 64));
    v1 = __dadd_rn(v1, __shfl_xor(v1, off, 64));
    v2 = __dadd_rn(v2, __shfl_xor(v2, off, 64));
  }
  __syncthreads();                       // tile reads done; reuse LDS
  double *red = reinterpret_cast<double *>(smem);
  const int nw = (NT + 63) >> 6;
  if ((tid & 63) == 0) {
    red[3 * (tid >> 6) + 0] = v0;
    red[3 * (tid >> 6) + 1] = v1;
    red[3 * (tid >> 6) + 2] = v2;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int w = 0; w < nw; ++w) {
      s0 = __dadd_rn(s0, red[3 * w + 0]);
      s1 = __dadd_rn(s1, red[3 * w + 1]);
      s2 = __dadd_rn(s2, red[3 * w + 2]);
    }
    out[0] = s0;
    out[1] = s1;
    out[2] = s2;
  }
}

// MAXT: largest work-group this instantiation serves; WPE: waves per SIMD
// it must fit (bounds the register budget so two work-groups share a CU).
template <typename T, int R, int MAXT, int WPE>
__global__ void __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(WPE))) k_pass(const PassArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
  constexpr int NS = 1 << R;
  const uint32_t NT = blockDim.x;
  const uint32_t tid = threadIdx.x;
  const int b = (int)(blockIdx.x % (uint32_t)a.B);
  const uint32_t tile = blockIdx.x / (uint32_t)a.B;

  const DevPass &ps = *a.pass;
  uint32_t tilebase = 0;
  for (int i = 0; i < a.ntile_bits; ++i) tilebase |= ((tile >> i) & 1u) << ps.nlq[i];
  cx<T> *st = a.state + (uint64_t)b * a.state_stride;
  const int lt = a.L - R;
  uint32_t dlo = 0;
  for (int i = 0; i < lt; ++i) dlo |= ((tid >> i) & 1u) << ps.locq[i];
  // Global-index bits of the coalesced layout's slot k: OR of hbit[b] over
  // the set bits b of k.
  uint32_t hbit[R];
#pragma unroll
  for (int bb = 0; bb < R; ++bb) hbit[bb] = 1u << ps.locq[lt + bb];
  auto dhi = [&](int k) {
    uint32_t v = 0;
#pragma unroll
    for (int bb = 0; bb < R; ++bb)
      if ((k >> bb) & 1) v |= hbit[bb];
    return v;
  };

  // Load the tile (coalesced: thread-id bits are the low local bits).
  if (a.flags & PF_FIRST) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const uint32_t g = tilebase | dlo | dhi(k);
      lds[swz<T>((uint32_t)k * NT + tid)] = cx<T>{g == a.init_index ? T(1) : T(0), T(0)};
    }
  } else {
    cx<T> v[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = st[tilebase | dlo | dhi(k)];
#pragma unroll
    for (int k = 0; k < NS; ++k) lds[swz<T>((uint32_t)k * NT + tid)] = v[k];
  }
  __syncthreads();

  // Pauli frame at the start of this pass.
  const uint32_t *ev = a.events + (size_t)b * a.ev_stride;
  const int ne = a.ev_count[b];
  int ep = 0;
  uint32_t fx = 0, fz = 0, fc = 0;
  while (ep < ne) {
    const uint32_t e = ev[ep];
    if ((int)(e >> 8) >= a.op_begin) break;
    frame_apply(e, fx, fz, fc);
    ++ep;
  }

  for (int s = a.seg_begin; s < a.seg_end; ++s) {
    const DevSeg &sg = a.segs[s];
    uint32_t jb = 0, gb = tilebase;
    for (int i = 0; i < lt; ++i) {
      const uint32_t bit = (tid >> i) & 1u;
      jb |= bit << sg.tpos[i];
      gb |= bit << sg.tq[i];
    }
    uint32_t jbit[R], rq[R];
#pragma unroll
    for (int bb = 0; bb < R; ++bb) {
      jbit[bb] = 1u << sg.rpos[bb];
      rq[bb] = sg.rq[bb];
    }
    auto jaddr = [&](int r) {
      uint32_t j = jb;
#pragma unroll
      for (int bb = 0; bb < R; ++bb)
        if ((r >> bb) & 1) j |= jbit[bb];
      return swz<T>(j);
    };
    cx<T> v[NS];
#pragma unroll
    for (int r = 0; r < NS; ++r) v[r] = lds[jaddr(r)];
    for (int o = sg.op_begin; o < sg.op_end; ++o) {
      apply_op<R, T>(a.ops[o], v, gb, rq, fx, fz);
      while (ep < ne) {
        const uint32_t e = ev[ep];
        if ((int)(e >> 8) != o) break;
        frame_apply(e, fx, fz, fc);
        ++ep;
      }
    }
#pragma unroll
    for (int r = 0; r < NS; ++r) lds[jaddr(r)] = v[r];
    __syncthreads();
  }

  // The epilogue recomputes its addresses instead of keeping 2^R of them
  // live across the segment loop.
  asm volatile("" : "+v"(dlo));
  const size_t ntiles = (size_t)1 << a.ntile_bits;
  if (a.flags & PF_SCORE) {
    double ovr = 0.0, ovi = 0.0, nrm = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const uint32_t g = tilebase | dlo | dhi(k);
      const cx<T> s = lds[swz<T>((uint32_t)k * NT + tid)];
      const cx<T> r = a.ref[g ^ fx];
      double sr = (double)s.x, si = (double)s.y;
      if (__popc(fz & g) & 1u) {
        sr = -sr;
        si = -si;
      }
      const double rr = (double)r.x, ri = (double)r.y;
      ovr = __dadd_rn(ovr, __fma_rn(ri, si, __dmul_rn(rr, sr)));
      ovi = __dadd_rn(ovi, __fma_rn(-ri, sr, __dmul_rn(rr, si)));
      nrm = __dadd_rn(nrm, __fma_rn(si, si, __dmul_rn(sr, sr)));
    }
    block_reduce3(ovr, ovi, nrm, a.partials + ((size_t)b * ntiles + tile) * 3, smem_raw);
  } else {
    double nrm = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const uint32_t g = tilebase | dlo | dhi(k);
      const cx<T> s = lds[swz<T>((uint32_t)k * NT + tid)];
      st[g] = s;
      const double sr = (double)s.x, si = (double)s.y;
      nrm = __dadd_rn(nrm, __fma_rn(si, si, __dmul_rn(sr, sr)));
    }
    if (a.flags & PF_NORM)
      block_reduce3(nrm, nrm, nrm, a.partials + ((size_t)b * ntiles + tile) * 3, smem_raw);
  }
  if (a.frame_out && tile == 0 && tid == 0) {
    a.frame_out[4 * b + 0] = fx;
    a.frame_out[4 * b + 1] = fz;
    a.frame_out[4 * b + 2] = fc & 3u;
  }
}

template <typename T>
hipError_t launch_pass(const PassArgs<T> &a, int R, int nthreads, hipStream_t s) {
  const size_t ntiles = (size_t)1 << a.ntile_bits;
  const size_t blocks = ntiles * (size_t)a.B;
  size_t lds = ((size_t)1 << a.L) * sizeof(cx<T>);
  if (lds < 16 * 3 * sizeof(double)) lds = 16 * 3 * sizeof(double);
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
  // R = 4 work-groups are 2^(L-4) threads: 512 for complex64 (L = 13),
  // 256 for complex128 (L = 12); two of them share a CU's LDS.
  constexpr int MAXT4 = sizeof(T) == 4 ? 512 : 256;
  constexpr int WPE4 = sizeof(T) == 4 ? 4 : 2;
  if (nthreads > (R == 4 ? MAXT4 : 1024)) return hipErrorInvalidValue;
  switch (R) {
    case 1: hipLaunchKernelGGL((k_pass<T, 1, 1024, 1>), dim3((uint32_t)blocks), dim3(nthreads), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_pass<T, 2, 1024, 1>), dim3((uint32_t)blocks), dim3(nthreads), lds, s, a); break;
    case 3: hipLaunchKernelGGL((k_pass<T, 3, 1024, 1>), dim3((uint32_t)blocks), dim3(nthreads), lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_pass<T, 4, MAXT4, WPE4>), dim3((uint32_t)blocks), dim3(nthreads), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_pass<float>(const PassArgs<float> &, int, int, hipStream_t);
template hipError_t launch_pass<double>(const PassArgs<double> &, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Fixed-order FP64 sum over tiles of component `comp` of the partials of
// trajectory b (block-wide; every thread returns the same value in tid 0).
DEV double sum_partials(const double *p, int ntiles, int comp, double *red) {
  const int tid = threadIdx.x, NT = blockDim.x;
  double acc = 0.0;
  for (int t = tid; t < ntiles; t += NT) acc = __dadd_rn(acc, p[(size_t)t * 3 + comp]);
  for (int off = 32; off > 0; off >>= 1) acc = __dadd_rn(acc, __shfl_xor(acc, off, 64));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  double s = 0.0;
  if (tid == 0)
    for (int w = 0; w < (NT >> 6); ++w) s = __dadd_rn(s, red[w]);
  return s;
}

__global__ void __launch_bounds__(256) k_finalize(const double *partials, int ntiles, const double *nref,
                                                  double tau, double *fid, uint64_t *count) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  const double *p = partials + (size_t)b * ntiles * 3;
  const double ovr = sum_partials(p, ntiles, 0, red);
  const double ovi = sum_partials(p, ntiles, 1, red);
  const double nrm = sum_partials(p, ntiles, 2, red);
  if (threadIdx.x == 0) {
    const double num = __fma_rn(ovi, ovi, __dmul_rn(ovr, ovr));
    const double F = __ddiv_rn(num, __dmul_rn(nref[0], nrm));
    fid[b] = F;
    if (F >= tau) atomicAdd((unsigned long long *)count, 1ull);
  }
}

hipError_t launch_finalize(const double *partials, int ntiles, int B, const double *nref, double tau,
                           double *fid, uint64_t *count, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(B), dim3(256), 0, s, partials, ntiles, nref, tau, fid, count);
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
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= dim) return;
  const uint32_t x = frame[0], z = frame[1], c = frame[2] & 3u;
  const uint64_t src = k ^ (uint64_t)x;
  cx<T> v = st[src];
  if (__popc(z & (uint32_t)src) & 1u) v = cneg(v);
  cx<T> o = v;
  if (c == 1u) o = cx<T>{-v.y, v.x};
  else if (c == 2u) o = cneg(v);
  else if (c == 3u) o = cx<T>{v.y, -v.x};
  out[k] = o;
}

template <typename T>
hipError_t launch_unframe(const cx<T> *st, cx<T> *out, uint64_t dim, const uint32_t *frame, hipStream_t s) {
  const uint64_t blocks = (dim + 255) / 256;
  hipLaunchKernelGGL((k_unframe<T>), dim3((uint32_t)blocks), dim3(256), 0, s, st, out, dim, frame);
  return hipGetLastError();
}

template hipError_t launch_unframe<float>(const cx<float> *, cx<float> *, uint64_t, const uint32_t *, hipStream_t);
template hipError_t launch_unframe<double>(const cx<double> *, cx<double> *, uint64_t, const uint32_t *,
                                           hipStream_t);

}  // namespace ntk
