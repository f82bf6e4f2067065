/*
 * nisq_oracle.c -- plain FP64 CPU oracle for Monte Carlo Pauli-error
 * state-vector simulation (ArsoNISQ, arXiv 2301.07264).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the GPU library is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What it computes, and where the paper defines it:
 *   - state vector of 2^n complex amplitudes, amplitude k <-> basis state |k>,
 *     measured with probability |a_k|^2                     (Sec. II, Eq. 1)
 *   - a circuit is an ordered list of one- and two-qubit gates; its size G is
 *     the number of gates                                   (Sec. II)
 *   - Pauli error model: after a gate, X, Z or Y may act; single-qubit action
 *     as in Eq. 2 (X swaps, Z negates |1>, Y = -i a1|0> + i a0|1>)
 *   - an error is simulated by appending the error gate right after the gate
 *                                                          (Sec. IV-B)
 *   - Monte Carlo: N runs; after a 1q gate X/Z/Y with p_X/p_Z/p_Y; after a
 *     2q gate the same, independently on each of its qubits (Sec. IV-B.2)
 *   - success probability = mean of the success criterion over the N
 *     simulated states                                      (Sec. IV-C)
 *   - tolerable error rate = rate at which the success probability meets a
 *     target, found by MC at varying rates                  (Sec. IV-D, Fig. 3)
 *   - exhaustive single-error simulation: reference state plus every single
 *     X/Z/Y error at every site, k+2m sites                 (Sec. IV-B.1, Eq. 3)
 *   - Eq. 4 (success probability from single-error results) and Eq. 5
 *     (closed-form tolerable uniform rate)                  (Sec. IV-C, IV-D)
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - qubit 0 is the least-significant bit of k;
 *   - R_P(theta) = exp(-i theta P / 2); U(a,b,c) = Rz(a) Ry(b) Rz(c) is one
 *     gate with one site; CP(phi) phases the |11> subspace by e^{i phi};
 *     RZZ(g) = exp(-i g Z(x)Z / 2); a 4x4 matrix on (qa, qb) uses local
 *     index b_qa + 2 b_qb;
 *   - "error rate" p is per touched qubit per gate, uniform p_X=p_Y=p_Z=p/3;
 *   - random draws: Philox4x64-10 (Salmon et al., SC'11), key = (seed,
 *     circuit id), counter = (site, trajectory, 0, 0).  A site fires iff
 *     word0 < thr(p_x+p_y+p_z); its type is X if word1 < thr(p_x/sum), else
 *     Y if word1 < thr((p_x+p_y)/sum), else Z (thr(1/3) and thr(2/3) when
 *     p_x = p_y = p_z, so that the split does not depend on the rate);
 *     thr(x) = floor(x * 2^64), or "always" when x >= 1.  The rate is not in the counter, so fired sets are
 *     nested across rates (common random numbers);
 *   - the fidelity criterion is the indicator F >= tau, with
 *     F = |<R|psi>|^2 / (<R|R><psi|psi>);
 *   - the tolerable-rate search is a safeguarded regula falsi (Illinois) in
 *     log10(p) on common random numbers (the paper names Powell's method
 *     without its settings).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Gate kinds (the oracle's own numbering of the gate vocabulary). */
enum {
  O_H = 0, O_X, O_Y, O_Z, O_S, O_T, O_RX, O_RY, O_RZ, O_U, O_U1Q,
  O_CNOT, O_CZ, O_CP, O_SWAP, O_RZZ, O_U2Q, O_NKIND
};

static int kind_arity(int kind) { return kind >= O_CNOT ? 2 : 1; }

/* ------------------------------------------------------------------------ */
/* Gate matrices, FP64.  Single-qubit: 2x2 row-major on basis (|0>,|1>).
 * Two-qubit: 4x4 row-major on local index b_q0 + 2*b_q1 (q0 = first listed). */

static void mat2_mul(const cplx *a, const cplx *b, cplx *out) {
  cplx r[4];
  r[0] = a[0] * b[0] + a[1] * b[2];
  r[1] = a[0] * b[1] + a[1] * b[3];
  r[2] = a[2] * b[0] + a[3] * b[2];
  r[3] = a[2] * b[1] + a[3] * b[3];
  memcpy(out, r, sizeof r);
}

static void rz_mat(double t, cplx *m) {
  m[0] = cexp(-I * t / 2); m[1] = 0; m[2] = 0; m[3] = cexp(I * t / 2);
}
static void ry_mat(double t, cplx *m) {
  double c = cos(t / 2), s = sin(t / 2);
  m[0] = c; m[1] = -s; m[2] = s; m[3] = c;
}
static void rx_mat(double t, cplx *m) {
  double c = cos(t / 2), s = sin(t / 2);
  m[0] = c; m[1] = -I * s; m[2] = -I * s; m[3] = c;
}

/* Fill m (4 entries for 1q kinds, 16 for 2q kinds).  umat: caller matrix for
 * U1Q/U2Q as interleaved (re, im) doubles, row-major.  Returns arity or -1. */
int orc_gate_matrix(int kind, const double *p, const double *umat, double *out_ri) {
  cplx m[16];
  int i;
  memset(m, 0, sizeof m);
  switch (kind) {
  case O_H: m[0] = m[1] = m[2] = M_SQRT1_2; m[3] = -M_SQRT1_2; break;
  case O_X: m[1] = 1; m[2] = 1; break;
  case O_Y: m[1] = -I; m[2] = I; break;               /* Eq. 2: Y|0> = i|1> */
  case O_Z: m[0] = 1; m[3] = -1; break;
  case O_S: m[0] = 1; m[3] = I; break;
  case O_T: m[0] = 1; m[3] = cexp(I * M_PI / 4); break;
  case O_RX: rx_mat(p[0], m); break;
  case O_RY: ry_mat(p[0], m); break;
  case O_RZ: rz_mat(p[0], m); break;
  case O_U: {
    cplx a[4], b[4], c[4];
    rz_mat(p[0], a); ry_mat(p[1], b); rz_mat(p[2], c);
    mat2_mul(a, b, m);      /* Rz(a) Ry(b) */
    mat2_mul(m, c, m);      /* ... Rz(c): Rz(c) acts first */
    break;
  }
  case O_U1Q:
    for (i = 0; i < 4; ++i) m[i] = umat[2 * i] + I * umat[2 * i + 1];
    break;
  case O_CNOT: /* control = q0 (bit 0 of local index), target = q1 */
    m[0 * 4 + 0] = 1;   /* |c=0,t=0> */
    m[2 * 4 + 2] = 1;   /* |c=0,t=1> (index 2) */
    m[1 * 4 + 3] = 1;   /* |c=1,t=1> -> |c=1,t=0> */
    m[3 * 4 + 1] = 1;   /* |c=1,t=0> -> |c=1,t=1> */
    break;
  case O_CZ: m[0] = 1; m[5] = 1; m[10] = 1; m[15] = -1; break;
  case O_CP: m[0] = 1; m[5] = 1; m[10] = 1; m[15] = cexp(I * p[0]); break;
  case O_SWAP: m[0] = 1; m[1 * 4 + 2] = 1; m[2 * 4 + 1] = 1; m[15] = 1; break;
  case O_RZZ:
    m[0] = cexp(-I * p[0] / 2); m[5] = cexp(I * p[0] / 2);
    m[10] = cexp(I * p[0] / 2); m[15] = cexp(-I * p[0] / 2);
    break;
  case O_U2Q:
    for (i = 0; i < 16; ++i) m[i] = umat[2 * i] + I * umat[2 * i + 1];
    break;
  default: return -1;
  }
  int dim = kind_arity(kind) == 1 ? 4 : 16;
  for (i = 0; i < dim; ++i) { out_ri[2 * i] = creal(m[i]); out_ri[2 * i + 1] = cimag(m[i]); }
  return kind_arity(kind);
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 64x64->128 multiplies with an S-box-free Feistel-like mix; the key is
 * bumped by the Weyl constants between rounds. */

static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL;  /* golden ratio */
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL;  /* sqrt(3) - 1 */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(PHILOX_M0, x0, &hi0, &lo0);
    mulhilo64(PHILOX_M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* thr(x): integer threshold for an event of probability x.  *always is set
 * when x >= 1 (the event happens for every draw). */
uint64_t orc_threshold(double x, int *always) {
  *always = 0;
  if (!(x > 0)) return 0;
  if (x >= 1.0) { *always = 1; return UINT64_MAX; }
  return (uint64_t)floor(ldexp(x, 64));
}

typedef struct {
  uint64_t t_fire, c_x, c_xy;
  int a_fire, a_x, a_xy;
} thresholds;

static void make_thresholds(double px, double py, double pz, thresholds *th) {
  double sum = px + py + pz;
  th->t_fire = orc_threshold(sum, &th->a_fire);
  if (sum > 0 && px == py && py == pz) {
    /* uniform model: the type split is exactly one third each, whatever the
     * rate (px / sum would round differently from rate to rate) */
    th->c_x = orc_threshold(1.0 / 3.0, &th->a_x);
    th->c_xy = orc_threshold(2.0 / 3.0, &th->a_xy);
  } else if (sum > 0) {
    th->c_x = orc_threshold(px / sum, &th->a_x);
    th->c_xy = orc_threshold((px + py) / sum, &th->a_xy);
  } else {
    th->c_x = th->c_xy = 0; th->a_x = th->a_xy = 0;
  }
}

/* Export of the three thresholds (for tests). */
void orc_thresholds(double px, double py, double pz, uint64_t out[3], int always[3]) {
  thresholds th;
  make_thresholds(px, py, pz, &th);
  out[0] = th.t_fire; out[1] = th.c_x; out[2] = th.c_xy;
  always[0] = th.a_fire; always[1] = th.a_x; always[2] = th.a_xy;
}

/* Pauli codes: 1 = X, 2 = Y, 3 = Z. */
static int draw_site(uint64_t seed, uint64_t cid, uint64_t site, uint64_t traj,
                     const thresholds *th) {
  uint64_t ctr[4] = {site, traj, 0, 0}, key[2] = {seed, cid}, w[4];
  orc_philox4x64_10(ctr, key, w);
  if (!(th->a_fire || w[0] < th->t_fire)) return 0;
  if (th->a_x || w[1] < th->c_x) return 1;
  if (th->a_xy || w[1] < th->c_xy) return 2;
  return 3;
}

/* Fired sites of one trajectory in site order.  Sites are numbered in gate
 * order, and within a gate in the order its qubits are listed (Sec. IV-B.1:
 * k + 2m sites).  Returns the count; writes at most cap entries. */
int64_t orc_sample_trajectory(uint64_t seed, uint64_t cid, uint64_t traj, int64_t S,
                              double px, double py, double pz,
                              int32_t *sites, uint8_t *paulis, int64_t cap) {
  thresholds th;
  make_thresholds(px, py, pz, &th);
  int64_t cnt = 0;
  for (int64_t s = 0; s < S; ++s) {
    int pa = draw_site(seed, cid, (uint64_t)s, traj, &th);
    if (pa) {
      if (cnt < cap) { sites[cnt] = (int32_t)s; paulis[cnt] = (uint8_t)pa; }
      ++cnt;
    }
  }
  return cnt;
}

/* ------------------------------------------------------------------------ */
/* State-vector kernels (Sec. II): plain loops over all amplitudes. */

static void apply_1q(int n, cplx *psi, int q, const cplx *m) {
  uint64_t dim = 1ULL << n, bit = 1ULL << q;
  for (uint64_t k = 0; k < dim; ++k) {
    if (k & bit) continue;
    cplx a0 = psi[k], a1 = psi[k | bit];
    psi[k] = m[0] * a0 + m[1] * a1;
    psi[k | bit] = m[2] * a0 + m[3] * a1;
  }
}

static void apply_2q(int n, cplx *psi, int qa, int qb, const cplx *m) {
  uint64_t dim = 1ULL << n, ba = 1ULL << qa, bb = 1ULL << qb;
  for (uint64_t k = 0; k < dim; ++k) {
    if ((k & ba) || (k & bb)) continue;
    uint64_t idx[4] = {k, k | ba, k | bb, k | ba | bb};   /* local b_a + 2 b_b */
    cplx in[4], out[4];
    for (int i = 0; i < 4; ++i) in[i] = psi[idx[i]];
    for (int r = 0; r < 4; ++r) {
      out[r] = 0;
      for (int c = 0; c < 4; ++c) out[r] += m[4 * r + c] * in[c];
    }
    for (int i = 0; i < 4; ++i) psi[idx[i]] = out[i];
  }
}

/* Same loops, parallel over amplitudes (used for the largest states). */
static void apply_1q_par(int n, cplx *psi, int q, const cplx *m) {
  int64_t half = (int64_t)1 << (n - 1);
  uint64_t bit = 1ULL << q, low = bit - 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < half; ++i) {
    uint64_t k = (((uint64_t)i & ~low) << 1) | ((uint64_t)i & low);
    cplx a0 = psi[k], a1 = psi[k | bit];
    psi[k] = m[0] * a0 + m[1] * a1;
    psi[k | bit] = m[2] * a0 + m[3] * a1;
  }
}

static void apply_2q_par(int n, cplx *psi, int qa, int qb, const cplx *m) {
  int64_t dim = (int64_t)1 << n;
  uint64_t ba = 1ULL << qa, bb = 1ULL << qb;
#pragma omp parallel for schedule(static)
  for (int64_t kk = 0; kk < dim; ++kk) {
    uint64_t k = (uint64_t)kk;
    if ((k & ba) || (k & bb)) continue;
    uint64_t idx[4] = {k, k | ba, k | bb, k | ba | bb};
    cplx in[4], out[4];
    for (int i = 0; i < 4; ++i) in[i] = psi[idx[i]];
    for (int r = 0; r < 4; ++r) {
      out[r] = 0;
      for (int c = 0; c < 4; ++c) out[r] += m[4 * r + c] * in[c];
    }
    for (int i = 0; i < 4; ++i) psi[idx[i]] = out[i];
  }
}

/* Pauli error gate on qubit q, exactly Eq. 2. */
static void apply_pauli(int n, cplx *psi, int q, int pauli, int par) {
  uint64_t dim = 1ULL << n, bit = 1ULL << q;
  int64_t k;
#pragma omp parallel for schedule(static) if (par)
  for (k = 0; k < (int64_t)dim; ++k) {
    uint64_t u = (uint64_t)k;
    if (u & bit) continue;
    cplx a0 = psi[u], a1 = psi[u | bit];
    if (pauli == 1) {            /* X: a1|0> + a0|1> */
      psi[u] = a1; psi[u | bit] = a0;
    } else if (pauli == 3) {     /* Z: a0|0> - a1|1> */
      psi[u | bit] = -a1;
    } else if (pauli == 2) {     /* Y: -i a1|0> + i a0|1> */
      psi[u] = -I * a1; psi[u | bit] = I * a0;
    }
  }
}

/* Exported single operations (tests pin these against brute force). */
int orc_apply_gate(int n, double *psi_ri, int kind, int q0, int q1,
                   const double *params, const double *umat) {
  double mri[32];
  cplx m[16];
  int ar = orc_gate_matrix(kind, params, umat, mri);
  if (ar < 0) return -1;
  for (int i = 0; i < (ar == 1 ? 4 : 16); ++i) m[i] = mri[2 * i] + I * mri[2 * i + 1];
  cplx *psi = (cplx *)psi_ri;
  if (ar == 1) apply_1q(n, psi, q0, m);
  else apply_2q(n, psi, q0, q1, m);
  return 0;
}

void orc_apply_pauli(int n, double *psi_ri, int q, int pauli) {
  apply_pauli(n, (cplx *)psi_ri, q, pauli, 0);
}

/* ------------------------------------------------------------------------ */
/* Circuit and trajectory. */

typedef struct {
  int n;
  int64_t G, S;
  const int32_t *kind, *q0, *q1;
  const double *params;      /* 3 per gate */
  const double *umats;       /* 32 doubles per gate (U1Q/U2Q only) */
  cplx *mats;                /* 16 per gate, built once */
} circuit;

static int circuit_init(circuit *c, int n, int64_t G, const int32_t *kind, const int32_t *q0,
                        const int32_t *q1, const double *params, const double *umats) {
  c->n = n; c->G = G; c->kind = kind; c->q0 = q0; c->q1 = q1;
  c->params = params; c->umats = umats;
  c->mats = (cplx *)calloc((size_t)(G > 0 ? G : 1) * 16, sizeof(cplx));
  if (!c->mats) return -1;
  c->S = 0;
  for (int64_t g = 0; g < G; ++g) {
    double mri[32];
    int ar = orc_gate_matrix(kind[g], params + 3 * g, umats ? umats + 32 * g : NULL, mri);
    if (ar < 0) return -1;
    for (int i = 0; i < (ar == 1 ? 4 : 16); ++i) c->mats[16 * g + i] = mri[2 * i] + I * mri[2 * i + 1];
    c->S += ar;
  }
  return 0;
}

static void circuit_free(circuit *c) { free(c->mats); }

/* One trajectory: psi <- e_init; for each gate: psi <- U_g psi, then the
 * sampled Pauli of each fired site of g, in listed-qubit order (Sec. IV-B,
 * IV-B.2).  fired sites must be sorted by site index. */
static void run_trajectory(const circuit *c, uint64_t init_index, const int32_t *fsite,
                           const uint8_t *fpauli, int64_t nf, cplx *psi, int par) {
  uint64_t dim = 1ULL << c->n;
  memset(psi, 0, dim * sizeof(cplx));
  psi[init_index] = 1.0;
  int64_t site = 0, f = 0;
  for (int64_t g = 0; g < c->G; ++g) {
    int ar = kind_arity(c->kind[g]);
    const cplx *m = c->mats + 16 * g;
    if (ar == 1) {
      if (par) apply_1q_par(c->n, psi, c->q0[g], m); else apply_1q(c->n, psi, c->q0[g], m);
    } else {
      if (par) apply_2q_par(c->n, psi, c->q0[g], c->q1[g], m);
      else apply_2q(c->n, psi, c->q0[g], c->q1[g], m);
    }
    for (int j = 0; j < ar; ++j, ++site) {
      while (f < nf && fsite[f] < site) ++f;
      if (f < nf && fsite[f] == site) {
        int q = (j == 0) ? c->q0[g] : c->q1[g];
        apply_pauli(c->n, psi, q, fpauli[f], par);
      }
    }
  }
}

/* F = |<R|psi>|^2 / (<R|R> <psi|psi>), plain sequential sums (Sec. II, IV-C). */
static double fidelity(int n, const cplx *r, const cplx *psi) {
  uint64_t dim = 1ULL << n;
  cplx ov = 0;
  double nr = 0, np = 0;
  for (uint64_t k = 0; k < dim; ++k) {
    ov += conj(r[k]) * psi[k];
    nr += creal(r[k]) * creal(r[k]) + cimag(r[k]) * cimag(r[k]);
    np += creal(psi[k]) * creal(psi[k]) + cimag(psi[k]) * cimag(psi[k]);
  }
  double a = cabs(ov);
  return a * a / (nr * np);
}

double orc_fidelity(int n, const double *r_ri, const double *psi_ri) {
  return fidelity(n, (const cplx *)r_ri, (const cplx *)psi_ri);
}

/* Final state of one trajectory with an explicit fired-site list. */
int orc_final_state_pattern(int n, int64_t G, const int32_t *kind, const int32_t *q0,
                            const int32_t *q1, const double *params, const double *umats,
                            uint64_t init_index, const int32_t *fsite, const uint8_t *fpauli,
                            int64_t nf, double *psi_out) {
  circuit c;
  if (circuit_init(&c, n, G, kind, q0, q1, params, umats)) { circuit_free(&c); return -1; }
  run_trajectory(&c, init_index, fsite, fpauli, nf, (cplx *)psi_out, n >= 20);
  circuit_free(&c);
  return 0;
}

/* Final state of trajectory `traj` under the Monte Carlo error model. */
int orc_final_state(int n, int64_t G, const int32_t *kind, const int32_t *q0,
                    const int32_t *q1, const double *params, const double *umats,
                    double px, double py, double pz, uint64_t seed, uint64_t cid,
                    uint64_t traj, double *psi_out) {
  circuit c;
  if (circuit_init(&c, n, G, kind, q0, q1, params, umats)) { circuit_free(&c); return -1; }
  int32_t *fs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c.S + 1));
  uint8_t *fp = (uint8_t *)malloc((size_t)(c.S + 1));
  int64_t nf = orc_sample_trajectory(seed, cid, traj, c.S, px, py, pz, fs, fp, c.S);
  run_trajectory(&c, 0, fs, fp, nf, (cplx *)psi_out, n >= 20);
  free(fs); free(fp);
  circuit_free(&c);
  return 0;
}

/* Monte Carlo success probability (Sec. IV-B.2, IV-C): trajectories
 * [t0, t0+N); fid_out[i] = F of trajectory t0+i; *count = #(F >= tau).
 * nthreads <= 0 uses the OpenMP default.  Returns 0 on success. */
int orc_run(int n, int64_t G, const int32_t *kind, const int32_t *q0, const int32_t *q1,
            const double *params, const double *umats, double px, double py, double pz,
            uint64_t seed, uint64_t cid, uint64_t t0, uint64_t N, double tau,
            int nthreads, double *fid_out, uint64_t *count, int *threads_used) {
  circuit c;
  if (circuit_init(&c, n, G, kind, q0, q1, params, umats)) { circuit_free(&c); return -1; }
  uint64_t dim = 1ULL << n;
  cplx *ref = (cplx *)malloc(dim * sizeof(cplx));
  if (!ref) { circuit_free(&c); return -2; }
  int big = n >= 22;   /* large states: parallel inside each gate */
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  if (threads_used) *threads_used = omp_get_max_threads();
#else
  if (threads_used) *threads_used = 1;
#endif
  run_trajectory(&c, 0, NULL, NULL, 0, ref, big);
  uint64_t cnt = 0;
  int err = 0;
  if (big) {
    cplx *psi = (cplx *)malloc(dim * sizeof(cplx));
    int32_t *fs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c.S + 1));
    uint8_t *fp = (uint8_t *)malloc((size_t)(c.S + 1));
    if (!psi || !fs || !fp) err = -2;
    for (uint64_t i = 0; i < N && !err; ++i) {
      int64_t nf = orc_sample_trajectory(seed, cid, t0 + i, c.S, px, py, pz, fs, fp, c.S);
      run_trajectory(&c, 0, fs, fp, nf, psi, 1);
      double F = fidelity(n, ref, psi);
      if (fid_out) fid_out[i] = F;
      if (F >= tau) ++cnt;
    }
    free(psi); free(fs); free(fp);
  } else {
#pragma omp parallel reduction(+ : cnt)
    {
      cplx *psi = (cplx *)malloc(dim * sizeof(cplx));
      int32_t *fs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c.S + 1));
      uint8_t *fp = (uint8_t *)malloc((size_t)(c.S + 1));
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < (int64_t)N; ++i) {
        int64_t nf = orc_sample_trajectory(seed, cid, t0 + (uint64_t)i, c.S, px, py, pz, fs, fp, c.S);
        run_trajectory(&c, 0, fs, fp, nf, psi, 0);
        double F = fidelity(n, ref, psi);
        if (fid_out) fid_out[i] = F;
        if (F >= tau) ++cnt;
      }
      free(psi); free(fs); free(fp);
    }
  }
  *count = cnt;
  free(ref);
  circuit_free(&c);
  return err;
}

/* Success probability at each listed uniform rate (p/3 per Pauli). */
int orc_sweep(int n, int64_t G, const int32_t *kind, const int32_t *q0, const int32_t *q1,
              const double *params, const double *umats, const double *rates, int R,
              uint64_t seed, uint64_t cid, uint64_t N, double tau, int nthreads, double *p_out) {
  for (int r = 0; r < R; ++r) {
    uint64_t cnt = 0;
    double p3 = rates[r] / 3.0;
    int rc = orc_run(n, G, kind, q0, q1, params, umats, p3, p3, p3, seed, cid, 0, N, tau,
                     nthreads, NULL, &cnt, NULL);
    if (rc) return rc;
    p_out[r] = (double)cnt / (double)N;
  }
  return 0;
}

/* Tolerable uniform rate (Sec. IV-D, MC branch; the paper names Powell's
 * method without its settings, the reading here is a safeguarded regula falsi
 * (Illinois) in x = log10 p on f(x) = P(10^x) - P*, with the same trajectories
 * at every probe).  Start from the bracket [p_lo, p_hi]; each step probes the
 * secant root of the bracket (the midpoint if that falls outside); returns the
 * first probe with |P - P*| <= tol, else the bracket midpoint once
 * p_hi/p_lo <= 1.001.  When one end is kept twice in a row, its f is halved.
 * Returns 1 if not bracketed (P(p_lo) < P* or P(p_hi) > P*). */
static double mc_success(int n, int64_t G, const int32_t *kind, const int32_t *q0, const int32_t *q1,
                         const double *params, const double *umats, double p, uint64_t seed, uint64_t cid,
                         uint64_t N, double tau, int nthreads, int *rc) {
  uint64_t cnt = 0;
  double p3 = p / 3.0;
  *rc = orc_run(n, G, kind, q0, q1, params, umats, p3, p3, p3, seed, cid, 0, N, tau, nthreads, NULL, &cnt, NULL);
  return (double)cnt / (double)N;
}

int orc_tolerable_rate(int n, int64_t G, const int32_t *kind, const int32_t *q0,
                       const int32_t *q1, const double *params, const double *umats,
                       double P_target, double tol, double p_lo, double p_hi,
                       uint64_t seed, uint64_t cid, uint64_t N, double tau, int nthreads,
                       double *p_star, int *n_probes) {
  int rc, probes = 0;
  double a = log10(p_lo), b = log10(p_hi);
  double fa = mc_success(n, G, kind, q0, q1, params, umats, p_lo, seed, cid, N, tau, nthreads, &rc) - P_target;
  if (rc) return rc;
  ++probes;
  double fb = mc_success(n, G, kind, q0, q1, params, umats, p_hi, seed, cid, N, tau, nthreads, &rc) - P_target;
  if (rc) return rc;
  ++probes;
  *n_probes = probes;
  if (fa < 0 || fb > 0) return 1;
  int side = 0;
  for (;;) {
    if (pow(10.0, b - a) <= 1.001) { *p_star = pow(10.0, 0.5 * (a + b)); break; }
    double x = (fa == fb) ? 0.5 * (a + b) : (a * fb - b * fa) / (fb - fa);
    if (!(x > a && x < b)) x = 0.5 * (a + b);
    double px = pow(10.0, x);
    double fx = mc_success(n, G, kind, q0, q1, params, umats, px, seed, cid, N, tau, nthreads, &rc) - P_target;
    if (rc) return rc;
    ++probes;
    if (fabs(fx) <= tol) { *p_star = px; break; }
    if (fx > 0) {
      a = x; fa = fx;
      if (side == 1) fb *= 0.5;
      side = 1;
    } else {
      b = x; fb = fx;
      if (side == -1) fa *= 0.5;
      side = -1;
    }
  }
  *n_probes = probes;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive single-error simulation (Sec. IV-B.1, Eq. 3): for every site s
 * and every Pauli e in {X, Y, Z}, simulate the circuit with exactly that one
 * error and evaluate the fidelity against the reference.
 * fid_out is [S][3] (columns X, Y, Z).  Returns 0. */
int orc_exhaustive(int n, int64_t G, const int32_t *kind, const int32_t *q0, const int32_t *q1,
                   const double *params, const double *umats, int nthreads, double *fid_out) {
  circuit c;
  if (circuit_init(&c, n, G, kind, q0, q1, params, umats)) { circuit_free(&c); return -1; }
  uint64_t dim = 1ULL << n;
  cplx *ref = (cplx *)malloc(dim * sizeof(cplx));
  int big = n >= 22;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  run_trajectory(&c, 0, NULL, NULL, 0, ref, big);
  int64_t total = 3 * c.S;
  if (big) {
    cplx *psi = (cplx *)malloc(dim * sizeof(cplx));
    for (int64_t i = 0; i < total; ++i) {
      int32_t s = (int32_t)(i / 3);
      uint8_t pa = (uint8_t)(1 + i % 3);
      run_trajectory(&c, 0, &s, &pa, 1, psi, 1);
      fid_out[i] = fidelity(n, ref, psi);
    }
    free(psi);
  } else {
#pragma omp parallel
    {
      cplx *psi = (cplx *)malloc(dim * sizeof(cplx));
#pragma omp for schedule(dynamic, 4)
      for (int64_t i = 0; i < total; ++i) {
        int32_t s = (int32_t)(i / 3);
        uint8_t pa = (uint8_t)(1 + i % 3);
        run_trajectory(&c, 0, &s, &pa, 1, psi, 0);
        fid_out[i] = fidelity(n, ref, psi);
      }
      free(psi);
    }
  }
  free(ref);
  circuit_free(&c);
  return 0;
}

double orc_eq5(double P_target, const double P_e[3], double P_R, double units);

/* Tolerable uniform rate by the paper's steps (Sec. IV-D, Fig. 3), fidelity
 * criterion:
 *   1. exhaustive single-error simulation (Sec. IV-B.1): the success
 *      probability P_e of the states with one error of type e, and P_R = 1;
 *   2. success evaluation at one average error: by Eq. 4 with E(N_e) = 1/3
 *      for each type, P1 = sum_e P_e / 3;
 *   3. P1 <= P*: at most one error is tolerable, and Eq. 5 gives the rate,
 *      with the S error locations as its units (the paper writes G);
 *   4. otherwise Monte Carlo at increasing rates p_k = 2^k / S (one average
 *      error at k = 0) while the success probability stays at or above P*;
 *      a rate within tol of P* is the answer, else orc_tolerable_rate
 *      searches between the last two rates.  (If the success probability at
 *      1/S is already below P*, the rates decrease by halves instead until
 *      it is not.)
 * method: 0 = Eq. 5, 1 = Monte Carlo; P4 (may be NULL): P_e (X, Y, Z), P_R.
 * Returns 0, 1 if no rate in [1e-9, 0.5] brackets P* (or P_R < P*), or an
 * error code of the runs. */
int orc_tolerable_rate_fig3(int n, int64_t G, const int32_t *kind, const int32_t *q0, const int32_t *q1,
                            const double *params, const double *umats, double P_target, double tol,
                            uint64_t seed, uint64_t cid, uint64_t N, double tau, int nthreads,
                            double *p_star, int *method, int *n_probes, double *P4) {
  int64_t S = 0;
  for (int64_t g = 0; g < G; ++g) S += kind_arity(kind[g]);
  *n_probes = 0;
  if (S == 0) return 1;
  double *fe = (double *)malloc(sizeof(double) * (size_t)(3 * S));
  if (!fe) return -2;
  int rc = orc_exhaustive(n, G, kind, q0, q1, params, umats, nthreads, fe);
  if (rc) { free(fe); return rc; }
  double P_e[3];
  for (int e = 0; e < 3; ++e) {
    double cnt = 0;
    for (int64_t s = 0; s < S; ++s) cnt += fe[3 * s + e] >= tau ? 1.0 : 0.0;
    P_e[e] = cnt / (double)S;
  }
  free(fe);
  const double P_R = 1.0 >= tau ? 1.0 : 0.0;
  if (P4) { P4[0] = P_e[0]; P4[1] = P_e[1]; P4[2] = P_e[2]; P4[3] = P_R; }
  if (P_R < P_target) return 1;
  const double P1 = (P_e[0] + P_e[1] + P_e[2]) / 3.0;
  if (P1 <= P_target && P1 != P_R) {
    *method = 0;
    *p_star = orc_eq5(P_target, P_e, P_R, (double)S);
    return 0;
  }
  *method = 1;
  int probes = 0;
  double p = 1.0 / (double)S;
  double P = mc_success(n, G, kind, q0, q1, params, umats, p, seed, cid, N, tau, nthreads, &rc);
  if (rc) return rc;
  ++probes;
  double lo, hi;
  if (fabs(P - P_target) <= tol) { *p_star = p; *n_probes = probes; return 0; }
  if (P >= P_target) {
    for (;;) {
      lo = p;
      p *= 2.0;
      if (p > 0.5) { *n_probes = probes; return 1; }
      P = mc_success(n, G, kind, q0, q1, params, umats, p, seed, cid, N, tau, nthreads, &rc);
      if (rc) return rc;
      ++probes;
      if (fabs(P - P_target) <= tol) { *p_star = p; *n_probes = probes; return 0; }
      if (P < P_target) { hi = p; break; }
    }
  } else {
    for (;;) {
      hi = p;
      p *= 0.5;
      if (p < 1e-9) { *n_probes = probes; return 1; }
      P = mc_success(n, G, kind, q0, q1, params, umats, p, seed, cid, N, tau, nthreads, &rc);
      if (rc) return rc;
      ++probes;
      if (fabs(P - P_target) <= tol) { *p_star = p; *n_probes = probes; return 0; }
      if (P >= P_target) { lo = p; break; }
    }
  }
  int k = 0;
  rc = orc_tolerable_rate(n, G, kind, q0, q1, params, umats, P_target, tol, lo, hi, seed, cid, N, tau, nthreads,
                          p_star, &k);
  *n_probes = probes + k;
  return rc;
}

/* Eq. 4 with per-type single-error success probabilities P_e (e = X, Y, Z),
 * the error-free success P_R, and expected error counts E_e. */
double orc_eq4(const double P_e[3], double P_R, const double E_e[3]) {
  double s = 0, se = 0;
  for (int e = 0; e < 3; ++e) { s += P_e[e] * E_e[e]; se += E_e[e]; }
  return s + P_R * (1.0 - se);
}

/* Eq. 5: tolerable uniform rate p = (1/units) (P - P_R) / (sum_e P_e/3 - P_R),
 * where units is the number of error locations (G in the paper's form). */
double orc_eq5(double P_target, const double P_e[3], double P_R, double units) {
  double avg = (P_e[0] + P_e[1] + P_e[2]) / 3.0;
  return (P_target - P_R) / (avg - P_R) / units;
}

/* ------------------------------------------------------------------------ */
/* Other success criteria (Sec. II): probability of measuring the correct
 * basis state k, and the heavy-output probability (binning): the total noisy
 * probability on the set of basis states whose ideal probability exceeds the
 * median of the ideal distribution. */

static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* Median of the 2^n ideal probabilities: for an even count, the mean of the
 * two middle values. */
double orc_median_prob(int n, const double *psi_ri) {
  uint64_t dim = 1ULL << n;
  double *p = (double *)malloc(dim * sizeof(double));
  for (uint64_t k = 0; k < dim; ++k)
    p[k] = psi_ri[2 * k] * psi_ri[2 * k] + psi_ri[2 * k + 1] * psi_ri[2 * k + 1];
  qsort(p, dim, sizeof(double), cmp_double);
  double med = (dim % 2) ? p[dim / 2] : 0.5 * (p[dim / 2 - 1] + p[dim / 2]);
  free(p);
  return med;
}

/* Value of a criterion on the final state psi given the ideal state ref:
 * crit 0 = fidelity, 1 = |psi_target|^2 / <psi|psi>, 2 = heavy-output
 * probability (noisy mass on {k : |ref_k|^2 > med}) / <psi|psi>. */
static double criterion_value(int n, const cplx *ref, const cplx *psi, int crit, uint64_t target, double med) {
  if (crit == 0) return fidelity(n, ref, psi);
  uint64_t dim = 1ULL << n;
  double norm = 0, heavy = 0;
  for (uint64_t k = 0; k < dim; ++k) {
    double pk = creal(psi[k]) * creal(psi[k]) + cimag(psi[k]) * cimag(psi[k]);
    double rk = creal(ref[k]) * creal(ref[k]) + cimag(ref[k]) * cimag(ref[k]);
    norm += pk;
    if (rk > med) heavy += pk;
  }
  if (crit == 1) {
    double pt = creal(psi[target]) * creal(psi[target]) + cimag(psi[target]) * cimag(psi[target]);
    return pt / norm;
  }
  return heavy / norm;
}

/* Per-trajectory values of a criterion: crit 1 = |a_target|^2 / <psi|psi>;
 * crit 2 = heavy-output probability.  Returns 0. */
int orc_run_criterion(int n, int64_t G, const int32_t *kind, const int32_t *q0, const int32_t *q1,
                      const double *params, const double *umats, double px, double py, double pz,
                      uint64_t seed, uint64_t cid, uint64_t t0, uint64_t N, int crit,
                      uint64_t target, int nthreads, double *val_out) {
  circuit c;
  if (circuit_init(&c, n, G, kind, q0, q1, params, umats)) { circuit_free(&c); return -1; }
  uint64_t dim = 1ULL << n;
  cplx *ref = (cplx *)malloc(dim * sizeof(cplx));
  run_trajectory(&c, 0, NULL, NULL, 0, ref, 0);
  double med = orc_median_prob(n, (const double *)ref);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
  {
    cplx *psi = (cplx *)malloc(dim * sizeof(cplx));
    int32_t *fs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c.S + 1));
    uint8_t *fp = (uint8_t *)malloc((size_t)(c.S + 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < (int64_t)N; ++i) {
      int64_t nf = orc_sample_trajectory(seed, cid, t0 + (uint64_t)i, c.S, px, py, pz, fs, fp, c.S);
      run_trajectory(&c, 0, fs, fp, nf, psi, 0);
      val_out[i] = criterion_value(n, ref, psi, crit, target, med);
    }
    free(psi); free(fs); free(fp);
  }
  free(ref);
  circuit_free(&c);
  return 0;
}

/* Exhaustive single-error branch (Sec. IV-B.1) under any criterion: value of
 * the criterion on each of the 3S single-error states, [S][3] (X, Y, Z), and
 * on the reference state (*ref_val).  Small circuits only (one state per
 * thread). */
int orc_exhaustive_criterion(int n, int64_t G, const int32_t *kind, const int32_t *q0, const int32_t *q1,
                             const double *params, const double *umats, int crit, uint64_t target,
                             int nthreads, double *val_out, double *ref_val) {
  circuit c;
  if (circuit_init(&c, n, G, kind, q0, q1, params, umats)) { circuit_free(&c); return -1; }
  uint64_t dim = 1ULL << n;
  cplx *ref = (cplx *)malloc(dim * sizeof(cplx));
  run_trajectory(&c, 0, NULL, NULL, 0, ref, 0);
  double med = crit == 2 ? orc_median_prob(n, (const double *)ref) : 0.0;
  *ref_val = criterion_value(n, ref, ref, crit, target, med);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  int64_t total = 3 * c.S;
#pragma omp parallel
  {
    cplx *psi = (cplx *)malloc(dim * sizeof(cplx));
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < total; ++i) {
      int32_t s = (int32_t)(i / 3);
      uint8_t pa = (uint8_t)(1 + i % 3);
      run_trajectory(&c, 0, &s, &pa, 1, psi, 0);
      val_out[i] = criterion_value(n, ref, psi, crit, target, med);
    }
    free(psi);
  }
  free(ref);
  circuit_free(&c);
  return 0;
}
