// Learned surrogate of the success-probability curve: a graph neural network
// over the circuit's gate graph, trained on Monte Carlo labels (the
// tolerable-rate search uses its prediction to bracket the rate).
//
// Graph of a circuit: one node per gate; an edge (both directions) between
// consecutive gates on the same qubit.  Node features (GNN_FIN = 32):
//   [0, 17)  one-hot gate kind (nt_gate_kind order)
//   [17, 23) sin and cos of the up to three angles (0 when absent)
//   23       ASAP layer of the gate / circuit depth
//   24       arity - 1
//   25       n / 16
//   26       1
//   [27, 32) 0
// Graph globals (GNN_GLOB = 4): n / 16, G / 2048, S / 4096, 1.
//
// Network (hidden width GNN_H = 64, GNN_L = 3 message-passing layers):
//   H0 = relu(X W_in + b_in)
//   A_l = mean over neighbours of H_{l-1};  H_l = relu(H_{l-1} Ws_l + A_l Wn_l + b_l)
//   r = mean over the graph's nodes of H_L;  z = [r, globals]
//   u = relu(z W_h1 + b_h1);  out = sigmoid(u W_h2 + b_h2)   (GNN_OUT = 13 rates)
// Loss: mean squared error over graphs and outputs.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace gnn {

constexpr int FIN = 32, H = 64, L = 3, GLOB = 4, OUT = 13, ZW = H + GLOB;

// Host graph of one circuit.
struct Graph {
  int n_nodes = 0;
  std::vector<float> x;          // [n_nodes][FIN]
  std::vector<int32_t> row_ptr;  // [n_nodes + 1]
  std::vector<int32_t> col;      // neighbour node indices (local)
  float glob[GLOB] = {0, 0, 0, 0};
};

// Offsets of the parameter blocks in the flat parameter vector.
struct Layout {
  size_t w_in, b_in, ws[L], wn[L], b[L], w_h1, b_h1, w_h2, b_h2, total;
  Layout();
};

// Kernel launch wrappers (gnn.hip).  bf16: MFMA with bf16 operands and FP32
// accumulation; otherwise plain FP32 FMA in a fixed order.
// C(i, j) (+)= sum_k A(i, k) B(k, j) [+ bias(j)] [relu], with
// A(i, k) = A[i * a_i + k * a_k], B(k, j) = B[k * b_k + j * b_j], C row-major
// ldc; M rows, K and N <= 128.
hipError_t gemm_rows(bool bf16, const float *A, long a_i, long a_k, const float *B, long b_k, long b_j, float *C,
                     long ldc, int M, int K, int N, const float *bias, bool relu, bool accumulate, hipStream_t s);
// C[K][N] (+)= sum_m A[m][k] B[m][n] (A row-major lda, B row-major ldb), the
// sum over m in fixed order (chunk partials, then a fixed-order reduction).
hipError_t gemm_tn(bool bf16, const float *A, long lda, const float *B, long ldb, float *C, int M, int K, int N,
                   float *partials, size_t partial_cap, bool accumulate, hipStream_t s);
// out[j] (+)= sum_m D[m][j], fixed order.
hipError_t colsum(const float *D, long ldd, int M, int N, float *out, float *partials, size_t partial_cap,
                  bool accumulate, hipStream_t s);
// Mean over neighbours of the batch's rows; row_ptr points at the batch's
// first row, col holds dataset node indices, base = the batch's first node.
hipError_t agg_mean(const float *Hm, const int32_t *row_ptr, const int32_t *col, int base, int M, int F, float *A,
                    hipStream_t s);
// Its transpose (symmetric adjacency): dH[u] += sum_{v ~ u} dA[v] / deg(v).
hipError_t agg_mean_t(const float *dA, const int32_t *row_ptr, const int32_t *col, int base, int M, int F,
                      float *dH, hipStream_t s);
hipError_t relu_bwd(const float *dY, const float *Y, int n, float *dZ, hipStream_t s);
hipError_t segment_mean(const float *Hm, const int32_t *gptr, int G, int F, float *R, long ldr, hipStream_t s);
hipError_t segment_mean_bwd(const float *dR, long ldr, const int32_t *node_graph, const int32_t *gptr, int g_base,
                            int M, int F, float *dH, hipStream_t s);
// o = sigmoid(v) in place; loss partial per graph; dV = 2 (o - y) o (1 - o) / (G * OUT)
hipError_t sigmoid_mse(float *V, const float *Y, int G, float *dV, float *loss_g, hipStream_t s);
hipError_t adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s);
hipError_t copy_cols(const float *src, long lds, float *dst, long ldd, int M, int N, hipStream_t s);

}  // namespace gnn
