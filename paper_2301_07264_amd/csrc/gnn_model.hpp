// Host side of the surrogate network: graph construction, the model and its
// training loop (kernels in gnn.hip, definitions in gnn.hpp).
#pragma once
#include <vector>

#include "engine.hpp"
#include "gnn.hpp"

namespace gnn {

// Rates of the 13 outputs: 10^(-5 + j / 4), j = 0 .. 12.
double output_rate(int j);

Graph build_graph(const nt::Circuit &c);

// A set of graphs resident on the device, nodes of consecutive graphs
// contiguous.
struct Dataset {
  int n_graphs = 0, n_nodes = 0;
  std::vector<int32_t> gptr;   // host copy, [n_graphs + 1]
  nt::DevBuf x, row_ptr, col, node_graph, gptr_d, glob, y;
  bool has_labels = false;
  void upload(const std::vector<Graph> &gs, const float *labels, hipStream_t s);
};

struct Model {
  nt::Ctx *cx = nullptr;
  Layout lay;
  nt::DevBuf params, grads, adam_m, adam_v;
  int64_t adam_t = 0;
  Dataset data;
  // activations and gradients of one batch
  nt::DevBuf h[L + 1], a[L], zc, u, v, dv, du, dzc, dh, dhp, dz, tmp, partials, loss_g;
  size_t cap_nodes = 0, cap_graphs = 0, partial_cap = 0;

  Model(nt::Ctx *c, uint64_t seed);
  void ensure(size_t nodes, size_t graphs);
  // forward over graphs [g0, g1) of ds; outputs (sigmoid) left in v, and
  // with labels the per-graph squared error in loss_g and dL/d(pre-sigmoid)
  // in dv.
  void forward(const Dataset &ds, int g0, int g1, bool bf16);
  // gradients of the batch loss into grads (overwritten); returns the loss.
  double loss_backward(const Dataset &ds, int g0, int g1, bool bf16);
  void adam_step(double lr);
  // mean loss of one epoch
  double train_epoch(int batch_graphs, double lr, uint64_t shuffle_seed);
};

}  // namespace gnn
