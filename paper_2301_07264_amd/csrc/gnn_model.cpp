// Surrogate network: graph construction, parameters, forward and backward
// passes and Adam, sequenced on the context's stream.
#include "gnn_model.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace gnn {

using nt::check_hip;

Layout::Layout() {
  size_t o = 0;
  w_in = o; o += (size_t)FIN * H;
  b_in = o; o += H;
  for (int l = 0; l < L; ++l) {
    ws[l] = o; o += (size_t)H * H;
    wn[l] = o; o += (size_t)H * H;
    b[l] = o; o += H;
  }
  w_h1 = o; o += (size_t)ZW * H;
  b_h1 = o; o += H;
  w_h2 = o; o += (size_t)H * OUT;
  b_h2 = o; o += OUT;
  total = o;
}

double output_rate(int j) { return std::pow(10.0, -5.0 + j / 4.0); }

Graph build_graph(const nt::Circuit &c) {
  Graph g;
  const int G = (int)c.gates.size();
  g.n_nodes = G;
  g.x.assign((size_t)G * FIN, 0.f);
  // ASAP layer of every gate and the previous gate on every qubit
  std::vector<int> layer(G, 0), last(c.n, -1), qdepth(c.n, 0);
  std::vector<std::vector<int>> nbr(G);
  int depth = 0;
  for (int i = 0; i < G; ++i) {
    const nt::HostGate &hg = c.gates[i];
    int lv = 0;
    for (int k = 0; k < hg.nq; ++k) lv = std::max(lv, qdepth[hg.q[k]]);
    layer[i] = lv;
    depth = std::max(depth, lv + 1);
    for (int k = 0; k < hg.nq; ++k) {
      const int q = hg.q[k];
      qdepth[q] = lv + 1;
      if (last[q] >= 0) {
        nbr[i].push_back(last[q]);
        nbr[last[q]].push_back(i);
      }
      last[q] = i;
    }
  }
  for (int i = 0; i < G; ++i) {
    const nt::HostGate &hg = c.gates[i];
    float *x = &g.x[(size_t)i * FIN];
    x[hg.kind] = 1.f;
    const int np = nt::kind_nparam(hg.kind);
    for (int j = 0; j < np; ++j) {
      x[17 + 2 * j] = (float)std::sin(hg.param[j]);
      x[18 + 2 * j] = (float)std::cos(hg.param[j]);
    }
    x[23] = depth > 0 ? (float)layer[i] / (float)depth : 0.f;
    x[24] = (float)(hg.nq - 1);
    x[25] = (float)c.n / 16.f;
    x[26] = 1.f;
  }
  g.row_ptr.assign(G + 1, 0);
  for (int i = 0; i < G; ++i) g.row_ptr[i + 1] = g.row_ptr[i] + (int32_t)nbr[i].size();
  g.col.reserve(g.row_ptr[G]);
  for (int i = 0; i < G; ++i)
    for (int v : nbr[i]) g.col.push_back(v);
  g.glob[0] = (float)c.n / 16.f;
  g.glob[1] = (float)G / 2048.f;
  g.glob[2] = (float)c.S / 4096.f;
  g.glob[3] = 1.f;
  return g;
}

void Dataset::upload(const std::vector<Graph> &gs, const float *labels, hipStream_t s) {
  n_graphs = (int)gs.size();
  gptr.assign(n_graphs + 1, 0);
  size_t ne = 0;
  for (int i = 0; i < n_graphs; ++i) {
    gptr[i + 1] = gptr[i] + gs[i].n_nodes;
    ne += gs[i].col.size();
  }
  n_nodes = gptr[n_graphs];
  std::vector<float> hx((size_t)std::max(n_nodes, 1) * FIN), hg((size_t)std::max(n_graphs, 1) * GLOB);
  std::vector<int32_t> hrp(n_nodes + 1), hcol(std::max<size_t>(ne, 1)), hng(std::max(n_nodes, 1));
  size_t e = 0;
  for (int i = 0; i < n_graphs; ++i) {
    const Graph &g = gs[i];
    const int base = gptr[i];
    std::memcpy(&hx[(size_t)base * FIN], g.x.data(), g.x.size() * sizeof(float));
    for (int v = 0; v < g.n_nodes; ++v) {
      hrp[base + v] = (int32_t)e + g.row_ptr[v];
      hng[base + v] = i;
    }
    for (int32_t c : g.col) hcol[e++] = base + c;
    std::memcpy(&hg[(size_t)i * GLOB], g.glob, sizeof g.glob);
  }
  hrp[n_nodes] = (int32_t)e;
  x.ensure(hx.size() * 4);
  row_ptr.ensure(hrp.size() * 4);
  col.ensure(hcol.size() * 4);
  node_graph.ensure(hng.size() * 4);
  gptr_d.ensure(gptr.size() * 4);
  glob.ensure(hg.size() * 4);
  check_hip(hipMemcpyAsync(x.p, hx.data(), hx.size() * 4, hipMemcpyHostToDevice, s), "upload graphs");
  check_hip(hipMemcpyAsync(row_ptr.p, hrp.data(), hrp.size() * 4, hipMemcpyHostToDevice, s), "upload graphs");
  check_hip(hipMemcpyAsync(col.p, hcol.data(), hcol.size() * 4, hipMemcpyHostToDevice, s), "upload graphs");
  check_hip(hipMemcpyAsync(node_graph.p, hng.data(), hng.size() * 4, hipMemcpyHostToDevice, s), "upload graphs");
  check_hip(hipMemcpyAsync(gptr_d.p, gptr.data(), gptr.size() * 4, hipMemcpyHostToDevice, s), "upload graphs");
  check_hip(hipMemcpyAsync(glob.p, hg.data(), hg.size() * 4, hipMemcpyHostToDevice, s), "upload graphs");
  has_labels = labels != nullptr;
  if (labels) {
    y.ensure((size_t)n_graphs * OUT * 4);
    check_hip(hipMemcpyAsync(y.p, labels, (size_t)n_graphs * OUT * 4, hipMemcpyHostToDevice, s), "upload labels");
  }
  check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");   // host arrays go out of scope
}

// splitmix64 (Steele, Lea, Flood, OOPSLA'14)
static uint64_t splitmix(uint64_t &z) {
  uint64_t r = (z += 0x9E3779B97F4A7C15ull);
  r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
  r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
  return r ^ (r >> 31);
}

Model::Model(nt::Ctx *c, uint64_t seed) : cx(c) {
  // Xavier-uniform weights, zero biases
  std::vector<float> p(lay.total, 0.f);
  uint64_t z = seed;
  auto fill = [&](size_t off, int fan_in, int fan_out) {
    const double a = std::sqrt(6.0 / (fan_in + fan_out));
    for (size_t i = 0; i < (size_t)fan_in * fan_out; ++i) {
      const double u = (double)(splitmix(z) >> 11) * 0x1.0p-53;
      p[off + i] = (float)((2.0 * u - 1.0) * a);
    }
  };
  fill(lay.w_in, FIN, H);
  for (int l = 0; l < L; ++l) {
    fill(lay.ws[l], H, H);
    fill(lay.wn[l], H, H);
  }
  fill(lay.w_h1, ZW, H);
  fill(lay.w_h2, H, OUT);
  params.ensure(lay.total * 4);
  grads.ensure(lay.total * 4);
  adam_m.ensure(lay.total * 4);
  adam_v.ensure(lay.total * 4);
  check_hip(hipMemcpy(params.p, p.data(), lay.total * 4, hipMemcpyHostToDevice), "upload parameters");
  check_hip(hipMemset(adam_m.p, 0, lay.total * 4), "hipMemset");
  check_hip(hipMemset(adam_v.p, 0, lay.total * 4), "hipMemset");
}

void Model::ensure(size_t nodes, size_t graphs) {
  nodes = std::max<size_t>(nodes, 1);
  graphs = std::max<size_t>(graphs, 1);
  if (nodes > cap_nodes) {
    for (int l = 0; l <= L; ++l) h[l].ensure(nodes * H * 4);
    for (int l = 0; l < L; ++l) a[l].ensure(nodes * H * 4);
    dh.ensure(nodes * H * 4);
    dhp.ensure(nodes * H * 4);
    dz.ensure(nodes * H * 4);
    tmp.ensure(nodes * H * 4);
    cap_nodes = nodes;
  }
  if (graphs > cap_graphs) {
    zc.ensure(graphs * ZW * 4);
    u.ensure(graphs * H * 4);
    v.ensure(graphs * OUT * 4);
    dv.ensure(graphs * OUT * 4);
    du.ensure(graphs * H * 4);
    dzc.ensure(graphs * ZW * 4);
    loss_g.ensure(graphs * 4);
    cap_graphs = graphs;
  }
  // chunk partials of the row reductions (chunks of 512 rows, <= 128 x 128)
  const size_t need = ((nodes + 511) / 512 + 1) * 128 * 128;
  if (need > partial_cap) {
    partials.ensure(need * 4);
    partial_cap = need;
  }
}

void Model::forward(const Dataset &ds, int g0, int g1, bool bf16) {
  hipStream_t s = cx->stream;
  const int n0 = ds.gptr[g0], M = ds.gptr[g1] - n0, Gb = g1 - g0;
  ensure(M, Gb);
  const float *P = params.as<float>();
  const float *X = ds.x.as<float>() + (size_t)n0 * FIN;
  const int32_t *rp = ds.row_ptr.as<int32_t>() + n0;
  const int32_t *col = ds.col.as<int32_t>();
  check_hip(gemm_rows(bf16, X, FIN, 1, P + lay.w_in, H, 1, h[0].as<float>(), H, M, FIN, H, P + lay.b_in, true, false,
                      s), "gnn input layer");
  for (int l = 0; l < L; ++l) {
    check_hip(agg_mean(h[l].as<float>(), rp, col, n0, M, H, a[l].as<float>(), s), "gnn aggregate");
    check_hip(gemm_rows(bf16, h[l].as<float>(), H, 1, P + lay.ws[l], H, 1, h[l + 1].as<float>(), H, M, H, H,
                        P + lay.b[l], false, false, s), "gnn layer");
    check_hip(gemm_rows(bf16, a[l].as<float>(), H, 1, P + lay.wn[l], H, 1, h[l + 1].as<float>(), H, M, H, H, nullptr,
                        true, true, s), "gnn layer");
  }
  check_hip(segment_mean(h[L].as<float>(), ds.gptr_d.as<int32_t>() + g0, Gb, H, zc.as<float>(), ZW, s), "gnn pool");
  check_hip(copy_cols(ds.glob.as<float>() + (size_t)g0 * GLOB, GLOB, zc.as<float>() + H, ZW, Gb, GLOB, s),
            "gnn globals");
  check_hip(gemm_rows(bf16, zc.as<float>(), ZW, 1, P + lay.w_h1, H, 1, u.as<float>(), H, Gb, ZW, H, P + lay.b_h1,
                      true, false, s), "gnn head");
  check_hip(gemm_rows(bf16, u.as<float>(), H, 1, P + lay.w_h2, OUT, 1, v.as<float>(), OUT, Gb, H, OUT, P + lay.b_h2,
                      false, false, s), "gnn head");
  const float *Y = ds.has_labels ? ds.y.as<float>() + (size_t)g0 * OUT : nullptr;
  check_hip(sigmoid_mse(v.as<float>(), Y, Gb, Y ? dv.as<float>() : nullptr, Y ? loss_g.as<float>() : nullptr, s),
            "gnn output");
}

double Model::loss_backward(const Dataset &ds, int g0, int g1, bool bf16) {
  if (!ds.has_labels) throw nt::Error(NT_ERR_INVALID_ARG, "surrogate data has no labels");
  hipStream_t s = cx->stream;
  forward(ds, g0, g1, bf16);
  const int n0 = ds.gptr[g0], M = ds.gptr[g1] - n0, Gb = g1 - g0;
  const float *P = params.as<float>();
  float *Gd = grads.as<float>();
  float *pt = partials.as<float>();
  const size_t pc = partial_cap;
  const int32_t *rp = ds.row_ptr.as<int32_t>() + n0;
  const int32_t *col = ds.col.as<int32_t>();
  // head
  check_hip(gemm_tn(bf16, u.as<float>(), H, dv.as<float>(), OUT, Gd + lay.w_h2, Gb, H, OUT, pt, pc, false, s),
            "gnn grad");
  check_hip(colsum(dv.as<float>(), OUT, Gb, OUT, Gd + lay.b_h2, pt, pc, false, s), "gnn grad");
  check_hip(gemm_rows(bf16, dv.as<float>(), OUT, 1, P + lay.w_h2, 1, OUT, du.as<float>(), H, Gb, OUT, H, nullptr,
                      false, false, s), "gnn grad");
  check_hip(relu_bwd(du.as<float>(), u.as<float>(), Gb * H, du.as<float>(), s), "gnn grad");
  check_hip(gemm_tn(bf16, zc.as<float>(), ZW, du.as<float>(), H, Gd + lay.w_h1, Gb, ZW, H, pt, pc, false, s),
            "gnn grad");
  check_hip(colsum(du.as<float>(), H, Gb, H, Gd + lay.b_h1, pt, pc, false, s), "gnn grad");
  check_hip(gemm_rows(bf16, du.as<float>(), H, 1, P + lay.w_h1, 1, H, dzc.as<float>(), ZW, Gb, H, ZW, nullptr, false,
                      false, s), "gnn grad");
  // pool
  check_hip(segment_mean_bwd(dzc.as<float>(), ZW, ds.node_graph.as<int32_t>() + n0, ds.gptr_d.as<int32_t>() + g0, g0,
                             M, H, dh.as<float>(), s), "gnn grad");
  // message-passing layers
  for (int l = L - 1; l >= 0; --l) {
    check_hip(relu_bwd(dh.as<float>(), h[l + 1].as<float>(), M * H, dz.as<float>(), s), "gnn grad");
    check_hip(gemm_tn(bf16, h[l].as<float>(), H, dz.as<float>(), H, Gd + lay.ws[l], M, H, H, pt, pc, false, s),
              "gnn grad");
    check_hip(gemm_tn(bf16, a[l].as<float>(), H, dz.as<float>(), H, Gd + lay.wn[l], M, H, H, pt, pc, false, s),
              "gnn grad");
    check_hip(colsum(dz.as<float>(), H, M, H, Gd + lay.b[l], pt, pc, false, s), "gnn grad");
    // dH_prev = dZ Ws^T + agg^T(dZ Wn^T)
    check_hip(gemm_rows(bf16, dz.as<float>(), H, 1, P + lay.ws[l], 1, H, dhp.as<float>(), H, M, H, H, nullptr, false,
                        false, s), "gnn grad");
    check_hip(gemm_rows(bf16, dz.as<float>(), H, 1, P + lay.wn[l], 1, H, tmp.as<float>(), H, M, H, H, nullptr, false,
                        false, s), "gnn grad");
    check_hip(agg_mean_t(tmp.as<float>(), rp, col, n0, M, H, dhp.as<float>(), s), "gnn grad");
    std::swap(dh.p, dhp.p);
    std::swap(dh.bytes, dhp.bytes);
  }
  check_hip(relu_bwd(dh.as<float>(), h[0].as<float>(), M * H, dz.as<float>(), s), "gnn grad");
  check_hip(gemm_tn(bf16, ds.x.as<float>() + (size_t)n0 * FIN, FIN, dz.as<float>(), H, Gd + lay.w_in, M, FIN, H, pt,
                    pc, false, s), "gnn grad");
  check_hip(colsum(dz.as<float>(), H, M, H, Gd + lay.b_in, pt, pc, false, s), "gnn grad");
  std::vector<float> lg(Gb);
  check_hip(hipMemcpyAsync(lg.data(), loss_g.p, (size_t)Gb * 4, hipMemcpyDeviceToHost, s), "copy loss");
  check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  double loss = 0;
  for (float x : lg) loss += x;
  return loss / ((double)Gb * OUT);
}

void Model::adam_step(double lr) {
  ++adam_t;
  const double b1 = 0.9, b2 = 0.999;
  const double c1 = 1.0 - std::pow(b1, (double)adam_t), c2 = 1.0 - std::pow(b2, (double)adam_t);
  check_hip(adam(params.as<float>(), grads.as<float>(), adam_m.as<float>(), adam_v.as<float>(), lay.total, (float)lr,
                 (float)b1, (float)b2, 1e-8f, (float)c1, (float)c2, cx->stream), "gnn adam");
}

double Model::train_epoch(int batch_graphs, double lr, uint64_t shuffle_seed) {
  const int ng = data.n_graphs;
  std::vector<int> order;
  for (int g0 = 0; g0 < ng; g0 += batch_graphs) order.push_back(g0);
  uint64_t z = shuffle_seed;
  for (size_t i = order.size(); i > 1; --i) std::swap(order[i - 1], order[splitmix(z) % i]);   // Fisher-Yates
  double tot = 0;
  int64_t cnt = 0;
  for (int g0 : order) {
    const int g1 = std::min(ng, g0 + batch_graphs);
    tot += loss_backward(data, g0, g1, true) * (g1 - g0);
    cnt += g1 - g0;
    adam_step(lr);
  }
  return cnt ? tot / (double)cnt : 0.0;
}

}  // namespace gnn
