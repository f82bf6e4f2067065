// Host-side driver for the address / undefined-behaviour sanitizer build of
// libnisqtol's host code (circuit loading and validation, the text format,
// the gate-pass planner with and without fusion, plan export, the surrogate's
// graph construction, Eq. 4 / Eq. 5, and the error paths of the C ABI).  No
// GPU is needed: nt_create must fail cleanly without one, and every other
// call here is host-only.  Usage: driver <circuit.txt>...; exit status 0
// when every check holds.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "nisqtol.h"

static int failures = 0;

#define CHECK(cond)                                                         \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

static void plan_checks(nt_circuit *c) {
  int n = 0;
  int64_t G = 0, S = 0;
  CHECK(nt_circuit_info(c, &n, &G, &S) == NT_OK);
  for (int prec : {NT_C64, NT_C128}) {
    for (int fuse : {1, 2, 3, 4}) {
      CHECK(nt_circuit_set_fusion(c, prec, fuse) == NT_OK);
      int np = 0, ns = 0, L = 0;
      CHECK(nt_plan_info(c, prec, &np, &ns, &L) == NT_OK);
      std::vector<int32_t> og(G), op(G), os(G);
      std::vector<uint64_t> pm(np), sm(ns);
      CHECK(nt_plan_export(c, prec, og.data(), op.data(), os.data(), pm.data(), sm.data()) == NT_OK);
      std::vector<int> seen(G, 0);
      for (int64_t k = 0; k < G; ++k) {
        CHECK(og[k] >= 0 && og[k] < G);
        if (og[k] >= 0 && og[k] < G) ++seen[og[k]];
        CHECK(op[k] >= 0 && op[k] < np);
        CHECK(os[k] >= 0 && os[k] < ns);
      }
      for (int64_t g = 0; g < G; ++g) CHECK(seen[g] == 1);
      int64_t ops = 0, blocks = 0;
      CHECK(nt_plan_ops(c, prec, &ops, &blocks) == NT_OK);
      // one op per gate without fusion; with it, each block applies at
      // least two gates and may bring one no-op pad
      if (fuse == 1) CHECK(blocks == 0 && ops == G);
      if (fuse != 1) CHECK(ops <= G && ops >= blocks && (G == 0 || ops > 0));
    }
    for (int L = 0; L <= 14; ++L) (void)nt_circuit_set_tile(c, prec, L);   // valid and invalid widths
    CHECK(nt_circuit_set_tile(c, prec, 0) == NT_OK);
    CHECK(nt_circuit_set_fusion(c, prec, 0) == NT_OK);
  }
  CHECK(nt_circuit_set_fusion(c, NT_C64, 5) == NT_ERR_INVALID_ARG);
  // the surrogate's graph of the circuit
  int64_t nn = 0, ne = 0;
  CHECK(nt_gnn_graph(c, nullptr, nullptr, nullptr, nullptr, &nn, &ne) == NT_OK);
  CHECK(nn == G);
  std::vector<float> x((size_t)nn * 32), glob(4);
  std::vector<int32_t> rp((size_t)nn + 1), col((size_t)ne);
  CHECK(nt_gnn_graph(c, x.data(), rp.data(), col.data(), glob.data(), &nn, &ne) == NT_OK);
  CHECK(rp[0] == 0 && rp[(size_t)nn] == ne);
}

int main(int argc, char **argv) {
  // no device: nt_create fails with NT_ERR_DEVICE and a message
  nt_ctx *ctx = nullptr;
  CHECK(nt_create(&ctx, 0, nullptr) == NT_ERR_DEVICE);
  CHECK(std::strlen(nt_last_error()) > 0);
  CHECK(std::strlen(nt_version()) > 0);
  // argument validation
  nt_circuit *c = nullptr;
  nt_gate g[2];
  std::memset(g, 0, sizeof g);
  g[0].kind = NT_CNOT;
  g[0].nq = 2;
  g[0].q[0] = 0;
  g[0].q[1] = 0;
  CHECK(nt_circuit_load(nullptr, 2, g, 1, &c) == NT_ERR_INVALID_ARG);   // duplicate qubits
  g[0].q[1] = 5;
  CHECK(nt_circuit_load(nullptr, 2, g, 1, &c) == NT_ERR_INVALID_ARG);   // qubit out of range
  g[0].kind = NT_U1Q;
  g[0].nq = 1;
  CHECK(nt_circuit_load(nullptr, 2, g, 1, &c) == NT_ERR_INVALID_ARG);   // matrix missing
  double bad[8] = {1, 0, 1, 0, 0, 0, 1, 0};
  g[0].matrix = bad;
  CHECK(nt_circuit_load(nullptr, 2, g, 1, &c) == NT_ERR_INVALID_ARG);   // not unitary
  g[0].kind = NT_RX;
  g[0].matrix = nullptr;
  g[0].param[0] = NAN;
  CHECK(nt_circuit_load(nullptr, 2, g, 1, &c) == NT_ERR_INVALID_ARG);   // non-finite angle
  CHECK(nt_circuit_load(nullptr, 40, g, 0, &c) == NT_ERR_INVALID_ARG);  // too many qubits
  CHECK(nt_circuit_load(nullptr, 2, g, (int64_t(1) << 19) + 1, &c) == NT_ERR_UNSUPPORTED);
  CHECK(nt_circuit_load_text(nullptr, "/nonexistent/circuit.txt", &c) == NT_ERR_INVALID_ARG);
  // a circuit without gates plans and exports
  CHECK(nt_circuit_load(nullptr, 3, g, 0, &c) == NT_OK);
  plan_checks(c);
  nt_circuit_free(c);
  // Eq. 4 / Eq. 5
  const double Pe[3] = {0.2, 0.5, 0.8}, E[3] = {0.1, 0.1, 0.1};
  double P = 0, p = 0;
  CHECK(nt_eq4(Pe, 1.0, E, &P) == NT_OK && std::fabs(P - (0.02 + 0.05 + 0.08 + 0.7)) < 1e-15);
  CHECK(nt_eq5(0.66, Pe, 1.0, 100.0, &p) == NT_OK && std::fabs(p - 0.34 / 0.5 / 100.0) < 1e-15);
  CHECK(nt_eq5(0.66, Pe, 0.5, 100.0, &p) == NT_ERR_INVALID_ARG);        // no change from single errors
  // the circuits given on the command line
  for (int i = 1; i < argc; ++i) {
    CHECK(nt_circuit_load_text(nullptr, argv[i], &c) == NT_OK);
    if (!c) continue;
    plan_checks(c);
    CHECK(nt_circuit_set_id(c, 17) == NT_OK);
    nt_circuit_free(c);
    c = nullptr;
  }
  nt_circuit_free(nullptr);
  nt_destroy(nullptr);
  if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
  else std::printf("host sanitizer driver: all checks passed on %d circuits\n", argc - 1);
  return failures ? 1 : 0;
}
