// Host-only driver of the planner (plan.cpp), built with the address and
// undefined-behaviour sanitizers by the CPU test suite: it plans the partitions
// given on stdin and prints the sizes and invariants of each plan, so that any
// out-of-bounds access or undefined operation in the host stage of bddc_setup
// stops the run.  Needs no GPU and no HIP runtime.
//
// stdin, one case per line:  dim nel0 nel1 nel2 constraints n0 cuts0... n1 cuts1... n2 cuts2...
//   (n_a cut positions per axis, 0 ... nel_a; nel2 = 1 and n2 = 2 "0 1" in 2D)
// stdout, per case: status n_free n_sub n_coarse sum_ni max_nci n_tiles factor_tasks
#include <cmath>
#include <cstdio>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "bddc_internal.h"

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    if (line.empty()) continue;
    std::istringstream in(line);
    bddc_mesh mesh{};
    uint32_t cons = 0;
    in >> mesh.dim >> mesh.nel[0] >> mesh.nel[1] >> mesh.nel[2] >> cons;
    std::vector<int64_t> cuts[3];
    bddc_partition part{};
    for (int a = 0; a < 3; ++a) {
      int n = 0;
      in >> n;
      cuts[a].resize(n);
      for (int q = 0; q < n; ++q) in >> cuts[a][q];
      part.nsub[a] = n - 1;
      part.cuts[a] = cuts[a].data();
    }
    bddc::Plan P;
    std::string err;
    const int rc = bddc::make_plan(&mesh, &part, cons, P, err);
    int64_t sum_ni = 0;
    for (auto& D : P.subs) sum_ni += D.n_i;
    // envelope storage: every stored tile (row i < T: columns fc[i] .. i; the
    // border row: 0 .. T) has its own index, all indices together fill
    // [0, n_tiles - 1), and every tile left of an envelope maps to the zero tile
    if (rc == 0) {
      std::vector<char> seen(P.n_tiles, 0);
      bool ok = true;
      for (auto& D : P.subs) {
        for (int i = 0; i < D.Tx; ++i)
          for (int j = 0; j <= i; ++j) {
            const int64_t t = bddc::env_tile(D, i, j);
            const bool inside = i >= D.T || j >= D.env[i].fc;
            if (t < 0 || t >= P.n_tiles) { ok = false; continue; }
            if (!inside) { ok = ok && t == P.n_tiles - 1; continue; }
            if (t == P.n_tiles - 1 || seen[t]) ok = false;
            seen[t] = 1;
          }
      }
      for (int64_t t = 0; t + 1 < P.n_tiles; ++t) ok = ok && seen[t];
      if (!ok) {
        std::fprintf(stderr, "envelope storage check failed\n");
        return 3;
      }
      // the factorisation flop count, by enumerating every tile update: for
      // each column k, a diagonal factorisation, then for every nonzero (i, k)
      // a panel solve and, for every nonzero (j, k) with k < j <= i, the update
      // of tile (i, j) (diagonal: one tile product, off-diagonal: two)
      double flops = 0.0;
      const double b3 = double(bddc::NB) * bddc::NB * bddc::NB;
      for (auto& D : P.subs) {
        auto nz = [&](int i, int k) { return i >= D.T || D.env[i].fc <= k; };
        for (int k = 0; k < D.T; ++k) {
          flops += b3 / 3.0;
          for (int i = k + 1; i < D.Tx; ++i) {
            if (!nz(i, k)) continue;
            flops += b3;
            for (int j = k + 1; j <= i; ++j)
              if (nz(j, k)) flops += j == i ? b3 : 2.0 * b3;
          }
        }
      }
      if (std::abs(flops - P.factor_flops) > 1e-12 * flops) {
        std::fprintf(stderr, "factorisation flop count %.17g differs from the enumeration %.17g\n",
                     P.factor_flops, flops);
        return 4;
      }
    }
    std::printf("%d %lld %d %d %lld %d %lld %lld\n", rc, (long long)P.n_free, P.nsubs, P.n_coarse,
                (long long)sum_ni, P.max_nci, (long long)P.n_tiles, (long long)(P.factor_tasks.size() / 3));
    if (rc) std::fprintf(stderr, "case failed: %s\n", err.c_str());
  }
  return 0;
}
