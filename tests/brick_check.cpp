// Host check of the stencil sweeps: for each lattice given on the command line (X Y Z T ...),
// the library's own brick choice (a2a::geom_to_geo) and both sweep orders (a2a::brick_site,
// x or y fastest inside a brick) visit every checkerboard site of a parity exactly once.
// Prints one line per lattice; exit status 1 on the first failure.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "runtime.h"

template <bool YFAST>
static bool bijection(const a2a::Geo& g) {
  std::vector<char> seen(g.hv, 0);
  for (int p = 0; p < g.hv; ++p) {
    const int s = a2a::brick_site<YFAST>(g, p);
    if (s < 0 || s >= g.hv || seen[s]) return false;
    seen[s] = 1;
  }
  return true;
}

int main(int argc, char** argv) {
  for (int i = 1; i + 3 < argc; i += 4) {
    a2a_geom geom;
    for (int m = 0; m < 4; ++m) geom.dims[m] = std::atoi(argv[i + m]);
    geom.t_bc = -1;
    a2a::Geo g;
    if (a2a::geom_to_geo(&geom, &g) != 0) {
      std::printf("%d %d %d %d: rejected\n", geom.dims[0], geom.dims[1], geom.dims[2], geom.dims[3]);
      return 1;
    }
    const bool ok = bijection<true>(g) && bijection<false>(g);
    std::printf("%d %d %d %d: brick %d x %d x %d x %d, %s\n", geom.dims[0], geom.dims[1], geom.dims[2], geom.dims[3],
                g.bxh, g.by, g.bz, g.bt, ok ? "bijection" : "NOT A BIJECTION");
    if (!ok) return 1;
  }
  return 0;
}
