// Level kernels for single applies, d = 3.
#include "bfly_d3.inc"

namespace bfly {

hipError_t shape_limits_d3(const Geo& g, int prec, ShapeLimits* out) {
  return on_d3(fz::LimitsOp{g, out}, g.q, g.phase, prec);
}

hipError_t run_levels_d3(const LevelArgs& la, int prec) {
  return on_d3(fz::SingleOp{la}, la.G->q, la.G->phase, prec);
}

}  // namespace bfly
