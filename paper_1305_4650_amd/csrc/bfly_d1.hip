// Level kernels for single applies, d = 1.
#include "bfly_d1.inc"

namespace bfly {

hipError_t shape_limits_d1(const Geo& g, int prec, ShapeLimits* out) {
  return on_d1(fz::LimitsOp{g, out}, g.q, g.phase, prec);
}

hipError_t run_levels_d1(const LevelArgs& la, int prec) {
  return on_d1(fz::SingleOp{la}, la.G->q, la.G->phase, prec);
}

}  // namespace bfly
