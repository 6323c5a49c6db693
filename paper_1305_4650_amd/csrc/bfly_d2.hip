// Level kernels for single applies, d = 2.
#include "bfly_d2.inc"

namespace bfly {

hipError_t shape_limits_d2(const Geo& g, int prec, ShapeLimits* out) {
  return on_d2(fz::LimitsOp{g, out}, g.q, g.phase, prec);
}

hipError_t run_levels_d2(const LevelArgs& la, int prec) {
  return on_d2(fz::SingleOp{la}, la.G->q, la.G->phase, prec);
}

}  // namespace bfly
