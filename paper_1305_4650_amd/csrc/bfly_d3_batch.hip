// Level kernels for batched applies, d = 3.
#include "bfly_d3.inc"

namespace bfly {

hipError_t run_batch_d3(const BatchGroup& bg, int prec) {
  if (bg.n == 0) return hipSuccess;
  return on_d3(fz::BatchOp{bg}, bg.inst[0].G.q, bg.inst[0].G.phase, prec);
}

}  // namespace bfly
