// Level kernels for batched applies, d = 1.
#include "bfly_d1.inc"

namespace bfly {

hipError_t run_batch_d1(const BatchGroup& bg, int prec) {
  if (bg.n == 0) return hipSuccess;
  return on_d1(fz::BatchOp{bg}, bg.inst[0].G.q, bg.inst[0].G.phase, prec);
}

}  // namespace bfly
