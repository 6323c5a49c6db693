// Level kernels for batched applies, d = 2.
#include "bfly_d2.inc"

namespace bfly {

hipError_t run_batch_d2(const BatchGroup& bg, int prec) {
  if (bg.n == 0) return hipSuccess;
  return on_d2(fz::BatchOp{bg}, bg.inst[0].G.q, bg.inst[0].G.phase, prec);
}

}  // namespace bfly
