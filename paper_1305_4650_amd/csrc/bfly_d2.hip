// Fused level kernels for d = 2: one instantiation per supported q and
// precision, plus phase-specialised ones for the benchmark workloads.  The
// expensive phases (hyperbolic and generalized Radon) process right-hand
// sides in chunks that share their phase factors; the Fourier phase costs a
// few flops, so chunking it only adds register pressure (measured slower).
#include "bfly_fused.inc"

namespace bfly {
namespace {

template <int Q>
hipError_t run_q(const LevelArgs& la, int prec) {
  const int ph = la.G->phase;
  (void)ph;
  if constexpr (Q == 5) {
    if (ph == 0)
      return prec == 0 ? fz::run_levels_t<2, Q, double, 0, 1>(la) : fz::run_levels_t<2, Q, float, 0, 1>(la);
  }
  if constexpr (Q == 5) {
    if (ph == 1)
      return prec == 0 ? fz::run_levels_t<2, Q, double, 1, BFLY_RHS_CHUNK_FP64>(la) : fz::run_levels_t<2, Q, float, 1, BFLY_RHS_CHUNK_FP32>(la);
  }
  if constexpr (Q == 6) {
    if (ph == 0)
      return prec == 0 ? fz::run_levels_t<2, Q, double, 0, 1>(la) : fz::run_levels_t<2, Q, float, 0, 1>(la);
  }
  return prec == 0 ? fz::run_levels_t<2, Q, double, -1, 1>(la) : fz::run_levels_t<2, Q, float, -1, 1>(la);
}

}  // namespace

hipError_t run_levels_d2(const LevelArgs& la, int prec) {
  switch (la.G->q) {
    case 2:
      return run_q<2>(la, prec);
    case 3:
      return run_q<3>(la, prec);
    case 4:
      return run_q<4>(la, prec);
    case 5:
      return run_q<5>(la, prec);
    case 6:
      return run_q<6>(la, prec);
    case 7:
      return run_q<7>(la, prec);
    case 8:
      return run_q<8>(la, prec);
    case 9:
      return run_q<9>(la, prec);
    case 10:
      return run_q<10>(la, prec);
    case 11:
      return run_q<11>(la, prec);
    case 12:
      return run_q<12>(la, prec);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace bfly
