// Phase-factor throughput microkernel: the cost of one factor exp(2 pi i tau)
// (reduction modulo 1 and sine/cosine) in each precision mode, measured with
// the very functions the level kernels call.  The paper evaluates these
// factors in batches with vector sine/cosine routines and counts them as the
// bulk of the work (Sec. 3); the measured rate fixes the per-factor cost used
// in the roofline accounting of an apply.
#include "bfly_fused.inc"

#include "../../include/bfly.h"

namespace bfly {
namespace fz {
namespace {

constexpr int kRateThreads = 256;
constexpr int kRateUnroll = 8;  // independent chains per thread

// Every thread evaluates iters factors (a multiple of kRateUnroll) at
// arguments tau = tau0 + k * step, tau0 spread over [0, span) turns, and
// sums them into out[thread] so that nothing is left unused.  Per factor the
// harness adds one FP64 add (the argument) and two adds (the sum).
template <typename Real>
__global__ __launch_bounds__(kRateThreads) void k_phase_rate(int64_t n, int64_t iters, double span,
                                                             double2* __restrict__ out) {
  using T = typename CT<Real>::T;
  stage_cis<2, Real>();
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kRateThreads + threadIdx.x;
  if (t >= n) return;
  const double step = 0.6180339887498949;  // turns between consecutive arguments of a chain
  double tau[kRateUnroll];
  T acc[kRateUnroll];
#pragma unroll
  for (int u = 0; u < kRateUnroll; ++u) {
    tau[u] = span * __builtin_amdgcn_fract((double)(t * kRateUnroll + u) * 0.7548776662466927);
    acc[u] = T{0, 0};
  }
  for (int64_t k = 0; k < iters; k += kRateUnroll) {
#pragma unroll
    for (int u = 0; u < kRateUnroll; ++u) {
      const T e = cis<Real>(tau[u]);
      acc[u].x += e.x;
      acc[u].y += e.y;
      tau[u] += step;
    }
  }
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < kRateUnroll; ++u) {
    s.x += (double)acc[u].x;
    s.y += (double)acc[u].y;
  }
  out[t] = s;
}

// Contraction-unit microkernel: the rate of FP32 multiply-adds on the VALU
// (v_fma_f32, 32 independent chains per lane) and on the matrix cores
// (v_mfma_f32_4x4x1_16b_f32: 16 blocks of a 4x4 outer product per wave, 8
// independent accumulators per wave), alone and interleaved in one
// instruction stream.  This is the choice between the two units for the
// interpolation contractions: the 16-block 4x4x1 form is the one that maps
// a lane's line of values to its own outputs (lane 4b + j supplies column j
// of block b and receives rows 0..3 of it), so a line job could move its
// q x q transforms onto it without moving data between lanes.
typedef float v4f __attribute__((ext_vector_type(4)));
template <int NM, int NV>
__global__ __launch_bounds__(kRateThreads) void k_contraction_rate(int64_t n, int64_t iters, float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * kRateThreads + threadIdx.x;
  if (t >= n) return;
  const float a = 1.0f + 1e-7f * (float)(t & 7), b = 1.0f - 1e-7f * (float)(t & 3);
  v4f acc[NM > 0 ? NM : 1];
  float f[NV > 0 ? NV : 1];
#pragma unroll
  for (int i = 0; i < (NM > 0 ? NM : 1); ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < (NV > 0 ? NV : 1); ++i) f[i] = (float)i;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < NM; ++i) acc[i] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc[i], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < NV; ++i) f[i] = fmaf(f[i], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < (NM > 0 ? NM : 1); ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
#pragma unroll
  for (int i = 0; i < (NV > 0 ? NV : 1); ++i) s += f[i];
  out[t] = s;
}

}  // namespace
}  // namespace fz
}  // namespace bfly

extern "C" int bfly_contraction_rate(int unit, int64_t n_threads, int64_t iters, void* out, void* stream) {
  if (unit < 0 || unit > 2 || n_threads < 1 || n_threads > ((int64_t)1 << 30) || iters < 1 || !out)
    return BFLY_EINVAL;
  if (n_threads % 64 != 0) return BFLY_EINVAL;  // whole waves (the matrix instruction is wave-wide)
  const unsigned blocks = (unsigned)((n_threads + bfly::fz::kRateThreads - 1) / bfly::fz::kRateThreads);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  float* o = static_cast<float*>(out);
  if (unit == 0)
    bfly::fz::k_contraction_rate<0, 32><<<blocks, bfly::fz::kRateThreads, 0, st>>>(n_threads, iters, o);
  else if (unit == 1)
    bfly::fz::k_contraction_rate<8, 0><<<blocks, bfly::fz::kRateThreads, 0, st>>>(n_threads, iters, o);
  else
    bfly::fz::k_contraction_rate<8, 32><<<blocks, bfly::fz::kRateThreads, 0, st>>>(n_threads, iters, o);
  return hipGetLastError() == hipSuccess ? BFLY_OK : BFLY_EDEVICE;
}

extern "C" int bfly_phase_rate(int prec, int64_t n_threads, int64_t iters, double span, void* out, void* stream) {
  if (prec != BFLY_FP64 && prec != BFLY_FP32) return BFLY_EINVAL;
  if (n_threads < 1 || n_threads > ((int64_t)1 << 30) || iters < 1 || iters % bfly::fz::kRateUnroll != 0 ||
      !(span >= 0.0 && span < 1e15) || !out)
    return BFLY_EINVAL;
  const unsigned blocks = (unsigned)((n_threads + bfly::fz::kRateThreads - 1) / bfly::fz::kRateThreads);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (prec == BFLY_FP64)
    bfly::fz::k_phase_rate<double><<<blocks, bfly::fz::kRateThreads, 0, st>>>(n_threads, iters, span,
                                                                                static_cast<double2*>(out));
  else
    bfly::fz::k_phase_rate<float><<<blocks, bfly::fz::kRateThreads, 0, st>>>(n_threads, iters, span,
                                                                               static_cast<double2*>(out));
  return hipGetLastError() == hipSuccess ? BFLY_OK : BFLY_EDEVICE;
}
