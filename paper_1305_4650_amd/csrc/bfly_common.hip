// Binning of the input points into source leaves, workspace helpers, and the
// dispatch of one apply to the fused level kernels (bfly_fused.inc).
//
// Steps of one apply (Alg. "alg:serial" of Poulson, Demanet, Maxwell & Ying,
// with the analytic Chebyshev translations of Sec. 1.4 "Avoiding quadratic
// precomputation"):
//   binning      leaf of every input point (level-0 source tree), stable sort
//                by leaf Morton index, CSR offsets per leaf      (this file)
//   k_first      leaf initialisation w_XB := V_XB g_B (Sec. 1), the
//                column-space merge-and-split stages (Sec. 1.1) and the
//                middle switch                                 (bfly_fused.inc)
//   k_second     row-space merge-and-split stages             (bfly_fused.inc)
//   k_final      f_AY := U_AY w_AY at every target (Sec. 1)     (bfly_fused.inc)
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cstdlib>

#include "bfly_internal.h"

namespace bfly {
namespace {

constexpr int kBlock = 256;

// Radix sort of the leaf keys: rocPRIM's onesweep algorithm above 64 Ki
// points (its default switches from merge sort only above 1 Mi; on MI355X
// the whole binning of 1 Mi points with 20-bit keys takes 0.13 ms this way,
// 0.16 ms with the ~20 merge passes).  The same configuration sizes the
// scratch in sort_storage_bytes.
using SortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                              rocprim::default_config, 65536>;

// leaf index along one dimension: floor((v - lo) / extent * n), clamped to
// [0, n-1]; NaN goes to 0
__device__ __forceinline__ int64_t bin1(double v, double lo, double ext, int64_t n) {
  const double u = ((v - lo) / ext) * (double)n;
  if (!(u >= 0.0)) return 0;
  if (u >= (double)n) return n - 1;
  const int64_t b = (int64_t)floor(u);
  return b > n - 1 ? n - 1 : b;
}

// Morton key of a level-0 source leaf (finest digit lowest)
template <int D>
__device__ __forceinline__ uint32_t morton(const int64_t* b, int ndig) {
  uint32_t m = 0;
  for (int k = 0; k < ndig; ++k)
#pragma unroll
    for (int j = 0; j < D; ++j) m |= (uint32_t)((b[j] >> k) & 1) << (D * k + j);
  return m;
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_bin(const Geo G, int64_t n, const double* __restrict__ pts,
                                                uint32_t* __restrict__ keys, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t b[3];
  const int64_t N = (int64_t)1 << G.L;
#pragma unroll
  for (int j = 0; j < D; ++j) b[j] = bin1(pts[i * D + j], G.slo[j], G.sD[j], N);
  keys[i] = morton<D>(b, G.L);
  idx[i] = (int32_t)i;
}

// offs[m] = first sorted position whose key is >= m, for m = 0..P
__global__ __launch_bounds__(kBlock) void k_offsets(int64_t n, int64_t P, const uint32_t* __restrict__ ks,
                                                    int32_t* __restrict__ offs) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n == 0) {
    for (int64_t m = k; m <= P; m += (int64_t)gridDim.x * blockDim.x) offs[m] = 0;
    return;
  }
  if (k >= n) return;
  const int64_t prev = k == 0 ? -1 : (int64_t)ks[k - 1];
  const int64_t cur = ks[k];
  for (int64_t m = prev + 1; m <= cur; ++m) offs[m] = (int32_t)k;
  if (k == n - 1)
    for (int64_t m = cur + 1; m <= P; ++m) offs[m] = (int32_t)n;
}

// N = 1: every point is in the single leaf
__global__ __launch_bounds__(kBlock) void k_iota(int64_t n, int32_t* __restrict__ perm,
                                                 uint32_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    perm[i] = (int32_t)i;
    keys[i] = 0u;
  }
}

inline unsigned blocks_for(int64_t n, int bs = kBlock) { return (unsigned)((n + bs - 1) / bs); }

template <int D>
hipError_t bin_sources(const Geo& G, int64_t n_in, const double* pts_in, const Work& w, hipStream_t st) {
  const int64_t P = (int64_t)1 << (D * G.L);
  StepTimer tb(kStepBin, st);
  if (n_in > 0) {
    k_bin<D><<<blocks_for(n_in), kBlock, 0, st>>>(G, n_in, pts_in, w.keys, w.idx);
    if (D * G.L > 0) {
      size_t tmp = w.sort_tmp_bytes;
      const hipError_t e = rocprim::radix_sort_pairs<SortConfig>(w.sort_tmp, tmp, w.keys, w.keys_sorted, w.idx, w.perm,
                                                     (unsigned)n_in, 0, D * G.L, st);
      if (e != hipSuccess) return e;
    } else {
      k_iota<<<blocks_for(n_in), kBlock, 0, st>>>(n_in, w.perm, w.keys_sorted);
    }
    k_offsets<<<blocks_for(n_in), kBlock, 0, st>>>(n_in, P, w.keys_sorted, w.offs);
  } else {
    k_offsets<<<blocks_for(P + 1), kBlock, 0, st>>>(0, P, nullptr, w.offs);
  }
  return hipGetLastError();
}

// Launch-shape overrides for tuning sweeps: BFLY_UB (fusion units per
// block), BFLY_KFUSE (stages per launch), BFLY_LDS (LDS budget in bytes).
void tune_from_env(LevelArgs& la) {
  static const int ub = [] { const char* v = getenv("BFLY_UB"); return v ? atoi(v) : 0; }();
  static const int kf = [] { const char* v = getenv("BFLY_KFUSE"); return v ? atoi(v) : 0; }();
  static const int lds = [] { const char* v = getenv("BFLY_LDS"); return v ? atoi(v) : 0; }();
  if (ub >= 1 && ub <= 64) la.ub_force = ub;
  if (kf >= 1 && kf <= 8) la.k_fuse = kf;
  if (lds >= 16384 && lds <= 163840) la.lds_budget = (size_t)lds;
}

}  // namespace

size_t weight_bytes(const Geo& g, int nrhs, int prec) {
  const size_t P = (size_t)1 << (g.d * g.L);
  return P * (size_t)g.r * (size_t)nrhs * (prec == 0 ? sizeof(double2) : sizeof(float2));
}

hipError_t sort_storage_bytes(int64_t n, int bits, size_t* bytes) {
  *bytes = 0;
  if (n <= 0 || bits <= 0) return hipSuccess;
  return rocprim::radix_sort_pairs<SortConfig>(nullptr, *bytes, (uint32_t*)nullptr, (uint32_t*)nullptr, (int32_t*)nullptr,
                                   (int32_t*)nullptr, (unsigned)n, 0, bits, (hipStream_t)0);
}

hipError_t run_apply(const Geo& g, int prec, int64_t n_in, const double* pts_in, const double* vals_in,
                     int64_t ld_in, int64_t n_out, const double* pts_out, double* vals_out, int64_t ld_out,
                     int nrhs, const Work& w, hipStream_t st) {
  const hipError_t e = g.d == 1 ? bin_sources<1>(g, n_in, pts_in, w, st)
                                : (g.d == 2 ? bin_sources<2>(g, n_in, pts_in, w, st)
                                            : bin_sources<3>(g, n_in, pts_in, w, st));
  if (e != hipSuccess) return e;
  LevelArgs la;
  la.G = &g;
  la.W = w.W;
  la.nrhs = nrhs;
  la.pts_in = pts_in;
  la.vals_in = vals_in;
  la.ld_in = ld_in;
  la.perm = w.perm;
  la.offs = w.offs;
  la.n_out = n_out;
  la.pts_out = pts_out;
  la.vals_out = vals_out;
  la.ld_out = ld_out;
  la.stream = st;
  tune_from_env(la);
  switch (g.d) {
    case 1:
      return run_levels_d1(la, prec);
    case 2:
      return run_levels_d2(la, prec);
    default:
      return run_levels_d3(la, prec);
  }
}

}  // namespace bfly
