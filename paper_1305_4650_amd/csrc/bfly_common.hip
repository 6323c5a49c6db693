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

// Sort of the leaf keys (stable, so both configurations give the same
// permutation): rocPRIM's radix_sort_pairs with its onesweep algorithm
// above 64 Ki keys when the stream is not being captured, and restricted to
// its merge sort when it is (onesweep clears scratch with hipMemsetAsync,
// and memset nodes in a captured graph are avoided here; the merge sort
// launches kernels only).  MI355X, 1 Mi 20-bit keys: the whole binning takes
// 0.13 ms with onesweep, 0.16 ms with the merge sort.
using SortFast = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                            rocprim::default_config, 65536>;
using SortMerge = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                             rocprim::default_config, ~size_t(0)>;

hipError_t sort_pairs(void* tmp, size_t tmp_bytes, const uint32_t* keys, uint32_t* keys_out, const int32_t* vals,
                      int32_t* vals_out, unsigned n, int bits, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return e;
  size_t b = tmp_bytes;
  if (cs == hipStreamCaptureStatusNone)
    return rocprim::radix_sort_pairs<SortFast>(tmp, b, keys, keys_out, vals, vals_out, n, 0, bits, st);
  return rocprim::radix_sort_pairs<SortMerge>(tmp, b, keys, keys_out, vals, vals_out, n, 0, bits, st);
}

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
      const hipError_t e =
          sort_pairs(w.sort_tmp, w.sort_tmp_bytes, w.keys, w.keys_sorted, w.idx, w.perm, (unsigned)n_in, D * G.L, st);
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

// ---- batched binning: all instances' points in one sort ----
struct BinItem {
  const double* pts;
  int64_t n, pbase;   // points, and the first global index of this instance
  uint32_t leafbase;
  int d, L;
  double slo[3], sD[3];
};
constexpr int kBinItems = 16;
struct BinArgs {
  int n;
  BinItem it[kBinItems];
};

__global__ __launch_bounds__(kBlock) void k_bin_batch(const BinArgs a, int64_t g0, int64_t g1,
                                                      uint32_t* __restrict__ keys, int32_t* __restrict__ idx) {
  const int64_t g = g0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= g1) return;
  int k = 0;
  while (k + 1 < a.n && a.it[k + 1].pbase <= g) ++k;
  const BinItem& it = a.it[k];
  const int64_t j = g - it.pbase;
  const int64_t N = (int64_t)1 << it.L;
  int64_t b[3] = {0, 0, 0};
  for (int i = 0; i < it.d; ++i) b[i] = bin1(it.pts[j * it.d + i], it.slo[i], it.sD[i], N);
  uint32_t m = 0;
  for (int l = 0; l < it.L; ++l)
    for (int i = 0; i < it.d; ++i) m |= (uint32_t)((b[i] >> l) & 1) << (it.d * l + i);
  keys[g] = it.leafbase + m;
  idx[g] = (int32_t)j;
}

// descriptors travel in kernel arguments, kPutItems at a time
constexpr int kPutItems = 8;
struct PutArgs {
  int n;
  ItemDesc d[kPutItems];
};
__global__ void k_put_items(const PutArgs a, ItemDesc* __restrict__ dst) {
  constexpr int words = (int)(sizeof(ItemDesc) / sizeof(uint32_t));
  static_assert(sizeof(ItemDesc) % sizeof(uint32_t) == 0, "descriptor size");
  for (int k = 0; k < a.n; ++k) {
    const uint32_t* s = reinterpret_cast<const uint32_t*>(&a.d[k]);
    uint32_t* o = reinterpret_cast<uint32_t*>(dst + k);
    for (int w = threadIdx.x; w < words; w += blockDim.x) o[w] = s[w];
  }
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

hipError_t put_items(ItemDesc* dst, const ItemDesc* src, int n, hipStream_t st) {
  for (int k0 = 0; k0 < n; k0 += kPutItems) {
    PutArgs a;
    a.n = std::min(kPutItems, n - k0);
    for (int k = 0; k < a.n; ++k) a.d[k] = src[k0 + k];
    k_put_items<<<1, 128, 0, st>>>(a, dst + k0);
  }
  return hipGetLastError();
}

hipError_t bin_batch(const BinInst* bi, int n, int64_t n_total, uint64_t leaves_total, const Work& w,
                     hipStream_t st) {
  StepTimer tb(kStepBin, st);
  int64_t pbase = 0;
  for (int k0 = 0; k0 < n; k0 += kBinItems) {
    BinArgs a;
    a.n = std::min(kBinItems, n - k0);
    const int64_t g0 = pbase;
    for (int k = 0; k < a.n; ++k) {
      const BinInst& b = bi[k0 + k];
      BinItem& it = a.it[k];
      it.pts = b.pts;
      it.n = b.n;
      it.pbase = pbase;
      it.leafbase = b.leafbase;
      it.d = b.G->d;
      it.L = b.G->L;
      for (int i = 0; i < 3; ++i) {
        it.slo[i] = b.G->slo[i];
        it.sD[i] = b.G->sD[i];
      }
      pbase += b.n;
    }
    if (pbase > g0) k_bin_batch<<<blocks_for(pbase - g0), kBlock, 0, st>>>(a, g0, pbase, w.keys, w.idx);
  }
  if (n_total > 0) {
    int bits = 0;
    while (bits < 32 && ((uint64_t)1 << bits) < leaves_total) ++bits;
    if (bits > 0) {
      const hipError_t e =
          sort_pairs(w.sort_tmp, w.sort_tmp_bytes, w.keys, w.keys_sorted, w.idx, w.perm, (unsigned)n_total, bits, st);
      if (e != hipSuccess) return e;
    } else {
      k_iota<<<blocks_for(n_total), kBlock, 0, st>>>(n_total, w.perm, w.keys_sorted);
    }
    k_offsets<<<blocks_for(n_total), kBlock, 0, st>>>(n_total, (int64_t)leaves_total, w.keys_sorted, w.offs);
  } else {
    k_offsets<<<blocks_for((int64_t)leaves_total + 1), kBlock, 0, st>>>(0, (int64_t)leaves_total, nullptr, w.offs);
  }
  return hipGetLastError();
}

void tune_batch_from_env(BatchGroup& bg) {
  LevelArgs la;
  tune_from_env(la);
  bg.k_fuse = la.k_fuse;
  bg.lds_budget = la.lds_budget;
  bg.ub_force = la.ub_force;
}

size_t weight_bytes(const Geo& g, int nrhs, int prec) {
  const size_t P = (size_t)1 << (g.d * g.L);
  return P * (size_t)g.r * (size_t)nrhs * (prec == 0 ? sizeof(double2) : sizeof(float2));
}

hipError_t sort_storage_bytes(int64_t n, int bits, size_t* bytes) {
  *bytes = 0;
  if (n <= 0 || bits <= 0) return hipSuccess;
  size_t fast = 0, merge = 0;
  hipError_t e = rocprim::radix_sort_pairs<SortFast>(nullptr, fast, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                                     (int32_t*)nullptr, (int32_t*)nullptr, (unsigned)n, 0, bits,
                                                     (hipStream_t)0);
  if (e != hipSuccess) return e;
  e = rocprim::radix_sort_pairs<SortMerge>(nullptr, merge, (uint32_t*)nullptr, (uint32_t*)nullptr, (int32_t*)nullptr,
                                           (int32_t*)nullptr, (unsigned)n, 0, bits, (hipStream_t)0);
  *bytes = std::max(fast, merge);
  return e;
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
