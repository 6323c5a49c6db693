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
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "bfly_internal.h"

namespace bfly {
namespace {

constexpr int kBlock = 256;

// ---- stable LSD radix sort of the 32-bit leaf keys with int32 payloads ----
// Passes go from the lowest digit (at most kMaxDigit bits) up; each pass is a
// stable counting sort by its digit, so the passes together give the stable
// sort by the whole key.  A pass is three launches:
//   k_digit_hist     digit counts of every tile of 256 KPT keys, stored
//                    digit-major: cnt[digit * ntile + tile]
//   k_digit_scan     exclusive prefix of each digit's row over the tiles (in
//                    place) and the row total tot[digit]
//   k_digit_scatter  stable rank of each key inside its tile (wave by wave,
//                    64 keys at a time, lanes of equal digit found by one
//                    ballot per digit bit), then the write to
//                    sum(tot below its digit) + row prefix + rank
// Kernels only (no memset), so a captured graph records launches alone; the
// permutation is the same on every run.
constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kMaxDigit = 11;

// Keys per thread (KPT) of the histogram and scatter kernels, from n alone
// (so workspace queries and applies agree): 16 for large sorts (fewer tiles,
// shorter count rows); small sorts take fewer, since a tile ranks its keys
// 64 at a time in a serial loop and more, shorter tiles run side by side.
inline int sort_kpt(int64_t n) { return n > (1 << 18) ? 16 : n > (1 << 14) ? 8 : 2; }

struct SortPlan {
  int passes = 0, width[3] = {0, 0, 0}, shift[3] = {0, 0, 0}, maxw = 0;
  int ntile = 0, kpt = 0;
};

SortPlan sort_plan(int64_t n, int bits) {
  SortPlan s;
  if (n <= 0 || bits <= 0) return s;
  s.passes = (bits + kMaxDigit - 1) / kMaxDigit;
  int sh = 0;
  for (int p = 0; p < s.passes; ++p) {
    s.width[p] = bits / s.passes + (p < bits % s.passes ? 1 : 0);
    s.shift[p] = sh;
    sh += s.width[p];
    s.maxw = std::max(s.maxw, s.width[p]);
  }
  s.kpt = sort_kpt(n);
  const int64_t tile = (int64_t)kSortThreads * s.kpt;
  s.ntile = (int)((n + tile - 1) / tile);
  return s;
}

inline size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// scratch: cnt [2^maxw][ntile], tot [2^maxw], and with two passes or more a
// second key / payload buffer for the passes to alternate with the output
size_t sort_bytes(const SortPlan& s, int64_t n) {
  if (s.passes == 0) return 0;
  const size_t B = (size_t)1 << s.maxw;
  size_t b = up256(4 * B * (size_t)s.ntile) + up256(4 * B);
  if (s.passes > 1) b += 2 * up256(4 * (size_t)n);
  return b;
}

template <int KPT>
__global__ __launch_bounds__(kSortThreads) void k_digit_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                             int nb, int ntile, int32_t* __restrict__ cnt) {
  __shared__ int32_t h[1 << kMaxDigit];
  const int B = 1 << nb;
  for (int i = threadIdx.x; i < B; i += kSortThreads) h[i] = 0;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t e0 = (int64_t)blockIdx.x * (kSortThreads * KPT) + (int64_t)w * 64 * KPT + lane;
  uint32_t k[KPT];
#pragma unroll
  for (int c = 0; c < KPT; ++c) {
    const int64_t e = e0 + c * 64;
    k[c] = e < n ? keys[e] : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < KPT; ++c)
    if (e0 + c * 64 < n) atomicAdd(&h[(k[c] >> shift) & (uint32_t)(B - 1)], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < B; i += kSortThreads) cnt[(int64_t)i * ntile + blockIdx.x] = h[i];
}

// one wave per digit; a lane takes 8 consecutive tiles of the row at a time
__global__ __launch_bounds__(kSortThreads) void k_digit_scan(int nb, int ntile, int32_t* __restrict__ cnt,
                                                             int32_t* __restrict__ tot) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int dig = blockIdx.x * kSortWaves + w;
  if (dig >= (1 << nb)) return;
  int32_t* row = cnt + (int64_t)dig * ntile;
  int32_t carry = 0;
  for (int t0 = 0; t0 < ntile; t0 += 64 * 8) {
    const int b = t0 + lane * 8;
    int32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = b + j < ntile ? row[b + j] : 0;
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int32_t x = v[j];
      v[j] = s;
      s += x;
    }
    int32_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    const int32_t ex = carry + incl - s;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (b + j < ntile) row[b + j] = ex + v[j];
    carry += __shfl(incl, 63);
  }
  if (lane == 0) tot[dig] = carry;
}

// vals == nullptr: the payload of key e is e
template <int KPT>
__global__ __launch_bounds__(kSortThreads) void k_digit_scatter(const uint32_t* __restrict__ keys,
                                                                const int32_t* __restrict__ vals, int64_t n, int shift,
                                                                int nb, int ntile, const int32_t* __restrict__ cnt,
                                                                const int32_t* __restrict__ tot,
                                                                uint32_t* __restrict__ keys_out,
                                                                int32_t* __restrict__ vals_out) {
  __shared__ int32_t h[kSortWaves][1 << kMaxDigit];
  __shared__ int32_t part[kSortWaves];
  const int B = 1 << nb;
  const uint32_t mask = (uint32_t)(B - 1);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t e0 = (int64_t)blockIdx.x * (kSortThreads * KPT) + (int64_t)w * 64 * KPT + lane;
  uint32_t k[KPT];
  int32_t v[KPT];
#pragma unroll
  for (int c = 0; c < KPT; ++c) {
    const int64_t e = e0 + c * 64;
    k[c] = e < n ? keys[e] : 0u;
    v[c] = e < n ? (vals ? vals[e] : (int32_t)e) : 0;
  }
  // every wave counts its own 64 KPT keys in its own row of h
  for (int i = lane; i < B; i += 64) h[w][i] = 0;
  const uint64_t lower = (1ull << lane) - 1ull;
  int32_t r[KPT];
#pragma unroll
  for (int c = 0; c < KPT; ++c) {
    const bool ok = e0 + c * 64 < n;
    const uint32_t d = (k[c] >> shift) & mask;
    uint64_t peers = __ballot(ok);
    for (int b = 0; b < nb; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t set = __ballot(bit);
      peers &= bit ? set : ~set;
    }
    r[c] = 0;
    if (ok) {
      // all lanes of the digit read the count before the lowest of them
      // (the leader) adds the group's size: one wave, LDS in program order
      const int32_t before = h[w][d];
      r[c] = before + __popcll(peers & lower);
      if ((peers & lower) == 0ull) h[w][d] = before + __popcll(peers);
    }
  }
  // digit bases: tot summed below the digit + this tile's row prefix, and
  // per wave the counts of the waves before it
  const int per = (B + kSortThreads - 1) / kSortThreads;
  const int d0 = threadIdx.x * per;
  int32_t s = 0;
  for (int j = 0; j < per; ++j)
    if (d0 + j < B) s += tot[d0 + j];
  int32_t incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) part[w] = incl;
  __syncthreads();
  int32_t base = incl - s;
  for (int ww = 0; ww < w; ++ww) base += part[ww];
  for (int j = 0; j < per; ++j) {
    const int dd = d0 + j;
    if (dd < B) {
      int32_t acc = base + cnt[(int64_t)dd * ntile + blockIdx.x];
      base += tot[dd];
#pragma unroll
      for (int ww = 0; ww < kSortWaves; ++ww) {
        const int32_t x = h[ww][dd];
        h[ww][dd] = acc;
        acc += x;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < KPT; ++c) {
    if (e0 + c * 64 < n) {
      const int64_t dst = (int64_t)h[w][(k[c] >> shift) & mask] + r[c];
      if (dst >= 0 && dst < n) {
        keys_out[dst] = k[c];
        vals_out[dst] = v[c];
      }
    }
  }
}

template <int KPT>
void sort_pass(const SortPlan& s, int pass, const uint32_t* kin, const int32_t* vin, int64_t n, int32_t* cnt,
               int32_t* tot, uint32_t* ko, int32_t* vo, hipStream_t st) {
  const int nb = s.width[pass];
  k_digit_hist<KPT><<<s.ntile, kSortThreads, 0, st>>>(kin, n, s.shift[pass], nb, s.ntile, cnt);
  k_digit_scan<<<((1 << nb) + kSortWaves - 1) / kSortWaves, kSortThreads, 0, st>>>(nb, s.ntile, cnt, tot);
  k_digit_scatter<KPT><<<s.ntile, kSortThreads, 0, st>>>(kin, vin, n, s.shift[pass], nb, s.ntile, cnt, tot, ko, vo);
}

// Stable sort of (keys, vals) by the low `bits` bits of the keys into
// (keys_out, vals_out); vals == nullptr stands for vals[e] = e.  n >= 1,
// 1 <= bits <= 32, tmp of sort_bytes(sort_plan(n, bits), n) bytes.
hipError_t radix_sort(const uint32_t* keys, const int32_t* vals, int64_t n, int bits, uint32_t* keys_out,
                      int32_t* vals_out, void* tmp, size_t tmp_bytes, hipStream_t st) {
  const SortPlan s = sort_plan(n, bits);
  if (s.passes == 0 || tmp_bytes < sort_bytes(s, n)) return hipErrorInvalidValue;
  const size_t B = (size_t)1 << s.maxw;
  char* p = static_cast<char*>(tmp);
  int32_t* cnt = reinterpret_cast<int32_t*>(p);
  p += up256(4 * B * (size_t)s.ntile);
  int32_t* tot = reinterpret_cast<int32_t*>(p);
  p += up256(4 * B);
  uint32_t* k_alt = reinterpret_cast<uint32_t*>(p);
  int32_t* v_alt = reinterpret_cast<int32_t*>(p + up256(4 * (size_t)n));
  const uint32_t* kin = keys;
  const int32_t* vin = vals;
  for (int pass = 0; pass < s.passes; ++pass) {
    // the last pass writes the output; earlier ones alternate with it
    const bool to_out = ((s.passes - 1 - pass) & 1) == 0;
    uint32_t* ko = to_out ? keys_out : k_alt;
    int32_t* vo = to_out ? vals_out : v_alt;
    if (s.kpt == 16)
      sort_pass<16>(s, pass, kin, vin, n, cnt, tot, ko, vo, st);
    else if (s.kpt == 8)
      sort_pass<8>(s, pass, kin, vin, n, cnt, tot, ko, vo, st);
    else
      sort_pass<2>(s, pass, kin, vin, n, cnt, tot, ko, vo, st);
    kin = ko;
    vin = vo;
  }
  return hipGetLastError();
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
                                                uint32_t* __restrict__ keys, int32_t* __restrict__ empty) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *empty = 0;  // k_offsets, launched after this kernel, sets it for an empty leaf
  if (i >= n) return;
  int64_t b[3];
  const int64_t N = (int64_t)1 << G.L;
#pragma unroll
  for (int j = 0; j < D; ++j) b[j] = bin1(pts[i * D + j], G.slo[j], G.sD[j], N);
  keys[i] = morton<D>(b, G.L);
}

// offs[m] = first sorted position whose key is >= m, for m = 0..P: one
// thread per m.  The search starts at m n / P (exact when every leaf holds
// one point), gallops away from it and finishes by bisection, so a leaf costs
// O(1) loads for evenly spread points and O(log n) however sparse they are.
// A leaf m < P without points (its first key >= m is not m) sets *empty = 1
// (with no points at all every leaf does, the flag needing no clearing).
__global__ __launch_bounds__(kBlock) void k_offsets(int64_t n, int64_t P, const uint32_t* __restrict__ ks,
                                                    int32_t* __restrict__ offs, int32_t* __restrict__ empty) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m > P) return;
  const int64_t g = P > 0 ? m * n / P : 0;  // m <= 2^30, n < 2^31: no overflow
  int64_t lo, hi;
  if (g < n && (int64_t)ks[g] < m) {  // the answer lies above g
    lo = g + 1;
    hi = n;
    for (int64_t step = 1;; step <<= 1) {
      const int64_t p = lo + step - 1;
      if (p >= n) break;
      if ((int64_t)ks[p] >= m) {
        hi = p;
        break;
      }
      lo = p + 1;
    }
  } else {  // the answer is at most g (g = n included)
    hi = g < n ? g : n;
    lo = 0;
    for (int64_t step = 1;; step <<= 1) {
      const int64_t p = hi - step;
      if (p < 0) break;
      if ((int64_t)ks[p] < m) {
        lo = p + 1;
        break;
      }
      hi = p;
    }
  }
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)ks[mid] < m)
      lo = mid + 1;
    else
      hi = mid;
  }
  offs[m] = (int32_t)lo;
  if (m < P && (lo == n || (int64_t)ks[lo] != m)) *empty = 1;
}

// ---- target-box occupancy (sparse targets) ----
__host__ __device__ inline int64_t tocc_base(int D, int l) { return (((int64_t)1 << (D * l)) - 1) / ((1 << D) - 1); }

__global__ __launch_bounds__(kBlock) void k_zero_words(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// every target marks the boxes that contain it on every level 0..L (its
// leaf as the final evaluation computes it)
template <int D>
__global__ __launch_bounds__(kBlock) void k_mark_targets(const Geo G, int64_t n, const double* __restrict__ pts,
                                                         uint8_t* __restrict__ occ) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t N = (int64_t)1 << G.L;
  int64_t b[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double u = ((pts[i * D + d] - G.tlo[d]) / G.tD[d]) * (double)N;
    int64_t v = 0;
    if (u >= 0.0) v = u >= (double)N ? N - 1 : (int64_t)floor(u);
    b[d] = v > N - 1 ? N - 1 : v;
  }
  for (int l = 0; l <= G.L; ++l) {
    uint32_t m = 0;
    for (int k = 0; k < l; ++k)
#pragma unroll
      for (int d = 0; d < D; ++d) m |= (uint32_t)(((b[d] >> (G.L - l)) >> k) & 1) << (D * k + d);
    occ[tocc_base(D, l) + m] = 1;
  }
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
    k_bin<D><<<blocks_for(n_in), kBlock, 0, st>>>(G, n_in, pts_in, w.keys, w.empty);
    if (D * G.L > 0) {
      const hipError_t e =
          radix_sort(w.keys, nullptr, n_in, D * G.L, w.keys_sorted, w.perm, w.sort_tmp, w.sort_tmp_bytes, st);
      if (e != hipSuccess) return e;
    } else {
      k_iota<<<blocks_for(n_in), kBlock, 0, st>>>(n_in, w.perm, w.keys_sorted);
    }
  }
  k_offsets<<<blocks_for(P + 1), kBlock, 0, st>>>(n_in, P, w.keys_sorted, w.offs, w.empty);
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
                                                      uint32_t* __restrict__ keys, int32_t* __restrict__ idx,
                                                      int32_t* __restrict__ empty) {
  const int64_t g = g0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) *empty = 0;  // k_offsets, launched after this kernel, sets it for an empty leaf
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
  // BFLY_KSPLIT=a,b,...: stages per launch for a tuning sweep
  static const std::vector<int> split = [] {
    std::vector<int> v;
    const char* e = getenv("BFLY_KSPLIT");
    for (const char* c = e; c && *c;) {
      const int k = atoi(c);
      if (k < 1 || k > 8 || v.size() >= 16) return std::vector<int>();
      v.push_back(k);
      c = strchr(c, ',');
      if (c) ++c;
    }
    return v;
  }();
  if (!split.empty()) {
    la.nsplit = (int)split.size();
    for (int i = 0; i < la.nsplit; ++i) la.split[i] = split[i];
  }
  // BFLY_STOP_STAGES=n: stop after the launches that end within n stages
  // (tests compare that level's weights with the oracle's)
  static const int stop = [] {
    const char* v = getenv("BFLY_STOP_STAGES");
    return v ? atoi(v) : -1;
  }();
  if (stop >= 0) la.stop_stages = stop;
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
    if (pbase > g0) k_bin_batch<<<blocks_for(pbase - g0), kBlock, 0, st>>>(a, g0, pbase, w.keys, w.idx, w.empty);
  }
  if (n_total > 0) {
    int bits = 0;
    while (bits < 32 && ((uint64_t)1 << bits) < leaves_total) ++bits;
    if (bits > 0) {
      const hipError_t e =
          radix_sort(w.keys, w.idx, n_total, bits, w.keys_sorted, w.perm, w.sort_tmp, w.sort_tmp_bytes, st);
      if (e != hipSuccess) return e;
    } else {
      k_iota<<<blocks_for(n_total), kBlock, 0, st>>>(n_total, w.perm, w.keys_sorted);
    }
  }
  k_offsets<<<blocks_for((int64_t)leaves_total + 1), kBlock, 0, st>>>(n_total, (int64_t)leaves_total,
                                                                      w.keys_sorted, w.offs, w.empty);
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
  *bytes = sort_bytes(sort_plan(n, bits), n);
  return hipSuccess;
}

size_t tocc_bytes(int d, int L) {
  const size_t b = (size_t)tocc_base(d, L + 1);
  return (b + 3) & ~(size_t)3;
}

hipError_t shape_limits(const Geo& g, int prec, ShapeLimits* out) {
  return g.d == 1 ? shape_limits_d1(g, prec, out)
                  : (g.d == 2 ? shape_limits_d2(g, prec, out) : shape_limits_d3(g, prec, out));
}

hipError_t run_apply(const Geo& g, int prec, int64_t n_in, const double* pts_in, const double* vals_in,
                     int64_t ld_in, int64_t n_out, const double* pts_out, double* vals_out, int64_t ld_out,
                     int nrhs, const Work& w, hipStream_t st, const TuneParams* force) {
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
  la.empty = w.empty;
  // fewer targets than leaves: some target boxes are empty on the last
  // levels, and the level kernels skip units whose target box is empty
  const int64_t P = (int64_t)1 << (g.d * g.L);
  if (n_out < P && w.tocc) {
    const int64_t words = (int64_t)(tocc_bytes(g.d, g.L) / 4);
    k_zero_words<<<(unsigned)std::min<int64_t>(blocks_for(words), 4096), kBlock, 0, st>>>(
        reinterpret_cast<uint32_t*>(w.tocc), words);
    if (n_out > 0) {
      if (g.d == 1)
        k_mark_targets<1><<<blocks_for(n_out), kBlock, 0, st>>>(g, n_out, pts_out, w.tocc);
      else if (g.d == 2)
        k_mark_targets<2><<<blocks_for(n_out), kBlock, 0, st>>>(g, n_out, pts_out, w.tocc);
      else
        k_mark_targets<3><<<blocks_for(n_out), kBlock, 0, st>>>(g, n_out, pts_out, w.tocc);
    }
    la.tocc = w.tocc;
  }
  la.n_out = n_out;
  la.pts_out = pts_out;
  la.vals_out = vals_out;
  la.ld_out = ld_out;
  la.stream = st;
  TuneParams tp;
  if (force || tune_lookup(g, nrhs, prec, &tp)) {
    const TuneParams& t = force ? *force : tp;
    la.ub_first = t.ub_first;
    la.ub_second = t.ub_second;
    la.rc_one = t.rc_one;
    la.nsplit = std::min(t.nsplit, 16);
    for (int i = 0; i < la.nsplit; ++i) la.split[i] = t.split[i];
  }
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
