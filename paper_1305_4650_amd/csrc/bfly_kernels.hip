// HIP kernels of the butterfly apply for gfx950 (wave64, CDNA4).
//
// Steps (Alg. "alg:serial" of Poulson, Demanet, Maxwell & Ying, with the
// analytic Chebyshev translations of Sec. 2 "Avoiding quadratic
// precomputation"):
//   k_bin/sort/k_offsets  leaf of every input point, stable CSR grouping
//   k_init                w_XB := V_XB g_B                       (Sec. 1)
//   k_stage_src           first-half merge-and-split (Sec. 1.1), column-space
//   k_switch              middle switch at level floor(L/2)      (Sec. 2)
//   k_stage_tgt           second-half merge-and-split, row-space
//   k_final               f_AY := U_AY w_AY at every target      (Sec. 1)
//
// Weight layout (in place across all levels).  The N^d (A,B) pairs of every
// level live in N^d slots of r * nrhs complex values.  Viewing a slot index
// as L digits of d bits, at level l the low l digits hold the target box A
// (digit k = the bits of A's (k+1)-th split, coarsest first) and the high
// L - l digits hold the source box B in Morton order (finest digit lowest).
// Stage l merges the 2^d source children (digit l) and splits the target
// into 2^d children, which land in the same digit: each merge-and-split
// group reads and writes the same 2^d slots, at stride 2^(d l).
//
// The phase tau is evaluated with the same IEEE operation sequence as its
// definition (the library is built with -ffp-contract=off); |tau| reaches
// ~2e3 turns and only tau mod 1 matters, so a different rounding of tau
// would show up as ~1e-12 relative noise.
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>

#include "bfly_internal.h"

namespace bfly {
namespace {

constexpr double kTwoPi = 6.283185307179586;
constexpr int kBlock = 256;

template <typename R>
struct Cx;
template <>
struct Cx<double> {
  using T = double2;
};
template <>
struct Cx<float> {
  using T = float2;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ void cfma(double m, double2 v, double2& acc) {
  acc.x = fma(m, v.x, acc.x);
  acc.y = fma(m, v.y, acc.y);
}
__device__ __forceinline__ void cfma(float m, float2 v, float2& acc) {
  acc.x = fmaf(m, v.x, acc.x);
  acc.y = fmaf(m, v.y, acc.y);
}

// ---------------------------------------------------------------------------
// phase functions: tau = Phi / (2 pi) of the forward kernel
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ double tau_fwd(const Geo& G, const double* x, const double* y) {
  switch (G.phase) {
    case 0: {  // Fourier: x . y
      double s = x[0] * y[0];
#pragma unroll
      for (int j = 1; j < D; ++j) s = s + x[j] * y[j];
      return s;
    }
    case 1: {  // hyperbolic Radon family: N x0 sqrt(y0^2 + x1^2 y1^2)
      if constexpr (D == 2) {
        double a = y[0] * y[0];
        double b = x[1] * x[1];
        double c = y[1] * y[1];
        double e = b * c;
        double s = a + e;
        double m = G.Nd * x[0];
        return m * sqrt(s);
      }
      return 0.0;
    }
    case 2: {  // generalized-Radon analogue
      if constexpr (D == 3) {
        double u0 = kTwoPi * x[0];
        double u1 = kTwoPi * x[1];
        double g0 = (2.0 + sin(u0) * sin(u1)) / 3.0;
        double g1 = (2.0 + cos(u0) * cos(u1)) / 3.0;
        double t0 = g0 * y[0];
        double t1 = g1 * y[1];
        double s = (t0 * t0 + t1 * t1) + y[2] * y[2];
        double dot = (x[0] * y[0] + x[1] * y[1]) + x[2] * y[2];
        return G.Nd * (dot + sqrt(s));
      }
      return 0.0;
    }
    default: {  // separable test phase: N (sum x^2 + sum y^3)
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        a = a + x[j] * x[j];
        b = b + (y[j] * y[j]) * y[j];
      }
      return G.Nd * (a + b);
    }
  }
}

// Phase between a target-role point t and a source-role point s.
template <int D>
__device__ __forceinline__ double tau_k(const Geo& G, const double* t, const double* s) {
  return G.adj ? -tau_fwd<D>(G, s, t) : tau_fwd<D>(G, t, s);
}

// exp(2 pi i tau): exact reduction to fr = tau - rint(tau) in [-1/2, 1/2]
// in FP64, then the sine/cosine in the working precision.
template <typename R>
__device__ __forceinline__ typename Cx<R>::T expi(double tau);
template <>
__device__ __forceinline__ double2 expi<double>(double tau) {
  double fr = tau - rint(tau);
  double a = kTwoPi * fr;
  double s, c;
  sincos(a, &s, &c);
  return make_double2(c, s);
}
template <>
__device__ __forceinline__ float2 expi<float>(double tau) {
  // v_sin_f32 / v_cos_f32 take their argument in turns; keep it in [0, 1)
  double fr = tau - floor(tau);
  float f = fminf((float)fr, 0x1.fffffep-1f);
  return make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
}

// ---------------------------------------------------------------------------
// tree geometry (Sec. 1): after l stages the target box is cut 2^l times per
// dimension and the source box N / 2^l times
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void tgt_box(const Geo& G, int lvl, const int* a, double* c, double* w) {
#pragma unroll
  for (int j = 0; j < D; ++j) {
    w[j] = ldexp(G.tD[j], -lvl);
    c[j] = G.tlo[j] + ((double)a[j] + 0.5) * w[j];
  }
}
template <int D>
__device__ __forceinline__ void src_box(const Geo& G, int lvl, const int* b, double* c, double* w) {
#pragma unroll
  for (int j = 0; j < D; ++j) {
    w[j] = ldexp(G.sD[j], -(G.L - lvl));
    c[j] = G.slo[j] + ((double)b[j] + 0.5) * w[j];
  }
}
// tensor Chebyshev node t (dimension 0 fastest)
template <int D>
__device__ __forceinline__ void node(const Geo& G, const double* c, const double* w, int t, double* out) {
#pragma unroll
  for (int j = 0; j < D; ++j) {
    int tj = t % G.q;
    t /= G.q;
    out[j] = c[j] + (0.5 * w[j]) * G.z[tj];
  }
}
__device__ __forceinline__ double lag1(const Geo& G, int k, double s) {
  double v = 1.0;
  for (int m = 0; m < G.q; ++m)
    if (m != k) v *= (s - G.z[m]) / (G.z[k] - G.z[m]);
  return v;
}
template <int D>
__device__ __forceinline__ double lagrange(const Geo& G, const double* c, const double* w, int t,
                                           const double* u) {
  double v = 1.0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    int tj = t % G.q;
    t /= G.q;
    v *= lag1(G, tj, (u[j] - c[j]) / (0.5 * w[j]));
  }
  return v;
}

__device__ __forceinline__ int64_t bin1(double v, double lo, double D, int64_t n) {
  double u = ((v - lo) / D) * (double)n;
  if (!(u >= 0.0)) return 0;
  if (u >= (double)n) return n - 1;
  int64_t b = (int64_t)floor(u);
  return b > n - 1 ? n - 1 : b;
}

// slot digits <-> box indices
template <int D>
__device__ __forceinline__ void decode_tgt(uint32_t lo, int lvl, int* a) {
#pragma unroll
  for (int j = 0; j < D; ++j) a[j] = 0;
  for (int k = 0; k < lvl; ++k)
#pragma unroll
    for (int j = 0; j < D; ++j) a[j] |= (int)((lo >> (D * k + j)) & 1u) << (lvl - 1 - k);
}
template <int D>
__device__ __forceinline__ void decode_src(uint32_t hi, int ndig, int* b) {
#pragma unroll
  for (int j = 0; j < D; ++j) b[j] = 0;
  for (int k = 0; k < ndig; ++k)
#pragma unroll
    for (int j = 0; j < D; ++j) b[j] |= (int)((hi >> (D * k + j)) & 1u) << k;
}
template <int D>
__device__ __forceinline__ uint32_t encode_src(const int64_t* b, int ndig) {
  uint32_t m = 0;
  for (int k = 0; k < ndig; ++k)
#pragma unroll
    for (int j = 0; j < D; ++j) m |= (uint32_t)((b[j] >> k) & 1) << (D * k + j);
  return m;
}
template <int D>
__device__ __forceinline__ uint32_t encode_tgt(const int64_t* a, int lvl) {
  uint32_t m = 0;
  for (int k = 0; k < lvl; ++k)
#pragma unroll
    for (int j = 0; j < D; ++j) m |= (uint32_t)((a[j] >> (lvl - 1 - k)) & 1) << (D * k + j);
  return m;
}

// child-interpolation table E[h][k][k2] = l_k((z_k2 + 2h - 1) / 2): the 1-D
// Lagrange polynomial k of a parent box at node k2 of its half h.
template <typename R>
__device__ __forceinline__ void fill_E(const Geo& G, R* E) {
  const int q = G.q;
  for (int i = threadIdx.x; i < 2 * q * q; i += blockDim.x) {
    int h = i / (q * q), k = (i / q) % q, k2 = i % q;
    E[i] = (R)lag1(G, k, (G.z[k2] + (double)(2 * h - 1)) * 0.5);
  }
}
// tensor product entry prod_j E[c_j][ta_j][tb_j]
template <int D, typename R>
__device__ __forceinline__ R tensor_E(const R* E, int q, int c, int ta, int tb) {
  R v = (R)1;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    v *= E[(((c >> j) & 1) * q + ta % q) * q + tb % q];
    ta /= q;
    tb /= q;
  }
  return v;
}

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// ---------------------------------------------------------------------------
// binning + CSR
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(kBlock) void k_bin(const Geo G, int64_t n, const double* __restrict__ pts,
                                                uint32_t* __restrict__ keys, int32_t* __restrict__ idx) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t b[3];
  const int64_t N = (int64_t)1 << G.L;
#pragma unroll
  for (int j = 0; j < D; ++j) b[j] = bin1(pts[i * D + j], G.slo[j], G.sD[j], N);
  keys[i] = encode_src<D>(b, G.L);
  idx[i] = (int32_t)i;
}

// offs[m] = first sorted position whose key is >= m, for m = 0..P
__global__ __launch_bounds__(kBlock) void k_offsets(int64_t n, int64_t P, const uint32_t* __restrict__ ks,
                                                    int32_t* __restrict__ offs) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n == 0) {
    for (int64_t m = k; m <= P; m += (int64_t)gridDim.x * blockDim.x) offs[m] = 0;
    return;
  }
  if (k >= n) return;
  int64_t prev = k == 0 ? -1 : (int64_t)ks[k - 1];
  int64_t cur = ks[k];
  for (int64_t m = prev + 1; m <= cur; ++m) offs[m] = (int32_t)k;
  if (k == n - 1)
    for (int64_t m = cur + 1; m <= P; ++m) offs[m] = (int32_t)n;
}

__global__ __launch_bounds__(kBlock) void k_iota(int64_t n, int32_t* __restrict__ perm,
                                                 uint32_t* __restrict__ keys) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    perm[i] = (int32_t)i;
    keys[i] = 0u;
  }
}

// ---------------------------------------------------------------------------
// initialisation: one thread per (leaf B, node t, rhs)
//   delta_t = e^{-i Phi(c_X, y_t)} sum_{y in B} L_t(y) e^{i Phi(c_X, y)} g(y)
// ---------------------------------------------------------------------------
template <int D, typename R>
__global__ __launch_bounds__(kBlock) void k_init(const Geo G, const double* __restrict__ pts,
                                                 const double2* __restrict__ vin, int64_t ldin,
                                                 const int32_t* __restrict__ perm,
                                                 const int32_t* __restrict__ offs,
                                                 typename Cx<R>::T* __restrict__ W, int nrhs) {
  using T = typename Cx<R>::T;
  const int64_t P = (int64_t)1 << (D * G.L);
  int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= P * G.r) return;
  const int rhs = blockIdx.y;
  const int64_t leaf = it / G.r;
  const int t = (int)(it % G.r);
  int b[3], a0[3] = {0, 0, 0};
  double c[3], w[3], cX[3], wX[3], u[3];
  decode_src<D>((uint32_t)leaf, G.L, b);
  src_box<D>(G, 0, b, c, w);
  tgt_box<D>(G, 0, a0, cX, wX);
  T acc = {0, 0};
  for (int32_t k = offs[leaf]; k < offs[leaf + 1]; ++k) {
    const int32_t i = perm[k];
    double y[3];
#pragma unroll
    for (int j = 0; j < D; ++j) y[j] = pts[(int64_t)i * D + j];
    T e = expi<R>(tau_k<D>(G, cX, y));
    double2 gv = vin[(int64_t)rhs * ldin + i];
    T v = {(R)gv.x, (R)gv.y};
    T m = cmul(e, v);
    cfma((R)lagrange<D>(G, c, w, t, y), m, acc);
  }
  node<D>(G, c, w, t, u);
  T e = expi<R>(-tau_k<D>(G, cX, u));
  W[((int64_t)leaf * G.r + t) * nrhs + rhs] = cmul(e, acc);
}

// group index -> (target box p at level lvl, source box b' at level lvl+1)
template <int D>
__device__ __forceinline__ void group_boxes(const Geo& G, int lvl, uint32_t gi, int* p, int* bp,
                                            uint32_t* lo, uint32_t* hi) {
  const int lob = D * lvl;
  *lo = lob ? (gi & ((1u << lob) - 1u)) : 0u;
  *hi = gi >> lob;
  decode_tgt<D>(*lo, lvl, p);
  decode_src<D>(*hi, G.L - lvl - 1, bp);
}
__device__ __forceinline__ uint32_t group_slot(uint32_t lo, uint32_t hi, int c, int lob, int d) {
  return (hi << (lob + d)) | ((uint32_t)c << lob) | lo;
}

// ---------------------------------------------------------------------------
// first half (column-space) stage l -> l+1.  For every group (P, B') and
// every child A' of P:
//   delta^{A'B'}_t = e^{-i Phi(c_A', y^{B'}_t)} sum_c sum_t2 L^{B'}_t(y^{B_c}_t2)
//                    e^{i Phi(c_A', y^{B_c}_t2)} delta^{P B_c}_t2
// ---------------------------------------------------------------------------
template <int D, typename R>
__global__ __launch_bounds__(kBlock) void k_stage_src(const Geo G, int lvl, typename Cx<R>::T* __restrict__ W,
                                                      int nrhs, int64_t ngroups, int gpb) {
  using T = typename Cx<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const int q = G.q, r = G.r, nc = 1 << D, lob = D * lvl;
  R* E = reinterpret_cast<R*>(smem);
  T* vin = reinterpret_cast<T*>(smem + align16(2 * q * q * sizeof(R)));
  T* vmod = vin + gpb * nc * r;
  const int rhs = blockIdx.y;
  const int64_t g0 = (int64_t)blockIdx.x * gpb;
  const int ng = (int)min((int64_t)gpb, ngroups - g0);
  fill_E<R>(G, E);
  for (int i = threadIdx.x; i < ng * nc * r; i += blockDim.x) {
    int g = i / (nc * r), c = (i / r) % nc, t = i % r;
    uint32_t lo, hi;
    const int lobits = lob;
    lo = lobits ? (uint32_t)(g0 + g) & ((1u << lobits) - 1u) : 0u;
    hi = (uint32_t)(g0 + g) >> lobits;
    uint32_t s = group_slot(lo, hi, c, lob, D);
    vin[i] = W[((int64_t)s * r + t) * nrhs + rhs];
  }
  __syncthreads();
  for (int cp = 0; cp < nc; ++cp) {
    for (int i = threadIdx.x; i < ng * nc * r; i += blockDim.x) {
      int g = i / (nc * r), c = (i / r) % nc, t2 = i % r;
      int p[3], bp[3], a[3], bc[3];
      uint32_t lo, hi;
      group_boxes<D>(G, lvl, (uint32_t)(g0 + g), p, bp, &lo, &hi);
      double cA[3], wA[3], cc[3], wc[3], y[3];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        a[j] = 2 * p[j] + ((cp >> j) & 1);
        bc[j] = 2 * bp[j] + ((c >> j) & 1);
      }
      tgt_box<D>(G, lvl + 1, a, cA, wA);
      src_box<D>(G, lvl, bc, cc, wc);
      node<D>(G, cc, wc, t2, y);
      vmod[i] = cmul(expi<R>(tau_k<D>(G, cA, y)), vin[i]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ng * r; i += blockDim.x) {
      int g = i / r, t = i % r;
      int p[3], bp[3], a[3];
      uint32_t lo, hi;
      group_boxes<D>(G, lvl, (uint32_t)(g0 + g), p, bp, &lo, &hi);
      T acc = {0, 0};
      for (int c = 0; c < nc; ++c)
        for (int t2 = 0; t2 < r; ++t2) cfma(tensor_E<D, R>(E, q, c, t, t2), vmod[(g * nc + c) * r + t2], acc);
      double cA[3], wA[3], cB[3], wB[3], y[3];
#pragma unroll
      for (int j = 0; j < D; ++j) a[j] = 2 * p[j] + ((cp >> j) & 1);
      tgt_box<D>(G, lvl + 1, a, cA, wA);
      src_box<D>(G, lvl + 1, bp, cB, wB);
      node<D>(G, cB, wB, t, y);
      uint32_t s = group_slot(lo, hi, cp, lob, D);
      W[((int64_t)s * r + t) * nrhs + rhs] = cmul(expi<R>(-tau_k<D>(G, cA, y)), acc);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// middle switch at level ls: delta^{AB}_t <- sum_s e^{i Phi(x^A_t, y^B_s)} delta^{AB}_s
// ---------------------------------------------------------------------------
template <int D, typename R>
__global__ __launch_bounds__(kBlock) void k_switch(const Geo G, typename Cx<R>::T* __restrict__ W, int nrhs,
                                                   int64_t nslots, int spb) {
  using T = typename Cx<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  T* vin = reinterpret_cast<T*>(smem);
  const int r = G.r, lob = D * G.ls;
  const int rhs = blockIdx.y;
  const int64_t s0 = (int64_t)blockIdx.x * spb;
  const int ns = (int)min((int64_t)spb, nslots - s0);
  for (int i = threadIdx.x; i < ns * r; i += blockDim.x)
    vin[i] = W[((s0 + i / r) * r + i % r) * nrhs + rhs];
  __syncthreads();
  for (int i = threadIdx.x; i < ns * r; i += blockDim.x) {
    const int g = i / r, t = i % r;
    const uint32_t s = (uint32_t)(s0 + g);
    int a[3], b[3];
    decode_tgt<D>(lob ? (s & ((1u << lob) - 1u)) : 0u, G.ls, a);
    decode_src<D>(s >> lob, G.L - G.ls, b);
    double cA[3], wA[3], cB[3], wB[3], xt[3], ys[3];
    tgt_box<D>(G, G.ls, a, cA, wA);
    src_box<D>(G, G.ls, b, cB, wB);
    node<D>(G, cA, wA, t, xt);
    T acc = {0, 0};
    for (int s2 = 0; s2 < r; ++s2) {
      node<D>(G, cB, wB, s2, ys);
      T m = cmul(expi<R>(tau_k<D>(G, xt, ys)), vin[g * r + s2]);
      acc.x += m.x;
      acc.y += m.y;
    }
    W[((int64_t)s * r + t) * nrhs + rhs] = acc;
  }
}

// ---------------------------------------------------------------------------
// second half (row-space) stage l -> l+1.  For every group (P, B') and every
// child A' of P:
//   delta^{A'B'}_t = sum_c e^{i Phi(x^{A'}_t, c_{B_c})} sum_t2 L^P_t2(x^{A'}_t)
//                    e^{-i Phi(x^P_t2, c_{B_c})} delta^{P B_c}_t2
// ---------------------------------------------------------------------------
template <int D, typename R>
__global__ __launch_bounds__(kBlock) void k_stage_tgt(const Geo G, int lvl, typename Cx<R>::T* __restrict__ W,
                                                      int nrhs, int64_t ngroups, int gpb) {
  using T = typename Cx<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const int q = G.q, r = G.r, nc = 1 << D, lob = D * lvl;
  R* E = reinterpret_cast<R*>(smem);
  T* vdem = reinterpret_cast<T*>(smem + align16(2 * q * q * sizeof(R)));
  const int rhs = blockIdx.y;
  const int64_t g0 = (int64_t)blockIdx.x * gpb;
  const int ng = (int)min((int64_t)gpb, ngroups - g0);
  fill_E<R>(G, E);
  // demodulate the 2^d input vectors of every group on the parent's nodes
  for (int i = threadIdx.x; i < ng * nc * r; i += blockDim.x) {
    int g = i / (nc * r), c = (i / r) % nc, t2 = i % r;
    int p[3], bp[3], bc[3];
    uint32_t lo, hi;
    group_boxes<D>(G, lvl, (uint32_t)(g0 + g), p, bp, &lo, &hi);
    uint32_t s = group_slot(lo, hi, c, lob, D);
    T v = W[((int64_t)s * r + t2) * nrhs + rhs];
    double cP[3], wP[3], cb[3], wb[3], xp[3];
#pragma unroll
    for (int j = 0; j < D; ++j) bc[j] = 2 * bp[j] + ((c >> j) & 1);
    tgt_box<D>(G, lvl, p, cP, wP);
    src_box<D>(G, lvl, bc, cb, wb);
    node<D>(G, cP, wP, t2, xp);
    vdem[i] = cmul(expi<R>(-tau_k<D>(G, xp, cb)), v);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ng * nc * r; i += blockDim.x) {
    int g = i / (nc * r), cp = (i / r) % nc, t = i % r;
    int p[3], bp[3], a[3], bc[3];
    uint32_t lo, hi;
    group_boxes<D>(G, lvl, (uint32_t)(g0 + g), p, bp, &lo, &hi);
    double cA[3], wA[3], xt[3], cb[3], wb[3];
#pragma unroll
    for (int j = 0; j < D; ++j) a[j] = 2 * p[j] + ((cp >> j) & 1);
    tgt_box<D>(G, lvl + 1, a, cA, wA);
    node<D>(G, cA, wA, t, xt);
    T acc = {0, 0};
    for (int c = 0; c < nc; ++c) {
      T sacc = {0, 0};
      for (int t2 = 0; t2 < r; ++t2) cfma(tensor_E<D, R>(E, q, cp, t2, t), vdem[(g * nc + c) * r + t2], sacc);
#pragma unroll
      for (int j = 0; j < D; ++j) bc[j] = 2 * bp[j] + ((c >> j) & 1);
      src_box<D>(G, lvl, bc, cb, wb);
      T m = cmul(expi<R>(tau_k<D>(G, xt, cb)), sacc);
      acc.x += m.x;
      acc.y += m.y;
    }
    uint32_t s = group_slot(lo, hi, cp, lob, D);
    W[((int64_t)s * r + t) * nrhs + rhs] = acc;
  }
}

// ---------------------------------------------------------------------------
// final evaluation: one thread per (target x, rhs), x in leaf A
//   f(x) = e^{i Phi(x, c_Y)} sum_t L^A_t(x) e^{-i Phi(x^A_t, c_Y)} delta^{AY}_t
// ---------------------------------------------------------------------------
template <int D, typename R>
__global__ __launch_bounds__(kBlock) void k_final(const Geo G, int64_t n, const double* __restrict__ pts,
                                                  const typename Cx<R>::T* __restrict__ W, int nrhs,
                                                  double2* __restrict__ vout, int64_t ldout) {
  using T = typename Cx<R>::T;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int rhs = blockIdx.y;
  const int64_t N = (int64_t)1 << G.L;
  double x[3];
  int64_t a64[3];
  int a[3], b0[3] = {0, 0, 0};
#pragma unroll
  for (int j = 0; j < D; ++j) {
    x[j] = pts[i * D + j];
    a64[j] = bin1(x[j], G.tlo[j], G.tD[j], N);
    a[j] = (int)a64[j];
  }
  const uint32_t s = encode_tgt<D>(a64, G.L);
  double cA[3], wA[3], cY[3], wY[3], u[3];
  tgt_box<D>(G, G.L, a, cA, wA);
  src_box<D>(G, G.L, b0, cY, wY);
  T acc = {0, 0};
  for (int t = 0; t < G.r; ++t) {
    node<D>(G, cA, wA, t, u);
    T m = cmul(expi<R>(-tau_k<D>(G, u, cY)), W[((int64_t)s * G.r + t) * nrhs + rhs]);
    cfma((R)lagrange<D>(G, cA, wA, t, x), m, acc);
  }
  T f = cmul(expi<R>(tau_k<D>(G, x, cY)), acc);
  vout[(int64_t)rhs * ldout + i] = make_double2((double)f.x, (double)f.y);
}

inline unsigned blocks_for(int64_t n, int bs = kBlock) { return (unsigned)((n + bs - 1) / bs); }

template <int D, typename R>
hipError_t run_apply_t(const Geo& G, int64_t n_in, const double* pts_in, const double* vals_in, int64_t ld_in,
                       int64_t n_out, const double* pts_out, double* vals_out, int64_t ld_out, int nrhs,
                       const Work& w, hipStream_t st) {
  using T = typename Cx<R>::T;
  const int64_t P = (int64_t)1 << (D * G.L);
  const int r = G.r, nc = 1 << D, q = G.q;
  T* W = reinterpret_cast<T*>(w.W);
  // 1. binning of the input points into the level-0 source leaves
  {
  StepTimer tb(kStepBin, st);
  if (n_in > 0) {
    k_bin<D><<<blocks_for(n_in), kBlock, 0, st>>>(G, n_in, pts_in, w.keys, w.idx);
    if (D * G.L > 0) {
      size_t tmp = w.sort_tmp_bytes;
      hipError_t e = rocprim::radix_sort_pairs(w.sort_tmp, tmp, w.keys, w.keys_sorted, w.idx, w.perm,
                                               (unsigned)n_in, 0, D * G.L, st);
      if (e != hipSuccess) return e;
    } else {
      k_iota<<<blocks_for(n_in), kBlock, 0, st>>>(n_in, w.perm, w.keys_sorted);
    }
    k_offsets<<<blocks_for(n_in), kBlock, 0, st>>>(n_in, P, w.keys_sorted, w.offs);
  } else {
    k_offsets<<<blocks_for(P + 1), kBlock, 0, st>>>(0, P, nullptr, w.offs);
  }
  }
  // 2. initialisation
  {
    StepTimer tt(kStepInit, st);
    dim3 grid(blocks_for(P * r), nrhs);
    k_init<D, R><<<grid, kBlock, 0, st>>>(G, pts_in, reinterpret_cast<const double2*>(vals_in), ld_in, w.perm,
                                          w.offs, W, nrhs);
  }
  // 3./5. stages and the switch
  const int64_t ngroups = P / nc;
  const int gpb = std::max(1, std::min(64, 1024 / (nc * r)));
  const size_t smem = align16(2 * q * q * sizeof(R)) + 2 * (size_t)gpb * nc * r * sizeof(T);
  dim3 sgrid((unsigned)((ngroups + gpb - 1) / gpb), nrhs);
  for (int l = 0; l < G.ls; ++l) {
    StepTimer tt(kStepSrc, st);
    k_stage_src<D, R><<<sgrid, kBlock, smem, st>>>(G, l, W, nrhs, ngroups, gpb);
  }
  {
    StepTimer tt(kStepSwitch, st);
    const int spb = std::max(1, std::min(64, 1024 / r));
    dim3 grid((unsigned)((P + spb - 1) / spb), nrhs);
    k_switch<D, R><<<grid, kBlock, (size_t)spb * r * sizeof(T), st>>>(G, W, nrhs, P, spb);
  }
  for (int l = G.ls; l < G.L; ++l) {
    StepTimer tt(kStepTgt, st);
    k_stage_tgt<D, R><<<sgrid, kBlock, smem, st>>>(G, l, W, nrhs, ngroups, gpb);
  }
  // 6. final evaluation
  if (n_out > 0) {
    StepTimer tt(kStepFinal, st);
    dim3 grid(blocks_for(n_out), nrhs);
    k_final<D, R><<<grid, kBlock, 0, st>>>(G, n_out, pts_out, W, nrhs, reinterpret_cast<double2*>(vals_out),
                                           ld_out);
  }
  return hipGetLastError();
}

}  // namespace

size_t weight_bytes(const Geo& g, int nrhs, int prec) {
  const size_t P = (size_t)1 << (g.d * g.L);
  return P * (size_t)g.r * (size_t)nrhs * (prec == 0 ? sizeof(double2) : sizeof(float2));
}

hipError_t sort_storage_bytes(int64_t n, int bits, size_t* bytes) {
  *bytes = 0;
  if (n <= 0 || bits <= 0) return hipSuccess;
  return rocprim::radix_sort_pairs(nullptr, *bytes, (uint32_t*)nullptr, (uint32_t*)nullptr, (int32_t*)nullptr,
                                   (int32_t*)nullptr, (unsigned)n, 0, bits, (hipStream_t)0);
}

hipError_t run_apply(const Geo& g, int prec, int64_t n_in, const double* pts_in, const double* vals_in,
                     int64_t ld_in, int64_t n_out, const double* pts_out, double* vals_out, int64_t ld_out,
                     int nrhs, const Work& w, hipStream_t st) {
#define BFLY_DISPATCH(DD)                                                                                  \
  return prec == 0 ? run_apply_t<DD, double>(g, n_in, pts_in, vals_in, ld_in, n_out, pts_out, vals_out,   \
                                             ld_out, nrhs, w, st)                                          \
                   : run_apply_t<DD, float>(g, n_in, pts_in, vals_in, ld_in, n_out, pts_out, vals_out,     \
                                            ld_out, nrhs, w, st);
  switch (g.d) {
    case 1:
      BFLY_DISPATCH(1)
    case 2:
      BFLY_DISPATCH(2)
    default:
      BFLY_DISPATCH(3)
  }
#undef BFLY_DISPATCH
}

}  // namespace bfly
