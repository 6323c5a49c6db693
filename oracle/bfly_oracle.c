/*
 * bfly_oracle.c -- TEST INFRASTRUCTURE ONLY (see bfly_oracle.h).
 *
 * A plain FP64 CPU implementation of
 *   (1) the direct sum f(x) = sum_y exp(i Phi(x,y)) g(y)        (Sec. 1, Eq. 1), and
 *   (2) the butterfly apply of Alg. "alg:serial" (Sec. 1.3) with the analytic
 *       tensor-product Chebyshev translation operators the paper runs for
 *       K = exp(i Phi) (Sec. 1.4 "Avoiding quadratic precomputation"):
 *       column-space (source) interpolation while the source boxes are small,
 *       the middle switch, then row-space (target) interpolation.
 *
 * The paper cites the translation operators rather than printing them; the
 * formulas used here are derived from its definitions of potentials and
 * expansion weights (Sec. 1) and of equivalent sources (Sec. 1.2), with the
 * readings recorded at the top of each step.  Translations are applied in
 * DENSE form (an r x 2^d r real matrix between two phase diagonals), which
 * shares nothing with the tensor-factored GPU kernels.
 *
 * Must be compiled with -ffp-contract=off: the phase tau is large (|tau| up to
 * ~2e3 turns) and is taken modulo 1, so its exact IEEE operation sequence is
 * part of the specification.
 *
 * Parallelism: OpenMP over independent output vectors / targets only; every
 * individual result is computed by one thread in the order written.
 */
#include "bfly_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_QMAX 40

typedef struct { double re, im; } cplx;

static const double TWO_PI = 6.283185307179586;

static inline cplx cmul(cplx a, cplx b) {
  cplx c;
  c.re = a.re * b.re - a.im * b.im;
  c.im = a.re * b.im + a.im * b.re;
  return c;
}

/* ------------------------------------------------------------------------ */
/* Phase functions (the kernel K = exp(2 pi i tau), Eq. (6)).             */
/* ------------------------------------------------------------------------ */

double orc_tau(int phase, int d, long N, const double* x, const double* y) {
  const double Nd = (double)N;
  switch (phase) {
    case ORC_FOURIER: { /* Phi = 2 pi x.y (Sec. 3, list of kernels) */
      double s = x[0] * y[0];
      for (int j = 1; j < d; ++j) s = s + x[j] * y[j];
      return s;
    }
    case ORC_HYPRADON2: { /* hyperbolic Radon family (Sec. 3.1), roles as in the workload */
      double a = y[0] * y[0];
      double b = x[1] * x[1];
      double c = y[1] * y[1];
      double e = b * c;
      double s = a + e;
      double m = Nd * x[0];
      return m * sqrt(s);
    }
    case ORC_GENRADON3: { /* generalized-Radon analogue (Sec. 3.2), workload form */
      double u0 = TWO_PI * x[0];
      double u1 = TWO_PI * x[1];
      double g0 = (2.0 + sin(u0) * sin(u1)) / 3.0;
      double g1 = (2.0 + cos(u0) * cos(u1)) / 3.0;
      double t0 = g0 * y[0];
      double t1 = g1 * y[1];
      double s = (t0 * t0 + t1 * t1) + y[2] * y[2];
      double dot = (x[0] * y[0] + x[1] * y[1]) + x[2] * y[2];
      return Nd * (dot + sqrt(s));
    }
    case ORC_GENRADON3_PI: { /* generalized-Radon analogue (Sec. 3.2) as the paper
                                prints it: Phi = pi (x.p + sqrt(gamma^2 + kappa^2)),
                                gamma = p0 g0(x), kappa = p1 g1(x); no N inside */
      double u0 = TWO_PI * x[0];
      double u1 = TWO_PI * x[1];
      double g0 = (2.0 + sin(u0) * sin(u1)) / 3.0;
      double g1 = (2.0 + cos(u0) * cos(u1)) / 3.0;
      double t0 = g0 * y[0];
      double t1 = g1 * y[1];
      double s = t0 * t0 + t1 * t1;
      double dot = (x[0] * y[0] + x[1] * y[1]) + x[2] * y[2];
      return 0.5 * (dot + sqrt(s));
    }
    case ORC_SEPARABLE: { /* additively separable test phase: K has rank one */
      double a = 0.0, b = 0.0;
      for (int j = 0; j < d; ++j) {
        a = a + x[j] * x[j];
        b = b + (y[j] * y[j]) * y[j];
      }
      return Nd * (a + b);
    }
    default:
      return 0.0;
  }
}

/* exp(2 pi i tau) with the exact reduction tau - rint(tau) first. */
static inline cplx expi(double tau) {
  double fr = tau - rint(tau);
  double a = TWO_PI * fr;
  cplx e;
  e.re = cos(a);
  e.im = sin(a);
  return e;
}

/* ------------------------------------------------------------------------ */
/* Problem description                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int d, L, q, r, phase, adj, ls, nrhs;
  long N, P;
  double slo[3], sD[3]; /* source-role box */
  double tlo[3], tD[3]; /* target-role box */
  double z[ORC_QMAX];
} prob;

/* Kernel phase between a target-role point t and a source-role point s.
 * The adjoint problem K^H(y, x) = exp(-i Phi(x, y)) has the y points as
 * targets and the x points as sources. */
static inline double tau_k(const prob* p, const double* t, const double* s) {
  if (p->adj) return -orc_tau(p->phase, p->d, p->N, s, t);
  return orc_tau(p->phase, p->d, p->N, t, s);
}

void orc_nodes(int q, double* z) {
  for (int k = 0; k < q; ++k) z[k] = cos((double)(2 * k + 1) * M_PI / (double)(2 * q));
}

static long bin1(double v, double lo, double hi, long n) {
  double D = hi - lo;
  double u = ((v - lo) / D) * (double)n;
  if (!(u >= 0.0)) return 0; /* also catches NaN */
  if (u >= (double)n) return n - 1;
  long b = (long)floor(u);
  return b > n - 1 ? n - 1 : b;
}

void orc_bin(int d, long n_per_dim, const double* lo, const double* hi,
             long n, const double* pts, long* out) {
  for (long i = 0; i < n; ++i)
    for (int j = 0; j < d; ++j) out[i * d + j] = bin1(pts[i * d + j], lo[j], hi[j], n_per_dim);
}

/* Boxes of the trees T_X (targets) and T_Y (sources) after `lvl` stages
 * (Sec. 1): target boxes are 2^lvl per dimension, source boxes N / 2^lvl. */
static void tgt_box(const prob* p, int lvl, const long* a, double* c, double* w) {
  for (int j = 0; j < p->d; ++j) {
    w[j] = ldexp(p->tD[j], -lvl);
    c[j] = p->tlo[j] + ((double)a[j] + 0.5) * w[j];
  }
}
static void src_box(const prob* p, int lvl, const long* b, double* c, double* w) {
  for (int j = 0; j < p->d; ++j) {
    w[j] = ldexp(p->sD[j], -(p->L - lvl));
    c[j] = p->slo[j] + ((double)b[j] + 0.5) * w[j];
  }
}

/* Tensor Chebyshev node t (dim 0 fastest) of the box with centre c, width w. */
static void node(const prob* p, const double* c, const double* w, int t, double* out) {
  for (int j = 0; j < p->d; ++j) {
    int tj = t % p->q;
    t /= p->q;
    out[j] = c[j] + (0.5 * w[j]) * p->z[tj];
  }
}

/* 1-D Lagrange polynomial of node k at reference coordinate s. */
static double lag1(const prob* p, int k, double s) {
  double v = 1.0;
  for (int m = 0; m < p->q; ++m)
    if (m != k) v *= (s - p->z[m]) / (p->z[k] - p->z[m]);
  return v;
}

/* Tensor Lagrange basis function t of the box (c, w) at point u. */
static double lagrange(const prob* p, const double* c, const double* w, int t, const double* u) {
  double v = 1.0;
  for (int j = 0; j < p->d; ++j) {
    int tj = t % p->q;
    t /= p->q;
    double s = (u[j] - c[j]) / (0.5 * w[j]);
    v *= lag1(p, tj, s);
  }
  return v;
}

static void decode(const prob* p, long lin, int bits, long* idx) {
  long mask = (1L << bits) - 1;
  for (int j = 0; j < p->d; ++j) idx[j] = (lin >> (bits * j)) & mask;
}
static long encode(const prob* p, const long* idx, int bits) {
  long lin = 0;
  for (int j = 0; j < p->d; ++j) lin |= idx[j] << (bits * j);
  return lin;
}
/* weight-vector index of the pair (A at target level lvl, B at source level lvl) */
static long pair_index(const prob* p, int lvl, long a_lin, long b_lin) {
  return (a_lin << (p->d * (p->L - lvl))) | b_lin;
}

/* Parent basis evaluated at the child's nodes, in reference geometry:
 * tab[c][t][t2] = L^{parent}_t(node t2 of child c).  The Lagrange basis is
 * invariant under the affine map of a box onto [-1,1]^d, so one table serves
 * every box of every level. */
static double* child_table(const prob* p) {
  int nc = 1 << p->d, r = p->r;
  double* tab = (double*)malloc(sizeof(double) * (size_t)nc * r * r);
  double pc[3] = {0, 0, 0}, pw[3] = {2, 2, 2};
  for (int c = 0; c < nc; ++c) {
    double cc[3], cw[3], u[3];
    for (int j = 0; j < p->d; ++j) {
      cc[j] = ((c >> j) & 1) ? 0.5 : -0.5;
      cw[j] = 1.0;
    }
    for (int t2 = 0; t2 < r; ++t2) {
      node(p, cc, cw, t2, u);
      for (int t = 0; t < r; ++t) tab[((size_t)c * r + t) * r + t2] = lagrange(p, pc, pw, t, u);
    }
  }
  return tab;
}

static int setup(prob* p, int d, long N, int q, int phase,
                 const double* slo, const double* shi, const double* tlo, const double* thi,
                 int adjoint, int switch_level, int nrhs) {
  if (d < 1 || d > 3) return 1;
  if (N < 1 || (N & (N - 1))) return 1;
  if (q < 1 || q > ORC_QMAX) return 1;
  if (nrhs < 1 || nrhs > 64) return 1;
  if (phase == ORC_HYPRADON2 && d != 2) return 1;
  if ((phase == ORC_GENRADON3 || phase == ORC_GENRADON3_PI) && d != 3) return 1;
  if (phase < 0 || phase > 4) return 1;
  memset(p, 0, sizeof(*p));
  p->d = d;
  p->N = N;
  p->L = 0;
  while ((1L << p->L) < N) ++p->L;
  p->q = q;
  p->r = 1;
  for (int j = 0; j < d; ++j) p->r *= q;
  p->P = 1L << (d * p->L);
  p->phase = phase;
  p->adj = adjoint ? 1 : 0;
  p->nrhs = nrhs;
  /* middle switch level (Sec. 1.4): floor(L/2) forward; the adjoint runs its
     levels in the mirror order of the forward's, so its middle is L - floor(L/2) */
  p->ls = switch_level < 0 ? (adjoint ? p->L - p->L / 2 : p->L / 2) : switch_level;
  if (p->ls > p->L) return 1;
  /* the adjoint swaps the roles of the two boxes */
  const double *sl = adjoint ? tlo : slo, *sh = adjoint ? thi : shi;
  const double *tl = adjoint ? slo : tlo, *th = adjoint ? shi : thi;
  for (int j = 0; j < d; ++j) {
    p->slo[j] = sl[j];
    p->sD[j] = sh[j] - sl[j];
    p->tlo[j] = tl[j];
    p->tD[j] = th[j] - tl[j];
    if (!(p->sD[j] > 0) || !(p->tD[j] > 0)) return 1;
  }
  orc_nodes(q, p->z);
  return 0;
}

static int threads(int nthreads) {
#ifdef _OPENMP
  return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Direct sum (Eq. 1 summed over all source boxes)                          */
/* ------------------------------------------------------------------------ */

int orc_direct(int phase, int d, long N, int adjoint,
               long n_in, const double* pts_in, const double* in, long ldin,
               long n_out, const double* pts_out, double* out, long ldout,
               int nrhs, int nthreads) {
  prob p;
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  if (setup(&p, d, N, 2, phase, lo, hi, lo, hi, adjoint, -1, nrhs)) return 1;
  int nt = threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
  for (long i = 0; i < n_out; ++i) {
    const double* t = pts_out + i * d;
    for (int k = 0; k < nrhs; ++k) {
      double sr = 0.0, si = 0.0;
      const double* g = in + 2 * (size_t)k * ldin;
      for (long j = 0; j < n_in; ++j) {
        cplx e = expi(tau_k(&p, t, pts_in + j * d));
        cplx v = {g[2 * j], g[2 * j + 1]};
        cplx m = cmul(e, v);
        sr += m.re;
        si += m.im;
      }
      out[2 * ((size_t)k * ldout + i)] = sr;
      out[2 * ((size_t)k * ldout + i) + 1] = si;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Butterfly apply (Alg. "alg:serial")                                      */
/* ------------------------------------------------------------------------ */

/* The apply; when dump is not NULL, the weights after step dump_at are
 * copied there (see orc_butterfly_dump). */
static int butterfly(int d, long N, int q, int phase,
                     const double* slo, const double* shi,
                     const double* tlo, const double* thi,
                     int adjoint, int switch_level,
                     long n_in, const double* pts_in, const double* in, long ldin,
                     long n_out, const double* pts_out, double* out, long ldout,
                     int nrhs, int nthreads, double* counts, int dump_at, double* dump) {
  prob pb;
  if (setup(&pb, d, N, q, phase, slo, shi, tlo, thi, adjoint, switch_level, nrhs)) return 1;
  const prob* p = &pb;
  const int nt = threads(nthreads);
  const int r = p->r, L = p->L, nc = 1 << d, R = nrhs;
  const long P = p->P;
  const size_t vec = (size_t)r * R; /* complex entries per weight vector */
  double n_phase = 0, n_mac = 0, n_cmac = 0;

  cplx* W = (cplx*)calloc((size_t)P * vec, sizeof(cplx));
  cplx* Wn = (cplx*)calloc((size_t)P * vec, sizeof(cplx));
  double* tab = child_table(p);
  if (!W || !Wn || !tab) {
    free(W);
    free(Wn);
    free(tab);
    return 2;
  }

  /* the weights after a step, for orc_butterfly_dump */
#define ORC_DUMP(step)                                                      \
  do {                                                                      \
    if (dump && dump_at == (step)) memcpy(dump, W, sizeof(cplx) * (size_t)P * vec); \
  } while (0)

  /* ---- 1. bin the sources into the N^d leaves of the source tree (stable) */
  long* leaf = (long*)malloc(sizeof(long) * (size_t)(n_in > 0 ? n_in : 1));
  long* start = (long*)calloc((size_t)P + 1, sizeof(long));
  long* order = (long*)malloc(sizeof(long) * (size_t)(n_in > 0 ? n_in : 1));
  for (long i = 0; i < n_in; ++i) {
    long b[3];
    for (int j = 0; j < d; ++j) b[j] = bin1(pts_in[i * d + j], p->slo[j], p->slo[j] + p->sD[j], N);
    leaf[i] = encode(p, b, L);
    start[leaf[i] + 1]++;
  }
  for (long b = 0; b < P; ++b) start[b + 1] += start[b];
  {
    long* pos = (long*)malloc(sizeof(long) * (size_t)P);
    memcpy(pos, start, sizeof(long) * (size_t)P);
    for (long i = 0; i < n_in; ++i) order[pos[leaf[i]]++] = i;
    free(pos);
  }

  /* ---- 2. initialisation w_XB := V_XB g_B (Sec. 1; Alg. "alg:serial").
   * Interpolating y -> exp(i(Phi(x,y) - Phi(c_X,y))) on B's Chebyshev nodes
   * gives delta^{XB}_t = e^{-i Phi(c_X, y_t)} sum_{y in B} L_t(y) e^{i Phi(c_X, y)} g(y):
   * the weights are equivalent sources located at the nodes of B. */
  {
    long a0[3] = {0, 0, 0};
    double cX[3], wX[3];
    tgt_box(p, 0, a0, cX, wX);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt) reduction(+ : n_phase, n_mac)
    for (long bl = 0; bl < P; ++bl) {
      long b[3];
      double c[3], w[3], u[3];
      decode(p, bl, L, b);
      src_box(p, 0, b, c, w);
      cplx* acc = W + (size_t)pair_index(p, 0, 0, bl) * vec;
      cplx m[64];
      for (long k = start[bl]; k < start[bl + 1]; ++k) {
        long i = order[k];
        const double* y = pts_in + i * d;
        cplx e = expi(tau_k(p, cX, y));
        n_phase += 1;
        for (int s = 0; s < R; ++s) {
          cplx v = {in[2 * ((size_t)s * ldin + i)], in[2 * ((size_t)s * ldin + i) + 1]};
          m[s] = cmul(e, v);
        }
        for (int t = 0; t < r; ++t) {
          double lv = lagrange(p, c, w, t, y);
          for (int s = 0; s < R; ++s) {
            acc[t * R + s].re += lv * m[s].re;
            acc[t * R + s].im += lv * m[s].im;
          }
        }
        n_mac += r;
      }
      for (int t = 0; t < r; ++t) {
        node(p, c, w, t, u);
        cplx e = expi(-tau_k(p, cX, u));
        n_phase += 1;
        for (int s = 0; s < R; ++s) acc[t * R + s] = cmul(e, acc[t * R + s]);
      }
    }
  }

  ORC_DUMP(0);

  /* ---- 3. first half: stages l = 0 .. ls-1, column-space interpolation.
   * Group = (parent target box P at level l, merged source box B' at level
   * l+1); each child target box A' of P gets
   *   delta^{A'B'}_t = e^{-i Phi(c_A', y^{B'}_t)} sum_c sum_t2 L^{B'}_t(y^{B_c}_t2)
   *                    e^{i Phi(c_A', y^{B_c}_t2)} delta^{P B_c}_t2,
   * i.e. the step-2 formula applied to the children's equivalent sources
   * (Sec. 1.3 "Translating equivalent sources"). */
  for (int l = 0; l < p->ls; ++l) {
    const int lb_out = L - l - 1; /* source bits per dim at level l+1 */
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt) reduction(+ : n_phase, n_mac)
    for (long po = 0; po < P; ++po) {
      long al = po >> (d * lb_out), bl = po & ((1L << (d * lb_out)) - 1);
      long a[3], pa[3], bp[3], bc[3];
      double cA[3], wA[3], cB[3], wB[3], cc[3], wc[3], u[3];
      decode(p, al, l + 1, a);
      for (int j = 0; j < d; ++j) pa[j] = a[j] >> 1;
      long pl = encode(p, pa, l);
      decode(p, bl, lb_out, bp);
      tgt_box(p, l + 1, a, cA, wA);
      src_box(p, l + 1, bp, cB, wB);
      cplx* acc = Wn + (size_t)po * vec;
      memset(acc, 0, sizeof(cplx) * vec);
      cplx m[64];
      for (int c = 0; c < nc; ++c) {
        for (int j = 0; j < d; ++j) bc[j] = 2 * bp[j] + ((c >> j) & 1);
        long bcl = encode(p, bc, L - l);
        const cplx* win = W + (size_t)pair_index(p, l, pl, bcl) * vec;
        src_box(p, l, bc, cc, wc);
        for (int t2 = 0; t2 < r; ++t2) {
          node(p, cc, wc, t2, u);
          cplx e = expi(tau_k(p, cA, u));
          n_phase += 1;
          for (int s = 0; s < R; ++s) m[s] = cmul(e, win[t2 * R + s]);
          for (int t = 0; t < r; ++t) {
            double lv = tab[((size_t)c * r + t) * r + t2];
            for (int s = 0; s < R; ++s) {
              acc[t * R + s].re += lv * m[s].re;
              acc[t * R + s].im += lv * m[s].im;
            }
          }
          n_mac += r;
        }
      }
      for (int t = 0; t < r; ++t) {
        node(p, cB, wB, t, u);
        cplx e = expi(-tau_k(p, cA, u));
        n_phase += 1;
        for (int s = 0; s < R; ++s) acc[t * R + s] = cmul(e, acc[t * R + s]);
      }
    }
    cplx* tmp = W;
    W = Wn;
    Wn = tmp;
    ORC_DUMP(l + 1);
  }

  /* ---- 4. middle switch at level ls (Sec. 1.4): equivalent sources at the
   * nodes of B become potentials at the nodes of A,
   *   delta^{AB}_t <- sum_s e^{i Phi(x^A_t, y^B_s)} delta^{AB}_s. */
  {
    const int l = p->ls, lb = L - l;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt) reduction(+ : n_phase, n_cmac)
    for (long pi = 0; pi < P; ++pi) {
      long al = pi >> (d * lb), bl = pi & ((1L << (d * lb)) - 1);
      long a[3], b[3];
      double cA[3], wA[3], cB[3], wB[3], xt[3], ys[3];
      decode(p, al, l, a);
      decode(p, bl, lb, b);
      tgt_box(p, l, a, cA, wA);
      src_box(p, l, b, cB, wB);
      const cplx* win = W + (size_t)pi * vec;
      cplx* wout = Wn + (size_t)pi * vec;
      memset(wout, 0, sizeof(cplx) * vec);
      for (int t = 0; t < r; ++t) {
        node(p, cA, wA, t, xt);
        for (int s2 = 0; s2 < r; ++s2) {
          node(p, cB, wB, s2, ys);
          cplx e = expi(tau_k(p, xt, ys));
          n_phase += 1;
          for (int s = 0; s < R; ++s) {
            cplx m = cmul(e, win[s2 * R + s]);
            wout[t * R + s].re += m.re;
            wout[t * R + s].im += m.im;
          }
          n_cmac += 1;
        }
      }
    }
    cplx* tmp = W;
    W = Wn;
    Wn = tmp;
    ORC_DUMP(p->ls + 1);
  }

  /* ---- 5. second half: stages l = ls .. L-1, row-space interpolation
   * (Sec. 1.3-1.4).  Weights are now potentials at the nodes of the target box.
   * Interpolating x -> exp(i(Phi(x,y) - Phi(x,c_B))) on the parent's nodes:
   *   delta^{A'B'}_t = sum_c e^{i Phi(x^{A'}_t, c_{B_c})} sum_t2 L^P_t2(x^{A'}_t)
   *                    e^{-i Phi(x^P_t2, c_{B_c})} delta^{P B_c}_t2. */
  for (int l = p->ls; l < L; ++l) {
    const int lb_out = L - l - 1;
    const long ngroups = P >> d;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt) reduction(+ : n_phase, n_mac)
    for (long gi = 0; gi < ngroups; ++gi) {
      long pl = gi >> (d * lb_out), bl = gi & ((1L << (d * lb_out)) - 1);
      long pa[3], bp[3], bc[3], a[3];
      double cP[3], wP[3], cBc[3], wBc[3], cA[3], wA[3], u[3];
      decode(p, pl, l, pa);
      decode(p, bl, lb_out, bp);
      tgt_box(p, l, pa, cP, wP);
      cplx* dm = (cplx*)malloc(sizeof(cplx) * (size_t)nc * vec);
      double cbc[8][3];
      /* demodulate the 2^d input vectors on the parent's nodes */
      for (int c = 0; c < nc; ++c) {
        for (int j = 0; j < d; ++j) bc[j] = 2 * bp[j] + ((c >> j) & 1);
        long bcl = encode(p, bc, L - l);
        src_box(p, l, bc, cBc, wBc);
        for (int j = 0; j < d; ++j) cbc[c][j] = cBc[j];
        const cplx* win = W + (size_t)pair_index(p, l, pl, bcl) * vec;
        for (int t2 = 0; t2 < r; ++t2) {
          node(p, cP, wP, t2, u);
          cplx e = expi(-tau_k(p, u, cBc));
          n_phase += 1;
          for (int s = 0; s < R; ++s) dm[((size_t)c * r + t2) * R + s] = cmul(e, win[t2 * R + s]);
        }
      }
      /* interpolate onto each child target box and re-modulate */
      for (int cp = 0; cp < nc; ++cp) {
        for (int j = 0; j < d; ++j) a[j] = 2 * pa[j] + ((cp >> j) & 1);
        long al = encode(p, a, l + 1);
        tgt_box(p, l + 1, a, cA, wA);
        cplx* wout = Wn + (size_t)pair_index(p, l + 1, al, bl) * vec;
        memset(wout, 0, sizeof(cplx) * vec);
        for (int t = 0; t < r; ++t) {
          node(p, cA, wA, t, u);
          for (int c = 0; c < nc; ++c) {
            cplx sacc[64];
            for (int s = 0; s < R; ++s) sacc[s].re = sacc[s].im = 0.0;
            for (int t2 = 0; t2 < r; ++t2) {
              /* L^P_t2 at child cp's node t == parent basis t2 at that node */
              double lv = tab[((size_t)cp * r + t2) * r + t];
              for (int s = 0; s < R; ++s) {
                sacc[s].re += lv * dm[((size_t)c * r + t2) * R + s].re;
                sacc[s].im += lv * dm[((size_t)c * r + t2) * R + s].im;
              }
            }
            n_mac += r;
            cplx e = expi(tau_k(p, u, cbc[c]));
            n_phase += 1;
            for (int s = 0; s < R; ++s) {
              cplx mm = cmul(e, sacc[s]);
              wout[t * R + s].re += mm.re;
              wout[t * R + s].im += mm.im;
            }
          }
        }
      }
      free(dm);
    }
    cplx* tmp = W;
    W = Wn;
    Wn = tmp;
    ORC_DUMP(l + 2);
  }
#undef ORC_DUMP

  /* ---- 6. final evaluation f_AY := U_AY w_AY (Sec. 1; Alg. "alg:serial"):
   * f(x) = e^{i Phi(x, c_Y)} sum_t L^A_t(x) e^{-i Phi(x^A_t, c_Y)} delta^{AY}_t. */
  {
    long b0[3] = {0, 0, 0};
    double cY[3], wY[3];
    src_box(p, L, b0, cY, wY);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt) reduction(+ : n_phase)
    for (long al = 0; al < P; ++al) {
      long a[3];
      double cA[3], wA[3], u[3];
      decode(p, al, L, a);
      tgt_box(p, L, a, cA, wA);
      cplx* wv = W + (size_t)pair_index(p, L, al, 0) * vec;
      for (int t = 0; t < r; ++t) {
        node(p, cA, wA, t, u);
        cplx e = expi(-tau_k(p, u, cY));
        n_phase += 1;
        for (int s = 0; s < R; ++s) wv[t * R + s] = cmul(e, wv[t * R + s]);
      }
    }
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt) reduction(+ : n_phase, n_mac)
    for (long i = 0; i < n_out; ++i) {
      const double* x = pts_out + i * d;
      long a[3];
      double cA[3], wA[3];
      for (int j = 0; j < d; ++j) a[j] = bin1(x[j], p->tlo[j], p->tlo[j] + p->tD[j], N);
      long al = encode(p, a, L);
      tgt_box(p, L, a, cA, wA);
      const cplx* wv = W + (size_t)pair_index(p, L, al, 0) * vec;
      cplx e = expi(tau_k(p, x, cY));
      n_phase += 1;
      for (int s = 0; s < R; ++s) {
        double sr = 0.0, si = 0.0;
        for (int t = 0; t < r; ++t) {
          double lv = lagrange(p, cA, wA, t, x);
          sr += lv * wv[t * R + s].re;
          si += lv * wv[t * R + s].im;
        }
        cplx v = {sr, si};
        cplx fo = cmul(e, v);
        out[2 * ((size_t)s * ldout + i)] = fo.re;
        out[2 * ((size_t)s * ldout + i) + 1] = fo.im;
      }
      n_mac += r;
    }
  }

  if (counts) {
    counts[0] = n_phase;
    counts[1] = n_mac;
    counts[2] = n_cmac;
    counts[3] = (double)L;
  }
  free(W);
  free(Wn);
  free(tab);
  free(leaf);
  free(start);
  free(order);
  return 0;
}

int orc_butterfly(int d, long N, int q, int phase,
                  const double* slo, const double* shi,
                  const double* tlo, const double* thi,
                  int adjoint, int switch_level,
                  long n_in, const double* pts_in, const double* in, long ldin,
                  long n_out, const double* pts_out, double* out, long ldout,
                  int nrhs, int nthreads, double* counts) {
  return butterfly(d, N, q, phase, slo, shi, tlo, thi, adjoint, switch_level, n_in, pts_in, in, ldin, n_out,
                   pts_out, out, ldout, nrhs, nthreads, counts, -1, NULL);
}

int orc_butterfly_dump(int d, long N, int q, int phase,
                       const double* slo, const double* shi,
                       const double* tlo, const double* thi,
                       int adjoint, int switch_level,
                       long n_in, const double* pts_in, const double* in, long ldin,
                       long n_out, const double* pts_out, double* out, long ldout,
                       int nrhs, int nthreads, int dump_at, double* dump) {
  return butterfly(d, N, q, phase, slo, shi, tlo, thi, adjoint, switch_level, n_in, pts_in, in, ldin, n_out,
                   pts_out, out, ldout, nrhs, nthreads, NULL, dump_at, dump);
}
