/*
 * bfly_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference for the butterfly apply of Poulson, Demanet,
 * Maxwell & Ying, "A Parallel Butterfly Algorithm" (sequential algorithm,
 * Alg. "alg:serial", with the analytic Chebyshev translation operators of
 * Sec. 1.4 "Avoiding quadratic precomputation"), and for the direct sum it
 * approximates (Eq. 1).  Only tests, the smoke check and the CPU-baseline leg
 * of the benchmark may call this library.  It shares no code with the GPU
 * library.
 *
 * Complex arrays are interleaved (re, im) doubles.  Point arrays are
 * row-major [n][d].  Right-hand side k of g lives at g + 2*k*ldg.
 */
#ifndef BFLY_ORACLE_H
#define BFLY_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

/* phase ids: tau = Phi / (2 pi), i.e. the phase in turns */
#define ORC_FOURIER   0 /* tau = x . y                                            */
#define ORC_HYPRADON2 1 /* tau = N x0 sqrt(y0^2 + x1^2 y1^2)                     d=2 */
#define ORC_GENRADON3 2 /* tau = N (x.y + sqrt(g0(x)^2 y0^2 + g1(x)^2 y1^2 + y2^2)) d=3 */
#define ORC_SEPARABLE 3 /* tau = N (sum_j x_j^2 + sum_j y_j^3)                    */
#define ORC_GENRADON3_PI 4 /* tau = (x.p + sqrt(gamma^2 + kappa^2)) / 2, gamma = p0 g0(x),
                              kappa = p1 g1(x): Phi = pi (...) exactly as printed, d=3 */

/* tau(x, y) of the forward kernel (test access to the phase definitions). */
double orc_tau(int phase, int d, long N, const double* x, const double* y);

/* 1-D Chebyshev nodes of the first kind, z_k = cos((2k+1) pi / (2q)). */
void orc_nodes(int q, double* z);

/* Leaf index per point: floor((p - lo)/(hi - lo) * n) clamped to [0, n-1],
 * per dimension; out[i*d + j]. */
void orc_bin(int d, long n_per_dim, const double* lo, const double* hi,
             long n, const double* pts, long* out);

/* Direct sum f(x_i) = sum_j exp(+-i Phi(x_i, y_j)) g(y_j) (sign = +1: K, -1: the
 * adjoint K^H with roles swapped, i.e. out(y_j) = sum_i exp(-i Phi(x_i, y_j)) in(x_i)).
 * Forward: pts_in = y (n_in), pts_out = x (n_out).  Adjoint: pts_in = x, pts_out = y. */
int orc_direct(int phase, int d, long N, int adjoint,
               long n_in, const double* pts_in, const double* in, long ldin,
               long n_out, const double* pts_out, double* out, long ldout,
               int nrhs, int nthreads);

/* Butterfly apply.  Forward: sources y in box [slo, shi), targets x in box
 * [tlo, thi), f = B g.  Adjoint (adjoint=1): the same plan geometry, but
 * the swapped problem is run: sources are the x points (box [tlo,thi)),
 * targets are the y points, phase -Phi(x, y).
 * switch_level < 0 selects the middle level: floor(L/2) forward, and
 * L - floor(L/2) for the adjoint, which is then the exact transpose of the
 * forward butterfly (its stages are the forward's transposed, level for
 * level, once the switch sits at the forward switch's mirror level).
 * counts (may be NULL) receives [phase evaluations, real x complex MACs per
 * RHS, switch complex MACs per RHS, stages run].  1 <= nrhs <= 64. */
int orc_butterfly(int d, long N, int q, int phase,
                  const double* slo, const double* shi,
                  const double* tlo, const double* thi,
                  int adjoint, int switch_level,
                  long n_in, const double* pts_in, const double* in, long ldin,
                  long n_out, const double* pts_out, double* out, long ldout,
                  int nrhs, int nthreads, double* counts);

/* orc_butterfly, with the weights after one step copied to dump (a debugging
 * and test hook, so that a stage of another implementation can be compared
 * with this one's): dump_at = 0 after the initialisation (level 0), k in
 * 1..ls after column-space stage k-1 (level k), ls+1 after the middle switch
 * (level ls), k in ls+2..L+1 after row-space stage k-2 (level k-1), before
 * the final evaluation.  dump holds P * r * nrhs complex values (P = N^d):
 * [pair][t][rhs], pair = (a << d (L - lvl)) | b for the target box index a
 * (lvl bits per dimension, dimension j at bits lvl*j) and the source box
 * index b (L - lvl bits per dimension, likewise); t = sum_j t_j q^j.  The
 * weights are the equivalent sources of Sec. 1.2 up to the switch and the
 * potentials at the target nodes after it.  A step outside 0..L+1 leaves
 * dump untouched; the other arguments and the return codes are
 * orc_butterfly's. */
int orc_butterfly_dump(int d, long N, int q, int phase,
                       const double* slo, const double* shi,
                       const double* tlo, const double* thi,
                       int adjoint, int switch_level,
                       long n_in, const double* pts_in, const double* in, long ldin,
                       long n_out, const double* pts_out, double* out, long ldout,
                       int nrhs, int nthreads, int dump_at, double* dump);

#ifdef __cplusplus
}
#endif
#endif
