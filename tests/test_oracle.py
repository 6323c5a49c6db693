"""Pins for the CPU oracle (runs without a GPU).

Each test checks the oracle against something other than itself: a library
routine (numpy FFT, numpy's Chebyshev module), a closed form, hand-worked
phase values, an invariant, or brute force (the direct sum, which the
butterfly must approach as the Chebyshev order grows).
"""
import json
import os

import numpy as np
import numpy.polynomial.chebyshev as npcheb
import pytest

from paper_1305_4650_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

@pytest.mark.parametrize("q", [1, 2, 3, 5, 8, 13])
def test_nodes_are_roots_of_chebyshev_T(orc, q):
    """Chebyshev grid (Sec. 1.4, analytic interpolation): first-kind nodes are the
    roots of T_q, as computed by numpy's Chebyshev module."""
    z = np.sort(orc.nodes(q))
    roots = np.sort(npcheb.Chebyshev.basis(q).roots().real)
    assert np.allclose(z, roots, atol=1e-15, rtol=0)


def test_phase_handworked_values(orc):
    """Phase definitions (Sec. 3.1, Sec. 3.2, Fourier kernel of Sec. 3) at
    points worked out by hand."""
    with open(os.path.join(GOLDEN, "phase_handworked.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        got = orc.tau(c["phase"], c["N"], c["x"], c["y"])
        assert abs(got - c["tau"]) <= 1e-12 * max(1.0, abs(c["tau"])), (c, got)


def test_binning_grid_and_edges(orc):
    """Half-open boxes, grid points on a face go to the upper box, the upper
    domain face and points outside are clamped, NaN goes to leaf 0."""
    N = 16
    lo, hi = np.array([1.0, 0.0]), np.array([2.0, 1.0])
    k = W.grid_index(N, 2)
    pts = lo + k * ((hi - lo) / N)  # lower faces of every cell
    assert np.array_equal(orc.bin_points(pts, lo, hi, N), k)
    edge = np.array([[2.0, 1.0], [0.5, -3.0], [7.0, 0.99999], [np.nan, 0.5]])
    assert np.array_equal(orc.bin_points(edge, lo, hi, N), [[15, 15], [0, 0], [15, 15], [0, 8]])


# --------------------------------------------------------------------------
# direct sum (Eq. 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,N", [(1, 64), (2, 64), (3, 8)])
def test_direct_sum_is_inverse_dft(orc, d, N):
    """Phi = 2 pi x.y with y = j/N, x = k: the direct sum is N^d ifftn(g)."""
    w = W.fourier_grid(N, d=d, nrhs=3, config_id=11)
    f = orc.direct("fourier", N, w.y, w.g, w.x)
    shape = (N,) * d
    for s in range(3):
        # grid order has dim 0 fastest = last numpy axis
        ref = N ** d * np.fft.ifftn(w.g[s].reshape(shape)).reshape(-1)
        assert rel(f[s], ref) < 1e-12


def test_direct_sum_plane_wave_geometric_series(orc):
    """g_j = exp(-2 pi i nu.y_j) on the uniform grid: product of geometric
    series (1 - w^N)/(1 - w), w = exp(2 pi i (k - nu)/N); integer nu gives a
    Kronecker delta of height N^d."""
    N, d = 32, 2
    w = W.fourier_grid(N, d=d)
    for nu in (np.array([3.25, 7.6]), np.array([5.0, 11.0])):
        g = np.exp(-2j * np.pi * (w.y @ nu))
        f = orc.direct("fourier", N, w.y, g, w.x)[0]
        ref = np.ones(N ** d, dtype=complex)
        for j in range(d):
            kj = w.x[:, j]
            if float(nu[j]).is_integer():
                ref *= np.where(np.isclose((kj - nu[j]) % N, 0), N, 0)
            else:
                om = np.exp(2j * np.pi * (kj - nu[j]) / N)
                ref *= (1 - om ** N) / (1 - om)
        assert np.abs(f - ref).max() < 1e-10 * N ** d


@pytest.mark.parametrize("phase", ["hypradon2", "genradon3", "fourier", "separable", "genradon3pi"])
def test_direct_sum_delta_source(orc, phase):
    """g = delta at y_j0 gives f(x) = exp(i Phi(x, y_j0)) at every target."""
    mk = {"hypradon2": lambda: W.hypradon2(8), "genradon3": lambda: W.genradon3(4),
          "fourier": lambda: W.fourier_grid(8), "separable": lambda: W.separable(8),
          "genradon3pi": lambda: W.genradon3pi(4)}[phase]
    w = mk()
    j0 = 5
    g = np.zeros(w.y.shape[0], complex)
    g[j0] = 1.0
    f = orc.direct(phase, w.N, w.y, g, w.x)[0]
    taus = np.array([orc.tau(phase, w.N, x, w.y[j0]) for x in w.x])
    ref = np.exp(2j * np.pi * (taus - np.rint(taus)))
    assert np.abs(f - ref).max() < 1e-15


@pytest.mark.parametrize("phase", ["hypradon2", "genradon3", "genradon3pi"])
def test_direct_sum_adjoint_identity(orc, phase):
    """<K g, f> = <g, K^H f>: pins the sign and the role swap of the adjoint."""
    w = {"hypradon2": lambda: W.hypradon2(8), "genradon3": lambda: W.genradon3(4),
         "genradon3pi": lambda: W.genradon3pi(4)}[phase]()
    fvec = W.random_rhs(W.rng(77, 1), 1, w.x.shape[0])
    Kg = orc.direct(phase, w.N, w.y, w.g, w.x)
    KHf = orc.direct(phase, w.N, w.x, fvec, w.y, adjoint=True)
    lhs = np.vdot(fvec, Kg)
    rhs = np.vdot(KHf, w.g)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs) * 10


def test_genradon3pi_axis_sources_are_half_frequency_sum(orc):
    """Sources on the p2 axis (p0 = p1 = 0) make gamma = kappa = 0, so the
    printed phase pi (x.p + sqrt(gamma^2 + kappa^2)) is pi x2 p2: with p2 =
    j - N/2, x2 = k/N and g = 1 the sum is a geometric series in
    w = exp(i pi k / N), the same for every x0, x1.  Pins the factor pi (not
    2 pi) and the x.p term."""
    N = 8
    p2 = np.arange(N, dtype=float) - N / 2
    y = np.stack([np.zeros(N), np.zeros(N), p2], axis=1)
    gen = W.rng(61, 0)
    k = np.arange(1, 2 * N, dtype=float)  # k = 0 and 2N would make w = 1
    x = np.stack([gen.random(k.size), gen.random(k.size), k / N], axis=1)
    f = orc.direct("genradon3pi", N, y, np.ones((1, N), complex), x)[0]
    w = np.exp(1j * np.pi * k / N)
    ref = np.exp(-1j * np.pi * k / 2) * (1 - w ** N) / (1 - w)
    assert np.abs(f - ref).max() < 1e-12


def test_hypradon_row_reduces_to_1d_dft(orc):
    """Sources on the row y1 = 0 of the hyperbolic-Radon grid see tau = N x0 y0,
    and with y0 = 1 + j/N, x0 = k/N this is a 1-D inverse DFT in k0 (times
    exp(2 pi i k0) = 1), the same for every k1."""
    N = 32
    w = W.hypradon2(N)
    y = W.grid_points(N, w.src_lo, w.src_hi)  # unjittered
    row = np.where(W.grid_index(N, 2)[:, 1] == 0)[0]
    g = np.zeros(N * N, complex)
    g[row] = w.g[0, :N]
    f = orc.direct("hypradon2", N, y, g, w.x)[0].reshape(N, N)  # [k1, k0]
    ref = N * np.fft.ifft(w.g[0, :N])
    for k1 in range(N):
        assert rel(f[k1], ref) < 1e-12


# --------------------------------------------------------------------------
# butterfly (Alg. "alg:serial" + analytic interpolation)
# --------------------------------------------------------------------------

def test_butterfly_operation_counts(orc):
    """Exact counts of the dense form: phase evaluations
    n_src + n_tgt + P (2r + L (2^d+1) r + r^2); real x complex MACs
    (n_src + n_tgt) r + P L 2^d r^2; switch complex MACs P r^2 (Sec. 1 and
    Sec. 1.1: O(r N^d) ends, O(r^2 N^d) per stage, log2 N stages)."""
    for w in (W.fourier_grid(16, d=1, q=4), W.hypradon2(8, q=3), W.genradon3(4, q=2),
              W.fourier_grid(1, d=2, q=3)):
        _, c = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g, w.x,
                             return_counts=True)
        d, N, q = w.d, w.N, w.q
        r, P, L = q ** d, N ** d, int(np.log2(N))
        n = w.y.shape[0] + w.x.shape[0]
        assert c["phase"] == n + P * (2 * r + L * (2 ** d + 1) * r + r * r)
        assert c["mac"] == n * r + P * L * 2 ** d * r * r
        assert c["cmac"] == P * r * r
        assert c["stages"] == L


def test_butterfly_cost_grows_as_Nd_logN(orc):
    """Operation count per point grows like log N (O(r^2 N^d log N) overall)."""
    prev = None
    for N in (8, 16, 32, 64):
        w = W.fourier_grid(N, d=2, q=3)
        _, c = orc.butterfly("fourier", N, 3, w.src_box, w.tgt_box, w.y, w.g, w.x,
                             return_counts=True)
        per_point_per_stage = (c["mac"] - 2 * N * N * 9) / (N * N * np.log2(N))
        if prev is not None:
            assert per_point_per_stage == prev
        prev = per_point_per_stage


@pytest.mark.parametrize("phase", ["separable"])
@pytest.mark.parametrize("d,N,q", [(1, 32, 2), (2, 16, 3), (3, 4, 2), (2, 1, 4)])
def test_butterfly_exact_for_separable_phase(orc, phase, d, N, q):
    """Phi = a(x) + b(y): every interpolated factor is constant in the
    interpolation variable and the Lagrange basis sums to one, so the
    butterfly reproduces the direct sum to rounding."""
    w = W.separable(N, d=d, q=q)
    fb = orc.butterfly(phase, N, q, w.src_box, w.tgt_box, w.y, w.g, w.x)
    fd = orc.direct(phase, N, w.y, w.g, w.x)
    assert rel(fb, fd) < 1e-13
    gb = orc.butterfly(phase, N, q, w.src_box, w.tgt_box, w.x, fd, w.y, adjoint=True)
    gd = orc.direct(phase, N, w.x, fd, w.y, adjoint=True)
    assert rel(gb, gd) < 1e-13


def _cheb_interp_eval(vals, pts_ref):
    """Tensor Chebyshev interpolant through first-kind nodes (numpy's
    chebpts1 ordering), evaluated at reference points in [-1,1]^k.
    vals has one axis of length q per variable."""
    k = vals.ndim
    q = vals.shape[0]
    z = npcheb.chebpts1(q)
    Vinv = np.linalg.inv(npcheb.chebvander(z, q - 1))
    C = vals
    for ax in range(k):
        C = np.moveaxis(np.tensordot(Vinv, C, axes=([1], [ax])), 0, ax)
    out = np.empty(pts_ref.shape[0], complex)
    for i, p in enumerate(pts_ref):
        v = C
        for ax in range(k):
            v = np.tensordot(npcheb.chebvander(np.array([p[ax]]), q - 1)[0], v, axes=([0], [0]))
        out[i] = v
    return out


@pytest.mark.parametrize("phase,d,q", [("hypradon2", 2, 4), ("fourier", 1, 6), ("fourier", 2, 3),
                                     ("genradon3pi", 3, 3)])
def test_butterfly_N1_is_two_sided_chebyshev_interpolation(orc, phase, d, q):
    """With N = 1 there are no stages: init, switch, final.  The result is the
    kernel exp(i(Phi(x,c_Y) + Phi(c_X,y))) times the two-sided tensor
    Chebyshev interpolant of h(x,y) = exp(i(Phi(x,y) - Phi(x,c_Y) - Phi(c_X,y))),
    computed here with numpy's Chebyshev series (chebpts1 / chebvander)."""
    gen = W.rng(123, 0)
    if phase == "hypradon2":
        slo, shi, tlo, thi = np.array([1.0, 0.0]), np.array([2.0, 1.0]), np.zeros(2), np.ones(2)
        Nphase = 1
    else:
        slo, shi, tlo, thi = np.zeros(d), np.ones(d), np.zeros(d), np.full(d, 0.7)
        Nphase = 1
    ns, nt = 7, 5
    y = slo + gen.random((ns, d)) * (shi - slo)
    x = tlo + gen.random((nt, d)) * (thi - tlo)
    g = W.random_rhs(gen, 1, ns)
    fb = orc.butterfly(phase, 1, q, (slo, shi), (tlo, thi), y, g, x)[0]

    cY, cX = (slo + shi) / 2, (tlo + thi) / 2
    hY, hX = (shi - slo) / 2, (thi - tlo) / 2
    z = npcheb.chebpts1(q)
    grids_x = [cX[j] + hX[j] * z for j in range(d)]
    grids_y = [cY[j] + hY[j] * z for j in range(d)]
    t = lambda a, b: orc.tau(phase, Nphase, np.asarray(a, float), np.asarray(b, float))
    # h at all node pairs: axes (x_0..x_{d-1}, y_0..y_{d-1})
    shape = (q,) * (2 * d)
    H = np.empty(shape, complex)
    for idx in np.ndindex(*shape):
        xv = [grids_x[j][idx[j]] for j in range(d)]
        yv = [grids_y[j][idx[d + j]] for j in range(d)]
        H[idx] = np.exp(2j * np.pi * (t(xv, yv) - t(xv, cY) - t(cX, yv)))
    ref = np.zeros(nt, complex)
    for i in range(nt):
        pts = np.concatenate([(x[i] - cX) / hX, np.zeros(d)])[None, :]
        kern = np.empty(ns, complex)
        for jj in range(ns):
            pts[0, d:] = (y[jj] - cY) / hY
            kern[jj] = _cheb_interp_eval(H, pts)[0] * np.exp(
                2j * np.pi * (t(x[i], cY) + t(cX, y[jj])))
        ref[i] = kern @ g[0]
    assert rel(fb, ref) < 1e-13


@pytest.mark.parametrize("mk,tol", [
    (lambda q: W.fourier_grid(16, d=1, q=q), 1e-11),
    (lambda q: W.fourier_grid(8, d=2, q=q), 1e-9),
    (lambda q: W.hypradon2(16, q=q), 1e-11),
])
def test_butterfly_converges_to_direct_sum(orc, mk, tol):
    """The butterfly approximates the direct sum with an error set by the
    Chebyshev order (Sec. 1: error <= eps ||g||_1 with eps(r) decreasing).
    Monotone decrease in q, reaching near machine precision: any wrong
    index, sign or table entry would stall the convergence."""
    errs = []
    for q in (2, 4, 6, 8, 10, 12, 15):
        w = mk(q)
        fb = orc.butterfly(w.phase, w.N, q, w.src_box, w.tgt_box, w.y, w.g, w.x)
        fd = orc.direct(w.phase, w.N, w.y, w.g, w.x)
        gb = orc.butterfly(w.phase, w.N, q, w.src_box, w.tgt_box, w.x, fd, w.y, adjoint=True)
        gd = orc.direct(w.phase, w.N, w.x, fd, w.y, adjoint=True)
        errs.append((rel(fb, fd), rel(gb, gd)))
    e = np.array(errs)
    assert np.all(np.diff(e[:, 0]) < 0) and np.all(np.diff(e[:, 1]) < 0), e
    assert e[-1, 0] < tol and e[-1, 1] < tol, e


def test_butterfly_genradon_error_decreases(orc):
    """The 3-D generalized-Radon phase has a square-root cone at y = 0 (a
    corner of the source box), so convergence is slow; it must still decrease."""
    errs = []
    for q in (2, 4, 6, 8):
        w = W.genradon3(4, q=q)
        fb = orc.butterfly(w.phase, w.N, q, w.src_box, w.tgt_box, w.y, w.g, w.x)
        fd = orc.direct(w.phase, w.N, w.y, w.g, w.x)
        errs.append(rel(fb, fd))
    assert np.all(np.diff(errs) < 0), errs


def test_butterfly_genradon3pi_error_decreases(orc):
    """The printed generalized-Radon phase has its square-root cone at p0 = p1
    = 0, inside the source box: convergence in q is slow but monotone."""
    errs = []
    for q in (2, 3, 4, 5, 6):
        w = W.genradon3pi(4, q=q)
        fb = orc.butterfly(w.phase, w.N, q, w.src_box, w.tgt_box, w.y, w.g, w.x)
        fd = orc.direct(w.phase, w.N, w.y, w.g, w.x)
        errs.append(rel(fb, fd))
    assert np.all(np.diff(errs) < 0), errs


def test_butterfly_genradon3pi_matches_stated_accuracy(orc):
    """Sec. 3.2 chooses r = 5^3 for roughly one percent relative error in the
    supremum norm.  With the printed phase, q = 5 and N = 16 the oracle's
    sup-norm error relative to max |f| lies between 0.5% and 3% (1.9%); the
    phase at twice or half its scale, or a dropped term, leaves that band."""
    w = W.genradon3pi(16, q=5)
    fb = orc.butterfly(w.phase, w.N, 5, w.src_box, w.tgt_box, w.y, w.g, w.x)
    fd = orc.direct(w.phase, w.N, w.y, w.g, w.x)
    e = np.abs(fb - fd).max() / np.abs(fd).max()
    assert 5e-3 < e < 3e-2, e


@pytest.mark.parametrize("mk", [
    lambda: W.hypradon2(8, q=3), lambda: W.hypradon2(32, q=4), lambda: W.hypradon2(16, q=3),
    lambda: W.fourier_grid(32, d=1, q=5), lambda: W.fourier_grid(2, d=2, q=4), lambda: W.genradon3(8, q=2),
    lambda: W.genradon3pi(2, q=3), lambda: W.hypradon2(1, q=4)])
def test_butterfly_adjoint_is_exact_transpose(orc, mk):
    """<B g, f> = <g, B' f> to rounding for the butterfly B and the adjoint
    butterfly B' at odd and even L (N = 1 ... 32): with the adjoint's switch
    at L - floor(L/2) every step of B' is the transpose of a step of B (in
    the demodulated variables), so B' = B^H exactly, not only up to the
    interpolation error.  Any transposed table, wrong node, sign or
    modulation centre in either direction breaks the identity at O(1)."""
    w = mk()
    fvec = W.random_rhs(W.rng(w.config_id, 2), 1, w.x.shape[0])
    Bg = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g, w.x)
    Bf = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.x, fvec, w.y, adjoint=True)
    lhs, rhs = np.vdot(fvec, Bg), np.vdot(Bf, w.g)
    scale = np.linalg.norm(fvec) * np.linalg.norm(Bg)
    assert abs(lhs - rhs) < 1e-14 * scale, (lhs, rhs)


def test_butterfly_linearity(orc):
    w = W.hypradon2(16, q=4, nrhs=2)
    a, b = 0.3 - 1.2j, 2.5 + 0.1j
    f = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g, w.x)
    fc = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y,
                       a * w.g[0] + b * w.g[1], w.x)[0]
    assert rel(fc, a * f[0] + b * f[1]) < 1e-14


def test_butterfly_multi_rhs_matches_single(orc):
    w = W.hypradon2(8, q=3, nrhs=3)
    f = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g, w.x)
    for s in range(3):
        fs = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g[s], w.x)[0]
        assert np.array_equal(fs, f[s])


def test_butterfly_switch_level_variants_agree_to_eps(orc):
    """Any switch level gives a valid butterfly; variants differ by O(eps_q)."""
    w = W.fourier_grid(16, d=2, q=8)
    fd = orc.direct(w.phase, w.N, w.y, w.g, w.x)
    for ls in range(0, 5):
        fb = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g, w.x,
                           switch_level=ls)
        assert rel(fb, fd) < 1e-3


def test_butterfly_points_anywhere_in_leaves(orc):
    """Empty leaves and leaves with several points (CSR semantics): the
    butterfly still approximates the direct sum."""
    gen = W.rng(99, 0)
    N, q = 8, 10
    slo, shi, tlo, thi = np.array([1.0, 0.0]), np.array([2.0, 1.0]), np.zeros(2), np.ones(2)
    y = slo + gen.random((37, 2)) ** 2 * (shi - slo)   # clustered, uneven
    x = tlo + gen.random((23, 2)) * (thi - tlo)
    g = W.random_rhs(gen, 2, 37)
    fb = orc.butterfly("hypradon2", N, q, (slo, shi), (tlo, thi), y, g, x)
    fd = orc.direct("hypradon2", N, y, g, x)
    assert rel(fb, fd) < 1e-6


def test_butterfly_empty_inputs(orc):
    w = W.hypradon2(4, q=3)
    out = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y[:0], np.zeros((1, 0)), w.x)
    assert np.all(out == 0)
    out = orc.butterfly(w.phase, w.N, w.q, w.src_box, w.tgt_box, w.y, w.g, w.x[:0])
    assert out.shape == (1, 0)


def test_oracle_rejects_bad_arguments(orc):
    w = W.hypradon2(4, q=3)
    with pytest.raises(ValueError):
        orc.butterfly(w.phase, 6, 3, w.src_box, w.tgt_box, w.y, w.g, w.x)  # N not 2^k
    with pytest.raises(ValueError):
        orc.butterfly("genradon3", 4, 3, w.src_box, w.tgt_box, w.y, w.g, w.x)  # d mismatch
