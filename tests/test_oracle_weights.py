"""Pins for the oracle's per-step weights (its debugging hook).

Every stage of the butterfly maps the weights of one level to the next by a
formula with an exact algebraic consequence, checked here on the dumps of
two consecutive steps with numpy's Chebyshev module standing in for the
oracle's own Lagrange basis:

* a column-space stage (Sec. 1.2-1.3) interpolates equivalent sources on the
  merged source box's Chebyshev grid, which keeps every moment of degree
  below q per dimension of the modulated sources;
* the middle switch (Sec. 1.4) is a dense sum over the q^d x q^d node pairs;
* a row-space stage (Sec. 1.3-1.4) evaluates the parent's demodulated
  interpolant at the child's nodes;
* the final evaluation (Sec. 1) interpolates the last weights at the target.

A single source must also leave nonzero weights only in the pairs whose
source box holds it.
"""
import itertools

import numpy as np
import numpy.polynomial.chebyshev as npcheb
import pytest

CASES = [
    # phase, d, N, q, switch level (-1: the default), adjoint
    ("hypradon2", 2, 16, 4, -1, False),
    ("fourier", 1, 64, 5, -1, False),
    ("fourier", 2, 8, 3, 1, False),
    ("genradon3", 3, 4, 3, -1, False),
    # odd L, where the adjoint's mirror switch level differs from floor(L/2)
    ("hypradon2", 2, 32, 3, -1, True),
    ("fourier", 1, 128, 5, -1, True),
    ("genradon3", 3, 8, 3, -1, True),
]


class Geo:
    """Box geometry of the dumps: level-lvl target boxes split the target box
    into 2^lvl per dimension, source boxes into 2^(L-lvl)."""

    def __init__(self, orc, phase, d, N, q, sw, adjoint, rng):
        self.orc, self.phase, self.d, self.N, self.q = orc, phase, d, N, q
        self.adjoint = adjoint
        self.L = N.bit_length() - 1
        # the adjoint's default switch is the mirror level L - floor(L/2)
        self.ls = (self.L - self.L // 2 if adjoint else self.L // 2) if sw < 0 else sw
        self.sw = sw
        self.slo = rng.uniform(-0.5, 0.2, d)
        self.shi = self.slo + rng.uniform(0.6, 1.2, d)
        self.tlo = rng.uniform(-0.3, 0.4, d)
        self.thi = self.tlo + rng.uniform(0.5, 1.0, d)
        self.z = orc.nodes(q)
        self.r = q ** d
        # node multi-indices, dimension 0 fastest
        self.tidx = np.array([[(t // q ** j) % q for j in range(d)] for t in range(self.r)])

    def level(self, step):
        if step <= self.ls:
            return step
        return step - 1

    def split(self, lvl, pair):
        lb = self.L - lvl
        a, b = pair >> (self.d * lb), pair & ((1 << (self.d * lb)) - 1)
        av = [(a >> (lvl * j)) & ((1 << lvl) - 1) for j in range(self.d)]
        bv = [(b >> (lb * j)) & ((1 << lb) - 1) for j in range(self.d)]
        return np.array(av), np.array(bv)

    def join(self, lvl, av, bv):
        lb = self.L - lvl
        a = sum(int(av[j]) << (lvl * j) for j in range(self.d))
        b = sum(int(bv[j]) << (lb * j) for j in range(self.d))
        return (a << (self.d * lb)) | b

    def tbox(self, lvl, av):
        w = (self.thi - self.tlo) / 2 ** lvl
        return self.tlo + (av + 0.5) * w, w

    def sbox(self, lvl, bv):
        w = (self.shi - self.slo) / 2 ** (self.L - lvl)
        return self.slo + (bv + 0.5) * w, w

    def grid(self, c, w):
        return c + 0.5 * w * self.z[self.tidx]

    def plan_boxes(self):
        """(source box, target box) of the plan: the roles' boxes, swapped
        for the adjoint (its sources lie in the plan's target box)."""
        roles = ((self.slo, self.shi), (self.tlo, self.thi))
        return roles[::-1] if self.adjoint else roles

    def e(self, x, y):
        """The kernel between target-role x and source-role y, one of them a
        single point: e^{i Phi(x, y)}, or for the adjoint e^{-i Phi(y, x)}."""
        x, y = np.atleast_2d(x), np.atleast_2d(y)
        if len(x) == 0 or len(y) == 0:
            return np.zeros(0, dtype=complex)
        n = max(len(x), len(y))
        x = np.broadcast_to(x, (n, self.d))
        y = np.broadcast_to(y, (n, self.d))
        if self.adjoint:
            tau = -np.array([self.orc.tau(self.phase, self.N, yi, xi) for xi, yi in zip(x, y)])
        else:
            tau = np.array([self.orc.tau(self.phase, self.N, xi, yi) for xi, yi in zip(x, y)])
        return np.exp(2j * np.pi * (tau - np.rint(tau)))

    def interp(self, c, w, vals, x):
        """Tensor Chebyshev interpolant through (grid(c, w), vals) at rows x,
        by a Chebyshev-Vandermonde solve (numpy's basis, not the oracle's)."""
        u = (x - c) / (0.5 * w)

        def vand(pts):
            V = np.ones((len(pts), self.r))
            for j in range(self.d):
                V *= npcheb.chebvander(pts[:, j], self.q - 1)[:, self.tidx[:, j]]
            return V

        coef = np.linalg.solve(vand(self.z[self.tidx]), vals)
        return vand(u) @ coef

    def weights(self, pts, g, step):
        return self.orc.butterfly_weights(self.phase, self.N, self.q, *self.plan_boxes(), pts, g, step,
                                          adjoint=self.adjoint, switch_level=self.sw)


def make(orc, case, seed, n=300, nrhs=2):
    rng = np.random.default_rng(seed)
    geo = Geo(orc, *case, rng)
    pts = geo.slo + (geo.shi - geo.slo) * rng.random((n, geo.d))
    g = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    return geo, pts, g


def monomials(geo, c, w, y):
    """(q^d, len(y)) products of (scaled coordinate)^m_j, m_j < q."""
    u = (y - c) / (0.5 * w)
    M = np.ones((geo.r, len(y)))
    for j in range(geo.d):
        M *= u[:, j][None, :] ** geo.tidx[:, j][:, None]
    return M


def close(a, b, scale, tol=1e-11):
    err = np.max(np.abs(a - b))
    assert err <= tol * scale, (err, scale)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}_d{c[1]}_N{c[2]}_q{c[3]}_s{c[4]}{'_adj' if c[5] else ''}")
def test_single_source_support(orc, case):
    geo, pts, g = make(orc, case, 11, n=1, nrhs=1)
    leaf = orc.bin_points(pts, geo.slo, geo.shi, geo.N)[0]
    for step in range(geo.L + 2):
        lvl = geo.level(step)
        w = geo.weights(pts, g, step)
        nz = np.flatnonzero(np.any(w != 0, axis=(1, 2)))
        want = sorted(geo.join(lvl, np.array(av), leaf >> lvl)
                      for av in itertools.product(range(2 ** lvl), repeat=geo.d))
        assert len(want) == 2 ** (geo.d * lvl)
        assert nz.tolist() == want, step


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}_d{c[1]}_N{c[2]}_q{c[3]}_s{c[4]}{'_adj' if c[5] else ''}")
def test_initialisation_keeps_moments(orc, case):
    """Step 0: sum_t y_t^m e^{i Phi(c_X, y_t)} delta_t equals the same moment of
    the leaf's own modulated sources, X the root target box."""
    geo, pts, g = make(orc, case, 12)
    w0 = geo.weights(pts, g, 0)
    leaves = orc.bin_points(pts, geo.slo, geo.shi, geo.N)
    cX, _ = geo.tbox(0, np.zeros(geo.d, dtype=int))
    for pair in range(geo.N ** geo.d):
        _, bv = geo.split(0, pair)
        c, w = geo.sbox(0, bv)
        inside = np.all(leaves == bv, axis=1)
        y = geo.grid(c, w)
        lhs = monomials(geo, c, w, y) @ (geo.e(cX, y)[:, None] * w0[pair])
        ys = pts[inside]
        rhs = monomials(geo, c, w, ys) @ (geo.e(cX, ys)[:, None] * g[:, inside].T)
        close(lhs, rhs, 1.0 + np.abs(g[:, inside]).sum())


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}_d{c[1]}_N{c[2]}_q{c[3]}_s{c[4]}{'_adj' if c[5] else ''}")
def test_column_stages_keep_moments(orc, case):
    """Column stage l -> l+1: for child target box A' of P and merged source box
    B' with children B_c, the modulated moments about c_A' of the new weights
    on B's grid equal those of the old weights of (P, B_c) on the children's grids."""
    geo, pts, g = make(orc, case, 13)
    prev = geo.weights(pts, g, 0)
    for step in range(1, geo.ls + 1):
        cur = geo.weights(pts, g, step)
        scale = np.abs(prev).sum(axis=(1, 2)).max()
        for pair in range(geo.N ** geo.d):
            av, bv = geo.split(step, pair)
            cA, _ = geo.tbox(step, av)
            cB, wB = geo.sbox(step, bv)
            y = geo.grid(cB, wB)
            lhs = monomials(geo, cB, wB, y) @ (geo.e(cA, y)[:, None] * cur[pair])
            rhs = 0
            for c in itertools.product((0, 1), repeat=geo.d):
                bc = 2 * bv + np.array(c)
                cc, wc = geo.sbox(step - 1, bc)
                yc = geo.grid(cc, wc)
                old = prev[geo.join(step - 1, av >> 1, bc)]
                rhs = rhs + monomials(geo, cB, wB, yc) @ (geo.e(cA, yc)[:, None] * old)
            close(lhs, rhs, scale * 2 ** geo.d * 4)
        prev = cur


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}_d{c[1]}_N{c[2]}_q{c[3]}_s{c[4]}{'_adj' if c[5] else ''}")
def test_switch_is_the_dense_node_sum(orc, case):
    geo, pts, g = make(orc, case, 14)
    before = geo.weights(pts, g, geo.ls)
    after = geo.weights(pts, g, geo.ls + 1)
    scale = np.abs(before).sum(axis=(1, 2)).max()
    for pair in range(geo.N ** geo.d):
        av, bv = geo.split(geo.ls, pair)
        x = geo.grid(*geo.tbox(geo.ls, av))
        y = geo.grid(*geo.sbox(geo.ls, bv))
        K = np.array([geo.e(xt, y) for xt in x])
        close(after[pair], K @ before[pair], scale)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}_d{c[1]}_N{c[2]}_q{c[3]}_s{c[4]}{'_adj' if c[5] else ''}")
def test_row_stages_interpolate_the_parent(orc, case):
    """Row stage l -> l+1: the weights of (A', B') at A's nodes x are
    sum_c e^{i Phi(x, c_Bc)} h_c(x), h_c the parent's interpolant of its
    weights of (P, B_c) demodulated by e^{-i Phi(x^P, c_Bc)}."""
    geo, pts, g = make(orc, case, 15)
    for step in range(geo.ls + 2, geo.L + 2):
        lvl = step - 2
        prev = geo.weights(pts, g, step - 1)
        cur = geo.weights(pts, g, step)
        scale = np.abs(prev).sum(axis=(1, 2)).max()
        for pair in range(geo.N ** geo.d):
            av, bv = geo.split(lvl + 1, pair)
            cA, wA = geo.tbox(lvl + 1, av)
            x = geo.grid(cA, wA)
            cP, wP = geo.tbox(lvl, av >> 1)
            xp = geo.grid(cP, wP)
            want = 0
            for c in itertools.product((0, 1), repeat=geo.d):
                bc = 2 * bv + np.array(c)
                cc, _ = geo.sbox(lvl, bc)
                old = prev[geo.join(lvl, av >> 1, bc)]
                h = geo.interp(cP, wP, np.conj(geo.e(xp, cc))[:, None] * old, x)
                want = want + geo.e(x, cc)[:, None] * h
            close(cur[pair], want, scale * 2 ** geo.d * 8, tol=1e-10)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}_d{c[1]}_N{c[2]}_q{c[3]}_s{c[4]}{'_adj' if c[5] else ''}")
def test_final_evaluation_of_the_last_weights(orc, case):
    """The apply's output at x in leaf A is e^{i Phi(x, c_Y)} times the leaf's
    interpolant of its last weights demodulated by e^{-i Phi(x^A_t, c_Y)},
    Y the root source box."""
    geo, pts, g = make(orc, case, 16)
    rng = np.random.default_rng(17)
    xs = geo.tlo + (geo.thi - geo.tlo) * rng.random((40, geo.d))
    out = orc.butterfly(geo.phase, geo.N, geo.q, *geo.plan_boxes(), pts, g, xs,
                        adjoint=geo.adjoint, switch_level=geo.sw)
    last = geo.weights(pts, g, geo.L + 1)
    cY, _ = geo.sbox(geo.L, np.zeros(geo.d, dtype=int))
    tleaf = orc.bin_points(xs, geo.tlo, geo.thi, geo.N)
    scale = np.abs(last).sum(axis=(1, 2)).max()
    for i, x in enumerate(xs):
        av = tleaf[i]
        cA, wA = geo.tbox(geo.L, av)
        xa = geo.grid(cA, wA)
        wv = last[geo.join(geo.L, av, np.zeros(geo.d, dtype=int))]
        h = geo.interp(cA, wA, np.conj(geo.e(xa, cY))[:, None] * wv, x[None, :])[0]
        close(out[:, i], geo.e(x, cY)[0] * h, scale * 8, tol=1e-10)


def test_last_weights_approach_the_potentials(orc):
    """After the last stage the weights are the potentials at the leaves'
    nodes, up to an interpolation error that decays spectrally with q (brute
    force: the direct sum at those nodes), for sources in [1,2]^2 and targets
    in [0,1]^2, where the phase is analytic."""
    errs = {}
    for q in (5, 7, 9, 11):
        rng = np.random.default_rng(18)
        geo = Geo(orc, "hypradon2", 2, 16, q, -1, False, rng)
        geo.slo, geo.shi = np.full(2, 1.0), np.full(2, 2.0)
        geo.tlo, geo.thi = np.zeros(2), np.ones(2)
        pts = geo.slo + rng.random((300, 2))
        g = rng.standard_normal((1, 300)) + 1j * rng.standard_normal((1, 300))
        last = geo.weights(pts, g, geo.L + 1)
        worst = 0.0
        for pair in rng.choice(geo.N ** geo.d, 12, replace=False):
            av, _ = geo.split(geo.L, pair)
            x = geo.grid(*geo.tbox(geo.L, av))
            ref = orc.direct(geo.phase, geo.N, pts, g, x)[0]
            worst = max(worst, np.linalg.norm(last[pair, :, 0] - ref) / np.linalg.norm(ref))
        errs[q] = worst
    assert errs[5] < 2e-2 and errs[11] < 1e-7, errs
    assert errs[5] > errs[7] > errs[9] > errs[11], errs
