"""Pins of the oracle's stencil, weights and mode basis against closed forms.

Each test checks the FP64 oracle against something fixed independently of it:
the Cox-de Boor B-spline of scipy, exact-rational moment identities, the
orthogonality that Eq. 14 is built to give (section 3.3), or hand-worked values.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import polypic_oracle as O

T_GRID = [Fr(k, 64) for k in range(-32, 32)]  # t in [-1/2, 1/2) on a dyadic grid


def _fr(v) -> Fr:
    return Fr(float(np.asarray(v).reshape(-1)[0]))


def test_bspline_is_cox_de_boor_quadratic():
    """N(d) equals the degree-2 cardinal B-spline on knots -3/2..3/2 (scipy)."""
    ref = BSpline.basis_element([-1.5, -0.5, 0.5, 1.5], extrapolate=False)
    d = np.random.default_rng(0).uniform(-1.499, 1.499, 2000)
    np.testing.assert_allclose(O.quadratic_bspline(d), ref(d), rtol=0, atol=1e-15)
    assert float(O.quadratic_bspline(1.5)) == 0.0 and float(O.quadratic_bspline(-2.0)) == 0.0


@pytest.mark.parametrize("t", T_GRID)
def test_weight_moments_exact(t):
    """P-1: sum w = 1, sum w z = 0, sum w z^2 = 1/4, sum w z^3 = t (1 - 4 t^2) / 4."""
    w = [_fr(v) for v in O.weights_1d(np.array([float(t)]))]
    z = [_fr(v) for v in O.node_offsets(np.array([float(t)]))]
    assert sum(w) == 1
    assert sum(wj * zj for wj, zj in zip(w, z)) == 0
    assert sum(wj * zj ** 2 for wj, zj in zip(w, z)) == Fr(1, 4)
    assert sum(wj * zj ** 3 for wj, zj in zip(w, z)) == t * (1 - 4 * t * t) / 4
    # closed forms of the three weights (appendix-style): (1-2t)^2/8, 3/4 - t^2, (1+2t)^2/8
    assert w == [(1 - 2 * t) ** 2 / 8, Fr(3, 4) - t * t, (1 + 2 * t) ** 2 / 8]


@pytest.mark.parametrize("t", T_GRID)
def test_ghat_orthogonal_and_monic(t):
    """P-2: sum w ghat = sum w ghat z = 0 and ghat is monic in z (second difference 2).

    Three conditions fix a monic quadratic uniquely, so this pins Eq. 14's reading.
    """
    tt = np.array([float(t)])
    w = [_fr(v) for v in O.weights_1d(tt)]
    z = [_fr(v) for v in O.node_offsets(tt)]
    g = [_fr(v) for v in O.ghat_1d(tt)]
    assert abs(sum(wj * gj for wj, gj in zip(w, g))) < Fr(1, 10 ** 15)
    assert abs(sum(wj * gj * zj for wj, gj, zj in zip(w, g, z))) < Fr(1, 10 ** 15)
    assert abs(g[0] - 2 * g[1] + g[2] - 2) < Fr(1, 10 ** 14)


def test_ghat_sign_is_forced():
    """With the opposite sign of a (Eq. 14's middle term) orthogonality to z fails."""
    for t in [Fr(1, 8), Fr(-3, 16), Fr(5, 16)]:
        z = [Fr(j - 1) - t for j in range(3)]
        w = [(1 - 2 * t) ** 2 / 8, Fr(3, 4) - t * t, (1 + 2 * t) ** 2 / 8]
        a = t * (1 - 4 * t * t)
        good = [zj * zj - a * zj - Fr(1, 4) for zj in z]
        bad = [zj * zj + a * zj - Fr(1, 4) for zj in z]
        assert sum(wj * gj * zj for wj, gj, zj in zip(w, good, z)) == 0
        assert sum(wj * gj * zj for wj, gj, zj in zip(w, bad, z)) != 0


@pytest.mark.parametrize("t", T_GRID)
def test_ghat_norm_and_cancellation(t):
    """P-3: ||ghat||_w^2 = (1-4t^2)^2 (3-4t^2)/16 and w_j ghat_j = K (1, -2, 1)."""
    tt = np.array([float(t)])
    w = [_fr(v) for v in O.weights_1d(tt)]
    g = [_fr(v) for v in O.ghat_1d(tt)]
    K = (1 - 4 * t * t) ** 2 * (3 - 4 * t * t) / 32
    norm = sum(wj * gj * gj for wj, gj in zip(w, g))
    assert abs(norm - (1 - 4 * t * t) ** 2 * (3 - 4 * t * t) / 16) < Fr(1, 10 ** 14)
    for j, dj in enumerate((1, -2, 1)):
        assert abs(w[j] * g[j] - K * dj) < Fr(1, 10 ** 15)
    q = O.projection_weights_1d(tt)
    assert [float(v[0]) for v in q[2]] == [1.0, -2.0, 1.0]


def test_stencil_hand_values():
    """Base node / offset on a dx = 1/32 grid: u = 10 -> (b 9, t 0); u = 10.5 -> (10, -1/2)."""
    g = O.Grid(36, 36, 36, 1 / 32, 32.0)
    x = np.array([[10 / 32, 10.5 / 32, np.float32(10.5 / 32) - np.float32(2 ** -24)]] * 3,
                 np.float32)
    b, t = O.stencil_base(g, x)
    assert list(b[0]) == [9, 10, 9]
    assert t[0, 0] == 0.0 and t[0, 1] == -0.5
    assert 0.4999 < t[0, 2] < 0.5


def test_stencil_uses_float32_rounding():
    """With inv_dx = 3, x = fl32(2.5 / 3) gives fl32(x * 3) = 2.5 exactly (b = 2, t = -1/2)
    although the exact product is just below 2.5 (which would give b = 1, t ~ +1/2)."""
    g = O.Grid(10, 10, 10, 1 / 3, 3.0)
    x32 = np.float32(2.5 / 3.0)
    assert Fr(float(x32)) * 3 < Fr(5, 2)
    b, t = O.stencil_base(g, np.full((3, 1), x32, np.float32))
    assert b[0, 0] == 2 and t[0, 0] == -0.5


def test_stencil_invariants_random():
    """For arbitrary origin / inv_dx: t in [-1/2, 1/2) and node b+1 is nearest to u."""
    rng = np.random.default_rng(3)
    g = O.Grid(200, 200, 200, 1 / 7.3, 7.3, (0.11, -0.27, 0.5))
    x = (np.array(g.origin)[:, None] + rng.uniform(2, 190, (3, 5000)) / 7.3).astype(np.float32)
    b, t = O.stencil_base(g, x)
    assert np.all(t >= -0.5) and np.all(t < 0.5)
    u = (x - np.float32(0) - np.array(g.origin, np.float32)[:, None]) * np.float32(7.3)
    assert np.all(np.abs(u.astype(np.float64) - (b + 1)) <= 0.5)


def test_morton_hand_values():
    """Bit k of b_x, b_y, b_z -> key bits 3k, 3k+1, 3k+2."""
    b = np.array([[1, 0, 0, 3, 2, 5, 257], [0, 1, 0, 0, 2, 3, 0], [0, 0, 1, 0, 2, 6, 1]])
    keys = O.morton_key(b)
    # (5,3,6): x=101 y=011 z=110 -> bit0: x1 y1 z0 -> 011 = 3; bit1: x0 y1 z1 -> 110 = 6;
    # bit2: x1 y0 z1 -> 101 = 5  => key = 3 + 6*8 + 5*64 = 371
    assert list(keys) == [1, 2, 4, 9, 56, 371, (1 << 24) | (1 << 2) | 1]


def _less_msb(p, q):
    """Z-order comparison by the most significant differing bit (no interleaving)."""
    best_axis, best_x = 0, 0
    for a in (2, 1, 0):  # z is the most significant of the three at equal bit level
        x = p[a] ^ q[a]
        if x and (best_x == 0 or (x.bit_length() > best_x.bit_length())):
            best_axis, best_x = a, x
    # ties at the same bit level: higher axis wins, handled by the scan order above
    return p[best_axis] < q[best_axis]


def test_morton_order_matches_msb_comparison():
    rng = np.random.default_rng(1)
    b = rng.integers(0, 300, (3, 400))
    keys = O.morton_key(b)
    pts = [tuple(int(v) for v in b[:, i]) for i in range(b.shape[1])]
    for i in range(0, 400, 2):
        p, q = pts[i], pts[i + 1]
        if p == q:
            assert keys[i] == keys[i + 1]
        else:
            assert (keys[i] < keys[i + 1]) == _less_msb(p, q)


def test_sort_is_stable_argsort():
    """P-15: sorted keys ascending; equal keys keep input order; perm is a permutation."""
    rng = np.random.default_rng(2)
    g = O.Grid(20, 20, 20, 1 / 16, 16.0)
    x = rng.uniform(3 / 16, 17 / 16, (3, 3000)).astype(np.float32)
    keys, perm = O.sort_keys(g, x)
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    assert sorted(perm.tolist()) == list(range(3000))
    same = keys[1:] == keys[:-1]
    assert np.all(perm[1:][same] > perm[:-1][same])


def _u32(x32, inv_dx):
    """u = fl32(x * inv_dx) for a float32 x and a power-of-two inv_dx (exact)."""
    return Fr(float(np.float32(x32) * np.float32(inv_dx)))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_stencil_range_check_at_the_switches(axis):
    """The 3-node stencil of the quadratic B-spline (section 3.1: support |d| < 3/2) must
    lie inside the N storage nodes of every axis.

    The stencil is the nearest node c and its two neighbours, with c = floor(u + 1/2)
    (a tie at u = k + 1/2 goes up), so it fits iff 1 <= c <= N - 2, i.e.
    0 <= b <= N - 3 with b = c - 1.  Positions sit exactly at the switches
    u = k + 1/2 and one float32 below them, on each axis in turn: b = 0 and b = N - 3
    are accepted, b = -1 and b = N - 2 rejected, and every oracle entry point raises
    OracleRangeError exactly for the rejected ones.  Independently of the oracle's b,
    the test checks in exact rationals that every lattice node with a nonzero B-spline
    weight lies in {c - 1, c, c + 1}.
    """
    n = 12
    inv = 8.0
    g = O.Grid(n, n, n, 1 / inv, inv)
    below = lambda v: np.nextafter(np.float32(v), np.float32(-np.inf))
    u_cases = [  # (u as float32, expected in range)
        (np.float32(0.5), True),            # b = 0, t = -1/2
        (below(0.5), False),                # b = -1
        (np.float32(n - 1.5), False),       # b = N - 2, t = -1/2
        (below(n - 1.5), True),             # b = N - 3, t just below 1/2
        (np.float32(5.0), True),
    ]
    P = len(u_cases)
    x = np.full((3, P), np.float32(5.0 / inv), np.float32)
    for i, (u, _) in enumerate(u_cases):
        x[axis, i] = np.float32(u) / np.float32(inv)   # exact: inv is a power of two
    expect = np.array([ok for _, ok in u_cases])
    b, _ = O.stencil_base(g, x)
    np.testing.assert_array_equal(b[axis], [0, -1, n - 2, n - 3, 4])
    np.testing.assert_array_equal(O.stencil_in_range(g, b), expect)

    for i, (u32, ok) in enumerate(u_cases):
        u = _u32(x[axis, i], inv)
        c = (u + Fr(1, 2)).__floor__()
        assert (1 <= c <= n - 2) == ok
        support = [k for k in range(-4, n + 4)
                   if float(O.quadratic_bspline(float(u - k))) > 0.0]
        assert set(support) <= {c - 1, c, c + 1}, (u, support, c)

    coeff = np.zeros((3, 1, 1), np.float32)
    vel = np.zeros((3, n, n, n))
    for i, (_, ok) in enumerate(u_cases):
        xi = x[:, i:i + 1]
        calls = [lambda: O.sort_keys(g, xi), lambda: O.p2g(g, xi, coeff, 1),
                 lambda: O.g2p(g, vel, xi, 1)]
        for call in calls:
            if ok:
                call()
            else:
                with pytest.raises(O.OracleRangeError):
                    call()
