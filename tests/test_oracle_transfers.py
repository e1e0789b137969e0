"""Pins of the oracle's P2G, grid update and G2P.

Each test checks the FP64 oracle against a fact fixed outside it: conservation
laws (Eq. 1-4 summed), textbook APIC (section 3.2 / Jiang et al.), the
interpolation system solved by numpy.linalg, exact reproduction of polynomial
fields, the lossless round trip the paper cites (abstract, section 5), PIC
(Eq. 1-8), closed forms, and the exact-rational golden fixture.
"""
import itertools
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import workloads as W
from oracle import polypic_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact.json")


def small_scene(seed=0, P=600, n=16, mass_random=True):
    """Random particles on a power-of-two grid, so that u * dx == x exactly."""
    s = W.random_scene(seed, n, P, n_lo=1, mass_random=mass_random)
    return s, O.grid_from_spec(s.grid)


def node_positions(g):
    iz, iy, ix = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx), indexing="ij")
    return [g.origin[0] + ix * g.dx, g.origin[1] + iy * g.dx, g.origin[2] + iz * g.dx]


def mode_eval(r, zh, t):
    """Mode r of Eq. 11 (quadratic factor per Eq. 14) at arbitrary zhat (3, ...) for offsets t."""
    out = 1.0
    for a, k in enumerate(O.MODES[r]):
        z = zh[a]
        if k == 1:
            out = out * z
        elif k == 2:
            aa = t[a] * (1 - 4 * t[a] ** 2)
            out = out * (z * z - aa * z - 0.25)
    return out


@pytest.mark.parametrize("n_modes", O.ALLOWED_N_MODES)
def test_mass_and_momentum_conserved(n_modes):
    """P-7: sum_i m_i = sum_p m_p and sum_i p_i = sum_p m_p c_p0 for every N_r."""
    s, g = small_scene()
    M, Q = O.p2g(g, s.x, s.coeff, n_modes, s.mass)
    m = s.mass.astype(np.float64)
    assert abs(M.sum() - m.sum()) < 1e-12 * m.sum()
    for a in range(3):
        ref = (m * s.coeff[a, 0].astype(np.float64)).sum()
        assert abs(Q[a].sum() - ref) < 1e-11 * np.abs(m).sum()


@pytest.mark.parametrize("n_modes", O.ALLOWED_N_MODES)
def test_angular_momentum_closed_form(n_modes):
    """P-8: sum_i x_i x p_i = sum_p m_p [x_p x c_p0 + (dx/4) sum_b e_b x c_{., 1+b}]."""
    s, g = small_scene(1)
    M, Q = O.p2g(g, s.x, s.coeff, n_modes, s.mass)
    X = node_positions(g)
    L = np.array([(X[1] * Q[2] - X[2] * Q[1]).sum(), (X[2] * Q[0] - X[0] * Q[2]).sum(),
                  (X[0] * Q[1] - X[1] * Q[0]).sum()])
    m = s.mass.astype(np.float64)
    x = s.x.astype(np.float64)
    c = s.coeff.astype(np.float64)
    ref = np.zeros(3)
    ref += (m * np.cross(x.T, c[:, 0].T).T).sum(axis=1)
    if n_modes >= 4:
        for b in range(3):
            e = np.zeros((3, 1))
            e[b] = 1.0
            ref += g.dx / 4 * (m * np.cross(np.broadcast_to(e, c[:, 1 + b].shape).T,
                                            c[:, 1 + b].T).T).sum(axis=1)
    np.testing.assert_allclose(L, ref, rtol=1e-11, atol=1e-11)


def _field_values(kind, X, rng):
    """A polynomial velocity field of the given kind evaluated at node positions X."""
    if kind == "affine":
        A = rng.standard_normal((3, 4))
        return [A[a, 0] + A[a, 1] * X[0] + A[a, 2] * X[1] + A[a, 3] * X[2] for a in range(3)], A
    if kind == "trilinear":
        A = rng.standard_normal((3, 8))
        out = []
        for a in range(3):
            v = 0.0
            for i, (px, py, pz) in enumerate(itertools.product(range(2), repeat=3)):
                v = v + A[a, i] * X[0] ** px * X[1] ** py * X[2] ** pz
            out.append(v)
        return out, A
    A = rng.standard_normal((3, 27))
    out = []
    for a in range(3):
        v = 0.0
        for i, (px, py, pz) in enumerate(itertools.product(range(3), repeat=3)):
            v = v + A[a, i] * X[0] ** px * X[1] ** py * X[2] ** pz
        out.append(v)
    return out, A


@pytest.mark.parametrize("kind,min_modes", [("affine", 4), ("trilinear", 8), ("triquadratic", 27)])
def test_g2p_reproduces_polynomial_fields(kind, min_modes):
    """P-9: the fitted polynomial equals the grid field everywhere in the stencil box."""
    s, g = small_scene(2, P=300)
    X = node_positions(g)
    rng = np.random.default_rng(5)
    V, _ = _field_values(kind, X, rng)
    # shift/scale so the field is O(1) on this unit-ish box
    vel = np.stack(V)
    b, t = O.stencil_base(g, s.x)
    for n_modes in [m for m in O.ALLOWED_N_MODES if m >= min_modes]:
        c, _, _ = O.g2p(g, vel, s.x, n_modes)
        zh = rng.uniform(-1.6, 1.6, (3, s.P))   # probe points in units of dx around x_p
        xp = s.x.astype(np.float64)
        probe = [xp[a] + zh[a] * g.dx for a in range(3)]
        Vp, _ = _field_values(kind, probe, np.random.default_rng(5))
        fit = np.zeros((3, s.P))
        for r in range(n_modes):
            fit += c[:, r] * mode_eval(r, zh, t)
        np.testing.assert_allclose(fit, np.stack(Vp), rtol=0, atol=1e-9 * np.abs(vel).max())


def test_g2p_27_modes_is_interpolation():
    """P-5: 27-mode G2P equals numpy.linalg.solve of E c = v on the 27 stencil nodes."""
    s, g = small_scene(3, P=200)
    vel = np.random.default_rng(0).standard_normal((3, g.nz, g.ny, g.nx))
    c, _, _ = O.g2p(g, vel, s.x, 27)
    b, t = O.stencil_base(g, s.x)
    for p in range(0, s.P, 7):
        E = np.zeros((27, 27))
        rhs = np.zeros((27, 3))
        for i, (jx, jy, jz) in enumerate(O.STENCIL):
            zh = np.array([jx - 1 - t[0, p], jy - 1 - t[1, p], jz - 1 - t[2, p]])
            for r in range(27):
                E[i, r] = mode_eval(r, zh, t[:, p])
            rhs[i] = vel[:, b[2, p] + jz, b[1, p] + jy, b[0, p] + jx]
        sol = np.linalg.solve(E, rhs)
        np.testing.assert_allclose(c[:, :, p], sol.T, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("n_modes", [4, 8])
def test_g2p_is_weighted_least_squares(n_modes):
    """Section 3.3: c minimises sum_i W_i (v_i - sum_r c_r s_r)^2 -- normal equations."""
    s, g = small_scene(4, P=200)
    vel = np.random.default_rng(1).standard_normal((3, g.nz, g.ny, g.nx))
    c, _, _ = O.g2p(g, vel, s.x, n_modes)
    b, t = O.stencil_base(g, s.x)
    for p in range(0, s.P, 5):
        S = np.zeros((27, n_modes))
        Wt = np.zeros(27)
        rhs = np.zeros((27, 3))
        for i, (jx, jy, jz) in enumerate(O.STENCIL):
            zh = np.array([jx - 1 - t[0, p], jy - 1 - t[1, p], jz - 1 - t[2, p]])
            Wt[i] = np.prod([float(O.quadratic_bspline(zh[a])) for a in range(3)])
            for r in range(n_modes):
                S[i, r] = mode_eval(r, zh, t[:, p])
            rhs[i] = vel[:, b[2, p] + jz, b[1, p] + jy, b[0, p] + jx]
        A = S.T @ (Wt[:, None] * S)
        sol = np.linalg.solve(A, S.T @ (Wt[:, None] * rhs))
        np.testing.assert_allclose(c[:, :, p], sol.T, rtol=1e-9, atol=1e-9)


def test_g2p_degenerate_t_is_the_limit():
    """At t = -1/2 (a vanishing weight) the quadratic coefficient is the limit t -> -1/2+."""
    g = O.Grid(10, 10, 10, 1 / 4, 4.0)
    vel = np.random.default_rng(2).standard_normal((3, 10, 10, 10))
    x = np.array([[4.5 / 4], [4.25 / 4], [3.875 / 4]], np.float32)  # t_x = -1/2 exactly
    c, _, _ = O.g2p(g, vel, x, 27)
    b, t = O.stencil_base(g, x)
    assert t[0, 0] == -0.5
    # normal equations at t_x = -1/2 + eps on the same stencil, eps -> 0
    prev = None
    for eps in (1e-4, 1e-5, 1e-6):
        tt = np.array([-0.5 + eps, t[1, 0], t[2, 0]])
        S = np.zeros((27, 27))
        Wt = np.zeros(27)
        rhs = np.zeros((27, 3))
        for i, (jx, jy, jz) in enumerate(O.STENCIL):
            zh = np.array([jx - 1 - tt[0], jy - 1 - tt[1], jz - 1 - tt[2]])
            Wt[i] = np.prod([float(O.quadratic_bspline(zh[a])) for a in range(3)])
            for r in range(27):
                S[i, r] = mode_eval(r, zh, tt)
            rhs[i] = vel[:, b[2, 0] + jz, b[1, 0] + jy, b[0, 0] + jx]
        sol = np.linalg.solve(S, rhs).T
        err = np.abs(sol - c[:, :, 0]).max()
        if prev is not None:
            assert err < prev  # converges to the oracle's value
        prev = err
    assert prev < 1e-4


def test_g2p_apic_special_case():
    """P-6: N_r = 4 is textbook APIC: v_p = sum w v_i, C = B D^-1 with D computed numerically."""
    s, g = small_scene(5, P=150)
    vel = np.random.default_rng(3).standard_normal((3, g.nz, g.ny, g.nx))
    c, _, _ = O.g2p(g, vel, s.x, 4)
    b, t = O.stencil_base(g, s.x)
    xp = s.x.astype(np.float64)
    for p in range(s.P):
        vp = np.zeros(3)
        B = np.zeros((3, 3))
        D = np.zeros((3, 3))
        for jx, jy, jz in O.STENCIL:
            xi = np.array([(b[0, p] + jx) * g.dx, (b[1, p] + jy) * g.dx, (b[2, p] + jz) * g.dx])
            d = xi - xp[:, p]
            w = np.prod([float(O.quadratic_bspline(d[a] / g.dx)) for a in range(3)])
            vi = vel[:, b[2, p] + jz, b[1, p] + jy, b[0, p] + jx]
            vp += w * vi
            B += w * np.outer(vi, d)
            D += w * np.outer(d, d)
        C = B @ np.linalg.inv(D)
        np.testing.assert_allclose(c[:, 0, p], vp, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(c[:, 1:4, p] / g.dx, C, rtol=1e-10, atol=1e-10)


def test_p2g_apic_special_case():
    """P-6 (P2G side): (mv)_i = sum_p m_p w_ip (v_p + C_p (x_i - x_p)), Eq. 9, collocated."""
    s, g = small_scene(6, P=150)
    M, Q = O.p2g(g, s.x, s.coeff, 4, s.mass)
    b, t = O.stencil_base(g, s.x)
    xp = s.x.astype(np.float64)
    Qr = np.zeros_like(Q)
    for p in range(s.P):
        C = s.coeff[:, 1:4, p].astype(np.float64) / g.dx
        for jx, jy, jz in O.STENCIL:
            xi = np.array([(b[0, p] + jx) * g.dx, (b[1, p] + jy) * g.dx, (b[2, p] + jz) * g.dx])
            d = xi - xp[:, p]
            w = np.prod([float(O.quadratic_bspline(d[a] / g.dx)) for a in range(3)])
            Qr[:, b[2, p] + jz, b[1, p] + jy, b[0, p] + jx] += \
                float(s.mass[p]) * w * (s.coeff[:, 0, p] + C @ d)
    np.testing.assert_allclose(Q, Qr, rtol=1e-11, atol=1e-12)


def test_pic_special_case():
    """P-13: N_r = 1 is PIC -- Eq. 1-5 for P2G and Eq. 6-8 for G2P."""
    s, g = small_scene(7, P=200)
    M, Q = O.p2g(g, s.x, s.coeff, 1, s.mass)
    v = O.grid_update(g, M, Q, 0.0, (0, 0, 0), 0)
    c, _, _ = O.g2p(g, v, s.x, 1)
    b, t = O.stencil_base(g, s.x)
    Mr = np.zeros_like(M)
    Qr = np.zeros_like(Q)
    ws = []
    for p in range(s.P):
        row = []
        for jx, jy, jz in O.STENCIL:
            w = 1.0
            for a, j in enumerate((jx, jy, jz)):
                w *= float(O.quadratic_bspline(b[a, p] + j - (t[a, p] + b[a, p] + 1)))
            m_ip = float(s.mass[p]) * w                      # Eq. 1
            Mr[b[2, p] + jz, b[1, p] + jy, b[0, p] + jx] += m_ip                     # Eq. 4
            Qr[:, b[2, p] + jz, b[1, p] + jy, b[0, p] + jx] += m_ip * s.coeff[:, 0, p].astype(np.float64)  # Eq. 2-3
            row.append(m_ip)
        ws.append(row)
    np.testing.assert_allclose(M, Mr, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(Q, Qr, rtol=1e-12, atol=1e-13)
    for p in range(s.P):
        mv = np.zeros(3)
        for (jx, jy, jz), m_ip in zip(O.STENCIL, ws[p]):
            mv += m_ip * v[:, b[2, p] + jz, b[1, p] + jy, b[0, p] + jx]  # Eq. 6-7
        np.testing.assert_allclose(c[:, 0, p], mv / float(s.mass[p]), rtol=1e-12, atol=1e-12)


def test_roundtrip_lossless_and_dissipative():
    """P-10: grid -> G2P -> P2G -> grid is the identity on occupied nodes at N_r = 27
    (the lossless transfer of the abstract / section 5); for N_r < 27 grid KE never grows."""
    s = W.config0(0)
    g = O.grid_from_spec(s.grid)
    v = np.random.default_rng(1).standard_normal((3, g.nz, g.ny, g.nx))
    kes = {}
    for n_modes in O.ALLOWED_N_MODES:
        c, _, _ = O.g2p(g, v, s.x, n_modes)
        M, Q = O.p2g(g, s.x, c, n_modes)
        v2 = O.grid_update(g, M, Q, 0.0, (0, 0, 0), 0)
        occ = M > 0
        ke0 = 0.5 * (M[None] * v ** 2).sum()
        kes[n_modes] = 0.5 * (M[None] * v2 ** 2).sum()
        if n_modes == 27:
            assert np.abs(v2[:, occ] - v[:, occ]).max() < 1e-12
            assert abs(kes[27] - ke0) < 1e-10 * ke0
        else:
            assert kes[n_modes] < ke0
    assert kes[1] < kes[4] < kes[8] < kes[27]


def test_g2p_shared_modes_agree_across_truncations():
    """P-11: orthogonality makes the first modes independent of N_r."""
    s, g = small_scene(8, P=300)
    vel = np.random.default_rng(4).standard_normal((3, g.nz, g.ny, g.nx))
    c27, _, _ = O.g2p(g, vel, s.x, 27)
    for n_modes in (1, 4, 8):
        c, _, _ = O.g2p(g, vel, s.x, n_modes)
        np.testing.assert_allclose(c, c27[:, :n_modes], rtol=1e-12, atol=1e-12)


def test_p2g_continuous_across_cell_switch():
    """P-12: the base node switches at u = k + 1/2 but the grid transfer is continuous."""
    g = O.Grid(12, 12, 12, 1 / 8, 8.0)
    rng = np.random.default_rng(9)
    c = rng.standard_normal((3, 27, 2)).astype(np.float32)
    c[:, :, 1] = c[:, :, 0]
    xa = np.float32(5.5 / 8)
    xb = np.nextafter(xa, np.float32(0))
    x = np.array([[xa, xb], [5.2 / 8, 5.2 / 8], [4.9 / 8, 4.9 / 8]], np.float32)
    b, _ = O.stencil_base(g, x)
    assert b[0, 0] != b[0, 1]
    for n_modes in O.ALLOWED_N_MODES:
        Ma, Qa = O.p2g(g, x[:, :1], c[:, :, :1], n_modes)
        Mb, Qb = O.p2g(g, x[:, 1:], c[:, :, 1:], n_modes)
        assert np.abs(Ma - Mb).max() < 1e-6
        assert np.abs(Qa - Qb).max() < 1e-5


def test_gravity_only_step_closed_form():
    """P-14: c = 0 and no walls: one step gives c'_0 = dt g exactly and c'_{r>0} = 0."""
    s = W.config0(0)
    g = O.grid_from_spec(s.grid)
    c0 = np.zeros_like(s.coeff)
    out = O.step(g, s.x, c0, 27, 1e-4, (0.0, -9.8, 0.0), 0, sort=False)
    np.testing.assert_allclose(out["coeff"][:, 0], np.array([[0.0], [-9.8e-4], [0.0]])
                               * np.ones((1, s.P)), rtol=1e-12, atol=1e-15)
    assert np.abs(out["coeff"][:, 1:]).max() < 1e-13


def test_grid_update_walls_hand_example():
    """Eq. 5 plus separating slip walls on an 8^3 grid with bc_layers = 1."""
    g = O.Grid(8, 8, 8, 0.25, 4.0)
    M = np.zeros((8, 8, 8))
    Q = np.zeros((3, 8, 8, 8))
    # node (ix, iy, iz) = (2, 4, 4): low x wall layer; momentum -2 along x, +1 along y
    M[4, 4, 2] = 2.0
    Q[:, 4, 4, 2] = [-4.0, 2.0, 6.0]
    # node (6, 4, 4): high x wall layer (N - 1 - 1 = 6); moving +x
    M[4, 4, 6] = 1.0
    Q[:, 4, 4, 6] = [3.0, -1.0, 0.0]
    # interior node (4, 4, 4)
    M[4, 4, 4] = 4.0
    Q[:, 4, 4, 4] = [4.0, 4.0, -4.0]
    v = O.grid_update(g, M, Q, 0.01, (0.0, -10.0, 0.0), 1)
    np.testing.assert_allclose(v[:, 4, 4, 2], [0.0, 1.0 - 0.1, 3.0])
    np.testing.assert_allclose(v[:, 4, 4, 6], [0.0, -1.0 - 0.1, 0.0])
    np.testing.assert_allclose(v[:, 4, 4, 4], [1.0, 1.0 - 0.1, -1.0])
    assert np.count_nonzero(v[:, M == 0]) == 0
    # no walls
    v0 = O.grid_update(g, M, Q, 0.01, (0.0, -10.0, 0.0), 0)
    np.testing.assert_allclose(v0[:, 4, 4, 2], [-2.0, 0.9, 3.0])


def test_advection_and_clamp():
    """x' = fl32(x + dt c'_0), kept inside [o + 2 dx, o + (N - 2) dx)."""
    g = O.Grid(12, 12, 12, 1 / 8, 8.0)
    vel = np.zeros((3, 12, 12, 12))
    vel[0] = 1.0
    vel[1] = -1e4    # pushes through the low wall
    vel[2] = 1e4     # pushes through the high wall
    x = np.array([[0.5], [0.3], [1.2]], np.float32)
    c, xo, _ = O.g2p(g, vel, x, 4, dt=0.01)
    assert xo[0, 0] == np.float32(0.5 + 0.01)
    assert xo[1, 0] == np.float32(2 / 8)
    assert xo[2, 0] == np.nextafter(np.float32(10 / 8), np.float32(0))


def test_f_update_affine_field():
    """F' = (I + dt C) F where C is the velocity gradient of an affine grid field."""
    s, g = small_scene(10, P=100)
    X = node_positions(g)
    rng = np.random.default_rng(11)
    A = rng.standard_normal((3, 3))
    vel = np.stack([0.3 + A[a, 0] * X[0] + A[a, 1] * X[1] + A[a, 2] * X[2] for a in range(3)])
    F = (np.eye(3).reshape(9, 1) + 0.01 * rng.standard_normal((9, s.P))).astype(np.float32)
    dt = 1e-3
    _, _, Fo = O.g2p(g, vel, s.x, 4, dt=dt, F=F)
    for p in range(s.P):
        Fp = F[:, p].astype(np.float64).reshape(3, 3)
        np.testing.assert_allclose(Fo[:, p].reshape(3, 3), (np.eye(3) + dt * A) @ Fp,
                                   rtol=1e-10, atol=1e-10)


def _load_golden():
    with open(GOLDEN) as f:
        doc = json.load(f)
    fr = lambda s: Fr(s)  # noqa: E731
    return doc, fr


@pytest.mark.parametrize("case_idx", range(4))
def test_oracle_matches_exact_golden(case_idx):
    """P-4: the FP64 oracle equals the exact-rational brute force on hand-placed particles
    that include t = -1/2, t = 0 and t = 1/2 - 2^-20 (golden fixture)."""
    doc, fr = _load_golden()
    case = doc["cases"][case_idx]
    n_modes = case["n_modes"]
    nx, ny, nz = doc["nodes"]
    g = O.Grid(nx, ny, nz, float(fr(doc["dx"])), float(fr(doc["inv_dx"])))
    x = np.array([[float(fr(v)) for v in p] for p in doc["x"]], np.float32).T
    mass = np.array([float(fr(m)) for m in doc["mass"]], np.float32)
    cin = np.array([[[float(fr(v)) for v in ca] for ca in c] for c in doc["coeff_in"]])
    cin = np.transpose(cin, (1, 2, 0)).astype(np.float32)  # (3, 27, P)
    M, Q = O.p2g(g, x, cin, n_modes, mass)
    dt = float(fr(doc["dt"]))
    grav = [float(fr(v)) for v in doc["gravity"]]
    v = O.grid_update(g, M, Q, dt, grav, doc["bc_layers"])
    c, xo, _ = O.g2p(g, v, x, n_modes, dt)
    for nd, ms, ps, vs in zip(case["nodes"], case["grid_mass"], case["grid_mom"], case["grid_vel"]):
        ix, iy, iz = nd
        assert abs(M[iz, iy, ix] - float(fr(ms))) < 1e-14
        for a in range(3):
            assert abs(Q[a, iz, iy, ix] - float(fr(ps[a]))) < 1e-13
            assert abs(v[a, iz, iy, ix] - float(fr(vs[a]))) < 1e-11 * max(1.0, abs(float(fr(vs[a]))))
    ref = np.array([[[float(fr(v)) for v in ca] for ca in cp] for cp in case["coeff"]])  # P,3,r
    np.testing.assert_allclose(np.transpose(c, (2, 0, 1)), ref, rtol=1e-9, atol=1e-10)
    xref = np.array(case["x_out"], np.float32).T
    assert np.all(np.abs(xo.astype(np.float64) - xref) <= np.spacing(np.abs(xref)))
