"""Pins of the staggered-grid (MAC) oracle (oracle/mac.py) against things fixed independently
of it: the exact-rational brute force on hand-placed particles (golden fixture), textbook
APIC written face by face (Eq. 9-10 with D computed from the face positions), the
collocated oracle on a lattice shifted by half a spacing, conservation per component,
reproduction of polynomial face fields, and the range of the face stencils.

Faces of component alpha sit at origin + (i + (1 - e_alpha)/2) dx (section 3, Table 1).
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import mac as MAC
from oracle import polypic_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact_mac.json")


def _scene(seed, n=16, P=300, dyadic_bits=None):
    rng = np.random.default_rng(seed)
    g = O.Grid(n + 4, n + 4, n + 4, 1.0 / n, float(n))
    u = 3.0 + rng.random((3, P)) * (n - 2.0)          # grid units, inside the domain
    if dyadic_bits:
        u = np.round(u * 2 ** dyadic_bits) / 2 ** dyadic_bits
    x = (u / n).astype(np.float32)
    c = np.zeros((3, 27, P), np.float32)
    c[:, 0] = rng.standard_normal((3, P))
    c[:, 1:] = 0.1 * rng.standard_normal((3, 26, P))
    m = (0.5 + rng.random(P)).astype(np.float32)
    return g, x, c, m


@pytest.mark.parametrize("case_idx", range(4))
def test_mac_oracle_matches_exact_golden(case_idx):
    """The FP64 MAC oracle equals the exact-rational brute force (normal equations, no
    orthogonality assumed) on six hand-placed particles, incl. staggered t = -1/2."""
    with open(GOLDEN) as f:
        doc = json.load(f)
    case = doc["cases"][case_idx]
    nm = case["n_modes"]
    nx, ny, nz = doc["nodes"]
    g = O.Grid(nx, ny, nz, float(Fr(doc["dx"])), float(Fr(doc["inv_dx"])))
    x = np.array([[float(Fr(v)) for v in p] for p in doc["x"]], np.float32).T
    mass = np.array([float(Fr(m)) for m in doc["mass"]], np.float32)
    cin = np.array([[[float(Fr(v)) for v in ca] for ca in c] for c in doc["coeff_in"]])
    cin = np.transpose(cin, (1, 2, 0)).astype(np.float32)
    M, Q = MAC.p2g(g, x, cin, nm, mass)
    dt = float(Fr(doc["dt"]))
    grav = [float(Fr(v)) for v in doc["gravity"]]
    v = MAC.grid_update(g, M, Q, dt, grav, doc["bc_layers"])
    c, xo, _ = MAC.g2p(g, v, x, nm, dt)
    total = 0
    for alpha, comp in enumerate(case["components"]):
        for fc, ms, ps, vs in zip(comp["faces"], comp["face_mass"], comp["face_mom"],
                                  comp["face_vel"]):
            ix, iy, iz = fc
            assert abs(M[alpha, iz, iy, ix] - float(Fr(ms))) < 1e-14
            assert abs(Q[alpha, iz, iy, ix] - float(Fr(ps))) < 1e-13
            vv = float(Fr(vs))
            assert abs(v[alpha, iz, iy, ix] - vv) < 1e-11 * max(1.0, abs(vv))
        total += len(comp["faces"])
        # no mass outside the brute force's faces
        assert abs(M[alpha].sum() - sum(float(Fr(m)) for m in comp["face_mass"])) < 1e-13
    assert total > 0
    ref = np.array([[[float(Fr(vv)) for vv in ca] for ca in cp] for cp in case["coeff"]])
    np.testing.assert_allclose(np.transpose(c, (2, 0, 1)), ref, rtol=1e-9, atol=1e-10)
    xref = np.array(case["x_out"], np.float32).T
    assert np.all(np.abs(xo.astype(np.float64) - xref) <= np.spacing(np.abs(xref)))


@pytest.mark.parametrize("n_modes", [1, 4, 8, 27])
def test_mac_mass_and_momentum_conserved_per_component(n_modes):
    """Partition of unity on every face lattice: sum_i m_{i alpha} = sum_p m_p and
    sum_i (mv)_{i alpha} = sum_p m_p c_{p 0 alpha} for each component (Eq. 1, 3, 4, 13)."""
    g, x, c, m = _scene(1)
    M, Q = MAC.p2g(g, x, c, n_modes, m)
    for a in range(3):
        assert abs(M[a].sum() - m.astype(np.float64).sum()) < 1e-12 * m.sum()
        ref = (m.astype(np.float64) * c[a, 0]).sum()
        assert abs(Q[a].sum() - ref) < 1e-11 * np.abs(m * c[a, 0]).sum()


@pytest.mark.parametrize("n_modes", [4, 27])
def test_mac_component_is_collocated_transfer_on_shifted_lattice(n_modes):
    """Component alpha of the MAC transfer is the collocated transfer (itself pinned) on
    a grid whose origin moves by dx/2 along the other two axes; positions are dyadic so
    that both float32 stencil formulas are exact."""
    g, x, c, m = _scene(2, dyadic_bits=12)
    M, Q = MAC.p2g(g, x, c, n_modes, m)
    rng = np.random.default_rng(5)
    vel = rng.standard_normal((3, g.nz, g.ny, g.nx))
    cm, _, _ = MAC.g2p(g, vel, x, n_modes)
    for alpha in range(3):
        org = tuple(0.5 * g.dx if a != alpha else 0.0 for a in range(3))
        gs = O.Grid(g.nx, g.ny, g.nz, g.dx, g.inv_dx, org)
        Mc, Qc = O.p2g(gs, x, c, n_modes, m)
        np.testing.assert_allclose(M[alpha], Mc, rtol=0, atol=1e-14)
        np.testing.assert_allclose(Q[alpha], Qc[alpha], rtol=0, atol=1e-13)
        cc, _, _ = O.g2p(gs, np.broadcast_to(vel[alpha], (3,) + vel.shape[1:]), x, n_modes)
        np.testing.assert_allclose(cm[alpha], cc[alpha], rtol=1e-12, atol=1e-12)


def _faces_near(g, xp, alpha):
    """Brute force: every face of component alpha with a nonzero B-spline weight for a
    particle at xp, with its world position and weight."""
    off = MAC.face_offset(alpha)
    out = []
    lo = [int(np.floor(xp[a] / g.dx - off[a])) - 2 for a in range(3)]
    for iz in range(lo[2], lo[2] + 5):
        for iy in range(lo[1], lo[1] + 5):
            for ix in range(lo[0], lo[0] + 5):
                pos = np.array([(i + off[a]) * g.dx for a, i in enumerate((ix, iy, iz))])
                w = float(np.prod([O.quadratic_bspline((xp[a] - pos[a]) / g.dx)
                                   for a in range(3)]))
                if w > 0.0:
                    out.append(((ix, iy, iz), pos, w))
    return out


def test_mac_apic_is_textbook_apic_per_face():
    """4 modes = APIC on faces (section 3.2, Eq. 9-10 with Table 1's c_{p alpha}).
    G2P: v_{p alpha} = sum_i w v_{i alpha}; c_{p alpha} = D^-1 sum_i w v_{i alpha} (x_{i alpha} - x_p)
    with D = sum_i w (x_{i alpha} - x_p)(x_{i alpha} - x_p)^T formed from the face positions.
    P2G: (mv)_{i alpha} = sum_p m_p w (v_{p alpha} + c_{p alpha} . (x_{i alpha} - x_p))."""
    g, x, c, m = _scene(3, P=40)
    rng = np.random.default_rng(6)
    vel = rng.standard_normal((3, g.nz, g.ny, g.nx))
    cm, _, _ = MAC.g2p(g, vel, x, 4)
    M, Q = MAC.p2g(g, x, c, 4, m)
    Mref = np.zeros_like(M)
    Qref = np.zeros_like(Q)
    for p in range(x.shape[1]):
        xp = x[:, p].astype(np.float64)
        for alpha in range(3):
            faces = _faces_near(g, xp, alpha)
            assert 8 <= len(faces) <= 27
            vp = sum(w * vel[alpha, i[2], i[1], i[0]] for i, _, w in faces)
            B = sum(w * vel[alpha, i[2], i[1], i[0]] * (pos - xp) for i, pos, w in faces)
            D = sum(w * np.outer(pos - xp, pos - xp) for _, pos, w in faces)
            cp = np.linalg.solve(D, B)
            assert abs(cm[alpha, 0, p] - vp) < 1e-12
            np.testing.assert_allclose(cm[alpha, 1:4, p] / g.dx, cp, rtol=1e-10, atol=1e-10)
            c_lin = c[alpha, 1:4, p].astype(np.float64) / g.dx
            mp, c0 = float(m[p]), float(c[alpha, 0, p])
            for i, pos, w in faces:
                Mref[alpha, i[2], i[1], i[0]] += mp * w
                Qref[alpha, i[2], i[1], i[0]] += mp * w * (c0 + c_lin @ (pos - xp))
    np.testing.assert_allclose(M, Mref, rtol=0, atol=1e-13)
    np.testing.assert_allclose(Q, Qref, rtol=0, atol=1e-12)


def test_mac_g2p_reproduces_polynomial_face_fields():
    """A triquadratic face field (a different one per component) is represented exactly at
    27 modes: the fitted expansion re-evaluated at the 27 faces of the stencil returns the
    field there; an affine field gives its value and gradient at 4 modes."""
    g, x, _, _ = _scene(4, P=50)
    rng = np.random.default_rng(8)
    coef = rng.standard_normal((3, 3, 3, 3))   # [alpha][px][py][pz] exponents 0..2
    nz, ny, nx = g.nz, g.ny, g.nx
    vel = np.zeros((3, nz, ny, nx))
    for alpha in range(3):
        off = MAC.face_offset(alpha)
        X = (np.arange(nx) + off[0]) * g.dx
        Y = (np.arange(ny) + off[1]) * g.dx
        Z = (np.arange(nz) + off[2]) * g.dx
        ZZ, YY, XX = np.meshgrid(Z, Y, X, indexing="ij")
        for i in range(3):
            for j in range(3):
                for k in range(3):
                    vel[alpha] += coef[alpha, i, j, k] * XX ** i * YY ** j * ZZ ** k
    cm, _, _ = MAC.g2p(g, vel, x, 27)
    for alpha in range(3):
        b, t = MAC.face_stencil(g, x, alpha)
        ph = [O.phi_1d(t[a]) for a in range(3)]
        for jx, jy, jz in O.STENCIL:
            val = np.zeros(x.shape[1])
            for r in range(27):
                kx, ky, kz = O.MODES[r]
                val += cm[alpha, r] * ph[0][kx][jx] * ph[1][ky][jy] * ph[2][kz][jz]
            ref = vel[alpha][b[2] + jz, b[1] + jy, b[0] + jx]
            np.testing.assert_allclose(val, ref, rtol=1e-10, atol=1e-10)
    # affine: value and gradient
    A = rng.standard_normal((3, 3))
    v0 = rng.standard_normal(3)
    for alpha in range(3):
        off = MAC.face_offset(alpha)
        X = (np.arange(nx) + off[0]) * g.dx
        Y = (np.arange(ny) + off[1]) * g.dx
        Z = (np.arange(nz) + off[2]) * g.dx
        ZZ, YY, XX = np.meshgrid(Z, Y, X, indexing="ij")
        vel[alpha] = v0[alpha] + A[alpha, 0] * XX + A[alpha, 1] * YY + A[alpha, 2] * ZZ
    c4, _, _ = MAC.g2p(g, vel, x, 4)
    xd = x.astype(np.float64)
    for alpha in range(3):
        np.testing.assert_allclose(c4[alpha, 0], v0[alpha] + A[alpha] @ xd, rtol=1e-11,
                                   atol=1e-11)
        for beta in range(3):
            np.testing.assert_allclose(c4[alpha, 1 + beta] / g.dx, A[alpha, beta], rtol=1e-9)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mac_face_stencils_range_at_the_switches(axis):
    """On a staggered axis the base face is floor(u) - 1, so the face stencils fit iff
    1 <= u on the low side; on the face-normal axis the collocated bound u < N - 1.5
    is the tighter one on the high side.  Positions exactly at u = 1 and N - 1.5 and one
    float32 below them: the oracle accepts exactly 1 <= u < N - 1.5."""
    n = 12
    g = O.Grid(n, n, n, 1 / 8, 8.0)
    below = lambda v: np.nextafter(np.float32(v), np.float32(-np.inf))
    cases = [(np.float32(1.0), True), (below(1.0), False),
             (np.float32(n - 1.5), False), (below(n - 1.5), True), (np.float32(5.0), True)]
    x = np.full((3, len(cases)), np.float32(5.0 / 8), np.float32)
    for i, (u, _) in enumerate(cases):
        x[axis, i] = np.float32(u) / np.float32(8.0)
    expect = np.array([ok for _, ok in cases])
    np.testing.assert_array_equal(MAC.faces_in_range(g, x), expect)
    # independent statement: all three face stencils {b..b+2} inside [0, N-1], with the
    # base face found from the exact face positions (nearest face c, ties up; b = c - 1)
    for i, (u, ok) in enumerate(cases):
        fits = True
        for alpha in range(3):
            shift = Fr(0) if axis == alpha else Fr(1, 2)
            uu = Fr(float(u)) - shift
            cface = (uu + Fr(1, 2)).__floor__()
            fits &= 1 <= cface <= n - 2
        assert fits == ok
    coeff = np.zeros((3, 1, 1), np.float32)
    vel = np.zeros((3, n, n, n))
    for i, (_, ok) in enumerate(cases):
        xi = x[:, i:i + 1]
        for call in (lambda: MAC.p2g(g, xi, coeff, 1), lambda: MAC.g2p(g, vel, xi, 1)):
            if ok:
                call()
            else:
                with pytest.raises(O.OracleRangeError):
                    call()
