"""Pins of the oracle's P2G with the affine back-map of Eq. 12 (``p2g_affine``).

The modes of a particle are evaluated at z'_i = (I + dt C)^-1 (x_i - x_p) / dx with the
quadratic factor of the position x_fit where its coefficients were fitted.  Pinned by
the exact-rational brute force (golden fixture, inverse by Gauss-Jordan), by reduction
to the plain P2G (itself pinned) at dt = 0, by the closed form of the 4-mode case
(a linear change of the linear coefficients), and by the closed-form total momentum of
the 8-mode case from the moments of the B-spline weights.
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import polypic_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact_affine.json")


def _scene(seed, n=16, P=200):
    rng = np.random.default_rng(seed)
    g = O.Grid(n + 4, n + 4, n + 4, 1.0 / n, float(n))
    u = 3.0 + rng.random((3, P)) * (n - 2.0)
    x = (u / n).astype(np.float32)
    x_fit = (x - (0.3 * rng.standard_normal((3, P))) / n).astype(np.float32)
    c = np.zeros((3, 27, P), np.float32)
    c[:, 0] = rng.standard_normal((3, P))
    c[:, 1:] = 0.3 * rng.standard_normal((3, 26, P))
    m = (0.5 + rng.random(P)).astype(np.float32)
    return g, x, x_fit, c, m


@pytest.mark.parametrize("case_idx", range(4))
def test_affine_p2g_matches_exact_golden(case_idx):
    with open(GOLDEN) as f:
        doc = json.load(f)
    case = doc["cases"][case_idx]
    nm = case["n_modes"]
    nx, ny, nz = doc["nodes"]
    g = O.Grid(nx, ny, nz, float(Fr(doc["dx"])), float(Fr(doc["inv_dx"])))
    x = np.array([[float(Fr(v)) for v in p] for p in doc["x"]], np.float32).T
    xf = np.array([[float(Fr(v)) for v in p] for p in doc["x_fit"]], np.float32).T
    mass = np.array([float(Fr(m)) for m in doc["mass"]], np.float32)
    cin = np.array([[[float(Fr(v)) for v in ca] for ca in c] for c in doc["coeff_in"]])
    cin = np.transpose(cin, (1, 2, 0)).astype(np.float32)
    M, Q = O.p2g_affine(g, x, cin, nm, float(Fr(doc["dt"])), x_fit=xf, mass=mass)
    for nd, ms, ps in zip(case["nodes"], case["grid_mass"], case["grid_mom"]):
        ix, iy, iz = nd
        assert abs(M[iz, iy, ix] - float(Fr(ms))) < 1e-14
        for a in range(3):
            assert abs(Q[a, iz, iy, ix] - float(Fr(ps[a]))) < 1e-12
    assert abs(M.sum() - sum(float(Fr(v)) for v in case["grid_mass"])) < 1e-13


@pytest.mark.parametrize("n_modes", [1, 4, 8, 27])
def test_affine_p2g_at_zero_dt_is_the_plain_p2g(n_modes):
    """dt = 0 (identity map) and the fit at the present position: exactly Eq. 13 as
    ``p2g`` evaluates it; the mass channel never depends on the map."""
    g, x, x_fit, c, m = _scene(1)
    M0, Q0 = O.p2g(g, x, c, n_modes, m)
    M1, Q1 = O.p2g_affine(g, x, c, n_modes, 0.0, mass=m)
    np.testing.assert_allclose(M1, M0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Q1, Q0, rtol=0, atol=1e-14)
    M2, _ = O.p2g_affine(g, x, c, n_modes, 2e-2, x_fit=x_fit, mass=m)
    np.testing.assert_allclose(M2, M0, rtol=0, atol=1e-15)


def test_affine_p2g_four_modes_is_a_linear_change_of_coefficients():
    """With 4 modes s_r(z') = (1, z') and z' = B zhat, B = (I + dt C)^-1, so the expansion
    is c_0 + (c_lin^T B) zhat: the plain P2G of the coefficients (c_0, B^T c_lin)."""
    g, x, x_fit, c, m = _scene(2)
    dt = 3e-2
    c4 = c[:, :4].astype(np.float64)
    P = x.shape[1]
    ct = c4.copy()
    for p in range(P):
        C = c4[:, 1:4, p] / g.dx               # C_ab = c_{a,1+b} / dx
        B = np.linalg.inv(np.eye(3) + dt * C)
        ct[:, 1:4, p] = c4[:, 1:4, p] @ B      # row a: sum_g c_{a,1+g} B_{g b}
    M0, Q0 = O.p2g(g, x, ct, 4, m)
    M1, Q1 = O.p2g_affine(g, x, c4, 4, dt, x_fit=x_fit, mass=m)
    np.testing.assert_allclose(M1, M0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Q1, Q0, rtol=1e-12, atol=1e-12)


def test_affine_p2g_eight_modes_total_momentum_closed_form():
    """Total momentum at 8 modes from the weight moments: with z' = B zhat and the product
    weight W, sum W z'_a z'_b = (B D B^T)_ab with D = diag(1/4), and
    sum W z'_x z'_y z'_z = sum_k B_xk B_yk B_zk mu3_k, mu3_k = t_k (1 - 4 t_k^2) / 4
    (the third moment of the 1-D weights), all other products vanishing."""
    g, x, x_fit, c, m = _scene(3)
    dt = 3e-2
    _, Q = O.p2g_affine(g, x, c, 8, dt, x_fit=x_fit, mass=m)
    _, t = O.stencil_base(g, x)
    c8 = c[:, :8].astype(np.float64)
    tot = np.zeros(3)
    pairs = {4: (0, 1), 5: (0, 2), 6: (1, 2)}       # modes 110, 101, 011
    for p in range(x.shape[1]):
        C = c8[:, 1:4, p] / g.dx
        B = np.linalg.inv(np.eye(3) + dt * C)
        S2 = 0.25 * B @ B.T
        mu3 = t[:, p] * (1.0 - 4.0 * t[:, p] ** 2) / 4.0
        S3 = sum(B[0, k] * B[1, k] * B[2, k] * mu3[k] for k in range(3))
        for a in range(3):
            v = c8[a, 0, p]
            for r, (i, j) in pairs.items():
                v += c8[a, r, p] * S2[i, j]
            v += c8[a, 7, p] * S3
            tot[a] += float(m[p]) * v
    np.testing.assert_allclose(Q.reshape(3, -1).sum(axis=1), tot, rtol=1e-11, atol=1e-11)
