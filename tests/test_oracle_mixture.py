"""Pins of the oracle's shared-grid liquid-fabric transfers (section 3.4, Eq. 15-20):
fluid particles scatter their fluid mass m_f into the fluid channels, solid particles
their mixture mass m_s + m_f into the solid channels, and each particle is fitted back
from its own phase's velocity.  Pinned by an exact-rational fixture built from the
independent brute force, by conservation per phase, and by the single-phase cases."""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import polypic_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact_mixture.json")


def _scene(seed, n=16, P=400):
    rng = np.random.default_rng(seed)
    g = O.Grid(n + 4, n + 4, n + 4, 1.0 / n, float(n))
    x = ((3.0 + rng.random((3, P)) * (n - 2.0)) / n).astype(np.float32)
    c = np.zeros((3, 27, P), np.float32)
    c[:, 0] = rng.standard_normal((3, P))
    c[:, 1:] = 0.1 * rng.standard_normal((3, 26, P))
    phase = (rng.random(P) < 0.4).astype(np.int32)
    m_s = (1.0 + rng.random(P)).astype(np.float32)
    m_f = (0.5 * rng.random(P)).astype(np.float32)
    return g, x, c, phase, m_s, m_f


@pytest.mark.parametrize("case_idx", range(4))
def test_mixture_oracle_matches_exact_golden(case_idx):
    with open(GOLDEN) as f:
        doc = json.load(f)
    case = doc["cases"][case_idx]
    nm = case["n_modes"]
    nx, ny, nz = doc["nodes"]
    g = O.Grid(nx, ny, nz, float(Fr(doc["dx"])), float(Fr(doc["inv_dx"])))
    x = np.array([[float(Fr(v)) for v in p] for p in doc["x"]], np.float32).T
    ms = np.array([float(Fr(v)) for v in doc["mass_s"]], np.float32)
    mf = np.array([float(Fr(v)) for v in doc["mass_f"]], np.float32)
    phase = np.array(doc["phase"], np.int32)
    cin = np.array([[[float(Fr(v)) for v in ca] for ca in c] for c in doc["coeff_in"]])
    cin = np.transpose(cin, (1, 2, 0)).astype(np.float32)
    M, Q = O.mixture_p2g(g, x, cin, nm, phase, mf, ms)
    dt = float(Fr(doc["dt"]))
    grav = [float(Fr(v)) for v in doc["gravity"]]
    V = O.mixture_grid_update(g, M, Q, dt, grav, doc["bc_layers"])
    c, _, _ = O.mixture_g2p(g, V, x, phase, nm, dt)
    for k, ph in enumerate(case["phases"]):
        for nd, ms_, ps_, vs_ in zip(ph["nodes"], ph["grid_mass"], ph["grid_mom"],
                                     ph["grid_vel"]):
            ix, iy, iz = nd
            assert abs(M[k, iz, iy, ix] - float(Fr(ms_))) < 1e-14
            for a in range(3):
                assert abs(Q[k, a, iz, iy, ix] - float(Fr(ps_[a]))) < 1e-13
                vv = float(Fr(vs_[a]))
                assert abs(V[k, a, iz, iy, ix] - vv) < 1e-11 * max(1.0, abs(vv))
        assert abs(M[k].sum() - sum(float(Fr(v)) for v in ph["grid_mass"])) < 1e-13
    ref = np.array([[[float(Fr(v)) for v in ca] for ca in cp] for cp in case["coeff"]])
    np.testing.assert_allclose(np.transpose(c, (2, 0, 1)), ref, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("n_modes", [4, 27])
def test_mixture_conserves_each_phase(n_modes):
    """Fluid channels: mass sum_fluid m_f and momentum sum_fluid m_f c_0 (Eq. 15-16);
    solid channels: sum_solid (m_s + m_f) and sum_solid (m_s + m_f) c_0 (Eq. 18-19)."""
    g, x, c, phase, ms, mf = _scene(1)
    M, Q = O.mixture_p2g(g, x, c, n_modes, phase, mf, ms)
    fl, so = phase == 0, phase == 1
    mass = [mf[fl].astype(np.float64), (ms[so].astype(np.float64) + mf[so])]
    vel = [c[:, 0, fl].astype(np.float64), c[:, 0, so].astype(np.float64)]
    for k in range(2):
        assert abs(M[k].sum() - mass[k].sum()) < 1e-12 * mass[k].sum()
        ref = (vel[k] * mass[k]).sum(axis=1)
        np.testing.assert_allclose(Q[k].reshape(3, -1).sum(axis=1), ref, rtol=1e-11,
                                   atol=1e-11)


def test_mixture_single_phase_cases():
    """All fluid: the fluid channels are the plain P2G at m_f and the solid ones empty.
    All solid without solid mass (m_s = 0): the solid channels carry exactly what the
    fluid ones carried, and each particle's fit comes from the field of its phase."""
    g, x, c, _, ms, mf = _scene(2)
    P = x.shape[1]
    zeros = np.zeros(P, np.int32)
    ones = np.ones(P, np.int32)
    M0, Q0 = O.mixture_p2g(g, x, c, 27, zeros, mf, ms)
    Mp, Qp = O.p2g(g, x, c, 27, mf)
    np.testing.assert_allclose(M0[0], Mp, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Q0[0], Qp, rtol=0, atol=1e-14)
    assert not M0[1].any() and not Q0[1].any()
    M1, Q1 = O.mixture_p2g(g, x, c, 27, ones, mf, np.zeros(P, np.float32))
    np.testing.assert_allclose(M1[1], M0[0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(Q1[1], Q0[0], rtol=0, atol=1e-14)
    rng = np.random.default_rng(3)
    V = rng.standard_normal((2, 3, g.nz, g.ny, g.nx))
    c0, _, _ = O.mixture_g2p(g, V, x, zeros, 8)
    c1, _, _ = O.mixture_g2p(g, V, x, ones, 8)
    np.testing.assert_allclose(c0, O.g2p(g, V[0], x, 8)[0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(c1, O.g2p(g, V[1], x, 8)[0], rtol=0, atol=1e-14)


def test_mixture_rejects_unknown_phase():
    g, x, c, phase, ms, mf = _scene(4, P=10)
    phase[3] = 2
    with pytest.raises(ValueError):
        O.mixture_p2g(g, x, c, 4, phase, mf, ms)
