"""Pins of the FP64 differentiable twin (oracle/adjoint.py).

* its forward step equals the numpy oracle's (P2G grid, grid velocity, G2P
  coefficients, advection);
* its autograd gradient of the velocity-matching loss equals central finite
  differences (float64, h = 1e-6 in cell units for positions, absolute for
  coefficients) along seeded random directions and single coordinates, away
  from the cell switches where the G2P coefficients jump (the quadratic-mode
  coefficient is discontinuous where the base node changes).  On the
  4,096-particle, 10-step case: directions with seeds 0-7 and 64 coordinates.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as A
from oracle import polypic_oracle as O


def small_case(seed=0, cells=16, block=4, lo=6):
    """Power-of-two grid: the float32 and float64 stencil formulas agree exactly."""
    rng = np.random.default_rng(seed)
    g = W.cubic_grid(cells)
    x = W.jittered_block(rng, g, (lo, lo, lo), (block,) * 3, (2, 2, 2))
    P = x.shape[1]
    c = np.zeros((3, 27, P))
    c[:, 0] = rng.standard_normal((3, P))
    c[:, 1:] = 0.1 * rng.standard_normal((3, 26, P))
    return g, O.grid_from_spec(g), x.astype(np.float64), c


def test_twin_forward_matches_oracle():
    gs, g, x, c = small_case(1)
    for n_modes in (1, 4, 8, 27):
        xo, co, grid = A.step(g, torch.from_numpy(x), torch.from_numpy(c[:, :n_modes]), n_modes,
                              1e-3, (0.0, -9.8, 0.0), 1)
        ref = O.step(g, x.astype(np.float32), c[:, :n_modes], n_modes, 1e-3, (0.0, -9.8, 0.0), 1,
                     sort=False)
        np.testing.assert_allclose(grid["grid_mass"].numpy(), ref["grid_mass"].ravel(), atol=1e-13)
        np.testing.assert_allclose(grid["grid_mom"].numpy(), ref["grid_mom"].reshape(3, -1),
                                   atol=1e-12)
        np.testing.assert_allclose(grid["grid_vel"].numpy(), ref["grid_vel"].reshape(3, -1),
                                   atol=1e-11)
        np.testing.assert_allclose(co.numpy(), ref["coeff"], rtol=1e-10, atol=1e-11)
        # the oracle rounds positions to float32; the twin keeps float64
        assert np.abs(xo.numpy() - ref["x"]).max() <= 2 * np.spacing(np.float32(1.0))


def safe_mask(g, x0, c0, n_modes, n_steps, dt, gravity, bc, margin=1e-3):
    """Particles whose every u stays more than `margin` cells away from k + 1/2."""
    safe = np.ones(x0.shape[1], bool)
    x, c = torch.from_numpy(x0), torch.from_numpy(c0)
    with torch.no_grad():
        for _ in range(n_steps + 1):
            u = x.numpy() * g.inv_dx - 0.5
            frac = u - np.floor(u)
            safe &= np.all((frac > margin) & (frac < 1 - margin), axis=0)
            x, c, _ = A.step(g, x, c, n_modes, dt, gravity, bc)
    return safe


def fd_check(g, x0, c0, n_modes, n_steps, dt, target, n_dirs, n_coords, seed0=0, rtol=1e-5):
    gravity, bc = (0.0, -9.8, 0.0), 1
    L, (gx, gc) = A.loss_and_grad(g, x0, c0, n_modes, n_steps, dt, gravity, bc, target)
    gx, gc = gx.numpy(), gc.numpy()
    safe = safe_mask(g, x0, c0, n_modes, n_steps, dt, gravity, bc)
    assert safe.mean() > 0.8

    def Lval(x, c):
        with torch.no_grad():
            xs, cs = A.rollout(g, torch.from_numpy(x), torch.from_numpy(c), n_modes, n_steps, dt,
                               gravity, bc)
            return float(A.loss(xs, cs, *target))

    hx = 1e-6 * g.dx
    hc = 1e-6
    for sd in range(seed0, seed0 + n_dirs):
        rng = np.random.default_rng(sd)
        dx = rng.standard_normal(x0.shape) * safe
        dc = rng.standard_normal(c0.shape) * safe
        fd = (Lval(x0 + hx * dx, c0 + hc * dc) - Lval(x0 - hx * dx, c0 - hc * dc)) / 2.0
        an = hx * float((gx * dx).sum()) + hc * float((gc * dc).sum())
        assert abs(fd - an) <= rtol * max(abs(an), 1e-6), (sd, fd, an)
    rng = np.random.default_rng(seed0 + 100)
    idx = np.flatnonzero(safe)
    for k in range(n_coords):
        p = int(rng.choice(idx))
        if k % 2 == 0:
            a = int(rng.integers(3))
            e = np.zeros_like(x0)
            e[a, p] = 1.0
            fd = (Lval(x0 + hx * e, c0) - Lval(x0 - hx * e, c0)) / (2 * hx)
            an = gx[a, p]
        else:
            a, r = int(rng.integers(3)), int(rng.integers(n_modes))
            e = np.zeros_like(c0)
            e[a, r, p] = 1.0
            fd = (Lval(x0, c0 + hc * e) - Lval(x0, c0 - hc * e)) / (2 * hc)
            an = gc[a, r, p]
        assert abs(fd - an) <= 1e-4 * max(abs(an), 1.0), (k, p, fd, an)


@pytest.mark.parametrize("n_modes", [4, 27])
def test_twin_gradient_matches_finite_differences_small(n_modes):
    gs, g, x, c = small_case(2)
    target = W.target_field_params(1)
    fd_check(g, x, c[:, :n_modes].copy(), n_modes, 3, 1e-3, target, n_dirs=4, n_coords=12)


def test_twin_gradient_matches_finite_differences_adjoint_case():
    """The 16^3-grid, 4,096-particle differentiable case over 10 steps of dt = 1e-4:
    central differences along random directions with seeds 0-7 and at 64 single
    coordinates (half positions, half coefficients)."""
    s = W.config3_fd(0)
    g = O.grid_from_spec(s.grid)
    target = W.target_field_params(0)
    fd_check(g, s.x.astype(np.float64), s.coeff.astype(np.float64), 27, s.n_steps, s.dt, target,
             n_dirs=8, n_coords=64)
