"""GPU adjoint against the FP64 autograd twin of the step (oracle/adjoint.py).

Bar: gradients within 1e-4 normwise relative error (FP32 device vs FP64 twin),
for one teacher-forced step with random upstream gradients and for the
10-step, 4,096-particle differentiable case through the autograd.Function.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as A
from oracle import polypic_oracle as O
from tests.gpu_util import dev, host, note, oracle_grid, rel, require_gpu

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-4


def scene(seed, P_block=6, cells=16, mass_random=False):
    rng = np.random.default_rng(seed)
    g = W.cubic_grid(cells)
    lo = (cells - P_block) // 2
    x = W.jittered_block(rng, g, (lo, lo, lo), (P_block,) * 3, (2, 2, 2))
    P = x.shape[1]
    c = np.zeros((3, 27, P), np.float32)
    c[:, 0] = rng.standard_normal((3, P))
    c[:, 1:] = 0.1 * rng.standard_normal((3, 26, P))
    m = (0.5 + rng.random(P)).astype(np.float32) if mass_random else None
    return g, x, c, m


@pytest.mark.parametrize("n_modes", [1, 4, 8, 27])
def test_single_step_adjoint_matches_twin(n_modes):
    pp = require_gpu()
    gs, x, c, m = scene(3, mass_random=True)
    P = x.shape[1]
    dt, grav, bc = 2e-3, (0.0, -9.8, 0.0), 1
    c = c[:, :n_modes].copy()
    rng = np.random.default_rng(7)
    gc_in = rng.standard_normal((3, n_modes, P))   # dL/dc' in input order
    gx_in = rng.standard_normal((3, P))            # dL/dx' in input order
    note(f"adjoint single step: P={P} n_modes={n_modes}")

    # FP64 twin: L = <gc, c'> + <gx, x'>
    og = O.grid_from_spec(gs)
    xt = torch.from_numpy(x.astype(np.float64)).requires_grad_(True)
    ct = torch.from_numpy(c.astype(np.float64)).requires_grad_(True)
    mt = torch.from_numpy(m.astype(np.float64)).requires_grad_(True)
    xo, co, grid = A.step(og, xt, ct, n_modes, dt, grav, bc, mass=mt)
    grid["grid_vel"].retain_grad()
    L = (torch.from_numpy(gc_in) * co).sum() + (torch.from_numpy(gx_in) * xo).sum()
    L.backward()

    # device: forward grid, then the three backward calls
    g = pp.grid_from_spec(gs)
    ps = pp.ParticleSet(g, n_modes, dev(x), dev(c), mass=dev(m), dt=dt, gravity=grav,
                        bc_layers=bc)
    ps.sort()
    ps.p2g()
    ps.grid_update()
    perm = ps.perm.long()
    gc_slot = dev(gc_in)[:, :, perm].contiguous()
    gx_slot = dev(gx_in)[:, perm].contiguous()
    N = 3 * (gs.nodes[0] * gs.nodes[1] * gs.nodes[2])
    gvb = torch.empty(N, device="cuda")
    gmb = torch.empty(N // 3, device="cuda")
    gpb = torch.empty(N, device="cuda")
    x_grad = torch.zeros(3, P, device="cuda")
    c_grad = torch.empty(3, n_modes, P, device="cuda")
    m_grad = torch.empty(P, device="cuda")
    pp.ops.polypic_g2p_backward(g, n_modes, dt, ps.grid_vel, ps.x, gc_slot, gvb, x_grad,
                                perm=ps.perm, x_out_grad=gx_slot, status_dev=ps.status)
    pp.ops.polypic_grid_update_backward(g, dt, grav, bc, ps.grid_mass, ps.grid_mom, gvb, gmb, gpb)
    pp.ops.polypic_p2g_backward(g, n_modes, ps.x, ps.coeff, gmb, gpb, c_grad, x_grad,
                                mass=ps.mass, perm=ps.perm, mass_grad=m_grad,
                                status_dev=ps.status)
    torch.cuda.synchronize()
    assert ps.status_flags() == 0
    e_v = rel(host(gvb), grid["grid_vel"].grad.numpy())
    e_x = rel(host(x_grad), xt.grad.numpy())
    e_c = rel(host(c_grad), ct.grad.numpy())
    e_m = rel(host(m_grad), mt.grad.numpy())
    note(f"  dL/dv {e_v:.2e}  dL/dx {e_x:.2e}  dL/dc {e_c:.2e}  dL/dm {e_m:.2e}")
    assert max(e_v, e_x, e_c, e_m) <= TOL_GRAD


def test_multistep_gradient_matches_twin():
    """Loss 1/2 sum |c_p0 - v*(x_p)|^2 after 10 steps on the 4,096-particle case."""
    pp = require_gpu()
    s = W.config3_fd(0)
    target = W.target_field_params(0)
    og = O.grid_from_spec(s.grid)
    note(f"adjoint 10 steps: P={s.P}")
    _, (gx_ref, gc_ref) = A.loss_and_grad(og, s.x.astype(np.float64), s.coeff.astype(np.float64),
                                          27, s.n_steps, s.dt, s.gravity, s.bc_layers, target)
    g = pp.grid_from_spec(s.grid)
    x0 = dev(s.x).requires_grad_(True)
    c0 = dev(s.coeff).requires_grad_(True)
    xS, cS = pp.polypic_steps(x0, c0, g, 27, s.n_steps, s.dt, s.gravity, s.bc_layers)
    Am, kap, ph = (torch.tensor(v, dtype=torch.float32, device="cuda") for v in target)
    vstar = Am.T @ torch.sin(2 * np.pi * (kap @ xS) + ph.reshape(-1, 1))
    L = 0.5 * ((cS[:, 0] - vstar) ** 2).sum()
    L.backward()
    e_x = rel(host(x0.grad), gx_ref.numpy())
    e_c = rel(host(c0.grad), gc_ref.numpy())
    note(f"  dL/dx0 {e_x:.2e}  dL/dc0 {e_c:.2e}")
    assert e_x <= TOL_GRAD and e_c <= TOL_GRAD


def test_autograd_outputs_match_forward_steps():
    """The autograd forward returns the state of stepping a ParticleSet.

    P2G accumulates with atomics, so the summation order (and the last bits)
    may differ between two runs: compared at the forward parity bar."""
    pp = require_gpu()
    gs, x, c, _ = scene(5)
    g = pp.grid_from_spec(gs)
    xS, cS = pp.polypic_steps(dev(x), dev(c), g, 27, 3, 1e-3)
    ps = pp.ParticleSet(g, 27, dev(x), dev(c), dt=1e-3)
    for _ in range(3):
        ps.step()
    order = ps.order
    assert rel(host(xS[:, order]), host(ps.x)) <= 1e-6
    assert rel(host(cS[:, :, order]), host(ps.coeff)) <= 1e-5


def test_autograd_raises_on_out_of_range_particle():
    """A particle whose stencil leaves the grid is skipped by every kernel and flagged in
    the device status word; the autograd forward reads the word and raises instead of
    returning outputs (and later zero gradients) silently.  With the check switched off
    the same call returns, and the in-range particles are stepped."""
    pp = require_gpu()
    gs, x, c, _ = scene(6)
    x = x.copy()
    x[0, 0] = np.float32(0.01)          # b_x = -1 on a 1/16 grid: out of range
    g = pp.grid_from_spec(gs)
    note("autograd out-of-range particle")
    x0 = dev(x).requires_grad_(True)
    c0 = dev(c).requires_grad_(True)
    with pytest.raises(pp.PolyPICError, match="left the grid"):
        pp.polypic_steps(x0, c0, g, 27, 2, 1e-3)
    xS, cS = pp.polypic_steps(x0, c0, g, 27, 2, 1e-3, check_status=False)
    torch.cuda.synchronize()
    assert torch.isfinite(cS).all()
