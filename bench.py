#!/usr/bin/env python3
"""Benchmark of the PolyPIC transfer step on one MI355X.

Workload: the dam-break case -- a 128^3-cell grid (132^3 nodes, dx = 1/128) with a
64 x 128 x 64-cell block of fluid at 8 particles per cell (4,194,304 particles,
jittered, at rest), 27 polynomial modes, dt = 1e-4, gravity -9.8, slip walls.
Synthetic seeded inputs (workloads.config1); no dataset is involved.

A step is one pass of the whole transfer path on device-resident data:
    cell-key radix sort -> P2G (27 modes) -> grid update -> G2P + advection
run as sort -> grid update -> G2P2G: the G2P of a step and the P2G of the next
are one kernel (polypic_g2p2g), which scatters the new state into the grid while
its coefficients are in registers (they are still written, not read back).  A
run with separate P2G and G2P calls is reported beside it ("unfused").  From the
second step on, the sort is the exact re-sort from the previous step's keys
(polypic_sort_update, bit-identical to a full sort); the full sort's time on the
same state is reported beside it.
The timed region is K consecutive steps between two device synchronisations;
per-phase times come from HIP events recorded, on the stream the kernels run on,
at the phase boundaries of every fifth of those steps (an event between two
kernels idles the queue for a few microseconds, so the other steps record none).

Prints one JSON line.  `value` = particles x steps / wall time of the timed
region (whole-step throughput); the P2G + G2P-only rate, per-phase times, the
4-mode (APIC) comparison, the roofline of the dominant kernel and the oracle's
CPU rate on a bounded sample are reported beside it.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --calib-copy      # plain device copy, for rocprofv3 byte calibration
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle transfers/sec (P2G+G2P, 27 modes, FP32) + bwd/fwd time ratio"
UNIT = "particle-transfers/s"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak (AMD published figure)
PROFILES = os.path.join(ROOT, "profiles")

# Algorithmic bytes per particle (float32, one pass over each stream):
#   P2G reads x (12 B), mass or the sort permutation (4 B) and 3 * n_modes coefficients;
#   G2P reads x (12 B), writes 3 * n_modes coefficients and x (12 B).
def p2g_bytes_per_particle(n_modes: int) -> int:
    return 12 + 4 + 12 * n_modes


def g2p_bytes_per_particle(n_modes: int) -> int:
    return 12 + 12 * n_modes + 12


#   G2P fused with the next P2G reads x (12 B) and the permutation (4 B), writes x (12 B)
#   and 3 * n_modes coefficients; the coefficients are not read back.
def g2p2g_bytes_per_particle(n_modes: int) -> int:
    return 12 + 4 + 12 + 12 * n_modes


#   a material-point set also reads and writes its deformation gradient (2 x 36 B) and its
#   mass (2 x 4 B; in place of the 4 B of the permutation it still reads)
def g2p2g_bytes_per_point_with_f(n_modes: int) -> int:
    return g2p2g_bytes_per_particle(n_modes) + 2 * 36 + 2 * 4


KERNEL_SOURCES = {
    "p2g": "paper_2308_01060_amd/csrc/polypic_p2g.hip",
    "g2p": "paper_2308_01060_amd/csrc/polypic_g2p.hip",
    "g2p2g": "paper_2308_01060_amd/csrc/polypic_g2p2g.hip",
}


# headers every kernel source includes: a change there changes the kernels too
KERNEL_HEADERS = (
    "paper_2308_01060_amd/csrc/polypic_device.hpp",
    "paper_2308_01060_amd/csrc/polypic_scene.hpp",
    "paper_2308_01060_amd/csrc/polypic_internal.hpp",
)


def source_digest(kernel: str) -> str:
    """Digest of the kernel's source file and the device headers it includes."""
    h = hashlib.sha256()
    for rel in (KERNEL_SOURCES[kernel],) + KERNEL_HEADERS:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None.

    profiles/traffic_<kernel>_<workload>.txt holds key = value lines, among them
    source_sha (digest of the kernel source when the counters were taken) and
    bytes_per_launch.  A changed source makes the figure stale: None.
    """
    path = os.path.join(PROFILES, f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha") != source_digest(kernel):
        return None
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-modes", type=int, default=27)
    ap.add_argument("--cells", type=int, default=128, help="grid cells per axis (dam break)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1048576,
                    help="particles in the oracle's timed sample")
    ap.add_argument("--no-apic", action="store_true", help="skip the 4-mode comparison run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the bwd/fwd timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-scenes timing")
    ap.add_argument("--no-unfused", action="store_true",
                    help="skip the reference run with separate P2G and G2P calls")
    ap.add_argument("--unfused-steps", type=int, default=30,
                    help="timed steps of the unfused reference run")
    ap.add_argument("--batch-steps", type=int, default=10, help="steps in the batched timing")
    ap.add_argument("--adjoint-steps", type=int, default=10,
                    help="differentiable steps in the bwd/fwd timing")
    ap.add_argument("--no-moving", action="store_true",
                    help="skip the dam break with moving state")
    ap.add_argument("--no-liquid-fabric", action="store_true",
                    help="skip the 256^3 liquid + fabric workload")
    ap.add_argument("--no-mac", action="store_true", help="skip the staggered-grid timing")
    ap.add_argument("--no-shared-grid", action="store_true",
                    help="skip the liquid + fabric timing on one shared grid")
    ap.add_argument("--no-affine", action="store_true",
                    help="skip the affine back-map timing")
    ap.add_argument("--no-paper-scale", action="store_true",
                    help="skip the paper-size dam break at 8 modes")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a plain device copy of known size (counter calibration)")
    return ap.parse_args()


def calib_copy():
    import torch

    n = 256 * 1024 * 1024  # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_read_per_launch": 4 * n,
                      "calib_copy_bytes_written_per_launch": 4 * n, "launches": 5}))


PHASE_EVERY = 5  # steps between two steps timed phase by phase


def time_steps(ps, steps: int, torch):
    """Run `steps` full steps; returns (wall_s, per-phase mean ms dict).

    Fused sets (the default) step as sort -> grid update (of the active regions) ->
    G2P2G, the P2G of each step having been done by the G2P2G of the step before;
    unfused sets as
    sort -> P2G -> grid update -> G2P.  Every PHASE_EVERY-th step records a timing
    event at each phase boundary, and the phase means come from those steps.  The
    others record none: on this stack each timing event recorded between two
    kernels leaves the queue idle for 5-13 us (kernel trace), about 30 us per
    step.  The instrumented steps stay inside the timed region, so they slow the
    whole-step figure slightly and never speed it up."""
    if ps.fused:
        if not ps.grid_current:
            raise RuntimeError("a fused set needs its grid current before the timed steps")
        if not ps.regions_valid:
            ps.step()  # (untimed) a step whose G2P2G flags the regions it scatters into
        names = ("sort", "grid_update", "g2p2g")
        # the grid update visits the flagged regions only and zeroes the sums it read; the
        # fused call adds into them and flags where it lands
        calls = (ps.sort, ps.grid_update_active, lambda: ps.g2p2g(accumulate=True))
    else:
        names = ("sort", "p2g", "grid_update", "g2p")
        calls = (ps.sort, ps.p2g, ps.grid_update, ps.g2p)
    timed = [k for k in range(steps) if k % PHASE_EVERY == PHASE_EVERY // 2] or [0]
    ev = {k: [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
          for k in timed}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        e = ev.get(k)
        if e is None:
            for call in calls:
                call()
        else:
            e[0].record()
            for j, call in enumerate(calls):
                call()
                e[j + 1].record()
        ps.swap()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phase = {n: 0.0 for n in names}
    for e in ev.values():
        for j, n in enumerate(names):
            phase[n] += e[j].elapsed_time(e[j + 1])
    return wall, {n: v / len(ev) for n, v in phase.items()}


def transfer_ms(phase) -> float:
    """Time of the two transfers of a step: P2G + G2P, or the fused G2P2G."""
    return phase["g2p2g"] if "g2p2g" in phase else phase["p2g"] + phase["g2p"]


def adjoint_timing(pp, torch, W, cells: int, n_modes: int, n_steps: int, reps: int = 3):
    """Forward and backward time of `n_steps` differentiable steps (polypic_steps).

    Scene: the dam-break geometry with moving state (c0 ~ N(0,1), higher modes
    ~ N(0,0.1)).  The upstream gradients are those of the velocity-matching loss
    1/2 sum_p |c_p0 - v*(x_p)|^2 on the final state, taken once outside the timed
    region; the timed backward is the library's reverse pass alone (per step: the G2P,
    grid-update and P2G adjoints from the checkpointed state and grid fields).
    Returns the median over `reps` repetitions, plus event times of the three
    adjoint calls of one step.
    """
    import numpy as np

    s = W.config1_moving(0, n=cells)
    g = pp.grid_from_spec(s.grid)
    x0 = torch.from_numpy(s.x).cuda().requires_grad_(True)
    c0 = torch.from_numpy(np.ascontiguousarray(s.coeff[:, :n_modes])).cuda().requires_grad_(True)
    A, kap, ph = (torch.tensor(v, dtype=torch.float32, device="cuda")
                  for v in W.target_field_params(0))

    def upstream(xS, cS):
        xd = xS.detach().requires_grad_(True)
        cd = cS.detach().requires_grad_(True)
        vstar = A.T @ torch.sin(2 * np.pi * (kap @ xd) + ph.reshape(-1, 1))
        L = 0.5 * ((cd[:, 0] - vstar) ** 2).sum()
        return torch.autograd.grad(L, (xd, cd))

    fwd, bwd = [], []
    for rep in range(reps + 1):          # the first repetition warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xS, cS = pp.polypic_steps(x0, c0, g, n_modes, n_steps, s.dt, s.gravity, s.bc_layers)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gx, gc = upstream(xS, cS)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        torch.autograd.backward((xS, cS), (gx, gc))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if rep > 0:
            fwd.append(t1 - t0)
            bwd.append(t3 - t2)
        x0.grad = None
        c0.grad = None
        del xS, cS, gx, gc

    # per-call event times of one step's adjoint
    ps = pp.ParticleSet(g, n_modes, x0.detach(), c0.detach(), dt=s.dt, gravity=s.gravity,
                        bc_layers=s.bc_layers, track_order=False)
    N = pp.ops.n_nodes(g)
    gvb = torch.empty(3 * N, device="cuda")
    gmb = torch.empty(N, device="cuda")
    gpb = torch.empty(3 * N, device="cuda")
    gxo = torch.randn(3, s.P, device="cuda")
    gco = torch.randn(3, n_modes, s.P, device="cuda")
    gxi = torch.zeros(3, s.P, device="cuda")
    gci = torch.empty(3, n_modes, s.P, device="cuda")
    for _ in range(2):  # as in the timed backward: particle arrays in a step's sort order
        ps.step()
    ps.sort()
    ps.p2g()
    ps.grid_update()
    names = ("g2p_backward", "grid_update_backward", "p2g_backward")
    acc = {n: [] for n in names}
    for rep in range(6):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        pp.ops.polypic_g2p_backward(g, n_modes, s.dt, ps.grid_vel, ps.x, gco, gvb, gxi,
                                    perm=ps.perm, x_out_grad=gxo, status_dev=ps.status)
        ev[1].record()
        pp.ops.polypic_grid_update_backward(g, s.dt, s.gravity, s.bc_layers, ps.grid_mass,
                                            ps.grid_mom, gvb, gmb, gpb)
        ev[2].record()
        pp.ops.polypic_p2g_backward(g, n_modes, ps.x, ps.coeff, gmb, gpb, gci, gxi,
                                    status_dev=ps.status)
        ev[3].record()
        torch.cuda.synchronize()
        if rep > 0:
            for j, n in enumerate(names):
                acc[n].append(ev[j].elapsed_time(ev[j + 1]))
    if ps.status_flags() != 0:
        raise RuntimeError(f"device status flags {ps.status_flags()} in the adjoint timing")
    f = float(np.median(fwd))
    b = float(np.median(bwd))
    return {
        "bwd_fwd_ratio": b / f,
        "fwd_ms": f * 1e3,
        "bwd_ms": b * 1e3,
        "n_steps": n_steps,
        "particles": s.P,
        "n_modes": n_modes,
        "workload": s.name,
        "bwd_step_phase_ms": {n: round(float(np.median(v)), 4) for n, v in acc.items()},
        "note": "forward steps as ParticleSet does (re-sort, grid update, fused G2P2G) and "
                "keeps per step (x, c), the permutation and the grid fields; backward runs "
                "the three adjoint calls per step, which recompute the stencil weights; "
                "bwd_step_phase_ms: one step's adjoint calls on a sorted state",
    }


def batch_timing(pp, torch, W, n_modes: int, steps: int, warmup: int):
    """64 independent scenes (grids of 64^3, 96^3 or 128^3 cells, log-uniform particle
    counts in [1e4, 2e6] at 8 per cell): one graph-captured batched step versus one
    ParticleSet step per scene.

    Positions come from workloads.batched_scenes(0); the coefficients (mode 0 ~ N(0,1),
    higher modes ~ N(0,0.1)) are drawn on the device from a seeded torch generator.
    """
    import numpy as np

    scenes = W.batched_scenes(0, coefficients=False)
    grids = [pp.grid_from_spec(s.grid) for s in scenes]
    counts = [s.P for s in scenes]
    P = int(sum(counts))
    x = torch.from_numpy(np.ascontiguousarray(np.concatenate([s.x for s in scenes], axis=1)))
    x = x.cuda()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(20_000)
    c = torch.randn(3, n_modes, P, generator=gen, device="cuda")
    c[:, 1:] *= 0.1
    s0 = scenes[0]
    bs = pp.BatchedParticleSet(grids, counts, n_modes, x, c, dt=s0.dt, gravity=s0.gravity,
                               bc_layers=s0.bc_layers)
    for _ in range(warmup):
        bs.step()
    choice = bs.autotune()

    def timed(fn, k):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k, e0.elapsed_time(e1) / k

    eager_wall, eager_ev = timed(bs.step, steps)
    bs.capture()
    bs.replay()
    graph_wall, graph_ev = timed(bs.replay, steps)
    if bs.status_flags() != 0:
        raise RuntimeError(f"device status flags {bs.status_flags()} in the batched timing")

    # the plain form: one ParticleSet per scene, stepped one after the other
    sets = []
    for k, sc in enumerate(scenes):
        sl = bs.scene_slice(k)
        sets.append(pp.ParticleSet(grids[k], n_modes, bs.x[:, sl].contiguous(),
                                   bs.coeff[:, :, sl].contiguous(), dt=sc.dt,
                                   gravity=sc.gravity, bc_layers=sc.bc_layers,
                                   track_order=False))  # fused, as the batched set
    del bs

    def per_scene_step():
        for ps in sets:
            ps.step()

    for _ in range(warmup):
        per_scene_step()
    single_wall, single_ev = timed(per_scene_step, steps)
    for ps in sets:
        if ps.status_flags() != 0:
            raise RuntimeError("device status flags in the per-scene timing")
    return {
        "workload": f"batch_64scenes_{P}",
        "scenes": len(scenes),
        "particles": P,
        "n_modes": n_modes,
        "steps": steps,
        "graph_ms_per_step": graph_wall * 1e3,
        "graph_transfers_per_s": P / graph_wall,
        "eager_batched_ms_per_step": eager_wall * 1e3,
        "per_scene_ms_per_step": single_wall * 1e3,
        "per_scene_transfers_per_s": P / single_wall,
        "speedup_vs_per_scene": single_wall / graph_wall,
        "event_ms_per_step": {"graph": round(graph_ev, 4), "eager_batched": round(eager_ev, 4),
                              "per_scene": round(single_ev, 4)},
        "p2g_config": {"block": choice.block, "schedule": choice.schedule, "brick": choice.brick,
                       "per_cu": choice.per_cu, "chosen_by": "polypic_batch_autotune"},
        "note": "whole fused steps (sort, grid update, G2P2G: G2P + advection + the next "
                "P2G) of every scene; per-scene form = one ParticleSet.step per scene, "
                "launched in turn",
    }


def _set_timing(pp, torch, ps, steps: int, warmup: int, bpp: int, workload: str):
    """Warm up, autotune and time one fused ParticleSet; rate, phases and the roofline of its
    G2P2G call (bpp algorithmic bytes per particle over the call's mean event time)."""
    for _ in range(warmup):
        ps.step()
    choice = ps.autotune()
    fused_choice = ps.autotune_fused()
    torch.cuda.synchronize()
    wall, phase = time_steps(ps, steps, torch)
    if ps.status_flags() != 0:
        raise RuntimeError(f"device status flags {ps.status_flags()} in {workload}")
    achieved = bpp * ps.P / (phase["g2p2g"] * 1e-3) / 1e9
    return {
        "workload": workload,
        "particles": ps.P,
        "n_modes": ps.n_modes,
        "steps": steps,
        "ms_per_step": wall * 1e3 / steps,
        "transfers_per_s": ps.P * steps / wall,
        "p2g_g2p_transfers_per_s": ps.P / (transfer_ms(phase) * 1e-3),
        "phase_ms": {k: round(v, 4) for k, v in phase.items()},
        "p2g_config": {"path": "cells" if choice.path == 1 else "bricks",
                       "block": choice.block, "schedule": choice.schedule,
                       "brick": choice.brick},
        "g2p2g_config": {"lane_group": fused_choice.lane_group,
                         "schedule": "xcd" if fused_choice.schedule == 1 else "linear"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("g2p2g", workload), "kernel": "g2p2g",
                     "bytes_per_particle": bpp},
    }


def moving_timing(pp, torch, W, cells: int, n_modes: int, steps: int, warmup: int):
    """The dam-break geometry with moving state (c0 ~ N(0,1), higher modes ~ N(0,0.1)):
    thousands of particles change cell per step, against tens at rest, and every momentum
    channel is non-zero."""
    import numpy as np

    s = W.config1_moving(0, n=cells)
    g = pp.grid_from_spec(s.grid)
    ps = pp.ParticleSet(g, n_modes, torch.from_numpy(s.x).cuda(),
                        torch.from_numpy(np.ascontiguousarray(s.coeff[:, :n_modes])).cuda(),
                        dt=s.dt, gravity=s.gravity, bc_layers=s.bc_layers, track_order=False)
    del s
    out = _set_timing(pp, torch, ps, steps, warmup, g2p2g_bytes_per_particle(n_modes),
                      f"dambreak_moving_{cells}cube_{ps.P}")
    out["data"] = "synthetic (seeded jittered dam-break block, workloads.config1_moving)"
    return out


def mac_timing(pp, torch, W, cells: int, n_modes: int, steps: int, warmup: int):
    """The moving dam break on a staggered (MAC) grid: every velocity component on its own
    faces with its own face mass.  A step is sort (re-sort) -> MAC P2G -> MAC grid update ->
    MAC G2P + advection, as separate calls.  Rooflines: P2G reads x, the permutation and
    the coefficients (12 + 4 + 12 n_modes B per particle); G2P reads x and the permutation
    and writes the coefficients and x (12 + 4 + 12 n_modes + 12 B)."""
    import numpy as np

    s = W.config1_moving(0, n=cells)
    g = pp.grid_from_spec(s.grid)
    ps = pp.MacParticleSet(g, n_modes, torch.from_numpy(s.x).cuda(),
                           torch.from_numpy(np.ascontiguousarray(s.coeff[:, :n_modes])).cuda(),
                           dt=s.dt, gravity=s.gravity, bc_layers=s.bc_layers, track_order=False)
    del s
    for _ in range(warmup):
        ps.step()
    torch.cuda.synchronize()
    wall, phase = time_steps(ps, steps, torch)
    if ps.status_flags() != 0:
        raise RuntimeError(f"device status flags {ps.status_flags()} in the MAC timing")
    P = ps.P
    roof = {}
    for k, bpp in (("p2g", p2g_bytes_per_particle(n_modes)),
                   ("g2p", g2p_bytes_per_particle(n_modes) + 4)):
        achieved = bpp * P / (phase[k] * 1e-3) / 1e9
        roof[k] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                   "bytes_per_particle": bpp}
    return {
        "workload": f"dambreak_moving_mac_{cells}cube_{P}",
        "particles": P,
        "n_modes": n_modes,
        "steps": steps,
        "ms_per_step": wall * 1e3 / steps,
        "transfers_per_s": P * steps / wall,
        "p2g_g2p_transfers_per_s": P / (transfer_ms(phase) * 1e-3),
        "phase_ms": {k: round(v, 4) for k, v in phase.items()},
        "roofline": roof,
        "note": "staggered grid: 3 face-mass and 3 face-momentum arrays; separate calls",
    }


def affine_timing(pp, torch, W, cells: int, n_modes: int, steps: int, warmup: int):
    """The moving dam break stepped with the affine back-map of Eq. 12 in P2G
    (AffineParticleSet: sort -> affine P2G -> grid update -> G2P, plus the gather of the
    fitting positions).  The affine P2G evaluates every mode at every node (no separable
    contraction), so its roofline is taken against the vector ALU as well: per particle
    27 nodes x 3 components x (27 + 9 + 3) multiply-adds on the mode factors, plus the
    mapped offsets and quadratic factors (27 x 3 x 15), at 2 flop each."""
    import numpy as np

    s = W.config1_moving(0, n=cells)
    g = pp.grid_from_spec(s.grid)
    ps = pp.AffineParticleSet(g, n_modes, torch.from_numpy(s.x).cuda(),
                              torch.from_numpy(np.ascontiguousarray(s.coeff[:, :n_modes])).cuda(),
                              dt=s.dt, gravity=s.gravity, bc_layers=s.bc_layers,
                              track_order=False)
    del s
    for _ in range(warmup):
        ps.step()
    torch.cuda.synchronize()
    wall, phase = time_steps(ps, steps, torch)
    if ps.status_flags() != 0:
        raise RuntimeError(f"device status flags {ps.status_flags()} in the affine timing")
    P = ps.P
    t = phase["p2g"] * 1e-3
    bpp = p2g_bytes_per_particle(n_modes) + 12      # + the fitting positions
    flops = 2 * 27 * 3 * (27 + 9 + 3 + 15) if n_modes == 27 else None
    out = {
        "workload": f"dambreak_moving_affine_{cells}cube_{P}",
        "particles": P,
        "n_modes": n_modes,
        "steps": steps,
        "ms_per_step": wall * 1e3 / steps,
        "transfers_per_s": P * steps / wall,
        "phase_ms": {k: round(v, 4) for k, v in phase.items()},
        "p2g_roofline_hbm": {"achieved": round(bpp * P / t / 1e9, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(bpp * P / t / 1e9 / HBM_PEAK_GBS, 4),
                             "bytes_per_particle": bpp},
    }
    if flops:
        out["p2g_roofline_alu"] = {"achieved": round(flops * P / t / 1e12, 2),
                                   "peak": 157.3, "unit": "TFLOP/s",
                                   "frac": round(flops * P / t / 1e12 / 157.3, 4),
                                   "flops_per_particle": flops}
    return out


def shared_grid_timing(pp, torch, W, n_modes: int, steps: int, warmup: int):
    """The liquid + fabric workload with both sets on ONE 260^3-node grid (section 3.4):
    16,777,216 fluid particles and 1,000,000 fabric points in one array, tagged by phase;
    fluid and solid channel sets per node.  A step is sort -> mixture P2G -> mixture grid
    update -> mixture G2P, separate calls.  Positions, masses and F from
    workloads.liquid_fabric_shared(0) without its coefficients, which are drawn on the
    device from a seeded torch generator."""
    import numpy as np

    s = W.liquid_fabric_shared(0)
    g = pp.grid_from_spec(s.grid)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(40_000)
    c = torch.randn(3, n_modes, s.P, generator=gen, device="cuda")
    c[:, 1:] *= 0.1
    ps = pp.MixtureParticleSet(g, n_modes, torch.from_numpy(s.x).cuda(), c,
                               torch.from_numpy(s.phase).cuda(), torch.from_numpy(s.mass_f).cuda(),
                               mass_s=torch.from_numpy(s.mass_s).cuda(),
                               F=torch.from_numpy(s.F).cuda(), dt=s.dt, gravity=s.gravity,
                               bc_layers=s.bc_layers, track_order=False)
    name = s.name
    del s, c
    for _ in range(warmup):
        ps.step()
    torch.cuda.synchronize()
    wall, phase = time_steps(ps, steps, torch)
    if ps.status_flags() != 0:
        raise RuntimeError(f"device status flags {ps.status_flags()} in the shared-grid timing")
    P = ps.P
    return {
        "workload": name,
        "particles": P,
        "n_modes": n_modes,
        "steps": steps,
        "ms_per_step": wall * 1e3 / steps,
        "transfers_per_s": P * steps / wall,
        "p2g_g2p_transfers_per_s": P / (transfer_ms(phase) * 1e-3),
        "phase_ms": {k: round(v, 4) for k, v in phase.items()},
        "note": "one particle array (phase, m_f, m_s, F per particle) and one grid with a "
                "fluid and a solid channel set; separate P2G and G2P calls",
    }


def liquid_fabric_timing(pp, torch, W, n_modes: int, steps: int, warmup: int):
    """The liquid + fabric workload: a falling block of 16,777,216 fluid particles (128 x 64
    x 128 cells at 16 per cell) and a 1000 x 1000 fabric sheet of 1,000,000 material
    points (per-point mass, deformation gradient F), each set on its own 256^3-cell grid
    (260^3 nodes), both at n_modes and stepped fused.  A step is one step of each set.

    Fluid positions come from workloads.config2_fluid(0); its coefficients (mode 0 ~ N(0,1),
    higher modes ~ N(0,0.1)) are drawn on the device from a seeded torch generator.  The
    fabric set is workloads.config2_fabric(0)."""
    import numpy as np

    sf = W.config2_fluid(0, coefficients=False)
    gf = pp.grid_from_spec(sf.grid)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(30_000)
    cf = torch.randn(3, n_modes, sf.P, generator=gen, device="cuda")
    cf[:, 1:] *= 0.1
    fluid = pp.ParticleSet(gf, n_modes, torch.from_numpy(sf.x).cuda(), cf, dt=sf.dt,
                           gravity=sf.gravity, bc_layers=sf.bc_layers, track_order=False)
    del cf
    fl = _set_timing(pp, torch, fluid, steps, warmup, g2p2g_bytes_per_particle(n_modes),
                     f"fluid_256cube_{sf.P}")
    del fluid
    sb = W.config2_fabric(0)
    gb = pp.grid_from_spec(sb.grid)
    fabric = pp.ParticleSet(gb, n_modes, torch.from_numpy(sb.x).cuda(),
                            torch.from_numpy(np.ascontiguousarray(sb.coeff[:, :n_modes])).cuda(),
                            mass=torch.from_numpy(sb.mass).cuda(), F=torch.from_numpy(sb.F).cuda(),
                            dt=sb.dt, gravity=sb.gravity, bc_layers=sb.bc_layers,
                            track_order=False)
    fb = _set_timing(pp, torch, fabric, steps, warmup, g2p2g_bytes_per_point_with_f(n_modes),
                     f"fabric_256cube_{sb.P}")
    del fabric
    P = sf.P + sb.P
    ms = fl["ms_per_step"] + fb["ms_per_step"]
    return {
        "workload": f"liquid_fabric_256cube_{sf.P}_{sb.P}",
        "particles": P,
        "n_modes": n_modes,
        "ms_per_step": ms,
        "transfers_per_s": P / (ms * 1e-3),
        "fluid": fl,
        "fabric": fb,
        "note": "one fused step of each set on its own 260^3-node grid (sort, grid update, "
                "G2P2G); fabric bytes add F read and written (72 B) and the mass read and "
                "written (8 B) per point",
    }


def paper_scale_timing(pp, torch, W, steps: int, warmup: int):
    """The paper's smallest fluid-only scene at its own size, mode count and time step
    (section 4, Table 2: about 311 thousand particles, 8 modes, dt = 2e-4): a
    36 x 36 x 30-cell block at 8 per cell (311,040 particles) on a 64^3-cell grid, at rest,
    at 8 modes (PolyPIC) and at 4 (APIC).  The paper's figures are whole steps of its
    liquid solver on one CPU; they are quoted beside the GPU transfer times as context."""
    import numpy as np

    s = W.paper_dambreak_small(0)
    g = pp.grid_from_spec(s.grid)
    out = {"workload": s.name, "particles": s.P, "dt": s.dt}
    for nm in (8, 4):
        ps = pp.ParticleSet(g, nm, torch.from_numpy(s.x).cuda(),
                            torch.from_numpy(np.ascontiguousarray(s.coeff[:, :nm])).cuda(),
                            dt=s.dt, gravity=s.gravity, bc_layers=s.bc_layers,
                            track_order=False)
        r = _set_timing(pp, torch, ps, steps, warmup, g2p2g_bytes_per_particle(nm), s.name)
        del ps
        out[f"modes_{nm}"] = {k: r[k] for k in ("ms_per_step", "transfers_per_s",
                                                "p2g_g2p_transfers_per_s", "phase_ms")}
    out["paper_table2_context"] = {
        "hardware": "Intel i9-12900K CPU (the paper's runs)",
        "what": "seconds per whole simulation step of the paper's liquid solver, transfers "
                "and everything else; not a transfer-only figure",
        "polypic_8_modes_s_per_step": 1.172, "apic_s_per_step": 0.510,
        "particles": {"polypic": 310839, "apic": 310929},
    }
    return out


# Workers of the all-cores oracle run: the state they need is set before the pool
# forks, so nothing large is pickled on the way in.
_ORACLE = {}


def _oracle_p2g_part(k):
    from oracle import polypic_oracle as O
    st = _ORACLE
    lo, hi = st["bounds"][k], st["bounds"][k + 1]
    return O.p2g(st["og"], st["x"][:, lo:hi], st["c"][:, :, lo:hi], st["n_modes"])


def _oracle_g2p_part(k):
    from oracle import polypic_oracle as O
    st = _ORACLE
    lo, hi = st["bounds"][k], st["bounds"][k + 1]
    O.g2p(st["og"], st["v"], st["x"][:, lo:hi], st["n_modes"], st["dt"])
    return hi - lo


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _config0_scene():
    import workloads as W
    return W.config0(0)


def _one_thread():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def cpu_baseline(scene, n_modes: int, sample: int):
    """The FP64 oracle, as it is, timed on host cores over a bounded sample.

    One core (BLAS pinned to one thread), then all cores: the same calls over
    particle chunks in a pool of forked workers (one thread each), the chunks'
    grids summed between P2G and the grid update.  Run before anything touches
    the GPU, so that the pool can fork."""
    import multiprocessing

    from threadpoolctl import threadpool_limits

    from oracle import polypic_oracle as O

    og = O.grid_from_spec(scene.grid)
    S = min(sample, scene.P)
    xs = scene.x[:, :S]
    cs = scene.coeff[:, :n_modes, :S]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        M, Q = O.p2g(og, xs, cs, n_modes)
        v = O.grid_update(og, M, Q, scene.dt, scene.gravity, scene.bc_layers)
        O.g2p(og, v, xs, n_modes, scene.dt)
        t1 = time.perf_counter() - t0

    n = max(1, min(16, os.cpu_count() or 1))  # the machine's CPU share for one GPU is 16
    bounds = [S * k // n for k in range(n + 1)]
    ctx = multiprocessing.get_context("fork")
    _ORACLE.update(og=og, x=xs, c=cs, n_modes=n_modes, dt=scene.dt, bounds=bounds)
    t0 = time.perf_counter()
    with ctx.Pool(n, initializer=_one_thread) as pool:
        parts = pool.map(_oracle_p2g_part, range(n))
    M = sum(p[0] for p in parts)
    Q = sum(p[1] for p in parts)
    _ORACLE["v"] = O.grid_update(og, M, Q, scene.dt, scene.gravity, scene.bc_layers)
    with ctx.Pool(n, initializer=_one_thread) as pool:
        done = sum(pool.map(_oracle_g2p_part, range(n)))
    tn = time.perf_counter() - t0
    _ORACLE.clear()
    assert done == S
    # configs[0] in full (32,768 particles), one core
    s0 = _config0_scene()
    og0 = O.grid_from_spec(s0.grid)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        M0, Q0 = O.p2g(og0, s0.x, s0.coeff, n_modes)
        v0 = O.grid_update(og0, M0, Q0, s0.dt, s0.gravity, s0.bc_layers)
        O.g2p(og0, v0, s0.x, n_modes, s0.dt)
        t_c0 = time.perf_counter() - t0
    sample_txt = (f"{S} particles (the first {S // (scene.P // (scene.grid.cells[2] // 2))} "
                  f"z-layers of cells of the dam-break block), one P2G + grid update + G2P at "
                  f"{n_modes} modes in float64 numpy")
    return {
        "value": S / t1,
        "unit": UNIT,
        "cores": 1,
        "kind": "oracle",
        "sample": f"{sample_txt}, {t1:.1f} s on one core",
        "cpu_model": _cpu_model(),
        "host_cpus": {"os_cpu_count": os.cpu_count(),
                      "affinity": len(os.sched_getaffinity(0)),
                      "share_used": n,
                      "note": "the all-cores run uses at most 16 workers: one GPU's share of "
                              "the host on this machine type"},
        "config0_full": {"value": s0.P / t_c0, "unit": UNIT, "cores": 1, "kind": "oracle",
                         "sample": f"all {s0.P} particles of the 32^3-cell parity case, one "
                                   f"P2G + grid update + G2P at {n_modes} modes, "
                                   f"{t_c0:.2f} s"},
        "all_cores": {"value": S / tn, "unit": UNIT, "cores": n, "kind": "oracle",
                      "sample": f"{sample_txt} over {n} particle chunks in {n} forked worker "
                                f"processes (grids summed between P2G and the update), "
                                f"{tn:.1f} s including the pools"},
    }


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not a measured configuration.",
              file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy()
        return

    import numpy as np

    import workloads as W

    scene = W.config1(0, n=args.cells)
    cpu = None
    if not args.no_cpu_baseline:  # first: the oracle's worker processes fork from here
        cpu = cpu_baseline(scene, args.n_modes, args.cpu_sample)

    import torch

    import paper_2308_01060_amd as pp

    torch.cuda.set_device(0)
    n_modes = args.n_modes
    P = scene.P
    workload = f"dambreak_{args.cells}cube_{P}"
    g = pp.grid_from_spec(scene.grid)
    x = torch.from_numpy(scene.x).cuda()
    c = torch.from_numpy(np.ascontiguousarray(scene.coeff[:, :n_modes])).cuda()
    ps = pp.ParticleSet(g, n_modes, x, c, dt=scene.dt, gravity=scene.gravity,
                        bc_layers=scene.bc_layers, track_order=False)
    for _ in range(args.warmup):
        ps.step()
    p2g_choice = ps.autotune()  # library autotuners, outside the timed region
    fused_choice = ps.autotune_fused()
    torch.cuda.synchronize()
    wall, phase = time_steps(ps, args.steps, torch)
    if ps.status_flags() != 0:
        raise RuntimeError(f"device status flags {ps.status_flags()} during the benchmark")
    ms_per_step = wall * 1e3 / args.steps
    value = P * args.steps / wall
    t_transfer = transfer_ms(phase)
    # The timed steps sort with polypic_sort_update (the previous step's keys; same
    # result as a full sort).  For reference, the full sort of the same state:
    full_sort_ms = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ps.sort(full=True)
        e1.record()
        torch.cuda.synchronize()
        full_sort_ms.append(e0.elapsed_time(e1))

    # 4-mode (APIC) comparison at the same size
    apic = None
    if not args.no_apic and n_modes != 4:
        c4 = torch.from_numpy(np.ascontiguousarray(scene.coeff[:, :4])).cuda()
        ps4 = pp.ParticleSet(g, 4, torch.from_numpy(scene.x).cuda(), c4, dt=scene.dt,
                             gravity=scene.gravity, bc_layers=scene.bc_layers,
                             track_order=False)
        for _ in range(args.warmup):
            ps4.step()
        choice4 = ps4.autotune()
        w4, ph4 = time_steps(ps4, args.steps, torch)
        apic = {"n_modes": 4, "ms_per_step": w4 * 1e3 / args.steps,
                "transfers_per_s": P * args.steps / w4,
                "p2g_g2p_transfers_per_s": P / (transfer_ms(ph4) * 1e-3),
                "p2g_config": {"path": "cells" if choice4.path == 1 else "bricks",
                               "block": choice4.block, "schedule": choice4.schedule,
                               "brick": choice4.brick},
                "phase_ms": {k: round(v, 4) for k, v in ph4.items()}}
        del ps4, c4

    # The same workload stepped unfused (separate P2G and G2P), for reference
    unfused = None
    if not args.no_unfused:
        psu = pp.ParticleSet(g, n_modes, torch.from_numpy(scene.x).cuda(),
                             torch.from_numpy(np.ascontiguousarray(scene.coeff[:, :n_modes])).cuda(),
                             dt=scene.dt, gravity=scene.gravity, bc_layers=scene.bc_layers,
                             track_order=False, fused=False)
        for _ in range(args.warmup):
            psu.step()
        psu.autotune()
        wu, phu = time_steps(psu, args.unfused_steps, torch)
        unfused = {"ms_per_step": wu * 1e3 / args.unfused_steps,
                   "transfers_per_s": P * args.unfused_steps / wu,
                   "p2g_g2p_transfers_per_s": P / (transfer_ms(phu) * 1e-3),
                   "steps": args.unfused_steps,
                   "phase_ms": {k: round(v, 4) for k, v in phu.items()}}
        del psu

    # roofline of the dominant kernel (HIP-event durations of its launches)
    if ps.fused:
        dom = "g2p2g"
        bpp = g2p2g_bytes_per_particle(n_modes)
        note = ("event time of the polypic_g2p2g call (the fused kernel alone: the grid "
                "update before it cleared the grid); bytes: x read, permutation, x and "
                "coefficients written")
    elif phase["p2g"] >= phase["g2p"]:
        dom, bpp = "p2g", p2g_bytes_per_particle(n_modes)
        note = "event time of the polypic_p2g call (grid clear, tile list and P2G kernels)"
    else:
        dom, bpp = "g2p", g2p_bytes_per_particle(n_modes)
        note = "event time of the polypic_g2p call (one kernel)"
    achieved = bpp * P / (phase[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom, workload), "kernel": dom,
                "bytes_per_particle": bpp, "note": note}

    moving = None
    if not args.no_moving:
        moving = moving_timing(pp, torch, W, args.cells, n_modes, args.steps, args.warmup)

    liquid_fabric = None
    if not args.no_liquid_fabric:
        liquid_fabric = liquid_fabric_timing(pp, torch, W, n_modes, args.steps, args.warmup)

    mac = None
    if not args.no_mac:
        mac = mac_timing(pp, torch, W, args.cells, n_modes, args.steps, args.warmup)

    shared = None
    if not args.no_shared_grid:
        shared = shared_grid_timing(pp, torch, W, n_modes, args.steps, args.warmup)

    affine = None
    if not args.no_affine:
        affine = affine_timing(pp, torch, W, args.cells, n_modes, args.steps, args.warmup)

    paper_scale = None
    if not args.no_paper_scale:
        paper_scale = paper_scale_timing(pp, torch, W, args.steps, args.warmup)

    adj = None
    if not args.no_adjoint:
        adj = adjoint_timing(pp, torch, W, args.cells, n_modes, args.adjoint_steps)
        if moving is not None:
            # one backward step (the three adjoint calls, event times) against one forward
            # step of the same moving state (sort, grid update, G2P2G, event times): the
            # ratio long rollouts converge to, without the forward's fixed costs
            bwd_step = sum(adj["bwd_step_phase_ms"].values())
            fwd_step = sum(moving["phase_ms"].values())
            adj["per_step"] = {"bwd_step_ms": round(bwd_step, 4),
                               "fwd_step_ms": round(fwd_step, 4),
                               "bwd_fwd_ratio": round(bwd_step / fwd_step, 3)}

    batch = None
    if not args.no_batch:
        batch = batch_timing(pp, torch, W, n_modes, args.batch_steps, 2)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded jittered dam-break block, workloads.config1)",
        "config": {"workload": workload, "n_modes": n_modes, "particles": P,
                   "grid_nodes": list(scene.grid.nodes), "ppc": 8, "dt": scene.dt,
                   "step": "sort (re-sort) + grid_update + g2p2g (G2P + advection fused with the "
                           "next step's P2G)"},
        "p2g_g2p_transfers_per_s": P / (t_transfer * 1e-3),
        "p2g_config": {"path": "cells" if p2g_choice.path == 1 else "bricks",
                       "block": p2g_choice.block, "schedule": p2g_choice.schedule,
                       "brick": p2g_choice.brick,
                       "chosen_by": "polypic_autotune_p2g"},
        "g2p2g_config": {"lane_group": fused_choice.lane_group,
                         "schedule": "xcd" if fused_choice.schedule == 1 else "linear",
                         "chosen_by": "polypic_autotune_g2p2g"},
        "phase_ms": {k: round(v, 4) for k, v in phase.items()},
        "unfused": unfused,
        "sort": {"timed": "polypic_sort_update (exact re-sort from the previous step's keys)",
                 "full_sort_ms": round(float(np.median(full_sort_ms)), 4)},
        "apic_4mode": apic,
        "moving": moving,
        "liquid_fabric": liquid_fabric,
        "paper_scale": paper_scale,
        "mac": mac,
        "shared_grid": shared,
        "affine_map": affine,
        "bwd_fwd_ratio": None if adj is None else round(adj["bwd_fwd_ratio"], 3),
        "bwd_fwd_ratio_per_step": (None if adj is None or "per_step" not in adj
                                   else adj["per_step"]["bwd_fwd_ratio"]),
        "adjoint": adj,
        "batched": batch,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
