"""Shared helpers of the GPU tests (test infrastructure)."""
import math
import sys

import numpy as np

from paper_2310_08344_amd import workloads as W


def say(*args):
    """Names the case on stdout before a GPU step, flushed."""
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


def host(t):
    return t.detach().to("cpu").numpy()


def rel(a, b):
    nb = float(np.linalg.norm(np.ravel(b)))
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b))) / (nb if nb > 0 else 1.0)


def diffadv_setup(nx, ny, D=1.0, vx=None, vy=None, cfl=50.0):
    """Periodic diffusion-advection on [0,1)^2 with nx x ny cells: returns
    (params dict, h).  Default velocity: cell Peclet number 1 per axis."""
    dx, dy = 1.0 / nx, 1.0 / ny
    vx = D / dx if vx is None else vx
    vy = D / dy if vy is None else vy
    h = cfl * W.diffadv_cfl_step(D, vx, vy, dx, dy)
    return dict(nx=nx, ny=ny, dx=dx, dy=dy, D=D, vx=vx, vy=vy), h


def closed_form_shift(D, vx, vy, dx, dy, safety=1.05):
    rho = 2.0 / W.diffadv_cfl_step(D, vx, vy, dx, dy)
    lam = -safety * rho
    return lam / 2.0, -lam / 4.0


def oracle_parity(gpu_outs, gpu_iters, run_oracle, tol):
    """Compares GPU outputs with the oracle.  When a borderline stop
    decision went the other way (iteration counts differ by one), the oracle
    is rerun with the GPU's counts and the event is reported."""
    ref = run_oracle(None)
    flipped = False
    if list(ref.iters) != list(gpu_iters):
        assert all(abs(a - b) <= 1 for a, b in zip(ref.iters, gpu_iters)), (ref.iters, gpu_iters)
        flipped = True
        say("stop decision differs by one sweep; comparing at the GPU's counts", ref.iters, gpu_iters)
        ref = run_oracle(list(gpu_iters))
    errs = [rel(g, r) for g, r in zip(gpu_outs, ref.p)]
    for e in errs:
        assert e <= tol, (errs, tol)
    return ref, errs, flipped


def oracle_step_parity(gpu_out, gpu_iters, run_step, tol):
    """Compares an integrator step with the oracle's.  Every phi action of
    the step has its own stop rule; when a borderline decision went the
    other way in one of them (counts differ by one), the oracle step is
    rerun forced to the GPU's counts, action by action, and compared at the
    same tolerance.  Returns (oracle step, relative error, flipped)."""
    ref = run_step(None)
    flipped = list(ref.iters) != list(gpu_iters)
    if flipped:
        assert all(abs(a - b) <= 1 for a, b in zip(ref.iters, gpu_iters)), (ref.iters, gpu_iters)
        say("stop decision differs by one sweep; comparing at the GPU's counts", ref.iters, gpu_iters)
        ref = run_step(list(gpu_iters))
    assert ref.status == "ok", ref.status
    err = rel(gpu_out, ref.u_next)
    assert err <= tol, (err, tol)
    return ref, err, flipped
