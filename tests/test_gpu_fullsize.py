"""The benchmarked workload at its full size, in the launch configuration the
benchmark times: periodic diffusion-advection on 4096^2 (D = 1, cell Peclet
number 1, h = 50 x CFL), phi_1, phi_2, phi_3 of the seeded N(0,1) vector from
one Newton basis at rtol 1e-8, after 20 power sweeps from the seeded start
vector, with the launch shapes the tuner picks (as the benchmark does) and
with the LDS-tile windows of six on 8-row tiles and 768 workgroups forced.

Checks: the spectral estimate against the oracle's power iteration (1e-12);
every output element by element against the oracle's Leja loop with the same
shift and scale (1e-10; a borderline stop flipped by the order of the norm
reductions is compared at the GPU's count); and against the exact Fourier
solution at ten times the tolerance.
"""
import numpy as np
import pytest

from oracle.exact import phi_fft
from oracle.operators import make_apply
from oracle.phi_action import leja_phi, power_iteration
from paper_2310_08344_amd import binding as B
from paper_2310_08344_amd import workloads as W
from tests.gpu_helpers import host, oracle_parity, rel, say

pytestmark = pytest.mark.gpu

N = 4096
LS = [1, 2, 3]


@pytest.fixture(scope="module")
def setup(lx):
    import torch
    p, v = W.config2(n=N)
    ctx = lx.context(n_max=p.N, k_max=3)
    dev = torch.device("cuda:0")
    tv = torch.as_tensor(v).to(dev)
    x0 = W.start_vector(N)
    say("full size: tune 4096^2 K=3")
    ctx.tune(B.make_operator(p), K=3, sweeps=8)
    say("full size: spectrum")
    rho, c, g = ctx.spectrum(B.make_operator(p), x0=torch.as_tensor(x0).to(dev), iters=20)
    A = make_apply(p)
    rho_o, _ = power_iteration(A, x0, 20)
    yield dict(ctx=ctx, p=p, v=v, tv=tv, rho=rho, rho_o=rho_o, c=c, g=g, A=A, ref={})
    ctx.close()


def _solve(s, forced):
    import torch
    ctx, p = s["ctx"], s["p"]
    outs = [torch.empty_like(s["tv"]) for _ in LS]
    if forced:
        ctx.set_depth(6, 8, 768)
        ctx.set_window_kernel(1)
    try:
        r = ctx.phi_leja(B.make_operator(p), s["tv"], outs, LS, p.h, s["c"], s["g"], rtol=1e-8, max_iters=300)
    finally:
        ctx.set_depth(0)
        ctx.set_window_kernel(0)
    return r, [host(o) for o in outs]


def _oracle(s, force):
    key = None if force is None else tuple(force)
    if key not in s["ref"]:
        p = s["p"]
        say("full size: oracle Leja loop", "own stop rule" if force is None else f"forced {force}")
        s["ref"][key] = leja_phi(s["A"], s["v"], [(l, 1.0, 1.0) for l in LS], p.h, s["c"], s["g"], 1e-8, 0.0, 300,
                                 force)
    return s["ref"][key]


def test_spectral_estimate_matches_oracle(setup):
    assert abs(setup["rho"] - setup["rho_o"]) <= 1e-12 * setup["rho_o"]


@pytest.mark.parametrize("forced", [False, True], ids=["tuned", "lds_windows_6_th8_768"])
def test_benchmarked_solve_matches_oracle_and_exact(setup, forced):
    s = setup
    say("full size: solve", "forced LDS windows" if forced else "tuned shapes")
    r, outs = _solve(s, forced)
    assert r.status == B.LX_OK
    if forced:
        assert r.stats["depth"] == 6 and r.stats["marching"] == 0
    say("depth", r.stats["depth"], "marching", r.stats["marching"], "sweeps", r.iters)
    _, errs, flipped = oracle_parity(outs, r.iters, lambda f: _oracle(s, f), 1e-10)
    p = s["p"]
    ex = [phi_fft(s["v"], l, p.h, p.D, p.vx, p.vy, p.dx, p.dy) for l in LS]
    e_ex = [rel(o, x) for o, x in zip(outs, ex)]
    say("oracle parity", errs, "flipped", flipped, "exact", e_ex)
    assert max(e_ex) <= 10 * 1e-8
