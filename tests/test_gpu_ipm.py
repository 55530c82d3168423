"""The lifted-KKT interior-point loop on the GPU (opf_ipm_solve) against the
oracle's loop (the same algorithm written plainly on the CPU with a sparse LU
and a dense positive-definiteness test), with the filter line search (the
default) and without it: both converge to the stopping tolerance 1e-4 and
reach the same point.  Iterates agree to rounding at first and the rounding
is amplified along the iterations, so the comparison is of the converged
solutions: objective to 1e-5 relative (the stopping tolerance leaves the
objective about that far from the optimum), x to 1e-3, and iteration counts
within 2; on an infeasible grid both stop with the same status."""
import numpy as np
import pytest

from oracle import opf_oracle as O
from paper_2405_14032_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _gpu_ipm(nets, torch, dev, **opts):
    from paper_2405_14032_amd import capi
    M = capi.Model(nets, device=0)
    M.use_current_torch_stream()
    F = capi.Chol(M)
    x = torch.full((M.n,), float("nan"), dtype=torch.float64, device=dev)
    y = torch.full((M.m,), float("nan"), dtype=torch.float64, device=dev)
    r = capi.ipm_solve(M, F, x, y, **opts)
    torch.cuda.synchronize()
    out = (r, x.cpu().numpy(), y.cpu().numpy(), list(M.x_off))
    F.close()
    M.close()
    return out


@pytest.mark.parametrize("line_search", [1, 0])
@pytest.mark.parametrize("name", ["tiny", "ragged_small"])
def test_ipm_matches_oracle(name, line_search, dev):
    import torch
    net = synth.config_network("tiny") if name == "tiny" else synth.make_network(301, 517, 63, 2, 41)
    print(f"ipm case {name}: {(net.N, net.B, net.G, net.T)} line_search={line_search}", flush=True)
    r, x, _, _ = _gpu_ipm([net], torch, dev, line_search=line_search)
    print("gpu", r, flush=True)
    ref = O.ipm_solve(net, line_search=bool(line_search))
    assert r["converged"] == 1 and ref["converged"]
    assert r["status_name"] == ref["status"] == "converged"
    assert abs(r["iterations"] - ref["iterations"]) <= 2, (r["iterations"], ref["iterations"])
    assert abs(r["objective"] - ref["objective"]) <= 1e-5 * abs(ref["objective"])
    assert abs(O.objective(net, x) - r["objective"]) <= 1e-9 * abs(r["objective"])
    assert np.max(np.abs(x - ref["x"])) <= 1e-3


def test_ipm_reports_stall_on_infeasible_grid(dev):
    """Every period's load above the total generating capacity (no feasible
    point): the line search finds no acceptable step within a few
    iterations and the loop stops with status "stalled", as the oracle's."""
    import dataclasses
    import torch
    base = synth.config_network("tiny")
    net = dataclasses.replace(base, pd=base.pd * 30, qd=base.qd * 30)
    assert np.all(net.pd.sum(axis=1) > net.pmax.sum())
    r, x, _, _ = _gpu_ipm([net], torch, dev, max_iter=100)
    print("gpu", r, flush=True)
    ref = O.ipm_solve(net, max_iter=100)
    assert r["status_name"] == ref["status"] == "stalled" and r["converged"] == 0
    assert abs(r["iterations"] - ref["iterations"]) <= 2, (r["iterations"], ref["iterations"])
    assert r["iterations"] <= 20 and r["theta"] > 1.0


@pytest.mark.timeout(600)
def test_ipm_uncapped_mid_grid_ends_with_a_status(dev):
    """The 2000-bus, 24-period grid with its loads as drawn (not capped):
    the loop either converges or reports a stall, well inside the iteration
    limit, instead of running into the limit."""
    import torch
    net = synth.config_network("mid")
    print("ipm case mid, uncapped loads", flush=True)
    r, x, _, _ = _gpu_ipm([net], torch, dev, max_iter=150)
    print("gpu", r, flush=True)
    assert r["status_name"] in ("converged", "stalled"), r
    assert np.all(np.isfinite(x))


@pytest.mark.timeout(600)
def test_ipm_mid_grid_capped_load_whole_solve(dev):
    """A whole solve at the 2000-bus, 24-period size (n = 422400) with loads
    capped at 30 % of capacity: converged to 1e-4, and the returned point,
    checked with the oracle's own functions, inside the variable bounds and
    the relaxed row bounds up to the stopping tolerance, with the objective
    the oracle computes there.  (The oracle's loop is too slow to run to
    the end at this size, so the point is checked, not compared.)"""
    import torch
    net = synth.cap_load(synth.config_network("mid"), 0.3)
    print("ipm case mid, loads capped at 0.3", flush=True)
    r, x, y, _ = _gpu_ipm([net], torch, dev)
    print("gpu", r, flush=True)
    assert r["converged"] == 1 and r["iterations"] <= 120
    xl, xu, cl, cu = O.bounds(net)
    relax, tol = 1e-4, 1e-4
    eq = cl == cu
    sl, su = np.where(eq, cl - relax, cl), np.where(eq, cu + relax, cu)
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))
    assert np.all(x >= xl) and np.all(x <= xu)
    c = O.constraints(net, x)
    assert np.all(c >= sl - tol) and np.all(c <= su + tol), (np.max(sl - c), np.max(c - su))
    assert abs(O.objective(net, x) - r["objective"]) <= 1e-9 * abs(r["objective"])


def test_ipm_batch_solves_each_instance(dev):
    """Two instances solved jointly: each instance's part is that
    instance's optimum (the oracle solving it alone)."""
    import torch
    nets = [synth.config_network("tiny"), synth.make_network(20, 30, 6, 3, 12)]
    r, x, _, offs = _gpu_ipm(nets, torch, dev)
    assert r["converged"] == 1
    total = 0.0
    for k, net in enumerate(nets):
        ref = O.ipm_solve(net)
        assert ref["converged"]
        xk = x[offs[k]:offs[k + 1]]
        assert abs(O.objective(net, xk) - ref["objective"]) <= 1e-5 * abs(ref["objective"]), k
        total += ref["objective"]
    assert abs(r["objective"] - total) <= 1e-5 * abs(total)


def test_ipm_inertia_correction_path(dev):
    """A static pivot threshold (5) above some of the tiny grid's pivots makes
    the first factorization of many iterations report static pivots: the
    loop raises delta_w until none is reported (more factorizations than
    iterations) and keeps making progress.  The threshold distorts the
    method (a regularised step every iteration), so only the first 15
    iterations are run."""
    import torch
    net = synth.config_network("tiny")
    r, x, _, _ = _gpu_ipm([net], torch, dev, pivot_tol=5.0, max_iter=15)
    assert r["iterations"] == 15 and r["factorizations"] >= r["iterations"] + 5
    assert r["err"] < 1.0  # from 40 at the start


@pytest.mark.parametrize("line_search", [1, 0])
def test_ipm_stops_when_inertia_correction_runs_out(line_search, dev):
    """A static pivot threshold (1e30) that no pivot passes at any delta_w
    up to dw_max (1e10): the first iteration's correction runs out and the
    loop returns the start point with status stalled (as the oracle's loop
    does when its positive-definiteness test never passes), after one
    factorization at delta_w = 0 and one per delta_w <= dw_max."""
    import torch
    net = synth.config_network("tiny")
    r, x, _, _ = _gpu_ipm([net], torch, dev, pivot_tol=1e30, max_iter=10, line_search=line_search)
    assert r["status_name"] == "stalled" and r["converged"] == 0 and r["iterations"] == 0
    grow = 100.0 if line_search else 8.0
    k = int(np.floor(np.log(1e10 / 1e-4) / np.log(grow) + 1e-9)) + 1
    assert r["factorizations"] == 1 + k, (r["factorizations"], k)
    x0 = O.ipm_start(net, 1e-4)["x"]
    assert np.max(np.abs(x - x0)) <= 1e-12 * max(1.0, np.max(np.abs(x0)))


def test_ipm_rejects_bad_options(dev):
    import torch
    from paper_2405_14032_amd import capi
    net = synth.config_network("tiny")
    M = capi.Model([net], device=0)
    F = capi.Chol(M)
    x = torch.empty(M.n, dtype=torch.float64, device=dev)
    for bad in (dict(tol=0.0), dict(sigma=1.5), dict(tau=1.0), dict(dw_grow=1.0), dict(kappa_mu=1.0),
                dict(theta_mu=1.0), dict(tau_min=1.0), dict(gamma_alpha=0.0)):
        with pytest.raises(capi.OpfError):
            capi.ipm_solve(M, F, x, **bad)
    F.close()
    M.close()


def test_ipm_rejects_chol_of_another_model(dev):
    # the factor object must come from the same model: the binding refuses
    # the pair, and so does the C ABI itself (OPF_EINVAL, nothing enqueued)
    import ctypes as C
    import torch
    from paper_2405_14032_amd import capi
    net = synth.config_network("tiny")
    M1 = capi.Model([net], device=0)
    M2 = capi.Model([net], device=0)
    F2 = capi.Chol(M2)
    x = torch.empty(M1.n, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError, match="another model"):
        capi.ipm_solve(M1, F2, x)
    r = capi.opf_ipm_result()
    assert capi.opf_ipm_solve(M1.h, F2.h, None, x.data_ptr(), None, C.byref(r)) == capi.OPF_EINVAL
    assert b"another model" in capi.opf_last_error()
    F2.close()
    M2.close()
    M1.close()
