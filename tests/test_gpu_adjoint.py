"""Adjoint form on the GPU: c(x, pd, qd) as a torch.autograd.Function.

Forward must match the oracle's constraint rows at the given load profile;
backward must return J(x)^T g (the oracle's transposed product) and the load
adjoint -(g_balP, g_balQ) (the load enters eq. (1b)-(1c) with coefficient
-1).  Independently of the oracle, the backward is checked against central
differences of the GPU forward and by torch.autograd.gradcheck on the 14-bus
case."""
import numpy as np
import pytest

from oracle import opf_oracle as O
from paper_2405_14032_amd import synth

import gpu_common as GC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cuda_dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def _load_tensors(nets, torch, dev, scale=1.0):
    pd = np.concatenate([net.pd.reshape(-1) * scale for net in nets])
    qd = np.concatenate([net.qd.reshape(-1) * scale for net in nets])
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    return t(pd), t(qd)


def _scaled(net, scale):
    import dataclasses
    return dataclasses.replace(net, pd=net.pd * scale, qd=net.qd * scale)


@pytest.mark.parametrize("which", ["tiny", "ragged_batch"])
def test_adjoint_matches_oracle(which, cuda_dev):
    import torch
    from paper_2405_14032_amd import autograd, capi
    if which == "tiny":
        nets = [synth.config_network("tiny")]
    else:
        nets = [synth.make_network(31, 45, 7, 3, seed=71), synth.make_network(14, 20, 5, 5, seed=72),
                synth.make_network(57, 80, 11, 2, seed=73)]
    pts = [synth.make_point(net, 20 + k) for k, net in enumerate(nets)]
    M = capi.Model(nets, device=0)
    dev = cuda_dev
    x = torch.tensor(np.concatenate([p.x for p in pts]), dtype=torch.float64, device=dev, requires_grad=True)
    pd, qd = _load_tensors(nets, torch, dev, scale=1.07)  # a load profile other than the built-in one
    pd.requires_grad_(True)
    qd.requires_grad_(True)
    c = autograd.opf_cons(x, pd, qd, M)
    g = torch.tensor(np.random.default_rng(5).standard_normal(M.m), dtype=torch.float64, device=dev)
    gx, gpd, gqd = torch.autograd.grad(c, (x, pd, qd), grad_outputs=g)
    torch.cuda.synchronize()
    c, gx, gpd, gqd, g = (a.detach().cpu().numpy() for a in (c, gx, gpd, gqd, g))
    xo = no = co = 0
    for net, p in zip(nets, pts):
        L = O.Layout(net)
        nl = net.T * net.N
        sn = _scaled(net, 1.07)
        oc, ocm = O.constraints(sn, p.x, with_mag=True)
        GC.assert_close(c[co:co + L.m], oc, ocm, GC.TOL, f"{which} forward c")
        ojt, ojm = O.jtprod(sn, p.x, g[co:co + L.m], with_mag=True)
        GC.assert_close(gx[xo:xo + L.n], ojt, ojm, GC.TOL, f"{which} backward x")
        ogp, ogq = O.load_adjoint(sn, g[co:co + L.m])
        assert np.array_equal(gpd[no:no + nl], ogp.reshape(-1)), f"{which} backward pd"
        assert np.array_equal(gqd[no:no + nl], ogq.reshape(-1)), f"{which} backward qd"
        xo += L.n
        co += L.m
        no += nl
    M.close()


def test_adjoint_central_differences(cuda_dev):
    """Directional derivative of g^T c along random (dx, dpd, dqd) by central
    differences (h = 1e-6) of the GPU forward, against the backward's inner
    product; c is smooth in x and affine in the load, so the quotient's
    truncation error is O(h^2) and rounding dominates (~1e-10 relative)."""
    import torch
    from paper_2405_14032_amd import autograd, capi
    net = synth.config_network("tiny")
    pt = synth.make_point(net, 9)
    M = capi.Model([net], device=0)
    dev = cuda_dev
    rng = np.random.default_rng(17)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    x0 = t(pt.x)
    pd0, qd0 = _load_tensors([net], torch, dev)
    g = t(rng.standard_normal(M.m))
    dx, dp, dq = t(rng.standard_normal(M.n)), t(rng.standard_normal(pd0.numel())), t(rng.standard_normal(qd0.numel()))
    x = x0.clone().requires_grad_(True)
    pd = pd0.clone().requires_grad_(True)
    qd = qd0.clone().requires_grad_(True)
    c = autograd.opf_cons(x, pd, qd, M)
    gx, gpd, gqd = torch.autograd.grad(c, (x, pd, qd), grad_outputs=g)
    adj = float((gx * dx).sum() + (gpd * dp).sum() + (gqd * dq).sum())
    h = 1e-6
    with torch.no_grad():
        cp = autograd.opf_cons(x0 + h * dx, pd0 + h * dp, qd0 + h * dq, M)
        cm = autograd.opf_cons(x0 - h * dx, pd0 - h * dp, qd0 - h * dq, M)
        fd = float((g * (cp - cm)).sum()) / (2 * h)
    torch.cuda.synchronize()
    assert abs(adj - fd) <= 1e-8 * max(1.0, abs(adj)), (adj, fd)
    M.close()


def test_adjoint_gradcheck_tiny(cuda_dev):
    import torch
    from paper_2405_14032_amd import autograd, capi
    net = synth.make_network(6, 8, 2, 2, seed=91)
    pt = synth.make_point(net, 4)
    M = capi.Model([net], device=0)
    dev = cuda_dev
    x = torch.tensor(pt.x, dtype=torch.float64, device=dev, requires_grad=True)
    pd, qd = _load_tensors([net], torch, dev)
    pd.requires_grad_(True)
    qd.requires_grad_(True)
    f = lambda a, b, c: autograd.opf_cons(a, b, c, M)
    assert torch.autograd.gradcheck(f, (x, pd, qd), eps=1e-6, atol=1e-7, rtol=1e-6)
    M.close()
