"""Parity at the paper-scale size (N=10000, B=13000, G=2000, T=168: 12.77M
variables) in the launch configuration the benchmark times (its tuned tile
shapes).  J, H, c, grad, f and J^T v are compared element by element with
the oracle; K on every row of four sampled periods (the oracle restricted to
those rows computes them exactly) and by structural properties everywhere."""
import os

import numpy as np
import pytest

from oracle import opf_oracle as O
from paper_2405_14032_amd import synth

import gpu_common as GC

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE_CACHE = os.path.join(ROOT, "paper_2405_14032_amd", "tune", "mi355x.json")


@pytest.mark.timeout(900)
def test_paper_scale_parity():
    import torch
    from paper_2405_14032_amd import capi
    dev = torch.device("cuda:0")
    net = synth.config_network("paper")
    pt = synth.make_point(net, 3)
    print(f"paper scale: N={net.N} B={net.B} G={net.G} T={net.T}", flush=True)
    M = capi.Model([net], device=0)
    M.use_current_torch_stream()
    os.makedirs(os.path.dirname(TUNE_CACHE), exist_ok=True)
    M.autotune(TUNE_CACHE)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    X, LAM, DX, D = t(pt.x), t(pt.lam), t(pt.diag_x), t(pt.dcon)
    e = lambda k: torch.empty(k, dtype=torch.float64, device=dev)
    out = dict(f=e(1), grad=e(M.n), c=e(M.m), jvals=e(M.nnz_jac), hvals=e(M.nnz_hess), jtv=e(M.n),
               kvals=e(M.nnz_kkt))
    M.sweep(M.sweep_args(x=X, lam=LAM, sigma=pt.sigma, v=LAM, diag_x=DX, dcon=D, **out))
    jr = torch.empty(M.nnz_jac, dtype=torch.int32, device=dev)
    jc = torch.empty_like(jr)
    hr = torch.empty(M.nnz_hess, dtype=torch.int32, device=dev)
    hc = torch.empty_like(hr)
    rp = torch.empty(M.n + 1, dtype=torch.int64, device=dev)
    ci = torch.empty(M.nnz_kkt, dtype=torch.int32, device=dev)
    M.jac_structure(jr, jc)
    M.hess_structure(hr, hc)
    M.kkt_structure(rp, ci)
    torch.cuda.synchronize()
    G = {k: v.cpu().numpy() for k, v in out.items()}
    jr, jc, hr, hc = (a.cpu().numpy().astype(np.int64) for a in (jr, jc, hr, hc))
    rp, ci = rp.cpu().numpy(), ci.cpu().numpy().astype(np.int64)
    M.close()
    print("gpu done; oracle J", flush=True)
    ojr, ojc, ojv, ojm = O.jacobian(net, pt.x, with_mag=True)
    assert np.array_equal(jr, ojr) and np.array_equal(jc, ojc)
    GC.assert_close(G["jvals"], ojv, ojm, GC.TOL, "paper J")
    print("oracle H", flush=True)
    ohr, ohc, ohv, ohm = O.hessian(net, pt.x, pt.lam, pt.sigma, with_mag=True)
    assert np.array_equal(hr, ohr) and np.array_equal(hc, ohc)
    GC.assert_close(G["hvals"], ohv, ohm, GC.TOL, "paper H")
    print("oracle c, grad, f, J^T v", flush=True)
    GC.assert_close(G["c"], *O.constraints(net, pt.x, with_mag=True), GC.TOL, "paper c")
    GC.assert_close(G["grad"], O.gradient(net, pt.x), O.gradient_mag(net, pt.x), GC.TOL, "paper grad")
    GC.assert_close(G["f"], np.array([O.objective(net, pt.x)]), np.array([O.objective_mag(net, pt.x)]),
                    GC.TOL, "paper f")
    GC.assert_close(G["jtv"], *O.jtprod(net, pt.x, pt.lam, with_mag=True), GC.TOL, "paper J^T v")
    # K: structural properties at full size
    L = O.Layout(net)
    assert rp[0] == 0 and rp[-1] == M.nnz_kkt and np.all(np.diff(rp) >= 1)
    rows = np.repeat(np.arange(L.n), np.diff(rp))
    assert np.all(ci <= rows)
    last = rp[1:] - 1
    assert np.array_equal(ci[last], np.arange(L.n))  # diagonal closes every row
    inner = np.ones(len(ci), dtype=bool)
    inner[rp[1:-1]] = False
    inner[0] = False
    assert np.all(np.diff(ci)[inner[1:]] > 0)  # strictly ascending within rows
    # K: every row of four sampled periods against the oracle
    print("oracle K (sampled periods)", flush=True)
    mask = np.zeros(L.n, dtype=bool)
    for tt in (0, 1, net.T // 2, net.T - 1):
        mask[tt * L.n_p:(tt + 1) * L.n_p] = True
    orp, oci, okv, okm = O.condensed(L.n, (ojr, ojc, ojv), (ohr, ohc, ohv), pt.diag_x, pt.dcon, row_mask=mask,
                                     jac_mag=ojm, hess_mag=ohm)
    sel = np.nonzero(mask)[0]
    a, b = rp[sel], rp[sel + 1]
    oa, ob = orp[sel], orp[sel + 1]
    assert np.array_equal(b - a, ob - oa)
    gidx = np.concatenate([np.arange(x, y) for x, y in zip(a, b)])
    oidx = np.concatenate([np.arange(x, y) for x, y in zip(oa, ob)])
    assert np.array_equal(ci[gidx], oci[oidx])
    GC.assert_close(G["kvals"][gidx], okv[oidx], okm[oidx], GC.TOL_KKT, "paper K sampled periods")
