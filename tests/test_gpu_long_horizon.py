"""Parity on the long-horizon shape of Table II: a 118-bus grid (186 lines,
54 generators) over 10080 periods (one week at 5-minute resolution, 11.0M
variables, the table's "11m" row), the regime where a period's lines fit
one tile and the work is spread over periods.  J, H, c, grad, f and J^T v
element by element against the oracle; K on every row of four sampled
periods and by structure everywhere."""
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
def test_long_horizon_parity():
    import torch
    from paper_2405_14032_amd import capi
    dev = torch.device("cuda:0")
    net = synth.make_network(118, 186, 54, 10080, 118)
    pt = synth.make_point(net, 118)
    L = O.Layout(net)
    print(f"long horizon: N={net.N} B={net.B} G={net.G} T={net.T} n={L.n} m={L.m}", flush=True)
    assert L.n == 10_967_040 and L.m == 16_057_386  # Table II: 11m variables, 16m constraints
    M = capi.Model([net], device=0)
    M.use_current_torch_stream()
    M.autotune(TUNE_CACHE)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    X, LAM, DX, D = t(pt.x), t(pt.lam), t(pt.diag_x), t(pt.dcon)
    e = lambda k: torch.full((k,), float("nan"), dtype=torch.float64, device=dev)
    out = dict(f=e(1), grad=e(M.n), c=e(M.m), jvals=e(M.nnz_jac), hvals=e(M.nnz_hess), jtv=e(M.n),
               kvals=e(M.nnz_kkt))
    M.sweep_graph(M.sweep_args(x=X, lam=LAM, sigma=pt.sigma, v=LAM, diag_x=DX, dcon=D, **out))
    rp = torch.empty(M.n + 1, dtype=torch.int64, device=dev)
    ci = torch.empty(M.nnz_kkt, dtype=torch.int32, device=dev)
    M.kkt_structure(rp, ci)
    torch.cuda.synchronize()
    G = {k: v.cpu().numpy() for k, v in out.items()}
    rp, ci = rp.cpu().numpy(), ci.cpu().numpy().astype(np.int64)
    M.close()
    print("gpu done; oracle", flush=True)
    ojr, ojc, ojv, ojm = O.jacobian(net, pt.x, with_mag=True)
    GC.assert_close(G["jvals"], ojv, ojm, GC.TOL, "long J")
    ohr, ohc, ohv, ohm = O.hessian(net, pt.x, pt.lam, pt.sigma, with_mag=True)
    GC.assert_close(G["hvals"], ohv, ohm, GC.TOL, "long H")
    GC.assert_close(G["c"], *O.constraints(net, pt.x, with_mag=True), GC.TOL, "long c")
    GC.assert_close(G["grad"], O.gradient(net, pt.x), O.gradient_mag(net, pt.x), GC.TOL, "long grad")
    GC.assert_close(G["f"], np.array([O.objective(net, pt.x)]), np.array([O.objective_mag(net, pt.x)]),
                    GC.TOL, "long f")
    GC.assert_close(G["jtv"], *O.jtprod(net, pt.x, pt.lam, with_mag=True), GC.TOL, "long J^T v")
    assert rp[0] == 0 and rp[-1] == M.nnz_kkt and np.all(np.diff(rp) >= 1)
    last = rp[1:] - 1
    assert np.array_equal(ci[last], np.arange(L.n))
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
    GC.assert_close(G["kvals"][gidx], okv[oidx], okm[oidx], GC.TOL_KKT, "long K sampled periods")
