"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and compute the oracle's values and cancellation scales on the same seeded
inputs."""
from __future__ import annotations

import numpy as np

from oracle import opf_oracle as O

TOL = 1e-12       # c, grad, f, J, H, J^T v: per value, relative to max(|ref|, mag)
TOL_KKT = 1e-10   # K after duplicate-slot summation


def assert_close(gpu, ref, mag, tol, what):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape, f"{what}: shape {gpu.shape} != {ref.shape}"
    err = np.abs(gpu - ref)
    bound = tol * np.maximum(np.abs(ref), np.asarray(mag, dtype=np.float64))
    bad = ~(err <= bound)
    if bad.any():
        k = int(np.argmax(np.where(bad, err / np.maximum(bound, 1e-300), 0)))
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} values exceed tol {tol}; e.g. [{k}] "
                             f"gpu={gpu.flat[k]!r} ref={ref.flat[k]!r} mag={np.asarray(mag).flat[k]!r}")


def oracle_all(net, pt, v=None, with_kkt=True):
    """Every oracle output with its magnitude scale."""
    L = O.Layout(net)
    v = pt.lam if v is None else v
    out = {}
    out["f"] = (O.objective(net, pt.x), O.objective_mag(net, pt.x))
    out["grad"] = (O.gradient(net, pt.x), O.gradient_mag(net, pt.x))
    out["c"] = O.constraints(net, pt.x, with_mag=True)
    jr, jc, jv, jm = O.jacobian(net, pt.x, with_mag=True)
    out["jac_idx"] = (jr, jc)
    out["jac"] = (jv, jm)
    hr, hc, hv, hm = O.hessian(net, pt.x, pt.lam, pt.sigma, with_mag=True)
    out["hess_idx"] = (hr, hc)
    out["hess"] = (hv, hm)
    out["jtv"] = O.jtprod(net, pt.x, v, with_mag=True)
    out["bounds"] = O.bounds(net)
    gp, gq = O.load_adjoint(net, pt.lam)
    out["load_adj"] = (gp.reshape(-1), gq.reshape(-1))
    if with_kkt:
        rp, ci, kv, km = O.condensed(L.n, (jr, jc, jv), (hr, hc, hv), pt.diag_x, pt.dcon, jac_mag=jm,
                                     hess_mag=hm)
        out["kkt_idx"] = (rp, ci)
        out["kkt"] = (kv, km)
    return out


def gpu_all(model, x, lam, sigma, v, diag_x, dcon, torch, dev, graph=False):
    """Run every evaluation call of the model on device tensors; returns
    host numpy arrays."""
    n, m = model.n, model.m
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    X, LAM, V, DX, D = t(x), t(lam), t(v), t(diag_x), t(dcon)
    z = lambda k, dt=torch.float64: torch.full((k,), float("nan"), dtype=dt, device=dev) if dt == torch.float64 \
        else torch.full((k,), -7, dtype=dt, device=dev)
    f = z(model.ninst)
    g, c, jv, hv, jtv, kv = z(n), z(m), z(model.nnz_jac), z(model.nnz_hess), z(n), z(model.nnz_kkt)
    model.use_current_torch_stream()
    if graph:
        args = model.sweep_args(x=X, lam=LAM, sigma=sigma, v=V, diag_x=DX, dcon=D, f=f, grad=g, c=c, jvals=jv,
                                hvals=hv, jtv=jtv, kvals=kv)
        model.sweep_graph(args)
    else:
        model.eval_obj(X, f)
        model.eval_grad(X, g)
        model.eval_cons(X, c)
        model.eval_jac(X, jv)
        model.eval_hess(X, LAM, sigma, hv)
        model.jtprod(X, V, jtv)
        model.assemble_condensed(hv, jv, DX, D, kv)
    jr, jc = z(model.nnz_jac, torch.int32), z(model.nnz_jac, torch.int32)
    hr, hc = z(model.nnz_hess, torch.int32), z(model.nnz_hess, torch.int32)
    rp, ci = z(n + 1, torch.int64), z(model.nnz_kkt, torch.int32)
    model.jac_structure(jr, jc)
    model.hess_structure(hr, hc)
    model.kkt_structure(rp, ci)
    lv, uv, lc, uc = z(n), z(n), z(m), z(m)
    model.bounds(lv, uv, lc, uc)
    nload = sum(net.T * net.N for net in model.nets)
    gpd, gqd = z(nload), z(nload)
    model.load_adjoint(LAM, gpd, gqd)
    torch.cuda.synchronize()
    h = lambda a: a.cpu().numpy()
    return dict(f=h(f), grad=h(g), c=h(c), jac=h(jv), hess=h(hv), jtv=h(jtv), kkt=h(kv),
                jac_idx=(h(jr), h(jc)), hess_idx=(h(hr), h(hc)), kkt_idx=(h(rp), h(ci)),
                bounds=(h(lv), h(uv), h(lc), h(uc)), load_adj=(h(gpd), h(gqd)))


def compare(G, R, what=""):
    """Element-wise parity of one instance (indices bit-exact)."""
    assert_close(G["f"], np.array([R["f"][0]]), np.array([R["f"][1]]), TOL, what + " f")
    assert_close(G["grad"], *R["grad"], TOL, what + " grad")
    assert_close(G["c"], *R["c"], TOL, what + " c")
    for key in ("jac_idx", "hess_idx"):
        for a, b in zip(G[key], R[key]):
            assert np.array_equal(a.astype(np.int64), b.astype(np.int64)), what + " " + key
    assert_close(G["jac"], *R["jac"], TOL, what + " J")
    assert_close(G["hess"], *R["hess"], TOL, what + " H")
    assert_close(G["jtv"], *R["jtv"], TOL, what + " J^T v")
    for a, b in zip(G["bounds"], R["bounds"]):
        assert np.array_equal(a, b), what + " bounds"
    for a, b in zip(G["load_adj"], R["load_adj"]):
        assert np.array_equal(a, b), what + " load adjoint"
    if "kkt" in R:
        assert np.array_equal(G["kkt_idx"][0], R["kkt_idx"][0]), what + " K rowptr"
        assert np.array_equal(G["kkt_idx"][1].astype(np.int64), R["kkt_idx"][1]), what + " K colind"
        assert_close(G["kkt"], *R["kkt"], TOL_KKT, what + " K")
