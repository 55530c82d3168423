"""HIP path against the oracle, element by element, through the C ABI."""
import numpy as np
import pytest

from oracle import opf_oracle as O
from paper_2405_14032_amd import synth

import gpu_common as GC
import pins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def _capi():
    from paper_2405_14032_amd import capi
    return capi


def _run_one(net, pt, torch_dev, graph=False, model=None):
    torch, dev = torch_dev
    capi = _capi()
    M = model or capi.Model([net], device=0)
    print(f"case N={net.N} B={net.B} G={net.G} T={net.T} graph={graph}", flush=True)
    G = GC.gpu_all(M, pt.x, pt.lam, pt.sigma, pt.lam, pt.diag_x, pt.dcon, torch, dev, graph=graph)
    return M, G


CASES = {
    "tiny": lambda: (synth.config_network("tiny"), 1, False),
    "tiny_stress": lambda: (synth.make_network(14, 20, 5, 4, 21), 21, True),
    "single_period": lambda: (synth.make_network(60, 90, 12, 1, 31), 31, False),
    "ragged": lambda: (synth.make_network(301, 517, 63, 7, 41), 41, True),
    "one_bus": lambda: (pins.manual_network(1, [], [], [], [], [], [0], T=3,
                                            pd=np.full((3, 1), 0.4)), 51, False),
    "two_bus": lambda: (pins.manual_network(2, [1], [0], [0.02], [0.2], [0.05], [1], T=2,
                                            pd=np.array([[0.3, 0.1], [0.35, 0.15]])), 52, False),
    "parallel": lambda: (pins.manual_network(4, [0, 0, 1, 1, 2], [1, 1, 0, 2, 3], [0.01] * 5,
                                             [0.1, 0.2, 0.15, 0.1, 0.3], [0.02] * 5, [1, 1, 3], T=3,
                                             pd=np.full((3, 4), 0.2)), 53, True),
}


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("nbus", [40, 120])
def test_parity_hub(nbus, graph, torch_dev):
    # with 120 buses the hub's K flow rows of one 256-line tile exceed the
    # on-chip budget, so the model falls back to narrower tiles
    net = pins.hub_network(nbus)
    pt = synth.make_point(net, 62, stress=True)
    M, G = _run_one(net, pt, torch_dev, graph=graph)
    R = GC.oracle_all(net, pt)
    GC.compare(G, R, f"hub{nbus} graph={graph}")


@pytest.mark.parametrize("name", list(CASES))
def test_parity_small(name, torch_dev):
    net, seed, stress = CASES[name]()
    pt = synth.make_point(net, seed, stress=stress)
    M, G = _run_one(net, pt, torch_dev)
    R = GC.oracle_all(net, pt)
    GC.compare(G, R, name)


def test_parity_mid(torch_dev):
    net = synth.config_network("mid")
    pt = synth.make_point(net, 2)
    M, G = _run_one(net, pt, torch_dev)
    R = GC.oracle_all(net, pt)
    GC.compare(G, R, "mid")


def test_parity_sigma_and_null_diag(torch_dev):
    torch, dev = torch_dev
    capi = _capi()
    net = synth.make_network(40, 60, 8, 3, 61)
    pt = synth.make_point(net, 61)
    pt.sigma = 0.37
    M = capi.Model([net], device=0)
    M.use_current_torch_stream()
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    X, LAM, D = t(pt.x), t(pt.lam), t(pt.dcon)
    jv = torch.empty(M.nnz_jac, dtype=torch.float64, device=dev)
    hv = torch.empty(M.nnz_hess, dtype=torch.float64, device=dev)
    kv = torch.empty(M.nnz_kkt, dtype=torch.float64, device=dev)
    M.eval_jac(X, jv)
    M.eval_hess(X, LAM, pt.sigma, hv)
    M.assemble_condensed(hv, jv, None, D, kv)
    torch.cuda.synchronize()
    L = O.Layout(net)
    jr, jc, jval, jmag = O.jacobian(net, pt.x, with_mag=True)
    hess_r, hess_c, hess_v, hess_m = O.hessian(net, pt.x, pt.lam, pt.sigma, with_mag=True)
    GC.assert_close(hv.cpu().numpy(), hess_v, hess_m, GC.TOL, "H sigma=0.37")
    rp, ci, kval, kmag = O.condensed(L.n, (jr, jc, jval), (hess_r, hess_c, hess_v), None, pt.dcon, jac_mag=jmag,
                                     hess_mag=hess_m)
    GC.assert_close(kv.cpu().numpy(), kval, kmag, GC.TOL_KKT, "K without diag_x")


def test_batched_equals_per_instance(torch_dev):
    torch, dev = torch_dev
    capi = _capi()
    nets = [synth.make_network(50, 75, 10, 4, 71), synth.make_network(33, 47, 6, 9, 72),
            synth.make_network(80, 112, 16, 2, 73)]
    pts = [synth.make_point(n, 71 + k) for k, n in enumerate(nets)]
    MB = capi.Model(nets, device=0)
    cat = lambda key: np.concatenate([getattr(p, key) for p in pts])
    print("batched case: 3 instances", flush=True)
    GB = GC.gpu_all(MB, cat("x"), cat("lam"), 1.0, cat("lam"), cat("diag_x"), cat("dcon"), torch, dev)
    for k, (net, pt) in enumerate(zip(nets, pts)):
        _, G1 = _run_one(net, pt, torch_dev)
        xs, xe = MB.x_off[k], MB.x_off[k + 1]
        cs, ce = MB.c_off[k], MB.c_off[k + 1]
        js, je = MB.j_off[k], MB.j_off[k + 1]
        hs, he = MB.h_off[k], MB.h_off[k + 1]
        ks, ke = MB.k_off[k], MB.k_off[k + 1]
        # element values bit-identical to the single-instance run
        for key, a, b in (("grad", xs, xe), ("c", cs, ce), ("jac", js, je), ("hess", hs, he),
                          ("jtv", xs, xe), ("kkt", ks, ke)):
            assert np.array_equal(GB[key][a:b], G1[key]), key
        # indices equal after the instance offsets
        assert np.array_equal(GB["jac_idx"][0][js:je] - cs, G1["jac_idx"][0])
        assert np.array_equal(GB["jac_idx"][1][js:je] - xs, G1["jac_idx"][1])
        assert np.array_equal(GB["hess_idx"][0][hs:he] - xs, G1["hess_idx"][0])
        assert np.array_equal(GB["kkt_idx"][0][xs:xe + 1] - ks, G1["kkt_idx"][0])
        assert np.array_equal(GB["kkt_idx"][1][ks:ke] - xs, G1["kkt_idx"][1])
        # objective: reduction order differs by tile layout
        assert abs(GB["f"][k] - G1["f"][0]) <= 1e-12 * abs(G1["f"][0])


def test_bitwise_deterministic(torch_dev):
    net = synth.make_network(400, 600, 80, 6, 81)
    pt = synth.make_point(net, 81)
    M, G1 = _run_one(net, pt, torch_dev)
    _, G2 = _run_one(net, pt, torch_dev, model=M)
    for key in ("f", "grad", "c", "jac", "hess", "jtv", "kkt"):
        assert np.array_equal(G1[key], G2[key]), key


def test_graph_sweep_replays_match_eager(torch_dev):
    torch, dev = torch_dev
    capi = _capi()
    net = synth.make_network(300, 450, 60, 5, 91)
    pt = synth.make_point(net, 91)
    M = capi.Model([net], device=0)
    _, E = _run_one(net, pt, torch_dev, model=M)
    for rep in range(3):
        # eager work between replays, then a replay of the recorded sweep
        _, G = _run_one(net, pt, torch_dev, model=M, graph=True)
        for key in ("f", "grad", "c", "jac", "hess", "jtv", "kkt"):
            assert np.array_equal(G[key], E[key]), (rep, key)


def test_autotuned_shapes_keep_parity(torch_dev, tmp_path):
    net = synth.make_network(500, 800, 100, 12, 95)
    pt = synth.make_point(net, 95)
    capi = _capi()
    M = capi.Model([net], device=0)
    cache = str(tmp_path / "tune.json")
    M.autotune(cache)
    _, G = _run_one(net, pt, torch_dev, model=M)
    R = GC.oracle_all(net, pt)
    GC.compare(G, R, "autotuned")
    # the cache reproduces the same shapes in a fresh model
    M2 = capi.Model([net], device=0)
    M2.autotune(cache)
    _, G2 = _run_one(net, pt, torch_dev, model=M2)
    for key in ("f", "grad", "c", "jac", "hess", "jtv", "kkt"):
        assert np.array_equal(G[key], G2[key]), key


@pytest.mark.parametrize("which", ["mid", "batched"])
def test_fused_jhk_bitwise_equals_separate_calls(which, torch_dev):
    torch, dev = torch_dev
    capi = _capi()
    if which == "mid":
        nets = [synth.config_network("mid")]
    else:
        nets = [synth.make_network(120, 170, 24, 5, 101), synth.make_network(77, 108, 15, 11, 102)]
    pts = [synth.make_point(n, 200 + k) for k, n in enumerate(nets)]
    M = capi.Model(nets, device=0)
    M.use_current_torch_stream()
    cat = lambda key: np.concatenate([getattr(p, key) for p in pts])
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    X, LAM, DX, D = t(cat("x")), t(cat("lam")), t(cat("diag_x")), t(cat("dcon"))
    e = lambda k: torch.full((k,), float("nan"), dtype=torch.float64, device=dev)
    j1, h1, k1 = e(M.nnz_jac), e(M.nnz_hess), e(M.nnz_kkt)
    j2, h2, k2 = e(M.nnz_jac), e(M.nnz_hess), e(M.nnz_kkt)
    print(f"fused vs separate: {which}", flush=True)
    M.eval_jac(X, j1)
    M.eval_hess(X, LAM, 0.37, h1)
    M.assemble_condensed(h1, j1, DX, D, k1)
    M.eval_jhk(X, LAM, 0.37, DX, D, j2, h2, k2)
    torch.cuda.synchronize()
    assert torch.equal(j1, j2)
    assert torch.equal(h1, h2)
    assert torch.equal(k1, k2)
    # and against the oracle (first instance)
    net, pt = nets[0], pts[0]
    L = O.Layout(net)
    jr, jc, jval, jmag = O.jacobian(net, pt.x, with_mag=True)
    hr, hc, hval, hmag = O.hessian(net, pt.x, pt.lam, 0.37, with_mag=True)
    _, _, kv, km = O.condensed(L.n, (jr, jc, jval), (hr, hc, hval), pt.diag_x, pt.dcon, jac_mag=jmag,
                               hess_mag=hmag)
    GC.assert_close(k2[:M.k_off[1]].cpu().numpy(), kv, km, GC.TOL_KKT, "fused K")


@pytest.mark.parametrize("which", ["mid", "batched"])
def test_fused_sweep_equals_separate_calls(which, torch_dev):
    torch, dev = torch_dev
    capi = _capi()
    if which == "mid":
        nets = [synth.config_network("mid")]
    else:
        nets = [synth.make_network(150, 210, 30, 6, 111), synth.make_network(64, 90, 13, 13, 112),
                pins.manual_network(4, [0, 0, 1, 1, 2], [1, 1, 0, 2, 3], [0.01] * 5, [0.1, 0.2, 0.15, 0.1, 0.3],
                                    [0.02] * 5, [1, 1, 3], T=3, pd=np.full((3, 4), 0.2))]
    pts = [synth.make_point(n, 300 + k) for k, n in enumerate(nets)]
    M = capi.Model(nets, device=0)
    cat = lambda key: np.concatenate([getattr(p, key) for p in pts])
    print(f"fused sweep vs separate: {which}", flush=True)
    v = np.random.default_rng(7).standard_normal(M.m)  # J^T v with v != lambda
    E = GC.gpu_all(M, cat("x"), cat("lam"), 0.37, v, cat("diag_x"), cat("dcon"), torch, dev, graph=False)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    X, LAM, V, DX, D = t(cat("x")), t(cat("lam")), t(v), t(cat("diag_x")), t(cat("dcon"))
    e = lambda k: torch.full((k,), float("nan"), dtype=torch.float64, device=dev)
    out = dict(f=e(M.ninst), grad=e(M.n), c=e(M.m), jvals=e(M.nnz_jac), hvals=e(M.nnz_hess), jtv=e(M.n),
               kvals=e(M.nnz_kkt))
    M.use_current_torch_stream()
    M.sweep(M.sweep_args(x=X, lam=LAM, sigma=0.37, v=V, diag_x=DX, dcon=D, **out))
    torch.cuda.synchronize()
    for key, ek in (("grad", "grad"), ("c", "c"), ("jvals", "jac"), ("hvals", "hess"), ("jtv", "jtv"),
                    ("kvals", "kkt")):
        assert np.array_equal(out[key].cpu().numpy(), E[ek]), key
    # the objective is summed in the sweep's own tile order (its generator
    # tiles' partials), so it agrees with the objective call to rounding:
    # the same terms, a different order
    for k, (net, pt) in enumerate(zip(nets, pts)):
        GC.assert_close(out["f"][k:k + 1].cpu().numpy(), E["f"][k:k + 1],
                        np.array([O.objective_mag(net, pt.x)]), GC.TOL, f"[{k}] f")
    f1 = out["f"].clone()
    out["f"].fill_(float("nan"))
    M.sweep(M.sweep_args(x=X, lam=LAM, sigma=0.37, v=V, diag_x=DX, dcon=D, **out))
    torch.cuda.synchronize()
    assert torch.equal(out["f"], f1)
