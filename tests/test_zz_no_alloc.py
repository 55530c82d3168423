"""The allocation-free sweep (opf_sweep_noalloc, scratch in the library's
static device array) against opf_sweep (scratch in the model's buffers),
through the C ABI: two calls in a row, the second on a smaller model, each
bitwise equal to the plain sweep on the same inputs (both run the same
kernels, which use no atomics), plus the rejection of a model whose scratch
exceeds the static array."""
import numpy as np
import pytest

from paper_2405_14032_amd import synth

pytestmark = pytest.mark.gpu

FULL = ("f", "grad", "c", "jvals", "hvals", "jtv", "kvals")
PARTIAL = ("f", "c", "jtv")  # objective partials and the separate J^T v kernels


def _buffers(torch, dev, M, keys):
    size = dict(f=M.ninst, grad=M.n, c=M.m, jvals=M.nnz_jac, hvals=M.nnz_hess, jtv=M.n, kvals=M.nnz_kkt)
    return {k: torch.full((size[k],), float("nan"), dtype=torch.float64, device=dev) for k in keys}


def _inputs(torch, dev, M, net, seed):
    pt = synth.make_point(net, seed)
    v = np.random.default_rng(seed + 1).standard_normal(M.m)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    return dict(x=t(pt.x), lam=t(pt.lam), sigma=0.37, v=t(v), diag_x=t(pt.diag_x), dcon=t(pt.dcon))


def _both(torch, dev, M, inp, keys):
    ref, got = _buffers(torch, dev, M, keys), _buffers(torch, dev, M, keys)
    M.use_current_torch_stream()
    M.sweep(M.sweep_args(**inp, **ref))
    torch.cuda.synchronize()
    M.sweep_noalloc(M.sweep_args(**inp, **got))
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_sweep_equals_sweep_two_calls():
    import torch
    from paper_2405_14032_amd import capi
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    cases = [("mid", synth.config_network("mid"), 801), ("tiny", synth.config_network("tiny"), 802)]
    models = []
    for name, net, seed in cases:
        print(f"noalloc sweep: {name} N={net.N} B={net.B} T={net.T}", flush=True)
        M = capi.Model([net], device=0)
        models.append(M)
        inp = _inputs(torch, dev, M, net, seed)
        for keys in (FULL, PARTIAL):
            ref, got = _both(torch, dev, M, inp, keys)
            for k in keys:
                r, g = ref[k].cpu().numpy(), got[k].cpu().numpy()
                assert not np.isnan(r).any(), f"{name} {k}: plain sweep left values unwritten"
                assert np.array_equal(r, g), f"{name} {k}: noalloc sweep differs from opf_sweep"
    for M in models:
        M.close()


def test_noalloc_sweep_rejects_models_beyond_static_scratch():
    import torch
    from paper_2405_14032_amd import capi
    dev = torch.device("cuda:0")
    # 22 doubles per line-period: 3200 lines x 64 periods need 36 MB > 32 MiB
    net = synth.make_network(2000, 3200, 400, 64, 803)
    print("noalloc sweep: rejection at N=2000 B=3200 T=64", flush=True)
    M = capi.Model([net], device=0)
    inp = _inputs(torch, dev, M, net, 804)
    out = _buffers(torch, dev, M, FULL)
    with pytest.raises(capi.OpfError) as ei:
        M.sweep_noalloc(M.sweep_args(**inp, **out))
    assert ei.value.code == capi.OPF_ERANGE
    assert "static buffer" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.isnan(out["kvals"]).all(), "a rejected call must enqueue nothing"
    M.close()


def test_noalloc_sweep_under_graph_capture():
    """The call the entry point is for: recorded into a HIP graph (torch's
    capture on a side stream, which refuses allocations during capture) and
    replayed three times with eager work in between (every output refilled
    with NaN first); each replay equals the plain sweep bitwise."""
    import torch
    from paper_2405_14032_amd import capi
    dev = torch.device("cuda:0")
    net = synth.make_network(300, 450, 60, 5, 805)
    print("noalloc sweep under graph capture: N=300 B=450 T=5", flush=True)
    M = capi.Model([net], device=0)
    inp = _inputs(torch, dev, M, net, 806)
    ref = _buffers(torch, dev, M, FULL)
    M.use_current_torch_stream()
    M.sweep(M.sweep_args(**inp, **ref))
    torch.cuda.synchronize()
    out = _buffers(torch, dev, M, FULL)
    args = M.sweep_args(**inp, **out)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        M.use_current_torch_stream()
        M.sweep_noalloc(args)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        M.use_current_torch_stream()
        M.sweep_noalloc(args)
    M.use_current_torch_stream()
    for rep in range(3):
        for k in FULL:
            out[k].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in FULL:
            assert torch.equal(out[k], ref[k]), f"replay {rep}: {k} differs from opf_sweep"
    del g
    M.close()
