"""The one-launch sweep (per-XCD queues of line, generator and bus tiles in
one persistent kernel) against the two-launch sweep on the same inputs:
bitwise equal outputs (the same per-element code, no atomics on values),
status bits clear, repeated launches and graph replays included."""
import os

import numpy as np
import pytest

from paper_2405_14032_amd import synth

import pins

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="the one-launch sweep is switched off: its runs on the smallest grid did not "
                                      "finish and the cause is not established")]

KEYS = ("f", "grad", "c", "jvals", "hvals", "jtv", "kvals")


def _model(capi, nets, split):
    old = os.environ.get("OPF_SWEEP_SPLIT")
    os.environ["OPF_SWEEP_SPLIT"] = "1" if split else "0"
    try:
        return capi.Model(nets, device=0)
    finally:
        if old is None:
            del os.environ["OPF_SWEEP_SPLIT"]
        else:
            os.environ["OPF_SWEEP_SPLIT"] = old


def _run(torch, dev, M, inp, graph=False, reps=1):
    e = lambda k: torch.full((k,), float("nan"), dtype=torch.float64, device=dev)
    out = dict(f=e(M.ninst), grad=e(M.n), c=e(M.m), jvals=e(M.nnz_jac), hvals=e(M.nnz_hess), jtv=e(M.n),
               kvals=e(M.nnz_kkt))
    M.use_current_torch_stream()
    args = M.sweep_args(**inp, **out)
    for _ in range(reps):
        (M.sweep_graph if graph else M.sweep)(args)
    torch.cuda.synchronize()
    return {k: out[k].cpu().numpy() for k in KEYS}


CASES = {
    "tiny": lambda: [synth.config_network("tiny")],
    "ragged": lambda: [synth.make_network(301, 517, 63, 7, 41)],
    "hub": lambda: [pins.hub_network(40)],
    "mid": lambda: [synth.config_network("mid")],
    "batched": lambda: [synth.make_network(150, 210, 30, 6, 111), synth.make_network(64, 90, 13, 13, 112),
                        pins.manual_network(4, [0, 0, 1, 1, 2], [1, 1, 0, 2, 3], [0.01] * 5,
                                            [0.1, 0.2, 0.15, 0.1, 0.3], [0.02] * 5, [1, 1, 3], T=3,
                                            pd=np.full((3, 4), 0.2))],
    "week": lambda: [synth.make_network(2000, 3200, 400, 168, 2)],
}


@pytest.mark.parametrize("which", list(CASES))
def test_one_launch_sweep_bitwise_equals_two_launch(which):
    import torch
    from paper_2405_14032_amd import capi
    dev = torch.device("cuda:0")
    nets = CASES[which]()
    print(f"one-launch sweep vs two launches: {which}", flush=True)
    pts = [synth.make_point(n, 700 + k) for k, n in enumerate(nets)]
    cat = lambda key: np.concatenate([getattr(p, key) for p in pts])
    MF, MS = _model(capi, nets, split=False), _model(capi, nets, split=True)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    v = np.random.default_rng(9).standard_normal(MF.m)
    inp = dict(x=t(cat("x")), lam=t(cat("lam")), sigma=0.37, v=t(v), diag_x=t(cat("diag_x")), dcon=t(cat("dcon")))
    ref = _run(torch, dev, MS, inp)
    for graph, reps in ((False, 1), (False, 3), (True, 3)):
        got = _run(torch, dev, MF, inp, graph=graph, reps=reps)
        for k in KEYS:
            assert not np.isnan(ref[k]).any(), f"{which} {k}: two-launch sweep left values unwritten"
            assert np.array_equal(got[k], ref[k]), f"{which} {k}: one-launch sweep differs (graph={graph})"
        assert MF.sweep_check() == 0, f"{which}: one-launch sweep status bits raised"
    MF.close()
    MS.close()
