"""The C ABI on the host: symbols, validation, error paths, host-only models
and the symbolic condensed-matrix pattern against the oracle (no GPU)."""
import ctypes as C
import os

import numpy as np
import pytest

from oracle import opf_oracle as O
from paper_2405_14032_amd import synth

import pins

capi = pytest.importorskip("paper_2405_14032_amd.capi")


def test_library_exports_every_header_symbol():
    names = capi.header_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(capi.lib, name), name


def _one(net):
    descs, keep = capi.make_descs([net])
    return descs, keep


def test_validate_accepts_synthetic_configs():
    for name in ("tiny", "mid"):
        assert capi.validate([synth.config_network(name)]) == capi.OPF_OK


@pytest.mark.parametrize("mutation,code", [
    ("bad_bus", capi.OPF_EINVAL),
    ("self_loop", capi.OPF_EINVAL),
    ("no_bus", capi.OPF_EINVAL),
    ("no_period", capi.OPF_EINVAL),
    ("bad_gen_bus", capi.OPF_EINVAL),
    ("bad_ref", capi.OPF_EINVAL),
    ("zero_impedance", capi.OPF_EINVAL),
    ("null_array", capi.OPF_EINVAL),
    ("overflow", capi.OPF_ERANGE),
])
def test_validate_rejects(mutation, code):
    net = synth.config_network("tiny")
    descs, keep = _one(net)
    d = descs[0]
    if mutation == "bad_bus":
        arr = np.array(net.f_bus, dtype=np.int32)
        arr[3] = net.N
        keep.append(arr)
        d.f_bus = arr.ctypes.data_as(C.POINTER(C.c_int32))
    elif mutation == "self_loop":
        arr = np.array(net.t_bus, dtype=np.int32)
        arr[2] = net.f_bus[2]
        keep.append(arr)
        d.t_bus = arr.ctypes.data_as(C.POINTER(C.c_int32))
    elif mutation == "no_bus":
        d.nbus = 0
    elif mutation == "no_period":
        d.nperiod = 0
    elif mutation == "bad_gen_bus":
        arr = np.array(net.gen_bus, dtype=np.int32)
        arr[0] = -1
        keep.append(arr)
        d.gen_bus = arr.ctypes.data_as(C.POINTER(C.c_int32))
    elif mutation == "bad_ref":
        d.ref_bus = net.N
    elif mutation == "zero_impedance":
        r = np.array(net.r)
        x = np.array(net.x)
        r[1] = 0.0
        x[1] = 0.0
        keep += [r, x]
        d.r = r.ctypes.data_as(C.POINTER(C.c_double))
        d.x = x.ctypes.data_as(C.POINTER(C.c_double))
    elif mutation == "null_array":
        d.pd = None
    elif mutation == "overflow":
        d.nbus = 1 << 28
        d.nperiod = 1 << 10
    assert capi.opf_validate(descs, 1) == code
    assert len(capi.opf_last_error()) > 0
    h = C.c_void_p()
    assert capi.opf_model_create(descs, 1, -1, C.byref(h)) == code
    assert not h.value


def test_injected_allocation_failure(monkeypatch):
    net = synth.config_network("tiny")
    descs, keep = _one(net)
    monkeypatch.setenv("OPF_TEST_FAIL_ALLOC", "1")
    h = C.c_void_p()
    assert capi.opf_model_create(descs, 1, -1, C.byref(h)) == capi.OPF_ENOMEM
    assert b"injected" in capi.opf_last_error()


def test_host_only_model_dims_and_offsets():
    nets = [synth.config_network("tiny"), synth.make_network(30, 45, 7, 5, 99)]
    M = capi.Model(nets, device=-1)
    tot = {"n": 0, "m": 0, "nnz_jac": 0, "nnz_hess": 0}
    for k, net in enumerate(nets):
        d = O.dims(net.N, net.B, net.G, net.T)
        assert M.x_off[k] == tot["n"] and M.c_off[k] == tot["m"]
        assert M.j_off[k] == tot["nnz_jac"] and M.h_off[k] == tot["nnz_hess"]
        for key in tot:
            tot[key] += d[key]
    assert (M.n, M.m, M.nnz_jac, M.nnz_hess) == (tot["n"], tot["m"], tot["nnz_jac"], tot["nnz_hess"])
    assert M.nnz_kkt == sum(pins.nnz_kkt_closed_form(net) for net in nets)


def test_host_only_model_refuses_evaluation():
    M = capi.Model([synth.config_network("tiny")], device=-1)
    assert capi.opf_eval_jac(M.h, None, None) == capi.OPF_ENODEV
    assert capi.opf_eval_jac(None, None, None) == capi.OPF_EINVAL


def _oracle_pattern(net, seed=1):
    pt = synth.make_point(net, seed)
    L = O.Layout(net)
    rp, ci, _, _ = O.condensed(L.n, O.jacobian(net, pt.x), O.hessian(net, pt.x, pt.lam), pt.diag_x, pt.dcon)
    return rp, ci


@pytest.mark.parametrize("shape", [(14, 20, 5, 4, 1), (200, 300, 40, 3, 5), (60, 90, 12, 1, 6), (2, 1, 1, 2, 7)])
def test_host_kkt_pattern_matches_oracle(shape):
    N, B, G, T, seed = shape
    net = synth.make_network(N, B, G, T, seed)
    M = capi.Model([net], device=-1)
    rp, ci = M.kkt_structure_host()
    orp, oci = _oracle_pattern(net, seed)
    assert np.array_equal(rp, orp)
    assert np.array_equal(ci.astype(np.int64), oci)


def test_host_kkt_pattern_parallel_lines_and_shared_generator_bus():
    # two parallel lines (0-1), an anti-parallel one (1-0), two generators on
    # bus 1: the pattern merges them like the oracle's sort-and-reduce
    net = pins.manual_network(4, [0, 0, 1, 1, 2], [1, 1, 0, 2, 3], [0.01] * 5, [0.1, 0.2, 0.15, 0.1, 0.3],
                              [0.02] * 5, [1, 1, 3], T=3)
    M = capi.Model([net], device=-1)
    rp, ci = M.kkt_structure_host()
    orp, oci = _oracle_pattern(net)
    assert np.array_equal(rp, orp)
    assert np.array_equal(ci.astype(np.int64), oci)


def test_host_kkt_pattern_batched_concatenation():
    nets = [synth.make_network(20, 30, 4, 3, 11), synth.make_network(15, 22, 3, 5, 12)]
    M = capi.Model(nets, device=-1)
    rp, ci = M.kkt_structure_host()
    for k, net in enumerate(nets):
        orp, oci = _oracle_pattern(net)
        a, b = M.x_off[k], M.x_off[k + 1]
        assert np.array_equal(rp[a:b + 1] - M.k_off[k], orp)
        assert np.array_equal(ci[M.k_off[k]:M.k_off[k + 1]].astype(np.int64) - a, oci)


def test_host_kkt_pattern_isolated_bus():
    # a bus with no line has no (va, vm) pair: its va row is the diagonal only
    net = pins.manual_network(1, [], [], [], [], [], [0], T=3, pd=np.full((3, 1), 0.4))
    M = capi.Model([net], device=-1)
    rp, ci = M.kkt_structure_host()
    orp, oci = _oracle_pattern(net)
    assert np.array_equal(rp, orp)
    assert np.array_equal(ci.astype(np.int64), oci)


def _fake_state(**over):
    # non-NULL placeholder addresses: validation happens before any device work
    st = capi.opf_ipm_state()
    for name in ("x", "s", "y", "zl", "zu", "vl", "vu", "xl", "xu", "sl", "su"):
        setattr(st, name, 0x1000)
    st.mu, st.delta_w, st.delta_c = 0.1, 1e-4, 1e-6
    for k, v in over.items():
        setattr(st, k, v)
    return st


@pytest.mark.parametrize("over", [dict(y=None), dict(su=None), dict(mu=-1.0), dict(delta_w=float("nan")),
                                  dict(delta_c=-1e-9)])
def test_condensation_calls_validate_state(over):
    M = capi.Model([synth.config_network("tiny")], device=-1)
    st = _fake_state(**over)
    p = 0x1000
    assert capi.opf_condensed_rhs(M.h, C.byref(st), p, p, p, p, p) == capi.OPF_EINVAL
    assert len(capi.opf_last_error()) > 0
    assert capi.opf_recover_step(M.h, C.byref(st), p, p, p, p, p, p, p, p) == capi.OPF_EINVAL
    assert capi.opf_condensed_rhs(M.h, None, p, p, p, p, p) == capi.OPF_EINVAL


def test_condensation_calls_need_outputs_and_a_device():
    M = capi.Model([synth.config_network("tiny")], device=-1)
    st = _fake_state()
    p = 0x1000
    assert capi.opf_condensed_rhs(M.h, C.byref(st), p, p, None, p, p) == capi.OPF_EINVAL
    assert capi.opf_recover_step(M.h, C.byref(st), p, p, p, p, p, None, p, p) == capi.OPF_EINVAL
    assert capi.opf_condensed_rhs(None, C.byref(st), p, p, p, p, p) == capi.OPF_EINVAL
    # valid arguments on a host-only model: no device to run on
    assert capi.opf_condensed_rhs(M.h, C.byref(st), p, p, p, p, p) == capi.OPF_ENODEV
    assert capi.opf_recover_step(M.h, C.byref(st), p, p, p, p, p, p, p, p) == capi.OPF_ENODEV
    assert capi.opf_jprod(M.h, p, p, p) == capi.OPF_ENODEV


def test_host_kkt_pattern_hub():
    # a 41-line star with doubled, anti-parallel and leaf lines and five
    # generators on the hub
    net = pins.hub_network()
    M = capi.Model([net], device=-1)
    rp, ci = M.kkt_structure_host()
    orp, oci = _oracle_pattern(net, 62)
    assert np.array_equal(rp, orp) and np.array_equal(ci.astype(np.int64), oci)


def test_host_only_model_refuses_the_interior_point_loop():
    # the loop needs a device; the host-only model reports it before any
    # pointer is touched, and the analysis itself works without one
    net = synth.config_network("tiny")
    M = capi.Model([net], device=-1)
    F = capi.Chol(M)
    import torch
    x = torch.empty(M.n, dtype=torch.float64)
    with pytest.raises(ValueError, match="host-only"):
        capi.ipm_solve(M, F, x)
    r = capi.opf_ipm_result()
    assert capi.opf_ipm_solve(M.h, F.h, None, x.data_ptr(), None, C.byref(r)) == -5
    o = capi.ipm_options()
    assert o.tol == 1e-4 and o.max_iter == 100 and o.tau == 0.99995 and o.verbose == 0
    F.close()
    M.close()


def test_cap_load_scales_to_the_capacity_fraction():
    """synth.cap_load: the peak period's total real load becomes the given
    fraction of the generation capacity, real and reactive loads scale by
    the same factor, a network already below the cap is left unchanged, and
    nothing else in the network moves."""
    net = synth.config_network("mid")
    cap = synth.cap_load(net, 0.3)
    s = cap.pd.sum() / net.pd.sum()
    assert 0.0 < s < 1.0
    assert abs(cap.pd.sum(axis=1).max() - 0.3 * net.pmax.sum()) <= 1e-12 * net.pmax.sum()
    np.testing.assert_allclose(cap.pd, s * net.pd, rtol=1e-13, atol=0)
    np.testing.assert_allclose(cap.qd, s * net.qd, rtol=1e-13, atol=0)
    for k in ("rate", "pmax", "pmin", "qmax", "qmin", "ramp", "vmin", "vmax", "f_bus", "t_bus"):
        assert np.array_equal(getattr(cap, k), getattr(net, k)), k
    same = synth.cap_load(net, 10.0)
    assert np.array_equal(same.pd, net.pd) and np.array_equal(same.qd, net.qd)


@pytest.mark.parametrize("B,G,T", [(13_421_773, 1, 1), (24_403_000, 1, 2)])
def test_validate_rejects_blocks_beyond_32bit_byte_offsets(B, G, T):
    # one period's H block (G + 40 B doubles) or line scratch (22 B doubles)
    # beyond 2^29 doubles cannot be addressed by a 32-bit byte offset: the
    # descriptor is refused before any line array is read (the arrays here
    # are untouched zero pages)
    N = 4
    net = synth.make_network(N, 3, 1, 1, 3)
    descs, keep = _one(net)
    d = descs[0]
    d.nbranch, d.ngen, d.nperiod = B, G, T
    big_i = np.zeros(B, dtype=np.int32)
    big_d = np.zeros(B)
    keep += [big_i, big_d]
    for name in ("f_bus", "t_bus"):
        setattr(d, name, big_i.ctypes.data_as(C.POINTER(C.c_int32)))
    for name in ("r", "x", "b_charge", "rate", "angmin", "angmax", "tap", "shift"):
        setattr(d, name, big_d.ctypes.data_as(C.POINTER(C.c_double)))
    assert capi.opf_validate(descs, 1) == capi.OPF_ERANGE
    assert b"4 GiB" in capi.opf_last_error()


def test_validate_accepts_largest_addressable_lines():
    # G + 40 B just at 2^29 - 1 doubles passes the size checks (the first
    # line, a self loop of zero pages, is then what stops validation)
    B = ((1 << 29) - 1 - 1) // 40
    net = synth.make_network(4, 3, 1, 1, 3)
    descs, keep = _one(net)
    d = descs[0]
    d.nbranch = B
    big_i = np.zeros(B, dtype=np.int32)
    big_d = np.zeros(B)
    keep += [big_i, big_d]
    for name in ("f_bus", "t_bus"):
        setattr(d, name, big_i.ctypes.data_as(C.POINTER(C.c_int32)))
    for name in ("r", "x", "b_charge", "rate", "angmin", "angmax", "tap", "shift"):
        setattr(d, name, big_d.ctypes.data_as(C.POINTER(C.c_double)))
    assert capi.opf_validate(descs, 1) == capi.OPF_EINVAL
    assert b"f == t" in capi.opf_last_error()


def test_binding_rejects_wrong_tensors_before_the_abi():
    # the binding checks dtype, contiguity, length and device of every tensor
    # before a pointer reaches the C ABI
    torch = pytest.importorskip("torch")
    n = 10
    f64 = torch.zeros(n, dtype=torch.float64)
    with pytest.raises(TypeError, match="dtype"):
        capi._dev_arg(torch.zeros(n, dtype=torch.float32), 0, n, "f64", "x")
    with pytest.raises(TypeError, match="dtype"):
        capi._dev_arg(torch.zeros(n, dtype=torch.int64), 0, n, "i32", "rows")
    with pytest.raises(ValueError, match="contiguous"):
        capi._dev_arg(torch.zeros((n, 2), dtype=torch.float64)[:, 0], 0, n, "f64", "x")
    with pytest.raises(ValueError, match="need 11"):
        capi._dev_arg(f64, 0, n + 1, "f64", "x")
    with pytest.raises(ValueError, match="cuda:0"):
        capi._dev_arg(f64, 0, n, "f64", "x")
    with pytest.raises(ValueError, match="required"):
        capi._dev_arg(None, 0, n, "f64", "x")
    assert capi._dev_arg(None, 0, n, "f64", "x", optional=True) is None
    with pytest.raises(TypeError, match="torch tensor"):
        capi._dev_arg(np.zeros(n), 0, n, "f64", "x")
    # a host-only model refuses device calls in the binding too
    M = capi.Model([synth.config_network("tiny")], device=-1)
    with pytest.raises(ValueError, match="host-only"):
        M.eval_cons(torch.zeros(M.n, dtype=torch.float64), torch.zeros(M.m, dtype=torch.float64))
    with pytest.raises(ValueError, match="need"):
        M.eval_cons(torch.zeros(M.n - 1, dtype=torch.float64), torch.zeros(M.m, dtype=torch.float64))
    M.close()
