"""Pins of the oracle's cancellation scales (the ``mag`` outputs every
parity bound uses) and of its bounds, on the CPU.

The scales are compared with an independent term-by-term enumeration
(``pins_mag``): complex monomials of the pi-model power differentiated
generically, plain summands elsewhere, the condensed matrix accumulated
over the pairs of each Jacobian row, the lifted-KKT formulas of Sec. III-B
evaluated in magnitude-carrying scalar arithmetic.  A planted inflation of
a scale is caught; every scale covers its value; single-term entries have
scale equal to their absolute value.

The bounds are pinned by the feasible sets they define: a point satisfies
a row's bounds exactly when it satisfies the paper's inequality (eq. (1f)
thermal limit sqrt(p^2 + q^2) <= S, (1g)-(1i) boxes, (1j) angle
difference, (1k) ramp), tested on random and boundary points.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import opf_oracle as O
from paper_2405_14032_amd import synth
import pins
import pins_mag as PM

RT = 1e-12  # summation-order rounding between two enumerations of the same terms


def _case(name):
    if name == "tiny":
        return pins.tiny_case()
    if name == "tiny-stress":
        return pins.tiny_case(stress=True)
    if name == "hub":
        net = pins.hub_network()
        return net, synth.make_point(net, 9)
    raise ValueError(name)


def _oracle_all(net, pt):
    L = O.Layout(net)
    c, cm = O.constraints(net, pt.x, with_mag=True)
    jr, jc, jv, jm = O.jacobian(net, pt.x, with_mag=True)
    hr, hc, hv, hm = O.hessian(net, pt.x, pt.lam, pt.sigma, with_mag=True)
    jtv, jtm = O.jtprod(net, pt.x, pt.lam, with_mag=True)
    rp, ci, kv, km = O.condensed(L.n, (jr, jc, jv), (hr, hc, hv), pt.diag_x, pt.dcon, jac_mag=jm, hess_mag=hm)
    return dict(L=L, c=(c, cm), J=(jr, jc, jv, jm), H=(hr, hc, hv, hm), jtv=(jtv, jtm), K=(rp, ci, kv, km),
                f=(O.objective(net, pt.x), O.objective_mag(net, pt.x)),
                grad=(O.gradient(net, pt.x), O.gradient_mag(net, pt.x)))


def mag_mismatch(net, pt):
    """Largest relative difference between the oracle's values / scales and
    the brute-force enumeration over c, f, grad, J, H, J^T v and K (0 when
    they agree to rounding; inf on a pattern mismatch)."""
    o = _oracle_all(net, pt)
    bf = PM.model_terms(net, pt.x, pt.lam, pt.sigma)
    worst = 0.0

    def rel(a, b, scale):
        a, b, scale = (np.asarray(v, dtype=np.float64) for v in (a, b, scale))
        return float(np.max(np.abs(a - b) / np.maximum(scale, 1e-300), initial=0.0))

    # constraints, objective, gradient
    worst = max(worst, rel(o["c"][0], bf["c"][0], bf["c"][1]), rel(o["c"][1], bf["c"][1], bf["c"][1]))
    worst = max(worst, rel(o["f"][0], bf["f"][0], bf["f"][1]), rel(o["f"][1], bf["f"][1], bf["f"][1]))
    worst = max(worst, rel(o["grad"][0], bf["grad"][0], np.maximum(bf["grad"][1], 1.0)),
                rel(o["grad"][1], bf["grad"][1], np.maximum(bf["grad"][1], 1.0)))
    # Jacobian: unique (row, col) entries
    jr, jc, jv, jm = o["J"]
    if len(jr) != len(bf["J"]):
        return math.inf
    for r, cc, v, mg in zip(jr, jc, jv, jm):
        e = bf["J"].get((int(r), int(cc)))
        if e is None:
            return math.inf
        worst = max(worst, abs(v - e[0]) / e[1], abs(mg - e[1]) / e[1])
    # Hessian: summed over duplicates
    hr, hc, hv, hm = o["H"]
    agg = {}
    for r, cc, v, mg in zip(hr, hc, hv, hm):
        a = agg.setdefault((int(r), int(cc)), [0.0, 0.0])
        a[0] += v
        a[1] += mg
    if set(agg) != set(bf["H"]):
        return math.inf
    for key, (v, mg) in agg.items():
        e = bf["H"][key]
        sc = max(e[1], 1e-300)
        worst = max(worst, abs(v - e[0]) / sc, abs(mg - e[1]) / sc)
    # J^T v from the brute-force Jacobian
    L = o["L"]
    jt, jtm = PM.jt_terms(bf["J"], pt.lam, L.n)
    worst = max(worst, rel(o["jtv"][0], jt, np.maximum(jtm, 1e-300)), rel(o["jtv"][1], jtm, np.maximum(jtm, 1e-300)))
    # K slot by slot
    rp, ci, kv, km = o["K"]
    K = PM.kkt_terms(bf["J"], bf["H"], pt.diag_x, pt.dcon, L.n)
    if len(ci) != len(K):
        return math.inf
    rows = np.repeat(np.arange(L.n), np.diff(rp))
    for r, cc, v, mg in zip(rows, ci, kv, km):
        e = K.get((int(r), int(cc)))
        if e is None:
            return math.inf
        sc = max(e[1], 1e-300)
        worst = max(worst, abs(v - e[0]) / sc, abs(mg - e[1]) / sc)
    return worst


@pytest.mark.parametrize("name", ["tiny", "tiny-stress", "hub"])
def test_scales_equal_brute_force_term_sums(name):
    net, pt = _case(name)
    assert mag_mismatch(net, pt) <= RT


@pytest.mark.parametrize("name", ["tiny", "hub"])
def test_scales_cover_values(name):
    net, pt = _case(name)
    o = _oracle_all(net, pt)
    slack = 1.0 + 1e-14
    for key in ("c", "jtv", "grad"):
        v, m = o[key]
        assert np.all(np.abs(v) <= m * slack), key
    assert abs(o["f"][0]) <= o["f"][1] * slack
    for key in ("J", "H"):
        v, m = o[key][2], o[key][3]
        assert np.all(np.abs(v) <= m * slack), key
    assert np.all(np.abs(o["K"][2]) <= o["K"][3] * slack)


def test_single_term_entries_have_scale_equal_to_value():
    net, pt = _case("tiny")
    o = _oracle_all(net, pt)
    L = o["L"]
    jr, jc, jv, jm = o["J"]
    unit = np.abs(jv) == 1.0
    # every +-1 entry (generation, line ends, reference, own flow, angle, ramp)
    assert unit.sum() == net.T * (2 * net.G + 4 * net.B + 1 + 4 * net.B + 2 * net.B) + 2 * net.G * (net.T - 1)
    assert np.all(jm[unit] == 1.0)
    # thermal Jacobian entries 2 p: one term each
    th_rows = np.zeros(L.m, dtype=bool)
    for t in range(net.T):
        th_rows[t * L.m_p + L.thf:t * L.m_p + L.ang] = True
    sel = th_rows[jr]
    assert np.all(jm[sel] == np.abs(jv[sel]))
    # thermal and objective Hessian entries: one term each
    hr, hc, hv, hm = o["H"]
    X = np.arange(L.n) % L.n_p
    single = (X[hr] >= L.flow[0]) | ((X[hr] >= L.pg) & (X[hr] < L.pg + net.G))
    single &= hr == hc
    flows_diag = (X[hr] >= L.flow[0]) & (hr == hc)
    assert flows_diag.sum() == 4 * net.B * net.T
    assert np.all(hm[single] == np.abs(hv[single]))
    # squared thermal rows and the reference row: scale equals the value
    c, cm = o["c"]
    C, M = c[:net.T * L.m_p].reshape(net.T, L.m_p), cm[:net.T * L.m_p].reshape(net.T, L.m_p)
    assert np.array_equal(C[:, L.thf:L.ang], M[:, L.thf:L.ang])
    assert np.array_equal(np.abs(C[:, L.ref]), M[:, L.ref])


def _lifted_case(seed=5):
    net, st = pins.ipm_case(seed=seed)
    c = O.constraints(net, st.x)
    grad = O.gradient(net, st.x)
    dx = np.random.default_rng(100 + seed).standard_normal(st.x.size)
    return net, st, c, grad, dx


@pytest.mark.parametrize("seed", [5, 6])
def test_lifted_scales_equal_brute_force(seed):
    net, st, c, grad, dx = _lifted_case(seed)
    _, _, rhs, rhs_m = O.condensed_rhs(net, st, grad, c, with_mag=True)
    steps, step_m = O.recover_step(net, st, c, dx, with_mag=True)
    J = PM.model_terms(net, st.x, np.zeros(len(st.s)), 1.0)["J"]
    bf = PM.lifted_terms(net, st, grad, c, J, dx)
    bv, bm = PM.split(bf["rhs"])
    assert np.all(np.abs(rhs - bv) <= RT * bm)
    assert np.all(np.abs(rhs_m - bm) <= RT * bm)
    for name, v, m in zip(("ds", "dy", "dzl", "dzu", "dvl", "dvu"), steps, step_m):
        bv, bm = PM.split(bf[name])
        assert np.all(np.abs(v - bv) <= RT * np.maximum(bm, 1e-300)), name
        assert np.all(np.abs(m - bm) <= RT * np.maximum(bm, 1e-300)), name
        assert np.all(np.abs(v) <= m * (1.0 + 1e-14)), name


# ------------------------------------------------------------------ planted
def test_planted_inflated_admittance_scale(monkeypatch):
    # a units slip in the self-admittance magnitude (x1e3) of the oracle's
    # derivative scales: values unchanged, every J / H / K bound looser
    orig = O._end_terms

    def bad(net, vm, va):
        out = list(orig(net, vm, va))
        m = list(out[6])
        m[0] = m[0] * 1e3
        out[6] = tuple(m)
        return tuple(out)

    monkeypatch.setattr(O, "_end_terms", bad)
    net, pt = _case("tiny")
    assert mag_mismatch(net, pt) > 1.0


def test_planted_inflated_single_scale(monkeypatch):
    # one Jacobian scale multiplied by 1e3
    orig = O.jacobian

    def bad(net, x, with_mag=False):
        out = orig(net, x, with_mag=with_mag)
        if with_mag:
            out[3][37] *= 1e3
        return out

    monkeypatch.setattr(O, "jacobian", bad)
    net, pt = _case("tiny")
    assert mag_mismatch(net, pt) > 1.0


def test_planted_inflated_lifted_scale(monkeypatch):
    orig = O._row_terms_mag

    def bad(st, c, R):
        qs_m, py_m, plo_m, phi_m = orig(st, c, R)
        return qs_m * 1e3, py_m, plo_m, phi_m

    monkeypatch.setattr(O, "_row_terms_mag", bad)
    net, st, c, grad, dx = _lifted_case()
    _, _, rhs, rhs_m = O.condensed_rhs(net, st, grad, c, with_mag=True)
    J = PM.model_terms(net, st.x, np.zeros(len(st.s)), 1.0)["J"]
    _, bm = PM.split(PM.lifted_terms(net, st, grad, c, J)["rhs"])
    assert np.max(np.abs(rhs_m - bm) / bm) > 1.0


# ------------------------------------------------------------------ bounds
def _rows(net):
    L = PM.Lay(net)
    lv, uv, lc, uc = O.bounds(net)
    return L, lv, uv, lc, uc


def _inside(v, lo, hi):
    return (v >= lo) & (v <= hi)


def test_bounds_define_the_thermal_limit():
    # eq. (1f): sqrt(p^2 + q^2) <= S at both ends.  For random flows and
    # flows placed just inside and just outside the circle of radius S, the
    # row value c = p^2 + q^2 lies within [lc, uc] exactly when the paper's
    # inequality holds.
    net, pt = pins.tiny_case()
    L, lv, uv, lc, uc = _rows(net)
    rng = np.random.default_rng(3)
    for trial in range(4):
        X = pt.x.copy()
        for t in range(net.T):
            for l in range(net.B):
                for e in range(2):
                    ang = rng.uniform(-math.pi, math.pi)
                    rad = net.rate[l] * (rng.uniform(0.2, 1.8) if trial == 0 else
                                         (1.0 - 1e-9, 1.0 + 1e-9, 0.5)[trial - 1])
                    X[L.flow(t, 2 * e, l)] = rad * math.cos(ang)
                    X[L.flow(t, 2 * e + 1, l)] = rad * math.sin(ang)
        c = O.constraints(net, X)
        for t in range(net.T):
            for l in range(net.B):
                for e in range(2):
                    r = L.th(t, e, l)
                    p, q = X[L.flow(t, 2 * e, l)], X[L.flow(t, 2 * e + 1, l)]
                    assert bool(_inside(c[r], lc[r], uc[r])) == (math.hypot(p, q) <= net.rate[l])


def test_bounds_define_boxes_angles_and_ramps():
    # eq. (1g)-(1i): vmin <= vm <= vmax, pmin <= pg <= pmax, qmin <= qg <= qmax,
    # no bound on angles and flows; eq. (1j): angmin <= va_i - va_j <= angmax;
    # eq. (1k): |pg_t - pg_{t-1}| <= ramp for t >= 1; balance, flow and
    # reference rows are equalities
    net, _ = pins.tiny_case()
    L, lv, uv, lc, uc = _rows(net)
    for t in range(net.T):
        for i in range(net.N):
            assert (lv[L.vm(t, i)], uv[L.vm(t, i)]) == (net.vmin[i], net.vmax[i])
            assert lv[L.va(t, i)] == -np.inf and uv[L.va(t, i)] == np.inf
            for q in range(2):
                assert lc[L.bal(t, q, i)] == 0.0 and uc[L.bal(t, q, i)] == 0.0
        for g in range(net.G):
            assert (lv[L.pg(t, g)], uv[L.pg(t, g)]) == (net.pmin[g], net.pmax[g])
            assert (lv[L.qg(t, g)], uv[L.qg(t, g)]) == (net.qmin[g], net.qmax[g])
        assert lc[L.ref(t)] == 0.0 and uc[L.ref(t)] == 0.0
        for l in range(net.B):
            for k in range(4):
                assert lv[L.flow(t, k, l)] == -np.inf and uv[L.flow(t, k, l)] == np.inf
                assert lc[L.cflow(t, k, l)] == 0.0 and uc[L.cflow(t, k, l)] == 0.0
            assert lc[L.th(t, 0, l)] == -np.inf and lc[L.th(t, 1, l)] == -np.inf
    # angle and ramp rows by their feasible sets at random and boundary points
    rng = np.random.default_rng(4)
    x = synth.make_point(net, 1).x.copy()
    for trial in range(3):
        X = x.copy()
        for t in range(net.T):
            X[L.va(t, 0):L.va(t, 0) + net.N] = rng.uniform(-1.0, 1.0, net.N)
            for g in range(net.G):
                if t >= 1:
                    step = net.ramp[g] * (rng.uniform(-2, 2) if trial == 0 else (1 - 1e-9, 1 + 1e-9)[trial - 1]
                                          * rng.choice([-1.0, 1.0]))
                    X[L.pg(t, g)] = X[L.pg(t - 1, g)] + step
        c = O.constraints(net, X)
        for t in range(net.T):
            for l in range(net.B):
                d = X[L.va(t, net.f_bus[l])] - X[L.va(t, net.t_bus[l])]
                r = L.ang(t, l)
                assert bool(_inside(c[r], lc[r], uc[r])) == (net.angmin[l] <= d <= net.angmax[l])
            if t >= 1:
                for g in range(net.G):
                    r = L.ramp(t, g)
                    d = X[L.pg(t, g)] - X[L.pg(t - 1, g)]
                    assert bool(_inside(c[r], lc[r], uc[r])) == (abs(d) <= net.ramp[g])
