"""Independent checks that pin the oracle to the mathematics.

Each ``check_*`` returns the worst violation it found (a non-negative
number); the tests assert it is below a threshold, and the planted-mistake
tests assert that a mutated oracle pushes it above.  None of these checks
re-types an oracle formula: they use finite differences, conservation laws,
homogeneity, textbook closed forms, dense brute force or the paper's
printed counts.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import opf_oracle as O
from paper_2405_14032_amd import synth


def tiny_case(seed=1, stress=False):
    net = synth.config_network("tiny") if seed == 1 else synth.make_network(14, 20, 5, 4, seed)
    pt = synth.make_point(net, seed, stress=stress)
    return net, pt


def manual_network(N, f_bus, t_bus, r, x, b, gen_bus, T=1, pd=None):
    """Small hand-built network (defaults for everything not given)."""
    B = len(f_bus)
    G = len(gen_bus)
    pd = np.zeros((T, N)) if pd is None else np.asarray(pd, dtype=float).reshape(T, N)
    return synth.Network(
        N=N, B=B, G=G, T=T, ref_bus=int(gen_bus[0]), vmin=np.full(N, 0.9), vmax=np.full(N, 1.1),
        f_bus=np.asarray(f_bus, np.int32), t_bus=np.asarray(t_bus, np.int32),
        r=np.asarray(r, float), x=np.asarray(x, float), b_charge=np.asarray(b, float),
        rate=np.full(B, 2.0), angmin=np.full(B, -math.pi / 6), angmax=np.full(B, math.pi / 6),
        tap=np.ones(B), shift=np.zeros(B), gen_bus=np.asarray(gen_bus, np.int32),
        c2=np.full(G, 0.05), c1=np.full(G, 20.0), c0=np.zeros(G), pmin=np.zeros(G),
        pmax=np.full(G, 3.0), qmin=np.full(G, -1.5), qmax=np.full(G, 1.5), ramp=np.full(G, 0.2),
        pd=pd, qd=0.3 * pd)


def hub_network(N=40):
    """A star: bus 7 joined to every other bus (one line reversed), two lines
    doubled (one of them anti-parallel), a few lines among the leaves, five
    generators on the hub, off-nominal taps and phase shifts: high-degree
    incidence loops, long K rows, several generators sharing balance rows."""
    hub = 7
    f, t = [], []
    for k in range(N):
        if k != hub:
            f.append(hub if k != 25 else k)
            t.append(k if k != 25 else hub)
    f += [hub, 20, 3, 11, 30]
    t += [3, hub, 4, 12, 31]
    B = len(f)
    rng = np.random.default_rng(61)
    net = manual_network(N, f, t, list(rng.uniform(0.005, 0.03, B)), list(rng.uniform(0.05, 0.3, B)),
                              list(rng.uniform(0.0, 0.08, B)), [hub, hub, 3, hub, 30, hub, hub], T=3,
                              pd=rng.uniform(0.0, 0.3, (3, N)))
    net.tap[:] = rng.uniform(0.95, 1.05, B)
    net.shift[:] = rng.uniform(-0.1, 0.1, B)
    return net


def dense_jac(net, x):
    L = O.Layout(net)
    r, c, v = O.jacobian(net, x)
    J = np.zeros((L.m, L.n))
    np.add.at(J, (r, c), v)
    return J


# ---------------------------------------------------------------- counts
def parse_count(s):
    s = s.strip()
    return int(s[:-1]), {"k": 1_000, "m": 1_000_000}[s[-1]]


def check_table2_counts(path):
    """Largest mismatch (in the table's rounding unit) between the closed-form
    n, m and Table II's printed nvars / ncons."""
    worst = 0
    for line in open(path):
        if not line.strip() or line.startswith("#"):
            continue
        name, N, B, G, T, nv, nc = line.split()
        d = O.dims(int(N), int(B), int(G), int(T))
        for got, printed in ((d["n"], nv), (d["m"], nc)):
            val, unit = parse_count(printed)
            worst = max(worst, abs(round(got / unit) - val))
    return worst


# ---------------------------------------------------------------- values
def check_flat_start(net):
    """At V = 1, theta = 0 with tap 1 / shift 0 the flows are the charging
    closed form: p = 0 at both ends, q = -b_c/2 at both ends.  The error is
    scaled by the series admittance magnitude, the size of the cancelling
    terms."""
    L = O.Layout(net)
    x = np.zeros(L.n)
    X = x.reshape(net.T, L.n_p)
    X[:, :net.N] = 1.0
    c = O.constraints(net, x)
    C = c[:net.T * L.m_p].reshape(net.T, L.m_p)
    worst = 0.0
    for k, expect in ((0, 0.0), (1, -0.5 * net.b_charge), (2, 0.0), (3, -0.5 * net.b_charge)):
        phi = -C[:, L.cflow[k]:L.cflow[k] + net.B]  # c = x_flow - phi, x_flow = 0
        yabs = 1.0 / np.hypot(net.r, net.x)
        worst = max(worst, float(np.max(np.abs(phi - expect) / (1 + yabs))))
    return worst


def check_lossless_line(seed=7):
    """Lossless, uncharged line (r = 0, b_c = 0): textbook
    p_f = V_i V_j sin(d)/x, q_f = (V_i^2 - V_i V_j cos d)/x, p_t = -p_f,
    q_t = (V_j^2 - V_i V_j cos d)/x."""
    rng = np.random.default_rng(seed)
    net = manual_network(3, [0, 1], [1, 2], [0.0, 0.0], [0.2, 0.35], [0.0, 0.0], [0], T=2)
    L = O.Layout(net)
    x = np.zeros(L.n)
    X = x.reshape(net.T, L.n_p)
    X[:, :3] = rng.uniform(0.9, 1.1, (2, 3))
    X[:, 3:6] = rng.uniform(-0.5, 0.5, (2, 3))
    vm, va = X[:, :3], X[:, 3:6]
    C = O.constraints(net, x)[:net.T * L.m_p].reshape(net.T, L.m_p)
    worst = 0.0
    for l in range(2):
        i, j, xl = net.f_bus[l], net.t_bus[l], net.x[l]
        d = va[:, i] - va[:, j]
        exp = [vm[:, i] * vm[:, j] * np.sin(d) / xl,
               (vm[:, i] ** 2 - vm[:, i] * vm[:, j] * np.cos(d)) / xl,
               -vm[:, i] * vm[:, j] * np.sin(d) / xl,
               (vm[:, j] ** 2 - vm[:, i] * vm[:, j] * np.cos(d)) / xl]
        for k in range(4):
            phi = -C[:, L.cflow[k] + l]
            worst = max(worst, float(np.max(np.abs(phi - exp[k]))))
    return worst


def check_conservation(net, pt):
    """Energy balance of a pi-model line with tau = 1: the power entering at
    both ends is the series loss plus the charging absorption:
    p_f + p_t = g |V_i - V_j|^2,
    q_f + q_t = -b |V_i - V_j|^2 - (b_c/2)(V_i^2 + V_j^2), y = g + jb."""
    L = O.Layout(net)
    X = pt.x.reshape(net.T, L.n_p)
    vm, va = X[:, :net.N], X[:, net.N:2 * net.N]
    C = O.constraints(net, pt.x)[:net.T * L.m_p].reshape(net.T, L.m_p)
    phi = [X[:, L.flow[k]:L.flow[k] + net.B] - C[:, L.cflow[k]:L.cflow[k] + net.B] for k in range(4)]
    g = net.r / (net.r ** 2 + net.x ** 2)
    b = -net.x / (net.r ** 2 + net.x ** 2)
    vi = vm[:, net.f_bus] * np.cos(va[:, net.f_bus]), vm[:, net.f_bus] * np.sin(va[:, net.f_bus])
    vj = vm[:, net.t_bus] * np.cos(va[:, net.t_bus]), vm[:, net.t_bus] * np.sin(va[:, net.t_bus])
    dv2 = (vi[0] - vj[0]) ** 2 + (vi[1] - vj[1]) ** 2
    ploss = g * dv2
    qloss = -b * dv2 - 0.5 * net.b_charge * (vm[:, net.f_bus] ** 2 + vm[:, net.t_bus] ** 2)
    e1 = np.abs(phi[0] + phi[2] - ploss) / (1 + np.abs(phi[0]))
    e2 = np.abs(phi[1] + phi[3] - qloss) / (1 + np.abs(phi[1]))
    return float(max(e1.max(), e2.max()))


def check_two_bus_balance():
    """Hand-worked 2-bus, 1-line, 1-generator case (lossless line x = 0.5,
    V = 1, theta_0 = pi/6, theta_1 = 0): p_f = sin(pi/6)/0.5 = 1,
    p_t = -1, q_f = q_t = (1 - cos(pi/6))/0.5.  With flows set to exactly
    those values, pg = 1.25, qg = 0.4 and loads pd = (0.25, 1.0),
    qd = (0.4 - q_f, -q_t): every balance row and every flow row is zero,
    the reference row and the angle row are pi/6, both thermal rows are
    1 + q_f^2."""
    qf = (1 - math.cos(math.pi / 6)) / 0.5
    pd = np.array([[0.25, 1.0]])
    net = manual_network(2, [0], [1], [0.0], [0.5], [0.0], [0], T=1, pd=pd)
    net.qd = np.array([[0.4 - qf, -qf]])
    L = O.Layout(net)
    x = np.zeros(L.n)
    x[0:2] = 1.0
    x[2] = math.pi / 6
    x[L.pg] = 1.25
    x[L.qg] = 0.4
    x[L.flow[0]] = 1.0
    x[L.flow[1]] = qf
    x[L.flow[2]] = -1.0
    x[L.flow[3]] = qf
    c = O.constraints(net, x)
    # rows: balP(2) balQ(2) ref cpf cqf cpt cqt thf tht ang
    expect = np.zeros(L.m)
    expect[L.ref] = math.pi / 6
    expect[L.thf] = 1.0 + qf ** 2
    expect[L.tht] = 1.0 + qf ** 2
    expect[L.ang] = math.pi / 6
    return float(np.max(np.abs(c - expect)))


def check_objective(net, pt):
    """Objective against a per-generator, per-period Python loop."""
    L = O.Layout(net)
    X = pt.x.reshape(net.T, L.n_p)
    tot = 0.0
    for t in range(net.T):
        for g in range(net.G):
            p = X[t, L.pg + g]
            tot += net.c2[g] * p * p + net.c1[g] * p + net.c0[g]
    return abs(O.objective(net, pt.x) - tot) / abs(tot)


def check_gradient_fd(net, pt, h=1e-6):
    """Gradient entries against central differences of the objective."""
    L = O.Layout(net)
    grad = O.gradient(net, pt.x)
    worst = 0.0
    for idx in list(range(L.pg, L.pg + net.G)) + [0, L.flow[0], L.n - 1]:
        xp, xm = pt.x.copy(), pt.x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (O.objective(net, xp) - O.objective(net, xm)) / (2 * h)
        worst = max(worst, abs(fd - grad[idx]) / (1 + abs(fd)))
    return worst


# ---------------------------------------------------------------- Jacobian
def check_jacobian_fd(net, pt, h=1e-6):
    """Dense central differences of c against the oracle's COO Jacobian."""
    L = O.Layout(net)
    J = dense_jac(net, pt.x)
    worst = 0.0
    for j in range(L.n):
        xp, xm = pt.x.copy(), pt.x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (O.constraints(net, xp) - O.constraints(net, xm)) / (2 * h)
        worst = max(worst, float(np.max(np.abs(fd - J[:, j]) / (1 + np.abs(fd)))))
    return worst


def check_jacobian_invariants(net, pt):
    """theta-translation: J[r, va_i] = -J[r, va_j] on flow rows; Euler
    (degree-2 homogeneity in V): vm_i dphi/dvm_i + vm_j dphi/dvm_j = 2 phi."""
    L = O.Layout(net)
    r, c, v = O.jacobian(net, pt.x)
    T, B = net.T, net.B
    per = v[:T * L.nnzj_p].reshape(T, L.nnzj_p)
    base = 2 * net.G + 4 * B + 1
    X = pt.x.reshape(T, L.n_p)
    vi = X[:, net.f_bus]
    vj = X[:, net.t_bus]
    C = O.constraints(net, pt.x)[:T * L.m_p].reshape(T, L.m_p)
    worst = 0.0
    for k in range(4):
        blk = lambda loc: per[:, base + (k * 5 + loc) * B: base + (k * 5 + loc + 1) * B]
        worst = max(worst, float(np.max(np.abs(blk(3) + blk(4)) / (1 + np.abs(blk(3))))))
        phi = X[:, L.flow[k]:L.flow[k] + B] - C[:, L.cflow[k]:L.cflow[k] + B]
        euler = -(vi * blk(1) + vj * blk(2))
        worst = max(worst, float(np.max(np.abs(euler - 2 * phi) / (1 + np.abs(phi)))))
    return worst


def check_dc_limit():
    """r = 0, b_c = 0 at flat start: d p_f / d theta_i = 1/x, so the flow
    row entries are J[cpf, va_i] = -1/x and J[cpf, va_j] = +1/x."""
    net = manual_network(3, [0, 2], [1, 1], [0.0, 0.0], [0.1, 0.25], [0.0, 0.0], [0], T=1)
    L = O.Layout(net)
    x = np.zeros(L.n)
    x[:3] = 1.0
    r, c, v = O.jacobian(net, x)
    J = {(int(a), int(b)): float(w) for a, b, w in zip(r, c, v)}
    worst = 0.0
    for l in range(2):
        row = L.cflow[0] + l
        i, j = net.f_bus[l], net.t_bus[l]
        worst = max(worst, abs(J[(row, L.va + i)] + 1 / net.x[l]) * net.x[l],
                    abs(J[(row, L.va + j)] - 1 / net.x[l]) * net.x[l])
    return worst


def check_jacobian_structure(net, pt):
    """Counts equal the closed forms, no duplicate (row, col), indices in range."""
    L = O.Layout(net)
    r, c, v = O.jacobian(net, pt.x)
    d = O.dims(net.N, net.B, net.G, net.T)
    bad = int(len(r) != d["nnz_jac"])
    key = r * L.n + c
    bad += int(len(np.unique(key)) != len(key))
    bad += int(r.min() < 0 or r.max() >= L.m or c.min() < 0 or c.max() >= L.n)
    return bad


# ---------------------------------------------------------------- Hessian
def check_hessian_fd(net, pt, h=1e-6):
    """Dense central differences of grad(sigma f + lam^T c) = sigma grad f +
    J^T lam against the oracle's Hessian COO (summed, symmetrised); also the
    symmetry of the finite-difference matrix itself."""
    L = O.Layout(net)
    H = O.hessian_dense(L.n, O.hessian(net, pt.x, pt.lam, pt.sigma))

    def grad_l(x):
        return pt.sigma * O.gradient(net, x) + O.jtprod(net, x, pt.lam)

    F = np.zeros((L.n, L.n))
    for j in range(L.n):
        xp, xm = pt.x.copy(), pt.x.copy()
        xp[j] += h
        xm[j] -= h
        F[:, j] = (grad_l(xp) - grad_l(xm)) / (2 * h)
    scale = 1 + np.abs(F)
    return float(max(np.max(np.abs(F - H) / scale), np.max(np.abs(F - F.T) / scale)))


def check_hessian_euler(net, pt):
    """Differentiated Euler relation on each flow function (degree 2 in V):
    vm_i phi_{vm_i vm_i} + vm_j phi_{vm_j vm_i} = dphi/dvm_i, and likewise
    for vm_j.  Hessians are taken with a unit multiplier on one flow row
    kind at a time (H = -Hess phi there)."""
    L = O.Layout(net)
    T, B = net.T, net.B
    X = pt.x.reshape(T, L.n_p)
    vi = X[:, net.f_bus]
    vj = X[:, net.t_bus]
    r, c, v = O.jacobian(net, pt.x)
    per = v[:T * L.nnzj_p].reshape(T, L.nnzj_p)
    base = 2 * net.G + 4 * B + 1
    worst = 0.0
    for k in range(4):
        lam = np.zeros(L.m)
        lam[:T * L.m_p].reshape(T, L.m_p)[:, L.cflow[k]:L.cflow[k] + B] = 1.0
        hr, hc, hv = O.hessian(net, pt.x, lam, 0.0)
        hp = hv.reshape(T, L.nnzh_p)
        pairs = O.PAIRS_FROM if k < 2 else O.PAIRS_TO
        d2 = {}
        for loc, ab in enumerate(pairs):
            d2[ab] = -hp[:, net.G + (k * 9 + loc) * B: net.G + (k * 9 + loc + 1) * B]
        zero = np.zeros((T, B))
        h00 = d2.get((0, 0), zero)
        h11 = d2.get((1, 1), zero)
        h10 = d2[(1, 0)]
        dphi_i = -per[:, base + (k * 5 + 1) * B: base + (k * 5 + 2) * B]
        dphi_j = -per[:, base + (k * 5 + 2) * B: base + (k * 5 + 3) * B]
        e1 = np.abs(vi * h00 + vj * h10 - dphi_i) / (1 + np.abs(dphi_i))
        e2 = np.abs(vi * h10 + vj * h11 - dphi_j) / (1 + np.abs(dphi_j))
        worst = max(worst, float(e1.max()), float(e2.max()))
    return worst


# ---------------------------------------------------------------- adjoints
def check_jtprod_directional(net, pt, ndir=4, h=1e-6):
    """<u, J^T lam> against the central difference of lam^T c along u."""
    rng = np.random.default_rng(3)
    L = O.Layout(net)
    jtl = O.jtprod(net, pt.x, pt.lam)
    worst = 0.0
    for _ in range(ndir):
        u = rng.standard_normal(L.n)
        fd = (pt.lam @ O.constraints(net, pt.x + h * u) - pt.lam @ O.constraints(net, pt.x - h * u)) / (2 * h)
        worst = max(worst, abs(fd - u @ jtl) / (1 + abs(fd)))
    return worst


def check_load_adjoint_fd(net, pt, h=1e-6):
    """d(lam^T c)/d pd[t, n] and d/d qd[t, n] by central differences."""
    gp, gq = O.load_adjoint(net, pt.lam)
    worst = 0.0
    for (t, n) in [(0, 0), (net.T - 1, net.N - 1), (net.T // 2, net.N // 2)]:
        for which, g in (("p", gp), ("q", gq)):
            pd, qd = net.pd.copy(), net.qd.copy()
            arr = pd if which == "p" else qd
            arr[t, n] += h
            cp = O.constraints(net, pt.x, pd, qd)
            arr[t, n] -= 2 * h
            cm = O.constraints(net, pt.x, pd, qd)
            fd = pt.lam @ ((cp - cm) / (2 * h))
            worst = max(worst, abs(fd - g[t, n]) / (1 + abs(fd)))
    return worst


# ---------------------------------------------------------------- condensed
def check_condensed_dense(net, pt):
    """Dense brute force H + diag + J^T D J (numpy dense products) against
    the oracle's sort-and-reduce CSR: values on the pattern, no dense nonzero
    outside it, diagonal present, rows sorted and lower."""
    L = O.Layout(net)
    jac = O.jacobian(net, pt.x)
    hess = O.hessian(net, pt.x, pt.lam, pt.sigma)
    rowptr, colind, vals, mag = O.condensed(L.n, jac, hess, pt.diag_x, pt.dcon)
    J = dense_jac(net, pt.x)
    H = O.hessian_dense(L.n, hess)
    K = np.tril(H + np.diag(pt.diag_x) + J.T @ (pt.dcon[:, None] * J))
    Kc = np.zeros_like(K)
    rows = np.repeat(np.arange(L.n), np.diff(rowptr))
    Kc[rows, colind] = vals
    worst = float(np.max(np.abs(K - Kc) / (1 + np.abs(K))))
    bad = 0
    for i in range(L.n):
        cs = colind[rowptr[i]:rowptr[i + 1]]
        bad += int(not np.all(np.diff(cs) > 0)) + int(cs[-1] != i) + int(np.any(cs > i))
    return worst + bad


def check_condensed_quadratic(net, pt, nvec=3):
    """u^T K_full u = u^T H u + sum diag_x u^2 + sum d (J u)^2 for random u,
    with K_full the symmetric matrix rebuilt from the lower CSR."""
    import scipy.sparse as sp
    L = O.Layout(net)
    jr, jc, jv = O.jacobian(net, pt.x)
    hess = O.hessian(net, pt.x, pt.lam, pt.sigma)
    rowptr, colind, vals, _ = O.condensed(L.n, (jr, jc, jv), hess, pt.diag_x, pt.dcon)
    K = sp.csr_matrix((vals, colind, rowptr), shape=(L.n, L.n))
    J = sp.coo_matrix((jv, (jr, jc)), shape=(L.m, L.n)).tocsr()
    Hl = sp.coo_matrix((hess[2], (hess[0], hess[1])), shape=(L.n, L.n)).tocsr()
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(nvec):
        u = rng.standard_normal(L.n)
        ku = K @ u + K.T @ u - K.diagonal() * u
        hu = Hl @ u + Hl.T @ u - Hl.diagonal() * u
        lhs = u @ ku
        ju = J @ u
        rhs = u @ hu + np.sum(pt.diag_x * u * u) + np.sum(pt.dcon * ju * ju)
        worst = max(worst, abs(lhs - rhs) / (abs(rhs) + 1e-300))
    return worst


def nnz_kkt_closed_form(net):
    """Independent count of the condensed pattern for a simple network (no
    parallel lines, at most one generator per bus): per period
    3N + 2G + 26B + sum_n k_n (k_n - 1), k_n = lines at n + generators at n,
    plus one ramp pair per generator and period t >= 1."""
    deg = np.bincount(net.f_bus, minlength=net.N) + np.bincount(net.t_bus, minlength=net.N)
    k = deg + np.bincount(net.gen_bus, minlength=net.N)
    per = 3 * net.N + 2 * net.G + 26 * net.B + int(np.sum(k * (k - 1)))
    return net.T * per + net.G * (net.T - 1)


# ---------------------------------------------------------------- lifted KKT
def ipm_case(N=6, B=8, G=2, T=3, seed=5):
    net = synth.make_network(N, B, G, T, seed)
    st = synth.make_ipm_state(*O.bounds(net), seed=seed)
    return net, st


def full_kkt_solution(net, st):
    """Dense solve of the full lifted KKT system of Sec. III-B (seven block
    rows: stationarity in x and s, the relaxed rows, four complementarity
    blocks), assembled block by block from its printed layout, with one
    multiplier per finite bound.  Returns (dx, ds, dy, dzl, dzu, dvl, dvu)
    with the bound steps scattered to full length (0 where absent)."""
    L = O.Layout(net)
    n, m = L.n, L.m
    x, s, y, mu, dw, dc = st.x, st.s, st.y, st.mu, st.delta_w, st.delta_c
    A = dense_jac(net, x)
    W = O.hessian_dense(n, O.hessian(net, x, -y, 1.0))  # W = Hess f - sum y_i Hess g_i
    c = O.constraints(net, x)
    grad = O.gradient(net, x)
    hl, hu, gl, gu = (np.isfinite(b) for b in (st.xl, st.xu, st.sl, st.su))
    Pl, Pu, Ql, Qu = np.eye(n)[hl], np.eye(n)[hu], np.eye(m)[gl], np.eye(m)[gu]
    sizes = [n, m, m, int(hl.sum()), int(hu.sum()), int(gl.sum()), int(gu.sum())]
    off = np.concatenate([[0], np.cumsum(sizes)])
    M = np.zeros((off[-1], off[-1]))

    def put(i, j, blk):
        M[off[i]:off[i + 1], off[j]:off[j + 1]] += blk

    zl, zu, vl, vu = st.zl[hl], st.zu[hu], st.vl[gl], st.vu[gu]
    put(0, 0, W + dw * np.eye(n))
    put(0, 2, A.T)
    put(0, 3, -Pl.T)
    put(0, 4, Pu.T)
    put(1, 1, dw * np.eye(m))
    put(1, 2, -np.eye(m))
    put(1, 5, -Ql.T)
    put(1, 6, Qu.T)
    put(2, 0, A)
    put(2, 1, -np.eye(m))
    put(2, 2, -dc * np.eye(m))
    put(3, 0, zl[:, None] * Pl)
    put(3, 3, np.diag(x[hl] - st.xl[hl]))
    put(4, 0, -zu[:, None] * Pu)
    put(4, 4, np.diag(st.xu[hu] - x[hu]))
    put(5, 1, vl[:, None] * Ql)
    put(5, 5, np.diag(s[gl] - st.sl[gl]))
    put(6, 1, -vu[:, None] * Qu)
    put(6, 6, np.diag(st.su[gu] - s[gu]))
    rhs = np.concatenate([
        grad - A.T @ y - Pl.T @ zl + Pu.T @ zu,
        -Ql.T @ vl + Qu.T @ vu + y,
        c - s,
        zl * (x[hl] - st.xl[hl]) - mu,
        zu * (st.xu[hu] - x[hu]) - mu,
        vl * (s[gl] - st.sl[gl]) - mu,
        vu * (st.su[gu] - s[gu]) - mu,
    ])
    sol = np.linalg.solve(M, rhs)
    blk = [sol[off[i]:off[i + 1]] for i in range(7)]
    out = blk[:3]
    for b, mask, size in ((blk[3], hl, n), (blk[4], hu, n), (blk[5], gl, m), (blk[6], gu, m)):
        full = np.zeros(size)
        full[mask] = b
        out.append(full)
    return out


def check_lifted_kkt(net, st):
    """Condense (oracle K with diag_x, D and the condensed right-hand side),
    solve the condensed system densely, recover the other steps, and compare
    every block with the full system's dense solution; returns the largest
    block error relative to that block's max norm."""
    L = O.Layout(net)
    c = O.constraints(net, st.x)
    grad = O.gradient(net, st.x)
    diag_x, dcon, rhs = O.condensed_rhs(net, st, grad, c)
    jac = O.jacobian(net, st.x)
    hess = O.hessian(net, st.x, -st.y, 1.0)
    rowptr, colind, vals, _ = O.condensed(L.n, jac, hess, diag_x, dcon)
    K = np.zeros((L.n, L.n))
    K[np.repeat(np.arange(L.n), np.diff(rowptr)), colind] = vals
    K = K + np.tril(K, -1).T
    dx = np.linalg.solve(K, rhs)
    mine = [dx] + list(O.recover_step(net, st, c, dx))
    ref = full_kkt_solution(net, st)
    return max(float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b))))) for a, b in zip(mine, ref))
