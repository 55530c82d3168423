"""Plain FP64 CPU oracle for the per-iteration model evaluation of the
multi-period AC OPF (Shin, Rao, Schanen, Maldonado, Anitescu, "Scalable
Multi-Period AC Optimal Power Flow Utilizing GPUs with High Memory
Capacities", arXiv 2405.14032).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library: the physics is written in complex-power form
(S = V * conj(I) on the pi-model admittances) with hand-derived derivatives
of that form, while the device path uses an expanded real trigonometric
form.  Every routine is written for clarity, vectorised with numpy over
elements, never blocked or fused.

Model (Sec. II, eq. (1a)-(1k)), with the readings taken where the
paper is silent or its printed formula is garbled:

* branch l = (i -> j) is a pi-model line with series admittance
  y = 1/(r + jx), total charging b_c, tap tau and shift phi; four flow
  variables per branch: the complex power S_f = pf + j qf entering the line
  at its from end and S_t = pt + j qt entering it at its to end
  (eq. (1d)-(1e) as the standard pi-model; the printed pair only shows the
  mutual term of one end);
* flow definition rows c = x_flow - phi(V) (eq. (1d)-(1e));
* bus balance: generation minus the flows leaving the bus through each
  incident line end minus the load (eq. (1b)-(1c));
* thermal limit in squared form at both ends (eq. (1f));
* angle difference theta_i - theta_j per line (eq. (1j));
* one two-sided ramp row per generator and period t >= 1 (eq. (1k));
* one reference-angle row va[ref, t] = 0 per period (needed for the
  constraint counts of Table II);
* quadratic cost c2 p^2 + c1 p + c0 per generator and period (eq. (1a)).

Lagrangian Hessian convention: sigma * Hess f + sum_i lambda_i Hess c_i
(Sec. III-B defines W as the Hessian of the Lagrangian; the sign of the
multipliers is the caller's).  Condensed matrix:
K = H + diag(diag_x) + J^T diag(d) J, lower triangle (Sec. III-B, M_cond,
with diag_x = delta_w + Sigma_x and d = D supplied by the caller).

Canonical 0-based layouts (a contract shared with the library):
  x per period: [vm N | va N | pg G | qg G | pf B | qf B | pt B | qt B]
  c per period: [balP N | balQ N | ref 1 | cpf B | cqf B | cpt B | cqt B |
                 thf B | tht B | ang B], then ramp rows (t-1)*G + g, t >= 1.
  J COO per period (index = block base + local * count + element):
     gen-balance (2 locals x G), branch-balance (4 x B), ref (1),
     flows ((k*5 + local) x B; k in pf,qf,pt,qt; local in own,vm_i,vm_j,
     va_i,va_j), thermal (4 x B), angle (2 x B); then the ramp block
     (t-1)*2G + local*G + g.
  H COO per period, lower (row >= col), duplicates kept:
     objective (G), flows ((k*9 + local) x B), thermal (4 x B).
  K: CSR, rows in x order, lower triangle, columns ascending, duplicates
     merged, diagonal always present.
"""
from __future__ import annotations

import numpy as np

# flow kinds: 0 = pf, 1 = qf, 2 = pt, 3 = qt
# local variable order of a branch: 0 = vm_i, 1 = vm_j, 2 = va_i, 3 = va_j
PAIRS_FROM = [(0, 0), (1, 0), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1), (3, 2), (3, 3)]
PAIRS_TO = [(1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1), (3, 2), (3, 3)]


# ----------------------------------------------------------------------------
# sizes and layout
# ----------------------------------------------------------------------------
def period_sizes(N, B, G):
    """Per-period counts: variables, constraint rows, J entries, H entries."""
    n_p = 2 * N + 2 * G + 4 * B
    m_p = 2 * N + 7 * B + 1
    nnzj_p = 2 * G + 30 * B + 1
    nnzh_p = G + 40 * B
    return n_p, m_p, nnzj_p, nnzh_p


def dims(N, B, G, T):
    """Total n, m, nnz(J), nnz(H) of a T-period instance (Sec. II, eq. (1);
    the ramp rows of eq. (1k) exist only for t >= 2 in the paper's 1-based
    numbering)."""
    n_p, m_p, nnzj_p, nnzh_p = period_sizes(N, B, G)
    return dict(n=T * n_p, m=T * m_p + G * (T - 1),
                nnz_jac=T * nnzj_p + 2 * G * (T - 1), nnz_hess=T * nnzh_p)


class Layout:
    """Index arithmetic for the canonical x / c layouts."""

    def __init__(self, net):
        N, B, G, T = net.N, net.B, net.G, net.T
        self.N, self.B, self.G, self.T = N, B, G, T
        self.n_p, self.m_p, self.nnzj_p, self.nnzh_p = period_sizes(N, B, G)
        # x block offsets inside one period
        self.vm, self.va = 0, N
        self.pg, self.qg = 2 * N, 2 * N + G
        self.flow = [2 * N + 2 * G + k * B for k in range(4)]
        # c block offsets inside one period
        self.balp, self.balq, self.ref = 0, N, 2 * N
        self.cflow = [2 * N + 1 + k * B for k in range(4)]
        self.thf, self.tht = 2 * N + 1 + 4 * B, 2 * N + 1 + 5 * B
        self.ang = 2 * N + 1 + 6 * B
        d = dims(N, B, G, T)
        self.n, self.m = d["n"], d["m"]

    def xt(self, t):
        """(T, 1) period offsets into x."""
        return (np.arange(self.T) * self.n_p)[:, None] if t is None else t * self.n_p

    def ct(self):
        return (np.arange(self.T) * self.m_p)[:, None]

    def ramp_row(self, t, g):
        return self.T * self.m_p + (t - 1) * self.G + g


def unpack_x(net, x):
    """Split x into (T, .) blocks vm, va, pg, qg, pf, qf, pt, qt."""
    L = Layout(net)
    X = np.asarray(x, dtype=np.float64).reshape(net.T, L.n_p)
    N, B, G = net.N, net.B, net.G
    vm = X[:, 0:N]
    va = X[:, N:2 * N]
    pg = X[:, 2 * N:2 * N + G]
    qg = X[:, 2 * N + G:2 * N + 2 * G]
    fl = [X[:, L.flow[k]:L.flow[k] + B] for k in range(4)]
    return vm, va, pg, qg, fl


# ----------------------------------------------------------------------------
# physics in complex-power form
# ----------------------------------------------------------------------------
def admittances(net):
    """Pi-model branch admittances (Y_ff, Y_ft, Y_tf, Y_tt): series y between
    the ends, j b_c / 2 shunt at each end, ideal transformer tau e^{j phi} on
    the from side."""
    y = 1.0 / (net.r + 1j * net.x)
    a = net.tap * np.exp(1j * net.shift)
    ytt = y + 0.5j * net.b_charge
    yff = ytt / (net.tap ** 2)
    yft = -y / np.conj(a)
    ytf = -y / a
    return yff, yft, ytf, ytt


def branch_power(net, vm, va):
    """Complex power entering each line at its from and to ends,
    S = V conj(I) with I = Y V (the definition; flows of eq. (1d)-(1e))."""
    yff, yft, ytf, ytt = admittances(net)
    V = vm * np.exp(1j * va)
    vf = V[:, net.f_bus]
    vt = V[:, net.t_bus]
    i_f = yff * vf + yft * vt
    i_t = ytf * vf + ytt * vt
    return vf * np.conj(i_f), vt * np.conj(i_t)


def _end_terms(net, vm, va):
    """Per end: self coefficient A and mutual term E of
    S = A |V_o|^2 + E V_i V_j  (expanded S = V conj(Y V)), with
    E_f = conj(Y_ft) e^{j delta}, E_t = conj(Y_tf) e^{-j delta},
    delta = va_i - va_j."""
    yff, yft, ytf, ytt = admittances(net)
    vi = vm[:, net.f_bus]
    vj = vm[:, net.t_bus]
    delta = va[:, net.f_bus] - va[:, net.t_bus]
    ef = np.conj(yft) * np.exp(1j * delta)
    et = np.conj(ytf) * np.exp(-1j * delta)
    return vi, vj, np.conj(yff), ef, np.conj(ytt), et, (np.abs(yff), np.abs(yft), np.abs(ytf), np.abs(ytt))


def _first_derivs(vi, vj, af, ef, at, et):
    """dS/d(vm_i, vm_j, va_i, va_j) for both ends (lists of 4 complex (T,B)).
    From end: S_f = A_f vi^2 + E_f vi vj, dE_f/dva_i = jE_f, dE_f/dva_j = -jE_f.
    To end:   S_t = A_t vj^2 + E_t vi vj, dE_t/dva_i = -jE_t, dE_t/dva_j = jE_t."""
    dsf = [2 * af * vi + ef * vj, ef * vi, 1j * ef * vi * vj, -1j * ef * vi * vj]
    dst = [et * vj, 2 * at * vj + et * vi, -1j * et * vi * vj, 1j * et * vi * vj]
    return dsf, dst


def _second_derivs(vi, vj, a_self, e, self_on_i, s):
    """Symmetric 4x4 second derivatives of S = A vo^2 + E vi vj w.r.t.
    (vm_i, vm_j, va_i, va_j); s = +1 for the from end (dE/dva_i = jE),
    s = -1 for the to end.  Returned as dict {(a, b): complex (T,B)}."""
    js = 1j * s
    zero = np.zeros_like(e)
    d = {}
    d[(0, 0)] = 2 * a_self * np.ones_like(vi) if self_on_i else zero
    d[(1, 1)] = zero if self_on_i else 2 * a_self * np.ones_like(vi)
    d[(1, 0)] = e
    d[(2, 0)] = js * e * vj
    d[(2, 1)] = js * e * vi
    d[(3, 0)] = -js * e * vj
    d[(3, 1)] = -js * e * vi
    d[(2, 2)] = (js * js) * e * vi * vj
    d[(3, 3)] = (js * js) * e * vi * vj
    d[(3, 2)] = (js * -js) * e * vi * vj
    return d


# ----------------------------------------------------------------------------
# objective, gradient, constraints (eq. (1a)-(1k))
# ----------------------------------------------------------------------------
def objective(net, x):
    """f = sum_t sum_g c2 pg^2 + c1 pg + c0 (eq. (1a), quadratic cost)."""
    _, _, pg, _, _ = unpack_x(net, x)
    return float(np.sum(net.c2 * pg ** 2 + net.c1 * pg + net.c0))


def objective_mag(net, x):
    _, _, pg, _, _ = unpack_x(net, x)
    return float(np.sum(np.abs(net.c2 * pg ** 2) + np.abs(net.c1 * pg) + np.abs(net.c0)))


def gradient(net, x):
    """grad f: 2 c2 pg + c1 on the pg entries, zero elsewhere (eq. (1a))."""
    L = Layout(net)
    _, _, pg, _, _ = unpack_x(net, x)
    g = np.zeros((net.T, L.n_p))
    g[:, L.pg:L.pg + net.G] = 2 * net.c2 * pg + net.c1
    return g.reshape(-1)


def gradient_mag(net, x):
    L = Layout(net)
    _, _, pg, _, _ = unpack_x(net, x)
    g = np.zeros((net.T, L.n_p))
    g[:, L.pg:L.pg + net.G] = np.abs(2 * net.c2 * pg) + np.abs(net.c1)
    return g.reshape(-1)


def constraints(net, x, pd=None, qd=None, with_mag=False):
    """All constraint rows in canonical order (eq. (1b)-(1f), (1j), (1k) and
    the reference-angle row).  With ``with_mag`` also returns, per row, the
    sum of the absolute values of its terms (the cancellation scale)."""
    L = Layout(net)
    pd = net.pd if pd is None else np.asarray(pd).reshape(net.T, net.N)
    qd = net.qd if qd is None else np.asarray(qd).reshape(net.T, net.N)
    T, N, B, G = net.T, net.N, net.B, net.G
    vm, va, pg, qg, (pf, qf, pt, qt) = unpack_x(net, x)
    sf, st = branch_power(net, vm, va)
    C = np.zeros((T, L.m_p))
    M = np.zeros((T, L.m_p))
    # balance: generation - flows leaving through each incident end - load
    balp = -pd.copy()
    balq = -qd.copy()
    magp = np.abs(pd).copy()
    magq = np.abs(qd).copy()
    for (arr, mag, gen, fr, to) in ((balp, magp, pg, pf, pt), (balq, magq, qg, qf, qt)):
        np.add.at(arr, (slice(None), net.gen_bus), gen)
        np.add.at(arr, (slice(None), net.f_bus), -fr)
        np.add.at(arr, (slice(None), net.t_bus), -to)
        np.add.at(mag, (slice(None), net.gen_bus), np.abs(gen))
        np.add.at(mag, (slice(None), net.f_bus), np.abs(fr))
        np.add.at(mag, (slice(None), net.t_bus), np.abs(to))
    C[:, L.balp:L.balp + N] = balp
    C[:, L.balq:L.balq + N] = balq
    M[:, L.balp:L.balp + N] = magp
    M[:, L.balq:L.balq + N] = magq
    C[:, L.ref] = va[:, net.ref_bus]
    M[:, L.ref] = np.abs(va[:, net.ref_bus])
    # flow definitions: x_flow - phi(V)
    phis = [sf.real, sf.imag, st.real, st.imag]
    yff, yft, ytf, ytt = (np.abs(v) for v in admittances(net))
    vi = vm[:, net.f_bus]
    vj = vm[:, net.t_bus]
    smag = [yff * vi ** 2 + yft * vi * vj] * 2 + [ytt * vj ** 2 + ytf * vi * vj] * 2
    for k, (xv, phi) in enumerate(zip((pf, qf, pt, qt), phis)):
        C[:, L.cflow[k]:L.cflow[k] + B] = xv - phi
        M[:, L.cflow[k]:L.cflow[k] + B] = np.abs(xv) + smag[k]
    # thermal limits, squared, both ends
    C[:, L.thf:L.thf + B] = pf ** 2 + qf ** 2
    C[:, L.tht:L.tht + B] = pt ** 2 + qt ** 2
    M[:, L.thf:L.thf + B] = pf ** 2 + qf ** 2
    M[:, L.tht:L.tht + B] = pt ** 2 + qt ** 2
    # angle difference
    C[:, L.ang:L.ang + B] = va[:, net.f_bus] - va[:, net.t_bus]
    M[:, L.ang:L.ang + B] = np.abs(va[:, net.f_bus]) + np.abs(va[:, net.t_bus])
    # ramp rows for t >= 1 (0-based)
    ramp = (pg[1:] - pg[:-1]).reshape(-1)
    rampm = (np.abs(pg[1:]) + np.abs(pg[:-1])).reshape(-1)
    c = np.concatenate([C.reshape(-1), ramp])
    if with_mag:
        return c, np.concatenate([M.reshape(-1), rampm])
    return c


def bounds(net):
    """Variable and row bounds (eq. (1f)-(1k); flows and angles free)."""
    L = Layout(net)
    T, N, B, G = net.T, net.N, net.B, net.G
    inf = np.inf
    lv = np.full((T, L.n_p), -inf)
    uv = np.full((T, L.n_p), inf)
    lv[:, L.vm:L.vm + N] = net.vmin
    uv[:, L.vm:L.vm + N] = net.vmax
    lv[:, L.pg:L.pg + G] = net.pmin
    uv[:, L.pg:L.pg + G] = net.pmax
    lv[:, L.qg:L.qg + G] = net.qmin
    uv[:, L.qg:L.qg + G] = net.qmax
    lc = np.zeros((T, L.m_p))
    uc = np.zeros((T, L.m_p))
    lc[:, L.thf:L.thf + B] = -inf
    lc[:, L.tht:L.tht + B] = -inf
    uc[:, L.thf:L.thf + B] = net.rate ** 2
    uc[:, L.tht:L.tht + B] = net.rate ** 2
    lc[:, L.ang:L.ang + B] = net.angmin
    uc[:, L.ang:L.ang + B] = net.angmax
    lr = np.tile(-net.ramp, T - 1)
    ur = np.tile(net.ramp, T - 1)
    return (lv.reshape(-1), uv.reshape(-1),
            np.concatenate([lc.reshape(-1), lr]), np.concatenate([uc.reshape(-1), ur]))


# ----------------------------------------------------------------------------
# sparse Jacobian (Sec. III-A: COO expanded per pattern)
# ----------------------------------------------------------------------------
def jacobian(net, x, with_mag=False):
    """Constraint Jacobian in canonical COO order: (rows, cols, vals[, mag])."""
    L = Layout(net)
    T, N, B, G = net.T, net.N, net.B, net.G
    xo = (np.arange(T) * L.n_p)[:, None]
    co = (np.arange(T) * L.m_p)[:, None]
    f, tb, gb = net.f_bus[None, :], net.t_bus[None, :], net.gen_bus[None, :]
    vm, va, pg, qg, fl = unpack_x(net, x)
    vi, vj, af, ef, at, et, (myff, myft, mytf, mytt) = _end_terms(net, vm, va)
    dsf, dst = _first_derivs(vi, vj, af, ef, at, et)
    # magnitude bounds of the derivative terms
    mdsf = [2 * myff * vi + myft * vj, myft * vi, myft * vi * vj, myft * vi * vj]
    mdst = [mytf * vj, 2 * mytt * vj + mytf * vi, mytf * vi * vj, mytf * vi * vj]
    R, Cc, V, Mg = [], [], [], []

    def put(r, c, v, mg=None):
        shape = np.broadcast_shapes(np.shape(r), np.shape(c), np.shape(v))
        R.append(np.broadcast_to(r, shape))
        Cc.append(np.broadcast_to(c, shape))
        vv = np.broadcast_to(np.asarray(v, dtype=np.float64), shape)
        V.append(vv)
        Mg.append(np.abs(vv) if mg is None else np.broadcast_to(mg, shape))

    ones_g = np.ones((T, G))
    ones_b = np.ones((T, B))
    # 1. generator terms of the balance rows
    put(co + L.balp + gb, xo + L.pg + np.arange(G)[None, :], ones_g)
    put(co + L.balq + gb, xo + L.qg + np.arange(G)[None, :], ones_g)
    # 2. line-end terms of the balance rows
    bidx = np.arange(B)[None, :]
    put(co + L.balp + f, xo + L.flow[0] + bidx, -ones_b)
    put(co + L.balq + f, xo + L.flow[1] + bidx, -ones_b)
    put(co + L.balp + tb, xo + L.flow[2] + bidx, -ones_b)
    put(co + L.balq + tb, xo + L.flow[3] + bidx, -ones_b)
    # 3. reference angle
    put(co + L.ref, xo + L.va + net.ref_bus, np.ones((T, 1)))
    # 4. flow definitions, kind-major then local then line
    busvar = [xo + L.vm + f, xo + L.vm + tb, xo + L.va + f, xo + L.va + tb]
    for k in range(4):
        ds = dsf if k < 2 else dst
        mds = mdsf if k < 2 else mdst
        part = (lambda z: z.real) if k % 2 == 0 else (lambda z: z.imag)
        row = co + L.cflow[k] + bidx
        put(row, xo + L.flow[k] + bidx, ones_b)
        for a in range(4):
            put(row, busvar[a], -part(ds[a]), mds[a])
    # 5. thermal rows
    put(co + L.thf + bidx, xo + L.flow[0] + bidx, 2 * fl[0])
    put(co + L.thf + bidx, xo + L.flow[1] + bidx, 2 * fl[1])
    put(co + L.tht + bidx, xo + L.flow[2] + bidx, 2 * fl[2])
    put(co + L.tht + bidx, xo + L.flow[3] + bidx, 2 * fl[3])
    # 6. angle rows
    put(co + L.ang + bidx, busvar[2], ones_b)
    put(co + L.ang + bidx, busvar[3], -ones_b)
    rows = np.concatenate([r.astype(np.int64) for r in R], axis=1).reshape(-1)
    cols = np.concatenate([c.astype(np.int64) for c in Cc], axis=1).reshape(-1)
    vals = np.concatenate(V, axis=1).reshape(-1)
    mags = np.concatenate(Mg, axis=1).reshape(-1)
    # ramp block: (ramp(t,g), pg_t) = +1 then (ramp(t,g), pg_{t-1}) = -1
    if T > 1:
        t = np.arange(1, T)[:, None]
        g = np.arange(G)[None, :]
        rr = L.ramp_row(t, g)
        r_rows = np.concatenate([rr, rr], axis=1).reshape(-1)
        r_cols = np.concatenate([t * L.n_p + L.pg + g, (t - 1) * L.n_p + L.pg + g], axis=1).reshape(-1)
        r_vals = np.concatenate([np.ones((T - 1, G)), -np.ones((T - 1, G))], axis=1).reshape(-1)
        rows = np.concatenate([rows, r_rows])
        cols = np.concatenate([cols, r_cols])
        vals = np.concatenate([vals, r_vals])
        mags = np.concatenate([mags, np.abs(r_vals)])
    if with_mag:
        return rows, cols, vals, mags
    return rows, cols, vals


# ----------------------------------------------------------------------------
# sparse Lagrangian Hessian (Sec. III-A/III-B: W = Hessian of the Lagrangian)
# ----------------------------------------------------------------------------
def hessian(net, x, lam, sigma=1.0, with_mag=False):
    """Lower-triangular COO of sigma Hess f + sum_i lam_i Hess c_i, canonical
    order, duplicates kept."""
    L = Layout(net)
    T, N, B, G = net.T, net.N, net.B, net.G
    lam = np.asarray(lam, dtype=np.float64)
    xo = (np.arange(T) * L.n_p)[:, None]
    LAM = lam[:T * L.m_p].reshape(T, L.m_p)
    f, tb = net.f_bus[None, :], net.t_bus[None, :]
    vm, va, pg, qg, fl = unpack_x(net, x)
    vi, vj, af, ef, at, et, (myff, myft, mytf, mytt) = _end_terms(net, vm, va)
    d2f = _second_derivs(vi, vj, af, ef, True, +1)
    d2t = _second_derivs(vi, vj, at, et, False, -1)
    # magnitude bounds: |A|, |E| times the same monomials
    m2f = _second_derivs(vi, vj, myff, myft * np.ones_like(vi), True, +1)
    m2t = _second_derivs(vi, vj, mytt, mytf * np.ones_like(vi), False, -1)
    busvar = [xo + L.vm + f, xo + L.vm + tb, xo + L.va + f, xo + L.va + tb]
    R, Cc, V, Mg = [], [], [], []
    # 1. objective
    gidx = xo + L.pg + np.arange(G)[None, :]
    hobj = np.broadcast_to(2.0 * sigma * net.c2, (T, G))
    R.append(gidx)
    Cc.append(gidx)
    V.append(hobj)
    Mg.append(np.abs(hobj))
    # 2. flow rows: -lam_k * Hess phi_k
    for k in range(4):
        d2, m2, pairs = (d2f, m2f, PAIRS_FROM) if k < 2 else (d2t, m2t, PAIRS_TO)
        part = (lambda z: z.real) if k % 2 == 0 else (lambda z: z.imag)
        lk = LAM[:, L.cflow[k]:L.cflow[k] + B]
        for (a, b) in pairs:
            ra, rb = busvar[a], busvar[b]
            R.append(np.maximum(ra, rb))
            Cc.append(np.minimum(ra, rb))
            V.append(-lk * part(d2[(a, b)]))
            Mg.append(np.abs(lk) * np.abs(m2[(a, b)]))
    # 3. thermal rows: 2 lam on the squared flow variables
    bidx = np.arange(B)[None, :]
    for k, th in ((0, L.thf), (1, L.thf), (2, L.tht), (3, L.tht)):
        v = xo + L.flow[k] + bidx
        h = 2.0 * LAM[:, th:th + B]
        R.append(v)
        Cc.append(v)
        V.append(h)
        Mg.append(np.abs(h))
    rows = np.concatenate([np.broadcast_to(r, (T, r.shape[1])).astype(np.int64) for r in R], axis=1).reshape(-1)
    cols = np.concatenate([np.broadcast_to(c, (T, c.shape[1])).astype(np.int64) for c in Cc], axis=1).reshape(-1)
    vals = np.concatenate([np.broadcast_to(v, (T, v.shape[1])) for v in V], axis=1).reshape(-1)
    mags = np.concatenate([np.broadcast_to(v, (T, v.shape[1])) for v in Mg], axis=1).reshape(-1)
    if with_mag:
        return rows, cols, vals, mags
    return rows, cols, vals


# ----------------------------------------------------------------------------
# adjoint products
# ----------------------------------------------------------------------------
def jtprod(net, x, v, with_mag=False):
    """J^T v by a COO sparse product over this module's own Jacobian."""
    import scipy.sparse as sp
    L = Layout(net)
    rows, cols, vals, mags = jacobian(net, x, with_mag=True)
    J = sp.coo_matrix((vals, (rows, cols)), shape=(L.m, L.n))
    out = J.T @ np.asarray(v, dtype=np.float64)
    if with_mag:
        Jm = sp.coo_matrix((mags, (rows, cols)), shape=(L.m, L.n))
        return out, Jm.T @ np.abs(v)
    return out


def load_adjoint(net, lam):
    """d(lam^T c)/d(pd, qd): the load enters the balance rows with
    coefficient -1 (eq. (1b)-(1c)), so the adjoint is -lam_balP, -lam_balQ,
    each shaped (T, N)."""
    L = Layout(net)
    LAM = np.asarray(lam)[:net.T * L.m_p].reshape(net.T, L.m_p)
    return -LAM[:, L.balp:L.balp + net.N].copy(), -LAM[:, L.balq:L.balq + net.N].copy()


# ----------------------------------------------------------------------------
# condensed KKT matrix (Sec. III-B: M_cond = W + delta_w I + Sigma_x + A^T D A)
# ----------------------------------------------------------------------------
def condensed(n, jac, hess, diag_x, dcon, row_mask=None, jac_mag=None, hess_mag=None):
    """K = lower(H + diag(diag_x) + J^T diag(dcon) J) by sort-and-reduce of
    every contribution (row, col, value).

    jac = (rows, cols, vals) with unique (row, col); hess = lower COO.
    Returns (rowptr int64 [n+1], colind int64, vals, mag) where mag is the
    per-slot sum of the contributions' magnitude scales: |d| m(J_a) m(J_b)
    for a product, m(H) for a Hessian entry, |diag| -- with m(.) the
    cancellation scale of a J / H entry when jac_mag / hess_mag are given
    (the terms an entry is made of), else its absolute value.  ``row_mask``
    (bool [n]) restricts the output to the selected rows (rowptr then still
    spans all n rows; the values of the selected rows are exactly those of
    the full matrix)."""
    jr, jc, jv = (np.asarray(a) for a in jac)
    hr, hc, hv = (np.asarray(a) for a in hess)
    jm = np.abs(jv) if jac_mag is None else np.asarray(jac_mag, dtype=np.float64)
    hm = np.abs(hv) if hess_mag is None else np.asarray(hess_mag, dtype=np.float64)
    dcon = np.asarray(dcon, dtype=np.float64)
    if diag_x is None:
        diag_x = np.zeros(n)
    if row_mask is not None:
        # keep J rows that touch a selected column; H entries in selected rows
        touch = row_mask[jc]
        keep_rows = np.zeros(int(jr.max()) + 1 if jr.size else 1, dtype=bool)
        keep_rows[jr[touch]] = True
        sel = keep_rows[jr]
        jr, jc, jv, jm = jr[sel], jc[sel], jv[sel], jm[sel]
        hs = row_mask[hr]
        hr, hc, hv, hm = hr[hs], hc[hs], hv[hs], hm[hs]
    # pairs of entries within each J row (entry with itself included)
    order = np.lexsort((jc, jr))
    jr, jc, jv, jm = jr[order], jc[order], jv[order], jm[order]
    if jr.size:
        key = jr * (n + 1) + jc
        if np.any(key[1:] == key[:-1]):
            raise ValueError("J has duplicate (row, col) entries")
    first = np.ones(jr.size, dtype=bool)
    first[1:] = jr[1:] != jr[:-1]
    start = np.maximum.accumulate(np.where(first, np.arange(jr.size), 0))
    pos = np.arange(jr.size) - start
    cnt = pos + 1
    e = np.repeat(np.arange(jr.size), cnt)
    q = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    p = start[e] + q
    pr = np.maximum(jc[e], jc[p])
    pc = np.minimum(jc[e], jc[p])
    pv = dcon[jr[e]] * jv[e] * jv[p]
    pm = np.abs(dcon[jr[e]]) * jm[e] * jm[p]
    diag_idx = np.arange(n) if row_mask is None else np.nonzero(row_mask)[0]
    dvals = np.asarray(diag_x, dtype=np.float64)[diag_idx]
    R = np.concatenate([pr, hr, diag_idx])
    C = np.concatenate([pc, hc, diag_idx])
    Vv = np.concatenate([pv, hv, dvals])
    Mv = np.concatenate([pm, hm, np.abs(dvals)])
    if row_mask is not None:
        s = row_mask[R]
        R, C, Vv, Mv = R[s], C[s], Vv[s], Mv[s]
    if np.any(C > R):
        raise ValueError("upper-triangular contribution")
    key = R.astype(np.int64) * n + C.astype(np.int64)
    o = np.argsort(key, kind="stable")
    key, Vv, Mv = key[o], Vv[o], Mv[o]
    uniq, first_idx = np.unique(key, return_index=True)
    vals = np.add.reduceat(Vv, first_idx) if key.size else np.zeros(0)
    mag = np.add.reduceat(Mv, first_idx) if key.size else np.zeros(0)
    rows = uniq // n
    cols = uniq % n
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cols.astype(np.int64), vals, mag


def hessian_dense(n, hess):
    """Dense symmetric matrix of a lower COO with duplicates (for tests)."""
    hr, hc, hv = hess
    H = np.zeros((n, n))
    np.add.at(H, (hr, hc), hv)
    return H + np.tril(H, -1).T


# ----------------------------------------------------------------------------
# lifted-KKT condensation: right-hand side and step recovery (Sec. III-B)
# ----------------------------------------------------------------------------
def jprod(net, x, v, with_mag=False):
    """J v by a COO sparse product over this module's own Jacobian (the
    A dx term of the step recovery)."""
    import scipy.sparse as sp
    L = Layout(net)
    rows, cols, vals, mags = jacobian(net, x, with_mag=True)
    J = sp.coo_matrix((vals, (rows, cols)), shape=(L.m, L.n))
    out = J @ np.asarray(v, dtype=np.float64)
    if with_mag:
        Jm = sp.coo_matrix((mags, (rows, cols)), shape=(L.m, L.n))
        return out, Jm @ np.abs(v)
    return out


def _bound_terms(val, lo, hi, zlo, zhi, mu):
    """Barrier terms of the box lo <= val <= hi, entry by entry.

    Returns (sigma, p_lo, p_hi, gap_lo, gap_hi, has_lo, has_hi):
    sigma = Z_lo (val - lo)^-1 + Z_hi (hi - val)^-1 (Sigma_x / Sigma_s of
    Sec. III-B), p_lo = Z_lo (val - lo) - mu and p_hi = Z_hi (hi - val) - mu
    (the complementarity residuals; reading: the paper prints two of the four
    with the wrong variable, each is read as the residual of its own bound).
    An infinite bound has no multiplier and contributes nothing (the limit
    of every term as the bound goes to infinity with its multiplier at 0)."""
    has_lo, has_hi = np.isfinite(lo), np.isfinite(hi)
    gap_lo = np.where(has_lo, val - np.where(has_lo, lo, 0.0), 1.0)
    gap_hi = np.where(has_hi, np.where(has_hi, hi, 0.0) - val, 1.0)
    zlo = np.where(has_lo, zlo, 0.0)
    zhi = np.where(has_hi, zhi, 0.0)
    sigma = zlo / gap_lo + zhi / gap_hi
    p_lo = np.where(has_lo, zlo * gap_lo - mu, 0.0)
    p_hi = np.where(has_hi, zhi * gap_hi - mu, 0.0)
    return sigma, p_lo, p_hi, gap_lo, gap_hi, has_lo, has_hi


def _row_terms(st, c):
    """Row-space quantities of Sec. III-B: Sigma_s, q_s, q_y = p_y, C, D and
    the slack-bound residuals.  p_s = -z_s_lo + z_s_hi + y, p_y = g(x) - s,
    q_s = p_s + (S - S_lo)^-1 p_lo - (S_hi - S)^-1 p_hi,
    C = (delta_c Sigma_s + (1 + delta_c delta_w) I)^-1,
    D = (Sigma_s + delta_w I) C."""
    sig_s, p_lo, p_hi, g_lo, g_hi, h_lo, h_hi = _bound_terms(st.s, st.sl, st.su, st.vl, st.vu, st.mu)
    vl = np.where(h_lo, st.vl, 0.0)
    vu = np.where(h_hi, st.vu, 0.0)
    p_s = -vl + vu + st.y
    p_y = np.asarray(c) - st.s
    q_s = p_s + np.where(h_lo, p_lo / g_lo, 0.0) - np.where(h_hi, p_hi / g_hi, 0.0)
    C = 1.0 / (st.delta_c * sig_s + (1.0 + st.delta_c * st.delta_w))
    D = (sig_s + st.delta_w) * C
    return dict(sig_s=sig_s, p_lo=p_lo, p_hi=p_hi, g_lo=g_lo, g_hi=g_hi, h_lo=h_lo, h_hi=h_hi, vl=vl, vu=vu,
                p_s=p_s, p_y=p_y, q_s=q_s, C=C, D=D)


def _row_terms_mag(st, c, R):
    """Cancellation scales of q_s and p_y (every term by its absolute value)."""
    ps_m = np.abs(R["vl"]) + np.abs(R["vu"]) + np.abs(st.y)
    plo_m = np.where(R["h_lo"], np.abs(R["vl"] * R["g_lo"]) + st.mu, 0.0)
    phi_m = np.where(R["h_hi"], np.abs(R["vu"] * R["g_hi"]) + st.mu, 0.0)
    qs_m = ps_m + plo_m / R["g_lo"] + phi_m / R["g_hi"]
    py_m = np.abs(np.asarray(c)) + np.abs(st.s)
    return qs_m, py_m, plo_m, phi_m


def condensed_rhs(net, st, grad, c, with_mag=False):
    """The condensed system's diagonal weights and right-hand side (Sec.
    III-B): diag_x = delta_w + Sigma_x, dcon = D and
    rhs = q_x + A^T (C q_s + D q_y), with p_x = grad f - A^T y - z_lo + z_hi
    and q_x = p_x + (X - X_lo)^-1 p_lo - (X_hi - X)^-1 p_hi.
    grad = grad f(x) and c = g(x) at st.x.  With ``with_mag`` also returns the
    cancellation scale of each rhs entry."""
    sig_x, pz_lo, pz_hi, gx_lo, gx_hi, hx_lo, hx_hi = _bound_terms(st.x, st.xl, st.xu, st.zl, st.zu, st.mu)
    zl = np.where(hx_lo, st.zl, 0.0)
    zu = np.where(hx_hi, st.zu, 0.0)
    R = _row_terms(st, c)
    jty, jty_m = jtprod(net, st.x, st.y, with_mag=True)
    p_x = np.asarray(grad) - jty - zl + zu
    q_x = p_x + np.where(hx_lo, pz_lo / gx_lo, 0.0) - np.where(hx_hi, pz_hi / gx_hi, 0.0)
    w = R["C"] * R["q_s"] + R["D"] * R["p_y"]
    jtw, jtw_m = jtprod(net, st.x, w, with_mag=True)
    rhs = q_x + jtw
    diag_x = st.delta_w + sig_x
    if not with_mag:
        return diag_x, R["D"], rhs
    qs_m, py_m, _, _ = _row_terms_mag(st, c, R)
    w_m = R["C"] * qs_m + R["D"] * py_m
    _, jtw_m = jtprod(net, st.x, w_m, with_mag=True)
    pzl_m = np.where(hx_lo, np.abs(zl * gx_lo) + st.mu, 0.0)
    pzu_m = np.where(hx_hi, np.abs(zu * gx_hi) + st.mu, 0.0)
    qx_m = np.abs(grad) + jty_m + np.abs(zl) + np.abs(zu) + pzl_m / gx_lo + pzu_m / gx_hi
    return diag_x, R["D"], rhs, qx_m + jtw_m


def recover_step(net, st, c, dx, with_mag=False):
    """Slack, multiplier and bound-multiplier steps from the condensed
    solution dx (Sec. III-B):
      ds  = C (A dx + delta_c q_s - q_y)   (reading: the printed formula
            carries A dx with the opposite sign, which contradicts the
            condensed system it comes from; eliminating the third block row
            of the full system gives this sign),
      dy  = (Sigma_s + delta_w I) ds - q_s,
      dz_lo = (X - X_lo)^-1 (-Z_lo dx + p_lo),  dz_hi = (X_hi - X)^-1 (Z_hi dx + p_hi),
      and the same for the slack bounds with ds.
    Returns (ds, dy, dzl, dzu, dvl, dvu)[, and their cancellation scales]."""
    _, pz_lo, pz_hi, gx_lo, gx_hi, hx_lo, hx_hi = _bound_terms(st.x, st.xl, st.xu, st.zl, st.zu, st.mu)
    zl = np.where(hx_lo, st.zl, 0.0)
    zu = np.where(hx_hi, st.zu, 0.0)
    R = _row_terms(st, c)
    adx, adx_m = jprod(net, st.x, dx, with_mag=True)
    dx = np.asarray(dx)
    ds = R["C"] * (adx + st.delta_c * R["q_s"] - R["p_y"])
    dy = (R["sig_s"] + st.delta_w) * ds - R["q_s"]
    dzl = np.where(hx_lo, (-zl * dx + pz_lo) / gx_lo, 0.0)
    dzu = np.where(hx_hi, (zu * dx + pz_hi) / gx_hi, 0.0)
    dvl = np.where(R["h_lo"], (-R["vl"] * ds + R["p_lo"]) / R["g_lo"], 0.0)
    dvu = np.where(R["h_hi"], (R["vu"] * ds + R["p_hi"]) / R["g_hi"], 0.0)
    out = (ds, dy, dzl, dzu, dvl, dvu)
    if not with_mag:
        return out
    qs_m, py_m, plo_m, phi_m = _row_terms_mag(st, c, R)
    ds_m = R["C"] * (adx_m + st.delta_c * qs_m + py_m)
    dy_m = (R["sig_s"] + st.delta_w) * ds_m + qs_m
    pzl_m = np.where(hx_lo, np.abs(zl * gx_lo) + st.mu, 0.0)
    pzu_m = np.where(hx_hi, np.abs(zu * gx_hi) + st.mu, 0.0)
    dzl_m = (np.abs(zl * dx) + pzl_m) / gx_lo
    dzu_m = (np.abs(zu * dx) + pzu_m) / gx_hi
    dvl_m = (np.abs(R["vl"]) * ds_m + plo_m) / R["g_lo"]
    dvu_m = (np.abs(R["vu"]) * ds_m + phi_m) / R["g_hi"]
    return out, (ds_m, dy_m, dzl_m, dzu_m, dvl_m, dvu_m)


# ----------------------------------------------------------------------------
# the condensed system (Sec. III-B): K dx = rhs
# ----------------------------------------------------------------------------
def kkt_full(n, rowptr, colind, vals):
    """The full symmetric K (scipy CSR) from its lower-triangle CSR: the
    strictly lower entries mirrored above the diagonal, the diagonal once."""
    import scipy.sparse as sp
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    Lo = sp.csr_matrix((vals, (rows, colind)), shape=(n, n))
    strict = sp.tril(Lo, -1)
    return (Lo + strict.T).tocsr()


def kkt_solve(n, rowptr, colind, vals, b):
    """dx with K dx = b for K given by its lower CSR (the condensed system of
    Sec. III-B), by a general sparse LU of the full symmetric matrix (a
    library primitive: the solution of a nonsingular system is unique, so any
    exact method defines it)."""
    import scipy.sparse.linalg as sla
    K = kkt_full(n, rowptr, colind, vals).tocsc()
    return sla.spsolve(K, np.asarray(b, dtype=np.float64))


def kkt_is_positive_definite(n, rowptr, colind, vals):
    """Whether K is positive definite, by a dense Cholesky attempt (small
    cases only): the property static pivoting relies on (Sec. III-B, K is
    positive definite after inertia correction)."""
    K = kkt_full(n, rowptr, colind, vals).toarray()
    try:
        np.linalg.cholesky(K)
        return True
    except np.linalg.LinAlgError:
        return False


# ----------------------------------------------------------------------------
# the lifted-KKT interior-point loop (Sec. III-B around the condensed system)
# ----------------------------------------------------------------------------
def ipm_start(net, relax=1e-4):
    """Starting iterate: flat voltages (vm = 1, va = 0), generation at the
    middle of its box, flows equal to the flows of that voltage profile (the
    flow rows hold), every bounded entry moved at least 1e-2 max(1, |bound|)
    (at most half the box) inside its bounds; slacks = c(x) moved inside the
    relaxed row bounds the same way; y = 0; bound multipliers 1 where the
    bound is finite."""
    L = Layout(net)
    xl, xu, cl, cu = bounds(net)
    eq = cl == cu
    sl = np.where(eq, cl - relax, cl)
    su = np.where(eq, cu + relax, cu)
    X = np.zeros((net.T, L.n_p))
    X[:, L.vm:L.vm + net.N] = 1.0
    X[:, L.pg:L.pg + net.G] = 0.5 * (net.pmin + net.pmax)
    X[:, L.qg:L.qg + net.G] = 0.5 * (net.qmin + net.qmax)
    C0 = constraints(net, X.reshape(-1))[:net.T * L.m_p].reshape(net.T, L.m_p)
    for k in range(4):
        X[:, L.flow[k]:L.flow[k] + net.B] = -C0[:, L.cflow[k]:L.cflow[k] + net.B]

    def inside(v, lo, hi):
        with np.errstate(invalid="ignore"):
            half = 0.5 * (hi - lo)
            pl = np.where(np.isfinite(lo), 1e-2 * np.maximum(1.0, np.abs(lo)), 0.0)
            pu = np.where(np.isfinite(hi), 1e-2 * np.maximum(1.0, np.abs(hi)), 0.0)
            pl = np.where(np.isfinite(half), np.minimum(pl, half), pl)
            pu = np.where(np.isfinite(half), np.minimum(pu, half), pu)
            v = np.where(np.isfinite(lo), np.maximum(v, lo + pl), v)
            return np.where(np.isfinite(hi), np.minimum(v, hi - pu), v)

    x = inside(X.reshape(-1), xl, xu)
    s = inside(constraints(net, x), sl, su)
    fin = lambda b: np.where(np.isfinite(b), 1.0, 0.0)
    return dict(x=x, s=s, y=np.zeros(L.m), zl=fin(xl), zu=fin(xu), vl=fin(sl), vu=fin(su),
                xl=xl, xu=xu, sl=sl, su=su)


def ipm_residuals(net, w, mu):
    """Residuals of the lifted KKT conditions at iterate w (Sec. III-B):
    p_x = grad f - J^T y - zl + zu, p_s = -vl + vu + y, q_y = c - s and the
    complementarity products of the finite bounds minus mu (absent bounds
    contribute nothing).  Returns (rd, rs, rp, gaps, c, grad)."""
    x, s = w["x"], w["s"]
    hl, hu, gl, gu = (np.isfinite(w[k]) for k in ("xl", "xu", "sl", "su"))
    grad, c = gradient(net, x), constraints(net, x)
    jr, jc, jv = jacobian(net, x)
    Jty = np.zeros(x.size)
    np.add.at(Jty, jc, jv * w["y"][jr])
    rd = grad - Jty - np.where(hl, w["zl"], 0.0) + np.where(hu, w["zu"], 0.0)
    rs = -np.where(gl, w["vl"], 0.0) + np.where(gu, w["vu"], 0.0) + w["y"]
    rp = c - s
    gaps = np.concatenate([w["zl"][hl] * (x[hl] - w["xl"][hl]), w["zu"][hu] * (w["xu"][hu] - x[hu]),
                           w["vl"][gl] * (s[gl] - w["sl"][gl]), w["vu"][gu] * (w["su"][gu] - s[gu])])
    return rd, rs, rp, gaps, c, grad


def ipm_solve(net, tol=1e-4, max_iter=100, relax=1e-4, sigma=0.1, tau=0.99995, delta_c=1e-8, dw_first=1e-4,
              dw_grow=8.0, dw_max=1e10, line_search=True, mu_init=0.1, kappa_eps=10.0, kappa_mu=0.2,
              theta_mu=1.5, tau_min=0.99, gamma_theta=1e-5, gamma_phi=1e-8, eta_phi=1e-8, s_theta=1.1,
              s_phi=2.3, delta=1.0, gamma_alpha=0.05, kappa_sigma=1e10, stall_iter=25, dw_grow_first=100.0,
              dw_shrink=1.0 / 3.0, dw_min=1e-20):
    """Primal-dual interior-point method on the lifted formulation of
    Sec. III-B: the rows c(x) are relaxed to sl <= s <= su with c(x) - s = 0
    (equality rows widened by +-relax), each iteration solves the condensed
    system K dx = rhs (condensed_rhs, the condensed matrix of the Hessian of
    the Lagrangian with lambda = -y, kkt_solve) and recovers the other step
    components (recover_step).  Sec. III-B takes the inertia correction from
    the filter interior-point method of Waechter and Biegler (2006) and says
    that a line search chooses the step length without naming one; the
    reading taken here is that method's filter line search:

    * inertia correction: delta_w = 0, else growing until K is positive
      definite (the condition static pivoting needs) -- without the line
      search from dw_first by dw_grow; with it as in that method: the first
      nonzero try is dw_first when no earlier iteration needed a correction,
      else max(dw_min, dw_shrink * the last one used), growing by
      dw_grow_first while no earlier iteration needed one, else by dw_grow;
    * the Newton step is the negated (dx, ds, dzl, dzu, dvl, dvu) with +dy
      (the condensed system is written for the residuals, not their negative);
    * fraction to the boundary, tau_k = max(tau_min, 1 - mu), one length for
      the primal (x, s) part and one for the bound multipliers;
    * with ``line_search`` (the default): a monotone barrier parameter
      (start mu_init; while the barrier problem's error -- the stopping
      measure with the complementarity products taken minus mu -- is at most
      kappa_eps mu, mu = max(tol / 10, min(kappa_mu mu, mu^theta_mu)) and the
      filter is emptied), and a backtracking line search (halving from the
      fraction-to-the-boundary length) on the barrier function
      phi = f - mu sum ln(distance to each finite bound) and the violation
      theta = |c(x) - s|_1: a trial point must not be dominated by a filter
      entry nor exceed theta_max = 1e4 max(1, theta_0); when phi decreases
      along the step (switching condition alpha (-phi'd)^s_phi >
      delta theta^s_theta) and theta <= theta_min = 1e-4 max(1, theta_0) it
      must satisfy the Armijo condition on phi (eta_phi), otherwise it must
      reduce theta by the factor (1 - gamma_theta) or phi by gamma_phi theta,
      and then (gamma_theta theta, phi - gamma_phi theta) joins the filter.
      The multipliers y move with the accepted primal length; afterwards each
      bound multiplier is kept within [mu / (kappa_sigma gap),
      kappa_sigma mu / gap].  When the length falls below alpha_min (gamma_alpha
      times the smallest length at which a decrease can still be required)
      the loop stops with status "stalled": the method's restoration phase,
      which would look for a less infeasible point, is not implemented, so a
      stall reports the instance as not solved (infeasible or too hard from
      this start).  The same status ends a run whose violation theta has not
      fallen below 0.9 of its best value for stall_iter iterations while
      max |c - s| > tol (steps still accepted, but no progress towards
      feasibility: what would send the method into restoration);
    * an iteration whose inertia correction would need delta_w > dw_max (no
      positive definite condensed matrix found) also ends the loop as
      "stalled", with or without the line search;
    * without ``line_search``: mu = sigma * (mean complementarity product) and
      the fraction-to-the-boundary lengths (tau) are taken as they are; y
      moves with the dual length;
    * stop when max(|p_x| / sd, |p_s| / sd, |c - s|, complementarity) <= tol,
      sd = max(1, mean |multiplier| / 100).

    Returns a dict: the iterate, objective, iterations, factorizations,
    converged, status ("converged", "stalled", "max_iter"), the final
    violation theta, and the per-iteration history (err, mu, delta_w,
    alpha_p, alpha_d, trials)."""
    L = Layout(net)
    n, m = L.n, L.m
    w = ipm_start(net, relax)
    hl, hu, gl, gu = (np.isfinite(w[k]) for k in ("xl", "xu", "sl", "su"))
    hist, nfact = [], 0
    status = "max_iter"
    mu = mu_init
    filt = []
    th0 = _violation(net, w["x"], w["s"])
    theta_max, theta_min = 1e4 * max(1.0, th0), 1e-4 * max(1.0, th0)
    th_best, it_best = th0, 0
    dw_last = 0.0

    for it in range(max_iter + 1):
        rd, rs, rp, gaps, c, grad = ipm_residuals(net, w, 0.0)
        mult = (np.abs(w["y"]).sum() + w["zl"].sum() + w["zu"].sum() + w["vl"].sum() + w["vu"].sum())
        sd = max(1.0, mult / (m + 2 * n) / 100.0)
        base = max(np.abs(rd).max() / sd, np.abs(rs).max() / sd, np.abs(rp).max())
        err = max(base, gaps.max() if gaps.size else 0.0)
        if err <= tol:
            status = "converged"
            break
        if it == max_iter:
            break
        if line_search:
            th = _violation(net, w["x"], w["s"])
            if th < 0.9 * th_best:
                th_best, it_best = th, it
            if stall_iter > 0 and it - it_best >= stall_iter and np.abs(rp).max() > tol:
                status = "stalled"
                break
            while mu > tol / 10.0:
                err_mu = max(base, np.abs(gaps - mu).max() if gaps.size else 0.0)
                if err_mu > kappa_eps * mu:
                    break
                mu = max(tol / 10.0, min(kappa_mu * mu, mu ** theta_mu))
                filt = []
            tau_k = max(tau_min, 1.0 - mu)
        else:
            mu = sigma * gaps.sum() / max(gaps.size, 1)
            tau_k = tau
        jac = jacobian(net, w["x"])
        hess = hessian(net, w["x"], -w["y"], 1.0)
        dw = 0.0
        while True:
            st = synth_state(w, mu, dw, delta_c)
            diag_x, D, rhs = condensed_rhs(net, st, grad, c)
            rp_, ci_, kv_, _ = condensed(n, jac, hess, diag_x, D)
            nfact += 1
            if kkt_is_positive_definite(n, rp_, ci_, kv_):
                break
            if not line_search:
                dw = dw_first if dw == 0.0 else dw * dw_grow
            elif dw == 0.0:
                dw = dw_first if dw_last == 0.0 else max(dw_min, dw_shrink * dw_last)
            else:
                dw *= dw_grow_first if dw_last == 0.0 else dw_grow
            if dw > dw_max:
                break
        if dw > dw_max:
            # no positive definite condensed matrix within dw_max: no step
            hist.append(dict(err=err, mu=mu, delta_w=dw, alpha_p=0.0, alpha_d=0.0, trials=0))
            status = "stalled"
            break
        if line_search and dw > 0.0:
            dw_last = dw
        dx = kkt_solve(n, rp_, ci_, kv_, rhs)
        ds, dy, dzl, dzu, dvl, dvu = recover_step(net, st, c, dx)
        step = dict(x=-dx, s=-ds, y=dy, zl=-dzl, zu=-dzu, vl=-dvl, vu=-dvu)
        ap = min(_max_step(w["x"], step["x"], w["xl"], hl, tau_k, False),
                 _max_step(w["x"], step["x"], w["xu"], hu, tau_k, True),
                 _max_step(w["s"], step["s"], w["sl"], gl, tau_k, False),
                 _max_step(w["s"], step["s"], w["su"], gu, tau_k, True))
        ad = min(_max_step(w[k], step[k], np.zeros(w[k].size), msk, tau_k, False)
                 for k, msk in (("zl", hl), ("zu", hu), ("vl", gl), ("vu", gu)))
        trials, ay = 1, ad
        if line_search:
            ph = _barrier(net, w, w["x"], w["s"], mu)
            dph = _barrier_slope(grad, w, step["x"], step["s"], mu)
            if dph < 0.0:
                amin = gamma_alpha * min(gamma_theta, gamma_phi * th / -dph, delta * th ** s_theta / (-dph) ** s_phi)
            else:
                amin = gamma_alpha * gamma_theta
            a, kind = ap, None
            while True:
                xt, stt = w["x"] + a * step["x"], w["s"] + a * step["s"]
                tht, pht = _violation(net, xt, stt), _barrier(net, w, xt, stt, mu)
                if tht <= theta_max and all(tht < tj or pht < pj for tj, pj in filt):
                    switching = dph < 0.0 and a * (-dph) ** s_phi > delta * th ** s_theta
                    if switching and th <= theta_min:
                        if pht <= ph + eta_phi * a * dph:
                            kind = "f"
                    elif tht <= (1.0 - gamma_theta) * th or pht <= ph - gamma_phi * th:
                        kind = "h"
                if kind is not None:
                    break
                a *= 0.5
                trials += 1
                if a < amin:
                    break
            if kind is None:
                hist.append(dict(err=err, mu=mu, delta_w=dw, alpha_p=0.0, alpha_d=0.0, trials=trials))
                status = "stalled"
                break
            if kind == "h":
                filt.append(((1.0 - gamma_theta) * th, ph - gamma_phi * th))
            ap, ay = a, a
        w = dict(w)
        for k in ("x", "s"):
            w[k] = w[k] + ap * step[k]
        w["y"] = w["y"] + ay * step["y"]
        for k in ("zl", "zu", "vl", "vu"):
            w[k] = w[k] + ad * step[k]
        if line_search:
            _safeguard(w, mu, kappa_sigma)
        hist.append(dict(err=err, mu=mu, delta_w=dw, alpha_p=ap, alpha_d=ad, trials=trials))
    return dict(w=w, x=w["x"], objective=objective(net, w["x"]), iterations=it, factorizations=nfact,
                converged=status == "converged", status=status, err=err,
                theta=_violation(net, w["x"], w["s"]), history=hist)


def _violation(net, x, s):
    """theta = |c(x) - s|_1, the violation the filter measures."""
    return float(np.abs(constraints(net, x) - s).sum())


def _barrier(net, w, x, s, mu):
    """phi_mu = f(x) - mu * (sum of ln(distance to each finite bound)) over
    the variable bounds and the relaxed row bounds."""
    out = objective(net, x)
    for v, key, upper in ((x, "xl", False), (x, "xu", True), (s, "sl", False), (s, "su", True)):
        b = w[key]
        sel = np.isfinite(b)
        gap = (b[sel] - v[sel]) if upper else (v[sel] - b[sel])
        out -= mu * np.log(gap).sum()
    return float(out)


def _barrier_slope(grad, w, px, ps, mu):
    """Directional derivative of phi_mu along the primal step (px, ps)."""
    out = float(np.dot(grad, px))
    for v, p, key, upper in ((w["x"], px, "xl", False), (w["x"], px, "xu", True), (w["s"], ps, "sl", False),
                             (w["s"], ps, "su", True)):
        b = w[key]
        sel = np.isfinite(b)
        gap = (b[sel] - v[sel]) if upper else (v[sel] - b[sel])
        out += mu * (p[sel] / gap).sum() if upper else -mu * (p[sel] / gap).sum()
    return out


def _safeguard(w, mu, kappa_sigma):
    """Keeps every bound multiplier within [mu / (kappa_sigma gap),
    kappa_sigma mu / gap] of its bound's distance (gap)."""
    for z, v, key, upper in (("zl", "x", "xl", False), ("zu", "x", "xu", True), ("vl", "s", "sl", False),
                             ("vu", "s", "su", True)):
        b = w[key]
        sel = np.isfinite(b)
        gap = (b[sel] - w[v][sel]) if upper else (w[v][sel] - b[sel])
        zz = w[z].copy()
        zz[sel] = np.maximum(np.minimum(zz[sel], kappa_sigma * mu / gap), mu / (kappa_sigma * gap))
        w[z] = zz


def _max_step(v, dv, b, mask, tau, upper):
    """Largest alpha <= 1 with v + alpha dv at least (1 - tau) of the way
    from the bound b (fraction to the boundary), over the masked entries."""
    sel = mask & ((dv > 0) if upper else (dv < 0))
    if not sel.any():
        return 1.0
    return float(min(1.0, np.min(tau * (b[sel] - v[sel]) / dv[sel])))


def synth_state(w, mu, delta_w, delta_c):
    """The iterate as the condensation routines take it."""
    from types import SimpleNamespace
    return SimpleNamespace(x=w["x"], s=w["s"], y=w["y"], zl=w["zl"], zu=w["zu"], vl=w["vl"], vu=w["vu"],
                           xl=w["xl"], xu=w["xu"], sl=w["sl"], su=w["su"], mu=mu, delta_w=delta_w, delta_c=delta_c)
