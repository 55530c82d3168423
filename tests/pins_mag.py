"""Brute-force cancellation scales: the per-value magnitude pass of the
oracle pinned against an independent enumeration of each value's terms.

The parity rule compares a device value with the oracle's value within
``tol * max(|ref|, mag)``, where ``mag`` is the sum of the absolute values
of the terms the value is made of.  The terms are fixed here as:

* flows: the complex monomials of the expanded complex power
  S = V conj(Y V) of a pi-model line end (Sec. II, eq. (1d)-(1e) read as
  the pi-model), coef * V_i^a V_j^b e^{j(p theta_i + q theta_j)}, each
  counted by its modulus (the real or imaginary part of a monomial is
  bounded by its modulus); a derivative of a flow is the sum of the
  derivatives of its monomials, each again counted by its modulus;
* every other row, Jacobian entry, Hessian entry and objective term: its
  plain summands (generation, flows and load of a balance row, the two
  angles of an angle row, the two generations of a ramp row, ...);
* products and sums propagate scales (a sum adds them, a product of two
  values multiplies them); a single rounded operation on inputs (a gap
  x - bound, the weights C and D) is an exact atomic input.

This module enumerates those terms one value at a time with plain Python
loops over periods, lines, buses and generators, differentiates the
monomials generically (power rule in V, factor j p in theta), accumulates
the condensed matrix over the pairs of each Jacobian row in a dict, and
evaluates the lifted-KKT formulas of Sec. III-B with a scalar
magnitude-carrying number type.  It shares no code with the oracle.
"""
from __future__ import annotations

import cmath
import math
from collections import defaultdict

import numpy as np


# ----------------------------------------------------------------- layout
class Lay:
    """Canonical per-period offsets (the x / c layout contract)."""

    def __init__(self, net):
        N, B, G, T = net.N, net.B, net.G, net.T
        self.N, self.B, self.G, self.T = N, B, G, T
        self.n_p = 2 * N + 2 * G + 4 * B
        self.m_p = 2 * N + 7 * B + 1
        self.n = T * self.n_p
        self.m = T * self.m_p + G * (T - 1)

    def vm(self, t, i):
        return t * self.n_p + i

    def va(self, t, i):
        return t * self.n_p + self.N + i

    def pg(self, t, g):
        return t * self.n_p + 2 * self.N + g

    def qg(self, t, g):
        return t * self.n_p + 2 * self.N + self.G + g

    def flow(self, t, k, l):
        return t * self.n_p + 2 * self.N + 2 * self.G + k * self.B + l

    def bal(self, t, q, i):  # q = 0 active, 1 reactive
        return t * self.m_p + q * self.N + i

    def ref(self, t):
        return t * self.m_p + 2 * self.N

    def cflow(self, t, k, l):
        return t * self.m_p + 2 * self.N + 1 + k * self.B + l

    def th(self, t, e, l):  # e = 0 from end, 1 to end
        return t * self.m_p + 2 * self.N + 1 + (4 + e) * self.B + l

    def ang(self, t, l):
        return t * self.m_p + 2 * self.N + 1 + 6 * self.B + l

    def ramp(self, t, g):
        return self.T * self.m_p + (t - 1) * self.G + g


# ------------------------------------------------------- monomial calculus
def line_admittances(net, l):
    """Pi-model of one line: series y = 1/(r + jx), half the charging at
    each end, an ideal transformer tau e^{j phi} on the from side."""
    y = 1.0 / complex(net.r[l], net.x[l])
    sh = 0.5j * net.b_charge[l]
    a = net.tap[l] * cmath.exp(1j * net.shift[l])
    return (y + sh) / (abs(a) ** 2), -y / a.conjugate(), -y / a, y + sh


def end_monomials(net, l):
    """Monomials (coef, a, b, p, q) of S = coef V_i^a V_j^b e^{j(p th_i + q th_j)}
    for the power entering line l at its from end (S_f = V_f conj(I_f),
    I_f = Y_ff V_f + Y_ft V_t) and at its to end (S_t = V_t conj(I_t),
    I_t = Y_tf V_f + Y_tt V_t)."""
    yff, yft, ytf, ytt = line_admittances(net, l)
    sf = [(yff.conjugate(), 2, 0, 0, 0), (yft.conjugate(), 1, 1, 1, -1)]
    st = [(ytt.conjugate(), 0, 2, 0, 0), (ytf.conjugate(), 1, 1, -1, 1)]
    return sf, st


def mono_d(m, var):
    """Derivative of a monomial by local variable var (0 vm_i, 1 vm_j,
    2 va_i, 3 va_j); None when it vanishes identically."""
    c, a, b, p, q = m
    if var == 0:
        return (c * a, a - 1, b, p, q) if a else None
    if var == 1:
        return (c * b, a, b - 1, p, q) if b else None
    if var == 2:
        return (c * 1j * p, a, b, p, q) if p else None
    return (c * 1j * q, a, b, p, q) if q else None


def mono_val(m, vi, vj, ti, tj):
    c, a, b, p, q = m
    return c * vi ** a * vj ** b * cmath.exp(1j * (p * ti + q * tj))


def sum_terms(monos, vi, vj, ti, tj):
    """(complex value, sum of moduli) of a list of monomials."""
    val, mag = 0j, 0.0
    for m in monos:
        if m is None:
            continue
        z = mono_val(m, vi, vj, ti, tj)
        val += z
        mag += abs(z)
    return val, mag


def part(z, k):
    return z.real if k % 2 == 0 else z.imag


# ---------------------------------------------------------- model terms
def model_terms(net, x, lam, sigma):
    """Every value of the evaluation with its brute-force scale.

    Returns dict with
      'f': (value, mag), 'grad': (values[n], mags[n]), 'c': (values[m], mags[m]),
      'J': {(row, col): [value, mag]}, 'H': {(row, col): [value, mag]} (lower,
      summed over duplicates)."""
    L = Lay(net)
    x = np.asarray(x, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    cval = np.zeros(L.m)
    cmag = np.zeros(L.m)
    J = defaultdict(lambda: [0.0, 0.0])
    H = defaultdict(lambda: [0.0, 0.0])
    grad = np.zeros(L.n)
    gmag = np.zeros(L.n)
    fval, fmag = 0.0, 0.0

    def jput(r, c, v, mg):
        J[(r, c)][0] += v
        J[(r, c)][1] += mg

    def hput(a, b, v, mg):
        key = (max(a, b), min(a, b))
        H[key][0] += v
        H[key][1] += mg

    def cput(r, terms):
        cval[r] += sum(terms)
        cmag[r] += sum(abs(v) for v in terms)

    monos = [end_monomials(net, l) for l in range(net.B)]
    for t in range(net.T):
        # objective, gradient, objective Hessian
        for g in range(net.G):
            p = x[L.pg(t, g)]
            terms = (net.c2[g] * p * p, net.c1[g] * p, net.c0[g])
            fval += sum(terms)
            fmag += sum(abs(v) for v in terms)
            grad[L.pg(t, g)] = 2.0 * net.c2[g] * p + net.c1[g]
            gmag[L.pg(t, g)] = abs(2.0 * net.c2[g] * p) + abs(net.c1[g])
            hput(L.pg(t, g), L.pg(t, g), 2.0 * sigma * net.c2[g], abs(2.0 * sigma * net.c2[g]))
        # balance rows: generation - flows leaving - load
        for i in range(net.N):
            for q in range(2):
                terms = [-(net.pd[t, i] if q == 0 else net.qd[t, i])]
                for g in range(net.G):
                    if net.gen_bus[g] == i:
                        col = L.pg(t, g) if q == 0 else L.qg(t, g)
                        terms.append(x[col])
                        jput(L.bal(t, q, i), col, 1.0, 1.0)
                for l in range(net.B):
                    for e, bus in ((0, net.f_bus[l]), (1, net.t_bus[l])):
                        if bus == i:
                            col = L.flow(t, 2 * e + q, l)
                            terms.append(-x[col])
                            jput(L.bal(t, q, i), col, -1.0, 1.0)
                cput(L.bal(t, q, i), terms)
        # reference angle
        cput(L.ref(t), [x[L.va(t, net.ref_bus)]])
        jput(L.ref(t), L.va(t, net.ref_bus), 1.0, 1.0)
        # lines
        for l in range(net.B):
            i, j = int(net.f_bus[l]), int(net.t_bus[l])
            vi, vj = x[L.vm(t, i)], x[L.vm(t, j)]
            ti, tj = x[L.va(t, i)], x[L.va(t, j)]
            cols = [L.vm(t, i), L.vm(t, j), L.va(t, i), L.va(t, j)]
            for k in range(4):
                ms = monos[l][0] if k < 2 else monos[l][1]
                row = L.cflow(t, k, l)
                xf = x[L.flow(t, k, l)]
                z, zm = sum_terms(ms, vi, vj, ti, tj)
                cval[row] = xf - part(z, k)
                cmag[row] = abs(xf) + zm
                jput(row, L.flow(t, k, l), 1.0, 1.0)
                lk = lam[row]
                for a in range(4):
                    d1 = [mono_d(m, a) for m in ms]
                    dz, dm = sum_terms(d1, vi, vj, ti, tj)
                    jput(row, cols[a], -part(dz, k), dm)
                    for b in range(a + 1):
                        d2 = [mono_d(m, b) if m is not None else None for m in d1]
                        hz, hm = sum_terms(d2, vi, vj, ti, tj)
                        if hm == 0.0:
                            continue  # identically zero: not a term
                        hput(cols[a], cols[b], -lk * part(hz, k), abs(lk) * hm)
            # thermal, both ends
            for e in range(2):
                fp, fq = x[L.flow(t, 2 * e, l)], x[L.flow(t, 2 * e + 1, l)]
                row = L.th(t, e, l)
                cput(row, [fp * fp, fq * fq])
                for kk, fv in ((2 * e, fp), (2 * e + 1, fq)):
                    jput(row, L.flow(t, kk, l), 2.0 * fv, abs(2.0 * fv))
                    hput(L.flow(t, kk, l), L.flow(t, kk, l), 2.0 * lam[row], abs(2.0 * lam[row]))
            # angle difference
            row = L.ang(t, l)
            cput(row, [ti, -tj])
            jput(row, L.va(t, i), 1.0, 1.0)
            jput(row, L.va(t, j), -1.0, 1.0)
        # ramp rows
        if t >= 1:
            for g in range(net.G):
                row = L.ramp(t, g)
                cput(row, [x[L.pg(t, g)], -x[L.pg(t - 1, g)]])
                jput(row, L.pg(t, g), 1.0, 1.0)
                jput(row, L.pg(t - 1, g), -1.0, 1.0)
    return dict(f=(fval, fmag), grad=(grad, gmag), c=(cval, cmag), J=dict(J), H=dict(H))


def jt_terms(J, v, n):
    """J^T v term by term: out[c] = sum_r J[r, c] v[r], scale sum_r m(J[r, c]) |v[r]|."""
    out = np.zeros(n)
    mag = np.zeros(n)
    for (r, c), (val, mg) in J.items():
        out[c] += val * v[r]
        mag[c] += mg * abs(v[r])
    return out, mag


def j_terms(J, u, m):
    """J u term by term, with its scale."""
    out = np.zeros(m)
    mag = np.zeros(m)
    for (r, c), (val, mg) in J.items():
        out[r] += val * u[c]
        mag[r] += mg * abs(u[c])
    return out, mag


def kkt_terms(J, H, diag_x, dcon, n):
    """lower(H + diag(diag_x) + J^T diag(dcon) J) slot by slot, accumulated
    in a dict over the pairs of entries of every Jacobian row (each
    unordered pair once, an entry with itself once)."""
    K = defaultdict(lambda: [0.0, 0.0])
    rows = defaultdict(list)
    for (r, c), (val, mg) in J.items():
        rows[r].append((c, val, mg))
    for r, ents in rows.items():
        for a in range(len(ents)):
            for b in range(a + 1):
                ca, va_, ma = ents[a]
                cb, vb, mb = ents[b]
                key = (max(ca, cb), min(ca, cb))
                K[key][0] += dcon[r] * va_ * vb
                K[key][1] += abs(dcon[r]) * ma * mb
    for key, (val, mg) in H.items():
        K[key][0] += val
        K[key][1] += mg
    for i in range(n):
        dx = 0.0 if diag_x is None else diag_x[i]
        K[(i, i)][0] += dx
        K[(i, i)][1] += abs(dx)
    return dict(K)


# --------------------------------------------- lifted-KKT formulas (III-B)
class MF:
    """A scalar carrying its value and its cancellation scale."""

    __slots__ = ("v", "m")

    def __init__(self, v, m=None):
        self.v = float(v)
        self.m = abs(self.v) if m is None else float(m)

    def __add__(self, o):
        o = o if isinstance(o, MF) else MF(o)
        return MF(self.v + o.v, self.m + o.m)

    __radd__ = __add__

    def __sub__(self, o):
        o = o if isinstance(o, MF) else MF(o)
        return MF(self.v - o.v, self.m + o.m)

    def __rsub__(self, o):
        return MF(o) - self

    def __neg__(self):
        return MF(-self.v, self.m)

    def __mul__(self, o):
        o = o if isinstance(o, MF) else MF(o)
        return MF(self.v * o.v, self.m * o.m)

    __rmul__ = __mul__

    def __truediv__(self, o):
        # division by an exact (atomic) quantity
        o = float(o.v if isinstance(o, MF) else o)
        return MF(self.v / o, self.m / abs(o))


def lifted_terms(net, st, grad, c, J, dx=None):
    """Condensed right-hand side rhs = q_x + A^T (C q_s + D q_y) and, when dx
    is given, the recovered steps (ds, dy, dzl, dzu, dvl, dvu), entry by
    entry in magnitude-carrying arithmetic, following the definitions of
    Sec. III-B (the slack step with the sign that solves the full system;
    each bound residual on its own bound; absent bounds contribute nothing).
    Gaps x - bound and the weights C, D are atomic inputs."""
    n, m = len(st.x), len(st.s)
    mu = st.mu
    rows_of = defaultdict(list)
    cols_of = defaultdict(list)
    for (r, cc), (val, mg) in J.items():
        rows_of[cc].append((r, MF(val, mg)))
        cols_of[r].append((cc, MF(val, mg)))

    def box(val, lo, hi, zlo, zhi):
        hl, hh = math.isfinite(lo), math.isfinite(hi)
        glo = val - lo if hl else None
        ghi = hi - val if hh else None
        sig = (zlo / glo if hl else 0.0) + (zhi / ghi if hh else 0.0)
        plo = MF(zlo) * MF(glo) - MF(mu) if hl else None
        phi = MF(zhi) * MF(ghi) - MF(mu) if hh else None
        return hl, hh, glo, ghi, sig, plo, phi

    # row quantities
    qs, py, Cw, Dw, rowbox = [], [], [], [], []
    for r in range(m):
        hl, hh, glo, ghi, sig, plo, phi = box(st.s[r], st.sl[r], st.su[r], st.vl[r], st.vu[r])
        ps = MF(st.y[r])
        if hl:
            ps = ps - MF(st.vl[r])
        if hh:
            ps = ps + MF(st.vu[r])
        q = ps
        if hl:
            q = q + plo / glo
        if hh:
            q = q - phi / ghi
        qs.append(q)
        py.append(MF(c[r]) - MF(st.s[r]))
        Cr = 1.0 / (st.delta_c * sig + (1.0 + st.delta_c * st.delta_w))
        Cw.append(Cr)
        Dw.append((sig + st.delta_w) * Cr)
        rowbox.append((hl, hh, glo, ghi, sig, plo, phi))
    w = [MF(Cw[r]) * qs[r] + MF(Dw[r]) * py[r] for r in range(m)]
    rhs = []
    xbox = []
    for i in range(n):
        hl, hh, glo, ghi, sig, plo, phi = box(st.x[i], st.xl[i], st.xu[i], st.zl[i], st.zu[i])
        xbox.append((hl, hh, glo, ghi, plo, phi))
        acc = MF(grad[i])
        for r, a in rows_of[i]:
            acc = acc - a * MF(st.y[r])
        if hl:
            acc = acc - MF(st.zl[i]) + plo / glo
        if hh:
            acc = acc + MF(st.zu[i]) - phi / ghi
        for r, a in rows_of[i]:
            acc = acc + a * w[r]
        rhs.append(acc)
    out = dict(rhs=rhs)
    if dx is None:
        return out
    ds, dy, dvl, dvu = [], [], [], []
    for r in range(m):
        hl, hh, glo, ghi, sig, plo, phi = rowbox[r]
        adx = MF(0.0, 0.0)
        for cc, a in cols_of[r]:
            adx = adx + a * MF(dx[cc])
        d = MF(Cw[r]) * (adx + MF(st.delta_c) * qs[r] - py[r])
        ds.append(d)
        dy.append(MF(sig + st.delta_w) * d - qs[r])
        dvl.append((-(MF(st.vl[r]) * d) + plo) / glo if hl else MF(0.0))
        dvu.append((MF(st.vu[r]) * d + phi) / ghi if hh else MF(0.0))
    dzl, dzu = [], []
    for i in range(n):
        hl, hh, glo, ghi, plo, phi = xbox[i]
        dzl.append((-(MF(st.zl[i]) * MF(dx[i])) + plo) / glo if hl else MF(0.0))
        dzu.append((MF(st.zu[i]) * MF(dx[i]) + phi) / ghi if hh else MF(0.0))
    out.update(ds=ds, dy=dy, dzl=dzl, dzu=dzu, dvl=dvl, dvu=dvu)
    return out


def split(mfs):
    return np.array([a.v for a in mfs]), np.array([a.m for a in mfs])
