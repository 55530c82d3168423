// Symbolic analysis of the condensed matrix for the static-pivot sparse
// Cholesky factorization (Sec. III-B: after inertia correction the condensed
// matrix is positive definite, so a Cholesky factorization without numerical
// pivoting, with static pivot replacement, applies).
//
// Structure exploited: K is block tridiagonal in time.  A period block
// couples to its neighbours only through the ramp rows (eq. (1k)), i.e. only
// through the pg variables, one (pg_t,g , pg_{t-1},g) entry per generator.
// Every period block has the same pattern.  So:
//   * one ordering of a period's variables serves all periods: the interior
//     (every variable except pg) by a constrained approximate minimum degree
//     ordering, the G pg variables last in their natural order;
//   * the interior factorization of all periods is one multifrontal tree,
//     evaluated batched over periods;
//   * the pg variables of period t form one dense front of G pivots whose
//     update rows are pg_{t+1}: a chain over t (block elimination in time).
//
// Pure C++ (no HIP), also usable for a host-only model.
#include "opf_chol_host.h"

#include <algorithm>
#include <cstring>
#include <numeric>
#include <queue>

namespace opf {

namespace {

// ------------------------------------------------------------------ AMD
// Approximate minimum degree on a quotient graph (variables and elements,
// supervariables, element absorption, approximate external degrees), with
// one constraint class deferred to the end.  Produces the assembly tree of
// the elimination directly: every eliminated pivot supervariable is a node
// whose update rows are the variables of its element at that moment.
struct AmdResult {
  // nodes in elimination order: pivot members, update rows (original
  // indices), children (node ids)
  std::vector<std::vector<int32_t>> piv, rows, kids;
  int32_t root = -1;  // the deferred-class node (last)
};

enum : int8_t { kVar = 0, kElem = 1, kAbsorbed = 2, kMerged = 3 };

AmdResult constrained_amd(int32_t n, const std::vector<int32_t>& xadj, const std::vector<int32_t>& adj,
                          const std::vector<int8_t>& deferred) {
  std::vector<std::vector<int32_t>> adjV(n), adjE(n), Le(n), mem(n);
  std::vector<int32_t> nv(n, 1), deg(n), esize(n, 0), node_of(n, -1);
  std::vector<int8_t> status(n, kVar);
  std::vector<int64_t> mark(n, 0), wmark(n, 0);
  std::vector<int64_t> w(n, 0);
  int64_t stamp = 0;
  for (int32_t i = 0; i < n; ++i) {
    adjV[i].assign(adj.begin() + xadj[i], adj.begin() + xadj[i + 1]);
    mem[i].push_back(i);
    deg[i] = (int32_t)adjV[i].size();
  }
  using QE = std::pair<int32_t, int32_t>;
  std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
  int32_t n_int = 0;
  for (int32_t i = 0; i < n; ++i)
    if (!deferred[i]) {
      pq.push({deg[i], i});
      ++n_int;
    }
  AmdResult R;
  int64_t nremain = n;
  int32_t elim_int = 0;
  std::vector<int32_t> Lp, kids;
  while (elim_int < n_int) {
    const QE top = pq.top();
    pq.pop();
    const int32_t p = top.second;
    if (status[p] != kVar || nv[p] == 0 || top.first != deg[p]) continue;
    // the pivot's element: union of its elements' variables and its own
    // variable neighbours
    ++stamp;
    mark[p] = stamp;
    Lp.clear();
    kids.clear();
    for (int32_t e : adjE[p]) {
      if (status[e] != kElem) continue;
      for (int32_t j : Le[e])
        if (status[j] == kVar && mark[j] != stamp) {
          mark[j] = stamp;
          Lp.push_back(j);
        }
      status[e] = kAbsorbed;
      kids.push_back(node_of[e]);
      Le[e].clear();
      Le[e].shrink_to_fit();
    }
    for (int32_t j : adjV[p])
      if (status[j] == kVar && mark[j] != stamp) {
        mark[j] = stamp;
        Lp.push_back(j);
      }
    status[p] = kElem;
    adjV[p].clear();
    adjV[p].shrink_to_fit();
    adjE[p].clear();
    adjE[p].shrink_to_fit();
    nremain -= nv[p];
    elim_int += nv[p];
    // prune the lists of the element's variables
    for (int32_t i : Lp) {
      auto& E = adjE[i];
      size_t k = 0;
      for (int32_t e : E)
        if (status[e] == kElem && e != p) E[k++] = e;
      E.resize(k);
      E.push_back(p);
      auto& V = adjV[i];
      k = 0;
      for (int32_t j : V)
        if (status[j] == kVar && mark[j] != stamp) V[k++] = j;
      V.resize(k);
    }
    // supervariables: variables of the element with identical lists (and
    // the same constraint class) become one
    {
      std::vector<std::pair<uint64_t, int32_t>> hs;
      hs.reserve(Lp.size());
      for (int32_t i : Lp) {
        auto& V = adjV[i];
        auto& E = adjE[i];
        std::sort(V.begin(), V.end());
        std::sort(E.begin(), E.end());
        uint64_t h = (uint64_t)deferred[i] * 0x9E3779B97F4A7C15ull + V.size() * 31 + E.size() * 131;
        for (int32_t j : V) h += (uint64_t)j * 2654435761ull;
        for (int32_t e : E) h += (uint64_t)e * 40503ull + 7;
        hs.push_back({h, i});
      }
      std::sort(hs.begin(), hs.end());
      for (size_t a = 0; a < hs.size();) {
        size_t b = a + 1;
        while (b < hs.size() && hs[b].first == hs[a].first) ++b;
        for (size_t x = a; x < b; ++x) {
          const int32_t i = hs[x].second;
          if (status[i] != kVar) continue;
          for (size_t y = x + 1; y < b; ++y) {
            const int32_t j = hs[y].second;
            if (status[j] != kVar || deferred[i] != deferred[j]) continue;
            if (adjV[i] != adjV[j] || adjE[i] != adjE[j]) continue;
            nv[i] += nv[j];
            nv[j] = 0;
            status[j] = kMerged;
            mem[i].insert(mem[i].end(), mem[j].begin(), mem[j].end());
            mem[j].clear();
            mem[j].shrink_to_fit();
            adjV[j].clear();
            adjV[j].shrink_to_fit();
            adjE[j].clear();
            adjE[j].shrink_to_fit();
          }
        }
        a = b;
      }
      size_t k = 0;
      for (int32_t i : Lp)
        if (status[i] == kVar) Lp[k++] = i;
      Lp.resize(k);
    }
    Le[p] = Lp;
    int64_t lpw = 0;
    for (int32_t i : Lp) lpw += nv[i];
    esize[p] = (int32_t)lpw;
    // |Le \ Lp| for the other elements next to the element's variables
    for (int32_t i : Lp)
      for (int32_t e : adjE[i]) {
        if (e == p) continue;
        if (wmark[e] != stamp) {
          wmark[e] = stamp;
          w[e] = esize[e];
        }
        w[e] -= nv[i];
      }
    // aggressive absorption of elements inside Lp
    for (int32_t i : Lp)
      for (int32_t e : adjE[i])
        if (e != p && wmark[e] == stamp && w[e] == 0 && status[e] == kElem) {
          status[e] = kAbsorbed;
          kids.push_back(node_of[e]);
          Le[e].clear();
          Le[e].shrink_to_fit();
        }
    // approximate external degrees
    for (int32_t i : Lp) {
      int64_t ext = 0;
      for (int32_t j : adjV[i]) ext += nv[j];
      int64_t se = 0;
      for (int32_t e : adjE[i])
        if (e != p && status[e] == kElem) se += w[e];
      const int64_t lex = lpw - nv[i];
      int64_t d = std::min<int64_t>((int64_t)deg[i] + lex, ext + lex + se);
      d = std::min<int64_t>(d, nremain - nv[i]);
      deg[i] = (int32_t)std::max<int64_t>(d, 0);
      if (!deferred[i]) pq.push({deg[i], i});
    }
    // the node
    node_of[p] = (int32_t)R.piv.size();
    R.piv.push_back(mem[p]);
    std::vector<int32_t> rows;
    rows.reserve(lpw);
    for (int32_t i : Lp) rows.insert(rows.end(), mem[i].begin(), mem[i].end());
    R.rows.push_back(std::move(rows));
    R.kids.push_back(kids);
  }
  // the deferred class: one root node in natural order; its children are
  // the elements still alive
  std::vector<int32_t> piv;
  for (int32_t i = 0; i < n; ++i)
    if (deferred[i]) piv.push_back(i);
  kids.clear();
  for (int32_t i = 0; i < n; ++i)
    if (status[i] == kElem) kids.push_back(node_of[i]);
  R.root = (int32_t)R.piv.size();
  R.piv.push_back(piv);
  R.rows.emplace_back();
  R.kids.push_back(kids);
  return R;
}

}  // namespace

// ------------------------------------------------------------------ plan
int chol_plan_build(const InstHost& I, const CholOptions& opt, CholPlan& P, std::string& err) {
  const int32_t np = (int32_t)I.n_p;
  const int32_t PG = 2 * I.N, G = I.G;
  P = CholPlan();
  P.n_p = np;
  P.G = G;
  P.T = I.T;
  P.n_int = np - G;
  // period graph from the K template (lower CSR over local rows)
  std::vector<int32_t> cnt(np + 1, 0);
  for (int32_t r = 0; r < np; ++r)
    for (int32_t q = I.krow[r]; q < I.krow[r + 1]; ++q) {
      const int32_t c = I.kcol[q];
      if (c == r) continue;
      ++cnt[r + 1];
      ++cnt[c + 1];
    }
  std::vector<int32_t> xadj(np + 1, 0);
  for (int32_t i = 0; i < np; ++i) xadj[i + 1] = xadj[i] + cnt[i + 1];
  std::vector<int32_t> adj(xadj[np]), fillp(xadj.begin(), xadj.end() - 1);
  for (int32_t r = 0; r < np; ++r)
    for (int32_t q = I.krow[r]; q < I.krow[r + 1]; ++q) {
      const int32_t c = I.kcol[q];
      if (c == r) continue;
      adj[fillp[r]++] = c;
      adj[fillp[c]++] = r;
    }
  std::vector<int8_t> deferred(np, 0);
  for (int32_t g = 0; g < G; ++g) deferred[PG + g] = 1;
  AmdResult A = constrained_amd(np, xadj, adj, deferred);
  const int32_t nn = (int32_t)A.piv.size();
  // postorder from the root (children in elimination order)
  std::vector<int32_t> post;
  post.reserve(nn);
  {
    std::vector<std::pair<int32_t, size_t>> st;
    st.push_back({A.root, 0});
    while (!st.empty()) {
      auto& top = st.back();
      if (top.second < A.kids[top.first].size()) {
        const int32_t c = A.kids[top.first][top.second++];
        st.push_back({c, 0});
      } else {
        post.push_back(top.first);
        st.pop_back();
      }
    }
  }
  if ((int32_t)post.size() != nn) {
    err = "chol analysis: assembly tree does not span every node";
    return OPF_EINVAL;
  }
  // new numbering: pivots in postorder
  P.perm.assign(np, -1);
  P.iperm.assign(np, -1);
  {
    int32_t k = 0;
    for (int32_t s : post)
      for (int32_t v : A.piv[s]) {
        P.perm[k] = v;
        P.iperm[v] = k;
        ++k;
      }
    if (k != np) {
      err = "chol analysis: ordering is not a permutation";
      return OPF_EINVAL;
    }
  }
  // nodes in postorder (root excluded), rows renumbered and sorted
  std::vector<int32_t> pos_of(nn, -1);
  for (int32_t k = 0; k < nn; ++k) pos_of[post[k]] = k;
  struct Nd {
    int32_t f, p, parent;
    std::vector<int32_t> rows;
    std::vector<int32_t> kids;
    bool alive;
    int64_t zeros;  // explicit zeros its factor block carries after merges
  };
  std::vector<Nd> nd(nn - 1);
  for (int32_t k = 0; k + 1 < nn; ++k) {
    const int32_t s = post[k];
    Nd& d = nd[k];
    d.f = P.iperm[A.piv[s][0]];
    d.p = (int32_t)A.piv[s].size();
    for (int32_t v : A.piv[s]) d.f = std::min(d.f, P.iperm[v]);
    d.rows.reserve(A.rows[s].size());
    for (int32_t v : A.rows[s]) d.rows.push_back(P.iperm[v]);
    std::sort(d.rows.begin(), d.rows.end());
    d.parent = -1;
    d.alive = true;
    d.zeros = 0;
  }
  for (int32_t k = 0; k < nn; ++k)
    for (int32_t c : A.kids[post[k]]) {
      const int32_t kc = pos_of[c];
      if (k + 1 < nn) {
        nd[kc].parent = k;
        nd[k].kids.push_back(kc);
      } else {
        nd[kc].parent = -1;  // child of the pg front
      }
    }
  for (auto& d : nd) std::sort(d.kids.begin(), d.kids.end());
  // relaxed amalgamation: fold children into a node while the merged front
  // stays nearly dense.  Any child qualifies (the one with the largest
  // update matrix first: merging it saves the most traffic), not only the
  // one whose pivots directly precede the node's: the merged node's pivots
  // are laid out contiguously afterwards, by a new elimination order.  The
  // test: c's rows lie in s's front, so c's columns in the merged front
  // carry c.p * (s.p + us - uc) zeros.
  std::vector<std::vector<std::pair<int32_t, int32_t>>> rng(nn - 1);  // pivot ranges (first, count)
  for (int32_t k = 0; k + 1 < nn; ++k) rng[k].push_back({nd[k].f, nd[k].p});
  for (int32_t k = 0; k + 1 < nn; ++k) {
    Nd& s = nd[k];
    for (;;) {
      int32_t best = -1;
      int64_t best_u = -1, best_z = 0;
      const int64_t us = (int64_t)s.rows.size();
      for (int32_t kc : s.kids) {
        const Nd& c = nd[kc];
        const int64_t uc = (int64_t)c.rows.size();
        const int64_t added = (int64_t)c.p * ((int64_t)s.p + us - uc);
        const int64_t pm = (int64_t)c.p + s.p;
        if (pm > opt.max_pivots) continue;
        const int64_t tot = pm * (pm + 1) / 2 + pm * us;
        const int64_t zeros = added + c.zeros + s.zeros;
        const bool small = pm <= opt.amalg_small;
        if (!(added == 0 || (small && zeros <= tot / 2) || zeros <= (int64_t)(opt.amalg_frac * tot))) continue;
        if (uc > best_u) {
          best = kc;
          best_u = uc;
          best_z = zeros;
        }
      }
      if (best < 0) break;
      Nd& c = nd[best];
      s.p += c.p;
      s.zeros = best_z;
      rng[k].insert(rng[k].begin(), rng[best].begin(), rng[best].end());  // the child's pivots first
      rng[best].clear();
      s.kids.erase(std::find(s.kids.begin(), s.kids.end(), best));
      s.kids.insert(s.kids.end(), c.kids.begin(), c.kids.end());
      std::sort(s.kids.begin(), s.kids.end());
      for (int32_t g : c.kids) nd[g].parent = k;
      c.alive = false;
      c.kids.clear();
      c.rows.clear();
      c.rows.shrink_to_fit();
    }
  }
  // the surviving nodes keep the postorder's relative order (children
  // before parents); each takes the next block of elimination positions for
  // its pivots, and the ordering and every row index are renumbered to match
  std::vector<int32_t> newid(nn - 1, -1), order2;
  order2.reserve(P.n_int);
  int32_t ns = 0;
  for (int32_t k = 0; k + 1 < nn; ++k) {
    if (!nd[k].alive) continue;
    newid[k] = ns++;
    nd[k].f = (int32_t)order2.size();
    for (const auto& r : rng[k])
      for (int32_t i = r.first; i < r.first + r.second; ++i) order2.push_back(i);
  }
  if ((int32_t)order2.size() != P.n_int) {
    err = "chol analysis: merged pivots do not cover the interior";
    return OPF_EINVAL;
  }
  {
    std::vector<int32_t> map_new(P.n_int, -1);
    for (int32_t i = 0; i < P.n_int; ++i) map_new[order2[i]] = i;
    std::vector<int32_t> perm2(np), iperm2(np, -1);
    for (int32_t i = 0; i < np; ++i) perm2[i] = i < P.n_int ? P.perm[order2[i]] : P.perm[i];
    for (int32_t i = 0; i < np; ++i) iperm2[perm2[i]] = i;
    P.perm.swap(perm2);
    P.iperm.swap(iperm2);
    for (int32_t k = 0; k + 1 < nn; ++k) {
      if (!nd[k].alive) continue;
      for (int32_t& r : nd[k].rows)
        if (r < P.n_int) r = map_new[r];
      std::sort(nd[k].rows.begin(), nd[k].rows.end());
    }
  }
  P.node_f.resize(ns);
  P.node_p.resize(ns);
  P.node_u.resize(ns);
  P.node_parent.resize(ns);
  P.row_ptr.assign(ns + 1, 0);
  for (int32_t k = 0, s = 0; k + 1 < nn; ++k) {
    if (!nd[k].alive) continue;
    P.node_f[s] = nd[k].f;
    P.node_p[s] = nd[k].p;
    P.node_u[s] = (int32_t)nd[k].rows.size();
    P.node_parent[s] = nd[k].parent < 0 ? -1 : newid[nd[k].parent];
    P.row_ptr[s + 1] = P.row_ptr[s] + (int64_t)nd[k].rows.size();
    ++s;
  }
  P.rows.resize(P.row_ptr[ns]);
  for (int32_t k = 0, s = 0; k + 1 < nn; ++k) {
    if (!nd[k].alive) continue;
    std::copy(nd[k].rows.begin(), nd[k].rows.end(), P.rows.begin() + P.row_ptr[s]);
    ++s;
  }
  P.nnodes = ns;
  // checks: pivots contiguous and covering the interior, rows after the
  // pivots, a parent's front holding every row of its child
  {
    int32_t expect = 0;
    for (int32_t s = 0; s < ns; ++s) {
      if (P.node_f[s] != expect) {
        err = "chol analysis: node pivots not contiguous";
        return OPF_EINVAL;
      }
      expect += P.node_p[s];
      const int32_t* r = P.rows.data() + P.row_ptr[s];
      for (int32_t a = 0; a < P.node_u[s]; ++a)
        if (r[a] < P.node_f[s] + P.node_p[s] || (a > 0 && r[a] <= r[a - 1])) {
          err = "chol analysis: bad node row structure";
          return OPF_EINVAL;
        }
    }
    if (expect != P.n_int) {
      err = "chol analysis: interior pivots do not cover the interior";
      return OPF_EINVAL;
    }
  }
  // relative positions of every node's rows in its parent's front (the pg
  // front of the period for a tree root: position = row - n_int)
  P.rel.resize(P.rows.size());
  for (int32_t s = 0; s < ns; ++s) {
    const int32_t* r = P.rows.data() + P.row_ptr[s];
    int32_t* out = P.rel.data() + P.row_ptr[s];
    const int32_t par = P.node_parent[s];
    if (par < 0) {
      for (int32_t a = 0; a < P.node_u[s]; ++a) {
        if (r[a] < P.n_int) {
          err = "chol analysis: tree root with an interior update row";
          return OPF_EINVAL;
        }
        out[a] = r[a] - P.n_int;
      }
      continue;
    }
    const int32_t pf = P.node_f[par], pp = P.node_p[par];
    const int32_t* pr = P.rows.data() + P.row_ptr[par];
    const int32_t pu = P.node_u[par];
    for (int32_t a = 0; a < P.node_u[s]; ++a) {
      if (r[a] >= pf && r[a] < pf + pp) {
        out[a] = r[a] - pf;
      } else {
        const int32_t* it = std::lower_bound(pr, pr + pu, r[a]);
        if (it == pr + pu || *it != r[a]) {
          err = "chol analysis: child row missing from its parent's front";
          return OPF_EINVAL;
        }
        out[a] = pp + (int32_t)(it - pr);
      }
    }
  }
  // children lists and levels (height above the leaves)
  P.kid_ptr.assign(ns + 1, 0);
  std::vector<int32_t> nk(ns, 0), roots;
  for (int32_t s = 0; s < ns; ++s)
    if (P.node_parent[s] >= 0) ++nk[P.node_parent[s]];
    else roots.push_back(s);
  for (int32_t s = 0; s < ns; ++s) P.kid_ptr[s + 1] = P.kid_ptr[s] + nk[s];
  P.kids.resize(P.kid_ptr[ns]);
  {
    std::vector<int64_t> fp(P.kid_ptr.begin(), P.kid_ptr.end() - 1);
    for (int32_t s = 0; s < ns; ++s)
      if (P.node_parent[s] >= 0) P.kids[fp[P.node_parent[s]]++] = s;
  }
  P.roots = roots;
  P.node_level.assign(ns, 0);
  int32_t H = 0;
  for (int32_t s = 0; s < ns; ++s) {  // postorder: children first
    int32_t h = 0;
    for (int64_t q = P.kid_ptr[s]; q < P.kid_ptr[s + 1]; ++q) h = std::max(h, P.node_level[P.kids[q]] + 1);
    P.node_level[s] = h;
    H = std::max(H, h + 1);
  }
  P.nlevels = H;
  // per-period storage of the interior factor: node s's (p+u) x p block,
  // column-major
  P.node_loff.resize(ns);
  int64_t off = 0;
  double fl = 0.0;
  for (int32_t s = 0; s < ns; ++s) {
    P.node_loff[s] = off;
    const int64_t p = P.node_p[s], u = P.node_u[s];
    off += (p + u) * p;
    // sum over the front's columns of (entries below the diagonal)^2, i.e.
    // two flops per multiply-add of the elimination
    fl += (double)p * p * p / 3.0 + (double)p * p * u + (double)p * u * u;
  }
  P.lsize = off;
  P.flops_period = fl;
  // update matrices: u x u column-major in a per-period arena, live from the
  // node's level to its parent's (tree roots: to the end of the interior
  // pass, when the pg front collects them); first-fit placement
  P.node_uoff.assign(ns, 0);
  {
    std::vector<std::vector<int32_t>> by_level(H + 1);
    for (int32_t s = 0; s < ns; ++s) by_level[P.node_level[s]].push_back(s);
    std::vector<std::vector<int32_t>> free_at(H + 2);
    for (int32_t s = 0; s < ns; ++s) {
      const int32_t par = P.node_parent[s];
      const int32_t end = par < 0 ? H : P.node_level[par];
      free_at[end + 1].push_back(s);
    }
    std::vector<std::pair<int64_t, int64_t>> holes;  // (offset, size), sorted
    int64_t top = 0;
    auto release = [&](int64_t o, int64_t sz) {
      holes.push_back({o, sz});
      std::sort(holes.begin(), holes.end());
      std::vector<std::pair<int64_t, int64_t>> m;
      for (auto& h : holes) {
        if (!m.empty() && m.back().first + m.back().second == h.first) m.back().second += h.second;
        else m.push_back(h);
      }
      holes.swap(m);
      if (!holes.empty() && holes.back().first + holes.back().second == top) {
        top = holes.back().first;
        holes.pop_back();
      }
    };
    int64_t peak = 0;
    for (int32_t h = 0; h <= H; ++h) {
      for (int32_t s : free_at[h]) {
        const int64_t u = P.node_u[s];
        if (u) release(P.node_uoff[s], u * u);
      }
      if (h == H) break;
      for (int32_t s : by_level[h]) {
        const int64_t sz = (int64_t)P.node_u[s] * P.node_u[s];
        if (!sz) continue;
        int64_t at = -1;
        for (size_t k = 0; k < holes.size(); ++k)
          if (holes[k].second >= sz) {
            at = holes[k].first;
            holes[k].first += sz;
            holes[k].second -= sz;
            if (holes[k].second == 0) holes.erase(holes.begin() + k);
            break;
          }
        if (at < 0) {
          at = top;
          top += sz;
        }
        P.node_uoff[s] = at;
        peak = std::max(peak, top);
      }
    }
    P.usize = std::max<int64_t>(peak, 1);
  }
  // level lists: small fronts (LDS kernels) and large ones (blocked)
  P.lvl_small_ptr.assign(H + 1, 0);
  P.lvl_large_ptr.assign(H + 1, 0);
  {
    std::vector<std::vector<int32_t>> sm(H), lg(H);
    for (int32_t s = 0; s < ns; ++s) {
      if (P.node_p[s] + P.node_u[s] <= opt.small_max) sm[P.node_level[s]].push_back(s);
      else lg[P.node_level[s]].push_back(s);
    }
    for (int32_t h = 0; h < H; ++h) {
      P.lvl_small.insert(P.lvl_small.end(), sm[h].begin(), sm[h].end());
      P.lvl_large.insert(P.lvl_large.end(), lg[h].begin(), lg[h].end());
      P.lvl_small_ptr[h + 1] = (int64_t)P.lvl_small.size();
      P.lvl_large_ptr[h + 1] = (int64_t)P.lvl_large.size();
    }
  }
  // extend-add work items per level: (node, first column) in blocks of
  // opt.col_block columns of the node's front
  P.lvl_items_ptr.assign(H + 1, 0);
  for (int32_t h = 0; h < H; ++h) {
    for (int32_t s = 0; s < ns; ++s) {
      if (P.node_level[s] != h) continue;
      const int32_t f = P.node_p[s] + P.node_u[s];
      for (int32_t c0 = 0; c0 < f; c0 += opt.col_block) {
        P.items.push_back(s);
        P.items.push_back(c0);
      }
    }
    P.lvl_items_ptr[h + 1] = (int64_t)P.items.size() / 2;
  }
  // the pg front of a period collects its tree roots: items over its G
  // columns
  for (int32_t c0 = 0; c0 < G; c0 += opt.col_block) P.root_items.push_back(c0);
  // destinations of the K template slots: >= 0 an interior factor offset,
  // < 0 the pg front, -1 - (col * 2G + row)
  P.slot_dst.resize(I.krow[np]);
  for (int32_t r = 0; r < np; ++r)
    for (int32_t q = I.krow[r]; q < I.krow[r + 1]; ++q) {
      const int32_t a = P.iperm[r], b = P.iperm[I.kcol[q]];
      const int32_t row = std::max(a, b), col = std::min(a, b);
      if (col >= P.n_int) {
        P.slot_dst[q] = -1 - ((int64_t)(col - P.n_int) * 2 * G + (row - P.n_int));
        continue;
      }
      // the node owning the column: binary search over node_f
      const int32_t s = (int32_t)(std::upper_bound(P.node_f.begin(), P.node_f.end(), col) - P.node_f.begin()) - 1;
      const int32_t p = P.node_p[s], u = P.node_u[s];
      int32_t lr;
      if (row < P.node_f[s] + p) {
        lr = row - P.node_f[s];
      } else {
        const int32_t* rr = P.rows.data() + P.row_ptr[s];
        const int32_t* it = std::lower_bound(rr, rr + u, row);
        if (it == rr + u || *it != row) {
          err = "chol analysis: K entry outside its node's front";
          return OPF_EINVAL;
        }
        lr = p + (int32_t)(it - rr);
      }
      P.slot_dst[q] = P.node_loff[s] + (int64_t)(col - P.node_f[s]) * (p + u) + lr;
    }
  // K positions of the template slots relative to the period block start,
  // for period 0 and for periods >= 1 (whose pg rows lead with a ramp slot)
  P.kpos0.resize(I.krow[np]);
  P.kpos1.resize(I.krow[np]);
  for (int32_t r = 0; r < np; ++r) {
    int32_t shift = 0;
    if (r >= PG && r < PG + G) shift = r - PG + 1;
    else if (r >= PG + G) shift = G;
    for (int32_t q = I.krow[r]; q < I.krow[r + 1]; ++q) {
      P.kpos0[q] = q;
      P.kpos1[q] = q + shift;
    }
  }
  P.ramp_pos.resize(G);
  for (int32_t g = 0; g < G; ++g) P.ramp_pos[g] = I.krow[PG + g] + g;
  // factor sizes and flops, interior and pg chain
  const double Gd = G;
  P.flops_chain = (double)I.T * Gd * Gd * Gd / 3.0 + (double)(I.T - 1) * 2.0 * Gd * Gd * Gd;
  return OPF_OK;
}

}  // namespace opf
