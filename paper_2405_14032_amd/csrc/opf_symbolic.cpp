// Descriptor validation, element tables and per-period symbolic plans.
//
// The paper's modelling layer analyses the sparsity of each repeated pattern
// once and expands it over the data (Sec. III-A).  Here that analysis is
// explicit: every line, bus and generator contributes a fixed set of J / H
// entries per period, and the condensed matrix K = H + diag + J^T D J
// (Sec. III-B) has one per-period template that is identical for all
// periods except the (pg_t, pg_{t-1}) ramp pair of periods t >= 1.
#include "opf_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace opf {

namespace {

const int64_t kI32Max = std::numeric_limits<int32_t>::max();

bool finite(double v) { return std::isfinite(v); }

}  // namespace

int validate_descs(const opf_instance_desc* desc, int32_t ninst, std::string& err) {
  if (!desc || ninst < 1) {
    err = "descriptor array is NULL or ninst < 1";
    return OPF_EINVAL;
  }
  int64_t tot_n = 0, tot_m = 0;
  for (int32_t k = 0; k < ninst; ++k) {
    const opf_instance_desc& d = desc[k];
    std::string where = "instance " + std::to_string(k) + ": ";
    if (d.nbus < 1 || d.nbranch < 0 || d.ngen < 1 || d.nperiod < 1) {
      err = where + "need nbus >= 1, nbranch >= 0, ngen >= 1, nperiod >= 1";
      return OPF_EINVAL;
    }
    if (d.ref_bus < 0 || d.ref_bus >= d.nbus) {
      err = where + "ref_bus out of range";
      return OPF_EINVAL;
    }
    const void* req[] = {d.vmin, d.vmax, d.gen_bus, d.c2, d.c1, d.pmin, d.pmax,
                         d.qmin, d.qmax, d.ramp, d.pd, d.qd};
    for (const void* p : req)
      if (!p) {
        err = where + "a required bus / generator / load array is NULL";
        return OPF_EINVAL;
      }
    if (d.nbranch > 0) {
      const void* reqb[] = {d.f_bus, d.t_bus, d.r, d.x, d.b_charge, d.rate, d.angmin, d.angmax};
      for (const void* p : reqb)
        if (!p) {
          err = where + "a required line array is NULL";
          return OPF_EINVAL;
        }
    }
    const int64_t N = d.nbus, B = d.nbranch, G = d.ngen, T = d.nperiod;
    const int64_t n_p = 2 * N + 2 * G + 4 * B, m_p = 2 * N + 7 * B + 1;
    const int64_t n = T * n_p, m = T * m_p + G * (T - 1);
    if (n_p > kI32Max || m_p > kI32Max || 2 * G + 30 * B + 1 > kI32Max || G + 40 * B > kI32Max) {
      err = where + "per-period sizes exceed int32";
      return OPF_ERANGE;
    }
    // every block a kernel addresses through a 32-bit byte offset (x, c, J,
    // H of one period, the line scratch of one period) stays below 4 GiB
    const int64_t blocks[] = {n_p, m_p, 2 * G + 30 * B + 1, G + 40 * B, kLineScratchDoubles * B};
    for (int64_t e : blocks)
      if (e > kMaxBlockDoubles) {
        err = where + "a per-period block exceeds the 4 GiB a 32-bit byte offset addresses";
        return OPF_ERANGE;
      }
    tot_n += n;
    tot_m += m;
    if (tot_n > kI32Max || tot_m > kI32Max) {
      err = where + "total variables / rows exceed int32 indices";
      return OPF_ERANGE;
    }
    for (int64_t l = 0; l < B; ++l) {
      int32_t f = d.f_bus[l], t = d.t_bus[l];
      if (f < 0 || f >= N || t < 0 || t >= N) {
        err = where + "line " + std::to_string(l) + " has a bus index out of range";
        return OPF_EINVAL;
      }
      if (f == t) {
        err = where + "line " + std::to_string(l) + " has f == t";
        return OPF_EINVAL;
      }
      double r = d.r[l], x = d.x[l];
      if (!finite(r) || !finite(x) || (r == 0.0 && x == 0.0) || !finite(d.b_charge[l])) {
        err = where + "line " + std::to_string(l) + " has a non-finite or zero impedance";
        return OPF_EINVAL;
      }
      if (d.tap && !(d.tap[l] > 0.0 && finite(d.tap[l]))) {
        err = where + "line " + std::to_string(l) + " has a non-positive tap";
        return OPF_EINVAL;
      }
      if (d.shift && !finite(d.shift[l])) {
        err = where + "line " + std::to_string(l) + " has a non-finite shift";
        return OPF_EINVAL;
      }
    }
    for (int64_t g = 0; g < G; ++g) {
      if (d.gen_bus[g] < 0 || d.gen_bus[g] >= N) {
        err = where + "generator " + std::to_string(g) + " has a bus index out of range";
        return OPF_EINVAL;
      }
    }
  }
  return OPF_OK;
}

int build_instance(const opf_instance_desc& d, InstHost& I, std::string& err) {
  const int32_t N = d.nbus, B = d.nbranch, G = d.ngen, T = d.nperiod;
  I.N = N;
  I.B = B;
  I.G = G;
  I.T = T;
  I.ref = d.ref_bus;
  I.n_p = 2LL * N + 2LL * G + 4LL * B;
  I.m_p = 2LL * N + 7LL * B + 1;
  I.nnzj_p = 2LL * G + 30LL * B + 1;
  I.nnzh_p = (int64_t)G + 40LL * B;
  I.n = (int64_t)T * I.n_p;
  I.m = (int64_t)T * I.m_p + (int64_t)G * (T - 1);
  I.nnzj = (int64_t)T * I.nnzj_p + 2LL * G * (T - 1);
  I.nnzh = (int64_t)T * I.nnzh_p;

  auto cp = [](const double* p, int64_t cnt, double dflt) {
    std::vector<double> v(cnt);
    for (int64_t i = 0; i < cnt; ++i) v[i] = p ? p[i] : dflt;
    return v;
  };
  I.f_bus.assign(d.f_bus, d.f_bus + B);
  I.t_bus.assign(d.t_bus, d.t_bus + B);
  I.gen_bus.assign(d.gen_bus, d.gen_bus + G);
  I.c2 = cp(d.c2, G, 0.0);
  I.c1 = cp(d.c1, G, 0.0);
  I.c0 = cp(d.c0, G, 0.0);
  I.pd = cp(d.pd, (int64_t)T * N, 0.0);
  I.qd = cp(d.qd, (int64_t)T * N, 0.0);
  I.vmin = cp(d.vmin, N, 0.0);
  I.vmax = cp(d.vmax, N, 0.0);
  I.pmin = cp(d.pmin, G, 0.0);
  I.pmax = cp(d.pmax, G, 0.0);
  I.qmin = cp(d.qmin, G, 0.0);
  I.qmax = cp(d.qmax, G, 0.0);
  I.ramp = cp(d.ramp, G, 0.0);
  I.rate = cp(d.rate, B, 0.0);
  I.angmin = cp(d.angmin, B, 0.0);
  I.angmax = cp(d.angmax, B, 0.0);

  // Pi-model admittances in real arithmetic: series y = 1/(r + jx) = g + jb,
  // charging j b_c / 2 at both ends, transformer a = tau e^{j phi} on the
  // from side: Y_tt = y + j b_c/2, Y_ff = Y_tt / tau^2,
  // Y_ft = -y / conj(a) = -(y / tau) e^{j phi}, Y_tf = -y / a = -(y / tau) e^{-j phi}.
  I.adm.assign(8 * (size_t)B, 0.0);
  for (int32_t l = 0; l < B; ++l) {
    const double r = d.r[l], x = d.x[l], bc = d.b_charge[l];
    const double tau = d.tap ? d.tap[l] : 1.0, phi = d.shift ? d.shift[l] : 0.0;
    const double den = r * r + x * x;
    const double g = r / den, b = -x / den;
    const double gtt = g, btt = b + 0.5 * bc;
    const double gff = gtt / (tau * tau), bff = btt / (tau * tau);
    const double cph = std::cos(phi), sph = std::sin(phi);
    // -(g + jb)(cos phi + j sin phi) / tau
    const double gft = -(g * cph - b * sph) / tau, bft = -(g * sph + b * cph) / tau;
    // -(g + jb)(cos phi - j sin phi) / tau
    const double gtf = -(g * cph + b * sph) / tau, btf = -(b * cph - g * sph) / tau;
    const double rec[8] = {gff, bff, gft, bft, gtf, btf, gtt, btt};
    for (int q = 0; q < 8; ++q) I.adm[(size_t)q * B + l] = rec[q];
  }

  // bus incidence sorted by (neighbour, line)
  std::vector<std::vector<std::pair<int32_t, int32_t>>> inc(N);  // (neighbour, l<<1|e)
  for (int32_t l = 0; l < B; ++l) {
    inc[I.f_bus[l]].push_back({I.t_bus[l], (l << 1) | 0});
    inc[I.t_bus[l]].push_back({I.f_bus[l], (l << 1) | 1});
  }
  I.bus_ptr.assign(N + 1, 0);
  I.bus_adj.clear();
  I.bus_nb.clear();
  I.bus_adj.reserve(2 * (size_t)B);
  I.bus_nb.reserve(2 * (size_t)B);
  for (int32_t n = 0; n < N; ++n) {
    std::sort(inc[n].begin(), inc[n].end());
    for (auto& e : inc[n]) {
      I.bus_adj.push_back(e.second);
      I.bus_nb.push_back(e.first);
    }
    I.bus_ptr[n + 1] = (int32_t)I.bus_adj.size();
  }
  std::vector<std::vector<int32_t>> gat(N);
  for (int32_t g = 0; g < G; ++g) gat[I.gen_bus[g]].push_back(g);
  I.bgen_ptr.assign(N + 1, 0);
  I.bgen.clear();
  for (int32_t n = 0; n < N; ++n) {
    for (int32_t g : gat[n]) I.bgen.push_back(g);
    I.bgen_ptr[n + 1] = (int32_t)I.bgen.size();
  }

  // ---- condensed-matrix template of one period (local rows / columns) ----
  const int64_t VA = N, PG = 2LL * N, QG = 2LL * N + G, FL = 2LL * N + 2LL * G;
  I.krow.assign(I.n_p + 1, 0);
  I.kcol.clear();
  I.ksrc.clear();
  std::vector<std::pair<int64_t, int32_t>> row;  // (col, src)
  auto flush = [&](int64_t r) {
    std::sort(row.begin(), row.end());
    for (size_t q = 1; q < row.size(); ++q)
      if (row[q].first == row[q - 1].first) return false;  // never expected
    for (auto& e : row) {
      I.kcol.push_back((int32_t)e.first);
      I.ksrc.push_back(e.second);
    }
    I.krow[r + 1] = (int32_t)I.kcol.size();
    row.clear();
    return true;
  };
  auto distinct_neighbours = [&](int32_t n) {
    std::vector<int32_t> nb;
    for (int32_t q = I.bus_ptr[n]; q < I.bus_ptr[n + 1]; ++q) {
      int32_t l = I.bus_adj[q] >> 1, e = I.bus_adj[q] & 1;
      int32_t m = e == 0 ? I.t_bus[l] : I.f_bus[l];
      if (nb.empty() || nb.back() != m) nb.push_back(m);
    }
    return nb;
  };
  bool ok = true;
  // vm rows: vm of lower-numbered neighbours, then the diagonal
  for (int32_t n = 0; n < N; ++n) {
    for (int32_t m : distinct_neighbours(n))
      if (m < n) row.push_back({m, kSrcNone});
    row.push_back({n, kSrcNone});
    ok &= flush(n);
  }
  // va rows: vm of every neighbour and of the bus itself (the bus's own
  // (va, vm) pair exists only through an incident line's flow rows), va of
  // lower-numbered neighbours, then the diagonal
  for (int32_t n = 0; n < N; ++n) {
    auto nb = distinct_neighbours(n);
    for (int32_t m : nb) row.push_back({m, kSrcNone});
    if (!nb.empty()) row.push_back({n, kSrcNone});
    for (int32_t m : nb)
      if (m < n) row.push_back({VA + m, kSrcNone});
    row.push_back({VA + n, kSrcNone});
    ok &= flush(VA + n);
  }
  // generator rows: same-bus generators with a lower index (shared balance
  // row), then the diagonal; the ramp pair of t >= 1 is added at expansion
  for (int which = 0; which < 2; ++which) {
    const int64_t base = which == 0 ? PG : QG;
    for (int32_t g = 0; g < G; ++g) {
      int32_t n = I.gen_bus[g];
      for (int32_t q = I.bgen_ptr[n]; q < I.bgen_ptr[n + 1]; ++q) {
        int32_t g2 = I.bgen[q];
        if (g2 < g) row.push_back({base + g2, (int32_t)(which * G + g2)});
      }
      row.push_back({base + g, kSrcNone});
      ok &= flush(base + g);
    }
  }
  // flow rows: the four bus variables of the line, the lower members of
  // the balance row the flow enters, the thermal partner, the diagonal
  I.kinfo.assign(4 * (size_t)B, 0);
  bool small = true;
  for (int k = 0; k < 4; ++k) {
    const bool is_p = (k % 2) == 0;
    for (int32_t l = 0; l < B; ++l) {
      const int32_t i = I.f_bus[l], j = I.t_bus[l];
      const int64_t own = FL + (int64_t)k * B + l;
      row.push_back({i, kSrcNone});
      row.push_back({j, kSrcNone});
      row.push_back({VA + i, kSrcNone});
      row.push_back({VA + j, kSrcNone});
      const int32_t b = k < 2 ? i : j;
      for (int32_t q = I.bgen_ptr[b]; q < I.bgen_ptr[b + 1]; ++q) {
        int32_t g = I.bgen[q];
        int64_t col = (is_p ? PG : QG) + g;
        if (col < own) row.push_back({col, (int32_t)((is_p ? 0 : G) + g)});
      }
      for (int32_t q = I.bus_ptr[b]; q < I.bus_ptr[b + 1]; ++q) {
        int32_t l2 = I.bus_adj[q] >> 1, e = I.bus_adj[q] & 1;
        int kind2 = (e == 0 ? 0 : 2) + (is_p ? 0 : 1);  // flow leaving at that end
        int64_t col = FL + (int64_t)kind2 * B + l2;
        if (col < own) row.push_back({col, (int32_t)(2LL * G + (int64_t)kind2 * B + l2)});
      }
      if (k == 1) row.push_back({FL + 0LL * B + l, kSrcThermal});
      if (k == 3) row.push_back({FL + 2LL * B + l, kSrcThermal});
      row.push_back({own, kSrcNone});
      ok &= flush(own);
      // partner slot kinds of the row just emitted (columns ascending:
      // generator partners come before every flow-variable partner)
      const int32_t p0 = I.krow[own] + 4, p1 = I.krow[own + 1] - 1;
      int32_t ngen = 0, th = 0xFFFF;
      for (int32_t q = p0; q < p1; ++q) {
        if (I.ksrc[q] == kSrcThermal) th = q - p0;
        else if (I.ksrc[q] >= 0 && I.ksrc[q] < 2 * G) ++ngen;
      }
      small &= (p1 - p0) < 0xFFFF;
      I.kinfo[(size_t)k * B + l] = (int32_t)((uint32_t)ngen | ((uint32_t)th << 16));
    }
  }
  if (!small) {
    err = "a bus has too many incident lines and generators for the condensed-matrix template";
    return OPF_ERANGE;
  }
  if (!ok) {
    err = "internal: duplicate column in the condensed-matrix template";
    return OPF_EINVAL;
  }
  if ((int64_t)I.kcol.size() > kI32Max) {
    err = "condensed-matrix template exceeds int32";
    return OPF_ERANGE;
  }
  if ((int64_t)I.kcol.size() + G > kMaxBlockDoubles) {
    err = "a period's block of the condensed matrix exceeds the 4 GiB a 32-bit byte offset addresses";
    return OPF_ERANGE;
  }
  I.nnzk_p = (int64_t)I.kcol.size();
  I.nnzk = (int64_t)T * I.nnzk_p + (int64_t)G * (T - 1);
  return OPF_OK;
}

int assign_offsets(std::vector<InstHost>& insts, std::string& err) {
  int64_t xo = 0, co = 0, jo = 0, ho = 0, ko = 0, lo = 0, so = 0;
  for (auto& I : insts) {
    I.x_off = xo;
    I.c_off = co;
    I.j_off = jo;
    I.h_off = ho;
    I.k_off = ko;
    I.ld_off = lo;
    I.s_off = so;
    xo += I.n;
    co += I.m;
    jo += I.nnzj;
    ho += I.nnzh;
    ko += I.nnzk;
    lo += (int64_t)I.T * I.N;
    // hand-off scratch: 22 doubles per line-period (two 8-value end records,
    // the shared cross pair, the separate J^T v record), rounded up to 64 B;
    // then the objective partials of the whole sweep
    I.o_off = so + line_scratch_doubles(I.B, I.T);
    so = I.o_off + obj_scratch_doubles(I.G, I.T);
  }
  if (xo > kI32Max || co > kI32Max) {
    err = "total variables / rows exceed int32 indices";
    return OPF_ERANGE;
  }
  return OPF_OK;
}

void kkt_structure_host(const std::vector<InstHost>& insts, int64_t* rowptr, int32_t* colind) {
  int64_t last = 0;
  for (const auto& I : insts) {
    const int64_t PG = 2LL * I.N;
    for (int32_t t = 0; t < I.T; ++t) {
      const int64_t kp = I.k_off + kkt_period_offset(I.nnzk_p, I.G, t);
      const int64_t xb = I.x_off + (int64_t)t * I.n_p;
      for (int64_t r = 0; r < I.n_p; ++r) {
        int64_t shift = 0;
        bool ramp = false;
        if (t >= 1) {
          if (r >= PG && r < PG + I.G) {
            shift = r - PG + 1;
            ramp = true;
          } else if (r >= PG + I.G) {
            shift = I.G;
          }
        }
        int64_t start = kp + I.krow[r] + shift - (ramp ? 1 : 0);
        rowptr[xb + r] = start;
        int64_t pos = start;
        if (ramp) colind[pos++] = (int32_t)(xb - I.n_p + r);
        for (int32_t p = I.krow[r]; p < I.krow[r + 1]; ++p) colind[pos++] = (int32_t)(xb + I.kcol[p]);
        last = pos;
      }
    }
  }
  int64_t ntot = insts.empty() ? 0 : insts.back().x_off + insts.back().n;
  rowptr[ntot] = last;
}

}  // namespace opf
