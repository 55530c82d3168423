// HIP kernels for gfx950 (FP64): per-iteration evaluation of the
// multi-period AC OPF model (Sec. II, eq. (1a)-(1k)), its sparse derivatives
// in per-pattern COO form (Sec. III-A) and the condensed KKT matrix of the
// lifted-KKT interior-point method (Sec. III-B).
//
// Execution model: every kernel walks a tile list.  A tile covers a range
// of elements of one class (lines, generators, buses, ...) of one instance
// over a range of periods; lane e of the block owns element e0 + e and
// walks the tile's periods, so consecutive lanes touch consecutive entries
// of every per-period SoA block (coalesced loads and stores).  The grid is
// either one block per tile or a persistent grid that strides over the list.
// Consecutive tiles go to the same XCD (the remap below), so each XCD's L2
// serves a contiguous run of periods.  No kernel uses atomics: each output
// slot has exactly one owning lane, which makes results bitwise
// reproducible.
//
// The flow physics is the pi-model in expanded real trigonometric form: for
// line l = (i -> j), delta = va_i - va_j, c = cos delta, s = sin delta and
// each of the four flows (pf, qf at the from end, pt, qt at the to end)
//   phi_k = S_k V_o^2 + V_i V_j (alpha_k c + beta_k s),   o = i or j,
// with (S, alpha, beta) = (Gff, Gft, Bft), (-Bff, -Bft, Gft),
// (Gtt, Gtf, -Btf), (-Btt, -Btf, -Gtf) from the admittances Y = G + jB.
// With w = alpha c + beta s and u = dw/d delta = beta c - alpha s:
//   dphi/dV_i = 2 S V_i [o=i] + V_j w,  dphi/dV_j = 2 S V_j [o=j] + V_i w,
//   dphi/dtheta_i = V_i V_j u = -dphi/dtheta_j,
//   d2phi: (Vi,Vi) 2S[o=i], (Vj,Vi) w, (Vj,Vj) 2S[o=j], (ti,Vi) V_j u,
//   (ti,Vj) V_i u, (ti,ti) -V_iV_j w, (tj,Vi) -V_j u, (tj,Vj) -V_i u,
//   (tj,ti) V_iV_j w, (tj,tj) -V_iV_j w.
#include "opf_device.h"

namespace opf {
namespace {

// Tiles v = b, b + grid, ... of block b run on XCD b % 8; give each XCD a
// contiguous run of the list (bijective on [0, ntiles)).
__device__ __forceinline__ int remap_tile(int v, int ntiles) {
  const int q = ntiles >> 3;
  if (v < (q << 3)) return (v & 7) * q + (v >> 3);
  return v;
}

// Sum over the 64 lanes of a wavefront (butterfly order; lane 0's result is
// the same on every run).  Every lane of the wavefront must take part.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct Coef {
  double S[4], al[4], be[4];
};

__device__ __forceinline__ void load_coef(const InstDev& I, int l, Coef& c) {
  const int64_t B = I.B;
  const double* a = I.adm;
  const double gff = a[l], bff = a[B + l], gft = a[2 * B + l], bft = a[3 * B + l];
  const double gtf = a[4 * B + l], btf = a[5 * B + l], gtt = a[6 * B + l], btt = a[7 * B + l];
  c.S[0] = gff;
  c.al[0] = gft;
  c.be[0] = bft;
  c.S[1] = -bff;
  c.al[1] = -bft;
  c.be[1] = gft;
  c.S[2] = gtt;
  c.al[2] = gtf;
  c.be[2] = -btf;
  c.S[3] = -btt;
  c.al[3] = -btf;
  c.be[3] = -gtf;
}

// Kind k's coefficients from an LDS copy of the line's eight admittances
// (SoA, stride bd): the same values load_coef gives for that kind, without
// keeping all twelve in registers across a loop over periods.
__device__ __forceinline__ void coef_kind_lds(const double* sadm, int bd, int tid, int k, Coef& c) {
  if (k == 0) {
    c.S[0] = sadm[tid];
    c.al[0] = sadm[2 * bd + tid];
    c.be[0] = sadm[3 * bd + tid];
  } else if (k == 1) {
    c.S[1] = -sadm[bd + tid];
    c.al[1] = -sadm[3 * bd + tid];
    c.be[1] = sadm[2 * bd + tid];
  } else if (k == 2) {
    c.S[2] = sadm[6 * bd + tid];
    c.al[2] = sadm[4 * bd + tid];
    c.be[2] = -sadm[5 * bd + tid];
  } else {
    c.S[3] = -sadm[7 * bd + tid];
    c.al[3] = -sadm[5 * bd + tid];
    c.be[3] = -sadm[4 * bd + tid];
  }
}

// Per-period block bases (local offsets inside one period).
struct Bases {
  int64_t N, B, G;
  int64_t xFL;                                     // first flow variable
  int64_t jBAL, jREF, jFLOW, jTH, jANG;            // J blocks
  int64_t cREF, cFLOW, cTHF, cTHT, cANG;           // c blocks
  int64_t hFLOW, hTH;                              // H blocks
  __device__ __forceinline__ explicit Bases(const InstDev& I) {
    N = I.N;
    B = I.B;
    G = I.G;
    xFL = 2 * N + 2 * G;
    jBAL = 2 * G;
    jREF = 2 * G + 4 * B;
    jFLOW = jREF + 1;
    jTH = jFLOW + 20 * B;
    jANG = jTH + 4 * B;
    cREF = 2 * N;
    cFLOW = 2 * N + 1;
    cTHF = cFLOW + 4 * B;
    cTHT = cTHF + B;
    cANG = cTHT + B;
    hFLOW = G;
    hTH = G + 36 * B;
  }
};

// w_k = alpha_k cos(delta) + beta_k sin(delta).
__device__ __forceinline__ double flow_w(const Coef& cf, int k, double s, double c) {
  return cf.al[k] * c + cf.be[k] * s;
}

// phi_k = S_k V_o^2 + V_i V_j w_k, the flow the kind's definition row equates.
__device__ __forceinline__ double flow_value(const Coef& cf, int k, double vi, double vj, double vv, double w) {
  const double vo = k < 2 ? vi : vj;
  return cf.S[k] * vo * vo + vv * w;
}

// First and second derivatives of flow kind k of one line at one period.
// Jk: the flow row's J entries (own, vm_i, vm_j, va_i, va_j); h: the nine
// lower-triangle Hessian entries of -ck * Hess(phi_k) in the local order of
// the kind (ck = the row's multiplier).  Every kernel that produces J or H
// values goes through this function, so separate and fused evaluations
// give bitwise identical values.
__device__ __forceinline__ void flow_kind(const Coef& cf, int k, double vi, double vj, double vv, double s,
                                          double c, double ck, double Jk[5], double h[9]) {
  const double w = flow_w(cf, k, s, c);
  const double u = cf.be[k] * c - cf.al[k] * s;
  const double dvi = (k < 2 ? 2.0 * cf.S[k] * vi : 0.0) + vj * w;
  const double dvj = (k < 2 ? 0.0 : 2.0 * cf.S[k] * vj) + vi * w;
  const double dti = vv * u;
  Jk[0] = 1.0;
  Jk[1] = -dvi;
  Jk[2] = -dvj;
  Jk[3] = -dti;
  Jk[4] = dti;
  if (k < 2) {
    h[0] = ck * (2.0 * cf.S[k]);
    h[1] = ck * w;
  } else {
    h[0] = ck * w;
    h[1] = ck * (2.0 * cf.S[k]);
  }
  h[2] = ck * (vj * u);
  h[3] = ck * (vi * u);
  h[4] = -ck * (vv * w);
  h[5] = -ck * (vj * u);
  h[6] = -ck * (vi * u);
  h[7] = ck * (vv * w);
  h[8] = -ck * (vv * w);
}

// J^T v of one line at one period from its flow-row J entries Jf: the four
// flow-variable outputs and the hand-off record of the bus-variable sums
// (vm_i, vm_j, va_i, va_j).  vbal = v of the balance rows each flow enters.
__device__ __forceinline__ void jt_line(const double vk[4], const double Jf[4][5], double vtf, double vtt,
                                        double vang, const double fl[4], const double vbal[4], double out[4],
                                        double rec[4]) {
  double svi = 0.0, svj = 0.0, sti = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    svi += vk[k] * Jf[k][1];
    svj += vk[k] * Jf[k][2];
    sti += vk[k] * Jf[k][3];
  }
  out[0] = vk[0] + vtf * (2.0 * fl[0]) - vbal[0];
  out[1] = vk[1] + vtf * (2.0 * fl[1]) - vbal[1];
  out[2] = vk[2] + vtt * (2.0 * fl[2]) - vbal[2];
  out[3] = vk[3] + vtt * (2.0 * fl[3]) - vbal[3];
  rec[0] = svi;
  rec[1] = svj;
  rec[2] = sti + vang;
  rec[3] = -sti - vang;
}

// Copies src[0 .. n) (LDS) to dst[0 .. n) in global memory, lane i writing
// element i - d with d = dst's offset inside its 64-byte line, so that each
// wave writes whole lines except at the two ends of the range.
__device__ __forceinline__ void aligned_out(const double* __restrict__ src, int n, double* dst) {
  const int d = (int)(((uintptr_t)dst >> 3) & 7);
  const rsrc_t rd = rsrc(dst - d);
  for (int i = (int)threadIdx.x; i < n + d; i += (int)blockDim.x) {
    const int p = i - d;
    if (p >= 0) bstn(rd, (uint32_t)i, src[p]);
  }
}

// ---------------------------------------------------------------- Jacobian
// One line tile of the Jacobian, block-cooperative: each lane evaluates its
// line's 30 entries, which leave through LDS in two rounds of 15 streams so
// that every stream is written with whole 64-byte lines (the per-period J
// block starts at an arbitrary 8-byte offset).  Dynamic LDS: [15][blockDim].
__device__ void jac_line_tile(const InstDev& I, const Tile& tl, const double* __restrict__ x,
                              double* __restrict__ jv, double* __restrict__ stg) {
  const Bases b(I);
  const int tid = (int)threadIdx.x, bd = (int)blockDim.x;
  const int l = tl.e0 + tid;
  const bool act = l < tl.e1;
  const int nl = tl.e1 - tl.e0;
  Coef cf;
  uint32_t vI = 0, vJ = 0;
  const uint32_t B8 = (uint32_t)b.B * 8u, N8 = (uint32_t)b.N * 8u, vL = (uint32_t)l * 8u;
  const uint32_t xFL8 = (uint32_t)b.xFL * 8u;
  if (act) {
    load_coef(I, l, cf);
    vI = (uint32_t)I.f_bus[l] * 8u;
    vJ = (uint32_t)I.t_bus[l] * 8u;
  }
  for (int t = tl.t0; t < tl.t1; ++t) {
    double val[30];
#pragma unroll
    for (int a = 0; a < 30; ++a) val[a] = 0.0;
    if (act) {
      const rsrc_t rX = rsrc(x + I.x_off + (int64_t)t * I.n_p);
      const double vi = bldv(rX, vI, 0), vj = bldv(rX, vJ, 0), ti = bldv(rX, vI, N8), tj = bldv(rX, vJ, N8);
      double fl[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) fl[k] = bldv(rX, vL, xFL8 + (uint32_t)k * B8);
      double sn, cs;
      sincos(ti - tj, &sn, &cs);
      const double vv = vi * vj;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double Jk[5], h[9];
        flow_kind(cf, k, vi, vj, vv, sn, cs, 0.0, Jk, h);
#pragma unroll
        for (int a = 0; a < 5; ++a) val[k * 5 + a] = Jk[a];
        val[20 + k] = -1.0;
        val[24 + k] = 2.0 * fl[k];
      }
      val[28] = 1.0;
      val[29] = -1.0;
    }
    double* jp = jv + I.j_off + (int64_t)t * I.nnzj_p;
    // stream s of the 30: flows (k * 5 + a), balance (20 + k), thermal (24 + k), angle (28, 29)
    auto stream_base = [&](int st) -> int64_t {
      if (st < 20) return b.jFLOW + (int64_t)st * b.B;
      if (st < 24) return b.jBAL + (int64_t)(st - 20) * b.B;
      if (st < 28) return b.jTH + (int64_t)(st - 24) * b.B;
      return b.jANG + (int64_t)(st - 28) * b.B;
    };
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (act) {
#pragma unroll
        for (int a = 0; a < 15; ++a) stg[a * bd + tid] = val[r * 15 + a];
      }
      __syncthreads();
      for (int a = 0; a < 15; ++a) aligned_out(stg + a * bd, nl, jp + stream_base(r * 15 + a) + tl.e0);
      __syncthreads();
    }
  }
}

__device__ void jac_gen(const InstDev& I, int g, int t0, int t1, double* __restrict__ jv) {
  const Bases b(I);
  for (int t = t0; t < t1; ++t) {
    double* jp = jv + I.j_off + (int64_t)t * I.nnzj_p;
    jp[g] = 1.0;
    jp[b.G + g] = 1.0;
    if (g == 0) jp[b.jREF] = 1.0;
    if (t >= 1) {
      double* jr = jv + I.j_off + (int64_t)I.T * I.nnzj_p + (int64_t)(t - 1) * 2 * b.G;
      jr[g] = 1.0;
      jr[b.G + g] = -1.0;
    }
  }
}

// Dynamic LDS: [15][blockDim] doubles (the staged line tiles).
__global__ void __launch_bounds__(512) k_jac(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                             int ntiles, const double* __restrict__ x, double* __restrict__ jv) {
  extern __shared__ double lds[];
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    if (tl.kind == TK_BRANCH) {
      jac_line_tile(I, tl, x, jv, lds);
      continue;
    }
    const int e = tl.e0 + (int)threadIdx.x;
    if (e < tl.e1) jac_gen(I, e, tl.t0, tl.t1, jv);
  }
}

// ---------------------------------------------------------------- Hessian
__device__ void hess_branch(const InstDev& I, int l, int t0, int t1, const double* __restrict__ x,
                            const double* __restrict__ lam, double* __restrict__ hv) {
  const Bases b(I);
  Coef cf;
  load_coef(I, l, cf);
  const uint32_t B8 = (uint32_t)b.B * 8u, N8 = (uint32_t)b.N * 8u, vL = (uint32_t)l * 8u;
  const uint32_t hFLOW8 = (uint32_t)b.hFLOW * 8u, hTH8 = (uint32_t)b.hTH * 8u, cFLOW8 = (uint32_t)b.cFLOW * 8u,
                 cTHF8 = (uint32_t)b.cTHF * 8u, cTHT8 = (uint32_t)b.cTHT * 8u;
  const uint32_t vI = (uint32_t)I.f_bus[l] * 8u, vJ = (uint32_t)I.t_bus[l] * 8u;
  double in[10];  // vi, vj, ti, tj, lambda of the 4 flow rows, the 2 thermal rows
  auto load = [&](int t, double* v) {
    const rsrc_t rX = rsrc(x + I.x_off + (int64_t)t * I.n_p), rL = rsrc(lam + I.c_off + (int64_t)t * I.m_p);
    v[0] = bldv(rX, vI, 0);
    v[1] = bldv(rX, vJ, 0);
    v[2] = bldv(rX, vI, N8);
    v[3] = bldv(rX, vJ, N8);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[4 + k] = bldv(rL, vL, cFLOW8 + (uint32_t)k * B8);
    v[8] = bldv(rL, vL, cTHF8);
    v[9] = bldv(rL, vL, cTHT8);
  };
  load(t0, in);
  for (int t = t0; t < t1; ++t) {
    const double vi = in[0], vj = in[1], ti = in[2], tj = in[3];
    double lk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) lk[k] = in[4 + k];
    const double lf = 2.0 * in[8], lt = 2.0 * in[9];
    if (t + 1 < t1) load(t + 1, in);
    const rsrc_t rH = rsrc(hv + I.h_off + (int64_t)t * I.nnzh_p);
    double s, c;
    sincos(ti - tj, &s, &c);
    const double vv = vi * vj;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double Jk[5], h[9];
      flow_kind(cf, k, vi, vj, vv, s, c, -lk[k], Jk, h);
#pragma unroll
      for (int a = 0; a < 9; ++a) bstvn(rH, vL, hFLOW8 + (uint32_t)(k * 9 + a) * B8, h[a]);
    }
    bstvn(rH, vL, hTH8, lf);
    bstvn(rH, vL, hTH8 + B8, lf);
    bstvn(rH, vL, hTH8 + 2 * B8, lt);
    bstvn(rH, vL, hTH8 + 3 * B8, lt);
  }
}

__global__ void __launch_bounds__(512) k_hess(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                              int ntiles, const double* __restrict__ x,
                                              const double* __restrict__ lam, double sigma,
                                              double* __restrict__ hv) {
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int e = tl.e0 + (int)threadIdx.x;
    if (e >= tl.e1) continue;
    if (tl.kind == TK_BRANCH) {
      hess_branch(I, e, tl.t0, tl.t1, x, lam, hv);
    } else {
      const double h = 2.0 * sigma * I.c2[e];
      for (int t = tl.t0; t < tl.t1; ++t) hv[I.h_off + (int64_t)t * I.nnzh_p + e] = h;
    }
  }
}

// ---------------------------------------------------------------- constraints
__device__ void cons_branch(const InstDev& I, int l, int t0, int t1, const double* __restrict__ x,
                            double* __restrict__ cv) {
  const Bases b(I);
  Coef cf;
  load_coef(I, l, cf);
  const uint32_t B8 = (uint32_t)b.B * 8u, N8 = (uint32_t)b.N * 8u, vL = (uint32_t)l * 8u;
  const uint32_t xFL8 = (uint32_t)b.xFL * 8u, cFLOW8 = (uint32_t)b.cFLOW * 8u, cTHF8 = (uint32_t)b.cTHF * 8u,
                 cTHT8 = (uint32_t)b.cTHT * 8u, cANG8 = (uint32_t)b.cANG * 8u;
  const uint32_t vI = (uint32_t)I.f_bus[l] * 8u, vJ = (uint32_t)I.t_bus[l] * 8u;
  double in[8];
  auto load = [&](int t, double* w) {
    const rsrc_t rX = rsrc(x + I.x_off + (int64_t)t * I.n_p);
    w[0] = bldv(rX, vI, 0);
    w[1] = bldv(rX, vJ, 0);
    w[2] = bldv(rX, vI, N8);
    w[3] = bldv(rX, vJ, N8);
#pragma unroll
    for (int k = 0; k < 4; ++k) w[4 + k] = bldv(rX, vL, xFL8 + (uint32_t)k * B8);
  };
  load(t0, in);
  for (int t = t0; t < t1; ++t) {
    const double vi = in[0], vj = in[1], ti = in[2], tj = in[3];
    double fl[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) fl[k] = in[4 + k];
    if (t + 1 < t1) load(t + 1, in);
    const rsrc_t rC = rsrc(cv + I.c_off + (int64_t)t * I.m_p);
    double s, c;
    sincos(ti - tj, &s, &c);
    const double vv = vi * vj;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      bstvn(rC, vL, cFLOW8 + (uint32_t)k * B8, fl[k] - flow_value(cf, k, vi, vj, vv, flow_w(cf, k, s, c)));
    bstvn(rC, vL, cTHF8, fl[0] * fl[0] + fl[1] * fl[1]);
    bstvn(rC, vL, cTHT8, fl[2] * fl[2] + fl[3] * fl[3]);
    bstvn(rC, vL, cANG8, ti - tj);
  }
}

__device__ void cons_bus(const InstDev& I, int n, int t0, int t1, const double* __restrict__ x,
                         double* __restrict__ cv) {
  const Bases b(I);
  const uint32_t B8 = (uint32_t)b.B * 8u, N8 = (uint32_t)b.N * 8u, G8 = (uint32_t)b.G * 8u;
  const uint32_t xFL8 = (uint32_t)b.xFL * 8u, vN = (uint32_t)n * 8u;
  const int q0 = I.bus_ptr[n], q1 = I.bus_ptr[n + 1];
  const int g0 = I.bgen_ptr[n], g1 = I.bgen_ptr[n + 1];
  const rsrc_t rAdj = rsrc(I.bus_adj), rBg = rsrc(I.bgen);
  for (int t = t0; t < t1; ++t) {
    const rsrc_t rX = rsrc(x + I.x_off + (int64_t)t * I.n_p);
    double bp = 0.0, bq = 0.0;
    for (int q = g0; q < g1; ++q) {
      const uint32_t g8 = (uint32_t)bldi(rBg, (uint32_t)q) * 8u;
      bp += bldv(rX, g8, 2 * N8);
      bq += bldv(rX, g8, 2 * N8 + G8);
    }
    // incident line ends, four in flight per lane; the flow leaving the bus
    // is (pf, qf) at a from end and (pt, qt) at a to end
    constexpr int U = 4;
    for (int aa = q0; aa < q1; aa += U) {
      int ad[U];
      double fp[U], fq[U];
#pragma unroll
      for (int u = 0; u < U; ++u) ad[u] = aa + u < q1 ? bldi(rAdj, (uint32_t)(aa + u)) : -1;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t o = ad[u] < 0 ? 0u : (uint32_t)(ad[u] >> 1) * 8u + ((ad[u] & 1) ? 2u * B8 : 0u);
        fp[u] = ad[u] < 0 ? 0.0 : bldv(rX, o, xFL8);
        fq[u] = ad[u] < 0 ? 0.0 : bldv(rX, o, xFL8 + B8);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ad[u] < 0) break;
        bp -= fp[u];
        bq -= fq[u];
      }
    }
    bp -= I.pd[(int64_t)t * b.N + n];
    bq -= I.qd[(int64_t)t * b.N + n];
    const rsrc_t rC = rsrc(cv + I.c_off + (int64_t)t * I.m_p);
    const double vref = n == I.ref ? bldv(rX, vN, N8) : 0.0;
    bstvn(rC, vN, 0, bp);
    bstvn(rC, vN, N8, bq);
    if (n == I.ref) bstn(rC, (uint32_t)b.cREF, vref);
  }
}

__global__ void __launch_bounds__(512) k_cons(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                              int ntiles, const double* __restrict__ x, double* __restrict__ cv) {
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int e = tl.e0 + (int)threadIdx.x;
    if (e >= tl.e1) continue;
    if (tl.kind == TK_BRANCH) {
      cons_branch(I, e, tl.t0, tl.t1, x, cv);
    } else if (tl.kind == TK_BUS) {
      cons_bus(I, e, tl.t0, tl.t1, x, cv);
    } else {
      const int64_t pg = 2LL * I.N + e;
      for (int t = tl.t0 < 1 ? 1 : tl.t0; t < tl.t1; ++t) {
        const double* xp = x + I.x_off + (int64_t)t * I.n_p;
        cv[I.c_off + (int64_t)I.T * I.m_p + (int64_t)(t - 1) * I.G + e] = xp[pg] - xp[pg - I.n_p];
      }
    }
  }
}

// ---------------------------------------------------------------- J v
// Forward product J(x) v, row by row in the canonical row order; the tiles
// are those of the constraint kernel (lines: flow, thermal and angle rows;
// buses: balance and reference rows; generators: ramp rows).
__device__ void jv_branch(const InstDev& I, int l, int t0, int t1, const double* __restrict__ x,
                          const double* __restrict__ v, double* __restrict__ out) {
  const Bases b(I);
  Coef cf;
  load_coef(I, l, cf);
  const uint32_t B8 = (uint32_t)b.B * 8u, N8 = (uint32_t)b.N * 8u, vL = (uint32_t)l * 8u;
  const uint32_t xFL8 = (uint32_t)b.xFL * 8u, cFLOW8 = (uint32_t)b.cFLOW * 8u, cTHF8 = (uint32_t)b.cTHF * 8u,
                 cTHT8 = (uint32_t)b.cTHT * 8u, cANG8 = (uint32_t)b.cANG * 8u;
  const uint32_t vI = (uint32_t)I.f_bus[l] * 8u, vJ = (uint32_t)I.t_bus[l] * 8u;
  double in[16];  // x: vi, vj, ti, tj, flows; v: the same eight entries
  auto load = [&](int t, double* w) {
    const rsrc_t rX = rsrc(x + I.x_off + (int64_t)t * I.n_p), rV = rsrc(v + I.x_off + (int64_t)t * I.n_p);
    w[0] = bldv(rX, vI, 0);
    w[1] = bldv(rX, vJ, 0);
    w[2] = bldv(rX, vI, N8);
    w[3] = bldv(rX, vJ, N8);
    w[8] = bldv(rV, vI, 0);
    w[9] = bldv(rV, vJ, 0);
    w[10] = bldv(rV, vI, N8);
    w[11] = bldv(rV, vJ, N8);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      w[4 + k] = bldv(rX, vL, xFL8 + (uint32_t)k * B8);
      w[12 + k] = bldv(rV, vL, xFL8 + (uint32_t)k * B8);
    }
  };
  load(t0, in);
  for (int t = t0; t < t1; ++t) {
    const double vi = in[0], vj = in[1], ti = in[2], tj = in[3];
    const double wvi = in[8], wvj = in[9], wti = in[10], wtj = in[11];
    double fl[4], wf[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      fl[k] = in[4 + k];
      wf[k] = in[12 + k];
    }
    if (t + 1 < t1) load(t + 1, in);
    const rsrc_t rO = rsrc(out + I.c_off + (int64_t)t * I.m_p);
    double sn, cs;
    sincos(ti - tj, &sn, &cs);
    const double vv = vi * vj;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double Jk[5], h[9];
      flow_kind(cf, k, vi, vj, vv, sn, cs, 0.0, Jk, h);
      bstvn(rO, vL, cFLOW8 + (uint32_t)k * B8, Jk[0] * wf[k] + Jk[1] * wvi + Jk[2] * wvj + Jk[3] * wti + Jk[4] * wtj);
    }
    bstvn(rO, vL, cTHF8, (2.0 * fl[0]) * wf[0] + (2.0 * fl[1]) * wf[1]);
    bstvn(rO, vL, cTHT8, (2.0 * fl[2]) * wf[2] + (2.0 * fl[3]) * wf[3]);
    bstvn(rO, vL, cANG8, wti - wtj);
  }
}

__device__ void jv_bus(const InstDev& I, int n, int t0, int t1, const double* __restrict__ v,
                       double* __restrict__ out) {
  const Bases b(I);
  const uint32_t B8 = (uint32_t)b.B * 8u, N8 = (uint32_t)b.N * 8u, G8 = (uint32_t)b.G * 8u;
  const uint32_t xFL8 = (uint32_t)b.xFL * 8u, vN = (uint32_t)n * 8u;
  const int q0 = I.bus_ptr[n], q1 = I.bus_ptr[n + 1];
  const int g0 = I.bgen_ptr[n], g1 = I.bgen_ptr[n + 1];
  const rsrc_t rAdj = rsrc(I.bus_adj), rBg = rsrc(I.bgen);
  for (int t = t0; t < t1; ++t) {
    const rsrc_t rV = rsrc(v + I.x_off + (int64_t)t * I.n_p);
    double bp = 0.0, bq = 0.0;
    for (int q = g0; q < g1; ++q) {
      const uint32_t g8 = (uint32_t)bldi(rBg, (uint32_t)q) * 8u;
      bp += bldv(rV, g8, 2 * N8);
      bq += bldv(rV, g8, 2 * N8 + G8);
    }
    constexpr int U = 4;
    for (int aa = q0; aa < q1; aa += U) {
      int ad[U];
      double fp[U], fq[U];
#pragma unroll
      for (int u = 0; u < U; ++u) ad[u] = aa + u < q1 ? bldi(rAdj, (uint32_t)(aa + u)) : -1;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t o = ad[u] < 0 ? 0u : (uint32_t)(ad[u] >> 1) * 8u + ((ad[u] & 1) ? 2u * B8 : 0u);
        fp[u] = ad[u] < 0 ? 0.0 : bldv(rV, o, xFL8);
        fq[u] = ad[u] < 0 ? 0.0 : bldv(rV, o, xFL8 + B8);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ad[u] < 0) break;
        bp -= fp[u];
        bq -= fq[u];
      }
    }
    const rsrc_t rO = rsrc(out + I.c_off + (int64_t)t * I.m_p);
    const double vref = n == I.ref ? bldv(rV, vN, N8) : 0.0;
    bstvn(rO, vN, 0, bp);
    bstvn(rO, vN, N8, bq);
    if (n == I.ref) bstn(rO, (uint32_t)b.cREF, vref);
  }
}

__global__ void __launch_bounds__(512) k_jv(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                            int ntiles, const double* __restrict__ x, const double* __restrict__ v,
                                            double* __restrict__ out) {
  for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
    const Tile tl = tiles[remap_tile(w, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int e = tl.e0 + (int)threadIdx.x;
    if (e >= tl.e1) continue;
    if (tl.kind == TK_BRANCH) {
      jv_branch(I, e, tl.t0, tl.t1, x, v, out);
    } else if (tl.kind == TK_BUS) {
      jv_bus(I, e, tl.t0, tl.t1, v, out);
    } else {
      const int64_t pg = 2LL * I.N + e;
      for (int t = tl.t0 < 1 ? 1 : tl.t0; t < tl.t1; ++t) {
        const double* vp = v + I.x_off + (int64_t)t * I.n_p;
        out[I.c_off + (int64_t)I.T * I.m_p + (int64_t)(t - 1) * I.G + e] = vp[pg] - vp[pg - I.n_p];
      }
    }
  }
}

// ------------------------------------------------- lifted-KKT condensation
// Barrier terms of one box lo <= val <= hi (Sec. III-B): sigma = z_lo / gap_lo
// + z_hi / gap_hi, the complementarity residuals z_lo gap_lo - mu and
// z_hi gap_hi - mu, and the gaps.  An infinite bound is absent: its
// multiplier is taken as 0, its gap as 1 and its residual as 0.
struct BoxTerms {
  double sig, plo, phi, glo, ghi, zlo, zhi;
  bool hlo, hhi;
};

__device__ __forceinline__ BoxTerms box_terms(double val, double lo, double hi, double zlo, double zhi,
                                              double mu) {
  BoxTerms b;
  b.hlo = __builtin_isfinite(lo);
  b.hhi = __builtin_isfinite(hi);
  b.glo = b.hlo ? val - lo : 1.0;
  b.ghi = b.hhi ? hi - val : 1.0;
  b.zlo = b.hlo ? zlo : 0.0;
  b.zhi = b.hhi ? zhi : 0.0;
  b.sig = b.zlo / b.glo + b.zhi / b.ghi;
  b.plo = b.hlo ? b.zlo * b.glo - mu : 0.0;
  b.phi = b.hhi ? b.zhi * b.ghi - mu : 0.0;
  return b;
}

// Row-space terms: q_s = p_s + p_lo / gap_lo - p_hi / gap_hi with
// p_s = -z_lo + z_hi + y, q_y = c - s, C = 1 / (dc sigma + 1 + dc dw).
struct RowTerms {
  BoxTerms b;
  double qs, qy, C;
};

__device__ __forceinline__ RowTerms row_terms(const IpmDev& st, int64_t r, double cr) {
  RowTerms R;
  const double sr = st.s[r], yr = st.y[r];
  R.b = box_terms(sr, st.sl[r], st.su[r], st.vl[r], st.vu[r], st.mu);
  const double ps = -R.b.zlo + R.b.zhi + yr;
  R.qy = cr - sr;
  R.qs = ps + R.b.plo / R.b.glo - R.b.phi / R.b.ghi;
  R.C = 1.0 / (st.dc * R.b.sig + (1.0 + st.dc * st.dw));
  return R;
}

// Rows: D and the vector w = C q_s + D q_y - y whose transposed product
// with J gives A^T (C q_s + D q_y) - A^T y.
__global__ void __launch_bounds__(256) k_rhs_rows(int64_t m, IpmDev st, const double* __restrict__ c,
                                                  double* __restrict__ dcon, double* __restrict__ w) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    const RowTerms R = row_terms(st, r, c[r]);
    const double D = (R.b.sig + st.dw) * R.C;
    dcon[r] = D;
    w[r] = R.C * R.qs + D * R.qy - st.y[r];
  }
}

// Variables: diag_x = dw + Sigma_x and rhs = q_x + (J^T w) with
// q_x (without its -A^T y term, carried by w) = grad - z_lo + z_hi
// + p_lo / gap_lo - p_hi / gap_hi; rhs holds J^T w on entry.
__global__ void __launch_bounds__(256) k_rhs_vars(int64_t n, IpmDev st, const double* __restrict__ grad,
                                                  double* __restrict__ diag_x, double* __restrict__ rhs) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const BoxTerms b = box_terms(st.x[i], st.xl[i], st.xu[i], st.zl[i], st.zu[i], st.mu);
    diag_x[i] = st.dw + b.sig;
    const double qx = grad[i] - b.zlo + b.zhi + b.plo / b.glo - b.phi / b.ghi;
    rhs[i] = qx + rhs[i];
  }
}

// Recovery, rows: ds = C (A dx + dc q_s - q_y), dy = (Sigma_s + dw) ds - q_s,
// and the slack-bound multiplier steps.
__global__ void __launch_bounds__(256) k_rec_rows(int64_t m, IpmDev st, const double* __restrict__ c,
                                                  const double* __restrict__ adx, double* __restrict__ ds,
                                                  double* __restrict__ dy, double* __restrict__ dvl,
                                                  double* __restrict__ dvu) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    const RowTerms R = row_terms(st, r, c[r]);
    const double d = R.C * (adx[r] + st.dc * R.qs - R.qy);
    ds[r] = d;
    dy[r] = (R.b.sig + st.dw) * d - R.qs;
    dvl[r] = R.b.hlo ? (-R.b.zlo * d + R.b.plo) / R.b.glo : 0.0;
    dvu[r] = R.b.hhi ? (R.b.zhi * d + R.b.phi) / R.b.ghi : 0.0;
  }
}

// Recovery, variables: the bound-multiplier steps of x.
__global__ void __launch_bounds__(256) k_rec_vars(int64_t n, IpmDev st, const double* __restrict__ dx,
                                                  double* __restrict__ dzl, double* __restrict__ dzu) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const BoxTerms b = box_terms(st.x[i], st.xl[i], st.xu[i], st.zl[i], st.zu[i], st.mu);
    const double d = dx[i];
    dzl[i] = b.hlo ? (-b.zlo * d + b.plo) / b.glo : 0.0;
    dzu[i] = b.hhi ? (b.zhi * d + b.phi) / b.ghi : 0.0;
  }
}

// ---------------------------------------------------------------- gradient
__global__ void __launch_bounds__(512) k_grad(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                              int ntiles, const double* __restrict__ x, double* __restrict__ gv) {
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int e = tl.e0 + (int)threadIdx.x;
    if (e >= tl.e1) continue;
    const int64_t PG = 2LL * I.N;
    const bool is_pg = e >= PG && e < PG + I.G;
    const double c2 = is_pg ? I.c2[e - PG] : 0.0, c1 = is_pg ? I.c1[e - PG] : 0.0;
    for (int t = tl.t0; t < tl.t1; ++t) {
      const int64_t idx = I.x_off + (int64_t)t * I.n_p + e;
      gv[idx] = is_pg ? 2.0 * c2 * x[idx] + c1 : 0.0;
    }
  }
}

// ---------------------------------------------------------------- objective
// Pass 1: per tile, a fixed-order block tree sum of c2 p^2 + c1 p + c0.
// Block 0 also clears zero[0 .. nzero) (the counters of the one-launch
// sweep, which follows this kernel).
__global__ void __launch_bounds__(512) k_obj_partial(const InstDev* __restrict__ insts,
                                                     const Tile* __restrict__ tiles, int ntiles,
                                                     const double* __restrict__ x, double* __restrict__ partial,
                                                     int32_t* __restrict__ zero, int nzero) {
  __shared__ double red[512];
  if (blockIdx.x == 0)
    for (int i = (int)threadIdx.x; i < nzero; i += blockDim.x) zero[i] = 0;
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const int ti = remap_tile(v, ntiles);
    const Tile tl = tiles[ti];
    const InstDev& I = insts[tl.inst];
    const int e = tl.e0 + (int)threadIdx.x;
    double acc = 0.0;
    if (e < tl.e1) {
      const double c2 = I.c2[e], c1 = I.c1[e], c0 = I.c0[e];
      for (int t = tl.t0; t < tl.t1; ++t) {
        const double p = x[I.x_off + (int64_t)t * I.n_p + 2LL * I.N + e];
        acc += c2 * p * p + c1 * p + c0;
      }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[ti] = red[0];
    __syncthreads();
  }
}

// Pass 2: one block per instance sums that instance's tile partials in a
// fixed order (strided per lane, then a tree).
__global__ void __launch_bounds__(256) k_obj_final(const int32_t* __restrict__ begin,
                                                   const double* __restrict__ partial, double* __restrict__ f) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  const int a = begin[k], z = begin[k + 1];
  double acc = 0.0;
  for (int q = a + (int)threadIdx.x; q < z; q += blockDim.x) acc += partial[q];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) f[k] = red[0];
}

// ---------------------------------------------------------------- J^T v
// Phase A: lines write their four flow-variable outputs and hand the bus
// contributions (vm_i, vm_j, va_i, va_j) to a per-line scratch record;
// generators write pg / qg.  Phase B: buses gather their incident records.
__device__ void jt_branch(const InstDev& I, int l, int t0, int t1, const double* __restrict__ x,
                          const double* __restrict__ vv_, double* __restrict__ out, double* __restrict__ scr) {
  const Bases b(I);
  Coef cf;
  load_coef(I, l, cf);
  const uint32_t B8 = (uint32_t)b.B * 8u, N8 = (uint32_t)b.N * 8u, vL = (uint32_t)l * 8u;
  const uint32_t xFL8 = (uint32_t)b.xFL * 8u, cFLOW8 = (uint32_t)b.cFLOW * 8u, cTHF8 = (uint32_t)b.cTHF * 8u,
                 cTHT8 = (uint32_t)b.cTHT * 8u, cANG8 = (uint32_t)b.cANG * 8u;
  const uint32_t vI = (uint32_t)I.f_bus[l] * 8u, vJ = (uint32_t)I.t_bus[l] * 8u;
  // x: vi, vj, ti, tj, flows; v: flow rows, thermal rows, angle row, balance rows at both ends
  double in[19];
  auto load = [&](int t, double* w) {
    const rsrc_t rX = rsrc(x + I.x_off + (int64_t)t * I.n_p), rV = rsrc(vv_ + I.c_off + (int64_t)t * I.m_p);
    w[0] = bldv(rX, vI, 0);
    w[1] = bldv(rX, vJ, 0);
    w[2] = bldv(rX, vI, N8);
    w[3] = bldv(rX, vJ, N8);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      w[4 + k] = bldv(rX, vL, xFL8 + (uint32_t)k * B8);
      w[8 + k] = bldv(rV, vL, cFLOW8 + (uint32_t)k * B8);
    }
    w[12] = bldv(rV, vL, cTHF8);
    w[13] = bldv(rV, vL, cTHT8);
    w[14] = bldv(rV, vL, cANG8);
    w[15] = bldv(rV, vI, 0);
    w[16] = bldv(rV, vI, N8);
    w[17] = bldv(rV, vJ, 0);
    w[18] = bldv(rV, vJ, N8);
  };
  load(t0, in);
  for (int t = t0; t < t1; ++t) {
    const double vi = in[0], vj = in[1], ti = in[2], tj = in[3];
    double fl[4], vk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      fl[k] = in[4 + k];
      vk[k] = in[8 + k];
    }
    const double vtf = in[12], vtt = in[13], vang = in[14];
    const double vbal[4] = {in[15], in[16], in[17], in[18]};
    if (t + 1 < t1) load(t + 1, in);
    double Jf[4][5], h[9];
    double s, c;
    sincos(ti - tj, &s, &c);
    const double vv = vi * vj;
#pragma unroll
    for (int k = 0; k < 4; ++k) flow_kind(cf, k, vi, vj, vv, s, c, 0.0, Jf[k], h);
    double o4[4], rec[4];
    jt_line(vk, Jf, vtf, vtt, vang, fl, vbal, o4, rec);
    const rsrc_t rO = rsrc(out + I.x_off + (int64_t)t * I.n_p);
#pragma unroll
    for (int k = 0; k < 4; ++k) bstvn(rO, vL, xFL8 + (uint32_t)k * B8, o4[k]);
    const rsrc_t rR = rsrc(jt_at(I, scr, t));
    bst2v(rR, vL * (uint32_t)kScratchJt, 0, make_double2(rec[0], rec[1]));
    bst2v(rR, vL * (uint32_t)kScratchJt, 16, make_double2(rec[2], rec[3]));
  }
}

// J^T v on the generator variables of one period: pg enters its balance row
// (+1) and the ramp rows of periods t (+1) and t + 1 (-1); qg its balance row.
__device__ __forceinline__ void jt_gen_period(const InstDev& I, int g, int n, int t, const double* __restrict__ vv_,
                                              double* __restrict__ out) {
  const int64_t N = I.N, G = I.G;
  const double* vr = vv_ + I.c_off + (int64_t)I.T * I.m_p;
  const double* vp = vv_ + I.c_off + (int64_t)t * I.m_p;
  double* op = out + I.x_off + (int64_t)t * I.n_p;
  double a = vp[n];
  if (t >= 1) a += vr[(int64_t)(t - 1) * G + g];
  if (t + 1 < I.T) a -= vr[(int64_t)t * G + g];
  op[2 * N + g] = a;
  op[2 * N + G + g] = vp[N + n];
}

__device__ void jt_gen(const InstDev& I, int g, int t0, int t1, const double* __restrict__ vv_,
                       double* __restrict__ out) {
  const int n = I.gen_bus[g];
  for (int t = t0; t < t1; ++t) jt_gen_period(I, g, n, t, vv_, out);
}

__global__ void __launch_bounds__(512) k_jt_a(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                              int ntiles, const double* __restrict__ x,
                                              const double* __restrict__ v, double* __restrict__ out,
                                              double* __restrict__ scr) {
  for (int q = blockIdx.x; q < ntiles; q += gridDim.x) {
    const Tile tl = tiles[remap_tile(q, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int e = tl.e0 + (int)threadIdx.x;
    if (e >= tl.e1) continue;
    if (tl.kind == TK_BRANCH)
      jt_branch(I, e, tl.t0, tl.t1, x, v, out, scr);
    else
      jt_gen(I, e, tl.t0, tl.t1, v, out);
  }
}

__global__ void __launch_bounds__(512) k_jt_b(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                              int ntiles, const double* __restrict__ v, double* __restrict__ out,
                                              const double* __restrict__ scr) {
  for (int q = blockIdx.x; q < ntiles; q += gridDim.x) {
    const Tile tl = tiles[remap_tile(q, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int n = tl.e0 + (int)threadIdx.x;
    if (n >= tl.e1) continue;
    const int q0 = I.bus_ptr[n], q1 = I.bus_ptr[n + 1];
    const rsrc_t rAdj = rsrc(I.bus_adj);
    const uint32_t vN = (uint32_t)n * 8u, N8 = (uint32_t)I.N * 8u;
    for (int t = tl.t0; t < tl.t1; ++t) {
      // the line's 4-value record: J^T v on vm_i, vm_j, va_i, va_j
      const rsrc_t rR = rsrc(jt_at(I, const_cast<double*>(scr), t));
      double svm = 0.0, sva = 0.0;
      constexpr int U = 4;
      for (int aa = q0; aa < q1; aa += U) {
        int ad[U];
        double rm[U], ra[U];
#pragma unroll
        for (int u = 0; u < U; ++u) ad[u] = aa + u < q1 ? bldi(rAdj, (uint32_t)(aa + u)) : -1;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t o = ad[u] < 0 ? 0u : (uint32_t)(ad[u] >> 1) * (uint32_t)(kScratchJt * 8) + ((ad[u] & 1) ? 8u : 0u);
          rm[u] = ad[u] < 0 ? 0.0 : bldv(rR, o, 0);
          ra[u] = ad[u] < 0 ? 0.0 : bldv(rR, o, 16);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (ad[u] < 0) break;
          svm += rm[u];
          sva += ra[u];
        }
      }
      if (n == I.ref) sva += v[I.c_off + (int64_t)t * I.m_p + 2LL * I.N];
      const rsrc_t rO = rsrc(out + I.x_off + (int64_t)t * I.n_p);
      bstvn(rO, vN, 0, svm);
      bstvn(rO, vN, N8, sva);
    }
  }
}

// ---------------------------------------------------------------- condensed
// K = lower(H + diag(diag_x) + J^T diag(d) J) on the fixed CSR.
//
// Line phase: a block owns the four flow-variable rows of K of its lines,
// one kind at a time.  Those rows are contiguous in K (rows are in x order),
// so the block first builds the kind's row segment in LDS (owner lane per
// row: the four bus-variable pairs of its flow row, the thermal partner,
// the diagonal, and for every balance-row partner d_bal * J_bal times the
// partner's J entry) and then streams the segment to HBM with consecutive
// lanes on consecutive slots.  Each line also sums its contributions to the
// bus-variable slots it touches into one 64-byte record per line end (the
// layout is described with rec_at) plus the shared cross pair.
// Generators own the pg / qg rows (balance partners, the ramp pair of
// t >= 1, diagonal).
// Bus phase: a bus owns its vm and va rows; one pass over its incident line
// ends (sorted by neighbour) sums the records, merging parallel lines, into
// an LDS copy of the block's row segments, streamed out the same way.
//
// One generator of the condensed assembly over its tile's periods: the pg
// and qg rows of K from the given J / H values.
__device__ void kkt_gen(const InstDev& I, int g, int t0, int t1, const double* __restrict__ H,
                        const double* __restrict__ J, const double* __restrict__ DX, const double* __restrict__ D,
                        double* __restrict__ K) {
  const int64_t N = I.N, G = I.G;
  const int n = I.gen_bus[g];
  const int64_t rp = 2 * N + g, rq = 2 * N + G + g;
  const int ps = I.krow[rp], pe = I.krow[rp + 1], qs = I.krow[rq], qe = I.krow[rq + 1];
  const double* jr = J + I.j_off + (int64_t)I.T * I.nnzj_p;  // ramp block of J
  const double* dr = D + I.c_off + (int64_t)I.T * I.m_p;     // ramp rows of D
  for (int t = t0; t < t1; ++t) {
    const double* jp = J + I.j_off + (int64_t)t * I.nnzj_p;
    const double* dp = D + I.c_off + (int64_t)t * I.m_p;
    double* kb = K + I.k_off + kkt_period_offset_dev(I.nnzk_p, I.G, t);
    const double Jgp = jp[g], Jgq = jp[G + g], Hg = H[I.h_off + (int64_t)t * I.nnzh_p + g];
    const double pbp = dp[n] * Jgp, pbq = dp[N + n] * Jgq;
    const int64_t xo = I.x_off + (int64_t)t * I.n_p;
    double diag = (DX ? DX[xo + rp] : 0.0) + pbp * Jgp + Hg;
    const int sp = t >= 1 ? g + 1 : 0, sq = t >= 1 ? (int)G : 0;
    if (t >= 1) {
      const double* jt = jr + (int64_t)(t - 1) * 2 * G;
      const double d = dr[(int64_t)(t - 1) * G + g];
      const double j0 = jt[g], j1 = jt[G + g];
      kb[ps + g] = d * j0 * j1;
      diag += d * j0 * j0;
    }
    if (t + 1 < I.T) {
      const double j1 = jr[(int64_t)t * 2 * G + G + g];
      diag += dr[(int64_t)t * G + g] * j1 * j1;
    }
    // balance partners of a generator row are generators
    for (int p = ps; p < pe - 1; ++p) kb[p + sp] = pbp * jp[I.ksrc[p]];
    kb[pe - 1 + sp] = diag;
    for (int p = qs; p < qe - 1; ++p) kb[p + sq] = pbq * jp[I.ksrc[p]];
    kb[qe - 1 + sq] = (DX ? DX[xo + rq] : 0.0) + pbq * Jgq;
  }
}

// One generator of the fused evaluation over its tile's periods: J, H and
// the generator rows of K (balance partners are generators, J = +1), and
// with SWEEP the ramp row, J^T v and gradient entries of pg / qg.  Loads of
// a period come before its stores (in-order completion counting), and the
// output streams use non-temporal stores; values are the same expressions
// as kkt_gen's.
template <bool SWEEP>
__device__ double fused_gen(const InstDev& I, int g, int t0, int t1, double sigma, double* __restrict__ H,
                          double* __restrict__ J, const double* __restrict__ DX, const double* __restrict__ D,
                          double* __restrict__ K, const double* __restrict__ X, const double* __restrict__ V,
                          double* __restrict__ C, double* __restrict__ JTV, double* __restrict__ GR) {
  const int64_t N = I.N, G = I.G;
  const int n = I.gen_bus[g];
  const int64_t rp = 2 * N + g, rq = 2 * N + G + g;
  const int ps = I.krow[rp], pe = I.krow[rp + 1], qs = I.krow[rq], qe = I.krow[rq + 1];
  double* jr = J + I.j_off + (int64_t)I.T * I.nnzj_p;   // ramp block of J
  const double* dr = D + I.c_off + (int64_t)I.T * I.m_p;  // ramp rows of D
  const double hobj = 2.0 * sigma * I.c2[g];
  const double c2g = SWEEP ? I.c2[g] : 0.0, c1g = SWEEP ? I.c1[g] : 0.0, c0g = SWEEP ? I.c0[g] : 0.0;
  const double* vr = SWEEP ? V + I.c_off + (int64_t)I.T * I.m_p : nullptr;
  double obj = 0.0;  // SWEEP: sum over the periods of c2 pg^2 + c1 pg + c0
  for (int t = t0; t < t1; ++t) {
    double* jp = J + I.j_off + (int64_t)t * I.nnzj_p;
    const double* dp = D + I.c_off + (int64_t)t * I.m_p;
    double* kb = K + I.k_off + kkt_period_offset_dev(I.nnzk_p, I.G, t);
    const int64_t xo = I.x_off + (int64_t)t * I.n_p;
    const int64_t co = I.c_off + (int64_t)t * I.m_p;
    const bool up = t >= 1, dn = t + 1 < I.T;
    // ---- loads
    const double dpn = dp[n], dqn = dp[N + n];
    const double dxp = DX ? DX[xo + rp] : 0.0, dxq = DX ? DX[xo + rq] : 0.0;
    const double drm = up ? dr[(int64_t)(t - 1) * G + g] : 0.0, drp = dn ? dr[(int64_t)t * G + g] : 0.0;
    double xg = 0.0, xgm = 0.0, vpn = 0.0, vqn = 0.0, vrm = 0.0, vrp = 0.0;
    if constexpr (SWEEP) {
      xg = X[xo + rp];
      xgm = up ? X[xo + rp - I.n_p] : 0.0;
      vpn = V[co + n];
      vqn = V[co + N + n];
      vrm = up ? vr[(int64_t)(t - 1) * G + g] : 0.0;
      vrp = dn ? vr[(int64_t)t * G + g] : 0.0;
    }
    // ---- stores
    const double Jgp = 1.0, Jgq = 1.0, Hg = hobj;
    __builtin_nontemporal_store(Jgp, jp + g);
    __builtin_nontemporal_store(Jgq, jp + G + g);
    if (g == 0) __builtin_nontemporal_store(1.0, jp + 2 * G + 4LL * I.B);  // reference-angle row
    __builtin_nontemporal_store(Hg, H + I.h_off + (int64_t)t * I.nnzh_p + g);
    if (up) {
      double* jt = jr + (int64_t)(t - 1) * 2 * G;
      __builtin_nontemporal_store(1.0, jt + g);
      __builtin_nontemporal_store(-1.0, jt + G + g);
    }
    const double pbp = dpn * Jgp, pbq = dqn * Jgq;
    double diag = dxp + pbp * Jgp + Hg;
    const int sp = up ? g + 1 : 0, sq = up ? (int)G : 0;
    if (up) {
      const double j0 = 1.0, j1 = -1.0;
      __builtin_nontemporal_store(drm * j0 * j1, kb + ps + g);
      diag += drm * j0 * j0;
    }
    if (dn) {
      const double j1 = -1.0;
      diag += drp * j1 * j1;
    }
    // balance partners of a generator row are generators (J = +1)
    for (int p = ps; p < pe - 1; ++p) __builtin_nontemporal_store(pbp * 1.0, kb + p + sp);
    __builtin_nontemporal_store(diag, kb + pe - 1 + sp);
    for (int p = qs; p < qe - 1; ++p) __builtin_nontemporal_store(pbq * 1.0, kb + p + sq);
    __builtin_nontemporal_store(dxq + pbq * Jgq, kb + qe - 1 + sq);
    if constexpr (SWEEP) {
      if (up) __builtin_nontemporal_store(xg - xgm, C + I.c_off + (int64_t)I.T * I.m_p + (int64_t)(t - 1) * G + g);
      double a = vpn;
      if (up) a += vrm;
      if (dn) a -= vrp;
      __builtin_nontemporal_store(a, JTV + xo + 2 * N + g);
      __builtin_nontemporal_store(vqn, JTV + xo + 2 * N + G + g);
      __builtin_nontemporal_store(2.0 * c2g * xg + c1g, GR + xo + rp);
      __builtin_nontemporal_store(0.0, GR + xo + rq);
      obj += c2g * xg * xg + c1g * xg + c0g;
    }
  }
  return obj;
}

// Streams a K row segment from LDS to HBM with consecutive lanes on
// consecutive slots.  GATHER: a slot whose template source is a J entry (a
// balance partner) holds the factor d_bal * J_bal and is multiplied by that
// entry.
template <bool GATHER, bool NT = false>
__device__ __forceinline__ void stream_segment(const double* __restrict__ seg, rsrc_t src, rsrc_t jp, double* dst,
                                               int len) {
  // GATHER: the template loads and J gathers of up to U slots per lane are
  // all issued before the first store (in-order completion counting).
  // Lane i writes slot i - d, d = the destination's offset inside its 64-byte
  // line, so every wave's stores cover whole lines except at the ends of the
  // segment (partial-line writes cost far more than their bytes).
  constexpr int U = GATHER ? 12 : 4;
  const int d = (int)(((uintptr_t)dst >> 3) & 7);
  const rsrc_t rd = rsrc(dst - d);
  const int bd = (int)blockDim.x;
  for (int p0 = (int)threadIdx.x; p0 < len + d; p0 += U * bd) {
    int sr[U];
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * bd - d;
      const bool ok = p >= 0 && p < len;
      sr[u] = (GATHER && ok) ? bldi(src, (uint32_t)p) : -2;
      v[u] = ok ? seg[p] : 0.0;
    }
    if (GATHER) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (sr[u] >= 0) v[u] *= bld(jp, (uint32_t)sr[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * bd - d;
      if (p >= 0 && p < len) {
        if (NT) bstn(rd, (uint32_t)(p + d), v[u]);
        else bst(rd, (uint32_t)(p + d), v[u]);
      }
    }
  }
}

// Hand-off records of a line tile through LDS: lane l leaves its line's 16
// values (two 64-byte end records) at a padded stride, then the block's
// records, contiguous in memory for lines e0 .. e1, are streamed out with
// consecutive lanes on consecutive 16-byte chunks (whole cache lines per
// wave instead of one partial line per lane).  Ends with a barrier, so the
// LDS region is free again.
__device__ __forceinline__ void stream_records(double* __restrict__ seg, int nl, rsrc_t dst) {
  __syncthreads();
  const int bd = (int)blockDim.x;
  for (int p = (int)threadIdx.x; p < nl * (kRecLine / 2); p += bd) {
    const int ln = p / (kRecLine / 2), c = (p % (kRecLine / 2)) * 2;
    bst2v(dst, (uint32_t)p * 16u, 0, make_double2(seg[ln * kRecLds + c], seg[ln * kRecLds + c + 1]));
  }
  __syncthreads();
}

// One line tile of the condensed assembly from given J and H values.  All
// J / H / weight loads of a line-period are issued before its first store
// (completions are counted in order); the four flow kinds then build their
// K rows one after the other in an LDS copy of the block's row segment,
// which is streamed out with consecutive lanes on consecutive slots, the
// balance-partner slots multiplied by the partner's J entry on the way.
__device__ void kkt_line_tile(const InstDev& I, const Tile& tl, const double* __restrict__ H,
                              const double* __restrict__ J, const double* __restrict__ DX,
                              const double* __restrict__ D, double* __restrict__ K, double* __restrict__ scr,
                              double* __restrict__ seg) {
  const Bases b(I);
  const uint32_t B8 = (uint32_t)b.B * 8u, G = (uint32_t)b.G;
  const uint32_t xFL8 = (uint32_t)b.xFL * 8u, jFLOW8 = (uint32_t)b.jFLOW * 8u, jBAL8 = (uint32_t)b.jBAL * 8u,
                 jTH8 = (uint32_t)b.jTH * 8u, jANG8 = (uint32_t)b.jANG * 8u, hFLOW8 = (uint32_t)b.hFLOW * 8u,
                 hTH8 = (uint32_t)b.hTH * 8u, cFLOW8 = (uint32_t)b.cFLOW * 8u, cTHF8 = (uint32_t)b.cTHF * 8u,
                 cTHT8 = (uint32_t)b.cTHT * 8u, cANG8 = (uint32_t)b.cANG * 8u, N8 = (uint32_t)b.N * 8u;
  const int tid = (int)threadIdx.x;
  const uint32_t l = (uint32_t)(tl.e0 + tid);
  const bool act = (int)l < tl.e1;
  const uint32_t vL = l * 8u, vL4 = l * 4u;
  const rsrc_t rKrow = rsrc(I.krow), rKsrc = rsrc(I.ksrc);
  const uint32_t FL4 = (uint32_t)b.xFL * 4u, Bq = (uint32_t)b.B * 4u;
  int sb[4], se[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    sb[k] = __builtin_amdgcn_readfirstlane(bldi(rKrow, (uint32_t)b.xFL + (uint32_t)k * (uint32_t)b.B + tl.e0));
    se[k] = __builtin_amdgcn_readfirstlane(bldi(rKrow, (uint32_t)b.xFL + (uint32_t)k * (uint32_t)b.B + tl.e1));
  }
  uint32_t vI = 0, vJ = 0;
  bool ilo = true;
  int rs[4] = {0, 0, 0, 0}, re[4] = {0, 0, 0, 0}, th[4] = {0xFFFF, 0xFFFF, 0xFFFF, 0xFFFF};
  if (act) {
    const int i = bldi(rsrc(I.f_bus), l), j = bldi(rsrc(I.t_bus), l);
    ilo = i < j;
    vI = (uint32_t)i * 8u;
    vJ = (uint32_t)j * 8u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      rs[k] = bldiv(rKrow, vL4, FL4 + (uint32_t)k * Bq) - sb[k];
      re[k] = bldiv(rKrow, vL4, FL4 + (uint32_t)k * Bq + 4u) - sb[k];
      th[k] = (int)((uint32_t)bldiv(rsrc(I.kinfo), vL4, (uint32_t)k * Bq) >> 16);
    }
  }
  for (int t = tl.t0; t < tl.t1; ++t) {
    const int64_t xo = I.x_off + (int64_t)t * I.n_p;
    const int64_t co = I.c_off + (int64_t)t * I.m_p;
    const rsrc_t rJ = rsrc(J + I.j_off + (int64_t)t * I.nnzj_p);
    const rsrc_t rH = rsrc(H + I.h_off + (int64_t)t * I.nnzh_p);
    const rsrc_t rD = rsrc(D + co);
    double* kbase = K + I.k_off + kkt_period_offset_dev(I.nnzk_p, I.G, t) + (t >= 1 ? G : 0);
    // ---- every load of this line-period
    double Jf[4][5], Hf[4][9], Jb[4], Jt[4], Hth[4], dfk[4], dbk[4], dxk[4], dth[2] = {0.0, 0.0};
    double Ja0 = 0.0, Ja1 = 0.0, dang = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Jb[k] = Jt[k] = Hth[k] = dfk[k] = dbk[k] = dxk[k] = 0.0;
#pragma unroll
      for (int a = 0; a < 5; ++a) Jf[k][a] = 0.0;
#pragma unroll
      for (int a = 0; a < 9; ++a) Hf[k][a] = 0.0;
    }
    if (act) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t kB8 = (uint32_t)k * B8;
#pragma unroll
        for (int a = 0; a < 5; ++a) Jf[k][a] = bldv(rJ, vL, jFLOW8 + (uint32_t)(k * 5 + a) * B8);
#pragma unroll
        for (int a = 0; a < 9; ++a) Hf[k][a] = bldv(rH, vL, hFLOW8 + (uint32_t)(k * 9 + a) * B8);
        Jb[k] = bldv(rJ, vL, jBAL8 + kB8);
        Jt[k] = bldv(rJ, vL, jTH8 + kB8);
        Hth[k] = bldv(rH, vL, hTH8 + kB8);
        dfk[k] = bldv(rD, vL, cFLOW8 + kB8);
        dbk[k] = bldv(rD, k < 2 ? vI : vJ, (k & 1) ? N8 : 0u);
      }
      if (DX) {
        const rsrc_t rDX = rsrc(DX + xo);
#pragma unroll
        for (int k = 0; k < 4; ++k) dxk[k] = bldv(rDX, vL, xFL8 + (uint32_t)k * B8);
      }
      dth[0] = bldv(rD, vL, cTHF8);
      dth[1] = bldv(rD, vL, cTHT8);
      dang = bldv(rD, vL, cANG8);
      Ja0 = bldv(rJ, vL, jANG8);
      Ja1 = bldv(rJ, vL, jANG8 + B8);
    }
    double q[10];
#pragma unroll
    for (int a = 0; a < 10; ++a) q[a] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (act) {
        const double* Jk = Jf[k];
        const double* hf = Hf[k];
        const double a1 = Jk[1], a2 = Jk[2], a3 = Jk[3], a4 = Jk[4];
        const double dk = dfk[k];
        const double d1 = dk * a1, d2 = dk * a2, d3 = dk * a3, d4 = dk * a4;
        if (k < 2) {
          q[0] += d1 * a1 + hf[0];
          q[6] += d2 * a2;
          q[4] += d2 * a1 + hf[1];
        } else {
          q[0] += d1 * a1;
          q[6] += d2 * a2 + hf[1];
          q[4] += d2 * a1 + hf[0];
        }
        q[1] += d3 * a1 + hf[2];
        q[3] += d3 * a2 + hf[3];
        q[2] += d3 * a3 + hf[4];
        q[9] += d4 * a1 + hf[5];
        q[7] += d4 * a2 + hf[6];
        q[5] += d4 * a3 + hf[7];
        q[8] += d4 * a4 + hf[8];
        const double pk = dk * Jk[0];
        double* row = seg + rs[k];
        if (ilo) {
          row[0] = pk * Jk[1];
          row[1] = pk * Jk[2];
          row[2] = pk * Jk[3];
          row[3] = pk * Jk[4];
        } else {
          row[0] = pk * Jk[2];
          row[1] = pk * Jk[1];
          row[2] = pk * Jk[4];
          row[3] = pk * Jk[3];
        }
        // partners: the factor d_bal J_bal (the stream-out multiplies by the
        // partner's J entry), or the thermal pair of odd kinds
        const double pb = dbk[k] * Jb[k];
        const double thv = dth[k >> 1] * Jt[k ^ 1] * Jt[k];
        for (int p = 0; p < re[k] - rs[k] - 5; ++p) seg[rs[k] + 4 + p] = p == th[k] ? thv : pb;
        seg[re[k] - 1] = dxk[k] + pk * Jk[0] + dth[k >> 1] * Jt[k] * Jt[k] + pb * Jb[k] + Hth[k];
      }
      __syncthreads();
      stream_segment<true, true>(seg, rsrc(I.ksrc + sb[k]), rJ, kbase + sb[k], se[k] - sb[k]);
      __syncthreads();
    }
    if (act) {
      q[2] += dang * Ja0 * Ja0;
      q[8] += dang * Ja1 * Ja1;
      q[5] += dang * Ja1 * Ja0;
      // records: the K sums of both ends (p, q and J^T v slots unused here)
      const double rec[kRecLine] = {q[0], q[1], q[2], q[3], 0.0, 0.0, 0.0, 0.0,
                                    q[6], q[7], q[8], q[9], 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < kRecLine; ++a) seg[tid * kRecLds + a] = rec[a];
      bst2v(rsrc(shared_at(I, scr, t)), vL * 2u, 0, make_double2(q[4], q[5]));
    }
    stream_records(seg, tl.e1 - tl.e0, rsrc(rec_at(I, scr, t) + (int64_t)tl.e0 * kRecLine));
  }
  (void)rKsrc;
}

// One line tile of the fused evaluation: J and H of the lines from x and
// lambda, written out and used directly for the flow rows of K (the partner
// J entries are the structural +1 / -1 of the balance rows); with SWEEP also
// the constraint rows, J^T v and gradient on the flow variables and the bus
// hand-off of p, q and J^T v.  Every load of a line-period is issued before
// its first store: vector-memory completions are counted in order, so a
// load issued after stores cannot be consumed before those stores are done.
// The partner kinds of each K flow row come from the template's per-row
// summary (leading generator partners, thermal slot), not from per-slot
// source indices.
template <bool SWEEP>
__device__ void fused_line_tile(const InstDev& I, const Tile& tl, const double* __restrict__ X,
                                const double* __restrict__ LAM, double* __restrict__ H, double* __restrict__ J,
                                const double* __restrict__ DX, const double* __restrict__ D, double* __restrict__ K,
                                double* __restrict__ scr, double* __restrict__ seg, double* sadm,
                                const double* __restrict__ V, double* __restrict__ C, double* __restrict__ JTV,
                                double* __restrict__ GR) {
  const Bases b(I);
  // element offsets inside one period block, as byte offsets (every period
  // block is far below 4 GiB)
  const uint32_t B8 = (uint32_t)b.B * 8u, N8 = (uint32_t)b.N * 8u, G = (uint32_t)b.G;
  const uint32_t xFL8 = (uint32_t)b.xFL * 8u, jFLOW8 = (uint32_t)b.jFLOW * 8u, jBAL8 = (uint32_t)b.jBAL * 8u,
                 jTH8 = (uint32_t)b.jTH * 8u, jANG8 = (uint32_t)b.jANG * 8u, hFLOW8 = (uint32_t)b.hFLOW * 8u,
                 hTH8 = (uint32_t)b.hTH * 8u, cFLOW8 = (uint32_t)b.cFLOW * 8u, cTHF8 = (uint32_t)b.cTHF * 8u,
                 cTHT8 = (uint32_t)b.cTHT * 8u, cANG8 = (uint32_t)b.cANG * 8u;
  const int tid = (int)threadIdx.x;
  const int bd = (int)blockDim.x;
  const uint32_t l = (uint32_t)(tl.e0 + tid);
  const bool act = (int)l < tl.e1;
  // lane offsets: every per-line stream is (uniform stream offset) + vL
  const uint32_t vL = l * 8u, vL4 = l * 4u;
  const rsrc_t rKrow = rsrc(I.krow);
  const uint32_t FL4 = (uint32_t)b.xFL * 4u, Bq = (uint32_t)b.B * 4u;
  int sb[4], se[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    sb[k] = __builtin_amdgcn_readfirstlane(bldi(rKrow, (uint32_t)b.xFL + (uint32_t)k * (uint32_t)b.B + tl.e0));
    se[k] = __builtin_amdgcn_readfirstlane(bldi(rKrow, (uint32_t)b.xFL + (uint32_t)k * (uint32_t)b.B + tl.e1));
  }
  // per-line constants of the tile: bus offsets, K row bounds and partner
  // summaries of the four flow rows, the admittances (into LDS)
  uint32_t vI = 0, vJ = 0;
  bool ilo = true;
  int rs[4] = {0, 0, 0, 0}, re[4] = {0, 0, 0, 0}, kinf[4] = {0, 0, 0, 0};
  if (act) {
    const int i = bldi(rsrc(I.f_bus), l), j = bldi(rsrc(I.t_bus), l);
    ilo = i < j;
    vI = (uint32_t)i * 8u;
    vJ = (uint32_t)j * 8u;
    const rsrc_t rA = rsrc(I.adm), rKi = rsrc(I.kinfo);
#pragma unroll
    for (int a = 0; a < 8; ++a) sadm[a * bd + tid] = bldv(rA, vL, (uint32_t)a * B8);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      rs[k] = bldiv(rKrow, vL4, FL4 + (uint32_t)k * Bq) - sb[k];
      re[k] = bldiv(rKrow, vL4, FL4 + (uint32_t)k * Bq + 4u) - sb[k];
      kinf[k] = bldiv(rKi, vL4, (uint32_t)k * Bq);
    }
  }
  for (int t = tl.t0; t < tl.t1; ++t) {
    const int64_t xo = I.x_off + (int64_t)t * I.n_p;
    const int64_t co = I.c_off + (int64_t)t * I.m_p;
    const rsrc_t rJ = rsrc(J + I.j_off + (int64_t)t * I.nnzj_p);
    const rsrc_t rH = rsrc(H + I.h_off + (int64_t)t * I.nnzh_p);
    const rsrc_t rD = rsrc(D + co), rX = rsrc(X + xo), rL = rsrc(LAM + co);
    double* kbase = K + I.k_off + kkt_period_offset_dev(I.nnzk_p, I.G, t) + (t >= 1 ? G : 0);
    // ---- every load of this line-period
    double vi = 0.0, vj = 0.0, ti = 0.0, tj = 0.0, fl[4] = {0.0, 0.0, 0.0, 0.0}, lf = 0.0, lt = 0.0;
    double dth[2] = {0.0, 0.0}, dang = 0.0, dfk[4], lamk[4], dbk[4], dxk[4], vk[4];
    double vtf = 0.0, vtt = 0.0, vang = 0.0, vbal[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) dfk[k] = lamk[k] = dbk[k] = dxk[k] = vk[k] = vbal[k] = 0.0;
    if (act) {
      vi = bldv(rX, vI, 0);
      vj = bldv(rX, vJ, 0);
      ti = bldv(rX, vI, N8);
      tj = bldv(rX, vJ, N8);
#pragma unroll
      for (int k = 0; k < 4; ++k) fl[k] = bldv(rX, vL, xFL8 + (uint32_t)k * B8);
      lf = 2.0 * bldv(rL, vL, cTHF8);
      lt = 2.0 * bldv(rL, vL, cTHT8);
      dth[0] = bldv(rD, vL, cTHF8);
      dth[1] = bldv(rD, vL, cTHT8);
      dang = bldv(rD, vL, cANG8);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        dfk[k] = bldv(rD, vL, cFLOW8 + (uint32_t)k * B8);
        lamk[k] = bldv(rL, vL, cFLOW8 + (uint32_t)k * B8);
        dbk[k] = bldv(rD, k < 2 ? vI : vJ, (k & 1) ? N8 : 0u);
      }
      if (DX) {
        const rsrc_t rDX = rsrc(DX + xo);
#pragma unroll
        for (int k = 0; k < 4; ++k) dxk[k] = bldv(rDX, vL, xFL8 + (uint32_t)k * B8);
      }
      if constexpr (SWEEP) {
        const rsrc_t rV = rsrc(V + co);
#pragma unroll
        for (int k = 0; k < 4; ++k) vk[k] = bldv(rV, vL, cFLOW8 + (uint32_t)k * B8);
        vtf = bldv(rV, vL, cTHF8);
        vtt = bldv(rV, vL, cTHT8);
        vang = bldv(rV, vL, cANG8);
        vbal[0] = bldv(rV, vI, 0);
        vbal[1] = bldv(rV, vI, N8);
        vbal[2] = bldv(rV, vJ, 0);
        vbal[3] = bldv(rV, vJ, N8);
      }
    }
    double sn = 0.0, cs = 0.0;
    sincos(ti - tj, &sn, &cs);
    const double vv = vi * vj;
    double q[10], Jt[4];
#pragma unroll
    for (int a = 0; a < 10; ++a) q[a] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) Jt[k] = 2.0 * fl[k];
    double svi = 0.0, svj = 0.0, sti = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t kB8 = (uint32_t)k * B8;
      if (act) {
        double Jk[5], hf[9];
        Coef cf;
        coef_kind_lds(sadm, bd, tid, k, cf);
        flow_kind(cf, k, vi, vj, vv, sn, cs, -lamk[k], Jk, hf);
#pragma unroll
        for (int a = 0; a < 5; ++a) bstvn(rJ, vL, jFLOW8 + (uint32_t)(k * 5 + a) * B8, Jk[a]);
#pragma unroll
        for (int a = 0; a < 9; ++a) bstvn(rH, vL, hFLOW8 + (uint32_t)(k * 9 + a) * B8, hf[a]);
        const double Jbk = -1.0;
        const double Hthk = k < 2 ? lf : lt;
        bstvn(rJ, vL, jBAL8 + kB8, Jbk);
        bstvn(rJ, vL, jTH8 + kB8, Jt[k]);
        bstvn(rH, vL, hTH8 + kB8, Hthk);
        if constexpr (SWEEP) {
          bstvn(rsrc(C + co), vL, cFLOW8 + kB8, fl[k] - flow_value(cf, k, vi, vj, vv, flow_w(cf, k, sn, cs)));
          svi += vk[k] * Jk[1];
          svj += vk[k] * Jk[2];
          sti += vk[k] * Jk[3];
        }
        // bus-variable contributions: d_k J_k,a J_k,b + H (local H order:
        // from end (0,0)(1,0)(2,0)(2,1)(2,2)(3,0)(3,1)(3,2)(3,3); to end
        // (1,0)(1,1)(2,0)(2,1)(2,2)(3,0)(3,1)(3,2)(3,3))
        const double a1 = Jk[1], a2 = Jk[2], a3 = Jk[3], a4 = Jk[4];
        const double dk = dfk[k];
        const double d1 = dk * a1, d2 = dk * a2, d3 = dk * a3, d4 = dk * a4;
        if (k < 2) {
          q[0] += d1 * a1 + hf[0];
          q[6] += d2 * a2;
          q[4] += d2 * a1 + hf[1];
        } else {
          q[0] += d1 * a1;
          q[6] += d2 * a2 + hf[1];
          q[4] += d2 * a1 + hf[0];
        }
        q[1] += d3 * a1 + hf[2];
        q[3] += d3 * a2 + hf[3];
        q[2] += d3 * a3 + hf[4];
        q[9] += d4 * a1 + hf[5];
        q[7] += d4 * a2 + hf[6];
        q[5] += d4 * a3 + hf[7];
        q[8] += d4 * a4 + hf[8];
        // this kind's K row into the LDS copy of the block's row segment
        const double pk = dk * Jk[0];
        double* row = seg + rs[k];
        if (ilo) {
          row[0] = pk * Jk[1];
          row[1] = pk * Jk[2];
          row[2] = pk * Jk[3];
          row[3] = pk * Jk[4];
        } else {
          row[0] = pk * Jk[2];
          row[1] = pk * Jk[1];
          row[2] = pk * Jk[4];
          row[3] = pk * Jk[3];
        }
        // partners: generators (+1) first, then line ends (-1), with the
        // thermal partner (odd kinds) at its summarised slot
        const double pb = dbk[k] * Jbk;
        const int ngen = kinf[k] & 0xFFFF, th = (int)((uint32_t)kinf[k] >> 16);
        const double thv = dth[k >> 1] * Jt[k ^ 1] * Jt[k];
        const double gv = pb * 1.0, lv = pb * -1.0;
        for (int p = 0; p < re[k] - rs[k] - 5; ++p) seg[rs[k] + 4 + p] = p == th ? thv : (p < ngen ? gv : lv);
        seg[re[k] - 1] = dxk[k] + pk * Jk[0] + dth[k >> 1] * Jt[k] * Jt[k] + pb * Jbk + Hthk;
      }
      __syncthreads();
      stream_segment<false, true>(seg, rKrow, rKrow, kbase + sb[k], se[k] - sb[k]);
      __syncthreads();
    }
    if (act) {
      const double Ja0 = 1.0, Ja1 = -1.0;
      bstvn(rJ, vL, jANG8, Ja0);
      bstvn(rJ, vL, jANG8 + B8, Ja1);
      q[2] += dang * Ja0 * Ja0;
      q[8] += dang * Ja1 * Ja1;
      q[5] += dang * Ja1 * Ja0;
      double jtr[4] = {0.0, 0.0, 0.0, 0.0};
      if constexpr (SWEEP) {
        const rsrc_t rC = rsrc(C + co), rO = rsrc(JTV + xo), rG = rsrc(GR + xo);
        bstvn(rC, vL, cTHF8, fl[0] * fl[0] + fl[1] * fl[1]);
        bstvn(rC, vL, cTHT8, fl[2] * fl[2] + fl[3] * fl[3]);
        bstvn(rC, vL, cANG8, ti - tj);
        bstvn(rO, vL, xFL8, vk[0] + vtf * (2.0 * fl[0]) - vbal[0]);
        bstvn(rO, vL, xFL8 + B8, vk[1] + vtf * (2.0 * fl[1]) - vbal[1]);
        bstvn(rO, vL, xFL8 + 2 * B8, vk[2] + vtt * (2.0 * fl[2]) - vbal[2]);
        bstvn(rO, vL, xFL8 + 3 * B8, vk[3] + vtt * (2.0 * fl[3]) - vbal[3]);
        jtr[0] = svi;
        jtr[1] = sti + vang;
        jtr[2] = svj;
        jtr[3] = -sti - vang;
#pragma unroll
        for (int k = 0; k < 4; ++k) bstvn(rG, vL, xFL8 + (uint32_t)k * B8, 0.0);
      }
      // hand-off: one 64-byte record per line end (through LDS), the shared
      // cross pair
      const double rec[kRecLine] = {q[0], q[1], q[2], q[3], fl[0], fl[1], jtr[0], jtr[1],
                                    q[6], q[7], q[8], q[9], fl[2], fl[3], jtr[2], jtr[3]};
#pragma unroll
      for (int a = 0; a < kRecLine; ++a) seg[tid * kRecLds + a] = rec[a];
      bst2v(rsrc(shared_at(I, scr, t)), vL * 2u, 0, make_double2(q[4], q[5]));
    }
    stream_records(seg, tl.e1 - tl.e0, rsrc(rec_at(I, scr, t) + (int64_t)tl.e0 * kRecLine));
  }
}

// Dynamic LDS: seg[cap_seg] doubles (the longest K row segment of a tile,
// at least the padded records of a block).
__global__ void __launch_bounds__(256) k_kkt_a(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                               int ntiles, int cap_seg, const double* __restrict__ H,
                                               const double* __restrict__ J, const double* __restrict__ DX,
                                               const double* __restrict__ D, double* __restrict__ K,
                                               double* __restrict__ scr) {
  extern __shared__ double lds[];
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    if (tl.kind == TK_BRANCH) {
      kkt_line_tile(I, tl, H, J, DX, D, K, scr, lds);
    } else {
      const int e = tl.e0 + (int)threadIdx.x;
      if (e < tl.e1) kkt_gen(I, e, tl.t0, tl.t1, H, J, DX, D, K);
    }
  }
}

// Fused form: J, H and the line / generator rows of K in one pass over x.
// Dynamic LDS: seg[cap_seg] doubles, then the lanes' admittances [8][blockDim].
__global__ void __launch_bounds__(256) k_jhk_a(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                               int ntiles, int cap_seg, const double* __restrict__ X,
                                               const double* __restrict__ LAM, double sigma, double* __restrict__ H,
                                               double* __restrict__ J, const double* __restrict__ DX,
                                               const double* __restrict__ D, double* __restrict__ K,
                                               double* __restrict__ scr) {
  extern __shared__ double lds[];
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    if (tl.kind == TK_BRANCH) {
      fused_line_tile<false>(I, tl, X, LAM, H, J, DX, D, K, scr, lds, lds + cap_seg, nullptr, nullptr, nullptr, nullptr);
    } else {
      const int e = tl.e0 + (int)threadIdx.x;
      if (e < tl.e1) fused_gen<false>(I, e, tl.t0, tl.t1, sigma, H, J, DX, D, K, nullptr, nullptr, nullptr, nullptr, nullptr);
    }
  }
}

// Whole sweep, lines and generators: J, H, K rows, constraint rows, J^T v and
// gradient entries of the line / generator variables in one pass over x.
// Dynamic LDS as in k_jhk_a.
__global__ void __launch_bounds__(256) k_sweep_a(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                                 int ntiles, int cap_seg, const double* __restrict__ X,
                                                 const double* __restrict__ LAM, double sigma,
                                                 const double* __restrict__ V, double* __restrict__ H,
                                                 double* __restrict__ J, const double* __restrict__ DX,
                                                 const double* __restrict__ D, double* __restrict__ K,
                                                 double* __restrict__ C, double* __restrict__ JTV,
                                                 double* __restrict__ GR, double* __restrict__ scr) {
  extern __shared__ double lds[];
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    if (tl.kind == TK_BRANCH) {
      fused_line_tile<true>(I, tl, X, LAM, H, J, DX, D, K, scr, lds, lds + cap_seg, V, C, JTV, GR);
    } else {
      const int e = tl.e0 + (int)threadIdx.x;
      double o = 0.0;
      if (e < tl.e1) o = fused_gen<true>(I, e, tl.t0, tl.t1, sigma, H, J, DX, D, K, X, V, C, JTV, GR);
      // the objective partial of this wavefront's 64 generators
      o = wave_sum(o);
      const int chunk = (tl.e0 + (int)(threadIdx.x & ~63u)) >> 6;
      if ((threadIdx.x & 63) == 0 && chunk * 64 < I.G) scr[obj_part_at(I, tl.t0, chunk)] = o;
    }
  }
}

// Bus rows of K for one tile.  The hand-off records, the shared pairs and
// the reference row's J entry are read past the CU's L1 (in the one-launch
// sweep they were written by other CUs of the XCD during the same launch, and
// a line holding another period's part may sit in this CU's L1 from an
// earlier tile).  SWEEP: the same pass also produces the bus's
// balance rows (and the reference row), J^T v on vm / va and their gradient
// entries, from the same walk over the incident line ends (the flow values
// of those ends and the J^T v hand-off records are gathered beside the
// condensed records).  Summation orders equal those of the separate kernels.
template <bool SWEEP>
__device__ void bus_tile(const InstDev& I, const Tile& tl, int cap_vm, const double* __restrict__ J,
                         const double* __restrict__ DX, const double* __restrict__ D, double* __restrict__ K,
                         const double* __restrict__ scr, double* __restrict__ lds, const double* __restrict__ X,
                         const double* __restrict__ V, double* __restrict__ C, double* __restrict__ JTV,
                         double* __restrict__ GR) {
  double* svm = lds;
  double* sva = lds + cap_vm;
  const int64_t N = I.N;
  const uint32_t N4 = (uint32_t)N * 4u, N8 = (uint32_t)N * 8u, G = (uint32_t)I.G;
  const int tid = (int)threadIdx.x;
  const int n = tl.e0 + tid;
  const bool act = n < tl.e1;
  // lane offsets (bytes): int32 tables and doubles indexed by the bus
  const uint32_t vN4 = (uint32_t)n * 4u, vN8 = (uint32_t)n * 8u;
  const rsrc_t rKrow = rsrc(I.krow);
  const int b0 = __builtin_amdgcn_readfirstlane(bldi(rKrow, (uint32_t)tl.e0));
  const int b1 = __builtin_amdgcn_readfirstlane(bldi(rKrow, (uint32_t)tl.e1));
  const int a0 = __builtin_amdgcn_readfirstlane(bldi(rKrow, (uint32_t)(N + tl.e0)));
  const int a1 = __builtin_amdgcn_readfirstlane(bldi(rKrow, (uint32_t)(N + tl.e1)));
  int q0 = 0, q1 = 0, vmr = 0, var = 0, clo = 0, lva = 0, call = 0, g0 = 0, g1 = 0;
  if (act) {
    const rsrc_t rBp = rsrc(I.bus_ptr);
    q0 = bldiv(rBp, vN4, 0);
    q1 = bldiv(rBp, vN4, 4);
    const int k0 = bldiv(rKrow, vN4, 0), k1 = bldiv(rKrow, vN4, 4);
    const int k2 = bldiv(rKrow, vN4, N4), k3 = bldiv(rKrow, vN4, N4 + 4);
    vmr = k0 - b0;
    var = k2 - a0;
    clo = k1 - k0 - 1;
    lva = k3 - k2;
    call = lva - clo - 2;
    if (SWEEP) {
      const rsrc_t rGp = rsrc(I.bgen_ptr);
      g0 = bldiv(rGp, vN4, 0);
      g1 = bldiv(rGp, vN4, 4);
    }
  }
  const rsrc_t rAdj = rsrc(I.bus_adj), rNb = rsrc(I.bus_nb);
  constexpr int U = 4;
  for (int t = tl.t0; t < tl.t1; ++t) {
    double* kb = K + I.k_off + kkt_period_offset_dev(I.nnzk_p, I.G, t);
    if (act) {
      const int64_t xo = I.x_off + (int64_t)t * I.n_p;
      const int64_t co = I.c_off + (int64_t)t * I.m_p;
      double* scr_m = const_cast<double*>(scr);
      // record of line end (l, e) at byte (2 l + e) * 64 = adjacency entry * 64
      static_assert(kRecEnd * sizeof(double) == 64 && kRecLine == 2 * kRecEnd, "hand-off record layout");
      const rsrc_t rR = rsrc(rec_at(I, scr_m, t)), rS = rsrc(shared_at(I, scr_m, t));
      const rsrc_t rD = rsrc(D + co), rX = rsrc(X + xo);
      // Loads are grouped by dependence so that one wave waits for memory
      // three times in the common case instead of once per step: (1) the
      // first 2U incidence entries, the first generator of the bus and the
      // bus's own inputs; (2) the records of the first U ends and the
      // generator's injections; (3) the records of the next U ends.  Longer
      // incidence lists and further generators continue in loops.  The
      // summation orders are unchanged.
      int ad[2 * U], nb[2 * U];
#pragma unroll
      for (int u = 0; u < 2 * U; ++u) {
        ad[u] = 0;
        nb[u] = -1;
      }
      if (I.B > 0) {  // (wave-uniform) entry 0 exists: lanes past their list load it and drop it
#pragma unroll
        for (int u = 0; u < 2 * U; ++u) {
          const bool ok = q0 + u < q1;
          const int aa = ok ? q0 + u : 0;
          const int a = bldi(rAdj, (uint32_t)aa), m = bldi(rNb, (uint32_t)aa);
          ad[u] = ok ? a : 0;
          nb[u] = ok ? m : -1;
        }
      }
      int gq = -1;
      if (SWEEP) {
        const int gi0 = bldi(rsrc(I.bgen), (uint32_t)(g1 > g0 ? g0 : 0));
        gq = g1 > g0 ? gi0 : -1;
      }
      double dxm = 0.0, dxa = 0.0, pdn = 0.0, qdn = 0.0;
      if (DX) {
        const rsrc_t rDX = rsrc(DX + xo);
        dxm = bldv(rDX, vN8, 0);
        dxa = bldv(rDX, vN8, N8);
      }
      if (SWEEP) {
        pdn = bldv(rsrc(I.pd + (int64_t)t * N), vN8, 0);
        qdn = bldv(rsrc(I.qd + (int64_t)t * N), vN8, 0);
      }
      double dref = 0.0;
      if (n == I.ref) {
        const double jr = bld_l2(rsrc(J + I.j_off + (int64_t)t * I.nnzj_p), (uint32_t)(2 * I.G + 4 * I.B));
        dref = bld(rD, (uint32_t)(2 * N)) * jr * jr;
      }
      double svm_s = 0.0, svavm_s = 0.0, sva_s = 0.0;
      double cvm = 0.0, cvavm = 0.0, cva = 0.0;
      double bp = 0.0, bq = 0.0, jvm = 0.0, jva = 0.0;
      int gi = 0, prev = -1;
      double2 r[U][4], x2[U];
      // records of the ends held in ad[o .. o + U) / nb[o .. o + U)
      auto gather = [&](const int* adu, const int* nbu) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool ok = nbu[u] >= 0;
          const uint32_t ro = (uint32_t)adu[u] * 64u;
          const int w1 = SWEEP ? 4 : 2;
#pragma unroll
          for (int w = 0; w < 4; ++w)
            r[u][w] = (ok && w < w1) ? bld2v_l2(rR, ro, (uint32_t)w * 16u) : make_double2(0.0, 0.0);
          x2[u] = (ok && nbu[u] < n) ? bld2v_l2(rS, (uint32_t)(adu[u] >> 1) * 16u, 0) : make_double2(0.0, 0.0);
        }
      };
      auto consume = [&](const int* nbu) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (nbu[u] < 0) break;
          const int m = nbu[u];
          if (prev >= 0 && m != prev) {
            if (prev < n) {
              svm[vmr + gi] = cvm;
              sva[var + gi] = cvavm;
              sva[var + call + 1 + gi] = cva;
            } else {
              sva[var + gi + 1] = cvavm;
            }
            ++gi;
            cvm = cvavm = cva = 0.0;
          }
          prev = m;
          svm_s += r[u][0].x;
          svavm_s += r[u][0].y;
          sva_s += r[u][1].x;
          cvavm += r[u][1].y;
          cvm += x2[u].x;
          cva += x2[u].y;
          if (SWEEP) {
            bp -= r[u][2].x;
            bq -= r[u][2].y;
            jvm += r[u][3].x;
            jva += r[u][3].y;
          }
        }
      };
      gather(ad, nb);
      if (SWEEP) {
        const uint32_t g8 = (uint32_t)(gq >= 0 ? gq : 0) * 8u;
        const double pg = bldv(rX, g8, 2 * N8), qg = bldv(rX, g8, 2 * N8 + G * 8u);
        if (gq >= 0) {
          bp += pg;
          bq += qg;
        }
        const rsrc_t rBg = rsrc(I.bgen);
        for (int q = g0 + 1; q < g1; ++q) {
          const uint32_t h8 = (uint32_t)bldi(rBg, (uint32_t)q) * 8u;
          bp += bldv(rX, h8, 2 * N8);
          bq += bldv(rX, h8, 2 * N8 + G * 8u);
        }
      }
      consume(nb);
      if (q1 - q0 > U) {
        gather(ad + U, nb + U);
        consume(nb + U);
      }
      for (int aa = q0 + 2 * U; aa < q1; aa += U) {
        int adu[U], nbu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool ok = aa + u < q1;
          adu[u] = ok ? bldi(rAdj, (uint32_t)(aa + u)) : 0;
          nbu[u] = ok ? bldi(rNb, (uint32_t)(aa + u)) : -1;
        }
        gather(adu, nbu);
        consume(nbu);
      }
      if (prev >= 0) {
        if (prev < n) {
          svm[vmr + gi] = cvm;
          sva[var + gi] = cvavm;
          sva[var + call + 1 + gi] = cva;
        } else {
          sva[var + gi + 1] = cvavm;
        }
      }
      svm[vmr + clo] = dxm + svm_s;
      if (q1 > q0) sva[var + clo] = svavm_s;  // (va_n, vm_n) exists only with an incident line
      sva[var + lva - 1] = dxa + sva_s + dref;
      if (SWEEP) {
        const rsrc_t rC = rsrc(C + co);
        bp -= pdn;
        bq -= qdn;
        bstvn(rC, vN8, 0, bp);
        bstvn(rC, vN8, N8, bq);
        if (n == I.ref) {
          bst(rC, (uint32_t)(2 * N), X[xo + N + n]);
          jva += V[co + 2 * N];
        }
        const rsrc_t rO = rsrc(JTV + xo), rG = rsrc(GR + xo);
        bstvn(rO, vN8, 0, jvm);
        bstvn(rO, vN8, N8, jva);
        bstvn(rG, vN8, 0, 0.0);
        bstvn(rG, vN8, N8, 0.0);
      }
    }
    __syncthreads();
    stream_segment<false, true>(svm, rKrow, rKrow, kb + b0, b1 - b0);
    stream_segment<false, true>(sva, rKrow, rKrow, kb + a0, a1 - a0);
    __syncthreads();
  }
}

// Dynamic LDS: vm-row segment [cap_vm] then va-row segment [cap_va].
__global__ void __launch_bounds__(512) k_kkt_b(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                               int ntiles, int cap_vm, const double* __restrict__ J,
                                               const double* __restrict__ DX, const double* __restrict__ D,
                                               double* __restrict__ K, const double* __restrict__ scr) {
  extern __shared__ double lds[];
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    bus_tile<false>(insts[tl.inst], tl, cap_vm, J, DX, D, K, scr, lds, nullptr, nullptr, nullptr, nullptr, nullptr);
  }
}

// Whole sweep, buses: K bus rows, balance and reference rows, J^T v and
// gradient entries of vm / va.
__global__ void __launch_bounds__(512) k_sweep_b(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                                 int ntiles, int cap_vm, const double* __restrict__ X,
                                                 const double* __restrict__ V, const double* __restrict__ J,
                                                 const double* __restrict__ DX, const double* __restrict__ D,
                                                 double* __restrict__ K, double* __restrict__ C,
                                                 double* __restrict__ JTV, double* __restrict__ GR,
                                                 const double* __restrict__ scr, const ObjFold of) {
  extern __shared__ double lds[];
  if (of.f) {
    // the objective: the line pass (the previous launch) left the partials
    __shared__ double wred[8];
    const int nw = (int)(blockDim.x >> 6);
    for (int k = blockIdx.x; k < of.ninst; k += gridDim.x) {
      const InstDev& I = insts[k];
      const int nc = (I.G + 63) >> 6, ng = (I.T + of.ppt - 1) / of.ppt;
      double acc = 0.0;
      for (int q = (int)threadIdx.x; q < ng * nc; q += (int)blockDim.x) {
        const int grp = q / nc;
        acc += scr[obj_part_at(I, grp * of.ppt, q - grp * nc)];
      }
      acc = wave_sum(acc);
      if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = acc;
      __syncthreads();
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += wred[w];
        of.f[k] = s;
      }
      __syncthreads();
    }
  }
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    bus_tile<true>(insts[tl.inst], tl, cap_vm, J, DX, D, K, scr, lds, X, V, C, JTV, GR);
  }
}

// ---------------------------------------------------------------- whole sweep, one launch
// The whole sweep as one persistent launch.  Every XCD drains a queue of its
// own (the XCD a block runs on is read from the hardware register, so the
// queue's tiles share that XCD's L2): line and generator tiles of a group of
// periods first, the group's bus tiles a couple of groups later.  A bus tile
// waits until every line and generator tile of its group has counted itself
// done, then reads the group's hand-off records, which are still in the
// XCD's L2 or the memory-side cache instead of coming back from HBM as in
// the two-launch form.  Tiles are handed out in queue order by a ticket
// counter, so every tile a bus tile waits for is already held by a running
// block of the same XCD and the waits always end; the spin is bounded
// anyway and a wait that runs out sets bit 0 of *flags.
// Counters (all zero at launch: the objective's partial pass or
// k_sweep_open clears them), each queue's on 128-byte lines of their own:
// ctr[32 q] ticket and ctr[32 q + 1] tiles finished of queue q; ctr[slot]
// tiles finished of a group (SweepItem::slot).  Every access to them is an
// atomic read-modify-write, so all of them execute where the increments
// do: the poll of a bus tile reads its group's count with max(count, 0),
// which returns the count unchanged (a plain cache-bypassing load would not
// observe increments held in the XCD's L2).
constexpr int kSweepCtrStride = 32;
constexpr int kSweepSpinLimit = 1 << 20;

__global__ void __launch_bounds__(256) k_sweep(const InstDev* __restrict__ insts, const SweepItem* __restrict__ items,
                                               const int32_t* __restrict__ qbeg, int nq, int32_t* __restrict__ ctr,
                                               int32_t* __restrict__ flags, int cap_seg, int cap_vm, int cap_va,
                                               const double* __restrict__ X, const double* __restrict__ LAM,
                                               double sigma, const double* __restrict__ V, double* __restrict__ H,
                                               double* __restrict__ J, const double* __restrict__ DX,
                                               const double* __restrict__ D, double* __restrict__ K,
                                               double* __restrict__ C, double* __restrict__ JTV,
                                               double* __restrict__ GR, double* __restrict__ scr) {
  extern __shared__ double lds[];
  __shared__ int s_item;
  int xcc;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
  const int q = xcc % nq;
  const int i0 = qbeg[q], nitems = qbeg[q + 1] - i0;
  int32_t* ticket = ctr + kSweepCtrStride * q;
  int32_t* qdone = ticket + 1;
  for (;;) {
    if (threadIdx.x == 0) s_item = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= nitems) break;
    const SweepItem w = items[i0 + it];
    const InstDev& I = insts[w.tl.inst];
    if (w.tl.kind == TK_BUS) {
      if (threadIdx.x == 0) {
        int spins = 0;
        while (__hip_atomic_fetch_max(ctr + w.slot, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < w.need) {
          __builtin_amdgcn_s_sleep(4);
          if (++spins > kSweepSpinLimit) {
            __hip_atomic_fetch_or(flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
      }
      __syncthreads();
      bus_tile<true>(I, w.tl, cap_vm, J, DX, D, K, scr, lds, X, V, C, JTV, GR);
    } else {
      if (w.tl.kind == TK_BRANCH) {
        fused_line_tile<true>(I, w.tl, X, LAM, H, J, DX, D, K, scr, lds, lds + cap_seg, V, C, JTV, GR);
      } else {
        const int e = w.tl.e0 + (int)threadIdx.x;
        if (e < w.tl.e1) fused_gen<true>(I, e, w.tl.t0, w.tl.t1, sigma, H, J, DX, D, K, X, V, C, JTV, GR);
      }
      // every store of the tile has been acknowledged by the XCD's L2
      // before the tile counts itself done
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr + w.slot, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) __hip_atomic_fetch_add(qdone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Clears the counters of k_sweep (one block).
__global__ void __launch_bounds__(256) k_sweep_open(int32_t* __restrict__ ctr, int n) {
  for (int i = (int)threadIdx.x; i < n; i += blockDim.x) ctr[i] = 0;
}

// After k_sweep: block k < ninst sums instance k's objective partials in the
// order of k_obj_final (when f is requested); block 0 also checks that every
// queue was drained (bit 1 of *flags otherwise).
__global__ void __launch_bounds__(256) k_sweep_close(const int32_t* __restrict__ begin,
                                                     const double* __restrict__ partial, double* __restrict__ f,
                                                     const int32_t* __restrict__ ctr,
                                                     const int32_t* __restrict__ qbeg, int nq,
                                                     int32_t* __restrict__ flags) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  if (k == 0 && threadIdx.x == 0) {
    for (int q = 0; q < nq; ++q)
      if (ctr[kSweepCtrStride * q + 1] != qbeg[q + 1] - qbeg[q]) *flags |= 2;
  }
  if (!f) return;
  const int a = begin[k], z = begin[k + 1];
  double acc = 0.0;
  for (int q = a + (int)threadIdx.x; q < z; q += blockDim.x) acc += partial[q];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) f[k] = red[0];
}

// ---------------------------------------------------------------- structure
__global__ void __launch_bounds__(512) k_jac_struct(const InstDev* __restrict__ insts,
                                                    const Tile* __restrict__ tiles, int ntiles,
                                                    int32_t* __restrict__ rows, int32_t* __restrict__ cols) {
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int e = tl.e0 + (int)threadIdx.x;
    if (e >= tl.e1) continue;
    const Bases b(I);
    const int64_t B = b.B, N = b.N, G = b.G;
    for (int t = tl.t0; t < tl.t1; ++t) {
      const int64_t jo = I.j_off + (int64_t)t * I.nnzj_p;
      const int32_t cr = (int32_t)(I.c_off + (int64_t)t * I.m_p);
      const int32_t xc = (int32_t)(I.x_off + (int64_t)t * I.n_p);
      if (tl.kind == TK_BRANCH) {
        const int l = e, i = I.f_bus[l], j = I.t_bus[l];
        const int32_t fl = xc + (int32_t)b.xFL + l;
        const int32_t brow[4] = {cr + i, cr + (int32_t)N + i, cr + j, cr + (int32_t)N + j};
        const int32_t bus[4] = {xc + i, xc + j, xc + (int32_t)N + i, xc + (int32_t)N + j};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          rows[jo + b.jBAL + k * B + l] = brow[k];
          cols[jo + b.jBAL + k * B + l] = fl + (int32_t)(k * B);
          const int32_t r = cr + (int32_t)(b.cFLOW + k * B) + l;
          const int64_t q = jo + b.jFLOW + (int64_t)(k * 5) * B + l;
          rows[q] = r;
          cols[q] = fl + (int32_t)(k * B);
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            rows[q + (a + 1) * B] = r;
            cols[q + (a + 1) * B] = bus[a];
          }
          rows[jo + b.jTH + k * B + l] = cr + (int32_t)((k < 2 ? b.cTHF : b.cTHT)) + l;
          cols[jo + b.jTH + k * B + l] = fl + (int32_t)(k * B);
        }
        rows[jo + b.jANG + l] = cr + (int32_t)b.cANG + l;
        cols[jo + b.jANG + l] = bus[2];
        rows[jo + b.jANG + B + l] = cr + (int32_t)b.cANG + l;
        cols[jo + b.jANG + B + l] = bus[3];
      } else {
        const int g = e, n = I.gen_bus[g];
        rows[jo + g] = cr + n;
        cols[jo + g] = xc + (int32_t)(2 * N) + g;
        rows[jo + G + g] = cr + (int32_t)N + n;
        cols[jo + G + g] = xc + (int32_t)(2 * N + G) + g;
        if (g == 0) {
          rows[jo + b.jREF] = cr + (int32_t)b.cREF;
          cols[jo + b.jREF] = xc + (int32_t)N + I.ref;
        }
        if (t >= 1) {
          const int64_t q = I.j_off + (int64_t)I.T * I.nnzj_p + (int64_t)(t - 1) * 2 * G;
          const int32_t rr = (int32_t)(I.c_off + (int64_t)I.T * I.m_p + (int64_t)(t - 1) * G) + g;
          rows[q + g] = rr;
          cols[q + g] = xc + (int32_t)(2 * N) + g;
          rows[q + G + g] = rr;
          cols[q + G + g] = xc - (int32_t)I.n_p + (int32_t)(2 * N) + g;
        }
      }
    }
  }
}

__global__ void __launch_bounds__(512) k_hess_struct(const InstDev* __restrict__ insts,
                                                     const Tile* __restrict__ tiles, int ntiles,
                                                     int32_t* __restrict__ rows, int32_t* __restrict__ cols) {
  // (a, b) pairs of the local variable list (vm_i, vm_j, va_i, va_j)
  const int pf_a[9] = {0, 1, 2, 2, 2, 3, 3, 3, 3}, pf_b[9] = {0, 0, 0, 1, 2, 0, 1, 2, 3};
  const int pt_a[9] = {1, 1, 2, 2, 2, 3, 3, 3, 3}, pt_b[9] = {0, 1, 0, 1, 2, 0, 1, 2, 3};
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int e = tl.e0 + (int)threadIdx.x;
    if (e >= tl.e1) continue;
    const Bases b(I);
    const int64_t B = b.B, N = b.N;
    for (int t = tl.t0; t < tl.t1; ++t) {
      const int64_t ho = I.h_off + (int64_t)t * I.nnzh_p;
      const int32_t xc = (int32_t)(I.x_off + (int64_t)t * I.n_p);
      if (tl.kind == TK_BRANCH) {
        const int l = e, i = I.f_bus[l], j = I.t_bus[l];
        const int32_t bus[4] = {xc + i, xc + j, xc + (int32_t)N + i, xc + (int32_t)N + j};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
          for (int p = 0; p < 9; ++p) {
            const int32_t ra = bus[k < 2 ? pf_a[p] : pt_a[p]], rb = bus[k < 2 ? pf_b[p] : pt_b[p]];
            const int64_t q = ho + b.hFLOW + (int64_t)(k * 9 + p) * B + l;
            rows[q] = ra > rb ? ra : rb;
            cols[q] = ra > rb ? rb : ra;
          }
          const int32_t fv = xc + (int32_t)(b.xFL + k * B) + l;
          rows[ho + b.hTH + k * B + l] = fv;
          cols[ho + b.hTH + k * B + l] = fv;
        }
      } else {
        const int32_t pv = xc + (int32_t)(2 * N) + e;
        rows[ho + e] = pv;
        cols[ho + e] = pv;
      }
    }
  }
}

__global__ void __launch_bounds__(512) k_kkt_struct(const InstDev* __restrict__ insts,
                                                    const Tile* __restrict__ tiles, int ntiles, int ninst,
                                                    int64_t* __restrict__ rowptr, int32_t* __restrict__ colind) {
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int r = tl.e0 + (int)threadIdx.x;
    if (r >= tl.e1) continue;
    const int64_t PG = 2LL * I.N;
    const int rs = I.krow[r], re = I.krow[r + 1];
    for (int t = tl.t0; t < tl.t1; ++t) {
      const int64_t kp = I.k_off + kkt_period_offset_dev(I.nnzk_p, I.G, t);
      const int64_t xb = I.x_off + (int64_t)t * I.n_p;
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
      int64_t pos = kp + rs + shift - (ramp ? 1 : 0);
      rowptr[xb + r] = pos;
      if (ramp) colind[pos++] = (int32_t)(xb - I.n_p + r);
      for (int p = rs; p < re; ++p) colind[pos++] = (int32_t)(xb + I.kcol[p]);
      if (tl.inst == ninst - 1 && r == I.n_p - 1 && t == I.T - 1) rowptr[I.x_off + (int64_t)I.T * I.n_p] = pos;
    }
  }
}

// ---------------------------------------------------------------- bounds
__global__ void __launch_bounds__(512) k_bounds(const InstDev* __restrict__ insts, const Tile* __restrict__ tiles,
                                                int ntiles, double* __restrict__ lv, double* __restrict__ uv,
                                                double* __restrict__ lc, double* __restrict__ uc) {
  const double inf = __builtin_huge_val();
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int e = tl.e0 + (int)threadIdx.x;
    if (e >= tl.e1) continue;
    const Bases b(I);
    const int64_t N = b.N, G = b.G, B = b.B;
    for (int t = tl.t0; t < tl.t1; ++t) {
      if (tl.kind == TK_VAR) {
        double lo = -inf, hi = inf;
        if (e < N) {
          lo = I.vmin[e];
          hi = I.vmax[e];
        } else if (e >= 2 * N && e < 2 * N + G) {
          lo = I.pmin[e - 2 * N];
          hi = I.pmax[e - 2 * N];
        } else if (e >= 2 * N + G && e < 2 * N + 2 * G) {
          lo = I.qmin[e - 2 * N - G];
          hi = I.qmax[e - 2 * N - G];
        }
        const int64_t q = I.x_off + (int64_t)t * I.n_p + e;
        lv[q] = lo;
        uv[q] = hi;
      } else if (tl.kind == TK_CON) {
        double lo = 0.0, hi = 0.0;
        if (e >= b.cTHF && e < b.cANG) {
          const int64_t l = e - (e >= b.cTHT ? b.cTHT : b.cTHF);
          lo = -inf;
          hi = I.rate[l] * I.rate[l];
        } else if (e >= b.cANG) {
          lo = I.angmin[e - b.cANG];
          hi = I.angmax[e - b.cANG];
        }
        (void)B;
        const int64_t q = I.c_off + (int64_t)t * I.m_p + e;
        lc[q] = lo;
        uc[q] = hi;
      } else if (t >= 1) {
        const int64_t q = I.c_off + (int64_t)I.T * I.m_p + (int64_t)(t - 1) * G + e;
        lc[q] = -I.ramp[e];
        uc[q] = I.ramp[e];
      }
    }
  }
}

// ---------------------------------------------------------------- load adjoint
__global__ void __launch_bounds__(512) k_load_adj(const InstDev* __restrict__ insts,
                                                  const Tile* __restrict__ tiles, int ntiles,
                                                  const double* __restrict__ lam, double* __restrict__ gpd,
                                                  double* __restrict__ gqd) {
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile tl = tiles[remap_tile(v, ntiles)];
    const InstDev& I = insts[tl.inst];
    const int n = tl.e0 + (int)threadIdx.x;
    if (n >= tl.e1) continue;
    for (int t = tl.t0; t < tl.t1; ++t) {
      const double* lp = lam + I.c_off + (int64_t)t * I.m_p;
      const int64_t q = I.ld_off + (int64_t)t * I.N + n;
      gpd[q] = -lp[n];
      gqd[q] = -lp[I.N + n];
    }
  }
}

dim3 grid_of(const Launch& L) { return dim3((unsigned)(L.grid > 0 ? L.grid : L.ntiles)); }

}  // namespace

#define OPF_LAUNCH(kernel, L, ...)                                                              \
  do {                                                                                          \
    if ((L).ntiles <= 0) return hipSuccess;                                                     \
    hipLaunchKernelGGL(kernel, grid_of(L), dim3((unsigned)(L).block), 0, (L).stream, (L).insts, \
                       (L).tiles, (L).ntiles, __VA_ARGS__);                                     \
    return hipGetLastError();                                                                   \
  } while (0)

hipError_t launch_jac(const Launch& L, const double* x, double* jv) {
  if (L.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_jac, grid_of(L), dim3((unsigned)L.block), L.smem, L.stream, L.insts, L.tiles, L.ntiles, x,
                     jv);
  return hipGetLastError();
}
hipError_t launch_hess(const Launch& L, const double* x, const double* lam, double sigma, double* hv) {
  OPF_LAUNCH(k_hess, L, x, lam, sigma, hv);
}
hipError_t launch_cons(const Launch& L, const double* x, double* c) { OPF_LAUNCH(k_cons, L, x, c); }
hipError_t launch_jv(const Launch& L, const double* x, const double* v, double* jv) {
  OPF_LAUNCH(k_jv, L, x, v, jv);
}

namespace {
// Grid of a flat launch: 256 lanes per block, at most 8 blocks per CU's
// worth (2048) of blocks, each striding over the range.
dim3 flat_grid(int64_t count) {
  const int64_t blocks = (count + 255) / 256;
  return dim3((unsigned)std::min<int64_t>(std::max<int64_t>(blocks, 1), 2048));
}
}  // namespace

hipError_t launch_rhs_rows(const Flat& F, const IpmDev& st, const double* c, double* dcon, double* w) {
  if (F.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rhs_rows, flat_grid(F.count), dim3(256), 0, F.stream, F.count, st, c, dcon, w);
  return hipGetLastError();
}
hipError_t launch_rhs_vars(const Flat& F, const IpmDev& st, const double* grad, double* diag_x, double* rhs) {
  if (F.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rhs_vars, flat_grid(F.count), dim3(256), 0, F.stream, F.count, st, grad, diag_x, rhs);
  return hipGetLastError();
}
hipError_t launch_rec_rows(const Flat& F, const IpmDev& st, const double* c, const double* adx, double* ds,
                           double* dy, double* dvl, double* dvu) {
  if (F.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rec_rows, flat_grid(F.count), dim3(256), 0, F.stream, F.count, st, c, adx, ds, dy, dvl,
                     dvu);
  return hipGetLastError();
}
hipError_t launch_rec_vars(const Flat& F, const IpmDev& st, const double* dx, double* dzl, double* dzu) {
  if (F.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rec_vars, flat_grid(F.count), dim3(256), 0, F.stream, F.count, st, dx, dzl, dzu);
  return hipGetLastError();
}
hipError_t launch_grad(const Launch& L, const double* x, double* g) { OPF_LAUNCH(k_grad, L, x, g); }
hipError_t launch_obj_partial(const Launch& L, const double* x, double* partial, int32_t* zero, int nzero) {
  OPF_LAUNCH(k_obj_partial, L, x, partial, zero, nzero);
}
hipError_t launch_obj_final(const int32_t* begin, int ninst, const double* partial, double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_obj_final, dim3((unsigned)ninst), dim3(256), 0, s, begin, partial, f);
  return hipGetLastError();
}
hipError_t launch_jt_a(const Launch& L, const double* x, const double* v, double* out, double* scratch) {
  OPF_LAUNCH(k_jt_a, L, x, v, out, scratch);
}
hipError_t launch_jt_b(const Launch& L, const double* v, double* out, const double* scratch) {
  OPF_LAUNCH(k_jt_b, L, v, out, scratch);
}
hipError_t launch_kkt_a(const Launch& L, const double* h, const double* j, const double* dx, const double* d,
                        double* k, double* scratch) {
  if (L.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kkt_a, grid_of(L), dim3((unsigned)L.block), L.smem, L.stream, L.insts, L.tiles, L.ntiles,
                     L.cap0, h, j, dx, d, k, scratch);
  return hipGetLastError();
}
hipError_t launch_jhk_a(const Launch& L, const double* x, const double* lam, double sigma, double* h, double* j,
                        const double* dx, const double* d, double* k, double* scratch) {
  if (L.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_jhk_a, grid_of(L), dim3((unsigned)L.block), L.smem, L.stream, L.insts, L.tiles, L.ntiles,
                     L.cap0, x, lam, sigma, h, j, dx, d, k, scratch);
  return hipGetLastError();
}
hipError_t launch_sweep_a(const Launch& L, const double* x, const double* lam, double sigma, const double* v,
                          double* h, double* j, const double* dx, const double* d, double* k, double* c, double* jtv,
                          double* g, double* scratch) {
  if (L.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sweep_a, grid_of(L), dim3((unsigned)L.block), L.smem, L.stream, L.insts, L.tiles, L.ntiles,
                     L.cap0, x, lam, sigma, v, h, j, dx, d, k, c, jtv, g, scratch);
  return hipGetLastError();
}
hipError_t launch_sweep_b(const Launch& L, const double* x, const double* v, const double* j, const double* dx,
                          const double* d, double* k, double* c, double* jtv, double* g, const double* scratch,
                          const ObjFold& of) {
  if (L.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sweep_b, grid_of(L), dim3((unsigned)L.block), L.smem, L.stream, L.insts, L.tiles, L.ntiles,
                     L.cap0, x, v, j, dx, d, k, c, jtv, g, scratch, of);
  return hipGetLastError();
}
hipError_t launch_kkt_b(const Launch& L, const double* j, const double* dx, const double* d, double* k,
                        const double* scratch) {
  if (L.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kkt_b, grid_of(L), dim3((unsigned)L.block), L.smem, L.stream, L.insts, L.tiles, L.ntiles,
                     L.cap0, j, dx, d, k, scratch);
  return hipGetLastError();
}
hipError_t launch_jac_struct(const Launch& L, int32_t* rows, int32_t* cols) {
  OPF_LAUNCH(k_jac_struct, L, rows, cols);
}
hipError_t launch_hess_struct(const Launch& L, int32_t* rows, int32_t* cols) {
  OPF_LAUNCH(k_hess_struct, L, rows, cols);
}
hipError_t launch_kkt_struct(const Launch& L, int ninst, int64_t* rowptr, int32_t* colind) {
  OPF_LAUNCH(k_kkt_struct, L, ninst, rowptr, colind);
}
hipError_t launch_bounds(const Launch& L, double* lv, double* uv, double* lc, double* uc) {
  OPF_LAUNCH(k_bounds, L, lv, uv, lc, uc);
}
hipError_t launch_load_adjoint(const Launch& L, const double* lam, double* gpd, double* gqd) {
  OPF_LAUNCH(k_load_adj, L, lam, gpd, gqd);
}


int sweep_fused_blocks_per_cu(int block, size_t smem) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sweep, block, smem) != hipSuccess) return 0;
  return occ;
}

hipError_t launch_sweep_fused(const FusedSweep& F, const double* x, const double* lam, double sigma,
                              const double* v, double* h, double* j, const double* dx, const double* d, double* k,
                              double* c, double* jtv, double* g, double* scratch) {
  if (F.grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sweep, dim3((unsigned)F.grid), dim3((unsigned)F.block), F.smem, F.stream, F.insts, F.items,
                     F.qbeg, F.nq, F.ctr, F.flags, F.cap_seg, F.cap_vm, F.cap_va, x, lam, sigma, v, h, j, dx, d, k, c, jtv,
                     g, scratch);
  return hipGetLastError();
}

hipError_t launch_sweep_open(int32_t* ctr, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_sweep_open, dim3(1), dim3(256), 0, s, ctr, n);
  return hipGetLastError();
}

hipError_t launch_sweep_close(const int32_t* begin, int ninst, const double* partial, double* f,
                              const int32_t* ctr, const int32_t* qbeg, int nq, int32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_sweep_close, dim3((unsigned)(f ? ninst : 1)), dim3(256), 0, s, begin, partial, f, ctr, qbeg,
                     nq, flags);
  return hipGetLastError();
}

}  // namespace opf
