// The lifted-KKT interior-point loop (Sec. III-B around the condensed
// system): element-wise and reduction kernels of the outer iteration and the
// opf_ipm_solve driver, which calls the library's own evaluation,
// condensation, factorization, solve and recovery entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/opf.h"
#include "opf_api_internal.h"

namespace opf {
namespace {

constexpr int kRedBlock = 256;
constexpr int kRedGrid = 512;

__device__ __forceinline__ bool fin(double v) { return isfinite(v); }

// Flat start of one instance: vm = 1, va = 0, pg and qg at the middle of
// their boxes, flows 0 (set from c next).
__global__ void k_start_flat(double* __restrict__ x, const double* __restrict__ xl, const double* __restrict__ xu,
                             int64_t n_p, int32_t N, int32_t G, int32_t T) {
  const int64_t n = n_p * T;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n_p;
    double v = 0.0;
    if (i < N) v = 1.0;
    else if (i >= 2 * N && i < 2 * N + 2 * G) v = 0.5 * (xl[e] + xu[e]);
    x[e] = v;
  }
}

// Flows equal to the flows of the current voltages: the flow rows read
// c = x_flow - phi(V) with x_flow = 0, so x_flow = -c.
__global__ void k_start_flows(double* __restrict__ x, const double* __restrict__ c, int64_t n_p, int64_t m_p,
                              int32_t N, int32_t B, int32_t G, int32_t T) {
  const int64_t n = 4LL * B * T;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e / (4LL * B), r = e % (4LL * B);
    x[t * n_p + 2 * N + 2 * G + r] = -c[t * m_p + 2 * N + 1 + r];
  }
}

// Moves v at least 1e-2 max(1, |bound|) (at most half the box) inside its
// finite bounds.
__device__ __forceinline__ double inside(double v, double lo, double hi) {
  const bool fl = fin(lo), fh = fin(hi);
  double pl = fl ? 1e-2 * fmax(1.0, fabs(lo)) : 0.0, pu = fh ? 1e-2 * fmax(1.0, fabs(hi)) : 0.0;
  if (fl && fh) {
    pl = fmin(pl, 0.5 * (hi - lo));
    pu = fmin(pu, 0.5 * (hi - lo));
  }
  if (fl) v = fmax(v, lo + pl);
  if (fh) v = fmin(v, hi - pu);
  return v;
}

__global__ void k_push_inside(double* __restrict__ v, const double* __restrict__ src, const double* __restrict__ lo,
                              const double* __restrict__ hi, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = inside(src[i], lo[i], hi[i]);
}

// Relaxed row bounds (equality rows widened by +-relax) and the starting
// multipliers: y = 0, bound multipliers 1 where the bound is finite.
__global__ void k_start_rows(const double* __restrict__ cl, const double* __restrict__ cu, double relax,
                             double* __restrict__ sl, double* __restrict__ su, double* __restrict__ y,
                             double* __restrict__ ly, double* __restrict__ vl, double* __restrict__ vu, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const bool eq = cl[i] == cu[i];
    const double a = eq ? cl[i] - relax : cl[i], b = eq ? cu[i] + relax : cu[i];
    sl[i] = a;
    su[i] = b;
    y[i] = 0.0;
    ly[i] = 0.0;
    vl[i] = fin(a) ? 1.0 : 0.0;
    vu[i] = fin(b) ? 1.0 : 0.0;
  }
}

__global__ void k_start_vars(const double* __restrict__ xl, const double* __restrict__ xu, double* __restrict__ zl,
                             double* __restrict__ zu, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    zl[i] = fin(xl[i]) ? 1.0 : 0.0;
    zu[i] = fin(xu[i]) ? 1.0 : 0.0;
  }
}

struct Iter {
  double *x, *s, *y, *ly, *zl, *zu, *vl, *vu;
  const double *xl, *xu, *sl, *su;
};

// Per-block partials of the residual measures: [0] max |p_x|, [1] max |p_s|,
// [2] max |c - s|, [3] max complementarity product, [4] their sum, [5]
// their count, [6] sum of |multipliers|, [7] number of non-finite terms
// (fmax would drop a NaN, so they are counted instead), [8] min
// complementarity product (with [3]: max |product - mu| for any mu).
constexpr int kNR = 9;

__device__ __forceinline__ void block_reduce(double* sh, int op, double& v) {
  // op 0: max, 1: sum, 2: min
  const int tid = (int)threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = kRedBlock / 2; off > 0; off >>= 1) {
    if (tid < off) {
      const double a = sh[tid], b = sh[tid + off];
      sh[tid] = op == 0 ? fmax(a, b) : (op == 1 ? a + b : fmin(a, b));
    }
    __syncthreads();
  }
  v = sh[0];
  __syncthreads();
}

__global__ void __launch_bounds__(kRedBlock) k_resid(Iter w, const double* __restrict__ grad,
                                                     const double* __restrict__ jtv, const double* __restrict__ c,
                                                     int64_t n, int64_t m, double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  double rd = 0.0, rs = 0.0, rp = 0.0, gmax = 0.0, gsum = 0.0, gcnt = 0.0, msum = 0.0, bad = 0.0, gmin = INFINITY;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const bool hl = fin(w.xl[i]), hu = fin(w.xu[i]);
    const double zl = hl ? w.zl[i] : 0.0, zu = hu ? w.zu[i] : 0.0;
    const double r = grad[i] - jtv[i] - zl + zu;
    if (!fin(r) || !fin(w.x[i])) bad += 1.0;
    rd = fmax(rd, fabs(r));
    if (hl) {
      const double g = zl * (w.x[i] - w.xl[i]);
      gmax = fmax(gmax, g);
      gmin = fmin(gmin, g);
      gsum += g;
      gcnt += 1.0;
    }
    if (hu) {
      const double g = zu * (w.xu[i] - w.x[i]);
      gmax = fmax(gmax, g);
      gmin = fmin(gmin, g);
      gsum += g;
      gcnt += 1.0;
    }
    msum += zl + zu;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
    const bool gl = fin(w.sl[i]), gu = fin(w.su[i]);
    const double vl = gl ? w.vl[i] : 0.0, vu = gu ? w.vu[i] : 0.0;
    const double a = -vl + vu + w.y[i], b = c[i] - w.s[i];
    if (!fin(a) || !fin(b)) bad += 1.0;
    rs = fmax(rs, fabs(a));
    rp = fmax(rp, fabs(b));
    if (gl) {
      const double g = vl * (w.s[i] - w.sl[i]);
      gmax = fmax(gmax, g);
      gmin = fmin(gmin, g);
      gsum += g;
      gcnt += 1.0;
    }
    if (gu) {
      const double g = vu * (w.su[i] - w.s[i]);
      gmax = fmax(gmax, g);
      gmin = fmin(gmin, g);
      gsum += g;
      gcnt += 1.0;
    }
    msum += vl + vu + fabs(w.y[i]);
  }
  block_reduce(sh, 0, rd);
  block_reduce(sh, 0, rs);
  block_reduce(sh, 0, rp);
  block_reduce(sh, 0, gmax);
  block_reduce(sh, 1, gsum);
  block_reduce(sh, 1, gcnt);
  block_reduce(sh, 1, msum);
  block_reduce(sh, 1, bad);
  block_reduce(sh, 2, gmin);
  if (threadIdx.x == 0) {
    double* o = part + (int64_t)blockIdx.x * kNR;
    o[8] = gmin;
    o[0] = rd;
    o[1] = rs;
    o[2] = rp;
    o[3] = gmax;
    o[4] = gsum;
    o[5] = gcnt;
    o[6] = msum;
    o[7] = bad;
  }
}

struct Step {
  const double *dx, *ds, *dy, *dzl, *dzu, *dvl, *dvu;  // as the condensed solve returns them
};

// Fraction to the boundary: the Newton step is (-dx, -ds, +dy, -dz, -dv).
// Per-block partials [0] primal length, [1] dual length.
__device__ __forceinline__ double ftb(double v, double d, double b, bool upper, double tau) {
  if (upper ? d > 0.0 : d < 0.0) return fmin(1.0, tau * (b - v) / d);
  return 1.0;
}

__global__ void __launch_bounds__(kRedBlock) k_steplen(Iter w, Step st, double tau, int64_t n, int64_t m,
                                                       double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  double ap = 1.0, ad = 1.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const double dx = -st.dx[i];
    if (fin(w.xl[i])) {
      ap = fmin(ap, ftb(w.x[i], dx, w.xl[i], false, tau));
      ad = fmin(ad, ftb(w.zl[i], -st.dzl[i], 0.0, false, tau));
    }
    if (fin(w.xu[i])) {
      ap = fmin(ap, ftb(w.x[i], dx, w.xu[i], true, tau));
      ad = fmin(ad, ftb(w.zu[i], -st.dzu[i], 0.0, false, tau));
    }
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
    const double ds = -st.ds[i];
    if (fin(w.sl[i])) {
      ap = fmin(ap, ftb(w.s[i], ds, w.sl[i], false, tau));
      ad = fmin(ad, ftb(w.vl[i], -st.dvl[i], 0.0, false, tau));
    }
    if (fin(w.su[i])) {
      ap = fmin(ap, ftb(w.s[i], ds, w.su[i], true, tau));
      ad = fmin(ad, ftb(w.vu[i], -st.dvu[i], 0.0, false, tau));
    }
  }
  block_reduce(sh, 2, ap);
  block_reduce(sh, 2, ad);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ap;
    part[2 * blockIdx.x + 1] = ad;
  }
}

__global__ void k_update(Iter w, Step st, double ap, double ad, int64_t n, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    w.x[i] -= ap * st.dx[i];
    if (fin(w.xl[i])) w.zl[i] -= ad * st.dzl[i];
    if (fin(w.xu[i])) w.zu[i] -= ad * st.dzu[i];
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
    w.s[i] -= ap * st.ds[i];
    w.y[i] += ad * st.dy[i];
    w.ly[i] = -w.y[i];
    if (fin(w.sl[i])) w.vl[i] -= ad * st.dvl[i];
    if (fin(w.su[i])) w.vu[i] -= ad * st.dvu[i];
  }
}

// The filter line search: per-block partials of the violation
// theta = sum |c - s| ([0]) and of sum ln(distance to each finite bound)
// ([1]) at the point (x, s); c = c(x).
__global__ void __launch_bounds__(kRedBlock) k_barrier(Iter w, const double* __restrict__ x,
                                                       const double* __restrict__ s, const double* __restrict__ c,
                                                       int64_t n, int64_t m, double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  double th = 0.0, lg = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    if (fin(w.xl[i])) lg += log(x[i] - w.xl[i]);
    if (fin(w.xu[i])) lg += log(w.xu[i] - x[i]);
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
    th += fabs(c[i] - s[i]);
    if (fin(w.sl[i])) lg += log(s[i] - w.sl[i]);
    if (fin(w.su[i])) lg += log(w.su[i] - s[i]);
  }
  block_reduce(sh, 1, th);
  block_reduce(sh, 1, lg);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = th;
    part[2 * blockIdx.x + 1] = lg;
  }
}

// Per-block partials of the barrier function's slope along the primal step
// (-dx, -ds): [0] grad f . (-dx), [1] sum over finite bounds of
// -step / (v - lo) and +step / (hi - v) (times mu on the host).
__global__ void __launch_bounds__(kRedBlock) k_slope(Iter w, Step st, const double* __restrict__ grad, int64_t n,
                                                     int64_t m, double* __restrict__ part) {
  __shared__ double sh[kRedBlock];
  double gd = 0.0, bd = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const double p = -st.dx[i];
    gd += grad[i] * p;
    if (fin(w.xl[i])) bd -= p / (w.x[i] - w.xl[i]);
    if (fin(w.xu[i])) bd += p / (w.xu[i] - w.x[i]);
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
    const double p = -st.ds[i];
    if (fin(w.sl[i])) bd -= p / (w.s[i] - w.sl[i]);
    if (fin(w.su[i])) bd += p / (w.su[i] - w.s[i]);
  }
  block_reduce(sh, 1, gd);
  block_reduce(sh, 1, bd);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = gd;
    part[2 * blockIdx.x + 1] = bd;
  }
}

// Trial point x + a (-dx), s + a (-ds).
__global__ void k_trial(Iter w, Step st, double a, double* __restrict__ xt, double* __restrict__ stl, int64_t n,
                        int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) xt[i] = w.x[i] - a * st.dx[i];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) stl[i] = w.s[i] - a * st.ds[i];
}

// Accepts the trial point: x, s from (xt, st), y with the primal length a,
// the bound multipliers with the dual length ad, then each bound multiplier
// kept within [mu / (ks gap), ks mu / gap].
__device__ __forceinline__ double guard(double z, double gap, double mu, double ks) {
  return fmax(fmin(z, ks * mu / gap), mu / (ks * gap));
}

__global__ void k_accept(Iter w, Step st, const double* __restrict__ xt, const double* __restrict__ stl, double a,
                         double ad, double mu, double ks, int64_t n, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const double x = xt[i];
    w.x[i] = x;
    if (fin(w.xl[i])) w.zl[i] = guard(w.zl[i] - ad * st.dzl[i], x - w.xl[i], mu, ks);
    if (fin(w.xu[i])) w.zu[i] = guard(w.zu[i] - ad * st.dzu[i], w.xu[i] - x, mu, ks);
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
    const double s = stl[i];
    w.s[i] = s;
    w.y[i] += a * st.dy[i];
    w.ly[i] = -w.y[i];
    if (fin(w.sl[i])) w.vl[i] = guard(w.vl[i] - ad * st.dvl[i], s - w.sl[i], mu, ks);
    if (fin(w.su[i])) w.vu[i] = guard(w.vu[i] - ad * st.dvu[i], w.su[i] - s, mu, ks);
  }
}

int grid_of(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

#define IPM_CHK(x)                    \
  do {                                \
    const int rc_ = (x);              \
    if (rc_ != OPF_OK) return rc_;    \
  } while (0)

#define IPM_HIP(call, what)                                                                   \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return api_fail(OPF_EHIP, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Buffers {
  std::vector<void*> p;
  ~Buffers() {
    for (void* q : p) (void)hipFree(q);
  }
  int get(int64_t count, double** out) {
    if (hipMalloc((void**)out, (size_t)std::max<int64_t>(1, count) * sizeof(double)) != hipSuccess)
      return api_fail(OPF_ENOMEM, "ipm: device allocation failed");
    p.push_back(*out);
    return OPF_OK;
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace opf

using namespace opf;

extern "C" {

void opf_ipm_default_options(opf_ipm_options* o) {
  if (!o) return;
  o->tol = 1e-4;
  o->max_iter = 100;
  o->relax = 1e-4;
  o->sigma = 0.1;
  o->tau = 0.99995;
  o->delta_c = 1e-8;
  o->dw_first = 1e-4;
  o->dw_grow = 8.0;
  o->dw_max = 1e10;
  o->pivot_tol = 0.0;
  o->verbose = 0;
  o->line_search = 1;
  o->mu_init = 0.1;
  o->kappa_eps = 10.0;
  o->kappa_mu = 0.2;
  o->theta_mu = 1.5;
  o->tau_min = 0.99;
  o->gamma_theta = 1e-5;
  o->gamma_phi = 1e-8;
  o->eta_phi = 1e-8;
  o->s_theta = 1.1;
  o->s_phi = 2.3;
  o->delta = 1.0;
  o->gamma_alpha = 0.05;
  o->kappa_sigma = 1e10;
  o->stall_iter = 25;
  o->dw_grow_first = 100.0;
  o->dw_shrink = 1.0 / 3.0;
  o->dw_min = 1e-20;
}

int opf_ipm_solve(opf_model* M, opf_chol* F, const opf_ipm_options* opt_in, double* x_out, double* y_out,
                  opf_ipm_result* res) {
  if (!M || !F || !x_out || !res) return api_fail(OPF_EINVAL, "ipm: model, chol, x or result is NULL");
  if (model_device(M) < 0) return api_fail(OPF_ENODEV, "model is host-only");
  if (chol_model(F) != M) return api_fail(OPF_EINVAL, "ipm: chol was analysed from another model");
  opf_ipm_options opt;
  if (opt_in) opt = *opt_in;
  else opf_ipm_default_options(&opt);
  if (!(opt.tol > 0.0) || opt.max_iter < 0 || !(opt.relax >= 0.0) || !(opt.sigma > 0.0 && opt.sigma < 1.0) ||
      !(opt.tau > 0.0 && opt.tau < 1.0) || !(opt.delta_c >= 0.0) || !(opt.dw_first > 0.0) || !(opt.dw_grow > 1.0) ||
      !(opt.dw_max >= opt.dw_first) || !std::isfinite(opt.pivot_tol))
    return api_fail(OPF_EINVAL, "ipm: invalid options");
  if (opt.line_search &&
      (!(opt.mu_init > 0.0) || !(opt.kappa_eps > 0.0) || !(opt.kappa_mu > 0.0 && opt.kappa_mu < 1.0) ||
       !(opt.theta_mu > 1.0) || !(opt.tau_min > 0.0 && opt.tau_min < 1.0) || !(opt.gamma_theta > 0.0) ||
       !(opt.gamma_phi > 0.0) || !(opt.eta_phi > 0.0) || !(opt.s_theta > 1.0) || !(opt.s_phi > 1.0) ||
       !(opt.delta > 0.0) || !(opt.gamma_alpha > 0.0) || !(opt.kappa_sigma >= 1.0) || opt.stall_iter < 0 ||
       !(opt.dw_grow_first > 1.0) || !(opt.dw_shrink > 0.0 && opt.dw_shrink < 1.0) || !(opt.dw_min > 0.0)))
    return api_fail(OPF_EINVAL, "ipm: invalid line-search options");
  std::memset(res, 0, sizeof(*res));
  const double t_start = now_s();
  // a factorization with static pivots is discarded here, so it may stop at
  // its first one (the caller's setting is restored on every return)
  struct StopGuard {
    opf_chol* f;
    int keep;
    ~StopGuard() { (void)opf_chol_set_stop_on_pivot(f, keep); }
  } stop_guard{F, opf_chol_stop_on_pivot(F)};
  if (opf_chol_set_stop_on_pivot(F, 1) != OPF_OK) return OPF_EINVAL;
  hipStream_t st = model_stream(M);
  opf_dims d;
  IPM_CHK(opf_model_dims(M, &d));
  const int64_t n = d.n, m = d.m;
  Buffers B;
  double *x, *s, *y, *ly, *zl, *zu, *vl, *vu, *xl, *xu, *cl, *cu, *sl, *su;
  double *grad, *c, *jtv, *diag_x, *dcon, *rhs, *dx, *ds, *dy, *dzl, *dzu, *dvl, *dvu, *jv, *hv, *kv, *part, *fobj;
  double *xt, *stl, *ct;  // line-search trial point and its constraints
  // variable-length (n) and row-length (m) work vectors
  for (double** p : {&x, &xl, &xu, &zl, &zu, &grad, &jtv, &diag_x, &rhs, &dx, &dzl, &dzu, &xt}) IPM_CHK(B.get(n, p));
  for (double** p : {&s, &y, &ly, &vl, &vu, &cl, &cu, &sl, &su, &c, &dcon, &ds, &dy, &dvl, &dvu, &stl, &ct})
    IPM_CHK(B.get(m, p));
  IPM_CHK(B.get(d.nnz_jac, &jv));
  IPM_CHK(B.get(d.nnz_hess, &hv));
  IPM_CHK(B.get(d.nnz_kkt, &kv));
  IPM_CHK(B.get((int64_t)kRedGrid * kNR, &part));
  IPM_CHK(B.get(d.ninst, &fobj));
  int32_t* npert = nullptr;
  IPM_HIP(hipMalloc((void**)&npert, sizeof(int32_t)), "ipm: allocation");
  B.p.push_back(npert);

  // starting iterate
  IPM_CHK(opf_bounds(M, xl, xu, cl, cu));
  const auto& insts = model_insts(M);
  for (const auto& I : insts)
    hipLaunchKernelGGL(k_start_flat, dim3(grid_of(I.n)), dim3(256), 0, st, x + I.x_off, xl + I.x_off, xu + I.x_off,
                       I.n_p, I.N, I.G, I.T);
  IPM_CHK(opf_eval_cons(M, x, c));
  for (const auto& I : insts)
    hipLaunchKernelGGL(k_start_flows, dim3(grid_of(4LL * I.B * I.T)), dim3(256), 0, st, x + I.x_off, c + I.c_off,
                       I.n_p, I.m_p, I.N, I.B, I.G, I.T);
  hipLaunchKernelGGL(k_push_inside, dim3(grid_of(n)), dim3(256), 0, st, x, x, xl, xu, n);
  hipLaunchKernelGGL(k_start_rows, dim3(grid_of(m)), dim3(256), 0, st, cl, cu, opt.relax, sl, su, y, ly, vl, vu, m);
  hipLaunchKernelGGL(k_start_vars, dim3(grid_of(n)), dim3(256), 0, st, xl, xu, zl, zu, n);
  IPM_CHK(opf_eval_cons(M, x, c));
  hipLaunchKernelGGL(k_push_inside, dim3(grid_of(m)), dim3(256), 0, st, s, c, sl, su, m);
  IPM_HIP(hipGetLastError(), "ipm: start kernels");

  Iter w{x, s, y, ly, zl, zu, vl, vu, xl, xu, sl, su};
  Step stp{dx, ds, dy, dzl, dzu, dvl, dvu};
  std::vector<double> hp((size_t)kRedGrid * kNR);
  std::vector<double> fh(d.ninst);
  double t_eval = 0, t_fac = 0, t_sol = 0;
  int it = 0, nfact = 0, trials = 0;
  double err = 0.0;
  int status = OPF_IPM_MAX_ITER;
  // theta = |c - s|_1, f and sum ln(gaps) at (xx, ss), so that
  // phi = f - mu sum ln(gaps); cc = c(xx) (computed here when eval_c)
  auto theta_phi = [&](const double* xx, const double* ss, double* cc, bool eval_c, double& th, double& fv,
                       double& lgv) -> int {
    if (eval_c) IPM_CHK(opf_eval_cons(M, xx, cc));
    IPM_CHK(opf_eval_obj(M, xx, fobj));
    hipLaunchKernelGGL(k_barrier, dim3(kRedGrid), dim3(kRedBlock), 0, st, w, xx, ss, (const double*)cc, n, m, part);
    IPM_HIP(hipGetLastError(), "ipm: barrier kernel");
    IPM_HIP(hipMemcpyAsync(hp.data(), part, 2 * kRedGrid * sizeof(double), hipMemcpyDeviceToHost, st), "ipm: copy");
    IPM_HIP(hipMemcpyAsync(fh.data(), fobj, d.ninst * sizeof(double), hipMemcpyDeviceToHost, st), "ipm: copy");
    IPM_HIP(hipStreamSynchronize(st), "ipm: sync");
    double t = 0.0, lg = 0.0, f = 0.0;
    for (int b = 0; b < kRedGrid; ++b) {
      t += hp[2 * b];
      lg += hp[2 * b + 1];
    }
    for (double v : fh) f += v;
    th = t;
    fv = f;
    lgv = lg;
    return OPF_OK;
  };
  // filter line search state (monotone mu, filter emptied when mu changes)
  const bool ls = opt.line_search != 0;
  double mu = opt.mu_init;
  std::vector<std::pair<double, double>> filt;
  double theta_max = 0.0, theta_min = 0.0, th_best = 0.0, dw_last = 0.0;
  int it_best = 0;
  if (ls) {
    double th0 = 0.0, f0 = 0.0, lg0 = 0.0;
    IPM_CHK(theta_phi(x, s, c, false, th0, f0, lg0));
    theta_max = 1e4 * std::max(1.0, th0);
    theta_min = 1e-4 * std::max(1.0, th0);
    th_best = th0;
  }
  for (;; ++it) {
    double t0 = now_s();
    IPM_CHK(opf_eval_grad(M, x, grad));
    IPM_CHK(opf_eval_cons(M, x, c));
    IPM_CHK(opf_jtprod(M, x, y, jtv));
    hipLaunchKernelGGL(k_resid, dim3(kRedGrid), dim3(kRedBlock), 0, st, w, (const double*)grad, (const double*)jtv,
                       (const double*)c, n, m, part);
    IPM_HIP(hipGetLastError(), "ipm: residual kernel");
    IPM_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st), "ipm: copy");
    IPM_HIP(hipStreamSynchronize(st), "ipm: sync");
    t_eval += now_s() - t0;
    double r[kNR] = {0, 0, 0, 0, 0, 0, 0, 0, INFINITY};
    for (int b = 0; b < kRedGrid; ++b)
      for (int k = 0; k < kNR; ++k) {
        const double v = hp[b * kNR + k];
        r[k] = k <= 3 ? std::max(r[k], v) : (k == 8 ? std::min(r[k], v) : r[k] + v);
      }
    const double sd = std::max(1.0, r[6] / (double)(m + 2 * n) / 100.0);
    const double base = std::max({r[0] / sd, r[1] / sd, r[2]});
    err = std::max(base, r[3]);
    if (r[7] > 0.0 || !std::isfinite(err))
      return api_fail(OPF_EINVAL, "ipm: the iterate is not finite at iteration " + std::to_string(it));
    if (opt.verbose)
      std::fprintf(stderr, "ipm %3d  err %.3e  |p_x| %.3e  |p_s| %.3e  |c-s| %.3e  compl %.3e  mu %.3e\n", it, err,
                   r[0], r[1], r[2], r[3], ls ? mu : opt.sigma * r[4] / std::max(1.0, r[5]));
    if (err <= opt.tol) {
      status = OPF_IPM_CONVERGED;
      break;
    }
    if (it >= opt.max_iter) break;
    double tau_k = opt.tau;
    double th = 0.0, fcur = 0.0, lgcur = 0.0;
    if (ls) {
      // no progress towards feasibility for stall_iter iterations: stalled
      IPM_CHK(theta_phi(x, s, c, false, th, fcur, lgcur));
      if (th < 0.9 * th_best) {
        th_best = th;
        it_best = it;
      }
      if (opt.stall_iter > 0 && it - it_best >= opt.stall_iter && r[2] > opt.tol) {
        status = OPF_IPM_STALLED;
        break;
      }
      // monotone mu: lowered while the barrier problem is solved to
      // kappa_eps mu (its error: the complementarity products minus mu)
      while (mu > opt.tol / 10.0) {
        const double err_mu = std::max(base, r[5] > 0.0 ? std::max(r[3] - mu, mu - r[8]) : 0.0);
        if (err_mu > opt.kappa_eps * mu) break;
        mu = std::max(opt.tol / 10.0, std::min(opt.kappa_mu * mu, std::pow(mu, opt.theta_mu)));
        filt.clear();
      }
      tau_k = std::max(opt.tau_min, 1.0 - mu);
    } else {
      mu = opt.sigma * r[4] / std::max(1.0, r[5]);
    }
    // inertia-corrected condensed system
    double dw = 0.0;
    opf_ipm_state ist{x, s, y, zl, zu, vl, vu, xl, xu, sl, su, mu, dw, opt.delta_c};
    for (;;) {
      ist.delta_w = dw;
      t0 = now_s();
      IPM_CHK(opf_condensed_rhs(M, &ist, grad, c, diag_x, dcon, rhs));
      IPM_CHK(opf_eval_jhk(M, x, ly, 1.0, diag_x, dcon, jv, hv, kv));
      IPM_HIP(hipStreamSynchronize(st), "ipm: sync");
      t_eval += now_s() - t0;
      t0 = now_s();
      IPM_CHK(opf_chol_factor(F, kv, opt.pivot_tol, 1.0, npert));
      int32_t hn = 0;
      IPM_HIP(hipMemcpyAsync(&hn, npert, sizeof(int32_t), hipMemcpyDeviceToHost, st), "ipm: copy");
      IPM_HIP(hipStreamSynchronize(st), "ipm: sync");
      t_fac += now_s() - t0;
      ++nfact;
      if (opt.verbose > 1) std::fprintf(stderr, "      factorization  delta_w %.1e  static pivots %d\n", dw, hn);
      if (hn == 0) break;
      if (!ls)
        dw = dw == 0.0 ? opt.dw_first : dw * opt.dw_grow;
      else if (dw == 0.0)
        dw = dw_last == 0.0 ? opt.dw_first : std::max(opt.dw_min, opt.dw_shrink * dw_last);
      else
        dw *= dw_last == 0.0 ? opt.dw_grow_first : opt.dw_grow;
      if (dw > opt.dw_max) break;
    }
    if (dw > opt.dw_max) {
      // no positive definite condensed matrix within dw_max: no step to take
      if (opt.verbose) std::fprintf(stderr, "      delta_w above %.1e: no step\n", opt.dw_max);
      status = OPF_IPM_STALLED;
      break;
    }
    if (ls && dw > 0.0) dw_last = dw;
    t0 = now_s();
    IPM_CHK(opf_chol_solve(F, rhs, dx));
    IPM_CHK(opf_recover_step(M, &ist, c, dx, ds, dy, dzl, dzu, dvl, dvu));
    hipLaunchKernelGGL(k_steplen, dim3(kRedGrid), dim3(kRedBlock), 0, st, w, stp, tau_k, n, m, part);
    IPM_HIP(hipGetLastError(), "ipm: step kernel");
    IPM_HIP(hipMemcpyAsync(hp.data(), part, 2 * kRedGrid * sizeof(double), hipMemcpyDeviceToHost, st), "ipm: copy");
    IPM_HIP(hipStreamSynchronize(st), "ipm: sync");
    double ap = 1.0, ad = 1.0;
    for (int b = 0; b < kRedGrid; ++b) {
      ap = std::min(ap, hp[2 * b]);
      ad = std::min(ad, hp[2 * b + 1]);
    }
    if (!ls) {
      if (opt.verbose) std::fprintf(stderr, "      delta_w %.1e  alpha_p %.3e  alpha_d %.3e\n", ist.delta_w, ap, ad);
      hipLaunchKernelGGL(k_update, dim3(grid_of(std::max(n, m))), dim3(256), 0, st, w, stp, ap, ad, n, m);
      IPM_HIP(hipGetLastError(), "ipm: update kernel");
      t_sol += now_s() - t0;
      continue;
    }
    // filter line search from the fraction-to-the-boundary length
    const double ph = fcur - mu * lgcur;
    hipLaunchKernelGGL(k_slope, dim3(kRedGrid), dim3(kRedBlock), 0, st, w, stp, (const double*)grad, n, m, part);
    IPM_HIP(hipGetLastError(), "ipm: slope kernel");
    IPM_HIP(hipMemcpyAsync(hp.data(), part, 2 * kRedGrid * sizeof(double), hipMemcpyDeviceToHost, st), "ipm: copy");
    IPM_HIP(hipStreamSynchronize(st), "ipm: sync");
    double gd = 0.0, bd = 0.0;
    for (int b = 0; b < kRedGrid; ++b) {
      gd += hp[2 * b];
      bd += hp[2 * b + 1];
    }
    const double dph = gd + mu * bd;
    const double amin = dph < 0.0 ? opt.gamma_alpha * std::min({opt.gamma_theta, opt.gamma_phi * th / -dph,
                                                                 opt.delta * std::pow(th, opt.s_theta) /
                                                                     std::pow(-dph, opt.s_phi)})
                                  : opt.gamma_alpha * opt.gamma_theta;
    double a = ap;
    int kind = 0;  // 1: Armijo on phi, 2: sufficient decrease (the point joins the filter)
    for (;;) {
      hipLaunchKernelGGL(k_trial, dim3(grid_of(std::max(n, m))), dim3(256), 0, st, w, stp, a, xt, stl, n, m);
      IPM_HIP(hipGetLastError(), "ipm: trial kernel");
      double tht = 0.0, ft = 0.0, lgt = 0.0;
      IPM_CHK(theta_phi(xt, stl, ct, true, tht, ft, lgt));
      const double pht = ft - mu * lgt;
      ++trials;
      bool ok = tht <= theta_max;
      for (const auto& e : filt)
        if (!(tht < e.first || pht < e.second)) ok = false;
      if (ok) {
        const bool switching = dph < 0.0 && a * std::pow(-dph, opt.s_phi) > opt.delta * std::pow(th, opt.s_theta);
        if (switching && th <= theta_min) {
          if (pht <= ph + opt.eta_phi * a * dph) kind = 1;
        } else if (tht <= (1.0 - opt.gamma_theta) * th || pht <= ph - opt.gamma_phi * th) {
          kind = 2;
        }
      }
      if (kind) break;
      a *= 0.5;
      if (a < amin) break;
    }
    if (opt.verbose)
      std::fprintf(stderr, "      delta_w %.1e  alpha_p %.3e (of %.3e)  alpha_d %.3e  theta %.3e  %s\n", ist.delta_w,
                   kind ? a : 0.0, ap, ad, th, kind == 1 ? "armijo" : (kind == 2 ? "filter" : "no step"));
    if (!kind) {
      status = OPF_IPM_STALLED;
      t_sol += now_s() - t0;
      break;
    }
    if (kind == 2) filt.push_back({(1.0 - opt.gamma_theta) * th, ph - opt.gamma_phi * th});
    hipLaunchKernelGGL(k_accept, dim3(grid_of(std::max(n, m))), dim3(256), 0, st, w, stp, (const double*)xt,
                       (const double*)stl, a, ad, mu, opt.kappa_sigma, n, m);
    IPM_HIP(hipGetLastError(), "ipm: accept kernel");
    t_sol += now_s() - t0;
  }
  IPM_CHK(opf_eval_obj(M, x, fobj));
  IPM_HIP(hipMemcpyAsync(fh.data(), fobj, d.ninst * sizeof(double), hipMemcpyDeviceToHost, st), "ipm: copy");
  IPM_HIP(hipMemcpyAsync(x_out, x, n * sizeof(double), hipMemcpyDeviceToDevice, st), "ipm: copy");
  if (y_out) IPM_HIP(hipMemcpyAsync(y_out, y, m * sizeof(double), hipMemcpyDeviceToDevice, st), "ipm: copy");
  IPM_HIP(hipStreamSynchronize(st), "ipm: sync");
  double fsum = 0.0;
  for (double v : fh) fsum += v;
  res->converged = status == OPF_IPM_CONVERGED ? 1 : 0;
  res->status = status;
  res->trials = trials;
  {
    double th = 0.0, fv = 0.0, lgv = 0.0;
    IPM_CHK(opf_eval_cons(M, x, c));
    IPM_CHK(theta_phi(x, s, c, false, th, fv, lgv));
    res->theta = th;
  }
  res->iterations = it;
  res->factorizations = nfact;
  res->objective = fsum;
  res->err = err;
  res->seconds = now_s() - t_start;
  res->t_eval = t_eval;
  res->t_factor = t_fac;
  res->t_solve = t_sol;
  return OPF_OK;
}

}  // extern "C"
