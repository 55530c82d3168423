// Static-pivot sparse Cholesky of the condensed matrix (Sec. III-B): device
// kernels and the opf_chol_* entry points.
//
// Numeric scheme (multifrontal, the plan from opf_chol_symbolic.cpp):
//   * the factor of every interior front s of every period lives in one
//     column-major (p+u) x p block (p pivots, u update rows); its update
//     matrix (u x u, lower part) lives in a workspace arena until the
//     parent has collected it;
//   * K's entries are written straight into the factor blocks; each front
//     then pulls its children's update matrices (extend-add, no atomics: a
//     work item owns a set of the parent's columns), is factored in place
//     (small fronts in LDS by one wavefront, large ones by blocked panel +
//     trailing-update kernels), batched over the periods of a chunk;
//   * the pg front of period t (G pivots) collects the period's tree roots
//     and its chain neighbour's update: a chain over t, eliminated from both
//     ends at once (fronts t < m carry update rows pg_{t+1}, fronts t > m
//     update rows pg_{t-1}, front m closes it; m = (T - 1) / 2), one front of
//     each side per launch, its large trailing updates as library GEMMs (see
//     blas_update).
// Solves run the same tree forward (update vectors pulled by the parent)
// and backward (gathers of the ancestors' solution), batched over periods.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/opf.h"
#include "opf_api_internal.h"
#include "opf_chol_host.h"

namespace opf {
namespace {

constexpr int kSmall = 64;   // largest front factored in LDS by one wavefront
constexpr int kNB = 64;      // panel width of the blocked fronts
constexpr int kTile = 128;   // trailing-update tile (8 x 8 outputs per thread)
constexpr int kChainCols = 128;  // column chunk of the chain's L21 z
constexpr int kStep = 1024;      // columns per trailing update of a blocked front
// Trailing updates of at least this many rows below the panel and panel
// columns go to the library's strided-batched GEMM (plain dense products);
// smaller ones stay on k_update.
constexpr int kBlasMinRows = 512;
constexpr int kBlasMinCols = 64;
constexpr int kBlasCols = 512;  // target columns per library product
// Only the pg chain's fronts (one or two periods per launch) go to the
// library: so few periods give k_update too few tiles to fill the GPU, and
// the chain runs its steps in sequence (measured at paper scale on the
// one-ended chain: 1.132 -> 1.065 s per factorization from 128 panel
// columns, 1.000 s from 64; the library on the batched interior fronts as
// well was slower, its long-running blocks holding the CUs the chain's short
// launches wait for).  The interior passes no library handle.
constexpr int kBwdCols = 16;     // earlier columns updated per block of a backward panel (a multiple of 4)

// Device view of one instance's plan.
struct CDev {
  const int32_t *node_f, *node_p, *node_u, *rel, *kids, *rows;
  const int64_t *node_loff, *node_uoff, *node_woff, *row_ptr, *kid_ptr;
  int64_t lsize, usize, wsize;
  int32_t n_p, n_int, G;
  const int32_t* stop;  // the static-pivot count when the factor stops at the first one, else NULL
};

// One front as the blocked kernels see it: factor block (ld x p, first p
// columns of the front) and update block (ldU x u), per-period strides.
struct FrontArg {
  double* L;
  int64_t Lstride;
  int32_t ld, p, u;
  double* U;
  int64_t Ustride;
  int32_t ldU;
  const int32_t* stop;  // as CDev::stop
};

// Whether the factorization stops at its first static pivot and one has
// been counted: the count read once per block by its first thread and
// shared, so every thread of the block takes the same branch.  A count
// raised by a concurrent kernel may be seen one launch late; the factor is
// then only discarded later.
__device__ __forceinline__ bool stopped(const int32_t* stop) {
  if (!stop) return false;
  __shared__ int32_t seen;
  if (threadIdx.x == 0) seen = *reinterpret_cast<const volatile int32_t*>(stop);
  __syncthreads();
  return seen > 0;
}

__device__ __forceinline__ int lower_bound_i32(const int32_t* a, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void k_fill(double* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// K's template slots of periods t0 .. t0+nt-1 into the factor blocks (or the
// pg front's pivot block).  Every destination receives one entry.
__global__ void k_scatter(const double* __restrict__ kv, int64_t k_off, int64_t nnzk_p, int32_t G, int32_t t0,
                          int32_t nslots, const int64_t* __restrict__ dst, const int32_t* __restrict__ kpos0,
                          const int32_t* __restrict__ kpos1, double* __restrict__ Lf, int64_t lsize,
                          double* __restrict__ Cf, int64_t csize) {
  const int t = t0 + (int)blockIdx.y;
  const int64_t kp = k_off + (int64_t)t * nnzk_p + (t >= 1 ? (int64_t)(t - 1) * G : 0);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nslots; q += gridDim.x * blockDim.x) {
    const double v = kv[kp + (t == 0 ? kpos0[q] : kpos1[q])];
    const int64_t d = dst[q];
    if (d >= 0) Lf[(int64_t)t * lsize + d] = v;
    else Cf[(int64_t)t * csize + (-1 - d)] = v;
  }
}

// The ramp pairs (pg_t,g , pg_{t-1},g), t in [t0, t0 + gridDim.y), t >= 1:
// entries of the L21 block (row G + g, column g) of the one of the two pg
// fronts that the chain eliminates first: front t-1 when t <= m (the chain's
// left side), front t otherwise (its right side).
__global__ void k_scatter_ramp(const double* __restrict__ kv, int64_t k_off, int64_t nnzk_p, int32_t G, int32_t t0,
                               int32_t m, const int32_t* __restrict__ ramp_pos, double* __restrict__ Cf,
                               int64_t csize) {
  const int t = t0 + (int)blockIdx.y;
  const int64_t kp = k_off + (int64_t)t * nnzk_p + (int64_t)(t - 1) * G;
  const int f = t <= m ? t - 1 : t;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x)
    Cf[(int64_t)f * csize + (int64_t)g * 2 * G + G + g] = kv[kp + ramp_pos[g]];
}

// Extend-add for the fronts of one level: work item (s, c0) owns columns
// [c0, c0 + cb) of front s; it clears their update part, then adds each
// child's update matrix entries that land there, child by child.
__global__ void __launch_bounds__(256) k_extend(CDev D, const int32_t* __restrict__ items, int64_t item0,
                                                int32_t cb, int32_t t0, double* __restrict__ Lf,
                                                double* __restrict__ Ar) {
  if (stopped(D.stop)) return;
  const int tt = (int)blockIdx.y;
  const int s = items[2 * (item0 + blockIdx.x)], c0 = items[2 * (item0 + blockIdx.x) + 1];
  const int p = D.node_p[s], u = D.node_u[s], ld = p + u;
  const int c1 = min(c0 + cb, ld);
  double* L = Lf + (int64_t)(t0 + tt) * D.lsize + D.node_loff[s];
  double* U = Ar + (int64_t)tt * D.usize + D.node_uoff[s];
  for (int j = max(c0, p); j < c1; ++j)
    for (int i = j + (int)threadIdx.x; i < ld; i += (int)blockDim.x) U[(int64_t)(j - p) * u + (i - p)] = 0.0;
  __syncthreads();
  for (int64_t q = D.kid_ptr[s]; q < D.kid_ptr[s + 1]; ++q) {
    const int c = D.kids[q];
    const int uc = D.node_u[c];
    const int32_t* rel = D.rel + D.row_ptr[c];
    const double* Uc = Ar + (int64_t)tt * D.usize + D.node_uoff[c];
    const int b0 = lower_bound_i32(rel, uc, c0), b1 = lower_bound_i32(rel, uc, c1);
    for (int b = b0; b < b1; ++b) {
      const int j = rel[b];
      double* dcol = j < p ? L + (int64_t)j * ld : U + (int64_t)(j - p) * u - p;  // row i at dcol[i]
      const double* scol = Uc + (int64_t)b * uc;
      // four entries per lane in flight: every load before any store (the
      // child's entries of one column land on distinct parent entries)
      constexpr int UN = 4;
      const int bd = (int)blockDim.x;
      for (int a = b + (int)threadIdx.x; a < uc; a += UN * bd) {
        int ii[UN];
        double vv[UN], pv[UN];
#pragma unroll
        for (int k = 0; k < UN; ++k) {
          const int aa = a + k * bd;
          ii[k] = aa < uc ? rel[aa] : -1;
          vv[k] = aa < uc ? scol[aa] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < UN; ++k) pv[k] = ii[k] >= 0 ? dcol[ii[k]] : 0.0;
#pragma unroll
        for (int k = 0; k < UN; ++k)
          if (ii[k] >= 0) dcol[ii[k]] = pv[k] + vv[k];
      }
    }
    __syncthreads();
  }
}

// The period's tree roots into its pg front (ld 2G, pivot block only).
__global__ void __launch_bounds__(256) k_extend_root(CDev D, const int32_t* __restrict__ roots, int32_t nroots,
                                                     int32_t cb, int32_t t0, double* __restrict__ Cf, int64_t csize,
                                                     const double* __restrict__ Ar) {
  if (stopped(D.stop)) return;
  const int tt = (int)blockIdx.y;
  const int c0 = (int)blockIdx.x * cb, c1 = min(c0 + cb, D.G);
  double* L = Cf + (int64_t)(t0 + tt) * csize;
  const int64_t ld = 2 * (int64_t)D.G;
  for (int k = 0; k < nroots; ++k) {
    const int c = roots[k];
    const int uc = D.node_u[c];
    const int32_t* rel = D.rel + D.row_ptr[c];
    const double* Uc = Ar + (int64_t)tt * D.usize + D.node_uoff[c];
    const int b0 = lower_bound_i32(rel, uc, c0), b1 = lower_bound_i32(rel, uc, c1);
    for (int b = b0; b < b1; ++b) {
      const int j = rel[b];
      for (int a = b + (int)threadIdx.x; a < uc; a += (int)blockDim.x)
        L[(int64_t)j * ld + rel[a]] += Uc[(int64_t)b * uc + a];
    }
    __syncthreads();
  }
}

// Static pivot rule: d <= tol (or NaN) is replaced by repl and counted.
__device__ __forceinline__ double pivot_sqrt(double d, double tol, double repl, int32_t* npert, bool count) {
  if (!(d > tol)) {
    d = repl;
    if (count) atomicAdd(npert, 1);
  }
  return sqrt(d);
}

// Broadcast of lane l's value to the whole wavefront (l uniform).
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const int2 w = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(w.x, l);
  r.y = __builtin_amdgcn_readlane(w.y, l);
  return __builtin_bit_cast(double, r);
}

// Right-looking elimination of the first p pivots of a front of order f <=
// 64 held by one wavefront, lane i owning row i in registers (a[j] = entry
// (i, j) for j <= i; the entries above the diagonal are scratch that no
// valid entry ever reads, so the updates run unmasked).  Pivot d_k comes
// from the broadcast diagonal; entry (j, k) of column k is broadcast from
// lane j.  Fully unrolled so that every register index is a constant.
__device__ __forceinline__ void chol_rows64(double (&a)[64], int p, int f, double tol, double repl,
                                            int32_t* npert) {
  const int i = (int)threadIdx.x;
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    if (k < p) {
      const double d = pivot_sqrt(lane_bcast(a[k], k), tol, repl, npert, i == 0);
      const double rd = 1.0 / d;
      a[k] = i > k ? a[k] * rd : (i == k ? d : a[k]);
#pragma unroll
      for (int j = k + 1; j < 64; ++j) {
        if (j < f) a[j] = fma(-a[k], lane_bcast(a[k], j), a[j]);
      }
    }
  }
}

// Small fronts (p + u <= 64): one wavefront per (front, period), the front
// in registers (one row per lane).
__global__ void __launch_bounds__(64) k_factor_small(CDev D, const int32_t* __restrict__ list, int64_t l0,
                                                     int32_t t0, double* __restrict__ Lf, double* __restrict__ Ar,
                                                     double tol, double repl, int32_t* __restrict__ npert) {
  if (stopped(D.stop)) return;
  const int tt = (int)blockIdx.y;
  const int s = list[l0 + blockIdx.x];
  const int p = D.node_p[s], u = D.node_u[s], f = p + u;
  const int i = (int)threadIdx.x;
  double* L = Lf + (int64_t)(t0 + tt) * D.lsize + D.node_loff[s];
  double* U = Ar + (int64_t)tt * D.usize + D.node_uoff[s];
  double a[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    a[j] = 0.0;
    if (j < f && i >= j && i < f) a[j] = j < p ? L[(int64_t)j * f + i] : U[(int64_t)(j - p) * u + (i - p)];
  }
  chol_rows64(a, p, f, tol, repl, npert);
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < f && i >= j && i < f) {
      if (j < p) L[(int64_t)j * f + i] = a[j];
      else U[(int64_t)(j - p) * u + (i - p)] = a[j];
    }
}

// Blocked front, one panel [k0, k0+kb), step 1: the kb x kb diagonal block
// factored in place by one wavefront per period (pivots counted here).
__global__ void __launch_bounds__(64) k_diag(FrontArg A, int32_t k0, int32_t kb, double tol, double repl,
                                             int32_t* __restrict__ npert) {
  if (stopped(A.stop)) return;
  double* L = A.L + (int64_t)blockIdx.x * A.Lstride;
  const int64_t ld = A.ld;
  const int i = (int)threadIdx.x;
  double a[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) a[j] = (j < kb && i >= j && i < kb) ? L[(int64_t)(k0 + j) * ld + k0 + i] : 0.0;
  chol_rows64(a, kb, kb, tol, repl, npert);
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < kb && i >= j && i < kb) L[(int64_t)(k0 + j) * ld + k0 + i] = a[j];
}

// Step 2: the rows below the panel, L21 = A21 L11^-T, 256 rows per block
// against the factored diagonal block (read-only here).
__global__ void __launch_bounds__(256) k_panel(FrontArg A, int32_t k0, int32_t kb) {
  __shared__ double Dg[kNB * (kNB + 1)];
  __shared__ double rdg[kNB];
  constexpr int S = kNB + 1;
  if (stopped(A.stop)) return;
  double* L = A.L + (int64_t)blockIdx.y * A.Lstride;
  const int64_t ld = A.ld;
  const int rows = A.p + A.u;
  const int tid = (int)threadIdx.x;
  for (int e = tid; e < kb * kb; e += (int)blockDim.x) {
    const int j = e / kb, i = e % kb;
    if (i >= j) Dg[j * S + i] = L[(int64_t)(k0 + j) * ld + k0 + i];
  }
  if (tid < kb) rdg[tid] = 1.0 / L[(int64_t)(k0 + tid) * ld + k0 + tid];
  __syncthreads();
  const int r = k0 + kb + (int)blockIdx.x * (int)blockDim.x + tid;
  if (r >= rows) return;
  double x[kNB];
#pragma unroll
  for (int j = 0; j < kNB; ++j) x[j] = j < kb ? L[(int64_t)(k0 + j) * ld + r] : 0.0;
#pragma unroll
  for (int j = 0; j < kNB; ++j) {
    if (j < kb) {
      double sacc = x[j];
#pragma unroll
      for (int l = 0; l < j; ++l) sacc -= x[l] * Dg[l * S + j];
      x[j] = sacc * rdg[j];
    }
  }
#pragma unroll
  for (int j = 0; j < kNB; ++j)
    if (j < kb) L[(int64_t)(k0 + j) * ld + r] = x[j];
}

// Trailing update after a panel: C -= P P^T on the lower part of rows and
// columns [k0+kb, p+u), 128 x 128 tiles on the FP64 matrix cores: each of
// the 4 wavefronts accumulates a 64 x 64 quarter as 4 x 4 products of
// 16 x 16 x 4 (v_mfma_f64_16x16x4: lane l supplies A(l%16, l/16) and
// B(l/16, l%16) and holds D(l/16 + 4r, l%16), r < 4).  The product is
// formed transposed (rows of the tile along the lanes) so that each lane
// group writes 16 consecutive rows of a column of the column-major front.
// The panel is staged through LDS 16 columns at a time.  Columns < p live
// in the factor block, the others in the update block.
typedef double dbl4 __attribute__((ext_vector_type(4)));

// Region: rows [r0, p+u) x columns [r0, min(cmax, p+u)), lower part, in
// 128 x 128 tiles enumerated column by column; panel columns [k0, k0+kb),
// kb <= 1024.  With dnext > 0, block 0 (the tile holding rows and columns
// [r0, r0+128)) then factors the next diagonal block [r0, r0+dnext) in
// place, which the next panel needs.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_update(FrontArg A, int32_t k0, int32_t kb, int32_t r0, int32_t cmax, int32_t dnext, double tol, double repl,
         int32_t* __restrict__ npert) {
  constexpr int KC = 16;
  constexpr int NLD = KC * kTile / 256;  // panel values per thread per chunk and side
  // two LDS buffers: the next chunk is loaded into registers while the
  // matrix cores work on the current one
  __shared__ double Pi[2][KC][kTile], Pj[2][KC][kTile];
  if (stopped(A.stop)) return;
  const int rows = A.p + A.u;
  const int R = (rows - r0 + kTile - 1) / kTile;
  // blocks are dealt round-robin to the 8 XCDs in launch order; give each
  // XCD a contiguous run of (period, tile) items so that neighbouring tiles,
  // which share panel slices, meet in the same L2
  const int ntl = (int)gridDim.x, total = ntl * (int)gridDim.y;
  int item = (int)(blockIdx.y * gridDim.x + blockIdx.x);
  const int q8 = total >> 3;
  if (item < (q8 << 3)) item = (item & 7) * q8 + (item >> 3);
  const int per = item / ntl;
  int x = item % ntl, tj = 0;
  while (x >= R - tj) {
    x -= R - tj;
    ++tj;
  }
  const int ti = tj + x;
  const int cend = min(cmax, rows);
  double* L = A.L + (int64_t)per * A.Lstride;
  double* U = A.U + (int64_t)per * A.Ustride;
  const int64_t ld = A.ld;
  const int i0 = r0 + ti * kTile, j0 = r0 + tj * kTile;
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv & 1, wc = wv >> 1;  // the wavefront's 64-row / 64-column quarter
  // a quarter wholly above the diagonal or right of the region contributes nothing
  const bool skip = i0 + wr * 64 + 63 < j0 + wc * 64 || j0 + wc * 64 >= cend;
  dbl4 acc[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[c][r] = (dbl4){0.0, 0.0, 0.0, 0.0};
  const int lr = lane & 15, lk = lane >> 4;
  double ri[NLD], rj[NLD];
  auto fetch = [&](int l0) {
    const int lb = min(KC, kb - l0);
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int e = tid + q * 256;
      const int l = e / kTile, rr = e % kTile;
      const int64_t col = (int64_t)(k0 + l0 + l) * ld;
      ri[q] = (l < lb && i0 + rr < rows) ? L[col + i0 + rr] : 0.0;
      rj[q] = (l < lb && j0 + rr < cend) ? L[col + j0 + rr] : 0.0;
    }
  };
  auto park = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int e = tid + q * 256;
      Pi[buf][e / kTile][e % kTile] = ri[q];
      Pj[buf][e / kTile][e % kTile] = rj[q];
    }
  };
  fetch(0);
  park(0);
  __syncthreads();
  int buf = 0;
  for (int l0 = 0; l0 < kb; l0 += KC) {
    const int lb = min(KC, kb - l0);
    const bool more = l0 + KC < kb;
    if (more) fetch(l0 + KC);
    if (!skip) {
      for (int k4 = 0; k4 < lb; k4 += 4) {
        double aj[4], bi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          aj[q] = Pj[buf][k4 + lk][wc * 64 + q * 16 + lr];
          bi[q] = Pi[buf][k4 + lk][wr * 64 + q * 16 + lr];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[c][r] = __builtin_amdgcn_mfma_f64_16x16x4f64(aj[c], bi[r], acc[c][r], 0, 0, 0);
      }
    }
    if (more) park(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (!skip) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 64 + r * 16 + lr;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = j0 + wc * 64 + c * 16 + lk + 4 * e;
          if (i >= rows || j >= cend || i < j) continue;
          if (j < A.p) L[(int64_t)j * ld + i] -= acc[c][r][e];
          else U[(int64_t)(j - A.p) * A.ldU + (i - A.p)] -= acc[c][r][e];
        }
      }
  }
  if (dnext > 0 && x == 0 && tj == 0) {
    __syncthreads();
    if (wv == 0) {
      double a[64];
#pragma unroll
      for (int j = 0; j < 64; ++j)
        a[j] = (j < dnext && lane >= j && lane < dnext) ? L[(int64_t)(r0 + j) * ld + r0 + lane] : 0.0;
      chol_rows64(a, dnext, dnext, tol, repl, npert);
#pragma unroll
      for (int j = 0; j < 64; ++j)
        if (j < dnext && lane >= j && lane < dnext) L[(int64_t)(r0 + j) * ld + r0 + lane] = a[j];
    }
  }
}

// G x G lower update block of pg front t-1 into the pivot block of front t.
__global__ void k_add_chain(const double* __restrict__ Us, int32_t G, double* __restrict__ C) {
  const int64_t n = (int64_t)G * G;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / G, i = e % G;
    if (i >= j) C[j * 2 * G + i] += Us[e];
  }
}

// ------------------------------------------------------------------ solves
__global__ void k_sub(double* __restrict__ y, const double* __restrict__ w, int32_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[i] -= w[i];
}

__global__ void k_gather(const double* __restrict__ b, int32_t n_p, int32_t T, const int32_t* __restrict__ perm,
                         double* __restrict__ Y) {
  const int64_t n = (int64_t)n_p * T;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e / n_p, k = e % n_p;
    Y[e] = b[t * n_p + perm[k]];
  }
}

__global__ void k_scatter_out(const double* __restrict__ Y, int32_t n_p, int32_t T,
                              const int32_t* __restrict__ perm, double* __restrict__ x) {
  const int64_t n = (int64_t)n_p * T;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e / n_p, k = e % n_p;
    x[t * n_p + perm[k]] = Y[e];
  }
}

// Forward, small fronts: v = b(pivots) - children's pivot-row updates,
// children's other rows summed into this front's update vector, then
// L11 z = v and w += L21 z.  W holds, per front, what its subtree
// subtracts from the right-hand side at the front's update rows.
__global__ void __launch_bounds__(64) k_fwd_small(CDev D, const int32_t* __restrict__ list, int64_t l0,
                                                  const double* __restrict__ Lf, double* __restrict__ Y,
                                                  double* __restrict__ W) {
  __shared__ double v[kSmall];
  const int t = (int)blockIdx.y;
  const int s = list[l0 + blockIdx.x];
  const int p = D.node_p[s], u = D.node_u[s], f = p + u, fs = D.node_f[s];
  const int i = (int)threadIdx.x;
  const double* L = Lf + (int64_t)t * D.lsize + D.node_loff[s];
  double* Yt = Y + (int64_t)t * D.n_p;
  double* Wt = W + (int64_t)t * D.wsize;
  if (i < f) v[i] = i < p ? Yt[fs + i] : 0.0;
  __syncthreads();
  for (int64_t q = D.kid_ptr[s]; q < D.kid_ptr[s + 1]; ++q) {
    const int c = D.kids[q];
    const int uc = D.node_u[c];
    const int32_t* rel = D.rel + D.row_ptr[c];
    const double* Wc = Wt + D.node_woff[c];
    for (int a = i; a < uc; a += (int)blockDim.x) {
      const int r = rel[a];
      if (r < p) v[r] -= Wc[a];
      else v[r] += Wc[a];
    }
    __syncthreads();
  }
  for (int k = 0; k < p; ++k) {
    if (i == k) v[k] /= L[(int64_t)k * f + k];
    __syncthreads();
    if (i > k && i < f) {
      const double z = v[k] * L[(int64_t)k * f + i];
      if (i < p) v[i] -= z;
      else v[i] += z;
    }
    __syncthreads();
  }
  if (i < p) Yt[fs + i] = v[i];
  else if (i < f) Wt[D.node_woff[s] + i - p] = v[i];
}

// Forward, large front, step 1: pull the children's update vectors (pivot
// rows subtracted from Y in place, other rows summed into this front's W).
__global__ void __launch_bounds__(256) k_fwd_pull(CDev D, int32_t s, double* __restrict__ Y,
                                                  double* __restrict__ W) {
  const int t = (int)blockIdx.x;
  const int p = D.node_p[s], u = D.node_u[s], fs = D.node_f[s];
  double* Yt = Y + (int64_t)t * D.n_p;
  double* Wt = W + (int64_t)t * D.wsize;
  double* Ws = Wt + D.node_woff[s];
  for (int a = (int)threadIdx.x; a < u; a += (int)blockDim.x) Ws[a] = 0.0;
  __syncthreads();
  for (int64_t q = D.kid_ptr[s]; q < D.kid_ptr[s + 1]; ++q) {
    const int c = D.kids[q];
    const int uc = D.node_u[c];
    const int32_t* rel = D.rel + D.row_ptr[c];
    const double* Wc = Wt + D.node_woff[c];
    for (int a = (int)threadIdx.x; a < uc; a += (int)blockDim.x) {
      const int r = rel[a];
      if (r < p) Yt[fs + r] -= Wc[a];
      else Ws[r - p] += Wc[a];
    }
    __syncthreads();
  }
}

// The period's tree roots' update vectors into its pg right-hand side.
__global__ void __launch_bounds__(256) k_fwd_root_pull(CDev D, const int32_t* __restrict__ roots, int32_t nroots,
                                                       double* __restrict__ Y, const double* __restrict__ W) {
  const int t = (int)blockIdx.x;
  double* Yp = Y + (int64_t)t * D.n_p + D.n_int;
  const double* Wt = W + (int64_t)t * D.wsize;
  for (int k = 0; k < nroots; ++k) {
    const int c = roots[k];
    const int uc = D.node_u[c];
    const int32_t* rel = D.rel + D.row_ptr[c];
    const double* Wc = Wt + D.node_woff[c];
    for (int a = (int)threadIdx.x; a < uc; a += (int)blockDim.x) Yp[rel[a]] -= Wc[a];
    __syncthreads();
  }
}

// Forward triangle L11 z = y (pivot part of one front), one panel
// [k0, k0+kb) per launch, grid (row blocks, periods): every block solves
// the panel's diagonal triangle (staged in LDS, one wavefront, the solved
// entry broadcast across lanes) from y, block 0 stores the solution in z,
// and each block subtracts the panel's contribution from its 256 rows of y
// below the panel.  y's panel entries are only read here and z is only
// written, so the blocks of one launch never touch an entry another block
// writes.
__global__ void __launch_bounds__(256) k_fwd_panel(const double* __restrict__ Lb, int64_t Lstride, int32_t ld,
                                                   int32_t p, int32_t k0, double* __restrict__ yb,
                                                   double* __restrict__ zb, int64_t ystride) {
  __shared__ double Tr[64 * 65];
  __shared__ double xs[64];
  const double* L = Lb + (int64_t)blockIdx.y * Lstride;
  double* y = yb + (int64_t)blockIdx.y * ystride;
  double* z = zb + (int64_t)blockIdx.y * ystride;
  const int tid = (int)threadIdx.x;
  const int kb = min(64, p - k0);
  // this thread's row of the panel below the triangle, loaded first so that
  // its latency overlaps the triangle (summed in column order afterwards)
  const int i = k0 + kb + (int)blockIdx.x * (int)blockDim.x + tid;
  const bool row = i < p;
  double rv[64];
#pragma unroll
  for (int l = 0; l < 64; ++l) rv[l] = (row && l < kb) ? L[(int64_t)(k0 + l) * ld + i] : 0.0;
  for (int e = tid; e < 64 * 64; e += (int)blockDim.x) {
    const int c = e >> 6, r = e & 63;
    if (c < kb && r < kb && r >= c) Tr[c * 65 + r] = L[(int64_t)(k0 + c) * ld + k0 + r];
  }
  __syncthreads();
  if (tid < 64) {
    // lane i holds entry i and the reciprocal of its diagonal; step k
    // broadcasts entry k and its reciprocal (uniform lane reads)
    double vi = tid < kb ? y[k0 + tid] : 0.0;
    const double ri = tid < kb ? 1.0 / Tr[tid * 65 + tid] : 0.0;
    for (int k = 0; k < kb; ++k) {
      const double xk = lane_bcast(vi, k) * lane_bcast(ri, k);
      if (tid == k) vi = xk;
      else if (tid > k && tid < kb) vi -= Tr[k * 65 + tid] * xk;
    }
    xs[tid] = vi;
    if (blockIdx.x == 0 && tid < kb) z[k0 + tid] = vi;
  }
  __syncthreads();
  if (row) {
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < 64; ++l)
      if (l < kb) acc += rv[l] * xs[l];
    y[i] -= acc;
  }
}

// w = L21 z with the columns split over chunks of cc (grid: row blocks x
// chunks); partial sums part[chunk][u], summed in chunk order next.
__global__ void __launch_bounds__(256) k_gemv_part(const double* __restrict__ L, int32_t ld, int32_t p, int32_t u,
                                                   const double* __restrict__ z, int32_t cc,
                                                   double* __restrict__ part) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= u) return;
  const int k0 = (int)blockIdx.y * cc, k1 = min(p, k0 + cc);
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) acc += L[(int64_t)k * ld + p + i] * z[k];
  part[(int64_t)blockIdx.y * u + i] = acc;
}

__global__ void k_gemv_sum(const double* __restrict__ part, int32_t nch, int32_t u, double* __restrict__ w) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= u) return;
  double acc = 0.0;
  for (int c = 0; c < nch; ++c) acc += part[(int64_t)c * u + i];
  w[i] = acc;
}

// Forward, w[i] (+)= sum_k L21[i, k] z[k] over the u update rows (rows p ..
// p+u-1 of the factor block); grid (row blocks, periods).
__global__ void __launch_bounds__(256) k_fwd_gemv(const double* __restrict__ Lb, int64_t Lstride, int32_t ld,
                                                  int32_t p, int32_t u, const double* __restrict__ zb,
                                                  int64_t zstride, double* __restrict__ wb, int64_t wstride,
                                                  int32_t accumulate) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= u) return;
  const double* L = Lb + (int64_t)blockIdx.y * Lstride + p + i;
  const double* z = zb + (int64_t)blockIdx.y * zstride;
  double acc = 0.0;
  for (int k = 0; k < p; ++k) acc += L[(int64_t)k * ld] * z[k];
  double* w = wb + (int64_t)blockIdx.y * wstride;
  w[i] = accumulate ? w[i] + acc : acc;
}

// Backward, v[j] = y[j] - sum_i L21[i, j] x_u[i] for the p pivot columns,
// one wavefront per column; x_u gathered through rows (or contiguous when
// rows is NULL).  Grid (column blocks of 4, periods).
__global__ void __launch_bounds__(256) k_bwd_gemv(const double* __restrict__ Lb, int64_t Lstride, int32_t ld,
                                                  int32_t p, int32_t u, const int32_t* __restrict__ rows,
                                                  const double* __restrict__ xb, int64_t xstride,
                                                  double* __restrict__ yb, int64_t ystride) {
  const int j = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  const int lane = (int)(threadIdx.x & 63);
  if (j >= p) return;
  const double* col = Lb + (int64_t)blockIdx.y * Lstride + (int64_t)j * ld + p;
  const double* xs = xb + (int64_t)blockIdx.y * xstride;
  double acc = 0.0;
  for (int a = lane; a < u; a += 64) acc += col[a] * xs[rows ? rows[a] : a];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) yb[(int64_t)blockIdx.y * ystride + j] -= acc;
}

// Backward triangle L11^T x = z (pivot part of one front), one panel
// [k0, k0+kb) per launch, panels from the last: every block solves the
// panel's triangle from z (panel entries only read here), block 0 stores x
// in y, and each block's 4 wavefronts subtract the panel's contribution
// from their columns j < k0 of z (one wavefront per column, lanes over the
// panel's rows).  Grid (column blocks of kBwdCols, periods).
__global__ void __launch_bounds__(256) k_bwd_panel(const double* __restrict__ Lb, int64_t Lstride, int32_t ld,
                                                   int32_t p, int32_t k0, double* __restrict__ yb,
                                                   double* __restrict__ zb, int64_t ystride) {
  __shared__ double Tr[64 * 65];
  __shared__ double xs[64];
  const double* L = Lb + (int64_t)blockIdx.y * Lstride;
  double* y = yb + (int64_t)blockIdx.y * ystride;
  double* z = zb + (int64_t)blockIdx.y * ystride;
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int kb = min(64, p - k0);
  // this wavefront's columns j < k0 (jb + wv, + 4, ...): their panel
  // entries, loaded first so that their latency overlaps the triangle
  const int jb = (int)blockIdx.x * kBwdCols, je = min(jb + kBwdCols, k0);
  constexpr int kPerWave = kBwdCols / 4;
  double cv[kPerWave];
#pragma unroll
  for (int q = 0; q < kPerWave; ++q) {
    const int j = jb + wv + 4 * q;
    cv[q] = (j < je && lane < kb) ? L[(int64_t)j * ld + k0 + lane] : 0.0;
  }
  for (int e = tid; e < 64 * 64; e += (int)blockDim.x) {
    const int c = e >> 6, r = e & 63;
    if (c < kb && r < kb && r >= c) Tr[c * 65 + r] = L[(int64_t)(k0 + c) * ld + k0 + r];
  }
  __syncthreads();
  if (tid < 64) {
    double vj = tid < kb ? z[k0 + tid] : 0.0;
    const double rj = tid < kb ? 1.0 / Tr[tid * 65 + tid] : 0.0;
    for (int k = kb - 1; k >= 0; --k) {
      const double xk = lane_bcast(vj, k) * lane_bcast(rj, k);
      if (tid == k) vj = xk;
      else if (tid < k) vj -= Tr[tid * 65 + k] * xk;
    }
    xs[tid] = tid < kb ? vj : 0.0;
    if (blockIdx.x == 0 && tid < kb) y[k0 + tid] = vj;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPerWave; ++q) {
    const int j = jb + wv + 4 * q;
    if (j < je) {
      double acc = lane < kb ? cv[q] * xs[lane] : 0.0;
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (lane == 0) z[j] -= acc;
    }
  }
}

// Backward, small fronts: gather x at the update rows, v = y - L21^T x_u,
// then L11^T x = v.
__global__ void __launch_bounds__(64) k_bwd_small(CDev D, const int32_t* __restrict__ list, int64_t l0,
                                                  const double* __restrict__ Lf, double* __restrict__ Y) {
  __shared__ double v[kSmall], xu[kSmall];
  const int t = (int)blockIdx.y;
  const int s = list[l0 + blockIdx.x];
  const int p = D.node_p[s], u = D.node_u[s], f = p + u, fs = D.node_f[s];
  const int i = (int)threadIdx.x;
  const double* L = Lf + (int64_t)t * D.lsize + D.node_loff[s];
  double* Yt = Y + (int64_t)t * D.n_p;
  const int32_t* rows = D.rows + D.row_ptr[s];
  if (i < u) xu[i] = Yt[rows[i]];
  __syncthreads();
  if (i < p) {
    double acc = Yt[fs + i];
    for (int a = 0; a < u; ++a) acc -= L[(int64_t)i * f + p + a] * xu[a];
    v[i] = acc;
  }
  __syncthreads();
  for (int k = p - 1; k >= 0; --k) {
    if (i == k) v[k] /= L[(int64_t)k * f + k];
    __syncthreads();
    if (i < k) v[i] -= L[(int64_t)i * f + k] * v[k];
    __syncthreads();
  }
  if (i < p) Yt[fs + i] = v[i];
}

int grid_for(int64_t n, int block) {
  const int64_t g = (n + block - 1) / block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65535));
}

}  // namespace
}  // namespace opf

using namespace opf;

// ------------------------------------------------------------------ object
namespace {

struct CholInst {
  CholPlan plan;
  const InstHost* I = nullptr;
  CDev dev{};
  int32_t *d_node_f = nullptr, *d_node_p = nullptr, *d_node_u = nullptr, *d_rel = nullptr, *d_kids = nullptr,
          *d_rows = nullptr, *d_perm = nullptr, *d_items = nullptr, *d_small = nullptr, *d_roots = nullptr,
          *d_kpos0 = nullptr, *d_kpos1 = nullptr, *d_ramp = nullptr;
  int64_t *d_loff = nullptr, *d_uoff = nullptr, *d_woff = nullptr, *d_rowptr = nullptr, *d_kidptr = nullptr,
          *d_slot = nullptr;
  double *Lf = nullptr, *Cf = nullptr, *Ar = nullptr, *W = nullptr, *Wc = nullptr, *Y = nullptr, *Z = nullptr;
  double* Gp = nullptr;  // column-chunk partials of the chain's L21 z
  std::vector<int64_t> woff;  // per-front offsets of the forward update vectors
  int64_t csize = 0, wsize = 0;
  int32_t chunk = 1, nlarge = 0;
};

}  // namespace

struct opf_chol {
  opf_model* model = nullptr;
  int device = -1;
  std::vector<CholInst> inst;
  double* Us = nullptr;  // two G x G update blocks of the pg chain, one per end (largest G)
  // the pg chain runs on a stream of its own, chunk by chunk, behind the
  // interior fronts of the next chunk (events order the two)
  hipStream_t cs = nullptr;
  std::vector<hipEvent_t> evs;
  // the large fronts of one level are independent: they are dealt in turn
  // to the model's stream and these streams, forked and joined by events per
  // level.  One is enough: with the model's and the chain's stream that
  // makes three, within the four hardware queues HIP gives a process by
  // default; more streams share queues, and work queued behind another
  // stream's event wait stalls (measured: one extra 1.76 s, two 2.36 s, none
  // 1.90 s per paper-scale factorization)
  static constexpr int kFrontStreams = 1;
  hipStream_t fs[kFrontStreams] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kFrontStreams] = {};
  // the solve recorded once into a HIP graph per (b, x) pair and replayed
  // on the model's stream (its launch sequence is fixed for the object)
  hipStream_t gs = nullptr;
  hipGraphExec_t gexec = nullptr;
  const double* gb = nullptr;
  double* gx = nullptr;
  bool use_graph = true;
  bool stop_on_pivot = false;  // skip the rest of a factorization after its first static pivot
  // the library handle of the large trailing updates (NULL: every update on
  // k_update); atomics off, so its products are reproducible run to run
  rocblas_handle blas = nullptr;
  std::vector<void*> allocs;
  double flops = 0.0, flops_int = 0.0;
  int64_t factor_entries = 0, arena_entries = 0;
};

const opf_model* opf::chol_model(const opf_chol* F) { return F ? F->model : nullptr; }

namespace {

// bytes of update-matrix workspace per instance: 25 periods of the
// 10000-bus grid (measured per factorization with the chain eliminated from
// both ends and the chunks cut from both ends in turn: 12 periods 0.858 s,
// 25 0.793 s, 38 0.832 s, 51 0.862 s, 76 0.838 s, before the symmetric cut)
constexpr int64_t kArenaBudget = 16LL << 30;

// Workspace budget: OPF_CHOL_ARENA_BYTES (bytes, > 0) overrides the default.
int64_t arena_budget() {
  const char* e = std::getenv("OPF_CHOL_ARENA_BYTES");
  if (e && *e) {
    const long long v = std::atoll(e);
    if (v > 0) return (int64_t)v;
  }
  return kArenaBudget;
}

template <class T>
int upload(opf_chol* F, const std::vector<T>& h, T** d) {
  const size_t bytes = std::max<size_t>(1, h.size()) * sizeof(T);
  if (hipMalloc((void**)d, bytes) != hipSuccess) return api_fail(OPF_ENOMEM, "chol: device allocation failed");
  F->allocs.push_back(*d);
  if (!h.empty() && hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return api_fail(OPF_EHIP, "chol: upload failed");
  return OPF_OK;
}

int dalloc(opf_chol* F, int64_t n, double** d) {
  if (hipMalloc((void**)d, (size_t)std::max<int64_t>(1, n) * sizeof(double)) != hipSuccess)
    return api_fail(OPF_ENOMEM, "chol: device allocation of " + std::to_string(n * 8) + " bytes failed");
  F->allocs.push_back(*d);
  return OPF_OK;
}

void release(opf_chol* F) {
  for (void* p : F->allocs) (void)hipFree(p);
  F->allocs.clear();
}

#define CHK(x)                      \
  do {                              \
    int rc_ = (x);                  \
    if (rc_ != OPF_OK) return rc_;  \
  } while (0)

#define LAUNCH_OK(what)                                                                       \
  do {                                                                                        \
    hipError_t e_ = hipGetLastError();                                                        \
    if (e_ != hipSuccess) return api_fail(OPF_EHIP, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

int setup_device(opf_chol* F, CholInst& C) {
  const CholPlan& P = C.plan;
  std::vector<int64_t>& woff = C.woff;
  woff.assign(P.nnodes, 0);
  int64_t w = 0;
  for (int32_t s = 0; s < P.nnodes; ++s) {
    woff[s] = w;
    w += P.node_u[s];
  }
  C.wsize = std::max<int64_t>(w, 1);
  std::vector<int32_t> items = P.items;
  CHK(upload(F, P.node_f, &C.d_node_f));
  CHK(upload(F, P.node_p, &C.d_node_p));
  CHK(upload(F, P.node_u, &C.d_node_u));
  CHK(upload(F, P.rel, &C.d_rel));
  CHK(upload(F, P.kids, &C.d_kids));
  CHK(upload(F, P.rows, &C.d_rows));
  CHK(upload(F, P.perm, &C.d_perm));
  CHK(upload(F, items, &C.d_items));
  CHK(upload(F, P.lvl_small, &C.d_small));
  CHK(upload(F, P.roots, &C.d_roots));
  CHK(upload(F, P.kpos0, &C.d_kpos0));
  CHK(upload(F, P.kpos1, &C.d_kpos1));
  CHK(upload(F, P.ramp_pos, &C.d_ramp));
  CHK(upload(F, P.node_loff, &C.d_loff));
  CHK(upload(F, P.node_uoff, &C.d_uoff));
  CHK(upload(F, woff, &C.d_woff));
  CHK(upload(F, P.row_ptr, &C.d_rowptr));
  CHK(upload(F, P.kid_ptr, &C.d_kidptr));
  CHK(upload(F, P.slot_dst, &C.d_slot));
  const int64_t T = P.T, G = P.G;
  C.csize = 2 * G * G;
  C.chunk = (int32_t)std::max<int64_t>(1, std::min<int64_t>(T, arena_budget() / (P.usize * 8)));
  CHK(dalloc(F, P.lsize * T, &C.Lf));
  CHK(dalloc(F, C.csize * T, &C.Cf));
  CHK(dalloc(F, P.usize * C.chunk, &C.Ar));
  CHK(dalloc(F, C.wsize * T, &C.W));
  CHK(dalloc(F, G * T, &C.Wc));
  CHK(dalloc(F, (int64_t)P.n_p * T, &C.Y));
  CHK(dalloc(F, (int64_t)P.n_p * T, &C.Z));
  CHK(dalloc(F, (int64_t)((G + kChainCols - 1) / kChainCols) * G, &C.Gp));
  CDev& D = C.dev;
  D.node_f = C.d_node_f;
  D.node_p = C.d_node_p;
  D.node_u = C.d_node_u;
  D.rel = C.d_rel;
  D.kids = C.d_kids;
  D.rows = C.d_rows;
  D.node_loff = C.d_loff;
  D.node_uoff = C.d_uoff;
  D.node_woff = C.d_woff;
  D.row_ptr = C.d_rowptr;
  D.kid_ptr = C.d_kidptr;
  D.lsize = P.lsize;
  D.usize = P.usize;
  D.wsize = C.wsize;
  D.n_p = P.n_p;
  D.n_int = P.n_int;
  D.G = P.G;
  return OPF_OK;
}

// Blocked factorization of one front over nt periods: 128-column steps of
// two 64-column sub-panels (diagonal block, rows below; the first
// sub-panel's update of the second's columns in between), then one
// trailing update with the 128-wide panel.  Each update launch also factors
// the next diagonal block.
// The same update through the library's strided-batched GEMM, every call
// batched over the nt periods by their strides.  The lower part of the
// target columns is covered by column blocks of kBlasCols: block [j, j+w)
// takes rows [j, end) in one product, so it also writes the upper part of
// its w x w diagonal block (no kernel reads above the diagonal of a factor
// or update block).  The library's SYRK measured 2-12 TFLOP/s on these
// shapes against 40-70 for GEMM.  Columns in the factor block first, then
// those in the update block; the next diagonal block is factored by a
// launch of its own afterwards.
int blas_update(rocblas_handle h, const FrontArg& A, int nt, int k0, int kb, int r0, int cend, int dnext,
                double tol, double repl, int32_t* npert, hipStream_t st) {
  const int rows = A.p + A.u;
  const int64_t ld = A.ld;
  if (rocblas_set_stream(h, st) != rocblas_status_success) return api_fail(OPF_EHIP, "chol: rocblas_set_stream failed");
  const double* P = A.L + (int64_t)k0 * ld;  // panel: row r of column k0 + c at P[c * ld + r]
  // columns [c, c + n) of the target, rows [c, rows), at C (leading dimension ldc, period stride sc)
  auto lower = [&](int c, int n, double* C, int64_t ldc, int64_t sc) -> int {
    const double mone = -1.0, one = 1.0;
    for (int j = 0; j < n; j += kBlasCols) {
      const int w = std::min(kBlasCols, n - j);
      const double* Aj = P + c + j;
      if (rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, rows - c - j, w, kb,
                                        &mone, Aj, (rocblas_int)ld, A.Lstride, Aj, (rocblas_int)ld, A.Lstride, &one,
                                        C + (int64_t)j * ldc + j, (rocblas_int)ldc, sc, nt) != rocblas_status_success)
        return api_fail(OPF_EHIP, "chol: rocblas_dgemm_strided_batched failed");
    }
    return OPF_OK;
  };
  const int n1 = std::min(A.p, cend) - r0;  // target columns in the factor block
  if (n1 > 0) CHK(lower(r0, n1, A.L + (int64_t)r0 * ld + r0, ld, A.Lstride));
  const int c0 = std::max(r0, A.p);
  const int n3 = cend - c0;  // target columns in the update block
  if (n3 > 0) CHK(lower(c0, n3, A.U + (int64_t)(c0 - A.p) * A.ldU + (c0 - A.p), A.ldU, A.Ustride));
  if (dnext > 0) {
    hipLaunchKernelGGL(k_diag, dim3(nt), dim3(64), 0, st, A, r0, dnext, tol, repl, npert);
    LAUNCH_OK("chol diagonal block");
  }
  return OPF_OK;
}

int launch_update(const FrontArg& A, int nt, int k0, int kb, int r0, int cmax, int dnext, double tol, double repl,
                  int32_t* npert, hipStream_t st, rocblas_handle h) {
  const int rows = A.p + A.u;
  const int cend = std::min(cmax, rows);
  if (r0 >= rows || cend <= r0) {
    if (dnext > 0) {
      hipLaunchKernelGGL(k_diag, dim3(nt), dim3(64), 0, st, A, r0, dnext, tol, repl, npert);
      LAUNCH_OK("chol diagonal block");
    }
    return OPF_OK;
  }
  if (h && kb >= kBlasMinCols && rows - r0 >= kBlasMinRows)
    return blas_update(h, A, nt, k0, kb, r0, cend, dnext, tol, repl, npert, st);
  const int64_t R = (rows - r0 + kTile - 1) / kTile, Cn = (cend - r0 + kTile - 1) / kTile;
  const int64_t ntiles = Cn * R - Cn * (Cn - 1) / 2;
  if (ntiles > 0x7fffffff) return api_fail(OPF_EINVAL, "chol: front too large");
  hipLaunchKernelGGL(k_update, dim3((unsigned)ntiles, nt), dim3(256), 0, st, A, k0, kb, r0, cmax, dnext, tol, repl,
                     npert);
  LAUNCH_OK("chol update");
  return OPF_OK;
}

// Columns [k, k+w) of a front whose diagonal block [k, k+64) is factored
// already, w a power of two >= 64: recursively the first half, the first
// half's update of the second half's columns (which also factors the second
// half's first diagonal block), the second half.  The rows below the block
// get their share of the panel through the panel kernels; the trailing
// columns are left to the caller.
int factor_cols(const FrontArg& A, int nt, int k, int w, double tol, double repl, int32_t* npert, hipStream_t st,
                rocblas_handle bh) {
  const int rows = A.p + A.u;
  if (k >= A.p) return OPF_OK;
  if (w == 64) {
    const int kb = std::min(64, A.p - k);
    if (rows > k + kb) {
      hipLaunchKernelGGL(k_panel, dim3((rows - k - kb + 255) / 256, nt), dim3(256), 0, st, A, k, kb);
      LAUNCH_OK("chol panel");
    }
    return OPF_OK;
  }
  const int h = w / 2;
  CHK(factor_cols(A, nt, k, h, tol, repl, npert, st, bh));
  const int kh = std::min(h, A.p - k);
  const int k2 = std::min(h, A.p - k - kh);
  if (k2 > 0) {
    const int r1 = k + kh;
    CHK(launch_update(A, nt, k, kh, r1, r1 + k2, std::min(64, k2), tol, repl, npert, st, bh));
    CHK(factor_cols(A, nt, r1, h, tol, repl, npert, st, bh));
  }
  return OPF_OK;
}

int factor_front(const FrontArg& A, int nt, double tol, double repl, int32_t* npert, hipStream_t st,
                 rocblas_handle bh) {
  const int rows = A.p + A.u;
  hipLaunchKernelGGL(k_diag, dim3(nt), dim3(64), 0, st, A, 0, std::min(64, A.p), tol, repl, npert);
  LAUNCH_OK("chol diagonal block");
  // kStep-column steps, each factored recursively, then one trailing update
  // with the kStep-wide panel; every update launch also factors the next
  // diagonal block
  for (int k0 = 0; k0 < A.p; k0 += kStep) {
    CHK(factor_cols(A, nt, k0, kStep, tol, repl, npert, st, bh));
    const int kb = std::min(kStep, A.p - k0), r0 = k0 + kb;
    const int dnext = r0 < A.p ? std::min(64, A.p - r0) : 0;
    CHK(launch_update(A, nt, k0, kb, r0, rows, dnext, tol, repl, npert, st, bh));
  }
  return OPF_OK;
}

int factor_inst(opf_chol* F, CholInst& C, const double* kv, double tol, double repl, int32_t* npert,
                hipStream_t st) {
  const CholPlan& P = C.plan;
  const InstHost& I = *C.I;
  const int T = P.T, G = P.G;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(P.lsize * T, 256)), dim3(256), 0, st, C.Lf, P.lsize * T);
  hipLaunchKernelGGL(k_fill, dim3(grid_for(C.csize * T, 256)), dim3(256), 0, st, C.Cf, C.csize * T);
  LAUNCH_OK("chol fill");
  // every ramp pair up front: they land in the pg front of the period
  // before, which the chain stream may be factoring while a later chunk's
  // interior runs
  if (T > 1) {
    hipLaunchKernelGGL(k_scatter_ramp, dim3(grid_for(G, 256), T - 1), dim3(256), 0, st, kv, I.k_off, I.nnzk_p, G, 1,
                       (T - 1) / 2, C.d_ramp, C.Cf, C.csize);
    LAUNCH_OK("chol ramp scatter");
  }
  const int nslots = (int)P.slot_dst.size();
  // The pg chain from both ends: left fronts kl = 0 .. m-1, right fronts
  // kr = T-1 .. m+1, a left and a right front per step while both sides
  // have one ready, then front m.  The interior chunks are cut from both
  // ends of the horizon in turn (C.chunk periods each, the rest in the
  // middle last), so both sides of the chain become ready together and the
  // steps left after the last chunk are about half of that chunk.
  const int m = (T - 1) / 2;
  std::vector<std::pair<int, int>> chunks;  // (first period, periods)
  {
    int a = 0, b = T;
    bool left = true;
    while (b - a > C.chunk) {
      if (left) {
        chunks.push_back({a, C.chunk});
        a += C.chunk;
      } else {
        chunks.push_back({b - C.chunk, C.chunk});
        b -= C.chunk;
      }
      left = !left;
    }
    if (b > a) chunks.push_back({a, b - a});
  }
  const int nchunk = (int)chunks.size();
  if (nchunk + 1 > (int)F->evs.size()) return api_fail(OPF_EINVAL, "chol: more period chunks than events");
  std::vector<char> ready(T, 0);
  int kl = 0, kr = T - 1;
  double* UsL = F->Us;
  double* UsR = F->Us + (int64_t)G * G;
  const int64_t gg = (int64_t)G * G;
  // front t's incoming chain update (from t-1 on the left, t+1 on the
  // right) into its pivot block
  auto add_in = [&](int t, const double* Ub) -> int {
    hipLaunchKernelGGL(k_add_chain, dim3(grid_for(gg, 256)), dim3(256), 0, F->cs, Ub, G, C.Cf + (int64_t)t * C.csize);
    LAUNCH_OK("chol chain add");
    return OPF_OK;
  };
  auto clear = [&](double* Ub, int64_t n) -> int {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, F->cs, Ub, n);
    LAUNCH_OK("chol chain clear");
    return OPF_OK;
  };
  // nt = 2: fronts kl and kr in one batch (period stride kr - kl)
  auto chain_front = [&](int t, int nt, int t2, int u, double* Ub) -> int {
    FrontArg A;
    A.L = C.Cf + (int64_t)t * C.csize;
    A.Lstride = nt > 1 ? (int64_t)(t2 - t) * C.csize : 0;
    A.ld = 2 * G;
    A.p = G;
    A.u = u;
    A.U = Ub;
    A.Ustride = nt > 1 ? gg : 0;
    A.ldU = G;
    A.stop = C.dev.stop;
    return factor_front(A, nt, tol, repl, npert, F->cs, F->blas);
  };
  auto chain_steps = [&](bool all) -> int {
    for (;;) {
      const bool l = kl < m && ready[kl], r = kr > m && ready[kr];
      if (l && r) {
        if (kl >= 1) CHK(add_in(kl, UsL));
        if (kr <= T - 2) CHK(add_in(kr, UsR));
        CHK(clear(F->Us, 2 * gg));
        CHK(chain_front(kl, 2, kr, G, UsL));
        ++kl;
        --kr;
      } else if (l && (kr <= m || all)) {
        if (kl >= 1) CHK(add_in(kl, UsL));
        CHK(clear(UsL, gg));
        CHK(chain_front(kl, 1, kl, G, UsL));
        ++kl;
      } else if (r && (kl >= m || all)) {
        if (kr <= T - 2) CHK(add_in(kr, UsR));
        CHK(clear(UsR, gg));
        CHK(chain_front(kr, 1, kr, G, UsR));
        --kr;
      } else {
        break;
      }
    }
    return OPF_OK;
  };
  for (int chunk_id = 0; chunk_id < nchunk; ++chunk_id) {
    const int t0 = chunks[chunk_id].first;
    const int nt = chunks[chunk_id].second;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(nslots, 256), nt), dim3(256), 0, st, kv, I.k_off, I.nnzk_p, G, t0,
                       nslots, C.d_slot, C.d_kpos0, C.d_kpos1, C.Lf, P.lsize, C.Cf, C.csize);
    LAUNCH_OK("chol scatter");
    for (int h = 0; h < P.nlevels; ++h) {
      const int64_t i0 = P.lvl_items_ptr[h], i1 = P.lvl_items_ptr[h + 1];
      if (i1 > i0) {
        hipLaunchKernelGGL(k_extend, dim3((unsigned)(i1 - i0), nt), dim3(256), 0, st, C.dev, C.d_items, i0,
                           CholOptions().col_block, t0, C.Lf, C.Ar);
        LAUNCH_OK("chol extend-add");
      }
      const int64_t s0 = P.lvl_small_ptr[h], s1 = P.lvl_small_ptr[h + 1];
      if (s1 > s0) {
        hipLaunchKernelGGL(k_factor_small, dim3((unsigned)(s1 - s0), nt), dim3(64), 0, st, C.dev, C.d_small, s0, t0,
                           C.Lf, C.Ar, tol, repl, npert);
        LAUNCH_OK("chol small fronts");
      }
      const int64_t q0 = P.lvl_large_ptr[h], q1 = P.lvl_large_ptr[h + 1];
      const int nfs = (int)std::min<int64_t>(opf_chol::kFrontStreams, q1 - q0 - 1);
      if (nfs > 0) {
        if (hipEventRecord(F->fork_ev, st) != hipSuccess) return api_fail(OPF_EHIP, "chol: front stream fork");
        for (int k = 0; k < nfs; ++k)
          if (hipStreamWaitEvent(F->fs[k], F->fork_ev, 0) != hipSuccess)
            return api_fail(OPF_EHIP, "chol: front stream fork");
      }
      for (int64_t q = q0; q < q1; ++q) {
        const int s = P.lvl_large[q];
        const int64_t slot = (q - q0) % (nfs + 1);
        hipStream_t fst = slot == 0 ? st : F->fs[slot - 1];
        FrontArg A;
        A.L = C.Lf + (int64_t)t0 * P.lsize + P.node_loff[s];
        A.Lstride = P.lsize;
        A.ld = P.node_p[s] + P.node_u[s];
        A.p = P.node_p[s];
        A.u = P.node_u[s];
        A.U = C.Ar + P.node_uoff[s];
        A.Ustride = P.usize;
        A.ldU = std::max(1, P.node_u[s]);
        A.stop = C.dev.stop;
        CHK(factor_front(A, nt, tol, repl, npert, fst, nullptr));
      }
      for (int k = 0; k < nfs; ++k)
        if (hipEventRecord(F->join_ev[k], F->fs[k]) != hipSuccess ||
            hipStreamWaitEvent(st, F->join_ev[k], 0) != hipSuccess)
          return api_fail(OPF_EHIP, "chol: front stream join");
    }
    const int cb = CholOptions().col_block;
    hipLaunchKernelGGL(k_extend_root, dim3((G + cb - 1) / cb, nt), dim3(256), 0, st, C.dev, C.d_roots,
                       (int32_t)P.roots.size(), cb, t0, C.Cf, C.csize, C.Ar);
    LAUNCH_OK("chol pg front assembly");
    // the chain steps this chunk makes ready, on the chain stream
    if (hipEventRecord(F->evs[chunk_id], st) != hipSuccess || hipStreamWaitEvent(F->cs, F->evs[chunk_id], 0) != hipSuccess)
      return api_fail(OPF_EHIP, "chol: chain stream ordering");
    for (int t = t0; t < t0 + nt; ++t) ready[t] = 1;
    CHK(chain_steps(chunk_id + 1 == nchunk));
  }
  // front m: both sides' last updates, no update rows
  if (m >= 1) CHK(add_in(m, UsL));
  if (m + 1 <= T - 1) CHK(add_in(m, UsR));
  CHK(chain_front(m, 1, m, 0, UsL));
  // the model's stream waits for the chain
  hipEvent_t done = F->evs.back();
  if (hipEventRecord(done, F->cs) != hipSuccess || hipStreamWaitEvent(st, done, 0) != hipSuccess)
    return api_fail(OPF_EHIP, "chol: chain stream join");
  return OPF_OK;
}

// Forward / backward triangle of one front's pivot block by panels (see
// k_fwd_panel / k_bwd_panel): y is the right-hand side in, z the forward
// solution; the backward pass reads z and leaves x in y.
int fwd_tri(const double* L, int64_t Ls, int ld, int p, double* y, double* z, int64_t ys, int nper,
            hipStream_t st) {
  for (int k0 = 0; k0 < p; k0 += 64) {
    const int below = p - k0 - std::min(64, p - k0);
    hipLaunchKernelGGL(k_fwd_panel, dim3(std::max(1, (below + 255) / 256), nper), dim3(256), 0, st, L, Ls, ld, p,
                       k0, y, z, ys);
  }
  LAUNCH_OK("chol forward triangle");
  return OPF_OK;
}

int bwd_tri(const double* L, int64_t Ls, int ld, int p, double* y, double* z, int64_t ys, int nper,
            hipStream_t st) {
  for (int k0 = ((p - 1) / 64) * 64; k0 >= 0; k0 -= 64)
    hipLaunchKernelGGL(k_bwd_panel, dim3(std::max(1, (k0 + kBwdCols - 1) / kBwdCols), nper), dim3(256), 0, st, L,
                       Ls, ld, p, k0, y, z, ys);
  LAUNCH_OK("chol backward triangle");
  return OPF_OK;
}

int solve_inst(CholInst& C, const double* b, double* x, hipStream_t st) {
  const CholPlan& P = C.plan;
  const InstHost& I = *C.I;
  const int T = P.T, G = P.G;
  const int64_t np = P.n_p;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(np * T, 256)), dim3(256), 0, st, b + I.x_off, P.n_p, T, C.d_perm, C.Y);
  LAUNCH_OK("chol gather");
  // forward through the interior trees, all periods at once (small fronts
  // leave their forward solution in Y, large ones in Z)
  for (int h = 0; h < P.nlevels; ++h) {
    const int64_t s0 = P.lvl_small_ptr[h], s1 = P.lvl_small_ptr[h + 1];
    if (s1 > s0) {
      hipLaunchKernelGGL(k_fwd_small, dim3((unsigned)(s1 - s0), T), dim3(64), 0, st, C.dev, C.d_small, s0, C.Lf,
                         C.Y, C.W);
      LAUNCH_OK("chol forward small");
    }
    for (int64_t q = P.lvl_large_ptr[h]; q < P.lvl_large_ptr[h + 1]; ++q) {
      const int s = P.lvl_large[q];
      const int p = P.node_p[s], u = P.node_u[s], fs = P.node_f[s];
      const double* L = C.Lf + P.node_loff[s];
      hipLaunchKernelGGL(k_fwd_pull, dim3(T), dim3(256), 0, st, C.dev, s, C.Y, C.W);
      CHK(fwd_tri(L, P.lsize, p + u, p, C.Y + fs, C.Z + fs, np, T, st));
      if (u > 0)
        hipLaunchKernelGGL(k_fwd_gemv, dim3((u + 255) / 256, T), dim3(256), 0, st, L, P.lsize, p + u, p, u,
                           (const double*)(C.Z + fs), np, C.W + C.woff[s], C.wsize, 1);
      LAUNCH_OK("chol forward large");
    }
  }
  hipLaunchKernelGGL(k_fwd_root_pull, dim3(T), dim3(256), 0, st, C.dev, C.d_roots, (int32_t)P.roots.size(), C.Y,
                     (const double*)C.W);
  LAUNCH_OK("chol forward roots");
  // forward along the pg chain, from both ends as it was factored: left
  // fronts ascending, right fronts descending, a left and a right front per
  // step while both sides have one, then front m
  const int m = (T - 1) / 2;
  auto off = [&](int t) { return (int64_t)t * np + P.n_int; };
  auto front = [&](int t) { return (const double*)(C.Cf + (int64_t)t * C.csize); };
  // y_t -= L21_s z_s of its chain neighbour s (held in Wc[s])
  auto pull = [&](int t, int s) -> int {
    hipLaunchKernelGGL(k_sub, dim3((G + 255) / 256), dim3(256), 0, st, C.Y + off(t),
                       (const double*)(C.Wc + (int64_t)s * G), G);
    LAUNCH_OK("chol forward chain");
    return OPF_OK;
  };
  // Wc[t] = L21_t z_t
  auto push = [&](int t) -> int {
    const int nch = (G + kChainCols - 1) / kChainCols;
    hipLaunchKernelGGL(k_gemv_part, dim3((G + 255) / 256, nch), dim3(256), 0, st, front(t), 2 * G, G, G,
                       (const double*)(C.Z + off(t)), kChainCols, C.Gp);
    hipLaunchKernelGGL(k_gemv_sum, dim3((G + 255) / 256), dim3(256), 0, st, (const double*)C.Gp, nch, G,
                       C.Wc + (int64_t)t * G);
    LAUNCH_OK("chol forward chain");
    return OPF_OK;
  };
  {
    int kl = 0, kr = T - 1;
    while (kl < m || kr > m) {
      const bool l = kl < m, r = kr > m;
      if (l && kl >= 1) CHK(pull(kl, kl - 1));
      if (r && kr <= T - 2) CHK(pull(kr, kr + 1));
      if (l && r)
        CHK(fwd_tri(front(kl), (int64_t)(kr - kl) * C.csize, 2 * G, G, C.Y + off(kl), C.Z + off(kl),
                    (int64_t)(kr - kl) * np, 2, st));
      else
        CHK(fwd_tri(front(l ? kl : kr), 0, 2 * G, G, C.Y + off(l ? kl : kr), C.Z + off(l ? kl : kr), 0, 1, st));
      if (l) CHK(push(kl));
      if (r) CHK(push(kr));
      if (l) ++kl;
      if (r) --kr;
    }
    if (m >= 1) CHK(pull(m, m - 1));
    if (m + 1 <= T - 1) CHK(pull(m, m + 1));
    CHK(fwd_tri(front(m), 0, 2 * G, G, C.Y + off(m), C.Z + off(m), 0, 1, st));
  }
  // backward along the pg chain: front m, then outwards (each front reads
  // its chain neighbour's solution, held in Y)
  {
    CHK(bwd_tri(front(m), 0, 2 * G, G, C.Y + off(m), C.Z + off(m), 0, 1, st));
    int kl = m - 1, kr = m + 1;
    while (kl >= 0 || kr <= T - 1) {
      const bool l = kl >= 0, r = kr <= T - 1;
      if (l)
        hipLaunchKernelGGL(k_bwd_gemv, dim3((G + 3) / 4, 1), dim3(256), 0, st, front(kl), (int64_t)0, 2 * G, G, G,
                           (const int32_t*)nullptr, (const double*)(C.Y + off(kl + 1)), (int64_t)0, C.Z + off(kl),
                           (int64_t)0);
      if (r)
        hipLaunchKernelGGL(k_bwd_gemv, dim3((G + 3) / 4, 1), dim3(256), 0, st, front(kr), (int64_t)0, 2 * G, G, G,
                           (const int32_t*)nullptr, (const double*)(C.Y + off(kr - 1)), (int64_t)0, C.Z + off(kr),
                           (int64_t)0);
      LAUNCH_OK("chol backward chain");
      if (l && r)
        CHK(bwd_tri(front(kl), (int64_t)(kr - kl) * C.csize, 2 * G, G, C.Y + off(kl), C.Z + off(kl),
                    (int64_t)(kr - kl) * np, 2, st));
      else
        CHK(bwd_tri(front(l ? kl : kr), 0, 2 * G, G, C.Y + off(l ? kl : kr), C.Z + off(l ? kl : kr), 0, 1, st));
      if (l) --kl;
      if (r) ++kr;
    }
  }
  // backward through the interior trees, top down
  for (int h = P.nlevels - 1; h >= 0; --h) {
    for (int64_t q = P.lvl_large_ptr[h]; q < P.lvl_large_ptr[h + 1]; ++q) {
      const int s = P.lvl_large[q];
      const int p = P.node_p[s], u = P.node_u[s], fs = P.node_f[s];
      const double* L = C.Lf + P.node_loff[s];
      if (u > 0)
        hipLaunchKernelGGL(k_bwd_gemv, dim3((p + 3) / 4, T), dim3(256), 0, st, L, P.lsize, p + u, p, u,
                           (const int32_t*)(C.d_rows + P.row_ptr[s]), (const double*)C.Y, np, C.Z + fs, np);
      CHK(bwd_tri(L, P.lsize, p + u, p, C.Y + fs, C.Z + fs, np, T, st));
      LAUNCH_OK("chol backward large");
    }
    const int64_t s0 = P.lvl_small_ptr[h], s1 = P.lvl_small_ptr[h + 1];
    if (s1 > s0) {
      hipLaunchKernelGGL(k_bwd_small, dim3((unsigned)(s1 - s0), T), dim3(64), 0, st, C.dev, C.d_small, s0, C.Lf,
                         C.Y);
      LAUNCH_OK("chol backward small");
    }
  }
  hipLaunchKernelGGL(k_scatter_out, dim3(grid_for(np * T, 256)), dim3(256), 0, st, (const double*)C.Y, P.n_p, T,
                     C.d_perm, x + I.x_off);
  LAUNCH_OK("chol scatter");
  return OPF_OK;
}

}  // namespace

// ============================================================== C ABI
extern "C" {

int opf_chol_analyze(opf_model* model, opf_chol** out) {
  if (!out) return api_fail(OPF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!model) return api_fail(OPF_EINVAL, "model is NULL");
  opf_chol* F = nullptr;
  try {
    F = new opf_chol();
    F->model = model;
    F->device = model_device(model);
    const auto& insts = model_insts(model);
    F->inst.resize(insts.size());
    CholOptions opt;
    int32_t maxG = 0;
    for (size_t k = 0; k < insts.size(); ++k) {
      CholInst& C = F->inst[k];
      C.I = &insts[k];
      std::string err;
      const int rc = chol_plan_build(insts[k], opt, C.plan, err);
      if (rc != OPF_OK) {
        delete F;
        return api_fail(rc, "instance " + std::to_string(k) + ": " + err);
      }
      const CholPlan& P = C.plan;
      C.nlarge = (int32_t)P.lvl_large.size();
      maxG = std::max(maxG, P.G);
      F->flops += P.flops_period * P.T + P.flops_chain;
      F->flops_int += P.flops_period * P.T;
      F->factor_entries += P.lsize * P.T + 2LL * P.G * P.G * P.T;
    }
    if (F->device >= 0) {
      if (hipSetDevice(F->device) != hipSuccess) {
        delete F;
        return api_fail(OPF_EHIP, "chol: hipSetDevice failed");
      }
      for (auto& C : F->inst) {
        const int rc = setup_device(F, C);
        if (rc != OPF_OK) {
          release(F);
          delete F;
          return rc;
        }
        F->arena_entries += C.plan.usize * C.chunk;
      }
      const int rc = dalloc(F, 2 * (int64_t)maxG * maxG, &F->Us);
      if (rc != OPF_OK) {
        release(F);
        delete F;
        return rc;
      }
      // default priority, no implicit ordering with the null stream
      int nev = 1;
      for (auto& C : F->inst) nev = std::max(nev, (C.plan.T + C.chunk - 1) / C.chunk + 1);
      bool ok = hipStreamCreateWithFlags(&F->cs, hipStreamNonBlocking) == hipSuccess &&
                hipStreamCreateWithFlags(&F->gs, hipStreamNonBlocking) == hipSuccess &&
                hipEventCreateWithFlags(&F->fork_ev, hipEventDisableTiming) == hipSuccess;
      for (int k = 0; ok && k < opf_chol::kFrontStreams; ++k)
        ok = hipStreamCreateWithFlags(&F->fs[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&F->join_ev[k], hipEventDisableTiming) == hipSuccess;
      for (int k = 0; ok && k < nev; ++k) {
        hipEvent_t e = nullptr;
        ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (ok) F->evs.push_back(e);
      }
      if (!ok) {
        opf_chol_destroy(F);
        return api_fail(OPF_EHIP, "chol: stream or event creation failed");
      }
      // OPF_CHOL_BLAS=0 keeps every trailing update on k_update
      const char* eb = std::getenv("OPF_CHOL_BLAS");
      if (!(eb && eb[0] == '0')) {
        if (rocblas_create_handle(&F->blas) != rocblas_status_success ||
            rocblas_set_atomics_mode(F->blas, rocblas_atomics_not_allowed) != rocblas_status_success ||
            rocblas_set_pointer_mode(F->blas, rocblas_pointer_mode_host) != rocblas_status_success) {
          opf_chol_destroy(F);
          return api_fail(OPF_EHIP, "chol: rocBLAS handle creation failed");
        }
      }
    } else {
      for (auto& C : F->inst) {
        C.chunk = (int32_t)std::max<int64_t>(1, std::min<int64_t>(C.plan.T, arena_budget() / (C.plan.usize * 8)));
        F->arena_entries += C.plan.usize * C.chunk;
      }
    }
  } catch (const std::bad_alloc&) {
    if (F) {
      release(F);
      delete F;
    }
    return api_fail(OPF_ENOMEM, "chol: host allocation failed");
  }
  *out = F;
  return OPF_OK;
}

void opf_chol_destroy(opf_chol* chol) {
  if (!chol) return;
  if (chol->device >= 0) (void)hipSetDevice(chol->device);
  if (chol->cs) (void)hipStreamSynchronize(chol->cs);
  if (chol->device >= 0) (void)hipDeviceSynchronize();
  if (chol->gexec) (void)hipGraphExecDestroy(chol->gexec);
  for (hipEvent_t e : chol->evs) (void)hipEventDestroy(e);
  if (chol->fork_ev) (void)hipEventDestroy(chol->fork_ev);
  for (int k = 0; k < opf_chol::kFrontStreams; ++k) {
    if (chol->join_ev[k]) (void)hipEventDestroy(chol->join_ev[k]);
    if (chol->fs[k]) (void)hipStreamDestroy(chol->fs[k]);
  }
  if (chol->blas) (void)rocblas_destroy_handle(chol->blas);
  if (chol->cs) (void)hipStreamDestroy(chol->cs);
  if (chol->gs) (void)hipStreamDestroy(chol->gs);
  release(chol);
  delete chol;
}

int opf_chol_get_info(const opf_chol* F, opf_chol_info* info) {
  if (!F || !info) return api_fail(OPF_EINVAL, "chol or info is NULL");
  std::memset(info, 0, sizeof(*info));
  info->factor_entries = F->factor_entries;
  info->arena_entries = F->arena_entries;
  info->flops = F->flops;
  info->flops_interior = F->flops_int;
  info->chunk = F->inst.empty() ? 0 : 0x7fffffff;
  for (const auto& C : F->inst) {
    info->nodes += C.plan.nnodes;
    info->levels = std::max(info->levels, C.plan.nlevels);
    info->chunk = std::min(info->chunk, C.chunk);
    info->large_nodes += (int32_t)C.plan.lvl_large.size();
  }
  return OPF_OK;
}

int opf_chol_tree_size(const opf_chol* F, int32_t inst, int32_t* nodes, int64_t* rows) {
  if (!F || !nodes || !rows) return api_fail(OPF_EINVAL, "NULL argument");
  if (inst < 0 || inst >= (int32_t)F->inst.size()) return api_fail(OPF_EINVAL, "instance out of range");
  *nodes = F->inst[inst].plan.nnodes;
  *rows = (int64_t)F->inst[inst].plan.rows.size();
  return OPF_OK;
}

int opf_chol_tree(const opf_chol* F, int32_t inst, int32_t* perm, int32_t* first, int32_t* npiv, int32_t* parent,
                  int64_t* rowptr, int32_t* rows) {
  if (!F || !perm || !first || !npiv || !parent || !rowptr || !rows) return api_fail(OPF_EINVAL, "NULL argument");
  if (inst < 0 || inst >= (int32_t)F->inst.size()) return api_fail(OPF_EINVAL, "instance out of range");
  const CholPlan& P = F->inst[inst].plan;
  std::copy(P.perm.begin(), P.perm.end(), perm);
  std::copy(P.node_f.begin(), P.node_f.end(), first);
  std::copy(P.node_p.begin(), P.node_p.end(), npiv);
  std::copy(P.node_parent.begin(), P.node_parent.end(), parent);
  std::copy(P.row_ptr.begin(), P.row_ptr.end(), rowptr);
  std::copy(P.rows.begin(), P.rows.end(), rows);
  return OPF_OK;
}

int opf_chol_factor(opf_chol* F, const double* kvals, double pivot_tol, double pivot_repl, int32_t* npert) {
  if (!F || !kvals || !npert) return api_fail(OPF_EINVAL, "chol, kvals or npert is NULL");
  if (F->device < 0) return api_fail(OPF_ENODEV, "model is host-only");
  if (!(pivot_repl > 0.0) || !std::isfinite(pivot_repl)) return api_fail(OPF_EINVAL, "pivot_repl must be > 0");
  if (std::isnan(pivot_tol)) return api_fail(OPF_EINVAL, "pivot_tol is NaN");
  if (hipSetDevice(F->device) != hipSuccess) return api_fail(OPF_EHIP, "hipSetDevice failed");
  hipStream_t st = model_stream(F->model);
  if (hipMemsetAsync(npert, 0, sizeof(int32_t), st) != hipSuccess) return api_fail(OPF_EHIP, "clearing npert");
  for (auto& C : F->inst) {
    C.dev.stop = F->stop_on_pivot ? npert : nullptr;
    CHK(factor_inst(F, C, kvals, pivot_tol, pivot_repl, npert, st));
  }
  return OPF_OK;
}

int opf_chol_solve(opf_chol* F, const double* b, double* x) {
  if (!F || !b || !x) return api_fail(OPF_EINVAL, "chol, b or x is NULL");
  if (F->device < 0) return api_fail(OPF_ENODEV, "model is host-only");
  if (hipSetDevice(F->device) != hipSuccess) return api_fail(OPF_EHIP, "hipSetDevice failed");
  hipStream_t st = model_stream(F->model);
  if (!F->use_graph) {
    for (auto& C : F->inst) CHK(solve_inst(C, b, x, st));
    return OPF_OK;
  }
  if (!F->gexec || F->gb != b || F->gx != x) {
    if (F->gexec) {
      (void)hipStreamSynchronize(st);
      (void)hipGraphExecDestroy(F->gexec);
      F->gexec = nullptr;
    }
    if (hipStreamBeginCapture(F->gs, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return api_fail(OPF_EHIP, "chol: solve capture");
    int rc = OPF_OK;
    for (auto& C : F->inst)
      if (rc == OPF_OK) rc = solve_inst(C, b, x, F->gs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(F->gs, &g);
    if (rc != OPF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess || !g) return api_fail(OPF_EHIP, "chol: solve capture end");
    const hipError_t ei = hipGraphInstantiate(&F->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      F->gexec = nullptr;
      return api_fail(OPF_EHIP, std::string("chol: solve graph: ") + hipGetErrorString(ei));
    }
    F->gb = b;
    F->gx = x;
  }
  if (hipGraphLaunch(F->gexec, st) != hipSuccess) return api_fail(OPF_EHIP, "chol: solve graph launch");
  return OPF_OK;
}

int opf_chol_set_stop_on_pivot(opf_chol* F, int enable) {
  if (!F) return api_fail(OPF_EINVAL, "chol is NULL");
  F->stop_on_pivot = enable != 0;
  return OPF_OK;
}

int opf_chol_stop_on_pivot(const opf_chol* F) { return F && F->stop_on_pivot ? 1 : 0; }

int opf_chol_set_graph(opf_chol* F, int enable) {
  if (!F) return api_fail(OPF_EINVAL, "chol is NULL");
  F->use_graph = enable != 0;
  return OPF_OK;
}

}  // extern "C"
