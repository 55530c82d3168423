// Device-visible instance descriptor, tile list entries and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace opf {

// One instance as the kernels see it: sizes, concatenation offsets and
// device pointers into the model's arena.  Lives in device memory (an array
// over instances) and is read with uniform loads.
struct InstDev {
  int32_t N, B, G, T, ref, pad;
  int64_t n_p, m_p, nnzj_p, nnzh_p, nnzk_p;
  int64_t x_off, c_off, j_off, h_off, k_off, ld_off, s_off, o_off;
  const int32_t *f_bus, *t_bus, *gen_bus;
  const double* adm;  // [8][B]: Gff Bff Gft Bft Gtf Btf Gtt Btt
  const double *c2, *c1, *c0;
  double *pd, *qd;  // [T][N]
  const int32_t *bus_ptr, *bus_adj, *bus_nb, *bgen_ptr, *bgen;
  const int32_t *krow, *kcol, *ksrc, *kinfo;
  const double *vmin, *vmax, *pmin, *pmax, *qmin, *qmax, *ramp, *rate, *angmin, *angmax;
};

// Element classes a tile can cover.
enum TileKind : int32_t {
  TK_BRANCH = 0,  // lines
  TK_GEN = 1,     // generators
  TK_BUS = 2,     // buses
  TK_VAR = 3,     // local variable slots of a period block
  TK_CON = 4,     // local constraint rows of a period block
  TK_KROW = 5     // local rows of the condensed-matrix template
};

// A tile: elements [e0, e1) of one kind of one instance over periods
// [t0, t1).  Thread threadIdx.x owns element e0 + threadIdx.x and walks the
// periods; e1 - e0 <= blockDim.x.
struct Tile {
  int32_t inst, kind, e0, e1, t0, t1;
};

// Start of period t's block of K inside one instance (device twin of the
// host helper in opf_host.h): periods t >= 1 carry G extra ramp-pair slots.
__device__ __forceinline__ int64_t kkt_period_offset_dev(int64_t nnzk_p, int32_t G, int32_t t) {
  return (int64_t)t * nnzk_p + (t >= 1 ? (int64_t)(t - 1) * G : 0);
}

// Buffer-resource access: a wave-uniform 128-bit descriptor (base address,
// unlimited extent) in scalar registers plus a 32-bit per-lane byte offset,
// the addressing form of the vector memory unit that needs no 64-bit
// per-lane address.  Used by the kernels that touch many arrays per element
// (each array block gets its own descriptor; offsets stay below 4 GiB
// because every such block is a per-period or per-instance slice).
using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ rsrc_t rsrc(const void* base) {
  // word 3 of the descriptor for raw (untyped) access on gfx9-family parts
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, -1, 0x00020000);
}
__device__ __forceinline__ double bld(rsrc_t r, uint32_t e) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8u, 0, 0));
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t e, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, e * 8u, 0, 0);
}
__device__ __forceinline__ int32_t bldi(rsrc_t r, uint32_t e) {
  return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, e * 4u, 0, 0);
}
// Split addressing: a per-lane byte offset (vo, shared by many accesses)
// plus a wave-uniform byte offset (so, in the instruction's scalar-offset
// operand), so a lane keeps a handful of offsets instead of one per stream.
__device__ __forceinline__ double bldv(rsrc_t r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
__device__ __forceinline__ void bstv(rsrc_t r, uint32_t vo, uint32_t so, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, vo, so, 0);
}
// Non-temporal variants (cache policy nt): output streams that no later
// step of the same kernel reads back.
__device__ __forceinline__ void bstvn(rsrc_t r, uint32_t vo, uint32_t so, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, vo, so, 2);
}
__device__ __forceinline__ void bstn(rsrc_t r, uint32_t e, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, e * 8u, 0, 2);
}
__device__ __forceinline__ int32_t bldiv(rsrc_t r, uint32_t vo, uint32_t so) {
  return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
}
__device__ __forceinline__ void bst2v(rsrc_t r, uint32_t vo, uint32_t so, double2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, vo, so, 0);
}
__device__ __forceinline__ double2 bld2v(rsrc_t r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
}
// Loads that miss in the CU's L1 and are served by the L2 (cache policy
// sc0): data another CU of the same XCD wrote earlier in the same launch.
__device__ __forceinline__ double2 bld2v_l2(rsrc_t r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 1));
}
__device__ __forceinline__ double bld_l2(rsrc_t r, uint32_t e) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8u, 0, 1));
}

// Per-instance scratch, in doubles, per line and period:
//  * a line -> bus hand-off record per line end (kRecEnd doubles, one
//    64-byte line): [0] the end's (vm,vm) diagonal sum, [1] its (va,vm)
//    pair, [2] (va,va) diagonal, [3] (va_end, vm_other) cross pair, [4] p and
//    [5] q of the flow leaving the bus through this end, [6] J^T v on vm,
//    [7] J^T v on va of the end's bus; records are [t][line][end][8];
//  * the line's (vm_i,vm_j) and (va_i,va_j) cross sums, [t][line][2], read
//    by the higher-numbered end (it owns those slots);
//  * the 4-value hand-off of the separate J^T v kernels, [t][line][4].
constexpr int kRecEnd = 8;
constexpr int kRecLine = 2 * kRecEnd;
constexpr int kShared = 2;
constexpr int kScratchJt = 4;
constexpr int kScratchPerLine = kRecLine + kShared + kScratchJt;
// LDS stride (doubles) of one line's two records when a line tile stages
// them (padded by one to spread the lanes over the LDS banks).
constexpr int kRecLds = kRecLine + 1;

__device__ __forceinline__ double* rec_at(const InstDev& I, double* scr, int t) {
  return scr + I.s_off + (int64_t)t * I.B * kRecLine;
}
__device__ __forceinline__ double* shared_at(const InstDev& I, double* scr, int t) {
  return scr + I.s_off + (int64_t)kRecLine * I.B * I.T + (int64_t)t * I.B * kShared;
}
__device__ __forceinline__ double* jt_at(const InstDev& I, double* scr, int t) {
  return scr + I.s_off + (int64_t)(kRecLine + kShared) * I.B * I.T + (int64_t)t * I.B * kScratchJt;
}
// Objective partials of the whole sweep, [t][64-generator chunk]: the slot of
// the generator tile starting at period t (only tile starts are written).
__device__ __forceinline__ int64_t obj_part_at(const InstDev& I, int t, int chunk) {
  return I.o_off + (int64_t)t * ((I.G + 63) >> 6) + chunk;
}

// Kernel launchers (opf_kernels.hip).  Each takes the device instance
// array, a device tile list and a launch shape; returns the HIP error of the
// launch.
struct Launch {
  const InstDev* insts;
  const Tile* tiles;
  int ntiles;
  int block;
  int grid;
  hipStream_t stream;
  int cap0 = 0;     // LDS segment capacity (doubles) of the staged kernels
  size_t smem = 0;  // dynamic LDS bytes
};

hipError_t launch_jac(const Launch& L, const double* x, double* jv);
hipError_t launch_hess(const Launch& L, const double* x, const double* lam, double sigma, double* hv);
hipError_t launch_cons(const Launch& L, const double* x, double* c);
hipError_t launch_grad(const Launch& L, const double* x, double* g);
hipError_t launch_obj_partial(const Launch& L, const double* x, double* partial, int32_t* zero, int nzero);
hipError_t launch_obj_final(const int32_t* inst_tile_begin, int ninst, const double* partial, double* f,
                            hipStream_t s);
hipError_t launch_jt_a(const Launch& L, const double* x, const double* v, double* out, double* scratch);
hipError_t launch_jt_b(const Launch& L, const double* v, double* out, const double* scratch);
hipError_t launch_kkt_a(const Launch& L, const double* h, const double* j, const double* dx, const double* d,
                        double* k, double* scratch);
hipError_t launch_jhk_a(const Launch& L, const double* x, const double* lam, double sigma, double* h, double* j,
                        const double* dx, const double* d, double* k, double* scratch);
// The objective carried by the two sweep kernels instead of two launches of
// its own: each wavefront of a generator tile of the line pass leaves the
// sum of its 64 generators' cost terms over the tile's periods in the
// instance's partial block of the scratch (obj_part_at), and the bus pass's
// first blocks sum instance k's partials into f[k] in a fixed order.  ppt:
// the line pass's periods per tile (its generator tiles start at multiples
// of ppt and at multiples of 64 generators).  f null: no objective.
struct ObjFold {
  int ninst = 0;
  int ppt = 0;
  double* f = nullptr;
};
hipError_t launch_sweep_a(const Launch& L, const double* x, const double* lam, double sigma, const double* v,
                          double* h, double* j, const double* dx, const double* d, double* k, double* c, double* jtv,
                          double* g, double* scratch);
hipError_t launch_sweep_b(const Launch& L, const double* x, const double* v, const double* j, const double* dx,
                          const double* d, double* k, double* c, double* jtv, double* g, const double* scratch,
                          const ObjFold& of);
hipError_t launch_kkt_b(const Launch& L, const double* j, const double* dx, const double* d, double* k,
                        const double* scratch);
// One iterate of the lifted interior-point method (device pointers over the
// concatenated instances; +-inf bounds are absent).
struct IpmDev {
  const double *x, *s, *y, *zl, *zu, *vl, *vu, *xl, *xu, *sl, *su;
  double mu, dw, dc;
};

// Flat element-wise launch over [0, count).
struct Flat {
  int64_t count;
  hipStream_t stream;
};

// One tile of the one-launch sweep.  slot: the counter of its group (an
// instance and a run of periods); a line or generator tile adds one to it
// when done, a bus tile (need > 0) first waits until it reaches need.
struct SweepItem {
  Tile tl;
  int32_t slot;
  int32_t need;
};

// Launch data of the one-launch sweep (k_sweep): per-XCD queues of items
// [qbeg[q], qbeg[q+1]), the counters (zeroed before the launch: ticket and
// finished tiles of queue q at 32 q and 32 q + 1, then the group slots),
// status flags.
struct FusedSweep {
  const InstDev* insts;
  const SweepItem* items;
  const int32_t* qbeg;
  int nq;
  int32_t* ctr;
  int32_t* flags;
  int cap_seg, cap_vm, cap_va;
  size_t smem;
  int grid;
  int block;  // elements per tile = threads per block (<= 256)
  hipStream_t stream;
};
int sweep_fused_blocks_per_cu(int block, size_t smem);
hipError_t launch_sweep_fused(const FusedSweep& F, const double* x, const double* lam, double sigma,
                              const double* v, double* h, double* j, const double* dx, const double* d, double* k,
                              double* c, double* jtv, double* g, double* scratch);
hipError_t launch_sweep_open(int32_t* ctr, int n, hipStream_t s);
hipError_t launch_sweep_close(const int32_t* begin, int ninst, const double* partial, double* f,
                              const int32_t* ctr, const int32_t* qbeg, int nq, int32_t* flags, hipStream_t s);

hipError_t launch_jv(const Launch& L, const double* x, const double* v, double* jv);
hipError_t launch_rhs_rows(const Flat& F, const IpmDev& st, const double* c, double* dcon, double* w);
hipError_t launch_rhs_vars(const Flat& F, const IpmDev& st, const double* grad, double* diag_x, double* rhs);
hipError_t launch_rec_rows(const Flat& F, const IpmDev& st, const double* c, const double* adx, double* ds,
                           double* dy, double* dvl, double* dvu);
hipError_t launch_rec_vars(const Flat& F, const IpmDev& st, const double* dx, double* dzl, double* dzu);
hipError_t launch_jac_struct(const Launch& L, int32_t* rows, int32_t* cols);
hipError_t launch_hess_struct(const Launch& L, int32_t* rows, int32_t* cols);
hipError_t launch_kkt_struct(const Launch& L, int ninst, int64_t* rowptr, int32_t* colind);
hipError_t launch_bounds(const Launch& L, double* lv, double* uv, double* lc, double* uc);
hipError_t launch_load_adjoint(const Launch& L, const double* lam, double* gpd, double* gqd);

}  // namespace opf
