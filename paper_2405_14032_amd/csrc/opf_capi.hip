// C ABI of libopf: model lifetime, tile lists, entry points, the graph-
// replayed sweep and the autotuner.  Every entry point returns a status code
// and never lets a C++ exception escape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <deque>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/opf.h"
#include "opf_device.h"
#include "opf_api_internal.h"
#include "opf_host.h"

using namespace opf;

static_assert(kScratchPerLine == kLineScratchDoubles, "line scratch layout of the device and the host checks");

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define OPF_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail(OPF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Kernel families, each with its own tile list and launch shape.
enum Op {
  OP_JAC,
  OP_HESS,
  OP_CONS,
  OP_GRAD,
  OP_OBJ,
  OP_JTA,
  OP_JTB,
  OP_KKA,
  OP_KKB,
  OP_JSTR,
  OP_HSTR,
  OP_KSTR,
  OP_BOUNDS,
  OP_LADJ,
  OP_JHKA,
  OP_SWA,
  OP_SWB,
  OP_JV,
  OP_RHSR,  // flat element-wise kernels (no tile list; timing ids only)
  OP_RHSV,
  OP_RECR,
  OP_RECV,
  OP_COUNT
};

const char* kOpName[OP_COUNT] = {"jac", "hess", "cons", "grad", "obj", "jt_a", "jt_b",
                                 "kkt_a", "kkt_b", "jac_struct", "hess_struct", "kkt_struct",
                                 "bounds", "load_adjoint", "jhk_a", "sweep_a", "sweep_b", "jv",
                                 "rhs_rows", "rhs_vars", "rec_rows", "rec_vars"};

struct Shape {
  int block = 256;  // elements per tile = threads per block
  int ppt = 1;      // periods per tile
  int grid = 0;     // 0: one block per tile; > 0: persistent grid size
};

struct TileList {
  Shape shape;
  Tile* d = nullptr;
  int n = 0;
  int cap = 0;
  std::vector<int32_t> inst_begin;  // first tile of each instance (+ total)
  int lds_cap = 0;                  // LDS segment capacity (doubles), staged kernels
  size_t smem = 0;                  // dynamic LDS bytes per block
};

// Largest dynamic LDS a block of the staged kernels may ask for.
constexpr size_t kMaxSmem = 64 * 1024;

}  // namespace

// ---------------------------------------------------------------- static scratch
// Device scratch of opf_sweep_noalloc (hand-off records, then the objective
// partials): a file-scope array, so that call needs no allocation.  Every
// device the library runs on holds its own copy until the process ends.  In
// host code the name below is only a stand-in: kernels get the device
// address looked up per device by static_scratch_lookup.
constexpr int64_t kStaticScratchBytes = 32LL << 20;
constexpr int64_t kStaticScratchDoubles = kStaticScratchBytes / (int64_t)sizeof(double);
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
double* g_static_ptr[kMaxDevices] = {};

// Device address of this device's copy of the static scratch array; the
// device must be current.  Looked up once per device (at model creation).
int static_scratch_lookup(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return OPF_EINVAL;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return OPF_EHIP;
    g_static_ptr[device] = static_cast<double*>(p);
  }
  *out = g_static_ptr[device];
  return OPF_OK;
}

}  // namespace

struct opf_model {
  int device = -1;
  int n_cu = 256;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  std::vector<InstHost> inst;
  int64_t n = 0, m = 0, nnzj = 0, nnzh = 0, nnzk = 0;
  char* arena = nullptr;
  InstDev* d_inst = nullptr;
  std::vector<InstDev> h_dev;  // host mirror of d_inst
  double* scratch = nullptr;
  int64_t scratch_doubles = 0;  // size of scratch (hand-off records, sweep objective partials)
  double* wbuf = nullptr;  // [m]: row vector of the condensation calls
  double* obj_partial = nullptr;
  // the one-launch sweep (k_sweep): per-XCD work queues built from the
  // sweep's line tile shape; off (two launches) when sw_ok is false
  int sw_nq = 0;  // XCDs of the device (queues); 0: unknown
  bool sw_ok = false;
  SweepItem* d_sw_items = nullptr;
  int32_t *d_sw_qbeg = nullptr, *d_sw_ctr = nullptr, *d_sw_flags = nullptr;
  int sw_items_cap = 0, sw_ctr_cap = 0, sw_nctr = 0, sw_grid = 0, sw_block = 0;
  int sw_cap_seg = 0, sw_cap_vm = 0, sw_cap_va = 0;
  size_t sw_smem = 0;
  int obj_partial_cap = 0;
  int32_t* d_obj_begin = nullptr;
  // the objective folded into the two-launch sweep (ObjFold); false when
  // the line pass's block is not whole wavefronts
  bool of_ok = false;
  TileList lists[OP_COUNT];
  // graph-replayed sweep
  hipGraphExec_t gexec = nullptr;
  opf_sweep_args gargs;
  bool gvalid = false;
  // per-kernel timing (opf_set_timing / opf_kernel_stats)
  struct Timed {
    int id;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::vector<Timed> pending;
  std::vector<hipEvent_t> events;  // free pool
  std::vector<hipEvent_t> all_events;
  double t_ms[OP_COUNT + 1] = {};
  int64_t t_n[OP_COUNT + 1] = {};
};

namespace {

bool host_only(const opf_model* M) { return M->device < 0; }

// Timing id of the objective's final reduction (not a tile-list op).
constexpr int kTimeObjFinal = OP_COUNT;

hipEvent_t take_event(opf_model* M) {
  if (!M->events.empty()) {
    hipEvent_t e = M->events.back();
    M->events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  M->all_events.push_back(e);
  return e;
}

// Brackets one kernel launch with events on the model's stream when timing
// is on (and the stream is not being recorded into a graph).
struct TimerScope {
  opf_model* M;
  int id;
  hipEvent_t a = nullptr;
  TimerScope(opf_model* m, int i) : M(m), id(i) {
    if (!M->timing) return;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(M->stream, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return;
    a = take_event(M);
    if (a && hipEventRecord(a, M->stream) != hipSuccess) {
      M->events.push_back(a);
      a = nullptr;
    }
  }
  ~TimerScope() {
    if (!a) return;
    hipEvent_t b = take_event(M);
    if (b && hipEventRecord(b, M->stream) == hipSuccess) {
      M->pending.push_back({id, a, b});
    } else {
      M->events.push_back(a);
      if (b) M->events.push_back(b);
    }
  }
};

void flush_timing(opf_model* M) {
  for (auto& r : M->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      M->t_ms[r.id] += ms;
      M->t_n[r.id] += 1;
    }
    M->events.push_back(r.a);
    M->events.push_back(r.b);
  }
  M->pending.clear();
}

// Element classes of each op (in launch order inside one list).
std::vector<int> kinds_of(int op) {
  switch (op) {
    case OP_JAC:
    case OP_HESS:
    case OP_JTA:
    case OP_KKA:
    case OP_JHKA:
    case OP_SWA:
    case OP_JSTR:
    case OP_HSTR:
      return {TK_BRANCH, TK_GEN};
    case OP_CONS:
    case OP_JV:
      return {TK_BRANCH, TK_BUS, TK_GEN};
    case OP_GRAD:
      return {TK_VAR};
    case OP_OBJ:
      return {TK_GEN};
    case OP_JTB:
    case OP_KKB:
    case OP_SWB:
    case OP_LADJ:
      return {TK_BUS};
    case OP_KSTR:
      return {TK_KROW};
    case OP_BOUNDS:
      return {TK_VAR, TK_CON, TK_GEN};
  }
  return {};
}

int64_t count_of(const InstHost& I, int kind) {
  switch (kind) {
    case TK_BRANCH:
      return I.B;
    case TK_GEN:
      return I.G;
    case TK_BUS:
      return I.N;
    case TK_VAR:
    case TK_KROW:
      return I.n_p;
    case TK_CON:
      return I.m_p;
  }
  return 0;
}

std::vector<Tile> make_tiles(const opf_model* M, int op, const Shape& s, std::vector<int32_t>& begin) {
  std::vector<Tile> out;
  begin.assign(M->inst.size() + 1, 0);
  // The bus kernels that read the line kernels' hand-off records walk the
  // instances and periods backwards: their first reads are then the records
  // written last, which the memory-side cache still holds.
  const bool rev = op == OP_SWB || op == OP_KKB || op == OP_JTB;
  const size_t ni = M->inst.size();
  for (size_t kk = 0; kk < ni; ++kk) {
    const size_t k = rev ? ni - 1 - kk : kk;
    begin[k] = (int32_t)out.size();
    const InstHost& I = M->inst[k];
    // period-major: the runs of the list that the kernels hand to each XCD
    // then hold every element class of their periods in proportion
    const int32_t ngrp = (I.T + s.ppt - 1) / s.ppt;
    for (int32_t gg = 0; gg < ngrp; ++gg) {
      const int32_t grp = rev ? ngrp - 1 - gg : gg;
      const int32_t t0 = grp * s.ppt;
      const int32_t t1 = std::min<int32_t>(I.T, t0 + s.ppt);
      for (int kind : kinds_of(op)) {
        const int64_t cnt = count_of(I, kind);
        for (int64_t e0 = 0; e0 < cnt; e0 += s.block) {
          Tile tl;
          tl.inst = (int32_t)k;
          tl.kind = kind;
          tl.e0 = (int32_t)e0;
          tl.e1 = (int32_t)std::min<int64_t>(cnt, e0 + s.block);
          tl.t0 = t0;
          tl.t1 = t1;
          out.push_back(tl);
        }
      }
    }
  }
  begin[M->inst.size()] = (int32_t)out.size();
  // Inside each XCD's run of the list (the kernels' remap_tile: XCD x takes
  // positions [x q, (x + 1) q), q = n / 8, and the last n mod 8 come after
  // them), generator tiles, the short ones, go after the others: a run then
  // ends on short blocks instead of leaving its CUs idle behind the last long
  // ones.  The per-instance begins stay those of the list before this step
  // (only the single-kind lists use them).
  if (kinds_of(op).size() > 1) {
    const size_t n = out.size(), q = n / 8;
    for (size_t x = 0; x <= 8; ++x) {
      const size_t a = x < 8 ? x * q : 8 * q, b = x < 8 ? (x + 1) * q : n;
      std::stable_partition(out.begin() + a, out.begin() + b, [](const Tile& t) { return t.kind != TK_GEN; });
    }
  }
  return out;
}

// LDS needs of the staged condensed kernels for a tile list: the longest
// contiguous K row segment a tile writes (per flow kind for the line phase,
// vm + va rows for the bus phase).
int lds_needs(const opf_model* M, int op, const std::vector<Tile>& tiles, const Shape& s, int& cap,
              size_t& smem) {
  cap = 0;
  smem = 0;
  if (op == OP_JAC) {  // staged line tiles: 15 streams of blockDim doubles
    smem = 15 * (size_t)s.block * sizeof(double);
    if (smem > kMaxSmem) return fail(OPF_EINVAL, "tile shape needs too much LDS for jac");
    return OPF_OK;
  }
  const bool line = op == OP_KKA || op == OP_JHKA || op == OP_SWA;
  if (!line && op != OP_KKB && op != OP_SWB) return OPF_OK;
  if (line && s.block > 256) return fail(OPF_EINVAL, "condensed line kernel: block > 256");
  int cap2 = 0;
  for (const Tile& tl : tiles) {
    const InstHost& I = M->inst[tl.inst];
    if (line && tl.kind == TK_BRANCH) {
      const int64_t FL = 2LL * I.N + 2LL * I.G;
      for (int k = 0; k < 4; ++k)
        cap = std::max<int>(cap, I.krow[FL + (int64_t)k * I.B + tl.e1] - I.krow[FL + (int64_t)k * I.B + tl.e0]);
    } else if (!line) {
      cap = std::max<int>(cap, I.krow[tl.e1] - I.krow[tl.e0]);
      cap2 = std::max<int>(cap2, I.krow[I.N + tl.e1] - I.krow[I.N + tl.e0]);
    }
  }
  // the line kernels stage their hand-off records in the segment region
  // (a padded stride per lane), and the fused ones also keep each lane's
  // eight admittances in LDS
  if (line) cap = std::max<int>(cap, kRecLds * s.block);
  const size_t adm = (op == OP_JHKA || op == OP_SWA) ? 8 * (size_t)s.block : 0;
  smem = line ? ((size_t)cap + adm) * sizeof(double)
              : ((size_t)cap + (size_t)cap2) * sizeof(double);
  if (smem > kMaxSmem) return fail(OPF_EINVAL, std::string("tile shape needs too much LDS for ") + kOpName[op]);
  return OPF_OK;
}

int build_fused(opf_model* M);

int set_shape(opf_model* M, int op, const Shape& s) {
  TileList& L = M->lists[op];
  std::vector<int32_t> begin;
  std::vector<Tile> tiles = make_tiles(M, op, s, begin);
  if (tiles.size() > (size_t)0x7fffffff) return fail(OPF_ERANGE, "tile list too long");
  int lds_cap = 0;
  size_t smem = 0;
  int rc0 = lds_needs(M, op, tiles, s, lds_cap, smem);
  if (rc0 != OPF_OK) return rc0;
  L.lds_cap = lds_cap;
  L.smem = smem;
  if ((int)tiles.size() > L.cap) {
    if (L.d) OPF_HIP(hipFree(L.d));
    L.d = nullptr;
    L.cap = 0;
    if (hipMalloc(&L.d, std::max<size_t>(1, tiles.size()) * sizeof(Tile)) != hipSuccess) {
      L.d = nullptr;
      return fail(OPF_ENOMEM, std::string("tile list allocation failed for ") + kOpName[op]);
    }
    L.cap = (int)tiles.size();
  }
  if (!tiles.empty())
    OPF_HIP(hipMemcpy(L.d, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice));
  L.n = (int)tiles.size();
  L.shape = s;
  L.inst_begin = begin;
  if (op == OP_OBJ) {
    if (L.n > M->obj_partial_cap) {
      if (M->obj_partial) OPF_HIP(hipFree(M->obj_partial));
      M->obj_partial = nullptr;
      if (hipMalloc(&M->obj_partial, std::max(1, L.n) * sizeof(double)) != hipSuccess)
        return fail(OPF_ENOMEM, "objective partial buffer allocation failed");
      M->obj_partial_cap = L.n;
    }
    OPF_HIP(hipMemcpy(M->d_obj_begin, begin.data(), begin.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  if (op == OP_SWA) M->of_ok = s.block % 64 == 0;
  M->gvalid = false;
  if (op == OP_SWA) return build_fused(M);
  return OPF_OK;
}

// Work queues of the one-launch sweep for the current line tile shape.
// Groups = (instance, run of periods); each XCD's queue gets a contiguous
// run of groups of about equal cost, and lists each group's line and
// generator tiles, then its bus tiles once enough later tiles have been
// listed that the group's line tiles are done by the time a block takes
// them.  Leaves the two-launch sweep in place (sw_ok false) when the
// device's XCD count is unknown or a tile does not fit the LDS budget.
// Switched off: its first two runs on the GPU (the smallest test grid) did
// not finish; the cause is not established, so the two-launch sweep is the
// one that runs and this builder leaves sw_ok false.
constexpr bool kOneLaunchSweep = false;

int build_fused(opf_model* M) {
  M->sw_ok = false;
  if (!kOneLaunchSweep || M->sw_nq <= 0 || M->device < 0) return OPF_OK;
  const int nq = M->sw_nq;
  const int blk = M->lists[OP_SWA].shape.block;
  if (blk > 256) return OPF_OK;
  // periods per group: the largest of 4..1 that spreads the groups evenly
  // over the queues (one instance: T / gp groups)
  int gp = 1;
  for (int c = 4; c >= 1; --c) {
    int64_t ng = 0;
    for (const auto& I : M->inst) ng += (I.T + c - 1) / c;
    const double per = (double)ng / nq, most = (double)((ng + nq - 1) / nq);
    if (M->inst.size() > 1 || ng >= nq * 8 || most <= per * 1.02) {
      gp = c;
      break;
    }
  }
  struct Grp {
    int inst, t0, t1;
    double cost;
  };
  std::vector<Grp> groups;
  double total = 0.0;
  for (size_t k = 0; k < M->inst.size(); ++k) {
    const InstHost& I = M->inst[k];
    for (int t0 = 0; t0 < I.T; t0 += gp) {
      const int t1 = std::min(I.T, t0 + gp);
      const double c = ((double)I.B + 0.3 * I.G + 0.5 * I.N) * (t1 - t0);
      groups.push_back({(int)k, t0, t1, c});
      total += c;
    }
  }
  const int ng = (int)groups.size();
  std::vector<std::vector<int>> qg(nq);
  double acc = 0.0;
  for (int g = 0; g < ng; ++g) {
    const double mid = acc + 0.5 * groups[g].cost;
    const int q = std::min(nq - 1, (int)(mid / std::max(total, 1e-300) * nq));
    qg[q].push_back(g);
    acc += groups[g].cost;
  }
  // launch shape first: the listing lag is counted in blocks per XCD
  // counter slots: each queue's tickets and its groups' counts on lines of
  // their own
  constexpr int kStride = 32;
  std::vector<int32_t> slot(ng, 0);
  int nctr = kStride * nq;
  for (int q = 0; q < nq; ++q) {
    for (int g : qg[q]) slot[g] = nctr++;
    nctr = (nctr + kStride - 1) / kStride * kStride;
  }
  auto tiles_of = [&](const Grp& G, int kind, std::vector<SweepItem>& out, int g, int need) {
    const InstHost& I = M->inst[G.inst];
    const int cnt = kind == TK_BRANCH ? I.B : kind == TK_GEN ? I.G : I.N;
    for (int e0 = 0; e0 < cnt; e0 += blk) {
      SweepItem it;
      it.tl = Tile{G.inst, kind, e0, std::min(cnt, e0 + blk), G.t0, G.t1};
      it.slot = slot[g];
      it.need = need;
      out.push_back(it);
    }
  };
  int cap_seg = kRecLds * blk, cap_vm = 0, cap_va = 0;
  for (const auto& I : M->inst) {
    const int64_t FL = 2LL * I.N + 2LL * I.G;
    for (int e0 = 0; e0 < I.B; e0 += blk) {
      const int e1 = std::min(I.B, e0 + blk);
      for (int k = 0; k < 4; ++k)
        cap_seg = std::max<int>(cap_seg, I.krow[FL + (int64_t)k * I.B + e1] - I.krow[FL + (int64_t)k * I.B + e0]);
    }
    for (int e0 = 0; e0 < I.N; e0 += blk) {
      const int e1 = std::min(I.N, e0 + blk);
      cap_vm = std::max<int>(cap_vm, I.krow[e1] - I.krow[e0]);
      cap_va = std::max<int>(cap_va, I.krow[I.N + e1] - I.krow[I.N + e0]);
    }
  }
  const size_t smem = (size_t)std::max<int64_t>((int64_t)cap_seg + 8LL * blk, (int64_t)cap_vm + cap_va) * sizeof(double);
  if (smem > kMaxSmem) return OPF_OK;
  const int occ = sweep_fused_blocks_per_cu(blk, smem);
  if (occ <= 0) return OPF_OK;
  const int grid = occ * M->n_cu;
  const int lag = std::max(1, grid / nq) * 3 / 2;
  std::vector<SweepItem> items;
  std::vector<int32_t> qbeg(nq + 1, 0), need(ng, 0);
  for (int q = 0; q < nq; ++q) {
    qbeg[q] = (int32_t)items.size();
    std::deque<std::pair<int, size_t>> pend;  // (group, listed items after its last line tile)
    auto flush = [&](bool all) {
      while (!pend.empty() && (all || items.size() - pend.front().second >= (size_t)lag)) {
        const int g = pend.front().first;
        tiles_of(groups[g], TK_BUS, items, g, need[g]);
        pend.pop_front();
      }
    };
    for (int g : qg[q]) {
      const size_t before = items.size();
      tiles_of(groups[g], TK_BRANCH, items, g, 0);
      tiles_of(groups[g], TK_GEN, items, g, 0);
      need[g] = (int32_t)(items.size() - before);
      pend.push_back({g, items.size()});
      flush(false);
    }
    flush(true);
  }
  qbeg[nq] = (int32_t)items.size();
  if (items.size() > (size_t)0x7fffffff) return OPF_OK;
  const int nitems = (int)items.size();
  if (nitems > M->sw_items_cap) {
    if (M->d_sw_items) OPF_HIP(hipFree(M->d_sw_items));
    M->d_sw_items = nullptr;
    M->sw_items_cap = 0;
    if (hipMalloc(&M->d_sw_items, std::max(1, nitems) * sizeof(SweepItem)) != hipSuccess) {
      M->d_sw_items = nullptr;
      return fail(OPF_ENOMEM, "sweep work list allocation failed");
    }
    M->sw_items_cap = nitems;
  }
  if (nctr > M->sw_ctr_cap) {
    if (M->d_sw_ctr) OPF_HIP(hipFree(M->d_sw_ctr));
    M->d_sw_ctr = nullptr;
    M->sw_ctr_cap = 0;
    if (hipMalloc(&M->d_sw_ctr, (size_t)nctr * sizeof(int32_t)) != hipSuccess)
      return fail(OPF_ENOMEM, "sweep counter allocation failed");
    M->sw_ctr_cap = nctr;
  }
  if (!M->d_sw_qbeg) {
    if (hipMalloc(&M->d_sw_qbeg, (nq + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&M->d_sw_flags, sizeof(int32_t)) != hipSuccess)
      return fail(OPF_ENOMEM, "sweep queue allocation failed");
    OPF_HIP(hipMemset(M->d_sw_flags, 0, sizeof(int32_t)));
  }
  OPF_HIP(hipMemcpy(M->d_sw_items, items.data(), items.size() * sizeof(SweepItem), hipMemcpyHostToDevice));
  OPF_HIP(hipMemcpy(M->d_sw_qbeg, qbeg.data(), qbeg.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  M->sw_nctr = nctr;
  M->sw_grid = grid;
  M->sw_block = blk;
  M->sw_cap_seg = cap_seg;
  M->sw_cap_vm = cap_vm;
  M->sw_cap_va = cap_va;
  M->sw_smem = smem;
  // OPF_SWEEP_SPLIT=1 keeps the two-launch sweep (for comparisons)
  const char* split = std::getenv("OPF_SWEEP_SPLIT");
  M->sw_ok = !(split && std::strcmp(split, "1") == 0);
  return OPF_OK;
}

// The default shape of an op, or narrower tiles when a tile's K rows do
// not fit the LDS budget (buses of high degree).
int set_default_shape(opf_model* M, int op) {
  Shape s;
  int rc = set_shape(M, op, s);
  for (int blk = s.block / 2; rc == OPF_EINVAL && blk >= 64; blk /= 2) {
    s.block = blk;
    rc = set_shape(M, op, s);
  }
  return rc;
}

Launch launch_of(const opf_model* M, int op) {
  const TileList& L = M->lists[op];
  Launch l;
  l.insts = M->d_inst;
  l.tiles = L.d;
  l.ntiles = L.n;
  l.block = L.shape.block;
  l.grid = L.shape.grid > 0 ? std::min(L.shape.grid, L.n) : 0;
  l.stream = M->stream;
  l.cap0 = L.lds_cap;
  l.smem = L.smem;
  return l;
}

// Simple bump allocator over one device allocation.
struct Arena {
  size_t size = 0;
  size_t take(size_t bytes) {
    size_t at = size;
    size += (bytes + 255) & ~size_t(255);
    return at;
  }
};

int upload_model(opf_model* M) {
  Arena a;
  struct Place {
    size_t f_bus, t_bus, gen_bus, adm, c2, c1, c0, pd, qd, bus_ptr, bus_adj, bus_nb, bgen_ptr, bgen, krow, kcol, ksrc, kinfo;
    size_t vmin, vmax, pmin, pmax, qmin, qmax, ramp, rate, angmin, angmax;
  };
  std::vector<Place> pl(M->inst.size());
  for (size_t k = 0; k < M->inst.size(); ++k) {
    const InstHost& I = M->inst[k];
    Place& p = pl[k];
    auto b4 = [](size_t n) { return n * 4; };
    auto b8 = [](size_t n) { return n * 8; };
    p.f_bus = a.take(b4(I.f_bus.size()));
    p.t_bus = a.take(b4(I.t_bus.size()));
    p.gen_bus = a.take(b4(I.gen_bus.size()));
    p.adm = a.take(b8(I.adm.size()));
    p.c2 = a.take(b8(I.c2.size()));
    p.c1 = a.take(b8(I.c1.size()));
    p.c0 = a.take(b8(I.c0.size()));
    p.pd = a.take(b8(I.pd.size()));
    p.qd = a.take(b8(I.qd.size()));
    p.bus_ptr = a.take(b4(I.bus_ptr.size()));
    p.bus_adj = a.take(b4(I.bus_adj.size()));
    p.bus_nb = a.take(b4(I.bus_nb.size()));
    p.bgen_ptr = a.take(b4(I.bgen_ptr.size()));
    p.bgen = a.take(b4(I.bgen.size()));
    p.krow = a.take(b4(I.krow.size()));
    p.kcol = a.take(b4(I.kcol.size()));
    p.ksrc = a.take(b4(I.ksrc.size()));
    p.kinfo = a.take(b4(I.kinfo.size()));
    p.vmin = a.take(b8(I.vmin.size()));
    p.vmax = a.take(b8(I.vmax.size()));
    p.pmin = a.take(b8(I.pmin.size()));
    p.pmax = a.take(b8(I.pmax.size()));
    p.qmin = a.take(b8(I.qmin.size()));
    p.qmax = a.take(b8(I.qmax.size()));
    p.ramp = a.take(b8(I.ramp.size()));
    p.rate = a.take(b8(I.rate.size()));
    p.angmin = a.take(b8(I.angmin.size()));
    p.angmax = a.take(b8(I.angmax.size()));
  }
  const size_t inst_at = a.take(sizeof(InstDev) * M->inst.size());
  std::vector<char> host(a.size, 0);
  auto put = [&](size_t at, const void* src, size_t bytes) {
    if (bytes) std::memcpy(host.data() + at, src, bytes);
  };
  if (hipMalloc(&M->arena, std::max<size_t>(a.size, 256)) != hipSuccess) {
    M->arena = nullptr;
    return fail(OPF_ENOMEM, "device arena allocation failed");
  }
  std::vector<InstDev> dv(M->inst.size());
  for (size_t k = 0; k < M->inst.size(); ++k) {
    const InstHost& I = M->inst[k];
    const Place& p = pl[k];
#define PUT(field) put(p.field, I.field.data(), I.field.size() * sizeof(I.field[0]))
    PUT(f_bus);
    PUT(t_bus);
    PUT(gen_bus);
    PUT(adm);
    PUT(c2);
    PUT(c1);
    PUT(c0);
    PUT(pd);
    PUT(qd);
    PUT(bus_ptr);
    PUT(bus_adj);
    PUT(bus_nb);
    PUT(bgen_ptr);
    PUT(bgen);
    PUT(krow);
    PUT(kcol);
    PUT(ksrc);
    PUT(kinfo);
    PUT(vmin);
    PUT(vmax);
    PUT(pmin);
    PUT(pmax);
    PUT(qmin);
    PUT(qmax);
    PUT(ramp);
    PUT(rate);
    PUT(angmin);
    PUT(angmax);
#undef PUT
    InstDev& d = dv[k];
    std::memset(&d, 0, sizeof(d));
    d.N = I.N;
    d.B = I.B;
    d.G = I.G;
    d.T = I.T;
    d.ref = I.ref;
    d.n_p = I.n_p;
    d.m_p = I.m_p;
    d.nnzj_p = I.nnzj_p;
    d.nnzh_p = I.nnzh_p;
    d.nnzk_p = I.nnzk_p;
    d.x_off = I.x_off;
    d.c_off = I.c_off;
    d.j_off = I.j_off;
    d.h_off = I.h_off;
    d.k_off = I.k_off;
    d.ld_off = I.ld_off;
    d.s_off = I.s_off;
    d.o_off = I.o_off;
    char* base = M->arena;
#define PTR(field, T) d.field = reinterpret_cast<T>(base + p.field)
    PTR(f_bus, const int32_t*);
    PTR(t_bus, const int32_t*);
    PTR(gen_bus, const int32_t*);
    PTR(adm, const double*);
    PTR(c2, const double*);
    PTR(c1, const double*);
    PTR(c0, const double*);
    PTR(pd, double*);
    PTR(qd, double*);
    PTR(bus_ptr, const int32_t*);
    PTR(bus_adj, const int32_t*);
    PTR(bus_nb, const int32_t*);
    PTR(bgen_ptr, const int32_t*);
    PTR(bgen, const int32_t*);
    PTR(krow, const int32_t*);
    PTR(kcol, const int32_t*);
    PTR(ksrc, const int32_t*);
    PTR(kinfo, const int32_t*);
    PTR(vmin, const double*);
    PTR(vmax, const double*);
    PTR(pmin, const double*);
    PTR(pmax, const double*);
    PTR(qmin, const double*);
    PTR(qmax, const double*);
    PTR(ramp, const double*);
    PTR(rate, const double*);
    PTR(angmin, const double*);
    PTR(angmax, const double*);
#undef PTR
  }
  put(inst_at, dv.data(), dv.size() * sizeof(InstDev));
  M->h_dev = dv;
  M->d_inst = reinterpret_cast<InstDev*>(M->arena + inst_at);
  OPF_HIP(hipMemcpy(M->arena, host.data(), a.size, hipMemcpyHostToDevice));
  return OPF_OK;
}

void release(opf_model* M) {
  if (!M) return;
  if (M->device >= 0) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != M->device) (void)hipSetDevice(M->device);
    if (M->gexec) (void)hipGraphExecDestroy(M->gexec);
    for (hipEvent_t e : M->all_events) (void)hipEventDestroy(e);
    for (auto& L : M->lists)
      if (L.d) (void)hipFree(L.d);
    if (M->arena) (void)hipFree(M->arena);
    if (M->scratch) (void)hipFree(M->scratch);
    if (M->wbuf) (void)hipFree(M->wbuf);
    if (M->obj_partial) (void)hipFree(M->obj_partial);
    if (M->d_obj_begin) (void)hipFree(M->d_obj_begin);
    for (void* p : {(void*)M->d_sw_items, (void*)M->d_sw_qbeg, (void*)M->d_sw_ctr, (void*)M->d_sw_flags})
      if (p) (void)hipFree(p);
    if (M->cap_stream) (void)hipStreamDestroy(M->cap_stream);
    if (cur >= 0 && cur != M->device) (void)hipSetDevice(cur);
  }
  delete M;
}

// Makes the model's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (dev < 0) return;
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      changed = hipSetDevice(dev) == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

#define OPF_CHECK_MODEL(M)                                                 \
  do {                                                                     \
    if (!(M)) return fail(OPF_EINVAL, "model is NULL");                    \
    if (host_only(M)) return fail(OPF_ENODEV, "model is host-only");       \
  } while (0)

#define OPF_REQUIRE(p, name)                                               \
  do {                                                                     \
    if (!(p)) return fail(OPF_EINVAL, std::string(name) + " is NULL");     \
  } while (0)

#define OPF_LAUNCHED(expr, what)                                                              \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(OPF_EHIP, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- enqueue helpers
// Device scratch of one enqueue: the line -> bus hand-off records and the
// objective's per-tile partial sums.  Normally the model's own buffers; the
// allocation-free sweep passes slices of the library's static array.
struct Work {
  double* scr;
  double* partial;
  int32_t* ctr;  // counters of the one-launch sweep
};

Work model_work(const opf_model* M) { return Work{M->scratch, M->obj_partial, M->d_sw_ctr}; }

int enq_obj(opf_model* M, const Work& w, const double* x, double* f) {
  { TimerScope ts_(M, OP_OBJ); OPF_LAUNCHED(launch_obj_partial(launch_of(M, OP_OBJ), x, w.partial, nullptr, 0), "objective kernel"); }
  {
    TimerScope ts_(M, kTimeObjFinal);
    OPF_LAUNCHED(launch_obj_final(M->d_obj_begin, (int)M->inst.size(), w.partial, f, M->stream),
                 "objective reduction kernel");
  }
  return OPF_OK;
}

int enq_jt(opf_model* M, const Work& w, const double* x, const double* v, double* out) {
  { TimerScope ts_(M, OP_JTA); OPF_LAUNCHED(launch_jt_a(launch_of(M, OP_JTA), x, v, out, w.scr), "J^T v line kernel"); }
  { TimerScope ts_(M, OP_JTB); OPF_LAUNCHED(launch_jt_b(launch_of(M, OP_JTB), v, out, w.scr), "J^T v bus kernel"); }
  return OPF_OK;
}

int enq_kkt(opf_model* M, const Work& w, const double* h, const double* j, const double* dx, const double* d, double* k) {
  { TimerScope ts_(M, OP_KKA); OPF_LAUNCHED(launch_kkt_a(launch_of(M, OP_KKA), h, j, dx, d, k, w.scr), "condensed line kernel"); }
  { TimerScope ts_(M, OP_KKB); OPF_LAUNCHED(launch_kkt_b(launch_of(M, OP_KKB), j, dx, d, k, w.scr), "condensed bus kernel"); }
  return OPF_OK;
}

int enq_jhk(opf_model* M, const Work& w, const double* x, const double* lam, double sigma, const double* dx, const double* d,
            double* j, double* h, double* k) {
  { TimerScope ts_(M, OP_JHKA); OPF_LAUNCHED(launch_jhk_a(launch_of(M, OP_JHKA), x, lam, sigma, h, j, dx, d, k, w.scr),
               "fused J/H/condensed line kernel"); }
  { TimerScope ts_(M, OP_KKB); OPF_LAUNCHED(launch_kkt_b(launch_of(M, OP_KKB), j, dx, d, k, w.scr), "condensed bus kernel"); }
  return OPF_OK;
}

int check_sweep_args(const opf_sweep_args* a) {
  if (!a) return fail(OPF_EINVAL, "sweep args are NULL");
  const bool need_x = a->f || a->grad || a->c || a->jvals || a->hvals || a->jtv;
  if (need_x && !a->x) return fail(OPF_EINVAL, "sweep: x is NULL");
  if (a->hvals && !a->lambda) return fail(OPF_EINVAL, "sweep: lambda is NULL");
  if (a->jtv && !a->v) return fail(OPF_EINVAL, "sweep: v is NULL");
  if (a->kvals && (!a->jvals || !a->hvals || !a->dcon))
    return fail(OPF_EINVAL, "sweep: kvals needs jvals, hvals and dcon");
  return OPF_OK;
}

int enq_sweep(opf_model* M, const Work& w, const opf_sweep_args* a) {
  int rc;
  // every per-element output requested: two fused passes (lines and
  // generators, then buses) that also carry the objective
  if (a->grad && a->c && a->jvals && a->hvals && a->jtv && a->kvals && M->sw_ok && w.ctr) {
    // one launch for lines, generators and buses (the objective's partial
    // pass first, which also clears the launch's counters)
    const int nctr = M->sw_nctr;
    if (a->f && M->lists[OP_OBJ].n > 0) {
      TimerScope ts_(M, OP_OBJ);
      OPF_LAUNCHED(launch_obj_partial(launch_of(M, OP_OBJ), a->x, w.partial, w.ctr, nctr), "objective kernel");
    } else {
      OPF_LAUNCHED(launch_sweep_open(w.ctr, nctr, M->stream), "sweep counter reset");
    }
    {
      TimerScope ts_(M, OP_SWA);
      FusedSweep F;
      F.insts = M->d_inst;
      F.items = M->d_sw_items;
      F.qbeg = M->d_sw_qbeg;
      F.nq = M->sw_nq;
      F.ctr = w.ctr;
      F.flags = M->d_sw_flags;
      F.cap_seg = M->sw_cap_seg;
      F.cap_vm = M->sw_cap_vm;
      F.cap_va = M->sw_cap_va;
      F.smem = M->sw_smem;
      F.grid = M->sw_grid;
      F.block = M->sw_block;
      F.stream = M->stream;
      OPF_LAUNCHED(launch_sweep_fused(F, a->x, a->lambda, a->sigma, a->v, a->hvals, a->jvals, a->diag_x, a->dcon,
                                      a->kvals, a->c, a->jtv, a->grad, w.scr),
                   "sweep kernel");
    }
    {
      TimerScope ts_(M, kTimeObjFinal);
      OPF_LAUNCHED(launch_sweep_close(M->d_obj_begin, (int)M->inst.size(), w.partial, a->f, w.ctr, M->d_sw_qbeg,
                                      M->sw_nq, M->d_sw_flags, M->stream),
                   "sweep close kernel");
    }
    return OPF_OK;
  }
  if (a->grad && a->c && a->jvals && a->hvals && a->jtv && a->kvals) {
    // the objective rides along in the two kernels when the tile lists allow
    ObjFold of;
    const bool fold = a->f && M->of_ok && M->lists[OP_SWA].n > 0 && M->lists[OP_SWB].n > 0;
    if (fold) {
      of.ninst = (int)M->inst.size();
      of.ppt = M->lists[OP_SWA].shape.ppt;
      of.f = a->f;
    }
    { TimerScope ts_(M, OP_SWA); OPF_LAUNCHED(launch_sweep_a(launch_of(M, OP_SWA), a->x, a->lambda, a->sigma, a->v, a->hvals, a->jvals, a->diag_x,
                                a->dcon, a->kvals, a->c, a->jtv, a->grad, w.scr),
                 "sweep line kernel"); }
    { TimerScope ts_(M, OP_SWB); OPF_LAUNCHED(launch_sweep_b(launch_of(M, OP_SWB), a->x, a->v, a->jvals, a->diag_x, a->dcon, a->kvals, a->c,
                                a->jtv, a->grad, w.scr, of),
                 "sweep bus kernel"); }
    if (a->f && !fold && (rc = enq_obj(M, w, a->x, a->f)) != OPF_OK) return rc;
    return OPF_OK;
  }
  // J, H and K together: the fused pass (K from the J / H values in registers)
  const bool fused = a->jvals && a->hvals && a->kvals;
  if (fused) {
    if ((rc = enq_jhk(M, w, a->x, a->lambda, a->sigma, a->diag_x, a->dcon, a->jvals, a->hvals, a->kvals)) != OPF_OK)
      return rc;
  } else {
    if (a->jvals) { TimerScope ts_(M, OP_JAC); OPF_LAUNCHED(launch_jac(launch_of(M, OP_JAC), a->x, a->jvals), "Jacobian kernel"); }
    if (a->hvals)
      { TimerScope ts_(M, OP_HESS); OPF_LAUNCHED(launch_hess(launch_of(M, OP_HESS), a->x, a->lambda, a->sigma, a->hvals), "Hessian kernel"); }
  }
  if (a->c) { TimerScope ts_(M, OP_CONS); OPF_LAUNCHED(launch_cons(launch_of(M, OP_CONS), a->x, a->c), "constraint kernel"); }
  if (a->grad) { TimerScope ts_(M, OP_GRAD); OPF_LAUNCHED(launch_grad(launch_of(M, OP_GRAD), a->x, a->grad), "gradient kernel"); }
  if (a->f && (rc = enq_obj(M, w, a->x, a->f)) != OPF_OK) return rc;
  if (a->jtv && (rc = enq_jt(M, w, a->x, a->v, a->jtv)) != OPF_OK) return rc;
  return OPF_OK;
}

}  // namespace

// Accessors for the other ABI translation units (opf_api_internal.h).
namespace opf {
int api_fail(int code, const std::string& msg) { return fail(code, msg); }
int model_device(const opf_model* M) { return M->device; }
hipStream_t model_stream(const opf_model* M) { return M->stream; }
const std::vector<InstHost>& model_insts(const opf_model* M) { return M->inst; }
int64_t model_n(const opf_model* M) { return M->n; }
int64_t model_nnzk(const opf_model* M) { return M->nnzk; }
}  // namespace opf

// ============================================================== C ABI
extern "C" {

const char* opf_last_error(void) { return g_err.c_str(); }

int opf_validate(const opf_instance_desc* desc, int32_t ninst) {
  try {
    std::string err;
    int rc = validate_descs(desc, ninst, err);
    if (rc != OPF_OK) return fail(rc, err);
    return OPF_OK;
  } catch (const std::bad_alloc&) {
    return fail(OPF_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(OPF_EINVAL, "unexpected host exception");
  }
}

int opf_model_create(const opf_instance_desc* desc, int32_t ninst, int device, opf_model** out) {
  if (!out) return fail(OPF_EINVAL, "out is NULL");
  *out = nullptr;
  opf_model* M = nullptr;
  try {
    std::string err;
    int rc = validate_descs(desc, ninst, err);
    if (rc != OPF_OK) return fail(rc, err);
    if (const char* inj = std::getenv("OPF_TEST_FAIL_ALLOC")) {
      if (std::strcmp(inj, "1") == 0) return fail(OPF_ENOMEM, "allocation failure injected by OPF_TEST_FAIL_ALLOC");
    }
    M = new opf_model();
    M->device = device;
    M->inst.resize(ninst);
    for (int32_t k = 0; k < ninst; ++k) {
      rc = build_instance(desc[k], M->inst[k], err);
      if (rc != OPF_OK) {
        release(M);
        return fail(rc, "instance " + std::to_string(k) + ": " + err);
      }
    }
    rc = assign_offsets(M->inst, err);
    if (rc != OPF_OK) {
      release(M);
      return fail(rc, err);
    }
    for (const auto& I : M->inst) {
      M->n += I.n;
      M->m += I.m;
      M->nnzj += I.nnzj;
      M->nnzh += I.nnzh;
      M->nnzk += I.nnzk;
    }
    if (device < 0) {
      *out = M;
      return OPF_OK;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
      release(M);
      return fail(OPF_EINVAL, "device " + std::to_string(device) + " is not available");
    }
    DeviceGuard guard(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
      M->n_cu = prop.multiProcessorCount;
    if ((rc = upload_model(M)) != OPF_OK) {
      std::string e = g_err;
      release(M);
      return fail(rc, e);
    }
    size_t scr = 0;
    for (const auto& I : M->inst) scr += (size_t)(line_scratch_doubles(I.B, I.T) + obj_scratch_doubles(I.G, I.T));
    M->scratch_doubles = (int64_t)scr;
    if (device < kMaxDevices) {
      double* sp = nullptr;
      if (static_scratch_lookup(device, &sp) != OPF_OK) {
        release(M);
        return fail(OPF_EHIP, "static scratch: hipGetSymbolAddress failed");
      }
    }
    if (hipMalloc(&M->scratch, std::max<size_t>(scr, 1) * sizeof(double)) != hipSuccess) {
      M->scratch = nullptr;
      release(M);
      return fail(OPF_ENOMEM, "scratch allocation failed");
    }
    if (hipMalloc(&M->wbuf, std::max<size_t>((size_t)M->m, 1) * sizeof(double)) != hipSuccess) {
      M->wbuf = nullptr;
      release(M);
      return fail(OPF_ENOMEM, "work vector allocation failed");
    }
    if (hipMalloc(&M->d_obj_begin, (ninst + 1) * sizeof(int32_t)) != hipSuccess) {
      M->d_obj_begin = nullptr;
      release(M);
      return fail(OPF_ENOMEM, "allocation failed");
    }
    if (hipStreamCreateWithFlags(&M->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      M->cap_stream = nullptr;
      release(M);
      return fail(OPF_EHIP, "stream creation failed");
    }
    {
      int nxcc = 0;
      if (hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, device) == hipSuccess && nxcc > 0 &&
          nxcc <= 64)
        M->sw_nq = nxcc;
    }
    for (int op = 0; op < OP_COUNT; ++op) {
      if ((rc = set_default_shape(M, op)) != OPF_OK) {
        std::string e = g_err;
        release(M);
        return fail(rc, e);
      }
    }
    *out = M;
    return OPF_OK;
  } catch (const std::bad_alloc&) {
    release(M);
    return fail(OPF_ENOMEM, "host allocation failed");
  } catch (...) {
    release(M);
    return fail(OPF_EINVAL, "unexpected host exception");
  }
}

void opf_model_destroy(opf_model* model) { release(model); }

int opf_model_dims(const opf_model* M, opf_dims* d) {
  if (!M || !d) return fail(OPF_EINVAL, "model or dims is NULL");
  d->n = M->n;
  d->m = M->m;
  d->nnz_jac = M->nnzj;
  d->nnz_hess = M->nnzh;
  d->nnz_kkt = M->nnzk;
  d->ninst = (int32_t)M->inst.size();
  return OPF_OK;
}

int opf_instance_offsets(const opf_model* M, int64_t* x_off, int64_t* c_off, int64_t* j_off, int64_t* h_off,
                         int64_t* k_off) {
  if (!M) return fail(OPF_EINVAL, "model is NULL");
  const size_t K = M->inst.size();
  for (size_t k = 0; k < K; ++k) {
    const InstHost& I = M->inst[k];
    if (x_off) x_off[k] = I.x_off;
    if (c_off) c_off[k] = I.c_off;
    if (j_off) j_off[k] = I.j_off;
    if (h_off) h_off[k] = I.h_off;
    if (k_off) k_off[k] = I.k_off;
  }
  if (x_off) x_off[K] = M->n;
  if (c_off) c_off[K] = M->m;
  if (j_off) j_off[K] = M->nnzj;
  if (h_off) h_off[K] = M->nnzh;
  if (k_off) k_off[K] = M->nnzk;
  return OPF_OK;
}

int opf_set_stream(opf_model* M, void* s) {
  OPF_CHECK_MODEL(M);
  M->stream = reinterpret_cast<hipStream_t>(s);
  return OPF_OK;
}

int opf_bounds(const opf_model* Mc, double* lv, double* uv, double* lc, double* uc) {
  opf_model* M = const_cast<opf_model*>(Mc);
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(lv && uv && lc && uc, "a bounds array");
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_BOUNDS); OPF_LAUNCHED(launch_bounds(launch_of(M, OP_BOUNDS), lv, uv, lc, uc), "bounds kernel"); }
  return OPF_OK;
}

int opf_jac_structure(const opf_model* Mc, int32_t* rows, int32_t* cols) {
  opf_model* M = const_cast<opf_model*>(Mc);
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(rows && cols, "rows / cols");
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_JSTR); OPF_LAUNCHED(launch_jac_struct(launch_of(M, OP_JSTR), rows, cols), "Jacobian structure kernel"); }
  return OPF_OK;
}

int opf_hess_structure(const opf_model* Mc, int32_t* rows, int32_t* cols) {
  opf_model* M = const_cast<opf_model*>(Mc);
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(rows && cols, "rows / cols");
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_HSTR); OPF_LAUNCHED(launch_hess_struct(launch_of(M, OP_HSTR), rows, cols), "Hessian structure kernel"); }
  return OPF_OK;
}

int opf_kkt_structure(const opf_model* Mc, int64_t* rowptr, int32_t* colind) {
  opf_model* M = const_cast<opf_model*>(Mc);
  if (!M) return fail(OPF_EINVAL, "model is NULL");
  OPF_REQUIRE(rowptr && colind, "rowptr / colind");
  try {
    if (host_only(M)) {
      kkt_structure_host(M->inst, rowptr, colind);
      return OPF_OK;
    }
  } catch (...) {
    return fail(OPF_EINVAL, "unexpected host exception");
  }
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_KSTR); OPF_LAUNCHED(launch_kkt_struct(launch_of(M, OP_KSTR), (int)M->inst.size(), rowptr, colind),
               "condensed structure kernel"); }
  return OPF_OK;
}

int opf_eval_obj(opf_model* M, const double* x, double* f) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(x && f, "x / f");
  DeviceGuard g(M->device);
  return enq_obj(M, model_work(M), x, f);
}

int opf_eval_grad(opf_model* M, const double* x, double* gr) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(x && gr, "x / g");
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_GRAD); OPF_LAUNCHED(launch_grad(launch_of(M, OP_GRAD), x, gr), "gradient kernel"); }
  return OPF_OK;
}

int opf_eval_cons(opf_model* M, const double* x, double* c) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(x && c, "x / c");
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_CONS); OPF_LAUNCHED(launch_cons(launch_of(M, OP_CONS), x, c), "constraint kernel"); }
  return OPF_OK;
}

int opf_eval_jac(opf_model* M, const double* x, double* jv) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(x && jv, "x / jvals");
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_JAC); OPF_LAUNCHED(launch_jac(launch_of(M, OP_JAC), x, jv), "Jacobian kernel"); }
  return OPF_OK;
}

int opf_eval_hess(opf_model* M, const double* x, const double* lam, double sigma, double* hv) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(x && lam && hv, "x / lambda / hvals");
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_HESS); OPF_LAUNCHED(launch_hess(launch_of(M, OP_HESS), x, lam, sigma, hv), "Hessian kernel"); }
  return OPF_OK;
}

int opf_jtprod(opf_model* M, const double* x, const double* v, double* out) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(x && v && out, "x / v / jtv");
  DeviceGuard g(M->device);
  return enq_jt(M, model_work(M), x, v, out);
}

int opf_set_load(opf_model* M, const double* pd, const double* qd) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(pd && qd, "pd / qd");
  DeviceGuard g(M->device);
  for (size_t k = 0; k < M->inst.size(); ++k) {
    const InstHost& I = M->inst[k];
    const size_t bytes = (size_t)I.T * I.N * sizeof(double);
    OPF_HIP(hipMemcpyAsync(M->h_dev[k].pd, pd + I.ld_off, bytes, hipMemcpyDeviceToDevice, M->stream));
    OPF_HIP(hipMemcpyAsync(M->h_dev[k].qd, qd + I.ld_off, bytes, hipMemcpyDeviceToDevice, M->stream));
  }
  return OPF_OK;
}

int opf_load_adjoint(opf_model* M, const double* lam, double* gpd, double* gqd) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(lam && gpd && gqd, "lambda / gpd / gqd");
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_LADJ); OPF_LAUNCHED(launch_load_adjoint(launch_of(M, OP_LADJ), lam, gpd, gqd), "load adjoint kernel"); }
  return OPF_OK;
}

int opf_jprod(opf_model* M, const double* x, const double* v, double* jv) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(x && v && jv, "x / v / jv");
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_JV); OPF_LAUNCHED(launch_jv(launch_of(M, OP_JV), x, v, jv), "J v kernel"); }
  return OPF_OK;
}

namespace {
int ipm_dev(const opf_ipm_state* st, IpmDev& d) {
  if (!st) return fail(OPF_EINVAL, "state is NULL");
  if (!(st->x && st->s && st->y && st->zl && st->zu && st->vl && st->vu && st->xl && st->xu && st->sl && st->su))
    return fail(OPF_EINVAL, "state: an array is NULL");
  if (!(std::isfinite(st->mu) && std::isfinite(st->delta_w) && std::isfinite(st->delta_c) && st->mu >= 0.0 &&
        st->delta_w >= 0.0 && st->delta_c >= 0.0))
    return fail(OPF_EINVAL, "state: mu, delta_w and delta_c must be finite and >= 0");
  d = IpmDev{st->x, st->s, st->y, st->zl, st->zu, st->vl, st->vu, st->xl, st->xu, st->sl, st->su,
             st->mu, st->delta_w, st->delta_c};
  return OPF_OK;
}
}  // namespace

int opf_condensed_rhs(opf_model* M, const opf_ipm_state* st, const double* grad, const double* c, double* diag_x,
                      double* dcon, double* rhs) {
  if (!M) return fail(OPF_EINVAL, "model is NULL");
  IpmDev d;
  int rc = ipm_dev(st, d);
  if (rc != OPF_OK) return rc;
  OPF_REQUIRE(grad && c && diag_x && dcon && rhs, "grad / c / diag_x / dcon / rhs");
  OPF_CHECK_MODEL(M);
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_RHSR); OPF_LAUNCHED(launch_rhs_rows(Flat{M->m, M->stream}, d, c, dcon, M->wbuf), "condensed rhs row kernel"); }
  if ((rc = enq_jt(M, model_work(M), st->x, M->wbuf, rhs)) != OPF_OK) return rc;
  { TimerScope ts_(M, OP_RHSV); OPF_LAUNCHED(launch_rhs_vars(Flat{M->n, M->stream}, d, grad, diag_x, rhs), "condensed rhs variable kernel"); }
  return OPF_OK;
}

int opf_recover_step(opf_model* M, const opf_ipm_state* st, const double* c, const double* dx, double* ds,
                     double* dy, double* dzl, double* dzu, double* dvl, double* dvu) {
  if (!M) return fail(OPF_EINVAL, "model is NULL");
  IpmDev d;
  int rc = ipm_dev(st, d);
  if (rc != OPF_OK) return rc;
  OPF_REQUIRE(c && dx && ds && dy && dzl && dzu && dvl && dvu, "c / dx / ds / dy / dzl / dzu / dvl / dvu");
  OPF_CHECK_MODEL(M);
  DeviceGuard g(M->device);
  { TimerScope ts_(M, OP_JV); OPF_LAUNCHED(launch_jv(launch_of(M, OP_JV), st->x, dx, M->wbuf), "J v kernel"); }
  { TimerScope ts_(M, OP_RECR); OPF_LAUNCHED(launch_rec_rows(Flat{M->m, M->stream}, d, c, M->wbuf, ds, dy, dvl, dvu), "step recovery row kernel"); }
  { TimerScope ts_(M, OP_RECV); OPF_LAUNCHED(launch_rec_vars(Flat{M->n, M->stream}, d, dx, dzl, dzu), "step recovery variable kernel"); }
  return OPF_OK;
}

int opf_assemble_condensed(opf_model* M, const double* hv, const double* jv, const double* dx, const double* d,
                           double* kv) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(hv && jv && d && kv, "hvals / jvals / dcon / kvals");
  DeviceGuard g(M->device);
  return enq_kkt(M, model_work(M), hv, jv, dx, d, kv);
}

int opf_eval_jhk(opf_model* M, const double* x, const double* lam, double sigma, const double* dx, const double* d,
                 double* jv, double* hv, double* kv) {
  OPF_CHECK_MODEL(M);
  OPF_REQUIRE(x && lam && d && jv && hv && kv, "x / lambda / dcon / jvals / hvals / kvals");
  DeviceGuard g(M->device);
  return enq_jhk(M, model_work(M), x, lam, sigma, dx, d, jv, hv, kv);
}

int opf_set_timing(opf_model* M, int enable) {
  OPF_CHECK_MODEL(M);
  DeviceGuard g(M->device);
  flush_timing(M);
  for (int i = 0; i <= OP_COUNT; ++i) {
    M->t_ms[i] = 0.0;
    M->t_n[i] = 0;
  }
  M->timing = enable != 0;
  return OPF_OK;
}

int opf_kernel_stats(opf_model* M, int32_t index, const char** name, int64_t* launches, double* total_ms) {
  OPF_CHECK_MODEL(M);
  if (index < 0 || index > OP_COUNT) return fail(OPF_ERANGE, "kernel index out of range");
  DeviceGuard g(M->device);
  flush_timing(M);
  if (name) *name = index == kTimeObjFinal ? "obj_final" : kOpName[index];
  if (launches) *launches = M->t_n[index];
  if (total_ms) *total_ms = M->t_ms[index];
  return OPF_OK;
}

int opf_sweep(opf_model* M, const opf_sweep_args* a) {
  OPF_CHECK_MODEL(M);
  int rc = check_sweep_args(a);
  if (rc != OPF_OK) return rc;
  DeviceGuard g(M->device);
  return enq_sweep(M, model_work(M), a);
}

int opf_sweep_graph(opf_model* M, const opf_sweep_args* a) {
  OPF_CHECK_MODEL(M);
  int rc = check_sweep_args(a);
  if (rc != OPF_OK) return rc;
  DeviceGuard g(M->device);
  if (!M->gvalid || std::memcmp(&M->gargs, a, sizeof(opf_sweep_args)) != 0) {
    if (M->gexec) {
      OPF_HIP(hipGraphExecDestroy(M->gexec));
      M->gexec = nullptr;
    }
    M->gvalid = false;
    hipStream_t keep = M->stream;
    M->stream = M->cap_stream;
    OPF_HIP(hipStreamBeginCapture(M->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = enq_sweep(M, model_work(M), a);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(M->cap_stream, &graph);
    M->stream = keep;
    if (rc != OPF_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(OPF_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&M->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      M->gexec = nullptr;
      return fail(OPF_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    M->gargs = *a;
    M->gvalid = true;
  }
  OPF_HIP(hipGraphLaunch(M->gexec, M->stream));
  return OPF_OK;
}

int opf_sweep_noalloc(opf_model* M, const opf_sweep_args* a) {
  OPF_CHECK_MODEL(M);
  int rc = check_sweep_args(a);
  if (rc != OPF_OK) return rc;
  const int64_t parts = ((int64_t)M->lists[OP_OBJ].n + 31) / 32 * 32;
  const int64_t ctrs = M->sw_ok ? ((int64_t)M->sw_nctr + 63) / 64 * 32 : 0;  // doubles holding the int32 counters
  const int64_t need = M->scratch_doubles + parts + ctrs;
  if (need > kStaticScratchDoubles)
    return fail(OPF_ERANGE, "opf_sweep_noalloc: the model needs " + std::to_string(need * 8) +
                                " bytes of scratch, the static buffer holds " + std::to_string(kStaticScratchBytes));
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (M->device < kMaxDevices) base = g_static_ptr[M->device];
  }
  if (!base) return fail(OPF_EHIP, "opf_sweep_noalloc: no static scratch on this device");
  DeviceGuard g(M->device);
  // no timing events here: their pool may have to create events
  const bool timing = M->timing;
  M->timing = false;
  rc = enq_sweep(M,
                 Work{base, base + M->scratch_doubles,
                      M->sw_ok ? reinterpret_cast<int32_t*>(base + M->scratch_doubles + parts) : nullptr},
                 a);
  M->timing = timing;
  return rc;
}

int opf_sweep_check(opf_model* M, int32_t* status) {
  OPF_CHECK_MODEL(M);
  if (!status) return fail(OPF_EINVAL, "status is NULL");
  *status = 0;
  if (!M->d_sw_flags) return OPF_OK;
  DeviceGuard g(M->device);
  OPF_HIP(hipStreamSynchronize(M->stream));
  int32_t v = 0;
  OPF_HIP(hipMemcpy(&v, M->d_sw_flags, sizeof(v), hipMemcpyDeviceToHost));
  if (v) OPF_HIP(hipMemset(M->d_sw_flags, 0, sizeof(int32_t)));
  *status = v;
  return OPF_OK;
}

}  // extern "C"

// ============================================================== autotuner
namespace {

std::string shape_key(const opf_model* M) {
  std::ostringstream s;
  s << "cu" << M->n_cu << "_k" << M->inst.size();
  int64_t sn = 0, sb = 0, sg = 0, st = 0;
  for (const auto& I : M->inst) {
    sn += (int64_t)I.N * I.T;
    sb += (int64_t)I.B * I.T;
    sg += (int64_t)I.G * I.T;
    st += I.T;
  }
  s << "_nt" << sn << "_bt" << sb << "_gt" << sg << "_t" << st;
  return s.str();
}

// Minimal reader for the cache written below: one line per key,
//   "key": {"op": [block, ppt, grid], ...}
bool read_cache(const char* path, const std::string& key, std::vector<Shape>& shapes) {
  if (!path) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  const std::string tag = "\"" + key + "\"";
  while (std::getline(f, line)) {
    if (line.find(tag) == std::string::npos) continue;
    shapes.assign(OP_COUNT, Shape());
    for (int op = 0; op < OP_COUNT; ++op) {
      std::string name = std::string("\"") + kOpName[op] + "\": [";
      size_t at = line.find(name);
      if (at == std::string::npos) return false;
      int b = 0, p = 0, g = 0;
      if (std::sscanf(line.c_str() + at + name.size(), "%d, %d, %d", &b, &p, &g) != 3) return false;
      if (b < 64 || b > 512 || (b & 63) || p < 1 || g < 0) return false;
      shapes[op].block = b;
      shapes[op].ppt = p;
      shapes[op].grid = g;
    }
    return true;
  }
  return false;
}

void write_cache(const char* path, const std::string& key, const opf_model* M) {
  if (!path) return;
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line;
    const std::string tag = "\"" + key + "\"";
    while (f && std::getline(f, line))
      if (line.find("\": {") != std::string::npos && line.find(tag) == std::string::npos) keep.push_back(line);
  }
  std::ostringstream s;
  s << "  \"" << key << "\": {";
  for (int op = 0; op < OP_COUNT; ++op) {
    const Shape& sh = M->lists[op].shape;
    s << "\"" << kOpName[op] << "\": [" << sh.block << ", " << sh.ppt << ", " << sh.grid << "]"
      << (op + 1 < OP_COUNT ? ", " : "");
  }
  s << "}";
  keep.push_back(s.str());
  std::ofstream o(path);
  o << "{\n";
  for (size_t i = 0; i < keep.size(); ++i) {
    std::string l = keep[i];
    while (!l.empty() && (l.back() == ',' || l.back() == ' ')) l.pop_back();
    o << l << (i + 1 < keep.size() ? ",\n" : "\n");
  }
  o << "}\n";
}

}  // namespace

extern "C" int opf_autotune(opf_model* M, const char* cache_path) {
  OPF_CHECK_MODEL(M);
  DeviceGuard guard(M->device);
  const std::string key = shape_key(M);
  std::vector<Shape> cached;
  int rc;
  if (read_cache(cache_path, key, cached)) {
    bool ok = true;
    for (int op = 0; op < OP_COUNT && ok; ++op) ok = set_shape(M, op, cached[op]) == OPF_OK;
    if (ok) return OPF_OK;
    for (int op = 0; op < OP_COUNT; ++op)  // stale entry: back to defaults, then tune
      if ((rc = set_default_shape(M, op)) != OPF_OK) return rc;
  }
  // scratch inputs / outputs for timing (contents only need to be finite)
  const size_t n = M->n, m = M->m;
  double *x = nullptr, *lam = nullptr, *dx = nullptr, *d = nullptr, *out_n = nullptr, *out_m = nullptr,
         *dx_out = nullptr;
  double *jv = nullptr, *hv = nullptr, *kv = nullptr;
  auto cleanup = [&]() {
    for (double* p : {x, lam, dx, d, out_n, out_m, dx_out, jv, hv, kv})
      if (p) (void)hipFree(p);
  };
  if (hipMalloc(&x, n * 8) != hipSuccess || hipMalloc(&lam, m * 8) != hipSuccess ||
      hipMalloc(&dx, n * 8) != hipSuccess || hipMalloc(&d, m * 8) != hipSuccess ||
      hipMalloc(&out_n, n * 8) != hipSuccess || hipMalloc(&out_m, m * 8) != hipSuccess ||
      hipMalloc(&dx_out, n * 8) != hipSuccess ||
      hipMalloc(&jv, M->nnzj * 8) != hipSuccess || hipMalloc(&hv, M->nnzh * 8) != hipSuccess ||
      hipMalloc(&kv, M->nnzk * 8) != hipSuccess) {
    cleanup();
    return fail(OPF_ENOMEM, "autotune buffers");
  }
  {
    std::vector<double> hx(n, 1.0), hm(m, 0.5);
    if (hipMemcpy(x, hx.data(), n * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dx, hx.data(), n * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(lam, hm.data(), m * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d, hm.data(), m * 8, hipMemcpyHostToDevice) != hipSuccess) {
      cleanup();
      return fail(OPF_EHIP, "autotune upload");
    }
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  auto run = [&](int op) -> hipError_t {
    switch (op) {
      case OP_JAC:
        return launch_jac(launch_of(M, op), x, jv);
      case OP_HESS:
        return launch_hess(launch_of(M, op), x, lam, 1.0, hv);
      case OP_CONS:
        return launch_cons(launch_of(M, op), x, out_m);
      case OP_GRAD:
        return launch_grad(launch_of(M, op), x, out_n);
      case OP_OBJ:
        return launch_obj_partial(launch_of(M, op), x, M->obj_partial, nullptr, 0);
      case OP_JTA:
        return launch_jt_a(launch_of(M, op), x, lam, out_n, M->scratch);
      case OP_JTB:
        return launch_jt_b(launch_of(M, op), lam, out_n, M->scratch);
      case OP_KKA:
        return launch_kkt_a(launch_of(M, op), hv, jv, dx, d, kv, M->scratch);
      case OP_KKB:
        return launch_kkt_b(launch_of(M, op), jv, dx, d, kv, M->scratch);
      case OP_JHKA:
        return launch_jhk_a(launch_of(M, op), x, lam, 1.0, hv, jv, dx, d, kv, M->scratch);
      case OP_SWA:
        return launch_sweep_a(launch_of(M, op), x, lam, 1.0, lam, hv, jv, dx, d, kv, out_m, out_n, dx_out,
                              M->scratch);
      case OP_SWB:
        return launch_sweep_b(launch_of(M, op), x, lam, jv, dx, d, kv, out_m, out_n, dx_out, M->scratch, ObjFold{});
      case OP_JV:
        return launch_jv(launch_of(M, op), x, dx, out_m);
    }
    return hipSuccess;
  };
  // fill J and H once so the condensed candidates read finite data
  (void)run(OP_JAC);
  (void)run(OP_HESS);
  const int tuned[] = {OP_JAC, OP_HESS, OP_CONS, OP_GRAD, OP_OBJ, OP_JTA, OP_JTB, OP_KKA, OP_KKB, OP_JHKA,
                       OP_SWA, OP_SWB, OP_JV};
  const int blocks[] = {64, 128, 256, 512};
  const int ppts[] = {1, 2, 4, 8};
  rc = OPF_OK;
  for (int op : tuned) {
    Shape best = M->lists[op].shape;
    float best_ms = 1e30f;
    for (int b : blocks) {
      if (op == OP_OBJ && b > 512) continue;
      for (int p : ppts) {
        for (int gm = 0; gm < 2; ++gm) {
          Shape s;
          s.block = b;
          s.ppt = p;
          s.grid = gm == 0 ? 0 : M->n_cu * (2048 / b);
          if (((op == OP_KKA || op == OP_JHKA || op == OP_SWA) && b > 256) ||
              (rc = set_shape(M, op, s)) != OPF_OK) {
            rc = OPF_OK;  // infeasible shape (block or LDS limit): skip it
            continue;
          }
          if (gm == 1 && M->lists[op].n <= s.grid) continue;  // same as one block per tile
          hipError_t he = run(op);
          if (he != hipSuccess) {
            rc = fail(OPF_EHIP, std::string("autotune launch: ") + hipGetErrorString(he));
            break;
          }
          float ms_min = 1e30f;
          for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(e0, M->stream);
            (void)run(op);
            (void)hipEventRecord(e1, M->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms_min = std::min(ms_min, ms);
          }
          if (ms_min < best_ms) {
            best_ms = ms_min;
            best = s;
          }
        }
        if (rc != OPF_OK) break;
      }
      if (rc != OPF_OK) break;
    }
    if (rc != OPF_OK) break;
    if ((rc = set_shape(M, op, best)) != OPF_OK) break;
  }
  (void)hipStreamSynchronize(M->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cleanup();
  if (rc != OPF_OK) return rc;
  // structure / bounds / adjoint kernels follow their evaluation siblings
  set_shape(M, OP_JSTR, M->lists[OP_JAC].shape);
  set_shape(M, OP_HSTR, M->lists[OP_HESS].shape);
  set_shape(M, OP_LADJ, M->lists[OP_JTB].shape);
  write_cache(cache_path, key, M);
  return OPF_OK;
}
