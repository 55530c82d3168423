// Host-side model building: descriptor validation, element tables and the
// per-period symbolic plans.  Pure C++ (no HIP), so it is also usable in a
// host-only model on a machine without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/opf.h"

namespace opf {

// Doubles of line scratch per line and period (the device layout: two
// 64-byte end records, the shared cross pair, four J^T v hand-off values).
constexpr int64_t kLineScratchDoubles = 22;
// Doubles of one instance's scratch: the line hand-off, then the whole
// sweep's objective partials ([T][one per 64 generators]), each block rounded
// up to whole 64-byte lines.
inline int64_t line_scratch_doubles(int64_t B, int64_t T) { return (kLineScratchDoubles * B * T + 7) / 8 * 8; }
inline int64_t obj_scratch_doubles(int64_t G, int64_t T) { return (T * ((G + 63) / 64) + 7) / 8 * 8; }
// Largest block of doubles that a 32-bit byte offset addresses; the kernels
// reach each per-period block of x, c, J, H, K and the line scratch, and
// each per-instance line table, through such an offset from the block base.
constexpr int64_t kMaxBlockDoubles = (int64_t(1) << 29) - 1;

// Slot source codes in the per-period condensed-matrix template.
constexpr int32_t kSrcNone = -2;     // slot filled from the owner's own data
constexpr int32_t kSrcThermal = -1;  // (qf,pf) / (qt,pt) pair of a thermal row

// One instance on the host: copies of the caller's arrays plus derived
// tables.  All indices are 0-based and local to the instance.
struct InstHost {
  int32_t N = 0, B = 0, G = 0, T = 0, ref = 0;
  // per-period sizes (t = 0 layout for the condensed matrix)
  int64_t n_p = 0, m_p = 0, nnzj_p = 0, nnzh_p = 0, nnzk_p = 0;
  // totals of this instance
  int64_t n = 0, m = 0, nnzj = 0, nnzh = 0, nnzk = 0;
  // offsets of this instance in the concatenated arrays
  int64_t x_off = 0, c_off = 0, j_off = 0, h_off = 0, k_off = 0, ld_off = 0;
  int64_t s_off = 0;  // scratch offset (doubles) of the line hand-off
  int64_t o_off = 0;  // scratch offset (doubles) of the objective partials

  std::vector<int32_t> f_bus, t_bus, gen_bus;
  // pi-model admittances, 8 arrays of B: Gff Bff Gft Bft Gtf Btf Gtt Btt
  std::vector<double> adm;
  std::vector<double> c2, c1, c0;
  std::vector<double> pd, qd;  // [T*N]
  std::vector<double> vmin, vmax, pmin, pmax, qmin, qmax, ramp, rate, angmin, angmax;
  // bus incidence, entries (l << 1 | end) sorted by (neighbour bus, l);
  // end 0: the bus is the line's from end, 1: its to end
  std::vector<int32_t> bus_ptr, bus_adj, bus_nb;  // bus_nb: neighbour bus of each entry
  // generators at each bus, ascending
  std::vector<int32_t> bgen_ptr, bgen;
  // condensed-matrix template of one period (t = 0 layout): CSR over the
  // n_p local rows, local column, and per slot the J local index of the
  // partner entry (kSrcNone / kSrcThermal otherwise)
  std::vector<int32_t> krow, kcol, ksrc;
  // per flow row (k * B + l): the kinds of its partner slots (the slots
  // between the four bus-variable slots and the diagonal), packed as
  // (number of leading generator partners) | (thermal slot offset << 16),
  // offset 0xFFFF when the row has no thermal partner
  std::vector<int32_t> kinfo;
};

// Validates the descriptors.  Returns OPF_OK or an error code with a message.
int validate_descs(const opf_instance_desc* desc, int32_t ninst, std::string& err);

// Builds one instance (assumes validate_descs passed).
int build_instance(const opf_instance_desc& d, InstHost& out, std::string& err);

// Assigns concatenation offsets and checks the int32 global index limits.
int assign_offsets(std::vector<InstHost>& insts, std::string& err);

// Global row pointer / column index of K for a host-only model.
void kkt_structure_host(const std::vector<InstHost>& insts, int64_t* rowptr, int32_t* colind);

// Start of period t's block of K inside one instance (the pg rows of periods
// t >= 1 carry one extra leading slot: the (pg_t, pg_{t-1}) ramp pair).
inline int64_t kkt_period_offset(int64_t nnzk_p, int32_t G, int32_t t) {
  return (int64_t)t * nnzk_p + (t >= 1 ? (int64_t)(t - 1) * G : 0);
}

}  // namespace opf
