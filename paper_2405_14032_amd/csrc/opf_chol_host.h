// Host-side plan of the static-pivot sparse Cholesky factorization of the
// condensed matrix (one plan per instance; every period shares it).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "opf_host.h"

namespace opf {

struct CholOptions {
  int32_t small_max = 64;     // fronts of at most this order are factored in LDS
  int32_t amalg_small = 16;   // merged pivot blocks up to this size: relaxed merge
  double amalg_frac = 0.05;   // otherwise merge while its zeros <= frac of the front
  int32_t max_pivots = 4096;  // no merge beyond this many pivots
  int32_t col_block = 32;     // columns per extend-add work item
};

// Local indices: "old" = position in the period block of x (the canonical
// layout), "new" = position in the elimination order.  The interior
// occupies new indices [0, n_int), the pg variables [n_int, n_p) in their
// natural order.
struct CholPlan {
  int32_t n_p = 0, n_int = 0, G = 0, T = 0;
  std::vector<int32_t> perm, iperm;  // new -> old, old -> new
  // interior nodes in postorder: first pivot, pivot count, update-row count,
  // parent (-1: the period's pg front)
  int32_t nnodes = 0, nlevels = 0;
  std::vector<int32_t> node_f, node_p, node_u, node_parent, node_level;
  std::vector<int64_t> row_ptr;   // [nnodes + 1] into rows / rel
  std::vector<int32_t> rows;      // update rows (new indices, ascending)
  std::vector<int32_t> rel;       // their positions in the parent's front
  std::vector<int64_t> kid_ptr;   // [nnodes + 1]
  std::vector<int32_t> kids;      // children, ascending
  std::vector<int32_t> roots;     // nodes whose parent is the pg front
  // per-period storage: interior factor (node blocks) and update arena
  std::vector<int64_t> node_loff, node_uoff;
  int64_t lsize = 0, usize = 0;
  // level schedule
  std::vector<int32_t> lvl_small, lvl_large;
  std::vector<int64_t> lvl_small_ptr, lvl_large_ptr;
  std::vector<int32_t> items;        // (node, first column) pairs
  std::vector<int64_t> lvl_items_ptr;
  std::vector<int32_t> root_items;   // first columns of the pg front's items
  // K template slot -> destination (see chol_plan_build), K positions
  std::vector<int64_t> slot_dst;
  std::vector<int32_t> kpos0, kpos1, ramp_pos;
  double flops_period = 0.0, flops_chain = 0.0;
};

int chol_plan_build(const InstHost& I, const CholOptions& opt, CholPlan& P, std::string& err);

}  // namespace opf
