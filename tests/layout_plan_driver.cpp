// Test driver: the row-packed layout planner (layout_plan.h) behind a C entry
// point that ctypes can call.  Built by tests/test_layout_plan.py with g++.
#include <cstring>

#include "layout_plan.h"

extern "C" {

// Plans the operator with n rows (row pointer rp, columns ci) for K slot groups
// per lane in units of `unit` lanes.  Returns the number of units, or -1 when a
// row needs too many lanes, or -2 when the caller's buffers are too small.  On
// success w0 (units + 1), col and map (units * unit * K slots) and meta
// (units * unit lanes) are filled.
int plan_packed(const int64_t *rp, const int32_t *ci, int32_t n, int K, int unit, int span16, int32_t *w0_out,
                int64_t w0_cap, int32_t *col_out, int32_t *map_out, int64_t slot_cap, uint16_t *meta_out,
                int64_t lane_cap) {
  std::vector<int32_t> lo(n, -1), hi(n, -1);
  for (int32_t r = 0; r < n; r++)
    for (int64_t k = rp[r]; k < rp[r + 1]; k++) {
      if (lo[r] < 0 || ci[k] < lo[r]) lo[r] = ci[k];
      if (ci[k] > hi[r]) hi[r] = ci[k];
    }
  std::vector<int32_t> w0 = aspamg::packed_units(rp, n, K, unit, lo.data(), hi.data(), span16 != 0);
  if (w0.empty()) return -1;
  std::vector<int32_t> col, map;
  std::vector<uint16_t> meta;
  aspamg::packed_slots(rp, ci, K, unit, w0, col, map, meta);
  if ((int64_t)w0.size() > w0_cap || (int64_t)col.size() > slot_cap || (int64_t)meta.size() > lane_cap) return -2;
  std::memcpy(w0_out, w0.data(), w0.size() * sizeof(int32_t));
  std::memcpy(col_out, col.data(), col.size() * sizeof(int32_t));
  std::memcpy(map_out, map.data(), map.size() * sizeof(int32_t));
  std::memcpy(meta_out, meta.data(), meta.size() * sizeof(uint16_t));
  return (int)w0.size() - 1;
}
}

extern "C" {

// Plans the sliced layout with L lanes per row and settles its padding
// columns.  Returns the number of slices, -1 when the slot groups overflow,
// -2 when the caller's buffers are too small.  *nbase receives the number of
// 16-bit column bases (0 when some slice spans more than 65,536 columns).
int plan_sliced(const int64_t *rp, const int32_t *ci, int32_t n, int L, int32_t *sptr_out, int64_t sptr_cap,
                int32_t *col_out, int32_t *map_out, int64_t slot_cap, int32_t *base_out, int32_t *nbase) {
  std::vector<int32_t> sptr = aspamg::sliced_ptr(rp, n, L);
  if (sptr.empty()) return -1;
  std::vector<int32_t> col, map;
  aspamg::sliced_slots(rp, ci, n, L, sptr, col, map);
  const int32_t ns = (int32_t)sptr.size() - 1;
  std::vector<int32_t> base = aspamg::settle_columns(col, ns, [&sptr](int32_t s) { return (int64_t)sptr[s]; });
  if ((int64_t)sptr.size() > sptr_cap || (int64_t)col.size() > slot_cap) return -2;
  std::memcpy(sptr_out, sptr.data(), sptr.size() * sizeof(int32_t));
  std::memcpy(col_out, col.data(), col.size() * sizeof(int32_t));
  std::memcpy(map_out, map.data(), map.size() * sizeof(int32_t));
  std::memcpy(base_out, base.data(), base.size() * sizeof(int32_t));
  *nbase = (int32_t)base.size();
  return ns;
}
}
