// Host planning of the two operator layouts, free of device code: for the
// sliced layout the slot groups of every slice, for the row-packed layout
// which rows form each packing unit and every lane's row and lane count; for
// both, every slot's source block and column, and the per-owner column bases
// of the 16-bit offsets.  The device arrays are built from these vectors
// (api.cpp); the kernels that read them are k_sell_spmv and k_pack_spmv.
#pragma once

#include <algorithm>
#include <cstdint>
#include <functional>
#include <vector>

namespace aspamg {

constexpr int kSell = 64;           // rows per SELL slice = one wavefront

// Slot-group pointers of the sliced layout with L lanes per row (L a power of
// two, 1-64): slice s holds rows s*64/L .. (s+1)*64/L - 1 and as many slot
// groups as its longest row needs (ceil(len / L)).  rp has n + 1 entries.
// Returns the n_slices + 1 pointers, or an empty vector when the slot groups
// would not fit int32 entry indices.
inline std::vector<int32_t> sliced_ptr(const int64_t *rp, int32_t n, int L) {
  const int rps = kSell / L;
  const int32_t ns = (n + rps - 1) / rps;
  std::vector<int32_t> sptr(ns + 1, 0);
  for (int32_t s = 0; s < ns; s++) {
    int64_t w = 0;
    for (int32_t r = s * rps; r < std::min(n, (s + 1) * rps); r++) w = std::max<int64_t>(w, (rp[r + 1] - rp[r] + L - 1) / L);
    if ((int64_t)sptr[s] + w >= (int64_t)INT32_MAX / 64) return {};
    sptr[s + 1] = sptr[s] + (int32_t)w;
  }
  return sptr;
}

// The slots of the sliced layout: entry e of slot group g of slice s belongs
// to row s*64/L + e/L and holds that row's block (g - sptr[s]) L + e % L.
// map[slot] is the source block (index into ci, -1 for padding), col[slot]
// its column (-1 for padding).  The vectors are resized here.
inline void sliced_slots(const int64_t *rp, const int32_t *ci, int32_t n, int L, const std::vector<int32_t> &sptr,
                         std::vector<int32_t> &col, std::vector<int32_t> &map) {
  const int rps = kSell / L;
  const int32_t nslices = (int32_t)sptr.size() - 1;
  col.assign((size_t)sptr.back() * 64, -1);
  map.assign((size_t)sptr.back() * 64, -1);
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t s = 0; s < nslices; s++) {
    for (int32_t g = sptr[s]; g < sptr[s + 1]; g++) {
      for (int e = 0; e < kSell; e++) {
        const int32_t r = s * rps + e / L;
        const int64_t k = (int64_t)(g - sptr[s]) * L + e % L;
        const int64_t len = r < n ? rp[r + 1] - rp[r] : 0;
        const int32_t src = k < len ? (int32_t)(rp[r] + k) : -1;
        map[(size_t)g * 64 + e] = src;
        col[(size_t)g * 64 + e] = src >= 0 ? ci[src] : -1;
      }
    }
  }
}

// Padding entries (column -1 on entry) take the smallest real column of their
// owner (slice or wavefront: entries [first(s)*64, first(s+1)*64)), 0 in an
// owner without real entries; returns the per-owner bases (that smallest
// column) when every owner spans at most 65,536 columns, else empty.
inline std::vector<int32_t> settle_columns(std::vector<int32_t> &col, int32_t nowners,
                                           const std::function<int64_t(int32_t)> &first) {
  std::vector<int32_t> base(nowners, 0);
  bool fits = true;
#pragma omp parallel for schedule(static) reduction(&& : fits)
  for (int32_t s = 0; s < nowners; s++) {
    int32_t lo = INT32_MAX, hi = -1;
    for (int64_t i = first(s) * 64; i < first(s + 1) * 64; i++)
      if (col[i] >= 0) {
        lo = std::min(lo, col[i]);
        hi = std::max(hi, col[i]);
      }
    if (hi < 0) lo = hi = 0;
    for (int64_t i = first(s) * 64; i < first(s + 1) * 64; i++)
      if (col[i] < 0) col[i] = lo;
    base[s] = lo;
    fits = fits && hi - lo <= 65535;
  }
  if (!fits) base.clear();
  return base;
}

// a row's lane count is kept in 8 bits of the lane metadata
constexpr int kPackMaxLanes = 255;

// Rows in matrix order, max(1, ceil(len/K)) lanes each, packed into units of
// `unit` lanes (64: one wavefront; 256: the four of one workgroup), a new unit
// whenever a row does not fit.  In a 256-lane unit a row may cross wavefronts
// (its lanes meet in LDS behind a workgroup barrier), so the unit leaves fewer
// lanes unused than a single wavefront would.  With span16 (every row on its
// own spans at most 65,536 columns; lo / hi are each row's smallest and
// largest column, -1 for an empty row) a new unit also starts where the next
// row would widen the unit's span beyond that, so a jump in the column
// numbering (the seam of a row-stacked operator) does not cost the whole
// operator its 16-bit column offsets.  rp has n + 1 entries.  Returns the
// first row of every unit (plus n at the end), or an empty vector when a row
// needs more than min(unit, kPackMaxLanes) lanes.
inline std::vector<int32_t> packed_units(const int64_t *rp, int32_t n, int K, int unit, const int32_t *lo,
                                         const int32_t *hi, bool span16) {
  std::vector<int32_t> w0;
  const int maxl = std::min(unit, kPackMaxLanes);
  int used = unit;
  int32_t wlo = INT32_MAX, whi = -1;
  for (int32_t r = 0; r < n; r++) {
    const int64_t len = rp[r + 1] - rp[r];
    const int64_t lr = std::max<int64_t>(1, (len + K - 1) / K);
    if (lr > maxl) return {};
    bool fresh = used + lr > unit;
    if (!fresh && span16 && hi[r] >= 0 && whi >= 0)
      fresh = (int64_t)std::max(whi, hi[r]) - std::min(wlo, lo[r]) > 65535;
    if (fresh) {
      w0.push_back(r);
      used = 0;
      wlo = INT32_MAX;
      whi = -1;
    }
    used += (int)lr;
    if (hi[r] >= 0) {
      wlo = std::min(wlo, lo[r]);
      whi = std::max(whi, hi[r]);
    }
  }
  w0.push_back(n);
  return w0;
}

// The slots of the units w0 (packed_units): unit u holds unit / 64 wavefronts
// of K slot groups, and slot group k of wavefront wv holds entry k of lanes
// 64 wv .. 64 wv + 63 of the unit.  Lane j of a row serves the row's blocks
// j K .. j K + K - 1.  map[slot] is the source block (index into ci, -1 for
// padding), col[slot] its column (-1 for padding).  meta[lane] is
// (lane count << 8 | row offset in the unit) on the first lane of a row,
// (row offset) on its other lanes and 0 on unused lanes.  The vectors are
// resized here.
inline void packed_slots(const int64_t *rp, const int32_t *ci, int K, int unit, const std::vector<int32_t> &w0,
                         std::vector<int32_t> &col, std::vector<int32_t> &map, std::vector<uint16_t> &meta) {
  const int kWaves = unit / 64;
  const int32_t nunits = (int32_t)w0.size() - 1;
  const size_t nslots = (size_t)nunits * kWaves * K * 64;
  col.assign(nslots, -1);
  map.assign(nslots, -1);
  meta.assign((size_t)nunits * unit, 0);
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t u = 0; u < nunits; u++) {
    // lane e of unit u serves blocks j K .. j K + K - 1 of row lrow[e]
    int32_t lrow[256], lj[256];
    int e = 0;
    for (int32_t r = w0[u]; r < w0[u + 1]; r++) {
      const int64_t len = rp[r + 1] - rp[r];
      const int lr = (int)std::max<int64_t>(1, (len + K - 1) / K);
      for (int j = 0; j < lr; j++, e++) {
        meta[(size_t)u * unit + e] = (uint16_t)(((j == 0 ? lr : 0) << 8) | (r - w0[u]));
        lrow[e] = r;
        lj[e] = j;
      }
    }
    for (int f = e; f < unit; f++) {
      lrow[f] = -1;
      lj[f] = 0;
    }
    for (int wv = 0; wv < kWaves; wv++)
      for (int k = 0; k < K; k++) {
        const size_t g = ((size_t)u * kWaves + wv) * K + k;
        for (int f = 0; f < 64; f++) {
          const int ln = wv * 64 + f;
          int32_t src = -1;
          if (lrow[ln] >= 0) {
            const int64_t b = (int64_t)lj[ln] * K + k;
            if (b < rp[lrow[ln] + 1] - rp[lrow[ln]]) src = (int32_t)(rp[lrow[ln]] + b);
          }
          map[g * 64 + f] = src;
          col[g * 64 + f] = src >= 0 ? ci[src] : -1;
        }
      }
  }
}

}  // namespace aspamg
