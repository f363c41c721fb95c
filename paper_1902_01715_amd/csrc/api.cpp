// C ABI of the aSP-AMG library: handle lifetime, device layouts, the
// V(nu1,nu2)-cycle driver and the PCG driver (one iteration captured as a HIP
// graph and replayed, with a device-side control block deciding convergence).
#include <type_traits>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>

#include "internal.h"

// sizes mirrored by the Python binding
static_assert(sizeof(aspamg_params) == 160, "aspamg_params layout changed");
static_assert(sizeof(aspamg_stats) == 104, "aspamg_stats layout changed");
static_assert(sizeof(aspamg_level_info_t) == 200, "aspamg_level_info_t layout changed");

namespace aspamg {

static thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }

void fail(aspamg_status code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(ASPAMG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void *dmalloc(aspamg_ctx *h, size_t bytes) {
  void *p = nullptr;
  if (bytes == 0) bytes = 16;
  if (hipMalloc(&p, bytes) != hipSuccess) fail(ASPAMG_ENOMEM, "device allocation failed");
  h->allocations.push_back(p);
  return p;
}

HostBSR transpose(const HostBSR &M) {
  HostBSR T;
  T.n = M.nc;
  T.nc = M.n;
  T.b = M.b;
  T.rp.assign(T.n + 1, 0);
  const int64_t nnz = M.nnzb();
  for (int64_t k = 0; k < nnz; k++) T.rp[M.ci[k] + 1]++;
  for (int32_t i = 0; i < T.n; i++) T.rp[i + 1] += T.rp[i];
  T.ci.resize(nnz);
  std::vector<int64_t> src(nnz);
  std::vector<int64_t> pos(T.rp.begin(), T.rp.end() - 1);
  for (int32_t i = 0; i < M.n; i++)
    for (int64_t k = M.rp[i]; k < M.rp[i + 1]; k++) {
      const int64_t q = pos[M.ci[k]]++;
      T.ci[q] = i;
      src[q] = k;
    }
  const int b = M.b, bb = b * b;
  T.v.resize((size_t)nnz * bb);
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < nnz; q++)
    for (int d = 0; d < b; d++)
      for (int e = 0; e < b; e++) T.v[(size_t)q * bb + e * b + d] = M.v[(size_t)src[q] * bb + d * b + e];
  return T;
}

// slot groups of the sliced layout with L lanes per row
static std::vector<int32_t> sliced_ptr(const HostBSR &M, int L) {
  std::vector<int32_t> sptr = sliced_ptr(M.rp.data(), M.n, L);
  if (sptr.empty()) fail(ASPAMG_EINVAL, "operator too large for the sliced layout");
  return sptr;
}

// Smallest and largest column of every row (-1, -1 for an empty row).
static void row_spans(const HostBSR &M, std::vector<int32_t> &lo, std::vector<int32_t> &hi) {
  lo.assign(M.n, -1);
  hi.assign(M.n, -1);
#pragma omp parallel for schedule(static)
  for (int32_t r = 0; r < M.n; r++)
    for (int64_t k = M.rp[r]; k < M.rp[r + 1]; k++) {
      const int32_t c = M.ci[k];
      if (lo[r] < 0 || c < lo[r]) lo[r] = c;
      if (c > hi[r]) hi[r] = c;
    }
}

// One candidate layout of an operator on the device: its index arrays (in a
// Sell whose values are not set) and the per-slot source map that scatters
// the operator's block values into any precision's copy.
struct Candidate {
  Sell<double> idx;
  int32_t *map = nullptr;
  int64_t nslots = 0;
};

// Device index arrays of a layout: slice/unit pointers, columns (16-bit
// offsets when `base` is not empty), the lane metadata of the row-packed
// layout, and the per-slot source map.
static Candidate upload_index(aspamg_ctx *h, const Sell<double> &shape, const std::vector<int32_t> &sptr,
                              const std::vector<int32_t> &col, const std::vector<int32_t> &base,
                              const std::vector<int32_t> &map, const std::vector<uint16_t> &meta) {
  Candidate c;
  c.idx = shape;
  Sell<double> &S = c.idx;
  S.sptr = dalloc<int32_t>(h, sptr.size());
  HIPCHK(hipMemcpyAsync(S.sptr, sptr.data(), sptr.size() * 4, hipMemcpyHostToDevice, h->stream));
  std::vector<uint16_t> c16;
  if (!base.empty()) {
    // owner of slot group g: the slice (sliced) or wavefront (row-packed) it belongs to
    c16.resize(col.size());
    const int32_t nowners = (int32_t)base.size();
#pragma omp parallel for schedule(static)
    for (int32_t s = 0; s < nowners; s++) {
      const int64_t g0 = S.pack ? (int64_t)s * S.pack : sptr[s];
      const int64_t g1 = S.pack ? (int64_t)(s + 1) * S.pack : sptr[s + 1];
      for (int64_t i = g0 * 64; i < g1 * 64; i++) c16[i] = (uint16_t)(col[i] - base[s]);
    }
    S.col16 = dalloc<uint16_t>(h, c16.size());
    S.cbase = dalloc<int32_t>(h, base.size());
    HIPCHK(hipMemcpyAsync(S.col16, c16.data(), c16.size() * 2, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(S.cbase, base.data(), base.size() * 4, hipMemcpyHostToDevice, h->stream));
  } else {
    S.col = dalloc<int32_t>(h, col.size());
    HIPCHK(hipMemcpyAsync(S.col, col.data(), col.size() * 4, hipMemcpyHostToDevice, h->stream));
  }
  if (!meta.empty()) {
    S.meta = dalloc<uint16_t>(h, meta.size());
    HIPCHK(hipMemcpyAsync(S.meta, meta.data(), meta.size() * 2, hipMemcpyHostToDevice, h->stream));
  }
  c.nslots = (int64_t)map.size();
  c.map = dalloc<int32_t>(h, std::max<size_t>(map.size(), 1));
  HIPCHK(hipMemcpyAsync(c.map, map.data(), map.size() * 4, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));   // the host arrays go out of scope
  return c;
}

// A Sell<T> with the layout fields and index arrays of S (shared, not copied)
// and no values.
template <typename T, typename U>
static Sell<T> same_index(const Sell<U> &S) {
  Sell<T> F;
  F.n = S.n;
  F.nc = S.nc;
  F.b = S.b;
  F.nslices = S.nslices;
  F.lanes = S.lanes;
  F.pack = S.pack;
  F.unit = S.unit;
  F.ngroups = S.ngroups;
  F.nnzb = S.nnzb;
  F.sptr = S.sptr;
  F.col = S.col;
  F.col16 = S.col16;
  F.cbase = S.cbase;
  F.meta = S.meta;
  return F;
}

// The candidate's copy in precision T: its index arrays, and values scattered
// from the operator's block values dv (device copy).
template <typename T>
static Sell<T> with_values(aspamg_ctx *h, const Candidate &c, const double *dv) {
  Sell<T> S = same_index<T>(c.idx);
  S.val = dalloc<T>(h, (size_t)std::max<int64_t>(S.values(), 1));
  launch_scatter_values<T>(c.nslots, c.map, dv, S.val, S.b, h->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return S;
}

static void free_index(aspamg_ctx *h, Candidate &c) {
  dfree(h, c.idx.sptr);
  dfree(h, c.idx.col);
  dfree(h, c.idx.col16);
  dfree(h, c.idx.cbase);
  dfree(h, c.idx.meta);
  c.idx = Sell<double>();
}

static Candidate packed_layout(aspamg_ctx *h, const HostBSR &M, int K, int unit, const std::vector<int32_t> &w0) {
  Sell<double> S;
  S.n = M.n;
  S.nc = M.nc;
  S.b = M.b;
  S.nnzb = M.nnzb();
  S.lanes = 0;
  S.pack = K;
  S.unit = unit;
  S.nslices = ((int32_t)w0.size() - 1) * (unit / 64);
  S.ngroups = (int64_t)S.nslices * K;
  std::vector<int32_t> col, map;
  std::vector<uint16_t> meta;
  packed_slots(M.rp.data(), M.ci.data(), K, unit, w0, col, map, meta);
  const int64_t Kp = K;
  std::vector<int32_t> base = settle_columns(col, S.nslices, [Kp](int32_t s) { return (int64_t)s * Kp; });
  return upload_index(h, S, w0, col, base, map, meta);
}

#ifndef ASPAMG_SCALAR_MIN_PACK
#define ASPAMG_SCALAR_MIN_PACK 4
#endif
constexpr int kScalarMinPack = ASPAMG_SCALAR_MIN_PACK;   // slot groups per lane, scalar row-packed

// Lanes per row of the sliced copy: force_lanes, or the smallest L that keeps
// kMinThreads lanes busy and then the L (up to 64) with the fewest padded
// slots, a larger L having to save at least 5%.  Returns L; *sptr receives
// the slice pointers.
static int sliced_plan(const HostBSR &M, int force_lanes, std::vector<int32_t> *sptr) {
  if (force_lanes) {
    *sptr = sliced_ptr(M, force_lanes);
    return force_lanes;
  }
  int L0 = 1, L = 1;
  while (L0 < 64 && (int64_t)M.n * L0 < kMinThreads) L0 *= 2;
  int64_t best = -1;
  for (int c = L0; c <= 64; c *= 2) {
    std::vector<int32_t> sp = sliced_ptr(M, c);
    const int64_t slots = (int64_t)sp.back() * 64;
    if (best < 0 || (double)slots < 0.95 * (double)best) {
      best = slots;
      L = c;
      sptr->swap(sp);
    }
  }
  return L;
}

static Candidate sliced_layout(aspamg_ctx *h, const HostBSR &M, int L, const std::vector<int32_t> &sptr) {
  Sell<double> S;
  S.n = M.n;
  S.nc = M.nc;
  S.b = M.b;
  S.nnzb = M.nnzb();
  S.lanes = L;
  S.nslices = (int32_t)sptr.size() - 1;
  S.ngroups = sptr.back();
  std::vector<int32_t> col, map;
  sliced_slots(M.rp.data(), M.ci.data(), M.n, L, sptr, col, map);
  std::vector<int32_t> base = settle_columns(col, S.nslices, [&sptr](int32_t s) { return (int64_t)sptr[s]; });
  return upload_index(h, S, sptr, col, base, map, {});
}

void dfree(aspamg_ctx *h, void *p) {
  if (!p) return;
  auto it = std::find(h->allocations.begin(), h->allocations.end(), p);
  if (it != h->allocations.end()) h->allocations.erase(it);
  (void)hipFree(p);
}

template <typename T>
void free_sell(aspamg_ctx *h, Sell<T> &S) {
  if (S.own_index) {
    dfree(h, S.sptr);
    dfree(h, S.col);
    dfree(h, S.col16);
    dfree(h, S.cbase);
    dfree(h, S.meta);
  }
  dfree(h, S.val);
  S = Sell<T>();
}

// Median launch times of y = C x for each candidate layout C over 7 rounds in
// which the candidates take turns (after one warm-up launch each), on the
// handle's stream.
template <typename T>
static std::vector<float> time_layouts(aspamg_ctx *h, const std::vector<Sell<T>> &C, const T *x, T *y) {
  const size_t n = C.size();
  constexpr int kReps = 7;
  std::vector<hipEvent_t> e(n + 1, nullptr);
  for (auto &ev : e) HIPCHK(hipEventCreate(&ev));
  std::vector<std::vector<float>> t(n, std::vector<float>(kReps, 0.f));
  try {
    for (const Sell<T> &c : C) launch_spmv<T, T, T>(c, x, y, nullptr, 1.0, nullptr, h->stream);
    for (int i = 0; i < kReps; i++) {
      HIPCHK(hipEventRecord(e[0], h->stream));
      for (size_t j = 0; j < n; j++) {
        launch_spmv<T, T, T>(C[j], x, y, nullptr, 1.0, nullptr, h->stream);
        HIPCHK(hipEventRecord(e[j + 1], h->stream));
      }
      HIPCHK(hipEventSynchronize(e[n]));
      for (size_t j = 0; j < n; j++) HIPCHK(hipEventElapsedTime(&t[j][i], e[j], e[j + 1]));
    }
  } catch (...) {
    for (auto &ev : e) (void)hipEventDestroy(ev);
    throw;
  }
  for (auto &ev : e) (void)hipEventDestroy(ev);
  std::vector<float> med(n);
  for (size_t j = 0; j < n; j++) {
    std::sort(t[j].begin(), t[j].end());
    med[j] = t[j][kReps / 2];
  }
  return med;
}

// Candidate layouts of M for the products of the solve phase, the sliced one
// first.  With force_lanes the sliced layout with that many lanes per row.
// Otherwise, for the timed choice, the sliced layout and the row-packed ones
// with units of one wavefront and of one workgroup, each with its K of fewest
// slots and every other K that stores at most 10% more, those storing at most
// 1.5 times the sliced slots; each precision's copy then times them on the
// device (keep_fastest).  Operators under kTimedSlots slots, or all of them
// without `timed`, get one layout: the wavefront-unit packing unless the
// workgroup unit stores 10% fewer slots, kept when it stores 10% fewer slots
// than the sliced layout.  Policy 2 forces the sliced layout, 3 and 4 the
// row-packed one with units of a workgroup and of a wavefront (sliced where a
// row needs more lanes than a unit holds).
static std::vector<Candidate> candidates(aspamg_ctx *h, const HostBSR &M, int force_lanes, bool timed) {
  const int policy = h->p.layout;
  if (M.nnzb() >= (int64_t)INT32_MAX) fail(ASPAMG_EINVAL, "operator too large for int32 block indices");
  std::vector<int32_t> sptr;
  const int L = sliced_plan(M, force_lanes, &sptr);
  std::vector<Candidate> C;
  if (force_lanes || M.n == 0 || M.nc == 0 || policy == 2) {
    C.push_back(sliced_layout(h, M, L, sptr));
    return C;
  }
  if (policy != 0) timed = false;
  struct Plan {
    int K = 0, unit = 0;
    int64_t slots = 0;
    std::vector<int32_t> w0;
  };
  // per unit (64, 256) and K (1, 2, 4, 8): the row-packed plan, K = 0 where a
  // row needs more lanes than the unit holds
  Plan all[2][4];
  std::vector<int32_t> lo, hi;
  row_spans(M, lo, hi);
  bool span16 = true;
  for (int32_t r = 0; r < M.n && span16; r++) span16 = hi[r] - lo[r] <= 65535;
  const int units[2] = {64, 256}, ks[4] = {1, 2, 4, 8};
  for (int u = 0; u < 2; u++)
    for (int i = 0; i < 4; i++) {
      // a scalar slot is one value: with fewer than kScalarMinPack per lane the
      // lane's share of a row is dominated by the in-row reduction
      if (M.b == 1 && ks[i] < kScalarMinPack) continue;
      std::vector<int32_t> w0 = packed_units(M.rp.data(), M.n, ks[i], units[u], lo.data(), hi.data(), span16);
      if (w0.empty()) continue;
      Plan &q = all[u][i];
      q.K = ks[i];
      q.unit = units[u];
      q.slots = (int64_t)(w0.size() - 1) * units[u] * ks[i];
      q.w0.swap(w0);
    }
  // pk[u]: the plan of fewest slots in unit u; alt[u]: the other K that store at
  // most 10% more slots (a smaller K gives a row more lanes and each lane a
  // shorter chain, a larger one each lane more work per row sum)
  Plan pk[2];
  std::vector<Plan> alt[2];
  for (int u = 0; u < 2; u++) {
    int bi = -1;
    for (int i = 0; i < 4; i++)
      if (all[u][i].K && (bi < 0 || all[u][i].slots < all[u][bi].slots)) bi = i;
    if (bi < 0) continue;
    for (int i = 0; i < 4; i++)
      if (i != bi && all[u][i].K && (double)all[u][i].slots <= 1.1 * (double)all[u][bi].slots)
        alt[u].push_back(std::move(all[u][i]));
    pk[u] = std::move(all[u][bi]);
  }
  auto packed = [&](const Plan &q) { C.push_back(packed_layout(h, M, q.K, q.unit, q.w0)); };
  if (policy == 3 || policy == 4) {
    const Plan &q = pk[policy == 3 ? 1 : 0];
    if (q.K) packed(q);
    else C.push_back(sliced_layout(h, M, L, sptr));
    return C;
  }
  // untimed choice: the wavefront unit unless the workgroup unit stores 10%
  // fewer slots (its barrier costs the most where the product is short)
  const Plan *best = pk[0].K ? &pk[0] : nullptr;
  if (pk[1].K && (!best || (double)pk[1].slots < 0.9 * (double)best->slots)) best = &pk[1];
  const int64_t sliced = (int64_t)sptr.back() * 64;
  if (!best) {                    // a row needs more than kPackMaxLanes lanes
    C.push_back(sliced_layout(h, M, L, sptr));
    return C;
  }
  // small operators sit at the launch-latency floor either way: no timing
  const int64_t fewest = pk[0].K && pk[1].K ? std::min(pk[0].slots, pk[1].slots) : best->slots;
  if (!timed || std::max<int64_t>(fewest, sliced) < kTimedSlots) {
    if ((double)best->slots >= 0.9 * (double)sliced) C.push_back(sliced_layout(h, M, L, sptr));
    else packed(*best);
    return C;
  }
  C.push_back(sliced_layout(h, M, L, sptr));
  for (int u = 0; u < 2; u++) {
    if (pk[u].K && (double)pk[u].slots <= 1.5 * (double)sliced) packed(pk[u]);
    for (const Plan &q : alt[u])
      if ((double)q.slots <= 1.5 * (double)sliced) packed(q);
  }
  return C;
}

// The block values of M on the device: dvals when given, else uploaded here
// (and freed with this object).
struct DeviceValues {
  aspamg_ctx *h;
  double *v;
  bool own;
  DeviceValues(aspamg_ctx *hh, const HostBSR &M, const double *dvals)
      : h(hh), v(const_cast<double *>(dvals)), own(dvals == nullptr) {
    if (own) {
      v = dalloc<double>(h, std::max<size_t>(M.v.size(), 1));
      if (!M.v.empty()) HIPCHK(hipMemcpyAsync(v, M.v.data(), M.v.size() * 8, hipMemcpyHostToDevice, h->stream));
    }
  }
  ~DeviceValues() {
    if (own) dfree(h, v);
  }
  DeviceValues(const DeviceValues &) = delete;
  DeviceValues &operator=(const DeviceValues &) = delete;
};

// The copies of every candidate in precision T; with more than one, each is
// timed on the device (7 rounds of turns, medians) and the fastest kept, a
// row-packed one having to beat the sliced one (first) by 5%.  The values of
// the others are freed; returns the kept copy, its candidate's index in *picked.
template <typename T>
static Sell<T> keep_fastest(aspamg_ctx *h, const HostBSR &M, const std::vector<Candidate> &C, const double *dv,
                            size_t *picked) {
  std::vector<Sell<T>> v;
  for (const Candidate &c : C) v.push_back(with_values<T>(h, c, dv));
  size_t pick = 0;
  if (v.size() > 1) {
    const size_t nx = (size_t)M.b * std::max<int32_t>(M.nc, 1), ny = (size_t)M.b * std::max<int32_t>(M.n, 1);
    T *x = nullptr, *y = nullptr;
    HIPCHK(hipMalloc(&x, sizeof(T) * nx));
    HIPCHK(hipMalloc(&y, sizeof(T) * ny));
    std::vector<float> t;
    try {
      HIPCHK(hipMemsetAsync(x, 0, sizeof(T) * nx, h->stream));
      t = time_layouts(h, v, x, y);
    } catch (...) {
      (void)hipFree(x);
      (void)hipFree(y);
      throw;
    }
    (void)hipFree(x);
    (void)hipFree(y);
    for (size_t j = 1; j < v.size(); j++)
      if (t[j] < 0.95f * t[0] && (pick == 0 || t[j] < t[pick])) pick = j;
  }
  for (size_t j = 0; j < v.size(); j++)
    if (j != pick) dfree(h, v[j].val);
  *picked = pick;
  return v[pick];
}

// Device copy of M used by the products of the solve phase, in precision T,
// in the layout chosen among candidates() (timed in T where there are several).
template <typename T>
Sell<T> upload_sell(aspamg_ctx *h, const HostBSR &M, int force_lanes, bool timed, const double *dvals) {
  DeviceValues dv(h, M, dvals);
  std::vector<Candidate> C = candidates(h, M, force_lanes, timed);
  size_t pick = 0;
  Sell<T> S = keep_fastest<T>(h, M, C, dv.v, &pick);
  for (size_t j = 0; j < C.size(); j++) {
    dfree(h, C[j].map);
    if (j != pick) free_index(h, C[j]);
  }
  return S;
}

// The FP64 and FP32 copies of M, each in the layout timed in its own
// precision.  The candidates' index arrays are built once for both; when the
// two copies pick the same candidate, the FP32 copy shares the FP64 copy's
// index arrays.
void upload_sell_pair(aspamg_ctx *h, const HostBSR &M, const double *dvals, Sell<double> &d64, Sell<float> &d32) {
  DeviceValues dv(h, M, dvals);
  std::vector<Candidate> C = candidates(h, M, 0, true);
  size_t p64 = 0, p32 = 0;
  d64 = keep_fastest<double>(h, M, C, dv.v, &p64);
  d32 = keep_fastest<float>(h, M, C, dv.v, &p32);
  d32.own_index = p32 != p64;
  for (size_t j = 0; j < C.size(); j++) {
    dfree(h, C[j].map);
    if (j != p64 && j != p32) free_index(h, C[j]);
  }
}

// FP32 copy of S in the same layout: the index arrays are shared with S (the
// copy does not own them), the values converted on the device.
Sell<float> derive_fp32(aspamg_ctx *h, const Sell<double> &S) {
  Sell<float> F = same_index<float>(S);
  F.own_index = false;
  const int64_t nv = S.values();
  F.val = dalloc<float>(h, (size_t)std::max<int64_t>(nv, 1));
  if (nv > 0) launch_narrow_values(S.ngroups * 64, S.val, F.val, S.b, h->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return F;
}

template Sell<double> upload_sell<double>(aspamg_ctx *, const HostBSR &, int, bool, const double *);
template Sell<float> upload_sell<float>(aspamg_ctx *, const HostBSR &, int, bool, const double *);
template void free_sell<double>(aspamg_ctx *, Sell<double> &);
template void free_sell<float>(aspamg_ctx *, Sell<float> &);

DevBSR upload_bsr(aspamg_ctx *h, const HostBSR &M) {
  DevBSR d;
  d.n = M.n;
  d.nc = M.nc;
  d.b = M.b;
  d.nnzb = M.nnzb();
  if (d.nnzb >= (int64_t)INT32_MAX) fail(ASPAMG_EINVAL, "operator too large for int32 block indices");
  std::vector<int32_t> rp32(M.rp.begin(), M.rp.end());
  d.rp = dalloc<int32_t>(h, rp32.size());
  d.ci = dalloc<int32_t>(h, std::max<size_t>(M.ci.size(), 1));
  d.v = dalloc<double>(h, std::max<size_t>(M.v.size(), 1));
  HIPCHK(hipMemcpyAsync(d.rp, rp32.data(), rp32.size() * 4, hipMemcpyHostToDevice, h->stream));
  if (!M.ci.empty()) HIPCHK(hipMemcpyAsync(d.ci, M.ci.data(), M.ci.size() * 4, hipMemcpyHostToDevice, h->stream));
  if (!M.v.empty()) HIPCHK(hipMemcpyAsync(d.v, M.v.data(), M.v.size() * 8, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return d;
}

// ---------------------------------------------------------------------------
// V(nu1, nu2)-cycle (Algorithm "AMG application in a V-cycle").  With the
// symmetric smoother M^{-1} = omega G^T G:
//   s = omega G^T G y                       (pre-smoothing from 0)
//   s += omega G^T G (y - A s)              (further pre-smoothing steps)
//   r = y - A s ; r_c = R r ; h_c = cycle(r_c) ; s += P h_c
//   s += omega G^T G (y - A s)              (nu2 post-smoothing steps)
// The first post-smoothing residual is formed as r - (A P) h_c, together with
// s + P h_c, by one product with the stacked operator [P; A P].  The coarsest
// level applies A_L^{-1} from its Cholesky factor.
// ---------------------------------------------------------------------------
template <typename T>
struct Ops;
template <>
struct Ops<double> {
  static const Sell<double> &A(const Level &L) { return L.A64; }
  static const Sell<double> &G(const Level &L) { return L.G64; }
  static const Sell<double> &GT(const Level &L) { return L.GT64; }
  static const Sell<double> &P(const Level &L) { return L.P64; }
  static const Sell<double> &R(const Level &L) { return L.R64; }
  static const Sell<double> &PAP(const Level &L) { return L.PAP64; }
  static const Sell<double> &M(const Level &L) { return L.M64; }
  static const LevelVecs<double> &V(const Level &L) { return L.v64; }
};
template <>
struct Ops<float> {
  static const Sell<float> &A(const Level &L) { return L.A32; }
  static const Sell<float> &G(const Level &L) { return L.G32; }
  static const Sell<float> &GT(const Level &L) { return L.GT32; }
  static const Sell<float> &P(const Level &L) { return L.P32; }
  static const Sell<float> &R(const Level &L) { return L.R32; }
  static const Sell<float> &PAP(const Level &L) { return L.PAP32; }
  static const Sell<float> &M(const Level &L) { return L.M32; }
  static const LevelVecs<float> &V(const Level &L) { return L.v32; }
};

template <typename T>
static void cycle_level(aspamg_ctx *h, int l, const T *y, T *z, const PcgCtrl *ctrl) {
  const Level &L = h->lev[l];
  hipStream_t s = h->stream;
  if (l == h->tail.level) {
    launch_dense_gemv<T>(h->tail.nd, h->tail.v, y, z, ctrl, s);
    return;
  }
  if (L.coarsest) {
    launch_dense_gemv<T>(h->coarse.nd, h->coarse.inv, y, z, ctrl, s);
    return;
  }
  using O = Ops<T>;
  const LevelVecs<T> &W = O::V(L);
  const LevelVecs<T> &Wn = O::V(h->lev[l + 1]);
  const double w = L.omega_s;
  // z = w G^T G x (+ z).  The FP32 cycle uses the merged M on small levels:
  // one launch, and one rounding of the FP64 product G^T G instead of an FP32
  // intermediate G x (the FP64 cycle keeps G and G^T, whose two launches cost
  // no more than M's larger FP64 copy there)
  constexpr bool kMergedFp32 = std::is_same<T, float>::value;
  const bool merged = kMergedFp32 && L.nnzb_M > 0;
  auto smooth = [&](const T *x, const T *add) {
    if (merged) {
      launch_spmv<T, T, T>(O::M(L), x, z, add, w, ctrl, s);
    } else {
      launch_spmv<T, T, T>(O::G(L), x, W.t, nullptr, 1.0, ctrl, s);
      launch_spmv<T, T, T>(O::GT(L), W.t, z, add, w, ctrl, s);
    }
  };
  for (int it = 0; it < h->p.nu1; it++) {
    if (it == 0) {
      smooth(y, nullptr);
    } else {
      launch_spmv<T, T, T>(O::A(L), z, W.r, y, -1.0, ctrl, s);
      smooth(W.r, z);
    }
  }
  launch_spmv<T, T, T>(O::A(L), z, W.r, y, -1.0, ctrl, s);
  launch_spmv<T, T, T>(O::R(L), W.r, Wn.y, nullptr, 1.0, ctrl, s);
  cycle_level<T>(h, l + 1, Wn.y, Wn.z, ctrl);
  // first post-smoothing step (nu2 >= 1): z += P e and r = (y - A z_pre) - (A P) e
  // in one stacked product (W.r still holds the pre-smoothing residual), or
  // z += P e and then r = y - A z
  if (L.stacked()) {
    launch_spmv_dual<T, T, T>(O::PAP(L), L.P.n, Wn.z, z, z, 1.0, W.r, W.r, -1.0, ctrl, s);
  } else {
    launch_spmv<T, T, T>(O::P(L), Wn.z, z, z, 1.0, ctrl, s);
    launch_spmv<T, T, T>(O::A(L), z, W.r, y, -1.0, ctrl, s);
  }
  for (int it = 0; it < h->p.nu2; it++) {
    if (it > 0) launch_spmv<T, T, T>(O::A(L), z, W.r, y, -1.0, ctrl, s);
    smooth(W.r, z);
  }
}

// The same cycle in FP64 on the nb columns of a row-major multi-vector
// ([3 n_l][nb]), with plain block-CSR products: forms the dense tail operator.
struct ColumnLevel {
  DevBSR A, G, GT, P, R;
  double *y = nullptr, *z = nullptr, *r = nullptr, *t = nullptr;
};

static void cycle_columns(aspamg_ctx *h, std::vector<ColumnLevel> &C, int l0, int l, const double *y, double *z,
                          int32_t nb) {
  const Level &L = h->lev[l];
  hipStream_t s = h->stream;
  if (L.coarsest) {
    launch_dense_mm(h->coarse.nd, h->coarse.inv, y, z, nb, s);
    return;
  }
  ColumnLevel &W = C[l - l0], &Wn = C[l + 1 - l0];
  const double w = L.omega_s;
  for (int it = 0; it < h->p.nu1; it++) {
    if (it == 0) {
      launch_bsr_mm(W.G, y, W.t, nullptr, 1.0, nb, s);
      launch_bsr_mm(W.GT, W.t, z, nullptr, w, nb, s);
    } else {
      launch_bsr_mm(W.A, z, W.r, y, -1.0, nb, s);
      launch_bsr_mm(W.G, W.r, W.t, nullptr, 1.0, nb, s);
      launch_bsr_mm(W.GT, W.t, z, z, w, nb, s);
    }
  }
  launch_bsr_mm(W.A, z, W.r, y, -1.0, nb, s);
  launch_bsr_mm(W.R, W.r, Wn.y, nullptr, 1.0, nb, s);
  cycle_columns(h, C, l0, l + 1, Wn.y, Wn.z, nb);
  launch_bsr_mm(W.P, Wn.z, z, z, 1.0, nb, s);
  for (int it = 0; it < h->p.nu2; it++) {
    launch_bsr_mm(W.A, z, W.r, y, -1.0, nb, s);
    launch_bsr_mm(W.G, W.r, W.t, nullptr, 1.0, nb, s);
    launch_bsr_mm(W.GT, W.t, z, z, w, nb, s);
  }
}

// Dense tail: the highest level t above the coarsest such that every level
// from t down has at most dense_tail_dof unknowns.  Its cycle maps y to z
// linearly; applying it to the columns of the identity gives that operator's
// columns, stored row by row (column c of the result is V e_c, so row r of
// the row-major result is row r of V).  The cycle then reads one dense FP64
// matrix at level t in place of the launches of levels t and below, each of
// which costs a dependent round trip on these small levels.
static void build_tail(aspamg_ctx *h) {
  const int lc = (int)h->lev.size() - 1;
  if (h->p.dense_tail_dof <= 0 || lc < 1) return;
  int t = lc;
  while (t > 0 && (int64_t)h->b * h->lev[t - 1].A.n <= h->p.dense_tail_dof) t--;
  if (t == lc) return;
  const int32_t nd = h->b * h->lev[t].A.n;
  std::vector<ColumnLevel> C(lc - t + 1);
  std::vector<void *> tmp;
  auto vec = [&](int32_t rows) {
    double *p = dalloc<double>(h, (size_t)rows * nd);
    tmp.push_back(p);
    return p;
  };
  auto keep = [&](const DevBSR &d) {
    tmp.push_back(d.rp);
    tmp.push_back(d.ci);
    tmp.push_back(d.v);
  };
  for (int l = t; l <= lc; l++) {
    const Level &L = h->lev[l];
    ColumnLevel &W = C[l - t];
    const int32_t rows = h->b * L.A.n;
    W.y = vec(rows);
    W.z = vec(rows);
    if (L.coarsest) continue;
    W.r = vec(rows);
    W.t = vec(rows);
    W.A = upload_bsr(h, L.A);
    W.G = upload_bsr(h, L.G);
    W.GT = upload_bsr(h, transpose(L.G));
    W.P = upload_bsr(h, L.P);
    W.R = upload_bsr(h, transpose(L.P));
    for (const DevBSR *d : {&W.A, &W.G, &W.GT, &W.P, &W.R}) keep(*d);
  }
  h->tail.v = dalloc<double>(h, (size_t)nd * nd);
  launch_eye(nd, C[0].y, h->stream);
  cycle_columns(h, C, t, t, C[0].y, h->tail.v, nd);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  for (void *p : tmp) dfree(h, p);
  h->tail.level = t;
  h->tail.nd = nd;
}

// z = M^{-1} r for FP64 vectors r, z of the fine level
static void precondition(aspamg_ctx *h, const double *r, double *z, const PcgCtrl *ctrl, bool fp32) {
  const int64_t n = (int64_t)h->n * h->b;
  if (fp32) {
    const Level &L0 = h->lev[0];
    launch_cast<double, float>(n, r, L0.v32.y, ctrl, h->stream);
    cycle_level<float>(h, 0, L0.v32.y, L0.v32.z, ctrl);
    launch_cast<float, double>(n, L0.v32.z, z, ctrl, h->stream);
  } else {
    cycle_level<double>(h, 0, r, z, ctrl);
  }
}

// One PCG iteration (Section 4; beta in the Polak-Ribiere form
// (r_{k+1}.z_{k+1} - r_{k+1}.z_k) / (r_k.z_k)).  After convergence the kernels
// that write u, r, p and the scalars are no-ops; the V-cycle kernels do not
// read the flag (a dependent load at the head of each of their ~40 launches)
// and recompute a z that no live kernel reads, for at most the rest of one
// host polling window.
static void pcg_iteration(aspamg_ctx *h, bool fp32) {
  hipStream_t s = h->stream;
  const int64_t n = (int64_t)h->n * h->b;
  const Level &L0 = h->lev[0];
  PcgCtrl *c = h->ctrl;
  // partial regions: [0] p.q, [1] r.r and [2] r.z_old (update), [3] r.z
  double *pq_part = h->part, *rr_part = h->part + kMaxPart, *rz_part = h->part + 3 * kMaxPart;
  launch_spmv_dot(L0.A64, h->vp, h->vq, pq_part, c, s);
  const int nv = vec_blocks(n);
  if (fp32) {
    // z (and z_old) stay in FP32: the update, r.z and p = z + beta p read them as they are
    launch_pcg_update<float>(n, h->vu, h->vr, h->vp, h->vq, L0.v32.z, pq_part, spmv_dot_blocks(L0.A64), rr_part,
                             L0.v32.y, c, s);
    cycle_level<float>(h, 0, L0.v32.y, L0.v32.z, nullptr);
    launch_pcg_rz<float>(n, h->vr, L0.v32.z, rz_part, rr_part, nv, c, s);
    launch_pcg_pupdate<float>(n, L0.v32.z, h->vp, rz_part, nv, c, s);
  } else {
    launch_pcg_update<double>(n, h->vu, h->vr, h->vp, h->vq, h->vz, pq_part, spmv_dot_blocks(L0.A64), rr_part,
                              nullptr, c, s);
    cycle_level<double>(h, 0, h->vr, h->vz, nullptr);
    launch_pcg_rz<double>(n, h->vr, h->vz, rz_part, rr_part, nv, c, s);
    launch_pcg_pupdate<double>(n, h->vz, h->vp, rz_part, nv, c, s);
  }
}

static void alloc_level_vectors(aspamg_ctx *h) {
  for (auto &L : h->lev) {
    const size_t n = (size_t)L.A.n * h->b;
    L.v64.y = dalloc<double>(h, n);
    L.v64.z = dalloc<double>(h, n);
    L.v64.r = dalloc<double>(h, n);
    L.v64.t = dalloc<double>(h, n);
    L.v32.y = dalloc<float>(h, n);
    L.v32.z = dalloc<float>(h, n);
    L.v32.r = dalloc<float>(h, n);
    L.v32.t = dalloc<float>(h, n);
  }
  const size_t n = (size_t)h->n * h->b;
  h->vu = dalloc<double>(h, n);
  h->vr = dalloc<double>(h, n);
  h->vp = dalloc<double>(h, n);
  h->vq = dalloc<double>(h, n);
  h->vz = dalloc<double>(h, n);
  h->part = dalloc<double>(h, 4 * kMaxPart);
  h->ctrl = dalloc<PcgCtrl>(h, 1);
  HIPCHK(hipHostMalloc((void **)&h->ctrl_host, sizeof(PcgCtrl), hipHostMallocDefault));
}

static void compute_complexities(aspamg_ctx *h) {
  double sn = 0, sa = 0, sg = 0, sga = 0;
  for (auto &L : h->lev) {
    sn += L.A.n;
    sa += (double)L.A.nnzb();
    if (!L.coarsest) {
      // scalar nonzeros: off-diagonal blocks b^2, diagonal block b(b+1)/2
      const double bb = (double)h->b * h->b, bd = h->b * (h->b + 1) / 2.0;
      sg += (double)(L.G.nnzb() - L.G.n) * bb + bd * L.G.n;
      sga += (double)L.A.nnzb() * bb;
    }
  }
  h->c_gd = sn / h->lev[0].A.n;
  h->c_op = sa / (double)h->lev[0].A.nnzb();
  h->c_fs = sga > 0 ? sg / sga : 0.0;
}

// Algorithmic bytes: each stored block once per use (9 values plus its column
// index, 4 or 2 bytes as stored), 18 vector passes per level, the dense tail
// or coarsest operator; one PCG iteration adds q = K p (p read, q written) and
// the vector kernels: the update reads u, r, p, q (FP64) and z and writes u, r
// (FP64) and r in the cycle precision s when s = 4; r.z reads r and z; the
// direction update reads z and p and writes p.  That is 96 B per unknown with
// an FP64 cycle and 88 B with an FP32 one.
template <typename T>
static double block_bytes(const Sell<T> &S) {
  return (double)S.b * S.b * sizeof(T) + S.index_bytes();
}

template <typename T>
static double level_bytes(const aspamg_ctx *h, const Level &L) {
  using O = Ops<T>;
  const double nA = (double)L.A.nnzb(), nG = (double)L.G.nnzb(), nP = (double)L.P.nnzb();
  // A: nu1 - 1 pre-smoothing residuals, the restriction residual and nu2 - 1
  // post-smoothing residuals; G and G^T once per smoothing step; R once; the
  // stacked [P; A P] once (first post-smoothing step, nu2 >= 1), or P and one
  // more A
  const double usesA = (double)(h->p.nu1 + h->p.nu2 - (L.stacked() ? 1 : 0));
  const double nu = (double)(h->p.nu1 + h->p.nu2);
  const bool merged = std::is_same<T, float>::value && L.nnzb_M > 0;
  const double smooth = merged ? (double)L.nnzb_M * block_bytes(O::M(L))
                               : nG * (block_bytes(O::G(L)) + block_bytes(O::GT(L)));
  const double post = L.stacked() ? (nP + (double)L.nnzb_AP) * block_bytes(O::PAP(L)) : nP * block_bytes(O::P(L));
  return usesA * nA * block_bytes(O::A(L)) + nu * smooth + nP * block_bytes(O::R(L)) + post +
         18.0 * h->b * L.A.n * sizeof(T);
}

static double cycle_bytes(const aspamg_ctx *h, int prec) {
  double B = 0.0;
  for (int l = 0; l < (int)h->lev.size(); l++) {
    const Level &L = h->lev[l];
    if (l == h->tail.level) {
      const double nd = h->tail.nd;
      B += nd * nd * 8.0 + 2.0 * nd * (prec == 32 ? 4.0 : 8.0);
      break;
    }
    if (L.coarsest) B += (double)h->coarse.nd * h->coarse.nd * 8.0;
    else B += prec == 32 ? level_bytes<float>(h, L) : level_bytes<double>(h, L);
  }
  return B;
}

static double kp_block_bytes(const aspamg_ctx *h) { return 8.0 * h->b * h->b + h->lev[0].A64.index_bytes(); }

static double iter_bytes(const aspamg_ctx *h, int prec) {
  const Level &L0 = h->lev[0];
  const double per_dof = prec == 32 ? 88.0 : 96.0;
  return (double)L0.A.nnzb() * kp_block_bytes(h) + (double)h->b * L0.A.n * (16.0 + per_dof) + cycle_bytes(h, prec);
}

template <typename T>
static bool is_device_ptr(const T *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

template <typename T>
static std::vector<T> fetch(const T *p, size_t n, hipStream_t s) {
  std::vector<T> v(n);
  if (n == 0) return v;
  if (is_device_ptr(p)) {
    HIPCHK(hipMemcpyAsync(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  } else {
    std::memcpy(v.data(), p, n * sizeof(T));
  }
  return v;
}

static void check_params(const aspamg_params &p) {
  if (p.k_g < 0 || p.rho_blocks < 1 || p.rho_blocks > kMaxGrowRho || p.theta < 1 || p.theta > kMaxTheta || p.n_max < 1 || p.n_max > kMaxPEntries || p.d_p < 1 ||
      p.lanczos_steps < 1 || p.lanczos_steps > 200 || p.nu1 < 1 || p.nu2 < 1 || p.max_levels < 1 ||
      (p.cycle_precision != 32 && p.cycle_precision != 64) || !(p.rtol >= 0) || p.max_it < 1 ||
      p.quant_bits < 8 || p.quant_bits > 52 || p.check_every < 1 || p.n_tv < 0 || p.n_tv > 64 ||
      p.n_rq < 0 || p.n_rq > 1000 ||
      p.layout < 0 || p.layout > 4 || p.dense_tail_dof < 0 || p.dense_tail_dof > kMaxTailDof ||
      (p.block_size != 1 && p.block_size != 3) ||
      !(p.kappa_p > 0) || !(p.omega_safety > 0))
    fail(ASPAMG_EINVAL, "invalid parameter value");
}

// gamma_{m+1} = (m+1) u / (1 - (m+1) u) for the longest scalar row of K (m
// stored entries): |fl(f - K u) - (f - K u)| <= gamma_{m+1} (|f| + |K| |u|)
// componentwise (Higham, "Accuracy and Stability of Numerical Algorithms",
// Sec. 3.5), whatever the order of the row's sums
double residual_gamma(const aspamg_ctx *h) {
  const HostBSR &A = h->lev[0].A;
  int64_t m = 0;
  for (int32_t i = 0; i < A.n; i++) m = std::max(m, A.rp[i + 1] - A.rp[i]);
  const double k = (double)(h->b * m + 1), u = std::ldexp(1.0, -53);
  return k * u / (1.0 - k * u);
}

}  // namespace aspamg

using namespace aspamg;

#define ABI_BEGIN try {
#define ABI_END                                   \
  }                                               \
  catch (const Error &e) {                        \
    g_last_error = e.msg;                         \
    return e.code;                                \
  }                                               \
  catch (const std::bad_alloc &) {                \
    g_last_error = "host allocation failed";      \
    return ASPAMG_ENOMEM;                         \
  }                                               \
  catch (...) {                                   \
    g_last_error = "unexpected internal error";   \
    return ASPAMG_EINVAL;                         \
  }

extern "C" {

const char *aspamg_last_error(void) { return g_last_error.c_str(); }

aspamg_status aspamg_default_params(aspamg_params *o) {
  if (!o) return ASPAMG_EINVAL;
  std::memset(o, 0, sizeof *o);
  o->k_g = 4;
  o->rho_g = 4;
  o->eps_g = 1e-3;
  o->n_tv = 0;
  o->n_rq = 0;
  o->theta = 5;
  o->n_max = 5;
  o->kappa_p = 50.0;
  o->rho_blocks = 3;
  o->omega_bar = 0.8;
  o->outer_fsai = 1;
  o->d_p = 2;
  o->eps_p = 1e-8;
  o->lanczos_steps = 30;
  o->omega_safety = 1.05;
  o->coarse_max_dof = 1500;
  o->max_levels = 25;
  o->stall_ratio = 0.9;
  o->nu1 = 1;
  o->nu2 = 1;
  o->cycle_precision = 64;
  o->rtol = 1e-10;
  o->max_it = 1000;
  o->quant_bits = 20;
  o->dense_max_dof = 16384;
  o->check_every = 4;
  o->use_graph = 1;
  o->layout = 0;
  o->dense_tail_dof = 4096;
  o->block_size = 3;
  return ASPAMG_OK;
}

aspamg_status aspamg_destroy(aspamg_handle h) {
  if (!h) return ASPAMG_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  destroy_batch(h->batch);
  h->batch = nullptr;
  for (int i = 0; i < 2; i++)
    if (h->graph[i]) (void)hipGraphExecDestroy(h->graph[i]);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (void *p : h->allocations) (void)hipFree(p);
  if (h->ctrl_host) (void)hipHostFree(h->ctrl_host);
  if (h->staging) (void)hipHostFree(h->staging);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return ASPAMG_OK;
}

static aspamg_status setup_impl(const aspamg_params *pp, int32_t n_nodes, int64_t nnzb, const int32_t *row_ptr,
                                const int32_t *col, const double *vals, int32_t n_tv, const double *V0,
                                void *hip_stream, aspamg_ctx *hraw, aspamg_handle *out) {
  struct NoDelete {
    void operator()(aspamg_ctx *) const {}
  };
  std::unique_ptr<aspamg_ctx, NoDelete> h(hraw);
  ABI_BEGIN
  if (!out || n_nodes <= 0 || nnzb < n_nodes || !row_ptr || !col || !vals || n_tv < 0 || (n_tv > 0 && !V0))
    fail(ASPAMG_EINVAL, "invalid arguments to aspamg_setup");
  aspamg_params p;
  if (pp) p = *pp;
  else aspamg_default_params(&p);
  if (p.n_tv != 0 && p.n_tv != n_tv)
    fail(ASPAMG_EINVAL, "params.n_tv (" + std::to_string(p.n_tv) + ") differs from the columns of V0 (" +
                            std::to_string(n_tv) + ")");
  p.n_tv = n_tv;
  check_params(p);
  const auto t0 = std::chrono::steady_clock::now();
  h->p = p;
  // every stream keeps the default priority; a private stream is created so
  // that the PCG iteration can be captured as a graph
  hipStream_t user = static_cast<hipStream_t>(hip_stream);
  HIPCHK(hipGetDevice(&h->device));
  HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
  noalloc_scratch_current_device();   // the no-allocation entry point's staging on this device
  if (user) HIPCHK(hipStreamSynchronize(user));
  h->ntv = n_tv;
  h->n = n_nodes;
  h->b = p.block_size;
  const int bb = h->b * h->b;
  HostBSR A;
  A.n = A.nc = n_nodes;
  A.b = h->b;
  {
    std::vector<int32_t> rp = fetch(row_ptr, (size_t)n_nodes + 1, h->stream);
    if (rp[0] != 0 || rp[n_nodes] != nnzb) fail(ASPAMG_EINVAL, "row_ptr inconsistent with nnzb");
    A.rp.assign(rp.begin(), rp.end());
  }
  A.ci = fetch(col, (size_t)nnzb, h->stream);
  A.v = fetch(vals, (size_t)nnzb * bb, h->stream);
  for (int32_t i = 0; i < n_nodes; i++) {
    if (A.rp[i + 1] < A.rp[i]) fail(ASPAMG_EINVAL, "row_ptr not monotone");
    bool diag = false;
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; k++) {
      if (A.ci[k] < 0 || A.ci[k] >= n_nodes) fail(ASPAMG_EINVAL, "column index out of range");
      if (k > A.rp[i] && A.ci[k] <= A.ci[k - 1]) fail(ASPAMG_EINVAL, "column indices not strictly ascending");
      diag |= A.ci[k] == i;
    }
    if (!diag) fail(ASPAMG_EINVAL, "missing diagonal block");
  }
  for (double x : A.v)
    if (!std::isfinite(x)) fail(ASPAMG_EINVAL, "non-finite matrix value");
  std::vector<double> V = n_tv ? fetch(V0, (size_t)n_nodes * h->b * n_tv, h->stream) : std::vector<double>();
  build_hierarchy(h.get(), std::move(A), std::move(V));
  alloc_level_vectors(h.get());
  build_tail(h.get());
  merge_smoothers(h.get());
  compute_complexities(h.get());
  h->prec = p.cycle_precision;
  HIPCHK(hipStreamSynchronize(h->stream));
  h->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = h.release();
  return ASPAMG_OK;
  ABI_END
}

aspamg_status aspamg_setup(const aspamg_params *pp, int32_t n_nodes, int64_t nnzb, const int32_t *row_ptr,
                           const int32_t *col, const double *vals, int32_t n_tv, const double *V0, void *hip_stream,
                           aspamg_handle *out) {
  if (out) *out = nullptr;
  aspamg_ctx *h = new (std::nothrow) aspamg_ctx();
  if (!h) return ASPAMG_ENOMEM;
  const aspamg_status rc = setup_impl(pp, n_nodes, nnzb, row_ptr, col, vals, n_tv, V0, hip_stream, h, out);
  if (rc != ASPAMG_OK) {
    if (out) *out = nullptr;
    aspamg_destroy(h);
  }
  return rc;
}

aspamg_status aspamg_set_cycle_precision(aspamg_handle h, int32_t bits) {
  if (!h || (bits != 32 && bits != 64)) return ASPAMG_EINVAL;
  h->prec = bits;
  return ASPAMG_OK;
}

static void fill_stats(aspamg_handle h, aspamg_stats *st, const PcgCtrl &c, double t_solve, double relres_true,
                       double relres_floor) {
  if (!st) return;
  st->status = c.status;
  st->iterations = c.iter;
  st->levels = (int32_t)h->lev.size();
  st->cycle_precision = h->prec;
  st->relres_recursive = c.relres;
  st->relres_true = relres_true;
  st->relres_floor = relres_floor;
  st->t_setup_s = h->t_setup;
  st->t_solve_s = t_solve;
  st->c_gd = h->c_gd;
  st->c_op = h->c_op;
  st->c_fs = h->c_fs;
  st->bytes_vcycle = cycle_bytes(h, h->prec);
  st->bytes_iter = iter_bytes(h, h->prec);
  st->tail_level = h->tail.level;
}

aspamg_status aspamg_solve(aspamg_handle h, const double *f_dev, double *u_dev, aspamg_stats *st) {
  ABI_BEGIN
  if (!h || !f_dev || !u_dev) fail(ASPAMG_EINVAL, "invalid arguments to aspamg_solve");
  hipStream_t s = h->stream;
  const int64_t n = (int64_t)h->n * h->b;
  const bool fp32 = h->prec == 32;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // control block
  PcgCtrl c0;
  std::memset(&c0, 0, sizeof c0);
  c0.status = ASPAMG_NOT_CONVERGED;
  c0.max_it = h->p.max_it;
  c0.rtol = h->p.rtol;
  *h->ctrl_host = c0;
  HIPCHK(hipEventRecord(e0, s));
  HIPCHK(hipMemcpyAsync(h->ctrl, h->ctrl_host, sizeof(PcgCtrl), hipMemcpyHostToDevice, s));
  // u = 0, r = f, |f|
  launch_fill(n, h->vu, 0.0, s);
  launch_copy(n, f_dev, h->vr, s);
  launch_dot(n, f_dev, f_dev, h->part, nullptr, s);
  launch_finish(kFinInitF, h->part, vec_blocks(n), h->ctrl, s);
  // z = M r, p = z, rz = r.z
  precondition(h, h->vr, h->vz, h->ctrl, fp32);
  launch_dot(n, h->vr, h->vz, h->part, h->ctrl, s);
  launch_finish(kFinInitRz, h->part, vec_blocks(n), h->ctrl, s);
  launch_copy(n, h->vz, h->vp, s);
  HIPCHK(hipGetLastError());
  hipGraphExec_t &gx = h->graph[fp32 ? 1 : 0];
  if (h->p.use_graph && !gx) {
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      pcg_iteration(h, fp32);
    } catch (...) {   // leave the stream out of capture mode before reporting
      hipGraph_t dead = nullptr;
      (void)hipStreamEndCapture(s, &dead);
      if (dead) (void)hipGraphDestroy(dead);
      throw;
    }
    HIPCHK(hipStreamEndCapture(s, &g));
    HIPCHK(hipGraphInstantiate(&gx, g, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(g));
  }
  const int every = h->p.check_every;
  for (;;) {
    HIPCHK(hipMemcpyAsync(h->ctrl_host, h->ctrl, sizeof(PcgCtrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h->ctrl_host->done) break;
    for (int k = 0; k < every; k++) {
      if (h->p.use_graph) HIPCHK(hipGraphLaunch(gx, s));
      else pcg_iteration(h, fp32);
    }
    HIPCHK(hipGetLastError());
  }
  launch_copy(n, h->vu, u_dev, s);
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  PcgCtrl c = *h->ctrl_host;
  // true residual |f - K u| / |f|, and the rounding bound of evaluating it
  launch_spmv<double, double, double>(h->lev[0].A64, h->vu, h->vq, f_dev, -1.0, nullptr, s);
  launch_dot(n, h->vq, h->vq, h->part, nullptr, s);
  const int nbnd = spmv_dot_blocks(h->lev[0].A64);
  launch_abs_bound(h->lev[0].A64, h->vu, f_dev, h->part + kMaxPart, s);
  std::vector<double> part(vec_blocks(n)), bpart(nbnd);
  HIPCHK(hipMemcpyAsync(part.data(), h->part, part.size() * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(bpart.data(), h->part + kMaxPart, bpart.size() * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double rr = 0.0, bb = 0.0;
  for (double x : part) rr += x;
  for (double x : bpart) bb += x;
  const double relres_true = c.fnorm > 0 ? std::sqrt(rr) / c.fnorm : 0.0;
  const double bound = c.fnorm > 0 ? residual_gamma(h) * std::sqrt(bb) / c.fnorm : 0.0;
  // converged (Section 4: the recursive residual) only when the recomputed
  // residual agrees: at most rtol, or within the rounding bound of its own
  // evaluation in FP64
  if (c.status == ASPAMG_OK && !(relres_true <= std::max(c.rtol, bound))) c.status = ASPAMG_NOT_CONVERGED;
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  fill_stats(h, st, c, ms * 1e-3, relres_true, bound);
  return (aspamg_status)c.status;
  ABI_END
}

aspamg_status aspamg_vcycle(aspamg_handle h, const double *y_dev, double *z_dev) {
  ABI_BEGIN
  if (!h || !y_dev || !z_dev) fail(ASPAMG_EINVAL, "invalid arguments to aspamg_vcycle");
  precondition(h, y_dev, z_dev, nullptr, h->prec == 32);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return ASPAMG_OK;
  ABI_END
}

aspamg_status aspamg_apply_operator(aspamg_handle h, int32_t level, int32_t which, int32_t precision,
                                    const double *x_dev, double *y_dev) {
  ABI_BEGIN
  if (!h || level < 0 || level >= (int32_t)h->lev.size() || which < 0 || which > 5 ||
      (precision != 32 && precision != 64) || !x_dev || !y_dev)
    fail(ASPAMG_EINVAL, "invalid arguments to aspamg_apply_operator");
  const Level &L = h->lev[level];
  if (L.coarsest && which != 0) fail(ASPAMG_EINVAL, "the coarsest level has only A");
  if (which == 5 && L.nnzb_M == 0) fail(ASPAMG_EINVAL, "this level applies G and G^T (no merged G^T G)");
  hipStream_t s = h->stream;
  if (precision == 64) {
    const Sell<double> *M[6] = {&L.A64, &L.G64, &L.GT64, &L.P64, &L.R64, &L.M64};
    launch_spmv<double, double, double>(*M[which], x_dev, y_dev, nullptr, 1.0, nullptr, s);
  } else {
    const Sell<float> *M[6] = {&L.A32, &L.G32, &L.GT32, &L.P32, &L.R32, &L.M32};
    const int64_t nx = (int64_t)M[which]->nc * h->b, ny = (int64_t)M[which]->n * h->b;
    float *xs = nullptr, *ys = nullptr;
    HIPCHK(hipMalloc(&xs, std::max<int64_t>(nx, 1) * 4));
    HIPCHK(hipMalloc(&ys, std::max<int64_t>(ny, 1) * 4));
    launch_cast<double, float>(nx, x_dev, xs, nullptr, s);
    launch_spmv<float, float, float>(*M[which], xs, ys, nullptr, 1.0, nullptr, s);
    launch_cast<float, double>(ny, ys, y_dev, nullptr, s);
    HIPCHK(hipStreamSynchronize(s));
    (void)hipFree(xs);
    (void)hipFree(ys);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ASPAMG_OK;
  ABI_END
}

aspamg_status aspamg_level_info(aspamg_handle h, int32_t level, aspamg_level_info_t *o) {
  if (!h || !o || level < 0 || level >= (int32_t)h->lev.size()) return ASPAMG_EINVAL;
  const Level &L = h->lev[level];
  std::memset(o, 0, sizeof *o);
  o->n = L.A.n;
  o->n_coarse = L.coarsest ? 0 : L.nc;
  o->nnzb_A = L.A.nnzb();
  o->nnzb_G = L.G.nnzb();
  o->nnzb_P = L.P.nnzb();
  o->has_smoother = !L.coarsest;
  o->fsai_rounds = L.fsai_rounds;
  o->lambda1 = L.lambda1;
  o->omega_q = L.omega_q;
  o->omega_s = L.omega_s;
  o->sell_slots_A = L.A64.slots();
  o->sell_slots_G = L.G64.slots();
  o->sell_slots_GT = L.GT64.slots();
  const Sell<double> *M64[5] = {&L.A64, &L.G64, &L.GT64, &L.P64, &L.R64};
  const Sell<float> *M32[5] = {&L.A32, &L.G32, &L.GT32, &L.P32, &L.R32};
  o->sell_index16 = 0;
  for (int k = 0; k < 5; k++) {
    o->sell_lanes64[k] = M64[k]->pack ? -M64[k]->pack : M64[k]->lanes;
    o->sell_lanes32[k] = M32[k]->pack ? -M32[k]->pack : M32[k]->lanes;
    if (M64[k]->col16) o->sell_index16 |= 1 << k;
    if (M32[k]->col16) o->sell_index16 |= 1 << (5 + k);
  }
  for (int k = 0; k < 5; k++) {
    o->sell_unit64[k] = M64[k]->pack ? M64[k]->unit : 0;
    o->sell_unit32[k] = M32[k]->pack ? M32[k]->unit : 0;
  }
  if (L.stacked()) {
    o->sell_stacked = L.PAP64.pack ? -L.PAP64.pack : L.PAP64.lanes;
    o->sell_stacked32 = L.PAP32.pack ? -L.PAP32.pack : L.PAP32.lanes;
    o->sell_stacked_unit64 = L.PAP64.pack ? L.PAP64.unit : 0;
    o->sell_stacked_unit32 = L.PAP32.pack ? L.PAP32.unit : 0;
  }
  o->nnzb_M = L.nnzb_M;
  if (L.PAP64.col16) o->sell_index16 |= 1 << 10;
  return ASPAMG_OK;
}

aspamg_status aspamg_level_matrix(aspamg_handle h, int32_t level, int32_t which, int64_t *row_ptr, int32_t *col,
                                  double *vals) {
  if (!h || level < 0 || level >= (int32_t)h->lev.size() || (which != 0 && which != 1 && which != 3))
    return ASPAMG_EINVAL;
  const Level &L = h->lev[level];
  const HostBSR &M = which == 0 ? L.A : which == 1 ? L.G : L.P;
  if (row_ptr && !M.rp.empty()) std::memcpy(row_ptr, M.rp.data(), M.rp.size() * 8);
  if (col && !M.ci.empty()) std::memcpy(col, M.ci.data(), M.ci.size() * 4);
  if (vals && !M.v.empty()) std::memcpy(vals, M.v.data(), M.v.size() * 8);
  return ASPAMG_OK;
}

aspamg_status aspamg_level_split(aspamg_handle h, int32_t level, int8_t *cf, int32_t *p_counts, int32_t *p_cols) {
  if (!h || level < 0 || level >= (int32_t)h->lev.size()) return ASPAMG_EINVAL;
  const Level &L = h->lev[level];
  if (cf && !L.cf.empty()) std::memcpy(cf, L.cf.data(), L.cf.size());
  if (p_counts && !L.pcount.empty()) std::memcpy(p_counts, L.pcount.data(), L.pcount.size() * 4);
  if (p_cols && !L.pcols.empty()) std::memcpy(p_cols, L.pcols.data(), L.pcols.size() * 4);
  return ASPAMG_OK;
}

aspamg_status aspamg_level_test_space(aspamg_handle h, int32_t level, double *V) {
  if (!h || level < 0 || level >= (int32_t)h->lev.size() || !V) return ASPAMG_EINVAL;
  const Level &L = h->lev[level];
  if (!L.V.empty()) std::memcpy(V, L.V.data(), L.V.size() * 8);
  return ASPAMG_OK;
}

aspamg_status aspamg_element_gradient(int64_t n_el, const int32_t *conn_dev, const double *Ke0_dev, int64_t ke_stride,
                                      const double *lam_dev, const double *u_dev, const double *scale_dev,
                                      double *grad_dev, void *hip_stream) {
  ABI_BEGIN
  if (n_el < 0 || (n_el > 0 && (!conn_dev || !Ke0_dev || !lam_dev || !u_dev || !grad_dev)) ||
      (ke_stride != 0 && ke_stride != 576))
    fail(ASPAMG_EINVAL, "invalid arguments to aspamg_element_gradient");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  launch_element_gradient(n_el, conn_dev, Ke0_dev, ke_stride, lam_dev, u_dev, scale_dev, grad_dev, s);
  HIPCHK(hipGetLastError());
  return ASPAMG_OK;
  ABI_END
}

aspamg_status aspamg_assembler_create(int32_t n_nodes, int64_t n_el, const int32_t *conn, const int8_t *constrained,
                                      const int32_t *row_ptr, const int32_t *col, const double *Ke0,
                                      int64_t ke_stride, void *hip_stream, aspamg_assembler *out) {
  if (out) *out = nullptr;
  auto *a = new aspamg_assembler_ctx();
  ABI_BEGIN
  if (!out || n_nodes <= 0 || n_el < 0 || !conn || !row_ptr || !col || !Ke0 || (ke_stride != 0 && ke_stride != 576))
    fail(ASPAMG_EINVAL, "invalid arguments to aspamg_assembler_create");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  a->stream = s;
  a->n_nodes = n_nodes;
  a->n_el = n_el;
  std::vector<int32_t> rp = fetch(row_ptr, (size_t)n_nodes + 1, s);
  const int64_t nnzb = rp[n_nodes];
  a->nnzb = nnzb;
  std::vector<int32_t> ci = fetch(col, (size_t)nnzb, s);
  std::vector<int32_t> cn = fetch(conn, (size_t)n_el * 8, s);
  std::vector<int8_t> cons = constrained ? fetch(constrained, (size_t)n_nodes, s) : std::vector<int8_t>(n_nodes, 0);
  std::vector<double> ke = fetch(Ke0, (size_t)(ke_stride ? n_el * 576 : 576), s);
  // contributions per slot, ascending element order (counting sort keeps it)
  std::vector<int64_t> cnt(nnzb + 1, 0);
  std::vector<int64_t> slot_of((size_t)n_el * 64, -1);
  std::vector<int8_t> diag(nnzb, 0);
  for (int64_t e = 0; e < n_el; e++)
    for (int a1 = 0; a1 < 8; a1++)
      for (int b1 = 0; b1 < 8; b1++) {
        const int32_t r = cn[e * 8 + a1], c = cn[e * 8 + b1];
        if (r < 0 || r >= n_nodes || c < 0 || c >= n_nodes) fail(ASPAMG_EINVAL, "connectivity out of range");
        if (cons[r] || cons[c]) continue;
        const int32_t *b = ci.data() + rp[r], *en = ci.data() + rp[r + 1];
        const int32_t *it = std::lower_bound(b, en, c);
        if (it == en || *it != c) fail(ASPAMG_EINVAL, "element coupling missing from the block pattern");
        const int64_t sl = it - ci.data();
        slot_of[e * 64 + a1 * 8 + b1] = sl;
        cnt[sl + 1]++;
      }
  for (int32_t i = 0; i < n_nodes; i++)
    if (cons[i]) {
      const int32_t *b = ci.data() + rp[i], *en = ci.data() + rp[i + 1];
      const int32_t *it = std::lower_bound(b, en, i);
      if (it == en || *it != i) fail(ASPAMG_EINVAL, "missing diagonal block");
      diag[it - ci.data()] = 1;
    }
  for (int64_t k = 0; k < nnzb; k++) cnt[k + 1] += cnt[k];
  std::vector<int32_t> contrib((size_t)cnt[nnzb] * 2 + 2);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t e = 0; e < n_el; e++)
    for (int ab = 0; ab < 64; ab++) {
      const int64_t sl = slot_of[e * 64 + ab];
      if (sl < 0) continue;
      const int64_t q = pos[sl]++;
      contrib[2 * q] = (int32_t)e;
      contrib[2 * q + 1] = ab;
    }
  auto up = [&](const void *src, size_t bytes) {
    void *d = nullptr;
    HIPCHK(hipMalloc(&d, std::max<size_t>(bytes, 16)));
    if (bytes) HIPCHK(hipMemcpy(d, src, bytes, hipMemcpyHostToDevice));
    return d;
  };
  a->slot_ptr = (int64_t *)up(cnt.data(), cnt.size() * 8);
  a->contrib = (int32_t *)up(contrib.data(), contrib.size() * 4);
  a->diag_identity = (int8_t *)up(diag.data(), diag.size());
  a->Ke0 = (double *)up(ke.data(), ke.size() * 8);
  a->ke_stride = ke_stride;
  *out = a;
  return ASPAMG_OK;
  ABI_END
}

aspamg_status aspamg_assemble(aspamg_assembler a, const double *E_dev, double *vals_dev) {
  ABI_BEGIN
  if (!a || !E_dev || !vals_dev) fail(ASPAMG_EINVAL, "invalid arguments to aspamg_assemble");
  launch_assemble(a->nnzb, a->slot_ptr, a->contrib, a->diag_identity, a->Ke0, a->ke_stride, E_dev, vals_dev,
                  a->stream);
  HIPCHK(hipGetLastError());
  return ASPAMG_OK;
  ABI_END
}

aspamg_status aspamg_assembler_destroy(aspamg_assembler a) {
  if (!a) return ASPAMG_OK;
  if (a->stream) (void)hipStreamSynchronize(a->stream);
  else (void)hipDeviceSynchronize();
  (void)hipFree(a->slot_ptr);
  (void)hipFree(a->contrib);
  (void)hipFree(a->diag_identity);
  (void)hipFree(a->Ke0);
  delete a;
  return ASPAMG_OK;
}

aspamg_status aspamg_time_kernel(aspamg_handle h, int32_t which, int32_t reps, double *avg_ms, double *alg_bytes) {
  ABI_BEGIN
  if (!h || which < 0 || which > 4 || reps < 1 || !avg_ms || !alg_bytes)
    fail(ASPAMG_EINVAL, "invalid arguments to aspamg_time_kernel");
  hipStream_t s = h->stream;
  const Level &L0 = h->lev[0];
  const double N = (double)L0.A.n;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double bytes = 0.0;
  auto run = [&]() {
    switch (which) {
      case 0:
        launch_spmv_dot(L0.A64, h->vp, h->vq, h->part, nullptr, s);
        break;
      case 1:
        launch_spmv<float, float, float>(L0.A32, L0.v32.z, L0.v32.r, L0.v32.y, -1.0, nullptr, s);
        break;
      case 2:
        launch_spmv<double, double, double>(L0.A64, L0.v64.z, L0.v64.r, L0.v64.y, -1.0, nullptr, s);
        break;
      case 3:
        cycle_level<float>(h, 0, L0.v32.y, L0.v32.z, nullptr);
        break;
      case 4:
        cycle_level<double>(h, 0, L0.v64.y, L0.v64.z, nullptr);
        break;
    }
  };
  const double nb = (double)L0.A.nnzb(), bsz = h->b;
  switch (which) {
    case 0: bytes = nb * kp_block_bytes(h) + N * bsz * 8.0 * 2.0; break;                          // K, p, q
    case 1: bytes = nb * block_bytes(h->lev[0].A32) + N * bsz * 4.0 * 3.0; break;                 // A32, s, y, r
    case 2: bytes = nb * kp_block_bytes(h) + N * bsz * 8.0 * 3.0; break;
    case 3: bytes = cycle_bytes(h, 32); break;
    case 4: bytes = cycle_bytes(h, 64); break;
  }
  // inputs: zero-filled vectors are enough for timing (the bytes streamed do not depend on values)
  run();
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipEventRecord(e0, s));
  for (int i = 0; i < reps; i++) run();
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  *avg_ms = (double)ms / reps;
  *alg_bytes = bytes;
  return ASPAMG_OK;
  ABI_END
}

aspamg_status aspamg_time_operator(aspamg_handle h, int32_t level, int32_t op, int32_t precision, int32_t reps,
                                   double *avg_ms, double *alg_bytes) {
  ABI_BEGIN
  if (!h || level < 0 || level >= (int32_t)h->lev.size() || op < 0 || op > 7 ||
      (precision != 32 && precision != 64) || reps < 1 || !avg_ms || !alg_bytes)
    fail(ASPAMG_EINVAL, "invalid arguments to aspamg_time_operator");
  const Level &L = h->lev[level];
  const bool dense = level == h->tail.level || L.coarsest;
  if (dense != (op == 6)) fail(ASPAMG_EINVAL, "op 6 is the dense operator of the tail or coarsest level, and only it");
  if (op == 4 && L.nnzb_M == 0) fail(ASPAMG_EINVAL, "this level stores no merged G^T G");
  if (op == 4 && precision == 64) fail(ASPAMG_EINVAL, "the merged G^T G is applied by the FP32 cycle only");
  if (op == 5 && !L.stacked()) fail(ASPAMG_EINVAL, "this level applies P and then A (no stacked [P; A P])");
  hipStream_t s = h->stream;
  const double n3 = (double)h->b * L.A.n, vs = precision == 32 ? 4.0 : 8.0, bsz = h->b;
  double bytes = 0.0;
  std::function<void()> run;
  auto setup_op = [&](auto tag) {
    using T = decltype(tag);
    using O = Ops<T>;
    const LevelVecs<T> &W = O::V(L);
    if (op == 6) {
      const int nd = level == h->tail.level ? h->tail.nd : h->coarse.nd;
      const double *D = level == h->tail.level ? h->tail.v : h->coarse.inv;
      run = [=]() { launch_dense_gemv<T>(nd, D, W.y, W.z, nullptr, s); };
      bytes = (double)nd * nd * 8.0 + 2.0 * nd * vs;
      return;
    }
    const LevelVecs<T> &Wn = O::V(h->lev[level + 1 < (int)h->lev.size() ? level + 1 : level]);
    const double w = L.omega_s;
    switch (op) {
      case 0:   // residual r = y - A z
        run = [=, &L]() { launch_spmv<T, T, T>(O::A(L), W.z, W.r, W.y, -1.0, nullptr, s); };
        bytes = (double)L.A.nnzb() * block_bytes(O::A(L)) + 3.0 * n3 * vs;
        break;
      case 1:   // t = G r
        run = [=, &L]() { launch_spmv<T, T, T>(O::G(L), W.r, W.t, nullptr, 1.0, nullptr, s); };
        bytes = (double)L.G.nnzb() * block_bytes(O::G(L)) + 2.0 * n3 * vs;
        break;
      case 2:   // z = z + w G^T t
        run = [=, &L]() { launch_spmv<T, T, T>(O::GT(L), W.t, W.z, W.z, w, nullptr, s); };
        bytes = (double)L.G.nnzb() * block_bytes(O::GT(L)) + 3.0 * n3 * vs;
        break;
      case 3:   // restriction r_c = R r
        run = [=, &L]() { launch_spmv<T, T, T>(O::R(L), W.r, Wn.y, nullptr, 1.0, nullptr, s); };
        bytes = (double)L.P.nnzb() * block_bytes(O::R(L)) + n3 * vs + bsz * L.nc * vs;
        break;
      case 4:   // z = z + w (G^T G) r, merged
        run = [=, &L]() { launch_spmv<T, T, T>(O::M(L), W.r, W.z, W.z, w, nullptr, s); };
        bytes = (double)L.nnzb_M * block_bytes(O::M(L)) + 3.0 * n3 * vs;
        break;
      case 5:   // stacked [P; A P] e: z + P e and r - (A P) e
        run = [=, &L]() {
          launch_spmv_dual<T, T, T>(O::PAP(L), L.P.n, Wn.z, W.z, W.z, 1.0, W.r, W.r, -1.0, nullptr, s);
        };
        bytes = ((double)L.P.nnzb() + (double)L.nnzb_AP) * block_bytes(O::PAP(L)) + 4.0 * n3 * vs + bsz * L.nc * vs;
        break;
      case 7:   // prolongation z += P e
        run = [=, &L]() { launch_spmv<T, T, T>(O::P(L), Wn.z, W.z, W.z, 1.0, nullptr, s); };
        bytes = (double)L.P.nnzb() * block_bytes(O::P(L)) + 2.0 * n3 * vs + bsz * L.nc * vs;
        break;
    }
  };
  if (precision == 32) setup_op(float{});
  else setup_op(double{});
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  run();
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipEventRecord(e0, s));
  for (int i = 0; i < reps; i++) run();
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  *avg_ms = (double)ms / reps;
  *alg_bytes = bytes;
  return ASPAMG_OK;
  ABI_END
}

aspamg_status aspamg_solve_batch(aspamg_handle h, int32_t k, const double *F_dev, int64_t ldf, double *U_dev,
                                 int64_t ldu, aspamg_stats *st) {
  ABI_BEGIN
  if (h && h->b != 3) fail(ASPAMG_EINVAL, "solve_batch needs 3x3 blocks (block_size 3)");
  const aspamg_status r = solve_batch_impl(h, k, F_dev, ldf, U_dev, ldu, st);
  if (st)
    for (int j = 0; j < k; j++) st[j].spmm_tile = batch_tile(h, h->prec);
  return r;
  ABI_END
}

}  // extern "C"
