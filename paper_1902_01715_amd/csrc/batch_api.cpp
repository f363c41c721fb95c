// Multi-right-hand-side PCG (aspamg_solve_batch): every load case runs the
// same V(nu1,nu2)-cycle through block SpMM kernels that fetch each stored block
// once per tile of KB right-hand sides.  Each column has its own alpha, beta
// and convergence test; finished columns are frozen (alpha = 0).  The SpMM tile
// KB is chosen per precision by timing one cycle for every candidate tile
// (results do not depend on it: each (row, column) sum runs in block order).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "batch.h"

namespace aspamg {

static void *bmalloc(BatchWork *w, size_t bytes) {
  void *p = nullptr;
  if (bytes == 0) bytes = 16;
  if (hipMalloc(&p, bytes) != hipSuccess) fail(ASPAMG_ENOMEM, "device allocation failed (batch)");
  w->allocations.push_back(p);
  return p;
}

template <typename T>
static DevBSRT<T> upload_plain(BatchWork *w, const HostBSR &M, hipStream_t s) {
  DevBSRT<T> d;
  d.n = M.n;
  d.nc = M.nc;
  d.nnzb = M.nnzb();
  // lane groups per row: long coarse-level rows are split (short rows run
  // faster unsplit, with more rows sharing each staged chunk)
  const double avg = M.n ? (double)d.nnzb / M.n : 0.0;
  d.split = avg < 40.0 ? 1 : (avg < 80.0 ? 4 : 8);
  std::vector<int32_t> rp(M.rp.begin(), M.rp.end());
  std::vector<T> v(std::max<size_t>(M.v.size(), 1));
  for (size_t i = 0; i < M.v.size(); i++) v[i] = (T)M.v[i];
  d.rp = (int32_t *)bmalloc(w, rp.size() * 4);
  d.ci = (int32_t *)bmalloc(w, std::max<size_t>(M.ci.size(), 1) * 4);
  d.v = (T *)bmalloc(w, v.size() * sizeof(T));
  HIPCHK(hipMemcpyAsync(d.rp, rp.data(), rp.size() * 4, hipMemcpyHostToDevice, s));
  if (!M.ci.empty()) HIPCHK(hipMemcpyAsync(d.ci, M.ci.data(), M.ci.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d.v, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return d;
}

void destroy_batch(BatchWork *w) {
  if (!w) return;
  for (int i = 0; i < 2; i++)
    if (w->graph[i]) (void)hipGraphExecDestroy(w->graph[i]);
  for (void *p : w->allocations) (void)hipFree(p);
  if (w->ctrl_host) (void)hipHostFree(w->ctrl_host);
  delete w;
}

static BatchWork *ensure_batch(aspamg_ctx *h, int kpad) {
  if (h->batch && h->batch->kpad == kpad) return h->batch;
  hipStream_t s = h->stream;
  HIPCHK(hipStreamSynchronize(s));
  destroy_batch(h->batch);
  h->batch = nullptr;
  BatchWork *w = new BatchWork();
  try {
    w->kpad = kpad;
    w->lev.resize(h->lev.size());
    for (size_t l = 0; l < h->lev.size(); l++) {
      const Level &L = h->lev[l];
      BatchLevel &B = w->lev[l];
      const size_t nv = (size_t)L.A.n * 3 * kpad;
      if (!L.coarsest) {
        const HostBSR GT = transpose(L.G), R = transpose(L.P);
        B.d.A = upload_plain<double>(w, L.A, s);
        B.d.G = upload_plain<double>(w, L.G, s);
        B.d.GT = upload_plain<double>(w, GT, s);
        B.d.P = upload_plain<double>(w, L.P, s);
        B.d.R = upload_plain<double>(w, R, s);
        B.f.A = upload_plain<float>(w, L.A, s);
        B.f.G = upload_plain<float>(w, L.G, s);
        B.f.GT = upload_plain<float>(w, GT, s);
        B.f.P = upload_plain<float>(w, L.P, s);
        B.f.R = upload_plain<float>(w, R, s);
      }
      B.d.y = (double *)bmalloc(w, nv * 8);
      B.d.z = (double *)bmalloc(w, nv * 8);
      B.d.r = (double *)bmalloc(w, nv * 8);
      B.d.t = (double *)bmalloc(w, nv * 8);
      B.f.y = (float *)bmalloc(w, nv * 4);
      B.f.z = (float *)bmalloc(w, nv * 4);
      B.f.r = (float *)bmalloc(w, nv * 4);
      B.f.t = (float *)bmalloc(w, nv * 4);
    }
    const size_t nv = (size_t)h->n * 3 * kpad;
    w->U = (double *)bmalloc(w, nv * 8);
    w->R = (double *)bmalloc(w, nv * 8);
    w->P = (double *)bmalloc(w, nv * 8);
    w->Q = (double *)bmalloc(w, nv * 8);
    w->Z = (double *)bmalloc(w, nv * 8);
    w->F = (double *)bmalloc(w, nv * 8);
    w->part = (double *)bmalloc(w, (size_t)2 * kBatchParts * kpad * 8);
    w->ctrl = (BatchCtrl *)bmalloc(w, sizeof(BatchCtrl));
    HIPCHK(hipHostMalloc((void **)&w->ctrl_host, sizeof(BatchCtrl), hipHostMallocDefault));
  } catch (...) {
    destroy_batch(w);
    throw;
  }
  h->batch = w;
  return w;
}

template <typename T>
static BatchOps<T> &bops(BatchLevel &B);
template <>
BatchOps<double> &bops<double>(BatchLevel &B) { return B.d; }
template <>
BatchOps<float> &bops<float>(BatchLevel &B) { return B.f; }

template <typename T>
static void cycle_batch(aspamg_ctx *h, BatchWork *w, int l, const T *y, T *z, int kb, const BatchCtrl *c) {
  hipStream_t s = h->stream;
  const int ld = w->kpad;
  const Level &L = h->lev[l];
  if (l == h->tail.level) {
    launch_dense_gemm<T>(h->tail.nd, h->tail.v, y, z, ld, c, s);
    return;
  }
  if (L.coarsest) {
    launch_dense_gemm<T>(h->coarse.nd, h->coarse.inv, y, z, ld, c, s);
    return;
  }
  BatchOps<T> &O = bops<T>(w->lev[l]);
  BatchOps<T> &On = bops<T>(w->lev[l + 1]);
  const double om = L.omega_s;
  for (int it = 0; it < h->p.nu1; it++) {
    if (it == 0) {
      launch_spmm<T>(O.G, y, O.t, nullptr, ld, kb, 1.0, c, s);
      launch_spmm<T>(O.GT, O.t, z, nullptr, ld, kb, om, c, s);
    } else {
      launch_spmm<T>(O.A, z, O.r, y, ld, kb, -1.0, c, s);
      launch_spmm<T>(O.G, O.r, O.t, nullptr, ld, kb, 1.0, c, s);
      launch_spmm<T>(O.GT, O.t, z, z, ld, kb, om, c, s);
    }
  }
  launch_spmm<T>(O.A, z, O.r, y, ld, kb, -1.0, c, s);
  launch_spmm<T>(O.R, O.r, On.y, nullptr, ld, kb, 1.0, c, s);
  cycle_batch<T>(h, w, l + 1, On.y, On.z, kb, c);
  launch_spmm<T>(O.P, On.z, z, z, ld, kb, 1.0, c, s);
  for (int it = 0; it < h->p.nu2; it++) {
    launch_spmm<T>(O.A, z, O.r, y, ld, kb, -1.0, c, s);
    launch_spmm<T>(O.G, O.r, O.t, nullptr, ld, kb, 1.0, c, s);
    launch_spmm<T>(O.GT, O.t, z, z, ld, kb, om, c, s);
  }
}

static void precondition_batch(aspamg_ctx *h, BatchWork *w, const double *r, double *z, const BatchCtrl *c,
                               bool fp32) {
  const int64_t n = (int64_t)h->n * 3 * w->kpad;
  if (fp32) {
    BatchOps<float> &O = w->lev[0].f;
    launch_cast<double, float>(n, r, O.y, nullptr, h->stream);
    cycle_batch<float>(h, w, 0, O.y, O.z, w->kb[1], c);
    launch_cast<float, double>(n, O.z, z, nullptr, h->stream);
  } else {
    cycle_batch<double>(h, w, 0, r, z, w->kb[0], c);
  }
}

static void pcg_iteration_batch(aspamg_ctx *h, BatchWork *w, bool fp32) {
  hipStream_t s = h->stream;
  const int ld = w->kpad;
  const int64_t nrow = (int64_t)h->n * 3;
  const int kb = w->kb[fp32 ? 1 : 0];
  BatchCtrl *c = w->ctrl;
  const BatchLevel &B0 = w->lev[0];
  launch_spmm_dot(B0.d.A, w->P, w->Q, ld, kb, w->part, c, s);
  launch_col_finish(kFinAlpha, w->part, spmm_dot_parts(B0.d.A, ld, kb), ld, c, s);
  if (fp32) {
    // z (and z_old) stay in FP32; the update writes the cycle input r in FP32
    launch_col_update<float>(nrow, w->U, w->R, w->P, w->Q, B0.f.z, B0.f.y, ld, w->part, c, s);
    launch_col_finish(kFinRr, w->part, batch_vec_blocks(nrow, ld), ld, c, s);
    cycle_batch<float>(h, w, 0, B0.f.y, B0.f.z, kb, c);
    launch_col_rz<float>(nrow, w->R, B0.f.z, ld, w->part, c, s);
    launch_col_finish(kFinBeta, w->part, batch_vec_blocks(nrow, ld), ld, c, s);
    launch_col_pupdate<float>(nrow, B0.f.z, w->P, ld, c, s);
  } else {
    launch_col_update<double>(nrow, w->U, w->R, w->P, w->Q, w->Z, nullptr, ld, w->part, c, s);
    launch_col_finish(kFinRr, w->part, batch_vec_blocks(nrow, ld), ld, c, s);
    cycle_batch<double>(h, w, 0, w->R, w->Z, kb, c);
    launch_col_rz<double>(nrow, w->R, w->Z, ld, w->part, c, s);
    launch_col_finish(kFinBeta, w->part, batch_vec_blocks(nrow, ld), ld, c, s);
    launch_col_pupdate<double>(nrow, w->Z, w->P, ld, c, s);
  }
}

// SpMM tile per precision: time one cycle for each candidate, keep the fastest
static void tune_tiles(aspamg_ctx *h, BatchWork *w) {
  hipStream_t s = h->stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (int p = 0; p < 2; p++) {
    if (w->kb[p]) continue;
    float best = 1e30f;
    int bestkb = std::min(4, w->kpad);
    for (int kb = 4; kb <= std::min(32, w->kpad); kb *= 2) {
      for (int rep = 0; rep < 3; rep++) {
        if (rep == 1) HIPCHK(hipEventRecord(e0, s));
        if (p == 0) cycle_batch<double>(h, w, 0, w->lev[0].d.y, w->lev[0].d.z, kb, nullptr);
        else cycle_batch<float>(h, w, 0, w->lev[0].f.y, w->lev[0].f.z, kb, nullptr);
      }
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        bestkb = kb;
      }
    }
    w->kb[p] = bestkb;
  }
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
}

// one chunk of k <= kBatchMax columns
static aspamg_status solve_chunk(aspamg_ctx *h, int k, const double *F, int64_t ldf, double *U, int64_t ldu,
                                 aspamg_stats *st) {
  int kpad = 4;
  while (kpad < k) kpad *= 2;
  BatchWork *w = ensure_batch(h, kpad);
  hipStream_t s = h->stream;
  const bool fp32 = h->prec == 32;
  const int64_t nrow = (int64_t)h->n * 3;
  const int ld = kpad;
  // the tuner runs cycles on zero-filled level vectors
  if (!w->kb[0] || !w->kb[1]) {
    const size_t nv = (size_t)h->n * 3 * kpad;
    HIPCHK(hipMemsetAsync(w->lev[0].d.y, 0, nv * 8, s));
    HIPCHK(hipMemsetAsync(w->lev[0].f.y, 0, nv * 4, s));
    tune_tiles(h, w);
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  BatchCtrl c0;
  std::memset(&c0, 0, sizeof c0);
  c0.max_it = h->p.max_it;
  c0.rtol = h->p.rtol;
  for (int j = 0; j < kBatchMax; j++) c0.status[j] = ASPAMG_NOT_CONVERGED;
  *w->ctrl_host = c0;
  HIPCHK(hipEventRecord(e0, s));
  HIPCHK(hipMemcpyAsync(w->ctrl, w->ctrl_host, sizeof(BatchCtrl), hipMemcpyHostToDevice, s));
  launch_copy_cols(nrow, k, F, ldf, w->F, ld, ld, s);
  launch_fill(nrow * ld, w->U, 0.0, s);
  launch_copy(nrow * ld, w->F, w->R, s);
  launch_col_dot(nrow, w->F, w->F, ld, w->part, w->ctrl, s);
  launch_col_finish(kFinInitF, w->part, batch_vec_blocks(nrow, ld), ld, w->ctrl, s);
  precondition_batch(h, w, w->R, w->Z, w->ctrl, fp32);
  launch_col_dot(nrow, w->R, w->Z, ld, w->part, w->ctrl, s);
  launch_col_finish(kFinInitRz, w->part, batch_vec_blocks(nrow, ld), ld, w->ctrl, s);
  launch_copy(nrow * ld, w->Z, w->P, s);
  HIPCHK(hipGetLastError());
  hipGraphExec_t &gx = w->graph[fp32 ? 1 : 0];
  if (h->p.use_graph && !gx) {
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    pcg_iteration_batch(h, w, fp32);
    HIPCHK(hipStreamEndCapture(s, &g));
    HIPCHK(hipGraphInstantiate(&gx, g, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(g));
  }
  for (;;) {
    HIPCHK(hipMemcpyAsync(w->ctrl_host, w->ctrl, sizeof(BatchCtrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (w->ctrl_host->all_done) break;
    for (int it = 0; it < h->p.check_every; it++) {
      if (h->p.use_graph) HIPCHK(hipGraphLaunch(gx, s));
      else pcg_iteration_batch(h, w, fp32);
    }
    HIPCHK(hipGetLastError());
  }
  launch_copy_cols(nrow, k, w->U, ld, U, ldu, k, s);
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  const BatchCtrl c = *w->ctrl_host;
  // true residuals F - K U per column
  launch_spmm<double>(w->lev[0].d.A, w->U, w->Q, w->F, ld, w->kb[0], -1.0, nullptr, s);
  launch_col_dot(nrow, w->Q, w->Q, ld, w->part, nullptr, s);
  const int nb = batch_vec_blocks(nrow, ld);
  std::vector<double> part((size_t)nb * ld), bpart((size_t)nb * ld);
  HIPCHK(hipMemcpyAsync(part.data(), w->part, part.size() * 8, hipMemcpyDeviceToHost, s));
  // and the rounding bound of evaluating it, column by column
  launch_abs_bound_cols(w->lev[0].d.A, w->U, w->F, ld, k, w->Q, s);
  launch_col_dot(nrow, w->Q, w->Q, ld, w->part, nullptr, s);
  HIPCHK(hipMemcpyAsync(bpart.data(), w->part, bpart.size() * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double gam = residual_gamma(h);
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  aspamg_status worst = ASPAMG_OK;
  for (int j = 0; j < k; j++) {
    double rr = 0.0, bb = 0.0;
    for (int b = 0; b < nb; b++) rr += part[(size_t)b * ld + j];
    for (int b = 0; b < nb; b++) bb += bpart[(size_t)b * ld + j];
    const double rel = c.fnorm[j] > 0 ? std::sqrt(rr) / c.fnorm[j] : 0.0;
    const double bound = c.fnorm[j] > 0 ? gam * std::sqrt(bb) / c.fnorm[j] : 0.0;
    aspamg_status sj = (aspamg_status)c.status[j];
    // converged only when the recomputed residual agrees (as for one column)
    if (sj == ASPAMG_OK && !(rel <= std::max(c.rtol, bound))) sj = ASPAMG_NOT_CONVERGED;
    if (sj < 0 && (worst >= 0 || sj < worst)) worst = sj;
    else if (worst == ASPAMG_OK && sj > 0) worst = sj;
    if (st) {
      aspamg_stats &o = st[j];
      std::memset(&o, 0, sizeof o);
      o.status = sj;
      o.iterations = c.iter[j];
      o.levels = (int32_t)h->lev.size();
      o.cycle_precision = h->prec;
      o.relres_recursive = c.relres[j];
      o.relres_true = rel;
      o.relres_floor = bound;
      o.t_setup_s = h->t_setup;
      o.t_solve_s = ms * 1e-3;
      o.c_gd = h->c_gd;
      o.c_op = h->c_op;
      o.c_fs = h->c_fs;
      o.tail_level = h->tail.level;
    }
  }
  return worst;
}

aspamg_status solve_batch_impl(aspamg_ctx *h, int32_t k, const double *F, int64_t ldf, double *U, int64_t ldu,
                               aspamg_stats *st) {
  if (!h || k < 1 || !F || !U || ldf < k || ldu < k) fail(ASPAMG_EINVAL, "invalid arguments to aspamg_solve_batch");
  aspamg_status worst = ASPAMG_OK;
  for (int j0 = 0; j0 < k; j0 += kBatchMax) {
    const int kc = std::min(kBatchMax, k - j0);
    const aspamg_status r = solve_chunk(h, kc, F + j0, ldf, U + j0, ldu, st ? st + j0 : nullptr);
    if (r < 0 && (worst >= 0 || r < worst)) worst = r;
    else if (worst == ASPAMG_OK && r > 0) worst = r;
  }
  return worst;
}

int batch_tile(const aspamg_ctx *h, int precision) {
  if (!h->batch) return 0;
  return h->batch->kb[precision == 32 ? 1 : 0];
}

}  // namespace aspamg
