// Multi-right-hand-side kernels: block-CSR SpMM over a tile of KB columns and
// the column-wise PCG vector operations with deterministic per-column
// reductions.  Vectors are stored [dof][ld] (right-hand sides fastest), so the
// KB lanes that share one block row read KB consecutive entries of every
// gathered x row, and every matrix block is fetched once for the whole tile.
#include <algorithm>

#include "batch.h"

namespace aspamg {

namespace {

__device__ __forceinline__ bool bdone(const BatchCtrl *c) { return c != nullptr && c->all_done != 0; }

// Y[:, tile] = alpha * (A X)[:, tile] (+ W[:, tile]) for the KB columns of
// tile blockIdx.y, and with DOT the per-column partials of X.Y.  Each lane
// takes CPT = 16 / sizeof(T) consecutive columns (one 16-byte load per
// gathered x entry), so a block row is served by S lane groups of KB / CPT
// lanes; group s takes the row's blocks s, s+S, s+2S, ..., and the S partial
// sums meet in LDS in group order.  A row group is 256 CPT / (KB S)
// consecutive rows.  The group's matrix blocks (a contiguous range of the
// block CSR) are staged in LDS, 256 CPT blocks at a time, by coalesced loads;
// the lanes read each block as an LDS broadcast and apply it to their CPT
// columns, so LDS delivers every block once per CPT columns and the global
// loads per block are the three x gathers of the tile.  Every column is
// summed in the same order as with one column per lane.
#ifndef ASPAMG_SPMM_CHUNK
#define ASPAMG_SPMM_CHUNK 256
#endif
#ifndef ASPAMG_SPMM_UNROLL
#define ASPAMG_SPMM_UNROLL 3
#endif
constexpr int kSpmmChunk = ASPAMG_SPMM_CHUNK;    // staged blocks per 16-byte column group
constexpr int kSpmmUnroll = ASPAMG_SPMM_UNROLL;  // blocks whose gathers are in flight together
#ifndef ASPAMG_SPMM_STAGE
#define ASPAMG_SPMM_STAGE 16
#endif
constexpr int kSpmmStage = ASPAMG_SPMM_STAGE;    // staging loads in flight per thread

template <typename T> struct Vec16;
template <> struct Vec16<float> {
  using type = float __attribute__((ext_vector_type(4)));
};
template <> struct Vec16<double> {
  using type = double __attribute__((ext_vector_type(2)));
};

template <typename T, bool HAS_W, bool DOT, int KB, int S>
__global__ void __launch_bounds__(256) k_bsr_spmm(int32_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col, const T *__restrict__ val,
                                                  const T *__restrict__ X, T *Y, const T *W, int32_t ld, T alpha,
                                                  double *__restrict__ part, const BatchCtrl *ctrl) {
  using V = typename Vec16<T>::type;
  constexpr int CPT = 16 / sizeof(T);
  constexpr int LPR = KB / CPT;          // lanes per row and lane group
  constexpr int TPR = LPR * S;
  constexpr int RPG = 256 / TPR;
  constexpr int CH = kSpmmChunk * CPT;   // matrix blocks staged in LDS at a time
  constexpr int U = kSpmmUnroll;
  constexpr int R = kSpmmStage;
  static_assert(KB % CPT == 0, "tile narrower than one lane");
  __shared__ T sv[CH * 9];
  __shared__ int32_t sc[CH];
  __shared__ V red[3][S > 1 ? 256 : 1];
  __shared__ double sm[DOT ? CPT : 1][DOT ? 256 : 1];
  if (bdone(ctrl)) return;              // the same for every thread of the grid
  // XCD x (workgroups are dealt to the 8 XCDs round-robin) owns one contiguous
  // range of row groups, and its workgroups take that range round-robin, so
  // the groups in flight on one XCD are neighbours and share gathered x rows
  // in its L2 and the MALL.
  const int32_t ngroups = (n + RPG - 1) / RPG;
  const int32_t nb = gridDim.x, xcd = blockIdx.x & 7, per = nb >> 3, rem = nb & 7;
  const int32_t nwx = per + (xcd < rem ? 1 : 0), wi = blockIdx.x >> 3;
  const int32_t gx0 = (int32_t)((int64_t)ngroups * xcd / 8), gx1 = (int32_t)((int64_t)ngroups * (xcd + 1) / 8);
  const int32_t w = blockIdx.x;          // this workgroup's partial slot
  const int lane = threadIdx.x % LPR, sp = (threadIdx.x / LPR) % S, lr = threadIdx.x / TPR;
  const int32_t j = blockIdx.y * KB + lane * CPT;
  double d[CPT];
#pragma unroll
  for (int q = 0; q < CPT; q++) d[q] = 0.0;
  for (int32_t g = gx0 + wi; g < gx1; g += nwx) {
    const int32_t r0 = g * RPG, row = r0 + lr;
    const int32_t b0 = rp[r0], b1 = rp[min(r0 + RPG, n)];
    const int32_t mb0 = row < n ? rp[row] : 0, mb1 = row < n ? rp[row + 1] : 0;
    V a0 = (V)0, a1 = (V)0, a2 = (V)0;
    for (int32_t cb = b0; cb < b1; cb += CH) {
      const int32_t cn = min(CH, b1 - cb);
      // staging: R loads per thread are issued before the first LDS store,
      // so a chunk costs one memory latency per 256 R entries, not one per 256
      const T *vsrc = val + (size_t)cb * 9;
      for (int i0 = threadIdx.x; i0 < cn * 9; i0 += 256 * R) {
        T t[R];
#pragma unroll
        for (int r = 0; r < R; r++) t[r] = i0 + 256 * r < cn * 9 ? vsrc[i0 + 256 * r] : (T)0;
#pragma unroll
        for (int r = 0; r < R; r++)
          if (i0 + 256 * r < cn * 9) sv[i0 + 256 * r] = t[r];
      }
      for (int i = threadIdx.x; i < cn; i += 256) sc[i] = col[cb + i];
      __syncthreads();
      const int32_t lo = max(mb0, cb), hi = min(mb1, cb + cn);
      // first block of this lane group's residue class at or after lo
      const int32_t first = lo + (((sp - (lo - mb0)) % S) + S) % S;
      // Full steps of U blocks issue their 3 U gathers before the first
      // product; the remaining blocks of the row go one at a time.  Products
      // are accumulated in block order either way.
      int32_t b = first;
      for (; b + (U - 1) * S < hi; b += U * S) {
        V x0[U], x1[U], x2[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int32_t c = sc[b + u * S - cb];
          x0[u] = *(const V *)(X + (size_t)(3 * c) * ld + j);
          x1[u] = *(const V *)(X + (size_t)(3 * c + 1) * ld + j);
          x2[u] = *(const V *)(X + (size_t)(3 * c + 2) * ld + j);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
          const T *v = sv + (b + u * S - cb) * 9;
#pragma unroll
          for (int q = 0; q < CPT; q++) {
            a0[q] += v[0] * x0[u][q] + v[1] * x1[u][q] + v[2] * x2[u][q];
            a1[q] += v[3] * x0[u][q] + v[4] * x1[u][q] + v[5] * x2[u][q];
            a2[q] += v[6] * x0[u][q] + v[7] * x1[u][q] + v[8] * x2[u][q];
          }
        }
      }
      for (; b < hi; b += S) {
        const int32_t c = sc[b - cb];
        const T *v = sv + (b - cb) * 9;
        const V x0 = *(const V *)(X + (size_t)(3 * c) * ld + j);
        const V x1 = *(const V *)(X + (size_t)(3 * c + 1) * ld + j);
        const V x2 = *(const V *)(X + (size_t)(3 * c + 2) * ld + j);
#pragma unroll
        for (int q = 0; q < CPT; q++) {
          a0[q] += v[0] * x0[q] + v[1] * x1[q] + v[2] * x2[q];
          a1[q] += v[3] * x0[q] + v[4] * x1[q] + v[5] * x2[q];
          a2[q] += v[6] * x0[q] + v[7] * x1[q] + v[8] * x2[q];
        }
      }
      __syncthreads();
    }
    if (S > 1) {
      red[0][threadIdx.x] = a0;
      red[1][threadIdx.x] = a1;
      red[2][threadIdx.x] = a2;
      __syncthreads();
      if (sp == 0) {
        a0 = a1 = a2 = (V)0;
        for (int q = 0; q < S; q++) {
          a0 += red[0][threadIdx.x + q * LPR];
          a1 += red[1][threadIdx.x + q * LPR];
          a2 += red[2][threadIdx.x + q * LPR];
        }
      }
      __syncthreads();
    }
    if (row < n && sp == 0) {
      const size_t o = (size_t)(3 * row) * ld + j;
      V y0, y1, y2;
      if (HAS_W) {
        // all three rows of W before the first store (Y may be W)
        const V w0 = *(const V *)(W + o), w1 = *(const V *)(W + o + ld), w2 = *(const V *)(W + o + 2 * ld);
        y0 = alpha * a0 + w0;
        y1 = alpha * a1 + w1;
        y2 = alpha * a2 + w2;
      } else {
        y0 = alpha * a0;
        y1 = alpha * a1;
        y2 = alpha * a2;
      }
      *(V *)(Y + o) = y0;
      *(V *)(Y + o + ld) = y1;
      *(V *)(Y + o + 2 * ld) = y2;
      if (DOT) {
        const V x0 = *(const V *)(X + o), x1 = *(const V *)(X + o + ld), x2 = *(const V *)(X + o + 2 * ld);
#pragma unroll
        for (int q = 0; q < CPT; q++)
          d[q] += ((double)x0[q] * a0[q] + (double)x1[q] * a1[q]) + (double)x2[q] * a2[q];
      }
    }
  }
  if (DOT) {
#pragma unroll
    for (int q = 0; q < CPT; q++) sm[q][threadIdx.x] = d[q];   // zero on the lanes of groups s > 0
    __syncthreads();
    if (threadIdx.x < KB) {
      const int ln = threadIdx.x / CPT, q = threadIdx.x % CPT;
      double s = 0.0;
      for (int r = 0; r < RPG; r++) s += sm[q][r * TPR + ln];
      part[(size_t)w * ld + blockIdx.y * KB + threadIdx.x] = s;
    }
  }
}

// Z = D Y for a dense row-major FP64 operator (the coarsest inverse or the
// dense tail), one thread per (row, column); the 256 / ld rows of a block share
// Y through the cache.  Four independent partial sums keep four loads of D and
// Y in flight per thread instead of one dependent chain of nd.
template <typename T>
__global__ void __launch_bounds__(256) k_dense_gemm(int32_t nd, const double *__restrict__ inv,
                                                    const T *__restrict__ Y, T *__restrict__ Z, int32_t ld,
                                                    const BatchCtrl *ctrl) {
  if (bdone(ctrl)) return;
  const int32_t t = blockIdx.x * 256 + threadIdx.x;
  const int32_t row = t / ld, j = t % ld;
  if (row >= nd) return;
  const double *a = inv + (size_t)row * nd;
  const T *y = Y + j;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int32_t i = 0;
  for (; i + 3 < nd; i += 4) {
    s0 += a[i] * (double)y[(size_t)i * ld];
    s1 += a[i + 1] * (double)y[(size_t)(i + 1) * ld];
    s2 += a[i + 2] * (double)y[(size_t)(i + 2) * ld];
    s3 += a[i + 3] * (double)y[(size_t)(i + 3) * ld];
  }
  for (; i < nd; i++) s0 += a[i] * (double)y[(size_t)i * ld];
  Z[(size_t)row * ld + j] = (T)((s0 + s1) + (s2 + s3));
}

// Column-wise vector kernels: a 256-thread block is (256/ld) dof rows x ld
// columns; every block walks dof rows with a grid stride and leaves one
// partial per column, summed later in block order.
__device__ __forceinline__ void col_partial(double v, double *sm, double *part, int32_t ld, int slot) {
  sm[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < ld) {
    double s = 0.0;
    for (int r = 0; r < 256 / ld; r++) s += sm[r * ld + threadIdx.x];
    part[((size_t)slot * gridDim.x + blockIdx.x) * ld + threadIdx.x] = s;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_col_dot(int64_t nrow, const double *__restrict__ A,
                                                 const double *__restrict__ B, int32_t ld, double *__restrict__ part,
                                                 const BatchCtrl *ctrl) {
  __shared__ double sm[256];
  if (bdone(ctrl)) return;
  const int rpb = 256 / ld, r0 = threadIdx.x / ld, j = threadIdx.x % ld;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * rpb + r0; i < nrow; i += (int64_t)gridDim.x * rpb)
    s += A[i * ld + j] * B[i * ld + j];
  col_partial(s, sm, part, ld, 0);
}

// z (z_old here) is read in the cycle precision TC; Rc (optional) receives r
// in that precision, the next cycle's input.
template <typename TC>
__global__ void __launch_bounds__(256) k_col_update(int64_t nrow, double *__restrict__ U, double *__restrict__ R,
                                                    const double *__restrict__ P, const double *__restrict__ Q,
                                                    const TC *__restrict__ Z, TC *__restrict__ Rc, int32_t ld,
                                                    double *__restrict__ part, const BatchCtrl *ctrl) {
  __shared__ double sm[256];
  if (bdone(ctrl)) return;
  const int rpb = 256 / ld, r0 = threadIdx.x / ld, j = threadIdx.x % ld;
  const double alpha = ctrl->alpha[j];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * rpb + r0; i < nrow; i += (int64_t)gridDim.x * rpb) {
    const int64_t o = i * ld + j;
    U[o] += alpha * P[o];
    const double ri = R[o] - alpha * Q[o];
    R[o] = ri;
    if (Rc) Rc[o] = (TC)ri;
    s1 += ri * ri;
    s2 += ri * (double)Z[o];
  }
  col_partial(s1, sm, part, ld, 0);
  col_partial(s2, sm, part, ld, 1);
}

// r.z partials per column, z in the cycle precision
template <typename TZ>
__global__ void __launch_bounds__(256) k_col_rz(int64_t nrow, const double *__restrict__ R,
                                                const TZ *__restrict__ Z, int32_t ld, double *__restrict__ part,
                                                const BatchCtrl *ctrl) {
  __shared__ double sm[256];
  if (bdone(ctrl)) return;
  const int rpb = 256 / ld, r0 = threadIdx.x / ld, j = threadIdx.x % ld;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * rpb + r0; i < nrow; i += (int64_t)gridDim.x * rpb) {
    const int64_t o = i * ld + j;
    s += R[o] * (double)Z[o];
  }
  col_partial(s, sm, part, ld, 0);
}

template <typename TZ>
__global__ void __launch_bounds__(256) k_col_pupdate(int64_t n, const TZ *__restrict__ Z, double *__restrict__ P,
                                                     int32_t ld, const BatchCtrl *ctrl) {
  if (bdone(ctrl)) return;
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < n; o += (int64_t)gridDim.x * 256)
    P[o] = (double)Z[o] + ctrl->beta[o % ld] * P[o];
}

// Per-column scalar steps; thread j owns column j.  A finished column gets
// alpha = 0 (its iterate is frozen) and keeps the iteration count at which it
// stopped.  all_done is raised when every column is finished.
__global__ void __launch_bounds__(1024) k_col_finish(int mode, const double *__restrict__ part, int nparts,
                                                     int32_t ld, BatchCtrl *ctrl) {
  __shared__ int32_t open[64];
  __shared__ double t0[1024], t1[1024];
  if (ctrl->all_done) return;
  // 1024/ld threads per column each sum a strided share of the partials, then
  // thread j adds the shares of column j in order (ld divides 1024)
  const int t = threadIdx.x, nr = 1024 / ld;
  {
    const int jj = t % ld, q0 = t / ld;
    double a = 0.0, b = 0.0;
    for (int q = q0; q < nparts; q += nr) a += part[(size_t)q * ld + jj];
    if (mode == kFinRr)
      for (int q = q0; q < nparts; q += nr) b += part[((size_t)nparts + q) * ld + jj];
    t0[t] = a;
    t1[t] = b;
  }
  if (t < 64) open[t] = 0;
  __syncthreads();
  const int j = t;
  if (j < ld) {
    double s0 = 0.0, s1 = 0.0;
    for (int q = 0; q < nr; q++) {
      s0 += t0[q * ld + j];
      s1 += t1[q * ld + j];
    }
    const bool dn = ctrl->done[j] != 0;
    switch (mode) {
      case kFinInitF:
        ctrl->fnorm[j] = sqrt(s0);
        ctrl->iter[j] = 0;
        ctrl->relres[j] = 0.0;
        if (!(s0 == s0)) { ctrl->status[j] = ASPAMG_ENAN; ctrl->done[j] = 1; }
        else if (s0 == 0.0) { ctrl->status[j] = ASPAMG_OK; ctrl->done[j] = 1; }
        else { ctrl->status[j] = ASPAMG_NOT_CONVERGED; ctrl->relres[j] = 1.0; }
        break;
      case kFinInitRz:
        ctrl->rz[j] = s0;
        if (!dn && !(s0 > 0.0)) { ctrl->status[j] = (s0 == s0) ? ASPAMG_EBREAKDOWN : ASPAMG_ENAN; ctrl->done[j] = 1; }
        break;
      case kFinAlpha:
        if (dn) { ctrl->alpha[j] = 0.0; break; }
        if (!(s0 > 0.0)) {
          ctrl->status[j] = (s0 == s0) ? ASPAMG_EBREAKDOWN : ASPAMG_ENAN;
          ctrl->done[j] = 1;
          ctrl->alpha[j] = 0.0;
        } else {
          ctrl->alpha[j] = ctrl->rz[j] / s0;
        }
        break;
      case kFinRr:
        if (dn) break;
        ctrl->rzo[j] = s1;
        ctrl->iter[j] += 1;
        ctrl->relres[j] = sqrt(s0) / ctrl->fnorm[j];
        if (!(s0 == s0)) { ctrl->status[j] = ASPAMG_ENAN; ctrl->done[j] = 1; }
        else if (sqrt(s0) <= ctrl->rtol * ctrl->fnorm[j]) { ctrl->status[j] = ASPAMG_OK; ctrl->done[j] = 1; }
        else if (ctrl->iter[j] >= ctrl->max_it) { ctrl->done[j] = 1; }
        break;
      case kFinBeta:
        if (dn) { ctrl->beta[j] = 0.0; break; }
        if (!(s0 > 0.0)) {
          ctrl->status[j] = (s0 == s0) ? ASPAMG_EBREAKDOWN : ASPAMG_ENAN;
          ctrl->done[j] = 1;
          ctrl->beta[j] = 0.0;
        } else {
          ctrl->beta[j] = (s0 - ctrl->rzo[j]) / ctrl->rz[j];
          ctrl->rz[j] = s0;
        }
        break;
    }
    open[j] = ctrl->done[j] ? 0 : 1;
  }
  __syncthreads();
  if (j == 0) {
    int any = 0;
    for (int q = 0; q < 64; q++) any += open[q];
    if (any == 0) ctrl->all_done = 1;
  }
}

__global__ void __launch_bounds__(256) k_copy_cols(int64_t nrow, int32_t k, const double *__restrict__ src, int64_t lds,
                                                   double *__restrict__ dst, int64_t ldd, int32_t kfill) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < nrow * kfill; t += (int64_t)gridDim.x * 256) {
    const int64_t i = t / kfill, j = t % kfill;
    dst[i * ldd + j] = j < k ? src[i * lds + j] : 0.0;
  }
}

// S[i][j] = |F[i][j]| + sum_k |A_ik| |U[k][j]| for the k columns (the
// componentwise bound of evaluating F - A U; rounding floor of the true
// residual).  One thread per (scalar row, column); the row's blocks are read
// by the k threads of the row from cache.
__global__ void __launch_bounds__(256) k_abs_bound_cols(int32_t n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        const double *__restrict__ v,
                                                        const double *__restrict__ U, const double *__restrict__ F,
                                                        int32_t ld, int32_t k, double *__restrict__ S) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = t / k;
  const int32_t j = (int32_t)(t % k);
  if (i >= (int64_t)n * 3) return;
  const int32_t I = (int32_t)(i / 3);
  const int d = (int)(i % 3);
  double a = 0.0;
  for (int32_t b = rp[I]; b < rp[I + 1]; b++) {
    const int32_t c = ci[b];
    const double *blk = v + (size_t)b * 9 + d * 3;
    a += fabs(blk[0]) * fabs(U[(size_t)(3 * c) * ld + j]) + fabs(blk[1]) * fabs(U[(size_t)(3 * c + 1) * ld + j]) +
         fabs(blk[2]) * fabs(U[(size_t)(3 * c + 2) * ld + j]);
  }
  S[(size_t)i * ld + j] = fabs(F[(size_t)i * ld + j]) + a;
}

}  // namespace

int batch_vec_blocks(int64_t nrow, int ld) {
  const int64_t rpb = 256 / ld;
  int64_t b = (nrow + rpb - 1) / rpb;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

// workgroups of a product over n rows in row groups of 256 cpt / (kb split)
// (cpt columns per lane): at most cap
static int spmm_wgs(int32_t n, int kb, int split, int cpt, int cap) {
  const int rpg = 256 * cpt / (kb * split);
  const int64_t groups = ((int64_t)n + rpg - 1) / rpg;
  return (int)std::max<int64_t>(1, std::min<int64_t>(groups, cap));
}

// Workgroups of one instantiation that the device holds at once (its compute
// units times the occupancy the kernel's LDS and registers allow), looked up
// once per instantiation.  A grid of exactly that many workgroups walks each
// XCD's row groups as one contiguous front; more workgroups than fit would
// each jump through the range in strides of the grid and scatter the rows in
// flight, whose gathered x rows then miss L2.
template <typename T, bool HAS_W, bool DOT, int KB, int S>
static int spmm_resident() {
  static int cached = 0;
  if (!cached) {
    int dev = 0, cus = 0, per = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_bsr_spmm<T, HAS_W, DOT, KB, S>, 256, 0));
    cached = std::max(8, cus * std::max(per, 1));
  }
  return cached;
}

template <typename T, bool HAS_W, bool DOT, int KB, int S>
static void spmm_ks(const DevBSRT<T> &A, const T *X, T *Y, const T *W, int ld, double alpha, double *part,
                    const BatchCtrl *c, hipStream_t s) {
  constexpr int CPT = 16 / sizeof(T);
  // every lane loads and stores CPT columns as one 16-byte vector
  const uintptr_t mis = (uintptr_t)X | (uintptr_t)Y | (uintptr_t)W;
  if ((mis & 15) != 0 || ld % CPT != 0) fail(ASPAMG_EINVAL, "SpMM operands must be 16-byte aligned column tiles");
  const int cap = std::min(DOT ? kBatchParts : 4096, spmm_resident<T, HAS_W, DOT, KB, S>() / (ld / KB));
  dim3 grid((unsigned)spmm_wgs(A.n, KB, S, CPT, std::max(cap, 8)), ld / KB);
  hipLaunchKernelGGL((k_bsr_spmm<T, HAS_W, DOT, KB, S>), grid, dim3(256), 0, s, A.n, A.rp, A.ci, A.v, X, Y, W, ld,
                     (T)alpha, part, c);
}

template <typename T, bool HAS_W, bool DOT, int KB>
static void spmm_k(const DevBSRT<T> &A, const T *X, T *Y, const T *W, int ld, double alpha, double *part,
                   const BatchCtrl *c, hipStream_t s) {
  switch (A.split) {
    case 1: spmm_ks<T, HAS_W, DOT, KB, 1>(A, X, Y, W, ld, alpha, part, c, s); break;
    case 2: spmm_ks<T, HAS_W, DOT, KB, 2>(A, X, Y, W, ld, alpha, part, c, s); break;
    case 4: spmm_ks<T, HAS_W, DOT, KB, 4>(A, X, Y, W, ld, alpha, part, c, s); break;
    case 8: spmm_ks<T, HAS_W, DOT, KB, 8>(A, X, Y, W, ld, alpha, part, c, s); break;
    default: fail(ASPAMG_EINVAL, "SpMM row split must be 1, 2, 4 or 8");
  }
}

template <typename T, bool HAS_W, bool DOT>
static void spmm_any(const DevBSRT<T> &A, const T *X, T *Y, const T *W, int ld, int kb, double alpha, double *part,
                     const BatchCtrl *c, hipStream_t s) {
  switch (kb) {
    case 4: spmm_k<T, HAS_W, DOT, 4>(A, X, Y, W, ld, alpha, part, c, s); break;
    case 8: spmm_k<T, HAS_W, DOT, 8>(A, X, Y, W, ld, alpha, part, c, s); break;
    case 16: spmm_k<T, HAS_W, DOT, 16>(A, X, Y, W, ld, alpha, part, c, s); break;
    case 32: spmm_k<T, HAS_W, DOT, 32>(A, X, Y, W, ld, alpha, part, c, s); break;
    default: fail(ASPAMG_EINVAL, "SpMM tile must be 4, 8, 16 or 32 columns");
  }
}

template <typename T>
void launch_spmm(const DevBSRT<T> &A, const T *X, T *Y, const T *W, int ld, int kb, double alpha,
                 const BatchCtrl *c, hipStream_t s) {
  if (A.n == 0) return;
  kb = kb > ld ? ld : kb;
  if (W) spmm_any<T, true, false>(A, X, Y, W, ld, kb, alpha, nullptr, c, s);
  else spmm_any<T, false, false>(A, X, Y, W, ld, kb, alpha, nullptr, c, s);
}
template void launch_spmm<double>(const DevBSRT<double> &, const double *, double *, const double *, int, int, double,
                                  const BatchCtrl *, hipStream_t);
template void launch_spmm<float>(const DevBSRT<float> &, const float *, float *, const float *, int, int, double,
                                 const BatchCtrl *, hipStream_t);

void launch_spmm_dot(const DevBSRT<double> &A, const double *X, double *Y, int ld, int kb, double *part,
                     const BatchCtrl *c, hipStream_t s) {
  kb = kb > ld ? ld : kb;
  spmm_any<double, false, true>(A, X, Y, nullptr, ld, kb, 1.0, part, c, s);
}
// workgroups (= partial slots) of launch_spmm_dot's grid, as spmm_ks sizes it
template <int KB, int S>
static int dot_grid(const DevBSRT<double> &A, int ld) {
  const int cap = std::min(kBatchParts, spmm_resident<double, false, true, KB, S>() / (ld / KB));
  return spmm_wgs(A.n, KB, S, 16 / (int)sizeof(double), std::max(cap, 8));
}
template <int KB>
static int dot_grid_k(const DevBSRT<double> &A, int ld) {
  switch (A.split) {
    case 1: return dot_grid<KB, 1>(A, ld);
    case 2: return dot_grid<KB, 2>(A, ld);
    case 4: return dot_grid<KB, 4>(A, ld);
    case 8: return dot_grid<KB, 8>(A, ld);
  }
  fail(ASPAMG_EINVAL, "SpMM row split must be 1, 2, 4 or 8");
}
int spmm_dot_parts(const DevBSRT<double> &A, int ld, int kb) {
  kb = kb > ld ? ld : kb;
  switch (kb) {
    case 4: return dot_grid_k<4>(A, ld);
    case 8: return dot_grid_k<8>(A, ld);
    case 16: return dot_grid_k<16>(A, ld);
    case 32: return dot_grid_k<32>(A, ld);
  }
  fail(ASPAMG_EINVAL, "SpMM tile must be 4, 8, 16 or 32 columns");
}

template <typename T>
void launch_dense_gemm(int nd, const double *inv, const T *Y, T *Z, int ld, const BatchCtrl *c, hipStream_t s) {
  const int64_t threads = (int64_t)nd * ld;
  hipLaunchKernelGGL(k_dense_gemm<T>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, nd, inv, Y, Z, ld, c);
}
template void launch_dense_gemm<double>(int, const double *, const double *, double *, int, const BatchCtrl *,
                                        hipStream_t);
template void launch_dense_gemm<float>(int, const double *, const float *, float *, int, const BatchCtrl *,
                                       hipStream_t);

void launch_col_dot(int64_t nrow, const double *A, const double *B, int ld, double *part, const BatchCtrl *c,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_col_dot, dim3(batch_vec_blocks(nrow, ld)), dim3(256), 0, s, nrow, A, B, ld, part, c);
}
template <typename TC>
void launch_col_update(int64_t nrow, double *U, double *R, const double *P, const double *Q, const TC *Z, TC *Rc,
                       int ld, double *part, const BatchCtrl *c, hipStream_t s) {
  hipLaunchKernelGGL(k_col_update<TC>, dim3(batch_vec_blocks(nrow, ld)), dim3(256), 0, s, nrow, U, R, P, Q, Z, Rc,
                     ld, part, c);
}
template void launch_col_update<double>(int64_t, double *, double *, const double *, const double *, const double *,
                                        double *, int, double *, const BatchCtrl *, hipStream_t);
template void launch_col_update<float>(int64_t, double *, double *, const double *, const double *, const float *,
                                       float *, int, double *, const BatchCtrl *, hipStream_t);
template <typename TZ>
void launch_col_rz(int64_t nrow, const double *R, const TZ *Z, int ld, double *part, const BatchCtrl *c,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_col_rz<TZ>, dim3(batch_vec_blocks(nrow, ld)), dim3(256), 0, s, nrow, R, Z, ld, part, c);
}
template void launch_col_rz<double>(int64_t, const double *, const double *, int, double *, const BatchCtrl *,
                                    hipStream_t);
template void launch_col_rz<float>(int64_t, const double *, const float *, int, double *, const BatchCtrl *,
                                   hipStream_t);
template <typename TZ>
void launch_col_pupdate(int64_t nrow, const TZ *Z, double *P, int ld, const BatchCtrl *c, hipStream_t s) {
  const int64_t n = nrow * ld;
  int64_t b = (n + 255) / 256;
  if (b > 2048) b = 2048;
  hipLaunchKernelGGL(k_col_pupdate<TZ>, dim3((unsigned)b), dim3(256), 0, s, n, Z, P, ld, c);
}
template void launch_col_pupdate<double>(int64_t, const double *, double *, int, const BatchCtrl *, hipStream_t);
template void launch_col_pupdate<float>(int64_t, const float *, double *, int, const BatchCtrl *, hipStream_t);
void launch_col_finish(int mode, const double *part, int nparts, int ld, BatchCtrl *c, hipStream_t s) {
  if (ld < 1 || ld > 64 || 1024 % ld != 0) fail(ASPAMG_EINVAL, "column count must divide 1024");
  hipLaunchKernelGGL(k_col_finish, dim3(1), dim3(1024), 0, s, mode, part, nparts, ld, c);
}
void launch_copy_cols(int64_t nrow, int k, const double *src, int64_t lds, double *dst, int64_t ldd, int kfill,
                      hipStream_t s) {
  int64_t b = (nrow * kfill + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)b), dim3(256), 0, s, nrow, k, src, lds, dst, ldd, kfill);
}

void launch_abs_bound_cols(const DevBSRT<double> &A, const double *U, const double *F, int ld, int k, double *S,
                           hipStream_t s) {
  const int64_t nt = (int64_t)A.n * 3 * k;
  hipLaunchKernelGGL(k_abs_bound_cols, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, A.n, A.rp, A.ci, A.v, U, F,
                     ld, k, S);
}

}  // namespace aspamg
