// Setup-phase kernels for gfx950: batched small dense SPD factorisations of the
// FSAI rows (one wavefront per block row, system staged in LDS), the batched
// least-squares solves of the interpolation weights, the two numeric SpGEMM
// phases of the Galerkin product, and the element-level kernels (gradient of a
// quadratic form and element-to-block assembly).
//
// This file is compiled with -ffp-contract=off: every sum runs in ascending
// index order with separately rounded products, so the FSAI rows and the
// Galerkin values are bitwise those of the sequential definition (IEEE
// binary64 +, -, *, / and sqrt are correctly rounded on the device).
#include "device_decisions.h"
#include "internal.h"

namespace aspamg {

namespace {

__device__ __forceinline__ int32_t find_col(const int32_t *ci, int32_t lo, int32_t hi, int32_t c) {
  // binary search in ci[lo, hi), -1 if absent
  hi -= 1;
  while (lo <= hi) {
    const int32_t mid = (lo + hi) >> 1;
    const int32_t v = ci[mid];
    if (v == c) return mid;
    if (v < c) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// One FSAI block row per 64-thread block.  With the local list
// l = [(J,e) for J in B] + [(I,0), (I,1), (I,2)] and M = A[l,l] (block of row
// l_p's node), the left-looking Cholesky M = L L^T is formed in LDS (packed
// lower triangle) with
//   L_jj = sqrt(M_jj - sum_{k<j} L_jk^2),  L_ij = (M_ij - sum_{k<j} L_ik L_jk) / L_jj,
// each sum in ascending k.  Scalar row d is g = L_md^{-T} e_md (md = 3|B|+d+1),
// obtained by back substitution with sums in ascending j, and psi_d = L_md,md^2.
__device__ __forceinline__ int tri(int i, int j) { return (i * (i + 1) >> 1) + j; }

__global__ void __launch_bounds__(64) k_fsai_rows(int32_t nrows, const int32_t *__restrict__ rows,
                                                  const int32_t *__restrict__ pat_ptr,
                                                  const int32_t *__restrict__ pat_nodes,
                                                  const int32_t *__restrict__ Arp, const int32_t *__restrict__ Aci,
                                                  const double *__restrict__ Av, int b, int mmax,
                                                  double *__restrict__ gout, double *__restrict__ psi, int32_t *fail) {
  extern __shared__ double L[];         // packed lower triangle, m(m+1)/2
  __shared__ int32_t nodes[kMaxFsaiNodes + 1];
  __shared__ int bad;
  const int32_t r = blockIdx.x;
  if (r >= nrows) return;
  const int lane = threadIdx.x;
  const int32_t I = rows[r];
  const int32_t p0 = pat_ptr[r], nb = pat_ptr[r + 1] - p0;
  const int m = b * nb + b;
  for (int q = lane; q <= nb; q += 64) nodes[q] = q < nb ? pat_nodes[p0 + q] : I;
  if (lane == 0) bad = 0;
  __syncthreads();
  // gather the lower triangle of M (node blocks p >= q)
  const int npairs = (nb + 1) * (nb + 1);
  for (int pq = lane; pq < npairs; pq += 64) {
    const int p = pq / (nb + 1), q = pq % (nb + 1);
    if (q > p) continue;
    const int32_t rn = nodes[p], cn = nodes[q];
    const int32_t k = find_col(Aci, Arp[rn], Arp[rn + 1], cn);
    const double *B = k >= 0 ? Av + (size_t)k * b * b : nullptr;
    for (int d = 0; d < b; d++)
      for (int e = 0; e < b; e++) {
        if (p == q && e > d) continue;
        L[tri(p * b + d, q * b + e)] = B ? B[d * b + e] : 0.0;
      }
  }
  __syncthreads();
  for (int j = 0; j < m; j++) {
    if (lane == 0) {
      double acc = 0.0;
      for (int k = 0; k < j; k++) acc += L[tri(j, k)] * L[tri(j, k)];
      const double d = L[tri(j, j)] - acc;
      if (!(d > 0.0)) bad = 1;
      L[tri(j, j)] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double ljj = L[tri(j, j)];
    for (int i = j + 1 + lane; i < m; i += 64) {
      double acc = 0.0;
      for (int k = 0; k < j; k++) acc += L[tri(i, k)] * L[tri(j, k)];
      L[tri(i, j)] = (L[tri(i, j)] - acc) / ljj;
    }
    __syncthreads();
  }
  if (bad) {
    if (lane == 0) *fail = 1;
    return;
  }
  if (lane < b) {
    const int d = lane;
    const int md = b * nb + d + 1;
    // compact output: the scalar rows of chunk row r start at b (b pat_ptr[r]
    // + b r), each b nb + b entries long (md used, the rest zero)
    const int rs = b * nb + b;
    double *g = gout + (size_t)b * (b * (size_t)p0 + b * (size_t)r) + (size_t)d * rs;
    const double lmm = L[tri(md - 1, md - 1)];
    g[md - 1] = 1.0 / lmm;
    for (int k = md - 2; k >= 0; k--) {
      double acc = 0.0;
      for (int jj = k + 1; jj < md; jj++) acc += L[tri(jj, k)] * g[jj];
      g[k] = -acc / L[tri(k, k)];
    }
    for (int k = md; k < rs; k++) g[k] = 0.0;
    psi[(size_t)r * b + d] = lmm * lmm;
  }
}

// Interpolation weights of one scalar row: Gram C^T C and C^T v of the chosen
// test-space rows, Cholesky, forward and back substitution (normal equations).
__global__ void __launch_bounds__(256) k_dpls_weights(int32_t nrows, const int32_t *__restrict__ row,
                                                      const int32_t *__restrict__ cnt,
                                                      const int32_t *__restrict__ sel, const double *__restrict__ V,
                                                      int ntv, double *__restrict__ w) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nrows) return;
  const int K = cnt[i];
  const double *v = V + (size_t)row[i] * ntv;
  double Gm[kMaxPEntries][kMaxPEntries], t[kMaxPEntries], y[kMaxPEntries], L[kMaxPEntries][kMaxPEntries];
  for (int a = 0; a < K; a++) {
    const double *ca = V + (size_t)sel[(size_t)i * kMaxPEntries + a] * ntv;
    double s = 0.0;
    for (int q = 0; q < ntv; q++) s += ca[q] * v[q];
    t[a] = s;
    for (int c = 0; c <= a; c++) {
      const double *cc = V + (size_t)sel[(size_t)i * kMaxPEntries + c] * ntv;
      double g = 0.0;
      for (int q = 0; q < ntv; q++) g += ca[q] * cc[q];
      Gm[a][c] = g;
    }
  }
  for (int j = 0; j < K; j++) {
    double acc = 0.0;
    for (int k = 0; k < j; k++) acc += L[j][k] * L[j][k];
    const double d = Gm[j][j] - acc;
    if (!(d > 0.0)) {
      // dependent columns (the kappa guard bounds cond(C^T C) by kappa_p^2, so
      // this is an error): NaN weights, which the host turns into a status
      for (int a = 0; a < K; a++) w[(size_t)i * kMaxPEntries + a] = __builtin_nan("");
      return;
    }
    L[j][j] = sqrt(d);
    for (int a = j + 1; a < K; a++) {
      double a2 = 0.0;
      for (int k = 0; k < j; k++) a2 += L[a][k] * L[j][k];
      L[a][j] = (Gm[a][j] - a2) / L[j][j];
    }
  }
  for (int a = 0; a < K; a++) {
    double acc = 0.0;
    for (int c = 0; c < a; c++) acc += L[a][c] * y[c];
    y[a] = (t[a] - acc) / L[a][a];
  }
  double ww[kMaxPEntries];
  for (int a = K - 1; a >= 0; a--) {
    double acc = 0.0;
    for (int c = a + 1; c < K; c++) acc += L[c][a] * ww[c];
    ww[a] = (y[a] - acc) / L[a][a];
  }
  for (int a = 0; a < K; a++) w[(size_t)i * kMaxPEntries + a] = ww[a];
}

// acc += X * Y for b x b blocks, each entry ((x0 y0 + x1 y1) + x2 y2) for b = 3.
// The block size is a template argument in the kernels below: their small
// accumulator arrays then stay in registers.
template <int b>
__device__ __forceinline__ void blk_mac(const double *X, const double *Y, double *acc) {
#pragma unroll
  for (int d = 0; d < b; d++)
#pragma unroll
    for (int e = 0; e < b; e++) {
      double s = X[d * b] * Y[e];
      for (int k = 1; k < b; k++) s += X[d * b + k] * Y[k * b + e];
      acc[d * b + e] += s;
    }
}

__device__ __forceinline__ int32_t row_of(const int32_t *rp, int32_t n, int32_t q) {
  // row containing position q (rp ascending)
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (rp[mid] <= q) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// T = A P with the pattern of T fixed: block (K, J) sums A_KL P_LJ over the
// blocks L of A's row K in ascending order.  One thread per block of T.
template <int b>
__global__ void __launch_bounds__(256) k_spgemm_ap(int32_t n, const int32_t *__restrict__ Arp,
                                                   const int32_t *__restrict__ Aci, const double *__restrict__ Av,
                                                   const int32_t *__restrict__ Prp, const int32_t *__restrict__ Pci,
                                                   const double *__restrict__ Pv, const int32_t *__restrict__ Trp,
                                                   const int32_t *__restrict__ Tci, double *__restrict__ Tv,
                                                   int64_t nnzT) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nnzT) return;
  const int32_t K = row_of(Trp, n, (int32_t)q);
  const int32_t J = Tci[q];
  constexpr int bb = b * b;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int32_t a = Arp[K]; a < Arp[K + 1]; a++) {
    const int32_t Lr = Aci[a];
    for (int32_t t = Prp[Lr]; t < Prp[Lr + 1]; t++) {
      if (Pci[t] == J) {
        blk_mac<b>(Av + (size_t)a * bb, Pv + (size_t)t * bb, acc);
        break;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < bb; k++) Tv[q * bb + k] = acc[k];
}

// A_c = R T: block (I, J) sums R_IK T_KJ over the blocks K of R's row I in
// ascending order.  One thread per block of A_c.
template <int b>
__global__ void __launch_bounds__(256) k_spgemm_rt(int32_t nc, const int32_t *__restrict__ Rrp,
                                                   const int32_t *__restrict__ Rci, const double *__restrict__ Rv,
                                                   const int32_t *__restrict__ Trp, const int32_t *__restrict__ Tci,
                                                   const double *__restrict__ Tv, const int32_t *__restrict__ Crp,
                                                   const int32_t *__restrict__ Cci, double *__restrict__ Cv,
                                                   int64_t nnzC) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nnzC) return;
  const int32_t I = row_of(Crp, nc, (int32_t)q);
  const int32_t J = Cci[q];
  constexpr int bb = b * b;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int32_t a = Rrp[I]; a < Rrp[I + 1]; a++) {
    const int32_t K = Rci[a];
    const int32_t t = find_col(Tci, Trp[K], Trp[K + 1], J);
    if (t >= 0) blk_mac<b>(Rv + (size_t)a * bb, Tv + (size_t)t * bb, acc);
  }
#pragma unroll
  for (int k = 0; k < bb; k++) Cv[q * bb + k] = acc[k];
}

// grad_e = -scale_e * lam_e^T K_e^0 u_e, one thread per element; a shared
// K_e^0 is staged in LDS.
__global__ void __launch_bounds__(256) k_element_gradient(int64_t n_el, const int32_t *__restrict__ conn,
                                                          const double *__restrict__ Ke0, int64_t ke_stride,
                                                          const double *__restrict__ lam,
                                                          const double *__restrict__ u,
                                                          const double *__restrict__ scale,
                                                          double *__restrict__ grad) {
  __shared__ double ks[576];
  if (ke_stride == 0)
    for (int i = threadIdx.x; i < 576; i += 256) ks[i] = Ke0[i];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_el) return;
  const double *K = ke_stride == 0 ? ks : Ke0 + e * ke_stride;
  double ue[24], le[24];
#pragma unroll
  for (int a = 0; a < 8; a++) {
    const int32_t nd = conn[e * 8 + a];
#pragma unroll
    for (int c = 0; c < 3; c++) {
      ue[a * 3 + c] = u[(size_t)nd * 3 + c];
      le[a * 3 + c] = lam[(size_t)nd * 3 + c];
    }
  }
  double s = 0.0;
  for (int i = 0; i < 24; i++) {
    double ku = 0.0;
#pragma unroll
    for (int j = 0; j < 24; j++) ku += K[i * 24 + j] * ue[j];
    s += le[i] * ku;
  }
  grad[e] = scale ? -(scale[e] * s) : -s;
}

// vals[slot] = sum over the slot's contributions (ascending element) of
// E_e * K_e^0[3a+d][3b+e]; constrained diagonal slots are I3.
__global__ void __launch_bounds__(256) k_assemble(int64_t nnzb, const int64_t *__restrict__ slot_ptr,
                                                  const int32_t *__restrict__ contrib,
                                                  const int8_t *__restrict__ diag_id,
                                                  const double *__restrict__ Ke0, int64_t ke_stride,
                                                  const double *__restrict__ E, double *__restrict__ vals) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= nnzb) return;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (diag_id[s]) {
    acc[0] = acc[4] = acc[8] = 1.0;
  } else {
    for (int64_t c = slot_ptr[s]; c < slot_ptr[s + 1]; c++) {
      const int32_t el = contrib[2 * c], ab = contrib[2 * c + 1];
      const int a = ab >> 3, b = ab & 7;
      const double *K = Ke0 + (size_t)el * ke_stride;
      const double Ee = E[el];
#pragma unroll
      for (int d = 0; d < 3; d++)
#pragma unroll
        for (int e = 0; e < 3; e++) acc[d * 3 + e] += Ee * K[(a * 3 + d) * 24 + b * 3 + e];
    }
  }
  for (int k = 0; k < 9; k++) vals[s * 9 + k] = acc[k];
}

// Y = alpha (M X) + W for a block-sparse M (row-major b x b blocks, block
// CSR) and row-major multi-vectors with nb columns ([b rows][nb]); one thread
// per block row and column, blocks summed in stored order.  W may alias Y.
template <int b>
__global__ void __launch_bounds__(256) k_bsr_mm(int32_t n, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                const double *__restrict__ X, double *Y, const double *W,
                                                double alpha, int32_t nb) {
  const int32_t c = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
  if (c >= nb || i >= n) return;
  double a[3] = {0.0, 0.0, 0.0};
  for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
    const double *blk = v + (size_t)k * b * b;
    const double *xj = X + (size_t)b * ci[k] * nb + c;
#pragma unroll
    for (int d = 0; d < b; d++) {
      double t = blk[d * b] * xj[0];
#pragma unroll
      for (int e = 1; e < b; e++) t += blk[d * b + e] * xj[e * (size_t)nb];
      a[d] += t;
    }
  }
  double *yi = Y + (size_t)b * i * nb + c;
  const double *wi = W ? W + (size_t)b * i * nb + c : nullptr;
#pragma unroll
  for (int d = 0; d < b; d++) yi[d * (size_t)nb] = alpha * a[d] + (wi ? wi[d * (size_t)nb] : 0.0);
}

// Y = D X for a dense row-major nd x nd matrix D and [nd][nb] multi-vectors.
__global__ void __launch_bounds__(256) k_dense_mm(int32_t nd, const double *__restrict__ D,
                                                  const double *__restrict__ X, double *__restrict__ Y, int32_t nb) {
  const int32_t c = blockIdx.x * 256 + threadIdx.x, r = blockIdx.y;
  if (c >= nb || r >= nd) return;
  const double *d = D + (size_t)r * nd;
  double a = 0.0;
  for (int32_t k = 0; k < nd; k++) a += d[k] * X[(size_t)k * nb + c];
  Y[(size_t)r * nb + c] = a;
}

// Layout values from the block values of the source matrix: slot i (slot
// group i / 64, lane i % 64) takes block src = map[i] (its 9 values at the
// lane's places in the group's 16-byte chunk rows and final run), or zeros
// when src < 0.
template <typename T>
__global__ void __launch_bounds__(256) k_scatter_values(int64_t nslots, const int32_t *__restrict__ map,
                                                        const double *__restrict__ v, T *__restrict__ val, int b) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nslots) return;
  const int32_t src = map[i];
  if (b == 1) {                         // scalar operator: one value per slot
    val[i] = src >= 0 ? (T)v[src] : (T)0;
    return;
  }
  constexpr int W = 16 / sizeof(T);   // values per 16-byte chunk
  T *g = val + (i >> 6) * 576;
  const int e = (int)(i & 63);
  const double *blk = src >= 0 ? v + (int64_t)src * 9 : nullptr;
#pragma unroll
  for (int q = 0; q < 8; q++) g[(q / W) * 64 * W + e * W + (q % W)] = blk ? (T)blk[q] : (T)0;
  g[512 + e] = blk ? (T)blk[8] : (T)0;
}

// FP32 copy of FP64 layout values: the same slots, each value rounded, moved
// from the FP64 chunk order (pairs) to the FP32 one (quads).
__global__ void __launch_bounds__(256) k_narrow_values(int64_t nslots, const double *__restrict__ v64,
                                                       float *__restrict__ v32, int b) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nslots) return;
  if (b == 1) {
    v32[i] = (float)v64[i];
    return;
  }
  const double *g = v64 + (i >> 6) * 576;
  float *o = v32 + (i >> 6) * 576;
  const int e = (int)(i & 63);
#pragma unroll
  for (int q = 0; q < 8; q++) o[(q / 4) * 256 + e * 4 + (q % 4)] = (float)g[(q / 2) * 128 + e * 2 + (q % 2)];
  o[512 + e] = (float)g[512 + e];
}

// y += a x and y = x / a (the Lanczos recurrence of the aFSAI set-up)
__global__ void __launch_bounds__(256) k_axpy(int64_t n, double a, const double *__restrict__ x,
                                              double *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] += a * x[i];
}
__global__ void __launch_bounds__(256) k_divided(int64_t n, double a, const double *__restrict__ x,
                                                 double *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = x[i] / a;
}

// position of column c in row r of A (columns ascending), or -1
__device__ __forceinline__ int32_t find_col(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, int32_t r,
                                            int32_t c) {
  int32_t lo = rp[r], hi = rp[r + 1] - 1;
  while (lo <= hi) {
    const int32_t mid = (lo + hi) >> 1, cm = ci[mid];
    if (cm == c) return mid;
    if (cm < c) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// (score, J) precedes (score', J') in the selection order: larger quantised
// score first, then the lower node
__device__ __forceinline__ bool grow_before(double a, int32_t ja, double b, int32_t jb) {
  return a != b ? a > b : ja < jb;
}

// aFSAI pattern growth (Section 3.1, the adaptive step) for the listed block
// rows, one wavefront per row, from the rows' current pattern B (ascending) and
// the scaled rows g that k_fsai_rows wrote for it.  Candidates are the nodes
// J < I outside B adjacent in A to B u {I}; with g' = g / g_last,
//   h_{(I,d),(J,e)} = sum over the pattern index k of A[(J,e), l_k] g'_k
// (summed over k ascending, whichever pattern node found the candidate),
// score_J = sum_d sum_e h^2, quantised.  The rho first candidates in the order
// (score descending, J ascending) are written to add[i*rho ..], -1 padded;
// nothing is added when |B| + rho exceeds kMaxFsaiNodes.  A candidate reached
// from several pattern nodes is scored once, by the pair of its first one.
template <int b>
__global__ void __launch_bounds__(64) k_fsai_grow(int32_t nrows, const int32_t *__restrict__ rows,
                                                  const int32_t *__restrict__ pat_ptr,
                                                  const int32_t *__restrict__ pat_nodes, const double *__restrict__ g,
                                                  const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                  const double *__restrict__ v, int rho, int qbits,
                                                  int32_t *__restrict__ add) {
  constexpr int GS = 3 * kMaxFsaiNodes + 3;
  __shared__ int32_t K[kMaxFsaiNodes + 1];
  __shared__ int32_t off[kMaxFsaiNodes + 2];
  __shared__ double gp[3][GS];
  const int32_t i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= nrows) return;
  const int32_t I = rows[i];
  const int32_t p0 = pat_ptr[i], nb = pat_ptr[i + 1] - p0;
  if (lane < rho) add[(size_t)i * rho + lane] = -1;
  if (nb + rho > kMaxFsaiNodes) return;                 // uniform in the wavefront
  // pattern nodes, then I; the candidate count of each (columns J < I of its row)
  if (lane <= nb) {
    const int32_t Kp = lane < nb ? pat_nodes[p0 + lane] : I;
    K[lane] = Kp;
    int32_t lo = rp[Kp], hi = rp[Kp + 1];
    while (lo < hi) {                                    // first column >= I
      const int32_t mid = (lo + hi) >> 1;
      if (ci[mid] < I) lo = mid + 1;
      else hi = mid;
    }
    off[lane + 1] = lo - rp[Kp];
  }
  // g' rows (compact layout of k_fsai_rows: rows of b nb + b entries)
  const int rs = b * nb + b;
  const double *gi = g + (size_t)b * (b * (size_t)p0 + b * (size_t)i);
  for (int t = lane; t < b * rs; t += 64) {
    const int d = t / rs, k = t % rs, md = b * nb + d + 1;
    if (k < md) gp[d][k] = gi[d * rs + k] / gi[d * rs + md - 1];
  }
  __syncthreads();
  if (lane == 0) {
    off[0] = 0;
    for (int p = 0; p <= nb; p++) off[p + 1] += off[p];
  }
  __syncthreads();
  const int32_t T = off[nb + 1];
  // this lane's best candidates, in selection order
  double bs[kMaxGrowRho];
  int32_t bj[kMaxGrowRho];
  int nbest = 0;
  for (int32_t t = lane; t < T; t += 64) {
    int p = 0;
    while (off[p + 1] <= t) p++;
    const int32_t J = ci[rp[K[p]] + (t - off[p])];
    // outside B (B ascending)
    int lo = 0, hi = nb - 1;
    bool inB = false;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      if (K[mid] == J) { inB = true; break; }
      if (K[mid] < J) lo = mid + 1;
      else hi = mid - 1;
    }
    if (inB) continue;
    // scored by its first pattern node only
    bool first = true;
    for (int q = 0; q < p && first; q++) first = find_col(rp, ci, J, K[q]) < 0;
    if (!first) continue;
    double h[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int q = p; q <= nb; q++) {
      const int32_t pos = find_col(rp, ci, J, K[q]);    // block (J, K_q)
      if (pos < 0) continue;
      const double *blk = v + (size_t)pos * b * b;
#pragma unroll
      for (int d = 0; d < b; d++) {
        const int kend = min(b, b * nb + d + 1 - b * q);
#pragma unroll
        for (int c = 0; c < b; c++) {
          if (c >= kend) break;
          const double gk = gp[d][b * q + c];
#pragma unroll
          for (int e = 0; e < b; e++) h[d * b + e] += blk[e * b + c] * gk;
        }
      }
    }
    double score = 0.0;
#pragma unroll
    for (int d = 0; d < b; d++)
#pragma unroll
      for (int e = 0; e < b; e++) score += h[d * b + e] * h[d * b + e];
    if (!(score > 0.0)) continue;
    const double qs = quantize_dev(score, qbits);
    // insert into this lane's sorted best list (at most rho kept)
    int at = nbest;
    while (at > 0 && grow_before(qs, J, bs[at - 1], bj[at - 1])) at--;
    if (at >= rho) continue;
    for (int m = min(nbest, rho - 1); m > at; m--) {
      bs[m] = bs[m - 1];
      bj[m] = bj[m - 1];
    }
    bs[at] = qs;
    bj[at] = J;
    if (nbest < rho) nbest++;
  }
  // rho rounds: the wavefront's first remaining candidate
  int head = 0;
  for (int r = 0; r < rho; r++) {
    double s = head < nbest ? bs[head] : -1.0;
    int32_t j = head < nbest ? bj[head] : 0x7FFFFFFF;
    int src = lane;
    for (int o = 32; o > 0; o >>= 1) {
      const double s2 = __shfl_xor(s, o, 64);
      const int32_t j2 = __shfl_xor(j, o, 64);
      const int src2 = __shfl_xor(src, o, 64);
      if (grow_before(s2, j2, s, j)) {
        s = s2;
        j = j2;
        src = src2;
      }
    }
    if (s < 0.0) break;                                  // no candidate left (uniform)
    if (lane == src) head++;
    if (lane == 0) add[(size_t)i * rho + r] = j;
  }
}

// Test-space iteration (SRQCG): columns stored one after another, n entries each.
// out = 2 (sz - q z) / f, the gradient of the Rayleigh quotient of z
__global__ void __launch_bounds__(256) k_rq_gradient(int64_t n, double q, double f, const double *__restrict__ sz,
                                                     const double *__restrict__ z, double *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = 2.0 * (sz[i] - q * z[i]) / f;
}
// Partial inner products in the test-space iteration's fixed order: entry
// block b (256 consecutive entries) summed from its first entry by one
// thread; the host adds the block sums from the first block on.
__global__ void __launch_bounds__(256) k_dot256(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                                               double *__restrict__ part) {
  const int64_t blk = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i0 = blk * 256;
  if (i0 >= n) return;
  const int64_t i1 = i0 + 256 < n ? i0 + 256 : n;
  double s = 0.0;
  for (int64_t i = i0; i < i1; i++) s += a[i] * b[i];
  part[blk] = s;
}

// y = M x on a plain block CSR, one thread per block row, each row's
// components summed over its blocks in stored order (the sequential product)
template <int b>
__global__ void __launch_bounds__(256) k_bsr_mv_seq(int32_t n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                   const double *__restrict__ x, double *__restrict__ y) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double a[3] = {0.0, 0.0, 0.0};
  for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
    const double *B = v + (size_t)k * b * b;
    const double *xx = x + (size_t)ci[k] * b;
#pragma unroll
    for (int d = 0; d < b; d++)
#pragma unroll
      for (int e = 0; e < b; e++) a[d] += B[d * b + e] * xx[e];
  }
#pragma unroll
  for (int d = 0; d < b; d++) y[(size_t)i * b + d] = a[d];
}

// y = x + b y
__global__ void __launch_bounds__(256) k_xpby(int64_t n, const double *__restrict__ x, double b,
                                              double *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = x[i] + b * y[i];
}
// Y[:, c] = sum over j ascending of X[:, j] U[j][c] (U row-major nt x nt)
__global__ void __launch_bounds__(256) k_combine_columns(int64_t n, int nt, const double *__restrict__ X,
                                                         const double *__restrict__ U, double *__restrict__ Y) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    for (int c = 0; c < nt; c++) {
      double s = 0.0;
      for (int j = 0; j < nt; j++) s += X[(size_t)j * n + i] * U[j * nt + c];
      Y[(size_t)c * n + i] = s;
    }
}

// X = the nd x nd identity, row-major
__global__ void __launch_bounds__(256) k_eye(int64_t nd, double *__restrict__ X) {
  const int64_t n = nd * nd;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    X[i] = (i / nd == i % nd) ? 1.0 : 0.0;
}

}  // namespace

void launch_bsr_mm(const DevBSR &M, const double *X, double *Y, const double *W, double alpha, int32_t nb,
                   hipStream_t s) {
  if (M.n == 0 || nb == 0) return;
  const dim3 grid((unsigned)((nb + 255) / 256), (unsigned)M.n);
  if (M.b == 1) hipLaunchKernelGGL(k_bsr_mm<1>, grid, dim3(256), 0, s, M.n, M.rp, M.ci, M.v, X, Y, W, alpha, nb);
  else hipLaunchKernelGGL(k_bsr_mm<3>, grid, dim3(256), 0, s, M.n, M.rp, M.ci, M.v, X, Y, W, alpha, nb);
}

void launch_dense_mm(int32_t nd, const double *D, const double *X, double *Y, int32_t nb, hipStream_t s) {
  if (nd == 0 || nb == 0) return;
  hipLaunchKernelGGL(k_dense_mm, dim3((unsigned)((nb + 255) / 256), (unsigned)nd), dim3(256), 0, s, nd, D, X, Y, nb);
}

template <typename T>
void launch_scatter_values(int64_t nslots, const int32_t *map, const double *v, T *val, int b, hipStream_t s) {
  if (nslots == 0) return;
  hipLaunchKernelGGL(k_scatter_values<T>, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, s, nslots, map, v,
                     val, b);
}
template void launch_scatter_values<double>(int64_t, const int32_t *, const double *, double *, int, hipStream_t);
template void launch_scatter_values<float>(int64_t, const int32_t *, const double *, float *, int, hipStream_t);

void launch_narrow_values(int64_t nslots, const double *v64, float *v32, int b, hipStream_t s) {
  if (nslots == 0) return;
  hipLaunchKernelGGL(k_narrow_values, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, s, nslots, v64, v32, b);
}

static unsigned setup_vec_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 2048);
}
void launch_axpy(int64_t n, double a, const double *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(setup_vec_blocks(n)), dim3(256), 0, s, n, a, x, y);
}
void launch_divided(int64_t n, double a, const double *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_divided, dim3(setup_vec_blocks(n)), dim3(256), 0, s, n, a, x, y);
}

void launch_rq_gradient(int64_t n, double q, double f, const double *sz, const double *z, double *out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_rq_gradient, dim3(setup_vec_blocks(n)), dim3(256), 0, s, n, q, f, sz, z, out);
}
int dot256_parts(int64_t n) { return (int)((n + 255) / 256); }
void launch_dot256(int64_t n, const double *a, const double *b, double *part, hipStream_t s) {
  const int64_t nb = dot256_parts(n);
  hipLaunchKernelGGL(k_dot256, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, n, a, b, part);
}
void launch_bsr_mv_seq(const DevBSR &M, const double *x, double *y, hipStream_t s) {
  if (M.n == 0) return;
  const dim3 grid((M.n + 255) / 256);
  if (M.b == 1) hipLaunchKernelGGL(k_bsr_mv_seq<1>, grid, dim3(256), 0, s, M.n, M.rp, M.ci, M.v, x, y);
  else hipLaunchKernelGGL(k_bsr_mv_seq<3>, grid, dim3(256), 0, s, M.n, M.rp, M.ci, M.v, x, y);
}
void launch_xpby(int64_t n, const double *x, double b, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_xpby, dim3(setup_vec_blocks(n)), dim3(256), 0, s, n, x, b, y);
}
void launch_combine_columns(int64_t n, int nt, const double *X, const double *U, double *Y, hipStream_t s) {
  hipLaunchKernelGGL(k_combine_columns, dim3(setup_vec_blocks(n)), dim3(256), 0, s, n, nt, X, U, Y);
}

void launch_eye(int32_t nd, double *X, hipStream_t s) {
  const int64_t n = (int64_t)nd * nd;
  const int64_t b = std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096);
  hipLaunchKernelGGL(k_eye, dim3((unsigned)b), dim3(256), 0, s, (int64_t)nd, X);
}

int launch_fsai_rows(const DevBSR &A, int32_t nrows, const int32_t *rows, const int32_t *pat_ptr,
                     const int32_t *pat_nodes, int mmax, double *g, double *psi, int32_t *fail_flag,
                     hipStream_t s) {
  if (nrows == 0) return 0;
  const size_t lds = (size_t)mmax * (mmax + 1) / 2 * sizeof(double);
  hipLaunchKernelGGL(k_fsai_rows, dim3(nrows), dim3(64), lds, s, nrows, rows, pat_ptr, pat_nodes, A.rp, A.ci, A.v,
                     A.b, mmax, g, psi, fail_flag);
  return 0;
}

void launch_fsai_grow(const DevBSR &A, int32_t nrows, const int32_t *rows, const int32_t *pat_ptr,
                      const int32_t *pat_nodes, const double *g, int rho, int qbits, int32_t *add, hipStream_t s) {
  if (nrows == 0) return;
  if (A.b == 1)
    hipLaunchKernelGGL(k_fsai_grow<1>, dim3(nrows), dim3(64), 0, s, nrows, rows, pat_ptr, pat_nodes, g, A.rp, A.ci,
                       A.v, rho, qbits, add);
  else
    hipLaunchKernelGGL(k_fsai_grow<3>, dim3(nrows), dim3(64), 0, s, nrows, rows, pat_ptr, pat_nodes, g, A.rp, A.ci,
                       A.v, rho, qbits, add);
}

void launch_dpls_weights(int32_t nrows, const int32_t *row, const int32_t *cnt, const int32_t *sel,
                         const double *V, int ntv, double *w, hipStream_t s) {
  if (nrows == 0) return;
  hipLaunchKernelGGL(k_dpls_weights, dim3((nrows + 255) / 256), dim3(256), 0, s, nrows, row, cnt, sel, V, ntv, w);
}

void launch_spgemm_ap(const DevBSR &A, const DevBSR &P, const DevBSR &T, hipStream_t s) {
  if (T.nnzb == 0) return;
  const dim3 grid((unsigned)((T.nnzb + 255) / 256));
  if (T.b == 1)
    hipLaunchKernelGGL(k_spgemm_ap<1>, grid, dim3(256), 0, s, T.n, A.rp, A.ci, A.v, P.rp, P.ci, P.v, T.rp, T.ci, T.v,
                       T.nnzb);
  else
    hipLaunchKernelGGL(k_spgemm_ap<3>, grid, dim3(256), 0, s, T.n, A.rp, A.ci, A.v, P.rp, P.ci, P.v, T.rp, T.ci, T.v,
                       T.nnzb);
}

void launch_spgemm_rt(const DevBSR &R, const DevBSR &T, const DevBSR &Ac, hipStream_t s) {
  if (Ac.nnzb == 0) return;
  const dim3 grid((unsigned)((Ac.nnzb + 255) / 256));
  if (Ac.b == 1)
    hipLaunchKernelGGL(k_spgemm_rt<1>, grid, dim3(256), 0, s, Ac.n, R.rp, R.ci, R.v, T.rp, T.ci, T.v, Ac.rp, Ac.ci,
                       Ac.v, Ac.nnzb);
  else
    hipLaunchKernelGGL(k_spgemm_rt<3>, grid, dim3(256), 0, s, Ac.n, R.rp, R.ci, R.v, T.rp, T.ci, T.v, Ac.rp, Ac.ci,
                       Ac.v, Ac.nnzb);
}

void launch_element_gradient(int64_t n_el, const int32_t *conn, const double *Ke0, int64_t ke_stride,
                             const double *lam, const double *u, const double *scale, double *grad,
                             hipStream_t s) {
  if (n_el == 0) return;
  hipLaunchKernelGGL(k_element_gradient, dim3((unsigned)((n_el + 255) / 256)), dim3(256), 0, s, n_el, conn, Ke0,
                     ke_stride, lam, u, scale, grad);
}

void launch_assemble(int64_t nnzb, const int64_t *slot_ptr, const int32_t *contrib, const int8_t *diag_id,
                     const double *Ke0, int64_t ke_stride, const double *E, double *vals, hipStream_t s) {
  if (nnzb == 0) return;
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)((nnzb + 255) / 256)), dim3(256), 0, s, nnzb, slot_ptr, contrib,
                     diag_id, Ke0, ke_stride, E, vals);
}

}  // namespace aspamg
