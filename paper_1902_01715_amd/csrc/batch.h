// Multi-right-hand-side solve: device layouts, control block and launchers.
#pragma once

#include "internal.h"

namespace aspamg {

constexpr int kBatchMax = 32;       // columns per batch (larger k is solved in chunks)
constexpr int kBatchParts = 1024;   // reduction partials per column

// per-column PCG state (device resident)
struct BatchCtrl {
  int32_t all_done;
  int32_t max_it;
  double rtol;
  int32_t done[kBatchMax], status[kBatchMax], iter[kBatchMax];
  double alpha[kBatchMax], beta[kBatchMax], rz[kBatchMax], rzo[kBatchMax], fnorm[kBatchMax], relres[kBatchMax];
};

// plain device block CSR in FP64 or FP32
template <typename T>
struct DevBSRT {
  int32_t n = 0, nc = 0;
  int32_t split = 1;       // lane groups per block row in the SpMM (1, 2, 4, 8)
  int64_t nnzb = 0;
  int32_t *rp = nullptr;
  int32_t *ci = nullptr;
  T *v = nullptr;
};

template <typename T>
struct BatchOps {
  DevBSRT<T> A, G, GT, P, R;
  T *y = nullptr, *z = nullptr, *r = nullptr, *t = nullptr;   // [3n][kpad]
};

struct BatchLevel {
  BatchOps<double> d;
  BatchOps<float> f;
};

struct BatchWork {
  int kpad = 0;
  int kb[2] = {0, 0};                  // tuned SpMM tile per precision (0: fp64, 1: fp32)
  std::vector<BatchLevel> lev;
  double *U = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr, *Z = nullptr, *F = nullptr, *part = nullptr;
  BatchCtrl *ctrl = nullptr, *ctrl_host = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  std::vector<void *> allocations;
};

int batch_vec_blocks(int64_t nrow, int ld);
int spmm_dot_parts(const DevBSRT<double> &A, int ld, int kb);
template <typename T>
void launch_spmm(const DevBSRT<T> &A, const T *X, T *Y, const T *W, int ld, int kb, double alpha, const BatchCtrl *c,
                 hipStream_t s);
void launch_spmm_dot(const DevBSRT<double> &A, const double *X, double *Y, int ld, int kb, double *part,
                     const BatchCtrl *c, hipStream_t s);
template <typename T>
void launch_dense_gemm(int nd, const double *inv, const T *Y, T *Z, int ld, const BatchCtrl *c, hipStream_t s);
void launch_col_dot(int64_t nrow, const double *A, const double *B, int ld, double *part, const BatchCtrl *c,
                    hipStream_t s);
// z in the cycle precision TC; Rc (optional) receives r in that precision
template <typename TC>
void launch_col_update(int64_t nrow, double *U, double *R, const double *P, const double *Q, const TC *Z, TC *Rc,
                       int ld, double *part, const BatchCtrl *c, hipStream_t s);
template <typename TZ>
void launch_col_rz(int64_t nrow, const double *R, const TZ *Z, int ld, double *part, const BatchCtrl *c,
                   hipStream_t s);
template <typename TZ>
void launch_col_pupdate(int64_t nrow, const TZ *Z, double *P, int ld, const BatchCtrl *c, hipStream_t s);
void launch_col_finish(int mode, const double *part, int nparts, int ld, BatchCtrl *c, hipStream_t s);
// S = |F| + |A| |U| on the first k columns (rounding bound of F - A U)
void launch_abs_bound_cols(const DevBSRT<double> &A, const double *U, const double *F, int ld, int k, double *S,
                           hipStream_t s);
void launch_copy_cols(int64_t nrow, int k, const double *src, int64_t lds, double *dst, int64_t ldd, int kfill,
                      hipStream_t s);

}  // namespace aspamg
