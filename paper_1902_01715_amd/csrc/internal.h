// Internal declarations of the aSP-AMG library: host data structures, the
// device layouts and the kernel launchers shared by the host translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "aspamg.h"
#include "layout_plan.h"

namespace aspamg {

constexpr int64_t kMinThreads = 262144;  // lanes per row grow until n * L reaches this
constexpr int64_t kTimedSlots = 1 << 20;  // layouts of larger operators are chosen by timing
// q = K p: lanes per row of the fine-level FP64 copy and workgroup size (one
// p.q partial per workgroup, each re-read by every block of the update
// kernel).  Measured on the cantilever: 4 lanes make the product 3% faster,
// but the 4x partial count costs the update kernel more than that.
#ifndef ASPAMG_KP_LANES
#define ASPAMG_KP_LANES 1
#endif
#ifndef ASPAMG_DOT_THREADS
#define ASPAMG_DOT_THREADS 256
#endif
constexpr int kKpLanes = ASPAMG_KP_LANES;
constexpr int kDotThreads = ASPAMG_DOT_THREADS;
constexpr int kMaxFsaiNodes = 32;   // off-diagonal nodes an FSAI row may hold
constexpr int kMaxGrowRho = 8;      // nodes one aFSAI growth step may add to a row
constexpr int kMaxPEntries = 8;     // interpolation entries per scalar row (n_max cap)
constexpr int kMaxTheta = 16;       // strong connections kept per node (theta cap)

// Error raised inside the library; converted to aspamg_status at the ABI.
struct Error {
  aspamg_status code;
  std::string msg;
};
[[noreturn]] void fail(aspamg_status code, const std::string &msg);
void hip_check(hipError_t e, const char *what);
#define HIPCHK(x) ::aspamg::hip_check((x), #x)

// Host b x b block CSR (int64 row pointer); b = 3 (nodal blocks) or 1
// (scalar CSR, the paper's point-wise method).
struct HostBSR {
  int32_t n = 0, nc = 0;
  int32_t b = 3;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;   // nnzb * b * b
  int64_t nnzb() const { return rp.empty() ? 0 : rp.back(); }
  int bb() const { return b * b; }
};

// Device plain BSR (int32 row pointer) used by setup kernels.
struct DevBSR {
  int32_t n = 0, nc = 0;
  int32_t b = 3;
  int64_t nnzb = 0;
  int32_t *rp = nullptr;
  int32_t *ci = nullptr;
  double *v = nullptr;
};

// Device layout of one stored 3x3-block operator, one of two forms.  In both,
// slot group g holds 64 entries: entry e has its column at col[g*64 + e] and
// its block values in the group's 576 values val[g*576 ...]: with W = 16 /
// sizeof(T) values per 16-byte chunk, block entry k < 8 at
// (k / W)*64*W + e*W + k % W and entry 8 at 512 + e.  Every load instruction of
// a wavefront then reads 64 lane-consecutive 16-byte chunks (or 64 consecutive
// entries 8); padded entries hold 0 and a valid column.
//
// Sliced ELL (pack == 0) with L lanes per block row (L a power of two,
// 1..64): slice s is the 64/L consecutive rows one wavefront serves and owns
// slot groups [sptr[s], sptr[s+1]); lane j of row r takes the row's blocks j,
// j+L, j+2L, ... as entry e = r*L + j, and the L partial sums of a row meet
// in a butterfly.  L = 1 suits long uniform rows (the fine-level operator).
//
// Row-packed (pack == K > 0): wavefront s owns the K slot groups [s*K, s*K+K)
// and the rows [sptr[s], sptr[s+1]); a row of len blocks takes
// max(1, ceil(len/K)) consecutive lanes, lane j holding its blocks
// j*K .. j*K+K-1, so padding is per row rather than per slice.
// meta[s*64 + e] = (lanes of the row << 8 on its first lane, else 0) | row
// offset inside the wavefront, or 0x00FF for an idle lane.
// With b = 1 (scalar operators) a slot holds one value: the group's 64
// values are val[g*64 + e].
template <typename T>
struct Sell {
  int32_t n = 0, nc = 0, nslices = 0;  // nslices = wavefronts of the launch
  int32_t b = 3;           // block size: values per slot b * b
  int32_t lanes = 1;       // L (sliced)
  int32_t pack = 0;        // K (row-packed), 0 for the sliced layout
  int32_t unit = 0;        // lanes per packing unit (row-packed): 64 or 256
  int64_t ngroups = 0;     // slot groups (64 entries each)
  int64_t nnzb = 0;        // real blocks
  int32_t *sptr = nullptr;
  int32_t *col = nullptr;      // int32 columns, or null when col16 is used
  uint16_t *col16 = nullptr;   // columns as offsets from cbase[s] of their slice / wavefront
  int32_t *cbase = nullptr;
  T *val = nullptr;
  uint16_t *meta = nullptr;
  bool own_index = true;   // false where the index arrays belong to another copy
  int64_t slots() const { return ngroups * 64; }
  int64_t values() const { return ngroups * 64 * b * b; }
  int index_bytes() const { return col16 ? 2 : 4; }
};

// Device-resident PCG control block (one per solve stream).
struct PcgCtrl {
  int32_t done;       // 1 once converged, failed or out of iterations
  int32_t status;     // aspamg_status
  int32_t iter;
  int32_t max_it;
  double rtol, fnorm;
  double alpha, beta, rz, rzo, pq, rr, relres;
  double rzk[2];      // r.z of iterate k in slot k & 1
  double pad[1];
};

template <typename T>
struct LevelVecs {
  T *y = nullptr;   // cycle input
  T *z = nullptr;   // cycle output / s
  T *r = nullptr;   // residual
  T *t = nullptr;   // G r
};

struct Level {
  HostBSR A, G, P;                 // FP64 host copies (decisions, exports)
  DevBSR dA;                       // plain FP64 device copy for setup kernels
  Sell<double> A64, G64, GT64, P64, R64;
  Sell<float> A32, G32, GT32, P32, R32;
  // [P; A P] stacked (2 N rows): the first post-smoothing step forms
  // z + P e and r_pre - (A P) e in one product.  Only where A P has at most
  // as many blocks as A (nnzb_AP > 0); elsewhere the step applies P, then A.
  Sell<double> PAP64;
  Sell<float> PAP32;
  int64_t nnzb_AP = 0;
  bool stacked() const { return nnzb_AP > 0; }
  // M = G^T G as one stored operator on small levels (nnzb_M > 0): each
  // smoothing step of the FP32 cycle is then one product instead of G
  // followed by G^T
  Sell<double> M64;
  Sell<float> M32;
  int64_t nnzb_M = 0;
  bool coarsest = false;
  double lambda1 = 0, omega_q = 0, omega_s = 0;
  int32_t fsai_rounds = 0;
  std::vector<int8_t> cf;
  std::vector<int32_t> cidx;
  int32_t nc = 0;
  std::vector<double> V;           // orthonormalised test space, [n][b][ntv]
  std::vector<int32_t> pcount, pcols;   // scalar P pattern
  LevelVecs<double> v64;
  LevelVecs<float> v32;
};

// Dense coarsest operator: explicit inverse A_L^{-1} = L^{-T} L^{-1} from the
// Cholesky factor, applied as one dense matrix-vector product.
struct Coarse {
  int32_t nd = 0;
  double *inv = nullptr;     // device nd x nd row-major
};

// Dense tail: the V-cycle from `level` down (its smoothing, transfers and the
// coarsest solve), a fixed linear operator, formed once as a dense nd x nd
// row-major FP64 matrix and applied as one product.  level = -1: none.
struct DenseTail {
  int32_t level = -1;
  int32_t nd = 0;
  double *v = nullptr;
};

struct BatchWork;  // multi-RHS buffers (solve_batch)

}  // namespace aspamg

struct aspamg_ctx {
  aspamg_params p;
  hipStream_t stream = nullptr;
  int32_t device = 0;                         // device current at setup (the stream's)
  int32_t ntv = 0;
  int32_t n = 0;                              // fine block rows
  int32_t b = 3;                              // unknowns per node (block size)
  std::vector<aspamg::Level> lev;
  aspamg::Coarse coarse;
  aspamg::DenseTail tail;
  int32_t prec = 64;
  // PCG vectors (FP64) and control
  double *vu = nullptr, *vr = nullptr, *vp = nullptr, *vq = nullptr, *vz = nullptr;
  double *part = nullptr;                     // reduction partials (4 x kMaxPart): K p, r.r, r.z_old, r.z
  aspamg::PcgCtrl *ctrl = nullptr;
  aspamg::PcgCtrl *ctrl_host = nullptr;       // pinned
  hipGraphExec_t graph[2] = {nullptr, nullptr};   // [0] fp64 cycle, [1] fp32 cycle
  const double *graph_f = nullptr;
  double t_setup = 0;
  double c_gd = 0, c_op = 0, c_fs = 0;
  aspamg::BatchWork *batch = nullptr;
  std::vector<void *> allocations;
  void *staging = nullptr;                    // pinned host staging for setup copies
  size_t staging_bytes = 0;
};

struct aspamg_assembler_ctx {
  hipStream_t stream = nullptr;
  int64_t nnzb = 0;
  int32_t n_nodes = 0;
  int64_t n_el = 0;
  int64_t *slot_ptr = nullptr;     // device: contribution list per block slot
  int32_t *contrib = nullptr;      // device: (element, local a*8+b) packed per contribution
  int8_t *diag_identity = nullptr; // device: 1 if the slot is a constrained diagonal block
  double *Ke0 = nullptr;
  int64_t ke_stride = 0;
};

namespace aspamg {

constexpr int kMaxPart = 8192;      // reduction partial slots per buffer
constexpr int kMaxTailDof = 8192;   // largest dense tail operator (512 MB in FP64)
constexpr int32_t kMergeMaxNodes = 10922;           // levels considered for M = G^T G
constexpr double kMergeMaxBytes = 16.0 * (1 << 20);  // ... kept when its FP32 copy is at most this

// ---- device memory helpers (tracked by the handle) ----
void *dmalloc(aspamg_ctx *h, size_t bytes);
template <typename T>
T *dalloc(aspamg_ctx *h, size_t n) { return static_cast<T *>(dmalloc(h, n * sizeof(T))); }
void dfree(aspamg_ctx *h, void *p);   // releases one dmalloc'd pointer early

// ---- layout builders (host) ----
HostBSR transpose(const HostBSR &M);
// dvals: M's block values already on the device (then M.v is not read)
template <typename T>
Sell<T> upload_sell(aspamg_ctx *h, const HostBSR &M, int force_lanes = 0, bool timed = true,
                    const double *dvals = nullptr);
template <typename T>
void free_sell(aspamg_ctx *h, Sell<T> &S);   // releases the device arrays of S
// FP32 copy in the same layout, sharing S's index arrays (never freed on its own)
Sell<float> derive_fp32(aspamg_ctx *h, const Sell<double> &S);
// FP64 and FP32 copies of M, each in the layout timed in its own precision
// (index arrays built once; shared when both copies pick the same layout)
void upload_sell_pair(aspamg_ctx *h, const HostBSR &M, const double *dvals, Sell<double> &d64, Sell<float> &d32);
DevBSR upload_bsr(aspamg_ctx *h, const HostBSR &M);

// ---- solve-path kernel launchers (kernels_solve.hip) ----
template <typename T, typename TX, typename TO>
void launch_spmv(const Sell<T> &A, const TX *x, TO *y, const TO *w, double alpha, const PcgCtrl *ctrl,
                 hipStream_t s);
// rows r < n1 of the stacked operator give y1[r] = a1 (S x)[r] + w1[r], rows
// r >= n1 give y2[r - n1] = a2 (S x)[r] + w2[r - n1]
template <typename T, typename TX, typename TO>
void launch_spmv_dual(const Sell<T> &S, int32_t n1, const TX *x, TO *y1, const TO *w1, double a1, TO *y2,
                      const TO *w2, double a2, const PcgCtrl *ctrl, hipStream_t s);
int spmv_dot_blocks(const Sell<double> &A);   // partials written by launch_spmv_dot (<= kMaxPart)
void launch_spmv_dot(const Sell<double> &A, const double *x, double *y, double *part, const PcgCtrl *ctrl,
                     hipStream_t s);
// partials (spmv_dot_blocks of them) of sum_i s_i^2, s_i = |f_i| + (|K| |u|)_i
void launch_abs_bound(const Sell<double> &A, const double *u, const double *f, double *part, hipStream_t s);
template <typename TV>
void launch_dense_gemv(int nd, const double *inv, const TV *y, TV *z, const PcgCtrl *ctrl, hipStream_t s);
template <typename TI, typename TO>
void launch_cast(int64_t n, const TI *x, TO *y, const PcgCtrl *ctrl, hipStream_t s);
void launch_fill(int64_t n, double *x, double v, hipStream_t s);
void launch_copy(int64_t n, const double *x, double *y, hipStream_t s);
void launch_dot(int64_t n, const double *a, const double *b, double *part, const PcgCtrl *ctrl, hipStream_t s);
// z in the cycle precision TC; rc (optional) receives r in that precision
template <typename TC>
void launch_pcg_update(int64_t n, double *u, double *r, const double *p, const double *q, const TC *z,
                       const double *pq_part, int npq, double *part, TC *rc, PcgCtrl *ctrl, hipStream_t s);
// r.z partials, and the convergence test on the update's r.r / r.z_old partials
template <typename TZ>
void launch_pcg_rz(int64_t n, const double *r, const TZ *z, double *part, const double *rr_part, int nrr,
                   PcgCtrl *ctrl, hipStream_t s);
template <typename TZ>
void launch_pcg_pupdate(int64_t n, const TZ *z, double *p, const double *rz_part, int nrz, PcgCtrl *ctrl,
                        hipStream_t s);
// finish modes
// (kFinRr and the batch modes are used by the multi-RHS column finisher; the
// single-RHS iteration tests convergence inside k_pcg_rz)
enum FinishMode { kFinInitF = 0, kFinInitRz = 1, kFinAlpha = 2, kFinRr = 3, kFinBeta = 4, kFinNorm = 5 };
void launch_finish(int mode, const double *part, int nparts, PcgCtrl *ctrl, hipStream_t s);
int vec_blocks(int64_t n);

// ---- setup kernel launchers (kernels_setup.hip) ----
// FSAI rows: for each listed block row I (rows[i]) with nodes pat[pat_ptr[i]..pat_ptr[i+1]),
// computes the three scaled rows g (stride gstride) and psi. Returns nonzero on a bad pivot.
int launch_fsai_rows(const DevBSR &A, int32_t nrows, const int32_t *rows, const int32_t *pat_ptr,
                     const int32_t *pat_nodes, int mmax, double *g, double *psi, int32_t *fail_flag,
                     hipStream_t s);
// aFSAI growth: for each listed block row (as for launch_fsai_rows, with the g it wrote) the
// rho (<= kMaxGrowRho) nodes to add, add[i*rho ..] (-1 padded), chosen by quantised scores.
void launch_fsai_grow(const DevBSR &A, int32_t nrows, const int32_t *rows, const int32_t *pat_ptr,
                      const int32_t *pat_nodes, const double *g, int rho, int qbits, int32_t *add, hipStream_t s);
// DPLS weights: for each listed scalar row i, K=cnt[i] chosen scalar rows sel[i*kMaxPEntries + k]
// of the fine-level test space V (ntv columns): w = (C^T C)^{-1} C^T v.
void launch_dpls_weights(int32_t nrows, const int32_t *row, const int32_t *cnt, const int32_t *sel,
                         const double *V, int ntv, double *w, hipStream_t s);
// coarsening on the device (kernels_coarsen.hip): sq_i = sqrt(n_II); the theta
// strongest connections of every node (keep[i*theta ..], nkeep[i]); the union
// symmetrisation in three stages (0: counts into cnt; 1: fill the rows bp of
// `both` through the cursors `at`, then sort and deduplicate each row into
// len; 2: compact into srp / sci); the independent-set rounds (cf: -1
// decoupled, 0 F, 1 C, 2 undecided; undecided counts the nodes left)
void launch_node_norms(int32_t n, const double *V, int ntv, int b, double *sq, hipStream_t s);
void launch_strong_topk(const DevBSR &A, const int8_t *excl, const double *V, int ntv, const double *sq, int theta,
                        int qbits, int32_t *keep, int32_t *nkeep, hipStream_t s);
void launch_union(int32_t n, int theta, const int32_t *keep, const int32_t *nkeep, int stage, int32_t *cnt,
                  int64_t *bp, int64_t *at, int32_t *both, int32_t *len, const int64_t *srp, int32_t *sci,
                  hipStream_t s);
void launch_mis_init(int32_t n, const int8_t *excl, int8_t *cf, hipStream_t s);
void launch_mis_round(int32_t n, const int64_t *srp, const int32_t *sci, int8_t *cf, int8_t *win, int32_t *undecided,
                      hipStream_t s);
// interpolation entries of the fine nodes fnodes[0..nf): pcount[bI+d] and the
// chosen fine scalar indices psel[(bI+d)*kMaxPEntries ..]; err set when a
// node's candidates exceed the kernel's limits
void launch_dpls_rows(int32_t nf, const int32_t *fnodes, const int64_t *srp, const int32_t *sci, const int8_t *cf,
                      const double *V, int ntv, int b, int d_p, int nmax, double kappa_q, double eps_p, int qbits,
                      int32_t *pcount, int32_t *psel, int32_t *err, hipStream_t s);
// RAP numeric phases
void launch_spgemm_ap(const DevBSR &A, const DevBSR &P, const DevBSR &T, hipStream_t s);
void launch_spgemm_rt(const DevBSR &R, const DevBSR &T, const DevBSR &Ac, hipStream_t s);
// setup-only products on row-major multi-vectors with nb columns (the dense tail operator)
void launch_bsr_mm(const DevBSR &M, const double *X, double *Y, const double *W, double alpha, int32_t nb,
                   hipStream_t s);
void launch_dense_mm(int32_t nd, const double *D, const double *X, double *Y, int32_t nb, hipStream_t s);
void launch_eye(int32_t nd, double *X, hipStream_t s);
void launch_axpy(int64_t n, double a, const double *x, double *y, hipStream_t s);     // y += a x
void launch_divided(int64_t n, double a, const double *x, double *y, hipStream_t s);  // y = x / a
// test-space iteration: out = 2 (sz - q z) / f; y = x + b y; Y = X U (columns of n entries, U nt x nt row-major)
void launch_rq_gradient(int64_t n, double q, double f, const double *sz, const double *z, double *out, hipStream_t s);
void launch_xpby(int64_t n, const double *x, double b, double *y, hipStream_t s);
// inner-product partials of 256-entry blocks (dot256_parts of them), each
// summed sequentially; y = M x with each row summed sequentially in stored order
int dot256_parts(int64_t n);
void launch_dot256(int64_t n, const double *a, const double *b, double *part, hipStream_t s);
void launch_bsr_mv_seq(const DevBSR &M, const double *x, double *y, hipStream_t s);
void launch_combine_columns(int64_t n, int nt, const double *X, const double *U, double *Y, hipStream_t s);
// layout values: slot i takes the b * b values of block map[i] of v (zeros when map[i] < 0)
template <typename T>
void launch_scatter_values(int64_t nslots, const int32_t *map, const double *v, T *val, int b, hipStream_t s);
// FP32 layout values from FP64 ones (same slots)
void launch_narrow_values(int64_t nslots, const double *v64, float *v32, int b, hipStream_t s);
void launch_element_gradient(int64_t n_el, const int32_t *conn, const double *Ke0, int64_t ke_stride,
                             const double *lam, const double *u, const double *scale, double *grad,
                             hipStream_t s);
void launch_assemble(int64_t nnzb, const int64_t *slot_ptr, const int32_t *contrib, const int8_t *diag_id,
                     const double *Ke0, int64_t ke_stride, const double *E, double *vals, hipStream_t s);

// ---- host setup (setup_host.cpp) ----
void build_hierarchy(aspamg_ctx *h, HostBSR &&A0, std::vector<double> &&V0);
// M = G^T G on the small smoothed levels above the dense tail
void merge_smoothers(aspamg_ctx *h);
double quantize(double s, int bits);

// message returned by aspamg_last_error for the calling thread
void set_last_error(const std::string &msg);
// device address of the no-allocation staging array on the current device
// (looked up once per device)
float *noalloc_scratch_current_device();

// gamma_{m+1} of the longest scalar row of the fine-level K: the relative
// rounding bound of recomputing a residual f - K u in FP64
double residual_gamma(const aspamg_ctx *h);

// ---- multi-RHS solve (batch_api.cpp) ----
aspamg_status solve_batch_impl(aspamg_ctx *h, int32_t k, const double *F, int64_t ldf, double *U, int64_t ldu,
                               aspamg_stats *st);
void destroy_batch(BatchWork *w);
int batch_tile(const aspamg_ctx *h, int precision);

}  // namespace aspamg
