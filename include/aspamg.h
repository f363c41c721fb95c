/*
 * aspamg.h -- C ABI of the MI355X aSP-AMG solver library (libaspamg.so).
 *
 * Solves K u = f for a symmetric positive definite elasticity stiffness matrix
 * K given as 3x3-block CSR (the problem statement of the paper, Section 1,
 * eq. (1): K from the integral of B^T D B over the elements) with PCG
 * preconditioned by one aSP-AMG V(nu1,nu2)-cycle (Section 2, Algorithms
 * "Recursive AMG Setup" and "AMG application in a V-cycle"; Section 3 for the
 * aFSAI smoother, the test space, the affinity coarsening and the DPLS
 * prolongation; Section 4 for the PCG start and stopping rule).
 *
 * Conventions shared by every entry point
 *   - DOF index = 3 * node + component.  Vectors are float64, node-major.
 *   - Block matrices: row_ptr int32 [n+1], col int32 [nnzb] sorted ascending in
 *     each row, vals float64 [nnzb][3][3] row-major blocks.
 *   - With params.block_size = 1 the same calls take a scalar CSR matrix (a
 *     "node" is one unknown, vals [nnz], V0 [n][n_tv]) and run the paper's
 *     point-wise method; every size stated below in units of 3 is then in
 *     units of 1.
 *   - A block row holding only its diagonal block is a constrained (Dirichlet)
 *     or decoupled node: it is never coarse and gets no interpolation.
 *   - A handle runs its device work on a private non-blocking stream (default
 *     priority) created by aspamg_setup, which first waits for the caller's
 *     stream; solve, vcycle and apply calls return when their work is done.
 *   - Every call returns aspamg_status; negative values are errors, positive
 *     values are warnings with valid outputs.  No C++ exception crosses the ABI.
 *     aspamg_last_error() returns a message for the last failing call of the
 *     calling thread.
 *   - A handle must not be used from two threads at once.
 */
#ifndef ASPAMG_H
#define ASPAMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ASPAMG_OK = 0,
  ASPAMG_NOT_CONVERGED = 1, /* warning: u holds the last iterate, stats are filled */
  ASPAMG_EINVAL = -1,       /* bad argument or unsupported input                    */
  ASPAMG_ENOMEM = -2,       /* host or device allocation failed                     */
  ASPAMG_EHIP = -3,         /* a HIP runtime call failed                            */
  ASPAMG_ENOT_SPD = -4,     /* a local FSAI system or the coarsest matrix has a pivot <= 0 */
  ASPAMG_EBREAKDOWN = -5,   /* PCG: p.q <= 0 or r.z <= 0 (indefinite preconditioner) */
  ASPAMG_ENAN = -6          /* non-finite residual                                  */
} aspamg_status;

typedef struct aspamg_ctx *aspamg_handle;   /* opaque; owns all hierarchy memory */

/* Setup and solve parameters.  The first eight are the paper's user parameters
 * (Table "Default input parameters"); the rest fix values the paper leaves
 * open.  aspamg_default_params() fills the defaults noted on each line. */
typedef struct {
  int32_t k_g;            /* 4     adaptive FSAI steps per row                          */
  int32_t rho_g;          /* 4     paper: scalar entries per step (informational)      */
  double  eps_g;          /* 1e-3  FSAI exit tolerance on the relative decrease of psi */
  int32_t n_tv;           /* 0     test vectors: 0 takes the n_tv argument of aspamg_setup
                           *       (the columns of V0); > 0 must equal it (EINVAL
                           *       otherwise).  The paper's default is 10: the six
                           *       rigid-body modes padded with random vectors.       */
  int32_t n_rq;           /* 0     SRQCG iterations on each level's test space before its
                           *       coarsening (Section 3.3, Algorithm "Test Space generation
                           *       by SRQCG", Ritz projection every iteration); 0 uses V0 as
                           *       given.  The paper's default is 10, with n_tv = 10.  0..1000 */
  int32_t theta;          /* 5     strong connections kept per node                     */
  int32_t n_max;          /* 5     max interpolation entries per scalar row (<= 8)      */
  double  kappa_p;        /* 50    max conditioning of a local least-squares fit        */
  int32_t rho_blocks;     /* 3     nodes added to an FSAI row per step (1..8)           */
  double  omega_bar;      /* 0.8   aFSAI outer loop target for omega = 2/lambda_1       */
  int32_t outer_fsai;     /* 1     run the aFSAI outer loop                             */
  int32_t d_p;            /* 2     max S-path length to interpolating coarse nodes      */
  double  eps_p;          /* 1e-8  relative least-squares residual tolerance            */
  int32_t lanczos_steps;  /* 30    Lanczos steps for lambda_1(G A G^T)                  */
  double  omega_safety;   /* 1.05  applied omega = min(1, 2 / (safety * lambda_1))      */
  int32_t coarse_max_dof; /* 1500  factor densely once 3 N_l <= this                    */
  int32_t max_levels;     /* 25                                                         */
  double  stall_ratio;    /* 0.9   stop coarsening when N_{l+1} > ratio * N_l           */
  int32_t nu1, nu2;       /* 1, 1  pre- and post-smoothing steps                        */
  int32_t cycle_precision;/* 64    64: FP64 V-cycle; 32: FP32 V-cycle inside FP64 PCG   */
  double  rtol;           /* 1e-10 stop when ||r_k|| <= rtol ||f||                       */
  int32_t max_it;         /* 1000                                                       */
  int32_t quant_bits;     /* 20    significant bits of quantised decision quantities    */
  int32_t dense_max_dof;  /* 16384 refuse a larger dense coarsest system                */
  int32_t check_every;    /* 4     PCG iterations per host convergence poll             */
  int32_t use_graph;      /* 1     replay the PCG iteration as a captured HIP graph     */
  int32_t layout;         /* 0     device layout of the stored operators: 0 time the
                           *       candidate layouts on the device for the larger operators,
                           *       separately for the FP64 and FP32 copies; 1 pick by stored
                           *       slots only (the same choice on every run); 2 sliced ELL
                           *       only; 3 row-packed only, rows packed into units of a
                           *       256-thread workgroup; 4 row-packed only, units of one
                           *       wavefront.  The fine-level FP64 operator of q = K p is
                           *       sliced with one lane per row in every case, and the FP32
                           *       copy of the fine-level K shares its layout.  Results do
                           *       not depend on the layout beyond the order of
                           *       floating-point sums within a row. */
  int32_t dense_tail_dof; /* 4096  the V-cycle from the highest level whose unknowns, and
                           *       those of every level below it, number at most this
                           *       (above the coarsest) is formed at setup as one dense FP64
                           *       operator and applied as one product; 0 keeps every level
                           *       sparse.  At most 8192.  The operator is the same; only the
                           *       rounding differs. */
  int32_t block_size;     /* 3     unknowns per node: 3 takes K as 3x3-block CSR (nodal
                           *       blocks, elasticity); 1 takes K as scalar CSR and runs
                           *       the paper's point-wise rules (Sections 3.1-3.5 with
                           *       1x1 blocks), row_ptr / col / vals then being plain CSR
                           *       and V0 [n][n_tv].  solve_batch and the assembler need
                           *       3. */
} aspamg_params;

typedef struct {
  int32_t status;           /* aspamg_status of the solve                             */
  int32_t iterations;       /* PCG iterations (products with K)                       */
  int32_t levels;           /* levels of the hierarchy                                */
  int32_t cycle_precision;  /* 64 or 32                                               */
  double  relres_recursive; /* ||r_k|| / ||f|| from the recurrence                     */
  double  relres_true;      /* ||f - K u|| / ||f|| recomputed at the end               */
  double  relres_floor;     /* gamma_{m+1} || |f| + |K| |u| || / ||f||: the rounding bound
                             * of that recomputation in FP64 (m = longest scalar row of
                             * K; Higham, "Accuracy and Stability of Numerical
                             * Algorithms", Sec. 3.5).  relres_true below it is noise. */
  double  t_setup_s;        /* setup wall time                                        */
  double  t_solve_s;        /* solve time, HIP events on the handle's stream          */
  double  c_gd, c_op, c_fs; /* grid, operator and FSAI complexities                   */
  double  bytes_vcycle;     /* algorithmic HBM bytes of one V-cycle                   */
  double  bytes_iter;       /* algorithmic HBM bytes of one PCG iteration             */
  int32_t spmm_tile;        /* right-hand sides per SpMM tile (solve_batch), else 0   */
  int32_t tail_level;       /* level applied as the dense tail operator, -1 if none   */
} aspamg_stats;

/* Per-level summary, see aspamg_level_info. */
typedef struct {
  int32_t n;               /* block rows (nodes) on the level                       */
  int32_t n_coarse;        /* coarse nodes chosen on this level (0 on the coarsest) */
  int64_t nnzb_A, nnzb_G, nnzb_P;
  int32_t has_smoother;    /* 0 on the coarsest level                               */
  int32_t fsai_rounds;     /* extra rounds of the aFSAI outer loop                  */
  double  lambda1, omega_q, omega_s;
  int64_t sell_slots_A, sell_slots_G, sell_slots_GT; /* stored block slots (padding incl.) */
  /* device layout of the stored operators A, G, G^T, P, R (index = `which` of
   * aspamg_apply_operator), FP64 and FP32 copies (each chosen for its own
   * precision): L > 0 for the sliced layout with L lanes per row, -K for the
   * row-packed layout with K slot groups per lane (its packing unit in
   * sell_unit64 / sell_unit32) */
  int32_t sell_lanes64[5], sell_lanes32[5];
  /* bit k (FP64 copy) and bit 5 + k (FP32 copy) set when operator k stores its
   * columns as 16-bit offsets from a per-slice base; bit 10 the same for the
   * row-stacked [P; A P] operator of the coarse-grid correction */
  int32_t sell_index16;
  /* layout of the FP64 copy of the row-stacked [P; A P] operator (same
   * encoding as sell_lanes64); 0 on the coarsest level and where A P has more
   * blocks than A (there the first post-smoothing step applies P, then A) */
  int32_t sell_stacked;
  /* blocks of M = G^T G when the FP32 cycle's smoothing applies it as one
   * stored operator (small levels above the dense tail), else 0 (G, then G^T;
   * the FP64 cycle always applies G, then G^T) */
  int64_t nnzb_M;
  /* lanes per packing unit of the row-packed copies of A, G, G^T, P, R: 64
   * (rows packed per wavefront) or 256 (per 256-thread workgroup, a row's
   * lanes possibly in different wavefronts); 0 for the sliced layout */
  int32_t sell_unit64[5], sell_unit32[5];
  /* the row-stacked operator's FP32 copy (encoded as sell_stacked) and the
   * packing units of its two copies (as sell_unit64) */
  int32_t sell_stacked32, sell_stacked_unit64, sell_stacked_unit32;
} aspamg_level_info_t;

/* Fill *out with the defaults.  out: caller-owned. */
aspamg_status aspamg_default_params(aspamg_params *out);

/* Build the hierarchy (Algorithm "Recursive AMG Setup").
 *   p        parameters (NULL = defaults).
 *   n_nodes  block rows of K; nnzb = row_ptr[n_nodes].
 *   row_ptr, col, vals  K in the block layout above, host or device pointers
 *            (classified with hipPointerGetAttributes); K must be symmetric in
 *            pattern and values with a diagonal block in every row.
 *   n_tv, V0 near-null-space vectors, float64 [n_nodes][3][n_tv] node-major
 *            (the six rigid-body modes for elasticity, Section 3.3), host or device.
 *   hip_stream  caller's hipStream_t whose pending work setup waits for (NULL = none).
 *   out      receives the handle; NULL on failure.
 * Every input is copied; the caller may free its arrays when the call returns.
 * Errors: EINVAL (shape/pattern), ENOT_SPD, ENOMEM, EHIP. */
aspamg_status aspamg_setup(const aspamg_params *p, int32_t n_nodes, int64_t nnzb,
                           const int32_t *row_ptr, const int32_t *col, const double *vals,
                           int32_t n_tv, const double *V0, void *hip_stream,
                           aspamg_handle *out);

/* Select the V-cycle precision for later solves: 64 (FP64 operators and
 * vectors) or 32 (FP32 operators and vectors inside FP64 PCG; the coarsest
 * solve, and the dense tail operator that contains it, stay FP64).  Both
 * copies are built by aspamg_setup. */
aspamg_status aspamg_set_cycle_precision(aspamg_handle h, int32_t bits);

/* PCG from u = 0 until ||r|| <= rtol ||f|| (Section 4: the recursive residual
 * of the iteration).
 *   f_dev, u_dev  float64 device vectors of 3*n_nodes entries (caller-owned).
 *   st            optional stats (may be NULL).
 * After the iteration the residual f - K u is recomputed.  OK requires both
 * the recursive test and relres_true <= max(rtol, relres_floor): the
 * recomputed residual is at most rtol, or within the rounding bound of its own
 * evaluation.  Otherwise NOT_CONVERGED (u = last iterate).  Also EBREAKDOWN,
 * ENAN or EHIP.  The stats carry no separate V-cycle time: the iteration runs
 * as one captured graph; aspamg_time_kernel (which = 3, 4) times the cycle. */
aspamg_status aspamg_solve(aspamg_handle h, const double *f_dev, double *u_dev,
                           aspamg_stats *st);

/* k independent solves sharing one hierarchy, through block SpMM kernels
 * that reuse every streamed matrix block for all right-hand sides.
 *   F_dev  float64 device, node-major [3*n_nodes][ldf] (column j = load case j)
 *   U_dev  float64 device, [3*n_nodes][ldu]
 *   st     optional array of k stats.
 * Each column has its own alpha, beta and convergence test; a converged column
 * is frozen.  Returns the worst column status. */
aspamg_status aspamg_solve_batch(aspamg_handle h, int32_t k, const double *F_dev, int64_t ldf,
                                 double *U_dev, int64_t ldu, aspamg_stats *st);

/* One preconditioner application z = M^{-1} y (one V-cycle) in the selected
 * precision.  y_dev, z_dev: float64 device vectors of 3*n_nodes entries. */
aspamg_status aspamg_vcycle(aspamg_handle h, const double *y_dev, double *z_dev);

/* Apply one stored operator of level l: which = 0 A_l, 1 G_l, 2 G_l^T, 3 P_l,
 * 4 R_l = P_l^T, 5 M_l = G_l^T G_l (only where nnzb_M > 0); precision 64 or
 * 32.  x_dev/y_dev are float64 device vectors sized by the operator's
 * columns/rows (converted when precision is 32; that path allocates two
 * staging vectors). */
aspamg_status aspamg_apply_operator(aspamg_handle h, int32_t level, int32_t which,
                                    int32_t precision, const double *x_dev, double *y_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same product
 * as aspamg_apply_operator, with the FP32 staging of x and y in a fixed
 * library array of 2^23 floats (32 MiB) per device instead of per-call
 * allocations; no hipMalloc, hipFree or other allocating routine is called.
 * Arguments and results as for aspamg_apply_operator (bitwise the same
 * output).  EINVAL when an FP32 product needs more staging than the array
 * holds (3 * (columns rounded up to 64) + 3 * rows values) or on bad
 * arguments.  Every call on one device shares that device's array and leaves
 * its last contents there: calls that overlap in time on one device (two
 * threads, or two handles on different streams) race and must be serialised
 * by the caller. */
aspamg_status aspamg_apply_operator_noalloc(aspamg_handle h, int32_t level, int32_t which,
                                            int32_t precision, const double *x_dev, double *y_dev);

/* Level summary. */
aspamg_status aspamg_level_info(aspamg_handle h, int32_t level, aspamg_level_info_t *out);

/* Copy a level's setup products to host arrays (caller-owned, sized from
 * aspamg_level_info): which = 0 A_l, 1 G_l, 3 P_l as block CSR with int64
 * row_ptr; any pointer may be NULL. */
aspamg_status aspamg_level_matrix(aspamg_handle h, int32_t level, int32_t which,
                                  int64_t *row_ptr, int32_t *col, double *vals);

/* Copy the C/F split (int8 per node: 1 coarse, 0 fine, -1 constrained or
 * decoupled) and the scalar interpolation pattern (counts[3n], cols[3n][n_max],
 * -1 padded, coarse scalar indices) of a level.  Any pointer may be NULL. */
aspamg_status aspamg_level_split(aspamg_handle h, int32_t level, int8_t *cf,
                                 int32_t *p_counts, int32_t *p_cols);

/* Copy a level's orthonormalised test space, float64 [n][3][n_tv] node-major
 * (host array, caller-owned): the rows the affinity SoC and the least-squares
 * interpolation of that level used (Section 3.3; after n_rq SRQCG iterations
 * when n_rq > 0).  The coarsest level keeps the restricted rows, not
 * orthonormalised. */
aspamg_status aspamg_level_test_space(aspamg_handle h, int32_t level, double *V);

/* Per-element derivative of lam^T K(E) u with respect to E_e for K = sum_e
 * E_e K_e^0 (the adjoint form of the compliance gradient):
 *   grad_e = -scale_e * lam_e^T K_e^0 u_e        (scale NULL -> 1)
 *   conn_dev  int32 [n_el][8] node ids (Q1 local order), device
 *   Ke0_dev   float64 [24][24] (ke_stride = 0, shared) or [n_el][24][24]
 *             (ke_stride = 576), node-major local DOFs, device
 *   lam_dev, u_dev  float64 device vectors (3 * n_nodes)
 *   grad_dev  float64 [n_el] device output.
 * Runs on hip_stream (NULL = default).  Errors: EINVAL, EHIP. */
aspamg_status aspamg_element_gradient(int64_t n_el, const int32_t *conn_dev,
                                      const double *Ke0_dev, int64_t ke_stride,
                                      const double *lam_dev, const double *u_dev,
                                      const double *scale_dev, double *grad_dev,
                                      void *hip_stream);

/* Element-to-block assembly of K(E) = sum_e E_e K_e^0 into a fixed block
 * pattern (the paper's K from element integrals, Section 1).  Rows and
 * columns of constrained nodes are eliminated: their diagonal block is I3 and
 * their couplings are absent from the pattern.  The assembler copies its
 * inputs (host or device); contributions to a block are summed in ascending
 * element order. */
typedef struct aspamg_assembler_ctx *aspamg_assembler;
aspamg_status aspamg_assembler_create(int32_t n_nodes, int64_t n_el, const int32_t *conn,
                                      const int8_t *constrained, const int32_t *row_ptr,
                                      const int32_t *col, const double *Ke0, int64_t ke_stride,
                                      void *hip_stream, aspamg_assembler *out);
/* vals_dev: float64 device [nnzb][3][3]; E_dev: float64 device [n_el]. */
aspamg_status aspamg_assemble(aspamg_assembler a, const double *E_dev, double *vals_dev);
aspamg_status aspamg_assembler_destroy(aspamg_assembler a);

/* Measurement entry point: launch one kernel of the solve path `reps` times
 * back to back on the handle's stream between two HIP events and report the
 * average duration per launch and the algorithmic HBM bytes of one launch
 * (every stored block, its column index and each vector entry counted once).
 *   which = 0  PCG product q = K p with the fused p.q partials (FP64)
 *           1  fine-level residual r = y - A s, FP32 operator and vectors
 *           2  fine-level residual r = y - A s, FP64
 *           3  one whole V-cycle in FP32 (every level; the dense tail or the
 *              coarsest solve included)
 *           4  one whole V-cycle in FP64
 *   avg_ms, alg_bytes: caller-owned outputs.  Errors: EINVAL, EHIP. */
aspamg_status aspamg_time_kernel(aspamg_handle h, int32_t which, int32_t reps, double *avg_ms,
                                 double *alg_bytes);

/* Measurement entry point: one product of the V-cycle on one level, launched
 * `reps` times back to back on the handle's stream between two HIP events,
 * as in aspamg_time_kernel (average ms per launch and algorithmic bytes of
 * one launch: each stored block with its column index once, each vector
 * entry read or written once).
 *   op = 0  residual r = y - A z          3  restriction r_c = R r
 *        1  t = G r                        4  z += w (G^T G) r, merged (FP32, where stored)
 *        2  z += w G^T t                   5  stacked [P; A P] e (first post-smoothing step)
 *        6  the dense operator of the tail level or of the coarsest level (only there)
 *        7  prolongation z += P e (where the level has no stacked [P; A P])
 *   precision 64 or 32.  Errors: EINVAL (level / op / precision), EHIP. */
aspamg_status aspamg_time_operator(aspamg_handle h, int32_t level, int32_t op, int32_t precision,
                                   int32_t reps, double *avg_ms, double *alg_bytes);

aspamg_status aspamg_destroy(aspamg_handle h);
const char *aspamg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ASPAMG_H */
