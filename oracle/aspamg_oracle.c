/*
 * aspamg_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, sequential, FP64 CPU implementation of the aSP-AMG setup and solve
 * phase (Franceschini, Paludetto Magri, Mazzucco, Spiezia, Janna, "A robust
 * adaptive algebraic multigrid linear solver for structural mechanics").  It is
 * the independent reference that the GPU library is checked against.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header or table with the GPU library.
 *
 * Every step follows the paper in its own order:
 *   recursive setup ............ Section 2, Algorithm "Recursive AMG Setup"
 *   V(nu1,nu2)-cycle ........... Section 2, Algorithm "AMG application in a V-cycle",
 *                                eqs. (2)-(4) (pre-/post-smoothing, coarse correction)
 *   aFSAI smoother ............. Section 3.1, S = I - omega G^T G A, and the
 *                                Algorithm "aFSAI Smoother Set-up"
 *   test space ................. Section 3.3 (V0 given; optional SRQCG smoothing by the
 *                                Algorithm "Test Space generation by SRQCG"; orthonormalised)
 *   affinity SoC + theta + MIS . Section 3.4, eq. (SoC)
 *   DPLS prolongation .......... Section 3.5, eq. (minDPLS) and the Algorithm
 *                                "Dynamic Pattern Least Squares Prolongation"
 *   Galerkin operator .......... Section 2, A_{k+1} = P^T A_k P
 *   PCG ........................ Section 4 (x0 = 0, stop on ||r|| < tol ||b||)
 * Where the paper is silent the readings are the ones listed in the design
 * notes; each is restated at its use site below.  The block size b (1, 2 or 3)
 * is a parameter: with b = 1 every rule is the paper's scalar rule.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math: every decision
 * quantity is plain IEEE binary64 +, -, *, /, sqrt in the order written here).
 * The row loops of the block product and the vector updates of the cycle and
 * of PCG carry OpenMP pragmas for a timing build with -fopenmp (rows are
 * independent, so results are bitwise those of the sequential build); the
 * default build ignores them.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OMAXLEV 32
#define OMAXB 3

/* ------------------------------------------------------------------------- */
/* parameters (the paper's defaults, Table "Default input parameters", plus   */
/* the readings for values the paper leaves unset)                             */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t b;              /* block size                                        */
  int32_t k_g;            /* adaptive FSAI steps per row (paper k_g = 4)       */
  int32_t rho_b;          /* nodes added per FSAI step                         */
  double  eps_g;          /* FSAI exit tolerance (paper 1e-3)                  */
  int32_t theta;          /* retained strong connections per node (paper 5)   */
  int32_t n_max;          /* max interpolation entries per row (paper 5)      */
  double  kappa_p;        /* max conditioning of the local LS (paper 50)       */
  double  omega_bar;      /* target damping of the outer aFSAI loop            */
  int32_t outer_fsai;     /* 1: run the Alg. aFSAI outer loop                  */
  int32_t d_p;            /* max path length for interpolation candidates      */
  double  eps_p;          /* relative LS residual tolerance                    */
  int32_t lanczos_steps;  /* Lanczos steps for lambda_1(G A G^T)               */
  double  omega_safety;   /* omega_s = min(1, 2 / (safety * lambda))           */
  int32_t coarse_max_dof; /* stop coarsening at b*N <= this                    */
  int32_t max_levels;
  double  stall_ratio;    /* stop if N_{l+1} > stall_ratio * N_l               */
  int32_t nu1, nu2;       /* pre / post smoothing steps                        */
  int32_t quant_bits;     /* significant bits of decision quantisation         */
  int32_t dense_max_dof;  /* refuse a dense coarsest system larger than this   */
  int32_t n_rq;           /* SRQCG iterations on each level's test space (0: none) */
  int32_t k_ritz;         /* Ritz projection every k_ritz SRQCG iterations     */
} oparams;

/* status codes */
#define O_OK 0
#define O_NOTCONV 1
#define O_EINVAL -1
#define O_ENOMEM -2
#define O_ENOTSPD -4
#define O_EBREAK -5
#define O_ENAN -6

/* block sparse row matrix: n block rows, blocks b x b row-major */
typedef struct {
  int32_t n, nc, b;       /* block rows, block columns, block size */
  int64_t nnzb;
  int64_t *rp;
  int32_t *ci;
  double *v;
} obsr;

typedef struct {
  obsr A;
  obsr G;                 /* FSAI factor (block lower triangular)   */
  obsr P, R;              /* prolongation n x nc and R = P^T        */
  double lambda1, omega_q, omega_s;
  int32_t fsai_rounds;    /* extra rounds of the outer aFSAI loop   */
  int8_t *cf;             /* 1 C, 0 F, -1 decoupled                 */
  int32_t *cidx;          /* coarse index of C nodes, else -1       */
  int32_t ncoarse;
  double *V;              /* n*b*ntv orthonormalised test space     */
  int64_t *srp;           /* strong graph S (node level)            */
  int32_t *sci;
  double *soc;            /* SoC on A's off-diagonal blocks (A's layout), 0 elsewhere */
  int32_t *pcount;        /* per scalar row: number of P entries     */
  int32_t *pcols;         /* per scalar row: n_max chosen scalar coarse columns (-1 pad) */
  double *work[6];        /* V-cycle work vectors */
} olevel;

typedef struct {
  oparams p;
  int32_t nlev;
  int32_t ntv;
  olevel lev[OMAXLEV];
  int32_t nd;             /* dense coarsest order */
  double *Ld;             /* dense Cholesky factor, row-major lower */
  double min_margin;      /* smallest relative decision margin seen */
} ohier;

static char o_err[512];
const char *oracle_last_error(void) { return o_err; }
static void seterr(const char *m) { snprintf(o_err, sizeof o_err, "%s", m); }

void oracle_default_params(oparams *p) {
  p->b = 3; p->k_g = 4; p->rho_b = 3; p->eps_g = 1e-3; p->theta = 5; p->n_max = 5;
  p->kappa_p = 50.0; p->omega_bar = 0.8; p->outer_fsai = 1; p->d_p = 2; p->eps_p = 1e-8;
  p->lanczos_steps = 30; p->omega_safety = 1.05; p->coarse_max_dof = 1500;
  p->max_levels = 25; p->stall_ratio = 0.9; p->nu1 = 1; p->nu2 = 1; p->quant_bits = 20;
  p->dense_max_dof = 16384; p->n_rq = 0; p->k_ritz = 1;
}

/* ------------------------------------------------------------------------- */
/* decision quantisation: s rounded to `bits` significant bits, ties to even  */
/* ------------------------------------------------------------------------- */
static int QB = 20;
static double qz(double s) {
  if (s == 0.0 || !isfinite(s)) return s;
  int e;
  double m = frexp(s, &e);             /* s = m * 2^e, 0.5 <= |m| < 1 */
  double r = nearbyint(ldexp(m, QB)); /* round half to even in the default mode */
  return ldexp(r, e - QB);
}

static void note_margin(ohier *h, double a, double b) {
  /* relative gap between two compared decision quantities */
  double den = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
  if (den == 0.0) return;
  double m = fabs(a - b) / den;
  if (m > 0.0 && m < h->min_margin) h->min_margin = m;   /* exact ties go to the index rule */
}

/* ------------------------------------------------------------------------- */
/* BSR helpers                                                                 */
/* ------------------------------------------------------------------------- */
static void bsr_free(obsr *M) {
  free(M->rp); free(M->ci); free(M->v);
  memset(M, 0, sizeof *M);
}

static const double *bsr_block(const obsr *M, int32_t r, int32_t c) {
  int64_t lo = M->rp[r], hi = M->rp[r + 1] - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    int32_t cm = M->ci[mid];
    if (cm == c) return M->v + mid * M->b * M->b;
    if (cm < c) lo = mid + 1; else hi = mid - 1;
  }
  return NULL;
}

/* y = M x (scalar vectors of length n*b / nc*b); sums in stored block order */
static void bsr_mv(const obsr *M, const double *x, double *y) {
  int b = M->b;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < M->n; i++) {
    double acc[OMAXB] = {0, 0, 0};
    for (int64_t k = M->rp[i]; k < M->rp[i + 1]; k++) {
      const double *B = M->v + k * b * b;
      const double *xx = x + (int64_t)M->ci[k] * b;
      for (int d = 0; d < b; d++)
        for (int e = 0; e < b; e++) acc[d] += B[d * b + e] * xx[e];
    }
    for (int d = 0; d < b; d++) y[(int64_t)i * b + d] = acc[d];
  }
}

static int bsr_transpose(const obsr *M, obsr *T) {
  int b = M->b;
  T->n = M->nc; T->nc = M->n; T->b = b; T->nnzb = M->nnzb;
  T->rp = calloc((size_t)T->n + 1, sizeof(int64_t));
  T->ci = malloc((size_t)(M->nnzb ? M->nnzb : 1) * sizeof(int32_t));
  T->v = malloc((size_t)(M->nnzb ? M->nnzb : 1) * b * b * sizeof(double));
  if (!T->rp || !T->ci || !T->v) return O_ENOMEM;
  for (int64_t k = 0; k < M->nnzb; k++) T->rp[M->ci[k] + 1]++;
  for (int32_t i = 0; i < T->n; i++) T->rp[i + 1] += T->rp[i];
  int64_t *pos = malloc(((size_t)T->n + 1) * sizeof(int64_t));
  if (!pos) return O_ENOMEM;
  memcpy(pos, T->rp, ((size_t)T->n + 1) * sizeof(int64_t));
  for (int32_t i = 0; i < M->n; i++)            /* ascending source rows -> sorted columns */
    for (int64_t k = M->rp[i]; k < M->rp[i + 1]; k++) {
      int64_t q = pos[M->ci[k]]++;
      T->ci[q] = i;
      const double *S = M->v + k * b * b;
      double *D = T->v + q * b * b;
      for (int d = 0; d < b; d++)
        for (int e = 0; e < b; e++) D[e * b + d] = S[d * b + e];
    }
  free(pos);
  return O_OK;
}

static double dot(const double *a, const double *b, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

/* The inner products of the test-space iteration in one fixed order: the
 * entries in consecutive blocks of 256, each block summed from its first
 * entry, then the block sums from the first block on.  x and y are read with
 * strides sx, sy (columns of a row-major multi-vector). */
#define ODOT_BLOCK 256
static double dotb(const double *x, int64_t sx, const double *y, int64_t sy, int64_t n) {
  double s = 0.0;
  for (int64_t b0 = 0; b0 < n; b0 += ODOT_BLOCK) {
    const int64_t b1 = b0 + ODOT_BLOCK < n ? b0 + ODOT_BLOCK : n;
    double t = 0.0;
    for (int64_t i = b0; i < b1; i++) t += x[i * sx] * y[i * sy];
    s += t;
  }
  return s;
}

/* ------------------------------------------------------------------------- */
/* small dense Cholesky, left-looking, sums in ascending k:                    */
/*   L_jj = sqrt(M_jj - sum_{k<j} L_jk^2),  L_ij = (M_ij - sum_{k<j} L_ik L_jk)/L_jj */
/* returns 0, or -1 at a non-positive pivot                                    */
/* ------------------------------------------------------------------------- */
static int chol_small(const double *M, double *L, int m) {
  for (int j = 0; j < m; j++) {
    double acc = 0.0;
    for (int k = 0; k < j; k++) acc += L[j * m + k] * L[j * m + k];
    double d = M[j * m + j] - acc;
    if (!(d > 0.0)) return -1;
    double ljj = sqrt(d);
    L[j * m + j] = ljj;
    for (int i = j + 1; i < m; i++) {
      double a2 = 0.0;
      for (int k = 0; k < j; k++) a2 += L[i * m + k] * L[j * m + k];
      L[i * m + j] = (M[i * m + j] - a2) / ljj;
    }
    for (int i = 0; i < j; i++) L[i * m + j] = 0.0;
  }
  return 0;
}

/* ========================================================================= */
/* aFSAI (Section 3.1).  Row formula: for block row I with pattern B (nodes    */
/* J < I, ascending) the local list is l = [(J,e) for J in B] + [(I,0..b-1)], */
/* M = A[l,l], M = L L^T, and scalar row (I,d) is g = L_{m_d}^{-T} e_{m_d}    */
/* with m_d = b|B| + d + 1: the FSAI row scaled so that diag(G A G^T) = 1;    */
/* psi_d = L_{m_d m_d}^2 is the minimum of g^T A g over the pattern with      */
/* unit last entry.                                                            */
/* ========================================================================= */
#define OMAXNB 32        /* cap on off-diagonal nodes per FSAI row */
typedef struct {
  int nb;                 /* |B| */
  int32_t nodes[OMAXNB];  /* B (ascending) */
  double g[OMAXB][OMAXNB * OMAXB + OMAXB];
  double psi[OMAXB];
  double psi_sum;
} frow;

static int fsai_factor_row(const obsr *A, int32_t I, frow *R, double *Mbuf, double *Lbuf) {
  int b = A->b, nb = R->nb, m = b * nb + b;
  /* gather M = A[l,l] using block rows of the local list */
  for (int p = 0; p < nb + 1; p++) {
    int32_t rn = p < nb ? R->nodes[p] : I;
    for (int q = 0; q < nb + 1; q++) {
      int32_t cn = q < nb ? R->nodes[q] : I;
      const double *B = bsr_block(A, rn, cn);
      for (int d = 0; d < b; d++)
        for (int e = 0; e < b; e++)
          Mbuf[(p * b + d) * m + q * b + e] = B ? B[d * b + e] : 0.0;
    }
  }
  if (chol_small(Mbuf, Lbuf, m)) return -1;
  double psum = 0.0;
  for (int d = 0; d < b; d++) {
    int md = b * nb + d + 1;            /* size of the leading block */
    double *g = R->g[d];
    g[md - 1] = 1.0 / Lbuf[(md - 1) * m + (md - 1)];
    for (int k = md - 2; k >= 0; k--) {
      double acc = 0.0;
      for (int j = k + 1; j < md; j++) acc += Lbuf[j * m + k] * g[j];
      g[k] = -acc / Lbuf[k * m + k];
    }
    double l = Lbuf[(md - 1) * m + (md - 1)];
    R->psi[d] = l * l;
    psum += R->psi[d];
  }
  R->psi_sum = psum;
  return 0;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

typedef struct { double q; int32_t j; } qcand;
static int cmp_qcand(const void *a, const void *b) {   /* descending q, then ascending j */
  const qcand *x = a, *y = b;
  if (x->q > y->q) return -1;
  if (x->q < y->q) return 1;
  return (x->j > y->j) - (x->j < y->j);
}

/* One adaptive step on row I (the pattern-growth rule): with g' = g / g_last
 * (unit last entry) the gradient entries h_{(I,d),(J,e)} = sum_k A[(J,e), l_k] g'_k
 * are formed for every node J < I outside B that is adjacent in A to B u {I};
 * score_J = sum_d sum_e h^2; the rho_b nodes with the largest quantised score
 * (ties to the lowest J) join B.  Returns the number of nodes added.
 * cand/qc must hold n entries. */
static int fsai_grow_row(ohier *h, const obsr *A, int32_t I, frow *R, int rho, int32_t *mark,
                         int32_t *cand, qcand *qc) {
  int b = A->b, nb = R->nb;
  int ncand = 0;
  if (nb + rho > OMAXNB) return 0;
  /* candidate nodes: A-neighbours of B u {I}, below I, not in B */
  for (int p = 0; p <= nb; p++) {
    int32_t K = p < nb ? R->nodes[p] : I;
    for (int64_t k = A->rp[K]; k < A->rp[K + 1]; k++) {
      int32_t J = A->ci[k];
      if (J >= I || mark[J] == I) continue;
      int inB = 0;
      for (int q = 0; q < nb; q++) if (R->nodes[q] == J) { inB = 1; break; }
      if (inB) continue;
      mark[J] = I;
      cand[ncand++] = J;
    }
  }
  if (ncand == 0) return 0;
  qsort(cand, ncand, sizeof(int32_t), cmp_i32);
  int nq = 0;
  for (int c = 0; c < ncand; c++) {
    int32_t J = cand[c];
    mark[J] = -1;
    double score = 0.0;
    for (int d = 0; d < b; d++) {
      int md = b * nb + d + 1;
      double glast = R->g[d][md - 1];
      for (int e = 0; e < b; e++) {
        double hh = 0.0;
        for (int k = 0; k < md; k++) {
          int32_t nk = (k / b) < nb ? R->nodes[k / b] : I;
          const double *B = bsr_block(A, J, nk);
          if (!B) continue;
          double gp = R->g[d][k] / glast;
          hh += B[e * b + (k % b)] * gp;
        }
        score += hh * hh;
      }
    }
    if (score > 0.0) { qc[nq].q = qz(score); qc[nq].j = J; nq++; }
  }
  if (nq == 0) return 0;
  qsort(qc, nq, sizeof(qcand), cmp_qcand);
  int add = nq < rho ? nq : rho;
  if (add < nq) note_margin(h, qc[add - 1].q, qc[add].q);
  for (int a = 0; a < add; a++) R->nodes[nb + a] = qc[a].j;
  R->nb = nb + add;
  qsort(R->nodes, R->nb, sizeof(int32_t), cmp_i32);
  return add;
}

/* patterns of all rows: pat[i*OMAXNB ..], pnb[i] */
typedef struct { int32_t *pat; int32_t *pnb; } fpatt;

static void load_row(const fpatt *F, int32_t I, frow *R) {
  R->nb = F->pnb[I];
  memcpy(R->nodes, F->pat + (int64_t)I * OMAXNB, R->nb * sizeof(int32_t));
}
static void store_row(fpatt *F, int32_t I, const frow *R) {
  F->pnb[I] = R->nb;
  memcpy(F->pat + (int64_t)I * OMAXNB, R->nodes, R->nb * sizeof(int32_t));
}

/* factor every row for its pattern and write G: off-diagonal blocks full,
 * diagonal block lower triangular */
static int fsai_assemble(const obsr *A, const fpatt *F, obsr *G, double *Mb, double *Lb) {
  int b = A->b;
  int32_t n = A->n;
  frow R;
  G->n = n; G->nc = n; G->b = b;
  G->rp = calloc((size_t)n + 1, sizeof(int64_t));
  if (!G->rp) return O_ENOMEM;
  for (int32_t i = 0; i < n; i++) G->rp[i + 1] = G->rp[i] + F->pnb[i] + 1;
  G->nnzb = G->rp[n];
  G->ci = malloc((size_t)G->nnzb * sizeof(int32_t));
  G->v = calloc((size_t)G->nnzb * b * b, sizeof(double));
  if (!G->ci || !G->v) return O_ENOMEM;
  for (int32_t i = 0; i < n; i++) {
    load_row(F, i, &R);
    if (fsai_factor_row(A, i, &R, Mb, Lb)) { seterr("aFSAI: local system not SPD"); return O_ENOTSPD; }
    int64_t base = G->rp[i];
    for (int p = 0; p <= R.nb; p++) {
      G->ci[base + p] = p < R.nb ? R.nodes[p] : i;
      double *B = G->v + (base + p) * b * b;
      for (int d = 0; d < b; d++)
        for (int e = 0; e < b; e++) {
          if (p == R.nb && e > d) continue;   /* strictly upper part of the diagonal block */
          B[d * b + e] = R.g[d][p * b + e];
        }
    }
  }
  return O_OK;
}

/* first pass of one row: start from B = {} (G = I before scaling), at most k_g
 * growth steps; stop early when psi decreases by no more than eps_g (quantised)
 * or when no candidate remains */
static int fsai_first_pass_row(ohier *h, const obsr *A, int32_t I, frow *R, int32_t *mark,
                               int32_t *cand, qcand *qc, double *Mb, double *Lb) {
  const oparams *p = &h->p;
  R->nb = 0;
  if (fsai_factor_row(A, I, R, Mb, Lb)) return O_ENOTSPD;
  double psi_prev = R->psi_sum;
  for (int s = 0; s < p->k_g; s++) {
    int add = fsai_grow_row(h, A, I, R, p->rho_b, mark, cand, qc);
    if (add == 0) break;
    if (fsai_factor_row(A, I, R, Mb, Lb)) return O_ENOTSPD;
    double dec = qz(psi_prev - R->psi_sum), thr = qz(p->eps_g * psi_prev);
    note_margin(h, psi_prev - R->psi_sum, p->eps_g * psi_prev);
    psi_prev = R->psi_sum;
    if (dec <= thr) break;
  }
  return O_OK;
}

/* plain Lanczos on S = G A G^T (R-F7 start vector), largest Ritz value by
 * Sturm bisection of the tridiagonal T_m */
static double sturm_max(const double *al, const double *be, int m) {
  double lo = al[0], hi = al[0];
  for (int i = 0; i < m; i++) {
    double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i < m - 1 ? fabs(be[i]) : 0.0);
    if (al[i] - r < lo) lo = al[i] - r;
    if (al[i] + r > hi) hi = al[i] + r;
  }
  for (int it = 0; it < 2000; it++) {
    double x = 0.5 * (lo + hi);
    if (x <= lo || x >= hi) break;
    /* count eigenvalues < x */
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < m; i++) {
      double off = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
      d = (al[i] - x) - (i > 0 ? off / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) cnt++;
    }
    if (cnt == m) hi = x; else lo = x;
  }
  return hi;
}

double oracle_lanczos_gagt(const obsr *A, const obsr *G, const obsr *GT, int steps) {
  int64_t n = (int64_t)A->n * A->b;
  double *v = calloc(n, sizeof(double)), *vp = calloc(n, sizeof(double));
  double *u = calloc(n, sizeof(double)), *t1 = calloc(n, sizeof(double)), *t2 = calloc(n, sizeof(double));
  double al[256], be[256];
  if (steps > 255) steps = 255;
  for (int64_t i = 0; i < n; i++) {
    uint64_t hsh = ((uint64_t)i * 2654435761ULL) & 0xFFFFFFFFULL;
    v[i] = (double)hsh / 4294967296.0 - 0.5;
  }
  double nv = sqrt(dot(v, v, n));
  for (int64_t i = 0; i < n; i++) v[i] /= nv;
  int m = 0;
  double bprev = 0.0;
  for (int j = 0; j < steps; j++) {
    bsr_mv(GT, v, t1);
    bsr_mv(A, t1, t2);
    bsr_mv(G, t2, u);
    if (j > 0) for (int64_t i = 0; i < n; i++) u[i] -= bprev * vp[i];
    double a = dot(v, u, n);
    for (int64_t i = 0; i < n; i++) u[i] -= a * v[i];
    double bb = sqrt(dot(u, u, n));
    al[m] = a; be[m] = bb; m++;
    if (!(bb > 1e-300)) break;
    for (int64_t i = 0; i < n; i++) { vp[i] = v[i]; v[i] = u[i] / bb; }
    bprev = bb;
  }
  double lam = sturm_max(al, be, m);
  free(v); free(vp); free(u); free(t1); free(t2);
  return lam;
}

/* Section 3.1 + Algorithm "aFSAI Smoother Set-up" with the readings:
 *   first pass per row as above; then, while omega_q = 2/lambda_1(G A G^T) is
 *   below omega_bar and G is sparser than A, every row gets one more step. */
static int fsai_build(ohier *h, olevel *L) {
  const obsr *A = &L->A;
  const oparams *p = &h->p;
  int b = A->b;
  int32_t n = A->n;
  fpatt F;
  F.pat = malloc((size_t)n * OMAXNB * sizeof(int32_t));
  F.pnb = calloc((size_t)n, sizeof(int32_t));
  int32_t *mark = malloc((size_t)n * sizeof(int32_t));
  int32_t *cand = malloc((size_t)n * sizeof(int32_t));
  qcand *qc = malloc((size_t)n * sizeof(qcand));
  int mmax = OMAXNB * b + b;
  double *Mb = malloc((size_t)mmax * mmax * sizeof(double));
  double *Lb = malloc((size_t)mmax * mmax * sizeof(double));
  frow R;
  int rc = O_OK;
  if (!F.pat || !F.pnb || !mark || !cand || !qc || !Mb || !Lb) { rc = O_ENOMEM; goto done; }
  for (int32_t i = 0; i < n; i++) mark[i] = -1;
  for (int32_t I = 0; I < n; I++) {
    if ((rc = fsai_first_pass_row(h, A, I, &R, mark, cand, qc, Mb, Lb))) {
      seterr("aFSAI: local system not SPD");
      goto done;
    }
    store_row(&F, I, &R);
  }
  if ((rc = fsai_assemble(A, &F, &L->G, Mb, Lb))) goto done;
  L->fsai_rounds = 0;
  for (;;) {
    obsr GT = {0};
    if ((rc = bsr_transpose(&L->G, &GT))) goto done;
    L->lambda1 = oracle_lanczos_gagt(A, &L->G, &GT, p->lanczos_steps);
    bsr_free(&GT);
    L->omega_q = 2.0 / L->lambda1;
    if (!p->outer_fsai) break;
    note_margin(h, L->omega_q, p->omega_bar);
    if (!(qz(L->omega_q) < qz(p->omega_bar))) break;
    if (!(L->G.nnzb < A->nnzb)) break;
    int changed = 0;
    for (int32_t I = 0; I < n; I++) {
      load_row(&F, I, &R);
      if (fsai_factor_row(A, I, &R, Mb, Lb)) { rc = O_ENOTSPD; seterr("aFSAI: local system not SPD"); goto done; }
      int add = fsai_grow_row(h, A, I, &R, p->rho_b, mark, cand, qc);
      if (add == 0) continue;
      changed = 1;
      store_row(&F, I, &R);
    }
    if (!changed) break;
    bsr_free(&L->G);
    if ((rc = fsai_assemble(A, &F, &L->G, Mb, Lb))) goto done;
    L->fsai_rounds++;
  }
  {
    double w = 2.0 / (p->omega_safety * L->lambda1);
    L->omega_s = w < 1.0 ? w : 1.0;
  }
done:
  free(F.pat); free(F.pnb); free(mark); free(cand); free(qc); free(Mb); free(Lb);
  return rc;
}

/* ========================================================================= */
/* test space (Section 3.3): canonical Cholesky-QR orthonormalisation.  Gram  */
/* W = V^T V summed over scalar rows in ascending order, W = L L^T, and each   */
/* row v_i <- L^{-1} v_i.  A column whose pivot is <= 1e-12 W_aa is dropped   */
/* (its entries become 0).                                                     */
/* ========================================================================= */
static int orthonormalize(double *V, int64_t nrows, int ntv) {
  double W[64 * 64], Lm[64 * 64];
  int drop[64];
  if (ntv > 64) return O_EINVAL;
  for (int a = 0; a < ntv; a++)
    for (int c = 0; c < ntv; c++) {
      double s = 0.0;
      for (int64_t i = 0; i < nrows; i++) s += V[i * ntv + a] * V[i * ntv + c];
      W[a * ntv + c] = s;
    }
  for (int j = 0; j < ntv; j++) {
    double acc = 0.0;
    for (int k = 0; k < j; k++) acc += Lm[j * ntv + k] * Lm[j * ntv + k];
    double d = W[j * ntv + j] - acc;
    drop[j] = !(d > 1e-12 * W[j * ntv + j]);
    double ljj = drop[j] ? 1.0 : sqrt(d);
    Lm[j * ntv + j] = ljj;
    for (int i = j + 1; i < ntv; i++) {
      if (drop[j]) { Lm[i * ntv + j] = 0.0; continue; }
      double a2 = 0.0;
      for (int k = 0; k < j; k++) a2 += Lm[i * ntv + k] * Lm[j * ntv + k];
      Lm[i * ntv + j] = (W[i * ntv + j] - a2) / ljj;
    }
  }
  double y[64];
  for (int64_t i = 0; i < nrows; i++) {
    double *v = V + i * ntv;
    for (int a = 0; a < ntv; a++) {
      if (drop[a]) { y[a] = 0.0; continue; }
      double acc = 0.0;
      for (int c = 0; c < a; c++) acc += Lm[a * ntv + c] * y[c];
      y[a] = (v[a] - acc) / Lm[a * ntv + a];
    }
    memcpy(v, y, ntv * sizeof(double));
  }
  return O_OK;
}

/* ========================================================================= */
/* test space by SRQCG (Section 3.3, Algorithm "Test Space generation by      */
/* SRQCG"): simultaneous minimisation of the Rayleigh quotients of the columns */
/* of Z for S = G A G^T by conjugate gradients, with a Ritz projection every   */
/* k_ritz iterations, then V = G^T Z.  Readings where the algorithm is terse:  */
/*   - the iterates live in the variable of S: A v = lambda (G^T G)^{-1} v      */
/*     becomes S z = lambda z with v = G^T z, which is why the algorithm ends   */
/*     with V = G^T Z.  V0 approximates the near kernel of A (v variable), so   */
/*     it enters as G^{-T} V0: Z0 = (I - S) G^{-T} V0.  On an unconstrained K   */
/*     with V0 the rigid-body modes, S G^{-T} V0 = G A V0 = 0 and the modes      */
/*     come back unchanged;                                                    */
/*   - every inner product is summed in the fixed order of dotb (blocks of 256  */
/*     entries), the same order the device uses;                               */
/*   - q is the Rayleigh quotient z^T S z / z^T z; f_i starts at 1 and is set   */
/*     to z_i^T z_i after each update of column i (not after a projection);     */
/*   - S Z is formed by products at every projection and then carried:         */
/*     S z_i <- S z_i + alpha S p_i after an update, S Z <- (S Z) U after a     */
/*     projection;                                                             */
/*   - the projection solves (Z^T S Z) U = (Z^T Z) U Lambda through the         */
/*     Cholesky factor of Z^T Z and Jacobi rotations, eigenvalues ascending,    */
/*     each eigenvector with its largest-magnitude entry positive (the first    */
/*     such entry on ties); it is skipped when Z^T Z is not positive definite;  */
/*   - a column update with 2(bc - ad) = 0 or Delta < 0 is skipped;            */
/*   - exactly k_max iterations run (no early exit).                           */
/* Z and V are row-major [nrows][nt] like the test space.                      */
/* ========================================================================= */

/* x <- G^{-T} x: back substitution with the rows of the lower triangular G,  */
/* scalar rows from the last to the first; x_r is divided by g_rr and then     */
/* g_rk x_r is subtracted from every x_k, k < r, of row r                      */
static void gt_solve(const obsr *G, double *x) {
  const int b = G->b;
  for (int64_t r = (int64_t)G->n * b - 1; r >= 0; r--) {
    const int32_t I = (int32_t)(r / b);
    const int d = (int)(r % b);
    const double *dg = bsr_block(G, I, I);
    x[r] /= dg[d * b + d];
    for (int64_t k = G->rp[I]; k < G->rp[I + 1]; k++) {
      const int32_t J = G->ci[k];
      const int ne = J < I ? b : d;          /* the diagonal block: columns e < d */
      for (int e = 0; e < ne; e++) x[(int64_t)J * b + e] -= G->v[k * b * b + d * b + e] * x[r];
    }
  }
}

/* S x = G (A (G^T x)) */
static void apply_gagt(const obsr *A, const obsr *G, const obsr *GT, const double *x, double *y, double *t1,
                       double *t2) {
  bsr_mv(GT, x, t1);
  bsr_mv(A, t1, t2);
  bsr_mv(G, t2, y);
}

/* symmetric m x m matrix C (destroyed): C = X diag(w) X^T by cyclic Jacobi
 * sweeps (Golub and Van Loan, "Matrix Computations", Section 8.5); w ascending,
 * eigenvectors in the columns of X */
static void jacobi_eigen(double *C, int m, double *w, double *X) {
  for (int i = 0; i < m; i++)
    for (int j = 0; j < m; j++) X[i * m + j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; i++)
      for (int j = 0; j < m; j++) {
        tot += C[i * m + j] * C[i * m + j];
        if (i != j) off += C[i * m + j] * C[i * m + j];
      }
    if (!(off > 1e-32 * tot)) break;
    for (int p = 0; p < m - 1; p++)
      for (int q = p + 1; q < m; q++) {
        double apq = C[p * m + q];
        if (apq == 0.0) continue;
        /* rotation that zeroes C[p][q]: tan t = sign(theta) / (|theta| + sqrt(theta^2 + 1)) */
        double theta = (C[q * m + q] - C[p * m + p]) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; k++) {      /* columns p, q: C <- C J */
          double ckp = C[k * m + p], ckq = C[k * m + q];
          C[k * m + p] = c * ckp - s * ckq;
          C[k * m + q] = s * ckp + c * ckq;
        }
        for (int k = 0; k < m; k++) {      /* rows p, q: C <- J^T C */
          double cpk = C[p * m + k], cqk = C[q * m + k];
          C[p * m + k] = c * cpk - s * cqk;
          C[q * m + k] = s * cpk + c * cqk;
        }
        for (int k = 0; k < m; k++) {      /* X <- X J */
          double xkp = X[k * m + p], xkq = X[k * m + q];
          X[k * m + p] = c * xkp - s * xkq;
          X[k * m + q] = s * xkp + c * xkq;
        }
      }
  }
  for (int i = 0; i < m; i++) w[i] = C[i * m + i];
  /* selection sort, ascending eigenvalues (stable for equal values) */
  for (int i = 0; i < m; i++) {
    int k = i;
    for (int j = i + 1; j < m; j++)
      if (w[j] < w[k]) k = j;
    if (k != i) {
      double tw = w[i]; w[i] = w[k]; w[k] = tw;
      for (int r = 0; r < m; r++) { double tx = X[r * m + i]; X[r * m + i] = X[r * m + k]; X[r * m + k] = tx; }
    }
  }
}

/* Ritz step: U with (Z^T S Z) U = (Z^T Z) U Lambda; returns -1 when Z^T Z is not SPD */
static int ritz_vectors(const double *Z, const double *SZ, int64_t nr, int nt, double *U) {
  double Ms[64 * 64], Mz[64 * 64], L[64 * 64], C[64 * 64], T[64 * 64], X[64 * 64], w[64];
  for (int a = 0; a < nt; a++)
    for (int c = 0; c < nt; c++) {
      Ms[a * nt + c] = dotb(Z + a, nt, SZ + c, nt, nr);
      Mz[a * nt + c] = dotb(Z + a, nt, Z + c, nt, nr);
    }
  for (int a = 0; a < nt; a++)          /* symmetric parts */
    for (int c = 0; c < a; c++) {
      double s = 0.5 * (Ms[a * nt + c] + Ms[c * nt + a]);
      Ms[a * nt + c] = Ms[c * nt + a] = s;
    }
  if (chol_small(Mz, L, nt)) return -1;
  /* T = L^{-1} Ms (forward substitution column by column), C = T L^{-T} */
  for (int c = 0; c < nt; c++)
    for (int i = 0; i < nt; i++) {
      double acc = Ms[i * nt + c];
      for (int k = 0; k < i; k++) acc -= L[i * nt + k] * T[k * nt + c];
      T[i * nt + c] = acc / L[i * nt + i];
    }
  for (int r = 0; r < nt; r++)
    for (int i = 0; i < nt; i++) {
      double acc = T[r * nt + i];
      for (int k = 0; k < i; k++) acc -= L[i * nt + k] * C[r * nt + k];
      C[r * nt + i] = acc / L[i * nt + i];
    }
  for (int a = 0; a < nt; a++)
    for (int c = 0; c < a; c++) {
      double s = 0.5 * (C[a * nt + c] + C[c * nt + a]);
      C[a * nt + c] = C[c * nt + a] = s;
    }
  jacobi_eigen(C, nt, w, X);
  /* U = L^{-T} X (back substitution), then the sign rule */
  for (int c = 0; c < nt; c++) {
    for (int i = nt - 1; i >= 0; i--) {
      double acc = X[i * nt + c];
      for (int k = i + 1; k < nt; k++) acc -= L[k * nt + i] * U[k * nt + c];
      U[i * nt + c] = acc / L[i * nt + i];
    }
    int imax = 0;
    for (int i = 1; i < nt; i++)
      if (fabs(U[i * nt + c]) > fabs(U[imax * nt + c])) imax = i;
    if (U[imax * nt + c] < 0.0)
      for (int i = 0; i < nt; i++) U[i * nt + c] = -U[i * nt + c];
  }
  return 0;
}

/* V (row-major [nr][nt], in: V0, out: G^T Z); rq (optional, nt entries):
 * the Rayleigh quotients of the columns of Z at the end */
static int srqcg(const obsr *A, const obsr *G, double *V, int nt, int kmax, int kritz, double *rq) {
  int64_t nr = (int64_t)A->n * A->b;
  if (nt < 1 || nt > 64 || kritz < 1 || kmax < 0) return O_EINVAL;
  obsr GT = {0};
  int rc = bsr_transpose(G, &GT);
  double *Z = malloc((size_t)nr * nt * sizeof(double)), *SZ = malloc((size_t)nr * nt * sizeof(double));
  double *Pd = malloc((size_t)nr * nt * sizeof(double));
  double *x = malloc((size_t)nr * sizeof(double)), *y = malloc((size_t)nr * sizeof(double));
  double *t1 = malloc((size_t)nr * sizeof(double)), *t2 = malloc((size_t)nr * sizeof(double));
  double *sp = malloc((size_t)nr * sizeof(double)), *g = malloc((size_t)nr * sizeof(double));
  double f[64], U[64 * 64];
  if (rc || !Z || !SZ || !Pd || !x || !y || !t1 || !t2 || !sp || !g) { rc = O_ENOMEM; goto done; }
  /* Z0 = (I - S) G^{-T} V0, orthonormalised */
  for (int c = 0; c < nt; c++) {
    for (int64_t i = 0; i < nr; i++) x[i] = V[i * nt + c];
    gt_solve(G, x);
    apply_gagt(A, G, &GT, x, y, t1, t2);
    for (int64_t i = 0; i < nr; i++) Z[i * nt + c] = x[i] - y[i];
  }
  if ((rc = orthonormalize(Z, nr, nt))) goto done;
  /* initial residuals and search directions */
  for (int c = 0; c < nt; c++) {
    for (int64_t i = 0; i < nr; i++) x[i] = Z[i * nt + c];
    apply_gagt(A, G, &GT, x, y, t1, t2);
    double e = dotb(x, 1, y, 1, nr), ff = dotb(x, 1, x, 1, nr);
    double q = ff > 0.0 ? e / ff : 0.0;
    for (int64_t i = 0; i < nr; i++) {
      SZ[i * nt + c] = y[i];
      Pd[i * nt + c] = 2.0 * (y[i] - q * x[i]);
    }
    f[c] = 1.0;
  }
  for (int k = 1; k <= kmax; k++) {
    if (k % kritz == 0) {
      for (int c = 0; c < nt; c++) {         /* S Z by products */
        for (int64_t i = 0; i < nr; i++) x[i] = Z[i * nt + c];
        apply_gagt(A, G, &GT, x, y, t1, t2);
        for (int64_t i = 0; i < nr; i++) SZ[i * nt + c] = y[i];
      }
      if (ritz_vectors(Z, SZ, nr, nt, U) == 0)
        for (int64_t i = 0; i < nr; i++) {   /* Z <- Z U, S Z <- (S Z) U, row by row */
          double zr[64], sr[64];
          for (int c = 0; c < nt; c++) {
            double s1 = 0.0, s2 = 0.0;
            for (int j = 0; j < nt; j++) {
              s1 += Z[i * nt + j] * U[j * nt + c];
              s2 += SZ[i * nt + j] * U[j * nt + c];
            }
            zr[c] = s1;
            sr[c] = s2;
          }
          memcpy(Z + i * nt, zr, nt * sizeof(double));
          memcpy(SZ + i * nt, sr, nt * sizeof(double));
        }
    }
    for (int c = 0; c < nt; c++) {
      /* column c: z = Z_c, p = P_c, sz = (S Z)_c, sp = S p */
      for (int64_t i = 0; i < nr; i++) x[i] = Pd[i * nt + c];
      apply_gagt(A, G, &GT, x, sp, t1, t2);
      const double *pc = Pd + c, *zc = Z + c, *szc = SZ + c;
      const double a = dotb(pc, nt, szc, nt, nr), b = dotb(pc, nt, sp, 1, nr), cc = dotb(pc, nt, zc, nt, nr),
                   d = dotb(pc, nt, pc, nt, nr), e = dotb(zc, nt, szc, nt, nr);
      const double fi = f[c];
      const double den = 2.0 * (b * cc - a * d);
      const double u1 = d * e - b * fi;
      const double delta = u1 * u1 - 4.0 * (b * cc - a * d) * (a * fi - cc * e);
      if (!(den != 0.0) || !(delta >= 0.0)) continue;
      const double alpha = (u1 + sqrt(delta)) / den;   /* minimiser of the quotient on z + alpha p */
      for (int64_t i = 0; i < nr; i++) {
        Z[i * nt + c] += alpha * Pd[i * nt + c];
        SZ[i * nt + c] += alpha * sp[i];
      }
      const double zz = dotb(Z + c, nt, Z + c, nt, nr), zsz = dotb(Z + c, nt, SZ + c, nt, nr);
      f[c] = zz;
      const double q = zsz / zz;
      /* gradient of the quotient, g = 2 (S z - q z) / f, and the new direction */
      for (int64_t i = 0; i < nr; i++) g[i] = 2.0 * (SZ[i * nt + c] - q * Z[i * nt + c]) / zz;
      const double beta = -dotb(g, 1, sp, 1, nr) / b;
      for (int64_t i = 0; i < nr; i++) Pd[i * nt + c] = g[i] + beta * Pd[i * nt + c];
    }
  }
  if (rq)
    for (int c = 0; c < nt; c++) {
      const double zz = dotb(Z + c, nt, Z + c, nt, nr), zsz = dotb(Z + c, nt, SZ + c, nt, nr);
      rq[c] = zz > 0.0 ? zsz / zz : 0.0;
    }
  /* V = G^T Z */
  for (int c = 0; c < nt; c++) {
    for (int64_t i = 0; i < nr; i++) x[i] = Z[i * nt + c];
    bsr_mv(&GT, x, y);
    for (int64_t i = 0; i < nr; i++) V[i * nt + c] = y[i];
  }
done:
  free(Z); free(SZ); free(Pd); free(x); free(y); free(t1); free(t2); free(sp); free(g);
  bsr_free(&GT);
  return rc;
}

/* ========================================================================= */
/* coarsening (Section 3.4)                                                    */
/* ========================================================================= */
static int decoupled(const obsr *A, int32_t i) {
  return A->rp[i + 1] - A->rp[i] == 1 && A->ci[A->rp[i]] == i;
}

/* node affinity: M_IJ = V_I V_J^T (b x b, sums over t ascending),
 * n_IJ = sum of squares of M_IJ in row-major order; for b = 1 this is
 * (v_i^T v_j)^2, the numerator of eq. (SoC). */
static double node_n(const double *V, int b, int ntv, int32_t I, int32_t J) {
  double s = 0.0;
  for (int d = 0; d < b; d++)
    for (int e = 0; e < b; e++) {
      double m = 0.0;
      const double *vi = V + ((int64_t)I * b + d) * ntv, *vj = V + ((int64_t)J * b + e) * ntv;
      for (int t = 0; t < ntv; t++) m += vi[t] * vj[t];
      s += m * m;
    }
  return s;
}

/* SoC[I,J] = n_IJ / (sqrt(n_II) sqrt(n_JJ)), evaluated with (I,J) ordered so that I < J */
static double soc_pair(const double *V, int b, int ntv, int32_t I, int32_t J, const double *sq) {
  int32_t a = I < J ? I : J, c = I < J ? J : I;
  double den = sq[a] * sq[c];
  if (!(den > 0.0)) return 0.0;
  return node_n(V, b, ntv, a, c) / den;
}

static uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct { int32_t deg; uint64_t hsh; int32_t id; } mkey;
static int cmp_mkey(const void *a, const void *b) {   /* descending (deg, hash), then ascending id */
  const mkey *x = a, *y = b;
  if (x->deg != y->deg) return x->deg > y->deg ? -1 : 1;
  if (x->hsh != y->hsh) return x->hsh > y->hsh ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

/* Greedy maximal independent set on the strong graph in descending key order:
 * a node becomes C unless one of its S-neighbours is already C. */
void oracle_mis(int32_t n, const int64_t *srp, const int32_t *sci, const int8_t *excluded, int8_t *cf) {
  mkey *keys = malloc((size_t)n * sizeof(mkey));
  int32_t nk = 0;
  for (int32_t i = 0; i < n; i++) {
    cf[i] = excluded && excluded[i] ? -1 : 2;   /* 2 = undecided */
    if (cf[i] == 2) {
      keys[nk].deg = (int32_t)(srp[i + 1] - srp[i]);
      keys[nk].hsh = splitmix64((uint64_t)i);
      keys[nk].id = i;
      nk++;
    }
  }
  qsort(keys, nk, sizeof(mkey), cmp_mkey);
  for (int32_t t = 0; t < nk; t++) {
    int32_t i = keys[t].id;
    int hasC = 0;
    for (int64_t k = srp[i]; k < srp[i + 1]; k++) if (cf[sci[k]] == 1) { hasC = 1; break; }
    cf[i] = hasC ? 0 : 1;
  }
  free(keys);
}

/* SoC on A's off-diagonal blocks -> keep min(theta, deg) strongest per node
 * (quantised, ties to the lowest J) -> symmetrise by union -> S. */
static int coarsen(ohier *h, olevel *L) {
  const obsr *A = &L->A;
  int b = A->b, ntv = h->ntv;
  int32_t n = A->n;
  double *sq = malloc((size_t)n * sizeof(double));
  L->soc = calloc((size_t)A->nnzb, sizeof(double));
  int8_t *excl = malloc((size_t)n);
  L->cf = malloc((size_t)n);
  if (!sq || !L->soc || !excl || !L->cf) return O_ENOMEM;
  for (int32_t i = 0; i < n; i++) {
    excl[i] = (int8_t)decoupled(A, i);
    sq[i] = sqrt(node_n(L->V, b, ntv, i, i));
  }
  for (int32_t i = 0; i < n; i++) {
    if (excl[i]) continue;
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; k++) {
      int32_t j = A->ci[k];
      if (j == i || excl[j]) continue;
      L->soc[k] = soc_pair(L->V, b, ntv, i, j, sq);
    }
  }
  /* theta filter: directed keep lists */
  int theta = h->p.theta;
  int32_t *keep = malloc((size_t)n * (theta > 0 ? theta : 1) * sizeof(int32_t));
  int32_t *nkeep = calloc((size_t)n, sizeof(int32_t));
  int64_t maxrow = 1;
  for (int32_t i = 0; i < n; i++) if (A->rp[i + 1] - A->rp[i] > maxrow) maxrow = A->rp[i + 1] - A->rp[i];
  qcand *qc = malloc((size_t)maxrow * sizeof(qcand));
  if (!keep || !nkeep || !qc) return O_ENOMEM;
  for (int32_t i = 0; i < n; i++) {
    if (excl[i]) continue;
    int nq = 0;
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; k++) {
      if (L->soc[k] > 0.0) { qc[nq].q = qz(L->soc[k]); qc[nq].j = A->ci[k]; nq++; }
    }
    qsort(qc, nq, sizeof(qcand), cmp_qcand);
    int kk = nq < theta ? nq : theta;
    if (kk < nq) note_margin(h, qc[kk - 1].q, qc[kk].q);
    for (int a = 0; a < kk; a++) keep[(int64_t)i * theta + a] = qc[a].j;
    nkeep[i] = kk;
  }
  /* union symmetrisation: edge {i,j} if i keeps j or j keeps i */
  int64_t *cnt = calloc((size_t)n + 1, sizeof(int64_t));
  for (int32_t i = 0; i < n; i++)
    for (int a = 0; a < nkeep[i]; a++) {
      int32_t j = keep[(int64_t)i * theta + a];
      int dup = 0;   /* j also keeps i: count once from the smaller end */
      for (int c = 0; c < nkeep[j]; c++) if (keep[(int64_t)j * theta + c] == i) { dup = 1; break; }
      if (dup && j < i) continue;
      cnt[i + 1]++; cnt[j + 1]++;
    }
  for (int32_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
  L->srp = cnt;
  L->sci = malloc((size_t)(cnt[n] ? cnt[n] : 1) * sizeof(int32_t));
  int64_t *pos = malloc(((size_t)n + 1) * sizeof(int64_t));
  memcpy(pos, cnt, ((size_t)n + 1) * sizeof(int64_t));
  for (int32_t i = 0; i < n; i++)
    for (int a = 0; a < nkeep[i]; a++) {
      int32_t j = keep[(int64_t)i * theta + a];
      int dup = 0;
      for (int c = 0; c < nkeep[j]; c++) if (keep[(int64_t)j * theta + c] == i) { dup = 1; break; }
      if (dup && j < i) continue;
      L->sci[pos[i]++] = j;
      L->sci[pos[j]++] = i;
    }
  for (int32_t i = 0; i < n; i++)
    qsort(L->sci + L->srp[i], L->srp[i + 1] - L->srp[i], sizeof(int32_t), cmp_i32);
  free(pos);
  oracle_mis(n, L->srp, L->sci, excl, L->cf);
  L->cidx = malloc((size_t)n * sizeof(int32_t));
  int32_t nc = 0;
  for (int32_t i = 0; i < n; i++) L->cidx[i] = L->cf[i] == 1 ? nc++ : -1;
  L->ncoarse = nc;
  free(sq); free(excl); free(keep); free(nkeep); free(qc);
  return O_OK;
}

/* ========================================================================= */
/* DPLS prolongation (Section 3.5, Algorithm "Dynamic Pattern Least Squares  */
/* Prolongation").  For scalar row (I,d) of an F node the target is           */
/* v = V[(I,d)], the candidates are the scalar rows (J,e) of C nodes within   */
/* S-distance d_p, ascending.  Householder form: after k accepted columns the */
/* residual r and every candidate c_a have been reflected by H_{k-1}..H_0, so */
/* their trailing parts (entries k..ntv-1) are their components orthogonal to */
/* the chosen columns.  With rho^2 = |r_tail|^2, delta_a^2 = |c_a,tail|^2 and */
/* pi_a = c_a,tail . r_tail, the affinity is pi_a^2 / (rho^2 delta_a^2) (at   */
/* step 0 the paper's affinity).  The argmax of the quantised affinity (> 0,  */
/* ties to the lowest candidate) is accepted unless max|R_kk| / min|R_kk|, a  */
/* lower bound of cond(V_{c,i}), would exceed kappa_p.  Stops at n_max       */
/* entries, or rho^2 <= eps_p^2 v.v, or when no candidate is eligible.        */
/* Weights: the least-squares fit V_c w = v of eq. (minDPLS) through its     */
/* normal equations (C^T C) w = C^T v, by Cholesky: equal in exact arithmetic */
/* to the back substitution w = R^{-1} (Q^T v) of the algorithm, and          */
/* well-conditioned because the kappa guard bounds cond(C^T C) by kappa_p^2.  */
/* Reflection of column u at step k (sums ascending in t):                    */
/*   delta = sqrt(sum_{t>=k} u_t^2), alpha = -delta if u_k >= 0 else delta,   */
/*   h = u_tail with h_k = u_k - alpha, s = h_k^2 + sum_{t>k} u_t^2,           */
/*   x_tail <- x_tail - (2 (h . x_tail) / s) h.                                */
/* ========================================================================= */
typedef struct {
  int k;
  int32_t col[16];     /* chosen scalar candidate indices into the candidate list */
  double w[16];
} dpls_out;

static int dpls_row(ohier *h, const double *v, const double *C, int nca, int ntv, dpls_out *o,
                    double *Cw, double *unused1, double *unused2) {
  (void)unused1; (void)unused2;
  const oparams *p = &h->p;
  double vv = 0.0;
  for (int s = 0; s < ntv; s++) vv += v[s] * v[s];
  o->k = 0;
  if (vv == 0.0) return 0;
  double r[64], Rm[16][16], hv[64];
  memcpy(r, v, ntv * sizeof(double));
  memcpy(Cw, C, (size_t)nca * ntv * sizeof(double));
  char *used = calloc(nca > 0 ? nca : 1, 1);
  const double thr = qz((p->eps_p * p->eps_p) * vv);
  int nmax = p->n_max < 16 ? p->n_max : 16;
  double dmax = 0.0, dmin = 0.0;
  int K = 0;
  while (K < nmax && K < ntv) {
    double rho2 = 0.0;
    for (int t = K; t < ntv; t++) rho2 += r[t] * r[t];
    if (!(qz(rho2) > thr)) break;
    int best = -1;
    double bestq = 0.0, bdel2 = 0.0, secondq = -1.0;
    for (int a = 0; a < nca; a++) {
      if (used[a]) continue;
      const double *c = Cw + (size_t)a * ntv;
      double del2 = 0.0, pi = 0.0;
      for (int t = K; t < ntv; t++) del2 += c[t] * c[t];
      if (!(del2 > 0.0)) continue;
      for (int t = K; t < ntv; t++) pi += c[t] * r[t];
      const double aff = (pi * pi) / (rho2 * del2);
      const double q = qz(aff);
      if (q > bestq) {
        if (best >= 0 && bestq > secondq) secondq = bestq;
        best = a; bestq = q; bdel2 = del2;
      } else if (q > secondq) {
        secondq = q;
      }
    }
    if (best < 0) break;
    if (secondq > 0.0) note_margin(h, bestq, secondq);
    const double del = sqrt(bdel2);
    const double mx = K ? (dmax > del ? dmax : del) : del;
    const double mn = K ? (dmin < del ? dmin : del) : del;
    note_margin(h, mx / mn, p->kappa_p);
    if (qz(mx / mn) > qz(p->kappa_p)) break;
    /* Householder reflection of the chosen column's trailing part */
    double *u = Cw + (size_t)best * ntv;
    const double alpha = u[K] >= 0.0 ? -del : del;
    for (int t = K; t < ntv; t++) hv[t] = u[t];
    hv[K] = u[K] - alpha;
    double sh = hv[K] * hv[K];
    for (int t = K + 1; t < ntv; t++) sh += hv[t] * hv[t];
    for (int a = 0; a <= nca; a++) {          /* a == nca: the residual r */
      if (a < nca && (used[a] || a == best)) continue;
      double *x = a < nca ? Cw + (size_t)a * ntv : r;
      double tau = 0.0;
      for (int t = K; t < ntv; t++) tau += hv[t] * x[t];
      const double fct = (2.0 * tau) / sh;
      for (int t = K; t < ntv; t++) x[t] = x[t] - fct * hv[t];
    }
    for (int i = 0; i < K; i++) Rm[i][K] = u[i];
    Rm[K][K] = alpha;
    dmax = mx; dmin = mn;
    o->col[K] = best;
    used[best] = 1;
    K++;
  }
  /* weights (the normal equations of the chosen columns, in the order chosen):
   * t_a = c_a . v, Gram g_ac = c_a . c_c (c <= a), Cholesky g = L L^T,
   * L y = t, L^T w = y; all sums ascending */
  double Gm[16][16], Lc[16][16], tt[16], y[16], w[16];
  for (int a = 0; a < K; a++) {
    const double *ca = C + (size_t)o->col[a] * ntv;
    double s1 = 0.0;
    for (int q = 0; q < ntv; q++) s1 += ca[q] * v[q];
    tt[a] = s1;
    for (int c = 0; c <= a; c++) {
      const double *cc = C + (size_t)o->col[c] * ntv;
      double g = 0.0;
      for (int q = 0; q < ntv; q++) g += ca[q] * cc[q];
      Gm[a][c] = g;
    }
  }
  for (int j = 0; j < K; j++) {
    double acc = 0.0;
    for (int k = 0; k < j; k++) acc += Lc[j][k] * Lc[j][k];
    const double dd = Gm[j][j] - acc;
    /* the kappa guard bounds cond(C^T C) by kappa_p^2, so a non-positive
     * pivot means the chosen columns are dependent: an error, not a fit */
    if (!(dd > 0.0)) { free(used); seterr("DPLS: weight Gram matrix not positive definite"); return O_ENOTSPD; }
    Lc[j][j] = sqrt(dd);
    for (int a = j + 1; a < K; a++) {
      double a2 = 0.0;
      for (int k = 0; k < j; k++) a2 += Lc[a][k] * Lc[j][k];
      Lc[a][j] = (Gm[a][j] - a2) / Lc[j][j];
    }
  }
  for (int a = 0; a < K; a++) {
    double acc = 0.0;
    for (int c = 0; c < a; c++) acc += Lc[a][c] * y[c];
    y[a] = (tt[a] - acc) / Lc[a][a];
  }
  for (int a = K - 1; a >= 0; a--) {
    double acc = 0.0;
    for (int c = a + 1; c < K; c++) acc += Lc[c][a] * w[c];
    w[a] = (y[a] - acc) / Lc[a][a];
  }
  (void)Rm;
  o->k = K;
  for (int k = 0; k < K; k++) o->w[k] = w[k];
  free(used);
  return 0;
}

/* interpolation candidates of node I (R-P1): the C nodes joined to I by a
 * path of at most d_p edges of the strong graph S, ascending.  Breadth-first
 * search; mark and dist hold -1 for every node on entry and on exit (mark is
 * set to I while the search runs). */
static int candidate_nodes(const olevel *L, int32_t I, int d_p, int32_t *mark, int32_t *frontier, int32_t *dist,
                           int32_t *cn) {
  int nf = 0, ncn = 0;
  frontier[nf++] = I; dist[I] = 0; mark[I] = I;
  for (int head = 0; head < nf; head++) {
    int32_t u = frontier[head];
    if (dist[u] >= d_p) continue;
    for (int64_t k = L->srp[u]; k < L->srp[u + 1]; k++) {
      int32_t w = L->sci[k];
      if (mark[w] == I) continue;
      mark[w] = I; dist[w] = dist[u] + 1;
      frontier[nf++] = w;
      if (L->cf[w] == 1) cn[ncn++] = w;
    }
  }
  for (int q = 0; q < nf; q++) { dist[frontier[q]] = -1; mark[frontier[q]] = -1; }
  qsort(cn, ncn, sizeof(int32_t), cmp_i32);
  return ncn;
}

static int build_P(ohier *h, olevel *L) {
  const obsr *A = &L->A;
  int b = A->b, ntv = h->ntv, nmax = h->p.n_max;
  int32_t n = A->n, nc = L->ncoarse;
  int32_t *mark = malloc((size_t)n * sizeof(int32_t));
  int32_t *cn = malloc((size_t)n * sizeof(int32_t));      /* candidate C nodes */
  int32_t *frontier = malloc((size_t)n * sizeof(int32_t));
  int32_t *dist = malloc((size_t)n * sizeof(int32_t));
  L->pcount = calloc((size_t)n * b, sizeof(int32_t));
  L->pcols = malloc((size_t)n * b * nmax * sizeof(int32_t));
  /* per row block lists, assembled afterwards */
  int64_t *rp = calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *tmpc = malloc(((size_t)b * nmax + 1) * sizeof(int32_t));
  if (!mark || !cn || !frontier || !dist || !L->pcount || !L->pcols || !rp || !tmpc) return O_ENOMEM;
  for (int64_t i = 0; i < (int64_t)n * b * nmax; i++) L->pcols[i] = -1;
  double *wv = malloc((size_t)n * b * nmax * sizeof(double));
  for (int32_t i = 0; i < n; i++) { mark[i] = -1; dist[i] = -1; }
  int cap = 1024;
  double *Cm = malloc((size_t)cap * b * ntv * sizeof(double));
  double *t = malloc((size_t)cap * b * sizeof(double)), *gaa = malloc((size_t)cap * b * sizeof(double));
  double *gbuf = malloc((size_t)cap * b * ntv * sizeof(double));
  int32_t *cnode = malloc((size_t)cap * b * sizeof(int32_t));
  int8_t *ccomp = malloc((size_t)cap * b);
  if (!wv || !Cm || !t || !gaa || !gbuf || !cnode || !ccomp) return O_ENOMEM;
  for (int32_t I = 0; I < n; I++) {
    if (L->cf[I] != 0) continue;
    int ncn = candidate_nodes(L, I, h->p.d_p, mark, frontier, dist, cn);
    if (ncn > cap) {
      cap = ncn;
      Cm = realloc(Cm, (size_t)cap * b * ntv * sizeof(double));
      t = realloc(t, (size_t)cap * b * sizeof(double)); gaa = realloc(gaa, (size_t)cap * b * sizeof(double));
      gbuf = realloc(gbuf, (size_t)cap * b * ntv * sizeof(double));
      cnode = realloc(cnode, (size_t)cap * b * sizeof(int32_t)); ccomp = realloc(ccomp, (size_t)cap * b);
    }
    int nca = 0;
    for (int c = 0; c < ncn; c++)
      for (int e = 0; e < b; e++) {
        memcpy(Cm + (int64_t)nca * ntv, L->V + ((int64_t)cn[c] * b + e) * ntv, ntv * sizeof(double));
        cnode[nca] = cn[c]; ccomp[nca] = (int8_t)e; nca++;
      }
    for (int d = 0; d < b; d++) {
      dpls_out o;
      int rc = dpls_row(h, L->V + ((int64_t)I * b + d) * ntv, Cm, nca, ntv, &o, gbuf, t, gaa);
      if (rc) return rc;
      int64_t r = (int64_t)I * b + d;
      L->pcount[r] = o.k;
      for (int k = 0; k < o.k; k++) {
        int a = o.col[k];
        L->pcols[r * nmax + k] = L->cidx[cnode[a]] * b + ccomp[a];
        wv[r * nmax + k] = o.w[k];
      }
    }
  }
  /* assemble P: C rows I_b at (I, c(I)); F rows: union of chosen coarse nodes */
  for (int32_t I = 0; I < n; I++) {
    int cntb = 0;
    if (L->cf[I] == 1) cntb = 1;
    else if (L->cf[I] == 0) {
      int m = 0;
      for (int d = 0; d < b; d++)
        for (int k = 0; k < L->pcount[(int64_t)I * b + d]; k++) tmpc[m++] = L->pcols[((int64_t)I * b + d) * nmax + k] / b;
      qsort(tmpc, m, sizeof(int32_t), cmp_i32);
      for (int a = 0; a < m; a++) if (a == 0 || tmpc[a] != tmpc[a - 1]) cntb++;
    }
    rp[I + 1] = rp[I] + cntb;
  }
  obsr *P = &L->P;
  P->n = n; P->nc = nc; P->b = b; P->nnzb = rp[n]; P->rp = rp;
  P->ci = malloc((size_t)(P->nnzb ? P->nnzb : 1) * sizeof(int32_t));
  P->v = calloc((size_t)(P->nnzb ? P->nnzb : 1) * b * b, sizeof(double));
  if (!P->ci || !P->v) return O_ENOMEM;
  for (int32_t I = 0; I < n; I++) {
    int64_t base = rp[I];
    if (L->cf[I] == 1) {
      P->ci[base] = L->cidx[I];
      for (int d = 0; d < b; d++) P->v[base * b * b + d * b + d] = 1.0;
    } else if (L->cf[I] == 0) {
      int m = 0;
      for (int d = 0; d < b; d++)
        for (int k = 0; k < L->pcount[(int64_t)I * b + d]; k++) tmpc[m++] = L->pcols[((int64_t)I * b + d) * nmax + k] / b;
      qsort(tmpc, m, sizeof(int32_t), cmp_i32);
      int u = 0;
      for (int a = 0; a < m; a++) if (a == 0 || tmpc[a] != tmpc[a - 1]) P->ci[base + u++] = tmpc[a];
      for (int d = 0; d < b; d++) {
        int64_t r = (int64_t)I * b + d;
        for (int k = 0; k < L->pcount[r]; k++) {
          int32_t sc = L->pcols[r * nmax + k];
          int32_t cnod = sc / b, e = sc % b;
          int q = 0;
          while (P->ci[base + q] != cnod) q++;
          P->v[(base + q) * b * b + d * b + e] = wv[r * nmax + k];
        }
      }
    }
  }
  free(mark); free(cn); free(frontier); free(dist); free(tmpc); free(wv);
  free(Cm); free(t); free(gaa); free(gbuf); free(cnode); free(ccomp);
  return bsr_transpose(&L->P, &L->R);
}

/* ========================================================================= */
/* Galerkin operator A_c = R (A P), R = P^T.  T = A P with T_KJ summed over   */
/* L ascending, then A_c = R T summed over K ascending; b x b products as      */
/* ((x0 y0 + x1 y1) + x2 y2).  Structural pattern, no dropping.               */
/* ========================================================================= */
static void blk_mul_acc(const double *X, const double *Y, double *acc, int b) {
  for (int d = 0; d < b; d++)
    for (int e = 0; e < b; e++) {
      double s = X[d * b] * Y[e];
      for (int k = 1; k < b; k++) s += X[d * b + k] * Y[k * b + e];
      acc[d * b + e] += s;
    }
}

static int spgemm(const obsr *X, const obsr *Y, obsr *Z) {
  int b = X->b;
  int32_t n = X->n, m = Y->nc;
  int32_t *mk = malloc((size_t)(m ? m : 1) * sizeof(int32_t));
  int32_t *lst = malloc((size_t)(m ? m : 1) * sizeof(int32_t));
  double *acc = malloc((size_t)(m ? m : 1) * b * b * sizeof(double));
  Z->n = n; Z->nc = m; Z->b = b;
  Z->rp = calloc((size_t)n + 1, sizeof(int64_t));
  if (!mk || !lst || !acc || !Z->rp) return O_ENOMEM;
  for (int32_t j = 0; j < m; j++) mk[j] = -1;
  for (int32_t i = 0; i < n; i++) {   /* symbolic */
    int64_t c = 0;
    for (int64_t k = X->rp[i]; k < X->rp[i + 1]; k++) {
      int32_t l = X->ci[k];
      for (int64_t q = Y->rp[l]; q < Y->rp[l + 1]; q++)
        if (mk[Y->ci[q]] != i) { mk[Y->ci[q]] = i; c++; }
    }
    Z->rp[i + 1] = Z->rp[i] + c;
  }
  Z->nnzb = Z->rp[n];
  Z->ci = malloc((size_t)(Z->nnzb ? Z->nnzb : 1) * sizeof(int32_t));
  Z->v = malloc((size_t)(Z->nnzb ? Z->nnzb : 1) * b * b * sizeof(double));
  if (!Z->ci || !Z->v) return O_ENOMEM;
  for (int32_t j = 0; j < m; j++) mk[j] = -1;
  for (int32_t i = 0; i < n; i++) {   /* numeric */
    int nl = 0;
    for (int64_t k = X->rp[i]; k < X->rp[i + 1]; k++) {
      int32_t l = X->ci[k];
      const double *Xb = X->v + k * b * b;
      for (int64_t q = Y->rp[l]; q < Y->rp[l + 1]; q++) {
        int32_t j = Y->ci[q];
        if (mk[j] != i) { mk[j] = i; lst[nl++] = j; memset(acc + (int64_t)j * b * b, 0, b * b * sizeof(double)); }
        blk_mul_acc(Xb, Y->v + q * b * b, acc + (int64_t)j * b * b, b);
      }
    }
    qsort(lst, nl, sizeof(int32_t), cmp_i32);
    for (int a = 0; a < nl; a++) {
      Z->ci[Z->rp[i] + a] = lst[a];
      memcpy(Z->v + (Z->rp[i] + a) * b * b, acc + (int64_t)lst[a] * b * b, b * b * sizeof(double));
    }
  }
  free(mk); free(lst); free(acc);
  return O_OK;
}

static int rap(const olevel *L, obsr *Ac) {
  obsr T = {0};
  int rc = spgemm(&L->A, &L->P, &T);
  if (rc) return rc;
  rc = spgemm(&L->R, &T, Ac);
  bsr_free(&T);
  return rc;
}

/* ========================================================================= */
/* hierarchy (Algorithm "Recursive AMG Setup")                                */
/* ========================================================================= */
static int copy_bsr_in(obsr *M, int32_t n, int b, const int64_t *rp, const int32_t *ci, const double *v) {
  M->n = n; M->nc = n; M->b = b; M->nnzb = rp[n];
  M->rp = malloc(((size_t)n + 1) * sizeof(int64_t));
  M->ci = malloc((size_t)(M->nnzb ? M->nnzb : 1) * sizeof(int32_t));
  M->v = malloc((size_t)(M->nnzb ? M->nnzb : 1) * b * b * sizeof(double));
  if (!M->rp || !M->ci || !M->v) return O_ENOMEM;
  memcpy(M->rp, rp, ((size_t)n + 1) * sizeof(int64_t));
  memcpy(M->ci, ci, (size_t)M->nnzb * sizeof(int32_t));
  memcpy(M->v, v, (size_t)M->nnzb * b * b * sizeof(double));
  return O_OK;
}

static void free_level(olevel *L) {
  bsr_free(&L->A); bsr_free(&L->G); bsr_free(&L->P); bsr_free(&L->R);
  free(L->cf); free(L->cidx); free(L->V); free(L->srp); free(L->sci); free(L->soc);
  free(L->pcount); free(L->pcols);
  for (int i = 0; i < 6; i++) free(L->work[i]);
  memset(L, 0, sizeof *L);
}

void oracle_free(ohier *h) {
  if (!h) return;
  for (int l = 0; l < h->nlev; l++) free_level(&h->lev[l]);
  free(h->Ld);
  free(h);
}

static int dense_factor(ohier *h, const obsr *A) {
  int b = A->b;
  int nd = A->n * b;
  if (nd > h->p.dense_max_dof) { seterr("coarsest level too large for a dense factorisation"); return O_EINVAL; }
  double *M = calloc((size_t)nd * nd, sizeof(double));
  h->Ld = calloc((size_t)nd * nd, sizeof(double));
  if (!M || !h->Ld) return O_ENOMEM;
  for (int32_t i = 0; i < A->n; i++)
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; k++)
      for (int d = 0; d < b; d++)
        for (int e = 0; e < b; e++)
          M[(int64_t)(i * b + d) * nd + A->ci[k] * b + e] = A->v[k * b * b + d * b + e];
  int rc = chol_small(M, h->Ld, nd);
  free(M);
  h->nd = nd;
  if (rc) { seterr("coarsest matrix not SPD"); return O_ENOTSPD; }
  return O_OK;
}

int oracle_setup(const oparams *p, int32_t n, const int64_t *rp, const int32_t *ci, const double *v,
                 int32_t ntv, const double *V0, ohier **out) {
  *out = NULL;
  if (p->b < 1 || p->b > OMAXB || n <= 0 || ntv < 0 || ntv > 64) { seterr("bad arguments"); return O_EINVAL; }
  ohier *h = calloc(1, sizeof(ohier));
  if (!h) return O_ENOMEM;
  h->p = *p; h->ntv = ntv; h->min_margin = INFINITY;
  QB = p->quant_bits;
  int b = p->b, rc;
  if ((rc = copy_bsr_in(&h->lev[0].A, n, b, rp, ci, v))) goto fail;
  h->lev[0].V = malloc((size_t)n * b * (ntv ? ntv : 1) * sizeof(double));
  if (!h->lev[0].V) { rc = O_ENOMEM; goto fail; }
  memcpy(h->lev[0].V, V0, (size_t)n * b * ntv * sizeof(double));
  for (int l = 0;; l++) {
    olevel *L = &h->lev[l];
    h->nlev = l + 1;
    int32_t N = L->A.n;
    if ((int64_t)N * b <= p->coarse_max_dof || l == p->max_levels - 1 || l == OMAXLEV - 1 || ntv == 0) break;
    if ((rc = fsai_build(h, L))) goto fail;
    if (p->n_rq > 0 && (rc = srqcg(&L->A, &L->G, L->V, ntv, p->n_rq, p->k_ritz, NULL))) goto fail;
    if ((rc = orthonormalize(L->V, (int64_t)N * b, ntv))) goto fail;
    if ((rc = coarsen(h, L))) goto fail;
    int32_t nF = 0;
    for (int32_t i = 0; i < N; i++) nF += L->cf[i] == 0;
    if (L->ncoarse == 0 || nF == 0 || (double)L->ncoarse > p->stall_ratio * (double)N) {
      /* coarsening stalled: this level becomes the coarsest */
      bsr_free(&L->G);
      break;
    }
    if ((rc = build_P(h, L))) goto fail;
    olevel *Ln = &h->lev[l + 1];
    if ((rc = rap(L, &Ln->A))) goto fail;
    Ln->V = malloc((size_t)L->ncoarse * b * ntv * sizeof(double));
    if (!Ln->V) { rc = O_ENOMEM; goto fail; }
    for (int32_t i = 0; i < N; i++)
      if (L->cidx[i] >= 0)
        memcpy(Ln->V + (int64_t)L->cidx[i] * b * ntv, L->V + (int64_t)i * b * ntv, (size_t)b * ntv * sizeof(double));
  }
  if ((rc = dense_factor(h, &h->lev[h->nlev - 1].A))) goto fail;
  for (int l = 0; l < h->nlev; l++) {
    int64_t nn = (int64_t)h->lev[l].A.n * b;
    for (int i = 0; i < 6; i++) {
      h->lev[l].work[i] = calloc((size_t)nn, sizeof(double));
      if (!h->lev[l].work[i]) { rc = O_ENOMEM; goto fail; }
    }
  }
  *out = h;
  return O_OK;
fail:
  oracle_free(h);
  return rc;
}

/* ========================================================================= */
/* V(nu1,nu2)-cycle (Algorithm "AMG application in a V-cycle"); the smoother  */
/* M^{-1} = omega_s G^T G is symmetric, so the post-smoother M^{-T} equals it */
/* ========================================================================= */
static void dense_solve(const ohier *h, const double *y, double *z) {
  int nd = h->nd;
  const double *L = h->Ld;
  for (int i = 0; i < nd; i++) {          /* L w = y */
    double acc = 0.0;
    for (int k = 0; k < i; k++) acc += L[(int64_t)i * nd + k] * z[k];
    z[i] = (y[i] - acc) / L[(int64_t)i * nd + i];
  }
  for (int i = nd - 1; i >= 0; i--) {     /* L^T z = w */
    double acc = 0.0;
    for (int k = i + 1; k < nd; k++) acc += L[(int64_t)k * nd + i] * z[k];
    z[i] = (z[i] - acc) / L[(int64_t)i * nd + i];
  }
}

/* s <- s + omega G^T G (y - A s); from_zero skips A when s = 0 */
static void smooth(const olevel *L, const double *y, double *s, int from_zero, double *r, double *t, double *u) {
  int64_t n = (int64_t)L->A.n * L->A.b;
  if (from_zero) memcpy(r, y, n * sizeof(double));
  else {
    bsr_mv(&L->A, s, r);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) r[i] = y[i] - r[i];
  }
  bsr_mv(&L->G, r, t);
  /* u = G^T t */
  memset(u, 0, n * sizeof(double));
  int b = L->G.b;
  for (int32_t i = 0; i < L->G.n; i++)
    for (int64_t k = L->G.rp[i]; k < L->G.rp[i + 1]; k++) {
      const double *B = L->G.v + k * b * b;
      int32_t j = L->G.ci[k];
      for (int d = 0; d < b; d++)
        for (int e = 0; e < b; e++) u[(int64_t)j * b + e] += B[d * b + e] * t[(int64_t)i * b + d];
    }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) s[i] = from_zero ? L->omega_s * u[i] : s[i] + L->omega_s * u[i];
}

static void vcycle(const ohier *h, int l, const double *y, double *z) {
  const olevel *L = &h->lev[l];
  if (l == h->nlev - 1) { dense_solve(h, y, z); return; }
  int64_t n = (int64_t)L->A.n * L->A.b;
  double *s = z, *r = L->work[0], *t = L->work[1], *u = L->work[2];
  const olevel *Ln = &h->lev[l + 1];
  double *rc = Ln->work[3], *hc = Ln->work[4];
  for (int it = 0; it < h->p.nu1; it++) smooth(L, y, s, it == 0, r, t, u);
  bsr_mv(&L->A, s, r);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) r[i] = y[i] - r[i];
  bsr_mv(&L->R, r, rc);
  vcycle(h, l + 1, rc, hc);
  bsr_mv(&L->P, hc, t);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) s[i] += t[i];
  for (int it = 0; it < h->p.nu2; it++) smooth(L, y, s, 0, r, t, u);
}

void oracle_vcycle(const ohier *h, const double *y, double *z) { vcycle(h, 0, y, z); }

/* ========================================================================= */
/* PCG (Section 4): x0 = 0, stop when ||r_k|| <= rtol ||f||, max_it cap;      */
/* beta = (r_{k+1}.z_{k+1} - r_{k+1}.z_k) / (r_k.z_k) (Polak-Ribiere form)     */
/* ========================================================================= */
int oracle_pcg(const ohier *h, const double *f, double *u, double rtol, int max_it,
               int32_t *iters, double *relres) {
  const obsr *K = &h->lev[0].A;
  int64_t n = (int64_t)K->n * K->b;
  double *r = malloc(n * sizeof(double)), *p = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double));
  double *z = malloc(n * sizeof(double)), *zo = malloc(n * sizeof(double));
  if (!r || !p || !q || !z || !zo) return O_ENOMEM;
  int rc = O_NOTCONV;
  double fn = sqrt(dot(f, f, n));
  memset(u, 0, n * sizeof(double));
  memcpy(r, f, n * sizeof(double));
  *iters = 0; *relres = 0.0;
  if (fn == 0.0) { rc = O_OK; goto done; }
  if (!isfinite(fn)) { rc = O_ENAN; goto done; }
  vcycle(h, 0, r, z);
  memcpy(p, z, n * sizeof(double));
  double rz = dot(r, z, n);
  if (!(rz > 0.0)) { rc = O_EBREAK; goto done; }
  for (int k = 1; k <= max_it; k++) {
    bsr_mv(K, p, q);
    double pq = dot(p, q, n);
    if (!(pq > 0.0)) { rc = isfinite(pq) ? O_EBREAK : O_ENAN; *iters = k; break; }
    double alpha = rz / pq;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) { u[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
    double rr = dot(r, r, n);
    *iters = k;
    *relres = sqrt(rr) / fn;
    if (!isfinite(rr)) { rc = O_ENAN; break; }
    if (sqrt(rr) <= rtol * fn) { rc = O_OK; break; }
    memcpy(zo, z, n * sizeof(double));
    vcycle(h, 0, r, z);
    double rzn = dot(r, z, n), rzo = dot(r, zo, n);
    if (!(rzn > 0.0)) { rc = isfinite(rzn) ? O_EBREAK : O_ENAN; break; }
    double beta = (rzn - rzo) / rz;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
    rz = rzn;
  }
done:
  free(r); free(p); free(q); free(z); free(zo);
  return rc;
}

/* ========================================================================= */
/* element gradient of a quadratic form: grad_e = -lam_e^T K_e u_e, with      */
/* K_e = E_e K_e^0 the derivative dK/dE_e = K_e^0 (24 x 24, node-major dofs)  */
/* ========================================================================= */
void oracle_element_gradient(int64_t n_el, const int32_t *conn, const double *Ke0, int64_t ke_stride,
                             const double *lam, const double *u, double *grad) {
  for (int64_t e = 0; e < n_el; e++) {
    const double *Ke = Ke0 + e * ke_stride;
    double le[24], ue[24];
    for (int a = 0; a < 8; a++)
      for (int c = 0; c < 3; c++) {
        le[a * 3 + c] = lam[(int64_t)conn[e * 8 + a] * 3 + c];
        ue[a * 3 + c] = u[(int64_t)conn[e * 8 + a] * 3 + c];
      }
    double s = 0.0;
    for (int i = 0; i < 24; i++) {
      double ku = 0.0;
      for (int j = 0; j < 24; j++) ku += Ke[i * 24 + j] * ue[j];
      s += le[i] * ku;
    }
    grad[e] = -s;
  }
}

/* ========================================================================= */
/* inspection exports for the tests                                           */
/* ========================================================================= */
/* threads of the OpenMP timing build (1 in the default build) */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int oracle_num_levels(const ohier *h) { return h->nlev; }
double oracle_min_margin(const ohier *h) { return h->min_margin; }
int oracle_coarse_order(const ohier *h) { return h->nd; }

/* info[0..9] = n, nnzb(A), nnzb(G), nnzb(P), ncoarse, fsai_rounds, has_G, has_P */
void oracle_level_info(const ohier *h, int l, int64_t *info, double *dinfo) {
  const olevel *L = &h->lev[l];
  info[0] = L->A.n; info[1] = L->A.nnzb; info[2] = L->G.nnzb; info[3] = L->P.nnzb;
  info[4] = L->ncoarse; info[5] = L->fsai_rounds; info[6] = L->G.rp != NULL; info[7] = L->P.rp != NULL;
  info[8] = L->srp ? L->srp[L->A.n] : 0;
  dinfo[0] = L->lambda1; dinfo[1] = L->omega_q; dinfo[2] = L->omega_s;
}

static void export_bsr(const obsr *M, int64_t *rp, int32_t *ci, double *v) {
  if (!M->rp) return;   /* not formed on this level (G, P of the coarsest) */
  if (rp) memcpy(rp, M->rp, ((size_t)M->n + 1) * sizeof(int64_t));
  if (ci) memcpy(ci, M->ci, (size_t)M->nnzb * sizeof(int32_t));
  if (v) memcpy(v, M->v, (size_t)M->nnzb * M->b * M->b * sizeof(double));
}
void oracle_level_A(const ohier *h, int l, int64_t *rp, int32_t *ci, double *v) { export_bsr(&h->lev[l].A, rp, ci, v); }
void oracle_level_G(const ohier *h, int l, int64_t *rp, int32_t *ci, double *v) { export_bsr(&h->lev[l].G, rp, ci, v); }
void oracle_level_P(const ohier *h, int l, int64_t *rp, int32_t *ci, double *v) { export_bsr(&h->lev[l].P, rp, ci, v); }
void oracle_level_cf(const ohier *h, int l, int8_t *cf) { memcpy(cf, h->lev[l].cf, (size_t)h->lev[l].A.n); }
void oracle_level_V(const ohier *h, int l, double *V) {
  memcpy(V, h->lev[l].V, (size_t)h->lev[l].A.n * h->lev[l].A.b * h->ntv * sizeof(double));
}
void oracle_level_S(const ohier *h, int l, int64_t *srp, int32_t *sci) {
  const olevel *L = &h->lev[l];
  memcpy(srp, L->srp, ((size_t)L->A.n + 1) * sizeof(int64_t));
  memcpy(sci, L->sci, (size_t)L->srp[L->A.n] * sizeof(int32_t));
}
void oracle_level_soc(const ohier *h, int l, double *soc) { memcpy(soc, h->lev[l].soc, (size_t)h->lev[l].A.nnzb * sizeof(double)); }
/* scalar P pattern: counts (n*b) and columns (n*b*n_max, -1 padded) */
void oracle_level_Pscalar(const ohier *h, int l, int32_t *cnt, int32_t *cols) {
  const olevel *L = &h->lev[l];
  memcpy(cnt, L->pcount, (size_t)L->A.n * L->A.b * sizeof(int32_t));
  memcpy(cols, L->pcols, (size_t)L->A.n * L->A.b * h->p.n_max * sizeof(int32_t));
}
/* interpolation candidates (C nodes within S-distance d_p) of every F node of
 * level l, CSR by node (C and decoupled nodes: empty); returns the total count
 * and fills ci only when it is not NULL */
int64_t oracle_level_candidates(const ohier *h, int l, int64_t *rp, int32_t *ci) {
  const olevel *L = &h->lev[l];
  int32_t n = L->A.n;
  int32_t *mark = malloc((size_t)n * sizeof(int32_t)), *frontier = malloc((size_t)n * sizeof(int32_t));
  int32_t *dist = malloc((size_t)n * sizeof(int32_t)), *cn = malloc((size_t)n * sizeof(int32_t));
  for (int32_t i = 0; i < n; i++) { mark[i] = -1; dist[i] = -1; }
  int64_t tot = 0;
  rp[0] = 0;
  for (int32_t I = 0; I < n; I++) {
    int ncn = L->cf && L->cf[I] == 0 ? candidate_nodes(L, I, h->p.d_p, mark, frontier, dist, cn) : 0;
    if (ci) memcpy(ci + tot, cn, (size_t)ncn * sizeof(int32_t));
    tot += ncn;
    rp[I + 1] = tot;
  }
  free(mark); free(frontier); free(dist); free(cn);
  return tot;
}
void oracle_coarse_factor(const ohier *h, double *Ld) { memcpy(Ld, h->Ld, (size_t)h->nd * h->nd * sizeof(double)); }

/* ---- unit exports used by the pins ---- */

/* FSAI rows for a fixed pattern: brp/bci give B per block row (nodes < I,
 * ascending); returns G in BSR form (grp sized n+1, gci/gv sized by grp) and
 * psi per scalar row */
int oracle_fsai_fixed(int32_t n, int b, const int64_t *rp, const int32_t *ci, const double *v,
                      const int64_t *brp, const int32_t *bci, int64_t *grp, int32_t *gci, double *gv,
                      double *psi) {
  obsr A = {0}, G = {0};
  int rc = copy_bsr_in(&A, n, b, rp, ci, v);
  if (rc) return rc;
  int mmax = OMAXNB * b + b;
  double *Mb = malloc((size_t)mmax * mmax * sizeof(double)), *Lb = malloc((size_t)mmax * mmax * sizeof(double));
  fpatt F;
  F.pat = malloc((size_t)n * OMAXNB * sizeof(int32_t));
  F.pnb = calloc((size_t)n, sizeof(int32_t));
  if (!Mb || !Lb || !F.pat || !F.pnb) return O_ENOMEM;
  frow R;
  for (int32_t i = 0; i < n && rc == O_OK; i++) {
    R.nb = (int)(brp[i + 1] - brp[i]);
    if (R.nb > OMAXNB) { rc = O_EINVAL; break; }
    memcpy(R.nodes, bci + brp[i], R.nb * sizeof(int32_t));
    if (fsai_factor_row(&A, i, &R, Mb, Lb)) { rc = O_ENOTSPD; break; }
    for (int d = 0; d < b; d++) psi[(int64_t)i * b + d] = R.psi[d];
    store_row(&F, i, &R);
  }
  if (rc == O_OK) rc = fsai_assemble(&A, &F, &G, Mb, Lb);
  if (rc == O_OK) export_bsr(&G, grp, gci, gv);
  bsr_free(&A); bsr_free(&G); free(Mb); free(Lb); free(F.pat); free(F.pnb);
  return rc;
}

/* first-pass adaptive FSAI (no outer loop) for selected block rows of A:
 * pattern (nodes, -1 padded to OMAXNB per row), scaled rows g and psi */
int oracle_fsai_rows(const oparams *p, int32_t n, const int64_t *rp, const int32_t *ci, const double *v,
                     int32_t nrows, const int32_t *rows_sel, int32_t *nodes_out, int32_t *nb_out,
                     double *g_out /* nrows * b * (OMAXNB*b+b) */, double *psi_out) {
  obsr A = {0};
  int b = p->b;
  int rc = copy_bsr_in(&A, n, b, rp, ci, v);
  if (rc) return rc;
  ohier *hh = calloc(1, sizeof(ohier));
  hh->p = *p; hh->min_margin = INFINITY; QB = p->quant_bits;
  int mmax = OMAXNB * b + b;
  double *Mb = malloc((size_t)mmax * mmax * sizeof(double)), *Lb = malloc((size_t)mmax * mmax * sizeof(double));
  int32_t *mark = malloc((size_t)n * sizeof(int32_t)), *cand = malloc((size_t)n * sizeof(int32_t));
  qcand *qc = malloc((size_t)n * sizeof(qcand));
  for (int32_t i = 0; i < n; i++) mark[i] = -1;
  frow R;
  for (int32_t r = 0; r < nrows && rc == O_OK; r++) {
    int32_t I = rows_sel[r];
    rc = fsai_first_pass_row(hh, &A, I, &R, mark, cand, qc, Mb, Lb);
    if (rc) break;
    nb_out[r] = R.nb;
    for (int q = 0; q < OMAXNB; q++) nodes_out[(int64_t)r * OMAXNB + q] = q < R.nb ? R.nodes[q] : -1;
    for (int d = 0; d < b; d++) {
      psi_out[(int64_t)r * b + d] = R.psi[d];
      for (int q = 0; q < mmax; q++) g_out[((int64_t)r * b + d) * mmax + q] = q < b * R.nb + d + 1 ? R.g[d][q] : 0.0;
    }
  }
  bsr_free(&A); free(Mb); free(Lb); free(mark); free(cand); free(qc); free(hh);
  return rc;
}

int oracle_max_nb(void) { return OMAXNB; }

/* SRQCG on a standalone matrix A (BSR, n block rows of size b) and factor G;
 * V is row-major [n*b][nt], V0 in and G^T Z out; rq receives the final
 * Rayleigh quotients of the columns of Z */
int oracle_srqcg(int32_t n, int b, const int64_t *rp, const int32_t *ci, const double *v, const int64_t *grp,
                 const int32_t *gci, const double *gv, int nt, double *V, int kmax, int kritz, double *rq) {
  obsr A = {0}, G = {0};
  int rc = copy_bsr_in(&A, n, b, rp, ci, v);
  if (rc) return rc;
  G.n = n; G.nc = n; G.b = b; G.nnzb = grp[n];
  G.rp = (int64_t *)grp; G.ci = (int32_t *)gci; G.v = (double *)gv;
  rc = srqcg(&A, &G, V, nt, kmax, kritz, rq);
  bsr_free(&A);
  return rc;
}

double oracle_lanczos(int32_t n, int b, const int64_t *rp, const int32_t *ci, const double *v,
                      const int64_t *grp, const int32_t *gci, const double *gv, int steps) {
  obsr A = {0}, G = {0}, GT = {0};
  copy_bsr_in(&A, n, b, rp, ci, v);
  G.n = n; G.nc = n; G.b = b; G.nnzb = grp[n];
  G.rp = (int64_t *)grp; G.ci = (int32_t *)gci; G.v = (double *)gv;
  bsr_transpose(&G, &GT);
  double lam = oracle_lanczos_gagt(&A, &G, &GT, steps);
  bsr_free(&A); bsr_free(&GT);
  return lam;
}

/* one DPLS row: target v (ntv), candidate rows C (nca x ntv);
 * outputs chosen candidate indices and weights (up to n_max) */
int oracle_dpls_row(const oparams *p, const double *v, const double *C, int nca, int ntv,
                    int32_t *chosen, double *w) {
  ohier hh; memset(&hh, 0, sizeof hh); hh.p = *p; hh.min_margin = INFINITY; QB = p->quant_bits;
  double *t = NULL, *gaa = NULL;
  double *gbuf = malloc((size_t)(nca ? nca : 1) * ntv * sizeof(double));
  dpls_out o;
  int rc = dpls_row(&hh, v, C, nca, ntv, &o, gbuf, t, gaa);
  free(t); free(gaa); free(gbuf);
  if (rc) return rc;
  for (int k = 0; k < o.k; k++) { chosen[k] = o.col[k]; w[k] = o.w[k]; }
  return o.k;
}

/* A_c = P^T A P through the oracle's RAP */
int oracle_rap(int32_t n, int32_t nc, int b, const int64_t *rp, const int32_t *ci, const double *v,
               const int64_t *prp, const int32_t *pci, const double *pv,
               int64_t *nnz_out, int64_t *crp, int32_t *cci, double *cv, int64_t cap) {
  olevel L; memset(&L, 0, sizeof L);
  int rc = copy_bsr_in(&L.A, n, b, rp, ci, v);
  if (rc) return rc;
  L.P.n = n; L.P.nc = nc; L.P.b = b; L.P.nnzb = prp[n];
  L.P.rp = malloc(((size_t)n + 1) * sizeof(int64_t)); memcpy(L.P.rp, prp, ((size_t)n + 1) * sizeof(int64_t));
  L.P.ci = malloc((size_t)(L.P.nnzb ? L.P.nnzb : 1) * sizeof(int32_t)); memcpy(L.P.ci, pci, (size_t)L.P.nnzb * sizeof(int32_t));
  L.P.v = malloc((size_t)(L.P.nnzb ? L.P.nnzb : 1) * b * b * sizeof(double)); memcpy(L.P.v, pv, (size_t)L.P.nnzb * b * b * sizeof(double));
  bsr_transpose(&L.P, &L.R);
  obsr Ac = {0};
  rc = rap(&L, &Ac);
  if (rc == O_OK) {
    *nnz_out = Ac.nnzb;
    if (Ac.nnzb <= cap) export_bsr(&Ac, crp, cci, cv);
  }
  bsr_free(&Ac); bsr_free(&L.A); bsr_free(&L.P); bsr_free(&L.R);
  return rc;
}

/* SoC of one node pair (canonical order: the smaller node first) */
double oracle_soc_node(const double *V, int b, int ntv, int32_t I, int32_t J) {
  int32_t a = I < J ? I : J, c = I < J ? J : I;
  double den = sqrt(node_n(V, b, ntv, a, a)) * sqrt(node_n(V, b, ntv, c, c));
  if (!(den > 0.0)) return 0.0;
  return node_n(V, b, ntv, a, c) / den;
}

void oracle_orthonormalize(double *V, int64_t nrows, int ntv) { orthonormalize(V, nrows, ntv); }
double oracle_quantize(double s, int bits) { int old = QB; QB = bits; double r = qz(s); QB = old; return r; }
uint64_t oracle_splitmix64(uint64_t x) { return splitmix64(x); }
