// Coarsening and interpolation-pattern decisions on the device (Sections 3.4
// and 3.5): the affinity strength of connection between neighbouring nodes,
// the theta filter and its union symmetrisation into the strong graph S, the
// maximal independent set (C/F split) as a fixed point of local-maximum rounds,
// and the greedy least-squares selection of the interpolation entries of every
// fine scalar row.  Nodes carry b unknowns (3, or 1 for scalar operators).
//
// Compiled with -ffp-contract=off: every decision quantity is the sequential
// IEEE binary64 sum written here (the host's definition, in the same order),
// rounded by the same quantiser before it is compared, so the decisions are
// bitwise those of the sequential rules.
#include "device_decisions.h"
#include "internal.h"

namespace aspamg {

namespace {

// n_IJ = sum over (d, e) in row-major order of (V_I,d . V_J,e)^2, each inner
// product summed over the test vectors in ascending order
__device__ __forceinline__ double node_affinity(const double *__restrict__ V, int ntv, int32_t I, int32_t J, int b) {
  double s = 0.0;
  for (int d = 0; d < b; d++)
    for (int e = 0; e < b; e++) {
      const double *vi = V + ((size_t)I * b + d) * ntv;
      const double *vj = V + ((size_t)J * b + e) * ntv;
      double m = 0.0;
      for (int t = 0; t < ntv; t++) m += vi[t] * vj[t];
      s += m * m;
    }
  return s;
}

__global__ void __launch_bounds__(256) k_node_norms(int32_t n, const double *__restrict__ V, int ntv, int b,
                                                    double *__restrict__ sq) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) sq[i] = sqrt(node_affinity(V, ntv, i, i, b));
}

// (q1, j1) ranks before (q2, j2): larger quantised strength, then lower node
__device__ __forceinline__ bool soc_before(double q1, int32_t j1, double q2, int32_t j2) {
  return q1 > q2 || (q1 == q2 && j1 < j2);
}

// theta filter: the min(theta, deg) strongest connections of every node.
// SoC[I,J] = n_IJ / (sqrt(n_II) sqrt(n_JJ)), evaluated with the smaller node
// first (so both directions are the same double), over the off-diagonal
// blocks of A between nodes that are not decoupled.
__global__ void __launch_bounds__(256) k_strong_topk(int32_t n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const int8_t *__restrict__ excl, const double *__restrict__ V,
                                                     int ntv, int b, const double *__restrict__ sq, int theta,
                                                     int qbits, int32_t *__restrict__ keep,
                                                     int32_t *__restrict__ nkeep) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double bq[kMaxTheta];
  int32_t bj[kMaxTheta];
  int nb = 0;
  if (!excl[i])
    for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
      const int32_t j = ci[k];
      if (j == i || excl[j]) continue;
      const int32_t a = min(i, j), c = max(i, j);
      const double den = sq[a] * sq[c];
      const double s = den > 0.0 ? node_affinity(V, ntv, a, c, b) / den : 0.0;
      if (!(s > 0.0)) continue;
      const double qs = quantize_dev(s, qbits);
      int at = nb;
      while (at > 0 && soc_before(qs, j, bq[at - 1], bj[at - 1])) at--;
      if (at >= theta) continue;
      for (int m = min(nb, theta - 1); m > at; m--) {
        bq[m] = bq[m - 1];
        bj[m] = bj[m - 1];
      }
      bq[at] = qs;
      bj[at] = j;
      if (nb < theta) nb++;
    }
  for (int a = 0; a < nb; a++) keep[(size_t)i * theta + a] = bj[a];
  nkeep[i] = nb;
}

// union symmetrisation: every kept edge in both rows
__global__ void __launch_bounds__(256) k_union_count(int32_t n, int theta, const int32_t *__restrict__ keep,
                                                     const int32_t *__restrict__ nkeep, int32_t *__restrict__ cnt) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int a = 0; a < nkeep[i]; a++) {
    atomicAdd(&cnt[i], 1);
    atomicAdd(&cnt[keep[(size_t)i * theta + a]], 1);
  }
}

__global__ void __launch_bounds__(256) k_union_fill(int32_t n, int theta, const int32_t *__restrict__ keep,
                                                    const int32_t *__restrict__ nkeep, int64_t *__restrict__ at,
                                                    int32_t *__restrict__ both) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int a = 0; a < nkeep[i]; a++) {
    const int32_t j = keep[(size_t)i * theta + a];
    both[atomicAdd((unsigned long long *)&at[i], 1ULL)] = j;
    both[atomicAdd((unsigned long long *)&at[j], 1ULL)] = i;
  }
}

// each row ascending without repeats (the fill order above is arbitrary; the
// sorted set is not)
__global__ void __launch_bounds__(256) k_union_sort(int32_t n, const int64_t *__restrict__ bp,
                                                    int32_t *__restrict__ both, int32_t *__restrict__ len) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int32_t *r = both + bp[i];
  const int m = (int)(bp[i + 1] - bp[i]);
  for (int a = 1; a < m; a++) {
    const int32_t v = r[a];
    int b = a;
    while (b > 0 && r[b - 1] > v) {
      r[b] = r[b - 1];
      b--;
    }
    r[b] = v;
  }
  int u = 0;
  for (int a = 0; a < m; a++)
    if (u == 0 || r[a] != r[u - 1]) r[u++] = r[a];
  len[i] = u;
}

__global__ void __launch_bounds__(256) k_union_compact(int32_t n, const int64_t *__restrict__ bp,
                                                       const int32_t *__restrict__ both,
                                                       const int64_t *__restrict__ srp, int32_t *__restrict__ sci) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t m = srp[i + 1] - srp[i];
  for (int64_t a = 0; a < m; a++) sci[srp[i] + a] = both[bp[i] + a];
}

// Maximal independent set in descending (|S_I|, hash(I), -I): a node joins C
// when no undecided S-neighbour ranks above it; the undecided neighbours of C
// nodes become F; rounds repeat until every node is decided.  Under one total
// order this fixed point is the set the sequential greedy in that order picks.
__device__ __forceinline__ bool mis_greater(const int64_t *srp, int32_t a, int32_t b) {
  const int64_t da = srp[a + 1] - srp[a], db = srp[b + 1] - srp[b];
  if (da != db) return da > db;
  const uint64_t ha = mix64_dev((uint64_t)a), hb = mix64_dev((uint64_t)b);
  if (ha != hb) return ha > hb;
  return a < b;
}

__global__ void __launch_bounds__(256) k_mis_init(int32_t n, const int8_t *__restrict__ excl,
                                                  int8_t *__restrict__ cf) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) cf[i] = excl[i] ? -1 : 2;
}

__global__ void __launch_bounds__(256) k_mis_pick(int32_t n, const int64_t *__restrict__ srp,
                                                  const int32_t *__restrict__ sci, const int8_t *__restrict__ cf,
                                                  int8_t *__restrict__ win) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  bool best = cf[i] == 2;
  if (best)
    for (int64_t k = srp[i]; k < srp[i + 1]; k++) {
      const int32_t j = sci[k];
      if (cf[j] == 2 && mis_greater(srp, j, i)) {
        best = false;
        break;
      }
    }
  win[i] = best;
}

__global__ void __launch_bounds__(256) k_mis_set_c(int32_t n, const int8_t *__restrict__ win, int8_t *__restrict__ cf) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n && win[i]) cf[i] = 1;
}

// undecided nodes next to a C node become F; the rest are counted
__global__ void __launch_bounds__(256) k_mis_set_f(int32_t n, const int64_t *__restrict__ srp,
                                                   const int32_t *__restrict__ sci, int8_t *__restrict__ cf,
                                                   int32_t *__restrict__ undecided) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n || cf[i] != 2) return;
  for (int64_t k = srp[i]; k < srp[i + 1]; k++)
    if (cf[sci[k]] == 1) {
      cf[i] = 0;
      return;
    }
  atomicAdd(undecided, 1);
}

// ---------------------------------------------------------------------------
// DPLS interpolation pattern (Section 3.5, Algorithm "Dynamic Pattern Least
// Squares Prolongation", Householder form): one 64-thread workgroup per fine
// node.  Lane 0 collects the C nodes within S-distance d_p (breadth-first,
// paths through any node; a hash set in LDS marks visited nodes) and sorts
// them; the scalar candidates are (J, e) in ascending order.  For each of the
// node's three scalar rows the greedy then runs with the candidates spread
// over the lanes: after k accepted columns the residual r and the candidates
// have been reflected k times, entries k.. of each vector being its part
// orthogonal to the chosen columns.  Candidate a has affinity
// pi^2 / (rho^2 delta^2) (rho^2 = |r_k..|^2, delta^2 = |c_k..|^2, pi = c_k.. .
// r_k..); the largest quantised affinity > 0 wins, ties to the lowest a,
// unless max|R_kk| / min|R_kk| would exceed kappa_p.  The row stops at n_max
// entries, at rho^2 <= eps_p^2 v.v (quantised) or when no candidate is
// eligible.  The reflection of step k: alpha = -delta if u_k >= 0 else +delta,
// h = u_k.. with h_k -= alpha, x_k.. -= (2 h . x_k.. / h . h) h.  Every sum is
// sequential in ascending t on one lane, as in the sequential rule.
// ---------------------------------------------------------------------------
constexpr int kHashSlots = 2048;     // visited set (nodes within distance d_p)
constexpr int kMaxReach = 1024;      // nodes within distance d_p of one node
constexpr int kMaxCoarse = 320;      // C nodes among them
constexpr int kCwMax = 5120;         // candidate values held per row (candidates x n_tv)

__device__ __forceinline__ bool dpls_better(double qa, int32_t a, double qb, int32_t b) {
  return qa > qb || (qa == qb && a < b);
}

__global__ void __launch_bounds__(64) k_dpls_rows(int32_t nf, const int32_t *__restrict__ fnodes,
                                                  const int64_t *__restrict__ srp, const int32_t *__restrict__ sci,
                                                  const int8_t *__restrict__ cf, const double *__restrict__ V, int ntv,
                                                  int b, int d_p, int nmax, double kappa_q, double eps_p, int qbits,
                                                  int32_t *__restrict__ pcount, int32_t *__restrict__ psel,
                                                  int32_t *__restrict__ err) {
  __shared__ int32_t hset[kHashSlots];
  __shared__ int32_t qnode[kMaxReach];
  __shared__ int8_t qdist[kMaxReach];
  __shared__ int32_t cn[kMaxCoarse];
  __shared__ double Cw[kCwMax];
  __shared__ double r[64], hv[64];
  __shared__ int8_t used[3 * kMaxCoarse];
  __shared__ int32_t s_ncn, s_ok, s_best;
  __shared__ double s_rho2, s_bdel2, s_sh;
  __shared__ double s_bq[64];
  __shared__ int32_t s_ba[64];
  const int lane = threadIdx.x;
  const int32_t I = fnodes[blockIdx.x];
  for (int a = lane; a < kHashSlots; a += 64) hset[a] = -1;
  __syncthreads();
  if (lane == 0) {
    int ok = 1, cnt = 0, ncn = 0;
    auto visit = [&](int32_t w) -> bool {       // true if w was not yet visited
      uint32_t hsh = (uint32_t)mix64_dev((uint64_t)w) & (kHashSlots - 1);
      while (true) {
        const int32_t v = hset[hsh];
        if (v == w) return false;
        if (v < 0) {
          hset[hsh] = w;
          return true;
        }
        hsh = (hsh + 1) & (kHashSlots - 1);
      }
    };
    visit(I);
    qnode[cnt] = I;
    qdist[cnt] = 0;
    cnt++;
    for (int head = 0; head < cnt && ok; head++) {
      const int32_t u = qnode[head];
      if (qdist[head] >= d_p) continue;
      for (int64_t k = srp[u]; k < srp[u + 1]; k++) {
        const int32_t w = sci[k];
        if (!visit(w)) continue;
        if (cnt == kMaxReach) {
          ok = 0;
          break;
        }
        qnode[cnt] = w;
        qdist[cnt] = (int8_t)(qdist[head] + 1);
        cnt++;
        if (cf[w] == 1) {
          if (ncn == kMaxCoarse) {
            ok = 0;
            break;
          }
          cn[ncn++] = w;
        }
      }
    }
    for (int a = 1; a < ncn; a++) {             // ascending node order
      const int32_t v = cn[a];
      int b = a;
      while (b > 0 && cn[b - 1] > v) {
        cn[b] = cn[b - 1];
        b--;
      }
      cn[b] = v;
    }
    if (ok && b * ncn * ntv > kCwMax) ok = 0;
    if (!ok) atomicOr(err, 1);
    s_ncn = ncn;
    s_ok = ok;
  }
  __syncthreads();
  if (!s_ok) return;
  const int nca = b * s_ncn;
  for (int d = 0; d < b; d++) {
    const size_t row = (size_t)I * b + d;
    for (int x = lane; x < nca * ntv; x += 64) {
      const int a = x / ntv, t = x % ntv;
      Cw[x] = V[((size_t)cn[a / b] * b + a % b) * ntv + t];
    }
    for (int a = lane; a < nca; a += 64) used[a] = 0;
    if (lane < ntv) r[lane] = V[row * ntv + lane];
    __syncthreads();
    double vv = 0.0;
    for (int t = 0; t < ntv; t++) vv += r[t] * r[t];
    int K = 0;
    int32_t chosen[kMaxPEntries];
    if (vv != 0.0) {
      const double thr = quantize_dev((eps_p * eps_p) * vv, qbits);
      double dmax = 0.0, dmin = 0.0;
      while (K < nmax && K < ntv) {
        if (lane == 0) {
          double rho2 = 0.0;
          for (int t = K; t < ntv; t++) rho2 += r[t] * r[t];
          s_rho2 = rho2;
        }
        __syncthreads();
        const double rho2 = s_rho2;
        if (!(quantize_dev(rho2, qbits) > thr)) break;
        double bq = 0.0, bdel2 = 0.0;
        int32_t ba = -1;
        for (int a = lane; a < nca; a += 64) {
          if (used[a]) continue;
          const double *c = Cw + a * ntv;
          double del2 = 0.0;
          for (int t = K; t < ntv; t++) del2 += c[t] * c[t];
          if (!(del2 > 0.0)) continue;
          double pi = 0.0;
          for (int t = K; t < ntv; t++) pi += c[t] * r[t];
          const double qa = quantize_dev((pi * pi) / (rho2 * del2), qbits);
          if (qa > bq) {
            bq = qa;
            ba = a;
            bdel2 = del2;
          }
        }
        s_bq[lane] = bq;
        s_ba[lane] = ba;
        __syncthreads();
        if (lane == 0) {
          int bl = -1;
          for (int l = 0; l < 64; l++) {
            if (s_ba[l] < 0) continue;
            if (bl < 0 || dpls_better(s_bq[l], s_ba[l], s_bq[bl], s_ba[bl])) bl = l;
          }
          s_best = bl < 0 ? -1 : s_ba[bl];
        }
        __syncthreads();
        const int32_t best = s_best;
        if (best < 0) break;
        if (ba == best) s_bdel2 = bdel2;
        __syncthreads();
        const double del = sqrt(s_bdel2);
        const double mx = K ? fmax(dmax, del) : del;
        const double mn = K ? fmin(dmin, del) : del;
        if (quantize_dev(mx / mn, qbits) > kappa_q) break;
        if (lane == 0) {
          const double *u = Cw + best * ntv;
          const double alpha = u[K] >= 0.0 ? -del : del;
          for (int t = K; t < ntv; t++) hv[t] = u[t];
          hv[K] = u[K] - alpha;
          double sh = hv[K] * hv[K];
          for (int t = K + 1; t < ntv; t++) sh += hv[t] * hv[t];
          s_sh = sh;
        }
        __syncthreads();
        const double sh = s_sh;
        for (int a = lane; a < nca; a += 64) {
          if (used[a] || a == best) continue;
          double *x = Cw + a * ntv;
          double tau = 0.0;
          for (int t = K; t < ntv; t++) tau += hv[t] * x[t];
          const double fct = (2.0 * tau) / sh;
          for (int t = K; t < ntv; t++) x[t] = x[t] - fct * hv[t];
        }
        __syncthreads();
        if (lane == 0) {
          double tau = 0.0;
          for (int t = K; t < ntv; t++) tau += hv[t] * r[t];
          const double fct = (2.0 * tau) / sh;
          for (int t = K; t < ntv; t++) r[t] = r[t] - fct * hv[t];
          used[best] = 1;
        }
        __syncthreads();
        dmax = mx;
        dmin = mn;
        chosen[K] = best;
        K++;
      }
    }
    if (lane == 0) {
      pcount[row] = K;
      for (int k = 0; k < K; k++) psel[row * kMaxPEntries + k] = cn[chosen[k] / b] * b + chosen[k] % b;
    }
    __syncthreads();
  }
}

}  // namespace

void launch_node_norms(int32_t n, const double *V, int ntv, int b, double *sq, hipStream_t s) {
  hipLaunchKernelGGL(k_node_norms, dim3((n + 255) / 256), dim3(256), 0, s, n, V, ntv, b, sq);
}

void launch_strong_topk(const DevBSR &A, const int8_t *excl, const double *V, int ntv, const double *sq, int theta,
                        int qbits, int32_t *keep, int32_t *nkeep, hipStream_t s) {
  hipLaunchKernelGGL(k_strong_topk, dim3((A.n + 255) / 256), dim3(256), 0, s, A.n, A.rp, A.ci, excl, V, ntv, A.b, sq,
                     theta, qbits, keep, nkeep);
}

void launch_union(int32_t n, int theta, const int32_t *keep, const int32_t *nkeep, int stage, int32_t *cnt,
                  int64_t *bp, int64_t *at, int32_t *both, int32_t *len, const int64_t *srp, int32_t *sci,
                  hipStream_t s) {
  const dim3 g((n + 255) / 256), b(256);
  switch (stage) {
    case 0: hipLaunchKernelGGL(k_union_count, g, b, 0, s, n, theta, keep, nkeep, cnt); break;
    case 1:
      hipLaunchKernelGGL(k_union_fill, g, b, 0, s, n, theta, keep, nkeep, at, both);
      hipLaunchKernelGGL(k_union_sort, g, b, 0, s, n, bp, both, len);
      break;
    case 2: hipLaunchKernelGGL(k_union_compact, g, b, 0, s, n, bp, both, srp, sci); break;
  }
}

void launch_mis_init(int32_t n, const int8_t *excl, int8_t *cf, hipStream_t s) {
  hipLaunchKernelGGL(k_mis_init, dim3((n + 255) / 256), dim3(256), 0, s, n, excl, cf);
}

void launch_mis_round(int32_t n, const int64_t *srp, const int32_t *sci, int8_t *cf, int8_t *win, int32_t *undecided,
                      hipStream_t s) {
  const dim3 g((n + 255) / 256), b(256);
  hipLaunchKernelGGL(k_mis_pick, g, b, 0, s, n, srp, sci, cf, win);
  hipLaunchKernelGGL(k_mis_set_c, g, b, 0, s, n, win, cf);
  hipLaunchKernelGGL(k_mis_set_f, g, b, 0, s, n, srp, sci, cf, undecided);
}

void launch_dpls_rows(int32_t nf, const int32_t *fnodes, const int64_t *srp, const int32_t *sci, const int8_t *cf,
                      const double *V, int ntv, int b, int d_p, int nmax, double kappa_q, double eps_p, int qbits,
                      int32_t *pcount, int32_t *psel, int32_t *err, hipStream_t s) {
  if (nf == 0) return;
  hipLaunchKernelGGL(k_dpls_rows, dim3(nf), dim3(64), 0, s, nf, fnodes, srp, sci, cf, V, ntv, b, d_p, nmax, kappa_q,
                     eps_p, qbits, pcount, psel, err);
}

}  // namespace aspamg
