// Host side of the aSP-AMG setup (Algorithm "Recursive AMG Setup"): the
// discrete decisions of every level (FSAI patterns, test-space basis, affinity
// strength, theta filter, coarse/fine split, interpolation patterns, Galerkin
// pattern) run here in a canonical order; the numerical bulk (FSAI row
// factorisations, Lanczos products, least-squares weights, Galerkin values)
// runs in HIP kernels on the handle's stream.
//
// Decision quantities use IEEE binary64 +, -, *, /, sqrt only, each sum in
// ascending index order as written below, and every comparison of scores is
// made on values rounded to `quant_bits` significant bits with ties broken by
// the lowest index.  This file is compiled with -ffp-contract=off.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>

#include "internal.h"

namespace aspamg {

// s rounded to `bits` significant bits (round to nearest, ties to even).  A
// normal double keeps the top bits of its 53-bit significand, rounding the
// dropped ones (a carry may step the exponent); zero, subnormal and
// non-finite values take the frexp / ldexp form of the same rounding.
double quantize(double s, int bits) {
  uint64_t u;
  std::memcpy(&u, &s, 8);
  const uint64_t ex = (u >> 52) & 0x7FF;
  if (ex == 0 || ex == 0x7FF) {
    if (s == 0.0 || !std::isfinite(s)) return s;
    int e;
    const double m = std::frexp(s, &e);
    const double r = std::nearbyint(std::ldexp(m, bits));
    return std::ldexp(r, e - bits);
  }
  const int drop = 53 - bits;
  const uint64_t mask = (1ULL << drop) - 1, half = 1ULL << (drop - 1);
  const uint64_t rem = u & mask;
  u &= ~mask;
  if (rem > half || (rem == half && ((u >> drop) & 1))) u += 1ULL << drop;
  double r;
  std::memcpy(&r, &u, 8);
  return r;
}

namespace {

struct Q {
  int bits;
  double operator()(double s) const { return quantize(s, bits); }
};

// position of block (r, c) in M, or -1
inline int64_t find_block(const HostBSR &M, int32_t r, int32_t c) {
  const int32_t *b = M.ci.data() + M.rp[r];
  const int32_t *e = M.ci.data() + M.rp[r + 1];
  const int32_t *it = std::lower_bound(b, e, c);
  return (it != e && *it == c) ? (int64_t)(it - M.ci.data()) : -1;
}

inline bool is_decoupled(const HostBSR &A, int32_t i) {
  return A.rp[i + 1] - A.rp[i] == 1 && A.ci[A.rp[i]] == i;
}

// ------------------------------------------------------------------------
// device helpers
// ------------------------------------------------------------------------
template <typename T>
T *upload(aspamg_ctx *h, const std::vector<T> &v) {
  T *d = dalloc<T>(h, std::max<size_t>(v.size(), 1));
  if (!v.empty()) HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
  return d;
}

// scratch device buffer freed at scope exit
struct Scratch {
  void *p = nullptr;
  explicit Scratch(size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (hipMalloc(&p, bytes) != hipSuccess) fail(ASPAMG_ENOMEM, "device scratch allocation failed");
  }
  ~Scratch() {
    if (p) (void)hipFree(p);
  }
  template <typename T>
  T *as() const { return static_cast<T *>(p); }
};

// Pinned host buffer of at least `bytes`, kept by the handle across setup
// steps (device-to-host copies into pinned memory run at full link speed).
void *staging(aspamg_ctx *h, size_t bytes) {
  if (bytes > h->staging_bytes) {
    if (h->staging) (void)hipHostFree(h->staging);
    h->staging = nullptr;
    h->staging_bytes = 0;
    if (hipHostMalloc(&h->staging, bytes, hipHostMallocDefault) != hipSuccess)
      fail(ASPAMG_ENOMEM, "pinned staging allocation failed");
    h->staging_bytes = bytes;
  }
  return h->staging;
}

template <typename T>
void to_device(hipStream_t s, T *d, const T *hsrc, size_t n) {
  if (n) HIPCHK(hipMemcpyAsync(d, hsrc, n * sizeof(T), hipMemcpyHostToDevice, s));
}
template <typename T>
void to_host(hipStream_t s, T *hdst, const T *d, size_t n) {
  if (n) HIPCHK(hipMemcpyAsync(hdst, d, n * sizeof(T), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------------
// aFSAI (Section 3.1).  Each block row I keeps a sorted node set B (J < I);
// the GPU factors A[l,l] and returns the three scaled rows g and psi, and
// from the same g the nodes the row's next growth step would add.
// ------------------------------------------------------------------------
struct FsaiState {
  int32_t n;
  int b;                          // unknowns per node
  int rho;                        // nodes per growth step
  std::vector<int32_t> nb;        // |B| per row
  std::vector<int32_t> nodes;     // n * kMaxFsaiNodes
  std::vector<double> g;          // n * b * gstride
  std::vector<double> psi;        // n * b
  std::vector<int32_t> add;       // n * rho: the next growth of the row's current pattern, -1 padded
  static constexpr int gstride = 3 * kMaxFsaiNodes + 3;
};

// Factor the listed rows on the GPU; store g / psi and the next growth in the state.
void fsai_factor(aspamg_ctx *h, const Level &L, FsaiState &F, const std::vector<int32_t> &rows) {
  if (rows.empty()) return;
  const int32_t nr = (int32_t)rows.size();
  const int gs = FsaiState::gstride;
  const int b = F.b;
  // chunk to bound device memory
  const int32_t chunk = 1 << 17;
  for (int32_t c0 = 0; c0 < nr; c0 += chunk) {
    const int32_t c1 = std::min(nr, c0 + chunk), m = c1 - c0;
    std::vector<int32_t> pptr(m + 1, 0), pnodes;
    int maxnb = 0;
    for (int32_t i = 0; i < m; i++) {
      const int32_t I = rows[c0 + i];
      pptr[i + 1] = pptr[i] + F.nb[I];
      maxnb = std::max(maxnb, F.nb[I]);
    }
    pnodes.resize(std::max<int32_t>(pptr[m], 1));
    for (int32_t i = 0; i < m; i++) {
      const int32_t I = rows[c0 + i];
      std::memcpy(pnodes.data() + pptr[i], F.nodes.data() + (size_t)I * kMaxFsaiNodes, F.nb[I] * sizeof(int32_t));
    }
    const size_t gn = (size_t)b * (b * (size_t)pptr[m] + b * (size_t)m);   // compact g entries
    Scratch drows(m * 4), dptr((m + 1) * 4), dnodes(pnodes.size() * 4), dg(gn * 8), dpsi((size_t)m * b * 8),
        dfail(4);
    to_device(h->stream, drows.as<int32_t>(), rows.data() + c0, m);
    to_device(h->stream, dptr.as<int32_t>(), pptr.data(), m + 1);
    to_device(h->stream, dnodes.as<int32_t>(), pnodes.data(), pnodes.size());
    HIPCHK(hipMemsetAsync(dfail.p, 0, 4, h->stream));
    const int mmax = b * maxnb + b;
    launch_fsai_rows(L.dA, m, drows.as<int32_t>(), dptr.as<int32_t>(), dnodes.as<int32_t>(), mmax, dg.as<double>(),
                     dpsi.as<double>(), dfail.as<int32_t>(), h->stream);
    HIPCHK(hipGetLastError());
    Scratch dadd((size_t)m * F.rho * 4);
    launch_fsai_grow(L.dA, m, drows.as<int32_t>(), dptr.as<int32_t>(), dnodes.as<int32_t>(), dg.as<double>(), F.rho,
                     h->p.quant_bits, dadd.as<int32_t>(), h->stream);
    HIPCHK(hipGetLastError());
    double *g = static_cast<double *>(staging(h, gn * 8));
    std::vector<double> psi((size_t)m * b);
    std::vector<int32_t> add((size_t)m * F.rho);
    int32_t bad = 0;
    to_host(h->stream, &bad, dfail.as<int32_t>(), 1);
    if (bad) fail(ASPAMG_ENOT_SPD, "aFSAI: a local system is not positive definite");
    to_host(h->stream, g, dg.as<double>(), gn);
    to_host(h->stream, psi.data(), dpsi.as<double>(), psi.size());
    to_host(h->stream, add.data(), dadd.as<int32_t>(), add.size());
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < m; i++) {
      const int32_t I = rows[c0 + i];
      const int rs = b * F.nb[I] + b;
      const double *src = g + (size_t)b * (b * (size_t)pptr[i] + b * (size_t)i);
      for (int d = 0; d < b; d++) {
        double *dst = F.g.data() + ((size_t)I * b + d) * gs;
        std::memcpy(dst, src + (size_t)d * rs, rs * sizeof(double));
        std::memset(dst + rs, 0, (gs - rs) * sizeof(double));
      }
      std::memcpy(F.psi.data() + (size_t)I * b, psi.data() + (size_t)i * b, b * sizeof(double));
      std::memcpy(F.add.data() + (size_t)I * F.rho, add.data() + (size_t)i * F.rho, F.rho * sizeof(int32_t));
    }
  }
}

inline double psi_sum(const FsaiState &F, int32_t I) {
  double s = 0.0;
  for (int d = 0; d < F.b; d++) s += F.psi[(size_t)I * F.b + d];
  return s;
}

// One growth step of row I (the adaptive step): the nodes the device chose
// from the row's current pattern and g (scores h_{(I,d),(J,e)} over the
// candidates J < I adjacent to B u {I}, the rho largest quantised, ties to the
// lowest J) join B.  Returns the number added.
int apply_growth(FsaiState &F, int32_t I) {
  const int32_t nb = F.nb[I];
  const int32_t *a = F.add.data() + (size_t)I * F.rho;
  int k = 0;
  while (k < F.rho && a[k] >= 0) k++;
  if (k == 0) return 0;
  int32_t *B = F.nodes.data() + (size_t)I * kMaxFsaiNodes;
  for (int j = 0; j < k; j++) B[nb + j] = a[j];
  F.nb[I] = nb + k;
  std::sort(B, B + nb + k);
  std::fill(F.add.data() + (size_t)I * F.rho, F.add.data() + (size_t)(I + 1) * F.rho, -1);
  return k;
}

HostBSR fsai_assemble(const FsaiState &F) {
  HostBSR G;
  const int32_t n = F.n;
  const int gs = FsaiState::gstride;
  const int b = F.b, bb = b * b;
  G.n = G.nc = n;
  G.b = b;
  G.rp.assign(n + 1, 0);
  for (int32_t i = 0; i < n; i++) G.rp[i + 1] = G.rp[i] + F.nb[i] + 1;
  G.ci.resize(G.rp[n]);
  G.v.assign((size_t)G.rp[n] * bb, 0.0);
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; i++) {
    const int nb = F.nb[i];
    const double *g = F.g.data() + (size_t)i * b * gs;
    for (int p = 0; p <= nb; p++) {
      const int64_t q = G.rp[i] + p;
      G.ci[q] = p < nb ? F.nodes[(size_t)i * kMaxFsaiNodes + p] : i;
      for (int d = 0; d < b; d++)
        for (int e = 0; e < b; e++) {
          if (p == nb && e > d) continue;
          G.v[(size_t)q * bb + d * b + e] = g[d * gs + p * b + e];
        }
    }
  }
  return G;
}

// lambda_1(G A G^T) by plain Lanczos on the GPU (FP64 SELL products), the
// largest Ritz value by Sturm bisection.
double lanczos_gagt(aspamg_ctx *h, const Level &L, const Sell<double> &G, const Sell<double> &GT, int steps) {
  const int64_t n = (int64_t)L.A.n * L.A.b;
  hipStream_t s = h->stream;
  std::vector<double> w(n);
  for (int64_t i = 0; i < n; i++) {
    const uint64_t hs = ((uint64_t)i * 2654435761ULL) & 0xFFFFFFFFULL;
    w[i] = (double)hs / 4294967296.0 - 0.5;
  }
  double nw = 0.0;
  for (int64_t i = 0; i < n; i++) nw += w[i] * w[i];
  nw = std::sqrt(nw);
  for (int64_t i = 0; i < n; i++) w[i] /= nw;
  Scratch dv(n * 8), dvp(n * 8), du(n * 8), dt1(n * 8), dt2(n * 8), dpart(kMaxPart * 8);
  double *v = dv.as<double>(), *vp = dvp.as<double>(), *u = du.as<double>();
  to_device(s, v, w.data(), n);
  std::vector<double> al, be;
  std::vector<double> hp(kMaxPart);
  const int nb = vec_blocks(n);
  auto dotv = [&](const double *a, const double *b) {
    launch_dot(n, a, b, dpart.as<double>(), nullptr, s);
    to_host(s, hp.data(), dpart.as<double>(), nb);
    double acc = 0.0;
    for (int i = 0; i < nb; i++) acc += hp[i];
    return acc;
  };
  // the recurrence on the device; the two inner products per step are summed
  // from their block partials in block order on the host
  double bprev = 0.0;
  for (int j = 0; j < steps; j++) {
    launch_spmv<double, double, double>(GT, v, dt1.as<double>(), nullptr, 1.0, nullptr, s);
    launch_spmv<double, double, double>(L.A64, dt1.as<double>(), dt2.as<double>(), nullptr, 1.0, nullptr, s);
    launch_spmv<double, double, double>(G, dt2.as<double>(), u, nullptr, 1.0, nullptr, s);
    // u -= bprev vp ; a = v.u ; u -= a v ; b = |u|
    if (j > 0) launch_axpy(n, -bprev, vp, u, s);
    const double a = dotv(v, u);
    launch_axpy(n, -a, v, u, s);
    const double bb = std::sqrt(dotv(u, u));
    al.push_back(a);
    be.push_back(bb);
    if (!(bb > 1e-300)) break;
    HIPCHK(hipMemcpyAsync(vp, v, n * 8, hipMemcpyDeviceToDevice, s));
    launch_divided(n, bb, u, v, s);
    bprev = bb;
  }
  HIPCHK(hipGetLastError());
  // Sturm bisection for the largest eigenvalue of the tridiagonal matrix
  const int m = (int)al.size();
  double lo = al[0], hi = al[0];
  for (int i = 0; i < m; i++) {
    const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(be[i]) : 0.0);
    lo = std::min(lo, al[i] - r);
    hi = std::max(hi, al[i] + r);
  }
  for (int it = 0; it < 2000; it++) {
    const double x = 0.5 * (lo + hi);
    if (x <= lo || x >= hi) break;
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < m; i++) {
      const double off = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
      d = (al[i] - x) - (i > 0 ? off / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) cnt++;
    }
    if (cnt == m) hi = x;
    else lo = x;
  }
  return hi;
}

// Wall time of the setup phases per level, printed to stderr when the
// environment variable ASPAMG_TRACE is set.
struct PhaseClock {
  bool on = std::getenv("ASPAMG_TRACE") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void tick(int level, const char *phase) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[aspamg] level %d %-12s %8.1f ms\n", level, phase,
                 std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

void build_fsai(aspamg_ctx *h, Level &L) {
  const aspamg_params &p = h->p;
  const Q q{p.quant_bits};
  const int32_t n = L.A.n;
  FsaiState F;
  F.n = n;
  F.b = L.A.b;
  F.nb.assign(n, 0);
  F.nodes.assign((size_t)n * kMaxFsaiNodes, -1);
  F.g.assign((size_t)n * F.b * FsaiState::gstride, 0.0);
  F.psi.assign((size_t)n * F.b, 0.0);
  F.rho = p.rho_blocks;
  F.add.assign((size_t)n * F.rho, -1);
  std::vector<int32_t> active(n);
  std::iota(active.begin(), active.end(), 0);
  PhaseClock clk;
  fsai_factor(h, L, F, active);
  clk.tick(-1, "fsai factor");
  std::vector<double> psi_prev(n);
  for (int32_t i = 0; i < n; i++) psi_prev[i] = psi_sum(F, i);
  for (int step = 0; step < p.k_g && !active.empty(); step++) {
    std::vector<char> grew(active.size(), 0);
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < (int64_t)active.size(); a++) grew[a] = apply_growth(F, active[a]) > 0;
    std::vector<int32_t> next;
    for (size_t a = 0; a < active.size(); a++)
      if (grew[a]) next.push_back(active[a]);
    clk.tick(-1, "fsai grow");
    fsai_factor(h, L, F, next);
    clk.tick(-1, "fsai factor");
    std::vector<int32_t> keep;
    for (int32_t I : next) {
      const double pn = psi_sum(F, I);
      const double dec = q(psi_prev[I] - pn), thr = q(p.eps_g * psi_prev[I]);
      psi_prev[I] = pn;
      if (!(dec <= thr)) keep.push_back(I);
    }
    active.swap(keep);
  }
  L.G = fsai_assemble(F);
  clk.tick(-1, "fsai assemble");
  L.fsai_rounds = 0;
  for (;;) {
    // device copies of G and G^T for the Lanczos estimate, in the layouts
    // chosen by stored slots (no timing: the loop may run many rounds)
    Sell<double> g = upload_sell<double>(h, L.G, 0, false);
    Sell<double> gt = upload_sell<double>(h, transpose(L.G), 0, false);
    clk.tick(-1, "fsai G upload");
    L.lambda1 = lanczos_gagt(h, L, g, gt, p.lanczos_steps);
    free_sell(h, g);
    free_sell(h, gt);
    clk.tick(-1, "lanczos");
    L.omega_q = 2.0 / L.lambda1;
    if (!p.outer_fsai) break;
    if (!(q(L.omega_q) < q(p.omega_bar))) break;
    if (!(L.G.nnzb() < L.A.nnzb())) break;
    std::vector<char> grew(n, 0);
#pragma omp parallel for schedule(static)
    for (int32_t I = 0; I < n; I++) grew[I] = apply_growth(F, I) > 0;
    std::vector<int32_t> rows;
    for (int32_t I = 0; I < n; I++)
      if (grew[I]) rows.push_back(I);
    if (rows.empty()) break;            // G unchanged
    fsai_factor(h, L, F, rows);
    L.G = fsai_assemble(F);
    L.fsai_rounds++;
  }
  // the level's operators: G and G^T of the final round, FP64 and FP32 copies
  // in the layouts timed on the device
  upload_sell_pair(h, L.G, nullptr, L.G64, L.G32);
  upload_sell_pair(h, transpose(L.G), nullptr, L.GT64, L.GT32);
  clk.tick(-1, "fsai G upload");
  const double w = 2.0 / (p.omega_safety * L.lambda1);
  L.omega_s = w < 1.0 ? w : 1.0;
}

// ------------------------------------------------------------------------
// test space (Section 3.3): Cholesky-QR orthonormalisation with the Gram
// matrix summed over scalar rows in ascending order; a column whose pivot is
// <= 1e-12 of its Gram diagonal is dropped (set to zero).
// ------------------------------------------------------------------------
void orthonormalize(std::vector<double> &V, int64_t nrows, int ntv) {
  std::vector<double> W((size_t)ntv * ntv), Lm((size_t)ntv * ntv, 0.0);
  // Gram entries (a <= c; W_ca is the same sum): the pairs are dealt to the
  // threads, and each thread streams the rows once for all its pairs, every
  // entry still summed over the rows in ascending order
  const int npairs = ntv * (ntv + 1) / 2;
  std::vector<int> pa(npairs), pc(npairs);
  for (int a = 0, k = 0; a < ntv; a++)
    for (int c = a; c < ntv; c++, k++) {
      pa[k] = a;
      pc[k] = c;
    }
#pragma omp parallel
  {
    const int t = omp_get_thread_num(), nt = omp_get_num_threads();
    std::vector<int> mine;
    for (int k = t; k < npairs; k += nt) mine.push_back(k);
    std::vector<double> acc(mine.size(), 0.0);
    for (int64_t i = 0; i < nrows; i++) {
      const double *v = V.data() + (size_t)i * ntv;
      for (size_t m = 0; m < mine.size(); m++) acc[m] += v[pa[mine[m]]] * v[pc[mine[m]]];
    }
    for (size_t m = 0; m < mine.size(); m++) {
      W[pa[mine[m]] * ntv + pc[mine[m]]] = acc[m];
      W[pc[mine[m]] * ntv + pa[mine[m]]] = acc[m];
    }
  }
  std::vector<char> drop(ntv, 0);
  for (int j = 0; j < ntv; j++) {
    double acc = 0.0;
    for (int k = 0; k < j; k++) acc += Lm[j * ntv + k] * Lm[j * ntv + k];
    const double d = W[j * ntv + j] - acc;
    drop[j] = !(d > 1e-12 * W[j * ntv + j]);
    const double ljj = drop[j] ? 1.0 : std::sqrt(d);
    Lm[j * ntv + j] = ljj;
    for (int i = j + 1; i < ntv; i++) {
      if (drop[j]) {
        Lm[i * ntv + j] = 0.0;
        continue;
      }
      double a2 = 0.0;
      for (int k = 0; k < j; k++) a2 += Lm[i * ntv + k] * Lm[j * ntv + k];
      Lm[i * ntv + j] = (W[i * ntv + j] - a2) / ljj;
    }
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nrows; i++) {
    double y[64];
    double *v = V.data() + (size_t)i * ntv;
    for (int a = 0; a < ntv; a++) {
      if (drop[a]) {
        y[a] = 0.0;
        continue;
      }
      double acc = 0.0;
      for (int c = 0; c < a; c++) acc += Lm[a * ntv + c] * y[c];
      y[a] = (v[a] - acc) / Lm[a * ntv + a];
    }
    std::memcpy(v, y, ntv * sizeof(double));
  }
}

// ------------------------------------------------------------------------
// test space by SRQCG (Section 3.3, Algorithm "Test Space generation by
// SRQCG"): the columns of Z minimise their Rayleigh quotients for
// S = G A G^T by conjugate gradients, with a Ritz projection every
// iteration (k_ritz = 1, as in the paper's experiments), then V = G^T Z.
//   - q is the Rayleigh quotient z^T S z / z^T z; f_i starts at 1 and is
//     z_i^T z_i after each update of column i (kept across a projection);
//   - S Z is formed by products at every projection and then carried
//     (S z_i += alpha S p_i; S Z <- (S Z) U);
//   - the projection solves (Z^T S Z) U = (Z^T Z) U Lambda through the
//     Cholesky factor of Z^T Z and Jacobi rotations, eigenvalues ascending,
//     each eigenvector with its largest-magnitude entry positive (the first
//     on ties); it is skipped when Z^T Z is not positive definite;
//   - a column update with 2(bc - ad) = 0 or a negative discriminant is
//     skipped; exactly n_rq iterations run.
// Products, vector updates and inner products run on the device (FP64 SELL
// products; inner products summed from block partials in block order); the
// nt x nt eigenproblems on the host.
// ------------------------------------------------------------------------

// C (symmetric m x m, row-major, destroyed) = X diag(w) X^T by cyclic Jacobi
// rotations; w ascending, eigenvectors in the columns of X.
void jacobi_sym(std::vector<double> &C, int m, std::vector<double> &w, std::vector<double> &X) {
  auto at = [m](std::vector<double> &M, int i, int j) -> double & { return M[(size_t)i * m + j]; };
  X.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; i++) at(X, i, i) = 1.0;
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0.0, all = 0.0;
    for (int i = 0; i < m; i++)
      for (int j = 0; j < m; j++) {
        const double c2 = at(C, i, j) * at(C, i, j);
        all += c2;
        if (i != j) off += c2;
      }
    if (!(off > 1e-32 * all)) break;
    for (int p = 0; p + 1 < m; p++)
      for (int q = p + 1; q < m; q++) {
        const double apq = at(C, p, q);
        if (apq == 0.0) continue;
        // the rotation angle t = tan(phi) zeroing C[p][q], the smaller root
        const double th = (at(C, q, q) - at(C, p, p)) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < m; k++) {
          const double a = at(C, k, p), b = at(C, k, q);
          at(C, k, p) = c * a - sn * b;
          at(C, k, q) = sn * a + c * b;
        }
        for (int k = 0; k < m; k++) {
          const double a = at(C, p, k), b = at(C, q, k);
          at(C, p, k) = c * a - sn * b;
          at(C, q, k) = sn * a + c * b;
        }
        for (int k = 0; k < m; k++) {
          const double a = at(X, k, p), b = at(X, k, q);
          at(X, k, p) = c * a - sn * b;
          at(X, k, q) = sn * a + c * b;
        }
      }
  }
  w.resize(m);
  for (int i = 0; i < m; i++) w[i] = at(C, i, i);
  for (int i = 0; i < m; i++) {   // ascending; the first smallest moves first
    int k = i;
    for (int j = i + 1; j < m; j++)
      if (w[j] < w[k]) k = j;
    if (k == i) continue;
    std::swap(w[i], w[k]);
    for (int r = 0; r < m; r++) std::swap(at(X, r, i), at(X, r, k));
  }
}

// U with (Z^T S Z) U = (Z^T Z) U Lambda from Ms = Z^T S Z (symmetrised) and
// Mz = Z^T Z; false when Mz is not positive definite.
bool ritz_basis(const std::vector<double> &Ms, const std::vector<double> &Mz, int m, std::vector<double> &U) {
  std::vector<double> L((size_t)m * m, 0.0), T((size_t)m * m), C((size_t)m * m), X, w;
  for (int j = 0; j < m; j++) {   // Mz = L L^T, left-looking
    double acc = 0.0;
    for (int k = 0; k < j; k++) acc += L[j * m + k] * L[j * m + k];
    const double d = Mz[j * m + j] - acc;
    if (!(d > 0.0)) return false;
    L[j * m + j] = std::sqrt(d);
    for (int i = j + 1; i < m; i++) {
      double a2 = 0.0;
      for (int k = 0; k < j; k++) a2 += L[i * m + k] * L[j * m + k];
      L[i * m + j] = (Mz[i * m + j] - a2) / L[j * m + j];
    }
  }
  for (int c = 0; c < m; c++)     // T = L^{-1} Ms
    for (int i = 0; i < m; i++) {
      double acc = Ms[i * m + c];
      for (int k = 0; k < i; k++) acc -= L[i * m + k] * T[k * m + c];
      T[i * m + c] = acc / L[i * m + i];
    }
  for (int r = 0; r < m; r++)     // C = T L^{-T}
    for (int i = 0; i < m; i++) {
      double acc = T[r * m + i];
      for (int k = 0; k < i; k++) acc -= L[i * m + k] * C[r * m + k];
      C[r * m + i] = acc / L[i * m + i];
    }
  for (int a = 0; a < m; a++)
    for (int c = 0; c < a; c++) C[a * m + c] = C[c * m + a] = 0.5 * (C[a * m + c] + C[c * m + a]);
  jacobi_sym(C, m, w, X);
  U.assign((size_t)m * m, 0.0);
  for (int c = 0; c < m; c++) {   // U = L^{-T} X, then the sign rule
    for (int i = m - 1; i >= 0; i--) {
      double acc = X[i * m + c];
      for (int k = i + 1; k < m; k++) acc -= L[k * m + i] * U[k * m + c];
      U[i * m + c] = acc / L[i * m + i];
    }
    int big = 0;
    for (int i = 1; i < m; i++)
      if (std::fabs(U[i * m + c]) > std::fabs(U[big * m + c])) big = i;
    if (U[big * m + c] < 0.0)
      for (int i = 0; i < m; i++) U[i * m + c] = -U[i * m + c];
  }
  return true;
}

// V ([n*3][nt] row-major) <- G^{-T} V: back substitution with the rows of the
// block lower triangular G, scalar rows from the last to the first.  x_r is
// divided by g_rr, then g_rk x_r is subtracted from x_k for every k < r of row
// r; each column sees exactly that sequence of operations.
static void gt_solve(const HostBSR &G, std::vector<double> &V, int nt) {
  const int b = G.b, bb = b * b;
  const int64_t nr = (int64_t)G.n * b;
  std::vector<int64_t> diag(G.n);
  for (int32_t I = 0; I < G.n; I++) {
    int64_t kd = G.rp[I + 1] - 1;
    while (kd >= G.rp[I] && G.ci[kd] != I) kd--;
    if (kd < G.rp[I]) fail(ASPAMG_EINVAL, "srqcg: FSAI factor without a diagonal block");
    diag[I] = kd;
  }
#pragma omp parallel for schedule(static, 1)
  for (int c = 0; c < nt; c++) {
    double *x = V.data() + c;
    for (int64_t r = nr - 1; r >= 0; r--) {
      const int32_t I = (int32_t)(r / b);
      const int d = (int)(r % b);
      const double xr = x[r * nt] / G.v[diag[I] * bb + d * b + d];
      x[r * nt] = xr;
      for (int64_t k = G.rp[I]; k < G.rp[I + 1]; k++) {
        const int32_t J = G.ci[k];
        const int ne = J < I ? b : d;     // in the diagonal block only the columns e < d
        for (int e = 0; e < ne; e++) x[((int64_t)J * b + e) * nt] -= G.v[k * bb + d * b + e] * xr;
      }
    }
  }
}

// L.V ([n][nt], in: the level's V0) <- G^T Z after kmax SRQCG iterations.  The
// iterates live in the variable of S = G A G^T (A v = lambda (G^T G)^{-1} v is
// S z = lambda z with v = G^T z, hence V = G^T Z at the end); V0 approximates
// the near kernel of A, so it enters as G^{-T} V0: Z0 = (I - S) G^{-T} V0.
void srqcg(aspamg_ctx *h, Level &L, int nt, int kmax) {
  const int64_t n = (int64_t)L.A.n * L.A.b;
  const size_t cols = (size_t)n * nt;
  hipStream_t s = h->stream;
  // inner products in the fixed order of 256-entry blocks and products summed
  // row by row in stored order, as the sequential definition sums them: the
  // test space, and every decision that depends on it, is then bitwise the
  // sequential one
  const int nb = dot256_parts(n);
  Scratch dZ(cols * 8), dSZ(cols * 8), dP(cols * 8), dW(cols * 8), dsp(n * 8), dg(n * 8), dt1(n * 8), dt2(n * 8),
      dU((size_t)nt * nt * 8), dpart((size_t)nb * std::max(5, 2 * nt * nt) * 8);
  double *Z = dZ.as<double>(), *SZ = dSZ.as<double>(), *Pd = dP.as<double>(), *W = dW.as<double>();
  double *sp = dsp.as<double>(), *g = dg.as<double>(), *part = dpart.as<double>();
  auto C = [n](double *M, int c) { return M + (size_t)c * n; };
  // plain block-CSR copies of G and G^T for the sequential products (A's is L.dA)
  const HostBSR GT = transpose(L.G);
  struct Plain {
    Scratch rp, ci, v;
    DevBSR d;
    Plain(hipStream_t s, const HostBSR &M)
        : rp(((size_t)M.n + 1) * 4), ci(std::max<size_t>(M.ci.size(), 1) * 4), v(std::max<size_t>(M.v.size(), 1) * 8) {
      std::vector<int32_t> rp32(M.rp.begin(), M.rp.end());
      to_device(s, rp.as<int32_t>(), rp32.data(), rp32.size());
      to_device(s, ci.as<int32_t>(), M.ci.data(), M.ci.size());
      to_device(s, v.as<double>(), M.v.data(), M.v.size());
      d.n = M.n;
      d.nc = M.nc;
      d.b = M.b;
      d.nnzb = M.nnzb();
      d.rp = rp.as<int32_t>();
      d.ci = ci.as<int32_t>();
      d.v = v.as<double>();
    }
  } pG(s, L.G), pGT(s, GT);
  auto apply_s = [&](const double *x, double *y) {
    launch_bsr_mv_seq(pGT.d, x, dt1.as<double>(), s);
    launch_bsr_mv_seq(L.dA, dt1.as<double>(), dt2.as<double>(), s);
    launch_bsr_mv_seq(pG.d, dt2.as<double>(), y, s);
  };
  std::vector<double> hp;
  using Pair = std::pair<const double *, const double *>;
  const size_t max_pairs = (size_t)std::max(5, 2 * nt * nt);
  auto dots = [&](const std::vector<Pair> &pr) {
    if (pr.size() > max_pairs) fail(ASPAMG_EINVAL, "srqcg: too many inner products in one batch");
    for (size_t k = 0; k < pr.size(); k++) launch_dot256(n, pr[k].first, pr[k].second, part + k * nb, s);
    HIPCHK(hipGetLastError());
    hp.resize(pr.size() * nb);
    to_host(s, hp.data(), part, pr.size() * nb);
    std::vector<double> out(pr.size(), 0.0);
    for (size_t k = 0; k < pr.size(); k++)
      for (int i = 0; i < nb; i++) out[k] += hp[k * nb + i];
    return out;
  };
  auto to_columns = [&](const std::vector<double> &rows, double *dst) {
    std::vector<double> cm(cols);
    for (int64_t i = 0; i < n; i++)
      for (int c = 0; c < nt; c++) cm[(size_t)c * n + i] = rows[(size_t)i * nt + c];
    to_device(s, dst, cm.data(), cols);
    HIPCHK(hipStreamSynchronize(s));
  };
  auto to_rows = [&](const double *src, std::vector<double> &rows) {
    std::vector<double> cm(cols);
    to_host(s, cm.data(), src, cols);
    rows.resize(cols);
    for (int64_t i = 0; i < n; i++)
      for (int c = 0; c < nt; c++) rows[(size_t)i * nt + c] = cm[(size_t)c * n + i];
  };
  // Z0 = (I - S) G^{-T} V0, orthonormalised
  gt_solve(L.G, L.V, nt);
  to_columns(L.V, W);
  for (int c = 0; c < nt; c++) {
    apply_s(C(W, c), C(SZ, c));
    HIPCHK(hipMemcpyAsync(C(Z, c), C(W, c), n * 8, hipMemcpyDeviceToDevice, s));
    launch_axpy(n, -1.0, C(SZ, c), C(Z, c), s);
  }
  HIPCHK(hipGetLastError());
  {
    std::vector<double> rows;
    to_rows(Z, rows);
    orthonormalize(rows, n, nt);
    to_columns(rows, Z);
  }
  // initial residuals and search directions
  std::vector<double> f(nt, 1.0);
  for (int c = 0; c < nt; c++) {
    apply_s(C(Z, c), C(SZ, c));
    const std::vector<double> ef = dots({{C(Z, c), C(SZ, c)}, {C(Z, c), C(Z, c)}});
    const double q = ef[1] > 0.0 ? ef[0] / ef[1] : 0.0;
    launch_rq_gradient(n, q, 1.0, C(SZ, c), C(Z, c), C(Pd, c), s);
  }
  std::vector<double> Ms((size_t)nt * nt), Mz((size_t)nt * nt), U;
  for (int k = 1; k <= kmax; k++) {
    // Ritz projection
    for (int c = 0; c < nt; c++) apply_s(C(Z, c), C(SZ, c));
    std::vector<Pair> pr;
    for (int a = 0; a < nt; a++)
      for (int c = 0; c < nt; c++) pr.push_back({C(Z, a), C(SZ, c)});
    for (int a = 0; a < nt; a++)
      for (int c = 0; c <= a; c++) pr.push_back({C(Z, a), C(Z, c)});
    const std::vector<double> m = dots(pr);
    size_t t = 0;
    for (int a = 0; a < nt; a++)
      for (int c = 0; c < nt; c++) Ms[a * nt + c] = m[t++];
    for (int a = 0; a < nt; a++)
      for (int c = 0; c <= a; c++) Mz[a * nt + c] = Mz[c * nt + a] = m[t++];
    for (int a = 0; a < nt; a++)
      for (int c = 0; c < a; c++) Ms[a * nt + c] = Ms[c * nt + a] = 0.5 * (Ms[a * nt + c] + Ms[c * nt + a]);
    if (ritz_basis(Ms, Mz, nt, U)) {
      to_device(s, dU.as<double>(), U.data(), U.size());
      launch_combine_columns(n, nt, Z, dU.as<double>(), W, s);
      std::swap(Z, W);
      launch_combine_columns(n, nt, SZ, dU.as<double>(), W, s);
      std::swap(SZ, W);
      HIPCHK(hipGetLastError());
    }
    // one conjugate-gradient step per column
    for (int c = 0; c < nt; c++) {
      double *z = C(Z, c), *p = C(Pd, c), *sz = C(SZ, c);
      apply_s(p, sp);
      const std::vector<double> v = dots({{p, sz}, {p, sp}, {p, z}, {p, p}, {z, sz}});
      const double a = v[0], b = v[1], cc = v[2], d = v[3], e = v[4], fi = f[c];
      const double den = 2.0 * (b * cc - a * d);
      const double u1 = d * e - b * fi;
      const double delta = u1 * u1 - 4.0 * (b * cc - a * d) * (a * fi - cc * e);
      if (!(den != 0.0) || !(delta >= 0.0)) continue;
      const double alpha = (u1 + std::sqrt(delta)) / den;
      launch_axpy(n, alpha, p, z, s);
      launch_axpy(n, alpha, sp, sz, s);
      const std::vector<double> zq = dots({{z, z}, {z, sz}});
      f[c] = zq[0];
      const double q = zq[1] / zq[0];
      launch_rq_gradient(n, q, zq[0], sz, z, g, s);
      const double beta = -dots({{g, sp}})[0] / b;
      launch_xpby(n, g, beta, p, s);
    }
  }
  // V = G^T Z
  for (int c = 0; c < nt; c++) launch_bsr_mv_seq(pGT.d, C(Z, c), C(W, c), s);
  HIPCHK(hipGetLastError());
  to_rows(W, L.V);
}

// ------------------------------------------------------------------------
// coarsening (Section 3.4)
// ------------------------------------------------------------------------
// ------------------------------------------------------------------------
// C/F split on the device (Section 3.4): strong graph S (theta filter of the
// affinity SoC, union symmetrisation) and its maximal independent set.  The
// decisions are bitwise those of the sequential rules (kernels_coarsen.hip).
// ------------------------------------------------------------------------
struct DevGraph {
  Scratch rp, ci;
  DevGraph(size_t n1, size_t nnz) : rp(n1 * 8), ci(nnz * 4) {}
};

std::unique_ptr<DevGraph> strong_graph_device(aspamg_ctx *h, const Level &L, const int8_t *dexcl, const double *dV,
                                              int ntv) {
  const aspamg_params &p = h->p;
  const int32_t n = L.A.n;
  hipStream_t s = h->stream;
  const int theta = p.theta;
  Scratch dsq((size_t)n * 8), dkeep((size_t)n * theta * 4), dnk((size_t)n * 4), dcnt((size_t)n * 4);
  launch_node_norms(n, dV, ntv, L.A.b, dsq.as<double>(), s);
  launch_strong_topk(L.dA, dexcl, dV, ntv, dsq.as<double>(), theta, p.quant_bits, dkeep.as<int32_t>(),
                     dnk.as<int32_t>(), s);
  HIPCHK(hipMemsetAsync(dcnt.p, 0, (size_t)n * 4, s));
  launch_union(n, theta, dkeep.as<int32_t>(), dnk.as<int32_t>(), 0, dcnt.as<int32_t>(), nullptr, nullptr, nullptr,
               nullptr, nullptr, nullptr, s);
  HIPCHK(hipGetLastError());
  std::vector<int32_t> cnt(n);
  to_host(s, cnt.data(), dcnt.as<int32_t>(), n);
  std::vector<int64_t> bp((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; i++) bp[(size_t)i + 1] = bp[i] + cnt[i];
  Scratch dbp(((size_t)n + 1) * 8), dat(((size_t)n + 1) * 8), dboth((size_t)std::max<int64_t>(bp[n], 1) * 4),
      dlen((size_t)n * 4);
  to_device(s, dbp.as<int64_t>(), bp.data(), bp.size());
  to_device(s, dat.as<int64_t>(), bp.data(), bp.size());
  launch_union(n, theta, dkeep.as<int32_t>(), dnk.as<int32_t>(), 1, nullptr, dbp.as<int64_t>(), dat.as<int64_t>(),
               dboth.as<int32_t>(), dlen.as<int32_t>(), nullptr, nullptr, s);
  HIPCHK(hipGetLastError());
  std::vector<int32_t> len(n);
  to_host(s, len.data(), dlen.as<int32_t>(), n);
  std::vector<int64_t> srp((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; i++) srp[(size_t)i + 1] = srp[i] + len[i];
  auto S = std::make_unique<DevGraph>((size_t)n + 1, (size_t)std::max<int64_t>(srp[n], 1));
  to_device(s, S->rp.as<int64_t>(), srp.data(), srp.size());
  launch_union(n, theta, nullptr, nullptr, 2, nullptr, dbp.as<int64_t>(), nullptr, dboth.as<int32_t>(), nullptr,
               S->rp.as<int64_t>(), S->ci.as<int32_t>(), s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return S;
}

// maximal independent set of S in descending (|S_I|, splitmix64(I), -I): local
// maximum rounds on the device until every node is decided; L.cf on the host
void mis_device(aspamg_ctx *h, Level &L, const DevGraph &S, const int8_t *dexcl, int8_t *dcf) {
  const int32_t n = L.A.n;
  hipStream_t s = h->stream;
  Scratch dwin((size_t)n), dund(4);
  launch_mis_init(n, dexcl, dcf, s);
  for (int round = 0;; round++) {
    if (round > n) fail(ASPAMG_EHIP, "independent set: no progress");
    HIPCHK(hipMemsetAsync(dund.p, 0, 4, s));
    launch_mis_round(n, S.rp.as<int64_t>(), S.ci.as<int32_t>(), dcf, dwin.as<int8_t>(), dund.as<int32_t>(), s);
    HIPCHK(hipGetLastError());
    int32_t und = 0;
    to_host(s, &und, dund.as<int32_t>(), 1);
    if (und == 0) break;
  }
  L.cf.resize(n);
  to_host(s, L.cf.data(), dcf, n);
}

void build_prolongation(aspamg_ctx *h, Level &L, const DevGraph &S, const int8_t *dcf, const double *dV) {
  const aspamg_params &p = h->p;
  const Q q{p.quant_bits};
  const int32_t n = L.A.n;
  const int ntv = h->ntv;
  const int nmax = std::min(p.n_max, kMaxPEntries);
  const int b = L.A.b, bb = b * b;
  hipStream_t s = h->stream;
  L.pcount.assign((size_t)n * b, 0);
  L.pcols.assign((size_t)n * b * p.n_max, -1);
  // interpolation entries of every fine scalar row, chosen on the device
  std::vector<int32_t> fnodes;
  for (int32_t I = 0; I < n; I++)
    if (L.cf[I] == 0) fnodes.push_back(I);
  std::vector<int32_t> selfine((size_t)n * b * kMaxPEntries, 0);
  {
    Scratch dfn(fnodes.size() * 4), dcnt((size_t)n * b * 4), dsel(selfine.size() * 4), derr(4);
    to_device(s, dfn.as<int32_t>(), fnodes.data(), fnodes.size());
    HIPCHK(hipMemsetAsync(dcnt.p, 0, (size_t)n * b * 4, s));
    HIPCHK(hipMemsetAsync(dsel.p, 0, selfine.size() * 4, s));
    HIPCHK(hipMemsetAsync(derr.p, 0, 4, s));
    launch_dpls_rows((int32_t)fnodes.size(), dfn.as<int32_t>(), S.rp.as<int64_t>(), S.ci.as<int32_t>(), dcf, dV, ntv,
                     b, p.d_p, nmax, q(p.kappa_p), p.eps_p, p.quant_bits, dcnt.as<int32_t>(), dsel.as<int32_t>(),
                     derr.as<int32_t>(), s);
    HIPCHK(hipGetLastError());
    int32_t err = 0;
    to_host(s, &err, derr.as<int32_t>(), 1);
    if (err)
      fail(ASPAMG_EINVAL, "DPLS: a fine node has more interpolation candidates than the device selection holds "
                          "(1024 nodes within distance d_p, 320 coarse ones, 5120 candidate values)");
    to_host(s, L.pcount.data(), dcnt.as<int32_t>(), (size_t)n * b);
    to_host(s, selfine.data(), dsel.as<int32_t>(), selfine.size());
  }
  for (size_t r = 0; r < (size_t)n * b; r++)
    for (int k = 0; k < L.pcount[r]; k++) {
      const int32_t f = selfine[r * kMaxPEntries + k];
      L.pcols[r * p.n_max + k] = L.cidx[f / b] * b + f % b;
    }
  // weights on the GPU: normal equations of the chosen columns
  std::vector<int32_t> rows, cnt, sel;
  for (int64_t r = 0; r < (int64_t)n * b; r++) {
    if (L.pcount[r] == 0) continue;
    rows.push_back((int32_t)r);
    cnt.push_back(L.pcount[r]);
    for (int k = 0; k < kMaxPEntries; k++) sel.push_back(selfine[(size_t)r * kMaxPEntries + k]);
  }
  std::vector<double> w((size_t)rows.size() * kMaxPEntries, 0.0);
  if (!rows.empty()) {
    Scratch dr(rows.size() * 4), dc(cnt.size() * 4), ds(sel.size() * 4), dw(w.size() * 8);
    to_device(h->stream, dr.as<int32_t>(), rows.data(), rows.size());
    to_device(h->stream, dc.as<int32_t>(), cnt.data(), cnt.size());
    to_device(h->stream, ds.as<int32_t>(), sel.data(), sel.size());
    launch_dpls_weights((int32_t)rows.size(), dr.as<int32_t>(), dc.as<int32_t>(), ds.as<int32_t>(), dV, ntv,
                        dw.as<double>(), h->stream);
    HIPCHK(hipGetLastError());
    to_host(h->stream, w.data(), dw.as<double>(), w.size());
    for (size_t i = 0; i < rows.size(); i++)
      for (int k = 0; k < cnt[i]; k++)
        if (std::isnan(w[i * kMaxPEntries + k])) fail(ASPAMG_ENOT_SPD, "DPLS: weight Gram matrix not positive definite");
  }
  std::vector<double> wr((size_t)n * b * kMaxPEntries, 0.0);
  for (size_t i = 0; i < rows.size(); i++)
    std::memcpy(wr.data() + (size_t)rows[i] * kMaxPEntries, w.data() + i * kMaxPEntries, kMaxPEntries * 8);
  // assemble P: C rows I3 at (I, c(I)); F rows: union of the chosen coarse nodes
  HostBSR &P = L.P;
  P.n = n;
  P.nc = L.nc;
  P.b = b;
  P.rp.assign(n + 1, 0);
  // coarse nodes of each row, sorted and unique (at most 3 kMaxPEntries)
  constexpr int kRowMax = 3 * kMaxPEntries;
  std::vector<int32_t> rowc((size_t)n * kRowMax), nrc(n, 0);
#pragma omp parallel for schedule(static)
  for (int32_t I = 0; I < n; I++) {
    int32_t *rc = rowc.data() + (size_t)I * kRowMax;
    int m = 0;
    if (L.cf[I] == 1) rc[m++] = L.cidx[I];
    else if (L.cf[I] == 0) {
      for (int d = 0; d < b; d++) {
        const size_t r = (size_t)I * b + d;
        for (int k = 0; k < L.pcount[r]; k++) rc[m++] = L.pcols[r * p.n_max + k] / b;
      }
      std::sort(rc, rc + m);
      m = (int)(std::unique(rc, rc + m) - rc);
    }
    nrc[I] = m;
  }
  for (int32_t I = 0; I < n; I++) P.rp[I + 1] = P.rp[I] + nrc[I];
  P.ci.resize(P.rp[n]);
  P.v.assign((size_t)P.rp[n] * bb, 0.0);
#pragma omp parallel for schedule(static)
  for (int32_t I = 0; I < n; I++) {
    const int64_t base = P.rp[I];
    const int32_t *rc = rowc.data() + (size_t)I * kRowMax;
    std::copy(rc, rc + nrc[I], P.ci.begin() + base);
    if (L.cf[I] == 1) {
      for (int d = 0; d < b; d++) P.v[(size_t)base * bb + d * (b + 1)] = 1.0;
    } else if (L.cf[I] == 0) {
      for (int d = 0; d < b; d++) {
        const size_t r = (size_t)I * b + d;
        for (int k = 0; k < L.pcount[r]; k++) {
          const int32_t sc = L.pcols[r * p.n_max + k];
          const int32_t cnod = sc / b, e = sc % b;
          const int64_t qpos = base + (std::lower_bound(rc, rc + nrc[I], cnod) - rc);
          P.v[(size_t)qpos * bb + d * b + e] = wr[r * kMaxPEntries + k];
        }
      }
    }
  }
}

// ------------------------------------------------------------------------
// Galerkin operator A_c = R (A P): patterns on the host, values on the GPU.
// ------------------------------------------------------------------------
HostBSR spgemm_pattern(const HostBSR &X, const HostBSR &Y, bool host_values = true) {
  HostBSR Z;
  Z.n = X.n;
  Z.nc = Y.nc;
  Z.b = X.b;
  Z.rp.assign(X.n + 1, 0);
  // two passes over the product structure: row lengths, then the columns of
  // each row written in place and sorted
#pragma omp parallel
  {
    std::vector<int32_t> mark(Y.nc, -1);
#pragma omp for schedule(dynamic, 512)
    for (int32_t i = 0; i < X.n; i++) {
      int64_t cnt = 0;
      for (int64_t k = X.rp[i]; k < X.rp[i + 1]; k++) {
        const int32_t l = X.ci[k];
        for (int64_t q = Y.rp[l]; q < Y.rp[l + 1]; q++) {
          const int32_t j = Y.ci[q];
          if (mark[j] != i) {
            mark[j] = i;
            cnt++;
          }
        }
      }
      Z.rp[i + 1] = cnt;
    }
  }
  for (int32_t i = 0; i < X.n; i++) Z.rp[i + 1] += Z.rp[i];
  Z.ci.resize(Z.rp[X.n]);
#pragma omp parallel
  {
    std::vector<int32_t> mark(Y.nc, -1);
#pragma omp for schedule(dynamic, 512)
    for (int32_t i = 0; i < X.n; i++) {
      int64_t at = Z.rp[i];
      for (int64_t k = X.rp[i]; k < X.rp[i + 1]; k++) {
        const int32_t l = X.ci[k];
        for (int64_t q = Y.rp[l]; q < Y.rp[l + 1]; q++) {
          const int32_t j = Y.ci[q];
          if (mark[j] != i) {
            mark[j] = i;
            Z.ci[at++] = j;
          }
        }
      }
      std::sort(Z.ci.begin() + Z.rp[i], Z.ci.begin() + Z.rp[i + 1]);
    }
  }
  if (host_values) Z.v.assign((size_t)Z.rp[X.n] * Z.bb(), 0.0);
  return Z;
}

struct DevTmp {
  std::vector<Scratch *> s;
  DevBSR make(const HostBSR &M, hipStream_t st, bool with_values) {
    DevBSR d;
    d.n = M.n;
    d.nc = M.nc;
    d.b = M.b;
    d.nnzb = M.nnzb();
    if (d.nnzb >= (int64_t)INT32_MAX) fail(ASPAMG_EINVAL, "operator too large for int32 block indices");
    std::vector<int32_t> rp32(M.rp.begin(), M.rp.end());
    s.push_back(new Scratch(rp32.size() * 4));
    d.rp = s.back()->as<int32_t>();
    s.push_back(new Scratch(std::max<size_t>(M.ci.size(), 1) * 4));
    d.ci = s.back()->as<int32_t>();
    s.push_back(new Scratch(std::max<size_t>((size_t)M.nnzb() * M.bb(), 1) * 8));
    d.v = s.back()->as<double>();
    to_device(st, d.rp, rp32.data(), rp32.size());
    to_device(st, d.ci, M.ci.data(), M.ci.size());
    if (with_values) to_device(st, d.v, M.v.data(), M.v.size());
    return d;
  }
  ~DevTmp() {
    for (auto *x : s) delete x;
  }
};

// A_c = R (A P).  The pattern of the intermediate T = A P is returned in *AP
// (no host values); its values stay on the device, in *dPAP = [P values;
// T values] (dalloc'd, the caller frees it), the block values of the stacked
// operator [P; A P].
HostBSR galerkin(aspamg_ctx *h, const Level &L, HostBSR *AP, double **dPAP) {
  HostBSR R = transpose(L.P);
  HostBSR T = spgemm_pattern(L.A, L.P, false);
  HostBSR Ac = spgemm_pattern(R, T);
  const int64_t nP = L.P.nnzb(), nT = T.nnzb();
  const int bb = L.P.bb();
  double *stack = dalloc<double>(h, (size_t)std::max<int64_t>(nP + nT, 1) * bb);
  DevTmp tmp;
  DevBSR dP = tmp.make(L.P, h->stream, true), dR = tmp.make(R, h->stream, true);
  DevBSR dT = tmp.make(T, h->stream, false), dC = tmp.make(Ac, h->stream, false);
  dT.v = stack + (size_t)nP * bb;
  if (nP > 0) HIPCHK(hipMemcpyAsync(stack, dP.v, (size_t)nP * bb * 8, hipMemcpyDeviceToDevice, h->stream));
  launch_spgemm_ap(L.dA, dP, dT, h->stream);
  launch_spgemm_rt(dR, dT, dC, h->stream);
  HIPCHK(hipGetLastError());
  to_host(h->stream, Ac.v.data(), dC.v, Ac.v.size());
  *AP = std::move(T);
  *dPAP = stack;
  return Ac;
}

// Pattern of [P; A P]: the rows of P, then those of A P (same columns); the
// block values are numbered in the same order (P's, then A P's)
HostBSR stack_rows(const HostBSR &P, const HostBSR &AP) {
  HostBSR S;
  S.n = P.n + AP.n;
  S.nc = P.nc;
  S.b = P.b;
  S.rp.resize((size_t)S.n + 1);
  for (int32_t i = 0; i <= P.n; i++) S.rp[i] = P.rp[i];
  for (int32_t i = 1; i <= AP.n; i++) S.rp[P.n + i] = P.rp[P.n] + AP.rp[i];
  S.ci = P.ci;
  S.ci.insert(S.ci.end(), AP.ci.begin(), AP.ci.end());
  return S;
}

// dense coarsest factor and explicit inverse (L^{-T} L^{-1})
void build_coarse(aspamg_ctx *h, const HostBSR &A) {
  const int b = A.b, bb = b * b;
  const int32_t nd = A.n * b;
  if (nd > h->p.dense_max_dof) fail(ASPAMG_EINVAL, "coarsest level too large for a dense factorisation");
  std::vector<double> M((size_t)nd * nd, 0.0), Lm((size_t)nd * nd, 0.0);
  for (int32_t i = 0; i < A.n; i++)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; k++)
      for (int d = 0; d < b; d++)
        for (int e = 0; e < b; e++) M[(size_t)(i * b + d) * nd + A.ci[k] * b + e] = A.v[(size_t)k * bb + d * b + e];
  // left-looking Cholesky, column by column, in one parallel region.  spd is
  // written only inside the single and read only after its barrier, so every
  // thread leaves the loop at the same column.
  bool spd = true;
#pragma omp parallel
  for (int32_t j = 0; j < nd; j++) {
#pragma omp single
    {
      double acc = 0.0;
      for (int32_t k = 0; k < j; k++) acc += Lm[(size_t)j * nd + k] * Lm[(size_t)j * nd + k];
      const double d = M[(size_t)j * nd + j] - acc;
      if (!(d > 0.0)) spd = false;
      else Lm[(size_t)j * nd + j] = std::sqrt(d);
    }   // implicit barrier: every thread sees spd and the pivot
    if (!spd) break;
    const double ljj = Lm[(size_t)j * nd + j];
#pragma omp for schedule(static)
    for (int32_t i = j + 1; i < nd; i++) {
      double a2 = 0.0;
      for (int32_t k = 0; k < j; k++) a2 += Lm[(size_t)i * nd + k] * Lm[(size_t)j * nd + k];
      Lm[(size_t)i * nd + j] = (M[(size_t)i * nd + j] - a2) / ljj;
    }
  }
  if (!spd) fail(ASPAMG_ENOT_SPD, "coarsest matrix is not positive definite");
  // X = L^{-1} (lower), column by column; row c of Xt holds column c of X so
  // that both products below read contiguous memory
  std::vector<double> Xt((size_t)nd * nd, 0.0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t c = 0; c < nd; c++) {
    double *xc = Xt.data() + (size_t)c * nd;
    for (int32_t i = c; i < nd; i++) {
      double acc = i == c ? 1.0 : 0.0;
      for (int32_t k = c; k < i; k++) acc -= Lm[(size_t)i * nd + k] * xc[k];
      xc[i] = acc / Lm[(size_t)i * nd + i];
    }
  }
  // inv = X^T X: inv[i][j] = sum over k >= max(i, j) of X[k][i] X[k][j]
  std::vector<double> inv((size_t)nd * nd, 0.0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t i = 0; i < nd; i++)
    for (int32_t j = 0; j <= i; j++) {
      const double *xi = Xt.data() + (size_t)i * nd, *xj = Xt.data() + (size_t)j * nd;
      double s = 0.0;
      for (int32_t k = std::max(i, j); k < nd; k++) s += xi[k] * xj[k];
      inv[(size_t)i * nd + j] = s;
      inv[(size_t)j * nd + i] = s;
    }
  h->coarse.nd = nd;
  h->coarse.inv = upload(h, inv);
}

// M = G^T G for one level, numeric product on the device (the Galerkin
// product's kernel with G^T and G as its operands), kept when its FP32 copy
// is small: there every product costs about one dependent memory round trip,
// so one launch of M replaces the launches of G and G^T in each smoothing step.
void merge_smoother(aspamg_ctx *h, Level &L) {
  const HostBSR GT = transpose(L.G);
  HostBSR M = spgemm_pattern(GT, L.G, false);
  if ((double)M.nnzb() * (4.0 * M.bb() + 2.0) > kMergeMaxBytes) return;   // FP32 values + 16-bit columns
  double *dM = dalloc<double>(h, (size_t)std::max<int64_t>(M.nnzb(), 1) * M.bb());
  {
    DevTmp tmp;
    DevBSR dGT = tmp.make(GT, h->stream, true), dG = tmp.make(L.G, h->stream, true);
    DevBSR dMb = tmp.make(M, h->stream, false);
    dMb.v = dM;
    launch_spgemm_ap(dGT, dG, dMb, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  upload_sell_pair(h, M, dM, L.M64, L.M32);
  dfree(h, dM);
  L.nnzb_M = M.nnzb();
}

}  // namespace

void merge_smoothers(aspamg_ctx *h) {
  const int end = h->tail.level >= 0 ? h->tail.level : (int)h->lev.size() - 1;
  for (int l = 0; l < end; l++) {
    Level &L = h->lev[l];
    if (L.coarsest || L.A.n > kMergeMaxNodes) continue;
    merge_smoother(h, L);
  }
}

// ------------------------------------------------------------------------
// hierarchy driver
// ------------------------------------------------------------------------
void build_hierarchy(aspamg_ctx *h, HostBSR &&A0, std::vector<double> &&V0) {
  PhaseClock clk;
  const aspamg_params &p = h->p;
  const Q q{p.quant_bits};
  const int ntv = h->ntv;
  h->lev.clear();
  h->lev.emplace_back();
  h->lev[0].A = std::move(A0);
  h->lev[0].V = std::move(V0);
  for (int l = 0;; l++) {
    Level &L = h->lev[l];
    const int32_t N = L.A.n;
    L.dA = upload_bsr(h, L.A);
    // lanes per fine row of q = K p; the layouts scatter from the block values of dA
    // the fine level's FP32 residual product streams K at the device's practical
    // rate in the q = K p layout; coarser levels choose a layout for FP32 too
    if (l == 0) {
      L.A64 = upload_sell<double>(h, L.A, kKpLanes, true, L.dA.v);
      L.A32 = derive_fp32(h, L.A64);
    } else {
      upload_sell_pair(h, L.A, L.dA.v, L.A64, L.A32);
    }
    clk.tick(l, "upload A");
    const int b = L.A.b;
    if ((int64_t)N * b <= p.coarse_max_dof || l == p.max_levels - 1 || l == 31 || ntv == 0) {
      L.coarsest = true;
      break;
    }
    build_fsai(h, L);
    clk.tick(l, "aFSAI");
    if (p.n_rq > 0) {
      srqcg(h, L, ntv, p.n_rq);
      clk.tick(l, "test space");
    }
    orthonormalize(L.V, (int64_t)N * b, ntv);
    std::vector<int8_t> excl(N);
    for (int32_t i = 0; i < N; i++) excl[i] = is_decoupled(L.A, i);
    Scratch dexcl((size_t)N), dV(L.V.size() * 8), dcf((size_t)N);
    to_device(h->stream, dexcl.as<int8_t>(), excl.data(), excl.size());
    to_device(h->stream, dV.as<double>(), L.V.data(), L.V.size());
    std::unique_ptr<DevGraph> S = strong_graph_device(h, L, dexcl.as<int8_t>(), dV.as<double>(), ntv);
    mis_device(h, L, *S, dexcl.as<int8_t>(), dcf.as<int8_t>());
    clk.tick(l, "coarsening");
    L.cidx.assign(N, -1);
    int32_t nc = 0, nF = 0;
    for (int32_t i = 0; i < N; i++) {
      if (L.cf[i] == 1) L.cidx[i] = nc++;
      nF += L.cf[i] == 0;
    }
    L.nc = nc;
    if (nc == 0 || nF == 0 || (double)nc > p.stall_ratio * (double)N) {
      L.G = HostBSR();
      L.coarsest = true;
      break;
    }
    build_prolongation(h, L, *S, dcf.as<int8_t>(), dV.as<double>());
    S.reset();
    clk.tick(l, "DPLS");
    HostBSR AP;              // pattern of A P
    double *dPAP = nullptr;  // [P; A P] block values, on the device
    HostBSR Ac = galerkin(h, L, &AP, &dPAP);
    clk.tick(l, "Galerkin");
    // device operators of this level (G and G^T come from build_fsai); the
    // FP32 copies choose their layouts in FP32, where the narrower values
    // shift the balance between the matrix stream and the row reductions
    upload_sell_pair(h, L.P, nullptr, L.P64, L.P32);
    upload_sell_pair(h, transpose(L.P), nullptr, L.R64, L.R32);
    // the stacked [P; A P] replaces the products with P and A of the first
    // post-smoothing step only where it stores no more blocks than A: the
    // interpolation of a rich test space can make A P denser than A
    if (AP.nnzb() <= L.A.nnzb()) {
      L.nnzb_AP = AP.nnzb();
      HostBSR PAP = stack_rows(L.P, AP);
      AP = HostBSR();
      upload_sell_pair(h, PAP, dPAP, L.PAP64, L.PAP32);
    }
    AP = HostBSR();
    dfree(h, dPAP);
    clk.tick(l, "upload G P R");
    std::vector<double> Vc((size_t)nc * b * ntv);
    for (int32_t i = 0; i < N; i++)
      if (L.cidx[i] >= 0)
        std::memcpy(Vc.data() + (size_t)L.cidx[i] * b * ntv, L.V.data() + (size_t)i * b * ntv, b * ntv * sizeof(double));
    h->lev.emplace_back();
    h->lev[l + 1].A = std::move(Ac);
    h->lev[l + 1].V = std::move(Vc);
  }
  build_coarse(h, h->lev.back().A);
  clk.tick((int)h->lev.size() - 1, "coarsest");
}

}  // namespace aspamg
