// Solve-phase kernels for gfx950: 3x3-block SpMV on the sliced and row-packed
// layouts with fused epilogues (axpy, the stacked [P; AP] product, the p.q
// partial of the PCG product), the dense coarsest-level product, precision
// casts and the PCG vector updates with deterministic reductions.
//
// All of this work is bound by HBM bandwidth (a 3x3 FP64 block is 18 flops per
// 74 bytes with a 16-bit column offset), so the kernels stream each matrix
// exactly once with fully coalesced 64-lane loads and keep per-row
// accumulators in registers.  Matrix cores are not used.
#include "internal.h"

namespace aspamg {

namespace {

__device__ __forceinline__ bool ctrl_done(const PcgCtrl *c) { return c != nullptr && c->done != 0; }

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).  The
// logical block index below gives every XCD one contiguous range of blocks,
// so neighbouring rows, whose x-gathers overlap, share one L2.
__device__ __forceinline__ int32_t xcd_block() {
  const int32_t nb = gridDim.x, b = blockIdx.x;
  const int32_t x = b & 7, per = nb >> 3, rem = nb & 7;
  return x * per + (x < rem ? x : rem) + (b >> 3);
}

// matrix entries are streamed exactly once per product: keep them out of the
// caches so that the gathered vector stays resident
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }

typedef double wide_f64 __attribute__((ext_vector_type(2)));
typedef float wide_f32 __attribute__((ext_vector_type(4)));

// One slot's 3x3 block times (x0, x1, x2), accumulated into a0..a2; g is the
// slot group (576 values), e the lane.  The first eight values of each lane
// lie in 16-byte chunks, 64 lanes side by side per chunk row: FP64 pairs
// (v0 v1)(v2 v3)(v4 v5)(v6 v7) at 128-entry strides, FP32 quads (v0..v3)(v4..v7)
// at a 256-entry stride; v8 of the 64 lanes follows at 512.
__device__ __forceinline__ void blk_fma(const double *g, int e, double x0, double x1, double x2, double &a0,
                                        double &a1, double &a2) {
  const wide_f64 *p = reinterpret_cast<const wide_f64 *>(g) + e;
  const wide_f64 c0 = __builtin_nontemporal_load(p), c1 = __builtin_nontemporal_load(p + 64),
                 c2 = __builtin_nontemporal_load(p + 128), c3 = __builtin_nontemporal_load(p + 192);
  const double v8 = __builtin_nontemporal_load(g + 512 + e);
  a0 += c0.x * x0 + c0.y * x1 + c1.x * x2;
  a1 += c1.y * x0 + c2.x * x1 + c2.y * x2;
  a2 += c3.x * x0 + c3.y * x1 + v8 * x2;
}
__device__ __forceinline__ void blk_fma(const float *g, int e, float x0, float x1, float x2, float &a0, float &a1,
                                        float &a2) {
  const wide_f32 *p = reinterpret_cast<const wide_f32 *>(g) + e;
  const wide_f32 c0 = __builtin_nontemporal_load(p), c1 = __builtin_nontemporal_load(p + 64);
  const float v8 = __builtin_nontemporal_load(g + 512 + e);
  a0 += c0.x * x0 + c0.y * x1 + c0.z * x2;
  a1 += c0.w * x0 + c1.x * x1 + c1.y * x2;
  a2 += c1.z * x0 + c1.w * x1 + v8 * x2;
}

// Slots per unrolled step of a lane's slot loop: a 3x3 block brings 72 bytes
// (FP64) per gather, a scalar slot 8, so the scalar loop keeps more slots'
// loads in flight per step.
#ifndef ASPAMG_SCALAR_UNROLL
#define ASPAMG_SCALAR_UNROLL 8
#endif
// For 3x3 blocks, 4 instead of 2 measured on the layered block: FP64 cycle
// 2.7% faster, FP32 cycle unchanged, q = K p 1.3% slower; 2 is kept.
#ifndef ASPAMG_BLOCK_UNROLL
#define ASPAMG_BLOCK_UNROLL 2
#endif
template <int B>
constexpr int kSlotUnroll = B == 1 ? ASPAMG_SCALAR_UNROLL : ASPAMG_BLOCK_UNROLL;

// One slot of a b x b block operator applied to the gathered x of column c:
// b = 3, the slot's 3x3 block from its group of 576 values (blk_fma); b = 1,
// the slot's one value at entry e of its group of 64 (scalar CSR).
template <int B, typename T, typename TX>
__device__ __forceinline__ void slot_fma(const T *g, int e, const TX *__restrict__ x, int32_t c, T &a0, T &a1,
                                         T &a2) {
  if constexpr (B == 3) {
    const T x0 = (T)x[3 * c], x1 = (T)x[3 * c + 1], x2 = (T)x[3 * c + 2];
    blk_fma(g, e, x0, x1, x2, a0, a1, a2);
  } else {
    a0 += ld_stream(g + e) * (T)x[c];
  }
}

// Deterministic sum over a 256-thread block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sm[0] + sm[1]) + (sm[2] + sm[3]);
  __syncthreads();
  return r;
}

// y[row] = alpha * (A x)[row] (+ w[row]) on the sliced layout with L lanes per
// block row.  A wavefront owns one slice of 64/L rows; lane e = r*L + j streams
// entry e of every slot group of the slice: 64 consecutive column entries,
// then the group's values in 16-byte chunks (blk_fma).  The L partial sums of
// a row meet in a butterfly and lane j = 0 writes the row.
// With DUAL, rows r >= n1 write y2[r - n1] = alpha2 (A x)[r] + w2[r - n1].
// CI is the stored column type: int32, or uint16 offsets from cbase[slice].
template <typename T, typename TX, typename TO, bool HAS_W, int L, bool DUAL, typename CI, int B>
__global__ void __launch_bounds__(256) k_sell_spmv(int32_t n, const int32_t *__restrict__ sptr,
                                                   const CI *__restrict__ col, const int32_t *__restrict__ cbase,
                                                   const T *__restrict__ val, const TX *__restrict__ x, TO *y,
                                                   const TO *w, T alpha, const PcgCtrl *ctrl, int32_t n1,
                                                   TO *y2, const TO *w2, T alpha2) {
  if (ctrl_done(ctrl)) return;
  const int32_t t = xcd_block() * 256 + threadIdx.x;
  const int32_t sl = t >> 6, e = t & 63;
  const int32_t row = sl * (64 / L) + e / L;
  if (row >= n) return;                 // whole lane groups leave together
  const int32_t g0 = sptr[sl], g1 = sptr[sl + 1];
  const int32_t cb = sizeof(CI) == 2 ? cbase[sl] : 0;
  // The writing lane loads its row of w before the product: the three loads
  // are in flight with the matrix stream instead of each waiting behind the
  // store before it (y and w may be the same vector).
  int32_t orow = row;
  if (DUAL && row >= n1) {
    orow = row - n1;
    y = y2;
    w = w2;
    alpha = alpha2;
  }
  TO w0 = 0, w1 = 0, w2v = 0;
  if (HAS_W && (e & (L - 1)) == 0) {
    const TO *wo = w + B * (size_t)orow;
    w0 = wo[0];
    if constexpr (B == 3) {
      w1 = wo[1];
      w2v = wo[2];
    }
  }
  T a0 = 0, a1 = 0, a2 = 0;
  const CI *cp = col + (size_t)g0 * 64 + e;
  const T *vp = val + (size_t)g0 * 64 * B * B;
  constexpr int UNR = kSlotUnroll<B>;
#pragma unroll UNR
  for (int32_t g = g0; g < g1; ++g) {
    const int32_t c = (int32_t)ld_stream(cp) + cb;
    slot_fma<B>(vp, e, x, c, a0, a1, a2);
    cp += 64;
    vp += 64 * B * B;
  }
  if (L > 1) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) {
      a0 += __shfl_xor(a0, o, L);
      if constexpr (B == 3) {
        a1 += __shfl_xor(a1, o, L);
        a2 += __shfl_xor(a2, o, L);
      }
    }
    if ((e & (L - 1)) != 0) return;
  }
  TO *yo = y + B * (size_t)orow;
  if (HAS_W) {
    yo[0] = (TO)(alpha * a0) + w0;
    if constexpr (B == 3) {
      yo[1] = (TO)(alpha * a1) + w1;
      yo[2] = (TO)(alpha * a2) + w2v;
    }
  } else {
    yo[0] = (TO)(alpha * a0);
    if constexpr (B == 3) {
      yo[1] = (TO)(alpha * a1);
      yo[2] = (TO)(alpha * a2);
    }
  }
}

// The same product on the row-packed layout: every lane streams its K slot
// groups (fully unrolled) and parks its three partial sums in LDS; the first
// lane of each row then adds the row's lanes in lane order and writes the row.
// Rows are packed into units of 64 << ushift lanes (ushift 0: one wavefront,
// 2: the workgroup's four) whose rows start at wrow[unit]; within a unit a
// row's lanes may lie in different wavefronts, and the sums wait for a
// workgroup barrier instead of a wavefront one.
template <typename T, typename TX, typename TO, bool HAS_W, int K, bool DUAL, typename CI, int B>
__global__ void __launch_bounds__(256) k_pack_spmv(int32_t nwaves, int32_t ushift, const int32_t *__restrict__ wrow,
                                                   const uint16_t *__restrict__ meta, const CI *__restrict__ col,
                                                   const int32_t *__restrict__ cbase, const T *__restrict__ val,
                                                   const TX *__restrict__ x, TO *y, const TO *w, T alpha,
                                                   const PcgCtrl *ctrl, int32_t n1, TO *y2, const TO *w2,
                                                   T alpha2) {
  __shared__ T part[B][256];
  if (ctrl_done(ctrl)) return;          // the same for every thread of the grid
  const int32_t t = xcd_block() * 256 + threadIdx.x;
  const int32_t wv = t >> 6, e = t & 63;
  const bool live = wv < nwaves;        // whole wavefronts
  uint32_t m = 0;
  T a0 = 0, a1 = 0, a2 = 0;
  // Every lane of a live wavefront finds the output row of its row (an
  // unused lane has offset 0: the unit's first row) and loads that row of w
  // with the matrix stream.  There is no branch on the metadata, so the
  // stream's loads are issued before the metadata arrives; the lanes of one
  // row load the same addresses.
  int32_t row = 0;
  TO w0 = 0, w1 = 0, w2v = 0;
  if (live) {
    m = meta[(size_t)wv * 64 + e];
    row = wrow[wv >> ushift] + (int32_t)(m & 0xFF);
    if (DUAL) {
      const bool second = row >= n1;
      row = second ? row - n1 : row;
      y = second ? y2 : y;
      w = second ? w2 : w;
      alpha = second ? alpha2 : alpha;
    }
    if (HAS_W) {
      const TO *wo = w + B * (size_t)row;
      w0 = wo[0];
      if constexpr (B == 3) {
        w1 = wo[1];
        w2v = wo[2];
      }
    }
    const int32_t cb = sizeof(CI) == 2 ? cbase[wv] : 0;
    const CI *cp = col + (size_t)wv * K * 64 + e;
    const T *vp = val + (size_t)wv * K * 64 * B * B;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int32_t c = (int32_t)ld_stream(cp + 64 * k) + cb;
      slot_fma<B>(vp + 64 * B * B * k, e, x, c, a0, a1, a2);
    }
  }
  part[0][threadIdx.x] = a0;
  if constexpr (B == 3) {
    part[1][threadIdx.x] = a1;
    part[2][threadIdx.x] = a2;
  }
  if (ushift == 0) {
    // the lanes of a row never leave their wavefront, whose LDS operations
    // complete in order: a wavefront-scope barrier suffices
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();                    // ushift is the same for the whole grid
  }
  const int cnt = (int)(m >> 8);
  if (!live || cnt == 0) return;
  T s0 = 0, s1 = 0, s2 = 0;
  for (int j = 0; j < cnt; ++j) {       // lanes of one row never leave their unit
    s0 += part[0][threadIdx.x + j];
    if constexpr (B == 3) {
      s1 += part[1][threadIdx.x + j];
      s2 += part[2][threadIdx.x + j];
    }
  }
  TO *yo = y + B * (size_t)row;
  if (HAS_W) {
    yo[0] = (TO)(alpha * s0) + w0;
    if constexpr (B == 3) {
      yo[1] = (TO)(alpha * s1) + w1;
      yo[2] = (TO)(alpha * s2) + w2v;
    }
  } else {
    yo[0] = (TO)(alpha * s0);
    if constexpr (B == 3) {
      yo[1] = (TO)(alpha * s1);
      yo[2] = (TO)(alpha * s2);
    }
  }
}

// q = K p with the block partial of p.q (PCG, FP64).
// Deterministic sum over an NT-thread block (NT = 256, 512 or 1024); the
// result is valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum_n(double v, double *sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    constexpr int nw = NT / 64;
    double h[nw / 4];
    for (int q = 0; q < nw / 4; q++) h[q] = (sm[4 * q] + sm[4 * q + 1]) + (sm[4 * q + 2] + sm[4 * q + 3]);
    for (int q = 0; q < nw / 4; q++) r += h[q];
  }
  __syncthreads();
  return r;
}

// q = K p on the sliced layout with L lanes per row, and the p.q partial of
// every kDotThreads-thread block.  Block b serves the `per` consecutive groups
// of kDotThreads lanes b*per .. b*per+per-1 (per = 1 up to kMaxPart blocks; a
// larger operator keeps kMaxPart partials and gives each block more rows).
template <typename CI, int L, int B>
__global__ void __launch_bounds__(kDotThreads) k_sell_spmv_dot(int32_t n, const int32_t *__restrict__ sptr,
                                                        const CI *__restrict__ col,
                                                        const int32_t *__restrict__ cbase,
                                                        const double *__restrict__ val,
                                                        const double *__restrict__ x, double *__restrict__ y,
                                                        double *__restrict__ part, const PcgCtrl *ctrl,
                                                        int32_t per) {
  __shared__ double sm[kDotThreads / 64];
  if (ctrl_done(ctrl)) return;
  double d = 0.0;
  for (int32_t it = 0; it < per; ++it) {
    const int32_t t = (xcd_block() * per + it) * kDotThreads + threadIdx.x;
    const int32_t sl = t >> 6, e = t & 63;
    const int32_t row = sl * (64 / L) + e / L;
    if (row < n) {                        // whole lane groups together
      const int32_t g0 = sptr[sl], g1 = sptr[sl + 1];
      const int32_t cb = sizeof(CI) == 2 ? cbase[sl] : 0;
      double a0 = 0, a1 = 0, a2 = 0;
      // the row's own p, for the dot, is loaded with the matrix stream
      double p0 = 0, p1 = 0, p2 = 0;
      if ((e & (L - 1)) == 0) {
        const double *xo = x + B * (size_t)row;
        p0 = xo[0];
        if constexpr (B == 3) {
          p1 = xo[1];
          p2 = xo[2];
        }
      }
      const CI *cp = col + (size_t)g0 * 64 + e;
      const double *vp = val + (size_t)g0 * 64 * B * B;
      constexpr int UNR = kSlotUnroll<B>;
#pragma unroll UNR
      for (int32_t g = g0; g < g1; ++g) {
        const int32_t c = (int32_t)ld_stream(cp) + cb;
        slot_fma<B>(vp, e, x, c, a0, a1, a2);
        cp += 64;
        vp += 64 * B * B;
      }
      if (L > 1) {
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) {
          a0 += __shfl_xor(a0, o, L);
          if constexpr (B == 3) {
            a1 += __shfl_xor(a1, o, L);
            a2 += __shfl_xor(a2, o, L);
          }
        }
      }
      if ((e & (L - 1)) == 0) {
        double *yo = y + B * (size_t)row;
        yo[0] = a0;
        if constexpr (B == 3) {
          yo[1] = a1;
          yo[2] = a2;
          d += (p0 * a0 + p1 * a1) + p2 * a2;
        } else {
          d += p0 * a0;
        }
      }
    }
  }
  const double s = block_sum_n<kDotThreads>(d, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Rounding floor of the recomputed residual: per scalar row
// s_i = |f_i| + sum_j |K_ij| |u_j| (the componentwise bound of evaluating
// f - K u, Higham, "Accuracy and Stability of Numerical Algorithms", Sec. 3.5),
// and the block partials of sum s_i^2.  Same layout and row mapping as
// k_sell_spmv_dot.
template <typename CI, int L, int B>
__global__ void __launch_bounds__(kDotThreads) k_sell_abs_bound(int32_t n, const int32_t *__restrict__ sptr,
                                                         const CI *__restrict__ col,
                                                         const int32_t *__restrict__ cbase,
                                                         const double *__restrict__ val,
                                                         const double *__restrict__ u, const double *__restrict__ f,
                                                         double *__restrict__ part, int32_t per) {
  __shared__ double sm[kDotThreads / 64];
  double d = 0.0;
  for (int32_t it = 0; it < per; ++it) {
    const int32_t t = (xcd_block() * per + it) * kDotThreads + threadIdx.x;
    const int32_t sl = t >> 6, e = t & 63;
    const int32_t row = sl * (64 / L) + e / L;
    if (row >= n) continue;
    const int32_t g0 = sptr[sl], g1 = sptr[sl + 1];
    const int32_t cb = sizeof(CI) == 2 ? cbase[sl] : 0;
    double a0 = 0, a1 = 0, a2 = 0;
    for (int32_t g = g0; g < g1; ++g) {
      const int32_t c = (int32_t)col[(size_t)g * 64 + e] + cb;
      if constexpr (B == 3) {
        const double x0 = fabs(u[3 * c]), x1 = fabs(u[3 * c + 1]), x2 = fabs(u[3 * c + 2]);
        const wide_f64 *p = reinterpret_cast<const wide_f64 *>(val + (size_t)g * 576) + e;
        const wide_f64 c0 = p[0], c1 = p[64], c2 = p[128], c3 = p[192];
        const double v8 = val[(size_t)g * 576 + 512 + e];
        a0 += fabs(c0.x) * x0 + fabs(c0.y) * x1 + fabs(c1.x) * x2;
        a1 += fabs(c1.y) * x0 + fabs(c2.x) * x1 + fabs(c2.y) * x2;
        a2 += fabs(c3.x) * x0 + fabs(c3.y) * x1 + fabs(v8) * x2;
      } else {
        a0 += fabs(val[(size_t)g * 64 + e]) * fabs(u[c]);
      }
    }
    if (L > 1) {
#pragma unroll
      for (int o = L / 2; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o, L);
        if constexpr (B == 3) {
          a1 += __shfl_xor(a1, o, L);
          a2 += __shfl_xor(a2, o, L);
        }
      }
    }
    if ((e & (L - 1)) == 0) {
      const double *fo = f + B * (size_t)row;
      if constexpr (B == 3) {
        const double s0 = fabs(fo[0]) + a0, s1 = fabs(fo[1]) + a1, s2 = fabs(fo[2]) + a2;
        d += (s0 * s0 + s1 * s1) + s2 * s2;
      } else {
        const double s0 = fabs(fo[0]) + a0;
        d += s0 * s0;
      }
    }
  }
  const double s = block_sum_n<kDotThreads>(d, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// z = D y for a dense row-major FP64 operator (the coarsest inverse, or the
// dense tail of the V-cycle): one wavefront per row, four independent partial
// sums per lane so that four 512-byte row segments are in flight, the matrix
// streamed past the caches (y stays resident).
template <typename TV>
__global__ void __launch_bounds__(256) k_dense_gemv(int32_t nd, const double *__restrict__ inv,
                                                    const TV *__restrict__ y, TV *__restrict__ z,
                                                    const PcgCtrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  const int32_t row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nd) return;
  const double *a = inv + (size_t)row * nd;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int32_t j = lane;
  for (; j + 192 < nd; j += 256) {
    s0 += ld_stream(a + j) * (double)y[j];
    s1 += ld_stream(a + j + 64) * (double)y[j + 64];
    s2 += ld_stream(a + j + 128) * (double)y[j + 128];
    s3 += ld_stream(a + j + 192) * (double)y[j + 192];
  }
  for (; j < nd; j += 64) s0 += ld_stream(a + j) * (double)y[j];
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) z[row] = (TV)s;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_cast(int64_t n, const TI *__restrict__ x, TO *__restrict__ y,
                                              const PcgCtrl *ctrl) {
  if (ctrl_done(ctrl)) return;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = (TO)x[i];
}

__global__ void __launch_bounds__(256) k_fill(int64_t n, double *__restrict__ x, double v) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] = v;
}

__global__ void __launch_bounds__(256) k_copy(int64_t n, const double *__restrict__ x, double *__restrict__ y) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = x[i];
}

__global__ void __launch_bounds__(256) k_dot(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                                             double *__restrict__ part, const PcgCtrl *ctrl) {
  __shared__ double sm[4];
  if (ctrl_done(ctrl)) return;
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += a[i] * b[i];
  s = block_sum(s, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// u += alpha p, r -= alpha q; partials of r.r and r.z (z = previous preconditioned residual).
// Fixed-order sum of np partials, the same in every block and returned to
// every thread of the block.
__device__ __forceinline__ double sum_parts(const double *part, int np, double *sm) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  return block_sum(s, sm);
}
__device__ __forceinline__ double sum_parts_all(const double *part, int np, double *sm, double *bc) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  s = block_sum(s, sm);
  if (threadIdx.x == 0) *bc = s;
  __syncthreads();
  return *bc;
}

// One PCG step on the iterate: alpha = rz_k / p.q (every block reduces the
// product's partials itself, in the same order), u += alpha p, r -= alpha q,
// and the partials of r.r and r.z_old (Polak-Ribiere); with rc, r is also
// written in the cycle precision.  A non-positive p.q ends the solve.
template <typename TC>
__global__ void __launch_bounds__(256) k_pcg_update(int64_t n, double *__restrict__ u, double *__restrict__ r,
                                                    const double *__restrict__ p, const double *__restrict__ q,
                                                    const TC *__restrict__ z, const double *__restrict__ pq_part,
                                                    int npq, double *__restrict__ part, TC *__restrict__ rc,
                                                    PcgCtrl *ctrl) {
  __shared__ double sm[4], bc;
  if (ctrl_done(ctrl)) return;
  const int32_t it = ctrl->iter;
  const double rz = ctrl->rzk[it & 1];
  const double pq = sum_parts_all(pq_part, npq, sm, &bc);
  if (!(pq > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctrl->pq = pq;
      ctrl->status = (pq == pq) ? ASPAMG_EBREAKDOWN : ASPAMG_ENAN;
      ctrl->iter = it + 1;
      ctrl->done = 1;
    }
    return;
  }
  const double alpha = rz / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->pq = pq;
    ctrl->alpha = alpha;
  }
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    u[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (rc) rc[i] = (TC)ri;
    s1 += ri * ri;
    s2 += ri * (double)z[i];
  }
  s1 = block_sum(s1, sm);
  s2 = block_sum(s2, sm);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[kMaxPart + blockIdx.x] = s2;
  }
}

// Convergence test after the update of iterate k + 1 (one thread): r.r and
// r.z_old from their block partials, the iteration count and the stop flag.
__device__ void finish_iteration(PcgCtrl *ctrl, double rr, double rzo) {
  ctrl->rr = rr;
  ctrl->rzo = rzo;
  ctrl->iter += 1;
  const double nr = sqrt(rr);
  ctrl->relres = nr / ctrl->fnorm;
  if (!(rr == rr) || rr == __builtin_inf()) { ctrl->status = ASPAMG_ENAN; ctrl->done = 1; }
  else if (nr <= ctrl->rtol * ctrl->fnorm) { ctrl->status = ASPAMG_OK; ctrl->done = 1; }
  else if (ctrl->iter >= ctrl->max_it) { ctrl->status = ASPAMG_NOT_CONVERGED; ctrl->done = 1; }
}

// Partials of r.z for the cycle output z (in the cycle precision).  Block 0
// also runs the convergence test on the r.r and r.z_old partials that the
// update left (it is the only writer of the flag in this launch, and the
// other blocks do not read it: their partials are unused once it is set).
template <typename TZ>
__global__ void __launch_bounds__(256) k_pcg_rz(int64_t n, const double *__restrict__ r, const TZ *__restrict__ z,
                                                double *__restrict__ part, const double *__restrict__ rr_part,
                                                int nrr, PcgCtrl *ctrl) {
  __shared__ double sm[4];
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += r[i] * (double)z[i];
  s = block_sum(s, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
  if (blockIdx.x != 0 || ctrl->done) return;     // uniform within block 0
  const double rr = sum_parts(rr_part, nrr, sm);
  const double rzo = sum_parts(rr_part + kMaxPart, nrr, sm);
  if (threadIdx.x == 0) finish_iteration(ctrl, rr, rzo);
}

// p = z + beta p with beta = (r.z - r.z_old) / rz_k (Polak-Ribiere); every
// block reduces the r.z partials itself, and block 0 keeps r.z as rz_{k+1}
// in the slot of the next iteration (the other slot is the one read here).
// A non-positive r.z ends the solve.
template <typename TZ>
__global__ void __launch_bounds__(256) k_pcg_pupdate(int64_t n, const TZ *__restrict__ z, double *__restrict__ p,
                                                     const double *__restrict__ rz_part, int nrz, PcgCtrl *ctrl) {
  __shared__ double sm[4], bc;
  if (ctrl_done(ctrl)) return;
  const int32_t it = ctrl->iter;        // already k + 1
  const double rz_old = ctrl->rzk[(it - 1) & 1], rzo = ctrl->rzo;
  const double rz = sum_parts_all(rz_part, nrz, sm, &bc);
  if (!(rz > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctrl->status = (rz == rz) ? ASPAMG_EBREAKDOWN : ASPAMG_ENAN;
      ctrl->done = 1;
    }
    return;
  }
  const double beta = (rz - rzo) / rz_old;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->rzk[it & 1] = rz;
    ctrl->rz = rz;
    ctrl->beta = beta;
  }
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = (double)z[i] + beta * p[i];
}


// Scalar steps of PCG, one block: fixed-order reductions of the partials.
__global__ void __launch_bounds__(256) k_finish(int mode, const double *__restrict__ part, int np, PcgCtrl *ctrl) {
  __shared__ double sm[4];
  if (ctrl->done) return;
  const double s0 = sum_parts(part, np, sm);
  if (threadIdx.x != 0) return;
  switch (mode) {
    case kFinInitF: {
      ctrl->fnorm = sqrt(s0);
      ctrl->iter = 0;
      ctrl->relres = 1.0;
      if (!(s0 == s0) || s0 == __builtin_inf()) { ctrl->status = ASPAMG_ENAN; ctrl->done = 1; }
      else if (s0 == 0.0) { ctrl->status = ASPAMG_OK; ctrl->relres = 0.0; ctrl->done = 1; }
      break;
    }
    case kFinInitRz: {
      ctrl->rz = s0;
      ctrl->rzk[0] = s0;
      if (!(s0 > 0.0)) { ctrl->status = (s0 == s0) ? ASPAMG_EBREAKDOWN : ASPAMG_ENAN; ctrl->done = 1; }
      break;
    }
    case kFinNorm: {
      ctrl->rr = s0;
      break;
    }
  }
}

}  // namespace

int vec_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T, typename TX, typename TO, bool HAS_W, int L, bool DUAL, int B>
static void launch_lb(const Sell<T> &A, const TX *x, TO *y, const TO *w, double alpha, const PcgCtrl *ctrl,
                      hipStream_t s, int32_t n1, TO *y2, const TO *w2, double alpha2) {
  const int64_t threads = (int64_t)A.nslices * 64;
  const dim3 grid((unsigned)((threads + 255) / 256));
  if (A.col16)
    hipLaunchKernelGGL((k_sell_spmv<T, TX, TO, HAS_W, L, DUAL, uint16_t, B>), grid, dim3(256), 0, s, A.n, A.sptr,
                       A.col16, A.cbase, A.val, x, y, w, (T)alpha, ctrl, n1, y2, w2, (T)alpha2);
  else
    hipLaunchKernelGGL((k_sell_spmv<T, TX, TO, HAS_W, L, DUAL, int32_t, B>), grid, dim3(256), 0, s, A.n, A.sptr,
                       A.col, nullptr, A.val, x, y, w, (T)alpha, ctrl, n1, y2, w2, (T)alpha2);
}
// the operator's block size picks the kernel: 3 (nodal blocks) or 1 (scalar)
template <typename T, typename TX, typename TO, bool HAS_W, int L, bool DUAL = false>
static void launch_l(const Sell<T> &A, const TX *x, TO *y, const TO *w, double alpha, const PcgCtrl *ctrl,
                     hipStream_t s, int32_t n1 = 0, TO *y2 = nullptr, const TO *w2 = nullptr, double alpha2 = 0) {
  if (A.b == 1) launch_lb<T, TX, TO, HAS_W, L, DUAL, 1>(A, x, y, w, alpha, ctrl, s, n1, y2, w2, alpha2);
  else launch_lb<T, TX, TO, HAS_W, L, DUAL, 3>(A, x, y, w, alpha, ctrl, s, n1, y2, w2, alpha2);
}

template <typename T, typename TX, typename TO, bool HAS_W>
static void launch_spmv_w(const Sell<T> &A, const TX *x, TO *y, const TO *w, double alpha, const PcgCtrl *ctrl,
                          hipStream_t s) {
  switch (A.lanes) {
    case 1: launch_l<T, TX, TO, HAS_W, 1>(A, x, y, w, alpha, ctrl, s); break;
    case 2: launch_l<T, TX, TO, HAS_W, 2>(A, x, y, w, alpha, ctrl, s); break;
    case 4: launch_l<T, TX, TO, HAS_W, 4>(A, x, y, w, alpha, ctrl, s); break;
    case 8: launch_l<T, TX, TO, HAS_W, 8>(A, x, y, w, alpha, ctrl, s); break;
    case 16: launch_l<T, TX, TO, HAS_W, 16>(A, x, y, w, alpha, ctrl, s); break;
    case 32: launch_l<T, TX, TO, HAS_W, 32>(A, x, y, w, alpha, ctrl, s); break;
    default: launch_l<T, TX, TO, HAS_W, 64>(A, x, y, w, alpha, ctrl, s); break;
  }
}

template <typename T, typename TX, typename TO, bool HAS_W, int K, bool DUAL, int B>
static void launch_kb(const Sell<T> &A, const TX *x, TO *y, const TO *w, double alpha, const PcgCtrl *ctrl,
                      hipStream_t s, int32_t n1, TO *y2, const TO *w2, double alpha2) {
  // units of one wavefront (ushift 0) or of the workgroup's four (ushift 2),
  // which then fill whole workgroups
  const int ushift = A.unit == 256 ? 2 : 0;
  if ((A.unit != 64 && A.unit != 256) || (ushift == 2 && A.nslices % 4 != 0))
    fail(ASPAMG_EINVAL, "row-packed layout with an unsupported packing unit");
  const dim3 grid((unsigned)((A.nslices + 3) / 4));
  if (A.col16)
    hipLaunchKernelGGL((k_pack_spmv<T, TX, TO, HAS_W, K, DUAL, uint16_t, B>), grid, dim3(256), 0, s, A.nslices,
                       ushift, A.sptr, A.meta, A.col16, A.cbase, A.val, x, y, w, (T)alpha, ctrl, n1, y2, w2, (T)alpha2);
  else
    hipLaunchKernelGGL((k_pack_spmv<T, TX, TO, HAS_W, K, DUAL, int32_t, B>), grid, dim3(256), 0, s, A.nslices,
                       ushift, A.sptr, A.meta, A.col, nullptr, A.val, x, y, w, (T)alpha, ctrl, n1, y2, w2, (T)alpha2);
}
template <typename T, typename TX, typename TO, bool HAS_W, int K, bool DUAL = false>
static void launch_k(const Sell<T> &A, const TX *x, TO *y, const TO *w, double alpha, const PcgCtrl *ctrl,
                     hipStream_t s, int32_t n1 = 0, TO *y2 = nullptr, const TO *w2 = nullptr, double alpha2 = 0) {
  if (A.b == 1) launch_kb<T, TX, TO, HAS_W, K, DUAL, 1>(A, x, y, w, alpha, ctrl, s, n1, y2, w2, alpha2);
  else launch_kb<T, TX, TO, HAS_W, K, DUAL, 3>(A, x, y, w, alpha, ctrl, s, n1, y2, w2, alpha2);
}

template <typename T, typename TX, typename TO, bool HAS_W>
static void launch_pack_w(const Sell<T> &A, const TX *x, TO *y, const TO *w, double alpha, const PcgCtrl *ctrl,
                          hipStream_t s) {
  switch (A.pack) {
    case 1: launch_k<T, TX, TO, HAS_W, 1>(A, x, y, w, alpha, ctrl, s); break;
    case 2: launch_k<T, TX, TO, HAS_W, 2>(A, x, y, w, alpha, ctrl, s); break;
    case 4: launch_k<T, TX, TO, HAS_W, 4>(A, x, y, w, alpha, ctrl, s); break;
    case 8: launch_k<T, TX, TO, HAS_W, 8>(A, x, y, w, alpha, ctrl, s); break;
    default: fail(ASPAMG_EINVAL, "row-packed layout with an unsupported group count");
  }
}

template <typename T, typename TX, typename TO>
void launch_spmv(const Sell<T> &A, const TX *x, TO *y, const TO *w, double alpha, const PcgCtrl *ctrl,
                 hipStream_t s) {
  if (A.n == 0) return;
  if (A.pack) {
    if (w) launch_pack_w<T, TX, TO, true>(A, x, y, w, alpha, ctrl, s);
    else launch_pack_w<T, TX, TO, false>(A, x, y, w, alpha, ctrl, s);
    return;
  }
  if (w) launch_spmv_w<T, TX, TO, true>(A, x, y, w, alpha, ctrl, s);
  else launch_spmv_w<T, TX, TO, false>(A, x, y, w, alpha, ctrl, s);
}

template <typename T, typename TX, typename TO>
void launch_spmv_dual(const Sell<T> &A, int32_t n1, const TX *x, TO *y1, const TO *w1, double a1, TO *y2,
                      const TO *w2, double a2, const PcgCtrl *ctrl, hipStream_t s) {
  if (A.n == 0) return;
  if (!w1 || !w2 || n1 < 0 || n1 > A.n) fail(ASPAMG_EINVAL, "stacked product needs both addends and 0 <= n1 <= n");
#define DUAL_ARGS A, x, y1, w1, a1, ctrl, s, n1, y2, w2, a2
  if (A.pack) {
    switch (A.pack) {
      case 1: launch_k<T, TX, TO, true, 1, true>(DUAL_ARGS); break;
      case 2: launch_k<T, TX, TO, true, 2, true>(DUAL_ARGS); break;
      case 4: launch_k<T, TX, TO, true, 4, true>(DUAL_ARGS); break;
      case 8: launch_k<T, TX, TO, true, 8, true>(DUAL_ARGS); break;
      default: fail(ASPAMG_EINVAL, "row-packed layout with an unsupported group count");
    }
  } else {
    switch (A.lanes) {
      case 1: launch_l<T, TX, TO, true, 1, true>(DUAL_ARGS); break;
      case 2: launch_l<T, TX, TO, true, 2, true>(DUAL_ARGS); break;
      case 4: launch_l<T, TX, TO, true, 4, true>(DUAL_ARGS); break;
      case 8: launch_l<T, TX, TO, true, 8, true>(DUAL_ARGS); break;
      case 16: launch_l<T, TX, TO, true, 16, true>(DUAL_ARGS); break;
      case 32: launch_l<T, TX, TO, true, 32, true>(DUAL_ARGS); break;
      default: launch_l<T, TX, TO, true, 64, true>(DUAL_ARGS); break;
    }
  }
#undef DUAL_ARGS
}
template void launch_spmv_dual<double, double, double>(const Sell<double> &, int32_t, const double *, double *,
                                                       const double *, double, double *, const double *, double,
                                                       const PcgCtrl *, hipStream_t);
template void launch_spmv_dual<float, float, float>(const Sell<float> &, int32_t, const float *, float *,
                                                    const float *, double, float *, const float *, double,
                                                    const PcgCtrl *, hipStream_t);

template void launch_spmv<double, double, double>(const Sell<double> &, const double *, double *, const double *,
                                                  double, const PcgCtrl *, hipStream_t);
template void launch_spmv<float, float, float>(const Sell<float> &, const float *, float *, const float *, double,
                                               const PcgCtrl *, hipStream_t);

// groups of kDotThreads lanes of the sliced operator, and the groups each
// block of the fused product serves so that at most kMaxPart blocks run
static int64_t dot_groups(const Sell<double> &A) {
  return ((int64_t)A.nslices * 64 + kDotThreads - 1) / kDotThreads;
}
static int32_t dot_per_block(const Sell<double> &A) {
  return (int32_t)((dot_groups(A) + kMaxPart - 1) / kMaxPart);
}
int spmv_dot_blocks(const Sell<double> &A) {
  const int64_t per = dot_per_block(A);
  return (int)((dot_groups(A) + per - 1) / per);
}

template <int L, int B>
static void launch_dot_lb(const Sell<double> &A, const double *x, double *y, double *part, const PcgCtrl *ctrl,
                          hipStream_t s) {
  const dim3 grid((unsigned)spmv_dot_blocks(A));
  const int32_t per = dot_per_block(A);
  if (A.col16)
    hipLaunchKernelGGL((k_sell_spmv_dot<uint16_t, L, B>), grid, dim3(kDotThreads), 0, s, A.n, A.sptr, A.col16,
                       A.cbase, A.val, x, y, part, ctrl, per);
  else
    hipLaunchKernelGGL((k_sell_spmv_dot<int32_t, L, B>), grid, dim3(kDotThreads), 0, s, A.n, A.sptr, A.col, nullptr,
                       A.val, x, y, part, ctrl, per);
}
template <int L>
static void launch_dot_l(const Sell<double> &A, const double *x, double *y, double *part, const PcgCtrl *ctrl,
                         hipStream_t s) {
  if (A.b == 1) launch_dot_lb<L, 1>(A, x, y, part, ctrl, s);
  else launch_dot_lb<L, 3>(A, x, y, part, ctrl, s);
}

void launch_spmv_dot(const Sell<double> &A, const double *x, double *y, double *part, const PcgCtrl *ctrl,
                     hipStream_t s) {
  if (A.pack) fail(ASPAMG_EINVAL, "q = K p needs the sliced layout");
  switch (A.lanes) {
    case 1: launch_dot_l<1>(A, x, y, part, ctrl, s); break;
    case 2: launch_dot_l<2>(A, x, y, part, ctrl, s); break;
    case 4: launch_dot_l<4>(A, x, y, part, ctrl, s); break;
    default: fail(ASPAMG_EINVAL, "q = K p supports 1, 2 or 4 lanes per row");
  }
}

template <int L, int B>
static void launch_abs_lb(const Sell<double> &A, const double *u, const double *f, double *part, hipStream_t s) {
  const dim3 grid((unsigned)spmv_dot_blocks(A));
  const int32_t per = dot_per_block(A);
  if (A.col16)
    hipLaunchKernelGGL((k_sell_abs_bound<uint16_t, L, B>), grid, dim3(kDotThreads), 0, s, A.n, A.sptr, A.col16,
                       A.cbase, A.val, u, f, part, per);
  else
    hipLaunchKernelGGL((k_sell_abs_bound<int32_t, L, B>), grid, dim3(kDotThreads), 0, s, A.n, A.sptr, A.col, nullptr,
                       A.val, u, f, part, per);
}
template <int L>
static void launch_abs_l(const Sell<double> &A, const double *u, const double *f, double *part, hipStream_t s) {
  if (A.b == 1) launch_abs_lb<L, 1>(A, u, f, part, s);
  else launch_abs_lb<L, 3>(A, u, f, part, s);
}

void launch_abs_bound(const Sell<double> &A, const double *u, const double *f, double *part, hipStream_t s) {
  if (A.pack) fail(ASPAMG_EINVAL, "residual bound needs the sliced layout of K");
  switch (A.lanes) {
    case 1: launch_abs_l<1>(A, u, f, part, s); break;
    case 2: launch_abs_l<2>(A, u, f, part, s); break;
    case 4: launch_abs_l<4>(A, u, f, part, s); break;
    default: fail(ASPAMG_EINVAL, "residual bound supports 1, 2 or 4 lanes per row");
  }
}

template <typename TV>
void launch_dense_gemv(int nd, const double *inv, const TV *y, TV *z, const PcgCtrl *ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_gemv<TV>, dim3((nd + 3) / 4), dim3(256), 0, s, nd, inv, y, z, ctrl);
}
template void launch_dense_gemv<double>(int, const double *, const double *, double *, const PcgCtrl *, hipStream_t);
template void launch_dense_gemv<float>(int, const double *, const float *, float *, const PcgCtrl *, hipStream_t);

template <typename TI, typename TO>
void launch_cast(int64_t n, const TI *x, TO *y, const PcgCtrl *ctrl, hipStream_t s) {
  hipLaunchKernelGGL((k_cast<TI, TO>), dim3(vec_blocks(n)), dim3(256), 0, s, n, x, y, ctrl);
}
template void launch_cast<double, float>(int64_t, const double *, float *, const PcgCtrl *, hipStream_t);
template void launch_cast<float, double>(int64_t, const float *, double *, const PcgCtrl *, hipStream_t);

void launch_fill(int64_t n, double *x, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(vec_blocks(n)), dim3(256), 0, s, n, x, v);
}
void launch_copy(int64_t n, const double *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(vec_blocks(n)), dim3(256), 0, s, n, x, y);
}
void launch_dot(int64_t n, const double *a, const double *b, double *part, const PcgCtrl *ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(vec_blocks(n)), dim3(256), 0, s, n, a, b, part, ctrl);
}
template <typename TC>
void launch_pcg_update(int64_t n, double *u, double *r, const double *p, const double *q, const TC *z,
                       const double *pq_part, int npq, double *part, TC *rc, PcgCtrl *ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_update<TC>, dim3(vec_blocks(n)), dim3(256), 0, s, n, u, r, p, q, z, pq_part, npq, part, rc,
                     ctrl);
}
template void launch_pcg_update<float>(int64_t, double *, double *, const double *, const double *, const float *,
                                       const double *, int, double *, float *, PcgCtrl *, hipStream_t);
template void launch_pcg_update<double>(int64_t, double *, double *, const double *, const double *, const double *,
                                        const double *, int, double *, double *, PcgCtrl *, hipStream_t);
template <typename TZ>
void launch_pcg_rz(int64_t n, const double *r, const TZ *z, double *part, const double *rr_part, int nrr,
                   PcgCtrl *ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_rz<TZ>, dim3(vec_blocks(n)), dim3(256), 0, s, n, r, z, part, rr_part, nrr, ctrl);
}
template void launch_pcg_rz<double>(int64_t, const double *, const double *, double *, const double *, int, PcgCtrl *,
                                    hipStream_t);
template void launch_pcg_rz<float>(int64_t, const double *, const float *, double *, const double *, int, PcgCtrl *,
                                   hipStream_t);
template <typename TZ>
void launch_pcg_pupdate(int64_t n, const TZ *z, double *p, const double *rz_part, int nrz, PcgCtrl *ctrl,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_pupdate<TZ>, dim3(vec_blocks(n)), dim3(256), 0, s, n, z, p, rz_part, nrz, ctrl);
}
template void launch_pcg_pupdate<double>(int64_t, const double *, double *, const double *, int, PcgCtrl *,
                                         hipStream_t);
template void launch_pcg_pupdate<float>(int64_t, const float *, double *, const double *, int, PcgCtrl *,
                                        hipStream_t);
void launch_finish(int mode, const double *part, int nparts, PcgCtrl *ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, mode, part, nparts, ctrl);
}

}  // namespace aspamg
