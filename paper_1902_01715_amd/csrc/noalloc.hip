// Operator application without device allocation, for callers that cannot
// allocate (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc).  The FP32 path of aspamg_apply_operator stages x and y in FP32
// vectors it allocates per call; this variant stages them in a fixed
// per-device array instead.
#include <mutex>

#include "internal.h"

namespace aspamg {

namespace {

// FP32 staging of x and y: 2^23 floats (32 MiB), resident on every device the
// library runs on until the process ends.  In host code the name stands for a
// host-side shadow: kernels get the device address from hipGetSymbolAddress.
constexpr int64_t kScratchFloats = int64_t(1) << 23;
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
float *g_scratch[kMaxDevices] = {};

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace

// Device address of `scratch` on the current device, looked up once per device
// (aspamg_setup calls this with the handle's device current).
float *noalloc_scratch_current_device() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(ASPAMG_EINVAL, "device ordinal beyond the no-allocation scratch table");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch[dev] = static_cast<float *>(p);
  }
  return g_scratch[dev];
}

static float *scratch_for(int dev) {
  if (dev < 0 || dev >= kMaxDevices) fail(ASPAMG_EINVAL, "device ordinal beyond the no-allocation scratch table");
  {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_scratch[dev]) return g_scratch[dev];
  }
  int cur = 0;                          // first call on this device: look it up there
  HIPCHK(hipGetDevice(&cur));
  HIPCHK(hipSetDevice(dev));
  float *p = nullptr;
  try {
    p = noalloc_scratch_current_device();
  } catch (...) {
    (void)hipSetDevice(cur);
    throw;
  }
  HIPCHK(hipSetDevice(cur));
  return p;
}

}  // namespace aspamg

using namespace aspamg;

extern "C" aspamg_status aspamg_apply_operator_noalloc(aspamg_handle h, int32_t level, int32_t which,
                                                       int32_t precision, const double *x_dev, double *y_dev) {
  try {
    if (!h || level < 0 || level >= (int32_t)h->lev.size() || which < 0 || which > 5 ||
        (precision != 32 && precision != 64) || !x_dev || !y_dev)
      fail(ASPAMG_EINVAL, "invalid arguments to aspamg_apply_operator_noalloc");
    const Level &L = h->lev[level];
    if (L.coarsest && which != 0) fail(ASPAMG_EINVAL, "the coarsest level has only A");
    if (which == 5 && L.nnzb_M == 0) fail(ASPAMG_EINVAL, "this level applies G and G^T (no merged G^T G)");
    hipStream_t s = h->stream;
    if (precision == 64) {
      const Sell<double> *M[6] = {&L.A64, &L.G64, &L.GT64, &L.P64, &L.R64, &L.M64};
      launch_spmv<double, double, double>(*M[which], x_dev, y_dev, nullptr, 1.0, nullptr, s);
    } else {
      const Sell<float> *M[6] = {&L.A32, &L.G32, &L.GT32, &L.P32, &L.R32, &L.M32};
      const int64_t nx = (int64_t)M[which]->nc * h->b, ny = (int64_t)M[which]->n * h->b;
      const int64_t need = round_up(nx, 64) + ny;
      if (need > kScratchFloats)
        fail(ASPAMG_EINVAL, "aspamg_apply_operator_noalloc: the operator needs " + std::to_string(need) +
                                " FP32 staging values; the fixed scratch holds " + std::to_string(kScratchFloats));
      float *xs = scratch_for(h->device);
      float *ys = xs + round_up(nx, 64);
      launch_cast<double, float>(nx, x_dev, xs, nullptr, s);
      launch_spmv<float, float, float>(*M[which], xs, ys, nullptr, 1.0, nullptr, s);
      launch_cast<float, double>(ny, ys, y_dev, nullptr, s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return ASPAMG_OK;
  } catch (const Error &e) {
    set_last_error(e.msg);
    return e.code;
  } catch (...) {
    set_last_error("unexpected internal error");
    return ASPAMG_EHIP;
  }
}
