// noalloc.cpp — qtt_dot_noalloc: the inner product of qtt_dot with its
// scratch (device ranks, result, environments) in a file-scope device
// array instead of a caller workspace, for callers that cannot allocate
// device memory.  The array's device address is looked up once per device
// (hipGetSymbolAddress with that device current) and only that address is
// passed to kernels and copies; the array's name is a host-side stand-in.
#include <mutex>
#include <string>

#include "internal.h"

namespace qtt {
namespace {

constexpr int64_t NOALLOC_DOUBLES = int64_t(1) << 21;   // 16 MiB per device
constexpr int64_t NOALLOC_HEAD = 64;                     // ranks and result

__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on the current device (looked up on the
// first call there).
qtt_status scratch_ptr(double **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(QTT_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(QTT_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(QTT_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = (double *)p;
  }
  *out = g_ptr[dev];
  return QTT_OK;
}

void packed_view_at(const qtt_tt *t, TTView &v, int32_t *rk_dev) {
  v.D = t->ncores;
  int64_t off = 0;
  for (int k = 0; k < t->ncores; ++k) {
    v.n[k] = t->nrow[k];
    v.m[k] = t->ncol ? t->ncol[k] : 1;
    v.off[k] = off;
    off += (int64_t)t->ranks[k] * v.n[k] * v.m[k] * t->ranks[k + 1];
  }
  for (int k = 0; k <= t->ncores; ++k) v.cap[k] = t->ranks[k];
  for (int k = t->ncores; k < QTT_MAXD; ++k) {
    v.n[k] = 1;
    v.m[k] = 1;
    v.off[k] = off;
  }
  v.rk = rk_dev;
  v.data = t->data;
}

}  // namespace
}  // namespace qtt

using namespace qtt;

extern "C" qtt_status qtt_dot_noalloc(const qtt_tt *x, const qtt_tt *y, double *out,
                                      void *stream) {
  qtt::clear_stale_error();
  qtt_status st;
  if ((st = check_tt(x, "x", true)) != QTT_OK) return st;
  if ((st = check_tt(y, "y", true)) != QTT_OK) return st;
  if (!out) return fail(QTT_E_INVAL, "out is NULL");
  if (x->ncores != y->ncores) return fail(QTT_E_SHAPE, "core counts differ");
  for (int k = 0; k < x->ncores; ++k) {
    const int nx = x->nrow[k] * (x->ncol ? x->ncol[k] : 1);
    const int ny = y->nrow[k] * (y->ncol ? y->ncol[k] : 1);
    if (nx != ny) return fail(QTT_E_SHAPE, "modes differ");
  }
  // sizes first (host only), so an oversized request fails before any
  // device call
  TTView vx, vy;
  packed_view_at(x, vx, nullptr);
  packed_view_at(y, vy, nullptr);
  const int64_t we = dot_ws_elems(vx, vy);
  if (NOALLOC_HEAD + we > NOALLOC_DOUBLES)
    return fail(QTT_E_CAPACITY, "qtt_dot_noalloc: the operands need " +
                                    std::to_string(NOALLOC_HEAD + we) +
                                    " doubles of scratch, more than its " +
                                    std::to_string(NOALLOC_DOUBLES));
  double *base = nullptr;
  if ((st = scratch_ptr(&base)) != QTT_OK) return st;
  int32_t *rk = (int32_t *)base;                  // 2 (QTT_MAXD + 1) ints
  double *res = base + NOALLOC_HEAD - 1;
  vx.rk = rk;
  vy.rk = rk + (QTT_MAXD + 1);
  hipStream_t s = (hipStream_t)stream;
  QTT_HIP(upload_ranks(vx, x->ranks, s));
  QTT_HIP(upload_ranks(vy, y->ranks, s));
  QTT_HIP(launch_dot(vx, vy, res, base + NOALLOC_HEAD, we, s));
  QTT_HIP(hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, s));
  QTT_HIP(hipStreamSynchronize(s));
  return QTT_OK;
}
