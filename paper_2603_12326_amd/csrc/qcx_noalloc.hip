// Inversion of caller-supplied dielectric matrices without any device
// allocation, for callers that cannot allocate (code under graph capture,
// serving loops, harnesses that forbid hipMalloc): the working copy of eps
// (the Gauss-Jordan kernels overwrite their matrices) and, when the caller
// passes no diag_out, the diagonal of the inverse live in one file-scope
// device array of fixed size.  Each GPU holds its own copy of the array until
// the process ends; its address on a device is looked up once, with that
// device current, when the first context is created there (noalloc_init).
// Frequencies are processed in chunks that fit the array.  Every call on a
// device shares that device's array: calls that overlap on one GPU (two
// streams, two contexts) race.
#include <mutex>

#include "ctx.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per device
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

namespace qcx {

hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  // the caller has made `device` current; the symbol's address differs per device
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

}  // namespace qcx

extern "C" {

int qcx_eps_inv_given_noalloc(qcx_ctx* ctx, int n_w, int n_G, const void* eps, int lfe,
                              double* loss_out, void* diag_out, void* epsM_out, int* status_out) {
  if (!ctx) return QCX_EINVAL;
  if (n_w < 1 || n_w > 65536) return fail(ctx, QCX_EINVAL, "need 1 <= n_w <= 65536");
  if (n_G < 1 || n_G > (lfe ? 1024 : 65536))
    return fail(ctx, QCX_EINVAL, lfe ? "need 1 <= n_G <= 1024" : "need 1 <= n_G <= 65536");
  if (!eps || !loss_out || !status_out)
    return fail(ctx, QCX_EINVAL, "eps, loss_out and status_out must be device buffers");
  const size_t n = (size_t)n_G;
  // scratch bytes per frequency: the working copy (LFE only) and the diagonal
  const size_t per_w = sizeof(cplx) * ((lfe ? n * n : 0) + (diag_out ? 0 : n));
  if (per_w > kScratchBytes)
    return fail(ctx, QCX_EINVAL, "one frequency needs more than the 64 MiB scratch (pass diag_out)");
  if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_scratch_ptr[ctx->device])
    return fail(ctx, QCX_EDEVICE, "scratch address of this device unknown");
  HIPCK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  char* base = static_cast<char*>(g_scratch_ptr[ctx->device]);
  const int chunk = per_w == 0 ? n_w : (int)std::min<size_t>(n_w, kScratchBytes / per_w);
  cplx* work = reinterpret_cast<cplx*>(base);
  cplx* dscr = reinterpret_cast<cplx*>(base + (lfe ? sizeof(cplx) * n * n * chunk : 0));
  const cplx* src = static_cast<const cplx*>(eps);
  cplx* dout = static_cast<cplx*>(diag_out);
  cplx* mout = static_cast<cplx*>(epsM_out);
  // the status starts clean on every call (a kernel, not a memset node)
  launch_set_int(status_out, INT_MAX, st);
  for (int w0 = 0; w0 < n_w; w0 += chunk) {
    const int m = std::min(chunk, n_w - w0);
    cplx* diag = dout ? dout + (size_t)w0 * n : dscr;
    if (lfe) {
      HIPCK(hipMemcpyAsync(work, src + (size_t)w0 * n * n, sizeof(cplx) * (size_t)m * n * n,
                           hipMemcpyDeviceToDevice, st));
      launch_gj_diag(work, n_G, m, diag, status_out, st, w0);
    } else {
      launch_nolfe_diag(src + (size_t)w0 * n * n, n_G, m, diag, status_out, st, w0);
    }
    LAUNCHCK("inverse (no allocation)");
    launch_loss(diag, n_G, m, loss_out + (size_t)w0 * n, mout ? mout + w0 : nullptr, st);
    LAUNCHCK("loss (no allocation)");
  }
  return QCX_OK;
}

}  // extern "C"
