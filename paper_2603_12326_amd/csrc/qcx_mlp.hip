// C ABI of the loss surrogate (include/qcx.h, "Surrogate"): an ensemble of
// 49 -> 256x4 -> 1 SiLU networks trained and evaluated by the kernels of
// k_mlp.hip on the owning context's device and stream.
#include "ctx.h"
#include "mlp.h"

static_assert(qcx::mlp::kIn == QCX_MLP_NIN && qcx::mlp::kNParam == QCX_MLP_NPARAM,
              "network shape of the C ABI");

using namespace qcx::mlp;

namespace {

struct Member {
  DevBuf p, m, v, g;                    // FP32 parameters, Adam moments, gradient
  DevBuf w1b, w[3], wt[3], w5b;         // bf16 copies
  long step = 0;
  WeightsB wb() const {
    WeightsB b;
    b.w1 = w1b.as<uint16_t>();
    for (int l = 0; l < 3; ++l) {
      b.w[l] = w[l].as<uint16_t>();
      b.wt[l] = wt[l].as<uint16_t>();
    }
    b.w5 = w5b.as<uint16_t>();
    return b;
  }
  void release() {
    DevBuf* all[] = {&p, &m, &v, &g, &w1b, &w[0], &w[1], &w[2], &wt[0], &wt[1], &wt[2], &w5b};
    for (DevBuf* b : all) b->release();
  }
};

constexpr int kMaxBatch = 16384;   // training rows per step
constexpr int kInferChunk = 65536; // rows per inference pass

}  // namespace

struct qcx_mlp {
  qcx_ctx* ctx = nullptr;
  std::vector<Member> mem;
  // training workspace (rows_p = batch padded to 64)
  int cap_rows = 0;
  DevBuf Z[4], Hb[4], HT[3], dZ[2], dZb[2], dZbT[2], y, dy, sq, hist, flag, red;
  // inference / query workspace
  DevBuf xq, ys, sel_counts;
  // qcx_mlp_infer: Q list, frequencies, the query grid, estimates, rejected
  // indices, the method's rows and where they go
  DevBuf iQ, iw, iqw, ierr, iidx, irows, isel;
  int cap_query = 0;
  double qmax = 1.0, wmax = 1.0, mu = 0.0, sigma = 1.0, calib = 1.0;
  Lattice lat{};
  bool have_encoding = false;
  ~qcx_mlp() {
    for (Member& m : mem) m.release();
    DevBuf* all[] = {&Z[0], &Z[1], &Z[2], &Z[3], &Hb[0], &Hb[1], &Hb[2], &Hb[3], &HT[0], &HT[1],
                     &HT[2], &dZ[0], &dZ[1], &dZb[0], &dZb[1], &dZbT[0], &dZbT[1], &y, &dy, &sq,
                     &hist, &flag, &red, &xq, &ys, &sel_counts, &iQ, &iw, &iqw, &ierr, &iidx, &irows,
                     &isel};
    for (DevBuf* b : all) b->release();
  }
};

namespace {

// qw[(iw, g)] = (Q_g, w_iw): the query grid of one momentum, w-major.
__global__ void k_fill_qw(const double* __restrict__ Q, int n_g, const double* __restrict__ w,
                          int n_w, double* qw) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_g * n_w) return;
  const int g = (int)(i % n_g), iw = (int)(i / n_g);
  qw[4 * i] = Q[3 * g];
  qw[4 * i + 1] = Q[3 * g + 1];
  qw[4 * i + 2] = Q[3 * g + 2];
  qw[4 * i + 3] = w[iw];
}

// out[sel[r]][g] = rows[r][g]: the method's rows into the answer.
__global__ void k_scatter_rows(const double* __restrict__ rows, const int* __restrict__ sel,
                               int n_sel, int n_g, double* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_sel * n_g) return;
  const int r = (int)(i / n_g), g = (int)(i % n_g);
  out[(size_t)sel[r] * n_g + g] = rows[i];
}

// The error estimate of each point in units of its curve's maximum (the
// normwise measure of a loss curve along frequency): for every G,
//   e[w][G] <- e[w][G] |L[w][G]| / max_w' |L[w'][G]|,
// e being the estimate relative to the point's own value, so that e bounds
// |L - L_method| / max_w |L| where the relative estimate bounds the relative
// error.  A non-finite estimate or prediction becomes infinite (rejected).
__global__ void k_normwise_err(const double* __restrict__ L, double* __restrict__ e, int n_w,
                               int n_g) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_g) return;
  double mx = 0.0;
  for (int w = 0; w < n_w; ++w) mx = fmax(mx, fabs(L[(size_t)w * n_g + g]));
  const double s = mx > 0.0 ? 1.0 / mx : 0.0;
  for (int w = 0; w < n_w; ++w) {
    const size_t i = (size_t)w * n_g + g;
    const double v = e[i] * fabs(L[i]) * s;
    e[i] = v == v ? v : INFINITY;
  }
}

int reserve_rows(qcx_mlp* m, int rows_p, bool training) {
  qcx_ctx* ctx = m->ctx;
  const size_t r = (size_t)rows_p;
  for (int l = 0; l < 4; ++l) {
    HIPCK(m->Hb[l].reserve(sizeof(uint16_t) * r * kW));
    if (training) HIPCK(m->Z[l].reserve(sizeof(float) * r * kW));
  }
  if (training) {
    for (int l = 0; l < 3; ++l) HIPCK(m->HT[l].reserve(sizeof(uint16_t) * r * kW));
    for (int s = 0; s < 2; ++s) {
      HIPCK(m->dZ[s].reserve(sizeof(float) * r * kW));
      HIPCK(m->dZb[s].reserve(sizeof(uint16_t) * r * kW));
      HIPCK(m->dZbT[s].reserve(sizeof(uint16_t) * r * kW));
    }
    HIPCK(m->dy.reserve(sizeof(float) * r));
    HIPCK(m->sq.reserve(sizeof(float) * r));
    HIPCK(m->red.reserve(sizeof(float) * std::max(red_floats(rows_p),
                                                   (size_t)store_ksplit(rows_p) * kW * kW)));
  }
  HIPCK(m->y.reserve(sizeof(float) * r));
  return QCX_OK;
}

// forward of one member over n rows of x (rows of order[off..] when order is
// set); training keeps Z, Hb and the transposes for the backward pass
void forward_rows(qcx_mlp* m, const Member& w, const float* x, const int* order, long off, int n,
                  int rows_p, bool training, float* y, hipStream_t st) {
  WeightsB wb = w.wb();
  const float* p = w.p.as<float>();
  launch_layer1(x, order, off, n, rows_p, wb.w1, p + kOffB1, training ? m->Z[0].as<float>() : nullptr,
                m->Hb[0].as<uint16_t>(), training ? m->HT[0].as<uint16_t>() : nullptr, rows_p, st);
  for (int l = 2; l <= 4; ++l) {
    EpiFwd e;
    e.bias = p + off_b(l);
    e.Z = training ? m->Z[l - 1].as<float>() : nullptr;
    e.Hb = m->Hb[l - 1].as<uint16_t>();
    e.HT = (training && l < 4) ? m->HT[l - 1].as<uint16_t>() : nullptr;
    e.ldt = rows_p;
    launch_gemm_fwd(m->Hb[l - 2].as<uint16_t>(), wb.w[l - 2], rows_p, kW, kW, e, st);
  }
  if (!training)
    launch_output(m->Hb[3].as<uint16_t>(), wb.w5, p + kOffB5, n, rows_p, y, nullptr, nullptr, 0,
                  nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, st);
}

// one gradient evaluation into w.g; the mean squared error into *loss_dev
void grad_rows(qcx_mlp* m, Member& w, const float* x, const float* t, const int* order, long off,
               int n, int rows_p, float* loss_dev, hipStream_t st) {
  forward_rows(m, w, x, order, off, n, rows_p, true, nullptr, st);
  WeightsB wb = w.wb();
  const float* p = w.p.as<float>();
  float* g = w.g.as<float>();
  launch_output(m->Hb[3].as<uint16_t>(), wb.w5, p + kOffB5, n, rows_p, m->y.as<float>(), t, order,
                off, m->dy.as<float>(), m->sq.as<float>(), m->Z[3].as<float>(), m->dZ[0].as<float>(),
                m->dZb[0].as<uint16_t>(), m->dZbT[0].as<uint16_t>(), rows_p, st);
  float* red = m->red.as<float>();
  launch_out_grad(m->Hb[3].as<uint16_t>(), m->dy.as<float>(), rows_p, g + kOffW5, g + kOffB5, red,
                  st);
  int s = 0;  // dZ set holding dz of the current layer
  for (int l = 4; l >= 2; --l) {
    // weight gradient dW_l = bf16(dz_l)^T bf16(h_{l-1}), bias gradient sum dz_l
    launch_gemm_store(m->dZbT[s].as<uint16_t>(), m->HT[l - 2].as<uint16_t>(), kW, kW, rows_p,
                      g + off_w(l), red, st);
    launch_colsum(m->dZ[s].as<float>(), rows_p, kW, g + off_b(l), red, st);
    EpiBwd e;
    e.Zprev = m->Z[l - 2].as<float>();
    e.dZ = m->dZ[1 - s].as<float>();
    e.dZb = m->dZb[1 - s].as<uint16_t>();
    e.dZbT = m->dZbT[1 - s].as<uint16_t>();
    e.ldt = rows_p;
    launch_gemm_bwd(m->dZb[s].as<uint16_t>(), wb.wt[l - 2], rows_p, kW, kW, e, st);
    s = 1 - s;
  }
  launch_w1_grad(m->dZ[s].as<float>(), x, order, off, n, g + kOffW1, g + kOffB1, red, st);
  launch_mean(m->sq.as<float>(), rows_p, n, loss_dev, st);
}

__global__ void k_check_order(const int* order, long n, int n_data, int* flag) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (order[i] < 0 || order[i] >= n_data)) atomicOr(flag, 1);
}

int check_member(qcx_mlp* m, int member) {
  if (member < 0 || member >= (int)m->mem.size())
    return fail(m->ctx, QCX_EINVAL, "member index out of range");
  return QCX_OK;
}

int rows_padded(int n) { return (n + kRowTile - 1) / kRowTile * kRowTile; }

}  // namespace

extern "C" {

int qcx_mlp_create(qcx_mlp** out, qcx_ctx* ctx, int n_members) {
  if (!out || !ctx) return QCX_EINVAL;
  *out = nullptr;
  if (n_members < 1 || n_members > 16) return fail(ctx, QCX_EINVAL, "n_members must be 1..16");
  HIPCK(hipSetDevice(ctx->device));
  qcx_mlp* m = new qcx_mlp();
  m->ctx = ctx;
  m->mem.resize(n_members);
  for (Member& w : m->mem) {
    const size_t np = sizeof(float) * kNParam;
    hipError_t e = hipSuccess;
    DevBuf* f32[] = {&w.p, &w.m, &w.v, &w.g};
    for (DevBuf* b : f32)
      if (e == hipSuccess) e = b->reserve(np);
    if (e == hipSuccess) e = w.w1b.reserve(sizeof(uint16_t) * kW * kIn);
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
      e = w.w[l].reserve(sizeof(uint16_t) * kW * kW);
      if (e == hipSuccess) e = w.wt[l].reserve(sizeof(uint16_t) * kW * kW);
    }
    if (e == hipSuccess) e = w.w5b.reserve(sizeof(uint16_t) * kW);
    if (e == hipSuccess) e = hipMemsetAsync(w.p.p, 0, np, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w.m.p, 0, np, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w.v.p, 0, np, ctx->stream);
    if (e == hipSuccess) launch_refresh(w.p.as<float>(), w.wb(), ctx->stream);
    if (e != hipSuccess) {
      delete m;
      return fail(ctx, e == hipErrorOutOfMemory ? QCX_ENOMEM : QCX_EDEVICE,
                  std::string("surrogate allocation: ") + hipGetErrorString(e));
    }
  }
  *out = m;
  return QCX_OK;
}

int qcx_mlp_destroy(qcx_mlp* m) {
  if (!m) return QCX_OK;
  (void)hipSetDevice(m->ctx->device);
  (void)hipStreamSynchronize(m->ctx->stream);
  delete m;
  return QCX_OK;
}

int qcx_mlp_set_params(qcx_mlp* m, int member, const float* params) {
  if (!m) return QCX_EINVAL;
  qcx_ctx* ctx = m->ctx;
  if (!params) return fail(ctx, QCX_EINVAL, "params is NULL");
  if (int rc = check_member(m, member)) return rc;
  for (int i = 0; i < kNParam; ++i)
    if (!std::isfinite(params[i])) return fail(ctx, QCX_EINVAL, "non-finite parameter");
  HIPCK(hipSetDevice(ctx->device));
  Member& w = m->mem[member];
  hipStream_t st = ctx->stream;
  HIPCK(hipMemcpyAsync(w.p.p, params, sizeof(float) * kNParam, hipMemcpyHostToDevice, st));
  HIPCK(hipMemsetAsync(w.m.p, 0, sizeof(float) * kNParam, st));
  HIPCK(hipMemsetAsync(w.v.p, 0, sizeof(float) * kNParam, st));
  w.step = 0;
  launch_refresh(w.p.as<float>(), w.wb(), st);
  LAUNCHCK("refresh");
  HIPCK(hipStreamSynchronize(st));  // params is the caller's pageable memory
  return QCX_OK;
}

int qcx_mlp_get_params(qcx_mlp* m, int member, float* params) {
  if (!m) return QCX_EINVAL;
  qcx_ctx* ctx = m->ctx;
  if (!params) return fail(ctx, QCX_EINVAL, "params is NULL");
  if (int rc = check_member(m, member)) return rc;
  HIPCK(hipSetDevice(ctx->device));
  HIPCK(hipMemcpyAsync(params, m->mem[member].p.p, sizeof(float) * kNParam, hipMemcpyDeviceToHost,
                       ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  return QCX_OK;
}

int qcx_mlp_forward(qcx_mlp* m, int member, int n, const float* x, float* y) {
  if (!m) return QCX_EINVAL;
  qcx_ctx* ctx = m->ctx;
  if (int rc = check_member(m, member)) return rc;
  if (n < 0 || (n > 0 && (!x || !y))) return fail(ctx, QCX_EINVAL, "bad n or NULL buffer");
  HIPCK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  for (int r0 = 0; r0 < n; r0 += kInferChunk) {
    const int nn = std::min(kInferChunk, n - r0), rp = rows_padded(nn);
    if (int rc = reserve_rows(m, rp, false)) return rc;
    forward_rows(m, m->mem[member], x + (size_t)r0 * kIn, nullptr, 0, nn, rp, false,
                 m->y.as<float>(), st);
    HIPCK(hipMemcpyAsync(y + r0, m->y.p, sizeof(float) * nn, hipMemcpyDeviceToDevice, st));
  }
  LAUNCHCK("surrogate forward");
  return QCX_OK;
}

int qcx_mlp_grad(qcx_mlp* m, int member, int n, const float* x, const float* t, float* grad,
                 float* loss) {
  if (!m) return QCX_EINVAL;
  qcx_ctx* ctx = m->ctx;
  if (int rc = check_member(m, member)) return rc;
  if (n < 1 || n > kMaxBatch) return fail(ctx, QCX_EINVAL, "n must be 1..16384");
  if (!x || !t || !grad) return fail(ctx, QCX_EINVAL, "NULL buffer");
  HIPCK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int rp = rows_padded(n);
  if (int rc = reserve_rows(m, rp, true)) return rc;
  HIPCK(m->hist.reserve(sizeof(float)));
  Member& w = m->mem[member];
  grad_rows(m, w, x, t, nullptr, 0, n, rp, m->hist.as<float>(), st);
  LAUNCHCK("surrogate gradient");
  HIPCK(hipMemcpyAsync(grad, w.g.p, sizeof(float) * kNParam, hipMemcpyDeviceToHost, st));
  float l = 0.0f;
  HIPCK(hipMemcpyAsync(&l, m->hist.p, sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  if (loss) *loss = l;
  return QCX_OK;
}

int qcx_mlp_train(qcx_mlp* m, int member, int n_data, const float* x, const float* t, int batch,
                  int n_steps, const int* order, float lr0, float lr1, float* loss_hist) {
  if (!m) return QCX_EINVAL;
  qcx_ctx* ctx = m->ctx;
  if (int rc = check_member(m, member)) return rc;
  if (n_data < 1 || !x || !t || !order) return fail(ctx, QCX_EINVAL, "bad data");
  if (batch < 1 || batch > kMaxBatch) return fail(ctx, QCX_EINVAL, "batch must be 1..16384");
  if (n_steps < 1) return fail(ctx, QCX_EINVAL, "n_steps must be >= 1");
  if (!(lr0 > 0.0f) || !(lr1 >= 0.0f)) return fail(ctx, QCX_EINVAL, "bad learning rates");
  HIPCK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const long n_idx = (long)n_steps * batch;
  // every sample index is checked before any step reads through it
  HIPCK(m->flag.reserve(sizeof(int)));
  HIPCK(hipMemsetAsync(m->flag.p, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_check_order, dim3((unsigned)((n_idx + 255) / 256)), dim3(256), 0, st, order,
                     n_idx, n_data, m->flag.as<int>());
  LAUNCHCK("order check");
  int bad = 0;
  HIPCK(hipMemcpyAsync(&bad, m->flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  if (bad) return fail(ctx, QCX_EINVAL, "order holds an index outside [0, n_data)");
  const int rp = rows_padded(batch);
  if (int rc = reserve_rows(m, rp, true)) return rc;
  HIPCK(m->hist.reserve(sizeof(float) * (size_t)n_steps));
  Member& w = m->mem[member];
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int s = 0; s < n_steps; ++s) {
    grad_rows(m, w, x, t, order, (long)s * batch, batch, rp, m->hist.as<float>() + s, st);
    ++w.step;
    const double lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + cos(kPi * s / n_steps));
    const float c1 = (float)(1.0 - pow((double)b1, (double)w.step));
    const float c2 = (float)(1.0 - pow((double)b2, (double)w.step));
    launch_adam(w.p.as<float>(), w.g.as<float>(), w.m.as<float>(), w.v.as<float>(), kNParam,
                (float)lr, b1, b2, c1, c2, eps, st);
    launch_refresh(w.p.as<float>(), w.wb(), st);
  }
  LAUNCHCK("surrogate training");
  if (loss_hist) {
    HIPCK(hipMemcpyAsync(loss_hist, m->hist.p, sizeof(float) * n_steps, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
  }
  return QCX_OK;
}

int qcx_mlp_set_encoding(qcx_mlp* m, double q_max, double w_max_eV, const double* lattice,
                         double mu, double sigma, double calib) {
  if (!m) return QCX_EINVAL;
  if (!(q_max > 0.0) || !(w_max_eV > 0.0) || !(sigma > 0.0) || !(calib >= 0.0) ||
      !std::isfinite(mu) || !lattice)
    return fail(m->ctx, QCX_EINVAL, "bad encoding constants");
  for (int i = 0; i < 9; ++i) {
    if (!std::isfinite(lattice[i])) return fail(m->ctx, QCX_EINVAL, "non-finite lattice");
    m->lat.a[i] = lattice[i];
  }
  m->qmax = q_max;
  m->wmax = w_max_eV;
  m->mu = mu;
  m->sigma = sigma;
  m->calib = calib;
  m->have_encoding = true;
  return QCX_OK;
}

int qcx_mlp_encode(qcx_mlp* m, int n, const double* qw, const double* loss, float* x, float* t) {
  if (!m) return QCX_EINVAL;
  qcx_ctx* ctx = m->ctx;
  if (!m->have_encoding) return fail(ctx, QCX_ESTATE, "qcx_mlp_set_encoding first");
  if (n < 0 || (n > 0 && (!qw || !x))) return fail(ctx, QCX_EINVAL, "bad n or NULL buffer");
  if (n == 0) return QCX_OK;
  HIPCK(hipSetDevice(ctx->device));
  launch_encode(qw, loss, n, m->qmax, m->wmax, m->lat, m->mu, m->sigma, x, t, ctx->stream);
  LAUNCHCK("encode");
  return QCX_OK;
}

int qcx_mlp_query(qcx_mlp* m, int n, const double* qw, double* loss, double* err, double tol,
                  int* reject_idx, int* n_reject) {
  if (!m) return QCX_EINVAL;
  qcx_ctx* ctx = m->ctx;
  if (!m->have_encoding) return fail(ctx, QCX_ESTATE, "qcx_mlp_set_encoding first");
  if (n < 0 || (n > 0 && (!qw || !loss))) return fail(ctx, QCX_EINVAL, "bad n or NULL buffer");
  if ((reject_idx || n_reject) && !(err && reject_idx && n_reject))
    return fail(ctx, QCX_EINVAL, "rejection needs err, reject_idx and n_reject");
  if (n_reject) *n_reject = 0;
  if (n == 0) return QCX_OK;
  HIPCK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int K = (int)m->mem.size();
  HIPCK(m->xq.reserve(sizeof(float) * kIn * (size_t)n));
  HIPCK(m->ys.reserve(sizeof(float) * (size_t)K * n));
  launch_encode(qw, nullptr, n, m->qmax, m->wmax, m->lat, m->mu, m->sigma, m->xq.as<float>(),
                nullptr, st);
  for (int k = 0; k < K; ++k)
    for (int r0 = 0; r0 < n; r0 += kInferChunk) {
      const int nn = std::min(kInferChunk, n - r0), rp = rows_padded(nn);
      if (int rc = reserve_rows(m, rp, false)) return rc;
      forward_rows(m, m->mem[k], m->xq.as<float>() + (size_t)r0 * kIn, nullptr, 0, nn, rp, false,
                   m->ys.as<float>() + (size_t)k * n + r0, st);
    }
  launch_decode(m->ys.as<float>(), K, n, m->mu, m->sigma, m->calib, loss, err, st);
  LAUNCHCK("surrogate query");
  if (reject_idx) {
    const int nb = select_blocks(n);
    HIPCK(m->sel_counts.reserve(sizeof(int) * ((size_t)nb + 1)));
    int* counts = m->sel_counts.as<int>();
    launch_select(err, n, tol, counts, nb, reject_idx, counts + nb, st);
    LAUNCHCK("select");
    HIPCK(hipMemcpyAsync(n_reject, counts + nb, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
  }
  return QCX_OK;
}

// Surrogate answer for the momentum of ctx's states with fallback to the
// method (include/qcx.h): the networks answer every (w, q + G); a point is
// rejected when its error estimate in units of its curve's maximum exceeds
// tol; the frequencies with any rejected point are recomputed by the method's
// own calls on ctx and their rows replaced.
int qcx_mlp_infer(qcx_mlp* m, qcx_ctx* ctx, int n_G, const int* G_int, int n_w,
                  const double* w_eV, double eta_eV, double tol, int precision, double* loss_out,
                  double* err_out, int* n_fallback) {
  if (!m || !ctx) return QCX_EINVAL;
  qcx_ctx* mc = m->ctx;
  if (n_fallback) *n_fallback = 0;
  if (mc->device != ctx->device) return fail(ctx, QCX_EINVAL, "networks and context on different devices");
  if (!m->have_encoding) return fail(ctx, QCX_ESTATE, "qcx_mlp_set_encoding first");
  if (!ctx->have_states) return fail(ctx, QCX_ESTATE, "set_states first");
  if (n_G < 1 || n_G > 4096 || !G_int) return fail(ctx, QCX_EINVAL, "need 1 <= n_G <= 4096");
  if (G_int[0] != 0 || G_int[1] != 0 || G_int[2] != 0)
    return fail(ctx, QCX_EINVAL, "G_int[0] must be (0,0,0)");
  if (n_w < 1 || n_w > 65536 || !w_eV) return fail(ctx, QCX_EINVAL, "need 1 <= n_w <= 65536");
  if ((long)n_w * n_G > (1L << 26)) return fail(ctx, QCX_EINVAL, "n_w * n_G above 2^26");
  for (int i = 0; i < n_w; ++i)
    if (!std::isfinite(w_eV[i])) return fail(ctx, QCX_EINVAL, "non-finite frequency");
  if (!(eta_eV >= 0.0) || !std::isfinite(eta_eV)) return fail(ctx, QCX_EINVAL, "eta must be >= 0");
  if (!(tol >= 0.0)) return fail(ctx, QCX_EINVAL, "tol must be >= 0");
  if (precision < QCX_FP64 || precision > QCX_SPLIT_BF16) return fail(ctx, QCX_EINVAL, "bad precision");
  if (!loss_out) return fail(ctx, QCX_EINVAL, "loss_out must be a device buffer");
  if (int rc = reject_capture(ctx)) return rc;
  if (int rc = reject_capture(mc)) return rc;
  HIPCK(hipSetDevice(ctx->device));
  // Q = q + G as qcx_pair_density forms it
  std::vector<double> Q(3 * (size_t)n_G);
  for (int g = 0; g < n_G; ++g)
    for (int x = 0; x < 3; ++x) {
      double v = ctx->q[x];
      for (int j = 0; j < 3; ++j) v += G_int[3 * g + j] * ctx->rec[3 * j + x];
      Q[3 * g + x] = v;
    }
  const size_t n = (size_t)n_w * n_G;
  hipStream_t ms = mc->stream;
  HIPCK(stage_begin(mc));
  HIPCK(upload(mc, m->iQ, Q.data(), Q.size()));
  HIPCK(upload(mc, m->iw, w_eV, (size_t)n_w));
  HIPCK(m->iqw.reserve(sizeof(double) * 4 * n));
  HIPCK(m->iidx.reserve(sizeof(int) * n));
  double* err = err_out;
  if (!err) {
    HIPCK(m->ierr.reserve(sizeof(double) * n));
    err = m->ierr.as<double>();
  }
  hipLaunchKernelGGL(k_fill_qw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ms,
                     m->iQ.as<double>(), n_G, m->iw.as<double>(), n_w, m->iqw.as<double>());
  LAUNCHCK("infer grid");
  if (int rc = qcx_mlp_query(m, (int)n, m->iqw.as<double>(), loss_out, err, 0.0, nullptr, nullptr))
    return rc;
  // the estimates in units of each G's curve maximum over these frequencies,
  // then the points above tol
  hipLaunchKernelGGL(k_normwise_err, dim3((unsigned)((n_G + 255) / 256)), dim3(256), 0, ms, loss_out,
                     err, n_w, n_G);
  const int nb = select_blocks((int)n);
  HIPCK(m->sel_counts.reserve(sizeof(int) * ((size_t)nb + 1)));
  int* counts = m->sel_counts.as<int>();
  launch_select(err, (int)n, tol, counts, nb, m->iidx.as<int>(), counts + nb, ms);
  LAUNCHCK("infer rejections");
  int nrej = 0;
  HIPCK(hipMemcpyAsync(&nrej, counts + nb, sizeof(int), hipMemcpyDeviceToHost, ms));
  HIPCK(hipStreamSynchronize(ms));  // the answers and rejections are complete
  if (nrej == 0) return QCX_OK;
  // frequencies with any rejected point (indices ascend, rows are w-major)
  std::vector<int> idx(nrej), sel;
  HIPCK(hipMemcpy(idx.data(), m->iidx.p, sizeof(int) * nrej, hipMemcpyDeviceToHost));
  for (int i : idx)
    if (sel.empty() || sel.back() != i / n_G) sel.push_back(i / n_G);
  std::vector<double> wsel(sel.size());
  for (size_t r = 0; r < sel.size(); ++r) wsel[r] = w_eV[sel[r]];
  const int ns = (int)sel.size();
  if (int rc = qcx_pair_density(ctx, n_G, G_int, nullptr)) return rc;
  if (int rc = qcx_chi0(ctx, ns, wsel.data(), eta_eV, precision, 1, nullptr)) return rc;
  if (int rc = qcx_eps_inv(ctx, 1, nullptr, nullptr)) return rc;
  HIPCK(m->irows.reserve(sizeof(double) * (size_t)ns * n_G));
  if (int rc = qcx_loss(ctx, m->irows.as<double>(), QCX_MEM_DEVICE)) return rc;
  HIPCK(stage_begin(ctx));
  HIPCK(upload(ctx, m->isel, sel.data(), sel.size()));
  const size_t nr = (size_t)ns * n_G;
  hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, ctx->stream,
                     m->irows.as<double>(), m->isel.as<int>(), ns, n_G, loss_out);
  LAUNCHCK("infer fallback rows");
  // asynchronous from here: deferred state checks and a singular eps of these
  // rows are reported by the next synchronising call on ctx
  if (n_fallback) *n_fallback = ns;
  return QCX_OK;
}

}  // extern "C"
