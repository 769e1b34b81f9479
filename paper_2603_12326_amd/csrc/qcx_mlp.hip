// C ABI of the loss surrogate (include/qcx.h, "Surrogate"): an ensemble of
// 5 -> 256x4 -> 1 SiLU networks trained and evaluated by the kernels of
// k_mlp.hip on the owning context's device and stream.
#include "ctx.h"
#include "mlp.h"

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
  DevBuf Z[4], Hb[4], HT[3], dZ[2], dZb[2], dZbT[2], y, dy, sq, hist, flag;
  // inference / query workspace
  DevBuf xq, ys, sel_counts;
  int cap_query = 0;
  double qmax = 1.0, wmax = 1.0, mu = 0.0, sigma = 1.0, calib = 1.0;
  bool have_encoding = false;
  ~qcx_mlp() {
    for (Member& m : mem) m.release();
    DevBuf* all[] = {&Z[0], &Z[1], &Z[2], &Z[3], &Hb[0], &Hb[1], &Hb[2], &Hb[3], &HT[0], &HT[1],
                     &HT[2], &dZ[0], &dZ[1], &dZb[0], &dZb[1], &dZbT[0], &dZbT[1], &y, &dy, &sq,
                     &hist, &flag, &xq, &ys, &sel_counts};
    for (DevBuf* b : all) b->release();
  }
};

namespace {

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
  launch_out_grad(m->Hb[3].as<uint16_t>(), m->dy.as<float>(), rows_p, g + kOffW5, g + kOffB5, st);
  int s = 0;  // dZ set holding dz of the current layer
  for (int l = 4; l >= 2; --l) {
    // weight gradient dW_l = bf16(dz_l)^T bf16(h_{l-1}), bias gradient sum dz_l
    launch_gemm_store(m->dZbT[s].as<uint16_t>(), m->HT[l - 2].as<uint16_t>(), kW, kW, rows_p,
                      g + off_w(l), st);
    launch_colsum(m->dZ[s].as<float>(), rows_p, kW, g + off_b(l), st);
    EpiBwd e;
    e.Zprev = m->Z[l - 2].as<float>();
    e.dZ = m->dZ[1 - s].as<float>();
    e.dZb = m->dZb[1 - s].as<uint16_t>();
    e.dZbT = m->dZbT[1 - s].as<uint16_t>();
    e.ldt = rows_p;
    launch_gemm_bwd(m->dZb[s].as<uint16_t>(), wb.wt[l - 2], rows_p, kW, kW, e, st);
    s = 1 - s;
  }
  launch_w1_grad(m->dZ[s].as<float>(), x, order, off, n, g + kOffW1, g + kOffB1, st);
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

int qcx_mlp_set_encoding(qcx_mlp* m, double q_max, double w_max_eV, double mu, double sigma,
                         double calib) {
  if (!m) return QCX_EINVAL;
  if (!(q_max > 0.0) || !(w_max_eV > 0.0) || !(sigma > 0.0) || !(calib >= 0.0) ||
      !std::isfinite(mu))
    return fail(m->ctx, QCX_EINVAL, "bad encoding constants");
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
  launch_encode(qw, loss, n, m->qmax, m->wmax, m->mu, m->sigma, x, t, ctx->stream);
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
  launch_encode(qw, nullptr, n, m->qmax, m->wmax, m->mu, m->sigma, m->xq.as<float>(), nullptr, st);
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

}  // extern "C"
