// Internal: the context behind the C ABI and host-side helpers shared by the
// runtime translation units.
#pragma once

#include <limits.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>


#include "common.h"

using namespace qcx;

namespace qcx {
struct BatchPlan;
void destroy_plan(BatchPlan* p);
}  // namespace qcx

namespace qcx {
// pinned staging ring of a context: buffers and bytes per buffer
constexpr int kStageSlots = 4;
constexpr size_t kStageBytes = (size_t)16 << 20;
}  // namespace qcx

struct qcx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // cell and basis
  bool have_basis = false;
  bool f0_valid = false;  // d_F0 holds the Q = 0 integrals of the current basis
  double lat[9], rec[9], vol = 0.0;
  int n_atoms = 0, n_sh = 0, n_ao = 0, lrange = 1, n_cells = 0;
  std::vector<int> sh_l, sh_off, cells;
  std::vector<double> sh_ex, sh_ctr, tvec;
  DevBuf d_sh_l, d_sh_ex, d_sh_ctr, d_sh_off, d_cells, d_tvec, d_shp;

  // states
  bool have_states = false;
  double q[3] = {0, 0, 0};
  int n_k = 0, n_occ = 0, n_b = 0, n_c = 0, n_t = 0;
  DevBuf d_kf, d_Ck, d_Ek, d_Ckq, d_Ekq, d_dt, d_ph, d_phq, d_S, d_F0, d_dev, d_flags;
  bool check_pending = false;  // device-input state checks not yet read back
  int check_nk = 0;

  // pair densities
  bool have_rho = false;
  int n_g = 0;
  size_t ldt = 0;
  DevBuf d_qc, d_G, d_Q, d_vq, d_F, d_M, d_R;  // q (set by qcx_set_states), G list, q + G, ...

  // chi0
  bool have_chi0 = false;
  int n_w = 0, prec = 0, hw64 = 1;
  double eta = 0.0;
  Chi0Geom geom{};
  int ks64 = 1, n_pairs64 = 0;
  int bulk_nst = 2;           // LDS pipeline of the last bulk launch (2, 3; 4: three
                              // stages with the slab one step ahead of the weights)
  int force_nst = 0;          // 0: tuned or heuristic pipeline; 2..4: this one
  int bulk_af = 4;            // row fragments per wave of the last bulk launch
  int autotune = 1;           // 0: fixed heuristic, 1: time candidates per shape
  double tune_ms = 0.0;       // time spent tuning in the last qcx_chi0
  Geom64 geom64{};
  DevBuf d_w, d_A, d_Alo, d_R32, d_pairs, d_rows, d_pairs64, d_C, d_C64, d_XY, d_hwP;
  // what d_pairs, d_rows and d_pairs64 last received (upload_cached)
  std::vector<int> h_pairs_up, h_rows_up, h_pairs64_up;
  // Kramers-Kronig route: energy order, sorted energies and sides, K ranges
  // per row tile, reduced bins, transform matrix
  DevBuf d_kk_rank, d_kk_ib, d_kk_xf, d_kk_chunks, d_kk_Rs, d_kk_S, d_kk_K;
  DevBuf d_Fg, d_Rp;  // optical limit: gradient integrals, band momentum matrices
  bool bulk_c64 = false;      // bulk partials reduced to FP64 (row chunks)

  // eps
  bool have_eps = false;
  bool sing_armed = false;  // d_sing holds the flag of an inversion not yet reported
  DevBuf d_eps, d_diag, d_epsM, d_loss, d_sing;

  // device memory of the buffers above (qcx_set_memory_limit)
  DevBudget budget;
  // event for ordering a batch against the streams of its other contexts
  hipEvent_t ev_order = nullptr;

  // pinned staging for host -> device copies: a ring of kStageSlots buffers,
  // one per call in turn; a call waits only until the copies of the call that
  // used its buffer kStageSlots calls earlier have completed, so the host can
  // run several calls ahead of the device
  struct StageSlot {
    void* p = nullptr;
    hipEvent_t done = nullptr;
    bool pending = false;
  };
  StageSlot stage_ring[qcx::kStageSlots];
  int stage_cur = -1;
  size_t stage_off = 0;
  // transition energies copied to pinned host memory right after
  // qcx_set_states computes them, once the Kramers-Kronig route has been
  // used (its host-side sort then overlaps the pair densities on the device)
  double* h_dt = nullptr;
  size_t h_dt_cap = 0;
  hipEvent_t ev_dt = nullptr;
  bool dt_prefetch = false, dt_valid = false, dt_pending = false;

  // timing: event pairs recorded on the stream without synchronising,
  // resolved by qcx_stage_times
  struct Span {
    hipEvent_t a, b;
    int stage;
  };
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<Span> spans;
  double t_acc[7] = {0, 0, 0, 0, 0, 0, 0};

  // batch plan owned by the first context of a batch (see qcx_batch.hip)
  qcx::BatchPlan* plan = nullptr;

  std::vector<DevBuf*> buffers() {
    return {&d_sh_l, &d_sh_ex, &d_sh_ctr, &d_sh_off, &d_cells, &d_tvec, &d_shp, &d_kf,
                     &d_Ck,   &d_Ek,    &d_Ckq,    &d_Ekq,    &d_dt,    &d_ph,   &d_phq,
                     &d_S,    &d_F0,    &d_dev,    &d_flags,    &d_qc, &d_G, &d_Q,      &d_vq,    &d_F,    &d_M,
                     &d_R,    &d_w,     &d_A,      &d_Alo,    &d_R32,   &d_pairs, &d_rows, &d_pairs64, &d_C, &d_C64,
                     &d_XY,   &d_hwP,   &d_eps,    &d_diag,   &d_epsM,  &d_loss,  &d_sing,
                     &d_kk_rank, &d_kk_ib, &d_kk_xf, &d_kk_chunks, &d_kk_Rs, &d_kk_S, &d_kk_K,
                     &d_Fg, &d_Rp};
  }
  qcx_ctx() {
    for (DevBuf* b : buffers()) b->budget = &budget;
  }
  ~qcx_ctx() {
    if (plan) qcx::destroy_plan(plan);
    for (DevBuf* b : buffers()) b->release();
    if (ev_order) (void)hipEventDestroy(ev_order);
    for (const Span& sp : spans) {
      (void)hipEventDestroy(sp.a);
      (void)hipEventDestroy(sp.b);
    }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (StageSlot& sl : stage_ring) {
      if (sl.pending && sl.done) (void)hipEventSynchronize(sl.done);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.p) (void)hipHostFree(sl.p);
    }
    if (dt_pending && ev_dt) (void)hipEventSynchronize(ev_dt);
    if (h_dt) (void)hipHostFree(h_dt);
    if (ev_dt) (void)hipEventDestroy(ev_dt);
  }
};

namespace qcx {

// deferred state checks of device-resident inputs (qcx_runtime.hip)
int check_deferred(qcx_ctx* ctx);
// Pair densities in two parts (qcx_runtime.hip): rho_prepare checks a G list
// on the host against the context's q (G = 0 first, q + G nonzero unless
// optical) and reserves the buffers for n_G rows; rho_enqueue launches
// kernels only (q + G and Coulomb factors from the device copy of q and the
// device G list, tail zeroing, cell Fourier integrals, densities), so that
// it can be captured into a graph.
int rho_prepare(qcx_ctx* ctx, int n_G, const int* G_int, bool need_g0, bool optical);
int rho_enqueue(qcx_ctx* ctx, const int* d_G, int n_G, bool optical, hipStream_t st);
// address of the no-allocation scratch array on `device`, looked up once per
// device with that device current (qcx_noalloc.hip)
hipError_t noalloc_init(int device);

inline int fail(qcx_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCK(call)                                                                   \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, e_ == hipErrorOutOfMemory ? QCX_ENOMEM : QCX_EDEVICE,          \
                  std::string(#call) + ": " + hipGetErrorString(e_));                 \
  } while (0)

#define LAUNCHCK(what)                                                                \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, QCX_EDEVICE, std::string("launch ") + what + ": " +            \
                                        hipGetErrorString(e_));                       \
  } while (0)

inline size_t roundup(size_t x, size_t m) { return (x + m - 1) / m * m; }

// Calls that stage host data (pinned ring, index tables cached by content,
// synchronous fallbacks) cannot be recorded into a graph: they return
// QCX_EINVAL while the context's stream is capturing.
inline int reject_capture(qcx_ctx* c) {
  hipStreamCaptureStatus s = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(c->stream, &s);
  if (e != hipSuccess) return fail(c, QCX_EDEVICE, std::string("hipStreamIsCapturing: ") + hipGetErrorString(e));
  if (s != hipStreamCaptureStatusNone)
    return fail(c, QCX_EINVAL, "this call stages host data and cannot be captured into a graph");
  return QCX_OK;
}


// Upload an index table unless the buffer already holds exactly these values
// (the pair tables repeat from call to call); `last` mirrors what `b` last
// received and must be the only record of writes to it.
template <class B>
inline hipError_t upload_cached(B* c, DevBuf& b, std::vector<int>& last,
                                const std::vector<int>& v);

// Begin a call that stages host data: take the next buffer of the ring and
// wait until the copies staged in it kStageSlots calls ago have left it.  All
// buffers are allocated on the first call (never inside a later, possibly
// captured, call).
inline hipError_t stage_begin(qcx_ctx* c) {
  if (!c->stage_ring[0].p) {
    for (qcx_ctx::StageSlot& sl : c->stage_ring) {
      hipError_t e = hipHostMalloc(&sl.p, kStageBytes);
      if (e != hipSuccess) {
        sl.p = nullptr;
        return e;
      }
      e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
  }
  c->stage_cur = (c->stage_cur + 1) % kStageSlots;
  qcx_ctx::StageSlot& sl = c->stage_ring[c->stage_cur];
  if (sl.pending) {
    hipError_t e = hipEventSynchronize(sl.done);
    if (e != hipSuccess) return e;
    sl.pending = false;
  }
  c->stage_off = 0;
  return hipSuccess;
}

// Copy n elements to a context buffer on the context's stream.  Host data goes
// through the pinned arena (or, if it does not fit, a synchronous copy), so the
// caller's array may be released as soon as the call returns.
template <class T>
inline hipError_t upload(qcx_ctx* c, DevBuf& b, const T* src, size_t n, bool dev_src = false) {
  const size_t bytes = n * sizeof(T);
  hipError_t e = b.reserve(bytes + 64);
  if (e != hipSuccess) return e;
  if (dev_src) return hipMemcpyAsync(b.p, src, bytes, hipMemcpyDeviceToDevice, c->stream);
  const size_t off = (c->stage_off + 255) / 256 * 256;
  qcx_ctx::StageSlot* sl = c->stage_cur >= 0 ? &c->stage_ring[c->stage_cur] : nullptr;
  if (sl && sl->p && off + bytes <= kStageBytes) {
    char* h = static_cast<char*>(sl->p) + off;
    memcpy(h, src, bytes);
    c->stage_off = off + bytes;
    e = hipMemcpyAsync(b.p, h, bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
    // record after every staged copy so that an early error return still
    // leaves the buffer guarded
    e = hipEventRecord(sl->done, c->stream);
    if (e == hipSuccess) sl->pending = true;
    return e;
  }
  e = hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

template <class B>
inline hipError_t upload_cached(B* c, DevBuf& b, std::vector<int>& last,
                                const std::vector<int>& v) {
  if (b.p && !v.empty() && last == v) return hipSuccess;
  last.clear();  // unknown contents until the copy below is queued
  hipError_t e = upload(c, b, v.data(), v.size());
  if (e == hipSuccess) last = v;
  return e;
}

// Queue a copy of the transition energies (d_dt, n_t values) to h_dt on the
// stream and record ev_dt after it.
inline hipError_t dt_to_host(qcx_ctx* c, int n_t) {
  hipError_t e = hipSuccess;
  if (!c->ev_dt && (e = hipEventCreateWithFlags(&c->ev_dt, hipEventDisableTiming)) != hipSuccess)
    return e;
  if (c->h_dt_cap < (size_t)n_t) {
    if (c->dt_pending && (e = hipEventSynchronize(c->ev_dt)) != hipSuccess) return e;
    c->dt_pending = false;
    if (c->h_dt) (void)hipHostFree(c->h_dt);
    c->h_dt = nullptr;
    c->h_dt_cap = 0;
    if ((e = hipHostMalloc((void**)&c->h_dt, sizeof(double) * n_t)) != hipSuccess) {
      c->h_dt = nullptr;
      return e;
    }
    c->h_dt_cap = n_t;
  }
  e = hipMemcpyAsync(c->h_dt, c->d_dt.p, sizeof(double) * n_t, hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(c->ev_dt, c->stream)) != hipSuccess) return e;
  c->dt_pending = true;
  return hipSuccess;
}

inline void inv3(const double m[9], double out[9]) {
  const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5], g = m[6], h = m[7],
               i = m[8];
  const double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
  out[0] = (e * i - f * h) / det;
  out[1] = (c * h - b * i) / det;
  out[2] = (b * f - c * e) / det;
  out[3] = (f * g - d * i) / det;
  out[4] = (a * i - c * g) / det;
  out[5] = (c * d - a * f) / det;
  out[6] = (d * h - e * g) / det;
  out[7] = (b * g - a * h) / det;
  out[8] = (a * e - b * d) / det;
}

inline hipError_t take_event(qcx_ctx* c, hipEvent_t* e) {
  if (!c->ev_pool.empty()) {
    *e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Open a timed span for `stage`; returns its index in *idx (or -1 when timing
// is off).
inline hipError_t span_begin(qcx_ctx* c, int stage, int* idx) {
  *idx = -1;
  if (!c->timing) return hipSuccess;
  qcx_ctx::Span sp{};
  hipError_t e = take_event(c, &sp.a);
  if (e != hipSuccess) return e;
  e = take_event(c, &sp.b);
  if (e != hipSuccess) return e;
  sp.stage = stage;
  e = hipEventRecord(sp.a, c->stream);
  if (e != hipSuccess) return e;
  c->spans.push_back(sp);
  *idx = (int)c->spans.size() - 1;
  return hipSuccess;
}

inline hipError_t span_end(qcx_ctx* c, int idx) {
  if (idx < 0) return hipSuccess;
  return hipEventRecord(c->spans[idx].b, c->stream);
}

// Resolve every recorded span into t_acc (synchronises the stream).
inline hipError_t spans_resolve(qcx_ctx* c) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  for (const qcx_ctx::Span& sp : c->spans) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, sp.a, sp.b);
    if (e != hipSuccess) return e;
    c->t_acc[sp.stage] += ms;
    if (sp.stage == 1) c->t_acc[5] += 1.0;
    c->ev_pool.push_back(sp.a);
    c->ev_pool.push_back(sp.b);
  }
  c->spans.clear();
  return hipSuccess;
}

}  // namespace qcx

