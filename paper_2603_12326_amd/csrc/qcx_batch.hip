// Batched path for many uneven (cell, q, frequency list, N_G) items.
//
// The pair densities of each context either come from the context itself
// (qcx_run_batch: qcx_pair_density already called) or are computed inside the
// plan from a G list per context (qcx_run_batch_rho: q + G and Coulomb factors
// from the device copy of q, cell Fourier integrals, fused Bloch sum and band
// contraction, all captured; new states set on the contexts between calls are
// picked up by the next replay).  A plan is built once per batch signature: per-item
// weights, R32 packs per context, pair tables, one tile list for the
// persistent bulk kernel (ordered by decreasing cost, so that small items fill
// the gaps left by large ones), per-item FP64 head/wings, and per-item
// assembly, inversion (one launch per inversion kernel class, covering every
// item of that class) and loss.  The sequence is captured into up to four
// hipGraphs (pair densities, operand preparation, the persistent bulk launch,
// everything after it) so that the stages can be timed on their own; later
// calls with the same
// signature replay them.  Capture records kernels only (counters and flags are
// reset by a one-thread kernel, not by memset nodes).
//
// Autotuning: the K split of every item follows from a target number of MFMA
// steps per split (more splits = more tiles to balance the persistent grid,
// fewer = less partial-sum traffic).  With autotuning on, a plan is built for
// each candidate target, its graphs are replayed and timed with HIP events,
// and the fastest plan is kept.
#include <chrono>

#include "ctx.h"

namespace qcx {

struct PlanItem {
  int ctx = 0;
  Chi0Geom g{};
  Geom64 g64{};
  int n_pairs64 = 0;
  double eta = 0.0, pref = 0.0;
  double* loss_out = nullptr;
  DevBuf w, A, Alo, pairs, rows, pairs64, C, XY, eps, diag, epsM, loss;
};

struct BatchPlan {
  std::vector<double> key;
  std::vector<qcx_ctx*> ctxs;  // the batch's contexts (part of the key)
  int precision = 0, lfe = 1, hw64 = 1, n_items = 0;
  std::vector<PlanItem> items;
  std::vector<DevBuf> r32;  // per context
  DevBuf d_items, d_tiles, d_counter, d_sing;
  static constexpr int kBranches = 4;  // parallel paths of a graph (see capture)
  DevBuf hwP[kBranches];  // pair-product tables of the head/wing GEMMs, one per path
  // multi-item inversion launches, one per kernel class present
  struct GjGroup {
    int cls = 0, n_jobs = 0, n_blocks = 0, max_n = 0;
    DevBuf jobs;
  };
  std::vector<GjGroup> gj;
  int n_tiles = 0, max_ng = 0, target_steps = 0, grid = 0;
  double tune_ms = 0.0;
  bool gather = false;
  bool rho = false;         // pair densities inside the plan (graph 0)
  std::vector<DevBuf> gs;   // per context: its G list (rho plans)
  static constexpr int kGraphs = 4;
  hipGraph_t graph[kGraphs] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t exec[kGraphs] = {nullptr, nullptr, nullptr, nullptr};
  ~BatchPlan() {
    for (int i = 0; i < kGraphs; ++i) {
      if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
      if (graph[i]) (void)hipGraphDestroy(graph[i]);
    }
    for (PlanItem& it : items) {
      DevBuf* b[] = {&it.w, &it.A, &it.Alo, &it.pairs, &it.rows, &it.pairs64, &it.C, &it.XY,
                     &it.eps, &it.diag, &it.epsM, &it.loss};
      for (DevBuf* x : b) x->release();
    }
    for (DevBuf& b : r32) b.release();
    for (DevBuf& b : gs) b.release();
    for (GjGroup& g : gj) g.jobs.release();
    d_items.release();
    d_tiles.release();
    for (DevBuf& b : hwP) b.release();
    d_counter.release();
    d_sing.release();
  }
};

void destroy_plan(BatchPlan* p) { delete p; }

namespace {

// Everything a plan's graphs bake in: buffer addresses, shapes, frequencies,
// output addresses, and for rho plans the G lists and what the pair-density
// kernels read (basis and state buffers, reciprocal vectors, M chunk buffer)
std::vector<double> batch_key(qcx_ctx* const* ctxs, int n_ctx, const qcx_item* items, int n_items,
                              int precision, int lfe, int hw64, const int* n_G,
                              const int* const* G_int) {
  std::vector<double> k = {(double)n_items, (double)precision, (double)lfe, (double)hw64,
                           (double)n_ctx, n_G ? 1.0 : 0.0};
  auto ptr = [&](const DevBuf& b) { k.push_back((double)(uintptr_t)b.p); };
  for (int c = 0; c < n_ctx; ++c) {
    const qcx_ctx* x = ctxs[c];
    k.push_back((double)(uintptr_t)x);
    k.push_back((double)(uintptr_t)x->d_R.p);
    k.push_back((double)(uintptr_t)x->d_dt.p);
    k.push_back((double)(uintptr_t)x->d_vq.p);
    k.push_back((double)x->n_g);
    k.push_back((double)x->n_t);
    k.push_back((double)x->ldt);
    k.push_back((double)x->n_k);
    k.push_back(x->vol);
    if (!n_G) continue;
    for (const DevBuf* b : {&x->d_qc, &x->d_Q, &x->d_F, &x->d_M, &x->d_Ck, &x->d_Ckq, &x->d_ph,
                            &x->d_shp, &x->d_tvec, &x->d_sh_l, &x->d_sh_ex, &x->d_sh_ctr,
                            &x->d_sh_off})
      ptr(*b);
    k.push_back((double)x->d_M.bytes);
    for (int v : {x->n_cells, x->n_sh, x->n_ao, x->n_b, x->n_occ}) k.push_back((double)v);
    for (int i = 0; i < 9; ++i) k.push_back(x->rec[i]);
    for (int i = 0; i < 3 * n_G[c]; ++i) k.push_back((double)G_int[c][i]);
  }
  for (int i = 0; i < n_items; ++i) {
    k.push_back((double)items[i].ctx);
    k.push_back((double)items[i].n_w);
    k.push_back(items[i].eta_eV);
    k.push_back((double)(uintptr_t)items[i].loss_out);
    for (int j = 0; j < items[i].n_w; ++j) k.push_back(items[i].w_eV[j]);
  }
  return k;
}

// K split of one item: the largest power of two (up to 64) that keeps at
// least target_steps MFMA steps per split, raised until no split sums more
// than 1024 steps in FP32 (the splits are added in FP64 by the assembly).
int ksplit_for(int ntb, int target_steps) {
  int ks = 1;
  while (ks < kMaxKsplit && ntb / (2 * ks) >= target_steps) ks *= 2;
  while (ks < kMaxKsplit && ntb > ks * 1024) ks *= 2;
  return ks;
}

// Streams of one capture: the capturing stream and kBranches streams forked
// from it.  Work enqueued on different branches between a fork() and the next
// join() forms independent paths of the graph (no order between them), so
// that small per-item kernels can overlap; join() makes the main stream wait
// for every branch (nothing if none was forked).
struct Branches {
  hipStream_t main = nullptr;
  hipStream_t br[BatchPlan::kBranches] = {};
  std::vector<hipEvent_t> events;
  hipError_t err = hipSuccess;
  bool forked = false;
  hipStream_t operator[](int i) const { return br[i % BatchPlan::kBranches]; }
  void chk(hipError_t e) {
    if (err == hipSuccess) err = e;
  }
  hipEvent_t event() {
    hipEvent_t ev = nullptr;
    chk(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    events.push_back(ev);
    return ev;
  }
  void fork() {
    hipEvent_t ev = event();
    chk(hipEventRecord(ev, main));
    for (hipStream_t b : br) chk(hipStreamWaitEvent(b, ev, 0));
    forked = true;
  }
  void join() {
    if (!forked) return;
    forked = false;
    for (hipStream_t b : br) {
      hipEvent_t ev = event();
      chk(hipEventRecord(ev, b));
      chk(hipStreamWaitEvent(main, ev, 0));
    }
  }
};

// Capture the work enqueued by fn(Branches&) into P->graph[i] and
// instantiate it; the capture runs on private streams (the caller's stream
// may be the legacy default stream, which cannot be captured), and branches
// left open by fn are joined at the end.
template <class F>
int capture(qcx_ctx* ctx, BatchPlan* P, int i, F&& fn) {
  Branches B;
  HIPCK(hipStreamCreateWithFlags(&B.main, hipStreamNonBlocking));
  for (hipStream_t& b : B.br) B.chk(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
  auto cleanup = [&]() {
    for (hipStream_t b : B.br)
      if (b) (void)hipStreamDestroy(b);
    (void)hipStreamDestroy(B.main);
    for (hipEvent_t ev : B.events) (void)hipEventDestroy(ev);
  };
  hipError_t e = B.err != hipSuccess ? B.err : hipStreamBeginCapture(B.main, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    cleanup();
    return fail(ctx, QCX_EDEVICE, std::string("begin capture: ") + hipGetErrorString(e));
  }
  fn(B);
  B.join();
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(B.main, &graph);
  if (e == hipSuccess) e = B.err;
  cleanup();
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(ctx, QCX_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  P->graph[i] = graph;
  e = hipGraphInstantiate(&P->exec[i], graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return fail(ctx, QCX_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  return QCX_OK;
}

// Replay a plan on the context's stream; timed spans (when timing is on):
// stage 0 the pair densities (rho plans), stage 1 the persistent bulk launch,
// stage 4 head/wings + assembly + inversion + loss, stage 3 the whole batch.
hipError_t launch_plan(qcx_ctx* ctx, const BatchPlan* P) {
  static constexpr int stage_of[BatchPlan::kGraphs] = {0, -1, 1, 4};
  int sp_all = -1, sp = -1;
  hipError_t e = span_begin(ctx, 3, &sp_all);
  if (e != hipSuccess) return e;
  for (int i = 0; i < BatchPlan::kGraphs; ++i) {
    if (!P->exec[i]) continue;
    const bool span = stage_of[i] >= 0;
    if (span && (e = span_begin(ctx, stage_of[i], &sp)) != hipSuccess) return e;
    if ((e = hipGraphLaunch(P->exec[i], ctx->stream)) != hipSuccess) return e;
    if (span && (e = span_end(ctx, sp)) != hipSuccess) return e;
  }
  return span_end(ctx, sp_all);
}

int build_plan(qcx_ctx* ctx, qcx_ctx* const* ctxs, int n_ctx, const qcx_item* items, int n_items,
               int precision, int lfe, int hw64, int target_steps, const int* n_G,
               const int* const* G_int, BatchPlan* P) {
  hipStream_t st = ctx->stream;
  P->rho = n_G != nullptr;
  P->target_steps = target_steps;
  P->precision = precision;
  P->lfe = lfe;
  P->hw64 = hw64;
  P->n_items = n_items;
  P->items.resize(n_items);
  P->r32.resize(n_ctx);
  const bool bulk = precision != QCX_FP64;
  const bool bf = precision == QCX_SPLIT_BF16;
  std::vector<int> ctx_ntp(n_ctx, 0);
  std::vector<BulkItem> bitems(n_items);
  std::vector<int4> tiles;
  // one bulk kernel serves every item: row-gather mode for all of them when
  // any item is large
  if (bulk)
    for (int i = 0; i < n_items; ++i)
      P->gather = P->gather || ctxs[items[i].ctx]->n_g >= kGatherMinNg;
  HIPCK(stage_begin(ctx));
  if (P->rho) {
    P->gs.resize(n_ctx);
    for (int c = 0; c < n_ctx; ++c) HIPCK(upload(ctx, P->gs[c], G_int[c], 3 * (size_t)n_G[c]));
  }
  for (int i = 0; i < n_items; ++i) {
    PlanItem& it = P->items[i];
    const qcx_item& in = items[i];
    qcx_ctx* c = ctxs[in.ctx];
    it.ctx = in.ctx;
    it.eta = in.eta_eV / kHartreeEV;
    it.pref = 2.0 / (c->n_k * c->vol);
    it.loss_out = in.loss_out;
    std::vector<double> w(in.n_w);
    for (int j = 0; j < in.n_w; ++j) w[j] = in.w_eV[j] / kHartreeEV;
    HIPCK(upload(ctx, it.w, w.data(), w.size()));
    Chi0Geom& g = it.g;
    g = Chi0Geom{};
    g.n_g = c->n_g;
    g.n_t = c->n_t;
    g.n_w = in.n_w;
    g.n_rows = 2 * in.n_w;
    g.n_pairs = c->n_g * (c->n_g + 1) / 2;
    it.n_pairs64 = bulk ? (hw64 ? c->n_g : 0) : g.n_pairs;
    g.p0 = bulk ? it.n_pairs64 : g.n_pairs;
    g.n_bulk = g.n_pairs - g.p0;
    g.n_bulkp = (int)roundup(std::max(g.n_bulk, 1), 128);
    if (bulk && g.n_bulk > 0) {
      g.n_rowsp = (int)roundup(g.n_rows, 32 * kBatchAF);
      g.c_rows = g.n_rowsp;
      const int ntb0 = (int)roundup(g.n_t, 16) / 16;
      g.ksplit = ksplit_for(ntb0, target_steps);
      g.n_tp = (int)roundup(g.n_t, 16 * g.ksplit);
      ctx_ntp[in.ctx] = std::max(ctx_ntp[in.ctx], g.n_tp);
      const size_t nA = (size_t)g.n_rowsp * g.n_tp;
      HIPCK(it.A.reserve(sizeof(uint16_t) * nA * (bf ? 1 : 2)));
      if (bf) HIPCK(it.Alo.reserve(sizeof(uint16_t) * nA));
      HIPCK(it.C.reserve(sizeof(float) * (size_t)g.ksplit * g.n_rowsp * 2 * g.n_bulkp));
      std::vector<int> pr(g.n_bulkp, 0);
      int b = 0, p = 0;
      for (int G = 0; G < g.n_g; ++G)
        for (int Gp = G; Gp < g.n_g; ++Gp, ++p)
          if (p >= g.p0) pr[b++] = G | (Gp << 16);
      g.gather = P->gather ? 1 : 0;
      if (P->gather) {
        std::vector<int> local, rows;
        if (!bulk_gather_tables(pr, local, rows))
          return fail(ctx, QCX_EDEVICE, "internal: a pair tile needs more rows than staged");
        HIPCK(upload(ctx, it.pairs, local.data(), local.size()));
        HIPCK(upload(ctx, it.rows, rows.data(), rows.size()));
      } else {
        HIPCK(upload(ctx, it.pairs, pr.data(), pr.size()));
      }
      for (int z = 0; z < g.ksplit; ++z)
        for (int y = 0; y < g.n_rowsp / (32 * kBatchAF); ++y)
          for (int x = 0; x < g.n_bulkp / 128; ++x) tiles.push_back(make_int4(i, x, y, z));
      P->max_ng = std::max(P->max_ng, g.n_g);
    } else {
      g.ksplit = 1;
      g.n_rowsp = 0;
      g.n_tp = (int)roundup(g.n_t, 16);
    }
    if (it.n_pairs64 > 0) {
      if (it.n_pairs64 == c->n_g) {
        geom_hw_init(it.g64, c->n_g, in.n_w, c->n_t, it.n_pairs64, (size_t)256 << 20);
        HIPCK(P->hwP[i % BatchPlan::kBranches].reserve(sizeof(double) * hw_ptable_doubles(it.g64)));
      } else {
        geom64_init(it.g64, c->n_g, in.n_w, c->n_t, it.n_pairs64, (size_t)256 << 20);
      }
      std::vector<int> tab(it.n_pairs64);
      int p = 0;
      for (int G = 0; G < c->n_g && p < it.n_pairs64; ++G)
        for (int Gp = G; Gp < c->n_g && p < it.n_pairs64; ++Gp, ++p) tab[p] = G | (Gp << 16);
      HIPCK(upload(ctx, it.pairs64, tab.data(), tab.size()));
      HIPCK(it.XY.reserve(sizeof(double) * (size_t)it.g64.ksplit * it.g64.n_rowsp *
                          it.g64.n_colp));
    }
    const int n = c->n_g;
    HIPCK(it.eps.reserve(sizeof(cplx) * (size_t)in.n_w * n * n));
    HIPCK(it.diag.reserve(sizeof(cplx) * (size_t)in.n_w * n));
    HIPCK(it.epsM.reserve(sizeof(cplx) * (size_t)in.n_w));
    if (!it.loss_out) HIPCK(it.loss.reserve(sizeof(double) * (size_t)in.n_w * n));
  }
  for (int c = 0; c < n_ctx; ++c)
    if (ctx_ntp[c] > 0)
      HIPCK(P->r32[c].reserve(sizeof(float) * 2 * (size_t)ctxs[c]->n_g * ctx_ntp[c]));
  for (int i = 0; i < n_items; ++i) {
    PlanItem& it = P->items[i];
    bitems[i] = BulkItem{it.A.as<float4>(), it.Alo.as<float4>(), P->r32[it.ctx].as<float4>(),
                         it.pairs.as<int>(), P->gather ? it.rows.as<int>() : nullptr, it.g,
                         it.C.as<float>()};
  }
  // cost order: longest K range first (all tiles of one item are equal)
  std::stable_sort(tiles.begin(), tiles.end(), [&](const int4& a, const int4& b) {
    const Chi0Geom& ga = P->items[a.x].g;
    const Chi0Geom& gb = P->items[b.x].g;
    return (ga.n_tp / ga.ksplit) > (gb.n_tp / gb.ksplit);
  });
  P->n_tiles = (int)tiles.size();
  HIPCK(upload(ctx, P->d_items, bitems.data(), bitems.size()));
  if (!tiles.empty()) HIPCK(upload(ctx, P->d_tiles, tiles.data(), tiles.size()));
  HIPCK(P->d_counter.reserve(sizeof(int)));
  HIPCK(P->d_sing.reserve(sizeof(int) * (size_t)n_items));
  // inversions: items of one kernel class share a launch, so that small items
  // do not leave the chip idle one after another
  std::vector<int> single_gj;  // items whose size has no multi-item kernel
  if (lfe) {
    std::vector<std::vector<GjJob>> by(8);
    std::vector<int> blocks(8, 0), maxn(8, 0);
    for (int i = 0; i < n_items; ++i) {
      PlanItem& it = P->items[i];
      const int n = ctxs[it.ctx]->n_g, cls = gj_class(n);
      if (cls >= 8) {
        single_gj.push_back(i);
        continue;
      }
      by[cls].push_back(GjJob{it.eps.as<cplx>(), it.diag.as<cplx>(), P->d_sing.as<int>() + i, n,
                              it.g.n_w, blocks[cls]});
      blocks[cls] += it.g.n_w;
      maxn[cls] = std::max(maxn[cls], n);
    }
    for (int c = 0; c < 8; ++c) {
      if (by[c].empty()) continue;
      BatchPlan::GjGroup g;
      g.cls = c;
      g.n_jobs = (int)by[c].size();
      g.n_blocks = blocks[c];
      g.max_n = maxn[c];
      HIPCK(upload(ctx, g.jobs, by[c].data(), by[c].size()));
      P->gj.push_back(std::move(g));
    }
  }
  HIPCK(hipStreamSynchronize(st));  // uploads complete before capture begins

  P->grid = std::min(P->n_tiles, 2 * 256);
  if (P->rho) {
    int rc_in = QCX_OK, c_bad = 0;
    int rc = capture(ctx, P, 0, [&](Branches& B) {
      B.fork();
      for (int c = 0; c < n_ctx && rc_in == QCX_OK; ++c)
        if ((rc_in = rho_enqueue(ctxs[c], P->gs[c].as<int>(), n_G[c], false, B[c])) != QCX_OK) c_bad = c;
    });
    if (rc != QCX_OK) return rc;
    if (rc_in != QCX_OK)
      return fail(ctx, rc_in, "context " + std::to_string(c_bad) + ": " + ctxs[c_bad]->err);
  }
  if (bulk) {
    int rc = capture(ctx, P, 1, [&](Branches& B) {
      B.fork();
      for (int c = 0; c < n_ctx; ++c) {
        if (ctx_ntp[c] == 0) continue;
        Chi0Geom gp{};
        gp.n_g = ctxs[c]->n_g;
        gp.n_tp = ctx_ntp[c];
        launch_pack_r32(ctxs[c]->d_R.as<cplx>(), ctxs[c]->ldt, gp, bf ? 0 : 1,
                        P->r32[c].as<float>(), B[c]);
      }
      for (int i = 0; i < n_items; ++i) {
        PlanItem& it = P->items[i];
        qcx_ctx* c = ctxs[it.ctx];
        if (it.g.n_bulk == 0) continue;
        if (bf)
          launch_weights_bf16(it.w.as<double>(), c->d_dt.as<double>(), it.eta, it.g,
                              it.A.as<uint16_t>(), it.Alo.as<uint16_t>(), B[i]);
        else
          launch_weights_f32(it.w.as<double>(), c->d_dt.as<double>(), it.eta, it.g,
                             it.A.as<float>(), B[i]);
      }
    });
    if (rc != QCX_OK) return rc;
  }
  if (P->n_tiles > 0) {
    int rc = capture(ctx, P, 2, [&](Branches& B) {
      launch_set_int(P->d_counter.as<int>(), 0, B.main);
      launch_bulk_persistent(bf, P->gather, P->d_items.as<BulkItem>(), P->d_tiles.as<int4>(),
                             P->n_tiles, P->d_counter.as<int>(), P->max_ng, P->grid, B.main);
    });
    if (rc != QCX_OK) return rc;
  }
  return capture(ctx, P, 3, [&](Branches& B) {
    // per item, each on one path: head/wings (or every pair in FP64), then
    // the assembly of eps
    B.fork();
    for (int i = 0; i < n_items; ++i) {
      PlanItem& it = P->items[i];
      qcx_ctx* c = ctxs[it.ctx];
      hipStream_t cs = B[i];
      if (it.n_pairs64 > 0 && it.n_pairs64 == c->n_g)
        launch_headwings_f64(c->d_R.as<cplx>(), c->ldt, it.w.as<double>(), c->d_dt.as<double>(),
                             it.eta, it.g64, it.pairs64.as<int>(),
                             P->hwP[i % BatchPlan::kBranches].as<double>(), it.XY.as<double>(), cs);
      else if (it.n_pairs64 > 0)
        launch_pairs_f64(c->d_R.as<cplx>(), c->ldt, it.w.as<double>(), c->d_dt.as<double>(),
                         it.eta, it.g64, it.pairs64.as<int>(), it.XY.as<double>(), cs);
      launch_set_int(P->d_sing.as<int>() + i, INT_MAX, cs);
      AsmArgs a{};
      a.C = (bulk && it.g.n_bulk > 0) ? it.C.as<float>() : nullptr;
      a.XY = it.n_pairs64 > 0 ? it.XY.as<double>() : nullptr;
      a.ks = it.g.ksplit;
      a.ks64 = it.g64.ksplit;
      a.n_rowsp64 = it.g64.n_rowsp;
      a.n_colp64 = it.g64.n_colp;
      a.n_pairs64 = it.n_pairs64;
      a.vq = c->d_vq.as<double>();
      a.pref = it.pref;
      launch_eps_assemble(a, it.g, it.eps.as<cplx>(), cs);
    }
    B.join();
    hipStream_t cs = B.main;
    if (lfe) {
      for (const BatchPlan::GjGroup& g : P->gj)
        launch_gj_jobs(g.cls, g.jobs.as<GjJob>(), g.n_jobs, g.n_blocks, g.max_n, cs);
      for (int i : single_gj) {
        PlanItem& it = P->items[i];
        launch_gj_diag(it.eps.as<cplx>(), ctxs[it.ctx]->n_g, it.g.n_w, it.diag.as<cplx>(),
                       P->d_sing.as<int>() + i, cs);
      }
    }
    for (int i = 0; i < n_items; ++i) {
      PlanItem& it = P->items[i];
      qcx_ctx* c = ctxs[it.ctx];
      if (!lfe)
        launch_nolfe_diag(it.eps.as<cplx>(), c->n_g, it.g.n_w, it.diag.as<cplx>(),
                          P->d_sing.as<int>() + i, cs);
      launch_loss(it.diag.as<cplx>(), c->n_g, it.g.n_w,
                  it.loss_out ? it.loss_out : it.loss.as<double>(), it.epsM.as<cplx>(), cs);
    }
  });
}

// Time one plan: one warm replay, then the mean of two timed replays (ms).
int time_plan(qcx_ctx* ctx, const BatchPlan* P, double* ms) {
  const bool was = ctx->timing;
  ctx->timing = false;
  hipEvent_t a = nullptr, b = nullptr;
  HIPCK(hipEventCreate(&a));
  HIPCK(hipEventCreate(&b));
  hipError_t e = launch_plan(ctx, P);
  if (e == hipSuccess) e = hipEventRecord(a, ctx->stream);
  for (int r = 0; r < 2 && e == hipSuccess; ++r) e = launch_plan(ctx, P);
  if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  ctx->timing = was;
  HIPCK(e);
  *ms = 0.5 * t;
  return QCX_OK;
}

// Both batch entry points; n_G and G_int are null for qcx_run_batch
int run_batch_impl(qcx_ctx* const* ctxs, int n_ctx, const int* n_G, const int* const* G_int,
                   const qcx_item* items, int n_items, int precision, int headwings_fp64, int lfe) {
  if (!ctxs || n_ctx < 1 || !ctxs[0]) return QCX_EINVAL;
  qcx_ctx* ctx = ctxs[0];
  if (!items || n_items < 1) return fail(ctx, QCX_EINVAL, "no items");
  if (precision < QCX_FP64 || precision > QCX_SPLIT_BF16) return fail(ctx, QCX_EINVAL, "bad precision");
  for (int c = 0; c < n_ctx; ++c) {
    if (!ctxs[c]) return fail(ctx, QCX_EINVAL, "NULL context");
    if (ctxs[c]->device != ctx->device) return fail(ctx, QCX_EINVAL, "contexts on different devices");
    const std::string cs = "context " + std::to_string(c);
    for (int d = 0; d < c; ++d)
      if (n_G && ctxs[d] == ctxs[c]) return fail(ctx, QCX_EINVAL, cs + " is listed twice");
    if (n_G) {
      if (!ctxs[c]->have_states) return fail(ctx, QCX_ESTATE, cs + " has no states");
      if (!G_int[c]) return fail(ctx, QCX_EINVAL, cs + ": NULL G list");
    } else if (!ctxs[c]->have_rho) {
      return fail(ctx, QCX_ESTATE, cs + " has no pair densities");
    }
    const int ng = n_G ? n_G[c] : ctxs[c]->n_g;
    if (lfe && ng > 1024) return fail(ctx, QCX_EINVAL, "LFE inversion limited to n_G <= 1024");
  }
  for (int i = 0; i < n_items; ++i) {
    const qcx_item& it = items[i];
    if (it.ctx < 0 || it.ctx >= n_ctx) return fail(ctx, QCX_EINVAL, "item context out of range");
    if (it.n_w < 1 || it.n_w > 65536 || !it.w_eV) return fail(ctx, QCX_EINVAL, "item frequencies");
    if (!(it.eta_eV >= 0.0)) return fail(ctx, QCX_EINVAL, "item eta");
    if (!it.loss_out) return fail(ctx, QCX_EINVAL, "item loss_out must be a device buffer");
    for (int j = 0; j < it.n_w; ++j)
      if (!std::isfinite(it.w_eV[j])) return fail(ctx, QCX_EINVAL, "non-finite frequency");
  }
  HIPCK(hipSetDevice(ctx->device));
  // the G lists: host checks against each context's q, buffers sized
  for (int c = 0; n_G && c < n_ctx; ++c)
    if (int rc = rho_prepare(ctxs[c], n_G[c], G_int[c], true, false))
      return fail(ctx, rc, "context " + std::to_string(c) + ": " + ctxs[c]->err);
  const int hw64 = headwings_fp64 ? 1 : 0;
  std::vector<double> key =
      batch_key(ctxs, n_ctx, items, n_items, precision, lfe ? 1 : 0, hw64, n_G, G_int);
  // the other contexts' pair densities and energies were produced on their
  // own streams: the batch (on ctxs[0]'s stream) waits for them
  std::vector<hipStream_t> others;
  for (int c = 1; c < n_ctx; ++c) {
    hipStream_t s = ctxs[c]->stream;
    if (s != ctx->stream && std::find(others.begin(), others.end(), s) == others.end()) {
      others.push_back(s);
      if (!ctxs[c]->ev_order) HIPCK(hipEventCreateWithFlags(&ctxs[c]->ev_order, hipEventDisableTiming));
      HIPCK(hipEventRecord(ctxs[c]->ev_order, s));
      HIPCK(hipStreamWaitEvent(ctx->stream, ctxs[c]->ev_order, 0));
    }
  }
  if (!ctx->plan || ctx->plan->key != key) {
    // building a plan stages host tables and captures graphs of its own
    if (int rc = reject_capture(ctx)) return rc;
    if (ctx->plan) destroy_plan(ctx->plan);
    ctx->plan = nullptr;
    const bool tune = ctx->autotune && precision != QCX_FP64;
    std::vector<int> cands = tune ? std::vector<int>{128, 256, 512, 1024} : std::vector<int>{256};
    const auto t0 = std::chrono::steady_clock::now();
    BatchPlan* best = nullptr;
    double best_ms = 0.0;
    for (int target : cands) {
      BatchPlan* P = new BatchPlan();
      P->key = key;
      int rc = build_plan(ctx, ctxs, n_ctx, items, n_items, precision, lfe ? 1 : 0, hw64, target,
                          n_G, G_int, P);
      double ms = 0.0;
      if (rc == QCX_OK && cands.size() > 1) rc = time_plan(ctx, P, &ms);
      if (rc != QCX_OK) {
        destroy_plan(P);
        if (best) destroy_plan(best);
        return rc;
      }
      if (!best || ms < best_ms) {
        if (best) destroy_plan(best);
        best = P;
        best_ms = ms;
      } else {
        destroy_plan(P);
      }
    }
    best->tune_ms = cands.size() > 1
                        ? std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count()
                        : 0.0;
    best->ctxs.assign(ctxs, ctxs + n_ctx);
    ctx->plan = best;
  }
  HIPCK(launch_plan(ctx, ctx->plan));
  for (int c = 0; n_G && c < n_ctx; ++c) ctxs[c]->have_rho = true;
  // and the other streams do not overwrite those buffers before the batch
  // has read them
  if (!others.empty()) {
    if (!ctx->ev_order) HIPCK(hipEventCreateWithFlags(&ctx->ev_order, hipEventDisableTiming));
    HIPCK(hipEventRecord(ctx->ev_order, ctx->stream));
    for (hipStream_t s : others) HIPCK(hipStreamWaitEvent(s, ctx->ev_order, 0));
  }
  return QCX_OK;
}

}  // namespace
}  // namespace qcx

extern "C" {

int qcx_run_batch(qcx_ctx* const* ctxs, int n_ctx, const qcx_item* items, int n_items,
                  int precision, int headwings_fp64, int lfe) {
  return run_batch_impl(ctxs, n_ctx, nullptr, nullptr, items, n_items, precision, headwings_fp64, lfe);
}

int qcx_run_batch_rho(qcx_ctx* const* ctxs, int n_ctx, const int* n_G, const int* const* G_int,
                      const qcx_item* items, int n_items, int precision, int headwings_fp64,
                      int lfe) {
  if (!ctxs || n_ctx < 1 || !ctxs[0]) return QCX_EINVAL;
  if (!n_G || !G_int) return fail(ctxs[0], QCX_EINVAL, "NULL G lists");
  return run_batch_impl(ctxs, n_ctx, n_G, G_int, items, n_items, precision, headwings_fp64, lfe);
}

int qcx_batch_config(qcx_ctx* ctx, int cfg[3], double* tune_ms) {
  if (!ctx || !cfg) return QCX_EINVAL;
  if (!ctx->plan) return fail(ctx, QCX_ESTATE, "no batch has run on this context");
  cfg[0] = ctx->plan->target_steps;
  cfg[1] = ctx->plan->n_tiles;
  cfg[2] = ctx->plan->grid;
  if (tune_ms) *tune_ms = ctx->plan->tune_ms;
  return QCX_OK;
}

int qcx_batch_sync(qcx_ctx* ctx) {
  if (!ctx) return QCX_EINVAL;
  HIPCK(hipSetDevice(ctx->device));
  HIPCK(hipStreamSynchronize(ctx->stream));
  if (int rc = check_deferred(ctx)) return rc;
  if (!ctx->plan) return QCX_OK;
  // deferred state checks of every context of the batch (their streams were
  // waited for by the batch itself)
  for (size_t c = 1; c < ctx->plan->ctxs.size(); ++c) {
    qcx_ctx* x = ctx->plan->ctxs[c];
    if (x == ctx) continue;
    HIPCK(hipStreamSynchronize(x->stream));
    if (int rc = check_deferred(x)) return fail(ctx, rc, "context " + std::to_string(c) + ": " + x->err);
  }
  std::vector<int> s(ctx->plan->n_items);
  HIPCK(hipMemcpy(s.data(), ctx->plan->d_sing.p, sizeof(int) * s.size(), hipMemcpyDeviceToHost));
  for (size_t i = 0; i < s.size(); ++i)
    if (s[i] != INT_MAX)
      return fail(ctx, QCX_ESINGULAR, "zero pivot in item " + std::to_string(i) + " at frequency index " +
                                          std::to_string(s[i]));
  return QCX_OK;
}

}  // extern "C"
