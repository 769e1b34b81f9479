// Host runtime behind the C ABI declared in include/qcx.h: context, device
// buffers, input validation, orchestration of the kernels on the caller's
// stream and per-stage HIP-event timing.
#include <limits.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <chrono>

#include "ctx.h"
#include "kk.h"

namespace {
std::string g_create_err;
}  // namespace

// Read back the deferred checks of device-resident states (stream already
// synchronised by the caller) and reset them.
int qcx::check_deferred(qcx_ctx* ctx) {
  if (!ctx->check_pending) return QCX_OK;
  int f[2] = {INT_MAX, INT_MAX};
  HIPCK(hipMemcpy(f, ctx->d_flags.p, sizeof(f), hipMemcpyDeviceToHost));
  const int reset[2] = {INT_MAX, INT_MAX};
  HIPCK(hipMemcpy(ctx->d_flags.p, reset, sizeof(reset), hipMemcpyHostToDevice));
  ctx->check_pending = false;
  if (f[0] != INT_MAX || f[1] != INT_MAX) {
    ctx->have_states = ctx->have_rho = ctx->have_chi0 = ctx->have_eps = false;
    if (f[0] != INT_MAX)
      return fail(ctx, QCX_EINVAL, "device states: non-finite energy or an empty band below an "
                                   "occupied band at k " + std::to_string(f[0]));
    const int nk = ctx->check_nk;
    return fail(ctx, QCX_ENONORTH,
                std::string("device states at ") + (f[1] < nk ? "k " : "k+q ") +
                    std::to_string(f[1] % nk) + " are not orthonormal (max|C^H S C - I| > 1e-10)");
  }
  return QCX_OK;
}

static int pick_ksplit(int blocks, int steps) {
  int ks = 1;
  while (ks < 16 && blocks * ks < 1024 && steps / (2 * ks) >= 8) ks *= 2;
  return ks;
}

// ---------------------------------------------------------------------------
// Autotuner of the bulk launch: per (device, precision, N_G, padded N_T,
// padded rows) shape, every candidate (K split, LDS pipeline depth) is timed
// on the real operands with HIP events and the fastest is kept for the
// process.  The weights and R slabs are padded to a multiple of 256
// transitions, so every K split up to 16 divides the same operands.
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
  int dev, prec, n_g, n_tp, n_rowsp, n_bulkp;
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, prec, n_g, n_tp, n_rowsp, n_bulkp) <
           std::tie(o.dev, o.prec, o.n_g, o.n_tp, o.n_rowsp, o.n_bulkp);
  }
};
struct TuneVal {
  int ks, nst;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

// FP32 partial sums of one launch are kept within this budget; larger shapes
// run in chunks of frequency rows, each reduced into FP64 partials
constexpr size_t kPartialBudget = (size_t)8 << 30;
// Kramers-Kronig route: bins per side, transitions per binning chunk, and the
// largest binned spectral function S[bins][2][pairs] held in HBM
constexpr int kKkMaxBins = 1 << 20;
constexpr int kKkChunkT = 256;
constexpr double kKkSpectralBudget = 16.0 * (1 << 30);
// Accuracy: one K split sums at most this many K steps (16 transitions
// each) in its FP32 accumulators; the splits are added in FP64
constexpr int kMaxStepsPerSplit = 1024;
constexpr size_t kLdsBytes = 160 * 1024;
// Bloch sums M(k; G) of one pass of the pair densities when they are not
// fused with the band contraction (k points in chunks within this budget)
constexpr size_t kMBudget = (size_t)8 << 30;

struct Cand {
  int ks, nst;
};

// smallest K split (power of two) that keeps every split within
// kMaxStepsPerSplit sequential FP32 accumulations
int ksplit_for_accuracy(int ntb) {
  int ks = 1;
  while (ks < kMaxKsplit && (size_t)ntb > (size_t)ks * kMaxStepsPerSplit) ks *= 2;
  return ks;
}

std::vector<Cand> bulk_candidates(const Chi0Geom& g, int af, int ks_min) {
  std::vector<Cand> c;
  const int ntb = g.n_tp / KSTEP_T;
  for (int ks = ks_min; ks <= kMaxKsplit; ks *= 2) {
    if (ks > ks_min && ntb / ks < 4) break;
    if (ks > ks_min && (size_t)ks * g.c_rows * 2 * g.n_bulkp * sizeof(float) > kPartialBudget)
      break;
    for (int nst = 2; nst <= 4; ++nst)  // 4: three stages, slab one step ahead
      if (bulk_lds_bytes(g.n_g, af, nst) <= kLdsBytes) c.push_back({ks, nst});
  }
  return c;
}
}  // namespace

extern "C" {

const char* qcx_build_info(void) {
  return "libqcx gfx950: rho FP64 (Hermite FT, 27-cell Bloch sum on FP64 MFMA fused with the "
         "band contraction), chi0 bulk FP32-MFMA "
         "32x32x2 / split-BF16-MFMA 32x32x16 (hi*hi+hi*lo+lo*hi), FP64 head/wings, FP64 "
         "Gauss-Jordan diag(eps^-1)";
}

int qcx_create(qcx_ctx** out, int device, void* hip_stream) {
  if (!out) {
    g_create_err = "out is NULL";
    return QCX_EINVAL;
  }
  *out = nullptr;
  int n = 0;
  const hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) {
    g_create_err = std::string("hipGetDeviceCount: ") + hipGetErrorString(e);
    return QCX_EDEVICE;
  }
  if (device < 0 || device >= n) {
    g_create_err = "no such HIP device";
    return QCX_EINVAL;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    g_create_err = "hipGetDeviceProperties failed";
    return QCX_EDEVICE;
  }
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_create_err = std::string("library built for gfx950, device is ") + prop.gcnArchName;
    return QCX_EDEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) {
    g_create_err = "hipSetDevice failed";
    return QCX_EDEVICE;
  }
  if (const hipError_t es = qcx::noalloc_init(device); es != hipSuccess) {
    g_create_err = std::string("scratch address: ") + hipGetErrorString(es);
    return QCX_EDEVICE;
  }
  qcx_ctx* c = new qcx_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  *out = c;
  return QCX_OK;
}

int qcx_destroy(qcx_ctx* ctx) {
  if (!ctx) return QCX_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return QCX_OK;
}

const char* qcx_last_error(const qcx_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int qcx_set_timing(qcx_ctx* ctx, int enable) {
  if (!ctx) return QCX_EINVAL;
  HIPCK(spans_resolve(ctx));
  ctx->timing = enable != 0;
  for (double& t : ctx->t_acc) t = 0.0;
  return QCX_OK;
}

int qcx_set_autotune(qcx_ctx* ctx, int mode) {
  if (!ctx) return QCX_EINVAL;
  if (mode != 0 && mode != 1) return fail(ctx, QCX_EINVAL, "mode must be 0 or 1");
  ctx->autotune = mode;
  return QCX_OK;
}

int qcx_set_bulk_pipeline(qcx_ctx* ctx, int nst) {
  if (!ctx) return QCX_EINVAL;
  if (nst != 0 && (nst < 2 || nst > 4)) return fail(ctx, QCX_EINVAL, "pipeline must be 0, 2, 3 or 4");
  ctx->force_nst = nst;
  return QCX_OK;
}

int qcx_bulk_config(qcx_ctx* ctx, int cfg[3], double* tune_ms) {
  if (!ctx || !cfg) return QCX_EINVAL;
  if (!ctx->have_chi0) return fail(ctx, QCX_ESTATE, "chi0 first");
  const bool bulk = ctx->geom.n_bulk > 0;
  cfg[0] = bulk ? ctx->geom.ksplit : 0;
  cfg[1] = bulk ? ctx->bulk_nst : 0;
  cfg[2] = bulk ? ctx->bulk_af : 0;
  if (tune_ms) *tune_ms = ctx->tune_ms;
  return QCX_OK;
}

int qcx_stage_times(qcx_ctx* ctx, double t[7]) {
  if (!ctx || !t) return QCX_EINVAL;
  HIPCK(spans_resolve(ctx));
  for (int i = 0; i < 7; ++i) t[i] = ctx->t_acc[i];
  return QCX_OK;
}

int qcx_sync(qcx_ctx* ctx) {
  if (!ctx) return QCX_EINVAL;
  HIPCK(hipSetDevice(ctx->device));
  HIPCK(hipStreamSynchronize(ctx->stream));
  if (int rc = check_deferred(ctx)) return rc;
  if (ctx->sing_armed && ctx->d_sing.p) {
    int s = INT_MAX;
    HIPCK(hipMemcpy(&s, ctx->d_sing.p, sizeof(int), hipMemcpyDeviceToHost));
    if (s != INT_MAX) {
      // reported once; a later inversion arms the flag again
      ctx->sing_armed = false;
      return fail(ctx, QCX_ESINGULAR,
                  "zero or non-finite pivot in eps at frequency index " + std::to_string(s));
    }
  }
  return QCX_OK;
}

int qcx_set_cell_basis(qcx_ctx* ctx, const double lat[9], int n_atoms, const double* xyz,
                       int n_shells, const int* shell_atom, const int* shell_l,
                       const double* shell_exp, int pure_d, int lattice_range) {
  if (!ctx) return QCX_EINVAL;
  if (!lat || !xyz || !shell_atom || !shell_l || !shell_exp)
    return fail(ctx, QCX_EINVAL, "NULL argument");
  if (n_atoms < 1 || n_shells < 1) return fail(ctx, QCX_EINVAL, "need atoms and shells");
  if (pure_d != 1) return fail(ctx, QCX_EINVAL, "only pure (spherical) d shells are supported");
  if (lattice_range < 0 || lattice_range > 3)
    return fail(ctx, QCX_EINVAL, "lattice_range must be 0..3");
  const double det = lat[0] * (lat[4] * lat[8] - lat[5] * lat[7]) -
                     lat[1] * (lat[3] * lat[8] - lat[5] * lat[6]) +
                     lat[2] * (lat[3] * lat[7] - lat[4] * lat[6]);
  if (!(fabs(det) > 1e-12)) return fail(ctx, QCX_EINVAL, "singular lattice");
  if (int rc = reject_capture(ctx)) return rc;
  HIPCK(hipSetDevice(ctx->device));
  ctx->have_basis = ctx->have_states = ctx->have_rho = ctx->have_chi0 = ctx->have_eps = false;
  ctx->f0_valid = false;
  memcpy(ctx->lat, lat, sizeof(double) * 9);
  double inv[9];
  inv3(lat, inv);
  // rows b_j = 2 pi (inv^T)_j
  for (int j = 0; j < 3; ++j)
    for (int x = 0; x < 3; ++x) ctx->rec[3 * j + x] = 2.0 * kPi * inv[3 * x + j];
  ctx->vol = fabs(det);
  ctx->n_atoms = n_atoms;
  ctx->n_sh = n_shells;
  ctx->sh_l.assign(shell_l, shell_l + n_shells);
  ctx->sh_ex.assign(shell_exp, shell_exp + n_shells);
  ctx->sh_ctr.resize(3 * (size_t)n_shells);
  ctx->sh_off.resize(n_shells);
  int off = 0;
  for (int s = 0; s < n_shells; ++s) {
    if (shell_l[s] < 0 || shell_l[s] > 2) return fail(ctx, QCX_EINVAL, "shell l must be 0..2");
    if (!(shell_exp[s] > 0.0)) return fail(ctx, QCX_EINVAL, "shell exponent must be > 0");
    if (shell_atom[s] < 0 || shell_atom[s] >= n_atoms)
      return fail(ctx, QCX_EINVAL, "shell atom index out of range");
    for (int x = 0; x < 3; ++x) ctx->sh_ctr[3 * s + x] = xyz[3 * shell_atom[s] + x];
    ctx->sh_off[s] = off;
    off += 2 * shell_l[s] + 1;
  }
  ctx->n_ao = off;
  ctx->lrange = lattice_range;
  ctx->cells.clear();
  ctx->tvec.clear();
  for (int a = -lattice_range; a <= lattice_range; ++a)
    for (int b = -lattice_range; b <= lattice_range; ++b)
      for (int c = -lattice_range; c <= lattice_range; ++c) {
        ctx->cells.push_back(a);
        ctx->cells.push_back(b);
        ctx->cells.push_back(c);
        for (int x = 0; x < 3; ++x)
          ctx->tvec.push_back(a * lat[x] + b * lat[3 + x] + c * lat[6 + x]);
      }
  ctx->n_cells = (int)ctx->cells.size() / 3;
  hipStream_t st = ctx->stream;
  HIPCK(stage_begin(ctx));
  HIPCK(upload(ctx, ctx->d_sh_l, ctx->sh_l.data(), ctx->sh_l.size()));
  HIPCK(upload(ctx, ctx->d_sh_ex, ctx->sh_ex.data(), ctx->sh_ex.size()));
  HIPCK(upload(ctx, ctx->d_sh_ctr, ctx->sh_ctr.data(), ctx->sh_ctr.size()));
  HIPCK(upload(ctx, ctx->d_sh_off, ctx->sh_off.data(), ctx->sh_off.size()));
  HIPCK(upload(ctx, ctx->d_cells, ctx->cells.data(), ctx->cells.size()));
  HIPCK(upload(ctx, ctx->d_tvec, ctx->tvec.data(), ctx->tvec.size()));
  // shell pairs in the order the Fourier-integral kernel takes them: sorted
  // by (l_a, l_b), so that a wave mostly evaluates one angular case
  std::vector<int> order(n_shells * n_shells);
  for (int i = 0; i < n_shells * n_shells; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return shell_l[x / n_shells] * 3 + shell_l[x % n_shells] <
           shell_l[y / n_shells] * 3 + shell_l[y % n_shells];
  });
  HIPCK(upload(ctx, ctx->d_shp, order.data(), order.size()));
  ctx->have_basis = true;
  return QCX_OK;
}

static ShellTab shell_tab(qcx_ctx* ctx) {
  ShellTab t;
  t.l = ctx->d_sh_l.as<int>();
  t.ex = ctx->d_sh_ex.as<double>();
  t.ctr = ctx->d_sh_ctr.as<double>();
  t.off = ctx->d_sh_off.as<int>();
  t.n_sh = ctx->n_sh;
  t.n_ao = ctx->n_ao;
  return t;
}

int qcx_set_states(qcx_ctx* ctx, const double q_cart[3], int n_k, const double* k_frac,
                   int n_occ, int n_bands, const double* C_k, const double* E_k,
                   const double* C_kq, const double* E_kq, int mem) {
  if (!ctx) return QCX_EINVAL;
  if (!ctx->have_basis) return fail(ctx, QCX_ESTATE, "set_cell_basis first");
  if (!q_cart || !k_frac || !C_k || !E_k || !C_kq || !E_kq)
    return fail(ctx, QCX_EINVAL, "NULL argument");
  if (mem != QCX_MEM_HOST && mem != QCX_MEM_DEVICE) return fail(ctx, QCX_EINVAL, "bad mem");
  if (n_k < 1 || n_occ < 1 || n_bands <= n_occ || n_bands > ctx->n_ao)
    return fail(ctx, QCX_EINVAL, "need n_k >= 1 and 1 <= n_occ < n_bands <= N_AO");
  const size_t n_t = 2 * (size_t)n_k * n_occ * (n_bands - n_occ);
  if (n_t > (size_t)1 << 30) return fail(ctx, QCX_EINVAL, "too many transitions");
  if (band_contract_lds(ctx->n_ao, n_bands, n_occ) > 160 * 1024)
    return fail(ctx, QCX_EINVAL, "N_AO x n_bands too large for the band kernel");
  if (int rc = reject_capture(ctx)) return rc;
  HIPCK(hipSetDevice(ctx->device));
  ctx->have_states = ctx->have_rho = ctx->have_chi0 = ctx->have_eps = false;
  hipStream_t st = ctx->stream;
  const bool dev = mem == QCX_MEM_DEVICE;
  // Host inputs are checked here; device inputs on the device, read back by
  // the next synchronising call (no round trip per call)
  const std::vector<double> ek = dev ? std::vector<double>() : std::vector<double>(E_k, E_k + (size_t)n_k * n_bands);
  const std::vector<double> ekq = dev ? std::vector<double>() : std::vector<double>(E_kq, E_kq + (size_t)n_k * n_bands);
  for (int k = 0; k < (dev ? 0 : n_k); ++k) {
    double vmax = -1e300, cmin = 1e300;
    for (int b = 0; b < n_bands; ++b) {
      const double e1 = ek[(size_t)k * n_bands + b], e2 = ekq[(size_t)k * n_bands + b];
      if (!std::isfinite(e1) || !std::isfinite(e2)) return fail(ctx, QCX_EINVAL, "non-finite energy");
      if (b < n_occ)
        vmax = std::max(vmax, std::max(e1, e2));
      else
        cmin = std::min(cmin, std::min(e1, e2));
    }
    if (!(cmin > vmax))
      return fail(ctx, QCX_EINVAL, "an empty band lies below an occupied band at k " +
                                       std::to_string(k));
  }
  memcpy(ctx->q, q_cart, sizeof(double) * 3);
  ctx->n_k = n_k;
  ctx->n_occ = n_occ;
  ctx->n_b = n_bands;
  ctx->n_c = n_bands - n_occ;
  ctx->n_t = (int)n_t;
  const size_t ncoef = (size_t)n_k * ctx->n_ao * n_bands * 2;
  HIPCK(stage_begin(ctx));
  HIPCK(upload(ctx, ctx->d_qc, q_cart, 3));
  HIPCK(upload(ctx, ctx->d_kf, k_frac, (size_t)n_k * 3, dev));
  HIPCK(upload(ctx, ctx->d_Ck, C_k, ncoef, dev));
  HIPCK(upload(ctx, ctx->d_Ckq, C_kq, ncoef, dev));
  HIPCK(upload(ctx, ctx->d_Ek, E_k, (size_t)n_k * n_bands, dev));
  HIPCK(upload(ctx, ctx->d_Ekq, E_kq, (size_t)n_k * n_bands, dev));

  // S(k) = M(k; 0) and S(k+q), then max |C^H S C - I|
  const int nT = ctx->n_cells, nao = ctx->n_ao;
  const double zero3[3] = {0.0, 0.0, 0.0};
  double qf[3];
  for (int i = 0; i < 3; ++i)
    qf[i] = (ctx->lat[3 * i] * q_cart[0] + ctx->lat[3 * i + 1] * q_cart[1] +
             ctx->lat[3 * i + 2] * q_cart[2]) / (2.0 * kPi);
  HIPCK(ctx->d_ph.reserve(sizeof(cplx) * (size_t)n_k * nT));
  HIPCK(ctx->d_phq.reserve(sizeof(cplx) * (size_t)n_k * nT));
  HIPCK(ctx->d_S.reserve(sizeof(cplx) * (size_t)n_k * nao * nao));
  HIPCK(ctx->d_dev.reserve(sizeof(double) * 2 * (size_t)n_k));
  if (!ctx->f0_valid) {  // the Q = 0 integrals depend on the basis only
    HIPCK(upload(ctx, ctx->d_Q, zero3, 3));
    HIPCK(ctx->d_F0.reserve(sizeof(cplx) * nT * (size_t)nao * nao));
    ShellTab sh = shell_tab(ctx);
    launch_cell_ft(sh, ctx->d_shp.as<int>(), ctx->d_tvec.as<double>(), nT, ctx->d_Q.as<double>(),
                   1, ctx->d_F0.as<cplx>(), st);
    LAUNCHCK("cell_ft(S)");
    ctx->f0_valid = true;
  }
  launch_bloch_phase(ctx->d_kf.as<double>(), n_k, zero3, ctx->d_cells.as<int>(), nT,
                     ctx->d_ph.as<cplx>(), st);
  launch_bloch_phase(ctx->d_kf.as<double>(), n_k, qf, ctx->d_cells.as<int>(), nT,
                     ctx->d_phq.as<cplx>(), st);
  LAUNCHCK("bloch_phase");
  launch_phase_sum(ctx->d_F0.as<cplx>(), ctx->d_ph.as<cplx>(), nT, 1, nao * nao, 0, n_k,
                   ctx->d_S.as<cplx>(), st);
  launch_orth_check(ctx->d_S.as<cplx>(), ctx->d_Ck.as<cplx>(), nao, n_bands, n_k,
                    ctx->d_dev.as<double>(), st);
  launch_phase_sum(ctx->d_F0.as<cplx>(), ctx->d_phq.as<cplx>(), nT, 1, nao * nao, 0, n_k,
                   ctx->d_S.as<cplx>(), st);
  launch_orth_check(ctx->d_S.as<cplx>(), ctx->d_Ckq.as<cplx>(), nao, n_bands, n_k,
                    ctx->d_dev.as<double>() + n_k, st);
  LAUNCHCK("orth_check");
  HIPCK(ctx->d_dt.reserve(sizeof(double) * n_t));
  launch_transition_energies(ctx->d_Ek.as<double>(), ctx->d_Ekq.as<double>(), n_k, n_bands, n_occ,
                             ctx->d_dt.as<double>(), st);
  LAUNCHCK("transition_energies");
  ctx->dt_valid = false;
  if (ctx->dt_prefetch) {
    HIPCK(dt_to_host(ctx, (int)n_t));
    ctx->dt_valid = true;
  }
  if (dev) {
    if (!ctx->d_flags.p) {
      HIPCK(ctx->d_flags.reserve(2 * sizeof(int)));
      const int init[2] = {INT_MAX, INT_MAX};
      HIPCK(hipMemcpy(ctx->d_flags.p, init, sizeof(init), hipMemcpyHostToDevice));
    }
    launch_state_flags(ctx->d_Ek.as<double>(), ctx->d_Ekq.as<double>(), n_k, n_bands, n_occ,
                       ctx->d_dev.as<double>(), 1e-10, ctx->d_flags.as<int>(), st);
    LAUNCHCK("state checks");
    ctx->check_pending = true;
    ctx->check_nk = n_k;
    ctx->have_states = true;
    return QCX_OK;
  }
  std::vector<double> devs(2 * (size_t)n_k);
  HIPCK(hipMemcpyAsync(devs.data(), ctx->d_dev.p, devs.size() * sizeof(double),
                       hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  for (int i = 0; i < 2 * n_k; ++i) {
    if (!(devs[i] <= 1e-10)) {
      char buf[160];
      snprintf(buf, sizeof buf, "states at %s %d are not orthonormal: max|C^H S C - I| = %.3e",
               i < n_k ? "k" : "k+q", i % n_k, devs[i]);
      return fail(ctx, QCX_ENONORTH, buf);
    }
  }
  ctx->have_states = true;
  return QCX_OK;
}

}  // extern "C"

// Bytes of one k point's Bloch sums M(k; G) for n_G rows (fallback path)
static size_t m_bytes_per_k(const qcx_ctx* ctx, int n_G) {
  return sizeof(cplx) * (size_t)n_G * ctx->n_ao * ctx->n_ao;
}

int qcx::rho_prepare(qcx_ctx* ctx, int n_G, const int* G_int, bool need_g0, bool optical) {
  if (n_G < 1 || n_G > 4096 || !G_int) return fail(ctx, QCX_EINVAL, "need 1 <= n_G <= 4096");
  if (need_g0 && (G_int[0] != 0 || G_int[1] != 0 || G_int[2] != 0))
    return fail(ctx, QCX_EINVAL, "G_int[0] must be (0,0,0)");
  for (int g = 0; g < n_G; ++g) {
    if (optical && g == 0) continue;
    double n2 = 0.0;
    for (int x = 0; x < 3; ++x) {
      double v = ctx->q[x];
      for (int j = 0; j < 3; ++j) v += G_int[3 * g + j] * ctx->rec[3 * j + x];
      n2 += v * v;
    }
    if (!(n2 > 0.0)) return fail(ctx, QCX_EINVAL, "q + G vanishes for G index " + std::to_string(g));
  }
  HIPCK(hipSetDevice(ctx->device));
  ctx->have_rho = ctx->have_chi0 = ctx->have_eps = false;
  const int nT = ctx->n_cells;
  HIPCK(ctx->d_Q.reserve(sizeof(double) * 3 * (size_t)n_G));
  HIPCK(ctx->d_vq.reserve(sizeof(double) * (size_t)n_G));
  HIPCK(ctx->d_F.reserve(m_bytes_per_k(ctx, n_G) * nT));
  ctx->ldt = roundup(ctx->n_t + 16, kLdtAlign);  // zero tail for padded and chunked readers
  HIPCK(ctx->d_R.reserve(sizeof(cplx) * ctx->ldt * n_G));
  if (!rho_fused_fits(ctx->n_ao, ctx->n_occ, nT)) {
    // Bloch sums M(k; G) of one pass of the fallback (k points in chunks)
    const size_t per_k = m_bytes_per_k(ctx, n_G);
    const int kc = (int)std::max<size_t>(1, std::min<size_t>(ctx->n_k, kMBudget / per_k));
    HIPCK(ctx->d_M.reserve(per_k * kc));
  }
  ctx->n_g = n_G;
  return QCX_OK;
}

// Bloch sum and band contraction of the `rows` rows of a G-major F: in one
// pass with M in LDS, or (large bases, many valence bands) through M chunks
// in ctx->d_M, whose capacity sets the k chunk
static int densities(qcx_ctx* ctx, const cplx* F, int rows, const cplx* bra, cplx* Rout,
                     hipStream_t st) {
  const int nT = ctx->n_cells, nao = ctx->n_ao;
  if (rho_fused_fits(nao, ctx->n_occ, nT)) {
    launch_rho_fused(F, ctx->d_ph.as<cplx>(), ctx->d_Ck.as<cplx>(), bra, nao, ctx->n_b, ctx->n_occ,
                     ctx->n_k, nT, rows, Rout, ctx->ldt, st);
    LAUNCHCK("rho_fused");
    return QCX_OK;
  }
  const size_t nee = (size_t)nao * nao;
  const size_t per = sizeof(cplx) * (size_t)rows * nee;
  const int kch = (int)std::max<size_t>(1, std::min<size_t>(ctx->n_k, ctx->d_M.bytes / per));
  for (int k0 = 0; k0 < ctx->n_k; k0 += kch) {
    const int nk = std::min(kch, ctx->n_k - k0);
    launch_phase_sum(F, ctx->d_ph.as<cplx>(), nT, rows, (int)nee, k0, nk, ctx->d_M.as<cplx>(), st);
    launch_band_contract(ctx->d_M.as<cplx>(), ctx->d_Ck.as<cplx>(), bra, nao, ctx->n_b, ctx->n_occ,
                         ctx->n_k, k0, nk, rows, Rout, ctx->ldt, st);
    LAUNCHCK("phase_sum/band_contract");
  }
  return QCX_OK;
}

int qcx::rho_enqueue(qcx_ctx* ctx, const int* d_G, int n_G, bool optical, hipStream_t st) {
  launch_q_plus_g(ctx->d_qc.as<double>(), d_G, ctx->rec, n_G, optical, ctx->d_Q.as<double>(),
                  ctx->d_vq.as<double>(), st);
  launch_zero_tail(ctx->d_R.as<cplx>(), ctx->ldt, ctx->n_t, n_G, st);
  LAUNCHCK("q_plus_g/zero_tail");
  launch_cell_ft(shell_tab(ctx), ctx->d_shp.as<int>(), ctx->d_tvec.as<double>(), ctx->n_cells,
                 ctx->d_Q.as<double>(), n_G, ctx->d_F.as<cplx>(), st);
  LAUNCHCK("cell_ft");
  // the bra states: k + q, or in the optical limit k itself
  const cplx* bra = optical ? ctx->d_Ck.as<cplx>() : ctx->d_Ckq.as<cplx>();
  return densities(ctx, ctx->d_F.as<cplx>(), n_G, bra, ctx->d_R.as<cplx>(), st);
}

extern "C" {

// Pair densities R[G][t] into ctx->d_R for the G list (G = 0 first when
// need_g0; qcx_loss_diag's chunks have no G = 0 requirement).  With
// qhat (the optical limit, App. C) the states must have q = 0; the k states
// serve on both sides, and the G = 0 row is replaced by its q -> 0 limit
// divided by |q| (k.p form, launch_optical_row) with Coulomb factor sqrt(4 pi).
static int pair_density_impl(qcx_ctx* ctx, int n_G, const int* G_int, void* rho_out, bool need_g0,
                             const double* qhat = nullptr) {
  if (!ctx) return QCX_EINVAL;
  if (!ctx->have_states) return fail(ctx, QCX_ESTATE, "set_states first");
  const bool optical = qhat != nullptr;
  double qh[3] = {0.0, 0.0, 0.0};
  if (optical) {
    if (ctx->q[0] != 0.0 || ctx->q[1] != 0.0 || ctx->q[2] != 0.0)
      return fail(ctx, QCX_EINVAL, "the optical limit needs states set with q = 0");
    const double nq = std::sqrt(qhat[0] * qhat[0] + qhat[1] * qhat[1] + qhat[2] * qhat[2]);
    if (!(nq > 0.0) || !std::isfinite(nq)) return fail(ctx, QCX_EINVAL, "qhat must be a nonzero direction");
    for (int x = 0; x < 3; ++x) qh[x] = qhat[x] / nq;
  }
  if (int rc = reject_capture(ctx)) return rc;
  if (int rc = rho_prepare(ctx, n_G, G_int, need_g0, optical)) return rc;
  hipStream_t st = ctx->stream;
  HIPCK(stage_begin(ctx));
  HIPCK(upload(ctx, ctx->d_G, G_int, 3 * (size_t)n_G));
  int sp_rho;
  HIPCK(span_begin(ctx, 0, &sp_rho));
  if (int rc = rho_enqueue(ctx, ctx->d_G.as<int>(), n_G, optical, st)) return rc;
  if (optical) {
    // transitions at the same k; then P = C^H D(k) C for the three gradient
    // components (their Bloch sums take the place of M) and the k.p row
    const int nT = ctx->n_cells;
    const size_t nee = (size_t)ctx->n_ao * ctx->n_ao;
    launch_transition_energies(ctx->d_Ek.as<double>(), ctx->d_Ek.as<double>(), ctx->n_k, ctx->n_b,
                               ctx->n_occ, ctx->d_dt.as<double>(), st);
    ctx->dt_valid = false;
    HIPCK(ctx->d_Fg.reserve(sizeof(cplx) * nT * 3 * nee));
    HIPCK(ctx->d_Rp.reserve(sizeof(cplx) * 3 * ctx->ldt));
    launch_grad_ft(shell_tab(ctx), ctx->d_tvec.as<double>(), nT, ctx->d_Fg.as<cplx>(), st);
    if (int rc = densities(ctx, ctx->d_Fg.as<cplx>(), 3, ctx->d_Ck.as<cplx>(), ctx->d_Rp.as<cplx>(), st))
      return rc;
    launch_optical_row(ctx->d_Rp.as<cplx>(), ctx->ldt, ctx->d_dt.as<double>(), ctx->n_t, qh,
                       ctx->d_R.as<cplx>(), st);
    LAUNCHCK("optical limit");
  }
  HIPCK(span_end(ctx, sp_rho));
  if (rho_out) {
    launch_rho_export(ctx->d_R.as<cplx>(), ctx->ldt, n_G, ctx->n_t, static_cast<cplx*>(rho_out), st);
    LAUNCHCK("rho_export");
  }
  ctx->have_rho = true;
  return QCX_OK;
}

int qcx_pair_density(qcx_ctx* ctx, int n_G, const int* G_int, void* rho_out) {
  return pair_density_impl(ctx, n_G, G_int, rho_out, true);
}

int qcx_pair_density_optical(qcx_ctx* ctx, int n_G, const int* G_int, const double* qhat,
                             void* rho_out) {
  if (!ctx) return QCX_EINVAL;
  if (!qhat) return fail(ctx, QCX_EINVAL, "qhat is NULL");
  return pair_density_impl(ctx, n_G, G_int, rho_out, true, qhat);
}

int qcx_loss_diag(qcx_ctx* ctx, int n_G, const int* G_int, int n_w, const double* w_eV,
                  double eta_eV, int precision, double* loss_out, void* inv_out) {
  if (!ctx) return QCX_EINVAL;
  if (!ctx->have_states) return fail(ctx, QCX_ESTATE, "set_states first");
  if (n_G < 1 || !G_int) return fail(ctx, QCX_EINVAL, "need n_G >= 1");
  if (n_w < 1 || n_w > 65536 || !w_eV) return fail(ctx, QCX_EINVAL, "need 1 <= n_w <= 65536");
  if (!(eta_eV >= 0.0) || !std::isfinite(eta_eV)) return fail(ctx, QCX_EINVAL, "eta must be >= 0");
  if (precision < QCX_FP64 || precision > QCX_SPLIT_BF16) return fail(ctx, QCX_EINVAL, "bad precision");
  if (!loss_out) return fail(ctx, QCX_EINVAL, "loss_out must be a device buffer");
  if (int rc = reject_capture(ctx)) return rc;
  HIPCK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  std::vector<double> w(n_w);
  for (int i = 0; i < n_w; ++i) {
    if (!std::isfinite(w_eV[i])) return fail(ctx, QCX_EINVAL, "non-finite frequency");
    w[i] = w_eV[i] / kHartreeEV;
  }
  HIPCK(stage_begin(ctx));
  HIPCK(upload(ctx, ctx->d_w, w.data(), w.size()));
  const double eta = eta_eV / kHartreeEV;
  const bool bulk = precision != QCX_FP64, bf = precision == QCX_SPLIT_BF16;
  constexpr int kChunk = 4096;
  // weights of the bulk once (they do not depend on G)
  Chi0Geom g{};
  g.n_t = ctx->n_t;
  g.n_w = n_w;
  g.n_rows = 2 * n_w;
  const int af = bulk_row_frags(g);
  g.n_rowsp = (int)roundup(g.n_rows, 32 * af);
  g.c_rows = g.n_rowsp;
  g.n_tp = (int)roundup(g.n_t, KSTEP_T * kMaxKsplit);
  if (bulk) {
    const size_t nA = (size_t)g.n_rowsp * g.n_tp;
    if (bf) {
      HIPCK(ctx->d_A.reserve(sizeof(uint16_t) * nA));
      HIPCK(ctx->d_Alo.reserve(sizeof(uint16_t) * nA));
      launch_weights_bf16(ctx->d_w.as<double>(), ctx->d_dt.as<double>(), eta, g,
                          ctx->d_A.as<uint16_t>(), ctx->d_Alo.as<uint16_t>(), st);
    } else {
      HIPCK(ctx->d_A.reserve(sizeof(float) * nA));
      launch_weights_f32(ctx->d_w.as<double>(), ctx->d_dt.as<double>(), eta, g, ctx->d_A.as<float>(),
                         st);
    }
    LAUNCHCK("weights");
  }
  int sp_all;
  HIPCK(span_begin(ctx, 3, &sp_all));
  for (int g0 = 0; g0 < n_G; g0 += kChunk) {
    const int nch = std::min(kChunk, n_G - g0);
    if (int rc = pair_density_impl(ctx, nch, G_int + 3 * (size_t)g0, nullptr, false)) return rc;
    HIPCK(stage_begin(ctx));
    std::vector<int> pairs;
    AsmArgs a{};
    a.vq = ctx->d_vq.as<double>();
    a.pref = 2.0 / (ctx->n_k * ctx->vol);
    g.n_g = nch;
    g.n_pairs = nch;
    g.p0 = 0;
    g.n_bulk = nch;
    g.n_bulkp = (int)roundup(nch, 128);
    if (bulk) {
      pairs.assign(g.n_bulkp, 0);
      for (int b = 0; b < nch; ++b) pairs[b] = b | (b << 16);
      g.gather = nch >= kGatherMinNg ? 1 : 0;
      if (g.gather) {
        std::vector<int> local, rows;
        if (!bulk_gather_tables(pairs, local, rows))
          return fail(ctx, QCX_EDEVICE, "internal: a pair tile needs more rows than staged");
        HIPCK(upload_cached(ctx, ctx->d_pairs, ctx->h_pairs_up, local));
        HIPCK(upload_cached(ctx, ctx->d_rows, ctx->h_rows_up, rows));
      } else {
        HIPCK(upload_cached(ctx, ctx->d_pairs, ctx->h_pairs_up, pairs));
      }
      const int blocks = (g.n_bulkp / 128) * (g.n_rowsp / (32 * af));
      g.ksplit = std::max(ksplit_for_accuracy(g.n_tp / KSTEP_T), pick_ksplit(blocks, g.n_tp / KSTEP_T));
      HIPCK(ctx->d_R32.reserve(sizeof(float) * 2 * (size_t)g.n_g * g.n_tp));
      HIPCK(ctx->d_C.reserve(sizeof(float) * (size_t)g.ksplit * g.n_rowsp * 2 * g.n_bulkp));
      launch_pack_r32(ctx->d_R.as<cplx>(), ctx->ldt, g, bf ? 0 : 1, ctx->d_R32.as<float>(), st);
      const int* rows_dev = g.gather ? ctx->d_rows.as<int>() : nullptr;
      int sp;
      HIPCK(span_begin(ctx, 1, &sp));
      if (bf)
        launch_bulk_bf16(ctx->d_A.as<uint16_t>(), ctx->d_Alo.as<uint16_t>(), ctx->d_R32.as<float>(),
                         ctx->d_pairs.as<int>(), rows_dev, g, 2, ctx->d_C.as<float>(), st);
      else
        launch_bulk_f32(ctx->d_A.as<float>(), ctx->d_R32.as<float>(), ctx->d_pairs.as<int>(), rows_dev,
                        g, 2, ctx->d_C.as<float>(), st);
      HIPCK(span_end(ctx, sp));
      LAUNCHCK("bulk (diagonal)");
      a.C = ctx->d_C.as<float>();
      a.ks = g.ksplit;
    } else {
      pairs.resize(nch);
      for (int b = 0; b < nch; ++b) pairs[b] = b | (b << 16);
      HIPCK(upload_cached(ctx, ctx->d_pairs64, ctx->h_pairs64_up, pairs));
      Geom64& g64 = ctx->geom64;
      geom64_init(g64, nch, n_w, ctx->n_t, nch, (size_t)512 << 20);
      HIPCK(ctx->d_XY.reserve(sizeof(double) * (size_t)g64.ksplit * g64.n_rowsp * g64.n_colp));
      int sp;
      HIPCK(span_begin(ctx, 2, &sp));
      launch_pairs_f64(ctx->d_R.as<cplx>(), ctx->ldt, ctx->d_w.as<double>(), ctx->d_dt.as<double>(),
                       eta, g64, ctx->d_pairs64.as<int>(), ctx->d_XY.as<double>(), st);
      HIPCK(span_end(ctx, sp));
      LAUNCHCK("pairs_f64 (diagonal)");
      a.XY = ctx->d_XY.as<double>();
      a.ks64 = g64.ksplit;
      a.n_rowsp64 = g64.n_rowsp;
      a.n_colp64 = g64.n_colp;
    }
    launch_diag_loss(a, g, nch, n_w, loss_out, static_cast<cplx*>(inv_out), n_G, g0, st);
    LAUNCHCK("diag_loss");
  }
  HIPCK(span_end(ctx, sp_all));
  // the pair densities left behind belong to the last chunk only
  ctx->have_rho = ctx->have_chi0 = ctx->have_eps = false;
  return QCX_OK;
}

int qcx_chi0(qcx_ctx* ctx, int n_w, const double* w_eV, double eta_eV, int precision,
             int headwings_fp64, void* chi0_out) {
  if (!ctx) return QCX_EINVAL;
  if (!ctx->have_rho) return fail(ctx, QCX_ESTATE, "pair_density first");
  if (n_w < 1 || n_w > 65536 || !w_eV) return fail(ctx, QCX_EINVAL, "need 1 <= n_w <= 65536");
  if (!(eta_eV >= 0.0) || !std::isfinite(eta_eV)) return fail(ctx, QCX_EINVAL, "eta must be >= 0");
  if (precision < QCX_FP64 || precision > QCX_SPLIT_BF16)
    return fail(ctx, QCX_EINVAL, "bad precision");

  if (int rc = reject_capture(ctx)) return rc;
  HIPCK(hipSetDevice(ctx->device));
  ctx->have_chi0 = ctx->have_eps = false;
  hipStream_t st = ctx->stream;
  std::vector<double> w(n_w);
  for (int i = 0; i < n_w; ++i) {
    if (!std::isfinite(w_eV[i])) return fail(ctx, QCX_EINVAL, "non-finite frequency");
    w[i] = w_eV[i] / kHartreeEV;
  }
  HIPCK(stage_begin(ctx));
  HIPCK(upload(ctx, ctx->d_w, w.data(), w.size()));
  ctx->n_w = n_w;
  ctx->eta = eta_eV / kHartreeEV;
  ctx->prec = precision;
  ctx->hw64 = headwings_fp64 ? 1 : 0;

  Chi0Geom& g = ctx->geom;
  g = Chi0Geom{};
  g.n_g = ctx->n_g;
  g.n_t = ctx->n_t;
  g.n_w = n_w;
  g.n_rows = 2 * n_w;
  g.n_pairs = ctx->n_g * (ctx->n_g + 1) / 2;
  if (precision == QCX_FP64) {
    ctx->n_pairs64 = g.n_pairs;
    g.p0 = g.n_pairs;
  } else {
    ctx->n_pairs64 = ctx->hw64 ? ctx->n_g : 0;
    g.p0 = ctx->n_pairs64;
  }
  g.n_bulk = g.n_pairs - g.p0;
  g.n_bulkp = (int)roundup(std::max(g.n_bulk, 1), 128);
  int sp_all, sp_bulk = -1, sp_hw = -1;
  HIPCK(span_begin(ctx, 3, &sp_all));
  if (g.n_bulk > 0) {
    g.n_rowsp = (int)roundup(g.n_rows, 128);
    const int af = bulk_row_frags(g);
    g.n_rowsp = (int)roundup(g.n_rows, 32 * af);
    const int blocks = (g.n_bulkp / 128) * (g.n_rowsp / (32 * af));
    g.n_tp = (int)roundup(g.n_t, KSTEP_T * kMaxKsplit);
    const int ks_acc = ksplit_for_accuracy(g.n_tp / KSTEP_T);
    // row chunks when even the smallest admissible split count overflows
    // the partial-sum budget
    const size_t row_bytes = 2 * (size_t)g.n_bulkp * sizeof(float);
    int chunk_rows = g.n_rowsp;
    if ((size_t)ks_acc * g.n_rowsp * row_bytes > kPartialBudget)
      chunk_rows = std::max(32 * af, (int)(kPartialBudget / (ks_acc * row_bytes)) / (32 * af) *
                                         (32 * af));
    const bool chunked = chunk_rows < g.n_rowsp;
    g.row_tile0 = 0;
    g.c_rows = chunk_rows;
    const std::vector<Cand> cands = bulk_candidates(g, af, ks_acc);
    if (cands.empty()) return fail(ctx, QCX_EINVAL, "no bulk tile configuration fits");
    // heuristic choice, used when tuning is off, under graph capture, or as
    // the candidate to beat
    Cand pick{std::max(ks_acc, pick_ksplit(blocks, g.n_tp / KSTEP_T)), 2};
    if (std::none_of(cands.begin(), cands.end(),
                     [&](const Cand& c) { return c.ks == pick.ks && c.nst == pick.nst; }))
      pick = cands.front();
    const TuneKey key{ctx->device, precision, g.n_g, g.n_tp, g.n_rowsp, g.n_bulkp};
    bool tune = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end())
        pick = {it->second.ks, it->second.nst};
      else
        tune = ctx->autotune != 0;
    }
    if (ctx->force_nst) {  // a pipeline forced by qcx_set_bulk_pipeline
      tune = false;
      const int ks = std::max(ks_acc, pick_ksplit(blocks, g.n_tp / KSTEP_T));
      auto it = std::find_if(cands.begin(), cands.end(), [&](const Cand& c) {
        return c.nst == ctx->force_nst && c.ks == ks;
      });
      if (it == cands.end())
        it = std::find_if(cands.begin(), cands.end(),
                          [&](const Cand& c) { return c.nst == ctx->force_nst; });
      if (it == cands.end()) return fail(ctx, QCX_EINVAL, "the forced bulk pipeline does not fit");
      pick = *it;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCK(hipStreamIsCapturing(st, &cap));
    if (cap != hipStreamCaptureStatusNone) tune = false;
    // very large shapes: a launch takes longer than tuning could repay
    // (estimated at 300 TFLOP/s FP32-equivalent), keep the heuristic
    const double est_ms = 2.0 * g.n_rowsp * 2.0 * g.n_bulkp * g.n_tp / 3e14 * 1e3;
    if (est_ms > 500.0 || chunked) tune = false;
    int max_ks = pick.ks;
    if (tune)
      for (const Cand& c : cands) max_ks = std::max(max_ks, c.ks);
    const size_t nA = (size_t)g.n_rowsp * g.n_tp;  // elements
    const size_t nC = (size_t)max_ks * g.c_rows * 2 * g.n_bulkp;
    HIPCK(ctx->d_R32.reserve(sizeof(float) * 2 * (size_t)g.n_g * g.n_tp));
    HIPCK(ctx->d_C.reserve(sizeof(float) * nC));
    if (chunked) HIPCK(ctx->d_C64.reserve(sizeof(double) * 2 * (size_t)g.n_rowsp * g.n_bulkp));
    ctx->bulk_c64 = chunked;
    std::vector<int> pairs(g.n_bulkp, 0);
    {
      int b = 0, p = 0;
      for (int G = 0; G < g.n_g; ++G)
        for (int Gp = G; Gp < g.n_g; ++Gp, ++p)
          if (p >= g.p0) pairs[b++] = G | (Gp << 16);
    }
    g.gather = g.n_g >= kGatherMinNg ? 1 : 0;
    if (g.gather) {
      std::vector<int> local, rows;
      if (!bulk_gather_tables(pairs, local, rows))
        return fail(ctx, QCX_EDEVICE, "internal: a pair tile needs more rows than staged");
      HIPCK(upload_cached(ctx, ctx->d_pairs, ctx->h_pairs_up, local));
      HIPCK(upload_cached(ctx, ctx->d_rows, ctx->h_rows_up, rows));
    } else {
      HIPCK(upload_cached(ctx, ctx->d_pairs, ctx->h_pairs_up, pairs));
    }
    const int* rows_dev = g.gather ? ctx->d_rows.as<int>() : nullptr;
    const bool bf = precision == QCX_SPLIT_BF16;
    launch_pack_r32(ctx->d_R.as<cplx>(), ctx->ldt, g, bf ? 0 : 1, ctx->d_R32.as<float>(), st);
    if (bf) {
      HIPCK(ctx->d_A.reserve(sizeof(uint16_t) * nA));
      HIPCK(ctx->d_Alo.reserve(sizeof(uint16_t) * nA));
      launch_weights_bf16(ctx->d_w.as<double>(), ctx->d_dt.as<double>(), ctx->eta, g,
                          ctx->d_A.as<uint16_t>(), ctx->d_Alo.as<uint16_t>(), st);
    } else {
      HIPCK(ctx->d_A.reserve(sizeof(float) * nA));
      launch_weights_f32(ctx->d_w.as<double>(), ctx->d_dt.as<double>(), ctx->eta, g,
                         ctx->d_A.as<float>(), st);
    }
    LAUNCHCK("weights/pack");
    auto run_bulk = [&](const Cand& c) {
      g.ksplit = c.ks;
      if (bf)
        launch_bulk_bf16(ctx->d_A.as<uint16_t>(), ctx->d_Alo.as<uint16_t>(),
                         ctx->d_R32.as<float>(), ctx->d_pairs.as<int>(), rows_dev, g, c.nst,
                         ctx->d_C.as<float>(), st);
      else
        launch_bulk_f32(ctx->d_A.as<float>(), ctx->d_R32.as<float>(), ctx->d_pairs.as<int>(),
                        rows_dev, g, c.nst, ctx->d_C.as<float>(), st);
    };
    ctx->tune_ms = 0.0;
    if (tune) {
      const auto t0 = std::chrono::steady_clock::now();
      hipEvent_t e0, e1;
      HIPCK(hipEventCreate(&e0));
      HIPCK(hipEventCreate(&e1));
      float best = 1e30f;
      run_bulk(cands.front());  // warm (code objects, caches)
      for (const Cand& c : cands) {
        HIPCK(hipEventRecord(e0, st));
        run_bulk(c);
        HIPCK(hipEventRecord(e1, st));
        LAUNCHCK("bulk (tuning)");
        HIPCK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCK(hipEventElapsedTime(&ms, e0, e1));
        // each split's partials are read once more by the assembly: add that
        // traffic at 5 TB/s so that more splits must earn their keep
        ms += (float)((double)c.ks * g.c_rows * 2 * g.n_bulkp * sizeof(float) / 5e9);
        if (ms < best) {
          best = ms;
          pick = c;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = {pick.ks, pick.nst};
      }
      ctx->tune_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    ctx->bulk_nst = pick.nst;
    ctx->bulk_af = af;
    HIPCK(span_begin(ctx, 1, &sp_bulk));
    if (!chunked) {
      run_bulk(pick);
    } else {
      for (int r0 = 0; r0 < g.n_rowsp; r0 += chunk_rows) {
        g.row_tile0 = r0 / (32 * af);
        g.c_rows = std::min(chunk_rows, g.n_rowsp - r0);
        run_bulk(pick);
        launch_reduce_partials(ctx->d_C.as<float>(), pick.ks, g.c_rows, g.n_bulkp,
                               ctx->d_C64.as<double>() + (size_t)r0 * 2 * g.n_bulkp, st);
      }
      g.row_tile0 = 0;
      g.c_rows = g.n_rowsp;
    }
    LAUNCHCK("bulk");
    HIPCK(span_end(ctx, sp_bulk));
  } else {
    g.ksplit = 1;
    g.n_rowsp = 0;
    g.n_tp = (int)roundup(g.n_t, 16);
  }
  if (ctx->n_pairs64 > 0) {
    Geom64& g64 = ctx->geom64;
    // head and wings alone (the pairs (0, G')): FP64 GEMM over a table of the
    // pair products; every pair (the FP64 path): products formed on the fly
    const bool hw = ctx->n_pairs64 == ctx->n_g;
    if (hw)
      geom_hw_init(g64, ctx->n_g, n_w, ctx->n_t, ctx->n_pairs64, (size_t)512 << 20);
    else
      geom64_init(g64, ctx->n_g, n_w, ctx->n_t, ctx->n_pairs64, (size_t)512 << 20);
    ctx->ks64 = g64.ksplit;
    std::vector<int> tab(ctx->n_pairs64);
    {
      int p = 0;
      for (int G = 0; G < ctx->n_g && p < ctx->n_pairs64; ++G)
        for (int Gp = G; Gp < ctx->n_g && p < ctx->n_pairs64; ++Gp, ++p) tab[p] = G | (Gp << 16);
    }
    HIPCK(upload_cached(ctx, ctx->d_pairs64, ctx->h_pairs64_up, tab));
    HIPCK(ctx->d_XY.reserve(sizeof(double) * (size_t)g64.ksplit * g64.n_rowsp * g64.n_colp));
    if (hw) HIPCK(ctx->d_hwP.reserve(sizeof(double) * hw_ptable_doubles(g64)));
    HIPCK(span_begin(ctx, 2, &sp_hw));
    if (hw)
      launch_headwings_f64(ctx->d_R.as<cplx>(), ctx->ldt, ctx->d_w.as<double>(),
                           ctx->d_dt.as<double>(), ctx->eta, g64, ctx->d_pairs64.as<int>(),
                           ctx->d_hwP.as<double>(), ctx->d_XY.as<double>(), st);
    else
      launch_pairs_f64(ctx->d_R.as<cplx>(), ctx->ldt, ctx->d_w.as<double>(), ctx->d_dt.as<double>(),
                       ctx->eta, g64, ctx->d_pairs64.as<int>(), ctx->d_XY.as<double>(), st);
    LAUNCHCK("pairs_f64");
    HIPCK(span_end(ctx, sp_hw));
  }
  HIPCK(span_end(ctx, sp_all));
  ctx->have_chi0 = true;
  if (chi0_out) {
    AsmArgs a{};
    a.C = (g.n_bulk > 0 && !ctx->bulk_c64) ? ctx->d_C.as<float>() : nullptr;
  a.C64 = (g.n_bulk > 0 && ctx->bulk_c64) ? ctx->d_C64.as<double>() : nullptr;
    a.XY = ctx->n_pairs64 > 0 ? ctx->d_XY.as<double>() : nullptr;
    a.ks = g.ksplit;
    a.ks64 = ctx->ks64;
    a.n_rowsp64 = ctx->geom64.n_rowsp;
    a.n_colp64 = ctx->geom64.n_colp;
    a.n_pairs64 = ctx->n_pairs64;
    a.vq = ctx->d_vq.as<double>();
    a.pref = 2.0 / (ctx->n_k * ctx->vol);
    launch_chi0_export(a, g, static_cast<cplx*>(chi0_out), st);
    LAUNCHCK("chi0_export");
  }
  return QCX_OK;
}

int qcx_chi0_kk(qcx_ctx* ctx, int n_w, const double* w_eV, double eta_eV, double bin_eV,
                void* chi0_out) {
  if (!ctx) return QCX_EINVAL;
  if (!ctx->have_rho) return fail(ctx, QCX_ESTATE, "pair_density first");
  if (n_w < 1 || n_w > 65536 || !w_eV) return fail(ctx, QCX_EINVAL, "need 1 <= n_w <= 65536");
  if (!(eta_eV >= 0.0) || !std::isfinite(eta_eV)) return fail(ctx, QCX_EINVAL, "eta must be >= 0");
  if (!(bin_eV > 0.0) || !std::isfinite(bin_eV)) return fail(ctx, QCX_EINVAL, "bin width must be > 0");
  if (int rc = reject_capture(ctx)) return rc;
  HIPCK(hipSetDevice(ctx->device));
  ctx->have_chi0 = ctx->have_eps = false;
  hipStream_t st = ctx->stream;
  std::vector<double> w(n_w);
  for (int i = 0; i < n_w; ++i) {
    if (!std::isfinite(w_eV[i])) return fail(ctx, QCX_EINVAL, "non-finite frequency");
    w[i] = w_eV[i] / kHartreeEV;
  }
  const double d = bin_eV / kHartreeEV, eta = eta_eV / kHartreeEV;
  const int n_t = ctx->n_t, n_half = n_t / 2, n_g = ctx->n_g;
  // transition energies on the host: queued by qcx_set_states once this route
  // has run (so the wait below ends before the pair densities do), else now
  if (!ctx->dt_valid) {
    HIPCK(dt_to_host(ctx, n_t));
    ctx->dt_prefetch = ctx->dt_valid = true;
  }
  HIPCK(hipEventSynchronize(ctx->ev_dt));
  ctx->dt_pending = false;
  const double* dt = ctx->h_dt;

  // Per side: interval floor(D / d) of every transition relative to the
  // side's lowest, a stable counting sort by interval, and the chunks.
  std::vector<int> rank(n_t), ib(n_t);  // rank[t]: position of t in energy order
  std::vector<double> xf(n_t);
  std::vector<KkChunk> chunks;
  int base[2] = {0, 0}, nbin[2] = {0, 0}, rows = 0;
  for (int s = 0; s < 2; ++s) {
    const int t_lo = s ? n_half : 0, t_hi = s ? n_t : n_half, cnt_t = t_hi - t_lo;
    double umin = INFINITY, umax = -INFINITY;
    for (int t = t_lo; t < t_hi; ++t) {
      const double u = dt[t] / d;
      if (!std::isfinite(u)) return fail(ctx, QCX_EINVAL, "non-finite transition energy");
      umin = std::min(umin, u);
      umax = std::max(umax, u);
    }
    if (!(std::fabs(umin) < 1e9 && std::fabs(umax) < 1e9) ||
        std::floor(umax) - std::floor(umin) + 2 > (double)kKkMaxBins)
      return fail(ctx, QCX_EINVAL, "too many bins: widen bin_eV");
    base[s] = (int)std::floor(umin);
    const int n_int = (int)std::floor(umax) - base[s] + 1;
    nbin[s] = n_int + 1;
    std::vector<int> iv(cnt_t), off(n_int + 1, 0);
    for (int t = 0; t < cnt_t; ++t) {
      iv[t] = (int)std::floor(dt[t_lo + t] / d) - base[s];
      ++off[iv[t] + 1];
    }
    for (int i = 0; i < n_int; ++i) off[i + 1] += off[i];
    std::vector<int> pos(off.begin(), off.end() - 1);
    for (int t = 0; t < cnt_t; ++t) {
      const int k = t_lo + pos[iv[t]]++;
      const double u = dt[t_lo + t] / d;
      rank[t_lo + t] = k;
      ib[k] = iv[t];
      xf[k] = u - std::floor(u);
    }
    // chunks of whole intervals [k0, k1), at most kKkChunkT transitions
    // unless one interval holds more; bin n_int (the side's last) is stored
    // by the tail pass of the last chunk
    for (int k0 = 0; k0 < n_int;) {
      int k1 = k0 + 1;
      while (k1 < n_int && off[k1 + 1] - off[k0] <= kKkChunkT) ++k1;
      chunks.push_back({rows + k0, k0, k1 - k0, t_lo + off[k0], t_lo + off[k1], rows + k1,
                        k1 < n_int ? 1 : 0});
      k0 = k1;
    }
    rows += nbin[s];
  }
  const int n_gp = (int)roundup(n_g, kKkTile);
  const size_t n_pairs = (size_t)n_g * (n_g + 1) / 2;
  const int rows_p = kk_rows_padded(rows), ldm = kk_ldm(n_w);
  // S (rows_p bins) and E (one row per chunk) share one buffer
  if ((double)(rows + chunks.size()) * 2 * n_pairs * sizeof(double) > kKkSpectralBudget)
    return fail(ctx, QCX_EINVAL, "binned spectral function exceeds 16 GB: widen bin_eV");
  if (chunks.size() > (size_t)INT_MAX) return fail(ctx, QCX_EINVAL, "too many bins");

  HIPCK(stage_begin(ctx));
  HIPCK(upload(ctx, ctx->d_w, w.data(), w.size()));
  HIPCK(upload(ctx, ctx->d_kk_rank, rank.data(), rank.size()));
  HIPCK(upload(ctx, ctx->d_kk_ib, ib.data(), ib.size()));
  HIPCK(upload(ctx, ctx->d_kk_xf, xf.data(), xf.size()));
  HIPCK(upload(ctx, ctx->d_kk_chunks, chunks.data(), chunks.size()));
  HIPCK(ctx->d_kk_Rs.reserve(sizeof(cplx) * (size_t)n_t * n_gp));
  const size_t e_off = (size_t)rows_p * 2 * n_pairs + kk_s_slack();
  HIPCK(ctx->d_kk_S.reserve(sizeof(double) * (e_off + chunks.size() * 2 * n_pairs)));
  HIPCK(ctx->d_kk_K.reserve(sizeof(double) * (size_t)rows_p * ldm));
  // bins past the last (padding of the transform's K tiles) are zero; the
  // binning writes every real bin
  HIPCK(hipMemsetAsync(ctx->d_kk_S.as<double>() + (size_t)rows * 2 * n_pairs, 0,
                       sizeof(double) * ((size_t)(rows_p - rows) * 2 * n_pairs + kk_s_slack()), st));
  HIPCK(ctx->d_C64.reserve(sizeof(double) * (size_t)2 * n_w * 2 * n_pairs));
  ctx->n_w = n_w;
  ctx->eta = eta;
  ctx->prec = QCX_FP64;
  ctx->hw64 = 0;
  ctx->n_pairs64 = 0;
  int sp_all, sp_bin, sp_tr;
  HIPCK(span_begin(ctx, 3, &sp_all));
  launch_kk_pack(ctx->d_R.as<cplx>(), ctx->ldt, n_g, n_gp, n_t, ctx->d_kk_rank.as<int>(),
                 ctx->d_kk_Rs.as<cplx>(), st);
  HIPCK(span_begin(ctx, 1, &sp_bin));
  launch_kk_bin(ctx->d_kk_Rs.as<cplx>(), n_gp, n_g, ctx->d_kk_ib.as<int>(), ctx->d_kk_xf.as<double>(),
                ctx->d_kk_chunks.as<KkChunk>(), (int)chunks.size(), ctx->d_kk_S.as<double>(),
                ctx->d_kk_S.as<double>() + e_off, st);
  HIPCK(span_end(ctx, sp_bin));
  LAUNCHCK("kk binning");
  launch_kk_matrix(ctx->d_w.as<double>(), n_w, eta, d, nbin[0], nbin[1], base[0], base[1], rows_p,
                   ldm, ctx->d_kk_K.as<double>(), st);
  // C64[2 n_w][2 n_pairs] = Kb^T S over the bins on FP64 MFMA
  const int nc = (int)(2 * n_pairs);
  HIPCK(span_begin(ctx, 6, &sp_tr));
  launch_kk_transform(ctx->d_kk_K.as<double>(), ldm, ctx->d_kk_S.as<double>(), nc, rows_p, 2 * n_w,
                      ctx->d_C64.as<double>(), st);
  HIPCK(span_end(ctx, sp_tr));
  LAUNCHCK("kk transform");
  HIPCK(span_end(ctx, sp_all));
  // what the assembly reads: one FP64 value of 2 n_w rows (Re K, Im K) x
  // (Re S, Im S) per pair
  Chi0Geom ga{};
  ga.n_g = n_g;
  ga.n_t = n_t;
  ga.n_w = n_w;
  ga.n_rows = ga.n_rowsp = ga.c_rows = 2 * n_w;
  ga.n_pairs = (int)n_pairs;
  ga.p0 = 0;
  ga.n_bulk = ga.n_bulkp = (int)n_pairs;
  ga.ksplit = 1;
  ctx->geom = ga;
  ctx->bulk_c64 = true;
  ctx->have_chi0 = true;
  if (chi0_out) {
    AsmArgs a{};
    a.C64 = ctx->d_C64.as<double>();
    a.ks = 1;
    a.vq = ctx->d_vq.as<double>();
    a.pref = 2.0 / (ctx->n_k * ctx->vol);
    launch_chi0_export(a, ga, static_cast<cplx*>(chi0_out), st);
    LAUNCHCK("chi0_export");
  }
  return QCX_OK;
}

int qcx_eps_inv(qcx_ctx* ctx, int lfe, void* diag_out, void* epsM_out) {
  if (!ctx) return QCX_EINVAL;
  if (!ctx->have_chi0) return fail(ctx, QCX_ESTATE, "chi0 first");
  if (lfe && ctx->n_g > 1024) return fail(ctx, QCX_EINVAL, "LFE inversion limited to n_G <= 1024");
  HIPCK(hipSetDevice(ctx->device));
  ctx->have_eps = false;
  hipStream_t st = ctx->stream;
  const Chi0Geom& g = ctx->geom;
  const int n = ctx->n_g, nw = ctx->n_w;
  HIPCK(ctx->d_eps.reserve(sizeof(cplx) * (size_t)nw * n * n));
  HIPCK(ctx->d_diag.reserve(sizeof(cplx) * (size_t)nw * n));
  HIPCK(ctx->d_epsM.reserve(sizeof(cplx) * (size_t)nw));
  HIPCK(ctx->d_loss.reserve(sizeof(double) * (size_t)nw * n));
  HIPCK(ctx->d_sing.reserve(sizeof(int)));
  launch_set_int(ctx->d_sing.as<int>(), INT_MAX, st);
  ctx->sing_armed = true;
  int sp_eps;
  HIPCK(span_begin(ctx, 4, &sp_eps));
  AsmArgs a{};
  a.C = (g.n_bulk > 0 && !ctx->bulk_c64) ? ctx->d_C.as<float>() : nullptr;
  a.C64 = (g.n_bulk > 0 && ctx->bulk_c64) ? ctx->d_C64.as<double>() : nullptr;
  a.XY = ctx->n_pairs64 > 0 ? ctx->d_XY.as<double>() : nullptr;
  a.ks = g.ksplit;
  a.ks64 = ctx->ks64;
  a.n_rowsp64 = ctx->geom64.n_rowsp;
  a.n_colp64 = ctx->geom64.n_colp;
  a.n_pairs64 = ctx->n_pairs64;
  a.vq = ctx->d_vq.as<double>();
  a.pref = 2.0 / (ctx->n_k * ctx->vol);
  launch_eps_assemble(a, g, ctx->d_eps.as<cplx>(), st);
  LAUNCHCK("eps_assemble");
  if (lfe)
    launch_gj_diag(ctx->d_eps.as<cplx>(), n, nw, ctx->d_diag.as<cplx>(), ctx->d_sing.as<int>(), st);
  else
    launch_nolfe_diag(ctx->d_eps.as<cplx>(), n, nw, ctx->d_diag.as<cplx>(), ctx->d_sing.as<int>(), st);
  LAUNCHCK("inverse");
  launch_loss(ctx->d_diag.as<cplx>(), n, nw, ctx->d_loss.as<double>(), ctx->d_epsM.as<cplx>(), st);
  LAUNCHCK("loss");
  HIPCK(span_end(ctx, sp_eps));
  if (diag_out)
    HIPCK(hipMemcpyAsync(diag_out, ctx->d_diag.p, sizeof(cplx) * (size_t)nw * n,
                         hipMemcpyDeviceToDevice, st));
  if (epsM_out)
    HIPCK(hipMemcpyAsync(epsM_out, ctx->d_epsM.p, sizeof(cplx) * (size_t)nw,
                         hipMemcpyDeviceToDevice, st));
  ctx->have_eps = true;
  return QCX_OK;
}

int qcx_eps_inv_given(qcx_ctx* ctx, int n_w, int n_G, const void* eps, int lfe, double* loss_out,
                      void* diag_out, void* epsM_out) {
  if (!ctx) return QCX_EINVAL;
  if (n_w < 1 || n_w > 65536) return fail(ctx, QCX_EINVAL, "need 1 <= n_w <= 65536");
  if (n_G < 1 || n_G > (lfe ? 1024 : 65536))
    return fail(ctx, QCX_EINVAL, lfe ? "need 1 <= n_G <= 1024" : "need 1 <= n_G <= 65536");
  if ((size_t)n_w * n_G * n_G > ((size_t)1 << 33)) return fail(ctx, QCX_EINVAL, "eps above 128 GB");
  if (!eps || !loss_out) return fail(ctx, QCX_EINVAL, "eps and loss_out must be device buffers");
  HIPCK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const size_t n = (size_t)n_G, nw = (size_t)n_w;
  // the inversion overwrites its matrices: work on a copy
  HIPCK(ctx->d_eps.reserve(sizeof(cplx) * nw * n * n));
  cplx* diag = static_cast<cplx*>(diag_out);
  if (!diag) {
    HIPCK(ctx->d_diag.reserve(sizeof(cplx) * nw * n));
    diag = ctx->d_diag.as<cplx>();
  }
  HIPCK(ctx->d_sing.reserve(sizeof(int)));
  // the context's own inversion results are no longer the latest
  ctx->have_eps = false;
  HIPCK(hipMemcpyAsync(ctx->d_eps.p, eps, sizeof(cplx) * nw * n * n, hipMemcpyDeviceToDevice, st));
  launch_set_int(ctx->d_sing.as<int>(), INT_MAX, st);
  ctx->sing_armed = true;
  if (lfe)
    launch_gj_diag(ctx->d_eps.as<cplx>(), n_G, n_w, diag, ctx->d_sing.as<int>(), st);
  else
    launch_nolfe_diag(ctx->d_eps.as<cplx>(), n_G, n_w, diag, ctx->d_sing.as<int>(), st);
  LAUNCHCK("inverse (given eps)");
  launch_loss(diag, n_G, n_w, loss_out, static_cast<cplx*>(epsM_out), st);
  LAUNCHCK("loss (given eps)");
  return QCX_OK;
}

int qcx_set_memory_limit(qcx_ctx* ctx, size_t bytes) {
  if (!ctx) return QCX_EINVAL;
  ctx->budget.limit = bytes;
  return QCX_OK;
}

int qcx_memory_used(const qcx_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return QCX_EINVAL;
  *bytes = ctx->budget.used;
  return QCX_OK;
}

int qcx_loss(qcx_ctx* ctx, double* out, int mem) {
  if (!ctx) return QCX_EINVAL;
  if (!ctx->have_eps) return fail(ctx, QCX_ESTATE, "eps_inv first");
  if (!out) return fail(ctx, QCX_EINVAL, "NULL out");
  HIPCK(hipSetDevice(ctx->device));
  const size_t bytes = sizeof(double) * (size_t)ctx->n_w * ctx->n_g;
  if (mem == QCX_MEM_DEVICE) {
    HIPCK(hipMemcpyAsync(out, ctx->d_loss.p, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    return QCX_OK;
  }
  if (mem != QCX_MEM_HOST) return fail(ctx, QCX_EINVAL, "bad mem");
  HIPCK(hipMemcpyAsync(out, ctx->d_loss.p, bytes, hipMemcpyDeviceToHost, ctx->stream));
  return qcx_sync(ctx);
}

}  // extern "C"
