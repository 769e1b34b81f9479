// From the dielectric function to scattering rates (Sec. III and Sec. II):
// three-dimensional momentum binning of the finite-momentum dielectric
// function eps(w, q + G), interpolation of bins without entries, the
// dynamic structure factor S(w, q) = q^2 / (2 pi alpha) Im(-1/eps) of Eq.
// (dynamic_structure_factor) averaged over directions, and the halo rate
//   dR/dw = rho_chi / (m_chi rho_T) * sigma_e / (4 pi mu^2)
//           * int dq q |F_DM(q)|^2 S(w, q) eta(v_min(q, w))
// (Eq. general_rate with the nonrelativistic cross section, Eq.
// cross_section; v_min of Eq. v_min with gamma = 1; F_DM of Eq. F_DM).
//
// Conventions: q in alpha m_e (= bohr^-1); shell s holds s dq <= |q| <
// (s + 1) dq; angular bins uniform in theta (acos(q_z / |q|), n_theta bins on
// [0, pi]) and phi (atan2(q_y, q_x) shifted to [0, 2 pi), n_phi bins); bin
// (s, i, j) = (s n_theta + i) n_phi + j.  The bin index of each entry is
// computed on the host (it depends only on q, not on w); the device sums
// eps over the entries of each bin, every bin of an add handled by one
// thread per frequency in entry order, so results do not depend on the
// launch.  Empty bins are filled in sweeps (each empty bin with filled
// neighbours among its 26 adjacent bins takes their mean; phi periodic;
// only bins filled before the sweep are used); the schedule depends only on
// which bins hold entries, so the host builds it and the device applies it
// to every frequency.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "ctx.h"

using qcx::cplx;
using qcx::DevBuf;

struct qcx_qbin {
  qcx_ctx* ctx = nullptr;
  int n_w = 0, n_shell = 0, n_theta = 0, n_phi = 0, n_ang = 0, n_bins = 0;
  double dq = 0.0;
  std::vector<long long> cnt;  // entries per bin
  DevBuf d_sum, d_eps, d_bins, d_off, d_ent, d_cnt, d_state, d_ft, d_fo, d_fi, d_om, d_w;
  void release() {
    DevBuf* all[] = {&d_sum, &d_eps, &d_bins, &d_off, &d_ent, &d_cnt,
                     &d_state, &d_ft, &d_fo, &d_fi, &d_om, &d_w};
    for (DevBuf* b : all) b->release();
  }
};

namespace qcx {
namespace {

constexpr double kAlpha = 7.2973525693e-3;      // fine-structure constant
constexpr double kMeEV = 510998.95;             // electron mass (eV)
constexpr double kAmeEV = kAlpha * kMeEV;       // alpha m_e (eV)
constexpr double kHbarcEVcm = 1.973269804e-5;   // hbar c (eV cm)
constexpr double kHbarEVs = 6.582119569e-16;    // hbar (eV s)
constexpr double kEVkg = 1.782661921e-36;       // eV / c^2 (kg)
constexpr double kCkms = 299792.458;            // c (km/s)
constexpr double kYear = 365.25 * 86400.0;      // s

// sum[w][bins[j]] += sum over entries ent[off[j] .. off[j+1]) of the value
// (eps, or 1 / value for kind 1)
__global__ void k_qbin_accum(const cplx* __restrict__ v, int ld, int kind, const int* __restrict__ bins,
                             const int* __restrict__ off, const int* __restrict__ ent, int n_pb,
                             int n_w, int n_bins, cplx* __restrict__ sum) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_pb * n_w) return;
  const int w = (int)(i / n_pb), j = (int)(i % n_pb);
  double re = 0.0, im = 0.0;
  for (int p = off[j]; p < off[j + 1]; ++p) {
    cplx x = v[(size_t)w * ld + ent[p]];
    if (kind == 1) {
      const double d = x.re * x.re + x.im * x.im;
      x = {x.re / d, -x.im / d};
    }
    re += x.re;
    im += x.im;
  }
  cplx& s = sum[(size_t)w * n_bins + bins[j]];
  s.re += re;
  s.im += im;
}

__global__ void k_qbin_mean(const cplx* __restrict__ sum, const int* __restrict__ cnt, int n_w,
                            int n_bins, cplx* __restrict__ eps) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_w * n_bins) return;
  const int c = cnt[i % n_bins];
  eps[i] = c > 0 ? cplx{sum[i].re / c, sum[i].im / c} : cplx{0.0, 0.0};
}

// one sweep: eps[w][tgt[j]] = mean of eps[w][nidx[noff[j] .. noff[j+1])]
__global__ void k_qbin_fill(cplx* __restrict__ eps, int n_w, int n_bins, const int* __restrict__ tgt,
                            const int* __restrict__ noff, const int* __restrict__ nidx, int n_t) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_w * n_t) return;
  const int w = (int)(i / n_t), j = (int)(i % n_t);
  double re = 0.0, im = 0.0;
  const int p0 = noff[j], p1 = noff[j + 1];
  for (int p = p0; p < p1; ++p) {
    const cplx x = eps[(size_t)w * n_bins + nidx[p]];
    re += x.re;
    im += x.im;
  }
  eps[(size_t)w * n_bins + tgt[j]] = {re / (p1 - p0), im / (p1 - p0)};
}

// S(w, q_s): solid-angle weighted mean of q_s^2 / (2 pi alpha) Im(-1/eps)
// over the filled bins of shell s (NaN if none)
__global__ void k_qbin_siso(const cplx* __restrict__ eps, const int* __restrict__ state,
                            const double* __restrict__ om, int n_w, int n_shell, int n_ang,
                            double dq, double* __restrict__ S) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_w * n_shell) return;
  const int w = (int)(i / n_shell), s = (int)(i % n_shell);
  const int n_bins = n_shell * n_ang;
  const double q = (s + 0.5) * dq, pre = q * q / (2.0 * kPi * kAlpha);
  double acc = 0.0, ws = 0.0;
  for (int a = 0; a < n_ang; ++a) {
    const int b = s * n_ang + a;
    if (state[b] <= 0) continue;
    const cplx e = eps[(size_t)w * n_bins + b];
    acc += om[a] * (pre * (e.im / (e.re * e.re + e.im * e.im)));   // Im(-1/eps)
    ws += om[a];
  }
  S[i] = ws > 0.0 ? acc / ws : __builtin_nan("");
}

struct Halo {
  double v0, vE, vesc;     // km/s
  double m_chi;            // eV
  double m2;               // (m_med / alpha m_e)^2, < 0 for the heavy limit
  double pref;             // everything in front of the q integral
};

// mean inverse speed (s/km) of the truncated Maxwell-Boltzmann halo above
// vmin (km/s): the standard closed form of int d^3v f(v) / v, v > vmin
__device__ double eta_shm(double vmin, const Halo& h) {
  const double x = vmin / h.v0, y = h.vE / h.v0, z = h.vesc / h.v0;
  const double rsp = 0.56418958354775628;  // 1 / sqrt(pi)
  const double ez = exp(-z * z);
  const double N = erf(z) - 2.0 * z * ez * rsp;
  double r;
  if (x < z - y)
    r = erf(x + y) - erf(x - y) - 4.0 * y * ez * rsp;
  else if (x < z + y)
    r = erf(z) - erf(x - y) - 2.0 * (z + y - x) * ez * rsp;
  else
    return 0.0;
  return r / (2.0 * N * y * h.v0);
}

__global__ void k_rate_halo(const double* __restrict__ w, int n_w, const double* __restrict__ S,
                            int n_shell, double dq, Halo h, double* __restrict__ rate) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_w) return;
  double tot = 0.0;
  for (int s = 0; s < n_shell; ++s) {
    const double Sv = S[(size_t)a * n_shell + s];
    if (!isfinite(Sv)) continue;
    const double q = (s + 0.5) * dq, q_ev = q * kAmeEV;
    const double vmin = (q_ev / (2.0 * h.m_chi) + w[a] / q_ev) * kCkms;
    const double eta = eta_shm(vmin, h) * kCkms;              // in units of 1/c
    const double F = h.m2 < 0.0 ? 1.0 : (1.0 + h.m2) / (q * q + h.m2);
    tot += dq * kAmeEV * q_ev * F * F * Sv * kAmeEV * kAmeEV * eta;
  }
  rate[a] = h.pref * tot;
}

inline unsigned blocks(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace qcx

using namespace qcx;

namespace {

int bin_of(const qcx_qbin* b, const double* q) {
#pragma clang fp contract(off)  // the same roundings as a plain evaluation of |q|
  const double r = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
  if (!(r > 0.0) || !(r < b->n_shell * b->dq)) return -1;
  const int s = std::min((int)std::floor(r / b->dq), b->n_shell - 1);
  const double th = std::acos(std::min(1.0, std::max(-1.0, q[2] / r)));
  double ph = std::atan2(q[1], q[0]);
  if (ph < 0.0) ph += 2.0 * kPi;
  const int i = std::min((int)std::floor(th / (kPi / b->n_theta)), b->n_theta - 1);
  const int j = std::min((int)std::floor(ph / (2.0 * kPi / b->n_phi)), b->n_phi - 1);
  return (s * b->n_theta + i) * b->n_phi + j;
}

// the distinct neighbours of bin id among the 26 adjacent bins
void neighbours(const qcx_qbin* b, int id, std::vector<int>& out) {
  out.clear();
  const int s = id / b->n_ang, rem = id % b->n_ang, i = rem / b->n_phi, j = rem % b->n_phi;
  for (int ds = -1; ds <= 1; ++ds)
    for (int di = -1; di <= 1; ++di)
      for (int dj = -1; dj <= 1; ++dj) {
        if (ds == 0 && di == 0 && dj == 0) continue;
        const int s2 = s + ds, i2 = i + di;
        if (s2 < 0 || s2 >= b->n_shell || i2 < 0 || i2 >= b->n_theta) continue;
        const int j2 = ((j + dj) % b->n_phi + b->n_phi) % b->n_phi;
        const int nb = (s2 * b->n_theta + i2) * b->n_phi + j2;
        if (std::find(out.begin(), out.end(), nb) == out.end()) out.push_back(nb);
      }
}

}  // namespace

extern "C" {

int qcx_qbin_create(qcx_qbin** out, qcx_ctx* ctx, int n_w, int n_shell, double dq, int n_theta,
                    int n_phi) {
  if (!out || !ctx) return QCX_EINVAL;
  *out = nullptr;
  if (n_w < 1 || n_w > 65536) return fail(ctx, QCX_EINVAL, "need 1 <= n_w <= 65536");
  if (n_shell < 1 || n_theta < 1 || n_theta > 360 || n_phi < 1 || n_phi > 720)
    return fail(ctx, QCX_EINVAL, "need n_shell >= 1, 1 <= n_theta <= 360, 1 <= n_phi <= 720");
  if (!(dq > 0.0) || !std::isfinite(dq)) return fail(ctx, QCX_EINVAL, "dq must be > 0");
  const double nb = (double)n_shell * n_theta * n_phi;
  if (nb > (double)(1 << 26) || nb * n_w * sizeof(cplx) > 32.0 * (1 << 30))
    return fail(ctx, QCX_EINVAL, "bin table above 2^26 bins or 32 GB");
  HIPCK(hipSetDevice(ctx->device));
  qcx_qbin* b = new qcx_qbin();
  b->ctx = ctx;
  b->n_w = n_w;
  b->n_shell = n_shell;
  b->n_theta = n_theta;
  b->n_phi = n_phi;
  b->n_ang = n_theta * n_phi;
  b->n_bins = (int)nb;
  b->dq = dq;
  b->cnt.assign(b->n_bins, 0);
  const size_t bytes = sizeof(cplx) * (size_t)n_w * b->n_bins;
  hipError_t e = b->d_sum.reserve(bytes);
  if (e == hipSuccess) e = hipMemsetAsync(b->d_sum.p, 0, bytes, ctx->stream);
  if (e != hipSuccess) {
    b->release();
    delete b;
    return fail(ctx, e == hipErrorOutOfMemory ? QCX_ENOMEM : QCX_EDEVICE, hipGetErrorString(e));
  }
  *out = b;
  return QCX_OK;
}

int qcx_qbin_destroy(qcx_qbin* b) {
  if (!b) return QCX_OK;
  (void)hipSetDevice(b->ctx->device);
  (void)hipStreamSynchronize(b->ctx->stream);
  b->release();
  delete b;
  return QCX_OK;
}

int qcx_qbin_reset(qcx_qbin* b) {
  if (!b) return QCX_EINVAL;
  qcx_ctx* ctx = b->ctx;
  HIPCK(hipSetDevice(ctx->device));
  std::fill(b->cnt.begin(), b->cnt.end(), 0);
  HIPCK(hipMemsetAsync(b->d_sum.p, 0, sizeof(cplx) * (size_t)b->n_w * b->n_bins, ctx->stream));
  return QCX_OK;
}

int qcx_qbin_add(qcx_qbin* b, int n, const double* qvec, const void* vals, int ld, int kind) {
  if (!b) return QCX_EINVAL;
  qcx_ctx* ctx = b->ctx;
  if (n < 1 || !qvec || !vals) return fail(ctx, QCX_EINVAL, "need n >= 1, qvec and vals");
  if (ld < n) return fail(ctx, QCX_EINVAL, "ld must be >= n");
  if (kind != QCX_QBIN_EPS && kind != QCX_QBIN_INV) return fail(ctx, QCX_EINVAL, "bad kind");
  for (int e = 0; e < 3 * n; ++e)
    if (!std::isfinite(qvec[e])) return fail(ctx, QCX_EINVAL, "non-finite momentum");
  if (int rc = reject_capture(ctx)) return rc;
  HIPCK(hipSetDevice(ctx->device));
  // entries grouped by bin (entry order kept inside a bin)
  std::vector<std::pair<int, int>> be;
  be.reserve(n);
  for (int e = 0; e < n; ++e) {
    const int id = bin_of(b, qvec + 3 * (size_t)e);
    if (id >= 0) be.push_back({id, e});
  }
  if (be.empty()) return QCX_OK;
  std::stable_sort(be.begin(), be.end(),
                   [](const std::pair<int, int>& x, const std::pair<int, int>& y) { return x.first < y.first; });
  std::vector<int> bins, off, ent(be.size());
  for (size_t p = 0; p < be.size(); ++p) {
    if (p == 0 || be[p].first != be[p - 1].first) {
      bins.push_back(be[p].first);
      off.push_back((int)p);
    }
    ent[p] = be[p].second;
    ++b->cnt[be[p].first];
  }
  off.push_back((int)be.size());
  HIPCK(stage_begin(ctx));
  HIPCK(upload(ctx, b->d_bins, bins.data(), bins.size()));
  HIPCK(upload(ctx, b->d_off, off.data(), off.size()));
  HIPCK(upload(ctx, b->d_ent, ent.data(), ent.size()));
  const int n_pb = (int)bins.size();
  hipLaunchKernelGGL(k_qbin_accum, dim3(blocks((long)n_pb * b->n_w)), dim3(256), 0, ctx->stream,
                     static_cast<const cplx*>(vals), ld, kind, b->d_bins.as<int>(), b->d_off.as<int>(),
                     b->d_ent.as<int>(), n_pb, b->n_w, b->n_bins, b->d_sum.as<cplx>());
  LAUNCHCK("qbin accumulate");
  return QCX_OK;
}

int qcx_qbin_finish(qcx_qbin* b, void* eps_out, double* S_out, int* state_out) {
  if (!b) return QCX_EINVAL;
  qcx_ctx* ctx = b->ctx;
  if (!S_out) return fail(ctx, QCX_EINVAL, "S_out is required");
  if (int rc = reject_capture(ctx)) return rc;
  HIPCK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int nb = b->n_bins, n_w = b->n_w;
  std::vector<int> cnt(nb), state(nb);
  for (int i = 0; i < nb; ++i) {
    cnt[i] = (int)std::min<long long>(b->cnt[i], INT_MAX);
    state[i] = b->cnt[i] > 0 ? 1 : 0;
  }
  // interpolation schedule: sweeps of (target, neighbours filled before it)
  std::vector<int> ft, fo, fi, sweep_t0;
  std::vector<int> nbr;
  for (;;) {
    const size_t t0 = ft.size();
    sweep_t0.push_back((int)t0);
    for (int id = 0; id < nb; ++id) {
      if (state[id] != 0) continue;
      neighbours(b, id, nbr);
      const size_t i0 = fi.size();
      for (int x : nbr)
        if (state[x] > 0) fi.push_back(x);
      if (fi.size() > i0) {
        ft.push_back(id);
        fo.push_back((int)i0);
      } else {
        fi.resize(i0);
      }
    }
    if (ft.size() == t0) {
      sweep_t0.pop_back();
      break;
    }
    for (size_t k = t0; k < ft.size(); ++k) state[ft[k]] = 2;
  }
  fo.push_back((int)fi.size());
  std::vector<double> om(b->n_ang);
  for (int i = 0; i < b->n_theta; ++i) {
    const double t1 = i * (kPi / b->n_theta), t2 = (i + 1) * (kPi / b->n_theta);
    for (int j = 0; j < b->n_phi; ++j) om[i * b->n_phi + j] = (2.0 * kPi / b->n_phi) * (std::cos(t1) - std::cos(t2));
  }
  HIPCK(stage_begin(ctx));
  HIPCK(upload(ctx, b->d_cnt, cnt.data(), cnt.size()));
  HIPCK(upload(ctx, b->d_state, state.data(), state.size()));
  HIPCK(upload(ctx, b->d_om, om.data(), om.size()));
  if (!ft.empty()) {
    HIPCK(upload(ctx, b->d_ft, ft.data(), ft.size()));
    HIPCK(upload(ctx, b->d_fo, fo.data(), fo.size()));
    HIPCK(upload(ctx, b->d_fi, fi.data(), fi.size()));
  }
  HIPCK(b->d_eps.reserve(sizeof(cplx) * (size_t)n_w * nb));
  hipLaunchKernelGGL(k_qbin_mean, dim3(blocks((long)n_w * nb)), dim3(256), 0, st, b->d_sum.as<cplx>(),
                     b->d_cnt.as<int>(), n_w, nb, b->d_eps.as<cplx>());
  for (size_t k = 0; k < sweep_t0.size(); ++k) {
    const int t0 = sweep_t0[k], t1 = k + 1 < sweep_t0.size() ? sweep_t0[k + 1] : (int)ft.size();
    hipLaunchKernelGGL(k_qbin_fill, dim3(blocks((long)n_w * (t1 - t0))), dim3(256), 0, st,
                       b->d_eps.as<cplx>(), n_w, nb, b->d_ft.as<int>() + t0, b->d_fo.as<int>() + t0,
                       b->d_fi.as<int>(), t1 - t0);
  }
  hipLaunchKernelGGL(k_qbin_siso, dim3(blocks((long)n_w * b->n_shell)), dim3(256), 0, st,
                     b->d_eps.as<cplx>(), b->d_state.as<int>(), b->d_om.as<double>(), n_w, b->n_shell,
                     b->n_ang, b->dq, S_out);
  LAUNCHCK("qbin finish");
  if (eps_out)
    HIPCK(hipMemcpyAsync(eps_out, b->d_eps.p, sizeof(cplx) * (size_t)n_w * nb, hipMemcpyDeviceToDevice, st));
  if (state_out) std::copy(state.begin(), state.end(), state_out);
  return QCX_OK;
}

int qcx_qbin_rate_halo(qcx_qbin* b, const double* w_eV, const double* S_iso, const qcx_halo* h,
                       double* rate_out) {
  if (!b) return QCX_EINVAL;
  qcx_ctx* ctx = b->ctx;
  if (!w_eV || !S_iso || !h || !rate_out) return fail(ctx, QCX_EINVAL, "NULL argument");
  const double pos[] = {h->m_chi_eV, h->sigma_e_cm2, h->rho_T_g_cm3, h->rho_chi_GeV_cm3,
                        h->v0_kms, h->vE_kms, h->vesc_kms};
  for (double x : pos)
    if (!(x > 0.0) || !std::isfinite(x)) return fail(ctx, QCX_EINVAL, "halo parameters must be > 0");
  if (!(h->m_med_eV >= 0.0)) return fail(ctx, QCX_EINVAL, "mediator mass must be >= 0 (inf: heavy)");
  std::vector<double> w(b->n_w);
  for (int a = 0; a < b->n_w; ++a) {
    if (!(w_eV[a] >= 0.0) || !std::isfinite(w_eV[a])) return fail(ctx, QCX_EINVAL, "frequencies must be >= 0");
    w[a] = w_eV[a];
  }
  if (int rc = reject_capture(ctx)) return rc;
  HIPCK(hipSetDevice(ctx->device));
  const double mu = h->m_chi_eV * kMeEV / (h->m_chi_eV + kMeEV);
  const double n_chi = h->rho_chi_GeV_cm3 * 1e9 / h->m_chi_eV * std::pow(kHbarcEVcm, 3);   // eV^3
  const double rho_T = h->rho_T_g_cm3 * 1e-3 / kEVkg * std::pow(kHbarcEVcm, 3);          // eV^4
  const double sigma = h->sigma_e_cm2 / (kHbarcEVcm * kHbarcEVcm);                       // eV^-2
  Halo hk;
  hk.v0 = h->v0_kms;
  hk.vE = h->vE_kms;
  hk.vesc = h->vesc_kms;
  hk.m_chi = h->m_chi_eV;
  hk.m2 = std::isinf(h->m_med_eV) ? -1.0 : (h->m_med_eV / kAmeEV) * (h->m_med_eV / kAmeEV);
  // eV^-1 (natural) -> events / kg / year / eV
  hk.pref = n_chi / rho_T * sigma / (4.0 * kPi * mu * mu) / kHbarEVs / kEVkg * kYear;
  HIPCK(stage_begin(ctx));
  HIPCK(upload(ctx, b->d_w, w.data(), w.size()));
  hipLaunchKernelGGL(k_rate_halo, dim3(blocks(b->n_w)), dim3(256), 0, ctx->stream, b->d_w.as<double>(),
                     b->n_w, S_iso, b->n_shell, b->dq, hk, rate_out);
  LAUNCHCK("rate_halo");
  return QCX_OK;
}

}  // extern "C"
