// Pair densities of Eq. (RPA) in one pass per (G, tile of 16 k points): the
// 27-cell Bloch sum of the Gaussian Fourier integrals and the band
// contraction, with M(k; Q) held in LDS only (never written to memory).
//
//   M_mu,nu(k; Q) = sum_T e^{ik.T} F_mu,nu(Q, T)            (Bloch sum)
//   X_mu,v = sum_nu M_mu,nu C_nu,v(k)                         (ket, valence)
//   U_v,nu = sum_mu conj(C_mu,v(k')) M_mu,nu                  (bra, valence)
//   rho_vc = sum_mu conj(C_mu,c(k')) X_mu,v,  sigma_vc = sum_nu U_v,nu C_nu,c(k)
//
// with k' = k + q (or k in the optical limit).  This is the valence-first
// order of the band contraction (2 N_AO^2 n_occ + 2 N_AO n_occ n_c complex
// multiply-adds per (k, G) after the 27 N_AO^2 of the Bloch sum).
//
// Layout of the work.  The AO pairs (mu, nu) are grouped into 4 x 4 tiles
// (mu-quad, nu-quad); N_AO is padded to 4 NQ with zero rows.  The Bloch sum of
// one tile for the block's 16 k points is one FP64 MFMA product (16 x 16
// output, K = cells in steps of 4): A = F of the tile's 16 AO pairs by 4
// cells, B = e^{ik.T} for 4 cells by 16 k points; a complex product is three
// real ones (Gauss).  Tiles are produced in NQ chunks: chunk s holds the
// "diagonal" tiles (i, (i + s) mod NQ), i < NQ.  Each (k, mu-quad) X owner and
// each (k, nu-quad) U owner then finds exactly one tile of its own in every
// chunk, so the 64 complex multiply-adds per owner, band quad and chunk are
// spread evenly and the X and U sums stay in registers across chunks.
//
// A block has 512 threads: waves 0-3 form the tiles on MFMA into one of two
// LDS buffers while waves 4-7 (the owners) contract the other buffer, one
// barrier per chunk.  A final stage, all waves, forms rho and sigma from X and
// U in LDS, one (side, k, conduction band) per thread, with coalesced stores
// along c; its coefficients are loaded two groups ahead.
//
// Measured on the N_G = 113 workload (512 k, 28 AOs, 4 + 16 bands): 0.52 ms
// per q, of which the MFMA Bloch sums ~0.19, the owners' contraction ~0.09
// and the final stage ~0.12; FP64 MFMA and FP64 VALU work of the two roles
// does not overlap on gfx950, so the phases add.
//
// Blocks are ordered XCD-aware in super-tiles of GS G vectors by KS k tiles,
// so that the F slabs and state coefficients of a super-tile are read from
// memory once per XCD and then served by its L2.
#include <utility>

#include "common.h"

namespace qcx {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kKT = 16;   // k points per block (one MFMA column tile)
constexpr int kNTS = 7;   // MFMA K steps of 4 cells (up to 28 cells)
constexpr int kVO = 4;    // valence bands held per owner

struct BlockPos {
  int g, kt;
  bool live;
};

// Blocks are dealt round-robin over the 8 XCDs; consecutive logical indices
// are placed on one XCD and walk super-tiles of gs x ks (G, k tile) pairs.
__device__ inline BlockPos block_pos(int n_g, int n_kt, int gs, int ks) {
  const int nsg = (n_g + gs - 1) / gs, nsk = (n_kt + ks - 1) / ks;
  const int total = nsg * nsk * gs * ks;
  const int per = (total + 7) / 8;
  const int b = blockIdx.x;
  const int logical = (b % 8) * per + b / 8;
  if (logical >= total) return {0, 0, false};
  const int tile = logical / (gs * ks), inner = logical % (gs * ks);
  const int g = (tile / nsk) * gs + inner / ks;
  const int kt = (tile % nsk) * ks + inner % ks;
  return {g, kt, g < n_g && kt < n_kt};
}

__device__ inline void cmac(cplx& acc, cplx a, cplx b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
}

template <int NQ>
__global__ void __launch_bounds__(512) k_rho_fused(const cplx* __restrict__ F,
                                                   const cplx* __restrict__ ph,
                                                   const cplx* __restrict__ Ck,
                                                   const cplx* __restrict__ Cb, int n_ao, int n_b,
                                                   int n_occ, int n_k, int n_t, int n_g, int gs,
                                                   int ks, cplx* __restrict__ R, size_t ldt) {
  constexpr int NA4 = 4 * NQ;
  // two chunks of M tiles [tile][pair in tile][k] (chunk s in buffer s % 2);
  // after the chunks X [mu][v][k] in the first
  __shared__ cplx sM[2 * NQ * 16 * kKT];
  // valence columns of C(k) [nu][v][k]; after the chunks U [v][nu][k]
  __shared__ cplx sCk[NA4 * kVO * kKT];
  // valence columns of C(k') [mu][v][k]
  __shared__ cplx sCb[NA4 * kVO * kKT];

  const int n_kt = (n_k + kKT - 1) / kKT;
  const BlockPos bp = block_pos(n_g, n_kt, gs, ks);
  if (!bp.live) return;
  const int g = bp.g, k0 = bp.kt * kKT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n_c = n_b - n_occ;
  const cplx* Fg = F + (size_t)g * n_t * n_ao * n_ao;

  // Roles: waves 0-3 form the Bloch sums on MFMA (tiles i = wave, wave + 4 of
  // each chunk), waves 4-7 contract the previous chunk, so every SIMD pairs
  // one MFMA-bound wave with one VALU/LDS-bound wave.
  const bool producer = wave < 4;
  constexpr int TPW = (NQ + 3) / 4;  // tiles per producer wave and chunk

  // A operands of the producer's tiles (tile (i, (i + s) mod NQ) of chunk s):
  // pair e = lane % 16 of the tile, cell T = 4 st + lane / 16
  double ar[TPW][kNTS], ai[TPW][kNTS];
  auto load_tiles = [&](int s) {
    const int e = lane & 15;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      const int i = wave + 4 * u;
      const int mu = 4 * i + (e >> 2), nu = 4 * ((i + s) % NQ) + (e & 3);
      const bool ok = i < NQ && mu < n_ao && nu < n_ao;
#pragma unroll
      for (int st = 0; st < kNTS; ++st) {
        const int T = 4 * st + (lane >> 4);
        cplx f = {0.0, 0.0};
        if (ok && T < n_t) f = Fg[((size_t)T * n_ao + mu) * n_ao + nu];
        ar[u][st] = f.re;
        ai[u][st] = f.im;
      }
    }
  };
  if (producer) load_tiles(0);

  {
    // every load of the staging first, then the stores
    constexpr int NS = (NA4 * kVO * kKT + 511) / 512;
    cplx a[NS], b[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int i = tid + 512 * j;
      const int kk = i % kKT, v = (i / kKT) % kVO, mu = i / (kVO * kKT);
      const int k = k0 + kk;
      a[j] = b[j] = {0.0, 0.0};
      if (i < NA4 * kVO * kKT && mu < n_ao && v < n_occ && k < n_k) {
        const size_t o = ((size_t)k * n_ao + mu) * n_b + v;
        a[j] = Ck[o];
        b[j] = Cb[o];
      }
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int i = tid + 512 * j;
      if (i < NA4 * kVO * kKT) {
        sCk[i] = a[j];
        sCb[i] = b[j];
      }
    }
  }

  // B operand of every K step: lane holds e^{ik.T} for cell T = 4 st + lane/16
  // and k = k0 + lane%16 (zero past the cells and the k points)
  double pre[kNTS], pim[kNTS];
  if (producer) {
    const int k = k0 + (lane & 15);
#pragma unroll
    for (int st = 0; st < kNTS; ++st) {
      const int T = 4 * st + (lane >> 4);
      cplx p = {0.0, 0.0};
      if (T < n_t && k < n_k) p = ph[(size_t)k * n_t + T];
      pre[st] = p.re;
      pim[st] = p.im;
    }
  }

  // Three real products per complex one (Gauss):  t1 = Fr Pr, t2 = Fi Pi,
  // t3 = (Fr + Fi)(Pr + Pi);  M = (t1 - t2) + i (t3 - t1 - t2).
  // Chunk s of the producer's tiles into buffer s % 2, pair 4 r + lane/16 of
  // a tile and k = lane%16 from D[4 r + lane/16][lane%16].
  auto bloch_store = [&](int s) {
    cplx* buf = sM + (size_t)(s & 1) * NQ * 16 * kKT;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      const int i = wave + 4 * u;
      if (i >= NQ) break;
      f64x4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = t1, t3 = t1;
#pragma unroll
      for (int st = 0; st < kNTS; ++st) {
        t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[u][st], pre[st], t1, 0, 0, 0);
        t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[u][st], pim[st], t2, 0, 0, 0);
        t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[u][st] + ai[u][st], pre[st] + pim[st], t3,
                                                  0, 0, 0);
      }
      const f64x4 mr = t1 - t2, mi = t3 - t1 - t2;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        buf[(i * 16 + 4 * r + (lane >> 4)) * kKT + (lane & 15)] = {mr[r], mi[r]};
    }
  };

  // consumer owners: 16 lanes (lane = k) per owner = (X or U, quad); all four
  // valence bands in registers
  const int ct = tid - 256;
  const int kk = ct & 15, o = ct >> 4;
  const bool xo = o < NQ;
  const bool owner = !producer && o < 2 * NQ;
  const int oq = xo ? o : o - NQ;  // the owner's mu-quad (X) or nu-quad (U)
  cplx acc[4][kVO];                // X[mu 4 oq + q][v] or U[v][nu 4 oq + q]
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int v = 0; v < kVO; ++v) acc[q][v] = {0.0, 0.0};

  // contraction of chunk s (buffer s % 2):
  // X owner (quad m): tile m, X[q][v] += M[q][p] C_k[4 nq + p][v];
  // U owner (quad n): tile (n - s) mod NQ, U[v][q] += conj(C_k'[4 mq + p][v]) M[p][q].
  // One loop for both: p runs over the summed index, q over the owner's.
  auto band = [&](int s) {
    const int tile = xo ? oq : (oq - s + NQ) % NQ;
    const int cq = xo ? (oq + s) % NQ : tile;  // quad of the coefficient rows
    const cplx* m = sM + (size_t)(s & 1) * NQ * 16 * kKT + (size_t)tile * 16 * kKT + kk;
    const cplx* cbase = (xo ? sCk : sCb) + (size_t)(4 * cq) * kVO * kKT + kk;
    const int sp = xo ? 1 : 4, sq = xo ? 4 : 1;  // pair index 4 (mu) + nu
    const double sg = xo ? 1.0 : -1.0;           // conjugate the bra coefficients
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      cplx c[kVO];
#pragma unroll
      for (int v = 0; v < kVO; ++v) {
        c[v] = cbase[(p * kVO + v) * kKT];
        c[v].im *= sg;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const cplx x = m[(p * sp + q * sq) * kKT];
#pragma unroll
        for (int v = 0; v < kVO; ++v) cmac(acc[q][v], x, c[v]);
      }
    }
  };

  if (producer) {
    bloch_store(0);
    if (NQ > 1) load_tiles(1);
  }
  __syncthreads();
  // iteration s: consumers contract chunk s while producers form chunk s + 1
#pragma unroll 1
  for (int s = 0; s + 1 < NQ; ++s) {
    if (producer) {
      bloch_store(s + 1);
      if (s + 2 < NQ) load_tiles(s + 2);
    } else if (owner) {
      band(s);
    }
    __syncthreads();
  }

  // last stage: thread (side, k point kk2, band lane cl); side 0 rho with
  // conj(C_k'[mu][c]), side 1 sigma with C_k[nu][c].  The first group of
  // coefficients loads during the last chunk's contraction.
  const int cl = tid & 15, kk2 = (tid >> 4) & 15, side = tid >> 8, k2 = k0 + kk2;
  const cplx* cc = (side ? Ck : Cb) + (size_t)(k2 < n_k ? k2 : 0) * n_ao * n_b + n_occ;
  // coefficients in groups of MB rows, two groups loaded ahead of the one in
  // use (the first two in flight during the last contraction)
  constexpr int MB = 8;
  cplx cf[MB], cn[MB], cn2[MB];
  auto load = [&](int c, int m0, cplx (&dst)[MB]) {
#pragma unroll
    for (int j = 0; j < MB; ++j) {
      const int mu = m0 + j;
      dst[j] = (mu < n_ao && c < n_c) ? cc[(size_t)mu * n_b + c] : cplx{0.0, 0.0};
    }
  };
  load(cl, 0, cf);
  load(cl, MB, cn);
  if (owner) band(NQ - 1);
  __syncthreads();

  // X -> sM [mu][v][k], U -> sCk [v][nu][k]
  if (owner) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < kVO; ++v) {
        if (xo)
          sM[((4 * oq + q) * kVO + v) * kKT + kk] = acc[q][v];
        else
          sCk[(v * NA4 + 4 * oq + q) * kKT + kk] = acc[q][v];
      }
  }
  __syncthreads();

  if (k2 >= n_k) return;
  const double sg = side ? 1.0 : -1.0;
  const cplx* y0 = side ? sCk + kk2 : sM + kk2;
  const int ys_mu = side ? kKT : kVO * kKT, ys_v = side ? NA4 * kKT : kKT;
  cplx* Rg = R + (size_t)g * ldt + ((size_t)side * n_k + k2) * n_occ * n_c;
  for (int c = cl; c < n_c; c += 16) {
    if (c != cl) {
      load(c, 0, cf);
      load(c, MB, cn);
    }
    cplx r[kVO];
#pragma unroll
    for (int v = 0; v < kVO; ++v) r[v] = {0.0, 0.0};
#pragma unroll 1
    for (int m0 = 0; m0 < NA4; m0 += MB) {
      if (m0 + 2 * MB < NA4) load(c, m0 + 2 * MB, cn2);
#pragma unroll
      for (int j = 0; j < MB; ++j) {
        // rows past the padded basis hold no X or U (the last group of a basis
        // of 4 NQ rows may be partial): never read them, even times zero
        if (m0 + j >= NA4) break;
        const cplx a = {cf[j].re, sg * cf[j].im};
        const cplx* y = y0 + (size_t)(m0 + j) * ys_mu;
#pragma unroll
        for (int v = 0; v < kVO; ++v) cmac(r[v], a, y[v * ys_v]);
      }
#pragma unroll
      for (int j = 0; j < MB; ++j) {
        cf[j] = cn[j];
        cn[j] = cn2[j];
      }
    }
#pragma unroll
    for (int v = 0; v < kVO; ++v)
      if (v < n_occ) Rg[(size_t)v * n_c + c] = r[v];
  }
}

}  // namespace

bool rho_fused_fits(int n_ao, int n_occ, int n_t) {
  return n_ao <= 32 && n_occ <= kVO && n_t <= 4 * kNTS;
}

void launch_rho_fused(const cplx* F, const cplx* ph, const cplx* Ck, const cplx* Cb, int n_ao,
                      int n_b, int n_occ, int n_k, int n_t, int n_g, cplx* R, size_t ldt,
                      hipStream_t st) {
  const int nq = (n_ao + 3) / 4;
  const int n_kt = (n_k + kKT - 1) / kKT;
  const int gs = 4, ks = n_kt < 8 ? n_kt : 8;
  const long total = (long)((n_g + gs - 1) / gs) * gs * ((n_kt + ks - 1) / ks) * ks;
  const dim3 grid((unsigned)(8 * ((total + 7) / 8)));
#define QCX_RF(N)                                                                               \
  case N:                                                                                       \
    hipLaunchKernelGGL(k_rho_fused<N>, grid, dim3(512), 0, st, F, ph, Ck, Cb, n_ao, n_b, n_occ, \
                       n_k, n_t, n_g, gs, ks, R, ldt);                                          \
    return;
  switch (nq) {
    QCX_RF(1)
    QCX_RF(2)
    QCX_RF(3)
    QCX_RF(4)
    QCX_RF(5)
    QCX_RF(6)
    QCX_RF(7)
    QCX_RF(8)
    default: return;
  }
#undef QCX_RF
}

}  // namespace qcx
