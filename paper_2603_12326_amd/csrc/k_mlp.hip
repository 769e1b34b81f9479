// Kernels of the loss surrogate: a 5 -> 256x4 -> 1 SiLU network trained and
// evaluated on the GPU.
//
// Arithmetic (BF16 weights, FP32 accumulation):
//   layer 1 (5 inputs): FP32 on the vector ALUs with bf16-rounded weights;
//   layers 2..4: v_mfma_f32_32x32x16_bf16 on bf16(h) and bf16(W), FP32 sums;
//   output: FP32 dot product of bf16(h4) and bf16(w5);
//   backward: the same products with bf16(dz); bias gradients, the loss and
//   the first layer's gradient in FP32; Adam on FP32 master weights, after
//   which the bf16 copies (and their transposes) are refreshed.
// Every GEMM is "NT": C[m][n] = sum_k A[m][k] B[n][k] with both operands
// k-contiguous, so forward (A = H, B = W), input gradient (A = dZ,
// B = W^T) and weight gradient (A = dZ^T, B = H^T) share one kernel; the
// epilogues that produce H and dZ also write their transposes for the
// weight-gradient product.
#include <math.h>

#include "mlp.h"

namespace qcx {
namespace mlp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline uint16_t to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline float from_bf16(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}
__device__ inline float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigm(z); }
__device__ inline float silu_grad(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// bf16 NT GEMM, block tile 64 x 64, 4 waves of 32 x 32, K step 32 staged in
// LDS (rows padded to 40 elements = 80 bytes, 16-byte aligned).
// Requirements (met by every caller: rows padded to 64, width 256): M % 64 ==
// N % 64 == 0, K % 32 == 0,
// lda = ldb = K.
// v_mfma_f32_32x32x16_bf16 lane layouts: A lane l holds A[l%32][8(l/32)+i],
// B lane l holds B[8(l/32)+i][l%32] (= Bt[l%32][...]), i = 0..7; result
// register r of lane l is C[8(r/4) + 4(l/32) + r%4][l%32].
// ---------------------------------------------------------------------------
constexpr int LDK = 40;
enum { EPI_FWD = 0, EPI_BWD = 1, EPI_STORE = 2 };

struct EpiAll {
  EpiFwd f;
  EpiBwd b;
  float* C;
};

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_nt(const uint16_t* __restrict__ A,
                                                 const uint16_t* __restrict__ B, int M, int N,
                                                 int K, EpiAll e) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[64 * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sB[64 * LDK];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  // K range of this block: split z of gridDim.z (EPI_STORE only; 1 otherwise)
  const int kper = K / gridDim.z, kb = blockIdx.z * kper, ke = kb + kper;
  const uint16_t* pa = A + (size_t)(m0 + lr) * K + kb + lk;
  const uint16_t* pb = B + (size_t)(n0 + lr) * K + kb + lk;
  f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
  uint4 ra = *reinterpret_cast<const uint4*>(pa);
  uint4 rb = *reinterpret_cast<const uint4*>(pb);
  for (int k0 = 0; k0 < ke - kb; k0 += 32) {
    __syncthreads();
    *reinterpret_cast<uint4*>(sA + lr * LDK + lk) = ra;
    *reinterpret_cast<uint4*>(sB + lr * LDK + lk) = rb;
    __syncthreads();
    if (k0 + 32 < ke - kb) {  // prefetch the next K step while this one computes
      ra = *reinterpret_cast<const uint4*>(pa + k0 + 32);
      rb = *reinterpret_cast<const uint4*>(pb + k0 + 32);
    }
#pragma unroll
    for (int kk = 0; kk < 32; kk += 16) {
      const bf16x8 af =
          *reinterpret_cast<const bf16x8*>(sA + (wm + (lane & 31)) * LDK + kk + 8 * (lane >> 5));
      const bf16x8 bf =
          *reinterpret_cast<const bf16x8*>(sB + (wn + (lane & 31)) * LDK + kk + 8 * (lane >> 5));
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bf, acc, 0, 0, 0);
    }
  }
  const int n = n0 + wn + (lane & 31);
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int mb = m0 + wm + 8 * g + 4 * (lane >> 5);  // rows mb .. mb+3
    if constexpr (EPI == EPI_STORE) {
      float* C = e.C + (size_t)blockIdx.z * M * N;
#pragma unroll
      for (int i = 0; i < 4; ++i) C[(size_t)(mb + i) * N + n] = acc[4 * g + i];
    } else if constexpr (EPI == EPI_FWD) {
      const float bias = e.f.bias[n];
      uint16_t hb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float z = acc[4 * g + i] + bias;
        if (e.f.Z) e.f.Z[(size_t)(mb + i) * N + n] = z;
        hb[i] = to_bf16(silu(z));
        e.f.Hb[(size_t)(mb + i) * N + n] = hb[i];
      }
      if (e.f.HT) {
        uint2 v;
        v.x = (uint32_t)hb[0] | ((uint32_t)hb[1] << 16);
        v.y = (uint32_t)hb[2] | ((uint32_t)hb[3] << 16);
        *reinterpret_cast<uint2*>(e.f.HT + (size_t)n * e.f.ldt + mb) = v;
      }
    } else {
      uint16_t db[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const size_t o = (size_t)(mb + i) * N + n;
        const float dz = acc[4 * g + i] * silu_grad(e.b.Zprev[o]);
        e.b.dZ[o] = dz;
        db[i] = to_bf16(dz);
        e.b.dZb[o] = db[i];
      }
      uint2 v;
      v.x = (uint32_t)db[0] | ((uint32_t)db[1] << 16);
      v.y = (uint32_t)db[2] | ((uint32_t)db[3] << 16);
      *reinterpret_cast<uint2*>(e.b.dZbT + (size_t)n * e.b.ldt + mb) = v;
    }
  }
}

// ---------------------------------------------------------------------------
// first layer: block = 256 threads = 256 neurons, 16 rows per block
// ---------------------------------------------------------------------------
constexpr int L1_ROWS = 16;
__global__ void __launch_bounds__(256) k_layer1(const float* __restrict__ x,
                                                const int* __restrict__ order, long off, int n,
                                                const uint16_t* __restrict__ w1b,
                                                const float* __restrict__ b1, float* Z1,
                                                uint16_t* H1b, uint16_t* H1T, int ldt) {
  __shared__ float sx[L1_ROWS][kIn];
  const int j = threadIdx.x, r0 = blockIdx.x * L1_ROWS;
  for (int e = j; e < L1_ROWS * kIn; e += 256) {
    const int r = r0 + e / kIn, c = e % kIn;
    float v = 0.0f;
    if (r < n) {
      const long src = order ? (long)order[off + r] : (long)r;
      v = x[src * kIn + c];
    }
    sx[e / kIn][c] = v;
  }
  __syncthreads();
  float w[kIn];
#pragma unroll
  for (int c = 0; c < kIn; ++c) w[c] = from_bf16(w1b[j * kIn + c]);
  const float b = b1[j];
  uint16_t hb[L1_ROWS];
#pragma unroll
  for (int r = 0; r < L1_ROWS; ++r) {
    float z = b;
#pragma unroll
    for (int c = 0; c < kIn; ++c) z += sx[r][c] * w[c];
    if (Z1) Z1[(size_t)(r0 + r) * kW + j] = z;
    hb[r] = to_bf16(silu(z));
    H1b[(size_t)(r0 + r) * kW + j] = hb[r];
  }
  if (H1T) {
    uint4* dst = reinterpret_cast<uint4*>(H1T + (size_t)j * ldt + r0);
#pragma unroll
    for (int q = 0; q < L1_ROWS / 8; ++q) {
      uint4 v;
      v.x = hb[8 * q + 0] | ((uint32_t)hb[8 * q + 1] << 16);
      v.y = hb[8 * q + 2] | ((uint32_t)hb[8 * q + 3] << 16);
      v.z = hb[8 * q + 4] | ((uint32_t)hb[8 * q + 5] << 16);
      v.w = hb[8 * q + 6] | ((uint32_t)hb[8 * q + 7] << 16);
      dst[q] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// output layer (+ loss and layer-4 backward in training): block = 256 threads
// = 256 neurons, 16 rows per block; the dot products reduce through LDS.
// ---------------------------------------------------------------------------
constexpr int OUT_ROWS = 16;
__global__ void __launch_bounds__(256) k_output(const uint16_t* __restrict__ H4b,
                                                const uint16_t* __restrict__ w5b,
                                                const float* __restrict__ b5, int n, float* y,
                                                const float* __restrict__ t,
                                                const int* __restrict__ order, long off,
                                                float* dy, float* sq, const float* Z4, float* dZ,
                                                uint16_t* dZb, uint16_t* dZbT, int ldt) {
  __shared__ float red[4][OUT_ROWS];
  __shared__ float sdy[OUT_ROWS];
  const int j = threadIdx.x, lane = j & 63, wave = j >> 6, r0 = blockIdx.x * OUT_ROWS;
  const float w = from_bf16(w5b[j]);
  for (int r = 0; r < OUT_ROWS; ++r) {
    float p = from_bf16(H4b[(size_t)(r0 + r) * kW + j]) * w;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) p += __shfl_xor(p, o, 64);
    if (lane == 0) red[wave][r] = p;
  }
  __syncthreads();
  if (j < OUT_ROWS) {
    const int r = r0 + j;
    const float yr = ((red[0][j] + red[1][j]) + (red[2][j] + red[3][j])) + b5[0];
    if (r < n) y[r] = yr;
    if (t) {
      float d = 0.0f, s = 0.0f;
      if (r < n) {
        const long src = order ? (long)order[off + r] : (long)r;
        const float e = yr - t[src];
        d = 2.0f * e / (float)n;
        s = e * e;
      }
      dy[r] = d;
      sq[r] = s;
      sdy[j] = d;
    }
  }
  if (!t) return;
  __syncthreads();
  uint16_t db[OUT_ROWS];
#pragma unroll
  for (int r = 0; r < OUT_ROWS; ++r) {
    const size_t o = (size_t)(r0 + r) * kW + j;
    const float dz = sdy[r] * w * silu_grad(Z4[o]);
    dZ[o] = dz;
    db[r] = to_bf16(dz);
    dZb[o] = db[r];
  }
  uint4* dst = reinterpret_cast<uint4*>(dZbT + (size_t)j * ldt + r0);
#pragma unroll
  for (int q = 0; q < OUT_ROWS / 8; ++q) {
    uint4 v;
    v.x = db[8 * q + 0] | ((uint32_t)db[8 * q + 1] << 16);
    v.y = db[8 * q + 2] | ((uint32_t)db[8 * q + 3] << 16);
    v.z = db[8 * q + 4] | ((uint32_t)db[8 * q + 5] << 16);
    v.w = db[8 * q + 6] | ((uint32_t)db[8 * q + 7] << 16);
    dst[q] = v;
  }
}

// ---------------------------------------------------------------------------
// column reductions over the batch (deterministic: fixed per-thread strides,
// fixed LDS tree).  Block = 256 threads = 4 row streams x 64 columns.
// ---------------------------------------------------------------------------
// Column sums over rows run in two stages, so that a batch of thousands of
// rows spreads over hundreds of blocks and the result does not depend on
// timing: blocks of kRedRows rows write one partial per column, then the
// partials are added in chunk order.
//   P[ch][c] = sum over rows r of chunk ch of A[r][c]
__global__ void __launch_bounds__(256) k_colsum_part(const float* __restrict__ A, int rows, int cols,
                                                     float* P) {
  __shared__ float part[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), s = threadIdx.x >> 6;
  const int r0 = blockIdx.y * kRedRows, r1 = min(rows, r0 + kRedRows);
  float acc = 0.0f;
  if (c < cols)
    for (int r = r0 + s; r < r1; r += 4) acc += A[(size_t)r * cols + c];
  part[s][threadIdx.x & 63] = acc;
  __syncthreads();
  if (s == 0 && c < cols)
    P[(size_t)blockIdx.y * cols + c] = (part[0][threadIdx.x] + part[1][threadIdx.x]) +
                                       (part[2][threadIdx.x] + part[3][threadIdx.x]);
}

// P[ch][c] = sum over chunk rows of dy[r] bf16(h4)[r][c] for c < kW, and
// P[ch][kW] = sum of dy[r]
__global__ void __launch_bounds__(256) k_out_grad_part(const uint16_t* __restrict__ H4b,
                                                       const float* __restrict__ dy, int rows,
                                                       float* P) {
  __shared__ float part[4][64], partb[4];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), s = threadIdx.x >> 6;
  const int r0 = blockIdx.y * kRedRows, r1 = min(rows, r0 + kRedRows);
  float acc = 0.0f, accb = 0.0f;
  for (int r = r0 + s; r < r1; r += 4) {
    const float d = dy[r];
    acc += d * from_bf16(H4b[(size_t)r * kW + c]);
    accb += d;
  }
  part[s][threadIdx.x & 63] = acc;
  if ((threadIdx.x & 63) == 0) partb[s] = accb;
  __syncthreads();
  float* Pc = P + (size_t)blockIdx.y * (kW + 1);
  if (s == 0)
    Pc[c] = (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
  if (blockIdx.x == 0 && threadIdx.x == 0) Pc[kW] = (partb[0] + partb[1]) + (partb[2] + partb[3]);
}

// P[ch][c][i] = sum over chunk rows of dz1[r][c] x[idx(r)][i] for i < kIn,
// P[ch][c][kIn] = sum of dz1[r][c]
__global__ void __launch_bounds__(256) k_w1_grad_part(const float* __restrict__ dZ1,
                                                      const float* __restrict__ x,
                                                      const int* __restrict__ order, long off,
                                                      int n, float* P) {
  __shared__ float part[4][64][kIn + 1];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), s = threadIdx.x >> 6;
  const int r0 = blockIdx.y * kRedRows, r1 = min(n, r0 + kRedRows);
  float acc[kIn + 1];
#pragma unroll
  for (int i = 0; i <= kIn; ++i) acc[i] = 0.0f;
  for (int r = r0 + s; r < r1; r += 4) {
    const float d = dZ1[(size_t)r * kW + c];
    const long src = order ? (long)order[off + r] : (long)r;
#pragma unroll
    for (int i = 0; i < kIn; ++i) acc[i] += d * x[src * kIn + i];
    acc[kIn] += d;
  }
#pragma unroll
  for (int i = 0; i <= kIn; ++i) part[s][threadIdx.x & 63][i] = acc[i];
  __syncthreads();
  float* Pc = P + (size_t)blockIdx.y * kW * (kIn + 1);
  for (int e = threadIdx.x; e < 64 * (kIn + 1); e += 256) {
    const int cc = e / (kIn + 1), i = e % (kIn + 1);
    Pc[(size_t)(blockIdx.x * 64 + cc) * (kIn + 1) + i] =
        (part[0][cc][i] + part[1][cc][i]) + (part[2][cc][i] + part[3][cc][i]);
  }
}

// out_j = sum over chunks of P[ch][j], in chunk order.  With stride = 0 it
// goes to out_a[j]; with stride > 0 the partial rows hold groups of stride
// values (c, i): i < stride - 1 goes to out_a[c (stride - 1) + i] and the
// last of each group to out_b[c] (a weight block and its bias).
__global__ void k_sum_parts(const float* __restrict__ P, int n_ch, int n, int stride, float* out_a,
                            float* out_b) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float acc = 0.0f;
  int ch = 0;
  for (; ch + 8 <= n_ch; ch += 8) {  // eight loads in flight, added in order
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = P[(size_t)(ch + u) * n + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; ch < n_ch; ++ch) acc += P[(size_t)ch * n + j];
  if (stride > 0) {
    const int c = j / stride, i = j % stride;
    if (i < stride - 1)
      out_a[c * (stride - 1) + i] = acc;
    else
      out_b[c] = acc;
  } else {
    out_a[j] = acc;
  }
}

__global__ void k_adam(float* p, const float* __restrict__ g, float* m, float* v, int n, float lr,
                       float b1, float b2, float c1, float c2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_refresh(const float* __restrict__ p, WeightsB wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kW * kIn) wb.w1[i] = to_bf16(p[kOffW1 + i]);
  if (i < kW) wb.w5[i] = to_bf16(p[kOffW5 + i]);
  if (i < kW * kW) {
    const int o = i / kW, in = i % kW;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const uint16_t b = to_bf16(p[kOffW2 + l * kLayerStride + i]);
      wb.w[l][i] = b;
      wb.wt[l][in * kW + o] = b;
    }
  }
}

__global__ void __launch_bounds__(256) k_mean(const float* __restrict__ sq, int rows, int n,
                                              float* out) {
  __shared__ float part[256];
  float a = 0.0f;
  for (int i = threadIdx.x; i < rows; i += 256) a += sq[i];
  part[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0] / (float)n;
}

// Features of a query (Q, w), computed in FP64 and rounded to FP32:
//   0      2|Q|/q_max - 1
//   1..3   Q/|Q| (zero for Q = 0)
//   4      2w/w_max - 1
//   then for j < kNFreq: sin, cos of pi 2^(j/2) w / w_max,
//   then for j < kNFreq: sin, cos of pi 2^(j/2) |Q| / q_max,
//   then for each primitive vector a_i and h = 1, 2: sin, cos of h Q.a_i.
// The last twelve are periodic under Q -> Q + any reciprocal lattice vector,
// which is how the loss of a crystal depends on the part of Q inside the
// zone; the Fourier features give the first layer scales finer than the
// plain coordinates.
__global__ void k_encode(const double* __restrict__ qw, const double* __restrict__ loss, int n,
                         double qmax, double wmax, Lattice lat, double mu, double sigma, float* x,
                         float* t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double qx = qw[4 * i], qy = qw[4 * i + 1], qz = qw[4 * i + 2], w = qw[4 * i + 3];
  const double q = sqrt(qx * qx + qy * qy + qz * qz);
  const double inv = q > 0.0 ? 1.0 / q : 0.0;
  float* xi = x + (size_t)kIn * i;
  xi[0] = (float)(2.0 * q / qmax - 1.0);
  xi[1] = (float)(qx * inv);
  xi[2] = (float)(qy * inv);
  xi[3] = (float)(qz * inv);
  xi[4] = (float)(2.0 * w / wmax - 1.0);
  const double pi = 3.141592653589793;
  int c = 5;
#pragma unroll
  for (int j = 0; j < kNFreq; ++j) {
    const double f = pi * ((j & 1) ? 1.4142135623730951 : 1.0) * (double)(1 << (j >> 1));
    xi[c++] = (float)sin(f * w / wmax);
    xi[c++] = (float)cos(f * w / wmax);
  }
#pragma unroll
  for (int j = 0; j < kNFreq; ++j) {
    const double f = pi * ((j & 1) ? 1.4142135623730951 : 1.0) * (double)(1 << (j >> 1));
    xi[c++] = (float)sin(f * q / qmax);
    xi[c++] = (float)cos(f * q / qmax);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double ph = qx * lat.a[3 * a] + qy * lat.a[3 * a + 1] + qz * lat.a[3 * a + 2];
#pragma unroll
    for (int h = 1; h <= 2; ++h) {
      xi[c++] = (float)sin(h * ph);
      xi[c++] = (float)cos(h * ph);
    }
  }
  if (loss && t) t[i] = (float)((log(fmax(loss[i], 1e-30)) - mu) / sigma);
}

__global__ void k_decode(const float* __restrict__ ys, int K, int n, double mu, double sigma,
                         double calib, double* loss, double* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, s2 = 0.0;
  for (int k = 0; k < K; ++k) {
    const double v = ys[(size_t)k * n + i];
    s += v;
    s2 += v * v;
  }
  const double m = s / K;
  const double var = K > 1 ? fmax(0.0, (s2 - K * m * m) / (K - 1)) : 0.0;
  loss[i] = exp(mu + sigma * m);
  if (err) err[i] = calib * sigma * sqrt(var);
}

constexpr int SEL_BLOCK = 256;
__global__ void __launch_bounds__(SEL_BLOCK) k_select_count(const double* __restrict__ err, int n,
                                                            double tol, int* counts) {
  __shared__ int c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  const int i = blockIdx.x * SEL_BLOCK + threadIdx.x;
  const unsigned long long m = __ballot(i < n && err[i] > tol);
  if ((threadIdx.x & 63) == 0) atomicAdd(&c, __popcll(m));
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

// exclusive scan of the per-block counts in one block; total into *count
__global__ void __launch_bounds__(1024) k_select_scan(int* counts, int nb, int* count) {
  __shared__ int part[1024];
  const int per = (nb + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  int s = 0;
  for (int b = b0; b < b0 + per && b < nb; ++b) s += counts[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan
    const int v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;
  for (int b = b0; b < b0 + per && b < nb; ++b) {
    const int c = counts[b];
    counts[b] = run;
    run += c;
  }
  if (threadIdx.x == 1023) count[0] = part[1023];
}

__global__ void __launch_bounds__(SEL_BLOCK) k_select_write(const double* __restrict__ err, int n,
                                                            double tol,
                                                            const int* __restrict__ offsets,
                                                            int* idx) {
  __shared__ int wbase[SEL_BLOCK / 64];
  const int i = blockIdx.x * SEL_BLOCK + threadIdx.x;
  const bool hit = i < n && err[i] > tol;
  const unsigned long long m = __ballot(hit);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wbase[wave] = __popcll(m);
  __syncthreads();
  int base = offsets[blockIdx.x];
  for (int w = 0; w < wave; ++w) base += wbase[w];
  if (hit) {
    const unsigned long long below = lane ? (m & ((1ull << lane) - 1)) : 0ull;
    idx[base + __popcll(below)] = i;
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <int EPI>
static void gemm(const uint16_t* A, const uint16_t* B, int M, int N, int K, const EpiAll& e,
                 hipStream_t st, int ksplit = 1) {
  hipLaunchKernelGGL(k_gemm_nt<EPI>, dim3(N / 64, M / 64, ksplit), dim3(256), 0, st, A, B, M, N, K,
                     e);
}

void launch_gemm_fwd(const uint16_t* A, const uint16_t* B, int M, int N, int K, const EpiFwd& f,
                     hipStream_t st) {
  EpiAll e{};
  e.f = f;
  gemm<EPI_FWD>(A, B, M, N, K, e, st);
}
void launch_gemm_bwd(const uint16_t* A, const uint16_t* B, int M, int N, int K, const EpiBwd& b,
                     hipStream_t st) {
  EpiAll e{};
  e.b = b;
  gemm<EPI_BWD>(A, B, M, N, K, e, st);
}
int store_ksplit(int K) {
  int ks = 1;  // at least 8 K steps of 32 per split, K / ks a multiple of 32
  while (ks < 16 && K % (64 * ks) == 0 && K / (2 * ks) >= 256) ks *= 2;
  return ks;
}

void launch_gemm_store(const uint16_t* A, const uint16_t* B, int M, int N, int K, float* C,
                       float* P, hipStream_t st) {
  EpiAll e{};
  const int ks = store_ksplit(K);
  e.C = ks > 1 ? P : C;
  gemm<EPI_STORE>(A, B, M, N, K, e, st, ks);
  if (ks > 1)
    hipLaunchKernelGGL(k_sum_parts, dim3((M * N + 255) / 256), dim3(256), 0, st, P, ks, M * N, 0, C,
                       nullptr);
}

void launch_layer1(const float* x, const int* order, long off, int n, int rows_p,
                   const uint16_t* w1b, const float* b1, float* Z1, uint16_t* H1b, uint16_t* H1T,
                   int ldt, hipStream_t st) {
  hipLaunchKernelGGL(k_layer1, dim3(rows_p / L1_ROWS), dim3(kW), 0, st, x, order, off, n, w1b, b1,
                     Z1, H1b, H1T, ldt);
}

void launch_output(const uint16_t* H4b, const uint16_t* w5b, const float* b5, int n, int rows_p,
                   float* y, const float* t, const int* order, long off, float* dy, float* sq,
                   const float* Z4, float* dZ, uint16_t* dZb, uint16_t* dZbT, int ldt,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_output, dim3(rows_p / OUT_ROWS), dim3(kW), 0, st, H4b, w5b, b5, n, y, t,
                     order, off, dy, sq, Z4, dZ, dZb, dZbT, ldt);
}

int red_chunks(int rows) { return (rows + kRedRows - 1) / kRedRows; }

size_t red_floats(int rows) { return (size_t)red_chunks(rows) * kW * (kIn + 1); }

void launch_colsum(const float* A, int rows, int cols, float* out, float* P, hipStream_t st) {
  const int nch = red_chunks(rows);
  hipLaunchKernelGGL(k_colsum_part, dim3((cols + 63) / 64, nch), dim3(256), 0, st, A, rows, cols, P);
  hipLaunchKernelGGL(k_sum_parts, dim3((cols + 255) / 256), dim3(256), 0, st, P, nch, cols, 0, out,
                     nullptr);
}

void launch_out_grad(const uint16_t* H4b, const float* dy, int rows, float* dw5, float* db5,
                     float* P, hipStream_t st) {
  const int nch = red_chunks(rows);
  hipLaunchKernelGGL(k_out_grad_part, dim3(kW / 64, nch), dim3(256), 0, st, H4b, dy, rows, P);
  // dw5 (kW values) then db5: one row of kW + 1 per chunk, the last element to db5
  hipLaunchKernelGGL(k_sum_parts, dim3((kW + 1 + 255) / 256), dim3(256), 0, st, P, nch, kW + 1,
                     kW + 1, dw5, db5);
}

void launch_w1_grad(const float* dZ1, const float* x, const int* order, long off, int n,
                    float* dW1, float* db1, float* P, hipStream_t st) {
  const int nch = red_chunks(n);
  hipLaunchKernelGGL(k_w1_grad_part, dim3(kW / 64, nch), dim3(256), 0, st, dZ1, x, order, off, n, P);
  const int tot = kW * (kIn + 1);
  hipLaunchKernelGGL(k_sum_parts, dim3((tot + 255) / 256), dim3(256), 0, st, P, nch, tot, kIn + 1,
                     dW1, db1);
}

void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float beta1,
                 float beta2, float c1, float c2, float eps, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m, v, n, lr, beta1,
                     beta2, c1, c2, eps);
}

void launch_refresh(const float* p, const WeightsB& wb, hipStream_t st) {
  hipLaunchKernelGGL(k_refresh, dim3(kW * kW / 256), dim3(256), 0, st, p, wb);
}

void launch_mean(const float* sq, int rows, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, st, sq, rows, n, out);
}

void launch_encode(const double* qw, const double* loss, int n, double qmax, double wmax,
                   const Lattice& lat, double mu, double sigma, float* x, float* t,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_encode, dim3((n + 255) / 256), dim3(256), 0, st, qw, loss, n, qmax, wmax,
                     lat, mu, sigma, x, t);
}

void launch_decode(const float* ys, int K, int n, double mu, double sigma, double calib,
                   double* loss, double* err, hipStream_t st) {
  hipLaunchKernelGGL(k_decode, dim3((n + 255) / 256), dim3(256), 0, st, ys, K, n, mu, sigma,
                     calib, loss, err);
}

int select_blocks(int n) { return (n + SEL_BLOCK - 1) / SEL_BLOCK; }

void launch_select(const double* err, int n, double tol, int* block_counts, int n_blocks, int* idx,
                   int* count, hipStream_t st) {
  hipLaunchKernelGGL(k_select_count, dim3(n_blocks), dim3(SEL_BLOCK), 0, st, err, n, tol,
                     block_counts);
  hipLaunchKernelGGL(k_select_scan, dim3(1), dim3(1024), 0, st, block_counts, n_blocks, count);
  hipLaunchKernelGGL(k_select_write, dim3(n_blocks), dim3(SEL_BLOCK), 0, st, err, n, tol,
                     block_counts, idx);
}

}  // namespace mlp
}  // namespace qcx
