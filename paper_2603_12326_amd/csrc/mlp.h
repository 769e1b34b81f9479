// Internal declarations of the surrogate network kernels (k_mlp.hip).
//
// Network 49 -> 256 -> 256 -> 256 -> 256 -> 1, SiLU after every hidden layer.
// Flat FP32 parameter vector: per layer W[n_out][n_in] row-major, then b.
// The 49 inputs are the features of a query (Q, w) formed by k_encode.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qcx {
namespace mlp {

constexpr int kNFreq = 8;                     // Fourier frequencies per scalar
constexpr int kIn = 5 + 4 * kNFreq + 12;       // 49 features
constexpr int kW = 256;
constexpr int kHidden = 4;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kW * kIn;
constexpr int kOffW2 = kOffB1 + kW;
constexpr int kLayerStride = kW * kW + kW;  // W_l then b_l for l = 2..4
constexpr int kOffW5 = kOffW2 + 3 * kLayerStride;
constexpr int kOffB5 = kOffW5 + kW;
constexpr int kNParam = kOffB5 + 1;         // 210433
constexpr int kRowTile = 64;                // rows are padded to this
constexpr int kRedRows = 64;                // rows per block of the gradient reductions

inline int off_w(int l) { return kOffW2 + (l - 2) * kLayerStride; }  // l = 2..4
inline int off_b(int l) { return off_w(l) + kW * kW; }

// bf16 copies of the weights used by the kernels (refreshed after updates)
struct WeightsB {
  uint16_t* w1;       // [256][kIn]
  uint16_t* w[3];     // layers 2..4, [out][in]
  uint16_t* wt[3];    // layers 2..4, [in][out]
  uint16_t* w5;       // [256]
};

// Epilogue variants of the bf16 NT GEMM C[M][N] = sum_k A[m][k] B[n][k].
struct EpiFwd {       // z = acc + bias; Z (optional) = z; Hb = bf16(silu z); HT (optional)
  const float* bias;
  float* Z;
  uint16_t* Hb;
  uint16_t* HT;
  int ldt;            // row length of HT (padded batch)
};
struct EpiBwd {       // dz = acc * silu'(Zprev); dZ (FP32), dZb, dZbT
  const float* Zprev;
  float* dZ;
  uint16_t* dZb;
  uint16_t* dZbT;
  int ldt;
};

void launch_gemm_fwd(const uint16_t* A, const uint16_t* B, int M, int N, int K, const EpiFwd& e,
                     hipStream_t st);
void launch_gemm_bwd(const uint16_t* A, const uint16_t* B, int M, int N, int K, const EpiBwd& e,
                     hipStream_t st);
// C = A B^T in FP32; K is split over up to 16 blocks per output tile when
// long (partials in P, store_ksplit(K) * M * N floats, added in split order)
int store_ksplit(int K);
void launch_gemm_store(const uint16_t* A, const uint16_t* B, int M, int N, int K, float* C,
                       float* P, hipStream_t st);

// first layer: rows r < n read x[idx(r)] (idx = order[off + r] or r), rows
// n..rows_p-1 read zeros
void launch_layer1(const float* x, const int* order, long off, int n, int rows_p,
                   const uint16_t* w1b, const float* b1, float* Z1, uint16_t* H1b, uint16_t* H1T,
                   int ldt, hipStream_t st);
// output layer: y = bf16(h4) . w5b + b5.  With t != NULL (training) also
// dy = 2 (y - t) / n_true (0 on padded rows), sq[r] = (y - t)^2, and the
// layer-4 backward dz4 = dy w5b silu'(Z4) into dZ / dZb / dZbT.
void launch_output(const uint16_t* H4b, const uint16_t* w5b, const float* b5, int n, int rows_p,
                   float* y, const float* t, const int* order, long off, float* dy, float* sq,
                   const float* Z4, float* dZ, uint16_t* dZb, uint16_t* dZbT, int ldt,
                   hipStream_t st);
// The gradient reductions below sum over rows in chunks of kRedRows (one
// block each) into a partial buffer P of red_floats(rows) floats, then add
// the chunks in order: deterministic, and spread over many blocks.
int red_chunks(int rows);
size_t red_floats(int rows);
// out[j] = sum_r A[r][j] for j < cols <= kW (FP32 A)
void launch_colsum(const float* A, int rows, int cols, float* out, float* P, hipStream_t st);
// dw5[j] = sum_r dy[r] bf16(h4)[r][j]; db5 = sum_r dy[r]
void launch_out_grad(const uint16_t* H4b, const float* dy, int rows, float* dw5, float* db5,
                     float* P, hipStream_t st);
// dW1[j][c] = sum_r dz1[r][j] x[idx(r)][c]; db1[j] = sum_r dz1[r][j]
void launch_w1_grad(const float* dZ1, const float* x, const int* order, long off, int n,
                    float* dW1, float* db1, float* P, hipStream_t st);
void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float beta1,
                 float beta2, float c1, float c2, float eps, hipStream_t st);
void launch_refresh(const float* p, const WeightsB& wb, hipStream_t st);
// sum of sq[0..rows) / n into *out
void launch_mean(const float* sq, int rows, int n, float* out, hipStream_t st);

// surrogate I/O: the kIn features of (Q, w) (see k_encode) and the
// standardised target t = (log max(L, 1e-30) - mu) / sigma
struct Lattice {
  double a[9];  // primitive vectors a_i = (a[3i], a[3i+1], a[3i+2]), bohr
};
void launch_encode(const double* qw, const double* loss, int n, double qmax, double wmax,
                   const Lattice& lat, double mu, double sigma, float* x, float* t,
                   hipStream_t st);
// ensemble of K outputs ys[k][n] -> loss = exp(mu + sigma mean), err = calib sigma sd
void launch_decode(const float* ys, int K, int n, double mu, double sigma, double calib,
                   double* loss, double* err, hipStream_t st);
// indices i with err[i] > tol, ascending, count in *count (device int)
void launch_select(const double* err, int n, double tol, int* block_counts, int n_blocks,
                   int* idx, int* count, hipStream_t st);
int select_blocks(int n);

}  // namespace mlp
}  // namespace qcx
