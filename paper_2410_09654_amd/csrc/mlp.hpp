// Kernels of the b_n continuation network: 16 -> 256 -> 256 -> 16 with GELU,
// BF16 operands on the MFMA units (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation, FP32 master weights and Adam.
//
// Matrix-core lane layout (wave64) of v_mfma_f32_16x16x32_bf16, A 16x32,
// B 32x16, D 16x16 fp32:
//   A: lane l holds row l%16, k = 8*(l/16) .. 8*(l/16)+7
//   B: lane l holds column l%16, k = 8*(l/16) .. 8*(l/16)+7
//   D: lane l holds column l%16, rows 4*(l/16) .. 4*(l/16)+3
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pauli {
namespace mlp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int NIN = 16, NHID = 256, NOUT = 16;
constexpr int64_t NPARAM = NHID * NIN + NHID + NHID * NHID + NHID + NOUT * NHID + NOUT;
// offsets in the flat parameter vector
constexpr int64_t OFF_W1 = 0, OFF_B1 = OFF_W1 + NHID * NIN;
constexpr int64_t OFF_W2 = OFF_B1 + NHID, OFF_B2 = OFF_W2 + NHID * NHID;
constexpr int64_t OFF_W3 = OFF_B2 + NHID, OFF_B3 = OFF_W3 + NOUT * NHID;

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2 and its derivative
// Phi(x) + x phi(x).
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
  return cdf + x * pdf;
}

enum Epilogue : int { EP_STORE = 0, EP_BIAS = 1, EP_BIAS_GELU = 2 };

struct GemmArgs {
  const uint16_t* A;  // A(m,k) = transA ? A[k*lda + m] : A[m*lda + k]
  const uint16_t* B;  // B(k,n) = transB ? B[n*ldb + k] : B[k*ldb + n]
  float* C;           // C[m*ldc + n]
  uint16_t* Cb;       // bf16 of GELU(C) (EP_BIAS_GELU) or nullptr
  const float* bias;  // [n]
  int lda, ldb, ldc;
  int transA, transB;
  int M, N, K;        // M, N multiples of 16; k >= K reads as zero
  int epilogue;
};

// One 64-thread wave per 16x16 output tile, four waves per 32x32 block tile.
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 32 + (wv >> 1) * 16;
  const int n0 = blockIdx.x * 32 + (wv & 1) * 16;
  if (m0 >= g.M || n0 >= g.N) return;
  const int r = lane & 15, kq = (lane >> 4) * 8;
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int q = 0; q < 8; q++) {
      const int k = k0 + kq + q;
      uint16_t av = 0, bv = 0;
      if (k < g.K) {
        av = g.transA ? g.A[(size_t)k * g.lda + (m0 + r)] : g.A[(size_t)(m0 + r) * g.lda + k];
        bv = g.transB ? g.B[(size_t)(n0 + r) * g.ldb + k] : g.B[(size_t)k * g.ldb + (n0 + r)];
      }
      a[q] = __builtin_bit_cast(__bf16, av);
      b[q] = __builtin_bit_cast(__bf16, bv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  const int n = n0 + r;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int m = m0 + (lane >> 4) * 4 + q;
    float v = acc[q];
    if (g.epilogue != EP_STORE) v = v + g.bias[n];
    g.C[(size_t)m * g.ldc + n] = v;
    if (g.epilogue == EP_BIAS_GELU) g.Cb[(size_t)m * g.ldc + n] = f2bf(gelu(v));
  }
}

__global__ void k_bf_to_f(const uint16_t* x, float* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = bf2f(x[i]);
}

__global__ void k_to_bf16(const float* x, uint16_t* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// Masked mean-squared error: per-row partial sums of mask*(y-t)^2 and of the
// mask (fixed order), and dL/dy = 2 mask (y - t) / sum(mask) rounded to bf16.
__global__ void k_mse_rows(const float* y, const float* t, const float* mask, int64_t rows,
                           double* row_err, double* row_cnt) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= rows) return;
  double e = 0.0, c = 0.0;
  for (int j = 0; j < NOUT; j++) {
    const double m = mask[b * NOUT + j];
    const double d = (double)y[b * NOUT + j] - (double)t[b * NOUT + j];
    e += m * d * d;
    c += m;
  }
  row_err[b] = e;
  row_cnt[b] = c;
}

__global__ void k_sum_rows(const double* row_err, const double* row_cnt, int64_t rows,
                           double* out) {
  __shared__ double se[256], sc[256];
  const int t = threadIdx.x;
  double e = 0.0, c = 0.0;
  for (int64_t b = t; b < rows; b += 256) {
    e += row_err[b];
    c += row_cnt[b];
  }
  se[t] = e;
  sc[t] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      se[t] += se[t + s];
      sc[t] += sc[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = sc[0] > 0 ? se[0] / sc[0] : 0.0;
    out[1] = sc[0];
  }
}

__global__ void k_mse_grad(const float* y, const float* t, const float* mask, int64_t n,
                           const double* loss_cnt, float* dy, uint16_t* dyb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double cnt = loss_cnt[1];
  const float g = cnt > 0 ? (float)(2.0 * (double)mask[i] * ((double)y[i] - (double)t[i]) / cnt) : 0.f;
  dy[i] = g;
  dyb[i] = f2bf(g);
}

// dZ = dY * GELU'(Z), in fp32 and bf16.
__global__ void k_gelu_back(const float* dy, const float* z, int64_t n, float* dz, uint16_t* dzb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = dy[i] * gelu_grad(z[i]);
  dz[i] = g;
  dzb[i] = f2bf(g);
}

// Bias gradient: column sums of d[rows][cols] in a fixed order (one thread
// per column, rows in ascending order).
__global__ void k_col_sum(const float* d, int64_t rows, int cols, float* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int64_t b = 0; b < rows; b++) s += d[b * cols + c];
  out[c] = s;
}

// Adam on the flat fp32 parameter vector; refreshes the bf16 copy.  The
// complements 1-b1 and 1-b2 come from the host in double precision: formed
// in float from a rounded b2 = 0.999 they would be off by 1.3e-5 relative.
__global__ void k_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, int64_t n,
                       float lr, float b1, float omb1, float b2, float omb2, float eps, float c1,
                       float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  const float pi = p[i] - lr * mh / (sqrtf(vh) + eps);
  p[i] = pi;
  pb[i] = f2bf(pi);
}

}  // namespace mlp
}  // namespace pauli
