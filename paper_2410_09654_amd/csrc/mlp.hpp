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

// ---------------------------------------------------------------------------
// Fused training step.  One block of 256 threads (four waves) takes SR rows
// of the minibatch (row i of the minibatch is row order[i] of the training
// set): forward, masked MSE and backward with every activation in LDS and
// every matrix product on the matrix cores (the same BF16 operands, FP32
// accumulation and epilogues as the layer-by-layer kernels above), then
// writes its rows' share of every parameter gradient to part[block][NPARAM]
// and of the loss to lpart[block] (sum mask (y - t)^2 and the minibatch's
// sum of mask).  k_mlp_reduce_adam sums the shares in block order and takes
// the Adam step.  Rows beyond the minibatch are zero with zero mask, so they
// contribute nothing.
// ---------------------------------------------------------------------------
constexpr int SR = 32;  // minibatch rows per block

struct StepArgs {
  const float* params;   // fp32 master weights (biases)
  const uint16_t* pb;    // bf16 weights
  const float* X;        // [n][16] training inputs
  const float* T;        // [n][16] targets
  const float* Mk;       // [n][16] target mask
  const int32_t* order;  // the minibatch's rows, `rows` entries
  int rows;
  float* part;           // [gridDim.x][NPARAM]
  double* lpart;         // [gridDim.x][2]
};

__device__ __forceinline__ bf16x8 bf8_lds(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}
__device__ __forceinline__ bf16x8 bf8_zero() {
  bf16x8 v;
#pragma unroll
  for (int q = 0; q < 8; q++) v[q] = __builtin_bit_cast(__bf16, (uint16_t)0);
  return v;
}
// 8 bf16 values p[0], p[stride], ..., p[7 stride]
__device__ __forceinline__ bf16x8 bf8_strided(const uint16_t* p, int stride) {
  bf16x8 v;
#pragma unroll
  for (int q = 0; q < 8; q++) v[q] = __builtin_bit_cast(__bf16, p[q * stride]);
  return v;
}
__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(256) void k_mlp_step(StepArgs a) {
  __shared__ __align__(16) uint16_t xb[SR][NIN];
  __shared__ __align__(16) float z1[SR][NHID];      // Z1, then dZ1
  __shared__ __align__(16) uint16_t y1b[SR][NHID];  // bf16 GELU(Z1), then bf16 dZ1
  __shared__ __align__(16) float z2[SR][NHID];      // Z2, then dZ2
  __shared__ __align__(16) uint16_t y2b[SR][NHID];  // bf16 GELU(Z2), then bf16 dZ2
  __shared__ float yv[SR][NOUT];                    // Y, then dY
  __shared__ __align__(16) uint16_t dyb[SR][NOUT];
  __shared__ int32_t rid[SR];
  __shared__ double dred[256];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, kq = (lane >> 4) * 8, rq = (lane >> 4) * 4;
  const int row0 = blockIdx.x * SR;
  const uint16_t* W1 = a.pb + OFF_W1;
  const uint16_t* W2 = a.pb + OFF_W2;
  const uint16_t* W3 = a.pb + OFF_W3;
  const float* B1 = a.params + OFF_B1;
  const float* B2 = a.params + OFF_B2;
  const float* B3 = a.params + OFF_B3;
  float* G = a.part + (size_t)blockIdx.x * NPARAM;

  // rows of this block and the minibatch's mask count (every block sums the
  // same values in the same order)
  if (tid < SR) rid[tid] = row0 + tid < a.rows ? a.order[row0 + tid] : -1;
  double c = 0.0;
  for (int e = tid; e < a.rows * NOUT; e += 256) c += (double)a.Mk[(size_t)a.order[e / NOUT] * NOUT + e % NOUT];
  dred[tid] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) dred[tid] += dred[tid + s];
    __syncthreads();
  }
  const double cnt = dred[0];
  for (int e = tid; e < SR * NIN; e += 256) {
    const int rr = e / NIN, j = e % NIN;
    xb[rr][j] = rid[rr] >= 0 ? f2bf(a.X[(size_t)rid[rr] * NIN + j]) : (uint16_t)0;
  }
  __syncthreads();

  // Z1 = Xb W1^T + b1 (K = 16: lanes of k >= 16 supply zeros), Y1 = GELU(Z1)
  for (int tt = wv; tt < 2 * (NHID / 16); tt += 4) {
    const int mt = tt / (NHID / 16), n = (tt % (NHID / 16)) * 16 + r;
    const bf16x8 av = kq < NIN ? bf8_lds(&xb[mt * 16 + r][kq]) : bf8_zero();
    const bf16x8 bv = kq < NIN ? *reinterpret_cast<const bf16x8*>(W1 + n * NIN + kq) : bf8_zero();
    const floatx4 acc = mfma(av, bv, floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const float v = acc[q] + B1[n];
      z1[mt * 16 + rq + q][n] = v;
      y1b[mt * 16 + rq + q][n] = f2bf(gelu(v));
    }
  }
  __syncthreads();
  // Z2 = Y1b W2^T + b2, Y2 = GELU(Z2)
  for (int tt = wv; tt < 2 * (NHID / 16); tt += 4) {
    const int mt = tt / (NHID / 16), n = (tt % (NHID / 16)) * 16 + r;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < NHID; k0 += 32)
      acc = mfma(bf8_lds(&y1b[mt * 16 + r][k0 + kq]),
                 *reinterpret_cast<const bf16x8*>(W2 + n * NHID + k0 + kq), acc);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const float v = acc[q] + B2[n];
      z2[mt * 16 + rq + q][n] = v;
      y2b[mt * 16 + rq + q][n] = f2bf(gelu(v));
    }
  }
  __syncthreads();
  // Y = Y2b W3^T + b3
  if (wv < 2) {
    const int mt = wv, n = r;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < NHID; k0 += 32)
      acc = mfma(bf8_lds(&y2b[mt * 16 + r][k0 + kq]),
                 *reinterpret_cast<const bf16x8*>(W3 + n * NHID + k0 + kq), acc);
#pragma unroll
    for (int q = 0; q < 4; q++) yv[mt * 16 + rq + q][n] = acc[q] + B3[n];
  }
  __syncthreads();
  // masked MSE share and dY = 2 mask (y - t) / sum(mask)
  double err = 0.0;
  for (int e = tid; e < SR * NOUT; e += 256) {
    const int rr = e / NOUT, j = e % NOUT;
    float g = 0.f;
    if (rid[rr] >= 0) {
      const size_t o = (size_t)rid[rr] * NOUT + j;
      const double m = a.Mk[o];
      const double d = (double)yv[rr][j] - (double)a.T[o];
      err += m * d * d;
      g = cnt > 0 ? (float)(2.0 * m * d / cnt) : 0.f;
    }
    yv[rr][j] = g;
    dyb[rr][j] = f2bf(g);
  }
  dred[tid] = err;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) dred[tid] += dred[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    a.lpart[2 * blockIdx.x] = dred[0];
    a.lpart[2 * blockIdx.x + 1] = cnt;
  }
  // db3 (fixed row order) and dW3 = dYb^T Y2b (M = 16, N = 256, K = SR)
  if (tid < NOUT) {
    float sm = 0.f;
    for (int rr = 0; rr < SR; rr++) sm += yv[rr][tid];
    G[OFF_B3 + tid] = sm;
  }
  for (int nt = wv; nt < NHID / 16; nt += 4) {
    const int n = nt * 16 + r;
    const floatx4 acc = mfma(bf8_strided(&dyb[kq][r], NOUT), bf8_strided(&y2b[kq][n], NHID),
                             floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int q = 0; q < 4; q++) G[OFF_W3 + (size_t)(rq + q) * NHID + n] = acc[q];
  }
  __syncthreads();
  // dY2 = dYb W3 (K = 16), dZ2 = dY2 GELU'(Z2) over Z2, bf16 copy over Y2b
  for (int tt = wv; tt < 2 * (NHID / 16); tt += 4) {
    const int mt = tt / (NHID / 16), n = (tt % (NHID / 16)) * 16 + r;
    const bf16x8 av = kq < NOUT ? bf8_lds(&dyb[mt * 16 + r][kq]) : bf8_zero();
    const bf16x8 bv = kq < NOUT ? bf8_strided(W3 + (size_t)kq * NHID + n, NHID) : bf8_zero();
    const floatx4 acc = mfma(av, bv, floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int rr = mt * 16 + rq + q;
      const float g = acc[q] * gelu_grad(z2[rr][n]);
      z2[rr][n] = g;
      y2b[rr][n] = f2bf(g);
    }
  }
  __syncthreads();
  // db2 and dW2 = dZ2b^T Y1b (M = N = 256, K = SR)
  {
    float sm = 0.f;
    for (int rr = 0; rr < SR; rr++) sm += z2[rr][tid];
    G[OFF_B2 + tid] = sm;
  }
  for (int tt = wv; tt < (NHID / 16) * (NHID / 16); tt += 4) {
    const int m0 = (tt / (NHID / 16)) * 16, n = (tt % (NHID / 16)) * 16 + r;
    const floatx4 acc = mfma(bf8_strided(&y2b[kq][m0 + r], NHID), bf8_strided(&y1b[kq][n], NHID),
                             floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int q = 0; q < 4; q++) G[OFF_W2 + (size_t)(m0 + rq + q) * NHID + n] = acc[q];
  }
  __syncthreads();
  // dY1 = dZ2b W2, dZ1 = dY1 GELU'(Z1) over Z1, bf16 copy over Y1b
  for (int tt = wv; tt < 2 * (NHID / 16); tt += 4) {
    const int mt = tt / (NHID / 16), n = (tt % (NHID / 16)) * 16 + r;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < NHID; k0 += 32)
      acc = mfma(bf8_lds(&y2b[mt * 16 + r][k0 + kq]),
                 bf8_strided(W2 + (size_t)(k0 + kq) * NHID + n, NHID), acc);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int rr = mt * 16 + rq + q;
      const float g = acc[q] * gelu_grad(z1[rr][n]);
      z1[rr][n] = g;
      y1b[rr][n] = f2bf(g);
    }
  }
  __syncthreads();
  // db1 and dW1 = dZ1b^T Xb (M = 256, N = 16, K = SR)
  {
    float sm = 0.f;
    for (int rr = 0; rr < SR; rr++) sm += z1[rr][tid];
    G[OFF_B1 + tid] = sm;
  }
  for (int mt = wv; mt < NHID / 16; mt += 4) {
    const floatx4 acc = mfma(bf8_strided(&y1b[kq][mt * 16 + r], NHID), bf8_strided(&xb[kq][r], NIN),
                             floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int q = 0; q < 4; q++) G[OFF_W1 + (size_t)(mt * 16 + rq + q) * NIN + r] = acc[q];
  }
}

// Gradient = the blocks' shares summed in block order; Adam step; the
// minibatch loss (sum of the shares over the mask count) into *loss.
__global__ void k_mlp_reduce_adam(const float* part, int nblk, float* grads, float* p, float* m,
                                  float* v, uint16_t* pb, float lr, float b1, float omb1, float b2,
                                  float omb2, float eps, float c1, float c2, const double* lpart,
                                  double* loss) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    double e = 0.0;
    for (int b = 0; b < nblk; b++) e += lpart[2 * b];
    const double cnt = lpart[1];
    *loss = cnt > 0 ? e / cnt : 0.0;
  }
  if (i >= NPARAM) return;
  float gi = 0.f;
  for (int b = 0; b < nblk; b++) gi += part[(size_t)b * NPARAM + i];
  grads[i] = gi;
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
