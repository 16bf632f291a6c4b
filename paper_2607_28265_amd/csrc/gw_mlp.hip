// Likelihood prescreen network 11 -> 256 -> 256 -> 256 -> 1 with exact GELU.
//
// Training (forward, backward, Adam) runs in FP32 on the vector ALUs through
// one LDS-tiled GEMM kernel (64 x 64 tiles, 4 x 4 outputs per thread, split-K
// with a fixed-order reduction for the weight gradients) and elementwise
// kernels; the FP32 master weights live on the device.  Inference runs the
// hidden layers on the matrix cores: BF16 weights (round-to-nearest-even,
// stored transposed so that one lane's K-run is contiguous) and BF16
// activations feed v_mfma_f32_16x16x16_bf16 with FP32 accumulation; bias and
// GELU are applied in FP32 between layers, and the 256 -> 1 output layer is an
// FP32 dot product reduced by shuffles and a fixed-order LDS combine.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "gw_ctx.h"

namespace gw {

constexpr int kIn = 11;
constexpr int kH = 256;
constexpr int kInPad = 32;  // K of the first layer padded for the MFMA K-step of 16
constexpr int64_t OW1 = 0;
constexpr int64_t OB1 = OW1 + kIn * kH;
constexpr int64_t OW2 = OB1 + kH;
constexpr int64_t OB2 = OW2 + kH * kH;
constexpr int64_t OW3 = OB2 + kH;
constexpr int64_t OB3 = OW3 + kH * kH;
constexpr int64_t OW4 = OB3 + kH;
constexpr int64_t OB4 = OW4 + kH;
constexpr int64_t kNPar = OB4 + 1;
// BF16 copies, transposed [out][in]: layer 1 [256][32], layers 2, 3 [256][256]
constexpr int64_t QW1 = 0;
constexpr int64_t QW2 = QW1 + kH * kInPad;
constexpr int64_t QW3 = QW2 + kH * kH;
constexpr int64_t kNQ = QW3 + kH * kH;

struct MlpScale {
  float xm[kIn];
  float xs_inv[kIn];
  double ym, ys;
};

// ---------------------------------------------------------------------------
// FP32 pieces (training and the reference forward)

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ inline float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__global__ void k_mlp_stdin(const double* __restrict__ x, int64_t n, MlpScale sc, float* __restrict__ xs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * kIn) return;
  const int j = (int)(i % kIn);
  xs[i] = ((float)x[i] - sc.xm[j]) * sc.xs_inv[j];
}

// C[z] = op(A) op(B) over the K range of split z (+ bias when z is the only
// split); op(A)(i, k) = TA ? A[k lda + i] : A[i lda + k], likewise for B.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, int k_per, const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                              int64_t c_split_stride, const float* __restrict__ bias) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int kb = blockIdx.z * k_per;
  const int ke = kb + k_per < K ? kb + k_per : K;
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      int ii, kk;
      if (TA) {
        kk = e >> 6;
        ii = e & 63;
      } else {
        ii = e >> 4;
        kk = e & 15;
      }
      const int gi = i0 + ii, gk = k0 + kk;
      float v = 0.0f;
      if (gi < M && gk < ke) v = TA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
      As[kk][ii] = v;
    }
    for (int e = threadIdx.x; e < 1024; e += 256) {
      int jj, kk;
      if (TB) {
        jj = e >> 4;
        kk = e & 15;
      } else {
        kk = e >> 6;
        jj = e & 63;
      }
      const int gj = j0 + jj, gk = k0 + kk;
      float v = 0.0f;
      if (gj < N && gk < ke) v = TB ? B[(int64_t)gj * ldb + gk] : B[(int64_t)gk * ldb + gj];
      Bs[kk][jj] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
    }
    __syncthreads();
  }
  float* Cz = C + (int64_t)blockIdx.z * c_split_stride;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + ty * 4 + r;
    if (i >= M) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + tx * 4 + c;
      if (j < N) Cz[(int64_t)i * ldc + j] = acc[r][c] + (bias ? bias[j] : 0.0f);
    }
  }
}

// out[e] = sum_z part[z][e] in split order.
__global__ void k_sum_splits(const float* __restrict__ part, int splits, int64_t count, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  float s = 0.0f;
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * count + e];
  out[e] = s;
}

__global__ void k_gelu_fwd(const float* __restrict__ z, float* __restrict__ a, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) a[e] = gelu_f(z[e]);
}

__global__ void k_gelu_bwd(float* __restrict__ d, const float* __restrict__ z, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) d[e] *= gelu_grad_f(z[e]);
}

// Loss 1/n sum (y - t)^2 on standardised targets and dy = 2 (y - t) / n; one
// workgroup, fixed-order tree for the loss.
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ y, const double* __restrict__ target,
                                             int64_t n, MlpScale sc, float* __restrict__ dy,
                                             float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.0f;
  const double iys = 1.0 / sc.ys;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const float t = (float)((target[i] - sc.ym) * iys);
    const float r = y[i] - t;
    dy[i] = 2.0f * r / (float)n;
    s += r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (float)n;
}

// db[j] = sum_i d[i][j]: workgroup = 64 columns x 4 waves; wave w sums rows
// i = w mod 4 in four interleaved partial sums (i mod 16), the 16 partials
// are added in a fixed order.
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ d, int64_t rows, int cols,
                                               float* __restrict__ db) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
  if (j < cols) {
    int64_t i = w;
    for (; i + 12 < rows; i += 16) {
      a0 += d[i * cols + j];
      a1 += d[(i + 4) * cols + j];
      a2 += d[(i + 8) * cols + j];
      a3 += d[(i + 12) * cols + j];
    }
    for (; i < rows; i += 4) a0 += d[i * cols + j];
  }
  red[w][lane] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (w == 0 && j < cols) db[j] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t count, float lr, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const float gg = g[e];
  const float mm = 0.9f * m[e] + 0.1f * gg;
  const float vv = 0.999f * v[e] + 0.001f * gg * gg;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
}

__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// BF16 transposed copies of W1 (K padded to 32 with zeros), W2, W3.
__global__ void k_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ q) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNQ) return;
  if (e < QW2) {
    const int o = (int)(e / kInPad), k = (int)(e % kInPad);
    q[e] = k < kIn ? to_bf16(p[OW1 + (int64_t)k * kH + o]) : 0;
  } else {
    const int64_t base = e < QW3 ? OW2 : OW3;
    const int64_t r = e - (e < QW3 ? QW2 : QW3);
    const int o = (int)(r / kH), k = (int)(r % kH);
    q[e] = to_bf16(p[base + (int64_t)k * kH + o]);
  }
}

// ---------------------------------------------------------------------------
// BF16 MFMA inference: one workgroup (8 waves) per 128 rows.  Each layer is
// computed transposed, out^T [feature][row] = W [feature][k] act^T [k][row],
// with the 16x16x32 BF16 matrix instruction (FP32 accumulation): operand A is
// a 16-feature x 32-k tile of the weights (read from memory, one k-step
// ahead), operand B a 32-k x 16-row tile of the activations (LDS, rows of
// kActStride bf16 so that the 16 rows of a read fall in distinct banks); a
// lane's 4 results are 4 consecutive features of one row, stored as one
// 8-byte write.  Wave w owns features 64 (w mod 4) .. + 63 of rows
// 64 (w / 4) .. + 63: 4 feature tiles x 4 row tiles.

typedef short s8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kInferRows = 128;
constexpr int kActStride = kH + 8;  // bf16 per activation row in LDS

__device__ inline f4v mfma_bf16_16x16x32(s8v a, s8v b, f4v c) {
  typedef __bf16 b8v __attribute__((ext_vector_type(8)));
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8v, a), __builtin_bit_cast(b8v, b), c, 0, 0,
                                                 0);
}

__global__ void __launch_bounds__(512) k_mlp_infer(const double* __restrict__ x, int64_t n, MlpScale sc,
                                                   const uint16_t* __restrict__ q, const float* __restrict__ p,
                                                   double* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint16_t act[kInferRows * kActStride];  // [row][k]
  __shared__ float red[4][kInferRows];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int fw = wave & 3, rw = wave >> 2;  // feature block, row half
  const int64_t r0 = (int64_t)blockIdx.x * kInferRows;
  // standardised input, K padded to 32
  for (int e = threadIdx.x; e < kInferRows * kInPad; e += 512) {
    const int row = e / kInPad, k = e % kInPad;
    float v = 0.0f;
    if (k < kIn && r0 + row < n) v = ((float)x[(r0 + row) * kIn + k] - sc.xm[k]) * sc.xs_inv[k];
    act[row * kActStride + k] = to_bf16(v);
  }
  __syncthreads();
  const int l16 = lane & 15;        // feature (A) / row (B) within a tile
  const int lk = (lane >> 4) * 8;   // this lane's 8 values of the 32-k step
  const int lf = (lane >> 4) * 4;   // first of this lane's 4 output features in a tile
  f4v acc[4][4];                    // [feature tile][row tile]
  for (int layer = 0; layer < 3; ++layer) {
    const int K = layer == 0 ? kInPad : kH;
    const uint16_t* __restrict__ W = q + (layer == 0 ? QW1 : (layer == 1 ? QW2 : QW3));
    const float* __restrict__ bias = p + (layer == 0 ? OB1 : (layer == 1 ? OB2 : OB3));
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) acc[ft][rt] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
    const uint16_t* __restrict__ wrow = W + (int64_t)(fw * 64 + l16) * K + lk;
    s8v a_cur[4], a_nxt[4];
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) a_cur[ft] = *(const s8v*)(wrow + (int64_t)ft * 16 * K);
    for (int k0 = 0; k0 < K; k0 += 32) {
      if (k0 + 32 < K) {
#pragma unroll
        for (int ft = 0; ft < 4; ++ft) a_nxt[ft] = *(const s8v*)(wrow + (int64_t)ft * 16 * K + k0 + 32);
      }
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        const s8v b = *(const s8v*)&act[(rw * 64 + rt * 16 + l16) * kActStride + k0 + lk];
#pragma unroll
        for (int ft = 0; ft < 4; ++ft) acc[ft][rt] = mfma_bf16_16x16x32(a_cur[ft], b, acc[ft][rt]);
      }
      if (k0 + 32 < K) {
#pragma unroll
        for (int ft = 0; ft < 4; ++ft) a_cur[ft] = a_nxt[ft];
      }
    }
    // bias + GELU in FP32; D[feature = lf + j][row = l16] per tile
#pragma unroll
    for (int ft = 0; ft < 4; ++ft) {
      const float4 bc = *(const float4*)&bias[fw * 64 + ft * 16 + lf];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        acc[ft][rt][0] = gelu_f(acc[ft][rt][0] + bc.x);
        acc[ft][rt][1] = gelu_f(acc[ft][rt][1] + bc.y);
        acc[ft][rt][2] = gelu_f(acc[ft][rt][2] + bc.z);
        acc[ft][rt][3] = gelu_f(acc[ft][rt][3] + bc.w);
      }
    }
    __syncthreads();  // every wave has read this layer's input
    if (layer < 2) {
#pragma unroll
      for (int ft = 0; ft < 4; ++ft)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
          const uint32_t lo = (uint32_t)to_bf16(acc[ft][rt][0]) | ((uint32_t)to_bf16(acc[ft][rt][1]) << 16);
          const uint32_t hi = (uint32_t)to_bf16(acc[ft][rt][2]) | ((uint32_t)to_bf16(acc[ft][rt][3]) << 16);
          *(uint2*)&act[(rw * 64 + rt * 16 + l16) * kActStride + fw * 64 + ft * 16 + lf] = make_uint2(lo, hi);
        }
      __syncthreads();
    }
  }
  // output layer 256 -> 1 in FP32: per-lane partial over its 16 features,
  // then the 4 lane groups that share a row, then the 4 feature blocks in order
  float w4[4][4];
#pragma unroll
  for (int ft = 0; ft < 4; ++ft) {
    const float4 w = *(const float4*)&p[OW4 + fw * 64 + ft * 16 + lf];
    w4[ft][0] = w.x;
    w4[ft][1] = w.y;
    w4[ft][2] = w.z;
    w4[ft][3] = w.w;
  }
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    float v = 0.0f;
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
      for (int j = 0; j < 4; ++j) v = fmaf(acc[ft][rt][j], w4[ft][j], v);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lane < 16) red[fw][rw * 64 + rt * 16 + l16] = v;
  }
  __syncthreads();
  if (threadIdx.x < kInferRows && r0 + threadIdx.x < n) {
    const int t = threadIdx.x;
    const float y = ((red[0][t] + red[1][t]) + (red[2][t] + red[3][t])) + p[OB4];
    out[r0 + t] = sc.ym + sc.ys * (double)y;
  }
}

// Prescreen decision per candidate: bit0 exact evaluation wanted, bit1 the
// prediction passes (pred >= log L* - margin), bit2 audited (a rejected
// candidate drawn for an exact check with probability audit_frac, Philox
// word 0 of counter (i, 0, 0, 0) under key (seed, 1)).
__device__ inline double audit_uniform(uint64_t seed, int64_t i) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c[4] = {(uint64_t)i, 0ull, 0ull, 0ull};
  uint64_t k0 = seed, k1 = 1ull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
  return ((double)(c[0] >> 11) + 0.5) * 1.1102230246251565404e-16;
}

__global__ void k_prescreen_flags(const double* __restrict__ pred, int64_t n, double cut, double audit_frac,
                                  uint64_t seed, int use_mlp, int32_t* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int f;
  if (!use_mlp) {
    f = 1;
  } else if (pred[i] >= cut) {
    f = 3;
  } else {
    f = audit_uniform(seed, i) < audit_frac ? 5 : 0;
  }
  flags[i] = f;
}

// Positions of the selected rows (bit0) by a one-workgroup scan; pos[n] holds
// the count.
__global__ void __launch_bounds__(256) k_select_scan(const int32_t* __restrict__ flags, int64_t n,
                                                     int64_t* __restrict__ pos) {
  __shared__ int64_t part[256];
  const int64_t per = (n + 255) / 256;
  const int64_t b = threadIdx.x * per;
  const int64_t e = b + per < n ? b + per : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += flags[i] & 1;
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int j = 0; j < 256; ++j) {
      const int64_t v = part[j];
      part[j] = run;
      run += v;
    }
    pos[n] = run;
  }
  __syncthreads();
  int64_t run = part[threadIdx.x];
  for (int64_t i = b; i < e; ++i) {
    pos[i] = run;
    run += flags[i] & 1;
  }
}

__global__ void k_gather_rows(const double* __restrict__ x, int64_t n, const int32_t* __restrict__ flags,
                              const int64_t* __restrict__ pos, double* __restrict__ xs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !(flags[i] & 1)) return;
  const int64_t j = pos[i];
  for (int d = 0; d < kIn; ++d) xs[j * kIn + d] = x[i * kIn + d];
}

__global__ void k_scatter_logl(const double* __restrict__ sub, int64_t n, const int32_t* __restrict__ flags,
                               const int64_t* __restrict__ pos, double* __restrict__ logl) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  logl[i] = (flags[i] & 1) ? sub[pos[i]] : -INFINITY;
}

__global__ void k_unscale(const float* __restrict__ y, int64_t n, MlpScale sc, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = sc.ym + sc.ys * (double)y[i];
}

}  // namespace gw

using namespace gw;

struct gw_mlp {
  gw_ctx* ctx = nullptr;
  float* p = nullptr;
  float* g = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  uint16_t* q = nullptr;
  bool q_dirty = true;
  int64_t t = 0;
  MlpScale sc{};
  uint64_t sc_version = 0;  // bumped whenever sc changes (a captured launch bakes sc in)
  float* ws = nullptr;  // training workspace
  int64_t ws_rows = 0;
  float* part = nullptr;  // split-K partials
  int64_t part_cap = 0;
  float* loss = nullptr;  // device scalar
  // prescreen workspace
  void* pre = nullptr;
  int64_t pre_cap = 0;
  int64_t* h_count = nullptr;  // pinned
};

namespace {

gw_status mlp_ws(gw_mlp* m, int64_t rows) {
  if (rows <= m->ws_rows) return GW_OK;
  if (m->ws) (void)hipFree(m->ws);
  m->ws = nullptr;
  m->ws_rows = 0;
  const size_t per = kIn + 6 * kH + 2 + 2 * kH;
  gw_status s = check_hip(hipMalloc((void**)&m->ws, (size_t)rows * per * sizeof(float)), "mlp workspace");
  if (s == GW_OK) m->ws_rows = rows;
  return s;
}

struct Act {
  float *xs, *z1, *a1, *z2, *a2, *z3, *a3, *y, *dy, *d0, *d1;
};

Act act_views(gw_mlp* m, int64_t rows) {
  Act a;
  float* w = m->ws;
  a.xs = w; w += rows * kIn;
  a.z1 = w; w += rows * kH;
  a.a1 = w; w += rows * kH;
  a.z2 = w; w += rows * kH;
  a.a2 = w; w += rows * kH;
  a.z3 = w; w += rows * kH;
  a.a3 = w; w += rows * kH;
  a.y = w; w += rows;
  a.dy = w; w += rows;
  a.d0 = w; w += rows * kH;
  a.d1 = w;
  return a;
}

// C = op(A) op(B) (+ bias); with splits > 1 the K range is split and the
// partial products are summed in split order (bias not allowed then).
gw_status gemm(gw_mlp* m, bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
               float* C, int ldc, const float* bias, int splits, hipStream_t st) {
  if (splits < 1) splits = 1;
  const int k_per = ((K + splits - 1) / splits + 15) / 16 * 16;
  splits = (K + k_per - 1) / k_per;
  if (splits < 1) splits = 1;
  float* out = C;
  int64_t stride = 0;
  if (splits > 1) {
    const int64_t need = (int64_t)splits * M * N;
    if (need > m->part_cap) {
      if (m->part) (void)hipFree(m->part);
      m->part = nullptr;
      m->part_cap = 0;
      gw_status s = check_hip(hipMalloc((void**)&m->part, need * sizeof(float)), "mlp partials");
      if (s != GW_OK) return s;
      m->part_cap = need;
    }
    out = m->part;
    stride = (int64_t)M * N;
    ldc = N;
  }
  dim3 grid((N + 63) / 64, (M + 63) / 64, splits);
  if (ta && tb) return set_error(GW_ENOTSUP, "gemm: both transposed");
  if (ta)
    hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, st, M, N, K, k_per, A, lda, B, ldb, out, ldc, stride,
                       splits > 1 ? nullptr : bias);
  else if (tb)
    hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, st, M, N, K, k_per, A, lda, B, ldb, out, ldc, stride,
                       splits > 1 ? nullptr : bias);
  else
    hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, st, M, N, K, k_per, A, lda, B, ldb, out, ldc,
                       stride, splits > 1 ? nullptr : bias);
  gw_status s = check_hip(hipGetLastError(), "gemm launch");
  if (s != GW_OK || splits == 1) return s;
  const int64_t cnt = (int64_t)M * N;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, m->part, splits, cnt, C);
  return check_hip(hipGetLastError(), "split-K reduce launch");
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// FP32 forward of ``rows`` standardised inputs already in a.xs.
gw_status forward32(gw_mlp* m, const Act& a, int64_t rows, hipStream_t st) {
  const int R = (int)rows;
  gw_status s = gemm(m, false, false, R, kH, kIn, a.xs, kIn, m->p + OW1, kH, a.z1, kH, m->p + OB1, 1, st);
  if (s == GW_OK) hipLaunchKernelGGL(k_gelu_fwd, dim3(nblk(rows * kH)), dim3(256), 0, st, a.z1, a.a1, rows * kH);
  if (s == GW_OK) s = gemm(m, false, false, R, kH, kH, a.a1, kH, m->p + OW2, kH, a.z2, kH, m->p + OB2, 1, st);
  if (s == GW_OK) hipLaunchKernelGGL(k_gelu_fwd, dim3(nblk(rows * kH)), dim3(256), 0, st, a.z2, a.a2, rows * kH);
  if (s == GW_OK) s = gemm(m, false, false, R, kH, kH, a.a2, kH, m->p + OW3, kH, a.z3, kH, m->p + OB3, 1, st);
  if (s == GW_OK) hipLaunchKernelGGL(k_gelu_fwd, dim3(nblk(rows * kH)), dim3(256), 0, st, a.z3, a.a3, rows * kH);
  if (s == GW_OK) s = gemm(m, false, false, R, 1, kH, a.a3, kH, m->p + OW4, 1, a.y, 1, m->p + OB4, 1, st);
  if (s == GW_OK) s = check_hip(hipGetLastError(), "mlp forward");
  return s;
}

// Loss and gradients of one batch into m->g.
gw_status grad32(gw_mlp* m, const double* x, const double* y, int64_t n, hipStream_t st) {
  gw_status s = mlp_ws(m, n);
  if (s != GW_OK) return s;
  Act a = act_views(m, n);
  hipLaunchKernelGGL(k_mlp_stdin, dim3(nblk(n * kIn)), dim3(256), 0, st, x, n, m->sc, a.xs);
  s = forward32(m, a, n, st);
  if (s != GW_OK) return s;
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, a.y, y, n, m->sc, a.dy, m->loss);
  const int R = (int)n;
  const int sp = (int)std::min<int64_t>(32, std::max<int64_t>(1, n / 256));
  float* g = m->g;
  // layer 4
  s = gemm(m, true, false, kH, 1, R, a.a3, kH, a.dy, 1, g + OW4, 1, nullptr, sp, st);
  if (s == GW_OK) hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, st, a.dy, n, 1, g + OB4);
  if (s == GW_OK) s = gemm(m, false, true, R, kH, 1, a.dy, 1, m->p + OW4, 1, a.d0, kH, nullptr, 1, st);
  if (s == GW_OK) hipLaunchKernelGGL(k_gelu_bwd, dim3(nblk(n * kH)), dim3(256), 0, st, a.d0, a.z3, n * kH);
  // layer 3
  if (s == GW_OK) s = gemm(m, true, false, kH, kH, R, a.a2, kH, a.d0, kH, g + OW3, kH, nullptr, sp, st);
  if (s == GW_OK) hipLaunchKernelGGL(k_colsum, dim3(kH / 64), dim3(256), 0, st, a.d0, n, kH, g + OB3);
  if (s == GW_OK) s = gemm(m, false, true, R, kH, kH, a.d0, kH, m->p + OW3, kH, a.d1, kH, nullptr, 1, st);
  if (s == GW_OK) hipLaunchKernelGGL(k_gelu_bwd, dim3(nblk(n * kH)), dim3(256), 0, st, a.d1, a.z2, n * kH);
  // layer 2
  if (s == GW_OK) s = gemm(m, true, false, kH, kH, R, a.a1, kH, a.d1, kH, g + OW2, kH, nullptr, sp, st);
  if (s == GW_OK) hipLaunchKernelGGL(k_colsum, dim3(kH / 64), dim3(256), 0, st, a.d1, n, kH, g + OB2);
  if (s == GW_OK) s = gemm(m, false, true, R, kH, kH, a.d1, kH, m->p + OW2, kH, a.d0, kH, nullptr, 1, st);
  if (s == GW_OK) hipLaunchKernelGGL(k_gelu_bwd, dim3(nblk(n * kH)), dim3(256), 0, st, a.d0, a.z1, n * kH);
  // layer 1
  if (s == GW_OK) s = gemm(m, true, false, kIn, kH, R, a.xs, kIn, a.d0, kH, g + OW1, kH, nullptr, sp, st);
  if (s == GW_OK) hipLaunchKernelGGL(k_colsum, dim3(kH / 64), dim3(256), 0, st, a.d0, n, kH, g + OB1);
  if (s == GW_OK) s = check_hip(hipGetLastError(), "mlp backward");
  return s;
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

namespace gw {

const gw_ctx* mlp_ctx(const gw_mlp* m) { return m->ctx; }

uint64_t mlp_scale_version(const gw_mlp* m) { return m->sc_version; }

gw_status mlp_prepare(gw_mlp* m, hipStream_t st) {
  if (!m->q_dirty) return GW_OK;
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(kNQ)), dim3(256), 0, st, m->p, m->q);
  gw_status s = check_hip(hipGetLastError(), "bf16 conversion launch");
  if (s == GW_OK) m->q_dirty = false;
  return s;
}

gw_status mlp_infer(gw_mlp* m, const double* x, int64_t n, double* out, hipStream_t st) {
  if (n == 0) return GW_OK;
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((n + kInferRows - 1) / kInferRows)), dim3(512), 0, st, x, n, m->sc,
                     m->q, m->p, out);
  return check_hip(hipGetLastError(), "mlp inference launch");
}

}  // namespace gw

extern "C" {

gw_status gw_mlp_create(gw_ctx* ctx, uint64_t seed, gw_mlp** out) {
  if (!ctx || !out) return set_error(GW_EINVAL, "gw_mlp_create: null argument");
  *out = nullptr;
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  gw_mlp* m = new (std::nothrow) gw_mlp();
  if (!m) return set_error(GW_ENOMEM, "gw_mlp_create: host allocation");
  m->ctx = ctx;
  for (int j = 0; j < kIn; ++j) {
    m->sc.xm[j] = 0.5f;
    m->sc.xs_inv[j] = 3.4641016f;  // 1 / sqrt(1/12): standardised uniform
  }
  m->sc.ym = 0.0;
  m->sc.ys = 1.0;
  // He-normal weights from a splitmix64 stream (Box-Muller), zero biases.
  std::vector<float> h(kNPar, 0.0f);
  uint64_t st = seed;
  auto normal = [&]() {
    const double u1 = ((splitmix(st) >> 11) + 0.5) * 1.1102230246251565e-16;
    const double u2 = ((splitmix(st) >> 11) + 0.5) * 1.1102230246251565e-16;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  };
  auto fill = [&](int64_t off, int fan_in, int64_t count) {
    const double sd = sqrt(2.0 / fan_in);
    for (int64_t e = 0; e < count; ++e) h[off + e] = (float)(sd * normal());
  };
  fill(OW1, kIn, kIn * kH);
  fill(OW2, kH, kH * kH);
  fill(OW3, kH, kH * kH);
  fill(OW4, kH, kH);
  float* bufs[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int i = 0; i < 4 && s == GW_OK; ++i) s = check_hip(hipMalloc((void**)&bufs[i], kNPar * sizeof(float)), "mlp");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&m->q, kNQ * sizeof(uint16_t)), "mlp");
  if (s == GW_OK) s = check_hip(hipMalloc((void**)&m->loss, sizeof(float)), "mlp");
  m->p = bufs[0];
  m->g = bufs[1];
  m->m = bufs[2];
  m->v = bufs[3];
  if (s == GW_OK) s = check_hip(hipMemcpy(m->p, h.data(), kNPar * sizeof(float), hipMemcpyHostToDevice), "mlp copy");
  if (s == GW_OK) s = check_hip(hipMemset(m->m, 0, kNPar * sizeof(float)), "mlp memset");
  if (s == GW_OK) s = check_hip(hipMemset(m->v, 0, kNPar * sizeof(float)), "mlp memset");
  if (s == GW_OK) s = check_hip(hipMemset(m->g, 0, kNPar * sizeof(float)), "mlp memset");
  if (s != GW_OK) {
    for (float* b : bufs)
      if (b) (void)hipFree(b);
    if (m->q) (void)hipFree(m->q);
    if (m->loss) (void)hipFree(m->loss);
    delete m;
    return s;
  }
  *out = m;
  return GW_OK;
}

gw_status gw_mlp_destroy(gw_mlp* m) {
  if (!m) return GW_OK;
  (void)hipSetDevice(m->ctx->device);
  float* bufs[] = {m->p, m->g, m->m, m->v, m->ws, m->part, m->loss};
  for (float* b : bufs)
    if (b) (void)hipFree(b);
  if (m->q) (void)hipFree(m->q);
  if (m->pre) (void)hipFree(m->pre);
  if (m->h_count) (void)hipHostFree(m->h_count);
  delete m;
  return GW_OK;
}

gw_status gw_mlp_n_params(int64_t* n) {
  if (!n) return set_error(GW_EINVAL, "gw_mlp_n_params: null");
  *n = kNPar;
  return GW_OK;
}

gw_status gw_mlp_set_scaling(gw_mlp* m, const double* x_mean, const double* x_std, double y_mean, double y_std) {
  if (!m || !x_mean || !x_std) return set_error(GW_EINVAL, "gw_mlp_set_scaling: null argument");
  for (int j = 0; j < kIn; ++j)
    if (!(x_std[j] > 0.0)) return set_error(GW_EINVAL, "gw_mlp_set_scaling: x_std must be > 0");
  if (!(y_std > 0.0) || !isfinite(y_mean)) return set_error(GW_EINVAL, "gw_mlp_set_scaling: bad y scaling");
  for (int j = 0; j < kIn; ++j) {
    m->sc.xm[j] = (float)x_mean[j];
    m->sc.xs_inv[j] = (float)(1.0 / x_std[j]);
  }
  m->sc.ym = y_mean;
  m->sc.ys = y_std;
  m->sc_version += 1;
  return GW_OK;
}

gw_status gw_mlp_set_params(gw_mlp* m, const float* host) {
  if (!m || !host) return set_error(GW_EINVAL, "gw_mlp_set_params: null argument");
  gw_status s = check_hip(hipMemcpy(m->p, host, kNPar * sizeof(float), hipMemcpyHostToDevice), "mlp copy");
  m->q_dirty = true;
  m->t = 0;
  if (s == GW_OK) s = check_hip(hipMemset(m->m, 0, kNPar * sizeof(float)), "mlp memset");
  if (s == GW_OK) s = check_hip(hipMemset(m->v, 0, kNPar * sizeof(float)), "mlp memset");
  return s;
}

gw_status gw_mlp_get_params(gw_mlp* m, float* host) {
  if (!m || !host) return set_error(GW_EINVAL, "gw_mlp_get_params: null argument");
  return check_hip(hipMemcpy(host, m->p, kNPar * sizeof(float), hipMemcpyDeviceToHost), "mlp copy");
}

gw_status gw_mlp_grad(gw_mlp* m, const double* x, const double* y, int64_t n, float* grads_host, float* loss_host,
                      void* stream) {
  if (!m || !x || !y || !grads_host) return set_error(GW_EINVAL, "gw_mlp_grad: null argument");
  if (n < 1 || n > (1 << 24)) return set_error(GW_EINVAL, "gw_mlp_grad: n out of range");
  hipStream_t st = (hipStream_t)stream;
  gw_status s = grad32(m, x, y, n, st);
  if (s == GW_OK)
    s = check_hip(hipMemcpyAsync(grads_host, m->g, kNPar * sizeof(float), hipMemcpyDeviceToHost, st), "copy");
  if (s == GW_OK && loss_host)
    s = check_hip(hipMemcpyAsync(loss_host, m->loss, sizeof(float), hipMemcpyDeviceToHost, st), "copy");
  if (s == GW_OK) s = check_hip(hipStreamSynchronize(st), "gw_mlp_grad sync");
  return s;
}

gw_status gw_mlp_train_step(gw_mlp* m, const double* x, const double* y, int64_t n, float lr, float* loss_host,
                            void* stream) {
  if (!m || !x || !y) return set_error(GW_EINVAL, "gw_mlp_train_step: null argument");
  if (n < 1 || n > (1 << 24)) return set_error(GW_EINVAL, "gw_mlp_train_step: n out of range");
  if (!(lr > 0.0f)) return set_error(GW_EINVAL, "gw_mlp_train_step: lr must be > 0");
  hipStream_t st = (hipStream_t)stream;
  gw_status s = grad32(m, x, y, n, st);
  if (s != GW_OK) return s;
  m->t += 1;
  const float c1 = (float)(1.0 / (1.0 - pow(0.9, (double)m->t)));
  const float c2 = (float)(1.0 / (1.0 - pow(0.999, (double)m->t)));
  hipLaunchKernelGGL(k_adam, dim3(nblk(kNPar)), dim3(256), 0, st, m->p, m->g, m->m, m->v, kNPar, lr, c1, c2);
  s = check_hip(hipGetLastError(), "adam launch");
  m->q_dirty = true;
  if (s == GW_OK && loss_host) {
    s = check_hip(hipMemcpyAsync(loss_host, m->loss, sizeof(float), hipMemcpyDeviceToHost, st), "copy");
    if (s == GW_OK) s = check_hip(hipStreamSynchronize(st), "gw_mlp_train_step sync");
  }
  return s;
}

gw_status gw_mlp_forward(gw_mlp* m, const double* x, int64_t n, double* out, int32_t use_bf16, void* stream) {
  if (!m || (n > 0 && (!x || !out))) return set_error(GW_EINVAL, "gw_mlp_forward: null argument");
  if (n < 0) return set_error(GW_EINVAL, "gw_mlp_forward: n < 0");
  if (n == 0) return GW_OK;
  hipStream_t st = (hipStream_t)stream;
  gw_status s = check_hip(hipSetDevice(m->ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  if (use_bf16) {
    if (m->q_dirty) {
      hipLaunchKernelGGL(k_to_bf16, dim3(nblk(kNQ)), dim3(256), 0, st, m->p, m->q);
      s = check_hip(hipGetLastError(), "bf16 conversion launch");
      if (s != GW_OK) return s;
      m->q_dirty = false;
    }
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((n + kInferRows - 1) / kInferRows)), dim3(512), 0, st, x, n, m->sc,
                     m->q, m->p, out);
    return check_hip(hipGetLastError(), "mlp inference launch");
  }
  const int64_t chunk = 1 << 16;
  s = mlp_ws(m, std::min(n, chunk));
  for (int64_t o = 0; o < n && s == GW_OK; o += chunk) {
    const int64_t r = std::min(chunk, n - o);
    Act a = act_views(m, std::min(n, chunk));
    hipLaunchKernelGGL(k_mlp_stdin, dim3(nblk(r * kIn)), dim3(256), 0, st, x + o * kIn, r, m->sc, a.xs);
    s = forward32(m, a, r, st);
    if (s == GW_OK) hipLaunchKernelGGL(k_unscale, dim3(nblk(r)), dim3(256), 0, st, a.y, r, m->sc, out + o);
    if (s == GW_OK) s = check_hip(hipGetLastError(), "mlp forward");
  }
  return s;
}

// Prescreened exact evaluation of unit-cube candidates (see gwswig.h).
gw_status gw_prescreen_batch(gw_ctx* ctx, gw_mlp* m, const double* x, int64_t n, double logl_star, double margin,
                             double audit_frac, uint64_t seed, int32_t use_mlp, int32_t like, int32_t prec,
                             double* logl, double* pred, int32_t* flags, int64_t* n_exact, void* stream) {
  if (!ctx || !m || !n_exact) return set_error(GW_EINVAL, "gw_prescreen_batch: null argument");
  if (n < 0) return set_error(GW_EINVAL, "gw_prescreen_batch: n < 0");
  *n_exact = 0;
  if (n == 0) return GW_OK;
  if (!x || !logl || !flags) return set_error(GW_EINVAL, "gw_prescreen_batch: null pointer");
  if (!(audit_frac >= 0.0 && audit_frac <= 1.0) || !isfinite(margin))
    return set_error(GW_EINVAL, "gw_prescreen_batch: audit_frac in [0, 1] and finite margin");
  if (like != GW_FULL && like != GW_HET) return set_error(GW_EINVAL, "gw_prescreen_batch: bad like");
  if (like == GW_HET && !ctx->het) return set_error(GW_ESTATE, "gw_prescreen_batch: heterodyne_setup missing");
  if (ctx->n_dist <= 0) return set_error(GW_ESTATE, "gw_prescreen_batch: distance marginal needs a distance grid");
  hipStream_t st = (hipStream_t)stream;
  gw_status s = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
  if (s != GW_OK) return s;
  // workspace: pred [n], pos [n + 1], x_sel [n][11], theta [n][13], logl_sel [n]
  const int64_t need = n * (1 + 1 + kIn + 13 + 1) + 1;
  if (!m->h_count) {
    s = check_hip(hipHostMalloc((void**)&m->h_count, sizeof(int64_t), hipHostMallocDefault), "pinned count");
    if (s != GW_OK) return s;
  }
  if (m->pre_cap < need) {
    if (m->pre) (void)hipFree(m->pre);
    m->pre = nullptr;
    m->pre_cap = 0;
    s = check_hip(hipMalloc(&m->pre, need * sizeof(double)), "prescreen workspace");
    if (s != GW_OK) return s;
    m->pre_cap = need;
  }
  double* d_pred = (double*)m->pre;
  int64_t* d_pos = (int64_t*)(d_pred + n);
  double* d_xs = (double*)(d_pos + n + 1);
  double* d_th = d_xs + n * kIn;
  double* d_sub = d_th + n * 13;
  if (use_mlp) {
    s = gw_mlp_forward(m, x, n, d_pred, 1, st);
    if (s != GW_OK) return s;
  }
  hipLaunchKernelGGL(k_prescreen_flags, dim3(nblk(n)), dim3(256), 0, st, (const double*)d_pred, n,
                     logl_star - margin, audit_frac, seed, use_mlp, flags);
  hipLaunchKernelGGL(k_select_scan, dim3(1), dim3(256), 0, st, (const int32_t*)flags, n, d_pos);
  hipLaunchKernelGGL(k_gather_rows, dim3(nblk(n)), dim3(256), 0, st, x, n, (const int32_t*)flags,
                     (const int64_t*)d_pos, d_xs);
  s = check_hip(hipGetLastError(), "prescreen launch");
  if (s == GW_OK)
    s = check_hip(hipMemcpyAsync(m->h_count, d_pos + n, sizeof(int64_t), hipMemcpyDeviceToHost, st), "copy");
  if (s == GW_OK) s = check_hip(hipStreamSynchronize(st), "prescreen count");
  if (s != GW_OK) return s;
  const int64_t ns = *m->h_count;
  if (ns > 0) {
    s = gw_prior_transform(ctx, d_xs, ns, d_th, stream);
    if (s == GW_OK) s = loglike_batch(ctx, d_th, ns, like, GW_MARG_PHASE_DIST, prec, d_sub, stream);
    if (s != GW_OK) return s;
  }
  hipLaunchKernelGGL(k_scatter_logl, dim3(nblk(n)), dim3(256), 0, st, (const double*)d_sub, n, (const int32_t*)flags,
                     (const int64_t*)d_pos, logl);
  s = check_hip(hipGetLastError(), "prescreen scatter launch");
  if (s == GW_OK && pred && use_mlp)
    s = check_hip(hipMemcpyAsync(pred, d_pred, n * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  *n_exact = ns;
  return s;
}

}  // extern "C"
