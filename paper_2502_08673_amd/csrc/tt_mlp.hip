// tt_mlp.hip -- BF16 kernels of the learned screen (gfx950): a strided GEMM
// on v_mfma_f32_32x32x16_bf16 with fp32 accumulation for the forward pass and
// both backward products, a bias-gradient column sum, the loss with its
// gradient, Adam with fp32 master weights, and the feature / label kernels.
//
// Network: 32 -> 256 -> 256 -> 256 -> 12, ReLU hidden layers, weights stored
// [out, in] row-major.  Loss averaged over a batch of B samples:
//   sum_j m_j * BCE(z_j, y_j) over the 8 support logits, plus the squared
//   error of the 4 histogram outputs (the kind of regression loss the paper
//   minimises by gradient descent in its Methodology section).
#include "tt_internal.h"

namespace tt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf16_to_f32(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

// Round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

struct GemmArgs {
  const uint16_t* A;  // A(m, k) = A[m * sam + k * sak]
  int64_t sam, sak;
  const uint16_t* B;  // B(k, n) = B[k * sbk + n * sbn]
  int64_t sbk, sbn;
  int M, N, K;
  const float* bias;      // [N] or NULL
  int relu;               // max(., 0) after the bias
  const uint16_t* mask;   // NULL, or zero the result where mask(m, n) <= 0
  int64_t smm, smn;
  float* Cf;              // fp32 result C[m * scf + n] or NULL
  int64_t scf;
  uint16_t* Cb;           // bf16 result or NULL
  int64_t scb;
};

// 64 x 64 block tile, four waves of 32 x 32, K in steps of 16.
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ uint16_t As[64][16 + 2];
  __shared__ uint16_t Bs[16][64 + 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    for (int e = tid; e < 64 * 16; e += 256) {
      const int r = e >> 4, c = e & 15;
      const int m = m0 + r, k = k0 + c;
      As[r][c] = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : (uint16_t)0;
    }
    for (int e = tid; e < 16 * 64; e += 256) {
      const int r = e >> 6, c = e & 63;
      const int k = k0 + r, n = n0 + c;
      Bs[r][c] = (k < g.K && n < g.N) ? g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn] : (uint16_t)0;
    }
    __syncthreads();
    // A operand: lane l carries A[wm + l%32][8*(l/32) + t]; B operand:
    // B[8*(l/32) + t][wn + l%32], t = 0..7.
    bf16x8 a, b;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      a[t] = __builtin_bit_cast(__bf16, As[wm + (lane & 31)][8 * (lane >> 5) + t]);
      b[t] = __builtin_bit_cast(__bf16, Bs[8 * (lane >> 5) + t][wn + (lane & 31)]);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    __syncthreads();
  }
  // Result register v of lane l: row 8*(v/4) + 4*(l/32) + v%4, column l%32.
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int n = n0 + wn + (lane & 31);
    if (m < g.M && n < g.N) {
      float x = acc[v];
      if (g.bias) x += g.bias[n];
      if (g.relu) x = fmaxf(x, 0.f);
      if (g.mask && !(bf16_to_f32(g.mask[(int64_t)m * g.smm + (int64_t)n * g.smn]) > 0.f)) x = 0.f;
      if (g.Cf) g.Cf[(int64_t)m * g.scf + n] = x;
      if (g.Cb) g.Cb[(int64_t)m * g.scb + n] = f32_to_bf16(x);
    }
  }
}

// Forward product with both operands contiguous along K (x[m][k] and
// W[n][k]): each lane loads its 8-element MFMA fragments with one 16-byte
// load straight from global memory (no LDS, no barriers).  One wave computes
// 32 rows x 64 columns (two 32x32x16 tiles sharing the A fragment); K must
// be a multiple of 16 and the rows 16-byte aligned.
__global__ __launch_bounds__(256) void gemm_fwd_direct_kernel(GemmArgs g) {
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int ntile = (g.N + 63) / 64;
  const int m0 = (wave / ntile) * 32, n0 = (wave % ntile) * 64;
  if (m0 >= g.M) return;
  const int am = m0 + (lane & 31);
  const int bn0 = n0 + (lane & 31), bn1 = bn0 + 32;
  const int kofs = 8 * (lane >> 5);
  const bool va = am < g.M, vb0 = bn0 < g.N, vb1 = bn1 < g.N;
  const uint16_t* pa = g.A + (int64_t)(va ? am : 0) * g.sam + kofs;
  const uint16_t* pb0 = g.B + (int64_t)(vb0 ? bn0 : 0) * g.sbn + kofs;
  const uint16_t* pb1 = g.B + (int64_t)(vb1 ? bn1 : 0) * g.sbn + kofs;
  f32x16 acc0, acc1;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc0[v] = acc1[v] = 0.f;
  const bf16x8 zero = {};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    bf16x8 a = va ? *reinterpret_cast<const bf16x8*>(pa + k0) : zero;
    bf16x8 b0 = vb0 ? *reinterpret_cast<const bf16x8*>(pb0 + k0) : zero;
    bf16x8 b1 = vb1 ? *reinterpret_cast<const bf16x8*>(pb1 + k0) : zero;
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int m = m0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const int n = n0 + 32 * h + (lane & 31);
      if (m < g.M && n < g.N) {
        float x = h ? acc1[v] : acc0[v];
        if (g.bias) x += g.bias[n];
        if (g.relu) x = fmaxf(x, 0.f);
        if (g.Cf) g.Cf[(int64_t)m * g.scf + n] = x;
        if (g.Cb) g.Cb[(int64_t)m * g.scb + n] = f32_to_bf16(x);
      }
    }
  }
}

static hipError_t gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// db[n] = sum_m dY[m, n]: partial sums over row slices, then a fixed-order
// reduction of the partials (deterministic).
constexpr int kColRows = 512;
__global__ void colsum_partial_kernel(const uint16_t* dY, int M, int N, float* part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int slice = blockIdx.y;
  if (n >= N) return;
  float acc = 0.f;
  const int r0 = slice * kColRows, r1 = min(M, r0 + kColRows);
  for (int m = r0; m < r1; ++m) acc += bf16_to_f32(dY[(int64_t)m * N + n]);
  part[(int64_t)slice * N + n] = acc;
}
__global__ void colsum_final_kernel(const float* part, int slices, int N, float* db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float acc = 0.f;
  for (int s = 0; s < slices; ++s) acc += part[(int64_t)s * N + n];
  db[n] = acc;
}

// Loss and dL/dz for logits z [B, 12] (row stride 12).
__global__ void loss_kernel(const float* z, int Bn, const float* y, const float* msk, const float* h, uint16_t* dz,
                            float* part) {
  __shared__ float red[256];
  float acc = 0.f;
  const float inv = 1.0f / (float)Bn;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Bn; i += gridDim.x * blockDim.x) {
    const float* zi = z + (int64_t)i * 12;
    for (int j = 0; j < 8; ++j) {
      const float zz = zi[j], yy = y[(int64_t)i * 8 + j], mm = msk[(int64_t)i * 8 + j];
      const float sp = fmaxf(zz, 0.f) + log1pf(expf(-fabsf(zz)));
      acc += mm * (sp - yy * zz);
      const float sg = 1.f / (1.f + expf(-zz));
      dz[(int64_t)i * 12 + j] = f32_to_bf16(mm * (sg - yy) * inv);
    }
    for (int v = 0; v < 4; ++v) {
      const float d = zi[8 + v] - h[(int64_t)i * 4 + v];
      acc += d * d;
      dz[(int64_t)i * 12 + 8 + v] = f32_to_bf16(2.f * d * inv);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void loss_final_kernel(const float* part, int parts, int Bn, float* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float acc = 0.f;
  for (int i = 0; i < parts; ++i) acc += part[i];
  loss[0] = acc / (float)Bn;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, uint16_t* pb, size_t n, float lr, float b1,
                            float b2, float eps, float bc1, float bc2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float upd = lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    const float pi = p[i] - upd;
    p[i] = pi;
    if (pb) pb[i] = f32_to_bf16(pi);
  }
}

// Screen input features [n, 32] (bf16) from device descriptors.
__global__ void features_kernel(const tt_neuron* desc, int n, uint16_t* x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const tt_neuron d = desc[i];
  const int F = d.F, b = d.b, o = d.o;
  const int dmax = (1 << b) - 1;
  float f[32];
  for (int k = 0; k < 32; ++k) f[k] = 0.f;
  int pos = 0, neg = 0;
  for (int j = 0; j < 8; ++j) {
    const int w = j < F ? (int)d.w[j] : 0;
    f[j] = (float)w / 8.f;
    f[8 + j] = (float)(w * dmax) / 32.f;
    pos += w > 0 ? w : 0;
    neg += w < 0 ? w : 0;
  }
  f[16] = (float)d.bias / 16.f;
  const int K = (1 << o) - 1;
  for (int k = 0; k < 7; ++k) f[17 + k] = (float)d.thr[k < K ? k : K - 1] / 32.f;
  f[24] = (float)(d.bias + pos * dmax) / 32.f;
  f[25] = (float)(d.bias + neg * dmax) / 32.f;
  f[26] = (float)b / 4.f;
  f[27 + (o - 1)] = 1.f;
  f[30] = (float)F / 8.f;
  f[31] = (float)d.act;
  for (int k = 0; k < 32; ++k) x[(int64_t)i * 32 + k] = f32_to_bf16(f[k]);
}

// Targets from exact support and histogram.
__global__ void labels_kernel(const tt_neuron* desc, int n, const uint8_t* support, const uint32_t* hist, float* y,
                              float* m, float* h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const tt_neuron d = desc[i];
  for (int j = 0; j < 8; ++j) {
    m[(int64_t)i * 8 + j] = j < d.F ? 1.f : 0.f;
    y[(int64_t)i * 8 + j] = (j < d.F && ((support[i] >> j) & 1)) ? 1.f : 0.f;
  }
  const uint32_t* hh = hist + (int64_t)i * 8;
  uint32_t bins[4];
  if (d.o == 1) {
    bins[0] = hh[0]; bins[1] = hh[1]; bins[2] = 0; bins[3] = 0;
  } else if (d.o == 2) {
    bins[0] = hh[0]; bins[1] = hh[1]; bins[2] = hh[2]; bins[3] = hh[3];
  } else {
    bins[0] = hh[0] + hh[1]; bins[1] = hh[2] + hh[3]; bins[2] = hh[4] + hh[5]; bins[3] = hh[6] + hh[7];
  }
  const float rows = (float)(1ull << (d.F * d.b));
  for (int v = 0; v < 4; ++v) h[(int64_t)i * 4 + v] = (float)bins[v] / rows;
}

// ------------------------------------------------------------- launchers
hipError_t mlp_forward(const uint16_t* x, int Bn, int in, const uint16_t* w, const float* bias, int out, int relu,
                       uint16_t* yb, float* yf, hipStream_t s) {
  GemmArgs g{};
  g.A = x; g.sam = in; g.sak = 1;
  g.B = w; g.sbk = 1; g.sbn = in;
  g.M = Bn; g.N = out; g.K = in;
  g.bias = bias; g.relu = relu;
  g.Cf = yf; g.scf = out;
  g.Cb = yb; g.scb = out;
  const bool aligned = ((uintptr_t)x % 16 == 0) && ((uintptr_t)w % 16 == 0) && (in % 16 == 0);
  if (aligned && Bn > 0) {
    const int64_t waves = (int64_t)((Bn + 31) / 32) * ((out + 63) / 64);
    hipLaunchKernelGGL(gemm_fwd_direct_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, g);
    return hipGetLastError();
  }
  return gemm(g, s);
}

hipError_t mlp_backward(const uint16_t* dy, int Bn, int out, const uint16_t* w, int in, const uint16_t* x,
                        int mask_relu, uint16_t* dx, float* dw, float* db, float* scratch, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (dx) {
    GemmArgs g{};
    g.A = dy; g.sam = out; g.sak = 1;
    g.B = w; g.sbk = in; g.sbn = 1;
    g.M = Bn; g.N = in; g.K = out;
    if (mask_relu) { g.mask = x; g.smm = in; g.smn = 1; }
    g.Cb = dx; g.scb = in;
    if ((e = gemm(g, s)) != hipSuccess) return e;
  }
  if (dw) {
    GemmArgs g{};
    g.A = dy; g.sam = 1; g.sak = out;
    g.B = x; g.sbk = in; g.sbn = 1;
    g.M = out; g.N = in; g.K = Bn;
    g.Cf = dw; g.scf = in;
    if ((e = gemm(g, s)) != hipSuccess) return e;
  }
  if (db) {
    const int slices = (Bn + kColRows - 1) / kColRows;
    hipLaunchKernelGGL(colsum_partial_kernel, dim3((out + 63) / 64, slices), dim3(64), 0, s, dy, Bn, out, scratch);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_final_kernel, dim3((out + 63) / 64), dim3(64), 0, s, scratch, slices, out, db);
    e = hipGetLastError();
  }
  return e;
}

int mlp_colsum_scratch_floats(int Bn, int out) { return ((Bn + kColRows - 1) / kColRows) * out; }

hipError_t mlp_loss(const float* z, int Bn, const float* y, const float* m, const float* h, uint16_t* dz,
                    float* loss, float* scratch, hipStream_t s) {
  const int blocks = 64;
  hipLaunchKernelGGL(loss_kernel, dim3(blocks), dim3(256), 0, s, z, Bn, y, m, h, dz, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, s, scratch, blocks, Bn, loss);
  return hipGetLastError();
}

hipError_t adam_step(float* p, const float* g, float* m, float* v, uint16_t* pb, size_t n, float lr, float b1,
                     float b2, float eps, float bc1, float bc2, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, g, m, v, pb, n, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

__global__ void cast_bf16_kernel(const float* x, uint16_t* y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = f32_to_bf16(x[i]);
}

hipError_t cast_bf16(const float* x, uint16_t* y, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(cast_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t screen_features(const tt_neuron* d, int n, uint16_t* x, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, n, x);
  return hipGetLastError();
}

hipError_t screen_labels(const tt_neuron* d, int n, const uint8_t* sup, const uint32_t* hist, float* y, float* m,
                         float* h, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(labels_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, n, sup, hist, y, m, h);
  return hipGetLastError();
}

}  // namespace tt
