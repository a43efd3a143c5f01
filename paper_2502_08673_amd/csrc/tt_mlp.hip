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
#include <algorithm>

#include "tt_internal.h"
#include "tt_mlp.h"

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

// Eight bf16 elements c0 .. c0 + 7 of a row as one 16-byte piece (zero past
// lim): one vector load when allowed and in range, else element loads.
__device__ __forceinline__ uint4 load_piece(const uint16_t* row, int c0, int lim, bool vec) {
  if (vec && c0 + 8 <= lim) return *reinterpret_cast<const uint4*>(row + c0);
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (c0 + e < lim) w[e >> 1] |= (uint32_t)row[c0 + e] << (16 * (e & 1));
  return make_uint4(w[0], w[1], w[2], w[3]);
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
  // Every load of the epilogue (bias, mask) is issued before its first store:
  // a load issued after a store waits for that store to complete.
  const int nn = n0 + wn + (lane & 31);
  const float bnn = (g.bias && nn < g.N) ? g.bias[nn] : 0.f;
  bool keep[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    keep[v] = true;
    if (g.mask && m < g.M && nn < g.N) keep[v] = bf16_to_f32(g.mask[(int64_t)m * g.smm + (int64_t)nn * g.smn]) > 0.f;
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int n = nn;
    if (m < g.M && n < g.N) {
      float x = acc[v] + bnn;
      if (g.relu) x = fmaxf(x, 0.f);
      if (!keep[v]) x = 0.f;
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
  // bias loaded before any store (a load after a store waits for it)
  const float bias0 = (g.bias && vb0) ? g.bias[bn0] : 0.f, bias1 = (g.bias && vb1) ? g.bias[bn1] : 0.f;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int m = m0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const int n = n0 + 32 * h + (lane & 31);
      if (m < g.M && n < g.N) {
        float x = (h ? acc1[v] : acc0[v]) + (h ? bias1 : bias0);
        if (g.relu) x = fmaxf(x, 0.f);
        if (g.Cf) g.Cf[(int64_t)m * g.scf + n] = x;
        if (g.Cb) g.Cb[(int64_t)m * g.scb + n] = f32_to_bf16(x);
      }
    }
  }
}

// Forward product with 256 output columns: a block of four waves takes 64
// rows x 256 columns, each wave 32 rows x 128 columns (four 32x32 fp32
// accumulator tiles).  The weights pass through LDS in K-chunks of 32,
// double buffered and shared by the four waves; every global load (the next
// weight chunk, the next A fragments) is issued one chunk ahead.  LDS rows
// are padded to 40 elements, so the sixteen lanes of each 128-bit read phase
// hit 64 distinct banks.
constexpr int kWideN = 256, kWideKC = 32, kWideRow = kWideKC + 8;
__global__ __launch_bounds__(256) void gemm_fwd_wide_kernel(GemmArgs g) {
  __shared__ uint16_t Ws[2][kWideN * kWideRow];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int n0 = (wave >> 1) * 128;
  const int am = m0 + (lane & 31);
  const bool va = am < g.M;
  const uint16_t* pa = g.A + (int64_t)(va ? am : 0) * g.sam + 8 * (lane >> 5);
  const int nchunks = g.K / kWideKC;
  f32x16 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[j][v] = 0.f;
  // a chunk is 256 rows x 32 elements = 1024 16-byte pieces, four per
  // thread: row tid / 4 + 64 i, elements 8 (tid % 4) .. + 7
  const int prow = tid >> 2, pq = tid & 3;
  const uint16_t* pw = g.B + (int64_t)prow * g.sbn + 8 * pq;
  const int64_t pstep = 64 * g.sbn;
  const bf16x8 zero = {};
  uint4 n0v = *reinterpret_cast<const uint4*>(pw);
  uint4 n1v = *reinterpret_cast<const uint4*>(pw + pstep);
  uint4 n2v = *reinterpret_cast<const uint4*>(pw + 2 * pstep);
  uint4 n3v = *reinterpret_cast<const uint4*>(pw + 3 * pstep);
  bf16x8 a0 = va ? *reinterpret_cast<const bf16x8*>(pa) : zero;
  bf16x8 a1 = va ? *reinterpret_cast<const bf16x8*>(pa + 16) : zero;
  {
    uint16_t* dst = &Ws[0][prow * kWideRow + 8 * pq];
    *reinterpret_cast<uint4*>(dst) = n0v;
    *reinterpret_cast<uint4*>(dst + 64 * kWideRow) = n1v;
    *reinterpret_cast<uint4*>(dst + 128 * kWideRow) = n2v;
    *reinterpret_cast<uint4*>(dst + 192 * kWideRow) = n3v;
  }
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    const bool more = c + 1 < nchunks;
    const bf16x8 ca0 = a0, ca1 = a1;
    if (more) {
      const uint16_t* q = pw + (c + 1) * kWideKC;
      n0v = *reinterpret_cast<const uint4*>(q);
      n1v = *reinterpret_cast<const uint4*>(q + pstep);
      n2v = *reinterpret_cast<const uint4*>(q + 2 * pstep);
      n3v = *reinterpret_cast<const uint4*>(q + 3 * pstep);
      a0 = va ? *reinterpret_cast<const bf16x8*>(pa + (c + 1) * kWideKC) : zero;
      a1 = va ? *reinterpret_cast<const bf16x8*>(pa + (c + 1) * kWideKC + 16) : zero;
    }
    const uint16_t* wb = &Ws[buf][(n0 + (lane & 31)) * kWideRow + 8 * (lane >> 5)];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(wb + 32 * j * kWideRow);
      acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ca0, b, acc[j], 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(wb + 32 * j * kWideRow + 16);
      acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ca1, b, acc[j], 0, 0, 0);
    }
    if (more) {
      uint16_t* dst = &Ws[buf ^ 1][prow * kWideRow + 8 * pq];
      *reinterpret_cast<uint4*>(dst) = n0v;
      *reinterpret_cast<uint4*>(dst + 64 * kWideRow) = n1v;
      *reinterpret_cast<uint4*>(dst + 128 * kWideRow) = n2v;
      *reinterpret_cast<uint4*>(dst + 192 * kWideRow) = n3v;
    }
    __syncthreads();
  }
  float bns[4];  // loaded before any store (a load after a store waits for it)
#pragma unroll
  for (int j = 0; j < 4; ++j) bns[j] = g.bias ? g.bias[n0 + 32 * j + (lane & 31)] : 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + 32 * j + (lane & 31);
    const float bn = bns[j];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int m = m0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      if (m < g.M) {
        float x = acc[j][v] + bn;
        if (g.relu) x = fmaxf(x, 0.f);
        if (g.Cf) g.Cf[(int64_t)m * g.scf + n] = x;
        if (g.Cb) g.Cb[(int64_t)m * g.scb + n] = f32_to_bf16(x);
      }
    }
  }
}

// Forward product with 256 output columns and K = 32 or 256, the shapes of
// the screening network at inference batch sizes: one block per CU keeps
// all of W in LDS (256 rows of K elements, padded by 8 so that the sixteen
// lanes of a 128-bit read phase hit 64 distinct banks) and its eight waves
// then walk 64-row x 128-column output tiles with no further barriers.  The
// MFMA computes the transposed tile (W rows as its A operand, X rows as its
// B operand), so each lane ends up with runs of four consecutive output
// columns of one row: 8-byte stores.  Each weight fragment read from LDS
// feeds two MFMAs (two row groups); X fragments come straight from global
// memory one k-step ahead.
template <int K>
__global__ __launch_bounds__(512) void gemm_fwd_persist_kernel(GemmArgs g) {
  extern __shared__ uint16_t Wl[];
  constexpr int RS = K + 8;
  // the bias lives in LDS after the weights: epilogue reads of it then never
  // wait behind this wave's earlier global stores
  float* bl = reinterpret_cast<float*>(Wl + kWideN * RS);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int p = tid; p < kWideN * (K / 8); p += 512) {
    const int n = p / (K / 8), q = p % (K / 8);
    *reinterpret_cast<uint4*>(&Wl[n * RS + 8 * q]) = *reinterpret_cast<const uint4*>(g.B + (int64_t)n * g.sbn + 8 * q);
  }
  for (int n = tid; n < kWideN; n += 512) bl[n] = g.bias ? g.bias[n] : 0.f;
  __syncthreads();
  const bf16x8 zero = {};
  auto frag = [&](bool valid, const uint16_t* row, int c0) -> bf16x8 {
    return valid ? *reinterpret_cast<const bf16x8*>(row + c0) : zero;
  };
  // K is taken in groups of KG: the MFMA's k-slot (h, e) of step s in group
  // G stands for k = KG G + (KG / 2) h + 8 s + e, the same for both operands,
  // so each lane reads KG / 2 contiguous elements of its X row per group.
  constexpr int KG = K < 64 ? K : 64, NS = KG / 16, NG = K / KG;
  const int ntiles = ((g.M + 63) / 64) * 2;
  for (int t = blockIdx.x * 8 + wave; t < ntiles; t += gridDim.x * 8) {
    const int m0 = (t >> 1) * 64, n0 = (t & 1) * 128;
    const int r0 = m0 + (lane & 31), r1 = r0 + 32;
    const bool v0 = r0 < g.M, v1 = r1 < g.M;
    const int hk = (KG / 2) * (lane >> 5);
    const uint16_t* pa0 = g.A + (int64_t)(v0 ? r0 : 0) * g.sam;
    const uint16_t* pa1 = g.A + (int64_t)(v1 ? r1 : 0) * g.sam;
    const uint16_t* wb = &Wl[(n0 + (lane & 31)) * RS + hk];
    f32x16 acc[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[r][j][v] = 0.f;
    bf16x8 x0[NS], x1[NS];
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      x0[st] = frag(v0, pa0, hk + 8 * st);
      x1[st] = frag(v1, pa1, hk + 8 * st);
    }
#pragma unroll
    for (int G = 0; G < NG; ++G) {
      bf16x8 c0[NS], c1[NS];
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        c0[st] = x0[st];
        c1[st] = x1[st];
      }
      if (G + 1 < NG) {
#pragma unroll
        for (int st = 0; st < NS; ++st) {
          x0[st] = frag(v0, pa0, KG * (G + 1) + hk + 8 * st);
          x1[st] = frag(v1, pa1, KG * (G + 1) + hk + 8 * st);
        }
      }
#pragma unroll
      for (int st = 0; st < NS; ++st) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bf16x8 w = *reinterpret_cast<const bf16x8*>(wb + 32 * j * RS + KG * G + 8 * st);
          acc[0][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, c0[st], acc[0][j], 0, 0, 0);
          acc[1][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, c1[st], acc[1][j], 0, 0, 0);
        }
      }
    }
    // register v of lane l: column n0 + 32 j + 8 (v / 4) + 4 (l / 32) + v % 4
    // of row m0 + 32 r + l % 32
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int m = m0 + 32 * r + (lane & 31);
      if (m < g.M) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int n = n0 + 32 * j + 8 * q + 4 * (lane >> 5);
            float x[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              x[e] = acc[r][j][4 * q + e] + bl[n + e];
              if (g.relu) x[e] = fmaxf(x[e], 0.f);
            }
            if (g.Cb) {
              const uint2 pk = make_uint2((uint32_t)f32_to_bf16(x[0]) | ((uint32_t)f32_to_bf16(x[1]) << 16),
                                          (uint32_t)f32_to_bf16(x[2]) | ((uint32_t)f32_to_bf16(x[3]) << 16));
              *reinterpret_cast<uint2*>(g.Cb + (int64_t)m * g.scb + n) = pk;
            }
            if (g.Cf) *reinterpret_cast<float4*>(g.Cf + (int64_t)m * g.scf + n) = make_float4(x[0], x[1], x[2], x[3]);
          }
        }
      }
    }
  }
}

template <int K>
static hipError_t launch_fwd_persist(const GemmArgs& g, hipStream_t s, bool* launched) {
  *launched = false;
  const size_t lds = sizeof(uint16_t) * kWideN * (K + 8) + sizeof(float) * kWideN;
  int dev = 0, cus = 0, max_lds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  if ((size_t)max_lds < lds) return hipSuccess;  // not launched: the caller takes another kernel
  if (lds > 65536) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_fwd_persist_kernel<K>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return hipSuccess;
    }
  }
  const int tiles = ((g.M + 63) / 64) * 2;
  const int grid = std::max(1, std::min(cus, (tiles + 7) / 8));
  hipLaunchKernelGGL(gemm_fwd_persist_kernel<K>, dim3(grid), dim3(512), lds, s, g);
  e = hipGetLastError();
  if (e == hipSuccess) *launched = true;
  return e;
}

static hipError_t gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// Input gradient of a layer, dX = (dY W) * [X > 0] (the mask is optional):
// W^T, padded with zeros to Kp columns (a multiple of 16), is built in
// scratch by transpose_pad_kernel, so both MFMA operands are K-contiguous
// rows loaded straight from global memory (16 bytes per lane; element loads
// for dY rows that are not 16-byte aligned, e.g. 12 columns).  One wave
// takes 32 rows x 64 columns and computes the transposed tile (W^T rows as
// the A operand), so each lane holds four consecutive columns of one row:
// 8-byte mask loads (all issued before the first store) and 8-byte stores.
__global__ void transpose_pad_kernel(const uint16_t* w, int out, int in, int Kp, uint16_t* wt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over wt = [in][Kp]
  if (i >= (int64_t)in * Kp) return;
  const int n = (int)(i / Kp), k = (int)(i % Kp);
  wt[i] = k < out ? w[(int64_t)k * in + n] : (uint16_t)0;
}

__global__ __launch_bounds__(256) void gemm_dx_kernel(const uint16_t* dy, int out, const uint16_t* wt, int Kp,
                                                     const uint16_t* x, int M, int N, uint16_t* dx) {
  const int lane = threadIdx.x & 63;
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int ntile = (N + 63) / 64;
  const int m0 = (wave / ntile) * 32, n0 = (wave % ntile) * 64;
  if (m0 >= M) return;
  const int am = m0 + (lane & 31);
  const int bn0 = n0 + (lane & 31), bn1 = bn0 + 32;
  const int kofs = 8 * (lane >> 5);
  const bool va = am < M, vb0 = bn0 < N, vb1 = bn1 < N;
  const bool vec_a = (out % 8) == 0 && ((uintptr_t)dy % 16) == 0;
  const uint16_t* pa = dy + (int64_t)(va ? am : 0) * out;
  const uint16_t* pb0 = wt + (int64_t)(vb0 ? bn0 : 0) * Kp + kofs;
  const uint16_t* pb1 = wt + (int64_t)(vb1 ? bn1 : 0) * Kp + kofs;
  f32x16 acc0, acc1;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc0[v] = acc1[v] = 0.f;
  const bf16x8 zero = {};
  for (int k0 = 0; k0 < Kp; k0 += 16) {
    const bf16x8 a = va ? __builtin_bit_cast(bf16x8, load_piece(pa, k0 + kofs, out, vec_a)) : zero;
    const bf16x8 b0 = vb0 ? *reinterpret_cast<const bf16x8*>(pb0 + k0) : zero;
    const bf16x8 b1 = vb1 ? *reinterpret_cast<const bf16x8*>(pb1 + k0) : zero;
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b0, a, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b1, a, acc1, 0, 0, 0);
  }
  // register v of lane l: column n0 + 32 h + 8 (v / 4) + 4 (l / 32) + v % 4 of row am
  if (!va) return;
  const bool vec_n = (N % 4) == 0;
  uint2 mk[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = n0 + 32 * h + 8 * q + 4 * (lane >> 5);
      mk[h][q] = make_uint2(0x3F803F80u, 0x3F803F80u);  // 1.0: keep
      if (x && vec_n && n < N) mk[h][q] = *reinterpret_cast<const uint2*>(x + (int64_t)am * N + n);
    }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = n0 + 32 * h + 8 * q + 4 * (lane >> 5);
      uint16_t o[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float v = h ? acc1[4 * q + e] : acc0[4 * q + e];
        uint32_t xb = ((e < 2 ? mk[h][q].x : mk[h][q].y) >> (16 * (e & 1))) & 0xFFFFu;
        if (x && !vec_n && n + e < N) xb = x[(int64_t)am * N + n + e];
        o[e] = (xb != 0u && (xb & 0x8000u) == 0u) ? f32_to_bf16(v) : (uint16_t)0;  // keep where X > 0
      }
      if (vec_n) {
        if (n < N)
          *reinterpret_cast<uint2*>(dx + (int64_t)am * N + n) =
              make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16), (uint32_t)o[2] | ((uint32_t)o[3] << 16));
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (n + e < N) dx[(int64_t)am * N + n + e] = o[e];
      }
    }
  }
}

// Weight and bias gradients of one layer, split over the batch (the K of
// dW = dY^T X): block (nx, my, s) takes the 64 x 64 tile (rows = outputs m,
// columns = inputs n) over batch slice s and writes its fp32 partial product
// to part[s][m][n]; the blocks of column tile 0 also write the slice's
// column sums of dY to dbp[s][m].  Both operands are batch-major (dY[b][m],
// X[b][n]): chunks of 64 batch rows are staged into LDS with 16-byte loads
// along the contiguous dimension (element loads where a row is not 16-byte
// aligned or the tile is ragged), and each lane then gathers its eight
// batch-consecutive MFMA elements from LDS.  A second kernel reduces the
// partials in a fixed order, so results do not depend on scheduling.
constexpr int kDwKC = 64, kDwRow = 64 + 8, kDwMaxSlices = 64;
__global__ __launch_bounds__(256) void gemm_dw_kernel(const uint16_t* dy, const uint16_t* x, int Bn, int M, int N,
                                                     int kslice, float* part, float* dbp) {
  __shared__ uint16_t As[kDwKC][kDwRow];  // dY[k][m0 + i]
  __shared__ uint16_t Bs[kDwKC][kDwRow];  // X[k][n0 + j]
  __shared__ float s_col[4][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = blockIdx.x * 64, m0 = blockIdx.y * 64, sl = blockIdx.z;
  const int kb = sl * kslice, ke = min(Bn, kb + kslice);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const bool vec_a = (M % 8) == 0 && ((uintptr_t)dy % 16) == 0;
  const bool vec_b = (N % 8) == 0 && ((uintptr_t)x % 16) == 0;
  const bool want_db = dbp && blockIdx.x == 0;
  float col = 0.f;  // column tid % 64 of dY over this thread's rows
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  for (int k0 = kb; k0 < ke; k0 += kDwKC) {
    // two 8-element pieces per thread and operand: row kk, columns 8 q ..
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = tid + 256 * h, kk = p >> 3, q = p & 7;
      const int k = k0 + kk;
      uint4 av = make_uint4(0u, 0u, 0u, 0u), bv = make_uint4(0u, 0u, 0u, 0u);
      if (k < ke) {
        av = load_piece(dy + (int64_t)k * M, m0 + 8 * q, M, vec_a);
        bv = load_piece(x + (int64_t)k * N, n0 + 8 * q, N, vec_b);
      }
      *reinterpret_cast<uint4*>(&As[kk][8 * q]) = av;
      *reinterpret_cast<uint4*>(&Bs[kk][8 * q]) = bv;
    }
    __syncthreads();
    if (want_db) {
#pragma unroll
      for (int r = 0; r < 16; ++r) col += bf16_to_f32(As[(tid >> 6) * 16 + r][tid & 63]);
    }
    // A operand: lane l carries dY[k = 16 st + 8 (l / 32) + t][m = wm + l % 32];
    // B operand: X[k = 16 st + 8 (l / 32) + t][n = wn + l % 32], t = 0..7.
#pragma unroll
    for (int st = 0; st < kDwKC / 16; ++st) {
      bf16x8 a, b;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        a[t] = __builtin_bit_cast(__bf16, As[16 * st + 8 * (lane >> 5) + t][wm + (lane & 31)]);
        b[t] = __builtin_bit_cast(__bf16, Bs[16 * st + 8 * (lane >> 5) + t][wn + (lane & 31)]);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  if (want_db) {
    s_col[tid >> 6][tid & 63] = col;
    __syncthreads();
    if (tid < 64 && m0 + tid < M)
      dbp[(int64_t)sl * M + m0 + tid] = (s_col[0][tid] + s_col[1][tid]) + (s_col[2][tid] + s_col[3][tid]);
  }
  // register v of lane l: row wm + 8 (v / 4) + 4 (l / 32) + v % 4, column wn + l % 32
  float* dst = part + (int64_t)sl * M * N;
  const int n = n0 + wn + (lane & 31);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (m < M && n < N) dst[(int64_t)m * N + n] = acc[v];
  }
}

// dw[i] = sum_s part[s][i] and db[m] = sum_s dbp[s][m], slices in order.
__global__ void dw_reduce_kernel(const float* part, const float* dbp, int S, int64_t MN, int M, float* dw, float* db) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (dw && i < MN) {
    // eight independent chains (slices s = c mod 8), combined in a fixed order
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int s2 = 0;
    for (; s2 + 8 <= S; s2 += 8) {
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] += part[(int64_t)(s2 + c) * MN + i];
    }
    for (int c = 0; s2 < S; ++s2, ++c) acc[c] += part[(int64_t)s2 * MN + i];
    dw[i] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  if (db && i < M) {
    float acc = 0.f;
    for (int s2 = 0; s2 < S; ++s2) acc += dbp[(int64_t)s2 * M + i];
    db[i] = acc;
  }
}

// Batch slices of the weight-gradient kernel: enough blocks to cover the
// chip (about 512), slices of whole 64-row chunks.
struct DwSplit {
  int S, kslice;
};
static DwSplit dw_split(int Bn, int M, int N) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  const int chunks = (Bn + kDwKC - 1) / kDwKC;
  int S = std::max(1, std::min(chunks, std::min(kDwMaxSlices, (512 + tiles - 1) / tiles)));
  const int per = (chunks + S - 1) / S;
  S = (chunks + per - 1) / per;
  return {S, per * kDwKC};
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

// Adam over up to kAdamMaxTensors tensors in one launch: the grid strides
// over their concatenation and each element finds its tensor by the offsets.
struct AdamMulti {
  int count;
  float* p[kAdamMaxTensors];
  const float* g[kAdamMaxTensors];
  float* m[kAdamMaxTensors];
  float* v[kAdamMaxTensors];
  uint16_t* pb[kAdamMaxTensors];
  size_t off[kAdamMaxTensors + 1];
};
__global__ void adam_multi_kernel(AdamMulti a, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const size_t total = a.off[a.count];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    int t = 0;
#pragma unroll
    for (int k = 1; k < kAdamMaxTensors; ++k) t += (k < a.count && i >= a.off[k]) ? 1 : 0;
    const size_t j = i - a.off[t];
    const float gi = a.g[t][j];
    const float mi = b1 * a.m[t][j] + (1.f - b1) * gi;
    const float vi = b2 * a.v[t][j] + (1.f - b2) * gi * gi;
    a.m[t][j] = mi;
    a.v[t][j] = vi;
    const float upd = lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    const float pi = a.p[t][j] - upd;
    a.p[t][j] = pi;
    if (a.pb[t]) a.pb[t][j] = f32_to_bf16(pi);
  }
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
// The 32 screen features of descriptor `dp` (see screen_features), rounded to
// bf16 and packed two per dword.  The first 48 bytes of the descriptor come
// in three 16-byte loads; every field is taken with a constant shift or
// index (no private arrays).
__device__ __forceinline__ void neuron_features(const tt_neuron* dp_, uint32_t (&pk)[16]) {
  const uint4* dp = reinterpret_cast<const uint4*>(dp_);
  const uint4 q0 = dp[0], q1 = dp[1], q2 = dp[2];
  const int F = (q2.y >> 16) & 0xFF, b = q2.y >> 24, o = q2.z & 0xFF, act = (q2.z >> 8) & 0xFF;
  const int bias = (int)(int16_t)(q2.y & 0xFFFFu);
  const uint64_t wv = (uint64_t)q0.x | ((uint64_t)q0.y << 32);
  const int th[7] = {(int)q0.z, (int)q0.w, (int)q1.x, (int)q1.y, (int)q1.z, (int)q1.w, (int)q2.x};
  const int dmax = (1 << b) - 1;
  const int K = (1 << o) - 1;
  const int th_last = K == 1 ? th[0] : (K == 3 ? th[2] : th[6]);
  float f[32];
  int pos = 0, neg = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int w = j < F ? (int)(int8_t)(uint8_t)(wv >> (8 * j)) : 0;
    f[j] = (float)w / 8.f;
    f[8 + j] = (float)(w * dmax) / 32.f;
    pos += w > 0 ? w : 0;
    neg += w < 0 ? w : 0;
  }
  f[16] = (float)bias / 16.f;
#pragma unroll
  for (int k = 0; k < 7; ++k) f[17 + k] = (float)(k < K ? th[k] : th_last) / 32.f;
  f[24] = (float)(bias + pos * dmax) / 32.f;
  f[25] = (float)(bias + neg * dmax) / 32.f;
  f[26] = (float)b / 4.f;
  f[27] = o == 1 ? 1.f : 0.f;
  f[28] = o == 2 ? 1.f : 0.f;
  f[29] = o == 3 ? 1.f : 0.f;
  f[30] = (float)F / 8.f;
  f[31] = (float)act;
#pragma unroll
  for (int k = 0; k < 16; ++k) pk[k] = (uint32_t)f32_to_bf16(f[2 * k]) | ((uint32_t)f32_to_bf16(f[2 * k + 1]) << 16);
}

__global__ void features_kernel(const tt_neuron* desc, int n, uint16_t* x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t pk[16];
  neuron_features(desc + i, pk);
  uint4* out = reinterpret_cast<uint4*>(x + (int64_t)i * 32);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = make_uint4(pk[4 * k], pk[4 * k + 1], pk[4 * k + 2], pk[4 * k + 3]);
}

// Whether the screen's wave pass takes this candidate under the zero-weight
// rule: its table reduced to the inputs of nonzero weight (or full, when
// every weight is nonzero) has more than 64 rows.  Descriptors whose fields
// are out of range are not taken (the screen flags them).
__device__ __forceinline__ bool wave_pass_candidate(const tt_neuron* dp_) {
  const uint4* dp = reinterpret_cast<const uint4*>(dp_);
  const uint4 q0 = dp[0], q2 = dp[2];
  const int F = (q2.y >> 16) & 0xFF, b = q2.y >> 24, o = q2.z & 0xFF, act = (q2.z >> 8) & 0xFF;
  const bool ok = F >= 1 && F <= TT_MAX_F && b >= 1 && b <= TT_MAX_B && o >= 1 && o <= TT_MAX_O && act <= 1 &&
                  F * b <= 16;
  const uint64_t wv = (uint64_t)q0.x | ((uint64_t)q0.y << 32);
  int k = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) k += (j < F && ((wv >> (8 * j)) & 0xFFu) != 0u) ? 1 : 0;
  const int LF = k == F ? F : (k > 0 ? k : 1);
  return ok && LF * b > 6;
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
// Whole-network inference, 32 -> 256 -> 256 -> 256 -> 12: a block of eight
// waves takes 128 rows and keeps their activations in LDS from layer to
// layer (one buffer of 128 rows x (256 + 8) bf16, overwritten in place: a
// layer's outputs stay in registers until every wave has finished reading
// its inputs), so only the features come from HBM and only the logits go
// back.  Weights: every thread loads its share of a whole hidden layer
// (two 16-byte pieces per 32-k chunk) one layer ahead, while the previous
// layer finishes, and the chunks pass through two LDS buffers, one barrier
// each; a block reads every weight from L2 once.  The biases and the output
// layer's weights sit in LDS from the start.  Wave w computes output
// columns 64 (w % 4) .. + 63 of rows 64 (w / 4) .. + 63: per 16-k step two
// weight fragments (MFMA A operand, rows = output columns) and two
// activation fragments (B operand, columns = rows) give four
// v_mfma_f32_32x32x16_bf16.  The 12-column output layer: waves 0-3 take
// 32 rows each, one weight fragment (rows 12-31 zero).  Rounding as in the
// layer-by-layer path: fp32 accumulation, bias, ReLU, round to nearest even
// bf16 between layers (v_cvt_pk_bf16_f32).
constexpr int kInferRows = 128;
constexpr int kActRow = 256 + 8;
constexpr int kWChunk = 32;
constexpr int kWRow = kWChunk + 8;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

struct InferArgs {
  const uint16_t* x;  // [n][32], or NULL: features computed from desc
  int n;
  const tt_neuron* desc;  // with x NULL: the candidates' descriptors (features computed here)
  int gated;              // with desc: only candidates the screen's wave pass takes
  const uint16_t* w[4];  // [256][32], [256][256], [256][256], [12][256]
  const float* b[4];     // [256], [256], [256], [12] (may be NULL)
  float* logits;         // [n][12]
  // list mode (gated, with list): the wave-pass candidates compacted per
  // span of kGateSpan candidates (list[span * kGateSpan + i], cnt[span]),
  // taken in chunks of kInferRows by a persistent grid
  const int32_t* list;
  const int32_t* cnt;
  int nspans;
};

// One 32-k chunk of a hidden layer: two 16-k steps of four MFMAs on the
// chunk in LDS buffer `buf` and the matching columns of H.
__device__ __forceinline__ void infer_chunk(const uint16_t* H, const uint16_t* Wc, int buf, int c, f32x16 (&acc)[2][2],
                                            int lane, int cg, int rg, int hk) {
#pragma unroll
  for (int st = 0; st < kWChunk / 16; ++st) {
    bf16x8 wf[2], hf[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
      wf[j] = *reinterpret_cast<const bf16x8*>(&Wc[(buf * 256 + 64 * cg + 32 * j + (lane & 31)) * kWRow + 16 * st + hk]);
#pragma unroll
    for (int r = 0; r < 2; ++r)
      hf[r] = *reinterpret_cast<const bf16x8*>(&H[(64 * rg + 32 * r + (lane & 31)) * kActRow + c * kWChunk + 16 * st + hk]);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[r][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[j], hf[r], acc[r][j], 0, 0, 0);
  }
}

// Bias (from LDS), ReLU, bf16: a hidden layer's outputs (registers) into H,
// then zeroed accumulators for the next layer.  Register v of lane l:
// column 64 cg + 32 j + 8 (v / 4) + 4 (l / 32) + v % 4 of row 64 rg + 32 r + l % 32.
__device__ __forceinline__ void infer_epilogue(f32x16 (&acc)[2][2], const float* bias, uint16_t* H, int lane, int cg,
                                               int rg) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int n = 64 * cg + 32 * j + 8 * qq + 4 * (lane >> 5);
      const float4 bn = *reinterpret_cast<const float4*>(bias + n);
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int m = 64 * rg + 32 * r + (lane & 31);
        const f32x2 lo = {fmaxf(acc[r][j][4 * qq + 0] + bn.x, 0.f), fmaxf(acc[r][j][4 * qq + 1] + bn.y, 0.f)};
        const f32x2 hi = {fmaxf(acc[r][j][4 * qq + 2] + bn.z, 0.f), fmaxf(acc[r][j][4 * qq + 3] + bn.w, 0.f)};
        *reinterpret_cast<uint2*>(&H[m * kActRow + n]) =
            make_uint2(__builtin_bit_cast(uint32_t, __builtin_convertvector(lo, bf16x2)),
                       __builtin_bit_cast(uint32_t, __builtin_convertvector(hi, bf16x2)));
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[r][j][v] = 0.f;
}

// The weight pieces of one hidden layer held by this thread: rows n0 and
// n0 + 128 of W, k offset kq + 32 c for chunk c.
#define TT_W_LOAD(P, W, K, c)                                                                        \
  const uint4 P##a##c = *reinterpret_cast<const uint4*>((W) + n0 * (K) + kq + (c) * kWChunk);         \
  const uint4 P##b##c = *reinterpret_cast<const uint4*>((W) + (n0 + 128) * (K) + kq + (c) * kWChunk);
#define TT_W_LOAD8(P, W)                                                                            \
  TT_W_LOAD(P, W, 256, 0) TT_W_LOAD(P, W, 256, 1) TT_W_LOAD(P, W, 256, 2) TT_W_LOAD(P, W, 256, 3) \
  TT_W_LOAD(P, W, 256, 4) TT_W_LOAD(P, W, 256, 5) TT_W_LOAD(P, W, 256, 6) TT_W_LOAD(P, W, 256, 7)
#define TT_W_STORE(P, buf, c)                                                    \
  *reinterpret_cast<uint4*>(&Wc[((buf) * 256 + n0) * kWRow + kq]) = P##a##c;       \
  *reinterpret_cast<uint4*>(&Wc[((buf) * 256 + n0 + 128) * kWRow + kq]) = P##b##c;
#define TT_W_STEP(P, c, next)                                \
  infer_chunk(H, Wc, (c) & 1, c, acc, lane, cg, rg, hk);     \
  TT_W_STORE(P, ((c) + 1) & 1, next)                         \
  __syncthreads();
#define TT_W_LAYER256(P)                                                                                  \
  TT_W_STORE(P, 0, 0)                                                                                     \
  __syncthreads(); /* chunk 0, and the layer's inputs in H */                                             \
  TT_W_STEP(P, 0, 1) TT_W_STEP(P, 1, 2) TT_W_STEP(P, 2, 3) TT_W_STEP(P, 3, 4) TT_W_STEP(P, 4, 5)         \
  TT_W_STEP(P, 5, 6) TT_W_STEP(P, 6, 7)                                                                   \
  infer_chunk(H, Wc, 1, 7, acc, lane, cg, rg, hk);                                                        \
  __syncthreads(); /* every wave is done with H and the chunk buffers */

// One pass of the network over rows 0 .. rows - 1 (at most kInferRows) of
// the block: row r is candidate cand[r] (gated and list modes) or base + r.
// Ends with a barrier (the next pass overwrites H, the weight buffers and
// the biases).
__device__ __forceinline__ void infer_pass(const InferArgs& a, uint16_t* H, uint16_t* Wc, uint16_t* W4s, float* Bs,
                                           const int32_t* cand, int base, int rows) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cg = wave & 3, rg = wave >> 2;
  const int hk = 8 * (lane >> 5);  // k offset of this lane's 8 elements in a 16-k step
  const int n0 = tid >> 2, kq = 8 * (tid & 3);
  // features (one 16-byte piece per thread; rows past the block's are
  // zero), output-layer weights, biases and the first layer's weights: all
  // loads issued at once
  uint4 xv = make_uint4(0u, 0u, 0u, 0u), w4v = make_uint4(0u, 0u, 0u, 0u);
  if (a.x && (tid >> 2) < rows)
    xv = *reinterpret_cast<const uint4*>(a.x + (int64_t)(base + (tid >> 2)) * 32 + 8 * (tid & 3));
  if (tid < 384) w4v = *reinterpret_cast<const uint4*>(a.w[3] + (tid >> 5) * 256 + 8 * (tid & 31));
  float bv[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) bv[l] = (a.b[l] && tid < (l < 3 ? 256 : 12)) ? a.b[l][tid] : 0.f;
  TT_W_LOAD(L1, a.w[0], 32, 0)
  if (a.x) {
    *reinterpret_cast<uint4*>(&H[(tid >> 2) * kActRow + 8 * (tid & 3)]) = xv;
  } else if (tid < kInferRows) {  // one thread per row computes its features
    uint32_t pk[16] = {};
    if (tid < rows) neuron_features(a.desc + (cand ? cand[tid] : base + tid), pk);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      *reinterpret_cast<uint4*>(&H[tid * kActRow + 8 * k]) = make_uint4(pk[4 * k], pk[4 * k + 1], pk[4 * k + 2],
                                                                        pk[4 * k + 3]);
  }
  if (tid < 384) *reinterpret_cast<uint4*>(&W4s[(tid >> 5) * kActRow + 8 * (tid & 31)]) = w4v;
  if (tid < 256) {
#pragma unroll
    for (int l = 0; l < 4; ++l) Bs[256 * l + tid] = bv[l];
  }
  TT_W_STORE(L1, 0, 0)
  __syncthreads();
  f32x16 acc[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[r][j][v] = 0.f;
  infer_chunk(H, Wc, 0, 0, acc, lane, cg, rg, hk);  // layer 1: 32 inputs, one chunk
  TT_W_LOAD8(L2, a.w[1])  // layer 2's weights, in flight during layer 1's epilogue
  __syncthreads();        // every wave is done with H and chunk buffer 0
  infer_epilogue(acc, Bs, H, lane, cg, rg);
  TT_W_LAYER256(L2)
  TT_W_LOAD8(L3, a.w[2])
  infer_epilogue(acc, Bs + 256, H, lane, cg, rg);
  TT_W_LAYER256(L3)
  infer_epilogue(acc, Bs + 512, H, lane, cg, rg);
  __syncthreads();  // the last hidden layer's outputs are in H
  if (wave < 4) {
    const int mb = 32 * wave;
    const int wr = lane & 31;  // weight row = output column; rows 12.. are zero
    f32x16 o;
#pragma unroll
    for (int v = 0; v < 16; ++v) o[v] = 0.f;
    const bf16x8 zero = {};
#pragma unroll
    for (int k0 = 0; k0 < 256; k0 += 16) {
      const bf16x8 wf = wr < 12 ? *reinterpret_cast<const bf16x8*>(&W4s[wr * kActRow + k0 + hk]) : zero;
      const bf16x8 hf = *reinterpret_cast<const bf16x8*>(&H[(mb + (lane & 31)) * kActRow + k0 + hk]);
      o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf, hf, o, 0, 0, 0);
    }
    const int r = mb + (lane & 31);
    if (r < rows) {
      const int64_t m = cand ? cand[r] : base + r;  // logits row = candidate
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int n = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (n < 12) a.logits[m * 12 + n] = o[v] + Bs[768 + n];
      }
    }
  }
  __syncthreads();  // the next pass overwrites H, the weight buffers and the biases
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2))) void mlp_infer_kernel(InferArgs a) {
  extern __shared__ uint16_t lds[];
  __shared__ int32_t s_list[2 * kInferRows];  // gated: this block's candidates
  __shared__ int32_t s_wcnt[4];
  uint16_t* H = lds;                                            // [128][kActRow]
  uint16_t* Wc = lds + kInferRows * kActRow;                    // [2][256][kWRow]
  uint16_t* W4s = Wc + 2 * 256 * kWRow;                         // [12][kActRow]: output-layer weights
  float* Bs = reinterpret_cast<float*>(W4s + 12 * kActRow);     // [4][256]: biases (zero where NULL)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (a.list) {
    // list mode: the spans' counts to prefix sums (at most 8 spans per
    // thread), then chunks of kInferRows rows of the compacted list; row g
    // lies in the last span whose prefix is at most g (a span with rows)
    __shared__ int32_t s_pre[kGateMaxSpans + 1];
    __shared__ int32_t s_wsum[8];
    const int per = (a.nspans + 511) / 512;
    int loc[8], sum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int sp = tid * per + k;
      loc[k] = k < per && sp < a.nspans ? a.cnt[sp] : 0;
      sum += loc[k];
    }
    int incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    int run = incl - sum, total = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      run += w < wave ? s_wsum[w] : 0;
      total += s_wsum[w];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int sp = tid * per + k;
      if (k < per && sp < a.nspans) s_pre[sp] = run;
      run += loc[k];
    }
    __syncthreads();
    for (int c = blockIdx.x; c * kInferRows < total; c += gridDim.x) {
      const int rows = min(kInferRows, total - c * kInferRows);
      if (tid < rows) {
        const int g = c * kInferRows + tid;
        int lo = 0, hi = a.nspans - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[mid] <= g)
            lo = mid;
          else
            hi = mid - 1;
        }
        s_list[tid] = a.list[(size_t)lo * kGateSpan + (g - s_pre[lo])];
      }
      __syncthreads();
      infer_pass(a, H, Wc, W4s, Bs, s_list, 0, rows);
    }
    return;
  }
  // Rows of this block: feature rows / candidates base .. base + cnt, or
  // (gated) the candidates among 2 * kInferRows consecutive ones that the
  // wave pass takes, compacted into s_list in order.
  int base = blockIdx.x * kInferRows, cnt;
  if (a.gated) {
    base = blockIdx.x * 2 * kInferRows;
    const bool take = tid < 2 * kInferRows && base + tid < a.n && wave_pass_candidate(a.desc + base + tid);
    const uint64_t m = __ballot(take);
    if (lane == 0 && wave < 4) s_wcnt[wave] = (int32_t)__popcll(m);
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wave && w < 4; ++w) off += s_wcnt[w];
    if (take) s_list[off + __popcll(m & ((1ull << lane) - 1ull))] = base + tid;
    cnt = s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
    __syncthreads();
  } else {
    cnt = min(kInferRows, a.n - base);
  }
  if (cnt <= 0) return;  // block-uniform
  for (int p = 0; p < cnt; p += kInferRows)
    infer_pass(a, H, Wc, W4s, Bs, a.gated ? s_list + p : nullptr, base + p, min(kInferRows, cnt - p));
}

#undef TT_W_LAYER256
#undef TT_W_STEP
#undef TT_W_STORE
#undef TT_W_LOAD8
#undef TT_W_LOAD

hipError_t mlp_infer(const uint16_t* x, int n, const uint16_t* const* w, const float* const* b, float* logits,
                     hipStream_t s, const tt_neuron* desc, int gated) {
  if (n <= 0) return hipSuccess;
  const size_t lds =
      sizeof(uint16_t) * ((size_t)kInferRows * kActRow + 2 * 256 * kWRow + 12 * kActRow) + sizeof(float) * 4 * 256;
  // more than 64 KiB of dynamic LDS: allowed per launch (cheap host call, no
  // per-process state to keep consistent across devices or threads)
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_infer_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  InferArgs a{};
  a.x = x;
  a.n = n;
  for (int l = 0; l < 4; ++l) {
    a.w[l] = w[l];
    a.b[l] = b[l];
  }
  a.logits = logits;
  a.desc = desc;
  a.gated = desc && gated ? 1 : 0;
  const int per_block = a.gated ? 2 * kInferRows : kInferRows;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)((n + per_block - 1) / per_block)), dim3(512), lds, s, a);
  return hipGetLastError();
}

// The wave pass's candidates, compacted span by span: block b scans
// candidates b kGateSpan .. (b + 1) kGateSpan - 1 and writes the ones taken,
// in order, to list[b kGateSpan ...] and their number to cnt[b].
__global__ __launch_bounds__(kGateSpan) void infer_gate_list_kernel(const tt_neuron* desc, int n, int32_t* list,
                                                                    int32_t* cnt) {
  __shared__ int32_t s_wcnt[kGateSpan / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long i = (long)blockIdx.x * kGateSpan + tid;
  const bool take = i < n && wave_pass_candidate(desc + i);
  const uint64_t m = __ballot(take);
  if (lane == 0) s_wcnt[wave] = (int32_t)__popcll(m);
  __syncthreads();
  int off = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kGateSpan / 64; ++w) {
    off += w < wave ? s_wcnt[w] : 0;
    total += s_wcnt[w];
  }
  if (take) list[(long)blockIdx.x * kGateSpan + off + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)i;
  if (tid == 0) cnt[blockIdx.x] = total;
}

hipError_t mlp_infer_gated_list(const tt_neuron* desc, int n, const uint16_t* const* w, const float* const* b,
                                float* logits, int32_t* work, int blocks, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nspans = (n + kGateSpan - 1) / kGateSpan;
  if (nspans > kGateMaxSpans || blocks < 1) return hipErrorInvalidValue;
  int32_t* list = work;
  int32_t* cnt = work + (size_t)nspans * kGateSpan;
  hipLaunchKernelGGL(infer_gate_list_kernel, dim3((unsigned)nspans), dim3(kGateSpan), 0, s, desc, n, list, cnt);
  const size_t lds =
      sizeof(uint16_t) * ((size_t)kInferRows * kActRow + 2 * 256 * kWRow + 12 * kActRow) + sizeof(float) * 4 * 256;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_infer_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  InferArgs a{};
  a.n = n;
  for (int l = 0; l < 4; ++l) {
    a.w[l] = w[l];
    a.b[l] = b[l];
  }
  a.logits = logits;
  a.desc = desc;
  a.gated = 1;
  a.list = list;
  a.cnt = cnt;
  a.nspans = nspans;
  const int grid = (int)std::min<long>(blocks, ((long)n + kInferRows - 1) / kInferRows);
  hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)grid), dim3(512), lds, s, a);
  return hipGetLastError();
}

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
  const bool out_aligned = ((uintptr_t)yb % 16 == 0) && ((uintptr_t)yf % 16 == 0);
  // The persistent kernel gives each block all of W: worth it only when the
  // row tiles fill at least half the chip (inference batches); training
  // batches take the direct-operand kernel.
  int cus = 0;
  {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
  }
  const bool big = ((int64_t)(Bn + 63) / 64) * 2 / 8 >= cus / 2;
  if (big && aligned && out_aligned && Bn > 0 && out == kWideN && (in == 32 || in == 256)) {
    bool launched = false;
    const hipError_t e = in == 32 ? launch_fwd_persist<32>(g, s, &launched) : launch_fwd_persist<256>(g, s, &launched);
    if (e != hipSuccess || launched) return e;
  }
  if (big && aligned && Bn > 0 && out == kWideN && in % kWideKC == 0) {
    hipLaunchKernelGGL(gemm_fwd_wide_kernel, dim3((unsigned)((Bn + 63) / 64)), dim3(256), 0, s, g);
    return hipGetLastError();
  }
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
    // W^T padded to Kp columns at the start of the scratch (the weight
    // gradient below reuses the space after this product, in stream order)
    const int Kp = (out + 15) / 16 * 16;
    uint16_t* wt = reinterpret_cast<uint16_t*>(scratch);
    const bool al = ((uintptr_t)x % 8 == 0) && ((uintptr_t)dx % 8 == 0) && ((uintptr_t)dy % 2 == 0);
    if (scratch && al) {
      const int64_t tn = (int64_t)in * Kp;
      hipLaunchKernelGGL(transpose_pad_kernel, dim3((unsigned)((tn + 255) / 256)), dim3(256), 0, s, w, out, in, Kp, wt);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const int64_t waves = (int64_t)((Bn + 31) / 32) * ((in + 63) / 64);
      hipLaunchKernelGGL(gemm_dx_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, dy, out, wt, Kp,
                         mask_relu ? x : nullptr, Bn, in, dx);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if ((e = gemm(g, s)) != hipSuccess) {
      return e;
    }
  }
  if (dw || db) {
    const DwSplit sp = dw_split(Bn, out, in);
    float* part = scratch;
    float* dbp = scratch + (size_t)sp.S * out * in;
    dim3 grid((unsigned)((in + 63) / 64), (unsigned)((out + 63) / 64), (unsigned)sp.S);
    hipLaunchKernelGGL(gemm_dw_kernel, grid, dim3(256), 0, s, dy, x, Bn, out, in, sp.kslice, part,
                       db ? dbp : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t MN = (int64_t)out * in;
    const int64_t cover = std::max<int64_t>(dw ? MN : 0, out);
    hipLaunchKernelGGL(dw_reduce_kernel, dim3((unsigned)((cover + 255) / 256)), dim3(256), 0, s, part, dbp, sp.S, MN,
                       out, dw, db);
    e = hipGetLastError();
  }
  return e;
}

size_t mlp_backward_scratch_floats(int Bn, int dim) {
  const size_t S = (size_t)std::min(kDwMaxSlices, (Bn + kDwKC - 1) / kDwKC);
  const size_t wt = ((size_t)dim * ((dim + 15) / 16 * 16) + 1) / 2;  // W^T of the input gradient (bf16)
  return std::max(S * ((size_t)dim * dim + dim), wt);
}

hipError_t mlp_loss(const float* z, int Bn, const float* y, const float* m, const float* h, uint16_t* dz,
                    float* loss, float* scratch, hipStream_t s) {
  const int blocks = 64;
  hipLaunchKernelGGL(loss_kernel, dim3(blocks), dim3(256), 0, s, z, Bn, y, m, h, dz, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, s, scratch, blocks, Bn, loss);
  return hipGetLastError();
}

hipError_t adam_step_multi(int count, float* const* p, const float* const* g, float* const* m, float* const* v,
                           uint16_t* const* pb, const size_t* n, float lr, float b1, float b2, float eps, float bc1,
                           float bc2, hipStream_t s) {
  AdamMulti a{};
  a.count = count;
  a.off[0] = 0;
  for (int t = 0; t < count; ++t) {
    a.p[t] = p[t];
    a.g[t] = g[t];
    a.m[t] = m[t];
    a.v[t] = v[t];
    a.pb[t] = pb ? pb[t] : nullptr;
    a.off[t + 1] = a.off[t] + n[t];
  }
  const size_t total = a.off[count];
  if (total == 0) return hipSuccess;
  size_t blocks = (total + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(adam_multi_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, lr, b1, b2, eps, bc1, bc2);
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
