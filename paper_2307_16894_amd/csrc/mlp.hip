// Warm-start network: a fully connected SiLU network predicting the Newton
// increment of the reduced coordinates, with its own BF16 / FP32 forward,
// FP32 backward and Adam kernels.
//
// Parameters live on the device zero-padded per layer ([Kp][Np] weights,
// [Np] biases; Kp, Np multiples of 32 / 16) as an FP32 master copy plus a
// BF16 copy.  Padded rows and columns stay exactly zero: padded inputs are
// zero, padded output gradients are zero, and Adam leaves a zero-gradient
// zero-moment entry unchanged.
#include <math.h>
#include <string.h>

#include <type_traits>
#include <vector>

#include "rom_common.h"

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

struct rom_mlp {
  int device, n_in, width, n_out, max_batch;
  int K[4], N[4];          // padded fan-in / fan-out per layer
  int64_t off_w[4], off_b[4], npad;  // offsets in the padded parameter vector
  int64_t nparam;          // unpadded count (host layout)
  float* P;                // [npad] FP32 master (padded)
  uint16_t* Pb;            // [npad] BF16 copy
  uint16_t* WT;            // [npad] BF16 weights transposed per layer ([N][K] at off_w), for the fused inference
  int wt_stale;            // WT predates the last change of Pb
  float* Mo;               // [npad] Adam first moment
  float* Vo;               // [npad] Adam second moment
  float* G;                // [npad] gradient
  int64_t t;               // Adam step counter
  float *xm, *xs, *ym, *ys;  // scaling (device)
  float* A32[4];           // [B][K_l] layer inputs (FP32)
  uint16_t* A16[4];        // [B][K_l] layer inputs (BF16)
  float* Z[4];             // [B][N_l] pre-activations
  float* dZ;               // [B][max N]
  float* dA;               // [B][max K]
  float* loss_part;        // [grid] partial losses
  float* kpart;            // [MLP_KSPLIT][max K][max N] partial products of a split inner dimension
  float* cpart;            // [MLP_CSPLIT][max N] partial column sums
  double* spart;           // [MLP_SSPLIT][n_in + n_out] partial sample moments
  float* loss_one;         // loss of one minibatch (epoch training)
};

namespace {

constexpr int MLP_KSPLIT = 16;  // most slices of a split inner dimension
constexpr int MLP_CSPLIT = 32;  // row slices of the bias-gradient column sum
constexpr int MLP_SSPLIT = 64;  // row slices of the sample moments (input / output scaling)

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// C[M][N] (ldc) = sum_k A(m, k) B(k, n) (+ bias[n]); A(m, k) = A[m * sa0 + k * sa1],
// B(k, n) = B[k * sb0 + n * sb1], one of sa0 / sa1 and one of sb0 / sb1 equal
// to 1 (row-major or transposed operands).  Workgroup tile TM x TM (64: wave
// tile 32 x 32 of 2 x 2 MFMA tiles of 16 x 16; 32: one 16 x 16 MFMA tile per
// wave, four times the workgroups for the small grids of the training
// products); per step of 32 inner indices the two operand tiles are loaded
// into LDS with TM / 8 contiguous elements per thread along whichever index is
// contiguous in memory, A as [m][k] and B as [n][k], so that each lane's MFMA
// operand is one LDS read.  Out-of-range operands read as zero.  The MFMA
// operands sit in the lanes and the inner index runs in the order of the
// per-lane global form this replaced (BF16: k = k0 + 8 g + t; FP32:
// k = k0 + 4 s + g), whatever the tile, so the products are the same bit for
// bit.  With gridDim.z > 1 workgroup z sums k in [z kchunk, (z + 1) kchunk)
// only and writes its product to C + z cstride (kchunk a multiple of 32).
constexpr int GM_K = 32;

template <bool BF16, int TM>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const void* __restrict__ Av, long sa0, long sa1,
                                              const void* __restrict__ Bv, long sb0, long sb1, float* __restrict__ C,
                                              long ldc, const float* __restrict__ bias, int kchunk, long cstride) {
  using E = typename std::conditional<BF16, uint16_t, float>::type;
  constexpr int LDK = GM_K + (BF16 ? 8 : 4);  // padded row (16 bytes)
  constexpr int TW = TM / 32;                 // MFMA tiles per wave and dimension
  constexpr int EL = TM / 8;                  // elements loaded per thread and operand
  __shared__ __attribute__((aligned(16))) E sA[TM * LDK];
  __shared__ __attribute__((aligned(16))) E sB[TM * LDK];
  const E* A = static_cast<const E*>(Av);
  const E* B = static_cast<const E*>(Bv);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  C += blockIdx.z * cstride;
  const int g = lane >> 4, c = lane & 15;
  const int mt = blockIdx.y * TM, nt = blockIdx.x * TM;
  const int mw = (wave >> 1) * 16 * TW, nw = (wave & 1) * 16 * TW;
  f4 acc[TW][TW];
#pragma unroll
  for (int i = 0; i < TW; ++i)
#pragma unroll
    for (int j = 0; j < TW; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
  // thread t loads EL contiguous elements: along k (row r = t / (32 / EL),
  // k = EL (t % (32 / EL))) or along m / n (k = t / (TM / EL), row EL (t % (TM / EL)))
  const bool a_k = (sa1 == 1), b_k = (sb0 == 1);
  constexpr int KG = GM_K / EL, RG = TM / EL;
  for (int k0 = kb; k0 < ke; k0 += GM_K) {
    {
      const int r = a_k ? tid / KG : EL * (tid % RG), kk = a_k ? EL * (tid % KG) : tid / RG;
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int rr = a_k ? r : r + e, ki = a_k ? kk + e : kk;
        const int m = mt + rr, k = k0 + ki;
        sA[rr * LDK + ki] = (m < M && k < ke) ? A[m * sa0 + k * sa1] : (E)0;
      }
    }
    {
      const int r = b_k ? tid / KG : EL * (tid % RG), kk = b_k ? EL * (tid % KG) : tid / RG;
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int rr = b_k ? r : r + e, ki = b_k ? kk + e : kk;
        const int n = nt + rr, k = k0 + ki;
        sB[rr * LDK + ki] = (n < N && k < ke) ? B[k * sb0 + n * sb1] : (E)0;
      }
    }
    __syncthreads();
    if constexpr (BF16) {
      bf8 a[TW], b[TW];
#pragma unroll
      for (int i = 0; i < TW; ++i) a[i] = *reinterpret_cast<const bf8*>(sA + (mw + 16 * i + c) * LDK + 8 * g);
#pragma unroll
      for (int j = 0; j < TW; ++j) b[j] = *reinterpret_cast<const bf8*>(sB + (nw + 16 * j + c) * LDK + 8 * g);
#pragma unroll
      for (int i = 0; i < TW; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int st = 0; st < GM_K / 4; ++st) {
        float a[TW], b[TW];
#pragma unroll
        for (int i = 0; i < TW; ++i) a[i] = sA[(mw + 16 * i + c) * LDK + 4 * st + g];
#pragma unroll
        for (int j = 0; j < TW; ++j) b[j] = sB[(nw + 16 * j + c) * LDK + 4 * st + g];
#pragma unroll
        for (int i = 0; i < TW; ++i)
#pragma unroll
          for (int j = 0; j < TW; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // accumulator layout of the 16 x 16 f32-output MFMAs: row 4 g + r, column c
#pragma unroll
  for (int i = 0; i < TW; ++i)
#pragma unroll
    for (int j = 0; j < TW; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mt + mw + 16 * i + 4 * g + r, n = nt + nw + 16 * j + c;
        if (m < M && n < N) C[m * ldc + n] = acc[i][j][r] + (bias ? bias[n] : 0.f);
      }
}

// layer input: x_hat = (x - mean) / std, zero padded to K0 columns; row b of
// the batch is row idx[b] of X (idx null: row b)
__global__ void k_scale_in(int B, int n_in, int K0, const float* __restrict__ X, const int* __restrict__ idx,
                           const float* __restrict__ xm, const float* __restrict__ xs, float* __restrict__ A32,
                           uint16_t* __restrict__ A16) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * K0) return;
  const int b = (int)(i / K0), k = (int)(i % K0);
  const long row = idx ? idx[b] : b;
  const float v = (k < n_in) ? (X[row * n_in + k] - xm[k]) / xs[k] : 0.f;
  A32[i] = v;
  A16[i] = bf16_bits(v);
}

// next layer input a = silu(z)
__global__ void k_silu(long count, const float* __restrict__ Z, float* __restrict__ A32, uint16_t* __restrict__ A16) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float v = silu_f(Z[i]);
  A32[i] = v;
  A16[i] = bf16_bits(v);
}

// raw prediction y = y_mean + y_std * z
__global__ void k_scale_out(int B, int n_out, int Np, const float* __restrict__ Z, const float* __restrict__ ym,
                            const float* __restrict__ ys, float* __restrict__ Y) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * n_out) return;
  const int b = (int)(i / n_out), k = (int)(i % n_out);
  Y[i] = ym[k] + ys[k] * Z[(long)b * Np + k];
}

// dLoss/dout = 2 (out - y_hat) / B on the real outputs, 0 on padding; partial losses per block
__global__ __launch_bounds__(256) void k_loss(int B, int n_out, int Np, const float* __restrict__ Z,
                                              const float* __restrict__ Y, const int* __restrict__ idx,
                                              const float* __restrict__ ym, const float* __restrict__ ys,
                                              float* __restrict__ dZ, float* __restrict__ part) {
  __shared__ float red[256];
  const long i = blockIdx.x * 256L + threadIdx.x;
  float l = 0.f;
  if (i < (long)B * Np) {
    const int b = (int)(i / Np), k = (int)(i % Np);
    const long row = idx ? idx[b] : b;
    float d = 0.f;
    if (k < n_out) {
      const float e = Z[i] - (Y[row * n_out + k] - ym[k]) / ys[k];
      l = e * e;
      d = 2.f * e / (float)B;
    }
    dZ[i] = d;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_zero_f32(float* __restrict__ x) {
  if (threadIdx.x == 0) x[0] = 0.f;
}
__global__ void k_add_f32(float* __restrict__ sum, const float* __restrict__ x) {
  if (threadIdx.x == 0) sum[0] += x[0];
}

// Column moments of the samples (columns 0 .. n_in - 1 of X, then n_out of
// Y), lane = column, the waves and the grid's y dimension slicing the rows:
// pass 0 the sum, pass 1 the sum of squared deviations from the mean, as
// FP64 partials [slice][column] added in slice order by k_col_finish.
__global__ __launch_bounds__(256) void k_col_moments(int N, int n_in, int n_out, const float* __restrict__ X,
                                                     const float* __restrict__ Y, int pass,
                                                     const float* __restrict__ xm, const float* __restrict__ ym,
                                                     double* __restrict__ part) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane, nc = n_in + n_out;
  const int S = gridDim.y, y = blockIdx.y;
  const long r0 = (long)N * y / S, r1 = (long)N * (y + 1) / S;
  double acc = 0.0;
  if (c < nc) {
    const bool isx = c < n_in;
    const float* src = isx ? X + c : Y + (c - n_in);
    const long ld = isx ? n_in : n_out;
    const double mean = pass ? (double)(isx ? xm[c] : ym[c - n_in]) : 0.0;
    for (long r = r0 + wave; r < r1; r += 4) {
      const double v = (double)src[r * ld] - mean;
      acc += pass ? v * v : v;
    }
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && c < nc) part[(long)y * nc + c] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// pass 0: mean = sum / N; pass 1: std = sqrt(sum of squares / (N - 1)), 1
// where it is below 1e-12 (a constant column)
__global__ void k_col_finish(int N, int n_in, int n_out, int pass, const double* __restrict__ part,
                             float* __restrict__ xm, float* __restrict__ xs, float* __restrict__ ym,
                             float* __restrict__ ys) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, nc = n_in + n_out;
  if (c >= nc) return;
  double t = 0.0;
  for (int y = 0; y < MLP_SSPLIT; ++y) t += part[(long)y * nc + c];
  if (pass == 0) {
    const float mean = (float)(t / N);
    if (c < n_in)
      xm[c] = mean;
    else
      ym[c - n_in] = mean;
  } else {
    const double sd = sqrt(t / (N - 1));
    const float v = sd > 1e-12 ? (float)sd : 1.0f;
    if (c < n_in)
      xs[c] = v;
    else
      ys[c - n_in] = v;
  }
}

// one workgroup of 256: strided partial sums, then a fixed-order tree
__global__ __launch_bounds__(256) void k_loss_final(int nblocks, int B, const float* __restrict__ part,
                                                    float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < nblocks; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (float)B;
}

// dZ = dA * silu'(Z)
__global__ void k_dsilu(long count, const float* __restrict__ dA, const float* __restrict__ Z,
                        float* __restrict__ dZ) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= count) return;
  dZ[i] = dA[i] * dsilu_f(Z[i]);
}

// partial column sums part[y][n] = sum of dZ[b][n] over the rows of slice y
// (gridDim.y slices of the batch); lanes take 64 consecutive columns, the
// four waves every fourth row, added in a fixed order
__global__ __launch_bounds__(256) void k_colsum_part(int B, int N, const float* __restrict__ dZ,
                                                     float* __restrict__ part) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n = blockIdx.x * 64 + lane;
  const int rows = (B + gridDim.y - 1) / gridDim.y, b0 = blockIdx.y * rows, b1 = min(B, b0 + rows);
  float s = 0.f;
  if (n < N)
    for (int b = b0 + wave; b < b1; b += 4) s += dZ[(long)b * N + n];
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && n < N) part[(long)blockIdx.y * N + n] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// out[i] = sum over s < S of part[s * stride + i], in order of s
__global__ void k_sum_slices(long count, int S, long stride, const float* __restrict__ part,
                             float* __restrict__ out) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= count) return;
  float s = 0.f;
  for (int z = 0; z < S; ++z) s += part[z * stride + i];
  out[i] = s;
}

__global__ void k_adam(long count, float* __restrict__ P, uint16_t* __restrict__ Pb, float* __restrict__ Mo,
                       float* __restrict__ Vo, const float* __restrict__ G, float lr, float c1, float c2) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float g = G[i];
  const float m = 0.9f * Mo[i] + 0.1f * g;
  const float v = 0.999f * Vo[i] + 0.001f * g * g;
  Mo[i] = m;
  Vo[i] = v;
  const float p = P[i] - lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
  P[i] = p;
  Pb[i] = bf16_bits(p);
}

// Fused BF16 inference (padded input and hidden widths up to MI_KMAX): one
// workgroup per MI_ROWS batch rows runs the four layers with the layer inputs
// in LDS as BF16.  Per output tile it issues the layer-by-layer path's MFMA
// with the same operands in the same lanes and the same inner-index order
// (k = k0 + 8 g + t), then adds the bias, applies SiLU and rounds to BF16 as
// that path's kernels do: the predictions are the same bit for bit.  The
// weights come from the transposed copy WT, so a lane's eight inner indices
// are one 16-byte load.
constexpr int MI_ROWS = 16, MI_KMAX = 256, MI_LDA = MI_KMAX + 8;  // LDS row stride: 16 bytes of padding

struct MlpLayout {
  int K[4], N[4];
  long off_w[4], off_b[4];
};

__global__ __launch_bounds__(256) void k_mlp_infer(int B, int n_in, int n_out, MlpLayout d,
                                                   const float* __restrict__ X, const float* __restrict__ xm,
                                                   const float* __restrict__ xs, const uint16_t* __restrict__ WT,
                                                   const float* __restrict__ P, const float* __restrict__ ym,
                                                   const float* __restrict__ ys, float* __restrict__ Y) {
  __shared__ __attribute__((aligned(16))) uint16_t act[2][MI_ROWS * MI_LDA];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int row0 = blockIdx.x * MI_ROWS;
  // scaled input x_hat = (x - mean) / std, zero padded
  for (int i = tid; i < MI_ROWS * d.K[0]; i += 256) {
    const int r = i / d.K[0], k = i - r * d.K[0], row = row0 + r;
    const float v = (row < B && k < n_in) ? (X[(long)row * n_in + k] - xm[k]) / xs[k] : 0.f;
    act[0][r * MI_LDA + k] = bf16_bits(v);
  }
  __syncthreads();
  for (int l = 0; l < 4; ++l) {
    const int K = d.K[l], N = d.N[l], NT = N / 16;
    const uint16_t* Ain = act[l & 1];
    uint16_t* Aout = act[(l + 1) & 1];
    const uint16_t* W = WT + d.off_w[l];
    const float* bias = P + d.off_b[l];
    f4 acc[MI_KMAX / 64];
#pragma unroll
    for (int u = 0; u < MI_KMAX / 64; ++u) acc[u] = (f4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
      const bf8 a = *reinterpret_cast<const bf8*>(Ain + c * MI_LDA + k0 + 8 * g);
#pragma unroll
      for (int u = 0; u < MI_KMAX / 64; ++u) {
        const int t = wave + 4 * u;  // column tiles dealt to the waves in turn
        if (t < NT) {
          const bf8 b = *reinterpret_cast<const bf8*>(W + (long)(16 * t + c) * K + k0 + 8 * g);
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[u], 0, 0, 0);
        }
      }
    }
    // accumulator layout: row 4 g + r, column c of the tile
#pragma unroll
    for (int u = 0; u < MI_KMAX / 64; ++u) {
      const int t = wave + 4 * u;
      if (t >= NT) continue;
      const int n = 16 * t + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = 4 * g + r;
        const float z = acc[u][r] + bias[n];
        if (l < 3) {
          Aout[rr * MI_LDA + n] = bf16_bits(silu_f(z));
        } else if (n < n_out && row0 + rr < B) {
          Y[(long)(row0 + rr) * n_out + n] = ym[n] + ys[n] * z;
        }
      }
    }
    __syncthreads();
  }
}

// WT[l][n][k] = Pb[l][k][n]
__global__ void k_transpose_w(MlpLayout d, const uint16_t* __restrict__ Pb, uint16_t* __restrict__ WT) {
  const int l = blockIdx.y;
  const long count = (long)d.K[l] * d.N[l];
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int n = (int)(i / d.K[l]), k = (int)(i - (long)n * d.K[l]);
  WT[d.off_w[l] + i] = Pb[d.off_w[l] + (long)k * d.N[l] + n];
}

__global__ void k_to_bf16(long count, const float* __restrict__ P, uint16_t* __restrict__ Pb) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < count) Pb[i] = bf16_bits(P[i]);
}

inline unsigned nblk(long count, int bs = 256) { return (unsigned)((count + bs - 1) / bs); }

// output tile: 64 x 64 while that fills the compute units, else 32 x 32
inline bool gemm_small_tiles(int M, int N) { return (long)((N + 63) / 64) * ((M + 63) / 64) < 256; }

template <bool BF16>
void gemm(int M, int N, int K, const void* A, long sa0, long sa1, const void* B, long sb0, long sb1, float* C,
          long ldc, const float* bias, hipStream_t s) {
  if (gemm_small_tiles(M, N)) {
    dim3 grid((N + 31) / 32, (M + 31) / 32);
    k_gemm<BF16, 32><<<grid, 256, 0, s>>>(M, N, K, A, sa0, sa1, B, sb0, sb1, C, ldc, bias, K + 31, 0);
  } else {
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    k_gemm<BF16, 64><<<grid, 256, 0, s>>>(M, N, K, A, sa0, sa1, B, sb0, sb1, C, ldc, bias, K + 31, 0);
  }
}

// C[M][N] (dense, ldc = N, no bias) with a long inner dimension: the grid of
// output tiles is small, so the inner dimension is split into slices whose
// products land in kpart and are then added in slice order
void gemm_split(rom_mlp* m, int M, int N, int K, const float* A, long sa0, long sa1, const float* B, long sb0,
                long sb1, float* C, hipStream_t s) {
  const bool small = gemm_small_tiles(M, N);
  const int TM = small ? 32 : 64;
  const int tiles = ((N + TM - 1) / TM) * ((M + TM - 1) / TM);
  int S = (256 + tiles - 1) / tiles;
  S = S < K / 128 ? S : K / 128;
  S = S < MLP_KSPLIT ? S : MLP_KSPLIT;
  if (S <= 1) {
    gemm<false>(M, N, K, A, sa0, sa1, B, sb0, sb1, C, N, nullptr, s);
    return;
  }
  const int kchunk = ((K + S - 1) / S + 31) / 32 * 32;
  S = (K + kchunk - 1) / kchunk;
  dim3 grid((N + TM - 1) / TM, (M + TM - 1) / TM, S);
  if (small)
    k_gemm<false, 32><<<grid, 256, 0, s>>>(M, N, K, A, sa0, sa1, B, sb0, sb1, m->kpart, N, nullptr, kchunk, (long)M * N);
  else
    k_gemm<false, 64><<<grid, 256, 0, s>>>(M, N, K, A, sa0, sa1, B, sb0, sb1, m->kpart, N, nullptr, kchunk, (long)M * N);
  k_sum_slices<<<nblk((long)M * N), 256, 0, s>>>((long)M * N, S, (long)M * N, m->kpart, C);
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void mlp_release(rom_mlp* m) {
  if (!m) return;
  void* bufs[] = {m->P, m->Pb, m->WT, m->Mo, m->Vo, m->G, m->xm, m->xs, m->ym, m->ys, m->dZ, m->dA, m->loss_part,
                  m->kpart, m->cpart, m->spart, m->loss_one};
  for (void* b : bufs) (void)hipFree(b);
  for (int l = 0; l < 4; ++l) {
    (void)hipFree(m->A32[l]);
    (void)hipFree(m->A16[l]);
    (void)hipFree(m->Z[l]);
  }
  delete m;
}

// forward from the scaled input already in A32[0] / A16[0]; output pre-activations in Z[3]
int mlp_forward_scaled(rom_mlp* m, int B, int prec, hipStream_t s) {
  for (int l = 0; l < 4; ++l) {
    const int K = m->K[l], N = m->N[l];
    if (prec == ROM_DT_BF16)
      gemm<true>(B, N, K, m->A16[l], K, 1, m->Pb + m->off_w[l], N, 1, m->Z[l], N, m->P + m->off_b[l], s);
    else
      gemm<false>(B, N, K, m->A32[l], K, 1, m->P + m->off_w[l], N, 1, m->Z[l], N, m->P + m->off_b[l], s);
    if (l < 3) k_silu<<<nblk((long)B * N), 256, 0, s>>>((long)B * N, m->Z[l], m->A32[l + 1], m->A16[l + 1]);
  }
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int mlp_gradients(rom_mlp* m, int B, const float* X, const float* Y, const int* idx, int prec, float* loss,
                  hipStream_t s) {
  k_scale_in<<<nblk((long)B * m->K[0]), 256, 0, s>>>(B, m->n_in, m->K[0], X, idx, m->xm, m->xs, m->A32[0],
                                                     m->A16[0]);
  int rc = mlp_forward_scaled(m, B, prec, s);
  if (rc != ROM_OK) return rc;
  const int Np = m->N[3];
  const unsigned nb = nblk((long)B * Np);
  k_loss<<<nb, 256, 0, s>>>(B, m->n_out, Np, m->Z[3], Y, idx, m->ym, m->ys, m->dZ, m->loss_part);
  if (loss) k_loss_final<<<1, 256, 0, s>>>((int)nb, B, m->loss_part, loss);
  for (int l = 3; l >= 0; --l) {
    const int K = m->K[l], N = m->N[l];
    if (l < 3) k_dsilu<<<nblk((long)B * N), 256, 0, s>>>((long)B * N, m->dA, m->Z[l], m->dZ);
    // dW = A^T dZ  (M = K, N = N, inner = B)
    gemm_split(m, K, N, B, m->A32[l], 1, K, m->dZ, N, 1, m->G + m->off_w[l], s);
    const int cs = B / 64 < MLP_CSPLIT ? (B / 64 > 0 ? B / 64 : 1) : MLP_CSPLIT;
    k_colsum_part<<<dim3((N + 63) / 64, cs), 256, 0, s>>>(B, N, m->dZ, m->cpart);
    k_sum_slices<<<nblk(N), 256, 0, s>>>(N, cs, N, m->cpart, m->G + m->off_b[l]);
    // dA_prev = dZ W^T  (M = B, N = K, inner = N)
    if (l > 0) gemm<false>(B, K, N, m->dZ, N, 1, m->P + m->off_w[l], 1, N, m->dA, K, nullptr, s);
  }
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int mlp_train_step(rom_mlp* m, int B, const float* X, const float* Y, const int* idx, float lr, int prec,
                   float* loss, hipStream_t s) {
  int rc = mlp_gradients(m, B, X, Y, idx, prec, loss, s);
  if (rc != ROM_OK) return rc;
  m->t += 1;
  const float c1 = 1.0f - powf(0.9f, (float)m->t), c2 = 1.0f - powf(0.999f, (float)m->t);
  k_adam<<<nblk(m->npad), 256, 0, s>>>(m->npad, m->P, m->Pb, m->Mo, m->Vo, m->G, lr, c1, c2);
  m->wt_stale = 1;
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

}  // namespace

extern "C" {

int rom_mlp_create(int32_t n_in, int32_t width, int32_t n_out, int32_t max_batch, int device, rom_mlp_handle* out) {
  if (!out || n_in < 1 || n_in > 1024 || width < 16 || width > 1024 || width % 32 || n_out < 1 || n_out > 1024 ||
      max_batch < 1 || max_batch > (1 << 20))
    return ROM_EINVAL;
  *out = nullptr;
  DeviceGuard guard(device);
  rom_mlp* m = new rom_mlp();
  memset(m, 0, sizeof(*m));
  m->device = device;
  m->n_in = n_in;
  m->width = width;
  m->n_out = n_out;
  m->max_batch = max_batch;
  const int K0 = (n_in + 31) / 32 * 32, No = (n_out + 15) / 16 * 16;
  const int Ks[4] = {K0, width, width, width}, Ns[4] = {width, width, width, No};
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    m->K[l] = Ks[l];
    m->N[l] = Ns[l];
    m->off_w[l] = o;
    o += (int64_t)Ks[l] * Ns[l];
    m->off_b[l] = o;
    o += Ns[l];
  }
  m->npad = o;
  m->nparam = (int64_t)n_in * width + width + 2 * ((int64_t)width * width + width) + (int64_t)width * n_out + n_out;
  bool ok = true;
  auto al = [&](void** p, size_t bytes) {
    if (ok && hipMalloc(p, bytes) != hipSuccess) ok = false;
    if (ok && hipMemset(*p, 0, bytes) != hipSuccess) ok = false;
  };
  al((void**)&m->P, 4 * o);
  al((void**)&m->Pb, 2 * o);
  al((void**)&m->WT, 2 * o);
  m->wt_stale = 1;
  al((void**)&m->Mo, 4 * o);
  al((void**)&m->Vo, 4 * o);
  al((void**)&m->G, 4 * o);
  al((void**)&m->xm, 4 * K0);
  al((void**)&m->xs, 4 * K0);
  al((void**)&m->ym, 4 * No);
  al((void**)&m->ys, 4 * No);
  const int maxKN = width > No ? (width > K0 ? width : K0) : No;
  for (int l = 0; l < 4; ++l) {
    al((void**)&m->A32[l], 4L * max_batch * Ks[l]);
    al((void**)&m->A16[l], 2L * max_batch * Ks[l]);
    al((void**)&m->Z[l], 4L * max_batch * Ns[l]);
  }
  al((void**)&m->dZ, 4L * max_batch * maxKN);
  al((void**)&m->dA, 4L * max_batch * maxKN);
  al((void**)&m->loss_part, 4L * ((long)max_batch * No / 256 + 2));
  long maxKxN = 0;
  for (int l = 0; l < 4; ++l) maxKxN = maxKxN > (long)Ks[l] * Ns[l] ? maxKxN : (long)Ks[l] * Ns[l];
  al((void**)&m->kpart, 4L * MLP_KSPLIT * maxKxN);
  al((void**)&m->cpart, 4L * MLP_CSPLIT * maxKN);
  al((void**)&m->spart, 8L * MLP_SSPLIT * (n_in + n_out));
  al((void**)&m->loss_one, 4L);
  if (!ok) {
    mlp_release(m);
    return ROM_EHIP;
  }
  // unit scaling until set
  std::vector<float> ones(K0 > No ? K0 : No, 1.0f);
  (void)hipMemcpy(m->xs, ones.data(), 4 * K0, hipMemcpyHostToDevice);
  (void)hipMemcpy(m->ys, ones.data(), 4 * No, hipMemcpyHostToDevice);
  *out = m;
  return ROM_OK;
}

int rom_mlp_free(rom_mlp_handle m) {
  if (!m) return ROM_EINVAL;
  DeviceGuard guard(m->device);
  mlp_release(m);
  return ROM_OK;
}

int rom_mlp_param_count(rom_mlp_handle m, int64_t* count) {
  if (!m || !count) return ROM_EINVAL;
  *count = m->nparam;
  return ROM_OK;
}

int rom_mlp_set_params(rom_mlp_handle m, const float* host, int64_t count) {
  if (!m || !host || count != m->nparam) return ROM_EINVAL;
  DeviceGuard guard(m->device);
  std::vector<float> pad(m->npad, 0.0f);
  const int fi[4] = {m->n_in, m->width, m->width, m->width}, fo[4] = {m->width, m->width, m->width, m->n_out};
  int64_t src = 0;
  for (int l = 0; l < 4; ++l) {
    for (int i = 0; i < fi[l]; ++i)
      for (int j = 0; j < fo[l]; ++j) pad[m->off_w[l] + (int64_t)i * m->N[l] + j] = host[src++];
    for (int j = 0; j < fo[l]; ++j) pad[m->off_b[l] + j] = host[src++];
  }
  if (hipMemcpy(m->P, pad.data(), 4 * m->npad, hipMemcpyHostToDevice) != hipSuccess) return ROM_EHIP;
  k_to_bf16<<<nblk(m->npad), 256>>>(m->npad, m->P, m->Pb);
  m->wt_stale = 1;
  if (hipMemset(m->Mo, 0, 4 * m->npad) != hipSuccess || hipMemset(m->Vo, 0, 4 * m->npad) != hipSuccess)
    return ROM_EHIP;
  m->t = 0;
  return hipDeviceSynchronize() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_mlp_get_params(rom_mlp_handle m, float* host, int64_t count) {
  if (!m || !host || count != m->nparam) return ROM_EINVAL;
  DeviceGuard guard(m->device);
  std::vector<float> pad(m->npad);
  if (hipDeviceSynchronize() != hipSuccess) return ROM_EHIP;
  if (hipMemcpy(pad.data(), m->P, 4 * m->npad, hipMemcpyDeviceToHost) != hipSuccess) return ROM_EHIP;
  const int fi[4] = {m->n_in, m->width, m->width, m->width}, fo[4] = {m->width, m->width, m->width, m->n_out};
  int64_t dst = 0;
  for (int l = 0; l < 4; ++l) {
    for (int i = 0; i < fi[l]; ++i)
      for (int j = 0; j < fo[l]; ++j) host[dst++] = pad[m->off_w[l] + (int64_t)i * m->N[l] + j];
    for (int j = 0; j < fo[l]; ++j) host[dst++] = pad[m->off_b[l] + j];
  }
  return ROM_OK;
}

int rom_mlp_set_scaling(rom_mlp_handle m, const float* xm, const float* xs, const float* ym, const float* ys) {
  if (!m || !xm || !xs || !ym || !ys) return ROM_EINVAL;
  for (int i = 0; i < m->n_in; ++i)
    if (!(xs[i] > 0) || !isfinite(xm[i])) return ROM_EINVAL;
  for (int i = 0; i < m->n_out; ++i)
    if (!(ys[i] > 0) || !isfinite(ym[i])) return ROM_EINVAL;
  DeviceGuard guard(m->device);
  bool ok = hipMemcpy(m->xm, xm, 4 * m->n_in, hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(m->xs, xs, 4 * m->n_in, hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(m->ym, ym, 4 * m->n_out, hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(m->ys, ys, 4 * m->n_out, hipMemcpyHostToDevice) == hipSuccess;
  return ok ? ROM_OK : ROM_EHIP;
}

int rom_mlp_forward(rom_mlp_handle m, int32_t B, const float* X, float* Y, int32_t prec, hipStream_t s) {
  if (!m || B < 0 || B > m->max_batch || (prec != ROM_DT_F32 && prec != ROM_DT_BF16)) return ROM_EINVAL;
  if (B == 0) return ROM_OK;
  if (!X || !Y) return ROM_EINVAL;
  DeviceGuard guard(m->device);
  if (prec == ROM_DT_BF16 && m->K[0] <= MI_KMAX && m->width <= MI_KMAX && m->N[3] <= MI_KMAX) {
    MlpLayout d;
    for (int l = 0; l < 4; ++l) {
      d.K[l] = m->K[l];
      d.N[l] = m->N[l];
      d.off_w[l] = m->off_w[l];
      d.off_b[l] = m->off_b[l];
    }
    if (m->wt_stale) {
      long most = 0;
      for (int l = 0; l < 4; ++l) most = most > (long)d.K[l] * d.N[l] ? most : (long)d.K[l] * d.N[l];
      k_transpose_w<<<dim3(nblk(most), 4), 256, 0, s>>>(d, m->Pb, m->WT);
      m->wt_stale = 0;
    }
    k_mlp_infer<<<(B + MI_ROWS - 1) / MI_ROWS, 256, 0, s>>>(B, m->n_in, m->n_out, d, X, m->xm, m->xs, m->WT, m->P,
                                                           m->ym, m->ys, Y);
    return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
  }
  k_scale_in<<<nblk((long)B * m->K[0]), 256, 0, s>>>(B, m->n_in, m->K[0], X, nullptr, m->xm, m->xs, m->A32[0],
                                                     m->A16[0]);
  int rc = mlp_forward_scaled(m, B, prec, s);
  if (rc != ROM_OK) return rc;
  k_scale_out<<<nblk((long)B * m->n_out), 256, 0, s>>>(B, m->n_out, m->N[3], m->Z[3], m->ym, m->ys, Y);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_mlp_infer(rom_mlp_handle m, int32_t B, const float* X, float* Y, int32_t prec, hipStream_t s) {
  return rom_mlp_forward(m, B, X, Y, prec, s);
}

// Network artifact: "PODECMN1", u32 version 1, n_in, width, n_out, u32 pad,
// then f32 x_mean [n_in], x_std [n_in], y_mean [n_out], y_std [n_out] and the
// parameters in the host layout of rom_mlp_set_params.
static size_t mlp_blob_bytes(int n_in, int width, int n_out, int64_t nparam) {
  return 32 + 4 * (2 * (size_t)n_in + 2 * (size_t)n_out + (size_t)nparam);
}

int rom_mlp_save(rom_mlp_handle m, void* blob, size_t capacity, size_t* bytes) {
  if (!m || !bytes) return ROM_EINVAL;
  const size_t need = mlp_blob_bytes(m->n_in, m->width, m->n_out, m->nparam);
  *bytes = need;
  if (!blob) return ROM_OK;
  if (capacity < need) return ROM_EINVAL;
  DeviceGuard guard(m->device);
  unsigned char* b = static_cast<unsigned char*>(blob);
  memset(b, 0, 32);
  memcpy(b, "PODECMN1", 8);
  const uint32_t hdr[4] = {1u, (uint32_t)m->n_in, (uint32_t)m->width, (uint32_t)m->n_out};
  memcpy(b + 8, hdr, sizeof(hdr));
  float* f = reinterpret_cast<float*>(b + 32);
  if (hipDeviceSynchronize() != hipSuccess) return ROM_EHIP;
  bool ok = hipMemcpy(f, m->xm, 4 * m->n_in, hipMemcpyDeviceToHost) == hipSuccess;
  ok = ok && hipMemcpy(f + m->n_in, m->xs, 4 * m->n_in, hipMemcpyDeviceToHost) == hipSuccess;
  ok = ok && hipMemcpy(f + 2 * m->n_in, m->ym, 4 * m->n_out, hipMemcpyDeviceToHost) == hipSuccess;
  ok = ok && hipMemcpy(f + 2 * m->n_in + m->n_out, m->ys, 4 * m->n_out, hipMemcpyDeviceToHost) == hipSuccess;
  if (!ok) return ROM_EHIP;
  return rom_mlp_get_params(m, f + 2 * m->n_in + 2 * m->n_out, m->nparam);
}

int rom_mlp_load(const void* blob, size_t bytes, int32_t max_batch, int device, rom_mlp_handle* out) {
  if (!blob || !out) return ROM_EINVAL;
  *out = nullptr;
  const unsigned char* b = static_cast<const unsigned char*>(blob);
  if (bytes < 32 || memcmp(b, "PODECMN1", 8) != 0) return ROM_EFORMAT;
  uint32_t hdr[4];
  memcpy(hdr, b + 8, sizeof(hdr));
  if (hdr[0] != 1) return ROM_EVERSION;
  const int n_in = (int)hdr[1], width = (int)hdr[2], n_out = (int)hdr[3];
  if (n_in < 1 || n_in > 1024 || width < 16 || width > 1024 || width % 32 || n_out < 1 || n_out > 1024)
    return ROM_EFORMAT;
  const int64_t nparam =
      (int64_t)n_in * width + width + 2 * ((int64_t)width * width + width) + (int64_t)width * n_out + n_out;
  if (bytes < mlp_blob_bytes(n_in, width, n_out, nparam)) return ROM_EFORMAT;
  std::vector<float> f((size_t)(2 * n_in + 2 * n_out + nparam));
  memcpy(f.data(), b + 32, 4 * f.size());
  for (float v : f)
    if (!isfinite(v)) return ROM_EFORMAT;
  rom_mlp_handle m = nullptr;
  int rc = rom_mlp_create(n_in, width, n_out, max_batch, device, &m);
  if (rc != ROM_OK) return rc;
  rc = rom_mlp_set_scaling(m, f.data(), f.data() + n_in, f.data() + 2 * n_in, f.data() + 2 * n_in + n_out);
  if (rc == ROM_EINVAL) rc = ROM_EFORMAT;  // a non-positive deviation in the file
  if (rc == ROM_OK) rc = rom_mlp_set_params(m, f.data() + 2 * n_in + 2 * n_out, nparam);
  if (rc != ROM_OK) {
    rom_mlp_free(m);
    return rc;
  }
  *out = m;
  return ROM_OK;
}

int rom_mlp_gradients(rom_mlp_handle m, int32_t B, const float* X, const float* Y, int32_t prec, float* grads,
                      float* loss, hipStream_t s) {
  if (!m || B < 1 || B > m->max_batch || !X || !Y || (prec != ROM_DT_F32 && prec != ROM_DT_BF16)) return ROM_EINVAL;
  DeviceGuard guard(m->device);
  int rc = mlp_gradients(m, B, X, Y, nullptr, prec, loss, s);
  if (rc != ROM_OK || !grads) return rc;
  // unpad into the host parameter layout
  const int fi[4] = {m->n_in, m->width, m->width, m->width}, fo[4] = {m->width, m->width, m->width, m->n_out};
  int64_t dst = 0;
  for (int l = 0; l < 4; ++l) {
    if (hipMemcpy2DAsync(grads + dst, 4 * fo[l], m->G + m->off_w[l], 4 * m->N[l], 4 * fo[l], fi[l],
                         hipMemcpyDeviceToDevice, s) != hipSuccess)
      return ROM_EHIP;
    dst += (int64_t)fi[l] * fo[l];
    if (hipMemcpyAsync(grads + dst, m->G + m->off_b[l], 4 * fo[l], hipMemcpyDeviceToDevice, s) != hipSuccess)
      return ROM_EHIP;
    dst += fo[l];
  }
  return ROM_OK;
}

int rom_mlp_train_step(rom_mlp_handle m, int32_t B, const float* X, const float* Y, float lr, int32_t prec,
                       float* loss, hipStream_t s) {
  if (!m || B < 1 || B > m->max_batch || !X || !Y || !(lr > 0) || (prec != ROM_DT_F32 && prec != ROM_DT_BF16))
    return ROM_EINVAL;
  DeviceGuard guard(m->device);
  return mlp_train_step(m, B, X, Y, nullptr, lr, prec, loss, s);
}

int rom_mlp_train_epoch(rom_mlp_handle m, int32_t N, const float* X, const float* Y, const int32_t* order,
                        int32_t batch, float lr, int32_t prec, float* loss_sum, hipStream_t s) {
  if (!m || N < 1 || batch < 1 || batch > m->max_batch || batch > N || !X || !Y || !order || !loss_sum ||
      !(lr > 0) || (prec != ROM_DT_F32 && prec != ROM_DT_BF16))
    return ROM_EINVAL;
  DeviceGuard guard(m->device);
  k_zero_f32<<<1, 64, 0, s>>>(loss_sum);
  for (int32_t b0 = 0; b0 + batch <= N; b0 += batch) {
    const int rc = mlp_train_step(m, batch, X, Y, order + b0, lr, prec, m->loss_one, s);
    if (rc != ROM_OK) return rc;
    k_add_f32<<<1, 64, 0, s>>>(loss_sum, m->loss_one);
  }
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_mlp_fit_scaling(rom_mlp_handle m, int32_t N, const float* X, const float* Y, hipStream_t s) {
  if (!m || N < 2 || !X || !Y) return ROM_EINVAL;
  DeviceGuard guard(m->device);
  const int nc = m->n_in + m->n_out;
  const dim3 grid((unsigned)((nc + 63) / 64), MLP_SSPLIT);
  // mean, then the sum of squared deviations from it (two passes, FP64 partials over row slices)
  for (int pass = 0; pass < 2; ++pass) {
    k_col_moments<<<grid, 256, 0, s>>>(N, m->n_in, m->n_out, X, Y, pass, m->xm, m->ym, m->spart);
    k_col_finish<<<(unsigned)((nc + 255) / 256), 256, 0, s>>>(N, m->n_in, m->n_out, pass, m->spart, m->xm, m->xs,
                                                              m->ym, m->ys);
  }
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

}  // extern "C"

// in-library entry for the warm start of rom_step: raw features -> raw dr
int rom_mlp_predict(rom_mlp* m, int B, const float* X, float* Y, hipStream_t s) {
  for (int b0 = 0; b0 < B; b0 += m->max_batch) {
    const int b = B - b0 < m->max_batch ? B - b0 : m->max_batch;
    const int rc = rom_mlp_forward(m, b, X + (size_t)b0 * m->n_in, Y + (size_t)b0 * m->n_out, ROM_DT_BF16, s);
    if (rc != ROM_OK) return rc;
  }
  return ROM_OK;
}
int rom_mlp_dims(const rom_mlp* m, int* n_in, int* n_out) {
  *n_in = m->n_in;
  *n_out = m->n_out;
  return ROM_OK;
}
