// Offline stage on the GPU: POD by the method of snapshots (Sec. 3.1, the
// fluctuation modes of eq. pod_disp, orthonormal in the V^p product; Sec.
// 3.2, the weighted-stress modes, orthonormal in L^2 of the parent domain).
// With snapshots S (columns s_j) and a symmetric positive definite weight M:
// the snapshot Gram matrix C = S^T M S = V diag(lambda) V^T, the leading
// modes phi_k = S v_k / sqrt(lambda_k), then one re-orthonormalisation
// phi <- phi L^-T with L L^T = phi^T M phi (Cholesky).
//
// The two Gram products (ns x ns and n x n over the long snapshot dimension)
// and the mode product run on FP64 MFMA; the ns x ns symmetric eigenproblem
// and the n x n Cholesky factorisation are small dense library steps
// (rocSOLVER).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "podecm.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int KSPLIT_MAX = 8;

// C (+ z * cstride for slice z) = A B^T (BT) or A B over the inner slice
// [z kchunk, (z + 1) kchunk): A [M][K] (lda, K contiguous); B [N][K] (ldb) when
// BT, else B [K][N] (ldb, N contiguous).  Workgroup 64 x 64 outputs, wave
// 32 x 32 (2 x 2 MFMA tiles of 16 x 16), 16 inner indices per round: lane
// (q, c) takes k = k0 + 4 q + s at MFMA step s, so that it reads four
// consecutive elements of its row.  Out-of-range operands read as zero.
template <bool BT>
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int N, int K, const double* __restrict__ A, long lda,
                                                  const double* __restrict__ B, long ldb, double* __restrict__ C,
                                                  long ldc, int kchunk, long cstride) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32, n0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    double a[2][4], b[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = m0 + 16 * i + c;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = k0 + 4 * q + s;
        a[i][s] = (m < M && k < ke) ? A[(long)m * lda + k] : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + 16 * j + c;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = k0 + 4 * q + s;
        b[j][s] = (n < N && k < ke) ? (BT ? B[(long)n * ldb + k] : B[(long)k * ldb + n]) : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
  }
  C += blockIdx.z * cstride;
  // output layout of the FP64 16 x 16 MFMA: row q + 4 r, column c
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + 16 * i + q + 4 * r, n = n0 + 16 * j + c;
        if (m < M && n < N) C[(long)m * ldc + n] = acc[i][j][r];
      }
}

// out[i] = sum over z < S of part[z * stride + i], in order of z
__global__ void k_sum_slices_f64(long count, int S, long stride, const double* __restrict__ part,
                                 double* __restrict__ out) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= count) return;
  double s = 0.0;
  for (int z = 0; z < S; ++z) s += part[z * stride + i];
  out[i] = s;
}

// Y[j][r] = m[r] X[j][r] (diagonal weight) for ns columns of length nrow
__global__ void k_weight_diag(long nrow, int ns, const double* __restrict__ m, const double* __restrict__ X,
                              double* __restrict__ Y) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= nrow * ns) return;
  Y[t] = m[t % nrow] * X[t];
}

// Y[j][r] = sum_e val[e] X[j][col[e]] over row r of a CSR matrix; lane per
// (row, group of eight columns)
__global__ void k_weight_csr(int nrow, int ns, const int* __restrict__ ptr, const int* __restrict__ col,
                             const double* __restrict__ val, const double* __restrict__ X, double* __restrict__ Y) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int groups = (ns + 7) / 8;
  if (t >= (long)nrow * groups) return;
  const int r = (int)(t % nrow), j0 = (int)(t / nrow) * 8;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int e = ptr[r]; e < ptr[r + 1]; ++e) {
    const double v = val[e];
    const int cc = col[e];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j0 + j < ns) acc[j] = fma(v, X[(long)(j0 + j) * nrow + cc], acc[j]);
  }
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j0 + j < ns) Y[(long)(j0 + j) * nrow + r] = acc[j];
}

// C <- (C + C^T) / 2 (rounding of the two triangles)
__global__ void k_symmetrize(int n, double* __restrict__ C) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  if (i < j) {
    const double v = 0.5 * (C[(long)i * n + j] + C[(long)j * n + i]);
    C[(long)i * n + j] = v;
    C[(long)j * n + i] = v;
  }
}

// eigenvalues ascending (D) and eigenvectors in the columns of V (column-
// major, ns x ns) -> lambda descending, WT[k][j] = v_k[j] / sqrt(lambda_k)
// for the n leading ones
__global__ void k_select(int ns, int n, const double* __restrict__ D, const double* __restrict__ V,
                         double* __restrict__ lambda, double* __restrict__ WT) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < ns) lambda[t] = D[ns - 1 - t];
  if (t >= (long)n * ns) return;
  const int k = (int)(t / ns), j = (int)(t % ns), kk = ns - 1 - k;
  WT[t] = V[(long)kk * ns + j] / sqrt(D[kk]);
}

// phi <- phi L^-T row by row: for each r, L y = phi[:, r] by forward
// substitution (L lower, column-major n x n), y written back in place
__global__ void k_trsm_rows(long nrow, int n, const double* __restrict__ Lcm, double* __restrict__ phi) {
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r >= nrow) return;
  for (int a = 0; a < n; ++a) {
    double s = phi[(long)a * nrow + r];
    for (int b = 0; b < a; ++b) s = fma(-Lcm[a + (long)b * n], phi[(long)b * nrow + r], s);
    phi[(long)a * nrow + r] = s / Lcm[a + (long)a * n];
  }
}

inline unsigned nblk(long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// C [M][N] = A B^T or A B with a split of the long inner dimension into
// slices added in order
struct Gemm {
  double* part;  // [KSPLIT_MAX][M][N]
  template <bool BT>
  void run(int M, int N, int K, const double* A, long lda, const double* B, long ldb, double* C, hipStream_t s) {
    const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
    int S = std::max(1, std::min(KSPLIT_MAX, (1024 + tiles - 1) / tiles));
    S = std::min(S, std::max(1, K / 256));
    const int kchunk = ((K + S - 1) / S + 15) / 16 * 16;
    S = (K + kchunk - 1) / kchunk;
    dim3 grid((N + 63) / 64, (M + 63) / 64, S);
    k_gemm_f64<BT><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, part, N, kchunk, (long)M * N);
    k_sum_slices_f64<<<nblk((long)M * N), 256, 0, s>>>((long)M * N, S, (long)M * N, part, C);
  }
};

struct PodWork {
  double *MS, *part, *C, *D, *E, *WT, *G;
  int* info;
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t pod_layout(long nrow, long ns, long n, PodWork* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const long big = std::max(ns * ns, n * nrow);  // split-K slices of the Gram and mode products
  double* MS = (double*)take(8 * (size_t)nrow * ns);
  double* part = (double*)take(8 * (size_t)KSPLIT_MAX * big);
  double* C = (double*)take(8 * (size_t)ns * ns);
  double* D = (double*)take(8 * (size_t)ns);
  double* E = (double*)take(8 * (size_t)ns);
  double* WT = (double*)take(8 * (size_t)n * ns);
  double* G = (double*)take(8 * (size_t)n * n);
  int* info = (int*)take(64);
  if (w) *w = PodWork{MS, part, C, D, E, WT, G, info};
  return off;
}


// ---------------------------------------------------------------------------
// Empirical cubature (Sec. 3.2, eqs. integralsbasis and integral_ecm): the
// greedy of the published method the paper defers to.  The integrands J
// (R x nq) weighted by the full rule: J diag(sqrt(w)) = U Sigma V^T, rank r
// (singular values above 1e-12 of the largest); Z = V^T_r diag(1/sqrt(w)),
// b = Z w.  From an empty set and res = b: add the point of largest positive
// Z_q . res / |Z_q| (lowest index on ties), least squares on the selected
// set, non-negative least squares when a weight comes out non-positive,
// points of zero weight leave, res = b - Z_S w_S; until |res| <= eps |b|, the
// point budget or no positive correlation.

constexpr int ECM_THREADS = 1024;
constexpr int ECM_SCORE_BLOCK = 256;

// Jh (column-major R x nq) = J (row-major R x nq) diag(sqrt(w))
__global__ void k_ecm_scale(int R, int nq, const double* __restrict__ J, const double* __restrict__ w,
                            double* __restrict__ Jh) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)R * nq) return;
  const int q = (int)(t / R), i = (int)(t % R);
  Jh[t] = J[(long)i * nq + q] * sqrt(w[q]);
}

// Jt (column-major nq x R: the transpose of the scaled J) = J diag(sqrt(w)),
// which has the layout of J itself
__global__ void k_ecm_scale_t(int R, int nq, const double* __restrict__ J, const double* __restrict__ w,
                              double* __restrict__ Jt) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)R * nq) return;
  Jt[t] = J[t] * sqrt(w[t % nq]);
}

// Zr[i][q] = V^T(i, q) / sqrt(w_q) for i < r (V^T column-major, ldv = R);
// cn[q] = |Z_q|
__global__ void k_ecm_z(int R, int r, int nq, const double* __restrict__ V, const double* __restrict__ w,
                        double* __restrict__ Zr, double* __restrict__ cn) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const double is = 1.0 / sqrt(w[q]);
  double s = 0.0;
  for (int i = 0; i < r; ++i) {
    const double z = V[i + (long)q * R] * is;
    Zr[(long)i * nq + q] = z;
    s = fma(z, z, s);
  }
  cn[q] = sqrt(s);
}

// R (column-major R x R, upper) from the QR factorisation left in Jt
// (column-major nq x R)
__global__ void k_copy_r(int R, int nq, const double* __restrict__ Jt, double* __restrict__ Rm) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)R * R) return;
  const int i = (int)(t % R), j = (int)(t / R);
  Rm[t] = (i <= j) ? Jt[i + (long)j * nq] : 0.0;
}

// Zr[i][q] = Vt[i][q] / sqrt(w_q) (Vt row-major r x nq); cn[q] = |Z_q|
__global__ void k_ecm_z_rows(int r, int nq, const double* __restrict__ Vt, const double* __restrict__ w,
                             double* __restrict__ Zr, double* __restrict__ cn) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const double is = 1.0 / sqrt(w[q]);
  double sacc = 0.0;
  for (int i = 0; i < r; ++i) {
    const double z = Vt[(long)i * nq + q] * is;
    Zr[(long)i * nq + q] = z;
    sacc = fma(z, z, sacc);
  }
  cn[q] = sqrt(sacc);
}

// b[i] = sum_q Zr[i][q] w[q]: a workgroup per i, fixed-order tree
__global__ __launch_bounds__(256) void k_ecm_b(int nq, const double* __restrict__ Zr, const double* __restrict__ w,
                                               double* __restrict__ b) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int q = threadIdx.x; q < nq; q += 256) s = fma(Zr[(long)i * nq + q], w[q], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) b[i] = red[0];
}

// score of every point, then the best of each workgroup (largest score,
// lowest index on ties); selected points score -inf
__global__ __launch_bounds__(ECM_SCORE_BLOCK) void k_ecm_score(int r, int nq, const double* __restrict__ Zr,
                                                               const double* __restrict__ cn,
                                                               const double* __restrict__ res,
                                                               const int* __restrict__ sel_flag,
                                                               double* __restrict__ best_v, int* __restrict__ best_i) {
  extern __shared__ double sres[];
  __shared__ double rv[ECM_SCORE_BLOCK];
  __shared__ int ri[ECM_SCORE_BLOCK];
  for (int i = threadIdx.x; i < r; i += ECM_SCORE_BLOCK) sres[i] = res[i];
  __syncthreads();
  const int q = blockIdx.x * ECM_SCORE_BLOCK + threadIdx.x;
  double v = -INFINITY;
  if (q < nq && !sel_flag[q]) {
    // in order of i, 16 loads of Z in flight per lane
    double s = 0.0;
    int i = 0;
    for (; i + 16 <= r; i += 16) {
      double zz[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) zz[u] = Zr[(long)(i + u) * nq + q];
#pragma unroll
      for (int u = 0; u < 16; ++u) s = fma(zz[u], sres[i + u], s);
    }
    for (; i < r; ++i) s = fma(Zr[(long)i * nq + q], sres[i], s);
    v = s / cn[q];
  }
  rv[threadIdx.x] = v;
  ri[threadIdx.x] = q;
  __syncthreads();
  for (int h = ECM_SCORE_BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double ov = rv[threadIdx.x + h];
      const int oi = ri[threadIdx.x + h];
      if (ov > rv[threadIdx.x] || (ov == rv[threadIdx.x] && oi < ri[threadIdx.x])) {
        rv[threadIdx.x] = ov;
        ri[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    best_v[blockIdx.x] = rv[0];
    best_i[blockIdx.x] = ri[0];
  }
}

// Greedy state, device side
struct EcmState {
  int k;        // selected points
  int status;   // 0 running, 1 no positive correlation, 2 dependent column
  int qstar;    // last chosen point
  int pad;
  double sstar; // its score
  double rn;    // |res|
};

// block-wide sum (fixed order), all threads receive it
__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = (blockDim.x + 63) >> 6;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += red[w];
  return t;
}

// Cholesky of the p x p matrix A (row-major, ld) into L (lower, row-major,
// ld), in one workgroup; returns false if a pivot is not positive
__device__ bool block_cholesky(int p, const double* __restrict__ A, double* __restrict__ Lm, int ld) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (long t = tid; t < (long)p * p; t += nt) {
    const int i = (int)(t / p), j = (int)(t % p);
    Lm[(long)i * ld + j] = (j <= i) ? A[(long)i * ld + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    const double d = Lm[(long)j * ld + j];
    __syncthreads();
    if (!(d > 0.0)) return false;
    const double sd = sqrt(d);
    for (int i = j + tid; i < p; i += nt) Lm[(long)i * ld + j] = (i == j) ? sd : Lm[(long)i * ld + j] / sd;
    __syncthreads();
    const int rows = p - j - 1;
    for (long t = tid; t < (long)rows * rows; t += nt) {
      const int i = j + 1 + (int)(t / rows), c = j + 1 + (int)(t % rows);
      if (c <= i) Lm[(long)i * ld + c] = fma(-Lm[(long)i * ld + j], Lm[(long)c * ld + j], Lm[(long)i * ld + c]);
    }
    __syncthreads();
  }
  return true;
}

// Triangular solves with the Cholesky factor (L lower, row-major, ld), in
// place on a vector in LDS, by the whole workgroup (every thread calls them).
// Blocks of TRI_NB unknowns: the diagonal block is staged in LDS (T, row
// stride TRI_LD against bank conflicts) and solved by wave 0 with one unknown
// per lane, column by column (the solved value is read from its lane, so no
// reduction sits on the sequential chain); the rest of the vector is then
// updated by all threads.
constexpr int TRI_NB = 64, TRI_LD = 65;

__device__ inline double readlane_d(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ void tri_stage(int kb, int nb, const double* __restrict__ Lm, int ld, double* T) {
  for (int t = threadIdx.x; t < nb * TRI_NB; t += blockDim.x) {
    const int a = t / TRI_NB, c = t % TRI_NB;
    if (c <= a) T[a * TRI_LD + c] = Lm[(long)(kb + a) * ld + kb + c];
  }
  __syncthreads();
}

// y <- L^-1 y (L is p x p)
__device__ void lower_solve(int p, const double* __restrict__ Lm, int ld, double* y, double* T) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  for (int kb = 0; kb < p; kb += TRI_NB) {
    const int nb = min(TRI_NB, p - kb);
    tri_stage(kb, nb, Lm, ld, T);
    if (tid < 64) {
      double v = (lane < nb) ? y[kb + lane] : 0.0;
      const double inv = (lane < nb) ? 1.0 / T[lane * TRI_LD + lane] : 0.0;
      for (int l = 0; l < nb; ++l) {
        const double xl = readlane_d(v, l) * readlane_d(inv, l);
        if (lane == l)
          v = xl;
        else if (lane > l && lane < nb)
          v = fma(-T[lane * TRI_LD + l], xl, v);
      }
      if (lane < nb) y[kb + lane] = v;
    }
    __syncthreads();
    for (int j = kb + nb + tid; j < p; j += nt) {
      const double* row = Lm + (long)j * ld + kb;
      double acc = y[j];
#pragma unroll 8
      for (int t = 0; t < nb; ++t) acc = fma(-row[t], y[kb + t], acc);
      y[j] = acc;
    }
    __syncthreads();
  }
}

// y <- L^-T y
__device__ void upper_solve(int p, const double* __restrict__ Lm, int ld, double* y, double* T) {
  if (p <= 0) return;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  for (int kb = ((p - 1) / TRI_NB) * TRI_NB; kb >= 0; kb -= TRI_NB) {
    const int nb = min(TRI_NB, p - kb);
    tri_stage(kb, nb, Lm, ld, T);
    if (tid < 64) {
      double v = (lane < nb) ? y[kb + lane] : 0.0;
      const double inv = (lane < nb) ? 1.0 / T[lane * TRI_LD + lane] : 0.0;
      for (int l = nb - 1; l >= 0; --l) {
        const double xl = readlane_d(v, l) * readlane_d(inv, l);
        if (lane == l)
          v = xl;
        else if (lane < l)
          v = fma(-T[l * TRI_LD + lane], xl, v);
      }
      if (lane < nb) y[kb + lane] = v;
    }
    __syncthreads();
    for (int j = tid; j < kb; j += nt) {
      double acc = y[j];
#pragma unroll 8
      for (int t = 0; t < nb; ++t) acc = fma(-Lm[(long)(kb + t) * ld + j], y[kb + t], acc);
      y[j] = acc;
    }
    __syncthreads();
  }
}

// One greedy iteration in one workgroup: pick the best point of the score
// blocks, append it, extend the Cholesky factor of the selected set's Gram
// matrix G = Z_S^T Z_S by one row, solve G w = Z_S^T b; if a weight is not
// positive, Lawson-Hanson non-negative least squares on (G, h) started from
// the previous (positive) weights with the new point at zero; drop points of
// zero weight (refactoring G); res = b - Z_S w.  yv = L^-1 h is kept from
// one iteration to the next: appending a point leaves its first k entries
// unchanged, so only the new one is computed; after points leave it is
// recomputed from the new factor.  Every branch that reaches a workgroup
// barrier is decided from shared values.
__global__ __launch_bounds__(ECM_THREADS) void k_ecm_update(
    int r, int nq, int mmax, int nblocks, const double* __restrict__ Zr, const double* __restrict__ b,
    const double* __restrict__ best_v, const int* __restrict__ best_i, int* __restrict__ S, double* __restrict__ ZS,
    double* __restrict__ G, double* __restrict__ Lm, double* __restrict__ Gp, double* __restrict__ Lp,
    double* __restrict__ hv, double* __restrict__ yv, double* __restrict__ w, double* __restrict__ res,
    int* __restrict__ sel_flag, EcmState* __restrict__ st) {
  extern __shared__ double sh[];
  double* x = sh;               // [mmax + 1] current solution
  double* z = x + mmax + 1;     // [mmax + 1] least-squares solution on the passive set
  double* hp = z + mmax + 1;    // [mmax + 1] h gathered on the passive set
  double* red = hp + mmax + 1;  // [32]
  double* T = red + 32;         // [TRI_NB * TRI_LD] diagonal block of a triangular solve
  int* pas = (int*)(T + TRI_NB * TRI_LD);  // [mmax + 1] passive flags
  int* pidx = pas + mmax + 1;   // [mmax + 1] passive indices in order
  __shared__ int s_q, s_k, s_flag, s_np, s_t;
  __shared__ double s_v, s_alpha;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  if (tid == 0) {
    double bv = -INFINITY;
    int bi = nq;
    for (int blk = 0; blk < nblocks; ++blk)
      if (best_v[blk] > bv || (best_v[blk] == bv && best_i[blk] < bi)) {
        bv = best_v[blk];
        bi = best_i[blk];
      }
    s_v = bv;
    s_q = bi;
    s_k = st->k;
  }
  __syncthreads();
  const int q = s_q, k = s_k;
  if (!(s_v > 0.0)) {
    if (tid == 0) {
      st->status = 1;
      st->sstar = s_v;
      st->qstar = q;
    }
    return;
  }
  // append Z_q as row k of ZS
  for (int i = tid; i < r; i += nt) ZS[(long)k * r + i] = Zr[(long)i * nq + q];
  if (tid == 0) {
    S[k] = q;
    sel_flag[q] = 1;
  }
  __syncthreads();
  // G[k][j] = G[j][k] = ZS[j] . ZS[k] (j <= k), h[k] = ZS[k] . b: a wave per
  // product, four products interleaved so that their loads and reductions overlap
  for (int j0 = 4 * wave; j0 <= k + 1; j0 += 4 * nw) {
    const double* zk = ZS + (long)k * r;
    const double* o[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) o[u] = (j0 + u <= k) ? ZS + (long)(j0 + u) * r : b;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = lane; i < r; i += 64) {
      const double zi = zk[i];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j0 + u <= k + 1) acc[u] = fma(o[u][i], zi, acc[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      for (int off = 32; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off);
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + u;
        if (j <= k) {
          G[(long)k * mmax + j] = acc[u];
          G[(long)j * mmax + k] = acc[u];
        } else if (j == k + 1) {
          hv[k] = acc[u];
        }
      }
    }
  }
  __syncthreads();
  // new row of the Cholesky factor: L[k][0..k) = L^-1 g, L[k][k] = sqrt(G_kk - |y|^2)
  for (int j = tid; j <= k; j += nt) hp[j] = z[j] = G[(long)k * mmax + j];
  __syncthreads();
  lower_solve(k, Lm, mmax, z, T);
  if (wave == 0) {
    double acc = 0.0;
    for (int t = lane; t < k; t += 64) acc = fma(z[t], z[t], acc);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    const double d2 = hp[k] - acc;
    // new entry of L^-1 h: (h_k - L[k][0..k) . yv[0..k)) / L[k][k]
    double ay = 0.0;
    for (int t = lane; t < k; t += 64) ay = fma(z[t], yv[t], ay);
    for (int off = 32; off > 0; off >>= 1) ay += __shfl_xor(ay, off);
    const double lkk = sqrt(fmax(d2, 0.0));
    if (lane == 0) s_flag = (d2 > 1e-14 * hp[k]) ? 0 : 1;
    for (int t = lane; t < k; t += 64) Lm[(long)k * mmax + t] = z[t];
    if (lane == 0) {
      Lm[(long)k * mmax + k] = lkk;
      yv[k] = (hv[k] - ay) / lkk;
    }
  }
  __syncthreads();
  if (s_flag) {  // the new column depends on the selected ones
    if (tid == 0) {
      st->status = 2;
      st->qstar = q;
      sel_flag[q] = 0;
    }
    return;
  }
  const int p = k + 1;
  // unconstrained least squares on all p points
  for (int j = tid; j < p; j += nt) x[j] = yv[j];
  __syncthreads();
  upper_solve(p, Lm, mmax, x, T);
  if (tid == 0) {
    int bad = 0;
    for (int j = 0; j < p; ++j) bad |= !(x[j] > 0.0);
    s_flag = bad;
  }
  __syncthreads();
  int pnew = p;
  if (s_flag) {
    // Lawson-Hanson from x = (previous weights, 0), passive = previous points
    double hmax = 0.0;
    for (int j = 0; j < p; ++j) hmax = fmax(hmax, fabs(hv[j]));
    const double tol = 1e-13 * hmax;
    for (int j = tid; j < p; j += nt) {
      x[j] = (j < k) ? w[j] : 0.0;
      pas[j] = j < k;
    }
    __syncthreads();
    for (int outer = 0; outer < 3 * p; ++outer) {
      // gradient on the active points; the largest above tol joins the passive set
      if (tid == 0) {
        double gb = tol;
        int tb = -1;
        for (int i = 0; i < p; ++i) {
          if (pas[i]) continue;
          double gi = hv[i];
          for (int j = 0; j < p; ++j) gi = fma(-G[(long)i * mmax + j], x[j], gi);
          if (gi > gb) {
            gb = gi;
            tb = i;
          }
        }
        s_t = tb;
        if (tb >= 0) pas[tb] = 1;
      }
      __syncthreads();
      if (s_t < 0) break;
      for (int inner = 0; inner < p; ++inner) {
        if (tid == 0) {
          int np = 0;
          for (int i = 0; i < p; ++i)
            if (pas[i]) pidx[np++] = i;
          s_np = np;
        }
        __syncthreads();
        const int np = s_np;
        for (long t = tid; t < (long)np * np; t += nt) {
          const int a = (int)(t / np), c = (int)(t % np);
          Gp[(long)a * mmax + c] = G[(long)pidx[a] * mmax + pidx[c]];
        }
        for (int a = tid; a < np; a += nt) z[a] = hv[pidx[a]];
        __syncthreads();
        const bool ok = block_cholesky(np, Gp, Lp, mmax);
        if (!ok) {
          if (tid == 0) st->status = 2;
          return;
        }
        lower_solve(np, Lp, mmax, z, T);
        upper_solve(np, Lp, mmax, z, T);
        if (tid == 0) {
          // step from x towards z as far as feasibility allows; the point
          // that limits the step (and any other at zero) leaves the passive set
          double alpha = 2.0;
          int ia = -1;
          for (int a = 0; a < np; ++a) {
            const int i = pidx[a];
            if (!(z[a] > 0.0)) {
              const double al = x[i] / (x[i] - z[a]);
              if (al < alpha) {
                alpha = al;
                ia = i;
              }
            }
          }
          s_alpha = alpha;
          if (alpha > 1.0) {
            for (int a = 0; a < np; ++a) x[pidx[a]] = z[a];
          } else {
            for (int a = 0; a < np; ++a) {
              const int i = pidx[a];
              x[i] = (i == ia) ? 0.0 : fma(alpha, z[a] - x[i], x[i]);
              if (!(x[i] > 0.0)) {
                x[i] = 0.0;
                pas[i] = 0;
              }
            }
          }
        }
        __syncthreads();
        if (s_alpha > 1.0) break;
      }
    }
    // keep the points of positive weight (order kept), refactor
    if (tid == 0) {
      int c = 0;
      for (int j = 0; j < p; ++j) {
        if (x[j] > 0.0) {
          pidx[c] = j;
          ++c;
        } else {
          sel_flag[S[j]] = 0;
        }
      }
      s_np = c;
    }
    __syncthreads();
    pnew = s_np;
    for (long t = tid; t < (long)pnew * pnew; t += nt) {
      const int a = (int)(t / pnew), c = (int)(t % pnew);
      Gp[(long)a * mmax + c] = G[(long)pidx[a] * mmax + pidx[c]];
    }
    for (int a = tid; a < pnew; a += nt) {
      z[a] = x[pidx[a]];
      hp[a] = hv[pidx[a]];
    }
    __syncthreads();
    // rows of ZS and S compacted in order (a row only moves down)
    for (int a = 0; a < pnew; ++a) {
      const int from = pidx[a];
      if (from != a)
        for (int i = tid; i < r; i += nt) ZS[(long)a * r + i] = ZS[(long)from * r + i];
      __syncthreads();
    }
    if (tid == 0)
      for (int a = 0; a < pnew; ++a) S[a] = S[pidx[a]];
    for (long t = tid; t < (long)pnew * pnew; t += nt) {
      const int a = (int)(t / pnew), c = (int)(t % pnew);
      G[(long)a * mmax + c] = Gp[(long)a * mmax + c];
    }
    for (int a = tid; a < pnew; a += nt) {
      x[a] = z[a];
      hv[a] = hp[a];
    }
    __syncthreads();
    if (!block_cholesky(pnew, G, Lm, mmax)) {
      if (tid == 0) st->status = 2;
      return;
    }
    for (int a = tid; a < pnew; a += nt) z[a] = hv[a];
    __syncthreads();
    lower_solve(pnew, Lm, mmax, z, T);
    for (int a = tid; a < pnew; a += nt) yv[a] = z[a];
  }
  for (int j = tid; j < pnew; j += nt) w[j] = x[j];
  __syncthreads();
  // res = b - sum_j w_j ZS[j] (in order of j), |res|; the weights are read
  // from LDS and the rows of ZS in batches of 8 loads in flight
  double part = 0.0;
  for (int i = tid; i < r; i += nt) {
    double v = b[i];
    int j = 0;
    for (; j + 8 <= pnew; j += 8) {
      double zz[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) zz[u] = ZS[(long)(j + u) * r + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) v = fma(-x[j + u], zz[u], v);
    }
    for (; j < pnew; ++j) v = fma(-x[j], ZS[(long)j * r + i], v);
    res[i] = v;
    part = fma(v, v, part);
  }
  const double rn2 = block_sum(part, red);
  if (tid == 0) {
    st->k = pnew;
    st->status = 0;
    st->qstar = q;
    st->sstar = s_v;
    st->rn = sqrt(rn2);
  }
}


struct EcmWork {
  double *Jh, *Sv, *V, *E, *tau, *Rm, *U, *Zr, *cn, *b, *res, *bv, *ZS, *G, *Lm, *Gp, *Lp, *hv, *yv, *w, *bn;
  int *bi, *S, *sel, *info;
  EcmState* st;
};

constexpr int ECM_MMAX = 1024;

size_t ecm_layout(long R, long nq, long mmax, EcmWork* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const long mn = std::min(R, nq), nblocks = (nq + ECM_SCORE_BLOCK - 1) / ECM_SCORE_BLOCK;
  EcmWork e;
  e.Jh = (double*)take(8 * (size_t)R * nq);
  e.Sv = (double*)take(8 * (size_t)mn);
  e.V = (double*)take(8 * (size_t)mn * nq);
  e.E = (double*)take(8 * (size_t)mn);
  e.tau = (double*)take(8 * (size_t)mn);
  e.Rm = (double*)take(8 * (size_t)mn * mn);
  e.U = (double*)take(8 * (size_t)mn * mn);
  e.Zr = (double*)take(8 * (size_t)mn * nq);
  e.cn = (double*)take(8 * (size_t)nq);
  e.b = (double*)take(8 * (size_t)mn);
  e.res = (double*)take(8 * (size_t)mn);
  e.bv = (double*)take(8 * (size_t)nblocks);
  e.ZS = (double*)take(8 * (size_t)mmax * mn);
  e.G = (double*)take(8 * (size_t)mmax * mmax);
  e.Lm = (double*)take(8 * (size_t)mmax * mmax);
  e.Gp = (double*)take(8 * (size_t)mmax * mmax);
  e.Lp = (double*)take(8 * (size_t)mmax * mmax);
  e.hv = (double*)take(8 * (size_t)mmax);
  e.yv = (double*)take(8 * (size_t)mmax);
  e.w = (double*)take(8 * (size_t)mmax);
  e.bn = (double*)take(8);
  e.bi = (int*)take(4 * (size_t)nblocks);
  e.S = (int*)take(4 * (size_t)mmax);
  e.sel = (int*)take(4 * (size_t)nq);
  e.info = (int*)take(64);
  e.st = (EcmState*)take(sizeof(EcmState));
  if (w) *w = e;
  return off;
}

// |b| in one workgroup
__global__ __launch_bounds__(256) void k_norm(int n, const double* __restrict__ v, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s = fma(v[i], v[i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(red[0]);
}

}  // namespace

extern "C" {

int rom_pod_workspace(int32_t nrow, int32_t ns, int32_t n, size_t* bytes) {
  if (!bytes || nrow < 1 || ns < 1 || n < 1 || n > ns) return ROM_EINVAL;
  *bytes = pod_layout(nrow, ns, n, nullptr, nullptr);
  return ROM_OK;
}

int rom_pod(int32_t nrow, int32_t ns, const double* S_dev, const double* mdiag_dev, const int32_t* csr_ptr_dev,
            const int32_t* csr_col_dev, const double* csr_val_dev, int32_t n, double* modes_dev, double* lambda_dev,
            void* work_dev, size_t work_bytes, hipStream_t stream) {
  if (nrow < 1 || ns < 1 || n < 1 || n > ns || !S_dev || !modes_dev || !lambda_dev || !work_dev) return ROM_EINVAL;
  const bool diag = mdiag_dev != nullptr, csr = csr_ptr_dev && csr_col_dev && csr_val_dev;
  if (diag == csr) return ROM_EINVAL;  // exactly one weight
  if (work_bytes < pod_layout(nrow, ns, n, nullptr, nullptr)) return ROM_EINVAL;
  PodWork w;
  pod_layout(nrow, ns, n, &w, (char*)work_dev);
  Gemm gemm{w.part};
  auto weight = [&](const double* X, double* Y, int cols) {
    if (diag)
      k_weight_diag<<<nblk((long)nrow * cols), 256, 0, stream>>>(nrow, cols, mdiag_dev, X, Y);
    else
      k_weight_csr<<<nblk((long)nrow * ((cols + 7) / 8)), 256, 0, stream>>>(nrow, cols, csr_ptr_dev, csr_col_dev,
                                                                           csr_val_dev, X, Y);
  };
  // C = S^T M S
  weight(S_dev, w.MS, ns);
  gemm.run<true>(ns, ns, nrow, S_dev, nrow, w.MS, nrow, w.C, stream);
  k_symmetrize<<<nblk((long)ns * ns), 256, 0, stream>>>(ns, w.C);
  if (hipGetLastError() != hipSuccess) return ROM_EHIP;
  rocblas_handle rb;
  if (rocblas_create_handle(&rb) != rocblas_status_success) return ROM_EHIP;
  int rc = ROM_OK;
  if (rocblas_set_stream(rb, stream) != rocblas_status_success ||
      rocsolver_dsyevd(rb, rocblas_evect_original, rocblas_fill_upper, ns, w.C, ns, w.D, w.E, w.info) !=
          rocblas_status_success)
    rc = ROM_EHIP;
  std::vector<double> D(ns);
  int info = 0;
  if (rc == ROM_OK && (hipMemcpyAsync(D.data(), w.D, 8L * ns, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                       hipMemcpyAsync(&info, w.info, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                       hipStreamSynchronize(stream) != hipSuccess))
    rc = ROM_EHIP;
  if (rc == ROM_OK && info != 0) rc = ROM_EHIP;
  // numerical rank of the snapshot Gram matrix: eigenvalues above 1e-13 of the largest
  if (rc == ROM_OK) {
    const double top = D[ns - 1];
    int rank = 0;
    for (int j = 0; j < ns; ++j) rank += D[j] > top * 1e-13;
    if (!(top > 0) || n > rank) rc = ROM_EINVAL;
  }
  if (rc == ROM_OK) {
    k_select<<<nblk(std::max<long>((long)n * ns, ns)), 256, 0, stream>>>(ns, n, w.D, w.C, lambda_dev, w.WT);
    // phi [n][nrow] = WT S (mode k = sum_j WT[k][j] s_j)
    gemm.run<false>(n, nrow, ns, w.WT, ns, S_dev, nrow, modes_dev, stream);
    // G = phi^T M phi, Cholesky, phi <- phi L^-T
    weight(modes_dev, w.MS, n);
    gemm.run<true>(n, n, nrow, modes_dev, nrow, w.MS, nrow, w.G, stream);
    k_symmetrize<<<nblk((long)n * n), 256, 0, stream>>>(n, w.G);
    if (hipGetLastError() != hipSuccess ||
        rocsolver_dpotrf(rb, rocblas_fill_lower, n, w.G, n, w.info) != rocblas_status_success)
      rc = ROM_EHIP;
    if (rc == ROM_OK) {
      k_trsm_rows<<<nblk(nrow), 256, 0, stream>>>(nrow, n, w.G, modes_dev);
      if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&info, w.info, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess)
        rc = ROM_EHIP;
      else if (info != 0)
        rc = ROM_EHIP;
    }
  }
  rocblas_destroy_handle(rb);
  return rc;
}


int rom_ecm_workspace(int32_t R, int32_t nq, int32_t m_max, size_t* bytes) {
  if (!bytes || R < 1 || nq < 1 || m_max < 1 || m_max > ECM_MMAX) return ROM_EINVAL;
  *bytes = ecm_layout(R, nq, m_max, nullptr, nullptr);
  return ROM_OK;
}

int rom_ecm(int32_t R, int32_t nq, const double* J_dev, const double* w_dev, double eps, int32_t m_max,
            int32_t* idx_dev, double* weights_dev, int32_t* m_out, double* hist_host, int32_t hist_cap,
            int32_t* hist_len, int32_t* rank_out, void* work_dev, size_t work_bytes, hipStream_t stream) {
  if (R < 1 || nq < 1 || !J_dev || !w_dev || !(eps >= 0) || m_max < 1 || m_max > ECM_MMAX || !idx_dev ||
      !weights_dev || !m_out || !work_dev)
    return ROM_EINVAL;
  if (work_bytes < ecm_layout(R, nq, m_max, nullptr, nullptr)) return ROM_EINVAL;
  EcmWork e;
  ecm_layout(R, nq, m_max, &e, (char*)work_dev);
  const int mn = std::min(R, nq), nblocks = (nq + ECM_SCORE_BLOCK - 1) / ECM_SCORE_BLOCK;
  // singular values and right singular vectors of Jh = J diag(sqrt(w)).
  // With no more integrands than points (the usual case) the tall transpose
  // is reduced first: Jh^T = Q Rm (Householder QR), Rm = U_R S V_R^T, so
  // that Jh = V_R S (Q U_R)^T and the right singular vectors are the columns
  // of Q U_R; only the R x R factor goes through the SVD.
  const bool tall = R <= nq;
  if (tall)
    k_ecm_scale_t<<<nblk((long)R * nq), 256, 0, stream>>>(R, nq, J_dev, w_dev, e.Jh);
  else
    k_ecm_scale<<<nblk((long)R * nq), 256, 0, stream>>>(R, nq, J_dev, w_dev, e.Jh);
  if (hipGetLastError() != hipSuccess) return ROM_EHIP;
  rocblas_handle rb;
  if (rocblas_create_handle(&rb) != rocblas_status_success) return ROM_EHIP;
  int rc = ROM_OK;
  if (rocblas_set_stream(rb, stream) != rocblas_status_success) rc = ROM_EHIP;
  if (rc == ROM_OK && tall) {
    if (rocsolver_dgeqrf(rb, nq, R, e.Jh, nq, e.tau) != rocblas_status_success) rc = ROM_EHIP;
    if (rc == ROM_OK) {
      k_copy_r<<<nblk((long)R * R), 256, 0, stream>>>(R, nq, e.Jh, e.Rm);
      if (hipGetLastError() != hipSuccess ||
          rocsolver_dorgqr(rb, nq, R, R, e.Jh, nq, e.tau) != rocblas_status_success ||
          rocsolver_dgesdd(rb, rocblas_svect_singular, rocblas_svect_none, R, R, e.Rm, R, e.Sv, e.U, R, nullptr, 1,
                           e.info) != rocblas_status_success)
        rc = ROM_EHIP;
    }
  } else if (rc == ROM_OK &&
             rocsolver_dgesvd(rb, rocblas_svect_none, rocblas_svect_singular, R, nq, e.Jh, R, e.Sv, nullptr, 1, e.V,
                              mn, e.E, rocblas_outofplace, e.info) != rocblas_status_success) {
    rc = ROM_EHIP;
  }
  std::vector<double> sv(mn);
  int info = 0;
  if (rc == ROM_OK && (hipMemcpyAsync(sv.data(), e.Sv, 8L * mn, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                       hipMemcpyAsync(&info, e.info, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                       hipStreamSynchronize(stream) != hipSuccess))
    rc = ROM_EHIP;
  rocblas_destroy_handle(rb);
  if (rc != ROM_OK) return rc;
  if (info != 0) return ROM_EHIP;
  int r = 0;
  for (int i = 0; i < mn; ++i) r += sv[i] > 1e-12 * sv[0];
  if (rank_out) *rank_out = r;
  if (r < 1) return ROM_EINVAL;
  // Z, column norms, b = Z w, |b|; empty selection, res = b
  if (tall) {
    // V^T (row-major r x nq) = U_R(:, :r)^T Q^T: one MFMA pass over Q
    dim3 grid((nq + 63) / 64, (r + 63) / 64, 1);
    k_gemm_f64<false><<<grid, 256, 0, stream>>>(r, nq, R, e.U, R, e.Jh, nq, e.V, nq, (R + 15) / 16 * 16, 0);
    k_ecm_z_rows<<<nblk(nq), 256, 0, stream>>>(r, nq, e.V, w_dev, e.Zr, e.cn);
  } else {
    k_ecm_z<<<nblk(nq), 256, 0, stream>>>(mn, r, nq, e.V, w_dev, e.Zr, e.cn);
  }
  k_ecm_b<<<r, 256, 0, stream>>>(nq, e.Zr, w_dev, e.b);
  k_norm<<<1, 256, 0, stream>>>(r, e.b, e.bn);
  EcmState st0{0, 0, -1, 0, 0.0, 0.0};
  if (hipMemsetAsync(e.sel, 0, 4L * nq, stream) != hipSuccess ||
      hipMemcpyAsync(e.res, e.b, 8L * r, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(e.st, &st0, sizeof(st0), hipMemcpyHostToDevice, stream) != hipSuccess)
    return ROM_EHIP;
  double bn = 0.0;
  if (hipMemcpyAsync(&bn, e.bn, 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return ROM_EHIP;
  const size_t sh_update = 8 * (3 * (size_t)(m_max + 1) + 32 + TRI_NB * TRI_LD) + 8 * (size_t)(m_max + 1);
  if (hipFuncSetAttribute((const void*)k_ecm_update, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh_update) !=
      hipSuccess)
    return ROM_EHIP;
  int hl = 0;
  if (hist_host && hist_cap > 0) hist_host[hl++] = 1.0;
  EcmState st = st0;
  st.rn = bn;
  long n_iter = 0;
  while (st.rn > eps * bn && st.k < m_max && n_iter < 10L * m_max) {
    ++n_iter;
    k_ecm_score<<<nblocks, ECM_SCORE_BLOCK, 8 * (size_t)r, stream>>>(r, nq, e.Zr, e.cn, e.res, e.sel, e.bv, e.bi);
    k_ecm_update<<<1, ECM_THREADS, sh_update, stream>>>(r, nq, m_max, nblocks, e.Zr, e.b, e.bv, e.bi, e.S, e.ZS, e.G,
                                                        e.Lm, e.Gp, e.Lp, e.hv, e.yv, e.w, e.res, e.sel,
                                                        e.st);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&st, e.st, sizeof(st), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return ROM_EHIP;
    if (st.status != 0) break;
    if (hist_host && hl < hist_cap) hist_host[hl++] = st.rn / bn;
  }
  if (hist_len) *hist_len = hl;
  *m_out = st.k;
  if (st.k > 0 && (hipMemcpyAsync(idx_dev, e.S, 4L * st.k, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
                   hipMemcpyAsync(weights_dev, e.w, 8L * st.k, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
                   hipStreamSynchronize(stream) != hipSuccess))
    return ROM_EHIP;
  return st.status == 2 ? ROM_EUNSUPPORTED : ROM_OK;
}

}  // extern "C"
