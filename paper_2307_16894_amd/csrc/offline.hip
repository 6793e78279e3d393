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

}  // extern "C"
