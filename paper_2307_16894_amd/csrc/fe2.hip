// Macro side of the two-scale problem (Sec. 4.2): a block of eight-node
// quadrilaterals with 2 x 2 Gauss points, whose quadrature points are the
// batch of the reduced RVE solve.  Total Lagrangian, plane strain: the macro
// deformation gradient at a point is Fbar = I + sum_a u_a (x) dN_a/dX, the
// internal force sum_p B_p^T Pbar_p w|J|, the tangent sum_p B_p^T Abar_p B_p
// w|J| with Pbar and Abar of the RVE (eqs. eff_stress_1, eff_stiffness_1).
// The top edge carries the downward traction T(x) = Tbar (1 - (2x/W - 1)^2)
// as a dead load; the compliance is the work of that load.
//
// Layout: nodes numbered by the caller (a numbering with a small bandwidth
// keeps the banded solve short), dofs 2 n + i, quadrature points p = 4 e + g.
// The free-dof stiffness is held as a band of kl sub- and kl + kl super-
// diagonals (room for the fill of row interchanges), row-major: row r keeps
// columns r - kl .. r + 2 kl at offset c - r + kl.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "podecm.h"

typedef double d4 __attribute__((ext_vector_type(4)));

struct rom_fe2 {
  int device;
  int nodes, elements, points, dofs, nfixed, nfree, ntop, kl, ldab;
  int stage;  // rows per LDS staging block of the LDS-window solve (0: the global-memory solve)
  double width;
  // device
  double *X, *dNdX, *wJ, *Xg, *band, *rhs, *ubuf, *xbuf;  // ubuf, xbuf: the LDS-window solve
  double *lbuf, *ybuf;  // blocked Cholesky (kl <= its limit): factor panels, solution; null otherwise
  int* done;            // 1 when the blocked Cholesky has solved the current system
  int *conn, *node_ptr, *node_ent, *dofmap, *fixed, *top;
};

namespace {

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

// parent coordinates of the eight nodes: corners counterclockwise from
// (-1, -1), then midsides of the bottom, right, top and left edges
__constant__ double c_node_xi[8] = {-1, 1, 1, -1, 0, 1, 0, -1};
__constant__ double c_node_eta[8] = {-1, -1, 1, 1, -1, 0, 1, 0};

// serendipity shape function of node a and its parent derivatives
__device__ void q8(int a, double xi, double eta, double& N, double& dxi, double& deta) {
  const double xa = c_node_xi[a], ea = c_node_eta[a];
  if (xa != 0.0 && ea != 0.0) {
    const double sx = 1.0 + xi * xa, se = 1.0 + eta * ea, t = xi * xa + eta * ea - 1.0;
    N = 0.25 * sx * se * t;
    dxi = 0.25 * xa * se * (t + sx);
    deta = 0.25 * ea * sx * (t + se);
  } else if (xa == 0.0) {
    const double se = 1.0 + eta * ea;
    N = 0.5 * (1.0 - xi * xi) * se;
    dxi = -xi * se;
    deta = 0.5 * ea * (1.0 - xi * xi);
  } else {
    const double sx = 1.0 + xi * xa;
    N = 0.5 * sx * (1.0 - eta * eta);
    dxi = 0.5 * xa * (1.0 - eta * eta);
    deta = -eta * sx;
  }
}

// per point: dN/dX [p][8][2], weight x det J (unit Gauss weights), position
__global__ void k_geometry(int points, const double* __restrict__ X, const int* __restrict__ conn,
                           double* __restrict__ dNdX, double* __restrict__ wJ, double* __restrict__ Xg) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= points) return;
  const int e = p >> 2, g = p & 3;
  const double s = 1.0 / sqrt(3.0);
  const double xi = (g == 0 || g == 3) ? -s : s, eta = (g < 2) ? -s : s;
  double dxi[8], deta[8], J00 = 0, J01 = 0, J10 = 0, J11 = 0, x = 0, y = 0;
  for (int a = 0; a < 8; ++a) {
    double N;
    q8(a, xi, eta, N, dxi[a], deta[a]);
    const int n = conn[8 * e + a];
    const double Xa = X[2 * n], Ya = X[2 * n + 1];
    J00 += Xa * dxi[a];  // dX / dxi
    J01 += Xa * deta[a];
    J10 += Ya * dxi[a];
    J11 += Ya * deta[a];
    x += N * Xa;
    y += N * Ya;
  }
  const double det = J00 * J11 - J01 * J10, inv = 1.0 / det;
  // dN/dX_J = dN/dxi_j (J^-1)_jJ
  for (int a = 0; a < 8; ++a) {
    dNdX[(size_t)p * 16 + 2 * a] = (dxi[a] * J11 - deta[a] * J10) * inv;
    dNdX[(size_t)p * 16 + 2 * a + 1] = (-dxi[a] * J01 + deta[a] * J00) * inv;
  }
  wJ[p] = det;
  Xg[2 * p] = x;
  Xg[2 * p + 1] = y;
}

__global__ void k_gradient(int points, const int* __restrict__ conn, const double* __restrict__ dNdX,
                           const double* __restrict__ u, double* __restrict__ F) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= points) return;
  const int e = p >> 2;
  double f[4] = {1.0, 0.0, 0.0, 1.0};
  for (int a = 0; a < 8; ++a) {
    const int n = conn[8 * e + a];
    const double gx = dNdX[(size_t)p * 16 + 2 * a], gy = dNdX[(size_t)p * 16 + 2 * a + 1];
    const double ux = u[2 * n], uy = u[2 * n + 1];
    f[0] = fma(ux, gx, f[0]);
    f[1] = fma(ux, gy, f[1]);
    f[2] = fma(uy, gx, f[2]);
    f[3] = fma(uy, gy, f[3]);
  }
  for (int c = 0; c < 4; ++c) F[4 * (size_t)p + c] = f[c];
}

// three-point Gauss rule on a quadratic edge, nodes (left, middle, right)
__device__ void edge_rule(int q, double& s, double& w) {
  const double r = sqrt(0.6);
  s = (q == 0) ? -r : (q == 1 ? 0.0 : r);
  w = (q == 1) ? 8.0 / 9.0 : 5.0 / 9.0;
}
__device__ void edge_shape(double s, double N[3], double dN[3]) {
  N[0] = 0.5 * s * (s - 1.0);
  N[1] = 1.0 - s * s;
  N[2] = 0.5 * s * (s + 1.0);
  dN[0] = s - 0.5;
  dN[1] = -2.0 * s;
  dN[2] = s + 0.5;
}

// one workgroup: zero f_ext, then one lane adds the edges in order (the
// corner nodes are shared by neighbouring edges)
__global__ void k_traction(int dofs, int ntop, const int* __restrict__ top, const double* __restrict__ X,
                           double Tbar, double width, double* __restrict__ fext) {
  for (int d = threadIdx.x; d < dofs; d += blockDim.x) fext[d] = 0.0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int t = 0; t < ntop; ++t) {
    const int nd[3] = {top[3 * t], top[3 * t + 1], top[3 * t + 2]};
    const double xs[3] = {X[2 * nd[0]], X[2 * nd[1]], X[2 * nd[2]]};
    for (int q = 0; q < 3; ++q) {
      double s, w, N[3], dN[3];
      edge_rule(q, s, w);
      edge_shape(s, N, dN);
      const double x = N[0] * xs[0] + N[1] * xs[1] + N[2] * xs[2];
      const double jac = fabs(dN[0] * xs[0] + dN[1] * xs[1] + dN[2] * xs[2]);
      const double xr = 2.0 * x / width - 1.0, T = Tbar * (1.0 - xr * xr);
      for (int a = 0; a < 3; ++a) fext[2 * nd[a] + 1] -= N[a] * T * jac * w;
    }
  }
}

__global__ void k_compliance(int ntop, const int* __restrict__ top, const double* __restrict__ X, double Tbar,
                             double width, const double* __restrict__ u, double* __restrict__ C) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double c = 0.0;
  for (int t = 0; t < ntop; ++t) {
    const int nd[3] = {top[3 * t], top[3 * t + 1], top[3 * t + 2]};
    const double xs[3] = {X[2 * nd[0]], X[2 * nd[1]], X[2 * nd[2]]};
    const double uy[3] = {u[2 * nd[0] + 1], u[2 * nd[1] + 1], u[2 * nd[2] + 1]};
    for (int q = 0; q < 3; ++q) {
      double s, w, N[3], dN[3];
      edge_rule(q, s, w);
      edge_shape(s, N, dN);
      const double x = N[0] * xs[0] + N[1] * xs[1] + N[2] * xs[2];
      const double jac = fabs(dN[0] * xs[0] + dN[1] * xs[1] + dN[2] * xs[2]);
      const double xr = 2.0 * x / width - 1.0, T = Tbar * (1.0 - xr * xr);
      c -= T * (N[0] * uy[0] + N[1] * uy[1] + N[2] * uy[2]) * jac * w;
    }
  }
  *C = c;
}

// res[d] = f_ext[d] - f_int[d]; lane per dof, gathering the (element, local
// node) entries of its node in a fixed order
__global__ void k_residual(int dofs, const int* __restrict__ node_ptr, const int* __restrict__ node_ent,
                           const double* __restrict__ dNdX, const double* __restrict__ wJ,
                           const double* __restrict__ Pbar, const double* __restrict__ fext, double* __restrict__ res) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= dofs) return;
  const int n = d >> 1, i = d & 1;
  double f = 0.0;
  for (int k = node_ptr[n]; k < node_ptr[n + 1]; ++k) {
    const int e = node_ent[k] >> 3, a = node_ent[k] & 7;
    for (int g = 0; g < 4; ++g) {
      const int p = 4 * e + g;
      const double* G = dNdX + (size_t)p * 16 + 2 * a;
      f = fma((Pbar[4 * (size_t)p + 2 * i] * G[0] + Pbar[4 * (size_t)p + 2 * i + 1] * G[1]), wJ[p], f);
    }
  }
  res[d] = fext[d] - f;
}

// norms[0] = ||res||_2, norms[1] = ||f_ext||_2 over the free dofs (one
// workgroup of 256, fixed-order tree)
__global__ __launch_bounds__(256) void k_norms(int dofs, const int* __restrict__ dofmap,
                                               const double* __restrict__ res, const double* __restrict__ fext,
                                               double* __restrict__ norms) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  for (int d = threadIdx.x; d < dofs; d += 256)
    if (dofmap[d] >= 0) {
      a = fma(res[d], res[d], a);
      b = fma(fext[d], fext[d], b);
    }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      s0[threadIdx.x] += s0[threadIdx.x + h];
      s1[threadIdx.x] += s1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    norms[0] = sqrt(s0[0]);
    norms[1] = sqrt(s1[0]);
  }
}

// Band of the free-dof tangent and right-hand side r_f - K_fd du_d: lane per
// free row, its band row zeroed and then gathered from the points of the
// elements that hold its node.
__global__ void k_assemble(int dofs, int kl, int ldab, const int* __restrict__ node_ptr,
                           const int* __restrict__ node_ent, const int* __restrict__ conn,
                           const int* __restrict__ dofmap, const double* __restrict__ dNdX,
                           const double* __restrict__ wJ, const double* __restrict__ Abar,
                           const double* __restrict__ res, const double* __restrict__ dud, double* __restrict__ band,
                           double* __restrict__ rhs) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= dofs) return;
  const int r = dofmap[d];
  if (r < 0) return;
  double* row = band + (size_t)r * ldab;
  for (int c = 0; c < ldab; ++c) row[c] = 0.0;
  double b = res[d];
  const int n = d >> 1, i = d & 1;
  for (int k = node_ptr[n]; k < node_ptr[n + 1]; ++k) {
    const int e = node_ent[k] >> 3, a = node_ent[k] & 7;
    for (int g = 0; g < 4; ++g) {
      const int p = 4 * e + g;
      const double* G = dNdX + (size_t)p * 16;
      const double* A = Abar + (size_t)p * 16;
      // row of B^T Abar for (a, i): v_kL = sum_J dN_a/dX_J A[iJ, kL] w|J|
      double v[4];
      for (int kL = 0; kL < 4; ++kL) v[kL] = (G[2 * a] * A[(2 * i) * 4 + kL] + G[2 * a + 1] * A[(2 * i + 1) * 4 + kL]) * wJ[p];
      for (int bn = 0; bn < 8; ++bn) {
        const int col_node = conn[8 * e + bn];
        for (int kk = 0; kk < 2; ++kk) {
          const double kv = v[2 * kk] * G[2 * bn] + v[2 * kk + 1] * G[2 * bn + 1];
          const int c = dofmap[2 * col_node + kk];
          if (c >= 0)
            row[c - r + kl] += kv;
          else if (dud)
            b -= kv * dud[-1 - c];
        }
      }
    }
  }
  rhs[r] = b;
}

// Banded LU with partial pivoting of the free-dof tangent, the row
// operations applied to the right-hand side as they are made, then back
// substitution; u_f += x, u_d += du_d.  One workgroup; info = 0, or k + 1 at
// a zero pivot in column k (u is then left unchanged).
constexpr int LU_THREADS = 1024;
__global__ __launch_bounds__(LU_THREADS) void k_band_solve(int nf, int kl, int ldab, double* __restrict__ band,
                                                           double* __restrict__ rhs, int dofs,
                                                           const int* __restrict__ dofmap, const int* __restrict__ fixed,
                                                           int nfixed, const double* __restrict__ dud,
                                                           double* __restrict__ u, int* __restrict__ info,
                                                           const int* __restrict__ done) {
  if (done && *done) return;  // solved by the blocked Cholesky
  __shared__ double s_mult[256];
  __shared__ int s_piv;
  __shared__ double s_pv;
  const int tid = threadIdx.x, ku = 2 * kl;
  auto at = [&](int rr, int c) -> double& { return band[(size_t)rr * ldab + (c - rr + kl)]; };
  for (int k = 0; k < nf; ++k) {
    const int last = min(nf - 1, k + kl);
    // pivot: the largest |a_ik| over i = k .. last, first on ties (wave 0)
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i <= last; i += 64) {
        const double v = fabs(at(i, k));
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) s_piv = bi;
    }
    __syncthreads();
    const int pr = s_piv;
    const int cend = min(nf - 1, k + ku);
    if (pr != k) {
      for (int c = k + tid; c <= cend; c += LU_THREADS) {
        const double t = at(k, c);
        at(k, c) = at(pr, c);
        at(pr, c) = t;
      }
      if (tid == 0) {
        const double t = rhs[k];
        rhs[k] = rhs[pr];
        rhs[pr] = t;
      }
    }
    __syncthreads();
    if (tid == 0) s_pv = at(k, k);
    __syncthreads();
    const double pv = s_pv;
    if (pv == 0.0) {
      if (tid == 0) *info = k + 1;
      return;
    }
    for (int i = k + 1 + tid; i <= last; i += LU_THREADS) s_mult[i - k - 1] = at(i, k) / pv;
    __syncthreads();
    const int rows = last - k, cols = cend - k;
    for (int t = tid; t < rows * cols; t += LU_THREADS) {
      const int i = k + 1 + t / cols, c = k + 1 + t % cols;
      at(i, c) = fma(-s_mult[i - k - 1], at(k, c), at(i, c));
    }
    for (int i = k + 1 + tid; i <= last; i += LU_THREADS) rhs[i] = fma(-s_mult[i - k - 1], rhs[k], rhs[i]);
    __syncthreads();
  }
  // back substitution on U (upper bandwidth 2 kl), one row at a time
  __shared__ double s_red[LU_THREADS / 64];
  for (int k = nf - 1; k >= 0; --k) {
    const int cend = min(nf - 1, k + ku);
    double s = 0.0;
    for (int c = k + 1 + tid; c <= cend; c += LU_THREADS) s = fma(at(k, c), rhs[c], s);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((tid & 63) == 0) s_red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < LU_THREADS / 64; ++w) t += s_red[w];
      rhs[k] = (rhs[k] - t) / at(k, k);
    }
    __syncthreads();
  }
  for (int d = tid; d < dofs; d += LU_THREADS) {
    const int r = dofmap[d];
    if (r >= 0) u[d] += rhs[r];
  }
  if (dud)
    for (int j = tid; j < nfixed; j += LU_THREADS) u[fixed[j]] += dud[j];
  if (tid == 0) *info = 0;
}

// The same factorisation with the active window in LDS: the rows k .. k +
// kl + 1 of step k, each holding its columns c .. c + 2 kl (position c mod
// Wc, Wc = 2 kl + 1) and its right-hand side (position Wc).  Row r lives in
// slot map[r mod (kl + 2)]; a row interchange swaps two map entries, and the
// row entering at step k takes the map entry (and the slot) of row k - 1,
// which left the window the step before.  Step k: wave 0 picks the pivot and
// swaps the map entries; the multipliers and slot offsets of the rows below;
// then the update of those rows by 4 (2 kl + 2) threads, each holding one
// column position (the right-hand side as one more) for every fourth row,
// while row k of U is copied out, column k of the rows below is cleared and
// row k + kl + 1 is copied in.  Rows in and out go through LDS staging blocks
// of B rows, moved to and from HBM once per B steps, so that no step waits
// on global memory.  Back substitution: blocks of kl + 2 rows of U and their
// right-hand sides staged in LDS, then one wave walks them, lane l holding
// x[k + 1 + l + 64 j] (j = 0, 1, 2) and the sum over the row by a wave
// reduction.  Needs 2 kl + 1 <= 192 and B >= 1.
constexpr int LDS_KL_MAX = 95;
constexpr int LDS_THREADS_MAX = 1024;  // 4 (2 kl + 2) threads rounded up to whole waves
constexpr int LDS_UNROLL = 4;
constexpr int LDS_STAGE_MAX = 32;
constexpr size_t LDS_BYTES_MAX = 160 * 1024;

size_t band_lds_bytes(int kl, int B) {
  const size_t S = kl + 2, RW = 2 * kl + 2;
  return 8 * (S * RW + 2 * (size_t)B * RW + kl + 1) + 4 * (size_t)(2 * kl + 3);
}
int band_stage_rows(int kl) {
  int B = LDS_STAGE_MAX;
  while (B > 0 && band_lds_bytes(kl, B) > LDS_BYTES_MAX) --B;
  return B;
}

__device__ void band_lu_lds(int nf, int kl, int ldab, int B, const double* __restrict__ band,
                            const double* __restrict__ rhs_in, double* __restrict__ ubuf, double* __restrict__ x,
                            int dofs, const int* __restrict__ dofmap, const int* __restrict__ fixed, int nfixed,
                            const double* __restrict__ dud, double* __restrict__ u, int* __restrict__ info,
                            double* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nt = blockDim.x;
  const int Wc = 2 * kl + 1, S = kl + 2, RW = Wc + 1;
  double* win = lds;                          // [S][RW]
  double* sin = win + (size_t)S * RW;         // [B][RW] rows about to enter (band columns r - kl .. r + kl, rhs)
  double* sout = sin + (size_t)B * RW;        // [B][RW] rows of U that left (columns k .. k + 2 kl, rhs)
  double* s_mult = sout + (size_t)B * RW;     // [kl + 1]
  int* s_off = (int*)(s_mult + kl + 1);       // [kl + 1] slot offsets of the rows below the pivot
  int* map = s_off + kl + 1;                  // [S]
  for (int t = tid; t < S * RW; t += nt) win[t] = 0.0;
  for (int t = tid; t < S; t += nt) map[t] = t;
  __syncthreads();
  // rows 0 .. kl: columns max(0, r - kl) .. r + kl
  for (int t = tid; t < (kl + 1) * RW; t += nt) {
    const int r = t / RW, j = t % RW;
    if (r >= nf) continue;
    double* row = win + (size_t)map[r % S] * RW;
    if (j == Wc) {
      row[Wc] = rhs_in[r];
    } else {
      const int c = r - kl + j;
      if (c >= 0) row[c % Wc] = band[(size_t)r * ldab + j];
    }
  }
  int kw = 0;  // k mod Wc
  for (int k = 0; k < nf; ++k) {
    const int kb = k % B;
    if (kb == 0) {
      // rows of U of the last block out, rows k + kl + 1 .. k + kl + B in
      for (int t = tid; t < B * RW && k > 0; t += nt) {
        const int r = k - B + t / RW, j = t % RW;
        if (j == Wc)
          x[r] = sout[t];
        else
          ubuf[(size_t)r * Wc + j] = sout[t];
      }
      for (int t = tid; t < B * RW; t += nt) {
        const int r = k + kl + 1 + t / RW, j = t % RW;
        if (r < nf) sin[t] = (j == Wc) ? rhs_in[r] : band[(size_t)r * ldab + j];
      }
      __syncthreads();
    }
    const int last = min(nf - 1, k + kl), nr = last - k, cend = min(nf - 1, k + 2 * kl), ncol = cend - k;
    if (wave == 0) {
      double best = -1.0;
      int bi = k;
      for (int i = k + lane; i <= last; i += 64) {
        const double v = fabs(win[(size_t)map[i % S] * RW + kw]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0 && bi != k) {
        const int a = map[k % S];
        map[k % S] = map[bi % S];
        map[bi % S] = a;
      }
    }
    __syncthreads();
    const int poff = map[k % S] * RW;
    const double pv = win[poff + kw];
    if (pv == 0.0) {
      if (tid == 0) *info = k + 1;
      return;
    }
    for (int i = tid; i < nr; i += nt) {
      const int o = map[(k + 1 + i) % S] * RW;
      s_off[i] = o;
      s_mult[i] = win[o + kw] / pv;
    }
    __syncthreads();
    // update: thread (g, p) takes position p of rows g, g + 4, ... below the
    // pivot (position Wc the right-hand side), four rows in flight (loads
    // before stores); a wave reads consecutive LDS words and broadcasts the
    // row offsets and multipliers
    {
      const int g = tid / RW, p = tid - g * RW;
      int q = p - kw - 1;
      q = (q < 0) ? q + Wc : q;
      if (g >= 4) {
        // threads beyond 4 (2 kl + 2): the launch is rounded up to whole waves
      } else if (p == Wc || q < ncol) {
        const double a = win[poff + p];
        for (int i0 = g; i0 < nr; i0 += 4 * LDS_UNROLL) {
          int o[LDS_UNROLL];
          double m[LDS_UNROLL], v[LDS_UNROLL];
#pragma unroll
          for (int w = 0; w < LDS_UNROLL; ++w) {
            const int i = i0 + 4 * w;
            o[w] = (i < nr) ? s_off[i] + p : -1;
            m[w] = (i < nr) ? s_mult[i] : 0.0;
          }
#pragma unroll
          for (int w = 0; w < LDS_UNROLL; ++w) v[w] = (o[w] >= 0) ? win[o[w]] : 0.0;
#pragma unroll
          for (int w = 0; w < LDS_UNROLL; ++w)
            if (o[w] >= 0) win[o[w]] = fma(-m[w], a, v[w]);
        }
      } else if (p == kw) {
        // column k of the rows below (never among the updated positions)
        for (int i = g; i < nr; i += 4) win[s_off[i] + kw] = 0.0;
      }
    }
    // row k of U (columns k .. k + 2 kl) and its right-hand side out; row
    // k + kl + 1 in, to the slot of row k - 1 (it left the window last step;
    // at k = 0 the spare slot), which no row k .. k + kl uses
    for (int j = tid; j < RW; j += nt) {
      int p = kw + j;
      p = (p >= Wc) ? p - Wc : p;
      sout[(size_t)kb * RW + j] = (j == Wc) ? win[poff + Wc] : ((k + j <= cend) ? win[poff + p] : 0.0);
    }
    const int rn = k + kl + 1;
    if (rn < nf) {
      double* row = win + (size_t)map[rn % S] * RW;
      const double* src = sin + (size_t)kb * RW;
      for (int j = tid; j < RW; j += nt) row[j == Wc ? Wc : (rn - kl + j) % Wc] = src[j];
    }
    __syncthreads();
    kw = (kw + 1 == Wc) ? 0 : kw + 1;
  }
  {  // the last, partial block of U out
    const int k0 = ((nf - 1) / B) * B, rows = nf - k0;
    for (int t = tid; t < rows * RW; t += nt) {
      const int r = k0 + t / RW, j = t % RW;
      if (j == Wc)
        x[r] = sout[t];
      else
        ubuf[(size_t)r * Wc + j] = sout[t];
    }
  }
  __syncthreads();
  // back substitution; x[] holds the forward-eliminated right-hand side
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;  // x[k + 1 + lane + 64 j]
  double* yb = win + (size_t)S * Wc;      // [S] right-hand sides of the block
  for (int kb = nf - 1; kb >= 0; kb -= S) {
    const int k0 = max(0, kb - S + 1), rows = kb - k0 + 1;
    for (int t = tid; t < rows * Wc; t += nt) win[t] = ubuf[(size_t)k0 * Wc + t];
    for (int t = tid; t < rows; t += nt) yb[t] = x[k0 + t];
    __syncthreads();
    if (wave == 0) {
      for (int k = kb; k >= k0; --k) {
        const double* U = win + (size_t)(k - k0) * Wc;
        const int jm = min(2 * kl, nf - 1 - k);
        double s = 0.0;
        if (lane + 1 <= jm) s = U[lane + 1] * r0;
        if (lane + 65 <= jm) s = fma(U[lane + 65], r1, s);
        if (lane + 129 <= jm) s = fma(U[lane + 129], r2, s);
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        const double xk = (yb[k - k0] - s) / U[0];
        const double t0 = __shfl(r0, 63), t1 = __shfl(r1, 63);
        r2 = __shfl_up(r2, 1);
        r1 = __shfl_up(r1, 1);
        r0 = __shfl_up(r0, 1);
        if (lane == 0) {
          r2 = t1;
          r1 = t0;
          r0 = xk;
          x[k] = xk;
        }
      }
    }
    __syncthreads();
  }
  for (int d = tid; d < dofs; d += nt) {
    const int r = dofmap[d];
    if (r >= 0) u[d] += x[r];
  }
  if (dud)
    for (int j = tid; j < nfixed; j += nt) u[fixed[j]] += dud[j];
  if (tid == 0) *info = 0;
}

// Banded Cholesky L L^T of the free-dof tangent (symmetric; positive
// definite while the material hardens), no row interchanges, blocked by
// panels of CH_NB columns.  The window holds rows k .. k + kl + CH_NB - 1
// with their columns from k up to the row (position c mod W, W = kl + CH_NB)
// and right-hand side (position W), row r in slot r mod W.  Panel k .. ke-1:
// one wave factors its columns (pivot, column of L, forward substitution of
// the right-hand side, update of the panel's later columns), with no
// workgroup barrier; then all threads apply the rank-CH_NB update to the
// rows and columns below the panel (a lane per column, all lanes of a wave
// on the same row, so the row's panel entries are broadcast and its column
// entries come from registers); the panel's columns of L go out and the next
// CH_NB rows come in through the staging blocks.  Back substitution with L^T
// as in the LU form.  Returns false (u untouched) at a pivot that is not
// positive.
constexpr int CH_NB = 8;
constexpr int CH_STAGE = 32;  // staging block, a multiple of CH_NB

size_t chol_lds_bytes(int kl) {
  const size_t W = kl + CH_NB, RW = W + 1, RB = kl + 2;
  return 8 * (W * RW + 2 * (size_t)CH_STAGE * RB) + 64;
}

__device__ bool band_chol_lds(int nf, int kl, int ldab, const double* __restrict__ band,
                              const double* __restrict__ rhs_in, double* __restrict__ ubuf, double* __restrict__ x,
                              double* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nt = blockDim.x;
  const int W = kl + CH_NB, S = W, RW = W + 1, RB = kl + 2;
  double* win = lds;                                  // [S][RW]
  double* sin = win + (size_t)S * RW;                 // [CH_STAGE][RB] rows about to enter: columns r - kl .. r, rhs
  double* sout = sin + (size_t)CH_STAGE * RB;         // [CH_STAGE][RB] columns of L that left: L(j + t, j), t = 0 .. kl; y_j
  __shared__ int s_fail;
  for (int t = tid; t < S * RW; t += nt) win[t] = 0.0;
  if (tid == 0) s_fail = 0;
  __syncthreads();
  for (int t = tid; t < W * (kl + 2); t += nt) {  // rows 0 .. W - 1
    const int r = t / (kl + 2), j = t % (kl + 2);
    if (r >= nf) continue;
    double* row = win + (size_t)(r % S) * RW;
    if (j == kl + 1) {
      row[W] = rhs_in[r];
    } else {
      const int c = r - kl + j;
      if (c >= 0) row[c % W] = band[(size_t)r * ldab + j];
    }
  }
  for (int k = 0; k < nf; k += CH_NB) {
    const int ke = min(k + CH_NB, nf), kb = k % CH_STAGE;
    if (kb == 0) {
      // the columns of the last block out; the rows entering during this block in
      for (int t = tid; t < CH_STAGE * RB && k > 0; t += nt) {
        const int j = k - CH_STAGE + t / RB, q = t % RB;
        if (q == kl + 1)
          x[j] = sout[t];
        else
          ubuf[(size_t)j * (kl + 1) + q] = sout[t];
      }
      for (int t = tid; t < CH_STAGE * RB; t += nt) {
        const int r = k + W + t / RB, q = t % RB;
        if (r < nf) sin[t] = (q == kl + 1) ? rhs_in[r] : band[(size_t)r * ldab + q];
      }
    }
    __syncthreads();
    if (wave == 0) {
      for (int j = k; j < ke; ++j) {
        const int sj = (j % S) * RW, pj = j % W, last = min(nf - 1, j + kl);
        const double d = win[sj + pj];
        if (!(d > 0.0)) {
          if (lane == 0) s_fail = 1;
          break;
        }
        const double sd = sqrt(d), isd = 1.0 / sd, yj = win[sj + W] * isd;
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
          win[sj + pj] = sd;
          win[sj + W] = yj;
        }
        for (int i = j + 1 + lane; i <= last; i += 64) {  // column j of L, forward substitution
          const int si = (i % S) * RW;
          const double l = win[si + pj] * isd;
          win[si + pj] = l;
          win[si + W] = fma(-l, yj, win[si + W]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int i = j + 1 + lane; i <= last; i += 64) {  // the panel's later columns c <= i
          const int si = (i % S) * RW;
          const double l = win[si + pj];
          // column c at position (= slot, S = W) pj + 1 + (c - j - 1), wrapped once
          int pc = pj + 1;
          for (int c = j + 1; c < ke && c <= i; ++c) {
            pc = (pc >= W) ? pc - W : pc;
            win[si + pc] = fma(-l, win[pc * RW + pj], win[si + pc]);
            ++pc;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    if (s_fail) return false;
    {
      // rank-CH_NB update: column c = ke + p, rows i = ke + g, ke + g + 4, ... with i >= c
      const int iend = min(nf - 1, k + kl + CH_NB - 1), ncols = iend - ke + 1;
      const int g = tid / W, p = tid - g * W;
      if (g < 4 && p < ncols) {
        // positions of the panel's columns (= slots, S = W), of column c and of row ke + g
        const int pk = k % W;
        int pp[CH_NB];
#pragma unroll
        for (int t = 0; t < CH_NB; ++t) pp[t] = (pk + t >= W) ? pk + t - W : pk + t;
        const int c = ke + p;
        int pc = pp[0] + (ke - k) + p;
        while (pc >= W) pc -= W;
        double lc[CH_NB];
#pragma unroll
        for (int t = 0; t < CH_NB; ++t) {
          const int j = k + t;
          lc[t] = (j < ke && c <= j + kl) ? win[pc * RW + pp[t]] : 0.0;
        }
        int sl = pp[0] + (ke - k) + g;  // slot of row i = ke + g, advanced by 4
        while (sl >= W) sl -= W;
        for (int i = ke + g; i <= iend; i += 4) {
          if (i >= c) {
            const int si = sl * RW;
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < CH_NB; ++t) {
              const int j = k + t;
              const double li = (j < ke && i <= j + kl) ? win[si + pp[t]] : 0.0;
              acc = fma(li, lc[t], acc);
            }
            win[si + pc] -= acc;
          }
          sl += 4;
          sl = (sl >= W) ? sl - W : sl;
        }
      }
      // the right-hand side of the rows below the panel was updated column by column in the panel
    }
    // the panel's columns of L and y out; rows ke + kl + CH_NB - ... : the next rows in
    for (int t = tid; t < (ke - k) * RB; t += nt) {
      const int j = k + t / RB, q = t % RB;
      sout[(size_t)(kb + t / RB) * RB + q] =
          (q == kl + 1) ? win[(j % S) * RW + W] : ((j + q < nf) ? win[((j + q) % S) * RW + j % W] : 0.0);
    }
    __syncthreads();
    for (int t = tid; t < (ke - k) * RB; t += nt) {
      const int r = k + W + t / RB, q = t % RB;
      if (r >= nf) continue;
      double* row = win + (size_t)(r % S) * RW;
      const double v = sin[(size_t)(kb + t / RB) * RB + q];
      if (q == kl + 1) {
        row[W] = v;
      } else {
        row[(r - kl + q) % W] = v;
      }
      if (q == 0)
        for (int z = r + 1; z < r + CH_NB; ++z) row[z % W] = 0.0;  // positions of columns beyond the row
    }
    __syncthreads();
  }
  {
    const int k0 = ((nf - 1) / CH_STAGE) * CH_STAGE, rows = nf - k0;
    for (int t = tid; t < rows * RB; t += nt) {
      const int j = k0 + t / RB, q = t % RB;
      if (q == kl + 1)
        x[j] = sout[t];
      else
        ubuf[(size_t)j * (kl + 1) + q] = sout[t];
    }
  }
  __syncthreads();
  // L^T x = y: x_k = (y_k - sum_j L(k + j, k) x_{k + j}) / L(k, k)
  const int Wl = kl + 1;
  double r0 = 0.0, r1 = 0.0;  // x[k + 1 + lane + 64 j]
  const int SB = (S * RW - 64) / (Wl + 1);  // rows of L^T per staged block
  double* yb = win + (size_t)SB * Wl;
  for (int kb = nf - 1; kb >= 0; kb -= SB) {
    const int k0 = max(0, kb - SB + 1), rows = kb - k0 + 1;
    for (int t = tid; t < rows * Wl; t += nt) win[t] = ubuf[(size_t)k0 * Wl + t];
    for (int t = tid; t < rows; t += nt) yb[t] = x[k0 + t];
    __syncthreads();
    if (wave == 0) {
      for (int k = kb; k >= k0; --k) {
        const double* Lc = win + (size_t)(k - k0) * Wl;
        const int jm = min(kl, nf - 1 - k);
        double sacc = 0.0;
        if (lane + 1 <= jm) sacc = Lc[lane + 1] * r0;
        if (lane + 65 <= jm) sacc = fma(Lc[lane + 65], r1, sacc);
        for (int off = 32; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off);
        const double xk = (yb[k - k0] - sacc) / Lc[0];
        const double t0 = __shfl(r0, 63);
        r1 = __shfl_up(r1, 1);
        r0 = __shfl_up(r0, 1);
        if (lane == 0) {
          r1 = t0;
          r0 = xk;
          x[k] = xk;
        }
      }
    }
    __syncthreads();
  }
  return true;
}

// LDS of the solve: the Cholesky form's or the LU form's, whichever is larger
size_t solve_lds_bytes(int kl, int B) { return std::max(band_lds_bytes(kl, B), chol_lds_bytes(kl)); }

__global__ __launch_bounds__(LDS_THREADS_MAX) void k_band_solve_lds(
    int nf, int kl, int ldab, int B, const double* __restrict__ band, const double* __restrict__ rhs_in,
    double* __restrict__ ubuf, double* __restrict__ x, int dofs, const int* __restrict__ dofmap,
    const int* __restrict__ fixed, int nfixed, const double* __restrict__ dud, double* __restrict__ u,
    int* __restrict__ info, const int* __restrict__ done) {
  if (done && *done) return;  // solved by the blocked Cholesky
  extern __shared__ double lds[];
  if (band_chol_lds(nf, kl, ldab, band, rhs_in, ubuf, x, lds)) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int d = tid; d < dofs; d += nt) {
      const int r = dofmap[d];
      if (r >= 0) u[d] += x[r];
    }
    if (dud)
      for (int j = tid; j < nfixed; j += nt) u[fixed[j]] += dud[j];
    if (tid == 0) *info = 0;
    return;
  }
  __syncthreads();
  band_lu_lds(nf, kl, ldab, B, band, rhs_in, ubuf, x, dofs, dofmap, fixed, nfixed, dud, u, info, lds);
}

// Blocked banded Cholesky of the free-dof tangent on FP64 MFMA, one
// workgroup of 256: the lower band is factored by panels of 16 columns with
// a window of WP = the next multiple of 16 of kl + 16 rows and columns in
// LDS, indexed modulo WP (the rows of a finished panel take the rows that
// enter the window).  Per panel: the 16 x 16 diagonal block factored by one
// wave, the rows below solved against it (a thread per row), the forward
// substitution of the right-hand side, the trailing window updated by the
// panel's outer product (16 x 16 x 4 FP64 MFMA tiles, the waves taking the
// tiles in turn), the panel stored for the backward substitution, and the
// entering rows loaded from the band.  Rows past nf are identity rows.  On
// success u_f += x, u_d += du_d and *done = 1; at a pivot that is not
// positive *done = 0 and nothing is written (the banded solve that follows
// then factors the same band).
constexpr int CB_KL_MAX = 112;  // WP <= 128: a 128 x 129 FP64 window, 129 KB of LDS

// value of lane l (uniform), through scalar registers
__device__ __forceinline__ double lane_d(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)v, l), hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__host__ __device__ inline int chol_blk_wp(int kl) { return (kl + 16 + 15) / 16 * 16; }
inline size_t chol_blk_lds_bytes(int kl) {
  const int wp = chol_blk_wp(kl);
  return (size_t)(wp * (wp + 1) + wp + 64) * 8;
}

__global__ __launch_bounds__(256) void k_band_chol_blk(int nf, int kl, int ldab, const double* __restrict__ band,
                                                        const double* __restrict__ rhs, double* __restrict__ lbuf,
                                                        double* __restrict__ y, int dofs, const int* __restrict__ dofmap,
                                                        const int* __restrict__ fixed, int nfixed,
                                                        const double* __restrict__ dud, double* __restrict__ u,
                                                        int* __restrict__ info, int* __restrict__ done) {
  extern __shared__ double lds[];
  const int WP = chol_blk_wp(kl), LDW = WP + 1, NBK = WP / 16;
  double* W = lds;              // [WP][LDW] lower triangle of the window, rows and columns by slot
  double* sb = lds + WP * LDW;  // [WP] right-hand side by slot
  double* sd = sb + WP;         // [16] reciprocal diagonal of the panel, [16] panel solution
  int* sflag = reinterpret_cast<int*>(sd + 32);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int np = (nf + 15) / 16;
  // A[g][c] of the (identity-extended) lower band, g >= c
  auto Aval = [&](int g, int c) -> double {
    if (g >= nf || c >= nf) return (g == c) ? 1.0 : 0.0;
    if (g - c > kl) return 0.0;
    return band[(size_t)g * ldab + (c - g + kl)];
  };
  // initial window: rows and columns 0 .. WP - 1
  for (int e = tid; e < WP * WP; e += 256) {
    const int r = e / WP, c = e - r * WP;
    W[r * LDW + c] = (r >= c) ? Aval(r, c) : 0.0;
  }
  for (int r = tid; r < WP; r += 256) sb[r] = (r < nf) ? rhs[r] : 0.0;
  if (tid == 0) *sflag = 0;
  __syncthreads();
  for (int pi = 0; pi < np; ++pi) {
    const int p = 16 * pi;
    const int s0 = p % WP;  // slot of row p (a multiple of 16: the panel's slots are s0 .. s0 + 15)
    auto slot = [&](int rel) { return (s0 + rel < WP) ? s0 + rel : s0 + rel - WP; };  // rel < WP
    // the rows that enter the window after this panel, loaded now (stored in step 6)
    double pre[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      pre[u] = 0.0;
      if (e < 16 * WP) {
        const int a = e / WP, c = e - a * WP, g = p + WP + a, gc = p + 16 + c;
        if (g >= gc) pre[u] = Aval(g, gc);
      }
    }
    const double preb = (tid < 16 && p + WP + tid < nf) ? rhs[p + WP + tid] : 0.0;
    // 1. the diagonal block, one wave: lane i holds row i
    if (wave == 0) {
      double row[16];
      const int si = slot(lane & 15);
#pragma unroll
      for (int j = 0; j < 16; ++j) row[j] = (lane < 16 && j <= lane) ? W[si * LDW + slot(j)] : 0.0;
      bool bad = false;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const double dkk = lane_d(row[k], k);
        if (!(dkk > 0.0) || !isfinite(dkk)) bad = true;
        const double lkk = sqrt(dkk);
        const double rl = 1.0 / lkk;
        if (lane == k) row[k] = lkk;
        if (lane > k && lane < 16) row[k] *= rl;
        const double lik = row[k];
#pragma unroll
        for (int j = k + 1; j < 16; ++j) {
          const double ljk = lane_d(row[k], j);
          if (lane >= j && lane < 16) row[j] = fma(-lik, ljk, row[j]);
        }
        if (lane == 0) sd[k] = rl;
      }
      if (lane < 16) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (j <= lane) W[si * LDW + slot(j)] = row[j];
      }
      if (lane == 0 && bad) *sflag = 1;
    }
    __syncthreads();
    if (*sflag) break;
    // 2. rows 16 .. WP - 1 against the diagonal block: l_r L_dd^T = s_r
    for (int r = 16 + tid; r < WP; r += 256) {
      const int sr = slot(r);
      double l[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        double v = W[sr * LDW + slot(k)];
        for (int j = 0; j < k; ++j) v = fma(-l[j], W[slot(k) * LDW + slot(j)], v);
        l[k] = v * sd[k];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) W[sr * LDW + slot(k)] = l[k];
    }
    // 3. forward substitution of the panel's right-hand side (wave 0)
    if (wave == 0) {
      double yi = (lane < 16) ? sb[slot(lane)] : 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const double yk = lane_d(yi, k) * sd[k];  // y_k = (b_k - sum_j<k l_kj y_j) / l_kk
        if (lane == k) yi = yk;
        if (lane > k && lane < 16) yi = fma(-W[slot(lane) * LDW + slot(k)], yk, yi);
      }
      if (lane < 16) {
        sd[16 + lane] = yi;
        if (p + lane < nf) y[p + lane] = yi;
      }
    }
    __syncthreads();
    // the rest of the right-hand side: b_r -= l_r . y_panel
    for (int r = 16 + tid; r < WP; r += 256) {
      const int sr = slot(r);
      double v = sb[sr];
#pragma unroll
      for (int k = 0; k < 16; ++k) v = fma(-W[sr * LDW + slot(k)], sd[16 + k], v);
      sb[sr] = v;
    }
    // 4. trailing update, tiles I >= J >= 1 of the window: W_IJ -= L_I L_J^T
    {
      const int i = lane & 15, kq = lane >> 4;
      int t = 0;
      for (int I = 1; I < NBK; ++I)
        for (int J = 1; J <= I; ++J, ++t) {
          if ((t & 3) != wave) continue;
          const int rI = slot(16 * I), rJ = slot(16 * J);
          d4 acc;
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) acc[jj] = W[(rI + kq + 4 * jj) * LDW + rJ + i];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int kc = slot(4 * kk + kq);
            const double a = -W[(rI + i) * LDW + kc];
            const double b = W[(rJ + i) * LDW + kc];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
          }
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) W[(rI + kq + 4 * jj) * LDW + rJ + i] = acc[jj];
        }
    }
    __syncthreads();
    // 5. the panel (rows 0 .. WP - 1 relative, its 16 columns) for the backward substitution
    double* L = lbuf + (size_t)pi * WP * 16;
    for (int e = tid; e < WP * 16; e += 256) {
      const int r = e >> 4, k = e & 15;
      L[e] = (r >= k) ? W[slot(r) * LDW + slot(k)] : 0.0;
    }
    __syncthreads();
    // 6. rows p + WP .. p + WP + 15 enter the window in the panel's slots
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      if (e < 16 * WP) {
        const int a = e / WP, c = e - a * WP;  // entering row a (slot of p + WP + a), window column c
        W[slot(a) * LDW + slot(16 + c)] = pre[u];
      }
    }
    if (tid < 16) sb[slot(tid)] = preb;
    __syncthreads();
  }
  if (*sflag) {
    if (tid == 0) *done = 0;
    return;
  }
  // backward substitution L^T x = y, panels in reverse; x over y in place
  for (int pi = np - 1; pi >= 0; --pi) {
    const int p = 16 * pi;
    const double* L = lbuf + (size_t)pi * WP * 16;
    // t_k = y_k - sum_r l_rk x_(p + r) over the rows below the panel (16 threads per k)
    {
      const int k = tid >> 4, q = tid & 15;
      double part = 0.0;
      for (int r = 16 + q; r < WP; r += 16) {
        const int g = p + r;
        if (g < nf) part = fma(L[r * 16 + k], y[g], part);
      }
      for (int o = 8; o > 0; o >>= 1) part += __shfl_xor(part, o);
      if (q == 0) sd[16 + k] = ((p + k < nf) ? y[p + k] : 0.0) - part;
    }
    __syncthreads();
    if (wave == 0) {
      double ti = (lane < 16) ? sd[16 + lane] : 0.0;
      const double ri = (lane < 16) ? 1.0 / L[lane * 16 + lane] : 0.0;
      for (int k = 15; k >= 0; --k) {
        const double xk = lane_d(ti, k) * lane_d(ri, k);
        if (lane == k) ti = xk;
        if (lane < k) ti = fma(-L[k * 16 + lane], xk, ti);
      }
      if (lane < 16 && p + lane < nf) y[p + lane] = ti;
    }
    __syncthreads();
  }
  for (int d = tid; d < dofs; d += 256) {
    const int r = dofmap[d];
    if (r >= 0) u[d] += y[r];
  }
  if (dud)
    for (int j = tid; j < nfixed; j += 256) u[fixed[j]] += dud[j];
  if (tid == 0) {
    *info = 0;
    *done = 1;
  }
}

inline unsigned nblk(long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

void release(rom_fe2* h) {
  if (!h) return;
  void* bufs[] = {h->X, h->dNdX, h->wJ, h->Xg, h->band, h->rhs, h->ubuf, h->xbuf, h->lbuf, h->ybuf, h->done,
                  h->conn, h->node_ptr, h->node_ent, h->dofmap, h->fixed, h->top};
  for (void* b : bufs) (void)hipFree(b);
  delete h;
}

}  // namespace

extern "C" {

int rom_fe2_create(int32_t nodes, int32_t elements, const double* X_host, const int32_t* conn_host, int32_t nfixed,
                   const int32_t* fixed_host, int32_t ntop, const int32_t* top_host, double width, int device,
                   rom_fe2_handle* out) {
  if (!out || nodes < 1 || elements < 1 || !X_host || !conn_host || nfixed < 0 || (nfixed > 0 && !fixed_host) ||
      ntop < 0 || (ntop > 0 && !top_host) || !(width > 0) || elements > (1 << 24))
    return ROM_EINVAL;
  *out = nullptr;
  const int dofs = 2 * nodes;
  for (long k = 0; k < 8L * elements; ++k)
    if (conn_host[k] < 0 || conn_host[k] >= nodes) return ROM_EINVAL;
  for (long k = 0; k < 3L * ntop; ++k)
    if (top_host[k] < 0 || top_host[k] >= nodes) return ROM_EINVAL;
  // dof map: free index, or -1 - (index in the fixed list)
  std::vector<int> dofmap(dofs, 0);
  for (int j = 0; j < nfixed; ++j) {
    const int d = fixed_host[j];
    if (d < 0 || d >= dofs || dofmap[d] < 0) return ROM_EINVAL;
    dofmap[d] = -1 - j;
  }
  int nfree = 0;
  for (int d = 0; d < dofs; ++d)
    if (dofmap[d] >= 0) dofmap[d] = nfree++;
  if (nfree < 1) return ROM_EINVAL;
  // node -> (element, local node) entries, elements ascending; bandwidth
  std::vector<int> cnt(nodes + 1, 0), ent;
  for (long k = 0; k < 8L * elements; ++k) ++cnt[conn_host[k] + 1];
  for (int n = 0; n < nodes; ++n) cnt[n + 1] += cnt[n];
  ent.resize(cnt[nodes]);
  std::vector<int> fill(cnt.begin(), cnt.end() - 1);
  int kl = 0;
  for (int e = 0; e < elements; ++e) {
    int lo = nfree, hi = -1;
    for (int a = 0; a < 8; ++a) {
      const int n = conn_host[8 * e + a];
      ent[fill[n]++] = 8 * e + a;
      for (int i = 0; i < 2; ++i) {
        const int r = dofmap[2 * n + i];
        if (r >= 0) {
          lo = std::min(lo, r);
          hi = std::max(hi, r);
        }
      }
    }
    if (hi >= lo) kl = std::max(kl, hi - lo);
  }
  if (kl > 255) return ROM_EUNSUPPORTED;  // multipliers of a column held in LDS
  DeviceGuard guard(device);
  rom_fe2* h = new rom_fe2();
  memset(h, 0, sizeof(*h));
  h->device = device;
  h->nodes = nodes;
  h->elements = elements;
  h->points = 4 * elements;
  h->dofs = dofs;
  h->nfixed = nfixed;
  h->nfree = nfree;
  h->ntop = ntop;
  h->kl = kl;
  h->ldab = 3 * kl + 1;
  h->width = width;
  bool ok = true;
  auto al = [&](void** p, size_t bytes) {
    if (ok && hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) ok = false;
  };
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (ok && bytes && hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) ok = false;
  };
  al((void**)&h->X, 8L * dofs);
  al((void**)&h->dNdX, 8L * 16 * h->points);
  al((void**)&h->wJ, 8L * h->points);
  al((void**)&h->Xg, 16L * h->points);
  al((void**)&h->band, 8L * nfree * h->ldab);
  al((void**)&h->rhs, 8L * nfree);
  h->stage = kl <= LDS_KL_MAX ? band_stage_rows(kl) : 0;
  if (h->stage > 0) {
    al((void**)&h->ubuf, 8L * nfree * (2 * kl + 1));
    al((void**)&h->xbuf, 8L * nfree);
    if (ok && hipFuncSetAttribute((const void*)k_band_solve_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)solve_lds_bytes(kl, h->stage)) != hipSuccess)
      ok = false;
  }
  if (kl <= CB_KL_MAX) {
    const int wp = chol_blk_wp(kl), np = (nfree + 15) / 16;
    al((void**)&h->lbuf, 8L * np * wp * 16);
    al((void**)&h->ybuf, 8L * nfree);
    al((void**)&h->done, 4);
    if (ok && hipFuncSetAttribute((const void*)k_band_chol_blk, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)chol_blk_lds_bytes(kl)) != hipSuccess)
      ok = false;
  }
  al((void**)&h->conn, 32L * elements);
  al((void**)&h->node_ptr, 4L * (nodes + 1));
  al((void**)&h->node_ent, 4L * ent.size());
  al((void**)&h->dofmap, 4L * dofs);
  al((void**)&h->fixed, 4L * nfixed);
  al((void**)&h->top, 12L * ntop);
  up(h->X, X_host, 8L * dofs);
  up(h->conn, conn_host, 32L * elements);
  up(h->node_ptr, cnt.data(), 4L * (nodes + 1));
  up(h->node_ent, ent.data(), 4L * ent.size());
  up(h->dofmap, dofmap.data(), 4L * dofs);
  up(h->fixed, fixed_host, 4L * nfixed);
  up(h->top, top_host, 12L * ntop);
  if (ok) {
    k_geometry<<<nblk(h->points), 256>>>(h->points, h->X, h->conn, h->dNdX, h->wJ, h->Xg);
    ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  }
  if (!ok) {
    release(h);
    return ROM_EHIP;
  }
  *out = h;
  return ROM_OK;
}

int rom_fe2_free(rom_fe2_handle h) {
  if (!h) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  release(h);
  return ROM_OK;
}

int rom_fe2_info(rom_fe2_handle h, int32_t* dofs, int32_t* free_dofs, int32_t* points, int32_t* kl) {
  if (!h) return ROM_EINVAL;
  if (dofs) *dofs = h->dofs;
  if (free_dofs) *free_dofs = h->nfree;
  if (points) *points = h->points;
  if (kl) *kl = h->kl;
  return ROM_OK;
}

int rom_fe2_points(rom_fe2_handle h, double* Xg_dev, hipStream_t s) {
  if (!h || !Xg_dev) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  return hipMemcpyAsync(Xg_dev, h->Xg, 16L * h->points, hipMemcpyDeviceToDevice, s) == hipSuccess ? ROM_OK
                                                                                                   : ROM_EHIP;
}

int rom_fe2_gradient(rom_fe2_handle h, const double* u_dev, double* Fbar_dev, hipStream_t s) {
  if (!h || !u_dev || !Fbar_dev) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  k_gradient<<<nblk(h->points), 256, 0, s>>>(h->points, h->conn, h->dNdX, u_dev, Fbar_dev);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_fe2_traction(rom_fe2_handle h, double Tbar, double* fext_dev, hipStream_t s) {
  if (!h || !fext_dev || !std::isfinite(Tbar)) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  k_traction<<<1, 256, 0, s>>>(h->dofs, h->ntop, h->top, h->X, Tbar, h->width, fext_dev);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_fe2_residual(rom_fe2_handle h, const double* Pbar_dev, const double* fext_dev, double* res_dev,
                     double* norms_dev, hipStream_t s) {
  if (!h || !Pbar_dev || !fext_dev || !res_dev) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  k_residual<<<nblk(h->dofs), 256, 0, s>>>(h->dofs, h->node_ptr, h->node_ent, h->dNdX, h->wJ, Pbar_dev, fext_dev,
                                           res_dev);
  if (norms_dev) k_norms<<<1, 256, 0, s>>>(h->dofs, h->dofmap, res_dev, fext_dev, norms_dev);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_fe2_solve(rom_fe2_handle h, const double* Abar_dev, const double* res_dev, const double* dud_dev,
                  double* u_dev, int32_t* info_dev, hipStream_t s) {
  if (!h || !Abar_dev || !res_dev || !u_dev || !info_dev) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  k_assemble<<<nblk(h->dofs), 256, 0, s>>>(h->dofs, h->kl, h->ldab, h->node_ptr, h->node_ent, h->conn, h->dofmap,
                                           h->dNdX, h->wJ, Abar_dev, res_dev, dud_dev, h->band, h->rhs);
  // the blocked Cholesky first; where a pivot is not positive (or the band
  // is too wide for it) the banded solve below factors the same band
  if (h->lbuf)
    k_band_chol_blk<<<1, 256, chol_blk_lds_bytes(h->kl), s>>>(h->nfree, h->kl, h->ldab, h->band, h->rhs, h->lbuf,
                                                             h->ybuf, h->dofs, h->dofmap, h->fixed, h->nfixed,
                                                             dud_dev, u_dev, info_dev, h->done);
  if (h->stage > 0)
    k_band_solve_lds<<<1, (4 * (2 * h->kl + 2) + 63) / 64 * 64, solve_lds_bytes(h->kl, h->stage), s>>>(
        h->nfree, h->kl, h->ldab, h->stage, h->band, h->rhs, h->ubuf, h->xbuf, h->dofs, h->dofmap, h->fixed,
        h->nfixed, dud_dev, u_dev, info_dev, h->done);
  else
    k_band_solve<<<1, LU_THREADS, 0, s>>>(h->nfree, h->kl, h->ldab, h->band, h->rhs, h->dofs, h->dofmap, h->fixed,
                                          h->nfixed, dud_dev, u_dev, info_dev, h->done);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_fe2_compliance(rom_fe2_handle h, double Tbar, const double* u_dev, double* C_dev, hipStream_t s) {
  if (!h || !u_dev || !C_dev || !std::isfinite(Tbar)) return ROM_EINVAL;
  DeviceGuard guard(h->device);
  k_compliance<<<1, 64, 0, s>>>(h->ntop, h->top, h->X, Tbar, h->width, u_dev, C_dev);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

}  // extern "C"
