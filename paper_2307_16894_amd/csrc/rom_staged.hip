// Staged form of the online solve: one kernel per stage of Algorithm 1
// (online), Newton loop enqueued by the host without synchronisation.
//
//   k_state_init   Sec. 3.4: c(mu), F_mu, F_mu^-1, |det F_mu| w_q at the ECM
//                  points; r = 0; virgin history (Appendix A).
//   k_step_begin   trial r <- committed r (initial guess), flags.
//   k_eval         one lane per (point, ECM point): kinematics
//                  F = Fbar + (sum_i r_i G_i) F_mu^-1, return map and tangent,
//                  weighted stress W = w |J| P F_mu^-T and the mapped tangent
//                  D = w |J| T^T A T (T: right multiplication by F_mu^-1).
//   k_assemble     f = sum_q G_q^T W_q, K = sum_q G_q^T D_q G_q
//                  (eqs. forcevector_ecm, stiffnessmatrix_ecm).
//   k_solve        ||f||_2, convergence, LU with partial pivoting, Newton
//                  update (eq. red_newton).
//   k_effective    eq. eff_stress_1, tangent problems eq. tangent_problem_red
//                  with the LU of K*, eq. eff_stiffness_1.
//   k_finish       commit converged points, write per-point outputs.
#include "rom_staged.h"

namespace {

__device__ __forceinline__ void mu_to_c(int kind, const double* __restrict__ mu, double r0, double void_area,
                                        double* cc) {
  if (kind == 0) {
    cc[0] = mu[0] / r0 - 1.0;
    cc[1] = mu[1] / r0 - 1.0;
  } else if (kind == 2) {
    cc[0] = mu[0] - 1.0;  // every inclusion scaled by zeta about its centre
  } else {
    for (int v = 0; v < 4; ++v) {
      const double kappa = mu[2 * v], theta = mu[2 * v + 1];
      const double a = sqrt(void_area / (M_PI * kappa));
      const double b = kappa * a;
      double s, c;
      sincos(theta, &s, &c);
      cc[3 * v + 0] = (a * c * c + b * s * s) / r0 - 1.0;
      cc[3 * v + 1] = (a * s * s + b * c * c) / r0 - 1.0;
      cc[3 * v + 2] = (a - b) * s * c / r0;
    }
  }
}

__global__ void k_fill_i32(int* __restrict__ p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(128) void k_state_init(int n, int m, int c, int kind, int n_mu, double r0,
                                                     double void_area, const double* __restrict__ mu,
                                                     const double* __restrict__ w, const double* __restrict__ Gd,
                                                     double* __restrict__ rc, double* __restrict__ hc,
                                                     double* __restrict__ tmu, int* __restrict__ muok,
                                                     int* __restrict__ count, double* __restrict__ fbc,
                                                     double* __restrict__ mu_copy) {
  const int p = blockIdx.y;
  const int q = blockIdx.x * 128 + threadIdx.x;
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < n; i += 128) rc[(size_t)p * n + i] = 0.0;
    if (threadIdx.x < 4) fbc[4 * (size_t)p + threadIdx.x] = (threadIdx.x == 0 || threadIdx.x == 3) ? 1.0 : 0.0;
    if (threadIdx.x < n_mu) mu_copy[(size_t)p * n_mu + threadIdx.x] = mu[(size_t)p * n_mu + threadIdx.x];
  }
  if (q >= m) return;
  double cc[12];
  mu_to_c(kind, mu + (size_t)p * n_mu, r0, void_area, cc);
  double F0 = 1.0, F1 = 0.0, F2 = 0.0, F3 = 1.0;
  for (int k = 0; k < c; ++k) {
    const double* g = Gd + (size_t)k * 4 * m + q;
    F0 += cc[k] * g[0];
    F1 += cc[k] * g[m];
    F2 += cc[k] * g[2 * m];
    F3 += cc[k] * g[3 * m];
  }
  const double J = F0 * F3 - F1 * F2;
  double* t = tmu + (size_t)p * 5 * m + q;
  t[0] = F3 / J;
  t[m] = -F1 / J;
  t[2 * m] = -F2 / J;
  t[3 * m] = F0 / J;
  t[4 * m] = w[q] * fabs(J);
  double* h = hc + (size_t)p * 6 * m + q;
  h[0] = 1.0;
  h[m] = 0.0;
  h[2 * m] = 0.0;
  h[3 * m] = 1.0;
  h[4 * m] = 1.0;
  h[5 * m] = 0.0;
  if (!(J > 0.0)) {
    muok[p] = 0;
    atomicAdd(count, 1);
  }
}

__global__ void k_step_begin(int P, int n, const double* __restrict__ rc, double* __restrict__ rt,
                             const int* __restrict__ muok, int* __restrict__ done, int* __restrict__ status,
                             int* __restrict__ iters, double* __restrict__ res) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < P * n) rt[idx] = rc[idx];
  if (idx < P) {
    const int ok = muok[idx];
    done[idx] = ok ? 0 : 1;
    status[idx] = ok ? ROM_ST_MAXITER : ROM_ST_BADMU;
    iters[idx] = 0;
    res[idx] = ok ? 0.0 : __builtin_nan("");
  }
}

// Kinematics of the ECM point (eq. forcevector_ecm, argument of P).
__device__ __forceinline__ void point_kinematics(int n, int m, int q, const double* __restrict__ Gt,
                                                 const double* __restrict__ rp, const double* __restrict__ Fb,
                                                 const double Fi[4], double F[4]) {
  double H0 = 0.0, H1 = 0.0, H2 = 0.0, H3 = 0.0;
  const double* g = Gt + q;
  for (int i = 0; i < n; ++i) {
    const double ri = rp[i];
    H0 = fma(ri, g[0], H0);
    H1 = fma(ri, g[m], H1);
    H2 = fma(ri, g[2 * m], H2);
    H3 = fma(ri, g[3 * m], H3);
    g += 4 * (size_t)m;
  }
  F[0] = Fb[0] + H0 * Fi[0] + H1 * Fi[2];
  F[1] = Fb[1] + H0 * Fi[1] + H1 * Fi[3];
  F[2] = Fb[2] + H2 * Fi[0] + H3 * Fi[2];
  F[3] = Fb[3] + H2 * Fi[1] + H3 * Fi[3];
}

__global__ __launch_bounds__(64) void k_eval(int n, int m, J2Params mp, J2Params mp2, const int* __restrict__ phase,
                                             const double* __restrict__ Gt,
                                             const double* __restrict__ Fbar, const double* __restrict__ rt,
                                             const double* __restrict__ hc, double* __restrict__ ht,
                                             const double* __restrict__ tmu, const int* __restrict__ done,
                                             double* __restrict__ D, double* __restrict__ W) {
  const int p = blockIdx.y;
  if (done[p]) return;
  const int q = blockIdx.x * 64 + threadIdx.x;
  if (q >= m) return;
  const double* t = tmu + (size_t)p * 5 * m + q;
  const double Fi[4] = {t[0], t[m], t[2 * m], t[3 * m]};
  const double wJ = t[4 * m];
  double F[4];
  point_kinematics(n, m, q, Gt, rt + (size_t)p * n, Fbar + 4 * (size_t)p, Fi, F);
  const double* h = hc + (size_t)p * 6 * m + q;
  const double Fp[4] = {h[0], h[m], h[2 * m], h[3 * m]};
  double P[4], A[16], Fpn[4], Fp33n, xin;
  j2_point<true>(F, Fp, h[4 * m], h[5 * m], point_params(mp, mp2, phase, q), P, A, Fpn, Fp33n, xin);
  double* ho = ht + (size_t)p * 6 * m + q;
  ho[0] = Fpn[0];
  ho[m] = Fpn[1];
  ho[2 * m] = Fpn[2];
  ho[3 * m] = Fpn[3];
  ho[4 * m] = Fp33n;
  ho[5 * m] = xin;
  // W = w|J| P F_mu^-T : W_ir = sum_j P_ij Fi_rj
  double* Wo = W + (size_t)p * 4 * m + q;
  Wo[0] = wJ * (P[0] * Fi[0] + P[1] * Fi[1]);
  Wo[m] = wJ * (P[0] * Fi[2] + P[1] * Fi[3]);
  Wo[2 * m] = wJ * (P[2] * Fi[0] + P[3] * Fi[1]);
  Wo[3 * m] = wJ * (P[2] * Fi[2] + P[3] * Fi[3]);
  // AT[x][(k s)] = sum_l A[x][(k l)] Fi[s][l]
  double AT[16];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int s = 0; s < 2; ++s)
        AT[4 * x + 2 * k + s] = A[4 * x + 2 * k] * Fi[2 * s] + A[4 * x + 2 * k + 1] * Fi[2 * s + 1];
  // D[(i r)][y] = w|J| sum_j Fi[r][j] AT[(i j)][y]
  double* Do = D + (size_t)p * 16 * m + q;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int y = 0; y < 4; ++y)
        Do[(size_t)(4 * (2 * i + r) + y) * m] =
            wJ * (Fi[2 * r] * AT[4 * (2 * i) + y] + Fi[2 * r + 1] * AT[4 * (2 * i + 1) + y]);
}

// K = sum_q G_q^T D_q G_q and f = sum_q G_q^T W_q for one point per block.
// G chunks and H = D G are staged in LDS; each thread owns 4x4 tiles of K.
#define AS_QC 8
__global__ __launch_bounds__(256) void k_assemble(int n, int npad, int m, const double* __restrict__ Gq,
                                                  const double* __restrict__ D, const double* __restrict__ W,
                                                  const int* __restrict__ done, double* __restrict__ K,
                                                  double* __restrict__ f) {
  const int p = blockIdx.x;
  if (done[p]) return;
  __shared__ double sG[AS_QC * 4 * ROM_NMAX];
  __shared__ double sH[AS_QC * 4 * ROM_NMAX];
  __shared__ double sD[AS_QC * 16];
  __shared__ double sW[AS_QC * 4];
  const int tid = threadIdx.x;
  const int nt = npad / 4;
  const int ntiles = nt * nt;
  double acc[4][16];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 16; ++b) acc[a][b] = 0.0;
  double accf = 0.0;
  const int chunk = AS_QC * 4 * npad;
  for (int q0 = 0; q0 < m; q0 += AS_QC) {
    const int nq = min(AS_QC, m - q0);
    for (int idx = tid; idx < chunk; idx += 256) {
      const int qq = idx / (4 * npad);
      sG[idx] = (qq < nq) ? Gq[(size_t)q0 * 4 * npad + idx] : 0.0;
    }
    if (tid < AS_QC * 16) {
      const int qq = tid / 16, k = tid % 16;
      sD[tid] = (qq < nq) ? D[((size_t)p * 16 + k) * m + q0 + qq] : 0.0;
    }
    if (tid < AS_QC * 4) {
      const int qq = tid / 4, a = tid % 4;
      sW[tid] = (qq < nq) ? W[((size_t)p * 4 + a) * m + q0 + qq] : 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < chunk; idx += 256) {
      const int qq = idx / (4 * npad);
      const int a = (idx / npad) % 4;
      const int j = idx % npad;
      const double* g = sG + qq * 4 * npad + j;
      const double* d = sD + qq * 16 + a * 4;
      sH[idx] = d[0] * g[0] + d[1] * g[npad] + d[2] * g[2 * npad] + d[3] * g[3 * npad];
    }
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      const int t = tid + 256 * tt;
      if (t < ntiles) {
        const int i0 = 4 * (t / nt), j0 = 4 * (t % nt);
        for (int r = 0; r < AS_QC * 4; ++r) {
          const double* gi = sG + r * npad + i0;
          const double* hj = sH + r * npad + j0;
          const double g0 = gi[0], g1 = gi[1], g2 = gi[2], g3 = gi[3];
          const double h0 = hj[0], h1 = hj[1], h2 = hj[2], h3 = hj[3];
          acc[tt][0] = fma(g0, h0, acc[tt][0]);
          acc[tt][1] = fma(g0, h1, acc[tt][1]);
          acc[tt][2] = fma(g0, h2, acc[tt][2]);
          acc[tt][3] = fma(g0, h3, acc[tt][3]);
          acc[tt][4] = fma(g1, h0, acc[tt][4]);
          acc[tt][5] = fma(g1, h1, acc[tt][5]);
          acc[tt][6] = fma(g1, h2, acc[tt][6]);
          acc[tt][7] = fma(g1, h3, acc[tt][7]);
          acc[tt][8] = fma(g2, h0, acc[tt][8]);
          acc[tt][9] = fma(g2, h1, acc[tt][9]);
          acc[tt][10] = fma(g2, h2, acc[tt][10]);
          acc[tt][11] = fma(g2, h3, acc[tt][11]);
          acc[tt][12] = fma(g3, h0, acc[tt][12]);
          acc[tt][13] = fma(g3, h1, acc[tt][13]);
          acc[tt][14] = fma(g3, h2, acc[tt][14]);
          acc[tt][15] = fma(g3, h3, acc[tt][15]);
        }
      }
    }
    if (tid < npad) {
      for (int r = 0; r < AS_QC * 4; ++r) accf = fma(sG[r * npad + tid], sW[r], accf);
    }
    __syncthreads();
  }
  double* Kp = K + (size_t)p * n * n;
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) {
    const int t = tid + 256 * tt;
    if (t < ntiles) {
      const int i0 = 4 * (t / nt), j0 = 4 * (t % nt);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (i0 + a < n && j0 + b < n) Kp[(size_t)(i0 + a) * n + j0 + b] = acc[tt][4 * a + b];
    }
  }
  if (tid < n) f[(size_t)p * n + tid] = accf;
}

__device__ __forceinline__ double block_sum_256(double v, double* red) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// LU with partial pivoting of the n x n matrix in LDS (row-major), block of
// 256 threads; spiv receives the pivot row of each step.
__device__ void lu_factor_lds(int n, double* sA, int* spiv, double* red) {
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < n; i += 64) {
        const double v = fabs(sA[i * n + k]);
        if (v > best || (v == best && i < bi)) {
          best = v;
          bi = i;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) spiv[k] = bi;
    }
    __syncthreads();
    const int pr = spiv[k];
    if (pr != k) {
      for (int j = tid; j < n; j += blockDim.x) {
        const double t = sA[k * n + j];
        sA[k * n + j] = sA[pr * n + j];
        sA[pr * n + j] = t;
      }
    }
    __syncthreads();
    const double piv = sA[k * n + k];
    for (int i = k + 1 + tid; i < n; i += blockDim.x) sA[i * n + k] /= piv;
    __syncthreads();
    const int w = n - k - 1;
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      const int i = k + 1 + idx / w, j = k + 1 + idx % w;
      sA[i * n + j] = fma(-sA[i * n + k], sA[k * n + j], sA[i * n + j]);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_solve(int n, int it, int max_iter, int fixed, double tol,
                                               double* __restrict__ K, const double* __restrict__ f,
                                               int* __restrict__ piv, double* __restrict__ rt,
                                               int* __restrict__ done, int* __restrict__ status,
                                               int* __restrict__ iters, double* __restrict__ res) {
  const int p = blockIdx.x;
  if (done[p]) return;
  extern __shared__ double sm[];
  double* sA = sm;
  double* sb = sA + n * n;
  double* red = sb + n;
  int* spiv = reinterpret_cast<int*>(red + 8);
  const int tid = threadIdx.x;
  double* Kp = K + (size_t)p * n * n;
  for (int idx = tid; idx < n * n; idx += 256) sA[idx] = Kp[idx];
  double part = 0.0;
  for (int i = tid; i < n; i += 256) {
    const double v = f[(size_t)p * n + i];
    sb[i] = -v;
    part += v * v;
  }
  const double rn = sqrt(block_sum_256(part, red));
  const bool last = (it == max_iter - 1);
  bool stop;
  int st;
  if (!isfinite(rn)) {
    stop = true;
    st = ROM_ST_NONFINITE;
  } else if (fixed) {
    stop = last;
    st = (rn <= tol) ? ROM_ST_CONVERGED : ROM_ST_MAXITER;
  } else if (rn <= tol) {
    stop = true;
    st = ROM_ST_CONVERGED;
  } else {
    stop = last;
    st = ROM_ST_MAXITER;
  }
  lu_factor_lds(n, sA, spiv, red);
  for (int idx = tid; idx < n * n; idx += 256) Kp[idx] = sA[idx];
  for (int i = tid; i < n; i += 256) piv[(size_t)p * n + i] = spiv[i];
  if (tid == 0) {
    iters[p] = it + 1;
    res[p] = rn;
    status[p] = st;
    if (stop) done[p] = 1;
  }
  if (stop) return;
  // solve L U x = Pm b
  if (tid == 0)
    for (int k = 0; k < n; ++k) {
      const int pr = spiv[k];
      if (pr != k) {
        const double t = sb[k];
        sb[k] = sb[pr];
        sb[pr] = t;
      }
    }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double bk = sb[k];
    for (int i = k + 1 + tid; i < n; i += 256) sb[i] = fma(-sA[i * n + k], bk, sb[i]);
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    if (tid == 0) sb[k] /= sA[k * n + k];
    __syncthreads();
    const double bk = sb[k];
    for (int i = tid; i < k; i += 256) sb[i] = fma(-sA[i * n + k], bk, sb[i]);
    __syncthreads();
  }
  for (int i = tid; i < n; i += 256) rt[(size_t)p * n + i] += sb[i];
}

// Effective stress and stiffness at the returned state (Sec. 3.3).
__global__ __launch_bounds__(128) void k_effective(int n, int npad, int m, double inv_area, J2Params mp,
                                                   J2Params mp2, const int* __restrict__ phase,
                                                   const double* __restrict__ Gt, const double* __restrict__ Gq,
                                                   const double* __restrict__ Fbar, const double* __restrict__ rt,
                                                   const double* __restrict__ hc, const double* __restrict__ tmu,
                                                   const int* __restrict__ muok, const double* __restrict__ LU,
                                                   const int* __restrict__ piv, double* __restrict__ Pbar,
                                                   double* __restrict__ Abar, double* __restrict__ zk) {
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  if (!muok[p]) {
    if (tid < 4) Pbar[4 * (size_t)p + tid] = __builtin_nan("");
    if (tid < 16) Abar[16 * (size_t)p + tid] = __builtin_nan("");
    return;
  }
  __shared__ double sE[128 * 33];
  __shared__ double sC[ROM_NMAX * 8];
  double accP[4] = {0, 0, 0, 0}, accA[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) accA[k] = 0.0;
  double cacc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) cacc[k] = 0.0;
  const double* Fb = Fbar + 4 * (size_t)p;
  for (int q0 = 0; q0 < m; q0 += 128) {
    const int q = q0 + tid;
    double* e = sE + tid * 33;
    if (q < m) {
      const double* t = tmu + (size_t)p * 5 * m + q;
      const double Fi[4] = {t[0], t[m], t[2 * m], t[3 * m]};
      const double wJ = t[4 * m];
      double F[4];
      point_kinematics(n, m, q, Gt, rt + (size_t)p * n, Fb, Fi, F);
      const double* h = hc + (size_t)p * 6 * m + q;
      const double Fp[4] = {h[0], h[m], h[2 * m], h[3 * m]};
      double P[4], A[16], Fpn[4], Fp33n, xin;
      j2_point<true>(F, Fp, h[4 * m], h[5 * m], point_params(mp, mp2, phase, q), P, A, Fpn, Fp33n, xin);
#pragma unroll
      for (int k = 0; k < 4; ++k) accP[k] += wJ * P[k];
#pragma unroll
      for (int k = 0; k < 16; ++k) accA[k] += wJ * A[k];
      // E[(i r)][y] = w|J| sum_j Fi[r][j] A[(i j)][y]  -> C = sum_q G_q^T E_q
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int y = 0; y < 4; ++y)
            e[4 * (2 * i + r) + y] = wJ * (Fi[2 * r] * A[4 * (2 * i) + y] + Fi[2 * r + 1] * A[4 * (2 * i + 1) + y]);
      // Et[(k s)][x] = w|J| sum_l A[x][(k l)] Fi[s][l]  -> Ct = sum_q G_q^T Et_q
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int x = 0; x < 4; ++x)
            e[16 + 4 * (2 * k + s) + x] = wJ * (A[4 * x + 2 * k] * Fi[2 * s] + A[4 * x + 2 * k + 1] * Fi[2 * s + 1]);
    } else {
      for (int k = 0; k < 32; ++k) e[k] = 0.0;
    }
    __syncthreads();
    const int nq = min(128, m - q0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int o = tid + 128 * k;
      if (o < 8 * n) {
        const int which = o / (4 * n);
        const int oo = o % (4 * n);
        const int i = oo / 4, y = oo % 4;
        double s = cacc[k];
        for (int qq = 0; qq < nq; ++qq) {
          const double* g = Gq + (size_t)(q0 + qq) * 4 * npad + i;
          const double* ee = sE + qq * 33 + 16 * which + y;
          s = fma(g[0], ee[0], s);
          s = fma(g[npad], ee[4], s);
          s = fma(g[2 * npad], ee[8], s);
          s = fma(g[3 * npad], ee[12], s);
        }
        cacc[k] = s;
      }
    }
    __syncthreads();
  }
  // reduce accP, accA over the block
  double* red = sE;
  for (int k = 0; k < 20; ++k) {
    double v = (k < 4) ? accP[k] : accA[k - 4];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((tid & 63) == 0) red[k * 2 + (tid >> 6)] = v;
  }
  // C (n x 4) and Ct (n x 4) to LDS
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int o = tid + 128 * k;
    if (o < 8 * n) sC[o] = cacc[k];
  }
  __syncthreads();
  double* Y = sC;           // C, then K^-1 C in place
  const double* Ct = sC + 4 * n;
  const double* LUp = LU + (size_t)p * n * n;
  const int* pv = piv + (size_t)p * n;
  if (tid < 4)
    for (int k = 0; k < n; ++k) {
      const int pr = pv[k];
      if (pr != k) {
        const double t = Y[4 * k + tid];
        Y[4 * k + tid] = Y[4 * pr + tid];
        Y[4 * pr + tid] = t;
      }
    }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    for (int idx = tid; idx < 4 * (n - k - 1); idx += 128) {
      const int i = k + 1 + idx / 4, y = idx % 4;
      Y[4 * i + y] = fma(-LUp[(size_t)i * n + k], Y[4 * k + y], Y[4 * i + y]);
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    if (tid < 4) Y[4 * k + tid] /= LUp[(size_t)k * n + k];
    __syncthreads();
    for (int idx = tid; idx < 4 * k; idx += 128) {
      const int i = idx / 4, y = idx % 4;
      Y[4 * i + y] = fma(-LUp[(size_t)i * n + k], Y[4 * k + y], Y[4 * i + y]);
    }
    __syncthreads();
  }
  for (int idx = tid; idx < 4 * n; idx += 128) zk[(size_t)p * 4 * n + idx] = Y[idx];  // K*^-1 C
  if (tid < 16) {
    const int x = tid / 4, y = tid % 4;
    double s = red[(4 + tid) * 2] + red[(4 + tid) * 2 + 1];
    for (int i = 0; i < n; ++i) s -= Ct[4 * i + x] * Y[4 * i + y];
    Abar[16 * (size_t)p + tid] = s * inv_area;
  }
  if (tid < 4) Pbar[4 * (size_t)p + tid] = (red[tid * 2] + red[tid * 2 + 1]) * inv_area;
}

__global__ __launch_bounds__(256) void k_finish(int n, int m, int commit, const double* __restrict__ Fbar,
                                                double* __restrict__ fbc, const int* __restrict__ status,
                                                const int* __restrict__ iters, const double* __restrict__ res,
                                                const double* __restrict__ rt, double* __restrict__ rc,
                                                const double* __restrict__ ht, double* __restrict__ hc,
                                                int* __restrict__ st_out, int* __restrict__ it_out,
                                                double* __restrict__ res_out, unsigned int* __restrict__ sub) {
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int st = status[p];
  if (tid == 0) {
    st_out[p] = st;
    it_out[p] = iters[p];
    res_out[p] = res[p];
    sub[p] = (st == ROM_ST_CONVERGED) ? (1u << 31) : 0u;  // the plain step: no cutting in this form
  }
  if (!(commit && st == ROM_ST_CONVERGED)) return;
  if (tid < 4) fbc[4 * (size_t)p + tid] = Fbar[4 * (size_t)p + tid];
  for (int i = tid; i < n; i += 256) rc[(size_t)p * n + i] = rt[(size_t)p * n + i];
  for (int i = tid; i < 6 * m; i += 256) hc[(size_t)p * 6 * m + i] = ht[(size_t)p * 6 * m + i];
}

// Commit of a trial step's state at its converged points (status converged,
// or converged after the warm start fell back): r, history and Fbar, the
// copies the step itself makes with commit set.  One workgroup per point.
__global__ __launch_bounds__(256) void k_commit_trial(int n, int m, const double* __restrict__ Fbar,
                                                      const int* __restrict__ status, double* __restrict__ fbc,
                                                      const double* __restrict__ rt, double* __restrict__ rc,
                                                      const double* __restrict__ ht, double* __restrict__ hc) {
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int st = status[p];
  if (st != ROM_ST_CONVERGED && st != ROM_ST_FALLBACK) return;
  if (tid < 4) fbc[4 * (size_t)p + tid] = Fbar[4 * (size_t)p + tid];
  for (int i = tid; i < n; i += 256) rc[(size_t)p * n + i] = rt[(size_t)p * n + i];
  for (int i = tid; i < 6 * m; i += 256) hc[(size_t)p * 6 * m + i] = ht[(size_t)p * 6 * m + i];
}

// Inputs of the warm-start network for the step to Fbar: mu, Fbar - Fbar_committed,
// r_committed and eight statistics of the committed plastic state weighted by
// w_q |det F_mu|: mean / max / standard deviation of xi, yielded fraction,
// mean of F^pl - I.  One block per point.
// One wave per point (four points per workgroup): the lanes walk the ECM
// points with stride 64 and the nine sums are reduced across the wave.
__global__ __launch_bounds__(256) void k_features(int P, int n, int m, int n_mu, const double* __restrict__ mu,
                                                  const double* __restrict__ Fbar, const double* __restrict__ fbc,
                                                  const double* __restrict__ rc, const double* __restrict__ hc,
                                                  const double* __restrict__ tmu, float* __restrict__ X) {
  const int lane = threadIdx.x & 63, p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= P) return;
  const int nf = n_mu + 4 + n + 8;
  float* x = X + (size_t)p * nf;
  double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // sum w, w xi, w xi^2, w [xi>0], w (Fp - I) (4), max xi
  const double* h = hc + (size_t)p * 6 * m;
  const double* t = tmu + (size_t)p * 5 * m;
  for (int q = lane; q < m; q += 64) {
    const double w = t[4 * m + q], xi = h[5 * m + q];
    s[0] += w;
    s[1] += w * xi;
    s[2] += w * xi * xi;
    s[3] += (xi > 0.0) ? w : 0.0;
    s[4] += w * (h[q] - 1.0);
    s[5] += w * h[m + q];
    s[6] += w * h[2 * m + q];
    s[7] += w * (h[3 * m + q] - 1.0);
    s[8] = fmax(s[8], xi);
  }
#pragma unroll
  for (int k = 0; k < 9; ++k)
    for (int o = 32; o > 0; o >>= 1) {
      const double u = __shfl_xor(s[k], o);
      s[k] = (k == 8) ? fmax(s[k], u) : s[k] + u;
    }
  if (lane == 0) {
    const double W = s[0], mean = s[1] / W;
    float* st = x + n_mu + 4 + n;
    st[0] = (float)mean;
    st[1] = (float)s[8];
    st[2] = (float)sqrt(fmax(s[2] / W - mean * mean, 0.0));
    st[3] = (float)(s[3] / W);
    for (int k = 0; k < 4; ++k) st[4 + k] = (float)(s[4 + k] / W);
  }
  if (lane < n_mu) x[lane] = (float)mu[(size_t)p * n_mu + lane];
  if (lane < 4) x[n_mu + lane] = (float)(Fbar[4 * (size_t)p + lane] - fbc[4 * (size_t)p + lane]);
  for (int i = lane; i < n; i += 64) x[n_mu + 4 + i] = (float)rc[(size_t)p * n + i];
}

__global__ void k_path_gather(int P, const double* __restrict__ paths, int max_steps, const int* __restrict__ nsteps,
                              const int* __restrict__ step, double* __restrict__ Fbar, int* __restrict__ active) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int k = step[p];
  const int on = (k < nsteps[p] && k < max_steps) ? 1 : 0;
  active[p] = on;
  if (on)
    for (int c = 0; c < 4; ++c) Fbar[4 * (size_t)p + c] = paths[((size_t)p * max_steps + k) * 4 + c];
}

__global__ void k_path_advance(int P, const int* __restrict__ active, int* __restrict__ step) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P && active[p]) step[p] += 1;
}

}  // namespace

int rom_launch_path_gather(int P, const double* paths, int max_steps, const int* nsteps, const int* step, double* Fbar,
                           int* active, hipStream_t s) {
  k_path_gather<<<(P + 255) / 256, 256, 0, s>>>(P, paths, max_steps, nsteps, step, Fbar, active);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_launch_path_advance(int P, const int* active, int* step, hipStream_t s) {
  k_path_advance<<<(P + 255) / 256, 256, 0, s>>>(P, active, step);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_launch_features(const rom_model* h, int P, const double* Fbar, const void* state, float* X, hipStream_t s) {
  const StateLayout L = rom_state_layout(h, P);
  void* st = const_cast<void*>(state);
  k_features<<<(P + 3) / 4, 256, 0, s>>>(P, h->n, h->m, h->n_mu, field<double>(st, L, F_MU), Fbar, field<double>(st, L, F_FBC),
                               field<double>(st, L, F_RC), field<double>(st, L, F_HC), field<double>(st, L, F_TMU), X);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

namespace {

// Training samples of the warm-start network from a solved load step, in
// point order: for every converged point, its features X_feat[p] (taken
// before the step) and dr = r_committed - r_before in FP32, appended at
// *count (device counter, advanced).  One workgroup walks the batch in blocks
// of 1024 points, ranking the converged ones with a ballot per wave.
__global__ __launch_bounds__(1024) void k_warm_samples(int P, int n, int nf, const float* __restrict__ X_feat,
                                                        const double* __restrict__ rc,
                                                        const double* __restrict__ r_before,
                                                        const int* __restrict__ status, float* __restrict__ X_out,
                                                        float* __restrict__ Y_out, int* __restrict__ count) {
  __shared__ int wsum[16];
  __shared__ int base0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) base0 = *count;
  __syncthreads();
  int base = base0;
  for (int p0 = 0; p0 < P; p0 += 1024) {
    const int p = p0 + threadIdx.x;
    const bool ok = p < P && status[p] == ROM_ST_CONVERGED;
    const unsigned long long bal = __ballot(ok);
    if (lane == 0) wsum[wave] = __popcll(bal);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      off += (w < wave) ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (ok) {
      const long d = base + off + __popcll(bal & ((1ull << lane) - 1ull));
      for (int j = 0; j < nf; ++j) X_out[d * nf + j] = X_feat[(long)p * nf + j];
      for (int i = 0; i < n; ++i) Y_out[d * n + i] = (float)(rc[(long)p * n + i] - r_before[(long)p * n + i]);
    }
    base += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base;
}

}  // namespace

int rom_launch_warm_samples(const rom_model* h, int P, const void* state, const float* X_feat, const double* r_before,
                            const int* status, float* X_out, float* Y_out, int* count, hipStream_t s) {
  const StateLayout L = rom_state_layout(h, P);
  void* st = const_cast<void*>(state);
  k_warm_samples<<<1, 1024, 0, s>>>(P, h->n, rom_n_features(h), X_feat, field<double>(st, L, F_RC), r_before, status,
                                    X_out, Y_out, count);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_launch_commit_trial(const rom_model* h, int P, const double* Fbar, void* state, const int* status,
                            hipStream_t s) {
  const StateLayout L = rom_state_layout(h, P);
  k_commit_trial<<<P, 256, 0, s>>>(h->n, h->m, Fbar, status, field<double>(state, L, F_FBC),
                                   field<double>(state, L, F_RT), field<double>(state, L, F_RC),
                                   field<double>(state, L, F_HT), field<double>(state, L, F_HC));
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_staged_setup() {
  // k_solve keeps the n x n matrix in LDS: up to ~132 KB at n = 128.
  const size_t lds = (size_t)(ROM_NMAX * ROM_NMAX + ROM_NMAX + 8) * 8 + ROM_NMAX * 4;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return e == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_launch_state_init(const rom_model* h, int P, const double* mu, void* state, hipStream_t s) {
  const StateLayout L = rom_state_layout(h, P);
  int* muok = field<int>(state, L, F_MUOK);
  int* count = field<int>(state, L, F_COUNT);
  k_fill_i32<<<(P + 255) / 256, 256, 0, s>>>(muok, P, 1);
  k_fill_i32<<<1, 64, 0, s>>>(count, 16, 0);
  k_fill_i32<<<(P + 255) / 256, 256, 0, s>>>(field<int>(state, L, F_SUB), P, 0);  // no step made yet
  dim3 g((h->m + 127) / 128, P);
  k_state_init<<<g, 128, 0, s>>>(h->n, h->m, h->c, h->kind, h->n_mu, h->r0, h->void_area, mu, h->w, h->Gd,
                                 field<double>(state, L, F_RC), field<double>(state, L, F_HC),
                                 field<double>(state, L, F_TMU), muok, count, field<double>(state, L, F_FBC),
                                 field<double>(state, L, F_MU));
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

int rom_launch_step_staged(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o,
                           int32_t* st_out, int32_t* it_out, double* res_out, hipStream_t s) {
  const StateLayout L = rom_state_layout(h, P);
  const int n = h->n, m = h->m;
  double* rc = field<double>(state, L, F_RC);
  double* rt = field<double>(state, L, F_RT);
  double* hc = field<double>(state, L, F_HC);
  double* ht = field<double>(state, L, F_HT);
  double* tmu = field<double>(state, L, F_TMU);
  int* muok = field<int>(state, L, F_MUOK);
  int* done = field<int>(state, L, F_DONE);
  int* status = field<int>(state, L, F_STATUS);
  int* iters = field<int>(state, L, F_ITERS);
  double* res = field<double>(state, L, F_RES);
  double* D = field<double>(state, L, F_D);
  double* W = field<double>(state, L, F_W);
  double* K = field<double>(state, L, F_K);
  double* f = field<double>(state, L, F_F);
  int* piv = field<int>(state, L, F_PIV);
  const int tot = P * n > P ? P * n : P;
  k_step_begin<<<(tot + 255) / 256, 256, 0, s>>>(P, n, rc, rt, muok, done, status, iters, res);
  const size_t solve_lds = (size_t)(n * n + n + 8) * 8 + (size_t)n * 4;
  for (int it = 0; it < o.max_iter; ++it) {
    k_eval<<<dim3((m + 63) / 64, P), 64, 0, s>>>(n, m, h->mp, h->mp2, h->phase, h->Gt, Fbar, rt, hc, ht, tmu, done,
                                                 D, W);
    if (rom_timing_mark(h, 0, s) != ROM_OK) return ROM_EHIP;
    k_assemble<<<P, 256, 0, s>>>(n, h->npad, m, h->Gq, D, W, done, K, f);
    if (rom_timing_mark(h, 1, s) != ROM_OK) return ROM_EHIP;
    k_solve<<<P, 256, solve_lds, s>>>(n, it, o.max_iter, o.fixed_iters, o.tol, K, f, piv, rt, done, status,
                                      iters, res);
  }
  k_effective<<<P, 128, 0, s>>>(n, h->npad, m, 1.0 / h->cell_area, h->mp, h->mp2, h->phase, h->Gt, h->Gq, Fbar, rt, hc, tmu, muok,
                                K, piv, field<double>(state, L, F_PBAR), field<double>(state, L, F_ABAR),
                                field<double>(state, L, F_ZK));
  k_finish<<<P, 256, 0, s>>>(n, m, o.commit, Fbar, field<double>(state, L, F_FBC), status, iters, res, rt, rc, ht,
                             hc, st_out, it_out, res_out, field<unsigned int>(state, L, F_SUB));
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}
