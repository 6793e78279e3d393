// Fused form of the online solve: one kernel launch per load step, one
// workgroup per macro point running the whole Newton loop of eq. red_newton
// on the device.
//
// Per Newton evaluation the workgroup walks the ECM points in chunks of 256
// (one lane per point): kinematics, return map and tangent (Appendix A),
// then the weighted stress W = w|J| P F_mu^-T, the mapped tangent
// D = w|J| T^T A T and E = w|J| T^T A (T: right multiplication by F_mu^-1) go
// to LDS.  Each wave contracts 64 of the chunk's points on FP64 MFMA
// (v_mfma_f64_16x16x4: the 4-long inner dimension is the 4 gradient
// components of one ECM point):
//     K_ext[i][j] = sum_q sum_a G_q[a][i] B_q[a][j],
//     B_q[:, j] = D_q G_q[:, j] (j < n),  W_q (j = n),  E_q[:, j-n-1] (n < j <= n+4)
// so the residual f = sum_q G_q^T W_q (eq. forcevector_ecm) and
// C = sum_q G_q^T E_q (right-hand sides of eq. tangent_problem_red) come out
// of the padding columns of the stiffness tiles (eq. stiffnessmatrix_ecm).
// K is symmetric (the tangent of the appendix model is major-symmetric), so
// only tiles I <= J are contracted and the rest is mirrored.  Gaussian
// elimination with partial pivoting on [K | f | C] in LDS gives the Newton
// update and K*^-1 C for the effective stiffness (eq. eff_stiffness_1).
#include "rom_fused.h"

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int FCH = 256;  // ECM points per chunk
constexpr int QS = 20;    // LDS record per point in the Newton loop: D (16), W (4)

struct FusedArgs {
  int n, m, max_iter, fixed, commit;
  double tol, inv_area;
  J2Params mp;
  const double* Gt;
  const double* Gq;
  const double* Fbar;
  double* rc;
  double* rt;
  double* hc;
  double* ht;
  const double* tmu;
  const int* muok;
  double* Pbar;
  double* Abar;
  int* st_out;
  int* it_out;
  double* res_out;
};

// ECM points per chunk of the effective-quantity pass (E records sit above the LU)
template <int T>
constexpr int ech() {
  return T >= 8 ? 128 : FCH;
}
// LDS: chunk records / [K | f] with its LU and the E records, then r, C, C copy, scratch, pivots
template <int T>
constexpr int main_doubles() {
  return (FCH * QS > 256 * T * T + 16 * ech<T>()) ? FCH * QS : 256 * T * T + 16 * ech<T>();
}
template <int T>
constexpr int lds_doubles() {
  return main_doubles<T>() + 16 * T * 9 + 128 + 16 * T;
}

// F = Fbar + (sum_i r_i G_i(q)) F_mu^-1 at ECM point q (argument of P in
// eq. forcevector_ecm); r is read from LDS.
__device__ __forceinline__ void kinematics(int n, int m, int q, const double* __restrict__ Gt, const double* sR,
                                           const double Fb[4], const double Fi[4], double F[4]) {
  double H0 = 0.0, H1 = 0.0, H2 = 0.0, H3 = 0.0;
  const double* g = Gt + q;
  for (int i = 0; i < n; ++i) {
    const double ri = sR[i];
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

// E[(i r)][y] = w|J| sum_j Fi[r][j] A[(i j)][y]   (E = w|J| T^T A)
__device__ __forceinline__ void mapped_left(const double A[16], const double Fi[4], double wJ, double E[16]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int y = 0; y < 4; ++y)
        E[4 * (2 * i + r) + y] = wJ * (Fi[2 * r] * A[4 * (2 * i) + y] + Fi[2 * r + 1] * A[4 * (2 * i + 1) + y]);
}

template <int T>
__global__ __launch_bounds__(256) void k_fused(const FusedArgs a) {
  constexpr int NPAD = 16 * T;
  constexpr int NT = T * (T + 1) / 2;
  constexpr int MAT = main_doubles<T>();
  constexpr int ECH = ech<T>();
  extern __shared__ double smem[];
  double* sQ = smem;              // [FCH][QS] chunk records
  double* sK = smem;              // [NPAD][NPAD] [K | f] and its LU (after the contraction)
  double* sE = smem + NPAD * NPAD;  // [ECH][16] E records of the effective-quantity pass
  double* sR = smem + MAT;        // [NPAD] current r
  double* sC = sR + NPAD;         // [NPAD][4] C = sum_q G_q^T E_q, then K^-1 C
  double* sC0 = sC + 4 * NPAD;    // [NPAD][4] copy of C
  double* sX = sC0 + 4 * NPAD;    // reduction scratch (128)
  int* sPiv = reinterpret_cast<int*>(sX + 128);  // [NPAD] pivot rows of the LU

  const int p = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = a.n, m = a.m;
  if (!a.muok[p]) {
    if (tid < 4) a.Pbar[4 * (size_t)p + tid] = __builtin_nan("");
    if (tid < 16) a.Abar[16 * (size_t)p + tid] = __builtin_nan("");
    if (tid == 0) {
      a.st_out[p] = ROM_ST_BADMU;
      a.it_out[p] = 0;
      a.res_out[p] = __builtin_nan("");
    }
    return;
  }
  for (int i = tid; i < NPAD; i += 256) sR[i] = (i < n) ? a.rc[(size_t)p * n + i] : 0.0;
  const double Fb[4] = {a.Fbar[4 * (size_t)p], a.Fbar[4 * (size_t)p + 1], a.Fbar[4 * (size_t)p + 2],
                        a.Fbar[4 * (size_t)p + 3]};
  const double* tmu = a.tmu + (size_t)p * 5 * m;
  const double* hc = a.hc + (size_t)p * 6 * m;
  double* ht = a.ht + (size_t)p * 6 * m;
  __syncthreads();

  const int k_row = lane >> 4, c_col = lane & 15;
  int status = ROM_ST_MAXITER, iters = 0;
  double rn = 0.0;
  for (int it = 0; it < a.max_iter; ++it) {
    d4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = (d4){0.0, 0.0, 0.0, 0.0};

    for (int q0 = 0; q0 < m; q0 += FCH) {
      const int q = q0 + tid;
      if (q < m) {
        const double Fi[4] = {tmu[q], tmu[m + q], tmu[2 * m + q], tmu[3 * m + q]};
        const double wJ = tmu[4 * m + q];
        double F[4];
        kinematics(n, m, q, a.Gt, sR, Fb, Fi, F);
        const double Fp[4] = {hc[q], hc[m + q], hc[2 * m + q], hc[3 * m + q]};
        double P[4], Fpn[4], Fp33n, xin;
        double D[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) D[k] = 0.0;
        // D = w|J| T^T A T accumulated column by column of A
        j2_point_cols<true>(F, Fp, hc[4 * m + q], hc[5 * m + q], a.mp, P, Fpn, Fp33n, xin,
                            [&](int v, double c0, double c1, double c2, double c3) {
                              const double e0 = wJ * (Fi[0] * c0 + Fi[1] * c1);
                              const double e1 = wJ * (Fi[2] * c0 + Fi[3] * c1);
                              const double e2 = wJ * (Fi[0] * c2 + Fi[1] * c3);
                              const double e3 = wJ * (Fi[2] * c2 + Fi[3] * c3);
                              const int k = v >> 1, l = v & 1;
#pragma unroll
                              for (int s2 = 0; s2 < 2; ++s2) {
                                const double t = Fi[2 * s2 + l];
                                D[0 + 2 * k + s2] = fma(e0, t, D[0 + 2 * k + s2]);
                                D[4 + 2 * k + s2] = fma(e1, t, D[4 + 2 * k + s2]);
                                D[8 + 2 * k + s2] = fma(e2, t, D[8 + 2 * k + s2]);
                                D[12 + 2 * k + s2] = fma(e3, t, D[12 + 2 * k + s2]);
                              }
                            });
        ht[q] = Fpn[0];
        ht[m + q] = Fpn[1];
        ht[2 * m + q] = Fpn[2];
        ht[3 * m + q] = Fpn[3];
        ht[4 * m + q] = Fp33n;
        ht[5 * m + q] = xin;
        double* rec = sQ + tid * QS;
#pragma unroll
        for (int k = 0; k < 16; ++k) rec[k] = D[k];
        // W = w|J| P F_mu^-T
        rec[16] = wJ * (P[0] * Fi[0] + P[1] * Fi[1]);
        rec[17] = wJ * (P[0] * Fi[2] + P[1] * Fi[3]);
        rec[18] = wJ * (P[2] * Fi[0] + P[3] * Fi[1]);
        rec[19] = wJ * (P[2] * Fi[2] + P[3] * Fi[3]);
      }
      __syncthreads();
      // contraction of this wave's share of the chunk on FP64 MFMA
      const int qend = min(FCH, m - q0);
      const int qa = wave * 64, qb = min(qa + 64, qend);
      for (int ql = qa; ql < qb; ++ql) {
        const double* Gp = a.Gq + (size_t)(q0 + ql) * 4 * NPAD;
        const double* rq = sQ + ql * QS;
        const double d0 = rq[4 * k_row], d1 = rq[4 * k_row + 1], d2 = rq[4 * k_row + 2], d3 = rq[4 * k_row + 3];
        const double wk = rq[16 + k_row];
        double Aop[T], Bop[T];
#pragma unroll
        for (int J = 0; J < T; ++J) {
          const int col = 16 * J + c_col;
          const double g0 = Gp[col], g1 = Gp[NPAD + col], g2 = Gp[2 * NPAD + col], g3 = Gp[3 * NPAD + col];
          Aop[J] = (k_row == 0) ? g0 : (k_row == 1) ? g1 : (k_row == 2) ? g2 : g3;
          Bop[J] = (col < n) ? (d0 * g0 + d1 * g1 + d2 * g2 + d3 * g3) : ((col == n) ? wk : 0.0);
        }
        int t = 0;
#pragma unroll
        for (int J = 0; J < T; ++J)
#pragma unroll
          for (int I = 0; I <= J; ++I) {
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Aop[I], Bop[J], acc[t], 0, 0, 0);
            ++t;
          }
      }
      __syncthreads();
    }
    // reduce the four waves' tiles into [K | f] (ld NPAD), mirror K's lower part
    for (int w = 0; w < 4; ++w) {
      if (wave == w) {
        int t = 0;
#pragma unroll
        for (int J = 0; J < T; ++J)
#pragma unroll
          for (int I = 0; I <= J; ++I) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int row = 16 * I + k_row + 4 * j, col = 16 * J + c_col;
              double v = acc[t][j];
              if (w > 0) v += sK[row * NPAD + col];
              sK[row * NPAD + col] = v;
              if (I < J && w == 3) sK[col * NPAD + row] = v;
            }
            ++t;
          }
      }
      __syncthreads();
    }
    double part = 0.0;
    if (tid < n) {
      const double fv = sK[tid * NPAD + n];
      part = fv * fv;
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) sX[wave] = part;
    __syncthreads();
    rn = sqrt(sX[0] + sX[1] + sX[2] + sX[3]);
    iters = it + 1;
    const bool last = (it == a.max_iter - 1);
    bool stop;
    if (!isfinite(rn)) {
      stop = true;
      status = ROM_ST_NONFINITE;
    } else if (a.fixed) {
      stop = last;
      status = (rn <= a.tol) ? ROM_ST_CONVERGED : ROM_ST_MAXITER;
    } else if (rn <= a.tol) {
      stop = true;
      status = ROM_ST_CONVERGED;
    } else {
      stop = last;
      status = ROM_ST_MAXITER;
    }
    // LU with partial pivoting of K, applied to the column f as it goes
    const int nc = n + 1;
    for (int k = 0; k < n; ++k) {
      if (wave == 0) {
        double best = -1.0;
        int bi = k;
        for (int i = k + lane; i < n; i += 64) {
          const double v = fabs(sK[i * NPAD + k]);
          if (v > best) {
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
        if (lane == 0) sPiv[k] = bi;
      }
      __syncthreads();
      const int pr = sPiv[k];
      if (pr != k)
        for (int j = tid; j < nc; j += 256) {
          const double t = sK[k * NPAD + j];
          sK[k * NPAD + j] = sK[pr * NPAD + j];
          sK[pr * NPAD + j] = t;
        }
      __syncthreads();
      const double inv = 1.0 / sK[k * NPAD + k];
      const int rows = n - k - 1, cols = nc - k - 1;
      for (int idx = tid; idx < rows * cols; idx += 256) {
        const int i = k + 1 + idx / cols, j = k + 1 + idx % cols;
        sK[i * NPAD + j] = fma(-sK[i * NPAD + k] * inv, sK[k * NPAD + j], sK[i * NPAD + j]);
      }
      __syncthreads();
      for (int i = k + 1 + tid; i < n; i += 256) sK[i * NPAD + k] *= inv;  // store the multiplier
      __syncthreads();
    }
    // back substitution of the f column: x = K^-1 f
    for (int k = n - 1; k >= 0; --k) {
      if (tid == 0) sK[k * NPAD + n] /= sK[k * NPAD + k];
      __syncthreads();
      for (int i = tid; i < k; i += 256) sK[i * NPAD + n] = fma(-sK[i * NPAD + k], sK[k * NPAD + n], sK[i * NPAD + n]);
      __syncthreads();
    }
    if (stop) break;
    if (tid < n) sR[tid] -= sK[tid * NPAD + n];  // K dr = -f
    __syncthreads();
  }

  // Effective quantities at the returned state (Sec. 3.3): one more pass over
  // the ECM points for Pbar = sum wJ P, sum wJ A and C = sum_q G_q^T E_q; the
  // LU of K* (= K of the last evaluation) then gives K*^-1 C.
  double accP[4] = {0.0, 0.0, 0.0, 0.0}, accA[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) accA[k] = 0.0;
  double cacc[2] = {0.0, 0.0};
  for (int q0 = 0; q0 < m; q0 += ECH) {
    const int q = q0 + tid;
    if (tid < ECH && q < m) {
      const double Fi[4] = {tmu[q], tmu[m + q], tmu[2 * m + q], tmu[3 * m + q]};
      const double wJ = tmu[4 * m + q];
      double F[4];
      kinematics(n, m, q, a.Gt, sR, Fb, Fi, F);
      const double Fp[4] = {hc[q], hc[m + q], hc[2 * m + q], hc[3 * m + q]};
      double P[4], Fpn[4], Fp33n, xin;
      double* e = sE + tid * 16;
      // sum w|J| A and the E = w|J| T^T A records, column by column of A
      j2_point_cols<true>(F, Fp, hc[4 * m + q], hc[5 * m + q], a.mp, P, Fpn, Fp33n, xin,
                          [&](int v, double c0, double c1, double c2, double c3) {
                            accA[v] = fma(wJ, c0, accA[v]);
                            accA[4 + v] = fma(wJ, c1, accA[4 + v]);
                            accA[8 + v] = fma(wJ, c2, accA[8 + v]);
                            accA[12 + v] = fma(wJ, c3, accA[12 + v]);
                            e[0 + v] = wJ * (Fi[0] * c0 + Fi[1] * c1);
                            e[4 + v] = wJ * (Fi[2] * c0 + Fi[3] * c1);
                            e[8 + v] = wJ * (Fi[0] * c2 + Fi[1] * c3);
                            e[12 + v] = wJ * (Fi[2] * c2 + Fi[3] * c3);
                          });
#pragma unroll
      for (int k = 0; k < 4; ++k) accP[k] = fma(wJ, P[k], accP[k]);
    }
    __syncthreads();
    const int nq = min(ECH, m - q0);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int o = tid + 256 * u;  // output (i, y) = (o / 4, o % 4)
      if (o < 4 * n) {
        const int i = o >> 2, y = o & 3;
        double s = cacc[u];
        for (int qq = 0; qq < nq; ++qq) {
          const double* g = a.Gq + (size_t)(q0 + qq) * 4 * NPAD + i;
          const double* e = sE + qq * 16 + y;
          s = fma(g[0], e[0], s);
          s = fma(g[NPAD], e[4], s);
          s = fma(g[2 * NPAD], e[8], s);
          s = fma(g[3 * NPAD], e[12], s);
        }
        cacc[u] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int o = tid + 256 * u;
    if (o < 4 * n) {
      sC[o] = cacc[u];
      sC0[o] = cacc[u];
    }
  }
#pragma unroll
  for (int k = 0; k < 20; ++k) {
    double v = (k < 4) ? accP[k] : accA[k - 4];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) sX[4 * k + wave] = v;
  }
  __syncthreads();
  // Y = K*^-1 C in place: row permutation, unit-lower and upper solves (4 RHS)
  if (tid < 4)
    for (int k = 0; k < n; ++k) {
      const int pr = sPiv[k];
      if (pr != k) {
        const double t = sC[4 * k + tid];
        sC[4 * k + tid] = sC[4 * pr + tid];
        sC[4 * pr + tid] = t;
      }
    }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    for (int idx = tid; idx < 4 * (n - k - 1); idx += 256) {
      const int i = k + 1 + (idx >> 2), y = idx & 3;
      sC[4 * i + y] = fma(-sK[i * NPAD + k], sC[4 * k + y], sC[4 * i + y]);
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    if (tid < 4) sC[4 * k + tid] /= sK[k * NPAD + k];
    __syncthreads();
    for (int idx = tid; idx < 4 * k; idx += 256) {
      const int i = idx >> 2, y = idx & 3;
      sC[4 * i + y] = fma(-sK[i * NPAD + k], sC[4 * k + y], sC[4 * i + y]);
    }
    __syncthreads();
  }
  if (tid < 20) {
    const double v = ((sX[4 * tid] + sX[4 * tid + 1]) + sX[4 * tid + 2]) + sX[4 * tid + 3];
    if (tid < 4) {
      a.Pbar[4 * (size_t)p + tid] = v * a.inv_area;
    } else {
      const int e = tid - 4, x = e >> 2, y = e & 3;
      double acc2 = v;
      for (int i = 0; i < n; ++i) acc2 = fma(-sC0[4 * i + x], sC[4 * i + y], acc2);
      a.Abar[16 * (size_t)p + e] = acc2 * a.inv_area;
    }
  }
  for (int i = tid; i < n; i += 256) a.rt[(size_t)p * n + i] = sR[i];
  if (tid == 0) {
    a.st_out[p] = status;
    a.it_out[p] = iters;
    a.res_out[p] = rn;
  }
  if (a.commit && status == ROM_ST_CONVERGED) {
    for (int i = tid; i < n; i += 256) a.rc[(size_t)p * n + i] = sR[i];
    double* hcw = a.hc + (size_t)p * 6 * m;
    for (int q = tid; q < m; q += 256)
#pragma unroll
      for (int k = 0; k < 6; ++k) hcw[k * m + q] = ht[k * m + q];
  }
}

template <int T>
int launch_t(const FusedArgs& a, int P, hipStream_t s) {
  const size_t lds = (size_t)lds_doubles<T>() * 8;
  k_fused<T><<<P, 256, lds, s>>>(a);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

template <int T>
int setup_t() {
  const size_t lds = (size_t)lds_doubles<T>() * 8;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused<T>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess
             ? ROM_OK
             : ROM_EHIP;
}

}  // namespace

int rom_fused_tiles(int n) { return (n + 5 + 15) / 16; }

int rom_fused_setup() {
  int rc = ROM_OK;
  if (rc == ROM_OK) rc = setup_t<2>();
  if (rc == ROM_OK) rc = setup_t<3>();
  if (rc == ROM_OK) rc = setup_t<4>();
  if (rc == ROM_OK) rc = setup_t<5>();
  if (rc == ROM_OK) rc = setup_t<6>();
  if (rc == ROM_OK) rc = setup_t<7>();
  if (rc == ROM_OK) rc = setup_t<8>();
  return rc;
}

int rom_launch_step_fused(rom_model* h, int P, const double* Fbar, void* state, const rom_opts& o,
                          int32_t* st_out, int32_t* it_out, double* res_out, hipStream_t s) {
  if (o.contraction != ROM_DT_F64) return ROM_EUNSUPPORTED;
  const int T = rom_fused_tiles(h->n);
  if (T < 2 || T > 8 || 16 * T != h->npad) return ROM_EUNSUPPORTED;
  const StateLayout L = rom_state_layout(h, P);
  FusedArgs a;
  a.n = h->n;
  a.m = h->m;
  a.max_iter = o.max_iter;
  a.fixed = o.fixed_iters;
  a.commit = o.commit;
  a.tol = o.tol;
  a.inv_area = 1.0 / h->cell_area;
  a.mp = h->mp;
  a.Gt = h->Gt;
  a.Gq = h->Gq;
  a.Fbar = Fbar;
  a.rc = field<double>(state, L, F_RC);
  a.rt = field<double>(state, L, F_RT);
  a.hc = field<double>(state, L, F_HC);
  a.ht = field<double>(state, L, F_HT);
  a.tmu = field<double>(state, L, F_TMU);
  a.muok = field<int>(state, L, F_MUOK);
  a.Pbar = field<double>(state, L, F_PBAR);
  a.Abar = field<double>(state, L, F_ABAR);
  a.st_out = st_out;
  a.it_out = it_out;
  a.res_out = res_out;
  if (rom_timing_mark(h, 0, s) != ROM_OK) return ROM_EHIP;
  int rc;
  switch (T) {
    case 2: rc = launch_t<2>(a, P, s); break;
    case 3: rc = launch_t<3>(a, P, s); break;
    case 4: rc = launch_t<4>(a, P, s); break;
    case 5: rc = launch_t<5>(a, P, s); break;
    case 6: rc = launch_t<6>(a, P, s); break;
    case 7: rc = launch_t<7>(a, P, s); break;
    default: rc = launch_t<8>(a, P, s); break;
  }
  if (rom_timing_mark(h, 1, s) != ROM_OK) return ROM_EHIP;
  return rc;
}
