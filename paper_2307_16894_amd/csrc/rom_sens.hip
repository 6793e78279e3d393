// Shape sensitivities of the effective stress (eq. eff_sensitivities_full,
// with the ECM rule) at the trial state of the last step, the committed
// history held fixed.  With F = Fbar + H F_mu^-1, H = sum_i r_i G_i(q):
//   at fixed r, per ECM point and shape parameter k,
//     dF_mu = sum_c (dc_c/dmu_k) grad dhat_c,  dF_mu^-1 = -F_mu^-1 dF_mu F_mu^-1,
//     d(w|J|) = w|J| tr(F_mu^-1 dF_mu),  X = H dF_mu^-1,
//     b = d(w|J|) P F_mu^-T + w|J| (A : X) F_mu^-T + w|J| P dF_mu^-T   (df/dmu_k = sum_q G_q^T b),
//     d = w|J| A : X + d(w|J|) P                                     (direct term);
//   the reduced equilibrium gives dr/dmu_k = -K^-1 df/dmu_k, and its share
//   of dPbar is sum_q w|J| A : (G dr F_mu^-1) = -(K^-1 C)^T df/dmu_k with C the
//   right-hand sides of the tangent problems (eq. tangent_problem_red; K and
//   A symmetric), whose K*^-1 C the step left in the state:
//     dPbar/dmu_k = (sum_q d - (K*^-1 C)^T df/dmu_k) / |cell|.
#include "rom_fused.h"
#include "rom_fused_impl.h"

namespace {

constexpr int SENS_MU = 8;  // most shape parameters of a parameter map
constexpr int SCH = 128;    // ECM points per chunk

// d c / d mu of the shape-to-coefficient maps, [c][n_mu] (row c_index, column
// shape parameter): kind 0 c = (a, b) / r0 - 1; kind 1 per void
// S = R(theta) diag(a, b) R(theta)^T / r0 with a = sqrt(A_v / (pi kappa)),
// b = kappa a (da/dkappa = -a / (2 kappa), db/dkappa = a / 2); kind 2
// c = zeta - 1.
__device__ void mu_to_dc(int kind, const double* mu, double r0, double void_area, int n_mu, double* dc) {
  for (int i = 0; i < 12 * n_mu; ++i) dc[i] = 0.0;
  if (kind == 0) {
    dc[0 * n_mu + 0] = 1.0 / r0;
    dc[1 * n_mu + 1] = 1.0 / r0;
    return;
  }
  if (kind == 2) {
    dc[0] = 1.0;
    return;
  }
  for (int v = 0; v < 4; ++v) {
    const double kappa = mu[2 * v], theta = mu[2 * v + 1];
    const double a = sqrt(void_area / (M_PI * kappa)), b = kappa * a;
    const double da = -a / (2.0 * kappa), db = 0.5 * a;
    double sn, cs;
    sincos(theta, &sn, &cs);
    dc[(3 * v + 0) * n_mu + 2 * v] = (da * cs * cs + db * sn * sn) / r0;
    dc[(3 * v + 1) * n_mu + 2 * v] = (da * sn * sn + db * cs * cs) / r0;
    dc[(3 * v + 2) * n_mu + 2 * v] = (da - db) * sn * cs / r0;
    dc[(3 * v + 0) * n_mu + 2 * v + 1] = 2.0 * sn * cs * (b - a) / r0;
    dc[(3 * v + 1) * n_mu + 2 * v + 1] = 2.0 * sn * cs * (a - b) / r0;
    dc[(3 * v + 2) * n_mu + 2 * v + 1] = (a - b) * (cs * cs - sn * sn) / r0;
  }
}

// One workgroup per point.  Lanes take the ECM points of a chunk (material
// and the per-parameter b, d); then df/dmu = sum_q G_q^T b over the chunk on
// MFMA, the waves splitting its points.
__global__ __launch_bounds__(256) void k_sens(int n, int npad, int m, int c, int kind, int n_mu, double r0,
                                              double void_area, double inv_area, J2Params mp, J2Params mp2,
                                              const int* __restrict__ phase,
                                              const double* __restrict__ Gt, const double* __restrict__ Gq,
                                              const double* __restrict__ Gd, const double* __restrict__ Fbar,
                                              const double* __restrict__ rt, const double* __restrict__ hc,
                                              const double* __restrict__ tmu, const double* __restrict__ mu,
                                              const int* __restrict__ muok, const double* __restrict__ zk,
                                              double* __restrict__ out) {
  const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* o = out + (size_t)p * 4 * n_mu;
  if (!muok[p]) {
    if (tid < 4 * n_mu) o[tid] = __builtin_nan("");
    return;
  }
  __shared__ double sB[SCH * SENS_MU * 4];   // b of the chunk's points
  __shared__ double sR[ROM_NMAX];            // trial r
  __shared__ double sDc[12 * SENS_MU];       // d c / d mu
  __shared__ double sDw[SENS_MU * 4 * 4];    // wave partials of the direct term
  __shared__ double sBf[ROM_NMAX * SENS_MU]; // df / dmu
  for (int i = tid; i < n; i += 256) sR[i] = rt[(size_t)p * n + i];
  if (tid == 0) mu_to_dc(kind, mu + (size_t)p * n_mu, r0, void_area, n_mu, sDc);
  __syncthreads();
  const double Fb[4] = {Fbar[4 * (size_t)p], Fbar[4 * (size_t)p + 1], Fbar[4 * (size_t)p + 2],
                        Fbar[4 * (size_t)p + 3]};
  const double* tq = tmu + (size_t)p * 5 * m;
  const double* hq = hc + (size_t)p * 6 * m;
  double d[SENS_MU][4];
#pragma unroll
  for (int k = 0; k < SENS_MU; ++k)
#pragma unroll
    for (int r = 0; r < 4; ++r) d[k][r] = 0.0;
  // df/dmu = sum_q G_q^T b_q on MFMA: A = G_q^T (row tile I: lane (k, i) holds
  // component k of mode 16 I + i), B = b_q (lane (k, j) holds b_q[k] of
  // parameter j), the four components as the inner dimension; each wave takes
  // a quarter of a chunk's points, the wave sums are added at the end
  constexpr int TMAX = ROM_NMAX / 16;
  const int T = npad / 16, k_row = lane >> 4, c_col = lane & 15;
  d4 acc[TMAX];
#pragma unroll
  for (int t = 0; t < TMAX; ++t) acc[t] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int q0 = 0; q0 < m; q0 += SCH) {
    const int q = q0 + tid;
    if (tid < SCH && q < m) {
      const double Fi[4] = {tq[q], tq[m + q], tq[2 * m + q], tq[3 * m + q]};
      const double wJ = tq[4 * m + q];
      double H[4] = {0.0, 0.0, 0.0, 0.0};
      for (int i = 0; i < n; ++i) {
        const double* g = Gt + (size_t)i * 4 * m + q;
        const double ri = sR[i];
#pragma unroll
        for (int b = 0; b < 4; ++b) H[b] = fma(ri, g[b * m], H[b]);
      }
      double F[4];
      kin_F(Fb, H[0], H[1], H[2], H[3], Fi, F);
      const double Fp[4] = {hq[q], hq[m + q], hq[2 * m + q], hq[3 * m + q]};
      double P[4], A[16], Fpn[4], Fp33n, xin;
      j2_point<true>(F, Fp, hq[4 * m + q], hq[5 * m + q], point_params(mp, mp2, phase, q), P, A, Fpn, Fp33n, xin);
#pragma unroll
      for (int k = 0; k < SENS_MU; ++k) {
        if (k >= n_mu) break;
        double dF[4] = {0.0, 0.0, 0.0, 0.0};
        for (int cc = 0; cc < c; ++cc) {
          const double s = sDc[cc * n_mu + k];
#pragma unroll
          for (int a = 0; a < 4; ++a) dF[a] = fma(s, Gd[((size_t)cc * 4 + a) * m + q], dF[a]);
        }
        // T1 = F_mu^-1 dF_mu; dF_mu^-1 = -T1 F_mu^-1; d(w|J|) = w|J| tr T1
        const double T1[4] = {Fi[0] * dF[0] + Fi[1] * dF[2], Fi[0] * dF[1] + Fi[1] * dF[3],
                              Fi[2] * dF[0] + Fi[3] * dF[2], Fi[2] * dF[1] + Fi[3] * dF[3]};
        const double dFi[4] = {-(T1[0] * Fi[0] + T1[1] * Fi[2]), -(T1[0] * Fi[1] + T1[1] * Fi[3]),
                               -(T1[2] * Fi[0] + T1[3] * Fi[2]), -(T1[2] * Fi[1] + T1[3] * Fi[3])};
        const double dwJ = wJ * (T1[0] + T1[3]);
        const double X[4] = {H[0] * dFi[0] + H[1] * dFi[2], H[0] * dFi[1] + H[1] * dFi[3],
                             H[2] * dFi[0] + H[3] * dFi[2], H[2] * dFi[1] + H[3] * dFi[3]};
        double AX[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          AX[r] = A[4 * r] * X[0] + A[4 * r + 1] * X[1] + A[4 * r + 2] * X[2] + A[4 * r + 3] * X[3];
        double* bq = sB + ((size_t)tid * SENS_MU + k) * 4;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int a2 = 0; a2 < 2; ++a2) {
            const double pf = P[2 * i] * Fi[2 * a2] + P[2 * i + 1] * Fi[2 * a2 + 1];
            const double af = AX[2 * i] * Fi[2 * a2] + AX[2 * i + 1] * Fi[2 * a2 + 1];
            const double pd = P[2 * i] * dFi[2 * a2] + P[2 * i + 1] * dFi[2 * a2 + 1];
            bq[2 * i + a2] = dwJ * pf + wJ * (af + pd);
          }
#pragma unroll
        for (int r = 0; r < 4; ++r) d[k][r] += wJ * AX[r] + dwJ * P[r];
      }
    }
    __syncthreads();
    const int qend = min(SCH, m - q0);
    const int qa = (wave * qend) >> 2, qb = ((wave + 1) * qend) >> 2;
    for (int ql = qa; ql < qb; ++ql) {
      const double* g = Gq + ((size_t)(q0 + ql) * 4 + k_row) * npad + c_col;
      const double bv = (c_col < n_mu) ? sB[((size_t)ql * SENS_MU + c_col) * 4 + k_row] : 0.0;
#pragma unroll
      for (int t = 0; t < TMAX; ++t)
        if (t < T) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[16 * t], bv, acc[t], 0, 0, 0);
    }
    __syncthreads();
  }
  // direct term over the workgroup; df/dmu to LDS
#pragma unroll
  for (int k = 0; k < SENS_MU; ++k) {
    if (k >= n_mu) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = d[k][r];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) sDw[(k * 4 + r) * 4 + wave] = v;
    }
  }
  // wave sums of df/dmu in a fixed order (output row k_row + 4 j of tile t,
  // column c_col); sB is free after the last chunk
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < TMAX; ++t) {
        if (t >= T) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = 16 * t + k_row + 4 * j;
          if (i < n && c_col < n_mu) {
            const double v = acc[t][j];
            sBf[i + n * c_col] = (w == 0) ? v : sBf[i + n * c_col] + v;
          }
        }
      }
    }
    __syncthreads();
  }
  if (tid < 4 * n_mu) {
    const int r = tid / n_mu, k = tid % n_mu;
    const double* w4 = sDw + (k * 4 + r) * 4;
    double s = ((w4[0] + w4[1]) + w4[2]) + w4[3];
    const double* z = zk + (size_t)p * 4 * n;
    for (int i = 0; i < n; ++i) s = fma(-z[4 * i + r], sBf[i + n * k], s);
    o[r * n_mu + k] = s * inv_area;
  }
}

}  // namespace

int rom_launch_shape_sensitivity(rom_model* h, int P, const double* Fbar, const void* state, double* out,
                                 hipStream_t s) {
  if (h->n_mu > SENS_MU || h->n_mu > 16 || h->c > 12 || h->npad > ROM_NMAX) return ROM_EUNSUPPORTED;
  const StateLayout L = rom_state_layout(h, P);
  void* st = const_cast<void*>(state);
  k_sens<<<P, 256, 0, s>>>(h->n, h->npad, h->m, h->c, h->kind, h->n_mu, h->r0, h->void_area, 1.0 / h->cell_area,
                           h->mp, h->mp2, h->phase, h->Gt, h->Gq, h->Gd, Fbar, field<double>(st, L, F_RT), field<double>(st, L, F_HC),
                           field<double>(st, L, F_TMU), field<double>(st, L, F_MU), field<int>(st, L, F_MUOK),
                           field<double>(st, L, F_ZK), out);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}
