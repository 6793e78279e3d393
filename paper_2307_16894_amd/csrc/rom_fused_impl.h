// Fused form of the online solve: one kernel launch per load step, one
// workgroup per macro point running the whole Newton loop of eq. red_newton
// on the device.
//
// Per Newton evaluation the workgroup walks the ECM points in chunks of 256
// (one lane per point): kinematics, return map and tangent (Appendix A), the
// weighted stress W = w|J| P F_mu^-T and the mapped tangent
// D = w|J| T^T A T (T: right multiplication by F_mu^-1) go to LDS.  The
// contraction K = sum_q G_q^T D_q G_q (eq. stiffnessmatrix_ecm) then runs on
// MFMA with the 4 gradient components of an ECM point as the inner
// dimension:
//   FP64  v_mfma_f64_16x16x4: B_q = [D_q G_q | W_q], so the residual
//         f = sum_q G_q^T W_q (eq. forcevector_ecm) comes out of the padding
//         column n of the stiffness tiles;
//   FP32  v_mfma_f32_16x16x4 on FP32 operands, FP32 accumulation;
//   BF16  v_mfma_f32_16x16x32_bf16, eight ECM points per instruction, FP32
//         accumulation;
// in the reduced-precision forms f is accumulated separately in FP64, so the
// residual, the return map and the solve stay FP64.  K is symmetric (the
// tangent of the appendix model is major-symmetric), so only tiles I <= J are
// contracted and the rest is mirrored.  Small n: the four waves split the
// points; large n: they split the tiles.  Gaussian elimination with partial
// pivoting in LDS gives the Newton update.  At the returned state one more
// pass over the ECM points gives Pbar (eq. eff_stress_1), sum w|J| A and
// C = sum_q G_q^T E_q (E = w|J| T^T A), and Abar = sum w|J| A - C^T K*^-1 C
// (eqs. tangent_problem_red, eff_stiffness_1) with K* the last K.
#pragma once
#include "rom_fused_args.h"

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int FCH = 256;  // ECM points per chunk
constexpr int QS = 20;    // LDS record per point in the Newton loop: D (16), W (4)



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
  return main_doubles<T>() + 16 * T * 9 + 128 + 16 * T;  // r, C, solutions, scratch, two int arrays
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


// Solve K X = B in LDS by Gaussian elimination with partial pivoting, rows
// left in place: at step k the pivot is the remaining row with the largest
// |a[r][k]| (lowest index on ties), and every other remaining row is
// eliminated against it.  a has leading dimension ld; B occupies columns
// rhs0 .. rhs0 + nrhs - 1.  The solution of unknown k is written to
// x[k * 4 + c].  Two barriers per elimination step, one per back step.
__device__ void gauss_solve(double* a, int ld, int n, int rhs0, int nrhs, int* sStep, int* sOrder, double* x) {
  const int tid = threadIdx.x, lane = tid & 63;
  for (int i = tid; i < n; i += blockDim.x) sStep[i] = n;  // n: not yet a pivot
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = n;
      for (int i = lane; i < n; i += 64) {
        if (sStep[i] == n) {
          const double v = fabs(a[i * ld + k]);
          if (v > best) {
            best = v;
            bi = i;
          }
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
      if (lane == 0) {
        if (bi == n)  // only non-finite entries left: take the first remaining row
          for (bi = 0; bi < n - 1 && sStep[bi] != n; ++bi) {
          }
        sOrder[k] = bi;
        sStep[bi] = k;
      }
    }
    __syncthreads();
    const int pr = sOrder[k];
    const double inv = 1.0 / a[pr * ld + k];
    const int nk = n - 1 - k;
    const int ncols = nk + nrhs;
    for (int idx = tid; idx < n * ncols; idx += blockDim.x) {
      const int r = idx / ncols, jj = idx - r * ncols;
      if (sStep[r] < n) continue;  // already a pivot row (includes pr)
      const int j = (jj < nk) ? k + 1 + jj : rhs0 + (jj - nk);
      a[r * ld + j] = fma(-a[r * ld + k] * inv, a[pr * ld + j], a[r * ld + j]);
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int pr = sOrder[k];
    const double inv = 1.0 / a[pr * ld + k];
    for (int idx = tid; idx < n * nrhs; idx += blockDim.x) {
      const int r = idx / nrhs, c = idx - r * nrhs;
      const double xk = a[pr * ld + rhs0 + c] * inv;
      if (r == 0) x[k * 4 + c] = xk;
      if (sStep[r] < k) a[r * ld + rhs0 + c] = fma(-a[r * ld + k], xk, a[r * ld + rhs0 + c]);
    }
    __syncthreads();
  }
}

// G_q[b][16 J + c] for the four gradient components b and all column blocks J.
template <int T>
__device__ __forceinline__ void load_g(double (&g)[4][T], const double* __restrict__ Gp, int c_col) {
  constexpr int NPAD = 16 * T;
#pragma unroll
  for (int J = 0; J < T; ++J)
#pragma unroll
    for (int b = 0; b < 4; ++b) g[b][J] = Gp[b * NPAD + 16 * J + c_col];
}

// Upper-triangle tile t (column-major over J, then I <= J) -> (I, J).
__host__ __device__ constexpr int tile_I(int t) {
  int J = 0;
  while (t > J) {
    t -= J + 1;
    ++J;
  }
  return t;
}
__host__ __device__ constexpr int tile_J(int t) {
  int J = 0;
  while (t > J) {
    t -= J + 1;
    ++J;
  }
  return J;
}

__device__ __forceinline__ __bf16 to_bf16(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (operands are finite)
  return __builtin_bit_cast(__bf16, (uint16_t)(u >> 16));
}

enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };
template <int PREC>
struct Acc {
  typedef f4 type;
};
template <>
struct Acc<PREC_F64> {
  typedef d4 type;
};

// Contraction of points [qa, qb) of the chunk into the tiles t = W, W + TW, ...
// (TW = 1: all tiles).  FP64 also accumulates f in column n of the tiles; the
// reduced-precision forms add G_q[k][j] W_q[k] to fpart (FP64) when do_f.
template <int T, int PREC, int W, int TW>
__device__ __forceinline__ void contract(typename Acc<PREC>::type* acc, double (&fpart)[T], bool do_f,
                                         const double* __restrict__ Gq, const double* sQ, int q0, int qa, int qb,
                                         int n, int k_row, int c_col) {
  constexpr int NPAD = 16 * T;
  constexpr int NT = T * (T + 1) / 2;
  if (qa >= qb) return;
  if constexpr (PREC != PREC_BF16) {
    // one ECM point per step; the next point's G is loaded during this point's MFMAs
    double gc[4][T];
    load_g<T>(gc, Gq + (size_t)(q0 + qa) * 4 * NPAD, c_col);
    for (int ql = qa; ql < qb; ++ql) {
      double gn[4][T];
      load_g<T>(gn, Gq + (size_t)(q0 + min(ql + 1, qb - 1)) * 4 * NPAD, c_col);
      const double* rq = sQ + ql * QS;
      const double d0 = rq[4 * k_row], d1 = rq[4 * k_row + 1], d2 = rq[4 * k_row + 2], d3 = rq[4 * k_row + 3];
      const double wk = rq[16 + k_row];
      double Aop[T], Bop[T];
#pragma unroll
      for (int J = 0; J < T; ++J) {
        const int col = 16 * J + c_col;
        Aop[J] = (k_row == 0) ? gc[0][J] : (k_row == 1) ? gc[1][J] : (k_row == 2) ? gc[2][J] : gc[3][J];
        const double h = d0 * gc[0][J] + d1 * gc[1][J] + d2 * gc[2][J] + d3 * gc[3][J];
        if constexpr (PREC == PREC_F64) {
          Bop[J] = (col < n) ? h : ((col == n) ? wk : 0.0);
        } else {
          Bop[J] = (col < n) ? h : 0.0;
          if (do_f) fpart[J] = fma(Aop[J], wk, fpart[J]);
        }
      }
#pragma unroll
      for (int t = W, u = 0; t < NT; t += TW, ++u) {
        if constexpr (PREC == PREC_F64)
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(Aop[tile_I(t)], Bop[tile_J(t)], acc[u], 0, 0, 0);
        else
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)Aop[tile_I(t)], (float)Bop[tile_J(t)], acc[u], 0,
                                                         0, 0);
      }
#pragma unroll
      for (int b2 = 0; b2 < 4; ++b2)
#pragma unroll
        for (int J = 0; J < T; ++J) gc[b2][J] = gn[b2][J];
    }
  } else {
    // eight ECM points per step: lane group g = k_row holds points 2g, 2g + 1
    // of the step; inner index k = 8 g + 4 h + b (point 2g + h, component b)
    for (int qs = qa; qs < qb; qs += 8) {
      float D[2][16];
      double Wv[2][4];
      bool live[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int ql = qs + 2 * k_row + h;
        live[h] = ql < qb;
        const double* rq = sQ + (live[h] ? ql : qa) * QS;
#pragma unroll
        for (int k = 0; k < 16; ++k) D[h][k] = live[h] ? (float)rq[k] : 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) Wv[h][k] = live[h] ? rq[16 + k] : 0.0;
      }
      bf8 Aop[T], Bop[T];
#pragma unroll
      for (int J = 0; J < T; ++J) {
        const int col = 16 * J + c_col;
        double g[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int ql = qs + 2 * k_row + h;
          const double* Gp = Gq + (size_t)(q0 + (live[h] ? ql : qa)) * 4 * NPAD + col;
#pragma unroll
          for (int b = 0; b < 4; ++b) g[h][b] = live[h] ? Gp[b * NPAD] : 0.0;
        }
        if (do_f) {
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int b = 0; b < 4; ++b) fpart[J] = fma(g[h][b], Wv[h][b], fpart[J]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float g0 = (float)g[h][0], g1 = (float)g[h][1], g2 = (float)g[h][2], g3 = (float)g[h][3];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            Aop[J][4 * h + b] = to_bf16((float)g[h][b]);
            const float hv = D[h][4 * b] * g0 + D[h][4 * b + 1] * g1 + D[h][4 * b + 2] * g2 + D[h][4 * b + 3] * g3;
            Bop[J][4 * h + b] = to_bf16(col < n ? hv : 0.0f);
          }
        }
      }
#pragma unroll
      for (int t = W, u = 0; t < NT; t += TW, ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop[tile_I(t)], Bop[tile_J(t)], acc[u], 0, 0, 0);
    }
  }
}

// Store (ACCUM: add) the tiles t = W, W + TW, ... into sK (ld NPAD); when
// MIRROR, also the transposed tile below the diagonal.
template <int T, int PREC, int W, int TW>
__device__ __forceinline__ void store_acc(const typename Acc<PREC>::type* acc, double* sK, bool accum, bool mirror,
                                          int k_row, int c_col) {
  constexpr int NPAD = 16 * T;
  constexpr int NT = T * (T + 1) / 2;
#pragma unroll
  for (int t = W, u = 0; t < NT; t += TW, ++u) {
    const int I = tile_I(t), J = tile_J(t);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // output layouts: FP64 row = k_row + 4 j, FP32 accumulators row = 4 k_row + j
      const int row = 16 * I + (PREC == PREC_F64 ? k_row + 4 * j : 4 * k_row + j), col = 16 * J + c_col;
      double v = (double)acc[u][j];
      if (accum) v += sK[row * NPAD + col];
      sK[row * NPAD + col] = v;
      if (mirror && I < J) sK[col * NPAD + row] = v;
    }
  }
}

// The whole load step of macro point p on one workgroup.  SPLIT 0: the four
// waves split the ECM points of a chunk; SPLIT 1: they split the tiles.
template <int T, int PREC, int SPLIT>
__device__ void solve_point(const FusedArgs& a, const int p, double* smem) {
  constexpr int NPAD = 16 * T;
  constexpr int NT = T * (T + 1) / 2;
  constexpr int MAT = main_doubles<T>();
  constexpr int ECH = ech<T>();
  double* sQ = smem;              // [FCH][QS] chunk records
  double* sK = smem;              // [NPAD][NPAD] [K | f] and its LU (after the contraction)
  double* sE = smem + NPAD * NPAD;  // [ECH][16] E records of the effective-quantity pass
  double* sR = smem + MAT;        // [NPAD] current r
  double* sC = sR + NPAD;         // [NPAD][4] C = sum_q G_q^T E_q, then K^-1 C
  double* sSol = sC + 4 * NPAD;   // [NPAD][4] solutions of the eliminations
  double* sX = sSol + 4 * NPAD;   // reduction scratch (128)
  int* sStep = reinterpret_cast<int*>(sX + 128);  // [NPAD] elimination step of each row
  int* sOrder = sStep + NPAD;                     // [NPAD] pivot row of each step

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = a.n, m = a.m;
  if (a.active && !a.active[p]) return;  // skipped: state and outputs untouched
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
  // initial guess: the committed r, plus the predicted increment with a warm start
  for (int i = tid; i < NPAD; i += 256) {
    double v = 0.0;
    if (i < n) {
      v = a.rc[(size_t)p * n + i];
      if (a.dr) v += (double)a.dr[(size_t)p * n + i];
      a.rg[(size_t)p * n + i] = v;
    }
    sR[i] = v;
  }
  double Fb[4] = {a.Fbar[4 * (size_t)p], a.Fbar[4 * (size_t)p + 1], a.Fbar[4 * (size_t)p + 2],
                  a.Fbar[4 * (size_t)p + 3]};
  // load-step cutting: targets F0 + (t / 2^D) (Fbar - F0) on the segment from
  // the committed F0; sF0 / sF1 hold the two ends
  double* sF0 = sX + 96;
  double* sF1 = sX + 100;
  if (tid < 4) {
    sF0[tid] = a.fbc[4 * (size_t)p + tid];
    sF1[tid] = Fb[tid];
  }
  const int full = 1 << a.max_sub;
  int t_done = 0, stride = full, total = 0;
  const double* tmu = a.tmu + (size_t)p * 5 * m;
  const double* hc = a.hc + (size_t)p * 6 * m;
  double* ht = a.ht + (size_t)p * 6 * m;
  __syncthreads();

  const int k_row = lane >> 4, c_col = lane & 15;
  int status = ROM_ST_MAXITER, iters = 0;
  double rn = 0.0, rn0 = 0.0;
  bool fell_back = false;
  for (int attempt = 0;; ++attempt) {
  for (int it = 0; it < a.max_iter; ++it) {
    constexpr bool QSPLIT = (SPLIT == 0);             // waves split the points (else the tiles)
    constexpr int NACC = QSPLIT ? NT : (NT + 3) / 4;  // large n: waves split the tiles
    typedef typename Acc<PREC>::type AccV;
    AccV acc[NACC];
#pragma unroll
    for (int t = 0; t < NACC; ++t) acc[t] = (AccV){0, 0, 0, 0};
    double fpart[T];  // FP64 residual partials of the reduced-precision forms
#pragma unroll
    for (int J = 0; J < T; ++J) fpart[J] = 0.0;

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
      // contraction of the chunk
      const int qend = min(FCH, m - q0);
      if constexpr (QSPLIT) {
        contract<T, PREC, 0, 1>(acc, fpart, true, a.Gq, sQ, q0, wave * 64, min(wave * 64 + 64, qend), n, k_row,
                                c_col);
      } else {
        switch (wave) {
          case 0: contract<T, PREC, 0, 4>(acc, fpart, true, a.Gq, sQ, q0, 0, qend, n, k_row, c_col); break;
          case 1: contract<T, PREC, 1, 4>(acc, fpart, false, a.Gq, sQ, q0, 0, qend, n, k_row, c_col); break;
          case 2: contract<T, PREC, 2, 4>(acc, fpart, false, a.Gq, sQ, q0, 0, qend, n, k_row, c_col); break;
          default: contract<T, PREC, 3, 4>(acc, fpart, false, a.Gq, sQ, q0, 0, qend, n, k_row, c_col); break;
        }
      }
      __syncthreads();
    }
    // [K | f] into LDS (ld NPAD); K's lower part by symmetry
    if constexpr (QSPLIT) {
      for (int w = 0; w < 4; ++w) {
        if (wave == w) store_acc<T, PREC, 0, 1>(acc, sK, w > 0, w == 3, k_row, c_col);
        __syncthreads();
      }
    } else {
      switch (wave) {
        case 0: store_acc<T, PREC, 0, 4>(acc, sK, false, true, k_row, c_col); break;
        case 1: store_acc<T, PREC, 1, 4>(acc, sK, false, true, k_row, c_col); break;
        case 2: store_acc<T, PREC, 2, 4>(acc, sK, false, true, k_row, c_col); break;
        default: store_acc<T, PREC, 3, 4>(acc, sK, false, true, k_row, c_col); break;
      }
      __syncthreads();
    }
    if constexpr (PREC != PREC_F64) {
      // f in FP64: sum over the lane groups, then over the waves in a fixed order
#pragma unroll
      for (int J = 0; J < T; ++J) {
        double v = fpart[J];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (k_row == 0) sSol[wave * NPAD + 16 * J + c_col] = v;
      }
      __syncthreads();
      if (tid < n) {
        const double v = QSPLIT ? ((sSol[tid] + sSol[NPAD + tid]) + sSol[2 * NPAD + tid]) + sSol[3 * NPAD + tid]
                                : sSol[tid];
        sK[tid * NPAD + n] = v;
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
    if (it == 0) rn0 = rn;
    if (stop) break;
    // warm start judged by plain Newton: no tenfold drop of ||f|| after two
    // updates -> restart from the committed r
    if (a.dr && attempt == 0 && !fell_back && it == 2 && !(rn <= 0.1 * rn0)) {
      fell_back = true;
      for (int i = tid; i < n; i += 256) sR[i] = a.rc[(size_t)p * n + i];
      __syncthreads();
      continue;
    }
    // Newton update: K dr = -f
    gauss_solve(sK, NPAD, n, n, 1, sStep, sOrder, sSol);
    if (tid < n) sR[tid] -= sSol[4 * tid];
    __syncthreads();
  }
  total += iters;
  if (status == ROM_ST_CONVERGED) {
    t_done += stride;
    if (t_done == full) break;
    // a converged sub-step becomes the committed start of the next attempt
    // (each thread copies the ECM points it wrote)
    double* hcw = a.hc + (size_t)p * 6 * m;
    for (int q = tid; q < m; q += 256)
#pragma unroll
      for (int k = 0; k < 6; ++k) hcw[k * m + q] = ht[k * m + q];
    for (int i = tid; i < n; i += 256) a.rc[(size_t)p * n + i] = sR[i];
    if (tid < 4) a.fbc[4 * (size_t)p + tid] = Fb[tid];
    stride = min(2 * stride, full - t_done);
  } else {
    if (stride == 1) break;  // the smallest sub-step failed too
    stride >>= 1;
    for (int i = tid; i < n; i += 256) sR[i] = a.rc[(size_t)p * n + i];
  }
  const int t_next = t_done + stride;
  const double frac = ldexp((double)t_next, -a.max_sub);
#pragma unroll
  for (int k = 0; k < 4; ++k) Fb[k] = (t_next == full) ? sF1[k] : sF0[k] + frac * (sF1[k] - sF0[k]);
  __syncthreads();
  }
  iters = total;

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
    if (o < 4 * n) sC[o] = cacc[u];
  }
#pragma unroll
  for (int k = 0; k < 20; ++k) {
    double v = (k < 4) ? accP[k] : accA[k - 4];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) sX[4 * k + wave] = v;
  }
  __syncthreads();
  // Y = K*^-1 C with K* = K of the last evaluation (still in sK, not eliminated)
  for (int idx = tid; idx < 4 * n; idx += 256) sK[(idx >> 2) * NPAD + n + 1 + (idx & 3)] = sC[idx];
  __syncthreads();
  gauss_solve(sK, NPAD, n, n + 1, 4, sStep, sOrder, sSol);
  if (tid < 20) {
    const double v = ((sX[4 * tid] + sX[4 * tid + 1]) + sX[4 * tid + 2]) + sX[4 * tid + 3];
    if (tid < 4) {
      a.Pbar[4 * (size_t)p + tid] = v * a.inv_area;
    } else {
      const int e = tid - 4, x = e >> 2, y = e & 3;
      double acc2 = v;
      for (int i = 0; i < n; ++i) acc2 = fma(-sC[4 * i + x], sSol[4 * i + y], acc2);
      a.Abar[16 * (size_t)p + e] = acc2 * a.inv_area;
    }
  }
  for (int i = tid; i < n; i += 256) a.rt[(size_t)p * n + i] = sR[i];
  if (tid == 0) {
    a.st_out[p] = (status == ROM_ST_CONVERGED && fell_back) ? ROM_ST_FALLBACK : status;
    a.it_out[p] = iters;
    a.res_out[p] = rn;
  }
  if (a.commit && status == ROM_ST_CONVERGED) {
    if (tid < 4) a.fbc[4 * (size_t)p + tid] = Fb[tid];
    for (int i = tid; i < n; i += 256) a.rc[(size_t)p * n + i] = sR[i];
    double* hcw = a.hc + (size_t)p * 6 * m;
    for (int q = tid; q < m; q += 256)
#pragma unroll
      for (int k = 0; k < 6; ++k) hcw[k * m + q] = ht[k * m + q];
  }
}

// one workgroup per point of the batch
template <int T, int PREC, int SPLIT>
__global__ __launch_bounds__(256) void k_fused(const FusedArgs a) {
  extern __shared__ double smem[];
  solve_point<T, PREC, SPLIT>(a, blockIdx.x, smem);
}

// persistent workgroups pulling points from the device-side work list
template <int T, int PREC, int SPLIT>
__global__ __launch_bounds__(256) void k_fused_queue(const FusedArgs a) {
  extern __shared__ double smem[];
  __shared__ int s_idx;
  const int nlist = *a.nlist;
  while (true) {
    if (threadIdx.x == 0) s_idx = atomicAdd(a.counter, 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= nlist) break;
    solve_point<T, PREC, SPLIT>(a, a.list[idx], smem);
    __syncthreads();
  }
}

template <int T, int PREC, int SPLIT>
int launch_one(const FusedArgs& a, int grid, int P, hipStream_t s) {
  const size_t lds = (size_t)lds_doubles<T>() * 8;
  if (grid > 0)
    k_fused_queue<T, PREC, SPLIT><<<grid, 256, lds, s>>>(a);
  else
    k_fused<T, PREC, SPLIT><<<P, 256, lds, s>>>(a);
  return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
}

template <int T, int PREC>
int launch_prec(const FusedArgs& a, int split, int grid, int P, hipStream_t s) {
  if constexpr (T <= 5) {
    if (split == 0) return launch_one<T, PREC, 0>(a, grid, P, s);
  }
  return launch_one<T, PREC, 1>(a, grid, P, s);
}

template <int T>
int fused_launch(const FusedArgs& a, int prec, int split, int grid, int P, hipStream_t s) {
  if (prec == ROM_DT_F64) return launch_prec<T, PREC_F64>(a, split, grid, P, s);
  if (prec == ROM_DT_F32) return launch_prec<T, PREC_F32>(a, split, grid, P, s);
  return launch_prec<T, PREC_BF16>(a, split, grid, P, s);
}

template <typename K>
int set_lds(K kern, size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds) == hipSuccess
             ? ROM_OK
             : ROM_EHIP;
}

template <int T, int PREC, int SPLIT>
int setup_one() {
  const size_t lds = (size_t)lds_doubles<T>() * 8;
  int rc = set_lds(&k_fused<T, PREC, SPLIT>, lds);
  if (rc == ROM_OK) rc = set_lds(&k_fused_queue<T, PREC, SPLIT>, lds);
  return rc;
}

template <int T>
int fused_setup() {
  int rc = ROM_OK;
  if constexpr (T <= 5) {
    if (rc == ROM_OK) rc = setup_one<T, PREC_F64, 0>();
    if (rc == ROM_OK) rc = setup_one<T, PREC_F32, 0>();
    if (rc == ROM_OK) rc = setup_one<T, PREC_BF16, 0>();
  }
  if (rc == ROM_OK) rc = setup_one<T, PREC_F64, 1>();
  if (rc == ROM_OK) rc = setup_one<T, PREC_F32, 1>();
  if (rc == ROM_OK) rc = setup_one<T, PREC_BF16, 1>();
  return rc;
}

}  // namespace

#define ROM_FUSED_DEFINE(T)                                                                             \
  int rom_fused_launch_##T(const FusedArgs& a, int prec, int split, int grid, int P, hipStream_t s) { \
    return fused_launch<T>(a, prec, split, grid, P, s);                                                \
  }                                                                                                    \
  int rom_fused_setup_##T() { return fused_setup<T>(); }
