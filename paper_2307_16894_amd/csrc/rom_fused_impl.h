// Fused form of the online solve: one kernel launch per load step, one
// workgroup per macro point running the whole Newton loop of eq. red_newton
// on the device.
//
// Per Newton evaluation the workgroup walks the ECM points in chunks of 256
// (one lane per point): kinematics, return map and tangent (Appendix A), and
// an LDS record per point with
//   D = w|J| T^T A T    (T: right multiplication by F_mu^-1),
//   W = w|J| P F_mu^-T and F_mu.
// The contraction then runs on MFMA with the four gradient components of an
// ECM point as the inner dimension, as sum_q A_q^T B_q with
//   A_q = [G_q | R_q]            (R_q: four rows carrying F_mu, see below),
//   B_q = [D_q G_q | W_q | E_q]  (columns n, n + 1 .. n + 4; E = D T^-1 =
//                                 w|J| T^T A, the mapped tangent),
// padded to 16 T rows and columns (16 T >= n + 5).  B_q itself comes out of
// an MFMA per column tile, D_q [G_q | V_q] with V_q = T^-1 in the columns
// n + 1 .. n + 4 (and W_q put in column n), so that each lane loads only its
// own gradient component of G_q.  One contraction therefore
// gives, at the state of the evaluation,
//   K = sum_q G_q^T D_q G_q                (eq. stiffnessmatrix_ecm),
//   f = sum_q G_q^T W_q                    (eq. forcevector_ecm, column n),
//   C = sum_q G_q^T E_q                    (the right-hand sides of the four
//                                           tangent problems, eq. tangent_problem_red),
// and through the rows R_q (row n + 2i + J carries F_mu[J][.] against the
// components (i, .) of W and E, which undoes the F_mu^-T of W and of T^T)
//   sum_q w|J| P  and  sum_q w|J| A        (eqs. eff_stress_1, eff_stiffness_1).
// Only the tiles I <= J are contracted (K and the padding blocks are symmetric
// or above the diagonal); the rest of K is mirrored.  The padding block
// starts at pad_base(n): n, or the next tile boundary when the block would
// cross one (n mod 16 >= 12), so that it lies in the last tile row and column
// (an entry of its rows against its columns in a tile below the diagonal
// would not be contracted).
//   FP64  v_mfma_f64_16x16x4f64 (H = D [G | V] on v_mfma_f64_4x4x4f64);
//   FP32  v_mfma_f32_16x16x4f32 on FP32 operands, FP32 accumulation;
//   BF16  v_mfma_f32_16x16x32_bf16, eight ECM points per instruction, FP32
//         accumulation (H on v_mfma_f32_16x16x16_bf16);
// in the reduced-precision forms f and sum w|J| P are accumulated separately
// in FP64, so the residual, the stress, the return map and the solve stay
// FP64 (K, C and sum w|J| A carry the contraction precision).  Small n: the
// four waves split the points; large n: they split the tiles.  Gauss-Jordan
// elimination with partial pivoting on [K | f | C], with the matrix spread
// over the registers of the workgroup, gives the Newton update and
// K^-1 C; at the returned state Abar = sum w|J| A - C^T K*^-1 C with K* the K
// of the last evaluation (Sec. 3.3).
#pragma once
#include "rom_fused_args.h"

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int FCH = 256;  // ECM points per chunk of the material phase
constexpr int CCH = 128;  // ECM points per contraction chunk (records staged in LDS by the phased kernel)
static_assert(FCH % CCH == 0 && CCH * 2 == 256, "contraction chunks tile the material chunks; two lanes per record");
constexpr int QS = 24;    // LDS record per point
constexpr int R_D = 0, R_W = 16, R_FM = 20;

template <int T>
constexpr int ldk() {
  return 16 * T + 1;  // leading dimension of [K | f | C] in LDS
}
template <int T>
constexpr int main_doubles() {
  return (FCH * QS > 16 * T * ldk<T>()) ? FCH * QS : 16 * T * ldk<T>();
}
// LDS: chunk records / [K | f | C]; then r, C copy, multipliers (2 x 128),
// pivot values (128), misc (32), pivot order and pivot exchange (ints)
template <int T>
constexpr int lds_doubles() {
  return main_doubles<T>() + 16 * T + 4 * 16 * T + 256 + 128 + 32 + (16 * T + 8) / 2;
}
// phased contraction kernel: records of one contraction chunk / [K | f | C]
template <int T>
constexpr int cs_main_doubles() {
  return (CCH * QS > 16 * T * ldk<T>()) ? CCH * QS : 16 * T * ldk<T>();
}
template <int T>
constexpr int cs_lds_doubles() {
  return cs_main_doubles<T>() + 16 * T + 4 * 16 * T + 256 + 128 + 32 + (16 * T + 8) / 2;
}

// F = Fbar + H F_mu^-1 with H = sum_i r_i G_i(q) (argument of P in eq.
// forcevector_ecm), from the four components of H.  Helpers that different
// kernels share are written with explicit fma (and the library is built with
// multiply-add fusion within expressions only): fusion left to the code
// generator depends on the surrounding code, and the fused and phased kernels
// would round differently.
__device__ __forceinline__ void kin_F(const double Fb[4], double H0, double H1, double H2, double H3,
                                      const double Fi[4], double F[4]) {
  F[0] = fma(H1, Fi[2], fma(H0, Fi[0], Fb[0]));
  F[1] = fma(H1, Fi[3], fma(H0, Fi[1], Fb[1]));
  F[2] = fma(H3, Fi[2], fma(H2, Fi[0], Fb[2]));
  F[3] = fma(H3, Fi[3], fma(H2, Fi[1], Fb[3]));
}

// F at ECM point q with H = sum_i r_i G_i(q) accumulated mode by mode (one
// fma per mode and component, in mode order); r is read from LDS.  The loads
// of eight modes are issued before their use, so that they are in flight
// together (issued one at a time the loop is a chain of memory round trips).
__device__ __forceinline__ void kinematics(int n, int m, int q, const double* __restrict__ Gt, const double* sR,
                                           const double Fb[4], const double Fi[4], double F[4]) {
  double H0 = 0.0, H1 = 0.0, H2 = 0.0, H3 = 0.0;
  const double* g = Gt + q;
  const size_t st = 4 * (size_t)m;
  int i = 0;
  for (; i + 8 <= n; i += 8) {
    double v[8][4];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int b = 0; b < 4; ++b) v[u][b] = g[u * st + b * m];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double ri = sR[i + u];
      H0 = fma(ri, v[u][0], H0);
      H1 = fma(ri, v[u][1], H1);
      H2 = fma(ri, v[u][2], H2);
      H3 = fma(ri, v[u][3], H3);
    }
    g += 8 * st;
  }
  for (; i < n; ++i) {
    const double ri = sR[i];
    H0 = fma(ri, g[0], H0);
    H1 = fma(ri, g[m], H1);
    H2 = fma(ri, g[2 * m], H2);
    H3 = fma(ri, g[3 * m], H3);
    g += st;
  }
  kin_F(Fb, H0, H1, H2, H3, Fi, F);
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)u, l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
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

// Tile split (large n): the column tiles J (J + 1 tiles I <= J each) are dealt
// to the four waves largest first, each to the least loaded wave, so that a
// wave forms B for its own columns only; owns<T, W, TW>(J) is true for the
// columns of wave W (all columns when TW = 1).
template <int T>
constexpr int col_owner(int J) {
  int load[4] = {0, 0, 0, 0}, owner = 0;
  for (int c = T - 1; c >= 0; --c) {
    int w = 0;
    for (int k = 1; k < 4; ++k)
      if (load[k] < load[w]) w = k;
    load[w] += c + 1;
    if (c == J) owner = w;
  }
  return owner;
}
template <int T>
constexpr int split_tiles() {
  int load[4] = {0, 0, 0, 0};
  for (int c = T - 1; c >= 0; --c) {
    int w = 0;
    for (int k = 1; k < 4; ++k)
      if (load[k] < load[w]) w = k;
    load[w] += c + 1;
  }
  int mx = 0;
  for (int k = 0; k < 4; ++k) mx = load[k] > mx ? load[k] : mx;
  return mx;
}
template <int T, int W, int TW>
constexpr bool owns(int J) {
  return TW == 1 || col_owner<T>(J) == W;
}

// Per-lane constants of the padding rows and columns (n is the same for all
// points of a launch):
//   A side, tile row In = n / 16: lane row 16 In + c_col in [n, n + 4) takes
//     F_mu[J'][j] from the record when its component i matches (row n + 2i' + J');
//   B side, tiles In and In + 1: lane column n takes W[k_row]; lane columns
//     n + 1 + (k, l) feed the H MFMA with V[(k', s)][(k, l)] = delta(k', k)
//     F_mu[l][s] (the entries of T^-1, right multiplication by F_mu) in place
//     of G, so that H = D V = E there.
// First row / column of the padding block: n, or the next tile boundary when
// its five columns would cross one (n mod 16 >= 12), so that the whole block
// lies in the last tile row and column (every padding entry in tiles I <= J;
// tiles 0 .. T - 2 hold gradient entries only); the columns in between are
// zero.
__host__ __device__ __forceinline__ int pad_base(int n) { return (n & 15) <= 11 ? n : (n + 15) & ~15; }

struct Pad {
  int nb;       // pad_base(n)
  int In;       // tile row / column of index nb
  bool a_use;   // this lane's A value in tile In comes from the record
  int a_off;    // its record offset
  int w_use;    // bit t: this lane's B value in tile In + t is W[k_row]
  int v_use;    // bit t: this lane's H-MFMA B value in tile In + t is V
  int v_zero;   // bit t: ... and that V entry is zero
  int v_off0, v_off1;  // record offsets of the V entries
};

__device__ __forceinline__ Pad make_pad(int n, int k_row, int c_col) {
  Pad d;
  d.nb = pad_base(n);
  d.In = d.nb >> 4;
  const int row = 16 * d.In + c_col, ar = row - d.nb;
  d.a_use = (ar >= 0 && ar < 4 && (ar >> 1) == (k_row >> 1));
  d.a_off = d.a_use ? R_FM + 2 * (ar & 1) + (k_row & 1) : R_FM;
  d.w_use = d.v_use = d.v_zero = 0;
  int off[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int dc = 16 * (d.In + t) + c_col - d.nb;
    off[t] = R_FM;
    if (dc == 0) d.w_use |= 1 << t;
    if (dc >= 1 && dc <= 4) {
      const int y = dc - 1;  // (k, l) = (y >> 1, y & 1); k_row = (k', s)
      d.v_use |= 1 << t;
      if ((k_row >> 1) != (y >> 1)) d.v_zero |= 1 << t;
      off[t] = R_FM + 2 * (y & 1) + (k_row & 1);
    }
  }
  d.v_off0 = off[0];
  d.v_off1 = off[1];
  return d;
}

// Loads of one ECM point for the FP64 / FP32 contraction: the lane's own
// gradient component of every tile (A side of K, B side of H).
template <int T>
struct GLoad {
  double a[T];
};

template <int T>
__device__ __forceinline__ void load_g(GLoad<T>& L, const double* __restrict__ Gp, int k_row, int c_col) {
  constexpr int NPAD = 16 * T;
#pragma unroll
  for (int I = 0; I < T; ++I) L.a[I] = Gp[k_row * NPAD + 16 * I + c_col];
}

// MFMA operands of one ECM point: A[I] for tile row I, B[J] for tile column J.
template <int T>
struct Ops {
  double A[T], B[T];
};

// Operands of the point with record rq and loads L (and, in the
// reduced-precision forms, its FP64 residual partial G_q[k_row][col] W_q[k_row]).
// H = D [G | V] comes from an MFMA per column tile, B = the lane's G
// component, and H[k_row][col] lands in lane (k_row, c_col), where the
// contraction wants it as its B operand.  FP64: v_mfma_f64_4x4x4f64, whose
// four blocks b take the columns 4b .. 4b + 3 of the tile (block b: A[i][k]
// from lane 16 k + 4 b + i, B[k][j] from lane 16 k + 4 b + j, C[i][j] to lane
// 16 i + 4 b + j), so every lane holds D[c_col mod 4][k_row]: a quarter of the
// issue cycles of the 16 x 16 x 4 form.  FP32: v_mfma_f32_16x16x4f32, output
// rows 4 k_row + j, D in A rows 0, 4, 8, 12.
template <int T, int PREC, int W, int TW>
__device__ __forceinline__ void make_ops(Ops<T>& O, double (&fpart)[T], bool do_f, const GLoad<T>& L,
                                         const double* rq, const Pad& pd, int k_row, int n, int c_col) {
  constexpr bool F64 = (PREC == PREC_F64);
  const int drow = F64 ? (c_col & 3) : (c_col >> 2);
  const double dv = rq[R_D + 4 * drow + k_row];
  const double dop = (F64 || (c_col & 3) == 0) ? dv : 0.0;
  const double xa = rq[pd.a_off], xw = rq[R_W + k_row], xv0 = rq[pd.v_off0], xv1 = rq[pd.v_off1];
  // The padding block lies in the last tile (pad_base), so the other tiles
  // take G alone, resolved at compile time.  The FP64 tile-split kernels keep
  // the selects at the run-time tile index In (and In + 1, unused): their
  // code schedule came out faster that way (264 against 286 ms per step on
  // the n = 100 four-void workload), while the compile-time form is faster
  // for every other kernel.
  constexpr bool PADC = !(PREC == PREC_F64 && TW != 1);
#pragma unroll
  for (int J = 0; J < T; ++J) {
    double g = L.a[J];
    bool wsel = false;
    if (PADC ? (J == T - 1) : (J == pd.In)) {
      g = (pd.v_use & 1) ? ((pd.v_zero & 1) ? 0.0 : xv0) : g;
      wsel = pd.w_use & 1;
    }
    if (!PADC && J == pd.In + 1) {
      g = (pd.v_use & 2) ? ((pd.v_zero & 2) ? 0.0 : xv1) : g;
      wsel = pd.w_use & 2;
    }
    double h = 0.0;
    if (!owns<T, W, TW>(J)) {
      // not this wave's column: B unused
    } else if constexpr (PREC == PREC_F64) {
      h = __builtin_amdgcn_mfma_f64_4x4x4f64(dop, g, 0.0, 0, 0, 0);
    } else {
      const f4 hz = __builtin_amdgcn_mfma_f32_16x16x4f32((float)dop, (float)g, (f4){0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
      h = (double)hz[0];
    }
    O.B[J] = wsel ? xw : h;
    double av = L.a[J];
    if (PADC ? (J == T - 1) : (J == pd.In)) av = pd.a_use ? xa : av;
    O.A[J] = av;
  }
  if constexpr (PREC != PREC_F64) {
    if (do_f) {
#pragma unroll
      for (int J = 0; J < T; ++J) fpart[J] = fma(L.a[J], xw, fpart[J]);  // columns n and above: never read
    }
  }
}

// The MFMAs of one point into the tiles of this wave (all tiles when TW = 1,
// else the tiles v = W, W + 4, ... in the order J = 0.., I = 0..J).
template <int T, int PREC, int W, int TW>
__device__ __forceinline__ void mfma_ops(typename Acc<PREC>::type* acc, const Ops<T>& O) {
  int u = 0;
#pragma unroll
  for (int J = 0; J < T; ++J) {
#pragma unroll
    for (int I = 0; I <= J; ++I) {
      if (owns<T, W, TW>(J)) {
        if constexpr (PREC == PREC_F64)
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(O.A[I], O.B[J], acc[u], 0, 0, 0);
        else
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)O.A[I], (float)O.B[J], acc[u], 0, 0, 0);
        ++u;
      }
    }
  }
}

// Contraction of points [qa, qb) of the chunk (FP64 / FP32 operands).  The
// G loads run two points ahead (three rotating register sets) and the
// operands of the next point are formed while the current point's MFMAs
// execute.
template <int T, int PREC, int W, int TW>
__device__ __forceinline__ void contract_range(typename Acc<PREC>::type* acc, double (&fpart)[T], bool do_f,
                                               const double* __restrict__ Gq, const double* sQ, int q0, int qa,
                                               int qb, const Pad& pd, int n, int k_row, int c_col) {
  constexpr int NPAD = 16 * T;
  if (qa >= qb) return;
  const double* Gb = Gq + (size_t)q0 * 4 * NPAD;
  const int ql_max = qb - 1;
  GLoad<T> L0, L1, L2;
  load_g<T>(L0, Gb + (size_t)qa * 4 * NPAD, k_row, c_col);
  load_g<T>(L1, Gb + (size_t)min(qa + 1, ql_max) * 4 * NPAD, k_row, c_col);
  Ops<T> O;
  make_ops<T, PREC, W, TW>(O, fpart, do_f, L0, sQ + qa * QS, pd, k_row, n, c_col);
  for (int ql = qa; ql < qb; ql += 3) {
    load_g<T>(L2, Gb + (size_t)min(ql + 2, ql_max) * 4 * NPAD, k_row, c_col);
    mfma_ops<T, PREC, W, TW>(acc, O);
    if (ql + 1 >= qb) break;
    make_ops<T, PREC, W, TW>(O, fpart, do_f, L1, sQ + (ql + 1) * QS, pd, k_row, n, c_col);
    load_g<T>(L0, Gb + (size_t)min(ql + 3, ql_max) * 4 * NPAD, k_row, c_col);
    mfma_ops<T, PREC, W, TW>(acc, O);
    if (ql + 2 >= qb) break;
    make_ops<T, PREC, W, TW>(O, fpart, do_f, L2, sQ + (ql + 2) * QS, pd, k_row, n, c_col);
    load_g<T>(L1, Gb + (size_t)min(ql + 4, ql_max) * 4 * NPAD, k_row, c_col);
    mfma_ops<T, PREC, W, TW>(acc, O);
    if (ql + 3 >= qb) break;
    make_ops<T, PREC, W, TW>(O, fpart, do_f, L0, sQ + (ql + 3) * QS, pd, k_row, n, c_col);
  }
}

// BF16: eight ECM points per instruction.  Up to four column tiles lane
// group g = k_row holds points g and g + 4 of the step, inner index
// k = 8 g + 4 h + b (point g + 4 h, component b), and H = D [G | V] of a
// column tile comes from two
// v_mfma_f32_16x16x16_bf16, four points each: rows (point, b), inner index
// (point, c), A = D block-diagonal (lane 16 g + i holds row i mod 4 of the D
// of its own point where i / 4 = g, else zeros), B = the lane's G (or V) in
// bf16, so that lane 16 g + c receives column c of H for its own point; f is
// accumulated in FP64 from the FP64 G loads.  Wider, lane group g holds
// points 2 g and 2 g + 1 (k = 8 g + 4 h + b for point 2 g + h) and each lane
// forms its column of H in FP32 with fma from the FP32 D and G (the H
// product measured slower there: 114 against 113 ms per step at n = 100).
// The loads of one column tile run while the previous tile is formed.
struct G8 {
  double g[2][4];  // [point h][component b] of one column tile
};

typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

// G of the lane's two points in one column tile (HM: the points g and g + 4
// of the H-product form, else 2 g and 2 g + 1)
template <int T, bool HM>
__device__ __forceinline__ void load_g8(G8& L, const double* __restrict__ Gb, int qs, int J, int qa, int qb,
                                        int k_row, int c_col) {
  constexpr int NPAD = 16 * T;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int ql = HM ? qs + k_row + 4 * h : qs + 2 * k_row + h;
    const double* Gp = Gb + (size_t)(ql < qb ? ql : qa) * 4 * NPAD + 16 * J + c_col;
#pragma unroll
    for (int b = 0; b < 4; ++b) L.g[h][b] = Gp[b * NPAD];
  }
}

// One step of eight points from qs (FULL: all eight below qb, no selects of
// dead points), the first column tile of the next step prefetched into cur.
template <int T, int W, int TW, bool FULL>
__device__ __forceinline__ void bf16_step(f4* acc, double (&fpart)[T], bool do_f, G8& cur, const double* __restrict__ Gb,
                                          const double* sQ, int qs, int qa, int qb, const Pad& pd, int k_row,
                                          int c_col) {
  const int arow = 16 * pd.In + c_col - pd.nb;  // padding-row offset of this lane in tile In
  const bool apad = arow >= 0 && arow < 4, aodd = arow & 1;
  const bool dlane = (c_col >> 2) == k_row;  // lanes holding D in the A operand of the H products
  bf4 Dh[2];
  float Fm[2][4];
  double Wv[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int ql = qs + k_row + 4 * h;
    const bool live = FULL || ql < qb;
    const double* rq = sQ + (live ? ql : qa) * QS;
    const float* rf = reinterpret_cast<const float*>(rq + R_D) + 4 * (c_col & 3);
#pragma unroll
    for (int k = 0; k < 4; ++k) Dh[h][k] = (__bf16)((live && dlane) ? rf[k] : 0.0f);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Fm[h][k] = live ? (float)rq[R_FM + k] : 0.0f;
      Wv[h][k] = live ? rq[R_W + k] : 0.0;
    }
  }
  G8 nxt;
  bf8 Aop[T];
  int u = 0;
#pragma unroll
  for (int J = 0; J < T; ++J) {
    if (J + 1 < T)
      load_g8<T, true>(nxt, Gb, qs, J + 1, qa, qb, k_row, c_col);
    else
      load_g8<T, true>(nxt, Gb, min(qs + 8, qb - 1), 0, qa, qb, k_row, c_col);
    const int col = 16 * J + c_col, dc = col - pd.nb;
    const bool ecol = dc >= 1 && dc <= 4, wcol = dc == 0;
    const int ek = (dc - 1) >> 1, el = (dc - 1) & 1;
    // f partials of every lane (those of the columns n and above are never read)
    if (do_f) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int b = 0; b < 4; ++b) fpart[J] = fma(cur.g[h][b], Wv[h][b], fpart[J]);
    }
    bf4 Gh[2];  // B operand of the H products
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float g[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) g[c] = (float)cur.g[h][c];
      if (J < T - 1) {
        // tiles left of the padding block (resolved at compile time): G in
        // both operands
#pragma unroll
        for (int c = 0; c < 4; ++c) Gh[h][c] = (__bf16)g[c];
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          // V[c][(ek, el)] for c = (k', s): F_mu[el][s] when k' = ek
          const float fv = el ? Fm[h][2 + (c & 1)] : Fm[h][c & 1];
          Gh[h][c] = (__bf16)(ecol ? (((c >> 1) == ek) ? fv : 0.0f) : g[c]);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          float av = g[b];
          if (apad)  // the last tile is the tile row of the padding block
            av = ((arow >> 1) == (b >> 1)) ? (aodd ? Fm[h][2 + (b & 1)] : Fm[h][b & 1]) : 0.0f;
          Aop[J][4 * h + b] = (__bf16)av;
        }
      }
    }
    if (J < T - 1) Aop[J] = __builtin_shufflevector(Gh[0], Gh[1], 0, 1, 2, 3, 4, 5, 6, 7);
    if (owns<T, W, TW>(J)) {
      bf8 Bop;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f4 Hv = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, Dh[h]), __builtin_bit_cast(s4, Gh[h]),
                                                               (f4){0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
#pragma unroll
        for (int b = 0; b < 4; ++b) Bop[4 * h + b] = (__bf16)((J == T - 1 && wcol) ? (float)Wv[h][b] : Hv[b]);
      }
#pragma unroll
      for (int I = 0; I <= J; ++I) {
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop[I], Bop, acc[u], 0, 0, 0);
        ++u;
      }
    }
    cur = nxt;
  }
}

template <int T, int W, int TW>
__device__ __forceinline__ void contract_range_bf16_mfma(f4* acc, double (&fpart)[T], bool do_f,
                                                    const double* __restrict__ Gq, const double* sQ, int q0, int qa,
                                                    int qb, const Pad& pd, int n, int k_row, int c_col) {
  constexpr int NPAD = 16 * T;
  if (qa >= qb) return;
  const double* Gb = Gq + (size_t)q0 * 4 * NPAD;
  G8 cur;
  load_g8<T, true>(cur, Gb, qa, 0, qa, qb, k_row, c_col);
  int qs = qa;
  for (; qs + 8 <= qb; qs += 8) bf16_step<T, W, TW, true>(acc, fpart, do_f, cur, Gb, sQ, qs, qa, qb, pd, k_row, c_col);
  if (qs < qb) bf16_step<T, W, TW, false>(acc, fpart, do_f, cur, Gb, sQ, qs, qa, qb, pd, k_row, c_col);
}

template <int T, int W, int TW>
__device__ __forceinline__ void contract_range_bf16_valu(f4* acc, double (&fpart)[T], bool do_f,
                                                    const double* __restrict__ Gq, const double* sQ, int q0, int qa,
                                                    int qb, const Pad& pd, int n, int k_row, int c_col) {
  constexpr int NPAD = 16 * T;
  if (qa >= qb) return;
  const double* Gb = Gq + (size_t)q0 * 4 * NPAD;
  const int arow = 16 * pd.In + c_col - pd.nb;  // padding-row offset of this lane in tile In
  const bool apad = arow >= 0 && arow < 4, aodd = arow & 1;
  // E columns: B = D V with V[(k', s)][(k, l)] = delta(k', k) F_mu[l][s] in place of G
  G8 cur, nxt;
  load_g8<T, false>(cur, Gb, qa, 0, qa, qb, k_row, c_col);
  for (int qs = qa; qs < qb; qs += 8) {
    float D[2][16], Fm[2][4];
    double Wv[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int ql = qs + 2 * k_row + h;
      const bool live = ql < qb;
      const double* rq = sQ + (live ? ql : qa) * QS;
      const float* rf = reinterpret_cast<const float*>(rq + R_D);
#pragma unroll
      for (int k = 0; k < 16; ++k) D[h][k] = live ? rf[k] : 0.0f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Fm[h][k] = live ? (float)rq[R_FM + k] : 0.0f;
        Wv[h][k] = live ? rq[R_W + k] : 0.0;
      }
    }
    bf8 Aop[T];
    int u = 0;
#pragma unroll
    for (int J = 0; J < T; ++J) {
      if (J + 1 < T)
        load_g8<T, false>(nxt, Gb, qs, J + 1, qa, qb, k_row, c_col);
      else
        load_g8<T, false>(nxt, Gb, min(qs + 8, qb - 1), 0, qa, qb, k_row, c_col);
      const int col = 16 * J + c_col, dc = col - pd.nb;
      const bool ecol = dc >= 1 && dc <= 4, wcol = dc == 0;
      const int ek = (dc - 1) >> 1, el = (dc - 1) & 1;
      // f partials of every lane (those of the columns n and above are never read)
      if (do_f) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int b = 0; b < 4; ++b) fpart[J] = fma(cur.g[h][b], Wv[h][b], fpart[J]);
      }
      bf8 Bop;
      if (J < T - 1) {
        // tiles left of the padding block (resolved at compile time): G in
        // both operands, the same arithmetic as below without the selects
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          float g[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) g[c] = (float)cur.g[h][c];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const float hv = D[h][4 * b] * g[0] + D[h][4 * b + 1] * g[1] + D[h][4 * b + 2] * g[2] + D[h][4 * b + 3] * g[3];
            Aop[J][4 * h + b] = (__bf16)g[b];
            Bop[4 * h + b] = (__bf16)hv;
          }
        }
      } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          float g[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) g[c] = (float)cur.g[h][c];
          float gb[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            // V[c][(ek, el)] for c = (k', s): F_mu[el][s] when k' = ek
            const float fv = el ? Fm[h][2 + (c & 1)] : Fm[h][c & 1];
            gb[c] = ecol ? (((c >> 1) == ek) ? fv : 0.0f) : g[c];
          }
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            float av = g[b];
            if (apad)  // this branch is the last tile, the tile row of the padding block
              av = ((arow >> 1) == (b >> 1)) ? (aodd ? Fm[h][2 + (b & 1)] : Fm[h][b & 1]) : 0.0f;
            float hv = D[h][4 * b] * gb[0] + D[h][4 * b + 1] * gb[1] + D[h][4 * b + 2] * gb[2] + D[h][4 * b + 3] * gb[3];
            if (wcol) hv = (float)Wv[h][b];
            Aop[J][4 * h + b] = (__bf16)av;
            Bop[4 * h + b] = (__bf16)hv;
          }
        }
      }
      if (owns<T, W, TW>(J)) {
#pragma unroll
        for (int I = 0; I <= J; ++I) {
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop[I], Bop, acc[u], 0, 0, 0);
          ++u;
        }
      }
      cur = nxt;
    }
  }
}


template <int T, int PREC, int W, int TW>
__device__ __forceinline__ void contract_any(typename Acc<PREC>::type* acc, double (&fpart)[T], bool do_f,
                                             const double* __restrict__ Gq, const double* sQ, int q0, int qa, int qb,
                                             const Pad& pd, int n, int k_row, int c_col) {
  if constexpr (PREC == PREC_BF16 && T <= 4)
    contract_range_bf16_mfma<T, W, TW>(acc, fpart, do_f, Gq, sQ, q0, qa, qb, pd, n, k_row, c_col);
  else if constexpr (PREC == PREC_BF16)
    contract_range_bf16_valu<T, W, TW>(acc, fpart, do_f, Gq, sQ, q0, qa, qb, pd, n, k_row, c_col);
  else
    contract_range<T, PREC, W, TW>(acc, fpart, do_f, Gq, sQ, q0, qa, qb, pd, n, k_row, c_col);
}

// Store (ACCUM: add) the tiles of wave W into sK (ld LD); when MIRROR, also
// the transposed tile below the diagonal.
template <int T, int PREC, int W, int TW>
__device__ __forceinline__ void store_acc(const typename Acc<PREC>::type* acc, double* sK, bool accum, bool mirror,
                                          int n, int k_row, int c_col) {
  constexpr int LD = ldk<T>();
  int u = 0;
#pragma unroll
  for (int J = 0; J < T; ++J) {
#pragma unroll
    for (int I = 0; I <= J; ++I) {
      if (owns<T, W, TW>(J)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // output layouts: FP64 row = k_row + 4 j, FP32 accumulators row = 4 k_row + j
          const int row = 16 * I + (PREC == PREC_F64 ? k_row + 4 * j : 4 * k_row + j), col = 16 * J + c_col;
          // K is kept exactly symmetric: in the diagonal tiles its entries
          // below the diagonal are the mirror of those above (the padding rows
          // and columns are not symmetric quantities and stay as computed)
          const bool upper_k = row < col && col < n;
          if (I == J && row > col && row < n) continue;
          double x = (double)acc[u][j];
          if (accum) x += sK[row * LD + col];
          sK[row * LD + col] = x;
          if (mirror && (I < J || upper_k)) sK[col * LD + row] = x;
        }
        ++u;
      }
    }
  }
}

// Unsigned maximum over the 64 lanes of a wave with DPP moves (quad
// permutations, row mirrors, row broadcasts); returned uniform.
__device__ __forceinline__ unsigned int wave_max_u32(unsigned int v) {
  v = max(v, (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = max(v, (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = max(v, (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
  v = max(v, (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast15
  v = max(v, (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast31
  return (unsigned int)__builtin_amdgcn_readlane((int)v, 63);
}

// Pivot key of a candidate row: the upper 32 bits of |v| (sign, exponent and
// 20 mantissa bits, monotone in |v|) plus one, so that every candidate beats
// the rows that are not candidates (key 0).  Candidates within a relative
// 2^-20 of the largest count as ties and the lowest row index wins, which
// keeps the choice of partial pivoting (a pivot of maximal magnitude up to
// that factor).
__device__ __forceinline__ unsigned int pivot_key(double v, bool cand) {
  const unsigned int hi = (unsigned int)((unsigned long long)__double_as_longlong(v) >> 32) & 0x7fffffffu;
  return cand ? hi + 1u : 0u;
}

// Gauss-Jordan elimination with partial pivoting of the n x (n + 5) system
// [K | f | C] in sK (ld LD): lane l of wave w holds rows l (and l + 64) in the
// columns j = w + 4 c.  Step k: the wave owning column k picks the pivot row
// (largest |a[r][k]| among the rows not yet pivots) and publishes it with the
// multipliers a[r][k] / a[pr][k] of all other rows; every wave then
// eliminates column k from those rows with the unscaled pivot row (pivot rows
// stay unscaled and are divided by their pivot at the end).  One barrier per
// step.  On return sK[ord[k]][pad_base(n) + y] holds unknown k of right-hand side y
// (y = 0: f, 1..4: C) with ord[k] = sOrd[k].
template <int T>
__device__ void gauss_jordan(double* sK, int n, double* sL, double* sPv, int* sOrd, int* sPiv) {
  constexpr int NPAD = 16 * T, LD = ldk<T>();
  constexpr int ROWS = NPAD > 64 ? 2 : 1, COLS = NPAD / 4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ncol = pad_base(n) + 5;  // K, zero columns up to the padding base, then [f | C]
  double a[ROWS][COLS];
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = min(lane + 64 * s, NPAD - 1);
#pragma unroll
    for (int c = 0; c < COLS; ++c) a[s][c] = sK[r * LD + wave + 4 * c];
  }
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = lane + 64 * s;
#pragma unroll
    for (int c = 0; c < COLS; ++c)
      if (r >= n || wave + 4 * c >= ncol) a[s][c] = 0.0;
  }
  unsigned int pivmask = 0;  // bit s: row lane + 64 s is already a pivot
  for (int k = 0; k < n; ++k) {
    const int ow = k & 3, oc = k >> 2;
    double* L = sL + (k & 1) * 128;
    if (wave == ow) {
      double v[ROWS];
      unsigned int key[ROWS];
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        v[s] = a[s][0];
#pragma unroll
        for (int c = 1; c < COLS; ++c) v[s] = (c == oc) ? a[s][c] : v[s];
        const int r = lane + 64 * s;
        key[s] = pivot_key(v[s], r < n && !((pivmask >> s) & 1u));
      }
      unsigned int kmax = key[0];
      if constexpr (ROWS == 2) kmax = max(kmax, key[1]);
      const unsigned int M = wave_max_u32(kmax);
      const unsigned long long b0 = __ballot(key[0] == M);
      int pr;
      if (b0) {
        pr = __builtin_ctzll(b0);
      } else {
        const unsigned long long b1 = __ballot(ROWS == 2 && key[ROWS - 1] == M);
        pr = 64 + __builtin_ctzll(b1);
      }
      // multipliers of every row but the pivot row (the pivot is uniform:
      // read from its lane)
      double pv = readlane_d(v[0], pr & 63);
      if constexpr (ROWS == 2) pv = (pr >> 6) ? readlane_d(v[ROWS - 1], pr & 63) : pv;
      const double inv = 1.0 / pv;
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        const bool is_p = (lane + 64 * s == pr);
        L[lane + 64 * s] = is_p ? 0.0 : v[s] * inv;
      }
      if (lane == 0) sPv[pr] = pv;
      if (lane == 0) {
        sPiv[k & 1] = pr;
        sOrd[k] = pr;
      }
    }
    __syncthreads();
    double mlt[ROWS];
#pragma unroll
    for (int s = 0; s < ROWS; ++s) mlt[s] = L[lane + 64 * s];
    const int pr = __builtin_amdgcn_readfirstlane(sPiv[k & 1]);
    const int pl = pr & 63, ps = pr >> 6;
    double prow[COLS];
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
      double src = a[0][c];
      if constexpr (ROWS == 2) src = ps ? a[1][c] : a[0][c];
      prow[c] = readlane_d(src, pl);
    }
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
#pragma unroll
      for (int c = 0; c < COLS; ++c) a[s][c] = fma(-mlt[s], prow[c], a[s][c]);
      if (lane + 64 * s == pr) pivmask |= 1u << s;
    }
  }
  // the right-hand-side columns, divided by the pivots, back to LDS
#pragma unroll
  for (int s = 0; s < ROWS; ++s) {
    const int r = lane + 64 * s;
    const double rinv = (r < n) ? 1.0 / sPv[r] : 0.0;
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
      const int j = wave + 4 * c;
      if (r < n && j >= n && j < ncol) sK[r * LD + j] = a[s][c] * rinv;
    }
  }
  __syncthreads();
}

// Two FP32 values in one record slot (the BF16 form keeps D in FP32): the
// first in the low half, as in an FP32 array over the slots.
__device__ __forceinline__ double pack_f32x2(float lo, float hi) {
  const unsigned long long u =
      ((unsigned long long)__float_as_uint(hi) << 32) | (unsigned long long)__float_as_uint(lo);
  return __longlong_as_double((long long)u);
}

// Return map and tangent (Appendix A) of ECM point q at the deformation
// gradient F: P, the trial history (to ht, point fastest), and
//   D = w|J| T^T A T (T: right multiplication by F_mu^-1), accumulated column
//     v = (k, l) of A at a time: E[.][v] = w|J| T^T A[.][v],
//     D[b][(k, s)] += E[b][(k, l)] F_mu^-1[s][l];
// Fi = F_mu^-1 and w = w|J| are returned with them.
__device__ __forceinline__ void point_material(const double F[4], int m, int q, const double* __restrict__ tmu,
                                               const double* __restrict__ hc, double* __restrict__ ht,
                                               const J2Params& mp, double D[16], double P[4], double Fi[4],
                                               double& w) {
#pragma unroll
  for (int k = 0; k < 4; ++k) Fi[k] = tmu[k * m + q];
  const double wl = tmu[4 * m + q];
  w = wl;
  const double Fp[4] = {hc[q], hc[m + q], hc[2 * m + q], hc[3 * m + q]};
  double Fpn[4], Fp33n, xin;
#pragma unroll
  for (int k = 0; k < 16; ++k) D[k] = 0.0;
  const double Fi0 = Fi[0], Fi1 = Fi[1], Fi2 = Fi[2], Fi3 = Fi[3];
  j2_point_cols<true>(F, Fp, hc[4 * m + q], hc[5 * m + q], mp, P, Fpn, Fp33n, xin,
                      [&](int v, double c0, double c1, double c2, double c3) {
                        const double e0 = wl * (Fi0 * c0 + Fi1 * c1);
                        const double e1 = wl * (Fi2 * c0 + Fi3 * c1);
                        const double e2 = wl * (Fi0 * c2 + Fi1 * c3);
                        const double e3 = wl * (Fi2 * c2 + Fi3 * c3);
                        const int k = v >> 1, l = v & 1;
                        const double t0 = l ? Fi1 : Fi0, t1 = l ? Fi3 : Fi2;
#pragma unroll
                        for (int s2 = 0; s2 < 2; ++s2) {
                          const double t = s2 ? t1 : t0;
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
}

// D of a contraction record at rec[k * rs] (rows R_D ..): FP64, or in the
// BF16 form FP32 values two per slot.
template <int PREC>
__device__ __forceinline__ void put_record_d(double* rec, int rs, const double D[16]) {
  if constexpr (PREC == PREC_BF16) {
#pragma unroll
    for (int j = 0; j < 8; ++j) rec[(R_D + j) * rs] = pack_f32x2((float)D[2 * j], (float)D[2 * j + 1]);
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) rec[(R_D + k) * rs] = D[k];
  }
}

// W = w|J| P F_mu^-T and F_mu (from the stored F_mu^-1) of an LDS record
// (explicit fma, see kin_F).
__device__ __forceinline__ void put_record_wf(double* rec, const double P[4], const double Fi[4], double w) {
  rec[R_W] = w * fma(P[1], Fi[1], P[0] * Fi[0]);
  rec[R_W + 1] = w * fma(P[1], Fi[3], P[0] * Fi[2]);
  rec[R_W + 2] = w * fma(P[3], Fi[1], P[2] * Fi[0]);
  rec[R_W + 3] = w * fma(P[3], Fi[3], P[2] * Fi[2]);
  const double idet = 1.0 / fma(Fi[0], Fi[3], -(Fi[1] * Fi[2]));
  rec[R_FM] = Fi[3] * idet;
  rec[R_FM + 1] = -Fi[1] * idet;
  rec[R_FM + 2] = -Fi[2] * idet;
  rec[R_FM + 3] = Fi[0] * idet;
}

// Rows of the phased form's point-fastest records in global memory: D (16
// rows, 8 in the BF16 form) then P (4); W and F_mu are formed again when the
// records are staged for the contraction.
template <int PREC>
constexpr int rec_p_row() {
  return PREC == PREC_BF16 ? 8 : 16;
}

// Accumulators of one evaluation: the MFMA tiles of this wave, and in the
// reduced-precision forms the FP64 residual partials and sum w|J| P.
template <int T, int PREC, int SPLIT>
struct EvalAcc {
  static constexpr int NACC = (SPLIT == 0) ? T * (T + 1) / 2 : split_tiles<T>();
  typename Acc<PREC>::type acc[NACC];
  double fpart[T];
  double accP[4];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int t = 0; t < NACC; ++t) acc[t] = (typename Acc<PREC>::type){0, 0, 0, 0};
#pragma unroll
    for (int J = 0; J < T; ++J) fpart[J] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) accP[k] = 0.0;
  }
};

// Contraction of the records sQ of chunk [q0, q0 + qend): SPLIT 0 the waves
// take a quarter of the points each, SPLIT 1 every wave takes all points for
// its column tiles.
template <int T, int PREC, int SPLIT>
__device__ __forceinline__ void contract_chunk(EvalAcc<T, PREC, SPLIT>& E, const double* __restrict__ Gq,
                                               const double* sQ, int q0, int qend, const Pad& pd, int n, int wave,
                                               int k_row, int c_col) {
  if constexpr (SPLIT == 0) {
    const int qa = (wave * qend) >> 2, qb = ((wave + 1) * qend) >> 2;
    contract_any<T, PREC, 0, 1>(E.acc, E.fpart, true, Gq, sQ, q0, qa, qb, pd, n, k_row, c_col);
  } else {
    switch (wave) {
      case 0: contract_any<T, PREC, 0, 4>(E.acc, E.fpart, true, Gq, sQ, q0, 0, qend, pd, n, k_row, c_col); break;
      case 1: contract_any<T, PREC, 1, 4>(E.acc, E.fpart, false, Gq, sQ, q0, 0, qend, pd, n, k_row, c_col); break;
      case 2: contract_any<T, PREC, 2, 4>(E.acc, E.fpart, false, Gq, sQ, q0, 0, qend, pd, n, k_row, c_col); break;
      default: contract_any<T, PREC, 3, 4>(E.acc, E.fpart, false, Gq, sQ, q0, 0, qend, pd, n, k_row, c_col); break;
    }
  }
}

// [K | f | C] and the padding rows into LDS (K's lower part by symmetry; in
// the reduced-precision forms f and sum w|J| P from the FP64 partials, over
// the lane groups and the waves in a fixed order), C of the evaluation to sC
// (kept for Abar); returns ||f||_2, the same on every lane.
template <int T, int PREC, int SPLIT>
__device__ __forceinline__ double assemble(const EvalAcc<T, PREC, SPLIT>& E, double* sK, double* sC, double* sX,
                                           int n, int tid, int lane, int wave, int k_row, int c_col) {
  constexpr int NPAD = 16 * T, LD = ldk<T>();
  const int nb = pad_base(n);
  if constexpr (SPLIT == 0) {
    for (int w = 0; w < 4; ++w) {
      if (wave == w) store_acc<T, PREC, 0, 1>(E.acc, sK, w > 0, w == 3, n, k_row, c_col);
      __syncthreads();
    }
  } else {
    switch (wave) {
      case 0: store_acc<T, PREC, 0, 4>(E.acc, sK, false, true, n, k_row, c_col); break;
      case 1: store_acc<T, PREC, 1, 4>(E.acc, sK, false, true, n, k_row, c_col); break;
      case 2: store_acc<T, PREC, 2, 4>(E.acc, sK, false, true, n, k_row, c_col); break;
      default: store_acc<T, PREC, 3, 4>(E.acc, sK, false, true, n, k_row, c_col); break;
    }
    __syncthreads();
  }
  if constexpr (PREC != PREC_F64) {
    double* sFp = sC;  // [4][NPAD] wave partials of f, before C is copied
#pragma unroll
    for (int J = 0; J < T; ++J) {
      double v = E.fpart[J];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (k_row == 0) sFp[wave * NPAD + 16 * J + c_col] = v;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double v = E.accP[k];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) sX[4 * k + wave] = v;
    }
    __syncthreads();
    if (tid < n) {
      const double v = (SPLIT == 0) ? ((sFp[tid] + sFp[NPAD + tid]) + sFp[2 * NPAD + tid]) + sFp[3 * NPAD + tid]
                                    : sFp[tid];
      sK[tid * LD + nb] = v;
    }
    if (tid < 4) sK[(nb + tid) * LD + nb] = ((sX[4 * tid] + sX[4 * tid + 1]) + sX[4 * tid + 2]) + sX[4 * tid + 3];
    __syncthreads();
  }
  for (int idx = tid; idx < 4 * n; idx += 256) sC[idx] = sK[(idx >> 2) * LD + nb + 1 + (idx & 3)];
  double part = 0.0;
  if (tid < n) {
    const double fv = sK[tid * LD + nb];
    part = fv * fv;
  }
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
  if (lane == 0) sX[wave] = part;
  __syncthreads();
  return sqrt(sX[0] + sX[1] + sX[2] + sX[3]);
}

// Status of evaluation it (0-based) of an attempt with residual norm rn;
// returns whether the attempt stops here.
__device__ __forceinline__ bool eval_status(const FusedArgs& a, int it, double rn, int& status) {
  const bool last = (it == a.max_iter - 1);
  if (!isfinite(rn)) {
    status = ROM_ST_NONFINITE;
    return true;
  }
  if (a.fixed) {
    status = (rn <= a.tol) ? ROM_ST_CONVERGED : ROM_ST_MAXITER;
    return last;
  }
  if (rn <= a.tol) {
    status = ROM_ST_CONVERGED;
    return true;
  }
  status = ROM_ST_MAXITER;
  return last;
}

// Effective quantities at the returned state (after the elimination of the
// evaluation): Pbar = sum w|J| P, Abar = sum w|J| A - C^T K*^-1 C, per unit
// cell area (Sec. 3.3); K*^-1 C itself to the state.
template <int T>
__device__ __forceinline__ void write_effective(const FusedArgs& a, int p, const double* sK, const double* sC,
                                                const int* sOrd, int n, int tid) {
  constexpr int LD = ldk<T>();
  const int nb = pad_base(n);
  if (tid < 20) {
    const double inv_area = a.inv_area;
    if (tid < 4) {
      a.Pbar[4 * (size_t)p + tid] = sK[(nb + tid) * LD + nb] * inv_area;
    } else {
      const int e = tid - 4, x = e >> 2, y = e & 3;
      double acc2 = sK[(nb + x) * LD + nb + 1 + y];
      for (int i = 0; i < n; ++i) acc2 = fma(-sC[4 * i + x], sK[sOrd[i] * LD + nb + 1 + y], acc2);
      a.Abar[16 * (size_t)p + e] = acc2 * inv_area;
    }
  }
  // K*^-1 C, kept for the shape sensitivities of the returned state
  for (int idx = tid; idx < 4 * n; idx += 256)
    a.zk[(size_t)p * 4 * n + idx] = sK[sOrd[idx >> 2] * LD + nb + 1 + (idx & 3)];
  __syncthreads();
}

// Outputs of a finished load step, and the commit of a converged one (r,
// history and the Fbar reached).
__device__ __forceinline__ void finish_point(const FusedArgs& a, int p, const double* sR, const double Fb[4],
                                             int status, bool fell_back, int iters, double rn, unsigned int sub,
                                             int tid) {
  const int n = a.n, m = a.m;
  if (!a.refine) {
    for (int i = tid; i < n; i += 256) a.rt[(size_t)p * n + i] = sR[i];
    if (tid == 0) {
      a.st_out[p] = (status == ROM_ST_CONVERGED && fell_back) ? ROM_ST_FALLBACK : status;
      a.it_out[p] = iters;
      a.res_out[p] = rn;
      a.sub[p] = sub;
    }
  }
  // a refining launch commits every point it evaluates: the step judged them converged
  if (a.commit && (a.refine || (!a.defer && status == ROM_ST_CONVERGED))) {
    if (tid < 4) a.fbc[4 * (size_t)p + tid] = Fb[tid];
    for (int i = tid; i < n; i += 256) a.rc[(size_t)p * n + i] = sR[i];
    double* hcw = a.hc + (size_t)p * 6 * m;
    const double* ht = a.ht + (size_t)p * 6 * m;
    for (int q = tid; q < m; q += 256)
#pragma unroll
      for (int k = 0; k < 6; ++k) hcw[k * m + q] = ht[k * m + q];
  }
}

// NaN outputs of a point whose shape parameters were rejected.
__device__ __forceinline__ void bad_mu_outputs(const FusedArgs& a, int p, int tid) {
  if (tid < 4) a.Pbar[4 * (size_t)p + tid] = __builtin_nan("");
  if (tid < 16) a.Abar[16 * (size_t)p + tid] = __builtin_nan("");
  if (tid == 0) {
    a.st_out[p] = ROM_ST_BADMU;
    a.it_out[p] = 0;
    a.res_out[p] = __builtin_nan("");
    a.sub[p] = 0u;
  }
}

// LDS of the fused and phased contraction kernels (computed in each kernel:
// pointers returned in a struct upset the instruction selection of the
// compiler for some tile counts):
//   sQ [FCH or CCH][QS] chunk records, shared with sK [NPAD][LD] [K | f | C] (after
//   the contraction); then sR [NPAD] current r, sC [NPAD][4] C of the
//   evaluation, sL [2][128] pivot columns of the elimination, sPv [128] pivot
//   value of each row, sX [32] reductions and the load-step ends, sOrd [NPAD]
//   pivot row of each step, sPiv [2] pivot exchange.
#define ROM_SOLVE_LDS(T, smem, MAT)                             \
  double* sQ = (smem);                                          \
  double* sK = (smem);                                          \
  double* sR = (smem) + (MAT);                                  \
  double* sC = sR + 16 * (T);                                   \
  double* sL = sC + 4 * 16 * (T);                               \
  double* sPv = sL + 256;                                       \
  double* sX = sPv + 128;                                       \
  int* sOrd = reinterpret_cast<int*>(sX + 32);                  \
  int* sPiv = sOrd + 16 * (T);

// The whole load step of macro point p on one workgroup.  SPLIT 0: the four
// waves split the ECM points of a chunk; SPLIT 1: they split the tiles.  With
// a.resume the point starts at evaluation phi[0] of attempt 0 from the trial
// r in rt (the state left by the phased launches; phi[0] = 0: from the start).
template <int T, int PREC, int SPLIT>
__device__ void solve_point(const FusedArgs& a, const int p, double* smem) {
  constexpr int NPAD = 16 * T;
  constexpr int LD = ldk<T>();
  ROM_SOLVE_LDS(T, smem, main_doubles<T>())

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = a.n, m = a.m;
  if (a.active && !a.active[p]) return;  // skipped: state and outputs untouched
  if (a.refine) {
    const int s0 = a.st_out[p];
    if (s0 != ROM_ST_CONVERGED && s0 != ROM_ST_FALLBACK) return;
  }
  if (!a.muok[p]) {
    bad_mu_outputs(a, p, tid);
    return;
  }
  int it0 = 0;
  bool fell_back = false;
  double rn = 0.0, rn0 = 0.0;
  if (a.resume) {
    // per-point values, the same on every lane
    it0 = __builtin_amdgcn_readfirstlane(a.phi[2 * (size_t)p]);
    fell_back = __builtin_amdgcn_readfirstlane(a.phi[2 * (size_t)p + 1]) != 0;
    rn0 = a.phd[2 * (size_t)p];
  }
  // initial guess: the committed r, plus the predicted increment with a warm
  // start (resumed: the trial r reached)
  for (int i = tid; i < NPAD; i += 256) {
    double v = 0.0;
    if (i < n) {
      if (it0 > 0 || a.refine) {
        v = a.rt[(size_t)p * n + i];
      } else {
        v = a.rc[(size_t)p * n + i];
        if (a.dr) v += (double)a.dr[(size_t)p * n + i];
        a.rg[(size_t)p * n + i] = v;
      }
    }
    sR[i] = v;
  }
  double Fb[4] = {a.Fbar[4 * (size_t)p], a.Fbar[4 * (size_t)p + 1], a.Fbar[4 * (size_t)p + 2],
                  a.Fbar[4 * (size_t)p + 3]};
  // load-step cutting: targets F0 + (t / 2^D) (Fbar - F0) on the segment from
  // the committed F0; sF0 / sF1 hold the two ends
  double* sF0 = sX + 16;
  double* sF1 = sX + 20;
  if (tid < 4) {
    sF0[tid] = a.fbc[4 * (size_t)p + tid];
    sF1[tid] = Fb[tid];
  }
  const int full = 1 << a.max_sub;
  int t_done = 0, stride = full, total = 0;
  unsigned int sub = 0u;  // end points of the converged sub-steps
  const double* tmu = a.tmu + (size_t)p * 5 * m;
  const double* hc = a.hc + (size_t)p * 6 * m;
  double* ht = a.ht + (size_t)p * 6 * m;
  const int k_row = lane >> 4, c_col = lane & 15;
  const Pad pd = make_pad(n, k_row, c_col);
  __syncthreads();

  int status = ROM_ST_MAXITER, iters = 0;
  for (int attempt = 0;; ++attempt) {
    for (int it = (attempt == 0) ? it0 : 0; it < a.max_iter; ++it) {
      EvalAcc<T, PREC, SPLIT> E;
      E.zero();
      for (int q0 = 0; q0 < m; q0 += FCH) {
        const int q = q0 + tid;
        if (q < m) {
          double F[4], D[16], P[4], Fi[4], wJ;
#pragma unroll
          for (int k = 0; k < 4; ++k) Fi[k] = tmu[k * m + q];
          kinematics(n, m, q, a.Gt, sR, Fb, Fi, F);
          point_material(F, m, q, tmu, hc, ht, point_params(a.mp, a.mp2, a.phase, q), D, P, Fi, wJ);
          put_record_d<PREC>(sQ + tid * QS, 1, D);
          put_record_wf(sQ + tid * QS, P, Fi, wJ);
          if constexpr (PREC != PREC_F64) {
#pragma unroll
            for (int k = 0; k < 4; ++k) E.accP[k] = fma(wJ, P[k], E.accP[k]);
          }
        }
        __syncthreads();
        // contraction in chunks of CCH points, as the phased kernel makes it
        const int qend = min(FCH, m - q0);
        for (int c0 = 0; c0 < qend; c0 += CCH)
          contract_chunk<T, PREC, SPLIT>(E, a.Gq, sQ + c0 * QS, q0 + c0, min(CCH, qend - c0), pd, n, wave, k_row,
                                         c_col);
        __syncthreads();
      }
      rn = assemble<T, PREC, SPLIT>(E, sK, sC, sX, n, tid, lane, wave, k_row, c_col);
      iters = it + 1;
      bool stop = eval_status(a, it, rn, status);
      if (it == 0) rn0 = rn;
      // warm start judged by plain Newton: no tenfold drop of ||f|| after two
      // updates -> restart from the committed r
      if (!stop && a.dr && attempt == 0 && !fell_back && it == 2 && !(rn <= 0.1 * rn0)) {
        fell_back = true;
        for (int i = tid; i < n; i += 256) sR[i] = a.rc[(size_t)p * n + i];
        __syncthreads();
        continue;
      }
      // K x = [f | C]: the Newton update and K^-1 C
      gauss_jordan<T>(sK, n, sL, sPv, sOrd, sPiv);
      if (stop) {
        write_effective<T>(a, p, sK, sC, sOrd, n, tid);
        break;
      }
      if (tid < n) sR[tid] -= sK[sOrd[tid] * LD + pad_base(n)];
      __syncthreads();
    }
    total += iters;
    if (status == ROM_ST_CONVERGED) {
      t_done += stride;
      sub |= substep_bit(t_done, a.max_sub);
      if (t_done == full) break;
      // a converged sub-step becomes the committed start of the next attempt
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
  finish_point(a, p, sR, Fb, status, fell_back, total, rn, sub, tid);
}

// Phased form, contraction launch: one evaluation of each listed point from
// the records of the material launch (same chunks and order as the fused
// kernel, so the two forms agree bit for bit), then the elimination and the
// Newton / status logic of attempt 0.  A point that stops is finished here;
// one that goes on is listed for the next phased evaluation, or after ph_k
// evaluations for the fused kernel; an attempt that fails with load-step
// cutting on is handed to the fused kernel from its start.
// waves per SIMD the contraction kernel is compiled for, up to three column
// tiles: four for FP64 (measured 4% faster than three at n = 40), three for
// BF16 (7% faster than the compiler's two, with the record loads not
// prefetched); the compiler's choice otherwise
template <int T, int PREC>
constexpr int cs_waves() {
  return (T <= 3 && PREC == PREC_F64) ? 4 : ((T <= 3 && PREC == PREC_BF16) ? 3 : 1);
}

template <int T, int PREC, int SPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(cs_waves<T, PREC>()))) void k_ph_cs(
    const FusedArgs a) {
  extern __shared__ double smem[];
  constexpr int NPAD = 16 * T;
  constexpr int LD = ldk<T>();
  const int idx = blockIdx.x;
  if (idx >= *a.cin) return;
  const int p = a.lin[idx];
  ROM_SOLVE_LDS(T, smem, cs_main_doubles<T>())
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = a.n, m = a.m;
  for (int i = tid; i < NPAD; i += 256) sR[i] = (i < n) ? a.rt[(size_t)p * n + i] : 0.0;
  const int it = __builtin_amdgcn_readfirstlane(a.phi[2 * (size_t)p]);
  bool fell_back = __builtin_amdgcn_readfirstlane(a.phi[2 * (size_t)p + 1]) != 0;
  double rn0 = a.phd[2 * (size_t)p];
  const double rn_prev = a.phd[2 * (size_t)p + 1];
  const double* rec = a.rec + (size_t)p * ROM_REC_ROWS * m;
  const int k_row = lane >> 4, c_col = lane & 15;
  const Pad pd = make_pad(n, k_row, c_col);

  EvalAcc<T, PREC, SPLIT> E;
  E.zero();
  const double* tmu = a.tmu + (size_t)p * 5 * m;
  constexpr int RP = rec_p_row<PREC>();
  if constexpr (PREC != PREC_F64) {
    // FP64 sum of w|J| P, lane tid over the points q = tid mod FCH (the fused kernel's order)
    for (int q = tid; q < m; q += FCH) {
      const double wJ = tmu[4 * m + q];
#pragma unroll
      for (int k = 0; k < 4; ++k) E.accP[k] = fma(wJ, rec[(size_t)(RP + k) * m + q], E.accP[k]);
    }
  }
  // records of a chunk into LDS, two lanes per point: D (the first eight rows),
  // and the rest of D with W and F_mu formed from P and F_mu^-1
  const int j = tid & (CCH - 1), kh = tid / CCH;
  constexpr int DR = (PREC == PREC_BF16) ? 1 : 2;  // record rows of D in halves of eight
  if constexpr (PREC != PREC_F32 || T > 4) {
    for (int q0 = 0; q0 < m; q0 += CCH) {
      const int qend = min(CCH, m - q0), q = q0 + j;
      if (j < qend) {
        double* dst = sQ + j * QS;
        double v[8];
        if (DR == 2 || kh == 0) {
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = rec[(size_t)(8 * kh + k) * m + q];
        }
        if (kh == 1) {
          double P[4], Fi[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) P[k] = rec[(size_t)(RP + k) * m + q];
#pragma unroll
          for (int k = 0; k < 4; ++k) Fi[k] = tmu[k * m + q];
          const double w = tmu[4 * m + q];
          put_record_wf(dst, P, Fi, w);
        }
        if (DR == 2 || kh == 0) {
#pragma unroll
          for (int k = 0; k < 8; ++k) dst[R_D + 8 * kh + k] = v[k];
        }
      }
      __syncthreads();
      contract_chunk<T, PREC, SPLIT>(E, a.Gq, sQ, q0, qend, pd, n, wave, k_row, c_col);
      __syncthreads();
    }
  } else {
    // FP32 up to four column tiles: the global loads of the next chunk are
    // issued before the current chunk is contracted (the FP64, BF16 and wider
    // contractions are faster with these registers for themselves)
    double v[8], Pv[4], Fv[4], wv = 0.0;
    auto load_chunk = [&](int q0) {
      const int q = q0 + j;
      if (q < m) {
        if (DR == 2 || kh == 0) {
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = rec[(size_t)(8 * kh + k) * m + q];
        }
        if (kh == 1) {
#pragma unroll
          for (int k = 0; k < 4; ++k) Pv[k] = rec[(size_t)(RP + k) * m + q];
#pragma unroll
          for (int k = 0; k < 4; ++k) Fv[k] = tmu[k * m + q];
          wv = tmu[4 * m + q];
        }
      }
    };
    load_chunk(0);
    for (int q0 = 0; q0 < m; q0 += CCH) {
      const int qend = min(CCH, m - q0);
      if (j < qend) {
        double* dst = sQ + j * QS;
        if (DR == 2 || kh == 0) {
#pragma unroll
          for (int k = 0; k < 8; ++k) dst[R_D + 8 * kh + k] = v[k];
        }
        if (kh == 1) put_record_wf(dst, Pv, Fv, wv);
      }
      __syncthreads();
      load_chunk(q0 + CCH);
      contract_chunk<T, PREC, SPLIT>(E, a.Gq, sQ, q0, qend, pd, n, wave, k_row, c_col);
      __syncthreads();
    }
  }
  const double rn = assemble<T, PREC, SPLIT>(E, sK, sC, sX, n, tid, lane, wave, k_row, c_col);
  if (a.refine) {
    // effective quantities of a point the step reported converged, at its
    // returned state, and the commit the step left to this launch
    gauss_jordan<T>(sK, n, sL, sPv, sOrd, sPiv);
    write_effective<T>(a, p, sK, sC, sOrd, n, tid);
    const double Fb[4] = {a.Fbar[4 * (size_t)p], a.Fbar[4 * (size_t)p + 1], a.Fbar[4 * (size_t)p + 2],
                          a.Fbar[4 * (size_t)p + 3]};
    finish_point(a, p, sR, Fb, ROM_ST_CONVERGED, false, 0, rn, 0u, tid);
    return;
  }
  if (a.sys) {
    // the elimination and what follows run in the solve launch: the system
    // by columns of n rows, then the effective-quantity rows and ||f||
    double* sy = a.sys + (size_t)p * rom_sys_stride(NPAD, n);
    const int nb = pad_base(n), ncol = nb + 5;
    for (int e = tid; e < ncol * n; e += 256) {
      const int c = e / n, r = e - c * n;
      sy[e] = sK[r * LD + c];
    }
    double* ex = sy + (size_t)NPAD * n;
    if (tid < 4) ex[tid] = sK[(nb + tid) * LD + nb];
    else if (tid < 20) ex[tid] = sK[(nb + ((tid - 4) >> 2)) * LD + nb + 1 + ((tid - 4) & 3)];
    else if (tid == 20) ex[20] = rn;
    return;
  }
  int status;
  const bool stop = eval_status(a, it, rn, status);
  if (it == 0) rn0 = rn;
  int next = it + 1;
  if (!stop && a.dr && !fell_back && it == 2 && !(rn <= 0.1 * rn0)) {
    // the warm start is dropped: the next evaluation starts from the committed r
    fell_back = true;
    for (int i = tid; i < n; i += 256) a.rt[(size_t)p * n + i] = a.rc[(size_t)p * n + i];
  } else {
    gauss_jordan<T>(sK, n, sL, sPv, sOrd, sPiv);
    if (stop) {
      if (status == ROM_ST_CONVERGED || a.max_sub == 0) {
        write_effective<T>(a, p, sK, sC, sOrd, n, tid);
        const double Fb[4] = {a.Fbar[4 * (size_t)p], a.Fbar[4 * (size_t)p + 1], a.Fbar[4 * (size_t)p + 2],
                              a.Fbar[4 * (size_t)p + 3]};
        finish_point(a, p, sR, Fb, status, fell_back, it + 1, rn, status == ROM_ST_CONVERGED ? (1u << 31) : 0u,
                     tid);
        return;
      }
      next = 0;  // failed attempt: the fused kernel redoes the point with load-step cutting
      fell_back = false;
    } else {
      for (int i = tid; i < n; i += 256) a.rt[(size_t)p * n + i] = sR[i] - sK[sOrd[i] * LD + pad_base(n)];
    }
  }
  if (tid == 0) {
    a.phi[2 * (size_t)p] = next;
    a.phi[2 * (size_t)p + 1] = fell_back ? 1 : 0;
    a.phd[2 * (size_t)p] = rn0;
    a.phd[2 * (size_t)p + 1] = rn;
    // a point converging slowly at the early hand-over goes to the side stream
    const bool slow = a.ph_early > 0 && next == a.ph_early && it > 0 && !(rn <= a.ph_slow * rn_prev);
    if (next > 0 && next < a.ph_k && !slow)
      a.lout[atomicAdd(a.cout, 1)] = p;
    else if (slow)
      a.early[atomicAdd(a.cearly, 1)] = p;
    else
      a.hand[atomicAdd(a.chand, 1)] = p;
  }
}

// Step K of the one-wave elimination of the solve launch (K a constant): the
// lane's row in registers with the right-hand sides in x[0 .. 4] and column j
// of K in x[5 + j]; pivot row, multipliers and fma per entry as in
// gauss_jordan(); columns left of the pivot column are not updated (no later
// step and no right-hand side reads them).
template <int NPAD, int K>
__device__ __forceinline__ void solve_step(double (&x)[NPAD], int n, int lane, bool& piv, int& kp, double& pvr) {
  if (K >= n) return;
  const unsigned int key = pivot_key(x[5 + K], lane < n && !piv);
  const unsigned int M = wave_max_u32(key);
  const int pr = __builtin_ctzll(__ballot(key == M));
  const double pv = readlane_d(x[5 + K], pr);
  const double inv = 1.0 / pv;
  const double mlt = (lane == pr) ? 0.0 : x[5 + K] * inv;
  if (lane == pr) {
    piv = true;
    kp = K;
    pvr = pv;
  }
  // the pivot row's entries read from its lane into scalar registers
#pragma unroll
  for (int c = 0; c < NPAD; ++c)
    if (c < 5 || c > 5 + K) x[c] = fma(-mlt, readlane_d(x[c], pr), x[c]);
}

template <int NPAD, int... Ks>
__device__ __forceinline__ void solve_steps(std::integer_sequence<int, Ks...>, double (&x)[NPAD], int n, int lane,
                                            bool& piv, int& kp, double& pvr) {
  (solve_step<NPAD, Ks>(x, n, lane, piv, kp, pvr), ...);
}

// Phased form up to ROM_SOLVE_NPAD columns, solve launch: one wave per listed
// point takes the system [K | f | C] the contraction launch left in HBM and
// runs the elimination of gauss_jordan() -- the same pivot rows (same key,
// lowest row on ties), multipliers and fma per entry, so the same results bit
// for bit -- with the lane's row in registers and the steps unrolled, so that
// the pivot column is a fixed register in each; every lane reads the pivot
// row's entries from the pivot lane (scalar registers), and no workgroup
// barrier is taken.  Then the status, the
// Newton update or the effective quantities and the commit, and the lists,
// as the contraction kernel does them in place.
template <int T>
__global__ __launch_bounds__(256) void k_ph_s(const FusedArgs a) {
  constexpr int NPAD = 16 * T;
  static_assert(NPAD <= ROM_SOLVE_NPAD && NPAD <= 64, "one row per lane");
  __shared__ double sZ[4][64 * 4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int idx = blockIdx.x * 4 + wave;
  if (idx >= *a.cin) return;
  const int p = __builtin_amdgcn_readfirstlane(a.lin[idx]);
  const int n = a.n, nb = pad_base(n), ncol = nb + 5;
  const double* sy = a.sys + (size_t)p * rom_sys_stride(NPAD, n);
  const double* ex = sy + (size_t)NPAD * n;  // sum w|J| P (4), sum w|J| A (16), ||f||
  const double rn = ex[20];
  const int it = __builtin_amdgcn_readfirstlane(a.phi[2 * (size_t)p]);
  bool fell_back = __builtin_amdgcn_readfirstlane(a.phi[2 * (size_t)p + 1]) != 0;
  double rn0 = a.phd[2 * (size_t)p];
  const double rn_prev = a.phd[2 * (size_t)p + 1];
  double* rt = a.rt + (size_t)p * n;
  int status;
  const bool stop = eval_status(a, it, rn, status);
  if (it == 0) rn0 = rn;
  int next = it + 1;
  if (!stop && a.dr && !fell_back && it == 2 && !(rn <= 0.1 * rn0)) {
    // the warm start is dropped: the next evaluation starts from the committed r
    fell_back = true;
    for (int i = lane; i < n; i += 64) rt[i] = a.rc[(size_t)p * n + i];
  } else if (stop && !(status == ROM_ST_CONVERGED || a.max_sub == 0)) {
    next = 0;  // failed attempt: the fused kernel redoes the point with load-step cutting
    fell_back = false;
  } else {
    // registers: the right-hand sides (f, C) first, then the columns of K
    double x[NPAD];
#pragma unroll
    for (int y = 0; y < 5; ++y) x[y] = (lane < n) ? sy[(size_t)(nb + y) * n + lane] : 0.0;
#pragma unroll
    for (int c = 0; c + 5 < NPAD; ++c) x[5 + c] = (lane < n && c < n) ? sy[(size_t)c * n + lane] : 0.0;
    bool piv = false;
    int kp = 0;        // the step at which this lane's row was the pivot row
    double pvr = 1.0;  // and its pivot
    solve_steps<NPAD>(std::make_integer_sequence<int, NPAD - 5>{}, x, n, lane, piv, kp, pvr);
    // unknown kp of the right-hand sides y, divided by the row's pivot
    const double rinv = (lane < n) ? 1.0 / pvr : 0.0;
    double xs[5];
#pragma unroll
    for (int y = 0; y < 5; ++y) xs[y] = x[y] * rinv;
    if (!stop) {
      if (lane < n) rt[kp] = rt[kp] - xs[0];
    } else {
      // effective quantities at the returned state (Sec. 3.3), K*^-1 C kept
      if (lane < n) {
#pragma unroll
        for (int y = 0; y < 4; ++y) sZ[wave][4 * kp + y] = xs[1 + y];
      }
      __builtin_amdgcn_wave_barrier();
      const double inv_area = a.inv_area;
      if (lane < 4) {
        a.Pbar[4 * (size_t)p + lane] = ex[lane] * inv_area;
      } else if (lane < 20) {
        const int e = lane - 4, xx = e >> 2, yy = e & 3;
        double acc2 = ex[4 + e];
        for (int i = 0; i < n; ++i) acc2 = fma(-sy[(size_t)(nb + 1 + xx) * n + i], sZ[wave][4 * i + yy], acc2);
        a.Abar[16 * (size_t)p + e] = acc2 * inv_area;
      }
      for (int e = lane; e < 4 * n; e += 64) a.zk[(size_t)p * 4 * n + e] = sZ[wave][e];
      // outputs of the finished step and the commit of a converged one
      if (lane == 0) {
        a.st_out[p] = (status == ROM_ST_CONVERGED && fell_back) ? ROM_ST_FALLBACK : status;
        a.it_out[p] = it + 1;
        a.res_out[p] = rn;
        a.sub[p] = (status == ROM_ST_CONVERGED) ? (1u << 31) : 0u;
      }
      if (a.commit && !a.defer && status == ROM_ST_CONVERGED) {
        const int m = a.m;
        if (lane < 4) a.fbc[4 * (size_t)p + lane] = a.Fbar[4 * (size_t)p + lane];
        for (int i = lane; i < n; i += 64) a.rc[(size_t)p * n + i] = rt[i];
        double* hcw = a.hc + (size_t)p * 6 * m;
        const double* ht = a.ht + (size_t)p * 6 * m;
        for (int q = lane; q < 6 * m; q += 64) hcw[q] = ht[q];
      }
      return;
    }
  }
  if (lane == 0) {
    a.phi[2 * (size_t)p] = next;
    a.phi[2 * (size_t)p + 1] = fell_back ? 1 : 0;
    a.phd[2 * (size_t)p] = rn0;
    a.phd[2 * (size_t)p + 1] = rn;
    // a point converging slowly at the early hand-over goes to the side stream
    const bool slow = a.ph_early > 0 && next == a.ph_early && it > 0 && !(rn <= a.ph_slow * rn_prev);
    if (next > 0 && next < a.ph_k && !slow)
      a.lout[atomicAdd(a.cout, 1)] = p;
    else if (slow)
      a.early[atomicAdd(a.cearly, 1)] = p;
    else
      a.hand[atomicAdd(a.chand, 1)] = p;
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

// The point split keeps every tile's accumulator in each wave: FP64 up to
// five column tiles, FP32 accumulators (half the registers) up to eight.
template <int T, int PREC>
constexpr bool point_split_ok() {
  return T <= 5 || PREC != PREC_F64;
}

template <int T, int PREC>
int launch_prec(const FusedArgs& a, int split, int grid, int P, hipStream_t s) {
  if constexpr (point_split_ok<T, PREC>()) {
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
  if constexpr (16 * T <= ROM_PHASED_NPAD)
    if (rc == ROM_OK) rc = set_lds(&k_ph_cs<T, PREC, SPLIT>, (size_t)cs_lds_doubles<T>() * 8);
  return rc;
}

template <int T, int PREC>
int phased_cs_prec(const FusedArgs& a, int split, int P, hipStream_t s) {
  if constexpr (16 * T > ROM_PHASED_NPAD) {
    return ROM_EUNSUPPORTED;
  } else {
    const size_t lds = (size_t)cs_lds_doubles<T>() * 8;
    bool done = false;
    if constexpr (point_split_ok<T, PREC>()) {
      if (split == 0) {
        k_ph_cs<T, PREC, 0><<<P, 256, lds, s>>>(a);
        done = true;
      }
    }
    if (!done) k_ph_cs<T, PREC, 1><<<P, 256, lds, s>>>(a);
    return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
  }
}

template <int T>
int phased_solve(const FusedArgs& a, int P, hipStream_t s) {
  if constexpr (16 * T > ROM_SOLVE_NPAD) {
    return ROM_EUNSUPPORTED;
  } else {
    k_ph_s<T><<<(P + 3) / 4, 256, 0, s>>>(a);
    return hipGetLastError() == hipSuccess ? ROM_OK : ROM_EHIP;
  }
}

template <int T>
int phased_cs(const FusedArgs& a, int prec, int split, int P, hipStream_t s) {
  if (prec == ROM_DT_F64) return phased_cs_prec<T, PREC_F64>(a, split, P, s);
  if (prec == ROM_DT_F32) return phased_cs_prec<T, PREC_F32>(a, split, P, s);
  return phased_cs_prec<T, PREC_BF16>(a, split, P, s);
}

template <int T>
int fused_setup() {
  static_assert(lds_doubles<T>() * 8 <= 160 * 1024, "LDS of the fused kernel exceeds the workgroup limit");
  int rc = ROM_OK;
  if constexpr (point_split_ok<T, PREC_F64>())
    if (rc == ROM_OK) rc = setup_one<T, PREC_F64, 0>();
  if (rc == ROM_OK) rc = setup_one<T, PREC_F32, 0>();
  if (rc == ROM_OK) rc = setup_one<T, PREC_BF16, 0>();
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
  int rom_phased_cs_##T(const FusedArgs& a, int prec, int split, int P, hipStream_t s) {              \
    return phased_cs<T>(a, prec, split, P, s);                                                         \
  }                                                                                                    \
  int rom_phased_solve_##T(const FusedArgs& a, int P, hipStream_t s) { return phased_solve<T>(a, P, s); } \
  int rom_fused_setup_##T() { return fused_setup<T>(); }
