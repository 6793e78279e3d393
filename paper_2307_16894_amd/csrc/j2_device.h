// Finite-strain J2 material point for the ECM-point lanes (Appendix A of
// arXiv 2307.16894: small-strain J2 with linear isotropic hardening, lifted
// to finite strain by F = F^el F^pl, a logarithmic elastic strain and the
// exponential update of F^pl, eq. j2_10).  Plane strain, F_33 = 1.
//
// Formulated in the current configuration, which is equivalent for an
// isotropic model: with b^el_tr = F (C^pl_n)^-1 F^T the trial Hencky strain is
// eps_tr = 1/2 ln b^el_tr, the small-strain radial return gives the Kirchhoff
// stress tau (which equals F^el S (F^el)^T of eqs. j2_8, j2_9), and
// P = tau F^-T.  The exponential update F^pl_{n+1} = exp(gamma r_hat) F^pl_n
// (r_hat in the intermediate configuration) is evaluated as
// F^pl_n F^-1 exp(gamma r) F with r the spatial flow direction.
//
// The consistent tangent A = dP/dF at fixed history (the paper gives no
// formula) is the chain
//   dF -> db (b = F Cp^-1 F^T) -> d eps (derivative of the 2x2 matrix log in
//   closed form) -> d tau (elastoplastic tangent of radial return with
//   linear hardening) -> dP = d tau F^-T - P dF^T F^-T.
// 2x2 tensors are [11, 12, 21, 22]; A[4 * (2i+j) + (2k+l)] = dP_ij/dF_kl.
#pragma once
#include <hip/hip_runtime.h>

struct J2Params {
  double lam, G, K, sy0, H;
};

// g(y) = atanh(sqrt y) / sqrt y and g'(y); g is analytic at y = 0, where the
// two eigenvalues of b coincide (every virgin point at Fbar = I).
__host__ __device__ inline void atanh_ratio(double y, double& g, double& gp) {
  if (y < 0.05) {
    const int KS = 14;
    double a = 1.0 / (2 * KS + 1);
    double b = (double)KS / (2 * KS + 1);
#pragma unroll
    for (int k = KS - 1; k >= 0; --k) {
      a = fma(a, y, 1.0 / (2 * k + 1));
      if (k >= 1) b = fma(b, y, (double)k / (2 * k + 1));
    }
    g = a;
    gp = b;
  } else {
    double x = sqrt(y);
    g = atanh(x) / x;
    gp = (1.0 / (1.0 - y) - g) / (2.0 * y);
  }
}

// cosh(sqrt z) and sinh(sqrt z)/sqrt z, analytic at z = 0.
__host__ __device__ inline void cosh_sinhc(double z, double& ch, double& sh) {
  if (z < 0.05) {
    // cosh: sum z^k/(2k)!, sinhc: sum z^k/(2k+1)!
    double c = 0.0, s = 0.0;
    double fc = 1.0, fs = 1.0, zk = 1.0;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      c += zk / fc;
      s += zk / fs;
      fc *= (2.0 * k + 1.0) * (2.0 * k + 2.0);
      fs *= (2.0 * k + 2.0) * (2.0 * k + 3.0);
      zk *= z;
    }
    ch = c;
    sh = s;
  } else {
    double x = sqrt(z);
    ch = cosh(x);
    sh = sinh(x) / x;
  }
}

// One material evaluation at fixed committed history (Fp, Fp33, xi).
// Outputs P (4) and the trial history; when WANT_A, the columns of the
// tangent A[:, v] = dP/dF_v (v = 2k + l) are handed to sink(v, c0, c1, c2, c3)
// one at a time, so callers can fold them into what they need without
// holding all of A.
template <bool WANT_A, typename Sink>
__host__ __device__ inline void j2_point_cols(const double F[4], const double Fp[4], double Fp33, double xi,
                                              const J2Params& mp, double P[4], double Fpn[4], double& Fp33n,
                                              double& xin, Sink&& sink) {
  const double SQ32 = 1.2247448713915890491;  // sqrt(3/2)
  // (C^pl)^-1 = Fp^-1 Fp^-T
  const double dFp = Fp[0] * Fp[3] - Fp[1] * Fp[2];
  const double a0 = Fp[3] / dFp, a1 = -Fp[1] / dFp, a2 = -Fp[2] / dFp, a3 = Fp[0] / dFp;
  const double c00 = a0 * a0 + a1 * a1;
  const double c01 = a0 * a2 + a1 * a3;
  const double c11 = a2 * a2 + a3 * a3;
  // X = Cp^-1 F^T, b = F X
  const double X00 = c00 * F[0] + c01 * F[1];
  const double X01 = c00 * F[2] + c01 * F[3];
  const double X10 = c01 * F[0] + c11 * F[1];
  const double X11 = c01 * F[2] + c11 * F[3];
  const double b00 = F[0] * X00 + F[1] * X10;
  const double b01 = F[0] * X01 + F[1] * X11;
  const double b11 = F[2] * X01 + F[3] * X11;
  // eps = 1/2 ln b = 1/2 [ l0 I + h (b - m I) ]
  const double m = 0.5 * (b00 + b11);
  const double dd = 0.5 * (b00 - b11);
  const double s2 = dd * dd + b01 * b01;
  const double y = s2 / (m * m);
  double g, gp;
  atanh_ratio(y, g, gp);
  const double h = g / m;
  const double detb = b00 * b11 - b01 * b01;
  const double l0 = 0.5 * log(detb);
  const double e00 = 0.5 * (l0 + h * dd);
  const double e11 = 0.5 * (l0 - h * dd);
  const double e01 = 0.5 * h * b01;
  const double e33 = -log(Fp33);  // F^el_33 = 1/F^pl_33
  const double tre = e00 + e11 + e33;
  const double G2 = 2.0 * mp.G;
  const double t00 = mp.lam * tre + G2 * e00;
  const double t11 = mp.lam * tre + G2 * e11;
  const double t33 = mp.lam * tre + G2 * e33;
  const double t01 = G2 * e01;
  const double pm = (t00 + t11 + t33) * (1.0 / 3.0);
  const double d00 = t00 - pm, d11 = t11 - pm, d33 = t33 - pm, d01 = t01;
  const double nd = sqrt(d00 * d00 + d11 * d11 + 2.0 * d01 * d01 + d33 * d33);
  const double q = SQ32 * nd;
  const double fy = q - (mp.sy0 + mp.H * xi);
  double gam = 0.0, beta = 1.0, cn = 0.0;
  double n00 = 0.0, n11 = 0.0, n01 = 0.0, n33 = 0.0;
  if (fy > 0.0) {  // a trial state exactly on the yield surface is elastic
    const double G3 = 3.0 * mp.G;
    gam = fy / (G3 + mp.H);
    beta = 1.0 - G3 * gam / q;
    cn = 6.0 * mp.G * mp.G * (1.0 / (G3 + mp.H) - gam / q);
    const double inv = 1.0 / nd;
    n00 = d00 * inv;
    n11 = d11 * inv;
    n01 = d01 * inv;
    n33 = d33 * inv;
  }
  const double tau00 = pm + beta * d00;
  const double tau11 = pm + beta * d11;
  const double tau01 = beta * d01;
  // F^-T
  const double dF = F[0] * F[3] - F[1] * F[2];
  const double it00 = F[3] / dF, it01 = -F[2] / dF, it10 = -F[1] / dF, it11 = F[0] / dF;
  P[0] = tau00 * it00 + tau01 * it10;
  P[1] = tau00 * it01 + tau01 * it11;
  P[2] = tau01 * it00 + tau11 * it10;
  P[3] = tau01 * it01 + tau11 * it11;
  // history: F^pl_{n+1} = F^pl_n F^-1 exp(gamma r) F, r = sqrt(3/2) n
  xin = xi + gam;
  if (gam > 0.0) {
    const double k = gam * SQ32;
    const double M00 = k * n00, M11 = k * n11, M01 = k * n01;
    const double mm = 0.5 * (M00 + M11), md = 0.5 * (M00 - M11);
    double ch, sh;
    cosh_sinhc(md * md + M01 * M01, ch, sh);
    const double em = exp(mm);
    const double E00 = em * (ch + sh * md), E11 = em * (ch - sh * md), E01 = em * sh * M01;
    // Finv = F^-1 = (F^-T)^T
    const double f00 = it00, f01 = it10, f10 = it01, f11 = it11;
    // Y = E F
    const double Y00 = E00 * F[0] + E01 * F[2], Y01 = E00 * F[1] + E01 * F[3];
    const double Y10 = E01 * F[0] + E11 * F[2], Y11 = E01 * F[1] + E11 * F[3];
    // Z = F^-1 Y
    const double Z00 = f00 * Y00 + f01 * Y10, Z01 = f00 * Y01 + f01 * Y11;
    const double Z10 = f10 * Y00 + f11 * Y10, Z11 = f10 * Y01 + f11 * Y11;
    Fpn[0] = Fp[0] * Z00 + Fp[1] * Z10;
    Fpn[1] = Fp[0] * Z01 + Fp[1] * Z11;
    Fpn[2] = Fp[2] * Z00 + Fp[3] * Z10;
    Fpn[3] = Fp[2] * Z01 + Fp[3] * Z11;
    Fp33n = exp(k * n33) * Fp33;
  } else {
    Fpn[0] = Fp[0];
    Fpn[1] = Fp[1];
    Fpn[2] = Fp[2];
    Fpn[3] = Fp[3];
    Fp33n = Fp33;
  }
  if (!WANT_A) return;
  const double Xr[2][2] = {{X00, X01}, {X10, X11}};
  const double itr[2][2] = {{it00, it01}, {it10, it11}};
  const double im = 1.0 / m;
  const double idet = 1.0 / detb;
#pragma unroll
  for (int ab = 0; ab < 4; ++ab) {
    const int a = ab >> 1, bb = ab & 1;
    // db for dF = E_ab
    const double db00 = (a == 0) ? 2.0 * Xr[bb][0] : 0.0;
    const double db11 = (a == 1) ? 2.0 * Xr[bb][1] : 0.0;
    const double db01 = ((a == 0) ? Xr[bb][1] : 0.0) + ((a == 1) ? Xr[bb][0] : 0.0);
    const double dm = 0.5 * (db00 + db11);
    const double ddd = 0.5 * (db00 - db11);
    const double ds2 = 2.0 * dd * ddd + 2.0 * b01 * db01;
    const double dy = (ds2 - 2.0 * s2 * dm * im) * im * im;
    const double dh = (gp * dy - g * dm * im) * im;
    const double dl0 = 0.5 * (b11 * db00 - 2.0 * b01 * db01 + b00 * db11) * idet;
    const double de00 = 0.5 * (dl0 + dh * dd + h * ddd);
    const double de11 = 0.5 * (dl0 - dh * dd - h * ddd);
    const double de01 = 0.5 * (dh * b01 + h * db01);
    const double trde = de00 + de11;
    const double nde = n00 * de00 + n11 * de11 + 2.0 * n01 * de01;
    const double iso = mp.K * trde - G2 * beta * trde * (1.0 / 3.0);
    const double dt00 = iso + G2 * beta * de00 - cn * n00 * nde;
    const double dt11 = iso + G2 * beta * de11 - cn * n11 * nde;
    const double dt01 = G2 * beta * de01 - cn * n01 * nde;
    const double P0b = bb ? P[1] : P[0];
    const double P1b = bb ? P[3] : P[2];
    sink(ab, dt00 * itr[0][0] + dt01 * itr[1][0] - P0b * itr[a][0],
         dt00 * itr[0][1] + dt01 * itr[1][1] - P0b * itr[a][1],
         dt01 * itr[0][0] + dt11 * itr[1][0] - P1b * itr[a][0],
         dt01 * itr[0][1] + dt11 * itr[1][1] - P1b * itr[a][1]);
  }
}

// Convenience form returning the whole tangent A[4 * (2i+j) + (2k+l)].
template <bool WANT_A>
__host__ __device__ inline void j2_point(const double F[4], const double Fp[4], double Fp33, double xi,
                                         const J2Params& mp, double P[4], double A[16], double Fpn[4],
                                         double& Fp33n, double& xin) {
  j2_point_cols<WANT_A>(F, Fp, Fp33, xi, mp, P, Fpn, Fp33n, xin,
                        [&](int v, double c0, double c1, double c2, double c3) {
                          A[v] = c0;
                          A[4 + v] = c1;
                          A[8 + v] = c2;
                          A[12 + v] = c3;
                        });
}
