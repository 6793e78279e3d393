"""Floating-point operation count of the material point and of the per-point
weighting, for the roofline's algorithmic flop count.

The device header's return map and tangent (csrc/j2_device.h) and the
weighting of point_material / put_record_wf are compiled on the host with
every double replaced by a counting number type: each executed addition,
subtraction, multiplication, division and square root counts one, a fused
multiply-add two, and each call of log, exp, atanh, cosh or sinh one (their
own instruction sequences are not counted, so the figure is a lower bound).
Four states cover the branches: elastic and plastic, with coincident and
distinct eigenvalues of the trial strain.

    python -m paper_2307_16894_amd.flop_count   (prints JSON)
"""
import json
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))

PRELUDE = r'''
#include <cmath>
#include <cstdio>
static long long g_ops = 0, g_tr = 0;
struct cnt {
  double v;
  cnt() : v(0) {}
  cnt(double x) : v(x) {}
  explicit operator double() const { return v; }
};
#define BIN(op) \
  inline cnt operator op(cnt a, cnt b) { ++g_ops; return cnt(a.v op b.v); } \
  inline cnt operator op(cnt a, double b) { ++g_ops; return cnt(a.v op b); } \
  inline cnt operator op(double a, cnt b) { ++g_ops; return cnt(a op b.v); }
BIN(+) BIN(-) BIN(*) BIN(/)
#define CMP(op) \
  inline bool operator op(cnt a, cnt b) { return a.v op b.v; } \
  inline bool operator op(cnt a, double b) { return a.v op b; }
CMP(<) CMP(>) CMP(<=) CMP(>=)
inline cnt operator-(cnt a) { return cnt(-a.v); }
inline cnt& operator+=(cnt& a, cnt b) { a = a + b; return a; }
inline cnt& operator*=(cnt& a, cnt b) { a = a * b; return a; }
inline cnt fma(cnt a, cnt b, cnt c) { g_ops += 2; return cnt(std::fma(a.v, b.v, c.v)); }
inline cnt sqrt(cnt a) { ++g_ops; return cnt(std::sqrt(a.v)); }
#define TR(f) inline cnt f(cnt a) { ++g_tr; return cnt(std::f(a.v)); }
TR(log) TR(exp) TR(atanh) TR(cosh) TR(sinh)
#define __host__
#define __device__
'''

MAIN = r'''
int main() {
  J2Params mp;
  const cnt E = 1.0, nu = 0.3;
  mp.G = (E / (2.0 * (1.0 + nu))).v; mp.lam = (E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))).v;
  mp.K = mp.lam + 2.0 * mp.G / 3.0; mp.sy0 = 0.01; mp.H = 0.05;
  const double cases[4][4] = {{1.0, 0.0, 0.0, 1.0}, {1.003, 0.001, 0.0, 0.998},
                              {1.04, 0.0, 0.0, 1.0}, {1.05, 0.02, 0.01, 0.97}};
  printf("[");
  for (int c = 0; c < 4; ++c) {
    cnt F[4], Fp[4] = {1.0, 0.0, 0.0, 1.0}, P[4], Fpn[4], Fp33n, xin, D[16];
    for (int k = 0; k < 4; ++k) F[k] = cases[c][k];
    const cnt Fi[4] = {1.02, 0.01, -0.01, 0.97};
    const cnt wl = 0.5;
    g_ops = g_tr = 0;
    for (int k = 0; k < 16; ++k) D[k] = 0.0;
    j2_point_cols<true>(F, Fp, cnt(1.0), cnt(0.0), mp, P, Fpn, Fp33n, xin,
                        [&](int v, cnt c0, cnt c1, cnt c2, cnt c3) { (void)v; (void)c0; (void)c1; (void)c2; (void)c3; });
    const long long cm = g_ops, tr = g_tr;
    g_ops = 0;
    // weighting: D = w|J| T^T A T accumulated per tangent column, W = w|J| P F_mu^-T
    j2_point_cols<true>(F, Fp, cnt(1.0), cnt(0.0), mp, P, Fpn, Fp33n, xin,
                        [&](int v, cnt c0, cnt c1, cnt c2, cnt c3) {
                          const cnt e0 = wl * (Fi[0] * c0 + Fi[1] * c1);
                          const cnt e1 = wl * (Fi[2] * c0 + Fi[3] * c1);
                          const cnt e2 = wl * (Fi[0] * c2 + Fi[1] * c3);
                          const cnt e3 = wl * (Fi[2] * c2 + Fi[3] * c3);
                          const int k = v >> 1, l = v & 1;
                          const cnt t0 = l ? Fi[1] : Fi[0], t1 = l ? Fi[3] : Fi[2];
                          for (int s2 = 0; s2 < 2; ++s2) {
                            const cnt t = s2 ? t1 : t0;
                            D[0 + 2 * k + s2] = fma(e0, t, D[0 + 2 * k + s2]);
                            D[4 + 2 * k + s2] = fma(e1, t, D[4 + 2 * k + s2]);
                            D[8 + 2 * k + s2] = fma(e2, t, D[8 + 2 * k + s2]);
                            D[12 + 2 * k + s2] = fma(e3, t, D[12 + 2 * k + s2]);
                          }
                        });
    const long long wd = g_ops - cm;
    g_ops = 0;
    cnt W[4];
    W[0] = wl * fma(P[1], Fi[1], P[0] * Fi[0]);
    W[1] = wl * fma(P[1], Fi[3], P[0] * Fi[2]);
    W[2] = wl * fma(P[3], Fi[1], P[2] * Fi[0]);
    W[3] = wl * fma(P[3], Fi[3], P[2] * Fi[2]);
    const long long ww = g_ops;
    printf("%s{\"F\": [%g, %g, %g, %g], \"plastic\": %d, \"material\": %lld, \"transcendental\": %lld, "
           "\"weighting\": %lld}", c ? ", " : "", cases[c][0], cases[c][1], cases[c][2], cases[c][3],
           (xin > 0.0) ? 1 : 0, cm, tr, wd + ww);
  }
  printf("]\n");
  return 0;
}
'''


def count():
    src = open(os.path.join(HERE, 'csrc', 'j2_device.h')).read()
    src = src.replace('#include <hip/hip_runtime.h>', '').replace('#pragma once', '')
    src = re.sub(r'\bdouble\b', 'cnt', src)
    src = src.replace('struct J2Params {\n  cnt lam, G, K, sy0, H;', 'struct J2Params {\n  double lam, G, K, sy0, H;')
    with tempfile.TemporaryDirectory() as d:
        cpp = os.path.join(d, 'count.cpp')
        with open(cpp, 'w') as fh:
            fh.write(PRELUDE + src + MAIN)
        exe = os.path.join(d, 'count')
        subprocess.run(['g++', '-std=c++17', '-O0', '-o', exe, cpp], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    cases = json.loads(out)
    return dict(cases=cases, material_min=min(c['material'] + c['transcendental'] for c in cases),
                weighting=max(c['weighting'] for c in cases))


if __name__ == '__main__':
    print(json.dumps(count()))
    sys.exit(0)
