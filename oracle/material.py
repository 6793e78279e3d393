"""Material point of the RVE: Appendix A of the paper.

Small-strain J2 plasticity with linear isotropic hardening (eqs. j2_1..j2_6),
extended to large strains by the multiplicative split F = F^el F^pl and the
logarithmic elastic strain of the elastic right Cauchy-Green tensor
(eqs. j2_7..j2_10).  Plane strain: F_33 = 1, all out-of-plane shears zero.

Readings of the appendix taken here (each also listed in the design notes):

* the small-strain tensor is eps = 1/2 ln C^el (Hencky strain).  Taking
  eps = ln C^el literally would make the exponential update of F^pl and the
  small-strain limit inconsistent (the limit would be 2x the linear strain);
* the intermediate stress is S = 2 sigma : d eps / d C^el, and since sigma and
  C^el share eigenvectors this contraction equals sigma (C^el)^-1;
* the first Piola-Kirchhoff stress is P = F^el S (F^pl)^-T.  The printed
  (F^el)^-1 breaks the symmetry of P F^T (balance of angular momentum);
* a trial state exactly on the yield surface (f = 0) is elastic;
* the consistent tangent A = dP/dF at fixed history (the appendix gives no
  formula) is obtained by complex-step differentiation of the same update.

All functions are vectorised over leading axes; tensors are (..., 2, 2)
arrays holding the in-plane block, with the 33 components carried separately.
Complex input is accepted so that the complex-step tangent can reuse the
update unchanged; branch decisions use real parts only.
"""
import numpy as np

SQRT32 = np.sqrt(1.5)


def lame(E, nu):
    """Lame constants (lambda, G) of isotropic linear elasticity D in eq. j2_1."""
    G = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return lam, G


def _series(z, coeffs):
    out = np.zeros_like(z)
    zk = np.ones_like(z)
    for c in coeffs:
        out = out + c * zk
        zk = zk * z
    return out


_ATANH_C = [1.0 / (2 * k + 1) for k in range(14)]
_COSH_C = []
_SINHC_C = []
_f = 1.0
for _k in range(1, 30):
    _f *= _k
    if _k % 2 == 0:
        _COSH_C.append(1.0 / _f)
    else:
        _SINHC_C.append(1.0 / _f)
_COSH_C = [1.0] + _COSH_C[:13]
_SINHC_C = _SINHC_C[:14]


def _atanh_sqrt_over_sqrt(y):
    """atanh(sqrt(y)) / sqrt(y): an analytic function of y (series near 0)."""
    y = np.asarray(y)
    small = np.abs(y) < 1e-2
    ys = np.where(small, y, 0.0)
    yl = np.where(small, 0.25, y)
    sq = np.sqrt(yl)
    return np.where(small, _series(ys, _ATANH_C), np.arctanh(sq) / sq)


def _cosh_sqrt_and_sinhc(z):
    """(cosh(sqrt z), sinh(sqrt z)/sqrt z): analytic in z (series near 0)."""
    z = np.asarray(z)
    small = np.abs(z) < 1e-2
    zs = np.where(small, z, 0.0)
    zl = np.where(small, 1.0, z)
    s = np.sqrt(zl)
    ch = np.where(small, _series(zs, _COSH_C), np.cosh(s))
    sh = np.where(small, _series(zs, _SINHC_C), np.sinh(s) / s)
    return ch, sh


def _sym_parts(A):
    a = A[..., 0, 0]
    d = A[..., 1, 1]
    b = 0.5 * (A[..., 0, 1] + A[..., 1, 0])
    return a, b, d


def _from_isotropic_form(c0, c1, a, b, d, m):
    """c0 I + c1 (A - m I) for the symmetric 2x2 A = [[a, b], [b, d]]."""
    out = np.empty(np.shape(a) + (2, 2), dtype=np.result_type(c0, c1, a))
    out[..., 0, 0] = c0 + c1 * (a - m)
    out[..., 1, 1] = c0 + c1 * (d - m)
    out[..., 0, 1] = c1 * b
    out[..., 1, 0] = c1 * b
    return out


def logm_sym2(C):
    """Matrix logarithm of a symmetric positive-definite 2x2 tensor.

    With eigenvalues m +- s (m the mean, s the half spread), the spectral
    definition ln C = sum_i ln(c_i) N_i (x) N_i equals
    c0 I + c1 (C - m I) with c0 = (ln c_1 + ln c_2)/2 = ln(det C)/2 and
    c1 = (ln c_1 - ln c_2)/(c_1 - c_2) = atanh(s/m)/s, which stays analytic
    when the eigenvalues coincide (C = I at the first evaluation).
    """
    a, b, d = _sym_parts(C)
    m = 0.5 * (a + d)
    s2 = 0.25 * (a - d) ** 2 + b * b
    c1 = _atanh_sqrt_over_sqrt(s2 / (m * m)) / m
    c0 = 0.5 * np.log(a * d - b * b)
    return _from_isotropic_form(c0, c1, a, b, d, m)


def expm_sym2(A):
    """Matrix exponential of a symmetric 2x2 tensor (spectral definition).

    exp A = e^m [cosh(s) I + sinh(s)/s (A - m I)], eigenvalues m +- s.
    """
    a, b, d = _sym_parts(A)
    m = 0.5 * (a + d)
    s2 = 0.25 * (a - d) ** 2 + b * b
    ch, sh = _cosh_sqrt_and_sinhc(s2)
    em = np.exp(m)
    return _from_isotropic_form(em * ch, em * sh, a, b, d, m)


def inv2(A):
    det = A[..., 0, 0] * A[..., 1, 1] - A[..., 0, 1] * A[..., 1, 0]
    out = np.empty_like(A)
    out[..., 0, 0] = A[..., 1, 1] / det
    out[..., 1, 1] = A[..., 0, 0] / det
    out[..., 0, 1] = -A[..., 0, 1] / det
    out[..., 1, 0] = -A[..., 1, 0] / det
    return out


def tr2(A):
    return np.swapaxes(A, -1, -2)


def j2_update(F, Fp, Fp33, xi, mat):
    """One implicit load step of the appendix model at fixed committed history.

    Parameters
    ----------
    F     : (..., 2, 2) in-plane deformation gradient (F_33 = 1).
    Fp    : (..., 2, 2) committed in-plane plastic deformation gradient F^pl_n.
    Fp33  : (...)       committed F^pl_33.
    xi    : (...)       committed equivalent plastic strain xi_n.
    mat   : (E, nu, sigma_y0, H), scalars or arrays of the batch shape (...)
            (a material per point: several phases).

    Returns (P, Fp_new, Fp33_new, xi_new, gamma), P the in-plane 1PK stress.
    """
    E, nu, sy0, H = (np.asarray(v, dtype=np.float64) for v in mat)
    lam, G = lame(E, nu)
    G2 = G[..., None, None]  # G against (..., 2, 2) tensors
    # trial elastic state, eq. j2_7 with eps = 1/2 ln C^el
    Fe_tr = F @ inv2(Fp)
    Ce_tr = tr2(Fe_tr) @ Fe_tr
    eps = 0.5 * logm_sym2(Ce_tr)
    eps33 = -np.log(Fp33)  # F^el_33 = 1 / F^pl_33 because F_33 = 1
    treps = eps[..., 0, 0] + eps[..., 1, 1] + eps33
    # eq. j2_1 (trial: eps^pl carried by F^pl)
    sig = 2.0 * G2 * eps
    sig[..., 0, 0] += lam * treps
    sig[..., 1, 1] += lam * treps
    sig33 = 2.0 * G * eps33 + lam * treps
    p = (sig[..., 0, 0] + sig[..., 1, 1] + sig33) / 3.0
    dev = sig.copy()
    dev[..., 0, 0] -= p
    dev[..., 1, 1] -= p
    dev33 = sig33 - p
    nd = np.sqrt(dev[..., 0, 0] ** 2 + dev[..., 1, 1] ** 2 + dev[..., 0, 1] ** 2
                 + dev[..., 1, 0] ** 2 + dev33 ** 2)
    # eq. j2_2: von Mises yield function; KKT conditions eq. j2_6
    fy = SQRT32 * nd - (sy0 + H * xi)
    plastic = np.real(fy) > 0.0
    # linear hardening: the consistency condition gives gamma in closed form
    gam = np.where(plastic, fy / (3.0 * G + H), 0.0)
    nds = np.where(np.real(nd) > 0.0, nd, 1.0)
    # eq. j2_3: flow direction
    r = SQRT32 * dev / nds[..., None, None]
    r33 = SQRT32 * dev33 / nds
    sig_new = sig - 2.0 * G2 * gam[..., None, None] * r
    xi_new = xi + gam
    # eq. j2_10: exponential update of F^pl
    Fp_new = expm_sym2(gam[..., None, None] * r) @ Fp
    Fp33_new = np.exp(gam * r33) * Fp33
    # eqs. j2_8, j2_9
    Fe = F @ inv2(Fp_new)
    Ce = tr2(Fe) @ Fe
    S = sig_new @ inv2(Ce)
    P = Fe @ S @ tr2(inv2(Fp_new))
    return P, Fp_new, Fp33_new, xi_new, gam


def j2_point(F, Fp, Fp33, xi, mat, h=1e-30):
    """Stress, consistent tangent and trial history at fixed committed history.

    A[..., i, j, k, l] = dP_ij / dF_kl is computed by complex-step
    differentiation (Squire & Trapp 1998): Im P(F + i h E_kl) / h, exact to
    rounding because no difference of nearby values is formed.

    Returns (P, A, Fp_new, Fp33_new, xi_new, gamma).
    """
    F = np.asarray(F, dtype=np.float64)
    P, Fp_new, Fp33_new, xi_new, gam = j2_update(F, Fp, Fp33, xi, mat)
    A = np.empty(F.shape + (2, 2), dtype=np.float64)
    for k in range(2):
        for l in range(2):
            Fc = F.astype(np.complex128)
            Fc[..., k, l] += 1j * h
            Pc = j2_update(Fc, Fp, Fp33, xi, mat)[0]
            A[..., :, :, k, l] = Pc.imag / h
    return P, A, Fp_new, Fp33_new, xi_new, gam


def virgin_history(shape):
    """F^pl = I, xi = 0 at the start (appendix)."""
    Fp = np.zeros(tuple(shape) + (2, 2))
    Fp[..., 0, 0] = 1.0
    Fp[..., 1, 1] = 1.0
    return Fp, np.ones(shape), np.zeros(shape)
