"""Shape sensitivities dPbar/dmu of the oracle (eq. eff_sensitivities_full in
its ECM form, committed history held fixed) against what fixes them
independently: central finite differences of the coefficient map and of the
solved effective stress, and the zero load where the stress vanishes for
every shape."""
import numpy as np

import workloads
from oracle import auxiliary as aux
from oracle.rom import ROM
from tests.conftest import rom_path


def test_coefficient_jacobian_matches_central_differences():
    cases = ((0, np.array([0.2, 0.31]), 0.25, None),
             (1, np.array([1.2, 0.3, 1.0, 0.0, 1.5, 1.0, 1.3, 2.5]), np.sqrt(0.075 / np.pi), 0.075))
    h = 1e-6
    for kind, mu, r0, A in cases:
        Jc = aux.coefficient_jacobian(kind, mu, r0, A)
        fd = np.stack([(aux.coefficients(kind, mu + h * e, r0, A) - aux.coefficients(kind, mu - h * e, r0, A)) / (2 * h)
                       for e in np.eye(len(mu))], axis=1)
        assert Jc.shape == fd.shape
        assert np.abs(Jc - fd).max() < 1e-8 * max(1.0, np.abs(Jc).max())


def _state(rom, mu, path):
    """Committed history after all but the last step, and the solved last step."""
    hist, r = rom.virgin(), np.zeros(rom.n)
    Finv, J = rom.transformation(mu)
    for k in range(len(path) - 1):
        s = rom.step(r, hist, path[k], Finv, J, tol=1e-12, max_iter=40)
        assert s['status'] == 0
        r, hist = s['r'], s['hist']
    s = rom.step(r, hist, path[-1], Finv, J, tol=1e-12, max_iter=40)
    assert s['status'] == 0
    return hist, s['r']


def _fd(rom, mu, r, Fb, hist, h=1e-6):
    out = np.zeros((4, len(mu)))
    for j in range(len(mu)):
        e = np.zeros(len(mu))
        e[j] = h
        P = []
        for sg in (1, -1):
            Fi, Jm = rom.transformation(mu + sg * e)
            t = rom.step(r, hist, Fb, Fi, Jm, tol=1e-13, max_iter=40)
            assert t['status'] == 0
            P.append(t['Pbar'])
        out[:, j] = (P[0] - P[1]) / (2 * h)
    return out


def test_sensitivity_matches_finite_differences_one_void():
    rom = ROM(rom_path('onevoid_n20_m120'))
    mu = workloads.one_void_mu(3, 1)[0]
    path = workloads.monotone_paths(3, 1, 4, (0.03, 0.05))[0]
    hist, r = _state(rom, mu, path)
    assert np.mean(hist[2] > 0) > 0.5  # a plastic state
    S = rom.shape_sensitivity(mu, r, path[-1], hist)
    fd = _fd(rom, mu, r, path[-1], hist)
    assert np.abs(S - fd).max() < 1e-7 * np.abs(S).max()


def test_sensitivity_matches_finite_differences_four_voids():
    rom = ROM(rom_path('fourvoid_n60_m800'))
    mu = workloads.four_void_mu(3, 1)[0]
    path = workloads.monotone_paths(3, 1, 3, (0.02, 0.03))[0]
    hist, r = _state(rom, mu, path)
    S = rom.shape_sensitivity(mu, r, path[-1], hist)
    assert S.shape == (4, 8)
    fd = _fd(rom, mu, r, path[-1], hist)
    assert np.abs(S - fd).max() < 1e-6 * np.abs(S).max()


def test_zero_load_has_zero_sensitivity():
    rom = ROM(rom_path('onevoid_n20_m120'))
    mu = workloads.one_void_mu(4, 1)[0]
    S = rom.shape_sensitivity(mu, np.zeros(rom.n), np.eye(2), rom.virgin())
    assert np.abs(S).max() == 0.0
