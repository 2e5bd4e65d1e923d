"""Pins of the oracle's stiffness closure (Sec. II C 3, eqPk, App. B) against references that do
not come from the oracle: scipy's Bessel functions, the orientation integral eqCdef1 evaluated
by brute-force quadrature of the rotated four-index tensor, and the paper's printed isotropic
values (tests/golden/paper_values.json)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sp

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
KX = tuple(GOLD["table_IV_Kx"]["value"][k] for k in ("K1111", "K1122", "K2222", "K1212"))


@pytest.mark.parametrize("n", [0, 1, 2, 4])
def test_bessel_series_matches_scipy(n):
    for k in np.concatenate([np.linspace(0.0, 5.0, 21), np.linspace(5.0, 60.0, 23)]):
        ref = sp.iv(n, k)
        got = oracle.bessel_i(n, k)
        assert abs(got - ref) <= 1e-13 * max(ref, 1e-300) + (1e-300 if ref == 0 else 0), (n, k, got, ref)


def test_app_b_bracket_is_k3_i4():
    # App. B's bracket (k(k^2+24) I0 - 8(k^2+6) I1) / k^3 equals I4(k) (Bessel recurrence);
    # checked with scipy where the printed form does not cancel catastrophically
    for k in np.linspace(1.0, 50.0, 50):
        br = (k * (k * k + 24) * sp.iv(0, k) - 8 * (k * k + 6) * sp.iv(1, k)) / k ** 3
        assert abs(br - sp.iv(4, k)) <= 1e-9 * sp.iv(4, k)
        assert abs(oracle.bessel_i(4, k) - br) <= 1e-9 * br


def test_k_of_p_inverts_eqPk():
    for p in np.concatenate([np.linspace(1e-4, 0.9, 40), [0.95, 0.97, 0.98, 0.99]]):
        k = oracle.k_of_p(p)
        assert abs(sp.iv(1, k) / sp.iv(0, k) - p) <= 2e-15, p
    assert oracle.k_of_p(0.0) == 0.0
    # k at the clamp and at the equilibrium polarization of Table III
    assert abs(oracle.k_of_p(0.99) - 50.25384740) < 1e-7
    assert abs(oracle.k_of_p(math.sqrt(0.9)) - 10.01578) < 1e-4


def _kx_tensor(Kx):
    K1111, K1122, K2222, K1212 = Kx
    K = np.zeros((2, 2, 2, 2))
    K[0, 0, 0, 0] = K1111
    K[1, 1, 1, 1] = K2222
    K[0, 0, 1, 1] = K[1, 1, 0, 0] = K1122
    K[0, 1, 0, 1] = K[0, 1, 1, 0] = K[1, 0, 0, 1] = K[1, 0, 1, 0] = K1212
    return K


def quadrature_stiffness(Px, Py, Kx, P_clamp=0.99, M=4096):
    """C_ijkl = int g(theta - theta_P; k) Q Q Q Q K^x dtheta (eqCTens, eqrotate) by the trapezoid
    rule on a periodic grid, returned as the operator on plain components (Xxx, Xyy, Xxy)."""
    P = math.hypot(Px, Py)
    p = min(P, P_clamp)
    k = 0.0 if p == 0 else float(_k_scipy(p))
    thP = math.atan2(Py, Px)
    th = 2 * math.pi * np.arange(M) / M
    g = np.exp(k * (np.cos(th - thP) - 1.0))
    g /= g.sum()
    c, s = np.cos(th), np.sin(th)
    Q = np.stack([np.stack([c, -s], -1), np.stack([s, c], -1)], -2)   # (M, 2, 2): Q x^ = n^
    K = _kx_tensor(Kx)
    Kr = np.einsum("mia,mjb,mkc,mld,abcd->mijkl", Q, Q, Q, Q, K)
    C = np.einsum("m,mijkl->ijkl", g, Kr)
    rows = [(0, 0), (1, 1), (0, 1)]
    M3 = np.zeros((3, 3))
    for a, (i, j) in enumerate(rows):
        M3[a, 0] = C[i, j, 0, 0]
        M3[a, 1] = C[i, j, 1, 1]
        M3[a, 2] = C[i, j, 0, 1] + C[i, j, 1, 0]
    return M3


def _k_scipy(p):
    from scipy.optimize import brentq
    return brentq(lambda k: sp.ive(1, k) / sp.ive(0, k) - p, 1e-12, 1e4, xtol=1e-15, rtol=1e-15)


def test_closed_form_equals_orientation_integral():
    rng = np.random.default_rng(7)
    for trial in range(25):
        Kx = tuple(rng.uniform(-0.5, 1.0, size=4))
        P = rng.uniform(0.0, 1.05)
        th = rng.uniform(-math.pi, math.pi)
        Px, Py = P * math.cos(th), P * math.sin(th)
        C = oracle.stiffness(Px, Py, Kx)
        Q = quadrature_stiffness(Px, Py, Kx)
        scale = max(abs(x) for x in Kx)
        assert np.max(np.abs(C - Q)) <= 1e-12 * scale, (trial, C, Q)


def test_isotropic_values_printed_in_paper():
    gold = GOLD["isotropic_stiffness_table_IV"]["value"]
    C = oracle.stiffness(0.0, 0.0, KX)
    assert abs(C[0, 0] - gold["C11"]) < 1e-15 and abs(C[1, 1] - gold["C11"]) < 1e-15
    assert abs(C[0, 1] - gold["C12"]) < 1e-15 and abs(C[1, 0] - gold["C12"]) < 1e-15
    assert abs(C[2, 2] - gold["C33"]) < 1e-15
    assert abs(C[2, 2] - (C[0, 0] - C[0, 1])) < 1e-15
    for (i, j) in [(0, 2), (1, 2), (2, 0), (2, 1)]:
        assert C[i, j] == 0.0


def test_scalar_limit_recovers_scalar_modulus():
    # C~12 = 0 (K1111 + 6 K1122 - 4 K1212 + K2222 = 0) makes the isotropic C~ a multiple of I
    Kmod = 0.02
    C = oracle.stiffness(0.0, 0.0, (Kmod, 0.0, Kmod, Kmod / 2))
    assert np.allclose(C, Kmod * np.eye(3), atol=1e-17)
    # K^x itself isotropic: every rotation of it is the same tensor, so any orientation
    # distribution averages to it and the scalar model of Sec. II B holds at every P
    for P, th in ((0.5, 0.3), (0.9, 2.0), (0.99, -1.1)):
        C = oracle.stiffness(P * math.cos(th), P * math.sin(th), (Kmod, 0.0, Kmod, Kmod / 2))
        assert np.allclose(C, Kmod * np.eye(3), rtol=0, atol=1e-16), (P, th, C)


def test_strong_alignment_tends_to_kx():
    # k -> infinity along x: g -> delta at theta = 0 and C~ -> K~x (eqKmatrix, plain components),
    # with a deviation that shrinks like 1/k
    K1111, K1122, K2222, K1212 = KX
    target = np.array([[K1111, K1122, 0], [K1122, K2222, 0], [0, 0, 2 * K1212]])
    devs = []
    for p in (0.99, 0.995, 0.998):
        C = oracle.stiffness(p, 0.0, KX, P_clamp=p)
        k = oracle.k_of_p(p)
        dev = np.max(np.abs(C - target))
        assert dev <= 4.0 * max(KX) / k
        devs.append(dev)
    assert devs[0] > devs[1] > devs[2]


def test_clamp_only_enters_k():
    # |P| above the clamp: same C~ as at the clamp, same direction
    a = oracle.stiffness(1.2 * math.cos(0.3), 1.2 * math.sin(0.3), KX)
    b = oracle.stiffness(0.99 * math.cos(0.3), 0.99 * math.sin(0.3), KX)
    assert np.max(np.abs(a - b)) < 1e-15


def test_stiffness_even_in_P_and_period_pi():
    rng = np.random.default_rng(3)
    for _ in range(10):
        P = rng.uniform(0.1, 0.95)
        th = rng.uniform(0, 2 * math.pi)
        a = oracle.stiffness(P * math.cos(th), P * math.sin(th), KX)
        b = oracle.stiffness(-P * math.cos(th), -P * math.sin(th), KX)
        assert np.max(np.abs(a - b)) < 1e-16
