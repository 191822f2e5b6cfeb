"""Pins of ``oracle.fidelity`` (CPU only), the metric every state-parity
check uses: F(a, b) = |<a|b>|^2 / (<a|a><b|b>).

Each case is fixed by something other than the function's own formula:
orthogonal states, the overlap of |0> and |+>, global phases, the scaling
invariance of the normalised form, the closed-form overlap of two
single-qubit rotations on the Bloch sphere, a product state (the overlap
factorises), and an explicit element-by-element overlap written as a
Python loop. A plausible slip (no conjugate, no normalisation, the real
part instead of the modulus, a missing square) fails at least one of them.
"""
import cmath
import math

import numpy as np
import pytest

import oracle


def test_orthogonal_states_give_zero():
    e0 = np.array([1, 0, 0, 0], dtype=np.complex128)
    e3 = np.array([0, 0, 0, 1], dtype=np.complex128)
    assert oracle.fidelity(e0, e3) == 0.0
    # |+> and |-> are orthogonal although no component vanishes
    r = 1 / math.sqrt(2)
    plus = np.array([r, r], dtype=np.complex128)
    minus = np.array([r, -r], dtype=np.complex128)
    assert abs(oracle.fidelity(plus, minus)) <= 1e-16
    # |+i> and |-i>: orthogonal only when the first argument is conjugated
    pi_ = np.array([r, 1j * r])
    mi_ = np.array([r, -1j * r])
    assert abs(oracle.fidelity(pi_, mi_)) <= 1e-16
    assert abs(oracle.fidelity(pi_, pi_) - 1.0) <= 1e-15


def test_zero_and_plus_give_one_half():
    r = 1 / math.sqrt(2)
    e0 = np.array([1, 0], dtype=np.complex128)
    plus = np.array([r, r], dtype=np.complex128)
    assert abs(oracle.fidelity(e0, plus) - 0.5) <= 1e-15
    assert abs(oracle.fidelity(plus, e0) - 0.5) <= 1e-15


@pytest.mark.parametrize("alpha", [0.3, math.pi / 2, math.pi, 4.0])
def test_global_phase_gives_one(alpha):
    g = np.random.default_rng(7)
    a = g.standard_normal(64) + 1j * g.standard_normal(64)
    a /= np.linalg.norm(a)
    b = cmath.exp(1j * alpha) * a
    assert abs(oracle.fidelity(a, b) - 1.0) <= 1e-14
    # the real part of the overlap alone would give cos^2(alpha), not 1
    assert abs(oracle.fidelity(a, b) - math.cos(alpha) ** 2) > 1e-3 or abs(math.sin(alpha)) < 1e-3


@pytest.mark.parametrize("sa,sb", [(2.0, 1.0), (1.0, 0.25), (3.0, 1e-3), (1e3, 7.0)])
def test_invariant_under_scaling_of_either_argument(sa, sb):
    g = np.random.default_rng(11)
    a = g.standard_normal(32) + 1j * g.standard_normal(32)
    b = g.standard_normal(32) + 1j * g.standard_normal(32)
    f = oracle.fidelity(a, b)
    assert 0.0 < f < 1.0
    assert abs(oracle.fidelity(sa * a, sb * b) - f) <= 1e-13
    assert abs(oracle.fidelity(sa * a, b) - f) <= 1e-13


@pytest.mark.parametrize("t1,t2", [(0.0, math.pi), (0.4, 1.9), (2.5, -0.7), (math.pi / 3, math.pi / 3)])
def test_two_rotations_on_the_bloch_sphere(t1, t2):
    """RY(t)|0> = (cos t/2, sin t/2): two such states overlap in
    cos((t1 - t2)/2), so F = cos^2((t1 - t2)/2); RZ phases on both sides
    (e^{-i p/2}, e^{i p/2}) with different p change it to
    |c1 c2 e^{i d/2} + s1 s2 e^{-i d/2}|^2, d = p1 - p2."""
    a = np.array([math.cos(t1 / 2), math.sin(t1 / 2)], dtype=np.complex128)
    b = np.array([math.cos(t2 / 2), math.sin(t2 / 2)], dtype=np.complex128)
    assert abs(oracle.fidelity(a, b) - math.cos((t1 - t2) / 2) ** 2) <= 1e-15
    p1, p2 = 0.9, -0.35
    ap = a * np.array([cmath.exp(-0.5j * p1), cmath.exp(0.5j * p1)])
    bp = b * np.array([cmath.exp(-0.5j * p2), cmath.exp(0.5j * p2)])
    d = p1 - p2
    c1, s1, c2, s2 = math.cos(t1 / 2), math.sin(t1 / 2), math.cos(t2 / 2), math.sin(t2 / 2)
    ref = abs(c1 * c2 * cmath.exp(0.5j * d) + s1 * s2 * cmath.exp(-0.5j * d)) ** 2
    assert abs(oracle.fidelity(ap, bp) - ref) <= 1e-15


def test_product_states_factorise():
    """For product states the overlap is the product of the single-qubit
    overlaps (qubit q is bit q of the index)."""
    g = np.random.default_rng(3)
    n = 6
    fa, fb, ref = [], [], 1.0
    for _ in range(n):
        u = g.standard_normal(2) + 1j * g.standard_normal(2)
        v = g.standard_normal(2) + 1j * g.standard_normal(2)
        u /= np.linalg.norm(u)
        v /= np.linalg.norm(v)
        fa.append(u)
        fb.append(v)
        ref *= abs(np.conj(u[0]) * v[0] + np.conj(u[1]) * v[1]) ** 2
    a, b = fa[0], fb[0]
    for q in range(1, n):
        a = np.kron(fa[q], a)
        b = np.kron(fb[q], b)
    assert abs(oracle.fidelity(a, b) - ref) <= 1e-14


def test_random_pair_against_an_explicit_loop():
    """Overlap and norms summed component by component in Python."""
    g = np.random.default_rng(5)
    a = g.standard_normal(16) + 1j * g.standard_normal(16)
    b = g.standard_normal(16) + 1j * g.standard_normal(16)
    ov_re = ov_im = na = nb = 0.0
    for k in range(16):
        ar, ai, br, bi = a[k].real, a[k].imag, b[k].real, b[k].imag
        ov_re += ar * br + ai * bi   # conj(a) b, real part
        ov_im += ar * bi - ai * br   # conj(a) b, imaginary part
        na += ar * ar + ai * ai
        nb += br * br + bi * bi
    ref = (ov_re * ov_re + ov_im * ov_im) / (na * nb)
    assert abs(oracle.fidelity(a, b) - ref) <= 1e-14
    assert 0.0 <= oracle.fidelity(a, b) <= 1.0


def test_sensitivity_at_the_parity_bar():
    """A state rotated by a small angle eps away from the reference has
    1 - F = sin^2(eps/2): at eps = 2e-3 that is 1e-6, the parity bar, so
    a metric that read ~1 for every pair would be caught here."""
    g = np.random.default_rng(9)
    a = g.standard_normal(128) + 1j * g.standard_normal(128)
    a /= np.linalg.norm(a)
    w = g.standard_normal(128) + 1j * g.standard_normal(128)
    w -= np.vdot(a, w) * a
    w /= np.linalg.norm(w)
    for eps in (2e-3, 1e-2, 0.5):
        b = math.cos(eps / 2) * a + math.sin(eps / 2) * w
        assert abs((1 - oracle.fidelity(a, b)) - math.sin(eps / 2) ** 2) <= 1e-13
