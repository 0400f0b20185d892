"""Pins of the oracle's Symanzik gauge action and force.

* The action is checked against an independent sum over loops based at each
  site (plaquettes and rectangles built from array shifts, parallelograms
  traced as the hexagons of the unit 3-cubes that avoid a body diagonal),
  class by class.
* The force is the derivative of that independent action: central finite
  differences along random su(3) directions at several links, class by class.
* Traceless anti-Hermitian, zero on the free field, gauge covariant, and
  symmetric under translations and axis permutations.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1712_00143_amd import synth


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def _sh(f, d, mu, k):
    return synth._shift(f, d, mu, k)


def _loop(U, d, steps):
    """Product of links along a closed path of signed steps (+-(axis+1)),
    started at every site: [V][3][3]."""
    V = U.shape[0]
    P = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 3, 3)).copy()
    off = [0, 0, 0, 0]
    for st in steps:
        ax = abs(st) - 1
        if st > 0:
            L = U[:, ax]
            for a in range(4):
                L = _sh(L, d, a, off[a]) if off[a] else L
            off[ax] += 1
        else:
            off[ax] -= 1
            L = U[:, ax]
            for a in range(4):
                L = _sh(L, d, a, off[a]) if off[a] else L
            L = _dag(L)
        P = P @ L
    return P


def _hexagons(i, j, k):
    """The four six-link loops of the unit cube spanned by axes i, j, k that
    avoid a pair of opposite corners, as signed steps from a starting corner."""
    axes = (i, j, k)
    loops = []
    for diag in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        far = tuple(1 - b for b in diag)
        corners = [c for c in itertools.product((0, 1), repeat=3) if c not in (diag, far)]
        start = corners[0]
        path, cur, seen = [], start, {start}
        for _ in range(6):
            adj = [c for c in corners if sum(a != b for a, b in zip(c, cur)) == 1 and c not in seen]
            n = adj[0] if adj else start
            assert sum(a != b for a, b in zip(n, cur)) == 1
            a = [q for q in range(3) if n[q] != cur[q]][0]
            path.append((axes[a] + 1) * (1 if n[a] > cur[a] else -1))
            cur = n
            seen.add(cur)
        assert cur == start
        assert len(path) == 6
        loops.append((start, path))
    return loops


def independent_action(U, d, beta, c):
    tr = lambda P: np.trace(P, axis1=-2, axis2=-1).real.sum()
    V = U.shape[0]
    sp = sum(tr(_loop(U, d, [mu + 1, nu + 1, -(mu + 1), -(nu + 1)])) for mu in range(4) for nu in range(mu + 1, 4))
    sr = sum(tr(_loop(U, d, [mu + 1, mu + 1, nu + 1, -(mu + 1), -(mu + 1), -(nu + 1)]))
             for mu in range(4) for nu in range(4) if nu != mu)
    sg = 0.0
    for i, j, k in itertools.combinations(range(4), 3):
        for start, path in _hexagons(i, j, k):
            sg += tr(_loop(U, d, path))     # the sum over x does not depend on the start corner
    return beta * (c[0] * (6 * V - sp / 3) + c[1] * (12 * V - sr / 3) + c[2] * (16 * V - sg / 3))


CLASSES = [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0), (1.0, -0.0833, -0.0133)]


@pytest.mark.parametrize("c", CLASSES)
def test_action_matches_loop_sum(c):
    d = (4, 4, 6, 4)
    U = synth.thin_links(d, 0.5, 3)
    s_or = oracle.gauge_action(d, U, 5.7, c)
    s_in = independent_action(U, d, 5.7, c)
    assert abs(s_or - s_in) <= 1e-12 * abs(s_in)


def _expm_su3(X):
    w, v = np.linalg.eigh(-1j * X)
    return (v * np.exp(1j * w)[None, :]) @ _dag(v)


@pytest.mark.parametrize("c", CLASSES)
def test_force_is_the_derivative_of_the_action(c):
    d = (4, 4, 4, 6)
    U = synth.thin_links(d, 0.5, 5)
    beta = 6.0
    F = oracle.gauge_force(d, U, beta, c)
    rng = np.random.default_rng(6)
    eps = 1e-4
    for trial in range(4):
        s, mu = int(rng.integers(synth.volume(d))), int(rng.integers(4))
        H = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        X = 0.5 * (H - _dag(H))
        X -= np.trace(X) / 3 * np.eye(3)
        Up, Um = U.copy(), U.copy()
        Up[s, mu] = _expm_su3(eps * X) @ U[s, mu]
        Um[s, mu] = _expm_su3(-eps * X) @ U[s, mu]
        fd = (independent_action(Up, d, beta, c) - independent_action(Um, d, beta, c)) / (2 * eps)
        an = -np.trace(X @ F[s, mu]).real
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (trial, fd, an)


def test_force_structure_free_field_and_covariance():
    d = (4, 6, 4, 4)
    c = CLASSES[3]
    U = synth.thin_links(d, 0.4, 8)
    F = oracle.gauge_force(d, U, 5.5, c)
    assert np.abs(F + _dag(F)).max() < 1e-13
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-13
    assert np.abs(F).max() > 0.1
    fb, _ = synth.unit_links(d, phased=False)
    assert np.abs(oracle.gauge_force(d, fb, 5.5, c)).max() < 1e-14
    assert abs(oracle.gauge_action(d, fb, 5.5, c)) < 1e-10
    g = synth.random_su3(synth.volume(d), 9)
    Fg = oracle.gauge_force(d, synth.gauge_transform(U, d, g), 5.5, c)
    for mu in range(4):
        assert np.abs(Fg[:, mu] - g @ F[:, mu] @ _dag(g)).max() < 1e-12
    s0 = oracle.gauge_action(d, U, 5.5, c)
    assert abs(oracle.gauge_action(d, synth.gauge_transform(U, d, g), 5.5, c) - s0) < 1e-10 * abs(s0)


def test_force_translation_and_axis_permutation():
    d = (4, 4, 4, 4)
    c = CLASSES[3]
    U = synth.thin_links(d, 0.5, 10)
    F4 = oracle.gauge_force(d, U, 6.0, c).reshape(4, 4, 4, 4, 4, 3, 3)
    U4 = U.reshape(F4.shape)
    sh = (-1, -3, 0, -2)
    got = oracle.gauge_force(d, np.roll(U4, sh, axis=(0, 1, 2, 3)).reshape(U.shape), 6.0, c)
    assert np.abs(got - np.roll(F4, sh, axis=(0, 1, 2, 3)).reshape(U.shape)).max() < 1e-12
    for p in [(1, 0, 2, 3), (3, 2, 1, 0), (2, 3, 0, 1)]:
        inv = np.argsort([3 - p[3 - a] for a in range(4)])
        Up, Fp = np.empty_like(U4), np.empty_like(F4)
        for mu in range(4):
            Up[..., p[mu], :, :] = np.transpose(U4[..., mu, :, :], list(inv) + [4, 5])
            Fp[..., p[mu], :, :] = np.transpose(F4[..., mu, :, :], list(inv) + [4, 5])
        got = oracle.gauge_force(d, Up.reshape(U.shape), 6.0, c)
        assert np.abs(got - Fp.reshape(U.shape)).max() < 1e-12


def test_small_extents_are_refused():
    d = (2, 4, 4, 4)
    U = synth.thin_links(d, 0.4, 1)
    with pytest.raises(ValueError):
        oracle.gauge_force(d, U, 6.0, CLASSES[0])
    with pytest.raises(ValueError):
        oracle.gauge_action(d, U, 6.0, CLASSES[0])
