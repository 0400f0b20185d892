"""Pins of the oracle's HISQ link smearing to facts outside its own code.

The smearing (two fat7 levels with a U(3) projection between, Lepage and
Naik terms at the second; HISQ action, Follana et al. hep-lat/0610092, the
link smearing of the paper's Section 2 run-time breakdown) is pinned by:

* the free field: unit thin links give fat = 9/8 eta, long = -1/24 eta;
* constant commuting links, where every path collapses to the link itself;
* transverse-identity fields, where the path sum becomes a convolution of
  the one non-trivial direction whose weights follow from counting the
  orderings of each displacement (for the HISQ coefficients, the separable
  kernel [1/4, 1/2, 1/4] per transverse axis);
* gauge covariance under random site rotations, translation and axis
  permutation symmetry;
* the nested-staple recursion (5- and 7-staples as staples of staples),
  built on whole fields with array shifts;
* the polar factor against numpy's SVD, and the unitarity of the Naik
  products the composition yields.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1712_00143_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def _rng_coefs(seed):
    return tuple(np.random.default_rng(seed).uniform(-1.0, 1.0, 5))


def test_free_field():
    d = (4, 6, 4, 4)
    fb, _ = synth.unit_links(d, phased=False)
    eta = synth.staggered_phases(d)[:, :, None, None]
    one = np.eye(3)
    fat, lng = oracle.hisq_smear(d, fb)
    assert np.abs(fat - 9 / 8 * eta * one).max() < 1e-14
    assert np.abs(lng + 1 / 24 * eta * one).max() < 1e-15
    # level 1 alone averages to exactly the unit link
    v = oracle.fat7(d, fb, oracle.HISQ_LEVEL1)
    assert np.abs(v - one).max() < 1e-15


def test_constant_commuting_links_collapse_every_path():
    d = (4, 4, 6, 4)
    V = synth.volume(d)
    th = np.random.default_rng(5).uniform(-np.pi, np.pi, (4, 3))
    D = np.array([np.diag(np.exp(1j * t)) for t in th])           # U(3), commuting
    U = np.broadcast_to(D, (V, 4, 3, 3)).copy()
    c = _rng_coefs(11)
    npath = c[0] + 6 * c[1] + 24 * c[2] + 48 * c[3] + 6 * c[4]
    assert np.abs(oracle.fat7(d, U, c) - npath * U).max() < 1e-13
    assert np.abs(oracle.unitarize(U) - U).max() < 1e-15
    fat, lng = oracle.hisq_smear(d, U)
    eta = synth.staggered_phases(d)[:, :, None, None]
    assert np.abs(fat - 9 / 8 * eta * U).max() < 1e-13
    assert np.abs(lng + 1 / 24 * eta * (U @ U @ U)).max() < 1e-14


def _roll(field4, dims, mu, k):
    """field(x + k mu) on a [L3][L2][L1][L0] array."""
    return np.roll(field4, -k, axis=3 - mu)


@pytest.mark.parametrize("mu", [0, 1, 2, 3])
def test_transverse_identity_is_a_convolution(mu):
    d = (4, 6, 4, 6)
    V = synth.volume(d)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()
    U[:, mu] = synth.random_su3(V, 40 + mu)
    M = U[:, mu].reshape(d[3], d[2], d[1], d[0], 3, 3)
    perp = [nu for nu in range(4) if nu != mu]

    def shifted(off):
        f = M
        for nu, o in zip(perp, off):
            f = _roll(f, d, nu, o)
        return f

    # generic coefficients: a displacement with k non-zero unit offsets is
    # reached by k! orderings of its k transverse steps
    c = _rng_coefs(20 + mu)
    weight = {0: c[0], 1: c[1], 2: 2 * c[2], 3: 6 * c[3]}
    ref = np.zeros_like(M)
    for off in itertools.product((-1, 0, 1), repeat=3):
        ref = ref + weight[sum(o != 0 for o in off)] * shifted(off)
    for j in range(3):
        for s in (-2, 2):
            off = [0, 0, 0]
            off[j] = s
            ref = ref + c[4] * shifted(off)
    out = oracle.fat7(d, U, c)[:, mu].reshape(M.shape)
    assert np.abs(out - ref).max() < 1e-13

    # HISQ level 1: the separable [1/4, 1/2, 1/4] kernel on each transverse axis
    sep = M
    for nu in perp:
        sep = 0.25 * _roll(sep, d, nu, -1) + 0.5 * sep + 0.25 * _roll(sep, d, nu, 1)
    v1 = oracle.fat7(d, U, oracle.HISQ_LEVEL1)[:, mu].reshape(M.shape)
    assert np.abs(v1 - sep).max() < 1e-14
    # level 2: the same kernel plus 1/2 of the link minus 1/16 two steps out
    lep = sum(_roll(M, d, nu, s) for nu in perp for s in (-2, 2))
    v2 = oracle.fat7(d, U, oracle.HISQ_LEVEL2)[:, mu].reshape(M.shape)
    assert np.abs(v2 - (sep + 0.5 * M - lep / 16)).max() < 1e-14


def test_gauge_covariance():
    d = (4, 6, 4, 8)
    V = synth.volume(d)
    U = synth.thin_links(d, 0.4, 7)
    g = synth.random_su3(V, 8)
    Ug = synth.gauge_transform(U, d, g)
    c = _rng_coefs(9)

    def shifted_dag(mu, k):
        return _dag(synth._shift(g, d, mu, k))

    f, fg = oracle.fat7(d, U, c), oracle.fat7(d, Ug, c)
    n, ng = oracle.naik_product(d, U), oracle.naik_product(d, Ug)
    fat, lng = oracle.hisq_smear(d, U)
    fatg, lngg = oracle.hisq_smear(d, Ug)
    for mu in range(4):
        assert np.abs(fg[:, mu] - g @ f[:, mu] @ shifted_dag(mu, 1)).max() < 1e-12
        assert np.abs(ng[:, mu] - g @ n[:, mu] @ shifted_dag(mu, 3)).max() < 1e-13
        assert np.abs(fatg[:, mu] - g @ fat[:, mu] @ shifted_dag(mu, 1)).max() < 1e-12
        assert np.abs(lngg[:, mu] - g @ lng[:, mu] @ shifted_dag(mu, 3)).max() < 1e-13
    # the polar factor is covariant on both sides: (g V h^+) -> g W h^+
    Vm = f.reshape(-1, 3, 3)
    h = synth.random_su3(Vm.shape[0], 10)
    gg = synth.random_su3(Vm.shape[0], 12)
    assert np.abs(oracle.unitarize(gg @ Vm @ _dag(h)) - gg @ oracle.unitarize(Vm) @ _dag(h)).max() < 1e-13


def test_translation_and_axis_permutation():
    d = (4, 4, 4, 4)
    U = synth.thin_links(d, 0.5, 13)
    c = _rng_coefs(14)
    out = oracle.fat7(d, U, c)
    U4 = U.reshape(4, 4, 4, 4, 4, 3, 3)
    o4 = out.reshape(U4.shape)
    # translation by (1, 2, 0, 3)
    sh = (-3, 0, -2, -1)
    t_out = oracle.fat7(d, np.roll(U4, sh, axis=(0, 1, 2, 3)).reshape(U.shape), c)
    assert np.abs(t_out - np.roll(o4, sh, axis=(0, 1, 2, 3)).reshape(U.shape)).max() < 1e-13
    # axis permutations: x'_{p[nu]} = x_nu and link direction mu -> p[mu]
    for p in [(2, 1, 0, 3), (1, 2, 3, 0), (3, 0, 2, 1)]:
        ax = [3 - p[3 - a] for a in range(4)]          # array axis of x_nu -> axis of x'_{p[nu]}
        inv = np.argsort(ax)
        Up = np.empty_like(U4)
        op = np.empty_like(o4)
        for mu in range(4):
            Up[..., p[mu], :, :] = np.transpose(U4[..., mu, :, :], list(inv) + [4, 5])
            op[..., p[mu], :, :] = np.transpose(o4[..., mu, :, :], list(inv) + [4, 5])
        got = oracle.fat7(d, Up.reshape(U.shape), c)
        assert np.abs(got - op.reshape(U.shape)).max() < 1e-13


def test_polar_factor_matches_svd():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((200, 3, 3)) + 1j * rng.standard_normal((200, 3, 3))
    W = oracle.unitarize(A)
    u, s, vh = np.linalg.svd(A)
    assert np.abs(W - u @ vh).max() < 1e-12
    assert np.abs(_dag(W) @ W - np.eye(3)).max() < 1e-14
    # on the level-1 smeared links of a realistic field
    d = (4, 4, 4, 6)
    v = oracle.fat7(d, synth.thin_links(d, 0.4, 4), oracle.HISQ_LEVEL1).reshape(-1, 3, 3)
    u, s, vh = np.linalg.svd(v)
    assert np.abs(oracle.unitarize(v) - u @ vh).max() < 1e-13
    # unitary input is a fixed point
    q = synth.random_su3(50, 2)
    assert np.abs(oracle.unitarize(q) - q).max() < 1e-15


def test_polar_iteration_reports_singular_input():
    A = np.zeros((3, 3, 3), dtype=np.complex128)
    A[0] = np.eye(3)
    A[1] = np.diag([1.0, 1.0, 0.0])       # singular
    A[2] = np.eye(3)
    with pytest.raises(ArithmeticError):
        oracle.unitarize(A)


def _staple(U, d, mu, nu, M):
    """sum over s = +-1 of the staple of field M (a link field in direction mu)
    through direction nu: U_nu(x) M(x+nu) U_nu(x+mu)^+ + U_nu(x-nu)^+ M(x-nu) U_nu(x-nu+mu)."""
    Un = U[:, nu]
    up = Un @ synth._shift(M, d, nu, 1) @ _dag(synth._shift(Un, d, mu, 1))
    Um = synth._shift(Un, d, nu, -1)
    dn = _dag(Um) @ synth._shift(M, d, nu, -1) @ synth._shift(synth._shift(Un, d, mu, 1), d, nu, -1)
    return up + dn


def test_nested_staple_recursion_equals_path_sum():
    # The 5- and 7-staples are staples of staples: building them by nesting the
    # one-step staple on whole fields (array shifts) must give the path sum.
    d = (4, 4, 6, 4)
    U = synth.thin_links(d, 0.5, 31)
    c = _rng_coefs(32)
    out = oracle.fat7(d, U, c)
    for mu in range(4):
        ref = c[0] * U[:, mu]
        perp = [nu for nu in range(4) if nu != mu]
        for nu in perp:
            s3 = _staple(U, d, mu, nu, U[:, mu])
            ref = ref + c[1] * s3
            # Lepage: the staple of the same-sign staple, per sign
            Un = U[:, nu]
            up = Un @ synth._shift(Un, d, nu, 1) @ synth._shift(U[:, mu], d, nu, 2) \
                @ _dag(synth._shift(synth._shift(Un, d, mu, 1), d, nu, 1)) @ _dag(synth._shift(Un, d, mu, 1))
            m1 = synth._shift(Un, d, nu, -1)
            m2 = synth._shift(Un, d, nu, -2)
            dn = _dag(m1) @ _dag(m2) @ synth._shift(U[:, mu], d, nu, -2) \
                @ synth._shift(m2, d, mu, 1) @ synth._shift(m1, d, mu, 1)
            ref = ref + c[4] * (up + dn)
            for rho in perp:
                if rho == nu:
                    continue
                s5 = _staple(U, d, mu, rho, s3)
                ref = ref + c[2] * s5
                sig = [x for x in perp if x not in (nu, rho)][0]
                ref = ref + c[3] * _staple(U, d, mu, sig, s5)
        assert np.abs(out[:, mu] - ref).max() < 1e-12


def test_hisq_smear_composition():
    d = (4, 4, 4, 6)
    U = synth.thin_links(d, 0.4, 33)
    fat, lng = oracle.hisq_smear(d, U)
    eta = synth.staggered_phases(d)[:, :, None, None]
    # the Naik links are products of three U(3) matrices
    n = -24.0 * eta * lng
    assert np.abs(_dag(n) @ n - np.eye(3)).max() < 1e-13
    # and the whole is the composition of the separately pinned stages
    W = oracle.unitarize(oracle.fat7(d, U, oracle.HISQ_LEVEL1))
    assert np.abs(fat - eta * oracle.fat7(d, W, oracle.HISQ_LEVEL2)).max() < 1e-14
    assert np.abs(lng + eta / 24 * oracle.naik_product(d, W)).max() < 1e-15
