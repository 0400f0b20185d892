"""Pins for the oracle's solvers and preconditioner network: dense LAPACK
solves, residual collinearity of the shifted systems, monotonicity in the
shift, special weight choices of the PTC layer that reduce to known operators,
gauge equivariance, and central finite differences for the adjoint."""
import numpy as np
import pytest

import oracle
from paper_1712_00143_amd import synth


def _dense_A(dims, fat, lng, m, sigma=0.0):
    h = synth.volume(dims) // 2
    I = np.eye(3 * h)
    return np.stack([oracle.apply_A(dims, fat, lng, m, I[j].reshape(h, 3), sigma).reshape(-1)
                     for j in range(3 * h)], axis=1)


@pytest.mark.parametrize("dims,eps,m", [((4, 4, 4, 4), 0.3, 0.1), ((2, 2, 2, 2), 0.3, 0.1),
                                        ((4, 4, 4, 4), 0.3, 0.02)])
def test_cg_matches_dense_solve(dims, eps, m):
    fat, lng = synth.make_links(dims, eps, seed=0)
    b = synth.gaussian_even(dims, 500)
    A = _dense_A(dims, fat, lng, m)
    xs = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
    x, it, tr, ok = oracle.cg(dims, fat, lng, m, b, tol=1e-10)
    assert ok and tr <= 1e-10
    lam = np.linalg.eigvalsh(A)
    kappa = lam.max() / lam.min()
    assert np.linalg.norm(x - xs) <= kappa * 1e-10 * np.linalg.norm(xs)
    assert np.linalg.norm(b.reshape(-1) - A @ x.reshape(-1)) <= 1e-10 * np.linalg.norm(b)


def test_cg_warm_start_and_sigma():
    dims = (4, 4, 4, 4)
    fat, lng = synth.make_links(dims, 0.3, seed=1)
    b = synth.gaussian_even(dims, 7)
    A = _dense_A(dims, fat, lng, 0.05, sigma=0.3)
    xs = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
    x, it, tr, ok = oracle.cg(dims, fat, lng, 0.05, b, tol=1e-12, sigma=0.3, x0=0.9 * xs)
    assert ok and np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_multishift_matches_dense_solves():
    dims = (4, 4, 4, 4)
    fat, lng = synth.make_links(dims, 0.2, seed=2000)
    m = 0.01
    shifts = synth.shifts_log(12)
    b = synth.gaussian_even(dims, 2500)
    x, iters, rel, ok = oracle.multishift(dims, fat, lng, m, shifts, b, tol=1e-8)
    assert ok
    A0 = _dense_A(dims, fat, lng, m)
    I = np.eye(A0.shape[0])
    norms = []
    for k, s in enumerate(shifts):
        xs = np.linalg.solve(A0 + s * I, b.reshape(-1))
        lam = np.linalg.eigvalsh(A0 + s * I)
        assert rel[k] <= 1e-8
        assert np.linalg.norm(x[k].reshape(-1) - xs) <= lam.max() / lam.min() * 1e-8 * np.linalg.norm(xs)
        norms.append(np.linalg.norm(x[k]))
    assert all(a > b_ for a, b_ in zip(norms, norms[1:]))       # ||x_k|| decreases with sigma_k
    # larger shifts converge in fewer Krylov iterations
    assert iters[-1] < iters[0]


def test_multishift_residuals_collinear():
    """Before refinement the shifted residuals b - (A+s_k) x_k are parallel to
    the base residual (checked after a fixed small number of iterations)."""
    dims = (4, 4, 4, 4)
    fat, lng = synth.make_links(dims, 0.3, seed=3)
    m = 0.1
    shifts = np.array([0.01, 0.1, 0.5])
    b = synth.gaussian_even(dims, 4)
    x, iters, rel, ok = oracle.multishift(dims, fat, lng, m, shifts, b, tol=1e-3, maxiter=6)
    res = [b - oracle.apply_A(dims, fat, lng, m, x[k], shifts[k]) for k in range(3)]
    # refinement may have run for shifts that missed tol; skip those
    for k in range(1, 3):
        if iters[k] == iters[0]:
            c = np.vdot(res[0], res[k]) / np.vdot(res[0], res[0])
            assert np.linalg.norm(res[k] - c * res[0]) <= 1e-8 * np.linalg.norm(res[k])


def test_fcg_identity_matches_dense():
    dims = (4, 4, 4, 4)
    fat, lng = synth.make_links(dims, 0.3, seed=0)
    b = synth.gaussian_even(dims, 500)
    m = 0.1
    xs = np.linalg.solve(_dense_A(dims, fat, lng, m), b.reshape(-1)).reshape(b.shape)
    x, it, tr, ok = oracle.fcg(dims, fat, lng, m, None, b)
    assert ok and tr <= 1e-10
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    # with the identity preconditioner FCG(1) is CG: same iteration count
    _, it_cg, _, _ = oracle.cg(dims, fat, lng, m, b)
    assert abs(it - it_cg) <= 1


def _rand_weights(chans, seed, scale=0.1, ident=True):
    rng = np.random.default_rng(seed)
    ws = []
    for cin, cout in zip(chans[:-1], chans[1:]):
        w = scale * (rng.standard_normal((cout, cin, 9)) + 1j * rng.standard_normal((cout, cin, 9)))
        if ident:
            w[:, :, 0] += 1.0 / cin
        ws.append(w)
    return ws


def test_fcg_with_network_converges():
    dims = (4, 4, 4, 4)
    fat, lng = synth.make_links(dims, 0.3, seed=5)
    b = synth.gaussian_even(dims, 6)
    m = 0.1
    xs = np.linalg.solve(_dense_A(dims, fat, lng, m), b.reshape(-1)).reshape(b.shape)
    ws = _rand_weights([1, 4, 4, 1], 1, scale=0.02)
    x, it, tr, ok = oracle.fcg(dims, fat, lng, m, ws, b)
    assert ok and tr <= 1e-10
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_ptc_identity_and_one_hop_dslash():
    dims = (4, 4, 6, 4)
    fat, lng = synth.make_links(dims, 0.3, seed=8)
    psi = synth.gaussian_full(dims, 9, 2)
    w = np.zeros((2, 2, 9), complex)
    w[0, 0, 0] = w[1, 1, 0] = 1.0
    assert np.abs(oracle.ptc_layer(dims, fat, w, psi) - psi).max() == 0.0
    # w_{+mu} = 1, w_{-mu} = -1: the one-hop part of D
    w1 = np.zeros((1, 1, 9), complex)
    w1[0, 0, 1::2] = 1.0
    w1[0, 0, 2::2] = -1.0
    out = oracle.ptc_layer(dims, fat, w1, psi[:1])[0]
    ref = oracle.dslash_full(dims, fat, np.zeros_like(lng), psi[0])
    assert np.linalg.norm(out - ref) <= 1e-14 * np.linalg.norm(ref)


def test_ptc_gauge_equivariance():
    dims = (4, 4, 4, 6)
    fat, _ = synth.make_links(dims, 0.3, seed=10)
    V = synth.volume(dims)
    G = synth.random_su3(V, seed=11)
    fat2 = np.empty_like(fat)
    for mu in range(4):
        fat2[:, mu] = G @ fat[:, mu] @ np.conj(np.swapaxes(synth._shift(G, dims, mu, 1), -1, -2))
    ws = _rand_weights([2, 3], 12, scale=1.0)[0]
    psi = synth.gaussian_full(dims, 13, 2)
    out = oracle.ptc_layer(dims, fat, ws, psi)
    out2 = oracle.ptc_layer(dims, fat2, ws, np.einsum("sij,csj->csi", G, psi))
    ref = np.einsum("sij,csj->csi", G, out)
    assert np.linalg.norm(out2 - ref) <= 1e-13 * np.linalg.norm(ref)


def test_ptc_adjoint_identity():
    """<g, L(a)> = <L^+(g), a> (the input gradient is the exact adjoint)."""
    dims = (4, 6, 4, 4)
    fat, _ = synth.make_links(dims, 0.3, seed=14)
    w = _rand_weights([3, 2], 15, scale=1.0)[0]
    a = synth.gaussian_full(dims, 16, 3)
    g = synth.gaussian_full(dims, 17, 2)
    gin, _ = oracle.ptc_layer_adj(dims, fat, w, a, g)
    lhs = np.vdot(g, oracle.ptc_layer(dims, fat, w, a))
    rhs = np.vdot(gin, a)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_ptc_loss_gradient_finite_differences():
    dims = (4, 4, 4, 4)
    fat, lng = synth.make_links(dims, 0.25, seed=18)
    h = synth.volume(dims) // 2
    ws = _rand_weights([1, 2, 2, 1], 19, scale=0.3)
    rs = [synth.gaussian_even(dims, 20 + i) for i in range(2)]
    es = [synth.gaussian_even(dims, 30 + i) for i in range(2)]
    loss, grads = oracle.ptc_loss_and_grad(dims, fat, ws, rs, es)
    rng = np.random.default_rng(0)
    hstep = 1e-6
    for trial in range(6):
        l = int(rng.integers(0, 3))
        idx = tuple(int(rng.integers(0, s)) for s in ws[l].shape)
        for part, unit in ((0, 1.0), (1, 1j)):
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += hstep * unit
            wm[l][idx] -= hstep * unit
            lp, _ = oracle.ptc_loss_and_grad(dims, fat, wp, rs, es)
            lm, _ = oracle.ptc_loss_and_grad(dims, fat, wm, rs, es)
            fd = (lp - lm) / (2 * hstep)
            an = grads[l][idx].real if part == 0 else grads[l][idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, idx, part, fd, an)


def test_ptc_energy_loss_is_the_energy_norm_misfit_and_its_gradient():
    """The energy-norm loss equals its definition, min over one complex c of
    sum_b |e_b - c z_b|_A^2 / |e_b|_A^2 divided by B, with the A-norms formed
    from the operator and c found by a numerical minimiser; and its gradient
    matches central finite differences."""
    from scipy.optimize import minimize
    dims = (4, 4, 4, 4)
    m = 0.1
    fat, lng = synth.make_links(dims, 0.25, seed=18)
    ws = _rand_weights([1, 2, 2, 1], 19, scale=0.3)
    es = [synth.gaussian_even(dims, 30 + i) for i in range(3)]
    rs = [oracle.apply_A(dims, fat, lng, m, e) for e in es]
    loss, grads = oracle.ptc_loss_and_grad(dims, fat, ws, rs, es, energy=(lng, m))
    zs = [oracle.ptc_apply(dims, fat, ws, r) for r in rs]

    Aes = [oracle.apply_A(dims, fat, lng, m, e) for e in es]
    Azs = [oracle.apply_A(dims, fat, lng, m, z) for z in zs]

    def misfit(c):   # |e - c z|_A^2 = <e - c z, A e - c A z> (A linear)
        cc = c[0] + 1j * c[1]
        return sum(float(np.vdot(e - cc * z, ae - cc * az).real) / float(np.vdot(e, ae).real)
                   for e, z, ae, az in zip(es, zs, Aes, Azs)) / len(es)

    best = minimize(misfit, [0.1, 0.0], method="Nelder-Mead", options={"xatol": 1e-10, "fatol": 1e-14})
    assert 0.0 < loss < 1.0
    assert abs(best.fun - loss) <= 1e-8, (best.fun, loss)
    rng = np.random.default_rng(3)
    hstep = 1e-6
    for trial in range(4):
        l = int(rng.integers(0, 3))
        idx = tuple(int(rng.integers(0, s)) for s in ws[l].shape)
        for part, unit in ((0, 1.0), (1, 1j)):
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += hstep * unit
            wm[l][idx] -= hstep * unit
            lp, _ = oracle.ptc_loss_and_grad(dims, fat, wp, rs, es, energy=(lng, m))
            lm, _ = oracle.ptc_loss_and_grad(dims, fat, wm, rs, es, energy=(lng, m))
            fd = (lp - lm) / (2 * hstep)
            an = grads[l][idx].real if part == 0 else grads[l][idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, idx, part, fd, an)


def test_ptc_network_is_hermitian_psd_and_adjoint_weights():
    """M = E^+ K^+ K E is Hermitian and positive semidefinite, and the layer
    with adjoint_weights(W) is the adjoint layer of W."""
    dims = (4, 4, 4, 6)
    fat, _ = synth.make_links(dims, 0.25, seed=44)
    ws = _rand_weights([1, 3, 2], 45, scale=0.7, ident=False)
    u = synth.gaussian_even(dims, 46)
    v = synth.gaussian_even(dims, 47)
    Mu = oracle.ptc_apply(dims, fat, ws, u)
    Mv = oracle.ptc_apply(dims, fat, ws, v)
    assert abs(np.vdot(u, Mv) - np.vdot(Mu, v)) <= 1e-12 * abs(np.vdot(u, Mv))
    assert np.vdot(v, Mv).real > 0 and abs(np.vdot(v, Mv).imag) <= 1e-12 * abs(np.vdot(v, Mv))
    g = synth.gaussian_full(dims, 48, 3)
    a = oracle.ptc_layer_adjoint(dims, fat, ws[0], g)
    b = oracle.ptc_layer(dims, fat, oracle.adjoint_weights(ws[0]), g)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


def test_ptc_loss_scale_invariance_and_exact_target():
    """The loss depends only on the direction of M(r) relative to the target:
    it is unchanged when the target is scaled by a complex number, vanishes
    when the target is a multiple of M(r), and equals 1 when the target is
    orthogonal to M(r).  With zero weights M is the identity."""
    dims = (4, 4, 4, 4)
    fat, _ = synth.make_links(dims, 0.25, seed=40)
    ws = _rand_weights([1, 2, 1], 41, scale=0.5)
    r = synth.gaussian_even(dims, 42)
    e = synth.gaussian_even(dims, 43)
    l0, g0 = oracle.ptc_loss_and_grad(dims, fat, ws, [r], [e])
    l1, _ = oracle.ptc_loss_and_grad(dims, fat, ws, [r], [(2.0 - 1.5j) * e])
    assert 0.0 < l0 < 1.0 and abs(l0 - l1) < 1e-14
    zero = [np.zeros_like(w) for w in ws]
    assert np.array_equal(oracle.ptc_apply(dims, fat, zero, r), r)
    z = oracle.ptc_apply(dims, fat, ws, r)
    lz, gz = oracle.ptc_loss_and_grad(dims, fat, ws, [r], [(0.3 + 0.7j) * z])
    assert abs(lz) < 1e-14 and max(np.abs(g).max() for g in gz) < 1e-10
    ortho = e - np.vdot(z, e) / np.vdot(z, z) * z
    lo, _ = oracle.ptc_loss_and_grad(dims, fat, ws, [r], [ortho])
    assert abs(lo - 1.0) < 1e-12


def test_adam_first_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2, so the update is
    -lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = oracle.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-2)
    assert np.allclose(p1, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # constant gradient: every step moves by ~lr * sign(g)
    q, m, v = p.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 20):
        q, m, v = oracle.adam_step(q, g, m, v, t, lr=1e-3)
    assert np.allclose(q, p - 19e-3 * np.sign(g), atol=1e-9)


def _poly_weights(chans, a, lam):
    """K = a (1 + D_f^2 / lam): r and D_f r in channels 0 and 1, one more hop
    on channel 1, then a * ch0 + (a / lam) * ch1 (the last layer takes the
    second hop itself when there are only two layers)."""
    hop = np.zeros(9, complex)
    hop[1::2], hop[2::2] = 1.0, -1.0
    ws = []
    n = len(chans) - 1
    for l, (ci, co) in enumerate(zip(chans[:-1], chans[1:])):
        w = np.zeros((co, ci, 9), complex)
        if l == 0:
            w[0, 0, 0] = 1.0
            w[1, 0] = hop
        elif l < n - 1:
            w[0, 0, 0] = 1.0
            w[1, 1] = hop if l == 1 else np.eye(1, 9, 0)[0]
        if l == n - 1:
            w[0, 0, 0] = a
            w[0, 1] = hop * (a / lam) if l == 1 else np.eye(1, 9, 0)[0] * (a / lam)
        ws.append(w)
    return ws


@pytest.mark.parametrize("chans", [(1, 4, 4, 1), (1, 2, 1), (1, 2, 2, 2, 1)])
def test_ptc_polynomial_weights_free_field_closed_form(chans):
    """Free field: D_f^2 = sum_mu nabla_mu^2 with nabla = T - T^-1, so an
    even-site plane wave of momentum p is an eigenvector of -D_f^2 with
    t = 4 sum_mu sin^2 p_mu, and the network with the polynomial weights gives
    M = 1 + a^2 (1 - t / lam)^2 on it."""
    dims = (4, 6, 4, 8)
    fat, _ = synth.unit_links(dims)
    x = synth.coords(dims)[synth.even_sites(dims)]
    chi = np.array([0.3 - 0.2j, 1.0, -0.5j])
    a, lam = 3.0, 16.0
    ws = _poly_weights(chans, a, lam)
    for n in [(1, 2, 1, 3), (0, 0, 0, 0), (2, 3, 2, 4), (1, 0, 3, 5)]:
        p = 2 * np.pi * np.array(n) / np.array(dims)
        v = np.exp(1j * (x @ p))[:, None] * chi[None, :]
        t = 4 * np.sum(np.sin(p) ** 2)
        z = oracle.ptc_apply(dims, fat, ws, v)
        ref = (1.0 + a * a * (1.0 - t / lam) ** 2) * v
        assert np.linalg.norm(z - ref) <= 1e-13 * np.linalg.norm(ref), (chans, n)
