"""FP64 CPU oracle for the HISQ even-odd Dslash, CG, multi-shift CG, PTC
preconditioner, flexible CG and HISQ link smearing.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  It shares no code with the
HIP path.  The arithmetic lives in ``hisq_oracle.c`` (plain C, OpenMP over
sites); this module marshals numpy arrays into it and adds the plain Adam
step used to check the optimiser kernel.

Every function pins to something outside itself in ``tests/test_oracle_*.py``
(anti-Hermiticity, free-field closed form, gauge covariance, dense solves,
finite differences).  The one exception is noted where it occurs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hisq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
    return _lib


_IA4 = ctypes.c_int * 4


def _dims(dims):
    return _IA4(*[int(x) for x in dims])


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _links(fat, lng):
    f, fp = _c(fat)
    l, lp = _c(lng)
    return (f, l), fp, lp


def dslash_full(dims, fat, lng, psi):
    """D psi on the full lattice; psi [V][3] -> [V][3]."""
    lib = _load()
    keep, fp, lp = _links(fat, lng)
    a, ap = _c(psi)
    out = np.empty_like(a)
    lib.orc_dslash_full(_dims(dims), fp, lp, ap, out.ctypes.data_as(ctypes.c_void_p))
    return out


def dslash_half(dims, fat, lng, out_parity, psi_half):
    """D_eo (out_parity 0) or D_oe (1) on half vectors [V/2][3]."""
    lib = _load()
    keep, fp, lp = _links(fat, lng)
    a, ap = _c(psi_half)
    out = np.empty_like(a)
    lib.orc_dslash_half(_dims(dims), fp, lp, ctypes.c_int(out_parity), ap,
                        out.ctypes.data_as(ctypes.c_void_p))
    return out


def apply_A(dims, fat, lng, mass, psi_even, sigma=0.0):
    """(4 m^2 + sigma - D_eo D_oe) psi on even vectors."""
    lib = _load()
    keep, fp, lp = _links(fat, lng)
    a, ap = _c(psi_even)
    out = np.empty_like(a)
    lib.orc_apply_A(_dims(dims), fp, lp, ctypes.c_double(mass), ctypes.c_double(sigma), ap,
                    out.ctypes.data_as(ctypes.c_void_p))
    return out


def true_residual(dims, fat, lng, mass, b, x, sigma=0.0):
    """||b - (A + sigma) x|| / ||b|| in FP64."""
    lib = _load()
    lib.orc_true_residual.restype = ctypes.c_double
    keep, fp, lp = _links(fat, lng)
    bb, bp = _c(b)
    xx, xp = _c(x)
    return lib.orc_true_residual(_dims(dims), fp, lp, ctypes.c_double(mass),
                                 ctypes.c_double(sigma), bp, xp)


def cg(dims, fat, lng, mass, b, tol=1e-10, maxiter=100000, sigma=0.0, x0=None):
    """Returns (x, iterations, true relative residual, converged)."""
    lib = _load()
    keep, fp, lp = _links(fat, lng)
    bb, bp = _c(b)
    x = np.zeros_like(bb) if x0 is None else np.array(x0, dtype=np.complex128, copy=True)
    it = ctypes.c_int(0)
    tr = ctypes.c_double(0)
    rc = lib.orc_cg(_dims(dims), fp, lp, ctypes.c_double(mass), ctypes.c_double(sigma), bp,
                    x.ctypes.data_as(ctypes.c_void_p), ctypes.c_double(tol),
                    ctypes.c_int(maxiter), ctypes.byref(it), ctypes.byref(tr))
    return x, it.value, tr.value, rc == 0


def multishift(dims, fat, lng, mass, shifts, b, tol=1e-8, maxiter=100000):
    """Returns (x [nshift][h][3], iters[nshift], rel[nshift], converged)."""
    lib = _load()
    keep, fp, lp = _links(fat, lng)
    bb, bp = _c(b)
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    ns = len(shifts)
    x = np.zeros((ns,) + bb.shape, dtype=np.complex128)
    iters = np.zeros(ns, dtype=np.int32)
    rel = np.zeros(ns)
    rc = lib.orc_multishift(_dims(dims), fp, lp, ctypes.c_double(mass), ctypes.c_int(ns),
                            shifts.ctypes.data_as(ctypes.c_void_p), bp,
                            x.ctypes.data_as(ctypes.c_void_p), ctypes.c_double(tol),
                            ctypes.c_int(maxiter), iters.ctypes.data_as(ctypes.c_void_p),
                            rel.ctypes.data_as(ctypes.c_void_p))
    return x, iters, rel, rc == 0


def ptc_layer(dims, fat, w, act):
    """One PTC layer: w [cout][cin][9], act [cin][V][3] -> [cout][V][3]."""
    lib = _load()
    f, fp = _c(fat)
    w, wp = _c(w)
    a, ap = _c(act)
    cout, cin = w.shape[0], w.shape[1]
    out = np.empty((cout,) + a.shape[1:], dtype=np.complex128)
    lib.orc_ptc_layer(_dims(dims), fp, ctypes.c_int(cin), ctypes.c_int(cout), wp, ap,
                      out.ctypes.data_as(ctypes.c_void_p))
    return out


def ptc_layer_adj(dims, fat, w, act, gout, need_gin=True):
    """(g_in or None, g_w) of one PTC layer for output gradient gout."""
    lib = _load()
    f, fp = _c(fat)
    w, wp = _c(w)
    a, ap = _c(act)
    g, gp = _c(gout)
    cout, cin = w.shape[0], w.shape[1]
    gw = np.empty_like(w)
    gin = np.empty_like(a) if need_gin else None
    lib.orc_ptc_layer_adj(_dims(dims), fp, ctypes.c_int(cin), ctypes.c_int(cout), wp, ap, gp,
                          gin.ctypes.data_as(ctypes.c_void_p) if need_gin else None,
                          gw.ctypes.data_as(ctypes.c_void_p))
    return gin, gw


def _flat_weights(weights):
    return np.concatenate([np.ascontiguousarray(w, dtype=np.complex128).ravel()
                           for w in weights])


def ptc_apply(dims, fat, weights, r_even):
    """z = M(r): even embed -> layers -> even projection.  weights: list of
    [cout][cin][9] arrays."""
    lib = _load()
    f, fp = _c(fat)
    chans = np.array([weights[0].shape[1]] + [w.shape[0] for w in weights], dtype=np.int32)
    wf = _flat_weights(weights)
    r, rp = _c(r_even)
    z = np.empty_like(r)
    lib.orc_ptc_apply(_dims(dims), fp, ctypes.c_int(len(weights)),
                      chans.ctypes.data_as(ctypes.c_void_p),
                      wf.ctypes.data_as(ctypes.c_void_p), rp,
                      z.ctypes.data_as(ctypes.c_void_p))
    return z


def fcg(dims, fat, lng, mass, weights, b, tol=1e-10, maxiter=100000):
    """Flexible CG with the PTC network as preconditioner (weights=None: the
    identity).  Returns (x, iterations, true relative residual, converged)."""
    lib = _load()
    keep, fp, lp = _links(fat, lng)
    bb, bp = _c(b)
    x = np.zeros_like(bb)
    it = ctypes.c_int(0)
    tr = ctypes.c_double(0)
    if weights:
        chans = np.array([weights[0].shape[1]] + [w.shape[0] for w in weights], dtype=np.int32)
        wf = _flat_weights(weights)
        nl, cp, wp = len(weights), chans.ctypes.data_as(ctypes.c_void_p), \
            wf.ctypes.data_as(ctypes.c_void_p)
    else:
        nl, cp, wp = 0, None, None
    rc = lib.orc_fcg(_dims(dims), fp, lp, ctypes.c_double(mass), ctypes.c_int(nl), cp, wp,
                     bp, x.ctypes.data_as(ctypes.c_void_p), ctypes.c_double(tol),
                     ctypes.c_int(maxiter), ctypes.byref(it), ctypes.byref(tr))
    return x, it.value, tr.value, rc == 0


def ptc_layer_adjoint(dims, fat, w, g):
    """L^+ g for the layer with weights w ([cout][cin][9]): [cout][V][3] -> [cin][V][3]."""
    lib = _load()
    f, fp = _c(fat)
    w, wp = _c(w)
    gg, gp = _c(g)
    cout, cin = w.shape[0], w.shape[1]
    gin = np.empty((cin,) + gg.shape[1:], dtype=np.complex128)
    lib.orc_ptc_layer_adj(_dims(dims), fp, ctypes.c_int(cin), ctypes.c_int(cout), wp, None, gp,
                          gin.ctypes.data_as(ctypes.c_void_p), None)
    return gin


def adjoint_weights(w):
    """Weights of L^+ for the layer with weights w: W'[c'][c][k'] = conj(W[c][c'][k]),
    k' the reversed path (identity stays, +mu <-> -mu)."""
    perm = [0] + [k + 1 if (k - 1) % 2 == 0 else k - 1 for k in range(1, 9)]
    return np.conj(np.transpose(w, (1, 0, 2))[:, :, perm])


def ptc_loss_and_grad(dims, fat, weights, r_even_batch, e_even_batch, energy=None):
    """Loss of a batch of (residual, error) pairs for z_i = M(r_i),
    M = 1 + E^+ K^+ K E (K the layer stack):
        L = 1 - |S|^2 / (B Q),  S = sum_i <z_i, e_i> / |e_i|^2,
                                Q = sum_i |z_i|^2 / |e_i|^2,
    i.e. min_c sum_i |z_i - c e_i|^2 / |e_i|^2, normalised by sum_i |z_i|^2/|e_i|^2:
    it asks for one common c with M A e_i = M r_i ~ c e_i on every pair (M A
    close to a multiple of 1) and is invariant to the scale of M, which the
    flexible CG does not see.  Gradient (dL/dRe z + i dL/dIm z):
        g_i = -2 (conj(S) e_i Q - |S|^2 z_i) / (B Q^2 |e_i|^2).
    Weight gradients follow by the layer adjoints; the adjoint half uses the
    weights W' = adjoint_weights(W), and a gradient G' with respect to W'
    contributes adjoint_weights(G') to that of W.

    energy = (lng, mass): the same misfit in the energy norm of A instead,
    min_c sum_i |e_i - c z_i|_A^2 / |e_i|_A^2 with |v|_A^2 = <v, A v> -- the
    norm CG minimises.  With A e_i = r_i and w_i = <e_i, r_i>:
        S = sum_i <z_i, r_i> / w_i,  Q = sum_i <z_i, A z_i> / w_i,
        L = 1 - |S|^2 / (B Q),
        g_i = -2 (conj(S) r_i Q - |S|^2 A z_i) / (B Q^2 w_i)."""
    V = int(np.prod(dims))
    nl = len(weights)
    even = _even_lex(dims)
    grads = [np.zeros_like(w, dtype=np.complex128) for w in weights]
    wadj = [adjoint_weights(w) for w in weights]
    npair = len(r_even_batch)
    fwd = []
    S, Q = 0j, 0.0
    for r, e in zip(r_even_batch, e_even_batch):
        a = np.zeros((1, V, 3), dtype=np.complex128)
        a[0, even] = r
        acts = [a]
        for w in weights:
            acts.append(ptc_layer(dims, fat, w, acts[-1]))
        bs = [None] * (nl + 1)
        bs[nl] = acts[nl]
        for l in range(nl, 0, -1):
            bs[l - 1] = ptc_layer(dims, fat, wadj[l - 1], bs[l])
        z = r + bs[0][0, even]          # M = 1 + E^+ K^+ K E
        if energy is None:
            t, zw, ee = e, z, float(np.vdot(e, e).real)
        else:
            t, zw, ee = r, apply_A(dims, fat, energy[0], energy[1], z), float(np.vdot(e, r).real)
        S += np.vdot(z, t) / ee
        Q += float(np.vdot(z, zw).real) / ee
        fwd.append((acts, bs, zw, t, ee))
    loss = 1.0 - abs(S) ** 2 / (npair * Q)
    for acts, bs, zw, t, ee in fwd:
        g = np.zeros((1, V, 3), dtype=np.complex128)
        g[0, even] = -2.0 * (np.conj(S) * t * Q - abs(S) ** 2 * zw) / (npair * Q * Q * ee)
        # adjoint half, in reverse order of application
        for l in range(1, nl + 1):
            gin, gw = ptc_layer_adj(dims, fat, wadj[l - 1], bs[l], g)
            grads[l - 1] += adjoint_weights(gw)
            g = gin
        # forward half
        for l in range(nl - 1, -1, -1):
            gin, gw = ptc_layer_adj(dims, fat, weights[l], acts[l], g, need_gin=(l > 0))
            grads[l] += gw
            g = gin
    return loss, grads


def _even_lex(dims):
    L0, L1, L2, L3 = dims
    t, z, y, x = np.meshgrid(np.arange(L3), np.arange(L2), np.arange(L1), np.arange(L0),
                             indexing="ij")
    par = ((x + y + z + t) % 2).reshape(-1)
    return np.nonzero(par == 0)[0]


def adam_step(param, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015) on real arrays; step counts from 1.  Returns the
    new (param, m, v).  Complex parameters are handled as (Re, Im) pairs by the
    caller."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ------------------------------------------------------------- link smearing

HISQ_LEVEL1 = (1 / 8, 1 / 16, 1 / 64, 1 / 384, 0.0)
HISQ_LEVEL2 = (5 / 8, 1 / 16, 1 / 64, 1 / 384, -1 / 16)


def fat7(dims, links, coefs):
    """Path-sum smearing of links [V][4][3][3] with coefs (c1, c3, c5, c7,
    cLepage): one-link, 3-, 5-, 7-staples and Lepage paths, summed path by
    path (hisq_oracle.c states the path list)."""
    lib = _load()
    u, up = _c(links)
    c = (ctypes.c_double * 5)(*[float(x) for x in coefs])
    out = np.empty_like(u)
    lib.orc_fat7(_dims(dims), c, up, out.ctypes.data_as(ctypes.c_void_p))
    return out


def unitarize(mats):
    """Unitary polar factor V (V^+ V)^{-1/2} of every 3x3 in mats [..., 3, 3]
    (Newton iteration).  Raises if any matrix does not converge."""
    lib = _load()
    m, mp = _c(mats)
    out = np.empty_like(m)
    n = m.size // 9
    lib.orc_unitarize.restype = ctypes.c_int
    bad = lib.orc_unitarize(ctypes.c_long(n), mp, out.ctypes.data_as(ctypes.c_void_p))
    if bad:
        raise ArithmeticError(f"polar iteration did not converge for {bad} matrices")
    return out


def naik_product(dims, links):
    """W_mu(x) W_mu(x+mu) W_mu(x+2mu) for every site and direction."""
    lib = _load()
    u, up = _c(links)
    out = np.empty_like(u)
    lib.orc_naik_product(_dims(dims), up, out.ctypes.data_as(ctypes.c_void_p))
    return out


def hisq_smear(dims, thin):
    """(fat, long) HISQ links, phases folded, from thin SU(3) links."""
    lib = _load()
    u, up = _c(thin)
    fat = np.empty_like(u)
    lng = np.empty_like(u)
    lib.orc_hisq_smear.restype = ctypes.c_int
    bad = lib.orc_hisq_smear(_dims(dims), up, fat.ctypes.data_as(ctypes.c_void_p),
                             lng.ctypes.data_as(ctypes.c_void_p))
    if bad:
        raise ArithmeticError(f"polar iteration did not converge for {bad} links")
    return fat, lng


# --------------------------------------------------------------- gauge force

def gauge_force(dims, links, beta, coefs):
    """Symanzik gauge force F [V][4][3][3] (traceless anti-Hermitian) of thin
    links; coefs = (plaquette, rectangle, parallelogram) weights."""
    lib = _load()
    u, up = _c(links)
    c = (ctypes.c_double * 3)(*[float(x) for x in coefs])
    out = np.empty_like(u)
    lib.orc_gauge_force.restype = ctypes.c_int
    if lib.orc_gauge_force(_dims(dims), up, ctypes.c_double(beta), c, out.ctypes.data_as(ctypes.c_void_p)):
        raise ValueError("the gauge force needs every extent >= 4")
    return out


def gauge_action(dims, links, beta, coefs):
    """S = beta sum_loops c (1 - Re Tr U_loop / 3)."""
    lib = _load()
    u, up = _c(links)
    c = (ctypes.c_double * 3)(*[float(x) for x in coefs])
    lib.orc_gauge_action.restype = ctypes.c_double
    s = lib.orc_gauge_action(_dims(dims), up, ctypes.c_double(beta), c)
    if np.isnan(s):
        raise ValueError("the gauge action needs every extent >= 4")
    return float(s)


# ------------------------------------------------------------- fermion force
#
# Q(U) = sum_k alpha_k X_k^+ A X_k, A = 4 m^2 - D_eo D_oe on the links
# smeared from the thin links U, for fixed even vectors X_k (in the RHMD step
# the multi-shift solutions X_k = (A + sigma_k)^-1 Phi; the pseudofermion
# action's derivative is then -dQ).  The force is F_mu(x) = TA[U_mu(x)
# G_mu(x)] with G the gradient dQ = sum Re Tr(dU_mu(x) G_mu(x)), so that
# U_mu(x) -> exp(eps X) U_mu(x), X in su(3), changes Q at the rate
# Re Tr(X F_mu(x)).


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def _shift_sites(field, dims, mu, k):
    L0, L1, L2, L3 = dims
    f = field.reshape((L3, L2, L1, L0) + field.shape[1:])
    return np.roll(f, -k, axis=3 - mu).reshape(field.shape)


def fermion_force_links(dims, fat, lng, alphas, xs):
    """Gradients (OF, OL) [V][4][3][3] of Q with respect to the (phased) fat
    and long links: dQ = sum Re Tr(dF_mu(x) OF_mu(x) + dL_mu(x) OL_mu(x)).
    With Y = D_oe X on odd sites and Psi = (X, Y), eps(x) = +1 (-1) on even
    (odd) sites, dQ = -sum_k alpha_k (Psi'^+ dD Psi), Psi' = eps Psi, so
      OF_mu(x) = -2 eps(x) sum_k alpha_k Psi_k(x+mu) Psi_k(x)^+
      OL_mu(x) = -2 eps(x) sum_k alpha_k Psi_k(x+3mu) Psi_k(x)^+."""
    V = int(np.prod(dims))
    c = np.stack(np.meshgrid(*[np.arange(n) for n in dims[::-1]], indexing="ij")[::-1], -1).reshape(-1, 4)
    par = c.sum(axis=1) % 2
    eps = np.where(par == 0, 1.0, -1.0)
    OF = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    OL = np.zeros_like(OF)
    for a, x in zip(alphas, xs):
        y = dslash_half(dims, fat, lng, 1, x)
        psi = np.zeros((V, 3), dtype=np.complex128)
        psi[par == 0] = x
        psi[par == 1] = y
        for mu in range(4):
            p1 = _shift_sites(psi, dims, mu, 1)
            p3 = _shift_sites(psi, dims, mu, 3)
            OF[:, mu] += -2.0 * a * eps[:, None, None] * (p1[:, :, None] * np.conj(psi)[:, None, :])
            OL[:, mu] += -2.0 * a * eps[:, None, None] * (p3[:, :, None] * np.conj(psi)[:, None, :])
    return OF, OL


def fat7_adjoint(dims, links, coefs, G):
    """Gradient with respect to links of sum Re Tr(fat7(links)_mu(x) G_mu(x))."""
    lib = _load()
    u, up = _c(links)
    g, gp = _c(G)
    c = (ctypes.c_double * 5)(*[float(x) for x in coefs])
    out = np.zeros_like(u)
    lib.orc_fat7_adjoint(_dims(dims), c, up, gp, out.ctypes.data_as(ctypes.c_void_p))
    return out


def naik_adjoint(dims, links, G):
    """Gradient with respect to W of sum Re Tr(N_mu(x) G_mu(x)), N = W W W."""
    lib = _load()
    u, up = _c(links)
    g, gp = _c(G)
    out = np.zeros_like(u)
    lib.orc_naik_adjoint(_dims(dims), up, gp, out.ctypes.data_as(ctypes.c_void_p))
    return out


def unitarize_adjoint(V, G):
    """Gradient with respect to V of Re Tr(W(V) G), W = V (V^+ V)^{-1/2}, from
    the singular values: V = A S B^+, W = A B^+, dW = A Om B^+ with
    Om_ij = (K_ij - conj(K_ji)) / (s_i + s_j), K = A^+ dV B; so the gradient
    is B M A^+ with M = (C - C^+) / (s_i + s_j), C = B^+ G A."""
    a, s, bh = np.linalg.svd(V)
    C = bh @ G @ a
    M = (C - _dag(C)) / (s[..., :, None] + s[..., None, :])
    return _dag(bh) @ M @ _dag(a)


def _ta(M):
    A = 0.5 * (M - _dag(M))
    return A - np.trace(A, axis1=-2, axis2=-1)[..., None, None] / 3.0 * np.eye(3)


def hisq_fermion_force(dims, thin, alphas, xs):
    """F_mu(x) = TA[U_mu(x) G_mu(x)] (see above) for thin links U, weights
    alphas and even vectors xs: the chain rule through the Naik product, the
    second fat7 level, the U(3) projection and the first fat7 level."""
    Vl = fat7(dims, thin, HISQ_LEVEL1)
    W = unitarize(Vl)
    fat, lng = hisq_smear(dims, thin)
    OF, OL = fermion_force_links(dims, fat, lng, alphas, xs)
    eta = np.ones((int(np.prod(dims)), 4))
    c = np.stack(np.meshgrid(*[np.arange(n) for n in dims[::-1]], indexing="ij")[::-1], -1).reshape(-1, 4)
    for mu in range(1, 4):
        eta[:, mu] = (-1.0) ** (c[:, :mu].sum(axis=1) % 2)
    GX = eta[:, :, None, None] * OF
    GN = -eta[:, :, None, None] / 24.0 * OL
    GW = fat7_adjoint(dims, W, HISQ_LEVEL2, GX) + naik_adjoint(dims, W, GN)
    GV = unitarize_adjoint(Vl, GW)
    GU = fat7_adjoint(dims, thin, HISQ_LEVEL1, GV)
    return _ta(thin @ GU)


def fermion_force_objective(dims, thin, alphas, xs, mass=0.1):
    """Q(U) = sum_k alpha_k Re(X_k^+ A X_k) on the links smeared from U (the
    mass only adds a constant)."""
    fat, lng = hisq_smear(dims, thin)
    return float(sum(a * np.vdot(x, apply_A(dims, fat, lng, mass, x)).real for a, x in zip(alphas, xs)))
