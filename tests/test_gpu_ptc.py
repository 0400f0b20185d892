"""Learned PTC preconditioner on the GPU against the oracle: layer forward,
input and weight gradients, FP16-weight inference, harvested pairs, one
training step (loss and Adam), and the flexible CG with its fallback."""
import numpy as np
import pytest

import oracle
from _parity import check
from paper_1712_00143_amd import synth

pytestmark = pytest.mark.gpu


def _hisq():
    from paper_1712_00143_amd import hisq
    return hisq


def _split(dims, a):
    """[C][V][3] lex order -> [C][2][h][3] parity split (cb order)."""
    ev, od = synth.even_sites(dims), synth.odd_sites(dims)
    return np.stack([a[:, ev], a[:, od]], axis=1)


def _unsplit(dims, s):
    ev, od = synth.even_sites(dims), synth.odd_sites(dims)
    out = np.zeros((s.shape[0], synth.volume(dims), 3), dtype=np.complex128)
    out[:, ev] = s[:, 0]
    out[:, od] = s[:, 1]
    return out


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64).view(np.float32).reshape(-1)).cuda()


def _host(t, shape):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.complex64).astype(np.complex128).reshape(shape)


def _rand_w(chans, seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return [scale * (rng.standard_normal((b, a, 9)) + 1j * rng.standard_normal((b, a, 9)))
            for a, b in zip(chans[:-1], chans[1:])]


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def lat6():
    H = _hisq()
    dims = (6, 4, 4, 8)
    fat, lng = synth.make_links(dims, 0.25, seed=4000)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    yield dims, fat, lng, lat
    lat.close()


@pytest.mark.parametrize("layer", [0, 1, 2])
def test_layer_forward_and_backward(lat6, layer):
    import torch
    H = _hisq()
    dims, fat, lng, lat = lat6
    chans = (1, 4, 4, 1)
    net = H.PTC(lat, chans)
    ws = _rand_w(chans, 10 + layer)
    net.set_weights(ws)
    cin, cout = chans[layer], chans[layer + 1]
    a = synth.gaussian_full(dims, 20 + layer, cin)
    g = synth.gaussian_full(dims, 30 + layer, cout)
    h = synth.volume(dims) // 2
    w32 = [w.astype(np.complex64).astype(np.complex128) for w in ws]   # GPU master weights are FP32
    ref = oracle.ptc_layer(dims, fat, w32[layer], a)
    out = torch.zeros(cout * 2 * h * 6, device="cuda")
    net.layer_forward(layer, _dev(_split(dims, a)), out)
    got = _unsplit(dims, _host(out, (cout, 2, h, 3)))
    check(got, ref, 1e-6, ("forward", layer))
    gin_ref, gw_ref = oracle.ptc_layer_adj(dims, fat, w32[layer], a, g)
    gin = torch.zeros(cin * 2 * h * 6, device="cuda")
    gw = net.layer_backward(layer, _dev(_split(dims, a)), _dev(_split(dims, g)), gin)
    check(_unsplit(dims, _host(gin, (cin, 2, h, 3))), gin_ref, 1e-6, ("input gradient", layer))
    assert _rel(gw, gw_ref) <= 1e-5
    net.close()


def test_apply_fp16_weights_matches_oracle(lat6):
    import torch
    H = _hisq()
    dims, fat, lng, lat = lat6
    chans = (1, 4, 4, 1)
    net = H.PTC(lat, chans)
    ws = _rand_w(chans, 3, scale=0.3)
    net.set_weights(ws)
    # the inference copy is the FP32 master rounded to IEEE binary16 (nearest even)
    w32 = [w.astype(np.complex64) for w in ws]
    w16 = [(w.real.astype(np.float16).astype(np.float64) + 1j * w.imag.astype(np.float16).astype(np.float64))
           for w in w32]
    r = synth.gaussian_even(dims, 5)
    ref = oracle.ptc_apply(dims, fat, w16, r)
    h = r.shape[0]
    z = torch.zeros(h * 6, device="cuda")
    net.apply(_dev(r), z)
    check(_host(z, (h, 3)), ref, 1e-5)
    net.close()


def test_harvest_pairs_are_error_residual_pairs():
    H = _hisq()
    dims = (8, 8, 8, 8)
    fat, lng = synth.make_links(dims, 0.25, seed=4001)
    m = 0.1
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    net = H.PTC(lat)
    b = synth.gaussian_even(dims, 4501)
    n = net.harvest(lat, m, b, every=5, maxpairs=100)
    assert n >= 5 and net.pair_count() == n
    h = b.shape[0]
    nb = np.linalg.norm(b)
    for i in range(n):
        r, e = net.get_pair(i, h)
        # A e_i = r_i - r*, |r*| <= 1e-12 |b|; pairs below 1e-9 |b| are dropped
        nr = np.linalg.norm(r)
        assert nr >= 0.99e-9 * nb
        Ae = oracle.apply_A(dims, fat, lng, m, e)
        assert _rel(Ae, r) <= 1e-5 + 1.5e-12 * nb / nr, (i, _rel(Ae, r))
    r0, e0 = net.get_pair(0, h)
    assert _rel(r0, b) <= 1e-6            # x_0 = 0: the first residual is b
    net.close()
    lat.close()


@pytest.mark.parametrize("loss", ["energy", "euclidean"])
def test_one_training_step_matches_oracle(loss):
    H = _hisq()
    dims = (4, 4, 4, 6)
    fat, lng = synth.make_links(dims, 0.25, seed=4002)
    m = 0.1
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    chans = (1, 2, 2, 1)
    net = H.PTC(lat, chans)
    w0 = _rand_w(chans, 7, scale=0.4)
    net.set_weights(w0)
    b = synth.gaussian_even(dims, 4502)
    n = net.harvest(lat, m, b, every=4, maxpairs=8)
    h = b.shape[0]
    pairs = [net.get_pair(i, h) for i in range(n)]
    net.set_loss(H.HISQ_LOSS_ENERGY if loss == "energy" else H.HISQ_LOSS_EUCLIDEAN)
    lr = 1e-3
    got_loss = net.train(1, batch=1, lr=lr, seed=11)[0]
    w1 = net.get_weights()
    w0f = [w.astype(np.complex64).astype(np.complex128) for w in w0]
    energy = (lng, m) if loss == "energy" else None
    cands = [oracle.ptc_loss_and_grad(dims, fat, w0f, [r], [e], energy=energy) for r, e in pairs]
    k = int(np.argmin([abs(c[0] - got_loss) for c in cands]))
    lo, grads = cands[k]
    assert abs(lo - got_loss) <= 1e-5 * lo
    for l in range(3):
        for part in ("real", "imag"):
            g = getattr(grads[l], part)
            p0 = getattr(w0f[l], part)
            p1, _, _ = oracle.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr=lr)
            got = getattr(w1[l], part)
            big = np.abs(g) > 1e-3 * np.abs(g).max()
            assert np.allclose(got[big], p1[big], atol=2e-6, rtol=0), (l, part)
    net.close()
    lat.close()


def _identity_weights(chans):
    ws = []
    for a, b in zip(chans[:-1], chans[1:]):
        w = np.zeros((b, a, 9), dtype=np.complex128)
        for c in range(min(a, b)):
            w[c, c, 0] = 1.0
        ws.append(w)
    return ws


def test_fcg_with_identity_net_is_cg():
    H = _hisq()
    dims = (8, 8, 8, 8)
    fat, lng = synth.make_links(dims, 0.25, seed=4003)
    m = 0.05
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    net = H.PTC(lat)
    net.set_weights(_identity_weights((1, 4, 4, 1)))
    b = synth.gaussian_even(dims, 4503)
    p = H.hisq_default_params(tol=1e-10, sloppy=1)
    x, info = net.cg_learned(lat, m, b, params=p)
    assert info["converged"] == 1 and info["fell_back"] == 0
    assert oracle.true_residual(dims, fat, lng, m, b, x) <= 1e-10
    _, ci = lat.cg(m, b, params=p)
    assert abs(info["iters"] - ci["iters"]) <= 0.1 * ci["iters"] + 5
    net.close()
    lat.close()


def test_fcg_falls_back_on_breakdown():
    H = _hisq()
    dims = (4, 4, 4, 8)
    fat, lng = synth.make_links(dims, 0.25, seed=4004)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    net = H.PTC(lat)
    ws = _identity_weights((1, 4, 4, 1))
    ws[1][0, 0, 0] = np.nan
    net.set_weights(ws)
    b = synth.gaussian_even(dims, 4504)
    x, info = net.cg_learned(lat, 0.1, b, params=H.hisq_default_params(tol=1e-10, sloppy=1))
    assert info["fell_back"] == 1 and info["converged"] == 1
    assert oracle.true_residual(dims, fat, lng, 0.1, b, x) <= 1e-10
    # an all-zero network (the initial state) is M = 1: plain CG, no hand-over
    net2 = H.PTC(lat)
    p = H.hisq_default_params(tol=1e-10, sloppy=1)
    x2, info2 = net2.cg_learned(lat, 0.1, b, params=p)
    assert info2["fell_back"] == 0 and oracle.true_residual(dims, fat, lng, 0.1, b, x2) <= 1e-10
    _, ci = lat.cg(0.1, b, params=p)
    assert abs(info2["iters"] - ci["iters"]) <= 0.1 * ci["iters"] + 5
    net.close()
    net2.close()
    lat.close()


@pytest.mark.parametrize("flags", [0, 4], ids=["eager", "graph"])
def test_fcg_hands_over_at_half_maxiter(flags):
    """The flexible CG stops at maxiter / 2 iterations (checked after each
    chunk and after each device-gated restart) and hands its iterate to CG,
    which gets the rest of maxiter: enough here to converge, and the same
    solution as without the cap to the solver tolerance."""
    H = _hisq()
    dims = (8, 8, 8, 8)
    m = 0.01
    fat, lng = synth.make_links(dims, 0.25, seed=4010)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    net = H.PTC(lat, (1, 4, 4, 1))
    net.init_polynomial(a=4.0, c=1.2)
    b = synth.gaussian_even(dims, 4510)
    _, free = net.cg_learned(lat, m, b, params=H.hisq_default_params(tol=1e-10, sloppy=1, flags=flags))
    assert free["fell_back"] == 0
    cap = free["iters"]   # the FCG stops near cap / 2 iterations
    p = H.hisq_default_params(tol=1e-10, sloppy=1, maxiter=cap, check_every=8, flags=flags)
    x, info = net.cg_learned(lat, m, b, params=p, raise_on_fail=False)
    assert info["fell_back"] == 1
    assert cap // 2 <= info["fcg_iters"] <= cap // 2 + 8
    if info["converged"]:
        assert oracle.true_residual(dims, fat, lng, m, b, x) <= 1.5e-10
    assert info["iters"] <= cap + 8
    net.close()
    lat.close()


@pytest.mark.parametrize("chans", [(1, 4, 4, 1), (1, 4, 1)], ids=["1-4-4-1", "1-4-1"])
def test_training_lowers_loss_and_reports_gain(chans):
    """Train from small random weights on fields 0..3 (pairs harvested by the
    solver itself, energy-norm loss), test on a held-out field.  Asserted: the
    training loss falls, the flexible CG with the trained network reaches the
    FP64 true residual 1e-10 without a hand-over to plain CG, and it needs
    fewer iterations than the untrained network (M = 1, i.e. plain CG): the
    network learns a preconditioner by itself (321 -> 106 iterations when
    this was written)."""
    H = _hisq()
    dims = (8, 8, 8, 8)
    m = 0.02
    lats = []
    net = None
    for j in range(4):
        fat, lng = synth.make_links(dims, 0.25, seed=4100 + j)
        L = H.Lattice(dims)
        L.load_links(fat, lng)
        lats.append(L)
        if net is None:
            net = H.PTC(L, chans)
            net.set_weights(_rand_w(chans, 77, scale=0.05))
        for s in range(2):
            net.harvest(L, m, synth.gaussian_even(dims, 4600 + 10 * j + s), every=10, maxpairs=40)
    losses = net.train(400, batch=8, lr=3e-3, seed=1)
    assert losses[-50:].mean() < losses[:10].mean()
    fat, lng = synth.make_links(dims, 0.25, seed=4199)
    T = H.Lattice(dims)
    T.load_links(fat, lng)
    b = synth.gaussian_even(dims, 4699)
    p = H.hisq_default_params(tol=1e-10, sloppy=1)
    x, info = net.cg_learned(T, m, b, params=p)
    assert info["converged"] == 1 and info["fell_back"] == 0
    assert oracle.true_residual(dims, fat, lng, m, b, x) <= 1e-10
    untrained = H.PTC(T, chans)          # zero weights: M = 1
    _, i0 = untrained.cg_learned(T, m, b, params=p)
    start = H.PTC(T, chans)              # the network's own starting point, untrained
    start.set_weights(_rand_w(chans, 77, scale=0.05))
    _, i1 = start.cg_learned(T, m, b, params=p)
    print(f"learned-preconditioner gain: iterations {i0['iters']} (M = 1), {i1['iters']} (random start, "
          f"untrained) -> {info['iters']} (trained), ratio {i1['iters'] / info['iters']:.3f}; "
          f"loss {losses[:10].mean():.4f} -> {losses[-50:].mean():.4f}")
    assert info["iters"] <= 0.8 * i0["iters"], (info["iters"], i0["iters"])
    assert info["iters"] <= 0.8 * i1["iters"], (info["iters"], i1["iters"])
    start.close()
    untrained.close()
    for L in lats + [T]:
        L.close()


def test_polynomial_start_free_field():
    """The library's polynomial start on the 4^4 free field: the power
    iteration finds the top of -D_f^2 exactly (16 = 4 * 4 sin^2(pi/2)), the
    weights are the documented ones, and M on an even plane wave is
    1 + a^2 (1 - c t/16)^2 (FP16 inference weights: 2e-3)."""
    from test_oracle_solvers import _poly_weights
    H = _hisq()
    dims = (4, 4, 4, 4)
    fat, lng = synth.unit_links(dims)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    for chans, c in [((1, 4, 4, 1), 1.0), ((1, 2, 1), 1.2)]:
        net = H.PTC(lat, chans)
        a = 3.0
        lam = net.init_polynomial(a=a, c=c, iters=60)
        assert abs(lam - 16.0) <= 1e-4 * 16.0, lam
        ref = _poly_weights(chans, a, lam / c)
        for w, r in zip(net.get_weights(), ref):
            assert np.abs(w - r).max() <= 1e-6 * a
        x = synth.coords(dims)[synth.even_sites(dims)]
        chi = np.array([1.0, 0.5j, -0.25])
        for n in [(1, 0, 0, 0), (1, 1, 2, 0), (0, 0, 0, 0), (1, 1, 1, 1)]:
            p = 2 * np.pi * np.array(n) / np.array(dims)
            v = np.exp(1j * (x @ p))[:, None] * chi[None, :]
            t = 4 * np.sum(np.sin(p) ** 2)
            r = _dev(v)
            z = r.clone()
            net.apply(r, z)
            got = _host(z, v.shape)
            want = (1.0 + a * a * (1.0 - c * t / 16.0) ** 2) * v
            assert _rel(got, want) <= 2e-3, (chans, n, _rel(got, want))
        net.close()
    one = H.PTC(lat, (1, 1))
    with pytest.raises(H.HisqError) as ei:
        one.init_polynomial()
    assert ei.value.status == H.HISQ_ERR_ARG
    one.close()
    net = H.PTC(lat, (1, 4, 4, 1))
    for bad in [dict(a=0.0), dict(c=0.0), dict(c=5.0), dict(iters=0)]:
        with pytest.raises(H.HisqError) as ei:
            net.init_polynomial(**bad)
        assert ei.value.status == H.HISQ_ERR_ARG, bad
    net.close()
    lat.close()


def test_polynomial_start_cuts_fcg_iterations():
    """8^4, m = 0.01: the polynomial start cuts the flexible CG's iteration
    count to under half of plain CG's and reaches the FP64 true residual
    without a hand-over.  The oracle's FCG with the same FP16-rounded weights
    is FP64 throughout; the GPU iterates in FP32 with FP64 reliable updates,
    which costs some conjugacy: its count may exceed the oracle's by up to
    25 % (mixed FP32 plain CG on this problem: 505 against the FP64 446)."""
    H = _hisq()
    dims = (8, 8, 8, 8)
    m = 0.01
    fat, lng = synth.make_links(dims, 0.25, seed=77)
    b = synth.gaussian_even(dims, 78)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    net = H.PTC(lat, (1, 4, 4, 1))
    lam = net.init_polynomial(a=4.0, c=1.2, iters=30)
    assert 10.0 < lam < 16.0, lam
    p = H.hisq_default_params(tol=1e-10, sloppy=1)
    x, info = net.cg_learned(lat, m, b, params=p)
    assert info["converged"] == 1 and info["fell_back"] == 0
    assert oracle.true_residual(dims, fat, lng, m, b, x) <= 1e-10
    _, ci = lat.cg(m, b, params=p)
    ws16 = [w.astype(np.complex64).real.astype(np.float16).astype(np.float64)
            + 1j * w.astype(np.complex64).imag.astype(np.float16).astype(np.float64) for w in net.get_weights()]
    _, it_o, tr_o, ok_o = oracle.fcg(dims, fat, lng, m, ws16, b, tol=1e-10)
    print(f"polynomial start: FCG {info['iters']} iterations (oracle {it_o}), plain CG {ci['iters']}, "
          f"lambda {lam:.4f}")
    assert ok_o and info["iters"] <= 0.5 * ci["iters"]
    assert it_o - 2 <= info["iters"] <= 1.25 * it_o + 2
    net.close()
    lat.close()


def test_fcg_graph_replay_matches_eager():
    """The captured iteration chunk gives the eager launches' result bit for
    bit (same kernels, same order), on two solves in a row (the second
    replays the cached graph) and after a change of weights (read from device
    memory by the replay)."""
    H = _hisq()
    dims = (8, 8, 8, 8)
    m = 0.01
    fat, lng = synth.make_links(dims, 0.25, seed=77)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    net = H.PTC(lat, (1, 4, 4, 1))
    net.init_polynomial(a=4.0, c=1.2)
    pe = H.hisq_default_params(tol=1e-10, sloppy=1)
    pg = H.hisq_default_params(tol=1e-10, sloppy=1, flags=H.HISQ_USE_GRAPH)
    for k, seed in enumerate([78, 79]):
        b = synth.gaussian_even(dims, seed)
        xe, ie = net.cg_learned(lat, m, b, params=pe)
        xg, ig = net.cg_learned(lat, m, b, params=pg)
        assert ie["converged"] == 1 and ig["converged"] == 1
        assert ie["iters"] == ig["iters"] and ie["reliable_updates"] == ig["reliable_updates"]
        assert np.array_equal(xe, xg), k
        assert oracle.true_residual(dims, fat, lng, m, b, xg) <= 1e-10
    net.init_polynomial(a=2.0, c=1.0)
    b = synth.gaussian_even(dims, 80)
    xe, ie = net.cg_learned(lat, m, b, params=pe)
    xg, ig = net.cg_learned(lat, m, b, params=pg)
    assert ie["iters"] == ig["iters"] and np.array_equal(xe, xg)
    net.close()
    lat.close()


def test_fcg_chunk_lengths_do_not_change_the_solve():
    """The flexible CG's chunk lengths (planned from the residual's decay, at
    most check_every) and its device-gated restart after a reliable update
    leave the solve unchanged bit for bit, eager or graph-captured."""
    H = _hisq()
    dims = (8, 8, 8, 8)
    m = 0.01
    fat, lng = synth.make_links(dims, 0.25, seed=81)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    net = H.PTC(lat, (1, 4, 4, 1))
    net.init_polynomial(a=4.0, c=1.2)
    b = synth.gaussian_even(dims, 82)
    ref = {}
    for ce in (1, 5, 16, 32):
        for fl in (0, H.HISQ_USE_GRAPH):
            for delta in (0.1, 0.01):
                p = H.hisq_default_params(tol=1e-10, sloppy=1, check_every=ce, delta=delta, flags=fl)
                x, info = net.cg_learned(lat, m, b, params=p)
                assert info["converged"] == 1 and not info["fell_back"]
                if delta not in ref:
                    ref[delta] = (x, info["iters"], info["reliable_updates"])
                    assert oracle.true_residual(dims, fat, lng, m, b, x) <= 1e-10
                    assert len(lat.residual_history()) == info["reliable_updates"]
                else:
                    x0, it0, rel0 = ref[delta]
                    assert info["iters"] == it0 and info["reliable_updates"] == rel0, (ce, fl, delta)
                    assert np.array_equal(x, x0), (ce, fl, delta)
    net.close()
    lat.close()


def test_checkpoint_save_load(tmp_path):
    """A saved network restores exactly: the same weights, and training goes
    on from the restored Adam state as it does in the network it came from.
    Files of another shape, foreign files and missing files are refused."""
    H = _hisq()
    dims = (4, 4, 4, 6)
    fat, lng = synth.make_links(dims, 0.25, seed=4010)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    chans = (1, 2, 2, 1)
    b = synth.gaussian_even(dims, 4510)
    a = H.PTC(lat, chans)
    a.set_weights(_rand_w(chans, 9, scale=0.3))
    a.harvest(lat, 0.1, b, every=4, maxpairs=8)
    a.train(3, batch=2, lr=1e-3, seed=5)
    path = str(tmp_path / "net.ptc")
    a.save(path)
    c = H.PTC(lat, chans)
    c.harvest(lat, 0.1, b, every=4, maxpairs=8)
    c.load(path)
    for wa, wc in zip(a.get_weights(), c.get_weights()):
        assert np.array_equal(wa, wc)
    la = a.train(2, batch=2, lr=1e-3, seed=6)
    lc = c.train(2, batch=2, lr=1e-3, seed=6)
    assert np.array_equal(la, lc)
    for wa, wc in zip(a.get_weights(), c.get_weights()):
        assert np.array_equal(wa, wc)
    other = H.PTC(lat, (1, 4, 4, 1))
    for bad in [path, str(tmp_path / "missing.ptc")]:
        with pytest.raises(H.HisqError) as ei:
            (other if bad == path else c).load(bad)
        assert ei.value.status == H.HISQ_ERR_IO
    junk = tmp_path / "junk.ptc"
    junk.write_bytes(b"HISQPTC1" + b"\x00" * 12)
    with pytest.raises(H.HisqError) as ei:
        c.load(str(junk))
    assert ei.value.status == H.HISQ_ERR_IO
    for n in (a, c, other):
        n.close()
    lat.close()


# ---- transports on FP16 recon-12 fat links -------------------------------
#
# Bars: the oracle runs on the exact FP64 links; the GPU stores each fat link
# as two FP16 rows over the field scale (relative rounding <= 2^-11 per real)
# and rebuilds the third row, so a transported vector carries about 2^-11
# relative error per link, summed over the 9 paths: 2e-3 relative l2, the
# bar of the FP16 Dslash, with the per-site bound of _parity.check.

TOL16 = 2e-3


def test_transport_format_default_and_errors(lat6):
    H = _hisq()
    dims, fat, lng, lat = lat6
    net = H.PTC(lat, (1, 2, 1))
    assert net.get_transport() == (1, 18)
    net.set_transport(2, 12)
    assert net.get_transport() == (2, 12)
    for bad in [(0, 18), (1, 12), (2, 18)]:
        with pytest.raises(H.HisqError) as ei:
            net.set_transport(*bad)
        assert ei.value.status == H.HISQ_ERR_ARG
    assert net.get_transport() == (2, 12)
    net.close()


@pytest.mark.parametrize("layer", [0, 1, 2])
def test_layer_fp16_transports_match_oracle(lat6, layer):
    """Forward, input gradient and weight gradient of one layer with the
    transports on FP16 recon-12 fat links (the format the flexible CG runs
    on), against the oracle on the FP64 links."""
    import torch
    H = _hisq()
    dims, fat, lng, lat = lat6
    chans = (1, 4, 4, 1)
    net = H.PTC(lat, chans)
    net.set_transport(2, 12)
    ws = _rand_w(chans, 40 + layer)
    net.set_weights(ws)
    cin, cout = chans[layer], chans[layer + 1]
    a = synth.gaussian_full(dims, 50 + layer, cin)
    g = synth.gaussian_full(dims, 60 + layer, cout)
    h = synth.volume(dims) // 2
    w32 = [w.astype(np.complex64).astype(np.complex128) for w in ws]
    ref = oracle.ptc_layer(dims, fat, w32[layer], a)
    out = torch.zeros(cout * 2 * h * 6, device="cuda")
    net.layer_forward(layer, _dev(_split(dims, a)), out)
    got = _unsplit(dims, _host(out, (cout, 2, h, 3)))
    check(got, ref, TOL16, ("forward", layer))
    gin_ref, gw_ref = oracle.ptc_layer_adj(dims, fat, w32[layer], a, g)
    gin = torch.zeros(cin * 2 * h * 6, device="cuda")
    gw = net.layer_backward(layer, _dev(_split(dims, a)), _dev(_split(dims, g)), gin)
    check(_unsplit(dims, _host(gin, (cin, 2, h, 3))), gin_ref, TOL16, ("input gradient", layer))
    assert _rel(gw, gw_ref) <= TOL16, ("weight gradient", layer, _rel(gw, gw_ref))
    net.close()


def test_apply_fp16_transports_matches_oracle(lat6):
    """z = M(r) with FP16 weights and FP16 recon-12 transports against the
    oracle's M on the FP16-rounded weights and the FP64 links; the same
    network with FP32 transports stays at the FP32 bar."""
    import torch
    H = _hisq()
    dims, fat, lng, lat = lat6
    chans = (1, 4, 4, 1)
    net = H.PTC(lat, chans)
    ws = _rand_w(chans, 8, scale=0.3)
    net.set_weights(ws)
    w32 = [w.astype(np.complex64) for w in ws]
    w16 = [(w.real.astype(np.float16).astype(np.float64) + 1j * w.imag.astype(np.float16).astype(np.float64))
           for w in w32]
    r = synth.gaussian_even(dims, 9)
    ref = oracle.ptc_apply(dims, fat, w16, r)
    h = r.shape[0]
    z = torch.zeros(h * 6, device="cuda")
    net.apply(_dev(r), z)
    check(_host(z, (h, 3)), ref, 1e-5, "fp32 transports")
    net.set_transport(2, 12)
    net.apply(_dev(r), z)
    check(_host(z, (h, 3)), ref, TOL16, "fp16 transports")
    net.close()


def test_cg_learned_fp16_transports_16x16x16x16():
    """The learned flexible CG with FP16 recon-12 transports on a 16^4 field of
    the learned-preconditioner workload (eps 0.25, m 0.005), polynomial start
    trained on pairs of the same field with the same transports: the FP64
    true residual of the solution, recomputed by the oracle, is <= 1e-10,
    with no hand-over to plain CG."""
    H = _hisq()
    w = synth.C4
    fat, lng = synth.make_links(w.dims, w.eps, seed=4000)
    lat = H.Lattice(w.dims)
    lat.load_links(fat, lng)
    net = H.PTC(lat, (1, 2, 1))
    net.set_transport(2, 12)
    net.init_polynomial(a=4.0, c=1.2)
    net.harvest(lat, w.mass, synth.gaussian_even(w.dims, 4500), every=20, maxpairs=30)
    losses = net.train(60, batch=4, lr=1e-3, seed=3)
    assert np.all(np.isfinite(losses))
    b = synth.gaussian_even(w.dims, 4900)
    for flags in (0, H.HISQ_USE_GRAPH):
        x, info = net.cg_learned(lat, w.mass, b, params=H.hisq_default_params(tol=1e-10, sloppy=1, flags=flags))
        tr = oracle.true_residual(w.dims, fat, lng, w.mass, b, x)
        print(f"fp16-transport learned FCG, flags {flags}: {info['iters']} iterations, oracle true residual {tr:.2e}")
        assert info["converged"] == 1 and info["fell_back"] == 0, info
        assert tr <= 1e-10, tr
    net.close()
    lat.close()


# ---- FP16 activation storage of inference ---------------------------------
#
# Bar: each stored activation entry is rounded to 2^-11 of its site's scale,
# three times per hidden activation chain of the 1->4->4->1 network and its
# adjoint; 2e-3 relative l2 on M r - r (the part the layers produce), which
# is what FP16 storage puts at stake (the identity term is added in FP32).

@pytest.mark.parametrize("transport", [(1, 18), (2, 12)])
@pytest.mark.parametrize("chans", [(1, 4, 4, 1), (1, 2, 1)])
def test_apply_fp16_activations_matches_oracle(lat6, transport, chans):
    import torch
    H = _hisq()
    dims, fat, lng, lat = lat6
    net = H.PTC(lat, chans)
    net.set_transport(*transport)
    net.set_activations(2)
    ws = _rand_w(chans, 12, scale=0.3)
    net.set_weights(ws)
    w32 = [w.astype(np.complex64) for w in ws]
    w16 = [(w.real.astype(np.float16).astype(np.float64) + 1j * w.imag.astype(np.float16).astype(np.float64))
           for w in w32]
    r = synth.gaussian_even(dims, 13)
    ref = oracle.ptc_apply(dims, fat, w16, r)
    h = r.shape[0]
    z = torch.zeros(h * 6, device="cuda")
    net.apply(_dev(r), z)
    got = _host(z, (h, 3))
    check(got - r, ref - r, 2e-3, ("fp16 activations", transport, chans))
    net.close()


def test_cg_learned_fp16_activations_graph_and_eager():
    """The learned flexible CG with FP16 activations and FP16 recon-12
    transports on a 12^4 field: oracle true residual <= 1e-10 without a
    hand-over, and the graph-captured iteration gives the eager bits."""
    H = _hisq()
    dims = (12, 12, 12, 12)
    fat, lng = synth.make_links(dims, 0.25, seed=4800)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    net = H.PTC(lat, (1, 4, 4, 1))
    net.set_transport(2, 12)
    net.set_activations(2)
    net.init_polynomial(a=4.0, c=1.2)
    b = synth.gaussian_even(dims, 4801)
    m = 0.01
    xs = []
    for flags in (0, H.HISQ_USE_GRAPH, H.HISQ_USE_GRAPH):
        x, info = net.cg_learned(lat, m, b, params=H.hisq_default_params(tol=1e-10, sloppy=1, flags=flags))
        tr = oracle.true_residual(dims, fat, lng, m, b, x)
        assert info["converged"] == 1 and info["fell_back"] == 0 and tr <= 1e-10, (flags, info, tr)
        xs.append(x)
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[1], xs[2])
    net.close()
    lat.close()


_FORCED_INFER_CHILD = r'''
import json, os, sys
import numpy as np
import torch
import oracle
from paper_1712_00143_amd import synth, hisq as H

arch = torch.cuda.get_device_properties(0).gcnArchName.replace(" ", "_")
W = int(sys.argv[1])
dims = (6, 4, 4, 8)                       # h = 384: six tiles per parity
fat, lng = synth.make_links(dims, 0.25, seed=4000)
h = synth.volume(dims) // 2
t = (h + 63) // 64
path = os.environ["HISQ_TUNE_CACHE"]
lines = []
for p, r in ((1, 18), (2, 12)):
    for chans in ((1, 4, 4, 1), (1, 2, 1), (1, 8, 8, 1)):
        L = len(chans) - 1
        def wl(cin, cout):               # matrix-core shapes only where they exist
            return W if cout >= cin or W < 256 else W & 255
        for l in range(L):               # forward layers, then the adjoint ones
            ci, co = chans[l], chans[l + 1]
            lines.append(f"ptcinf:{arch}:t{t}:p{p}:r{r}:{ci}x{co}:k{0 if l == 0 else 1}0:np2 {wl(ci, co)} 0 0 1.0")
        for l in range(L - 1, -1, -1):
            last = l == 0
            ci, co = chans[l + 1], chans[l]
            lines.append(f"ptcinf:{arch}:t{t}:p{p}:r{r}:{ci}x{co}:k1{1 if last else 0}:np{1 if last else 2} {wl(ci, co)} 0 0 1.0")
with open(path, "w") as f:
    f.write("\n".join(sorted(set(lines))) + "\n")
lat = H.Lattice(dims)
lat.load_links(fat, lng)
rng = np.random.default_rng(3)
worst = 0.0
for p, r in ((1, 18), (2, 12)):
    for chans in ((1, 4, 4, 1), (1, 2, 1), (1, 8, 8, 1)):
        net = H.PTC(lat, chans)
        net.set_transport(p, r)
        net.set_activations(2)
        ws = [0.3 * (rng.standard_normal((b, a, 9)) + 1j * rng.standard_normal((b, a, 9)))
              for a, b in zip(chans[:-1], chans[1:])]
        net.set_weights(ws)
        w16 = [(w.astype(np.complex64).real.astype(np.float16).astype(np.float64)
                + 1j * w.astype(np.complex64).imag.astype(np.float16).astype(np.float64)) for w in ws]
        for scale in (1.0, 1e-9):        # the residual's magnitude must not matter
            rv = scale * synth.gaussian_even(dims, 17)
            ref = oracle.ptc_apply(dims, fat, w16, rv)
            x = torch.from_numpy(rv.astype(np.complex64).view(np.float32).reshape(-1)).cuda()
            z = torch.zeros_like(x)
            net.apply(x, z)
            torch.cuda.synchronize()
            got = z.cpu().numpy().view(np.complex64).astype(np.complex128).reshape(-1, 3)
            d, e = got - rv.astype(np.complex64).astype(np.complex128), ref - rv
            rel = float(np.linalg.norm(d - e) / np.linalg.norm(e))
            site = float(np.linalg.norm(d - e, axis=1).max() / (np.linalg.norm(e) / np.sqrt(h)))
            worst = max(worst, rel)
            assert rel <= 2e-3 and site <= 2e-2, (W, p, r, chans, scale, rel, site)
        net.close()
lat.close()
with open(path) as f:
    n = sum(1 for ln in f if ln.strip())
assert n == len(set(lines)), "tuner added entries: a forced key did not match"
print(json.dumps({"W": W, "worst": worst}))
'''


@pytest.mark.parametrize("W", [1, 3, 9, 259, 265])
def test_fp16_activation_layers_every_shape(tmp_path, W):
    """Every block shape of the FP16-activation inference layers (W = 1, 3, 9:
    vector-ALU channel mixing; 259, 265 = 3, 9 with the matrix-core mixing,
    used by the layers with at least as many outputs as inputs), forced
    through a prefilled tuner cache in a child process, for 1-4-4-1, 1-2-1
    and 1-8-8-1 networks on both transport formats and on a residual scaled
    by 1e-9: M r - r against the oracle at the FP16-activation bar."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ)
    env["HISQ_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    env["PYTHONPATH"] = root + os.pathsep + env.get("PYTHONPATH", "")
    print(f"forced inference shape child W={W}", flush=True)
    r = subprocess.run([sys.executable, "-c", _FORCED_INFER_CHILD, str(W)], cwd=root, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert '"W": %d' % W in r.stdout, r.stdout
