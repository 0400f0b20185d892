"""GPU CG solves checked against the oracle: every solution's FP64 true
residual is recomputed by the oracle, and small systems are compared with the
oracle's (dense-pinned) solution within kappa * tol."""
import numpy as np
import pytest

import oracle
from paper_1712_00143_amd import synth

pytestmark = pytest.mark.gpu


def _hisq():
    from paper_1712_00143_amd import hisq
    return hisq


def test_c0_plain_fp64_cg():
    H = _hisq()
    w = synth.C0
    fat, lng = w.links()
    b = w.sources()[0]
    lat = H.Lattice(w.dims)
    lat.load_links(fat, lng)
    x, info = lat.cg(w.mass, b, params=H.hisq_default_params(tol=1e-10))
    assert info["converged"] == 1
    tr = oracle.true_residual(w.dims, fat, lng, w.mass, b, x)
    assert tr <= 1e-10
    xo, it, tro, ok = oracle.cg(w.dims, fat, lng, w.mass, b, tol=1e-12)
    # kappa of A on 4^4 at m = 0.1 is below 500
    assert np.linalg.norm(x - xo) <= 500 * 1e-10 * np.linalg.norm(xo)
    assert abs(info["true_residual"] - tr) <= 1e-3 * tr + 1e-14
    lat.close()


@pytest.mark.parametrize("sloppy,recon", [(1, 18), (1, 12), (2, 12), (2, 18), (0, 12)])
def test_mixed_precision_cg(sloppy, recon):
    H = _hisq()
    dims = (8, 8, 8, 12)
    fat, lng = synth.make_links(dims, 0.2, seed=77)
    m = 0.05
    b = synth.gaussian_even(dims, 577)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(sloppy, recon)
    p = H.hisq_default_params(tol=1e-10, sloppy=sloppy, recon=recon)
    x, info = lat.cg(m, b, params=p)
    assert info["converged"] == 1
    assert info["reliable_updates"] >= 1
    tr = oracle.true_residual(dims, fat, lng, m, b, x)
    assert tr <= 1e-10, (tr, info)
    lat.close()


def test_graph_replay_matches_eager_bitwise():
    H = _hisq()
    dims = (8, 8, 8, 8)
    fat, lng = synth.make_links(dims, 0.3, seed=5)
    b = synth.gaussian_even(dims, 6)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    p0 = H.hisq_default_params(tol=1e-10, sloppy=1, check_every=8)
    p1 = H.hisq_default_params(tol=1e-10, sloppy=1, check_every=8, flags=H.HISQ_USE_GRAPH)
    x0, i0 = lat.cg(0.05, b, params=p0)
    x1, i1 = lat.cg(0.05, b, params=p1)
    x2, i2 = lat.cg(0.05, b, params=p1)      # replay an already captured graph
    assert i0["iters"] == i1["iters"] == i2["iters"]
    assert np.array_equal(x0, x1) and np.array_equal(x1, x2)
    lat.close()


def test_chunk_lengths_do_not_change_the_solve():
    """The host only chooses how many iterations run between its reads of the
    solver state (planned from the residual's decay, at most check_every):
    every launch behind a pause is gated, so the iterates, the iteration and
    reliable-update counts and the solution are the same bits for any
    check_every, eager or graph-captured (chunks of 32, 16, 8, 4, 2 and 1)."""
    H = _hisq()
    dims = (8, 8, 8, 8)
    fat, lng = synth.make_links(dims, 0.3, seed=15)
    b = synth.gaussian_even(dims, 16)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    ref = None
    for ce in (1, 3, 16, 32):
        for fl in (0, H.HISQ_USE_GRAPH):
            for delta in (0.1, 0.01):
                p = H.hisq_default_params(tol=1e-10, sloppy=1, check_every=ce, delta=delta, flags=fl)
                x, info = lat.cg(0.02, b, params=p)
                assert info["converged"] == 1
                key = (delta,)
                if ref is None:
                    ref = {}
                if key not in ref:
                    ref[key] = (x, info["iters"], info["reliable_updates"])
                    assert oracle.true_residual(dims, fat, lng, 0.02, b, x) <= 1e-10
                else:
                    x0, it0, rel0 = ref[key]
                    assert info["iters"] == it0 and info["reliable_updates"] == rel0, (ce, fl, delta)
                    assert np.array_equal(x, x0), (ce, fl, delta)
    lat.close()


def test_warm_start_and_zero_source():
    H = _hisq()
    dims = (4, 4, 4, 8)
    fat, lng = synth.make_links(dims, 0.3, seed=9)
    b = synth.gaussian_even(dims, 10)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    xo, _, _, _ = oracle.cg(dims, fat, lng, 0.1, b, tol=1e-13)
    x0 = xo * (1 + 1e-4)
    p = H.hisq_default_params(tol=1e-10, flags=H.HISQ_X_IS_GUESS)
    x, info = lat.cg(0.1, b, x=x0.copy(), params=p)
    assert oracle.true_residual(dims, fat, lng, 0.1, b, x) <= 1e-10
    _, it_cold = lat.cg(0.1, b)
    assert info["iters"] < it_cold["iters"]
    z, iz = lat.cg(0.1, np.zeros_like(b))
    assert iz["converged"] == 1 and np.abs(z).max() == 0.0
    lat.close()


def test_not_converged_reports_best_iterate():
    H = _hisq()
    dims = (8, 8, 8, 8)
    fat, lng = synth.make_links(dims, 0.3, seed=11)
    b = synth.gaussian_even(dims, 12)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    p = H.hisq_default_params(tol=1e-10, maxiter=20, check_every=4)
    x, info = lat.cg(0.01, b, params=p, raise_on_fail=False)
    assert info["converged"] == 0 and info["status"] == H.HISQ_ERR_NOT_CONVERGED
    assert 20 <= info["iters"] <= 24
    tr = oracle.true_residual(dims, fat, lng, 0.01, b, x)
    assert tr < 1.0
    with pytest.raises(H.HisqError):
        lat.cg(-0.1, b)
    lat.close()


def test_batch_cg_uneven():
    H = _hisq()
    shapes = [(4, 4, 4, 4), (8, 8, 8, 8), (6, 6, 6, 6), (8, 8, 8, 16)]
    lats, bs, ms, links = [], [], [], []
    for j, d in enumerate(shapes):
        fat, lng = synth.make_links(d, 0.1 + 0.1 * j, seed=3000 + j)
        L = H.Lattice(d)
        L.load_links(fat, lng)
        L.prepare_links(1, 18)
        lats.append(L)
        links.append((fat, lng))
        bs.append(synth.gaussian_even(d, 3500 + j))
        ms.append([0.2, 0.05, 0.1, 0.02][j])
    p = H.hisq_default_params(tol=1e-10, sloppy=1, flags=H.HISQ_USE_GRAPH)
    xs, infos = H.hisq_batch_cg(lats, ms, bs, params=p)
    for j, d in enumerate(shapes):
        assert infos[j]["converged"] == 1
        tr = oracle.true_residual(d, *links[j], ms[j], bs[j], xs[j])
        assert tr <= 1e-10
        # the batched solve follows the same recurrence as a lone solve
        x1, i1 = lats[j].cg(ms[j], bs[j], params=H.hisq_default_params(tol=1e-10, sloppy=1))
        assert abs(i1["iters"] - infos[j]["iters"]) <= 16
    assert infos[0]["iters"] < infos[3]["iters"]
    for L in lats:
        L.close()


def test_fp16_links_small_mass_restart():
    """16^4 at m = 0.005 (condition number near 5e5): the FP16-link operator's
    own solution leaves a true residual of about 0.1, so continuing the old
    search direction after a reliable update stalls.  The restart rule keeps
    the FP16 solve within 1.5x the FP64 iteration count."""
    H = _hisq()
    w = synth.C4
    fat, lng = w.links()
    b = w.sources()[0]
    lat = H.Lattice(w.dims)
    lat.load_links(fat, lng)
    _, ref = lat.cg(w.mass, b, params=H.hisq_default_params(tol=1e-10))
    lat.prepare_links(2, 12)
    p = H.hisq_default_params(tol=1e-10, sloppy=2, recon=12, maxiter=4 * ref["iters"])
    x, info = lat.cg(w.mass, b, params=p)
    print("fp64", ref["iters"], "fp16 r12", info["iters"], "restarts", info["restarts"])
    assert info["converged"] == 1
    assert info["restarts"] >= 1
    assert info["iters"] <= 1.5 * ref["iters"]
    tr = oracle.true_residual(w.dims, fat, lng, w.mass, b, x)
    assert tr <= 1e-10
    lat.close()


@pytest.mark.parametrize("graph", [0, 1])
def test_batch_cg_one_lattice_shares_links(graph):
    """Six problems on one handle (different masses and sources): the FP32
    iterations go through the multi-right-hand-side kernel in groups of four
    and two; every solution reaches the FP64 true residual, and each follows
    the same recurrence as its lone solve (the two kernels round differently
    in FP32, so the counts agree to a few per cent, not exactly)."""
    H = _hisq()
    dims = (8, 8, 8, 12)
    fat, lng = synth.make_links(dims, 0.2, seed=611)
    L = H.Lattice(dims)
    L.load_links(fat, lng)
    L.prepare_links(1, 18)
    ms = [0.3, 0.02, 0.1, 0.05, 0.2, 0.01]
    bs = [synth.gaussian_even(dims, 620 + j) for j in range(len(ms))]
    p = H.hisq_default_params(tol=1e-10, sloppy=1, flags=H.HISQ_USE_GRAPH if graph else 0)
    xs, infos = H.hisq_batch_cg([L] * len(ms), ms, bs, params=p)
    for j, m in enumerate(ms):
        assert infos[j]["converged"] == 1
        assert oracle.true_residual(dims, fat, lng, m, bs[j], xs[j]) <= 1e-10
        _, i1 = L.cg(m, bs[j], params=H.hisq_default_params(tol=1e-10, sloppy=1))
        assert abs(i1["iters"] - infos[j]["iters"]) <= 0.06 * i1["iters"] + 8, (j, i1["iters"], infos[j]["iters"])
    assert infos[5]["iters"] > infos[0]["iters"]
    L.close()


@pytest.mark.parametrize("nprob,flags", [(3, 0), (5, "no_tune"), (2, 0)])
def test_batch_cg_one_lattice_group_sizes(nprob, flags):
    """One-lattice sets whose FP64 reliable updates run through the
    shared-link kernel in a group smaller than four (two or three problems:
    the whole set) or in groups of four with a ragged last group (five
    problems, default launch shapes): every solution reaches the FP64 true
    residual."""
    H = _hisq()
    dims = (8, 8, 8, 8)
    fat, lng = synth.make_links(dims, 0.2, seed=640 + nprob)
    L = H.Lattice(dims)
    L.load_links(fat, lng)
    L.prepare_links(1, 18)
    ms = [0.3, 0.05, 0.1, 0.02, 0.2][:nprob]
    bs = [synth.gaussian_even(dims, 650 + j) for j in range(nprob)]
    fl = H.HISQ_NO_TUNE if flags == "no_tune" else 0
    p = H.hisq_default_params(tol=1e-10, sloppy=1, flags=fl)
    xs, infos = H.hisq_batch_cg([L] * nprob, ms, bs, params=p)
    for j, m in enumerate(ms):
        assert infos[j]["converged"] == 1, (j, infos[j])
        assert oracle.true_residual(dims, fat, lng, m, bs[j], xs[j]) <= 1e-10
        assert infos[j]["reliable_updates"] >= 1
    L.close()


def test_batch_cg_reordered_problems():
    """Two batched calls led by the same handle, with the same sizes in a
    different order, reuse the work set; the tile-to-problem map must follow
    the new order."""
    H = _hisq()
    shapes = [(4, 4, 4, 4), (8, 8, 8, 8), (6, 6, 6, 6)]
    lats, links = [], []
    for j, d in enumerate(shapes):
        fat, lng = synth.make_links(d, 0.25, seed=640 + j)
        L = H.Lattice(d)
        L.load_links(fat, lng)
        L.prepare_links(1, 18)
        lats.append(L)
        links.append((fat, lng))
    bs = [synth.gaussian_even(d, 650 + j) for j, d in enumerate(shapes)]
    p = H.hisq_default_params(tol=1e-10, sloppy=1)
    for order in ([0, 1, 2], [0, 2, 1]):
        xs, infos = H.hisq_batch_cg([lats[k] for k in order], [0.1] * 3, [bs[k] for k in order], params=p)
        for q, k in enumerate(order):
            assert infos[q]["converged"] == 1
            assert oracle.true_residual(shapes[k], *links[k], 0.1, bs[k], xs[q]) <= 1e-10
    for L in lats:
        L.close()


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (6, 6, 6, 6), (4, 4, 8, 8)])
def test_cg_small_lattices(dims):
    """Small lattices (1, 2, 11 and 4 tiles): the same iteration count as the
    oracle's FP64 CG to within a few per cent (different summation order),
    FP64 true residual below tol, the batched path (one problem) agreeing,
    and the maxiter limit honoured."""
    H = _hisq()
    fat, lng = synth.make_links(dims, 0.3, seed=31)
    b = synth.gaussian_even(dims, 32)
    m = 0.05
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    x, info = lat.cg(m, b, params=H.hisq_default_params(tol=1e-10))
    assert info["converged"] == 1 and info["status"] == 0
    assert oracle.true_residual(dims, fat, lng, m, b, x) <= 1e-10
    assert abs(info["true_residual"] - oracle.true_residual(dims, fat, lng, m, b, x)) <= 1e-3 * info["true_residual"] + 1e-15
    _, it_o, _, _ = oracle.cg(dims, fat, lng, m, b, tol=1e-10)
    # the three FP64 CGs sum in different orders; near kappa ~ 1e3 that moves
    # the iteration count by a few per cent
    assert abs(info["iters"] - it_o) <= 0.04 * it_o + 3, (info["iters"], it_o)
    xb, ib = H.hisq_batch_cg([lat], [m], [b], params=H.hisq_default_params(tol=1e-10))
    assert ib[0]["converged"] == 1 and abs(ib[0]["iters"] - info["iters"]) <= 0.04 * it_o + 3
    assert oracle.true_residual(dims, fat, lng, m, b, xb[0]) <= 1e-10
    if info["iters"] > 12:
        x2, i2 = lat.cg(m, b, params=H.hisq_default_params(tol=1e-10, maxiter=10), raise_on_fail=False)
        assert i2["converged"] == 0 and i2["status"] == H.HISQ_ERR_NOT_CONVERGED and 10 <= i2["iters"] <= 10 + 16
        assert oracle.true_residual(dims, fat, lng, m, b, x2) < 1.0
    lat.close()


def test_batch_cg_workload_sizes():
    """The batched workload's own lattice sizes (8^4, 12^4, 16^4, 16^3x32) and
    parameter draws, two problems of each, in one batched FP32 solve with FP64
    reliable updates: every FP64 true residual recomputed by the oracle."""
    H = _hisq()
    ws = synth.batch_workload(nper=16)
    pick = [ws[k] for k in (0, 5, 16, 21, 32, 37, 48, 53)]
    lats, bs, links = [], [], []
    for w in pick:
        fat, lng = w.links()
        L = H.Lattice(w.dims)
        L.load_links(fat, lng)
        L.prepare_links(1, 18)
        lats.append(L)
        links.append((fat, lng))
        bs.append(w.sources()[0])
    p = H.hisq_default_params(tol=1e-10, sloppy=1, flags=H.HISQ_USE_GRAPH)
    xs, infos = H.hisq_batch_cg(lats, [w.mass for w in pick], bs, params=p)
    for q, w in enumerate(pick):
        assert infos[q]["converged"] == 1
        assert oracle.true_residual(w.dims, *links[q], w.mass, bs[q], xs[q]) <= 1e-10, (q, w.dims, w.mass)
    for L in lats:
        L.close()


@pytest.mark.parametrize("sloppy,recon", [(0, 18), (1, 18), (2, 12)])
def test_cg_above_fused_step_size(sloppy, recon):
    """16^3x40 has 1280 tiles per parity, above the size where the vector
    kernels sum the tile partials themselves: the iteration takes the
    finisher path, and must reach the same FP64 true residual."""
    H = _hisq()
    dims = (16, 16, 16, 40)
    fat, lng = synth.make_links(dims, 0.2, seed=71)
    b = synth.gaussian_even(dims, 72)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(sloppy, recon)
    x, info = lat.cg(0.05, b, params=H.hisq_default_params(tol=1e-10, sloppy=sloppy, recon=recon,
                                                           flags=H.HISQ_USE_GRAPH))
    assert info["converged"] == 1
    assert oracle.true_residual(dims, fat, lng, 0.05, b, x) <= 1e-10
    lat.close()


def test_residual_history():
    """The FP64 true residual of every reliable update is recorded: one per
    reliable update, the last equal to the reported (and the oracle's) true
    residual of the solution, the earlier ones above the target; batched
    solves keep one history per problem."""
    H = _hisq()
    dims = (8, 8, 8, 12)
    fat, lng = synth.make_links(dims, 0.2, seed=78)
    m = 0.05
    b = synth.gaussian_even(dims, 578)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    with pytest.raises(H.HisqError) as ei:
        lat.residual_history()
    assert ei.value.status == H.HISQ_ERR_STATE
    x, info = lat.cg(m, b, params=H.hisq_default_params(tol=1e-10, sloppy=1))
    hist = lat.residual_history()
    assert len(hist) == info["reliable_updates"] >= 2
    assert hist[-1] == info["true_residual"]
    tr = oracle.true_residual(dims, fat, lng, m, b, x)
    assert abs(hist[-1] - tr) <= 1e-6 * tr
    assert np.all(hist[:-1] > 1e-10) and hist[-1] <= 1e-10
    with pytest.raises(H.HisqError) as ei:
        lat.residual_history(1)
    assert ei.value.status == H.HISQ_ERR_ARG
    # batched: one history per problem, on the leading handle
    d2 = (4, 4, 4, 8)
    f2, l2 = synth.make_links(d2, 0.3, seed=79)
    L2 = H.Lattice(d2)
    L2.load_links(f2, l2)
    L2.prepare_links(1, 18)
    b2 = synth.gaussian_even(d2, 579)
    xs, infos = H.hisq_batch_cg([lat, L2], [m, 0.1], [b, b2], params=H.hisq_default_params(tol=1e-10, sloppy=1))
    for k in range(2):
        hk = lat.residual_history(k)
        assert len(hk) == infos[k]["reliable_updates"] and hk[-1] == infos[k]["true_residual"]
    tr2 = oracle.true_residual(d2, f2, l2, 0.1, b2, xs[1])
    assert abs(lat.residual_history(1)[-1] - tr2) <= 1e-6 * tr2
    L2.close()
    lat.close()


def test_solves_are_bitwise_reproducible():
    """No atomics and fixed reduction orders: the same solve twice gives the
    same iterate, iteration count and residual history, bit for bit."""
    H = _hisq()
    dims = (8, 8, 8, 8)
    fat, lng = synth.make_links(dims, 0.25, seed=81)
    b = synth.gaussian_even(dims, 581)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    out = []
    for _ in range(2):
        x, info = lat.cg(0.02, b, params=H.hisq_default_params(tol=1e-10, sloppy=1, flags=H.HISQ_USE_GRAPH))
        out.append((x, info["iters"], lat.residual_history()))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2])
    lat.close()


def test_stagnation_stop():
    """With HISQ_STOP_STAGNATION an unreachable target (1e-17, below FP64
    rounding of the true residual) ends after the true residual stops falling,
    long before maxiter, with HISQ_ERR_NOT_CONVERGED and the last iterate,
    which is as good as FP64 allows."""
    H = _hisq()
    dims = (4, 4, 4, 8)
    fat, lng = synth.make_links(dims, 0.25, seed=82)
    b = synth.gaussian_even(dims, 582)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    p = H.hisq_default_params(tol=1e-17, sloppy=1, flags=H.HISQ_STOP_STAGNATION)
    p.maxiter = 50000
    x, info = lat.cg(0.1, b, params=p, raise_on_fail=False)
    assert info["converged"] == 0 and info["status"] == H.HISQ_ERR_NOT_CONVERGED
    assert info["iters"] < 5000, info["iters"]
    hist = lat.residual_history()
    assert len(hist) >= 4 and min(hist[-3:]) >= hist[-4]
    assert oracle.true_residual(dims, fat, lng, 0.1, b, x) <= 1e-13
    lat.close()
