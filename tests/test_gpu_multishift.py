"""Multi-RHS Dslash and multi-shift CG on the GPU against the oracle."""
import numpy as np
import pytest

import oracle
from _parity import check
from paper_1712_00143_amd import synth

pytestmark = pytest.mark.gpu


def _hisq():
    from paper_1712_00143_amd import hisq
    return hisq


@pytest.mark.parametrize("nrhs", [2, 3, 4, 6, 11])
@pytest.mark.parametrize("prec,recon,tol", [(1, 18, 5e-6), (1, 12, 5e-6), (2, 12, 2e-3)])
def test_mrhs_dslash_matches_oracle(nrhs, prec, recon, tol):
    H = _hisq()
    dims = (6, 4, 8, 4)
    fat, lng = synth.make_links(dims, 0.3, seed=51)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(prec, recon)
    psi = synth.gaussian_even(dims, 52, nrhs)
    out = np.zeros_like(psi)
    for par in (0, 1):
        lat.dslash(par, prec, recon, psi, out, nrhs=nrhs)
        for j in range(nrhs):
            ref = oracle.dslash_half(dims, fat, lng, par, psi[j])
            check(out[j], ref, tol, (par, j))
    lat.close()


@pytest.mark.parametrize("no_tune", [False, True])
def test_mrhs_dslash_many_groups_ragged_tile(no_tune):
    """Thirteen right-hand sides (three full groups of four and a group of
    one) on a lattice whose last tile is ragged (h = 288): every output of
    the groups-innermost launch against the oracle, tuned and default shape."""
    H = _hisq()
    dims = (6, 4, 6, 4)
    fat, lng = synth.make_links(dims, 0.3, seed=57)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    nrhs = 13
    psi = synth.gaussian_even(dims, 58, nrhs)
    out = np.zeros_like(psi)
    for par in (0, 1):
        lat.dslash(par, 1, 18, psi, out, nrhs=nrhs, flags=H.HISQ_NO_TUNE if no_tune else 0)
        for j in range(nrhs):
            ref = oracle.dslash_half(dims, fat, lng, par, psi[j])
            check(out[j], ref, 5e-6, (par, j))
    lat.close()


def test_mrhs_dslash_device_matches_single():
    import torch
    H = _hisq()
    dims = (8, 8, 8, 8)
    fat, lng = synth.make_links(dims, 0.2, seed=53)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    psi = synth.gaussian_even(dims, 54, 4).astype(np.complex64)
    x = torch.from_numpy(psi.view(np.float32).reshape(-1)).cuda()
    y = torch.empty_like(x)
    lat.dslash(0, 1, 18, x, y, nrhs=4)
    torch.cuda.synchronize()
    h = psi.shape[1]
    for j in range(4):
        yj = torch.empty(6 * h, device="cuda", dtype=torch.float32)
        lat.dslash(0, 1, 18, x[j * 6 * h:(j + 1) * 6 * h].contiguous(), yj)
        torch.cuda.synchronize()
        # same arithmetic per right-hand side, different summation grouping
        a, b = y[j * 6 * h:(j + 1) * 6 * h], yj
        assert (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item() < 1e-6
    lat.close()


def test_multishift_small_vs_oracle_and_dense():
    H = _hisq()
    dims = (4, 4, 4, 4)
    fat, lng = synth.make_links(dims, 0.2, seed=2000)
    m = 0.01
    shifts = synth.shifts_log(12)
    b = synth.gaussian_even(dims, 2500, 4)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    x, infos = lat.multishift_cg(m, shifts, b, params=H.hisq_default_params(tol=1e-8, sloppy=1))
    for j in range(4):
        xo, it, rel, ok = oracle.multishift(dims, fat, lng, m, shifts, b[j], tol=1e-10)
        for k, s in enumerate(shifts):
            tr = oracle.true_residual(dims, fat, lng, m, b[j], x[j, k], sigma=s)
            assert tr <= 1e-8, (j, k, tr)
            assert infos[j * 12 + k]["converged"] == 1
            # kappa(A + s) <= 16.7 / (4 m^2 + s) on this lattice
            kappa = 16.7 / (4 * m * m + s)
            assert np.linalg.norm(x[j, k] - xo[k]) <= kappa * 1.1e-8 * np.linalg.norm(xo[k])
    lat.close()


def test_multishift_device_pointers_match_host_path():
    """Sources and solutions in device memory give the same solutions as the
    host-pointer path (same kernels, same order: bitwise)."""
    import torch
    H = _hisq()
    dims = (6, 4, 4, 6)
    fat, lng = synth.make_links(dims, 0.2, seed=2100)
    m = 0.02
    shifts = synth.shifts_log(5)
    b = synth.gaussian_even(dims, 2600, 3)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    p = H.hisq_default_params(tol=1e-9, sloppy=1)
    xh, ih = lat.multishift_cg(m, shifts, b, params=p)
    h = b.shape[1]
    bd = torch.from_numpy(np.ascontiguousarray(b).view(np.float64).ravel()).cuda()
    xd = torch.zeros(3 * 5 * h * 6, dtype=torch.float64, device="cuda")
    _, idv = lat.multishift_cg(m, shifts, bd, x=xd, params=H.hisq_default_params(tol=1e-9, sloppy=1))
    torch.cuda.synchronize()
    xdh = xd.cpu().numpy().view(np.complex128).reshape(3, 5, h, 3)
    assert np.array_equal(xdh, xh)
    assert [i["iters"] for i in idv] == [i["iters"] for i in ih]
    for j in range(3):
        for k, s in enumerate(shifts):
            assert oracle.true_residual(dims, fat, lng, m, b[j], xdh[j, k], sigma=s) <= 1e-9
    lat.close()


def test_multishift_fp16_recon12():
    H = _hisq()
    dims = (8, 8, 8, 8)
    fat, lng = synth.make_links(dims, 0.2, seed=2100)
    m = 0.02
    shifts = np.array([0.0, 1e-3, 1e-2, 0.1, 1.0])
    b = synth.gaussian_even(dims, 2600, 2)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(2, 12)
    x, infos = lat.multishift_cg(m, shifts, b, params=H.hisq_default_params(tol=1e-9, sloppy=2, recon=12))
    for j in range(2):
        for k, s in enumerate(shifts):
            assert oracle.true_residual(dims, fat, lng, m, b[j], x[j, k], sigma=s) <= 1e-9
    # smaller shifts need more iterations
    its = [infos[k]["iters"] for k in range(5)]
    assert its[0] >= its[-1]
    lat.close()


def test_multishift_full_size_24x24x24x48():
    """The multi-shift workload at full size: 24^3x48, 12 shifts in [1e-4, 1],
    4 sources, m = 0.01, tolerance 1e-8 on every shift (FP64 true residual
    recomputed by the oracle)."""
    H = _hisq()
    w = synth.C2
    fat, lng = w.links()
    b = w.sources()
    shifts = synth.shifts_log(12)
    lat = H.Lattice(w.dims)
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    x, infos = lat.multishift_cg(w.mass, shifts, b, params=H.hisq_default_params(
        tol=1e-8, sloppy=1, flags=H.HISQ_USE_GRAPH))
    lat.close()
    for j in range(4):
        for k, s in enumerate(shifts):
            assert infos[j * 12 + k]["converged"] == 1
            tr = oracle.true_residual(w.dims, fat, lng, w.mass, b[j], x[j, k], sigma=s)
            assert tr <= 1e-8, (j, k, tr)


def test_multishift_errors():
    H = _hisq()
    dims = (4, 4, 4, 4)
    lat = H.Lattice(dims)
    fat, lng = synth.make_links(dims, 0.2, seed=1)
    lat.load_links(fat, lng)
    b = synth.gaussian_even(dims, 1, 1)
    with pytest.raises(H.HisqError) as ei:
        lat.multishift_cg(0.1, np.zeros(65), b)
    assert ei.value.status == H.HISQ_ERR_ARG
    with pytest.raises(H.HisqError) as ei:
        lat.multishift_cg(0.1, [0.1, 0.2], b)          # FP32 link set not prepared
    assert ei.value.status == H.HISQ_ERR_STATE
    lat.close()


_FORCED_MRHS_CHILD = r'''
import json, os, sys
import numpy as np
import torch
import oracle
from paper_1712_00143_amd import synth, hisq as H

arch = torch.cuda.get_device_properties(0).gcnArchName.replace(" ", "_")
shape = int(sys.argv[1])                  # 512: matrix-core kernel, else waves of the vector-ALU kernel
path = os.environ["HISQ_TUNE_CACHE"]
cases = [(6, 4, 6, 4), (8, 8, 8, 8)]      # h = 288 (ragged last tile), 2048
lines = []
for dims in cases:
    t = (synth.volume(dims) // 2 + 63) // 64
    for p, r in ((1, 18), (1, 12), (2, 12)):
        lines.append(f"mrhs2:{arch}:p{p}:r{r}:t{t}:nr4 {shape} 1 0 1.0")
    lines.append(f"mrhs2:{arch}:p0:r18:t{t}:nr4 8 1 0 1.0")   # the FP64 reliable updates (vector ALU)
with open(path, "w") as f:
    f.write("\n".join(lines) + "\n")
tol = {1: 5e-6, 2: 2e-3}
worst = {}
for k, dims in enumerate(cases):
    fat, lng = synth.make_links(dims, 0.3, seed=61 + k)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    h = synth.volume(dims) // 2
    for p, r in ((1, 18), (1, 12), (2, 12)):
        lat.prepare_links(p, r)
        for nrhs in (4, 6, 13):           # full groups, and a last group of 2 or 1
            psi = synth.gaussian_even(dims, 80 + nrhs, nrhs)
            out = np.zeros_like(psi)
            for par in (0, 1):
                lat.dslash(par, p, r, psi, out, nrhs=nrhs)
                for j in range(nrhs):
                    ref = oracle.dslash_half(dims, fat, lng, par, psi[j])
                    rel = float(np.linalg.norm(out[j] - ref) / np.linalg.norm(ref))
                    site = float(np.linalg.norm(out[j] - ref, axis=1).max() / (np.linalg.norm(ref) / np.sqrt(h)))
                    worst[(p, r)] = max(worst.get((p, r), 0.0), rel)
                    assert rel <= tol[p] and site <= 10 * tol[p], (shape, dims, p, r, nrhs, par, j, rel, site)
    # the shared-link CG of several problems on one lattice runs its sloppy
    # operator (AX epilogue with the per-tile p.Ap sums) through the same launch
    lats = [lat] * 5
    ms = [0.1, 0.12, 0.15, 0.2, 0.25]
    bs = [synth.gaussian_even(dims, 90 + q) for q in range(5)]
    xs, infos = H.hisq_batch_cg(lats, ms, bs, params=H.hisq_default_params(tol=1e-10, sloppy=1))
    for q in range(5):
        tr = oracle.true_residual(dims, fat, lng, ms[q], bs[q], xs[q])
        assert infos[q]["converged"] == 1 and tr <= 1e-10, (shape, dims, q, tr)
    lat.close()
with open(path) as f:
    n = sum(1 for ln in f if ln.strip())
assert n == len(lines), "tuner added entries: a forced key did not match"
print(json.dumps({"shape": shape, "worst": {f"{k[0]}_{k[1]}": v for k, v in worst.items()}}))
'''


@pytest.mark.parametrize("shape", [512, 4])
def test_mrhs_dslash_forced_matrix_core_and_vector_kernels(tmp_path, shape):
    """The four-right-hand-side Dslash forced onto the matrix-core kernel
    (shape 512) and onto the vector-ALU kernel with four waves, through a
    prefilled tuner cache in a child process: FP32 recon-18 / recon-12 and
    FP16 recon-12 links, 4, 6 and 13 right-hand sides (partial last groups),
    a ragged last tile, every output against the oracle with the per-site
    bound, and the shared-link batched CG (AX epilogue) to the oracle's
    true residual 1e-10."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ)
    env["HISQ_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    env["PYTHONPATH"] = root + os.pathsep + env.get("PYTHONPATH", "")
    print(f"forced multi-RHS shape child {shape}", flush=True)
    r = subprocess.run([sys.executable, "-c", _FORCED_MRHS_CHILD, str(shape)], cwd=root, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert '"shape": %d' % shape in r.stdout, r.stdout
