"""The no-allocation CG entry point (hisq_cg_noalloc) against hisq_cg.

Two calls in a row on one device, the second on a smaller lattice and in
another precision, so the second reuses the static work buffer the first
filled: each solution must be the one hisq_cg computes (the same kernels in
the same launch shape, so the same bits), reach the FP64 true residual the
oracle recomputes, and report the same iteration counts.  Then the error
paths: host vectors, graphs, a lattice larger than the buffer."""
import numpy as np
import pytest

import oracle
from paper_1712_00143_amd import synth

pytestmark = pytest.mark.gpu


def _solve_pair(H, torch, dims, eps, seed, m, sloppy, recon):
    fat, lng = synth.make_links(dims, eps, seed=seed)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    lat.prepare_links(sloppy, recon)
    b = synth.gaussian_even(dims, seed + 500)
    bd = torch.from_numpy(b.view(np.float64).ravel()).cuda()
    prm = dict(tol=1e-10, sloppy=sloppy, recon=recon)
    x_ref = torch.zeros_like(bd)
    _, info_ref = lat.cg(m, bd, x=x_ref, params=H.hisq_default_params(**prm))
    x_na = torch.full_like(bd, 7.0)          # garbage in x: a cold start must ignore it
    _, info_na = lat.cg_noalloc(m, bd, x_na, params=H.hisq_default_params(**prm))
    torch.cuda.synchronize()
    xr = x_ref.cpu().numpy().view(np.complex128).reshape(-1, 3)
    xn = x_na.cpu().numpy().view(np.complex128).reshape(-1, 3)
    tr = oracle.true_residual(dims, fat, lng, m, b, xn)
    print(f"noalloc {dims} sloppy {sloppy} r{recon}: iters {info_na['iters']} vs {info_ref['iters']}, "
          f"oracle true residual {tr:.2e}, max |x - x_cg| {np.abs(xn - xr).max():.2e}", flush=True)
    assert info_na["converged"] == 1 and tr <= 1e-10
    assert info_na["iters"] == info_ref["iters"]
    assert info_na["reliable_updates"] == info_ref["reliable_updates"]
    assert np.array_equal(xn, xr)
    lat.close()


def test_noalloc_cg_matches_cg_two_calls():
    import torch
    from paper_1712_00143_amd import hisq as H
    print("noalloc call 1: 8x8x8x16 mixed FP32", flush=True)
    _solve_pair(H, torch, (8, 8, 8, 16), 0.2, 7100, 0.05, 1, 18)
    print("noalloc call 2: 6x4x4x6 plain FP64 (smaller)", flush=True)
    _solve_pair(H, torch, (6, 4, 4, 6), 0.3, 7200, 0.1, 0, 18)
    print("noalloc call 3: 4x4x4x8 mixed FP16 recon-12 (smaller again)", flush=True)
    _solve_pair(H, torch, (4, 4, 4, 8), 0.25, 7300, 0.1, 2, 12)


def test_noalloc_cg_errors():
    import torch
    from paper_1712_00143_amd import hisq as H
    dims = (4, 4, 4, 4)
    fat, lng = synth.make_links(dims, 0.3, seed=7400)
    lat = H.Lattice(dims)
    lat.load_links(fat, lng)
    b = synth.gaussian_even(dims, 7401)
    bd = torch.from_numpy(b.view(np.float64).ravel()).cuda()
    xd = torch.zeros_like(bd)
    with pytest.raises(H.HisqError) as ei:                    # host vectors
        lat.cg_noalloc(0.1, b, np.zeros_like(b))
    assert ei.value.status == H.HISQ_ERR_ARG
    with pytest.raises(H.HisqError) as ei:                    # graphs allocate
        lat.cg_noalloc(0.1, bd, xd, params=H.hisq_default_params(flags=H.HISQ_USE_GRAPH))
    assert ei.value.status == H.HISQ_ERR_ARG
    with pytest.raises(H.HisqError) as ei:                    # sloppy set not prepared
        lat.cg_noalloc(0.1, bd, xd, params=H.hisq_default_params(sloppy=1))
    assert ei.value.status == H.HISQ_ERR_STATE
    lat.close()
    big = H.Lattice((32, 32, 32, 32))                         # work set beyond the 64 MiB buffer
    bb = torch.zeros(big.h * 6, dtype=torch.float64, device="cuda")
    with pytest.raises(H.HisqError) as ei:
        big.cg_noalloc(0.1, bb, torch.zeros_like(bb))
    assert ei.value.status == H.HISQ_ERR_ARG
    big.close()
