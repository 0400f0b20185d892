"""Element-wise parity bars shared by the GPU tests.

rel_l2 is the relative l2 error over the whole field.  A global norm hides a
bug confined to a few sites (one wrong site of 524 288 adds about 1.4e-3 to
the relative l2 error), so every parity check also bounds the error of each
site: max_s |out_s - ref_s| over the root-mean-square site norm of ref,
against SITE_FACTOR times the l2 bar.  For rounding errors spread over all
sites the per-site maximum stays within a few times the l2 value (the
largest of 10^5-10^6 chi-square samples with 6 degrees of freedom is about
2.5 times their rms); a wrong site is off by about its own norm.
"""
import numpy as np

SITE_FACTOR = 10.0


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def site_max(a, b):
    """Largest per-site error over the rms site norm of b; a and b are
    [..., sites, 3] complex arrays (a site is the last axis)."""
    a = np.asarray(a).reshape(-1, np.asarray(a).shape[-1])
    b = np.asarray(b).reshape(-1, np.asarray(b).shape[-1])
    err = np.linalg.norm(a - b, axis=1)
    rms = np.linalg.norm(b) / np.sqrt(b.shape[0])
    return float(err.max() / rms)


def check(out, ref, tol, what=""):
    """Assert the relative l2 bar and the per-site bar; returns both values."""
    r, s = rel_l2(out, ref), site_max(out, ref)
    assert r <= tol, (what, "rel l2", r, tol)
    assert s <= SITE_FACTOR * tol, (what, "per-site max", s, SITE_FACTOR * tol)
    return r, s
