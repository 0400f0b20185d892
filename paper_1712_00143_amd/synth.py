"""Seeded synthetic inputs for the HISQ Dslash / CG workloads.

This module builds the *inputs* of the solver: gauge links, sources and
per-problem parameters.  It contains none of the solver's arithmetic (no
Dslash, no Krylov recurrences, no preconditioner): both the HIP library and
the CPU oracle consume the arrays it returns, and nothing else is shared
between them.

Recipe (the paper benchmarks an equilibrated 16^4 configuration and L^4 per
node volume sweeps, Section 4 and Section 4.1; those ensembles are not
available, so seeded synthetic fields of the same shapes stand in for them):

* base links  F~_mu(x) = 0.9 * exp(i*eps*H),  H = sum_a omega_a lambda_a / 2,
  omega_a ~ N(0,1), lambda_a the Gell-Mann matrices (exp by Hermitian
  eigendecomposition);
* long links  L~_mu(x) = -(1/24) F~_mu(x) F~_mu(x+mu) F~_mu(x+2mu);
* staggered phases eta_mu(x) = (-1)^(x_0+...+x_{mu-1}) folded into both;
* sources: complex Gaussian (Re, Im ~ N(0,1)) on even sites.

Layout of every link array: complex128 ``[V][4][3][3]`` with the site index
lex(x) = x0 + L0*(x1 + L1*(x2 + L2*x3)) (x fastest) and mu = 0..3 <-> x,y,z,t.
Even-parity vectors: complex128 ``[V/2][3]`` indexed by lex(x)//2 over even
sites (valid because L0 is even).

Seeds: field j of workload c uses ``1000*c + j``; its sources ``+500``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1] = -1j
_GELL_MANN[1][1, 0] = 1j
_GELL_MANN[2][0, 0] = 1
_GELL_MANN[2][1, 1] = -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2] = -1j
_GELL_MANN[4][2, 0] = 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2] = -1j
_GELL_MANN[6][2, 1] = 1j
_GELL_MANN[7][0, 0] = _GELL_MANN[7][1, 1] = 1 / math.sqrt(3)
_GELL_MANN[7][2, 2] = -2 / math.sqrt(3)

FAT_SCALE = 0.9


def volume(dims) -> int:
    return int(np.prod(dims))


def check_dims(dims) -> tuple:
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError(f"lattice extents must be 4 even numbers >= 2, got {dims}")
    return dims


def coords(dims) -> np.ndarray:
    """Integer coordinates [V][4] in lex order (x fastest)."""
    L0, L1, L2, L3 = dims
    t, z, y, x = np.meshgrid(np.arange(L3), np.arange(L2), np.arange(L1),
                             np.arange(L0), indexing="ij")
    return np.stack([x, y, z, t], axis=-1).reshape(-1, 4)


def staggered_phases(dims) -> np.ndarray:
    """eta_mu(x) = (-1)^(sum_{nu<mu} x_nu) as float [V][4]."""
    c = coords(dims)
    eta = np.ones((c.shape[0], 4))
    for mu in range(1, 4):
        eta[:, mu] = (-1.0) ** (c[:, :mu].sum(axis=1) % 2)
    return eta


def even_sites(dims) -> np.ndarray:
    """lex indices of the even sites, in the order of the even-vector index."""
    c = coords(dims)
    return np.nonzero(c.sum(axis=1) % 2 == 0)[0]


def odd_sites(dims) -> np.ndarray:
    c = coords(dims)
    return np.nonzero(c.sum(axis=1) % 2 == 1)[0]


def _expi_hermitian(H: np.ndarray) -> np.ndarray:
    w, v = np.linalg.eigh(H)
    return (v * np.exp(1j * w)[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def _su3_field(dims, eps: float, seed: int) -> np.ndarray:
    dims = check_dims(dims)
    V = volume(dims)
    rng = np.random.default_rng(seed)
    omega = rng.standard_normal((V, 4, 8))
    H = np.einsum("sma,aij->smij", omega, _GELL_MANN / 2.0)
    return _expi_hermitian(eps * H)


def base_links(dims, eps: float, seed: int) -> np.ndarray:
    """Unphased F~ = 0.9 exp(i eps H) as complex128 [V][4][3][3]."""
    return FAT_SCALE * _su3_field(dims, eps, seed)


def thin_links(dims, eps: float, seed: int) -> np.ndarray:
    """Thin gauge links U = exp(i eps H) in SU(3), unphased, [V][4][3][3]:
    the input of the HISQ smearing."""
    return _su3_field(dims, eps, seed)


def tile_field(field: np.ndarray, dims, reps) -> np.ndarray:
    """Periodic copy of a site-major field [V, ...] on the lattice
    dims * reps (each extent repeated reps[mu] times)."""
    L0, L1, L2, L3 = dims
    f = field.reshape((L3, L2, L1, L0) + field.shape[1:])
    f = np.tile(f, (reps[3], reps[2], reps[1], reps[0]) + (1,) * (field.ndim - 1))
    return f.reshape((-1,) + field.shape[1:])


def gauge_transform(links: np.ndarray, dims, g: np.ndarray) -> np.ndarray:
    """U'_mu(x) = g(x) U_mu(x) g(x+mu)^+ for site matrices g [V][3][3]."""
    out = np.empty_like(links)
    for mu in range(4):
        out[:, mu] = g @ links[:, mu] @ np.conj(np.swapaxes(_shift(g, dims, mu, 1), -1, -2))
    return out


def _shift(field: np.ndarray, dims, mu: int, k: int) -> np.ndarray:
    """field(x + k*mu) for a site-major array [V, ...]."""
    L0, L1, L2, L3 = dims
    f = field.reshape((L3, L2, L1, L0) + field.shape[1:])
    axis = 3 - mu
    return np.roll(f, -k, axis=axis).reshape(field.shape)


def long_from_base(fat_base: np.ndarray, dims) -> np.ndarray:
    """L~_mu(x) = -(1/24) F~_mu(x) F~_mu(x+mu) F~_mu(x+2mu) (unphased)."""
    out = np.empty_like(fat_base)
    for mu in range(4):
        f = fat_base[:, mu]
        out[:, mu] = -(1.0 / 24.0) * (f @ _shift(f, dims, mu, 1) @ _shift(f, dims, mu, 2))
    return out


def fold_phases(links: np.ndarray, dims) -> np.ndarray:
    return links * staggered_phases(dims)[:, :, None, None]


def make_links(dims, eps: float, seed: int, phased: bool = True):
    """(fat, long) complex128 [V][4][3][3], staggered phases folded in."""
    dims = check_dims(dims)
    fb = base_links(dims, eps, seed)
    lb = long_from_base(fb, dims)
    if not phased:
        return fb, lb
    return fold_phases(fb, dims), fold_phases(lb, dims)


def unit_links(dims, phased: bool = True):
    """Free field: F~ = 1, L~ = -1/24 (so that L = F F F * -1/24)."""
    dims = check_dims(dims)
    V = volume(dims)
    fb = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()
    lb = -(1.0 / 24.0) * fb
    if not phased:
        return fb, lb
    return fold_phases(fb, dims), fold_phases(lb, dims)


def gaussian_even(dims, seed: int, nvec: int | None = None) -> np.ndarray:
    """Complex Gaussian source(s) on even sites: [h][3] (or [nvec][h][3])."""
    dims = check_dims(dims)
    h = volume(dims) // 2
    rng = np.random.default_rng(seed)
    shape = (h, 3) if nvec is None else (nvec, h, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def gaussian_full(dims, seed: int, nchan: int = 1) -> np.ndarray:
    dims = check_dims(dims)
    rng = np.random.default_rng(seed)
    shape = (nchan, volume(dims), 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-ish random SU(3) matrices (QR of a complex Gaussian, det fixed)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]


def shifts_log(n: int = 12, lo: float = 1e-4, hi: float = 1.0) -> np.ndarray:
    """n shifts log-spaced in [lo, hi], endpoints included."""
    return np.logspace(math.log10(lo), math.log10(hi), n)


@dataclass
class Workload:
    """One named workload: lattice, link recipe, mass, sources."""
    name: str
    dims: tuple
    eps: float
    mass: float
    seed: int
    nsrc: int = 1

    def links(self):
        return make_links(self.dims, self.eps, self.seed)

    def sources(self):
        return gaussian_even(self.dims, self.seed + 500, self.nsrc)


# The five workloads (seeds 1000*c + j).
C0 = Workload("plain-fp64-cg-4^4", (4, 4, 4, 4), 0.3, 0.1, 0, 1)
C1 = Workload("mixed-cg-16^3x32", (16, 16, 16, 32), 0.2, 0.02, 1000, 4)
C2 = Workload("multishift-24^3x48", (24, 24, 24, 48), 0.2, 0.01, 2000, 4)
C4 = Workload("learned-fcg-16^4", (16, 16, 16, 16), 0.25, 0.005, 4000, 4)


def batch_workload(nper: int = 16, seed0: int = 3000):
    """The uneven batch: nper each of 8^4, 12^4, 16^4, 16^3x32.

    eps ~ U[0.1, 0.4], mass ~ logU[0.005, 0.2], one source each.  Returns a
    list of Workload objects (field j uses seed 3000 + j).
    """
    shapes = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (16, 16, 16, 32)]
    rng = np.random.default_rng(seed0 + 999)
    out = []
    j = 0
    for s in shapes:
        for _ in range(nper):
            eps = float(rng.uniform(0.1, 0.4))
            mass = float(math.exp(rng.uniform(math.log(0.005), math.log(0.2))))
            out.append(Workload(f"batch-{j}", s, eps, mass, seed0 + j, 1))
            j += 1
    return out
