"""Host-side arithmetic the kernels rely on, checked on the CPU."""
import numpy as np


def _mulhi_div(n, d):
    """Quotient by the reciprocal m = ceil(2^32 / d), as the site decomposition
    computes it: floor(n * m / 2^32)."""
    m = ((1 << 32) + d - 1) // d
    return (n * m) >> 32


def test_reciprocal_division_exact_when_n_times_d_fits():
    """n // d == umulhi(n, ceil(2^32/d)) whenever n * d <= 2^32 (the bound the
    library checks before using it: V * max(L0, L1, L2) <= 2^32)."""
    rng = np.random.default_rng(5)
    for d in list(range(2, 300)) + [384, 512, 1000, 1024, 4096, 65535]:
        nmax = (1 << 32) // d
        ns = set(int(v) for v in rng.integers(0, nmax + 1, 2000))
        # the worst cases sit just below multiples of d and at the bound
        ns.update(range(max(0, nmax - 3 * d), nmax + 1))
        ns.update(k * d - 1 for k in range(1, 50) if k * d - 1 <= nmax)
        for n in ns:
            assert _mulhi_div(n, d) == n // d, (n, d)


def test_reciprocal_division_bound_is_needed():
    """Beyond the bound the shortcut fails for some n, so the check matters."""
    d = 3
    m = ((1 << 32) + d - 1) // d
    bad = [n for n in range((1 << 32) // d, (1 << 32) // d + 5 * (1 << 31) // d, 7919)
           if (n * m) >> 32 != n // d]
    assert bad
