"""The temperature solve interpolates an inverse table of the emission per unit mass,
S(T) = sum kappa_abs B_nu(T) dnu, with 65536 entries in ln S between S(2 K) and S(3000 K) and a
cubic Hermite in ln T(ln S) between entries, and takes no Newton step after it.  This pins the
table size: on the dust tables of the workloads, the interpolated ln T at points between
entries equals the Newton root of the same sum to rounding (numpy, FP64; the device code is
held to the oracle's bisection within 1e-10 by the GPU parity tests)."""
import numpy as np
import pytest

import gen

H, K, C = 6.62607015e-27, 1.380649e-16, 2.99792458e10
N_TAB = 65536


def _sums(t, nu, dnu, kabs):
    x = H * nu[None, :] / (K * t[:, None])
    with np.errstate(over="ignore", invalid="ignore"):
        em = np.expm1(x)
        b = 2.0 * H * nu ** 3 / C ** 2 / em
        dterm = np.where(np.isfinite(em), b * x * ((em + 1.0) / em), 0.0)
    return (kabs * b * dnu).sum(1), (kabs * dnu * dterm / t[:, None]).sum(1)


def _root(y, nu, dnu, kabs, lo, hi):
    u = np.full_like(y, 0.5 * (lo + hi))
    for _ in range(100):
        t = np.exp(u)
        s, ds = _sums(t, nu, dnu, kabs)
        u = np.clip(u - (np.log(s) - y) / (t * ds / s), lo, hi)
    return u


@pytest.mark.parametrize("make", [lambda: gen.c5(packets=1), lambda: gen.c2(packets=1),
                                  lambda: gen.c3(packets=1)])
def test_table_interpolation_is_the_root(make):
    d = make().dusts[0]
    nu = C / (d.lambda_um * 1e-4)
    o = np.argsort(nu)
    nu = nu[o]
    dnu = np.empty_like(nu)
    dnu[1:-1] = 0.5 * (nu[2:] - nu[:-2])
    dnu[0], dnu[-1] = 0.5 * (nu[1] - nu[0]), 0.5 * (nu[-1] - nu[-2])
    kabs = ((1.0 - d.albedo) * d.kappa_ext)[o]
    lo, hi = np.log(2.0), np.log(3000.0)
    s_lo, _ = _sums(np.array([2.0]), nu, dnu, kabs)
    s_hi, _ = _sums(np.array([3000.0]), nu, dnu, kabs)
    y0 = np.log(s_lo[0])
    dy = (np.log(s_hi[0]) - y0) / (N_TAB - 1)
    i = np.random.default_rng(3).integers(0, N_TAB - 1, 1500)
    f = np.random.default_rng(4).uniform(0.0, 1.0, i.size)
    u0 = _root(y0 + i * dy, nu, dnu, kabs, lo, hi)
    u1 = _root(y0 + (i + 1) * dy, nu, dnu, kabs, lo, hi)
    ue = _root(y0 + (i + f) * dy, nu, dnu, kabs, lo, hi)
    s0, ds0 = _sums(np.exp(u0), nu, dnu, kabs)
    s1, ds1 = _sums(np.exp(u1), nu, dnu, kabs)
    g0, g1 = s0 / (np.exp(u0) * ds0) * dy, s1 / (np.exp(u1) * ds1) * dy
    f2, f3 = f * f, f * f * f
    u = (2 * f3 - 3 * f2 + 1) * u0 + (f3 - 2 * f2 + f) * g0 + (3 * f2 - 2 * f3) * u1 + (f3 - f2) * g1
    assert np.abs(u - ue).max() < 1e-13
