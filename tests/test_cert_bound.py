"""The certified scan's half-width, checked on the CPU against float32 models of
the matrix-core form.

The certified FP32 scan (search tile 16) rejects a (row, query) pair when
Dt - e exceeds the query's current k-th canonical value, where
Dt = fl(|q|^2 + |x|^2) - 2 x.q (L2) or -x.q (IP) comes from the matrix cores
and e = e1 (|x|^2 + |q|^2) + e0.  That is safe only if Dt - e never exceeds the
pair's own canonical value (sequential fma over ascending dimensions).  The
matrix cores' summation order is not documented, so the dot product is
modelled here in several float32 orders (sequential, reversed, blocks of 4,
pairwise tree), each product and sum rounded once, on data built to stress
the bound: a large common offset (cancellation), tiny magnitudes
(subnormal terms), integer grids and normal data.  The constants mirror the
kernel's: cf = (5d + 32) 2^-24 (IP: (4d + 32) 2^-24), e1 = 2 cf (IP: cf / 2)
+ sqrt(d) 2^-122, e0 = sqrt(d) 2^-122 + d 2^-120.
"""
import numpy as np
import pytest

F = np.float32


def _fma32(a, b, c):
    """float32 fma: the exact a*b + c rounded once (float64 holds a*b exactly;
    the sum's own float64 rounding is far below a float32 unit here)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F)


def _canonical(q, x, metric):
    r = np.zeros(x.shape[0], F)
    for j in range(x.shape[1]):
        if metric == 0:
            t = (q[j] - x[:, j]).astype(F)
            r = _fma32(t, t, r)
        else:
            r = _fma32(np.full(x.shape[0], q[j], F), x[:, j], r)
    return r


def _dot(q, x, order):
    p = (x * q[None, :]).astype(F)           # products rounded to float32
    d = x.shape[1]
    if order == "seq":
        acc = np.zeros(x.shape[0], F)
        for j in range(d):
            acc = (acc + p[:, j]).astype(F)
        return acc
    if order == "rev":
        acc = np.zeros(x.shape[0], F)
        for j in reversed(range(d)):
            acc = (acc + p[:, j]).astype(F)
        return acc
    if order == "block4":
        acc = np.zeros(x.shape[0], F)
        for j0 in range(0, d, 4):
            s = p[:, j0]
            for j in range(j0 + 1, min(j0 + 4, d)):
                s = (s + p[:, j]).astype(F)
            acc = (acc + s).astype(F)
        return acc
    if order == "tree":
        v = p
        while v.shape[1] > 1:
            if v.shape[1] % 2:
                v = np.concatenate([v, np.zeros((v.shape[0], 1), F)], 1)
            v = (v[:, 0::2] + v[:, 1::2]).astype(F)
        return v[:, 0]
    raise ValueError(order)


def _sqnorm(v):
    """Squared norms by sequential float32 fma, as the kernels store them."""
    r = np.zeros(v.shape[0], F)
    for j in range(v.shape[1]):
        r = _fma32(v[:, j], v[:, j], r)
    return r


def _half_width(d, metric, s):
    u = 2.0 ** -24
    cf = ((5 * d + 32) if metric == 0 else (4 * d + 32)) * u
    ca, cb = np.sqrt(d) * 2.0 ** -122, d * 2.0 ** -120
    e1 = F((2 * cf if metric == 0 else 0.5 * cf) + ca)
    e0 = F(ca + cb)
    return _fma32(np.full(s.shape, e1, F), s, np.full(s.shape, e0, F))


def _data(kind, rng, n, d):
    if kind == "normal":
        return rng.standard_normal((n, d)).astype(F)
    if kind == "offset":
        return (300.0 + rng.standard_normal((n, d))).astype(F)
    if kind == "tiny":
        return (1e-19 * rng.standard_normal((n, d))).astype(F)
    if kind == "grid":
        return rng.integers(0, 256, (n, d)).astype(F)
    raise ValueError(kind)


@pytest.mark.parametrize("metric", [0, 1])
@pytest.mark.parametrize("kind,d", [("normal", 128), ("offset", 96), ("offset", 256), ("tiny", 48),
                                    ("grid", 128), ("normal", 5), ("offset", 17)])
def test_half_width_covers_dot_product_form(kind, d, metric):
    rng = np.random.default_rng([d, metric, len(kind)])
    x = _data(kind, rng, 2000, d)
    q = x[7] + (np.float32(1e-3) * x[7] * rng.standard_normal(d)).astype(F)   # near a row: small distances
    q = q.astype(F)
    xn = _sqnorm(x)
    qn = _sqnorm(q[None, :])[0]
    s = (np.full(x.shape[0], qn, F) + xn).astype(F)
    e = _half_width(d, metric, s)
    r = _canonical(q, x, metric)
    worst = 0.0
    for order in ("seq", "rev", "block4", "tree"):
        acc = _dot(q, x, order)
        if metric == 0:
            dt = _fma32(np.full(acc.shape, F(-2.0), F), acc, s)
            gap = dt.astype(np.float64) - r.astype(np.float64)   # must stay <= e
        else:
            gap = r.astype(np.float64) - acc.astype(np.float64)    # score: canonical <= acc + e
        assert np.all(gap <= e.astype(np.float64)), (order, float((gap / e).max()))
        worst = max(worst, float(np.max(np.abs(gap) / e)))
    assert worst < 0.5, worst   # the bound keeps a factor of two over the modelled errors


def test_half_width_rejects_a_too_small_bound():
    """The offset data needs the d-proportional term: a bound of 4 units of
    2^-24 (|x|^2 + |q|^2), independent of d, is broken by the same models."""
    rng = np.random.default_rng(11)
    d = 256
    x = _data("offset", rng, 2000, d)
    q = (x[3] + np.float32(0.01) * rng.standard_normal(d)).astype(F)
    xn = _sqnorm(x)
    qn = _sqnorm(q[None, :])[0]
    s = (np.full(x.shape[0], qn, F) + xn).astype(F)
    r = _canonical(q, x, 0)
    small = (4 * 2.0 ** -24) * s.astype(np.float64)
    broken = False
    for order in ("seq", "rev", "block4", "tree"):
        dt = _fma32(np.full(x.shape[0], F(-2.0), F), _dot(q, x, order), s)
        broken |= bool(np.any(dt.astype(np.float64) - r.astype(np.float64) > small))
    assert broken
