"""The device reciprocal square root every pair evaluation uses (hardware
estimate plus one third-order refinement) against a correctly rounded
1/sqrt(x), over the whole range the integrators feed it, including the
large-n kernels' r^2 floor of 1e-100.  Bar: at most 1 ulp."""
import decimal
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def inputs():
    rng = np.random.default_rng(5)
    parts = [
        10.0 ** rng.uniform(-100, 100, 400000),                  # every scale of r^2
        rng.uniform(1.0, 4.0, 200000),                           # every mantissa (1/sqrt period 4)
        np.ldexp(1.0, np.arange(-330, 331, 2)).astype(np.float64),  # exact even powers of 2
        np.array([1e-100, 1e100, 1.0, 2.0, 3.0, 0.5, 4.0 - 2 ** -50]),
        np.nextafter(1.0, 2.0) + np.arange(64) * np.spacing(1.0),  # just above 1
        1.0 - np.arange(1, 65) * np.spacing(0.5),                # just below 1
    ]
    return np.concatenate(parts)


def ulp_error(x, y):
    """|y - 1/sqrt(x)| in units of the last place of y, with the reference
    in extended precision (64-bit significand) or, where long double is no
    wider than double, in 40-digit decimal."""
    if np.finfo(np.longdouble).nmant >= 63:
        ref = np.longdouble(1) / np.sqrt(x.astype(np.longdouble))
        return np.abs((y.astype(np.longdouble) - ref) / np.spacing(y).astype(np.longdouble)).astype(np.float64)
    decimal.getcontext().prec = 40
    out = np.empty(len(x))
    for i, (xi, yi) in enumerate(zip(x, y)):
        r = 1 / decimal.Decimal(float(xi)).sqrt()
        out[i] = float(abs(decimal.Decimal(float(yi)) - r) / decimal.Decimal(float(np.spacing(yi))))
    return out


def test_rsqrt_within_one_ulp(fb):
    import torch
    x = inputs()
    say("rsqrt", x.size, "values")
    y = fb.eval_rsqrt(torch.from_numpy(x).cuda()).cpu().numpy()
    err = ulp_error(x, y)
    worst = int(np.argmax(err))
    say("max ulp error", err.max(), "at x =", x[worst], "mean", err.mean(),
        "fraction above 0.5 ulp", np.mean(err > 0.5))
    assert err.max() <= 1.0, (err.max(), x[worst], y[worst])
    # spot check of the extended-precision reference against 40 digits
    decimal.getcontext().prec = 40
    for i in np.random.default_rng(6).choice(x.size, 200, replace=False):
        r = 1 / decimal.Decimal(float(x[i])).sqrt()
        e = float(abs(decimal.Decimal(float(y[i])) - r) / decimal.Decimal(float(np.spacing(y[i]))))
        assert abs(e - err[i]) < 1e-3, (x[i], e, err[i])
    # exact even powers of two: the root is a power of two, so exact
    p = np.ldexp(1.0, np.arange(-330, 331, 2))
    yp = fb.eval_rsqrt(torch.from_numpy(p).cuda()).cpu().numpy()
    assert np.array_equal(yp, np.ldexp(1.0, -np.arange(-330, 331, 2) // 2))
