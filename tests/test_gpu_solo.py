"""Stateless batch steps (fb_hermite_steps_device): a homogeneous batch in
the caller's device tensors, integrated in place with a caller workspace.
It runs the ensemble's kernels and plan, so it must equal the ensemble path
bitwise, and the oracle to 1e-10."""
import math
import sys

import numpy as np
import pytest

from paper_1208_1157_amd import gen
from tests.helpers import assert_parity, oracle_fixed

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def tensors(ens):
    import torch
    return (torch.from_numpy(ens.mass.copy()).cuda(), torch.from_numpy(ens.pos.copy()).cuda(),
            torch.from_numpy(ens.vel.copy()).cuda())


@pytest.mark.parametrize("n,n_sys", [(3, 1000), (6, 333), (11, 70), (16, 5)])
def test_equals_ensemble_path_and_oracle(fb, ora, n, n_sys):
    import torch
    ens = gen.ragged_hill(n_sys, seed=40 + n, n_lo=n, n_hi=n)
    h, steps = 2 * math.pi / 2000, 120
    say("solo steps", n, n_sys)
    m, x, v = tensors(ens)
    status = torch.full((n_sys,), -1, dtype=torch.int32, device="cuda")
    fb.hermite_steps_device(n, m, x, v, steps, h, status=status)
    torch.cuda.synchronize()
    E = fb.from_gen(ens)
    E.integrate_steps(steps, h)
    ref = E.state()
    E.close()
    assert np.array_equal(x.cpu().numpy(), ref["pos"]) and np.array_equal(v.cpu().numpy(), ref["vel"])
    assert np.array_equal(status.cpu().numpy(), ref["status"]) and np.all(ref["status"] == fb.DONE)
    assert np.array_equal(m.cpu().numpy(), ens.mass)
    X, V, _, _ = oracle_fixed(ora, ens, h, steps)
    assert_parity(ens.n_body, x.cpu().numpy(), v.cpu().numpy(), X, V, label=f"solo n={n}")


def test_argument_checks(fb):
    import torch
    m = torch.ones(6, dtype=torch.float64, device="cuda")
    x = torch.zeros(6, 3, dtype=torch.float64, device="cuda")
    v = torch.zeros(6, 3, dtype=torch.float64, device="cuda")
    for n, steps, dt in ((17, 1, 0.1), (3, -1, 0.1), (3, 1, 0.0), (3, 1, float("nan"))):
        with pytest.raises(fb.FewbodyError) as ei:
            fb.hermite_steps_device(n, m, x, v, steps, dt)
        assert ei.value.code == fb.E_INVAL, (n, steps, dt)
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(fb.FewbodyError) as ei:
        fb.hermite_steps_device(3, m, x, v, 1, 0.1, workspace=small)
    assert ei.value.code == fb.E_NOMEM
    assert fb.lib().fb_hermite_steps_workspace_bytes(10, 17) == 0
