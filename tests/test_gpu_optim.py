"""GPU: the Adam step over surfel parameters (gs2d_params_adam) against the oracle
(oracle/optim.py), three steps in a row on seeded data, at ragged and large sizes, with
the clamps active on some entries."""

import numpy as np
import pytest
import torch

from oracle import optim
from tests.gpu_common import dev, host

pytestmark = pytest.mark.gpu

LR = (1.6e-4, 1e-3, 2e-3, 5e-3, 5e-2, 2.5e-3)


@pytest.fixture(scope="module")
def ms():
    from paper_2506_00970_amd import mapstate

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return mapstate


@pytest.mark.parametrize("n", [1, 3, 4096, 300_001])
def test_params_adam_matches_oracle(ms, n):
    g = np.random.default_rng(n)
    p = g.uniform(0.0, 1.0, (15, n)).astype(np.float32)
    p[9:11] = g.uniform(1e-4, 0.05, (2, n))
    p[11] = g.uniform(0.0, 1.0, n)
    P = dev(p)
    opt = ms.ParamAdam(P, lr=LR, eps=1e-8, weight_decay=0.01, s_min=1e-3, o_min=0.01, o_max=0.99)
    rp, rm, rv = p.astype(np.float64), np.zeros((15, n)), np.zeros((15, n))
    for t in range(1, 4):
        grad = g.standard_normal((15, n)).astype(np.float32)
        opt.step(P, dev(grad))
        torch.cuda.synchronize()
        # the ABI's constants are float32: the oracle takes the same float32 values
        f = lambda x: float(np.float32(x))
        rp, rm, rv = optim.adam_step(rp, grad, rm, rv, t, [f(x) for x in LR], beta1=f(0.9), beta2=f(0.999),
                                     eps=f(1e-8), weight_decay=f(0.01), s_min=f(1e-3), o_min=f(0.01), o_max=f(0.99))
        got = host(P)
        np.testing.assert_allclose(got, rp, rtol=0, atol=2e-7 * np.maximum(1.0, np.abs(rp)).max())
        np.testing.assert_allclose(host(opt.m), rm, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(host(opt.v), rv, rtol=1e-5, atol=1e-9)
        rp = got.astype(np.float64)  # continue both from the device's float32 state
        rm, rv = host(opt.m), host(opt.v)
    assert np.any(got[9:11] == np.float32(1e-3)) or n < 100  # the clamps were hit
