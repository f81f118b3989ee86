"""The allocation-free read-back (pulbm_read_fields_noalloc) against
pulbm_read_fields through the C ABI: bit for bit on two calls in a row on
different cases, the second smaller (2D after 3D), then the larger again, in
FP32, FP64 and FP16 storage; a case beyond the fixed staging array is refused
with EINVAL and the case stays readable."""
import numpy as np
import pytest

from paper_2512_01027_amd import binding as B
from paper_2512_01027_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(cfg, R, steps, seed):
    phi, P, u = W.droplet(cfg, R, center=(cfg["nx"] * 0.45, cfg["ny"] * 0.55, cfg["nz"] * 0.5))
    phi = np.clip(phi + W.random_smooth(cfg, seed, amp=0.02), 0, 1)
    c = B.Case(cfg)
    c.init_fields(phi, P, u)
    c.step(steps)
    return c


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("store", ["fp32", "fp64", "fp16"])
def test_noalloc_read_equals_read_fields(store):
    big = _case(W.base_case(3, 70, 41, 23, wall=(0, 0, 1), gravity=(0.0, 0.0, -1e-5), store=store), 8.0, 9, 3)
    small = _case(W.base_case(2, 37, 29, sigma=0.01, store=store), 7.0, 13, 4)
    rb = big.read_fields()
    rs = small.read_fields()
    assert _same(big.read_fields_noalloc(), rb)
    assert _same(small.read_fields_noalloc(), rs)  # the second call, on a smaller case
    assert _same(big.read_fields_noalloc(), rb)
    # the state is not changed by either read: stepping on gives the same
    big.step(2)
    assert _same(big.read_fields_noalloc(), big.read_fields())
    big.close()
    small.close()


def test_noalloc_read_rejects_a_case_beyond_the_array():
    c = _case(W.base_case(3, 120, 120, 120, store="fp32"), 20.0, 1, 5)
    with pytest.raises(B.PulbmError) as e:
        c.read_fields_noalloc()
    assert e.value.code == B.EINVAL
    assert "allocation-free" in str(e.value)
    phi, _, _ = c.read_fields()
    assert np.isfinite(phi).all()
    c.close()
