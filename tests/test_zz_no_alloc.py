"""GPU check of kc_grad_params_noalloc, the gradient entry point that uses a
static device array instead of a hierarchy and workspace: its results equal
kc_grad_params' (same kernels, same tiles, same merge order) on two calls in
a row, the second with a smaller input, and inputs beyond its fixed size are
rejected on the host."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def test_noalloc_gradient_equals_hierarchy_gradient():
    from paper_2010_00626_amd import kcycle as K
    print("[no-alloc] two calls, the second smaller", flush=True)
    rng = np.random.default_rng(21)
    for specs in ([(511, 0.4, 1e-3), (127, 2.2, 0.05), (1023, 1.0, 1e-4)], [(63, 0.1, 1e-2)]):
        lams = [dev(rng.uniform(-1, 1, (s[0], s[0]))) for s in specs]
        us = [dev(rng.uniform(-1, 1, (s[0], s[0]))) for s in specs]
        H = K.Hierarchy(specs)
        ref_t, ref_e = H.grad_params(lams, us)
        H.close()
        got_t, got_e = K.grad_params_noalloc(specs, lams, us)
        assert got_t == ref_t and got_e == ref_e, (specs, got_t, ref_t, got_e, ref_e)
    # a pitched array (ld > n) as well
    n = 255
    big_l = dev(rng.uniform(-1, 1, (n, n + 37)))
    big_u = dev(rng.uniform(-1, 1, (n, n + 37)))
    lam, u = big_l[:, :n], big_u[:, :n]
    H = K.Hierarchy([(n, 0.9, 3e-3)])
    ref = H.grad_params([lam], [u])
    H.close()
    assert K.grad_params_noalloc([(n, 0.9, 3e-3)], [lam], [u]) == ref


def test_noalloc_rejects_inputs_beyond_its_size():
    from paper_2010_00626_amd import kcycle as K
    print("[no-alloc] size limits", flush=True)
    one = [torch.zeros((1, 1), dtype=torch.float64, device="cuda")]
    with pytest.raises(K.KCycleError):
        K.grad_params_noalloc([(1, 0.3, 1e-3)] * 65, one * 65, one * 65)
    n = 16383
    x = [torch.empty((n, n), dtype=torch.float64, device="cuda") for _ in range(2)]
    with pytest.raises(K.KCycleError) as e:
        K.grad_params_noalloc([(n, 0.3, 1e-3)] * 2, x, x)
    assert "scratch" in str(e.value)
    del x
    torch.cuda.empty_cache()
