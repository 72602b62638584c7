"""afc_step_ssprk3_noalloc (work vectors in the library's fixed per-GPU array)
against afc_step_ssprk3 through the C ABI: two calls in a row, the second on
a smaller problem, and its refusals."""
import numpy as np
import pytest

from paper_2110_15676_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _afc():
    from paper_2110_15676_amd import afc

    return afc


def _opts(**kw):
    afc = _afc()
    o = afc.afc_default_options(**kw)
    o.stream = torch.cuda.current_stream().cuda_stream
    return o


def _dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda:0")


def _rel(a, b):
    l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    mx = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
    return float(max(l2, mx))


def _pair(inst, stages):
    """Two handles of the same instance: one for each entry point.  The
    no-alloc handle gets its explicit-stage coefficients from one ordinary
    step on a scratch copy of u (the entry point builds nothing itself)."""
    afc = _afc()
    ha = afc.afc_create_instance(inst, _opts(ssp_stages=stages), conv=False)
    hb = afc.afc_create_instance(inst, _opts(ssp_stages=stages), conv=False)
    F = _dev(inst.F)
    afc.afc_step_ssprk3(hb, _dev(inst.u0), F, inst.params["dt"])
    return ha, hb, F


@pytest.mark.parametrize("stages", [3, 2, 1])
def test_noalloc_matches_ssprk3_on_two_calls_second_smaller(stages):
    afc = _afc()
    for n in (24, 10):  # the second call's problem is smaller than the first's
        inst = I.config2(n)
        dt = inst.params["dt"]
        print("noalloc stages=%d n=%d N=%d" % (stages, n, inst.N), flush=True)
        ha, hb, F = _pair(inst, stages)
        try:
            ua = _dev(inst.u0)
            ub = _dev(inst.u0)
            for _ in range(2):
                sa, _ = afc.afc_step_ssprk3(ha, ua, F, dt)
                sb, stb = afc.afc_step_ssprk3_noalloc(hb, ub, F, dt)
                assert sa == 0 and sb == 0, stb
            x, y = ua.cpu().numpy(), ub.cpu().numpy()
            assert _rel(y, x) <= 1e-12
            assert np.array_equal(x, y)  # same kernels on the same data
        finally:
            afc.afc_destroy(ha)
            afc.afc_destroy(hb)


def test_noalloc_refuses_what_it_cannot_do_without_allocating():
    afc = _afc()
    inst = I.config2(8)
    dt = inst.params["dt"]
    h = afc.afc_create_instance(inst, _opts(), conv=False)
    try:
        u = _dev(inst.u0)
        F = _dev(inst.F)
        # a fresh handle has no slot-order coefficients yet
        st, _ = afc.afc_step_ssprk3_noalloc(h, u, F, dt, raise_on_error=False)
        assert st == afc.AFC_EINVAL and "not built" in afc.afc_last_error(h)
        assert np.array_equal(u.cpu().numpy(), inst.u0)
        afc.afc_step_ssprk3(h, u.clone(), F, dt)
        st, _ = afc.afc_step_ssprk3_noalloc(h, u, F, -1.0, raise_on_error=False)
        assert st == afc.AFC_EINVAL
        afc.afc_set_options(h, _opts(profile=1))
        st, _ = afc.afc_step_ssprk3_noalloc(h, u, F, dt, raise_on_error=False)
        assert st == afc.AFC_EINVAL and "profil" in afc.afc_last_error(h)
        assert np.array_equal(u.cpu().numpy(), inst.u0)
    finally:
        afc.afc_destroy(h)


def test_noalloc_refuses_a_problem_beyond_its_array():
    """Q1 113^3 (1,481,544 nodes): six work vectors need 71.1 MB > 64 MiB."""
    afc = _afc()
    inst = I.config3(113)
    assert 6 * ((inst.N + 63) // 64) * 64 * 8 > afc.AFC_NOALLOC_SCRATCH_BYTES
    h = afc.afc_create_instance(inst, _opts(), conv=True)
    try:
        u = torch.zeros(inst.N, dtype=torch.float64, device="cuda:0")
        F = _dev(inst.F)
        st, _ = afc.afc_step_ssprk3_noalloc(h, u, F, 1e-3, raise_on_error=False)
        assert st == afc.AFC_EINVAL and "work space" in afc.afc_last_error(h)
        assert float(u.abs().max()) == 0.0
    finally:
        afc.afc_destroy(h)
