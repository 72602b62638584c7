"""Handles created on a non-default stream: every setup copy and fill must be
ordered on that stream (regression: the SELL padding fill used to run on the
null stream and could overwrite the converted matrix)."""
import numpy as np
import pytest

from paper_2110_15676_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solve(inst, stream, prec):
    from paper_2110_15676_amd import afc

    with torch.cuda.stream(stream):
        o = afc.afc_default_options(precision=prec, fp_tol=1e-8, fp_tol_mode=afc.AFC_TOL_REL, fp_maxit=300,
                                    lin_atol=0.0, lin_rtol=1e-10)
        o.stream = stream.cuda_stream
        h = afc.afc_create_instance(inst, o, conv=True)
        try:
            u = torch.zeros(inst.N, dtype=torch.float64, device="cuda:0")
            F = torch.tensor(inst.F, device="cuda:0")
            stream.synchronize()
            st, stats = afc.afc_solve_stationary(h, u, F, init_low_order=True)
            return st, u.cpu().numpy(), stats
        finally:
            afc.afc_destroy(h)


@pytest.mark.parametrize("prec", [0, 1])
def test_side_stream_matches_default_stream(prec):
    inst = I.config3(14)
    ref = _solve(inst, torch.cuda.default_stream(), prec)
    side = torch.cuda.Stream()
    got = _solve(inst, side, prec)
    assert ref[0] >= 0 and got[0] >= 0
    assert got[2]["fp_iters"] == ref[2]["fp_iters"]
    assert np.array_equal(got[1], ref[1])
