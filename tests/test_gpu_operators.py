"""The solvers' SELL-64 kernels, one application each, element by element
against the oracle's CSR operator (afc_apply_operator through the C ABI).

A is the stationary MCL low-order operator with Dirichlet identity rows
(Sec. 4, the matrix every refinement residual and Krylov step applies),
D = diag(A).  The outer FP64 refinement would hide an error in an inner SpMV
(the solve still reaches its tolerance, only with more Krylov iterations), so
each kernel is checked here on its own:

* FP64 kernels (refinement residual, FP64 GMRES SpMV, BiCGStab SpMV): every
  entry within 1e-13 of the row's absolute sum sum_j |a_ij| |x_j| (rounding
  of 27 products is a few 1e-16 of it; a wrong or missing neighbour is
  O(1e-2) of it).
* FP32 SpMV of the mixed GMRES: against the same FP32 values (a_ij / a_jj
  rounded to FP32, unit diagonal) and FP32 x, summed in FP64, within 4e-6 of
  the row's absolute sum.
* The FP64 GMRES and BiCGStab SpMVs form D^{-1}_j x_j and sum in slot order
  alike, so they must agree bitwise.

Meshes: Q1 at 12^3 and 20^3 (most slices are full uniform slices whose x
values are taken by stencil runs with lane rotates, the rest gathers), the
same 12^3 problem renumbered (no uniform slices: per-row offsets), and P1
(other patterns).  Seeded random x and y.
"""
import numpy as np
import pytest

from oracle import afc_oracle as O
from paper_2110_15676_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _afc():
    from paper_2110_15676_amd import afc

    return afc


def _dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda:0")


def _instances():
    return {
        "q1_12": lambda: I.config3(12),
        "q1_20": lambda: I.config3(20),
        "q1_12_renumbered": lambda: I.renumbered(I.config3(12)),
        "p1_8": lambda: I.config1(8),
    }


@pytest.mark.parametrize("name", ["q1_12", "q1_20", "q1_12_renumbered", "p1_8"])
def test_sell_kernels_match_the_csr_operator(name):
    afc = _afc()
    inst = _instances()[name]()
    P = O.problem_from_instance(inst, conv=True)
    _, As = O.stationary_matrix(P)
    N = P.N
    rows = np.repeat(np.arange(N), np.diff(P.row_ptr))
    diag = As[P.diag_pos]
    dinv = 1.0 / diag
    rng = np.random.default_rng((7, N))
    x = rng.standard_normal(N)
    y0 = rng.standard_normal(N)
    absA = np.abs(As)

    o = afc.afc_default_options()
    o.stream = torch.cuda.current_stream().cuda_stream
    h = afc.afc_create_instance(inst, o, conv=True)
    try:
        xd = _dev(x)
        print("%s: N=%d, residual kernel" % (name, N), flush=True)
        yd = _dev(y0)
        afc.afc_apply_operator(h, afc.AFC_APPLY_RESIDUAL, xd, yd)
        got = yd.cpu().numpy()
        ref = y0 - P.matvec(As, x)
        scale = np.abs(y0) + P.matvec(absA, np.abs(x))
        err = np.abs(got - ref) / scale
        print("  residual: max error / row abs sum %.2e at row %d" % (err.max(), int(err.argmax())), flush=True)
        assert err.max() <= 1e-13

        z = dinv * x
        ref = P.matvec(As, z)
        scale = P.matvec(absA, np.abs(z))
        outs = {}
        for op, label in ((afc.AFC_APPLY_SCALED64, "FP64 SpMV"), (afc.AFC_APPLY_BICG, "BiCGStab SpMV")):
            print("%s: %s" % (name, label), flush=True)
            yd = _dev(np.full(N, np.nan))
            afc.afc_apply_operator(h, op, xd, yd)
            got = yd.cpu().numpy()
            err = np.abs(got - ref) / scale
            print("  %s: max error / row abs sum %.2e at row %d" % (label, err.max(), int(err.argmax())), flush=True)
            assert np.all(np.isfinite(got))
            assert err.max() <= 1e-13
            outs[op] = got
        assert np.array_equal(outs[afc.AFC_APPLY_SCALED64], outs[afc.AFC_APPLY_BICG])

        print("%s: FP32 SpMV" % name, flush=True)
        off = P.col != rows
        v32 = (As * dinv[P.col]).astype(np.float32).astype(np.float64)
        x32 = x.astype(np.float32).astype(np.float64)
        ref32 = np.zeros(N)
        np.add.at(ref32, rows[off], v32[off] * x32[P.col[off]])
        ref32 += x32
        scale32 = np.abs(x32)
        np.add.at(scale32, rows[off], np.abs(v32[off] * x32[P.col[off]]))
        yd = _dev(np.full(N, np.nan))
        afc.afc_apply_operator(h, afc.AFC_APPLY_SCALED32, xd, yd)
        got = yd.cpu().numpy()
        err = np.abs(got - ref32) / scale32
        print("  FP32 SpMV: max error / row abs sum %.2e at row %d" % (err.max(), int(err.argmax())), flush=True)
        assert err.max() <= 4e-6
    finally:
        afc.afc_destroy(h)


def test_apply_operator_rejects_bad_arguments():
    afc = _afc()
    inst = I.config3(4)
    o = afc.afc_default_options()
    o.stream = torch.cuda.current_stream().cuda_stream
    h = afc.afc_create_instance(inst, o, conv=True)
    try:
        x = _dev(np.ones(inst.N))
        for op in (-1, 4):
            with pytest.raises(afc.AFCError):
                afc.afc_apply_operator(h, op, x, _dev(np.zeros(inst.N)))
        with pytest.raises(afc.AFCError):
            afc.afc_apply_operator(h, afc.AFC_APPLY_SCALED64, x, x)  # aliased
    finally:
        afc.afc_destroy(h)
