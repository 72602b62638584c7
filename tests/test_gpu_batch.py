"""Batched persistent CN-FCT launch through the C ABI: parity with the oracle
per instance, and every instance bitwise the same alone and in the mix."""
import numpy as np
import pytest

from oracle import afc_oracle as O
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
    o = afc.afc_default_options(krylov=afc.AFC_KRYLOV_BICGSTAB, **kw)
    o.stream = torch.cuda.current_stream().cuda_stream
    return o


PARITY = dict(fp_tol=1e-14, fp_tol_mode=0, fp_maxit=100, lin_atol=1e-15, lin_rtol=0.0)


def _mixed_instances(count, nmax):
    ps = I.config4_params(count, nmin=4, nmax=nmax)
    return [I.config4_instance(p) for p in ps]


def _pack(insts, offs, attr):
    out = np.zeros(offs[-1])
    for k, inst in enumerate(insts):
        out[offs[k]:offs[k + 1]] = getattr(inst, attr)
    return out


def test_batch_parity_with_oracle():
    afc = _afc()
    insts = _mixed_instances(10, 10)
    print("batch parity: sizes", [i.N for i in insts], flush=True)
    b = afc.afc_batch_create(insts, _opts(**PARITY))
    try:
        offs = afc.afc_batch_offsets(b, len(insts))
        u = torch.tensor(_pack(insts, offs, "u0"), device="cuda:0")
        F = torch.tensor(_pack(insts, offs, "F"), device="cuda:0")
        dts = [1e-3] * len(insts)
        st, stats = afc.afc_batch_step_cn(b, u, F, dts, 3)
        assert st == 0, stats
        x = u.cpu().numpy()
        for k, inst in enumerate(insts):
            P = O.problem_from_instance(inst, conv=False)
            ref = inst.u0.copy()
            for _ in range(3):
                ref, _ = O.cn_fct_step(P, ref, inst.F, inst.F, 1e-3, tol=1e-14, tol_mode="abs", maxit=100,
                                       lin="bicgstab", lin_atol=1e-15)
            got = x[offs[k]:offs[k + 1]]
            rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            assert rel <= 1e-10, (k, rel)
            assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max(), k
            assert stats[k]["fp_iters"] > 0
    finally:
        afc.afc_batch_destroy(b)


def test_batch_alone_equals_mix_bitwise():
    afc = _afc()
    insts = _mixed_instances(16, 14)
    opts = _opts(fp_tol=1e-12, fp_maxit=50, lin_atol=1e-12)
    b = afc.afc_batch_create(insts, opts)
    try:
        offs = afc.afc_batch_offsets(b, len(insts))
        u = torch.tensor(_pack(insts, offs, "u0"), device="cuda:0")
        F = torch.tensor(_pack(insts, offs, "F"), device="cuda:0")
        afc.afc_batch_step_cn(b, u, F, [1e-3] * len(insts), 4)
        mix = u.cpu().numpy()
    finally:
        afc.afc_batch_destroy(b)
    for k in (0, 5, 11):
        b1 = afc.afc_batch_create([insts[k]], opts)
        try:
            u1 = torch.tensor(insts[k].u0, device="cuda:0")
            F1 = torch.tensor(insts[k].F, device="cuda:0")
            afc.afc_batch_step_cn(b1, u1, F1, [1e-3], 4)
            alone = u1.cpu().numpy()
        finally:
            afc.afc_batch_destroy(b1)
        assert np.array_equal(alone, mix[offs[k]:offs[k + 1]]), k


def test_batch_matches_single_handle_path():
    """The persistent batch and the multi-kernel afc_step_cn agree within 1e-10."""
    afc = _afc()
    insts = _mixed_instances(3, 9)
    b = afc.afc_batch_create(insts, _opts(**PARITY))
    try:
        offs = afc.afc_batch_offsets(b, len(insts))
        u = torch.tensor(_pack(insts, offs, "u0"), device="cuda:0")
        F = torch.tensor(_pack(insts, offs, "F"), device="cuda:0")
        afc.afc_batch_step_cn(b, u, F, [2e-3] * len(insts), 2)
        x = u.cpu().numpy()
    finally:
        afc.afc_batch_destroy(b)
    for k, inst in enumerate(insts):
        h = afc.afc_create_instance(inst, _opts(**PARITY), conv=False)
        try:
            uk = torch.tensor(inst.u0, device="cuda:0")
            Fk = torch.tensor(inst.F, device="cuda:0")
            for _ in range(2):
                afc.afc_step_cn(h, uk, Fk, Fk, 2e-3)
            ref = uk.cpu().numpy()
        finally:
            afc.afc_destroy(h)
        got = x[offs[k]:offs[k + 1]]
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_batch_rejects_gmres_options():
    afc = _afc()
    insts = _mixed_instances(2, 5)
    o = _opts()
    o.krylov = afc.AFC_KRYLOV_GMRES
    with pytest.raises(afc.AFCError) as e:
        afc.afc_batch_create(insts, o)
    assert e.value.status == afc.AFC_EINVAL


def test_batch_rejects_offsets_beyond_16_bits():
    """The batch stores 16-bit column offsets; an instance whose renumbered
    pattern needs more is refused with EINVAL and a message naming it, before
    any launch."""
    afc = _afc()
    big = I.renumbered(I.config4_instance(I.config4_params(1, 32, 32)[0]))
    assert big.N > 32768
    insts = _mixed_instances(2, 5) + [big]
    with pytest.raises(afc.AFCError) as e:
        afc.afc_batch_create(insts, _opts())
    assert e.value.status == afc.AFC_EINVAL
    assert "instance 2" in str(e.value) or "16-bit" in str(e.value)


def test_batch_results_identical_under_every_schedule():
    """Workgroup size and workgroup count change only the speed: every
    instance ends bitwise the same under each schedule, and alone (with a
    different schedule) as in the mix."""
    afc = _afc()
    insts = _mixed_instances(12, 12)
    opts = _opts(fp_tol=1e-12, fp_maxit=50, lin_atol=1e-12)
    b = afc.afc_batch_create(insts, opts)
    results = {}
    try:
        offs = afc.afc_batch_offsets(b, len(insts))
        u0 = torch.tensor(_pack(insts, offs, "u0"), device="cuda:0")
        F = torch.tensor(_pack(insts, offs, "F"), device="cuda:0")
        for threads in (256, 512, 1024):
            for wgs in (0, 1, 5):
                print("batch schedule threads=%d workgroups=%d" % (threads, wgs), flush=True)
                afc.afc_batch_set_schedule(b, threads, wgs)
                assert afc.afc_batch_get_schedule(b) == (threads, wgs)
                u = u0.clone()
                st, _ = afc.afc_batch_step_cn(b, u, F, [1e-3] * len(insts), 3)
                assert st >= 0
                results[(threads, wgs)] = u.cpu().numpy()
    finally:
        afc.afc_batch_destroy(b)
    ref = results[(1024, 0)]
    for key, x in results.items():
        assert np.array_equal(x, ref), key
    k = 7
    b1 = afc.afc_batch_create([insts[k]], opts)
    try:
        afc.afc_batch_set_schedule(b1, 256, 1)
        u1 = torch.tensor(insts[k].u0, device="cuda:0")
        afc.afc_batch_step_cn(b1, u1, torch.tensor(insts[k].F, device="cuda:0"), [1e-3], 3)
        assert np.array_equal(u1.cpu().numpy(), ref[offs[k]:offs[k + 1]])
    finally:
        afc.afc_batch_destroy(b1)


def test_batch_autotune_keeps_inputs_and_picks_a_candidate():
    afc = _afc()
    insts = _mixed_instances(20, 10)
    b = afc.afc_batch_create(insts, _opts(fp_tol=1e-12, fp_maxit=50, lin_atol=1e-12))
    try:
        offs = afc.afc_batch_offsets(b, len(insts))
        u = torch.tensor(_pack(insts, offs, "u0"), device="cuda:0")
        F = torch.tensor(_pack(insts, offs, "F"), device="cuda:0")
        before = u.clone()
        chosen, times = afc.afc_batch_autotune(b, u, F, [1e-3] * len(insts), trial_steps=1)
        print("autotune chose", chosen, "trial ms", [round(t, 3) for t in times], flush=True)
        assert torch.equal(u, before)
        assert chosen[0] in (256, 512, 1024) and 1 <= chosen[1] <= len(insts)
        assert afc.afc_batch_get_schedule(b) == chosen
        assert len(times) >= 3 and all(t > 0 for t in times)
    finally:
        afc.afc_batch_destroy(b)


def test_batch_full_size_sampled_instances():
    """The batched CN workload at full size (256 P1 instances, n in 8..32,
    20 steps, one launch, autotuned schedule): the smallest, a median and the
    largest instance against the oracle, both sides at the parity tolerances
    (fixed point sqrt(N) 1e-14, linear solves 1e-14 ||b||), element-wise and
    in L2 within 1e-10."""
    afc = _afc()
    ps = I.config4_params(256)
    insts = [I.config4_instance(p) for p in ps]
    opts = _opts(fp_tol=1e-14, fp_tol_mode=0, fp_maxit=100, lin_atol=0.0, lin_rtol=1e-14)
    b = afc.afc_batch_create(insts, opts)
    try:
        offs = afc.afc_batch_offsets(b, len(insts))
        u = torch.tensor(_pack(insts, offs, "u0"), device="cuda:0")
        F = torch.tensor(_pack(insts, offs, "F"), device="cuda:0")
        afc.afc_batch_autotune(b, u, F, [1e-3] * len(insts), 1)
        st, stats = afc.afc_batch_step_cn(b, u, F, [1e-3] * len(insts), 20)
        assert st >= 0
        x = u.cpu().numpy()
    finally:
        afc.afc_batch_destroy(b)
    sizes = np.array([inst.N for inst in insts])
    order = np.argsort(sizes, kind="stable")
    for k in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        inst = insts[k]
        print("batch full size: instance %d, N=%d" % (k, inst.N), flush=True)
        P = O.problem_from_instance(inst, conv=False)
        ref = inst.u0.copy()
        for _ in range(20):
            ref, rst = O.cn_fct_step(P, ref, inst.F, inst.F, 1e-3, tol=1e-14, tol_mode="abs", maxit=100,
                                     lin="bicgstab", lin_atol=0.0, lin_rtol=1e-14)
            assert rst.status == O.STATUS_OK
        got = x[offs[k]:offs[k + 1]]
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref), k
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max(), k
