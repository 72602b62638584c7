"""Host SELL-64 layout (afc_sell_layout, no GPU): every CSR entry lands in its
own slot of its row's lane, carries its column offset, padding offsets stay
inside [0, N), and an SpMV evaluated through the layout equals the CSR SpMV."""
import numpy as np
import pytest

from paper_2110_15676_amd import inputs as I


def _afc():
    from paper_2110_15676_amd import afc

    afc.lib()
    return afc


def _check_layout(row_ptr, col):
    afc = _afc()
    N = row_ptr.shape[0] - 1
    info, slp, sdl, pat, pos, lane = afc.afc_sell_layout(row_ptr, col)
    nsl = (N + 63) // 64
    assert info["slices"] == nsl
    assert slp[0] == 0 and np.all(np.diff(slp) % 64 == 0) and slp[-1] == info["slots"]
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    sl = rows // 64
    # each entry in its row's slice and lane, no slot used twice
    assert np.all(pos >= slp[sl]) and np.all(pos < slp[sl + 1])
    assert np.all((pos - slp[sl]) % 64 == rows % 64)
    assert np.unique(pos).shape[0] == pos.shape[0]
    # padded length = longest row of the slice
    rl = np.zeros(nsl * 64, dtype=np.int64)
    rl[:N] = np.diff(row_ptr)
    assert np.array_equal((slp[1:] - slp[:-1]) // 64, rl.reshape(nsl, 64).max(axis=1))
    # offset of every slot (uniform: shared pattern; else per-lane)
    delta = np.zeros(info["slots"], dtype=np.int64)
    uniform = 0
    for s in range(nsl):
        L = (slp[s + 1] - slp[s]) // 64
        uniform += int(sdl[s] < 0)
        if L == 0:
            continue
        if sdl[s] < 0:
            p = pat[~sdl[s]: ~sdl[s] + L]
            delta[slp[s]: slp[s + 1]] = np.repeat(p, 64)
        else:
            delta[slp[s]: slp[s + 1]] = lane[sdl[s]: sdl[s] + 64 * L]
    assert uniform == info["uniform_slices"]
    assert np.array_equal(delta[pos], col.astype(np.int64) - rows)
    # every slot of a real row reads an existing node
    slot = np.arange(info["slots"])
    slot_sl = np.searchsorted(slp, slot, side="right") - 1
    slot_row = slot_sl * 64 + (slot - slp[slot_sl]) % 64
    real = slot_row < N
    j = slot_row[real] + delta[real]
    assert np.all(j >= 0) and np.all(j < N)
    # SpMV through the layout (padding values 0) equals the CSR SpMV
    rng = np.random.default_rng(7)
    a = rng.standard_normal(col.shape[0])
    x = rng.standard_normal(N)
    vals = np.zeros(info["slots"])
    vals[pos] = a
    y = np.zeros(N)
    np.add.at(y, slot_row[real], vals[real] * x[j])
    ref = np.zeros(N)
    np.add.at(ref, rows, a * x[col])
    assert np.allclose(y, ref, rtol=1e-13, atol=1e-13)
    return info


def test_q1_structured_mostly_uniform():
    # 17^3 nodes: only slices within one z-layer of the first and the last
    # node can see an offset leave [0, N)
    inst = I.config3(16)
    info = _check_layout(inst.row_ptr, inst.col)
    assert info["uniform_slices"] >= info["slices"] - 2 * (-(-(17 * 17 + 17 + 1) // 64))
    assert info["pattern_ints"] < 27 * info["uniform_slices"]  # patterns are shared


def test_q1_run_slices_read_in_range():
    """The FP64 residual takes full uniform slices whose 27 offsets are nine
    runs (c - 1, c, c + 1) by loading x[i + c] per run and shifting across
    lanes; lane 0 also reads x[i0 + c - 1] and lane 63 x[i0 + 63 + c + 1].
    Those are column indices of the slice's own rows, so the layout must keep
    them in [0, N); and a Q1 mesh must give such slices (most of them)."""
    afc = _afc()
    for n in (12, 16):
        inst = I.config3(n)
        N = inst.N
        info, slp, sdl, pat, pos, lane = afc.afc_sell_layout(inst.row_ptr, inst.col)
        runs = 0
        for s in range(info["slices"]):
            L = (slp[s + 1] - slp[s]) // 64
            if sdl[s] >= 0 or L != 27 or s * 64 + 64 > N:
                continue
            p = pat[~sdl[s]: ~sdl[s] + 27].astype(np.int64)
            c = p[1::3]
            if not (np.array_equal(p[0::3], c - 1) and np.array_equal(p[2::3], c + 1)):
                continue
            runs += 1
            i0 = s * 64
            rows = i0 + np.arange(64)
            j = rows[:, None] + p[None, :]
            assert np.all(j >= 0) and np.all(j < N)
            assert np.all(i0 + c - 1 >= 0) and np.all(i0 + 63 + c + 1 < N)
        assert runs >= 0.75 * info["slices"], (n, runs, info["slices"])


def test_p1_structured():
    inst = I.config1(6)
    info = _check_layout(inst.row_ptr, inst.col)
    assert info["uniform_slices"] > 0


def test_renumbered_falls_back_to_lane_offsets():
    inst = I.renumbered(I.config3(8))
    info = _check_layout(inst.row_ptr, inst.col)
    assert info["uniform_slices"] < info["slices"]
    assert info["lane_delta_slots"] > 0


def test_long_row_layout():
    # one row of 67 entries: its slice pads every lane to 67 slots
    inst = I.with_long_row(I.config3(6), extra=40)
    info = _check_layout(inst.row_ptr, inst.col)
    assert info["slots"] >= 64 * 67


def test_ragged_rows_empty_rows_and_tiny_sizes():
    rng = np.random.default_rng(3)
    for N in (1, 63, 64, 65, 200):
        rl = rng.integers(0, 6, size=N)
        rl[rng.integers(0, N)] = 0
        rl = np.minimum(rl, N)
        rp = np.concatenate([[0], np.cumsum(rl)]).astype(np.int32)
        col = np.concatenate([np.sort(rng.choice(N, size=k, replace=False)) for k in rl]
                             + [np.zeros(0, dtype=np.int64)]).astype(np.int32)
        _check_layout(rp, col)


def test_banded_is_uniform_except_edges():
    N = 1000
    rows, cols = [], []
    for i in range(N):
        for d in (-3, -1, 0, 1, 3):
            if 0 <= i + d < N:
                rows.append(i)
                cols.append(i + d)
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=N))]).astype(np.int32)
    info = _check_layout(rp, np.array(cols, dtype=np.int32))
    # only the first and the last slice see an offset leave [0, N)
    assert info["uniform_slices"] == info["slices"] - 2
    assert info["pattern_ints"] == 5


def test_duplicate_entries_use_lane_offsets():
    rp = np.array([0, 2, 3], dtype=np.int32)
    col = np.array([1, 1, 0], dtype=np.int32)
    info = _check_layout(rp, col)
    assert info["uniform_slices"] == 0


def test_malformed_pattern_rejected():
    afc = _afc()
    with pytest.raises(afc.AFCError):
        afc.afc_sell_layout(np.array([0, 1, 2], dtype=np.int32), np.array([0, 5], dtype=np.int32))
    with pytest.raises(afc.AFCError):
        afc.afc_sell_layout(np.array([0, 2, 1], dtype=np.int32), np.array([0, 1], dtype=np.int32))
