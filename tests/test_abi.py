"""C-ABI library checks that need no GPU: it loads, exports every declared
entry point, and rejects malformed input on the host before any device call."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "afc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(afc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2110_15676_amd import afc

    L = afc.lib()
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n
    assert sorted(afc.EXPORTS) == names


def test_default_options_and_status_strings():
    from paper_2110_15676_amd import afc

    o = afc.afc_default_options()
    assert o.restart == 30 and o.krylov == afc.AFC_KRYLOV_GMRES and o.ssp_stages == 3
    assert o.omega == 1.0 and o.prelimit == 2.0
    assert afc.afc_status_str(0) == "ok"
    assert "invalid" in afc.afc_status_str(afc.AFC_EINVAL)


def _tiny():
    # 3-node chain, diagonal present, symmetric pattern
    rp = np.array([0, 2, 5, 7], np.int32)
    col = np.array([0, 1, 0, 1, 2, 1, 2], np.int32)
    M = np.array([2, 1, 1, 4, 1, 1, 2], float) / 6
    K = np.array([-1, 1, 1, -2, 1, 1, -1], float)
    return rp, col, M, K


@pytest.mark.parametrize("case", ["unsorted", "no_diag", "asym", "rowptr", "colrange", "dirichlet", "mass",
                                  "options"])
def test_create_rejects_malformed_input(case):
    from paper_2110_15676_amd import afc

    rp, col, M, K = _tiny()
    di, dv = None, None
    opts = afc.afc_default_options()
    if case == "unsorted":
        col = np.array([1, 0, 0, 1, 2, 1, 2], np.int32)
    elif case == "no_diag":
        rp = np.array([0, 1, 4, 6], np.int32)
        col = np.array([1, 0, 1, 2, 1, 2], np.int32)
        M, K = M[1:], K[1:]
    elif case == "asym":
        rp = np.array([0, 2, 4, 6], np.int32)
        col = np.array([0, 1, 1, 2, 1, 2], np.int32)
        M, K = M[:6], K[:6]
    elif case == "rowptr":
        rp = np.array([0, 3, 2, 7], np.int32)
    elif case == "colrange":
        col = np.array([0, 1, 0, 1, 5, 1, 2], np.int32)
    elif case == "dirichlet":
        di, dv = np.array([0, 0], np.int32), np.zeros(2)
    elif case == "mass":
        M = -M
    elif case == "options":
        opts.restart = 0
    with pytest.raises(afc.AFCError) as e:
        afc.afc_create(rp, col, M, K, None, None, di, dv, opts)
    assert e.value.status == afc.AFC_EINVAL


def test_product_path_never_reaches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2110_15676_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "afc_oracle" not in text, f
