"""C ABI checks that need no GPU: the library loads, exports every declared symbol,
and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "htsvd.h")).read()
    return sorted(set(re.findall(r"\b(htsvd_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2512_23569_amd as ht
    lib = ht.lib()
    declared = _declared()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(ht.exported_symbols()) == declared


def test_default_params_and_ref_count():
    import paper_2512_23569_amd as ht
    p = ht.htsvd_default_params(3)
    assert (p.ps, p.stride, p.window, p.K, p.gcp_num, p.gcp_den, p.gamma_rank) == (8, 4, 31, 32, 6, 5, 13)
    assert abs(p.beta - 1.2) < 1e-6 and p.subimage == 128 and p.n_vote == 15
    q = ht.htsvd_default_params(1)
    assert (q.window, q.K) == (21, 16)
    import oracle
    for n, s in ((256, 4), (4000, 3), (3000, 3), (9, 1), (17, 5)):
        assert ht.htsvd_ref_count(n, 8, s) == len(oracle.ref_grid(n, 8, s))
    with pytest.raises(ht.HtsvdError):
        ht.htsvd_default_params(2)


def test_null_context_is_rejected():
    import paper_2512_23569_amd as ht
    L = ht.lib()
    p = ht.htsvd_params()
    st = L.htsvd_denoise(None, None, 8, 8, 1, 8, 1.0, ctypes.byref(p), None, 8, None)
    assert st == ht.HTSVD_EINVAL
    assert "null" in ht.htsvd_last_error()
    assert L.htsvd_block_match(None, None, 8, 8, 1, 8, ctypes.byref(p), None, None, None) == ht.HTSVD_EINVAL
