"""Host-side checks of the C ABI: the library loads without a GPU and exports
every function include/pd.h declares."""
import os
import re

import paper_2605_20816_amd as pdl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(pd_[a-z0-9_]+)\s*\(", src))
    return names


def test_header_symbols_exported():
    L = pdl.lib()
    declared = _declared()
    assert {"pd_create", "pd_objective_grad", "pd_assign", "pd_fit", "pd_features"} <= declared
    for name in declared:
        assert hasattr(L, name), name
    assert declared <= set(pdl.exported_symbols()) | {"pd_destroy"}


def test_num_features_host():
    for d in range(0, 9):
        assert pdl.num_features(d) == (d + 1) * (d + 2) // 2
    assert pdl.num_features(-1) == 0 and pdl.num_features(9) == 0


def test_fit_state_size_host():
    """pd_fit_state_size: header, the ring of history + 1 slots of s and y, rho,
    the two Gram matrices and D^-1; 0 for arguments pd_fit would reject."""
    for N, d, m in [(2, 1, 1), (7, 3, 10), (4895, 6, 10), (100, 8, 32)]:
        K = (d + 1) * (d + 2) // 2
        NK = N * K
        want = 16 + 2 * (m + 1) * NK + (m + 1) + 2 * (m + 1) ** 2 + NK
        assert pdl.fit_state_size(N, d, m) == want
    assert pdl.fit_state_size(4895, 6, 10) * 8 < 32e6  # the c5 state: about 25 MB
    for bad in [(1, 2, 10), (10, 0, 10), (10, 9, 10), (10, 2, 0), (10, 2, 33)]:
        assert pdl.fit_state_size(*bad) == 0
