"""The selector's decision rule on injected timing tables (section 3.1:
the fastest implementation is kept), without a GPU: the library's
xab_select_rule against the rule written out (least time over the valid
classes, lowest index among equal times), and the class-validity mask."""
import numpy as np
import pytest

import paper_2405_01599_amd as xab


def rule(times, valid):
    best = None
    for k, (t, v) in enumerate(zip(times, valid)):
        if not v or not np.isfinite(t) or t < 0:
            continue
        if best is None or t < times[best]:
            best = k
    return best


def test_rule_ties_go_to_the_lowest_class():
    t = [0.5, 0.3, 0.3, 0.9, 0.3]
    assert xab.select_rule(t, [1] * 5) == (0, 1)
    assert xab.select_rule(t, [1, 0, 1, 1, 1]) == (0, 2)
    assert xab.select_rule(t, [1, 0, 0, 1, 1]) == (0, 4)


def test_rule_skips_invalid_and_unmeasured_classes():
    # -1 marks a class that was not timed; NaN and infinity are no time
    t = [-1.0, np.nan, np.inf, 2.0, 1.0]
    assert xab.select_rule(t, [1, 1, 1, 1, 1]) == (0, 4)
    assert xab.select_rule(t, [1, 1, 1, 1, 0]) == (0, 3)
    s, c = xab.select_rule(t, [1, 1, 1, 0, 0])
    assert s == -6 and c == -1
    s, c = xab.select_rule([], [])
    assert s == -6 and c == -1


def test_rule_on_random_tables_with_ties():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        n = int(rng.integers(1, xab.NCLASSES + 1))
        # few distinct values so that ties are common; some classes invalid
        t = rng.choice(np.array([0.1, 0.2, 0.25, 1.0, -1.0], dtype=np.float32), n)
        v = (rng.random(n) < 0.8).astype(np.int32)
        want = rule(list(t), list(v))
        s, c = xab.select_rule(t, v)
        if want is None:
            assert s == -6 and c == -1
        else:
            assert s == 0 and c == want


def test_rule_argument_errors():
    import ctypes
    L = xab.lib()
    c = ctypes.c_int32()
    assert L.xab_select_rule(None, None, 0, None) == -1
    assert L.xab_select_rule(None, None, -1, ctypes.byref(c)) == -2
    assert L.xab_select_rule(None, None, 3, ctypes.byref(c)) == -1


def test_class_validity_mask():
    # general matrices: row split, nnz split, segmented scan, column-blocked,
    # SELL, BCSR; lower-stored symmetric ones: the atomic and S3 classes
    sym = [k for k in range(xab.NCLASSES) if xab.class_applies(k, True) == 1]
    gen = [k for k in range(xab.NCLASSES) if xab.class_applies(k, False) == 1]
    assert sym == [9, 10, 11]
    assert gen == [0, 1, 2, 3, 4, 5, 6, 7, 8, 12, 13, 14]
    for k in sym:
        assert xab.class_params(k)[0] in (xab.SYM_ATOMIC, xab.SYM_S3)
    for k in gen:
        assert xab.class_params(k)[0] not in (xab.SYM_ATOMIC, xab.SYM_S3)
    assert xab.class_applies(-1, False) == -2
    assert xab.class_applies(xab.NCLASSES, True) == -2
