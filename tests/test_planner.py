"""Host-side planner of the HIP library (no device needed): rotation keys of
the Z / T transforms against Table 3 and the closed forms of Tables 1 and 2."""
import csv
import math
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def he():
    from paper_2305_17341_amd import he as H
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("library not built")
    return H


def test_planner_reproduces_table3(he):
    rows = [r for r in csv.DictReader(l for l in open(os.path.join(HERE, "golden", "table3_ZT_keys.csv"))
                                      if not l.startswith("#"))]
    for r in rows:
        nprime = int(r["maxdiag"])
        keys = he.lintrans_rot_steps(r["matrix"], 128, int(r["n1"]), 0 if nprime == 127 else nprime)
        assert 45 * (len(keys) + 1) == int(r["rtk_mb"]), r


@pytest.mark.parametrize("n,n1", [(16, 4), (64, 8), (128, 8), (128, 16), (256, 16)])
def test_dh_bsgs_key_counts_are_table1(he, n, n1):
    n2 = n // n1
    assert len(he.lintrans_rot_steps("Z", n, n1)) == n1 + 2 * n2 - 2
    assert len(he.lintrans_rot_steps("T", n, n1)) == n1 + n2 - 2


@pytest.mark.parametrize("n,n1,nprime", [(128, 8, 32), (128, 8, 64), (128, 16, 32), (128, 16, 64), (64, 8, 16)])
def test_dcd_key_counts_are_table2(he, n, n1, nprime):
    n2p = nprime // n1
    assert len(he.lintrans_rot_steps("Z", n, n1, nprime)) == n1 + 2 * n2p - 1
    assert len(he.lintrans_rot_steps("T", n, n1, nprime)) == n1 + n2p - 1


def test_planner_matches_oracle_factor_keys(he, oracle_mod):
    from tests.test_oracle_dcd import transform_keys
    for n, n1, nprime in [(128, 16, 32), (64, 8, 16), (32, 4, 8), (16, 4, 15)]:
        for m in ("Z", "T"):
            want = transform_keys(oracle_mod, m, n, n1, nprime)
            got = set(he.lintrans_rot_steps(m, n, n1, 0 if nprime >= n - 1 else nprime))
            assert got == want, (n, n1, nprime, m)


@pytest.mark.parametrize("n,n1,n1p", [(16, 4, 2), (64, 8, 4), (128, 8, 2), (128, 16, 4), (128, 16, 8),
                                      (256, 16, 4)])
def test_smpkeysub_key_counts_are_table2(he, n, n1, n1p):
    """Table 2, SmpKeySub rows: MinRotKeys n1' + 2 n2 - 2 for Z and n1' + n2 - 2
    for T; the baby-step keys are exactly the prefix a j', 0 < j' < n1'"""
    n2 = n // n1
    z = he.smpkeysub_rot_steps("Z", n, n1, n1p)
    t = he.smpkeysub_rot_steps("T", n, n1, n1p)
    assert len(z) == n1p + 2 * n2 - 2
    assert len(t) == n1p + n2 - 2
    assert {s for s in z if abs(s) < n1} == set(range(1, n1p))
    assert {s for s in t if s % (n * n1)} == {n * j for j in range(1, n1p)}
    # the giant steps are those of plain dh-BSGS
    assert {s for s in z if abs(s) >= n1} == {s for s in he.lintrans_rot_steps("Z", n, n1) if abs(s) >= n1}
    # no prefix (n1' = 0 or n1' >= n1): plain dh-BSGS
    assert he.smpkeysub_rot_steps("Z", n, n1, 0) == he.lintrans_rot_steps("Z", n, n1)
    assert he.smpkeysub_rot_steps("T", n, n1, n1) == he.lintrans_rot_steps("T", n, n1)
