"""The slack filter of the row kernels (a row skips its candidate pass when
no candidate can be taken) is sound: on rows whose slack sits at the
filter's threshold, every row the filter calls quiet is left unchanged by
the oracle's first round, while the naive threshold max |a| (ub - lb) is
not safe.  The GPU parity test of the same rows is in
test_gpu_parity.py."""
import numpy as np
import pytest

import oracle
from helpers import filter_quiet, row_instance, slack_edge_instance


def _changes(sub):
    r, lb, ub = oracle.propagate(sub)
    return r["status"] != 0 or not (np.array_equal(lb, sub["lb"]) and np.array_equal(ub, sub["ub"]))


@pytest.mark.parametrize("seed,count,lengths", [(0, 400, (1, 7)), (1, 400, (1, 7)),
                                                (2, 400, (1, 7)), (3, 60, (50, 400))])
def test_quiet_rows_never_change(seed, count, lengths):
    inst, info = slack_edge_instance(seed, count=count, lengths=lengths)
    quiet = 0
    for k, (mn, mx, w) in enumerate(info):
        if not filter_quiet(mn, mx, 0, 0, inst["lo"][k], inst["hi"][k], w):
            continue
        quiet += 1
        assert not _changes(row_instance(inst, k)), k
    assert quiet >= count // 4  # the rule is exercised, not vacuous


def test_naive_threshold_is_unsafe():
    """Slack placed at max |a| (ub - lb): rows the naive rule would skip do
    tighten (integer rounding of a candidate at the bound, rounding of the
    candidate formula), so the rule above needs its unit and margins."""
    inst, info = slack_edge_instance(5, count=400, naive=True)
    bad = 0
    for k in range(inst["m"]):
        rp = inst["row_ptr"]
        c = inst["col"][rp[k]:rp[k + 1]]
        v = inst["val"][rp[k]:rp[k + 1]]
        w = max(abs(a) * (inst["ub"][j] - inst["lb"][j]) for a, j in zip(v, c))
        mn, mx, _ = info[k]
        if filter_quiet(mn, mx, 0, 0, inst["lo"][k], inst["hi"][k], w) and _changes(row_instance(inst, k)):
            bad += 1
    assert bad > 0
