"""The entry point that allocates nothing (mcs_solve_batch_static): the
library's static device scratch as the workspace, compared with the
workspace entry (mcs_solve_batch) on the same pairs, on two calls in a row,
the second with a smaller batch."""
import numpy as np
import pytest
from _easy import easy_c4

import mcs_instances as mi
import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _check_same(pairs, got, ref):
    assert len(got) == len(ref) == len(pairs)
    for (G, H), a, b in zip(pairs, got, ref):
        assert a.optimal and b.optimal
        assert a.size == b.size
        assert len(a.mapping) == a.size and oracle.check.is_valid(G, H, a.mapping)


def test_static_scratch_matches_workspace_entry(gpu):
    from paper_1908_06418_amd import solve_batch, solve_batch_static
    rng = np.random.default_rng(9)
    # (the default launch of these batches needs more workspace than the
    # static scratch holds: four wavefronts of 16-lane searches per CU fit,
    # for both entries)
    tun = {"waves_per_cu": 4, "seg_lanes": 16}
    first = easy_c4(200, start=200)[0]
    second = [(mi.random_small(rng, int(rng.integers(0, 14)), 0.4, True, 2),
               mi.random_small(rng, int(rng.integers(0, 14)), 0.4, True, 2)) for _ in range(12)]
    second += first[:20]
    for k, pairs in enumerate((first, second)):
        _say(f"static scratch, call {k + 1}: {len(pairs)} pairs")
        got = solve_batch_static(pairs, time_limit_s=60, tuning=tun)
        ref = solve_batch(pairs, time_limit_s=60, tuning=tun)
        _check_same(pairs, got, ref)
    small = second[:12]
    assert [r.size for r in solve_batch_static(small, time_limit_s=60, tuning=tun)] == \
        [oracle.mcs(G, H)["size"] for G, H in small]


def test_static_scratch_rejects_what_does_not_fit(gpu):
    """A batch whose workspace exceeds the static scratch, and the graph
    mode, are refused before any device work."""
    from paper_1908_06418_amd import McsError, _abi, solve_batch_static, workspace_size
    wide = mi.pairs_w(ns=(100,), seeds=range(2))
    assert workspace_size(wide) > _abi.MCS_STATIC_SCRATCH_BYTES
    with pytest.raises(McsError) as e:
        solve_batch_static(wide, time_limit_s=60)
    assert e.value.status == _abi.MCS_E_WORKSPACE
    with pytest.raises(McsError) as e:
        solve_batch_static(easy_c4(4)[0], time_limit_s=60, tuning={"use_graph": 1})
    assert e.value.status == _abi.MCS_E_INVALID
    # the entry still works after the refusals
    pairs = easy_c4(8)[0]
    assert [r.size for r in solve_batch_static(pairs, time_limit_s=60,
                                               tuning={"waves_per_cu": 4, "seg_lanes": 16})] == \
        [oracle.mcs(G, H)["size"] for G, H in pairs]
