"""The word-size sweep (the axis of the paper's Fig. 1) runs end to end on
small single-length workloads: every filtered match list equals the
oracle's element by element (and the GPU brute force's, checked inside the
sweep), and every survivor count equals the oracle's count of pairs with
F_D <= 2k under the same symbol map."""
import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

pytestmark = pytest.mark.gpu

VARIANTS = {"occ": oracle.OCC, "count": oracle.COUNT, "pos": oracle.POS}


def test_fixed_length_sweep_small(gpu):
    from paper_1711_08475_amd import lensweep

    print("[case] length sweep small", flush=True)
    args = lensweep.parse(["--words", "4000", "--queries", "150", "--lengths", "3,9,17", "--steps", "2",
                           "--warmup", "1"])
    res = lensweep.run(args)
    assert len(res) == 9
    refs = {}
    for row, hits, mp in res:
        L = row["length"]
        d, q = datagen.fixed_length_workload(4000, 150, L, 41 + L)
        if L not in refs:
            refs[L] = oracle.match(d, q, oracle.HAM, 1)
        assert np.array_equal(hits, refs[L]), row
        assert row["matches"] == refs[L].shape[0]
        variant = VARIANTS[row["fingerprint"][:-2]]
        ex, surv, _ = oracle.filter_stats(d, q, variant, 16, mp, oracle.HAM, 1)
        assert (row["examined"], row["survivors"]) == (ex, surv), row
        assert 0.0 <= row["rejection_rate"] <= 1.0
