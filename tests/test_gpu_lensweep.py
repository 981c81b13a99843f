"""The word-size sweep runs end to end on small single-length workloads and
its filtered match lists equal the brute force's (checked inside the sweep)
and the oracle's."""
import json

import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

pytestmark = pytest.mark.gpu


def test_fixed_length_sweep_small(gpu, capsys):
    from paper_1711_08475_amd import lensweep

    print("[case] length sweep small", flush=True)
    assert lensweep.main(["--words", "4000", "--queries", "150", "--lengths", "3,9,17", "--steps", "2",
                          "--warmup", "1"]) == 0
    rows = [json.loads(line) for line in capsys.readouterr().out.splitlines() if line.startswith("{")]
    assert len(rows) == 9
    for r in rows:
        d, q = datagen.fixed_length_workload(4000, 150, r["length"], 41 + r["length"])
        assert r["matches"] == oracle.match(d, q, oracle.HAM, 1).shape[0]
        assert 0.0 <= r["rejection_rate"] <= 1.0
