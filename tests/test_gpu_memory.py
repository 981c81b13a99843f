"""Device memory accounting and the FPM_ENOMEM path, forced from the host:
with a limit on the library's device memory, an index build, a host-buffer
match, a plan and the growth of a plan's match buffer fail with FPM_ENOMEM,
release everything they had taken, and the next call without the limit
succeeds with the oracle's result."""
import gc

import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def fpm(gpu):
    from paper_1711_08475_amd import fpm as f

    f.lib()
    yield f
    f.fpm_set_device_memory_limit(0)


def test_memory_limit_gives_enomem_and_a_clean_state(fpm):
    d, q = datagen.english_workload(20_000, 300, 5, "3-15", 0.5)
    ref = oracle.match(d, q, oracle.LEV, 1)
    say("memory limit: index build")
    gc.collect()  # buffers of earlier tests' objects are released before counting
    base = fpm.fpm_device_memory_in_use()
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    with_ix = fpm.fpm_device_memory_in_use()
    assert with_ix > base
    try:
        # room for half of a second index
        fpm.fpm_set_device_memory_limit(with_ix + (with_ix - base) // 2)
        with pytest.raises(fpm.FpmError) as e:
            fpm.fpm_build_fingerprints(d, "occ", 16, "common")
        assert e.value.status == fpm.FPM_ENOMEM
        assert fpm.fpm_device_memory_in_use() == with_ix  # the failed build released what it took
        say("memory limit: match and plan")
        fpm.fpm_set_device_memory_limit(with_ix + 4096)
        for sched in (fpm.FPM_SCHED_PLAIN, fpm.FPM_SCHED_BATCHED):
            with pytest.raises(fpm.FpmError) as e:
                fpm.fpm_match(ix, q, "lev", 1, fpm.options(schedule=sched))
            assert e.value.status == fpm.FPM_ENOMEM
            assert fpm.fpm_device_memory_in_use() == with_ix
        with pytest.raises(fpm.FpmError) as e:
            fpm.fpm_plan_create(ix, 300, int(q[1][-1]), "lev", 1)
        assert e.value.status == fpm.FPM_ENOMEM
        assert fpm.fpm_device_memory_in_use() == with_ix
    finally:
        fpm.fpm_set_device_memory_limit(0)
    e = None  # the caught errors' tracebacks hold the frames that took the index as an argument
    say("memory limit lifted")
    assert np.array_equal(fpm.fpm_match(ix, q, "lev", 1), ref)
    ix2 = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    assert np.array_equal(fpm.fpm_get_fingerprints(ix2), fpm.fpm_get_fingerprints(ix))
    del ix2
    assert fpm.fpm_device_memory_in_use() == with_ix
    del ix
    assert fpm.fpm_device_memory_in_use() == base


def test_match_buffer_growth_under_a_limit(fpm):
    """A plan whose match buffer must grow: under a limit the growth fails
    with FPM_ENOMEM and the plan keeps its buffers; once the limit is lifted
    the same plan grows, reruns and returns the oracle's list."""
    import torch

    d, q = datagen.english_workload(20_000, 300, 6, "3-15", 0.5)
    ref = oracle.match(d, q, oracle.LEV, 2)
    assert ref.shape[0] > 64
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    qb = torch.from_numpy(q[0].copy()).cuda()
    qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
    torch.cuda.synchronize()
    nq = q[1].size - 1
    plan = fpm.fpm_plan_create(ix, nq, int(q[1][-1]), "lev", 2, fpm.options(schedule=1, match_capacity=16))
    gc.collect()
    held = fpm.fpm_device_memory_in_use()
    try:
        fpm.fpm_set_device_memory_limit(held + 1024)
        say("growth under a limit")
        fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
        with pytest.raises(fpm.FpmError) as e:
            fpm.fpm_plan_result(plan)
        assert e.value.status == fpm.FPM_ENOMEM
        assert fpm.fpm_device_memory_in_use() == held
    finally:
        fpm.fpm_set_device_memory_limit(0)
    say("growth without a limit")
    assert np.array_equal(fpm.fpm_plan_copy_matches(plan), ref)
    fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
    assert np.array_equal(fpm.fpm_plan_copy_matches(plan), ref)


def test_default_filter_unit_is_the_vector_alus(fpm):
    """Default options run the filter on the vector ALUs for every key
    family; the matrix cores run it only on request."""
    d, q = datagen.english_workload(5_000, 200, 9, "3-15", 0.5)
    ref = oracle.match(d, q, oracle.LEV, 1)
    for bits in (16, 32):
        ix = fpm.fpm_build_fingerprints(d, "occ", bits, "common")
        for sched in (fpm.FPM_SCHED_PLAIN, fpm.FPM_SCHED_BATCHED):
            got, st = fpm.fpm_match(ix, q, "lev", 1, fpm.options(schedule=sched), with_stats=True)
            assert st["filter_unit"] == fpm.FPM_UNIT_VALU
            assert np.array_equal(got, ref)
        got, st = fpm.fpm_match(ix, q, "lev", 1, fpm.options(filter_unit="matrix"), with_stats=True)
        assert st["filter_unit"] == fpm.FPM_UNIT_MATRIX
        assert np.array_equal(got, ref)
