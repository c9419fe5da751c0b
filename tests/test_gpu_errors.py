"""Failure handling of the library on the GPU: a run that runs out of its
device-memory budget partway through a step reports ENOMEM, and every later
call that would touch its (released) device buffers is refused with ESTATE
instead of launching kernels on them."""
import pytest

from paper_2006_14956_amd import fciqmc as F
from paper_2006_14956_amd import inputs
from tests.gpu_helpers import make_gpu_run

pytestmark = pytest.mark.gpu


def test_out_of_budget_run_is_refused_afterwards():
    s = inputs.molecule_8o8e()
    # the device bytes a run holds right after init (one bucket, the
    # smallest record slabs), without a budget
    sysd, probe = make_gpu_run(s, tau=0.01, target=1e6, seed=3, n_initial=50.0, max_dets=1024,
                               max_spawns=65536)
    base = F.fciqmc_run_device_bytes(probe)
    F.fciqmc_free_run(probe)
    # the same run with a budget only a little above that: growing towards
    # the 1e6 target has to allocate more and fails
    p = F.fciqmc_params_default(tau=0.01, walker_target=1e6, seed=3, n_initial=50.0,
                                max_dets=1024, max_spawns=65536, hbm_budget_bytes=base + (1 << 20))
    run = F.fciqmc_init(sysd, p)
    code = None
    for _ in range(400):
        try:
            F.fciqmc_step(run, 10)
        except F.FciqmcError as e:
            code = e.code
            break
    assert code == F.ENOMEM, code
    assert F.fciqmc_run_device_bytes(run) <= base + (1 << 20)
    # the failed call left nothing to step on: refused, with no launch
    for call in (lambda: F.fciqmc_step(run, 1), lambda: F.fciqmc_get_walkers(run),
                 lambda: F.fciqmc_step(run, 1)):
        with pytest.raises(F.FciqmcError) as ei:
            call()
        assert ei.value.code in (F.ESTATE, F.ENOMEM), ei.value.code
    # the energy report (host data) stays available; freeing works
    F.fciqmc_energy(run)
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)


def test_out_of_budget_batch_member_is_refused():
    s = inputs.molecule_8o8e()
    sysd, probe = make_gpu_run(s, tau=0.01, target=1e6, seed=4, n_initial=50.0, max_dets=1024,
                               max_spawns=65536)
    base = F.fciqmc_run_device_bytes(probe)
    F.fciqmc_free_run(probe)
    p = F.fciqmc_params_default(tau=0.01, walker_target=1e6, seed=4, n_initial=50.0,
                                max_dets=1024, max_spawns=65536, hbm_budget_bytes=base + (1 << 20))
    small = F.fciqmc_init(sysd, p)
    ok = F.fciqmc_init(sysd, F.fciqmc_params_default(tau=0.01, walker_target=500.0, seed=5))
    batch = F.fciqmc_batch_create()
    F.fciqmc_batch_add(batch, small)
    F.fciqmc_batch_add(batch, ok)
    code = None
    for _ in range(400):
        try:
            F.fciqmc_batch_step(batch, 10)
        except F.FciqmcError as e:
            code = e.code
            break
    assert code == F.ENOMEM, code
    with pytest.raises(F.FciqmcError) as ei:
        F.fciqmc_batch_step(batch, 1)
    assert ei.value.code == F.ESTATE
    # without the broken member the batch steps again
    F.fciqmc_batch_remove(batch, small)
    F.fciqmc_batch_step(batch, 5)
    F.fciqmc_batch_free(batch)
    F.fciqmc_free_run(small)
    F.fciqmc_free_run(ok)
    F.fciqmc_free_system(sysd)
