"""GPU: the request server.  Solves admitted into a running mix, stepped in
shared launches and retired on their own convergence checks give the same
step counts, attempt counts and energy reports as the same solves run
alone; admission respects the device-memory budget in arrival order."""
import pytest

from paper_2006_14956_amd import fciqmc as F
from paper_2006_14956_amd import inputs
from tests.gpu_helpers import assert_same_report, ref_of, solve_alone

pytestmark = pytest.mark.gpu


def _requests():
    """Small solves of the three shapes: molecules (uniform, integer), a
    Hubbard lattice (initiators), a two-word PCHB molecule."""
    out = []
    for i in range(4):
        s = inputs.synthetic_molecule(8, 4, 4, seed=20 + i)
        out.append((s, dict(tau=0.01, walker_target=2e3 * (i + 1), seed=i, shift_damping=0.3,
                            conv_tol=0.05)))
    h = inputs.hubbard(4, 2, 1.0, 4.0, 4, 4)
    ra, rb = ref_of(h)
    out.append((h, dict(tau=0.01, walker_target=5e3, initiator_na=3.0, excitgen=F.GEN_LATTICE,
                        ref_alpha=ra, ref_beta=rb, seed=7, shift_damping=0.3, conv_tol=0.05)))
    m = inputs.synthetic_molecule(10, 4, 3, seed=8)
    out.append((m, dict(tau=0.01, walker_target=4e3, excitgen=F.GEN_PCHB, det_words=2, seed=8,
                        shift_damping=0.3, conv_tol=0.05)))
    return out


INTERVAL, MAX_STEPS = 50, 2000


def _load(reqs):
    return [(F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri), p)
            for s, p in reqs]


def _check_against_solo(srv, tickets, loaded):
    for t, (sysd, p) in zip(tickets, loaded):
        info = F.fciqmc_server_info(srv, t)
        assert info["state"] == F.REQ_DONE, info
        steps, att, e = solve_alone(sysd, F.fciqmc_params_default(**p), INTERVAL, MAX_STEPS)
        assert info["steps"] == steps and info["attempts"] == att, (info["steps"], steps)
        assert info["converged"] == e["converged"]
        assert_same_report(info["energy"], e)
        assert info["t_arrival"] <= info["t_admit"] <= info["t_done"]


def test_server_results_equal_solo_runs():
    loaded = _load(_requests())
    srv = F.fciqmc_server_create(200 << 30, max_running=64)
    tickets = [F.fciqmc_server_submit(srv, sysd, F.fciqmc_params_default(**p), INTERVAL, MAX_STEPS)
               for sysd, p in loaded[:3]]
    # the others arrive while the first ones run
    running, queued = F.fciqmc_server_poll(srv, 120)
    assert running == 3 and queued == 0
    tickets += [F.fciqmc_server_submit(srv, sysd, F.fciqmc_params_default(**p), INTERVAL, MAX_STEPS)
                for sysd, p in loaded[3:]]
    while True:
        running, queued = F.fciqmc_server_poll(srv, 100)
        if running == 0 and queued == 0:
            break
    assert any(F.fciqmc_server_info(srv, t)["converged"] for t in tickets)
    _check_against_solo(srv, tickets, loaded)
    F.fciqmc_server_free(srv)
    for sysd, _ in loaded:
        F.fciqmc_free_system(sysd)


def test_admission_respects_budget_in_arrival_order():
    # four molecules of one size: equal reservations, two fit the budget
    loaded = _load([(s, dict(p, walker_target=4e3)) for s, p in _requests()[:4]])
    needs = [F.fciqmc_estimate_bytes(sysd, F.fciqmc_params_default(**p)) for sysd, p in loaded]
    assert len(set(needs)) == 1
    need = needs[0]
    srv = F.fciqmc_server_create(int(2.5 * need), max_running=64)
    tickets = [F.fciqmc_server_submit(srv, sysd, F.fciqmc_params_default(**p), INTERVAL, MAX_STEPS)
               for sysd, p in loaded]
    peak = 0
    while True:
        running, queued = F.fciqmc_server_poll(srv, 10)
        peak = max(peak, running)
        assert running <= 2
        if running == 0 and queued == 0:
            break
    assert peak == 2
    admits = [F.fciqmc_server_info(srv, t)["t_admit"] for t in tickets]
    assert admits == sorted(admits)
    _check_against_solo(srv, tickets, loaded)
    F.fciqmc_server_free(srv)
    for sysd, _ in loaded:
        F.fciqmc_free_system(sysd)


def test_running_limit_and_oversized_request():
    loaded = _load(_requests()[:3])
    srv = F.fciqmc_server_create(200 << 30, max_running=1)
    tickets = [F.fciqmc_server_submit(srv, sysd, F.fciqmc_params_default(**p), INTERVAL, MAX_STEPS)
               for sysd, p in loaded]
    while True:
        running, queued = F.fciqmc_server_poll(srv, 50)
        assert running <= 1
        if running == 0 and queued == 0:
            break
    _check_against_solo(srv, tickets, loaded)
    F.fciqmc_server_free(srv)
    # a request larger than the whole budget fails without running
    sysd, p = loaded[0]
    srv = F.fciqmc_server_create(1 << 20, max_running=4)
    t = F.fciqmc_server_submit(srv, sysd, F.fciqmc_params_default(**p), INTERVAL, MAX_STEPS)
    assert F.fciqmc_server_poll(srv, 5) == (0, 0)
    info = F.fciqmc_server_info(srv, t)
    assert info["state"] == F.REQ_FAILED and info["error"] == F.ENOMEM and info["steps"] == 0
    F.fciqmc_server_free(srv)
    for sysd, _ in loaded:
        F.fciqmc_free_system(sysd)
