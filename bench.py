"""Benchmark: spawn attempts per second of the FCIQMC step on one MI355X.

A step is one full pass of the hot path (spawn, death, annihilation with the
initiator rule, estimators, shift update) over the walker population.  The
default workload is the 4x4 periodic Hubbard model (t=1, U=4, 8 up + 8 down,
Neel reference), integer walkers with a 1e6 walker target, initiator n_a=3,
dtau=0.005, lattice excitation generator, Philox seed 1.  The population is
first grown until the shift varies (not timed: initialisation), then
`--warmup` steps run untimed while the shift settles the population at the
target, and `--steps` steps are timed.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from paper_2006_14956_amd import inputs
    import paper_2006_14956_amd.fciqmc as F
    if name == "hubbard4x4":
        s = inputs.hubbard_4x4()
        p = dict(tau=0.005, walker_target=1e6, initiator_na=3.0, excitgen=F.GEN_LATTICE, seed=1,
                 shift_damping=0.3, ref_alpha=s.ref_alpha, ref_beta=s.ref_beta)
        desc = {"workload": "hubbard_4x4_periodic_U4_t1_8up8dn_neel",
                "walkers_target": 1e6, "initiator_na": 3, "tau": 0.005,
                "excitation_generator": "lattice", "walkers": "integer", "det_bits": 64,
                "shift_damping": 0.3}
        return s, p, desc
    if name == "mol40":
        s = inputs.molecule_40o26e()
        p = dict(tau=0.0012, walker_target=1e8, initiator_na=3.0, mode=F.MODE_REAL, c_min=1.0,
                 excitgen=F.GEN_PCHB, seed=1, shift_damping=0.3, n_initial=1000.0)
        desc = {"workload": "synthetic_molecule_26e40o_damped_rank40", "walkers_target": 1e8,
                "initiator_na": 3, "tau": 0.0012, "excitation_generator": "pchb",
                "walkers": "real", "c_min": 1.0, "det_bits": 128, "shift_damping": 0.3}
        return s, p, desc
    if name == "mol8":
        s = inputs.molecule_8o8e()
        p = dict(tau=0.01, walker_target=1e4, seed=1)
        desc = {"workload": "synthetic_molecule_8e8o_4900dets", "walkers_target": 1e4,
                "tau": 0.01, "excitation_generator": "uniform", "walkers": "integer",
                "det_bits": 64}
        return s, p, desc
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(kernel, d_in, d_out, recs, words, vbytes):
    """Bytes the method must move per launch (see the measurement notes)."""
    key = 8 * words
    rec = {(1, 4): 16, (1, 8): 24, (2, 4): 24, (2, 8): 32}[(words, vbytes)]
    if kernel == "spawn":        # parent key + value + attempt prefix, records out
        return d_in * (key + vbytes + 4) + recs * rec
    if kernel == "annihilate":   # entries in (key, value, diagonal), records in, entries out
        return d_in * (key + vbytes + 8) + recs * rec + d_out * (key + vbytes + 8 + 4)
    return 0


def measure(F, np, torch, stream, name, steps, warmup):
    """Grow, settle and time one workload; returns the run and its figures."""
    s, pd, desc = workload(name)
    sysd = F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri)
    run = F.fciqmc_init(sysd, F.fciqmc_params_default(**pd), stream=stream)
    # initialisation: grow until the shift varies (not timed)
    t0 = time.perf_counter()
    grown = 0
    while grown < 5000:
        st = F.fciqmc_step(run, 10)
        grown += 10
        if st[-1]["vary_shift"]:
            break
    log(f"[{name}] grown {grown} steps in {time.perf_counter() - t0:.2f}s: N_w={st[-1]['nw']:.4g} "
        f"dets={st[-1]['ndets']} S={st[-1]['shift']:.4f}")
    if warmup:
        st = F.fciqmc_step(run, warmup)
        log(f"[{name}] warmup {warmup}: N_w={st[-1]['nw']:.4g} dets={st[-1]['ndets']} "
            f"S={st[-1]['shift']:.4f} E_proj={st[-1]['e_proj']:.5f}")
    F.fciqmc_profile(run, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = F.fciqmc_step(run, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    ms, nsteps, layout = F.fciqmc_profile(run, False)
    attempts = sum(x["attempts"] for x in st)
    spawns = sum(x["spawns"] for x in st)
    log(f"[{name}] timed {steps} steps in {wall:.4f}s: {attempts / wall:.4e} attempts/s, "
        f"{1e3 * wall / steps:.4f} ms/step; kernels (ms total): "
        + ", ".join(f"{k}={v:.2f}" for k, v in ms.items()))
    # roofline of the dominant kernel from the live event timings
    words = 1 if s.n_orb <= 32 else 2
    vbytes = 4 if pd.get("mode", F.MODE_INTEGER) == F.MODE_INTEGER else 8
    dets = [x["ndets"] for x in st]
    d_in = float(np.mean([st[0]["ndets"]] + dets[:-1]))
    d_out = float(np.mean(dets))
    recs = spawns / len(st)
    kern = {k: {"ms_per_launch": v / nsteps,
                "algorithmic_bytes": algorithmic_bytes(k, d_in, d_out, recs, words, vbytes)}
            for k, v in ms.items()}
    for k in kern:
        a = kern[k]["algorithmic_bytes"]
        kern[k]["achieved_GBps"] = a / (kern[k]["ms_per_launch"] * 1e-3) / 1e9 if a else None
    dom = max(("spawn", "annihilate"), key=lambda k: ms[k])
    roof = roofline(kern, dom)
    desc = dict(desc, dets_mean=d_out, spawns_per_step=recs, attempts_per_step=attempts / len(st),
                buckets=layout["buckets"], ms_per_step=1e3 * wall / steps,
                attempts_per_s=attempts / wall)
    return s, pd, desc, run, sysd, st, wall, ms, nsteps, layout, kern, roof


BATCH_DESC = {"workload": "batched_64_synthetic_molecules_8to24_orbitals",
              "instances": 64, "integral_seeds": "0..63", "philox_seeds": "0..63",
              "orbitals": "uniform 8..24", "electrons": "2*floor(N/2), Sz=0",
              "walkers_target": "log-uniform 1e4..1e6 per instance",
              "tau": "min(0.005, 0.3 / sum_j |H_0j|) per instance",
              "excitation_generator": "uniform", "walkers": "integer", "initiator": "off",
              "shift_damping": 0.3, "det_bits": 64}


def ref_row_norm(F, np, sysd, s):
    """sum_j |H_0j| over the single and double excitations of the aufbau
    reference, with the library's matrix elements."""
    from itertools import combinations
    na, nb, N = s.n_alpha, s.n_beta, s.n_orb
    ra, rb = (1 << na) - 1, (1 << nb) - 1
    occ_a, vir_a = list(range(na)), list(range(na, N))
    occ_b, vir_b = list(range(nb)), list(range(nb, N))
    tgt = []
    for i in occ_a:
        for a in vir_a:
            tgt.append((ra ^ (1 << i) ^ (1 << a), rb))
    for i in occ_b:
        for a in vir_b:
            tgt.append((ra, rb ^ (1 << i) ^ (1 << a)))
    for (i, j) in combinations(occ_a, 2):
        for (a, b) in combinations(vir_a, 2):
            tgt.append((ra ^ (1 << i) ^ (1 << j) ^ (1 << a) ^ (1 << b), rb))
    for (i, j) in combinations(occ_b, 2):
        for (a, b) in combinations(vir_b, 2):
            tgt.append((ra, rb ^ (1 << i) ^ (1 << j) ^ (1 << a) ^ (1 << b)))
    for i in occ_a:
        for a in vir_a:
            for j in occ_b:
                for b in vir_b:
                    tgt.append((ra ^ (1 << i) ^ (1 << a), rb ^ (1 << j) ^ (1 << b)))
    dj = np.array(tgt, dtype=np.uint64)
    di = np.tile(np.array([[ra, rb]], dtype=np.uint64), (len(dj), 1))
    return float(np.abs(F.fciqmc_matrix_elements(sysd, di, dj)).sum())


def measure_batched(F, np, steps, warmup, grow_max, tune_steps, plain=True):
    """64 independent molecules advanced as one batch (tuned), then the same
    populations from the same state advanced one run after another."""
    from paper_2006_14956_amd import inputs
    mols = inputs.batched_molecules()
    systems, runs, params = [], [], []
    batch = F.fciqmc_batch_create()
    for i, (s, target) in enumerate(mols):
        sysd = F.fciqmc_load_integrals(s.n_orb, s.n_alpha, s.n_beta, s.e_core, s.h1, s.eri)
        # dtau = 0.005, lowered where the reference row would spawn more than
        # 0.3 walkers per walker and step
        tau = min(0.005, 0.3 / ref_row_norm(F, np, sysd, s))
        p = dict(tau=tau, walker_target=target, seed=i, shift_damping=0.3)
        run = F.fciqmc_init(sysd, F.fciqmc_params_default(**p))
        F.fciqmc_batch_add(batch, run)
        systems.append(sysd)
        runs.append(run)
        params.append(p)
    t0 = time.perf_counter()
    grown = 0
    while grown < grow_max:
        st = F.fciqmc_batch_step(batch, 100)
        grown += 100
        if all(x["vary_shift"] for x in st[-1]):
            break
    last = st[-1]
    taus = [p["tau"] for p in params]
    log(f"[batched] dtau per instance: min {min(taus):.4g} max {max(taus):.4g}")
    log(f"[batched] grown {grown} steps in {time.perf_counter() - t0:.1f}s: "
        f"{sum(x['vary_shift'] for x in last)}/64 varying, N_w total {sum(x['nw'] for x in last):.4g}")
    if warmup:
        F.fciqmc_batch_step(batch, warmup)
    tune = F.fciqmc_batch_tune(batch, tune_steps)
    log(f"[batched] tuned: {tune}")
    # the state both timings start from
    snap = [(F.fciqmc_get_walkers(r), F.fciqmc_get_checkpoint(r)) for r in runs]
    F.fciqmc_batch_profile(batch, True)
    t1 = time.perf_counter()
    st = F.fciqmc_batch_step(batch, steps)
    wall = time.perf_counter() - t1
    ms, nsteps = F.fciqmc_batch_profile(batch, False)
    att = sum(x["attempts"] for row in st for x in row)
    final_b = [x["nw"] for x in st[-1]]
    rate_b = att / wall
    log(f"[batched] timed {steps} steps in {wall:.3f}s: {rate_b:.4e} attempts/s, "
        f"{1e3 * wall / steps:.4f} ms/step; kernels (ms total): "
        + ", ".join(f"{k}={v:.2f}" for k, v in ms.items()))
    ndets = sum(x["ndets"] for x in st[-1])
    F.fciqmc_batch_free(batch)
    for r in runs:
        F.fciqmc_free_run(r)
    out = {"config": dict(BATCH_DESC, steps=steps, grown_steps=grown,
                          walkers_total=float(sum(final_b)), dets_total=int(ndets)),
           "value": rate_b, "unit": "attempts/s", "ms_per_step": 1e3 * wall / steps,
           "kernels_ms_per_step": {k: v / max(1, nsteps) for k, v in ms.items()},
           "tune": tune}
    if plain:
        solo = []
        for i, ((a, b, v), ck) in enumerate(snap):
            r = F.fciqmc_init(systems[i], F.fciqmc_params_default(**params[i]))
            F.fciqmc_set_walkers(r, a, b, v)
            F.fciqmc_set_checkpoint(r, **ck)
            solo.append(r)
        t2 = time.perf_counter()
        sst = [F.fciqmc_step(r, steps) for r in solo]
        wall_p = time.perf_counter() - t2
        att_p = sum(x["attempts"] for rs in sst for x in rs)
        same = all(rs[-1]["nw"] == nb for rs, nb in zip(sst, final_b))
        log(f"[plain] {steps} steps of each run in turn: {wall_p:.3f}s, {att_p / wall_p:.4e} attempts/s; "
            f"final populations equal to the batch's: {same}")
        for r in solo:
            F.fciqmc_free_run(r)
        out.update(plain_value=att_p / wall_p, plain_wall_s=wall_p, batched_wall_s=wall,
                   speedup_vs_plain=wall_p / wall, same_trajectories=same)
    for sysd in systems:
        F.fciqmc_free_system(sysd)
    return out


def roofline(kern, k):
    ab = kern[k]["algorithmic_bytes"]
    achieved = ab / (kern[k]["ms_per_launch"] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": k, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "algorithmic_bytes_per_launch": ab, "ms_per_launch": kern[k]["ms_per_launch"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--workload", default="hubbard4x4")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--second", default="mol40",
                    help="second workload measured after the first ('' to skip)")
    ap.add_argument("--second-steps", type=int, default=60)
    ap.add_argument("--second-warmup", type=int, default=400)
    ap.add_argument("--batched-steps", type=int, default=1000,
                    help="timed steps of the 64-molecule batch (0 to skip)")
    ap.add_argument("--batched-warmup", type=int, default=200)
    ap.add_argument("--batched-grow", type=int, default=20000)
    ap.add_argument("--batched-tune", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "path is a design, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2006_14956_amd.fciqmc as F

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    s, pd, desc, run, sysd, st, wall, ms, nsteps, layout, kern, roof = measure(
        F, np, torch, stream, args.workload, args.steps, args.warmup)
    attempts = sum(x["attempts"] for x in st)
    spawns = sum(x["spawns"] for x in st)
    value = attempts / wall
    words = 1 if s.n_orb <= 32 else 2
    d_out = float(np.mean([x["ndets"] for x in st]))
    recs = spawns / len(st)

    cpu = None
    if not args.no_cpu:
        import oracle
        a, b, v = F.fciqmc_get_walkers(run)
        ck = F.fciqmc_get_checkpoint(run)
        osys = oracle.System.from_inputs(s, words=words)
        orun = oracle.Run(osys, ref=(pd.get("ref_alpha", 0), pd.get("ref_beta", 0)),
                          tau=pd["tau"], target=pd["walker_target"],
                          n_a=pd.get("initiator_na", -1.0), zeta=pd.get("shift_damping", 0.05),
                          gen={F.GEN_UNIFORM: oracle.GEN_UNIFORM, F.GEN_LATTICE: oracle.GEN_LATTICE,
                               F.GEN_PCHB: oracle.GEN_PCHB}[pd.get("excitgen", F.GEN_UNIFORM)],
                          seed=pd["seed"])
        orun.set_walkers(a, b, v)
        orun.set_state(ck["iter"], ck["shift"], ck["vary_shift"], ck["last_update_iter"],
                       ck["last_update_nw"])
        c0 = time.perf_counter()
        oatt = 0
        osteps = 0
        while osteps == 0 or time.perf_counter() - c0 < args.cpu_seconds:
            oatt += orun.step(1)[0]["attempts"]
            osteps += 1
        cwall = time.perf_counter() - c0
        cpu = {"value": oatt / cwall, "unit": "attempts/s", "cores": 1, "kind": "oracle",
               "sample": f"{osteps} oracle steps from the GPU's state after the timed region "
                         f"({len(v)} determinants), {cwall:.1f}s on one host core"}
        log(f"cpu oracle: {osteps} steps, {oatt / cwall:.4e} attempts/s")

    second = None
    if args.second:
        F.fciqmc_free_run(run)
        F.fciqmc_free_system(sysd)
        run = sysd = None
        _, _, desc2, run2, sys2, _, wall2, _, _, _, kern2, _ = measure(
            F, np, torch, stream, args.second, args.second_steps, args.second_warmup)
        second = {"config": desc2, "value": desc2["attempts_per_s"], "unit": "attempts/s",
                  "ms_per_step": desc2["ms_per_step"], "kernels": kern2,
                  "roofline_annihilate": roofline(kern2, "annihilate")}
        F.fciqmc_free_run(run2)
        F.fciqmc_free_system(sys2)

    batched = None
    if args.batched_steps:
        batched = measure_batched(F, np, args.batched_steps, args.batched_warmup, args.batched_grow,
                                  args.batched_tune)

    out = {
        "metric": "spawn attempts/s (spawn+annihilate+death)",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": desc,
        "kernels": kern,
        "roofline": roof,
        "cpu_baseline": cpu,
        "second_workload": second,
        "batched": batched,
    }
    print(json.dumps(out), flush=True)
    if run is not None:
        F.fciqmc_free_run(run)
        F.fciqmc_free_system(sysd)


if __name__ == "__main__":
    main()
