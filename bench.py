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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--workload", default="hubbard4x4")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
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
    s, pd, desc = workload(args.workload)
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
    log(f"grown {grown} steps in {time.perf_counter() - t0:.2f}s: N_w={st[-1]['nw']:.0f} "
        f"dets={st[-1]['ndets']} S={st[-1]['shift']:.4f}")
    if args.warmup:
        st = F.fciqmc_step(run, args.warmup)
        log(f"warmup {args.warmup}: N_w={st[-1]['nw']:.0f} dets={st[-1]['ndets']} "
            f"S={st[-1]['shift']:.4f} E_proj={st[-1]['e_proj']:.5f}")

    F.fciqmc_profile(run, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = F.fciqmc_step(run, args.steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    wall = t2 - t1
    ms, nsteps, layout = F.fciqmc_profile(run, False)
    attempts = sum(x["attempts"] for x in st)
    spawns = sum(x["spawns"] for x in st)
    dets = [x["ndets"] for x in st]
    value = attempts / wall
    log(f"timed {args.steps} steps in {wall:.4f}s: {value:.4e} attempts/s, "
        f"{1e3 * wall / args.steps:.4f} ms/step; kernels (ms total): "
        + ", ".join(f"{k}={v:.2f}" for k, v in ms.items()))

    # roofline of the dominant kernel from the live event timings
    words = 1 if s.n_orb <= 32 else 2
    vbytes = 4
    d_in = float(np.mean([st[0]["ndets"]] + dets[:-1]))
    d_out = float(np.mean(dets))
    recs = spawns / len(st)
    dom = max(("spawn", "annihilate"), key=lambda k: ms[k])
    per_launch_ms = ms[dom] / nsteps
    ab = algorithmic_bytes(dom, d_in, d_out, recs, words, vbytes)
    achieved = ab / (per_launch_ms * 1e-3) / 1e9
    kern = {k: {"ms_per_launch": v / nsteps,
                "algorithmic_bytes": algorithmic_bytes(k, d_in, d_out, recs, words, vbytes)}
            for k, v in ms.items()}
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "algorithmic_bytes_per_launch": ab, "ms_per_launch": per_launch_ms}

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
        "config": dict(desc, dets_mean=d_out, spawns_per_step=recs,
                       attempts_per_step=attempts / len(st), buckets=layout["buckets"]),
        "kernels": kern,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    F.fciqmc_free_run(run)
    F.fciqmc_free_system(sysd)


if __name__ == "__main__":
    main()
