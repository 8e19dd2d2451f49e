#!/usr/bin/env python3
"""Benchmark of the batched direct-SCF energy/force path on one MI355X.

One step = one pass of the whole path over the batch: geometry setup (shell
pairs, Schwarz bounds, work lists, one-electron matrices, orthogonaliser), SCF
of every bead to convergence (Fock builds, DIIS, eigensolves) and analytic
forces.  Default workload: (H2O)8, RHF/6-31G* (Cartesian d, 152 basis
functions), 16 path-integral beads, FP64, SCF to 1e-8 Eh / 1e-6 commutator,
Schwarz cutoff 1e-12.

Printed metric: screened shell quartets evaluated by the Fock builds per second
of wall time (whole job).  Also reported: bead SCF iterations/s, bead energy +
force evaluations/s, the roofline of the dominant Fock-build class kernel
(algorithmic FLOPs / HIP-event kernel time vs the FP64 vector peak) and the
oracle's rate on the host cores over a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK_FP64_VECTOR_TFLOPS = 78.6   # 256 CU x 128 FP64 FLOP/clk x 2.4 GHz


def cpu_baseline(w, seconds: float):
    """Oracle Fock builds (direct J/K, McMurchie-Davidson) on bead 0, 1, ...
    until `seconds` of CPU wall time: screened shell quartets per second."""
    import numpy as np
    import inputs
    import oracle
    from oracle import rhf
    basis = inputs.load_basis(w["basis"])
    nq_total, t_total, beads = 0, 0.0, 0
    for z, x in list(w["instances"]) * 8:
        b = oracle.build_basis(basis, z, x)
        Q = oracle.schwarz(b)
        S, T, V = oracle.one_electron(b)
        X = rhf.orthogonaliser(S)
        nocc = int(np.sum(z)) // 2
        P, _, _ = rhf._density(X.T @ (T + V) @ X, X, nocc)
        t0 = time.perf_counter()
        _, _, nq = oracle.jk(b, P, 1e-12, Q)
        t_total += time.perf_counter() - t0
        nq_total += nq
        beads += 1
        if t_total >= seconds:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=nq_total / t_total, unit="screened shell-quartets/s", cores=threads,
                kind="oracle",
                sample=f"{beads} Fock build(s) (J and K at the core-guess density) of "
                       f"the beads of {w['label']}, {t_total:.1f} s on the host")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter profile
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size), or None
    when there is none or the kernel's sources changed since it was taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "fock_unit_0000_w8_16beads_hbm.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    for src in rec["source_files"]:
        with open(os.path.join(here, src), "rb") as f:
            h.update(f.read())
    return rec["hbm_bytes_per_dispatch"] if h.hexdigest() == rec["source_sha256"] else None


def guess_study(w, n_steps, dt_fs=0.25, temperature=300.0):
    """Ring-polymer MD on the workload's beads: the previous-step guess run
    integrates n_steps; the learned-guess run replays the same geometries,
    trains after every step from step 1 (5 full-batch Adam steps) and predicts
    from step 3."""
    import numpy as np
    import inputs
    from paper_1601_02713_amd import beadscf, md
    z = w["instances"][0][0]
    xb = np.array([x for _, x in w["instances"]])
    v = inputs.maxwell_boltzmann(z, len(xb), temperature, 4)
    opts = beadscf.default_opts(e_tol=w["e_tol"], comm_tol=w["comm_tol"], max_iter=60)
    basis = inputs.load_basis(w["basis"])
    e1, e2 = beadscf.Engine(0), beadscf.Engine(0)
    try:
        poly = md.RingPolymer(z, xb.copy(), v, temperature)
        def log(kind):
            return lambda r: print(f"[guess study] {kind} guess: MD step {r.step} done",
                                   file=sys.stderr, flush=True)
        ref, traj = md.run(e1, poly, n_steps, dt_fs, guess="previous", opts=opts, basis=basis,
                           log=log("previous-step"))
        lrn, _ = md.run(e2, poly, n_steps, dt_fs, guess="learned", opts=opts, geometries=traj,
                        train_from=1, train_steps=5, predict_from=3, basis=basis,
                        log=log("learned"))
    finally:
        e1.close()
        e2.close()
    k0 = 3
    it_ref = np.array([r.iterations for r in ref[k0:]], float)
    it_lrn = np.array([r.iterations for r in lrn[k0:]], float)
    dE = max(float(np.abs(a.energies - b.energies).max()) for a, b in zip(ref, lrn))
    return {
        "workload": w["label"], "md_steps": n_steps, "dt_fs": dt_fs, "compared_steps": f"{k0}..{n_steps - 1}",
        "scf_iterations_per_bead_previous_guess": float(it_ref.mean()),
        "scf_iterations_per_bead_learned_guess": float(it_lrn.mean()),
        "ms_per_step_previous_guess": float(np.mean([r.scf_ms + r.force_ms for r in ref[k0:]])),
        "ms_per_step_learned_guess_excl_training": float(np.mean([r.scf_ms + r.force_ms for r in lrn[k0:]])),
        "training_ms_per_step": float(np.mean([r.train_ms for r in lrn[k0:]])),
        "fallbacks": int(sum(int(((r.status & beadscf.STATUS_FALLBACK) != 0).sum()) for r in lrn[k0:])),
        "max_abs_dE_learned_vs_previous_Eh": dE,
    }


def per_instance_study(w, n, opts):
    """The first n instances of the workload through one batched engine, then
    each through an engine of its own (one launch sequence per instance), both
    warmed up first so that autotuning stays out of the timing: setup, SCF and
    forces per pass, wall clock."""
    import numpy as np
    import inputs
    from paper_1601_02713_amd import beadscf

    inst = w["instances"][:n]
    basis = inputs.load_basis(w["basis"])

    def engine(group):
        e = beadscf.Engine(0)
        e.load_basis(basis)
        e.set_instances([z for z, _ in group])
        return e

    def run(e, group):
        e.set_geometries([x for _, x in group])
        E, it, st = e.run_scf(opts)
        e.forces()
        return E, it

    eb = engine(inst)
    run(eb, inst)
    t0 = time.perf_counter()
    Eb, itb = run(eb, inst)
    t_batched = time.perf_counter() - t0
    eb.close()
    t_single, dE, its = 0.0, 0.0, []
    for k, one in enumerate(inst):
        e = engine([one])
        run(e, [one])
        t0 = time.perf_counter()
        E1, it1 = run(e, [one])
        t_single += time.perf_counter() - t0
        e.close()
        dE = max(dE, abs(float(E1[0]) - float(Eb[k])))
        its.append(int(it1[0]))
        print(f"[per-instance] instance {k} done", file=sys.stderr, flush=True)
    return {"instances": n, "batched_ms": t_batched * 1e3, "per_instance_ms": t_single * 1e3,
            "speedup": t_single / t_batched, "max_abs_dE_Eh": dE,
            "scf_iterations_batched": [int(v) for v in itb], "scf_iterations_single": its}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="w8_beads")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--split", type=float, default=1e-4,
                    help="mixed precision: quartets with Q_ab Q_cd below this run in FP32")
    ap.add_argument("--graph", type=int, choices=[0, 1], default=1,
                    help="replay each SCF iteration's steps after the Fock build from a HIP graph")
    ap.add_argument("--per-instance", type=int, default=0, metavar="N",
                    help="also time the first N instances batched against one engine each")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--guess-steps", type=int, default=8,
                    help="MD steps of the learned-guess study (0 skips it)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout is a design note and is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import inputs
    from paper_1601_02713_amd import beadscf

    w = inputs.workload(args.workload)
    Zs = [z for z, _ in w["instances"]]
    xs = [x for _, x in w["instances"]]
    eng = beadscf.Engine(0)
    eng.load_basis(inputs.load_basis(w["basis"]))
    eng.set_instances(Zs)
    prec = beadscf.BSCF_MIXED if args.precision == "mixed" else beadscf.BSCF_FP64
    opts = beadscf.default_opts(e_tol=w["e_tol"], comm_tol=w["comm_tol"], schwarz_tol=1e-12,
                                precision=prec, guess=beadscf.GUESS_CORE, max_iter=60,
                                fp32_split_tol=args.split, graph=args.graph)

    def step():
        eng.set_geometries(xs)
        E, it, st = eng.run_scf(opts)
        F = eng.forces()
        return E, it, st, F

    for k in range(args.warmup):
        step()
        print(f"[bench] warm-up step {k} done", file=sys.stderr, flush=True)
    eng.reset_stats()
    eng.set_profiling(True)
    iters = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        E, it, st, F = step()
        iters += int(np.sum(it))
        print(f"[bench] timed step {k} done", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    eng.set_profiling(False)
    st_json = eng.stats()
    wall = t1 - t0
    cls = st_json["classes"]
    done_q = sum(c["done_quartets"] for c in cls.values())
    k_ms = sum(c["kernel_ms"] for c in cls.values())
    k_fl = sum(c["done_flops"] for c in cls.values())
    # dominant class: the largest time alone (the autotuner's timing of the
    # chosen variant), not the largest time under the concurrent launch, where
    # a short kernel waiting behind others can look long
    fvar = 0 if prec == beadscf.BSCF_FP64 else 1
    def alone(k):   # the autotuner's time of the chosen variant
        v = cls[k]
        return v["tune_ms"][v["variant"][0]] if fvar == 0 else v["tune_ms_mixed"][v["variant"][1]]
    dom = max((k for k in cls if cls[k]["launches"]), key=alone)
    fock_gpu_ms = st_json["t_fock_gpu_ms"]
    per_class = {k: {"quartets_per_build": v["quartets"], "prim_quartets_per_build": v["prim_quartets"],
                     "ms_per_launch": v["kernel_ms"] / max(v["launches"], 1),
                     "tflops": (v["done_flops"] / (v["kernel_ms"] * 1e-3) / 1e12) if v["kernel_ms"] else None,
                     "kernel": ["lane", "coop", "lane-fp64"][v["variant"][fvar]],
                     "grad_ms_per_launch": v["grad_ms"] / max(v["grad_launches"], 1),
                     "grad_kernel": "lane" if v["variant"][2] == 0 else "coop",
                     "isolated_ms": {"lane": v["tune_ms"][0], "coop": v["tune_ms"][1],
                                     "grad_lane": v["tune_ms"][2], "grad_coop": v["tune_ms"][3]}}
                 for k, v in cls.items() if v["launches"]}
    d = cls[dom]
    ach = d["done_flops"] / (d["kernel_ms"] * 1e-3) / 1e12 if d["kernel_ms"] > 0 else 0.0
    dom_kernel = {"lane": f"fock_unit_kernel<Cls{dom}, double, false>" if fvar == 0
                  else f"fock_unit_kernel<Cls{dom}, double, true>",
                  "lane-fp64": f"fock_unit_kernel<Cls{dom}, double, false>",
                  "coop": f"coop_fock_kernel<CoopE{dom}>"}[per_class[dom]["kernel"]]
    n_inst = len(xs)
    out = {
        "metric": "screened shell-quartets/s",
        "value": done_q / wall,
        "unit": "shell-quartets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == beadscf.BSCF_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w["label"], "instances": n_inst, "basis_functions": eng.nbf[0],
                   "scf_e_tol": w["e_tol"], "scf_comm_tol": w["comm_tol"],
                   "schwarz_tol": 1e-12, "guess": "core", "graph": bool(args.graph)},
        "bead_scf_steps_per_s": iters / wall,
        "bead_energy_force_per_s": n_inst * args.steps / wall,
        "scf_iterations_per_bead": iters / (n_inst * args.steps),
        "fock_build_ms": fock_gpu_ms / max(st_json["fock_builds"], 1),
        "fock_builds_per_step": st_json["fock_builds"] / args.steps,
        "fock_quartets_per_s": done_q / (fock_gpu_ms * 1e-3) if fock_gpu_ms else None,
        "fock_tflops": k_fl / (fock_gpu_ms * 1e-3) / 1e12 if fock_gpu_ms else None,
        "fock_frac_fp64_peak": (k_fl / (fock_gpu_ms * 1e-3) / 1e12 / PEAK_FP64_VECTOR_TFLOPS) if fock_gpu_ms else None,
        "phase_ms_per_step": {k: st_json[k] / args.steps for k in
                              ("t_setup_ms", "t_scf_ms", "t_grad_ms", "t_fock_ms", "t_work_ms",
                               "t_work_host_ms")},
        "work_list_host_phases_ms_per_step": [v / args.steps for v in st_json["t_work_phase_ms"]],
        "density": {"method": "sp2", "calls_per_step": st_json["sp2_calls"] / args.steps,
                    "projection_steps_per_call": st_json["sp2_steps"] / max(st_json["sp2_calls"], 1),
                    "projection_steps_needed_per_call":
                        st_json["sp2_steps_needed"] / max(st_json["sp2_calls"], 1),
                    "fallbacks": st_json["sp2_fallbacks"]},
        "roofline": {"bound": "alu",
                     "kernel": dom_kernel,
                     "achieved": ach, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / PEAK_FP64_VECTOR_TFLOPS, "traffic": measured_traffic(dom_kernel),
                     "traffic_unit": "bytes per launch",
                     "launches": d["launches"],
                     "avg_launch_ms": d["kernel_ms"] / max(d["launches"], 1),
                     "alone_ms": alone(dom)},
        "energies_first_bead": float(E[0]),
        "classes": per_class,
    }
    if prec == beadscf.BSCF_MIXED:
        # accuracy of the timed (mixed) result against the FP64 path, bead by bead
        fp32 = sum(c["done_quartets_fp32"] for c in cls.values())
        o64 = beadscf.default_opts(e_tol=w["e_tol"], comm_tol=w["comm_tol"], schwarz_tol=1e-12,
                                   precision=beadscf.BSCF_FP64, guess=beadscf.GUESS_CORE,
                                   max_iter=60)
        E64, _, _ = eng.run_scf(o64)
        F64 = eng.forces()
        dE = np.abs(np.asarray(E) - E64)
        dF = np.array([np.abs(a - b).max() for a, b in zip(F, F64)])
        out["mixed_precision"] = {
            "fp32_split_tol": args.split, "fp32_quartet_share": fp32 / max(done_q, 1),
            "max_abs_dE_vs_fp64_Eh": float(dE.max()), "max_abs_dF_vs_fp64_Eh_per_bohr": float(dF.max()),
            "per_bead_abs_dE_Eh": [float(v) for v in dE],
            "per_bead_max_abs_dF_Eh_per_bohr": [float(v) for v in dF]}
    if args.per_instance > 0:
        out["per_instance"] = per_instance_study(w, args.per_instance, opts)
    if args.guess_steps > 0:
        eng.close()
        out["learned_guess"] = guess_study(w, args.guess_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
