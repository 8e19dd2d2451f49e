#!/usr/bin/env python3
"""Benchmark of the batched direct-SCF energy/force path on one MI355X.

Default (--mode md): ring-polymer MD of (H2O)32, RHF/6-31G* (Cartesian d,
608 basis functions), 32 beads, 0.25 fs steps at 300 K (PILE-L thermostat,
Maxwell-Boltzmann start).  One step = one pass of the whole path over the
batch: the device integrator moves every bead, the geometry setup (shell
pairs, Schwarz bounds, screened work lists, one-electron matrices,
orthogonaliser), the SCF of every bead to 1e-8 Eh / 1e-6 commutator with
Schwarz cutoff 1e-12, the analytic forces, and the in-run training of the
learned guess.

Two legs on the same geometries:
  * the timed path: mixed precision (FP32 primitive integrals below the
    Schwarz-product split, FP64 accumulation) with the learned SCF guess
    (trained after every step from step 1, predicting from step 3);
  * the plain FP64 GPU path with the paper's standard previous-step guess,
    replaying the timed path's geometries.
Both are timed over the same steps after the same warm-up steps, and their
per-bead energies and forces are compared (the timed path counts only if it
is within 1e-6 Eh and 1e-5 Eh/bohr of the FP64 path on every bead).

Printed metric: screened shell quartets per second of Fock-build GPU time
(the Schwarz-screened quartets of every instance each build covered, full
or incremental, over the HIP-event time of the builds), next to bead SCF
iterations per second, bead energy + force evaluations per second and the
wall time per MD step, with the FP64 leg's figures and the ratios.  Also:
the roofline of the dominant Fock-build class kernel (algorithmic FLOPs
counted from the kernel code over its HIP-event launch time against the FP64
vector peak) and the oracle's rate on the host cores over a bounded sample.

--mode scf times setup + SCF + forces of a fixed batch (the earlier form of
this benchmark; --workload w8_beads, w16_beads, uneven, ...).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

PEAK_FP64_VECTOR_TFLOPS = 78.6   # 256 CU x 128 FP64 FLOP/clk x 2.4 GHz
PEAK_FP64_MATRIX_TFLOPS = 78.6   # dense FP64 MFMA, the published figure
PEAK_HBM_GBS = 8000.0            # HBM3E
FS = 41.341373336
HERE = os.path.dirname(os.path.abspath(__file__))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- CPU baseline

def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, seconds: float):
    """The oracle's direct J/K (McMurchie-Davidson, canonical screened quartet
    list, OpenMP) on bead 0 of the workload over a strided sample of its
    quartet list, on all host threads and on one: screened shell quartets
    per second."""
    import numpy as np
    import inputs
    import oracle
    z, x = w["instances"][0]
    b = oracle.build_basis(inputs.load_basis(w["basis"]), z, x)
    Q = oracle.schwarz(b)
    rng = np.random.default_rng([4242, 1])
    A = rng.standard_normal((b["nbf"], b["nbf"]))
    P = 0.01 * (A + A.T)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def rate(stride, nt):
        t0 = time.perf_counter()
        _, _, nq = oracle.jk_sample(b, P, stride, nt, 1e-12, Q)
        return nq, time.perf_counter() - t0

    def sized(stride, nt, target):
        # a short probe underestimates the rate (fixed costs), so the stride
        # is refined until the sample takes about the target time
        nq, t = rate(stride, nt)
        for _ in range(4):
            if t >= 0.5 * target or stride == 1:
                break
            stride = max(1, int(stride * t / target))
            nq, t = rate(stride, nt)
        return stride, nq, t

    stride, nq, t = sized(4096, threads, seconds)
    s1, nq1, t1 = sized(stride * threads, 1, seconds / 3)
    return dict(value=nq / t, unit="screened shell-quartets/s", cores=threads, kind="oracle",
                cpu_model=cpu_model(), one_core_value=nq1 / t1,
                sample=f"every {stride}th quartet of the canonical Schwarz-screened list of bead 0 of "
                       f"{w['label']} ({nq} shell quartets, J and K at a seeded density), {t:.1f} s "
                       f"on {threads} threads; one thread: every {s1}th, {nq1} quartets, {t1:.1f} s")


# --------------------------------------------------------------- roofline data

def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from a committed counter profile of
    this workload (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known
    size), or None when there is none or its sources changed since."""
    pdir = os.path.join(HERE, "profiles")
    for name in sorted(os.listdir(pdir)) if os.path.isdir(pdir) else []:
        if not name.endswith("_hbm.json"):
            continue
        with open(os.path.join(pdir, name)) as f:
            rec = json.load(f)
        if rec.get("kernel") != kernel or rec.get("workload") != workload:
            continue
        h = hashlib.sha256()
        try:
            for src in rec["source_files"]:
                with open(os.path.join(HERE, src), "rb") as f:
                    h.update(f.read())
        except OSError:   # a generated source not built here
            continue
        if h.hexdigest() == rec["source_sha256"]:
            return rec["hbm_bytes_per_dispatch"]
    return None


def nout_of(tag):
    """Cartesian integrals of one shell quartet of class tag ("LaLbLcLd")."""
    n = 1
    for ch in tag:
        l = int(ch)
        n *= (l + 1) * (l + 2) // 2
    return n


def kernel_name(dom, variant, mixed):
    if variant == "coop":
        return f"coop_fock_kernel<CoopE{dom}>"
    if variant == "lane" and mixed:
        return f"fock_unit_kernel<Cls{dom}, double, true>"
    return f"fock_unit_kernel<Cls{dom}, double, false>"


def fock_summary(st, mixed, workload):
    """Screened quartets per Fock-build second, per-class figures and the
    roofline of the class kernel with the most time in the timed builds."""
    cls = st["classes"]
    fvar = 1 if mixed else 0
    screened = sum(c["screened_quartets_built"] for c in cls.values())
    fock_gpu_s = st["t_fock_gpu_ms"] * 1e-3
    per_class = {}
    for k, v in cls.items():
        if not v["launches"]:
            continue
        var = ["lane", "coop", "lane-fp64"][v["variant"][fvar]]
        per_class[k] = {
            "screened_quartets_per_build": v["quartets"], "prim_quartets_per_build": v["prim_quartets"],
            "kernel": var, "launches": v["launches"],
            "ms_per_launch": v["kernel_ms"] / v["launches"],
            "tflops": v["done_flops"] / (v["kernel_ms"] * 1e-3) / 1e12 if v["kernel_ms"] else None,
            "flops_per_prim_quartet": v["prim_flops"], "flops_per_quartet_hrr": v["hrr_flops"],
            "fp32_quartet_share": v["done_quartets_fp32"] / max(v["done_quartets"], 1),
            "grad_kernel": "lane" if v["variant"][2] == 0 else "coop",
            "grad_ms_per_launch": v["grad_ms"] / max(v["grad_launches"], 1),
            # the gradient's algorithmic FLOPs (setup, Boys to L + 1, raised and
            # lowered VRR per evaluated primitive quartet, contraction per
            # evaluated quartet, counted on the device) per forces call, and
            # their rate in the concurrent schedule and alone
            "grad_flops_per_call": v["grad_flops"] / max(v["grad_launches"], 1),
            "grad_tflops": v["grad_flops"] / (v["grad_ms"] * 1e-3) / 1e12 if v["grad_ms"] else None,
            "grad_alone_tflops": (v["grad_flops"] / max(v["grad_launches"], 1)
                                  / (v["tune_ms"][2 + v["variant"][2]] * 1e-3) / 1e12
                                  if v["tune_ms"][2 + v["variant"][2]] else None),
            # the autotuner's timing of the chosen kernels, each alone on the GPU
            "alone_ms": (v["tune_ms_mixed"][v["variant"][1]] if mixed else v["tune_ms"][v["variant"][0]]),
            "grad_alone_ms": v["tune_ms"][2 + v["variant"][2]]}
    dom = max(per_class, key=lambda k: cls[k]["kernel_ms"])
    d = cls[dom]
    avg_ms = d["kernel_ms"] / d["launches"]
    ach = d["done_flops"] / d["launches"] / (avg_ms * 1e-3) / 1e12
    kname = kernel_name(dom, per_class[dom]["kernel"], mixed)
    # the same kernel alone: the autotuner's time of a full build and the
    # algorithmic FLOPs of a full build of the class (the concurrent build
    # stretches each kernel's own duration)
    full_flops = d["prim_quartets"] * d["prim_flops"] + d["quartets"] * (
        d["hrr_flops"] + 12.0 * nout_of(dom))
    alone = per_class[dom]["alone_ms"]
    roof = {"bound": "alu", "kernel": kname, "achieved": ach, "peak": PEAK_FP64_VECTOR_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / PEAK_FP64_VECTOR_TFLOPS,
            "alone": {"ms_full_build": alone,
                      "achieved": full_flops / (alone * 1e-3) / 1e12 if alone else None,
                      "frac": full_flops / (alone * 1e-3) / 1e12 / PEAK_FP64_VECTOR_TFLOPS
                      if alone else None},
            "traffic": measured_traffic(kname, workload), "traffic_unit": "bytes per launch",
            "launches": d["launches"], "avg_launch_ms": avg_ms,
            "flops_per_launch": d["done_flops"] / d["launches"],
            "flop_count": "per primitive quartet the setup, Boys and VRR FLOPs counted from the "
                          "kernel code by the generator, per contracted quartet the HRR plus 12 "
                          "per Cartesian integral (J and K digestion), over the quartets each "
                          "launch evaluated"}
    fp32 = sum(c["done_quartets_fp32"] for c in cls.values())
    done = sum(c["done_quartets"] for c in cls.values())
    flops = sum(c["done_flops"] for c in cls.values())
    return {"screened_quartets_per_s": screened / fock_gpu_s if fock_gpu_s else None,
            "screened_quartets_built": screened, "fock_gpu_ms": st["t_fock_gpu_ms"],
            "fock_builds": st["fock_builds"], "quartets_evaluated": done,
            "fp32_quartet_share": fp32 / max(done, 1),
            "fock_tflops": flops / fock_gpu_s / 1e12 if fock_gpu_s else None,
            "classes": per_class, "roofline": roof}


# --------------------------------------------------------------------- MD mode

def md_bench(args):
    import numpy as np
    import inputs
    from paper_1601_02713_amd import beadscf, md

    w = inputs.workload(args.workload)
    basis = inputs.load_basis(w["basis"])
    z = w["instances"][0][0]
    xb = np.array([x for _, x in w["instances"]])
    P = len(xb)
    masses = np.array([md.MASS_AMU[int(v)] for v in z]) * md.AMU
    v0 = inputs.maxwell_boltzmann(z, P, args.temperature, 4)
    total = args.warmup + args.steps
    prec = beadscf.BSCF_MIXED if args.precision == "mixed" else beadscf.BSCF_FP64
    use_learned = args.guess == "learned"

    def opts(precision, guess):
        return beadscf.default_opts(e_tol=w["e_tol"], comm_tol=w["comm_tol"], schwarz_tol=1e-12,
                                    precision=precision, guess=guess, max_iter=60,
                                    fp32_split_tol=args.split, graph=args.graph)

    # ---- the timed path: integrate, mixed precision, learned guess
    eng = beadscf.Engine(0)
    eng.load_basis(basis)
    eng.set_instances([z] * P)
    eng.set_geometries(list(xb))
    eng.pimd_init(masses, v0 * masses[None, :, None],
                  beadscf.pimd_default_opts(dt=args.dt_fs * FS, temperature=args.temperature,
                                            thermostat=1, tau_centroid=100 * FS, seed=1))
    traj, Eh, Fh, its, train_ms = [], [], [], [], []
    t0 = None
    for step in range(total):
        if step == args.warmup:
            eng.reset_stats()
            eng.set_profiling(True)
            t0 = time.perf_counter()
        if step == 0:
            E, it, st = eng.run_scf(opts(prec, beadscf.GUESS_CORE))
            F = eng.forces()
        else:
            g = beadscf.GUESS_PREVIOUS
            if use_learned and step >= args.predict_from:
                g = beadscf.GUESS_LEARNED
            elif args.guess == "extrapolated":
                g = beadscf.GUESS_EXTRAPOLATED
            E, it, st, F = eng.pimd_step(opts(prec, g), return_forces=True)
        tt = time.perf_counter()
        if use_learned and step >= 1:
            eng.guess_train(args.train_steps)
        train_ms.append((time.perf_counter() - tt) * 1e3)
        traj.append(eng.pimd_state()[0])
        Eh.append(E)
        Fh.append(np.array(F))
        its.append(it)
        log(f"timed path: MD step {step} done ({'timed' if step >= args.warmup else 'warm-up'}, "
            f"{it.mean():.2f} SCF iterations per bead)")
    wall = time.perf_counter() - t0
    eng.set_profiling(False)
    sh = eng.stats()
    nbf = eng.nbf[0]
    eng.close()

    # ---- the plain FP64 GPU path on the same geometries, previous-step guess
    nb = min(args.baseline_steps or args.steps, args.steps)
    e64 = beadscf.Engine(0)
    e64.load_basis(basis)
    e64.set_instances([z] * P)
    E64, F64, its64 = [], [], []
    tb = None
    for step in range(args.warmup + nb):
        if step == args.warmup:
            e64.reset_stats()
            e64.set_profiling(True)
            tb = time.perf_counter()
        e64.set_geometries(list(traj[step]))
        E, it, st = e64.run_scf(opts(beadscf.BSCF_FP64,
                                     beadscf.GUESS_CORE if step == 0 else beadscf.GUESS_PREVIOUS))
        F = e64.forces()
        E64.append(E)
        F64.append(np.array(F))
        its64.append(it)
        log(f"plain FP64 path: MD step {step} done")
    wall64 = time.perf_counter() - tb
    e64.set_profiling(False)
    s64 = e64.stats()
    e64.close()

    k0 = args.warmup
    dE = max(float(np.abs(Eh[k] - E64[k]).max()) for k in range(k0, k0 + nb))
    dF = max(float(np.abs(Fh[k] - F64[k]).max()) for k in range(k0, k0 + nb))
    head = fock_summary(sh, prec == beadscf.BSCF_MIXED, w["label"])
    base = fock_summary(s64, False, w["label"])
    it_h = float(np.mean([its[k].mean() for k in range(k0, total)]))
    it_b = float(np.mean([its64[k].mean() for k in range(k0, k0 + nb)]))
    scf_h = float(sum(its[k].sum() for k in range(k0, total))) / wall
    scf_b = float(sum(its64[k].sum() for k in range(k0, k0 + nb))) / wall64
    step_h, step_b = wall / args.steps * 1e3, wall64 / nb * 1e3
    out = {
        "metric": "screened shell-quartets/s and bead SCF-steps/s vs plain FP64 GPU at 1e-6 Eh",
        "value": head["screened_quartets_per_s"],
        "unit": "screened shell-quartets/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_h,
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == beadscf.BSCF_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": w["label"], "mode": "ring-polymer MD",
                   "beads": P, "basis_functions": nbf, "dt_fs": args.dt_fs,
                   "temperature_K": args.temperature, "thermostat": "PILE-L",
                   "precision": args.precision, "fp32_split_tol": args.split,
                   "guess": args.guess, "scf_e_tol": w["e_tol"], "scf_comm_tol": w["comm_tol"],
                   "schwarz_tol": 1e-12},
        "bead_scf_steps_per_s": scf_h,
        "bead_energy_force_per_s": P * args.steps / wall,
        "md_step_ms": step_h,
        "scf_iterations_per_bead": it_h,
        "training_ms_per_step": float(np.mean(train_ms[k0:])),
        "fock": {k: v for k, v in head.items() if k not in ("roofline",)},
        "roofline": head["roofline"],
        # t_work_ms: the SCF's wait for the screened work lists and their
        # upload; t_work_host_ms: the host build of the lists (on worker
        # threads, behind the geometry's device set-up)
        "phase_ms_per_step": {k: sh[k] / args.steps for k in
                              ("t_setup_ms", "t_scf_ms", "t_grad_ms", "t_fock_ms", "t_work_ms",
                               "t_work_host_ms")},
        # the host build's phases: ket lists, per (class, instance) parts, merges
        "work_host_phases_ms_per_step": [v / args.steps for v in sh["t_work_phase_ms"]],
        "plain_fp64_gpu": {
            "steps": nb, "guess": "previous-step orbitals",
            "screened_quartets_per_s": base["screened_quartets_per_s"],
            "bead_scf_steps_per_s": scf_b, "bead_energy_force_per_s": P * nb / wall64,
            "md_step_ms": step_b, "scf_iterations_per_bead": it_b,
            "fock_tflops": base["fock_tflops"], "roofline": base["roofline"]},
        "vs_plain_fp64_gpu": {
            "screened_quartets_per_s": head["screened_quartets_per_s"] / base["screened_quartets_per_s"],
            "bead_scf_steps_per_s": scf_h / scf_b,
            "bead_energy_force_per_s": step_b / step_h,
            "md_step_time": step_b / step_h},
        "accuracy_vs_plain_fp64_gpu": {"max_abs_dE_Eh": dE, "max_abs_dF_Eh_per_bohr": dF,
                                       "within_1e-6_Eh_1e-5_Eh_per_bohr": dE <= 1e-6 and dF <= 1e-5},
    }
    if not args.no_cpu_baseline:
        log("oracle sample on the host")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------- B3LYP mode

def xc_summary(st, nbf):
    """Per-step XC kernel times and rooflines (HIP events over the timed
    region): the basis and point kernels against HBM bandwidth (algorithmic
    bytes per grid point 8 m + 32 and 16 m + 32, m the functions the point
    takes: n in the dense form, its chunk's in the sparse one), the two
    products per chunk (Z = B P and X^T B, 2 G m^2 FLOPs each per instance,
    m padded to the bucket width) against the FP64 matrix peak."""
    x = st["xc"]
    pts = x["points"]
    rows = {}
    for k, (nbytes, flops) in {"basis": (x["basis_bytes"], None), "point": (x["point_bytes"], None),
                               "gemm": (None, x["gemm_flops"] / 2),
                               "gemm_v": (None, x["gemm_flops"] / 2)}.items():
        ms, launches = x["ms"][k]
        if not launches or not ms:
            continue
        if nbytes is not None:
            a = nbytes / (ms * 1e-3) / 1e9
            rows[k] = {"bound": "hbm", "achieved": a, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": a / PEAK_HBM_GBS, "ms": ms, "launches": launches,
                       "avg_launch_ms": ms / launches, "bytes_per_point": nbytes / max(pts, 1)}
        else:
            a = flops / (ms * 1e-3) / 1e12
            rows[k] = {"bound": "mfma", "achieved": a, "peak": PEAK_FP64_MATRIX_TFLOPS, "unit": "TFLOP/s",
                       "frac": a / PEAK_FP64_MATRIX_TFLOPS, "ms": ms, "launches": launches,
                       "avg_launch_ms": ms / launches}
    return rows


def b3lyp_bench(args):
    """Ring-polymer MD at B3LYP, the paper's level of theory (Section 3.1):
    every step the B3LYP SCF of all beads from the previous step's orbitals,
    the B3LYP forces and the PILE-L integrator, as in the MD mode; then as
    many Hartree-Fock MD steps from the same start, for the cost of the
    exchange-correlation part."""
    import numpy as np
    import inputs
    from paper_1601_02713_amd import beadscf, md

    w = inputs.workload(args.workload)
    basis = inputs.load_basis(w["basis"])
    z = w["instances"][0][0]
    xb = np.array([x for _, x in w["instances"]])
    P = len(xb)
    masses = np.array([md.MASS_AMU[int(v)] for v in z]) * md.AMU
    v0 = inputs.maxwell_boltzmann(z, P, args.temperature, 4)
    total = args.warmup + args.steps
    prec = beadscf.BSCF_MIXED if args.precision == "mixed" else beadscf.BSCF_FP64

    def opts(guess):
        return beadscf.default_opts(e_tol=w["e_tol"], comm_tol=w["comm_tol"], schwarz_tol=1e-12,
                                    precision=prec, guess=guess, max_iter=60,
                                    fp32_split_tol=args.split, graph=args.graph)

    def run(xc):
        name = "B3LYP" if xc else "Hartree-Fock"
        eng = beadscf.Engine(0)
        eng.load_basis(basis)
        eng.set_instances([z] * P)
        eng.set_xc(beadscf.XC_B3LYP if xc else beadscf.XC_NONE)
        eng.set_geometries(list(xb))
        eng.pimd_init(masses, v0 * masses[None, :, None],
                      beadscf.pimd_default_opts(dt=args.dt_fs * FS, temperature=args.temperature,
                                                thermostat=1, tau_centroid=100 * FS, seed=1))
        its, Es, t0 = [], [], None
        for k in range(total):
            if k == args.warmup:
                eng.reset_stats()
                eng.set_profiling(True)
                t0 = time.perf_counter()
            if k == 0:
                E, it, st = eng.run_scf(opts(beadscf.GUESS_CORE))
                F = eng.forces()
            else:
                E, it, st, F = eng.pimd_step(opts(beadscf.GUESS_PREVIOUS), return_forces=True)
            if np.any(st != 0):
                raise RuntimeError(f"SCF did not converge: status {st}")
            if not np.all(np.isfinite(np.concatenate([np.ravel(f) for f in F]))):
                raise RuntimeError("non-finite forces")
            its.append(it)
            Es.append(E)
            log(f"{name}: MD step {k} done ({it.mean():.2f} SCF iterations per bead)")
        wall = time.perf_counter() - t0
        eng.set_profiling(False)
        stats = eng.stats()
        nbf = eng.nbf[0]
        npts = eng.xc_grid_size(0)
        eng.close()
        return wall, np.array(its[args.warmup:]), Es, stats, nbf, npts

    wall, its, Es, st, nbf, npts = run(True)
    wall_hf, its_hf, _, st_hf, _, _ = run(False)
    fs = fock_summary(st, prec == beadscf.BSCF_MIXED, w["label"])
    xr = xc_summary(st, nbf)
    dom = max(xr, key=lambda k: xr[k]["ms"])
    x = st["xc"]
    K = args.steps
    out = {
        "metric": "screened shell-quartets/s and bead SCF-steps/s vs plain FP64 GPU at 1e-6 Eh",
        "value": fs["screened_quartets_per_s"], "unit": "screened shell-quartets/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == beadscf.BSCF_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w["label"].replace("RHF", "B3LYP"), "mode": "ring-polymer MD",
                   "beads": P, "basis_functions": nbf, "grid": "60 radial x 288 angular per atom",
                   "grid_points_per_bead": npts, "dt_fs": args.dt_fs,
                   "temperature_K": args.temperature, "thermostat": "PILE-L",
                   "precision": args.precision, "guess": "previous-step orbitals",
                   "scf_e_tol": w["e_tol"], "scf_comm_tol": w["comm_tol"], "schwarz_tol": 1e-12},
        "md_step_ms": wall / K * 1e3,
        "phase_ms_per_step": {"t_scf_ms": st["t_scf_ms"] / K, "t_grad_ms": st["t_grad_ms"] / K},
        "bead_scf_steps_per_s": float(its.sum()) / wall,
        "scf_iterations_per_bead": float(its.mean()),
        "xc": {"builds": x["builds"], "ms_per_build": x["ms"]["build"][0] / max(x["builds"], 1),
               "share_of_scf_time": x["ms"]["build"][0] / (st["t_scf_ms"] or 1),
               "gradient_ms_per_step": {"basis_function_term": x["ms"]["grad_basis_term"][0] / K,
                                        "weight_term": x["ms"]["grad_weight_term"][0] / K},
               "kernels": xr},
        "fock": {k: v for k, v in fs.items() if k != "roofline"},
        "fock_roofline": fs["roofline"],
        "roofline": {k: v for k, v in xr[dom].items()} | {"kernel": f"xc {dom}", "traffic": None},
        "hartree_fock_md": {
            "ms_per_step": wall_hf / K * 1e3,
            "phase_ms_per_step": {"t_scf_ms": st_hf["t_scf_ms"] / K,
                                  "t_grad_ms": st_hf["t_grad_ms"] / K},
            "bead_scf_steps_per_s": float(its_hf.sum()) / wall_hf,
            "scf_iterations_per_bead": float(its_hf.mean())},
        "b3lyp_over_hf_step_time": wall / wall_hf,
        "energies_last_step_Eh": [float(v) for v in Es[-1]],
    }
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ string mode

def string_bench(args):
    """String method on proton transfer in H5O2+ (a synthetic reaction):
    images on the straight line between the mirrored reactant and product,
    ends held, every iteration the SCF of every image, forces and the
    device update; timed iterations after warm-up ones."""
    import numpy as np
    import inputs
    from paper_1601_02713_amd import beadscf

    n = args.images
    z, x0 = inputs.zundel_path(n)
    basis = "6-31g*"
    eng = beadscf.Engine(0)
    eng.load_basis(inputs.load_basis(basis))
    eng.set_instances([z] * n, [1] * n)
    eng.set_geometries(list(x0))
    eng.string_init(step=0.5, fix_ends=1)
    prec = beadscf.BSCF_MIXED if args.precision == "mixed" else beadscf.BSCF_FP64
    so = beadscf.default_opts(e_tol=1e-8, comm_tol=1e-6, schwarz_tol=1e-12, precision=prec,
                              guess=beadscf.GUESS_PREVIOUS, max_iter=60, fp32_split_tol=args.split)
    its, Es = [], []
    t0 = None
    for k in range(args.warmup + args.steps):
        if k == args.warmup:
            eng.reset_stats()
            eng.set_profiling(True)
            t0 = time.perf_counter()
        E, it, st, _ = eng.string_step(so)
        its.append(it)
        Es.append(E)
        log(f"string iteration {k} done ({it.min()}-{it.max()} SCF iterations per image)")
    wall = time.perf_counter() - t0
    eng.set_profiling(False)
    st = eng.stats()
    fs = fock_summary(st, prec == beadscf.BSCF_MIXED, f"H5O2+ proton transfer, {n} images")
    _, arc = eng.string_state()
    eng.close()
    timed = np.array(its[args.warmup:])
    out = {
        "metric": "screened shell-quartets/s and bead SCF-steps/s vs plain FP64 GPU at 1e-6 Eh",
        "value": fs["screened_quartets_per_s"], "unit": "screened shell-quartets/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == beadscf.BSCF_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"H5O2+ proton transfer, RHF/6-31G*, {n} images", "mode": "string method",
                   "step_bohr2_per_Eh": 0.5, "ends": "held", "precision": args.precision,
                   "guess": "previous-step orbitals", "scf_e_tol": 1e-8, "scf_comm_tol": 1e-6},
        "image_scf_steps_per_s": float(timed.sum()) / wall,
        "image_energy_force_per_s": n * args.steps / wall,
        "scf_iterations_per_image": {"mean": float(timed.mean()), "min": int(timed.min()),
                                     "max": int(timed.max())},
        "fock": {k: v for k, v in fs.items() if k != "roofline"},
        "roofline": fs["roofline"],
        "energy_profile_Eh": [float(v) for v in Es[-1]],
        "arc_positions": [float(v) for v in arc],
    }
    print(json.dumps(out), flush=True)


# -------------------------------------------------------------------- SCF mode

def per_instance_study(w, n, opts):
    """The first n instances of the workload through one batched engine, then
    each through an engine of its own, both warmed up first (autotuning stays
    out of the timing): setup, SCF and forces per pass, wall clock."""
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
        log(f"per-instance: instance {k} done")
    return {"instances": n, "batched_ms": t_batched * 1e3, "per_instance_ms": t_single * 1e3,
            "speedup": t_single / t_batched, "max_abs_dE_Eh": dE,
            "scf_iterations_batched": [int(v) for v in itb], "scf_iterations_single": its}


def scf_bench(args):
    import numpy as np
    import inputs
    from paper_1601_02713_amd import beadscf

    w = inputs.workload(args.workload)
    xs = [x for _, x in w["instances"]]
    eng = beadscf.Engine(0)
    eng.load_basis(inputs.load_basis(w["basis"]))
    eng.set_instances([z for z, _ in w["instances"]])
    prec = beadscf.BSCF_MIXED if args.precision == "mixed" else beadscf.BSCF_FP64
    opts = beadscf.default_opts(e_tol=w["e_tol"], comm_tol=w["comm_tol"], schwarz_tol=1e-12,
                                precision=prec, guess=beadscf.GUESS_CORE, max_iter=60,
                                fp32_split_tol=args.split, graph=args.graph)

    def step():
        eng.set_geometries(xs)
        E, it, st = eng.run_scf(opts)
        return E, it, eng.forces()

    for k in range(args.warmup):
        step()
        log(f"warm-up step {k} done")
    eng.reset_stats()
    eng.set_profiling(True)
    iters = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        E, it, F = step()
        iters += int(np.sum(it))
        log(f"timed step {k} done")
    wall = time.perf_counter() - t0
    eng.set_profiling(False)
    st = eng.stats()
    fs = fock_summary(st, prec == beadscf.BSCF_MIXED, w["label"])
    n = len(xs)
    out = {
        "metric": "screened shell-quartets/s and bead SCF-steps/s vs plain FP64 GPU at 1e-6 Eh",
        "value": fs["screened_quartets_per_s"], "unit": "screened shell-quartets/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == beadscf.BSCF_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w["label"], "mode": "setup + SCF + forces of a fixed batch",
                   "instances": n, "basis_functions": eng.nbf[0], "precision": args.precision,
                   "scf_e_tol": w["e_tol"], "scf_comm_tol": w["comm_tol"], "schwarz_tol": 1e-12,
                   "guess": "core", "graph": args.graph},
        "bead_scf_steps_per_s": iters / wall,
        "bead_energy_force_per_s": n * args.steps / wall,
        "scf_iterations_per_bead": iters / (n * args.steps),
        "fock": {k: v for k, v in fs.items() if k != "roofline"},
        "roofline": fs["roofline"],
        "phase_ms_per_step": {k: st[k] / args.steps for k in
                              ("t_setup_ms", "t_scf_ms", "t_grad_ms", "t_fock_ms", "t_work_ms")},
        "density": {"projection_steps_per_call": st["sp2_steps"] / max(st["sp2_calls"], 1),
                    "fallbacks": st["sp2_fallbacks"]},
    }
    eng.close()
    if args.per_instance > 0:
        out["per_instance"] = per_instance_study(w, args.per_instance, opts)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["md", "scf", "string", "b3lyp"], default="md")
    ap.add_argument("--images", type=int, default=120, help="string mode: images of the path")
    ap.add_argument("--workload", default=None,
                    help="md: w8_beads, w16_beads, w32_beads (default); scf: any named workload")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="timed path precision (md default mixed, scf default fp64)")
    ap.add_argument("--guess", choices=["learned", "previous", "extrapolated"], default="learned")
    ap.add_argument("--split", type=float, default=1e-4,
                    help="mixed precision: quartets with Q_ab Q_cd below this run in FP32")
    ap.add_argument("--dt-fs", type=float, default=0.25)
    ap.add_argument("--temperature", type=float, default=300.0)
    ap.add_argument("--train-steps", type=int, default=5)
    ap.add_argument("--predict-from", type=int, default=3)
    ap.add_argument("--baseline-steps", type=int, default=0,
                    help="timed steps of the plain FP64 leg (default: as many as the timed path)")
    ap.add_argument("--graph", type=int, choices=[0, 1, 2], default=1)
    ap.add_argument("--per-instance", type=int, default=0, metavar="N")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout is a design note and is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    if args.mode == "md":
        args.workload = args.workload or "w32_beads"
        args.precision = args.precision or "mixed"
        if args.warmup < 1:
            sys.exit("md mode needs at least one warm-up step (step 0 is the starting point)")
        md_bench(args)
    elif args.mode == "b3lyp":
        args.workload = args.workload or "w8_beads"
        b3lyp_bench(args)
    elif args.mode == "string":
        args.precision = args.precision or "fp64"
        string_bench(args)
    else:
        args.workload = args.workload or "w8_beads"
        args.precision = args.precision or "fp64"
        scf_bench(args)


if __name__ == "__main__":
    main()
