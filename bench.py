"""Benchmark: atom-steps/s of the all-GPU polyethylene MD step on one MI355X.

Default workload: 1,000 chains x 300 united atoms (300,000 atoms), 0.80 g/cm^3, Maxwell
velocities at 500 K, Berendsen quench towards 300 K, dt = 1 fs, bins rebuilt every step,
mixed precision (FP32 forces, FP64 state), hipGraph-replayed steps.  The grown melt is first
relaxed by --relax-steps steps of the same form (its forced close contacts resolve within a few
tens of steps); every form is timed from the relaxed state.  Beside it, in the same JSON line:
  - the plain FP64 GPU form on the same input and steps (FP64 everywhere, no graph, its own
    autotuned grid and kernel), and the same FP64 form graph-replayed;
  - the force error of the mixed form against the FP64 oracle (at the grown melt and at the end
    of the timed run), norm-wise over the oracle's RMS force;
  - per-phase kernel times and the roofline position of the Lennard-Jones kernel;
  - the batched workload (64 boxes, about 4.3M atoms) in four forms and the 30M-atom melt,
    short runs of each;
  - the FP64 CPU oracle timed on a bounded sample of the workload;
  - from the end state of the timed run: Verlet neighbour lists (skin 1 A, rebuilt when an atom
    has moved more than half the skin), the paper's leap-frog + Nose-Hoover integrator with the
    centre-of-mass velocity removed every step, the Newton-3 half shell, and one Section 5
    observables call.

``--workload`` selects one of the other presets instead (their own JSON line, same keys):
melt3M_mixed (NVT throughput, then the NVE energy drift over 1,000 steps), ensemble64_mixed
(64 boxes in one launch sequence, the smallest box checked against the oracle) or
melt30M_mixed (throughput and per-kernel algorithmic HBM rates at 30M atoms).

Prints ONE JSON line.  Inputs are synthetic (seeded melts); see pe_melt.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "atom-steps/s (and ns/day) mixed/batched vs plain FP64 GPU at <=1e-5 force err"
PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector (vendor figure)
LJ_FLOP_PER_CANDIDATE = 8     # 3 sub, 1 mul + 2 fma (=4) for r^2, 1 compare
LJ_FLOP_PER_PAIR = 13         # rcp, r^-6 (2 mul), force factor (fma + 2 mul), 3 fma accumulations


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def candidate_and_pair_counts(pos, box, start, M, R, rc, n_chains, chain_len):
    """Candidates the stencil walk tests (sum over atoms of the atoms in the (2R+1)^3 cells
    around its cell) and in-cutoff ordered pairs (excluding self and 1-2/1-3 chain pairs)."""
    import numpy as np
    from scipy.spatial import cKDTree
    cnt = np.diff(start).reshape(M[2], M[1], M[0]).astype(np.int64)
    neigh = np.zeros_like(cnt)
    for oz in range(-R, R + 1):
        for oy in range(-R, R + 1):
            for ox in range(-R, R + 1):
                neigh += np.roll(cnt, shift=(oz, oy, ox), axis=(0, 1, 2))
    candidates = int((cnt * neigh).sum())
    p = np.mod(pos.T, box)
    p = np.minimum(p, np.nextafter(box, 0))
    tree = cKDTree(p, boxsize=box)
    n_le = int(tree.count_neighbors(tree, rc * (1 - 1e-12)))
    excluded = n_chains * 2 * ((chain_len - 1) + (chain_len - 2))
    pairs = n_le - pos.shape[1] - excluded
    return candidates, pairs


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "lj_tile_mixed_melt300k_traffic.json")
LJ_SOURCE = os.path.join(ROOT, "paper_1001_3764_amd", "csrc", "md_lj.hip")


def lj_source_hash():
    """SHA-256 of the LJ kernels' source with comments and blank lines left out, so that the
    counter record follows the code, not its commentary."""
    import hashlib
    import re
    with open(LJ_SOURCE) as fh:
        text = fh.read()
    lines = [re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines()]
    code = "\n".join(line for line in lines if line.strip())
    return hashlib.sha256(code.encode()).hexdigest()


def counter_record(kernel_name):
    """The committed rocprofv3 counter record of the LJ kernel (HBM bytes per launch, FP32 VALU
    flops per launch), if it was taken on the current LJ source and the same kernel; else {}."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return {}
    if rec.get("source_sha256") != lj_source_hash() or rec.get("kernel") != kernel_name:
        return {}
    return rec


def cpu_model():
    """The host CPU's model name and logical CPU count (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            names = [l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")]
        return {"model": names[0] if names else "unknown", "logical_cpus": len(names) or os.cpu_count()}
    except OSError:
        return {"model": "unknown", "logical_cpus": os.cpu_count()}


def canonical_candidates(n_atoms, box, rc):
    """Candidates per atom of the paper's grid search (Section 3.2): the 27 cells of edge
    L / floor(L / rc) around the atom's cell, at the box's mean density."""
    import numpy as np
    box = np.asarray(box, dtype=float)
    M = np.floor(box / rc)
    return 27.0 * float(np.prod(box / M)) * n_atoms / float(np.prod(box))


def cpu_baseline(ff, melt, budget_s=12.0, max_steps=100, threads=None):
    import numpy as np
    import oracle as O
    threads = O.set_threads(threads or int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    f0, _ = O.forces(ff, melt.pos, melt.types, melt.box, melt.chain_len)
    p, v, f = melt.pos, melt.vel, f0
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps:
        p, v, f, _ = O.run(ff, p, v, f, melt.types, melt.box, melt.chain_len, 1, T0=300.0)
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    cpu = cpu_model()
    return {"value": melt.n_atoms * steps / dt, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
            "sample": "%d step(s) of the same %d-atom melt (FP64 C oracle, OpenMP over atoms), %.1f s"
                      % (steps, melt.n_atoms, dt),
            "cpu_model": cpu["model"], "host_logical_cpus": cpu["logical_cpus"]}


def lj_roofline(N, box, rc, cand_stencil, pairs, lj_ms, kern, R, homes):
    """Roofline position of the LJ kernel.  Algorithmic work per atom (the flop count of the
    paper's grid search): 8 flop for each of the C = 27 (L/M)^3 n candidates of the 27 cells of
    edge L/M >= rc (M = floor(L/rc)) and 13 flop for each pair inside the cutoff; one launch
    processes the N atoms.  `frac` is that over the event-timed launch and the FP32 vector peak.
    Beside it: the same count over the candidates of the stencil the kernel walks (an effective
    rate: the kernel's filter skips about half of them), and, from the committed counter record
    when it was taken on the current source, the measured HBM bytes and FP32 VALU flops."""
    cand_canon = canonical_candidates(N, box, rc) * N
    flop = LJ_FLOP_PER_CANDIDATE * cand_canon + LJ_FLOP_PER_PAIR * pairs
    flop_stencil = LJ_FLOP_PER_CANDIDATE * cand_stencil + LJ_FLOP_PER_PAIR * pairs
    achieved = flop / (lj_ms * 1e-3) / 1e12
    kname = "k_lj_tile" if kern in (2, 3) else "k_lj_atom"
    rec = counter_record("%s/R%d/K%d/H%d" % (kname, R, kern, homes))
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
           "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": rec.get("bytes_per_launch"),
           "kernel": "%s (Lennard-Jones, mixed, R=%d, lj_kernel %d, %d atoms per wavefront)" % (kname, R, kern, homes),
           "avg_launch_ms": round(lj_ms, 5),
           "flop_per_launch": flop, "candidates_per_atom_canonical": round(cand_canon / N, 2),
           "pairs_per_launch": pairs,
           "flop_basis": "per atom: 8 flop x 27 (L/M)^3 n candidates of the 27-cell grid of edge L/M >= rc "
                         "+ 13 flop x the pairs inside the cutoff; x N atoms per launch",
           "frac_of_unpacked_fp32_78_6": round(achieved / 78.6, 4),
           "stencil_candidates_per_launch": cand_stencil,
           "frac_stencil_effective": round(flop_stencil / (lj_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)}
    if rec.get("valu_fp32_flops_per_launch"):
        cf = rec["valu_fp32_flops_per_launch"]
        out["counter_fp32_tflops"] = round(cf / (lj_ms * 1e-3) / 1e12, 3)
        out["counter_over_algorithmic"] = round(cf / flop, 4)
        out["counter_basis"] = "64 x SQ_INSTS_VALU_FLOPS_FP32 per launch (FMA = 2) from %s" % \
            os.path.relpath(TRAFFIC_RECORD, ROOT)
    if rec.get("bytes_per_launch"):
        out["traffic_over_algorithmic"] = round(rec["bytes_per_launch"] / rec["algorithmic_bytes_per_launch"], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--fp64-steps", type=int, default=200, help="FP64 steps of the other workloads")
    ap.add_argument("--relax-steps", type=int, default=500,
                    help="steps of the mixed form that relax each grown melt before anything is timed")
    ap.add_argument("--cell-div", type=int, default=0, help="0 = autotune")
    ap.add_argument("--lj-kernel", type=int, default=0, help="0 = autotune")
    ap.add_argument("--tile-homes", type=int, default=0, help="cell-tile atoms per wavefront (0 = autotune)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-nlist", action="store_true", help="skip the neighbour-list form")
    ap.add_argument("--no-leapfrog", action="store_true", help="skip the leap-frog + Nose-Hoover form")
    ap.add_argument("--no-halfshell", action="store_true", help="skip the Newton-3 half-shell LJ form")
    ap.add_argument("--no-observables", action="store_true", help="skip the Section 5 observables")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 64-box batched sub-result")
    ap.add_argument("--no-30m", action="store_true", help="skip the 30M-atom sub-result")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first copy a device buffer of this many MiB (HBM counter calibration)")
    ap.add_argument("--workload", default="melt300k_mixed",
                    choices=["melt300k_mixed", "melt3M_mixed", "ensemble64_mixed", "melt30M_mixed"])
    ap.add_argument("--nve-steps", type=int, default=1000, help="melt3M_mixed: NVE drift window")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (one process, no collectives); --gpus %d is not supported"
              % args.gpus, flush=True)
        sys.exit(2)
    if args.workload != "melt300k_mixed":
        return run_other_workload(args)

    import numpy as np
    import torch

    from paper_1001_3764_amd.md import MDSystem
    from pe_melt import WORKLOADS, make_melt, polyethylene_forcefield

    wl = WORKLOADS["melt300k_mixed"]
    ff = polyethylene_forcefield()
    t = time.perf_counter()
    melt = make_melt(wl.n_chains[0], density=wl.density, T=wl.T_init[0], seed_melt=wl.seeds[0][0],
                     seed_vel=wl.seeds[0][1])
    log("melt: %d atoms, L=%.3f A (%.1fs)" % (melt.n_atoms, melt.box[0], time.perf_counter() - t))
    N = melt.n_atoms
    dev = torch.device("cuda:0")
    if args.calib_copy_mb > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the HBM counters
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize(dev)
        del src, dst

    def mixed_system(pos, vel):
        return MDSystem(ff, [melt.n_chains], melt.box[None, :], [wl.T0[0]], pos, vel, melt.types,
                        chain_len=wl.chain_len, dt=wl.dt_fs, tau=wl.tau_fs, precision="mixed",
                        cell_div=args.cell_div, lj_kernel=args.lj_kernel, use_graph=not args.no_graph, device=dev,
                        tile_homes=args.tile_homes)

    # ---- the input: the grown melt (its forces checked against the oracle below), relaxed by
    # relax_steps steps of the mixed form toward T0; every timed form starts from that state ----
    s = mixed_system(melt.pos, melt.vel)
    f_mixed = s.forces()
    f_mixed_lj = s.forces(lj_only=True)
    p_start, v_start, grown = relax_input(s, args.relax_steps, N, dev)
    s.close()

    # ---- mixed precision, graph-replayed: the headline ----
    s = mixed_system(p_start, v_start)
    R, kern, homes = s.tuning(homes=True)
    log("mixed: cell_div R=%d, lj kernel %d, %d atoms per wavefront" % (R, kern, homes))
    M, _, _ = s.grid(0)
    s.step(args.warmup)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    e_end = s.energies()[0]
    wall = t1 - t0
    value = N * args.steps / wall
    ms_per_step = 1e3 * wall / args.steps
    log("mixed: %.3f ms/step, %.3e atom-steps/s, T=%.1f K" % (ms_per_step, value, e_end["temperature"]))

    # per-phase kernel durations, HIP events on the library's stream
    n_prof = min(args.steps, 500)
    phases = s.step_timed(n_prof)
    phase_avg = {k: v / n_prof for k, v in phases.items()}
    start_prof, _ = s.bins()
    pos_prof, vel_prof = s.state()
    f_end = s.forces()
    f_end_lj = s.forces(lj_only=True)

    # Section 5 observables of the end-of-run state (pair-distance histogram, dihedral
    # statistics, chain shape), one md_observables call including the copies to the host
    observables = None
    if not args.no_observables:
        try:
            s.observables(rdf_bins=210, rdf_rmax=10.5, dih_bins=72)
            reps = 5
            a = time.perf_counter()
            for _ in range(reps):
                o = s.observables(rdf_bins=210, rdf_rmax=10.5, dih_bins=72)
            b_ = time.perf_counter()
            cls = o["dihedral_classes"][0].astype(float)
            observables = {"ms_per_call": 1e3 * (b_ - a) / reps, "rdf_bins": 210, "rdf_rmax_A": 10.5,
                           "dih_bins": 72, "pairs_counted": int(o["pair_counts"][0].sum()),
                           "trans_fraction": float(cls[0] / cls.sum()),
                           "mean_rg2_A2": float(o["chain_shape"][:, 0].mean()),
                           "mean_ree2_A2": float((o["chain_shape"][:, 1:] ** 2).sum(axis=1).mean())}
            log("observables: %.3f ms per call, trans fraction %.4f, <Rg^2> %.1f A^2"
                % (observables["ms_per_call"], observables["trans_fraction"], observables["mean_rg2_A2"]))
        except Exception as exc:
            log("observables failed: %r" % (exc,))
    s.close()

    # ---- the paper's force path beside it: Verlet lists (skin 1 A) rebuilt when an atom has
    # moved more than half the skin, from the state the timed run ended in (mixed, graph-replayed) ----
    nlist = None
    if not args.no_nlist:
        try:
            sn = MDSystem(ff, [melt.n_chains], melt.box[None, :], [wl.T0[0]], pos_prof, vel_prof, melt.types,
                          chain_len=wl.chain_len, dt=wl.dt_fs, tau=wl.tau_fs, precision="mixed", cell_div=0,
                          use_graph=not args.no_graph, device=dev, nl_skin=1.0, nl_every=0)
            Rn, sn_kern = sn.tuning()
            fn_lj = sn.forces(lj_only=True)
            sn.step(50)
            torch.cuda.synchronize(dev)
            a = time.perf_counter()
            n_nl = min(args.steps, 2000)
            sn.step(n_nl)
            torch.cuda.synchronize(dev)
            b_ = time.perf_counter()
            # the device error word: a run the library flagged reports no rate
            status = "ok"
            try:
                sn.energies()
            except Exception as exc:
                status = str(exc)
            ph = {k: v / 100 for k, v in sn.step_timed(100).items()} if status == "ok" else None
            builds = sn.list_builds() if status == "ok" else None
            sn.close()
            ok = status == "ok"
            nlist = {"value": N * n_nl / (b_ - a) if ok else None, "unit": "atom-steps/s", "steps": n_nl,
                     "ms_per_step": 1e3 * (b_ - a) / n_nl if ok else None, "skin_A": 1.0,
                     "rebuild": "when an atom has moved more than half the skin since the last build",
                     "list_builds": builds, "cell_div": Rn,
                     "phases_ms_avg": {k: round(v, 5) for k, v in ph.items()} if ph else None, "status": status,
                     "lj_kernel": sn_kern,
                     # the list path's LJ force against the cell path's at the same positions,
                     # over the RMS of the total force (reading of the 1e-5 criterion) and of the
                     # LJ force alone
                     "lj_force_max_diff_vs_cell_path_over_frms": float(
                         np.max(np.sqrt(np.sum((fn_lj - f_end_lj) ** 2, axis=0)))
                         / np.sqrt(np.mean(np.sum(f_end ** 2, axis=0)))),
                     "lj_force_max_diff_vs_cell_path_over_lj_frms": float(
                         np.max(np.sqrt(np.sum((fn_lj - f_end_lj) ** 2, axis=0)))
                         / np.sqrt(np.mean(np.sum(f_end_lj ** 2, axis=0))))}
            log("nlist: %.3f ms/step, %.3e atom-steps/s (%s)" % (nlist["ms_per_step"], nlist["value"], status))
        except Exception as exc:
            log("nlist run failed: %r" % (exc,))

    # ---- the paper's integrator: leap-frog + Nose-Hoover (300 K, tau_T 100 fs) with the COM
    # velocity removed every step, same grid and kernel as the headline, from its end state ----
    leapfrog = None
    if not args.no_leapfrog:
        try:
            sl = MDSystem(ff, [melt.n_chains], melt.box[None, :], [wl.T0[0]], pos_prof, vel_prof, melt.types,
                          chain_len=wl.chain_len, dt=wl.dt_fs, tau=100.0, precision="mixed", cell_div=R,
                          lj_kernel=kern, use_graph=not args.no_graph, device=dev, integrator="leapfrog",
                          remove_com=True)
            sl.step(50)
            torch.cuda.synchronize(dev)
            a = time.perf_counter()
            n_lf = min(args.steps, 2000)
            sl.step(n_lf)
            torch.cuda.synchronize(dev)
            b_ = time.perf_counter()
            ph = {k: v / 100 for k, v in sl.step_timed(100).items()}
            e_lf = sl.energies()[0]
            sl.close()
            leapfrog = {"value": N * n_lf / (b_ - a), "unit": "atom-steps/s", "steps": n_lf,
                        "ms_per_step": 1e3 * (b_ - a) / n_lf, "thermostat": "nose-hoover", "tau_T_fs": 100.0,
                        "remove_com": True, "T_K": e_lf["temperature"], "xi_per_fs": e_lf["nh_xi"],
                        "phases_ms_avg": {k: round(v, 5) for k, v in ph.items()}}
            log("leapfrog+NH: %.3f ms/step, %.3e atom-steps/s" % (leapfrog["ms_per_step"], leapfrog["value"]))
        except Exception as exc:
            log("leapfrog run failed: %r" % (exc,))

    # ---- Newton-3 half shell (opt-in kernel): each pair once, both forces added to int64
    # fixed-point accumulators with device atomics; same grid, from the end-of-run state ----
    halfshell = None
    if not args.no_halfshell:
        try:
            from paper_1001_3764_amd.md import MD_LJ_HALFSHELL
            sh = MDSystem(ff, [melt.n_chains], melt.box[None, :], [wl.T0[0]], pos_prof, vel_prof, melt.types,
                          chain_len=wl.chain_len, dt=wl.dt_fs, tau=wl.tau_fs, precision="mixed", cell_div=R,
                          lj_kernel=MD_LJ_HALFSHELL, use_graph=not args.no_graph, device=dev)
            fh_lj = sh.forces(lj_only=True)
            sh.step(20)
            torch.cuda.synchronize(dev)
            a = time.perf_counter()
            n_hs = min(args.steps, 1000)
            sh.step(n_hs)
            torch.cuda.synchronize(dev)
            b_ = time.perf_counter()
            ph = {k: v / 50 for k, v in sh.step_timed(50).items()}
            sh.close()
            halfshell = {"value": N * n_hs / (b_ - a), "unit": "atom-steps/s", "steps": n_hs,
                         "ms_per_step": 1e3 * (b_ - a) / n_hs, "lj_kernel": MD_LJ_HALFSHELL, "cell_div": R,
                         "phases_ms_avg": {k: round(v, 5) for k, v in ph.items()},
                         "lj_force_max_diff_vs_cell_path_over_frms": float(
                             np.max(np.sqrt(np.sum((fh_lj - f_end_lj) ** 2, axis=0)))
                             / np.sqrt(np.mean(np.sum(f_end ** 2, axis=0))))}
            log("half shell: %.3f ms/step, %.3e atom-steps/s (LJ %.3f ms)" %
                (halfshell["ms_per_step"], halfshell["value"], ph["lj"]))
        except Exception as exc:
            log("half-shell run failed: %r" % (exc,))

    cand, pairs = candidate_and_pair_counts(pos_prof, melt.box, start_prof, M, R, ff["rc"], melt.n_chains,
                                            melt.chain_len)
    roofline = lj_roofline(N, melt.box, ff["rc"], cand, pairs, phase_avg["lj"], kern, R, homes)

    # ---- force error of the mixed form against the FP64 oracle, at the grown melt and at the
    # state the timed run ended in (same positions on both sides) ----
    force_err = {}
    try:
        import oracle as O
        O.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
        for label, pos, f_gpu, f_gpu_lj in (("initial_melt", melt.pos, f_mixed, f_mixed_lj),
                                            ("end_of_run", pos_prof, f_end, f_end_lj)):
            fo_lj, _ = O.lj_cells(ff, pos, melt.types, melt.box, melt.chain_len)
            fo_b, _ = O.bonded(ff, pos, melt.box, melt.chain_len)
            fo = fo_lj + fo_b
            frms = np.sqrt(np.mean(np.sum(fo ** 2, axis=0)))
            dnorm = np.sqrt(np.sum((f_gpu - fo) ** 2, axis=0))
            d_lj = np.sqrt(np.sum((f_gpu_lj - fo_lj) ** 2, axis=0))
            d_b = np.sqrt(np.sum((f_gpu - f_gpu_lj - fo_b) ** 2, axis=0))
            fnorm = np.sqrt(np.sum(fo ** 2, axis=0))
            # per-atom relative error, each atom against its own force with F_rms as the floor
            force_err[label] = {"max_rel": float((dnorm / np.maximum(fnorm, frms)).max()),
                                "max_over_frms": float(dnorm.max() / frms),
                                "rms_rel": float(np.sqrt(np.sum(dnorm ** 2) / np.sum(fo ** 2))),
                                "lj_max_over_frms": float(d_lj.max() / frms),
                                "bonded_max_over_frms": float(d_b.max() / frms),
                                "frms": float(frms),
                                "max_abs_force_over_frms": float(fnorm.max() / frms)}
            log("mixed force error vs oracle (%s): %s" % (label, force_err[label]))
    except Exception as exc:   # the metric line is still printed
        log("force error check failed: %r" % (exc,))

    # ---- plain FP64 GPU form (FP64 everywhere, no graph, its own autotuned grid and kernel): the
    # same warm-up and timed steps from the same relaxed melt; and the same FP64 form graph-replayed,
    # to separate the effect of precision from that of the saved launches ----
    plain = plain_graph = None
    if not args.no_fp64:
        for graph in (False, True):
            s64 = MDSystem(ff, [melt.n_chains], melt.box[None, :], [wl.T0[0]], p_start, v_start, melt.types,
                           chain_len=wl.chain_len, dt=wl.dt_fs, tau=wl.tau_fs, precision="fp64", cell_div=0,
                           lj_kernel=0, use_graph=graph, device=dev)
            R64, k64 = s64.tuning()
            s64.step(args.warmup)
            torch.cuda.synchronize(dev)
            a = time.perf_counter()
            s64.step(args.steps)
            torch.cuda.synchronize(dev)
            b = time.perf_counter()
            s64.close()
            v64 = N * args.steps / (b - a)
            rec = {"value": v64, "unit": "atom-steps/s", "steps": args.steps, "warmup": args.warmup,
                   "ms_per_step": 1e3 * (b - a) / args.steps, "cell_div": R64, "lj_kernel": k64, "graph": graph}
            if graph:
                plain_graph = rec
            else:
                plain = rec
            log("fp64 (%s): %.3f ms/step, %.3e atom-steps/s" % ("graph" if graph else "no graph", rec["ms_per_step"], v64))

    # ---- the batched and the largest workloads, short runs in the same process ----
    sub_steps, sub_warm = min(args.steps, 100), min(args.warmup, 10)
    ensemble = large = None
    if not args.no_ensemble:
        try:
            ensemble = sub_ensemble(args, ff, dev, sub_steps, sub_warm)
        except Exception as exc:
            log("ensemble64 run failed: %r" % (exc,))
    if not args.no_30m:
        try:
            large = sub_melt30M(args, ff, dev, sub_steps, sub_warm)
        except Exception as exc:
            log("melt30M run failed: %r" % (exc,))

    cpu = cpu1 = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(ff, melt)
            log("cpu oracle: %.3e atom-steps/s on %d threads" % (cpu["value"], cpu["cores"]))
            # one core: the kind of baseline the paper compares against (single-core CPU MD)
            cpu1 = cpu_baseline(ff, melt, budget_s=4.0, max_steps=1, threads=1)
            log("cpu oracle, 1 thread: %.3e atom-steps/s" % cpu1["value"])
        except Exception as exc:
            log("cpu baseline failed: %r" % (exc,))

    out = {
        "metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": wl.name, "atoms": N, "chains": melt.n_chains, "chain_len": melt.chain_len,
                   "density_g_cm3": wl.density, "box_A": round(float(melt.box[0]), 4),
                   "T_init_K": wl.T_init[0], "T0_K": wl.T0[0], "thermostat": "berendsen",
                   "tau_fs": wl.tau_fs, "dt_fs": wl.dt_fs, "precision": "mixed (FP32 force, FP64 state)",
                   "cell_div": R, "cells_per_dim": [int(x) for x in M], "lj_kernel": kern, "tile_homes": homes,
                   "graph": not args.no_graph, "bins_rebuilt_every_step": True,
                   "relax_steps": args.relax_steps},
        "grown_melt_first_steps": grown,
        "ns_per_day": (1e3 / ms_per_step) * wl.dt_fs * 86400 * 1e-6,
        "force_err_vs_fp64_oracle": force_err,
        "plain_fp64_gpu": plain,
        "speedup_vs_plain_fp64": (value / plain["value"]) if plain else None,
        "fp64_gpu_graph": plain_graph,
        "speedup_vs_fp64_graph": (value / plain_graph["value"]) if plain_graph else None,
        "phases_ms_avg": {k: round(v, 5) for k, v in phase_avg.items()},
        # the HBM-bound per-atom kernels: algorithmic bytes per atom x atoms / event-timed phase
        "per_atom_kernels_hbm": {k: {"GBps": round(ALGO_BYTES_PER_ATOM[k] * N / (phase_avg[k] * 1e-3) / 1e9, 1),
                                     "frac_of_8TBps": round(ALGO_BYTES_PER_ATOM[k] * N / (phase_avg[k] * 1e-3) / 8e12, 4),
                                     "bytes_per_atom": ALGO_BYTES_PER_ATOM[k]} for k in ALGO_BYTES_PER_ATOM},
        "final_temperature_K": e_end["temperature"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_1thread": cpu1,
        "nlist_form": nlist,
        "leapfrog_nh_form": leapfrog,
        "halfshell_form": halfshell,
        "observables": observables,
        "ensemble64_mixed": ensemble,
        "melt30M_mixed": large,
    }
    print(json.dumps(out), flush=True)


# Algorithmic HBM bytes per atom of the per-atom phases (mixed form; see the kernel table of
# the design notes): integrate+bin, scatter, rank+payload, bonded+kick.
ALGO_BYTES_PER_ATOM = {"integrate_bin": 117, "scatter": 16, "rank_payload": 61, "bonded_kick": 97}


def _concat(melts):
    import numpy as np
    return (np.concatenate([m.pos for m in melts], axis=1), np.concatenate([m.vel for m in melts], axis=1),
            np.concatenate([m.types for m in melts]), np.stack([m.box for m in melts]),
            [m.n_chains for m in melts])


def relax_input(s, steps, n_atoms, dev):
    """Relaxes a grown melt: `steps` steps of system s (the grown configuration has close
    contacts that the first few hundred femtoseconds push apart, and it starts above T0).
    Returns the relaxed positions and velocities and the rate of those first steps (None for
    steps = 0)."""
    import torch
    if steps <= 0:
        p, v = s.state()
        return p, v, None
    torch.cuda.synchronize(dev)
    a = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - a
    p, v = s.state()
    log("relaxed the grown melt: %d steps, %.3f ms/step" % (steps, 1e3 * wall / steps))
    return p, v, {"steps": steps, "ms_per_step": 1e3 * wall / steps, "value": n_atoms * steps / wall,
                  "unit": "atom-steps/s"}


def _timed(s, warmup, steps, dev):
    import torch
    s.step(warmup)
    torch.cuda.synchronize(dev)
    a = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize(dev)
    return time.perf_counter() - a


def sampled_force_error(ff, melt, f_gpu, n_sample, seed):
    """Norm-wise force error max_i |F_gpu,i - F_ora,i| / F_rms on n_sample uniformly drawn atoms:
    the oracle's LJ force of those atoms (subset of its grid search over the whole system) and
    the bonded force of their whole chains; F_rms is estimated from the same sample."""
    import numpy as np
    import oracle as O
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(melt.n_atoms, size=n_sample, replace=False))
    fo_lj, _ = O.lj_cells(ff, melt.pos, melt.types, melt.box, melt.chain_len, subset=sample)
    L = melt.chain_len
    chains = np.unique(sample // L)
    idx = (chains[:, None] * L + np.arange(L)[None, :]).ravel()
    fo_b_sub, _ = O.bonded(ff, melt.pos[:, idx], melt.box, L)
    where = np.searchsorted(idx, sample)
    fo = fo_lj + fo_b_sub[:, where]
    frms = float(np.sqrt(np.mean(np.sum(fo ** 2, axis=0))))
    d = np.sqrt(np.sum((f_gpu[:, sample] - fo) ** 2, axis=0))
    return {"max_over_frms": float(d.max() / frms), "frms_estimate": frms, "atoms_sampled": int(n_sample)}


def tuning_classes(sizes, tunings):
    """The autotuner's choices over boxes of different sizes: for each distinct (cell_div,
    lj_kernel, atoms per wavefront), how many boxes took it and the range of their atom counts."""
    classes = {}
    for n, t in zip(sizes, tunings):
        key = "R%d/K%d/H%d" % tuple(t)
        c = classes.setdefault(key, {"boxes": 0, "atoms_min": n, "atoms_max": n})
        c["boxes"] += 1
        c["atoms_min"] = min(c["atoms_min"], n)
        c["atoms_max"] = max(c["atoms_max"], n)
    return classes


def sub_ensemble(args, ff, dev, steps, warmup):
    """The batched workload (64 boxes of 20..400 chains at 250..450 K, about 4.3M atoms), in the
    four forms that separate precision from batching: mixed batched and graph-replayed (one
    launch sequence for all boxes), FP64 batched, and one context per box in each precision.
    Same warm-up and timed steps for each, from the relaxed melts; the smallest box's forces
    against the oracle at the grown melts."""
    import numpy as np
    import oracle as O
    from paper_1001_3764_amd.md import MDSystem
    from pe_melt import WORKLOADS, build_melts
    wl = WORKLOADS["ensemble64_mixed"]
    t = time.perf_counter()
    melts = build_melts(wl, threads=16)
    pos, vel, types, boxes, chains = _concat(melts)
    N = pos.shape[1]
    log("ensemble64: %d boxes, %d atoms (%.1fs)" % (len(melts), N, time.perf_counter() - t))
    # the smallest box's forces at the grown melts; then the grown melts relaxed (mixed, batched,
    # graph-replayed) and every form timed from the relaxed state
    s = MDSystem(ff, chains, boxes, list(wl.T0), pos, vel, types, chain_len=wl.chain_len, dt=wl.dt_fs,
                 tau=wl.tau_fs, precision="mixed", cell_div=0, lj_kernel=0, use_graph=True, device=dev)
    b = int(np.argmin([m.n_atoms for m in melts]))
    off = sum(x.n_atoms for x in melts[:b])
    m = melts[b]
    f = s.forces()[:, off:off + m.n_atoms]
    pos, vel, grown = relax_input(s, args.relax_steps, N, dev)
    s.close()
    O.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    fo, _ = O.forces(ff, m.pos, m.types, m.box, m.chain_len)
    frms = float(np.sqrt(np.mean(np.sum(fo ** 2, axis=0))))
    smallest = {"box": b, "atoms": m.n_atoms,
                "force_max_err_over_frms": float(np.max(np.sqrt(np.sum((f - fo) ** 2, axis=0))) / frms)}
    forms = {}
    R = kern = None
    for precision, graph in (("mixed", True), ("fp64", False)):
        s = MDSystem(ff, chains, boxes, list(wl.T0), pos, vel, types, chain_len=wl.chain_len, dt=wl.dt_fs,
                     tau=wl.tau_fs, precision=precision, cell_div=0, lj_kernel=0, use_graph=graph, device=dev)
        if precision == "mixed":
            R, kern = s.tuning()
        tuning = list(s.tuning())
        wall = _timed(s, warmup, steps, dev)
        s.close()
        forms["%s_batched%s" % (precision, "_graph" if graph else "")] = {
            "value": N * steps / wall, "ms_per_step": 1e3 * wall / steps, "tuning": tuning}
    # one context per box, each autotuned for its own box (cell size, kernel, atoms per wavefront)
    per_box_tuning = None
    for precision, graph in (("mixed", True), ("fp64", False)):
        ctxs = []
        off = 0
        for b, m in enumerate(melts):
            sl = slice(off, off + m.n_atoms)
            ctxs.append(MDSystem(ff, [m.n_chains], m.box[None, :], [wl.T0[b]], pos[:, sl], vel[:, sl], types[sl],
                                 chain_len=wl.chain_len, dt=wl.dt_fs, tau=wl.tau_fs, precision=precision,
                                 cell_div=0, lj_kernel=0, use_graph=graph, device=dev))
            off += m.n_atoms
        if precision == "mixed":
            per_box_tuning = tuning_classes([m.n_atoms for m in melts], [c.tuning(homes=True) for c in ctxs])
        for c in ctxs:
            c.step(warmup)
        import torch
        torch.cuda.synchronize(dev)
        a = time.perf_counter()
        for c in ctxs:
            c.step(steps)
        torch.cuda.synchronize(dev)
        wall = time.perf_counter() - a
        for c in ctxs:
            c.close()
        forms["%s_per_box%s" % (precision, "_graph" if graph else "")] = {
            "value": N * steps / wall, "ms_per_step": 1e3 * wall / steps}
    for k, v in forms.items():
        log("ensemble64 %s: %.3e atom-steps/s" % (k, v["value"]))
    mb = forms["mixed_batched_graph"]["value"]
    return {"workload": wl.name, "boxes": len(melts), "atoms": N, "steps": steps, "warmup": warmup,
            "relax_steps": args.relax_steps, "grown_melts_first_steps": grown,
            "value": mb, "unit": "atom-steps/s", "forms": forms,
            "mixed_batched_over_fp64_per_box": mb / forms["fp64_per_box"]["value"],
            "mixed_batched_over_fp64_batched": mb / forms["fp64_batched"]["value"],
            "mixed_batched_over_mixed_per_box": mb / forms["mixed_per_box_graph"]["value"],
            "per_box_tuning": per_box_tuning,
            "smallest_box_vs_oracle": smallest, "fits_in_default_run": True}


def sub_melt30M(args, ff, dev, steps, warmup):
    """The largest single-box workload (30,000,000 atoms, 0.85 g/cm^3, 300 K): mixed
    (graph-replayed) and plain FP64 rates over the same steps from the relaxed melt, the mixed
    form's sampled force error against the oracle at the grown melt, and each phase's algorithmic
    HBM rate from HIP-event timings."""
    from paper_1001_3764_amd.md import MDSystem
    from pe_melt import WORKLOADS, build_melts
    wl = WORKLOADS["melt30M_mixed"]
    t = time.perf_counter()
    melt = build_melts(wl, threads=16)[0]
    N = melt.n_atoms
    log("melt30M: %d atoms (%.1fs)" % (N, time.perf_counter() - t))
    out = {"workload": wl.name, "atoms": N, "steps": steps, "warmup": warmup, "relax_steps": args.relax_steps,
           "unit": "atom-steps/s", "fits_in_default_run": True}

    def system(precision, pos, vel, graph):
        return MDSystem(ff, [melt.n_chains], melt.box[None, :], [wl.T0[0]], pos, vel, melt.types,
                        chain_len=wl.chain_len, dt=wl.dt_fs, tau=wl.tau_fs, precision=precision, cell_div=0,
                        lj_kernel=0, use_graph=graph, device=dev)

    # forces at the grown melt, then the melt relaxed; the timed forms start from the relaxed state
    s = system("mixed", melt.pos, melt.vel, True)
    f_grown = s.forces()
    pos, vel, out["grown_melt_first_steps"] = relax_input(s, args.relax_steps, N, dev)
    s.close()
    out["force_err_vs_fp64_oracle"] = sampled_force_error(ff, melt, f_grown, 2000, 30)
    del f_grown
    s = system("mixed", pos, vel, True)
    out["tuning"] = list(s.tuning())
    wall = _timed(s, warmup, steps, dev)
    out["value"] = N * steps / wall
    out["ms_per_step"] = 1e3 * wall / steps
    n_prof = max(2, min(steps, 10))
    ph = {k: v / n_prof for k, v in s.step_timed(n_prof).items()}
    s.close()
    out["phases_ms_avg"] = {k: round(v, 4) for k, v in ph.items()}
    out["algorithmic_hbm_GBps_per_phase"] = {
        k: round(ALGO_BYTES_PER_ATOM[k] * N / (ph[k] * 1e-3) / 1e9, 1) for k in ALGO_BYTES_PER_ATOM}
    s64 = system("fp64", pos, vel, False)
    wall = _timed(s64, warmup, steps, dev)
    out["plain_fp64_gpu"] = {"value": N * steps / wall, "ms_per_step": 1e3 * wall / steps,
                             "tuning": list(s64.tuning()), "graph": False}
    s64.close()
    out["mixed_over_plain_fp64"] = out["value"] / out["plain_fp64_gpu"]["value"]
    log("melt30M: mixed %.3e, fp64 %.3e atom-steps/s, force err %.3e"
        % (out["value"], out["plain_fp64_gpu"]["value"], out["force_err_vs_fp64_oracle"]["max_over_frms"]))
    return out


def run_other_workload(args):
    """The non-default presets: same JSON keys, their own extra fields."""
    import numpy as np
    import torch

    from paper_1001_3764_amd.md import MDSystem
    from pe_melt import WORKLOADS, build_melts, polyethylene_forcefield

    wl = WORKLOADS[args.workload]
    ff = polyethylene_forcefield()
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    melts = build_melts(wl, threads=16)
    N = sum(m.n_atoms for m in melts)
    log("%s: %d box(es), %d atoms (%.1fs)" % (wl.name, len(melts), N, time.perf_counter() - t))
    pos = np.concatenate([m.pos for m in melts], axis=1)
    vel = np.concatenate([m.vel for m in melts], axis=1)
    types = np.concatenate([m.types for m in melts])
    boxes = np.stack([m.box for m in melts])
    chains = [m.n_chains for m in melts]

    def make(precision, T0, p=pos, v=vel, graph=not args.no_graph):
        return MDSystem(ff, chains, boxes, T0, p, v, types, chain_len=wl.chain_len, dt=wl.dt_fs,
                        tau=wl.tau_fs, precision=precision, cell_div=args.cell_div, lj_kernel=args.lj_kernel,
                        use_graph=graph, device=dev)

    steps = args.steps if args.steps != 10000 else wl.steps   # the preset's own length by default
    s = make("mixed", list(wl.T0))
    pos, vel, grown = relax_input(s, args.relax_steps, N, dev)
    s.close()
    s = make("mixed", list(wl.T0), pos, vel)
    R, kern = s.tuning()
    s.step(args.warmup)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    value = N * steps / wall
    ms_per_step = 1e3 * wall / steps
    energies = s.energies()
    log("mixed: R=%d kernel %d, %.3f ms/step, %.3e atom-steps/s" % (R, kern, ms_per_step, value))
    n_prof = min(steps, 200)
    phases = {k: v / n_prof for k, v in s.step_timed(n_prof).items()}
    hbm = {k: round(ALGO_BYTES_PER_ATOM[k] * N / (phases[k] * 1e-3) / 1e9, 1) for k in ALGO_BYTES_PER_ATOM}
    extra = {"phases_ms_avg": {k: round(v, 5) for k, v in phases.items()},
             "algorithmic_hbm_GBps_per_phase": hbm,
             "final_temperature_K": [round(e["temperature"], 3) for e in energies][:8]}

    if wl.name == "melt3M_mixed":
        # NVE energy drift from the NVT end state, mixed and FP64, both graph-replayed
        p_end, v_end = s.state()
        s.close()
        drift = {}
        for precision in ("mixed", "fp64"):
            sn = make(precision, [0.0], p_end, v_end)
            rows = []
            for k in range(args.nve_steps // 100 + 1):
                if k:
                    sn.step(100)
                e = sn.energies()[0]
                rows.append((100 * k, e["e_kin"] + e["e_lj"] + e["e_bond"] + e["e_angle"] + e["e_dih"],
                             e["e_kin"] + e["e_lj_shifted"] + e["e_bond"] + e["e_angle"] + e["e_dih"],
                             e["temperature"]))
            sn.close()
            r = np.array(rows)
            slope = np.polyfit(r[:, 0], r[:, 1], 1)[0]
            slope_s = np.polyfit(r[:, 0], r[:, 2], 1)[0]
            ke0 = 1.5 * N * 1.987204259e-3 * r[0, 3]
            drift[precision] = {
                "steps": args.nve_steps, "E_total_start_kcal_mol": r[0, 1], "E_total_end_kcal_mol": r[-1, 1],
                "drift_kcal_mol_per_atom_per_ns": slope / N * 1e6 / wl.dt_fs,
                "drift_shifted_kcal_mol_per_atom_per_ns": slope_s / N * 1e6 / wl.dt_fs,
                "max_abs_dev_over_KE": float(np.max(np.abs(r[:, 1] - r[0, 1])) / ke0),
                "T_K": [round(x, 3) for x in r[:, 3]]}
            log("NVE %s: drift %.3e (shifted %.3e) kcal/mol/atom/ns, max |E - E0| / KE %.2e"
                % (precision, drift[precision]["drift_kcal_mol_per_atom_per_ns"],
                   drift[precision]["drift_shifted_kcal_mol_per_atom_per_ns"], drift[precision]["max_abs_dev_over_KE"]))
        extra["nve_drift"] = drift
    else:
        s.close()

    if wl.name == "ensemble64_mixed":
        # the smallest box against the oracle, in a fresh context (same launch sequence)
        import oracle as O
        O.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
        b = int(np.argmin([m.n_atoms for m in melts]))
        m = melts[b]
        off = sum(x.n_atoms for x in melts[:b])
        sc = make("mixed", list(wl.T0))
        f = sc.forces()[:, off:off + m.n_atoms]
        sc.close()
        fo, _ = O.forces(ff, m.pos, m.types, m.box, m.chain_len)
        frms = np.sqrt(np.mean(np.sum(fo ** 2, axis=0)))
        err = float(np.max(np.sqrt(np.sum((f - fo) ** 2, axis=0))) / frms)
        extra["smallest_box"] = {"box": b, "atoms": m.n_atoms, "force_max_err_over_frms": err}
        log("smallest box %d (%d atoms): force error %.3e" % (b, m.n_atoms, err))

    if wl.name == "ensemble64_mixed":
        # the same 64 boxes one context (one launch sequence) per box, stepped in turn: separates
        # the effect of batching from that of precision
        per_box = {}
        box_steps = 100
        for precision, graph in (("mixed", not args.no_graph), ("fp64", False)):
            ctxs = []
            off = 0
            for m in melts:
                sl = slice(off, off + m.n_atoms)
                ctxs.append(MDSystem(ff, [m.n_chains], m.box[None, :], [wl.T0[len(ctxs)]], pos[:, sl], vel[:, sl],
                                     types[sl], chain_len=wl.chain_len, dt=wl.dt_fs, tau=wl.tau_fs,
                                     precision=precision, cell_div=0, lj_kernel=0, use_graph=graph, device=dev))
                off += m.n_atoms
            for c in ctxs:
                c.step(5)
            torch.cuda.synchronize(dev)
            a = time.perf_counter()
            for c in ctxs:
                c.step(box_steps)
            torch.cuda.synchronize(dev)
            b_ = time.perf_counter()
            tunes = [c.tuning(homes=True) for c in ctxs]
            for c in ctxs:
                c.close()
            per_box["%s_per_box%s" % (precision, "_graph" if graph else "")] = {
                "value": N * box_steps / (b_ - a), "unit": "atom-steps/s", "steps": box_steps,
                "ms_per_step_all_boxes": 1e3 * (b_ - a) / box_steps}
            if precision == "mixed":
                per_box["per_box_tuning"] = tuning_classes([m.n_atoms for m in melts], tunes)
            log("%s per box (%s): %.3e atom-steps/s" % (precision, "graph" if graph else "no graph",
                                                        N * box_steps / (b_ - a)))
        extra["per_box_forms"] = per_box

    plain = None
    if not args.no_fp64:
        fp_steps = min(args.fp64_steps, 200)
        s64 = make("fp64", list(wl.T0), pos, vel, graph=False)
        s64.step(10)
        torch.cuda.synchronize(dev)
        a = time.perf_counter()
        s64.step(fp_steps)
        torch.cuda.synchronize(dev)
        b_ = time.perf_counter()
        plain = {"value": N * fp_steps / (b_ - a), "unit": "atom-steps/s", "steps": fp_steps,
                 "ms_per_step": 1e3 * (b_ - a) / fp_steps, "tuning": list(s64.tuning()), "graph": False}
        s64.close()
        log("fp64: %.3f ms/step, %.3e atom-steps/s" % (plain["ms_per_step"], plain["value"]))

    out = {
        "metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": wl.name, "boxes": len(melts), "atoms": N, "chains": int(sum(chains)),
                   "chain_len": wl.chain_len, "density_g_cm3": wl.density, "tiles": wl.tiles,
                   "T0_K": [wl.T0[0], wl.T0[-1]], "thermostat": "berendsen", "tau_fs": wl.tau_fs,
                   "dt_fs": wl.dt_fs, "precision": "mixed (FP32 force, FP64 state)", "cell_div": R,
                   "lj_kernel": kern, "graph": not args.no_graph, "bins_rebuilt_every_step": True,
                   "relax_steps": args.relax_steps},
        "grown_melt_first_steps": grown,
        "ns_per_day": (1e3 / ms_per_step) * wl.dt_fs * 86400 * 1e-6,
        "plain_fp64_gpu": plain,
        "speedup_vs_plain_fp64": (value / plain["value"]) if plain else None,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
