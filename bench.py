#!/usr/bin/env python3
"""Deep Potential MD throughput on one MI355X.

Headline: mixed precision (FP16 matrix-core products) with the student
embedding net.  The timed region starts with the in-run training of the
student on the current frame (sampling, teacher targets, Adam, least-squares
output layer), then runs the MD steps with the student, the full teacher
nets judging its forces every 20 steps (fallback above 1e-3 eV/A) on the
atoms of a 60 A cube placed anew each time (teacher evaluated on the cube
and its rc margin; --judge-side 0 judges every atom).  The same
precision without the student, the FP64 path and the MIX-32 (FP32) path are
timed after it for comparison.

One step = one velocity-Verlet MD step of the whole hot path: periodic wrap,
device-side skin check (cell list + candidate list rebuilt when an atom has
moved more than skin/2), formatted neighbour list, environment matrix, fused
embedding + descriptor, fitting net forward/backward, energy reduction,
embedding backward with force and virial scatter, and the two half kicks.
Inputs (coordinates, velocities, types) are resident in HBM before the
timed region starts.

Default workload: FCC copper, 50^3 conventional cells = 500,000 atoms,
a = 3.634 A, 0.05 A Gaussian jitter, rc 8 A, rcs 2 A, sel 512, embedding
1-25-50-100, M2 16, fitting 240x3, random seeded weights, 1 fs steps,
Maxwell-Boltzmann velocities at 300 K, skin 2 A.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

PEAK = {"f64_mfma": 78.6, "f32_mfma": 157.3, "f32_valu": 157.3, "f16_mfma": 2500.0, "bf16_mfma": 2500.0, "hbm": 8000.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic(spec, n_atoms, n_pairs, emb=None, affine=False, mixed=True, table=False, n_cand=0.0):
    """Algorithmic work per evaluation, by kernel (no recompute, no padding):
    flops for the network kernels, bytes for the list/env kernels.  `emb`
    overrides the embedding widths (the student's 16-32-100); `affine`: the
    last embedding layer is affine, so T = W3^T (sum h2 R^T) + b3 (sum R)^T
    and its products move from per pair to per atom; `table`: h2(s) (and
    dh2/ds) come from the cubic Hermite table, 4 multiply-adds per feature
    each, instead of the first two layers."""
    emb = (1,) + tuple(emb if emb is not None else spec.emb)
    M1, M2 = spec.M1, spec.M2
    fw = (M1 * M2,) + tuple(spec.fit) + (1,)
    fit_macs = sum(fw[l] * fw[l + 1] for l in range(len(fw) - 1))
    if affine:
        W1, W2 = emb[1], emb[2]
        hidden = 4 * W2 if table else W1 + W1 * W2   # h2 per pair: table or layers 1 and 2
        # per pair: h2 R^T (4 W2); per atom: W3^T H (4 W2 M1), b3 sum R (4 M1), D (4 M1 M2)
        e_fwd = 2.0 * n_pairs * (hidden + 4 * W2) + 2.0 * n_atoms * (4 * W2 * M1 + 4 * M1 + 4 * M1 * M2)
        # per pair: h, h' through layers 1-2 (2 hidden), M^T h2 and M^T h2' (8 W2);
        # per atom: M = W3 dT (4 W2 M1), b3^T dT (4 M1), dT from dD (8 M1 M2)
        e_bwd = 2.0 * n_pairs * (2 * hidden + 8 * W2) + 2.0 * n_atoms * (4 * W2 * M1 + 4 * M1 + 8 * M1 * M2)
    else:
        layer_macs = sum(emb[l] * emb[l + 1] for l in range(len(emb) - 1))
        # G(s) forward + T += G R^T per pair, D = T T<^T per atom
        e_fwd = 2.0 * n_pairs * (layer_macs + 4 * M1) + 2.0 * n_atoms * (4 * M1 * M2)
        # dE/dR = G^T dT, dE/dG = dT R, reverse through the layers per pair; dT per atom
        e_bwd = 2.0 * n_pairs * (layer_macs + 8 * M1) + 2.0 * n_atoms * (8 * M1 * M2)
    return {
        "embed_fwd": e_fwd,
        "embed_bwd": e_bwd,
        "fit": 2.0 * n_atoms * 2 * fit_macs,
        # bytes: per real slot nlist 4 B + neighbour position 32 B in, R (FP32 in
        # mixed precision: 16 B, and no (d, r); else 32 B and (d, r) 32 B) out
        "env": n_pairs * (4 + 32 + (16.0 if mixed else 64.0)) + n_atoms * (32 + 4 * spec.ntypes),
        # bytes: per candidate (neighbours within rc + skin, n_cand per atom)
        # its index 4 B + position 32 B in; per real slot 4 B out (and in
        # 16-bit mixed precision, where the format kernel also writes the
        # environment rows, R in FP32 16 B); own position and counts per atom
        "format": n_cand * (4 + 32) + n_pairs * (4 + (16.0 if mixed else 0.0)) + n_atoms * (32 + 4 * spec.ntypes),
    }


# kernel of each timed kernel-level phase (as named in the profiles) and the
# source group whose hash the PMC summary records
PHASE_KERNEL = {
    ("embed_bwd_main", True): ("k_embed_bwd_cells<16, 32, 100, 0, true>", "k_embed_mix"),
    ("embed_fwd", True): ("k_embed_fwd_lin<16, 32, 100, 0>", "k_embed_mix"),
    ("embed_bwd_main", False): ("k_embed_bwd_mix<25, 50, 100, 0, 0>", "k_embed_mix"),
    ("embed_fwd", False): ("k_embed_fwd_mix<25, 50, 100, 0, 0>", "k_embed_mix"),
    ("fit_fwd", True): ("k_fit_fwd<0, 15>", "k_fit_mix"),
    ("fit_fwd", False): ("k_fit_fwd<0, 15>", "k_fit_mix"),
    ("fit_bwd", True): ("k_fit_bwd<0, 15>", "k_fit_mix"),
    ("fit_bwd", False): ("k_fit_bwd<0, 15>", "k_fit_mix"),
    ("format", True): ("k_format", "k_nlist"),
    ("format", False): ("k_format", "k_nlist"),
    ("env", True): ("k_env<HIP_vector_type<float, 4u> >", "k_env"),
    ("env", False): ("k_env<HIP_vector_type<float, 4u> >", "k_env"),
}
HASH_FILES = {"k_embed_mix": ("k_embed_mix.hip", "dp_mix.h", "dp_internal.h"),
              "k_fit_mix": ("k_fit_mix.hip", "dp_mix.h", "dp_internal.h"),
              "k_nlist": ("k_nlist.hip", "dp_internal.h"), "k_env": ("k_env.hip", "dp_internal.h")}
PMC_FILE = os.path.join(HERE, "profiles", "cu500k_fp16_student_pmc.txt")


def source_hash(group):
    import hashlib
    h = hashlib.sha256()
    for f in HASH_FILES[group]:
        h.update(open(os.path.join(HERE, "paper_2005_00223_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def pmc_row(phase, precision, student):
    """The committed rocprofv3 PMC summary's row for the phase's kernel
    (FP16 headline precision only): HBM bytes per dispatch (FETCH_SIZE and
    WRITE_SIZE scaled by the copy calibration recorded there), MFMA busy and
    VALU active fractions; None when there is no such row or the kernel's
    sources changed after the counters were taken."""
    key = PHASE_KERNEL.get((phase, student))
    if precision != "fp16" or key is None or not os.path.exists(PMC_FILE):
        return None
    name, group = key
    text = open(PMC_FILE).read()
    if f"# source-hash {group}: {source_hash(group)}" not in text:
        return None
    lines = text.splitlines()
    head = next((ln.split() for ln in lines if ln.startswith("kernel ")), None)
    row = next((ln for ln in lines if ln.startswith("dpk::" + name + "  ")), None)
    if head is None or row is None:
        return None
    vals = row[len("dpk::" + name):].split()
    rec = dict(zip(head[1:], (float(v) for v in vals)))
    return {"traffic": rec["hbm_GB"] * 1e9, "mfma_util": rec["mfma_busy"], "valu_active": rec["valu_active"]}


def cpu_baseline(w, blob, seconds, log_fn):
    """Time the FP64 CPU oracle on a bounded sample of centre atoms of the
    same workload; returns s per atom per evaluation (= per MD step)."""
    from oracle import oracle as O
    o = O.Oracle(blob)
    n = len(w["types"])
    rng = np.random.default_rng(12345)
    k = min(n, 2048)
    cen = np.sort(rng.choice(n, size=k, replace=False))
    t0 = time.perf_counter()
    o.eval(w["coords"], w["types"], w["box"], centres=cen)
    dt = time.perf_counter() - t0
    k2 = int(min(n, max(k, seconds / max(dt / k, 1e-9))))
    cen2 = np.sort(rng.choice(n, size=k2, replace=False))
    log(f"[cpu] oracle sample: {k2} centre atoms (pilot {k} atoms in {dt:.2f} s)")
    t0 = time.perf_counter()
    o.eval(w["coords"], w["types"], w["box"], centres=cen2)
    dt2 = time.perf_counter() - t0
    return {"value": dt2 / k2, "unit": "s/step/atom", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{k2} random centre atoms of the same {n}-atom configuration, one FP64 evaluation "
                      f"(energy, forces, virial of their environments) in {dt2:.1f} s"}


def accuracy(args, w, blob, m, m64, x, t, student, frame):
    """Forces, energy and virial of the benchmarked path (and, when given,
    of the same precision's teacher nets and of the FP64 GPU path) at the
    configuration x, against the FP64 oracle: every atom ('full', one
    oracle evaluation of the whole frame) or N sampled atoms (one oracle
    evaluation over them and their neighbours, which makes their forces
    exact)."""
    from oracle import oracle as O
    n = len(w["types"])
    spec = w["spec"]
    xf = x.cpu().numpy()
    paths = {"timed": m.compute(x, t, w["box"])}
    nl = None
    if args.rmse != "full":
        nl, _ = m.nlist(n, spec.nnei, spec.ntypes)
        nl = nl.cpu().numpy()
    if student:
        m.student_use(False)
        paths["teacher"] = m.compute(x, t, w["box"])
        m.student_use(True)
    if m64 is not None:
        paths["fp64"] = m64.compute(x, t, w["box"])
    paths = {k: (e.item(), f.cpu().numpy(), v.cpu().numpy().reshape(9)) for k, (e, f, v) in paths.items()}
    o = O.Oracle(blob)
    t0 = time.perf_counter()
    if args.rmse == "full":
        r = o.eval(xf, w["types"], w["box"])
        ks = np.arange(n)
        what = f"all {n} atoms"
    else:
        rng = np.random.default_rng(7)
        ks = np.sort(rng.choice(n, size=int(args.rmse), replace=False))
        cen = np.unique(np.concatenate([ks, nl[ks][nl[ks] >= 0]]))
        r = o.eval(xf, w["types"], w["box"], centres=cen)
        what = f"{ks.size} random atoms"
    t_or = time.perf_counter() - t0
    acc = {"frame": frame, "atoms": what, "oracle_seconds": t_or, "oracle_threads": O.num_threads(),
           "force_rms": float(np.sqrt((r["force"][ks] ** 2).sum(1).mean()))}
    for k, (e, f, v) in paths.items():
        df = f[ks] - r["force"][ks]
        acc[k] = {"force_rmse": float(np.sqrt((df ** 2).sum(1).mean())),
                  "force_max_abs_err": float(np.abs(df).max())}
        if args.rmse == "full":
            acc[k].update(energy_err_per_atom=abs(e - r["energy"]) / n,
                          energy_rel_err=abs(e - r["energy"]) / abs(r["energy"]),
                          virial_rel_err=float(np.abs(v - r["virial"].reshape(9)).max() / np.abs(r["virial"]).max()))
        log(f"[bench] {frame}: {k} vs oracle ({what}): force RMSE {acc[k]['force_rmse']:.3e} eV/A, "
            f"max {acc[k]['force_max_abs_err']:.3e}")
    return acc


def profile_summary(kind, root, command):
    """Condense rocprofv3 CSV output under `root` into the text summaries
    kept in profiles/.  kind "kernels": the --kernel-trace --stats table
    (calls, mean and total ms, share per kernel).  kind "pmc": one --pmc run
    per sub-directory (counter passes); per kernel the mean per dispatch of
    the duration, MFMA busy (SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE x
    1024 SIMDs, the GRBM count summed over the 8 XCDs), VALU and LDS active
    (SQ_ACTIVE_INST_VALU / _LDS in 4-cycle units, same denominator), LDS bank
    conflict cycles per LDS instruction, FETCH_SIZE and WRITE_SIZE (KiB) and
    the HBM bytes they give after the copy calibration (a 1 GiB device copy,
    bench.py --copy-probe-mb 1024, in the same runs)."""
    import csv
    import glob
    from collections import defaultdict
    out = [f"# rocprofv3 {'kernel' if kind == 'kernels' else 'PMC'} summary", f"# command: {command}"]
    if kind == "kernels":
        f = glob.glob(os.path.join(root, "**", "*kernel_stats.csv"), recursive=True)[0]
        rows = list(csv.DictReader(open(f)))
        out.append(f"# condensed from {os.path.basename(f)} by bench.py --profile-summary kernels")
        out.append("%-62s %6s %10s %10s %6s" % ("kernel", "calls", "avg_ms", "total_ms", "pct"))
        for r in rows:
            out.append("%-62s %6s %10.4f %10.3f %6.2f" % (r["Name"].split("(")[0].replace("void ", "")[:62], r["Calls"],
                                                         float(r["AverageNs"]) / 1e6, float(r["TotalDurationNs"]) / 1e6,
                                                         float(r["Percentage"])))
        return "\n".join(out) + "\n"
    vals = defaultdict(lambda: defaultdict(lambda: defaultdict(float)))
    dur = defaultdict(dict)
    for f in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            k = r["Kernel_Name"].split("(")[0].replace("void ", "")
            d = (f, r["Dispatch_Id"])
            vals[k][r["Counter_Name"]][d] += float(r["Counter_Value"])
            dur[k][d] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6

    def mean(k, c):
        v = vals[k].get(c)
        return sum(v.values()) / len(v) if v else float("nan")
    # the calibration copies are the largest copy dispatches (1 GiB each);
    # without them the factors measured that way on this GPU (2 and 1) apply
    copy = vals.get("__amd_rocclr_copyBuffer", {})
    cw = max(copy.get("WRITE_SIZE", {0: 0.0}).values())
    if cw >= 1048576.0:
        cf = max(copy.get("FETCH_SIZE", {0: 524288.0}).values())
        ff, fw = 1048576.0 / cf, 1048576.0 / cw
        out.append(f"# calibration: 1 GiB device copy reads FETCH_SIZE {cf:.0f} KiB, WRITE_SIZE {cw:.0f} KiB -> "
                   f"factors fetch x{ff:.3f}, write x{fw:.3f}")
    else:
        ff, fw = 2.0, 1.0
        out.append("# calibration: no copy probe in these runs; factors fetch x2, write x1 (a 1 GiB device copy "
                   "reads FETCH_SIZE = 1/2 and WRITE_SIZE = 1 x its bytes on this GPU)")
    out.append("# hbm_GB = (FETCH_SIZE * fetch factor + WRITE_SIZE * write factor) * 1024 / 1e9, per dispatch;"
               " mfma_busy, valu_active, lds_active are fractions of the kernel's SIMD-cycles")
    for g in HASH_FILES:
        out.append(f"# source-hash {g}: {source_hash(g)}")
    out.append("%-50s %5s %9s %9s %11s %10s %8s %11s %11s %8s" % (
        "kernel", "disp", "ms", "mfma_busy", "valu_active", "lds_active", "bank/lds", "FETCH_KiB", "WRITE_KiB",
        "hbm_GB"))
    order = sorted(dur, key=lambda k: -sum(dur[k].values()) / len(dur[k]))
    for k in order:
        if not k.startswith("dpk::"):
            continue
        ms = sum(dur[k].values()) / len(dur[k])
        cyc = mean(k, "GRBM_GUI_ACTIVE") / 8.0 * 1024.0
        hbm = (mean(k, "FETCH_SIZE") * ff + mean(k, "WRITE_SIZE") * fw) * 1024 / 1e9
        npass = len({f for f, _ in dur[k]})
        out.append("%-50s %5d %9.4f %9.4f %11.4f %10.4f %8.3f %11.0f %11.0f %8.3f" % (
            k[:50], len(dur[k]) // max(npass, 1), ms, mean(k, "SQ_VALU_MFMA_BUSY_CYCLES") / cyc,
            mean(k, "SQ_ACTIVE_INST_VALU") * 4 / cyc, mean(k, "SQ_ACTIVE_INST_LDS") * 4 / cyc,
            mean(k, "SQ_LDS_BANK_CONFLICT") / max(mean(k, "SQ_INSTS_LDS"), 1.0),
            mean(k, "FETCH_SIZE"), mean(k, "WRITE_SIZE"), hbm))
    return "\n".join(out) + "\n"


def cpu_grid(args, log_fn):
    """The FP64 CPU oracle timed on this host with all threads and with one
    thread: one evaluation each of the 192- and 12,288-atom water boxes and
    the 32,000-atom copper box, 100 velocity-Verlet steps of the 12,288-atom
    water box (all threads), and the 500,000-atom copper box (all threads:
    the whole frame; one thread: a sample of 2,048 random centre atoms and
    their neighbour lists)."""
    from oracle import oracle as O
    from paper_2005_00223_amd import synth
    rows = []
    nthr = O.num_threads()

    def one(name, threads, centres=None, steps=0):
        log_fn(f"[cpu-grid] {name}: {threads} threads, {'%d steps' % steps if steps else 'one evaluation'} ...")
        w = synth.workload(name)
        o = O.Oracle(synth.pack_blob(w["spec"]))
        n = len(w["types"])
        t0 = time.perf_counter()
        if steps:
            v0 = synth.maxwell_boltzmann(w["masses"][w["types"]], w["temp"], w["vseed"])
            o.verlet(w["coords"], v0, w["types"], w["box"], w["masses"], w["dt_fs"], steps, every=steps,
                     nthreads=threads)
        else:
            o.eval(w["coords"], w["types"], w["box"], centres=centres, nthreads=threads)
        dt = time.perf_counter() - t0
        k = n if centres is None else len(centres)
        r = {"workload": name, "atoms": n, "threads": threads,
             "what": f"{steps} Verlet steps" if steps else (f"1 evaluation of {k} centre atoms"),
             "seconds": dt, "s_per_atom_per_eval": dt / (k * max(steps, 1))}
        log_fn(f"[cpu-grid] {r}")
        rows.append(r)

    # the oracle keeps the last thread count it was given: always pass one
    for name in ("water192", "water12288", "cu32000"):
        one(name, nthr)
        one(name, 1)
    one("water12288", nthr, steps=100)
    one("cu500k", nthr)
    rng = np.random.default_rng(5)
    one("cu500k", 1, centres=np.sort(rng.choice(500000, size=2048, replace=False)))
    return {"metric": "FP64 CPU oracle time per atom per evaluation", "unit": "s/atom", "host_threads": nthr,
            "rows": rows}


def rank_share(args, log_fn):
    """One GPU's share of the spatial decomposition (Section V-D): brick
    (0, 0, 0) of a 2 x 2 x 2 cut of the workload with its ghost shell of
    rc + skin, evaluated with its own atoms as centres and the ghosts as
    neighbours only (dp_compute_local), timed beside the whole-box
    evaluation on the same GPU."""
    import torch
    from paper_2005_00223_amd import synth
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload(args.workload)
    spec = w["spec"]
    n = len(w["types"])
    m = DPModel(synth.pack_blob(spec), args.precision)
    shell = spec.rcut + args.skin
    sh = synth.brick_share(w["coords"], w["types"], w["box"], (2, 2, 2), (0, 0, 0), shell)
    xb = torch.tensor(sh["coords"], dtype=torch.float64, device=m.device)
    tb = torch.tensor(sh["types"], dtype=torch.int32, device=m.device)
    xa = torch.tensor(w["coords"], dtype=torch.float64, device=m.device)
    ta = torch.tensor(w["types"], dtype=torch.int32, device=m.device)

    def timed(fn, k=5):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    t_brick = timed(lambda: m.compute_local(xb, tb, sh["box"], sh["n_local"]))
    t_box = timed(lambda: m.compute(xa, ta, w["box"]))
    nl = sh["n_local"]
    log_fn(f"[rank-share] brick: {nl} owned + {len(tb) - nl} ghosts, {t_brick * 1e3:.2f} ms; whole box {n} atoms "
           f"{t_box * 1e3:.2f} ms")
    return {"metric": "rank-share evaluation time (E+F+virial of one brick of a 2x2x2 decomposition)",
            "value": t_brick * 1e3, "unit": "ms", "higher_is_better": False, "n_gpus": 1, "dtype": args.precision,
            "data": "synthetic",
            "config": {"workload": args.workload, "atoms": n, "owned": nl, "ghosts": int(len(tb) - nl),
                       "shell_A": shell},
            "whole_box_ms": t_box * 1e3, "brick_over_eighth_of_box": t_brick / (t_box / 8.0),
            "ghost_exchange_bytes_each_way": int((len(tb) - nl) * 24)}


def sweep(args, log_fn):
    """Embedding-size study (Sec. VII-D, Fig. 7): the copper sweep workload
    (15^3 FCC cells, 13,500 atoms, rc 8 A, sel 512) with embedding nets
    (W/2, W, 2W) for last-layer matrices W x 2W, teacher nets only, MD steps
    of the whole path.  FLOPs are the method's algorithmic count per step
    (embedding forward + backward per real pair, descriptor, fitting
    forward + backward); nets up to 128 wide run the register-resident
    kernels, wider ones the 16-bit GEMM path, with its activations stored as
    one 16-bit value (mix16, the paper's MIX-16) and/or as hi + lo halves
    (split, two products per weight)."""
    import torch
    from paper_2005_00223_amd import synth
    from paper_2005_00223_amd.model import DPModel
    w = synth.workload("cu13500")
    n = len(w["types"])
    rows = []
    for size in args.sweep_sizes.split(","):
        a, b = (int(v) for v in size.lower().split("x"))
        emb = (a // 2, a, b)
        spec = synth.copper_model(1, emb=emb)
        for storage in args.wide_storage.split(","):
            m = DPModel(synth.pack_blob(spec), args.precision)
            m.set_wide_storage(0 if storage == "split" else 1)
            x = torch.tensor(w["coords"], dtype=torch.float64, device=m.device)
            v = torch.tensor(synth.maxwell_boltzmann(w["masses"][w["types"]], w["temp"], w["vseed"]),
                             dtype=torch.float64, device=m.device)
            t = torch.tensor(w["types"], dtype=torch.int32, device=m.device)
            f = torch.zeros((n, 3), dtype=torch.float64, device=m.device)

            def md(k):
                return m.md_run(x, v, t, w["box"], w["masses"], w["dt_fs"], k, skin=args.skin, thermo_every=k, forces=f)

            md(max(1, args.warmup))
            m.enable_timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            md(args.steps)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / args.steps
            phases = {k: m.timing(k) for k in ("format", "env", "embed_fwd", "fit", "embed_bwd", "total")}
            m.enable_timing(False)
            _, nr = m.nlist(n, spec.nnei, spec.ntypes, with_list=False)
            pairs = float(nr.sum().item())
            alg = algorithmic(spec, n, pairs)
            flops = alg["embed_fwd"] + alg["embed_bwd"] + alg["fit"]
            st = m.stats()
            wide = st["wide_evals"] > 0
            row = {"matrix": f"{a}x{b}", "emb": list(emb), "path": "gemm" if wide else "fused",
                   "storage": storage if wide else "split",
                   "ms_per_step": sec * 1e3, "tflops": flops / sec / 1e12,
                   "embed_tflops": (alg["embed_fwd"] + alg["embed_bwd"]) / ((phases["embed_fwd"] + phases["embed_bwd"])
                                                                            * 1e-3) / 1e12,
                   "gflop_per_step": flops / 1e9, "phase_ms": {k: round(vv, 4) for k, vv in phases.items()}}
            log_fn(f"[sweep] {a}x{b} ({row['path']}, {row['storage']}): {sec * 1e3:.2f} ms/step, {row['tflops']:.1f} TFLOP/s, "
                   f"embedding {row['embed_tflops']:.1f} TFLOP/s")
            rows.append(row)
            del m, x, v, t, f
            torch.cuda.empty_cache()
            if not wide:
                break  # the register-resident kernels have one storage
    pk = {"fp16": "f16_mfma", "bf16": "bf16_mfma"}[args.precision]
    return {"metric": "embedding-size study: FLOP/s of MD steps vs last-layer matrix (Fig. 7)", "unit": "TFLOP/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "dtype": args.precision, "data": "synthetic",
            "peak_tflops": PEAK[pk],
            "config": {"workload": f"cu13500: FCC Cu {n} atoms, rc 8 A, sel 512, M2 16, fit 240x3, "
                                   "embedding (W/2, W, 2W), teacher nets"},
            "sizes": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cu500k")
    ap.add_argument("--precision", default="fp16", choices=["fp64", "fp32", "fp16", "bf16"])
    ap.add_argument("--no-student", action="store_true", help="time the teacher nets only")
    ap.add_argument("--judge-every", type=int, default=20)
    ap.add_argument("--judge-side", type=float, default=60.0,
                    help="judge the atoms of a cube of this side (A) at a new place each time; 0 = all atoms")
    ap.add_argument("--teacher-steps", type=int, default=5,
                    help="steps of the same precision without the student, timed for comparison (0 = skip)")
    ap.add_argument("--fp64-steps", type=int, default=3, help="FP64 steps timed for the comparison (0 = skip)")
    ap.add_argument("--fp32-steps", type=int, default=3,
                    help="MIX-32 steps timed after the FP64 comparison (0 = skip)")
    ap.add_argument("--rmse", default="full",
                    help="force accuracy at the final frame vs the oracle: 'full' (every atom, one oracle "
                         "evaluation of the whole frame), N (N sampled atoms, local oracle evaluations) or 0")
    ap.add_argument("--rmse-frame0", action="store_true", help="also check the accuracy of the start frame")
    ap.add_argument("--skin", type=float, default=2.0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="embedding-size study (Fig. 7) on 13,500 copper atoms instead of the headline run")
    ap.add_argument("--sweep-sizes", default="64x128,128x256,256x512,512x1024,1024x2048")
    ap.add_argument("--wide-storage", default="mix16,split",
                    help="activation storage of the GEMM path in the sweep: mix16, split or both")
    ap.add_argument("--profile-summary", nargs=3, metavar=("KIND", "DIR", "COMMAND"),
                    help="condense rocprofv3 CSV output (KIND kernels or pmc) under DIR into a profiles/ text summary")
    ap.add_argument("--cpu-grid", action="store_true", help="time the CPU oracle on several workloads, all and one thread")
    ap.add_argument("--rank-share", action="store_true",
                    help="time one brick of a 2x2x2 spatial decomposition (owned atoms + rc+skin ghost shell)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (traffic-counter calibration)")
    args = ap.parse_args()
    if args.profile_summary:
        kind, root, command = args.profile_summary
        sys.stdout.write(profile_summary(kind, root, command))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "spatial decomposition is a design, not code", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_00223_amd import synth
    from paper_2005_00223_amd.model import DPModel

    if args.copy_probe_mb > 0:
        src = torch.empty(args.copy_probe_mb << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: 3 copies of {args.copy_probe_mb} MiB")
        del src, dst
    if args.cpu_grid:
        print(json.dumps(cpu_grid(args, log)), flush=True)
        return
    if args.rank_share:
        print(json.dumps(rank_share(args, log)), flush=True)
        return
    if args.sweep:
        if args.precision not in ("fp16", "bf16"):
            print("bench.py: the embedding-size study runs in fp16 or bf16", file=sys.stderr)
            sys.exit(2)
        print(json.dumps(sweep(args, log)), flush=True)
        return
    w = synth.workload(args.workload)
    spec = w["spec"]
    blob = synth.pack_blob(spec)
    n = len(w["types"])
    student = not args.no_student
    log(f"[bench] workload {args.workload}: {n} atoms, precision {args.precision}, student {student}")
    m = DPModel(blob, args.precision)
    dev = m.device
    x = torch.tensor(w["coords"], dtype=torch.float64, device=dev)
    v = torch.tensor(synth.maxwell_boltzmann(w["masses"][w["types"]], w["temp"], w["vseed"]),
                     dtype=torch.float64, device=dev)
    t = torch.tensor(w["types"], dtype=torch.int32, device=dev)
    f = torch.zeros((n, 3), dtype=torch.float64, device=dev)

    def md(model, steps, every):
        return model.md_run(x, v, t, w["box"], w["masses"], w["dt_fs"], steps, skin=args.skin,
                            thermo_every=every, forces=f)

    acc0 = None
    if args.rmse_frame0 and args.rmse != "0":
        acc0 = accuracy(args, w, blob, m, DPModel(blob, "fp64") if args.precision != "fp64" else None, x, t,
                        False, "frame 0")
    if args.warmup > 0:
        md(m, args.warmup, args.warmup)
        if student:  # load and run the student kernels once
            m.student_train(adam_steps=10, ls_samples=8192)
            m.student_use(True)
            md(m, 1, 1)
            m.student_use(False)
    elif student:  # the in-run training samples the lists of an evaluated frame
        m.compute(x, t, w["box"])
    torch.cuda.synchronize()
    log("[bench] warmup done")
    out_extra = {}
    if student:
        m.student_judge(args.judge_every, 1e-3, sample_side=args.judge_side)
    m.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if student:
        # in-run training on the current frame (its lists are the warmup's last)
        fit = m.student_train()
        m.student_use(True)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
    th = md(m, args.steps, min(args.judge_every if student else 20, args.steps))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("[bench] timed steps done")
    sec = t1 - t0
    s_step = sec / args.steps
    st = m.stats()
    if student:
        out_extra["student"] = {
            "train_ms": t_train * 1e3, "md_ms_per_step": (sec - t_train) / args.steps * 1e3,
            "fit_rel_rmse_G": fit, "judge_every": args.judge_every, "judge_max_force_rmse": 1e-3,
            "judge_cube_side_A": args.judge_side, "judge_atoms": st["judge_atoms"],
            "last_judge_force_rmse": st["last_judge_rmse"], "teacher_fallbacks": st["teacher_fallbacks"],
            "student_evals": st["student_evals"],
            "net": "1-16-32-100 (tanh, tanh + doubling skip, affine) per type pair; Adam 500 x 4096 samples "
                   "+ FP64 least-squares output layer on 262144 samples, all inside the timed region"}
        log(f"[bench] student: train {t_train * 1e3:.1f} ms, G rel RMSE {fit:.2e}, judge RMSE "
            f"{st['last_judge_rmse']:.2e}, fallbacks {st['teacher_fallbacks']}")
    phases = {k: m.timing(k) for k in ("lists", "format", "env", "embed_fwd", "fit", "embed_bwd", "total",
                                       "fit_fwd", "fit_bwd", "embed_bwd_main")}
    _, nr = m.nlist(n, spec.nnei, spec.ntypes, with_list=False)
    n_pairs = float(nr.sum().item())
    used_student = student and st["teacher_fallbacks"] == 0
    # candidates (neighbours within rc + skin) per atom: the real pairs scaled by the volume ratio
    n_cand = n_pairs * ((spec.rcut + args.skin) / spec.rcut) ** 3
    alg = algorithmic(spec, n, n_pairs, emb=(16, 32, spec.M1) if used_student else None, affine=used_student,
                      mixed=args.precision in ("fp16", "bf16"), table=used_student and st["table_evals"] > 0,
                      n_cand=n_cand)
    thn = th.cpu().numpy()
    drift = float((thn[-1, 3] - thn[0, 3]) / n) if len(thn) > 1 else 0.0
    # the longest single kernel of the step (kernel-level phases)
    kern = max(("format", "env", "embed_fwd", "fit_fwd", "fit_bwd", "embed_bwd_main"), key=lambda k: phases[k])
    work = {"format": alg["format"], "env": alg["env"], "embed_fwd": alg["embed_fwd"], "fit_fwd": alg["fit"] / 2,
            "fit_bwd": alg["fit"] / 2, "embed_bwd_main": alg["embed_bwd"]}[kern]
    if kern in ("env", "format"):
        ach = work / (phases[kern] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm"], "unit": "GB/s", "frac": ach / PEAK["hbm"]}
    elif kern in ("embed_fwd", "embed_bwd_main") and used_student and args.precision in ("fp16", "bf16"):
        # the student's embedding kernels spend their time in FP32 vector work
        # (table interpolation, operand splits) and the FP64 force pass, not in
        # the matrix cores: priced against the FP32 vector peak.  The work is
        # the per-feature count of the method (h2 and its slope for every
        # feature of every pair); the backward's projected table reaches the
        # same result with less arithmetic per pair, so its rate here is an
        # algorithmic one, not the instructions the kernel issues
        # (valu_active, from the counters, is that)
        ach = work / (phases[kern] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": ach, "peak": PEAK["f32_valu"], "unit": "TFLOP/s",
                "frac": ach / PEAK["f32_valu"]}
    else:
        pk = {"fp64": "f64_mfma", "fp32": "f32_mfma", "fp16": "f16_mfma", "bf16": "bf16_mfma"}[args.precision]
        ach = work / (phases[kern] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": PEAK[pk], "unit": "TFLOP/s", "frac": ach / PEAK[pk]}
    pm = pmc_row(kern, args.precision, used_student)
    kname = PHASE_KERNEL.get((kern, used_student), (kern,))[0] if args.precision == "fp16" else kern
    roof.update(kernel=kname, kernel_ms=phases[kern],
                traffic=pm["traffic"] if pm else None)
    if pm:
        roof.update(traffic_GBps=pm["traffic"] / (phases[kern] * 1e-3) / 1e9, mfma_util=pm["mfma_util"],
                    valu_active=pm["valu_active"], counters="profiles/cu500k_fp16_student_pmc.txt")
    if args.workload.startswith("cu"):
        wl = (f"{args.workload}: FCC Cu {n} atoms, rc 8 A, sel 512, emb 1-25-50-100, M2 16, fit 240x3, "
              f"NVE 1 fs, skin {args.skin} A")
    else:
        wl = args.workload
    out = {
        "metric": "s/step/atom (E+F+virial), mixed+student vs FP64 at force RMSE <=1e-3 eV/A",
        "value": s_step / n,
        "unit": "s/step/atom",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": s_step * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16", "bf16": "bf16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": wl, "precision": args.precision,
                   "student": "1-16-32-100, trained in the timed region" if student else "none",
                   "atoms": n, "real_pairs": int(n_pairs)},
        "ns_per_day": w["dt_fs"] * 86400e-6 / s_step,
        "phase_ms": {k: round(v, 4) for k, v in phases.items()},
        "energy_drift_eV_per_atom": drift,
        "roofline": roof,
    }
    out.update(out_extra)
    # per-step times of the comparison paths: the difference of a 1-step and
    # a (1 + k)-step run, since every run also evaluates its start frame
    def step_time(model, xx, vv, ff, k):
        def run(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            model.md_run(xx, vv, t, w["box"], w["masses"], w["dt_fs"], steps, skin=args.skin,
                         thermo_every=steps, forces=ff)
            torch.cuda.synchronize()
            return time.perf_counter() - t0
        t1 = run(1)
        return (run(1 + k) - t1) / k

    m64 = None
    if args.precision != "fp64" and args.fp64_steps > 0:
        m64 = DPModel(blob, "fp64")
    # force accuracy of the timed path at the final MD frame, against the oracle
    if args.rmse != "0":
        acc = accuracy(args, w, blob, m, m64, x, t, student, f"final MD frame (step {args.steps})")
        if acc0 is not None:
            out["accuracy_frame0"] = acc0
        out["accuracy"] = acc
        out["force_rmse_vs_oracle"] = acc["timed"]["force_rmse"]
        out["force_rms"] = acc["force_rms"]
        out["force_rmse_sample"] = (f"{acc['atoms']} of the final MD frame, "
                                    f"{'student' if used_student else 'teacher'} nets vs the oracle's teacher")
        log(f"[bench] force RMSE vs oracle {out['force_rmse_vs_oracle']:.3e} eV/A")
    if args.precision != "fp64" and args.teacher_steps > 0:
        m.student_use(False)
        m.enable_timing(False)
        sT = step_time(m, x, v, f, args.teacher_steps)
        out["mixed_teacher_s_per_step_atom"] = sT / n
        log(f"[bench] mixed teacher {sT * 1e3:.1f} ms/step")
    if m64 is not None:
        f64 = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        s64 = step_time(m64, x.clone(), v.clone(), f64, args.fp64_steps)
        out["fp64_s_per_step_atom"] = s64 / n
        out["speedup_vs_fp64"] = s64 / s_step
        log(f"[bench] fp64 {s64 * 1e3:.1f} ms/step")
        if args.fp32_steps > 0 and args.precision != "fp32":
            # the paper's third policy (MIX-32) on the same configuration
            del m64
            m32 = DPModel(blob, "fp32")
            s32 = step_time(m32, x.clone(), v.clone(), f64, args.fp32_steps)
            out["fp32_s_per_step_atom"] = s32 / n
            log(f"[bench] fp32 (MIX-32) {s32 * 1e3:.1f} ms/step")
            del m32
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, blob, args.cpu_seconds, log)
        out["cpu_baseline"]["gpu_over_cpu"] = out["cpu_baseline"]["value"] / out["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
