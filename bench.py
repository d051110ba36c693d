#!/usr/bin/env python3
"""Orbital-update iterations per second on one MI355X.

Workload (mixed96): periodic box of side 24 bohr on a 96^3 grid, 64 Gaussian
ions with Z = 4 and width 0.5 bohr at seeded positions (minimum separation
1.5 bohr), N = 128 doubly occupied orbitals from a seeded atom-centred start.
One step is one call of pou_orbital_update_step: Algorithm M with n_org = 1
(direction, Barzilai-Borwein step, backtracking with the trial energy,
Cholesky-QR orthonormalisation).  The orbital block lives in HBM before the
timed region starts.

`value` is the mixed-precision rate; the FP64 rate, their ratio, the energy
difference after FP64 refinement, the roofline of the dominant kernel (HIP
events over the timed region) and the oracle timed on the host are reported
in the same JSON line.
"""
import argparse
import json
import statistics
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "orbital-update iters/sec at 96³ grid N=128, mixed vs FP64 at |ΔE|≤1e-6 Ha"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mixed96.json")
KERNEL_SOURCES = {"apply": "dense_kernels.hip", "gram": "dense_kernels.hip",
                  "apply_gram": "dense_kernels.hip",
                  "hamiltonian": "grid_kernels.hip", "trial": "dense_kernels.hip",
                  "commit": "grid_kernels.hip", "density": "grid_kernels.hip"}


def source_sha(name):
    import hashlib
    path = os.path.join(ROOT, "paper_1510_07230_amd", "csrc", name)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(group):
    """HBM bytes per launch of the group's kernel from the committed rocprofv3
    counter runs, or None if absent or the kernel source changed since."""
    try:
        rec = json.load(open(TRAFFIC_FILE))["groups"][group]
    except Exception:
        return None
    if rec.get("source_sha") != source_sha(KERNEL_SOURCES[group]):
        return None
    return rec["bytes_per_launch"]


def algorithmic_bytes(group, N, ng, es):
    """Bytes one launch of a kernel group must move at minimum (each operand once)."""
    B = N * ng * es
    return {
        "hamiltonian": 2 * B + ng * es,     # read W, write H W, read V_eff once
        "apply": 2 * B + ng * 8,            # read X, write L^-1 X, write rho (fused)
        "apply_gram": B,                    # read X once (L^-1 X stays on chip)
        "gram": B,                          # read the block once
        "trial": 3 * B,                     # read W, H W; write W - tau Z (+ its Gram)
        # the Barzilai-Borwein traces read W, H W, W_new, H W_new; the kernel's
        # write of W_new into the caller's block is counted apart (abi_bytes)
        "commit": 4 * B,
        "density": B + ng * 8,
    }.get(group)


def abi_bytes(group, N, ng, es):
    """Bytes a launch moves for the interface rather than the method: the
    accept kernel writes the new iterate into the caller's block U (one block),
    which the method itself keeps in place."""
    return N * ng * es if group == "commit" else 0


# MFMA peaks of MI355X (dense), FLOP/s
PEAK_FLOPS = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15}


def mfma_floor(group, N, ng, es):
    """(algorithmic flops, time floor on the matrix cores in s) of one launch.

    A triangular apply L^-1 X and a symmetric Gram X X^T each take N(N+1)
    flops per grid point.  The mixed first Gram runs on BF16 MFMA; the fused
    apply + second Gram does the apply as four BF16 products (hi/lo pieces of
    both operands) and the Gram of the three-piece W1 as six, so its floor is
    ten BF16 products.  Above 128 FP32 orbitals the apply and the second Gram
    are four split-BF16 products each."""
    tri = float(N * (N + 1) * ng)
    wide = "f64" if es == 8 else "f32"
    big = es == 4 and N > 128  # FP32 orbitals above 128: split-BF16 kernels
    if group == "apply":
        return tri, (4 * tri / PEAK_FLOPS["bf16"]) if big else tri / PEAK_FLOPS[wide]
    if group == "apply_gram":
        return 2 * tri, 10 * tri / PEAK_FLOPS["bf16"]
    if group == "trial":
        if N > 128:  # the trial point alone; its Gram is the "gram" group
            return 0.0, 0.0
        return tri, tri / PEAK_FLOPS["bf16" if es == 4 else "f64"]
    if group == "gram":
        # above 128 FP32 orbitals the group alternates the BF16 first Gram and
        # the split-BF16 (four products) second Gram: 2.5 products on average
        return tri, (2.5 * tri / PEAK_FLOPS["bf16"]) if big else tri / PEAK_FLOPS[wide]
    return 0.0, 0.0


def groups_roofline(prof, N, ng, es):
    """Roofline record of every kernel group with algorithmic bytes, from the
    breakdown pass (average launch time of the group)."""
    out = {}
    for g, (ms, n) in prof.items():
        if n <= 0 or algorithmic_bytes(g, N, ng, es) is None:
            continue
        r = roofline_of(g, N, ng, es, ms / n * 1e-3)
        out[g] = {k: r[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
        out[g]["avg_launch_ms"] = round(ms / n, 5)
    return out


def roofline_of(group, N, ng, es, avg_s):
    """Roofline record of one kernel group from its average launch time."""
    abytes = algorithmic_bytes(group, N, ng, es)
    flops, t_mfma = mfma_floor(group, N, ng, es)
    t_hbm = abytes / (HBM_PEAK_GBS * 1e9)
    if t_mfma > t_hbm:
        peak = flops / t_mfma / 1e12
        achieved = flops / avg_s / 1e12
        return {"bound": "mfma", "achieved": round(achieved, 2), "peak": round(peak, 2),
                "unit": "TFLOP/s", "frac": round(t_mfma / avg_s, 4),
                "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": abytes}
    achieved = abytes / avg_s / 1e9
    rec = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": abytes,
           "algorithmic_flops_per_launch": flops}
    extra = abi_bytes(group, N, ng, es)
    if extra:
        rec["abi_copy_bytes_per_launch"] = extra
        rec["frac_with_abi_copy"] = round((abytes + extra) / avg_s / 1e9 / HBM_PEAK_GBS, 4)
    return rec


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, single_thread=True):
    """Time the oracle's Algorithm-M step on this workload (bounded sample:
    one step with the host's BLAS/LAPACK threads, one with a single thread)."""
    import numpy as np
    import synth
    from oracle import ks, algm
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    R, Z, s = synth.atoms(cfg)
    so = ks.System(cfg.n, cfg.L, R, Z, s, synth.occupations(cfg))
    X = synth.orbitals(cfg)
    A = algm.AlgorithmM(X, so, algm.Params())
    t0 = time.perf_counter()
    A.step()
    t = time.perf_counter() - t0
    out = {"value": 1.0 / t, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
           "cpu": cpu_model(), "host_cpus": len(os.sched_getaffinity(0)),
           "sample": f"one oracle Algorithm-M step (trial orth + energy + H W) on the full "
                     f"{cfg.n}^3 / N={cfg.norb} workload, {t:.1f} s, BLAS/LAPACK on {threads} "
                     f"threads (NumPy's elementwise work and FFTs run on one); the oracle's "
                     f"initial orthonormalisation and energy are not timed"}
    if single_thread:
        with threadpool_limits(1):
            t0 = time.perf_counter()
            A.step()
            t1 = time.perf_counter() - t0
        out["single_thread"] = {"value": 1.0 / t1, "unit": "iters/s", "cores": 1,
                                "sample": f"the next oracle step with one thread, {t1:.1f} s"}
    return out


def run(args):
    import numpy as np
    import torch
    import synth
    import paper_1510_07230_amd as pk

    cfg = synth.CONFIGS[args.workload]
    R, Z, s = synth.atoms(cfg)
    occ = synth.occupations(cfg)
    X = synth.orbitals(cfg)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    g64 = pk.System(cfg.n, cfg.L, R, Z, s, occ, precision="fp64")
    U64 = g64.new_block(X)
    del X
    err0 = g64.orthonormalize_(U64)
    W0 = U64.clone()
    progress(f"start orthonormalised (err {err0:.2e})")

    N, ng = cfg.norb, cfg.ng

    def dominant(prof, es):
        cand = {k: v for k, v in prof.items()
                if algorithmic_bytes(k, N, ng, es) is not None and v[1] > 0}
        return max(cand, key=lambda k: cand[k][0])

    def timed(g, U, steps, warmup, es):
        """Warm-up steps; a breakdown pass that times every kernel group with
        events (not used for the rate, since each event record idles the
        stream for a few microseconds); then the timed pass, where events
        bracket only the launches of the dominant group."""
        for _ in range(warmup):
            g.step_(U)
        g.profile(True)
        for _ in range(steps):
            g.step_(U)
        prof_all = g.profile_read()
        dom = dominant(prof_all, es)
        g.profile(True, groups=[dom])
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for _ in range(steps):
            infos.append(g.step_(U))
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        prof_dom = g.profile_read()[dom]
        g.profile(False)
        return t, infos, prof_all, dom, prof_dom

    t64, inf64, prof64, dom64, pd64 = timed(g64, U64, args.steps, args.warmup, 8)
    progress(f"fp64: {args.steps / t64:.1f} it/s, E={inf64[-1]['E']:.10f}")

    g32 = pk.System(cfg.n, cfg.L, R, Z, s, occ, precision="mixed")
    U32 = W0.to(torch.float32).contiguous()
    g32.orthonormalize_(U32)
    t32, inf32, prof32, dom, pd32 = timed(g32, U32, args.steps, args.warmup, 4)
    progress(f"mixed: {args.steps / t32:.1f} it/s, E={inf32[-1]['E']:.10f}")

    # variant: mixed with one FP32-accurate Cholesky-QR pass instead of the
    # BF16 Gram + CholeskyQR2 of the specified mixed form (reported, not the value)
    extras = not args.no_extras
    if extras:
        g1 = pk.System(cfg.n, cfg.L, R, Z, s, occ, precision="mixed",
                       params=pk.default_params(orth_passes=1))
        U1 = W0.to(torch.float32).contiguous()
        g1.orthonormalize_(U1)
        t1, _, _, _, _ = timed(g1, U1, args.steps, args.warmup, 4)
        progress(f"mixed, one FP32 Cholesky-QR pass: {args.steps / t1:.1f} it/s")
        del g1, U1

    # cost of the section 3.3 modifications that keep the iteration unchanged:
    # subspace diagonalisation (here after every step, n_diag = 1, to time it;
    # the paper's runs use n_diag = 100) and one full-Sigma residual of eq. "gra"
    if extras:
        g2 = pk.System(cfg.n, cfg.L, R, Z, s, occ, precision="mixed",
                       params=pk.default_params(n_diag=1))
        U2 = W0.to(torch.float32).contiguous()
        g2.orthonormalize_(U2)
        n_rot = 10
        for _ in range(2):
            g2.step_(U2)
        torch.cuda.synchronize()
        t0r = time.perf_counter()
        for _ in range(n_rot):
            g2.step_(U2)
        torch.cuda.synchronize()
        t_rot_step = (time.perf_counter() - t0r) / n_rot
        t0r = time.perf_counter()
        res2, _ = g2.residual(U2)
        torch.cuda.synchronize()
        t_res = time.perf_counter() - t0r
        rot_ms = 1000.0 * (t_rot_step - t32 / args.steps)
        progress(f"subspace rotation: {rot_ms:.2f} ms each; residual {1000 * t_res:.2f} ms")
        del g2, U2

    # roofline of the dominant kernel group of the mixed run, from the events
    # of the timed pass
    avg_ms = pd32[0] / pd32[1]
    roofline = roofline_of(dom, N, ng, 4, avg_ms * 1e-3)
    roofline.update({"kernel": dom, "traffic": measured_traffic(dom),
                     "avg_launch_ms": round(avg_ms, 5), "launches_timed": pd32[1],
                "groups_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in prof32.items()},
                "fp64_groups_ms_per_step": {k: round(v[0] / args.steps, 4)
                                            for k, v in prof64.items()},
                "fp64_dominant": {"kernel": dom64, "avg_launch_ms": round(pd64[0] / pd64[1], 5)},
                "groups_roofline": groups_roofline(prof32, N, ng, 4),
                "fp64_groups_roofline": groups_roofline(prof64, N, ng, 8),
                "note": "groups_ms_per_step and groups_roofline come from a separate pass "
                        "with every group timed"})

    out = {
        "metric": METRIC,
        "value": round(args.steps / t32, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * t32 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.n}^3 periodic grid, L={cfg.L:g} bohr, "
                               f"{cfg.natoms} Gaussian ions Z={cfg.Z} sigma={cfg.sigma}, "
                               f"N={N} orbitals (f=2), {cfg.start}-start seeded; "
                               "mixed = FP32 orbitals/stencil, BF16-MFMA first Gram, FP32 second "
                               "Gram and apply, FP64 Cholesky and reductions",
                   "n": cfg.n, "L": cfg.L, "norb": N, "natoms": cfg.natoms},
        "fp64": {"value": round(args.steps / t64, 3), "unit": "iters/s",
                 "ms_per_step": round(1000.0 * t64 / args.steps, 4)},
        "speedup_mixed_over_fp64": round(t64 / t32, 3),
        "mean_trials_per_step": {"mixed": float(np.mean([i["s"] + 1 for i in inf32])),
                                 "fp64": float(np.mean([i["s"] + 1 for i in inf64]))},
        "roofline": roofline,
    }

    if extras:
        out["mixed_one_pass_fp32_gram"] = {
            "value": round(args.steps / t1, 3), "unit": "iters/s",
            "note": "one FP32-accurate Cholesky-QR pass instead of BF16 Gram + CholeskyQR2"}
        out["section_3_3"] = {
            "subspace_rotation_ms": round(rot_ms, 3),
            "rotation_per_step_at_n_diag_100_ms": round(rot_ms / 100.0, 4),
            "residual_ms": round(1000.0 * t_res, 3), "residual": res2,
            "note": "rotation cost = mixed step time with n_diag = 1 minus the mixed step "
                    "time; n_org = 2 is not timed (plain BB steps without a safeguard diverge "
                    "on this workload)"}
    if args.calibrate_copy:
        # a plain copy kernel of known size (one FP32 block, read once and
        # written once) for scaling the FETCH_SIZE / WRITE_SIZE counters
        tmp = torch.empty_like(U32)
        for _ in range(3):
            g32.convert(U32, tmp)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": U32.numel() * 4, "write": U32.numel() * 4}
        del tmp
    if not args.no_converge:
        out["delta_E"] = converge(args, cfg, R, Z, s, occ, g64, g32, W0, progress)
        if args.converge_starts > 1:
            # the same comparison from further starts of the same kind: the
            # Barzilai-Borwein iteration's progress varies from one trajectory
            # to the next, so one start gives one sample of the speed-up
            runs = [out["delta_E"]]
            for k in range(1, args.converge_starts):
                Wk = g64.new_block(synth.orbitals(cfg, variant=k))
                g64.orthonormalize_(Wk)
                progress(f"start {k}")
                runs.append(converge(args, cfg, R, Z, s, occ, g64, g32, Wk, progress,
                                     oracle_energy=False))
                del Wk
            sp = [r["time_to_1e-6_s"]["speedup"] for r in runs]
            out["delta_E"]["starts"] = [
                {"fp64_s": r["time_to_1e-6_s"]["fp64"],
                 "mixed_then_fp64_s": r["time_to_1e-6_s"]["mixed_then_fp64"],
                 "speedup": r["time_to_1e-6_s"]["speedup"], "mixed_steps": r["mixed_steps"],
                 "refine_steps": r["refine_steps"], "fp64_steps": r["fp64_steps"]}
                for r in runs]
            ok = [x for x in sp if x is not None]
            # the median proper: the mean of the two middle values for an even count
            out["delta_E"]["median_speedup"] = statistics.median(ok) if ok else None
    if not args.no_cpu_baseline:
        progress("oracle CPU baseline")
        del g64, g32, U64, U32, W0
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


def mixed_switch(df, info):
    """Rule that ends the mixed phase: the first step whose backtracking
    exhausted s_max (no trial met eq. "ene-de").  Near the minimum the energy
    decrease the test asks for, rho1 tau ||Z||^2, falls below the resolution of
    an energy evaluated from FP32 orbitals and FP32 stencil sums, and the test
    starts failing on rounding noise: at 96^3 x 128 the first such step comes
    about 1e-3 Ha above the minimum, after which mixed steps average 3 to 7
    trials and stall near 1e-4 Ha, while FP64 steps keep converging at about
    1.2 trials.  A 3-step mean of df below 1e-10 also ends the phase."""
    if info is not None and info.get("accepted", 1) == 0:
        return True
    return len(df) >= 3 and float(sum(df[-3:])) / 3.0 < 1e-10


def converge(args, cfg, R, Z, s, occ, g64, g32, W0, progress, oracle_energy=True):
    """Time to |dE| <= 1e-6 Ha from the same orthonormal start by two routes:
    FP64 steps alone, and mixed steps switched (mixed_switch) to FP64
    refinement steps.  Both converge by the 3-step mean of df < 1e-13
    (section 4.2).  The reference is the FP64 route's converged energy; the
    oracle's energy of the final FP64 iterate is reported beside it.  The
    wall time includes the host's step loop (each step synchronises)."""
    import numpy as np
    import torch
    import paper_1510_07230_amd as pk

    def run(g, U, done, cap_s, cap_steps):
        E, t, df = [], [], []
        t0 = time.perf_counter()
        info = None
        while len(E) < cap_steps and time.perf_counter() - t0 < cap_s:
            info = g.step_(U)
            E.append(info["E"])
            df.append(info["df"])
            t.append(time.perf_counter() - t0)
            if done(df, info):
                return E, t, info, True
        return E, t, info, False

    def df_rule(df, info):
        return len(df) >= 3 and float(np.mean(df[-3:])) < 1e-13

    def time_to(E, t, E_ref, tol=1e-6):
        """Time of the first step after which every energy stays within tol."""
        k = len(E)
        while k > 0 and abs(E[k - 1] - E_ref) <= tol:
            k -= 1
        return t[k] if k < len(E) else None

    cap = args.converge_seconds
    # route A: FP64 alone
    U64 = W0.clone()
    g64.reset_history()
    EA, tA, iA, cA = run(g64, U64, df_rule, cap, 200000)
    E_ref = iA["E"]
    progress(f"fp64 route: {len(EA)} steps, {tA[-1]:.2f} s, converged={cA}, E={E_ref:.12f}")
    # route B: mixed, then FP64 refinement
    U32 = W0.to(torch.float32).contiguous()
    g32.reset_history()
    t0 = time.perf_counter()
    EB1, tB1, iB1, cB1 = run(g32, U32, mixed_switch, cap, 200000)
    gr = pk.System(cfg.n, cfg.L, R, Z, s, occ, precision="fp64")
    t1 = time.perf_counter()
    Ur = gr.new_block()
    gr.convert(U32, Ur)
    gr.orthonormalize_(Ur)
    t_switch = time.perf_counter() - t1
    EB2, tB2, iB2, cB2 = run(gr, Ur, df_rule, cap, 200000)
    off = tB1[-1] + t_switch
    EB = EB1 + EB2
    tB = tB1 + [off + x for x in tB2]
    progress(f"mixed route: {len(EB1)} mixed steps ({tB1[-1]:.2f} s), {len(EB2)} FP64 steps "
             f"({tB2[-1]:.2f} s), E={iB2['E']:.12f}")
    G = gr.gram(Ur)
    orth_err = float(np.max(np.abs(G - np.eye(G.shape[0]))))
    ttA = time_to(EA, tA, E_ref)
    ttB = time_to(EB, tB, E_ref)
    res64, _ = g64.residual(U64)
    resr, _ = gr.residual(Ur)
    out = {"fp64_E": E_ref, "fp64_converged": cA, "fp64_steps": len(EA),
           "mixed_steps": len(EB1), "mixed_E_at_switch": iB1["E"],
           "mixed_switched_by_rule": cB1,
           "refined_E": iB2["E"], "refine_steps": len(EB2), "refine_converged": cB2,
           "abs_delta_E": abs(iB2["E"] - E_ref), "orth_err_refined": orth_err,
           "residual_fp64": res64, "residual_refined": resr,
           "time_to_1e-6_s": {"fp64": ttA, "mixed_then_fp64": ttB,
                              "speedup": (ttA / ttB) if (ttA and ttB) else None},
           "time_to_converged_s": {"fp64": tA[-1], "mixed_then_fp64": tB[-1]},
           "criterion": "converged: 3-step mean of df < 1e-13; the mixed phase ends at the first "
                        "step that exhausts s_max (or a 3-step mean df < 1e-10); time_to_1e-6 = "
                        "wall time (host loop included) until E stays within 1e-6 Ha of the FP64 "
                        "route's converged energy"}
    if oracle_energy and not args.no_oracle_energy:
        from oracle import ks
        so = ks.System(cfg.n, cfg.L, R, Z, s, occ)
        Wf = U64.detach().cpu().numpy()
        E_o = ks.energy(Wf, so).E
        out["oracle_E_of_fp64_iterate"] = E_o
        out["abs_E_gpu_minus_oracle_fp64"] = abs(E_ref - E_o)
        progress(f"oracle energy of the final FP64 iterate {E_o:.12f} (|dE| {abs(E_ref - E_o):.2e})")
    progress(f"time to |dE|<=1e-6: fp64 {ttA} s, mixed+refine {ttB} s; |dE| refined "
             f"{out['abs_delta_E']:.2e}, orth {orth_err:.2e}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mixed96")
    ap.add_argument("--converge-seconds", type=float, default=40.0)
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--converge-starts", type=int, default=1,
                    help="repeat the time-to-solution comparison from this many starts")
    ap.add_argument("--no-oracle-energy", action="store_true",
                    help="skip the oracle's energy of the final FP64 iterate")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the one-pass variant and the section 3.3 timings")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
